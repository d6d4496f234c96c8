"""Face-block global trace system and the uncondensed global system (oracle; test only).

Section 2.4: K couples trace dofs on faces that share an element; it is stored
as one dense (M P_F) x (M P_F) block per (face, neighbour slot), with
S = 2 N_lfe - 1 slots per face. Section 4.2: the blocks of face f are merged
from the element Schur complements of its two neighbours.

Slot order (the paper does not fix one): slot 0 is f itself; slots
1..N_lfe-1 are the other faces of e1 in local-face order; slots N_lfe..2N_lfe-2
the other faces of e2. A boundary face leaves the e2 slots empty (nbr = -1).

Block storage: K[f][s][col][row] (column-major blocks: the order in which the
paper lists the dimensions M x P_F x M x P_F x (2N_lfe-1) x N_F, first fastest).
"""
import numpy as np
import scipy.sparse as sp


def slot_faces(f2e, e2f, f):
    """Neighbour faces of f per slot (-1 for empty) and their (element, local face)."""
    L = e2f.shape[1]
    e1, l1, e2, l2 = f2e[f]
    nbr = [f]
    src = [None]
    for l in range(L):
        if l != l1:
            nbr.append(e2f[e1, l])
            src.append((e1, l))
    for l in range(L):
        if e2 >= 0 and l != l2:
            nbr.append(e2f[e2, l])
            src.append((e2, l))
        elif e2 < 0 and l != 0:
            nbr.append(-1)
            src.append(None)
    return nbr, src


def _elem_block(Kbar, e, lr, lc, dims, perm):
    """Block of Kbar[e] coupling local face lr (rows) to lc (cols) in canonical dof order."""
    M, PF = dims["ncomp"], dims["npf"]
    nb = M * PF
    out = np.zeros((nb, nb))
    for mr in range(M):
        for jr in range(PF):
            jrl = perm[e, lr, jr] if perm is not None else jr
            for mc in range(M):
                for jc in range(PF):
                    jcl = perm[e, lc, jc] if perm is not None else jc
                    out[mr * PF + jr, mc * PF + jc] = Kbar[e, (lr * M + mr) * PF + jrl, (lc * M + mc) * PF + jcl]
    return out


def _elem_vec(rbar, e, l, dims, perm):
    M, PF = dims["ncomp"], dims["npf"]
    out = np.zeros(M * PF)
    for m in range(M):
        for j in range(PF):
            jl = perm[e, l, j] if perm is not None else j
            out[m * PF + j] = rbar[e, (l * M + m) * PF + jl]
    return out


def assemble(Kbar, rbar, f2e, e2f, dims, perm=None):
    """Face blocks K (nf, S, nb, nb) as [f][s][col][row], nbr (nf, S), r (nf*nb)."""
    nf = f2e.shape[0]
    L = e2f.shape[1]
    S = 2 * L - 1
    nb = dims["ncomp"] * dims["npf"]
    K = np.zeros((nf, S, nb, nb))
    nbr = np.full((nf, S), -1, np.int64)
    r = np.zeros(nf * nb)
    for f in range(nf):
        e1, l1, e2, l2 = f2e[f]
        faces, src = slot_faces(f2e, e2f, f)
        nbr[f] = faces
        blk = _elem_block(Kbar, e1, l1, l1, dims, perm)
        rv = _elem_vec(rbar, e1, l1, dims, perm)
        if e2 >= 0:
            blk = blk + _elem_block(Kbar, e2, l2, l2, dims, perm)
            rv = rv + _elem_vec(rbar, e2, l2, dims, perm)
        K[f, 0] = blk.T
        r[f * nb:(f + 1) * nb] = rv
        for s in range(1, S):
            if src[s] is None:
                continue
            e, l = src[s]
            lr = l1 if e == e1 else l2
            K[f, s] = _elem_block(Kbar, e, lr, l, dims, perm).T
    return K, nbr, r


def to_sparse(K, nbr, n_col_faces=None):
    """scipy CSR matrix of the face-block system (row block f, column block nbr[f][s]).

    K/nbr may hold a subset of face rows; n_col_faces then gives the column count."""
    nf, S, nb, _ = K.shape
    ncf = nf if n_col_faces is None else n_col_faces
    rows, cols, vals = [], [], []
    rr, cc = np.meshgrid(np.arange(nb), np.arange(nb), indexing="ij")
    for f in range(nf):
        for s in range(S):
            g = nbr[f, s]
            if g < 0:
                continue
            blk = K[f, s].T                   # [row][col]
            rows.append(f * nb + rr.ravel())
            cols.append(g * nb + cc.ravel())
            vals.append(blk.ravel())
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf * nb, ncf * nb))


def uncondensed_system(blk, e2f, dims, perm=None):
    """Global (q, u, uhat) system assembled element by element (Section 2.3, eq. matrixform).

    Unknown order: all element (q, u) blocks element-major, then the face traces.
    Trace rows of the two elements sharing a face are summed, as in the face assembly."""
    from .condense import local_system
    M, D, P, PF, L = dims["ncomp"], dims["dim"], dims["npe"], dims["npf"], dims["nlfe"]
    ne, nf = dims["ne"], dims["nf"]
    nqu = M * D * P + M * P
    nb = M * PF
    N = ne * nqu + nf * nb
    A = sp.lil_matrix((N, N))
    rhs = np.zeros(N)
    for e in range(ne):
        Ae, CF, GH, r_qu = local_system(blk, e, dims)
        o = e * nqu
        A[o:o + nqu, o:o + nqu] = Ae
        rhs[o:o + nqu] = r_qu
        # trace index map of element e
        tmap = np.zeros(L * nb, np.int64)
        for l in range(L):
            f = e2f[e, l]
            for m in range(M):
                for j in range(PF):
                    jl = perm[e, l, j] if perm is not None else j
                    tmap[(l * M + m) * PF + jl] = ne * nqu + f * nb + m * PF + j
        for a in range(L * nb):
            A[o:o + nqu, tmap[a]] = A[o:o + nqu, tmap[a]] + CF[:, a:a + 1]
        for a in range(L * nb):
            ra = tmap[a]
            A[ra, o:o + nqu] = A[ra, o:o + nqu] + GH[a:a + 1, :]
            for b in range(L * nb):
                A[ra, tmap[b]] += blk["J"][e][a, b]
            rhs[ra] += blk["rt"][e][a]
    return A.tocsc(), rhs, nqu
