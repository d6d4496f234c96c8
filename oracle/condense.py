"""Element-level static condensation and recovery (oracle; test infrastructure only).

Follows the plain definition of Section 2.3: with the element's q/u block
  Ae = [[A, B], [D, E]],
eq. 13-b gives the element Schur complement  Kbar = J - [G H] Ae^{-1} [C; F]
and eq. 13-c the condensed right-hand side  rbar = r_t - [G H] Ae^{-1} [r_q; r_u]
with r_q = 0 (Section 4.1). Recovery uses [dq; du] = Ae^{-1}([r_q; r_u] - [C; F] duhat).
The local matrices are rebuilt in full from the structured inputs
(A = I_{MD} (x) M^e, B and C component-diagonal, eq. w16) and solved with one
LAPACK call per element: no two-stage elimination as on the GPU.

`dims` is a dict with ne, nf, ncomp (M), dim (D), npe (P_E), npf (P_F), nlfe (N_lfe).
Dof orders: q (m, d, i), u (m, i), element trace (l, m, j).
"""
import numpy as np


def full_local(blk, e, dims):
    """Dense A, B, C of element e rebuilt from (Minv, Bd, Cd) (eq. w15/w16)."""
    M, D, P, PF, L = dims["ncomp"], dims["dim"], dims["npe"], dims["npf"], dims["nlfe"]
    Me = np.linalg.inv(blk["Minv"][e])
    Bd = blk["Bd"][e]                    # (D, P, P)
    Cd = blk["Cd"][e]                    # (D, P, L*PF)
    nq, nu, nt = M * D * P, M * P, L * M * PF
    A = np.zeros((nq, nq))
    Bm = np.zeros((nq, nu))
    Cm = np.zeros((nq, nt))
    for m in range(M):
        for d in range(D):
            r0 = (m * D + d) * P
            A[r0:r0 + P, r0:r0 + P] = Me
            Bm[r0:r0 + P, m * P:(m + 1) * P] = Bd[d]
            for l in range(L):
                c0 = (l * M + m) * PF
                Cm[r0:r0 + P, c0:c0 + PF] = Cd[d][:, l * PF:(l + 1) * PF]
    return A, Bm, Cm


def local_system(blk, e, dims):
    A, Bm, Cm = full_local(blk, e, dims)
    Ae = np.block([[A, Bm], [blk["D"][e], blk["E"][e]]])
    CF = np.vstack([Cm, blk["F"][e]])
    GH = np.hstack([blk["G"][e], blk["H"][e]])
    r_qu = np.concatenate([np.zeros(A.shape[0]), blk["ru"][e]])
    return Ae, CF, GH, r_qu


def condense(blk, dims, elems=None):
    """Kbar (n, nt, nt) and rbar (n, nt) by one dense solve per element (eq. 13-b, 13-c).

    `elems` selects a subset of elements (default: all)."""
    ne = blk["J"].shape[0]
    elems = range(ne) if elems is None else elems
    nt = blk["J"].shape[1]
    Kbar = np.zeros((len(elems), nt, nt))
    rbar = np.zeros((len(elems), nt))
    for k, e in enumerate(elems):
        Ae, CF, GH, r_qu = local_system(blk, e, dims)
        X = np.linalg.solve(Ae, np.column_stack([CF, r_qu]))
        Kbar[k] = blk["J"][e] - GH @ X[:, :nt]
        rbar[k] = blk["rt"][e] - GH @ X[:, nt]
    return Kbar, rbar


def element_trace(xhat, e2f, perm, e, dims):
    """Element trace vector (l, m, j) of element e gathered from the face vector.

    perm[e][l][j] is the element-local face dof that holds canonical face dof j
    (None: identity)."""
    M, PF, L = dims["ncomp"], dims["npf"], dims["nlfe"]
    nb = M * PF
    out = np.zeros(L * nb)
    for l in range(L):
        f = e2f[e, l]
        xf = xhat[f * nb:(f + 1) * nb].reshape(M, PF)
        for m in range(M):
            for j in range(PF):
                jl = perm[e, l, j] if perm is not None else j
                out[(l * M + m) * PF + jl] = xf[m, j]
    return out


def recover(blk, xhat, e2f, dims, perm=None, elems=None):
    """(dq, du) per element from the trace solution (recovery equation of Section 2.3)."""
    ne = blk["J"].shape[0]
    elems = range(ne) if elems is None else elems
    M, D, P = dims["ncomp"], dims["dim"], dims["npe"]
    dq = np.zeros((len(elems), M * D * P))
    du = np.zeros((len(elems), M * P))
    for k, e in enumerate(elems):
        Ae, CF, GH, r_qu = local_system(blk, e, dims)
        ue = element_trace(xhat, e2f, perm, e, dims)
        s = np.linalg.solve(Ae, r_qu - CF @ ue)
        nq = M * D * P
        dq[k] = s[:nq]
        du[k] = s[nq:]
    return dq, du
