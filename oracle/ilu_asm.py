"""ILU-ASM: additive Schwarz on multi-element subdomains with block ILU(0) local solves
(oracle; test infrastructure only).

Section 3.3 defines ASM as z = sum_l R_l^T K_l^{-1} R_l y with K_l = R_l K R_l^T the matrix of a
subdomain (an element or a small patch of elements); the conclusions propose replacing the
exact local solve by an incomplete LU factorisation on multi-element subdomains. Here:

* subdomain l is the patch of elements [l G, (l+1) G) (G consecutive elements), its unknowns
  the trace blocks of the patch's faces in increasing face order;
* K_l is K restricted to those faces: block (a, b) is K[f_a][s] for the slot s with
  nbr[f_a][s] = f_b, zero when f_b is not a neighbour of f_a (the block pattern of K);
* block ILU(0) on that pattern in the natural order: for each block row i and each pattern
  column k < i, L_ik = A_ik A_kk^{-1} (A_kk as already updated), then A_ij -= L_ik A_kj for the
  pattern columns j > k of row i; U is the updated upper part (diagonal blocks included);
* z = sum_l R_l^T U_l^{-1} L_l^{-1} R_l y (unit block-lower L).

With G = 1 every pair of an element's faces is coupled in K, the pattern is dense and ILU(0)
is the exact block LU factorisation: the preconditioner is then the element ASM of Section 4.6.
K is the face-block matrix of oracle.assemble: K[f][s] stored [col][row], nbr[f][s] (-1 empty).
"""
import numpy as np


def subdomain_faces(e2f, G):
    """Sorted face lists of the patches of G consecutive elements."""
    ne = e2f.shape[0]
    return [np.unique(e2f[e0:min(e0 + G, ne)].ravel()) for e0 in range(0, ne, G)]


def local_matrix(K, nbr, faces):
    """(K_l as a dense block array [n][n][nb][nb] (row, col), pattern [n][n] bool)."""
    nb = K.shape[2]
    n = len(faces)
    pos = {int(f): a for a, f in enumerate(faces)}
    A = np.zeros((n, n, nb, nb))
    pat = np.zeros((n, n), dtype=bool)
    for a, f in enumerate(faces):
        for s in range(nbr.shape[1]):
            g = int(nbr[f, s])
            if g >= 0 and g in pos:
                b = pos[g]
                A[a, b] = K[f, s].T          # stored [col][row]
                pat[a, b] = True
    return A, pat


def block_ilu0(A, pat):
    """Block ILU(0) in place on a copy: returns (LU, pat) with the unit-lower multipliers below
    and U on and above the block diagonal."""
    F = A.copy()
    n = F.shape[0]
    for i in range(1, n):
        for k in range(i):
            if not pat[i, k]:
                continue
            F[i, k] = F[i, k] @ np.linalg.inv(F[k, k])
            for j in range(k + 1, n):
                if pat[i, j] and pat[k, j]:
                    F[i, j] = F[i, j] - F[i, k] @ F[k, j]
    return F


def lu_solve(F, pat, r):
    """U^{-1} L^{-1} r for the block factors of block_ilu0 (r: [n][nb])."""
    n = F.shape[0]
    x = np.array(r, dtype=np.float64, copy=True)
    for i in range(n):                       # forward: unit block-lower
        for k in range(i):
            if pat[i, k]:
                x[i] = x[i] - F[i, k] @ x[k]
    for i in range(n - 1, -1, -1):           # backward: block-upper
        for j in range(i + 1, n):
            if pat[i, j]:
                x[i] = x[i] - F[i, j] @ x[j]
        x[i] = np.linalg.solve(F[i, i], x[i])
    return x


def setup(K, nbr, e2f, G):
    """The factorised subdomains: a list of (faces, F, pattern)."""
    out = []
    for faces in subdomain_faces(e2f, G):
        A, pat = local_matrix(K, nbr, faces)
        out.append((faces, block_ilu0(A, pat), pat))
    return out


def apply(subs, y, nb):
    """z = sum_l R_l^T (L_l U_l)^{-1} R_l y."""
    Y = y.reshape(-1, nb)
    Z = np.zeros_like(Y)
    for faces, F, pat in subs:
        Z[faces] += lu_solve(F, pat, Y[faces])
    return Z.reshape(-1)
