"""Restarted (F)GMRES and block-Jacobi (oracle; test infrastructure only).

Section 3.1 / 4.4: restarted GMRES(m) with Arnoldi (classical or modified
Gram-Schmidt), Hessenberg reduction by Givens rotations and back substitution;
the update x += V y (here x += Z y for the flexible, right-preconditioned form).
Sections 3.2 / 4.5: block-Jacobi inverts the diagonal face blocks K_ff and
applies z_f = P_f^{-1} y_f face by face.

The paper preconditions on the left; the GPU path uses right-preconditioned
FGMRES so that the stopping test sees the true residual. Both are here:
`fgmres` (right) is the parity reference, `gmres_left` the paper's form.
"""
import numpy as np


def bj_inverses(K):
    """P_f^{-1} for every face: inverse of the slot-0 block. K is [f][s][col][row];
    the result is stored the same way, [f][col][row]."""
    nf = K.shape[0]
    out = np.zeros((nf,) + K.shape[2:])
    for f in range(nf):
        Kff = K[f, 0].T                      # [row][col]
        out[f] = np.linalg.inv(Kff).T
    return out


def bj_apply(Binv, y):
    nf, nb, _ = Binv.shape
    Y = y.reshape(nf, nb)
    return np.einsum("fcr,fc->fr", Binv, Y).reshape(-1)


def asm_matrices(Kbar, K, f2e, e2f, dims):
    """Additive Schwarz subdomain matrices, one per element (Section 4.6): start from the
    element Schur complement Kbar^e (nt x nt, row-major, blocks of nb = M P_F per local face)
    and replace the diagonal block of every local face l by the sum of both neighbours'
    diagonal blocks, Kbar^{e1}_{l1 l1} + Kbar^{e2}_{l2 l2} (on a boundary face only e1
    contributes). Faces in their canonical orientation (no permutation). Returns P [ne][nt][nt]."""
    M, PF, L = dims["ncomp"], dims["npf"], dims["nlfe"]
    nb = M * PF
    P = np.array(Kbar, dtype=np.float64, copy=True)
    for f in range(f2e.shape[0]):
        e1, l1, e2, l2 = (int(v) for v in f2e[f])
        if e2 < 0:
            continue
        s1 = slice(l1 * nb, (l1 + 1) * nb)
        s2 = slice(l2 * nb, (l2 + 1) * nb)
        enriched = Kbar[e1][s1, s1] + Kbar[e2][s2, s2]
        P[e1][s1, s1] = enriched
        P[e2][s2, s2] = enriched
    return P


def asm_inverses(P):
    return np.array([np.linalg.inv(Pe) for Pe in P])


def asm_apply(Pinv, e2f, y, dims):
    """z = sum_e R_e^T (P^e)^{-1} R_e y (Section 3.3 / 4.6): gather the element's face slices
    of y, apply the element inverse, add the result back onto the faces."""
    M, PF, L = dims["ncomp"], dims["npf"], dims["nlfe"]
    nb = M * PF
    nf = y.size // nb
    Y = y.reshape(nf, nb)
    Z = np.zeros_like(Y)
    for e in range(Pinv.shape[0]):
        ye = np.concatenate([Y[int(e2f[e, l])] for l in range(L)])
        ze = Pinv[e] @ ye
        for l in range(L):
            Z[int(e2f[e, l])] += ze[l * nb:(l + 1) * nb]
    return Z.reshape(-1)


def _orth(V, w, j, method):
    """Orthogonalise w against V[:j+1]; returns coefficients h (j+1,) and w."""
    if method == "mgs":
        h = np.zeros(j + 1)
        for i in range(j + 1):
            h[i] = V[i] @ w
            w = w - h[i] * V[i]
        return h, w
    h = V[:j + 1] @ w
    w = w - V[:j + 1].T @ h
    if method == "cgs2":
        h2 = V[:j + 1] @ w
        w = w - V[:j + 1].T @ h2
        h = h + h2
    return h, w


def _givens(a, b):
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def fgmres(matvec, b, prec=None, x0=None, restart=50, rtol=1e-10, atol=0.0, max_iters=1000,
           orth="cgs2", hist=None):
    """Right-preconditioned flexible GMRES(m). Stops when the true residual
    ||b - K x|| <= max(rtol ||b||, atol), checked at every restart and whenever the
    Givens estimate says so. Returns (x, info dict)."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    prec = prec if prec is not None else (lambda v: v)
    bnorm = np.linalg.norm(b)
    target = max(rtol * bnorm, atol)
    its = 0
    cycles = 0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if hist is not None:
            hist.append(beta)
        if beta <= target or its >= max_iters:
            return x, dict(iters=its, cycles=cycles, converged=beta <= target, resid=beta / bnorm)
        cycles += 1
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = prec(V[j])
            w = matvec(Z[j])
            h, w = _orth(V, w, j, orth)
            H[:j + 1, j] = h
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            if hist is not None:
                hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= target or its >= max_iters:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y


def gmres_dcgs2(matvec, b, prec=None, x0=None, restart=50, rtol=1e-10, atol=0.0, max_iters=1000, hist=None):
    """Right-preconditioned GMRES(m) (Section 3.1; x = x0 + M^{-1} V y, for a fixed linear
    preconditioner) whose Arnoldi process uses delayed classical Gram-Schmidt with
    reorthogonalisation (DCGS2: Swirydowicz, Langou, Ananthan, Yang, Thomas, Numer. Linear
    Algebra Appl. 28 (2021) e2343). Same iterates as CGS2 Arnoldi in exact arithmetic.

    Step j applies the operator B = K M^{-1} to the not yet reorthogonalised vector
    vt_j (one CGS pass, unnormalised) and takes all inner products in one sweep:
        a = V_{j-1}^T vt_j, alpha = vt_j^T vt_j, c = V_{j-1}^T wt, gamma = vt_j^T wt  (wt = B vt_j).
    Then  rho = sqrt(alpha - a^T a),  v_j = (vt_j - V_{j-1} a) / rho  (the delayed second pass),
    column j-1 of the Hessenberg matrix gains H[:j, j-1] += a and H[j, j-1] = rho, and with
    t = H[:j+1, :j] a (so that B v_j = (wt - V_j t) / rho) the new column and vector are
        h = ([c; (gamma - a^T c) / rho] - t) / rho,
        vt_{j+1} = wt / rho - V_j (t / rho + h).
    Column j-1 is thus final one step late, and so is the Givens residual estimate; a cycle
    that runs all m steps ends with one more reorthogonalisation sweep for vt_m.
    Returns (x, info) like fgmres."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    prec = prec if prec is not None else (lambda v: v)
    bnorm = np.linalg.norm(b)
    target = max(rtol * bnorm, atol)
    its = 0
    cycles = 0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if hist is not None:
            hist.append(beta)
        if beta <= target or its >= max_iters:
            return x, dict(iters=its, cycles=cycles, converged=beta <= target, resid=beta / bnorm)
        cycles += 1
        m = min(restart, max_iters - its)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        R = np.zeros((m + 1, m))          # H with the Givens rotations applied
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta

        def finish_column(col):
            """Apply the previous rotations and a new one to Hessenberg column col."""
            R[:col + 2, col] = H[:col + 2, col]
            for i in range(col):
                t = cs[i] * R[i, col] + sn[i] * R[i + 1, col]
                R[i + 1, col] = -sn[i] * R[i, col] + cs[i] * R[i + 1, col]
                R[i, col] = t
            cs[col], sn[col] = _givens(R[col, col], R[col + 1, col])
            R[col, col] = cs[col] * R[col, col] + sn[col] * R[col + 1, col]
            R[col + 1, col] = 0.0
            g[col + 1] = -sn[col] * g[col]
            g[col] = cs[col] * g[col]

        def reorth(j):
            """Delayed second pass for vt_j: returns a, rho and fixes column j-1."""
            a = V[:j] @ V[j]
            rho = np.sqrt(V[j] @ V[j] - a @ a)
            if j > 0:
                H[:j, j - 1] += a
                H[j, j - 1] = rho
            return a, rho

        k = 0
        done = False
        for j in range(m):
            wt = matvec(prec(V[j]))
            a, rho = reorth(j)
            if j > 0:
                finish_column(j - 1)
                its += 1
                k = j
                if hist is not None:
                    hist.append(abs(g[j]))
                if abs(g[j]) <= target or its >= max_iters:
                    done = True
                    break
            c = V[:j] @ wt
            gamma = V[j] @ wt
            t = H[:j + 1, :j] @ a
            vj = (V[j] - V[:j].T @ a) / rho
            h = (np.append(c, (gamma - a @ c) / rho) - t) / rho
            V[j] = vj
            V[j + 1] = wt / rho - V[:j + 1].T @ (t / rho + h)
            H[:j + 1, j] = h
        if not done:
            reorth(m)
            finish_column(m - 1)
            its += 1
            k = m
            if hist is not None:
                hist.append(abs(g[m]))
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - R[i, i + 1:k] @ y[i + 1:k]) / R[i, i]
        x = x + prec(V[:k].T @ y)


def gmres_left(matvec, b, prec, restart=50, rtol=1e-6, max_iters=1000, orth="cgs"):
    """Left-preconditioned GMRES(m) as the paper states it (Section 3.1):
    GMRES on P^{-1} K x = P^{-1} b, stopping on the preconditioned residual."""
    op = lambda v: prec(matvec(v))
    pb = prec(b)
    x, info = fgmres(op, pb, None, None, restart, rtol, 0.0, max_iters, orth)
    return x, info
