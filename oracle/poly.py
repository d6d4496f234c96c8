"""Polynomial preconditioner (oracle; test infrastructure only).

Section 3.4 and Section 4.7:
  * one Arnoldi/GMRES(P) cycle with modified Gram-Schmidt from a random vector
    gives the Hessenberg H_{P+1,P};
  * the harmonic Ritz values theta_j are the eigenvalues of
    H_{P,P} + h_{P+1,P}^2 (H_{P,P}^T)^{-1} e_P e_P^T;
  * they are put in Leja order, complex-conjugate pairs adjacent;
  * the preconditioner is p(B) = sum_j Q_j with
    Q_j = (I - B/theta_1)...(I - B/theta_{j-1}) / theta_j.
Hybrid form (Section 4.7): z = p(B) M^{-1} y with B = M^{-1} K, M the block-Jacobi
preconditioner, and the theta_j taken from Arnoldi on B.

The apply here is the complex product form evaluated literally (complex128),
keeping the real part; the GPU path uses a real paired recurrence instead.
Chebyshev acceleration (Saad, Iterative Methods for Sparse Linear Systems,
2nd ed., Algorithm 12.1) is the alternative smoother on a real interval.
"""
import numpy as np


def arnoldi_mgs(op, v0, P):
    """H (P+1, P) and basis V (P+1, n) of one Arnoldi cycle with MGS."""
    n = v0.shape[0]
    V = np.zeros((P + 1, n))
    H = np.zeros((P + 1, P))
    V[0] = v0 / np.linalg.norm(v0)
    for j in range(P):
        w = op(V[j])
        for i in range(j + 1):
            H[i, j] = V[i] @ w
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:
            return H[:j + 2, :j + 1], V[:j + 2]
        V[j + 1] = w / H[j + 1, j]
    return H, V


def harmonic_ritz(H):
    """Eigenvalues of H_P + h^2 H_P^{-T} e_P e_P^T (Section 4.7)."""
    P = H.shape[1]
    Hp = H[:P, :P].copy()
    h = H[P, P - 1] if H.shape[0] > P else 0.0
    eP = np.zeros(P)
    eP[-1] = 1.0
    f = np.linalg.solve(Hp.T, eP)
    Hm = Hp.copy()
    Hm[:, -1] += h * h * f
    return np.linalg.eigvals(Hm)


def leja_order(theta, drop_rel=1e-12):
    """Leja ordering with conjugate pairs adjacent (positive imaginary part first).

    Start with the value of largest modulus; then repeatedly take the candidate
    maximising the product of distances to the values already chosen (sum of
    logs; a value equal to a chosen one scores minus infinity); ties go to the lower
    index. Values with |theta| < drop_rel*max|theta| are dropped. A repeated value (the
    added roots of the safeguard below) is a candidate as often as it occurs."""
    th = np.asarray(theta, complex)
    th = th[np.abs(th) >= drop_rel * np.abs(th).max()]
    # canonicalise: real values exactly real, pairs as (a+ib, a-ib) with b > 0 kept once
    reals = [complex(t.real, 0.0) for t in th if t.imag == 0.0]
    ups = [t for t in th if t.imag > 0.0]
    cand = reals + ups
    out = []
    remaining = list(range(len(cand)))
    while remaining:
        if not out:
            scores = [abs(cand[k]) for k in remaining]
        else:
            scores = [sum(np.log(abs(cand[k] - s)) if cand[k] != s else -np.inf for s in out)
                      for k in remaining]
        best = remaining[int(np.argmax(scores))]
        remaining.remove(best)
        t = cand[best]
        out.append(t)
        if t.imag > 0.0:
            out.append(np.conj(t))
    return np.array(out)


def pof(theta, k):
    """Product of the other factors at root k: prod_{i != k} |1 - theta_k / theta_i| (Loe and
    Morgan, Numer. Linear Algebra Appl. 29 (2022) e2427). |pi(lambda)| near theta_k grows like
    pof(k) |lambda - theta_k| / |theta_k|."""
    th = np.asarray(theta, complex)
    return float(np.prod([abs(1 - th[k] / th[i]) for i in range(th.size) if i != k]))


def added_roots(theta, reach=1.1, max_copies=2):
    """Safeguard (not in the paper): extra copies of the outermost root.

    Harmonic Ritz values from one short Arnoldi cycle can stop short of the upper end of the
    spectrum of B. Just beyond the root of largest real part t the residual polynomial
    pi(z) = prod_j (1 - z / theta_j) grows like pof(k) times the relative distance, and where it
    exceeds 1 in modulus with the wrong sign, z p(z) = 1 - pi(z) turns negative: p(B) B becomes
    indefinite and GMRES stalls. While |pi(reach * t)| > 1 (the polynomial is not safe 10%
    beyond its outermost root), one more copy of t (and of its conjugate, for a complex root) is
    added, up to max_copies: each copy multiplies pi by (1 - z/t), of modulus below 1 on
    (0, 2 Re t) for real t, so it only damps pi over the spectrum, and by 0.1 at reach * t. This
    is the added-roots idea of Loe and Morgan applied to the outermost root with a test on pi
    itself. Returns the values to add (possibly empty)."""
    th = np.asarray(theta, complex)
    if th.size < 2:
        return np.zeros(0, complex)
    t = th[int(np.argmax(th.real))]
    if not t.real > 0.0:
        return np.zeros(0, complex)
    add = []
    for _ in range(max_copies):
        if abs(residual_poly(np.concatenate([th, np.array(add, complex)]), reach * t)) <= 1.0:
            break
        add += [t, np.conj(t)] if t.imag != 0.0 else [t]
    return np.array(add, complex)


def pp_roots(H, drop_rel=1e-12):
    """The roots the polynomial preconditioner uses: the harmonic Ritz values (those below
    drop_rel of the largest modulus dropped), the added copies of added_roots, all in Leja
    order (a duplicate has distance zero to its twin and so comes after every other value).
    Returns (roots, number added)."""
    th = np.asarray(harmonic_ritz(H), complex)
    th = th[np.abs(th) >= drop_rel * np.abs(th).max()]
    # canonical pairs: exactly conjugate members
    th = np.array([complex(t.real, 0.0) if t.imag == 0.0 else t for t in th])
    add = added_roots(th)
    return leja_order(np.concatenate([th, add]), drop_rel=0.0), int(add.size)


def apply_product(opB, theta, t):
    """z = sum_j Q_j t, Q_j = prod_{i<j} (I - B/theta_i) / theta_j, in complex arithmetic."""
    q = t.astype(complex)
    z = np.zeros_like(q)
    for j, th in enumerate(theta):
        z = z + q / th
        if j + 1 < len(theta):
            Bq = opB(q.real) + 1j * opB(q.imag)
            q = q - Bq / th
    return z.real


def residual_poly(theta, lam):
    """pi(lambda) = prod_j (1 - lambda/theta_j) = 1 - lambda p(lambda)."""
    lam = np.asarray(lam, complex)
    out = np.ones_like(lam)
    for th in theta:
        out = out * (1 - lam / th)
    return out


def p_scalar(theta, lam):
    """p(lambda) = sum_j prod_{i<j}(1 - lambda/theta_i) / theta_j."""
    lam = np.asarray(lam, complex)
    out = np.zeros_like(lam)
    pr = np.ones_like(lam)
    for th in theta:
        out = out + pr / th
        pr = pr * (1 - lam / th)
    return out


def chebyshev(opA, b, alpha, beta, P):
    """Chebyshev acceleration on [alpha, beta] (Saad, Algorithm 12.1), x0 = 0,
    P iterates (P-1 applications of A). Returns x_P."""
    th = 0.5 * (beta + alpha)
    de = 0.5 * (beta - alpha)
    s1 = th / de
    rho = 1.0 / s1
    x = np.zeros_like(b)
    r = b.copy()
    d = r / th
    for k in range(P):
        x = x + d
        if k + 1 == P:
            break
        r = r - opA(d)
        rho_n = 1.0 / (2 * s1 - rho)
        d = rho_n * rho * d + (2 * rho_n / de) * r
        rho = rho_n
    return x
