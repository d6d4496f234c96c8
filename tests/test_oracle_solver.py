"""Pins of the oracle's Krylov solver and preconditioners against mathematics.

FGMRES: identity in one iteration, termination within N iterations with a full
Krylov space, monotone residual estimates within a cycle, agreement with a
direct solve. Block-Jacobi: P_f^{-1} K_ff = I. Polynomial preconditioner
(Section 4.7): closed form on diagonal matrices, the residual polynomial
vanishing at every harmonic Ritz value, p(B) = B^{-1} when P = N, the
harmonic Ritz values as roots of the GMRES(P) residual polynomial, the
real paired recurrence equal to the complex product form. Chebyshev: the
textbook error bound on an SPD diagonal matrix.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from oracle import krylov, poly
from workloads import configs

from helpers import oracle_pipeline


def test_fgmres_identity_one_iteration():
    b = np.random.default_rng(0).standard_normal(50)
    x, info = krylov.fgmres(lambda v: v, b, rtol=1e-13)
    assert info["iters"] == 1 and info["converged"]
    assert np.allclose(x, b, atol=1e-14)


@pytest.mark.parametrize("orth", ["mgs", "cgs", "cgs2"])
def test_fgmres_full_space_terminates(orth):
    rng = np.random.default_rng(1)
    N = 30
    A = rng.standard_normal((N, N)) + N * np.eye(N) * 0.3
    b = rng.standard_normal(N)
    hist = []
    x, info = krylov.fgmres(lambda v: A @ v, b, restart=N, rtol=1e-12, orth=orth, hist=hist)
    assert info["converged"] and info["iters"] <= N
    assert np.linalg.norm(A @ x - b) <= 1e-11 * np.linalg.norm(b)
    est = hist[1:info["iters"] + 1]
    assert all(est[i + 1] <= est[i] * (1 + 1e-12) for i in range(len(est) - 1))


def test_fgmres_bj_matches_direct_on_c1():
    pb = configs.c1()
    out = oracle_pipeline(pb)
    A = out["A"]
    Binv = krylov.bj_inverses(out["K"])
    for f in range(out["K"].shape[0]):
        assert np.allclose(Binv[f].T @ out["K"][f, 0].T, np.eye(pb.nb), atol=1e-12)
    x, info = krylov.fgmres(lambda v: A @ v, out["r"], prec=lambda v: krylov.bj_apply(Binv, v),
                            restart=50, rtol=1e-12)
    assert info["converged"]
    assert np.linalg.norm(x - out["x"]) <= 1e-10 * np.linalg.norm(out["x"])


def test_pp_diagonal_closed_form():
    lam = np.linspace(0.5, 4.0, 40)
    theta = poly.leja_order(np.array([0.7, 1.5, 2.5 + 0.3j, 2.5 - 0.3j, 3.6]))
    y = np.random.default_rng(2).standard_normal(40)
    z = poly.apply_product(lambda v: lam * v, theta, y)
    assert np.allclose(z, poly.p_scalar(theta, lam).real * y, rtol=1e-12, atol=1e-13)
    # 1 - lam p(lam) = prod (1 - lam/theta_j) vanishes at every theta_j
    assert np.abs(1 - theta * poly.p_scalar(theta, theta)).max() < 1e-12
    assert np.abs(poly.residual_poly(theta, theta)).max() < 1e-12


def test_pp_full_degree_is_exact_inverse():
    rng = np.random.default_rng(3)
    N = 12
    Bm = rng.standard_normal((N, N)) * 0.2 + np.diag(np.linspace(1, 3, N))
    H, V = poly.arnoldi_mgs(lambda v: Bm @ v, rng.standard_normal(N), N)
    th = poly.leja_order(poly.harmonic_ritz(H))
    ev = np.sort_complex(np.linalg.eigvals(Bm))
    assert np.allclose(np.sort_complex(th), ev, atol=1e-8)
    y = rng.standard_normal(N)
    z = poly.apply_product(lambda v: Bm @ v, th, y)
    assert np.allclose(z, np.linalg.solve(Bm, y), rtol=1e-8, atol=1e-9)


def test_harmonic_ritz_are_gmres_residual_roots():
    rng = np.random.default_rng(4)
    N, P = 60, 8
    Bm = rng.standard_normal((N, N)) * 0.1 + np.diag(np.linspace(1, 5, N))
    v = rng.standard_normal(N)
    H, V = poly.arnoldi_mgs(lambda u: Bm @ u, v, P)
    th = poly.harmonic_ritz(H)
    # || pi(B) v || equals the GMRES(P) residual norm min_y || beta e1 - H y ||
    r = v.astype(complex)
    for t in th:
        r = r - (Bm @ r) / t
    beta = np.linalg.norm(v)
    e1 = np.zeros(P + 1)
    e1[0] = beta
    y, *_ = np.linalg.lstsq(H, e1, rcond=None)
    gm = np.linalg.norm(e1 - H @ y)
    assert abs(np.linalg.norm(r) - gm) < 1e-10 * beta


def test_paired_real_recurrence_equals_product_form():
    rng = np.random.default_rng(5)
    N = 40
    Bm = rng.standard_normal((N, N)) * 0.1 + np.diag(np.linspace(1, 4, N))
    H, V = poly.arnoldi_mgs(lambda u: Bm @ u, rng.standard_normal(N), 10)
    th = poly.leja_order(poly.harmonic_ritz(H))
    assert np.any(th.imag != 0)
    y = rng.standard_normal(N)
    # real recurrence: w += q/theta, q -= Bq/theta; pairs: w += (2a q - Bq)/|t|^2,
    # q -= (2a/|t|^2) Bq - (1/|t|^2) B^2 q
    q, w = y.copy(), np.zeros(N)
    j = 0
    while j < len(th):
        t = th[j]
        last = (j + (2 if t.imag != 0 else 1)) >= len(th)
        if t.imag == 0:
            w = w + q / t.real
            if not last:
                q = q - (Bm @ q) / t.real
            j += 1
        else:
            a, m2 = t.real, abs(t) ** 2
            Bq = Bm @ q
            w = w + (2 * a * q - Bq) / m2
            if not last:
                q = q - (2 * a / m2) * Bq + (Bm @ Bq) / m2
            j += 2
    z = poly.apply_product(lambda u: Bm @ u, th, y)
    assert np.allclose(w, z, rtol=1e-11, atol=1e-12)


def test_chebyshev_bound_spd_diagonal():
    lam = np.linspace(1.0, 100.0, 200)
    b = np.random.default_rng(6).standard_normal(200)
    for P in (3, 6, 10):
        x = poly.chebyshev(lambda v: lam * v, b, 1.0, 100.0, P)
        # residual after P iterates: b - A x_P; bound 2 ((sqrt(k)-1)/(sqrt(k)+1))^P
        kap = 100.0
        bound = 2 * ((np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)) ** P
        assert np.linalg.norm(b - lam * x) <= bound * np.linalg.norm(b) * (1 + 1e-12)


def test_leja_keeps_pairs_adjacent_and_starts_at_max_modulus():
    th = np.array([1.0, 2 + 1j, 2 - 1j, 0.5, 3.0])
    o = poly.leja_order(th)
    assert abs(o[0]) == max(abs(th))
    for k, t in enumerate(o):
        if t.imag > 0:
            assert o[k + 1] == np.conj(t)


def _krylov_min_residual(B, r0, k):
    """min over y of ||r0 - B K y|| with K an orthonormal basis of span{r0, B r0, ..., B^{k-1} r0}
    (explicit Krylov vectors, orthonormalised by a QR factorisation, then least squares)."""
    vecs = [r0]
    for _ in range(k - 1):
        vecs.append(B @ vecs[-1])
    Q, _ = np.linalg.qr(np.array(vecs).T)
    y, *_ = np.linalg.lstsq(B @ Q, r0, rcond=None)
    return np.linalg.norm(r0 - B @ Q @ y)


def _block_system(seed, nf=12, nb=5, off=0.3):
    rng = np.random.default_rng(seed)
    N = nf * nb
    A = rng.standard_normal((N, N)) * off + np.diag(2.0 + rng.random(N))
    Binv = np.zeros((nf, nb, nb))
    for f in range(nf):
        blk = A[f * nb:(f + 1) * nb, f * nb:(f + 1) * nb]
        Binv[f] = np.linalg.inv(blk).T
    return A, Binv, rng.standard_normal(N)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_gmres_dcgs2_is_minimal_residual(k):
    """After k steps, right-preconditioned GMRES attains the least-squares minimum of
    ||b - K M^{-1} u|| over the Krylov space of K M^{-1} (brute force)."""
    A, Binv, b = _block_system(3)
    prec = lambda v: krylov.bj_apply(Binv, v)
    B = A @ np.array([prec(e) for e in np.eye(A.shape[0])]).T
    hist = []
    x, info = krylov.gmres_dcgs2(lambda v: A @ v, b, prec=prec, restart=50, rtol=0.0, max_iters=k, hist=hist)
    assert info["iters"] == k
    ref = _krylov_min_residual(B, b, k)
    assert abs(np.linalg.norm(b - A @ x) - ref) <= 1e-10 * np.linalg.norm(b)
    assert abs(hist[k] - ref) <= 1e-10 * np.linalg.norm(b)       # Givens estimate


def test_gmres_dcgs2_matches_cgs2_fgmres_iterates():
    """Delayed reorthogonalisation changes no iterate (exact arithmetic): the residual
    histories of DCGS2-GMRES and CGS2-FGMRES agree step by step over several restarts."""
    A, Binv, b = _block_system(4, nf=30, nb=4, off=0.1)
    prec = lambda v: krylov.bj_apply(Binv, v)
    h1, h2 = [], []
    x1, i1 = krylov.fgmres(lambda v: A @ v, b, prec=prec, restart=7, rtol=1e-11, max_iters=400, hist=h1)
    x2, i2 = krylov.gmres_dcgs2(lambda v: A @ v, b, prec=prec, restart=7, rtol=1e-11, max_iters=400, hist=h2)
    assert i1["converged"] and i2["converged"] and i1["iters"] == i2["iters"] and i1["cycles"] == i2["cycles"]
    assert len(h1) == len(h2)
    bn = np.linalg.norm(b)
    assert max(abs(p - q) for p, q in zip(h1, h2)) <= 1e-9 * bn
    assert np.linalg.norm(x1 - x2) <= 1e-9 * np.linalg.norm(x1)


def test_gmres_dcgs2_bj_matches_direct_on_c1():
    pb = configs.c1()
    out = oracle_pipeline(pb)
    Binv = krylov.bj_inverses(out["K"])
    x, info = krylov.gmres_dcgs2(lambda v: out["A"] @ v, out["r"], prec=lambda v: krylov.bj_apply(Binv, v),
                                 restart=20, rtol=1e-12)
    assert info["converged"] and info["cycles"] >= 2
    assert np.linalg.norm(x - out["x"]) <= 1e-10 * np.linalg.norm(out["x"])


def _face_dofs(f, nb):
    return np.arange(f * nb, (f + 1) * nb)


@pytest.mark.parametrize("make", [lambda: configs.c1(n=3), lambda: configs.c2(n=2, p=1),
                                  lambda: configs.c5(n=1, p=1)])
def test_asm_subdomain_matrix_is_restricted_global_matrix(make):
    """The enriched element matrix equals R_e K R_e^T: the assembled global matrix restricted
    to the faces of the element (Section 3.3 defines K_l that way)."""
    pb = make()
    out = oracle_pipeline(pb)
    d = pb.dims()
    nb = d["ncomp"] * d["npf"]
    P = krylov.asm_matrices(out["Kbar"], out["K"], pb.mesh.f2e, pb.mesh.e2f, d)
    A = out["A"].tocsr()
    for e in range(pb.mesh.ne):
        idx = np.concatenate([_face_dofs(int(f), nb) for f in pb.mesh.e2f[e]])
        Re = A[idx][:, idx].toarray()
        assert np.allclose(P[e], Re, rtol=0, atol=1e-12 * np.abs(Re).max())


def test_asm_single_element_is_exact_inverse():
    """One element: every face belongs to it, so ASM is the exact inverse of K."""
    pb = configs.c1(n=1)
    out = oracle_pipeline(pb)
    d = pb.dims()
    Pinv = krylov.asm_inverses(krylov.asm_matrices(out["Kbar"], out["K"], pb.mesh.f2e, pb.mesh.e2f, d))
    y = np.random.default_rng(3).standard_normal(out["r"].size)
    z = krylov.asm_apply(Pinv, pb.mesh.e2f, y, d)
    assert np.allclose(out["A"] @ z, y, atol=1e-11 * np.abs(y).max())


def test_asm_converges_faster_than_bj():
    """ASM-preconditioned FGMRES needs fewer iterations than block-Jacobi on the Poisson
    workload (the paper's observation, Section 5), and both reach the direct solution."""
    pb = configs.c1()
    out = oracle_pipeline(pb)
    d = pb.dims()
    Pinv = krylov.asm_inverses(krylov.asm_matrices(out["Kbar"], out["K"], pb.mesh.f2e, pb.mesh.e2f, d))
    A = out["A"]
    x1, i_asm = krylov.fgmres(lambda v: A @ v, out["r"], prec=lambda v: krylov.asm_apply(Pinv, pb.mesh.e2f, v, d),
                              restart=50, rtol=1e-11)
    Binv = krylov.bj_inverses(out["K"])
    x2, i_bj = krylov.fgmres(lambda v: A @ v, out["r"], prec=lambda v: krylov.bj_apply(Binv, v),
                             restart=50, rtol=1e-11)
    assert i_asm["converged"] and i_bj["converged"] and i_asm["iters"] < i_bj["iters"]
    for x in (x1, x2):
        assert np.linalg.norm(x - out["x"]) <= 1e-9 * np.linalg.norm(out["x"])


def test_bj_apply_inverts_each_diagonal_block():
    """bj_apply(bj_inverses(K), K_ff y_f) = y_f face by face for non-symmetric blocks stored
    column-major ([f][s][col][row]); a transposed apply (P_f^{-T}) fails this."""
    rng = np.random.default_rng(21)
    nf, nb, S = 7, 4, 3
    K = rng.standard_normal((nf, S, nb, nb))
    for f in range(nf):
        K[f, 0] += 3.0 * np.eye(nb) + np.triu(rng.standard_normal((nb, nb)), 1) * 2.0
    y = rng.standard_normal(nf * nb)
    Ky = np.concatenate([K[f, 0].T @ y[f * nb:(f + 1) * nb] for f in range(nf)])   # K_ff[row][col] = K[f,0,col,row]
    Binv = krylov.bj_inverses(K)
    assert np.allclose(krylov.bj_apply(Binv, Ky), y, rtol=1e-12, atol=1e-12)
    transposed = np.einsum("frc,fc->fr", Binv, Ky.reshape(nf, nb)).reshape(-1)
    assert not np.allclose(transposed, y, atol=1e-3)


def test_bj_apply_hand_example():
    """One 2x2 face block K_ff = [[1, 2], [0, 1]] (row-major), stored column-major as
    [[1, 0], [2, 1]]: P^{-1} = [[1, -2], [0, 1]], so P^{-1} (0, 1) = (-2, 1)."""
    K = np.zeros((1, 1, 2, 2))
    K[0, 0] = [[1.0, 0.0], [2.0, 1.0]]        # [col][row]
    Binv = krylov.bj_inverses(K)
    assert np.array_equal(Binv[0], np.array([[1.0, 0.0], [-2.0, 1.0]]))
    assert np.array_equal(krylov.bj_apply(Binv, np.array([0.0, 1.0])), np.array([-2.0, 1.0]))


def test_leja_greedy_choice_hand_example():
    """Leja order of {1, 4.4, 0.5, 8}, worked by hand: start at the largest modulus 8; the
    farthest from 8 is 0.5 (7.5); then the product of distances to {8, 0.5} is 7 x 0.5 = 3.5
    for 1 and 3.6 x 3.9 = 14.04 for 4.4, so 4.4; then 1. (A sum of distances would tie at
    7.5 and take 1 first.) The second example separates the product from a max-min rule:
    {10, 0.1, 4, 1.5, 8.9} starts 10, 0.1 (9.9 away), then 4 (6 x 3.9 = 23.4 against
    8.5 x 1.4 = 11.9 and 1.1 x 8.8 = 9.68); with {10, 0.1, 4} chosen, 8.9 scores
    1.1 x 8.8 x 4.9 = 47.4 and 1.5 scores 8.5 x 1.4 x 2.5 = 29.8, so 8.9 comes before 1.5,
    where the largest smallest distance (1.4 against 1.1) would take 1.5."""
    o = poly.leja_order(np.array([1.0, 4.4, 0.5, 8.0]))
    assert np.array_equal(o, np.array([8.0, 0.5, 4.4, 1.0], complex))
    o = poly.leja_order(np.array([10.0, 0.1, 4.0, 1.5, 8.9]))
    assert np.array_equal(o, np.array([10.0, 0.1, 4.0, 8.9, 1.5], complex))


def test_leja_conjugate_pair_follows_partner():
    """{3, 1+2i, 1-2i, 2.5}: start at 3 (|1+2i| = 2.24); |1+2i - 3| = 2.83 beats |2.5 - 3| = 0.5,
    so the pair comes next, positive imaginary part first, then 2.5."""
    o = poly.leja_order(np.array([3.0, 1 + 2j, 1 - 2j, 2.5]))
    assert np.array_equal(o, np.array([3.0, 1 + 2j, 1 - 2j, 2.5]))


def test_pof_hand_example():
    """theta = {1, 2, 4}: at the root 1 the other factors are |1 - 1/2| |1 - 1/4| = 0.375; at 4 they
    are |1 - 4| |1 - 2| = 3."""
    assert poly.pof(np.array([1.0, 2.0, 4.0]), 0) == pytest.approx(0.375, rel=1e-15)
    assert poly.pof(np.array([1.0, 2.0, 4.0]), 2) == pytest.approx(3.0, rel=1e-15)


def test_added_roots_hand_examples():
    """pi(z) = prod (1 - z/theta) at 1.1 t, t the root of largest real part, worked by hand:
    {1, 2}: (1 - 1.1)(1 - 2.2) = 0.12, nothing added; {0.05, 1}: (1 - 22)(1 - 1.1) = 2.1 > 1, one
    copy of 1 makes it 2.1 x (-0.1) = -0.21, so one copy; {0.001, 1}: (1 - 1100)(-0.1) = 109.9, then
    10.99, then 1.099 -- still above 1, but at most two copies are added."""
    assert poly.added_roots(np.array([1.0, 2.0])).size == 0
    assert np.array_equal(poly.added_roots(np.array([0.05, 1.0])), np.array([1.0], complex))
    assert np.array_equal(poly.added_roots(np.array([0.001, 1.0])), np.array([1.0, 1.0], complex))
    # a complex outermost root t = 1 + 0.1i goes in with its conjugate. At 1.1 t the factors of t
    # and conj(t) have moduli |1 - 1.1| = 0.1 and |1 - 1.1 t / conj(t)| = |1 - 1.1 (0.99 + 0.2i) /
    # 1.01| = |-0.07822 - 0.21782i| = 0.23144; with 0.03 as the third value its factor is
    # |1 - (36.667 + 3.667i)| = 35.855 and |pi| = 0.8298, nothing added; with 0.002 it is
    # |1 - (550 + 55i)| = 551.75, |pi| = 12.77, and one pair brings it to 12.77 x 0.02314 = 0.2955
    t = 1 + 0.1j
    assert abs(poly.residual_poly(np.array([0.03, t, np.conj(t)]), 1.1 * t)) == pytest.approx(0.8298, rel=1e-3)
    assert poly.added_roots(np.array([0.03, t, np.conj(t)])).size == 0
    add = poly.added_roots(np.array([0.002, t, np.conj(t)]))
    assert add.size == 2 and set(np.round(add, 15)) == {t, np.conj(t)}
    # a single value or a spectrum in the left half plane: nothing to add
    assert poly.added_roots(np.array([0.5])).size == 0
    assert poly.added_roots(np.array([-1.0, -2.0])).size == 0


def test_added_roots_only_damp_the_residual_polynomial():
    """Each copy of a real root t multiplies pi by (1 - z/t), of modulus below 1 on (0, 2t): the
    residual polynomial with the copies is nowhere larger in modulus there."""
    th = np.array([0.01, 0.2, 0.9, 1.7, 2.4, 2.95])
    add = poly.added_roots(th)
    assert add.size >= 1
    z = np.linspace(1e-3, 2 * 2.95 - 1e-3, 4001)
    old = np.abs([poly.residual_poly(th, x) for x in z])
    new = np.abs([poly.residual_poly(np.concatenate([th, add]), x) for x in z])
    assert np.all(new <= old * (1 + 1e-14))


@pytest.mark.parametrize("spectrum", ["geometric", "outliers"])
def test_added_roots_make_p_b_b_positive_on_model_spectra(spectrum):
    """The safeguard's purpose, on diagonal matrices whose spectra reach past the harmonic Ritz
    values of a 10-step Arnoldi cycle (geometric on [0.01, 3.1]; uniform on [0.01, 2.6] with three
    outliers at 2.9, 3.0, 3.4): with the added roots, lambda p(lambda) = 1 - pi(lambda) is
    positive at every eigenvalue for eight start vectors, so p(B) B is positive definite; on the
    geometric spectrum it is negative at some eigenvalue for at least one start vector without
    them."""
    N = 300
    lam = (np.geomspace(0.01, 3.1, N) if spectrum == "geometric"
           else np.concatenate([np.linspace(0.01, 2.6, N - 3), [2.9, 3.0, 3.4]]))
    worst_without = np.inf
    for seed in range(8):
        rng = np.random.default_rng(seed)
        H, _ = poly.arnoldi_mgs(lambda v: lam * v, rng.standard_normal(N), 10)
        roots, n_added = poly.pp_roots(H)
        th = poly.harmonic_ritz(H)
        assert n_added == roots.size - th.size
        with_add = min((1 - poly.residual_poly(roots, x)).real for x in lam)
        without = min((1 - poly.residual_poly(th, x)).real for x in lam)
        assert with_add > 0.1, (seed, with_add)
        worst_without = min(worst_without, without)
    assert worst_without < 0 or spectrum == "outliers"


def test_pp_roots_leja_order_with_copies():
    """{0.05, 1} gets one copy of 1 (hand example above); Leja order starts at the largest
    modulus, 1, then 0.05, and the copy, at distance zero from its twin, comes last."""
    o = poly.leja_order(np.concatenate([np.array([0.05, 1.0]), poly.added_roots(np.array([0.05, 1.0]))]),
                        drop_rel=0.0)
    assert np.array_equal(o, np.array([1.0, 0.05, 1.0], complex))
    o = poly.leja_order(np.array([3.0, 0.5, 3.0, 3.0, 1.0]), drop_rel=0.0)
    assert np.array_equal(o, np.array([3.0, 0.5, 1.0, 3.0, 3.0], complex))


def test_leja_drops_tiny_values():
    o = poly.leja_order(np.array([2.0, 1e-14, 1.0]), drop_rel=1e-12)
    assert np.array_equal(o, np.array([2.0, 1.0], complex))


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_gmres_left_is_minimal_preconditioned_residual(k):
    """Left-preconditioned GMRES (Section 3.1) after k steps minimises ||P^{-1}(b - K x)|| over
    x in the Krylov space of P^{-1}K started at P^{-1}b (brute force), which differs from the
    right-preconditioned minimum of ||b - K x||."""
    A, Binv, b = _block_system(5)
    prec = lambda v: krylov.bj_apply(Binv, v)
    Pinv = np.array([prec(e) for e in np.eye(A.shape[0])]).T
    x, info = krylov.gmres_left(lambda v: A @ v, b, prec, restart=50, rtol=0.0, max_iters=k)
    assert info["iters"] == k
    ref = _krylov_min_residual(Pinv @ A, Pinv @ b, k)
    assert abs(np.linalg.norm(Pinv @ (b - A @ x)) - ref) <= 1e-10 * np.linalg.norm(Pinv @ b)
    if k > 1:
        xr, _ = krylov.fgmres(lambda v: A @ v, b, prec=prec, restart=50, rtol=0.0, max_iters=k)
        assert np.linalg.norm(x - xr) > 1e-8 * np.linalg.norm(xr)


def test_gmres_left_exact_preconditioner_one_step():
    A, _, b = _block_system(6)
    Ainv = np.linalg.inv(A)
    x, info = krylov.gmres_left(lambda v: A @ v, b, lambda v: Ainv @ v, rtol=1e-12)
    assert info["converged"] and info["iters"] == 1
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("orth", ["cgs", "mgs", "cgs2"])
@pytest.mark.parametrize("k", [1, 3, 6])
def test_fgmres_each_orth_is_minimal_residual(orth, k):
    """Right-preconditioned FGMRES with a fixed preconditioner attains, after k steps, the
    least-squares minimum of ||b - K M^{-1} u|| over the Krylov space (brute force), whichever
    Gram-Schmidt variant builds the basis (Section 4.4 names CGS and MGS)."""
    A, Binv, b = _block_system(7)
    prec = lambda v: krylov.bj_apply(Binv, v)
    B = A @ np.array([prec(e) for e in np.eye(A.shape[0])]).T
    hist = []
    x, info = krylov.fgmres(lambda v: A @ v, b, prec=prec, restart=50, rtol=0.0, max_iters=k, orth=orth,
                            hist=hist)
    ref = _krylov_min_residual(B, b, k)
    assert abs(np.linalg.norm(b - A @ x) - ref) <= 1e-10 * np.linalg.norm(b)
    assert abs(hist[k] - ref) <= 1e-10 * np.linalg.norm(b)
