"""Pins of the oracle's ILU-ASM (block ILU(0) on multi-element subdomains, additive):

* one-element subdomains: the pattern is dense, ILU(0) is the exact factorisation and the
  preconditioner equals the element ASM (itself pinned to the restricted global matrix);
* the defining property of ILU(0): (L U)_ij = A_ij on every pattern block;
* a subdomain covering the whole mesh with a dense block pattern would be an exact solve; with
  the sparse face pattern the factorisation is inexact, but the apply is still a fixed linear
  map, so FGMRES with it reaches the direct solution.
"""
import numpy as np
import pytest

from oracle import assemble, condense, ilu_asm, krylov
from workloads import configs

from helpers import oracle_pipeline


def _c1():
    pb = configs.c1(n=4)
    return pb, oracle_pipeline(pb)


def test_single_element_subdomains_equal_element_asm():
    pb, out = _c1()
    d = pb.dims()
    nb = d["ncomp"] * d["npf"]
    subs = ilu_asm.setup(out["K"], out["nbr"], pb.mesh.e2f, 1)
    Pinv = krylov.asm_inverses(krylov.asm_matrices(out["Kbar"], out["K"], pb.mesh.f2e, pb.mesh.e2f, d))
    y = np.random.default_rng(3).standard_normal(out["r"].size)
    z_ilu = ilu_asm.apply(subs, y, nb)
    z_asm = krylov.asm_apply(Pinv, pb.mesh.e2f, y, d)
    assert np.abs(z_ilu - z_asm).max() <= 1e-11 * np.abs(z_asm).max()
    assert all(pat.all() for _, _, pat in subs)                 # dense patterns


@pytest.mark.parametrize("G", [2, 4, 8])
def test_ilu0_reproduces_the_matrix_on_its_pattern(G):
    pb, out = _c1()
    for faces in ilu_asm.subdomain_faces(pb.mesh.e2f, G)[:3]:
        A, pat = ilu_asm.local_matrix(out["K"], out["nbr"], faces)
        F = ilu_asm.block_ilu0(A, pat)
        n, nb = F.shape[0], F.shape[2]
        Lm = np.zeros((n * nb, n * nb))
        Um = np.zeros((n * nb, n * nb))
        for i in range(n):
            for j in range(n):
                if i > j and pat[i, j]:
                    Lm[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb] = F[i, j]
                elif i <= j and pat[i, j]:
                    Um[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb] = F[i, j]
            Lm[i * nb:(i + 1) * nb, i * nb:(i + 1) * nb] = np.eye(nb)
        LU = Lm @ Um
        Ad = A.transpose(0, 2, 1, 3).reshape(n * nb, n * nb)
        for i in range(n):
            for j in range(n):
                if pat[i, j]:
                    blk = (slice(i * nb, (i + 1) * nb), slice(j * nb, (j + 1) * nb))
                    assert np.abs(LU[blk] - Ad[blk]).max() <= 1e-11 * np.abs(Ad).max()
        # the apply solves with exactly these factors
        r = np.random.default_rng(G).standard_normal((n, nb))
        x = ilu_asm.lu_solve(F, pat, r)
        assert np.abs(LU @ x.ravel() - r.ravel()).max() <= 1e-10 * np.abs(r).max()


def test_fgmres_with_ilu_asm_reaches_the_direct_solution():
    pb, out = _c1()
    d = pb.dims()
    nb = d["ncomp"] * d["npf"]
    subs = ilu_asm.setup(out["K"], out["nbr"], pb.mesh.e2f, 4)
    x, info = krylov.fgmres(lambda v: out["A"] @ v, out["r"], prec=lambda v: ilu_asm.apply(subs, v, nb),
                            restart=50, rtol=1e-12, max_iters=500)
    assert info["converged"]
    assert np.abs(x - out["x"]).max() <= 1e-9 * np.abs(out["x"]).max()


def test_ilu0_without_fill_is_the_exact_factorisation():
    """On a block-tridiagonal pattern elimination creates no fill outside the pattern, so ILU(0)
    is the exact block LU and its solve equals a dense solve (an ordering or pattern mistake in
    the update would leave a residual)."""
    rng = np.random.default_rng(21)
    n, nb = 9, 3
    pat = np.zeros((n, n), dtype=bool)
    for i in range(n):
        pat[i, max(0, i - 1):min(n, i + 2)] = True
    A = np.where(pat[:, :, None, None], rng.standard_normal((n, n, nb, nb)), 0.0)
    for i in range(n):
        A[i, i] += 6.0 * np.eye(nb)
    F = ilu_asm.block_ilu0(A, pat)
    r = rng.standard_normal((n, nb))
    x = ilu_asm.lu_solve(F, pat, r)
    Ad = A.transpose(0, 2, 1, 3).reshape(n * nb, n * nb)
    ref = np.linalg.solve(Ad, r.ravel())
    assert np.abs(x.ravel() - ref).max() <= 1e-12 * np.abs(ref).max()
    # an arrow pattern (first block row and column full) does fill in: ILU(0) is then inexact
    arrow = pat.copy()
    arrow[0, :] = arrow[:, 0] = True
    A2 = np.where(arrow[:, :, None, None], rng.standard_normal((n, n, nb, nb)), 0.0)
    for i in range(n):
        A2[i, i] += 6.0 * np.eye(nb)
    F2 = ilu_asm.block_ilu0(A2, arrow)
    x2 = ilu_asm.lu_solve(F2, arrow, r)
    ref2 = np.linalg.solve(A2.transpose(0, 2, 1, 3).reshape(n * nb, n * nb), r.ravel())
    assert np.abs(x2.ravel() - ref2).max() > 1e-8 * np.abs(ref2).max()
    # ... yet L U matches A2 on every pattern block (fill is dropped, never propagated)
    for i in range(n):
        for j in range(n):
            if arrow[i, j]:
                lu = sum(F2[i, k] @ F2[k, j] for k in range(min(i, j + 1)) if arrow[i, k] and arrow[k, j])
                lu = lu + (F2[i, j] if i <= j else 0.0)
                assert np.abs(lu - A2[i, j]).max() <= 1e-11 * np.abs(A2).max(), (i, j)
