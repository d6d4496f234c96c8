"""Host-side checks of the C ABI library (no GPU needed): it loads, exports every
symbol include/hdg.h declares, and its host-only spectral helpers agree with
LAPACK / the oracle's harmonic Ritz values."""
import os
import re

import numpy as np
import pytest

import oracle
from oracle import poly

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2512_13619_amd", "libhdg.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhdg.so not built (run __graft_entry__.build())")


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "hdg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hdg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2512_13619_amd import hdg
    lib = hdg.load()
    decl = _declared_symbols()
    assert len(decl) >= 18
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(hdg.SYMBOLS)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (5, 2), (12, 3), (30, 4), (64, 5)])
def test_hessenberg_eigvals_match_lapack(n, seed):
    from paper_2512_13619_amd import hdg
    rng = np.random.default_rng(seed)
    H = np.triu(rng.standard_normal((n, n)), -1)
    got = np.sort_complex(hdg.hessenberg_eigvals(H))
    ref = np.sort_complex(np.linalg.eigvals(H))
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-10 * np.abs(ref).max())


def test_hessenberg_eigvals_special_matrices():
    from paper_2512_13619_amd import hdg
    # already triangular, repeated eigenvalues, a rotation (pure imaginary pair)
    T = np.triu(np.arange(1.0, 17.0).reshape(4, 4))
    assert np.allclose(np.sort(hdg.hessenberg_eigvals(T).real), [1, 6, 11, 16])
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    assert np.allclose(np.sort_complex(hdg.hessenberg_eigvals(R)), [-1j, 1j])
    Z = np.zeros((3, 3))
    assert np.allclose(hdg.hessenberg_eigvals(Z), 0)


@pytest.mark.parametrize("P,seed", [(5, 0), (10, 1), (20, 2)])
def test_harmonic_ritz_matches_oracle(P, seed):
    from paper_2512_13619_amd import hdg
    rng = np.random.default_rng(seed)
    N = 80
    Bm = rng.standard_normal((N, N)) * 0.15 + np.diag(np.linspace(0.5, 4, N))
    H, _ = poly.arnoldi_mgs(lambda v: Bm @ v, rng.standard_normal(N), P)
    got = hdg.harmonic_ritz(H)
    ref = poly.leja_order(poly.harmonic_ritz(H))
    assert len(got) == len(ref)
    assert np.allclose(np.sort_complex(got), np.sort_complex(ref), rtol=1e-8, atol=1e-10)
    assert abs(got[0]) == pytest.approx(np.abs(ref).max(), rel=1e-10)
    for k, t in enumerate(got):
        if t.imag > 0:
            assert got[k + 1] == np.conj(t)
    # the Leja product property: each value maximises the distance product to the previous ones
    for k in range(1, len(got)):
        if got[k - 1].imag > 0 and got[k] == np.conj(got[k - 1]):
            continue
        score = lambda z: sum(np.log(abs(z - s)) for s in got[:k])
        rest = [z for z in got[k:] if z.imag >= 0]
        assert score(got[k]) >= max(score(z) for z in rest) - 1e-9


@pytest.mark.parametrize("spectrum,seed", [("geometric", 0), ("geometric", 1), ("geometric", 7), ("random", 3)])
def test_poly_roots_match_oracle(spectrum, seed):
    """The roots the solver's polynomial preconditioner uses (harmonic Ritz values, the added
    copies of the outermost one, Leja order) against the oracle's, value by value in order, on
    Arnoldi cycles whose Ritz values stop short of the spectrum (geometric on [0.01, 3.1]: copies
    are added) and on a nonsymmetric matrix."""
    from paper_2512_13619_amd import hdg
    rng = np.random.default_rng(seed)
    N = 300
    if spectrum == "geometric":
        lam = np.geomspace(0.01, 3.1, N)
        op = lambda v: lam * v
    else:
        Bm = rng.standard_normal((N, N)) * 0.1 + np.diag(np.linspace(0.5, 4, N))
        op = lambda v: Bm @ v
    H, _ = poly.arnoldi_mgs(op, rng.standard_normal(N), 10)
    got, n_added = hdg.poly_roots(H)
    ref, ref_added = poly.pp_roots(H)
    assert n_added == ref_added and len(got) == len(ref)
    if spectrum == "geometric":
        assert n_added > 0
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-9 * scale, (got, ref)


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    from paper_2512_13619_amd import hdg
    with pytest.raises(hdg.HdgError):
        hdg._ptr(torch.zeros(4, dtype=torch.float64), torch.float64, 4, "x")


def test_package_dirk_tableaus_meet_order_conditions():
    """The DIRK tableaus the device driver uses (written out in the package) are lower triangular
    with one diagonal value, stiffly accurate, and of order 1, 2, 3 (Section 2.2's DIRK(s, p))."""
    import numpy as np
    from paper_2512_13619_amd.pipeline import dirk_tableau
    for scheme, order in (("be", 1), ("dirk22", 2), ("dirk33", 3)):
        A = np.array(dirk_tableau(scheme))
        b, c = A[-1], A.sum(1)
        assert np.allclose(np.tril(A), A) and np.allclose(np.diag(A), A[0, 0])
        assert abs(c[-1] - 1.0) < 1e-15 and abs(b.sum() - 1.0) < 1e-15
        if order >= 2:
            assert abs(b @ c - 0.5) < 1e-14
        if order >= 3:
            assert abs(b @ c ** 2 - 1.0 / 3.0) < 1e-14 and abs(b @ (A @ c) - 1.0 / 6.0) < 1e-14
