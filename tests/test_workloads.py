"""Checks of the seeded input generator: face frames, normals, Jacobians."""
import numpy as np
import pytest
import torch

from workloads import configs
from workloads import mesh as Mh
from workloads import physics as Ph
from workloads.blocks import HDGProblem


@pytest.mark.parametrize("etype", ["quad", "hex", "tri", "tet"])
def test_shared_faces_see_same_points_and_opposite_normals(etype):
    mk = {"quad": Mh.structured_quads, "hex": Mh.structured_hexes, "tri": Mh.structured_tris,
          "tet": Mh.kuhn_tets}[etype]
    m = mk(3 if etype != "tet" else 2, 0.1, 9)
    pb = HDGProblem(m, 2, Ph.Poisson(m.dim, 1.0))
    g = pb.geometry(0, m.ne)
    xf, ndA = g["xf"].numpy(), g["ndA"].numpy()
    for f in range(m.nf):
        e1, l1, e2, l2 = m.f2e[f]
        if e2 < 0:
            continue
        assert np.abs(xf[e1, l1] - xf[e2, l2]).max() < 1e-13
        assert np.abs(ndA[e1, l1] + ndA[e2, l2]).max() < 1e-13
    # outward normals integrate to zero over each closed element boundary
    assert np.abs(ndA.sum(axis=(1, 2))).max() < 1e-13
    assert (g["det"].numpy() > 0).all()


def test_face_counts():
    assert Mh.structured_hexes(4).nf == 3 * 4 * 4 * 5
    assert Mh.structured_quads(8).nf == 144
    m = Mh.kuhn_tets(2)
    assert m.ne == 48 and int(m.boundary.sum()) == 2 * 2 * 2 * 6


def test_ns_flux_jacobians_match_central_differences():
    ph = configs.navier_stokes(3, 0.1)
    rng = np.random.default_rng(0)
    x = torch.as_tensor(rng.random((6, 3)))
    u = ph.state(x)
    q = torch.as_tensor(rng.standard_normal((6, 5, 3)) * 0.1)
    F, Fu, Fq = ph.flux_jacobians(u, q)
    h = 1e-6
    for b in range(5):
        du = torch.zeros_like(u)
        du[:, b] = h
        fd = (ph.flux(u + du, q) - ph.flux(u - du, q)) / (2 * h)
        assert torch.allclose(Fu[..., b], fd, rtol=1e-6, atol=1e-8)
        for d in range(3):
            dq = torch.zeros_like(q)
            dq[:, b, d] = h
            fd = (ph.flux(u, q + dq) - ph.flux(u, q - dq)) / (2 * h)
            assert torch.allclose(Fq[..., b, d], fd, rtol=1e-6, atol=1e-8)


def test_elasticity_jacobian_matches_autodiff():
    ph = Ph.Elasticity()
    u = torch.zeros(4, 3, dtype=torch.float64)
    q = torch.as_tensor(np.random.default_rng(1).standard_normal((4, 3, 3)))
    F, Fu, Fq = ph.flux_jacobians(u, q)
    F2, Fu2, Fq2 = Ph.Physics.flux_jacobians(ph, u, q)
    assert torch.allclose(Fq, Fq2, atol=1e-14)
    assert torch.allclose(F, F2, atol=1e-14)


def test_generator_is_deterministic_and_chunk_independent():
    pb = configs.c1(n=4)
    a = pb.element_blocks(0, 16)
    b = pb.element_blocks(4, 9)
    c = pb.element_blocks(0, 16)
    for k in a:
        assert torch.equal(a[k], c[k])
        # batched BLAS may round differently for another chunking: equal to rounding
        assert torch.allclose(a[k][4:9], b[k], rtol=1e-12, atol=1e-14 * a[k].abs().max().item())
