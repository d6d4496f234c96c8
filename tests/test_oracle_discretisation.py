"""Pins of the input generator + oracle discretisation chain against mathematics.

Quadrature exactness, basis identities, exact reproduction of polynomial
solutions (patch test), brute-force uncondensed solves equal to condensation
plus recovery (eq. 13-a..13-c), SPD of the condensed interior operator,
null spaces of single-element Schur complements (Section 4.2: Kbar^e alone is
not invertible) and O(h^{p+1}) convergence.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle
from workloads import basis as B
from workloads import configs
from workloads import mesh as Mh
from workloads import physics as Ph
from workloads import quadrature as Q
from workloads.blocks import HDGProblem

from helpers import blocks_np, l2_error, nodal_points, oracle_pipeline


@pytest.mark.parametrize("etype,n", [("quad", 3), ("hex", 3), ("tri", 4), ("tet", 4)])
def test_quadrature_exact_on_monomials(etype, n):
    pts, w = Q.cell_rule(etype, n)
    dim = pts.shape[1]
    import itertools
    for e in itertools.product(range(2 * n), repeat=dim):
        if etype in ("quad", "hex"):
            if max(e) > 2 * n - 1:
                continue
            exact = np.prod([1.0 / (k + 1) for k in e])
        else:
            if sum(e) > 2 * n - 2:
                continue
            # int over unit simplex of x^a y^b (z^c) = a! b! c! / (a+b+c+dim)!
            exact = np.prod([math.factorial(k) for k in e]) / math.factorial(sum(e) + dim)
        val = np.sum(w * np.prod(pts ** np.array(e), axis=1))
        assert abs(val - exact) < 1e-14 * max(1.0, abs(exact)) + 1e-15


@pytest.mark.parametrize("etype,p", [("quad", 1), ("quad", 3), ("hex", 2), ("tri", 2), ("tet", 2)])
def test_basis_partition_of_unity_and_nodality(etype, p):
    dim = Mh.DIM[etype]
    pts = np.random.default_rng(0).random((20, dim)) * (0.5 if etype in ("tri", "tet") else 1.0)
    phi, dphi = B.cell_basis(etype, p, pts)
    assert np.allclose(phi.sum(1), 1.0, atol=1e-13)
    assert np.allclose(dphi.sum(1), 0.0, atol=1e-11)
    nodes = B.tensor_nodes(p, dim) if etype in ("quad", "hex") else B.simplex_nodes(p, dim)
    phin, _ = B.cell_basis(etype, p, nodes)
    assert np.allclose(phin, np.eye(len(nodes)), atol=1e-12)


def _poly2(x):
    return (1 + x[..., 0] - 2 * x[..., 1] + 0.5 * x[..., 0] ** 2 + x[..., 0] * x[..., 1]
            - 0.3 * x[..., 1] ** 2)[..., None]


def _poly3(x):
    return (_poly2(x)[..., 0] + 0.2 * x[..., 0] ** 3 - 0.4 * x[..., 0] * x[..., 1] ** 2)[..., None]


@pytest.mark.parametrize("etype,p,ex", [("quad", 2, _poly2), ("quad", 3, _poly3), ("tri", 2, _poly2),
                                        ("tri", 3, _poly3)])
def test_patch_poisson_reproduces_polynomials(etype, p, ex):
    m = Mh.structured_quads(3, 0.1, 7) if etype == "quad" else Mh.structured_tris(3, 0.1, 7)
    pb = HDGProblem(m, p, Ph.Poisson(2, 1.0, exact=ex))
    out = oracle_pipeline(pb)
    uex = ex(torch.as_tensor(nodal_points(pb))).numpy()[..., 0]
    assert np.abs(out["du"] - uex).max() < 1e-11
    # q = grad u at the nodes
    xs = torch.as_tensor(nodal_points(pb)).reshape(-1, 2).requires_grad_(True)
    g = torch.autograd.grad(ex(xs).sum(), xs)[0].detach().numpy().reshape(pb.mesh.ne, -1, 2)
    dq = out["dq"].reshape(pb.mesh.ne, 1, 2, pb.npe)
    assert np.abs(dq[:, 0].transpose(0, 2, 1) - g).max() < 1e-10


def _rigid_linear(x):
    return torch.stack([0.1 + x[..., 0] + 0.3 * x[..., 1] - 0.2 * x[..., 2],
                        -0.2 + 0.5 * x[..., 0] * 1.0 + x[..., 2],
                        0.3 - x[..., 1] + 0.25 * x[..., 2] + x[..., 0] * x[..., 1]], dim=-1)


def test_patch_elasticity_hex():
    m = Mh.structured_hexes(2, 0.1, 11)
    pb = HDGProblem(m, 2, Ph.Elasticity(1.0, 0.3, 1.0, exact=_rigid_linear))
    out = oracle_pipeline(pb)
    uex = _rigid_linear(torch.as_tensor(nodal_points(pb))).numpy()     # (E, P, 3)
    du = out["du"].reshape(pb.mesh.ne, 3, pb.npe).transpose(0, 2, 1)
    assert np.abs(du - uex).max() < 1e-11


def test_patch_poisson_tet():
    m = Mh.kuhn_tets(2, 0.1, 5)
    ex = lambda x: (1 + x[..., 0] - x[..., 1] * x[..., 2] + 0.5 * x[..., 2] ** 2)[..., None]
    pb = HDGProblem(m, 2, Ph.Poisson(3, 1.0, exact=ex))
    out = oracle_pipeline(pb)
    uex = ex(torch.as_tensor(nodal_points(pb))).numpy()[..., 0]
    assert np.abs(out["du"] - uex).max() < 1e-11


@pytest.mark.parametrize("case", ["poisson_quad_p1", "poisson_quad_p3", "elast_hex_p1", "burgers_tri_p2",
                                  "ns_hex_p1", "ns_tet_p1"])
def test_brute_force_uncondensed_equals_condensed(case):
    if case == "poisson_quad_p1":
        pb = HDGProblem(Mh.structured_quads(2, 0.1, 3), 1, Ph.Poisson(2, 1.0, exact=configs.poisson_sin))
    elif case == "poisson_quad_p3":
        pb = HDGProblem(Mh.structured_quads(3, 0.1, 3), 3, Ph.Poisson(2, 1.0, exact=configs.poisson_sin))
    elif case == "elast_hex_p1":
        pb = HDGProblem(Mh.structured_hexes(2, 0.1, 3), 1, Ph.Elasticity(exact=Ph.elasticity_manufactured))
    elif case == "burgers_tri_p2":
        pb = HDGProblem(Mh.structured_tris(2, 0.1, 3), 2, Ph.Burgers(nu=0.01))
    elif case == "ns_hex_p1":
        pb = HDGProblem(Mh.structured_hexes(1, 0.0, 3), 1, configs.navier_stokes(3, 0.1))
    else:
        pb = HDGProblem(Mh.kuhn_tets(1, 0.0, 5), 1, configs.navier_stokes(5, 0.1))
    out = oracle_pipeline(pb)
    Aun, rhs, nqu = oracle.assemble.uncondensed_system(out["blk"], pb.mesh.e2f, out["dims"])
    s = spla.spsolve(Aun, rhs)
    ne = pb.mesh.ne
    scale = max(1.0, np.abs(out["x"]).max())
    assert np.abs(s[ne * nqu:] - out["x"]).max() < 1e-12 * scale * 100
    loc = s[:ne * nqu].reshape(ne, nqu)
    nq = out["dq"].shape[1]
    assert np.abs(loc[:, nq:] - out["du"]).max() < 1e-10 * max(1.0, np.abs(out["du"]).max())
    assert np.abs(loc[:, :nq] - out["dq"]).max() < 1e-10 * max(1.0, np.abs(out["dq"]).max())


def _interior(pb, nb):
    inter = np.where(~pb.mesh.boundary)[0]
    return (inter[:, None] * nb + np.arange(nb)).ravel()


@pytest.mark.parametrize("which", ["poisson", "elasticity"])
def test_condensed_interior_operator_is_spd(which):
    if which == "poisson":
        pb = configs.c1(n=4)
    else:
        pb = configs.c2(n=2, p=1)
    out = oracle_pipeline(pb)
    idx = _interior(pb, pb.nb)
    AI = out["A"].toarray()[np.ix_(idx, idx)]
    assert np.abs(AI - AI.T).max() <= 1e-13 * np.abs(AI).max()
    np.linalg.cholesky(AI)
    assert np.linalg.eigvalsh(AI).min() > 0


def test_element_schur_null_spaces():
    # Poisson: interior element (no boundary face): Kbar^e 1 = 0
    pb = configs.c1(n=4)
    blk = blocks_np(pb)
    Kb, _ = oracle.condense.condense(blk, pb.dims())
    inner = [e for e in range(pb.mesh.ne) if not pb.mesh.boundary[pb.mesh.e2f[e]].any()]
    assert inner
    for e in inner:
        assert np.abs(Kb[e] @ np.ones(pb.nt)).max() < 1e-12 * np.abs(Kb[e]).max()
    # elasticity: the traces of the 6 rigid-body modes
    pb = configs.c2(n=3, p=1)
    blk = blocks_np(pb)
    e = 13    # the centre element of 3^3
    assert not pb.mesh.boundary[pb.mesh.e2f[e]].any()
    Kb, _ = oracle.condense.condense(blk, pb.dims(), elems=[e])
    # face nodes in physical coordinates
    from workloads.blocks import _frame_tables, _map_tables
    frames = _frame_tables("hex")
    fid = pb.fid.numpy()[e]
    X = pb.X.numpy()[e]
    pts = []
    for l in range(6):
        o, A = frames[l][fid[l]]
        xi = o[None] + pb.fnodes @ A.T
        N, _ = _map_tables("hex", xi)
        pts.append(N @ X)
    pts = np.stack(pts)                  # (L, PF, 3)
    modes = [lambda x: np.stack([np.ones(len(x)), 0 * x[:, 0], 0 * x[:, 0]], -1),
             lambda x: np.stack([0 * x[:, 0], np.ones(len(x)), 0 * x[:, 0]], -1),
             lambda x: np.stack([0 * x[:, 0], 0 * x[:, 0], np.ones(len(x))], -1),
             lambda x: np.stack([-x[:, 1], x[:, 0], 0 * x[:, 0]], -1),
             lambda x: np.stack([0 * x[:, 0], -x[:, 2], x[:, 1]], -1),
             lambda x: np.stack([x[:, 2], 0 * x[:, 0], -x[:, 0]], -1)]
    for md in modes:
        v = np.zeros(pb.nt)
        for l in range(6):
            val = md(pts[l])             # (PF, 3)
            for m in range(3):
                v[(l * 3 + m) * pb.npf:(l * 3 + m + 1) * pb.npf] = val[:, m]
        assert np.abs(Kb[0] @ v).max() < 1e-12 * np.abs(Kb[0]).max() * np.abs(v).max()


@pytest.mark.parametrize("p", [1, 2])
def test_convergence_rate_manufactured(p):
    errs = []
    for n in (4, 8, 16):
        pb = configs.c1(n=n, p=p)
        out = oracle_pipeline(pb)
        errs.append(l2_error(pb, out["du"], configs.poisson_sin))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= p + 1 - 0.3, (errs, rates)
