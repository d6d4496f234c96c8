"""Pins of the oracle's element residual/Jacobian generation and damped Newton iteration
(Section 4.1, Section 4.4) against mathematics and an independent implementation:

* the Jacobian blocks equal central differences of the residual (exact up to rounding: the
  residual is at most quadratic in the state), including A = I (x) M, B_d and C_d from R_q;
* the consistent q makes R_q vanish;
* at the input generator's linearisation state the blocks equal the generator's own
  (an independent einsum implementation of the same weak form);
* Newton on a linear problem converges in one full step, on Burgers quadratically;
* the DIRK tableaus meet their order conditions, the stage time term's derivative is c M, and
  DIRK steps of the heat equation converge in time at orders 1, 2, 3.
"""
import numpy as np
import pytest

import oracle.dirk as ODK
import oracle.elements as OE
import oracle.newton as ON
from workloads import mesh as Mh
from workloads import physics as Ph
from workloads.blocks import HDGProblem

from helpers import blocks_np


def _np(d):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in d.items()}


def _model(inp):
    return dict(nu=inp["nu"], tau=inp["tau"], beta=inp["beta"], gamma=inp["gamma"])


def _burgers_forcing(x):
    import torch
    return (torch.sin(np.pi * x[..., 0]) * torch.sin(2 * np.pi * x[..., 1]))[..., None]


CASES = {
    "burgers_tri_p3": lambda: HDGProblem(Mh.structured_tris(2, 0.0, 4), 3, Ph.Burgers(nu=0.05)),
    "burgers_quad_p2": lambda: HDGProblem(Mh.structured_quads(3, 0.1, 4), 2,
                                          Ph.Burgers(nu=0.01, forcing=_burgers_forcing)),
    "poisson_quad_p2": lambda: HDGProblem(Mh.structured_quads(3, 0.1, 5), 2, Ph.Poisson(2, 1.0, forcing=_burgers_forcing)),
}


@pytest.mark.parametrize("name", ["burgers_tri_p3", "burgers_quad_p2"])
def test_jacobian_blocks_equal_central_differences(name):
    pb = CASES[name]()
    inp = _np(pb.newton_inputs())
    m = _model(inp)
    rng = np.random.default_rng(3)
    d = pb.dims()
    P, PF, L, D = d["npe"], d["npf"], d["nlfe"], d["dim"]
    eps = 1e-3
    for e in (0, d["ne"] - 1):
        q = rng.standard_normal((D, P))
        u = rng.standard_normal(P)
        uh = rng.standard_normal((L, PF))
        Mm, Bd, Cd = OE.mass_and_q_operators(inp, e)
        Dm, Em, Fm, Gm, Hm, Jm = OE.jacobian(inp, m, e, q, u, uh)

        def fd(var, idx):
            xs = [q.copy(), u.copy(), uh.copy()]
            xp = [a.copy() for a in xs]
            xm = [a.copy() for a in xs]
            xp[var].flat[idx] += eps
            xm[var].flat[idx] -= eps
            rp = OE.residual(inp, m, e, *xp)
            rm = OE.residual(inp, m, e, *xm)
            return [(a - b).ravel() / (2 * eps) for a, b in zip(rp, rm)]

        cols = [[fd(v, k) for k in range(n)] for v, n in ((0, D * P), (1, P), (2, L * PF))]
        jac = {v: [np.column_stack([c[r] for c in cols[v]]) for r in range(3)] for v in range(3)}
        A = np.kron(np.eye(D), Mm)
        Bm = np.vstack([Bd[k] for k in range(D)])
        Cm = np.vstack([Cd[k] for k in range(D)])
        scale = max(np.abs(Em).max(), 1.0)
        for got, want in ((jac[0][0], A), (jac[1][0], Bm), (jac[2][0], Cm), (jac[0][1], Dm), (jac[1][1], Em),
                          (jac[2][1], Fm), (jac[0][2], Gm), (jac[1][2], Hm), (jac[2][2], Jm)):
            assert np.abs(got - want).max() < 1e-9 * scale


@pytest.mark.parametrize("name", ["burgers_tri_p3", "poisson_quad_p2"])
def test_consistent_q_zeroes_q_residual(name):
    pb = CASES[name]()
    inp = _np(pb.newton_inputs())
    rng = np.random.default_rng(5)
    d = pb.dims()
    u = rng.standard_normal(d["npe"])
    uh = rng.standard_normal((d["nlfe"], d["npf"]))
    q = OE.consistent_q(inp, 1, u, uh)
    Rq, _, _ = OE.residual(inp, _model(inp), 1, q, u, uh)
    assert np.abs(Rq).max() < 1e-12 * max(np.abs(q).max(), 1.0)


@pytest.mark.parametrize("name", ["burgers_tri_p3", "burgers_quad_p2", "poisson_quad_p2"])
def test_blocks_equal_generator_at_its_state(name):
    pb = CASES[name]()
    inp = _np(pb.newton_inputs())
    got = OE.element_blocks(inp, _model(inp), inp["u0"], inp["uhat0"], pb.mesh.e2f)
    want = blocks_np(pb)
    for k in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt"):
        scale = max(np.abs(want[k]).max(), 1e-300)
        assert np.abs(got[k].reshape(want[k].shape) - want[k]).max() < 1e-11 * max(scale, 1.0), k


def test_newton_linear_problem_one_step():
    pb = CASES["poisson_quad_p2"]()
    inp = _np(pb.newton_inputs())
    d = pb.dims()
    _, _, hist = ON.damped_newton(inp, _model(inp), inp["u0"], inp["uhat0"], pb.mesh.e2f, pb.mesh.f2e, d,
                                  rtol=1e-11)
    assert hist[0]["alpha"] == 1.0
    assert hist[1]["norm"] < 1e-11 * hist[0]["norm"]
    assert len(hist) == 2


def test_newton_burgers_converges_quadratically():
    pb = CASES["burgers_quad_p2"]()
    inp = _np(pb.newton_inputs())
    d = pb.dims()
    u, uh, hist = ON.damped_newton(inp, _model(inp), inp["u0"], inp["uhat0"], pb.mesh.e2f, pb.mesh.f2e, d,
                                   rtol=1e-12)
    n = [h["norm"] for h in hist]
    assert n[-1] <= 1e-12 * n[0]
    assert len(n) <= 8
    # the last full steps square the residual (up to a modest constant)
    k = max(i for i in range(1, len(n) - 1) if n[i] > 1e-9 * n[0]) if len(n) > 2 else 1
    assert n[k + 1] <= 10 * n[k] ** 2 / n[0] + 1e-13 * n[0]
    # the converged state solves the discrete equations: every element residual vanishes
    blk = OE.element_blocks(inp, _model(inp), u, uh, pb.mesh.e2f)
    assert np.abs(blk["ru"]).max() <= 1e-11 * n[0]


# ---- implicit stages and DIRK time stepping (Section 2.2) ---------------------------------
@pytest.mark.parametrize("scheme,order", [("be", 1), ("dirk22", 2), ("dirk33", 3)])
def test_dirk_tableau_order_conditions(scheme, order):
    A, b, c = ODK.tableau(scheme)
    assert np.allclose(np.tril(A), A) and np.allclose(np.diag(A), A[0, 0])
    assert np.allclose(b, A[-1]) and abs(c[-1] - 1.0) < 1e-15          # stiffly accurate
    assert abs(b.sum() - 1.0) < 1e-14
    if order >= 2:
        assert abs(b @ c - 0.5) < 1e-14
    if order >= 3:
        assert abs(b @ c ** 2 - 1.0 / 3.0) < 1e-14
        assert abs(b @ (A @ c) - 1.0 / 6.0) < 1e-14


def test_time_term_derivatives_equal_central_differences():
    pb = CASES["burgers_tri_p3"]()
    inp = _np(pb.newton_inputs())
    m = _model(inp)
    rng = np.random.default_rng(9)
    d = pb.dims()
    P, PF, L, D = d["npe"], d["npf"], d["nlfe"], d["dim"]
    e, c = 2, 3.7
    q, u, uh = rng.standard_normal((D, P)), rng.standard_normal(P), rng.standard_normal((L, PF))
    un, rx = rng.standard_normal(P), rng.standard_normal(P)
    _, Em, *_ = OE.jacobian(inp, m, e, q, u, uh, c)
    eps = 1e-3
    cols = []
    for k in range(P):
        up, um = u.copy(), u.copy()
        up[k] += eps
        um[k] -= eps
        cols.append((OE.residual(inp, m, e, q, up, uh, (c, un, rx))[1] -
                     OE.residual(inp, m, e, q, um, uh, (c, un, rx))[1]) / (2 * eps))
    assert np.abs(np.column_stack(cols) - Em).max() < 1e-9 * np.abs(Em).max()
    # the time term itself: c M (u - u_n) + r_x
    Mm, _, _ = OE.mass_and_q_operators(inp, e)
    r1 = OE.residual(inp, m, e, q, u, uh, (c, un, rx))[1] - OE.residual(inp, m, e, q, u, uh)[1]
    assert np.abs(r1 - (c * Mm @ (u - un) + rx)).max() < 1e-12 * np.abs(r1).max()


def test_dirk_temporal_convergence_orders():
    """Heat equation (Poisson flux, zero data) from sin(pi x) sin(pi y): the error at T against a
    fine DIRK(3,3) reference falls by 2^p per halving of dt (p = 1, 2, 3)."""
    from helpers import nodal_points
    pb = HDGProblem(Mh.structured_tris(2, 0.0, 7), 2, Ph.Poisson(2, 1.0))
    inp = _np(pb.newton_inputs())
    m = _model(inp)
    d = pb.dims()
    xn = nodal_points(pb)
    u0 = np.sin(np.pi * xn[..., 0]) * np.sin(np.pi * xn[..., 1])
    uh0 = np.zeros_like(inp["uhat0"])
    T = 0.1
    args = (inp, m, u0, uh0, pb.mesh.e2f, pb.mesh.f2e, d)
    ref, _, _ = ODK.dirk_steps(*args, T / 64, 64, "dirk33")
    for scheme, p, ns in (("be", 1, (4, 8, 16)), ("dirk22", 2, (4, 8, 16)), ("dirk33", 3, (4, 8))):
        err = [np.abs(ODK.dirk_steps(*args, T / n, n, scheme)[0] - ref).max() for n in ns]
        rates = [np.log2(err[k] / err[k + 1]) for k in range(len(err) - 1)]
        assert all(abs(r - p) < 0.35 for r in rates), (scheme, err, rates)


def test_pseudo_transient_reaches_the_newton_solution():
    """Pseudo-transient continuation converges to the same discrete solution as damped Newton
    (the steady equations have one solution near the start), its first step with dtau -> inf is
    a Newton step, and on a linear problem it converges once dtau has grown."""
    pb = CASES["burgers_quad_p2"]()
    inp = _np(pb.newton_inputs())
    m = _model(inp)
    d = pb.dims()
    args = (inp, m, inp["u0"], inp["uhat0"], pb.mesh.e2f, pb.mesh.f2e, d)
    u_n, uh_n, _ = ON.damped_newton(*args, rtol=1e-12)
    u_p, uh_p, hist = ON.pseudo_transient(*args, 0.05, rtol=1e-12)
    assert hist[-1]["norm"] <= 1e-12 * hist[0]["norm"]
    assert np.abs(u_p - u_n).max() < 1e-9 * np.abs(u_n).max()
    assert np.abs(uh_p - uh_n).max() < 1e-9 * np.abs(uh_n).max()
    # dtau -> inf: one pseudo-step is the undamped Newton step
    u1, uh1, h1 = ON.pseudo_transient(*args, 1e300, max_steps=1)
    un1, uhn1, hn1 = ON.damped_newton(*args, max_steps=1, min_alpha=1.0)
    assert np.abs(u1 - un1).max() < 1e-12 * np.abs(un1).max()
    # linear problem
    pb2 = CASES["poisson_quad_p2"]()
    inp2 = _np(pb2.newton_inputs())
    _, _, h2 = ON.pseudo_transient(inp2, _model(inp2), inp2["u0"], inp2["uhat0"], pb2.mesh.e2f, pb2.mesh.f2e,
                                   pb2.dims(), 0.01, rtol=1e-11)
    assert h2[-1]["norm"] <= 1e-11 * h2[0]["norm"] and len(h2) < 30
