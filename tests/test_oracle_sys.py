"""Pins of the oracle's element residuals and Jacobian blocks for M-component models (linear
elasticity, compressible Navier-Stokes; Section 2.1, Section 2.2, Section 4.1) and of its damped
Newton iteration on them (Section 4.4), against mathematics and an independent implementation:

* the Jacobian blocks equal central differences of the residual on random states;
* the flux derivatives satisfy Euler's identity for the homogeneous convective flux and the
  linearity of the viscous flux in q, and are exact for the linear elasticity flux;
* a uniform freestream is an exact discrete steady state of Navier-Stokes (the assembled
  residual vanishes) and an affine displacement one of elasticity without load (patch test);
* at the input generator's linearisation states the blocks equal the generator's own
  (forward-mode autodiff and einsum contractions, a different route);
* Newton reaches the affine elasticity solution in one step and converges quadratically on a
  backward-Euler Navier-Stokes step.
"""
import numpy as np
import pytest
import torch

import oracle.elements_sys as OS
import oracle.newton as ON
from workloads import configs
from workloads import mesh as Mh
from workloads import physics as Ph
from workloads.blocks import HDGProblem


def _np(d):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in d.items()}


def _elast(n=2, p=1, amp=0.05):
    return HDGProblem(Mh.structured_hexes(n, amp, 2), p, Ph.Elasticity(exact=Ph.elasticity_manufactured))


CASES = {
    "elast_hex_p1": lambda: _elast(),
    "ns_hex_p1": lambda: configs.c3(n=2, p=1),
    "ns_tet_p1": lambda: configs.c5(n=1, p=1),
}


def _time_term(inp):
    m = inp["model"]
    return dict(c=1.0 / m["dt"], u_prev=inp["u0"], r_extra=None) if m["kind"] == "navier_stokes" else None


@pytest.mark.parametrize("name", list(CASES))
def test_blocks_equal_the_generators_at_its_state(name):
    pb = CASES[name]()
    inp = _np(pb.newton_inputs_sys())
    gen = _np(pb.element_blocks())
    ob = OS.element_blocks(inp, inp["model"], inp["u0"], inp["uhat0"], pb.mesh.e2f, _time_term(inp))
    for k in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J"):
        a, b = ob[k].reshape(gen[k].shape), gen[k]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max(), k
    # the residual rows are small differences of O(1) flux terms: compare against the flux scale
    for k in ("ru", "rt"):
        a, b = ob[k].reshape(gen[k].shape), gen[k]
        assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max()), k


def _random_state(pb, inp, rng, amp):
    d = pb.dims()
    M, P, PF, L, D = d["ncomp"], d["npe"], d["npf"], d["nlfe"], d["dim"]
    u = inp["u0"][0] + amp * rng.standard_normal((M, P))
    uh = inp["uhat0"][pb.mesh.e2f[0]] + amp * rng.standard_normal((L, M, PF))
    q = amp * rng.standard_normal((M, D, P))
    return q, u, uh


@pytest.mark.parametrize("name", ["elast_hex_p1", "ns_hex_p1", "ns_tet_p1"])
def test_jacobian_blocks_equal_central_differences(name):
    pb = CASES[name]()
    inp = _np(pb.newton_inputs_sys())
    m = inp["model"]
    rng = np.random.default_rng(11)
    q, u, uh = _random_state(pb, inp, rng, 0.05)
    c = 1.0 / m["dt"] if "dt" in m else 0.0
    tt = (c, u.copy(), None)
    Dm, Em, Fm, Gm, Hm, Jm = OS.jacobian(inp, m, 0, q, u, uh, c)

    def R(qq, uu, hh):
        _, Ru, Rt = OS.residual(inp, m, 0, qq, uu, hh, tt)
        return Ru.ravel(), Rt.ravel()
    # step 1e-5: truncation ~h^2 |R'| and rounding ~eps |R| / h both stay near 1e-11
    h = 1e-5
    for blocks, x, shape in (((Dm, Gm), q, q.shape), ((Em, Hm), u, u.shape), ((Fm, Jm), uh, uh.shape)):
        cols = rng.choice(x.size, size=min(x.size, 8), replace=False)
        for col in cols:
            xp, xm = x.copy().ravel(), x.copy().ravel()
            xp[col] += h
            xm[col] -= h
            args_p = [q, u, uh]
            args_m = [q, u, uh]
            idx = 0 if x is q else (1 if x is u else 2)
            args_p[idx] = xp.reshape(shape)
            args_m[idx] = xm.reshape(shape)
            rup, rtp = R(*args_p)
            rum, rtm = R(*args_m)
            for blk, diff in ((blocks[0], (rup - rum) / (2 * h)), (blocks[1], (rtp - rtm) / (2 * h))):
                scale = max(np.abs(blk).max(), 1e-30)
                assert np.abs(blk[:, col] - diff).max() <= 1e-7 * scale + 1e-9, (name, col)


def test_navier_stokes_flux_identities():
    m = dict(kind="navier_stokes", Re=1000.0, Pr=0.72, gamma=1.4, tau=3.0)
    rng = np.random.default_rng(4)
    for _ in range(5):
        rho = 1.0 + 0.2 * rng.random()
        v = rng.standard_normal(3)
        p = 2.0 + rng.random()
        u = np.array([rho, *(rho * v), p / 0.4 + 0.5 * rho * v @ v])
        q0 = np.zeros((5, 3))
        F, Fu, _ = OS.flux_and_jacobians(m, u, q0)
        # the convective flux is homogeneous of degree one in u: (dF/du) u = F
        assert np.allclose(np.einsum("axb,b->ax", Fu, u), F, rtol=1e-13, atol=1e-13)
        # pressure from the energy row of the state
        assert np.isclose(F[1, 0] - u[1] * v[0], p, rtol=1e-13)
        # the viscous flux is linear in q: (dF/dq) q = F(u, q) - F(u, 0)
        q = rng.standard_normal((5, 3))
        Fq_full, _, Fq = OS.flux_and_jacobians(m, u, q)
        assert np.allclose(np.einsum("axbd,bd->ax", Fq, q), Fq_full - F, rtol=1e-12, atol=1e-14)
    me = dict(kind="elasticity", lam=0.5769230769230769, mu=0.3846153846153846, tau=1.0)
    q = rng.standard_normal((3, 3))
    F, Fu, Fq = OS.flux_and_jacobians(me, np.zeros(3), q)
    assert np.allclose(np.einsum("axbd,bd->ax", Fq, q), F, atol=1e-14) and not Fu.any()
    # isotropic Hooke's law: the shear q_01 = 1 (strain 1/2) gives F_01 = F_10 = -mu, no normal stress
    s = np.zeros((3, 3))
    s[0, 1] = 1.0
    Fs, _, _ = OS.flux_and_jacobians(me, np.zeros(3), s)
    assert np.isclose(Fs[0, 1], -me["mu"]) and np.isclose(Fs[1, 0], -me["mu"]) and abs(Fs[0, 0]) < 1e-15


def _assembled_norm(pb, blk):
    d = pb.dims()
    return ON._norm_from_blocks(blk, pb.mesh.e2f, pb.mesh.f2e, d)


@pytest.mark.parametrize("name", ["ns_hex_p1", "ns_tet_p1"])
def test_uniform_freestream_is_a_discrete_steady_state(name):
    pb = CASES[name]()
    inp = _np(pb.newton_inputs_sys())
    ph = pb.phys
    uinf = ph.dirichlet(torch.zeros(1, 3, dtype=torch.float64)).numpy()[0]
    d = pb.dims()
    u = np.broadcast_to(uinf[None, :, None], (d["ne"], 5, d["npe"])).copy()
    uh = np.broadcast_to(uinf[None, :, None], (d["nf"], 5, d["npf"])).copy()
    blk = OS.element_blocks(inp, inp["model"], u, uh, pb.mesh.e2f, dict(c=1.0 / inp["model"]["dt"], u_prev=u))
    assert np.abs(blk["q"]).max() < 1e-12
    # flux scale: |F(u_inf)| = p_inf + rho u^2 ~ 3.9
    assert _assembled_norm(pb, blk) < 1e-12 * 4.0 * np.sqrt(d["ne"])


def _affine_problem(p=1):
    A = np.array([[0.3, -0.2, 0.1], [0.05, 0.4, -0.3], [-0.1, 0.2, 0.25]])
    b = np.array([0.1, -0.2, 0.05])

    def affine(x):
        return x @ torch.as_tensor(A.T) + torch.as_tensor(b)
    ph = Ph.Elasticity(E=1.0, nu=0.3, tau=1.0)
    ph.linear = False
    ph.state = affine
    ph.dirichlet = affine
    return HDGProblem(Mh.structured_hexes(2, 0.1, 7), p, ph), A


@pytest.mark.parametrize("p", [1, 2])
def test_affine_displacement_patch_test(p):
    pb, A = _affine_problem(p)
    inp = _np(pb.newton_inputs_sys())
    blk = OS.element_blocks(inp, inp["model"], inp["u0"], inp["uhat0"], pb.mesh.e2f)
    # q = grad u exactly, and the assembled residual vanishes
    assert np.abs(blk["q"] - A[None, :, :, None]).max() < 1e-12
    assert _assembled_norm(pb, blk) < 1e-12


def test_newton_elasticity_one_step_to_the_affine_solution():
    pb, A = _affine_problem(2)
    inp = _np(pb.newton_inputs_sys())
    d = pb.dims()
    u0 = np.zeros_like(inp["u0"])
    uh0 = np.zeros_like(inp["uhat0"])
    u, uh, hist = ON.damped_newton(inp, inp["model"], u0, uh0, pb.mesh.e2f, pb.mesh.f2e, d, rtol=1e-12)
    assert len(hist) == 2 and hist[0]["alpha"] == 1.0 and hist[1]["norm"] < 1e-11 * hist[0]["norm"]
    assert np.abs(u - inp["u0"]).max() < 1e-11 and np.abs(uh - inp["uhat0"]).max() < 1e-11


def test_newton_navier_stokes_backward_euler_step_converges_quadratically():
    pb = configs.c3(n=2, p=1)
    inp = _np(pb.newton_inputs_sys())
    d = pb.dims()
    m = inp["model"]
    # a larger step than the workload's so that the first residual is far from zero
    c = 0.2 / m["dt"]
    tt = dict(c=c, u_prev=inp["u0"], r_extra=None)
    rng = np.random.default_rng(2)
    u0 = inp["u0"] + 0.02 * rng.standard_normal(inp["u0"].shape)
    u, uh, hist = ON.damped_newton(inp, m, u0, inp["uhat0"], pb.mesh.e2f, pb.mesh.f2e, d, rtol=1e-12, tt=tt)
    norms = [h["norm"] for h in hist]
    assert norms[-1] < 1e-12 * norms[0] and len(norms) <= 7
    # quadratic: the error ratio of the last full steps falls faster than linearly
    r = [norms[k + 1] / norms[k] for k in range(len(norms) - 1)]
    assert r[-1] < 0.1 * r[0] or norms[-1] < 1e-14
