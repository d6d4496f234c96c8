"""Device element residuals and Jacobian blocks of the M-component models (linear elasticity,
compressible Navier-Stokes) and the damped Newton loop on them, against the oracle
(Section 2.1, Section 2.2, Section 4.1, Section 4.4): hdg_element_blocks_sys, Pipeline.newton."""
import numpy as np
import pytest
import torch

import oracle.elements_sys as OS
import oracle.newton as ON
from workloads import configs
from workloads import mesh as Mh
from workloads import physics as Ph
from workloads.blocks import HDGProblem

from test_gpu_parity import relerr, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2512_13619_amd import hdg
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return hdg.Context(0)


def _elast(n, p, amp=0.05):
    return HDGProblem(Mh.structured_hexes(n, amp, 2), p, Ph.Elasticity(exact=Ph.elasticity_manufactured))


CASES = {
    "elast_hex_p1": lambda: _elast(2, 1),
    "elast_hex_p3": lambda: _elast(2, 3),
    "ns_hex_p1": lambda: configs.c3(n=2, p=1),
    "ns_hex_p2": lambda: configs.c3(n=2, p=2),
    "ns_tet_p2": lambda: configs.c5(n=1, p=2),
}
_cache = {}


def case(name):
    if name not in _cache:
        pb = CASES[name]()
        inp = pb.newton_inputs_sys()
        _cache[name] = (pb, inp, {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in inp.items()})
    return _cache[name]


def geom_dev(inp):
    g = {k: inp[k].cuda().contiguous() for k in ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD",
                                                  "bnd")}
    g["nqv"], g["nqf"] = inp["nqv"], inp["nqf"]
    return g


def time_term_np(inp_np, u_prev):
    m = inp_np["model"]
    return dict(c=1.0 / m["dt"], u_prev=u_prev, r_extra=None) if m["kind"] == "navier_stokes" else None


def random_state(inp_np, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    u = inp_np["u0"] + amp * rng.standard_normal(inp_np["u0"].shape)
    uh = inp_np["uhat0"] + amp * rng.standard_normal(inp_np["uhat0"].shape)
    return u, uh


def compare(out, ref, tag):
    for k in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "q"):
        got = out[k].cpu().numpy().reshape(ref[k].shape)
        err = relerr(got, ref[k])
        assert err < 1e-12, (tag, k, err)
    for k in ("ru", "rt"):
        got = out[k].cpu().numpy().reshape(ref[k].shape)
        err = np.abs(got - ref[k]).max() / max(1.0, np.abs(ref[k]).max())
        assert err < 1e-12, (tag, k, err)


@pytest.mark.parametrize("name", list(CASES))
def test_element_blocks_sys_match_oracle(ctx, name):
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case(name)
    d = pb.dims()
    say("element blocks sys", name, d)
    u, uh = random_state(inp_np, 1)
    up = inp_np["u0"]
    ref = OS.element_blocks(inp_np, inp_np["model"], u, uh, pb.mesh.e2f, time_term_np(inp_np, up))
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    out = pl.element_arrays()
    tt = None
    if inp_np["model"]["kind"] == "navier_stokes":
        tt = dict(c=1.0 / inp_np["model"]["dt"], u_prev=torch.as_tensor(up).cuda().flatten())
    pl.element_blocks(geom_dev(inp), inp_np["model"], torch.as_tensor(u).cuda().flatten(),
                      torch.as_tensor(uh).cuda().flatten(), out, time_term=tt)
    torch.cuda.synchronize()
    compare(out, ref, name)


@pytest.mark.parametrize("name", ["ns_hex_p1", "elast_hex_p1"])
def test_residual_only_and_kept_mass(ctx, name):
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case(name)
    d = pb.dims()
    u, uh = random_state(inp_np, 2)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    full = pl.element_arrays()
    ud, uhd = torch.as_tensor(u).cuda().flatten(), torch.as_tensor(uh).cuda().flatten()
    g = geom_dev(inp)
    m = inp_np["model"]
    pl.element_blocks(g, m, ud, uhd, full)
    kept = pl.element_arrays()
    for k in ("Minv", "Bd", "Cd"):
        kept[k].copy_(full[k])
    pl.element_blocks(g, m, ud, uhd, kept, keep_mass=True)
    res = {"ru": torch.full_like(full["ru"], np.nan), "rt": torch.full_like(full["rt"], np.nan),
           "Minv": full["Minv"]}
    pl.element_blocks(g, m, ud, uhd, res, residual_only=True, keep_mass=True)
    torch.cuda.synchronize()
    for k in ("D", "E", "F", "G", "H", "J", "ru", "rt"):
        assert torch.equal(kept[k], full[k]), k
    assert torch.equal(res["ru"], full["ru"]) and torch.equal(res["rt"], full["rt"])
    nrm = ctx.residual_norm(d, pl.f2e, res["ru"], res["rt"])
    ref = OS.element_blocks(inp_np, m, u, uh, pb.mesh.e2f)
    want = ON._norm_from_blocks(ref, pb.mesh.e2f, pb.mesh.f2e, d)
    assert abs(nrm - want) <= 1e-11 * want


def test_newton_navier_stokes_matches_oracle(ctx):
    """One backward-Euler step of the Navier-Stokes linearisation workload on a small mesh
    (a larger step than the workload's, and a perturbed start, so that Newton takes several
    steps): the device damped Newton against the oracle's, step by step."""
    from paper_2512_13619_amd.pipeline import Pipeline
    pb = configs.c3(n=2, p=1)
    inp = pb.newton_inputs_sys()
    inp_np = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in inp.items()}
    d = pb.dims()
    m = inp_np["model"]
    c = 0.2 / m["dt"]
    rng = np.random.default_rng(2)
    u0 = inp_np["u0"] + 0.02 * rng.standard_normal(inp_np["u0"].shape)
    tt_np = dict(c=c, u_prev=inp_np["u0"], r_extra=None)
    uo, uho, hist_o = ON.damped_newton(inp_np, m, u0, inp_np["uhat0"], pb.mesh.e2f, pb.mesh.f2e, d, rtol=1e-11,
                                       tt=tt_np)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    u = torch.as_tensor(u0).cuda().flatten().contiguous()
    uh = torch.as_tensor(inp_np["uhat0"]).cuda().flatten().contiguous()
    tt = dict(c=c, u_prev=torch.as_tensor(inp_np["u0"]).cuda().flatten())
    hist = pl.newton(geom_dev(inp), m, u, uh, tol=1e-11, time_term=tt, restart=50, max_iters=5000, rtol=1e-13,
                     prec="bj", orth="cgs2")
    say("newton ns", [(h["norm"], h["alpha"]) for h in hist], [(h["norm"], h["alpha"]) for h in hist_o])
    assert len(hist) == len(hist_o)
    for a, b in zip(hist, hist_o):
        assert a["alpha"] == b["alpha"] or b["alpha"] == 0.0
        assert abs(a["norm"] - b["norm"]) <= 1e-7 * hist_o[0]["norm"] + 1e-8 * b["norm"], (a, b)
    assert relerr(u.cpu().numpy(), uo.ravel()) < 1e-9 and relerr(uh.cpu().numpy(), uho.ravel()) < 1e-9


def test_newton_elasticity_one_step(ctx):
    """Linear elasticity with the manufactured load: one full Newton step from zero reaches the
    discrete solution (the oracle's, from the same zero start)."""
    from paper_2512_13619_amd.pipeline import Pipeline
    pb = _elast(2, 2)
    inp = pb.newton_inputs_sys()
    inp_np = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in inp.items()}
    d = pb.dims()
    m = inp_np["model"]
    z_u, z_uh = np.zeros_like(inp_np["u0"]), np.zeros_like(inp_np["uhat0"])
    uo, uho, hist_o = ON.damped_newton(inp_np, m, z_u, z_uh, pb.mesh.e2f, pb.mesh.f2e, d, rtol=1e-12)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    u = torch.zeros(z_u.size, dtype=torch.float64, device="cuda")
    uh = torch.zeros(z_uh.size, dtype=torch.float64, device="cuda")
    hist = pl.newton(geom_dev(inp), m, u, uh, tol=1e-12, restart=50, max_iters=5000, rtol=1e-14, prec="bj",
                     orth="cgs2")
    say("newton elasticity", [h["norm"] for h in hist], [h["norm"] for h in hist_o])
    assert len(hist) == 2 and hist[0]["alpha"] == 1.0
    assert relerr(u.cpu().numpy(), uo.ravel()) < 1e-10 and relerr(uh.cpu().numpy(), uho.ravel()) < 1e-10


def test_element_blocks_sys_full_size_sampled(ctx):
    """The Navier-Stokes hex workload at full size (16^3 hexes, p = 2, 4096 elements) at its
    linearisation state with the backward-Euler term: sampled elements against the oracle."""
    from paper_2512_13619_amd.pipeline import Pipeline
    pb = configs.c3(device="cuda")
    inp = pb.newton_inputs_sys()
    d = pb.dims()
    say("full size", d)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    out = pl.element_arrays()
    m = inp["model"]
    u, uh = inp["u0"].flatten(), inp["uhat0"].flatten()
    pl.element_blocks(geom_dev(inp), m, u, uh, out, time_term=dict(c=1.0 / m["dt"], u_prev=u.clone()))
    torch.cuda.synchronize()
    # the generator's own blocks at the same state (forward-mode autodiff, einsum): every element,
    # in chunks
    ne = d["ne"]
    for e0 in range(0, ne, 512):
        e1 = min(ne, e0 + 512)
        gen = pb.element_blocks(e0, e1)
        for k in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J"):
            want = gen[k]
            got = out[k].view((ne,) + tuple(want.shape[1:]))[e0:e1]
            err = float(((got - want).abs().max() / want.abs().max()).item())
            assert err < 1e-12, (e0, k, err)
        for k in ("ru", "rt"):
            want = gen[k]
            got = out[k].view((ne,) + tuple(want.shape[1:]))[e0:e1]
            assert float((got - want).abs().max().item()) < 1e-12 * max(1.0, float(want.abs().max().item())), (e0, k)
        del gen
    # and three sampled elements against the oracle
    inp_np = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in inp.items()}
    uh_el = OS.element_trace_values(inp_np["uhat0"], pb.mesh.e2f)
    for e in (0, 1717, d["ne"] - 1):
        q = OS.consistent_q(inp_np, e, inp_np["u0"][e], uh_el[e])
        _, Ru, Rt = OS.residual(inp_np, m, e, q, inp_np["u0"][e], uh_el[e], (1.0 / m["dt"], inp_np["u0"][e], None))
        Dm, Em, Fm, Gm, Hm, Jm = OS.jacobian(inp_np, m, e, q, inp_np["u0"][e], uh_el[e], 1.0 / m["dt"])
        for k, ref in (("D", Dm), ("E", Em), ("F", Fm), ("G", Gm), ("H", Hm), ("J", Jm)):
            got = out[k].view(d["ne"], *ref.shape)[e].cpu().numpy()
            assert relerr(got, ref) < 1e-12, (e, k)
        got = out["ru"].view(d["ne"], -1)[e].cpu().numpy()
        assert np.abs(got + Ru.ravel()).max() < 1e-12 * max(1.0, np.abs(Ru).max()), e
