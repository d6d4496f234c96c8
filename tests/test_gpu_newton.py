"""Device element residuals/Jacobian blocks and the damped Newton loop against the oracle
(Section 4.1, Section 4.4): hdg_element_blocks, hdg_residual_norm, Pipeline.newton."""
import numpy as np
import pytest
import torch

import oracle.elements as OE
import oracle.newton as ON
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


def _forcing(x):
    return (torch.sin(np.pi * x[..., 0]) * torch.sin(2 * np.pi * x[..., 1]))[..., None]


CASES = {
    "burgers_tri_p3": lambda: HDGProblem(Mh.structured_tris(3, 0.0, 4), 3, Ph.Burgers(nu=0.05)),
    "burgers_quad_p2": lambda: HDGProblem(Mh.structured_quads(3, 0.1, 4), 2, Ph.Burgers(nu=0.01, forcing=_forcing)),
    "burgers_quad_p4": lambda: HDGProblem(Mh.structured_quads(4, 0.05, 6), 4, Ph.Burgers(nu=0.02, forcing=_forcing)),
    "poisson_tri_p2": lambda: HDGProblem(Mh.structured_tris(3, 0.1, 5), 2, Ph.Poisson(2, 1.0, forcing=_forcing)),
}
_cache = {}


def case(name):
    if name not in _cache:
        pb = CASES[name]()
        inp = pb.newton_inputs()
        _cache[name] = (pb, inp, {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in inp.items()})
    return _cache[name]


def _model(inp):
    return dict(nu=inp["nu"], tau=inp["tau"], beta=inp["beta"], gamma=inp["gamma"])


def _geom_dev(inp):
    g = {k: inp[k].cuda().contiguous() for k in ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD",
                                                  "bnd")}
    g["nqv"], g["nqf"] = inp["nqv"], inp["nqf"]
    return g


def _random_state(pb, inp_np, seed):
    rng = np.random.default_rng(seed)
    u = inp_np["u0"] + 0.3 * rng.standard_normal(inp_np["u0"].shape)
    uh = inp_np["uhat0"] + 0.3 * rng.standard_normal(inp_np["uhat0"].shape)
    return u, uh


@pytest.mark.parametrize("name", list(CASES))
def test_element_blocks_match_oracle(ctx, name):
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case(name)
    d = pb.dims()
    say("element blocks", name, d)
    u, uh = _random_state(pb, inp_np, 1)
    ref = OE.element_blocks(inp_np, _model(inp_np), u, uh, pb.mesh.e2f)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    out = pl.element_arrays()
    ctx.element_blocks(d, _geom_dev(inp), _model(inp), pl.e2f, torch.as_tensor(u).cuda().flatten(),
                       torch.as_tensor(uh).cuda().flatten(), out)
    torch.cuda.synchronize()
    for k in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt", "q"):
        got = out[k].cpu().numpy().reshape(ref[k].shape)
        err = relerr(got, ref[k])
        assert err < 1e-12, (k, err)


def test_residual_only_and_norm(ctx):
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case("burgers_tri_p3")
    d = pb.dims()
    u, uh = _random_state(pb, inp_np, 2)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    full = pl.element_arrays()
    ud, uhd = torch.as_tensor(u).cuda().flatten(), torch.as_tensor(uh).cuda().flatten()
    ctx.element_blocks(d, _geom_dev(inp), _model(inp), pl.e2f, ud, uhd, full)
    res = {"ru": torch.full_like(full["ru"], np.nan), "rt": torch.full_like(full["rt"], np.nan)}
    ctx.element_blocks(d, _geom_dev(inp), _model(inp), pl.e2f, ud, uhd, res, residual_only=True)
    torch.cuda.synchronize()
    assert torch.equal(res["ru"], full["ru"]) and torch.equal(res["rt"], full["rt"])
    nrm = ctx.residual_norm(d, pl.f2e, res["ru"], res["rt"])
    ref = OE.element_blocks(inp_np, _model(inp_np), u, uh, pb.mesh.e2f)
    want = ON._norm_from_blocks(ref, pb.mesh.e2f, pb.mesh.f2e, d)
    assert abs(nrm - want) <= 1e-12 * want


@pytest.mark.parametrize("name,prec", [("burgers_quad_p2", "bj"), ("burgers_tri_p3", "asm"),
                                       ("poisson_tri_p2", "bj"), ("burgers_quad_p4", "ilu_asm")])
def test_newton_matches_oracle(ctx, name, prec):
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case(name)
    d = pb.dims()
    say("newton", name, prec)
    m = _model(inp_np)
    u_ref, uh_ref, hist_ref = ON.damped_newton(inp_np, m, inp_np["u0"], inp_np["uhat0"], pb.mesh.e2f, pb.mesh.f2e,
                                               d, rtol=1e-11)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    u = inp["u0"].cuda().flatten().clone()
    uh = inp["uhat0"].cuda().flatten().clone()
    g = _geom_dev(inp)
    hist = pl.newton(g, _model(inp), u, uh, tol=1e-11, restart=50, max_iters=2000, rtol=1e-13, prec=prec)
    say("  steps", [(f"{h['norm']:.3e}", h["alpha"], h["iters"]) for h in hist])
    assert len(hist) == len(hist_ref)
    assert [h["alpha"] for h in hist] == [h["alpha"] for h in hist_ref]
    for a, b in zip(hist, hist_ref):
        assert abs(a["norm"] - b["norm"]) <= 1e-7 * hist_ref[0]["norm"]
    assert relerr(u.cpu().numpy(), u_ref.ravel()) < 1e-9
    assert relerr(uh.cpu().numpy(), uh_ref.ravel()) < 1e-9


def test_element_blocks_rejects_bad_input(ctx):
    from paper_2512_13619_amd import hdg
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case("poisson_tri_p2")
    d = dict(pb.dims())
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    out = pl.element_arrays()
    u = inp["u0"].cuda().flatten()
    uh = inp["uhat0"].cuda().flatten()
    g = _geom_dev(inp)
    with pytest.raises(hdg.HdgError):           # matrices requested but missing
        ctx.element_blocks(d, g, _model(inp), pl.e2f, u, uh, {"ru": out["ru"], "rt": out["rt"]})
    ne, P, D, L = d["ne"], d["npe"], d["dim"], d["nlfe"]
    Qv = 4000                                   # one element's LDS above 64 KiB: rejected on the host
    big = dict(g, nqv=Qv, wdet=torch.zeros(ne * Qv, dtype=torch.float64, device="cuda"),
               dphix=torch.zeros(ne * Qv * P * D, dtype=torch.float64, device="cuda"),
               phi=torch.zeros(Qv * P, dtype=torch.float64, device="cuda"),
               src=torch.zeros(ne * Qv, dtype=torch.float64, device="cuda"))
    with pytest.raises(hdg.HdgError) as ei:
        ctx.element_blocks(d, big, _model(inp), pl.e2f, u, uh, out)
    assert "LDS" in str(ei.value)
    # no elements: nothing to do
    per_elem = ("wdet", "dphix", "phif", "ndA", "dA", "src", "uD", "bnd")
    g0 = {k: (v[:0] if k in per_elem else v) for k, v in g.items()}
    ctx.element_blocks(dict(d, ne=0), g0, _model(inp), pl.e2f[:0], u[:0], uh, {k: v[:0] for k, v in out.items()})


# ---- implicit stages and DIRK time stepping (Section 2.2) ----------------------------------
def test_element_blocks_time_term_matches_oracle(ctx):
    from paper_2512_13619_amd import hdg
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case("burgers_quad_p2")
    d = pb.dims()
    u, uh = _random_state(pb, inp_np, 4)
    rng = np.random.default_rng(6)
    un = rng.standard_normal(u.shape)
    rx = rng.standard_normal(u.shape)
    c = 7.5
    ref = OE.element_blocks(inp_np, _model(inp_np), u, uh, pb.mesh.e2f, dict(c=c, u_prev=un, r_extra=rx))
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    out = pl.element_arrays()
    tt = dict(c=c, u_prev=torch.as_tensor(un).cuda().flatten(), r_extra=torch.as_tensor(rx).cuda().flatten())
    ctx.element_blocks(d, _geom_dev(inp), _model(inp), pl.e2f, torch.as_tensor(u).cuda().flatten(),
                       torch.as_tensor(uh).cuda().flatten(), out, time_term=tt)
    torch.cuda.synchronize()
    for k in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt", "q"):
        err = relerr(out[k].cpu().numpy().reshape(ref[k].shape), ref[k])
        assert err < 1e-12, (k, err)
    with pytest.raises(hdg.HdgError):
        ctx.element_blocks(d, _geom_dev(inp), _model(inp), pl.e2f, torch.as_tensor(u).cuda().flatten(),
                           torch.as_tensor(uh).cuda().flatten(), out, time_term=dict(c=1.0))


@pytest.mark.parametrize("name,scheme,dt,nsteps", [("burgers_quad_p2", "dirk22", 0.05, 2),
                                                   ("burgers_tri_p3", "dirk33", 0.1, 1),
                                                   ("poisson_tri_p2", "be", 0.02, 2)])
def test_dirk_steps_match_oracle(ctx, name, scheme, dt, nsteps):
    import oracle.dirk as ODK
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case(name)
    d = pb.dims()
    say("dirk", name, scheme, dt, nsteps)
    u_ref, uh_ref, hists_ref = ODK.dirk_steps(inp_np, _model(inp_np), inp_np["u0"], inp_np["uhat0"], pb.mesh.e2f,
                                              pb.mesh.f2e, d, dt, nsteps, scheme, newton_rtol=1e-12)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    u = inp["u0"].cuda().flatten().clone()
    uh = inp["uhat0"].cuda().flatten().clone()
    hists = pl.dirk(_geom_dev(inp), _model(inp), u, uh, dt, nsteps, scheme, tol=1e-12, restart=50, max_iters=2000,
                    rtol=1e-13, prec="bj")
    assert len(hists) == len(hists_ref)
    for h, hr in zip(hists, hists_ref):
        assert [x["alpha"] for x in h] == [x["alpha"] for x in hr]
    assert relerr(u.cpu().numpy(), u_ref.ravel()) < 1e-9
    assert relerr(uh.cpu().numpy(), uh_ref.ravel()) < 1e-9


@pytest.mark.parametrize("name,scheme,dt,nsteps", [("burgers_quad_p2", "dirk22", 0.05, 2),
                                                   ("burgers_tri_p3", "dirk33", 0.1, 1),
                                                   ("poisson_tri_p2", "be", 0.02, 2)])
def test_dirk_chord_reuse_reaches_the_oracle_states(ctx, name, scheme, dt, nsteps):
    """DIRK steps whose Newton solves keep the linearisation (condensation factors, assembled blocks,
    block-Jacobi setup) across Newton steps and stages, refreshing it after a weak step: the states
    equal the oracle's exact-Newton DIRK states, and most steps reuse the kept linearisation."""
    import oracle.dirk as ODK
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case(name)
    d = pb.dims()
    say("dirk chord", name, scheme, dt, nsteps)
    u_ref, uh_ref, _ = ODK.dirk_steps(inp_np, _model(inp_np), inp_np["u0"], inp_np["uhat0"], pb.mesh.e2f,
                                      pb.mesh.f2e, d, dt, nsteps, scheme, newton_rtol=1e-12)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    u = inp["u0"].cuda().flatten().clone()
    uh = inp["uhat0"].cuda().flatten().clone()
    hists = pl.dirk(_geom_dev(inp), _model(inp), u, uh, dt, nsteps, scheme, tol=1e-12, max_steps=60, restart=50,
                    max_iters=2000, rtol=1e-13, prec="bj", reuse="chord")
    steps = [x for h in hists for x in h[:-1]]
    fresh = sum(x["fresh"] for x in steps)
    say("  steps", len(steps), "fresh", fresh)
    assert all(h[-1]["norm"] <= 1e-12 * h[0]["norm"] for h in hists)
    assert fresh < len(steps)
    assert relerr(u.cpu().numpy(), u_ref.ravel()) < 1e-9
    assert relerr(uh.cpu().numpy(), uh_ref.ravel()) < 1e-9


# ---- the bench-size workload (2D Burgers, 128^2 quads, p = 4): sampled elements ------------
def _bench_problem():
    return HDGProblem(Mh.structured_quads(128, 0.05, 6), 4, Ph.Burgers(nu=0.01, forcing=_forcing), device="cuda")


def _sampled_geom(inp, elems):
    """The oracle's geometry dict for the sampled elements only (element index = position)."""
    per = ("wdet", "dphix", "phif", "ndA", "dA", "src", "uD", "bnd")
    g = {k: inp[k][elems].cpu().numpy() for k in per}
    g["phi"], g["psi"] = inp["phi"].cpu().numpy(), inp["psi"].cpu().numpy()
    return g


def test_element_blocks_full_size_sampled(ctx):
    from paper_2512_13619_amd.pipeline import Pipeline
    pb = _bench_problem()
    d = pb.dims()
    say("element blocks full size", d)
    inp = pb.newton_inputs()
    geom = _geom_dev(inp)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f, keep_fp32=False)
    out = pl.element_arrays()
    rng = np.random.default_rng(12)
    u = inp["u0"].flatten() + 0.2 * torch.as_tensor(rng.standard_normal(inp["u0"].numel())).cuda()
    uh = inp["uhat0"].flatten() + 0.2 * torch.as_tensor(rng.standard_normal(inp["uhat0"].numel())).cuda()
    ctx.element_blocks(d, geom, _model(inp), pl.e2f, u, uh, out)
    torch.cuda.synchronize()
    elems = np.sort(rng.choice(d["ne"], 24, replace=False))
    g = _sampled_geom(inp, elems)
    m = _model(inp)
    P, PF, L, D = d["npe"], d["npf"], d["nlfe"], d["dim"]
    nt = L * PF
    un = u.cpu().numpy().reshape(d["ne"], P)
    uhn = uh.cpu().numpy().reshape(d["nf"], PF)
    for k, e in enumerate(elems):
        ue, uhe = un[e], uhn[pb.mesh.e2f[e]]
        Mm, Bd, Cd = OE.mass_and_q_operators(g, k)
        q = OE.consistent_q(g, k, ue, uhe)
        _, Ru, Rt = OE.residual(g, m, k, q, ue, uhe)
        Dm, Em, Fm, Gm, Hm, Jm = OE.jacobian(g, m, k, q, ue, uhe)
        ref = dict(Minv=np.linalg.inv(Mm), Bd=Bd, Cd=Cd, D=Dm, E=Em, F=Fm, G=Gm, H=Hm, J=Jm, ru=-Ru,
                   rt=-Rt.ravel(), q=q)
        for key, val in ref.items():
            got = out[key].view(d["ne"], -1)[e].cpu().numpy().reshape(val.shape)
            err = relerr(got, val)
            assert err < 1e-12, (int(e), key, err)


def test_newton_full_size_residual_property(ctx):
    """At the bench size the Newton loop's final state solves the discrete equations: the
    library's norm drops by 1e-10 and the oracle's residual of sampled elements at that state
    is at the same level."""
    from paper_2512_13619_amd.pipeline import Pipeline
    pb = _bench_problem()
    d = pb.dims()
    inp = pb.newton_inputs()
    geom = _geom_dev(inp)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f, keep_fp32=False)
    u = inp["u0"].flatten().clone()
    uh = inp["uhat0"].flatten().clone()
    hist = pl.newton(geom, _model(inp), u, uh, tol=1e-10, restart=50, max_iters=20000, rtol=1e-10, prec="bj",
                     orth="dcgs2", fold_prec=True)
    say("  full-size newton", [(f"{h['norm']:.2e}", h["alpha"]) for h in hist])
    assert hist[-1]["norm"] <= 1e-10 * hist[0]["norm"]
    rng = np.random.default_rng(13)
    elems = np.sort(rng.choice(d["ne"], 24, replace=False))
    g = _sampled_geom(inp, elems)
    m = _model(inp)
    un = u.cpu().numpy().reshape(d["ne"], d["npe"])
    uhn = uh.cpu().numpy().reshape(d["nf"], d["npf"])
    worst = 0.0
    for k, e in enumerate(elems):
        ue, uhe = un[e], uhn[pb.mesh.e2f[e]]
        q = OE.consistent_q(g, k, ue, uhe)
        _, Ru, _ = OE.residual(g, m, k, q, ue, uhe)
        worst = max(worst, np.abs(Ru).max())
    assert worst <= 1e-9 * hist[0]["norm"], worst


# ---- many independent instances (the batched Poisson/Burgers workload) ----------------------
def _batch_instances():
    def f2(x):
        return (torch.cos(np.pi * x[..., 0]) * torch.sin(np.pi * x[..., 1]))[..., None]
    return [HDGProblem(Mh.structured_quads(4, 0.0, 4), 2, Ph.Burgers(nu=0.01, forcing=_forcing)),
            HDGProblem(Mh.structured_tris(3, 0.0, 4), 3, Ph.Burgers(nu=0.05)),
            HDGProblem(Mh.structured_quads(4, 0.0, 4), 1, Ph.Poisson(2, 1.0, forcing=f2)),
            HDGProblem(Mh.structured_tris(2, 0.0, 4), 4, Ph.Poisson(2, 1.0, forcing=_forcing)),
            HDGProblem(Mh.structured_quads(3, 0.0, 4), 4, Ph.Burgers(nu=0.02, forcing=f2))]


def test_batch_newton_matches_per_instance_oracle(ctx):
    from paper_2512_13619_amd.pipeline import BatchPipeline
    pbs = _batch_instances()
    say("batch newton", [(pb.etype, pb.mesh.ne, pb.p, type(pb.phys).__name__) for pb in pbs])
    inps = [pb.newton_inputs() for pb in pbs]
    bp = BatchPipeline(ctx, [pb.dims() for pb in pbs], [pb.mesh.f2e for pb in pbs], [pb.mesh.e2f for pb in pbs])
    keys = ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD", "bnd")
    geom = {k: torch.cat([inp[k].reshape(-1) for inp in inps]).cuda().contiguous() for k in keys}
    u = torch.cat([inp["u0"].reshape(-1) for inp in inps]).cuda().contiguous()
    uh = torch.cat([inp["uhat0"].reshape(-1) for inp in inps]).cuda().contiguous()
    models = [_model(inp) for inp in inps]
    hists = bp.newton([inp["nqv"] for inp in inps], [inp["nqf"] for inp in inps], geom, models, u, uh, tol=1e-11,
                      restart=50, max_iters=3000, rtol=1e-13, prec="bj")
    ou, oh = bp.bt.offsets("du"), bp.bt.offsets("vec")
    for i, (pb, inp) in enumerate(zip(pbs, inps)):
        inp_np = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in inp.items()}
        u_ref, uh_ref, h_ref = ON.damped_newton(inp_np, _model(inp_np), inp_np["u0"], inp_np["uhat0"], pb.mesh.e2f,
                                                pb.mesh.f2e, pb.dims(), rtol=1e-11)
        say("  instance", i, [(f"{h['norm']:.2e}", h["alpha"]) for h in hists[i]])
        assert [h["alpha"] for h in hists[i]] == [h["alpha"] for h in h_ref], i
        for a, b in zip(hists[i], h_ref):
            assert abs(a["norm"] - b["norm"]) <= 1e-7 * h_ref[0]["norm"], i
        assert relerr(u[ou[i]:ou[i + 1]].cpu().numpy(), u_ref.ravel()) < 1e-9, i
        assert relerr(uh[oh[i]:oh[i + 1]].cpu().numpy(), uh_ref.ravel()) < 1e-9, i


def test_batch_element_blocks_match_single_instance(ctx):
    """The batched kernel writes, for every instance, what the single-instance kernel writes."""
    from paper_2512_13619_amd.pipeline import BatchPipeline, Pipeline
    pbs = _batch_instances()
    inps = [pb.newton_inputs() for pb in pbs]
    bp = BatchPipeline(ctx, [pb.dims() for pb in pbs], [pb.mesh.f2e for pb in pbs], [pb.mesh.e2f for pb in pbs])
    keys = ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD", "bnd")
    geom = {k: torch.cat([inp[k].reshape(-1) for inp in inps]).cuda().contiguous() for k in keys}
    rng = np.random.default_rng(21)
    us = [inp["u0"].reshape(-1).cuda() + 0.3 * torch.as_tensor(rng.standard_normal(inp["u0"].numel())).cuda()
          for inp in inps]
    uhs = [inp["uhat0"].reshape(-1).cuda() + 0.3 * torch.as_tensor(rng.standard_normal(inp["uhat0"].numel())).cuda()
           for inp in inps]
    out = bp.element_arrays()
    bp.bt.element_blocks([inp["nqv"] for inp in inps], [inp["nqf"] for inp in inps], geom,
                         [_model(inp) for inp in inps], bp.e2f, torch.cat(us), torch.cat(uhs), out)
    norms = bp.bt.residual_norms(bp.f2e, out["ru"], out["rt"])
    for i, (pb, inp) in enumerate(zip(pbs, inps)):
        pl = Pipeline(ctx, pb.dims(), pb.mesh.f2e, pb.mesh.e2f)
        ref = pl.element_arrays()
        ctx.element_blocks(pb.dims(), _geom_dev(inp), _model(inp), pl.e2f, us[i], uhs[i], ref)
        for k in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt", "q"):
            o = bp.bt.offsets("dq" if k == "q" else k)
            assert torch.equal(out[k][o[i]:o[i + 1]], ref[k]), (i, k)
        want = ctx.residual_norm(pb.dims(), pl.f2e, ref["ru"], ref["rt"])
        assert abs(norms[i] - want) <= 1e-13 * want, (i, norms[i], want)


def test_batch_pseudo_transient_matches_per_instance_oracle(ctx):
    from paper_2512_13619_amd.pipeline import BatchPipeline
    pbs = _batch_instances()
    inps = [pb.newton_inputs() for pb in pbs]
    bp = BatchPipeline(ctx, [pb.dims() for pb in pbs], [pb.mesh.f2e for pb in pbs], [pb.mesh.e2f for pb in pbs])
    keys = ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD", "bnd")
    geom = {k: torch.cat([inp[k].reshape(-1) for inp in inps]).cuda().contiguous() for k in keys}
    u = torch.cat([inp["u0"].reshape(-1) for inp in inps]).cuda().contiguous()
    uh = torch.cat([inp["uhat0"].reshape(-1) for inp in inps]).cuda().contiguous()
    hists = bp.pseudo_transient([inp["nqv"] for inp in inps], [inp["nqf"] for inp in inps], geom,
                                [_model(inp) for inp in inps], u, uh, 0.05, tol=1e-11, restart=50, max_iters=3000,
                                rtol=1e-13, prec="bj")
    ou, oh = bp.bt.offsets("du"), bp.bt.offsets("vec")
    for i, (pb, inp) in enumerate(zip(pbs, inps)):
        inp_np = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in inp.items()}
        u_ref, uh_ref, h_ref = ON.pseudo_transient(inp_np, _model(inp_np), inp_np["u0"], inp_np["uhat0"],
                                                   pb.mesh.e2f, pb.mesh.f2e, pb.dims(), 0.05, rtol=1e-11)
        say("  ptc instance", i, len(hists[i]) - 1, f"{hists[i][-1]['norm']:.2e}")
        assert len(hists[i]) == len(h_ref), i
        for a, b in zip(hists[i], h_ref):
            assert abs(a["norm"] - b["norm"]) <= 1e-7 * h_ref[0]["norm"], i
            assert abs(a["dtau"] - b["dtau"]) <= 1e-6 * max(b["dtau"], 1e-300), i
        assert relerr(u[ou[i]:ou[i + 1]].cpu().numpy(), u_ref.ravel()) < 1e-9, i
        assert relerr(uh[oh[i]:oh[i + 1]].cpu().numpy(), uh_ref.ravel()) < 1e-9, i


def test_kept_mass_matrices_give_identical_blocks(ctx):
    """HDG_ELEM_KEEP_MASS (M^-1, B_d, C_d kept from an earlier call on the mesh) gives bitwise the
    blocks and residuals of a full evaluation, single-mesh and batched, and leaves the kept
    arrays untouched."""
    from paper_2512_13619_amd.pipeline import BatchPipeline, Pipeline
    pb, inp, inp_np = case("burgers_quad_p4")
    d = pb.dims()
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    u0, uh0 = _random_state(pb, inp_np, 8)
    u1, uh1 = _random_state(pb, inp_np, 9)
    t = lambda a: torch.as_tensor(a).cuda().flatten()
    full, kept = pl.element_arrays(), pl.element_arrays()
    ctx.element_blocks(d, _geom_dev(inp), _model(inp), pl.e2f, t(u0), t(uh0), kept)     # forms M^-1, B_d, C_d
    ctx.element_blocks(d, _geom_dev(inp), _model(inp), pl.e2f, t(u1), t(uh1), full)
    saved = {k: kept[k].clone() for k in ("Minv", "Bd", "Cd")}
    ctx.element_blocks(d, _geom_dev(inp), _model(inp), pl.e2f, t(u1), t(uh1), kept, keep_mass=True)
    for k in full:
        assert torch.equal(full[k], kept[k]), k
    for k, v in saved.items():
        assert torch.equal(v, kept[k]), k
    res = {"ru": torch.zeros_like(full["ru"]), "rt": torch.zeros_like(full["rt"]), "Minv": kept["Minv"]}
    ctx.element_blocks(d, _geom_dev(inp), _model(inp), pl.e2f, t(u1), t(uh1), res, residual_only=True,
                       keep_mass=True)
    assert torch.equal(res["ru"], full["ru"]) and torch.equal(res["rt"], full["rt"])
    # batched
    pbs = _batch_instances()
    inps = [q.newton_inputs() for q in pbs]
    bp = BatchPipeline(ctx, [q.dims() for q in pbs], [q.mesh.f2e for q in pbs], [q.mesh.e2f for q in pbs])
    keys = ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD", "bnd")
    geom = {k: torch.cat([x[k].reshape(-1) for x in inps]).cuda().contiguous() for k in keys}
    args = ([x["nqv"] for x in inps], [x["nqf"] for x in inps], geom, [_model(x) for x in inps], bp.e2f)
    ub = torch.cat([x["u0"].reshape(-1) for x in inps]).cuda()
    uhb = torch.cat([x["uhat0"].reshape(-1) for x in inps]).cuda()
    fb, kb = bp.element_arrays(), bp.element_arrays()
    bp.bt.element_blocks(*args, 0.5 * ub, 0.5 * uhb, kb)
    bp.bt.element_blocks(*args, ub, uhb, fb)
    bp.bt.element_blocks(*args, ub, uhb, kb, keep_mass=True)
    for k in fb:
        assert torch.equal(fb[k], kb[k]), k


def test_inexact_newton_reaches_the_same_solution(ctx):
    """Eisenstat-Walker forcing (looser linear solves early on) converges to the oracle's
    discrete solution, with no more Newton steps than the oracle needs plus two."""
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case("burgers_quad_p2")
    d = pb.dims()
    u_ref, uh_ref, h_ref = ON.damped_newton(inp_np, _model(inp_np), inp_np["u0"], inp_np["uhat0"], pb.mesh.e2f,
                                            pb.mesh.f2e, d, rtol=1e-11)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    u = inp["u0"].cuda().flatten().clone()
    uh = inp["uhat0"].cuda().flatten().clone()
    hist = pl.newton(_geom_dev(inp), _model(inp), u, uh, tol=1e-11, restart=50, max_iters=2000, rtol=1e-13,
                     prec="bj", forcing="ew")
    say("  inexact newton", [(f"{h['norm']:.2e}", h["alpha"], h["iters"]) for h in hist])
    assert hist[-1]["norm"] <= 1e-11 * hist[0]["norm"]
    assert len(hist) <= len(h_ref) + 2
    assert relerr(u.cpu().numpy(), u_ref.ravel()) < 1e-8
    assert relerr(uh.cpu().numpy(), uh_ref.ravel()) < 1e-8


@pytest.mark.parametrize("name", ["burgers_quad_p2", "burgers_tri_p3"])
def test_pseudo_transient_single_mesh_matches_oracle(ctx, name):
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, inp, inp_np = case(name)
    d = pb.dims()
    u_ref, uh_ref, h_ref = ON.pseudo_transient(inp_np, _model(inp_np), inp_np["u0"], inp_np["uhat0"], pb.mesh.e2f,
                                               pb.mesh.f2e, d, 0.05, rtol=1e-11)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    u = inp["u0"].cuda().flatten().clone()
    uh = inp["uhat0"].cuda().flatten().clone()
    hist = pl.pseudo_transient(_geom_dev(inp), _model(inp), u, uh, 0.05, tol=1e-11, restart=50, max_iters=2000,
                               rtol=1e-13, prec="bj")
    assert len(hist) == len(h_ref)
    for a, b in zip(hist, h_ref):
        assert abs(a["norm"] - b["norm"]) <= 1e-7 * h_ref[0]["norm"]
        assert abs(a["dtau"] - b["dtau"]) <= 1e-6 * max(b["dtau"], 1e-300)
    assert relerr(u.cpu().numpy(), u_ref.ravel()) < 1e-9
    assert relerr(uh.cpu().numpy(), uh_ref.ravel()) < 1e-9


def test_batch_dirk_matches_per_instance_oracle(ctx):
    import oracle.dirk as ODK
    from paper_2512_13619_amd.pipeline import BatchPipeline
    pbs = _batch_instances()
    inps = [pb.newton_inputs() for pb in pbs]
    bp = BatchPipeline(ctx, [pb.dims() for pb in pbs], [pb.mesh.f2e for pb in pbs], [pb.mesh.e2f for pb in pbs])
    keys = ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD", "bnd")
    geom = {k: torch.cat([inp[k].reshape(-1) for inp in inps]).cuda().contiguous() for k in keys}
    u = torch.cat([inp["u0"].reshape(-1) for inp in inps]).cuda().contiguous()
    uh = torch.cat([inp["uhat0"].reshape(-1) for inp in inps]).cuda().contiguous()
    stages = bp.dirk([inp["nqv"] for inp in inps], [inp["nqf"] for inp in inps], geom, [_model(inp) for inp in inps],
                     u, uh, 0.05, 1, "dirk22", tol=1e-12, restart=50, max_iters=3000, rtol=1e-13, prec="bj")
    assert len(stages) == 2
    ou, oh = bp.bt.offsets("du"), bp.bt.offsets("vec")
    for i, (pb, inp) in enumerate(zip(pbs, inps)):
        inp_np = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in inp.items()}
        u_ref, uh_ref, h_ref = ODK.dirk_steps(inp_np, _model(inp_np), inp_np["u0"], inp_np["uhat0"], pb.mesh.e2f,
                                              pb.mesh.f2e, pb.dims(), 0.05, 1, "dirk22", newton_rtol=1e-12)
        for st, hr in zip(stages, h_ref):
            assert [x["alpha"] for x in st[i]] == [x["alpha"] for x in hr], i
        assert relerr(u[ou[i]:ou[i + 1]].cpu().numpy(), u_ref.ravel()) < 1e-9, i
        assert relerr(uh[oh[i]:oh[i + 1]].cpu().numpy(), uh_ref.ravel()) < 1e-9, i
