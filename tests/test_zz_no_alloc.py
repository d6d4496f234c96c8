"""The allocation-free residual norm (hdg_residual_norm_noalloc, fixed per-device scratch)
against hdg_residual_norm, called through the C ABI: two calls in a row, the second on a
smaller mesh, so the second reads a scratch array that still holds the first call's data."""
import numpy as np
import pytest
import torch

from workloads import mesh as Mh
from workloads import physics as Ph
from workloads.blocks import HDGProblem

pytestmark = pytest.mark.gpu


def _forcing(x):
    return (torch.sin(np.pi * x[..., 0]) * torch.sin(2 * np.pi * x[..., 1]))[..., None]


def _residual(ctx, pb, seed):
    """Element residual rows (ru, rt) at a seeded state, from the device element kernel."""
    from paper_2512_13619_amd.pipeline import Pipeline
    inp = pb.newton_inputs()
    d = pb.dims()
    rng = np.random.default_rng(seed)
    u = inp["u0"].cpu().numpy() + 0.3 * rng.standard_normal(tuple(inp["u0"].shape))
    uh = inp["uhat0"].cpu().numpy() + 0.3 * rng.standard_normal(tuple(inp["uhat0"].shape))
    g = {k: inp[k].cuda().contiguous() for k in ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD",
                                                  "bnd")}
    g["nqv"], g["nqf"] = inp["nqv"], inp["nqf"]
    model = dict(nu=inp["nu"], tau=inp["tau"], beta=inp["beta"], gamma=inp["gamma"])
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    res = pl.element_arrays()
    ctx.element_blocks(d, g, model, pl.e2f, torch.as_tensor(u).cuda().flatten(), torch.as_tensor(uh).cuda().flatten(),
                       res, residual_only=True)
    torch.cuda.synchronize()
    return d, pl.f2e, res["ru"], res["rt"]


def test_residual_norm_noalloc_matches_allocating_entry_point():
    from paper_2512_13619_amd import hdg
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ctx = hdg.Context(0)
    big = HDGProblem(Mh.structured_quads(24, 0.1, 4), 4, Ph.Burgers(nu=0.01, forcing=_forcing))
    small = HDGProblem(Mh.structured_tris(5, 0.05, 6), 2, Ph.Burgers(nu=0.05))
    for pb, seed in ((big, 1), (small, 2)):
        d, f2e, ru, rt = _residual(ctx, pb, seed)
        want = ctx.residual_norm(d, f2e, ru, rt)
        got = ctx.residual_norm(d, f2e, ru, rt, noalloc=True)
        print(f"[gpu-test] noalloc residual norm ne={d['ne']} nf={d['nf']}: {got!r} vs {want!r}", flush=True)
        # same kernels, same reduction order: identical
        assert np.isfinite(want) and want > 0 and got == want, (got, want)


def test_residual_norm_noalloc_rejects_oversize():
    from paper_2512_13619_amd import hdg
    ctx = hdg.Context(0)
    d = dict(ne=1, nf=1 << 21, ncomp=1, dim=2, npe=3, npf=2, nlfe=3)
    ru = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(hdg.HdgError) as ei:
        ctx.residual_norm(d, torch.zeros((1 << 21) * 4, dtype=torch.int32, device="cuda"), ru,
                          torch.zeros(3 * 2, dtype=torch.float64, device="cuda"), noalloc=True)
    assert ei.value.status == -1 and "scratch" in str(ei.value)
