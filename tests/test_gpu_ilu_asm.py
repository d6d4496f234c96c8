"""ILU-ASM on the GPU (hdg_ilu_asm_create / hdg_ilu_asm_apply and GMRES with HDG_PREC_ILU_ASM)
against the oracle (Section 3.3's ASM on multi-element subdomains with block ILU(0) solves)."""
import numpy as np
import pytest
import torch

from oracle import ilu_asm, krylov

from test_gpu_parity import case_data, _dev_matrix, orth_kw, relerr, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2512_13619_amd import hdg
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return hdg.Context(0)


def _e2f(pb):
    return torch.as_tensor(pb.mesh.e2f.astype(np.int32)).cuda().contiguous()


@pytest.mark.parametrize("name,G", [("c1", 1), ("c1", 2), ("c1", 4), ("c1", 8), ("poisson_quad_p3", 3),
                                    ("burgers_tri_p4", 4)])
def test_ilu_asm_apply_matches_oracle(ctx, name, G):
    pb, out = case_data(name)
    d = pb.dims()
    nb = d["ncomp"] * d["npf"]
    say("ilu-asm apply", name, G)
    K, _, nbr = _dev_matrix(out)
    h = ctx.ilu_asm_create(d, K, nbr, _e2f(pb), G)
    y = np.random.default_rng(G).standard_normal(out["r"].size)
    z = torch.zeros(y.size, dtype=torch.float64, device="cuda")
    ctx.ilu_asm_apply(h, torch.as_tensor(y).cuda(), z)
    torch.cuda.synchronize()
    ref = ilu_asm.apply(ilu_asm.setup(out["K"], out["nbr"], pb.mesh.e2f, G), y, nb)
    err = relerr(z.cpu().numpy(), ref)
    say("  rel err", err)
    assert err < 1e-11, err
    h.close()


def test_single_element_subdomains_equal_element_asm(ctx):
    pb, out = case_data("c1")
    d = pb.dims()
    K, _, nbr = _dev_matrix(out)
    e2f = _e2f(pb)
    f2e = torch.as_tensor(pb.mesh.f2e.astype(np.int32)).cuda().contiguous()
    ne, L = d["ne"], d["nlfe"]
    nt = L * d["ncomp"] * d["npf"]
    Kbar = torch.as_tensor(out["Kbar"]).cuda().contiguous()
    inv64 = torch.zeros(ne * nt * nt, dtype=torch.float64, device="cuda")
    ctx.asm_setup(d, Kbar, K, e2f, inv64, None)
    y = torch.as_tensor(np.random.default_rng(5).standard_normal(out["r"].size)).cuda()
    za = torch.zeros_like(y)
    ctx.asm_apply(d, inv64, None, f2e, e2f, y, za, "fp64")
    zi = torch.zeros_like(y)
    h = ctx.ilu_asm_create(d, K, nbr, e2f, 1)
    ctx.ilu_asm_apply(h, y, zi)
    torch.cuda.synchronize()
    assert relerr(zi.cpu().numpy(), za.cpu().numpy()) < 1e-11


@pytest.mark.parametrize("orth", ["cgs2", "dcgs2"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gmres_ilu_asm_matches_oracle(ctx, orth, precision):
    pb, out = case_data("c1")
    d = pb.dims()
    nb = d["ncomp"] * d["npf"]
    K, K32, nbr = _dev_matrix(out)
    h = ctx.ilu_asm_create(d, K, nbr, _e2f(pb), 4)
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    st = ctx.gmres_solve(d, K, K32, nbr, r, x, restart=50, max_iters=500, rtol=1e-12, prec="ilu_asm", ilu=h,
                         precision=precision, **orth_kw(orth))
    subs = ilu_asm.setup(out["K"], out["nbr"], pb.mesh.e2f, 4)
    solver = krylov.fgmres if orth == "cgs2" else krylov.gmres_dcgs2
    _, info = solver(lambda v: out["A"] @ v, out["r"], prec=lambda v: ilu_asm.apply(subs, v, nb), restart=50,
                     rtol=1e-12, max_iters=500)
    say("ilu-asm gmres", orth, precision, st["iters"], info["iters"])
    assert st["converged"], st
    if precision == "fp64":
        assert abs(st["iters"] - info["iters"]) <= 1
    assert relerr(x.cpu().numpy(), out["x"]) < (1e-10 if precision == "fp64" else 1e-8)


def test_ilu_asm_rejects_oversized_subdomains_and_missing_handle(ctx):
    from paper_2512_13619_amd import hdg
    pb, out = case_data("c1")
    d = pb.dims()
    K, K32, nbr = _dev_matrix(out)
    with pytest.raises(hdg.HdgError):
        ctx.ilu_asm_create(d, K, nbr, _e2f(pb), 16)      # 42 faces x 3 dofs > 88
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    with pytest.raises(hdg.HdgError):
        ctx.gmres_solve(d, K, K32, nbr, r, x, prec="ilu_asm")
