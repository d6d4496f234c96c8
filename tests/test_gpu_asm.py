"""Additive Schwarz with element patches on the GPU (hdg_asm_setup, hdg_asm_apply and the
ASM / ASM-PP / ASM-Chebyshev solves) against the oracle (Section 3.3, Section 4.6)."""
import sys

import numpy as np
import pytest
import torch

from oracle import krylov

from test_gpu_parity import case_data, _dev_matrix, orth_kw, relerr, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2512_13619_amd import hdg
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return hdg.Context(0)


def _asm_dev(ctx, pb, out, fp32=True):
    d = pb.dims()
    ne, L = d["ne"], d["nlfe"]
    nb = d["ncomp"] * d["npf"]
    nt = L * nb
    Kbar = torch.as_tensor(out["Kbar"]).cuda().contiguous()
    K = torch.as_tensor(out["K"]).cuda().contiguous()
    e2f = torch.as_tensor(pb.mesh.e2f.astype(np.int32)).cuda().contiguous()
    f2e = torch.as_tensor(pb.mesh.f2e.astype(np.int32)).cuda().contiguous()
    inv64 = torch.zeros(ne * nt * nt, dtype=torch.float64, device="cuda")
    inv32 = torch.zeros(ne * nt * nt, dtype=torch.float32, device="cuda") if fp32 else None
    ctx.asm_setup(d, Kbar, K, e2f, inv64, inv32)
    return dict(inv64=inv64, inv32=inv32, f2e=f2e, e2f=e2f)


def _oracle_inv(pb, out):
    d = pb.dims()
    return krylov.asm_inverses(krylov.asm_matrices(out["Kbar"], out["K"], pb.mesh.f2e, pb.mesh.e2f, d))


@pytest.mark.parametrize("name", ["c1", "elast_hex_p3", "ns_hex_p2", "ns_tet_p2"])
def test_asm_setup_matches_oracle_inverses(ctx, name):
    pb, out = case_data(name)
    say("asm setup", name)
    d = pb.dims()
    ne, L = d["ne"], d["nlfe"]
    nb = d["ncomp"] * d["npf"]
    a = _asm_dev(ctx, pb, out)
    torch.cuda.synchronize()
    ref = _oracle_inv(pb, out)                                # [ne][nt][nt]
    # inv[e][l][l'][col][row] = P^{-1}(l nb + row, l' nb + col)
    g = a["inv64"].cpu().numpy().reshape(ne, L, L, nb, nb).transpose(0, 1, 4, 2, 3).reshape(ne, L * nb, L * nb)
    err = max(relerr(g[e], ref[e]) for e in range(ne))
    say("  max rel err", err)
    assert err < 1e-10, err
    assert np.array_equal(a["inv32"].cpu().numpy(), a["inv64"].cpu().numpy().astype(np.float32))


@pytest.mark.parametrize("name", ["c1", "elast_hex_p3", "ns_tet_p2"])
def test_asm_apply_matches_oracle(ctx, name):
    pb, out = case_data(name)
    say("asm apply", name)
    d = pb.dims()
    a = _asm_dev(ctx, pb, out)
    y = np.random.default_rng(11).standard_normal(out["r"].size)
    ref = krylov.asm_apply(_oracle_inv(pb, out), pb.mesh.e2f, y, d)
    yd = torch.as_tensor(y).cuda()
    z = torch.zeros_like(yd)
    ctx.asm_apply(d, a["inv64"], None, a["f2e"], a["e2f"], yd, z, "fp64")
    assert relerr(z.cpu().numpy(), ref) < 1e-10
    ctx.asm_apply(d, None, a["inv32"], a["f2e"], a["e2f"], yd, z, "mixed")
    assert relerr(z.cpu().numpy(), ref) < 1e-5


@pytest.mark.parametrize("orth", ["cgs2", "dcgs2"])
@pytest.mark.parametrize("precision,prec", [("fp64", "asm"), ("mixed", "asm"), ("fp64", "asm_poly"),
                                            ("mixed", "asm_poly"), ("fp64", "asm_cheb")])
def test_gmres_asm_solution(ctx, precision, prec, orth):
    pb, out = case_data("c1")
    say("solve asm c1", precision, prec, orth)
    a = _asm_dev(ctx, pb, out)
    K, K32, nbr = _dev_matrix(out)
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    v0 = torch.as_tensor(np.random.default_rng(7).standard_normal(r.numel())).cuda()
    st = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, x, restart=50, max_iters=2000, rtol=1e-13, prec=prec,
                         poly_v0=v0, poly_degree=6, precision=precision, asm=a, **orth_kw(orth))
    assert st["converged"], st
    ex = relerr(x.cpu().numpy(), out["x"])
    say("  iters", st["iters"], "err", ex)
    assert ex < (1e-10 if precision == "fp64" else 1e-8), ex


@pytest.mark.parametrize("orth", ["cgs2", "dcgs2"])
def test_gmres_asm_history_matches_oracle(ctx, orth):
    pb, out = case_data("c1")
    d = pb.dims()
    a = _asm_dev(ctx, pb, out, fp32=False)
    K, _, nbr = _dev_matrix(out)
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    st = ctx.gmres_solve(d, K, None, nbr, r, x, restart=50, max_iters=500, rtol=1e-12, prec="asm", hist_len=600,
                         asm=a, **orth_kw(orth))
    Pinv = _oracle_inv(pb, out)
    hist = []
    solver = krylov.fgmres if orth == "cgs2" else krylov.gmres_dcgs2
    _, info = solver(lambda v: out["A"] @ v, out["r"], prec=lambda v: krylov.asm_apply(Pinv, pb.mesh.e2f, v, d),
                     restart=50, rtol=1e-12, max_iters=500, hist=hist)
    assert abs(st["iters"] - info["iters"]) <= 1
    n = min(20, len(hist), len(st["hist"]))
    assert np.allclose(st["hist"][:n], hist[:n], rtol=1e-6)


def test_asm_requires_its_data(ctx):
    from paper_2512_13619_amd import hdg
    pb, out = case_data("c1")
    K, K32, nbr = _dev_matrix(out)
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    with pytest.raises(hdg.HdgError):
        ctx.gmres_solve(pb.dims(), K, K32, nbr, r, x, prec="asm")
