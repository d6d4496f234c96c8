"""GPU parity: every entry point of libhdg.so against the FP64 oracle on the same
seeded inputs (element blocks from `workloads`), through the C ABI.

Tolerances: integer/index outputs and pure copies bit-exact; FP64 arithmetic to
a few hundred ulps of the data scale (different but stable elimination orders);
FGMRES solutions to 1e-10 relative (FP64 path) and 1e-8 (mixed path).
"""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle
from oracle import krylov, poly
from workloads import configs
from workloads import mesh as Mh
from workloads import physics as Ph
from workloads.blocks import HDGProblem

from helpers import blocks_np, oracle_pipeline

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2512_13619_amd import hdg
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return hdg.Context(0)


def make_case(name):
    if name == "c1":
        return configs.c1()
    if name == "poisson_quad_p3":
        return HDGProblem(Mh.structured_quads(3, 0.1, 3), 3, Ph.Poisson(2, 1.0, exact=configs.poisson_sin))
    if name == "elast_hex_p1":
        return HDGProblem(Mh.structured_hexes(2, 0.1, 3), 1, Ph.Elasticity(exact=Ph.elasticity_manufactured))
    if name == "elast_hex_p3":
        return HDGProblem(Mh.structured_hexes(2, 0.05, 2), 3, Ph.Elasticity(exact=Ph.elasticity_manufactured))
    if name == "ns_hex_p2":
        return HDGProblem(Mh.structured_hexes(2, 0.0, 3), 2, configs.navier_stokes(3, 0.07))
    if name == "ns_hex_p3":
        return HDGProblem(Mh.structured_hexes(2, 0.05, 7), 3, configs.navier_stokes(3, 0.07))
    if name == "ns_tet_p2":
        return HDGProblem(Mh.kuhn_tets(1, 0.1, 5), 2, configs.navier_stokes(5, 0.035))
    if name == "burgers_tri_p4":
        return HDGProblem(Mh.structured_tris(3, 0.0, 4), 4, Ph.Burgers(nu=0.01))
    raise KeyError(name)


# ns_hex_p3 (nu = 320, 80x80 face blocks) takes the large-element paths: LU panels in LDS,
# substitution in LDS slabs with a separate Schur product, block-Jacobi inverses in LDS, the
# tile-by-tile fold
CASES = ["c1", "poisson_quad_p3", "elast_hex_p1", "elast_hex_p3", "ns_hex_p2", "ns_tet_p2", "burgers_tri_p4",
         "ns_hex_p3"]
_cache = {}


def case_data(name):
    if name not in _cache:
        pb = make_case(name)
        out = oracle_pipeline(pb)
        _cache[name] = (pb, out)
    return _cache[name]


def to_dev(blk):
    return {k: torch.as_tensor(v).to("cuda").contiguous() for k, v in blk.items()}


def orth_kw(orth):
    """'dcgs2+fold': delayed CGS2 with the block-Jacobi inverses folded into the operator blocks."""
    if orth == "dcgs2+fold":
        return dict(orth="dcgs2", fold_prec=True)
    return dict(orth=orth)


ORTHS = ["cgs2", "dcgs2", "dcgs2+fold", "cgs", "mgs"]


def oracle_solver(orth):
    """The oracle routine a GPU orthogonalisation option is compared with: flexible GMRES with the
    same Gram-Schmidt variant, or GMRES with delayed CGS2 (whose iterates equal CGS2's)."""
    if orth in ("cgs2", "cgs", "mgs"):
        return lambda *a, **k: krylov.fgmres(*a, orth=orth, **k)
    return krylov.gmres_dcgs2


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def blockerr(a, b, nblocks, floor=1e-8):
    """Largest error of a block (element or face) relative to that block's own largest entry
    (at least floor times the whole array's), so that blocks of small magnitude are checked on
    their own scale rather than on the array's."""
    a = np.asarray(a).reshape(nblocks, -1)
    b = np.asarray(b).reshape(nblocks, -1)
    scale = np.maximum(np.abs(b).max(axis=1), floor * max(np.abs(b).max(), 1e-300))
    return float((np.abs(a - b).max(axis=1) / scale).max())


@pytest.mark.parametrize("name", CASES)
def test_condense_matches_oracle(ctx, name):
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, out = case_data(name)
    say("condense", name, pb.dims())
    pl = Pipeline(ctx, pb.dims(), pb.mesh.f2e, pb.mesh.e2f)
    blk = to_dev(out["blk"])
    pl.condense(blk)
    torch.cuda.synchronize()
    Kb = pl.Kbar.cpu().numpy()
    rb = pl.rbar.cpu().numpy()
    ek, er = relerr(Kb, out["Kbar"]), relerr(rb, out["rbar"])
    ne = pb.dims()["ne"]
    bk, br = blockerr(Kb, out["Kbar"], ne), blockerr(rb, out["rbar"], ne)
    say("condense errors", ek, er, "per element", bk, br)
    assert ek < 1e-11 and er < 1e-11, (ek, er)
    assert bk < 1e-10 and br < 1e-10, (bk, br)


@pytest.mark.parametrize("name", ["c1", "elast_hex_p3", "ns_tet_p2", "ns_hex_p3"])
def test_assemble_is_exact(ctx, name):
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, out = case_data(name)
    say("assemble", name)
    pl = Pipeline(ctx, pb.dims(), pb.mesh.f2e, pb.mesh.e2f)
    pl.Kbar.copy_(torch.as_tensor(out["Kbar"]))
    pl.rbar.copy_(torch.as_tensor(out["rbar"]))
    pl.assemble()
    torch.cuda.synchronize()
    assert np.array_equal(pl.nbr.cpu().numpy(), out["nbr"])
    assert np.array_equal(pl.K64.cpu().numpy(), out["K"])
    assert np.array_equal(pl.r.cpu().numpy(), out["r"])
    assert np.array_equal(pl.K32.cpu().numpy(), out["K"].astype(np.float32))


def test_assemble_and_recover_with_face_permutation(ctx):
    """Element blocks with permuted element-local face dofs + perm == canonical result."""
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, out = case_data("poisson_quad_p3")
    say("perm")
    dims = pb.dims()
    L, PF, M, ne = dims["nlfe"], dims["npf"], dims["ncomp"], dims["ne"]
    rng = np.random.default_rng(11)
    perm = np.stack([np.stack([rng.permutation(PF) for _ in range(L)]) for _ in range(ne)])   # canonical j -> local
    # trace index map: canonical (l,m,j) -> local (l,m,perm[e,l,j])
    blk = {k: v.copy() for k, v in out["blk"].items()}
    nt = L * M * PF
    for e in range(ne):
        src = np.zeros(nt, np.int64)     # local index -> canonical index
        for l in range(L):
            for m in range(M):
                for j in range(PF):
                    src[(l * M + m) * PF + perm[e, l, j]] = (l * M + m) * PF + j
        blk["F"][e] = blk["F"][e][:, src]
        blk["G"][e] = blk["G"][e][src, :]
        blk["H"][e] = blk["H"][e][src, :]
        blk["J"][e] = blk["J"][e][np.ix_(src, src)]
        blk["rt"][e] = blk["rt"][e][src]
        csrc = np.zeros(L * PF, np.int64)
        for l in range(L):
            for j in range(PF):
                csrc[l * PF + perm[e, l, j]] = l * PF + j
        blk["Cd"][e] = blk["Cd"][e][:, :, csrc]
    pl = Pipeline(ctx, dims, pb.mesh.f2e, pb.mesh.e2f, perm=perm)
    dblk = to_dev(blk)
    pl.condense(dblk)
    pl.assemble()
    torch.cuda.synchronize()
    ek, er = relerr(pl.K64.cpu().numpy(), out["K"]), relerr(pl.r.cpu().numpy(), out["r"])
    assert ek < 1e-11 and er < 1e-11, (ek, er)
    pl.x.copy_(torch.as_tensor(out["x"]))
    ctx.recover(dims, pl.local, dblk["Minv"], dblk["Bd"], dblk["Cd"], pl.e2f, pl.perm, pl.x, pl.du, pl.dq)
    torch.cuda.synchronize()
    eu, eq = relerr(pl.du.cpu().numpy(), out["du"]), relerr(pl.dq.cpu().numpy(), out["dq"])
    assert eu < 1e-10 and eq < 1e-10, (eu, eq)


def _dev_matrix(out):
    K = torch.as_tensor(out["K"]).cuda().contiguous()
    return K, K.float().contiguous(), torch.as_tensor(out["nbr"].astype(np.int32)).cuda().contiguous()


@pytest.mark.parametrize("name", ["c1", "elast_hex_p3", "ns_hex_p2", "ns_tet_p2", "burgers_tri_p4", "ns_hex_p3"])
def test_matvec_fp64_and_fp32(ctx, name):
    pb, out = case_data(name)
    say("matvec", name)
    K, K32, nbr = _dev_matrix(out)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(out["r"].shape[0])
    xd = torch.as_tensor(x).cuda()
    y = torch.zeros_like(xd)
    ctx.matvec(pb.dims(), K, None, nbr, xd, y, "fp64")
    ref = out["A"] @ x
    assert relerr(y.cpu().numpy(), ref) < 1e-13
    ctx.matvec(pb.dims(), None, K32, nbr, xd, y, "mixed")
    # FP32 storage error bound (Higham, dot products): |y32 - y| <= gamma_n |K| |x| with u = 2^-24
    n = out["K"].shape[1] * out["K"].shape[2]
    u = 2.0 ** -24
    bound = (n * u / (1 - n * u)) * (abs(out["A"]) @ np.abs(x)) + 1e-300
    assert np.all(np.abs(y.cpu().numpy() - ref) <= bound * 1.01 + 1e-15 * np.abs(ref).max())


@pytest.mark.parametrize("name", ["c1", "elast_hex_p3", "ns_tet_p2", "ns_hex_p3"])
def test_bj_inverse_and_apply(ctx, name):
    pb, out = case_data(name)
    say("bj", name)
    K, _, nbr = _dev_matrix(out)
    nf, nb = out["K"].shape[0], out["K"].shape[2]
    B64 = torch.zeros(nf, nb, nb, dtype=torch.float64, device="cuda")
    B32 = torch.zeros(nf, nb, nb, dtype=torch.float32, device="cuda")
    ctx.bj_setup(pb.dims(), K, B64, B32)
    ref = krylov.bj_inverses(out["K"])
    assert relerr(B64.cpu().numpy(), ref) < 1e-10
    eb = blockerr(B64.cpu().numpy(), ref, nf)
    say("bj per face", eb)
    assert eb < 1e-10, eb
    assert np.array_equal(B32.cpu().numpy(), B64.cpu().numpy().astype(np.float32))
    y = torch.as_tensor(np.random.default_rng(2).standard_normal(nf * nb)).cuda()
    z = torch.zeros_like(y)
    ctx.bj_apply(pb.dims(), B64, None, y, z)
    assert relerr(z.cpu().numpy(), krylov.bj_apply(ref, y.cpu().numpy())) < 1e-10


@pytest.mark.parametrize("name", ["c1", "elast_hex_p1", "ns_tet_p2"])
def test_poly_apply_matches_product_form(ctx, name):
    pb, out = case_data(name)
    say("poly", name)
    K, K32, nbr = _dev_matrix(out)
    nf, nb = out["K"].shape[0], out["K"].shape[2]
    Binv = krylov.bj_inverses(out["K"])
    B64 = torch.as_tensor(Binv).cuda().contiguous()
    opB = lambda v: krylov.bj_apply(Binv, out["A"] @ v)
    rng = np.random.default_rng(3)
    H, _ = poly.arnoldi_mgs(opB, rng.standard_normal(nf * nb), 10)
    th, n_added = poly.pp_roots(H)
    say("  roots", len(th), "added", n_added)
    y = rng.standard_normal(nf * nb)
    ref = poly.apply_product(opB, th, krylov.bj_apply(Binv, y))
    yd = torch.as_tensor(y).cuda()
    z = torch.zeros_like(yd)
    ctx.poly_apply(pb.dims(), K, None, nbr, B64, None, th, yd, z)
    assert relerr(z.cpu().numpy(), ref) < 1e-9, relerr(z.cpu().numpy(), ref)


@pytest.mark.parametrize("orth", ORTHS)
@pytest.mark.parametrize("precision,prec", [("fp64", "bj"), ("mixed", "bj"), ("fp64", "bj_poly"),
                                            ("mixed", "bj_poly"), ("fp64", "none"), ("fp64", "bj_cheb")])
def test_gmres_solution_c1(ctx, precision, prec, orth):
    pb, out = case_data("c1")
    say("solve c1", precision, prec, orth)
    K, K32, nbr = _dev_matrix(out)
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    v0 = torch.as_tensor(np.random.default_rng(7).standard_normal(r.numel())).cuda()
    st = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, x, restart=50, max_iters=2000, rtol=1e-13, prec=prec,
                         poly_v0=v0, precision=precision, poly_degree=10, **orth_kw(orth))
    assert st["converged"], st
    tol = 1e-10 if precision == "fp64" else 1e-8
    ex = relerr(x.cpu().numpy(), out["x"])
    say("solve errors", st["iters"], ex)
    assert ex < tol, ex
    true = np.linalg.norm(out["r"] - out["A"] @ x.cpu().numpy()) / np.linalg.norm(out["r"])
    assert true <= 1e-13 * 1.01


@pytest.mark.parametrize("prec", ["bj_poly", "bj_cheb"])
def test_poly_setup_ignores_stale_hessenberg_entries(prec):
    """The polynomial setup's Hessenberg matrix is zero below the subdiagonal whatever the kept
    workspace holds: a context whose earlier solves (restart 50, then restart 4) left other values
    where the new layout's zero entries lie gives the same Ritz values and iterates as a fresh one."""
    from paper_2512_13619_amd import hdg
    pb, out = case_data("c1")
    say("stale hessenberg", prec)
    K, K32, nbr = _dev_matrix(out)
    r = torch.as_tensor(out["r"]).cuda()
    v0 = torch.as_tensor(np.random.default_rng(7).standard_normal(r.numel())).cuda()
    used = hdg.Context(0)
    for m in (50, 4):
        x = torch.zeros_like(r)
        used.gmres_solve(pb.dims(), K, K32, nbr, r, x, restart=m, max_iters=40, rtol=1e-13, prec="bj")
    res = []
    for c in (used, hdg.Context(0)):
        x = torch.zeros_like(r)
        st = c.gmres_solve(pb.dims(), K, K32, nbr, r, x, restart=7, max_iters=2000, rtol=1e-12, prec=prec,
                           poly_v0=v0, poly_degree=6)
        assert st["converged"], st
        res.append((st["theta"], x.cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])
    assert relerr(res[0][1], out["x"]) < 1e-9


@pytest.mark.parametrize("orth", ORTHS)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gmres_graph_replay_equals_direct(ctx, precision, orth):
    """A captured-and-replayed cycle gives bitwise the same iterates as direct launches."""
    pb, out = case_data("c1")
    say("graph", precision, orth)
    K, K32, nbr = _dev_matrix(out)
    r = torch.as_tensor(out["r"]).cuda()
    xa = torch.zeros_like(r)
    xb = torch.zeros_like(r)
    sa = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, xa, restart=10, max_iters=2000, rtol=1e-12,
                         precision=precision, use_graph=False, **orth_kw(orth))
    sb = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, xb, restart=10, max_iters=2000, rtol=1e-12,
                         precision=precision, use_graph=True, **orth_kw(orth))
    assert sa["converged"] and sb["converged"] and sa["iters"] == sb["iters"] and sb["cycles"] > 2
    assert torch.equal(xa, xb)
    # eager work between replays, then a second graph solve
    xc = torch.zeros_like(r)
    r2 = (r * 1.0).contiguous()
    sc = ctx.gmres_solve(pb.dims(), K, K32, nbr, r2, xc, restart=10, max_iters=2000, rtol=1e-12,
                         precision=precision, use_graph=True, **orth_kw(orth))
    assert torch.equal(xa, xc) and sc["iters"] == sa["iters"]


@pytest.mark.parametrize("orth", ORTHS)
@pytest.mark.parametrize("prec", ["bj", "bj_poly"])
def test_gmres_phase_timing_changes_nothing(ctx, prec, orth):
    """Event timing of the Arnoldi phases leaves the iterates bitwise unchanged and covers
    exactly the Arnoldi steps that ran (with delayed reorthogonalisation, also the step
    whose operator application a converged cycle leaves unused)."""
    pb, out = case_data("c1")
    say("phase timing", prec, orth)
    K, K32, nbr = _dev_matrix(out)
    r = torch.as_tensor(out["r"]).cuda()
    v0 = torch.as_tensor(np.random.default_rng(7).standard_normal(r.numel())).cuda()
    xa = torch.zeros_like(r)
    xb = torch.zeros_like(r)
    kw = dict(restart=10, max_iters=2000, rtol=1e-12, prec=prec, poly_degree=4, poly_v0=v0, precision="mixed",
              **orth_kw(orth))
    sa = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, xa, use_graph=True, **kw)
    sb = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, xb, use_graph=True, time_phases=True, **kw)
    assert sa["converged"] and sb["converged"] and torch.equal(xa, xb)
    assert sa["n_timed"] == 0 and sa["t_matvec"] == 0.0
    assert sb["iters"] == sa["iters"]
    extra = 1 if orth.startswith("dcgs2") and sb["iters"] % 10 != 0 else 0
    assert sb["n_timed"] == sb["iters"] + extra
    assert sb["t_matvec"] > 0 and sb["t_orth"] > 0
    assert sb["t_prec"] > 0 or (orth == "dcgs2+fold" and prec == "bj")
    assert sb["t_prec"] + sb["t_matvec"] + sb["t_orth"] <= sb["t_total"]


@pytest.mark.parametrize("orth", ORTHS)
def test_gmres_history_matches_oracle_fgmres(ctx, orth):
    pb, out = case_data("c1")
    K, K32, nbr = _dev_matrix(out)
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    st = ctx.gmres_solve(pb.dims(), K, None, nbr, r, x, restart=50, max_iters=500, rtol=1e-12, prec="bj",
                         hist_len=600, **orth_kw(orth))
    Binv = krylov.bj_inverses(out["K"])
    hist = []
    _, info = oracle_solver(orth)(lambda v: out["A"] @ v, out["r"], prec=lambda v: krylov.bj_apply(Binv, v),
                                  restart=50, rtol=1e-12, max_iters=500, hist=hist)
    assert abs(st["iters"] - info["iters"]) <= 1
    n = min(20, len(hist), len(st["hist"]))
    assert np.allclose(st["hist"][:n], hist[:n], rtol=1e-6)


@pytest.mark.parametrize("orth", ORTHS)
def test_gmres_long_cycle_matches_oracle(ctx, orth):
    """One restart cycle longer than 64 steps (beyond the fused CGS2 sweeps) and than 78
    (beyond the LDS staging of the Hessenberg columns in the delayed-CGS2 kernel): c1 without
    a preconditioner needs about 110 steps; restart 200 is the largest the library takes."""
    pb, out = case_data("c1")
    say("long cycle", orth)
    K, K32, nbr = _dev_matrix(out)
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    st = ctx.gmres_solve(pb.dims(), K, None, nbr, r, x, restart=200, max_iters=1000, rtol=1e-12, prec="none",
                         hist_len=300, **orth_kw(orth))
    hist = []
    _, info = oracle_solver(orth)(lambda v: out["A"] @ v, out["r"], restart=200, rtol=1e-12, max_iters=1000,
                                  hist=hist)
    assert st["converged"] and st["cycles"] == 1 and st["iters"] > 80, st
    assert abs(st["iters"] - info["iters"]) <= 1
    n = min(80, len(hist), len(st["hist"]))
    assert np.allclose(st["hist"][:n], hist[:n], rtol=1e-6)
    assert relerr(x.cpu().numpy(), out["x"]) < 1e-10


@pytest.mark.parametrize("orth", ORTHS)
def test_gmres_zero_rhs(ctx, orth):
    """b = 0 with x0 = 0: converged before the first step, x untouched."""
    pb, out = case_data("c1")
    K, K32, nbr = _dev_matrix(out)
    r = torch.zeros(out["r"].shape[0], dtype=torch.float64, device="cuda")
    x = torch.zeros_like(r)
    st = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, x, restart=20, max_iters=100, rtol=1e-10, prec="bj",
                         precision="mixed", **orth_kw(orth))
    assert st["converged"] and st["iters"] == 0, st
    assert torch.count_nonzero(x).item() == 0


def test_condense_empty_and_ragged_chunks(ctx):
    """Condensing an element range of length 0 touches nothing; condensing a ragged split of
    the elements (chunks of 3, 1 and the rest) equals condensing them all at once."""
    pb, out = case_data("elast_hex_p1")
    d = pb.dims()
    ne = d["ne"]
    M, D, P, PF, L = d["ncomp"], d["dim"], d["npe"], d["npf"], d["nlfe"]
    nu, nt = M * P, L * M * PF
    blk = to_dev(out["blk"])
    Kall = torch.empty(ne, nt, nt, dtype=torch.float64, device="cuda")
    rall = torch.empty(ne, nt, dtype=torch.float64, device="cuda")
    lall = torch.empty(ne, nu * (nu + nt + 1), dtype=torch.float64, device="cuda")
    ctx.condense(d, blk, Kall, rall, lall)
    Kc = torch.full_like(Kall, 7.0)
    rc = torch.full_like(rall, 7.0)
    lc = torch.full_like(lall, 7.0)
    ctx.condense(d, {k: v[:0] for k, v in blk.items()}, Kc[:0], rc[:0], lc[:0], ne_chunk=0)
    torch.cuda.synchronize()
    assert bool((Kc == 7.0).all()) and bool((rc == 7.0).all()) and bool((lc == 7.0).all())
    e0 = 0
    for n in (3, 1, ne - 4):
        sl = slice(e0, e0 + n)
        ctx.condense(d, {k: v[sl].contiguous() for k, v in blk.items()}, Kc[sl], rc[sl], lc[sl], ne_chunk=n)
        e0 += n
    torch.cuda.synchronize()
    assert torch.equal(Kc, Kall) and torch.equal(rc, rall) and torch.equal(lc, lall)



def test_condense_with_8_byte_aligned_blocks(ctx):
    """[D;G] blocks whose storage starts 8 bytes past a 16-byte boundary take the 8-byte staging
    form of the q-elimination and give the same bits as aligned ones."""
    pb, out = case_data("elast_hex_p1")
    d = pb.dims()
    ne = d["ne"]
    M, P, PF, L = d["ncomp"], d["npe"], d["npf"], d["nlfe"]
    nu, nt = M * P, L * M * PF
    blk = to_dev(out["blk"])
    odd = dict(blk)
    for k in ("D", "G"):
        buf = torch.empty(blk[k].numel() + 1, dtype=torch.float64, device="cuda")
        v = buf[1:].view(blk[k].shape)
        v.copy_(blk[k])
        assert v.data_ptr() % 16 == 8
        odd[k] = v
    res = []
    for b in (blk, odd):
        K = torch.empty(ne, nt, nt, dtype=torch.float64, device="cuda")
        r = torch.empty(ne, nt, dtype=torch.float64, device="cuda")
        lo = torch.empty(ne, nu * (nu + nt + 1), dtype=torch.float64, device="cuda")
        ctx.condense(d, b, K, r, lo)
        res.append((K, r, lo))
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(*res))
    assert relerr(res[1][0].cpu().numpy(), out["Kbar"]) < 1e-11

@pytest.mark.parametrize("name", ["c1", "elast_hex_p3", "ns_hex_p2", "ns_tet_p2", "ns_hex_p3"])
def test_pipeline_end_to_end(ctx, name):
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, out = case_data(name)
    say("e2e", name)
    pl = Pipeline(ctx, pb.dims(), pb.mesh.f2e, pb.mesh.e2f)
    blk = to_dev(out["blk"])
    pl.condense(blk)
    pl.assemble()
    st = pl.solve(restart=50, max_iters=3000, rtol=1e-13, prec="bj")
    assert st["converged"], st
    pl.recover(blk["Minv"], blk["Bd"], blk["Cd"])
    torch.cuda.synchronize()
    ex = relerr(pl.x.cpu().numpy(), out["x"])
    eu, eq = relerr(pl.du.cpu().numpy(), out["du"]), relerr(pl.dq.cpu().numpy(), out["dq"])
    d = pb.dims()
    # the solve stops on a residual relative to the whole right-hand side, so a face whose trace
    # values are near zero (a homogeneous boundary) carries an error on the global scale: faces
    # are held to their own scale down to 1e-3 of the largest trace value
    bx = blockerr(pl.x.cpu().numpy(), out["x"], d["nf"], floor=1e-3)
    bu, bq = blockerr(pl.du.cpu().numpy(), out["du"], d["ne"]), blockerr(pl.dq.cpu().numpy(), out["dq"], d["ne"])
    say("e2e errors", st["iters"], ex, eu, eq, "per face / element", bx, bu, bq)
    assert ex < 1e-10 and eu < 1e-10 and eq < 1e-10, (ex, eu, eq)
    assert bx < 1e-9 and bu < 1e-9 and bq < 1e-9, (bx, bu, bq)
    # Newton update of the trace state (alpha = 1 for a single linearisation)
    state = torch.zeros_like(pl.x)
    ctx.newton_update(1.0, pl.x, state)
    torch.cuda.synchronize()
    assert torch.equal(state, pl.x)



@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_folded_solve_large_blocks(ctx, precision):
    """80x80 face blocks: the tile-by-tile fold of the block-Jacobi inverses (from LDS-kernel
    inverses) into the operator, solved with delayed CGS2, against the oracle's direct solution."""
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, out = case_data("ns_hex_p3")
    say("fold large", precision)
    pl = Pipeline(ctx, pb.dims(), pb.mesh.f2e, pb.mesh.e2f)
    pl.condense(to_dev(out["blk"]))
    pl.assemble()
    st = pl.solve(restart=50, max_iters=3000, rtol=1e-12, prec="bj", orth="dcgs2", fold_prec=True,
                  precision=precision)
    assert st["converged"], st
    assert relerr(pl.x.cpu().numpy(), out["x"]) < 1e-9

def test_failure_paths(ctx):
    from paper_2512_13619_amd import hdg
    from paper_2512_13619_amd.pipeline import Pipeline
    pb, out = case_data("c1")
    say("failures")
    blk = {k: v.copy() for k, v in out["blk"].items()}
    blk["E"][5] = 0.0
    blk["D"][5] = 0.0
    pl = Pipeline(ctx, pb.dims(), pb.mesh.f2e, pb.mesh.e2f)
    with pytest.raises(hdg.HdgError) as ei:
        pl.condense(to_dev(blk))
    assert ei.value.status == -3 and "element 5" in str(ei.value)
    K, K32, nbr = _dev_matrix(out)
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    st = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, x, max_iters=1, rtol=1e-13)
    assert st["status"] == 1 and st["iters"] == 1 and not st["converged"]
    rn = r.clone()
    rn[3] = float("nan")
    with pytest.raises(hdg.HdgError) as ei:
        ctx.gmres_solve(pb.dims(), K, K32, nbr, rn, x)
    assert ei.value.status == -4
    with pytest.raises(hdg.HdgError) as ei:
        ctx.gmres_solve(pb.dims(), K, None, nbr, r, x, precision="mixed")
    assert ei.value.status == -1


def _oracle_theta(out, v0, P):
    """Leja-ordered harmonic Ritz values of one MGS Arnoldi(P) cycle on B = M^{-1} K (block-Jacobi M)
    started at v0 (Section 4.7), computed by the oracle."""
    Binv = krylov.bj_inverses(out["K"])
    opB = lambda v: krylov.bj_apply(Binv, out["A"] @ v)
    H, _ = poly.arnoldi_mgs(opB, v0, P)
    return Binv, opB, poly.leja_order(poly.harmonic_ritz(H))


@pytest.mark.parametrize("name", ["c1", "elast_hex_p1", "ns_tet_p2"])
def test_poly_setup_theta_matches_oracle(ctx, name):
    """The roots a BJ-PP(10) solve uses (its device MGS Arnoldi on B = M^{-1}K; harmonic Ritz values,
    the added copies of the outermost one and Leja order on the host) against the oracle's from the
    same start vector, value by value in the same order, with the added-root flag set exactly when
    the oracle adds copies; and the solve's Chebyshev interval against the reading's formula on the
    oracle's harmonic Ritz values."""
    pb, out = case_data(name)
    say("theta", name)
    K, K32, nbr = _dev_matrix(out)
    N = out["r"].shape[0]
    v0 = np.random.default_rng(7).standard_normal(N)
    Binv, opB, th = _oracle_theta(out, v0, 10)
    H, _ = poly.arnoldi_mgs(opB, v0, 10)
    roots, n_added = poly.pp_roots(H)
    r = torch.as_tensor(out["r"]).cuda()
    v0d = torch.as_tensor(v0).cuda()
    x = torch.zeros_like(r)
    st = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, x, restart=30, max_iters=2000, rtol=1e-12, prec="bj_poly",
                         poly_v0=v0d, poly_degree=10, precision="fp64")
    from paper_2512_13619_amd import hdg
    assert st["converged"] and st["fallback_flags"] == (hdg.FALLBACK["pp_added_root"] if n_added else 0), st
    scale = np.abs(roots).max()
    say("theta errors", len(roots), n_added, np.abs(st["theta"] - roots).max() / scale)
    assert st["theta"].shape == roots.shape
    assert np.abs(st["theta"] - roots).max() <= 1e-9 * scale
    # Chebyshev interval: beta = 1.05 max Re theta, alpha = max(min Re theta, beta / 1000)
    x.zero_()
    st = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, x, restart=30, max_iters=2000, rtol=1e-12, prec="bj_cheb",
                         poly_v0=v0d, poly_degree=10, precision="fp64")
    beta = 1.05 * th.real.max()
    alpha = max(th.real.min(), beta / 1000)
    assert st["converged"], st
    assert abs(st["cheb_beta"] - beta) <= 1e-9 * beta and abs(st["cheb_alpha"] - alpha) <= 1e-9 * beta


@pytest.mark.parametrize("name", ["c1", "elast_hex_p1", "ns_tet_p2"])
@pytest.mark.parametrize("degree", [1, 2, 10])
def test_cheb_apply_matches_oracle(ctx, name, degree):
    """The Chebyshev preconditioner's apply (fused face-operator steps) entry by entry against the
    oracle's Chebyshev acceleration (Saad, Algorithm 12.1) on B = M^{-1}K applied to M^{-1}y, over the
    interval the solve would take from the oracle's Ritz values."""
    pb, out = case_data(name)
    say("cheb apply", name, degree)
    K, K32, nbr = _dev_matrix(out)
    N = out["r"].shape[0]
    rng = np.random.default_rng(9)
    Binv, opB, th = _oracle_theta(out, rng.standard_normal(N), 10)
    beta = 1.05 * th.real.max()
    alpha = max(th.real.min(), beta / 1000)
    y = rng.standard_normal(N)
    ref = poly.chebyshev(opB, krylov.bj_apply(Binv, y), alpha, beta, degree)
    B64 = torch.as_tensor(Binv).cuda().contiguous()
    yd = torch.as_tensor(y).cuda()
    z = torch.zeros_like(yd)
    ctx.cheb_apply(pb.dims(), K, None, nbr, B64, None, degree, alpha, beta, yd, z)
    e = relerr(z.cpu().numpy(), ref)
    say("cheb errors", e)
    assert e < 1e-10, e
    # mixed: FP32 blocks and inverses, FP64 vectors -- within a few FP32 rounding units
    z32 = torch.zeros_like(yd)
    ctx.cheb_apply(pb.dims(), None, K32, nbr, None, B64.float().contiguous(), degree, alpha, beta, yd, z32,
                   precision="mixed")
    assert relerr(z32.cpu().numpy(), ref) < 1e-4


def test_cheb_apply_rejects_bad_interval(ctx):
    from paper_2512_13619_amd import hdg
    pb, out = case_data("c1")
    K, K32, nbr = _dev_matrix(out)
    B64 = torch.as_tensor(krylov.bj_inverses(out["K"])).cuda().contiguous()
    y = torch.ones(out["r"].shape[0], dtype=torch.float64, device="cuda")
    z = torch.zeros_like(y)
    for a, b, deg in ((0.0, 1.0, 3), (2.0, 1.0, 3), (0.5, 1.0, 0), (0.5, 1.0, 65)):
        with pytest.raises(hdg.HdgError) as ei:
            ctx.cheb_apply(pb.dims(), K, None, nbr, B64, None, deg, a, b, y, z)
        assert ei.value.status == -1
    assert torch.count_nonzero(z).item() == 0


@pytest.mark.parametrize("orth", ["cgs2", "dcgs2"])
def test_mixed_refinement_stagnation_switches_to_fp64(ctx, orth):
    """The mixed path's safeguard, forced from the host: an FP32 matrix that is not K's rounding (its
    off-diagonal blocks scaled by 1.6) makes every inner cycle converge on the wrong operator, so the
    true FP64 residual stalls; the solve switches its remaining cycles to the FP64 blocks, sets
    HDG_FALLBACK_MIXED_TO_FP64 and still reaches the oracle's solution."""
    from paper_2512_13619_amd import hdg
    pb, out = case_data("c1")
    say("mixed fallback", orth)
    K, K32, nbr = _dev_matrix(out)
    bad = K.clone()
    bad[:, 1:] *= 1.6
    bad32 = bad.float().contiguous()
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    st = ctx.gmres_solve(pb.dims(), K, bad32, nbr, r, x, restart=20, max_iters=4000, rtol=1e-13, prec="bj",
                         precision="mixed", **orth_kw(orth))
    say("  ", st["iters"], st["cycles"], st["fallback_flags"], st["fp64_cycles"])
    assert st["converged"] and st["fallback_flags"] & hdg.FALLBACK["mixed_to_fp64"], st
    assert 0 < st["fp64_cycles"] < st["cycles"]
    assert relerr(x.cpu().numpy(), out["x"]) < 1e-10
    # the proper FP32 rounding never triggers it
    x.zero_()
    st = ctx.gmres_solve(pb.dims(), K, K32, nbr, r, x, restart=20, max_iters=4000, rtol=1e-13, prec="bj",
                         precision="mixed", **orth_kw(orth))
    assert st["converged"] and st["fallback_flags"] == 0 and st["fp64_cycles"] == 0, st


@pytest.mark.parametrize("prec", ["bj_poly", "bj_cheb"])
def test_poly_breakdown_falls_back_to_block_jacobi(ctx, prec):
    """The polynomial setup's safeguard, forced from the host: with the off-diagonal blocks zeroed,
    B = M^{-1}K is the identity, so the setup's Arnoldi breaks down at its first step; the solve
    flags the breakdown, runs with block-Jacobi alone, and converges in one step."""
    from paper_2512_13619_amd import hdg
    pb, out = case_data("c1")
    K, K32, nbr = _dev_matrix(out)
    Kd = K.clone()
    Kd[:, 1:] = 0.0
    r = torch.as_tensor(out["r"]).cuda()
    x = torch.zeros_like(r)
    v0 = torch.as_tensor(np.random.default_rng(7).standard_normal(r.numel())).cuda()
    st = ctx.gmres_solve(pb.dims(), Kd, Kd.float().contiguous(), nbr, r, x, restart=20, max_iters=100, rtol=1e-12,
                         prec=prec, poly_v0=v0, poly_degree=10)
    f = st["fallback_flags"]
    assert f & hdg.FALLBACK["pp_breakdown"] and f & hdg.FALLBACK["pp_to_base"], st
    assert st["converged"] and st["iters"] == 1, st
    Binv = krylov.bj_inverses(Kd.cpu().numpy())
    assert relerr(x.cpu().numpy(), krylov.bj_apply(Binv, out["r"])) < 1e-12
