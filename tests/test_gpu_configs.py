"""GPU parity on the workload configurations.

* Reduced meshes (same physics, element type, degree, preconditioner as each
  workload): the whole GPU path against the oracle's direct solve, FP64 path to
  1e-10 and mixed path to 1e-8 relative.
* Full-size workloads (24^3 hex elasticity p=3; 16^3 hex Navier-Stokes p=2;
  32^3 x 6 tet Navier-Stokes p=2) in the launch configuration bench.py uses:
  condensation of sampled elements against the oracle's dense solves, assembled
  face rows of sampled faces against the oracle's own assembly, the residual of
  sampled rows of K x - r evaluated from the oracle's rows, and recovery of
  sampled elements against the oracle's dense recovery.
"""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle
from oracle import assemble as oasm
from oracle import condense as ocnd
from workloads import configs

from helpers import oracle_pipeline

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2512_13619_amd import hdg
    assert torch.cuda.is_available()
    return hdg.Context(0)


def relerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


REDUCED = {
    # name: (problem factory, preconditioner, poly degree)
    "c2_elasticity_3cube_p3": (lambda: configs.c2(n=3), "bj", 10),
    "c3_ns_hex_3cube_p2": (lambda: configs.c3(n=3), "bj_cheb", 10),
    "c5_ns_tet_2cube_p2": (lambda: configs.c5(n=2), "bj_poly", 10),
    "c4_burgers_tri": (lambda: configs.c4_instance(3), "bj_poly", 10),
}


@pytest.mark.parametrize("orth", ["cgs2", "dcgs2", "dcgs2+fold"])
@pytest.mark.parametrize("name", list(REDUCED))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reduced_workload_solution(ctx, name, precision, orth):
    from paper_2512_13619_amd.pipeline import Pipeline
    make, prec, P = REDUCED[name]
    pb = make()
    say("reduced", name, precision, orth, pb.dims())
    out = oracle_pipeline(pb)
    pl = Pipeline(ctx, pb.dims(), pb.mesh.f2e, pb.mesh.e2f)
    blk = {k: torch.as_tensor(v).cuda().contiguous() for k, v in out["blk"].items()}
    pl.condense(blk)
    pl.assemble()
    v0 = torch.as_tensor(np.random.default_rng(7).standard_normal(pl.x.numel())).cuda()
    st = pl.solve(restart=50, max_iters=5000, rtol=1e-13, prec=prec, poly_degree=P, poly_v0=v0,
                  precision=precision, use_graph=True, orth=orth.split("+")[0], fold_prec=orth.endswith("fold"))
    pl.recover(blk["Minv"], blk["Bd"], blk["Cd"])
    torch.cuda.synchronize()
    ex = relerr(pl.x.cpu().numpy(), out["x"])
    eu = relerr(pl.du.cpu().numpy(), out["du"])
    say("  iters", st["iters"], "err x", ex, "err u", eu)
    assert st["converged"], st
    tol = 1e-10 if precision == "fp64" else 1e-8
    assert ex < tol and eu < tol, (ex, eu)


@pytest.mark.parametrize("prec", ["asm", "asm_poly"])
@pytest.mark.parametrize("name", ["c2_elasticity_3cube_p3", "c5_ns_tet_2cube_p2"])
def test_reduced_workload_asm(ctx, name, prec):
    """The reduced workloads with the additive Schwarz preconditioners (mixed precision,
    delayed CGS2): solution against the oracle's direct solve."""
    from paper_2512_13619_amd.pipeline import Pipeline
    make, _, P = REDUCED[name]
    pb = make()
    say("reduced asm", name, prec, pb.dims())
    out = oracle_pipeline(pb)
    pl = Pipeline(ctx, pb.dims(), pb.mesh.f2e, pb.mesh.e2f)
    blk = {k: torch.as_tensor(v).cuda().contiguous() for k, v in out["blk"].items()}
    pl.condense(blk)
    pl.assemble()
    pl.asm_setup()
    v0 = torch.as_tensor(np.random.default_rng(7).standard_normal(pl.x.numel())).cuda()
    st = pl.solve(restart=50, max_iters=5000, rtol=1e-13, prec=prec, poly_degree=P, poly_v0=v0,
                  precision="mixed", orth="dcgs2")
    torch.cuda.synchronize()
    ex = relerr(pl.x.cpu().numpy(), out["x"])
    say("  iters", st["iters"], "err x", ex)
    assert st["converged"] and ex < 1e-8, (st, ex)


# ---------------------------------------------------------------------------------------------
FULL = {
    "c2": (lambda: configs.c2(device="cuda"), "bj", "mixed"),
    "c3": (lambda: configs.c3(device="cuda"), "bj_cheb", "mixed"),
    "c5": (lambda: configs.c5(device="cuda"), "bj_poly", "mixed"),
}


def _sample(n, k, rng):
    base = np.unique(np.concatenate([[0, n - 1], rng.choice(n, size=min(n, k), replace=False)]))
    return base


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", list(FULL))
def test_full_size_sampled(ctx, name):
    from paper_2512_13619_amd.pipeline import Pipeline
    make, prec, precision = FULL[name]
    pb = make()
    d = pb.dims()
    say("full", name, d)
    rng = np.random.default_rng(123)
    ne, nf = d["ne"], d["nf"]
    nb = d["ncomp"] * d["npf"]
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    samp_f = _sample(nf, 12, rng)
    e_need = set()
    for f in samp_f:
        e1, l1, e2, l2 = pb.mesh.f2e[f]
        e_need.add(int(e1))
        if e2 >= 0:
            e_need.add(int(e2))
    samp_e = np.unique(np.concatenate([_sample(ne, 12, rng), np.array(sorted(e_need))]))
    host_blk = {}
    keep = {}
    chunk = 1024
    for e0 in range(0, ne, chunk):
        e1 = min(ne, e0 + chunk)
        b = pb.element_blocks(e0, e1)
        pl.condense(b, e0, e1)
        for k in ("Minv", "Bd", "Cd"):
            keep.setdefault(k, []).append(b[k])
        sel = samp_e[(samp_e >= e0) & (samp_e < e1)]
        for e in sel:
            host_blk[int(e)] = {k: v[e - e0].cpu().numpy() for k, v in b.items()}
        del b
    keep = {k: torch.cat(v).contiguous() for k, v in keep.items()}
    torch.cuda.synchronize()
    say("  condensed")
    order = sorted(host_blk)
    hb = {k: np.stack([host_blk[e][k] for e in order]) for k in host_blk[order[0]]}
    Kb_o, rb_o = ocnd.condense(hb, d)
    idx = {e: i for i, e in enumerate(order)}
    Kb_g = pl.Kbar[torch.as_tensor(order, device="cuda")].cpu().numpy()
    ek = max(relerr(Kb_g[i], Kb_o[i]) for i in range(len(order)))
    say("  Kbar sample err", ek)
    assert ek < 1e-10, ek
    pl.assemble()
    v0 = torch.as_tensor(np.random.default_rng(7).standard_normal(pl.x.numel())).cuda()
    st = pl.solve(restart=50, max_iters=20000, rtol=1e-8, prec=prec, poly_degree=10, poly_v0=v0,
                  precision=precision, use_graph=True, orth="dcgs2", fold_prec=True)
    say("  solve", st["iters"], st["rel_resid_true"], st["t_total"])
    assert st["converged"] and st["rel_resid_true"] <= 1e-8
    pl.recover(keep["Minv"], keep["Bd"], keep["Cd"])
    torch.cuda.synchronize()
    x = pl.x.cpu().numpy()
    rn = float(pl.r.norm().item())
    K_g = pl.K64[torch.as_tensor(samp_f, device="cuda")].cpu().numpy()
    nbr_g = pl.nbr[torch.as_tensor(samp_f, device="cuda")].cpu().numpy()
    r_g = pl.r.view(nf, nb)[torch.as_tensor(samp_f, device="cuda")].cpu().numpy()
    # oracle rows of the sampled faces from its own element Schur complements (sparse by element)
    class _ByElem:
        def __init__(self, arr):
            self.arr = arr

        def __getitem__(self, key):
            return self.arr[(idx[key[0]],) + tuple(key[1:])]
    Kfull = _ByElem(Kb_o)
    rfull = _ByElem(rb_o)
    worst_k, worst_res = 0.0, 0.0
    for a, f in enumerate(samp_f):
        e1, l1, e2, l2 = pb.mesh.f2e[f]
        faces, src = oasm.slot_faces(pb.mesh.f2e, pb.mesh.e2f, f)
        assert list(nbr_g[a]) == list(faces)
        blk0 = oasm._elem_block(Kfull, e1, l1, l1, d, None)
        rv = oasm._elem_vec(rfull, e1, l1, d, None)
        rscale = np.abs(rv).max()
        if e2 >= 0:
            blk0 = blk0 + oasm._elem_block(Kfull, e2, l2, l2, d, None)
            rv2 = oasm._elem_vec(rfull, e2, l2, d, None)
            rscale = max(rscale, np.abs(rv2).max())
            rv = rv + rv2
        scale = np.abs(blk0).max()
        worst_k = max(worst_k, np.abs(K_g[a, 0].T - blk0).max() / scale)
        # the face residual sums the two elements' contributions, which nearly cancel where the
        # state is close to a steady one: its rounding is bounded relative to the contributions
        worst_k = max(worst_k, np.abs(r_g[a] - rv).max() / max(rscale, 1e-300))
        row = blk0 @ x[f * nb:(f + 1) * nb]
        for s in range(1, len(faces)):
            if src[s] is None:
                continue
            e, l = src[s]
            lr = l1 if e == e1 else l2
            B = oasm._elem_block(Kfull, e, lr, l, d, None)
            worst_k = max(worst_k, np.abs(K_g[a, s].T - B).max() / scale)
            g = faces[s]
            row = row + B @ x[g * nb:(g + 1) * nb]
        worst_res = max(worst_res, np.linalg.norm(rv - row) / rn)
    say("  face rows err", worst_k, "sampled residual rows", worst_res)
    assert worst_k < 1e-10
    # each row's residual is bounded by the global one (rtol 1e-8), up to the FP64 rounding of the rows
    assert worst_res <= 1.2e-8
    # recovery of sampled elements with the GPU trace solution
    dq_o, du_o = ocnd.recover(hb, x, pb.mesh.e2f[order], d, elems=range(len(order)))
    du_g = pl.du[torch.as_tensor(order, device="cuda")].cpu().numpy()
    dq_g = pl.dq[torch.as_tensor(order, device="cuda")].cpu().numpy()
    eu, eq = relerr(du_g, du_o), relerr(dq_g, dq_o)
    say("  recovery err", eu, eq)
    assert eu < 1e-10 and eq < 1e-10
