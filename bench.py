"""Benchmark of the HDG hot path on one MI355X.

A step is one pass of the whole hot path over the resident element blocks of the
3D linear-elasticity workload (unit cube, 24^3 hexes jittered +-0.05h, p=3,
16 dofs/face x 3 components, 288x288 element Schur blocks):
  condensation -> face assembly -> GMRES(50)+block-Jacobi to rtol 1e-8 -> recovery
(delayed CGS2 Arnoldi by default; --orth cgs2 runs the flexible form with CGS2).
The headline value is the mixed-precision step (FP32 matrix and block inverses in
the Krylov cycles, FP64 residual/Arnoldi/Givens/update); the FP64 step, the solve
times and the block-matvec and block-Jacobi bandwidths are reported next to it. The
kernel rates come from HIP events that the library records on its own stream
around every matvec, preconditioner and orthogonalisation of the timed solves.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
METRIC = "time-to-1e-8 solve + block-matvec HBM GB/s, mixed-precision vs FP64, 1 GPU"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def gen_blocks(pb, chunk=256):
    import torch
    d = pb.dims()
    ne = d["ne"]
    M, D, P, PF, L = d["ncomp"], d["dim"], d["npe"], d["npf"], d["nlfe"]
    nu, nq, nt = M * P, M * D * P, L * M * PF
    shapes = dict(Minv=(P, P), Bd=(D, P, P), Cd=(D, P, L * PF), D=(nu, nq), E=(nu, nu), F=(nu, nt), G=(nt, nq),
                  H=(nt, nu), J=(nt, nt), ru=(nu,), rt=(nt,))
    blk = {k: torch.empty((ne,) + s, dtype=torch.float64, device="cuda") for k, s in shapes.items()}
    for e0 in range(0, ne, chunk):
        e1 = min(ne, e0 + chunk)
        b = pb.element_blocks(e0, e1)
        for k in blk:
            blk[k][e0:e1].copy_(b[k])
        del b
    torch.cuda.synchronize()
    return blk


def matvec_bytes(nbr_np, nb, wbytes):
    """Algorithmic bytes of one block matvec: non-empty K blocks, nbr, x once, y once."""
    import numpy as np
    nf, S = nbr_np.shape
    nblocks = int((nbr_np >= 0).sum())
    return nblocks * nb * nb * wbytes + nf * S * 4 + 2 * nf * nb * 8


def condense_flops(d):
    """Algorithmic FP64 flops of condensing one element: W = M^-1 [B_d | C_d] (each d), the
    q-elimination product per component, LU of Ebar, the two triangular solves with the nt+1
    right-hand sides [Fbar | r_u], and the Schur product Hbar (Ebar^-1 [Fbar | r_u])."""
    M, D, P, PF, L = d["ncomp"], d["dim"], d["npe"], d["npf"], d["nlfe"]
    nu, nt = M * P, L * M * PF
    R, NW = nu + nt, P + L * PF
    return (2 * D * P * P * NW + 2 * M * R * D * P * NW + 2 * nu ** 3 / 3 + 2 * nu * nu * (nt + 1)
            + 2 * nt * nu * (nt + 1))


# The single-mesh workloads bench.py runs (--config): the default is the headline. tag names the
# workload in the profiles/ records; prec is the preconditioner the workload states.
WORKLOADS = {
    "c2": dict(tag="elasticity24_p3", prec="bj",
               text="3D linear elasticity E=1 nu=0.3, unit cube {n}^3 hexes jitter 0.05h, p={p}, tau=1"),
    "c3": dict(tag="ns_hex16_p2", prec="bj_cheb",
               text="3D compressible Navier-Stokes linearisation Re=1000 Mach 0.5, unit cube {n}^3 hexes, p={p}, "
                    "freestream + 5% Gaussian bumps, backward Euler dt=10h/((p+1)(|v|+c))"),
    "c5": dict(tag="ns_tet32_p2", prec="bj_poly",
               text="3D compressible Navier-Stokes linearisation Re=1000 Mach 0.5, unit cube {n}^3 x 6 Kuhn tets "
                    "jitter 0.1h, p={p}, freestream + 5% Gaussian bumps, backward Euler dt=10h/((p+1)(|v|+c))"),
}
WORKLOAD_SIZES = {"c2": (24, 3), "c3": (16, 2), "c5": (32, 2)}
PREC_TEXT = {"bj": "block-Jacobi", "bj_poly": "block-Jacobi + Ritz-Leja polynomial(10)",
             "bj_cheb": "block-Jacobi + Chebyshev(10)", "asm": "element ASM", "asm_poly": "ASM + polynomial(10)",
             "asm_cheb": "ASM + Chebyshev(10)", "none": "no preconditioner"}


def fp32_matvec_kernel(tuned, nb, S):
    """Name of the FP32 block-matvec kernel instance the timed solves launched: the measured
    configuration (threads per face, rows per thread) when the autotuner ran."""
    if tuned:
        for k, v in tuned["table"].items():
            if k.startswith(f"face:m32:p32:m20:k0:nb{nb}:S{S}:"):
                return f"k_face_op<float,float,{v[0]},false,0,{v[1]}> (FP32 block matvec, measured configuration)"
    return "k_face_op<float,float,TEAM,false,0,VEC> (FP32 block matvec, built-in configuration rule)"


def measured_traffic(kernel, tag):
    """Counter-measured HBM bytes per launch of a face-operator kernel instance (the profiles/
    record face_operator_counters_<tag>.json, FETCH_SIZE and WRITE_SIZE calibrated on a device
    copy), or None when the record has no entry for it or the kernel source changed since the
    counters were taken."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", f"face_operator_counters_{tag}.json")
    try:
        rec = json.load(open(rec_path))
        src = open(os.path.join(ROOT, rec["kernel_source"]), "rb").read()
    except Exception:
        return None
    if hashlib.sha256(src).hexdigest() != rec["kernel_source_sha256"]:
        return None
    k = rec["kernels"].get(kernel.split(" ")[0])
    return k["traffic_bytes"] if k else None


def time_matvec(ctx, pl, precision, reps=100):
    import torch
    x = torch.randn(pl.x.numel(), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    K64 = pl.K64 if precision == "fp64" else None
    K32 = pl.K32 if precision == "mixed" else None
    for _ in range(3):
        ctx.matvec(pl.dims, K64, K32, pl.nbr, x, y, precision)
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        ctx.matvec(pl.dims, K64, K32, pl.nbr, x, y, precision)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def cpu_baseline(pb, blk, pl, iters, budget_s=20.0):
    """The FP64 oracle timed on the host on a bounded sample of the same workload."""
    import numpy as np
    import torch
    import oracle
    from oracle import krylov
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    d = pb.dims()
    ne, nf = d["ne"], d["nf"]
    nb = d["ncomp"] * d["npf"]
    # condensation: dense solve per element
    def sample(n):
        return {k: v[:n].cpu().numpy() for k, v in blk.items()}
    s = sample(2)
    t = time.perf_counter()
    oracle.condense.condense(s, d)
    t_el = (time.perf_counter() - t) / 2
    n_el = int(max(2, min(ne, (0.5 * budget_s) / max(t_el, 1e-6))))
    s = sample(n_el)
    t = time.perf_counter()
    oracle.condense.condense(s, d)
    t_el = (time.perf_counter() - t) / n_el
    # recovery costs the same dense solve per element
    s1 = {k: v[:2] for k, v in s.items()}
    t = time.perf_counter()
    oracle.condense.recover(s1, np.zeros(nf * nb), pb.mesh.e2f, d, elems=[0, 1])
    t_rec = (time.perf_counter() - t) / 2
    # one FGMRES iteration: CSR matvec (sampled face rows, scaled), block-Jacobi, CGS2 at j = 25
    nfs = min(nf, 2000)
    K = pl.K64[:nfs].cpu().numpy()
    nbr = pl.nbr[:nfs].cpu().numpy().astype(np.int64)
    A = oracle.assemble.to_sparse(K, nbr, n_col_faces=nf)
    x = np.random.default_rng(0).standard_normal(nf * nb)
    t = time.perf_counter()
    for _ in range(5):
        A @ x
    t_mv = (time.perf_counter() - t) / 5 * nf / nfs
    Binv = krylov.bj_inverses(K[:200])
    t = time.perf_counter()
    krylov.bj_apply(Binv, x[:200 * nb])
    t_bj = (time.perf_counter() - t) * nf / 200
    V = np.random.default_rng(1).standard_normal((26, nf * nb))
    t = time.perf_counter()
    krylov._orth(V, x.copy(), 24, "cgs2")
    t_orth = time.perf_counter() - t
    t_iter = t_mv + t_bj + t_orth
    total = ne * (t_el + t_rec) + iters * t_iter
    return {"value": total, "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": (f"dense-solve condensation of {n_el} elements ({t_el * 1e3:.2f} ms/element) and recovery "
                       f"of 2 elements scaled to {ne}; one FGMRES iteration = CSR matvec on {nfs} face rows "
                       f"scaled to {nf} ({t_mv:.3f} s) + block-Jacobi on 200 faces scaled ({t_bj:.3f} s) + CGS2 at "
                       f"j=25 ({t_orth:.3f} s), times the GPU's {iters} iterations; FP64 numpy/scipy")}


def second_stage(args, pl, blk, d, stream):
    """A DIRK-type second stage: the same matrix with new element right-hand sides. The first
    stage is condensed keeping its factors (untimed, with assembly and a solve that sets up
    block-Jacobi); the timed stage recondenses the right-hand side only, assembles r, solves
    reusing the block-Jacobi inverses and folded blocks, and recovers."""
    import numpy as np
    import torch
    pl.condense(blk, keep=True)
    pl.assemble()
    kw = dict(restart=50, max_iters=20000, rtol=1e-8, prec="bj", orth=args.orth, precision="mixed",
              fold_prec=not args.no_fold)
    st1 = pl.solve(**kw)
    rng = np.random.default_rng(31)
    ru = torch.as_tensor(rng.standard_normal((d["ne"], pl.nu))).cuda()
    rt = torch.as_tensor(rng.standard_normal((d["ne"], pl.nt))).cuda()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    ev[0].record(stream)
    pl.condense_rhs(ru, rt)
    ev[1].record(stream)
    pl.assemble_rhs()
    ev[2].record(stream)
    st2 = pl.solve(reuse_setup=True, **kw)
    ev[3].record(stream)
    pl.recover(blk["Minv"], blk["Bd"], blk["Cd"])
    ev[4].record(stream)
    torch.cuda.synchronize()
    if not st2["converged"]:
        raise RuntimeError(f"second stage did not converge: {st2}")
    ph = dict(condense_rhs=ev[0].elapsed_time(ev[1]) / 1e3, assemble_rhs=ev[1].elapsed_time(ev[2]) / 1e3,
              solve=ev[2].elapsed_time(ev[3]) / 1e3, recover=ev[3].elapsed_time(ev[4]) / 1e3)
    out = dict(stage_s=ev[0].elapsed_time(ev[4]) / 1e3, phases_s=ph, iters=st2["iters"],
               rel_resid=st2["rel_resid_true"], first_stage_iters=st1["iters"],
               note="same matrix, seeded new element right-hand sides; condensation factors kept from the "
                    "first stage, block-Jacobi inverses and folded blocks reused")
    pl.Hbar = pl.ipiv = None
    torch.cuda.empty_cache()
    log("second stage", out)
    return out


def element_bytes(d, nqv, nqf, residual_only, keep_mass=False):
    """Algorithmic HBM bytes per element of hdg_element_blocks (scalar model): the element's
    geometry and state read once, every output written once (reference tables not counted);
    with the mass matrices kept, M^-1 is read and M^-1, B_d, C_d are not written."""
    P, PF, L, D = d["npe"], d["npf"], d["nlfe"], d["dim"]
    nt = L * PF
    rd = nqv * (1 + P * D + 1) + L * nqf * (P + D + 2) + P + nt + 2 * L * 4 / 8
    wr = P + nt + D * P
    if not residual_only:
        wr += P * D * P + P * P + P * nt + nt * D * P + nt * P + nt * nt
    if keep_mass:
        rd += P * P
    elif not residual_only:
        wr += P * P + D * P * P + D * P * nt
    return 8 * (rd + wr)


def newton_bench(args):
    """Damped Newton on 2D viscous Burgers (nu = 0.01, smooth forcing) on n x n jittered quads of
    degree p: the element-block kernel timed alone, then the whole Newton loop (element blocks,
    condensation, assembly, GMRES(50) with block-Jacobi folded into the blocks and delayed CGS2
    to 1e-10, recovery, step halving) to a residual reduction of 1e-10; then two DIRK(2,2) steps of
    dt = 0.05 from the same initial state, each stage solved the same way."""
    import numpy as np
    import torch
    from paper_2512_13619_amd import hdg
    from paper_2512_13619_amd.pipeline import Pipeline
    from workloads import mesh as Mh
    from workloads import physics as Ph
    from workloads.blocks import HDGProblem

    def forcing(x):
        return (torch.sin(np.pi * x[..., 0]) * torch.sin(2 * np.pi * x[..., 1]))[..., None]
    n, p = args.newton, args.p
    pb = HDGProblem(Mh.structured_quads(n, 0.05, 6), p, Ph.Burgers(nu=0.01, forcing=forcing), device="cuda")
    d = pb.dims()
    inp = pb.newton_inputs()
    geom = {k: inp[k].contiguous() for k in ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD", "bnd")}
    geom["nqv"], geom["nqf"] = inp["nqv"], inp["nqf"]
    model = dict(nu=inp["nu"], tau=inp["tau"], beta=inp["beta"], gamma=inp["gamma"])
    ctx = hdg.Context(0)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f, keep_fp32=True)
    blk = pl.element_arrays()
    u = inp["u0"].flatten().clone()
    uh = inp["uhat0"].flatten().clone()
    stream = torch.cuda.current_stream()
    rates = {}
    ctx.element_blocks(d, geom, model, pl.e2f, u, uh, blk)
    for ro, keep in ((False, False), (True, False), (False, True), (True, True)):
        reps = 20
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            ctx.element_blocks(d, geom, model, pl.e2f, u, uh, blk, residual_only=ro, keep_mass=keep)
        ev1.record(stream)
        torch.cuda.synchronize()
        t = ev0.elapsed_time(ev1) / 1e3 / reps
        by = element_bytes(d, geom["nqv"], geom["nqf"], ro, keep) * d["ne"]
        name = ("residual_only" if ro else "blocks") + ("_kept_mass" if keep else "")
        rates[name] = dict(ms=t * 1e3, bytes=by, GBs=by / t / 1e9)
    runs = {}
    for graph in (False, True):
        u.copy_(inp["u0"].flatten())
        uh.copy_(inp["uhat0"].flatten())
        torch.cuda.synchronize()
        ts = time.perf_counter()
        hist = pl.newton(geom, model, u, uh, tol=1e-10, restart=50, max_iters=20000, rtol=1e-10, prec="bj",
                         orth="dcgs2", fold_prec=True, use_graph=graph)
        torch.cuda.synchronize()
        runs["graph" if graph else "direct"] = time.perf_counter() - ts
    t_newton = min(runs.values())
    # inexact Newton: Eisenstat-Walker forcing for the linear solves' tolerance
    u.copy_(inp["u0"].flatten())
    uh.copy_(inp["uhat0"].flatten())
    torch.cuda.synchronize()
    ts = time.perf_counter()
    hew = pl.newton(geom, model, u, uh, tol=1e-10, restart=50, max_iters=20000, rtol=1e-10, prec="bj",
                    orth="dcgs2", fold_prec=True, forcing="ew")
    torch.cuda.synchronize()
    ew = dict(s=time.perf_counter() - ts, steps=len(hew) - 1, gmres_iters=sum(x["iters"] for x in hew),
              reduction=hew[-1]["norm"] / hew[0]["norm"], alphas=[x["alpha"] for x in hew[:-1]])
    # the same with the mixed-precision linear solves (FP32 blocks, FP64 restart residuals)
    u.copy_(inp["u0"].flatten())
    uh.copy_(inp["uhat0"].flatten())
    torch.cuda.synchronize()
    ts = time.perf_counter()
    hm = pl.newton(geom, model, u, uh, tol=1e-10, restart=50, max_iters=20000, rtol=1e-10, prec="bj",
                   orth="dcgs2", fold_prec=True, forcing="ew", precision="mixed")
    torch.cuda.synchronize()
    ew["mixed"] = dict(s=time.perf_counter() - ts, steps=len(hm) - 1, gmres_iters=sum(x["iters"] for x in hm),
                       reduction=hm[-1]["norm"] / hm[0]["norm"])
    # the exact-tolerance Newton loop with ILU-ASM on 2-element patches, refactorised per step
    u.copy_(inp["u0"].flatten())
    uh.copy_(inp["uhat0"].flatten())
    torch.cuda.synchronize()
    ts = time.perf_counter()
    hi = pl.newton(geom, model, u, uh, tol=1e-10, restart=50, max_iters=20000, rtol=1e-10, prec="ilu_asm",
                   ilu_patch=2, orth="dcgs2")
    torch.cuda.synchronize()
    ilu = dict(s=time.perf_counter() - ts, steps=len(hi) - 1, gmres_iters=sum(x["iters"] for x in hi),
               reduction=hi[-1]["norm"] / hi[0]["norm"])
    # two DIRK(2,2) steps of dt = 0.05 from the initial state (a few Newton steps per stage)
    u.copy_(inp["u0"].flatten())
    uh.copy_(inp["uhat0"].flatten())
    torch.cuda.synchronize()
    ts = time.perf_counter()
    dh = pl.dirk(geom, model, u, uh, 0.05, 2, "dirk22", tol=1e-10, restart=50, max_iters=20000, rtol=1e-10,
                 prec="bj", orth="dcgs2", fold_prec=True)
    torch.cuda.synchronize()
    t_dirk = time.perf_counter() - ts
    dirk = dict(scheme="dirk22", dt=0.05, steps=2, s=t_dirk,
                stages=[dict(newton_steps=len(h) - 1, gmres_iters=sum(x["iters"] for x in h),
                             alphas=[x["alpha"] for x in h[:-1]]) for h in dh])
    # the same steps keeping the linearisation across Newton steps and stages (chord Newton with
    # refresh): residual-only element evaluations, right-hand-side condensation with the kept
    # factors and the kept block-Jacobi setup
    u.copy_(inp["u0"].flatten())
    uh.copy_(inp["uhat0"].flatten())
    torch.cuda.synchronize()
    ts = time.perf_counter()
    dc = pl.dirk(geom, model, u, uh, 0.05, 2, "dirk22", tol=1e-10, max_steps=60, restart=50, max_iters=20000,
                 rtol=1e-10, prec="bj", orth="dcgs2", fold_prec=True, reuse="chord")
    torch.cuda.synchronize()
    dirk["chord_reuse"] = dict(s=time.perf_counter() - ts,
                               stages=[dict(newton_steps=len(h) - 1, fresh=sum(x["fresh"] for x in h[:-1]),
                                            gmres_iters=sum(x["iters"] for x in h)) for h in dc])
    print(json.dumps({"profile": "newton", "workload": f"2D viscous Burgers nu=0.01, {n}x{n} quads jitter 0.05, "
                      f"p={p}", "dims": d, "nqv": geom["nqv"], "nqf": geom["nqf"], "element_kernel": rates,
                      "newton_s": t_newton, "newton_s_by_launch": runs, "newton_inexact_ew": ew,
                      "newton_ilu_asm_G2": ilu, "dirk": dirk,
                      "steps": len(hist) - 1, "gmres_iters": sum(x["iters"] for x in hist),
                      "history": [dict(norm=h["norm"], alpha=h["alpha"], iters=h["iters"]) for h in hist]}),
          flush=True)


def newton_batch_bench(args):
    """Damped Newton on the 512-instance Poisson/Burgers workload (seeded instance draws: element
    type, n in 4..32, p in 1..4, PDE, forcing), all instances in one batch: per-instance element
    blocks, condensation, assembly, block-Jacobi FGMRES to 1e-10, recovery, step halving, each
    instance stopping at a residual reduction of 1e-10."""
    import numpy as np
    import torch
    from paper_2512_13619_amd import hdg
    from paper_2512_13619_amd.pipeline import BatchPipeline
    from workloads import configs

    t0 = time.perf_counter()
    pbs = [configs.c4_instance(i, device="cuda") for i in range(args.newton_batch)]
    inps = [pb.newton_inputs() for pb in pbs]
    keys = ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD", "bnd")
    geom = {k: torch.cat([inp[k].reshape(-1) for inp in inps]).contiguous() for k in keys}
    u0 = torch.cat([inp["u0"].reshape(-1) for inp in inps]).contiguous()
    uh0 = torch.cat([inp["uhat0"].reshape(-1) for inp in inps]).contiguous()
    models = [dict(nu=inp["nu"], tau=inp["tau"], beta=inp["beta"], gamma=inp["gamma"]) for inp in inps]
    nqv, nqf = [inp["nqv"] for inp in inps], [inp["nqf"] for inp in inps]
    ctx = hdg.Context(0)
    bp = BatchPipeline(ctx, [pb.dims() for pb in pbs], [pb.mesh.f2e for pb in pbs], [pb.mesh.e2f for pb in pbs])
    log(f"batch of {len(pbs)} instances, {sum(pb.mesh.ne for pb in pbs)} elements, "
        f"{bp.bt.total('vec')} trace dofs ({time.perf_counter() - t0:.1f} s to generate)")
    blk = bp.element_arrays()
    bp.bt.element_blocks(nqv, nqf, geom, models, bp.e2f, u0, uh0, blk)
    reps = 10
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        bp.bt.element_blocks(nqv, nqf, geom, models, bp.e2f, u0, uh0, blk)
    ev1.record()
    torch.cuda.synchronize()
    t_blk = ev0.elapsed_time(ev1) / 1e3 / reps
    runs = []
    for _ in range(2):
        u, uh = u0.clone(), uh0.clone()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        hists = bp.newton(nqv, nqf, geom, models, u, uh, tol=1e-10, max_steps=30, restart=30, max_iters=5000,
                          rtol=1e-10, prec="bj", use_graph=True)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - ts)
    # pseudo-transient continuation (backward Euler in pseudo-time, SER growth of dtau)
    u, uh = u0.clone(), uh0.clone()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ph = bp.pseudo_transient(nqv, nqf, geom, models, u, uh, 0.05, tol=1e-10, max_steps=200, restart=30,
                             max_iters=5000, rtol=1e-10, prec="bj", use_graph=True)
    torch.cuda.synchronize()
    t_ptc = time.perf_counter() - ts
    ptc_steps = [len(h) - 1 for h in ph]
    ptc = dict(dtau0=0.05, linear_rtol=1e-10, s=t_ptc,
               converged=int(sum(h[-1]["norm"] <= 1e-10 * h[0]["norm"] for h in ph)),
               steps_max=max(ptc_steps), steps_mean=float(np.mean(ptc_steps)))
    # the same with looser linear solves (each pseudo-step is only a step towards the steady state)
    u, uh = u0.clone(), uh0.clone()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ph6 = bp.pseudo_transient(nqv, nqf, geom, models, u, uh, 0.05, tol=1e-10, max_steps=200, restart=30,
                              max_iters=5000, rtol=1e-6, prec="bj", use_graph=True)
    torch.cuda.synchronize()
    st6 = [len(h) - 1 for h in ph6]
    ptc_loose = dict(dtau0=0.05, linear_rtol=1e-6, s=time.perf_counter() - ts,
                     converged=int(sum(h[-1]["norm"] <= 1e-10 * h[0]["norm"] for h in ph6)),
                     steps_max=max(st6), steps_mean=float(np.mean(st6)))
    # two DIRK(2,2) steps of dt = 0.05 for every instance (damped Newton per stage)
    u, uh = u0.clone(), uh0.clone()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    dst = bp.dirk(nqv, nqf, geom, models, u, uh, 0.05, 2, "dirk22", tol=1e-10, max_steps=30, restart=30,
                  max_iters=5000, rtol=1e-10, prec="bj", use_graph=True)
    torch.cuda.synchronize()
    dirk = dict(scheme="dirk22", dt=0.05, steps=2, s=time.perf_counter() - ts,
                stage_newton_steps_max=[max(len(h) - 1 for h in st) for st in dst],
                converged_all_stages=int(sum(all(st[i][-1]["norm"] <= 1e-10 * st[i][0]["norm"] for st in dst)
                                             for i in range(len(pbs)))))
    steps = [len(h) - 1 for h in hists]
    conv = [h[-1]["norm"] <= 1e-10 * h[0]["norm"] for h in hists]
    damped = sum(1 for h in hists if any(x["alpha"] < 1.0 for x in h[:-1]))
    print(json.dumps({"profile": "newton_batch", "workload": f"{len(pbs)} seeded Poisson/Burgers instances "
                      "(quads/triangles, n 4..32, p 1..4)", "instances": len(pbs),
                      "elements": int(sum(pb.mesh.ne for pb in pbs)), "trace_dofs": bp.bt.total("vec"),
                      "element_blocks_s": t_blk, "newton_s": min(runs), "newton_runs_s": runs,
                      "converged": int(sum(conv)), "steps_max": max(steps), "steps_mean": float(np.mean(steps)),
                      "instances_damped": damped, "pseudo_transient": ptc, "pseudo_transient_loose": ptc_loose,
                      "dirk": dirk,
                      "not_converged": [dict(instance=i, etype=pbs[i].etype, ne=pbs[i].mesh.ne, p=pbs[i].p,
                                             pde=type(pbs[i].phys).__name__, steps=steps[i],
                                             reduction=hists[i][-1]["norm"] / hists[i][0]["norm"],
                                             alphas=[x["alpha"] for x in hists[i][:-1]][-8:],
                                             gmres_iters=[x["iters"] for x in hists[i][:-1]][-8:])
                                        for i in range(len(hists)) if not conv[i]],
                      "gmres_iters_per_step_max": [max((h[k]["iters"] for h in hists if k < len(h) - 1), default=0)
                                                   for k in range(max(steps))],
                      "burgers": int(sum(1 for pb in pbs if type(pb.phys).__name__ == "Burgers"))}), flush=True)


def ilu_apply_bytes(e2f, nbr, G, nb):
    """Algorithmic bytes of one ILU-ASM application: per subdomain (n faces, b off-diagonal blocks
    of K's pattern among them) the stored blocks and inverted pivots ((b + n) nb^2 doubles), their
    codes and column pointers (b + 2n + 1 int32), the face list, y gathered and the local result
    written (2 n nb doubles); then the face sum reads the local results and writes z."""
    import numpy as np
    total = 0
    N = nbr.shape[0] * nb
    for e0 in range(0, e2f.shape[0], G):
        faces = np.unique(e2f[e0:e0 + G])
        n = faces.size
        g = nbr[faces]
        b = int(np.isin(g, faces).sum()) - int((g == faces[:, None]).any(axis=1).sum())
        total += 8 * ((b + n) * nb * nb + 2 * n * nb + n * nb) + 4 * (b + 3 * n + 1)
    return total + 8 * N


def precond_bench(args):
    """One linearisation of 2D viscous Burgers on n x n quads (degree --p): the trace system solved
    with GMRES(50) + block-Jacobi, element-patch ASM and ILU-ASM on patches of G consecutive
    elements (G = 2, 4, 8) to 1e-10: setup and solve times, iterations, the preconditioner
    application's rate."""
    import numpy as np
    import torch
    from paper_2512_13619_amd import hdg
    from paper_2512_13619_amd.pipeline import Pipeline
    from workloads import mesh as Mh
    from workloads import physics as Ph
    from workloads.blocks import HDGProblem

    def forcing(x):
        return (torch.sin(np.pi * x[..., 0]) * torch.sin(2 * np.pi * x[..., 1]))[..., None]
    n, p = args.precond_compare, args.p
    pb = HDGProblem(Mh.structured_quads(n, 0.05, 6), p, Ph.Burgers(nu=0.01, forcing=forcing), device="cuda")
    d = pb.dims()
    inp = pb.newton_inputs()
    geom = {k: inp[k].contiguous() for k in ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD", "bnd")}
    geom["nqv"], geom["nqf"] = inp["nqv"], inp["nqf"]
    model = dict(nu=inp["nu"], tau=inp["tau"], beta=inp["beta"], gamma=inp["gamma"])
    ctx = hdg.Context(0)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f, keep_fp32=False)
    blk = pl.element_arrays()
    ctx.element_blocks(d, geom, model, pl.e2f, inp["u0"].flatten().contiguous(), inp["uhat0"].flatten().contiguous(),
                       blk)
    pl.condense(blk)
    pl.assemble()
    torch.cuda.synchronize()
    N = d["nf"] * d["ncomp"] * d["npf"]
    res = {}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    kw = dict(restart=50, max_iters=20000, rtol=1e-10, orth="dcgs2")
    st, t = timed(lambda: pl.solve(prec="bj", **kw))
    res["bj"] = dict(iters=st["iters"], solve_s=t)
    _, ts = timed(lambda: pl.asm_setup(fp32=False))
    st, t = timed(lambda: pl.solve(prec="asm", **kw))
    res["asm"] = dict(iters=st["iters"], setup_s=ts, solve_s=t)
    y = torch.randn(N, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(y)
    nbr_h = pl.nbr.cpu().numpy().reshape(d["nf"], -1)
    for G in (2, 4, 8):
        try:
            h, ts = timed(lambda: ctx.ilu_asm_create(d, pl.K64, pl.nbr, pl.e2f, G))
        except hdg.HdgError as e:
            res[f"ilu_asm_G{G}"] = dict(error=str(e))
            continue
        pl.x.zero_()
        st, t = timed(lambda: ctx.gmres_solve(d, pl.K64, None, pl.nbr, pl.r, pl.x, prec="ilu_asm", ilu=h, **kw))
        reps = 200
        _, ta = timed(lambda: [ctx.ilu_asm_apply(h, y, z) for _ in range(reps)])
        nbytes = ilu_apply_bytes(pb.mesh.e2f, nbr_h, G, d["ncomp"] * d["npf"])
        res[f"ilu_asm_G{G}"] = dict(iters=st["iters"], converged=bool(st["converged"]), setup_s=ts, solve_s=t,
                                    apply_ms=ta / reps * 1e3, apply_bytes=nbytes, apply_GBps=nbytes / (ta / reps) / 1e9)
        h.close()
    print(json.dumps({"profile": "preconditioners", "workload": f"2D viscous Burgers nu=0.01, {n}x{n} quads jitter "
                      f"0.05, p={p}, first linearisation", "dims": d, "trace_dofs": N, "results": res}), flush=True)


def batch_linear_bench(args):
    """The 512-instance batched workload's linear step: batched condensation (one persistent launch),
    assembly, segmented GMRES(50) + block-Jacobi to rtol 1e-8 per instance (each restart cycle replayed
    as a hipGraph) and recovery, over all instances' first linearisation; mixed precision (FP32 blocks
    and inverses inside the cycles) against FP64, each warmed up and averaged over --steps."""
    import numpy as np
    import torch
    from paper_2512_13619_amd import hdg
    from workloads import configs

    t0 = time.perf_counter()
    pbs = [configs.c4_instance(i, device="cuda") for i in range(512)]
    ctx = hdg.Context(0)
    bt = hdg.Batch(ctx, [pb.dims() for pb in pbs])
    names = ["Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt"]
    parts = {k: [] for k in names}
    for pb in pbs:
        b = pb.element_blocks()
        for k in names:
            parts[k].append(b[k].reshape(-1))
    blk = {k: torch.cat(parts[k]).contiguous() for k in names}
    del parts
    i32 = lambda arrs: torch.as_tensor(np.concatenate([a.reshape(-1) for a in arrs]).astype(np.int32)).cuda()
    f2e, e2f = i32([pb.mesh.f2e for pb in pbs]), i32([pb.mesh.e2f for pb in pbs])
    z = lambda n, dt=torch.float64: torch.zeros(n, dtype=dt, device="cuda")
    Kbar, rbar, local = z(bt.total("Kbar")), z(bt.total("rbar")), z(bt.total("local"))
    K64, K32 = z(bt.total("K")), z(bt.total("K"), torch.float32)
    nbr = torch.zeros(bt.total("nbr"), dtype=torch.int32, device="cuda")
    r, x = z(bt.total("vec")), z(bt.total("vec"))
    du, dq = z(bt.total("du")), z(bt.total("dq"))
    ne_all = sum(pb.mesh.ne for pb in pbs)
    log(f"batch of 512 instances, {ne_all} elements, {bt.total('vec')} trace dofs "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    stream = torch.cuda.current_stream()

    def step(precision):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(stream)
        bt.condense(blk, Kbar, rbar, local)
        ev[1].record(stream)
        bt.assemble(f2e, e2f, Kbar, rbar, K64, K32, nbr, r)
        ev[2].record(stream)
        x.zero_()
        st, stats = bt.gmres_solve(K64, K32, nbr, r, x, restart=50, max_iters=20000, rtol=1e-8, prec="bj",
                                   precision=precision, use_graph=True)
        ev[3].record(stream)
        bt.recover(local, blk["Minv"], blk["Bd"], blk["Cd"], e2f, x, du, dq)
        ev[4].record(stream)
        torch.cuda.synchronize()
        if st != 0 or not all(s_["converged"] for s_ in stats):
            raise RuntimeError(f"{precision} batch solve: {sum(s_['converged'] for s_ in stats)} of 512 converged")
        ph = dict(condense=ev[0].elapsed_time(ev[1]) / 1e3, assemble=ev[1].elapsed_time(ev[2]) / 1e3,
                  solve=ev[2].elapsed_time(ev[3]) / 1e3, recover=ev[3].elapsed_time(ev[4]) / 1e3)
        return stats, ph

    out = {}
    xs = {}
    for precision in ("mixed", "fp64"):
        for _ in range(max(args.warmup, 1)):
            step(precision)
        times, phs = [], []
        for _ in range(args.steps):
            t1 = time.perf_counter()
            stats, ph = step(precision)
            times.append(time.perf_counter() - t1)
            phs.append(ph)
        its = [s_["iters"] for s_ in stats]
        out[precision] = dict(step_s=float(np.mean(times)), step_s_minmax=[min(times), max(times)],
                              phases_s={k: float(np.mean([p_[k] for p_ in phs])) for k in phs[0]},
                              iters_max=max(its), iters_total=int(sum(its)),
                              rel_resid_max=max(s_["rel_resid_true"] for s_ in stats))
        xs[precision] = x.clone()
        log(precision, out[precision])
    dx = float(((xs["mixed"] - xs["fp64"]).norm() / xs["fp64"].norm()).item())
    print(json.dumps({"profile": "batch_linear", "metric": METRIC, "unit": "s", "higher_is_better": False,
                      "workload": "512 seeded 2D Poisson/Burgers instances (quads/triangles, n 4..32, p 1..4), "
                                  "first linearisation; batched condensation, assembly, segmented GMRES(50) + "
                                  "block-Jacobi to rtol 1e-8 per instance (hipGraph cycles), recovery",
                      "instances": 512, "elements": ne_all, "trace_dofs": bt.total("vec"),
                      "steps": args.steps, "warmup": max(args.warmup, 1), "mixed": out["mixed"],
                      "fp64": out["fp64"], "mixed_vs_fp64_speedup": out["fp64"]["step_s"] / out["mixed"]["step_s"],
                      "mixed_vs_fp64_solution_reldiff": dx, "tuned_grid": bt.tuned_grid()}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=["c2", "c3", "c5", "c4"],
                    help="workload: c2 the elasticity headline; c3 / c5 the Navier-Stokes linearisations on hexes / "
                         "Kuhn tets; c4 the 512-instance batched linear solve")
    ap.add_argument("--n", type=int, default=0, help="cells per direction (0: the workload's own size)")
    ap.add_argument("--p", type=int, default=0, help="degree (0: the workload's own degree)")
    ap.add_argument("--prec", default="", help="preconditioner of the timed solves (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--also", default="",
                    help="comma-separated preconditioners (asm, asm_poly, bj_poly, ...) to time in one extra "
                         "mixed-precision step each after the headline")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the measurement of the face operator's launch configurations (setup, untimed) and "
                         "use the library's built-in rule")
    ap.add_argument("--no-fold", action="store_true",
                    help="apply block-Jacobi separately in every step instead of folding it into the blocks")
    ap.add_argument("--orth", default="dcgs2", choices=["cgs2", "dcgs2", "cgs", "mgs"],
                    help="Arnoldi orthogonalisation of the solves (dcgs2: GMRES with delayed CGS2, two "
                         "sweeps over the basis per step; cgs2: flexible GMRES with three)")
    ap.add_argument("--no-stage2", action="store_true",
                    help="skip the timing of a second stage with new right-hand sides (kept condensation "
                         "factors, reused block-Jacobi setup)")
    ap.add_argument("--profile-condense", type=int, default=0,
                    help="condense the resident elements this many times (for MFMA counters), then exit")
    ap.add_argument("--profile-matvec", type=int, default=0,
                    help="build the workload's matrix, tune the face operator, run this many FP32 and FP64 block "
                         "matvecs and block-Jacobi applies, a third as many FP32 Chebyshev(10) applies, and three "
                         "1 GiB device copies (counter calibration), then exit")
    ap.add_argument("--newton", type=int, default=0,
                    help="instead of the headline: damped Newton on 2D viscous Burgers with this many quads per "
                         "direction at degree --p (element-kernel rates and the Newton loop), then exit")
    ap.add_argument("--newton-batch", type=int, default=0,
                    help="instead of the headline: damped Newton on this many instances of the batched "
                         "Poisson/Burgers workload in one batch (512: the whole workload), then exit")
    ap.add_argument("--precond-compare", type=int, default=0,
                    help="instead of the headline: one Burgers linearisation on this many quads per direction "
                         "solved with block-Jacobi, element ASM and ILU-ASM (patches of 2, 4, 8 elements), then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported (the hot path is "
              f"single-GPU; multi-GPU sharding is a design note only).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2512_13619_amd import hdg
    from paper_2512_13619_amd.pipeline import Pipeline
    from workloads import configs

    torch.cuda.set_device(0)
    if args.config != "c4":
        n0, p0 = WORKLOAD_SIZES[args.config]
        args.n = args.n or n0
        args.p = args.p or p0
    if args.newton > 0:
        newton_bench(args)
        return
    if args.newton_batch > 0:
        newton_batch_bench(args)
        return
    if args.precond_compare > 0:
        precond_bench(args)
        return
    if args.config == "c4":
        batch_linear_bench(args)
        return
    wl = WORKLOADS[args.config]
    prec_main = args.prec or wl["prec"]
    headline = args.config == "c2"
    t0 = time.perf_counter()
    pb = getattr(configs, args.config)(n=args.n, p=args.p, device="cuda")
    d = pb.dims()
    log("workload", d)
    blk = gen_blocks(pb)
    log(f"element blocks resident: {sum(v.numel() for v in blk.values()) * 8 / 1e9:.1f} GB "
        f"({time.perf_counter() - t0:.1f} s)")
    ctx = hdg.Context(0)
    pl = Pipeline(ctx, d, pb.mesh.f2e, pb.mesh.e2f)
    stream = torch.cuda.current_stream()
    if args.profile_condense > 0:
        for _ in range(args.profile_condense):
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            pl.condense(blk)
            ev1.record(stream)
            torch.cuda.synchronize()
            t = ev0.elapsed_time(ev1) / 1e3
            fl = condense_flops(d) * d["ne"]
            print(json.dumps({"profile": "condensation", "s": t, "TFLOPs": fl / t / 1e12,
                              "flops": fl}), flush=True)
        return
    if args.profile_matvec > 0:
        pl.condense(blk)
        pl.assemble()
        del blk
        torch.cuda.synchronize()
        reps = args.profile_matvec
        nb = d["ncomp"] * d["npf"]
        N = d["nf"] * nb
        B64 = torch.empty(d["nf"] * nb * nb, dtype=torch.float64, device="cuda")
        B32 = torch.empty(d["nf"] * nb * nb, dtype=torch.float32, device="cuda")
        ctx.bj_setup(pl.dims, pl.K64, B64, B32)
        tuned = None
        if not args.no_tune:      # the configuration the bench's timed solves launch
            ctx.autotune(pl.dims, pl.K64, pl.K32, pl.nbr, B64, B32, reps=10)
            tuned = dict(table=hdg.tune_table().get("entries", {}))
        t32 = time_matvec(ctx, pl, "mixed", reps)
        t64 = time_matvec(ctx, pl, "fp64", reps)
        y = torch.randn(N, dtype=torch.float64, device="cuda")
        z = torch.empty_like(y)

        def timed(fn, n):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(n):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / 1e3 / n
        tbj32 = timed(lambda: ctx.bj_apply(pl.dims, None, B32, y, z, "mixed"), reps)
        tbj64 = timed(lambda: ctx.bj_apply(pl.dims, B64, None, y, z, "fp64"), reps)
        # Chebyshev(10) on B = M^-1 K (interval [0.05, 2]): nine fused steps (block row product, block
        # inverse, three-term recurrence in the epilogue) after one block-Jacobi apply
        tch32 = timed(lambda: ctx.cheb_apply(pl.dims, None, pl.K32, pl.nbr, None, B32, 10, 0.05, 2.0, y, z, "mixed"),
                      max(1, reps // 3))
        nbr_np = pl.nbr.cpu().numpy()
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")      # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        bj_bytes = lambda w: d["nf"] * nb * nb * w + 2 * N * 8
        # one fused Chebyshev step: K's non-empty blocks, nbr, the block inverses, the gathered input
        # (read once), r and x_c read, r, d_next and x_c written
        step_bytes = matvec_bytes(nbr_np, nb, 4) - 2 * N * 8 + d["nf"] * nb * nb * 4 + 3 * N * 8 + 3 * N * 8
        print(json.dumps({"profile": "block matvec", "fp32_ms": t32 * 1e3, "fp64_ms": t64 * 1e3,
                          "fp32_bytes": matvec_bytes(nbr_np, nb, 4), "fp64_bytes": matvec_bytes(nbr_np, nb, 8),
                          "fp32_GBs": matvec_bytes(nbr_np, nb, 4) / t32 / 1e9,
                          "fp64_GBs": matvec_bytes(nbr_np, nb, 8) / t64 / 1e9,
                          "bj32_ms": tbj32 * 1e3, "bj32_bytes": bj_bytes(4), "bj32_GBs": bj_bytes(4) / tbj32 / 1e9,
                          "bj64_ms": tbj64 * 1e3, "bj64_bytes": bj_bytes(8), "bj64_GBs": bj_bytes(8) / tbj64 / 1e9,
                          "cheb32_apply_ms": tch32 * 1e3, "cheb32_step_bytes": step_bytes,
                          "copy_bytes_each_way": src.numel() * 8, "tuned": tuned}), flush=True)
        return

    v0 = torch.as_tensor(np.random.default_rng(7).standard_normal(d["nf"] * d["ncomp"] * d["npf"])).cuda()

    def step(precision, prec=prec_main):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ev[0].record(stream)
        pl.condense(blk)
        ev[1].record(stream)
        pl.assemble()
        ev[2].record(stream)
        if prec.startswith("asm"):        # additive Schwarz subdomain inverses
            pl.asm_setup(fp32=precision == "mixed")
        ev[3].record(stream)
        st = pl.solve(restart=50, max_iters=20000, rtol=1e-8, prec=prec, orth=args.orth, precision=precision,
                      time_phases=True, fold_prec=not args.no_fold, poly_degree=10, poly_v0=v0)
        ev[4].record(stream)
        pl.recover(blk["Minv"], blk["Bd"], blk["Cd"])
        ev[5].record(stream)
        torch.cuda.synchronize()
        ph = dict(condense=ev[0].elapsed_time(ev[1]) / 1e3, assemble=ev[1].elapsed_time(ev[2]) / 1e3,
                  solve=ev[3].elapsed_time(ev[4]) / 1e3, recover=ev[4].elapsed_time(ev[5]) / 1e3)
        if prec.startswith("asm"):
            ph["asm_setup"] = ev[2].elapsed_time(ev[3]) / 1e3
        if not st["converged"]:
            raise RuntimeError(f"{precision} {prec} solve did not converge: {st}")
        return st, ph

    def timed_steps(precision, warmup, steps):
        """warmup untimed steps (they also size the context's workspaces for this precision), then
        `steps` steps each timed by the host clock between device synchronisations; returns the mean
        step time, the per-step times, the last stats and the mean phase times."""
        for _ in range(warmup):
            st, ph = step(precision)
            log("warmup", precision, st["iters"], ph)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        times, phs = [], []
        for _ in range(steps):
            t1 = time.perf_counter()
            st, ph = step(precision)          # ends with a device synchronisation
            times.append(time.perf_counter() - t1)
            phs.append(ph)
        torch.cuda.synchronize()
        mean = (time.perf_counter() - ts) / max(steps, 1)
        phm = {k: float(np.mean([p[k] for p in phs])) for k in phs[0]} if phs else ph
        log(precision, "step", mean, st["iters"], phm)
        return mean, times, st, phm

    tuned = None
    if not args.no_tune:
        # setup, outside the timed region: the library measures the face operator's launch
        # configurations (threads per face, rows per thread) on this workload's assembled matrix and
        # block-Jacobi inverses, and every later launch of the process uses the fastest
        pl.condense(blk)
        pl.assemble()
        nbt = d["ncomp"] * d["npf"]
        B64 = torch.empty(d["nf"] * nbt * nbt, dtype=torch.float64, device="cuda")
        B32 = torch.empty(d["nf"] * nbt * nbt, dtype=torch.float32, device="cuda")
        ctx.bj_setup(pl.dims, pl.K64, B64, B32)
        t0t = time.perf_counter()
        ntuned = ctx.autotune(pl.dims, pl.K64, pl.K32, pl.nbr, B64, B32, reps=10)
        tuned = dict(variants=ntuned, seconds=time.perf_counter() - t0t, table=hdg.tune_table().get("entries", {}))
        del B64, B32
        log("autotune", tuned)
    t_mixed, times_mixed, st_mixed, ph_mixed = timed_steps("mixed", args.warmup, args.steps)
    x_mixed = pl.x.clone()
    t_fp64 = None
    times_fp64 = None
    st64 = None
    ph64 = None
    if not args.no_fp64:
        # the FP64 leg is warmed up and averaged like the mixed one (its warm-up also grows the
        # context's folded-block workspace to the FP64 size outside the timed region)
        t_fp64, times_fp64, st64, ph64 = timed_steps("fp64", max(1, min(args.warmup, 2)), args.steps)
        dx = float(((x_mixed - pl.x).norm() / pl.x.norm()).item())
    else:
        dx = None
    # kernel rates inside the timed solves: the library records HIP events on its own stream
    # around the preconditioner, the matvec and the orthogonalisation of every Arnoldi step
    nbr_np = pl.nbr.cpu().numpy()
    nb = d["ncomp"] * d["npf"]
    N = d["nf"] * nb
    b32 = matvec_bytes(nbr_np, nb, 4)
    b64 = matvec_bytes(nbr_np, nb, 8)
    bj32 = d["nf"] * nb * nb * 4 + 2 * N * 8
    bj64 = d["nf"] * nb * nb * 8 + 2 * N * 8

    folded = args.orth == "dcgs2" and not args.no_fold

    def rates(stt, bmv, bbj):
        n = max(stt["n_timed"], 1)
        t_mv, t_bj = stt["t_matvec"] / n, stt["t_prec"] / n
        out = dict(n_timed=stt["n_timed"], matvec_ms=t_mv * 1e3, matvec_GBs=bmv / t_mv / 1e9,
                   t_matvec_s=stt["t_matvec"], t_prec_s=stt["t_prec"], t_orth_s=stt["t_orth"])
        if prec_main == "bj":
            if not folded:    # with the inverses folded into the blocks no step applies block-Jacobi
                out.update(bj_apply_ms=t_bj * 1e3, bj_apply_GBs=bbj / t_bj / 1e9)
        elif prec_main in ("bj_poly", "bj_cheb") and t_bj > 0:
            # a degree-P polynomial applies the operator P-1 times; with block-Jacobi folded each
            # application is one block row product over the folded blocks (the matvec's bytes), else
            # a product and a block-Jacobi apply; the vector traffic of the recurrences is not counted
            P = 10
            per = bmv if folded else bmv + bbj
            pb_bytes = (P - 1) * per + (0 if folded else bbj)
            out.update(prec_apply_ms=t_bj * 1e3, prec_apply_bytes_lower=pb_bytes,
                       prec_apply_GBs_lower=pb_bytes / t_bj / 1e9, npoly=stt.get("npoly"),
                       fallback_flags=stt.get("fallback_flags"))
        return out
    r32 = rates(st_mixed, b32, bj32)
    r64 = rates(st64, b64, bj64) if st64 else None
    log("in-solve rates mixed", r32)
    log("in-solve rates fp64", r64)
    bj_loop = None
    if folded and prec_main == "bj":
        # the block-Jacobi apply (once per cycle when folded) in a loop of its own
        B64 = torch.empty(d["nf"] * nb * nb, dtype=torch.float64, device="cuda")
        B32 = torch.empty(d["nf"] * nb * nb, dtype=torch.float32, device="cuda")
        ctx.bj_setup(pl.dims, pl.K64, B64, B32)
        y = torch.randn(N, dtype=torch.float64, device="cuda")
        z = torch.empty_like(y)
        for _ in range(3):
            ctx.bj_apply(pl.dims, None, B32, y, z, "mixed")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(50):
            ctx.bj_apply(pl.dims, None, B32, y, z, "mixed")
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / 50
        bj_loop = dict(fp32_ms=t * 1e3, fp32_GBs=bj32 / t / 1e9, launches=50, set_GB=bj32 / 1e9)
        del B64, B32
        log("block-Jacobi apply loop", bj_loop)
    line = {
        "metric": METRIC,
        "value": t_mixed,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 matrix/f64 vectors (mixed)",
        "data": ("synthetic (seeded jittered mesh, manufactured elasticity load)" if args.config == "c2" else
                 "synthetic (seeded mesh, seeded Gaussian-bump linearisation state)"),
        "config": {"workload": wl["text"].format(n=args.n, p=args.p) +
                               f"; {'GMRES' if args.orth == 'dcgs2' else 'FGMRES'}(50)+{PREC_TEXT[prec_main]} "
                               f"({args.orth.upper()}"
                               f"{', folded K M^-1' if folded else ''}) rtol 1e-8",
                   "ne": d["ne"], "nf": d["nf"], "ndof": d["nf"] * nb, "face_block": nb,
                   "element_schur": pl.nt},
        "solve_s_mixed": ph_mixed["solve"],
        "phases_s_mixed": ph_mixed,
        "iters_mixed": st_mixed["iters"],
        "rel_resid_mixed": st_mixed["rel_resid_true"],
        "step_s_mixed_minmax": [min(times_mixed), max(times_mixed)] if times_mixed else None,
        "step_s_fp64": t_fp64,
        "step_s_fp64_minmax": [min(times_fp64), max(times_fp64)] if times_fp64 else None,
        "steps_fp64": len(times_fp64) if times_fp64 else 0,
        "mixed_vs_fp64_speedup": (t_fp64 / t_mixed) if t_fp64 else None,
        "solve_s_fp64": ph64["solve"] if ph64 else None,
        "phases_s_fp64": ph64,
        "iters_fp64": st64["iters"] if st64 else None,
        "rel_resid_fp64": st64["rel_resid_true"] if st64 else None,
        "mixed_vs_fp64_solution_reldiff": dx,
        "condense_TFLOPs": condense_flops(d) * d["ne"] / ph_mixed["condense"] / 1e12,
        "condense_frac_fp64_peak": condense_flops(d) * d["ne"] / ph_mixed["condense"] / 1e12 / PEAK_FP64_TFLOPS,
        "kernels_mixed": r32,
        "kernels_fp64": r64,
        "bj_apply_loop": bj_loop,
        "autotune": tuned,
        "roofline": {"bound": "hbm", "achieved": r32["matvec_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": r32["matvec_GBs"] / PEAK_HBM_GBS,
                     "traffic": (measured_traffic(fp32_matvec_kernel(tuned, nb, 2 * d["nlfe"] - 1), wl["tag"])
                                 if (args.n, args.p) == WORKLOAD_SIZES[args.config] else None),
                     "kernel": fp32_matvec_kernel(tuned, nb, 2 * d["nlfe"] - 1),
                     "bytes_per_launch": b32, "launches_timed": r32["n_timed"],
                     "timing": "HIP events recorded at the start and end of each matvec kernel of the timed mixed "
                               "solves (hipExtLaunchKernelGGL on the library's stream)"},
    }
    extra = []
    for prec in [p for p in args.also.split(",") if p]:
        torch.cuda.synchronize()
        ts = time.perf_counter()
        st_x, ph_x = step("mixed", prec)
        t_x = time.perf_counter() - ts
        extra.append(dict(prec=prec, step_s=t_x, phases_s=ph_x, iters=st_x["iters"],
                          rel_resid=st_x["rel_resid_true"], t_matvec_s=st_x["t_matvec"], t_prec_s=st_x["t_prec"],
                          t_orth_s=st_x["t_orth"]))
        log("extra", extra[-1])
        if prec.startswith("asm"):
            pl.asm_inv64 = pl.asm_inv32 = None
            torch.cuda.empty_cache()
    if extra:
        line["other_preconditioners_mixed"] = extra
    if not args.no_stage2 and headline:
        line["second_stage_mixed"] = second_stage(args, pl, blk, d, stream)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pb, blk, pl, st_mixed["iters"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
