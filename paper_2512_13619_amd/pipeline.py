"""Device buffers and the order of the four entry points (condense -> assemble
-> solve -> recover). Allocation and sequencing only; all arithmetic runs in
libhdg.so."""
import torch

from . import hdg


class Pipeline:
    """One mesh/space: owns K (FP64 and FP32), nbr, r, x and the recovery data."""

    def __init__(self, ctx, dims, f2e, e2f, perm=None, device="cuda", keep_fp32=True):
        self.ctx = ctx
        self.dims = dict(dims)
        d = self.dims
        self.device = device
        i32 = lambda a: torch.as_tensor(a, dtype=torch.int32).contiguous().to(device)
        self.f2e = i32(f2e)
        self.e2f = i32(e2f)
        self.perm = None if perm is None else i32(perm)
        M, D, P, PF, L = d["ncomp"], d["dim"], d["npe"], d["npf"], d["nlfe"]
        self.nu, self.nq, self.nt, self.nb, self.S = M * P, M * D * P, L * M * PF, M * PF, 2 * L - 1
        ne, nf = d["ne"], d["nf"]
        z = lambda *s, dt=torch.float64: torch.zeros(*s, dtype=dt, device=device)
        self.Kbar = z(ne, self.nt, self.nt)
        self.rbar = z(ne, self.nt)
        self.local = z(ne, self.nu, self.nu + self.nt + 1)
        self.K64 = z(nf, self.S, self.nb, self.nb)
        self.K32 = z(nf, self.S, self.nb, self.nb, dt=torch.float32) if keep_fp32 else None
        self.nbr = torch.zeros(nf, self.S, dtype=torch.int32, device=device)
        self.r = z(nf * self.nb)
        self.x = z(nf * self.nb)
        self.du = z(ne, self.nu)
        self.dq = z(ne, self.nq)

    def condense(self, blk, e0=0, e1=None, keep=False):
        """Condense elements [e0, e1) from device blocks that cover exactly that range. keep=True
        also retains the factors a later right-hand side needs (condense_rhs)."""
        e1 = self.dims["ne"] if e1 is None else e1
        if not keep:
            self.ctx.condense(self.dims, blk, self.Kbar[e0:e1], self.rbar[e0:e1], self.local[e0:e1],
                              ne_chunk=e1 - e0)
            return
        if getattr(self, "Hbar", None) is None:
            ne = self.dims["ne"]
            self.Hbar = torch.zeros(ne, self.nt, self.nu, dtype=torch.float64, device=self.device)
            self.ipiv = torch.zeros(ne, self.nu, dtype=torch.int32, device=self.device)
        self.ctx.condense_keep(self.dims, blk, self.Kbar[e0:e1], self.rbar[e0:e1], self.local[e0:e1],
                               self.Hbar[e0:e1], self.ipiv[e0:e1], ne_chunk=e1 - e0)

    def condense_rhs(self, ru, rt):
        """New element right-hand sides with the kept factors (the matrices unchanged)."""
        self.ctx.condense_rhs(self.dims, self.local, self.Hbar, self.ipiv, ru, rt, self.rbar)

    def assemble_rhs(self):
        self.ctx.assemble_rhs(self.dims, self.f2e, self.perm, self.rbar, self.r)

    def assemble(self):
        self.ctx.assemble(self.dims, self.f2e, self.e2f, self.perm, self.Kbar, self.rbar, self.K64, self.K32,
                          self.nbr, self.r)

    def asm_setup(self, fp32=True):
        """Additive Schwarz inverses of the element patches (needs Kbar and K64)."""
        d = self.dims
        n = d["ne"] * self.nt * self.nt
        self.asm_inv64 = torch.empty(n, dtype=torch.float64, device=self.device)
        self.asm_inv32 = torch.empty(n, dtype=torch.float32, device=self.device) if fp32 else None
        self.ctx.asm_setup(d, self.Kbar, self.K64, self.e2f, self.asm_inv64, self.asm_inv32)
        return dict(inv64=self.asm_inv64, inv32=self.asm_inv32, f2e=self.f2e, e2f=self.e2f)

    def solve(self, **kw):
        """GMRES on the assembled system (kw as hdg.Context.gmres_solve). prec="asm*" uses the
        patches of the last asm_setup; prec="ilu_asm" without a handle factorises the current K
        on patches of kw.pop("ilu_patch", 2) consecutive elements for this solve only."""
        self.x.zero_()
        if str(kw.get("prec", "")).startswith("asm") and "asm" not in kw:
            kw["asm"] = dict(inv64=self.asm_inv64, inv32=self.asm_inv32, f2e=self.f2e, e2f=self.e2f)
        G = kw.pop("ilu_patch", 2)
        if kw.get("prec") == "ilu_asm" and kw.get("ilu") is None:
            h = self.ctx.ilu_asm_create(self.dims, self.K64, self.nbr, self.e2f, G)
            try:
                return self.ctx.gmres_solve(self.dims, self.K64, self.K32, self.nbr, self.r, self.x, ilu=h, **kw)
            finally:
                h.close()
        return self.ctx.gmres_solve(self.dims, self.K64, self.K32, self.nbr, self.r, self.x, **kw)

    def recover(self, Minv, Bd, Cd):
        self.ctx.recover(self.dims, self.local, Minv, Bd, Cd, self.e2f, self.perm, self.x, self.du, self.dq)

    def element_arrays(self):
        """Device buffers for the element blocks (hdg_element_blocks, hdg_element_blocks_sys)."""
        d = self.dims
        ne, D, P = d["ne"], d["dim"], d["npe"]
        z = lambda n: torch.zeros(ne * n, dtype=torch.float64, device=self.device)
        nu, nq, nt = self.nu, self.nq, self.nt
        return dict(Minv=z(P * P), Bd=z(D * P * P), Cd=z(D * P * d["nlfe"] * d["npf"]), D=z(nu * nq), E=z(nu * nu),
                    F=z(nu * nt),
                    G=z(nt * nq), H=z(nt * nu), J=z(nt * nt), ru=z(nu), rt=z(nt), q=z(nq))

    def element_blocks(self, geom, model, u, uhat, out, **kw):
        """Element residuals / blocks of the model: M-component models (a dict with "kind")
        through hdg_element_blocks_sys, scalar convection-diffusion models through
        hdg_element_blocks."""
        if "kind" in model:
            return self.ctx.element_blocks_sys(self.dims, geom, model, self.e2f, u, uhat, out, **kw)
        return self.ctx.element_blocks(self.dims, geom, model, self.e2f, u, uhat, out, **kw)

    def newton(self, geom, model, u, uhat, tol=1e-10, atol=0.0, max_steps=20, min_alpha=2.0 ** -10, time_term=None,
               forcing=None, reuse=None, refresh=0.25, **solve_kw):
        """Damped Newton iteration (Section 4.4) on a scalar convection-diffusion model or an
        M-component model (elasticity, Navier-Stokes: model has a "kind").

        u [ne*M*npe] and uhat [nf*M*npf] (device, float64) hold the state and are updated in place.
        Each step: element blocks at the state, condensation, assembly, preconditioned GMRES,
        recovery, then alpha = 1, 1/2, 1/4, ... until the residual norm decreases (or alpha
        reaches min_alpha); stops once the norm is at most max(tol * initial norm, atol).
        time_term: an implicit stage's mass term (hdg_element_blocks).
        forcing="ew": inexact Newton, the linear solves' relative tolerance follows Eisenstat and
        Walker's choice 2 (SIAM J. Sci. Comput. 17 (1996)): eta_0 = 0.01, eta_k = 0.9 (||R_k|| /
        ||R_{k-1}||)^2, kept above 0.9 eta_{k-1}^2 when that exceeds 0.1, at most 0.1, and not
        below solve_kw["rtol"] nor below what the stopping test needs; None: solve_kw["rtol"].
        reuse="chord": the linearisation (condensation factors, assembled blocks, block-Jacobi
        inverses and folded blocks) is kept from the step that formed it, and later steps only
        evaluate the residual, condense and assemble its right-hand side with the kept factors
        (hdg_condense_rhs, hdg_assemble_rhs) and solve with the kept preconditioner setup; a step
        whose residual norm fell by less than the factor `refresh`, or that needed a damped step,
        makes the next step form the linearisation afresh. The residual is always the exact one,
        so the iteration reaches the same solution (chord Newton with refresh). The kept
        linearisation also carries over to the next call with the same time-term factor c (the
        stages of a DIRK step, Section 2.2); self.jac_valid = False forgets it.
        solve_kw go to the linear solves (restart, rtol, prec, ...). Returns one
        dict(norm, alpha, iters, fresh) per step and a last entry with the final norm. Sequencing
        only: evaluation, solve and updates run in libhdg.so."""
        d = self.dims
        chord = reuse == "chord"
        if reuse not in (None, "chord"):
            raise ValueError(f"reuse must be None or 'chord', not {reuse!r}")
        c = float(time_term["c"]) if time_term else 0.0
        if chord and getattr(self, "jac_c", None) != c:
            self.jac_valid = False
        if not chord:
            self.jac_valid = False
        if getattr(self, "_blk", None) is None:
            self._blk = self.element_arrays()
            self._mass_ready = False
        blk = self._blk

        def evaluate(residual_only):
            """Element residuals (and, unless residual-only, matrices) at the state; returns whether
            the matrices were left out."""
            ro = residual_only and self._mass_ready
            self.element_blocks(geom, model, u, uhat, blk, time_term=time_term, residual_only=ro,
                                keep_mass=self._mass_ready)
            self._mass_ready = True
            return ro

        have_matrices = not evaluate(residual_only=chord and self.jac_valid)
        nrm = self.ctx.residual_norm(d, self.f2e, blk["ru"], blk["rt"])
        n0 = nrm
        hist = []
        rtol_min = solve_kw.get("rtol", 1e-8)
        eta, prev = 0.01, None
        for _ in range(max_steps):
            if nrm <= max(tol * n0, atol):
                break
            if forcing == "ew":
                if prev is not None:
                    e = 0.9 * (nrm / prev) ** 2
                    if 0.9 * eta * eta > 0.1:
                        e = max(e, 0.9 * eta * eta)
                    eta = min(e, 0.1)
                solve_kw["rtol"] = max(eta, rtol_min, 0.5 * max(tol * n0, atol) / nrm)
            fresh = not (chord and self.jac_valid)
            if fresh:
                if not have_matrices:
                    evaluate(residual_only=False)
                self.condense(blk, keep=chord)
                self.assemble()
                if str(solve_kw.get("prec", "")).startswith("asm"):
                    # additive Schwarz patches of this linearisation
                    self.asm_setup(fp32=solve_kw.get("precision", "fp64") == "mixed")
                st = self.solve(**solve_kw)
                if chord:
                    self.jac_valid, self.jac_c = True, c
            else:
                self.condense_rhs(blk["ru"], blk["rt"])
                self.assemble_rhs()
                kw = dict(solve_kw)
                if kw.get("prec", "bj") in ("bj", "bj_poly", "bj_cheb"):
                    kw["reuse_setup"] = True
                st = self.solve(**kw)
            self.recover(blk["Minv"], blk["Bd"], blk["Cd"])
            alpha, applied = 1.0, 0.0
            while True:
                self.ctx.newton_update(alpha - applied, self.du, u)
                self.ctx.newton_update(alpha - applied, self.x, uhat)
                applied = alpha
                # the trial state's blocks: kept as the next step's linearisation if accepted
                # (M^-1, B_d, C_d depend on the mesh only: kept from the first evaluation); with a
                # kept linearisation only the residual
                have_matrices = not evaluate(residual_only=chord)
                trial = self.ctx.residual_norm(d, self.f2e, blk["ru"], blk["rt"])
                if trial < nrm or alpha <= min_alpha:
                    break
                alpha *= 0.5
            if chord and (alpha < 1.0 or trial > refresh * nrm):
                self.jac_valid = False
            hist.append(dict(norm=nrm, alpha=alpha, iters=st["iters"], fresh=fresh))
            prev, nrm = nrm, trial
        hist.append(dict(norm=nrm, alpha=0.0, iters=0, fresh=False))
        return hist

    def pseudo_transient(self, geom, model, u, uhat, dtau0, tol=1e-10, atol=0.0, max_steps=200, dtau_max=1e12,
                         **solve_kw):
        """Pseudo-transient continuation (backward Euler in pseudo-time, Section 2.2, with switched
        evolution relaxation) on one mesh: a pseudo-step is one full Newton step on
        R(u) + M (u - u_k)/dtau_k = 0 from u_k, then dtau_{k+1} = min(dtau_k ||R(u_k)|| /
        ||R(u_{k+1})||, dtau_max); stops at max(tol ||R(u_0)||, atol) of the steady residual.
        u, uhat updated in place. Returns dict(norm, dtau, iters) per step and a final entry."""
        d = self.dims
        blk = self.element_arrays()
        res = {"ru": blk["ru"], "rt": blk["rt"], "Minv": blk["Minv"]}
        u_prev = torch.zeros_like(u)
        self.element_blocks(geom, model, u, uhat, blk)      # forms M^-1, B_d, C_d once
        nrm = self.ctx.residual_norm(d, self.f2e, blk["ru"], blk["rt"])
        stop = max(tol * nrm, atol)
        dtau = float(dtau0)
        hist = []
        for _ in range(max_steps):
            if nrm <= stop:
                break
            u_prev.copy_(u)
            self.element_blocks(geom, model, u, uhat, blk, keep_mass=True, time_term=dict(c=1.0 / dtau, u_prev=u_prev))
            self.condense(blk)
            self.assemble()
            if str(solve_kw.get("prec", "")).startswith("asm"):
                self.asm_setup(fp32=solve_kw.get("precision", "fp64") == "mixed")
            st = self.solve(**solve_kw)
            self.recover(blk["Minv"], blk["Bd"], blk["Cd"])
            self.ctx.newton_update(1.0, self.du, u)
            self.ctx.newton_update(1.0, self.x, uhat)
            self.element_blocks(geom, model, u, uhat, res, residual_only=True, keep_mass=True)
            new = self.ctx.residual_norm(d, self.f2e, blk["ru"], blk["rt"])
            hist.append(dict(norm=nrm, dtau=dtau, iters=st["iters"]))
            dtau = dtau_max if new == 0.0 else min(dtau * nrm / new, dtau_max)
            nrm = new
        hist.append(dict(norm=nrm, dtau=0.0, iters=0))
        return hist

    def dirk(self, geom, model, u, uhat, dt, nsteps, scheme="dirk22", **newton_kw):
        """nsteps steps of a stiffly accurate DIRK scheme (Section 2.2) of size dt; u, uhat are
        advanced in place. Stage i solves, by Newton, the steady system plus the time term
        c M (U_i - u_n) + sum_{j<i} (a_ij/a) R_s(U_j) with c = 1/(a dt), R_s the steady u-rows;
        u_{n+1} = U_s. newton_kw go to Pipeline.newton; with reuse="chord" the stages share one
        kept linearisation (all stages have the same c), refreshed by newton's rule. Returns the
        Newton histories of every stage."""
        A = dirk_tableau(scheme)
        s, a = len(A), A[0][0]
        ne, nu = self.dims["ne"], self.nu
        self.jac_valid = False
        z = lambda: torch.zeros(ne * nu, dtype=torch.float64, device=self.device)
        un = z()
        hists = []
        res = {"ru": z(), "rt": torch.zeros(ne * self.nt, dtype=torch.float64, device=self.device)}
        for _ in range(nsteps):
            un.zero_()
            self.ctx.newton_update(1.0, u, un)         # u_n
            minus_rs = []                                 # -R_s(U_j) of the finished stages
            for i in range(s):
                rx = None
                if i > 0:
                    rx = z()
                    for j in range(i):
                        self.ctx.newton_update(-A[i][j] / a, minus_rs[j], rx)
                tt = dict(c=1.0 / (a * dt), u_prev=un, r_extra=rx)
                hists.append(self.newton(geom, model, u, uhat, time_term=tt, **newton_kw))
                if i < s - 1:
                    self.element_blocks(geom, model, u, uhat, res, residual_only=True)
                    minus_rs.append(res["ru"].clone())
        return hists


def dirk_tableau(scheme):
    """Lower-triangular Butcher matrix of a stiffly accurate DIRK scheme (b = its last row):
    backward Euler; Alexander's two-stage scheme with a = 1 - 1/sqrt(2); Alexander's three-stage
    scheme with a = 0.43586652150845899942 (the root in (1/6, 1/2) of a^3 - 3a^2 + 3a/2 - 1/6)."""
    if scheme == "be":
        return [[1.0]]
    if scheme == "dirk22":
        a = 1.0 - 0.5 ** 0.5
        return [[a, 0.0], [1.0 - a, a]]
    if scheme == "dirk33":
        a = 0.43586652150845899942
        b1 = -(6.0 * a * a - 16.0 * a + 1.0) / 4.0
        b2 = (6.0 * a * a - 20.0 * a + 5.0) / 4.0
        return [[a, 0.0, 0.0], [(1.0 + a) / 2.0 - a, a, 0.0], [b1, b2, a]]
    raise ValueError(f"unknown DIRK scheme {scheme!r}")


class BatchPipeline:
    """Many independent instances (hdg_batch_* entry points): concatenated buffers of the
    condensation, assembly, solve and recovery, and a damped Newton loop per instance."""

    def __init__(self, ctx, dims_list, f2e_list, e2f_list, device="cuda", keep_fp32=True):
        import numpy as np
        self.ctx = ctx
        self.bt = hdg.Batch(ctx, dims_list)
        self.device = device
        bt = self.bt
        i32 = lambda arrs: torch.as_tensor(np.concatenate([np.asarray(a).reshape(-1) for a in arrs])
                                           .astype(np.int32)).to(device)
        self.f2e = i32(f2e_list)
        self.e2f = i32(e2f_list)
        z = lambda n, dt=torch.float64: torch.zeros(n, dtype=dt, device=device)
        self.Kbar, self.rbar, self.local = z(bt.total("Kbar")), z(bt.total("rbar")), z(bt.total("local"))
        self.K64 = z(bt.total("K"))
        self.K32 = z(bt.total("K"), torch.float32) if keep_fp32 else None
        self.nbr = torch.zeros(bt.total("nbr"), dtype=torch.int32, device=device)
        self.r, self.x = z(bt.total("vec")), z(bt.total("vec"))
        self.du, self.dq = z(bt.total("du")), z(bt.total("dq"))

    def element_arrays(self):
        z = lambda n: torch.zeros(n, dtype=torch.float64, device=self.device)
        out = {k: z(self.bt.total(k)) for k in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt")}
        out["q"] = z(self.bt.total("dq"))
        return out

    def condense(self, blk):
        self.bt.condense(blk, self.Kbar, self.rbar, self.local)

    def assemble(self):
        self.bt.assemble(self.f2e, self.e2f, self.Kbar, self.rbar, self.K64, self.K32, self.nbr, self.r)

    def solve(self, **kw):
        self.x.zero_()
        return self.bt.gmres_solve(self.K64, self.K32, self.nbr, self.r, self.x, **kw)

    def recover(self, Minv, Bd, Cd):
        self.bt.recover(self.local, Minv, Bd, Cd, self.e2f, self.x, self.du, self.dq)

    def newton(self, nqv, nqf, geom, models, u, uhat, tol=1e-10, atol=0.0, max_steps=20, min_alpha=2.0 ** -10,
               time_term=None, **solve_kw):
        """Damped Newton (Section 4.4) for every instance at once: each instance has its own
        residual norm, step halving and stopping test (max(tol * initial norm, atol)); a
        converged instance gets a zero right-hand side and no update while the others go on.
        u, uhat: batch arrays (DU / VEC offsets), updated in place. time_term = dict(c (per
        instance), u_prev, r_extra=None): an implicit stage. Returns one history per instance
        (as Pipeline.newton)."""
        import numpy as np
        bt = self.bt
        n = bt.n
        blk = self.element_arrays()
        tt = {} if time_term is None else dict(c=time_term["c"], u_prev=time_term["u_prev"],
                                                r_extra=time_term.get("r_extra"))
        bt.element_blocks(nqv, nqf, geom, models, self.e2f, u, uhat, blk, **tt)
        nrm = bt.residual_norms(self.f2e, blk["ru"], blk["rt"])
        stop = np.maximum(tol * nrm, atol)
        hists = [[] for _ in range(n)]
        off = bt.offsets("vec")
        for _ in range(max_steps):
            active = nrm > stop
            if not active.any():
                break
            self.condense(blk)
            self.assemble()
            for i in np.nonzero(~active)[0]:
                self.r[off[i]:off[i + 1]] = 0.0           # converged: no correction
            _, stats = self.solve(**solve_kw)
            self.recover(blk["Minv"], blk["Bd"], blk["Cd"])
            alpha = np.where(active, 1.0, 0.0)
            applied = np.zeros(n)
            pending = active.copy()
            while True:
                bt.newton_update(np.where(pending, alpha - applied, 0.0), self.du, u, self.x, uhat)
                applied = np.where(pending, alpha, applied)
                bt.element_blocks(nqv, nqf, geom, models, self.e2f, u, uhat, blk, keep_mass=True, **tt)
                trial = bt.residual_norms(self.f2e, blk["ru"], blk["rt"])
                accept = pending & ((trial < nrm) | (alpha <= min_alpha))
                for i in np.nonzero(accept)[0]:
                    hists[i].append(dict(norm=float(nrm[i]), alpha=float(alpha[i]), iters=int(stats[i]["iters"])))
                    nrm[i] = trial[i]
                pending &= ~accept
                if not pending.any():
                    break
                alpha = np.where(pending, alpha * 0.5, alpha)
        for i in range(n):
            hists[i].append(dict(norm=float(nrm[i]), alpha=0.0, iters=0))
        return hists

    def pseudo_transient(self, nqv, nqf, geom, models, u, uhat, dtau0, tol=1e-10, atol=0.0, max_steps=200,
                         dtau_max=1e12, **solve_kw):
        """Pseudo-transient continuation for every instance (backward Euler in pseudo-time,
        Section 2.2, with switched evolution relaxation): a pseudo-step is one full Newton step
        on R(u) + M (u - u_k)/dtau_k = 0 from u_k, then dtau_{k+1} = min(dtau_k ||R(u_k)|| /
        ||R(u_{k+1})||, dtau_max), per instance; each instance stops at max(tol ||R(u_0)||, atol)
        of its steady residual. Returns one history per instance: dict(norm, dtau, iters) per
        step and a last entry with the final norm."""
        import numpy as np
        bt = self.bt
        n = bt.n
        blk = self.element_arrays()
        res = {"ru": blk["ru"], "rt": blk["rt"], "Minv": blk["Minv"]}
        u_prev = torch.zeros_like(u)
        bt.element_blocks(nqv, nqf, geom, models, self.e2f, u, uhat, blk)   # forms M^-1, B_d, C_d once
        nrm = bt.residual_norms(self.f2e, blk["ru"], blk["rt"])
        stop = np.maximum(tol * nrm, atol)
        dtau = np.full(n, float(dtau0))
        hists = [[] for _ in range(n)]
        off = bt.offsets("vec")
        for _ in range(max_steps):
            active = nrm > stop
            if not active.any():
                break
            u_prev.copy_(u)
            bt.element_blocks(nqv, nqf, geom, models, self.e2f, u, uhat, blk, c=np.where(active, 1.0 / dtau, 0.0),
                              u_prev=u_prev, keep_mass=True)
            self.condense(blk)
            self.assemble()
            for i in np.nonzero(~active)[0]:
                self.r[off[i]:off[i + 1]] = 0.0
            _, stats = self.solve(**solve_kw)
            self.recover(blk["Minv"], blk["Bd"], blk["Cd"])
            bt.newton_update(np.where(active, 1.0, 0.0), self.du, u, self.x, uhat)
            bt.element_blocks(nqv, nqf, geom, models, self.e2f, u, uhat, res, residual_only=True, keep_mass=True)
            new = bt.residual_norms(self.f2e, blk["ru"], blk["rt"])
            for i in np.nonzero(active)[0]:
                hists[i].append(dict(norm=float(nrm[i]), dtau=float(dtau[i]), iters=int(stats[i]["iters"])))
                # an exactly solved instance has reached its steady state: dtau at its cap
                dtau[i] = dtau_max if new[i] == 0.0 else min(dtau[i] * nrm[i] / new[i], dtau_max)
                nrm[i] = new[i]
        for i in range(n):
            hists[i].append(dict(norm=float(nrm[i]), dtau=0.0, iters=0))
        return hists

    def dirk(self, nqv, nqf, geom, models, u, uhat, dt, nsteps, scheme="dirk22", **newton_kw):
        """nsteps DIRK steps (Section 2.2) of size dt for every instance: stage i solves the
        steady system plus c M (U_i - u_n) + sum_{j<i} (a_ij/a) R_s(U_j), c = 1/(a dt), with the
        batched damped Newton; u_{n+1} = U_s. Returns the per-instance Newton histories of every
        stage (a list per stage)."""
        import numpy as np
        A = dirk_tableau(scheme)
        s_, a = len(A), A[0][0]
        bt = self.bt
        n = bt.n
        z = lambda: torch.zeros(bt.total("du"), dtype=torch.float64, device=self.device)
        un = z()
        res = {"ru": z(), "rt": torch.zeros(bt.total("rt"), dtype=torch.float64, device=self.device)}
        out = []
        for _ in range(nsteps):
            un.copy_(u)
            minus_rs = []
            for i in range(s_):
                rx = None
                if i > 0:
                    rx = z()
                    for j in range(i):
                        bt.newton_update(np.full(n, -A[i][j] / a), minus_rs[j], rx, self.x, torch.zeros_like(self.x))
                tt = dict(c=np.full(n, 1.0 / (a * dt)), u_prev=un, r_extra=rx)
                out.append(self.newton(nqv, nqf, geom, models, u, uhat, time_term=tt, **newton_kw))
                if i < s_ - 1:
                    bt.element_blocks(nqv, nqf, geom, models, self.e2f, u, uhat, res, residual_only=True)
                    minus_rs.append(res["ru"].clone())
        return out
