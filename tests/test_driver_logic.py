"""Host logic of the batched Newton and pseudo-transient drivers (BatchPipeline), on the CPU.

The library calls are replaced by a stand-in whose instances are scalar equations R_i(u) = 0
(the element evaluation returns -R_i, the "solve" returns the Newton correction of the
linearised equation, with the time term where given). The drivers' per-instance bookkeeping
(step halving on the residual norm, stopping, freezing converged instances, the pseudo-time
step growth) is checked against plain loops written here from Section 4.4 and Section 2.2.
"""
import math

import numpy as np
import torch

from paper_2512_13619_amd.pipeline import BatchPipeline


FUNCS = [  # R(u), R'(u), u0
    (lambda u: u ** 3 - 2.0, lambda u: 3 * u ** 2, 1.0),
    (lambda u: math.atan(u), lambda u: 1.0 / (1.0 + u * u), 2.0),      # undamped Newton diverges
    (lambda u: u - 0.5, lambda u: 1.0, 3.0),                             # linear: one step
    (lambda u: math.atan(u - 1.0) + 0.1 * u, lambda u: 1.0 / (1.0 + (u - 1.0) ** 2) + 0.1, 5.0),
]


class StandInBatch:
    """What BatchPipeline calls on hdg.Batch, for n scalar instances (one u entry each)."""

    def __init__(self, funcs):
        self.f = funcs
        self.n = len(funcs)

    def total(self, name):
        return self.n

    def offsets(self, name):
        return np.arange(self.n + 1)

    def element_blocks(self, nqv, nqf, geom, models, e2f, u, uhat, out, residual_only=False, c=None, u_prev=None,
                       keep_mass=False):
        cc = np.zeros(self.n) if c is None else np.asarray(c, float)
        up = np.zeros(self.n) if u_prev is None else u_prev.numpy()
        uu = u.numpy()
        for i, (R, dR, _) in enumerate(self.f):
            out["ru"][i] = -(R(uu[i]) + cc[i] * (uu[i] - up[i]))
            out["rt"][i] = 0.0
            if not residual_only:
                out["E"][i] = dR(uu[i]) + cc[i]

    def residual_norms(self, f2e, ru, rt):
        return np.abs(ru.numpy())

    def condense(self, blk, Kbar, rbar, local):
        self.blk = blk

    def assemble(self, f2e, e2f, Kbar, rbar, K64, K32, nbr, r):
        r.copy_(self.blk["ru"])

    def gmres_solve(self, K64, K32, nbr, r, x, **kw):
        x.zero_()
        return 0, [dict(iters=1) for _ in range(self.n)]

    def recover(self, local, Minv, Bd, Cd, e2f, x, du, dq):
        du.copy_(self.blk["ru"] / self.blk["E"])      # rhs zeroed for converged instances has no effect here

    def newton_update(self, alpha, du, u, x, uhat):
        u.add_(torch.as_tensor(alpha) * du)


def stand_in_pipeline(funcs):
    bp = BatchPipeline.__new__(BatchPipeline)
    bp.bt = StandInBatch(funcs)
    bp.device = "cpu"
    z = lambda: torch.zeros(len(funcs), dtype=torch.float64)
    bp.f2e = bp.e2f = torch.zeros(len(funcs), dtype=torch.int32)
    bp.Kbar, bp.rbar, bp.local, bp.K64, bp.K32 = z(), z(), z(), z(), None
    bp.nbr = torch.zeros(len(funcs), dtype=torch.int32)
    bp.r, bp.x, bp.du, bp.dq = z(), z(), z(), z()
    return bp


def reference_newton(R, dR, u, tol, max_steps=30, min_alpha=2.0 ** -10):
    n = n0 = abs(R(u))
    hist = []
    for _ in range(max_steps):
        if n <= tol * n0:
            break
        d = -R(u) / dR(u)
        a = 1.0
        while True:
            t = abs(R(u + a * d))
            if t < n or a <= min_alpha:
                break
            a *= 0.5
        hist.append((n, a))
        u, n = u + a * d, t
    return u, hist


def reference_ptc(R, dR, u, tol, dtau, max_steps=200, dtau_max=1e12):
    n = n0 = abs(R(u))
    hist = []
    for _ in range(max_steps):
        if n <= tol * n0:
            break
        u = u - R(u) / (dR(u) + 1.0 / dtau)
        new = abs(R(u))
        hist.append((n, dtau))
        dtau = dtau_max if new == 0.0 else min(dtau * n / new, dtau_max)
        n = new
    return u, hist


def test_batched_newton_bookkeeping_matches_per_instance_loops():
    bp = stand_in_pipeline(FUNCS)
    u = torch.tensor([f[2] for f in FUNCS], dtype=torch.float64)
    uhat = torch.zeros(len(FUNCS), dtype=torch.float64)
    hists = bp.newton(None, None, None, None, u, uhat, tol=1e-12, max_steps=30)
    for i, (R, dR, u0) in enumerate(FUNCS):
        u_ref, h_ref = reference_newton(R, dR, u0, 1e-12)
        assert [h["alpha"] for h in hists[i][:-1]] == [a for _, a in h_ref], i
        assert np.allclose([h["norm"] for h in hists[i][:-1]], [n for n, _ in h_ref], rtol=1e-12, atol=0), i
        assert abs(u[i].item() - u_ref) <= 1e-12 * max(1.0, abs(u_ref)), i
    assert any(h["alpha"] < 1.0 for h in hists[1][:-1])       # atan from 2 needs damping
    assert len(hists[2]) == 2                                 # the linear instance: one full step


def test_batched_pseudo_transient_bookkeeping_matches_per_instance_loops():
    bp = stand_in_pipeline(FUNCS)
    u = torch.tensor([f[2] for f in FUNCS], dtype=torch.float64)
    uhat = torch.zeros(len(FUNCS), dtype=torch.float64)
    hists = bp.pseudo_transient(None, None, None, None, u, uhat, 0.05, tol=1e-12)
    for i, (R, dR, u0) in enumerate(FUNCS):
        u_ref, h_ref = reference_ptc(R, dR, u0, 1e-12, 0.05)
        assert len(hists[i]) - 1 == len(h_ref), i
        assert np.allclose([h["dtau"] for h in hists[i][:-1]], [d for _, d in h_ref], rtol=1e-12, atol=0), i
        assert abs(u[i].item() - u_ref) <= 1e-12 * max(1.0, abs(u_ref)), i
        assert hists[i][-1]["norm"] <= 1e-12 * hists[i][0]["norm"], i
