"""Damped Newton iteration on the HDG system (oracle; test infrastructure only).

Section 4.4: at each Newton step the residual is evaluated, the linearised system is
condensed, assembled and solved for the trace correction, the element corrections are
recovered, and the state is updated with a step alpha that starts at 1 and is halved while
the residual norm does not decrease. Here the trace system is solved exactly (sparse LU),
which is the plain definition of what the preconditioned GMRES approximates.

Residual norm: ||R||^2 = sum_e ||R_u^e||^2 + sum_f ||R_f||^2, where R_f is the trace
residual of face f summed over the face's elements (the assembled trace rows; R_q = 0 for
consistent states).
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import assemble, condense, elements, elements_sys


def element_blocks(g, m, u, uhat, e2f, tt=None):
    """The element blocks of the model: M-component models (m has a "kind") through
    elements_sys, scalar convection-diffusion models through elements."""
    mod = elements_sys if "kind" in m else elements
    return mod.element_blocks(g, m, u, uhat, e2f, tt)


def residual_norm(g, m, u, uhat, e2f, f2e, dims, tt=None):
    blk = element_blocks(g, m, u, uhat, e2f, tt)
    return _norm_from_blocks(blk, e2f, f2e, dims), blk


def _norm_from_blocks(blk, e2f, f2e, dims):
    # assembled trace residual: the face vector of the element trace rows (zero matrix part)
    ne, nt = blk["rt"].shape
    _, _, r_face = assemble.assemble(np.zeros((ne, nt, nt)), blk["rt"], f2e, e2f, dims)
    return float(np.sqrt(np.sum(blk["ru"] ** 2) + np.sum(r_face ** 2)))


def damped_newton(g, m, u0, uhat0, e2f, f2e, dims, rtol=1e-10, atol=1e-14, max_steps=20, min_alpha=2.0 ** -10,
                  tt=None):
    """Returns (u, uhat, history); history[k] = dict(norm, alpha) for step k (norm before it).
    tt: the time term of an implicit stage (elements.element_blocks)."""
    u = u0.copy()
    uhat = uhat0.copy()
    nrm, blk = residual_norm(g, m, u, uhat, e2f, f2e, dims, tt)
    n0 = nrm
    hist = []
    for _ in range(max_steps):
        if nrm <= max(rtol * n0, atol):
            break
        Kb, rb = condense.condense(blk, dims)
        K, nbr, r = assemble.assemble(Kb, rb, f2e, e2f, dims)
        dx = spla.spsolve(assemble.to_sparse(K, nbr).tocsc(), r)
        _, du = condense.recover(blk, dx, e2f, dims)
        du = du.reshape(u.shape)
        duhat = dx.reshape(uhat.shape)
        alpha = 1.0
        while True:
            ut = u + alpha * du
            uht = uhat + alpha * duhat
            nt_, blkt = residual_norm(g, m, ut, uht, e2f, f2e, dims, tt)
            if nt_ < nrm or alpha <= min_alpha:
                break
            alpha *= 0.5
        hist.append(dict(norm=nrm, alpha=alpha))
        u, uhat, nrm, blk = ut, uht, nt_, blkt
    hist.append(dict(norm=nrm, alpha=0.0))
    return u, uhat, hist


def pseudo_transient(g, m, u0, uhat0, e2f, f2e, dims, dtau0, rtol=1e-10, atol=1e-14, max_steps=200, dtau_max=1e12):
    """Pseudo-transient continuation (backward Euler in pseudo-time, Section 2.2's use of DIRK
    schemes for pseudo-transient runs) with switched evolution relaxation (Mulder and Van Leer,
    J. Comput. Phys. 59 (1985); analysed by Kelley and Keyes, SIAM J. Numer. Anal. 35 (1998)):
    each pseudo-step is one full Newton step on R(u) + M (u - u_k) / dtau_k = 0 from u_k (whose
    residual at u_k is the steady one), then dtau_{k+1} = min(dtau_k ||R(u_k)|| / ||R(u_{k+1})||,
    dtau_max). Stops at ||R|| <= max(rtol ||R(u_0)||, atol) (steady norm). Returns (u, uhat,
    history) with history[k] = dict(norm, dtau) before step k."""
    u, uhat = u0.copy(), uhat0.copy()
    nrm, _ = residual_norm(g, m, u, uhat, e2f, f2e, dims)
    n0 = nrm
    dtau = dtau0
    hist = []
    for _ in range(max_steps):
        if nrm <= max(rtol * n0, atol):
            break
        blk = element_blocks(g, m, u, uhat, e2f, dict(c=1.0 / dtau, u_prev=u.copy(), r_extra=None))
        Kb, rb = condense.condense(blk, dims)
        K, nbr, r = assemble.assemble(Kb, rb, f2e, e2f, dims)
        dx = spla.spsolve(assemble.to_sparse(K, nbr).tocsc(), r)
        _, du = condense.recover(blk, dx, e2f, dims)
        u = u + du.reshape(u.shape)
        uhat = uhat + dx.reshape(uhat.shape)
        new, _ = residual_norm(g, m, u, uhat, e2f, f2e, dims)
        hist.append(dict(norm=nrm, dtau=dtau))
        dtau = dtau_max if new == 0.0 else min(dtau * nrm / new, dtau_max)
        nrm = new
    hist.append(dict(norm=nrm, dtau=0.0))
    return u, uhat, hist
