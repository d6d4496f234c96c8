"""Diagonally implicit Runge-Kutta time stepping of the HDG system (oracle; test
infrastructure only).

Section 2.2: a DIRK(s, p) scheme has a lower-triangular Butcher tableau with equal diagonal
entries a, and each step solves s implicit stages in sequence. For the semi-discrete system
M du/dt + R_s(u) = 0 (R_s: the steady u-rows of the weak form; the q- and trace equations
hold at every stage), stage i solves
  M (U_i - u_n) / dt + sum_{j <= i} a_ij R_s(U_j) = 0,   R_t(U_i) = 0,
i.e. after division by a: the steady system plus the time term c M (U_i - u_n) with
c = 1/(a dt) and the known r_x = sum_{j < i} (a_ij / a) R_s(U_j). The schemes used here are
stiffly accurate (b = the last row of the tableau), so u_{n+1} = U_s and uhat_{n+1} = Uhat_s.
Each stage is solved by the damped Newton iteration of Section 4.4 (newton.py).

Tableaus (Alexander, SIAM J. Numer. Anal. 14 (1977)): backward Euler DIRK(1,1);
DIRK(2,2) with a = 1 - 1/sqrt(2); DIRK(3,3) with a the root in (1/6, 1/2) of
a^3 - 3a^2 + 3a/2 - 1/6 = 0.
"""
import numpy as np

from . import elements, newton


def tableau(name):
    """(A, b, c) of a stiffly accurate DIRK scheme: 'be', 'dirk22' or 'dirk33'."""
    if name == "be":
        A = np.array([[1.0]])
    elif name == "dirk22":
        a = 1.0 - 1.0 / np.sqrt(2.0)
        A = np.array([[a, 0.0], [1.0 - a, a]])
    elif name == "dirk33":
        r = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
        a = float(next(x.real for x in r if abs(x.imag) < 1e-12 and 1 / 6 < x.real < 0.5))
        t2 = (1.0 + a) / 2.0
        b1 = -(6 * a * a - 16 * a + 1) / 4.0
        b2 = (6 * a * a - 20 * a + 5) / 4.0
        A = np.array([[a, 0.0, 0.0], [t2 - a, a, 0.0], [b1, b2, a]])
    else:
        raise KeyError(name)
    return A, A[-1].copy(), A.sum(1)


def spatial_u_residual(g, m, u, uhat, e2f):
    """R_s at the state: the steady u-rows (ne, P) with consistent q."""
    return -elements.element_blocks(g, m, u, uhat, e2f)["ru"]


def dirk_steps(g, m, u0, uhat0, e2f, f2e, dims, dt, nsteps, scheme="dirk22", newton_rtol=1e-12):
    """nsteps DIRK steps of size dt from (u0, uhat0); returns (u, uhat, histories of every stage)."""
    A, _, _ = tableau(scheme)
    s = A.shape[0]
    a = A[0, 0]
    u, uhat = u0.copy(), uhat0.copy()
    hists = []
    for _ in range(nsteps):
        Rs = []
        U, Uh = u, uhat
        for i in range(s):
            rx = None
            for j in range(i):
                rx = (A[i, j] / a) * Rs[j] if rx is None else rx + (A[i, j] / a) * Rs[j]
            tt = dict(c=1.0 / (a * dt), u_prev=u, r_extra=rx)
            U, Uh, h = newton.damped_newton(g, m, U, Uh, e2f, f2e, dims, rtol=newton_rtol, tt=tt)
            hists.append(h)
            if i < s - 1:
                Rs.append(spatial_u_residual(g, m, U, Uh, e2f))
        u, uhat = U, Uh
    return u, uhat, hists
