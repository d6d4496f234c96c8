"""Element residuals and Jacobian blocks of the HDG system for M-component conservation laws
(oracle; test infrastructure only).

Model (Section 2.1): du/dt + div F(u, q) = s with q = grad u, F an M x D flux. Two fluxes:
  elasticity      F = -sigma(q),  sigma = lam tr(eps) I + 2 mu eps,  eps = (q + q^T)/2
                  (u the displacement, M = D = 3);
  Navier-Stokes   F = F_c(u) - F_v(u, q) in conservative variables u = (rho, rho v, rho E),
                  p = (gamma - 1)(rho E - |rho v|^2 / (2 rho)),
                  F_c = (rho v, rho v v^T + p I, (rho E + p) v),
                  F_v = (0, tau_v, tau_v v + kappa grad e),  mu = 1/Re, Stokes hypothesis
                  tau_v = mu (grad v + grad v^T) - (2/3) mu (div v) I,
                  e = E - |v|^2/2 the specific internal energy, kappa = mu gamma / Pr
                  (the Fourier heat flux written with grad e: T proportional to e), and
                  grad v, grad e formed from the conservative gradients q by the chain rule.
Numerical flux (Section 2.2 with S = tau I): fhat = F(uhat, q).n + tau (u - uhat); Dirichlet
trace rows uhat - u_D on boundary faces.

Residuals of one element from the weak form of Section 2.2, test functions r = phi_i e_(m,d),
w = phi_i e_m, mu = psi_j e_m (components m, directions d):
  R_q[m,d,i] = (q_md, phi_i) + (u_m, d phi_i/dx_d) - <uhat_m n_d, phi_i>
  R_u[m,i]   = -(F_m, grad phi_i) + <fhat_m, phi_i> - (s_m, phi_i)  [+ c (u_m - u_n,m, phi_i) + r_x]
  R_t[l,m,j] = -<fhat_m, psi_j>_l  (interior face; the trace rows negated as in the scalar case)
               <uhat_m - u_D,m, psi_j>_l  (Dirichlet face)
D, E, F, G, H, J are the derivatives of R_u and R_t with respect to q, u and uhat (Section 4.1
gives E; the others follow the same rule), with the pointwise flux derivatives taken by the
complex-step method (Squire and Trapp, SIAM Rev. 40 (1998)): dF/dx = Im F(x + i h) / h with
h = 1e-30, exact to rounding for fluxes built from arithmetic operations.

Dof order: u (m, i) -> m P + i; q (m, d, i) -> (m D + d) P + i; element trace (l, m, j) ->
(l M + m) PF + j; uhat per face (m, j) -> m PF + j (canonical face order).
Inputs as for elements.py, with src[e][x][M], uD[e][l][x][M], u[e][M][P], uhat[nf][M][PF].
Loops follow the formulas: one element at a time, one quadrature point at a time.
"""
import numpy as np

from .elements import mass_and_q_operators

H_CS = 1e-30


def flux_elasticity(m, u, q):
    """F (M, D) of linear elasticity at one point: -sigma(q)."""
    D = q.shape[1]
    tr = sum(q[k, k] for k in range(D))
    sig = m["lam"] * tr * np.eye(D) + m["mu"] * (q + q.T)
    return -sig


def flux_navier_stokes(m, u, q):
    """F (5, 3) of the compressible Navier-Stokes equations at one point."""
    g = m["gamma"]
    mu = 1.0 / m["Re"]
    kappa = mu * g / m["Pr"]
    rho, mom, rE = u[0], u[1:4], u[4]
    v = mom / rho
    p = (g - 1.0) * (rE - 0.5 * (mom[0] * v[0] + mom[1] * v[1] + mom[2] * v[2]))
    E = rE / rho
    F = np.zeros((5, 3), dtype=u.dtype)
    # convective part
    F[0] = mom
    for a in range(3):
        F[1 + a] = mom[a] * v
        F[1 + a, a] += p
    F[4] = (rE + p) * v
    # viscous part from the conservative gradients: grad v = (grad(rho v) - v grad rho)/rho
    grho = q[0]
    gv = np.array([(q[1 + a] - v[a] * grho) / rho for a in range(3)])     # gv[a][d] = dv_a/dx_d
    div = gv[0, 0] + gv[1, 1] + gv[2, 2]
    tv = mu * (gv + gv.T) - (2.0 / 3.0) * mu * div * np.eye(3)
    # grad e = (grad(rho E) - E grad rho)/rho - sum_a v_a grad v_a
    ge = (q[4] - E * grho) / rho - (v[0] * gv[0] + v[1] * gv[1] + v[2] * gv[2])
    F[1:4] -= tv
    F[4] -= tv.T @ v + kappa * ge
    return F


FLUXES = {"elasticity": flux_elasticity, "navier_stokes": flux_navier_stokes}


def flux_and_jacobians(m, u, q):
    """F (M, D), dF/du (M, D, M), dF/dq (M, D, M, D) at one point, the derivatives by complex step."""
    f = FLUXES[m["kind"]]
    M, D = q.shape
    F = f(m, u.astype(float), q.astype(float))
    Fu = np.zeros((M, D, M))
    Fq = np.zeros((M, D, M, D))
    for b in range(M):
        du = u.astype(complex)
        du[b] += 1j * H_CS
        Fu[:, :, b] = f(m, du, q.astype(complex)).imag / H_CS
        for d in range(D):
            dq = q.astype(complex)
            dq[b, d] += 1j * H_CS
            Fq[:, :, b, d] = f(m, u.astype(complex), dq).imag / H_CS
    return F, Fu, Fq


def consistent_q(g, e, u, uh_el):
    """q[m][d][i] with R_q = 0: q_md = -M^{-1}(B_d u_m + C_d uhat_m) (eq. w16), per component."""
    Mm, Bd, Cd = mass_and_q_operators(g, e)
    M = u.shape[0]
    L = uh_el.shape[0]
    out = np.zeros((M, Bd.shape[0], u.shape[1]))
    for a in range(M):
        uh_m = np.concatenate([uh_el[l, a] for l in range(L)])
        for d in range(Bd.shape[0]):
            out[a, d] = -np.linalg.solve(Mm, Bd[d] @ u[a] + Cd[d] @ uh_m)
    return out


def _geom(g, e):
    return (g["wdet"][e], g["dphix"][e], g["phi"], g["phif"][e], g["psi"], g["ndA"][e], g["dA"][e],
            g["src"][e], g["uD"][e], g["bnd"][e])


def residual(g, m, e, q, u, uh, tt=None):
    """R_q (M, D, P), R_u (M, P), R_t (L, M, PF) of element e at (q, u, uhat_el); tt = (c, u_n, r_x)."""
    wdet, dphix, phi, phif, psi, ndA, dA, src, uD, bnd = _geom(g, e)
    Qv, P = phi.shape
    L, Qf, _ = phif.shape
    PF = psi.shape[1]
    D = dphix.shape[2]
    M = u.shape[0]
    tau = m["tau"]
    f = FLUXES[m["kind"]]
    Rq = np.zeros((M, D, P))
    Ru = np.zeros((M, P))
    Rt = np.zeros((L, M, PF))
    for k in range(Qv):
        uk = u @ phi[k]                       # (M,)
        qk = q @ phi[k]                       # (M, D)
        for a in range(M):
            for d in range(D):
                Rq[a, d] += wdet[k] * (qk[a, d] * phi[k] + uk[a] * dphix[k, :, d])
        Fk = f(m, uk, qk)
        Ru -= wdet[k] * (Fk @ dphix[k].T)     # (M, P): sum_d F[a,d] dphi_i/dx_d
        Ru -= wdet[k] * np.outer(src[k], phi[k])
        if tt is not None:
            Ru += tt[0] * wdet[k] * np.outer(uk - tt[1] @ phi[k], phi[k])
    if tt is not None and tt[2] is not None:
        Ru += tt[2]
    for l in range(L):
        for k in range(Qf):
            uf = u @ phif[l, k]
            qf = q @ phif[l, k]
            uhf = uh[l] @ psi[k]              # (M,)
            for a in range(M):
                for d in range(D):
                    Rq[a, d] -= uhf[a] * ndA[l, k, d] * phif[l, k]
            fhat = f(m, uhf, qf) @ ndA[l, k] + tau * (uf - uhf) * dA[l, k]
            Ru += np.outer(fhat, phif[l, k])
            if bnd[l]:
                Rt[l] += dA[l, k] * np.outer(uhf - uD[l, k], psi[k])
            else:
                Rt[l] -= np.outer(fhat, psi[k])
    return Rq, Ru, Rt


def jacobian(g, m, e, q, u, uh, c=0.0):
    """D (MP, MDP), E (MP, MP), F (MP, LMPF), G (LMPF, MDP), H (LMPF, MP), J (LMPF, LMPF)."""
    wdet, dphix, phi, phif, psi, ndA, dA, src, uD, bnd = _geom(g, e)
    Qv, P = phi.shape
    L, Qf, _ = phif.shape
    PF = psi.shape[1]
    D = dphix.shape[2]
    M = u.shape[0]
    tau = m["tau"]
    I = np.eye(M)
    Dm = np.zeros((M, P, M, D, P))
    Em = np.zeros((M, P, M, P))
    Fm = np.zeros((M, P, L, M, PF))
    Gm = np.zeros((L, M, PF, M, D, P))
    Hm = np.zeros((L, M, PF, M, P))
    Jm = np.zeros((L, M, PF, L, M, PF))
    for k in range(Qv):
        uk = u @ phi[k]
        qk = q @ phi[k]
        _, Fu, Fq = flux_and_jacobians(m, uk, qk)
        for a in range(M):
            for b in range(M):
                # -(dF_a/du_b phi_j, grad phi_i) and -(dF_a/dq_bd phi_j, grad phi_i)
                Em[a, :, b, :] -= wdet[k] * np.outer(dphix[k] @ Fu[a, :, b], phi[k])
                for d in range(D):
                    Dm[a, :, b, d, :] -= wdet[k] * np.outer(dphix[k] @ Fq[a, :, b, d], phi[k])
            Em[a, :, a, :] += c * wdet[k] * np.outer(phi[k], phi[k])
    for l in range(L):
        for k in range(Qf):
            qf = q @ phif[l, k]
            uhf = uh[l] @ psi[k]
            _, Fu, Fq = flux_and_jacobians(m, uhf, qf)
            n = ndA[l, k]
            Z = np.einsum("axb,x->ab", Fu, n)          # d(F.n)/d uhat
            Y = np.einsum("axbd,x->abd", Fq, n)        # d(F.n)/d q
            pp = np.outer(phif[l, k], phif[l, k])
            ps = np.outer(phif[l, k], psi[k])
            for a in range(M):
                Em[a, :, a, :] += tau * dA[l, k] * pp
                for b in range(M):
                    for d in range(D):
                        Dm[a, :, b, d, :] += Y[a, b, d] * pp
                    Fm[a, :, l, b, :] += (Z[a, b] - tau * dA[l, k] * I[a, b]) * ps
                    if bnd[l]:
                        Jm[l, a, :, l, b, :] += I[a, b] * dA[l, k] * np.outer(psi[k], psi[k])
                    else:
                        for d in range(D):
                            Gm[l, a, :, b, d, :] -= Y[a, b, d] * ps.T
                        Hm[l, a, :, b, :] -= tau * I[a, b] * dA[l, k] * ps.T
                        Jm[l, a, :, l, b, :] -= (Z[a, b] - tau * I[a, b] * dA[l, k]) * np.outer(psi[k], psi[k])
    nu, nq, nt = M * P, M * D * P, L * M * PF
    return (Dm.reshape(nu, nq), Em.reshape(nu, nu), Fm.reshape(nu, nt), Gm.reshape(nt, nq), Hm.reshape(nt, nu),
            Jm.reshape(nt, nt))


def element_trace_values(uhat, e2f):
    """uhat_el[e][l][m][j] = uhat[e2f[e][l]][m][j] (canonical face order on both sides)."""
    return uhat[e2f]


def element_blocks(g, m, u, uhat, e2f, tt=None):
    """Every element's condensation inputs at the state (u [ne][M][P], uhat [nf][M][PF]) with
    consistent q: Minv, Bd, Cd, D, E, F, G, H, J, ru = -R_u, rt = -R_t (flattened in the dof
    orders above) and q [ne][M][D][P]. tt = dict(c, u_prev [ne][M][P], r_extra [ne][M][P] or None)."""
    ne = u.shape[0]
    uh_el = element_trace_values(uhat, e2f)
    out = {k: [] for k in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt", "q")}
    for e in range(ne):
        Mm, Bd, Cd = mass_and_q_operators(g, e)
        q = consistent_q(g, e, u[e], uh_el[e])
        tte = None
        if tt is not None:
            rx = tt.get("r_extra")
            tte = (tt["c"], tt["u_prev"][e], None if rx is None else rx[e])
        _, Ru, Rt = residual(g, m, e, q, u[e], uh_el[e], tte)
        Dm, Em, Fm, Gm, Hm, Jm = jacobian(g, m, e, q, u[e], uh_el[e], 0.0 if tt is None else tt["c"])
        for k, v in (("Minv", np.linalg.inv(Mm)), ("Bd", Bd), ("Cd", Cd), ("D", Dm), ("E", Em), ("F", Fm),
                     ("G", Gm), ("H", Hm), ("J", Jm), ("ru", -Ru.ravel()), ("rt", -Rt.ravel()), ("q", q)):
            out[k].append(v)
    return {k: np.array(v) for k, v in out.items()}
