"""Element residuals and Jacobian blocks of the HDG backward-Euler/steady system for scalar
convection-diffusion models (oracle; test infrastructure only).

Model (Section 2.1 with M = 1): F(u, q) = beta u^2/2 + gamma u - nu q (a D-vector), source
s(x), numerical flux fhat = F(uhat, q).n + tau (u - uhat) (the flux of the backward-Euler
system with S = tau I, Section 2.2), Dirichlet rows uhat - u_D on boundary faces.
Poisson is beta = gamma = 0, nu = 1; the 2D viscous Burgers workload is beta = (1, 0),
gamma = (0, 1).

Residuals of one element, written from the weak form of Section 2.2 with test functions
r = phi_i e_d, w = phi_i, mu = psi_j (the steady case: no 1/dt term):
  R_q[d, i] = (q_d, phi_i) + (u, d phi_i/dx_d) - <uhat n_d, phi_i>
  R_u[i]    = -(F(u, q), grad phi_i) + <fhat, phi_i> - (s, phi_i)
  R_t[l, j] = -<fhat, psi_j>_l           on interior faces (sign reading: trace rows negated)
              <uhat - u_D, psi_j>_l       on Dirichlet faces
The linearised system of Section 2.3 is
  [A B C; D E F; G H J] [dq; du; duhat] = -[R_q; R_u; R_t],
with A = I_D (x) M, B = B_d, C = C_d (eq. w16, derivative on the test function) and
D, E, F, G, H, J the derivatives of R_u and R_t (Section 4.1 gives E; the others follow
the same rule). Elements carry q consistent with the q-equation (R_q = 0), so
q = -M^{-1}(B_d u + C_d uhat) per direction (eq. w16) and r_q = 0 (Section 4.1).

Inputs (numpy, float64): the mesh's quadrature geometry
  wdet[e][q]          volume weights times |det J|
  dphix[e][q][i][x]   physical gradients of the element basis at volume points
  phi[q][i]           element basis at volume points (reference)
  phif[e][l][q][i]    element basis at the points of local face l
  psi[q][j]           face basis at face points (canonical face order)
  ndA[e][l][q][x]     outward normal times face weight, dA[e][l][q] face weight
  src[e][q]           source at volume points; uD[e][l][q] Dirichlet data at face points
  bnd[e][l]           1 on boundary faces
and the state u[e][i] (nodal), uhat_el[e][l][j] (the element's face values).
Time term (one implicit stage, Section 2.2): with c = 1/(a_ii dt), the previous step's u_n and
the earlier stages' contribution r_x (known), the u-rows become
  R_u + c (u - u_n, phi_i) + r_x[i],   so E gains c M;
c = 0 and no r_x is the steady system.
Loops follow the formulas: one element at a time, one quadrature point at a time.
"""
import numpy as np


def flux(m, u, q):
    """F(u, q) for a scalar u and gradient q (D,)."""
    return np.array([m["beta"][x] * u * u / 2 + m["gamma"][x] * u - m["nu"] * q[x] for x in range(len(q))])


def flux_du(m, u, D):
    """dF_x/du = beta_x u + gamma_x."""
    return np.array([m["beta"][x] * u + m["gamma"][x] for x in range(D)])


def flux_dq(m, D):
    """dF_x/dq_d = -nu delta_xd."""
    return -m["nu"] * np.eye(D)


def _element_geom(g, e):
    return (g["wdet"][e], g["dphix"][e], g["phi"], g["phif"][e], g["psi"], g["ndA"][e], g["dA"][e],
            g["src"][e], g["uD"][e], g["bnd"][e])


def mass_and_q_operators(g, e):
    """M, B_d, C_d of element e (eq. w16, derivative on the test function)."""
    wdet, dphix, phi, phif, psi, ndA, dA, *_ = _element_geom(g, e)
    Qv, P = phi.shape
    L, Qf, _ = phif.shape
    PF = psi.shape[1]
    D = dphix.shape[2]
    Mm = np.zeros((P, P))
    Bd = np.zeros((D, P, P))
    Cd = np.zeros((D, P, L * PF))
    for q in range(Qv):
        Mm += wdet[q] * np.outer(phi[q], phi[q])
        for d in range(D):
            Bd[d] += wdet[q] * np.outer(dphix[q, :, d], phi[q])
    for l in range(L):
        for q in range(Qf):
            for d in range(D):
                Cd[d][:, l * PF:(l + 1) * PF] -= ndA[l, q, d] * np.outer(phif[l, q], psi[q])
    return Mm, Bd, Cd


def consistent_q(g, e, u, uh):
    """q[d][i] with R_q = 0: q_d = -M^{-1}(B_d u + C_d uhat)."""
    Mm, Bd, Cd = mass_and_q_operators(g, e)
    return np.stack([-np.linalg.solve(Mm, Bd[d] @ u + Cd[d] @ uh.ravel()) for d in range(Bd.shape[0])])


def residual(g, m, e, q, u, uh, tt=None):
    """(R_q (D, P), R_u (P,), R_t (L, PF)) of element e at the state (q, u, uhat); tt = (c, u_n, r_x)
    adds the implicit stage's time term to R_u (r_x may be None)."""
    wdet, dphix, phi, phif, psi, ndA, dA, src, uD, bnd = _element_geom(g, e)
    Qv, P = phi.shape
    L, Qf, _ = phif.shape
    PF = psi.shape[1]
    D = dphix.shape[2]
    Rq = np.zeros((D, P))
    Ru = np.zeros(P)
    Rt = np.zeros((L, PF))
    for k in range(Qv):
        uk = phi[k] @ u
        qk = np.array([phi[k] @ q[d] for d in range(D)])
        for d in range(D):
            Rq[d] += wdet[k] * (qk[d] * phi[k] + uk * dphix[k, :, d])
        Fk = flux(m, uk, qk)
        Ru -= wdet[k] * (dphix[k] @ Fk)
        Ru -= wdet[k] * src[k] * phi[k]
        if tt is not None:
            Ru += tt[0] * wdet[k] * (uk - phi[k] @ tt[1]) * phi[k]
    if tt is not None and tt[2] is not None:
        Ru += tt[2]
    for l in range(L):
        for k in range(Qf):
            uf = phif[l, k] @ u
            qf = np.array([phif[l, k] @ q[d] for d in range(D)])
            uhf = psi[k] @ uh[l]
            for d in range(D):
                Rq[d] -= uhf * ndA[l, k, d] * phif[l, k]
            fhat = flux(m, uhf, qf) @ ndA[l, k] + m["tau"] * (uf - uhf) * dA[l, k]
            Ru += fhat * phif[l, k]
            if bnd[l]:
                Rt[l] += dA[l, k] * (uhf - uD[l, k]) * psi[k]
            else:
                Rt[l] -= fhat * psi[k]
    return Rq, Ru, Rt


def jacobian(g, m, e, q, u, uh, c=0.0):
    """D (P, D*P), E (P, P), F (P, L*PF), G (L*PF, D*P), H (L*PF, P), J (L*PF, L*PF): the
    derivatives of R_u and R_t with respect to q (d, j), u and uhat (l, j); c = time-term factor."""
    wdet, dphix, phi, phif, psi, ndA, dA, src, uD, bnd = _element_geom(g, e)
    Qv, P = phi.shape
    L, Qf, _ = phif.shape
    PF = psi.shape[1]
    D = dphix.shape[2]
    tau = m["tau"]
    Dm = np.zeros((P, D, P))
    Em = np.zeros((P, P))
    Fm = np.zeros((P, L, PF))
    Gm = np.zeros((L, PF, D, P))
    Hm = np.zeros((L, PF, P))
    Jm = np.zeros((L, PF, L, PF))
    Fq = flux_dq(m, D)
    for k in range(Qv):
        uk = phi[k] @ u
        Fu = flux_du(m, uk, D)
        # -(dF/du phi_j, grad phi_i), -(dF/dq_d phi_j, grad phi_i)
        Em -= wdet[k] * np.outer(dphix[k] @ Fu, phi[k])
        Em += c * wdet[k] * np.outer(phi[k], phi[k])
        for d in range(D):
            Dm[:, d, :] -= wdet[k] * np.outer(dphix[k] @ Fq[:, d], phi[k])
    for l in range(L):
        for k in range(Qf):
            uhf = psi[k] @ uh[l]
            Fu = flux_du(m, uhf, D)
            n = ndA[l, k]
            # dfhat/du = tau, dfhat/dq_d = (dF/dq_d).n, dfhat/duhat = (dF/du).n - tau
            Em += tau * dA[l, k] * np.outer(phif[l, k], phif[l, k])
            for d in range(D):
                Dm[:, d, :] += (Fq[:, d] @ n) * np.outer(phif[l, k], phif[l, k])
            Fm[:, l, :] += (Fu @ n - tau * dA[l, k]) * np.outer(phif[l, k], psi[k])
            if bnd[l]:
                Jm[l, :, l, :] += dA[l, k] * np.outer(psi[k], psi[k])
            else:
                for d in range(D):
                    Gm[l, :, d, :] -= (Fq[:, d] @ n) * np.outer(psi[k], phif[l, k])
                Hm[l] -= tau * dA[l, k] * np.outer(psi[k], phif[l, k])
                Jm[l, :, l, :] -= (Fu @ n - tau * dA[l, k]) * np.outer(psi[k], psi[k])
    return (Dm.reshape(P, D * P), Em, Fm.reshape(P, L * PF), Gm.reshape(L * PF, D * P),
            Hm.reshape(L * PF, P), Jm.reshape(L * PF, L * PF))


def element_trace_values(uhat, e2f):
    """uhat_el[e][l][j] = uhat[e2f[e][l]][j] (canonical face order on both sides)."""
    return uhat[e2f]


def element_blocks(g, m, u, uhat, e2f, tt=None):
    """Every element's condensation inputs at the state (u, uhat) with consistent q:
    Minv, Bd, Cd, D, E, F, G, H, J, ru = -R_u, rt = -R_t, and q itself. tt = dict(c, u_prev (ne, P),
    r_extra (ne, P) or None) adds an implicit stage's time term."""
    ne, P = u.shape
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
                     ("G", Gm), ("H", Hm), ("J", Jm), ("ru", -Ru), ("rt", -Rt.ravel()), ("q", q)):
            out[k].append(v)
    return {k: np.array(v) for k, v in out.items()}
