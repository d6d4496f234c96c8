"""Conservation-law models F(u, q), s(x) used to generate element blocks.

The paper's general frame is du/dt + div F(u, grad u) = s (Section 2.1). Each
model supplies the flux F (M x D per point), a source depending on position
only, the global Lax-Friedrichs constant tau (S = tau I), the Dirichlet data,
and the linearisation state. Fluxes are written on batched torch tensors so
their Jacobians can be taken with forward-mode autodiff.
"""
import math
import torch


class Physics:
    M = 1
    D = 2
    tau = 1.0
    dt = None          # backward-Euler step (None: steady)
    linear = True      # linear flux and zero linearisation state

    def flux(self, u, q):          # u (..., M), q (..., M, D) -> (..., M, D)
        raise NotImplementedError

    def source(self, x):           # x (..., D) -> (..., M)
        return torch.zeros(x.shape[:-1] + (self.M,), dtype=x.dtype, device=x.device)

    def dirichlet(self, x):        # boundary data u_D
        return torch.zeros(x.shape[:-1] + (self.M,), dtype=x.dtype, device=x.device)

    def state(self, x):            # linearisation point u0 (nodal interpolation)
        return torch.zeros(x.shape[:-1] + (self.M,), dtype=x.dtype, device=x.device)

    def flux_jacobians(self, u, q):
        """Returns F, dF/du (..., M, D, M), dF/dq (..., M, D, M, D)."""
        sh = u.shape[:-1]
        M, D = self.M, self.D
        uf = u.reshape(-1, M)
        qf = q.reshape(-1, M, D)

        def f(uu, qq):
            return self.flux(uu, qq)
        F = self.flux(uf, qf)
        Fu = torch.func.vmap(torch.func.jacfwd(f, argnums=0))(uf, qf)
        Fq = torch.func.vmap(torch.func.jacfwd(f, argnums=1))(uf, qf)
        return F.reshape(sh + (M, D)), Fu.reshape(sh + (M, D, M)), Fq.reshape(sh + (M, D, M, D))


class Poisson(Physics):
    """-Laplace(u) = f: F = -q, s = f."""

    def __init__(self, dim=2, tau=1.0, exact=None, forcing=None):
        self.D = dim
        self.M = 1
        self.tau = tau
        self._exact = exact
        self._forcing = forcing

    def flux(self, u, q):
        return -q

    def conv_diff(self):
        """F = beta u^2/2 + gamma u - nu q with these coefficients (see Burgers)."""
        return dict(nu=1.0, beta=[0.0] * self.D, gamma=[0.0] * self.D)

    def source(self, x):
        if self._forcing is not None:
            return self._forcing(x)
        if self._exact is None:
            return super().source(x)
        return laplacian_forcing(self._exact, x)

    def dirichlet(self, x):
        if self._exact is None:
            return super().dirichlet(x)
        return self._exact(x)

    def flux_jacobians(self, u, q):
        sh = u.shape[:-1]
        D = self.D
        Fu = torch.zeros(sh + (1, D, 1), dtype=u.dtype, device=u.device)
        eye = torch.eye(D, dtype=u.dtype, device=u.device)
        Fq = (-eye).reshape(1, D, 1, D).expand(sh + (1, D, 1, D))
        return self.flux(u, q), Fu, Fq


def laplacian_forcing(exact, x):
    """f = -Laplace(exact) evaluated with autodiff (per component)."""
    xs = x.detach().reshape(-1, x.shape[-1]).clone().requires_grad_(True)
    with torch.enable_grad():
        u = exact(xs)
        out = []
        for m in range(u.shape[-1]):
            g = torch.autograd.grad(u[:, m].sum(), xs, create_graph=True)[0]
            lap = sum(torch.autograd.grad(g[:, d].sum(), xs, retain_graph=True)[0][:, d]
                      for d in range(xs.shape[1]))
            out.append(-lap)
    return torch.stack(out, dim=-1).detach().reshape(x.shape[:-1] + (u.shape[-1],))


class Elasticity(Physics):
    """Linear elasticity: F = -sigma(q), sigma = lam tr(eps) I + 2 mu eps, eps = sym(q)."""

    def __init__(self, E=1.0, nu=0.3, tau=1.0, exact=None):
        self.M = 3
        self.D = 3
        self.tau = tau
        self.lam = E * nu / ((1 + nu) * (1 - 2 * nu))
        self.mu = E / (2 * (1 + nu))
        self._exact = exact

    def stress(self, q):
        tr = q.diagonal(dim1=-2, dim2=-1).sum(-1)
        eye = torch.eye(3, dtype=q.dtype, device=q.device)
        return self.lam * tr[..., None, None] * eye + self.mu * (q + q.transpose(-1, -2))

    def flux(self, u, q):
        return -self.stress(q)

    def flux_jacobians(self, u, q):
        sh = u.shape[:-1]
        d = torch.eye(3, dtype=u.dtype, device=u.device)
        # dsigma_{ae}/dq_{bd} = lam d_ae d_bd + mu (d_ab d_ed + d_ad d_eb)
        C = (self.lam * torch.einsum("ae,bd->aebd", d, d)
             + self.mu * (torch.einsum("ab,ed->aebd", d, d) + torch.einsum("ad,eb->aebd", d, d)))
        Fq = (-C).expand(sh + (3, 3, 3, 3))
        Fu = torch.zeros(sh + (3, 3, 3), dtype=u.dtype, device=u.device)
        return self.flux(u, q), Fu, Fq

    def source(self, x):
        if self._exact is None:
            return super().source(x)
        # f = -div sigma(grad u)
        xs = x.detach().reshape(-1, 3).clone().requires_grad_(True)
        with torch.enable_grad():
            u = self._exact(xs)
            G = torch.stack([torch.autograd.grad(u[:, m].sum(), xs, create_graph=True)[0]
                             for m in range(3)], dim=1)          # (n, 3, 3) = du_m/dx_d
            S = self.stress(G)
            div = torch.stack([sum(torch.autograd.grad(S[:, a, e].sum(), xs, retain_graph=True)[0][:, e]
                                   for e in range(3)) for a in range(3)], dim=-1)
        return (-div).detach().reshape(x.shape[:-1] + (3,))

    def dirichlet(self, x):
        if self._exact is None:
            return super().dirichlet(x)
        return self._exact(x)


def elasticity_manufactured(x):
    """u_c = sin(pi(x+c/3)) sin(pi(y+c/5)) sin(pi(z+c/7)), c = 0, 1, 2."""
    pi = math.pi
    comps = [torch.sin(pi * (x[..., 0] + c / 3)) * torch.sin(pi * (x[..., 1] + c / 5))
             * torch.sin(pi * (x[..., 2] + c / 7)) for c in range(3)]
    return torch.stack(comps, dim=-1)


class Burgers(Physics):
    """2D viscous Burgers du/dy + d(u^2/2)/dx - nu Lap u = 0 as a conservation law:
    F = (u^2/2 - nu q_x, u - nu q_y), linearised about the state u0(x)."""

    def __init__(self, nu=0.01, tau=1.0, forcing=None, u0=None, uD=None):
        self.M = 1
        self.D = 2
        self.nu = nu
        self.tau = tau
        self.linear = False
        self._forcing = forcing
        self._u0 = u0 if u0 is not None else (lambda x: (1 - 2 * x[..., :1]))
        self._uD = uD if uD is not None else (lambda x: (1 - 2 * x[..., :1]))

    def flux(self, u, q):
        fx = 0.5 * u[..., 0] ** 2 - self.nu * q[..., 0, 0]
        fy = u[..., 0] - self.nu * q[..., 0, 1]
        return torch.stack([fx, fy], dim=-1)[..., None, :]

    def conv_diff(self):
        """Scalar convection-diffusion form F_x = beta_x u^2/2 + gamma_x u - nu q_x."""
        return dict(nu=self.nu, beta=[1.0, 0.0], gamma=[0.0, 1.0])

    def source(self, x):
        if self._forcing is None:
            return super().source(x)
        return self._forcing(x)

    def dirichlet(self, x):
        return self._uD(x)

    def state(self, x):
        return self._u0(x)


class NavierStokes(Physics):
    """Compressible Navier-Stokes in conservative variables (rho, rho v, rho E), 3D.

    Nondimensional freestream rho = 1, |v| = 1 along x, p = 1/(gamma Mach^2);
    mu = 1/Re, Stokes hypothesis, heat flux kappa = mu gamma/(Pr (gamma-1)) * grad(e),
    with e = p/((gamma-1) rho) the specific internal energy. Backward Euler with step dt.
    The state is freestream plus seeded Gaussian bumps in the primitive variables.
    """

    def __init__(self, Re=1000.0, Mach=0.5, dt=0.07, Pr=0.72, gamma=1.4, bumps=None):
        self.M = 5
        self.D = 3
        self.Re, self.Mach, self.Pr, self.gamma = Re, Mach, Pr, gamma
        self.dt = dt
        self.linear = False
        self.p_inf = 1.0 / (gamma * Mach ** 2)
        self.tau = 1.0 + 1.0 / Mach        # |v_inf| + c_inf
        self.bumps = bumps                 # list of (centres (8,3), signs (8,)) per primitive var

    def primitive_to_conservative(self, r, v, p):
        g = self.gamma
        E = p / ((g - 1) * r) + 0.5 * (v * v).sum(-1)
        return torch.cat([r[..., None], r[..., None] * v, (r * E)[..., None]], dim=-1)

    def freestream(self, x):
        sh = x.shape[:-1]
        r = torch.ones(sh, dtype=x.dtype, device=x.device)
        v = torch.zeros(sh + (3,), dtype=x.dtype, device=x.device)
        v[..., 0] = 1.0
        p = torch.full(sh, self.p_inf, dtype=x.dtype, device=x.device)
        return r, v, p

    def state(self, x):
        r, v, p = self.freestream(x)
        if self.bumps is not None:
            scale = [1.0, 1.0, 1.0, 1.0, self.p_inf]
            fields = []
            for k, (cen, sgn) in enumerate(self.bumps):
                c = torch.as_tensor(cen, dtype=x.dtype, device=x.device)
                s = torch.as_tensor(sgn, dtype=x.dtype, device=x.device)
                d2 = ((x[..., None, :] - c) ** 2).sum(-1)
                g = (s * torch.exp(-d2 / (2 * 0.1 ** 2))).sum(-1)
                fields.append(0.05 * scale[k] * g / float(self._bump_norm[k]))
            r = r + fields[0]
            v = v + torch.stack(fields[1:4], dim=-1)
            p = p + fields[4]
        return self.primitive_to_conservative(r, v, p)

    def set_bump_norms(self, norms):
        self._bump_norm = norms

    def dirichlet(self, x):
        return self.primitive_to_conservative(*self.freestream(x))

    def flux(self, u, q):
        g = self.gamma
        r = u[..., 0]
        m = u[..., 1:4]
        rE = u[..., 4]
        v = m / r[..., None]
        p = (g - 1) * (rE - 0.5 * (m * v).sum(-1))
        # convective flux F_c[a][e]
        Fc_r = m
        Fc_m = m[..., :, None] * v[..., None, :] + p[..., None, None] * torch.eye(3, dtype=u.dtype, device=u.device)
        Fc_E = (rE + p)[..., None] * v
        # gradients of primitives from conservative gradients q = grad u
        gr = q[..., 0, :]                      # (.., D)
        gm = q[..., 1:4, :]                    # (.., 3, D)
        gE = q[..., 4, :]
        gv = (gm - v[..., :, None] * gr[..., None, :]) / r[..., None, None]
        mu = 1.0 / self.Re
        div = gv.diagonal(dim1=-2, dim2=-1).sum(-1)
        tau_v = mu * (gv + gv.transpose(-1, -2)) - (2.0 / 3.0) * mu * div[..., None, None] * torch.eye(3, dtype=u.dtype, device=u.device)
        # e = E - |v|^2/2, grad e = (grad(rE) - E grad r)/r - v . grad v
        E = rE / r
        ge = (gE - E[..., None] * gr) / r[..., None] - (v[..., :, None] * gv).sum(-2)
        kappa = mu * g / (self.Pr * (g - 1)) * (g - 1)   # in terms of grad e: kappa_T grad T with T ~ (g-1) e
        heat = kappa * ge
        Fv_r = torch.zeros_like(Fc_r)
        Fv_m = tau_v
        Fv_E = (tau_v * v[..., :, None]).sum(-2) + heat
        Fr = (Fc_r - Fv_r)[..., None, :]
        Fm = Fc_m - Fv_m
        FE = (Fc_E - Fv_E)[..., None, :]
        return torch.cat([Fr, Fm, FE], dim=-2)
