"""The five synthetic workloads (seeded) and small variants of them.

Every workload is synthetic: the paper's meshes and scripts are not available.
  C1  2D Poisson, unit square, 8x8 quads jittered +-0.1h (seed 1), p=2, tau=1,
      u = sin(pi x) sin(pi y), Dirichlet.
  C2  3D linear elasticity (E=1, nu=0.3), unit cube, 24^3 hexes jittered +-0.05h
      (seed 2), p=3, tau=1, manufactured smooth displacement, Dirichlet.
  C3  3D compressible Navier-Stokes linearisation (Re=1000, Mach 0.5) on 16^3
      hexes, p=2, freestream + seeded Gaussian bumps (5%), backward Euler.
  C4  512 independent 2D Poisson/Burgers instances, mixed tri/quad meshes.
  C5  3D Navier-Stokes on 32^3 x 6 Kuhn tets (jitter +-0.1h, seed 5), p=2.
"""
import math
import numpy as np
import torch

from . import mesh as Mh
from . import physics as Ph
from .blocks import HDGProblem


def poisson_sin(x):
    return (torch.sin(math.pi * x[..., 0]) * torch.sin(math.pi * x[..., 1]))[..., None]


def poisson_sin_forcing(x):
    return (2 * math.pi ** 2 * torch.sin(math.pi * x[..., 0]) * torch.sin(math.pi * x[..., 1]))[..., None]


def c1(n=8, p=2, amp=0.1, seed=1, device="cpu"):
    m = Mh.structured_quads(n, amp, seed)
    ph = Ph.Poisson(dim=2, tau=1.0, exact=poisson_sin, forcing=poisson_sin_forcing)
    return HDGProblem(m, p, ph, device=device)


def c2(n=24, p=3, amp=0.05, seed=2, device="cpu"):
    m = Mh.structured_hexes(n, amp, seed)
    ph = Ph.Elasticity(E=1.0, nu=0.3, tau=1.0, exact=Ph.elasticity_manufactured)
    return HDGProblem(m, p, ph, device=device)


def ns_bumps(seed):
    """8 Gaussian bumps per primitive variable: centres U[0.2,0.8]^3, signs +-1."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(5):
        c = rng.uniform(0.2, 0.8, size=(8, 3))
        s = rng.choice([-1.0, 1.0], size=8)
        out.append((c, s))
    return out


def _bump_norms(bumps, npts=32):
    """max |sum of bumps| over a sampling grid (normalises each field to 1)."""
    ax = (np.arange(npts) + 0.5) / npts
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    out = []
    for c, s in bumps:
        d2 = ((g[:, None, :] - c[None]) ** 2).sum(-1)
        out.append(np.abs((s * np.exp(-d2 / (2 * 0.1 ** 2))).sum(-1)).max())
    return out


def navier_stokes(seed, dt):
    b = ns_bumps(seed)
    ph = Ph.NavierStokes(Re=1000.0, Mach=0.5, dt=dt, bumps=b)
    ph.set_bump_norms(_bump_norms(b))
    return ph


def c3(n=16, p=2, seed=3, device="cpu"):
    m = Mh.structured_hexes(n, 0.0, seed)
    dt = 10.0 * (1.0 / n) / ((p + 1) * (1.0 + 1.0 / 0.5))
    return HDGProblem(m, p, navier_stokes(seed, dt), device=device)


def c5(n=32, p=2, amp=0.1, seed=5, device="cpu"):
    m = Mh.kuhn_tets(n, amp, seed)
    dt = 10.0 * (1.0 / n) / ((p + 1) * (1.0 + 1.0 / 0.5))
    return HDGProblem(m, p, navier_stokes(seed, dt), device=device)


def c4_instance(i, base_seed=4, device="cpu"):
    """Instance i of the batched workload: type, size, degree, PDE drawn from seed 4e6+i."""
    rng = np.random.default_rng(4_000_000 + i)
    etype = "quad" if rng.random() < 0.5 else "tri"
    n = int(rng.integers(4, 33))
    p = int(rng.integers(1, 5))
    pde = "poisson" if rng.random() < 0.5 else "burgers"
    a = rng.standard_normal(4)
    kx = rng.integers(1, 4, size=4)
    ky = rng.integers(1, 4, size=4)

    def forcing(x):
        f = sum(float(a[k]) * torch.sin(int(kx[k]) * math.pi * x[..., 0]) * torch.sin(int(ky[k]) * math.pi * x[..., 1])
                for k in range(4))
        return f[..., None]
    m = Mh.structured_quads(n, 0.0, base_seed) if etype == "quad" else Mh.structured_tris(n, 0.0, base_seed)
    if pde == "poisson":
        ph = Ph.Poisson(dim=2, tau=1.0, forcing=forcing)
    else:
        ph = Ph.Burgers(nu=0.01, tau=1.0, forcing=forcing)
    return HDGProblem(m, p, ph, device=device)
