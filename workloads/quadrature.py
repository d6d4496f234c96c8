"""Quadrature rules and nodal sets on reference cells (input generator, not the method).

Reference cells use [0,1] coordinates: the unit square/cube for quads/hexes,
and the unit simplex {x_i >= 0, sum x_i <= 1} for triangles/tets.
The paper only says integrals are evaluated "at quadrature points" (Section 4.1,
mass matrices M = Phi W); the rule used here is a fixed written choice:
tensor Gauss-Legendre with p+2 points per direction, and collapsed
Gauss-Jacobi (conical product) rules with p+2 points per direction on simplices.
"""
import numpy as np
from scipy.special import roots_jacobi


def gauss_legendre01(n):
    """n-point Gauss-Legendre rule on [0,1]; exact for degree 2n-1."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto01(p):
    """p+1 Gauss-Lobatto-Legendre nodes on [0,1] (p >= 1)."""
    if p == 1:
        z = np.array([-1.0, 1.0])
    else:
        dP = np.polynomial.legendre.Legendre.basis(p).deriv()
        z = np.concatenate([[-1.0], np.sort(dP.roots().real), [1.0]])
    return 0.5 * (z + 1.0)


def _jacobi01(n, alpha):
    """Rule for int_0^1 g(u) (1-u)^alpha du (alpha = 0, 1, 2)."""
    x, w = roots_jacobi(n, alpha, 0.0)
    u = 0.5 * (x + 1.0)
    return u, w * 0.5 ** (alpha + 1)


def tensor_rule(n, dim):
    x1, w1 = gauss_legendre01(n)
    grids = np.meshgrid(*([x1] * dim), indexing="ij")
    wg = np.meshgrid(*([w1] * dim), indexing="ij")
    # first coordinate fastest
    pts = np.stack([g.transpose().reshape(-1) for g in grids], axis=1)
    wts = np.prod(np.stack([g.transpose().reshape(-1) for g in wg], axis=1), axis=1)
    return pts, wts


def simplex_rule(n, dim):
    """Collapsed (Duffy/conical-product) rule on the unit simplex.

    triangle: (x,y) = (u, v(1-u)),           Jacobian (1-u)
    tet:      (x,y,z) = (u, v(1-u), w(1-u)(1-v)), Jacobian (1-u)^2 (1-v)
    The (1-u)^k factors are absorbed into Gauss-Jacobi weights.
    """
    if dim == 1:
        return gauss_legendre01(n)[0][:, None], gauss_legendre01(n)[1]
    if dim == 2:
        u, wu = _jacobi01(n, 1)
        v, wv = gauss_legendre01(n)
        U, V = np.meshgrid(u, v, indexing="ij")
        WU, WV = np.meshgrid(wu, wv, indexing="ij")
        pts = np.stack([U.ravel(), (V * (1 - U)).ravel()], axis=1)
        return pts, (WU * WV).ravel()
    if dim == 3:
        u, wu = _jacobi01(n, 2)
        v, wv = _jacobi01(n, 1)
        w, ww = gauss_legendre01(n)
        U, V, W = np.meshgrid(u, v, w, indexing="ij")
        WU, WV, WW = np.meshgrid(wu, wv, ww, indexing="ij")
        pts = np.stack([U.ravel(), (V * (1 - U)).ravel(), (W * (1 - U) * (1 - V)).ravel()], axis=1)
        return pts, (WU * WV * WW).ravel()
    raise ValueError(dim)


def cell_rule(etype, n):
    if etype == "quad":
        return tensor_rule(n, 2)
    if etype == "hex":
        return tensor_rule(n, 3)
    if etype == "tri":
        return simplex_rule(n, 2)
    if etype == "tet":
        return simplex_rule(n, 3)
    raise ValueError(etype)


def face_rule(etype, n):
    """Rule on the canonical face parameter domain of the cell's faces."""
    if etype in ("quad", "tri"):
        x, w = gauss_legendre01(n)
        return x[:, None], w
    if etype == "hex":
        return tensor_rule(n, 2)
    if etype == "tet":
        return simplex_rule(n, 2)
    raise ValueError(etype)
