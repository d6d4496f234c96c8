"""Polynomial bases on reference cells and faces (input generator, not the method).

Element space: Q^p (tensor Lagrange at Gauss-Lobatto nodes) on quads/hexes,
P^p (Lagrange at equispaced nodes) on triangles/tets. Face space: the same
family on the face's canonical parameter domain. The paper writes complete
polynomials P^k for every cell (Section 2.1); tensor cells use Q^p here so that
a hex face of degree 3 carries 16 dofs.
"""
import itertools
import numpy as np

from .quadrature import gauss_lobatto01


def lagrange1d(nodes, x):
    """Values and first derivatives of the 1D Lagrange basis on `nodes` at `x`.

    Returns (V, dV) with shape (len(x), len(nodes)).
    """
    nodes = np.asarray(nodes, float)
    x = np.asarray(x, float)
    n = len(nodes)
    V = np.ones((len(x), n))
    dV = np.zeros((len(x), n))
    for k in range(n):
        others = [m for m in range(n) if m != k]
        denom = np.prod([nodes[k] - nodes[m] for m in others])
        for m in others:
            V[:, k] *= (x - nodes[m])
        for drop in others:
            term = np.ones(len(x))
            for m in others:
                if m != drop:
                    term *= (x - nodes[m])
            dV[:, k] += term
        V[:, k] /= denom
        dV[:, k] /= denom
    return V, dV


def tensor_basis(p, dim, pts):
    """Q^p Lagrange basis (GLL nodes, first index fastest) at points (n, dim).

    Returns phi (n, P) and dphi (n, P, dim).
    """
    z = gauss_lobatto01(p)
    ones = [lagrange1d(z, pts[:, d]) for d in range(dim)]
    n = pts.shape[0]
    P = (p + 1) ** dim
    phi = np.ones((n, P))
    dphi = np.ones((n, P, dim))
    for idx in range(P):
        ijk = [(idx // (p + 1) ** d) % (p + 1) for d in range(dim)]
        for d in range(dim):
            V, dV = ones[d]
            phi[:, idx] *= V[:, ijk[d]]
            for e in range(dim):
                dphi[:, idx, e] *= (dV[:, ijk[d]] if d == e else V[:, ijk[d]])
    return phi, dphi


def tensor_nodes(p, dim):
    z = gauss_lobatto01(p)
    P = (p + 1) ** dim
    out = np.zeros((P, dim))
    for idx in range(P):
        for d in range(dim):
            out[idx, d] = z[(idx // (p + 1) ** d) % (p + 1)]
    return out


def simplex_exponents(p, dim):
    return [e for e in itertools.product(range(p + 1), repeat=dim) if sum(e) <= p]


def simplex_nodes(p, dim):
    """Equispaced nodes of the unit simplex, ordered like simplex_exponents."""
    return np.array([[e[d] / p for d in range(dim)] for e in simplex_exponents(p, dim)], float)


def _monomials(exps, pts):
    n, dim = pts.shape
    V = np.ones((n, len(exps)))
    dV = np.zeros((n, len(exps), dim))
    for k, e in enumerate(exps):
        for d in range(dim):
            V[:, k] *= pts[:, d] ** e[d]
        for g in range(dim):
            if e[g] == 0:
                continue
            t = np.full(n, float(e[g]))
            for d in range(dim):
                t = t * (pts[:, d] ** (e[d] - 1 if d == g else e[d]))
            dV[:, k, g] = t
    return V, dV


def simplex_basis(p, dim, pts):
    """P^p Lagrange basis at equispaced simplex nodes, evaluated at pts."""
    exps = simplex_exponents(p, dim)
    nodes = simplex_nodes(p, dim)
    Vn, _ = _monomials(exps, nodes)
    C = np.linalg.inv(Vn)          # columns: coefficients of each nodal function
    V, dV = _monomials(exps, pts)
    phi = V @ C
    dphi = np.einsum("nkd,ki->nid", dV, C)
    return phi, dphi


def cell_basis(etype, p, pts):
    if etype == "quad":
        return tensor_basis(p, 2, pts)
    if etype == "hex":
        return tensor_basis(p, 3, pts)
    if etype == "tri":
        return simplex_basis(p, 2, pts)
    if etype == "tet":
        return simplex_basis(p, 3, pts)
    raise ValueError(etype)


def face_basis(etype, p, fpts):
    """Trace basis on the canonical face parameter domain of an `etype` cell."""
    if etype in ("quad", "tri"):
        return tensor_basis(p, 1, fpts)[0]
    if etype == "hex":
        return tensor_basis(p, 2, fpts)[0]
    if etype == "tet":
        return simplex_basis(p, 2, fpts)[0]
    raise ValueError(etype)


def npe(etype, p):
    return {"quad": (p + 1) ** 2, "hex": (p + 1) ** 3,
            "tri": (p + 1) * (p + 2) // 2, "tet": (p + 1) * (p + 2) * (p + 3) // 6}[etype]


def npf(etype, p):
    return {"quad": p + 1, "tri": p + 1, "hex": (p + 1) ** 2,
            "tet": (p + 1) * (p + 2) // 2}[etype]
