"""Shared helpers for the tests: run the oracle pipeline on a generated problem."""
import numpy as np
import scipy.sparse.linalg as spla
import torch

import oracle
from workloads.blocks import _map_tables


def blocks_np(pb, e0=0, e1=None):
    return {k: v.cpu().numpy() for k, v in pb.element_blocks(e0, e1).items()}


def oracle_pipeline(pb, blk=None, perm=None):
    """Condense, assemble, direct solve, recover. Returns a dict of everything."""
    blk = blocks_np(pb) if blk is None else blk
    dims = pb.dims()
    Kb, rb = oracle.condense.condense(blk, dims)
    K, nbr, r = oracle.assemble.assemble(Kb, rb, pb.mesh.f2e, pb.mesh.e2f, dims, perm)
    A = oracle.assemble.to_sparse(K, nbr)
    x = spla.spsolve(A.tocsc(), r)
    dq, du = oracle.condense.recover(blk, x, pb.mesh.e2f, dims, perm)
    return dict(blk=blk, dims=dims, Kbar=Kb, rbar=rb, K=K, nbr=nbr, r=r, A=A, x=x, dq=dq, du=du)


def nodal_points(pb):
    Nn, _ = _map_tables(pb.etype, pb.enodes)
    return np.einsum("nv,evi->eni", Nn, pb.X.cpu().numpy())


def l2_error(pb, du, exact):
    """L2 norm of u_h - u over the mesh, with the generator's volume rule."""
    g = pb.geometry(0, pb.mesh.ne)
    phi = pb.phi.cpu().numpy()
    M = pb.M
    uh = np.einsum("qi,emi->eqm", phi, du.reshape(pb.mesh.ne, M, pb.npe))
    ue = exact(g["xq"]).cpu().numpy()
    w = g["wdet"].cpu().numpy()
    return float(np.sqrt(np.einsum("eq,eqm->", w, (uh - ue) ** 2)))
