"""HDG element blocks for one Newton linearisation (input generator, not the method).

For every element this produces the local matrices of the linearised system
(the 3x3 block form of Section 2.3) in the structure Section 4.1 uses:
  A = I_{MD} (x) M^e (mass), B_d, C_d (the q-equation),
  D, E, F, r_u (the u-equation), G, H, J, r_t (the trace equation).
The GPU path and the oracle both consume these arrays; neither condenses here.

Index conventions (C order, last index fastest):
  u dofs    (m, i)       -> m*P_E + i
  q dofs    (m, d, i)    -> (m*D + d)*P_E + i
  trace     (l, m, j)    -> (l*M + m)*P_F + j
  B_d[d][i][j] = int dphi_i/dx_d phi_j        (derivative on the test function)
  C_d[d][i][(l,j)] = -int_{face l} phi_i psi_j n_d
Trace rows use -<fhat, mu> on interior faces and <uhat - u_D, mu> on Dirichlet
faces (every boundary face is Dirichlet).
"""
import numpy as np
import torch

from . import basis as B
from . import quadrature as Q
from .mesh import LOCAL_FACES, REF_VERTS
from . import physics as Ph


def _frame_tables(etype):
    """All canonical face frames per local face: (nlfe, nframe) origins/axes."""
    R = REF_VERTS[etype]
    frames = []
    for l, loc in enumerate(LOCAL_FACES[etype]):
        fl = []
        if etype in ("quad", "tri"):
            for flip in (0, 1):
                i0, i1 = (0, 1) if flip == 0 else (1, 0)
                o = R[loc[i0]]
                fl.append((o, (R[loc[i1]] - o)[:, None]))
        elif etype == "hex":
            for k0 in range(4):
                for sw in (0, 1):
                    nb = [k0 ^ 1, k0 ^ 2]
                    if sw:
                        nb = nb[::-1]
                    o = R[loc[k0]]
                    fl.append((o, np.stack([R[loc[nb[0]]] - o, R[loc[nb[1]]] - o], axis=1)))
        elif etype == "tet":
            import itertools
            for order in itertools.permutations(range(3)):
                o = R[loc[order[0]]]
                fl.append((o, np.stack([R[loc[order[1]]] - o, R[loc[order[2]]] - o], axis=1)))
        frames.append(fl)
    return frames


def frame_ids(mesh):
    """Index of each (e, l) canonical frame inside _frame_tables(etype)[l]."""
    et = mesh.etype
    out = np.zeros((mesh.ne, mesh.nlfe), np.int64)
    for l, loc in enumerate(LOCAL_FACES[et]):
        gid = mesh.elems[:, list(loc)]
        if et in ("quad", "tri"):
            out[:, l] = (gid[:, 0] > gid[:, 1]).astype(np.int64)
        elif et == "hex":
            k0 = np.argmin(gid, axis=1)
            a = np.take_along_axis(gid, (k0 ^ 1)[:, None], 1)[:, 0]
            b = np.take_along_axis(gid, (k0 ^ 2)[:, None], 1)[:, 0]
            out[:, l] = k0 * 2 + (a > b)
        elif et == "tet":
            import itertools
            perms = {p: k for k, p in enumerate(itertools.permutations(range(3)))}
            order = np.argsort(gid, axis=1)
            out[:, l] = [perms[tuple(o)] for o in order]
    return out


def _map_tables(etype, xi):
    """Shape functions of the geometric map at reference points xi (n, dim)."""
    R = REF_VERTS[etype]
    dim = R.shape[1]
    nv = R.shape[0]
    if etype in ("tri", "tet"):
        N = np.zeros((xi.shape[0], nv))
        N[:, 0] = 1 - xi.sum(1)
        N[:, 1:] = xi
        dN = np.zeros((xi.shape[0], nv, dim))
        dN[:, 0, :] = -1
        for k in range(dim):
            dN[:, k + 1, k] = 1
        return N, dN
    N = np.ones((xi.shape[0], nv))
    dN = np.ones((xi.shape[0], nv, dim))
    for v in range(nv):
        bits = R[v]
        for d in range(dim):
            f = xi[:, d] if bits[d] else 1 - xi[:, d]
            df = 1.0 if bits[d] else -1.0
            N[:, v] *= f
            for g in range(dim):
                dN[:, v, g] *= (df if g == d else f)
    return N, dN


class HDGProblem:
    """A mesh, a polynomial degree and a physics model; generates element blocks."""

    def __init__(self, mesh, p, physics, device="cpu", nq=None):
        self.mesh = mesh
        self.p = p
        self.phys = physics
        self.device = torch.device(device)
        et = mesh.etype
        self.etype = et
        self.D = mesh.dim
        assert physics.D == self.D
        self.M = physics.M
        self.npe = B.npe(et, p)
        self.npf = B.npf(et, p)
        self.nlfe = mesh.nlfe
        self.nq_ = p + 2 if nq is None else nq
        self._tables()

    # ---- sizes -----------------------------------------------------------------
    @property
    def nu(self):
        return self.M * self.npe

    @property
    def nqd(self):
        return self.M * self.D * self.npe

    @property
    def nt(self):
        return self.M * self.npf * self.nlfe

    @property
    def nb(self):
        return self.M * self.npf

    def dims(self):
        return dict(ne=self.mesh.ne, nf=self.mesh.nf, ncomp=self.M, dim=self.D,
                    npe=self.npe, npf=self.npf, nlfe=self.nlfe)

    # ---- reference tables --------------------------------------------------------
    def _tables(self):
        et, p, dev = self.etype, self.p, self.device
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
        xv, wv = Q.cell_rule(et, self.nq_)
        phi, dphi = B.cell_basis(et, p, xv)
        Nv, dNv = _map_tables(et, xv)
        self.xv, self.wv, self.phi, self.dphi = t(xv), t(wv), t(phi), t(dphi)
        self.Nv, self.dNv = t(Nv), t(dNv)
        # faces
        sf, wf = Q.face_rule(et, self.nq_)
        psi = B.face_basis(et, p, sf)
        self.wf, self.psi = t(wf), t(psi)
        frames = _frame_tables(et)
        nfr = len(frames[0])
        Qf = sf.shape[0]
        phif = np.zeros((self.nlfe, nfr, Qf, self.npe))
        Nf = np.zeros((self.nlfe, nfr, Qf, REF_VERTS[et].shape[0]))
        dNf = np.zeros((self.nlfe, nfr, Qf, REF_VERTS[et].shape[0], self.D))
        axes = np.zeros((self.nlfe, nfr, self.D, self.D - 1))
        cen = REF_VERTS[et].mean(0)
        nref = np.zeros((self.nlfe, self.D))
        for l in range(self.nlfe):
            nref[l] = REF_VERTS[et][list(LOCAL_FACES[et][l])].mean(0) - cen
            for k, (o, A) in enumerate(frames[l]):
                xi = o[None, :] + sf @ A.T
                phif[l, k] = B.cell_basis(et, p, xi)[0]
                Nf[l, k], dNf[l, k] = _map_tables(et, xi)
                axes[l, k] = A
        self.phif_tab, self.Nf_tab, self.dNf_tab = t(phif), t(Nf), t(dNf)
        self.axes_tab, self.nref = t(axes), t(nref)
        self.fid = torch.as_tensor(frame_ids(self.mesh), device=dev)
        self.X = t(self.mesh.verts[self.mesh.elems])            # (ne, nv, dim)
        self.bnd = torch.as_tensor(self.mesh.boundary[self.mesh.e2f], device=dev)   # (ne, nlfe)
        # nodal points of the element basis and of the face basis (for interpolation)
        if et in ("quad", "hex"):
            self.enodes = B.tensor_nodes(p, self.D)
            self.fnodes = B.tensor_nodes(p, self.D - 1)
        else:
            self.enodes = B.simplex_nodes(p, self.D)
            self.fnodes = B.simplex_nodes(p, self.D - 1) if self.D == 3 else B.tensor_nodes(p, 1)

    # ---- geometry ----------------------------------------------------------------
    def geometry(self, e0, e1):
        X = self.X[e0:e1]
        xq = torch.einsum("qv,evi->eqi", self.Nv, X)
        J = torch.einsum("qvj,evi->eqij", self.dNv, X)
        det = torch.linalg.det(J)
        Jinv = torch.linalg.inv(J)
        dphix = torch.einsum("qpj,eqji->eqpi", self.dphi, Jinv)
        wdet = self.wv * det
        fid = self.fid[e0:e1]
        lidx = torch.arange(self.nlfe, device=self.device)[None, :]
        phif = self.phif_tab[lidx, fid]                    # (E, nlfe, Qf, npe)
        Nf = self.Nf_tab[lidx, fid]
        dNf = self.dNf_tab[lidx, fid]
        ax = self.axes_tab[lidx, fid]                      # (E, nlfe, D, D-1)
        xf = torch.einsum("elqv,evi->elqi", Nf, X)
        Jf = torch.einsum("elqvj,evi->elqij", dNf, X)
        tang = torch.einsum("elqij,eljk->elqik", Jf, ax)   # physical tangents (.., D, D-1)
        if self.D == 2:
            t0 = tang[..., 0]
            cand = torch.stack([t0[..., 1], -t0[..., 0]], dim=-1)
        else:
            cand = torch.cross(tang[..., 0], tang[..., 1], dim=-1)
        nout = torch.einsum("elqji,lj->elqi", torch.linalg.inv(Jf), self.nref)
        sgn = torch.sign((cand * nout).sum(-1, keepdim=True))
        ndA = cand * sgn * self.wf[None, None, :, None]
        dA = torch.linalg.norm(cand, dim=-1) * self.wf[None, None, :]
        return dict(xq=xq, det=det, wdet=wdet, dphix=dphix, phif=phif, xf=xf, ndA=ndA, dA=dA)

    # ---- linearisation state --------------------------------------------------------
    def _state(self, e0, e1, g):
        """Nodal u0 and uhat0 from the physics state; q0 from the q-equation so r_q = 0."""
        ph = self.phys
        E = e1 - e0
        M, D = self.M, self.D
        if ph.linear:
            z = torch.zeros
            return (z(E, M, self.npe, dtype=torch.float64, device=self.device),
                    z(E, self.nlfe, M, self.npf, dtype=torch.float64, device=self.device))
        X = self.X[e0:e1]
        en = torch.as_tensor(self.enodes, dtype=torch.float64, device=self.device)
        Nn, _ = _map_tables(self.etype, self.enodes)
        xn = torch.einsum("nv,evi->eni", torch.as_tensor(Nn, dtype=torch.float64, device=self.device), X)
        u0 = ph.state(xn).permute(0, 2, 1)                       # (E, M, npe)
        # face nodes: canonical params -> element reference -> physical
        fid = self.fid[e0:e1]
        frames = _frame_tables(self.etype)
        uh = torch.zeros(E, self.nlfe, M, self.npf, dtype=torch.float64, device=self.device)
        for l in range(self.nlfe):
            for k, (o, A) in enumerate(frames[l]):
                sel = (fid[:, l] == k).nonzero().flatten()
                if sel.numel() == 0:
                    continue
                xi = o[None, :] + self.fnodes @ A.T
                Nn, _ = _map_tables(self.etype, xi)
                xp = torch.einsum("nv,evi->eni", torch.as_tensor(Nn, dtype=torch.float64, device=self.device), X[sel])
                uh[sel, l] = ph.state(xp).permute(0, 2, 1)
        del en
        return u0, uh

    # ---- blocks -----------------------------------------------------------------
    def element_blocks(self, e0=0, e1=None):
        if e1 is None:
            e1 = self.mesh.ne
        g = self.geometry(e0, e1)
        ph = self.phys
        E = e1 - e0
        M, D, P, PF, L = self.M, self.D, self.npe, self.npf, self.nlfe
        tau = ph.tau
        phi, psi = self.phi, self.psi
        wdet, dphix, phif, ndA, dA = g["wdet"], g["dphix"], g["phif"], g["ndA"], g["dA"]
        intr = (~self.bnd[e0:e1]).to(torch.float64)             # (E, L)
        bndm = self.bnd[e0:e1].to(torch.float64)

        Mm = torch.einsum("eq,qi,qj->eij", wdet, phi, phi)
        Minv = torch.linalg.inv(Mm)
        Bd = torch.einsum("eq,eqid,qj->edij", wdet, dphix, phi)
        Cd = -torch.einsum("elqd,elqi,qj->edilj", ndA, phif, psi).reshape(E, D, P, L * PF)

        # state at quadrature points
        u0n, uhn = self._state(e0, e1, g)
        # q0 = -Minv (B_d u0_m + C_d uhat0_m)  (so that the q residual vanishes)
        uh_m = uhn.permute(0, 2, 1, 3).reshape(E, M, L * PF)    # (E, M, L*PF)
        t = torch.einsum("edij,emj->emdi", Bd, u0n) + torch.einsum("edil,eml->emdi", Cd, uh_m)
        q0n = -torch.einsum("eij,emdj->emdi", Minv, t)            # (E, M, D, npe)
        uq = torch.einsum("qi,emi->eqm", phi, u0n)
        qq = torch.einsum("qi,emdi->eqmd", phi, q0n)
        uf = torch.einsum("elqi,emi->elqm", phif, u0n)
        qf = torch.einsum("elqi,emdi->elqmd", phif, q0n)
        uhf = torch.einsum("qj,elmj->elqm", psi, uhn)

        F0, Fu, Fq = ph.flux_jacobians(uq, qq)                   # volume
        Ff, Fuf, Fqf = ph.flux_jacobians(uhf, qf)                # faces: F(uhat, q)
        s0 = ph.source(g["xq"])

        eyeM = torch.eye(M, dtype=torch.float64, device=self.device)
        # ---- D: d R_u / d q
        X1 = torch.einsum("eq,eqaxbd,eqix->eqaibd", wdet, Fq, dphix)
        Dm = -torch.einsum("eqaibd,qj->eaibdj", X1, phi)
        Y = torch.einsum("elqaxbd,elqx->elqabd", Fqf, ndA)
        Dm = Dm + torch.einsum("elqabd,elqi,elqj->eaibdj", Y, phif, phif)
        Dm = Dm.reshape(E, M * P, M * D * P)
        # ---- E
        massf = torch.einsum("elq,elqi,elqj->eij", dA, phif, phif)
        Em = torch.zeros(E, M, P, M, P, dtype=torch.float64, device=self.device)
        if ph.dt is not None:
            Em = Em + (1.0 / ph.dt) * torch.einsum("ab,eij->eaibj", eyeM, Mm)
        X2 = torch.einsum("eq,eqaxb,eqix->eqaib", wdet, Fu, dphix)
        Em = Em - torch.einsum("eqaib,qj->eaibj", X2, phi)
        Em = Em + tau * torch.einsum("ab,eij->eaibj", eyeM, massf)
        Em = Em.reshape(E, M * P, M * P)
        # ---- F
        Z = torch.einsum("elqaxb,elqx->elqab", Fuf, ndA) - tau * eyeM * dA[..., None, None]
        Fm = torch.einsum("elqab,elqi,qj->eailbj", Z, phif, psi).reshape(E, M * P, L * M * PF)
        # ---- r_u = -R_u
        fhat = torch.einsum("elqax,elqx->elqa", Ff, ndA) + tau * (uf - uhf) * dA[..., None]
        Ru = -torch.einsum("eq,eqa,qi->eai", wdet, s0, phi)
        Ru = Ru - torch.einsum("eq,eqax,eqix->eai", wdet, F0, dphix)
        Ru = Ru + torch.einsum("elqa,elqi->eai", fhat, phif)
        if ph.dt is not None:
            pass    # (u0 - u_prev)/dt = 0: the previous step equals the state
        ru = (-Ru).reshape(E, M * P)
        # ---- trace rows
        Gm = -torch.einsum("el,elqabd,elqk,qj->elajbdk", intr, Y, phif, psi)
        Gm = Gm.reshape(E, L * M * PF, M * D * P)
        Hm = -tau * torch.einsum("el,ab,elq,elqk,qj->elajbk", intr, eyeM, dA, phif, psi)
        Hm = Hm.reshape(E, L * M * PF, M * P)
        Zt = tau * eyeM * dA[..., None, None] - torch.einsum("elqaxb,elqx->elqab", Fuf, ndA)
        Jint = torch.einsum("el,elqab,qk,qj->elajbk", intr, Zt, psi, psi)
        Jbnd = torch.einsum("el,ab,elq,qk,qj->elajbk", bndm, eyeM, dA, psi, psi)
        Jl = Jint + Jbnd                                           # (E, L, M, PF, M, PF)
        Jm = torch.zeros(E, L, M, PF, L, M, PF, dtype=torch.float64, device=self.device)
        for l in range(L):
            Jm[:, l, :, :, l] = Jl[:, l]
        Jm = Jm.reshape(E, L * M * PF, L * M * PF)
        uD = ph.dirichlet(g["xf"])                                 # (E, L, Qf, M)
        Rt_int = -torch.einsum("elqa,qj->elaj", fhat, psi)
        Rt_bnd = torch.einsum("elq,elqa,qj->elaj", dA, uhf - uD, psi)
        Rt = intr[..., None, None] * Rt_int + bndm[..., None, None] * Rt_bnd
        rt = (-Rt).reshape(E, L * M * PF)
        out = dict(Minv=Minv, Bd=Bd, Cd=Cd, D=Dm, E=Em, F=Fm, G=Gm, H=Hm, J=Jm, ru=ru, rt=rt)
        return {k: v.contiguous() for k, v in out.items()}

    def newton_inputs(self):
        """Inputs of the element residual/Jacobian generation for scalar convection-diffusion
        models (Poisson, Burgers): the mesh's quadrature geometry, the reference tables, the
        source and Dirichlet data at quadrature points, the model coefficients and the initial
        state (nodal u per element, canonical face values uhat per face). Float64 tensors on
        the problem's device; bnd is int32."""
        assert self.M == 1 and hasattr(self.phys, "conv_diff")
        ne, L = self.mesh.ne, self.nlfe
        g = self.geometry(0, ne)
        u0, uh_el = self._state(0, ne, g)
        f2e = torch.as_tensor(self.mesh.f2e, device=self.device).long()
        uhat0 = uh_el[f2e[:, 0], f2e[:, 1], 0].contiguous()              # (nf, npf)
        cd = self.phys.conv_diff()
        return dict(
            wdet=g["wdet"].contiguous(), dphix=g["dphix"].contiguous(), phi=self.phi.contiguous(),
            phif=g["phif"].contiguous(), psi=self.psi.contiguous(), ndA=g["ndA"].contiguous(),
            dA=g["dA"].contiguous(), src=self.phys.source(g["xq"])[..., 0].contiguous(),
            uD=self.phys.dirichlet(g["xf"])[..., 0].contiguous(),
            bnd=self.bnd.to(torch.int32).contiguous(), nqv=int(self.wv.shape[0]), nqf=int(self.wf.shape[0]),
            nu=float(cd["nu"]), tau=float(self.phys.tau), beta=list(cd["beta"]), gamma=list(cd["gamma"]),
            u0=u0[:, 0].contiguous(), uhat0=uhat0)

    def newton_inputs_sys(self):
        """Inputs of the element residual/Jacobian generation for the M-component models
        (elasticity, Navier-Stokes): the mesh's quadrature geometry and reference tables as in
        newton_inputs, the source src (ne, nqv, M) and Dirichlet data uD (ne, nlfe, nqf, M) at
        quadrature points, the model description and the linearisation state as the initial
        state: u0 (ne, M, npe) nodal, uhat0 (nf, M, npf) canonical face values."""
        ph = self.phys
        assert self.M > 1
        ne = self.mesh.ne
        g = self.geometry(0, ne)
        u0, uh_el = self._state(0, ne, g)
        f2e = torch.as_tensor(self.mesh.f2e, device=self.device).long()
        uhat0 = uh_el[f2e[:, 0], f2e[:, 1]].contiguous()                 # (nf, M, npf)
        if isinstance(ph, Ph.Elasticity):
            model = dict(kind="elasticity", tau=float(ph.tau), lam=float(ph.lam), mu=float(ph.mu))
        else:
            model = dict(kind="navier_stokes", tau=float(ph.tau), Re=float(ph.Re), Pr=float(ph.Pr),
                         gamma=float(ph.gamma), dt=float(ph.dt))
        return dict(
            wdet=g["wdet"].contiguous(), dphix=g["dphix"].contiguous(), phi=self.phi.contiguous(),
            phif=g["phif"].contiguous(), psi=self.psi.contiguous(), ndA=g["ndA"].contiguous(),
            dA=g["dA"].contiguous(), src=ph.source(g["xq"]).contiguous(),
            uD=ph.dirichlet(g["xf"]).contiguous(),
            bnd=self.bnd.to(torch.int32).contiguous(), nqv=int(self.wv.shape[0]), nqf=int(self.wf.shape[0]),
            model=model, u0=u0.contiguous(), uhat0=uhat0)

    def state_dofs(self, e0=0, e1=None):
        """Nodal linearisation state (u0 (E,M,npe), uhat0 (E,L,M,npf))."""
        if e1 is None:
            e1 = self.mesh.ne
        return self._state(e0, e1, None)
