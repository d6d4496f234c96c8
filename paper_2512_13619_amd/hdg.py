"""ctypes binding of libhdg.so (include/hdg.h): argument marshalling only.

Device arrays are torch tensors on a ROCm device; the binding checks dtype,
contiguity, device and sizes and passes raw pointers. Every computation runs in
the library's HIP kernels; there is no fallback: if libhdg.so is missing or the
GPU is absent, calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdg.so")

HDG_OK, HDG_NOT_CONVERGED = 0, 1
PREC = {"none": 0, "bj": 1, "bj_poly": 2, "bj_cheb": 3, "asm": 4, "asm_poly": 5, "asm_cheb": 6, "ilu_asm": 7}
ORTH = {"cgs2": 0, "cgs": 1, "mgs": 2, "dcgs2": 3}
FALLBACK = {"pp_breakdown": 1, "pp_small_ritz": 2, "pp_no_interval": 4, "pp_to_base": 8, "mixed_to_fp64": 16, "stagnated": 32, "pp_added_root": 64}
PRECISION = {"fp64": 0, "mixed": 1}

# every symbol declared in include/hdg.h
SYMBOLS = ["hdg_create", "hdg_destroy", "hdg_set_stream", "hdg_last_error", "hdg_release_workspace",
           "hdg_local_size", "hdg_condense", "hdg_condense_keep", "hdg_condense_rhs", "hdg_assemble_blocks",
           "hdg_assemble_rhs", "hdg_solve_opts_default", "hdg_gmres_solve",
           "hdg_recover_local", "hdg_newton_update", "hdg_element_blocks", "hdg_residual_norm", "hdg_residual_norm_noalloc", "hdg_element_blocks_sys", "hdg_autotune", "hdg_tune_table", "hdg_asm_setup", "hdg_asm_apply", "hdg_matvec", "hdg_bj_setup",
           "hdg_bj_apply", "hdg_poly_apply", "hdg_cheb_apply", "hdg_hessenberg_eigvals", "hdg_harmonic_ritz", "hdg_poly_roots", "hdg_batch_create", "hdg_batch_destroy",
           "hdg_batch_offsets", "hdg_batch_tuned_grid", "hdg_condense_batch", "hdg_assemble_batch",
           "hdg_gmres_solve_batch", "hdg_recover_batch", "hdg_element_blocks_batch", "hdg_residual_norm_batch",
           "hdg_newton_update_batch", "hdg_ilu_asm_create", "hdg_ilu_asm_destroy", "hdg_ilu_asm_apply"]

BATCH_ARRAYS = ["Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt", "Kbar", "rbar", "local", "du", "dq",
                "K", "nbr", "vec", "f2e", "e2f", "binv"]


class HdgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hdg status {status}: {msg}")
        self.status = status


class Dims(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("ne", "nf", "ncomp", "dim", "npe", "npf", "nlfe")]


class ElemBlocks(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt")]


class ElemGeom(ctypes.Structure):
    _fields_ = [("nqv", ctypes.c_int32), ("nqf", ctypes.c_int32)] + \
        [(n, ctypes.c_void_p) for n in ("wdet", "dphix", "phi", "phif", "psi", "ndA", "dA", "src", "uD", "bnd")]


class ConvDiff(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("tau", ctypes.c_double), ("beta", ctypes.c_double * 3),
                ("gamma", ctypes.c_double * 3)]


class SysModel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tau", ctypes.c_double), ("lam", ctypes.c_double),
                ("mu", ctypes.c_double), ("Re", ctypes.c_double), ("Pr", ctypes.c_double),
                ("gamma", ctypes.c_double)]


MODEL_KIND = {"elasticity": 1, "navier_stokes": 2}


class TimeTerm(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("u_prev", ctypes.c_void_p), ("r_extra", ctypes.c_void_p)]


class ElemArrays(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt", "q")]


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("atol", ctypes.c_double), ("prec", ctypes.c_int32), ("poly_degree", ctypes.c_int32),
                ("poly_v0", ctypes.c_void_p), ("orth", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("resid_hist_h", ctypes.POINTER(ctypes.c_double)), ("resid_hist_len", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("time_phases", ctypes.c_int32), ("fold_prec", ctypes.c_int32),
                ("asm_inv64", ctypes.c_void_p), ("asm_inv32", ctypes.c_void_p), ("asm_f2e", ctypes.c_void_p),
                ("asm_e2f", ctypes.c_void_p), ("reuse_setup", ctypes.c_int32), ("ilu_asm", ctypes.c_void_p)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("cycles", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("npoly", ctypes.c_int32), ("rel_resid_true", ctypes.c_double), ("rel_resid_est", ctypes.c_double),
                ("t_setup", ctypes.c_double), ("t_total", ctypes.c_double),
                ("theta_re", ctypes.c_double * 64), ("theta_im", ctypes.c_double * 64),
                ("hist_len", ctypes.c_int32), ("n_timed", ctypes.c_int32), ("t_prec", ctypes.c_double),
                ("t_matvec", ctypes.c_double), ("t_orth", ctypes.c_double), ("cheb_alpha", ctypes.c_double),
                ("cheb_beta", ctypes.c_double), ("fallback_flags", ctypes.c_int32), ("fp64_cycles", ctypes.c_int32)]


_lib = None


def load():
    """Load libhdg.so (built in-tree by __graft_entry__.build / paper_2512_13619_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HdgError(-5, f"{LIB_PATH} is missing: build it first (python -m paper_2512_13619_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pd = ctypes.POINTER(Dims)
    lib.hdg_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
    lib.hdg_destroy.argtypes = [vp]
    lib.hdg_set_stream.argtypes = [vp, vp]
    lib.hdg_last_error.argtypes = [vp]
    lib.hdg_last_error.restype = ctypes.c_char_p
    lib.hdg_release_workspace.argtypes = [vp]
    lib.hdg_local_size.argtypes = [pd]
    lib.hdg_local_size.restype = ctypes.c_size_t
    lib.hdg_condense.argtypes = [vp, pd, i64, ctypes.POINTER(ElemBlocks), vp, vp, vp]
    lib.hdg_assemble_blocks.argtypes = [vp, pd, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hdg_condense_keep.argtypes = [vp, pd, i64, ctypes.POINTER(ElemBlocks), vp, vp, vp, vp, vp]
    lib.hdg_condense_rhs.argtypes = [vp, pd, i64, vp, vp, vp, vp, vp, vp]
    lib.hdg_assemble_rhs.argtypes = [vp, pd, vp, vp, vp, vp]
    lib.hdg_solve_opts_default.argtypes = [ctypes.POINTER(SolveOpts)]
    lib.hdg_solve_opts_default.restype = None
    lib.hdg_gmres_solve.argtypes = [vp, pd, vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                    ctypes.POINTER(SolveStats)]
    lib.hdg_recover_local.argtypes = [vp, pd, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hdg_newton_update.argtypes = [vp, i64, dbl, vp, vp]
    lib.hdg_element_blocks.argtypes = [vp, pd, ctypes.POINTER(ElemGeom), ctypes.POINTER(ConvDiff),
                                       ctypes.POINTER(TimeTerm), vp, vp, vp, i32, ctypes.POINTER(ElemArrays)]
    lib.hdg_residual_norm.argtypes = [vp, pd, vp, vp, vp, ctypes.POINTER(dbl)]
    lib.hdg_residual_norm_noalloc.argtypes = [vp, pd, vp, vp, vp, ctypes.POINTER(dbl)]
    lib.hdg_autotune.argtypes = [vp, pd, vp, vp, vp, vp, vp, i32, ctypes.POINTER(i32)]
    lib.hdg_tune_table.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    lib.hdg_tune_table.restype = ctypes.c_size_t
    lib.hdg_element_blocks_sys.argtypes = [vp, pd, ctypes.POINTER(ElemGeom), ctypes.POINTER(SysModel),
                                           ctypes.POINTER(TimeTerm), vp, vp, vp, i32, ctypes.POINTER(ElemArrays)]
    lib.hdg_matvec.argtypes = [vp, pd, vp, vp, vp, i32, vp, vp]
    lib.hdg_bj_setup.argtypes = [vp, pd, vp, vp, vp]
    lib.hdg_bj_apply.argtypes = [vp, pd, vp, vp, i32, vp, vp]
    lib.hdg_asm_setup.argtypes = [vp, pd, vp, vp, vp, vp, vp]
    lib.hdg_asm_apply.argtypes = [vp, pd, vp, vp, i32, vp, vp, vp, vp]
    lib.hdg_poly_apply.argtypes = [vp, pd, vp, vp, vp, vp, vp, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                   vp, vp]
    lib.hdg_cheb_apply.argtypes = [vp, pd, vp, vp, vp, vp, vp, i32, i32, dbl, dbl, vp, vp]
    pdbl = ctypes.POINTER(dbl)
    lib.hdg_hessenberg_eigvals.argtypes = [ctypes.c_int, pdbl, ctypes.c_int, pdbl, pdbl]
    lib.hdg_harmonic_ritz.argtypes = [ctypes.c_int, pdbl, dbl, pdbl, pdbl, ctypes.POINTER(ctypes.c_int)]
    lib.hdg_poly_roots.argtypes = [ctypes.c_int, pdbl, dbl, pdbl, pdbl, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int)]
    lib.hdg_batch_create.argtypes = [vp, i32, pd, ctypes.POINTER(vp)]
    lib.hdg_batch_destroy.argtypes = [vp]
    lib.hdg_batch_offsets.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64)]
    lib.hdg_batch_tuned_grid.argtypes = [vp]
    lib.hdg_condense_batch.argtypes = [vp, vp, ctypes.POINTER(ElemBlocks), vp, vp, vp]
    lib.hdg_assemble_batch.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hdg_gmres_solve_batch.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                          ctypes.POINTER(SolveStats)]
    lib.hdg_recover_batch.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hdg_element_blocks_batch.argtypes = [vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ElemGeom),
                                             ctypes.POINTER(ConvDiff), ctypes.POINTER(dbl), vp, vp, vp, vp, vp,
                                             i32, ctypes.POINTER(ElemArrays)]
    lib.hdg_residual_norm_batch.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(dbl)]
    lib.hdg_ilu_asm_create.argtypes = [vp, pd, vp, vp, vp, i32, ctypes.POINTER(vp)]
    lib.hdg_ilu_asm_destroy.argtypes = [vp]
    lib.hdg_ilu_asm_apply.argtypes = [vp, vp, vp, vp]
    lib.hdg_newton_update_batch.argtypes = [vp, vp, ctypes.POINTER(dbl), vp, vp, vp, vp]
    for name in SYMBOLS:
        if name not in ("hdg_last_error", "hdg_local_size", "hdg_solve_opts_default",
                        "hdg_hessenberg_eigvals", "hdg_harmonic_ritz", "hdg_poly_roots", "hdg_tune_table"):
            getattr(lib, name).restype = ctypes.c_int
    lib.hdg_hessenberg_eigvals.restype = ctypes.c_int
    lib.hdg_harmonic_ritz.restype = ctypes.c_int
    lib.hdg_poly_roots.restype = ctypes.c_int
    _lib = lib
    return lib


def make_dims(d):
    return Dims(*(int(d[k]) for k in ("ne", "nf", "ncomp", "dim", "npe", "npf", "nlfe")))


def _ptr(t, dtype, numel=None, name="array", allow_none=False):
    import torch
    if t is None:
        if allow_none:
            return None
        raise HdgError(-1, f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise HdgError(-1, f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise HdgError(-1, f"{name} must be on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise HdgError(-1, f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise HdgError(-1, f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise HdgError(-2, f"{name} has {t.numel()} entries, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


# ---- host-only helpers (no GPU needed) ----------------------------------------------------
def tune_table():
    """The measured launch-configuration table (hdg_tune_table) as a dict."""
    import json
    lib = load()
    n = lib.hdg_tune_table(None, 0)
    buf = ctypes.create_string_buffer(max(int(n), 1))
    lib.hdg_tune_table(buf, len(buf))
    return json.loads(buf.value.decode()) if buf.value else {}


def hessenberg_eigvals(H):
    lib = load()
    H = np.ascontiguousarray(H, dtype=np.float64)
    n = H.shape[0]
    wr = np.zeros(n)
    wi = np.zeros(n)
    pd = ctypes.POINTER(ctypes.c_double)
    rc = lib.hdg_hessenberg_eigvals(n, H.ctypes.data_as(pd), n, wr.ctypes.data_as(pd), wi.ctypes.data_as(pd))
    if rc != 0:
        raise HdgError(rc, "eigenvalue iteration failed")
    return wr + 1j * wi


def poly_roots(H, drop_rel=1e-12):
    """H: (P+1) x P Arnoldi Hessenberg. Returns (roots in Leja order, number of added copies):
    the roots the solver's polynomial preconditioner uses (hdg_poly_roots)."""
    lib = load()
    H = np.ascontiguousarray(H, dtype=np.float64)
    P = H.shape[1]
    tr = np.zeros(P + 4)
    ti = np.zeros(P + 4)
    n = ctypes.c_int(0)
    na = ctypes.c_int(0)
    pd = ctypes.POINTER(ctypes.c_double)
    rc = lib.hdg_poly_roots(P, H.ctypes.data_as(pd), drop_rel, tr.ctypes.data_as(pd), ti.ctypes.data_as(pd),
                            ctypes.byref(n), ctypes.byref(na))
    if rc != 0:
        raise HdgError(rc, "polynomial root computation failed")
    return tr[:n.value] + 1j * ti[:n.value], na.value


def harmonic_ritz(H, drop_rel=1e-12):
    """H: (P+1) x P Arnoldi Hessenberg. Returns Leja-ordered harmonic Ritz values."""
    lib = load()
    H = np.ascontiguousarray(H, dtype=np.float64)
    P = H.shape[1]
    tr = np.zeros(P + 1)
    ti = np.zeros(P + 1)
    n = ctypes.c_int(0)
    pd = ctypes.POINTER(ctypes.c_double)
    rc = lib.hdg_harmonic_ritz(P, H.ctypes.data_as(pd), drop_rel, tr.ctypes.data_as(pd), ti.ctypes.data_as(pd),
                               ctypes.byref(n))
    if rc != 0:
        raise HdgError(rc, "harmonic Ritz computation failed")
    return tr[:n.value] + 1j * ti[:n.value]


# ---- device context -----------------------------------------------------------------------
class Context:
    def __init__(self, device=0, stream=None):
        import torch
        self.lib = load()
        self.device = device
        self.h = ctypes.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self._stream = s
        st = self.lib.hdg_create(ctypes.byref(self.h), device, ctypes.c_void_p(s.cuda_stream))
        if st != HDG_OK:
            raise HdgError(st, "hdg_create failed (no GPU or bad device)")

    def close(self):
        if self.h:
            self.lib.hdg_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self):
        return self._stream

    def _check(self, st):
        if st < 0:
            raise HdgError(st, self.lib.hdg_last_error(self.h).decode())
        return st

    def release_workspace(self):
        self._check(self.lib.hdg_release_workspace(self.h))

    # (1)
    def condense(self, dims, blk, Kbar, rbar, local, ne_chunk=None):
        import torch
        d = make_dims(dims)
        ne = int(dims["ne"]) if ne_chunk is None else int(ne_chunk)
        M, D, P, PF, L = (int(dims[k]) for k in ("ncomp", "dim", "npe", "npf", "nlfe"))
        nu, nq, nt = M * P, M * D * P, L * M * PF
        f64 = torch.float64
        sizes = dict(Minv=P * P, Bd=D * P * P, Cd=D * P * L * PF, D=nu * nq, E=nu * nu, F=nu * nt, G=nt * nq,
                     H=nt * nu, J=nt * nt, ru=nu, rt=nt)
        names = [f[0] for f in ElemBlocks._fields_]
        eb = ElemBlocks(*[_ptr(blk[k], f64, ne * sizes[k], k) for k in names])
        return self._check(self.lib.hdg_condense(self.h, ctypes.byref(d), ne, ctypes.byref(eb),
                                                 _ptr(Kbar, f64, ne * nt * nt, "Kbar"), _ptr(rbar, f64, ne * nt, "rbar"),
                                                 _ptr(local, f64, ne * nu * (nu + nt + 1), "local")))

    def condense_keep(self, dims, blk, Kbar, rbar, local, Hbar, ipiv, ne_chunk=None):
        import torch
        d = make_dims(dims)
        ne = int(dims["ne"]) if ne_chunk is None else int(ne_chunk)
        M, D, P, PF, L = (int(dims[k]) for k in ("ncomp", "dim", "npe", "npf", "nlfe"))
        nu, nq, nt = M * P, M * D * P, L * M * PF
        f64 = torch.float64
        sizes = dict(Minv=P * P, Bd=D * P * P, Cd=D * P * L * PF, D=nu * nq, E=nu * nu, F=nu * nt, G=nt * nq,
                     H=nt * nu, J=nt * nt, ru=nu, rt=nt)
        names = [f[0] for f in ElemBlocks._fields_]
        eb = ElemBlocks(*[_ptr(blk[k], f64, ne * sizes[k], k) for k in names])
        return self._check(self.lib.hdg_condense_keep(
            self.h, ctypes.byref(d), ne, ctypes.byref(eb), _ptr(Kbar, f64, ne * nt * nt, "Kbar"),
            _ptr(rbar, f64, ne * nt, "rbar"), _ptr(local, f64, ne * nu * (nu + nt + 1), "local"),
            _ptr(Hbar, f64, ne * nt * nu, "Hbar"), _ptr(ipiv, torch.int32, ne * nu, "ipiv")))

    def condense_rhs(self, dims, local, Hbar, ipiv, ru, rt, rbar, ne_chunk=None):
        import torch
        d = make_dims(dims)
        ne = int(dims["ne"]) if ne_chunk is None else int(ne_chunk)
        M, P, PF, L = (int(dims[k]) for k in ("ncomp", "npe", "npf", "nlfe"))
        nu, nt = M * P, L * M * PF
        f64 = torch.float64
        return self._check(self.lib.hdg_condense_rhs(
            self.h, ctypes.byref(d), ne, _ptr(local, f64, ne * nu * (nu + nt + 1), "local"),
            _ptr(Hbar, f64, ne * nt * nu, "Hbar"), _ptr(ipiv, torch.int32, ne * nu, "ipiv"),
            _ptr(ru, f64, ne * nu, "ru"), _ptr(rt, f64, ne * nt, "rt"), _ptr(rbar, f64, ne * nt, "rbar")))

    def assemble_rhs(self, dims, f2e, perm, rbar, r):
        import torch
        d = make_dims(dims)
        ne, nf, M, PF, L = (int(dims[k]) for k in ("ne", "nf", "ncomp", "npf", "nlfe"))
        nb, nt = M * PF, L * M * PF
        return self._check(self.lib.hdg_assemble_rhs(
            self.h, ctypes.byref(d), _ptr(f2e, torch.int32, nf * 4, "f2e"),
            _ptr(perm, torch.int32, ne * L * PF, "perm", allow_none=True),
            _ptr(rbar, torch.float64, ne * nt, "rbar"), _ptr(r, torch.float64, nf * nb, "r")))

    # (2)
    def assemble(self, dims, f2e, e2f, perm, Kbar, rbar, K64, K32, nbr, r):
        import torch
        d = make_dims(dims)
        ne, nf, M, PF, L = (int(dims[k]) for k in ("ne", "nf", "ncomp", "npf", "nlfe"))
        nb, S, nt = M * PF, 2 * L - 1, L * M * PF
        return self._check(self.lib.hdg_assemble_blocks(
            self.h, ctypes.byref(d), _ptr(f2e, torch.int32, nf * 4, "f2e"), _ptr(e2f, torch.int32, ne * L, "e2f"),
            _ptr(perm, torch.int32, ne * L * PF, "perm", allow_none=True),
            _ptr(Kbar, torch.float64, ne * nt * nt, "Kbar"), _ptr(rbar, torch.float64, ne * nt, "rbar"),
            _ptr(K64, torch.float64, nf * S * nb * nb, "K64"),
            _ptr(K32, torch.float32, nf * S * nb * nb, "K32", allow_none=True),
            _ptr(nbr, torch.int32, nf * S, "nbr"), _ptr(r, torch.float64, nf * nb, "r")))

    # (3)
    def gmres_solve(self, dims, K64, K32, nbr, r, x, restart=50, max_iters=1000, rtol=1e-8, atol=0.0,
                    prec="bj", poly_degree=10, poly_v0=None, orth="cgs2", precision="fp64", hist_len=0,
                    use_graph=False, time_phases=False, fold_prec=False, asm=None, reuse_setup=False, ilu=None):
        import torch
        d = make_dims(dims)
        nf, M, PF, L = (int(dims[k]) for k in ("nf", "ncomp", "npf", "nlfe"))
        nb, S = M * PF, 2 * L - 1
        N = nf * nb
        o = SolveOpts()
        self.lib.hdg_solve_opts_default(ctypes.byref(o))
        o.restart, o.max_iters, o.rtol, o.atol = restart, max_iters, rtol, atol
        o.prec, o.poly_degree, o.orth, o.precision = PREC[prec], poly_degree, ORTH[orth], PRECISION[precision]
        o.poly_v0 = _ptr(poly_v0, torch.float64, N, "poly_v0", allow_none=True)
        o.use_graph = 1 if use_graph else 0
        o.time_phases = 1 if time_phases else 0
        o.fold_prec = 1 if fold_prec else 0
        o.reuse_setup = 1 if reuse_setup else 0
        if ilu is not None:      # IluAsm from ilu_asm_create
            o.ilu_asm = ilu.h
        if asm is not None:      # dict(inv64=..., inv32=..., f2e=..., e2f=...) from asm_setup
            nt2 = int(dims["ne"]) * (L * nb) ** 2
            o.asm_inv64 = _ptr(asm["inv64"], torch.float64, nt2, "asm_inv64")
            o.asm_inv32 = _ptr(asm.get("inv32"), torch.float32, nt2, "asm_inv32", allow_none=True)
            o.asm_f2e = _ptr(asm["f2e"], torch.int32, nf * 4, "asm_f2e")
            o.asm_e2f = _ptr(asm["e2f"], torch.int32, int(dims["ne"]) * L, "asm_e2f")
        hist = np.zeros(max(hist_len, 1))
        if hist_len > 0:
            o.resid_hist_h = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            o.resid_hist_len = hist_len
        stats = SolveStats()
        st = self._check(self.lib.hdg_gmres_solve(
            self.h, ctypes.byref(d), _ptr(K64, torch.float64, nf * S * nb * nb, "K64"),
            _ptr(K32, torch.float32, nf * S * nb * nb, "K32", allow_none=True), _ptr(nbr, torch.int32, nf * S, "nbr"),
            _ptr(r, torch.float64, N, "r"), _ptr(x, torch.float64, N, "x"), ctypes.byref(o), ctypes.byref(stats)))
        out = {f[0]: getattr(stats, f[0]) for f in SolveStats._fields_ if f[0] not in ("theta_re", "theta_im")}
        out["status"] = st
        out["theta"] = np.array([stats.theta_re[i] + 1j * stats.theta_im[i] for i in range(stats.npoly)])
        out["hist"] = hist[:stats.hist_len].copy() if hist_len > 0 else None
        return out

    # (4)
    def recover(self, dims, local, Minv, Bd, Cd, e2f, perm, xhat, du, dq):
        import torch
        d = make_dims(dims)
        ne, nf, M, D, P, PF, L = (int(dims[k]) for k in ("ne", "nf", "ncomp", "dim", "npe", "npf", "nlfe"))
        nu, nq, nt, nb = M * P, M * D * P, L * M * PF, M * PF
        f64 = torch.float64
        return self._check(self.lib.hdg_recover_local(
            self.h, ctypes.byref(d), _ptr(local, f64, ne * nu * (nu + nt + 1), "local"),
            _ptr(Minv, f64, ne * P * P, "Minv"), _ptr(Bd, f64, ne * D * P * P, "Bd"),
            _ptr(Cd, f64, ne * D * P * L * PF, "Cd"), _ptr(e2f, torch.int32, ne * L, "e2f"),
            _ptr(perm, torch.int32, ne * L * PF, "perm", allow_none=True), _ptr(xhat, f64, nf * nb, "xhat"),
            _ptr(du, f64, ne * nu, "du"), _ptr(dq, f64, ne * nq, "dq")))

    # (5)
    def newton_update(self, alpha, delta, state):
        import torch
        n = state.numel()
        return self._check(self.lib.hdg_newton_update(self.h, n, float(alpha), _ptr(delta, torch.float64, n, "delta"),
                                                      _ptr(state, torch.float64, n, "state")))

    def element_blocks(self, dims, geom, model, e2f, u, uhat, out, residual_only=False, time_term=None,
                       keep_mass=False):
        """Element residuals (and Jacobian blocks unless residual_only) at the state (u, uhat):
        geom holds the quadrature geometry (wdet, dphix, phi, phif, psi, ndA, dA, src, uD, bnd,
        nqv, nqf), model the coefficients (nu, tau, beta, gamma), out the device outputs;
        time_term = dict(c, u_prev, r_extra=None) for an implicit stage; keep_mass: out's Minv,
        Bd, Cd hold this mesh's from an earlier call (read, not recomputed or written)."""
        import torch
        d = make_dims(dims)
        ne, nf, M, D, P, PF, L = (int(dims[k]) for k in ("ne", "nf", "ncomp", "dim", "npe", "npf", "nlfe"))
        Qv, Qf = int(geom["nqv"]), int(geom["nqf"])
        f64 = torch.float64
        gsz = dict(wdet=ne * Qv, dphix=ne * Qv * P * D, phi=Qv * P, phif=ne * L * Qf * P, psi=Qf * PF,
                   ndA=ne * L * Qf * D, dA=ne * L * Qf, src=ne * Qv, uD=ne * L * Qf)
        g = ElemGeom(Qv, Qf, *[_ptr(geom[k], f64, gsz[k], k) for k in gsz],
                     _ptr(geom["bnd"], torch.int32, ne * L, "bnd"))
        beta = list(model["beta"]) + [0.0] * (3 - len(model["beta"]))
        gamma = list(model["gamma"]) + [0.0] * (3 - len(model["gamma"]))
        m = ConvDiff(float(model["nu"]), float(model["tau"]), (ctypes.c_double * 3)(*beta),
                     (ctypes.c_double * 3)(*gamma))
        nu, nq, nt = M * P, M * D * P, L * M * PF
        osz = dict(Minv=P * P, Bd=D * P * P, Cd=D * P * nt, D=nu * nq, E=nu * nu, F=nu * nt, G=nt * nq,
                   H=nt * nu, J=nt * nt, ru=nu, rt=nt, q=nq)
        o = ElemArrays(*[_ptr(out.get(k), f64, ne * osz[k], k, allow_none=True) for k in osz])
        tt = None
        if time_term is not None:
            tt = ctypes.byref(TimeTerm(float(time_term["c"]), _ptr(time_term.get("u_prev"), f64, ne * P, "u_prev",
                                                                     allow_none=True),
                                       _ptr(time_term.get("r_extra"), f64, ne * P, "r_extra", allow_none=True)))
        return self._check(self.lib.hdg_element_blocks(
            self.h, ctypes.byref(d), ctypes.byref(g), ctypes.byref(m), tt, _ptr(e2f, torch.int32, ne * L, "e2f"),
            _ptr(u, f64, ne * P, "u"), _ptr(uhat, f64, nf * PF * M, "uhat"),
            (1 if residual_only else 0) | (2 if keep_mass else 0), ctypes.byref(o)))

    def element_blocks_sys(self, dims, geom, model, e2f, u, uhat, out, residual_only=False, time_term=None,
                           keep_mass=False):
        """hdg_element_blocks_sys for the M-component models: geom as for element_blocks with
        src (ne, nqv, M) and uD (ne, nlfe, nqf, M); model = dict(kind="elasticity", tau, lam, mu)
        or dict(kind="navier_stokes", tau, Re, Pr, gamma); u (ne, M, npe) and uhat (nf, M, npf)
        flattened; time_term = dict(c, u_prev, r_extra=None)."""
        import torch
        d = make_dims(dims)
        ne, nf, M, D, P, PF, L = (int(dims[k]) for k in ("ne", "nf", "ncomp", "dim", "npe", "npf", "nlfe"))
        Qv, Qf = int(geom["nqv"]), int(geom["nqf"])
        f64 = torch.float64
        gsz = dict(wdet=ne * Qv, dphix=ne * Qv * P * D, phi=Qv * P, phif=ne * L * Qf * P, psi=Qf * PF,
                   ndA=ne * L * Qf * D, dA=ne * L * Qf, src=ne * Qv * M, uD=ne * L * Qf * M)
        g = ElemGeom(Qv, Qf, *[_ptr(geom[k], f64, gsz[k], k) for k in gsz],
                     _ptr(geom["bnd"], torch.int32, ne * L, "bnd"))
        if model["kind"] not in MODEL_KIND:
            raise HdgError(-1, f"unknown model kind {model['kind']!r}")
        m = SysModel(MODEL_KIND[model["kind"]], float(model["tau"]), float(model.get("lam", 0.0)),
                     float(model.get("mu", 0.0)), float(model.get("Re", 0.0)), float(model.get("Pr", 0.0)),
                     float(model.get("gamma", 0.0)))
        nu, nq, nt = M * P, M * D * P, L * M * PF
        osz = dict(Minv=P * P, Bd=D * P * P, Cd=D * P * L * PF, D=nu * nq, E=nu * nu, F=nu * nt, G=nt * nq,
                   H=nt * nu, J=nt * nt, ru=nu, rt=nt, q=nq)
        o = ElemArrays(*[_ptr(out.get(k), f64, ne * osz[k], k, allow_none=True) for k in osz])
        tt = None
        if time_term is not None:
            tt = ctypes.byref(TimeTerm(float(time_term["c"]), _ptr(time_term.get("u_prev"), f64, ne * nu, "u_prev",
                                                                     allow_none=True),
                                       _ptr(time_term.get("r_extra"), f64, ne * nu, "r_extra", allow_none=True)))
        return self._check(self.lib.hdg_element_blocks_sys(
            self.h, ctypes.byref(d), ctypes.byref(g), ctypes.byref(m), tt, _ptr(e2f, torch.int32, ne * L, "e2f"),
            _ptr(u, f64, ne * nu, "u"), _ptr(uhat, f64, nf * PF * M, "uhat"),
            (1 if residual_only else 0) | (2 if keep_mass else 0), ctypes.byref(o)))

    def autotune(self, dims, K64, K32, nbr, Binv64=None, Binv32=None, reps=10):
        """hdg_autotune: measure the face operator's launch configurations on this matrix (and
        its block-Jacobi inverses when given); returns the number of variants timed."""
        import torch
        d = make_dims(dims)
        nf, M, PF, L = (int(dims[k]) for k in ("nf", "ncomp", "npf", "nlfe"))
        nb, S = M * PF, 2 * L - 1
        n = ctypes.c_int32(0)
        self._check(self.lib.hdg_autotune(
            self.h, ctypes.byref(d), _ptr(K64, torch.float64, nf * S * nb * nb, "K64"),
            _ptr(K32, torch.float32, nf * S * nb * nb, "K32", allow_none=True), _ptr(nbr, torch.int32, nf * S, "nbr"),
            _ptr(Binv64, torch.float64, nf * nb * nb, "Binv64", allow_none=True),
            _ptr(Binv32, torch.float32, nf * nb * nb, "Binv32", allow_none=True), int(reps), ctypes.byref(n)))
        return n.value

    def residual_norm(self, dims, f2e, ru, rt, noalloc=False):
        """hdg_residual_norm, or with noalloc=True hdg_residual_norm_noalloc (fixed device scratch)."""
        import torch
        d = make_dims(dims)
        ne, nf, M, P, PF, L = (int(dims[k]) for k in ("ne", "nf", "ncomp", "npe", "npf", "nlfe"))
        out = ctypes.c_double(0.0)
        fn = self.lib.hdg_residual_norm_noalloc if noalloc else self.lib.hdg_residual_norm
        self._check(fn(
            self.h, ctypes.byref(d), _ptr(f2e, torch.int32, nf * 4, "f2e"), _ptr(ru, torch.float64, ne * M * P, "ru"),
            _ptr(rt, torch.float64, ne * L * M * PF, "rt"), ctypes.byref(out)))
        return out.value

    def ilu_asm_create(self, dims, K64, nbr, e2f, G):
        """Block ILU(0) factors of the patches of G consecutive elements (hdg_ilu_asm_create)."""
        import torch
        d = make_dims(dims)
        nf, M, PF, L, ne = (int(dims[k]) for k in ("nf", "ncomp", "npf", "nlfe", "ne"))
        nb, S = M * PF, 2 * L - 1
        h = ctypes.c_void_p()
        self._check(self.lib.hdg_ilu_asm_create(self.h, ctypes.byref(d), _ptr(K64, torch.float64, nf * S * nb * nb, "K64"),
                                                _ptr(nbr, torch.int32, nf * S, "nbr"),
                                                _ptr(e2f, torch.int32, ne * L, "e2f"), int(G), ctypes.byref(h)))
        return IluAsm(self, h, nf * nb)

    def ilu_asm_apply(self, ilu, y, z):
        import torch
        return self._check(self.lib.hdg_ilu_asm_apply(self.h, ilu.h, _ptr(y, torch.float64, ilu.n, "y"),
                                                      _ptr(z, torch.float64, ilu.n, "z")))

    # building blocks
    def matvec(self, dims, K64, K32, nbr, x, y, precision="fp64"):
        import torch
        d = make_dims(dims)
        nf, M, PF, L = (int(dims[k]) for k in ("nf", "ncomp", "npf", "nlfe"))
        nb, S = M * PF, 2 * L - 1
        return self._check(self.lib.hdg_matvec(
            self.h, ctypes.byref(d), _ptr(K64, torch.float64, nf * S * nb * nb, "K64", allow_none=True),
            _ptr(K32, torch.float32, nf * S * nb * nb, "K32", allow_none=True), _ptr(nbr, torch.int32, nf * S, "nbr"),
            PRECISION[precision], _ptr(x, torch.float64, nf * nb, "x"), _ptr(y, torch.float64, nf * nb, "y")))

    def bj_setup(self, dims, K64, Binv64, Binv32=None):
        import torch
        d = make_dims(dims)
        nf, M, PF, L = (int(dims[k]) for k in ("nf", "ncomp", "npf", "nlfe"))
        nb, S = M * PF, 2 * L - 1
        return self._check(self.lib.hdg_bj_setup(
            self.h, ctypes.byref(d), _ptr(K64, torch.float64, nf * S * nb * nb, "K64"),
            _ptr(Binv64, torch.float64, nf * nb * nb, "Binv64"),
            _ptr(Binv32, torch.float32, nf * nb * nb, "Binv32", allow_none=True)))

    def bj_apply(self, dims, Binv64, Binv32, y, z, precision="fp64"):
        import torch
        d = make_dims(dims)
        nf, nb = int(dims["nf"]), int(dims["ncomp"]) * int(dims["npf"])
        return self._check(self.lib.hdg_bj_apply(
            self.h, ctypes.byref(d), _ptr(Binv64, torch.float64, nf * nb * nb, "Binv64", allow_none=True),
            _ptr(Binv32, torch.float32, nf * nb * nb, "Binv32", allow_none=True), PRECISION[precision],
            _ptr(y, torch.float64, nf * nb, "y"), _ptr(z, torch.float64, nf * nb, "z")))

    def asm_setup(self, dims, Kbar, K64, e2f, inv64, inv32=None):
        import torch
        d = make_dims(dims)
        ne, nf, M, PF, L = (int(dims[k]) for k in ("ne", "nf", "ncomp", "npf", "nlfe"))
        nb, S = M * PF, 2 * L - 1
        nt = L * nb
        return self._check(self.lib.hdg_asm_setup(
            self.h, ctypes.byref(d), _ptr(Kbar, torch.float64, ne * nt * nt, "Kbar"),
            _ptr(K64, torch.float64, nf * S * nb * nb, "K64"), _ptr(e2f, torch.int32, ne * L, "e2f"),
            _ptr(inv64, torch.float64, ne * nt * nt, "inv64", allow_none=True),
            _ptr(inv32, torch.float32, ne * nt * nt, "inv32", allow_none=True)))

    def asm_apply(self, dims, inv64, inv32, f2e, e2f, y, z, precision="fp64"):
        import torch
        d = make_dims(dims)
        ne, nf, M, PF, L = (int(dims[k]) for k in ("ne", "nf", "ncomp", "npf", "nlfe"))
        nb = M * PF
        nt = L * nb
        return self._check(self.lib.hdg_asm_apply(
            self.h, ctypes.byref(d), _ptr(inv64, torch.float64, ne * nt * nt, "inv64", allow_none=True),
            _ptr(inv32, torch.float32, ne * nt * nt, "inv32", allow_none=True), PRECISION[precision],
            _ptr(f2e, torch.int32, nf * 4, "f2e"), _ptr(e2f, torch.int32, ne * L, "e2f"),
            _ptr(y, torch.float64, nf * nb, "y"), _ptr(z, torch.float64, nf * nb, "z")))

    def poly_apply(self, dims, K64, K32, nbr, Binv64, Binv32, theta, y, z, precision="fp64"):
        import torch
        d = make_dims(dims)
        nf, M, PF, L = (int(dims[k]) for k in ("nf", "ncomp", "npf", "nlfe"))
        nb, S = M * PF, 2 * L - 1
        th = np.asarray(theta, complex)
        tr = np.ascontiguousarray(th.real, dtype=np.float64)
        ti = np.ascontiguousarray(th.imag, dtype=np.float64)
        pd = ctypes.POINTER(ctypes.c_double)
        return self._check(self.lib.hdg_poly_apply(
            self.h, ctypes.byref(d), _ptr(K64, torch.float64, nf * S * nb * nb, "K64", allow_none=True),
            _ptr(K32, torch.float32, nf * S * nb * nb, "K32", allow_none=True), _ptr(nbr, torch.int32, nf * S, "nbr"),
            _ptr(Binv64, torch.float64, nf * nb * nb, "Binv64", allow_none=True),
            _ptr(Binv32, torch.float32, nf * nb * nb, "Binv32", allow_none=True), PRECISION[precision], len(th),
            tr.ctypes.data_as(pd), ti.ctypes.data_as(pd), _ptr(y, torch.float64, nf * nb, "y"),
            _ptr(z, torch.float64, nf * nb, "z")))

    def cheb_apply(self, dims, K64, K32, nbr, Binv64, Binv32, degree, alpha, beta, y, z, precision="fp64"):
        import torch
        d = make_dims(dims)
        nf, M, PF, L = (int(dims[k]) for k in ("nf", "ncomp", "npf", "nlfe"))
        nb, S = M * PF, 2 * L - 1
        return self._check(self.lib.hdg_cheb_apply(
            self.h, ctypes.byref(d), _ptr(K64, torch.float64, nf * S * nb * nb, "K64", allow_none=True),
            _ptr(K32, torch.float32, nf * S * nb * nb, "K32", allow_none=True), _ptr(nbr, torch.int32, nf * S, "nbr"),
            _ptr(Binv64, torch.float64, nf * nb * nb, "Binv64", allow_none=True),
            _ptr(Binv32, torch.float32, nf * nb * nb, "Binv32", allow_none=True), PRECISION[precision],
            int(degree), float(alpha), float(beta), _ptr(y, torch.float64, nf * nb, "y"),
            _ptr(z, torch.float64, nf * nb, "z")))


class IluAsm:
    """Handle of ILU-ASM factors (device memory owned by the library until close)."""

    def __init__(self, ctx, h, n):
        self.ctx, self.lib, self.h, self.n = ctx, ctx.lib, h, n

    def close(self):
        if self.h:
            self.lib.hdg_ilu_asm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Device descriptor tables for many independent instances (hdg_batch_* entry points).

    Arrays are the concatenation of the instances' arrays; `offsets(name)` gives each
    instance's start (prefix sums of the per-instance sizes) in entries of that array."""

    def __init__(self, ctx, dims_list):
        self.ctx = ctx
        self.lib = ctx.lib
        self.n = len(dims_list)
        self.dims_list = [dict(d) for d in dims_list]
        arr = (Dims * self.n)(*[make_dims(d) for d in dims_list])
        self.h = ctypes.c_void_p()
        ctx._check(self.lib.hdg_batch_create(ctx.h, self.n, arr, ctypes.byref(self.h)))
        self._off = {}
        for k, name in enumerate(BATCH_ARRAYS):
            o = np.zeros(self.n + 1, dtype=np.int64)
            self.lib.hdg_batch_offsets(self.h, k, o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
            self._off[name] = o

    def offsets(self, name):
        return self._off[name]

    def total(self, name):
        return int(self._off[name][-1])

    def tuned_grid(self):
        return int(self.lib.hdg_batch_tuned_grid(self.h))

    def close(self):
        if self.h:
            self.lib.hdg_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def condense(self, blk, Kbar, rbar, local):
        import torch
        f64 = torch.float64
        names = [f[0] for f in ElemBlocks._fields_]
        eb = ElemBlocks(*[_ptr(blk[k], f64, self.total(k), k) for k in names])
        return self.ctx._check(self.lib.hdg_condense_batch(
            self.ctx.h, self.h, ctypes.byref(eb), _ptr(Kbar, f64, self.total("Kbar"), "Kbar"),
            _ptr(rbar, f64, self.total("rbar"), "rbar"), _ptr(local, f64, self.total("local"), "local")))

    def element_blocks(self, nqv, nqf, geom, models, e2f, u, uhat, out, residual_only=False, c=None, u_prev=None,
                       keep_mass=False, r_extra=None):
        """Batched hdg_element_blocks: nqv, nqf and models (dicts nu, tau, beta, gamma) per
        instance; geom's arrays concatenated in instance order; the rest are batch arrays;
        c (per instance) with u_prev: a time term per instance."""
        import torch
        f64 = torch.float64
        n = self.n
        gsz = dict(wdet=0, dphix=0, phi=0, phif=0, psi=0, ndA=0, dA=0, src=0, uD=0, bnd=0)
        for d, qv, qf in zip(self.dims_list, nqv, nqf):
            ne, P, PF, L, D = (int(d[k]) for k in ("ne", "npe", "npf", "nlfe", "dim"))
            gsz["wdet"] += ne * qv; gsz["dphix"] += ne * qv * P * D; gsz["phi"] += qv * P
            gsz["phif"] += ne * L * qf * P; gsz["psi"] += qf * PF; gsz["ndA"] += ne * L * qf * D
            gsz["dA"] += ne * L * qf; gsz["src"] += ne * qv; gsz["uD"] += ne * L * qf; gsz["bnd"] += ne * L
        g = ElemGeom(0, 0, *[_ptr(geom[k], f64, gsz[k], k) for k in list(gsz)[:-1]],
                     _ptr(geom["bnd"], torch.int32, gsz["bnd"], "bnd"))
        ms = (ConvDiff * n)()
        for i, m in enumerate(models):
            beta = list(m["beta"]) + [0.0] * (3 - len(m["beta"]))
            gamma = list(m["gamma"]) + [0.0] * (3 - len(m["gamma"]))
            ms[i] = ConvDiff(float(m["nu"]), float(m["tau"]), (ctypes.c_double * 3)(*beta),
                             (ctypes.c_double * 3)(*gamma))
        qv_a = (ctypes.c_int32 * n)(*[int(v) for v in nqv])
        qf_a = (ctypes.c_int32 * n)(*[int(v) for v in nqf])
        names = ["Minv", "Bd", "Cd", "D", "E", "F", "G", "H", "J", "ru", "rt"]
        ptrs = [_ptr(out.get(k), f64, self.total(k), k, allow_none=True) for k in names]
        ptrs.append(_ptr(out.get("q"), f64, self.total("dq"), "q", allow_none=True))
        o = ElemArrays(*ptrs)
        c_a = None
        if c is not None:
            c_np = np.ascontiguousarray(c, dtype=np.float64)
            assert c_np.shape == (n,)
            c_a = c_np.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return self.ctx._check(self.lib.hdg_element_blocks_batch(
            self.ctx.h, self.h, qv_a, qf_a, ctypes.byref(g), ms, c_a,
            _ptr(u_prev, f64, self.total("du"), "u_prev", allow_none=True),
            _ptr(r_extra, f64, self.total("du"), "r_extra", allow_none=True),
            _ptr(e2f, torch.int32, self.total("e2f"), "e2f"),
            _ptr(u, f64, self.total("du"), "u"), _ptr(uhat, f64, self.total("vec"), "uhat"),
            (1 if residual_only else 0) | (2 if keep_mass else 0), ctypes.byref(o)))

    def residual_norms(self, f2e, ru, rt):
        import torch
        out = np.zeros(self.n)
        self.ctx._check(self.lib.hdg_residual_norm_batch(
            self.ctx.h, self.h, _ptr(f2e, torch.int32, self.total("f2e"), "f2e"),
            _ptr(ru, torch.float64, self.total("ru"), "ru"), _ptr(rt, torch.float64, self.total("rt"), "rt"),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def newton_update(self, alpha, du, u, x, uhat):
        import torch
        al = np.ascontiguousarray(alpha, dtype=np.float64)
        assert al.shape == (self.n,)
        return self.ctx._check(self.lib.hdg_newton_update_batch(
            self.ctx.h, self.h, al.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            _ptr(du, torch.float64, self.total("du"), "du"), _ptr(u, torch.float64, self.total("du"), "u"),
            _ptr(x, torch.float64, self.total("vec"), "x"), _ptr(uhat, torch.float64, self.total("vec"), "uhat")))

    def assemble(self, f2e, e2f, Kbar, rbar, K64, K32, nbr, r):
        import torch
        return self.ctx._check(self.lib.hdg_assemble_batch(
            self.ctx.h, self.h, _ptr(f2e, torch.int32, self.total("f2e"), "f2e"),
            _ptr(e2f, torch.int32, self.total("e2f"), "e2f"), _ptr(Kbar, torch.float64, self.total("Kbar"), "Kbar"),
            _ptr(rbar, torch.float64, self.total("rbar"), "rbar"), _ptr(K64, torch.float64, self.total("K"), "K64"),
            _ptr(K32, torch.float32, self.total("K"), "K32", allow_none=True),
            _ptr(nbr, torch.int32, self.total("nbr"), "nbr"), _ptr(r, torch.float64, self.total("vec"), "r")))

    def gmres_solve(self, K64, K32, nbr, r, x, restart=50, max_iters=1000, rtol=1e-8, atol=0.0, prec="bj",
                    orth="cgs2", precision="fp64", use_graph=False):
        import torch
        o = SolveOpts()
        self.lib.hdg_solve_opts_default(ctypes.byref(o))
        o.restart, o.max_iters, o.rtol, o.atol = restart, max_iters, rtol, atol
        o.prec, o.orth, o.precision = PREC[prec], ORTH[orth], PRECISION[precision]
        o.use_graph = 1 if use_graph else 0
        stats = (SolveStats * self.n)()
        st = self.ctx._check(self.lib.hdg_gmres_solve_batch(
            self.ctx.h, self.h, _ptr(K64, torch.float64, self.total("K"), "K64"),
            _ptr(K32, torch.float32, self.total("K"), "K32", allow_none=True),
            _ptr(nbr, torch.int32, self.total("nbr"), "nbr"), _ptr(r, torch.float64, self.total("vec"), "r"),
            _ptr(x, torch.float64, self.total("vec"), "x"), ctypes.byref(o), stats))
        out = [{k[0]: getattr(s_, k[0]) for k in SolveStats._fields_ if k[0] not in ("theta_re", "theta_im")}
               for s_ in stats]
        return st, out

    def recover(self, local, Minv, Bd, Cd, e2f, xhat, du, dq):
        import torch
        f64 = torch.float64
        return self.ctx._check(self.lib.hdg_recover_batch(
            self.ctx.h, self.h, _ptr(local, f64, self.total("local"), "local"),
            _ptr(Minv, f64, self.total("Minv"), "Minv"), _ptr(Bd, f64, self.total("Bd"), "Bd"),
            _ptr(Cd, f64, self.total("Cd"), "Cd"), _ptr(e2f, torch.int32, self.total("e2f"), "e2f"),
            _ptr(xhat, f64, self.total("vec"), "xhat"), _ptr(du, f64, self.total("du"), "du"),
            _ptr(dq, f64, self.total("dq"), "dq")))
