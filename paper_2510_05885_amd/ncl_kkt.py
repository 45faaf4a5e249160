"""Python binding of libncl_kkt.so (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels; torch is used
for device memory (tensors passed by data pointer) and streams.  The binding
fails loudly when the compiled library is missing — there is no fallback.

    kkt = KKT.analyze(n, m, W_colptr, W_rowidx, J_rowptr, J_colidx, form="condensed")
    kkt.factor(W_val, Sigma, J_val, rho)          # device float64 tensors
    X, info = kkt.solve(B)                        # B: (order, nrhs) device float64
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libncl_kkt.so")

NCL_CONDENSED, NCL_STABILIZED = 0, 1
NCL_FP64, NCL_FP32_IR = 0, 1
NCL_ORDER_ND, NCL_ORDER_NATURAL, NCL_ORDER_USER = 0, 1, 2
NCL_PIVOT_GLOBAL, NCL_PIVOT_BLOCK, NCL_PIVOT_ABSOLUTE = 0, 1, 2
NCL_OK = 0
NCL_ERR_ARG, NCL_ERR_PATTERN, NCL_ERR_ALLOC, NCL_ERR_HIP, NCL_ERR_STATE, NCL_ERR_NONFINITE = -1, -2, -3, -4, -5, -6
NCL_ERR_SCRATCH = -7
NCL_WARN_INERTIA, NCL_WARN_IR_NOT_CONVERGED, NCL_WARN_FELL_BACK_FP64 = 1, 2, 3

EXPORTED = [
    "ncl_kkt_default_options", "ncl_kkt_analyze", "ncl_kkt_analyze_host", "ncl_kkt_analyze_batched",
    "ncl_kkt_factor", "ncl_kkt_factor_batched", "ncl_kkt_solve", "ncl_kkt_inertia",
    "ncl_kkt_inertia_batched", "ncl_kkt_backward", "ncl_kkt_backward_noalloc", "ncl_kkt_get_stats", "ncl_kkt_get_perm",
    "ncl_kkt_get_supernodes", "ncl_kkt_get_system_times", "ncl_kkt_set_timing", "ncl_kkt_get_timing",
    "ncl_kkt_destroy", "ncl_kkt_strerror", "ncl_kkt_factor_k1s", "ncl_kkt_k1s_rhs", "ncl_kkt_k1s_recover",
    "ncl_kkt_recover_dy", "ncl_kkt_recover_dr", "ncl_kkt_recover_dz", "ncl_kkt_barrier_sigma",
    "ncl_kkt_factor_regularized", "ncl_qp_default_options", "ncl_qp_solve",
]


class Options(C.Structure):
    _fields_ = [("form", C.c_int32), ("precision", C.c_int32), ("pivot_eps", C.c_double),
                ("ir_max_steps", C.c_int32), ("ir_tol", C.c_double), ("ir_stall", C.c_double),
                ("ordering", C.c_int32), ("user_perm", C.POINTER(C.c_int32)), ("use_graphs", C.c_int32),
                ("small_front_max", C.c_int32), ("relax_big_zeros", C.c_double), ("fp32_sticky", C.c_int32),
                ("pivot_scale", C.c_int32), ("ir_cw_tol", C.c_double), ("persistent", C.c_int32),
                ("persistent_grid", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("ir_steps", C.c_int32), ("fell_back_fp64", C.c_int32),
                ("backward_error", C.c_double), ("backward_error0", C.c_double),
                ("backward_error_cw", C.c_double), ("resid_rel2", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("order", C.c_int64), ("nnz_K_lower", C.c_int64), ("nnz_L", C.c_int64),
                ("flops_factor", C.c_double), ("n_supernodes", C.c_int64), ("n_levels", C.c_int64),
                ("max_front", C.c_int64), ("n_large_fronts", C.c_int64), ("device_bytes", C.c_int64),
                ("analyze_seconds", C.c_double), ("nnz_L_exact", C.c_int64), ("flops_exact", C.c_double)]


class Timing(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int64 * 8), ("update_flops", C.c_double),
                ("small_flops", C.c_double), ("assemble_bytes", C.c_double), ("solve_bytes", C.c_double),
                ("panel_flops", C.c_double), ("diag_flops", C.c_double)]

    CLASSES = ("assemble", "small_fronts", "large_assembly", "large_panel", "large_update_mfma",
               "solve_sweeps", "residual", "large_diag")

    def as_dict(self):
        return {"ms": {k: self.ms[i] for i, k in enumerate(self.CLASSES)},
                "launches": {k: int(self.launches[i]) for i, k in enumerate(self.CLASSES)},
                "update_flops": self.update_flops, "small_flops": self.small_flops,
                "assemble_bytes": self.assemble_bytes, "solve_bytes": self.solve_bytes,
                "panel_flops": self.panel_flops, "diag_flops": self.diag_flops}


class QpOptions(C.Structure):
    _fields_ = [("eta_star", C.c_double), ("omega_star", C.c_double), ("max_outer", C.c_int32),
                ("max_inner", C.c_int32), ("precision", C.c_int32), ("print_level", C.c_int32)]


class QpResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer", C.c_int32), ("inner", C.c_int32),
                ("extrapolated", C.c_int32), ("primal_inf", C.c_double), ("dual_inf", C.c_double)]


_lib = None


def lib():
    """Load the compiled library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2510_05885_amd/build.py "
                           "(__graft_entry__.build()); there is no fallback path")
    # torch ships its own HIP runtime with the same soname; load it first so the
    # library binds to that one copy instead of a second runtime from /opt/rocm.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    pi32 = C.POINTER(C.c_int32)
    ph = C.POINTER(C.c_void_p)
    L.ncl_kkt_default_options.argtypes = [C.POINTER(Options)]
    L.ncl_kkt_default_options.restype = None
    for nm in ("ncl_kkt_analyze", "ncl_kkt_analyze_host"):
        f = getattr(L, nm)
        f.argtypes = [ph, C.POINTER(Options), i32, i32, pi32, pi32, pi32, pi32]
        f.restype = C.c_int
    L.ncl_kkt_analyze_batched.argtypes = [ph, C.POINTER(Options), i32, pi32, pi32, C.POINTER(pi32),
                                          C.POINTER(pi32), C.POINTER(pi32), C.POINTER(pi32)]
    L.ncl_kkt_analyze_batched.restype = C.c_int
    L.ncl_kkt_factor.argtypes = [vp, vp, vp, vp, dbl, vp]
    L.ncl_kkt_factor.restype = C.c_int
    L.ncl_kkt_factor_batched.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double), vp]
    L.ncl_kkt_factor_batched.restype = C.c_int
    L.ncl_kkt_factor_k1s.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_double), vp]
    L.ncl_kkt_factor_k1s.restype = C.c_int
    L.ncl_kkt_factor_regularized.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_double, C.c_double, C.c_double,
                                             C.POINTER(C.c_double), C.POINTER(C.c_int32), vp]
    L.ncl_kkt_factor_regularized.restype = C.c_int
    L.ncl_kkt_k1s_rhs.argtypes = [vp] * 7
    L.ncl_kkt_k1s_rhs.restype = C.c_int
    L.ncl_kkt_k1s_recover.argtypes = [vp] * 7
    L.ncl_kkt_k1s_recover.restype = C.c_int
    L.ncl_kkt_recover_dy.argtypes = [vp] * 8
    L.ncl_kkt_recover_dy.restype = C.c_int
    L.ncl_kkt_recover_dr.argtypes = [vp] * 7
    L.ncl_kkt_recover_dr.restype = C.c_int
    L.ncl_kkt_recover_dz.argtypes = [vp] * 7 + [C.c_double, vp, vp, vp]
    L.ncl_kkt_recover_dz.restype = C.c_int
    L.ncl_kkt_barrier_sigma.argtypes = [vp] * 8
    L.ncl_kkt_barrier_sigma.restype = C.c_int
    L.ncl_kkt_solve.argtypes = [vp, vp, i64, vp, i64, i32, vp, C.POINTER(SolveInfo)]
    L.ncl_kkt_solve.restype = C.c_int
    L.ncl_kkt_inertia.argtypes = [vp] + [C.POINTER(C.c_int64)] * 4
    L.ncl_kkt_inertia.restype = C.c_int
    L.ncl_kkt_inertia_batched.argtypes = [vp, C.POINTER(C.c_int64)]
    L.ncl_kkt_inertia_batched.restype = C.c_int
    for nm in ("ncl_kkt_backward", "ncl_kkt_backward_noalloc"):
        f = getattr(L, nm)
        f.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp, vp, vp, vp]
        f.restype = C.c_int
    L.ncl_kkt_get_stats.argtypes = [vp, C.POINTER(Stats)]
    L.ncl_kkt_get_stats.restype = C.c_int
    L.ncl_kkt_get_perm.argtypes = [vp, pi32]
    L.ncl_kkt_get_perm.restype = C.c_int
    L.ncl_kkt_get_supernodes.argtypes = [vp, pi32, pi32, C.POINTER(C.c_int64), pi32]
    L.ncl_kkt_get_supernodes.restype = C.c_int
    L.ncl_kkt_get_system_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.ncl_kkt_get_system_times.restype = C.c_int
    L.ncl_kkt_set_timing.argtypes = [vp, i32]
    L.ncl_kkt_set_timing.restype = C.c_int
    L.ncl_kkt_get_timing.argtypes = [vp, C.POINTER(Timing)]
    L.ncl_kkt_get_timing.restype = C.c_int
    L.ncl_kkt_destroy.argtypes = [vp]
    L.ncl_kkt_destroy.restype = None
    L.ncl_qp_default_options.argtypes = [C.POINTER(QpOptions)]
    L.ncl_qp_default_options.restype = None
    L.ncl_qp_solve.argtypes = [C.POINTER(QpOptions), i32, i32, pi32, pi32, vp, vp, pi32, pi32, vp, vp, vp, vp,
                               vp, vp, vp, vp, C.POINTER(QpResult), vp]
    L.ncl_qp_solve.restype = C.c_int
    L.ncl_kkt_strerror.argtypes = [C.c_int]
    L.ncl_kkt_strerror.restype = C.c_char_p
    _lib = L
    return L


class NCLError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lib().ncl_kkt_strerror(code).decode()} (status {code})")


def _check(code, where):
    if code < 0:
        raise NCLError(code, where)
    return code


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _ptr(t):
    """Device pointer of a torch tensor (checked by _dev first)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _dev(t, numel, name, allow_none=False):
    """Checks that t is a contiguous float64 tensor on a GPU with `numel`
    elements (the library reads and writes exactly that many)."""
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return _ptr(t)


def _dev_cols(t, rows, name):
    """Checks a (rows, nrhs) column-major (or (rows,)) float64 CUDA tensor;
    returns (pointer, leading dimension, nrhs)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() == 1 or (t.dim() == 2 and t.shape[1] == 1):
        if t.shape[0] != rows or t.stride(0) != 1:
            raise ValueError(f"{name} must be a contiguous vector of length {rows}")
        return _ptr(t), rows, 1
    if t.dim() != 2 or t.shape[0] != rows or t.stride(0) != 1 or t.stride(1) < rows:
        raise ValueError(f"{name} must be ({rows}, nrhs) column-major with leading dimension >= {rows}")
    return _ptr(t), t.stride(1), t.shape[1]


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


_FORMS = {"condensed": NCL_CONDENSED, "stabilized": NCL_STABILIZED}
_PRECS = {"fp64": NCL_FP64, "fp32_ir": NCL_FP32_IR}
_ORDS = {"nd": NCL_ORDER_ND, "natural": NCL_ORDER_NATURAL, "user": NCL_ORDER_USER}
_PIVS = {"global": NCL_PIVOT_GLOBAL, "block": NCL_PIVOT_BLOCK, "absolute": NCL_PIVOT_ABSOLUTE}


def make_options(form="condensed", precision="fp64", pivot_eps=0.0, ir_max_steps=10, ir_tol=1e-12,
                 ir_stall=0.5, ordering="nd", user_perm=None, use_graphs=True, small_front_max=0,
                 relax_big_zeros=-1.0, fp32_sticky=True, pivot_scale="global", ir_cw_tol=0.0, persistent=-1,
                 persistent_grid=0):
    o = Options()
    lib().ncl_kkt_default_options(C.byref(o))
    o.form = _FORMS[form] if isinstance(form, str) else int(form)
    o.precision = _PRECS[precision] if isinstance(precision, str) else int(precision)
    o.pivot_eps = float(pivot_eps)
    o.ir_max_steps = int(ir_max_steps)
    o.ir_tol = float(ir_tol)
    o.ir_stall = float(ir_stall)
    o.use_graphs = 1 if use_graphs else 0
    o.small_front_max = int(small_front_max)
    o.relax_big_zeros = float(relax_big_zeros)
    o.fp32_sticky = 1 if fp32_sticky else 0
    o.pivot_scale = _PIVS[pivot_scale] if isinstance(pivot_scale, str) else int(pivot_scale)
    o.ir_cw_tol = float(ir_cw_tol)
    o.persistent = int(persistent)
    o.persistent_grid = int(persistent_grid)
    keep = None
    if user_perm is not None:
        keep, p = _i32(user_perm)
        o.ordering = NCL_ORDER_USER
        o.user_perm = p
    else:
        o.ordering = _ORDS[ordering] if isinstance(ordering, str) else int(ordering)
    return o, keep


@dataclass
class Info:
    status: int
    ir_steps: int
    fell_back_fp64: bool
    backward_error: float
    backward_error0: float
    backward_error_cw: float
    resid_rel2: float


class KKT:
    """One analyzed KKT pattern (or a batch of independent ones)."""

    def __init__(self, handle, order, S, nnzW, nnzJ, form, n=None, m=0):
        self._h = handle
        self.m = m                            # rows of J (all systems)
        self.order = order
        self.S = S
        self.nnzW = nnzW
        self.nnzJ = nnzJ
        self.form = form
        self.n = order if n is None else n    # primal size (length of Sigma)
        self.generation = 0                   # bumped by every factor call

    # ---------------------------------------------------------------- create
    @classmethod
    def analyze(cls, n, m, W_colptr, W_rowidx, J_rowptr, J_colidx, host_only=False, **opts):
        o, keep = make_options(**opts)
        arrs = [_i32(a) for a in (W_colptr, W_rowidx, J_rowptr, J_colidx)]
        h = C.c_void_p()
        f = lib().ncl_kkt_analyze_host if host_only else lib().ncl_kkt_analyze
        _check(f(C.byref(h), C.byref(o), int(n), int(m), *[a[1] for a in arrs]), "ncl_kkt_analyze")
        del keep
        order = n if o.form == NCL_CONDENSED else n + m
        return cls(h, order, 1, int(arrs[0][0][-1]), int(arrs[2][0][-1]) if m > 0 else 0, o.form, n=int(n),
                   m=int(m))

    @classmethod
    def from_input(cls, inp, host_only=False, **opts):
        return cls.analyze(inp.n, inp.m, inp.W_colptr, inp.W_rowidx, inp.J_rowptr, inp.J_colidx,
                           host_only=host_only, **opts)

    @classmethod
    def analyze_batched(cls, inputs, **opts):
        o, keep = make_options(**opts)
        cnt = len(inputs)
        ns = np.array([i.n for i in inputs], np.int32)
        ms = np.array([i.m for i in inputs], np.int32)
        held = []
        tabs = []
        for field in ("W_colptr", "W_rowidx", "J_rowptr", "J_colidx"):
            ptrs = (C.POINTER(C.c_int32) * cnt)()
            for k, i in enumerate(inputs):
                a, p = _i32(getattr(i, field))
                held.append(a)
                ptrs[k] = p
            tabs.append(ptrs)
        h = C.c_void_p()
        _check(lib().ncl_kkt_analyze_batched(C.byref(h), C.byref(o), cnt, ns.ctypes.data_as(C.POINTER(C.c_int32)),
                                              ms.ctypes.data_as(C.POINTER(C.c_int32)), *tabs),
               "ncl_kkt_analyze_batched")
        del keep
        return cls(h, int(ns.sum()), cnt, int(sum(int(i.W_colptr[-1]) for i in inputs)),
                   int(sum(int(i.J_rowptr[-1]) for i in inputs)), o.form, m=int(ms.sum()))

    def close(self):
        if self._h:
            lib().ncl_kkt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- numeric
    def factor(self, W_val, Sigma, J_val, rho, stream=None):
        """Assemble and factor on the device (W_val, Sigma, J_val: float64 CUDA
        tensors of nnz(W), n and nnz(J) elements; rho a float, or one per
        system for a batched handle).  Returns the status (0 or a warning)."""
        pw = _dev(W_val, self.nnzW, "W_val", allow_none=self.nnzW == 0)
        ps = _dev(Sigma, self.n, "Sigma")
        pj = _dev(J_val, self.nnzJ, "J_val", allow_none=self.nnzJ == 0)
        st = _stream(stream)
        self.generation += 1
        if self.S == 1 and np.ndim(rho) == 0:
            rc = lib().ncl_kkt_factor(self._h, pw, ps, pj, float(rho), st)
        else:
            r = np.ascontiguousarray(np.asarray(rho, np.float64).reshape(-1))
            if r.size != self.S:
                raise ValueError(f"rho has {r.size} values, expected one per system ({self.S})")
            rc = lib().ncl_kkt_factor_batched(self._h, pw, ps, pj, r.ctypes.data_as(C.POINTER(C.c_double)), st)
        return _check(rc, "ncl_kkt_factor")

    # ------------------------------------------- slack elimination, recovery
    # Sigma_s: one value per row of J (float64 CUDA), +inf on equality rows.
    def factor_k1s(self, W_val, Sigma_t, J_val, Sigma_s, rho, stream=None):
        """Assemble and factor K1s (eq. K1s): K1 with the products of row r of
        J weighted by Sigma_s,r / (rho + Sigma_s,r)."""
        pw = _dev(W_val, self.nnzW, "W_val", allow_none=self.nnzW == 0)
        ps = _dev(Sigma_t, self.n, "Sigma_t")
        pj = _dev(J_val, self.nnzJ, "J_val", allow_none=self.nnzJ == 0)
        pss = _dev(Sigma_s, self.m, "Sigma_s")
        r = np.ascontiguousarray(np.asarray(rho, np.float64).reshape(-1))
        if r.size != self.S:
            raise ValueError(f"rho has {r.size} values, expected one per system ({self.S})")
        self.generation += 1
        rc = lib().ncl_kkt_factor_k1s(self._h, pw, ps, pj, pss, r.ctypes.data_as(C.POINTER(C.c_double)),
                                      _stream(stream))
        return _check(rc, "ncl_kkt_factor_k1s")

    def factor_regularized(self, W_val, Sigma, J_val, rho, delta_init=1e-4, growth=8.0, delta_max=1e40,
                           Sigma_s=None, stream=None):
        """Inertia correction: factors with delta = 0, delta_init, delta_init *
        growth, ... until the inertia is the expected one.  Returns (status,
        delta, factorizations)."""
        pw = _dev(W_val, self.nnzW, "W_val", allow_none=self.nnzW == 0)
        ps = _dev(Sigma, self.n, "Sigma")
        pj = _dev(J_val, self.nnzJ, "J_val", allow_none=self.nnzJ == 0)
        pss = _dev(Sigma_s, self.m, "Sigma_s", allow_none=True)
        d, a = C.c_double(), C.c_int32()
        self.generation += 1
        rc = lib().ncl_kkt_factor_regularized(self._h, pw, ps, pj, pss, float(rho), float(delta_init),
                                              float(growth), float(delta_max), C.byref(d), C.byref(a),
                                              _stream(stream))
        return _check(rc, "ncl_kkt_factor_regularized"), d.value, a.value

    def _out(self, t, numel, like):
        import torch
        return torch.empty(numel, dtype=torch.float64, device=like.device) if t is None else t

    def k1s_rhs(self, J_val, r_t, r_s, Sigma_s, b=None, stream=None):
        """b = r_t + rho J_I^T (Sigma_s + rho I)^-1 r_s (length n)."""
        b = self._out(b, self.n, r_t)
        _check(lib().ncl_kkt_k1s_rhs(self._h, _dev(J_val, self.nnzJ, "J_val", self.nnzJ == 0),
                                     _dev(r_t, self.n, "r_t"), _dev(r_s, self.m, "r_s"),
                                     _dev(Sigma_s, self.m, "Sigma_s"), _dev(b, self.n, "b"), _stream(stream)),
               "ncl_kkt_k1s_rhs")
        return b

    def k1s_recover(self, J_val, dt, r_s, Sigma_s, ds=None, stream=None):
        """Delta s = (Sigma_s + rho I)^-1 (rho J_I dt + r_s); 0 on equality rows."""
        ds = self._out(ds, self.m, dt)
        _check(lib().ncl_kkt_k1s_recover(self._h, _dev(J_val, self.nnzJ, "J_val", self.nnzJ == 0),
                                         _dev(dt, self.n, "dt"), _dev(r_s, self.m, "r_s"),
                                         _dev(Sigma_s, self.m, "Sigma_s"), _dev(ds, self.m, "ds"), _stream(stream)),
               "ncl_kkt_k1s_recover")
        return ds

    def recover_dy(self, J_val, dx, c, y_k, y, dy=None, stream=None):
        """Delta y = -rho (J dx + c) + y_k - y."""
        dy = self._out(dy, self.m, dx)
        _check(lib().ncl_kkt_recover_dy(self._h, _dev(J_val, self.nnzJ, "J_val", self.nnzJ == 0),
                                        _dev(dx, self.n, "dx"), _dev(c, self.m, "c"), _dev(y_k, self.m, "y_k"),
                                        _dev(y, self.m, "y"), _dev(dy, self.m, "dy"), _stream(stream)),
               "ncl_kkt_recover_dy")
        return dy

    def recover_dr(self, dy, y_k, y, r, dr=None, stream=None):
        """Delta r = (dy - y_k + y) / rho - r."""
        dr = self._out(dr, self.m, dy)
        _check(lib().ncl_kkt_recover_dr(self._h, _dev(dy, self.m, "dy"), _dev(y_k, self.m, "y_k"),
                                        _dev(y, self.m, "y"), _dev(r, self.m, "r"), _dev(dr, self.m, "dr"),
                                        _stream(stream)), "ncl_kkt_recover_dr")
        return dr

    def recover_dz(self, x, l, u, z_l, z_u, dx, mu, dz_l=None, dz_u=None, stream=None):
        """(Delta z_l, Delta z_u) of the eliminated bound-multiplier blocks."""
        dz_l = self._out(dz_l, self.n, x)
        dz_u = self._out(dz_u, self.n, x)
        ptrs = [_dev(a, self.n, nm) for a, nm in ((x, "x"), (l, "l"), (u, "u"), (z_l, "z_l"), (z_u, "z_u"),
                                                   (dx, "dx"))]
        _check(lib().ncl_kkt_recover_dz(self._h, *ptrs, float(mu), _dev(dz_l, self.n, "dz_l"),
                                        _dev(dz_u, self.n, "dz_u"), _stream(stream)), "ncl_kkt_recover_dz")
        return dz_l, dz_u

    def barrier_sigma(self, x, l, u, z_l, z_u, sigma=None, stream=None):
        """Sigma = Z_l / (x - l) + Z_u / (u - x)."""
        sigma = self._out(sigma, self.n, x)
        ptrs = [_dev(a, self.n, nm) for a, nm in ((x, "x"), (l, "l"), (u, "u"), (z_l, "z_l"), (z_u, "z_u"))]
        _check(lib().ncl_kkt_barrier_sigma(self._h, *ptrs, _dev(sigma, self.n, "sigma"), _stream(stream)),
               "ncl_kkt_barrier_sigma")
        return sigma

    def solve(self, B, X=None, stream=None):
        """Solve K X = B (B: (order,) or (order, nrhs) float64 on the device)."""
        import torch
        if not isinstance(B, torch.Tensor) or B.dtype != torch.float64 or not B.is_cuda:
            raise TypeError("B must be a float64 CUDA tensor")
        vec = B.dim() == 1
        B2 = B.reshape(self.order, -1)
        Bc = B2.t().contiguous().t() if not B2.t().is_contiguous() else B2   # column-major view
        nrhs = Bc.shape[1]
        if X is None:
            X = torch.empty((nrhs, self.order), dtype=torch.float64, device=B.device).t()
        px, ldx, nx = _dev_cols(X, self.order, "X")
        if nx != nrhs:
            raise ValueError(f"X has {nx} columns, expected {nrhs}")
        info = SolveInfo()
        rc = lib().ncl_kkt_solve(self._h, _ptr(Bc), self.order, px, ldx, nrhs, _stream(stream), C.byref(info))
        _check(rc, "ncl_kkt_solve")
        out = X.reshape(self.order) if vec else X
        return out, Info(rc, info.ir_steps, bool(info.fell_back_fp64), info.backward_error, info.backward_error0,
                         info.backward_error_cw, info.resid_rel2)

    def inertia(self):
        v = [C.c_int64() for _ in range(4)]
        _check(lib().ncl_kkt_inertia(self._h, *[C.byref(x) for x in v]), "ncl_kkt_inertia")
        return tuple(int(x.value) for x in v)

    def inertia_batched(self):
        out = np.zeros(4 * self.S, np.int64)
        _check(lib().ncl_kkt_inertia_batched(self._h, out.ctypes.data_as(C.POINTER(C.c_int64))),
               "ncl_kkt_inertia_batched")
        return out.reshape(self.S, 4)

    def backward(self, J_val, X, Lam, gW=None, gSigma=None, gJ=None, gRho=None, stream=None, noalloc=False):
        """Adjoint of the last factorization's solve (condensed form): X and Lam
        are (order, nrhs) column-major with the same leading dimension;
        gradients are overwritten (gRho: one value per system).  noalloc=True
        calls ncl_kkt_backward_noalloc (fixed library scratch)."""
        px, ldx, nx = _dev_cols(X, self.order, "X")
        pl, ldl, nl = _dev_cols(Lam, self.order, "Lambda")
        if nx != nl or ldx != ldl:
            raise ValueError("X and Lambda must have the same shape and leading dimension")
        pj = _dev(J_val, self.nnzJ, "J_val", allow_none=self.nnzJ == 0)
        f = lib().ncl_kkt_backward_noalloc if noalloc else lib().ncl_kkt_backward
        _check(f(self._h, pj, px, pl, ldx, nx,
                                      _dev(gW, self.nnzW, "gW", True), _dev(gSigma, self.order, "gSigma", True),
                                      _dev(gJ, self.nnzJ, "gJ", True), _dev(gRho, self.S, "gRho", True),
                                      _stream(stream)),
               "ncl_kkt_backward")

    # ---------------------------------------------------------------- inspect
    def stats(self) -> dict:
        s = Stats()
        _check(lib().ncl_kkt_get_stats(self._h, C.byref(s)), "ncl_kkt_get_stats")
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def perm(self):
        p = np.zeros(self.order, np.int32)
        _check(lib().ncl_kkt_get_perm(self._h, p.ctypes.data_as(C.POINTER(C.c_int32))), "ncl_kkt_get_perm")
        return p

    def supernodes(self):
        ns = self.stats()["n_supernodes"]
        first = np.zeros(ns + 1, np.int32)
        parent = np.zeros(ns, np.int32)
        rp = np.zeros(ns + 1, np.int64)
        P32 = C.POINTER(C.c_int32)
        _check(lib().ncl_kkt_get_supernodes(self._h, first.ctypes.data_as(P32), parent.ctypes.data_as(P32),
                                            rp.ctypes.data_as(C.POINTER(C.c_int64)), None), "supernodes")
        rows = np.zeros(max(int(rp[-1]), 1), np.int32)
        _check(lib().ncl_kkt_get_supernodes(self._h, None, None, None, rows.ctypes.data_as(P32)), "supernodes")
        return first, parent, rp, rows[:int(rp[-1])]

    def system_times(self):
        """(factor_ms, solve_ms) per system of the last persistent factor + solve,
        in ms from the start of the factor launch."""
        f = np.zeros(self.S)
        sv = np.zeros(self.S)
        P = C.POINTER(C.c_double)
        _check(lib().ncl_kkt_get_system_times(self._h, f.ctypes.data_as(P), sv.ctypes.data_as(P)),
               "ncl_kkt_get_system_times")
        return f, sv

    def set_timing(self, on=True):
        _check(lib().ncl_kkt_set_timing(self._h, 1 if on else 0), "ncl_kkt_set_timing")

    def timing(self) -> dict:
        t = Timing()
        _check(lib().ncl_kkt_get_timing(self._h, C.byref(t)), "ncl_kkt_get_timing")
        return t.as_dict()


def _autograd_function():
    import torch

    class KKTSolve(torch.autograd.Function):
        """X = K(W, Sigma, J, rho)^-1 B for the condensed form, with the adjoint
        of the factorization: the backward pass solves with the same factor
        (K is symmetric) and scatters -lambda x^T onto the stored entries of W,
        Sigma and J (through rho J^T J) and onto rho."""

        @staticmethod
        def forward(ctx, kkt, W_val, Sigma, J_val, rho, B):
            if kkt.S != 1 or kkt.form != NCL_CONDENSED:
                raise ValueError("kkt_solve differentiates one condensed system")
            rho_v = float(rho.item()) if torch.is_tensor(rho) else float(rho)
            kkt.factor(W_val.detach(), Sigma.detach(), J_val.detach(), rho_v)
            X, info = kkt.solve(B.detach())
            ctx.kkt = kkt
            ctx.generation = kkt.generation
            ctx.save_for_backward(J_val.detach(), X)
            ctx.rho_is_tensor = torch.is_tensor(rho)
            ctx.info = info
            return X

        @staticmethod
        def backward(ctx, Xbar):
            kkt = ctx.kkt
            if kkt.generation != ctx.generation:
                # the adjoint solve and the rho used by the gradient kernels are
                # those of the handle's current factorization
                raise RuntimeError("kkt_solve backward: the KKT handle was refactored after this forward "
                                   "pass; run backward before factoring it again, or use one handle per solve")
            J_val, X = ctx.saved_tensors
            Lam, _ = kkt.solve(Xbar.contiguous() if Xbar.dim() == 1 else Xbar)
            dev = X.device
            gW = torch.empty(kkt.nnzW, dtype=torch.float64, device=dev)
            gS = torch.empty(kkt.order, dtype=torch.float64, device=dev)
            gJ = torch.empty(kkt.nnzJ, dtype=torch.float64, device=dev)
            gR = torch.empty(kkt.S, dtype=torch.float64, device=dev)
            X2 = X.reshape(kkt.order, -1)
            L2 = Lam.reshape(kkt.order, -1)
            Xc = X2.t().contiguous().t()
            Lc = L2.t().contiguous().t()
            kkt.backward(J_val, Xc, Lc, gW, gS, gJ, gR)
            grho = gR.reshape(()) if ctx.rho_is_tensor else None
            return None, gW, gS, gJ, grho, Lam

    return KKTSolve


_KKTSolve = None


def kkt_solve(kkt, W_val, Sigma, J_val, rho, B):
    """Differentiable X = K^-1 B (condensed form) through the library."""
    global _KKTSolve
    if _KKTSolve is None:
        _KKTSolve = _autograd_function()
    return _KKTSolve.apply(kkt, W_val, Sigma, J_val, rho, B)


@dataclass
class QpSolution:
    x: object               # device tensors
    y: object
    z_l: object
    z_u: object
    status: int             # 0 optimal, 1 infeasible, 2 outer-iteration limit
    outer: int
    inner: int
    extrapolated: int
    primal_inf: float
    dual_inf: float


def qp_solve(n, m, Q_colptr, Q_rowidx, Q_val, q, A_rowptr, A_colidx, A_val, b, l, u, x0,
             eta_star=1e-8, omega_star=1e-8, max_outer=100, max_inner=100, precision="fp64", print_level=0,
             stream=None):
    """Algorithm 1 on min 1/2 x^T Q x + q^T x s.t. A x = b, l <= x <= u
    (ncl_qp_solve).  Patterns are host arrays (Q lower CSC, A CSR); values and
    vectors float64 CUDA tensors; x0 is copied, not overwritten."""
    import torch
    L = lib()
    o = QpOptions()
    L.ncl_qp_default_options(C.byref(o))
    o.eta_star, o.omega_star = float(eta_star), float(omega_star)
    o.max_outer, o.max_inner = int(max_outer), int(max_inner)
    o.precision = _PRECS[precision] if isinstance(precision, str) else int(precision)
    o.print_level = int(print_level)
    qc, qcp = _i32(Q_colptr)
    qr, qrp = _i32(Q_rowidx)
    if len(qc) != n + 1:
        raise ValueError("Q_colptr must have n + 1 entries")
    ac, acp = _i32(A_rowptr if m > 0 else [0])
    ai, aip = _i32(A_colidx if m > 0 else [0])
    if m > 0 and len(ac) != m + 1:
        raise ValueError("A_rowptr must have m + 1 entries")
    nnzQ, nnzA = int(qc[-1]), int(ac[-1]) if m > 0 else 0
    _dev(x0, n, "x0")
    x = x0.clone()
    y = torch.zeros(max(m, 1), dtype=torch.float64, device=x.device)
    z_l = torch.zeros_like(x)
    z_u = torch.zeros_like(x)
    res = QpResult()
    rc = L.ncl_qp_solve(C.byref(o), int(n), int(m), qcp, qrp, _dev(Q_val, nnzQ, "Q_val"), _dev(q, n, "q"),
                        acp, aip, _dev(A_val, nnzA, "A_val") if m > 0 else None,
                        _dev(b, m, "b") if m > 0 else None, _dev(l, n, "l"), _dev(u, n, "u"),
                        _ptr(x), _ptr(y), _ptr(z_l), _ptr(z_u), C.byref(res), _stream(stream))
    _check(rc, "ncl_qp_solve")
    return QpSolution(x, y[:m], z_l, z_u, int(res.status), int(res.outer), int(res.inner),
                      int(res.extrapolated), float(res.primal_inf), float(res.dual_inf))
