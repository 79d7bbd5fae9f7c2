"""Thin ctypes binding of libfdfd.so (argument marshalling only).

Every step of the solve runs in the library's HIP kernels; this module only
passes device pointers of torch tensors and the current HIP stream.  If the
library has not been built, importing the binding raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfdfd.so")

FDFD_OK, FDFD_ERR_ARG, FDFD_ERR_STATE, FDFD_ERR_NOMEM, FDFD_ERR_HIP, FDFD_ERR_NUMERIC, FDFD_WARN_PIVOT = range(7)
FDFD_C128, FDFD_C64_IR = 0, 1
FDFD_ANALYZE_HOST_ONLY = 1
FDFD_PROFILE = 2
FDFD_GRAPH = 4
FDFD_POL_TE = 8
FDFD_GRAD_ACCUMULATE, FDFD_GRAD_SUM_SYSTEMS = 1, 2
FDFD_TABLE_PERM, FDFD_TABLE_FRONTS, FDFD_TABLE_UPDATE, FDFD_TABLE_TASKS, FDFD_TABLE_SWEEP_ITEMS = 0, 1, 2, 3, 4

EXPORTED = ["fdfd_analyze", "fdfd_refactor", "fdfd_solve", "fdfd_solve_noalloc", "fdfd_adjoint_grad", "fdfd_query",
            "fdfd_kernel_stats", "fdfd_get_table", "fdfd_param_forward", "fdfd_param_backward",
            "fdfd_param_last_error", "fdfd_status_str", "fdfd_last_error", "fdfd_destroy"]


class Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("npml_x", ctypes.c_int32), ("npml_y", ctypes.c_int32),
                ("nsys", ctypes.c_int32), ("max_rhs", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("device", ctypes.c_int32),
                ("leaf", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("small_lds", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("mem_cap_bytes", ctypes.c_int64),
                ("syrk_group", ctypes.c_int32), ("split_kb", ctypes.c_int32),
                ("block_split", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nfronts", ctypes.c_int64), ("nlevels", ctypes.c_int64),
                ("nnz_factor", ctypes.c_int64), ("factor_bytes", ctypes.c_int64),
                ("update_bytes", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("refactor_flops", ctypes.c_double), ("schur_flops", ctypes.c_double),
                ("max_front", ctypes.c_int32), ("max_pivots", ctypes.c_int32),
                ("leaf", ctypes.c_int32), ("n_perturbed", ctypes.c_int32),
                ("min_pivot_ratio", ctypes.c_double),
                ("ir_steps_solve", ctypes.c_int32), ("ir_steps_adjoint", ctypes.c_int32),
                ("rel_residual_solve", ctypes.c_double), ("rel_residual_adjoint", ctypes.c_double),
                ("device_flags", ctypes.c_int32), ("small_levels", ctypes.c_int32),
                ("refactor_ms", ctypes.c_double), ("solve_ms", ctypes.c_double), ("adjoint_ms", ctypes.c_double),
                ("rhs_group", ctypes.c_int32), ("syrk_group", ctypes.c_int32), ("split_kb", ctypes.c_int32),
                ("block_split", ctypes.c_int32), ("small_lds", ctypes.c_int32), ("reserved3", ctypes.c_int32),
                ("analyze_ms", ctypes.c_double), ("setup_ms", ctypes.c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("alg_flops", ctypes.c_double)]


class ParamDesc(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("h", ctypes.c_int32), ("i0", ctypes.c_int32), ("j0", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("radius", ctypes.c_double),
                ("beta", ctypes.c_double), ("eta", ctypes.c_double), ("eps_min", ctypes.c_double),
                ("eps_max", ctypes.c_double)]


class FDFDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfdfd.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FDFDError(-1, f"{path} is missing: run `python -m paper_2307_05388_amd.build`")
    # torch ships its own HIP runtime (same soname).  Importing torch first makes
    # the library bind to that copy, so torch streams and pointers are valid in
    # it and only one runtime is ever mapped.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    _check_single_runtime()
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.fdfd_analyze.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(vp)]
    lib.fdfd_refactor.argtypes = [vp, vp, i64, ctypes.POINTER(dbl), vp]
    lib.fdfd_solve.argtypes = [vp, vp, vp, i32, i32, dbl, vp]
    lib.fdfd_solve_noalloc.argtypes = [vp, vp, vp, i32, i32, dbl, vp]
    lib.fdfd_adjoint_grad.argtypes = [vp, vp, vp, i32, i32, dbl, vp, vp, i32, vp]
    lib.fdfd_query.argtypes = [vp, ctypes.POINTER(Info)]
    lib.fdfd_get_table.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32), i64]
    lib.fdfd_kernel_stats.argtypes = [vp, ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
    lib.fdfd_status_str.argtypes = [i32]
    lib.fdfd_status_str.restype = ctypes.c_char_p
    lib.fdfd_last_error.argtypes = [vp]
    lib.fdfd_last_error.restype = ctypes.c_char_p
    lib.fdfd_destroy.argtypes = [vp]
    lib.fdfd_destroy.restype = None
    lib.fdfd_param_forward.argtypes = [ctypes.POINTER(ParamDesc), vp, vp, vp, vp]
    lib.fdfd_param_backward.argtypes = [ctypes.POINTER(ParamDesc), vp, vp, vp, vp, vp]
    lib.fdfd_param_last_error.argtypes = []
    lib.fdfd_param_last_error.restype = ctypes.c_char_p
    for name in ["fdfd_analyze", "fdfd_refactor", "fdfd_solve", "fdfd_solve_noalloc", "fdfd_adjoint_grad",
                 "fdfd_query", "fdfd_get_table", "fdfd_kernel_stats", "fdfd_param_forward",
                 "fdfd_param_backward"]:
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check_single_runtime():
    try:
        maps = open("/proc/self/maps").read()
    except OSError:
        return
    paths = {ln.split()[-1] for ln in maps.splitlines() if "libamdhip64" in ln}
    if len(paths) > 1:
        raise FDFDError(-1, f"two HIP runtimes are mapped: {sorted(paths)}")


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Cached analysis + factors of one grid (all systems share the pattern)."""

    def __init__(self, nx, ny, npml_x, npml_y=None, nsys=1, max_rhs=1, prec="c128",
                 device=-1, leaf=0, host_only=False, mem_cap_bytes=0, profile=False, graph=False,
                 small_lds=0, tuned=True, pol="tm", syrk_group=0, split_kb=0, block_split=0):
        """With every layout knob at 0 (leaf, small_lds, syrk_group, split_kb,
        block_split) and tuned=True the layout comes from the autotuner's
        table for this GPU and workload when it has an entry.  pol: "tm" (Ez)
        or "te" (Hz, FDFD_POL_TE)."""
        if pol not in ("tm", "te"):
            raise ValueError(f"unknown polarisation {pol!r}")
        self._lib = load_library()
        self._h = ctypes.c_void_p()
        self.tuned_entry = None
        if tuned and (leaf, small_lds, syrk_group, split_kb, block_split) == (0, 0, 0, 0, 0):
            from .autotune import lookup
            hit = lookup(nx, ny, npml_x, nsys, max_rhs, "c64" if prec in ("c64", FDFD_C64_IR) else "c128")
            if hit:
                leaf, small_lds = hit["leaf"], hit["small_lds"]
                syrk_group, split_kb, block_split = hit["syrk_group"], hit["split_kb"], hit["block_split"]
                self.tuned_entry = hit
        d = Desc(nx=nx, ny=ny, npml_x=npml_x, npml_y=npml_x if npml_y is None else npml_y,
                 nsys=nsys, max_rhs=max_rhs, prec=FDFD_C64_IR if prec in ("c64", FDFD_C64_IR) else FDFD_C128,
                 device=device, leaf=leaf, small_lds=small_lds,
                 syrk_group=syrk_group, split_kb=split_kb, block_split=block_split,
                 flags=(FDFD_ANALYZE_HOST_ONLY if host_only else 0) | (FDFD_PROFILE if profile else 0)
                 | (FDFD_GRAPH if graph else 0) | (FDFD_POL_TE if pol == "te" else 0),
                 mem_cap_bytes=mem_cap_bytes)
        if prec not in ("c64", "c128", FDFD_C64_IR, FDFD_C128):
            raise ValueError(f"unknown precision {prec!r}")
        st = self._lib.fdfd_analyze(ctypes.byref(d), ctypes.byref(self._h))
        if st != FDFD_OK:
            raise FDFDError(st, self._lib.fdfd_last_error(None).decode())
        self.nx, self.ny, self.N = nx, ny, nx * ny
        self.nsys, self.max_rhs = nsys, max_rhs
        self.prec = "c64" if d.prec == FDFD_C64_IR else "c128"
        self.pol = pol
        self.host_only = host_only
        self.generation = 0

    # -- helpers --------------------------------------------------------
    def _check(self, st):
        if st not in (FDFD_OK, FDFD_WARN_PIVOT):
            raise FDFDError(st, self._lib.fdfd_last_error(self._h).decode())
        return st

    def close(self):
        if self._h:
            self._lib.fdfd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass

    # -- the four calls -------------------------------------------------
    def refactor(self, eps, omegas, stream=None):
        """eps: float64 CUDA tensor (ny, nx) shared, or (nsys, ny, nx)."""
        import torch
        assert eps.is_cuda and eps.dtype == torch.float64 and eps.is_contiguous()
        stride = 0 if eps.dim() == 2 else self.N
        om = (ctypes.c_double * self.nsys)(*[float(w) for w in np.atleast_1d(omegas)])
        self._check(self._lib.fdfd_refactor(self._h, _ptr(eps), stride, om, _stream_handle(stream)))
        self.generation += 1

    def solve(self, b, x=None, max_ir=0, tol=0.0, stream=None):
        """b: complex128 CUDA tensor (nsys, nrhs, N); returns x of the same shape."""
        import torch
        assert b.is_cuda and b.dtype == torch.complex128 and b.is_contiguous()
        nrhs = b.shape[-2] if b.dim() >= 2 else 1
        if x is None:
            x = torch.empty_like(b)
        self._check(self._lib.fdfd_solve(self._h, _ptr(b), _ptr(x), nrhs, max_ir, tol,
                                         _stream_handle(stream)))
        return x

    def solve_noalloc(self, b, x, max_ir=0, tol=0.0, stream=None):
        """fdfd_solve_noalloc: the forward solve with its work vectors in the
        library's static device array (x must be given; nothing is allocated)."""
        import torch
        assert b.is_cuda and b.dtype == torch.complex128 and b.is_contiguous()
        assert x.shape == b.shape and x.dtype == b.dtype and x.is_contiguous()
        nrhs = b.shape[-2] if b.dim() >= 2 else 1
        self._check(self._lib.fdfd_solve_noalloc(self._h, _ptr(b), _ptr(x), nrhs, max_ir, tol,
                                                 _stream_handle(stream)))
        return x

    def adjoint_grad(self, x, g, lam=None, grad=None, flags=0, max_ir=0, tol=0.0, stream=None):
        """Adjoint solve with the cached factor + gradient -2 w^2 Re(lam x)."""
        import torch
        assert x.shape == g.shape and g.dtype == torch.complex128 and g.is_contiguous()
        nrhs = g.shape[-2] if g.dim() >= 2 else 1
        if grad is None:
            shape = (self.N,) if flags & FDFD_GRAD_SUM_SYSTEMS else (self.nsys, self.N)
            grad = torch.empty(shape, dtype=torch.float64, device=g.device)
        lp = _ptr(lam) if lam is not None else ctypes.c_void_p()
        self._check(self._lib.fdfd_adjoint_grad(self._h, _ptr(x), _ptr(g), nrhs, max_ir, tol, lp,
                                                _ptr(grad), flags, _stream_handle(stream)))
        return grad

    def query(self):
        info = Info()
        st = self._lib.fdfd_query(self._h, ctypes.byref(info))
        out = {k: getattr(info, k) for k, _ in Info._fields_}
        out["status"] = st
        out["status_str"] = self._lib.fdfd_status_str(st).decode()
        if st not in (FDFD_OK, FDFD_WARN_PIVOT):
            out["error"] = self._lib.fdfd_last_error(self._h).decode()
        return out

    def kernel_stats(self):
        """Per-kernel event totals since the last call (plans made with profile=True)."""
        buf = (KernelStat * 32)()
        n = ctypes.c_int32()
        self._check(self._lib.fdfd_kernel_stats(self._h, buf, 32, ctypes.byref(n)))
        return {buf[i].name.decode(): {"launches": buf[i].launches, "total_ms": buf[i].total_ms,
                                       "alg_bytes": buf[i].alg_bytes, "alg_flops": buf[i].alg_flops}
                for i in range(n.value)}

    def table(self, which):
        info = self.query() if self.host_only else None
        if which == FDFD_TABLE_PERM:
            n = self.N
        elif which == FDFD_TABLE_FRONTS:
            info = info or self.query()
            n = 4 * info["nfronts"]
        elif which in (FDFD_TABLE_TASKS, FDFD_TABLE_SWEEP_ITEMS):
            # grown until the table fits (fdfd_get_table refuses a short buffer)
            out = np.zeros(1 << 12, dtype=np.int32)
            while True:
                st = self._lib.fdfd_get_table(self._h, which, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                              out.size)
                if st == FDFD_OK:
                    break
                out = np.zeros(out.size * 4, dtype=np.int32)
            if which == FDFD_TABLE_TASKS:
                return out[1:1 + 5 * int(out[0])].reshape(-1, 5)
            # (height H, item offsets, fronts)
            nit = int(out[0])
            ptr = out[2:3 + nit].copy()
            return int(out[1]), ptr, out[3 + nit:3 + nit + int(ptr[-1])].copy()
        else:
            fr = self.table(FDFD_TABLE_FRONTS).reshape(-1, 4)
            n = int(fr[:, 2].sum())
        out = np.zeros(max(1, n), dtype=np.int32)
        st = self._lib.fdfd_get_table(self._h, which, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), out.size)
        self._check(st)
        return out[:n]


def param_desc(w, h, radius, beta, eta=0.5, eps_min=2.085, eps_max=12.11, i0=0, j0=0, nx=None, ny=None):
    """Descriptor of the design parametrisation (a compact block by default)."""
    return ParamDesc(w=w, h=h, i0=i0, j0=j0, nx=w if nx is None else nx, ny=h if ny is None else ny,
                     radius=radius, beta=beta, eta=eta, eps_min=eps_min, eps_max=eps_max)


def param_forward(desc, theta, rho, eps, stream=None):
    """fdfd_param_forward on device tensors (float64)."""
    lib = load_library()
    st = lib.fdfd_param_forward(ctypes.byref(desc), _ptr(theta), _ptr(rho), _ptr(eps), _stream_handle(stream))
    if st != FDFD_OK:
        raise FDFDError(st, lib.fdfd_param_last_error().decode())


def param_backward(desc, rho, grad_eps, work, grad_theta, stream=None):
    """fdfd_param_backward on device tensors (float64)."""
    lib = load_library()
    st = lib.fdfd_param_backward(ctypes.byref(desc), _ptr(rho), _ptr(grad_eps), _ptr(work), _ptr(grad_theta),
                                 _stream_handle(stream))
    if st != FDFD_OK:
        raise FDFDError(st, lib.fdfd_param_last_error().decode())


def status_str(code: int) -> str:
    return load_library().fdfd_status_str(code).decode()
