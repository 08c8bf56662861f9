"""Thin ctypes binding of libhmle.so (the C ABI declared in include/hmle.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device buffers are torch tensors on the GPU (float64, contiguous); a tensor of
shape (c, n) is an n x c column-major block with leading dimension n.
The library must be built (paper_2303_10102_amd.build); importing this module
without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np

LIBPATH = Path(__file__).resolve().with_name("libhmle.so")
PARAM_NAMES = ("kappa", "alpha", "tau2", "sigma2", "tau2_2")   # tau2_2: bivariate model only

_lib = None


class HmleError(RuntimeError):
    def __init__(self, func, status, msg):
        super().__init__(f"{func} failed with status {status}: {msg}")
        self.status = status


STATUS = {0: "HM_OK", 1: "HM_E_INVAL", 2: "HM_E_NOMEM", 3: "HM_E_NOT_SPD", 4: "HM_E_RANK",
          5: "HM_E_NONFINITE", 6: "HM_E_STATE", 7: "HM_E_DEVICE"}

_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I = C.c_int

_SIGS = {
    "hm_last_error": ([], C.c_char_p),
    "hm_ctx_create": ([_I, _P, _P, _P, _P, C.POINTER(_P)], _I),
    "hm_ctx_destroy": ([_P], None),
    "hm_model_create": ([_I, _P, _I, _I, _I, C.POINTER(_P)], _I),
    "hm_model_create_spde": ([_P, _I, _I, _I, C.c_double, _I, C.POINTER(_I), C.c_longlong, _I, C.POINTER(_P)], _I),
    "hm_model_create_op": ([_P, _I, _D, _I, _I, _P, _P, C.POINTER(_P)], _I),
    "hm_model_create_adr": ([_P, _I, C.c_double, C.c_double, C.c_double, _I, C.POINTER(_P)], _I),
    "hm_model_destroy": ([_P], None),
    "hm_model_info": ([_P, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)], _I),
    "hm_model_rows": ([_P, C.POINTER(_I)], _I),
    "hm_model_set_stream": ([_P, _P], _I),
    "hm_model_autotune": ([_P, _I, _D], _I),
    "hm_model_tuning": ([_P, C.POINTER(_I), C.POINTER(C.c_longlong), _I], _I),
    "hm_model_perm": ([_P, C.POINTER(_I)], _I),
    "hm_kapply": ([_P, _D, _P, _I, _I, _P, _I, _I], _I),
    "hm_kapply_noalloc": ([_P, _D, _P, _I, _I, _P, _I, _I], _I),
    "hm_sketch_create": ([_P, _P, _I, _I, _D, C.POINTER(_P)], _I),
    "hm_sketch_create_tol": ([_P, _P, _I, _I, C.c_double, _D, C.POINTER(_P)], _I),
    "hm_sketch_destroy": ([_P], None),
    "hm_sketch_ranks": ([_P, C.POINTER(_I), C.POINTER(_I)], _I),
    "hm_H_create": ([_P, _I, C.POINTER(_I), C.POINTER(_P)], _I),
    "hm_H_destroy": ([_P], None),
    "hm_build": ([_P, _D], _I),
    "hm_factor": ([_P], _I),
    "hm_logdet": ([_P, _D], _I),
    "hm_solve": ([_P, _P, _P, C.c_longlong, C.c_longlong], _I),
    "hm_loglik_grad": ([_P, _P, _D, _D], _I),
    "hm_fisher": ([_P, _D], _I),
    "hm_iteration": ([_P, _D, _P, _D, _D, _D], _I),
    "hm_H_set_precision": ([_P, _I], _I),
    "hm_iteration_batched": ([_I, C.POINTER(_P), _D, C.POINTER(_P), _D, _D, _D], _I),
    "hm_loglik_grad_adjoint": ([_P, _D, _P, _D, _D], _I),
    "hm_loglik": ([_P, _D, _P, _D], _I),
    "hm_grad_reverse": ([_P, _D], _I),
    "hm_stats": ([_P, _P, C.c_size_t], _I),
    "hm_stats_reset": ([_P], _I),
    "hm_export": ([_P, _I, _P], _I),
    "hm_profile_enable": ([_P, _I], _I),
    "hm_profile_read": ([_P, _D, C.POINTER(C.c_longlong), _D, _D], _I),
}
PROFILE_FAMILIES = {"expand": 0, "reduce": 1, "dst": 2, "leaf_gemm": 4}


def lib():
    """Load libhmle.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIBPATH.exists():
            raise RuntimeError(f"{LIBPATH} is missing: build it with paper_2303_10102_amd.build.build()")
        L = C.CDLL(str(LIBPATH))
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(func, st):
    if st != 0:
        msg = lib().hm_last_error().decode(errors="replace")
        raise HmleError(func, STATUS.get(st, st), msg)


def _theta(t):
    """theta_full as a C array: 4 entries, or 5 for the bivariate model (second nugget last)."""
    vals = [float(x) for x in t]
    if len(vals) not in (4, 5):
        raise ValueError("theta_full has 4 entries (5 for the bivariate model)")
    return (C.c_double * len(vals))(*vals)


def _ptr(t):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Context:
    """hm_ctx: device, stream and the allocator of the library's device memory.

    allocator="torch" hands every device buffer of the models, sketches and H handles
    created with this context to torch's caching allocator (so torch.cuda.memory_allocated
    accounts for them and the memory is reused by torch after release);
    allocator="hip" lets the library call hipMalloc / hipFree itself.
    """

    def __init__(self, device=0, stream=None, allocator="torch"):
        import torch
        self.device = int(device)
        self.stream_handle = int(_stream_handle(stream).value or 0)
        self._cb = None
        alloc = free = None
        if allocator == "torch":
            def _alloc(uctx, nbytes):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream_handle)
                except Exception:          # out of memory: the library reports HM_E_NOMEM
                    return None

            release = torch.cuda.caching_allocator_delete

            def _free(uctx, ptr):
                try:
                    release(int(ptr))
                except Exception:         # interpreter shutdown: torch has already gone
                    pass

            self._cb = (_ALLOC_FN(_alloc), _FREE_FN(_free))
            alloc = C.cast(self._cb[0], C.c_void_p)
            free = C.cast(self._cb[1], C.c_void_p)
        elif allocator != "hip":
            raise ValueError("allocator must be 'torch' or 'hip'")
        h = _P()
        _check("hm_ctx_create", lib().hm_ctx_create(self.device, C.c_void_p(self.stream_handle), alloc, free, None,
                                                    C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().hm_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """SPDE stencil covariance model on a dim-D Dirichlet grid of side N.

    Device memory comes from a Context (by default one of its own backed by torch's
    caching allocator); h is the grid spacing (default 1/(N+1), the unit square).
    obs: optional grid indices (x fastest in 2D) of the observed nodes; the model is then
    the observed subset (n = len(obs), observation order = obs), the physics on the full
    grid and the nugget on the observations.
    nvars=2: the bivariate co-kriging model (y1 = B^-1 w, y2 = A^-1 B^-1 w at every node,
    stacked (y1; y2), n = 2 N^dim), theta_full = (kappa, alpha, tau2_1, sigma2, tau2_2)."""

    def __init__(self, dim, N, leaf, device=0, stream=None, ctx=None, h=None, allocator="torch", obs=None,
                 nvars=1):
        import torch
        self.device = torch.device("cuda", device)
        self.ctx = ctx if ctx is not None else Context(device, stream, allocator)
        self._own_ctx = ctx is None
        hh = _P()
        spacing = 1.0 / (N + 1) if h is None else float(h)
        if obs is None:
            oidx, nobs = None, 0
        else:
            self._obs = np.ascontiguousarray(np.asarray(obs), dtype=np.int32)
            oidx, nobs = self._obs.ctypes.data_as(C.POINTER(C.c_int)), int(self._obs.size)
        with torch.cuda.device(device):
            _check("hm_model_create_spde",
                   lib().hm_model_create_spde(self.ctx._h, dim, N, N if dim == 2 else 1, spacing, int(nvars), oidx,
                                              nobs, leaf, C.byref(hh)))
        self.nvars = int(nvars)
        self._h = hh
        n, lv, lf = _I(), _I(), _I()
        _check("hm_model_info", lib().hm_model_info(hh, C.byref(n), C.byref(lv), C.byref(lf)))
        self.dim, self.N, self.n, self.levels, self.leaf = dim, N, n.value, lv.value, lf.value
        self.h = spacing
        rows = _I()
        _check("hm_model_rows", lib().hm_model_rows(hh, C.byref(rows)))
        self.rows = rows.value      # tree-ordered layout: n, or more with padded leaves

    def set_stream(self, stream):
        """Move the model's later work to another torch stream (None = current stream)."""
        _check("hm_model_set_stream", lib().hm_model_set_stream(self._h, _stream_handle(stream)))
        self.stream = stream
        if self._own_ctx:      # later allocations are used on the new stream
            self.ctx.stream_handle = int(_stream_handle(stream).value or 0)

    def autotune(self, kc):
        """Time the panel-kernel variants on this model's shapes and keep the fastest."""
        rep = (C.c_double * 8)()
        _check("hm_model_autotune", lib().hm_model_autotune(self._h, int(kc), rep))
        return dict(expand_ms={1: rep[0], 2: rep[1], 3: rep[2]},
                    reduce_ms={"never": rep[3], "below_1024": rep[4], "always": rep[5]},
                    expand_variant=int(rep[6]), reduce_split_below=int(rep[7]))

    def tuning(self, expand_variant=None, reduce_split_below=None):
        """Read the chosen kernel variants, or set them (both arguments given)."""
        rb, thr = _I(0), C.c_longlong(0)
        if expand_variant is None:
            _check("hm_model_tuning", lib().hm_model_tuning(self._h, C.byref(rb), C.byref(thr), 0))
            return rb.value, thr.value
        rb.value, thr.value = int(expand_variant), int(reduce_split_below)
        _check("hm_model_tuning", lib().hm_model_tuning(self._h, C.byref(rb), C.byref(thr), 1))
        return rb.value, thr.value

    def perm(self):
        """Tree position -> grid index (rows entries; -1 on padding rows)."""
        out = (C.c_int * self.rows)()
        _check("hm_model_perm", lib().hm_model_perm(self._h, out))
        return np.frombuffer(out, dtype=np.int32).copy()

    def kapply(self, theta_full, X, which=0, out=None, noalloc=False):
        """Y = op X for X a (c, rows) float64 CUDA tensor in tree order; op = K, dK/dkappa, dK/dalpha.
        noalloc: use hm_kapply_noalloc (fixed per-device scratch, no allocation)."""
        import torch
        c, n = X.shape
        Y = torch.empty_like(X) if out is None else out
        fn = "hm_kapply_noalloc" if noalloc else "hm_kapply"
        _check(fn, getattr(lib(), fn)(self._h, _theta(theta_full), _ptr(X), n, c, _ptr(Y), n, which))
        return Y

    def profile_enable(self, family):
        """Time every launch of a kernel family ('expand', 'reduce', 'dst', 'leaf_gemm'; None = off)."""
        fam = -1 if family is None else PROFILE_FAMILIES[family]
        _check("hm_profile_enable", lib().hm_profile_enable(self._h, fam))

    def profile_read(self):
        ms, fl, by = C.c_double(), C.c_double(), C.c_double()
        n = C.c_longlong()
        _check("hm_profile_read", lib().hm_profile_read(self._h, C.byref(ms), C.byref(n), C.byref(fl), C.byref(by)))
        return dict(ms=ms.value, launches=n.value, flops=fl.value, bytes=by.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().hm_model_destroy(self._h)
            self._h = None
        if getattr(self, "_own_ctx", False) and getattr(self, "ctx", None) is not None:
            self.ctx.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_OP_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_void_p, C.c_longlong,
                     C.c_longlong, C.c_void_p, C.c_longlong, C.c_void_p)


class _DLDevice(C.Structure):
    _fields_ = [("device_type", C.c_int32), ("device_id", C.c_int32)]


class _DLDataType(C.Structure):
    _fields_ = [("code", C.c_uint8), ("bits", C.c_uint8), ("lanes", C.c_uint16)]


class _DLTensor(C.Structure):
    _fields_ = [("data", C.c_void_p), ("device", _DLDevice), ("ndim", C.c_int32), ("dtype", _DLDataType),
                ("shape", C.POINTER(C.c_int64)), ("strides", C.POINTER(C.c_int64)), ("byte_offset", C.c_uint64)]


class _DLManagedTensor(C.Structure):
    _fields_ = [("dl_tensor", _DLTensor), ("manager_ctx", C.c_void_p), ("deleter", C.c_void_p)]


def device_view(ptr, c, ld, n, device):
    """A (c, n) float64 torch view of the column-major n x c device block at ptr with
    leading dimension ld (no copy), through DLPack; the memory stays the caller's."""
    import torch
    shape = (C.c_int64 * 2)(c, n)
    strides = (C.c_int64 * 2)(ld, 1)
    dev_type = 10 if torch.version.hip else 2        # kDLROCM / kDLCUDA
    mt = _DLManagedTensor(_DLTensor(C.c_void_p(ptr), _DLDevice(dev_type, device), 2, _DLDataType(2, 64, 1),
                                    shape, strides, 0), None, None)
    keep = (shape, strides, mt)
    C.pythonapi.PyCapsule_New.restype = C.py_object
    C.pythonapi.PyCapsule_New.argtypes = [C.c_void_p, C.c_char_p, C.c_void_p]
    cap = C.pythonapi.PyCapsule_New(C.addressof(mt), b"dltensor", None)
    t = torch.from_dlpack(cap)
    t._hmle_keep = keep          # the DLPack structs live as long as the view
    return t


class OpModel(Model):
    """A model on scattered points with a caller-supplied covariance operator
    (hm_model_create_op): K(theta) = sigma2 K_op(theta0, theta1) + tau2 I.

    op(which, theta_full, X, Y): X, Y are (c, n) float64 CUDA views in the caller's point
    order; write Y = K_op X (which 0), dK_op/dtheta0 X (1) or dK_op/dtheta1 X (2).  It
    runs on the model's stream (made current while it runs)."""

    def __init__(self, coords, leaf, op, device=0, stream=None, ctx=None, allocator="torch"):
        import torch
        self.device = torch.device("cuda", device)
        self.ctx = ctx if ctx is not None else Context(device, stream, allocator)
        self._own_ctx = ctx is None
        xy = np.ascontiguousarray(np.asarray(coords, dtype=np.float64))
        if xy.ndim == 1:
            xy = xy[:, None]
        n, dim = xy.shape
        self._op = op
        dev = int(device)

        def _cb(uctx, which, theta, X, ldx, c, Y, ldy, stream_h):
            try:
                th = [theta[i] for i in range(4)]
                Xv = device_view(X, int(c), int(ldx), n, dev)
                Yv = device_view(Y, int(c), int(ldy), n, dev)
                if stream_h:
                    with torch.cuda.stream(torch.cuda.ExternalStream(int(stream_h), device=self.device)):
                        op(int(which), th, Xv, Yv)
                else:                     # the null stream
                    with torch.cuda.stream(torch.cuda.default_stream(self.device)):
                        op(int(which), th, Xv, Yv)
                return 0
            except Exception as exc:      # reported as HM_E_DEVICE by the library
                import traceback
                traceback.print_exception(exc)
                return 1

        self._cb = _OP_FN(_cb)
        hh = _P()
        with torch.cuda.device(device):
            _check("hm_model_create_op", lib().hm_model_create_op(self.ctx._h, dim, xy.ctypes.data_as(_D), n, leaf,
                                                                  C.cast(self._cb, C.c_void_p), None, C.byref(hh)))
        self._h = hh
        nn, lv, lf = _I(), _I(), _I()
        _check("hm_model_info", lib().hm_model_info(hh, C.byref(nn), C.byref(lv), C.byref(lf)))
        self.dim, self.N, self.n, self.levels, self.leaf = dim, 0, nn.value, lv.value, lf.value
        self.h = None
        rows = _I()
        _check("hm_model_rows", lib().hm_model_rows(hh, C.byref(rows)))
        self.rows = rows.value


class AdrModel(Model):
    """The advection-diffusion-reaction model (hm_model_create_adr) on an N x N grid:
    K = sigma2 L^{-1} B^{-2} L^{-T} + tau2 I with theta_full = (kappa, c, tau2, sigma2)."""

    def __init__(self, N, leaf, kd, vx, vy, device=0, stream=None, ctx=None, allocator="torch"):
        import torch
        self.device = torch.device("cuda", device)
        self.ctx = ctx if ctx is not None else Context(device, stream, allocator)
        self._own_ctx = ctx is None
        hh = _P()
        with torch.cuda.device(device):
            _check("hm_model_create_adr", lib().hm_model_create_adr(self.ctx._h, int(N), float(kd), float(vx),
                                                                    float(vy), int(leaf), C.byref(hh)))
        self._h = hh
        nn, lv, lf = _I(), _I(), _I()
        _check("hm_model_info", lib().hm_model_info(hh, C.byref(nn), C.byref(lv), C.byref(lf)))
        self.dim, self.N, self.n, self.levels, self.leaf = 2, int(N), nn.value, lv.value, lf.value
        self.h = 1.0 / (N + 1)
        rows = _I()
        _check("hm_model_rows", lib().hm_model_rows(hh, C.byref(rows)))
        self.rows = rows.value


class Sketch:
    """Fixed test matrices and frozen compression (created once at theta0)."""

    def __init__(self, model, omega, rank, oversample, theta0_full, rank_tol=None):
        """rank_tol: None for the default truncation (1e-10), else the relative singular
        value below which a block's sample directions are dropped (hm_sketch_create_tol)."""
        h = _P()
        if rank_tol is None:
            _check("hm_sketch_create", lib().hm_sketch_create(model._h, _ptr(omega), rank, oversample,
                                                              _theta(theta0_full), C.byref(h)))
        else:
            _check("hm_sketch_create_tol", lib().hm_sketch_create_tol(model._h, _ptr(omega), rank, oversample,
                                                                      float(rank_tol), _theta(theta0_full),
                                                                      C.byref(h)))
        self._h, self.model = h, model

    def ranks(self):
        nint = (1 << self.model.levels) - 1
        k = (C.c_int * nint)()
        kc = _I()
        _check("hm_sketch_ranks", lib().hm_sketch_ranks(self._h, k, C.byref(kc)))
        return np.frombuffer(k, dtype=np.int32).copy(), kc.value

    def close(self):
        if getattr(self, "_h", None):
            lib().hm_sketch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HMatrix:
    """K~(theta) with derivative matrices for the free parameters, factorisation and traces."""

    def __init__(self, sketch, free):
        idx = [PARAM_NAMES.index(f) if isinstance(f, str) else int(f) for f in free]
        arr = (C.c_int * max(1, len(idx)))(*idx)
        h = _P()
        _check("hm_H_create", lib().hm_H_create(sketch._h, len(idx), arr, C.byref(h)))
        self._h, self.sketch, self.p = h, sketch, len(idx)
        self.free_idx = tuple(idx)
        self.model = sketch.model

    def set_precision(self, precision):
        """'fp64' (default), 'mixed32' (FP32 MFMA panel products where the policy allows) or
        'mixedbf16' (as mixed32, with BF16 operands in the score and Fisher trace panels)."""
        self._eval_token = None   # the autograd function re-evaluates if needed
        code = {"fp64": 0, "mixed32": 1, "mixedbf16": 2}[precision]
        _check("hm_H_set_precision", lib().hm_H_set_precision(self._h, code))
        self.precision = precision

    def build(self, theta_full):
        self._eval_token = None   # the autograd function re-evaluates if needed
        _check("hm_build", lib().hm_build(self._h, _theta(theta_full)))

    def factor(self):
        _check("hm_factor", lib().hm_factor(self._h))

    def logdet(self):
        out = C.c_double()
        _check("hm_logdet", lib().hm_logdet(self._h, C.byref(out)))
        return out.value

    def solve(self, y):
        """K~^{-1} y for y of shape (n,) or (nrhs, n) (each row one right-hand side), grid order."""
        import torch
        x = torch.empty_like(y)
        nrhs = 1 if y.dim() == 1 else y.shape[0]
        _check("hm_solve", lib().hm_solve(self._h, _ptr(y), _ptr(x), nrhs, y.shape[-1]))
        return x

    def loglik_grad(self, y):
        self._eval_token = None   # the autograd function re-evaluates if needed
        ll = C.c_double()
        g = (C.c_double * max(1, self.p))()
        _check("hm_loglik_grad", lib().hm_loglik_grad(self._h, _ptr(y), C.byref(ll), g))
        return ll.value, np.array(g[:self.p])

    def fisher(self):
        f = (C.c_double * max(1, self.p * self.p))()
        _check("hm_fisher", lib().hm_fisher(self._h, f))
        return np.array(f[:self.p * self.p]).reshape(self.p, self.p)

    def iteration(self, theta_full, y):
        self._eval_token = None   # the autograd function re-evaluates if needed
        ll = C.c_double()
        g = (C.c_double * max(1, self.p))()
        f = (C.c_double * max(1, self.p * self.p))()
        _check("hm_iteration", lib().hm_iteration(self._h, _theta(theta_full), _ptr(y), C.byref(ll), g, f))
        return ll.value, np.array(g[:self.p]), np.array(f[:self.p * self.p]).reshape(self.p, self.p)

    def loglik_grad_adjoint(self, theta_full, y):
        """(L~, NLL gradient) by reverse mode through factorisation and construction."""
        self._eval_token = None   # the autograd function re-evaluates if needed
        ll = C.c_double()
        g = (C.c_double * max(1, self.p))()
        _check("hm_loglik_grad_adjoint",
               lib().hm_loglik_grad_adjoint(self._h, _theta(theta_full), _ptr(y), C.byref(ll), g))
        return ll.value, np.array(g[:self.p])

    def loglik(self, theta_full, y):
        """L~ alone: K~ built without derivative matrices, factored; keeps K~^{-1} y."""
        self._eval_token = None   # the autograd function re-evaluates if needed
        ll = C.c_double()
        _check("hm_loglik", lib().hm_loglik(self._h, _theta(theta_full), _ptr(y), C.byref(ll)))
        return ll.value

    def grad_reverse(self):
        """NLL gradient by the reverse sweep for the last construction and sample."""
        g = (C.c_double * max(1, self.p))()
        _check("hm_grad_reverse", lib().hm_grad_reverse(self._h, g))
        return np.array(g[:self.p])

    def stats(self):
        """Work counters and per-phase device milliseconds (hm_stats)."""
        st = _Stats()
        _check("hm_stats", lib().hm_stats(self._h, C.byref(st), C.sizeof(st)))
        return {name: getattr(st, name) for name, _ in _Stats._fields_}

    def stats_reset(self):
        _check("hm_stats_reset", lib().hm_stats_reset(self._h))

    def export(self, what):
        import torch
        m = self.model
        _, kc = self.sketch.ranks()
        if what in (0, 1, 2):
            shape = (m.levels * kc, m.rows)
        else:
            shape = (1 << m.levels, m.leaf, m.leaf)
        out = torch.empty(shape, dtype=torch.float64, device=m.device)
        _check("hm_export", lib().hm_export(self._h, what, _ptr(out)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().hm_H_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Stats(C.Structure):
    _fields_ = [(name, C.c_longlong) for name in (
        "kapply_calls", "kapply_columns", "kapply_deriv_columns", "builds", "deriv_builds", "factors",
        "loglik_evals", "grad_evals", "reverse_sweeps", "fisher_evals", "solve_rhs")] + \
        [(name, C.c_double) for name in ("ms_build", "ms_factor", "ms_loglik", "ms_fisher", "ms_reverse",
                                         "ms_solve")] + [("device_bytes", C.c_longlong)]


def place_fields(cost, nstreams):
    """Longest-first placement of fields on streams: fields in decreasing cost, each on
    the stream with the least cost so far (ties to the lower stream).  Returns (lanes,
    order): lanes[q] lists stream q's fields in enqueue order, and order interleaves the
    lanes (first field of every stream, then the second, ...), so that every stream has
    work at once."""
    nstreams = max(1, int(nstreams))
    load = [0.0] * nstreams
    lanes = [[] for _ in range(nstreams)]
    for f in sorted(range(len(cost)), key=lambda i: -cost[i]):
        q = min(range(nstreams), key=lambda j: load[j])
        load[q] += cost[f]
        lanes[q].append(f)
    order = []
    for r in range(max((len(x) for x in lanes), default=0)):
        for q in range(nstreams):
            if r < len(lanes[q]):
                order.append(lanes[q][r])
    return lanes, order


class Batch:
    """Independent fields iterated together (hm_iteration_batched).

    Every field is an HMatrix on a Model of its own.  The schedule decides how many
    streams run concurrently, which field goes on which stream and the enqueue order:
    fields are taken longest first (by measured or estimated cost) and placed on the
    least-loaded stream; the enqueue order interleaves the streams so that each one
    starts at once.  `tune` measures every field alone and times the batch under
    each candidate stream count, keeping the fastest.
    """

    def __init__(self, Hs):
        import torch
        self.Hs = list(Hs)
        models = [H.model for H in self.Hs]
        if len({id(m) for m in models}) != len(models):
            raise ValueError("every field needs a Model of its own (one stream per model)")
        self.device = models[0].device if models else torch.device("cuda", 0)
        # estimated cost per iteration ~ n kc^2 levels^2 (panel products over the tree)
        self.cost = []
        for H in self.Hs:
            _, kc = H.sketch.ranks()
            m = H.model
            self.cost.append(float(m.n) * kc * kc * m.levels * m.levels)
        self.order = list(range(len(self.Hs)))
        self.nstreams = 0
        self.streams = []
        self.set_schedule(1)

    def set_schedule(self, nstreams, cost=None):
        import torch
        cost = self.cost if cost is None else list(cost)
        nstreams = max(1, min(int(nstreams), max(1, len(self.Hs))))
        if nstreams != self.nstreams:
            self.streams = [torch.cuda.Stream(device=self.device) for _ in range(nstreams)]
            self.nstreams = nstreams
        lanes, order = place_fields(cost, nstreams)
        for q, lane in enumerate(lanes):
            for f in lane:
                self.Hs[f].model.set_stream(self.streams[q])
        self.order = order
        self.lanes = lanes
        return lanes

    def iteration(self, thetas, ys, want_grad=True, want_fim=True):
        """One iteration of every field: (loglik[nf], [grad_f], [fim_f]) in field order."""
        import torch
        nf = len(self.Hs)
        th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).reshape(nf, 4))
        order = self.order
        hs = (_P * max(1, nf))(*[self.Hs[f]._h for f in order])
        yp = (_P * max(1, nf))(*[_ptr(ys[f]) for f in order])
        tho = np.ascontiguousarray(th[order])
        ps = [self.Hs[f].p for f in order]
        ll = (C.c_double * max(1, nf))()
        g = (C.c_double * max(1, sum(ps))) () if want_grad else None
        fm = (C.c_double * max(1, sum(p * p for p in ps)))() if want_fim else None
        torch.cuda.current_stream(self.device).synchronize()   # samples written on the current stream
        for H in self.Hs:
            H._eval_token = None
        _check("hm_iteration_batched",
               lib().hm_iteration_batched(nf, hs, tho.ctypes.data_as(_D), yp, ll,
                                          g if want_grad else None, fm if want_fim else None))
        lls = np.zeros(nf)
        grads = [None] * nf
        fims = [None] * nf
        go = fo = 0
        for pos, f in enumerate(order):
            p = ps[pos]
            lls[f] = ll[pos]
            if want_grad:
                grads[f] = np.array(g[go:go + p])
            if want_fim:
                fims[f] = np.array(fm[fo:fo + p * p]).reshape(p, p)
            go += p
            fo += p * p
        return lls, grads, fims

    def tune_kernels(self):
        """Autotune the panel-kernel variants once per distinct field shape and copy the
        choice to every field of that shape; returns the per-shape reports."""
        reports, chosen = {}, {}
        for H in self.Hs:
            m = H.model
            _, kc = H.sketch.ranks()
            key = (m.dim, m.N, m.leaf, kc)
            if key not in chosen:
                reports[key] = m.autotune(kc)
                chosen[key] = m.tuning()
            else:
                m.tuning(*chosen[key])
        return reports

    def tune(self, thetas, ys, candidates=(1, 2, 4, 8), reps=1):
        """Pick the stream count by timing; returns the measurements."""
        import time
        import torch
        nf = len(self.Hs)
        th = np.asarray(thetas, dtype=np.float64).reshape(nf, 4)
        solo = []
        for f, H in enumerate(self.Hs):
            H.model.set_stream(None)
            H.iteration(th[f], ys[f])                      # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                H.iteration(th[f], ys[f])
            torch.cuda.synchronize()
            solo.append((time.perf_counter() - t0) / reps)
        self.nstreams = 0
        timings = {}
        for ns in candidates:
            if ns > max(1, nf):
                continue
            self.set_schedule(ns, cost=solo)
            self.iteration(th, ys)                          # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                self.iteration(th, ys)
            torch.cuda.synchronize()
            timings[ns] = (time.perf_counter() - t0) / reps
        best = min(timings, key=timings.get)
        self.set_schedule(best, cost=solo)
        self.cost = solo
        return dict(solo_s=solo, sequential_s=float(sum(solo)), batch_s=timings, best_streams=best)


def _make_loglik_function():
    import torch

    class HLogLik(torch.autograd.Function):
        """L~(theta, y) as a differentiable torch function; backward is the adjoint.

        apply(H, theta, y, theta_full):
          H          HMatrix (its sketch fixes the test matrices, Sec. 3.3)
          theta      float64 CPU tensor of H's p free parameters, in H's order
          y          float64 CUDA tensor (n,), grid order
          theta_full the 4 parameters (kappa, alpha, tau2, sigma2) the others are taken from
        Returns a 0-d float64 CPU tensor.  forward builds and factors K~ only and
        evaluates L~ (hm_loglik); backward runs the reverse sweep (hm_grad_reverse) for
        d/dtheta and one solve for d/dy = -K~^{-1} y.  If H was evaluated elsewhere in
        between, backward first re-evaluates L~ at the saved point.
        """

        @staticmethod
        def forward(ctx, H, theta, y, theta_full):
            full = [float(t) for t in theta_full]
            th = theta.detach().cpu().double().reshape(-1)
            if th.numel() != H.p:
                raise ValueError(f"theta has {th.numel()} entries, H has {H.p} free parameters")
            for q, k in enumerate(H.free_idx):
                full[k] = float(th[q])
            yd = y.detach()
            ll = H.loglik(full, yd)
            ctx.H, ctx.full, ctx.y = H, full, yd
            ctx.token = H._eval_token = object()
            return torch.tensor(ll, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gout):
            H = ctx.H
            if getattr(H, "_eval_token", None) is not ctx.token:
                H.loglik(ctx.full, ctx.y)
                H._eval_token = ctx.token
            gt = gy = None
            if ctx.needs_input_grad[1]:
                gt = gout.detach().cpu().double() * torch.from_numpy(-H.grad_reverse())
            if ctx.needs_input_grad[2]:
                gy = -gout.detach().to(ctx.y.device, torch.float64) * H.solve(ctx.y)
            return None, gt, gy, None

    return HLogLik


HLogLik = _make_loglik_function()
