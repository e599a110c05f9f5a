"""irlsu: IRLS + PCG weighted-L1 phase unwrapping on AMD MI355X (gfx950).

Thin Python binding of the C ABI declared in ``include/irlsu.h``: argument
marshalling only.  Every step of the computation runs in the HIP kernels of
``lib/libirlsu.so``; PyTorch provides device memory and the stream.  There
is no CPU fallback: if the library is missing, loading fails loudly.

Method: Dubois-Taine, Akiki, d'Aspremont, "Iteratively Reweighted Least
Squares for Phase Unwrapping", arXiv 2401.09961 (Section 2 problem,
Algorithm 1 IRLS, Algorithm 2 PCG, Section 3.3 preconditioner).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

__all__ = [
    "IrlsuError", "Params", "Stats", "Plan", "unwrap", "load_library",
    "library_path", "PRECISIONS", "DECLARED_SYMBOLS", "UnwrapFn", "Batch",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "lib", "libirlsu.so")

PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
IRLSU_MAX_IRLS = 256

# every function declared in include/irlsu.h
DECLARED_SYMBOLS = (
    "irlsu_status_string", "irlsu_params_default", "irlsu_plan_create",
    "irlsu_plan_create_ex", "irlsu_plan_destroy", "irlsu_plan_info", "irlsu_workspace_bytes",
    "irlsu_unwrap", "irlsu_adjoint", "irlsu_adjoint_implicit", "irlsu_setup", "irlsu_weights",
    "irlsu_operator", "irlsu_precond", "irlsu_precond_timed", "irlsu_profile_arm",
    "irlsu_profile_result", "irlsu_round_congruent", "irlsu_augmented_workspace_bytes",
    "irlsu_unwrap_augmented", "irlsu_batch_create", "irlsu_batch_destroy",
    "irlsu_batch_workspace_bytes", "irlsu_unwrap_batched", "irlsu_pcg",
    "irlsu_test_fail_alloc", "irlsu_operator_noalloc", "irlsu_stream_probe",
    "irlsu_plan_autotune", "irlsu_plan_set_tune", "irlsu_plan_get_tune", "irlsu_batch_autotune",
)

STATUS = {
    0: "OK", 1: "NOT_CONVERGED", -1: "ERR_INVALID_ARG", -2: "ERR_SHAPE",
    -3: "ERR_NONFINITE", -4: "ERR_BAD_WEIGHTS", -5: "ERR_BREAKDOWN",
    -6: "ERR_HIP", -7: "ERR_OOM", -8: "ERR_UNSUPPORTED", -9: "ERR_WORKSPACE",
}


class IrlsuError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__(f"irlsu status {code} ({self.name}) {msg}".strip())


class Params(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double), ("pcg_rtol", ctypes.c_double),
        ("l1_target", ctypes.c_double), ("irls_iters", ctypes.c_int32),
        ("pcg_max", ctypes.c_int32), ("true_res_every", ctypes.c_int32),
        ("poll_every", ctypes.c_int32), ("flexible", ctypes.c_int32),
        ("cg_schedule", ctypes.c_int32), ("cg_m0", ctypes.c_int32),
        ("sd_guard", ctypes.c_int32), ("cg_eps_tol", ctypes.c_double),
        ("cg_alpha", ctypes.c_double), ("graph", ctypes.c_int32),
        ("reserved_", ctypes.c_int32),
    ]


CG_SCHEDULES = {"fixed": 0, "adaptive": 1}
# Sufficient-decrease guard of the augmented form (Theorem 3)
SD_GUARDS = {"off": 0, "check": 1, "candidate_only": 2}


class IterStats(ctypes.Structure):
    _fields_ = [("L1", ctypes.c_double), ("H", ctypes.c_double),
                ("relres", ctypes.c_double), ("pcg_iters", ctypes.c_int32),
                ("status", ctypes.c_int32), ("delta", ctypes.c_double),
                ("pcg_cap", ctypes.c_int32), ("guard", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("irls_done", ctypes.c_int32), ("pcg_total", ctypes.c_int32),
        ("target_hit", ctypes.c_int32), ("status", ctypes.c_int32),
        ("L1_final", ctypes.c_double), ("H_final", ctypes.c_double),
        ("schedule_stop", ctypes.c_int32), ("reserved_", ctypes.c_int32),
        ("iter", IterStats * IRLSU_MAX_IRLS),
    ]

    def to_dict(self):
        n = self.irls_done
        hist = [dict(k=k, L1=self.iter[k].L1, H=self.iter[k].H,
                     relres=self.iter[k].relres, iters=self.iter[k].pcg_iters,
                     status=self.iter[k].status, delta=self.iter[k].delta,
                     cap=self.iter[k].pcg_cap, guard=self.iter[k].guard)
                for k in range(min(n + 1, IRLSU_MAX_IRLS))]
        return dict(irls_done=n, pcg_total=self.pcg_total,
                    target_hit=bool(self.target_hit), status=self.status,
                    L1_final=self.L1_final, H_final=self.H_final,
                    schedule_stop=bool(self.schedule_stop), history=hist)


class Tile(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("w", ctypes.c_void_p),
                ("Cv", ctypes.c_void_p), ("ldcv", ctypes.c_int64),
                ("Ch", ctypes.c_void_p), ("ldch", ctypes.c_int64),
                ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64)]


class Tune(ctypes.Structure):
    _fields_ = [("stencil_rows", ctypes.c_int32), ("update_blocks", ctypes.c_int32),
                ("small_tiles", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("stencil_us", ctypes.c_double), ("update_us", ctypes.c_double),
                ("precond_us", ctypes.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("M", ctypes.c_int64),
                ("Np", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("elem_bytes", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_size_t), ("plan_bytes", ctypes.c_size_t),
                ("folded", ctypes.c_int32), ("form", ctypes.c_int32)]


# form of the preconditioner products (irlsu_plan_create_ex)
PLAN_FORMS = {"auto": 0, "dense": 1, "folded": 2, "fast": 3}
IRLSU_MAX_LAUNCHES = 32
LAUNCH_KINDS = {0: "product", 1: "rows_dct2", 2: "transpose", 3: "cols", 4: "rows_dct3",
                5: "butterfly", 6: "dots", 7: "prologue", 8: "partials", 9: "stencil",
                10: "axpy", 11: "residual", 12: "update_dct2", 13: "alpha"}


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libirlsu.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I64, I32, D, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    sig = {
        "irlsu_status_string": (ctypes.c_char_p, [I32]),
        "irlsu_params_default": (I32, [ctypes.POINTER(Params), I32]),
        "irlsu_plan_create": (I32, [ctypes.POINTER(P), I64, I64, I32, P]),
        "irlsu_plan_create_ex": (I32, [ctypes.POINTER(P), I64, I64, I32, I32, P]),
        "irlsu_plan_destroy": (I32, [P]),
        "irlsu_plan_info": (I32, [P, ctypes.POINTER(PlanDesc)]),
        "irlsu_workspace_bytes": (SZ, [P]),
        "irlsu_unwrap": (I32, [P, P, I64, P, P, I64, P, I64, P, ctypes.POINTER(Params),
                               P, I64, P, SZ, ctypes.POINTER(Stats), P]),
        "irlsu_adjoint": (I32, [P, P, I64, ctypes.POINTER(Params), P, I64, P, I64, P, I64,
                                P, SZ, ctypes.POINTER(Stats), P]),
        "irlsu_adjoint_implicit": (I32, [P, P, I64, ctypes.POINTER(Params), P, I64, P, I64, P,
                                         I64, P, SZ, ctypes.POINTER(Stats), P]),
        "irlsu_setup": (I32, [P, P, I64, P, P, I64, P, I64, P, P, P, P, P, P]),
        "irlsu_batch_create": (I32, [ctypes.POINTER(P), ctypes.POINTER(I64), I32, I32, P]),
        "irlsu_batch_destroy": (I32, [P]),
        "irlsu_batch_workspace_bytes": (SZ, [P]),
        "irlsu_unwrap_batched": (I32, [P, ctypes.POINTER(Tile), ctypes.POINTER(Params), P, SZ,
                                       ctypes.POINTER(Stats), P]),
        "irlsu_weights": (I32, [P, D, P, P, P, P, P, P, P, P, P, P, SZ, P]),
        "irlsu_operator": (I32, [P, P, P, P, P, P, P, SZ, P]),
        "irlsu_operator_noalloc": (I32, [P, P, P, P, P, P, P]),
        "irlsu_stream_probe": (I32, [I32, P, P, P, P, SZ, I32, I32, ctypes.POINTER(D), P]),
        "irlsu_plan_autotune": (I32, [P, ctypes.c_char_p, ctypes.POINTER(Tune), P, SZ, P]),
        "irlsu_plan_set_tune": (I32, [P, ctypes.POINTER(Tune)]),
        "irlsu_plan_get_tune": (I32, [P, ctypes.POINTER(Tune)]),
        "irlsu_batch_autotune": (I32, [P, ctypes.c_char_p, P, SZ, P]),
        "irlsu_precond": (I32, [P, P, P, P, P, SZ, P]),
        "irlsu_pcg": (I32, [P, P, P, P, P, ctypes.POINTER(Params), ctypes.POINTER(I32),
                            ctypes.POINTER(D), P, SZ, P]),
        "irlsu_test_fail_alloc": (None, [I32]),
        "irlsu_precond_timed": (I32, [P, P, P, P, SZ, I32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(I32), ctypes.POINTER(I32), P]),
        "irlsu_profile_arm": (I32, [P, I32, I32]),
        "irlsu_round_congruent": (I32, [P, P, I64, P, I64, P, I64, P, SZ, P]),
        "irlsu_augmented_workspace_bytes": (SZ, [P]),
        "irlsu_unwrap_augmented": (I32, [P, P, I64, P, P, I64, P, I64, P, D, D, P, I64, P, SZ,
                                         P, P]),
        "irlsu_profile_result": (I32, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I32),
                                       ctypes.POINTER(I32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code, what=""):
    if code < 0:
        raise IrlsuError(code, what)
    return code


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


PROBES = {"copy": 0, "read": 1, "3r1w": 2}


def stream_probe(kind, nbytes=256 << 20, grids=(256, 512, 1024, 2048), reps=10):
    """Measured HBM ceiling of one streaming mix (the library's own kernel):
    {grid: GB/s of algorithmic bytes} and the best, for 'copy' (1 read +
    1 write), 'read' and '3r1w' (3 reads + 1 write) over nbytes per array."""
    import torch
    lib = load_library()
    narr = {"copy": 2, "read": 1, "3r1w": 4}[kind]
    bufs = [torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
            for _ in range(narr)]
    a = bufs[0]
    b = bufs[1] if kind == "3r1w" else None
    c = bufs[2] if kind == "3r1w" else None
    d = bufs[-1] if kind != "read" else None
    moved = {"copy": 2, "read": 1, "3r1w": 4}[kind] * nbytes
    out = {}
    for g in grids:
        ms = ctypes.c_double()
        _check(lib.irlsu_stream_probe(PROBES[kind], _ptr(a), _ptr(b), _ptr(c), _ptr(d), nbytes,
                                      int(g), int(reps), ctypes.byref(ms), _stream()),
               "stream_probe")
        out[g] = moved / (ms.value * 1e-3) / 1e9
    del bufs
    return {"GBps_by_grid": {str(g): round(v, 1) for g, v in out.items()},
            "best_GBps": round(max(out.values()), 1), "bytes_per_array": nbytes}


def default_params(precision="f32") -> Params:
    p = Params()
    _check(load_library().irlsu_params_default(ctypes.byref(p), PRECISIONS[precision]))
    return p


class Plan:
    """A plan for N x M images at one precision, bound to a torch device.

    Owns the device basis tables (through the library) and a workspace
    tensor allocated by torch.
    """

    def __init__(self, N: int, M: int, precision: str = "f32", device=None, form: str = "auto"):
        import torch
        self.lib = load_library()
        self.precision = precision
        self.device = (torch.device("cuda", torch.cuda.current_device()) if device is None
                       else torch.device(device))
        with torch.cuda.device(self.device):
            h = ctypes.c_void_p()
            _check(self.lib.irlsu_plan_create_ex(ctypes.byref(h), int(N), int(M),
                                                 PRECISIONS[precision], PLAN_FORMS[form],
                                                 _stream()), "plan_create")
            self.handle = h
            d = PlanDesc()
            _check(self.lib.irlsu_plan_info(h, ctypes.byref(d)))
            self.desc = d
            self.workspace = torch.empty(int(d.workspace_bytes), dtype=torch.uint8, device=self.device)
        self.N, self.M, self.Np, self.ld = d.N, d.M, d.Np, d.ld
        self.folded = bool(d.folded)
        self.form = {v: k for k, v in PLAN_FORMS.items()}[d.form]
        self.dtype = torch.float64 if d.elem_bytes == 8 else torch.float32

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.irlsu_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    # ---- layout helpers (internal layout: Np x ld, zero padded) --------
    def to_internal(self, A, rows=None, cols=None, dtype=None):
        import torch
        out = torch.zeros((self.Np, self.ld), dtype=dtype or self.dtype, device=self.device)
        r = A.shape[0] if rows is None else rows
        c = A.shape[1] if cols is None else cols
        out[:r, :c] = A[:r, :c].to(out.dtype)
        return out

    def from_internal(self, A, rows=None, cols=None):
        return A[: (rows or self.N), : (cols or self.M)]

    # ---- whole path -----------------------------------------------------
    def new_workspace(self):
        import torch
        return torch.empty(int(self.desc.workspace_bytes), dtype=torch.uint8, device=self.device)

    def unwrap(self, X, weights=None, *, Cv=None, Ch=None, U0=None, params: Optional[Params] = None,
               out=None, stats: bool = False, workspace=None):
        import torch
        ws = self.workspace if workspace is None else workspace
        X = _mat(X, self.dtype)
        assert X.shape == (self.N, self.M), "X shape does not match the plan"
        w = None if weights is None else _mat(weights, self.dtype, like=X)
        Cv_t = None if Cv is None else _mat(Cv, self.dtype)
        Ch_t = None if Ch is None else _mat(Ch, self.dtype)
        U = out if out is not None else torch.empty((self.N, self.M), dtype=self.dtype, device=self.device)
        U0_t = None if U0 is None else _mat(U0, self.dtype, like=U)
        st = Stats() if stats else None
        code = self.lib.irlsu_unwrap(
            self.handle, _ptr(X), X.stride(0), _ptr(w),
            _ptr(Cv_t), Cv_t.stride(0) if Cv_t is not None else 0,
            _ptr(Ch_t), Ch_t.stride(0) if Ch_t is not None else 0,
            _ptr(U0_t), ctypes.byref(params) if params is not None else None,
            _ptr(U), U.stride(0), _ptr(ws), ws.numel(),
            ctypes.byref(st) if st is not None else None, _stream())
        _check(code, "unwrap")
        if stats:
            d = st.to_dict()
            d["code"] = code
            return U, d
        return U

    def adjoint(self, gU, *, params: Optional[Params] = None, workspace=None, stats: bool = False,
                implicit: bool = False):
        """Gradients (gCv, gCh, gX) of a loss with dL/dU = gU through the
        frozen-weight map at the U of the last unwrap that used `workspace`
        (implicit=True: through the Huber minimiser itself, the full implicit
        derivative)."""
        import torch
        ws = self.workspace if workspace is None else workspace
        g = _mat(gU, self.dtype)
        gCv = torch.empty((self.N - 1, self.M), dtype=self.dtype, device=self.device)
        gCh = torch.empty((self.N, self.M - 1), dtype=self.dtype, device=self.device)
        gX = torch.empty((self.N, self.M), dtype=self.dtype, device=self.device)
        st = Stats() if stats else None
        fn = self.lib.irlsu_adjoint_implicit if implicit else self.lib.irlsu_adjoint
        code = fn(
            self.handle, _ptr(g), g.stride(0), ctypes.byref(params) if params is not None else None,
            _ptr(gCv), gCv.stride(0), _ptr(gCh), gCh.stride(0), _ptr(gX), gX.stride(0),
            _ptr(ws), ws.numel(), ctypes.byref(st) if st is not None else None, _stream())
        _check(code, "adjoint")
        if stats:
            d = st.to_dict()
            d["code"] = code
            return gCv, gCh, gX, d
        return gCv, gCh, gX

    # ---- step-level entry points -----------------------------------------
    def setup(self, X, weights=None, Cv=None, Ch=None):
        import torch
        X = _mat(X, self.dtype)
        w = None if weights is None else _mat(weights, self.dtype, like=X)
        Cv_t = None if Cv is None else _mat(Cv, self.dtype)
        Ch_t = None if Ch is None else _mat(Ch, self.dtype)
        outs = [torch.empty((self.Np, self.ld), dtype=self.dtype, device=self.device) for _ in range(4)]
        flags = torch.zeros(1, dtype=torch.int32, device=self.device)
        _check(self.lib.irlsu_setup(
            self.handle, _ptr(X), X.stride(0), _ptr(w),
            _ptr(Cv_t), Cv_t.stride(0) if Cv_t is not None else 0,
            _ptr(Ch_t), Ch_t.stride(0) if Ch_t is not None else 0,
            *[_ptr(o) for o in outs], _ptr(flags), _stream()), "setup")
        return (*outs, flags)

    def weights(self, eps, U, Gv, Gh, Cv, Ch):
        import torch
        assert U.dtype == torch.float64 and U.shape == (self.Np, self.ld)
        outs = [torch.empty((self.Np, self.ld), dtype=self.dtype, device=self.device) for _ in range(3)]
        obj = torch.zeros(3, dtype=torch.float64, device=self.device)
        _check(self.lib.irlsu_weights(
            self.handle, float(eps), _ptr(U), _ptr(Gv), _ptr(Gh), _ptr(Cv), _ptr(Ch),
            *[_ptr(o) for o in outs], _ptr(obj), _ptr(self.workspace), self.workspace.numel(),
            _stream()), "weights")
        return (*outs, obj)

    def operator(self, Ov, Oh, p):
        import torch
        q = torch.empty_like(p)
        pq = torch.zeros(1, dtype=torch.float64, device=self.device)
        _check(self.lib.irlsu_operator(self.handle, _ptr(Ov), _ptr(Oh), _ptr(p), _ptr(q), _ptr(pq),
                                       _ptr(self.workspace), self.workspace.numel(), _stream()),
               "operator")
        return q, pq

    def operator_noalloc(self, Ov, Oh, p, q=None, pq=None):
        """irlsu_operator without workspace (the library's scratch holds the
        partial sums); q and pq may be passed in so that nothing is
        allocated by this call."""
        import torch
        q = torch.empty_like(p) if q is None else q
        pq = torch.zeros(1, dtype=torch.float64, device=self.device) if pq is None else pq
        _check(self.lib.irlsu_operator_noalloc(self.handle, _ptr(Ov), _ptr(Oh), _ptr(p), _ptr(q),
                                               _ptr(pq), _stream()), "operator_noalloc")
        return q, pq

    def precond(self, r):
        import torch
        z = torch.empty_like(r)
        rz = torch.zeros(1, dtype=torch.float64, device=self.device)
        _check(self.lib.irlsu_precond(self.handle, _ptr(r), _ptr(z), _ptr(rz),
                                      _ptr(self.workspace), self.workspace.numel(), _stream()),
               "precond")
        return z, rz

    def autotune(self, cache_path=None):
        """Measure and apply the fastest launch shapes (cached in the JSON
        file cache_path when given); returns the choice as a dict."""
        t = Tune()
        path = None if cache_path is None else os.fsencode(str(cache_path))
        _check(self.lib.irlsu_plan_autotune(self.handle, path, ctypes.byref(t), _ptr(self.workspace),
                                            self.workspace.numel(), _stream()), "plan_autotune")
        return t.to_dict()

    def set_tune(self, stencil_rows=0, update_blocks=0, small_tiles=0):
        t = Tune(stencil_rows, update_blocks, small_tiles, 0, 0.0, 0.0, 0.0)
        _check(self.lib.irlsu_plan_set_tune(self.handle, ctypes.byref(t)), "plan_set_tune")

    def get_tune(self):
        t = Tune()
        _check(self.lib.irlsu_plan_get_tune(self.handle, ctypes.byref(t)), "plan_get_tune")
        return t.to_dict()

    def pcg(self, Ov, Oh, b, x=None, *, params: Optional[Params] = None):
        """Algorithm 2 on D^T Omega D x = b (internal layout; x FP64, warm
        start in / solution out).  Returns (x, status code, iterations,
        relative residual); negative codes raise."""
        import torch
        if x is None:
            x = torch.zeros((self.Np, self.ld), dtype=torch.float64, device=self.device)
        assert x.dtype == torch.float64 and x.shape == (self.Np, self.ld) and x.is_contiguous()
        for t in (Ov, Oh, b):
            assert t.dtype == self.dtype and t.shape == (self.Np, self.ld) and t.is_contiguous()
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        code = self.lib.irlsu_pcg(self.handle, _ptr(Ov), _ptr(Oh), _ptr(b), _ptr(x),
                                  ctypes.byref(params) if params is not None else None,
                                  ctypes.byref(it), ctypes.byref(rel), _ptr(self.workspace),
                                  self.workspace.numel(), _stream())
        _check(code, "pcg")
        return x, code, it.value, rel.value

    def unwrap_augmented(self, X, weights=None, *, tau=1e-2, delta=1e-6,
                         params: Optional[Params] = None, stats: bool = False):
        """The paper's augmented form (U, V^v, V^h) with tau, delta: returns
        U (and the stats dict; history H holds F_delta)."""
        import torch
        X = _mat(X, self.dtype)
        w = None if weights is None else _mat(weights, self.dtype, like=X)
        nbytes = self.lib.irlsu_augmented_workspace_bytes(self.handle)
        ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        U = torch.empty((self.N, self.M), dtype=self.dtype, device=self.device)
        st = Stats() if stats else None
        code = self.lib.irlsu_unwrap_augmented(
            self.handle, _ptr(X), X.stride(0), _ptr(w), None, 0, None, 0,
            ctypes.byref(params) if params is not None else None, float(tau), float(delta),
            _ptr(U), U.stride(0), _ptr(ws), ws.numel(),
            ctypes.byref(st) if st is not None else None, _stream())
        _check(code, "unwrap_augmented")
        if stats:
            d = st.to_dict()
            d["code"] = code
            return U, d
        return U

    def round_congruent(self, X, U, out=None):
        """X + 2 pi rint((U + c - X) / 2 pi), c = arg sum exp(i (X - U)):
        U made 2 pi-congruent to X (the rounded output of Section 4)."""
        import torch
        X = _mat(X, self.dtype)
        U = _mat(U, self.dtype)
        out = torch.empty_like(U) if out is None else out
        _check(self.lib.irlsu_round_congruent(self.handle, _ptr(X), X.stride(0), _ptr(U),
                                              U.stride(0), _ptr(out), out.stride(0),
                                              _ptr(self.workspace), self.workspace.numel(),
                                              _stream()), "round_congruent")
        return out

    def profile_arm(self, irls_k, pcg_l):
        """Record per-launch events for PCG iteration pcg_l of IRLS
        iteration irls_k during the next unwrap (negative: disarm)."""
        _check(self.lib.irlsu_profile_arm(self.handle, int(irls_k), int(pcg_l)), "profile_arm")

    def profile_result(self):
        """[(kind, ms)] of the launches recorded for the armed iteration."""
        ms = (ctypes.c_double * IRLSU_MAX_LAUNCHES)()
        kind = (ctypes.c_int32 * IRLSU_MAX_LAUNCHES)()
        n = ctypes.c_int32()
        _check(self.lib.irlsu_profile_result(self.handle, ms, kind, ctypes.byref(n)),
               "profile_result")
        return [(LAUNCH_KINDS[kind[i]], ms[i]) for i in range(n.value)]

    def precond_timed(self, r, reps=5):
        """Per-launch HIP-event timing of the preconditioner: a list of
        (kind, mean ms) for the launches of one application, in order."""
        ms = (ctypes.c_double * IRLSU_MAX_LAUNCHES)()
        kind = (ctypes.c_int32 * IRLSU_MAX_LAUNCHES)()
        n = ctypes.c_int32()
        z = r.new_empty(r.shape)
        _check(self.lib.irlsu_precond_timed(self.handle, _ptr(r), _ptr(z), _ptr(self.workspace),
                                            self.workspace.numel(), int(reps), ms, kind,
                                            ctypes.byref(n), _stream()), "precond_timed")
        return [(LAUNCH_KINDS[kind[i]], ms[i]) for i in range(n.value)]


class Batch:
    """Uneven tiles unwrapped together: one grouped launch per PCG phase."""

    def __init__(self, shapes, precision: str = "bf16", device=None):
        import torch
        self.lib = load_library()
        self.shapes = [(int(n), int(m)) for n, m in shapes]
        self.precision = precision
        self.device = (torch.device("cuda", torch.cuda.current_device()) if device is None
                       else torch.device(device))
        flat = (ctypes.c_int64 * (2 * len(self.shapes)))(*[v for nm in self.shapes for v in nm])
        with torch.cuda.device(self.device):
            h = ctypes.c_void_p()
            _check(self.lib.irlsu_batch_create(ctypes.byref(h), flat, len(self.shapes),
                                               PRECISIONS[precision], _stream()), "batch_create")
            self.handle = h
            nbytes = self.lib.irlsu_batch_workspace_bytes(h)
            self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.irlsu_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, cache_path=None):
        """Measured operator band heights per tile shape (cached in the JSON
        file cache_path when given)."""
        path = None if cache_path is None else os.fsencode(str(cache_path))
        _check(self.lib.irlsu_batch_autotune(self.handle, path, _ptr(self.workspace),
                                             self.workspace.numel(), _stream()), "batch_autotune")

    def unwrap(self, Xs, weights=None, *, params: Optional[Params] = None, stats: bool = False):
        import torch
        n = len(self.shapes)
        keep, outs = [], []
        tiles = (Tile * n)()
        for t, (N, M) in enumerate(self.shapes):
            X = _mat(Xs[t], torch.float32)
            w = None if weights is None or weights[t] is None else _mat(weights[t], torch.float32, like=X)
            U = torch.empty((N, M), dtype=torch.float32, device=self.device)
            keep += [X, w]
            outs.append(U)
            tiles[t] = Tile(X.data_ptr(), X.stride(0), None if w is None else w.data_ptr(),
                            None, 0, None, 0, U.data_ptr(), U.stride(0))
        st = (Stats * n)() if stats else None
        code = self.lib.irlsu_unwrap_batched(self.handle, tiles, ctypes.byref(params) if params else None,
                                             _ptr(self.workspace), self.workspace.numel(), st, _stream())
        _check(code, "unwrap_batched")
        if stats:
            return outs, [st[t].to_dict() for t in range(n)]
        return outs


def _mat(A, dtype, like=None):
    import torch
    if not isinstance(A, torch.Tensor):
        A = torch.as_tensor(A)
    dev = like.device if like is not None else (A.device if A.is_cuda else torch.device("cuda"))
    A = A.to(device=dev, dtype=dtype)
    if A.dim() != 2 or A.stride(1) != 1:
        A = A.contiguous()
    if like is not None and A.stride(0) != like.stride(0):
        A = A.contiguous()
        assert A.stride(0) == like.stride(0), "weights must share the stride of X"
    return A


def unwrap(X, weights=None, *, Cv=None, Ch=None, precision: str = "f32", params=None,
           stats=False, plan: Optional[Plan] = None):
    """Unwrap a wrapped phase image on the current GPU.

    X: N x M tensor (float64 for precision "f64", float32 otherwise);
    weights: optional per-pixel weights; Cv, Ch: optional per-edge weights
    ((N-1) x M and N x (M-1)).  Returns the mean-zero unwrapped U (and a stats
    dict with ``stats=True``).
    """
    import torch
    if not isinstance(X, torch.Tensor):
        X = torch.as_tensor(X)
    N, M = X.shape
    own = plan is None
    if own:
        plan = Plan(N, M, precision)
    try:
        return plan.unwrap(X, weights, Cv=Cv, Ch=Ch, params=params, stats=stats)
    finally:
        if own:
            plan.close()


def _autograd_function():
    import torch

    class UnwrapFn(torch.autograd.Function):
        """U = unwrap(X, Cv, Ch) with a hand-written adjoint (X, Cv, Ch may
        carry a leading batch dimension: one unwrap and one adjoint per grid).

        forward runs the IRLS + PCG path on a workspace of its own; backward
        runs one extra PCG solve on the converged system with the weights
        frozen (irlsu_adjoint), or through the Huber minimiser itself when
        implicit is true (irlsu_adjoint_implicit), and returns gradients for
        X and the per-edge weights Cv, Ch.
        """

        @staticmethod
        def forward(ctx, X, Cv, Ch, plan, params=None, adj_params=None, implicit=False):
            # a leading batch dimension runs one unwrap per grid, each on a
            # workspace of its own that its backward reuses
            batched = X.dim() == 3
            Xs = list(X) if batched else [X]
            Cvs = list(Cv) if batched else [Cv]
            Chs = list(Ch) if batched else [Ch]
            wss, Us = [], []
            for x, cv, ch in zip(Xs, Cvs, Chs):
                ws = plan.new_workspace()
                Us.append(plan.unwrap(x, Cv=cv, Ch=ch, params=params, workspace=ws))
                wss.append(ws)
            ctx.plan, ctx.wss, ctx.batched = plan, wss, batched
            ctx.adj_params = adj_params if adj_params is not None else params
            ctx.implicit = bool(implicit)
            return torch.stack(Us) if batched else Us[0]

        @staticmethod
        def backward(ctx, gU):
            gs = list(gU) if ctx.batched else [gU]
            outs = [ctx.plan.adjoint(g.contiguous(), params=ctx.adj_params, workspace=ws,
                                     implicit=ctx.implicit) for g, ws in zip(gs, ctx.wss)]
            ctx.wss = None
            if ctx.batched:
                gCv, gCh, gX = (torch.stack([o[i] for o in outs]) for i in range(3))
            else:
                gCv, gCh, gX = outs[0]
            return gX, gCv, gCh, None, None, None, None

    return UnwrapFn


class _LazyFn:
    _fn = None

    def apply(self, *args):
        if _LazyFn._fn is None:
            _LazyFn._fn = _autograd_function()
        return _LazyFn._fn.apply(*args)


UnwrapFn = _LazyFn()
