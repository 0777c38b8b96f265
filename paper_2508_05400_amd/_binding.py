"""ctypes binding of librks.so with the C-ABI's names (argument marshalling only).

Host arrays are NumPy arrays; device buffers are any object with a
``data_ptr()`` method (e.g. a torch CUDA tensor) or a raw integer address.
Every computation runs in the HIP library: if it is missing, loading fails
with an error instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librks.so")

RKS_OK, RKS_ENOTCONV = 0, 1
RKS_EINVAL, RKS_ENOMEM, RKS_EHIP, RKS_ENAN, RKS_ESTATE, RKS_EBREAKDOWN, RKS_EDENSE = -1, -2, -3, -4, -5, -6, -7
WHICH = {"LM": 0, "SM": 1, "LR": 2, "SR": 3}
SKETCH = {"gauss": 0, "sparse": 1}
PRECISION = {"fp64": 0, "fp32": 1, "v32": 1, "bf16": 2, "vbf16": 2, "fp32+fx16": 3, "v32_fx16": 3}
SPMV_LAYOUT = {"auto": 0, "rows": 1, "column_blocks": 2, "sliced": 3}
METHOD = {"rks": 0, "ks_cgs2": 1}
A_VALUES = {"auto": 0, "fp64": 1}


class RksCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class RksOpts(ctypes.Structure):
    _fields_ = [("sketch_kind", ctypes.c_int32), ("zeta", ctypes.c_int32),
                ("sketch_seed", ctypes.c_uint64), ("start_seed", ctypes.c_uint64),
                ("precision", ctypes.c_int32), ("max_restarts", ctypes.c_int32),
                ("lock", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("whiten_tol", ctypes.c_double), ("stream", ctypes.c_void_p),
                ("resid_tol", ctypes.c_double), ("refine", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("spmv_layout", ctypes.c_int32),
                ("method", ctypes.c_int32), ("keep", ctypes.c_int32), ("graphs", ctypes.c_int32),
                ("stall_restarts", ctypes.c_int32), ("a_values", ctypes.c_int32)]


class RksStats(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("matvecs", ctypes.c_int64), ("locked", ctypes.c_int32), ("keff", ctypes.c_int32),
                ("whitenings", ctypes.c_int32), ("breakdowns", ctypes.c_int32), ("dense_fail", ctypes.c_int32),
                ("max_est", ctypes.c_double), ("stop_reason", ctypes.c_int32),
                ("resid_checks", ctypes.c_int32), ("max_resid", ctypes.c_double),
                ("restarts_lo", ctypes.c_int32), ("refined", ctypes.c_int32), ("t_lo", ctypes.c_double),
                ("max_resid_lo", ctypes.c_double),
                ("t_total", ctypes.c_double), ("t_host", ctypes.c_double),
                ("t_spmv", ctypes.c_double), ("t_reduce", ctypes.c_double), ("t_ls", ctypes.c_double),
                ("t_update", ctypes.c_double), ("t_rotate", ctypes.c_double),
                ("n_spmv", ctypes.c_int64), ("n_update", ctypes.c_int64), ("n_rotate", ctypes.c_int64),
                ("bytes_spmv", ctypes.c_double), ("bytes_update", ctypes.c_double),
                ("bytes_rotate", ctypes.c_double), ("n_timed_steps", ctypes.c_int64),
                ("n_timed_rotate", ctypes.c_int64), ("bytes_timed_spmv", ctypes.c_double),
                ("bytes_timed_update", ctypes.c_double), ("bytes_timed_rotate", ctypes.c_double),
                ("n_timed_whole", ctypes.c_int64), ("t_step", ctypes.c_double),
                ("bytes_timed_whole", ctypes.c_double), ("spmv_layout", ctypes.c_int32),
                ("keep", ctypes.c_int32), ("hist_est", ctypes.c_double * 512), ("a_distinct", ctypes.c_int32)]

    def as_dict(self) -> dict:
        out = {f: getattr(self, f) for f, _ in self._fields_ if f != "hist_est"}
        out["hist_est"] = list(self.hist_est[:min(self.restarts + 1, 512)])
        return out


_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "rks_opts_default": (None, [ctypes.POINTER(RksOpts)]),
    "rks_create": (ctypes.c_int, [ctypes.POINTER(RksCsr), _I32, _I32, _I32, _I32, _D,
                                  ctypes.POINTER(RksOpts), ctypes.POINTER(ctypes.c_void_p)]),
    "rks_solve": (ctypes.c_int, [_P, _P, _I32, ctypes.POINTER(RksStats)]),
    "rks_num_pairs": (_I32, [_P]),
    "rks_eigpairs": (ctypes.c_int, [_P, _P, _P, _P, _I32, _P]),
    "rks_destroy": (None, [_P]),
    "rks_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "rks_last_error": (ctypes.c_char_p, [_P]),
    "rks_sketch": (ctypes.c_int, [_P, _P, _P]),
    "rks_spmv_sketch": (ctypes.c_int, [_P, _P, _P, _P]),
    "rks_sketch_noalloc": (ctypes.c_int, [_I64, _I32, _I32, _I32, ctypes.c_uint64, _P, _P, _P]),
    "rks_arnoldi": (ctypes.c_int, [_P, _P, _I32]),
    "rks_get_state": (ctypes.c_int, [_P, ctypes.POINTER(_I32), _P, _P, _P]),
    "rks_rotate": (ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P]),
    "rks_host_schur": (ctypes.c_int, [_I32, _P, _P]),
    "rks_host_order": (ctypes.c_int, [_I32, _P, _P, _I32, _I32, ctypes.POINTER(_I32)]),
    "rks_net_conv3x3_forward": (ctypes.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _P]),
    "rks_net_conv3x3_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _I32,
                                                _I32, _P]),
    "rks_net_subspace_loss": (ctypes.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, _P]),
    "rks_net_adam": (ctypes.c_int, [_P, _P, _P, _P, _I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, _I32, _P]),
    "rks_net_upsample": (ctypes.c_int, [_P, _I32, _I32, _P, _I32, _I32, _P]),
    "rks_copy_probe": (ctypes.c_int, [_P, _P, _I64, _I32, ctypes.POINTER(_D), _P]),
    "rks_read_probe": (ctypes.c_int, [_P, _I64, _I32, ctypes.POINTER(_D), _P]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librks.so (built by ``__graft_entry__.build()``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: run __graft_entry__.build() first")
    # PyTorch-ROCm ships its own HIP runtime.  Loading it first makes this
    # library bind to that same runtime instead of a second copy (two HIP
    # runtimes in one process do not share devices).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class RksError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rks error {code}: {msg}")
        self.code = code


def _ptr(x):
    """Address of a host NumPy array or a device buffer (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _is_device(x) -> bool:
    return x is not None and (hasattr(x, "data_ptr") or isinstance(x, int))


def _check(ctx, code: int, allow=(RKS_OK,)) -> int:
    if code in allow:
        return code
    lib = load()
    msg = lib.rks_last_error(ctx).decode() if ctx else ""
    if not msg:
        msg = lib.rks_strerror(code).decode()
    raise RksError(code, msg)


def rks_opts_default(**kw) -> RksOpts:
    o = RksOpts()
    load().rks_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "sketch_kind" and isinstance(v, str):
            v = SKETCH[v]
        if k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        if k == "spmv_layout" and isinstance(v, str):
            v = SPMV_LAYOUT[v]
        if k == "method" and isinstance(v, str):
            v = METHOD[v]
        if k == "a_values" and isinstance(v, str):
            v = A_VALUES[v]
        if k == "stream" and v is not None and not isinstance(v, int):
            v = int(v.cuda_stream)
        setattr(o, k, v)
    return o


def rks_create(row_ptr, col, val, n, k, m, d, which, tol, opts: RksOpts = None):
    """Create a solver context (CSR arrays on host as NumPy or on device)."""
    lib = load()
    on_dev = _is_device(row_ptr)
    if not on_dev:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        nnz = int(row_ptr[-1])
    else:
        nnz = int(val.numel())
    a = RksCsr(int(n), nnz, _ptr(row_ptr), _ptr(col), _ptr(val), 1 if on_dev else 0)
    if isinstance(which, str):
        which = WHICH[which]
    ctx = ctypes.c_void_p()
    code = lib.rks_create(ctypes.byref(a), int(k), int(m), int(d), int(which), float(tol),
                          ctypes.byref(opts) if opts is not None else None, ctypes.byref(ctx))
    if code != RKS_OK:
        raise RksError(code, lib.rks_last_error(None).decode() or lib.rks_strerror(code).decode())
    return ctx


def rks_solve(ctx, u0=None, stats: RksStats = None) -> int:
    u0p = None
    on_dev = 0
    if u0 is not None:
        if _is_device(u0):
            on_dev = 1
        else:
            u0 = np.ascontiguousarray(u0, dtype=np.float64)
        u0p = _ptr(u0)
    st = stats if stats is not None else RksStats()
    code = load().rks_solve(ctx, u0p, on_dev, ctypes.byref(st))
    return _check(ctx, code, allow=(RKS_OK, RKS_ENOTCONV))


def rks_num_pairs(ctx) -> int:
    return int(load().rks_num_pairs(ctx))


def rks_eigpairs(ctx, lam_re, lam_im, X, resid) -> int:
    x_dev = 1 if _is_device(X) else 0
    return _check(ctx, load().rks_eigpairs(ctx, _ptr(lam_re), _ptr(lam_im), _ptr(X), x_dev, _ptr(resid)))


def rks_destroy(ctx) -> None:
    if ctx:
        load().rks_destroy(ctx)


def rks_strerror(code: int) -> str:
    return load().rks_strerror(code).decode()


def rks_last_error(ctx) -> str:
    return load().rks_last_error(ctx).decode()


def rks_sketch(ctx, x_dev, z_dev) -> int:
    return _check(ctx, load().rks_sketch(ctx, _ptr(x_dev), _ptr(z_dev)))


def rks_sketch_noalloc(n, d, sketch_kind, zeta, sketch_seed, x_dev, z_dev, stream=None) -> int:
    if isinstance(sketch_kind, str):
        sketch_kind = SKETCH[sketch_kind]
    return _check(None, load().rks_sketch_noalloc(int(n), int(d), int(sketch_kind), int(zeta), int(sketch_seed),
                                                  _ptr(x_dev), _ptr(z_dev), _stream(stream)))


def rks_spmv_sketch(ctx, x_dev, w_dev, z_dev) -> int:
    return _check(ctx, load().rks_spmv_sketch(ctx, _ptr(x_dev), _ptr(w_dev), _ptr(z_dev)))


def rks_arnoldi(ctx, u0=None) -> int:
    u0p, on_dev = None, 0
    if u0 is not None:
        if _is_device(u0):
            on_dev = 1
        else:
            u0 = np.ascontiguousarray(u0, dtype=np.float64)
        u0p = _ptr(u0)
    return _check(ctx, load().rks_arnoldi(ctx, u0p, on_dev))


def rks_get_state(ctx, B=None, S=None, U=None) -> int:
    nc = ctypes.c_int32(0)
    _check(ctx, load().rks_get_state(ctx, ctypes.byref(nc), _ptr(B), _ptr(S), _ptr(U)))
    return int(nc.value)


def rks_rotate(ctx, in0, min_, out0, kout, Y) -> int:
    Y = np.asfortranarray(Y, dtype=np.float64)
    return _check(ctx, load().rks_rotate(ctx, int(in0), int(min_), int(out0), int(kout), _ptr(Y)))


def rks_host_schur(A):
    """Real Schur form (T, Z) of a small dense matrix with the library's host code."""
    T = np.asfortranarray(A, dtype=np.float64).copy(order="F")
    n = T.shape[0]
    Z = np.zeros((n, n), order="F")
    _check(None, load().rks_host_schur(n, _ptr(T), _ptr(Z)))
    return T, Z


def rks_host_order(T, Z, which, kw):
    T = np.array(T, dtype=np.float64, order="F")
    Z = np.array(Z, dtype=np.float64, order="F")
    p = ctypes.c_int32(0)
    if isinstance(which, str):
        which = WHICH[which]
    _check(None, load().rks_host_order(T.shape[0], _ptr(T), _ptr(Z), int(which), int(kw), ctypes.byref(p)))
    return T, Z, int(p.value)


def _stream(stream):
    if stream is None:
        return None
    return stream if isinstance(stream, int) else int(stream.cuda_stream)


def rks_net_conv3x3_forward(x, w, b, y, B, Cin, Cout, H, W, dil, relu, stream=None) -> int:
    return _check(None, load().rks_net_conv3x3_forward(_ptr(x), _ptr(w), _ptr(b), _ptr(y), B, Cin, Cout, H, W,
                                                       dil, int(relu), _stream(stream)))


def rks_net_conv3x3_backward(x, w, y, dy, dx, dw, db, B, Cin, Cout, H, W, dil, relu, stream=None) -> int:
    return _check(None, load().rks_net_conv3x3_backward(_ptr(x), _ptr(w), _ptr(y), _ptr(dy), _ptr(dx), _ptr(dw),
                                                        _ptr(db), B, Cin, Cout, H, W, dil, int(relu),
                                                        _stream(stream)))


def rks_net_subspace_loss(u, V, loss, du, B, P, K, stream=None) -> int:
    return _check(None, load().rks_net_subspace_loss(_ptr(u), _ptr(V), _ptr(loss), _ptr(du), B, P, K,
                                                     _stream(stream)))


def rks_net_adam(w, g, m, v, n, lr, t, b1=0.9, b2=0.999, eps=1e-8, stream=None) -> int:
    return _check(None, load().rks_net_adam(_ptr(w), _ptr(g), _ptr(m), _ptr(v), int(n), lr, b1, b2, eps, int(t),
                                            _stream(stream)))


def rks_net_upsample(u, h, w, out, H, W, stream=None) -> int:
    return _check(None, load().rks_net_upsample(_ptr(u), h, w, _ptr(out), H, W, _stream(stream)))


def rks_read_probe(src, nbytes, iters=20, stream=None) -> float:
    """Achieved GB/s of a plain streaming read of nbytes of a device buffer."""
    g = ctypes.c_double(0.0)
    _check(None, load().rks_read_probe(_ptr(src), int(nbytes), int(iters), ctypes.byref(g), _stream(stream)))
    return g.value


def rks_copy_probe(src, dst, nbytes, iters=20, stream=None) -> float:
    """Achieved GB/s (read + write) of a plain device copy of nbytes."""
    g = ctypes.c_double(0.0)
    _check(None, load().rks_copy_probe(_ptr(src), _ptr(dst), int(nbytes), int(iters), ctypes.byref(g),
                                       _stream(stream)))
    return g.value
