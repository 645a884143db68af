"""ctypes binding of libmpchol (include/mpchol.h): argument marshalling only.

Every call goes straight to the C ABI of the HIP library; no arithmetic of
the method happens here.  Device buffers are torch tensors (used for memory
and streams only); host buffers are numpy arrays.  A missing library raises
at import of the first call -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libmpchol.so")

OK, NOT_SPD = 0, 1
EINVAL, ENOMEM, EHIP, EORDER, EBUDGET, EUNSUPPORTED = -1, -2, -3, -4, -5, -6
P64, P32, P16, P8 = 0, 1, 2, 3
LO16_F16, LO16_BF16 = 0, 1
RULE_FP64, RULE_NORM, RULE_BAND, RULE_USER, RULE_LEARNED = 0, 1, 2, 3, 4
BAND_DP_SP, BAND_DP_SP_HP, BAND_DP_HP = 1, 2, 3
LO32_FP32, LO32_BF16X3 = 0, 1
LO64_FP64, LO64_INT8 = 0, 1
LO8_TILE, LO8_MX = 0, 1
MLP_NPARAM = 4996


class MpcholError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        detail = last_error() if status == -3 or status == -2 else ""
        super().__init__(f"{where}: {strerror(status)} ({status})" + (f" [{detail}]" if detail else ""))


class Opts(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("lo16", C.c_int32), ("band", C.c_int32),
                ("allowed", C.c_uint32), ("band_variant", C.c_int32), ("verify", C.c_int32),
                ("verify_eps", C.c_double), ("profile", C.c_int32), ("lo32", C.c_int32), ("lo64", C.c_int32),
                ("lo8", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("tile", C.c_int32), ("nt", C.c_int32), ("tiles_per_class", C.c_int64 * 4),
                ("flops_per_class", C.c_double * 4), ("total_fro", C.c_double), ("t_map_ms", C.c_double),
                ("t_factor_ms", C.c_double), ("t_solve_ms", C.c_double), ("t_sample_ms", C.c_double),
                ("t_residual_ms", C.c_double), ("t_gemm_ms", C.c_double * 4), ("gemm_launches", C.c_int64 * 4),
                ("gemm_flops", C.c_double * 4), ("fallbacks", C.c_int32), ("rule_used", C.c_int32),
                ("verify_first", C.c_double), ("t_samples_ms", C.c_double), ("t_gemm_int8_ms", C.c_double),
                ("gemm_int8_launches", C.c_int64), ("gemm_int8_flops", C.c_double)]


_lib = None


def lib():
    """Load libmpchol.so; raises if it has not been built.

    torch is imported first: its bundled HIP runtime carries the same SONAME
    (libamdhip64.so.7) as the one libmpchol.so links, so loading torch first
    makes the library bind to torch's runtime -- one runtime per process,
    whose streams and device pointers both sides share.  Loading the library
    first would bring in a second HIP runtime when torch is imported later.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIBPATH):
            raise ImportError(f"libmpchol.so not built at {LIBPATH}: run __graft_entry__.build() "
                              "or python paper_2408_04440_amd/build.py")
        L = C.CDLL(LIBPATH)
        vp, i32, i64, d, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
        sig = {
            "mpchol_default_opts": (None, [C.POINTER(Opts)]),
            "mpchol_create": (C.c_int, [C.POINTER(vp), i64, i32, C.POINTER(Opts)]),
            "mpchol_destroy": (C.c_int, [vp]),
            "mpchol_set_matrix": (C.c_int, [vp, vp, i64, i32]),
            "mpchol_set_generator": (C.c_int, [vp, vp, vp, d, d]),
            "mpchol_set_samples": (C.c_int, [vp, vp, i64, i64, d, d, i32]),
            "mpchol_precision_map": (C.c_int, [vp, i32, d, vp, vp]),
            "mpchol_factor": (C.c_int, [vp, C.POINTER(i64)]),
            "mpchol_logdet": (C.c_int, [vp, C.POINTER(d)]),
            "mpchol_solve": (C.c_int, [vp, i32, vp, i64]),
            "mpchol_sample": (C.c_int, [vp, i32, u64, vp, i64]),
            "mpchol_sample_z": (C.c_int, [vp, i32, vp, i64, vp, i64]),
            "mpchol_sample_noalloc": (C.c_int, [vp, i32, u64, vp, i64]),
            "mpchol_normal_draws": (C.c_int, [vp, i64, u64, vp, vp]),
            "mpchol_backward_error": (C.c_int, [vp, C.POINTER(d), vp]),
            "mpchol_backward_error_estimate": (C.c_int, [vp, i32, u64, C.POINTER(d)]),
            "mpchol_backward_error_matrix": (C.c_int, [vp, vp, i64, i32, C.POINTER(d), vp]),
            "mpchol_get_factor": (C.c_int, [vp, vp, i64]),
            "mpchol_get_tile_scales": (C.c_int, [vp, vp]),
            "mpchol_get_stats": (C.c_int, [vp, C.POINTER(Stats)]),
            "mpchol_set_verify": (C.c_int, [vp, i32, d]),
            "mpchol_strerror": (C.c_char_p, [C.c_int]),
            "mpchol_last_error": (C.c_char_p, []),
            "mpchol_selector_set": (C.c_int, [vp, vp, i64]),
            "mpchol_selector_features": (C.c_int, [vp, d, vp]),
            "mpchol_selector_labels": (C.c_int, [vp, d, vp, C.POINTER(d), vp]),
            "mpchol_mlp_create": (C.c_int, [C.POINTER(vp), i32, vp]),
            "mpchol_mlp_destroy": (C.c_int, [vp]),
            "mpchol_mlp_set_params": (C.c_int, [vp, vp, i64]),
            "mpchol_mlp_get_params": (C.c_int, [vp, vp, i64]),
            "mpchol_mlp_get_state": (C.c_int, [vp, vp, vp, vp, C.POINTER(i32), i64]),
            "mpchol_mlp_set_state": (C.c_int, [vp, vp, vp, vp, i32, i64]),
            "mpchol_mlp_grad": (C.c_int, [vp, vp, vp, i64, vp, C.c_float, vp, C.POINTER(C.c_float)]),
            "mpchol_mlp_train_step": (C.c_int, [vp, vp, vp, i64, vp, C.c_float, C.c_float, C.POINTER(C.c_float)]),
            "mpchol_mlp_predict": (C.c_int, [vp, vp, i64, vp, vp]),
            "mpchol_sht_create": (C.c_int, [C.POINTER(vp), i32, i32, i32, i32, i32, vp]),
            "mpchol_sht_destroy": (C.c_int, [vp]),
            "mpchol_sht_forward": (C.c_int, [vp, vp, i64, vp]),
            "mpchol_sht_inverse": (C.c_int, [vp, vp, i64, vp]),
            "mpchol_sht_info": (C.c_int, [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]),
            "mpchol_sht_last_error": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().mpchol_strerror(int(status)).decode()


def last_error() -> str:
    return lib().mpchol_last_error().decode()


def _chk(rc, where, allow_not_spd=False):
    if rc < 0 or (rc == NOT_SPD and not allow_not_spd):
        raise MpcholError(rc, where)
    return rc


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def _colmajor_ld(t, n):
    """Leading dimension of a column-major 2-D tensor/array view (stride (1, ld))."""
    if t.dim() == 1:
        return max(n, t.shape[0])
    s = t.stride()
    if s[0] != 1:
        raise ValueError("expected a column-major view (stride (1, ld)); pass X.T of a contiguous (cols, rows) tensor")
    return s[1] if t.shape[1] > 1 else max(n, t.shape[0])


def _check_device(t, dtype, name, rows=None, cols=None, numel=None):
    """A device buffer the kernels will read or write: a CUDA torch tensor of
    `dtype` holding at least `rows` x `cols` (a column-major view) or `numel`
    elements.  Raises ValueError before any library call, so a wrong buffer
    never reaches a kernel."""
    if not hasattr(t, "is_cuda") or not t.is_cuda:
        raise ValueError(f"{name}: expected a CUDA torch tensor")
    if str(t.dtype) != "torch." + dtype:
        raise ValueError(f"{name}: expected dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, need {numel}")
    if rows is not None:
        r = t.shape[0]
        c = 1 if t.dim() == 1 else t.shape[1]
        if t.dim() > 2 or r < rows or (cols is not None and c < cols):
            raise ValueError(f"{name}: shape {tuple(t.shape)}, need at least ({rows}, {cols if cols else 1})")


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch

            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:
            return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# --------------------------------------------------------------------- handle
def mpchol_default_opts() -> Opts:
    o = Opts()
    lib().mpchol_default_opts(C.byref(o))
    return o


def mpchol_create(n, tile, device=0, stream=None, lo16=LO16_F16, band=1, allowed=0xF, band_variant=BAND_DP_HP,
                  verify=0, verify_eps=1e-9, profile=0, lo32=None, lo64=None, lo8=None):
    o = mpchol_default_opts()
    o.device, o.stream, o.lo16, o.band = device, _stream_ptr(stream), lo16, band
    o.allowed, o.band_variant, o.verify, o.verify_eps, o.profile = allowed, band_variant, verify, verify_eps, profile
    if lo32 is not None:
        o.lo32 = lo32
    if lo64 is not None:
        o.lo64 = lo64
    if lo8 is not None:
        o.lo8 = lo8
    h = C.c_void_p()
    _chk(lib().mpchol_create(C.byref(h), int(n), int(tile), C.byref(o)), "mpchol_create")
    return h


def mpchol_destroy(h):
    _chk(lib().mpchol_destroy(h), "mpchol_destroy")


def mpchol_set_matrix(h, A, n=None):
    """A: torch float64 column-major view on the device, or a numpy array (host)."""
    if isinstance(A, np.ndarray):
        A = np.asfortranarray(A, dtype=np.float64)
        rc = lib().mpchol_set_matrix(h, A.ctypes.data_as(C.c_void_p), A.shape[0], 0)
    else:
        _check_device(A, "float64", "A", rows=A.shape[0], cols=A.shape[0])
        rc = lib().mpchol_set_matrix(h, _ptr(A), _colmajor_ld(A, A.shape[0]), 1)
    _chk(rc, "mpchol_set_matrix")


def mpchol_set_generator(h, sigma, x, rho, nugget, n=None):
    """sigma, x: host arrays of at least n values (n: the handle's order, read
    from its stats when not given)."""
    sigma = np.ascontiguousarray(sigma, dtype=np.float64).ravel()
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    n = mpchol_get_stats(h)["n"] if n is None else n
    if sigma.size < n or x.size < n:
        raise ValueError(f"mpchol_set_generator: sigma ({sigma.size}) and x ({x.size}) need {n} values")
    _chk(lib().mpchol_set_generator(h, sigma.ctypes.data_as(C.c_void_p), x.ctypes.data_as(C.c_void_p), float(rho),
                                    float(nugget)), "mpchol_set_generator")


def mpchol_set_samples(h, Xi, scale, nugget, m=None):
    """Sigma = scale * Xi Xi^T + nugget I.  Xi: numpy n x m (host), or a
    torch float64 column-major device view (Xi.T of a contiguous (m, n))."""
    if isinstance(Xi, np.ndarray):
        Xi = np.asfortranarray(Xi, dtype=np.float64)
        rc = lib().mpchol_set_samples(h, Xi.ctypes.data_as(C.c_void_p), Xi.shape[0], Xi.shape[1], float(scale),
                                      float(nugget), 0)
    else:
        m = int(Xi.shape[1] if m is None else m)
        _check_device(Xi, "float64", "Xi", rows=Xi.shape[0], cols=m)
        rc = lib().mpchol_set_samples(h, _ptr(Xi), _colmajor_ld(Xi, Xi.shape[0]), m, float(scale), float(nugget), 1)
    _chk(rc, "mpchol_set_samples")


def mpchol_precision_map(h, rule, eps=1e-9, user_map=None, nt=None):
    st = mpchol_get_stats(h) if nt is None else None
    nt = nt if nt is not None else st["nt"]
    out = np.zeros((nt, nt), dtype=np.uint8, order="F")
    um = None
    if user_map is not None:
        um = np.asfortranarray(user_map, dtype=np.uint8)
        assert um.shape == (nt, nt)
    _chk(lib().mpchol_precision_map(h, int(rule), float(eps), None if um is None else um.ctypes.data_as(C.c_void_p),
                                    out.ctypes.data_as(C.c_void_p)), "mpchol_precision_map")
    return out


def mpchol_factor(h):
    """Returns info (0, or the 1-based failing column)."""
    info = C.c_int64(0)
    _chk(lib().mpchol_factor(h, C.byref(info)), "mpchol_factor", allow_not_spd=True)
    return int(info.value)


def mpchol_logdet(h):
    v = C.c_double(0.0)
    _chk(lib().mpchol_logdet(h, C.byref(v)), "mpchol_logdet")
    return v.value


def mpchol_solve(h, B, n):
    """B: torch float64 column-major (n x nrhs) view or 1-D (n,) tensor on the device; overwritten."""
    nrhs = 1 if B.dim() == 1 else B.shape[1]
    _check_device(B, "float64", "B", rows=n, cols=nrhs)
    _chk(lib().mpchol_solve(h, int(nrhs), _ptr(B), _colmajor_ld(B, n)), "mpchol_solve")


def mpchol_sample(h, ndraws, seed, Y, n):
    _check_device(Y, "float32", "Y", rows=n, cols=int(ndraws))
    _chk(lib().mpchol_sample(h, int(ndraws), C.c_uint64(seed), _ptr(Y), _colmajor_ld(Y, n)), "mpchol_sample")


def mpchol_sample_noalloc(h, ndraws, seed, Y, n):
    _check_device(Y, "float32", "Y", rows=n, cols=int(ndraws))
    _chk(lib().mpchol_sample_noalloc(h, int(ndraws), C.c_uint64(seed), _ptr(Y), _colmajor_ld(Y, n)),
         "mpchol_sample_noalloc")


def mpchol_sample_z(h, Z, Y, n):
    nd = 1 if Z.dim() == 1 else Z.shape[1]
    _check_device(Z, "float32", "Z", rows=n, cols=nd)
    _check_device(Y, "float32", "Y", rows=n, cols=nd)
    _chk(lib().mpchol_sample_z(h, int(nd), _ptr(Z), _colmajor_ld(Z, n), _ptr(Y), _colmajor_ld(Y, n)),
         "mpchol_sample_z")


def mpchol_normal_draws(h, count, seed, z=None, raw=None):
    if z is not None:
        _check_device(z, "float32", "z", numel=int(count))
    if raw is not None:
        if str(raw.dtype) not in ("torch.int32", "torch.uint32"):
            raise ValueError(f"raw: expected a 32-bit integer tensor, got {raw.dtype}")
        _check_device(raw, str(raw.dtype)[6:], "raw", numel=int(count))
    _chk(lib().mpchol_normal_draws(h, int(count), C.c_uint64(seed), _ptr(z), _ptr(raw)), "mpchol_normal_draws")


def mpchol_backward_error(h, tiles=False, nt=None):
    be = C.c_double(0.0)
    tr = None
    if tiles:
        nt = nt if nt is not None else mpchol_get_stats(h)["nt"]
        tr = np.zeros((nt, nt), order="F")
    _chk(lib().mpchol_backward_error(h, C.byref(be), None if tr is None else tr.ctypes.data_as(C.c_void_p)),
         "mpchol_backward_error")
    return (be.value, tr) if tiles else be.value


def mpchol_backward_error_matrix(h, A, tiles=False, nt=None):
    """||A - L L^T||_F / ||A||_F for the caller's A: a numpy array (host) or a
    torch float64 column-major device view; with tiles=True also the per-tile
    squared residuals (nt x nt)."""
    be = C.c_double(0.0)
    tr = None
    if tiles:
        nt = nt if nt is not None else mpchol_get_stats(h)["nt"]
        tr = np.zeros((nt, nt), order="F")
    trp = None if tr is None else tr.ctypes.data_as(C.c_void_p)
    if isinstance(A, np.ndarray):
        A = np.asfortranarray(A, dtype=np.float64)
        rc = lib().mpchol_backward_error_matrix(h, A.ctypes.data_as(C.c_void_p), A.shape[0], 0, C.byref(be), trp)
    else:
        _check_device(A, "float64", "A")
        rc = lib().mpchol_backward_error_matrix(h, _ptr(A), _colmajor_ld(A, A.shape[0]), 1, C.byref(be), trp)
    _chk(rc, "mpchol_backward_error_matrix")
    return (be.value, tr) if tiles else be.value


def mpchol_backward_error_estimate(h, sets=2, seed=7):
    be = C.c_double(0.0)
    _chk(lib().mpchol_backward_error_estimate(h, int(sets), C.c_uint64(seed), C.byref(be)),
         "mpchol_backward_error_estimate")
    return be.value


def mpchol_get_factor(h, L, n):
    _check_device(L, "float64", "L", rows=n, cols=n)
    _chk(lib().mpchol_get_factor(h, _ptr(L), _colmajor_ld(L, n)), "mpchol_get_factor")


def mpchol_get_tile_scales(h, nt):
    t = np.zeros((nt, nt), dtype=np.int32, order="F")
    _chk(lib().mpchol_get_tile_scales(h, t.ctypes.data_as(C.c_void_p)), "mpchol_get_tile_scales")
    return t


def mpchol_set_verify(h, mode, eps):
    _chk(lib().mpchol_set_verify(h, int(mode), float(eps)), "mpchol_set_verify")


def mpchol_get_stats(h):
    s = Stats()
    _chk(lib().mpchol_get_stats(h, C.byref(s)), "mpchol_get_stats")
    out = {}
    for name, _ in Stats._fields_:
        v = getattr(s, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out


# --------------------------------------------------------------------- selector
def mpchol_selector_set(h, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _chk(lib().mpchol_selector_set(h, p.ctypes.data_as(C.c_void_p), p.size), "mpchol_selector_set")


def mpchol_selector_features(h, eps, nt):
    f = np.zeros((nt * nt, 8), dtype=np.float32)
    _chk(lib().mpchol_selector_features(h, float(eps), f.ctypes.data_as(C.c_void_p)), "mpchol_selector_features")
    return f


def mpchol_selector_labels(h, eps, nt, rates=None):
    """(labels, measured backward error); rates: optional per-class update rates (4 values, TFLOP/s)."""
    lab = np.zeros((nt, nt), dtype=np.uint8, order="F")
    be = C.c_double(0.0)
    r = None if rates is None else np.ascontiguousarray(rates, dtype=np.float64)
    if r is not None and r.size != 4:
        raise ValueError("rates: 4 values (FP64, FP32, 16-bit, FP8)")
    _chk(lib().mpchol_selector_labels(h, float(eps), lab.ctypes.data_as(C.c_void_p), C.byref(be),
                                      None if r is None else r.ctypes.data_as(C.c_void_p)), "mpchol_selector_labels")
    return lab, be.value


def mpchol_mlp_create(device=0, stream=None):
    m = C.c_void_p()
    _chk(lib().mpchol_mlp_create(C.byref(m), int(device), _stream_ptr(stream)), "mpchol_mlp_create")
    return m


def mpchol_mlp_destroy(m):
    _chk(lib().mpchol_mlp_destroy(m), "mpchol_mlp_destroy")


def mpchol_mlp_set_params(m, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _chk(lib().mpchol_mlp_set_params(m, p.ctypes.data_as(C.c_void_p), p.size), "mpchol_mlp_set_params")


def mpchol_mlp_get_params(m):
    p = np.zeros(MLP_NPARAM, dtype=np.float32)
    _chk(lib().mpchol_mlp_get_params(m, p.ctypes.data_as(C.c_void_p), p.size), "mpchol_mlp_get_params")
    return p


def mpchol_mlp_get_state(m):
    """(params, m1, m2, step): the trainer's parameters, Adam moments and step count."""
    p, m1, m2 = (np.zeros(MLP_NPARAM, dtype=np.float32) for _ in range(3))
    st = C.c_int32(0)
    _chk(lib().mpchol_mlp_get_state(m, p.ctypes.data_as(C.c_void_p), m1.ctypes.data_as(C.c_void_p),
                                    m2.ctypes.data_as(C.c_void_p), C.byref(st), MLP_NPARAM), "mpchol_mlp_get_state")
    return p, m1, m2, int(st.value)


def mpchol_mlp_set_state(m, params, m1, m2, step):
    arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (params, m1, m2)]
    if any(a.size != MLP_NPARAM for a in arrs):
        raise ValueError(f"mpchol_mlp_set_state: params and moments need {MLP_NPARAM} values each")
    _chk(lib().mpchol_mlp_set_state(m, *(a.ctypes.data_as(C.c_void_p) for a in arrs), int(step), MLP_NPARAM),
         "mpchol_mlp_set_state")


def _cw(cw):
    return (C.c_float * 4)(*[float(v) for v in cw])


def mpchol_mlp_grad(m, X, y, cw, alpha, grad):
    loss = C.c_float(0.0)
    _chk(lib().mpchol_mlp_grad(m, _ptr(X), _ptr(y), X.shape[0], _cw(cw), float(alpha), _ptr(grad), C.byref(loss)),
         "mpchol_mlp_grad")
    return loss.value


def mpchol_mlp_train_step(m, X, y, cw, alpha, lr, want_loss=True):
    loss = C.c_float(0.0)
    _chk(lib().mpchol_mlp_train_step(m, _ptr(X), _ptr(y), X.shape[0], _cw(cw), float(alpha), float(lr),
                                     C.byref(loss) if want_loss else None), "mpchol_mlp_train_step")
    return loss.value if want_loss else None


def mpchol_mlp_predict(m, X, logits=None, cls=None):
    _chk(lib().mpchol_mlp_predict(m, _ptr(X), X.shape[0], _ptr(logits), _ptr(cls)), "mpchol_mlp_predict")


# ------------------------------------------------------------------------ SHT
def mpchol_sht_create(L, ntheta, nphi, tmax, device=0, stream=None):
    """Transform object for band limit L on an N_theta x N_phi grid, up to tmax
    fields per call."""
    s = C.c_void_p()
    rc = lib().mpchol_sht_create(C.byref(s), int(L), int(ntheta), int(nphi), int(tmax), int(device),
                                 _stream_ptr(stream))
    if rc < 0:
        raise MpcholError(rc, "mpchol_sht_create: " + lib().mpchol_sht_last_error().decode())
    return s


def mpchol_sht_destroy(s):
    if s:
        lib().mpchol_sht_destroy(s)


def _sht_check(t, shape, what):
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous tensor of shape {tuple(shape)}, got {tuple(t.shape)}")


def mpchol_sht_forward(s, Z, f, L):
    """device Z (T, N_theta, N_phi) float64 -> device f (T, L^2) float64."""
    T = Z.shape[0]
    _sht_check(f, (T, L * L), "f")
    if not Z.is_contiguous():
        raise ValueError("Z must be contiguous")
    _chk(lib().mpchol_sht_forward(s, _ptr(Z), int(T), _ptr(f)), "mpchol_sht_forward")


def mpchol_sht_inverse(s, f, Z, L):
    """device f (T, L^2) float64 -> device Z (T, N_theta, N_phi) float64."""
    T = f.shape[0]
    _sht_check(f, (T, L * L), "f")
    if not Z.is_contiguous() or Z.shape[0] != T:
        raise ValueError("Z must be contiguous with T fields")
    _chk(lib().mpchol_sht_inverse(s, _ptr(f), int(T), _ptr(Z)), "mpchol_sht_inverse")


def mpchol_sht_info(s):
    tb, wb, fl = C.c_int64(), C.c_int64(), C.c_int64()
    _chk(lib().mpchol_sht_info(s, C.byref(tb), C.byref(wb), C.byref(fl)), "mpchol_sht_info")
    return {"table_bytes": tb.value, "work_bytes": wb.value, "gemm_flops_per_step": fl.value}
