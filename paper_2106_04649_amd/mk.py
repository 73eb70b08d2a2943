"""ctypes binding of the C ABI in include/mk.h (argument marshalling only).

Every step of the Marchenko series runs in the HIP kernels of libmk.so; this
module only converts numpy arrays / torch tensors into pointers, passes the
torch stream, and turns status codes into exceptions.  If the library is
missing it raises: there is no fallback path.

Functions carry the ABI's names: mk_plan, mk_load_R, mk_set_focal,
mk_iterate, mk_iterate_tol, mk_get, mk_image, mk_passes, mk_profile,
mk_destroy, the series-tail calls mk_tail_* and the network calls mk_net_*.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MK_LIBRARY selects another build of the same library, such as
# libmk_checked.so (device-side bounds checks); it must exist as well
LIB_PATH = os.environ.get("MK_LIBRARY") or os.path.join(HERE, "libmk.so")
CHECKED_LIB_PATH = os.path.join(HERE, "libmk_checked.so")

MK_OK, MK_ERR_ARG, MK_ERR_STATE, MK_ERR_OOM, MK_ERR_HIP, MK_ERR_UNSUPPORTED, MK_ERR_DIVERGED = range(7)
MK_R_C64, MK_R_F16S, MK_R_BF16S = 0, 1, 2
MK_F1PLUS, MK_F1MINUS, MK_GPLUS, MK_GMINUS, MK_F2PLUS, MK_PMINUS, MK_GTOTAL = 0, 1, 2, 3, 4, 5, 6
MK_FLAG_GRAPH, MK_FLAG_PROFILE, MK_FLAG_AUTOTUNE, MK_FLAG_FAST_X, MK_FLAG_ROW_R, MK_FLAG_WALK, MK_FLAG_GRID = \
    0x1, 0x2, 0x4, 0x8, 0x10, 0x20, 0x40
FIELDS = {"f1plus": MK_F1PLUS, "f1minus": MK_F1MINUS, "Gplus": MK_GPLUS, "Gminus": MK_GMINUS,
          "f2plus": MK_F2PLUS, "pminus": MK_PMINUS, "Gtotal": MK_GTOTAL}
KERNEL_KINDS = {"contract": 0, "epilogue": 1, "norms": 2, "init": 3, "gassembly": 4, "image": 5}


class mk_plan_desc(ctypes.Structure):
    _fields_ = [
        ("nr", ctypes.c_int32),
        ("ns", ctypes.c_int32),
        ("nt", ctypes.c_int32),
        ("iw_lo", ctypes.c_int32),
        ("iw_hi", ctypes.c_int32),
        ("nf_max", ctypes.c_int32),
        ("dt", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("div_factor", ctypes.c_double),
        ("rprec", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
        ("r_dev_bytes", ctypes.c_int64),
    ]


class MKError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2106_04649_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    sigs = {
        "mk_plan": (i32, [ctypes.POINTER(mk_plan_desc), ctypes.POINTER(P)]),
        "mk_load_R": (i32, [P, P, ctypes.c_int]),
        "mk_set_focal": (i32, [P, i32, P, P, i32, P, ctypes.c_int]),
        "mk_iterate": (i32, [P, i32, P]),
        "mk_iterate_tol": (i32, [P, ctypes.c_double, i32, ctypes.POINTER(i32), P]),
        "mk_get": (i32, [P, i32, P, ctypes.c_int]),
        "mk_passes": (i32, [P, ctypes.POINTER(i32)]),
        "mk_image": (i32, [P, ctypes.POINTER(ctypes.c_double)]),
        "mk_tune": (i32, [P, i32]),
        "mk_contract_variant": (i32, [P, i32, ctypes.POINTER(i32)]),
        "mk_profile": (i32, [P, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                             ctypes.c_int]),
        "mk_destroy": (i32, [P]),
        "mk_state_bytes": (i32, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "mk_get_state": (i32, [P, P, ctypes.c_size_t]),
        "mk_set_state": (i32, [P, P, ctypes.c_size_t]),
        "mk_tail_record": (i32, [P, i32, i32]),
        "mk_tail_load": (i32, [P, P, i32]),
        "mk_tail_history": (i32, [P, P, ctypes.c_int]),
        "mk_tail_apply": (i32, [P, i32, P]),
        "mk_net_param_count": (i32, [i32, i32]),
        "mk_net_last_error": (ctypes.c_char_p, []),
        "mk_net_forward": (i32, [P, P, i32, i32, i32, i32, P, P, P]),
        "mk_net_backward": (i32, [P, P, P, P, i32, i32, i32, i32, P, P, P]),
        "mk_net_loss": (i32, [P, P, P, i32, i32, ctypes.c_float, P, P, P, i32, P]),
        "mk_net_loss_noalloc": (i32, [P, P, P, i32, i32, ctypes.c_float, P, P, i32, P]),
        "mk_net_adam": (i32, [P, P, P, P, P, i32, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, P]),
        "mk_net_round": (i32, [P, P, i32, P]),
        "mk_strerror": (ctypes.c_char_p, [i32]),
        "mk_last_error": (ctypes.c_char_p, [P]),
        "mk_device_checks": (i32, [ctypes.POINTER(ctypes.c_uint32)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, plan: Optional[int]) -> None:
    if status == MK_OK:
        return
    lib = load_library()
    msg = lib.mk_last_error(plan).decode() or lib.mk_strerror(status).decode()
    raise MKError(status, msg)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype: str) -> Tuple[int, int, object]:
    """(pointer, on_device, keepalive) of a contiguous numpy array or torch tensor."""
    if x is None:
        return 0, 0, None
    if _is_torch(x):
        import torch

        want = {"float32": torch.float32, "int32": torch.int32, "complex64": torch.complex64}[dtype]
        if x.dtype != want:
            raise TypeError(f"expected a {dtype} tensor, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr(), 1 if x.is_cuda else 0, x
    a = np.ascontiguousarray(x, dtype=np.dtype(dtype))
    return a.ctypes.data, 0, a


def _expect_shape(x, shape, what: str) -> None:
    """Raise ValueError unless x has exactly `shape` (the library reads that many elements)."""
    got = tuple(int(v) for v in x.shape)
    if got != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {got}")


def _current_stream() -> int:
    import torch

    return torch.cuda.current_stream().cuda_stream


class Plan:
    """Owner of an mk_plan_t handle (destroyed with the object)."""

    def __init__(self, handle: int, desc: mk_plan_desc):
        self.handle = handle
        self.desc = desc
        self.nf = 0

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                load_library().mk_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def mk_plan(nr: int, ns: int, nt: int, dt: float, dx: float, band: Optional[Tuple[int, int]] = None,
            nf_max: int = 1, rprec: int = MK_R_C64, flags: int = 0, div_factor: float = 0.0,
            stream: Optional[int] = None, r_dev_bytes: int = 0) -> Plan:
    """r_dev_bytes > 0 caps the device memory holding R (below R's size, R is
    streamed from pinned host memory in slabs of frequency bins)."""
    lib = load_library()
    lo, hi = band if band is not None else (0, nt // 2)
    if stream is None:
        stream = _current_stream()
    d = mk_plan_desc(nr, ns, nt, lo, hi, nf_max, dt, dx, div_factor, rprec, flags, stream, int(r_dev_bytes))
    h = ctypes.c_void_p()
    _check(lib.mk_plan(ctypes.byref(d), ctypes.byref(h)), None)
    return Plan(h.value, d)


def mk_load_R(plan: Plan, R) -> None:
    """R: complex64 [nr][B][ns], or float32 [nr][B][ns][2] (numpy or torch, host or device)."""
    d = plan.desc
    shape = (d.nr, d.iw_hi - d.iw_lo + 1, d.ns)
    if (_is_torch(R) and R.dtype.is_complex) or (isinstance(R, np.ndarray) and np.iscomplexobj(R)):
        _expect_shape(R, shape, "R")
    else:
        _expect_shape(R, shape + (2,), "R (interleaved float32 pairs)")
    if _is_torch(R) and R.dtype.is_complex:
        import torch

        R = torch.view_as_real(R)
        ptr, dev, keep = _ptr(R, "float32")
    elif isinstance(R, np.ndarray) and np.iscomplexobj(R):
        keep = np.ascontiguousarray(R, dtype=np.complex64)
        ptr, dev = keep.ctypes.data, 0
    else:
        ptr, dev, keep = _ptr(R, "float32")
    _check(load_library().mk_load_R(plan.handle, ptr, dev), plan.handle)


def mk_set_focal(plan: Plan, Gd, itd, shift: int, band=None) -> None:
    """Gd float32 [nf][nr][nt], itd int32 [nf][nr], band int32 [nf][2] or None."""
    d = plan.desc
    nf = int(Gd.shape[0]) if len(Gd.shape) == 3 else -1
    if not 1 <= nf <= d.nf_max:
        raise ValueError(f"Gd must have shape [nf][{d.nr}][{d.nt}] with 1 <= nf <= {d.nf_max}")
    _expect_shape(Gd, (nf, d.nr, d.nt), "Gd")
    _expect_shape(itd, (nf, d.nr), "itd")
    if band is not None:
        _expect_shape(band, (nf, 2), "band")
    gp, gdev, gk = _ptr(Gd, "float32")
    ip, idev, ik = _ptr(itd, "int32")
    bp, bdev, bk = _ptr(band, "int32")
    if band is not None and bdev != gdev:
        raise ValueError("Gd and band must both be host or both be device arrays")
    if idev != gdev:
        raise ValueError("Gd and itd must both be host or both be device arrays")
    _check(load_library().mk_set_focal(plan.handle, nf, gp, ip, int(shift), bp, gdev), plan.handle)
    plan.nf = nf


def mk_iterate(plan: Plan, niter: int, want_norms: bool = True) -> Optional[np.ndarray]:
    """Run niter passes; returns ||N_i|| as float64 [niter][nf] (synchronises) or None."""
    if want_norms and niter > 0:
        out = np.zeros((niter, plan.nf), dtype=np.float64)
        _check(load_library().mk_iterate(plan.handle, int(niter), out.ctypes.data), plan.handle)
        return out
    _check(load_library().mk_iterate(plan.handle, int(niter), None), plan.handle)
    return None


def mk_iterate_tol(plan: Plan, tol: float, max_passes: int) -> Tuple[int, np.ndarray]:
    """Passes until the library's error estimate is within tol (or max_passes):
    returns (passes run, estimate per focal point as float64 [nf])."""
    est = np.zeros(plan.nf, dtype=np.float64)
    n = ctypes.c_int32()
    _check(load_library().mk_iterate_tol(plan.handle, float(tol), int(max_passes), ctypes.byref(n),
                                         est.ctypes.data), plan.handle)
    return n.value, est


def mk_get(plan: Plan, field, out=None):
    """Copy a field [nf][nr][nt] float32 into out (torch device tensor or numpy), returns out."""
    fid = FIELDS[field] if isinstance(field, str) else int(field)
    shape = (plan.nf, plan.desc.nr, plan.desc.nt)
    if out is None:
        import torch

        out = torch.empty(shape, dtype=torch.float32, device="cuda")
    if tuple(out.shape) != shape:
        raise ValueError(f"out must have shape {shape}")
    if _is_torch(out):
        ptr, dev, _ = _ptr(out, "float32")
    else:
        if out.dtype != np.float32 or not out.flags.c_contiguous:
            raise TypeError("out must be a C-contiguous float32 array")
        ptr, dev = out.ctypes.data, 0
    _check(load_library().mk_get(plan.handle, fid, ptr, dev), plan.handle)
    return out


def mk_image(plan: Plan) -> np.ndarray:
    """Double-focusing image per focal point (float64 [nf], the caller's focal order)."""
    out = np.zeros(plan.nf, dtype=np.float64)
    _check(load_library().mk_image(plan.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), plan.handle)
    return out


def mk_passes(plan: Plan) -> int:
    v = ctypes.c_int32()
    _check(load_library().mk_passes(plan.handle, ctypes.byref(v)), plan.handle)
    return v.value


def mk_tune(plan: Plan, mode: int) -> None:
    """-1 heuristic, -2 autotune, 0 GEMV, v >= 1 MFMA tile shape v - 1."""
    _check(load_library().mk_tune(plan.handle, int(mode)), plan.handle)


def mk_contract_variant(plan: Plan, ncols: int) -> int:
    v = ctypes.c_int32()
    _check(load_library().mk_contract_variant(plan.handle, int(ncols), ctypes.byref(v)), plan.handle)
    return v.value


def mk_profile(plan: Plan, kind, reset: bool = False) -> Tuple[float, int]:
    k = KERNEL_KINDS[kind] if isinstance(kind, str) else int(kind)
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load_library().mk_profile(plan.handle, k, ctypes.byref(ms), ctypes.byref(n), int(reset)),
           plan.handle)
    return ms.value, n.value


def mk_get_state(plan: Plan) -> bytes:
    """The current series' state as an opaque blob (checkpoint)."""
    lib = load_library()
    n = ctypes.c_size_t()
    _check(lib.mk_state_bytes(plan.handle, ctypes.byref(n)), plan.handle)
    buf = ctypes.create_string_buffer(n.value)
    _check(lib.mk_get_state(plan.handle, buf, n.value), plan.handle)
    return buf.raw


def mk_set_state(plan: Plan, blob: bytes) -> None:
    """Resume the series saved by mk_get_state (same plan shape, R loaded)."""
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    _check(load_library().mk_set_state(plan.handle, buf, len(blob)), plan.handle)
    # the blob's header: 8 magic bytes, then int32 nr, nt, iw_lo, iw_hi, ns_pad, rprec, flags, nf, ...
    plan.nf = int.from_bytes(bytes(blob)[36:40], "little", signed=True)


def mk_device_checks() -> int:
    """Bit mask of the kernel files whose device-side bounds checks failed
    since the last call (0: none), from the checked build; raises MKError
    (MK_ERR_UNSUPPORTED) on the normal build."""
    v = ctypes.c_uint32(0)
    _check(load_library().mk_device_checks(ctypes.byref(v)), None)
    return int(v.value)


def mk_destroy(plan: Plan) -> None:
    if plan.handle:
        _check(load_library().mk_destroy(plan.handle), None)
        plan.handle = None


# --- series tail ------------------------------------------------------------

TAIL_NET, TAIL_GEOMETRIC, TAIL_NONE = 0, 1, 2


def mk_tail_record(plan: Plan, k: int, T: int) -> None:
    _check(load_library().mk_tail_record(plan.handle, int(k), int(T)), plan.handle)
    plan.tail_kT = (int(k), int(T))


def mk_tail_load(plan: Plan, params) -> None:
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(load_library().mk_tail_load(plan.handle, a.ctypes.data, a.size), plan.handle)


def mk_tail_history(plan: Plan, out=None):
    k, T = plan.tail_kT
    shape = (plan.nf, plan.desc.nr, k, T)
    if out is None:
        out = np.zeros(shape, np.float32)
    _expect_shape(out, shape, "out")
    if _is_torch(out):
        ptr, dev, _ = _ptr(out, "float32")
    else:
        if out.dtype != np.float32 or not out.flags.c_contiguous:
            raise TypeError("out must be a C-contiguous float32 array")
        ptr, dev = out.ctypes.data, 0
    _check(load_library().mk_tail_history(plan.handle, ptr, dev), plan.handle)
    return out


def mk_tail_apply(plan: Plan, mode: int = TAIL_NET) -> np.ndarray:
    res = np.zeros(plan.nf, np.float64)
    _check(load_library().mk_tail_apply(plan.handle, int(mode), res.ctypes.data), plan.handle)
    return res


# --- series-tail network (device tensors only) --------------------------------


def _dev(t, dtype="float32"):
    import torch

    want = {"float32": torch.float32, "float64": torch.float64}[dtype]
    if not (t.is_cuda and t.dtype == want and t.is_contiguous()):
        raise TypeError(f"expected a contiguous CUDA {dtype} tensor")
    return t.data_ptr()


def _net_check(status: int) -> None:
    if status != MK_OK:
        raise MKError(status, load_library().mk_net_last_error().decode())


def mk_net_param_count(k: int, hidden: int = 64) -> int:
    return int(load_library().mk_net_param_count(int(k), int(hidden)))


def net_hidden(nparams: int, k: int) -> int:
    """Hidden width of a parameter vector of nparams floats for k inputs."""
    for h in range(1, 129):
        if mk_net_param_count(k, h) == nparams:
            return h
    raise ValueError(f"{nparams} parameters fit no hidden width for k={k}")


def mk_net_forward(params, x, work, y, stream=None, hidden=None) -> None:
    N, k, T = x.shape
    h = net_hidden(params.numel(), k) if hidden is None else int(hidden)
    s = _current_stream() if stream is None else stream
    _net_check(load_library().mk_net_forward(_dev(params), _dev(x), N, k, h, T, _dev(work), _dev(y), s))


def mk_net_backward(params, x, work, gy, grads, work2, stream=None, hidden=None) -> None:
    N, k, T = x.shape
    h = net_hidden(params.numel(), k) if hidden is None else int(hidden)
    s = _current_stream() if stream is None else stream
    _net_check(load_library().mk_net_backward(_dev(params), _dev(x), _dev(work), _dev(gy), N, k, h, T,
                                              _dev(grads), _dev(work2), s))


def mk_net_loss(y, target, mask, count, gy, loss, part, stream=None) -> None:
    N, _, T = y.shape
    s = _current_stream() if stream is None else stream
    _net_check(load_library().mk_net_loss(_dev(y), _dev(target), _dev(mask), N, T, float(count), _dev(gy),
                                          _dev(loss, "float64"), _dev(part, "float64"), part.numel(), s))


def mk_net_loss_noalloc(y, target, mask, count, gy, loss, nparts=256, stream=None) -> None:
    """mk_net_loss with the partial sums in the library's fixed scratch array
    (no buffer from the caller, nothing allocated; nparts <= 1024)."""
    N, _, T = y.shape
    s = _current_stream() if stream is None else stream
    _net_check(load_library().mk_net_loss_noalloc(_dev(y), _dev(target), _dev(mask), N, T, float(count),
                                                  _dev(gy), _dev(loss, "float64"), int(nparts), s))


def mk_net_adam(w, wq, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None) -> None:
    s = _current_stream() if stream is None else stream
    _net_check(load_library().mk_net_adam(_dev(w), _dev(wq), _dev(g), _dev(m), _dev(v), w.numel(), int(step),
                                          float(lr), float(b1), float(b2), float(eps), s))


def mk_net_round(w, wq, stream=None) -> None:
    s = _current_stream() if stream is None else stream
    _net_check(load_library().mk_net_round(_dev(w), _dev(wq), w.numel(), s))
