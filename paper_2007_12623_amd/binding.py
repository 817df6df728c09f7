"""Thin Python binding of libstereo_mi355x.so (argument marshalling only).

Every function has the name of the C entry point it calls (include/stereo.h)
and takes torch tensors: device tensors for device arrays, the current HIP
stream of torch for `stream`.  All arithmetic runs in the library's HIP
kernels; nothing here computes.  Loading fails loudly when the library has
not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstereo_mi355x.so")

ST_OK, ST_EINVAL, ST_ENOMEM, ST_EHIP, ST_ENODEV, ST_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
ST_FP32, ST_FP16, ST_BF16 = 0, 1, 2
STATUS_NAMES = {0: "ST_OK", -1: "ST_EINVAL", -2: "ST_ENOMEM", -3: "ST_EHIP", -4: "ST_ENODEV",
                -5: "ST_EUNSUPPORTED"}

# every symbol include/stereo.h declares
EXPORTS = ("st_default_params", "st_create", "st_destroy", "st_last_error", "stereo_match",
           "stereo_match_batched", "stereo_refine_forward", "stereo_refine_backward",
           "stereo_refine_step", "stereo_debug_get", "st_window_stats", "st_match_wta",
           "st_subpixel", "st_lr_check", "st_radial_outlier", "st_fill", "st_hc_smooth", "st_reproject", "st_research",
           "st_autotune", "st_set_variant", "st_num_variants", "st_variant_name", "st_version",
           "stereo_time_matcher", "stereo_match_noalloc", "st_autotune_batched",
           "st_batch_variant")


class StereoError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class st_params(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("subpixel", C.c_int32), ("lr_check", C.c_int32),
                ("lr_tol", C.c_int32), ("radial_iters", C.c_int32), ("radial_r0", C.c_int32),
                ("radial_dr", C.c_int32), ("radial_thresh", C.c_float),
                ("fill_radial_r", C.c_int32), ("fill_min_lines", C.c_int32),
                ("fill_disk_r", C.c_int32), ("fill_disk_min_frac", C.c_float),
                ("smooth_radius", C.c_int32), ("smooth_iters", C.c_int32),
                ("smooth_alpha", C.c_float), ("precision", C.c_int32),
                ("debug_outputs", C.c_int32), ("research", C.c_int32),
                ("research_range", C.c_int32), ("research_eta", C.c_float),
                ("chessboard", C.c_int32)]


class st_pair(C.Structure):
    _fields_ = [("left", C.c_void_p), ("right", C.c_void_p), ("H", C.c_int32), ("W", C.c_int32),
                ("pitch", C.c_int32), ("dmin", C.c_int32), ("dmax", C.c_int32),
                ("win", C.c_int32), ("disparity", C.c_void_p), ("valid_mask", C.c_void_p)]


_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        # torch ships its own HIP runtime under the same soname as the ROCm
        # one the library was linked against: loading torch first makes the
        # library bind to that runtime, so the process holds one HIP runtime
        # (with the ROCm copy loaded first, torch then finds no GPU)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, f32 = C.c_void_p, C.c_int, C.c_float
        sig = {
            "st_default_params": (None, [C.POINTER(st_params)]),
            "st_create": (i32, [C.POINTER(vp), i32]),
            "st_destroy": (None, [vp]),
            "st_last_error": (C.c_char_p, []),
            "st_version": (C.c_char_p, []),
            "stereo_match": (i32, [vp, vp, vp, i32, i32, i32, i32, i32, i32,
                                   C.POINTER(st_params), vp, vp, vp]),
            "stereo_match_noalloc": (i32, [vp, vp, vp, i32, i32, i32, i32, i32, i32,
                                           C.POINTER(st_params), vp, vp, vp]),
            "stereo_match_batched": (i32, [vp, C.POINTER(st_pair), i32, C.POINTER(st_params), vp]),
            "stereo_refine_forward": (i32, [vp, vp, vp, vp, vp, i32, i32, i32, i32, f32, vp, vp, vp]),
            "stereo_refine_backward": (i32, [vp, vp, vp, vp, vp, i32, i32, i32, i32, f32, vp, vp]),
            "stereo_refine_step": (i32, [vp, vp, vp, vp, i32, i32, f32, f32, vp]),
            "stereo_debug_get": (i32, [vp, C.c_char_p, C.POINTER(vp)]),
            "st_window_stats": (i32, [vp, vp, i32, i32, i32, i32, i32, vp, vp, vp, vp]),
            "st_match_wta": (i32, [vp, vp, vp] + [i32] * 8 + [vp, vp, vp, vp, vp]),
            "st_subpixel": (i32, [vp, vp, vp] + [i32] * 7 + [vp, vp, vp, vp, vp, vp, vp]),
            "st_lr_check": (i32, [vp, vp, vp, vp, vp, i32, i32, i32, vp, vp]),
            "st_radial_outlier": (i32, [vp, vp, vp, i32, i32, i32, f32, vp, vp]),
            "st_fill": (i32, [vp, vp, vp, i32, i32, i32, i32, i32, f32, vp, vp, vp]),
            "st_hc_smooth": (i32, [vp, vp, vp, i32, i32, i32, i32, f32, vp, vp]),
            "st_reproject": (i32, [vp, vp, i32, i32, vp, vp, vp]),
            "st_research": (i32, [vp, vp, vp] + [i32] * 7 + [vp, vp, vp, i32, f32, vp, vp]),
            "st_autotune": (i32, [vp, i32, i32, i32, i32, i32, i32, C.POINTER(i32), vp]),
            "st_set_variant": (i32, [vp, i32]),
            "st_autotune_batched": (i32, [vp, C.POINTER(st_pair), i32, C.POINTER(st_params), i32,
                                          C.POINTER(i32), vp]),
            "st_batch_variant": (i32, [vp, i32]),
            "stereo_time_matcher": (i32, [vp, C.POINTER(st_pair), i32, C.POINTER(st_params), i32,
                                          C.POINTER(C.c_float), vp]),
            "st_num_variants": (i32, []),
            "st_variant_name": (C.c_char_p, [i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def st_last_error() -> str:
    return lib().st_last_error().decode()


def _check(rc: int) -> None:
    if rc != ST_OK:
        raise StereoError(rc, st_last_error())


def st_default_params(**overrides) -> st_params:
    p = st_params()
    lib().st_default_params(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def preset(name: str, **overrides) -> st_params:
    """Parameter sets of the standard workloads.
    small: 320x240 / 7x7 - LR check, one fill pass, 5x5 smoothing (R=2, K=1);
    full:  960x540 / 11x11 - 3 outlier/fill alternations (r = 10, 20, 30),
           smoothing radius 15, K = 3 (the paper's constants)."""
    if name == "small":
        base = dict(radial_iters=0, smooth_radius=2, smooth_iters=1)
    elif name == "full":
        base = {}
    else:
        raise ValueError(name)
    base.update(overrides)
    return st_default_params(**base)


def _stream(stream=None) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _p(t) -> int | None:
    return None if t is None else t.data_ptr()


class Handle:
    """Owns an st_handle (device scratch, tuning table, batched graph)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().st_create(C.byref(h), device))
        self.h = h

    def close(self):
        if self.h:
            lib().st_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    @property
    def value(self):
        return self.h


_default = None


def default_handle() -> Handle:
    global _default
    if _default is None:
        _default = Handle(0)
    return _default


def _h(handle):
    return (handle or default_handle()).h


# ---------------------------------------------------------------- whole path
def stereo_match(left, right, dmin, dmax, win, params=None, disparity=None, valid_mask=None,
                 handle=None, stream=None):
    """left/right: uint8 (H, W) device tensors (row pitch = stride(0))."""
    import torch
    assert left.dtype == torch.uint8 and right.dtype == torch.uint8 and left.is_cuda
    assert left.shape == right.shape and left.stride() == right.stride() and left.stride(1) == 1
    H, W = left.shape
    if params is None:
        params = st_default_params()
    if disparity is None:
        disparity = torch.empty((H, W), dtype=torch.float32, device=left.device)
    if valid_mask is None:
        valid_mask = torch.empty((H, W), dtype=torch.uint8, device=left.device)
    _check(lib().stereo_match(_h(handle), left.data_ptr(), right.data_ptr(), H, W, left.stride(0),
                              dmin, dmax, win, C.byref(params), disparity.data_ptr(),
                              valid_mask.data_ptr(), _stream(stream)))
    return disparity, valid_mask


def stereo_match_noalloc(left, right, dmin, dmax, win, params, disparity, valid_mask,
                         handle=None, stream=None):
    """stereo_match with every intermediate in the library's fixed per-GPU
    scratch array (no device allocation); the outputs must be given."""
    import torch
    assert left.dtype == torch.uint8 and right.dtype == torch.uint8 and left.is_cuda
    assert left.shape == right.shape and left.stride() == right.stride() and left.stride(1) == 1
    H, W = left.shape
    _check(lib().stereo_match_noalloc(_h(handle), left.data_ptr(), right.data_ptr(), H, W,
                                      left.stride(0), dmin, dmax, win, C.byref(params),
                                      disparity.data_ptr(), valid_mask.data_ptr(),
                                      _stream(stream)))
    return disparity, valid_mask


def stereo_match_batched(pairs, params=None, handle=None, stream=None):
    """pairs: list of dicts with left, right (uint8 device tensors), dmin, dmax,
    win and optional disparity / valid_mask outputs.  Returns the outputs."""
    if params is None:
        params = st_default_params()
    arr, outs = _pair_array(pairs)
    _check(lib().stereo_match_batched(_h(handle), arr, len(pairs), C.byref(params),
                                      _stream(stream)))
    return outs


def _pair_array(pairs):
    import torch
    arr = (st_pair * len(pairs))()
    outs = []
    for i, q in enumerate(pairs):
        L, R = q["left"], q["right"]
        H, W = L.shape
        d = q.get("disparity")
        m = q.get("valid_mask")
        if d is None:
            d = torch.empty((H, W), dtype=torch.float32, device=L.device)
            q["disparity"] = d
        if m is None:
            m = torch.empty((H, W), dtype=torch.uint8, device=L.device)
            q["valid_mask"] = m
        arr[i] = st_pair(L.data_ptr(), R.data_ptr(), H, W, L.stride(0), q["dmin"], q["dmax"],
                         q["win"], d.data_ptr(), m.data_ptr())
        outs.append((d, m))
    return arr, outs


def stereo_time_matcher(pairs, params=None, reps=10, handle=None, stream=None) -> float:
    """Average ms of the batched matcher kernel alone (HIP events on the stream).
    Output tensors are attached to the pair dicts on first use."""
    if params is None:
        params = st_default_params()
    arr, _ = _pair_array(pairs)
    ms = C.c_float(0.0)
    _check(lib().stereo_time_matcher(_h(handle), arr, len(pairs), C.byref(params), reps,
                                     C.byref(ms), _stream(stream)))
    return ms.value


def stereo_debug_get(name, shape, dtype, handle=None):
    """Copy of a debug intermediate of the last debug stereo_match call."""
    import torch
    ptr = C.c_void_p()
    _check(lib().stereo_debug_get(_h(handle), name.encode(), C.byref(ptr)))
    out = torch.empty(shape, dtype=dtype, device="cuda")
    nbytes = out.numel() * out.element_size()
    # device-to-device copy of the handle-owned buffer through the HIP runtime
    torch.cuda.current_stream().synchronize()
    hip = _hip_runtime()
    rc = hip.hipMemcpy(C.c_void_p(out.data_ptr()), ptr, C.c_size_t(nbytes), 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    return _hip


# ---------------------------------------------------------------- stages
def st_window_stats(img, win, chess=False, handle=None, stream=None):
    import torch
    H, W = img.shape
    S = torch.empty((H, W), dtype=torch.int32, device=img.device)
    SS = torch.empty_like(S)
    inv = torch.empty((H, W), dtype=torch.float32, device=img.device)
    _check(lib().st_window_stats(_h(handle), img.data_ptr(), H, W, img.stride(0), win, int(chess),
                                 S.data_ptr(), SS.data_ptr(), inv.data_ptr(), _stream(stream)))
    return S, SS, inv


def st_match_wta(left, right, dmin, dmax, win, precision=ST_FP32, chess=False, handle=None,
                 stream=None):
    import torch
    H, W = left.shape
    dev = left.device
    oL = torch.empty((H, W), dtype=torch.int16, device=dev)
    oR = torch.empty_like(oL)
    mL = torch.empty((H, W), dtype=torch.uint8, device=dev)
    mR = torch.empty_like(mL)
    _check(lib().st_match_wta(_h(handle), left.data_ptr(), right.data_ptr(), H, W, left.stride(0),
                              dmin, dmax, win, int(chess), precision, oL.data_ptr(), mL.data_ptr(),
                              oR.data_ptr(), mR.data_ptr(), _stream(stream)))
    return oL, mL, oR, mR


def st_subpixel(left, right, dmin, dmax, win, oL, mL, chess=False, handle=None, stream=None):
    import torch
    H, W = left.shape
    dev = left.device
    zb = torch.empty((H, W), dtype=torch.float64, device=dev)
    zm = torch.empty_like(zb)
    zp = torch.empty_like(zb)
    dl = torch.empty((H, W), dtype=torch.float32, device=dev)
    _check(lib().st_subpixel(_h(handle), left.data_ptr(), right.data_ptr(), H, W, left.stride(0),
                             dmin, dmax, win, int(chess), oL.data_ptr(), mL.data_ptr(), zb.data_ptr(),
                             zm.data_ptr(), zp.data_ptr(), dl.data_ptr(), _stream(stream)))
    return zb, zm, zp, dl


def st_lr_check(oL, mL, oR, mR, tol=1, handle=None, stream=None):
    import torch
    H, W = oL.shape
    out = torch.empty((H, W), dtype=torch.uint8, device=oL.device)
    _check(lib().st_lr_check(_h(handle), oL.data_ptr(), mL.data_ptr(), oR.data_ptr(),
                             mR.data_ptr(), H, W, tol, out.data_ptr(), _stream(stream)))
    return out


def st_radial_outlier(o, m, r, thresh=2.5, handle=None, stream=None):
    import torch
    H, W = o.shape
    out = torch.empty((H, W), dtype=torch.uint8, device=o.device)
    _check(lib().st_radial_outlier(_h(handle), o.data_ptr(), m.data_ptr(), H, W, r, thresh,
                                   out.data_ptr(), _stream(stream)))
    return out


def st_fill(o, m, radial_r=50, min_lines=2, disk_r=20, min_frac=0.25, handle=None, stream=None):
    import torch
    H, W = o.shape
    oo = torch.empty_like(o)
    mo = torch.empty_like(m)
    _check(lib().st_fill(_h(handle), o.data_ptr(), m.data_ptr(), H, W, radial_r, min_lines,
                         disk_r, min_frac, oo.data_ptr(), mo.data_ptr(), _stream(stream)))
    return oo, mo


def st_hc_smooth(s, m, R, K, alpha=0.1, handle=None, stream=None):
    import torch
    H, W = s.shape
    out = torch.empty((H, W), dtype=torch.float32, device=s.device)
    _check(lib().st_hc_smooth(_h(handle), s.data_ptr(), m.data_ptr(), H, W, R, K, alpha,
                              out.data_ptr(), _stream(stream)))
    return out


def st_research(left, right, dmin, dmax, win, o, m, d, range_=5, eta=0.01, chess=False,
                handle=None, stream=None):
    """One Eq. (4) re-search: new int16 disparities around d (float64)."""
    import torch
    H, W = left.shape
    out = torch.empty_like(o)
    _check(lib().st_research(_h(handle), left.data_ptr(), right.data_ptr(), H, W, left.stride(0),
                             dmin, dmax, win, int(chess), o.data_ptr(), m.data_ptr(), d.data_ptr(), range_,
                             eta, out.data_ptr(), _stream(stream)))
    return out


def st_reproject(disparity, Q, handle=None, stream=None):
    """Disparity map (H x W float, device) -> H x W x 3 points with the 4x4
    reprojection matrix Q (any array-like of 16 numbers, row-major)."""
    import torch
    H, W = disparity.shape
    qv = np.asarray(Q, dtype=np.float64).ravel()
    if qv.size != 16:
        raise ValueError("Q must hold 16 numbers")
    q = (C.c_double * 16)(*qv.tolist())
    xyz = torch.empty((H, W, 3), dtype=torch.float32, device=disparity.device)
    _check(lib().st_reproject(_h(handle), disparity.data_ptr(), H, W, q, xyz.data_ptr(),
                              _stream(stream)))
    return xyz


def st_autotune(H, W, dmin, dmax, win, precision=ST_FP32, handle=None, stream=None) -> int:
    best = C.c_int(-1)
    _check(lib().st_autotune(_h(handle), H, W, dmin, dmax, win, precision, C.byref(best),
                             _stream(stream)))
    return best.value


def st_autotune_batched(pairs, params=None, reps=3, handle=None, stream=None) -> list:
    """Tune the persistent launch of every window size of this batch layout;
    returns the variant chosen for each pair."""
    if params is None:
        params = st_default_params()
    arr, _ = _pair_array(pairs)
    best = (C.c_int * len(pairs))()
    _check(lib().st_autotune_batched(_h(handle), arr, len(pairs), C.byref(params), reps, best,
                                     _stream(stream)))
    return list(best)


def st_batch_variant(win: int, handle=None) -> int:
    return lib().st_batch_variant(_h(handle), win)


def st_set_variant(variant: int, handle=None) -> None:
    _check(lib().st_set_variant(_h(handle), variant))


def st_num_variants() -> int:
    return lib().st_num_variants()


def st_variant_name(v: int) -> str:
    return lib().st_variant_name(v).decode()


# ---------------------------------------------------------------- refinement
def stereo_refine_forward(left, right, d, mask, win, lam=0.1, want_z=False, handle=None,
                          stream=None):
    import torch
    H, W = left.shape
    E = torch.empty((), dtype=torch.float64, device=left.device)
    Z = torch.empty((H, W), dtype=torch.float32, device=left.device) if want_z else None
    _check(lib().stereo_refine_forward(_h(handle), left.data_ptr(), right.data_ptr(), d.data_ptr(),
                                       mask.data_ptr(), H, W, left.stride(0), win, lam, _p(Z),
                                       E.data_ptr(), _stream(stream)))
    return (E, Z) if want_z else E


def stereo_refine_backward(left, right, d, mask, win, lam=0.1, handle=None, stream=None):
    import torch
    H, W = left.shape
    g = torch.empty((H, W), dtype=torch.float32, device=left.device)
    _check(lib().stereo_refine_backward(_h(handle), left.data_ptr(), right.data_ptr(),
                                        d.data_ptr(), mask.data_ptr(), H, W, left.stride(0), win,
                                        lam, g.data_ptr(), _stream(stream)))
    return g


def stereo_refine_step(d, g, mask, tau=0.05, max_step=0.25, handle=None, stream=None):
    H, W = d.shape
    _check(lib().stereo_refine_step(_h(handle), d.data_ptr(), g.data_ptr(), mask.data_ptr(), H, W,
                                    tau, max_step, _stream(stream)))
    return d


def _refine_fn():
    import torch

    class RefineZNCC(torch.autograd.Function):
        """E(d) = sum_Omega (1 - ZNCC) + lambda TV(d); backward by the hand-written kernel."""

        @staticmethod
        def forward(ctx, d, left, right, mask, win, lam, handle=None):
            d = d.contiguous()
            ctx.save_for_backward(d, left, right, mask)
            ctx.win, ctx.lam, ctx.handle = win, lam, handle
            return stereo_refine_forward(left, right, d, mask, win, lam, handle=handle)

        @staticmethod
        def backward(ctx, gE):
            d, left, right, mask = ctx.saved_tensors
            g = stereo_refine_backward(left, right, d, mask, ctx.win, ctx.lam, handle=ctx.handle)
            return g * gE.to(g.dtype), None, None, None, None, None, None

    return RefineZNCC


_RefineZNCC = None


def RefineZNCC():
    """The torch.autograd.Function class (created on first use)."""
    global _RefineZNCC
    if _RefineZNCC is None:
        _RefineZNCC = _refine_fn()
    return _RefineZNCC


def refine(left, right, d0, mask, win, steps=20, lam=0.1, tau=0.05, max_step=0.25, handle=None):
    """Clamped gradient descent on the refinement energy; returns (d, energies)."""
    d = d0.clone()
    energies = []
    for _ in range(steps):
        E = stereo_refine_forward(left, right, d, mask, win, lam, handle=handle)
        g = stereo_refine_backward(left, right, d, mask, win, lam, handle=handle)
        energies.append(E)
        stereo_refine_step(d, g, mask, tau, max_step, handle=handle)
    return d, energies
