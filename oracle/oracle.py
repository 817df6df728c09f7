"""Python access to the CPU oracle (``stereo_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product path.  Argument
marshalling only; every step is computed in the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "stereo_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over rows/disparities)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp",
                               "-shared", "-fPIC", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _setup(_lib)
    return _lib


P = np.ctypeslib.ndpointer
u8 = P(dtype=np.uint8, flags="C_CONTIGUOUS")
i32 = P(dtype=np.int32, flags="C_CONTIGUOUS")
i64 = P(dtype=np.int64, flags="C_CONTIGUOUS")
f64 = P(dtype=np.float64, flags="C_CONTIGUOUS")


class Params(C.Structure):
    _fields_ = [("subpixel", C.c_int32), ("lr_check", C.c_int32), ("lr_tol", C.c_int32),
                ("radial_iters", C.c_int32), ("radial_r0", C.c_int32), ("radial_dr", C.c_int32),
                ("radial_thresh", C.c_double), ("fill_radial_r", C.c_int32),
                ("fill_min_lines", C.c_int32), ("fill_disk_r", C.c_int32),
                ("fill_disk_frac", C.c_double), ("smooth_radius", C.c_int32),
                ("smooth_iters", C.c_int32), ("smooth_alpha", C.c_double),
                ("research", C.c_int32), ("research_range", C.c_int32),
                ("research_eta", C.c_double), ("chess", C.c_int32)]


def params_c1(**kw):
    """320x240 setting: LR check, one fill pass, 5x5 (R=2) smoothing, K=1."""
    p = dict(subpixel=1, lr_check=1, lr_tol=1, radial_iters=0, radial_r0=10, radial_dr=10,
             radial_thresh=2.5, fill_radial_r=50, fill_min_lines=2, fill_disk_r=20,
             fill_disk_frac=0.25, smooth_radius=2, smooth_iters=1, smooth_alpha=0.1, research=0,
             research_range=5, research_eta=0.01, chess=0)
    p.update(kw)
    return Params(**p)


def params_c2(**kw):
    """Full pipeline: 3 outlier/fill alternations r=10,20,30, R=15, K=3."""
    p = dict(subpixel=1, lr_check=1, lr_tol=1, radial_iters=3, radial_r0=10, radial_dr=10,
             radial_thresh=2.5, fill_radial_r=50, fill_min_lines=2, fill_disk_r=20,
             fill_disk_frac=0.25, smooth_radius=15, smooth_iters=3, smooth_alpha=0.1, research=0,
             research_range=5, research_eta=0.01, chess=0)
    p.update(kw)
    return Params(**p)


def _setup(L):
    L.or_window_stats.argtypes = [u8] + [C.c_int] * 6 + [i64, i64, i64, u8]
    L.or_window_stats.restype = C.c_int
    L.or_zncc_windows.argtypes = [u8, u8, C.c_int]
    L.or_zncc_windows.restype = C.c_double
    L.or_match.argtypes = [u8, u8] + [C.c_int] * 10 + [i32, u8, f64, f64, f64, f64, i32, u8, f64, f64]
    L.or_match.restype = C.c_int
    L.or_subpixel.argtypes = [C.c_int64, i32, u8, f64, f64, f64, C.c_int, C.c_int, f64]
    L.or_subpixel.restype = None
    L.or_lr_check.argtypes = [C.c_int, C.c_int, i32, u8, i32, u8, C.c_int, u8]
    L.or_lr_check.restype = None
    L.or_radial_outlier.argtypes = [C.c_int, C.c_int, i32, u8, C.c_int, C.c_double, u8]
    L.or_radial_outlier.restype = None
    L.or_fill.argtypes = [C.c_int, C.c_int, i32, u8, C.c_int, C.c_int, C.c_int, C.c_double]
    L.or_fill.restype = C.c_int
    L.or_hc_smooth.argtypes = [C.c_int, C.c_int, f64, u8, C.c_int, C.c_int, C.c_double, f64]
    L.or_hc_smooth.restype = C.c_int
    L.or_research.argtypes = [u8, u8] + [C.c_int] * 7 + [i32, u8, f64, C.c_int, C.c_double, i32]
    L.or_research.restype = None
    L.or_hc_research.argtypes = ([u8, u8] + [C.c_int] * 7 + [i32, u8, C.c_int, C.c_int, C.c_double,
                                                             C.c_double, C.c_int, C.c_void_p, f64])
    L.or_hc_research.restype = C.c_int
    L.or_reproject.argtypes = [C.c_int, C.c_int, f64, f64, f64]
    L.or_reproject.restype = None
    vp = C.c_void_p
    L.or_pipeline.argtypes = [u8, u8] + [C.c_int] * 6 + [C.POINTER(Params), f64, u8,
                                                          vp, vp, vp, vp, vp]
    L.or_pipeline.restype = C.c_int
    L.or_refine_energy.argtypes = [u8, u8, C.c_int, C.c_int, C.c_int, C.c_int, f64, u8,
                                   C.c_double, vp]
    L.or_refine_energy.restype = C.c_double
    L.or_refine_energy_local.argtypes = [u8, u8, C.c_int, C.c_int, C.c_int, C.c_int, f64, u8,
                                         C.c_double, C.c_int, C.c_int]
    L.or_refine_energy_local.restype = C.c_double


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def window_stats(img, win, brute=False, chess=False):
    img = _c(img, np.uint8)
    H, W = img.shape
    S = np.zeros((H, W), np.int64); SS = np.zeros_like(S); V = np.zeros_like(S)
    ins = np.zeros((H, W), np.uint8)
    rc = lib().or_window_stats(img, H, W, W, win, int(brute), int(chess), S, SS, V, ins)
    assert rc == 0, rc
    return S, SS, V, ins


def zncc_windows(a, b):
    a = _c(a, np.uint8).ravel(); b = _c(b, np.uint8).ravel()
    assert a.size == b.size
    return lib().or_zncc_windows(a, b, a.size)


def match(left, right, dmin, dmax, win, rows=None, brute=False, chess=False):
    """Cost volume + WTA for rows [y0, y1) (default all rows)."""
    L = _c(left, np.uint8); R = _c(right, np.uint8)
    H, W = L.shape
    y0, y1 = (0, H) if rows is None else rows
    n = (y1 - y0, W)
    out = dict(oL=np.zeros(n, np.int32), mL=np.zeros(n, np.uint8), zbest=np.zeros(n),
               gap=np.zeros(n), zm=np.zeros(n), zp=np.zeros(n), oR=np.zeros(n, np.int32),
               mR=np.zeros(n, np.uint8), zbestR=np.zeros(n), gapR=np.zeros(n))
    rc = lib().or_match(L, R, H, W, W, dmin, dmax, win, y0, y1, int(brute), int(chess), out["oL"],
                        out["mL"], out["zbest"], out["gap"], out["zm"], out["zp"], out["oR"],
                        out["mR"], out["zbestR"], out["gapR"])
    assert rc == 0, rc
    return out


def subpixel(o, m, zm, z0, zp, dmin, dmax):
    o = _c(o, np.int32); m = _c(m, np.uint8)
    zm = _c(zm, np.float64); z0 = _c(z0, np.float64); zp = _c(zp, np.float64)
    out = np.zeros(o.shape, np.float64)
    lib().or_subpixel(o.size, o, m, zm, z0, zp, dmin, dmax, out)
    return out


def lr_check(oL, mL, oR, mR, tol=1):
    oL = _c(oL, np.int32); oR = _c(oR, np.int32); mL = _c(mL, np.uint8); mR = _c(mR, np.uint8)
    H, W = oL.shape
    out = np.zeros((H, W), np.uint8)
    lib().or_lr_check(H, W, oL, mL, oR, mR, tol, out)
    return out


def radial_outlier(o, m, r, thresh=2.5):
    o = _c(o, np.int32); m = _c(m, np.uint8)
    H, W = o.shape
    out = np.zeros((H, W), np.uint8)
    lib().or_radial_outlier(H, W, o, m, r, thresh, out)
    return out


def fill(o, m, radial_r=50, min_lines=2, disk_r=20, min_frac=0.25):
    o = _c(o, np.int32).copy(); m = _c(m, np.uint8).copy()
    H, W = o.shape
    rc = lib().or_fill(H, W, o, m, radial_r, min_lines, disk_r, min_frac)
    assert rc == 0, rc
    return o, m


def hc_smooth(s, m, R, K, alpha=0.1):
    s = _c(s, np.float64); m = _c(m, np.uint8)
    H, W = s.shape
    out = np.zeros((H, W), np.float64)
    rc = lib().or_hc_smooth(H, W, s, m, R, K, alpha, out)
    assert rc == 0, rc
    return out


def research(left, right, dmin, dmax, win, o, m, d, range_=5, eta=0.01, chess=False):
    """One Eq. (4) re-search of every valid pixel around d (float64 H x W)."""
    L = _c(left, np.uint8); R = _c(right, np.uint8)
    H, W = L.shape
    out = np.zeros((H, W), np.int32)
    lib().or_research(L, R, H, W, W, win, int(chess), dmin, dmax, _c(o, np.int32), _c(m, np.uint8),
                      _c(d, np.float64), range_, eta, out)
    return out


def hc_research(left, right, dmin, dmax, win, o, m, R, K, alpha=0.1, eta=0.01, range_=5,
                chess=False, d_init=None):
    """Eqs. (1)-(4): returns (d^K, final o).  d_init: d^0 (default o)."""
    L = _c(left, np.uint8); Rr = _c(right, np.uint8)
    H, W = L.shape
    oo = _c(o, np.int32).copy()
    out = np.zeros((H, W), np.float64)
    di = None if d_init is None else _c(d_init, np.float64)
    rc = lib().or_hc_research(L, Rr, H, W, W, win, int(chess), dmin, dmax, oo, _c(m, np.uint8), R, K, alpha,
                              eta, range_, None if di is None else di.ctypes.data, out)
    assert rc == 0, rc
    return out, oo


def reproject(disp, Q):
    """H x W disparities (NaN = invalid) -> H x W x 3 points, Q 4x4 row-major."""
    d = _c(disp, np.float64)
    H, W = d.shape
    q = _c(np.asarray(Q, dtype=np.float64).reshape(16), np.float64)
    out = np.zeros((H, W, 3), np.float64)
    lib().or_reproject(H, W, d, q, out)
    return out


def pipeline(left, right, dmin, dmax, win, params, intermediates=False):
    L = _c(left, np.uint8); R = _c(right, np.uint8)
    H, W = L.shape
    disp = np.zeros((H, W), np.float64)
    mask = np.zeros((H, W), np.uint8)
    inter = None
    ptrs = [None] * 5
    if intermediates:
        inter = dict(o_wta=np.zeros((H, W), np.int32), m_wta=np.zeros((H, W), np.uint8),
                     delta=np.zeros((H, W), np.float64), o_post=np.zeros((H, W), np.int32),
                     m_lr=np.zeros((H, W), np.uint8))
        ptrs = [inter[k].ctypes.data for k in ("o_wta", "m_wta", "delta", "o_post", "m_lr")]
    rc = lib().or_pipeline(L, R, H, W, W, dmin, dmax, win, C.byref(params), disp, mask, *ptrs)
    assert rc == 0, rc
    if intermediates:
        return disp, mask, inter
    return disp, mask


def refine_energy(left, right, d, valid, win, lam=0.1, want_z=False):
    L = _c(left, np.uint8); R = _c(right, np.uint8)
    H, W = L.shape
    d = _c(d, np.float64); v = _c(valid, np.uint8)
    Z = np.zeros((H, W), np.float64) if want_z else None
    E = lib().or_refine_energy(L, R, H, W, W, win, d, v, lam,
                               Z.ctypes.data if want_z else None)
    return (E, Z) if want_z else E


def refine_energy_local(left, right, d, valid, win, lam, qx, qy):
    """Terms of the refinement energy that depend on d(qy, qx)."""
    L = _c(left, np.uint8); R = _c(right, np.uint8)
    H, W = L.shape
    return lib().or_refine_energy_local(L, R, H, W, W, win, _c(d, np.float64),
                                        _c(valid, np.uint8), lam, int(qx), int(qy))
