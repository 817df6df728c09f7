"""Pins of the refinement energy: closed form, autograd and finite differences."""
import numpy as np
import pytest

from oracle import refine_autograd as ra


def _pair(seed, H=24, W=40, k=4):
    r = np.random.default_rng(seed)
    wide = r.integers(0, 256, size=(H, W + k), dtype=np.uint8)
    L = np.ascontiguousarray(wide[:, :W])   # L(x) = R(x - k)
    R = np.ascontiguousarray(wide[:, k:])
    return L, R


def test_energy_zero_for_exact_integer_shift(orc):
    L, R = _pair(1)
    H, W = L.shape
    d = np.full((H, W), 4.0)
    valid = np.ones((H, W), np.uint8)
    valid[:, :8] = 0   # where x - 4 would leave the image the warp is clamped
    E = orc.refine_energy(L, R, d, valid, 5, lam=0.1)
    assert abs(E) < 1e-9


def test_energy_tv_closed_form(orc):
    L, R = _pair(2)
    H, W = L.shape
    r = np.random.default_rng(3)
    d = r.normal(3.0, 1.0, size=(H, W))
    valid = (r.random((H, W)) > 0.3).astype(np.uint8)
    # window larger than the image: Omega is empty, E = lambda * TV
    E = orc.refine_energy(L, R, d, valid, 41, lam=0.5)
    tv = 0.0
    for y in range(H):
        for x in range(W):
            if not valid[y, x]:
                continue
            if x + 1 < W and valid[y, x + 1]:
                tv += abs(d[y, x + 1] - d[y, x])
            if y + 1 < H and valid[y + 1, x]:
                tv += abs(d[y + 1, x] - d[y, x])
    assert E == pytest.approx(0.5 * tv, rel=1e-14)


def test_energy_matches_autograd_value(orc):
    L, R = _pair(4)
    H, W = L.shape
    r = np.random.default_rng(5)
    d = 4.0 + r.uniform(-0.8, 0.8, size=(H, W))
    valid = np.ones((H, W), np.uint8)
    valid[:, :7] = 0
    valid[r.random((H, W)) < 0.05] = 0
    E_c = orc.refine_energy(L, R, d, valid, 5, lam=0.1)
    E_t, _ = ra.energy_and_grad(L, R, d, valid, 5, lam=0.1)
    assert E_c == pytest.approx(E_t, rel=1e-12, abs=1e-10)


def test_autograd_gradient_matches_central_differences(orc):
    L, R = _pair(6)
    H, W = L.shape
    r = np.random.default_rng(7)
    d = 4.0 + r.uniform(-0.8, 0.8, size=(H, W))
    valid = np.ones((H, W), np.uint8)
    valid[:, :7] = 0
    lam, win, hstep = 0.1, 5, 1e-3
    _, g = ra.energy_and_grad(L, R, d, valid, win, lam=lam)
    checked = 0
    for (y, x) in zip(r.integers(3, H - 3, 60), r.integers(9, W - 3, 60)):
        u = x - d[y, x]
        if abs(u - round(u)) < 2 * hstep:
            continue  # lerp kink
        nb = [d[y, x + 1], d[y, x - 1], d[y + 1, x], d[y - 1, x]]
        if any(abs(v - d[y, x]) < 2 * hstep for v in nb):
            continue  # TV kink
        dp = d.copy(); dp[y, x] += hstep
        dm = d.copy(); dm[y, x] -= hstep
        fd = (orc.refine_energy(L, R, dp, valid, win, lam) -
              orc.refine_energy(L, R, dm, valid, win, lam)) / (2 * hstep)
        assert g[y, x] == pytest.approx(fd, rel=1e-5, abs=1e-7)
        checked += 1
    assert checked > 30


def test_local_energy_differences_equal_global(orc):
    L, R = _pair(8)
    H, W = L.shape
    r = np.random.default_rng(9)
    d = 4.0 + r.uniform(-0.8, 0.8, size=(H, W))
    valid = np.ones((H, W), np.uint8)
    valid[:, :7] = 0
    valid[r.random((H, W)) < 0.05] = 0
    for (y, x) in zip(r.integers(0, H, 25), r.integers(0, W, 25)):
        dp = d.copy(); dp[y, x] += 0.01
        dm = d.copy(); dm[y, x] -= 0.013
        g = orc.refine_energy(L, R, dp, valid, 5, 0.1) - orc.refine_energy(L, R, dm, valid, 5, 0.1)
        lo = (orc.refine_energy_local(L, R, dp, valid, 5, 0.1, x, y) -
              orc.refine_energy_local(L, R, dm, valid, 5, 0.1, x, y))
        assert lo == pytest.approx(g, abs=1e-9)
