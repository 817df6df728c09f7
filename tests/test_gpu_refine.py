"""Differentiable refinement: energy against the FP64 oracle, gradient against
torch float64 autograd on the CPU and against central differences."""
import numpy as np
import pytest

from gpu_util import cu, np_
from paper_2007_12623_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2007_12623_amd import binding
    return binding


def _small(seed=5):
    r = np.random.default_rng(seed)
    p = synth.make_pair(48, 90, 15, seed)
    L, R = p["left"], p["right"]
    gt = p["gt_left"]
    d = np.where(np.isnan(gt), 5.0, gt) + r.uniform(-0.3, 0.3, size=L.shape)
    valid = (~np.isnan(gt)).astype(np.uint8)
    valid[r.random(L.shape) < 0.03] = 0
    return L, R, d.astype(np.float32), valid


@pytest.mark.parametrize("win,lam", [(5, 0.1), (7, 0.0), (11, 0.5)])
def test_forward_matches_oracle(B, orc, win, lam):
    L, R, d, v = _small()
    E, Z = B.stereo_refine_forward(cu(L), cu(R), cu(d), cu(v), win, lam, want_z=True)
    lam32 = float(np.float32(lam))   # the library takes lambda as a float
    Eo, Zo = orc.refine_energy(L, R, d.astype(np.float64), v, win, lam32, want_z=True)
    Zg = np_(Z)
    fin = ~np.isnan(Zo)
    assert np.array_equal(~np.isnan(Zg), fin)
    dz = np.abs(Zg[fin] - Zo[fin])
    k = int(np.argmax(dz))
    print(f"max |dZ| {dz.max():.3g} at {np.argwhere(fin)[k]}, Z {Zo[fin][k]:.9f}; "
          f"E {float(E.item()):.12g} vs {Eo:.12g}")
    np.testing.assert_allclose(Zg[fin], Zo[fin], atol=2e-7)
    assert float(E.item()) == pytest.approx(Eo, rel=1e-10, abs=1e-9)


@pytest.mark.parametrize("win,lam", [(5, 0.1), (7, 0.0), (11, 0.5)])
def test_backward_matches_autograd(B, win, lam):
    from oracle import refine_autograd as ra
    L, R, d, v = _small(6)
    g = np_(B.stereo_refine_backward(cu(L), cu(R), cu(d), cu(v), win, lam))
    _, gr = ra.energy_and_grad(L, R, d.astype(np.float64), v, win, float(np.float32(lam)))
    np.testing.assert_allclose(g, gr, rtol=1e-4, atol=1e-5)


def test_autograd_function(B):
    import torch
    L, R, d, v = _small(7)
    Lt, Rt, vt = cu(L), cu(R), cu(v)
    dt = cu(d).requires_grad_(True)
    E = B.RefineZNCC().apply(dt, Lt, Rt, vt, 7, 0.1)
    (2.0 * E).backward()
    g = B.stereo_refine_backward(Lt, Rt, cu(d), vt, 7, 0.1)
    torch.testing.assert_close(dt.grad, 2.0 * g)


def test_full_size_descent_with_finite_differences(B, orc):
    """960x540, from the plain path's o + delta on left-right-valid pixels:
    20 clamped steps; at steps 0, 10 and 19 the gradient at 256 seeded pixels
    (away from interpolation and |.| kinks) matches central differences
    (h = 1e-3) of the oracle's FP64 energy."""
    import torch
    seq = synth.c2_sequence(1)
    L, R = seq[0]["left"], seq[0]["right"]
    Lt, Rt = cu(L), cu(R)
    Hh, Ww = L.shape
    h = B.Handle(0)
    try:
        prm = B.preset("full", debug_outputs=1)
        B.stereo_match(Lt, Rt, 0, 127, 11, prm, handle=h)
        o = np_(B.stereo_debug_get("o_wta", (Hh, Ww), torch.int16, handle=h)).astype(np.float64)
        dl = np_(B.stereo_debug_get("delta", (Hh, Ww), torch.float32, handle=h)).astype(np.float64)
        mlr = np_(B.stereo_debug_get("m_lr", (Hh, Ww), torch.uint8, handle=h))
    finally:
        h.close()
    d = torch.tensor((o + dl).astype(np.float32), device="cuda")
    mask = cu(mlr)
    win, lam, hs = 11, 0.1, 1e-3
    r = np.random.default_rng(3003)
    energies = []
    checked = {}
    for step in range(20):
        E = B.stereo_refine_forward(Lt, Rt, d, mask, win, lam)
        g = B.stereo_refine_backward(Lt, Rt, d, mask, win, lam)
        energies.append(float(E.item()))
        if step in (0, 10, 19):
            dn = np_(d).astype(np.float64)
            gn = np_(g)
            n = 0
            tries = 0
            while n < 256 and tries < 20000:
                tries += 1
                y = int(r.integers(8, Hh - 8))
                x = int(r.integers(8, Ww - 8))
                if not mlr[y, x]:
                    continue
                # d(q) moves only q's own interpolation coordinate: keep it off integers
                u = x - dn[y, x]
                if abs(u - round(u)) < 2 * hs:
                    continue
                nb = [dn[y, x + 1], dn[y, x - 1], dn[y + 1, x], dn[y - 1, x]]
                if any(abs(a - dn[y, x]) < 2 * hs for a in nb):
                    continue
                dp = dn.copy(); dp[y, x] += hs
                dm = dn.copy(); dm[y, x] -= hs
                fd = (orc.refine_energy_local(L, R, dp, mlr, win, lam, x, y) -
                      orc.refine_energy_local(L, R, dm, mlr, win, lam, x, y)) / (2 * hs)
                assert gn[y, x] == pytest.approx(fd, rel=1e-3, abs=2e-4), (step, y, x)
                n += 1
            checked[step] = n
        B.stereo_refine_step(d, g, mask, 0.05, 0.25)
    assert all(v == 256 for v in checked.values()), checked
    assert energies[-1] < energies[0]
