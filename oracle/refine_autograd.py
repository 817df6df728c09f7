"""Reference gradient of the refinement energy by torch float64 autograd on CPU.

TEST INFRASTRUCTURE ONLY (imported by the tests, never by the product path).
It is a second, independent transcription of the energy that the C oracle
evaluates in ``or_refine_energy``:

  E(d) = sum_{p in Omega} (1 - Z_p(d)) + lambda * TV(d)

with R_w(q) the right row linearly interpolated at q_x - d(q) (clamped to
[0, W-1]; at an integer coordinate the right-hand segment is used, which is
torch's floor convention), Z_p the mean-form ZNCC of the left window and the
R_w window around p, Omega the valid pixels whose whole window is inside the
image, valid and of non-zero left variance, and TV the sum of absolute
forward differences over valid right/down neighbour pairs.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def omega_mask(left: np.ndarray, valid: np.ndarray, win: int) -> np.ndarray:
    """Pixels whose window is inside the image, all valid, non-flat on the left."""
    H, W = left.shape
    h = win // 2
    v = torch.from_numpy(valid.astype(np.float64))[None, None]
    cnt = F.avg_pool2d(v, win, stride=1) * (win * win)
    Lt = torch.from_numpy(left.astype(np.float64))[None, None]
    m = F.avg_pool2d(Lt, win, stride=1)
    m2 = F.avg_pool2d(Lt * Lt, win, stride=1)
    var = m2 - m * m
    ok = (cnt[0, 0] > win * win - 0.5) & (var[0, 0] > 1e-9)
    out = np.zeros((H, W), bool)
    out[h:H - h, h:W - h] = ok.numpy()
    return out & (valid != 0)


def energy_and_grad(left, right, d, valid, win, lam=0.1):
    """Return (E, dE/dd) in float64 for a float disparity field d."""
    H, W = left.shape
    h = win // 2
    n = win * win
    L = torch.from_numpy(left.astype(np.float64))
    R = torch.from_numpy(right.astype(np.float64))
    dt = torch.tensor(np.asarray(d, dtype=np.float64), requires_grad=True)
    xs = torch.arange(W, dtype=torch.float64)[None, :].expand(H, W)
    u = torch.clamp(xs - dt, 0.0, W - 1.0)
    i0 = torch.floor(u).detach()
    i0 = torch.clamp(i0, max=W - 1).long()
    i1 = torch.clamp(i0 + 1, max=W - 1)
    t = u - i0.to(torch.float64)
    r0 = torch.gather(R, 1, i0)
    r1 = torch.gather(R, 1, i1)
    rw = r0 * (1 - t) + r1 * t
    om = torch.from_numpy(omega_mask(left, valid, win))
    # windows around every interior pixel via unfold: (n, (H-2h)*(W-2h))
    a = F.unfold(L[None, None], win)[0]
    b = F.unfold(rw[None, None], win)[0]
    a = a - a.mean(0, keepdim=True)
    b = b - b.mean(0, keepdim=True)
    sab = (a * b).sum(0)
    saa = (a * a).sum(0)
    sbb = (b * b).sum(0)
    omi = om[h:H - h, h:W - h].reshape(-1)
    den = torch.sqrt(saa * sbb)
    safe = omi & (sbb > 0)
    z = torch.where(safe, sab / torch.where(safe, den, torch.ones_like(den)),
                    torch.zeros_like(den))
    E = (1.0 - z)[omi].sum()
    vt = torch.from_numpy(valid != 0)
    pr = vt[:, 1:] & vt[:, :-1]
    pd = vt[1:, :] & vt[:-1, :]
    tv = (dt[:, 1:] - dt[:, :-1]).abs()[pr].sum() + (dt[1:, :] - dt[:-1, :]).abs()[pd].sum()
    E = E + lam * tv
    E.backward()
    g = dt.grad.numpy().copy()
    return float(E.detach()), g
