"""Helpers shared by the GPU tests (no arithmetic of the method)."""
import numpy as np


def cu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def np_(t):
    return t.detach().cpu().numpy()


def tie_mask(gap, thr=1e-5):
    """Pixels whose oracle top-2 gap is small enough for either answer."""
    g = np.where(np.isnan(gap), np.inf, gap)
    return g <= thr


def dilate(mask, r):
    """Square dilation by r pixels (r >= 0)."""
    if r <= 0:
        return mask.copy()
    from scipy.ndimage import maximum_filter
    return maximum_filter(mask.astype(np.uint8), size=2 * r + 1, mode="constant") > 0
