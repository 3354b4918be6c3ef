"""Comparison helpers of the GPU-vs-oracle parity tests.

Both implementations emit, per path sample, an FNV-1a hash of the sequence of
discrete decisions (faces hit, occlusion codes, environment texels, lobes,
terminations).  A pixel whose samples' hashes differ is a discrete-decision
flip (float32 against float64 landing on different sides of a comparison); it
is counted and excluded from the radiance comparison, and flipped samples are
masked out of both backward passes.
"""
import numpy as np

RAD_RTOL = 1e-4          # per-pixel relative tolerance of the radiance
GRAD_RTOL = 1e-3         # relative L2 tolerance of dV and dmat
FLIP_MAX = 1e-3          # largest admissible fraction of flipped pixels


def radiance_check(gpu_img, ora_img, flipped_pix, view_slices, rtol=RAD_RTOL):
    """gpu_img, ora_img: [npix, 3]; flipped_pix: bool [npix].  Returns (n_bad, n_checked, worst)."""
    g = np.asarray(gpu_img, np.float64)
    o = np.asarray(ora_img, np.float64)
    bad = 0
    worst = 0.0
    checked = 0
    for sl in view_slices:
        og, oo, fl = g[sl], o[sl], flipped_pix[sl]
        floor = 1e-3 * np.maximum(oo.mean(axis=0), 1e-12)
        scale = np.maximum(np.abs(oo), floor[None, :])
        err = np.abs(og - oo) / scale
        err = err[~fl]
        checked += err.shape[0]
        bad += int((err.max(axis=1) > rtol).sum()) if err.size else 0
        worst = max(worst, float(err.max()) if err.size else 0.0)
    return bad, checked, worst


def view_slices(cams):
    out, off = [], 0
    for c in cams:
        n = c.width * c.height
        out.append(slice(off, off + n))
        off += n
    return out


def rel_l2(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
