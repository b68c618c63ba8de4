"""Comparison of GPU images with oracle images (float64, with every admissible
alternative where a threshold decision is within rounding of its boundary)."""
import numpy as np

RGB_TOL = 1e-3          # max-abs per channel, float32 path
DEPTH_REL = 1e-3        # |d - d_ref| <= 1e-3 * max(1, d_ref)
ALPHA_TOL = 1e-3        # max-abs of 1 - T


def _within(rgb, depth, alpha, r_rgb, r_depth, r_alpha, rgb_tol, depth_rel, alpha_tol):
    """Per-element test of one GPU pixel set against reference values."""
    ok = (np.abs(rgb - r_rgb).max(axis=-1) <= rgb_tol)
    ok &= np.abs(depth - r_depth) / np.maximum(1.0, np.abs(r_depth)) <= depth_rel
    if alpha is not None:
        ok &= np.abs(alpha - r_alpha) <= alpha_tol
    return ok


def compare(gpu_rgb, gpu_depth, ref, gpu_alpha=None, rgb_tol=RGB_TOL, depth_rel=DEPTH_REL, alpha_tol=ALPHA_TOL):
    """Every pixel must match the oracle's primary result (rgb, depth and, if
    given, alpha together); a pixel that does not, and whose primary run met a
    flagged threshold decision, must match one of its admissible variants,
    every one of which is enumerated (no pixel passes unchecked)."""
    gr = np.asarray(gpu_rgb, np.float64)
    gd = np.asarray(gpu_depth, np.float64)
    ga = None if gpu_alpha is None else np.asarray(gpu_alpha, np.float64)
    ok0 = _within(gr, gd, ga, ref.rgb, ref.depth, ref.alpha, rgb_tol, depth_rel, alpha_tol)
    flagged = ref.nflag > 0
    bad_calm = int((~ok0 & ~flagged).sum())
    by_variant, bad_flagged = 0, 0
    for y, x in zip(*np.nonzero(~ok0 & flagged)):
        vr, vd, va = ref.pixel_variants(x, y)
        okv = _within(gr[y, x][None], gd[y, x], None if ga is None else ga[y, x], vr, vd, va,
                      rgb_tol, depth_rel, alpha_tol)
        if okv.any():
            by_variant += 1
        else:
            bad_flagged += 1
    e_rgb = np.abs(gr - ref.rgb).max(axis=-1)
    e_dep = np.abs(gd - ref.depth) / np.maximum(1.0, np.abs(ref.depth))
    out = dict(
        ok=bad_calm == 0 and bad_flagged == 0, n_bad=bad_calm + bad_flagged, n_pix=int(ok0.size),
        n_flagged=int(flagged.sum()), n_by_variant=by_variant,
        max_rgb_unflagged=float(e_rgb[~flagged].max()) if (~flagged).any() else 0.0,
        max_depth_rel_unflagged=float(e_dep[~flagged].max()) if (~flagged).any() else 0.0,
        max_rgb=float(e_rgb.max()), mean_rgb=float(np.abs(gr - ref.rgb).mean()),
    )
    if ga is not None:
        e_alp = np.abs(ga - ref.alpha)
        out["max_alpha_unflagged"] = float(e_alp[~flagged].max()) if (~flagged).any() else 0.0
    return out


def psnr(a, b, peak=1.0):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(peak * peak / mse)
