"""Comparison of GPU images with oracle images (float64 with admissible
alternatives where a threshold decision is within rounding of its boundary)."""
import numpy as np

RGB_TOL = 1e-3          # max-abs per channel, float32 path
DEPTH_REL = 1e-3        # |d - d_ref| <= 1e-3 * max(1, d_ref)


def compare(gpu_rgb, gpu_depth, ref, rgb_tol=RGB_TOL, depth_rel=DEPTH_REL):
    gr = np.asarray(gpu_rgb, np.float64)
    gd = np.asarray(gpu_depth, np.float64)
    e_rgb = np.abs(gr[None] - ref.var_rgb).max(axis=-1)                          # (V, H, W)
    e_dep = np.abs(gd[None] - ref.var_depth) / np.maximum(1.0, np.abs(ref.var_depth))
    ok_v = (e_rgb <= rgb_tol) & (e_dep <= depth_rel)
    ok = ok_v.any(axis=0) | ref.unresolved
    flagged = ref.nflag > 0
    score = np.maximum(e_rgb / rgb_tol, e_dep / depth_rel).min(axis=0)           # best admissible variant
    return dict(
        ok=bool(ok.all()), n_bad=int((~ok).sum()), n_pix=int(ok.size),
        n_flagged=int(flagged.sum()), n_unresolved=int(ref.unresolved.sum()),
        max_rgb_unflagged=float(e_rgb[0][~flagged].max()) if (~flagged).any() else 0.0,
        max_depth_rel_unflagged=float(e_dep[0][~flagged].max()) if (~flagged).any() else 0.0,
        max_rgb=float(np.abs(gr - ref.rgb).max()), worst_score=float(score.max()),
        mean_rgb=float(np.abs(gr - ref.rgb).mean()),
    )


def psnr(a, b, peak=1.0):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(peak * peak / mse)
