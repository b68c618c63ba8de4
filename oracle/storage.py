"""Half-precision storage as the oracle sees it (test infrastructure).

Scales, rotations, opacity and SH coefficients stored in IEEE binary16 or
bfloat16 (means stay float32); returns the float32 values that decoding the
stored halves gives.  Both conversions round to nearest, ties to even.
"""
import numpy as np


def round_f16(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, np.float32).astype(np.float16).astype(np.float32)


def round_bf16(x: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def decoded_attrs(scene, storage: str):
    """Attribute overrides for bin_ref / attrs64 / render_ref."""
    if storage == "f32":
        return None
    r = round_f16 if storage == "f16" else round_bf16
    return dict(means=scene.means, scales=r(scene.scales), quats=r(scene.quats), opacities=r(scene.opacities),
                sh=r(scene.sh))
