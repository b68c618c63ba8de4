"""Writes tests/golden/cfg0_digest.json from the CPU oracle alone.

The paper prints no worked example, so the stored values here are the oracle's
own output on the seeded 128x96 / 4096-Gaussian workload, kept to detect any
unintended change of the oracle.  Only ``oracle`` and the input generator are
called.  Re-run only when a change to the oracle is justified by a passage of
the paper (or a documented reading of it), and say which in the commit.
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import render_ref  # noqa: E402
from paper_2604_25459_amd import synth  # noqa: E402


def digest():
    scene, batch = synth.make_config(0)
    r = render_ref(scene, batch, variants=False)
    b = r.bins
    h = lambda a: hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
    return {
        "workload": "config 0: 1 env, 128x96, 4096 Gaussians, SH degree 1, tile 16",
        "visible": int(b.visible.sum()),
        "pairs": int(b.keys.size),
        "keys_sha256": h(b.keys.astype("<u8")),
        "values_sha256": h(b.values.astype("<u4")),
        "ranges_sha256": h(b.ranges.astype("<i8")),
        "rgb_sum": float(r.rgb.sum()),
        "depth_sum": float(r.depth.sum()),
        "alpha_sum": float(r.alpha.sum()),
        "visited_sum": int(r.visited.sum()),
        "pixel_32_48_rgb": [float(x) for x in r.rgb[48, 32]],
    }


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg0_digest.json")
    with open(out, "w") as f:
        json.dump(digest(), f, indent=1)
    print("wrote", out)
