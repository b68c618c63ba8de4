"""The oracle still produces the stored config-0 digest (regression guard)."""
import json
import os

import pytest

from tests.golden.make_golden import digest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_cfg0_digest_unchanged():
    with open(os.path.join(HERE, "golden", "cfg0_digest.json")) as f:
        ref = json.load(f)
    cur = digest()
    for k in ("visible", "pairs", "keys_sha256", "values_sha256", "ranges_sha256", "visited_sum"):
        assert cur[k] == ref[k], k
    for k in ("rgb_sum", "depth_sum", "alpha_sum"):
        assert cur[k] == pytest.approx(ref[k], rel=1e-12), k
    assert cur["pixel_32_48_rgb"] == pytest.approx(ref["pixel_32_48_rgb"], abs=1e-12)
