"""Pins of the oracle's admissible-result enumeration and of its half-precision
decoding (CPU only).

Threshold decisions of the image model (skip a Gaussian whose alpha is below
1/255; stop before adding one that takes transmittance below 1e-4) can go
either way in binary32 when the float64 value lies within rounding of the
boundary.  The oracle then lists every admissible result: flip bit k inverts
the k-th flagged decision met by that run.  These tests build pixels whose
decisions sit at relative distance 1e-4 from a boundary and check every
enumerated result against the closed form of the branch it stands for, so a
wrong bit-to-decision mapping, a result taken from the wrong branch, or a
missing widening of the flip set fails here.

Half precision: the storage decoders must equal IEEE round-to-nearest-even
conversion, checked against torch's own float16 / bfloat16 casts (ties of both
parities, subnormals, the largest finite values, zeros and infinities).
"""
from types import SimpleNamespace

import numpy as np
import pytest

from oracle.render import DEFAULT_MARGIN, composite64
from oracle.storage import round_bf16, round_f16

A_MIN = 1.0 / 255.0
T_MIN = 1e-4
BG = np.array([0.2, 0.3, 0.4])


def _pixel(opacities, colours, depths, max_flags=3):
    """One 1x1 image whose only tile lists Gaussians centred on the pixel
    centre (q = 0, so each alpha is its opacity), in the given order."""
    n = len(opacities)
    bins = SimpleNamespace(ranges=np.array([[0, n]], np.int64), values=np.arange(n, dtype=np.uint32), tiles_x=1)
    at = dict(u=np.full(n, 0.5), v=np.full(n, 0.5), conic=np.tile([1.0, 0.0, 1.0], (n, 1)),
              opacity=np.asarray(opacities, np.float64), rgb=np.asarray(colours, np.float64).reshape(n, 3),
              z=np.asarray(depths, np.float64))
    return composite64(bins, at, 1, 1, 16, BG, DEFAULT_MARGIN, max_flags, True)


def _closed(alphas, colours, depths, taken):
    """Front-to-back result of adding exactly the Gaussians marked taken
    (each with its alpha): C = sum c_k a_k T_k + bg T, depth = sum z a T / (1 - T)."""
    T, C, D = 1.0, np.zeros(3), 0.0
    for a, c, z, t in zip(alphas, colours, depths, taken):
        if t:
            C += np.asarray(c) * a * T
            D += z * a * T
            T *= 1.0 - a
    return C + BG * T, (D / (1.0 - T) if T < 1.0 else 0.0), 1.0 - T


def _check(ref, f, expect):
    rgb, depth, alpha = expect
    np.testing.assert_allclose(ref.var_rgb[f, 0, 0], rgb, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ref.var_depth[f, 0, 0], depth, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ref.var_alpha[f, 0, 0], alpha, rtol=0, atol=1e-12)


COL = [(0.9, 0.5, 0.1), (0.1, 0.8, 0.3), (0.4, 0.2, 0.9), (0.7, 0.7, 0.2)]


@pytest.mark.parametrize("delta", [1e-4, -1e-4])
def test_alpha_skip_flag_both_branches(delta):
    """alpha = (1 + delta)/255: float64 takes it iff delta > 0; the flipped
    variant is the other branch."""
    a = (1.0 + delta) / 255.0
    ref = _pixel([a], COL[:1], [2.0])
    assert ref.nflag[0, 0] == 1 and not ref.unresolved[0, 0]
    take = delta > 0
    _check(ref, 0, _closed([a], COL[:1], [2.0], [take]))
    _check(ref, 1, _closed([a], COL[:1], [2.0], [not take]))
    # bits beyond the flagged decisions change nothing
    for f in range(2, 8):
        _check(ref, f, _closed([a], COL[:1], [2.0], [take if f % 2 == 0 else not take]))
    if take:       # alpha of the primary result is the Gaussian's own
        np.testing.assert_allclose(ref.alpha[0, 0], a, rtol=1e-15)
    else:
        assert ref.alpha[0, 0] == 0.0 and ref.depth[0, 0] == 0.0


@pytest.mark.parametrize("delta", [1e-4, -1e-4])
def test_transmittance_stop_flag_both_branches(delta):
    """Three stacked Gaussians, alpha 0.95, 0.95, then a3 with
    0.0025 (1 - a3) = 1e-4 (1 + delta): float64 adds the third iff delta > 0
    (stop before adding it otherwise); the flipped variant is the other branch."""
    a3 = 1.0 - 0.04 * (1.0 + delta)
    alphas = [0.95, 0.95, a3]
    ref = _pixel(alphas, COL[:3], [1.0, 2.0, 3.0])
    assert ref.nflag[0, 0] == 1
    add3 = delta > 0
    _check(ref, 0, _closed(alphas, COL[:3], [1.0, 2.0, 3.0], [True, True, add3]))
    _check(ref, 1, _closed(alphas, COL[:3], [1.0, 2.0, 3.0], [True, True, not add3]))
    # transmittance left by the primary: just above 1e-4 after adding the third, else 0.05^2
    T = 1.0 - ref.alpha[0, 0]
    np.testing.assert_allclose(T, T_MIN * (1.0 + delta) if add3 else 0.0025, rtol=1e-9)


def test_two_flags_map_to_bits_in_list_order():
    """Gaussians A then B, alphas (1 + 1e-4)/255 (taken) and (1 - 1e-4)/255
    (skipped): bit 0 flips A, bit 1 flips B, independently."""
    aA, aB = (1.0 + 1e-4) / 255.0, (1.0 - 1e-4) / 255.0
    ref = _pixel([aA, aB], COL[:2], [1.0, 2.0])
    assert ref.nflag[0, 0] == 2
    for f in range(4):
        _check(ref, f, _closed([aA, aB], COL[:2], [1.0, 2.0], [not (f & 1), bool(f & 2)]))


def test_flip_that_meets_a_new_flag_is_widened():
    """A flagged skip (G3, alpha (1 - 1e-4)/255) in front of G4 whose stop
    decision is flagged only when G3 was taken: the unflipped run meets one
    flagged decision, its flip meets two.  With one flip bit the enumeration is
    marked unresolved; pixel_variants widens to two and lists every branch."""
    a3 = (1.0 - 1e-4) / 255.0
    t3 = 0.05 * 0.05 * (1.0 - a3)                      # transmittance after G3 when it is taken
    a4 = 1.0 - T_MIN * (1.0 - 1e-4) / t3               # then G4 lands 1e-4 below the stop threshold
    alphas = [0.95, 0.95, a3, a4]
    cols, zs = COL, [1.0, 2.0, 3.0, 4.0]
    ref1 = _pixel(alphas, cols, zs, max_flags=1)
    assert ref1.nflag[0, 0] == 1 and ref1.unresolved[0, 0]
    ref2 = _pixel(alphas, cols, zs, max_flags=2)
    assert not ref2.unresolved[0, 0]
    skip3_add4 = _closed(alphas, cols, zs, [True, True, False, True])
    take3_stop4 = _closed(alphas, cols, zs, [True, True, True, False])
    take3_add4 = _closed(alphas, cols, zs, [True, True, True, True])
    _check(ref2, 0, skip3_add4)
    _check(ref2, 1, take3_stop4)      # bit 0: take G3; G4's flagged stop then holds
    _check(ref2, 2, skip3_add4)       # bit 1 names no decision of that run
    _check(ref2, 3, take3_add4)       # bits 0 and 1: take G3, and do not stop at G4
    rgb, depth, alpha = ref2.pixel_variants(0, 0)
    assert rgb.shape == (4, 3)
    for k, e in enumerate((skip3_add4, take3_stop4, skip3_add4, take3_add4)):
        np.testing.assert_allclose(rgb[k], e[0], atol=1e-12)
        np.testing.assert_allclose(depth[k], e[1], atol=1e-12)
        np.testing.assert_allclose(alpha[k], e[2], atol=1e-12)


def test_decisions_outside_the_margin_are_not_flagged():
    a = (1.0 + 2 * DEFAULT_MARGIN) / 255.0
    ref = _pixel([a, (1.0 - 2 * DEFAULT_MARGIN) / 255.0], COL[:2], [1.0, 2.0])
    assert ref.nflag[0, 0] == 0
    for f in range(8):
        _check(ref, f, _closed([a, 0.0], COL[:2], [1.0, 2.0], [True, False]))
    assert ref.pixel_variants(0, 0)[0].shape == (1, 3)


# ------------------------------------------------------------------ half precision
def _special_bits():
    rng = np.random.default_rng(12)
    parts = [
        rng.integers(0, 2**32, 200_000, dtype=np.uint64).astype(np.uint32),          # every exponent
        (rng.integers(0, 2**15, 20_000, dtype=np.uint64).astype(np.uint32) << 17) | 0x8000,   # ties, bit 16 = 0
        (rng.integers(0, 2**15, 20_000, dtype=np.uint64).astype(np.uint32) << 17) | 0x18000,  # ties, bit 16 = 1
        rng.integers(1, 0x00800000, 20_000, dtype=np.uint64).astype(np.uint32),      # subnormals
        np.array([0x00008000, 0x00018000, 0x007F8000, 0x007FFFFF, 0x00800000, 0x7F7FFFFF, 0x7F7F8000,
                  0x7F7F7FFF, 0x7F7E8000, 0x7F800000, 0x00000000, 0x3F800000, 0x3F808000, 0x3F818000], np.uint32),
    ]
    b = np.concatenate(parts)
    b = np.concatenate([b, b | np.uint32(0x80000000)])                               # both signs
    f = b.view(np.float32)
    return f[~np.isnan(f)]


def test_round_bf16_matches_ieee_conversion():
    torch = pytest.importorskip("torch")
    x = _special_bits()
    want = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(round_bf16(x).view(np.uint32), want.view(np.uint32))


def test_round_f16_matches_ieee_conversion():
    torch = pytest.importorskip("torch")
    x = _special_bits()
    want = torch.from_numpy(x.copy()).to(torch.float16).to(torch.float32).numpy()
    with np.errstate(over="ignore"):
        got = round_f16(x)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))
