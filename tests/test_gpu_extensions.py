"""GPU parity of the extensions: body-attached cameras (tile lists bit-exact,
pixels within tolerance of the oracle) and the fused observation epilogue
(u8 codes / halves within the oracle's admissible values, float outputs
unchanged by it, identical through the serving loop)."""
import numpy as np
import pytest

from oracle import bin_ref, observe_codes, render_ref
from paper_2604_25459_amd import synth
from tests.parity import compare

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def R():
    _torch()
    from paper_2604_25459_amd import gsr
    r = gsr.Renderer(0)
    yield r
    r.close()


def _wrist_batch(scene, E, seed):
    """Slot 0: world camera orbiting the origin; slot 1: camera riding on body
    1, a per-env body-frame look-at offset at radius U[0.3, 1] (camera-pose
    randomisation), 90 degree field of view, near plane 0.02."""
    rng = np.random.default_rng(seed)
    head = synth.pinhole(160, 120, 60.0)
    wrist = synth.pinhole(96, 64, 90.0, near=0.02)
    wrist.attach_body = 1
    vm = np.stack([synth.orbit_viewmats(rng, E, 3.0, 6.0), synth.orbit_viewmats(rng, E, 0.3, 1.0)])
    poses = synth.random_poses(rng, E, scene.n_bodies)
    return synth.Batch(cams=[head, wrist], viewmats=vm, poses=poses, bg=np.array([0.1, 0.2, 0.3], np.float32))


def test_attached_camera_bins_and_pixels(R):
    from paper_2604_25459_amd import gsr
    scene = synth.make_scene(31, 20_000, 3, 3_000, sh_degree=3, half_box=4.0)
    batch = _wrist_batch(scene, 6, 5)
    sid = R.add_synth_scene(scene)
    cams, vm, poses = gsr.batch_tensors(batch)
    assert cams[1].attach_body == 1
    out = R.render(sid, cams, vm, poses, bg=tuple(batch.bg), alpha=True)
    for c, e in ((1, 0), (1, 3), (0, 2)):
        image = batch.image_index(c, e)
        got = R.debug_bins(sid, cams, vm, poses, image)
        ref_b = bin_ref(scene, batch, c, e, got["tile_size"])
        np.testing.assert_array_equal(got["keys"], ref_b.keys)
        np.testing.assert_array_equal(got["values"], ref_b.values)
        np.testing.assert_array_equal(got["ranges"], ref_b.ranges)
        ref = render_ref(scene, batch, c, e, R.tile_size)
        rgb, depth, alpha = (t[e].cpu().numpy() for t in out[c])
        res = compare(rgb, depth, ref, gpu_alpha=alpha)
        print(f"[attached c={c} e={e}] pairs={len(ref_b.keys)} {res}", flush=True)
        assert len(ref_b.keys) > 0 and res["ok"], res
    # an invalid body index is refused before any device work
    bad = [gsr.Camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.near, c.attach_body) for c in cams]
    bad[1].attach_body = scene.n_bodies
    with pytest.raises(gsr.GsrError) as ei:
        R.render(sid, bad, vm, poses)
    assert ei.value.code == gsr.GSR_E_INVALID
    R.remove_scene(sid)


def _params(torch, n, seed):
    g = torch.Generator().manual_seed(seed)
    gain = (2.0 ** (torch.rand(n, generator=g) * 2 - 1)).float()          # +-1 EV
    contrast = (0.6 + 0.8 * torch.rand(n, generator=g)).float()
    bright = (0.2 * torch.rand(n, generator=g) - 0.1).float()
    return gain, contrast, bright


@pytest.mark.parametrize("fmt", ["u8", "f16"])
def test_observation_epilogue_matches_oracle(R, fmt):
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(3, n_envs=4)                # two slots of different sizes
    sid = R.add_synth_scene(scene)
    cams, vm, poses = gsr.batch_tensors(batch)
    E, C = batch.n_envs, batch.n_cams
    gain, contrast, bright = _params(torch, C * E, 17)
    dev = vm.device
    rgb, depth, _ = R.alloc_outputs(cams, E)
    plain_rgb, plain_depth, _ = R.alloc_outputs(cams, E)
    dt = torch.uint8 if fmt == "u8" else torch.float16
    obs_t = torch.empty(rgb.numel(), dtype=dt, device=dev)
    obs = gsr.Observation(fmt, obs_t, gain.to(dev), contrast.to(dev), bright.to(dev))
    R.render_into(sid, cams, vm, poses, plain_rgb, plain_depth, bg=tuple(batch.bg))
    R.render_into(sid, cams, vm, poses, rgb, depth, bg=tuple(batch.bg), obs=obs)
    # the epilogue changes neither the float colour nor the depth
    assert torch.equal(rgb, plain_rgb) and torch.equal(depth, plain_depth)
    # observation only (no float colour requested): the same observation
    obs_only = torch.empty_like(obs_t)
    depth2 = torch.empty_like(depth)
    R.render_into(sid, cams, vm, poses, None, depth2, bg=tuple(batch.bg),
                  obs=gsr.Observation(fmt, obs_only, gain.to(dev), contrast.to(dev), bright.to(dev)))
    assert torch.equal(obs_only, obs_t) and torch.equal(depth2, depth)
    # codes against the oracle (every admissible result of flagged decisions)
    base = 0
    for c, cam in enumerate(cams):
        npx = cam.width * cam.height
        for e in range(E):
            k = c * E + e
            if e in (0, E - 1):
                ref = render_ref(scene, batch, c, e, R.tile_size)
                got = obs_t[3 * (base + e * npx):3 * (base + (e + 1) * npx)].view(cam.height, cam.width, 3)
                got = got.cpu().numpy().astype(np.float64)
                lo = hi = None
                for v in range(ref.var_rgb.shape[0]):
                    l, h = observe_codes(ref.var_rgb[v], float(gain[k]), float(contrast[k]), float(bright[k]),
                                         fmt=fmt)
                    lo = l if lo is None else np.minimum(lo, l)
                    hi = h if hi is None else np.maximum(hi, h)
                ok = (got >= lo) & (got <= hi)
                # pixels outside the first variants' codes: every admissible variant of that pixel
                for y, x in zip(*np.nonzero(~ok.all(axis=-1))):
                    for vr in ref.pixel_variants(x, y)[0]:
                        l, h = observe_codes(vr[None, None], float(gain[k]), float(contrast[k]), float(bright[k]),
                                             fmt=fmt)
                        ok[y, x] |= (got[y, x] >= l[0, 0]) & (got[y, x] <= h[0, 0])
                print(f"[obs {fmt} c={c} e={e}] flagged channels {np.mean(hi != lo):.4f}, bad {int((~ok).sum())}",
                      flush=True)
                assert ok.all()
        base += E * npx
    R.remove_scene(sid)


def test_server_observation_equals_solo(R):
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene = synth.make_scene(41, 20_000, 2, 2_000, sh_degree=3, half_box=4.0)
    sid = R.add_synth_scene(scene, "f16")
    rng = np.random.default_rng(2)
    S = gsr.Server(R, n_streams=1)
    jobs = []
    for k in range(5):
        E = 3 + k
        b = synth.Batch(cams=[synth.pinhole(128, 96, 60.0)], viewmats=synth.orbit_viewmats(rng, E, 3.0, 6.0)[None],
                        poses=synth.random_poses(rng, E, scene.n_bodies))
        cams, vm, poses = gsr.batch_tensors(b)
        gain, contrast, bright = (t.to(vm.device) for t in _params(torch, E, 100 + k))
        rgb, depth, _ = R.alloc_outputs(cams, E)
        o = torch.empty(rgb.numel(), dtype=torch.uint8, device=vm.device)
        obs = gsr.Observation("u8", o, gain, contrast, bright)
        jobs.append((cams, vm, poses, obs, S.submit(sid, cams, vm, poses, None, depth, obs=obs)))
    for cams, vm, poses, obs, t in jobs:
        S.wait(t)
        solo = torch.empty_like(obs.out)
        _, depth, _ = R.alloc_outputs(cams, int(vm.shape[1]))
        R.render_into(sid, cams, vm, poses, None, depth,
                      obs=gsr.Observation("u8", solo, obs.gain, obs.contrast, obs.brightness))
        torch.cuda.synchronize()
        assert torch.equal(solo, obs.out)
    S.close()
    R.remove_scene(sid)
