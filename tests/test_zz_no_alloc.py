"""gsr_render_noalloc (all device working memory in the library's fixed
scratch array) against gsr_render, through the C ABI: two calls in a row,
the second with a smaller input, each bit-identical to gsr_render on the same
inputs; a two-camera batch whose chunks mix image sizes; and the size limit
rejected before any device work."""
import numpy as np
import pytest

from paper_2604_25459_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _both(R, sid, batch):
    """(gsr_render, gsr_render_noalloc) outputs for one batch; the noalloc
    outputs start as NaN so that an unwritten pixel shows."""
    torch = _torch()
    from paper_2604_25459_amd import gsr
    cams, vm, poses = gsr.batch_tensors(batch)
    E = batch.n_envs
    ref = R.alloc_outputs(cams, E, alpha=True)
    got = [t.fill_(float("nan")) for t in R.alloc_outputs(cams, E, alpha=True)]
    bg = tuple(float(x) for x in batch.bg)
    R.render_into(sid, cams, vm, poses, ref[0], ref[1], ref[2], bg)
    R.render_into(sid, cams, vm, poses, got[0], got[1], got[2], bg, noalloc=True)
    torch.cuda.synchronize()
    return ref, got


def _assert_same(ref, got, what):
    torch = _torch()
    for name, a, b in zip(("rgb", "depth", "alpha"), ref, got):
        assert not torch.isnan(b).any(), f"{what}: {name} has unwritten values"
        assert torch.equal(a, b), f"{what}: {name} differs, max |d| = {(a - b).abs().max().item():.3g}"


def test_noalloc_matches_render_twice_then_smaller():
    _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(1)          # 140k Gaussians, SH3, 8 bodies, 320x240
    print("noalloc: config 1 scene, 16 envs then 5 envs", flush=True)
    R = gsr.Renderer(0)
    try:
        sid = R.add_synth_scene(scene)
        first = batch.subset(range(16))          # more images than one chunk of the scratch holds
        ref, got = _both(R, sid, first)
        _assert_same(ref, got, "16 envs")
        second = batch.subset([3, 17, 40, 41, 63])
        ref2, got2 = _both(R, sid, second)
        _assert_same(ref2, got2, "5 envs")
        # the first call's results were not disturbed by the second
        assert not np.isnan(got[0].cpu().numpy()).any()
    finally:
        R.close()


def test_noalloc_two_camera_sizes_and_half_storage():
    _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(3, n_envs=3)   # 596k Gaussians, 128x128 wrist + 640x480 head cameras
    print("noalloc: config 3 scene (bf16), 3 envs x 2 cameras", flush=True)
    R = gsr.Renderer(0)
    try:
        sid = R.add_synth_scene(scene, "bf16")
        ref, got = _both(R, sid, batch)
        _assert_same(ref, got, "config 3, 3 envs x 2 cameras")
    finally:
        R.close()


def test_noalloc_rejects_more_images_than_its_limit():
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(0)
    R = gsr.Renderer(0)
    try:
        sid = R.add_synth_scene(scene)
        E = 4097
        cam = synth.Camera(8, 8, 8.0, 8.0, 4.0, 4.0, 0.01)
        vm = torch.from_numpy(np.broadcast_to(batch.viewmats[:, :1], (1, E, 3, 4)).copy()).cuda()
        rgb, depth, _ = R.alloc_outputs([cam], E)
        with pytest.raises(gsr.GsrError) as ex:
            R.render_into(sid, [cam], vm, torch.zeros((E, 0, 7), device="cuda"), rgb, depth, noalloc=True)
        assert ex.value.code == gsr.GSR_E_INVALID
        assert "GSR_NOALLOC_MAX_IMAGES" in str(ex.value)
    finally:
        R.close()
