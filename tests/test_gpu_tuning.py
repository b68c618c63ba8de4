"""hipGraph replay and autotuned launch parameters change no pixel: every
replay and every parameter set gives the bits of the eager default render."""
import time

import numpy as np
import pytest

from paper_2604_25459_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_graph_replays_match_eager():
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(1, n_envs=8)
    Rg = gsr.Renderer(0)                  # graphs on (default)
    Re = gsr.Renderer(0, graphs=False)
    sg, se = Rg.add_synth_scene(scene), Re.add_synth_scene(scene)
    cams, vm, _ = gsr.batch_tensors(batch)
    dev = vm.device
    for step in range(4):                 # new poses every step: one capture, then replays
        poses = torch.from_numpy(synth.make_poses(1, step, 8, scene.n_bodies)).to(dev)
        eager = Re.render(se, cams, vm, poses, alpha=True)
        torch.cuda.synchronize()
        replay = Rg.render(sg, cams, vm, poses, alpha=True)
        torch.cuda.synchronize()
        for a, b in zip(eager[0], replay[0]):
            assert torch.equal(a, b), f"step {step}"
    Rg.close()
    Re.close()


def test_two_stream_chunks_match_one_stream():
    """Alternate memory chunks on two streams give the bits of one stream, and
    work queued on the caller's stream after the call sees finished images."""
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(3, n_envs=8)       # 16 images in chunks of 3: six chunks
    R1 = gsr.Renderer(0, overlap=False)
    R2 = gsr.Renderer(0)
    s1, s2 = R1.add_synth_scene(scene), R2.add_synth_scene(scene)
    cams, vm, poses = gsr.batch_tensors(batch)
    R1.set_tuning(s1, cams, vm, poses, chunk_images=3)
    R2.set_tuning(s2, cams, vm, poses, chunk_images=3)
    dev = vm.device
    for step in range(3):                 # new poses every step: graph capture, then replays
        poses = torch.from_numpy(synth.make_poses(3, step, 8, scene.n_bodies)).to(dev)
        ref = [[t.clone() for t in slot] for slot in R1.render(s1, cams, vm, poses, alpha=True)]
        got = [[t.clone() for t in slot] for slot in R2.render(s2, cams, vm, poses, alpha=True)]
        torch.cuda.synchronize()
        for slot_ref, slot_got in zip(ref, got):
            for a, b in zip(slot_ref, slot_got):
                assert torch.equal(a, b), f"step {step}"
    R1.close()
    R2.close()


def test_trim_releases_working_memory_and_changes_no_pixel():
    """gsr_trim frees the idle working sets (two-stream chunks hold two); the
    next render allocates again and gives the same bits."""
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(3, n_envs=8)
    R = gsr.Renderer(0)
    sid = R.add_synth_scene(scene)
    cams, vm, poses = gsr.batch_tensors(batch)
    R.set_tuning(sid, cams, vm, poses, chunk_images=3)
    ref = [[t.clone() for t in slot] for slot in R.render(sid, cams, vm, poses, alpha=True)]
    torch.cuda.synchronize()
    freed = R.trim()
    print("trim freed", freed, flush=True)
    assert freed > 100 << 20                 # the working sets of a 596k-Gaussian scene
    assert R.trim() <= 4 << 20               # nothing left to free
    got = R.render(sid, cams, vm, poses, alpha=True)
    torch.cuda.synchronize()
    for slot_ref, slot_got in zip(ref, got):
        for a, b in zip(slot_ref, slot_got):
            assert torch.equal(a, b)
    R.close()


def test_two_stream_lidar_chunks_match_one_stream():
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene = synth.make_scene(52, 120_000, 3, 20_000, sh_degree=0, half_box=3.0)
    rng = np.random.default_rng(7)
    E = 12
    lid = synth.rotating_lidar(16, 256, -20, 20)
    ros = synth.rosette_lidar(16, 128, half_fov_deg=35.0, s0=0.7)       # listed rays in the same call
    vm = torch.from_numpy(np.stack([synth.sensor_viewmats(rng, E, 0.5, 2.5, 0.1),
                                    synth.sensor_viewmats(rng, E, 0.5, 2.5, 0.1)])).cuda()
    poses = torch.from_numpy(synth.random_poses(rng, E, scene.n_bodies)).cuda()
    out = []
    for overlap in (False, True):
        R = gsr.Renderer(0, chunk_bytes=64 << 20, overlap=overlap)   # a few scans per chunk
        sid = R.add_synth_scene(scene)
        res = R.render_lidar(sid, [lid, ros], vm, poses)
        out.append([(r.clone(), h.clone()) for r, h in res])
        torch.cuda.synchronize()
        R.close()
    for (r0, h0), (r1, h1) in zip(out[0], out[1]):
        assert torch.equal(r0, r1) and torch.equal(h0, h1)
    assert (out[0][0][1] > 0.1).sum() > 100 and (out[0][1][1] > 0.1).sum() > 100


@pytest.mark.parametrize("params", [dict(tile_size=8, lds_batch=64), dict(tile_size=8, lds_batch=256),
                                    dict(tile_size=32, lds_batch=512), dict(lds_batch=512, images_per_thread=1),
                                    dict(images_per_thread=8, persistent=1), dict(persistent=1, chunk_images=3),
                                    dict(bin_schedule=0), dict(bin_schedule=1, tile_size=8, lds_batch=128),
                                    dict(lds_batch=256), dict(lds_batch=128, persistent=1),
                                    dict(tile_size=32, lds_batch=128), dict(images_per_thread=16),
                                    dict(images_per_thread=16, chunk_images=2, tile_size=8)])
def test_tuning_changes_no_pixel(params):
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(3, n_envs=5)       # two camera slots of different sizes
    R = gsr.Renderer(0)
    sid = R.add_synth_scene(scene, "bf16")
    cams, vm, poses = gsr.batch_tensors(batch)
    ref = R.render(sid, cams, vm, poses, alpha=True)
    R.set_tuning(sid, cams, vm, poses, **params)
    got = R.tuning(sid, cams, vm, poses)
    for k, v in params.items():
        assert got[k] == v
    for _ in range(2):
        out = R.render(sid, cams, vm, poses, alpha=True)
        for slot_ref, slot_out in zip(ref, out):
            for a, b in zip(slot_ref, slot_out):
                assert torch.equal(a, b), params
    R.close()


def test_autotune_and_cache_roundtrip(tmp_path):
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(1, n_envs=16)
    R = gsr.Renderer(0)
    sid = R.add_synth_scene(scene)
    cams, vm, poses = gsr.batch_tensors(batch)
    ref = R.render(sid, cams, vm, poses)
    rgb, depth, _ = R.alloc_outputs(cams, 16)
    best = R.autotune(sid, cams, vm, poses, rgb, depth)
    print("autotuned", best, flush=True)
    assert best["tile_size"] in (8, 16, 32) and best["ms"] > 0
    assert R.tuning(sid, cams, vm, poses) == best
    out = R.render(sid, cams, vm, poses)
    assert torch.equal(out[0][0], ref[0][0]) and torch.equal(out[0][1], ref[0][1])
    path = str(tmp_path / "tune.jsonl")
    R.save_tuning(path)
    R2 = gsr.Renderer(0)
    sid2 = R2.add_synth_scene(scene)
    R2.load_tuning(path)
    loaded = R2.tuning(sid2, cams, vm, poses)
    assert {k: v for k, v in loaded.items() if k != "ms"} == {k: v for k, v in best.items() if k != "ms"}
    assert loaded["ms"] == pytest.approx(best["ms"], rel=1e-6)
    R2.close()
    R.close()


def test_schedules_agree_on_wide_splats():
    """Splats wider than the image cover every column of a transposed group
    (64 entries x 64 columns all set, so a tile list takes more than one
    128-byte line per group); both list schedules must still produce the same
    pixels bit for bit."""
    torch = _torch()
    from paper_2604_25459_amd import gsr
    from tests.scenes import one_camera, scene_from
    rng = np.random.default_rng(4)
    n = 600
    means = rng.uniform([-1.5, -1.0, 2.0], [1.5, 1.0, 4.0], (n, 3))
    scales = np.exp(rng.normal(np.log(0.8), 0.3, (n, 3)))          # each covers most of the image
    scene = scene_from(means, scales, rng.standard_normal((n, 4)), rng.uniform(0.02, 0.3, n),
                       rng.uniform(0, 1, (n, 1, 3)), degree=0)
    batch = one_camera(640, 480, 400.0)
    R = gsr.Renderer(0)
    sid = R.add_synth_scene(scene)
    cams, vm, poses = gsr.batch_tensors(batch)
    outs = []
    for sched in (0, 1):
        R.set_tuning(sid, cams, vm, poses, bin_schedule=sched)
        outs.append(R.render(sid, cams, vm, poses, alpha=True))
    for a, b in zip(outs[0][0], outs[1][0]):
        assert torch.equal(a, b)
    R.close()


def test_transposed_schedule_on_a_wide_image():
    """1920 x 1080 at 16-pixel tiles: 120 tile columns and 68 tile rows, so
    the transposed schedule runs two 64-column windows per row segment at
    level 2 and two 64-row windows per block at level 1.  Its tile lists
    equal the oracle's bit for bit, and both schedules give the same pixels."""
    torch = _torch()
    from paper_2604_25459_amd import gsr, synth
    from oracle import bin_ref
    scene = synth.make_scene(63, 40_000, 2, 4_000, sh_degree=1, half_box=4.0)
    rng = np.random.default_rng(21)
    batch = synth.Batch(cams=[synth.pinhole(1920, 1080, 70.0)], viewmats=synth.orbit_viewmats(rng, 2, 3.0, 5.0)[None],
                        poses=synth.random_poses(rng, 2, scene.n_bodies))
    R = gsr.Renderer(0)
    sid = R.add_synth_scene(scene)
    cams, vm, poses = gsr.batch_tensors(batch)
    outs = []
    for sched in (0, 1):
        R.set_tuning(sid, cams, vm, poses, bin_schedule=sched)
        outs.append(R.render(sid, cams, vm, poses, alpha=True))
        if sched == 1:
            got = R.debug_bins(sid, cams, vm, poses, 1)
            ref = bin_ref(scene, batch, 0, 1, got["tile_size"])
            assert ref.ranges.shape[0] == 120 * 68
            np.testing.assert_array_equal(got["keys"], ref.keys)
            np.testing.assert_array_equal(got["values"], ref.values)
            np.testing.assert_array_equal(got["ranges"], ref.ranges)
    for a, b in zip(outs[0][0], outs[1][0]):
        assert torch.equal(a, b)
    R.close()


def test_async_render_returns_before_the_device_finishes():
    """After a render that sizes the tile lists of a job shape, renders of that
    shape enqueue every chunk without waiting for its totals: the call returns
    while the device still works, and the images equal a render that waits at
    every chunk."""
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(2, n_envs=512)
    Ra = gsr.Renderer(0)
    Rs = gsr.Renderer(0, sync_lists=True)
    sa, ss = Ra.add_synth_scene(scene), Rs.add_synth_scene(scene)
    cams, vm, _ = gsr.batch_tensors(batch)
    dev = vm.device
    rgb_a, depth_a, _ = Ra.alloc_outputs(cams, 512)
    rgb_s, depth_s, _ = Rs.alloc_outputs(cams, 512)
    stream = torch.cuda.current_stream(dev)
    for step in range(3):
        poses = torch.from_numpy(synth.make_poses(2, step, 512, scene.n_bodies)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ra.render_into(sa, cams, vm, poses, rgb_a, depth_a)
        t_call = time.perf_counter() - t0
        pending = not stream.query()
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t0
        print(f"step {step}: call {1e3 * t_call:.2f} ms, render {1e3 * t_all:.2f} ms, pending {pending}", flush=True)
        if step > 0:                   # step 0 plans the lists (waits at every chunk)
            assert pending and t_call < 0.5 * t_all
        Rs.render_into(ss, cams, vm, poses, rgb_s, depth_s)
        torch.cuda.synchronize()
        assert torch.equal(rgb_a, rgb_s) and torch.equal(depth_a, depth_s), f"step {step}"
    Ra.close()
    Rs.close()


def test_list_overflow_falls_back_with_identical_bits():
    """Asynchronous chunks whose tile lists exceed a small capacity set from
    the host write no lists; the fallback rasteriser composites them from the
    depth-ordered Gaussians, and images and work counts equal the planned
    render's bit for bit (two camera sizes, chunks on two streams)."""
    torch = _torch()
    from paper_2604_25459_amd import gsr
    scene, batch = synth.make_config(3, n_envs=6)
    R = gsr.Renderer(0, list_cap=2000)
    sid = R.add_synth_scene(scene)
    cams, vm, poses = gsr.batch_tensors(batch)
    R.set_tuning(sid, cams, vm, poses, chunk_images=4)     # three chunks, alternating streams
    rgb, depth, alpha = R.alloc_outputs(cams, 6, alpha=True)
    npx = rgb.numel() // 3
    work = torch.zeros(npx * 2, dtype=torch.int32, device=rgb.device)
    R.render_into(sid, cams, vm, poses, rgb, depth, alpha, work=work)      # plans the lists
    torch.cuda.synchronize()
    ref = [t.clone() for t in (rgb, depth, alpha, work)]
    for k in range(3):
        for t in (rgb, depth, alpha):
            t.fill_(float("nan"))
        work.fill_(-1)
        R.render_into(sid, cams, vm, poses, rgb, depth, alpha, work=work)  # overflows into the fallback
        torch.cuda.synchronize()
        for a, b in zip(ref, (rgb, depth, alpha, work)):
            assert torch.equal(a, b), f"render {k}"
    R.close()
