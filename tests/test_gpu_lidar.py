"""GPU parity of the batch LiDAR: ranges and hit probabilities of a rotating
and a body-mounted solid-state sensor against the float64 per-ray oracle
(every ray against every Gaussian), plus the full-turn seam and invalid
arguments."""
import math

import numpy as np
import pytest

from oracle import lidar_ref
from paper_2604_25459_amd import synth
from tests.scenes import scene_from

pytestmark = pytest.mark.gpu

HIT_TOL = 1e-3
RANGE_REL = 1e-3


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


def _tensors(batch):
    import torch
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(np.ascontiguousarray(batch.viewmats, np.float32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(batch.poses, np.float32)).to(dev))


def _compare(got_range, got_hit, ref, label, scene, batch, l, e, min_hits=20):
    """Every ray matches the oracle's result, or, if one of its threshold
    decisions is flagged, one of its admissible results (all enumerated)."""
    from oracle import lidar_ray_variants

    def within(r, h, rr, hh):
        return (np.abs(h - hh) <= HIT_TOL) & (np.abs(r - rr) / np.maximum(1.0, rr) <= RANGE_REL)

    ok = within(got_range, got_hit, ref.range, ref.hit)
    calm = ~ref.flagged
    by_variant = 0
    for y, x in zip(*np.nonzero(~ok & ref.flagged)):
        rr, hh = lidar_ray_variants(scene, batch, l, e, y, x)
        if within(got_range[y, x], got_hit[y, x], rr, hh).any():
            ok[y, x] = True
            by_variant += 1
    e_hit = np.abs(got_hit - ref.hit)
    e_rng = np.abs(got_range - ref.range) / np.maximum(1.0, ref.range)
    print(f"[{label}] rays {ok.size} flagged {int(ref.flagged.sum())} matched by a variant {by_variant} "
          f"hits {int((ref.hit > 0).sum())} max hit err (unflagged) {e_hit[calm].max():.2e} "
          f"max range rel err (unflagged) {e_rng[calm].max():.2e}", flush=True)
    assert ok.all(), (label, int((~ok).sum()))
    assert (ref.hit > 0.1).sum() >= min_hits   # the scans see something


def test_lidar_rotating_and_mounted_match_oracle(R):
    from paper_2604_25459_amd import gsr
    scene = synth.make_scene(51, 4_000, 3, 800, sh_degree=0, half_box=3.0)
    rng = np.random.default_rng(6)
    E = 3
    rot = synth.rotating_lidar(16, 128, -20, 20)
    sec = synth.sector_lidar(8, 64, 70, -25, 15)
    sec.attach_body = 1
    # mounted sensor: 0.8 m behind body 1's origin, looking at it, heading jittered per env
    off = np.zeros((E, 3, 4), np.float32)
    for e in range(E):
        yaw = rng.uniform(-0.3, 0.3)
        Rm = np.array([[math.cos(yaw), -math.sin(yaw), 0], [math.sin(yaw), math.cos(yaw), 0], [0, 0, 1]])
        c = np.array([-0.8, 0.0, 0.2])
        off[e, :, :3] = Rm.T
        off[e, :, 3] = -Rm.T @ c
    vm = np.stack([synth.sensor_viewmats(rng, E, 0.5, 2.5, 0.1), off])
    poses = synth.random_poses(rng, E, scene.n_bodies)
    batch = synth.LidarBatch(cams=[rot, sec], viewmats=vm, poses=poses)
    sid = R.add_synth_scene(scene)
    vm_t, poses_t = _tensors(batch)
    out = R.render_lidar(sid, [rot, sec], vm_t, poses_t)
    for l, e in ((0, 0), (0, 2), (1, 1)):
        ref = lidar_ref(scene, batch, l, e)
        _compare(out[l][0][e].cpu().numpy(), out[l][1][e].cpu().numpy(), ref, f"lidar {l} env {e}", scene, batch, l,
                 e)
    # the same scans again: deterministic
    again = R.render_lidar(sid, [rot, sec], vm_t, poses_t)
    import torch
    for (r0, h0), (r1, h1) in zip(out, again):
        assert torch.equal(r0, r1) and torch.equal(h0, h1)
    R.remove_scene(sid)


def test_lidar_seam_and_near_sensor(R):
    # a splat straddling the seam behind the sensor, and one that encloses the sensor
    scene = scene_from([[-3.0, 0.0, 0.0], [0.05, 0.0, 0.0], [2.0, 1.0, 0.3]], [[0.3, 0.3, 0.3], [0.4, 0.4, 0.4],
                                                                              [0.2, 0.05, 0.1]],
                       opac=[0.8, 0.3, 0.9], degree=0)
    lid = synth.rotating_lidar(8, 96, -30, 30, near=0.05)
    vm = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32).reshape(1, 1, 3, 4)
    batch = synth.LidarBatch(cams=[lid], viewmats=vm, poses=np.zeros((1, 0, 7), np.float32))
    sid = R.add_synth_scene(scene)
    vm_t, poses_t = _tensors(batch)
    out = R.render_lidar(sid, [lid], vm_t, poses_t)
    ref = lidar_ref(scene, batch, 0, 0)
    _compare(out[0][0][0].cpu().numpy(), out[0][1][0].cpu().numpy(), ref, "seam", scene, batch, 0, 0, min_hits=5)
    assert ref.hit[4, 0] > 0.3 and ref.hit[4, -1] > 0.3
    R.remove_scene(sid)


def test_lidar_invalid_arguments(R):
    from paper_2604_25459_amd import gsr
    scene = synth.make_scene(52, 500, 1, 100, sh_degree=0)
    sid = R.add_synth_scene(scene)
    rng = np.random.default_rng(1)
    good = synth.rotating_lidar(4, 32, -10, 10)
    vm = synth.sensor_viewmats(rng, 2, 1.0, 2.0)[None]
    poses = synth.random_poses(rng, 2, 1)
    vm_t, poses_t = _tensors(synth.LidarBatch(cams=[good], viewmats=vm, poses=poses))
    bad_cases = []
    b = synth.rotating_lidar(4, 32, -10, 10)
    b.elevations = b.elevations[::-1].copy()           # descending
    bad_cases.append(b)
    b = synth.rotating_lidar(4, 32, -10, 10)
    b.az_step = 1.0                                    # 32 rad > one turn
    bad_cases.append(b)
    b = synth.rotating_lidar(4, 32, -10, 10)
    b.attach_body = 1                                  # the scene has one body
    bad_cases.append(b)
    b = synth.rotating_lidar(4, 32, -10, 10)
    b.near_range = 0.0
    bad_cases.append(b)
    b = synth.rosette_lidar(4, 32)
    b.ray_az = b.ray_az.copy()
    b.ray_az[1, 3] = 3.5                               # listed azimuth beyond pi
    bad_cases.append(b)
    b = synth.rosette_lidar(4, 32)
    b.ray_el = b.ray_el.copy()
    b.ray_el[0, 0] = 1.6                               # listed elevation beyond pi/2
    bad_cases.append(b)
    for bad in bad_cases:
        with pytest.raises(gsr.GsrError) as ei:
            R.render_lidar(sid, [bad], vm_t, poses_t)
        assert ei.value.code == gsr.GSR_E_INVALID
    R.render_lidar(sid, [good], vm_t, poses_t)         # and the good one still renders
    _torch().cuda.synchronize()
    R.remove_scene(sid)


def test_listed_rays_rosette_match_oracle(R):
    """Non-repetitive (rosette) scans, listed ray by ray, in one call with a
    rotating grid: every ray against the float64 per-ray oracle."""
    scene = synth.make_scene(53, 4_000, 3, 800, sh_degree=0, half_box=3.0)
    rng = np.random.default_rng(8)
    E = 2
    ros = synth.rosette_lidar(16, 128, half_fov_deg=35.0, s0=0.3)
    rot = synth.rotating_lidar(8, 64, -20, 20)
    vm = np.stack([synth.sensor_viewmats(rng, E, 0.5, 2.5, 0.1), synth.sensor_viewmats(rng, E, 0.5, 2.5, 0.1)])
    poses = synth.random_poses(rng, E, scene.n_bodies)
    batch = synth.LidarBatch(cams=[ros, rot], viewmats=vm, poses=poses)
    sid = R.add_synth_scene(scene)
    vm_t, poses_t = _tensors(batch)
    out = R.render_lidar(sid, [ros, rot], vm_t, poses_t)
    for l, e in ((0, 0), (0, 1), (1, 1)):
        ref = lidar_ref(scene, batch, l, e)
        _compare(out[l][0][e].cpu().numpy(), out[l][1][e].cpu().numpy(), ref, f"listed {l} env {e}", scene, batch, l,
                 e)
    R.remove_scene(sid)


def test_listed_rays_edge_cases(R):
    """Listed rays at the seam (azimuth exactly -pi and pi), near the poles,
    duplicated, and many sharing one elevation, in a 3 x 37 list (neither a
    multiple of the tile size), around splats that straddle the seam behind
    the sensor, sit above it and enclose it: every ray against the oracle."""
    scene = scene_from([[-3.0, 0.0, 0.0], [0.05, 0.0, 0.0], [2.0, 1.0, 0.3], [0.3, 0.1, 4.0], [1.5, -0.2, 0.0]],
                       [[0.3, 0.3, 0.3], [0.4, 0.4, 0.4], [0.2, 0.05, 0.1], [0.5, 0.5, 0.2], [0.1, 0.1, 0.1]],
                       opac=[0.8, 0.3, 0.9, 0.7, 0.95], degree=0)
    rng = np.random.default_rng(12)
    n = 3 * 37
    az = rng.uniform(-math.pi, math.pi, n)
    el = rng.uniform(-0.4, 0.4, n)
    az[:6] = [-math.pi, math.pi, -math.pi, math.pi, 0.0, 0.0]      # the seam, twice each
    el[:6] = [0.0, 0.0, 0.05, -0.05, 0.0, 0.0]                     # and a duplicated ray straight ahead
    el[6:10] = [1.55, -1.55, 1.5, -1.5]                            # near the poles
    el[10:40] = 0.1                                                 # thirty rays on one elevation
    az32 = np.clip(az.astype(np.float32), np.float32(-math.pi), np.float32(math.pi))
    lid = synth.LidarSpec(width=37, height=3, az0=0.0, az_step=0.0, elevations=np.zeros(0, np.float32),
                          near_range=0.05, pattern=2, ray_az=az32.reshape(3, 37),
                          ray_el=el.astype(np.float32).reshape(3, 37))
    vm = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32).reshape(1, 1, 3, 4)
    batch = synth.LidarBatch(cams=[lid], viewmats=vm, poses=np.zeros((1, 0, 7), np.float32))
    sid = R.add_synth_scene(scene)
    vm_t, poses_t = _tensors(batch)
    out = R.render_lidar(sid, [lid], vm_t, poses_t)
    ref = lidar_ref(scene, batch, 0, 0)
    _compare(out[0][0][0].cpu().numpy(), out[0][1][0].cpu().numpy(), ref, "listed edges", scene, batch, 0, 0,
             min_hits=5)
    assert ref.hit[0, 0] > 0.3 and ref.hit[0, 1] > 0.3              # the seam rays see the splat behind
    R.remove_scene(sid)


def test_listed_rays_equal_the_grid_they_list(R):
    """A rotating grid's rays (their binary32 angles, as the kernel forms
    them), listed in a shuffled order and another band shape, give the grid's
    own results ray for ray, and both give the same bits with 8 x 8 ray
    tiles: the evaluation per (ray, Gaussian) does not depend on how the rays
    are binned."""
    scene = synth.make_scene(54, 3_000, 2, 500, sh_degree=0, half_box=3.0)
    rng = np.random.default_rng(9)
    E = 2
    grid = synth.rotating_lidar(16, 96, -25, 15)
    c = np.arange(grid.width, dtype=np.float32)
    az = np.float32(grid.az0) + (c + np.float32(0.5)) * np.float32(grid.az_step)
    az_all = np.broadcast_to(az[None, :], (grid.height, grid.width)).reshape(-1)
    el_all = np.broadcast_to(np.asarray(grid.elevations, np.float32)[:, None], (grid.height, grid.width)).reshape(-1)
    perm = rng.permutation(az_all.size)
    from paper_2604_25459_amd import gsr
    listed = gsr.LidarRays(width=64, height=24, ray_az=az_all[perm].reshape(24, 64),
                           ray_el=el_all[perm].reshape(24, 64), near_range=grid.near_range)
    vm1 = synth.sensor_viewmats(rng, E, 0.5, 2.5, 0.1)
    batch = synth.LidarBatch(cams=[grid, listed], viewmats=np.stack([vm1, vm1]),
                             poses=synth.random_poses(rng, E, scene.n_bodies))
    sid = R.add_synth_scene(scene)
    vm_t, poses_t = _tensors(batch)
    out = R.render_lidar(sid, [grid, listed], vm_t, poses_t)
    for e in range(E):
        g_rng = out[0][0][e].cpu().numpy().reshape(-1)[perm]
        g_hit = out[0][1][e].cpu().numpy().reshape(-1)[perm]
        l_rng = out[1][0][e].cpu().numpy().reshape(-1)
        l_hit = out[1][1][e].cpu().numpy().reshape(-1)
        print(f"[listed = grid] env {e} hits {(g_hit > 0.1).sum()} max |d range| {np.abs(l_rng - g_rng).max():.2e} "
              f"max |d hit| {np.abs(l_hit - g_hit).max():.2e}", flush=True)
        assert (g_hit > 0.1).sum() >= 20
        np.testing.assert_array_equal(l_rng, g_rng)
        np.testing.assert_array_equal(l_hit, g_hit)
    R.remove_scene(sid)
    # 8 x 8 ray tiles (other bands per tile row, other tile azimuth tables): the same bits again
    R8 = gsr.Renderer(0, tile_size=8)
    try:
        sid8 = R8.add_synth_scene(scene)
        out8 = R8.render_lidar(sid8, [grid, listed], vm_t, poses_t)
        for l in range(2):
            for k in range(2):
                np.testing.assert_array_equal(out8[l][k].cpu().numpy(), out[l][k].cpu().numpy())
        R8.remove_scene(sid8)
    finally:
        R8.close()


def _sampled_compare(R, scene, batch, lidars, got, n_samples, label, seed=0):
    """Sampled rays of every slot and env against the per-ray oracle (the
    primary result or one of its admissible variants)."""
    from oracle import lidar_ray_variants
    rng = np.random.default_rng(seed)
    E = batch.n_envs
    checked = hits = 0
    for l, lid in enumerate(lidars):
        rng_l, hit_l = got[l]
        for e in range(E):
            rows = rng.integers(0, lid.height, n_samples)
            cols = rng.integers(0, lid.width, n_samples)
            for r, c in zip(rows, cols):
                rr, hh = lidar_ray_variants(scene, batch, l, e, int(r), int(c))
                gr, gh = float(rng_l[e, r, c]), float(hit_l[e, r, c])
                ok = (np.abs(gh - hh) <= HIT_TOL) & (np.abs(gr - rr) / np.maximum(1.0, rr) <= RANGE_REL)
                assert ok.any(), (label, l, e, int(r), int(c), gr, gh, rr[0], hh[0])
                checked += 1
                hits += hh[0] > 0.1
    print(f"[{label}] sampled rays {checked}, hit {hits}", flush=True)
    assert hits >= checked // 10


def test_heightmap_grid_and_rotating_slots_match_oracle(R):
    """A heightmap grid and a rotating sensor in one call (both ray kinds in one
    launch): every ray of both against the float64 oracle."""
    scene = synth.make_scene(57, 4_000, 3, 800, sh_degree=0, half_box=2.0)
    rng = np.random.default_rng(9)
    E = 3
    grid = synth.height_grid(24, 40, 0.08)
    rot = synth.rotating_lidar(8, 96, -30, 10)
    vm = synth.sensor_viewmats(rng, E, 0.0, 1.5, 1.2)     # sensors 1.2 m up, within 1.5 m of the axis
    batch = synth.LidarBatch(cams=[grid, rot], viewmats=np.stack([vm, vm]), poses=synth.random_poses(rng, E, 3))
    vmt, pt = _tensors(batch)
    got = R.render_lidar(R.add_synth_scene(scene), [grid, rot], vmt, pt)
    for l in range(2):
        for e in range(E):
            ref = lidar_ref(scene, batch, l, e)
            _compare(got[l][0][e].cpu().numpy(), got[l][1][e].cpu().numpy(), ref, f"slot {l} env {e}", scene,
                     batch, l, e, min_hits=10)


def test_heightmap_sheet_reads_its_height(R):
    """A flat sheet of Gaussians 0.7 m below the sensor plane: every ray over
    the sheet reads range 0.7 (its centres' depth) and a high hit fraction."""
    xs = np.arange(-1.0, 1.001, 0.04)
    means = [[x, y, -0.7] for x in xs for y in xs]
    scene = scene_from(means, [[0.04, 0.04, 0.003]] * len(means), opac=0.35, degree=0)
    grid = synth.height_grid(32, 32, 0.05)
    batch = synth.LidarBatch(cams=[grid], viewmats=np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None, None]
                             .astype(np.float32), poses=np.zeros((1, 0, 7), np.float32))
    vmt, pt = _tensors(batch)
    (rg, hit), = R.render_lidar(R.add_synth_scene(scene), [grid], vmt, pt)
    rg, hit = rg[0].cpu().numpy(), hit[0].cpu().numpy()
    assert (hit > 0.5).all()
    np.testing.assert_allclose(rg, np.float32(0.7), rtol=1e-5)
    ref = lidar_ref(scene, batch)
    _compare(rg, hit, ref, "sheet", scene, batch, 0, 0)


def test_lidar_at_benchmark_scale_sampled(R):
    """The benchmark's sensors on the 300k-Gaussian workload-2 scene (long
    tile-row lists, segmented scatter): a rotating 32 x 1024 LiDAR, a 64 x 64
    heightmap grid and a 96 x 256 rosette of listed rays, rays sampled in
    every env against the oracle."""
    scene, _ = synth.make_config(2, n_envs=1)
    rng = np.random.default_rng(11)
    E = 3
    rot = synth.rotating_lidar(32, 1024, -25.0, 15.0)
    grid = synth.height_grid(64, 64, 0.05)
    ros = synth.rosette_lidar(96, 256, 35.0)
    vm = synth.sensor_viewmats(rng, E, 0.5, 3.0, 0.2)
    poses = synth.make_poses(2, 0, E, scene.n_bodies)
    batch = synth.LidarBatch(cams=[rot, grid, ros], viewmats=np.stack([vm, vm, vm]), poses=poses)
    vmt, pt = _tensors(batch)
    got = R.render_lidar(R.add_synth_scene(scene), [rot, grid, ros], vmt, pt)
    got = [(r.cpu().numpy(), h.cpu().numpy()) for r, h in got]
    _sampled_compare(R, scene, batch, [rot, grid, ros], got, 24, "benchmark scale")
