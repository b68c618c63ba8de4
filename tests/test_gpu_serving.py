"""Serving loop (continuous batching) on the GPU: every request's images are
identical, bit for bit, to rendering that request alone; requests arriving
while batches run are merged; memory admission rejects what can never fit."""
import numpy as np
import pytest

from paper_2604_25459_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _scene(seed, n_static, n_bodies):
    return synth.make_scene(seed, n_static, n_bodies, 2_000, sh_degree=3, half_box=4.0)


def _request(rng, scene, envs, sizes):
    cams = [synth.pinhole(w, h, 60.0) for (w, h) in sizes]
    vm = np.stack([synth.orbit_viewmats(rng, envs, 3.0, 6.0) for _ in cams], axis=0)
    poses = synth.random_poses(rng, envs, scene.n_bodies)
    return synth.Batch(cams=cams, viewmats=vm, poses=poses, bg=np.array([0.1, 0.2, 0.3], np.float32))


def test_server_results_equal_solo_renders():
    torch = _torch()
    from paper_2604_25459_amd import gsr
    R = gsr.Renderer(0)
    scenes = [_scene(11, 20_000, 4), _scene(12, 30_000, 2)]
    sids = [R.add_synth_scene(s) for s in scenes]
    rng = np.random.default_rng(5)
    size_sets = [[(128, 128)], [(320, 240)], [(96, 64)], [(128, 128), (320, 240)]]
    reqs = []
    # two large requests first keep both workers busy so the rest queue up and merge
    for k in range(14):
        si = 0 if k < 10 else 1
        envs = 48 if k < 2 else int(rng.integers(1, 9))
        reqs.append((si, _request(rng, scenes[si], envs, size_sets[k % len(size_sets)])))
    S = gsr.Server(R, n_streams=2)
    tickets, outs = [], []
    for si, b in reqs:
        cams, vm, poses = gsr.batch_tensors(b)
        rgb, depth, alpha = R.alloc_outputs(cams, b.n_envs, alpha=True)
        tickets.append(S.submit(sids[si], cams, vm, poses, rgb, depth, alpha, bg=tuple(b.bg)))
        outs.append((cams, vm, poses, rgb, depth, alpha))
    infos = [S.wait(t) for t in tickets]
    st = S.stats()
    print("server stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert st["batches"] < len(reqs), "no request was merged"
    assert max(i["batch_requests"] for i in infos) > 1
    assert st["latency_p99_us"] >= st["latency_p50_us"] > 0
    for (si, b), (cams, vm, poses, rgb, depth, alpha), info in zip(reqs, outs, infos):
        assert info["status"] == 0
        assert info["t_submit_us"] <= info["t_admit_us"] <= info["t_start_us"] <= info["t_complete_us"]
        solo = R.render(sids[si], cams, vm, poses, bg=tuple(b.bg), alpha=True)
        got = R.split(cams, b.n_envs, rgb, depth, alpha)
        for (r0, d0, a0), (r1, d1, a1) in zip(solo, got):
            assert torch.equal(r0, r1) and torch.equal(d0, d1) and torch.equal(a0, a1)
    S.close()
    R.close()


def test_server_memory_admission():
    """A request larger than the server's memory budget is rendered in chunks
    that fit it (and equals its solo render); one whose single image can never
    fit is rejected; the memory in flight never exceeds the budget."""
    torch = _torch()
    from paper_2604_25459_amd import gsr
    R = gsr.Renderer(0)
    scene = _scene(13, 20_000, 2)
    sid = R.add_synth_scene(scene)
    huge = synth.make_scene(14, 800_000, 0, 0, sh_degree=0, half_box=4.0)
    hid = R.add_synth_scene(huge)
    budget = 96 << 20
    S = gsr.Server(R, n_streams=2, memory_budget=budget)
    rng = np.random.default_rng(9)
    one = _request(rng, huge, 1, [(640, 480)])      # one image of an 800k-Gaussian scene: > 96 MiB
    cams, vm, poses = gsr.batch_tensors(one)
    rgb, depth, _ = R.alloc_outputs(cams, one.n_envs)
    with pytest.raises(gsr.GsrError) as ei:
        S.submit(hid, cams, vm, poses, rgb, depth)
    assert ei.value.code == gsr.GSR_E_REJECTED
    big = _request(rng, scene, 64, [(640, 480)])    # 64 images: more than the budget, rendered in chunks
    bc, bv, bp = gsr.batch_tensors(big)
    brgb, bdepth, _ = R.alloc_outputs(bc, big.n_envs)
    tickets = [S.submit(sid, bc, bv, bp, brgb, bdepth, bg=tuple(big.bg))]
    keep = []
    for k in range(6):
        b = _request(rng, scene, 4, [(320, 240)])
        c, v, p = gsr.batch_tensors(b)
        o = R.alloc_outputs(c, b.n_envs)
        keep.append((c, v, p, o))
        tickets.append(S.submit(sid, c, v, p, o[0], o[1]))
    for t in tickets:
        S.wait(t)
    st = S.stats()
    assert st["rejected"] == 1 and st["completed"] == 7
    assert 0 < st["in_flight_bytes_max"] <= budget
    solo = R.render(sid, bc, bv, bp, bg=tuple(big.bg))
    got = R.split(bc, big.n_envs, brgb, bdepth)
    assert torch.equal(solo[0][0], got[0][0]) and torch.equal(solo[0][1], got[0][1])
    with pytest.raises(gsr.GsrError) as ei:
        S.wait(tickets[0])
    assert ei.value.code == gsr.GSR_E_NOT_FOUND
    S.close()
    R.close()
