#!/usr/bin/env python3
"""Throughput benchmark of the batched 3D Gaussian Splatting renderer.

A step renders every environment of the workload once, with new body poses
(poses are resampled each step, cameras fixed per env), inputs already
resident in HBM.  Default workload: 2048 envs x 1 camera at 640x480, a
200k-Gaussian background plus 10 rigid bodies x 10k Gaussians, SH degree 3,
float32 storage (seeded synthetic scene, standing in for the paper's
reconstructed scenes).

Prints one JSON line: env-frames/s (whole job), the plain per-env path's rate
on the same GPU, per-stage device times, the roofline of the dominant kernel
and the CPU oracle's rate on a bounded sample.
"""
import argparse
import csv
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# Algorithmic floating-point work of one per-pixel evaluation of a list entry
# (offset 2, quadratic form with pre-scaled conic 7 counting an FMA as 2,
# adding log2(o) 1, exp2 1) and of one accepted Gaussian (1 - a 1, T' 1,
# weight 1, four accumulations 8).
FLOPS_EVAL = 11
FLOPS_ACCEPT = 11
# Sources that fix what the rasteriser reads and writes: a counter summary
# taken on other sources gives no traffic figure.
RASTER_SOURCES = ("paper_2604_25459_amd/csrc/k_raster.hip",)
PMC_SUMMARY = "profiles/k_raster_cfg2_2048env_640x480_f32_pmc.json"
UTIL_SUMMARY = "profiles/k_raster_cfg2_2048env_640x480_f32_valu_lds.json"
UTIL_COUNTERS = ("SQ_ACTIVE_INST_VALU", "SQ_LDS_IDX_ACTIVE", "SQ_INSTS_LDS_LOAD_BANDWIDTH", "SQ_BUSY_CU_CYCLES",
                 "GRBM_GUI_ACTIVE")
# LDS read bandwidth of a CDNA4 compute unit (bytes per clock)
LDS_BYTES_PER_CLK = 256
CALIB_BYTES = 1 << 30


def raster_source_hash():
    h = hashlib.sha256()
    for rel in RASTER_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _pmc_rows(path, counter):
    with open(path, newline="") as f:
        rows = [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def pmc_summary(fetch_csv, write_csv, out_path, command):
    """Condense two counter runs of the same bench command (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch) into HBM bytes per rasteriser launch.  Each
    counter is scaled by what it reads for the calibration copy (the first
    device-to-device copy kernel, 1 GiB read and 1 GiB written)."""
    out = {"command": command, "source_sha256": raster_source_hash(), "sources": list(RASTER_SOURCES)}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _pmc_rows(path, counter)
        calib = next(r for r in rows if "copyBuffer" in r["Kernel_Name"])
        kib = float(calib["Counter_Value"])
        factor = (CALIB_BYTES / 1024.0) / kib
        if not 0.25 <= factor <= 4.0:
            raise SystemExit(f"{counter}: calibration copy read {kib} KiB, not near 1 GiB")
        rast = [float(r["Counter_Value"]) for r in rows if "k_raster" in r["Kernel_Name"]]
        if not rast:
            raise SystemExit(f"{counter}: no rasteriser dispatch in {path}")
        key = counter.split("_")[0].lower()
        out[f"{key}_calibration_kib"] = kib
        out[f"{key}_factor"] = factor
        out[f"{key}_kib_per_dispatch"] = sum(rast) / len(rast)
        out[f"{key}_dispatches"] = len(rast)
        out[f"{key}_bytes_per_launch"] = sum(rast) / len(rast) * 1024.0 * factor
    out["traffic_bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def util_summary(counter_csv, agent_csv, out_path, command):
    """Condense one counter run (UTIL_COUNTERS) into the rasteriser's VALU
    and LDS use per launch.  The SQ counters are summed over the SIMDs of
    the chip; GRBM_GUI_ACTIVE over its XCDs, so it divided by their number is
    the launch's duration in shader clocks.  VALU busy = quad-cycles of VALU
    issue x 4 / (SIMDs x clocks); LDS busy = cycles with indexed LDS work /
    (CUs x clocks); LDS bytes = 64-byte units loaded x 64."""
    with open(agent_csv) as f:
        agent = next(r for r in csv.DictReader(f) if r["Agent_Type"] == "GPU")
    n_xcc, cus = int(agent["Num_Xcc"]), int(agent["Cu_Count"])
    simds = cus * int(agent["Simd_Per_Cu"])
    clk_mhz = float(agent["Max_Engine_Clk_Fcompute"])
    per = {}
    with open(counter_csv) as f:
        for r in csv.DictReader(f):
            if "k_raster<" not in r["Kernel_Name"]:
                continue
            d = per.setdefault(r["Dispatch_Id"], {})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
            d["ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    launches = [d for d in per.values() if all(c in d for c in UTIL_COUNTERS)]
    if not launches:
        raise SystemExit(f"no rasteriser dispatch with all of {UTIL_COUNTERS} in {counter_csv}")
    rows = []
    for d in launches:
        clocks = d["GRBM_GUI_ACTIVE"] / n_xcc
        rows.append({"ms": d["ns"] * 1e-6, "clock_ghz": clocks / d["ns"],
                     "valu_busy": d["SQ_ACTIVE_INST_VALU"] * 4.0 / (simds * clocks),
                     "cu_busy": d["SQ_BUSY_CU_CYCLES"] * 4.0 / (simds * clocks),
                     "lds_busy": d["SQ_LDS_IDX_ACTIVE"] / (cus * clocks),
                     "lds_bytes": d["SQ_INSTS_LDS_LOAD_BANDWIDTH"] * 64.0})
    mean = {k: sum(r[k] for r in rows) / len(rows) for k in rows[0]}
    lds_gbs = mean["lds_bytes"] / (mean["ms"] * 1e-3) / 1e9
    lds_peak = cus * LDS_BYTES_PER_CLK * clk_mhz * 1e6 / 1e9
    out = {"command": command, "source_sha256": raster_source_hash(), "sources": list(RASTER_SOURCES),
           "counters": list(UTIL_COUNTERS), "dispatches": len(rows), "cus": cus, "simds": simds, "xcds": n_xcc,
           "avg_ms": mean["ms"], "clock_ghz": mean["clock_ghz"], "valu_busy": mean["valu_busy"],
           "cu_busy": mean["cu_busy"], "lds_busy": mean["lds_busy"], "lds_read_bytes_per_launch": mean["lds_bytes"],
           "lds_read_gbs": lds_gbs, "lds_peak_gbs": lds_peak, "lds_read_frac": lds_gbs / lds_peak,
           "lds_peak_basis": f"{cus} CUs x {LDS_BYTES_PER_CLK} B/clock x {clk_mhz:.0f} MHz"}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def measured_util():
    """VALU / LDS use of the rasteriser from the committed counter summary,
    or None when it was taken on other rasteriser sources."""
    path = os.path.join(ROOT, UTIL_SUMMARY)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        s = json.load(f)
    if s.get("source_sha256") != raster_source_hash():
        return None
    return {k: s[k] for k in ("valu_busy", "lds_busy", "lds_read_gbs", "lds_peak_gbs", "lds_read_frac", "clock_ghz")}


def measured_traffic(tuning):
    """HBM bytes per rasteriser launch from the committed counter summary, or
    None when it was taken on other rasteriser sources or launch parameters."""
    path = os.path.join(ROOT, PMC_SUMMARY)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        s = json.load(f)
    if s.get("source_sha256") != raster_source_hash():
        return None
    if tuning is not None and s.get("tuning") is not None:
        # only the launch parameters of the rasteriser itself matter here
        keys = ("tile_size", "lds_batch", "persistent")
        if any(s["tuning"].get(k) != tuning.get(k) for k in keys):
            return None
    return s["traffic_bytes_per_launch"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_serving(R, args):
    """Replay the first `serve_seconds` of the seeded Poisson trace (200 req/s,
    1-256 envs, 128x128 / 320x240 / 640x480, FP16 scenes of 50k-1M Gaussians
    plus 4-16 bodies) in real time through the continuous-batching server.
    Latency = submission to completion on the device."""
    import threading
    import numpy as np
    import torch
    from paper_2604_25459_amd import gsr, synth

    dev = torch.device("cuda", 0)
    trace = [r for r in synth.serving_trace() if r.arrival_s < args.serve_seconds]
    K = max(1, min(args.serve_scenes, 32))
    log(f"[serve] {len(trace)} requests over {args.serve_seconds:.0f} s, pool of {K} resident scenes (FP16)")
    scenes = [synth.serving_pool_scene(k) for k in range(K)]
    sids = [R.add_synth_scene(sc, "f16") for sc in scenes]
    prepared = []
    for idx, req in enumerate(trace):
        sc = scenes[req.scene % K]
        b = synth.serving_batch(req, sc, idx)
        prepared.append((req, req.scene % K, b))
    S = gsr.Server(R, n_streams=args.serve_streams)
    # warm the server's workspaces (one request per resolution)
    for w, h in synth.SERVE_RESOLUTIONS:
        b = synth.serving_batch(synth.Request(0.0, 4, w, h, 0), scenes[0], 10**6 + w)
        cams, vm, poses = gsr.batch_tensors(b)
        rgb, depth, _ = R.alloc_outputs(cams, b.n_envs)
        torch.cuda.synchronize()
        S.wait(S.submit(sids[0], cams, vm, poses, rgb, depth))
    base = S.stats()
    tickets = []
    lock = threading.Lock()
    done_images = [0]
    lat = []
    t0 = time.perf_counter()

    def producer():
        for req, si, b in prepared:
            now = time.perf_counter() - t0
            if req.arrival_s > now:
                time.sleep(req.arrival_s - now)
            cams, vm, poses = gsr.batch_tensors(b)
            rgb, depth, _ = R.alloc_outputs(cams, b.n_envs)
            torch.cuda.current_stream(dev).synchronize()
            t = S.submit(sids[si], cams, vm, poses, rgb, depth)
            with lock:
                tickets.append((t, b.n_envs * b.n_cams))
        with lock:
            tickets.append((None, 0))

    th = threading.Thread(target=producer)
    th.start()
    k = 0
    while True:
        with lock:
            item = tickets[k] if k < len(tickets) else False
        if item is False:
            time.sleep(0.0005)
            continue
        t, n_img = item
        if t is None:
            break
        info = S.wait(t)
        lat.append(info["t_complete_us"] - info["t_submit_us"])
        done_images[0] += n_img
        k += 1
    wall = time.perf_counter() - t0
    th.join()
    st = S.stats()
    S.close()
    for sid in sids:
        R.remove_scene(sid)
    n = st["completed"] - base["completed"]
    lat_ms = np.asarray(lat, np.float64) / 1000.0
    out = {"requests": n, "arrival_rate_hz": 200.0, "trace_seconds": args.serve_seconds, "scenes": K,
           "streams": args.serve_streams, "latency_p50_ms": float(np.percentile(lat_ms, 50)),
           "latency_p99_ms": float(np.percentile(lat_ms, 99)), "latency_max_ms": float(lat_ms.max()),
           "env_frames_per_s": done_images[0] / wall, "wall_s": wall,
           "mean_batch_requests": st["mean_batch_requests"], "batches": st["batches"] - base["batches"]}
    log(f"[serve] {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--envs", type=int, default=0, help="truncate the workload's env count (0 = full)")
    ap.add_argument("--plain-envs", type=int, default=64, help="envs timed on the plain per-env path (0 = skip)")
    ap.add_argument("--cpu-images", type=int, default=3, help="images rendered by the CPU oracle (0 = skip)")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="seconds of the Poisson serving trace replayed in real time (0 = skip)")
    ap.add_argument("--serve-scenes", type=int, default=8, help="resident scenes in the serving pool (trace uses 32)")
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--no-autotune", action="store_true", help="skip the launch-parameter autotuner")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first copy 1 GiB device to device (calibrates the memory counters)")
    ap.add_argument("--no-count", action="store_true", help="skip the counting renders of the roofline")
    ap.add_argument("--obs-steps", type=int, default=3, help="steps timed with the u8 observation epilogue (0 = skip)")
    ap.add_argument("--lidar-steps", type=int, default=3, help="steps of the batch-LiDAR leg (0 = skip)")
    ap.add_argument("--no-storage-check", dest="storage_check", action="store_false",
                    help="skip the FP16/BF16 storage leg (throughput and per-image error)")
    ap.add_argument("--no-graphs", action="store_true", help="launch every stage eagerly (no graph replay)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run every memory chunk on the render stream (no two-stream chunk overlap)")
    ap.add_argument("--no-one-stream-leg", dest="one_stream_leg", action="store_false",
                    help="skip the comparison leg that runs the same steps on one stream")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the counter summary of two rocprofv3 --pmc runs of this bench and exit")
    ap.add_argument("--pmc-util-summary", nargs=2, metavar=("COUNTER_CSV", "AGENT_CSV"),
                    help="write the VALU / LDS summary of one rocprofv3 --pmc run of this bench and exit")
    ap.add_argument("--pmc-out", default=None, help="output of --pmc-summary / --pmc-util-summary")
    ap.add_argument("--pmc-command", default="", help="command line recorded in the counter summary")
    ap.add_argument("--pmc-tuning", default="", help="JSON of the launch parameters the counted run used")
    args = ap.parse_args()

    if args.pmc_util_summary:
        util_summary(args.pmc_util_summary[0], args.pmc_util_summary[1],
                     args.pmc_out or os.path.join(ROOT, UTIL_SUMMARY), args.pmc_command)
        return
    if args.pmc_summary:
        args.pmc_out = args.pmc_out or os.path.join(ROOT, PMC_SUMMARY)
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.pmc_out, args.pmc_command)
        if args.pmc_tuning:
            with open(args.pmc_out) as f:
                s = json.load(f)
            s["tuning"] = json.loads(args.pmc_tuning)
            with open(args.pmc_out, "w") as f:
                json.dump(s, f, indent=1)
                f.write("\n")
        return

    if args.gpus != 1:
        print(json.dumps({"error": "libgsr renders on one GPU per process and this benchmark times one GPU; "
                          "run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2604_25459_amd import gsr, synth

    if args.calibration_copy:
        x = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)                       # device-to-device copy kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del x, y
        log("[bench] calibration: 1 GiB device-to-device copy done")

    log(f"[bench] config {args.config}: generating workload")
    scene, batch = synth.make_config(args.config, n_envs=args.envs or None)
    E, C = batch.n_envs, batch.n_cams
    R = gsr.Renderer(0, tile_size=args.tile, profile=True, graphs=not args.no_graphs, overlap=not args.no_overlap)
    sid = R.add_synth_scene(scene, args.storage)
    cams, vm, _ = gsr.batch_tensors(batch)
    dev = torch.device("cuda", 0)
    n_pose_steps = args.warmup + args.steps
    poses = [torch.from_numpy(synth.make_poses(args.config, s, E, scene.n_bodies)).to(dev)
             for s in range(n_pose_steps)]
    rgb, depth, _ = R.alloc_outputs(cams, E)
    stream = torch.cuda.current_stream(dev)

    tuning = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tuning = R.autotune(sid, cams, vm, poses[0], rgb, depth)
        log(f"[bench] autotuned in {time.perf_counter() - t0:.1f} s: {tuning}")
    log(f"[bench] warmup {args.warmup} steps of {E} envs x {C} cams")
    for s in range(args.warmup):
        R.render_into(sid, cams, vm, poses[s], rgb, depth, None, tuple(batch.bg))
    torch.cuda.synchronize()
    R.stage_times(reset=True)

    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        R.render_into(sid, cams, vm, poses[args.warmup + s], rgb, depth, None, tuple(batch.bg))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = R.stage_times(reset=True)
    sec = t1 - t0
    value = E * args.steps / sec
    ms_per_step = 1000.0 * sec / args.steps
    log(f"[bench] {value:.1f} env-frames/s, {ms_per_step:.2f} ms/step, stages {st}")

    # the same steps with every chunk on the render stream: the gain of the
    # two-stream overlap, and a stage breakdown in which no stages share the GPU
    one_stream = None
    if not args.no_overlap and args.one_stream_leg:
        R1 = gsr.Renderer(0, tile_size=args.tile, profile=True, graphs=not args.no_graphs, overlap=False)
        sid1 = R1.add_synth_scene(scene, args.storage)
        if tuning:
            R1.set_tuning(sid1, cams, vm, poses[0], **{k: v for k, v in tuning.items() if k != "ms"})
        R1.render_into(sid1, cams, vm, poses[0], rgb, depth, None, tuple(batch.bg))
        torch.cuda.synchronize()
        R1.stage_times(reset=True)
        t0 = time.perf_counter()
        for s in range(args.steps):
            R1.render_into(sid1, cams, vm, poses[args.warmup + s], rgb, depth, None, tuple(batch.bg))
        torch.cuda.synchronize()
        osec = time.perf_counter() - t0
        ost = R1.stage_times(reset=True)
        one_stream = {"value": E * args.steps / osec, "unit": "env-frames/s",
                      "ms_per_step": 1000.0 * osec / args.steps,
                      "stages_ms_per_step": {k: v / args.steps for k, v in ost.items() if k in R.STAGES}}
        R1.close()
        del R1
        log(f"[bench] one stream: {one_stream['value']:.1f} env-frames/s, stages {one_stream['stages_ms_per_step']}")

    # policy-ready observations: same workload, u8 pixels with per-image exposure /
    # contrast / brightness randomisation fused into the rasteriser, no float colour
    observation = None
    if args.obs_steps:
        g = torch.Generator().manual_seed(7)
        n_img = E * C
        gain = (2.0 ** (torch.rand(n_img, generator=g) - 0.5)).to(dev)
        contrast = (0.8 + 0.4 * torch.rand(n_img, generator=g)).to(dev)
        bright = (0.1 * torch.rand(n_img, generator=g) - 0.05).to(dev)
        obs_out = torch.empty(rgb.numel(), dtype=torch.uint8, device=dev)
        obs = gsr.Observation("u8", obs_out, gain, contrast, bright)
        R.render_into(sid, cams, vm, poses[args.warmup], None, depth, None, tuple(batch.bg), obs=obs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.obs_steps):
            R.render_into(sid, cams, vm, poses[args.warmup + s % args.steps], None, depth, None, tuple(batch.bg),
                          obs=obs)
        torch.cuda.synchronize()
        osec = time.perf_counter() - t0
        R.stage_times(reset=True)
        observation = {"value": E * args.obs_steps / osec, "unit": "env-frames/s", "format": "u8",
                       "steps": args.obs_steps, "randomisation": "gain 2^U[-0.5,0.5], contrast U[0.8,1.2], "
                                                                  "brightness U[-0.05,0.05] per image"}
        del obs_out
        log(f"[bench] observation path (u8 + randomisation) {observation['value']:.1f} env-frames/s")

    # batch LiDAR on the same scene and poses: one rotating 32 x 1024 sensor per env
    lidar = None
    if args.lidar_steps:
        lid = synth.rotating_lidar(32, 1024, -25.0, 15.0)
        lrng = np.random.default_rng(11)
        lvm = torch.from_numpy(synth.sensor_viewmats(lrng, E, 0.5, 3.0, 0.2)[None]).to(dev)
        n_rays = E * lid.width * lid.height
        l_range = torch.empty(n_rays, dtype=torch.float32, device=dev)
        l_hit = torch.empty(n_rays, dtype=torch.float32, device=dev)
        R.render_lidar_into(sid, [lid], lvm, poses[args.warmup], l_range, l_hit)
        torch.cuda.synchronize()
        R.stage_times(reset=True)
        t0 = time.perf_counter()
        for s in range(args.lidar_steps):
            R.render_lidar_into(sid, [lid], lvm, poses[args.warmup + s % args.steps], l_range, l_hit)
        torch.cuda.synchronize()
        lsec = time.perf_counter() - t0
        lst = R.stage_times(reset=True)
        lidar = {"value": E * args.lidar_steps / lsec, "unit": "env-scans/s",
                 "rays_per_s": n_rays * args.lidar_steps / lsec, "steps": args.lidar_steps,
                 "sensor": "rotating, 32 beams [-25, 15] deg x 1024 columns", "envs": E,
                 "ms_per_step": 1000.0 * lsec / args.lidar_steps,
                 "stages_ms_per_step": {k: v / args.lidar_steps for k, v in lst.items() if k in R.STAGES},
                 "hit_fraction": float((l_hit > 0.5).float().mean())}
        del l_range, l_hit
        log(f"[bench] LiDAR {lidar['value']:.1f} env-scans/s ({lidar['rays_per_s'] / 1e9:.2f} G rays/s)")

    # half-precision storage: throughput of the same step, and the per-image
    # error of every image against the float32-storage render of the same
    # step (storage error; both are checked against the oracle in the tests)
    storage = None
    if args.storage_check and args.storage == "f32":
        storage = {}
        ref_rgb = rgb.clone()                    # last timed step, float32 storage
        last = poses[args.warmup + args.steps - 1]
        for st_name in ("f16", "bf16"):
            hsid = R.add_synth_scene(scene, st_name)
            R.render_into(hsid, cams, vm, last, rgb, depth, None, tuple(batch.bg))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(args.steps):
                R.render_into(hsid, cams, vm, poses[args.warmup + s], rgb, depth, None, tuple(batch.bg))
            torch.cuda.synchronize()
            hsec = time.perf_counter() - t0
            R.stage_times(reset=True)
            per_img = []
            base = 0
            for cam in cams:                     # per camera slot: [E, H*W*3]
                n = E * cam.width * cam.height * 3
                d = (rgb[base:base + n] - ref_rgb[base:base + n]).view(E, -1).double()
                per_img.append((d.abs().amax(dim=1), d.abs().mean(dim=1), (d * d).mean(dim=1)))
                base += n
            mx = torch.cat([p[0] for p in per_img]).cpu().numpy()
            ma = torch.cat([p[1] for p in per_img]).cpu().numpy()
            mse = torch.cat([p[2] for p in per_img]).cpu().numpy()
            psnr = 10.0 * np.log10(1.0 / np.maximum(mse, 1e-30))
            storage[st_name] = {"value": E * args.steps / hsec, "unit": "env-frames/s",
                                "scene_bytes": R.scene_info(hsid)[2],
                                "error_vs_f32_storage_per_image": {
                                    "images": int(mx.size), "max_abs_max": float(mx.max()),
                                    "mean_abs_mean": float(ma.mean()), "psnr_db_min": float(psnr.min()),
                                    "psnr_db_median": float(np.median(psnr))}}
            R.remove_scene(hsid)
            log(f"[bench] {st_name} storage: {storage[st_name]}")
        del ref_rgb

    # plain per-env path on a subset (same GPU, same kernels, one image per launch chain)
    plain = None
    if args.plain_envs:
        pe = min(args.plain_envs, E)
        sub = batch.subset(range(pe))
        pcams, pvm, _ = gsr.batch_tensors(sub)
        prgb, pdep, _ = R.alloc_outputs(pcams, pe)
        pposes = poses[args.warmup][:pe].contiguous()
        R.render_into(sid, pcams, pvm, pposes, prgb, pdep, None, tuple(batch.bg), plain=True)
        torch.cuda.synchronize()
        R.stage_times(reset=True)
        t0 = time.perf_counter()
        R.render_into(sid, pcams, pvm, pposes, prgb, pdep, None, tuple(batch.bg), plain=True)
        torch.cuda.synchronize()
        psec = time.perf_counter() - t0
        R.stage_times(reset=True)
        plain = {"value": pe / psec, "unit": "env-frames/s", "envs_timed": pe}
        log(f"[bench] plain path {plain['value']:.1f} env-frames/s over {pe} envs")

    serving = run_serving(R, args) if args.serve_seconds > 0 else None

    # oracle on the host cores, bounded sample of the same workload
    cpu = None
    if args.cpu_images:
        from oracle import oracle_threads, render_ref
        b0 = synth.make_config(args.config, n_envs=args.envs or None, step=args.warmup)[1]
        cores = oracle_threads()
        t0 = time.perf_counter()
        for k in range(args.cpu_images):
            render_ref(scene, b0, 0, (k * 997) % E, args.tile, variants=False)
        csec = time.perf_counter() - t0
        cpu = {"value": args.cpu_images / csec, "unit": "env-frames/s", "cores": cores, "kind": "oracle",
               "sample": f"{args.cpu_images} envs of step {args.warmup} (float32 binning spec on one thread + "
                         f"float64 compositing on {cores} OpenMP threads)"}
        log(f"[bench] oracle {cpu['value']:.3f} env-frames/s on {cores} cores")

    # roofline of the dominant kernel (the rasteriser, bound by vector ALU
    # work): exact per-pixel work of every timed step, from counting renders
    # of the same poses with the same launch parameters (untimed)
    roof = None
    raster_ms = st["raster"] / max(st["raster_launches"], 1)
    if not args.no_count and raster_ms > 0:
        npx = rgb.numel() // 3
        work = torch.empty(npx * 2, dtype=torch.int32, device=dev)
        visits = accepts = 0
        for s in range(args.steps):
            R.render_into(sid, cams, vm, poses[args.warmup + s], rgb, depth, None, tuple(batch.bg), work=work)
            w = work.view(npx, 2)
            visits += int(w[:, 0].sum(dtype=torch.int64))
            accepts += int(w[:, 1].sum(dtype=torch.int64))
        torch.cuda.synchronize()
        R.stage_times(reset=True)
        del work
        flops_step = (visits * FLOPS_EVAL + accepts * FLOPS_ACCEPT) / args.steps
        launches_per_step = st["raster_launches"] / args.steps
        flops_launch = flops_step / launches_per_step
        achieved = flops_launch / (raster_ms * 1e-3) / 1e12
        traffic = measured_traffic(tuning)
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": "k_raster", "avg_ms": raster_ms, "launches_per_step": launches_per_step,
                "flop_per_launch": flops_launch,
                "visits_per_pixel": visits / (npx * args.steps), "accepts_per_pixel": accepts / (npx * args.steps),
                "units": "list entries up to each pixel's termination x 11 flop + blended Gaussians x 11 flop"}
        if traffic is not None:
            # counted HBM bytes over the launch time measured here
            roof["hbm_gbs"] = traffic / (raster_ms * 1e-3) / 1e9
            roof["hbm_frac"] = roof["hbm_gbs"] / HBM_PEAK_GBS
        roof["valu_lds"] = measured_util()
        log(f"[bench] raster {roof['visits_per_pixel']:.1f} visits, {roof['accepts_per_pixel']:.1f} blends per "
            f"pixel; {achieved:.2f} TFLOP/s algorithmic over {raster_ms:.2f} ms per launch")

    # whole-path algorithmic HBM bytes per env-frame with the measured V and P
    # per image: V (R + 8) + P (12 + 24 + 4 + R) + W H 16 + scene / E, R = 40 B
    n_img_step = E * C
    V = st["visible"] / max(st["renders"], 1) / n_img_step
    P = st["pairs"] / max(st["renders"], 1) / n_img_step
    px_env = sum(c.width * c.height for c in cams)
    scene_bytes = R.scene_info(sid)[2]
    b_alg = C * (V * 48 + P * 80) + px_env * 16 + scene_bytes / E
    path = {"visible_per_image": V, "pairs_per_image": P, "pairs_per_step": P * n_img_step,
            "alg_bytes_per_env_frame": b_alg,
            "alg_hbm_frac": b_alg * value / (HBM_PEAK_GBS * 1e9)}
    props = torch.cuda.get_device_properties(dev)
    host = {"gpu": props.name, "arch": getattr(props, "gcnArchName", ""),
            "host_cores": len(os.sched_getaffinity(0)), "nproc": os.cpu_count()}

    out = {
        "metric": "env-frames/s at 640x480 x 2048 envs vs plain path; p50/p99 request latency",
        "value": value, "unit": "env-frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage if args.storage != "f32" else "f32", "data": "synthetic",
        "config": {"workload": synth.CONFIG_NAMES[args.config], "envs": E, "cams": C,
                   "resolution": [[c.width, c.height] for c in cams], "gaussians": scene.n,
                   "sh_degree": scene.sh_degree, "storage": args.storage, "tile": args.tile,
                   "tuning": tuning, "chunk_streams": 1 if args.no_overlap else 2},
        "plain_path": plain,
        "observation_path": observation,
        "lidar": lidar,
        "half_storage": storage,
        "serving": serving,
        "stages_ms_per_step": {k: v / args.steps for k, v in st.items() if k in R.STAGES},
        "one_stream": one_stream,
        "path": path,
        "host": host,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    R.close()


if __name__ == "__main__":
    main()
