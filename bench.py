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
import math
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
                 "SQ_INSTS_VALU", "GRBM_GUI_ACTIVE")
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
    # every kernel of the counted step: calibrated HBM bytes per dispatch
    kern = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        key = counter.split("_")[0].lower()
        for r in _pmc_rows(path, counter):
            name = r["Kernel_Name"]
            if "copyBuffer" in name or "elementwise" in name or "fillBuffer" in name:
                continue
            short = name.replace("void ", "").replace("gsr::", "").replace("(anonymous namespace)::", "").split("(")[0]
            k = kern.setdefault(short, {})
            k.setdefault(f"{key}_bytes", []).append(float(r["Counter_Value"]) * 1024.0 * out[f"{key}_factor"])
    out["kernels"] = {n: {"dispatches": len(v.get("fetch_bytes", [])),
                          "fetch_bytes_per_dispatch": sum(v.get("fetch_bytes", [0])) / max(1, len(v.get("fetch_bytes", []))),
                          "write_bytes_per_dispatch": sum(v.get("write_bytes", [0])) / max(1, len(v.get("write_bytes", [])))}
                      for n, v in sorted(kern.items())}
    # the counted command renders one step of the 2048-image default workload:
    # its rasteriser launches each cover this many images
    out["images_per_launch"] = 2048 / out["fetch_dispatches"]
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def util_summary(counter_csv, agent_csv, out_path, command):
    """Condense one counter run (UTIL_COUNTERS) into the rasteriser's VALU
    and LDS use per launch (and the same figures for every other kernel of
    the run under "kernels").  The SQ counters are summed over the SIMDs of
    the chip; GRBM_GUI_ACTIVE over its XCDs, so it divided by their number is
    the launch's duration in shader clocks.  VALU busy = quad-cycles of VALU
    issue x 4 / (SIMDs x clocks); LDS busy = cycles with indexed LDS work /
    (CUs x clocks); LDS bytes = 64-byte units loaded x 64."""
    with open(agent_csv) as f:
        agent = next(r for r in csv.DictReader(f) if r["Agent_Type"] == "GPU")
    n_xcc, cus = int(agent["Num_Xcc"]), int(agent["Cu_Count"])
    simds = cus * int(agent["Simd_Per_Cu"])
    clk_mhz = float(agent["Max_Engine_Clk_Fcompute"])
    per, names = {}, {}
    with open(counter_csv) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"]
            if "copyBuffer" in name or "elementwise" in name or "fillBuffer" in name or "reduce_kernel" in name:
                continue
            d = per.setdefault(r["Dispatch_Id"], {})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
            d["ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            names[r["Dispatch_Id"]] = (name.replace("void ", "").replace("gsr::", "")
                                       .replace("(anonymous namespace)::", "").split("(")[0])

    def util_row(d):
        clocks = d["GRBM_GUI_ACTIVE"] / n_xcc
        return {"ms": d["ns"] * 1e-6, "clock_ghz": clocks / d["ns"],
                "valu_busy": d["SQ_ACTIVE_INST_VALU"] * 4.0 / (simds * clocks),
                "valu_instr": d["SQ_INSTS_VALU"],
                "valu_issue": d["SQ_INSTS_VALU"] * 4.0 / (simds * clocks),
                "cu_busy": d["SQ_BUSY_CU_CYCLES"] * 4.0 / (simds * clocks),
                "lds_busy": d["SQ_LDS_IDX_ACTIVE"] / (cus * clocks),
                "lds_bytes": d["SQ_INSTS_LDS_LOAD_BANDWIDTH"] * 64.0}

    complete = {k: d for k, d in per.items() if all(c in d for c in UTIL_COUNTERS) and d["GRBM_GUI_ACTIVE"] > 0}
    rows = [util_row(d) for k, d in complete.items() if names[k].startswith("k_raster<")]
    if not rows:
        raise SystemExit(f"no rasteriser dispatch with all of {UTIL_COUNTERS} in {counter_csv}")
    mean = {k: sum(r[k] for r in rows) / len(rows) for k in rows[0]}
    # every other kernel of the run, launches of 50 us or more (shorter ones
    # are mostly launch overhead and clock ramp)
    by_kernel = {}
    for k, d in complete.items():
        if d["ns"] >= 50_000:
            by_kernel.setdefault(names[k], []).append(util_row(d))
    kernels = {}
    for name, rs in sorted(by_kernel.items()):
        m = {k: sum(r[k] for r in rs) / len(rs) for k in rs[0]}
        kernels[name] = {"dispatches": len(rs), "avg_ms": m["ms"], "valu_issue_frac": m["valu_issue"],
                         "valu_busy": m["valu_busy"], "lds_busy": m["lds_busy"]}
    lds_gbs = mean["lds_bytes"] / (mean["ms"] * 1e-3) / 1e9
    lds_peak = cus * LDS_BYTES_PER_CLK * clk_mhz * 1e6 / 1e9
    out = {"command": command, "source_sha256": raster_source_hash(), "sources": list(RASTER_SOURCES),
           "counters": list(UTIL_COUNTERS), "dispatches": len(rows), "cus": cus, "simds": simds, "xcds": n_xcc,
           "avg_ms": mean["ms"], "clock_ghz": mean["clock_ghz"], "valu_busy": mean["valu_busy"],
           "valu_instr_per_launch": mean["valu_instr"], "valu_issue_frac": mean["valu_issue"],
           "valu_issue_basis": "wave64 VALU instructions x 4 cycles (16-lane SIMDs) / (SIMDs x shader clocks)",
           "cu_busy": mean["cu_busy"], "lds_busy": mean["lds_busy"], "lds_read_bytes_per_launch": mean["lds_bytes"],
           "lds_read_gbs": lds_gbs, "lds_peak_gbs": lds_peak, "lds_read_frac": lds_gbs / lds_peak,
           "lds_peak_basis": f"{cus} CUs x {LDS_BYTES_PER_CLK} B/clock x {clk_mhz:.0f} MHz", "kernels": kernels}
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
    return {k: s[k] for k in ("valu_busy", "valu_issue_frac", "lds_busy", "lds_read_gbs", "lds_peak_gbs",
                              "lds_read_frac", "clock_ghz") if k in s}


def measured_traffic(tuning, images_per_launch):
    """HBM bytes per rasteriser launch from the committed counter summary, or
    None when it was taken on other rasteriser sources, launch parameters or
    launch sizes."""
    path = os.path.join(ROOT, PMC_SUMMARY)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        s = json.load(f)
    if s.get("source_sha256") != raster_source_hash():
        return None
    if s.get("images_per_launch") is None or abs(s["images_per_launch"] - images_per_launch) > 0.5:
        return None
    if tuning is not None and s.get("tuning") is not None:
        # only the launch parameters of the rasteriser itself matter here
        keys = ("tile_size", "lds_batch", "persistent")
        if any(s["tuning"].get(k) != tuning.get(k) for k in keys):
            return None
    return s["traffic_bytes_per_launch"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _free():
    """Drop unreferenced tensors and hand PyTorch's cached blocks back, so the
    library's own allocations in the next leg find the memory."""
    import gc
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def sampled_envs(E, k):
    """k distinct envs spread over [0, E) (seeded, reproducible)."""
    out = []
    for j in range(E):
        e = (j * 997) % E
        if e not in out:
            out.append(e)
        if len(out) == min(k, E):
            break
    return out


def oracle_error(scene, batch, images, tile, pairs):
    """Per-image error of GPU images against the float64 oracle on the scene's
    original float32 attributes.  `images` maps (slot, env) to the GPU's
    float32 RGB [H, W, 3] (numpy); `pairs` lists the (slot, env) keys.  Pixels
    with a threshold decision near its boundary (flagged by the oracle) are
    reported apart, since either branch is admissible there."""
    import numpy as np
    from oracle import render_ref
    rows = []
    for c, e in pairs:
        ref = render_ref(scene, batch, c, e, tile, variants=False)
        d = np.abs(np.asarray(images[(c, e)], np.float64) - ref.rgb)
        calm = ref.nflag == 0
        mse = float(np.mean(d * d))
        rows.append({"slot": c, "env": e, "max_abs": float(d.max()),
                     "max_abs_unflagged": float(d[calm].max()) if calm.any() else 0.0,
                     "mean_abs": float(d.mean()), "flagged_pixels": int((~calm).sum()),
                     "psnr_db": float(10.0 * np.log10(1.0 / mse)) if mse > 0 else float("inf")})
    ps = [r["psnr_db"] for r in rows]
    return {"reference": "float64 oracle on the original float32 attributes", "images": len(rows),
            "max_abs_max": max(r["max_abs"] for r in rows),
            "max_abs_unflagged_max": max(r["max_abs_unflagged"] for r in rows),
            "mean_abs_mean": sum(r["mean_abs"] for r in rows) / len(rows),
            "psnr_db_min": min(ps), "psnr_db_median": float(np.median(ps)), "per_image": rows}


def gpu_images(cams, E, rgb, pairs):
    """(slot, env) -> float32 RGB [H, W, 3] as numpy, from a flat render output."""
    out, base = {}, 0
    for c, cam in enumerate(cams):
        n = E * cam.width * cam.height * 3
        view = rgb[base:base + n].view(E, cam.height, cam.width, 3)
        for (cc, e) in pairs:
            if cc == c:
                out[(c, e)] = view[e].cpu().numpy()
        base += n
    return out


def timed_steps(R, sid, cams, vm, poses, rgb, depth, bg, steps, first=0, obs=None):
    """Seconds for `steps` renders (poses[first + s]) bracketed by device syncs."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        R.render_into(sid, cams, vm, poses[(first + s) % len(poses)], rgb, depth, None, bg, obs=obs)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def plain_rate(R, sid, batch, poses_t, n_envs, bg):
    """Env-frames/s of the plain per-env path (one image per launch chain,
    host sync per image) over the first n_envs envs, after one warm render."""
    import torch
    from paper_2604_25459_amd import gsr
    pe = min(n_envs, batch.n_envs)
    sub = batch.subset(range(pe))
    pcams, pvm, _ = gsr.batch_tensors(sub)
    prgb, pdep, _ = R.alloc_outputs(pcams, pe)
    pp = poses_t[:pe].contiguous()
    R.render_into(sid, pcams, pvm, pp, prgb, pdep, None, bg, plain=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R.render_into(sid, pcams, pvm, pp, prgb, pdep, None, bg, plain=True)
    torch.cuda.synchronize()
    return {"value": pe / (time.perf_counter() - t0), "unit": "env-frames/s", "envs_timed": pe}


def config_leg(cfg, storage, args, steps, n_plain, n_err):
    """Batched throughput of workload `cfg` (autotuned, poses resampled each
    step), the plain per-env path's rate, and per-image error against the
    oracle on sampled envs of the last timed step."""
    import numpy as np
    import torch
    from paper_2604_25459_amd import gsr, synth
    dev = torch.device("cuda", 0)
    log(f"[cfg{cfg}] generating workload")
    scene, batch = synth.make_config(cfg)
    E, C = batch.n_envs, batch.n_cams
    bg = tuple(float(x) for x in batch.bg)
    R = gsr.Renderer(0, tile_size=args.tile, profile=True)
    try:
        sid = R.add_synth_scene(scene, storage)
        cams, vm, _ = gsr.batch_tensors(batch)
        warm = max(2, args.warmup)
        pose_np = [synth.make_poses(cfg, s, E, scene.n_bodies) for s in range(warm + steps)]
        poses = [torch.from_numpy(p).to(dev) for p in pose_np]
        rgb, depth, _ = R.alloc_outputs(cams, E)
        tuning = R.autotune(sid, cams, vm, poses[0], rgb, depth) if not args.no_autotune else None
        for s in range(warm):
            R.render_into(sid, cams, vm, poses[s], rgb, depth, None, bg)
        sec = timed_steps(R, sid, cams, vm, poses, rgb, depth, bg, steps, first=warm)
        value = E * steps / sec
        out = {"workload": synth.CONFIG_NAMES[cfg], "storage": storage, "envs": E, "cams": C,
               "resolution": [[c.width, c.height] for c in cams], "gaussians": scene.n, "steps": steps,
               "value": value, "unit": "env-frames/s", "ms_per_step": 1000.0 * sec / steps, "tuning": tuning}
        log(f"[cfg{cfg}] {value:.1f} env-frames/s ({1000.0 * sec / steps:.3f} ms/step), tuning {tuning}")
        last = warm + steps - 1
        if n_err:
            pairs = [(c, e) for c in range(C) for e in sampled_envs(E, n_err)]
            imgs = gpu_images(cams, E, rgb, pairs)
            b_last = synth.Batch(cams=batch.cams, viewmats=batch.viewmats, poses=pose_np[last], bg=batch.bg)
            out["error_vs_oracle"] = oracle_error(scene, b_last, imgs, args.tile, pairs)
            log(f"[cfg{cfg}] error vs oracle: max-abs {out['error_vs_oracle']['max_abs_max']:.3g} "
                f"(unflagged {out['error_vs_oracle']['max_abs_unflagged_max']:.3g}), "
                f"PSNR min {out['error_vs_oracle']['psnr_db_min']:.1f} dB")
        if n_plain:
            out["plain_path"] = plain_rate(R, sid, batch, poses[last], n_plain, bg)
            log(f"[cfg{cfg}] plain path {out['plain_path']['value']:.1f} env-frames/s")
        del rgb, depth, poses
        return out
    finally:
        R.close()


def run_serving(R, args):
    """Replay the seeded Poisson trace (200 req/s, 1-256 envs, 128x128 /
    320x240 / 640x480, a pool of FP16 scenes of 50k-1M Gaussians plus 4-16
    bodies) in real time through the continuous-batching server; then the
    first `plain_serve_seconds` of the same trace through the plain per-env
    path, one request at a time in arrival order (the baseline without
    batching).  Latency = completion on the device - scheduled arrival."""
    import threading
    import numpy as np
    import torch
    from paper_2604_25459_amd import gsr, synth

    dev = torch.device("cuda", 0)
    K = max(1, min(args.serve_scenes, 32))
    trace = [r for r in synth.serving_trace(pool=32) if r.arrival_s < args.serve_seconds]
    log(f"[serve] {len(trace)} requests over {args.serve_seconds:.0f} s, pool of {K} resident scenes (FP16)")
    scenes, sids = [], []
    for k in range(K):
        sc = synth.serving_pool_scene(k)
        scenes.append(sc)
        sids.append(R.add_synth_scene(sc, "f16"))
    log(f"[serve] scene pool resident: {sum(s.n for s in scenes)} Gaussians")
    prepared = [(req, req.scene % K, synth.serving_batch(req, scenes[req.scene % K], idx))
                for idx, req in enumerate(trace)]
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
    infos = []
    t0_us = time.monotonic_ns() // 1000

    refused = []

    def producer():
        try:
            for k, (req, si, b) in enumerate(prepared):
                now = time.monotonic_ns() // 1000 - t0_us
                if req.arrival_s * 1e6 > now:
                    time.sleep((req.arrival_s * 1e6 - now) * 1e-6)
                cams, vm, poses = gsr.batch_tensors(b)
                rgb, depth, _ = R.alloc_outputs(cams, b.n_envs)
                torch.cuda.current_stream(dev).synchronize()
                try:
                    t = S.submit(sids[si], cams, vm, poses, rgb, depth)
                except gsr.GsrError as ex:
                    if ex.code != gsr.GSR_E_REJECTED:
                        raise
                    refused.append(k)
                    continue
                with lock:
                    tickets.append((t, k, b.n_envs * b.n_cams))
        finally:
            with lock:
                tickets.append((None, -1, 0))     # the waiter stops here, also after an error

    th = threading.Thread(target=producer)
    th.start()
    k = 0
    n_img = 0
    while True:
        with lock:
            item = tickets[k] if k < len(tickets) else False
        if item is False:
            time.sleep(0.0005)
            continue
        t, idx, ni = item
        if t is None:
            break
        info = S.wait(t)
        infos.append((idx, info))
        n_img += ni
        k += 1
    wall = (time.monotonic_ns() // 1000 - t0_us) * 1e-6
    th.join()
    st = S.stats()
    S.close()
    arr = np.array([prepared[i][0].arrival_s * 1e6 + t0_us for i, _ in infos])
    done = np.array([inf["t_complete_us"] for _, inf in infos], np.float64)
    sub = np.array([inf["t_submit_us"] for _, inf in infos], np.float64)
    lat = (done - arr) / 1000.0
    lat_sub = (done - sub) / 1000.0
    breq = np.array([inf["batch_requests"] for _, inf in infos])
    hist = {str(v): int((breq == v).sum()) for v in sorted(set(breq.tolist()))}
    out = {"requests": st["completed"] - base["completed"], "arrival_rate_hz": 200.0,
           "trace_seconds": args.serve_seconds, "scenes": K, "streams": args.serve_streams,
           "latency_p50_ms": float(np.percentile(lat, 50)), "latency_p99_ms": float(np.percentile(lat, 99)),
           "latency_max_ms": float(lat.max()),
           "latency_from_submit_p50_ms": float(np.percentile(lat_sub, 50)),
           "latency_from_submit_p99_ms": float(np.percentile(lat_sub, 99)),
           "env_frames_per_s": n_img / wall, "wall_s": wall,
           "batches": st["batches"] - base["batches"], "mean_batch_requests": st["mean_batch_requests"],
           "requests_by_batch_size": hist, "requests_rejected": len(refused),
           "requests_merged": int((breq > 1).sum())}
    log(f"[serve] p50 {out['latency_p50_ms']:.2f} ms, p99 {out['latency_p99_ms']:.2f} ms, "
        f"{out['env_frames_per_s']:.0f} env-frames/s, {out['requests_merged']} requests merged")

    # the plain per-env path on the first seconds of the same trace
    if args.plain_serve_seconds > 0:
        pre = [(i, p) for i, p in enumerate(prepared) if p[0].arrival_s < args.plain_serve_seconds]
        lat_p = []
        n_pimg = 0
        t0 = time.monotonic_ns() // 1000
        for i, (req, si, b) in pre:
            now = time.monotonic_ns() // 1000 - t0
            if req.arrival_s * 1e6 > now:
                time.sleep((req.arrival_s * 1e6 - now) * 1e-6)
            cams, vm, poses = gsr.batch_tensors(b)
            rgb, depth, _ = R.alloc_outputs(cams, b.n_envs)
            R.render_into(sids[si], cams, vm, poses, rgb, depth, plain=True)
            torch.cuda.synchronize()
            lat_p.append((time.monotonic_ns() // 1000 - t0) - req.arrival_s * 1e6)
            n_pimg += b.n_envs * b.n_cams
        pwall = (time.monotonic_ns() // 1000 - t0) * 1e-6
        lat_p = np.asarray(lat_p) / 1000.0
        served_same = np.array([lat[j] for j, (i, _) in enumerate(infos)
                                if prepared[i][0].arrival_s < args.plain_serve_seconds])
        out["plain_path"] = {
            "trace_seconds": args.plain_serve_seconds, "requests": len(pre),
            "latency_p50_ms": float(np.percentile(lat_p, 50)), "latency_p99_ms": float(np.percentile(lat_p, 99)),
            "latency_max_ms": float(lat_p.max()), "env_frames_per_s": n_pimg / pwall, "wall_s": pwall,
            "served_same_requests_p50_ms": float(np.percentile(served_same, 50)),
            "served_same_requests_p99_ms": float(np.percentile(served_same, 99)),
            "policy": "one request at a time in arrival order, gsr_render_plain, host sync per image"}
        log(f"[serve] plain path on the first {args.plain_serve_seconds:.0f} s: "
            f"p50 {out['plain_path']['latency_p50_ms']:.1f} ms, p99 {out['plain_path']['latency_p99_ms']:.1f} ms "
            f"(served: p99 {out['plain_path']['served_same_requests_p99_ms']:.1f} ms)")
    for sid in sids:
        R.remove_scene(sid)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--envs", type=int, default=0, help="truncate the workload's env count (0 = full)")
    ap.add_argument("--plain-envs", type=int, default=64, help="envs timed on the plain per-env path (0 = skip)")
    ap.add_argument("--cpu-images", type=int, default=16, help="envs rendered by the CPU oracle (0 = skip)")
    ap.add_argument("--cpu-images-1t", type=int, default=2, help="envs rendered by the oracle on one thread")
    ap.add_argument("--err-envs", type=int, default=4,
                    help="sampled envs per workload whose images are checked against the oracle (0 = skip)")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="seconds of the Poisson serving trace replayed in real time (0 = skip)")
    ap.add_argument("--serve-scenes", type=int, default=32, help="resident scenes in the serving pool")
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--plain-serve-seconds", type=float, default=5.0,
                    help="seconds of the same trace replayed through the plain per-env path (0 = skip)")
    ap.add_argument("--no-configs", dest="configs", action="store_false",
                    help="skip the legs of workloads 0, 1 and 3")
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

    import traceback

    import numpy as np
    import torch

    from paper_2604_25459_amd import gsr, synth

    out = {"metric": "env-frames/s at 640x480 x 2048 envs vs plain path; p50/p99 request latency",
           "value": None, "unit": "env-frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.storage, "data": "synthetic"}

    def leg(name, fn):
        """Run one optional leg; a failure becomes {"error": ...} and the rest goes on."""
        t0 = time.perf_counter()
        try:
            out[name] = fn()
        except Exception as ex:      # noqa: BLE001 -- recorded in the JSON line
            traceback.print_exc()
            out[name] = {"error": f"{type(ex).__name__}: {ex}"}
        log(f"[bench] leg {name} took {time.perf_counter() - t0:.1f} s")
        _free()

    if args.calibration_copy:
        x = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)                       # device-to-device copy kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del x, y
        log("[bench] calibration: 1 GiB device-to-device copy done")

    # ------------------------------------------------------------ headline
    log(f"[bench] config {args.config}: generating workload")
    scene, batch = synth.make_config(args.config, n_envs=args.envs or None)
    E, C = batch.n_envs, batch.n_cams
    bg = tuple(float(x) for x in batch.bg)
    R = gsr.Renderer(0, tile_size=args.tile, profile=True, graphs=not args.no_graphs, overlap=not args.no_overlap)
    sid = R.add_synth_scene(scene, args.storage)
    cams, vm, _ = gsr.batch_tensors(batch)
    dev = torch.device("cuda", 0)
    n_pose_steps = args.warmup + args.steps
    pose_np = [synth.make_poses(args.config, s, E, scene.n_bodies) for s in range(n_pose_steps)]
    poses = [torch.from_numpy(p).to(dev) for p in pose_np]
    rgb, depth, _ = R.alloc_outputs(cams, E)

    tuning = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tuning = R.autotune(sid, cams, vm, poses[0], rgb, depth)
        log(f"[bench] autotuned in {time.perf_counter() - t0:.1f} s: {tuning}")
    log(f"[bench] warmup {args.warmup} steps of {E} envs x {C} cams")
    for s in range(args.warmup):
        R.render_into(sid, cams, vm, poses[s], rgb, depth, None, bg)
    torch.cuda.synchronize()
    R.stage_times(reset=True)

    log(f"[bench] timing {args.steps} steps")
    sec = timed_steps(R, sid, cams, vm, poses, rgb, depth, bg, args.steps, first=args.warmup)
    st = R.stage_times(reset=True)
    value = E * args.steps / sec
    ms_per_step = 1000.0 * sec / args.steps
    log(f"[bench] {value:.1f} env-frames/s, {ms_per_step:.2f} ms/step, stages {st}")
    out.update({"value": value, "ms_per_step": ms_per_step,
                "config": {"workload": synth.CONFIG_NAMES[args.config], "envs": E, "cams": C,
                           "resolution": [[c.width, c.height] for c in cams], "gaussians": scene.n,
                           "sh_degree": scene.sh_degree, "storage": args.storage, "tile": args.tile,
                           "tuning": tuning, "chunk_streams": 1 if args.no_overlap else 2},
                "stages_ms_per_step": {k: v / args.steps for k, v in st.items() if k in R.STAGES}})
    last = args.warmup + args.steps - 1

    # whole-path algorithmic HBM bytes per env-frame with the measured V and P
    # per image: V (R + 8) + P (12 + 24 + 4 + R) + W H 16 + scene / E, R = 40 B
    n_img_step = E * C
    V = st["visible"] / max(st["renders"], 1) / n_img_step
    P = st["pairs"] / max(st["renders"], 1) / n_img_step
    px_env = sum(c.width * c.height for c in cams)
    scene_bytes = R.scene_info(sid)[2]
    b_alg = C * (V * 48 + P * 80) + px_env * 16 + scene_bytes / E
    out["path"] = {"visible_per_image": V, "pairs_per_image": P, "pairs_per_step": P * n_img_step,
                   "alg_bytes_per_env_frame": b_alg, "alg_hbm_frac": b_alg * value / (HBM_PEAK_GBS * 1e9)}
    props = torch.cuda.get_device_properties(dev)
    out["host"] = {"gpu": props.name, "arch": getattr(props, "gcnArchName", ""),
                   "host_cores": len(os.sched_getaffinity(0)), "nproc": os.cpu_count()}

    # roofline of the dominant kernel (the rasteriser, bound by vector ALU
    # work): exact per-pixel work of every timed step, from counting renders
    # of the same poses with the same launch parameters (untimed)
    def roofline():
        # the launch time of the rasteriser running alone: from the one-stream
        # leg (the same steps, every chunk on one stream) when it ran; in the
        # two-stream steps a launch shares the GPU with the next chunk's binning
        # on the other stream, so its event interval is not its own cost
        raster_ms_two = st["raster"] / max(st["raster_launches"], 1)
        one = out.get("one_stream") or {}
        raster_ms = one.get("raster_ms_per_launch") or raster_ms_two
        if args.no_count or raster_ms <= 0:
            return None
        npx = rgb.numel() // 3
        work = torch.empty(npx * 2, dtype=torch.int32, device=dev)
        scratch_rgb = torch.empty_like(rgb)
        scratch_depth = torch.empty_like(depth)
        visits = accepts = 0
        for s in range(args.steps):
            R.render_into(sid, cams, vm, poses[args.warmup + s], scratch_rgb, scratch_depth, None, bg, work=work)
            w = work.view(npx, 2)
            visits += int(w[:, 0].sum(dtype=torch.int64))
            accepts += int(w[:, 1].sum(dtype=torch.int64))
        torch.cuda.synchronize()
        R.stage_times(reset=True)
        del work, scratch_rgb, scratch_depth
        flops_step = (visits * FLOPS_EVAL + accepts * FLOPS_ACCEPT) / args.steps
        launches_per_step = st["raster_launches"] / args.steps
        flops_launch = flops_step / launches_per_step
        achieved = flops_launch / (raster_ms * 1e-3) / 1e12
        traffic = measured_traffic(tuning, E * C / launches_per_step)
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": "k_raster", "avg_ms": raster_ms,
                "avg_ms_source": "one-stream leg" if one.get("raster_ms_per_launch") else "timed steps",
                "avg_ms_two_stream_steps": raster_ms_two, "launches_per_step": launches_per_step,
                "flop_per_launch": flops_launch,
                "visits_per_pixel": visits / (npx * args.steps), "accepts_per_pixel": accepts / (npx * args.steps),
                "units": "list entries up to each pixel's termination x 11 flop + blended Gaussians x 11 flop"}
        if traffic is not None:
            roof["hbm_gbs"] = traffic / (raster_ms * 1e-3) / 1e9
            roof["hbm_frac"] = roof["hbm_gbs"] / HBM_PEAK_GBS
        roof["valu_lds"] = measured_util()
        log(f"[bench] raster {roof['visits_per_pixel']:.1f} visits, {roof['accepts_per_pixel']:.1f} blends per "
            f"pixel; {achieved:.2f} TFLOP/s algorithmic over {raster_ms:.2f} ms per launch")
        return roof


    # per-image error of the timed path's last step against the oracle
    def headline_error():
        pairs = [(c, e) for c in range(C) for e in sampled_envs(E, args.err_envs)]
        imgs = gpu_images(cams, E, rgb, pairs)
        b_last = synth.Batch(cams=batch.cams, viewmats=batch.viewmats, poses=pose_np[last], bg=batch.bg)
        r = oracle_error(scene, b_last, imgs, args.tile, pairs)
        log(f"[bench] error vs oracle: max-abs {r['max_abs_max']:.3g} (unflagged {r['max_abs_unflagged_max']:.3g})")
        return r

    if args.err_envs:
        leg("error_vs_oracle", headline_error)

    # the same steps with every chunk on the render stream: the gain of the
    # two-stream overlap, and a stage breakdown in which no stages share the GPU
    def one_stream_leg():
        R1 = gsr.Renderer(0, tile_size=args.tile, profile=True, graphs=not args.no_graphs, overlap=False)
        try:
            sid1 = R1.add_synth_scene(scene, args.storage)
            if tuning:
                R1.set_tuning(sid1, cams, vm, poses[0], **{k: v for k, v in tuning.items() if k != "ms"})
            R1.render_into(sid1, cams, vm, poses[0], rgb, depth, None, bg)
            torch.cuda.synchronize()
            R1.stage_times(reset=True)
            osec = timed_steps(R1, sid1, cams, vm, poses, rgb, depth, bg, args.steps, first=args.warmup)
            ost = R1.stage_times(reset=True)
            r = {"value": E * args.steps / osec, "unit": "env-frames/s", "ms_per_step": 1000.0 * osec / args.steps,
                 "stages_ms_per_step": {k: v / args.steps for k, v in ost.items() if k in R.STAGES},
                 "raster_ms_per_launch": ost["raster"] / max(ost["raster_launches"], 1)}
            log(f"[bench] one stream: {r['value']:.1f} env-frames/s, stages {r['stages_ms_per_step']}")
            return r
        finally:
            R1.close()

    if not args.no_overlap and args.one_stream_leg:
        leg("one_stream", one_stream_leg)

    # after the one-stream leg: the rasteriser's own launch time comes from it
    leg("roofline", roofline)

    # policy-ready observations: same workload, u8 pixels with per-image exposure /
    # contrast / brightness randomisation fused into the rasteriser, no float colour
    def observation_leg():
        g = torch.Generator().manual_seed(7)
        n_img = E * C
        gain = (2.0 ** (torch.rand(n_img, generator=g) - 0.5)).to(dev)
        contrast = (0.8 + 0.4 * torch.rand(n_img, generator=g)).to(dev)
        bright = (0.1 * torch.rand(n_img, generator=g) - 0.05).to(dev)
        obs_out = torch.empty(rgb.numel(), dtype=torch.uint8, device=dev)
        obs = gsr.Observation("u8", obs_out, gain, contrast, bright)
        R.render_into(sid, cams, vm, poses[args.warmup], None, depth, None, bg, obs=obs)
        osec = timed_steps(R, sid, cams, vm, poses, None, depth, bg, args.obs_steps, first=args.warmup, obs=obs)
        R.stage_times(reset=True)
        r = {"value": E * args.obs_steps / osec, "unit": "env-frames/s", "format": "u8", "steps": args.obs_steps,
             "randomisation": "gain 2^U[-0.5,0.5], contrast U[0.8,1.2], brightness U[-0.05,0.05] per image"}
        log(f"[bench] observation path (u8 + randomisation) {r['value']:.1f} env-frames/s")
        return r

    if args.obs_steps:
        leg("observation_path", observation_leg)

    # batch LiDAR on the same scene and poses: one rotating 32 x 1024 sensor per env
    def lidar_leg():
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
        r = {"value": E * args.lidar_steps / lsec, "unit": "env-scans/s",
             "rays_per_s": n_rays * args.lidar_steps / lsec, "steps": args.lidar_steps,
             "sensor": "rotating, 32 beams [-25, 15] deg x 1024 columns", "envs": E,
             "ms_per_step": 1000.0 * lsec / args.lidar_steps,
             "stages_ms_per_step": {k: v / args.lidar_steps for k, v in lst.items() if k in R.STAGES},
             "hit_fraction": float((l_hit > 0.5).float().mean())}
        log(f"[bench] LiDAR {r['value']:.1f} env-scans/s ({r['rays_per_s'] / 1e9:.2f} G rays/s)")
        # heightmap scanner: a 64 x 64 grid of downward rays at 5 cm under each sensor
        hm = synth.height_grid(64, 64, 0.05)
        n_hm = E * hm.width * hm.height
        h_range = torch.empty(n_hm, dtype=torch.float32, device=dev)
        h_hit = torch.empty(n_hm, dtype=torch.float32, device=dev)
        R.render_lidar_into(sid, [hm], lvm, poses[args.warmup], h_range, h_hit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.lidar_steps):
            R.render_lidar_into(sid, [hm], lvm, poses[args.warmup + s % args.steps], h_range, h_hit)
        torch.cuda.synchronize()
        hsec = time.perf_counter() - t0
        R.stage_times(reset=True)
        r["heightmap"] = {"value": E * args.lidar_steps / hsec, "unit": "env-scans/s",
                          "sensor": "heightmap grid, 64 x 64 downward rays at 0.05 m", "envs": E,
                          "ms_per_step": 1000.0 * hsec / args.lidar_steps,
                          "hit_fraction": float((h_hit > 0.5).float().mean())}
        log(f"[bench] heightmap {r['heightmap']['value']:.1f} env-scans/s")
        # non-repetitive (rosette) scanner, 96 x 256 listed rays per scan over a
        # 70 deg field; every scan takes the next phase of the rosette (new rays)
        n_ros = 96 * 256
        ds = math.pi * (3.0 - math.sqrt(5.0))
        ros = [synth.rosette_lidar(96, 256, 35.0, s0=k * n_ros * ds) for k in range(args.lidar_steps + 1)]
        o_range = torch.empty(E * n_ros, dtype=torch.float32, device=dev)
        o_hit = torch.empty(E * n_ros, dtype=torch.float32, device=dev)
        R.render_lidar_into(sid, [ros[0]], lvm, poses[args.warmup], o_range, o_hit)
        torch.cuda.synchronize()
        R.stage_times(reset=True)
        t0 = time.perf_counter()
        for s in range(args.lidar_steps):
            R.render_lidar_into(sid, [ros[s + 1]], lvm, poses[args.warmup + s % args.steps], o_range, o_hit)
        torch.cuda.synchronize()
        osec = time.perf_counter() - t0
        ost = R.stage_times(reset=True)
        r["rosette"] = {"value": E * args.lidar_steps / osec, "unit": "env-scans/s",
                        "rays_per_s": E * n_ros * args.lidar_steps / osec,
                        "sensor": "non-repetitive rosette, 96 x 256 listed rays in a 70 deg field, new rays every scan",
                        "envs": E, "ms_per_step": 1000.0 * osec / args.lidar_steps,
                        "stages_ms_per_step": {k: v / args.lidar_steps for k, v in ost.items() if k in R.STAGES},
                        "hit_fraction": float((o_hit > 0.5).float().mean())}
        log(f"[bench] rosette LiDAR {r['rosette']['value']:.1f} env-scans/s "
            f"({r['rosette']['rays_per_s'] / 1e9:.2f} G rays/s)")
        return r

    if args.lidar_steps:
        leg("lidar", lidar_leg)

    # half-precision storage on the same workload, with the float32 leg's
    # launch parameters: throughput, per-image error against the oracle on
    # the original float32 attributes (sampled envs), and against the
    # float32-storage render of the same step (every image, float32 math)
    def storage_leg():
        res = {}
        ref_rgb = rgb.clone()                    # last timed step, float32 storage
        for st_name in ("f16", "bf16"):
            hsid = R.add_synth_scene(scene, st_name)
            try:
                if tuning:
                    R.set_tuning(hsid, cams, vm, poses[0], **{k: v for k, v in tuning.items() if k != "ms"})
                R.render_into(hsid, cams, vm, poses[last], rgb, depth, None, bg)
                hsec = timed_steps(R, hsid, cams, vm, poses, rgb, depth, bg, args.steps, first=args.warmup)
                R.stage_times(reset=True)
                mx, ma, mse = [], [], []
                base = 0
                for cam in cams:                 # per camera slot, a few images at a time
                    hw3 = cam.width * cam.height * 3
                    for e0 in range(0, E, 64):
                        e1 = min(E, e0 + 64)
                        d = (rgb[base + e0 * hw3:base + e1 * hw3] - ref_rgb[base + e0 * hw3:base + e1 * hw3])
                        d = d.view(e1 - e0, hw3).abs_()
                        mx.append(d.amax(dim=1))
                        ma.append(d.mean(dim=1))
                        mse.append((d * d).mean(dim=1))
                        del d
                    base += E * hw3
                mx = torch.cat(mx).cpu().numpy()
                ma = torch.cat(ma).cpu().numpy()
                mse = torch.cat(mse).cpu().numpy().astype(np.float64)
                psnr = 10.0 * np.log10(1.0 / np.maximum(mse, 1e-30))
                r = {"value": E * args.steps / hsec, "unit": "env-frames/s", "scene_bytes": R.scene_info(hsid)[2],
                     "error_vs_f32_storage_per_image": {
                         "images": int(mx.size), "max_abs_max": float(mx.max()), "mean_abs_mean": float(ma.mean()),
                         "psnr_db_min": float(psnr.min()), "psnr_db_median": float(np.median(psnr))}}
                if args.err_envs:
                    pairs = [(c, e) for c in range(C) for e in sampled_envs(E, args.err_envs)]
                    imgs = gpu_images(cams, E, rgb, pairs)
                    b_last = synth.Batch(cams=batch.cams, viewmats=batch.viewmats, poses=pose_np[last], bg=batch.bg)
                    r["error_vs_oracle"] = oracle_error(scene, b_last, imgs, args.tile, pairs)
                res[st_name] = r
                log(f"[bench] {st_name} storage: {r['value']:.1f} env-frames/s, "
                    f"vs oracle max-abs {r.get('error_vs_oracle', {}).get('max_abs_max')}, "
                    f"PSNR min {r.get('error_vs_oracle', {}).get('psnr_db_min')}")
            finally:
                R.remove_scene(hsid)
        del ref_rgb
        return res

    if args.storage_check and args.storage == "f32":
        leg("half_storage", storage_leg)

    # plain per-env path on a subset (same GPU, same kernels, one image per launch chain)
    if args.plain_envs:
        leg("plain_path", lambda: plain_rate(R, sid, batch, poses[last], args.plain_envs, bg))

    # the other workloads: 0 (plain 128x96), 1 (64 x 320x240), 3 (512 x two uneven cameras, BF16)
    if args.configs:
        cfgs = {}

        def cfg_legs():
            for cfg, storage, steps, n_plain in ((0, "f32", 200, 1), (1, "f32", 50, 64), (3, "bf16", args.steps, 64)):
                try:
                    cfgs[str(cfg)] = config_leg(cfg, storage, args, steps, n_plain, max(1, args.err_envs // 2))
                except Exception as ex:      # noqa: BLE001
                    traceback.print_exc()
                    cfgs[str(cfg)] = {"error": f"{type(ex).__name__}: {ex}"}
                _free()
            return cfgs

        leg("configs", cfg_legs)

    if args.serve_seconds > 0:
        leg("serving", lambda: run_serving(R, args))

    # oracle on the host cores, bounded sample of the same workload
    def cpu_leg():
        from oracle import oracle_threads, render_ref, set_oracle_threads
        b0 = synth.Batch(cams=batch.cams, viewmats=batch.viewmats, poses=pose_np[args.warmup], bg=batch.bg)
        envs = sampled_envs(E, args.cpu_images)
        cores = oracle_threads()
        t0 = time.perf_counter()
        for e in envs:
            for c in range(C):
                render_ref(scene, b0, c, e, args.tile, variants=False)
        csec = time.perf_counter() - t0
        r = {"value": len(envs) / csec, "unit": "env-frames/s", "cores": cores, "kind": "oracle",
             "sample": f"{len(envs)} envs of step {args.warmup} (float32 binning spec on one thread + "
                       f"float64 compositing on {cores} OpenMP threads)"}
        if args.cpu_images_1t:
            set_oracle_threads(1)
            try:
                envs1 = envs[:args.cpu_images_1t]
                t0 = time.perf_counter()
                for e in envs1:
                    for c in range(C):
                        render_ref(scene, b0, c, e, args.tile, variants=False)
                r["single_thread"] = {"value": len(envs1) / (time.perf_counter() - t0), "unit": "env-frames/s",
                                      "cores": 1, "envs": len(envs1)}
            finally:
                set_oracle_threads(cores)
        log(f"[bench] oracle {r['value']:.3f} env-frames/s on {cores} cores")
        return r

    if args.cpu_images:
        leg("cpu_baseline", cpu_leg)

    print(json.dumps(out), flush=True)
    R.close()


if __name__ == "__main__":
    main()
