#!/usr/bin/env python3
"""Throughput of the IRT-PS hot path on one MI355X.

One step is one whole IRT-PS reconstruction (Sec. IV of the paper): plain
photometric stereo and integration of the input images, then T passes of
trace -> subtract -> PS -> integrate, all in the library's HIP kernels behind
the C ABI.  Inputs are resident in HBM before the timed region.

Default workload: 2048x2048 RGB fBm terrain (Hurst 0.7, peak-to-peak 256 px),
per-channel albedo U[0.3, 0.9], 16 Fibonacci lights, 256x512 log-normal
environment; solve with 256 spp, 3 bounces, 5 iterations (FP32).  The input
images are rendered on the GPU (64 spp, 3 bounces) before timing.

Prints one JSON line.  `value` is traced gather segments (rays) per second of
the whole job; `radiance_samples_per_s` counts K C per segment (one path serves
every light and channel), and the direct light's shadow rays are counted apart
(`shadow_rays_per_step`, `shadow_rays_per_s` over the whole step).  The `roofline` object is for the tracer kernel, timed with HIP
events around its launches inside the timed steps: it is bound by VALU issue,
so it is given in lane-operations (counted wave64 VALU instructions times
their active lanes, from the committed counter profile of the same machine
code) against the full-lane peak measured with the issue-rate probe;
`hbm_yardstick` gives the tracer's algorithmic bytes against 8 TB/s, with the
fabric bytes (copy-calibrated FETCH_SIZE + WRITE_SIZE, MALL hits included) of
the counter profile.  `cpu_baseline` is the CPU oracle on bounded samples of
the same workload (all host threads, and one thread).

`small` times the 64^2 bowl launch by launch and replayed from a HIP graph;
`groove512` times the 512^2 V-groove and checks its normals against the
oracle's whole solve.  Two more legs compare the multi-job modes with the
plain per-job path on the same GPU (objects `batched` and `served`):
- batched: 64 independent jobs (side log-uniform 128..1024, bowl / V-groove /
  fBm, grey, K 6..20; 64 spp, 2 bounces, 4 iterations) run one at a time
  through the plain solve and then as one batch replayed from a HIP graph;
- served: the first jobs of a seeded Poisson arrival trace at 20 jobs/s (side
  log-uniform 256..2048, RGB fBm, K 8..16; 128 spp, 2 bounces, 5 iterations)
  replayed through a FIFO loop over the plain solve and through the
  continuous-batching server; latency is arrival to completion.
Both legs require every job's outputs to be bit-identical to the plain path.
`variants` times the paper's variants (shadow-aware PS, robust integration,
the r-ray images) and the scene inside Cornell-like walls on the main
workload, each with its normal and depth error against the ground truth.
"""
import argparse
import json
import os
import struct
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("rays/s + reconstructions/s (batched/served vs plain) at ≤0.05° normal err; p99")
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: scene factory kwargs
    "fbm2048_rgb": dict(size=2048, channels=3, num_lights=16, env_shape=(256, 512), ptp=256.0,
                        spp=256, bounces=3, iterations=5, render_spp=64, render_bounces=3),
    "fbm1024_rgb": dict(size=1024, channels=3, num_lights=16, env_shape=(256, 512), ptp=128.0,
                        spp=256, bounces=3, iterations=5, render_spp=64, render_bounces=3),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_trace_fbm2048_rgb_counters.md")
VALU_PROBE_PROFILE = os.path.join(ROOT, "profiles", "k_probe_valu_calibration.md")
TRACER_SYMBOL = "_ZN5irtps4kern7k_traceILi3EEEvNS0_9TraceArgsE"  # k_trace<3>


def _elf_sections(data):
    shoff = struct.unpack_from("<Q", data, 0x28)[0]
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3a)
    secs = []
    for i in range(shnum):
        name, typ, _flags, addr, offset, size, link, _info, _align, _ent = struct.unpack_from(
            "<IIQQQQIIQQ", data, shoff + i * shentsize)
        secs.append({"name": name, "type": typ, "addr": addr, "offset": offset, "size": size, "link": link})
    names = secs[shstrndx]
    for sec in secs:
        raw = data[names["offset"] + sec["name"]:]
        sec["name"] = raw[:raw.index(b"\0")].decode()
    return secs


def tracer_digest():
    """sha256 of the machine code of k_trace<3> in the built library (the
    gfx950 code object of its offload bundle): a counter profile is only quoted
    for the kernel it was taken on.  None if the library cannot be read."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "paper_1811_02357_amd", "libirtps.so"), "rb") as f:
            data = f.read()
        fat = next(s for s in _elf_sections(data) if s["name"] == ".hip_fatbin")
        bundle = data[fat["offset"]:fat["offset"] + fat["size"]]
        if bundle[:24] != b"__CLANG_OFFLOAD_BUNDLE__":
            return None
        code, p = None, 32
        for _ in range(struct.unpack_from("<Q", bundle, 24)[0]):
            off, size, tlen = struct.unpack_from("<QQQ", bundle, p)
            if b"gfx950" in bundle[p + 24:p + 24 + tlen]:
                code = bundle[off:off + size]
            p += 24 + tlen
        secs = _elf_sections(code)
        symtab = next(s for s in secs if s["type"] == 2)
        strs, text = secs[symtab["link"]], next(s for s in secs if s["name"] == ".text")
        for k in range(symtab["size"] // 24):
            st_name, st_info, _o, _x, st_value, st_size = struct.unpack_from("<IBBHQQ", code, symtab["offset"] + 24 * k)
            raw = code[strs["offset"] + st_name:]
            if raw[:raw.index(b"\0")].decode() == TRACER_SYMBOL and (st_info & 0xf) == 2:
                fo = text["offset"] + (st_value - text["addr"])
                return hashlib.sha256(code[fo:fo + st_size]).hexdigest()
    except (OSError, StopIteration, struct.error, ValueError, TypeError):
        return None
    return None


def profiled_values(workload):
    """The values the committed tracer counter profile hands to this script
    (HBM bytes per launch from copy-calibrated FETCH_SIZE / WRITE_SIZE, VALU
    wave instructions per launch, lane utilisation), or None when the profile
    is missing, is for another workload, or was taken on other tracer sources."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            kv = dict(line.strip("- \n").split(": ", 1) for line in f if line.startswith("- ") and ": " in line)
        digest = tracer_digest()
        if kv.get("workload") != workload or digest is None or kv.get("tracer_code_sha256") != digest:
            return None
        return {"traffic": float(kv["traffic_bytes_per_launch"]),
                "valu": float(kv["valu_wave_instructions_per_launch"]),
                "lanes": float(kv["valu_lane_utilisation"])}
    except (OSError, KeyError, ValueError):
        return None


def probe_rates():
    """The measured VALU issue rates (wave64 instructions per second, every lane
    active) from the committed calibration profile: the peak (the fastest
    instruction kind) and the rate of each kind, or None."""
    try:
        with open(VALU_PROBE_PROFILE) as f:
            kv = dict(line.strip("- \n").split(": ", 1) for line in f if line.startswith("- ") and ": " in line)
        return {"peak": float(kv["valu_peak_wave_instructions_per_s"]),
                "integer_shift_xor_add": float(kv["valu_integer_wave_instructions_per_s"]),
                "register_move": float(kv["valu_move_wave_instructions_per_s"]),
                "fma_f32": float(kv["valu_fma_wave_instructions_per_s"])}
    except (OSError, KeyError, ValueError):
        return None


def profiled_traffic(workload):
    v = profiled_values(workload)
    return None if v is None else v["traffic"]


# Nominal VALU issue rate: 256 CUs x 4 SIMDs, one wave64 instruction per 4
# cycles each at 2.4 GHz (non-packed: the kernels are built without packed FP32),
# i.e. 39.3 T lane-operations/s; the measured peak comes from the issue-rate
# probe (irtps_probe_valu), whose calibration profile bench.py reads.
VALU_ISSUE_NOMINAL = 256 * 4 * 2.4e9 / 4


def algorithmic_bytes(cnt, npx, K, C, iterations):
    """Bytes the tracer launches of one solve must move, by the tracer's
    yardstick: a hit reads the direct radiance of every light and channel at
    the hit sample (4 K C), a continuation also reads albedo and normal there
    (4 C + 12), an escape reads one environment texel (4 C); per pixel the
    origin's normal and albedo (12 + 4 C) are read and the K C gathered values
    written.  The launches also correct each pixel (stage 5 with the fitted
    albedo): per pixel and iteration the K C input values and the direct row
    (4 K C + 4 K) are read and the K C corrected values written, plus the K C
    values of E in the last iteration."""
    hits, esc, cont = cnt[1], cnt[2], cnt[3]
    gather = hits * 4 * K * C + cont * (4 * C + 12) + esc * 4 * C + iterations * npx * (12 + 4 * C + 4 * K * C)
    correction = iterations * npx * (8 * K * C + 4 * K) + npx * 4 * K * C
    return gather + correction


def _oracle_tile_solve(sc, t):
    """The CPU oracle, as it stands, on the t x t centre tile of the terrain: the
    whole solve (all stages, same K, C, spp, bounces, iterations).  Returns
    (segments, seconds, threads)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1811_02357_amd import scenes
    y0 = x0 = (sc.width - t) // 2
    h = np.ascontiguousarray(sc.heights[y0:y0 + t, x0:x0 + t])
    tile = scenes._scene("tile", h, sc.albedo[:, y0:y0 + t, x0:x0 + t], sc.light_dirs,
                         sc.light_intensity, sc.env)
    I0, _ = O.render(tile.heights, tile.normals, tile.albedo, tile.light_dirs, tile.light_intensity,
                     tile.env, sc.render_spp, sc.render_bounces, 0)
    t0 = time.perf_counter()
    r = O.solve(I0, tile.light_dirs, tile.light_intensity, tile.env, sc.spp, sc.bounces,
                sc.iterations, seed=sc.seed)
    return r["counters"]["segments"], time.perf_counter() - t0, O.num_threads()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sc, args):
    """The oracle on the host's cores (all threads, a 512^2 tile) and on one
    thread (a 128^2 tile, in a child process with OMP_NUM_THREADS=1)."""
    import subprocess
    seg, dt, threads = _oracle_tile_solve(sc, args.cpu_tile)
    one = None
    if args.cpu_tile_1t > 0:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-tile", str(args.cpu_tile_1t),
               "--workload", args.workload]
        r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
    out = {"value": seg / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
           "cpu": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": (f"{args.cpu_tile}x{args.cpu_tile} centre tile of the {sc.width}^2 terrain, whole solve "
                      f"(T={sc.iterations}, spp {sc.spp}, B {sc.bounces}, K {sc.num_lights}, "
                      f"C {sc.channels}) on {threads} threads: {seg} segments in {dt:.1f} s")}
    if one is not None:
        out["one_thread"] = {"value": one["segments"] / one["s"], "unit": "rays/s", "cores": one["threads"],
                             "sample": (f"{args.cpu_tile_1t}x{args.cpu_tile_1t} centre tile, whole solve, "
                                        f"one thread: {one['segments']} segments in {one['s']:.1f} s")}
    out["bowl64_whole"] = _oracle_small_solve()
    return out


def _oracle_small_solve():
    """The oracle's whole solve of the 64 x 64 bowl (K 8, grey; spp 16, B 1,
    T 3) on all host threads, inputs rendered by the oracle (untimed): a full
    run, not a sample."""
    from oracle import oracle as O
    from paper_1811_02357_amd import scenes
    sc = scenes.bowl_64()
    I0, _ = O.render_scene(sc)
    t0 = time.perf_counter()
    r = O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, sc.spp, sc.bounces, sc.iterations, seed=sc.seed)
    dt = time.perf_counter() - t0
    seg = r["counters"]["segments"]
    return {"value": seg / dt, "unit": "rays/s", "cores": O.num_threads(), "s": dt,
            "reconstructions_per_s": 1.0 / dt,
            "sample": f"64x64 bowl, whole solve (K 8, spp 16, B 1, T 3): {seg} segments in {dt:.3f} s"}


def _job(sc, dev, irtps, torch, np):
    """Render one job's input images on the GPU and return solve() arguments."""
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    env = T(sc.env)
    I0 = irtps.render(T(sc.heights), T(sc.normals), T(sc.albedo), sc.light_dirs, sc.light_intensity,
                      env, sc.render_spp, sc.render_bounces, seed=sc.seed)
    return dict(images=I0, light_dirs=sc.light_dirs, light_intensity=sc.light_intensity, env=env,
                spp=sc.spp, bounces=sc.bounces, iterations=sc.iterations, seed=sc.seed)


def _same(a, b, torch):
    return all(torch.equal(a[k], b[k]) for k in ("normals", "albedo", "depth", "indirect", "counters"))


def batched_leg(args, dev):
    """64 jobs one at a time through the plain solve vs one batched solve."""
    import numpy as np
    import torch
    from paper_1811_02357_amd import irtps, scenes
    n = args.batched_jobs
    log(f"bench: batched leg, generating {n} jobs")
    jobs = [_job(scenes.batched_job(j), dev, irtps, torch, np) for j in range(n)]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1) / 1e3

    plain_outs = [irtps.solve(**j) for j in jobs]  # warm-up and reference outputs
    torch.cuda.synchronize()
    plain_t = []
    for r in range(args.mode_reps):
        outs, dt = timed(lambda: [irtps.solve(**j, out=o) for j, o in zip(jobs, plain_outs)])
        plain_t.append(dt)
    ws = torch.empty(irtps.batch_workspace_bytes(jobs), dtype=torch.uint8, device=dev)
    bouts = [irtps._outputs_for(j["images"], dev) for j in jobs]
    irtps.batch_solve(jobs, graph=True, outs=bouts, workspace=ws)  # warm-up, graph capture
    torch.cuda.synchronize()
    batch_t = []
    for r in range(args.mode_reps):
        _, dt = timed(lambda: irtps.batch_solve(jobs, graph=True, outs=bouts, workspace=ws))
        batch_t.append(dt)
    same = all(_same(a, b, torch) for a, b in zip(plain_outs, bouts))
    seg = int(sum(int(o["counters"][0]) for o in plain_outs))
    px = sum(int(j["images"].shape[2] * j["images"].shape[3]) for j in jobs)
    tp, tb = float(np.median(plain_t)), float(np.median(batch_t))
    log(f"bench: batched {tb * 1e3:.1f} ms vs plain {tp * 1e3:.1f} ms for {n} jobs")
    return {"jobs": n, "pixels": px, "segments": seg, "equal_to_plain": bool(same),
            "plain": {"s": tp, "rays_per_s": seg / tp, "reconstructions_per_s": n / tp,
                      "p99_s": float(np.quantile(plain_t, 0.99))},
            "batched": {"s": tb, "rays_per_s": seg / tb, "reconstructions_per_s": n / tb,
                        "p99_s": float(np.quantile(batch_t, 0.99)), "graph": True,
                        "tuned_classes": irtps.tuning_entries()},
            "speedup": tp / tb, "repeats": args.mode_reps}


def groove_leg(args, dev):
    """The 512 x 512 V-groove (12 lights, grey, 32 x 64 environment; spp 64,
    B 2, T 5): input images rendered by the CPU oracle, solves timed one by one
    through the plain solve, and the GPU normals compared with the oracle's
    whole solve on every pixel (the metric's 0.05 degree gate)."""
    import numpy as np
    import torch
    from oracle import oracle as O
    from paper_1811_02357_amd import irtps, scenes
    sc = scenes.vgroove_512()
    log("bench: C2 leg, 512^2 V-groove, oracle render and solve")
    I0, _ = O.render_scene(sc)
    ref = O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, sc.spp, sc.bounces, sc.iterations, seed=sc.seed)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    job = dict(images=T(I0), light_dirs=sc.light_dirs, light_intensity=sc.light_intensity, env=T(sc.env),
               spp=sc.spp, bounces=sc.bounces, iterations=sc.iterations, seed=sc.seed)
    ws = torch.empty(irtps.workspace_bytes(**job), dtype=torch.uint8, device=dev)
    out = irtps.solve(**job, workspace=ws)  # warm-up
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(args.groove_reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        irtps.solve(**job, out=out, workspace=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    n = out["normals"].cpu().numpy().astype(np.float64)
    rn = ref["normals"].astype(np.float64)
    cosang = (n * rn).sum(-1) / (np.linalg.norm(n, axis=-1) * np.linalg.norm(rn, axis=-1))
    ang = np.degrees(np.arccos(np.clip(cosang, -1, 1)))
    seg = int(out["counters"][0])
    med = float(np.median(ts))
    log(f"bench: C2 solve {med:.2f} ms, max normal angle vs oracle {ang.max():.2e} deg")
    return {"workload": "vgroove512: 512x512 V-groove (60 deg, depth 64) + 8 px egg-crate, K 12, grey, "
                        "env 32x64 U[0,0.5]; spp 64, bounces 2, iterations 5",
            "repeats": args.groove_reps, "median_ms": med, "p99_ms": float(np.quantile(ts, 0.99)),
            "rays_per_s": seg / (med / 1e3), "reconstructions_per_s": 1e3 / med, "segments": seg,
            "max_normal_err_deg_vs_oracle": float(ang.max()),
            "counters_equal_oracle": out["counters"].cpu().numpy().tolist()[:4] == [
                ref["counters"][k] for k in ("segments", "hits", "escapes", "continuations")]}


def variants_leg(args, dev):
    """The paper's variants and the environment as geometry on the main
    workload (2048^2 RGB fBm, K 16, spp 256, B 3, T 5): whole solves timed (one
    warm-up, median of two) and their normals and depth compared with the
    ground truth.  plain: the default loop; shadow_aware: per-pixel light
    masks in PS; robust: Huber integration; exact_r1..3: the r-ray image in
    place of the gather; box: the scene inside Cornell-like walls of height
    300 px (inputs rendered in the walls), solved with the walls, and
    box_not_modelled: the same images solved with the environment map alone."""
    import numpy as np
    import torch
    from paper_1811_02357_amd import irtps, scenes
    wl = WORKLOADS[args.workload]
    sc = scenes.fbm_terrain(seed=0, **wl)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    gt_n = T(sc.normals).double()
    gt_h = T(sc.heights).double()
    env = T(sc.env)

    def render(box):
        return irtps.render(T(sc.heights), T(sc.normals), T(sc.albedo), sc.light_dirs, sc.light_intensity, env,
                            sc.render_spp, sc.render_bounces, seed=0, box=box)

    walls = scenes.cornell_walls(sc.channels, (64, 128), seed=1)
    box = irtps.Box(300.0, T(walls))
    inputs = {"env": render(None), "box": render(box)}
    runs = [("plain", "env", 0, None), ("shadow_aware", "env", irtps.FLAG_SHADOW_AWARE_PS, None),
            ("robust", "env", irtps.FLAG_ROBUST_INTEGRATION, None),
            ("exact_r1", "env", irtps.flag_exact_r(1), None), ("exact_r2", "env", irtps.flag_exact_r(2), None),
            ("exact_r3", "env", irtps.flag_exact_r(3), None),
            ("box", "box", 0, box), ("box_not_modelled", "box", 0, None)]
    stream = torch.cuda.current_stream()
    res = {}
    for name, src, flags, bx in runs:
        I0 = inputs[src]
        job = dict(images=I0, light_dirs=sc.light_dirs, light_intensity=sc.light_intensity, env=env, spp=sc.spp,
                   bounces=sc.bounces, iterations=sc.iterations, seed=sc.seed, flags=flags, box=bx)
        ws = torch.empty(irtps.workspace_bytes(**{k: v for k, v in job.items()}), dtype=torch.uint8, device=dev)
        out = irtps.solve(**job, workspace=ws)  # warm-up
        ts = []
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            irtps.solve(**job, out=out, workspace=ws)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        n = out["normals"].double()
        cosang = (n * gt_n).sum(-1) / (n.norm(dim=-1) * gt_n.norm(dim=-1))
        ang = torch.rad2deg(torch.arccos(cosang.clamp(-1, 1)))
        d = out["depth"].double()
        rms = float(((d - d.mean()) - (gt_h - gt_h.mean())).pow(2).mean().sqrt())
        res[name] = {"ms": float(np.median(ts)), "segments": int(out["counters"][0]),
                     "median_normal_err_deg": float(ang.median()), "p90_normal_err_deg": float(ang.quantile(0.9)),
                     "depth_rms_px": rms}
        log(f"bench: variant {name}: {res[name]['ms']:.1f} ms, median normal error "
            f"{res[name]['median_normal_err_deg']:.3f} deg, depth rms {rms:.2f} px")
        del ws, out
        torch.cuda.empty_cache()
    return {"workload": args.workload, "box": {"height_px": 300.0, "texture": [64, 128]}, "runs": res}


def small_leg(args, dev):
    """The 64 x 64 bowl (8 lights, grey, spp 16, B 1, T 3), a solve short enough
    that launches matter: timed call by call through the plain solve (kernels
    launched one by one on the stream), through the plain solve replayed from a
    captured HIP graph (IRTPS_FLAG_GRAPH), and through a one-job batched solve
    whose iterations replay a captured HIP graph."""
    import numpy as np
    import torch
    from paper_1811_02357_amd import irtps, scenes
    n = args.small_reps
    log(f"bench: small leg, bowl 64x64, {n} solves each way")
    stream = torch.cuda.Stream()  # graphs need a stream other than the legacy default one
    torch.cuda.set_stream(stream)
    job = _job(scenes.bowl_64(), dev, irtps, torch, np)

    def each(fn):
        ts = []
        for _ in range(n):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return np.array(ts)

    ws = torch.empty(irtps.workspace_bytes(**job), dtype=torch.uint8, device=dev)
    out = irtps.solve(**job, workspace=ws)  # warm-up and reference
    plain = each(lambda: irtps.solve(**job, out=out, workspace=ws))
    gout = irtps._outputs_for(job["images"], dev)
    gws = torch.empty(irtps.workspace_bytes(**job), dtype=torch.uint8, device=dev)
    irtps.solve(**job, flags=irtps.FLAG_GRAPH, out=gout, workspace=gws)  # warm-up, graph capture
    solve_graph = each(lambda: irtps.solve(**job, flags=irtps.FLAG_GRAPH, out=gout, workspace=gws))
    bws = torch.empty(irtps.batch_workspace_bytes([job]), dtype=torch.uint8, device=dev)
    bout = [irtps._outputs_for(job["images"], dev)]
    irtps.batch_solve([job], graph=True, outs=bout, workspace=bws)  # warm-up, graph capture
    graph = each(lambda: irtps.batch_solve([job], graph=True, outs=bout, workspace=bws))
    torch.cuda.synchronize()
    same = _same(out, bout[0], torch) and _same(out, gout, torch)
    torch.cuda.set_stream(torch.cuda.default_stream(dev))
    log(f"bench: small solve {np.median(plain):.3f} ms plain, {np.median(solve_graph):.3f} ms graph-replayed "
        f"solve, {np.median(graph):.3f} ms graph-replayed one-job batch")
    stats = lambda t: {"median_ms": float(np.median(t)), "p99_ms": float(np.quantile(t, 0.99)),
                       "reconstructions_per_s": 1e3 / float(np.median(t))}
    return {"workload": "bowl64: 64x64 bowl, K 8, grey, env 2x4 uniform; spp 16, bounces 1, iterations 3",
            "repeats": n, "equal_to_plain": bool(same), "plain": stats(plain), "graph": stats(solve_graph),
            "batch_graph": stats(graph), "speedup": float(np.median(plain) / np.median(solve_graph))}


def served_leg(args, dev):
    """A truncated Poisson arrival trace through a FIFO loop over the plain
    solve and through the continuous-batching server."""
    import numpy as np
    import torch
    from paper_1811_02357_amd import irtps, scenes
    arr = scenes.served_arrivals(20.0, 60.0, seed=0)[:args.served_jobs]
    n = len(arr)
    log(f"bench: served leg, generating {n} jobs")
    jobs = [_job(scenes.served_job(j), dev, irtps, torch, np) for j in range(n)]
    torch.cuda.synchronize()

    def replay_plain():
        outs, lat, done = [], [], 0.0
        t0 = time.perf_counter()
        for a, job in zip(arr, jobs):
            now = time.perf_counter() - t0
            if now < a:
                time.sleep(a - now)
            outs.append(irtps.solve(**job))
            torch.cuda.synchronize()
            done = time.perf_counter() - t0
            lat.append(done - a)
        return outs, np.asarray(lat), done - arr[0]

    irtps.solve(**jobs[0])  # warm-up
    torch.cuda.synchronize()
    log("bench: served leg, FIFO over the plain solve")
    plain_outs, plain_lat, plain_span = replay_plain()
    seg = int(sum(int(o["counters"][0]) for o in plain_outs))

    budget = int(args.served_budget_gib * (1 << 30))

    def replay_server(fill):
        srv = irtps.Server(budget, device=dev, fill_pixels=fill)
        try:
            ids = []
            t0 = time.perf_counter()
            for a, job in zip(arr, jobs):
                now = time.perf_counter() - t0
                if now < a:
                    time.sleep(a - now)
                ids.append(srv.submit(job))
            sts = [srv.wait(i, 600.0) for i in ids]
            torch.cuda.synchronize()
            ok = all(st.state == irtps.JOB_DONE for st in sts)
            lat = np.asarray([st.end_s - st.submit_s for st in sts])
            span = max(st.end_s for st in sts) - min(st.submit_s for st in sts)
            same = ok and all(_same(a, srv.outputs(i), torch) for a, i in zip(plain_outs, ids))
            stats = srv.stats()
        finally:
            srv.close()
        return lat, span, same, stats

    def summary(l, sp):
        return {"jobs_per_s": n / sp, "rays_per_s": seg / sp, "p50_latency_s": float(np.quantile(l, 0.5)),
                "p99_latency_s": float(np.quantile(l, 0.99)), "span_s": sp}

    res = {"jobs": n, "arrival_rate_per_s": 20.0, "offered_s": float(arr[-1]), "segments": seg,
           "plain_fifo": summary(plain_lat, plain_span)}
    same_all = True
    runs = [("served", args.served_fill), ("served_every_job", 0)]
    runs += [(f"served_fill_{f}", f) for f in args.served_extra_fills]
    for name, fill in runs:
        log(f"bench: served leg, continuous-batching server (fill_pixels {fill})")
        lat, span, same, stats = replay_server(fill)
        same_all = same_all and same
        res[name] = dict(summary(lat, span), budget_gib=args.served_budget_gib, fill_pixels=fill,
                         scheduler_iterations=int(stats["iterations"]))
        log(f"bench: served (fill {fill}) {span:.2f} s vs FIFO plain {plain_span:.2f} s for {n} jobs")
    res["equal_to_plain"] = bool(same_all)
    res["speedup"] = plain_span / res["served"]["span_s"]
    return res


def served_sweep(args, dev):
    """Sustainable arrival rate of the server on the served workload law: for
    rising Poisson rates, jobs arrive for `sweep_window` seconds (cycling
    through a pool of `sweep_pool` jobs of the law, inputs rendered on the GPU
    beforehand) and the sweep stops at the first rate the GPU cannot keep up
    with: fewer than 95% of the arrival rate completed per second over the
    trial, or latencies of the last third of the jobs more than twice those of
    the first third (a growing backlog)."""
    import numpy as np
    import torch
    from paper_1811_02357_amd import irtps, scenes
    log(f"bench: served sweep, generating a pool of {args.sweep_pool} jobs")
    pool = [_job(scenes.served_job(j), dev, irtps, torch, np) for j in range(args.sweep_pool)]
    torch.cuda.synchronize()
    budget = int(args.served_budget_gib * (1 << 30))
    trials = []
    for rate in args.sweep_rates:
        arr = scenes.served_arrivals(rate, args.sweep_window, seed=1)
        srv = irtps.Server(budget, device=dev, fill_pixels=args.served_fill)
        try:
            ids = []
            t0 = time.perf_counter()
            for k, a in enumerate(arr):
                now = time.perf_counter() - t0
                if now < a:
                    time.sleep(a - now)
                job = pool[k % len(pool)]
                K, C, Hh, W = job["images"].shape
                out = {"normals": torch.empty((Hh, W, 3), device=dev), "albedo": torch.empty((C, Hh, W), device=dev),
                       "depth": torch.empty((Hh, W), device=dev), "indirect": None, "counters": None}
                ids.append(srv.submit(job, outs=out))
            sts = [srv.wait(i, 600.0) for i in ids]
        finally:
            srv.close()
        del srv  # its workspace and the trial's outputs go before the next trial's
        torch.cuda.empty_cache()
        ok = all(st.state == irtps.JOB_DONE for st in sts)
        lat = np.asarray([st.end_s - st.submit_s for st in sts])
        span = max(st.end_s for st in sts) - min(st.submit_s for st in sts)
        third = max(len(lat) // 3, 1)
        growth = float(np.median(lat[-third:]) / max(np.median(lat[:third]), 1e-9))
        done_rate = len(lat) / span
        sustained = ok and done_rate >= 0.95 * len(arr) / args.sweep_window and growth <= 2.0
        trials.append({"rate_per_s": rate, "jobs": len(arr), "completed_per_s": done_rate,
                       "p50_latency_s": float(np.quantile(lat, 0.5)), "p99_latency_s": float(np.quantile(lat, 0.99)),
                       "latency_growth_last_vs_first_third": growth, "sustained": bool(sustained)})
        log(f"bench: served sweep rate {rate}/s: {len(arr)} jobs, {done_rate:.2f} done/s, "
            f"p50 {np.quantile(lat, 0.5):.3f} s, p99 {np.quantile(lat, 0.99):.3f} s, growth {growth:.2f}")
        torch.cuda.empty_cache()
        if not sustained:
            break
    ok_rates = [t["rate_per_s"] for t in trials if t["sustained"]]
    return {"window_s": args.sweep_window, "pool": len(pool), "fill_pixels": args.served_fill,
            "trials": trials, "sustainable_rate_per_s": max(ok_rates) if ok_rates else None,
            "first_unsustained_rate_per_s": next((t["rate_per_s"] for t in trials if not t["sustained"]), None)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fbm2048_rgb", choices=sorted(WORKLOADS))
    ap.add_argument("--flat", action="store_true", help="walk every crossing (no pyramid skips)")
    ap.add_argument("--cpu-tile", type=int, default=512)
    ap.add_argument("--cpu-tile-1t", type=int, default=128, help="tile of the one-thread oracle timing (0: off)")
    ap.add_argument("--oracle-tile", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--groove-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="all",
                    choices=["all", "plain", "small", "groove", "batched", "served", "served-sweep", "variants"],
                    help="plain: the main workload only; small/groove/batched/served/served-sweep/variants: the "
                         "main workload and that leg (served-sweep is not part of all)")
    ap.add_argument("--sweep-rates", type=lambda v: [float(x) for x in v.split(",") if x],
                    default=[6.0, 9.0, 12.0, 15.0, 18.0, 21.0, 24.0, 27.0])
    ap.add_argument("--sweep-window", type=float, default=5.0)
    ap.add_argument("--sweep-pool", type=int, default=12)
    ap.add_argument("--small-reps", type=int, default=200)
    ap.add_argument("--batched-jobs", type=int, default=64)
    ap.add_argument("--served-jobs", type=int, default=60)
    ap.add_argument("--served-budget-gib", type=float, default=96.0)
    ap.add_argument("--served-fill", type=int, default=1 << 21,
                    help="server fill_pixels: the oldest job, then least-remaining-work jobs, this many pixels per round")
    ap.add_argument("--served-extra-fills", type=lambda v: [int(x) for x in v.split(",") if x], default=[],
                    help="more fill_pixels values to replay the served trace with (comma-separated)")
    ap.add_argument("--mode-reps", type=int, default=3)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES device to device three times (calibrates byte counters) and exit")
    ap.add_argument("--valu-probe", type=int, default=0, metavar="ITERS",
                    help="only launch the VALU issue-rate probe (ITERS rounds of 16 integer instructions "
                         "per lane, 8 waves per SIMD) three times each with 64, 32, 16 and 1 active lanes "
                         "per wave, print the fastest launch times and exit")
    args = ap.parse_args()

    if args.oracle_tile:
        # child of cpu_baseline: the oracle alone (no GPU touched)
        from paper_1811_02357_amd import scenes
        sc = scenes.fbm_terrain(seed=0, **WORKLOADS[args.workload])
        seg, dt, threads = _oracle_tile_solve(sc, args.oracle_tile)
        print(json.dumps({"segments": seg, "s": dt, "threads": threads}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent jobs would shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1811_02357_amd import irtps, scenes

    dev = torch.device("cuda:0")
    if args.copy_probe:
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n, "launches": 3}), flush=True)
        return
    if args.valu_probe:
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        blocks = cus * 8  # 256-thread blocks: 8 waves per SIMD
        stream = torch.cuda.current_stream()
        irtps.probe_valu(blocks, 16)  # warm-up

        def best_ms(active, kind):
            ms = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                irtps.probe_valu(blocks, args.valu_probe, active, kind)
                e1.record(stream)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            return min(ms)

        # launch order: integer kind at 64, 32, 16, 1 active lanes, then the
        # register-move and fma kinds at 64 (three launches each)
        res = {str(active): best_ms(active, 0) for active in (64, 32, 16, 1)}
        kinds = {"integer_shift_xor_add": res["64"], "register_move": best_ms(64, 1), "fma_f32": best_ms(64, 2)}
        loop = blocks * 4 * 16 * args.valu_probe
        print(json.dumps({"valu_probe": {"cus": cus, "blocks": blocks, "iters": args.valu_probe,
                                         "min_ms_by_active_lanes": res, "min_ms_by_kind": kinds,
                                         "loop_wave_instructions": loop,
                                         "rate_per_s_by_kind": {k: loop / (v / 1e3) for k, v in kinds.items()}}}),
              flush=True)
        return
    wl = WORKLOADS[args.workload]
    log(f"bench: building scene {args.workload}")
    sc = scenes.fbm_terrain(seed=0, **wl)
    W, Hh, C, K = sc.width, sc.height, sc.channels, sc.num_lights
    npx = W * Hh
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    env = T(sc.env)
    log("bench: rendering input images on the GPU")
    I0 = irtps.render(T(sc.heights), T(sc.normals), T(sc.albedo), sc.light_dirs, sc.light_intensity,
                      env, sc.render_spp, sc.render_bounces, seed=0)
    torch.cuda.synchronize()
    flags = irtps.FLAG_FLAT_TRAVERSAL if args.flat else 0
    out = {"normals": torch.empty((Hh, W, 3), device=dev), "albedo": torch.empty((C, Hh, W), device=dev),
           "depth": torch.empty((Hh, W), device=dev), "indirect": torch.empty((K, C, Hh, W), device=dev),
           "counters": torch.zeros(irtps.NUM_COUNTERS, dtype=torch.int64, device=dev)}
    nbytes = irtps.workspace_bytes(I0, sc.light_dirs, sc.light_intensity, env, sc.spp, sc.bounces,
                                   sc.iterations, flags=flags)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)

    def step():
        irtps.solve(I0, sc.light_dirs, sc.light_intensity, env, sc.spp, sc.bounces, sc.iterations,
                    seed=sc.seed, flags=flags, out=out, workspace=ws)

    for w in range(args.warmup):
        log(f"bench: warmup {w + 1}/{args.warmup}")
        step()
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    irtps.profile_begin()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for s in range(args.steps):
        step()
        evs[s + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    trace_ms, launches = irtps.profile_end()
    step_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)]
    log(f"bench: steps {['%.1f' % x for x in step_ms]} ms, wall {wall:.3f} s")
    cnt = out["counters"].cpu().numpy().astype(np.int64).tolist()  # per solve (zeroed per call)

    ms_per_step = sum(step_ms) / args.steps
    seg_per_step = cnt[0]
    value = seg_per_step * args.steps / (sum(step_ms) / 1e3)
    per_launch_ms = trace_ms / max(launches, 1)
    bytes_per_launch = algorithmic_bytes(cnt, npx, K, C, sc.iterations) / sc.iterations
    achieved = bytes_per_launch / (per_launch_ms / 1e3) / 1e9
    line = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W}x{Hh} fBm terrain, C={C}, K={K} Fibonacci lights, "
                               f"env {sc.env.shape[0]}x{sc.env.shape[1]} log-normal",
                   "spp": sc.spp, "bounces": sc.bounces, "iterations": sc.iterations,
                   "traversal": "flat" if args.flat else "pyramid",
                   "schedule": irtps.get_schedule(W, Hh, C, K, sc.bounces)},
        "reconstructions_per_s": args.steps / (sum(step_ms) / 1e3),
        "p99_ms": float(np.quantile(step_ms, 0.99)),
        "segments_per_step": seg_per_step,
        "counters_per_step": {"segments": cnt[0], "hits": cnt[1], "escapes": cnt[2], "continuations": cnt[3]},
        # one gather segment serves every light and channel: K C radiance samples
        "radiance_samples_per_s": value * K * C,
        # the direct light's shadow rays (K per sample and iteration), counted
        # apart from the gather segments; rate over the whole step
        "shadow_rays_per_step": K * npx * sc.iterations,
        "shadow_rays_per_s": K * npx * sc.iterations * args.steps / (sum(step_ms) / 1e3),
        "trace_kernel": {"launches": launches, "avg_ms": per_launch_ms,
                         "share_of_step": trace_ms / sum(step_ms)},
        # the tracer's bytes by the algorithmic yardstick against HBM; the
        # fabric traffic (copy-calibrated FETCH_SIZE + WRITE_SIZE, MALL hits
        # included) from the counter profile of the same kernel
        "hbm_yardstick": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": bytes_per_launch,
                          "fabric_bytes_per_launch": None if args.flat else profiled_traffic(args.workload)},
    }
    prof = None if args.flat else profiled_values(args.workload)
    rates = probe_rates()
    if prof is not None and rates is not None:
        # The binding limit is VALU issue: the counted wave64 VALU instructions of
        # the profiled kernel over this run's launch time, each carrying the
        # profile's mean active lanes.  The roofline is in lane-operations
        # (instructions x active lanes) against the measured full-lane peak, the
        # issue rate of the fastest instruction kind (register moves); the
        # issue rate itself lies between the probe's kinds.
        peak = rates["peak"]
        issue = prof["valu"] / (per_launch_ms / 1e3)
        lane_ops = issue * 64 * prof["lanes"] / 1e12
        line["roofline"] = {"bound": "alu", "achieved": lane_ops, "peak": peak * 64 / 1e12,
                            "unit": "Tlane-op/s", "frac": lane_ops / (peak * 64 / 1e12),
                            "traffic": prof["traffic"]}
        line["valu"] = {"wave_instructions_per_launch": prof["valu"], "issue_per_s": issue,
                        "issue_frac_of_peak": issue / peak, "lane_utilisation": prof["lanes"],
                        "useful_lane_frac_of_peak": issue * prof["lanes"] / peak,
                        "probe_issue_per_s": {k: v for k, v in rates.items() if k != "peak"},
                        "nominal_issue_per_s": VALU_ISSUE_NOMINAL,
                        "sources": [os.path.relpath(TRAFFIC_PROFILE, ROOT), os.path.relpath(VALU_PROBE_PROFILE, ROOT)]}
    else:
        line["roofline"] = dict(line["hbm_yardstick"], bound="hbm",
                                traffic=line["hbm_yardstick"]["fabric_bytes_per_launch"])
    del ws, out, I0
    torch.cuda.empty_cache()
    if args.mode in ("all", "small"):
        line["small"] = small_leg(args, dev)
    if args.mode in ("all", "groove"):
        line["groove512"] = groove_leg(args, dev)
        torch.cuda.empty_cache()
    if args.mode in ("all", "batched"):
        line["batched"] = batched_leg(args, dev)
        torch.cuda.empty_cache()
    if args.mode in ("all", "served"):
        line["served"] = served_leg(args, dev)
        torch.cuda.empty_cache()
    if args.mode in ("all", "variants"):
        line["variants"] = variants_leg(args, dev)
        torch.cuda.empty_cache()
    if args.mode == "served-sweep":
        line["served_sweep"] = served_sweep(args, dev)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline on a tile")
        line["cpu_baseline"] = cpu_baseline(sc, args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
