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
the whole job; the roofline object is for the tracer kernel, timed with HIP
events around its launches inside the timed steps; `cpu_baseline` is the CPU
oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
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


def algorithmic_bytes(cnt, npx, K, C):
    """Bytes the gather must move per the tracer's yardstick: a hit reads the
    direct radiance of every light and channel at the hit sample (4 K C), a
    continuation also reads albedo and normal there (4 C + 12), an escape reads
    one environment texel (4 C); per pixel the origin's normal and albedo
    (12 + 4 C) are read and the K C gathered values written."""
    hits, esc, cont = cnt[1], cnt[2], cnt[3]
    return (hits * 4 * K * C + cont * (4 * C + 12) + esc * 4 * C + npx * (12 + 4 * C + 4 * K * C))


def cpu_baseline(sc, args):
    """The CPU oracle, as it stands, on a tile of the same terrain: the whole
    solve (all stages, same K, C, spp, bounces, iterations)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1811_02357_amd import scenes
    t = args.cpu_tile
    y0 = x0 = (sc.width - t) // 2
    h = np.ascontiguousarray(sc.heights[y0:y0 + t, x0:x0 + t])
    tile = scenes._scene("tile", h, sc.albedo[:, y0:y0 + t, x0:x0 + t], sc.light_dirs,
                         sc.light_intensity, sc.env)
    I0, _ = O.render(tile.heights, tile.normals, tile.albedo, tile.light_dirs, tile.light_intensity,
                     tile.env, sc.render_spp, sc.render_bounces, 0)
    t0 = time.perf_counter()
    r = O.solve(I0, tile.light_dirs, tile.light_intensity, tile.env, sc.spp, sc.bounces,
                sc.iterations, seed=sc.seed)
    dt = time.perf_counter() - t0
    seg = r["counters"]["segments"]
    return {"value": seg / dt, "unit": "rays/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": (f"{t}x{t} centre tile of the {sc.width}^2 terrain, whole solve "
                       f"(T={sc.iterations}, spp {sc.spp}, B {sc.bounces}, K {sc.num_lights}, "
                       f"C {sc.channels}): {seg} segments in {dt:.1f} s")}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fbm2048_rgb", choices=sorted(WORKLOADS))
    ap.add_argument("--flat", action="store_true", help="walk every crossing (no pyramid skips)")
    ap.add_argument("--cpu-tile", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent jobs would shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1811_02357_amd import irtps, scenes

    dev = torch.device("cuda:0")
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
    bytes_per_launch = algorithmic_bytes(cnt, npx, K, C) / sc.iterations
    achieved = bytes_per_launch / (per_launch_ms / 1e3) / 1e9
    line = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W}x{Hh} fBm terrain, C={C}, K={K} Fibonacci lights, "
                               f"env {sc.env.shape[0]}x{sc.env.shape[1]} log-normal",
                   "spp": sc.spp, "bounces": sc.bounces, "iterations": sc.iterations,
                   "traversal": "flat" if args.flat else "pyramid"},
        "reconstructions_per_s": args.steps / (sum(step_ms) / 1e3),
        "p99_ms": float(np.quantile(step_ms, 0.99)),
        "segments_per_step": seg_per_step,
        "counters_per_step": {"segments": cnt[0], "hits": cnt[1], "escapes": cnt[2], "continuations": cnt[3]},
        "trace_kernel": {"launches": launches, "avg_ms": per_launch_ms,
                         "share_of_step": trace_ms / sum(step_ms)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline on a tile")
        line["cpu_baseline"] = cpu_baseline(sc, args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
