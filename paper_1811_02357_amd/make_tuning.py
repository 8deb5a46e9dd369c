#!/usr/bin/env python3
"""Autotune the tracer schedule for the benchmark's job classes on this GPU and
write the tuning table next to the package (tuning_<arch>.json), which the
binding loads at start-up.  Needs a GPU; takes about a minute.

    python -m paper_1811_02357_amd.make_tuning [--out PATH]
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))


def _job(sc, dev, irtps, torch, np):
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    env = T(sc.env)
    I0 = irtps.render(T(sc.heights), T(sc.normals), T(sc.albedo), sc.light_dirs, sc.light_intensity,
                      env, sc.render_spp, sc.render_bounces, seed=sc.seed)
    return dict(images=I0, light_dirs=sc.light_dirs, light_intensity=sc.light_intensity, env=env,
                spp=sc.spp, bounces=sc.bounces, iterations=sc.iterations, seed=sc.seed)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import numpy as np
    import torch
    from paper_1811_02357_amd import irtps, scenes

    dev = torch.device("cuda:0")
    irtps.tuning_clear()
    seen = set()

    def tune(sc, label):
        K, C = sc.num_lights, sc.channels
        key = (round(0.5 * np.log2(sc.width * sc.height)), int(np.ceil(np.log2(K))), C, sc.bounces)
        if key in seen:
            return
        seen.add(key)
        job = _job(sc, dev, irtps, torch, np)
        t0 = time.time()
        best, ms = irtps.autotune(job)
        print(f"{label}: class {key} -> {best}: {ms[(best['tile_w'], best['ready_batch'])]:.3f} ms "
              f"(16 x 16, 32 lanes: {ms[(16, 32)]:.3f} ms; {time.time() - t0:.1f} s)", flush=True)
        del job
        torch.cuda.empty_cache()

    for size, ptp in ((2048, 256.0), (1024, 128.0)):
        tune(scenes.fbm_terrain(seed=0, size=size, channels=3, num_lights=16, env_shape=(256, 512), ptp=ptp,
                                spp=256, bounces=3, iterations=5, render_spp=64, render_bounces=3),
             f"fbm{size}_rgb")
    for j in range(64):
        tune(scenes.batched_job(j), f"batched job {j}")
    for j in range(48):
        tune(scenes.served_job(j), f"served job {j}")
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    out = args.out or os.path.join(HERE, f"tuning_{arch}.json")
    irtps.tuning_save(out)
    print(f"{irtps.tuning_entries()} entries -> {out}")


if __name__ == "__main__":
    main()
