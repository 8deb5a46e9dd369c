"""The HIP path at the full sizes of the benchmark workloads, in the launch
configuration bench.py times, checked where the oracle can afford it: sampled
pixels of the 2048^2 RGB gather and shadow stages against the oracle's
per-pixel entry points (bitwise), and the batched and served modes at their
full job laws against the plain path (bitwise, any size)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1811_02357_amd import irtps, scenes
from test_gpu_parity import H, T, assert_radiance, dev, say  # noqa: F401  (dev is a fixture)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def terrain():
    say("building the 2048^2 RGB fBm terrain")
    return scenes.fbm_terrain(seed=0, size=2048, channels=3, num_lights=16, env_shape=(256, 512), ptp=256.0,
                              spp=256, bounces=3, iterations=5, render_spp=64, render_bounces=3)


def _sample_pixels(W, Hh, count, seed):
    rng = np.random.default_rng(seed)
    corners = [0, W - 1, (Hh - 1) * W, Hh * W - 1]
    edges = [rng.integers(0, W), (Hh - 1) * W + rng.integers(0, W), rng.integers(0, Hh) * W,
             rng.integers(0, Hh) * W + W - 1, 2 * W + 2, (Hh - 3) * W + W - 3]
    inner = rng.choice(W * Hh, size=count, replace=False)
    return np.unique(np.concatenate([corners, edges, inner]).astype(np.int64))


def test_trace_2048_rgb_sampled(dev, terrain):
    sc = terrain
    Hh, W, K, C = sc.height, sc.width, sc.num_lights, sc.channels
    say(f"case: gather at {W}x{Hh} C={C} K={K}, spp 256, B 3, t 2, sampled pixels")
    rng = np.random.default_rng(11)
    S = rng.uniform(0.0, 1.2, size=(Hh, W, K)).astype(np.float32)  # any direct field will do
    seed = 0x5EED_0002
    G = irtps.trace(T(sc.heights, dev), T(sc.normals, dev), T(sc.albedo, dev), T(S, dev), T(sc.env, dev),
                    256, 3, seed, t=2)
    pix = _sample_pixels(W, Hh, 768, 12)
    ref, rc = O.trace_at(sc.heights, sc.normals, sc.albedo, S, sc.env, 256, 3, seed, pix, t=2)
    got = H(G).reshape(Hh * W, K, C)[pix]
    say(f"  {pix.size} pixels, oracle events {rc}")
    assert_radiance(got, ref, "G 2048 sampled")
    assert np.array_equal(got, ref)


def test_direct_2048_sampled(dev, terrain):
    sc = terrain
    Hh, W, K = sc.height, sc.width, sc.num_lights
    say(f"case: direct irradiance with shadows at {W}x{Hh}, K={K}, sampled pixels")
    S = irtps.direct(T(sc.heights, dev), T(sc.normals, dev), sc.light_dirs, sc.light_intensity)
    pix = _sample_pixels(W, Hh, 4096, 13)
    ref = O.direct_at(sc.heights, sc.normals, sc.light_dirs, pix, sc.light_intensity)
    got = H(S).reshape(Hh * W, K)[pix]
    say(f"  {pix.size} pixels, shadowed fraction {np.mean(ref == 0):.3f}")
    assert np.array_equal(got, ref)


def _render_job(sc, dev):
    env = T(sc.env, dev)
    I0 = irtps.render(T(sc.heights, dev), T(sc.normals, dev), T(sc.albedo, dev), sc.light_dirs,
                      sc.light_intensity, env, sc.render_spp, sc.render_bounces, seed=sc.seed)
    return dict(images=I0, light_dirs=sc.light_dirs, light_intensity=sc.light_intensity, env=env,
                spp=sc.spp, bounces=sc.bounces, iterations=sc.iterations, seed=sc.seed)


KEYS = ("normals", "albedo", "depth", "indirect", "counters")


def test_batched_64_jobs_equal_plain(dev):
    say("case: 64 batched jobs (side 128..1024, K 6..20, 64 spp, B 2, T 4) vs each alone")
    jobs = [_render_job(scenes.batched_job(j), dev) for j in range(64)]
    outs = irtps.batch_solve(jobs, graph=True)
    for k, job in enumerate(jobs):
        alone = irtps.solve(**job)
        for key in KEYS:
            assert torch.equal(outs[k][key], alone[key]), (k, key)
    say("  all 64 jobs bit-identical to their plain solves")


def test_served_jobs_equal_plain(dev):
    say("case: 8 served jobs (side 256..2048, RGB, K 8..16, 128 spp, B 2, T 5) vs each alone")
    jobs = [_render_job(scenes.served_job(j), dev) for j in range(8)]
    torch.cuda.synchronize()
    srv = irtps.Server(64 << 30, device=dev)
    try:
        ids = []
        for k, job in enumerate(jobs):
            ids.append(srv.submit(job))
            if k == 2:
                srv.wait(ids[0], 120.0)
        for jid in ids:
            st = srv.wait(jid, 300.0)
            assert st.state == irtps.JOB_DONE and st.status == 0
        torch.cuda.synchronize()
        for k, job in enumerate(jobs):
            alone = irtps.solve(**job)
            for key in KEYS:
                assert torch.equal(srv.outputs(ids[k])[key], alone[key]), (k, key)
        say(f"  served == alone; stats {srv.stats()}")
    finally:
        srv.close()
