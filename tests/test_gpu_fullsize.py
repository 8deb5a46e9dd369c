"""The HIP path at the full sizes of the benchmark workloads, in the launch
configuration bench.py times, checked where the oracle can afford it: on the
2048^2 RGB frame, teacher-forced with seeded inputs, the pyramid (against its
definition), direct shading, correction, PS (plain and shadow-aware) and
integration on every pixel, the r-ray image and its pull-push fill on every
pixel, and the gather on sampled pixels (the oracle's per-pixel entry point),
all bitwise; served jobs of the batched and served
workload laws (side <= 512) against the oracle's whole solve; and the batched
and served modes at their full job laws against the plain path (bitwise, any
size)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1811_02357_amd import irtps, scenes
from test_gpu_parity import H, T, _compare_solve, assert_radiance, dev, say  # noqa: F401  (dev is a fixture)

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


def test_direct_2048_full_frame(dev, terrain):
    sc = terrain
    Hh, W, K = sc.height, sc.width, sc.num_lights
    say(f"case: direct irradiance with shadows at {W}x{Hh}, K={K}, every pixel")
    S = H(irtps.direct(T(sc.heights, dev), T(sc.normals, dev), sc.light_dirs, sc.light_intensity))
    ref = O.direct(sc.heights, sc.normals, sc.light_dirs, sc.light_intensity)
    say(f"  shadowed or facing away: {np.mean(ref == 0):.3f}; equal {np.mean(S == ref) * 100:.4f}%")
    assert np.array_equal(S, ref)


def test_exact_r_trace_and_fill_2048_full_frame(dev, terrain):
    """The r-ray variant on the 2048^2 RGB frame, every pixel: the r-ray image
    and its valid mask (r = 1, 2, 3), then the pull-push fill of its holes,
    teacher-forced on the true surface, against the oracle bit for bit."""
    sc = terrain
    Hh, W = sc.height, sc.width
    dH, dn, drho, denv = T(sc.heights, dev), T(sc.normals, dev), T(sc.albedo, dev), T(sc.env, dev)
    pyr = irtps.build_pyramid(dH)
    for r in (1, 2, 3):
        say(f"case: r-ray image r={r} and its fill at {W}x{Hh} C=3, every pixel")
        E, valid = irtps.trace_exact_r(dH, dn, drho, denv, r, 0x5EED_0003, t=1, pyramid=pyr)
        F = irtps.fill_missing(E, valid)
        ref, ok = O.trace_exact_r(sc.heights, sc.normals, sc.albedo, sc.env, r, 0x5EED_0003, t=1)
        say(f"  valid {ok.mean():.4f}")
        assert np.array_equal(H(valid), ok)
        assert np.array_equal(H(E), np.transpose(ref, (1, 2, 0)))
        assert np.array_equal(H(F), np.transpose(O.fill_missing(ref, ok), (1, 2, 0)))


def _window_max(a, lo, width, axis):
    """max of a[lo + c s ... lo + c s + width - 1] along `axis` for every start
    lo + c s (clipped to the array), by doubling windows (van Herk)."""
    a = np.moveaxis(a, axis, 0)
    n = a.shape[0]
    pad = np.concatenate([np.full((1,) + a.shape[1:], -np.inf, a.dtype), a,
                          np.full((width + 2,) + a.shape[1:], -np.inf, a.dtype)])
    m, p = pad, 1
    while 2 * p <= width:
        m = np.maximum(m[:-p], m[p:])
        p *= 2
    full = np.maximum(m[:len(m) - (width - p)], m[width - p:])  # windows of exactly `width`
    return full, n


def test_pyramid_2048_full_frame(dev, terrain):
    """Every level of the pyramid: cell (cx, cy) of level l holds the maximum of
    the samples [cx 2^l - 1, (cx + 1) 2^l + 1] x [cy 2^l - 1, (cy + 1) 2^l + 1]
    (its cell grown by one sample), or +inf when the cell comes within two
    samples of the border."""
    sc = terrain
    Hf = sc.heights
    Hh, W = Hf.shape
    say(f"case: pyramid levels at {W}x{Hh}, every cell")
    pyr = H(irtps.build_pyramid(T(Hf, dev)))
    wc, hc, off, l = W - 1, Hh - 1, 0, 0
    while True:
        s = 1 << l
        lvl = pyr[off:off + wc * hc].reshape(hc, wc)
        # padded index i + 1 holds sample i; window start for cell c is sample c s - 1
        rows, _ = _window_max(Hf.astype(np.float64), 0, s + 3, 1)
        rows = rows[np.arange(wc) * s]                         # [wc][Hh]
        both, _ = _window_max(np.moveaxis(rows, 0, 1), 0, s + 3, 0)
        want = both[np.arange(hc) * s]                         # [hc][wc]
        cx, cy = np.arange(wc) * s, np.arange(hc) * s
        inner = ((cy >= 2) & (cy + s <= Hh - 3))[:, None] & ((cx >= 2) & (cx + s <= W - 3))[None, :]
        want = np.where(inner, want, np.inf)
        assert np.array_equal(lvl.astype(np.float64), want), l
        off += wc * hc
        if wc == 1 and hc == 1:
            break
        wc, hc, l = (wc + 1) // 2, (hc + 1) // 2, l + 1
    say(f"  {l + 1} levels equal")


def test_correct_ps_integrate_2048_full_frame(dev, terrain):
    """Stage 5 (fitted and previous albedo), Eq.4 (plain and shadow-aware) and
    the integration (8 cold cycles, then 4 warm) at 2048^2 RGB with 16 lights,
    every pixel, seeded inputs."""
    sc = terrain
    Hh, W, K, C = sc.height, sc.width, sc.num_lights, sc.channels
    say(f"case: correct / PS / integrate at {W}x{Hh}, K={K}, C={C}, every pixel")
    rng = np.random.default_rng(17)
    F32 = np.float32
    I0 = rng.uniform(0.0, 2.0, (K, C, Hh, W)).astype(F32)
    G = rng.uniform(0.0, 0.5, (K, C, Hh, W)).astype(F32)
    S = rng.uniform(0.0, 1.0, (Hh, W, K)).astype(F32)
    S[S < 0.3] = 0                                            # some lights dropped per pixel
    rho = rng.uniform(0.2, 1.0, (C, Hh, W)).astype(F32)
    Gd = T(np.transpose(G, (2, 3, 0, 1)), dev)
    for mode in (irtps.RHO_FIT, irtps.RHO_PREV):
        E, A = irtps.correct(T(I0, dev), Gd, T(S, dev), T(rho, dev), mode)
        rE, rA = O.correct(I0, G, S, rho, mode)
        assert np.array_equal(H(E), rE) and np.array_equal(H(A), rA), mode
        say(f"  correct mode {mode}: equal")
    del Gd, E, G, rE
    n, r = irtps.ps_solve(A, sc.light_dirs, sc.light_intensity)
    rn, rr = O.ps_solve(O.ps_matrix(sc.light_dirs, sc.light_intensity), rA)
    assert np.array_equal(H(n), rn) and np.array_equal(H(r), rr)
    nm, rm = irtps.ps_solve_masked(A, T(S, dev), sc.light_dirs, sc.light_intensity)
    rnm, rrm = O.ps_solve_masked(sc.light_dirs, sc.light_intensity, rA, S)
    assert np.array_equal(H(nm), rnm) and np.array_equal(H(rm), rrm)
    say("  PS plain and shadow-aware: equal")
    del A, rA, I0
    nt = sc.normals
    cold = irtps.integrate(T(nt, dev), None, 8)
    rc = O.integrate(nt, None, 8)
    assert np.array_equal(H(cold), rc)
    warm = irtps.integrate(T(rnm, dev), cold, 4)
    assert np.array_equal(H(warm), O.integrate(rnm, rc, 4))
    say("  integration cold and warm: equal")


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


def test_served_workload_jobs_against_oracle(dev):
    """Served mode against the oracle's whole solve: jobs of the served law
    (RGB fBm, K 8..16, 128 spp, B 2, T 5) and of the batched law (grey bowl /
    V-groove / fBm, K 6..20, 64 spp, B 2, T 4) with side <= 512, inputs
    rendered by the oracle, all resident in one server at once."""
    picks = [scenes.served_job(0), scenes.served_job(4), scenes.batched_job(3), scenes.batched_job(6),
             scenes.batched_job(2)]
    say("case: served jobs vs the oracle: " + ", ".join(f"{sc.name} {sc.width}^2 K{sc.num_lights} C{sc.channels}"
                                                        for sc in picks))
    jobs, refs = [], []
    for sc in picks:
        I0, _ = O.render_scene(sc)  # inputs from the oracle, never from the GPU
        refs.append(O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, sc.spp, sc.bounces, sc.iterations,
                            seed=sc.seed))
        jobs.append(dict(images=T(I0, dev), light_dirs=sc.light_dirs, light_intensity=sc.light_intensity,
                         env=T(sc.env, dev), spp=sc.spp, bounces=sc.bounces, iterations=sc.iterations,
                         seed=sc.seed))
    torch.cuda.synchronize()
    srv = irtps.Server(16 << 30, device=dev)
    try:
        ids = [srv.submit(job) for job in jobs]
        for jid in ids:
            st = srv.wait(jid, 300.0)
            assert st.state == irtps.JOB_DONE and st.status == 0
        torch.cuda.synchronize()
        for sc, jid, ref in zip(picks, ids, refs):
            got = {k: H(v) for k, v in srv.outputs(jid).items()}
            _compare_solve(ref, got, f"served {sc.name}")
            assert np.array_equal(got["depth"], ref["depth"]) and np.array_equal(got["indirect"], ref["indirect"])
    finally:
        srv.close()


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
