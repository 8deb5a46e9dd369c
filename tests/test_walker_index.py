"""The walker's resume index (host check of the bound it relies on).

After skipping a pyramid cell the walker needs, for the family of grid lines it
did not leave through, the smallest crossing index m >= 1 whose parameter
t = m |1/d| (binary32 product, as the walk computes it) is at or after the
cell's exit t.  It takes ceil(t |d|) and tries its two neighbours, which is
exact when the travel t |d| stays below 2^15 samples (both the estimate and the
true threshold are then within 2^-8 of t |d|).  This test checks that claim in
binary32 against a brute-force search, on random directions and exits and on
exits placed exactly on, and one ulp either side of, crossing parameters; and
that the near-horizon pass at a walk's start passes over no crossing beyond the
near bound's reach.
"""
import numpy as np

f32 = np.float32


def three_candidates(ainv, d_abs, t):
    est = np.maximum(np.ceil(f32(t) * f32(d_abs)), f32(1))
    lo, hi = est - f32(1), est + f32(1)
    take_lo = (lo >= 1) & (lo * ainv >= t)
    take_est = est * ainv >= t
    return np.where(take_lo, lo, np.where(take_est, est, hi)).astype(np.int64)


def brute_force(ainv, d_abs, t):
    """Smallest m >= 1 with fl(m ainv) >= t, by scanning a wide window around
    t |d| (the products are monotone in m, so the window's first success is the
    answer once the index below the window fails)."""
    out = np.empty(t.shape, np.int64)
    for n in range(t.size):
        c = int(np.floor(np.float64(t[n]) * np.float64(d_abs[n])))
        first = max(1, c - 64)
        if first > 1:
            assert not (f32(first - 1) * ainv[n] >= t[n])
        m = first
        while not (f32(m) * ainv[n] >= t[n]):
            m += 1
        out[n] = m
    return out


def _directions(rng, n):
    d = rng.uniform(-1, 1, n).astype(f32)
    d[: n // 8] = (rng.uniform(1e-6, 1e-3, n // 8) * rng.choice([-1, 1], n // 8)).astype(f32)
    d[d == 0] = f32(0.5)
    return np.abs(d).astype(f32), np.abs(f32(1) / d).astype(f32)


def test_three_candidates_equal_brute_force_on_random_exits():
    rng = np.random.default_rng(7)
    n = 20000
    d_abs, ainv = _directions(rng, n)
    travel = rng.uniform(0, 16384, n)
    t = (travel / d_abs.astype(np.float64)).astype(f32)
    np.testing.assert_array_equal(three_candidates(ainv, d_abs, t), brute_force(ainv, d_abs, t))


def test_three_candidates_on_and_next_to_crossing_parameters():
    rng = np.random.default_rng(8)
    n = 6000
    d_abs, ainv = _directions(rng, n)
    m = rng.integers(1, 16384, n)
    on = (m.astype(f32) * ainv).astype(f32)
    for t in (on, np.nextafter(on, f32(np.inf)), np.nextafter(on, f32(0))):
        t = t.astype(f32)
        np.testing.assert_array_equal(three_candidates(ainv, d_abs, t), brute_force(ainv, d_abs, t))


def test_near_pass_passes_over_only_crossings_within_the_near_reach():
    """A walk that only the near horizon bound clears resumes each family at its
    first crossing with fl(m |1/d|) >= t_lim, t_lim = 24 rsq(dx^2 + dy^2) 0.999
    (the hardware reciprocal square root is within a few ulp: here it is taken
    8 ulp either side of the exact value).  Every crossing passed over must lie
    within 24 samples of horizontal travel, exactly, where the near bound proves
    that it misses; and the resumed crossing is the brute-force first one."""
    rng = np.random.default_rng(9)
    n = 4000
    reach = 24
    theta = rng.uniform(0, 2 * np.pi, n)
    r = np.where(rng.random(n) < 0.2, rng.uniform(1e-4, 1e-2, n), rng.uniform(0.05, 1, n))
    dx, dy = (r * np.cos(theta)).astype(f32), (r * np.sin(theta)).astype(f32)
    dx[:50] = f32(0)
    dy[50:100] = f32(-0.0)
    hd2 = (dx * dx + dy * dy).astype(f32)
    exact = 1.0 / np.sqrt(hd2.astype(np.float64))
    for ulps in (-8, 0, 8):
        rsq = exact.astype(f32)
        for _ in range(abs(ulps)):
            rsq = np.nextafter(rsq, f32(np.inf) if ulps > 0 else f32(0))
        t_lim = (f32(reach) * rsq * f32(0.999)).astype(f32)
        for d in (dx, dy):
            d_abs = np.abs(d).astype(f32)
            with np.errstate(divide="ignore"):
                ainv = np.abs(f32(1) / d).astype(f32)
            moving = d_abs > 0
            m = three_candidates(ainv[moving], d_abs[moving], t_lim[moving])
            np.testing.assert_array_equal(m, brute_force(ainv[moving], d_abs[moving], t_lim[moving]))
            # the last crossing passed over, m - 1, at its exact parameter
            travel = (m - 1) / d_abs[moving].astype(np.float64) * np.sqrt(hd2[moving].astype(np.float64))
            assert np.all(travel < reach), travel.max()
