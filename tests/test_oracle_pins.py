"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself: a
closed form of the paper's equations, an exact solver, brute force, an
exhaustive sweep against binary64 libm, or an invariant of the estimator.  The
paper prints no worked example, so no value here is copied from it; every
expected number is derived in the test from the cited equation.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1811_02357_amd import scenes
from tests.fp32 import fmaf

F32 = np.float32


def angle_deg(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    c = (a * b).sum(-1) / (np.linalg.norm(a, axis=-1) * np.linalg.norm(b, axis=-1))
    return np.degrees(np.arccos(np.clip(c, -1.0, 1.0)))


# ---------------------------------------------------------------------------
# Random numbers: Philox4x32-10 as a stream of 24-bit uniforms.
def test_philox_uniform_and_decorrelated():
    R = 200_000
    ctr = np.zeros((R, 4), np.uint32)
    ctr[:, 0] = np.arange(R) % 4096          # pixel
    ctr[:, 1] = np.arange(R) // 4096          # sample
    ctr[:, 2] = 1
    out = O.philox_n(ctr, (0, 0))
    u = (out >> 8).astype(np.float64) * 2.0 ** -24
    # chi-square over 64 bins per output word (63 dof: 99.99% quantile ~ 116)
    for w in range(4):
        hist = np.bincount((u[:, w] * 64).astype(int), minlength=64)
        chi2 = ((hist - R / 64) ** 2 / (R / 64)).sum()
        assert chi2 < 116, (w, chi2)
    # neighbouring counters and the four words are uncorrelated
    c = np.corrcoef(u.T)
    assert np.abs(c - np.eye(4)).max() < 0.01
    assert abs(np.corrcoef(u[:-1, 0], u[1:, 0])[0, 1]) < 0.01
    # a change of key or of any counter word changes every output word
    base = O.philox([5, 6, 7, 8], [9, 10])
    for pert_c, pert_k in [([6, 6, 7, 8], [9, 10]), ([5, 7, 7, 8], [9, 10]), ([5, 6, 8, 8], [9, 10]),
                           ([5, 6, 7, 9], [9, 10]), ([5, 6, 7, 8], [10, 10]), ([5, 6, 7, 8], [9, 11])]:
        other = O.philox(pert_c, pert_k)
        assert all(a != b for a, b in zip(base, other))


def test_philox_is_a_bijection_on_a_counter_slice():
    """For a fixed key Philox is a permutation of 128-bit counters; on 2^16
    counters that differ in word 0 no two outputs may collide."""
    ctr = np.zeros((1 << 16, 4), np.uint32)
    ctr[:, 0] = np.arange(1 << 16)
    out = O.philox_n(ctr, (123, 456))
    packed = out[:, 0].astype(np.uint64) << np.uint64(32) | out[:, 1].astype(np.uint64)
    assert np.unique(packed).size == 1 << 16


def _philox_reference(ctr, key):
    """Philox4x32-10 written here from its definition (Salmon, Moraes, Dror and
    Shaw, SC'11): ten rounds of two 32x32 -> 64 multiplications by the round
    multipliers, the high halves mixed with the other counter words and the key,
    the key bumped by the Weyl constants between rounds.  Independent of the
    oracle's C code; plain Python integers."""
    M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
    mask = 0xFFFFFFFF
    x0, x1, x2, x3 = (int(v) & mask for v in ctr)
    k0, k1 = (int(v) & mask for v in key)
    for r in range(10):
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = (((p1 >> 32) ^ x1 ^ k0) & mask, p1 & mask, ((p0 >> 32) ^ x3 ^ k1) & mask, p0 & mask)
        k0, k1 = (k0 + W0) & mask, (k1 + W1) & mask
    return [x0, x1, x2, x3]


def test_philox_matches_an_independent_implementation():
    rng = np.random.default_rng(17)
    ctrs = rng.integers(0, 1 << 32, size=(300, 4), dtype=np.uint64).astype(np.uint32)
    keys = rng.integers(0, 1 << 32, size=(300, 2), dtype=np.uint64).astype(np.uint32)
    ctrs[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 2, 3, 4], [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344]]
    keys[:4] = [[0, 0], [0xFFFFFFFF] * 2, [5, 6], [0xA4093822, 0x299F31D0]]
    for c, k in zip(ctrs, keys):
        assert list(O.philox(c.tolist(), k.tolist())) == _philox_reference(c, k), (c, k)
    # the batch entry point draws the same words
    out = O.philox_n(ctrs, (int(keys[2, 0]), int(keys[2, 1])))
    for c, o in zip(ctrs[:20], out[:20]):
        assert o.tolist() == _philox_reference(c, keys[2])


def test_philox_published_known_answers():
    """Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) against the known-answer
    vectors its authors publish with their reference implementation (Random123):
    counter and key all zeros, all ones, and the digits of pi."""
    kat = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
           ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
           ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
            (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in kat:
        assert tuple(O.philox(list(ctr), list(key))) == want, (ctr, key)
        assert tuple(O.philox_n(np.array([ctr], np.uint32), key)[0].tolist()) == want


# ---------------------------------------------------------------------------
# Polynomials standing in for transcendentals.
def test_sincos_quarter_exhaustive():
    """All 2^24 arguments f = m 2^-24 against binary64 sin/cos of pi f / 2."""
    f = (np.arange(1 << 24, dtype=np.float64) * 2.0 ** -24).astype(F32)
    s, c = O.sincos_quarter_n(f)
    x = np.pi / 2 * f.astype(np.float64)
    es = np.abs(s.astype(np.float64) - np.sin(x))
    ec = np.abs(c.astype(np.float64) - np.cos(x))
    assert es.max() < 2.5e-7 and ec.max() < 2.5e-7, (es.max(), ec.max())
    # sin^2 + cos^2 = 1 to binary32 accuracy
    assert np.abs(s.astype(np.float64) ** 2 + c.astype(np.float64) ** 2 - 1).max() < 6e-7


def test_atan2_against_libm():
    rng = np.random.default_rng(0)
    y = rng.standard_normal(400_000).astype(F32) * F32(10) ** rng.uniform(-3, 3, 400_000).astype(F32)
    x = rng.standard_normal(400_000).astype(F32)
    special = np.array([[0, 1], [1, 0], [0, -1], [-1, 0], [1, 1], [-1, 1], [1, -1], [-1, -1],
                        [0, 0], [1e-30, 1], [1, 1e-30], [-0.0, -1]], F32)
    y = np.concatenate([y, special[:, 0]])
    x = np.concatenate([x, special[:, 1]])
    a = O.atan2_n(y, x).astype(np.float64)
    ref = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    ref[(x == 0) & (y == 0)] = 0.0
    err = np.abs(a - ref)
    # -pi and pi name the same angle on the negative x axis
    err = np.minimum(err, np.abs(np.abs(err) - 2 * np.pi))
    assert err.max() < 1e-6, err.max()


# ---------------------------------------------------------------------------
# Cosine-weighted directions (Eq.7 with p(w) = cos(theta)/pi).
def test_cosine_sampling_closed_form_about_z():
    rng = np.random.default_rng(1)
    u = (rng.integers(0, 1 << 24, size=(100_000, 2)) * 2.0 ** -24).astype(F32)
    n = np.tile(np.array([0, 0, 1], F32), (u.shape[0], 1))
    d = O.sample_cosine_n(n, u).astype(np.float64)
    u = u.astype(np.float64)
    # lifted disc point: z = sqrt(1-u1), radius sqrt(u1), azimuth 2 pi u2 from +x to +y
    assert np.abs(d[:, 2] - np.sqrt(1 - u[:, 0])).max() < 3e-7
    r = np.hypot(d[:, 0], d[:, 1])
    assert np.abs(r - np.sqrt(u[:, 0])).max() < 5e-7
    phi = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi)
    dphi = np.abs(phi - 2 * np.pi * u[:, 1])
    dphi = np.minimum(dphi, 2 * np.pi - dphi)
    ok = r > 1e-3
    assert (dphi[ok] * r[ok]).max() < 1e-6


def test_cosine_sampling_frame_about_any_normal():
    rng = np.random.default_rng(2)
    N = 100_000
    n = rng.standard_normal((N, 3))
    n[:10, :] = [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 0], [0, 0, 1e-8], [1, 1, 0], [0, -1, 0],
                 [1e-7, 0, -1], [0, 1e-7, 1], [-1, 0, 0]]
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n = n.astype(F32)
    u = (rng.integers(0, 1 << 24, size=(N, 2)) * 2.0 ** -24).astype(F32)
    d = O.sample_cosine_n(n, u).astype(np.float64)
    u64 = u.astype(np.float64)
    n64 = n.astype(np.float64)
    # unit length, and the component along n is the local z = sqrt(1 - u1)
    assert np.abs(np.linalg.norm(d, axis=1) - 1).max() < 1e-6
    assert np.abs((d * n64).sum(1) - np.sqrt(1 - u64[:, 0])).max() < 1e-6
    # the distribution is rotation invariant: cos(theta) to the normal has
    # cdf P(cos <= c) = c^2 (Kolmogorov-Smirnov against that law)
    c = np.sort((d * n64).sum(1))
    ks = np.abs(c ** 2 - np.arange(1, N + 1) / N).max()
    assert ks < 1.95 / math.sqrt(N) * 1.5


def test_cosine_sampling_mean_direction_is_two_thirds_n():
    """E[d] = (2/3) n for the cosine-weighted hemisphere."""
    rng = np.random.default_rng(3)
    N = 400_000
    nn = np.array([0.3, -0.5, 0.8], np.float64)
    nn /= np.linalg.norm(nn)
    n = np.tile(nn.astype(F32), (N, 1))
    u = (rng.integers(0, 1 << 24, size=(N, 2)) * 2.0 ** -24).astype(F32)
    d = O.sample_cosine_n(n, u).astype(np.float64)
    assert np.abs(d.mean(0) - 2.0 / 3.0 * nn).max() < 5 * 0.5 / math.sqrt(N)


# ---------------------------------------------------------------------------
# Equirectangular lookup.
def test_env_texel_matches_angles():
    rng = np.random.default_rng(4)
    d = rng.standard_normal((200_000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d = d.astype(F32)
    He, We = 32, 64
    rc = O.env_texel_n(d, He, We)
    dd = d.astype(np.float64)
    theta = np.arccos(np.clip(dd[:, 2], -1, 1))
    phi = np.mod(np.arctan2(dd[:, 1], dd[:, 0]), 2 * np.pi)
    ti = theta / np.pi * He
    pj = phi / (2 * np.pi) * We
    safe = (np.abs(ti - np.round(ti)) > 1e-4) & (np.abs(pj - np.round(pj)) > 1e-4)
    assert safe.mean() > 0.99
    assert np.array_equal(rc[safe, 0], np.floor(ti[safe]).astype(int))
    assert np.array_equal(rc[safe, 1], np.floor(pj[safe]).astype(int) % We)
    # poles and axes
    assert tuple(O.env_texel([0, 0, 1], He, We)) == (0, 0)
    assert O.env_texel([0, 0, -1], He, We)[0] == He - 1
    assert O.env_texel([0, 1, 0], He, We) == (He // 2, We // 4)


# ---------------------------------------------------------------------------
# Traversal: the merged crossing walk equals brute force over every crossing.
def brute_force_traverse(H, ij, d):
    """Every grid-line crossing of each ray, evaluated with exact binary32
    arithmetic, sorted by t (x-line first on ties); the first that is outside
    the domain ends the ray as an escape, the first below the surface is the hit."""
    H = np.asarray(H, F32)
    Hh, W = H.shape
    R = ij.shape[0]
    out = np.full((R, 2), -1, np.int32)
    i0 = ij[:, 0]
    j0 = ij[:, 1]
    dx, dy, dz = d[:, 0].astype(F32), d[:, 1].astype(F32), d[:, 2].astype(F32)
    ox, oy, oz = i0.astype(F32), j0.astype(F32), H[j0, i0]
    sx = np.where(np.signbit(dx), -1, 1)
    sy = np.where(np.signbit(dy), -1, 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv_dx = (F32(1) / dx).astype(F32)
        inv_dy = (F32(1) / dy).astype(F32)
    events = []  # (t, family, m, valid, hit, qi, qj)
    for fam, (n_lines, s_, inv, o_major, d_minor, o_minor, n_minor) in enumerate(
            [(W, sx, inv_dx, i0, dy, oy, Hh), (Hh, sy, inv_dy, j0, dx, ox, W)]):
        for m in range(1, n_lines + 1):
            major = o_major + s_ * m
            with np.errstate(invalid="ignore"):
                t = (F32(1) * (s_ * m).astype(F32) * inv).astype(F32)
            t = np.where(np.isnan(t), np.inf, t)
            minor = fmaf(np.where(np.isfinite(t), t, 0), d_minor, o_minor)
            inside = (major >= 0) & (major <= n_lines - 1) & (minor >= 0) & (minor <= n_minor - 1) & np.isfinite(t)
            m0 = np.floor(np.where(inside, minor, 0)).astype(np.int64)
            f = (np.where(inside, minor, 0) - m0.astype(F32)).astype(F32)
            maj = np.clip(major, 0, n_lines - 1)
            m1 = np.clip(m0 + 1, 0, n_minor - 1)
            if fam == 0:
                h0, h1 = H[m0, maj], H[m1, maj]
            else:
                h0, h1 = H[maj, m0], H[maj, m1]
            hl = fmaf(f, (h1 - h0).astype(F32), h0)
            hl = np.clip(hl, np.minimum(h0, h1), np.maximum(h0, h1))
            h = np.where(f == 0, h0, hl)
            z = fmaf(np.where(np.isfinite(t), t, 0), dz, oz)
            hit = inside & (z < h)
            q_minor = np.where(f < 0.5, m0, m0 + 1)
            qi = np.where(fam == 0, major, q_minor)
            qj = np.where(fam == 0, q_minor, major)
            events.append((t, np.full(R, fam), np.full(R, m), inside, hit, qi, qj))
    t = np.stack([e[0] for e in events], 1)
    fam = np.stack([e[1] for e in events], 1)
    inside = np.stack([e[3] for e in events], 1)
    hit = np.stack([e[4] for e in events], 1)
    qi = np.stack([e[5] for e in events], 1)
    qj = np.stack([e[6] for e in events], 1)
    for r in range(R):
        if dx[r] == 0 and dy[r] == 0:
            continue
        order = np.lexsort((fam[r], t[r]))
        for e in order:
            if not np.isfinite(t[r, e]):
                break
            if not inside[r, e]:
                break
            if hit[r, e]:
                out[r] = (qi[r, e], qj[r, e])
                break
    return out


def _ray_set(rng, W, Hh, R):
    ij = np.stack([rng.integers(0, W, R), rng.integers(0, Hh, R)], 1).astype(np.int32)
    d = rng.standard_normal((R, 3))
    kind = rng.integers(0, 6, R)
    d[kind == 1, 0] = 0.0                                  # in a y-line plane
    d[kind == 2, 1] = -0.0                                 # in an x-line plane
    diag = kind == 3
    d[diag, 1] = d[diag, 0] * rng.choice([-1, 1], diag.sum())  # exact diagonals: ties
    d[kind == 4, 0] *= 1e-6                                # nearly along y
    d[kind == 5, 2] = np.abs(d[kind == 5, 2]) * 0.05       # grazing, upward
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return ij, d.astype(F32)


@pytest.mark.parametrize("seed,W,Hh,amp", [(0, 8, 8, 2.0), (1, 8, 8, 0.3), (2, 7, 5, 3.0),
                                            (3, 2, 9, 1.0), (4, 12, 3, 1.5)])
def test_traverse_equals_brute_force(seed, W, Hh, amp):
    rng = np.random.default_rng(seed)
    H = rng.uniform(-amp, amp, size=(Hh, W)).astype(F32)
    H[0, 0] = H[0, 1]  # some equal neighbours: flat segments
    R = 20_000
    ij, d = _ray_set(rng, W, Hh, R)
    got = O.traverse_n(H, ij, d)
    ref = brute_force_traverse(H, ij, d)
    bad = np.where((got != ref).any(1))[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], ref[bad[:5]])
    assert 0.1 < (got[:, 0] >= 0).mean() < 0.9  # both outcomes well represented


def test_traverse_geometry_in_binary64():
    """Ray against the grid-line surface in binary64 geometry (no rounding rules):
    agrees with the oracle except where the ray passes within 1e-4 of the
    surface, of a segment midpoint or of the domain edge."""
    rng = np.random.default_rng(7)
    W = Hh = 8
    H = rng.uniform(-2, 2, size=(Hh, W))
    R = 5000
    ij, d = _ray_set(rng, W, Hh, R)
    got = O.traverse_n(H.astype(F32), ij, d)
    Hf = H.astype(F32).astype(np.float64)
    agree = 0
    amb = amb_nondiag = 0
    for r in range(R):
        o = np.array([ij[r, 0], ij[r, 1], Hf[ij[r, 1], ij[r, 0]]])
        dv = d[r].astype(np.float64)
        ev = []
        for m in range(1, W + 1):
            if dv[0] != 0:
                X = ij[r, 0] + (m if dv[0] > 0 else -m)
                ev.append(((X - o[0]) / dv[0], 0, X))
        for m in range(1, Hh + 1):
            if dv[1] != 0:
                Y = ij[r, 1] + (m if dv[1] > 0 else -m)
                ev.append(((Y - o[1]) / dv[1], 1, Y))
        ev.sort()
        res, near = None, False
        for t, fam, L in ev:
            p = o + t * dv
            minor = p[1] if fam == 0 else p[0]
            nmin = Hh if fam == 0 else W
            d_minor = dv[1] if fam == 0 else dv[0]
            if d_minor != 0 and min(abs(minor), abs(minor - (nmin - 1))) < 1e-4:
                near = True  # grazing the domain edge: binary32 may land either side
            if not (0 <= L <= (W if fam == 0 else Hh) - 1) or not (0 <= minor <= nmin - 1):
                break
            m0 = int(math.floor(minor))
            f = minor - m0
            if fam == 0:
                h = Hf[m0, L] if f == 0 else Hf[m0, L] + f * (Hf[m0 + 1, L] - Hf[m0, L])
            else:
                h = Hf[L, m0] if f == 0 else Hf[L, m0] + f * (Hf[L, m0 + 1] - Hf[L, m0])
            if abs(p[2] - h) < 1e-4 or abs(f - 0.5) < 1e-4:
                near = True
            if p[2] < h:
                qm = m0 if f < 0.5 else m0 + 1
                res = (L, qm) if fam == 0 else (qm, L)
                break
        if near:
            amb += 1
            # exact diagonals run through sample points and rays nearly along a
            # grid line run along it, where binary32 rounding legitimately decides
            amb_nondiag += int(abs(d[r, 0]) != abs(d[r, 1]) and min(abs(d[r, 0]), abs(d[r, 1])) > 1e-4)
            continue
        exp = (-1, -1) if res is None else res
        agree += int(tuple(got[r]) == exp)
    assert agree == R - amb and amb_nondiag < R * 0.01, (agree, amb, amb_nondiag)


def test_traverse_flat_plane_never_hits():
    """A ray leaving a horizontal plane upwards never goes below it (P2)."""
    rng = np.random.default_rng(8)
    H = np.full((16, 16), 3.25, F32)
    ij, d = _ray_set(rng, 16, 16, 20_000)
    d[:, 2] = np.abs(d[:, 2])
    assert (O.traverse_n(H, ij, d)[:, 0] < 0).all()


# ---------------------------------------------------------------------------
# Eq.4: photometric-stereo solve.
def test_ps_matrix_closed_form_ring_lights():
    """8 lights at 45 deg elevation, azimuth k 45 deg: L^T L = diag(2, 2, 4), so
    M = diag(1/2, 1/2, 1/4) L^T."""
    sc = scenes.bowl_64()
    l = sc.light_dirs.astype(np.float64)
    M = O.ps_matrix(sc.light_dirs)
    ref = np.diag([0.5, 0.5, 0.25]) @ l.T
    assert np.abs(M - ref).max() < 2e-7


def test_ps_matrix_pseudo_inverse_and_singular():
    rng = np.random.default_rng(9)
    for K in (3, 5, 12, 64):
        l = rng.standard_normal((K, 3))
        l[:, 2] = np.abs(l[:, 2]) + 0.2
        l /= np.linalg.norm(l, axis=1, keepdims=True)
        s = rng.uniform(0.5, 2.0, K)
        M = O.ps_matrix(l.astype(F32), s.astype(F32))
        Ls = (s[:, None] * l.astype(F32).astype(np.float64))
        assert np.abs(M - np.linalg.pinv(Ls)).max() < 1e-6 * np.abs(np.linalg.pinv(Ls)).max()
    with pytest.raises(ValueError):  # coplanar lights
        O.ps_matrix(np.array([[1, 0, 0], [0, 1, 0], [0.6, 0.8, 0], [0.8, 0.6, 0]], F32))
    with pytest.raises(ValueError):  # fewer than three
        O.ps_matrix(np.array([[0, 0, 1], [0, 1, 0]], F32))


def test_ps_solve_recovers_lambertian_closed_form():
    """Eq.3 images a_k = rho (l_k . n), unshadowed: Eq.4 returns n and rho."""
    rng = np.random.default_rng(10)
    Hh, W, K = 13, 17, 9
    n = rng.standard_normal((Hh, W, 3))
    n[..., 2] = np.abs(n[..., 2]) + 1.0
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    l = scenes.fibonacci_lights(K).astype(np.float64)
    for C in (1, 3):
        rho = rng.uniform(0.2, 1.0, (C, Hh, W))
        A = np.einsum("kx,hwx->khw", l, n)[:, None] * rho[None]   # may be < 0: no clamp in Eq.3
        M = O.ps_matrix(l.astype(F32))
        nn, rr = O.ps_solve(M, A.astype(F32))
        assert angle_deg(nn, n).max() < 1e-3
        assert np.abs(rr / rho - 1).max() < 1e-5


def test_render_ps_shadow_free_bump():
    """Rendered with no inter-reflection (B = 0) and no environment, a bump of
    slope below 0.5 under 45 deg ring lights has neither attached nor cast
    shadows, so PS of the render returns the ground-truth normals (P1)."""
    W = 40
    yy, xx = np.mgrid[0:W, 0:W].astype(np.float64)
    r2 = (xx - 19.5) ** 2 + (yy - 19.5) ** 2
    h = 6.0 - r2 / 40.0                       # |grad| = r/20 < 0.5 inside r < 10
    h = np.where(r2 < 100.0, h, 6.0 - 100.0 / 40.0 + 0 * h)
    sc = scenes._scene("bump", h, np.full((1, W, W), 0.7), scenes.ring_lights([45.0] * 8, [45.0 * k for k in range(8)]),
                       np.ones(8), np.zeros((2, 4, 1)))
    I0, cnt = O.render(sc.heights, sc.normals, sc.albedo, sc.light_dirs, sc.light_intensity,
                       sc.env, spp=4, B=0)
    assert cnt["segments"] == 0
    S = O.direct(sc.heights, sc.normals, sc.light_dirs)
    assert (S > 0).all()
    n, rho = O.ps_solve(O.ps_matrix(sc.light_dirs), I0)
    assert angle_deg(n, sc.normals).max() < 1e-3
    assert np.abs(rho / 0.7 - 1).max() < 1e-5


# ---------------------------------------------------------------------------
# Eq.5-7: the gather.
def _flat_scene(W=8, L=0.2, rho=0.8, He=2, We=4):
    h = np.zeros((W, W))
    return scenes._scene("flat", h, np.full((1, W, W), rho), scenes.ring_lights([45.0] * 8, [45.0 * k for k in range(8)]),
                         np.ones(8), np.full((He, We, 1), L))


def test_uniform_environment_closed_form():
    """Unoccluded upward sample under uniform radiance L: each cosine-weighted
    sample contributes pi L, so G = pi L (P3); with L = 0.2 that is 0.6283185."""
    sc = _flat_scene()
    S = O.direct(sc.heights, sc.normals, sc.light_dirs)
    for spp, B in [(1, 1), (16, 1), (64, 3)]:
        G, cnt = O.trace(sc.heights, sc.normals, sc.albedo, S, sc.env, spp, B, seed=5)
        assert cnt["hits"] == 0 and cnt["escapes"] == cnt["segments"] == 64 * spp
        piL = float(F32(3.14159274) * F32(0.2))
        assert np.abs(G - piL).max() <= 2 * spp * np.spacing(F32(piL))
        assert abs(piL - 0.6283185) < 1e-7


def _irradiance_closed_form(env):
    """Cosine-weighted irradiance of an up-facing point under a piecewise-constant
    equirect map: sum over rows above the horizon of L (dphi/2)(sin^2 th1 - sin^2 th0)."""
    He, We = env.shape[:2]
    tot = np.zeros(env.shape[2])
    for i in range(He):
        th0, th1 = i * np.pi / He, (i + 1) * np.pi / He
        th1c = min(th1, np.pi / 2)
        if th0 >= np.pi / 2:
            break
        w = (2 * np.pi / We) / 2 * (np.sin(th1c) ** 2 - np.sin(th0) ** 2)
        tot += w * env[i].astype(np.float64).sum(0)
    return tot


def test_piecewise_environment_quadrature_and_mc():
    """P4: stratified quadrature (M x M midpoints in (u1, u2)) against the
    closed-form irradiance of a piecewise-constant map.  With two rows the map
    varies only in azimuth, whose texel edges fall on stratum edges, so the
    quadrature is exact up to the binary32 running sum (at most spp 2^-24
    relative for non-negative terms).  With eight rows plain MC, which is
    unbiased, lies within 4 sigma."""
    rng = np.random.default_rng(11)
    h = np.zeros((2, 2))
    S = np.zeros((2, 2, 3), F32)
    for He, We in [(2, 16), (8, 16)]:
        env = rng.uniform(0, 1, (He, We, 3)).astype(F32)
        sc = scenes._scene("flat2", h, np.full((3, 2, 2), 1.0), scenes.fibonacci_lights(3), np.ones(3), env)
        exact = _irradiance_closed_form(env)
        if He == 2:
            M = 64
            Gq, _ = O.trace(sc.heights, sc.normals, sc.albedo, S, env, M * M, 1, 0, flags=O.FLAG_QUADRATURE)
            assert np.abs(Gq[0, :, 0, 0] / exact - 1).max() < M * M * 2.0 ** -24 + 1e-6
        spp = 4096
        Gs = np.stack([O.trace(sc.heights, sc.normals, sc.albedo, S, env, spp, 1, seed)[0][0, :, 0, 0]
                       for seed in range(8)])
        sigma = Gs.std(0, ddof=1) / math.sqrt(Gs.shape[0])
        assert (np.abs(Gs.mean(0) - exact) < 4 * sigma + 1e-6).all()


def test_gather_mc_converges_to_quadrature():
    """P6/P7 on an 8x8 random surface, B = 1: MC at 4096 spp lies within 4 sigma of
    the dense quadrature, and quadrupling the samples halves the RMS error (Sec. IV)."""
    sc = scenes.tiny_scene(8, 8, seed=3, num_lights=4)
    S = O.direct(sc.heights, sc.normals, sc.light_dirs)
    Gq, _ = O.trace(sc.heights, sc.normals, sc.albedo, S, sc.env, 512 * 512, 1, 0, flags=O.FLAG_QUADRATURE)
    errs = {}
    for spp in (64, 256, 1024):
        e2 = []
        for seed in range(6):
            G, _ = O.trace(sc.heights, sc.normals, sc.albedo, S, sc.env, spp, 1, seed + 100)
            e2.append(((G - Gq) ** 2).mean())
        errs[spp] = math.sqrt(np.mean(e2))
    r1 = errs[64] / errs[256]
    r2 = errs[256] / errs[1024]
    assert 1.8 < r1 < 2.2 and 1.8 < r2 < 2.2, errs
    Gs = np.stack([O.trace(sc.heights, sc.normals, sc.albedo, S, sc.env, 4096, 1, seed)[0] for seed in range(16)])
    sigma = Gs.std(0, ddof=1) / math.sqrt(Gs.shape[0])
    z = np.abs(Gs.mean(0) - Gq) / np.maximum(sigma, 1e-7)
    assert (z < 4.5).mean() > 0.99 and z.max() < 7, (np.sort(z.ravel())[-8:])


def test_bounce_monotone_and_bounded():
    """P12: raising the path length only appends non-negative terms, so G grows
    element by element, exactly; G >= 0 and G <= B max(max rho S, pi max L)."""
    sc = scenes.tiny_scene(12, 10, seed=5, channels=3, num_lights=5)
    S = O.direct(sc.heights, sc.normals, sc.light_dirs)
    prev = None
    for B in (0, 1, 2, 3, 4):
        G, cnt = O.trace(sc.heights, sc.normals, sc.albedo, S, sc.env, 32, B, seed=9)
        assert (G >= 0).all()
        bound = B * max(float((sc.albedo.max() * S).max()), float(np.pi * sc.env.max()))
        assert (G <= bound * (1 + 1e-6) + 1e-30).all()
        if prev is not None:
            assert (G >= prev).all()
        prev = G


def test_concavity_only_light():
    """P13: bowl without environment light: the flat plane (above the bowl) gets
    no indirect light, exactly; samples inside the bowl do."""
    sc = scenes.bowl_64()
    S = O.direct(sc.heights, sc.normals, sc.light_dirs)
    # at the bowl centre a cosine-weighted ray clears the rim with probability
    # sin^2(90 - atan(16/24) deg) = 0.69, so 64 samples all escape with odds 5e-11
    G, cnt = O.trace(sc.heights, sc.normals, sc.albedo, S, np.zeros_like(sc.env), 64, 1, seed=0)
    yy, xx = np.mgrid[0:64, 0:64]
    r = np.hypot(xx - 31.5, yy - 31.5)
    assert (G[:, :, r > 25.5] == 0).all()
    assert (G.sum(0)[0][r < 20] > 0).all()


def test_gather_hit_contributions_bookkeeping():
    """Every segment is a hit or an escape; continuations only for B > 1."""
    sc = scenes.tiny_scene(9, 7, seed=6)
    S = O.direct(sc.heights, sc.normals, sc.light_dirs)
    G, c1 = O.trace(sc.heights, sc.normals, sc.albedo, S, sc.env, 8, 1, 0)
    assert c1["segments"] == 63 * 8 == c1["hits"] + c1["escapes"] and c1["continuations"] == 0
    G, c3 = O.trace(sc.heights, sc.normals, sc.albedo, S, sc.env, 8, 3, 0)
    assert c3["segments"] == c3["hits"] + c3["escapes"]
    assert c3["segments"] == 63 * 8 + c3["continuations"]


# ---------------------------------------------------------------------------
# Stage 5 and the loop.
def test_correction_modes_flat_region():
    """P14 on a flat plane under the 45 deg ring lights and uniform environment
    L = 0.2, albedo 0.8: I = rho (sin 45 + pi L).  Plain PS gives rho_0 = sqrt(2) I;
    the literal update rho_{t+1} = sqrt(2) (I - rho_t pi L) oscillates, while the
    fitted albedo is exact after one pass."""
    sc = _flat_scene(W=16)
    I0, _ = O.render(sc.heights, sc.normals, sc.albedo, sc.light_dirs, sc.light_intensity,
                     sc.env, 64, 1)
    s45 = math.sin(math.radians(45))
    I = 0.8 * (s45 + math.pi * 0.2)
    assert np.abs(I0 / I - 1).max() < 1e-5
    r0 = O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, 16, 1, 0)
    assert np.abs(r0["albedo"] / (math.sqrt(2) * I) - 1).max() < 1e-5
    rho = math.sqrt(2) * I
    for T in (1, 2, 3):
        rho = math.sqrt(2) * (I - rho * math.pi * 0.2)
        rp = O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, 16, 1, T, rho_mode=O.RHO_PREV)
        assert np.abs(rp["albedo"] / rho - 1).max() < 1e-4, (T, rp["albedo"].mean(), rho)
        rf = O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, 16, 1, T, rho_mode=O.RHO_FIT)
        assert np.abs(rf["albedo"] / 0.8 - 1).max() < 1e-5
        assert angle_deg(rf["normals"], np.array([0, 0, 1.0])).max() < 1e-3
    assert abs(math.sqrt(2) * I - 1.5108613) < 1e-6


def test_loop_fixed_point_at_ground_truth():
    """P8: images rendered with the solve's own sample stream (tag SOLVE, t = 0)
    from the ground truth; one correction from the ground-truth state removes the
    indirect term exactly, so PS returns the true normals where every light is
    visible."""
    sc = scenes.bowl_64()
    H, n, rho = sc.heights, sc.normals, sc.albedo
    S = O.direct(H, n, sc.light_dirs)
    G, _ = O.trace(H, n, rho, S, sc.env, 16, 1, seed=0, t=0, tag=O.TAG_SOLVE)
    I0 = (rho[None] * (np.transpose(S, (2, 0, 1))[:, None] + G)).astype(F32)
    M = O.ps_matrix(sc.light_dirs)
    lit = (S > 0).all(-1)
    assert lit.mean() > 0.5
    for mode in (O.RHO_PREV, O.RHO_FIT):
        E, A = O.correct(I0, G, S, rho, rho_mode=mode)
        nn, rr = O.ps_solve(M, A)
        assert angle_deg(nn[lit], n[lit]).max() < 1e-3
        assert np.abs(rr[0][lit] / 0.8 - 1).max() < 1e-5


# ---------------------------------------------------------------------------
# Integration (Sec. IV, stage 1).
def _normals_of_gradient(gx, gy):
    n = np.stack([-gx, -gy, np.ones_like(gx)], -1)
    return (n / np.linalg.norm(n, axis=-1, keepdims=True)).astype(F32)


def test_integrate_plane_exact():
    """P9(i): the normals of a plane H = a x + b y integrate back to that plane."""
    Hh, W = 37, 53
    yy, xx = np.mgrid[0:Hh, 0:W].astype(np.float64)
    a, b = 0.375, -0.625
    n = _normals_of_gradient(np.full((Hh, W), a), np.full((Hh, W), b))
    H = O.integrate(n, cycles=8)
    ref = a * xx + b * yy
    ref -= ref.min()
    assert np.abs(H - ref).max() < 1e-4 * max(1.0, ref.max())
    assert H.min() == 0.0


def test_integrate_quadratic_exact():
    """P9(ii): for a quadratic the mean of the end-point derivatives equals the
    forward difference, so the least-squares fit has zero residual."""
    Hh, W = 29, 31
    yy, xx = np.mgrid[0:Hh, 0:W].astype(np.float64)
    c1, c2, c3 = 0.01, -0.015, 0.005
    ref = c1 * xx ** 2 + c2 * yy ** 2 + c3 * xx * yy
    gx = 2 * c1 * xx + c3 * yy
    gy = 2 * c2 * yy + c3 * xx
    H = O.integrate(_normals_of_gradient(gx, gy), cycles=10)
    ref -= ref.min()
    assert np.abs(H - ref).max() < 2e-3


def _exact_lsq(n):
    """Least-squares heights in binary64 by a sparse direct solve of the Neumann
    graph Laplacian (one node pinned)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    n = n.astype(np.float64)
    Hh, W = n.shape[:2]
    nz = np.maximum(n[..., 2], 0.05)
    p = -n[..., 0] / nz
    q = -n[..., 1] / nz
    rows, cols, vals, rhs = [], [], [], []
    e = 0
    idx = np.arange(Hh * W).reshape(Hh, W)
    for j in range(Hh):
        for i in range(W - 1):
            rows += [e, e]; cols += [idx[j, i + 1], idx[j, i]]; vals += [1.0, -1.0]
            rhs.append(0.5 * (p[j, i] + p[j, i + 1])); e += 1
    for j in range(Hh - 1):
        for i in range(W):
            rows += [e, e]; cols += [idx[j + 1, i], idx[j, i]]; vals += [1.0, -1.0]
            rhs.append(0.5 * (q[j, i] + q[j + 1, i])); e += 1
    A = sp.csr_matrix((vals, (rows, cols)), shape=(e, Hh * W))
    L = (A.T @ A).tolil()
    b = A.T @ np.asarray(rhs)
    L[0, :] = 0
    L[0, 0] = 1
    b[0] = 0
    x = spl.spsolve(L.tocsr(), b).reshape(Hh, W)
    return x - x.min()


@pytest.mark.parametrize("shape", [(64, 64), (37, 61), (5, 33), (1, 17)])
def test_integrate_matches_exact_least_squares(shape):
    """P9(iii): the fixed-cycle multigrid against an exact sparse solve."""
    rng = np.random.default_rng(12)
    Hh, W = shape
    n = rng.standard_normal((Hh, W, 3))
    n[..., 2] = np.abs(n[..., 2]) + 0.5
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    n = n.astype(F32)
    H = O.integrate(n, cycles=8)
    ref = _exact_lsq(n)
    assert np.abs(H - ref).max() < 1e-3 * max(1.0, np.abs(ref).max())
    # warm start from the answer stays at the answer
    H2 = O.integrate(n, Hinit=H, cycles=2)
    assert np.abs(H2 - H).max() < 1e-4 * max(1.0, np.abs(ref).max())


# ---------------------------------------------------------------------------
# Whole loop.
def test_loop_improves_bowl_and_is_deterministic():
    """The loop removes inter-reflection bias (Sec. V): on the 64^2 bowl the IRT
    estimate is closer to the truth than plain PS; reruns are bitwise equal."""
    sc = scenes.bowl_64()
    I0, _ = O.render_scene(sc)
    r0 = O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, sc.spp, sc.bounces, 0)
    r3 = O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, sc.spp, sc.bounces, sc.iterations)
    e0 = angle_deg(r0["normals"], sc.normals).mean()
    e3 = angle_deg(r3["normals"], sc.normals).mean()
    assert e3 < 0.6 * e0
    assert abs(r3["albedo"].mean() - 0.8) < abs(r0["albedo"].mean() - 0.8)
    r3b = O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, sc.spp, sc.bounces, sc.iterations)
    for k in ("normals", "albedo", "depth", "indirect"):
        assert np.array_equal(r3[k], r3b[k])
    assert r3["counters"]["segments"] == 3 * 64 * 64 * 16


def test_loop_stop_rule():
    """The optional stop of Sec. IV (last paragraph): the loop ends after the
    first iteration whose surface change D_H = max |H_{t+1} - H_t| is below the
    tolerance.  D_H is measured here from separate fixed-T runs; a tolerance just
    above D_1 stops after one iteration and one between D_2 and D_1 after two,
    each run equal bit for bit to the fixed-T run of that length (the indirect
    images included); 0 runs all T."""
    sc = scenes.bowl_64()
    I0, _ = O.render_scene(sc)
    args = (I0, sc.light_dirs, sc.light_intensity, sc.env, sc.spp, sc.bounces)
    runs = [O.solve(*args, T) for T in range(4)]
    D = [float(np.abs(runs[t + 1]["depth"].astype(np.float64) - runs[t]["depth"]).max()) for t in range(3)]
    assert D[1] < D[0] and D[2] < D[0]
    full = O.solve(*args, 3, stop_tol=0.0)
    assert full["counters"]["iterations"] == 3
    assert np.array_equal(full["depth"], runs[3]["depth"])
    for stop_after, tol in ((1, np.nextafter(F32(D[0]), F32(np.inf))),
                            (2, F32(0.5 * (D[0] + D[1])) if D[1] < D[0] else None)):
        r = O.solve(*args, 3, stop_tol=float(tol))
        assert r["counters"]["iterations"] == stop_after, (stop_after, tol, D)
        for k in ("normals", "albedo", "depth", "indirect"):
            assert np.array_equal(r[k], runs[stop_after][k]), (stop_after, k)
    # a tolerance at D_1 itself does not stop (the change must be below it)
    r = O.solve(*args, 3, stop_tol=float(F32(D[0])))
    assert r["counters"]["iterations"] >= 2


def test_gather_paths_rebuilt_from_the_estimator():
    """The gather rebuilt path by path from Eq.7 and the colour products of
    Fig. 5: the same Philox stream and rays (pinned above), the path weight is
    the product of the albedos met so far, a hit adds weight x albedo x direct
    irradiance for every light, an escape adds weight x pi x environment and
    ends the path.  Summed in sample order with binary32 fma, it must equal the
    oracle bit for bit."""
    sc = scenes.tiny_scene(7, 6, seed=13, channels=3, num_lights=3)
    H, n, rho, env = sc.heights, sc.normals, sc.albedo, sc.env
    S = O.direct(H, n, sc.light_dirs)
    spp, B, seed, t = 5, 3, 77, 2
    G, cnt = O.trace(H, n, rho, S, env, spp, B, seed, t=t)
    Hh, W = H.shape
    K, C = S.shape[2], rho.shape[0]
    pi = F32(3.14159274)
    ref = np.zeros_like(G)
    segs = 0
    for j in range(Hh):
        for i in range(W):
            p = j * W + i
            hit_acc = np.zeros((K, C), F32)
            env_acc = np.zeros(C, F32)
            for s_ in range(spp):
                beta = np.ones(C, F32)
                oi, oj = i, j
                for b in range(1, B + 1):
                    r = O.philox([p, s_, t * 256 + b, O.TAG_SOLVE], [seed, 0])
                    u1 = F32((r[0] >> 8) * 2.0 ** -24)
                    u2 = F32((r[1] >> 8) * 2.0 ** -24)
                    d = O.sample_cosine(n[oj, oi], u1, u2)
                    q = O.traverse(H, oi, oj, d)
                    segs += 1
                    if q is None:
                        er, ec = O.env_texel(d, env.shape[0], env.shape[1])
                        env_acc = fmaf(beta, (pi * env[er, ec]).astype(F32), env_acc)
                        break
                    qi, qj = q
                    w = (beta * rho[:, qj, qi]).astype(F32)
                    hit_acc = fmaf(w[None, :], S[qj, qi][:, None], hit_acc)
                    beta, oi, oj = w, qi, qj
            ref[:, :, j, i] = ((hit_acc + env_acc[None, :]) / F32(spp)).astype(F32)
    assert segs == cnt["segments"]
    assert np.array_equal(G, ref)


def test_subset_entry_points_match_full_stages():
    """The pixel-subset forms are the full stages restricted to those pixels
    (they exist so that GPU results at full image sizes can be checked on a
    sample)."""
    sc = scenes.tiny_scene(24, 20, seed=3, channels=3, num_lights=5)
    S = O.direct(sc.heights, sc.normals, sc.light_dirs, sc.light_intensity)
    pix = np.array([0, 5, 77, 479, 200, 23])
    assert np.array_equal(O.direct_at(sc.heights, sc.normals, sc.light_dirs, pix, sc.light_intensity),
                          S.reshape(-1, 5)[pix])
    G, c = O.trace(sc.heights, sc.normals, sc.albedo, S, sc.env, 16, 3, 99, t=1)
    Ga, _ = O.trace_at(sc.heights, sc.normals, sc.albedo, S, sc.env, 16, 3, 99, pix, t=1)
    assert np.array_equal(Ga, G.reshape(5, 3, -1)[:, :, pix].transpose(2, 0, 1))
    _, call = O.trace_at(sc.heights, sc.normals, sc.albedo, S, sc.env, 16, 3, 99, np.arange(480), t=1)
    assert call == c


# ---------------------------------------------------------------------------
# Pins of the parts a shadow-free or hit-free scene cannot see.
def _step_surface(W, Hh, X0, h):
    """Floor at height 0 for columns i < X0, a plateau of height h from X0 on;
    long in y, so that every row sees the same step."""
    H = np.zeros((Hh, W), F32)
    H[:, X0:] = F32(h)
    return H


def test_direct_cast_shadow_of_a_step():
    """Eq.2 with cast shadows: a light in the x-z plane at elevation e on the
    plateau side shines on a floor sample at distance d = X0 - i from the step's
    face only if the shadow ray has climbed to the plateau's height h when it
    reaches the face, d tan e >= h (the crossing of column X0 is the first sample
    of height h it meets; with dy = 0 there are no other crossings).  Lit samples
    read s (n . l) = s l_z exactly (n = e_z); shadowed ones 0.  Lights pointing
    away from the step, and the plateau itself, are never shadowed.  Elevations
    and h are chosen so that no floor sample lies within 1e-3 of a tie."""
    W, Hh, X0, h = 48, 6, 30, 10.3
    H = _step_surface(W, Hh, X0, h)
    n = np.zeros((Hh, W, 3), F32)
    n[..., 2] = 1
    elev = np.radians([20.0, 33.0, 47.0, 61.0, 75.0, 40.0])
    toward = np.array([1, 1, 1, 1, 1, -1])            # +1: towards the step
    l = np.stack([toward * np.cos(elev), np.zeros_like(elev), np.sin(elev)], -1).astype(F32)
    s = np.array([1.0, 0.5, 2.0, 1.25, 0.75, 1.5], F32)
    S = O.direct(H, n, l, s)
    lz = l[:, 2]
    for k in range(len(elev)):
        tan_e = float(np.float64(lz[k]) / abs(np.float64(l[k, 0])))
        for i in range(W):
            if i < X0 and toward[k] > 0:
                margin = (X0 - i) * tan_e - h
                assert abs(margin) > 1e-3
                lit = margin > 0
            else:
                lit = True
            want = F32(s[k]) * lz[k] if lit else F32(0)
            assert (S[:, i, k] == want).all(), (k, i, S[0, i, k], want)
    # the scene really casts shadows, and not everywhere
    assert (S[:, :X0, :5] == 0).any() and (S[:, :X0, :5] > 0).any()


def test_cumulative_subtraction_flat_region():
    """Stage 5 as written, A_{t+1} = A_t - E_t (LITERAL_CUMULATIVE), on the P14
    flat region (45 deg ring lights, uniform L = 0.2, albedo 0.8, no hits, so
    G = pi L and Eq.4 gives rho = sqrt(2) a for a uniform image a).
    With the previous albedo rho_t: A_{t+1} = A_t - rho_t pi L, hence
    rho_{t+1} = rho_t (1 - sqrt(2) pi L) and rho_t = sqrt(2) I (1 - sqrt(2) pi L)^t.
    With the fitted albedo, 0.8 exactly while the normal is e_z, every step
    removes the same 0.8 pi L: A_t = 0.8 (sin45 - (t - 1) pi L) and
    rho_t = 0.8 |1 - (t - 1) sqrt(2) pi L| (A_3 < 0: the normal flips to -e_z,
    rho is still |g|).  Using I0 instead of A_t as the base gives 1.361274
    resp. 0.8 at t = 2."""
    sc = _flat_scene(W=16)
    I0, _ = O.render(sc.heights, sc.normals, sc.albedo, sc.light_dirs, sc.light_intensity,
                     sc.env, 64, 1)
    I = 0.8 * (math.sin(math.radians(45)) + math.pi * 0.2)
    q = 1 - math.sqrt(2) * math.pi * 0.2
    want_prev = {1: 0.16834532, 2: 0.018757610, 3: 0.0020900369}
    want_fit = {1: 0.8, 2: 0.089138730, 3: 0.62172254}
    for T in (1, 2, 3):
        assert abs(math.sqrt(2) * I * q ** T / want_prev[T] - 1) < 5e-6
        assert abs(0.8 * abs(1 - (T - 1) * (1 - q)) / want_fit[T] - 1) < 5e-6
        # each step cancels about 8/9 of the image, so binary32 error grows ~9x per step
        tol = 2e-6 * 9 ** T
        rp = O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, 16, 1, T, rho_mode=O.RHO_PREV,
                     flags=O.FLAG_LITERAL_CUMULATIVE)
        assert np.abs(rp["albedo"] / want_prev[T] - 1).max() < tol, (T, rp["albedo"].mean())
        rf = O.solve(I0, sc.light_dirs, sc.light_intensity, sc.env, 16, 1, T, rho_mode=O.RHO_FIT,
                     flags=O.FLAG_LITERAL_CUMULATIVE)
        assert np.abs(rf["albedo"] / want_fit[T] - 1).max() < tol, (T, rf["albedo"].mean())


def _step_view_factor(d, h):
    """Cosine-weighted fraction of the hemisphere of an up-facing point that an
    infinitely long step of height h at distance d blocks: the 2-D view factor
    1/2 (sin 90 - sin atan(d/h)) = 1/2 (1 - d / sqrt(d^2 + h^2))."""
    return 0.5 * (1.0 - d / math.hypot(d, h))


def test_gather_hit_weight_against_step_view_factor():
    """Eq.5-7 with a surface hit, B = 1: floor samples at distance d from a step
    of height h (long in y), n = e_z everywhere, uniform S_p, albedo rho_p and
    environment L.  A path that hits adds rho_p S_p to every light's sum, one that
    escapes pi L; so G = F rho_p S_p + (1 - F) pi L with F the blocked fraction.
    The surface is linear along grid lines, so the step's face is a one-sample
    ramp from column X0 - 1 to X0 and F lies between the view factors of a wall
    at d and at d - 1.  Checked: the hit fraction against that bracket (4 sigma),
    and G against hits rho_p S_p + escapes pi L (the estimator's own sum)."""
    W, Hh, X0, h, d = 64, 1025, 40, 32.0, 16
    H = _step_surface(W, Hh, X0, h)
    n = np.zeros((Hh, W, 3), F32)
    n[..., 2] = 1
    K, rho_p, S_p, L = 3, 0.3, 2.0, 0.05
    S = np.full((Hh, W, K), S_p, F32)
    S[..., 1] *= F32(0.5)
    rho = np.full((1, Hh, W), rho_p, F32)
    env = np.full((2, 4, 1), L, F32)
    rows = np.arange(256, 768)
    pix = rows * W + (X0 - d)
    spp = 512
    Gs, cnt = O.trace_at(H, n, rho, S, env, spp, 1, seed=21, pix=pix)
    assert cnt["segments"] == rows.size * spp == cnt["hits"] + cnt["escapes"]
    F_hat = cnt["hits"] / cnt["segments"]
    lo, hi = _step_view_factor(d, h), _step_view_factor(d - 1, h)
    sig = math.sqrt(hi * (1 - lo) / cnt["segments"])
    assert lo - 4 * sig < F_hat < hi + 4 * sig, (lo, F_hat, hi)
    # per pixel: G = (hits rho_p S_p[k] + escapes pi L) / spp, recomputed from
    # each pixel's own counts
    piL = float(F32(3.14159274) * F32(L))
    for m in range(0, rows.size, 37):
        _, c1 = O.trace_at(H, n, rho, S, env, spp, 1, seed=21, pix=pix[m:m + 1])
        for k in range(K):
            want = (c1["hits"] * float(F32(rho_p) * S[0, 0, k]) + c1["escapes"] * piL) / spp
            assert abs(Gs[m, k, 0] / want - 1) < 2 * spp * 2.0 ** -24, (m, k, Gs[m, k, 0], want)
    # and the mean over the rows lies in the bracket of the closed form
    Gm = Gs[:, 0, 0].astype(np.float64).mean()
    g = lambda F: F * rho_p * S_p + (1 - F) * math.pi * L
    assert g(lo) - 4 * sig * (rho_p * S_p - math.pi * L) < Gm < g(hi) + 4 * sig * (rho_p * S_p - math.pi * L)


def test_gather_second_bounce_weight_is_the_albedo_product():
    """Eq.5-7 with B = 2 on the step: a second segment starts at the first hit q
    with weight beta = rho(q) (Fig. 5's colour product), so with uniform
    rho_p, S_p and L every path adds one of rho_p S_p + rho_p^2 S_p,
    rho_p S_p + rho_p pi L, or pi L.  The counters split the segments: first
    hits = continuations c, second hits = hits - c, second escapes = 2c - hits,
    first escapes = escapes - (2c - hits); G must equal the sum they give.  A
    weight without the albedo product (rho_p S_p for a second hit) misses it."""
    W, Hh, X0, h, d = 40, 64, 24, 12.0, 3
    H = _step_surface(W, Hh, X0, h)
    n = np.zeros((Hh, W, 3), F32)
    n[..., 2] = 1
    rho_p, S_p, L = F32(0.6), F32(1.5), F32(0.1)
    S = np.full((Hh, W, 1), S_p, F32)
    rho = np.full((1, Hh, W), rho_p, F32)
    env = np.full((2, 4, 1), L, F32)
    spp = 256
    piL = float(F32(3.14159274) * L)
    two_hits = 0
    for j in range(8, 56, 6):
        p = j * W + (X0 - d)
        G, c = O.trace_at(H, n, rho, S, env, spp, 2, seed=3, pix=[p])
        cont, hits, esc = c["continuations"], c["hits"], c["escapes"]
        h2 = hits - cont
        e2 = 2 * cont - hits
        e1 = esc - e2
        assert min(h2, e2, e1) >= 0 and cont + e1 == spp
        want = (cont * float(rho_p * S_p) + e1 * piL + h2 * float(F32(rho_p * rho_p) * S_p)
                + e2 * float(rho_p * F32(piL))) / spp
        assert abs(G[0, 0, 0] / want - 1) < 4 * spp * 2.0 ** -24, (j, G[0, 0, 0], want)
        two_hits += h2
    assert two_hits > 0  # some second segments hit (from the ramp's floor end)


# ---------------------------------------------------------------------------
# Shadow-aware PS (Eq.4 over the lights that reach a pixel).
def _shadowed_scene():
    """A floor with a step (plateau of height 10 from column 30) cut by a
    narrow trench, and a paraboloid hill; 12 Fibonacci lights (elevations down
    to 2.4 deg): attached shadows on the hill's far sides, cast shadows in
    front of the step and behind the hill, almost none in the trench."""
    W, Hh = 48, 40
    yy, xx = np.mgrid[0:Hh, 0:W].astype(np.float64)
    h = np.where(xx >= 30, 10.0, 0.0)
    r2 = (xx - 14.0) ** 2 + (yy - 20.0) ** 2
    h = h + np.where(r2 < 64.0, 4.0 * (1 - r2 / 64.0), 0.0)
    # a narrow trench in the plateau: its floor sees fewer than three lights
    h = np.where((xx >= 39) & (xx <= 41) & (yy >= 6) & (yy <= 33), -12.0, h)
    rng = np.random.default_rng(4)
    rho = rng.uniform(0.3, 0.9, (3, Hh, W))
    K = 12
    s = np.linspace(0.8, 1.3, K)
    return scenes._scene("step_hill", h, rho, scenes.fibonacci_lights(K), s, np.zeros((2, 4, 3)))


def test_shadow_aware_ps_recovers_normals_where_three_lights_remain():
    """Images with no indirect light (B = 0, no environment) are I = rho S with
    S = s max(0, n.l) V.  At a pixel whose kept lights (S > 0) number at least
    three and are well conditioned, Eq.4 over those lights alone is exact: it
    returns n and rho.  Plain Eq.4 over all lights is wrong wherever a light is
    shadowed; where fewer than three lights remain the masked solve is the
    plain one, bit for bit."""
    sc = _shadowed_scene()
    I0, cnt = O.render(sc.heights, sc.normals, sc.albedo, sc.light_dirs, sc.light_intensity,
                       sc.env, spp=1, B=0)
    S = O.direct(sc.heights, sc.normals, sc.light_dirs, sc.light_intensity)
    l = sc.light_dirs.astype(np.float64) * sc.light_intensity.astype(np.float64)[:, None]
    kept = S > 0
    ok = np.zeros(kept.shape[:2], bool)
    for j in range(kept.shape[0]):
        for i in range(kept.shape[1]):
            Lp = l[kept[j, i]]
            if Lp.shape[0] >= 3:
                N = Lp.T @ Lp
                ok[j, i] = np.linalg.det(N) > 1e-7 * (np.trace(N) / 3) ** 3
    shadowed = ~kept.all(-1)
    assert shadowed.mean() > 0.2 and (ok & shadowed).sum() > 200
    n, rho = O.ps_solve_masked(sc.light_dirs, sc.light_intensity, I0, S)
    assert angle_deg(n[ok], sc.normals[ok]).max() < 1e-3
    assert np.abs(rho[:, ok] / sc.albedo[:, ok] - 1).max() < 1e-5
    n0, rho0 = O.ps_solve(O.ps_matrix(sc.light_dirs, sc.light_intensity), I0)
    assert angle_deg(n0[ok & shadowed], sc.normals[ok & shadowed]).max() > 1.0
    assert (~ok).any()
    assert (n[~ok] == n0[~ok]).all() and (rho[:, ~ok] == rho0[:, ~ok]).all()
    # unshadowed pixels: the kept rows are all rows; the same solve up to the
    # rounding of the per-pixel matrix
    full = kept.all(-1)
    assert angle_deg(n[full], n0[full]).max() < 1e-3


# ---------------------------------------------------------------------------
# Robust integration (Sec. IV stage 1, "M-estimator"): the Huber M-estimator by
# half-quadratic splitting on top of the least-squares multigrid.
def _edge_targets(n):
    n = n.astype(np.float64)
    nz = np.maximum(n[..., 2], 0.05)
    p, q = -n[..., 0] / nz, -n[..., 1] / nz
    return 0.5 * (p[:, :-1] + p[:, 1:]), 0.5 * (q[:-1] + q[1:])


def _huber_energy(H, gx, gy, delta):
    H = H.astype(np.float64)
    r = np.concatenate([((H[:, 1:] - H[:, :-1]) - gx).ravel(), ((H[1:] - H[:-1]) - gy).ravel()])
    a = np.abs(r)
    return float(np.where(a <= delta, 0.5 * r * r, delta * a - 0.5 * delta * delta).sum())


def _plane_with_outliers(W=40, Hh=36):
    """Normals of the plane H = 0.3 x - 0.2 y with a 2 x 2 block of wrong ones
    (a specular spike: a 60 deg tilt towards +x)."""
    gx = np.full((Hh, W), 0.3)
    gy = np.full((Hh, W), -0.2)
    n = _normals_of_gradient(gx, gy).astype(np.float64)
    n[17:19, 19:21] = [math.sin(math.radians(60)), 0.0, math.cos(math.radians(60))]
    yy, xx = np.mgrid[0:Hh, 0:W].astype(np.float64)
    ref = 0.3 * xx - 0.2 * yy
    return n.astype(F32), ref - ref.min()


def test_robust_integration_huber_energy_never_rises():
    """The Huber cost of a residual r is min over z of (r - z)^2 / 2 + delta |z|,
    attained at z = shrink(r).  A round sets z for the current surface (the
    joint cost then equals the Huber energy) and V-cycles lower the joint cost in
    H for that z; so the Huber energy of the surface never rises from round to
    round, and it falls while outliers remain."""
    n, _ = _plane_with_outliers()
    gx, gy = _edge_targets(n)
    e = [_huber_energy(O.integrate_robust(n, None, 8, delta=0.5, rounds=r, rcycles=2), gx, gy, 0.5)
         for r in range(0, 7)]
    for a, b in zip(e, e[1:]):
        assert b <= a * (1 + 1e-6) + 1e-6, e
    assert e[-1] < 0.9 * e[0], e


def test_robust_integration_without_outliers_is_least_squares():
    """With a threshold no residual reaches, every shrinkage is 0, the edge
    targets are the least-squares ones and the extra V-cycles stay at the exact
    least-squares surface (binary64 sparse solve) within 1e-3 px; with no round
    the result is or_integrate's, bit for bit."""
    rng = np.random.default_rng(12)
    for shape in [(24, 31), (9, 40)]:
        nn = rng.standard_normal((*shape, 3))
        nn[..., 2] = np.abs(nn[..., 2]) + 1.0
        nn = (nn / np.linalg.norm(nn, axis=-1, keepdims=True)).astype(F32)
        H = O.integrate_robust(nn, None, 8, delta=1e30, rounds=3, rcycles=2)
        assert np.abs(H - _exact_lsq(nn)).max() < 1e-3
        assert np.array_equal(O.integrate_robust(nn, None, 8, 0.5, 0, 2), O.integrate(nn, None, 8))


def test_robust_integration_suppresses_an_outlier_block():
    """A plane whose normals are wrong in one 2 x 2 block: least squares spreads
    the wrong gradients over a wide neighbourhood, the Huber solution keeps the
    plane away from the block.  A Huber edge pulls with at most delta instead of
    its residual (here about 0.7), so with delta = 0.1 the error more than 4
    samples from the block is at most a quarter of the L2 error there."""
    n, ref = _plane_with_outliers()
    l2 = O.integrate(n, None, 8)
    rb = O.integrate_robust(n, None, 8, delta=0.1, rounds=8, rcycles=2)
    Hh, W = n.shape[:2]
    yy, xx = np.mgrid[0:Hh, 0:W]
    far = (np.abs(yy - 17.5) > 4) | (np.abs(xx - 19.5) > 4)
    e_l2 = np.abs((l2 - l2[0, 0]) - (ref - ref[0, 0]))[far].max()
    e_rb = np.abs((rb - rb[0, 0]) - (ref - ref[0, 0]))[far].max()
    assert e_l2 > 0.2 and e_rb < 0.25 * e_l2, (e_l2, e_rb)


# ---------------------------------------------------------------------------
# The paper's r-ray variant (Sec. IV, tracing paragraph, Fig. 5) and the fill of
# the pixels it leaves empty.
@pytest.mark.parametrize("r", [1, 2, 3])
def test_exact_r_trace_is_the_gather_sample_that_escapes_on_its_r_th_ray(r):
    """The r-ray image uses the gather's sample 0 (same counters).  With no
    direct light (S = 0), spp 1 and B = r the gather adds only the environment
    term of an escape, so a pixel whose path escapes on ray r has exactly the
    gather's value; a path that escapes earlier gives the same gather value
    with B = r - 1 and r, one whose r-th ray hits gives 0 in both.  So the
    pixel is valid exactly where the gathers with B = r and B = r - 1 differ
    (every texel is positive), and its value is the B = r gather's."""
    sc = scenes.tiny_scene(23, 19, seed=7, channels=3, num_lights=4, amp=4.0)
    S0 = np.zeros(sc.heights.shape + (4,), F32)
    env = sc.env + F32(0.05)
    E, ok = O.trace_exact_r(sc.heights, sc.normals, sc.albedo, env, r, seed=99, t=2)
    Gr, _ = O.trace(sc.heights, sc.normals, sc.albedo, S0, env, 1, r, 99, t=2)
    Gp, _ = O.trace(sc.heights, sc.normals, sc.albedo, S0, env, 1, r - 1, 99, t=2)
    differ = (Gr[0] != Gp[0]).any(0)
    assert np.array_equal(ok.astype(bool), differ)
    assert np.array_equal(E[:, ok.astype(bool)], Gr[0][:, ok.astype(bool)])
    assert (E[:, ~ok.astype(bool)] == 0).all()
    assert 0 < ok.mean() < 1  # the scene leaves pixels empty at every depth


def test_fill_missing_pull_push():
    """Pull-push fill: pixels with a value keep it bit for bit; a constant field
    with holes is filled with that constant (3/4: weighted sums of it are
    exact); a pixel alone in its 2 x 2 block without a value takes the mean of
    its three siblings; with no valid pixel everything is 0."""
    rng = np.random.default_rng(3)
    E = rng.uniform(0, 1, (3, 37, 53)).astype(F32)
    ok = (rng.uniform(0, 1, (37, 53)) < 0.3).astype(np.uint8)
    F = O.fill_missing(E, ok)
    m = ok.astype(bool)
    assert np.array_equal(F[:, m], E[:, m]) and np.isfinite(F).all()
    assert np.array_equal(O.fill_missing(E, np.ones_like(ok)), E)
    c = np.full((1, 37, 53), 0.75, F32)
    assert (O.fill_missing(c, ok) == F32(0.75)).all()
    one = np.ones((8, 8), np.uint8)
    one[2, 5] = 0
    G = O.fill_missing(E[:1, :8, :8], one)
    sib = [E[0, 2, 4], E[0, 3, 4], E[0, 3, 5]]  # block rows 2-3, columns 4-5, in (0,0),(1,0),(0,1),(1,1) order
    assert G[0, 2, 5] == np.float32(np.float32(np.float32(sib[0] + sib[1]) + sib[2]) / np.float32(3))
    assert (O.fill_missing(E, np.zeros_like(ok)) == 0).all()


# ---------------------------------------------------------------------------
# The known environment as geometry (Sec. IV stages 0, 3 and 4): walls on the
# borders of the sample grid, up to height Z, open above.
def _wall_box(Z, th, tw, C, K, rng=None, S_val=None):
    rng = rng or np.random.default_rng(0)
    alb = rng.uniform(0.2, 0.9, (4, th, tw, C)).astype(F32)
    box = dict(Z=Z, albedo=alb)
    if S_val is not None:
        box["S"] = np.full((4, th, tw, K), S_val, F32)
    return box


def test_box_below_the_surface_changes_nothing():
    """Walls lower than every sample can never be met: a ray that leaves the
    surface crosses the border above it, so above the walls.  Gather, direct
    light, render and the loop then equal the environment-only oracle bit for bit."""
    sc = scenes.tiny_scene(17, 13, seed=3, channels=3, num_lights=6, amp=3.0)
    Hf = (sc.heights - sc.heights.min() + 1.0).astype(F32)
    box = _wall_box(0.5, 3, 5, 3, 6)
    box["S"] = O.box_shade(17, 13, box, sc.light_dirs, sc.light_intensity)
    S = O.direct(Hf, sc.normals, sc.light_dirs, sc.light_intensity)
    assert np.array_equal(O.direct(Hf, sc.normals, sc.light_dirs, sc.light_intensity, box_z=0.5), S)
    G0, c0 = O.trace(Hf, sc.normals, sc.albedo, S, sc.env, 16, 3, 5)
    G1, c1 = O.trace(Hf, sc.normals, sc.albedo, S, sc.env, 16, 3, 5, box=box)
    assert np.array_equal(G0, G1) and c0 == c1
    I0, _ = O.render(Hf, sc.normals, sc.albedo, sc.light_dirs, sc.light_intensity, sc.env, 8, 2, 1)
    I1, _ = O.render(Hf, sc.normals, sc.albedo, sc.light_dirs, sc.light_intensity, sc.env, 8, 2, 1, box=box)
    assert np.array_equal(I0, I1)


def _corner_factor(a, b, c):
    """View factor from a differential area to a parallel a x b rectangle at
    distance c with one corner above the area (the standard closed form)."""
    X, Y = a / c, b / c
    return (X / math.sqrt(1 + X * X) * math.atan(Y / math.sqrt(1 + X * X))
            + Y / math.sqrt(1 + Y * Y) * math.atan(X / math.sqrt(1 + Y * Y))) / (2 * math.pi)


def test_box_walls_take_their_view_factor():
    """Eq.5-7 on a flat floor in the box, one bounce, uniform wall albedo and
    wall irradiance, uniform environment: a sample sees the open top through the
    view factor F of the rectangle of the walls' rims (four corner rectangles
    from the sample's foot), so G = rho_w S_w (1 - F) + pi L F.  Cosine-weighted
    quadrature over 128^2 strata, at the centre and at off-centre samples."""
    W, Hh, Z, K = 9, 9, 4.0, 2
    Hf = np.zeros((Hh, W), F32)
    n = np.zeros((Hh, W, 3), F32)
    n[..., 2] = 1
    rho = np.full((3, Hh, W), 0.5, F32)
    env = np.empty((2, 4, 3), F32)
    env[:] = np.array([0.1, 0.2, 0.3], F32)
    box = dict(Z=Z, albedo=np.empty((4, 4, 6, 3), F32), S=np.empty((4, 4, 6, K), F32))
    box["albedo"][:] = np.array([0.6, 0.3, 0.9], F32)
    box["S"][..., 0], box["S"][..., 1] = 1.5, 0.25
    M = 128
    G, cnt = O.trace(Hf, n, rho, np.zeros((Hh, W, K), F32), env, M * M, 1, 0, flags=O.FLAG_QUADRATURE, box=box)
    assert cnt["hits"] == 0
    for i, j in ((4, 4), (2, 5), (1, 7), (6, 1)):
        F = sum(_corner_factor(a, b, Z) for a in (i, W - 1 - i) for b in (j, Hh - 1 - j))
        ref = np.array([[box["albedo"][0, 0, 0, c] * box["S"][0, 0, 0, k] * (1 - F) + math.pi * env[0, 0, c] * F
                         for c in range(3)] for k in range(K)])
        assert np.abs(G[:, :, j, i] - ref).max() <= 2e-3 * np.abs(ref).max(), (i, j)


def test_box_wall_and_texel_against_binary64_geometry():
    """The wall a ray meets and its texel, against an independent binary64
    intersection with the four planes (nearest plane ahead, height below Z),
    for rays from every kind of sample, away from texel edges, corners and the
    rim."""
    rng = np.random.default_rng(5)
    W, Hh, Z, th, tw = 23, 17, 6.0, 5, 7
    box = _wall_box(Z, th, tw, 1, 1)
    R = 20000
    ij = np.stack([rng.integers(0, W, R), rng.integers(0, Hh, R)], 1).astype(np.int32)
    ij[:50, 0] = 0
    ij[50:100, 1] = Hh - 1
    z0 = rng.uniform(-2.0, 8.0, R).astype(F32)
    d = rng.standard_normal((R, 3))
    d[:, 2] = np.abs(d[:, 2]) * rng.choice([-1, 1], R, p=[0.2, 0.8])
    d[:300, 1] = 0.0  # rays along x
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(F32)
    wall, tex = O.box_wall_n(W, Hh, box, ij, z0, d)
    x0, y0 = ij[:, 0].astype(np.float64), ij[:, 1].astype(np.float64)
    dd = d.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = np.where(dd[:, 0] > 0, (W - 1 - x0) / dd[:, 0], np.where(dd[:, 0] < 0, -x0 / dd[:, 0], np.inf))
        ty = np.where(dd[:, 1] > 0, (Hh - 1 - y0) / dd[:, 1], np.where(dd[:, 1] < 0, -y0 / dd[:, 1], np.inf))
    xw = tx <= ty
    t = np.where(xw, tx, ty)
    zw = z0 + t * dd[:, 2]
    ref_wall = np.where(zw < Z, np.where(xw, np.where(dd[:, 0] > 0, 1, 0), np.where(dd[:, 1] > 0, 3, 2)), -1)
    u = np.where(xw, y0 + t * dd[:, 1], x0 + t * dd[:, 0]) / np.where(xw, Hh - 1, W - 1)
    col = np.clip(np.floor(u * tw), 0, tw - 1)
    row = np.clip(np.floor(zw / Z * th), 0, th - 1)
    ref_tex = np.where(ref_wall >= 0, (ref_wall * th + row) * tw + col, -1)
    edge = lambda f: np.abs(f - np.round(f)) < 1e-4
    clear = (np.abs(tx - ty) > 1e-4 * np.maximum(t, 1)) & (np.abs(zw - Z) > 1e-4) & ~edge(u * tw) & \
        ~edge(zw / Z * th)
    assert clear.mean() > 0.95 and (ref_wall[clear] >= 0).mean() > 0.2 and (ref_wall[clear] < 0).mean() > 0.2
    assert np.array_equal(wall[clear], ref_wall[clear])
    assert np.array_equal(tex[clear], ref_tex[clear].astype(np.int32))


def test_box_shade_against_the_opposite_rim():
    """Eq.2 on the walls for lights in the x-z plane at elevation e: the inner
    face of wall 0 (x = 0, facing +x) gets s cos e where the light clears the
    rim of wall 1, i.e. at texel-centre heights z >= Z - (W - 1) tan e, and 0
    below; wall 1 faces away and walls 2, 3 are edge-on (cosine 0)."""
    W, Hh, Z, th, tw = 21, 15, 12.0, 24, 3
    box = _wall_box(Z, th, tw, 1, 1)
    es = np.radians([10.0, 25.0, 40.0, 70.0])
    l = np.stack([np.cos(es), np.zeros(4), np.sin(es)], 1).astype(F32)
    s = np.array([1.0, 0.7, 1.3, 0.9], F32)
    Sw = O.box_shade(W, Hh, box, l, s)
    zc = (np.arange(th) + 0.5) / th * Z
    for k, e in enumerate(es):
        lit = zc >= Z - (W - 1) * math.tan(e)
        away = np.abs(zc - (Z - (W - 1) * math.tan(e))) > 1e-3
        ref = np.where(lit, F32(s[k] * l[k, 0]), 0.0).astype(F32)
        for col in range(tw):
            assert np.array_equal(Sw[0, away, col, k], ref[away]), k
        assert lit.any() or e < 0.6
        assert (Sw[1:, ..., k] == 0).all()


def test_direct_with_walls_against_the_rim():
    """Direct light on a flat floor inside walls of height Z, lights in the x-z
    plane at elevation e towards +x: a sample at column i is lit (S = s sin e)
    when its shadow ray clears the rim of wall 1 before x = W - 1, i.e.
    i + Z / tan e <= W - 1, and dark otherwise (the floor casts no shadow)."""
    W, Hh, Z = 40, 6, 5.0
    Hf = np.zeros((Hh, W), F32)
    n = np.zeros((Hh, W, 3), F32)
    n[..., 2] = 1
    es = np.radians([15.0, 30.0, 55.0])
    l = np.stack([np.cos(es), np.zeros(3), np.sin(es)], 1).astype(F32)
    S = O.direct(Hf, n, l, None, box_z=Z)
    i = np.arange(W)
    for k, e in enumerate(es):
        edge = i + Z / math.tan(e)
        away = np.abs(edge - (W - 1)) > 1e-3
        ref = np.where(edge <= W - 1, F32(l[k, 2]), 0.0).astype(F32)
        for j in range(Hh):
            assert np.array_equal(S[j, away, k], ref[away]), (k, j)
    assert (O.direct(Hf, n, l) > 0).all()  # without walls every sample is lit
