"""Seeded synthetic scenes for IRT-PS (inputs only).

This module makes the ground-truth surfaces, albedos, calibrated lights and
environment maps that both the GPU library and the CPU oracle are fed.  It holds
none of the method's arithmetic: no shading, tracing, photometric-stereo solve
or integration.  Images are rendered from these scenes by the code under test.

The paper evaluates on a synthetic sphere, the Harvard photometric-stereo data
and a face set (Sec. V); none of those is used here.  The scenes stand in for
them with the concavities the paper targets (Sec. I, Sec. IV): a spherical bowl
in a plane, a V-groove with a sinusoid, and fractional-Brownian-motion terrain.

Conventions: sample (i, j) sits at world (x, y) = (i, j) (column i, row j),
heights are in pixel units with z towards an orthographic camera, a light
direction points from the surface towards the light, and environment texels are
radiance on an equirectangular map (row = polar angle from +z, column = azimuth
from +x towards +y).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "normals_from_heights", "ring_lights", "fibonacci_lights",
    "bowl_64", "vgroove_512", "fbm_terrain", "fbm_heights", "batched_job",
    "served_job", "served_arrivals", "tiny_scene", "cornell_walls", "in_box",
]


@dataclass
class Scene:
    name: str
    heights: np.ndarray          # [H][W] float32, ground truth
    normals: np.ndarray          # [H][W][3] float32, ground truth
    albedo: np.ndarray           # [C][H][W] float32, ground truth
    light_dirs: np.ndarray       # [K][3] float32
    light_intensity: np.ndarray  # [K] float32
    env: np.ndarray              # [He][We][C] float32 radiance
    spp: int = 16                # solve samples per pixel
    bounces: int = 1             # solve segments per path
    iterations: int = 3          # IRT iterations T
    seed: int = 0                # solve Philox key
    render_spp: int = 1024
    render_bounces: int = 1
    extra: dict = field(default_factory=dict)
    # walls around the surface: {"Z": height, "albedo": [4][th][tw][C]}, or None
    box: dict | None = None

    @property
    def width(self) -> int:
        return int(self.heights.shape[1])

    @property
    def height(self) -> int:
        return int(self.heights.shape[0])

    @property
    def channels(self) -> int:
        return int(self.albedo.shape[0])

    @property
    def num_lights(self) -> int:
        return int(self.light_dirs.shape[0])


def normals_from_heights(h: np.ndarray) -> np.ndarray:
    """Shading normals of a sampled surface: (-dH/dx, -dH/dy, 1) normalised, with
    central differences inside and one-sided differences on the border."""
    h = np.asarray(h, dtype=np.float64)
    gy, gx = np.gradient(h)  # axis 0 = rows (y), axis 1 = columns (x)
    n = np.stack([-gx, -gy, np.ones_like(h)], axis=-1)
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    return n.astype(np.float32)


def ring_lights(elev_deg, azim_deg) -> np.ndarray:
    e = np.radians(np.asarray(elev_deg, dtype=np.float64))
    a = np.radians(np.asarray(azim_deg, dtype=np.float64))
    l = np.stack([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)], axis=-1)
    return l.astype(np.float32)


def fibonacci_lights(k: int) -> np.ndarray:
    """K directions on the upper hemisphere: z_k = (k + 1/2)/K, azimuth k times
    the golden angle pi (3 - sqrt 5)."""
    idx = np.arange(k, dtype=np.float64)
    z = (idx + 0.5) / k
    phi = idx * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(1.0 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=-1).astype(np.float32)


def _scene(name, h, albedo, lights, intens, env, **kw) -> Scene:
    h = np.ascontiguousarray(h, dtype=np.float32)
    return Scene(
        name=name, heights=h, normals=normals_from_heights(h),
        albedo=np.ascontiguousarray(albedo, dtype=np.float32),
        light_dirs=np.ascontiguousarray(lights, dtype=np.float32),
        light_intensity=np.ascontiguousarray(intens, dtype=np.float32),
        env=np.ascontiguousarray(env, dtype=np.float32), **kw)


def bowl_heights(w: int, hgt: int, rim: float, depth: float) -> np.ndarray:
    """Spherical bowl of rim radius `rim` and depth `depth`, centred, in a flat
    plane at height 0."""
    R = (rim * rim + depth * depth) / (2.0 * depth)
    yy, xx = np.mgrid[0:hgt, 0:w].astype(np.float64)
    r2 = (xx - (w - 1) / 2.0) ** 2 + (yy - (hgt - 1) / 2.0) ** 2
    inside = r2 < rim * rim
    h = np.zeros((hgt, w))
    h[inside] = (R - depth) - np.sqrt(R * R - r2[inside])
    return h


def bowl_64() -> Scene:
    """64x64 spherical bowl (depth 16, rim radius 24) in a plane, albedo 0.8,
    grey; 8 unit lights at 45 deg elevation, azimuth k*45 deg; uniform
    environment radiance 0.2.  Solve: 16 spp, 1 bounce, 3 iterations, seed 0;
    input images rendered with 1024 spp and 1 bounce."""
    w = 64
    h = bowl_heights(w, w, rim=24.0, depth=16.0)
    lights = ring_lights([45.0] * 8, [45.0 * k for k in range(8)])
    return _scene("bowl64", h, np.full((1, w, w), 0.8), lights, np.ones(8),
                  np.full((2, 4, 1), 0.2), spp=16, bounces=1, iterations=3, seed=0,
                  render_spp=1024, render_bounces=1)


def vgroove_heights(w: int, hgt: int, depth: float, amp: float, period: float) -> np.ndarray:
    yy, xx = np.mgrid[0:hgt, 0:w].astype(np.float64)
    x0 = (w - 1) / 2.0
    groove = -np.maximum(0.0, depth - math.sqrt(3.0) * np.abs(xx - x0))
    return groove + amp * np.sin(2 * math.pi * xx / period) * np.sin(2 * math.pi * yy / period)


def vgroove_512(seed: int = 0, size: int = 512) -> Scene:
    """512x512 V-groove along y (walls 60 deg from horizontal, i.e. a 60 deg
    opening, depth 64) plus an 8 px egg-crate sinusoid of period 64; albedo
    i.i.d. U[0.5, 0.9]; 12 lights at elevations U[30, 70] deg, azimuth k*30 deg;
    32x64 environment with i.i.d. U[0, 0.5] radiance.  Solve: 64 spp, 2 bounces,
    5 iterations; images rendered with 256 spp and 2 bounces."""
    rng = np.random.default_rng(seed)
    h = vgroove_heights(size, size, 64.0, 8.0, 64.0)
    albedo = rng.uniform(0.5, 0.9, size=(1, size, size))
    elev = rng.uniform(30.0, 70.0, size=12)
    lights = ring_lights(elev, [30.0 * k for k in range(12)])
    env = rng.uniform(0.0, 0.5, size=(32, 64, 1))
    return _scene("vgroove512", h, albedo, lights, np.ones(12), env, spp=64, bounces=2,
                  iterations=5, seed=seed, render_spp=256, render_bounces=2)


def fbm_heights(size: int, hurst: float, ptp: float, rng: np.random.Generator) -> np.ndarray:
    """Fractional Brownian surface by spectral synthesis: amplitude |f|^-(H+1),
    uniform random phase, no DC term, rescaled to peak-to-peak `ptp` with
    minimum 0."""
    fy = np.fft.fftfreq(size)[:, None]
    fx = np.fft.rfftfreq(size)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    f[0, 0] = 1.0
    amp = f ** (-(hurst + 1.0))
    amp[0, 0] = 0.0
    phase = rng.uniform(0.0, 2.0 * math.pi, size=amp.shape)
    spec = amp * np.exp(1j * phase)
    h = np.fft.irfft2(spec, s=(size, size))
    h -= h.min()
    h *= ptp / h.max()
    return h


def fbm_terrain(seed: int = 0, size: int = 2048, channels: int = 3, num_lights: int = 16,
                env_shape=(256, 512), hurst: float = 0.7, ptp: float = 256.0,
                spp: int = 256, bounces: int = 3, iterations: int = 5,
                render_spp: int = 64, render_bounces: int = 3) -> Scene:
    """RGB fBm terrain (Hurst 0.7, peak-to-peak 256 at 2048^2) with per-channel
    albedo i.i.d. U[0.3, 0.9]; K lights on a hemisphere Fibonacci lattice;
    log-normal (mu=-1, sigma=1) HDR environment.  Solve: 256 spp, 3 bounces,
    5 iterations."""
    rng = np.random.default_rng(seed)
    h = fbm_heights(size, hurst, ptp, rng)
    albedo = rng.uniform(0.3, 0.9, size=(channels, size, size))
    env = np.exp(-1.0 + rng.standard_normal(size=(env_shape[0], env_shape[1], channels)))
    return _scene(f"fbm{size}", h, albedo, fibonacci_lights(num_lights), np.ones(num_lights),
                  env, spp=spp, bounces=bounces, iterations=iterations, seed=seed,
                  render_spp=render_spp, render_bounces=render_bounces)


def step_hill(seed: int = 4, w: int = 48, hgt: int = 40, channels: int = 3, num_lights: int = 12,
              env_shape=(2, 4), env_level: float = 0.0, spp: int = 16, bounces: int = 2,
              iterations: int = 3, render_spp: int = 0, render_bounces: int = 0) -> Scene:
    """A shadow-heavy surface: a floor with a step (a plateau of height 10 from
    column 30 w/48) cut by a narrow trench, and a paraboloid hill of height 4;
    albedo i.i.d. U[0.3, 0.9]; K Fibonacci lights (the lowest 2.4 deg above the
    horizon for K = 12) with intensities spread over [0.8, 1.3]; uniform
    environment `env_level`.  Without indirect light (render_bounces = 0,
    env_level = 0) the images hold attached and cast shadows only."""
    rng = np.random.default_rng(seed)
    f = w / 48.0
    yy, xx = np.mgrid[0:hgt, 0:w].astype(np.float64)
    h = np.where(xx >= 30 * f, 10.0, 0.0)
    r2 = (xx - 14.0 * f) ** 2 + (yy - hgt / 2.0) ** 2
    h = h + np.where(r2 < 64.0 * f * f, 4.0 * (1 - r2 / (64.0 * f * f)), 0.0)
    h = np.where((xx >= 39 * f) & (xx <= 41 * f) & (yy >= 0.15 * hgt) & (yy <= 0.85 * hgt), -12.0, h)
    albedo = rng.uniform(0.3, 0.9, size=(channels, hgt, w))
    intens = np.linspace(0.8, 1.3, num_lights)
    env = np.full((env_shape[0], env_shape[1], channels), env_level)
    return _scene("step_hill", h, albedo, fibonacci_lights(num_lights), intens, env, spp=spp,
                  bounces=bounces, iterations=iterations, seed=0, render_spp=max(render_spp, 1),
                  render_bounces=render_bounces)


def _loguniform_side(rng, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batched_job(j: int, lo: int = 128, hi: int = 1024) -> Scene:
    """Job j of the batched workload: square side log-uniform in [lo, hi]; a
    seeded choice of bowl (depth s/4, rim 0.375 s), V-groove (depth s/8 with an
    s/64 sinusoid of period s/8) or fBm (peak-to-peak s/8); grey; K uniform in
    6..20 ring lights at elevations U[30, 70] deg; albedo and environment as the
    512^2 groove.  Solve: 64 spp, 2 bounces, 4 iterations, Philox key j."""
    rng = np.random.default_rng(1000 + j)
    s = _loguniform_side(rng, lo, hi)
    kind = int(rng.integers(0, 3))
    if kind == 0:
        h = bowl_heights(s, s, rim=0.375 * s, depth=s / 4.0)
    elif kind == 1:
        h = vgroove_heights(s, s, s / 8.0, s / 64.0, s / 8.0)
    else:
        h = fbm_heights(s, 0.7, s / 8.0, rng)
    K = int(rng.integers(6, 21))
    albedo = rng.uniform(0.5, 0.9, size=(1, s, s))
    elev = rng.uniform(30.0, 70.0, size=K)
    lights = ring_lights(elev, [360.0 * k / K for k in range(K)])
    env = rng.uniform(0.0, 0.5, size=(32, 64, 1))
    return _scene(f"job{j}", h, albedo, lights, np.ones(K), env, spp=64, bounces=2,
                  iterations=4, seed=j, render_spp=64, render_bounces=2,
                  extra={"kind": ["bowl", "vgroove", "fbm"][kind]})


def served_job(j: int, lo: int = 256, hi: int = 2048) -> Scene:
    """Job j of the served workload: square side log-uniform in [lo, hi], RGB
    fBm (peak-to-peak s/8), K uniform in 8..16 Fibonacci lights, 128x256
    log-normal environment.  Solve: 128 spp, 2 bounces, 5 iterations, key j."""
    rng = np.random.default_rng(5000 + j)
    s = _loguniform_side(rng, lo, hi)
    K = int(rng.integers(8, 17))
    h = fbm_heights(s, 0.7, s / 8.0, rng)
    albedo = rng.uniform(0.3, 0.9, size=(3, s, s))
    env = np.exp(-1.0 + rng.standard_normal(size=(128, 256, 3)))
    return _scene(f"srv{j}", h, albedo, fibonacci_lights(K), np.ones(K), env, spp=128,
                  bounces=2, iterations=5, seed=j, render_spp=64, render_bounces=2)


def served_arrivals(rate: float = 20.0, duration: float = 60.0, seed: int = 0) -> np.ndarray:
    """Poisson arrival times (seconds) at `rate` jobs/s over `duration` s."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return np.asarray(out)
        out.append(t)


def tiny_scene(w: int = 8, hgt: int = 8, seed: int = 0, channels: int = 1,
               num_lights: int = 4, env_shape=(4, 8), amp: float = 2.0) -> Scene:
    """Small random heightfield for traversal and gather checks."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(-amp, amp, size=(hgt, w))
    albedo = rng.uniform(0.3, 0.9, size=(channels, hgt, w))
    lights = fibonacci_lights(num_lights)
    env = rng.uniform(0.0, 1.0, size=(env_shape[0], env_shape[1], channels))
    return _scene(f"tiny{w}x{hgt}", h, albedo, lights, np.ones(num_lights), env)


def cornell_walls(channels: int = 3, tex=(16, 32), seed: int = 0) -> np.ndarray:
    """Albedo [4][th][tw][C] of a Cornell-like box (Sec. IV stages 0 and 3): wall
    0 (x = 0) red, wall 1 (x = W - 1) green, walls 2 and 3 white, each times a
    seeded texture in [0.85, 1.15] (the paper allows textured walls); grey
    images take the channel mean."""
    base = np.array([[0.63, 0.07, 0.05], [0.12, 0.45, 0.09], [0.73, 0.73, 0.73], [0.73, 0.73, 0.73]])
    th, tw = tex
    rng = np.random.default_rng(seed)
    alb = base[:, None, None, :] * rng.uniform(0.85, 1.15, (4, th, tw, 1))
    if channels == 1:
        alb = alb.mean(axis=-1, keepdims=True)
    return np.ascontiguousarray(alb, dtype=np.float32)


def in_box(sc: Scene, height: float, tex=(16, 32), seed: int = 0) -> Scene:
    """The scene with Cornell-like walls of the given height around it."""
    sc.box = {"Z": float(height), "albedo": cornell_walls(sc.channels, tex, seed)}
    return sc
