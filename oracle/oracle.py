"""ctypes front end of the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark call this module; the product path never does.  Arrays are numpy,
float32, C-contiguous, in the layouts documented in irtps_oracle.h.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

TAG_SOLVE, TAG_RENDER = 0, 1
RHO_FIT, RHO_PREV = 0, 1
FLAG_QUADRATURE, FLAG_LITERAL_CUMULATIVE, FLAG_SHADOW_AWARE_PS, FLAG_ROBUST_INTEGRATION = 1, 2, 8, 32
ROBUST_DELTA, ROBUST_ROUNDS, ROBUST_CYCLES = 0.1, 6, 2

_f = ct.POINTER(ct.c_float)
_u32 = ct.POINTER(ct.c_uint32)
_i = ct.POINTER(ct.c_int)


class Counters(ct.Structure):
    _fields_ = [("v", ct.c_uint64 * 5)]

    def as_dict(self):
        return {"segments": self.v[0], "hits": self.v[1], "escapes": self.v[2],
                "continuations": self.v[3], "iterations": self.v[4]}


class OrBox(ct.Structure):
    _fields_ = [("Z", ct.c_float), ("th", ct.c_int), ("tw", ct.c_int), ("albedo", ct.c_void_p),
                ("S", ct.c_void_p)]


def _box(box, keep):
    """A box dict {"Z", "albedo" [4][th][tw][C], optional "S" [4][th][tw][K]} as an
    or_box (arrays kept alive in `keep`), or None."""
    if box is None:
        return None
    alb = _f32(box["albedo"])
    assert alb.ndim == 4 and alb.shape[0] == 4
    Sw = _f32(box.get("S"))
    keep += [alb, Sw]
    b = OrBox(float(box["Z"]), alb.shape[1], alb.shape[2], alb.ctypes.data,
              None if Sw is None else Sw.ctypes.data)
    return ct.byref(b), b


def lib():
    global _LIB
    if _LIB is None:
        path = os.environ.get("IRTPS_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            raise RuntimeError("oracle/liboracle.so is not built: run oracle/build.py")
        L = ct.CDLL(path)
        L.or_philox4x32_10.argtypes = [_u32, _u32, _u32]
        L.or_sin_quarter.argtypes = [ct.c_float]
        L.or_sin_quarter.restype = ct.c_float
        L.or_cos_quarter.argtypes = [ct.c_float]
        L.or_cos_quarter.restype = ct.c_float
        L.or_atan2.argtypes = [ct.c_float, ct.c_float]
        L.or_atan2.restype = ct.c_float
        L.or_sample_cosine.argtypes = [_f, ct.c_float, ct.c_float, _f]
        L.or_env_texel.argtypes = [_f, ct.c_int, ct.c_int, _i, _i]
        L.or_traverse.argtypes = [_f, ct.c_int, ct.c_int, ct.c_float, ct.c_int, ct.c_int, _f, _i, _i]
        L.or_traverse.restype = ct.c_int
        L.or_ps_matrix.argtypes = [ct.c_int, _f, _f, _f]
        L.or_ps_matrix.restype = ct.c_int
        L.or_ps_solve.argtypes = [ct.c_int] * 4 + [_f, _f, _f, _f]
        L.or_direct.argtypes = [ct.c_int] * 3 + [_f, _f, _f, _f, _f]
        L.or_ps_solve_masked.argtypes = [ct.c_int] * 4 + [_f] * 6
        L.or_ps_solve_masked.restype = ct.c_int
        L.or_trace.argtypes = ([ct.c_int] * 4 + [_f] * 5 + [ct.c_int] * 4 + [ct.c_uint64]
                               + [ct.c_int] * 3 + [_f, ct.POINTER(Counters)])
        L.or_correct.argtypes = [ct.c_int] * 6 + [_f] * 7
        _pll = ct.POINTER(ct.c_longlong)
        L.or_direct_at.argtypes = [ct.c_int] * 3 + [_f] * 4 + [ct.c_longlong, _pll, _f]
        L.or_trace_at.argtypes = ([ct.c_int] * 4 + [_f] * 5 + [ct.c_int] * 4 + [ct.c_uint64]
                                  + [ct.c_int] * 3 + [ct.c_longlong, _pll, _f, ct.POINTER(Counters)])
        L.or_integrate.argtypes = [ct.c_int, ct.c_int, _f, _f, ct.c_int, _f]
        _u8 = ct.POINTER(ct.c_uint8)
        L.or_trace_exact_r.argtypes = ([ct.c_int] * 3 + [_f] * 4 + [ct.c_int] * 3 + [ct.c_uint64]
                                       + [ct.c_int] * 2 + [_f, _u8])
        L.or_fill_missing.argtypes = [ct.c_int] * 3 + [_f, _u8]
        L.or_integrate_robust.argtypes = [ct.c_int, ct.c_int, _f, _f, ct.c_int, ct.c_float, ct.c_int, ct.c_int, _f]
        L.or_render.argtypes = ([ct.c_int] * 4 + [_f] * 6 + [ct.c_int] * 4 + [ct.c_uint64]
                                + [_f, ct.POINTER(Counters)])
        L.or_render.restype = ct.c_int
        L.or_solve.argtypes = ([ct.c_int] * 4 + [_f] * 4 + [ct.c_int] * 5 + [ct.c_uint64]
                               + [ct.c_int] * 4 + [ct.c_float] + [_f] * 4 + [ct.POINTER(Counters)])
        L.or_solve.restype = ct.c_int
        _bp = ct.POINTER(OrBox)
        L.or_direct_box.argtypes = [ct.c_int] * 3 + [_f] * 4 + [ct.c_float, _f]
        L.or_box_shade.argtypes = [ct.c_int] * 3 + [_bp, _f, _f, _f]
        L.or_box_wall_n.argtypes = [ct.c_int, ct.c_int, _bp, ct.c_longlong, _i, _f, _f, _i]
        L.or_trace_box.argtypes = ([ct.c_int] * 4 + [_f] * 5 + [ct.c_int] * 4 + [ct.c_uint64]
                                   + [ct.c_int] * 3 + [_bp, _f, ct.POINTER(Counters)])
        L.or_render_box.argtypes = ([ct.c_int] * 4 + [_f] * 6 + [ct.c_int] * 4 + [ct.c_uint64]
                                    + [_bp, _f, ct.POINTER(Counters)])
        L.or_render_box.restype = ct.c_int
        L.or_solve_box.argtypes = ([ct.c_int] * 4 + [_f] * 4 + [ct.c_int] * 5 + [ct.c_uint64]
                                   + [ct.c_int] * 4 + [ct.c_float, _bp] + [_f] * 4 + [ct.POINTER(Counters)])
        L.or_solve_box.restype = ct.c_int
        L.or_num_threads.restype = ct.c_int
        _ll = ct.c_longlong
        L.or_sincos_quarter_n.argtypes = [_ll, _f, _f, _f]
        L.or_atan2_n.argtypes = [_ll, _f, _f, _f]
        L.or_traverse_n.argtypes = [_f, ct.c_int, ct.c_int, _ll, _i, _f, _i]
        L.or_sample_cosine_n.argtypes = [_ll, _f, _f, _f]
        L.or_env_texel_n.argtypes = [_ll, _f, ct.c_int, ct.c_int, _i]
        L.or_philox_n.argtypes = [_ll, _u32, _u32, _u32]
        _LIB = L
    return _LIB


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float32 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(_f)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def num_threads() -> int:
    return lib().or_num_threads()


def philox(ctr, key):
    c = (ct.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ct.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ct.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def sin_quarter(f: float) -> float:
    return lib().or_sin_quarter(f)


def cos_quarter(f: float) -> float:
    return lib().or_cos_quarter(f)


def atan2(y: float, x: float) -> float:
    return lib().or_atan2(y, x)


def sample_cosine(n, u1: float, u2: float):
    nn = _f32(n)
    d = np.zeros(3, np.float32)
    lib().or_sample_cosine(_p(nn), u1, u2, _p(d))
    return d


def env_texel(d, He: int, We: int):
    dd = _f32(d)
    r, c = ct.c_int(), ct.c_int()
    lib().or_env_texel(_p(dd), He, We, ct.byref(r), ct.byref(c))
    return r.value, c.value


def traverse(H, i0: int, j0: int, d):
    H = _f32(H)
    Hh, W = H.shape
    dd = _f32(d)
    qi, qj = ct.c_int(-1), ct.c_int(-1)
    hit = lib().or_traverse(_p(H), W, Hh, float(H.max()), i0, j0, _p(dd), ct.byref(qi), ct.byref(qj))
    return (qi.value, qj.value) if hit else None


def _ip(a):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_i)


def sincos_quarter_n(f):
    f = _f32(f)
    s = np.empty_like(f)
    c = np.empty_like(f)
    lib().or_sincos_quarter_n(f.size, _p(f), _p(s), _p(c))
    return s, c


def atan2_n(y, x):
    y, x = _f32(y), _f32(x)
    a = np.empty_like(y)
    lib().or_atan2_n(y.size, _p(y), _p(x), _p(a))
    return a


def traverse_n(H, ij, d):
    """Rays from samples ij[R][2] = (i, j) along d[R][3]; returns q[R][2], -1 on escape."""
    H, d = _f32(H), _f32(d)
    ij = np.ascontiguousarray(ij, dtype=np.int32)
    q = np.empty_like(ij)
    lib().or_traverse_n(_p(H), H.shape[1], H.shape[0], ij.shape[0], _ip(ij), _p(d), _ip(q))
    return q


def sample_cosine_n(n, u):
    n, u = _f32(n), _f32(u)
    d = np.empty((u.shape[0], 3), np.float32)
    lib().or_sample_cosine_n(u.shape[0], _p(n), _p(u), _p(d))
    return d


def env_texel_n(d, He, We):
    d = _f32(d)
    rc = np.empty((d.shape[0], 2), np.int32)
    lib().or_env_texel_n(d.shape[0], _p(d), He, We, _ip(rc))
    return rc


def philox_n(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray([int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF], dtype=np.uint32)
    out = np.empty_like(ctr)
    pu = ct.POINTER(ct.c_uint32)
    lib().or_philox_n(ctr.shape[0], ctr.ctypes.data_as(pu), k.ctypes.data_as(pu), out.ctypes.data_as(pu))
    return out


def ps_matrix(l, s=None):
    l = _f32(l)
    K = l.shape[0]
    M = np.zeros((3, K), np.float32)
    rc = lib().or_ps_matrix(K, _p(l), _p(_f32(s)), _p(M))
    if rc != 0:
        raise ValueError("singular light configuration")
    return M


def ps_solve(M, A):
    """A: [K][C][H][W] -> normals [H][W][3], albedo [C][H][W]."""
    M, A = _f32(M), _f32(A)
    K, C, Hh, W = A.shape
    n = np.zeros((Hh, W, 3), np.float32)
    rho = np.zeros((C, Hh, W), np.float32)
    lib().or_ps_solve(W, Hh, C, K, _p(M), _p(A), _p(n), _p(rho))
    return n, rho


def ps_solve_masked(l, s, A, S):
    """Eq.4 per pixel over the lights with S[p][k] > 0 (at least three), else
    all lights.  A: [K][C][H][W], S: [H][W][K] -> normals, albedo."""
    l, s, A, S = _f32(l), _f32(s), _f32(A), _f32(S)
    K, C, Hh, W = A.shape
    assert S.shape == (Hh, W, K)
    n = np.zeros((Hh, W, 3), np.float32)
    rho = np.zeros((C, Hh, W), np.float32)
    if lib().or_ps_solve_masked(W, Hh, C, K, _p(l), _p(s), _p(A), _p(S), _p(n), _p(rho)) != 0:
        raise ValueError("singular light configuration")
    return n, rho


def direct(H, n, l, s=None, box_z=0.0):
    """S [H][W][K]; with box_z > 0 the walls of that height occlude too."""
    H, n, l = _f32(H), _f32(n), _f32(l)
    Hh, W = H.shape
    K = l.shape[0]
    S = np.zeros((Hh, W, K), np.float32)
    lib().or_direct_box(W, Hh, K, _p(H), _p(n), _p(l), _p(_f32(s)), float(box_z), _p(S))
    return S


def box_shade(W, Hh, box, l, s=None):
    """The walls' direct irradiance [4][th][tw][K] at texel centres."""
    l = _f32(l)
    keep = []
    bp, b = _box(box, keep)
    Sw = np.zeros((4, b.th, b.tw, l.shape[0]), np.float32)
    lib().or_box_shade(W, Hh, l.shape[0], bp, _p(l), _p(_f32(s)), _p(Sw))
    return Sw


def box_wall_n(W, Hh, box, ij, z0, d):
    """Per ray (origin sample ij [R][2], height z0 [R], direction d [R][3]): the
    wall met below Z (-1: through the top) and its texel index."""
    keep = []
    bp, _ = _box(box, keep)
    ij = np.ascontiguousarray(ij, dtype=np.int32)
    z0, d = _f32(z0), _f32(d)
    out = np.zeros((len(ij), 2), np.int32)
    lib().or_box_wall_n(W, Hh, bp, len(ij), ij.ctypes.data_as(_i), _p(z0), _p(d), out.ctypes.data_as(_i))
    return out[:, 0], out[:, 1]


def trace(H, n, rho, S, env, spp, B, seed, t=0, tag=TAG_SOLVE, flags=0, box=None):
    """G [K][C][H][W] and the event counts; box needs "S" (box_shade)."""
    H, n, rho, S, env = map(_f32, (H, n, rho, S, env))
    Hh, W = H.shape
    C = rho.shape[0]
    K = S.shape[2]
    He, We = env.shape[0], env.shape[1]
    assert env.shape[2] == C and C <= 4
    keep = []
    bx = _box(box, keep)
    if bx is not None:
        assert box["S"] is not None and np.shape(box["S"])[3] == K and np.shape(box["albedo"])[3] == C
    G = np.zeros((K, C, Hh, W), np.float32)
    cnt = Counters()
    lib().or_trace_box(W, Hh, C, K, _p(H), _p(n), _p(rho), _p(S), _p(env), He, We, spp, B,
                       int(seed), t, tag, flags, None if bx is None else bx[0], _p(G), ct.byref(cnt))
    return G, cnt.as_dict()


def _pix(pix):
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    return pix, pix.ctypes.data_as(ct.POINTER(ct.c_longlong))


def direct_at(H, n, l, pix, s=None):
    """S rows [len(pix)][K] at pixel indices pix (p = j W + i)."""
    H, n, l = _f32(H), _f32(n), _f32(l)
    Hh, W = H.shape
    K = l.shape[0]
    pix, pp = _pix(pix)
    assert pix.min() >= 0 and pix.max() < W * Hh
    out = np.zeros((pix.size, K), np.float32)
    lib().or_direct_at(W, Hh, K, _p(H), _p(n), _p(l), _p(_f32(s)), pix.size, pp, _p(out))
    return out


def trace_at(H, n, rho, S, env, spp, B, seed, pix, t=0, tag=TAG_SOLVE, flags=0):
    """G at pixel indices pix: [len(pix)][K][C], and those pixels' event counts."""
    H, n, rho, S, env = map(_f32, (H, n, rho, S, env))
    Hh, W = H.shape
    C = rho.shape[0]
    K = S.shape[2]
    He, We = env.shape[0], env.shape[1]
    assert env.shape[2] == C and C <= 4
    pix, pp = _pix(pix)
    assert pix.min() >= 0 and pix.max() < W * Hh
    out = np.zeros((pix.size, K, C), np.float32)
    cnt = Counters()
    lib().or_trace_at(W, Hh, C, K, _p(H), _p(n), _p(rho), _p(S), _p(env), He, We, spp, B,
                      int(seed), t, tag, flags, pix.size, pp, _p(out), ct.byref(cnt))
    return out, cnt.as_dict()


def correct(I0, G, S, rho, rho_mode=RHO_FIT, flags=0, Aprev=None, want_E=True):
    I0, G, S, rho = map(_f32, (I0, G, S, rho))
    K, C, Hh, W = I0.shape
    E = np.zeros_like(I0) if want_E else None
    A = np.zeros_like(I0)
    Aprev = _f32(Aprev) if Aprev is not None else I0
    lib().or_correct(W, Hh, C, K, rho_mode, flags, _p(I0), _p(Aprev), _p(G), _p(S), _p(rho),
                     _p(E), _p(A))
    return E, A


def integrate(n, Hinit=None, cycles=8):
    n = _f32(n)
    Hh, W = n.shape[:2]
    H = np.zeros((Hh, W), np.float32)
    lib().or_integrate(W, Hh, _p(n), _p(_f32(Hinit)), cycles, _p(H))
    return H


def flag_exact_r(r):
    return int(r) << 8


def trace_exact_r(H, n, rho, env, r, seed, t=0, tag=TAG_SOLVE):
    """The r-ray environment image [C][H][W] and its valid mask [H][W] (uint8)."""
    H, n, rho, env = map(_f32, (H, n, rho, env))
    Hh, W = H.shape
    C = rho.shape[0]
    assert env.shape[2] == C
    E = np.zeros((C, Hh, W), np.float32)
    ok = np.zeros((Hh, W), np.uint8)
    lib().or_trace_exact_r(W, Hh, C, _p(H), _p(n), _p(rho), _p(env), env.shape[0], env.shape[1], int(r),
                           int(seed), t, tag, _p(E), ok.ctypes.data_as(ct.POINTER(ct.c_uint8)))
    return E, ok


def fill_missing(E, valid):
    """Pull-push fill of E [C][H][W] where valid [H][W] is 0 (returns a copy)."""
    E = np.array(E, dtype=np.float32, order="C", copy=True)
    ok = np.ascontiguousarray(valid, dtype=np.uint8)
    C, Hh, W = E.shape
    lib().or_fill_missing(W, Hh, C, _p(E), ok.ctypes.data_as(ct.POINTER(ct.c_uint8)))
    return E


def integrate_robust(n, Hinit=None, cycles=8, delta=ROBUST_DELTA, rounds=ROBUST_ROUNDS, rcycles=ROBUST_CYCLES):
    n = _f32(n)
    Hh, W = n.shape[:2]
    H = np.zeros((Hh, W), np.float32)
    lib().or_integrate_robust(W, Hh, _p(n), _p(_f32(Hinit)), cycles, float(delta), rounds, rcycles, _p(H))
    return H


def render(H, n, rho, l, s, env, spp, B, seed=0, box=None):
    H, n, rho, l, s, env = map(_f32, (H, n, rho, l, s, env))
    Hh, W = H.shape
    C = rho.shape[0]
    K = l.shape[0]
    keep = []
    bx = _box(box, keep)
    I0 = np.zeros((K, C, Hh, W), np.float32)
    cnt = Counters()
    lib().or_render_box(W, Hh, C, K, _p(H), _p(n), _p(rho), _p(l), _p(s), _p(env),
                        env.shape[0], env.shape[1], spp, B, int(seed), None if bx is None else bx[0], _p(I0),
                        ct.byref(cnt))
    return I0, cnt.as_dict()


def render_scene(sc):
    return render(sc.heights, sc.normals, sc.albedo, sc.light_dirs, sc.light_intensity,
                  sc.env, sc.render_spp, sc.render_bounces, 0, box=getattr(sc, "box", None))


def solve(I0, l, s, env, spp, B, T, seed=0, rho_mode=RHO_FIT, flags=0,
          cycles_cold=8, cycles_warm=4, stop_tol=0.0, box=None):
    I0, l, s, env = map(_f32, (I0, l, s, env))
    K, C, Hh, W = I0.shape
    n = np.zeros((Hh, W, 3), np.float32)
    rho = np.zeros((C, Hh, W), np.float32)
    H = np.zeros((Hh, W), np.float32)
    E = np.zeros_like(I0)
    cnt = Counters()
    keep = []
    bx = _box(box, keep)
    rc = lib().or_solve_box(W, Hh, C, K, _p(I0), _p(l), _p(s), _p(env), env.shape[0], env.shape[1],
                            spp, B, T, int(seed), rho_mode, flags, cycles_cold, cycles_warm,
                            float(stop_tol), None if bx is None else bx[0], _p(n), _p(rho), _p(H), _p(E),
                            ct.byref(cnt))
    if rc == -2:
        raise ValueError("walls with the r-ray variant")
    if rc != 0:
        raise ValueError("singular light configuration")
    return {"normals": n, "albedo": rho, "depth": H, "indirect": E, "counters": cnt.as_dict()}
