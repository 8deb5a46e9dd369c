"""Python binding of libirtps (include/irtps.h): argument marshalling only.

Every function here checks shapes, takes device pointers and the current HIP
stream from torch tensors, and calls the C ABI of the same name; all work runs
in the library's HIP kernels.  torch provides device memory and streams only.
If libirtps.so is missing the import of the library fails loudly: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as ct
import functools
import glob
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libirtps.so")

OK = 0
RHO_FIT, RHO_PREV = 0, 1
FLAG_QUADRATURE, FLAG_LITERAL_CUMULATIVE, FLAG_FLAT_TRAVERSAL, FLAG_SHADOW_AWARE_PS = 1, 2, 4, 8
FLAG_GRAPH = 16  # irtps_solve: capture once in a hipGraph, replay on identical calls
FLAG_ROBUST_INTEGRATION = 32  # Huber M-estimator integration (plain solves only)
ROBUST_DELTA, ROBUST_ROUNDS, ROBUST_CYCLES = 0.1, 6, 2  # the loop's robust integration
FLAG_EXACT_R_MASK = 0x700  # the r-ray variant's bits (plain solves only)


def flag_exact_r(r):
    """IRTPS_FLAG_EXACT_R(r): the r-ray environment image (r in 1..7) in place of the gather."""
    return int(r) << 8


TAG_SOLVE, TAG_RENDER = 0, 1
NUM_COUNTERS = 5  # segments, hits, escapes, continuations, IRT iterations run

_vp = ct.c_void_p
_i32 = ct.c_int32
_i64 = ct.c_int64
_u64 = ct.c_uint64
_sz = ct.c_size_t


class IrtpsError(RuntimeError):
    def __init__(self, name, status, lib):
        msg = lib.irtps_status_string(status).decode()
        if status == 5:
            msg += f" (hipError {lib.irtps_last_hip_error()})"
        super().__init__(f"{name}: {msg} [{status}]")
        self.status = status


class BoxC(ct.Structure):
    """irtps_box."""
    _fields_ = [("height", ct.c_float), ("tex_h", _i32), ("tex_w", _i32), ("albedo_dev", _vp)]


class Box:
    """Walls of height `height` on the borders of the sample grid, open above;
    `albedo` a device tensor [4][tex_h][tex_w][C] (walls x = 0, x = W - 1,
    y = 0, y = H - 1; rows from height 0 to `height`, columns along the wall)."""

    def __init__(self, height, albedo):
        if not (isinstance(albedo, torch.Tensor) and albedo.dim() == 4 and albedo.shape[0] == 4):
            raise ValueError("box albedo must be a [4][tex_h][tex_w][C] tensor")
        self.height = float(height)
        self.albedo = albedo

    def c(self, C=None):
        if C is not None and self.albedo.shape[3] != C:
            raise ValueError(f"box albedo has {self.albedo.shape[3]} channels, expected {C}")
        return BoxC(self.height, self.albedo.shape[1], self.albedo.shape[2], _dev(self.albedo, name="box albedo"))


def _boxp(box, C=None):
    """(pointer or None, the struct to keep alive) for an optional Box."""
    if box is None:
        return None, None
    b = box.c(C)
    return ct.byref(b), b


class Problem(ct.Structure):
    _fields_ = [("width", _i32), ("height", _i32), ("channels", _i32), ("num_lights", _i32),
                ("images_dev", _vp), ("light_dirs_host", _vp), ("light_intensity_host", _vp),
                ("env_dev", _vp), ("env_h", _i32), ("env_w", _i32), ("box", ct.POINTER(BoxC))]


class Params(ct.Structure):
    _fields_ = [("spp", _i32), ("bounces", _i32), ("iterations", _i32), ("rho_mode", _i32),
                ("flags", _i32), ("mg_cycles_cold", _i32), ("mg_cycles_warm", _i32),
                ("stop_tol", ct.c_float), ("seed", _u64)]


class Outputs(ct.Structure):
    _fields_ = [("normals_dev", _vp), ("albedo_dev", _vp), ("depth_dev", _vp),
                ("indirect_dev", _vp), ("counters_dev", _vp)]


class Schedule(ct.Structure):
    _fields_ = [("tile_w", _i32), ("ready_batch", _i32)]


TUNE_CANDIDATES = 20


class ServerCfg(ct.Structure):
    _fields_ = [("max_resident_jobs", _i32), ("dry_run", _i32), ("table_bytes", _u64),
                ("reserved", _i32), ("fill_pixels", _i32)]


class JobStatus(ct.Structure):
    _fields_ = [("state", _i32), ("status", _i32), ("iteration", _i32), ("reserved", _i32),
                ("submit_s", ct.c_double), ("start_s", ct.c_double), ("end_s", ct.c_double)]


class ServerStats(ct.Structure):
    _fields_ = [("submitted", _u64), ("completed", _u64), ("failed", _u64), ("cancelled", _u64),
                ("resident", _i32), ("queued", _i32), ("bytes_in_use", _u64), ("bytes_budget", _u64),
                ("iterations", _u64), ("p50_latency_s", ct.c_double), ("p99_latency_s", ct.c_double),
                ("jobs_per_s", ct.c_double)]


JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED, JOB_CANCELLED = range(5)

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(the HIP library is required; there is no fallback)")
        L = ct.CDLL(LIB_PATH)
        L.irtps_status_string.restype = ct.c_char_p
        L.irtps_status_string.argtypes = [ct.c_int]
        L.irtps_abi_version.restype = ct.c_int
        L.irtps_last_hip_error.restype = ct.c_int
        P = ct.POINTER
        sigs = {
            "irtps_ps_matrix": [_i32, _vp, _vp, _vp],
            "irtps_workspace_bytes": [P(Problem), P(Params), P(_sz)],
            "irtps_solve": [P(Problem), P(Params), P(Outputs), _vp, _sz, _vp],
            "irtps_solve_static": [P(Problem), P(Params), P(Outputs), _vp],
            "irtps_ps_solve": [_i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp],
            "irtps_ps_solve_masked": [_i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
            "irtps_probe_valu": [_i32, _i32, _i32, _i32, _vp, _vp],
            "irtps_integrate_workspace_bytes": [_i32, _i32, P(_sz)],
            "irtps_integrate": [_i32, _i32, _vp, _vp, _i32, _vp, _vp, _sz, _vp],
            "irtps_integrate_robust": [_i32, _i32, _vp, _vp, _i32, ct.c_float, _i32, _i32, _vp, _vp, _sz, _vp],
            "irtps_pyramid_bytes": [_i32, _i32, P(_sz)],
            "irtps_build_pyramid": [_i32, _i32, _vp, _vp, _vp],
            "irtps_direct": [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, P(BoxC), _vp],
            "irtps_box_shade": [_i32, _i32, _i32, P(BoxC), _vp, _vp, _vp, _vp],
            "irtps_trace": [_i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _vp,
                            _i32, _i32, _u64, _i32, _i32, _i32, _vp, _vp, P(BoxC), _vp, _vp],
            "irtps_correct": [_i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                              _vp, _vp],
            "irtps_trace_exact_r": [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _i32, _vp, _i32, _u64,
                                    _i32, _i32, _i32, _vp, _vp, _vp],
            "irtps_fill_workspace_bytes": [_i32, _i32, _i32, P(_sz)],
            "irtps_fill_missing": [_i32, _i32, _i32, _vp, _vp, _vp, _sz, _vp],
            "irtps_render_workspace_bytes": [_i32, _i32, _i32, _i32, P(BoxC), P(_sz)],
            "irtps_render": [_i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32,
                             _i32, _i32, _u64, _vp, _vp, _sz, P(BoxC), _vp],
            "irtps_batch_workspace_bytes": [_i32, _vp, _vp, P(_sz)],
            "irtps_batch_solve": [_i32, _vp, _vp, _vp, _i32, _vp, _sz, _vp],
            "irtps_set_ready_batch": [_i32],
            "irtps_set_schedule": [_i32, _i32],
            "irtps_get_schedule": [_i32] * 5 + [P(Schedule)],
            "irtps_autotune": [P(Problem), P(Params), P(Outputs), _vp, _sz, _vp, P(Schedule), P(ct.c_float)],
            "irtps_tuning_save": [ct.c_char_p],
            "irtps_tuning_load": [ct.c_char_p, P(_i32)],
            "irtps_server_create": [P(ServerCfg), _vp, _sz, P(_vp)],
            "irtps_server_submit": [_vp, P(Problem), P(Params), P(Outputs), P(_u64)],
            "irtps_server_poll": [_vp, _u64, P(JobStatus)],
            "irtps_server_wait": [_vp, _u64, ct.c_double, P(JobStatus)],
            "irtps_server_cancel": [_vp, _u64],
            "irtps_server_stats": [_vp, P(ServerStats)],
            "irtps_server_destroy": [_vp],
            "irtps_get_ready_batch": [],
            "irtps_profile_begin": [],
            "irtps_profile_end": [P(ct.c_double), P(_i64)],
            "irtps_probe_philox": [_i64, _vp, _u64, _vp, _vp],
            "irtps_probe_sample": [_i64, _vp, _vp, _vp, _vp],
            "irtps_probe_env_texel": [_i64, _vp, _i32, _i32, _vp, _vp],
            "irtps_probe_traverse": [_i32, _i32, _vp, _vp, _i32, _i64, _vp, _vp, _vp, _vp],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ct.c_int
        _LIB = L
        load_shipped_tuning()
    return _LIB


def _check(name, status):
    if status != OK:
        raise IrtpsError(name, status, lib())


def _dev(t, dtype=torch.float32, shape=None, name="tensor"):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ct.c_void_p(t.data_ptr())


def _host_f32(a, shape=None, name="array"):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None and arr.shape != tuple(shape):
        raise ValueError(f"{name} has shape {arr.shape}, expected {tuple(shape)}")
    return arr, arr.ctypes.data_as(ct.c_void_p)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _alloc_ws(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _on_stream(fn):
    """Run a call with an explicit `stream` as if that stream were current, so
    that the workspace and outputs it allocates belong to the stream its kernels
    run on (the caching allocator then never hands them out while they run)."""
    @functools.wraps(fn)
    def call(*args, stream=None, **kw):
        if stream is None:
            return fn(*args, **kw)
        with torch.cuda.stream(stream):
            return fn(*args, **kw)
    return call


# ---------------------------------------------------------------------------
def ps_matrix(light_dirs, light_intensity=None):
    """Eq.4 solve matrix M = (L^T L)^-1 L^T, [3][K] (host computation)."""
    l, lp = _host_f32(light_dirs, name="light_dirs")
    K = l.shape[0]
    s, sp = _host_f32(light_intensity, (K,), "light_intensity")
    M = np.zeros((3, K), np.float32)
    _check("irtps_ps_matrix", lib().irtps_ps_matrix(K, lp, sp, M.ctypes.data_as(ct.c_void_p)))
    return M


def _problem(images, light_dirs, light_intensity, env, box=None):
    K, C, H, W = images.shape
    l, lp = _host_f32(light_dirs, (K, 3), "light_dirs")
    s, sp = _host_f32(light_intensity, (K,), "light_intensity")
    if env.dim() != 3 or env.shape[2] != C:
        raise ValueError("env must be [He][We][C]")
    bc = box.c(C) if box is not None else None
    pr = Problem(W, H, C, K, _dev(images, name="images"), lp, sp, _dev(env, name="env"),
                 env.shape[0], env.shape[1], ct.pointer(bc) if bc is not None else None)
    return pr, (l, s, bc)


@_on_stream
def solve(images, light_dirs, light_intensity, env, spp, bounces, iterations, seed=0,
          rho_mode=RHO_FIT, flags=0, mg_cycles_cold=0, mg_cycles_warm=0, out=None,
          workspace=None, stream=None, stop_tol=0.0, box=None):
    """The whole IRT-PS loop.  images [K][C][H][W], env [He][We][C] on the device.
    stop_tol > 0 ends the loop after the first iteration that moves the surface
    by less than stop_tol (pixel units) everywhere.
    box: a Box (walls around the surface) or None.
    Returns a dict of device tensors: normals, albedo, depth, indirect, counters."""
    K, C, H, W = images.shape
    dev = images.device
    pr, keep = _problem(images, light_dirs, light_intensity, env, box)
    pa = Params(spp, bounces, iterations, rho_mode, flags, mg_cycles_cold, mg_cycles_warm, float(stop_tol), seed)
    if out is None:
        out = {"normals": torch.empty((H, W, 3), device=dev),
               "albedo": torch.empty((C, H, W), device=dev),
               "depth": torch.empty((H, W), device=dev),
               "indirect": torch.empty((K, C, H, W), device=dev),
               "counters": torch.empty(NUM_COUNTERS, dtype=torch.int64, device=dev)}  # zeroed by the solve
    o = Outputs(_dev(out["normals"], shape=(H, W, 3), name="normals"),
                _dev(out["albedo"], shape=(C, H, W), name="albedo"),
                _dev(out["depth"], shape=(H, W), name="depth"),
                _dev(out.get("indirect"), shape=(K, C, H, W), name="indirect"),
                _dev(out.get("counters"), dtype=torch.int64, shape=(NUM_COUNTERS,), name="counters"))
    need = workspace_bytes(images, light_dirs, light_intensity, env, spp, bounces, iterations,
                           seed, rho_mode, flags, box=box)
    if workspace is None:
        workspace = _alloc_ws(need, dev)
    _check("irtps_solve", lib().irtps_solve(ct.byref(pr), ct.byref(pa), ct.byref(o),
                                            ct.c_void_p(workspace.data_ptr()),
                                            workspace.numel(), _stream(stream)))
    return out


STATIC_SCRATCH_BYTES = 64 << 20  # IRTPS_STATIC_SCRATCH_BYTES


@_on_stream
def solve_static(images, light_dirs, light_intensity, env, spp, bounces, iterations, seed=0,
                 rho_mode=RHO_FIT, flags=0, mg_cycles_cold=0, mg_cycles_warm=0, out=None, stream=None,
                 stop_tol=0.0, box=None):
    """solve() with the workspace in the library's own device scratch (no
    allocation by the library; the outputs are allocated here unless `out` is
    given).  Problems needing more than STATIC_SCRATCH_BYTES are refused."""
    K, C, H, W = images.shape
    dev = images.device
    pr, keep = _problem(images, light_dirs, light_intensity, env, box)
    pa = Params(spp, bounces, iterations, rho_mode, flags, mg_cycles_cold, mg_cycles_warm, float(stop_tol), seed)
    if out is None:
        out = {"normals": torch.empty((H, W, 3), device=dev),
               "albedo": torch.empty((C, H, W), device=dev),
               "depth": torch.empty((H, W), device=dev),
               "indirect": torch.empty((K, C, H, W), device=dev),
               "counters": torch.empty(NUM_COUNTERS, dtype=torch.int64, device=dev)}
    o = Outputs(_dev(out["normals"], shape=(H, W, 3), name="normals"),
                _dev(out["albedo"], shape=(C, H, W), name="albedo"),
                _dev(out["depth"], shape=(H, W), name="depth"),
                _dev(out.get("indirect"), shape=(K, C, H, W), name="indirect"),
                _dev(out.get("counters"), dtype=torch.int64, shape=(NUM_COUNTERS,), name="counters"))
    _check("irtps_solve_static", lib().irtps_solve_static(ct.byref(pr), ct.byref(pa), ct.byref(o), _stream(stream)))
    return out


def workspace_bytes(images, light_dirs, light_intensity, env, spp, bounces, iterations, seed=0,
                    rho_mode=RHO_FIT, flags=0, stop_tol=0.0, box=None):
    pr, keep = _problem(images, light_dirs, light_intensity, env, box)
    pa = Params(spp, bounces, iterations, rho_mode, flags, 0, 0, float(stop_tol), seed)
    n = _sz()
    _check("irtps_workspace_bytes", lib().irtps_workspace_bytes(ct.byref(pr), ct.byref(pa), ct.byref(n)))
    return n.value


@_on_stream
def ps_solve(A, light_dirs, light_intensity=None, stream=None):
    K, C, H, W = A.shape
    l, lp = _host_f32(light_dirs, (K, 3), "light_dirs")
    s, sp = _host_f32(light_intensity, (K,), "light_intensity")
    n = torch.empty((H, W, 3), device=A.device)
    rho = torch.empty((C, H, W), device=A.device)
    _check("irtps_ps_solve", lib().irtps_ps_solve(W, H, C, K, lp, sp, _dev(A, name="A"),
                                                  _dev(n), _dev(rho), _stream(stream)))
    return n, rho


@_on_stream
def ps_solve_masked(A, S, light_dirs, light_intensity=None, stream=None):
    """Eq.4 per pixel over the lights with S[p][k] > 0 (at least three), else
    all lights.  A [K][C][H][W], S [H][W][K] (irtps_direct)."""
    K, C, H, W = A.shape
    l, lp = _host_f32(light_dirs, (K, 3), "light_dirs")
    s, sp = _host_f32(light_intensity, (K,), "light_intensity")
    n = torch.empty((H, W, 3), device=A.device)
    rho = torch.empty((C, H, W), device=A.device)
    _check("irtps_ps_solve_masked", lib().irtps_ps_solve_masked(
        W, H, C, K, lp, sp, _dev(A, name="A"), _dev(S, shape=(H, W, K), name="S"), _dev(n), _dev(rho),
        _stream(stream)))
    return n, rho


@_on_stream
def integrate(normals, depth_init=None, cycles=8, stream=None):
    H, W = normals.shape[:2]
    nb = _sz()
    _check("irtps_integrate_workspace_bytes", lib().irtps_integrate_workspace_bytes(W, H, ct.byref(nb)))
    ws = _alloc_ws(nb.value, normals.device)
    depth = torch.empty((H, W), device=normals.device)
    _check("irtps_integrate", lib().irtps_integrate(
        W, H, _dev(normals, shape=(H, W, 3), name="normals"),
        _dev(depth_init, shape=(H, W), name="depth_init"), cycles, _dev(depth),
        ct.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    return depth


@_on_stream
def integrate_robust(normals, depth_init=None, cycles=8, delta=ROBUST_DELTA, rounds=ROBUST_ROUNDS,
                     rcycles=ROBUST_CYCLES, stream=None):
    H, W = normals.shape[:2]
    nb = _sz()
    _check("irtps_integrate_workspace_bytes", lib().irtps_integrate_workspace_bytes(W, H, ct.byref(nb)))
    ws = _alloc_ws(nb.value, normals.device)
    depth = torch.empty((H, W), device=normals.device)
    _check("irtps_integrate_robust", lib().irtps_integrate_robust(
        W, H, _dev(normals, shape=(H, W, 3), name="normals"),
        _dev(depth_init, shape=(H, W), name="depth_init"), cycles, float(delta), rounds, rcycles, _dev(depth),
        ct.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    return depth


@_on_stream
def build_pyramid(depth, stream=None):
    H, W = depth.shape
    nb = _sz()
    _check("irtps_pyramid_bytes", lib().irtps_pyramid_bytes(W, H, ct.byref(nb)))
    pyr = torch.empty(nb.value // 4, device=depth.device)
    _check("irtps_build_pyramid", lib().irtps_build_pyramid(W, H, _dev(depth, name="depth"),
                                                            _dev(pyr), _stream(stream)))
    return pyr


@_on_stream
def direct(depth, normals, light_dirs, light_intensity=None, pyramid=None, stream=None, box=None):
    """S [H][W][K]; with a Box its walls block shadow rays too."""
    H, W = depth.shape
    l, lp = _host_f32(light_dirs, name="light_dirs")
    K = l.shape[0]
    s, sp = _host_f32(light_intensity, (K,), "light_intensity")
    if pyramid is None:
        pyramid = build_pyramid(depth, stream)
    S = torch.empty((H, W, K), device=depth.device)
    bp, bkeep = _boxp(box)
    _check("irtps_direct", lib().irtps_direct(W, H, K, _dev(depth), _dev(normals, shape=(H, W, 3)),
                                              lp, sp, _dev(pyramid), _dev(S), bp, _stream(stream)))
    return S


@_on_stream
def box_shade(W, H, box, light_dirs, light_intensity=None, stream=None):
    """The walls' direct irradiance [4][tex_h][tex_w][K] at texel centres."""
    l, lp = _host_f32(light_dirs, name="light_dirs")
    K = l.shape[0]
    s, sp = _host_f32(light_intensity, (K,), "light_intensity")
    Sw = torch.empty((4, box.albedo.shape[1], box.albedo.shape[2], K), device=box.albedo.device)
    bp, bkeep = _boxp(box)
    _check("irtps_box_shade", lib().irtps_box_shade(W, H, K, bp, lp, sp, _dev(Sw), _stream(stream)))
    return Sw


@_on_stream
def trace(depth, normals, albedo, S, env, spp, bounces, seed=0, t=0, tag=TAG_SOLVE, flags=0,
          pyramid=None, counters=None, stream=None, box=None, wall_S=None):
    """Gathered radiance G, pixel-major [H][W][K][C]; with a Box, wall_S from box_shade."""
    H, W = depth.shape
    C = albedo.shape[0]
    K = S.shape[2]
    if pyramid is None:
        pyramid = build_pyramid(depth, stream)
    G = torch.empty((H, W, K, C), device=depth.device)
    bp, bkeep = _boxp(box, C)
    if box is not None and wall_S is None:
        raise ValueError("a box needs wall_S (box_shade)")
    _check("irtps_trace", lib().irtps_trace(
        W, H, C, K, _dev(depth), _dev(normals, shape=(H, W, 3)), _dev(albedo, shape=(C, H, W)),
        _dev(S, shape=(H, W, K)), _dev(env), env.shape[0], env.shape[1], _dev(pyramid),
        spp, bounces, seed, t, tag, flags, _dev(G),
        _dev(counters, dtype=torch.int64, shape=(NUM_COUNTERS,)), bp, _dev(wall_S, name="wall_S"),
        _stream(stream)))
    return G


@_on_stream
def trace_exact_r(depth, normals, albedo, env, r, seed=0, t=0, tag=TAG_SOLVE, flags=0, pyramid=None,
                  stream=None):
    """The r-ray environment image E [H][W][C] and its valid mask [H][W] (uint8)."""
    H, W = depth.shape
    C = albedo.shape[0]
    if pyramid is None:
        pyramid = build_pyramid(depth, stream)
    E = torch.empty((H, W, C), device=depth.device)
    valid = torch.empty((H, W), dtype=torch.uint8, device=depth.device)
    _check("irtps_trace_exact_r", lib().irtps_trace_exact_r(
        W, H, C, _dev(depth), _dev(normals, shape=(H, W, 3)), _dev(albedo, shape=(C, H, W)), _dev(env),
        env.shape[0], env.shape[1], _dev(pyramid), int(r), seed, t, tag, flags, _dev(E),
        _dev(valid, dtype=torch.uint8), _stream(stream)))
    return E, valid


@_on_stream
def fill_missing(E, valid, stream=None):
    """Pull-push fill of E [H][W][C] where valid [H][W] (uint8) is 0 (returns a new tensor)."""
    H, W, C = E.shape
    out = E.clone()
    nb = _sz()
    _check("irtps_fill_workspace_bytes", lib().irtps_fill_workspace_bytes(W, H, C, ct.byref(nb)))
    ws = _alloc_ws(nb.value, E.device)
    _check("irtps_fill_missing", lib().irtps_fill_missing(
        W, H, C, _dev(out), _dev(valid, dtype=torch.uint8, shape=(H, W), name="valid"),
        ct.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    return out


@_on_stream
def correct(I0, G, S, albedo, rho_mode=RHO_FIT, flags=0, A_prev=None, want_E=True, stream=None):
    """Stage 5: I0, A_prev [K][C][H][W]; G [H][W][K][C] (as irtps_trace returns it)."""
    K, C, H, W = I0.shape
    E = torch.empty_like(I0) if want_E else None
    A = torch.empty_like(I0)
    _check("irtps_correct", lib().irtps_correct(
        W, H, C, K, rho_mode, flags, _dev(I0), _dev(A_prev), _dev(G, shape=(H, W, K, C)),
        _dev(S, shape=(H, W, K)), _dev(albedo, shape=(C, H, W)), _dev(E), _dev(A), _stream(stream)))
    return E, A


@_on_stream
def render(depth, normals, albedo, light_dirs, light_intensity, env, spp, bounces, seed=0,
           stream=None, box=None):
    H, W = depth.shape
    C = albedo.shape[0]
    l, lp = _host_f32(light_dirs, name="light_dirs")
    K = l.shape[0]
    s, sp = _host_f32(light_intensity, (K,), "light_intensity")
    bp, bkeep = _boxp(box, C)
    nb = _sz()
    _check("irtps_render_workspace_bytes", lib().irtps_render_workspace_bytes(W, H, C, K, bp, ct.byref(nb)))
    ws = _alloc_ws(nb.value, depth.device)
    I = torch.empty((K, C, H, W), device=depth.device)
    _check("irtps_render", lib().irtps_render(
        W, H, C, K, _dev(depth), _dev(normals, shape=(H, W, 3)), _dev(albedo, shape=(C, H, W)),
        lp, sp, _dev(env), env.shape[0], env.shape[1], spp, bounces, seed, _dev(I),
        ct.c_void_p(ws.data_ptr()), ws.numel(), bp, _stream(stream)))
    return I


BATCH_GRAPH = 1


def _outputs_for(images, dev):
    K, C, H, W = images.shape
    return {"normals": torch.empty((H, W, 3), device=dev),
            "albedo": torch.empty((C, H, W), device=dev),
            "depth": torch.empty((H, W), device=dev),
            "indirect": torch.empty((K, C, H, W), device=dev),
            # the batched and served solves zero the counters themselves; no fill
            # kernel here, so a submit does not wait behind running work
            "counters": torch.empty(NUM_COUNTERS, dtype=torch.int64, device=dev)}


def _batch_structs(jobs, outs):
    n = len(jobs)
    probs = (Problem * n)()
    pars = (Params * n)()
    o = (Outputs * n)()
    keep = []
    for j, job in enumerate(jobs):
        pr, k = _problem(job["images"], job["light_dirs"], job.get("light_intensity"), job["env"], job.get("box"))
        keep.append(k)
        probs[j] = pr
        pars[j] = Params(job["spp"], job["bounces"], job["iterations"], job.get("rho_mode", RHO_FIT),
                         job.get("flags", 0), job.get("mg_cycles_cold", 0), job.get("mg_cycles_warm", 0),
                         float(job.get("stop_tol", 0.0)), job.get("seed", 0))
        if outs is not None:
            K, C, H, W = job["images"].shape
            out = outs[j]
            o[j] = Outputs(_dev(out["normals"], shape=(H, W, 3)), _dev(out["albedo"], shape=(C, H, W)),
                           _dev(out["depth"], shape=(H, W)),
                           _dev(out.get("indirect"), shape=(K, C, H, W)),
                           _dev(out.get("counters"), dtype=torch.int64, shape=(NUM_COUNTERS,)))
    return probs, pars, o, keep


def batch_workspace_bytes(jobs):
    probs, pars, _, keep = _batch_structs(jobs, None)
    nb = _sz()
    _check("irtps_batch_workspace_bytes", lib().irtps_batch_workspace_bytes(
        len(jobs), ct.cast(probs, ct.c_void_p), ct.cast(pars, ct.c_void_p), ct.byref(nb)))
    return nb.value


@_on_stream
def batch_solve(jobs, graph=False, outs=None, workspace=None, stream=None):
    """Many reconstructions in one set of launches.  `jobs` is a list of dicts
    with the arguments of solve() (images, light_dirs, light_intensity, env,
    spp, bounces, iterations, seed, rho_mode, flags); returns a list of output
    dicts like solve()."""
    dev = jobs[0]["images"].device
    if outs is None:
        outs = [_outputs_for(job["images"], dev) for job in jobs]
    probs, pars, o, keep = _batch_structs(jobs, outs)
    if workspace is None:
        workspace = _alloc_ws(batch_workspace_bytes(jobs), dev)
    _check("irtps_batch_solve", lib().irtps_batch_solve(
        len(jobs), ct.cast(probs, ct.c_void_p), ct.cast(pars, ct.c_void_p), ct.cast(o, ct.c_void_p),
        BATCH_GRAPH if graph else 0, ct.c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream)))
    return outs


class Server:
    """Continuous-batching server over a device memory budget (irtps_server_*).
    submit() takes the arguments of solve() as a dict and returns a job id; the
    job's output tensors are returned by outputs(id) and are valid once wait(id)
    reports JOB_DONE.  dry_run=True schedules without launching kernels."""

    def __init__(self, budget_bytes, device=None, max_resident_jobs=0, dry_run=False, table_bytes=0,
                 fill_pixels=0):
        self.device = device
        self.ws = None
        ptr = None
        if not dry_run:
            self.ws = torch.empty(int(budget_bytes), dtype=torch.uint8, device=device)
            ptr = ct.c_void_p(self.ws.data_ptr())
        cfg = ServerCfg(max_resident_jobs, 1 if dry_run else 0, table_bytes, 0, int(fill_pixels))
        h = ct.c_void_p()
        _check("irtps_server_create", lib().irtps_server_create(ct.byref(cfg), ptr, int(budget_bytes), ct.byref(h)))
        self.h = h
        self._jobs = {}

    def submit(self, job, outs=None):
        dev = job["images"].device
        if outs is None:
            outs = _outputs_for(job["images"], dev)
        probs, pars, o, keep = _batch_structs([job], [outs])
        # the server runs on a stream of its own: inputs and fresh outputs must be settled
        torch.cuda.current_stream(dev).synchronize()
        jid = _u64()
        _check("irtps_server_submit", lib().irtps_server_submit(self.h, ct.byref(probs[0]), ct.byref(pars[0]),
                                                                ct.byref(o[0]), ct.byref(jid)))
        self._jobs[jid.value] = (job, outs)  # keeps the device buffers alive
        return jid.value

    def poll(self, jid):
        st = JobStatus()
        _check("irtps_server_poll", lib().irtps_server_poll(self.h, jid, ct.byref(st)))
        return st

    def wait(self, jid, timeout_s=-1.0):
        st = JobStatus()
        rc = lib().irtps_server_wait(self.h, jid, timeout_s, ct.byref(st))
        if rc not in (OK, 8):
            _check("irtps_server_wait", rc)
        return st

    def cancel(self, jid):
        _check("irtps_server_cancel", lib().irtps_server_cancel(self.h, jid))

    def outputs(self, jid):
        return self._jobs[jid][1]

    def stats(self):
        st = ServerStats()
        _check("irtps_server_stats", lib().irtps_server_stats(self.h, ct.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.h:
            _check("irtps_server_destroy", lib().irtps_server_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_ready_batch(lanes):
    """Force the tracer's rays-per-wave batch (0: tuning table / default)."""
    _check("irtps_set_ready_batch", lib().irtps_set_ready_batch(lanes))


def get_ready_batch():
    return lib().irtps_get_ready_batch()


def set_schedule(tile_w=0, ready_batch=0):
    """Force the tracer's tile width and/or rays-per-wave batch (0: automatic)."""
    _check("irtps_set_schedule", lib().irtps_set_schedule(tile_w, ready_batch))


def get_schedule(W, H, C, K, B):
    sc = Schedule()
    _check("irtps_get_schedule", lib().irtps_get_schedule(W, H, C, K, B, ct.byref(sc)))
    return {"tile_w": sc.tile_w, "ready_batch": sc.ready_batch}


@_on_stream
def autotune(job, outs=None, workspace=None, stream=None):
    """Time the tracer's schedules on this job (arguments of solve()); the fastest
    enters the process's tuning table.  Returns (best, {(tile_w, ready_batch): ms})."""
    dev = job["images"].device
    if outs is None:
        outs = _outputs_for(job["images"], dev)
    probs, pars, o, keep = _batch_structs([job], [outs])
    if workspace is None:
        workspace = _alloc_ws(workspace_bytes(**job), dev)
    best = Schedule()
    ms = (ct.c_float * TUNE_CANDIDATES)()
    _check("irtps_autotune", lib().irtps_autotune(ct.byref(probs[0]), ct.byref(pars[0]), ct.byref(o[0]),
                                                  ct.c_void_p(workspace.data_ptr()), workspace.numel(),
                                                  _stream(stream), ct.byref(best), ms))
    cands = [(tw, rb) for tw in (8, 16, 32, 64) for rb in (24, 32, 40, 48, 56)]
    return {"tile_w": best.tile_w, "ready_batch": best.ready_batch}, dict(zip(cands, list(ms)))


def tuning_save(path):
    _check("irtps_tuning_save", lib().irtps_tuning_save(str(path).encode()))


def tuning_load(path):
    n = _i32()
    _check("irtps_tuning_load", lib().irtps_tuning_load(str(path).encode(), ct.byref(n)))
    return n.value


def load_shipped_tuning():
    """Merge the tuning tables shipped next to the library; only the one written
    on this device's architecture loads.  Returns the entries loaded."""
    total = 0
    for f in sorted(glob.glob(os.path.join(os.path.dirname(LIB_PATH), "tuning_*.json"))):
        n = _i32()
        if lib().irtps_tuning_load(f.encode(), ct.byref(n)) == OK:
            total += n.value
    return total


def tuning_clear():
    _check("irtps_tuning_clear", lib().irtps_tuning_clear())


def tuning_entries():
    return lib().irtps_tuning_entries()


def profile_begin():
    _check("irtps_profile_begin", lib().irtps_profile_begin())


def profile_end():
    """(summed tracer milliseconds, tracer launches) since profile_begin()."""
    ms, n = ct.c_double(), _i64()
    _check("irtps_profile_end", lib().irtps_profile_end(ct.byref(ms), ct.byref(n)))
    return ms.value, n.value


# ---- probes ----------------------------------------------------------------
def probe_valu(blocks, iters, active_lanes=64, kind=0, stream=None):
    """Launch the VALU issue-rate probe once (kind 0: integer shift/xor-add, 1:
    register moves, 2: fp32 fma); returns its output buffer."""
    out = torch.empty(blocks * 256, dtype=torch.int32, device=torch.device("cuda"))
    _check("irtps_probe_valu", lib().irtps_probe_valu(blocks, iters, active_lanes, kind,
                                                      _dev(out, dtype=torch.int32), _stream(stream)))
    return out


def probe_philox(ctr, seed):
    out = torch.empty_like(ctr)
    _check("irtps_probe_philox", lib().irtps_probe_philox(ctr.shape[0], _dev(ctr, dtype=torch.int32),
                                                          seed, _dev(out, dtype=torch.int32), _stream()))
    return out


def probe_sample(normals, u):
    d = torch.empty((u.shape[0], 3), device=u.device)
    _check("irtps_probe_sample", lib().irtps_probe_sample(u.shape[0], _dev(normals), _dev(u), _dev(d), _stream()))
    return d


def probe_env_texel(d, He, We):
    rc = torch.empty((d.shape[0], 2), dtype=torch.int32, device=d.device)
    _check("irtps_probe_env_texel", lib().irtps_probe_env_texel(d.shape[0], _dev(d), He, We,
                                                                _dev(rc, dtype=torch.int32), _stream()))
    return rc


def probe_traverse(depth, ij, d, flat, pyramid=None):
    H, W = depth.shape
    if pyramid is None:
        pyramid = build_pyramid(depth)
    q = torch.empty_like(ij)
    _check("irtps_probe_traverse", lib().irtps_probe_traverse(
        W, H, _dev(depth), _dev(pyramid), 1 if flat else 0, ij.shape[0],
        _dev(ij, dtype=torch.int32), _dev(d), _dev(q, dtype=torch.int32), _stream()))
    return q
