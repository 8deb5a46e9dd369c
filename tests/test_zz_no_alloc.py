"""The solve entry point that allocates nothing (irtps_solve_static): its
workspace is the library's own device scratch.  Called through the C ABI, its
outputs must equal irtps_solve's bit for bit, on two calls in a row (the second
with a smaller problem, so the scratch holds the first call's contents), and a
problem larger than the scratch must be refused."""
import ctypes as ct

import numpy as np
import pytest
import torch

from paper_1811_02357_amd import irtps, scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _inputs(sc, dev):
    """Input images rendered on the GPU from the scene's ground truth."""
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    I0 = irtps.render(T(sc.heights), T(sc.normals), T(sc.albedo), sc.light_dirs, sc.light_intensity,
                      T(sc.env), sc.render_spp, sc.render_bounces, seed=7)
    return I0, T(sc.env)


def _both(sc, dev, flags=0):
    I0, env = _inputs(sc, dev)
    args = (I0, sc.light_dirs, sc.light_intensity, env, sc.spp, sc.bounces, sc.iterations)
    ws = irtps.workspace_bytes(*args, seed=sc.seed, flags=flags)
    assert ws <= irtps.STATIC_SCRATCH_BYTES, ws
    ref = irtps.solve(*args, seed=sc.seed, flags=flags)
    got = irtps.solve_static(*args, seed=sc.seed, flags=flags)
    torch.cuda.synchronize()
    for k in ("normals", "albedo", "depth", "indirect", "counters"):
        a, b = ref[k].cpu().numpy(), got[k].cpu().numpy()
        assert np.array_equal(a, b), (sc.name, k, np.abs(a.astype(np.float64) - b).max())
    return ws


def test_static_solve_equals_solve_twice(dev):
    # first the 512 x 512 groove (most of the scratch), then a smaller bowl: the
    # scratch then holds the groove's contents when the bowl starts
    print("case: irtps_solve_static vs irtps_solve, vgroove 512^2 then bowl 64^2", flush=True)
    big = scenes.vgroove_512()
    big.render_spp, big.render_bounces = 16, 2
    w1 = _both(big, dev)
    small = scenes.bowl_64()
    small.render_spp = 64
    w2 = _both(small, dev, flags=irtps.FLAG_SHADOW_AWARE_PS)
    assert w2 < w1


def test_static_solve_refuses_oversized_problem(dev):
    print("case: irtps_solve_static refuses a problem larger than its scratch", flush=True)
    L = irtps.lib()
    K, C, side = 16, 3, 1024
    lights = scenes.fibonacci_lights(K)
    img = torch.zeros((K, C, side, side), device=dev)
    env = torch.zeros((4, 8, C), device=dev)
    pr = irtps.Problem(side, side, C, K, ct.c_void_p(img.data_ptr()), lights.ctypes.data_as(ct.c_void_p), None,
                       ct.c_void_p(env.data_ptr()), 4, 8)
    pa = irtps.Params(4, 1, 1, 0, 0, 0, 0, 0.0, 0)
    need = ct.c_size_t()
    assert L.irtps_workspace_bytes(ct.byref(pr), ct.byref(pa), ct.byref(need)) == 0
    assert need.value > irtps.STATIC_SCRATCH_BYTES
    n = torch.empty((side, side, 3), device=dev)
    a = torch.empty((C, side, side), device=dev)
    d = torch.empty((side, side), device=dev)
    o = irtps.Outputs(ct.c_void_p(n.data_ptr()), ct.c_void_p(a.data_ptr()), ct.c_void_p(d.data_ptr()), None, None)
    assert L.irtps_solve_static(ct.byref(pr), ct.byref(pa), ct.byref(o), None) == 3  # IRTPS_ERR_WORKSPACE
