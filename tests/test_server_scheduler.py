"""The served mode's scheduler on the CPU (dry run: no kernel is launched and
no buffer is touched; only admission, ordering, cancellation and statistics
are exercised).  The GPU tests check results alone vs in the mix."""
import ctypes as ct
import threading
import time

import numpy as np
import pytest

from paper_1811_02357_amd import irtps


def _submit_dry(srv, side, K=8, C=1, T=3):
    """Submit through the C ABI with placeholder device pointers (never dereferenced)."""
    L = irtps.lib()
    lights = np.ascontiguousarray(np.tile([[0.3, 0.2, 0.93]], (K, 1)), np.float32)
    lights[:, 0] += np.linspace(-0.3, 0.3, K)
    lights[:, 1] += np.sin(np.arange(K))
    lights /= np.linalg.norm(lights, axis=1, keepdims=True)
    lights = lights.astype(np.float32)
    pr = irtps.Problem(side, side, C, K, ct.c_void_p(4096), lights.ctypes.data_as(ct.c_void_p), None,
                       ct.c_void_p(4096), 4, 8)
    pa = irtps.Params(4, 1, T, 0, 0, 0, 0, 0, 0)
    out = irtps.Outputs(ct.c_void_p(4096), ct.c_void_p(4096), ct.c_void_p(4096), None, None)
    jid = ct.c_uint64()
    rc = L.irtps_server_submit(srv.h, ct.byref(pr), ct.byref(pa), ct.byref(out), ct.byref(jid))
    return rc, jid.value


def _footprint(side, K=8, C=1):
    n = ct.c_size_t()
    L = irtps.lib()
    lights = np.zeros((K, 3), np.float32)
    pr = irtps.Problem(side, side, C, K, ct.c_void_p(4096), lights.ctypes.data_as(ct.c_void_p), None,
                       ct.c_void_p(4096), 4, 8)
    pa = irtps.Params(4, 1, 3, 0, 0, 0, 0, 0, 0)
    assert L.irtps_workspace_bytes(ct.byref(pr), ct.byref(pa), ct.byref(n)) == 0
    return n.value


def test_admission_by_footprint_and_fifo():
    job_bytes = _footprint(256)
    table = 4 << 20
    budget = table + 3 * job_bytes + 1000  # room for three resident jobs
    srv = irtps.Server(budget, dry_run=True, table_bytes=table)
    try:
        ids = []
        for _ in range(10):
            rc, jid = _submit_dry(srv, 256)
            assert rc == 0
            ids.append(jid)
        max_res = 0
        while True:
            st = srv.stats()
            max_res = max(max_res, st["resident"])
            assert st["bytes_in_use"] <= st["bytes_budget"]
            if st["completed"] == 10:
                break
            time.sleep(0.001)
        assert max_res <= 3 and max_res >= 2
        starts = [srv.poll(j).start_s for j in ids]
        assert starts == sorted(starts)  # FIFO admission
        for j in ids:
            s = srv.poll(j)
            assert s.state == irtps.JOB_DONE and s.iteration == 3 and s.end_s >= s.start_s >= s.submit_s
        st = srv.stats()
        assert st["p99_latency_s"] >= st["p50_latency_s"] > 0 and st["jobs_per_s"] > 0
        assert st["bytes_in_use"] == 0 and st["resident"] == 0
    finally:
        srv.close()


def test_oversized_job_refused_and_cancel():
    job_bytes = _footprint(128)
    table = 2 << 20
    srv = irtps.Server(table + job_bytes + 256, dry_run=True, table_bytes=table, max_resident_jobs=1)
    try:
        rc, _ = _submit_dry(srv, 512)
        assert rc == 4  # IRTPS_ERR_OOM: can never fit
        rc, a = _submit_dry(srv, 128, T=200)
        rc2, b = _submit_dry(srv, 128, T=2)
        rc3, c = _submit_dry(srv, 128, T=2)
        assert rc == rc2 == rc3 == 0
        srv.cancel(c)  # queued behind a long job: dropped
        srv.cancel(a)  # resident: stops at an iteration boundary
        sb = srv.wait(b, 30.0)
        assert sb.state == irtps.JOB_DONE
        assert srv.wait(a, 30.0).state == irtps.JOB_CANCELLED
        assert srv.wait(c, 30.0).state == irtps.JOB_CANCELLED
        st = srv.stats()
        assert st["cancelled"] == 2 and st["completed"] == 1
    finally:
        srv.close()


def test_concurrent_submitters():
    srv = irtps.Server(256 << 20, dry_run=True)
    ids, lock = [], threading.Lock()

    def worker():
        for _ in range(20):
            rc, jid = _submit_dry(srv, 64, T=1)
            assert rc == 0
            with lock:
                ids.append(jid)

    try:
        th = [threading.Thread(target=worker) for _ in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert len(set(ids)) == 80
        for j in ids:
            assert srv.wait(j, 30.0).state == irtps.JOB_DONE
    finally:
        srv.close()


def test_invalid_server_arguments():
    L = irtps.lib()
    h = ct.c_void_p()
    cfg = irtps.ServerCfg(-1, 1, 0, 0, 0)
    assert L.irtps_server_create(ct.byref(cfg), None, 1 << 20, ct.byref(h)) == 1
    cfg = irtps.ServerCfg(0, 0, 0, 0, 0)
    assert L.irtps_server_create(ct.byref(cfg), None, 1 << 20, ct.byref(h)) == 3  # no workspace
    st = irtps.JobStatus()
    srv = irtps.Server(8 << 20, dry_run=True)
    try:
        assert L.irtps_server_poll(srv.h, 12345, ct.byref(st)) == 7
    finally:
        srv.close()


def test_cancel_of_only_job_wakes_its_waiter():
    """Cancelling every resident job leaves the scheduler idle: the round that
    retires them launches nothing, and it must still wake the jobs' waiters (a
    waiter that re-checked its job between the cancel call and that round would
    otherwise sleep until its time-out).  The window is a few microseconds wide,
    so this exercises the path rather than forcing the race."""
    srv = irtps.Server(256 << 20, dry_run=True)
    try:
        ids = []
        for _ in range(40):
            rc, jid = _submit_dry(srv, 64, T=1000)
            assert rc == 0
            ids.append(jid)
        t0 = time.monotonic()
        while srv.stats()["resident"] < 40:
            assert time.monotonic() - t0 < 20.0
            time.sleep(0.001)
        got = {}

        def waiter():
            t1 = time.monotonic()
            got["st"] = srv.wait(ids[0], 20.0)
            got["s"] = time.monotonic() - t1

        th = threading.Thread(target=waiter)
        th.start()
        time.sleep(0.03)  # the waiter is asleep while the jobs run
        for j in ids:
            srv.cancel(j)
        th.join(30.0)
        assert not th.is_alive()
        assert got["st"].state == irtps.JOB_CANCELLED
        assert got["s"] < 10.0  # woken by the cancellation, not by the time-out
        # the other jobs retire at the scheduler's next rounds, after cancel() returned
        t2 = time.monotonic()
        while srv.stats()["cancelled"] < 40:
            assert time.monotonic() - t2 < 20.0
            time.sleep(0.001)
        assert srv.stats()["cancelled"] == 40
    finally:
        srv.close()


def test_fill_policy_runs_short_jobs_first():
    """With fill_pixels, a round advances the oldest resident job, then those
    with the least remaining work until their pixels reach the target: short
    jobs submitted behind a long one finish long before it, in order of their
    work, and the long (oldest) job still advances every round."""
    srv = irtps.Server(256 << 20, dry_run=True, fill_pixels=2 * 64 * 64)
    try:
        rc, big = _submit_dry(srv, 64, T=400)
        assert rc == 0
        time.sleep(0.005)
        ids = []
        for T_ in (40, 20, 3):
            rc, j = _submit_dry(srv, 64, T=T_)
            assert rc == 0
            ids.append(j)
        sts = [srv.wait(j, 60.0) for j in ids]
        sb = srv.wait(big, 60.0)
        assert sb.state == irtps.JOB_DONE and sb.iteration == 400
        assert all(st.state == irtps.JOB_DONE for st in sts)
        assert [st.iteration for st in sts] == [40, 20, 3]
        # a round holds the big (oldest) job and one more: 3 finishes before 20
        # before 40, all before the big one
        assert sts[2].end_s < sts[1].end_s < sts[0].end_s < sb.end_s
    finally:
        srv.close()
    L = irtps.lib()
    h = ct.c_void_p()
    cfg = irtps.ServerCfg(0, 1, 0, 0, -1)
    assert L.irtps_server_create(ct.byref(cfg), None, 1 << 20, ct.byref(h)) == 1  # negative fill refused
