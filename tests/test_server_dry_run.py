"""Server scheduling on the CPU (dry-run mode: no device work).

A dry-run server completes every batch after the planner's time estimate,
so admission by footprint and slots, queueing order, rejection and latency
accounting are exercised without a GPU.  Matrix pointers are placeholders
that are never dereferenced in this mode.
"""

import ctypes
import time

import pytest

mmp = pytest.importorskip("paper_2601_07508_amd")

P = 1125899906842597


def job(m, n, k, base, p=P, u=0, v=0):
    j = mmp.MmpJob()
    j.p, j.u, j.v, j.m, j.n, j.k = p, u, v, m, n, k
    j.A, j.lda = base, k
    j.B, j.ldb = base + 8 * m * k + 4096, n
    j.C, j.ldc = base + 8 * (m * k + k * n) + 8192, n
    return j


def footprint(m, n, k, **kw):
    return mmp.footprint(P, m, n, k, **kw)


def test_admission_respects_budget_and_slots():
    m = n = k = 1024
    fp = footprint(m, n, k)
    with mmp.Server(hbm_budget=2 * fp + fp // 2, max_slots=8, dry_run=True) as srv:
        tickets = [srv.submit_raw(job(m, n, k, 0x10000000 * (i + 1))) for i in range(6)]
        peak_running = 0
        done = {}
        t0 = time.time()
        while len(done) < len(tickets) and time.time() - t0 < 30:
            st = srv.stats()
            peak_running = max(peak_running, st["running"])
            assert st["used_bytes"] <= 2 * fp + fp // 2
            for t in tickets:
                if t not in done:
                    r = srv.poll(t)
                    if r is not None:
                        done[t] = r
            time.sleep(1e-4)
        assert len(done) == 6 and all(s == 0 for s, _ in done.values())
        # the polls may miss every running batch on a loaded host; the
        # server's own high-water mark sees each launch
        assert peak_running <= 2
        st = srv.stats()
        assert 1 <= st["max_running"] <= 2
        assert st["submitted"] == 6 and st["completed"] == 6 and st["rejected"] == 0
        assert st["peak_used_bytes"] <= 2 * fp + fp // 2
        # FIFO: later tickets cannot finish much earlier than earlier ones
        lat = [done[t][1] for t in tickets]
        assert lat[-1] >= lat[0]


def test_slot_limit():
    m, n, k = 64, 64, 64
    with mmp.Server(hbm_budget=1 << 40, max_slots=1, dry_run=True) as srv:
        tickets = [srv.submit_raw(job(m, n, k, 0x10000000 * (i + 1))) for i in range(5)]
        for t in tickets:
            st, lat = srv.wait(t, 10.0)
            assert st == 0 and lat >= 0
        assert srv.stats()["max_batch"] == 1


def test_rejections():
    m = n = k = 2048
    fp = footprint(m, n, k)
    with mmp.Server(hbm_budget=fp, max_slots=4, dry_run=True) as srv:
        with pytest.raises(mmp.MmpError) as e:  # can never fit
            srv.submit_raw(job(4096, 4096, 4096, 0x10000000))
        assert e.value.status == -4
        t1 = srv.submit_raw(job(m, n, k, 0x20000000))
        with pytest.raises(mmp.MmpError) as e:  # full right now
            srv.submit_raw(job(m, n, k, 0x40000000), noqueue=True)
        assert e.value.status == -6
        srv.wait(t1, 30.0)
        assert srv.stats()["rejected"] == 2


def test_wait_timeout_and_forgotten_ticket():
    # a large product whose planner estimate is far above the timeout
    with mmp.Server(hbm_budget=1 << 44, max_slots=2, dry_run=True) as srv:
        t = srv.submit_raw(job(16384, 16384, 65536, 0x100000000, u=2, v=2))
        with pytest.raises(mmp.MmpError) as e:
            srv.wait(t, 0.01)
        assert e.value.status == -8
        small = srv.submit_raw(job(8, 8, 8, 0x2000000000))
        # the big one is still running: the small one waits behind nothing (2 slots)
        st, lat = srv.wait(small, 5.0)
        assert st == 0
        with pytest.raises(mmp.MmpError) as e:
            srv.poll(small)
        assert e.value.status == -7


def test_invalid_submissions():
    with mmp.Server(hbm_budget=1 << 30, max_slots=2, dry_run=True) as srv:
        with pytest.raises(mmp.MmpError) as e:
            srv.submit_raw(job(8, 8, 8, 0x1000, p=3))
        assert e.value.status == -1
        with pytest.raises(mmp.MmpError) as e:
            srv.submit_raw(job(8, 8, 8, 0x1000, p=2147483647, u=1, v=1))
        assert e.value.status == -2
    lib = mmp.lib()
    h = ctypes.c_void_p()
    assert lib.mmp_server_create(ctypes.byref(h), 0, 0, 4, 1) == -1
    assert lib.mmp_server_create(ctypes.byref(h), 0, 1 << 20, 0, 1) == -1
    assert lib.mmp_server_create(ctypes.byref(h), 0, 1 << 20, 4, 8) == -1


def test_failed_launch_wakes_waiters():
    # every launch fails on the host (testing flag): the request completes
    # with MMP_ENOMEM and a wait without a time limit returns
    import threading
    with mmp.Server(hbm_budget=1 << 30, max_slots=4, dry_run=True, fail_launches=True) as srv:
        t = srv.submit_raw(job(64, 64, 64, 0x10000000))
        out = {}
        th = threading.Thread(target=lambda: out.update(r=srv.wait(t, -1.0)), daemon=True)
        th.start()
        th.join(10.0)
        assert not th.is_alive(), "mmp_wait(-1) did not return after a failed launch"
        assert out["r"][0] == -4
        st = srv.stats()
        assert st["failed"] == 1 and st["used_bytes"] == 0 and st["running"] == 0
        # the server keeps serving: later requests fail the same way, promptly
        t2 = srv.submit_raw(job(8, 8, 8, 0x20000000))
        assert srv.wait(t2, 5.0)[0] == -4


@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 5, 3), (33, 70, 65), (100, 1, 130), (5, 300, 63)])
def test_footprint_covers_the_digit_planes(shape):
    # the admitted footprint is at least what an INT8-form launch allocates
    # (planes with rows rounded up to 16 and k to 64), for every digit count
    m, n, k = shape
    for p in (251, 65521, 16777213, 2147483647, 1099511627689, 281474976710597, 4503599627370449):
        pl = mmp.plan(p, m, n, k, form=mmp.FORM_INT8_WORDS, splits=1)
        fp = mmp.footprint(p, m, n, k, form=mmp.FORM_INT8_WORDS, splits=1)
        assert fp - 8 * (m * k + k * n + m * n) >= pl["workspace_bytes"], (p, shape)
