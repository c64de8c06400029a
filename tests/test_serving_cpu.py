"""Scheduler tests of the serving loop in its host-only simulate mode (no
GPU): admission by memory footprint, slot limits, rejection, bounded bypass,
empty requests, shutdown with queued work."""
import time

import pytest

import paper_1902_02104_amd as P
from paper_1902_02104_amd.serving import Server


def _foot(m, n, dtype=P.F32):
    eb = 8 if dtype == P.F64 else 4
    up = lambda x: (x + 255) // 256 * 256
    ws = P.workspace_bytes(m, n, 0, dtype=dtype)
    return up(m * n * eb) + up(n * (n + 1) // 2 * eb) + up(ws)


def test_requests_complete_and_account_memory():
    budget = 64 << 20
    with Server(budget, max_active=4, streams=2, simulate_tflops=1e-3) as s:
        tickets = [s.submit(1024, 64 + 16 * i) for i in range(12)]
        infos = [s.wait(t, timeout=30) for t in tickets]
        st = s.stats()
        assert st["completed"] == 12 and st["rejected"] == 0
        assert st["pool_peak"] <= budget
        for inf in infos:
            assert inf["t_submit"] <= inf["t_admit"] <= inf["t_launch"] <= inf["t_done"]
            assert inf["flops"] == inf["m"] * inf["n"] ** 2
        # at most max_active requests overlap in time
        ev = sorted([(i["t_admit"], 1) for i in infos] + [(i["t_done"], -1) for i in infos])
        cur = peak = 0
        for _, d in ev:
            cur += d
            peak = max(peak, cur)
        assert peak <= 4
        for t in tickets:
            s.release(t)
        assert s.stats()["pool_in_use"] == 0


def test_reject_oversized():
    with Server(8 << 20, simulate_tflops=1.0) as s:
        with pytest.raises(P.AtaError) as ei:
            s.submit(4096, 1024)  # 16 MB of A alone
        assert ei.value.status == 5
        assert s.stats()["rejected"] == 1


def test_admission_waits_for_memory():
    big = _foot(2048, 512)
    budget = big + big // 2  # room for one big request at a time
    with Server(budget, max_active=8, simulate_tflops=1e-3) as s:
        t1 = s.submit(2048, 512)
        t2 = s.submit(2048, 512)
        i1 = s.wait(t1, timeout=30)
        s.release(t1)
        i2 = s.wait(t2, timeout=30)
        assert i2["t_admit"] >= i1["t_done"] - 1e-3  # the second waited for the first's memory
        s.release(t2)


def test_small_requests_bypass_a_blocked_head():
    big = _foot(2048, 512)
    small = _foot(1024, 64)
    budget = big + 4 * small
    with Server(budget, max_active=8, simulate_tflops=2e-4) as s:
        t_run = s.submit(2048, 512)      # occupies most of the pool
        t_block = s.submit(2048, 512)    # cannot fit until the first is released
        smalls = [s.submit(1024, 64) for _ in range(3)]
        for t in smalls:
            inf = s.wait(t, timeout=30)
            s.release(t)
        _, ib = s.query(t_block)
        assert ib["state"] != 3  # still waiting: the small ones went ahead
        s.wait(t_run, timeout=30)
        s.release(t_run)
        s.wait(t_block, timeout=30)
        s.release(t_block)


def test_empty_request_and_bad_fields():
    with Server(1 << 20, simulate_tflops=1.0) as s:
        t = s.submit(0, 10)
        inf = s.wait(t, timeout=5)
        assert inf["state"] == 3
        with pytest.raises(P.AtaError):
            s.submit(10, 0)
        with pytest.raises(P.AtaError):
            s.submit(10, 10, dtype=P.F32_FP8)


def test_close_with_queued_work():
    s = Server(1 << 26, max_active=1, simulate_tflops=1e-4)
    for _ in range(5):
        s.submit(1024, 256)
    time.sleep(0.01)
    s.close()  # returns: in-flight work finishes, queued requests are dropped


def test_failed_request_is_released():
    """A request that ended with an error gives its memory back when it is
    released (the error status is reported by that call)."""
    fail_seed = 0xFFFFFFFFFFFFFFFF  # ATA_SERVER_SIM_FAIL_SEED
    with Server(64 << 20, max_active=4, simulate_tflops=1e-3) as s:
        ok = s.submit(1024, 64)
        bad = s.submit(1024, 128, seed=fail_seed)
        with pytest.raises(P.AtaError) as ei:
            s.wait(bad, timeout=30)
        assert ei.value.status == 2  # ATA_EHIP
        assert s.stats()["pool_in_use"] > 0
        with pytest.raises(P.AtaError) as ei:
            s.release(bad)
        assert ei.value.status == 2
        with pytest.raises(P.AtaError) as ei:
            s.release(bad)
        assert ei.value.status == 7  # ATA_ENOTFOUND: already released
        s.wait(ok, timeout=30)
        s.release(ok)
        assert s.stats()["pool_in_use"] == 0
