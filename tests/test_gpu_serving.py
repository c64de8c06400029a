"""GPU tests of the serving loop: oracle parity for mixed requests, results
bit-identical alone and in a mix, device-drawn inputs, grouped launches."""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srv_env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_02104_amd as P
    from paper_1902_02104_amd.serving import Server
    P.load()
    return torch, P, Server


SHAPES = [(1024, 64), (1500, 100), (2048, 200), (700, 300), (1200, 513), (3000, 640), (1100, 90), (900, 33)]


def test_mixed_requests_match_oracle(srv_env, orc):
    torch, P, Server = srv_env
    print("case: serving parity", flush=True)
    with Server(2 << 30, max_active=16, streams=4) as s:
        jobs = []
        for i, (m, n) in enumerate(SHAPES):
            for dt in (P.F64, P.F32):
                A = synthetic.integer(m, n, 500 + i, dtype=np.float64 if dt == P.F64 else np.float32)
                jobs.append((s.submit(m, n, dtype=dt, a=A, cutoff=128), A))
        for t, A in jobs:
            C = s.take(t)
            assert np.array_equal(C.astype(np.float64), orc.classical(A.astype(np.float64)))
        st = s.stats()
        assert st["completed"] == len(jobs) and st["batched_requests"] >= 1 and st["pool_in_use"] == 0


def test_alone_and_in_mix_are_bit_identical(srv_env):
    torch, P, Server = srv_env
    print("case: alone vs mix", flush=True)
    probe = [(1024, 64, 1), (2000, 300, 2), (1300, 700, 3), (4096, 128, 4)]
    with Server(4 << 30, max_active=32, streams=4) as s:
        alone = {}
        for m, n, seed in probe:
            t = s.submit(m, n, dtype=P.F32, seed=seed)
            alone[seed] = s.take(t)
        rng = np.random.default_rng(9)
        tickets = {}
        for k in range(30):
            m = int(rng.integers(1024, 5000))
            n = int(rng.integers(64, 800))
            tickets[("noise", k)] = s.submit(m, n, dtype=P.F32, seed=100 + k)
            if k % 7 == 0:
                m0, n0, sd = probe[(k // 7) % len(probe)]
                tickets[("probe", sd, k)] = s.submit(m0, n0, dtype=P.F32, seed=sd)
        for key, t in tickets.items():
            if key[0] == "probe":
                assert np.array_equal(s.take(t), alone[key[1]]), key
            else:
                s.wait(t)
                s.release(t)


def test_device_drawn_input(srv_env, orc):
    torch, P, Server = srv_env
    print("case: device-drawn input", flush=True)
    with Server(1 << 30, max_active=4, streams=2) as s:
        t = s.submit(3000, 257, dtype=P.F32, seed=1234, keep_a=True)
        C, A = s.take(t, want_a=True)
        assert abs(float(A.mean())) < 0.01 and abs(float(A.std()) - 1.0) < 0.01
        ref = orc.classical(A.astype(np.float64))
        assert orc.rel_fro(C.astype(np.float64), ref, 257) < 2e-6
        t2 = s.submit(3000, 257, dtype=P.F32, seed=1234, keep_a=True)
        C2, A2 = s.take(t2, want_a=True)
        assert np.array_equal(A, A2) and np.array_equal(C, C2)


def test_timestamps_and_rejection(srv_env):
    torch, P, Server = srv_env
    print("case: timestamps", flush=True)
    with Server(64 << 20, max_active=8, streams=2) as s:
        ts = [s.submit(1024, 64 * (i + 1), dtype=P.F32, seed=i) for i in range(6)]
        for t in ts:
            inf = s.wait(t)
            assert inf["t_submit"] <= inf["t_admit"] <= inf["t_launch"] <= inf["t_done"]
            s.release(t)
        with pytest.raises(P.AtaError):
            s.submit(65536, 4096, dtype=P.F32)  # 1 GiB of A > 64 MiB budget


def test_chunked_request_exact_and_identical_in_mix(srv_env, orc):
    """A request above the chunking threshold runs in row slabs whose Grams
    add up to C (the row split of the block equations): exact on integer
    input, and bit-identical alone and among other requests."""
    torch, P, Server = srv_env
    print("case: chunked request", flush=True)
    m, n = 40000, 1100  # 4.8e10 flops: three slabs of 16640, 16640 and 6720 rows
    A = synthetic.integer(m, n, 610)
    with Server(8 << 30, max_active=16, streams=4) as s:
        t = s.submit(m, n, dtype=P.F64, a=A)
        info = s.wait(t)
        assert info["slabs"] == 3
        C = s.take(t)
        assert np.array_equal(C, orc.classical_mt(A, threads=8))
        # FP32 device-drawn: alone, then among smaller requests
        t = s.submit(m, n, dtype=P.F32, seed=611)
        alone = s.take(t)
        rng = np.random.default_rng(12)
        noise = [s.submit(int(rng.integers(1024, 8000)), int(rng.integers(64, 900)), dtype=P.F32, seed=700 + k)
                 for k in range(12)]
        t = s.submit(m, n, dtype=P.F32, seed=611)
        noise += [s.submit(int(rng.integers(1024, 8000)), int(rng.integers(64, 900)), dtype=P.F32, seed=720 + k)
                  for k in range(12)]
        assert np.array_equal(s.take(t), alone)
        for k in noise:
            s.wait(k)
            s.release(k)
        assert s.stats()["pool_in_use"] == 0


def test_split_last_round_requests(srv_env, orc):
    """Requests whose plan is one SYRK of 528 tiles (n = 4000) run their last
    16 tiles K-split in a launch of their own: also where the request would
    otherwise join a grouped launch, and in every row slab of a chunked
    request (which accumulates into C).  Exact on integer input in both
    precisions, with the default and an explicit depth."""
    torch, P, Server = srv_env
    print("case: serving split last round", flush=True)
    n = 4000
    A1 = synthetic.integer(1000, n, 801)
    A2 = synthetic.integer(9000, n, 802)
    ref1 = orc.classical(A1)
    ref2 = orc.classical_mt(A2, threads=8)
    with Server(8 << 30, max_active=16, streams=4) as s:
        jobs = []
        for dt in (P.F64, P.F32):
            want = np.float64 if dt == P.F64 else np.float32
            for d in (None, 0):
                jobs.append((s.submit(1000, n, dtype=dt, a=A1.astype(want), max_depth=d), ref1, 1, dt, d))
                jobs.append((s.submit(9000, n, dtype=dt, a=A2.astype(want), max_depth=d), ref2, 3, dt, d))
        for t, ref, slabs, dt, d in jobs:
            assert s.wait(t)["slabs"] == slabs, (dt, d)
            assert np.array_equal(s.take(t).astype(np.float64), ref), (dt, d, slabs)
        assert s.stats()["pool_in_use"] == 0
