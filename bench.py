"""Benchmark of the ATA product (packed lower C = A^t A) on one MI355X.

Workload: square FP64 A of 10000 x 10000, entries i.i.d. uniform[-1, 1]
(synthetic stand-in for the paper's randomly generated order-10000 matrices),
leaf cutoff tuned over {128, 256, 512}.  A step is one full ATA product with
A and C resident in HBM.  The metric counts m*n^2 flops per product
(effective TFLOP/s); m*n*(n+1) is reported beside it.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
HBM_PEAK_GBS = 8000.0


def _profiled_traffic(kernel: str, n: int, key: str, work_items: int):
    """HBM bytes per launch of `kernel` from its committed counter summary
    (two rocprofv3 --pmc passes scaled by a plain copy), or None when the
    summary was taken on other kernel sources or on another launch (another
    configuration whose plan has a different tile list)."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "%s_%d_traffic.md" % (kernel, n))
    try:
        kv = dict(line.strip().split(": ", 1) for line in open(path) if line.startswith("    ") and ": " in line
                  and not line.strip().startswith("cd "))
        src = open(os.path.join(root, "paper_1902_02104_amd", "csrc", "ata_kernels.hip"), "rb").read()
    except OSError:
        return None
    if kv.get("kernels_source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    if kv.get("n") != str(n) or (kv.get("config") != key and kv.get("work_items") != str(work_items)):
        return None
    return float(kv["traffic_bytes_per_launch"])


def _sweep_configs(args):
    """Configurations of the method the headline is tuned over (see main)."""
    cutoffs = (128, 256, 512) if args.cutoff == 0 else (args.cutoff,)
    levels = (1, 2) if args.max_depth is None else ((args.max_depth,) if args.max_depth > 0 else ())
    forms = ("tiles", "intile", "opsums") if args.form == "tune" else (args.form,)
    out = []

    def add(c, d, f, v):
        key = "c%d_d0" % c if d == 0 else "c%d_d%d_%s%s" % (c, d, f, "_winograd" if v == "winograd" else "")
        out.append({"key": key, "cutoff": c, "levels": d, "form": f if d else "classical", "variant": v})

    for c in cutoffs:
        if args.max_depth in (None, 0):
            add(c, 0, "tiles", "strassen")
        for d in levels:
            for f in forms:
                add(c, d, f, "strassen")
        if args.variant_sweep and 1 in levels:
            for f in ("tiles", "intile"):
                if f in forms:
                    add(c, 1, f, "winograd")
    if args.cutoff == 0 and args.max_depth is None and args.form == "tune":
        out.append({"key": "default", "cutoff": 0, "levels": -1, "form": "default", "variant": "strassen"})
    return out


def _run_cfg(P, A, C, stream, cfg):
    if cfg["form"] == "default":
        P.gram(A, out=C, stream=stream)  # the library's defaults (adaptive depth)
    else:
        P.gram(A, cutoff=cfg["cutoff"], max_depth=cfg["levels"], variant=cfg["variant"], out=C, stream=stream,
               intile=cfg["form"] == "intile", operand_sums=cfg["form"] == "opsums")


def _plan_stats(P, m, n, cfg):
    if cfg["form"] == "default":
        return P.plan_info(m, n)
    return P.plan_info(m, n, cfg["cutoff"], max_depth=cfg["levels"], variant=cfg["variant"],
                       intile=cfg["form"] == "intile", operand_sums=cfg["form"] == "opsums")


def _profiled(P, fn, time_steps, steps):
    """Time `steps` calls with the library's per-launch HIP events on."""
    P.profile_enable(True)
    P.profile_collect()
    ms = time_steps(fn, steps)
    prof = P.profile_collect()
    P.profile_enable(False)
    return ms, prof


def _roofline(kt, st, cfg, steps, n):
    """Roofline record of the dominant kernel kind of a configuration:
    algorithmic flops per launch (2 per multiplication the launch performs,
    from the plan) over its average event-timed launch duration."""
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms, dom_launches = kt[dom]
    avg_ms = dom_ms / dom_launches
    # the mixed FP64 launch runs the product tiles and the classical tiles of
    # a phase together: its algorithmic work is all of their multiplications
    mult_keys = {"strassen": ("strassen_mults",), "gemm": ("gemm_mults",), "syrk": ("syrk_mults",),
                 "tiles": ("strassen_mults", "gemm_mults", "syrk_mults")}.get(dom)
    launches_per_step = dom_launches / steps
    if mult_keys:
        alg_flops = 2.0 * sum(st[k] for k in mult_keys) / launches_per_step
        roof = {"bound": "mfma", "achieved": alg_flops / (avg_ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "algorithmic_flops_per_launch": alg_flops}
    else:
        roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"] if roof["achieved"] else None
    form, levels = cfg["form"], st["max_hasa_depth"]
    two_term = form in ("tiles", "default") and levels == 1 and st["strassen_mults"] > 0
    roof["kernel"] = {"tiles": "k_tile_q_f64" if two_term else "k_tile_f64",
                      "strassen": "k_str_f64" if form == "intile" else "k_gemm_terms_f64",
                      "gemm": "k_tile_f64", "syrk": "k_tile_f64", "combine": "k_combine_f64"}.get(dom, dom)
    roof["traffic"] = _profiled_traffic(roof["kernel"], n, cfg["key"], st["work_items"])
    roof["avg_launch_ms"] = avg_ms
    roof["launches_per_step"] = launches_per_step
    return roof


def _log(msg):
    """Progress of the legs on stderr; stdout carries only the result line."""
    print("[bench %.0fs] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def _host_info():
    """The host's CPU model and core counts, and the share this process may use
    (its affinity mask, capped by OMP_NUM_THREADS when that is set: the GPU
    boxes allot each GPU a fixed share of their cores)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    share = affinity
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit():
        share = min(share, int(omp))
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": affinity,
            "omp_num_threads": int(omp) if omp.isdigit() else None, "threads": max(1, share)}


def _cpu_baseline(A_np, target_s: float):
    """The oracle's threaded classical product on a bounded sample of the
    same workload: the last rows of packed C (all columns j <= i).  Returns
    the baseline record and (first row, packed rows [first row, n))."""
    import oracle
    m, n = A_np.shape
    host = _host_info()
    threads = host["threads"]

    def first_row(entries):
        i0 = n
        while i0 > 0 and oracle.tri(n) - oracle.tri(i0) < entries:
            i0 -= 1
        return i0

    # Time slabs of the last rows, resizing from the last rate until one takes
    # most of the target; the oracle hands whole row tiles to its threads, so
    # small slabs run slower than large ones.
    ent, dt, rows = 4 * threads * n, 0.0, None
    for _ in range(6):
        i0 = first_row(ent)
        t = time.perf_counter()
        rows = oracle.classical_mt(A_np, rows=(i0, n), threads=threads)
        dt = time.perf_counter() - t
        ent = oracle.tri(n) - oracle.tri(i0)
        if dt >= 0.6 * target_s or i0 == 0:
            break
        ent = int(ent * min(16.0, target_s / max(dt, 1e-3)))
    flops = 2.0 * m * ent  # the same per-entry count as m*n^2 for the whole product
    rec = {
        "value": flops / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "packed rows [%d, %d) of the %dx%d product (%d entries, k ascending, no FMA), %.1f s"
                  % (i0, n, n, n, ent, dt),
        "host": host,
    }
    return rec, (i0, rows)


def _full_check(A_np, C_host, cpu_rows):
    """Every entry of the timed output against the oracle's plain definition:
    relative Frobenius error and the largest scaled error
    max |dC_ij| / sqrt(C_ii C_jj).  Rows the CPU-baseline sample did not
    cover are computed here (untimed)."""
    import oracle
    n = A_np.shape[1]
    threads = _host_info()["threads"]
    if cpu_rows is not None and cpu_rows[0] == 0:
        ref = cpu_rows[1]
    else:
        i0 = n if cpu_rows is None else cpu_rows[0]
        head = oracle.classical_mt(A_np, rows=(0, i0), threads=threads)
        ref = head if cpu_rows is None else np.concatenate([head, cpu_rows[1]])
    return {"entries": int(ref.size), "rel_fro": oracle.rel_fro(C_host, ref, n),
            "max_scaled_err": oracle.scaled_err(C_host, ref, n)}


def _square_leg(P, torch, dev, stream, n: int, args):
    """The square workload at another order: the same tuning (classical
    off-diagonal products and one Strassen level, product tiles and in-tile,
    and the library default), the classical SYRK on the same GPU, and the
    fastest output against the oracle entry by entry."""
    import oracle
    import synthetic
    A_np = synthetic.uniform(n, n, synthetic.SEED_SQUARE)
    A = torch.from_numpy(A_np).to(dev)
    C = torch.empty(P.tri(n), dtype=torch.float64, device=dev)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize(dev)
        return e0.elapsed_time(e1) / k

    cfgs = [c for c in _sweep_configs(args) if c["levels"] in (0, 1, -1) and c["variant"] == "strassen"
            and c["form"] != "opsums"]
    sweep = {c["key"]: timed(lambda: _run_cfg(P, A, C, stream, c), 5) for c in cfgs}
    best = min(sweep, key=sweep.get)
    cfg = {c["key"]: c for c in cfgs}[best]
    ms = timed(lambda: _run_cfg(P, A, C, stream, cfg), max(5, args.steps))
    got = C.cpu().numpy()
    # timed before the host oracle runs: an idle GPU starts the next calls at lower clocks
    cms = timed(lambda: P.gram(A, cutoff=n, max_depth=0, out=C, stream=stream), max(5, args.steps))
    ref = oracle.classical_mt(A_np, threads=_host_info()["threads"])
    flops = float(n) ** 3
    out = {"workload": "square FP64 A %dx%d, i.i.d. uniform[-1,1] (seed %d)" % (n, n, synthetic.SEED_SQUARE),
           "tuned": best, "ms": ms, "tflops_mn2": flops / (ms * 1e-3) / 1e12, "tuning_sweep_ms": sweep,
           "classical_ms": cms, "classical_tflops_mn2": flops / (cms * 1e-3) / 1e12,
           "rel_fro": oracle.rel_fro(got, ref, n), "max_scaled_err": oracle.scaled_err(got, ref, n)}
    _log("square %d: %s %.2f ms (classical %.2f ms), relF %.2e" % (n, best, ms, cms, out["rel_fro"]))
    return out


def _precision_forms(P, torch, dev, stream, n: int, steps: int, depths=(0, 1, 2)):
    """The 8192 x 8192 precision workload: FP32, bfloat16-split and e4m3
    leaves on the FP32-rounded uniform input, each timed and checked against
    the FP64 oracle (plain definition) of the same FP32 input."""
    import oracle
    import synthetic
    A32 = synthetic.uniform(n, n, synthetic.SEED_PRECISION, dtype=np.float32)
    At = torch.from_numpy(A32).to(dev)
    t0 = time.perf_counter()
    ref = oracle.classical_mt(A32.astype(np.float64))
    ref_s = time.perf_counter() - t0
    C = torch.empty(P.tri(n), dtype=torch.float64, device=dev)
    flops = float(n) ** 3
    out = {"workload": "square FP32 A %dx%d, uniform[-1,1] generated in FP64 (seed %d), C in FP64"
                       % (n, n, synthetic.SEED_PRECISION),
           "oracle": "FP64 plain definition on the FP32 input, %.1f s on the host" % ref_s}
    # (name, dtype, depths, MFMA products per classical product, MFMA peak TFLOP/s)
    for name, dt, mult, peak in (("fp32", P.F32, 1, 157.3), ("bf16x3", P.F32_BF16X3, 3, 2500.0),
                                 ("fp8_e4m3", P.F32_FP8, 1, 5000.0)):
        best = None
        for d in depths:
            fn = lambda: P.gram(At, dtype=dt | P.OUT_F64, cutoff=256, max_depth=d, out=C, stream=stream)
            fn()
            torch.cuda.synchronize(dev)
            ms = None
            for _ in range(2):  # the faster of two timed passes (the first may still see clocks ramp)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(steps):
                    fn()
                e1.record(stream)
                torch.cuda.synchronize(dev)
                t = e0.elapsed_time(e1) / steps
                ms = t if ms is None else min(ms, t)
            err = oracle.rel_fro(C.cpu().numpy(), ref, n)
            rec = {"ms": ms, "tflops_mn2": flops / (ms * 1e-3) / 1e12, "rel_fro_vs_fp64": err, "depth": d,
                   "cutoff": 256}
            rec["mfma_frac"] = mult * rec["tflops_mn2"] * P.plan_info(n, n, 256, dtype=dt, max_depth=d)["mults"] / \
                (n * P.tri(n)) / peak
            out["%s_d%d" % (name, d)] = rec
            _log("precision %s depth %d: %.2f ms" % (name, d, ms))
            if best is None or ms < best["ms"]:
                best = rec
        out[name] = best
    return out


def _freivalds_device(torch, C, A, n, gen):
    """|| C x - A^t (A x) || / (||A||_F^2 ||x||) for packed C and A on the
    device, in FP64 (torch's own products; A converted in row blocks)."""
    dev = C.device
    x = torch.randn(n, dtype=torch.float64, device=dev, generator=gen)
    full = torch.zeros(n, n, dtype=torch.float64, device=dev)
    il = torch.tril_indices(n, n, device=dev)
    full[il[0], il[1]] = C.double()
    cx = full @ x + full.t() @ x - torch.diagonal(full) * x
    del full, il
    atax = torch.zeros(n, dtype=torch.float64, device=dev)
    fro2 = 0.0
    for r0 in range(0, A.shape[0], 8192):
        blk = A[r0:r0 + 8192].double()
        atax += blk.t() @ (blk @ x)
        fro2 += float((blk * blk).sum())
    den = fro2 * float(x.norm())
    return float((cx - atax).norm()) / den if den > 0 else float((cx - atax).norm())


def _serving(P, torch, n_req: int, budget: int, max_active: int, streams: int, oracle_seconds: float):
    """Gram-request stream: Poisson arrivals, m log-uniform in [1024, 65536],
    n log-uniform in [64, 4096], FP32 N(0,1) entries drawn on the device.
    Closed loop first (all requests at t=0) to find the saturation rate X,
    then open loop at 0.5 X and 0.8 X.  Latency = completion - submission.
    A separate, untimed verification run of the same stream keeps every A:
    each result is checked by Freivalds' test on the device, and the oracle
    checks every 100th request with m n^2 <= 1e10 and then the others with
    m n^2 <= 1e10 (smallest first) within a time budget."""
    import queue
    import threading

    import oracle
    import synthetic
    from paper_1902_02104_amd.serving import Server

    t_unit, ms, ns = synthetic.request_stream(n_req, seed=synthetic.SEED_STREAM, rate_per_s=1.0)
    flops = ms.astype(np.float64) * ns.astype(np.float64) ** 2
    threads = _host_info()["threads"]

    def run(rate):
        with Server(budget, max_active=max_active, streams=streams) as s:
            q = queue.Queue()
            infos = [None] * n_req

            def releaser():
                for i in range(n_req):
                    tk = q.get()
                    infos[i] = s.wait(tk, timeout=600)
                    s.release(tk)

            th = threading.Thread(target=releaser)
            th.start()
            t0 = time.perf_counter()
            for i in range(n_req):
                if rate:
                    target = t0 + t_unit[i] / rate
                    while True:
                        dt = target - time.perf_counter()
                        if dt <= 0:
                            break
                        time.sleep(min(dt, 0.0005) if dt > 0.0002 else 0)
                q.put(s.submit(int(ms[i]), int(ns[i]), dtype=P.F32, seed=synthetic.SEED_REQUEST_BASE + i))
            th.join()
            st = s.stats()
        lat = np.array([r["t_done"] - r["t_submit"] for r in infos]) * 1e3
        t_first = min(r["t_submit"] for r in infos)
        t_last = max(r["t_done"] for r in infos)
        done_flops = float(sum(r["flops"] for r in infos))
        return {"requests": n_req, "makespan_s": t_last - t_first,
                "throughput_req_s": n_req / (t_last - t_first),
                "tflops_mn2": done_flops / (t_last - t_first) / 1e12,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "batched_requests": st["batched_requests"],
                "grouped_launches": st["batches"], "chunked_requests": int(sum(1 for r in infos if r["slabs"] > 1)),
                "pool_peak_gb": st["pool_peak"] / 1e9}

    def verify():
        small = [i for i in range(n_req) if flops[i] <= 1e10]
        order = small[::100] + sorted(set(small) - set(small[::100]), key=lambda i: flops[i])
        rank = {i: k for k, i in enumerate(order)}
        gen = torch.Generator(device="cuda").manual_seed(7)
        worst_f, worst_o, n_oracle, oracle_s = 0.0, 0.0, 0, 0.0
        with Server(budget, max_active=max_active, streams=streams) as s:
            # a window of requests in flight: results (and their kept A) are
            # taken in submission order, so the pool never fills with finished
            # requests that wait behind one it cannot admit
            window = 2 * max_active
            sub = lambda i: s.submit(int(ms[i]), int(ns[i]), dtype=P.F32, seed=synthetic.SEED_REQUEST_BASE + i,
                                     keep_a=True)
            tickets = [sub(i) for i in range(min(window, n_req))]
            for i in range(n_req):
                tk = tickets[i]
                if i + window < n_req:
                    tickets.append(sub(i + window))
                C, A = s.take(tk, want_a=True, device=True)
                worst_f = max(worst_f, _freivalds_device(torch, C, A, int(ns[i]), gen))
                if i in rank and (rank[i] < len(small[::100]) or oracle_s < oracle_seconds):
                    t = time.perf_counter()
                    An = A.cpu().numpy().astype(np.float64)
                    ref = oracle.classical_mt(An, threads=threads) if flops[i] > 1e8 else oracle.classical(An)
                    worst_o = max(worst_o, oracle.rel_fro(C.cpu().numpy().astype(np.float64), ref, int(ns[i])))
                    oracle_s += time.perf_counter() - t
                    n_oracle += 1
                del C, A
        return {"requests": n_req, "freivalds_checked": n_req, "max_freivalds_residual": worst_f,
                "oracle_checked": n_oracle, "oracle_candidates_mn2_le_1e10": len(small),
                "oracle_seconds": oracle_s, "max_rel_fro_vs_oracle": worst_o}

    closed = run(None)
    x = closed["throughput_req_s"]
    _log("serving closed loop: %.1f req/s" % x)
    out = {"workload": "%d requests, m log-uniform [1024, 65536], n log-uniform [64, 4096], FP32 N(0,1) "
                       "drawn on the device, HBM budget %.0f GB, %d in flight, %d streams"
                       % (n_req, budget / 1e9, max_active, streams),
           "saturation": closed}
    for frac in (0.5, 0.8):
        r = run(frac * x)
        r["rate_req_s"] = frac * x
        out["open_%.1fX" % frac] = r
        _log("serving open loop %.1fX: p50 %.2f ms p99 %.2f ms" % (frac, r["p50_ms"], r["p99_ms"]))
    out["verification"] = verify()
    _log("serving verification: Freivalds max %.2e over %d, oracle max relF %.2e over %d"
         % (out["verification"]["max_freivalds_residual"], n_req, out["verification"]["max_rel_fro_vs_oracle"],
            out["verification"]["oracle_checked"]))
    return out


def _tall_skinny(P, torch, dev, stream, m: int, n: int, steps: int):
    """Least-squares shaped input: N(0,1) entries, columns scaled by
    10^U(-3,3); FP64 and FP32 forms, 0-2 Strassen levels, with and without
    column equilibration; sampled entries against the oracle with the scaled
    error max |dC_ij| / sqrt(C_ii C_jj).  `best` is the fastest run whose
    scaled error meets the form's bound (FP64 1e-12, FP32 2e-5)."""
    import oracle
    import synthetic
    A64 = synthetic.tall_scaled(m, n)
    out = {"workload": "A %dx%d, N(0,1) with columns scaled by 10^U(-3,3) (seeds %d, %d)"
                       % (m, n, synthetic.SEED_TALL_Z, synthetic.SEED_TALL_SCALES)}
    rng = np.random.default_rng(7)
    pairs = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(40)]
    for name, dt, Anp, bound in (("fp64", P.F64, A64, 1e-12), ("fp32", P.F32, A64.astype(np.float32), 2e-5)):
        At = torch.from_numpy(Anp).to(dev)
        Ar = Anp.astype(np.float64)
        refs = {}
        for i, j in pairs:
            i, j = max(i, j), min(i, j)
            refs[(i, j)] = oracle.classical(np.ascontiguousarray(Ar[:, [j, i]]))
        best = None
        for d, eq in ((0, False), (1, False), (2, False), (1, True), (2, True)):
            fn = lambda: P.gram(At, dtype=dt if dt == P.F64 else dt | P.OUT_F64, cutoff=256, max_depth=d,
                                stream=stream, equilibrate=eq)
            C = fn()
            torch.cuda.synchronize(dev)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize(dev)
            ms_ = e0.elapsed_time(e1) / steps
            Cn = C.cpu().numpy()
            worst = 0.0
            for (i, j), ref in refs.items():
                cij = ref[1] if i != j else ref[0]
                worst = max(worst, abs(Cn[i * (i + 1) // 2 + j] - cij) / np.sqrt(ref[0] * ref[2]))
            rec = {"ms": ms_, "tflops_mn2": float(m) * n * n / (ms_ * 1e-3) / 1e12, "depth": d,
                   "equilibrated": eq, "scaled_err_sampled": worst}
            key = "%s_d%d%s" % (name, d, "_eq" if eq else "")
            out[key] = rec
            _log("tall %s: %.2f ms, scaled error %.2e" % (key, ms_, worst))
            if worst <= bound and (best is None or ms_ < best["ms"]):
                best = rec
        out[name] = best
        del At
    return out


def _normal_equations(P, torch, dev, stream, C0, n: int, steps: int):
    """Consumers of the product: the Cholesky factor of the headline's packed
    C (n^3/3 flops counted) with a solve check, and the whole least-squares
    chain (product, factor, A^t b, solves) on the 262144 x 2048 shape with
    uniform[-1,1] data, checked through the normal-equation residual
    ||A^t (A x - b)|| / (||A||_F^2 ||x||)."""
    import synthetic

    def timed(fn, k):
        fn()
        torch.cuda.synchronize(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize(dev)
        return e0.elapsed_time(e1) / k

    out = {}
    Cw = torch.empty_like(C0)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    t_copy = timed(lambda: Cw.copy_(C0), steps)
    t_fac = timed(lambda: (Cw.copy_(C0), P.cholesky(Cw, n, info=info, stream=stream)), steps) - t_copy
    assert int(info.item()) == 0
    full = torch.zeros((n, n), dtype=torch.float64, device=dev)
    il = torch.tril_indices(n, n, device=dev)
    full[il[0], il[1]] = C0
    full = full + full.t() - torch.diag(torch.diagonal(full))
    e = torch.ones(n, dtype=torch.float64, device=dev)
    b = full.mv(e)
    del full
    t_solve = timed(lambda: P.cholesky_solve(Cw, b.clone(), stream=stream), steps)
    x = P.cholesky_solve(Cw, b.clone(), stream=stream)
    torch.cuda.synchronize(dev)
    # the update kernel, timed by events on its own launch streams: C is read
    # and written once per trailing lower entry (16 B) for 2 w flops
    P.profile_enable(True)
    P.profile_collect()
    for _ in range(steps):
        Cw.copy_(C0)
        P.cholesky(Cw, n, info=info, stream=stream)
    torch.cuda.synchronize(dev)
    prof = P.profile_collect()
    P.profile_enable(False)
    upd_ms, upd_launches = prof["factor_update"]
    entries = sum((n - kb - min(64, n - kb)) * (n - kb - min(64, n - kb) + 1) // 2 for kb in range(0, n, 64))
    upd_bytes = 16.0 * entries * steps
    achieved = upd_bytes / (upd_ms * 1e-3) / 1e9
    roof_fac = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_chol_update_f64",
                "algorithmic_bytes_per_launch": upd_bytes / max(upd_launches, 1),
                "avg_launch_ms": upd_ms / max(upd_launches, 1),
                "mfma_tflops": 2 * 64 * entries * steps / (upd_ms * 1e-3) / 1e12,
                "panel_ms_per_factor": prof["factor_panel"][0] / steps}
    out["factor"] = {"n": n, "ms": t_fac, "tflops": n ** 3 / 3 / (t_fac * 1e-3) / 1e12, "roofline": roof_fac,
                     "frac_of_fp64_peak": n ** 3 / 3 / (t_fac * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                     "solve_ms_nrhs1": t_solve, "solve_max_err_vs_ones": float((x - 1.0).abs().max())}
    _log("normal equations: factor n=%d %.2f ms (%.1f TF/s), solve %.2f ms"
         % (n, t_fac, out["factor"]["tflops"], t_solve))
    m, k = 262144, 2048
    A = torch.from_numpy(synthetic.uniform(m, k, synthetic.SEED_TALL_Z)).to(dev)
    bb = torch.from_numpy(synthetic.uniform(m, 1, synthetic.SEED_TALL_SCALES)[:, 0].copy()).to(dev)
    t_chain = timed(lambda: P.normal_solve(A, bb, info=info, stream=stream), 3)
    t_gram = timed(lambda: P.gram(A, stream=stream), 3)
    t_atb = timed(lambda: P.atb(A, bb, stream=stream), 3)
    xs = P.normal_solve(A, bb, info=info, stream=stream)
    torch.cuda.synchronize(dev)
    g = A.t().mv(A.mv(xs) - bb)
    res = float(g.norm() / (torch.linalg.matrix_norm(A, "fro") ** 2 * xs.norm()))
    t_proj = timed(lambda: P.project(A, bb, info=info, stream=stream), 3)
    pb = P.project(A, bb, info=info, stream=stream)
    torch.cuda.synchronize(dev)
    orth = float(A.t().mv(bb - pb).norm() / (torch.linalg.matrix_norm(A, "fro") * bb.norm()))
    out["least_squares"] = {"workload": "A %dx%d uniform[-1,1] (seed %d), b uniform (seed %d), one right-hand side"
                                        % (m, k, synthetic.SEED_TALL_Z, synthetic.SEED_TALL_SCALES),
                            "ms": t_chain, "gram_ms": t_gram, "atb_ms": t_atb,
                            "atb_gbs": m * k * 8 / (t_atb * 1e-3) / 1e9, "info": int(info.item()),
                            "normal_eq_residual": res, "project_ms": t_proj, "project_orthogonality": orth}
    _log("normal equations: least squares %dx%d %.2f ms (product %.2f ms, A^t b %.3f ms), residual %.1e; "
         "projection %.2f ms, orthogonality %.1e" % (m, k, t_chain, t_gram, t_atb, res, t_proj, orth))
    del A
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--cutoff", type=int, default=0, help="0: tune over {128,256,512}")
    ap.add_argument("--max-depth", type=int, default=None, help="default: tune over {1, 2}")
    ap.add_argument("--no-variant-sweep", dest="variant_sweep", action="store_false",
                    help="do not time the Winograd variant in the sweep")
    ap.add_argument("--form", default="tune", choices=("tune", "intile", "tiles", "opsums"),
                    help="last Strassen level: in-tile, product tiles (fused sums), product tiles on operand sums "
                         "formed in a memory pass, or tuned (all three timed; the headline takes the fastest "
                         "fused form)")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-5000", action="store_true", help="skip the 5000 x 5000 leg")
    ap.add_argument("--no-check", action="store_true", help="skip the full-output oracle check")
    ap.add_argument("--no-classical", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--precision-n", type=int, default=8192)
    ap.add_argument("--precision-depths", default="0,1,2", help="Strassen levels timed for each precision form")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=10000)
    ap.add_argument("--serving-oracle-seconds", type=float, default=30.0,
                    help="time budget of the serving leg's oracle checks beyond every 100th small request")
    ap.add_argument("--serving-budget-gb", type=float, default=200.0)
    ap.add_argument("--no-tall", action="store_true")
    ap.add_argument("--no-normal", action="store_true", help="skip the Cholesky / least-squares leg")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the timed steps, copy this many bytes device to device three times "
                         "(a plain copy of known size for scaling hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(row sharding with one reduce of packed partials is the designed extension)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1902_02104_amd as P
    import synthetic

    P.load()
    dev = torch.device("cuda:0")
    n = m = args.n
    A_np = synthetic.uniform(m, n, synthetic.SEED_SQUARE)
    A = torch.from_numpy(A_np).to(dev)
    C = torch.empty(P.tri(n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    def run(cfg):
        _run_cfg(P, A, C, stream, cfg)

    def time_steps(fn, steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(dev)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize(dev)
        return e0.elapsed_time(e1) / steps

    # Tuning over the configurations of the method: the leaf cutoff over the
    # set the workload names, the Strassen levels per off-diagonal product
    # (0: classical off-diagonal products), the form of the Strassen levels
    # (product tiles or in-tile, both fusing the operand sums into the staged
    # loads; product tiles on operand sums formed in a memory pass are timed
    # for reference only), the Winograd variant, and the library's default
    # call (adaptive depth).  The headline takes the fastest; the fastest
    # configuration with at least one Strassen level is reported beside it.
    cfgs = _sweep_configs(args)
    sweep = {}
    for cfg in cfgs:
        run(cfg)
        sweep[cfg["key"]] = time_steps(lambda: run(cfg), 3)
        _log("sweep %s: %.2f ms" % (cfg["key"], sweep[cfg["key"]]))
    by_key = {c["key"]: c for c in cfgs}
    fused = {k: v for k, v in sweep.items() if by_key[k]["form"] != "opsums"} or sweep
    best = by_key[min(fused, key=fused.get)]
    strassen_keys = {k: v for k, v in fused.items() if by_key[k]["levels"] >= 1}
    best_str = by_key[min(strassen_keys, key=strassen_keys.get)] if strassen_keys else None

    for _ in range(args.warmup):
        run(best)
    ms = time_steps(lambda: run(best), args.steps)
    _log("timed %d steps (%s): %.3f ms/step" % (args.steps, best["key"], ms))
    C_host = C.cpu().numpy()  # the timed output, checked entry by entry below
    # Per-kernel split: the same steps again with HIP events around every
    # launch, on the stream each kernel is launched on (kept out of the
    # headline's timed region above).
    ms_prof, prof = _profiled(P, lambda: run(best), time_steps, args.steps)
    _log("profiled pass: %.3f ms/step" % ms_prof)
    st = _plan_stats(P, m, n, best)
    flops_mn2 = float(m) * n * n
    value = flops_mn2 / (ms * 1e-3) / 1e12
    kt = {k: v for k, v in prof.items() if v[1] > 0}
    roof = _roofline(kt, st, best, args.steps, n)

    strassen = None
    if best_str is not None:
        if best_str is best:
            s_ms, s_kt = ms, kt
        else:
            for _ in range(args.warmup):
                run(best_str)
            s_ms = time_steps(lambda: run(best_str), args.steps)
            _, s_prof = _profiled(P, lambda: run(best_str), time_steps, args.steps)
            s_kt = {k: v for k, v in s_prof.items() if v[1] > 0}
        s_st = _plan_stats(P, m, n, best_str)
        strassen = {"config": {k: best_str[k] for k in ("key", "cutoff", "levels", "form", "variant")},
                    "ms": s_ms, "tflops_mn2": flops_mn2 / (s_ms * 1e-3) / 1e12,
                    "mults_over_classical": s_st["mults"] / s_st["classical_mults"],
                    "kernels_ms_per_step": {k: v[0] / args.steps for k, v in s_kt.items()},
                    "roofline": _roofline(s_kt, s_st, best_str, args.steps, n)}
        _log("fastest with Strassen levels (%s): %.3f ms" % (best_str["key"], s_ms))

    sq5000 = None
    if not args.no_5000 and n != 5000:
        sq5000 = _square_leg(P, torch, dev, stream, 5000, args)

    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize(dev)
        del src, dst

    classical = None
    if not args.no_classical:
        csyrk = lambda: P.gram(A, cutoff=n, max_depth=0, out=C, stream=stream)
        csyrk()
        cms = time_steps(csyrk, 5)
        classical = {"ms": cms, "tflops_mn2": flops_mn2 / (cms * 1e-3) / 1e12,
                     "what": "classical SYRK on the same GPU (same MFMA tile kernel, cutoff >= n)"}

    forms = None
    if not args.no_precision:
        # 20 calls per timed pass: the sub-millisecond forms need that many for steady clocks
        forms = _precision_forms(P, torch, dev, stream, args.precision_n, 20,
                                 tuple(int(d) for d in args.precision_depths.split(",")))

    serving = None
    if not args.no_serving:
        serving = _serving(P, torch, args.serving_requests, int(args.serving_budget_gb * 1e9), 32, 4,
                           args.serving_oracle_seconds)

    tall = None
    if not args.no_tall:
        tall = _tall_skinny(P, torch, dev, stream, 262144, 2048, 3)

    normal = None
    if not args.no_normal:
        normal = _normal_equations(P, torch, dev, stream, C, n, 5)

    cpu, cpu_rows = None, None
    if not args.no_cpu:
        _log("oracle CPU baseline")
        cpu, cpu_rows = _cpu_baseline(A_np, args.cpu_seconds)
    check = None
    if not args.no_check:
        _log("full-output check against the oracle")
        check = _full_check(A_np, C_host, cpu_rows)
        _log("check: relF %.3e, max scaled error %.3e" % (check["rel_fro"], check["max_scaled_err"]))

    out = {
        "metric": "effective TFLOP/s of A^tA (m*n^2 counted), FP64 plain",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "square FP64 A %dx%d, i.i.d. uniform[-1,1] (seed %d), packed lower C = A^tA"
                        % (m, n, synthetic.SEED_SQUARE),
            "m": m, "n": n, "tuned": best["key"], "cutoff": st["cutoff"], "strassen_levels": st["max_hasa_depth"],
            "form": best["form"], "variant": best["variant"], "phases": st["phases"], "ata_depth": st["ata_depth"],
            "mults_over_classical": st["mults"] / st["classical_mults"], "tuning_sweep_ms": sweep,
        },
        "strassen_best": strassen,
        "square_5000": sq5000,
        "value_mn_n1": float(m) * n * (n + 1) / (ms * 1e-3) / 1e12,
        "roofline": roof,
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
        "classical_same_gpu": classical,
        "cpu_baseline": cpu,
        "precision_forms": forms,
        "serving": serving,
        "tall_skinny": tall,
        "normal_equations": normal,
        "check": check,
        "ms_per_step_profiled": ms_prof,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
