"""GPU parity of the reduced-precision forms.

Each form is checked three ways: bit-exact on inputs whose products and sums
the form represents exactly; tightly against the oracle's reference of what
the form computes (same conversions, exact FP64 products: only the FP32
accumulation rounding differs); and against the FP64 Gram matrix within the
form's stated error bound.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

# stated relative Frobenius bounds against the FP64 Gram of the FP32 input
BOUND_F32 = 2e-5
BOUND_BF16X3 = 5e-5
BOUND_FP8 = 5e-2
# against the oracle's reference of the same conversions (FP32 accumulation only)
TIGHT = 2e-6
# the e4m3 MFMA sums 128 products inside one instruction with its own internal
# accumulation (measured 5e-6 relative against exact products); a conversion
# error would show at the format's resolution, about 1e-2
TIGHT_FP8 = 2e-5


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_02104_amd as P
    P.load()
    return torch, P


def _gram(env, A32, dtype, **kw):
    torch, P = env
    A = torch.from_numpy(np.ascontiguousarray(A32, dtype=np.float32)).cuda()
    C = P.gram(A, dtype=dtype, **kw)
    torch.cuda.synchronize()
    return C.double().cpu().numpy()


def test_conversions_match_torch_casts(env, orc):
    torch, P = env
    print("case: conversions", flush=True)
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(300000) * 10.0 ** rng.uniform(-20, 20, 300000)).astype(np.float32)
    x = np.concatenate([x, np.array([0.0, -0.0, 1.0, 1.00390625, 65504.0, 3e38, 1e-40], np.float32)])
    hi, lo = P.precision_convert(torch.from_numpy(x).cuda(), P.F32_BF16X3)
    torch.cuda.synchronize()
    ref_hi = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy()
    assert np.array_equal(hi.cpu().numpy(), ref_hi)
    hf = torch.from_numpy(ref_hi).view(torch.bfloat16).float().numpy()
    ref_lo = torch.from_numpy(x - hf).to(torch.bfloat16).view(torch.int16).numpy()
    assert np.array_equal(lo.cpu().numpy(), ref_lo)
    # e4m3 (values inside the format's range; torch does not saturate)
    y = (rng.uniform(-448, 448, 300000) * 10.0 ** rng.uniform(-5, 0, 300000)).astype(np.float32)
    y = np.concatenate([y, np.array([448.0, -448.0, 0.0, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -11, 464.0 - 1e-3],
                                    np.float32)])
    q = P.precision_convert(torch.from_numpy(y).cuda(), P.F32_FP8)
    torch.cuda.synchronize()
    ref_q = torch.from_numpy(y).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(q.cpu().numpy(), ref_q)
    # saturation to the largest finite value (format definition)
    s = P.precision_convert(torch.tensor([1000.0, -500.0], dtype=torch.float32).cuda(), P.F32_FP8)
    assert s.cpu().tolist() == [0x7E, 0xFE]


@pytest.mark.parametrize("depth", [0, 1, 2])
def test_f32_integer_bit_exact(env, orc, depth):
    torch, P = env
    print("case: f32 integer depth", depth, flush=True)
    A = synthetic.integer(256, 192, synthetic.SEED_INTEGER_SMALL)
    exact = orc.classical(A)
    for out in (0, P.OUT_F64):
        C = _gram(env, A, P.F32 | out, cutoff=32, max_depth=depth)
        assert np.array_equal(C, exact)


@pytest.mark.parametrize("depth,bound", [(0, 2e-6), (1, BOUND_F32), (2, BOUND_F32)])
def test_f32_uniform(env, orc, depth, bound):
    torch, P = env
    print("case: f32 uniform depth", depth, flush=True)
    A = synthetic.uniform(700, 600, 8, dtype=np.float32)
    ref = orc.classical(A.astype(np.float64))
    for out in (0, P.OUT_F64):
        C = _gram(env, A, P.F32 | out, cutoff=64, max_depth=depth)
        assert orc.rel_fro(C, ref, 600) <= bound


def test_bf16x3(env, orc):
    torch, P = env
    print("case: bf16x3", flush=True)
    Ai = synthetic.integer(300, 200, 7).astype(np.float32)
    exact = orc.classical(Ai.astype(np.float64))
    for c in (32, 10 ** 6):
        assert np.array_equal(_gram(env, Ai, P.F32_BF16X3 | P.OUT_F64, cutoff=c), exact)
    A = synthetic.uniform(900, 500, 9, dtype=np.float32)
    ref = orc.gram_bf16x3(A)
    ex = orc.classical(A.astype(np.float64))
    for out in (0, P.OUT_F64):
        for c in (64, 10 ** 6):
            C = _gram(env, A, P.F32_BF16X3 | out, cutoff=c)
            assert orc.rel_fro(C, ref, 500) <= TIGHT
            assert orc.rel_fro(C, ex, 500) <= BOUND_BF16X3


def test_fp8(env, orc):
    torch, P = env
    print("case: fp8", flush=True)
    Ai = synthetic.integer(64, 150, 11).astype(np.float32)
    exact = orc.classical(Ai.astype(np.float64))
    for c in (16, 10 ** 6):
        assert np.array_equal(_gram(env, Ai, P.F32_FP8 | P.OUT_F64, cutoff=c), exact)
    A = synthetic.uniform(1000, 420, 12, dtype=np.float32)
    ref = orc.gram_fp8(A)
    ex = orc.classical(A.astype(np.float64))
    for out in (0, P.OUT_F64):
        for c in (64, 10 ** 6):
            C = _gram(env, A, P.F32_FP8 | out, cutoff=c)
            assert orc.rel_fro(C, ref, 420) <= TIGHT_FP8
            assert orc.rel_fro(C, ex, 420) <= BOUND_FP8


def test_reduced_precision_ragged_and_strided(env, orc):
    """Odd shapes, a row stride above n and a non-uniform recursion tree."""
    torch, P = env
    print("case: lp ragged", flush=True)
    for (m, n, c) in [(513, 600, 256), (77, 33, 8), (1, 5, 1), (130, 1, 4)]:
        A = synthetic.uniform(m, n, m + n, dtype=np.float32)
        buf = synthetic.with_lda(A, n + 3, fill=np.float32(1e30))
        At = torch.from_numpy(buf).cuda()[:, :n]
        for dt, ref in ((P.F32_BF16X3, orc.gram_bf16x3(A)), (P.F32_FP8, orc.gram_fp8(A))):
            C = P.gram(At, dtype=dt | P.OUT_F64, cutoff=c)
            torch.cuda.synchronize()
            tol = TIGHT_FP8 if dt == P.F32_FP8 else TIGHT
            assert orc.rel_fro(C.cpu().numpy(), ref, n) <= tol, (m, n, c, dt)
    with pytest.raises(P.AtaError):  # at most two expanded levels (one for Winograd)
        P.gram(torch.zeros(8, 8, device="cuda"), dtype=P.F32_FP8, max_depth=3)
    with pytest.raises(P.AtaError):
        P.gram(torch.zeros(8, 8, device="cuda"), dtype=P.F32_BF16X3, max_depth=2, variant="winograd")


def test_precision_forms_full_size_sampled(env, orc):
    """The 8192 x 8192 precision workload: sampled entries of each form
    against the oracle's reference of that form."""
    torch, P = env
    print("case: 8192 precision forms", flush=True)
    n = 8192
    A = synthetic.uniform(n, n, synthetic.SEED_PRECISION, dtype=np.float32)
    At = torch.from_numpy(A).cuda()
    rng = np.random.default_rng(3)
    pairs = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(24)] + [(n - 1, 0), (n - 1, n - 1)]
    A64 = A.astype(np.float64)
    s = orc.pow2_column_scales(A64)
    for dt in (P.F32, P.F32_BF16X3, P.F32_FP8):
        C = P.gram(At, dtype=dt | P.OUT_F64, cutoff=256).cpu().numpy()
        worst = 0.0
        for i, j in pairs:
            i, j = max(i, j), min(i, j)
            ai, aj = A[:, i], A[:, j]
            if dt == P.F32_BF16X3:
                hi, lo = orc.bf16_split(np.stack([ai, aj], 1))
                hi, lo = hi.astype(np.float64), lo.astype(np.float64)
                ref = hi[:, 0] @ hi[:, 1] + hi[:, 0] @ lo[:, 1] + lo[:, 0] @ hi[:, 1]
            elif dt == P.F32_FP8:
                qi = orc.e4m3_round(A64[:, i] * s[i])
                qj = orc.e4m3_round(A64[:, j] * s[j])
                ref = (qi @ qj) / s[i] / s[j]
            else:
                ref = A64[:, i] @ A64[:, j]
            scale = np.sqrt((A64[:, i] @ A64[:, i]) * (A64[:, j] @ A64[:, j]))
            worst = max(worst, abs(C[i * (i + 1) // 2 + j] - ref) / scale)
        assert worst <= (1e-5 if dt == P.F32_BF16X3 else 2e-5), (dt, worst)


def test_reduced_precision_split_k(env, orc):
    torch, P = env
    print("case: lp split-K", flush=True)
    A = synthetic.uniform(20000, 200, 13, dtype=np.float32)
    for dt, ref, tol in ((P.F32_BF16X3, orc.gram_bf16x3(A), TIGHT), (P.F32_FP8, orc.gram_fp8(A), TIGHT_FP8)):
        assert P.plan_info(20000, 200, 64, dtype=dt)["combine_tasks"] >= 1
        C = _gram(env, A, dt | P.OUT_F64, cutoff=64)
        assert orc.rel_fro(C, ref, 200) <= tol


# (rows, Strassen levels) -> staging of the 128 x 128 tiles (bfloat16 pairs, e4m3):
# 2 direct-to-LDS copies of 16 bytes, 1 of dwords, 0 through registers
COPY_PATH_CASES = [((2048, 1), (2, 2)), ((2047, 1), (2, 2)), ((2047, 0), (2, 2)), ((2044, 1), (1, 0)),
                   ((2040, 1), (1, 1)), ((2041, 1), (0, 0))]


def test_reduced_precision_copy_paths(env, orc):
    """Plans whose segment windows all start and end on 16 bytes of the
    converted copy (or end at its last row, past which the copy holds zeros)
    stage through 16-byte direct-to-LDS copies, on dwords through dword
    copies, otherwise through registers.  Every path is exact on
    small-integer inputs.  The row counts pick each path: the split rows of
    one Strassen level (ceil(m/2)) decide.  A 200000-row matrix runs split-K
    parts (boundaries on multiples of 16 rows) with 16-byte copies."""
    torch, P = env
    print("case: lp copy paths", flush=True)
    for (m, d), want in COPY_PATH_CASES:
        Ai = synthetic.integer(m, 130, m).astype(np.float32)
        exact = orc.classical(Ai.astype(np.float64))
        c = 64 if d else 10 ** 6
        for dt, w in zip((P.F32_BF16X3, P.F32_FP8), want):
            assert P.plan_info(m, 130, c, dtype=dt, max_depth=d)["lp_staging"] == w, (m, d, dt)
            assert np.array_equal(_gram(env, Ai, dt | P.OUT_F64, cutoff=c, max_depth=d), exact), (m, d, dt)
    Ai = synthetic.integer(200000, 64, 5).astype(np.float32)
    exact = orc.classical(Ai.astype(np.float64))
    for dt in (P.F32_BF16X3, P.F32_FP8):
        st = P.plan_info(200000, 64, 10 ** 6, dtype=dt)
        assert st["combine_tasks"] >= 1 and st["lp_staging"] == 2
        assert np.array_equal(_gram(env, Ai, dt | P.OUT_F64, cutoff=10 ** 6), exact), dt


# Strassen levels in the reduced-precision forms: relative Frobenius bounds
# against the FP64 Gram, per form and level count.  The operand sums double
# the operands' range and the combination adds up to four products, so the
# conversion error grows with each level; the bounds are twice the error of
# the oracle's reduced-precision recursion (exact products of the converted
# operands) on this workload: bfloat16 split 5.0e-6 and 8.4e-6, e4m3 4.2e-2
# and 7.1e-2 at one and two levels.
LP_STRASSEN_BOUND = {("bf16x3", 1): 5e-5, ("bf16x3", 2): 5e-5, ("fp8", 1): 8.4e-2, ("fp8", 2): 1.42e-1}


def _lp_dtype(P, fmt):
    return (P.F32_BF16X3 if fmt == "bf16x3" else P.F32_FP8) | P.OUT_F64


@pytest.mark.parametrize("fmt", ["bf16x3", "fp8"])
@pytest.mark.parametrize("depth", [1, 2])
def test_lowp_strassen_integer_exact(env, orc, fmt, depth):
    """Integers and their operand sums are exact in both formats (96 rows keep
    every FP32 partial sum of scaled e4m3 products below 2^24)."""
    torch, P = env
    print("case: lp strassen integer", fmt, depth, flush=True)
    A = synthetic.integer(96, 80, 71, dtype=np.float32)
    C = _gram(env, A, _lp_dtype(P, fmt), cutoff=16, max_depth=depth)
    assert np.array_equal(C, orc.classical(A.astype(np.float64)))


@pytest.mark.parametrize("fmt", ["bf16x3", "fp8"])
@pytest.mark.parametrize("depth", [1, 2])
def test_lowp_strassen_uniform(env, orc, fmt, depth):
    """Uniform input: within the form's Strassen bound of the FP64 Gram, and
    close to the oracle's reduced-precision recursion.  bfloat16 split: only
    the FP32 accumulation (and, at two levels, the order of the FP32 operand
    sums) differs.  e4m3: besides the MFMA's internal accumulation (TIGHT_FP8
    for classical leaves), the device merges the row chunks of the recursion
    into one K range per product and scales each operand row by its maximum
    over that range, the recursion by its maximum per chunk, so a row whose
    two maxima fall in different binades rounds differently (measured: 1.2e-5
    and 2.4e-5 at one and two levels)."""
    torch, P = env
    print("case: lp strassen uniform", fmt, depth, flush=True)
    A = synthetic.uniform(600, 450, 72, dtype=np.float32)
    ex = orc.classical(A.astype(np.float64))
    C = _gram(env, A, _lp_dtype(P, fmt), cutoff=64, max_depth=depth)
    err = orc.rel_fro(C, ex, 450)
    ref = orc.ata_lowp(A, fmt, 64, depth)
    dif = orc.rel_fro(C, ref, 450)
    print("   relF vs FP64 %.3e, vs reduced-precision recursion %.3e" % (err, dif), flush=True)
    assert err <= LP_STRASSEN_BOUND[(fmt, depth)]
    assert dif <= (TIGHT if fmt == "bf16x3" else 1e-4)


@pytest.mark.parametrize("m,n", [(6144, 6144), (6001, 5999), (9001, 5903)])
def test_fp8_large_tiles(env, orc, m, n):
    """e4m3 launches with at least one 256 x 256 tile per CU run on the large
    tiles (one launch of kind "gemm"; the 128 x 128 tiles of a single SYRK
    run as kind "syrk").  Every entry against the oracle's e4m3 reference;
    integer inputs with K = 64 stay exact (every partial sum below 2^24)."""
    torch, P = env
    print("case: fp8 large tiles", m, n, flush=True)
    A = synthetic.uniform(m, n, 41, dtype=np.float32)
    At = torch.from_numpy(A).cuda()
    P.profile_enable(True)
    P.profile_collect()
    C = P.gram(At, dtype=P.F32_FP8 | P.OUT_F64, cutoff=256, max_depth=0)
    prof = P.profile_collect()
    P.profile_enable(False)
    assert prof["gemm"][1] == 1 and prof["syrk"][1] == 0, prof
    rel = orc.rel_fro(C.cpu().numpy(), orc.gram_fp8(A), n)
    print("  relF vs e4m3 reference %.3e" % rel, flush=True)
    assert rel <= TIGHT_FP8
    Ai = synthetic.integer(64, n, 42).astype(np.float32)
    Ci = P.gram(torch.from_numpy(Ai).cuda(), dtype=P.F32_FP8 | P.OUT_F64, cutoff=256, max_depth=0)
    torch.cuda.synchronize()
    assert np.array_equal(Ci.cpu().numpy(), orc.classical(Ai.astype(np.float64)))


@pytest.mark.parametrize("m", [1000, 1001])
def test_bf16x3_split_last_round(env, orc, m):
    """A single SYRK of 300 tiles of 128 x 128 at one resident bfloat16-pair
    workgroup per CU: 256 tiles run whole, the last 44 run as a second launch
    with each K range split into parts (partials summed in part order).  Even
    m stages through direct-to-LDS copies, odd m through registers.  Every
    entry against the oracle's bfloat16-pair reference, and exact on small
    integers, with both output types."""
    torch, P = env
    n = 3000
    print("case: bf16x3 split last round", m, n, flush=True)
    A = synthetic.uniform(m, n, 43 + m, dtype=np.float32)
    At = torch.from_numpy(A).cuda()
    P.profile_enable(True)
    P.profile_collect()
    C = P.gram(At, dtype=P.F32_BF16X3 | P.OUT_F64, cutoff=256, max_depth=0)
    prof = P.profile_collect()
    P.profile_enable(False)
    assert prof["syrk"][1] == 2 and prof["gemm"][1] == 0, prof
    ref = orc.gram_bf16x3(A)
    assert orc.rel_fro(C.cpu().numpy(), ref, n) <= TIGHT
    C32 = P.gram(At, dtype=P.F32_BF16X3, cutoff=256, max_depth=0)
    torch.cuda.synchronize()
    assert orc.rel_fro(C32.double().cpu().numpy(), ref, n) <= TIGHT
    Ai = synthetic.integer(m, n, 44 + m).astype(np.float32)
    assert np.array_equal(_gram(env, Ai, P.F32_BF16X3 | P.OUT_F64, cutoff=256, max_depth=0),
                          orc.classical(Ai.astype(np.float64)))
