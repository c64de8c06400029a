"""GPU test of ata_ex_noalloc, the entry point that allocates nothing: its
output against ata_ex (the existing entry point) on the same inputs, for two
calls in a row with the second on a smaller input, through the C ABI."""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_02104_amd as P
    P.load()
    return torch, P


def _both(env, A_np, **kw):
    torch, P = env
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    ref = P.gram(A, **kw)
    out = torch.full_like(ref, float("nan"))
    out, used = P.gram_noalloc(A, out, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy(), used


def test_noalloc_matches_ata_ex_two_calls(env, orc):
    torch, P = env
    print("case: noalloc integer 700x500 then 300x200, default options", flush=True)
    # first call, then a smaller input: the scratch keeps the first call's
    # contents, which must not leak into the second result
    for (m, n, seed) in ((700, 500, 31), (300, 200, 32)):
        A = synthetic.integer(m, n, seed)
        got, ref, used = _both(env, A, cutoff=64)
        assert 0 < used <= P.NOALLOC_SCRATCH_BYTES
        assert np.array_equal(got, ref)
        assert np.array_equal(got, orc.classical(A))


def test_noalloc_workspace_forms(env, orc):
    """Forms that put workspace in the scratch array after the tables."""
    torch, P = env
    print("case: noalloc two in-tile levels, product tiles, e4m3 leaves", flush=True)
    A = synthetic.integer(640, 520, 33)
    ex = orc.classical(A)
    got, ref, used = _both(env, A, cutoff=64, max_depth=2)
    assert np.array_equal(got, ref) and np.array_equal(got, ex)
    got, ref, used = _both(env, A, cutoff=64, max_depth=1, intile=False)
    assert np.array_equal(got, ref) and np.array_equal(got, ex)
    # e4m3 leaves: 96 rows keep every scaled sum below 2^24, so FP32
    # accumulation is exact on these integers
    A8 = synthetic.integer(96, 520, 35)
    got, ref, used = _both(env, A8.astype(np.float32), cutoff=64, dtype=P.F32_FP8 | P.OUT_F64)
    assert used >= 520 * 96  # the converted copy of A is in the scratch
    ex8 = orc.classical(A8)
    assert np.array_equal(got, ex8) and np.array_equal(ref, ex8)


def test_noalloc_uniform_fp64(env, orc):
    torch, P = env
    print("case: noalloc uniform 900x700", flush=True)
    A = synthetic.uniform(900, 700, 34)
    got, ref, used = _both(env, A, cutoff=128)
    ex = orc.classical(A)
    assert orc.rel_fro(got, ex, 700) <= 1e-12
    assert orc.rel_fro(got, ref, 700) <= 1e-12


def test_noalloc_rejects_oversize(env):
    torch, P = env
    print("case: noalloc oversize bfloat16 split 6000x4096", flush=True)
    A = torch.zeros(6000, 4096, dtype=torch.float32, device="cuda")
    out = torch.zeros(P.tri(4096), dtype=torch.float64, device="cuda")
    with pytest.raises(P.AtaError) as ei:
        P.gram_noalloc(A, out, dtype=P.F32_BF16X3 | P.OUT_F64)
    assert ei.value.status == 4  # ATA_EWORKSPACE
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0  # nothing was launched
