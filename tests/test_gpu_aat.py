"""GPU parity of the companion product A A^t (ata_aat) against the oracle.

A A^t is by definition the Gram matrix of A^t (entry (i, j) = sum_k A[i,k]
A[j,k]), which the oracle computes as its plain definition applied to the
transposed array.  Integer inputs: exact in every form whose conversions
represent small integers exactly (FP64, FP32, BF16x3, FP8 with power-of-two
column scales).  Uniform FP32 inputs: the FP32 form's stated bound.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

BOUND_F32 = 2e-5


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_02104_amd as P
    P.load()
    return torch, P


def _aat(env, A, pad, dt, dtype, **kw):
    torch, P = env
    m, n = A.shape
    Ap = np.zeros((m, n + pad), dtype=A.dtype)
    Ap[:, :n] = A
    At = torch.from_numpy(Ap).to(dt).cuda()[:, :n]
    C = P.gram_rows(At, dtype=dtype, **kw)
    torch.cuda.synchronize()
    return C.double().cpu().numpy()


def test_aat_integer_exact_all_forms(env, orc):
    torch, P = env
    for m, n, pad in [(1, 1, 0), (7, 5, 3), (200, 300, 1), (513, 70, 0), (300, 1000, 2)]:
        A = synthetic.integer(m, n, 700 + m)
        ref = orc.classical(np.ascontiguousarray(A.T))
        forms = [(torch.float64, P.F64), (torch.float32, P.F32), (torch.float32, P.F32_BF16X3 | P.OUT_F64),
                 (torch.float32, P.F32_FP8 | P.OUT_F64)]
        for dt, dtype in forms:
            print("case: aat %dx%d pad %d dtype %#x" % (m, n, pad, dtype), flush=True)
            C = _aat(env, A, pad, dt, dtype, cutoff=64)
            assert np.array_equal(C, ref)


def test_aat_f32_uniform(env, orc):
    torch, P = env
    print("case: aat f32 uniform 600x700", flush=True)
    A = synthetic.uniform(600, 700, 9, dtype=np.float32)
    ref = orc.classical(np.ascontiguousarray(A.astype(np.float64).T))
    C = _aat(env, A, 0, torch.float32, P.F32 | P.OUT_F64, cutoff=64)
    assert orc.rel_fro(C, ref, 600) <= BOUND_F32


def test_aat_edges(env, orc):
    torch, P = env
    print("case: aat edges", flush=True)
    C = P.gram_rows(torch.zeros((4, 0), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert C.numel() == 10 and float(C.abs().max()) == 0.0
    C = P.gram_rows(torch.zeros((0, 5), dtype=torch.float64, device="cuda"))
    assert C.numel() == 0
