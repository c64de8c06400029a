"""GPU parity of the normal-equation consumers (Cholesky factor, triangular
solves, A^t B, and the chained least-squares solve) against the CPU oracle.

Exact cases: C = L0 L0^t for an integer lower L0 with diagonal entries in
{1, 2, 4}.  Every partial sum of the factorization and of the solves is then
an integer (or an integer times a power of two) far below 2^24, and every
division and square root is exact, so any summation order gives L0 and the
integer solution exactly, in FP64 and FP32; the GPU must equal the oracle bit
for bit.

Rounded cases (uniform data): both sides are backward stable, each with
||dC|| <= (n + 1) u ||C|| (Higham, Theorem 10.3), so by the perturbation bound
of the Cholesky factor ||dL||_F / ||L||_2 <= kappa_2(C) ||dC||_F / ||C||_2
the two factors differ by at most 4 (n + 1) u kappa_2(C) relative to ||L||_2;
the solutions of L L^t x = b likewise by 8 (n + 1) u kappa_2(C).  kappa_2 is
taken from the oracle's C by a library eigenvalue routine.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_02104_amd as P
    P.load()
    return torch, P


def _say(*a):
    print(*a, flush=True)


def _dev(torch, x, dt):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dt).cuda()


def _kappa(orc, Cp, n):
    ev = np.linalg.eigvalsh(orc.unpack(Cp, n))
    return float(ev[-1] / ev[0])


def _exact_case(orc, n, seed):
    L0 = synthetic.integer_factor(n, seed)
    return orc.pack(L0 @ L0.T), L0  # small integers: exact


@pytest.mark.parametrize("f32", [False, True])
def test_factor_integer_exact(env, orc, f32):
    torch, P = env
    dt = torch.float32 if f32 else torch.float64
    for n in (1, 2, 5, 63, 64, 65, 127, 130, 200, 257):
        _say("case: potrf exact n=%d f32=%s" % (n, f32))
        Cp, L0 = _exact_case(orc, n, 100 + n)
        ref, info_ref = orc.potrf(Cp, n)
        assert info_ref == 0 and np.array_equal(ref, orc.pack(L0))
        C = _dev(torch, Cp, dt)
        info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        P.cholesky(C, n, info=info)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        assert np.array_equal(C.cpu().double().numpy(), ref)


@pytest.mark.parametrize("f32", [False, True])
def test_factor_uniform_within_bound(env, orc, f32):
    torch, P = env
    dt = torch.float32 if f32 else torch.float64
    u = U32 if f32 else U64
    for n in (100, 300, 700):
        _say("case: potrf uniform n=%d f32=%s" % (n, f32))
        A = synthetic.uniform(3 * n + 5, n, 200 + n)
        Cp = orc.classical(A)
        if f32:
            Cp = Cp.astype(np.float32).astype(np.float64)  # the matrix the FP32 path factors
        ref, info = orc.potrf(Cp, n)
        assert info == 0
        C = _dev(torch, Cp, dt)
        P.cholesky(C, n)
        torch.cuda.synchronize()
        got = C.cpu().double().numpy()
        Lr = orc.unpack(ref, n)
        l2 = float(np.linalg.norm(np.tril(Lr), 2))
        err = float(np.linalg.norm(got - ref)) / l2  # packed: each entry once
        tol = 4 * (n + 1) * u * _kappa(orc, Cp, n)
        _say("   rel err %.3e tol %.3e" % (err, tol))
        assert err <= tol


@pytest.mark.parametrize("f32", [False, True])
def test_factor_reports_first_bad_pivot(env, orc, f32):
    torch, P = env
    dt = torch.float32 if f32 else torch.float64
    n = 130
    L0 = synthetic.integer_factor(n, 5)
    for p in (0, 63, 64, 70, 129):
        _say("case: potrf info p=%d f32=%s" % (p, f32))
        Cf = L0 @ L0.T
        Cf[p, p] -= L0[p, p] ** 2 + 1.0  # pivot p becomes exactly -1
        _, info_ref = orc.potrf(orc.pack(Cf), n)
        assert info_ref == p + 1
        C = _dev(torch, orc.pack(Cf), dt)
        info = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
        P.cholesky(C, n, info=info)
        torch.cuda.synchronize()
        assert int(info.item()) == p + 1
        got = C.cpu().double().numpy()
        # rows above p are final and exact
        assert np.array_equal(got[:orc.tri(p)], orc.pack(L0)[:orc.tri(p)])


@pytest.mark.parametrize("f32", [False, True])
def test_solve_integer_exact(env, orc, f32):
    torch, P = env
    dt = torch.float32 if f32 else torch.float64
    for n, r in [(1, 1), (65, 1), (64, 3), (200, 9), (257, 17)]:
        _say("case: potrs exact n=%d nrhs=%d f32=%s" % (n, r, f32))
        Cp, L0 = _exact_case(orc, n, 300 + n)
        X0 = synthetic.integer(n, r, 400 + n)
        Bn = orc.unpack(Cp, n) @ X0  # exact
        ref = orc.potrs(orc.pack(L0), n, Bn)
        assert np.array_equal(ref, X0)
        # row stride wider than nrhs: the extra columns must stay untouched
        Bw = np.full((n, r + 3), 99.0)
        Bw[:, :r] = Bn
        Bt = _dev(torch, Bw, dt)
        P.cholesky_solve(_dev(torch, orc.pack(L0), dt), Bt[:, :r], n)
        torch.cuda.synchronize()
        got = Bt.cpu().double().numpy()
        assert np.array_equal(got[:, :r], ref)
        assert np.all(got[:, r:] == 99.0)


def test_solve_vector_and_uniform(env, orc):
    torch, P = env
    n = 500
    A = synthetic.uniform(1600, n, 21)
    Cp = orc.classical(A)
    Lr, _ = orc.potrf(Cp, n)
    b = synthetic.uniform(n, 1, 22)[:, 0]
    xr = orc.potrs(Lr, n, b)
    _say("case: potrs uniform n=%d" % n)
    bt = _dev(torch, b, torch.float64)
    P.cholesky_solve(_dev(torch, Lr, torch.float64), bt)
    torch.cuda.synchronize()
    x = bt.cpu().numpy()
    err = float(np.linalg.norm(x - xr) / np.linalg.norm(xr))
    tol = 8 * (n + 1) * U64 * _kappa(orc, Cp, n)
    _say("   rel err %.3e tol %.3e" % (err, tol))
    assert err <= tol


@pytest.mark.parametrize("f32", [False, True])
def test_atb_integer_exact(env, orc, f32):
    torch, P = env
    dt = torch.float32 if f32 else torch.float64
    for m, n, r, pad in [(1, 1, 1, 0), (300, 7, 2, 1), (5000, 300, 9, 3), (70000, 3, 1, 0), (0, 5, 2, 0)]:
        _say("case: atb m=%d n=%d nrhs=%d f32=%s" % (m, n, r, f32))
        A = synthetic.integer(m, n, 500 + m)
        Bn = synthetic.integer(m, r, 600 + m)
        ref = orc.atb(A, Bn)
        Ap = np.zeros((m, n + pad))
        Ap[:, :n] = A
        At = _dev(torch, Ap, dt)[:, :n]
        out = P.atb(At, _dev(torch, Bn, dt))
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().double().numpy(), ref)


def test_normal_solve_matches_oracle_chain(env, orc):
    torch, P = env
    m, n, r = 4000, 300, 2
    _say("case: normal_solve m=%d n=%d" % (m, n))
    A = synthetic.uniform(m, n, 31)
    Bn = synthetic.uniform(m, r, 32)
    Cp = orc.classical(A)
    Lr, info = orc.potrf(Cp, n)
    xr = orc.potrs(Lr, n, orc.atb(A, Bn))
    info_t = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    X = P.normal_solve(_dev(torch, A, torch.float64), _dev(torch, Bn, torch.float64), info=info_t)
    torch.cuda.synchronize()
    assert int(info_t.item()) == 0
    err = float(np.linalg.norm(X.cpu().numpy() - xr) / np.linalg.norm(xr))
    # the GPU product itself differs from the oracle's by at most 1e-12
    # relative (the ATA parity bound), which the solve amplifies by kappa
    kap = _kappa(orc, Cp, n)
    tol = (8 * (n + 1) * U64 + 1e-12) * kap
    _say("   rel err %.3e tol %.3e" % (err, tol))
    assert err <= tol


def test_normal_solve_least_squares_shape(env):
    """The least-squares shape at a quarter of its rows (65536 x 2048): the
    solution satisfies the normal equations, A^t (A x - b) ~ 0, to the
    backward error of the chain (checked with torch FP64 products on the
    device, a property that holds at any size)."""
    torch, P = env
    m, n = 65536, 2048
    _say("case: normal_solve least-squares shape %dx%d" % (m, n))
    A = torch.from_numpy(synthetic.uniform(m, n, 41)).cuda()
    b = torch.from_numpy(synthetic.uniform(m, 1, 42)[:, 0].copy()).cuda()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    x = P.normal_solve(A, b, info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    g = A.t().mv(A.mv(x) - b)
    rel = float(g.norm() / (torch.linalg.matrix_norm(A, "fro") ** 2 * x.norm()))
    _say("   normal-equation residual %.3e" % rel)
    assert rel <= 64 * n * U64


def test_normal_solve_on_scaled_columns(env, orc):
    """The chain's default options on the least-squares data recipe (columns
    scaled by 10^U(-3,3)), at 32768 x 256: the product the chain factors
    (gram with default options) keeps the scaled error
    max |dC_ij| / sqrt(C_ii C_jj) at double precision, and the solution
    satisfies the normal equations to the chain's backward error."""
    torch, P = env
    m, n = 32768, 256
    _say("case: normal_solve on scaled columns %dx%d" % (m, n))
    A_np = synthetic.tall_scaled(m, n)
    A = torch.from_numpy(A_np).cuda()
    C = P.gram(A).cpu().numpy()
    ref = orc.classical(A_np)
    sc = orc.scaled_err(C, ref, n)
    _say("   default product scaled error %.3e" % sc)
    assert sc <= 1e-12
    b = torch.from_numpy(synthetic.uniform(m, 1, 43)[:, 0].copy()).cuda()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    x = P.normal_solve(A, b, info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    g = A.t().mv(A.mv(x) - b)
    rel = float(g.norm() / (torch.linalg.matrix_norm(A, "fro") ** 2 * x.norm()))
    _say("   normal-equation residual %.3e" % rel)
    assert rel <= 64 * n * U64


def test_edges(env, orc):
    torch, P = env
    _say("case: normal-equation edges")
    info = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    P.cholesky(torch.zeros(0, dtype=torch.float64, device="cuda"), 0, info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    C = torch.tensor([4.0], dtype=torch.float64, device="cuda")
    P.cholesky(C)
    B = torch.zeros((1, 0), dtype=torch.float64, device="cuda")
    P.cholesky_solve(C, B)
    torch.cuda.synchronize()
    assert float(C.item()) == 2.0
    with pytest.raises(TypeError):
        P.cholesky_solve(C, torch.zeros(1, dtype=torch.float32, device="cuda"))


def test_factor_after_releasing_caches(env, orc):
    """The lookahead stream of the factor is released with the other caches
    and created again on the next call."""
    torch, P = env
    _say("case: potrf around release_caches")
    n = 200
    Cp, L0 = _exact_case(orc, n, 77)
    for _ in range(2):
        C = _dev(torch, Cp, torch.float64)
        P.cholesky(C, n)
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy(), orc.pack(L0))
        P.release_caches()


def test_factor_full_order_of_least_squares_shape(env, orc):
    """The factor at the order of the least-squares shape's product (2048
    columns, 8192 rows here), element by element against the oracle's factor
    of the oracle's product, within the perturbation bound."""
    torch, P = env
    m, n = 8192, 2048
    _say("case: potrf full order n=%d" % n)
    A = synthetic.uniform(m, n, 51)
    Cp = orc.classical_mt(A, threads=16)
    ref, info = orc.potrf(Cp, n)
    assert info == 0
    C = _dev(torch, Cp, torch.float64)
    info_t = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    P.cholesky(C, n, info=info_t)
    torch.cuda.synchronize()
    assert int(info_t.item()) == 0
    got = C.cpu().numpy()
    Lr = orc.unpack(ref, n)
    err = float(np.linalg.norm(got - ref)) / float(np.linalg.norm(np.tril(Lr), 2))
    tol = 4 * (n + 1) * U64 * _kappa(orc, Cp, n)
    _say("   rel err %.3e tol %.3e" % (err, tol))
    assert err <= tol


def test_atb_full_least_squares_size_exact(env):
    """A^t B at the full least-squares shape (262144 x 2048, the launch
    configuration the benchmark times), through properties exact at any size:
    with integer A, B = [e_k, ones] must give row k of A and the column sums
    (checked in int64).  A is drawn on the device from a seeded generator."""
    torch, P = env
    m, n, k = 262144, 2048, 123457
    _say("case: atb full size %dx%d" % (m, n))
    g = torch.Generator(device="cuda")
    g.manual_seed(61)
    Ai = torch.randint(-3, 4, (m, n), generator=g, device="cuda", dtype=torch.int64)
    A = Ai.double()
    B = torch.zeros((m, 2), dtype=torch.float64, device="cuda")
    B[k, 0] = 1.0
    B[:, 1] = 1.0
    out = P.atb(A, B)
    torch.cuda.synchronize()
    assert torch.equal(out[:, 0], A[k])
    assert torch.equal(out[:, 1].long(), Ai.sum(0))


@pytest.mark.parametrize("f32", [False, True])
def test_factor_and_solve_full_order_exact(env, orc, f32):
    """Factor and solve at the full order of the least-squares product (2048),
    on the exactly factorable integer case: bit-exact against the oracle."""
    torch, P = env
    dt = torch.float32 if f32 else torch.float64
    n, r = 2048, 2
    _say("case: potrf + potrs exact n=%d f32=%s" % (n, f32))
    Cp, L0 = _exact_case(orc, n, 71)
    ref, info = orc.potrf(Cp, n)
    assert info == 0 and np.array_equal(ref, orc.pack(L0))
    X0 = synthetic.integer(n, r, 72)
    Bn = orc.unpack(Cp, n) @ X0  # exact
    C = _dev(torch, Cp, dt)
    P.cholesky(C, n)
    B = _dev(torch, Bn, dt)
    P.cholesky_solve(C, B, n)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().double().numpy(), ref)
    assert np.array_equal(B.cpu().double().numpy(), X0)


def test_project_exact_on_orthogonal_columns(env, orc):
    """Hadamard columns: A^t A = 256 I, so the whole chain is exact and the
    projection of A c + z (z orthogonal to the columns) is A c, on both sides."""
    torch, P = env
    _say("case: project exact 256x12")
    H = synthetic.hadamard(256)
    n = 12
    A = np.ascontiguousarray(H[:, :n])
    c = synthetic.integer(n, 2, 91)
    b = A @ c + H[:, n:] @ synthetic.integer(256 - n, 2, 92)
    ref = orc.project(A, b)
    assert np.array_equal(ref, A @ c)
    for dt in (torch.float64, torch.float32):
        out = P.project(_dev(torch, A, dt), _dev(torch, b, dt), cutoff=64)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().double().numpy(), ref)


def test_project_uniform_and_full_shape(env, orc):
    torch, P = env
    m, n = 3000, 200
    _say("case: project uniform %dx%d" % (m, n))
    A = synthetic.uniform(m, n, 93)
    b = synthetic.uniform(m, 1, 94)[:, 0]
    ref = orc.project(A, b)
    got = P.project(_dev(torch, A, torch.float64), _dev(torch, b, torch.float64)).cpu().numpy()
    kap = _kappa(orc, orc.classical(A), n)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    tol = (8 * (n + 1) * U64 + 1e-12) * kap
    _say("   rel err %.3e tol %.3e" % (err, tol))
    assert err <= tol
    # the least-squares shape at a quarter of its rows: the residual b - P b
    # is orthogonal to the columns and P is idempotent (torch FP64 checks)
    m, n = 65536, 2048
    _say("case: project least-squares shape %dx%d" % (m, n))
    At = torch.from_numpy(synthetic.uniform(m, n, 95)).cuda()
    bt = torch.from_numpy(synthetic.uniform(m, 1, 96)[:, 0].copy()).cuda()
    p = P.project(At, bt)
    pp = P.project(At, p)
    torch.cuda.synchronize()
    fro2 = float(torch.linalg.matrix_norm(At, "fro") ** 2)
    assert float(At.t().mv(bt - p).norm()) <= 64 * n * U64 * fro2 * float(bt.norm()) / np.sqrt(fro2)
    assert float((pp - p).norm()) <= 64 * n * U64 * float(p.norm())



def test_normal_solve_f32_within_bound(env, orc):
    """The chain in FP32 throughout (FP32 product, factor, right-hand side and
    solves) against the FP64 oracle chain: the FP32 product's own error (the
    form's 2e-5 bound) and the FP32 solve, both amplified by kappa."""
    torch, P = env
    m, n = 3000, 150
    _say("case: normal_solve f32 %dx%d" % (m, n))
    A = synthetic.uniform(m, n, 97).astype(np.float32).astype(np.float64)
    b = synthetic.uniform(m, 1, 98)[:, 0].astype(np.float32).astype(np.float64)
    Cp = orc.classical(A)
    L, _ = orc.potrf(Cp, n)
    xr = orc.potrs(L, n, orc.atb(A, b))
    info = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    x = P.normal_solve(_dev(torch, A, torch.float32), _dev(torch, b, torch.float32), info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    err = float(np.linalg.norm(x.cpu().double().numpy() - xr) / np.linalg.norm(xr))
    tol = (2e-5 + 8 * (n + 1) * U32) * _kappa(orc, Cp, n)
    _say("   rel err %.3e tol %.3e" % (err, tol))
    assert err <= tol
