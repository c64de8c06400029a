"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each pin is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign or index, a transposed operand, a misprinted Strassen product)
fails at least one of them; test_mutants_are_caught builds such mistakes into
the oracle and checks exactly that.
"""
import ctypes
import itertools
import os

import numpy as np
import pytest

import synthetic

HERE = os.path.dirname(os.path.abspath(__file__))


def _npl_from_paper_equation(l):
    # Section 4.1: npl(0) = 1, npl(1) = 6,
    # npl(l > 1) = 6*4^(l-1) + 2*sum_{k=0}^{l-2} 4^k 7^(l-1-k)
    if l == 0:
        return 1
    if l == 1:
        return 6
    return 6 * 4 ** (l - 1) + 2 * sum(4 ** k * 7 ** (l - 1 - k) for k in range(l - 1))


def _golden_npl():
    rows = []
    with open(os.path.join(HERE, "golden", "npl_counts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                a, b = line.split()
                rows.append((int(a), int(b)))
    return rows


# ---------------------------------------------------------------------------
# Plain definition
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n", [(1, 1), (7, 5), (64, 48), (256, 192), (33, 70)])
def test_classical_matches_library_product(orc, m, n):
    """O1 against numpy's A.T @ A (a BLAS routine) to double rounding."""
    A = synthetic.uniform(m, n, 11 + m + n)
    C = orc.classical(A)
    ref = orc.pack(A.T @ A)
    assert orc.rel_fro(C, ref, n) < 1e-14
    # exact on small integers
    Ai = synthetic.integer(m, n, 3 + m)
    assert np.array_equal(orc.classical(Ai), orc.pack(Ai.T @ Ai))


@pytest.mark.parametrize("m,n,rows,threads", [(100, 97, None, 3), (50, 200, (60, 130), 8),
                                              (1, 5, None, 2), (300, 1, None, 4)])
def test_classical_mt_bitwise_equal(orc, m, n, rows, threads):
    A = synthetic.uniform(m, n, 5)
    full = orc.classical(A)
    part = orc.classical_mt(A, rows=rows, threads=threads)
    i0, i1 = rows or (0, n)
    assert np.array_equal(part, full[orc.tri(i0):orc.tri(i1)])


def test_packed_layout_is_row_major_lower(orc):
    A = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    C = orc.classical(A)
    # C = A^t A = [[17, 22, 27], [22, 29, 36], [27, 36, 45]]
    assert C.tolist() == [17.0, 22.0, 29.0, 27.0, 36.0, 45.0]


def test_lda_padding_is_ignored(orc):
    A = synthetic.integer(40, 30, 9)
    buf = synthetic.with_lda(A, 37)
    view = buf[:, :30]
    assert np.array_equal(orc.classical(view), orc.classical(A))
    C, _ = orc.ata(view, cutoff=4)
    assert np.array_equal(C, orc.classical(A))


# ---------------------------------------------------------------------------
# Algorithm 1 (ATA) against the definition, exactly, on integer inputs
# ---------------------------------------------------------------------------

def test_ata_bruteforce_small_shapes(orc):
    """Every m, n <= 12, cutoff 1..4, both variants, several depth caps:
    all intermediates are small integers, so ATA must equal the definition
    exactly."""
    rng = np.random.default_rng(123)
    for m in range(1, 13):
        for n in range(1, 13):
            A = rng.integers(-3, 4, size=(m, n)).astype(np.float64)
            ref = orc.classical(A)
            for c in (1, 2, 3, 4):
                for var in ("strassen", "winograd"):
                    for md in (-1, 1):
                        C, _ = orc.ata(A, cutoff=c, variant=var, max_depth=md)
                        assert np.array_equal(C, ref), (m, n, c, var, md)


@pytest.mark.parametrize("shape", [(2, 2), (3, 2)])
def test_ata_exhaustive_pm1(orc, shape):
    """All matrices with entries in {-1, 0, 1} of the given shape, cutoff 1."""
    m, n = shape
    for vals in itertools.product((-1.0, 0.0, 1.0), repeat=m * n):
        A = np.array(vals).reshape(m, n)
        for var in ("strassen", "winograd"):
            C, _ = orc.ata(A, cutoff=1, variant=var)
            assert np.array_equal(C, orc.classical(A))


@pytest.mark.parametrize("m,n,c", [(256, 192, 32), (200, 77, 8), (65, 129, 16), (513, 300, 64),
                                   (1000, 40, 8)])
def test_ata_integer_exact_medium(orc, m, n, c):
    A = synthetic.integer(m, n, 1)
    ref = orc.classical(A)
    for var in ("strassen", "winograd"):
        C, cnt = orc.ata(A, cutoff=c, variant=var)
        assert np.array_equal(C, ref)


def test_ata_fp64_error_small(orc):
    """Uniform FP64 input of the 256 x 192 correctness workload: Strassen's
    extra rounding error at two levels stays near double precision."""
    A = synthetic.uniform(256, 192, synthetic.SEED_UNIFORM_SMALL)
    ref = orc.classical(A)
    for var in ("strassen", "winograd"):
        C, _ = orc.ata(A, cutoff=32, variant=var)
        assert orc.rel_fro(C, ref, 192) < 1e-14


# ---------------------------------------------------------------------------
# Structure: multiplication counts
# ---------------------------------------------------------------------------

def test_mult_count_matches_paper_npl(orc):
    """Cutoff 1 on 2^l x 2^l: Algorithm 1 performs npl(l) scalar products
    (golden values printed in Section 4.1; higher l from its equation)."""
    for l, npl in _golden_npl():
        assert orc.ata_mult_count(2 ** l, 2 ** l, 1) == npl
        assert _npl_from_paper_equation(l) == npl
    for l in range(4, 9):
        assert orc.ata_mult_count(2 ** l, 2 ** l, 1) == _npl_from_paper_equation(l)
    # the data-carrying recursion counts the same
    for l in range(0, 6):
        A = synthetic.integer(2 ** l, 2 ** l, l)
        _, cnt = orc.ata(A, cutoff=1)
        assert cnt["mults"] == _npl_from_paper_equation(l)


def test_mult_count_closed_form(orc):
    """T(n) = 4T(n/2) + 2*7^(log2 n - 1) solves to (2*7^l + 4^l)/3, not the
    (2/7) n^log2(7) bound the paper states (Section 3.1)."""
    for l in range(0, 10):
        cnt = orc.ata_mult_count(2 ** l, 2 ** l, 1)
        assert 3 * cnt == 2 * 7 ** l + 4 ** l
        if l >= 2:
            assert cnt > (2.0 / 7.0) * 7 ** l


def test_mult_count_classical_when_cutoff_large(orc):
    for m, n in [(10, 7), (300, 20), (5, 500)]:
        assert orc.ata_mult_count(m, n, 10 ** 6) == m * n * (n + 1) // 2


def test_c1_tree_shape(orc):
    """256 x 192 with cutoff 32: depth 3, 64 base-case leaves of 32 x 24 and
    186 classical HASA leaves of 24 x 32 x 24."""
    A = synthetic.integer(256, 192, 1)
    _, cnt = orc.ata(A, cutoff=32)
    assert cnt["ata_leaves"] == 64
    assert cnt["hasa_leaves"] == 186
    assert cnt["mults"] == 64 * 32 * (24 * 25 // 2) + 186 * 24 * 32 * 24
    assert cnt["mults"] == orc.ata_mult_count(256, 192, 32)


# ---------------------------------------------------------------------------
# HASA / Strassen formulas
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("M,K,N,c", [(4, 4, 4, 1), (7, 5, 9, 1), (16, 16, 16, 2), (33, 17, 21, 3),
                                     (64, 8, 64, 4)])
def test_hasa_equals_product_on_integers(orc, M, K, N, c):
    rng = np.random.default_rng(M * 100 + K)
    X = rng.integers(-4, 5, size=(M, K)).astype(np.float64)
    Y = rng.integers(-4, 5, size=(K, N)).astype(np.float64)
    for var in ("strassen", "winograd"):
        D, cnt = orc.hasa(X, Y, cutoff=c, variant=var)
        assert np.array_equal(D, X @ Y)


def test_printed_products_fail():
    """The HASA-P subsection prints M1 = (A11 + A12)(B11 + B22) and
    M7 = (A11 - A22)(B21 - B22); with the printed quadrant sums they do not
    give A B, while Strassen's M1 = (A11 + A22)(B11 + B22) and
    M7 = (A12 - A22)(B21 + B22) do."""
    rng = np.random.default_rng(0)

    def combine(a, b, printed):
        a11, a12, a21, a22 = a[0, 0], a[0, 1], a[1, 0], a[1, 1]
        b11, b12, b21, b22 = b[0, 0], b[0, 1], b[1, 0], b[1, 1]
        m1 = (a11 + a12) * (b11 + b22) if printed else (a11 + a22) * (b11 + b22)
        m2 = (a21 + a22) * b11
        m3 = a11 * (b12 - b22)
        m4 = a22 * (b21 - b11)
        m5 = (a11 + a12) * b22
        m6 = (a21 - a11) * (b11 + b12)
        m7 = (a11 - a22) * (b21 - b22) if printed else (a12 - a22) * (b21 + b22)
        return np.array([[m1 - m5 + m7 + m4, m3 + m5], [m2 + m4, m3 + m6 - m2 + m1]])

    bad = 0
    for _ in range(20):
        a = rng.integers(-5, 6, size=(2, 2)).astype(float)
        b = rng.integers(-5, 6, size=(2, 2)).astype(float)
        assert np.array_equal(combine(a, b, printed=False), a @ b)
        bad += not np.array_equal(combine(a, b, printed=True), a @ b)
    assert bad >= 18


# ---------------------------------------------------------------------------
# Special cases and invariants
# ---------------------------------------------------------------------------

def test_special_cases(orc):
    a = synthetic.integer(50, 1, 4)
    C, _ = orc.ata(a, cutoff=1)
    assert C.tolist() == [float(np.sum(a * a))]
    r = synthetic.integer(1, 9, 4)
    C, _ = orc.ata(r, cutoff=1)
    assert np.array_equal(C, orc.pack(np.outer(r[0], r[0])))
    I = np.eye(37)
    C, _ = orc.ata(I, cutoff=2)
    assert np.array_equal(C, orc.pack(np.eye(37)))


def test_hadamard_columns(orc):
    """H_256[:, :192] has orthogonal columns of squared norm 256."""
    H = synthetic.hadamard(256)[:, :192].copy()
    for var in ("strassen", "winograd"):
        C, _ = orc.ata(H, cutoff=32, variant=var)
        assert np.array_equal(C, orc.pack(256.0 * np.eye(192)))


def test_invariants(orc):
    A = synthetic.integer(300, 120, 8)
    C, _ = orc.ata(A, cutoff=16)
    n = 120
    diag = np.array([C[orc.tri(i + 1) - 1] for i in range(n)])
    assert np.array_equal(diag, np.sum(A * A, axis=0))
    assert diag.sum() == np.sum(A * A)
    full = orc.unpack(C, n)
    ones = np.ones(n)
    assert ones @ full @ ones == np.sum((A @ ones) ** 2)
    # Freivalds on random data, and positive definiteness
    Au = synthetic.uniform(300, 120, 9)
    Cu, _ = orc.ata(Au, cutoff=16)
    x = np.random.default_rng(1).standard_normal(n)
    assert orc.freivalds_residual(Cu, Au, x) < 1e-14
    np.linalg.cholesky(orc.unpack(Cu, n))


# ---------------------------------------------------------------------------
# The checkers every floating-point parity test goes through: relative
# Frobenius error, scaled error and the Freivalds residual, pinned to values
# worked out by hand, and shown to reject planted mistakes in their source.
# ---------------------------------------------------------------------------

# Packed lower triangle of [[4, 1, 2], [1, 9, 3], [2, 3, 16]]: squared
# Frobenius norm of the full matrix 16 + 81 + 256 + 2 (1 + 4 + 9) = 381.
_REF3 = np.array([4.0, 1.0, 9.0, 2.0, 3.0, 16.0])


def _checker_pins_hold(rel_fro, scaled_err, freivalds_residual):
    """True when all three checkers give the hand-worked values below."""
    ok = True
    d = 0.5
    # one off-diagonal entry (2, 1) off by d: it appears twice in the full matrix
    C = _REF3.copy()
    C[4] += d
    ok &= abs(rel_fro(C, _REF3, 3) - np.sqrt(2 * d * d) / np.sqrt(381.0)) < 1e-15
    # one diagonal entry (1, 1) off by d: it appears once
    C = _REF3.copy()
    C[2] += d
    ok &= abs(rel_fro(C, _REF3, 3) - d / np.sqrt(381.0)) < 1e-15
    ok &= rel_fro(_REF3, _REF3, 3) == 0.0
    # scaled error of (2, 1) is d / sqrt(C_11 C_22) = d / 12, of (1, 0) d / sqrt(4 * 9) = d / 6
    C = _REF3.copy()
    C[4] += d
    ok &= abs(scaled_err(C, _REF3, 3) - d / 12.0) < 1e-15
    C[1] -= 0.25 * d
    ok &= abs(scaled_err(C, _REF3, 3) - d / 12.0) < 1e-15  # 0.125 / 6 < 0.5 / 12
    C[1] -= 0.75 * d
    ok &= abs(scaled_err(C, _REF3, 3) - d / 6.0) < 1e-15
    # Freivalds: A 4 x 3 integer, ||A||_F^2 = 15; x = (1, 2, 2), ||x|| = 3
    A = np.array([[1.0, 2.0, 0.0], [0.0, 1.0, 1.0], [2.0, 0.0, 1.0], [1.0, 1.0, 1.0]])
    x = np.array([1.0, 2.0, 2.0])
    Cp = np.array([6.0, 3.0, 6.0, 3.0, 2.0, 3.0])  # A^t A = [[6, 3, 3], [3, 6, 2], [3, 2, 3]]
    ok &= freivalds_residual(Cp, A, x) == 0.0
    # entry (2, 0) off by 3: (C - A^t A) x = 3 (x_0 e_2 + x_2 e_0), norm 3 sqrt(5)
    Cp[3] += 3.0
    ok &= abs(freivalds_residual(Cp, A, x) - np.sqrt(5.0) / 15.0) < 1e-15
    # a diagonal entry (1, 1) off by 3: (C - A^t A) x = 3 x_1 e_1, norm 6
    Cp[3] -= 3.0
    Cp[2] += 3.0
    ok &= abs(freivalds_residual(Cp, A, x) - 6.0 / 45.0) < 1e-15
    return bool(ok)


def test_checkers_hand_values(orc):
    assert _checker_pins_hold(orc.rel_fro, orc.scaled_err, orc.freivalds_residual)
    # A hand-built packed matrix against numpy's norm of the unpacked difference.
    rng = np.random.default_rng(4)
    ref = rng.standard_normal(orc.tri(40))
    C = ref + 1e-7 * rng.standard_normal(ref.shape)
    want = np.linalg.norm(orc.unpack(C, 40) - orc.unpack(ref, 40)) / np.linalg.norm(orc.unpack(ref, 40))
    assert abs(orc.rel_fro(C, ref, 40) - want) <= 1e-12 * want


CHECKER_MUTANTS = [
    ("rel_fro", "np.full(d.shape, 2.0)", "np.full(d.shape, 1.0)", "off-diagonal entries counted once"),
    ("rel_fro", "w[diag] = 1.0", "w[diag] = 2.0", "diagonal entries counted twice"),
    ("rel_fro", "np.sum(w * ref * ref)", "np.sum(w * C * C)", "normalised by the result, not the reference"),
    ("scaled_err", "ref[tri(i + 1) - 1]", "ref[tri(i)]", "first entry of each row taken as the diagonal"),
    ("scaled_err", "diag[ii] * diag[jj]", "diag[ii] * diag[ii]", "row diagonal used twice"),
    ("freivalds_residual", "lhs = C @ x", "lhs = rhs = A.T @ (A @ x)", "residual that is always zero"),
    ("freivalds_residual", "C = unpack(", "C = np.tril(unpack(", "lower triangle only"),
    ("freivalds_residual", "float(np.linalg.norm(x))", "float(np.sum(x))", "wrong norm of x"),
]


def test_checker_mutants_are_caught(orc):
    """Each planted mistake in a checker's own source breaks a hand-worked pin."""
    import inspect
    import oracle as mod
    for name, old, new, what in CHECKER_MUTANTS:
        src = inspect.getsource(getattr(mod, name))
        assert old in src, (name, old)
        mutated = src.replace(old, new, 1)
        if new.startswith("C = np.tril("):
            mutated = mutated.replace("dtype=np.float64), n)", "dtype=np.float64), n))", 1)
        ns = {"np": np, "tri": mod.tri, "unpack": mod.unpack}
        exec(compile(mutated, "<mutant %s>" % what, "exec"), ns)
        fns = {"rel_fro": mod.rel_fro, "scaled_err": mod.scaled_err,
               "freivalds_residual": mod.freivalds_residual}
        fns[name] = ns[name]
        assert not _checker_pins_hold(**fns), "checker mutant survived: %s" % what


def test_power_of_two_column_scaling_is_exact_for_classical(orc):
    """Classical products commute exactly with power-of-two column scaling:
    (AD)^t (AD) = D (A^t A) D bitwise."""
    A = synthetic.uniform(80, 40, 2)
    d = np.exp2(np.random.default_rng(3).integers(-20, 20, size=40)).astype(np.float64)
    lhs = orc.classical(A * d[None, :])
    full = orc.unpack(orc.classical(A), 40)
    rhs = orc.pack(full * d[:, None] * d[None, :])
    assert np.array_equal(lhs, rhs)


def test_empty_and_degenerate(orc):
    C, _ = orc.ata(np.zeros((0, 5)), cutoff=4)
    assert np.array_equal(C, np.zeros(15))
    C, _ = orc.ata(np.zeros((5, 0)), cutoff=4)
    assert C.size == 0
    with pytest.raises(ValueError):
        orc.ata(np.ones((3, 3)), cutoff=0)


# ---------------------------------------------------------------------------
# Normal-equation consumers: Cholesky factor, triangular solves, A^t b
# ---------------------------------------------------------------------------

def _binom_lower(n):
    """Lower Pascal triangle, L[i][j] = C(i, j)."""
    from math import comb
    return np.array([[comb(i, j) if j <= i else 0 for j in range(n)] for i in range(n)], dtype=np.float64)


def _pascal(n):
    """Symmetric Pascal matrix, P[i][j] = C(i + j, i)."""
    from math import comb
    return np.array([[comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)


def test_potrf_pascal_closed_form(orc):
    # The symmetric Pascal matrix factors as (lower Pascal)(lower Pascal)^t,
    # every intermediate an integer: the factor is exact.
    for n in (1, 2, 7, 20):
        L, info = orc.potrf(orc.pack(_pascal(n)), n)
        assert info == 0
        assert np.array_equal(L, orc.pack(_binom_lower(n)))


def test_potrf_integer_factor_exact(orc):
    for n, seed in [(1, 0), (5, 1), (33, 2), (90, 3)]:
        L0 = synthetic.integer_factor(n, seed)
        L, info = orc.potrf(orc.pack(L0 @ L0.T), n)  # small integers: BLAS exact
        assert info == 0
        assert np.array_equal(L, orc.pack(L0))


def test_potrf_two_by_two_closed_form(orc):
    a, b, c = 3.0, 1.25, 7.5
    L, info = orc.potrf(np.array([a, b, c]), 2)
    l11 = np.sqrt(a)
    expect = np.array([l11, b / l11, np.sqrt(c - (b / l11) ** 2)])
    assert info == 0
    np.testing.assert_allclose(L, expect, rtol=4e-16, atol=0)


def test_potrf_matches_lapack_on_gram(orc):
    A = synthetic.uniform(400, 120, 11)
    C = orc.classical(A)
    L, info = orc.potrf(C, 120)
    ref = np.linalg.cholesky(orc.unpack(C, 120))  # LAPACK dpotrf
    assert info == 0
    np.testing.assert_allclose(orc.unpack(L, 120)[np.tril_indices(120)], ref[np.tril_indices(120)],
                               rtol=1e-12, atol=1e-12 * float(np.max(np.abs(ref))))


def test_potrf_info_names_first_bad_pivot(orc):
    n = 12
    L0 = synthetic.integer_factor(n, 4)
    for p in (0, 5, 11):
        C = L0 @ L0.T
        C[p, p] -= L0[p, p] ** 2 + 1.0  # pivot p becomes exactly -1
        _, info = orc.potrf(orc.pack(C), n)
        assert info == p + 1
    _, info = orc.potrf(orc.pack(np.diag([1.0, 1.0, 0.0, 1.0])), 4)
    assert info == 3


def test_potrs_exact_and_residual(orc):
    for n, r, seed in [(1, 1, 0), (17, 3, 1), (60, 2, 2)]:
        L0 = synthetic.integer_factor(n, seed)
        X0 = synthetic.integer(n, r, seed + 100)
        B = (L0 @ L0.T) @ X0  # small integers: exact
        X = orc.potrs(orc.pack(L0), n, B)
        assert np.array_equal(X, X0)
    A = synthetic.uniform(300, 80, 12)
    C = orc.unpack(orc.classical(A), 80)
    L, _ = orc.potrf(orc.pack(C), 80)
    B = synthetic.uniform(80, 4, 13)
    X = orc.potrs(L, 80, B)
    np.testing.assert_allclose(X, np.linalg.solve(C, B), rtol=1e-10, atol=1e-12)
    assert np.linalg.norm(C @ X - B) <= 1e-13 * np.linalg.norm(C) * np.linalg.norm(X)
    x1 = orc.potrs(L, 80, B[:, 0])
    assert x1.shape == (80,) and np.array_equal(x1, X[:, 0])


def test_atb_definition(orc):
    A = synthetic.integer(70, 23, 5)
    B = synthetic.integer(70, 3, 6)
    assert np.array_equal(orc.atb(A, B), A.T @ B)  # small integers: exact
    assert np.array_equal(orc.atb(A, B[:, 1]), A.T @ B[:, 1])


def test_project_exact_on_orthogonal_columns(orc):
    """Columns of a Hadamard matrix of order 256 are orthogonal with squared
    norm 256: A^t A = 256 I, its factor 16 I, and every step is exact.  The
    projection of A c + z, with z in the span of the other Hadamard columns,
    is exactly A c."""
    H = synthetic.hadamard(256)
    n = 12
    A = np.ascontiguousarray(H[:, :n])
    c = synthetic.integer(n, 2, 81)
    z = H[:, n:] @ synthetic.integer(256 - n, 2, 82)
    P = orc.project(A, A @ c + z)
    assert np.array_equal(P, A @ c)


def test_project_is_idempotent_and_orthogonal(orc):
    A = synthetic.uniform(300, 40, 83)
    b = synthetic.uniform(300, 1, 84)[:, 0]
    p = orc.project(A, b)
    np.testing.assert_allclose(orc.project(A, p), p, rtol=0, atol=1e-12 * np.linalg.norm(p))
    assert np.linalg.norm(A.T @ (b - p)) <= 1e-12 * np.linalg.norm(A) ** 2 * np.linalg.norm(b)
    ref = A @ np.linalg.lstsq(A, b, rcond=None)[0]  # LAPACK least squares
    np.testing.assert_allclose(p, ref, rtol=0, atol=1e-11 * np.linalg.norm(ref))


# ---------------------------------------------------------------------------
# Planted mistakes must be caught
# ---------------------------------------------------------------------------

MUTANTS = {
    1: "second addend of C11 dropped",
    2: "sign of M2 in D22 flipped",
    3: "transposed operand in the C21 product",
    4: "A21 taken at the wrong row offset",
    5: "M1 as misprinted",
    6: "M7 as misprinted",
    7: "Winograd U3 sign flipped",
    8: "first term of the base-case sum dropped",
    9: "first term of the Cholesky sum dropped",
    10: "Cholesky column divided by the wrong diagonal",
    11: "back substitution without the diagonal division",
    12: "first row of A^t b dropped",
}


def _run_pins(lib_path):
    """Return True if every integer-exactness pin passes for the library."""
    import oracle as orc
    lib = ctypes.CDLL(lib_path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.ora_ata.argtypes = [dp, i64, i64, i64, dp, i64, ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(orc.Counts)]
    ok = True
    rng = np.random.default_rng(7)
    for (m, n) in [(9, 8), (12, 12), (17, 10), (40, 33)]:
        A = rng.integers(-3, 4, size=(m, n)).astype(np.float64)
        ref = orc.pack(A.T @ A)  # numpy/BLAS on small integers is exact
        for var in (0, 1):
            C = np.zeros(orc.tri(n))
            cnt = orc.Counts()
            lib.ora_ata(A.ctypes.data_as(dp), m, n, n, C.ctypes.data_as(dp), 2, var, -1,
                        ctypes.byref(cnt))
            ok &= bool(np.array_equal(C, ref))
    # normal-equation consumers: exact integer factor, solve and right-hand side
    lib.ora_potrf.argtypes = [dp, i64]
    lib.ora_potrf.restype = i64
    lib.ora_potrs.argtypes = [dp, i64, dp, i64, i64]
    lib.ora_atb.argtypes = [dp, i64, i64, i64, dp, i64, i64, dp, i64]
    n = 20
    L0 = synthetic.integer_factor(n, 9)
    L = orc.pack(L0 @ L0.T)
    ok &= lib.ora_potrf(L.ctypes.data_as(dp), n) == 0 and bool(np.array_equal(L, orc.pack(L0)))
    X0 = synthetic.integer(n, 2, 10)
    B = np.ascontiguousarray((L0 @ L0.T) @ X0)
    lib.ora_potrs(orc.pack(L0).ctypes.data_as(dp), n, B.ctypes.data_as(dp), 2, 2)
    ok &= bool(np.array_equal(B, X0))
    A = synthetic.integer(30, 7, 11)
    Bv = synthetic.integer(30, 2, 12)
    out = np.zeros((7, 2))
    lib.ora_atb(A.ctypes.data_as(dp), 30, 7, 7, Bv.ctypes.data_as(dp), 2, 2, out.ctypes.data_as(dp), 2)
    ok &= bool(np.array_equal(out, A.T @ Bv))
    return ok


def test_mutants_are_caught(tmp_path):
    from oracle.build import build
    assert _run_pins(build(mutant=0, out=str(tmp_path / "clean.so")))
    for k, what in MUTANTS.items():
        path = build(mutant=k, out=str(tmp_path / ("mut%d.so" % k)))
        assert not _run_pins(path), "mutant %d (%s) survived the pins" % (k, what)


# ---------------------------------------------------------------------------
# Number formats
# ---------------------------------------------------------------------------

def test_bf16_round_matches_torch_cast(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(100000).astype(np.float32) * 10.0 ** rng.uniform(-30, 30, 100000).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0, 3.0e38, -1e-40], dtype=np.float32)])
    x = x[np.isfinite(x)].astype(np.float32)
    ours = orc.bf16_round(x)
    theirs = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    fin = np.isfinite(theirs)
    assert np.array_equal(ours[fin].view(np.uint32), theirs[fin].view(np.uint32))
    hi, lo = orc.bf16_split(x[:1000])
    assert np.all(np.abs((hi.astype(np.float64) + lo) - x[:1000]) <= np.abs(x[:1000]) * 2.0 ** -16 + 1e-45)


def test_e4m3_round_matches_torch_cast(orc):
    torch = pytest.importorskip("torch")
    if not hasattr(torch, "float8_e4m3fn"):
        pytest.skip("no float8 dtype")
    rng = np.random.default_rng(1)
    x = (rng.uniform(-448, 448, 200000) * 10.0 ** rng.uniform(-4, 0, 200000)).astype(np.float32)
    x = np.concatenate([x, np.array([448.0, -448.0, 0.0, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -11, 240.0, 248.0],
                                    dtype=np.float32)])
    ours = orc.e4m3_round(x)
    theirs = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(ours, theirs)
    # saturation (from the format's definition: largest finite value 448)
    assert orc.e4m3_round(np.array([1000.0, -470.0]))[0] == 448.0
    assert orc.e4m3_round(np.array([1000.0, -470.0]))[1] == -448.0


def test_pow2_scales(orc):
    A = np.array([[1.0, -3.0, 0.0], [0.5, 2.0, 0.0]])
    s = orc.pow2_column_scales(A)
    assert s.tolist() == [256.0, 128.0, 1.0]
    assert np.all(np.max(np.abs(A), axis=0) * s <= 448.0)


def test_precision_references_reduce_to_exact(orc):
    """On inputs the formats represent exactly the reduced-precision
    references equal the exact Gram matrix; on uniform data their errors sit
    at the formats' resolution."""
    Ai = synthetic.integer(40, 30, 3).astype(np.float32)  # small integers: bf16 and e4m3 exact
    exact = orc.classical(Ai.astype(np.float64))
    assert np.array_equal(orc.gram_bf16x3(Ai), exact)
    assert np.array_equal(orc.gram_fp8(Ai), exact)
    Au = synthetic.uniform(300, 64, 4).astype(np.float32)
    ex = orc.classical(Au.astype(np.float64))
    e_bf = orc.rel_fro(orc.gram_bf16x3(Au), ex, 64)
    e_f8 = orc.rel_fro(orc.gram_fp8(Au), ex, 64)
    assert 0 < e_bf < 2.0 ** -15
    assert 2.0 ** -8 < e_f8 < 2.0 ** -3


# ---------------------------------------------------------------------------
# Reduced-precision forms with Strassen levels (ata_lowp)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fmt", ["bf16x3", "fp8"])
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_lowp_exact_on_integers(orc, fmt, levels):
    """Small integers and their Strassen operand sums (|x| <= 12) are
    represented exactly by both formats at any power-of-two scale, so the
    reduced-precision recursion gives the exact product."""
    A = synthetic.integer(96, 70, 3).astype(np.float32)
    assert np.array_equal(orc.ata_lowp(A, fmt, 16, levels), orc.classical(A.astype(np.float64)))


def test_lowp_without_levels_is_the_classical_reference(orc):
    """With no Strassen level the recursion only regroups the classical
    product of the converted input (the pinned gram_bf16x3 / gram_fp8)."""
    U = synthetic.uniform(120, 90, 5).astype(np.float32)
    assert orc.rel_fro(orc.ata_lowp(U, "bf16x3", 16, 0), orc.gram_bf16x3(U), 90) < 1e-15
    assert orc.rel_fro(orc.ata_lowp(U, "fp8", 16, 0), orc.gram_fp8(U), 90) < 1e-15


def test_lowp_mutants_are_caught(orc, monkeypatch):
    """A wrong sign in a product or a combination breaks the integer pin."""
    import oracle as mod
    A = synthetic.integer(96, 70, 3).astype(np.float32)
    ex = orc.classical(A.astype(np.float64))
    bad = [list(p) for p in mod._LP_STRASSEN]
    bad[3] = ([(1, 1, 1)], [(1, 1, 0), (1, 0, 0)])  # M4 with Y21 + Y11
    monkeypatch.setattr(mod, "_LP_STRASSEN", [tuple(p) for p in bad])
    assert not np.array_equal(orc.ata_lowp(A, "bf16x3", 16, 1), ex)
    monkeypatch.undo()
    badd = [list(t) for t in mod._LP_STRASSEN_D]
    badd[3] = [(1, 0), (1, 1), (1, 2), (1, 5)]  # D22 with +M2
    monkeypatch.setattr(mod, "_LP_STRASSEN_D", badd)
    assert not np.array_equal(orc.ata_lowp(A, "fp8", 16, 1), ex)
