"""Host-side checks of libata.so that need no GPU: exported symbols, the
planner's structure against the oracle's recursion, argument validation."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1902_02104_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.lib_path()):
        from paper_1902_02104_amd.build import build
        build()
    return P.load()


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "ata.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ata\w*)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert "ata" in names and "ata_ex" in names and len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_status_strings(lib):
    assert P.load().ata_version().decode().count(".") == 2
    assert P.status_string(0) == "ok"
    assert "invalid" in P.status_string(-3)
    assert P.status_string(4) == "workspace too small"


CASES = [
    (256, 192, 32, -1), (256, 192, 32, 0), (256, 192, 32, 1), (256, 192, 32, 2),
    (5000, 5000, 128, 2), (10000, 10000, 256, 2), (10000, 10000, 512, 3), (262144, 2048, 256, 2),
    (513, 600, 256, 2), (517, 301, 40, 3), (65, 129, 16, -1), (7, 5, 1, -1), (12, 12, 2, -1),
    (1, 1, 1, -1), (1, 50, 4, -1), (50, 1, 4, -1), (1025, 513, 256, 2), (8192, 8192, 256, 2),
    (1000, 4096, 256, 2), (65536, 64, 256, 2),
]


@pytest.mark.parametrize("m,n,c,d", CASES)
def test_plan_multiplications_match_oracle_recursion(lib, orc, m, n, c, d):
    """The device plan forms exactly the scalar products of Algorithm 1 with
    HASA (same count as the oracle's literal recursion with the same cutoff
    and Strassen depth cap)."""
    for intile, opsums in ((False, False), (True, False), (False, True)):
        st = P.plan_info(m, n, c, max_depth=d, intile=intile, operand_sums=opsums)
        assert st["mults"] == orc.ata_mult_count(m, n, c, d)
        assert st["classical_mults"] == m * n * (n + 1) // 2


def test_plan_depth_zero_is_classical_count(lib, orc):
    for m, n, c in [(300, 200, 32), (1000, 77, 8)]:
        st = P.plan_info(m, n, c, max_depth=0)
        assert st["mults"] == st["classical_mults"]
        assert st["strassen_tasks"] == 0 and st["combine_tasks"] == 0


def test_plan_large_cutoff_is_one_syrk(lib):
    st = P.plan_info(300, 200, 10 ** 6)
    assert st["syrk_tasks"] == 1 and st["gemm_tasks"] == 0 and st["strassen_tasks"] == 0
    assert st["phases"] == 1 and st["ata_depth"] == 0


def test_plan_non_uniform_tree_uses_ordered_phases(lib, orc):
    # 513 rows straddle the cutoff 256 (257 recurses, 256 stops)
    st = P.plan_info(513, 600, 256, max_depth=2)
    assert st["phases"] == 2
    assert st["mults"] == orc.ata_mult_count(513, 600, 256, 2)


def test_winograd_depth_limits(lib, orc):
    for intile in (False, True):
        st = P.plan_info(2048, 2048, 64, variant="winograd", max_depth=2, intile=intile)
        assert st["mults"] == orc.ata_mult_count(2048, 2048, 64, 2)
    with pytest.raises(P.AtaError):
        P.plan_info(4096, 4096, 64, variant="winograd", max_depth=3)  # 16 operand terms


def test_workspace_size(lib):
    # in-tile form: one-level blocks write C directly; two-level blocks keep
    # the 7 products of their first level, each a quarter block
    assert P.workspace_bytes(256, 192, 32, max_depth=1, intile=True) == 0
    ws = P.workspace_bytes(10000, 10000, 256, max_depth=2, intile=True)
    expect = 8 * 7 * (2500 ** 2 + 2 * 1250 ** 2 + 4 * 625 ** 2 + 8 * 313 ** 2)
    assert expect <= ws < expect + 256  # rounded up to 256-byte alignment
    # product tiles: a block of d levels keeps all 7^d products, each of the
    # block's size halved (ceil) d times.  Off-diagonal blocks of 10000^2 at
    # cutoff 256: 5000^2, 2 x 2500^2, 4 x 1250^2, 8 x 625^2 (two levels each)
    # and 16 x (312 x 313) (one level; K = 625 rows)
    ws = P.workspace_bytes(10000, 10000, 256, max_depth=2, intile=False)
    expect = 8 * (49 * 1250 ** 2 + 2 * 49 * 625 ** 2 + 4 * 49 * 313 ** 2 + 8 * 49 * 157 ** 2 + 16 * 7 * 156 * 157)
    assert expect <= ws < expect + 256
    ws1 = P.workspace_bytes(256, 192, 32, max_depth=1, intile=False)
    assert ws1 > 0


def test_workspace_size_reduced_precision(lib):
    m, n = 1000, 300
    ldt = (m + 127) // 128 * 128
    bf = P.workspace_bytes(m, n, 0, dtype=P.F32_BF16X3, max_depth=0)
    f8 = P.workspace_bytes(m, n, 0, dtype=P.F32_FP8, max_depth=0)
    assert bf >= 2 * n * ldt * 2 + n * 4
    assert f8 >= n * ldt + n * 4 and f8 < bf
    # Strassen levels add the converted operand copy of the products
    assert P.workspace_bytes(m, n, 0, dtype=P.F32_FP8, max_depth=1) > f8
    with pytest.raises(P.AtaError):
        P.plan_info(m, n, 0, dtype=P.F32_FP8, max_depth=3)  # at most two expanded levels


def test_split_last_round_workspace(lib):
    """A single classical launch of more than one round (512 resident
    workgroups for FP64 and FP32 tiles, 256 for bfloat16 pairs) splits the K
    range of its last r tiles: into min(slots / r, K / 128) parts when r is
    at most half the slots, else into the smallest part count of at most 8
    that comes within 0.05 tile times of the best and saves a fifth of a tile
    time.  The workspace holds their FP64 partial tiles.  One round, or parts
    below two, splits nothing."""
    tile = 128 * 128 * 8
    for dt in (P.F64, P.F32, P.F32 | P.OUT_F64):
        assert P.workspace_bytes(1000, 4000, 256, dtype=dt, max_depth=0) == 16 * 7 * tile  # 528 tiles
        assert P.workspace_bytes(1000, 4200, 256, dtype=dt, max_depth=0) == 49 * 7 * tile  # 561 tiles
        assert P.workspace_bytes(1000, 3000, 256, dtype=dt, max_depth=0) == 0  # 300 tiles: one round
        assert P.workspace_bytes(100, 4000, 256, dtype=dt, max_depth=0) == 0  # 100 rows: one part
        # 820 tiles: the last 308 in 3 parts (two rounds of parts, 2/3 of a tile time instead of one)
        assert P.workspace_bytes(5000, 5000, 512, dtype=dt, max_depth=0) == 308 * 3 * tile
        # 990 tiles: 478 left, no part count up to 8 saves a fifth of a tile time; nor is K split as a whole
        assert P.workspace_bytes(5632, 5632, 512, dtype=dt, max_depth=0) == 0
    conv = lambda n: 2 * n * 1024 * 2 + n * 4  # bfloat16 hi and lo copies, rows padded to 1024
    bf = P.workspace_bytes(1000, 3000, 256, dtype=P.F32_BF16X3, max_depth=0)
    assert 44 * 5 * tile <= bf - conv(3000) < 44 * 5 * tile + 65536  # 300 tiles: 256 + 44 in 5 parts
    assert P.workspace_bytes(1000, 2000, 256, dtype=P.F32_BF16X3, max_depth=0) - conv(2000) < 65536  # 136 tiles


def test_split_k_part_counts(lib):
    """K splitting of launches with few tiles.  Classical tiles alone (FP64,
    FP32): the fewest parts whose rounds of the 512 resident workgroups come
    within half a percent of the best count, here 136 tiles x 15 parts = 2040
    (3.98 rounds; 45 parts would give 11.95).  Phases with Strassen product
    tiles keep the largest count allowed (6144 items targeted: 45 parts)."""
    for dt in (P.F64, P.F32):
        st = P.plan_info(262144, 2048, 256, dtype=dt, max_depth=0)
        assert st["work_items"] == 136 * 15 and st["combine_tasks"] == 1, st
    st = P.plan_info(262144, 2048, 256, dtype=P.F64, max_depth=1)
    assert st["work_items"] == 6120, st


def test_lp_staging_paths(lib):
    """Staging of the reduced-precision tiles from the plan's K windows: 16
    bytes of the copy per window start and end (8 bfloat16 pairs, 16 e4m3),
    where a window ending at the last row counts as aligned (zeros follow in
    the copy); else dwords (2 and 4 elements); else registers.  One Strassen
    level splits the rows at ceil(m/2); other dtypes report -1."""
    cases = {(2048, 1): (2, 2), (2047, 1): (2, 2), (2047, 0): (2, 2), (2044, 1): (1, 0), (2040, 1): (1, 1),
             (2041, 1): (0, 0), (4104, 1): (1, 1)}
    for (m, d), want in cases.items():
        got = tuple(P.plan_info(m, 130, 64, dtype=dt, max_depth=d)["lp_staging"] for dt in (P.F32_BF16X3, P.F32_FP8))
        assert got == want, (m, d, got)
    assert P.plan_info(2048, 130, 64, dtype=P.F64)["lp_staging"] == -1
    assert P.plan_info(2048, 130, 64, dtype=P.F32)["lp_staging"] == -1


def test_default_cutoff_is_in_tuned_set(lib):
    for m, n in [(256, 192), (5000, 5000), (10000, 10000), (262144, 2048)]:
        assert P.default_cutoff(m, n) in (128, 256, 512)


def test_argument_validation_without_gpu(lib):
    """Bad arguments are rejected before any device call (LAPACK-style codes)."""
    L = P.load()
    vp = ctypes.c_void_p
    buf = (ctypes.c_double * 64)()
    a = ctypes.cast(buf, vp)
    assert L.ata(a, -1, 4, 4, a, P.F64, 0, None) == -2
    assert L.ata(a, 4, -1, 4, a, P.F64, 0, None) == -3
    assert L.ata(a, 4, 4, 3, a, P.F64, 0, None) == -4
    assert L.ata(a, 4, 4, 4, None, P.F64, 0, None) == -5
    assert L.ata(None, 4, 4, 4, a, P.F64, 0, None) == -1
    assert L.ata(a, 4, 4, 4, a, 7, 0, None) == -6
    assert L.ata(a, 4, 4, 4, a, P.F64 | P.OUT_F64, 0, None) == -6
    assert L.ata(a, 4, 4, 4, a, P.F64, -5, None) == -7
    mis = ctypes.c_void_p(ctypes.addressof(buf) + 4)
    assert L.ata(mis, 4, 4, 4, a, P.F64, 0, None) == -1
    o = P.Opts()
    o.variant, o.max_depth, o.flags = 5, 2, 0
    assert L.ata_ex(a, 4, 4, 4, a, P.F64, 0, None, ctypes.byref(o), None, 0) == -9
    o.variant, o.max_depth = 0, -2
    assert L.ata_ex(a, 4, 4, 4, a, P.F64, 0, None, ctypes.byref(o), None, 0) == -9


def test_binding_refuses_host_tensors(lib):
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        P.gram(torch.zeros(4, 4, dtype=torch.float64))


def test_equilibration_workspace_and_options(lib):
    m, n = 1000, 300
    base = P.workspace_bytes(m, n, 64, max_depth=1)
    eq = P.workspace_bytes(m, n, 64, max_depth=1, equilibrate=True)
    # scales + per-256-row partial maxima + the scaled copy of A
    assert eq - base >= 8 * (n + 4 * n + m * n)
    assert eq - base < 8 * (n + 4 * n + m * n) + 3 * 256
    eq32 = P.workspace_bytes(m, n, 64, dtype=P.F32, max_depth=1, equilibrate=True)
    assert eq32 - P.workspace_bytes(m, n, 64, dtype=P.F32, max_depth=1) >= 4 * (n + 4 * n + m * n)
    with pytest.raises(P.AtaError):  # the reduced-precision forms scale columns themselves
        P.plan_info(m, n, 64, dtype=P.F32_FP8, equilibrate=True)
    o = P.Opts()
    o.flags = 0x100  # unknown flag
    st = P.PlanStats()
    assert lib.ata_plan_info(m, n, P.F64, 64, ctypes.byref(o), ctypes.byref(st)) != 0


def test_release_caches_without_device(lib):
    """Host-only plans (plan_info) are dropped and rebuilt identically."""
    before = P.plan_info(777, 333, 40, max_depth=2)
    P.release_caches()
    assert P.plan_info(777, 333, 40, max_depth=2) == before


def test_normal_equation_argument_validation_without_gpu(lib):
    """The factor, solve and A^t B entry points reject bad arguments before
    any device call, with the LAPACK-style position codes of ata.h."""
    L = P.load()
    vp = ctypes.c_void_p
    buf = (ctypes.c_double * 64)()
    a = ctypes.cast(buf, vp)
    assert L.ata_potrf(a, -1, P.F64, None, None) == -2
    assert L.ata_potrf(None, 4, P.F64, None, None) == -1
    assert L.ata_potrf(a, 4, P.F32_FP8, None, None) == -3
    assert L.ata_potrf(a, 4, P.F64 | P.OUT_F64, None, None) == -3
    assert L.ata_potrs(a, -1, a, 1, 1, P.F64, None) == -2
    assert L.ata_potrs(a, 4, a, -1, 1, P.F64, None) == -4
    assert L.ata_potrs(None, 4, a, 1, 1, P.F64, None) == -1
    assert L.ata_potrs(a, 4, None, 1, 1, P.F64, None) == -3
    assert L.ata_potrs(a, 4, a, 3, 2, P.F64, None) == -5
    assert L.ata_potrs(a, 4, a, 1, 1, 9, None) == -6
    assert L.ata_atb(a, -1, 4, 4, a, 1, 1, a, 1, P.F64, None) == -2
    assert L.ata_atb(a, 4, -1, 4, a, 1, 1, a, 1, P.F64, None) == -3
    assert L.ata_atb(a, 4, 4, 3, a, 1, 1, a, 1, P.F64, None) == -4
    assert L.ata_atb(None, 4, 4, 4, a, 1, 1, a, 1, P.F64, None) == -1
    assert L.ata_atb(a, 4, 4, 4, None, 1, 1, a, 1, P.F64, None) == -5
    assert L.ata_atb(a, 4, 4, 4, a, -1, 1, a, 1, P.F64, None) == -6
    assert L.ata_atb(a, 4, 4, 4, a, 2, 1, a, 2, P.F64, None) == -7
    assert L.ata_atb(a, 4, 4, 4, a, 1, 1, None, 1, P.F64, None) == -8
    assert L.ata_atb(a, 4, 4, 4, a, 2, 2, a, 1, P.F64, None) == -9
    assert L.ata_atb(a, 4, 4, 4, a, 1, 1, a, 1, P.F32_BF16X3, None) == -10
    assert L.ata_normal_solve(a, 4, 4, 4, a, 1, 1, a, 1, P.F64, -1, None, None) == -11
    assert L.ata_normal_solve(a, 4, 4, 4, a, 1, 1, None, 1, P.F64, 0, None, None) == -8
    assert L.ata_potrf(a, (1 << 22) + 1, P.F64, None, None) == 3  # ATA_EUNSUPPORTED
    mis = ctypes.c_void_p(ctypes.addressof(buf) + 4)
    assert L.ata_potrf(mis, 4, P.F64, None, None) == -1
    assert L.ata_potrf(a, 4, P.F64, ctypes.c_void_p(ctypes.addressof(buf) + 2), None) == -4
    assert L.ata_potrs(a, 4, mis, 1, 1, P.F64, None) == -3
    assert L.ata_atb(a, 4, 4, 4, a, 1, 1, mis, 1, P.F64, None) == -8
    assert L.ata_normal_solve(mis, 4, 4, 4, a, 1, 1, a, 1, P.F64, 0, None, None) == -1


def test_aat_argument_validation_without_gpu(lib):
    L = P.load()
    vp = ctypes.c_void_p
    buf = (ctypes.c_double * 64)()
    a = ctypes.cast(buf, vp)
    assert L.ata_aat(a, -1, 4, 4, a, P.F64, 0, None) == -2
    assert L.ata_aat(a, 4, -1, 4, a, P.F64, 0, None) == -3
    assert L.ata_aat(a, 4, 4, 3, a, P.F64, 0, None) == -4
    assert L.ata_aat(None, 4, 4, 4, a, P.F64, 0, None) == -1
    assert L.ata_aat(a, 4, 4, 4, None, P.F64, 0, None) == -5
    assert L.ata_aat(a, 4, 4, 4, a, 7, 0, None) == -6
    assert L.ata_aat(a, 4, 4, 4, a, P.F64, -1, None) == -7
    mis = ctypes.c_void_p(ctypes.addressof(buf) + 4)
    assert L.ata_aat(mis, 4, 4, 4, a, P.F64, 0, None) == -1


def test_project_argument_validation_without_gpu(lib):
    L = P.load()
    vp = ctypes.c_void_p
    buf = (ctypes.c_double * 64)()
    a = ctypes.cast(buf, vp)
    assert L.ata_project(a, -1, 4, 4, a, 1, 1, a, 1, P.F64, 0, None, None) == -2
    assert L.ata_project(a, 4, 4, 3, a, 1, 1, a, 1, P.F64, 0, None, None) == -4
    assert L.ata_project(a, 4, 4, 4, None, 1, 1, a, 1, P.F64, 0, None, None) == -5
    assert L.ata_project(a, 4, 4, 4, a, 1, 1, None, 1, P.F64, 0, None, None) == -8
    assert L.ata_project(a, 4, 4, 4, a, 2, 2, a, 1, P.F64, 0, None, None) == -9
    assert L.ata_project(a, 4, 4, 4, a, 1, 1, a, 1, P.F32_FP8, 0, None, None) == -10
    assert L.ata_project(a, 4, 4, 4, a, 1, 1, a, 1, P.F64, -1, None, None) == -11



def test_plan_cache_is_bounded_and_rebuilds():
    """Many distinct shapes (as a serving stream draws them) pass through the
    bounded plan cache; an evicted plan is rebuilt identically."""
    import paper_1902_02104_amd as P
    first = P.plan_info(700, 300, 64, max_depth=1)
    for i in range(600):
        P.plan_info(500 + i, 120 + (i % 37), 64, max_depth=1)
    again = P.plan_info(700, 300, 64, max_depth=1)
    assert again == first
