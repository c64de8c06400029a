// Consumers of the packed product on gfx950: the Cholesky factor of the
// packed lower C, the two triangular solves with it, the right-hand side A^t b
// of the normal equations and the product A X that applies the projection
// A (A^t A)^-1 A^t (Section 1 names both as uses of A^t A); and the transpose
// that gives the companion product A A^t.
//
// Storage: row-major packed lower triangle, element (i, j), j <= i, at
// i (i + 1) / 2 + j, so a row's entries left of the diagonal are contiguous.
// The factorization is right-looking over 64-column blocks: per block, one
// launch factors the diagonal block, one solves the rows below it, and one
// MFMA launch applies the rank-64 update to the trailing lower triangle.  The
// solves take one launch per 64-row block in each direction.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ata.h"
#include "ata_internal.h"
#include "ata_kernels.h"

namespace atalib {

namespace {

using detail::ProfScope;

constexpr int NB = 64;  // block width of the factorization and the solves

typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t pidx(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }

// Value of v in lane src (uniform) for every lane, through scalar registers.
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float lane_bcast(float v, int src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}

// Orders the LDS accesses of one wave (no instruction needed: a wave's LDS
// operations complete in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// ---------------------------------------------------------------------------
// Diagonal block of the factorization at block column kb (width w <= 64), one
// workgroup, in place.  Thread t owns column l = t & 63 and rows
// i = (t >> 6) + 4 q (q < 16) of the block, and keeps a running copy of its
// column's diagonal entry (updated by the same operation as the entry
// itself), so the owners of step j take the pivot from their own copy.
// Step j: the owners publish column j and 1 / pivot in LDS; after one
// barrier every thread scales the entries it reads by 1 / pivot (as LAPACK's
// unblocked factor scales the column) and applies the rank-one update to its
// entries with selects.  A finished column is scaled when it is stored.  The column buffer
// alternates between two halves by step parity: the barrier of step j + 1
// separates the reads of step j from the writes of step j + 2.  A pivot that
// is not positive is reported once through `info` (first failing column + 1,
// LAPACK's convention); the factorization carries on with the resulting NaNs.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_chol_diag(T* __restrict__ C, int64_t kb, int w, int32_t* __restrict__ info) {
    __shared__ T col[2][NB];
    __shared__ T rps[2];
    // on the critical path while the helper stream's update fills the CUs:
    // raise this wave's issue priority on its SIMD
    __builtin_amdgcn_s_setprio(3);
    const int t = threadIdx.x, l = t & 63, wv = t >> 6;
    T d[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = wv + 4 * q;
        d[q] = (i < w && l <= i) ? C[pidx(kb + i, kb + l)] : T(0);
    }
    T dd = l < w ? C[pidx(kb + l, kb + l)] : T(1);
    T myrp = T(1), mypiv = T(0);  // this thread's column: 1 / pivot and pivot
    for (int j = 0; j < w; ++j) {
        T* cb = col[j & 1];
        if (l == j) {
            // the owners publish column j unscaled with 1 / pivot; each reader
            // forms the scaled entries it needs (the same products), and a
            // column is scaled in place only when it is stored
            mypiv = sqrt(dd);
            myrp = T(1) / mypiv;
            if (wv == 0 && !(dd > T(0)) && info) atomicCAS(info, 0, (int32_t)(kb + j + 1));
#pragma unroll
            for (int q = 0; q < 16; ++q) cb[wv + 4 * q] = d[q];
            if (wv == 0) rps[j & 1] = myrp;
        }
        __syncthreads();
        const bool act = l > j && l < w;
        const T rpj = rps[j & 1];
        const T lj = cb[l] * rpj;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int i = wv + 4 * q;
            const T v = d[q] - (cb[i] * rpj) * lj;
            d[q] = (act && i >= l) ? v : d[q];
        }
        if (act) dd -= lj * lj;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = wv + 4 * q;
        if (i < w && l <= i) C[pidx(kb + i, kb + l)] = i > l ? d[q] * myrp : (i == l ? mypiv : d[q]);
    }
}

// ---------------------------------------------------------------------------
// Rows below the diagonal block: L21 = C21 L11^-t for rows
// R0 = kb + w + 64 b ... R0 + 63 (workgroup b), with the factored L11 staged
// in LDS.  Thread t owns column l = t & 63 and rows i = (t >> 6) + 4 q; each
// step scales column j (times the staged 1 / L11[j][j]) and subtracts its
// multiples from the later columns, the order the diagonal block uses.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_chol_rows(T* __restrict__ C, int64_t n, int64_t kb, int w) {
    __shared__ T ld[NB * (NB + 1)];
    __shared__ T col[NB];
    __shared__ T rcp[NB];
    __builtin_amdgcn_s_setprio(3);  // critical path, as in k_chol_diag
    const int t = threadIdx.x, l = t & 63, wv = t >> 6;
    const int64_t R0 = kb + w + (int64_t)NB * blockIdx.x;
    for (int e = t; e < NB * NB; e += 256) {
        const int row = e >> 6, c = e & 63;
        ld[row * (NB + 1) + c] = (row < w && c <= row) ? C[pidx(kb + row, kb + c)] : T(0);
    }
    if (t < w) rcp[t] = T(1) / C[pidx(kb + t, kb + t)];
    T r[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = wv + 4 * q;
        r[q] = (R0 + i < n && l < w) ? C[pidx(R0 + i, kb + l)] : T(0);
    }
    __syncthreads();
    // The rows of a wave (i = wv + 4 q) depend only on each other and on L11,
    // and the column entries col[wv + 4 q] are written and read by that wave
    // alone: the steps need wave-level ordering only.
    // The owner lane publishes its column unscaled; readers scale by the
    // staged 1 / L11[j][j] (the same products), and a column is scaled when
    // it is stored.
    for (int j = 0; j < w; ++j) {
        if (l == j) {
#pragma unroll
            for (int q = 0; q < 16; ++q) col[wv + 4 * q] = r[q];
        }
        wave_lds_fence();
        if (l > j && l < w) {
            const T lj = ld[l * (NB + 1) + j];
            const T rj = rcp[j];
#pragma unroll
            for (int q = 0; q < 16; ++q) r[q] -= (col[wv + 4 * q] * rj) * lj;
        }
        wave_lds_fence();
    }
    const T rl = l < w ? rcp[l] : T(0);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = wv + 4 * q;
        if (R0 + i < n && l < w) C[pidx(R0 + i, kb + l)] = r[q] * rl;
    }
}

// ---------------------------------------------------------------------------
// Trailing update: C[i][j] -= sum_{k < w} L[i][kb + k] L[j][kb + k] for
// s <= j <= i < n, s = kb + w, over the 64 x 64 tiles (ti, tj), tj <= ti, of
// the trailing lower triangle.  part 0 takes every tile, part 1 only the
// first tile column (tj = 0: the next diagonal block and the rows below it),
// part 2 the others; the tile comes from the linear workgroup index.  Each
// wave first loads its quarter of the C tile (those loads complete under the
// staging and the MFMAs), then both panel slices are staged transposed in
// LDS ([k][row], row stride 68: 4 mod 16 doubles, so the broadcast operand
// reads of the FP64 form fall on distinct banks) and four waves each form a
// 32 x 32 quarter on MFMA; on a diagonal tile the quarter above the diagonal
// is skipped.
//   FP64: v_mfma_f64_4x4x4f64 with the left operand broadcast to the four
//         blocks, a 4 x 16 x 4 product: left lane l = X[row l & 3][k l >> 4],
//         right lane l = Y[k l >> 4][col l & 15], result lane l =
//         D[row l >> 4][col l & 15].
//   FP32: v_mfma_f32_16x16x4f32: left lane l = X[row l & 15][k l >> 4],
//         right as above, result element e of lane l = D[row 4 (l >> 4) + e]
//         [col l & 15].
// ---------------------------------------------------------------------------
constexpr int UP = NB + 4;

// Row a and column c of linear index b in a lower triangle of tiles.
__device__ __forceinline__ void tri_decode(int64_t b, int64_t& a, int64_t& c) {
    a = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (a * (a + 1) / 2 > b) --a;
    while ((a + 1) * (a + 2) / 2 <= b) ++a;
    c = b - a * (a + 1) / 2;
}

template <typename T>
__global__ __launch_bounds__(256, 2) void k_chol_update(T* __restrict__ C, int64_t n, int64_t kb, int w, int tiles,
                                                        int part) {
    __shared__ T Pi[NB * UP];
    __shared__ T Pj[NB * UP];
    int64_t ti, tj;
    if (part == 1) {
        ti = blockIdx.x;
        tj = 0;
    } else if (part == 2) {
        tri_decode(blockIdx.x, ti, tj);
        ++ti;
        ++tj;
    } else {
        tri_decode(blockIdx.x, ti, tj);
    }
    if (ti >= tiles) return;
    const int64_t s = kb + w;
    const int64_t r0 = s + NB * ti, c0 = s + NB * tj;
    const bool diag = ti == tj;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wr = wv >> 1, wc = wv & 1;
    const bool active = !(diag && wr < wc);
    // C values of this wave's quarter, in the result layout of the MFMA form
    constexpr int NV = 16;
    T cv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        int64_t i, j;
        if constexpr (sizeof(T) == 8) {
            i = r0 + 32 * wr + 4 * (v >> 1) + (lane >> 4);
            j = c0 + 32 * wc + 16 * (v & 1) + (lane & 15);
        } else {
            i = r0 + 32 * wr + 16 * (v >> 3) + 4 * (lane >> 4) + (v & 3);
            j = c0 + 32 * wc + 16 * ((v >> 2) & 1) + (lane & 15);
        }
        cv[v] = (active && i < n && j <= i) ? C[pidx(i, j)] : T(0);
    }
    // panel slices: all 32 loads of a thread in flight before the LDS stores
    // (row (t >> 6) + 4 u, k = lane: one 512-byte row segment per wave load)
    T pv[16], qv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int row = (t >> 6) + 4 * u;
        const int64_t gi = r0 + row, gj = c0 + row;
        pv[u] = (gi < n && lane < w) ? C[pidx(gi, kb + lane)] : T(0);
        qv[u] = (!diag && gj < n && lane < w) ? C[pidx(gj, kb + lane)] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int row = (t >> 6) + 4 * u;
        Pi[lane * UP + row] = pv[u];
        if (!diag) Pj[lane * UP + row] = qv[u];
    }
    __syncthreads();
    if (!active) return;
    const T* Y = diag ? Pi : Pj;
    if constexpr (sizeof(T) == 8) {
        double acc[8][2];
#pragma unroll
        for (int g = 0; g < 8; ++g) acc[g][0] = acc[g][1] = 0.0;
        for (int k0 = 0; k0 < NB; k0 += 4) {
            const int kr = (k0 + (lane >> 4)) * UP;
            double a[8], bb[2];
#pragma unroll
            for (int g = 0; g < 8; ++g) a[g] = Pi[kr + 32 * wr + 4 * g + (lane & 3)];
#pragma unroll
            for (int h = 0; h < 2; ++h) bb[h] = Y[kr + 32 * wc + 16 * h + (lane & 15)];
#pragma unroll
            for (int g = 0; g < 8; ++g)
#pragma unroll
                for (int h = 0; h < 2; ++h) acc[g][h] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[g], bb[h], acc[g][h], 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int64_t i = r0 + 32 * wr + 4 * (v >> 1) + (lane >> 4);
            const int64_t j = c0 + 32 * wc + 16 * (v & 1) + (lane & 15);
            if (i < n && j <= i) C[pidx(i, j)] = cv[v] - acc[v >> 1][v & 1];
        }
    } else {
        f4_t acc[2][2];
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int h = 0; h < 2; ++h) acc[g][h] = f4_t{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < NB; k0 += 4) {
            const int kr = (k0 + (lane >> 4)) * UP;
            float a[2], bb[2];
#pragma unroll
            for (int g = 0; g < 2; ++g) a[g] = Pi[kr + 32 * wr + 16 * g + (lane & 15)];
#pragma unroll
            for (int h = 0; h < 2; ++h) bb[h] = Y[kr + 32 * wc + 16 * h + (lane & 15)];
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int h = 0; h < 2; ++h) acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[g], bb[h], acc[g][h], 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int64_t i = r0 + 32 * wr + 16 * (v >> 3) + 4 * (lane >> 4) + (v & 3);
            const int64_t j = c0 + 32 * wc + 16 * ((v >> 2) & 1) + (lane & 15);
            if (i < n && j <= i) C[pidx(i, j)] = cv[v] - acc[v >> 3][(v >> 2) & 1][v & 3];
        }
    }
}

// Sum of v over the 64 lanes of the wave (every lane receives it).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int RC = 8;  // right-hand sides per pass of the solve updates

// Stage the diagonal block d (width wd) of L in LDS, row stride NB + 1, with
// the reciprocal of each diagonal entry in place of the entry.
template <typename T>
__device__ void stage_diag(const T* __restrict__ L, int64_t d0, int wd, T* ld) {
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int row = e >> 6, c = e & 63;
        const T v = (row < wd && c <= row) ? L[pidx(d0 + row, d0 + c)] : T(0);
        ld[row * (NB + 1) + c] = (c == row && row < wd) ? T(1) / v : v;
    }
}

// ---------------------------------------------------------------------------
// Forward substitution L Y = B, one launch per block (B row-major n x nrhs,
// row stride ldb, overwritten by Y).  Launch k = -1 solves diagonal block 0.
// Launch k >= 0 (block k already solved): workgroup b subtracts
// L[block k+1+b rows][block k] Y_k from its 64 rows (one wave per row at a
// time, lane = column of block k, wave-wide sums); workgroup 0 then solves
// diagonal block k+1 with wave 0 (lane = row; column by column, each solved
// value broadcast from its lane through scalar registers and scaled by the
// staged reciprocal of the diagonal entry).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_fwd(const T* __restrict__ L, int64_t n, T* __restrict__ B, int64_t nrhs,
                                                  int64_t ldb, int64_t k) {
    __shared__ T ld[NB * (NB + 1)];
    __shared__ T ys[NB * RC];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t tb = k + 1 + blockIdx.x;  // target block
    const int64_t t0 = NB * tb;
    if (k >= 0) {
        const int64_t y0 = NB * k;
        // this wave's 16 rows of L[.][block k], all loads in flight at once
        T lv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int64_t i = t0 + wv + 4 * u;
            lv[u] = i < n ? L[pidx(i, y0 + lane)] : T(0);
        }
        for (int64_t r0 = 0; r0 < nrhs; r0 += RC) {
            const int rc = (int)(nrhs - r0 < RC ? nrhs - r0 : RC);
            __syncthreads();
            for (int e = t; e < NB * RC; e += 256) {
                const int c = e / RC, rr = e % RC;
                ys[e] = rr < rc ? B[(y0 + c) * ldb + r0 + rr] : T(0);
            }
            __syncthreads();
            for (int rr = 0; rr < rc; ++rr) {
                const T y = ys[lane * RC + rr];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int64_t i = t0 + wv + 4 * u;
                    const T s = wave_sum(lv[u] * y);
                    if (lane == 0 && i < n) B[i * ldb + r0 + rr] -= s;
                }
            }
        }
    }
    if (blockIdx.x != 0) return;
    const int wd = (int)(n - t0 < NB ? n - t0 : NB);
    __syncthreads();  // the rows just updated are read below
    stage_diag(L, t0, wd, ld);
    __syncthreads();
    if (wv != 0) return;
    for (int64_t r = 0; r < nrhs; ++r) {
        T x = lane < wd ? B[(t0 + lane) * ldb + r] : T(0);
        for (int c = 0; c < wd; ++c) {
            const T xc = lane_bcast(x, c) * ld[c * (NB + 1) + c];
            if (lane == c) x = xc;
            if (lane > c) x -= ld[lane * (NB + 1) + c] * xc;
        }
        if (lane < wd) B[(t0 + lane) * ldb + r] = x;
    }
}

// ---------------------------------------------------------------------------
// Back substitution L^t X = Y, one launch per block, last block first.
// Launch k = nblk solves the last diagonal block.  Launch k (block k solved)
// has k workgroups: workgroup b subtracts L[block k][block k-1-b]^t X_k from
// the rows of block k-1-b (lane = row of the target block, so the reads of a
// row of L are contiguous; the four waves split the rows of block k and their
// sums are added in a fixed order); workgroup 0 then solves diagonal block
// k-1 with wave 0, last column first.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_bwd(const T* __restrict__ L, int64_t n, T* __restrict__ B, int64_t nrhs,
                                                  int64_t ldb, int64_t k, int64_t nblk) {
    __shared__ T ld[NB * (NB + 1)];
    __shared__ T xs[NB * RC];
    __shared__ T red[4 * NB * RC];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int64_t d;  // diagonal block solved by workgroup 0
    if (k < nblk) {
        const int64_t x0 = NB * k;
        const int wk = (int)(n - x0 < NB ? n - x0 : NB);
        const int64_t tb = k - 1 - blockIdx.x;
        const int64_t c0 = NB * tb;
        // this wave's 16 rows of L[block k][block tb], all loads in flight at once
        T lv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int j = wv + 4 * u;
            lv[u] = j < wk ? L[pidx(x0 + j, c0 + lane)] : T(0);
        }
        for (int64_t r0 = 0; r0 < nrhs; r0 += RC) {
            const int rc = (int)(nrhs - r0 < RC ? nrhs - r0 : RC);
            __syncthreads();
            for (int e = t; e < NB * RC; e += 256) {
                const int j = e / RC, rr = e % RC;
                xs[e] = (j < wk && rr < rc) ? B[(x0 + j) * ldb + r0 + rr] : T(0);
            }
            __syncthreads();
            T acc[RC];
#pragma unroll
            for (int rr = 0; rr < RC; ++rr) acc[rr] = T(0);
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int j = wv + 4 * u;  // xs rows past wk hold zeros
#pragma unroll
                for (int rr = 0; rr < RC; ++rr) acc[rr] += lv[u] * xs[j * RC + rr];
            }
#pragma unroll
            for (int rr = 0; rr < RC; ++rr) red[(wv * NB + lane) * RC + rr] = acc[rr];
            __syncthreads();
            if (wv == 0) {
                for (int rr = 0; rr < rc; ++rr) {
                    const T s = ((red[lane * RC + rr] + red[(NB + lane) * RC + rr]) + red[(2 * NB + lane) * RC + rr]) +
                                red[(3 * NB + lane) * RC + rr];
                    B[(c0 + lane) * ldb + r0 + rr] -= s;
                }
            }
        }
        if (blockIdx.x != 0) return;
        d = k - 1;
    } else {
        d = nblk - 1;
    }
    const int64_t d0 = NB * d;
    const int wd = (int)(n - d0 < NB ? n - d0 : NB);
    __syncthreads();
    stage_diag(L, d0, wd, ld);
    __syncthreads();
    if (wv != 0) return;
    for (int64_t r = 0; r < nrhs; ++r) {
        T x = lane < wd ? B[(d0 + lane) * ldb + r] : T(0);
        for (int c = wd - 1; c >= 0; --c) {
            const T xc = lane_bcast(x, c) * ld[c * (NB + 1) + c];
            if (lane == c) x = xc;
            if (lane < c) x -= ld[c * (NB + 1) + lane] * xc;
        }
        if (lane < wd) B[(d0 + lane) * ldb + r] = x;
    }
}

// ---------------------------------------------------------------------------
// A^t B: partial sums over row chunks (workgroup = 256 columns x one chunk,
// thread = column, rows ascending, FP64 accumulation), then a pass that adds
// the chunks in order.  Each row of A is read once per eight right-hand
// sides, contiguously across the workgroup.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_atb_part(const T* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                  const T* __restrict__ B, int64_t nrhs, int64_t ldb, int64_t rows,
                                                  double* __restrict__ part) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t ch = blockIdx.y;
    const int64_t i0 = ch * rows;
    const int64_t i1 = i0 + rows < m ? i0 + rows : m;
    for (int64_t r0 = 0; r0 < nrhs; r0 += RC) {
        const int rc = (int)(nrhs - r0 < RC ? nrhs - r0 : RC);
        double acc[RC];
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) acc[rr] = 0.0;
        if (j < n) {
            for (int64_t i = i0; i < i1; ++i) {
                const double a = (double)A[i * lda + j];
#pragma unroll
                for (int rr = 0; rr < RC; ++rr)
                    if (rr < rc) acc[rr] += a * (double)B[i * ldb + r0 + rr];
            }
#pragma unroll
            for (int rr = 0; rr < RC; ++rr)
                if (rr < rc) part[(ch * n + j) * nrhs + r0 + rr] = acc[rr];
        }
    }
}

// ---------------------------------------------------------------------------
// A X for the projection A (A^t A)^-1 A^t B: one wave per row of A (four rows
// per workgroup), lanes striding the row's n entries (contiguous loads), FP64
// sums over lanes and a wave-wide sum per right-hand side.  X (n x nrhs) is
// small and read through the caches.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_ax(const T* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                            const T* __restrict__ X, int64_t nrhs, int64_t ldx, T* __restrict__ out,
                                            int64_t ldo) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= m) return;  // whole waves leave; no barrier follows
    const T* a = A + i * lda;
    for (int64_t r0 = 0; r0 < nrhs; r0 += RC) {
        const int rc = (int)(nrhs - r0 < RC ? nrhs - r0 : RC);
        double acc[RC];
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) acc[rr] = 0.0;
#pragma unroll 4
        for (int64_t j = lane; j < n; j += 64) {
            const double v = (double)a[j];
#pragma unroll
            for (int rr = 0; rr < RC; ++rr)
                if (rr < rc) acc[rr] += v * (double)X[j * ldx + r0 + rr];
        }
        for (int rr = 0; rr < rc; ++rr) {
            const double sum = wave_sum(acc[rr]);
            if (lane == 0) out[i * ldo + r0 + rr] = (T)sum;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_atb_sum(const double* __restrict__ part, int64_t chunks, int64_t n,
                                                 int64_t nrhs, T* __restrict__ out, int64_t ldo) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * nrhs) return;
    double s = 0.0;
    for (int64_t c = 0; c < chunks; ++c) s += part[c * n * nrhs + e];
    out[(e / nrhs) * ldo + e % nrhs] = (T)s;
}

// Right-looking factorization.  With a helper stream s2 and two events the
// update of block k is split: its first tile column (what block k + 1 needs)
// runs on s, the rest on s2, so the diagonal factor and row solve of block
// k + 1 overlap the bulk of the update.  Ordering: the rest of update k waits
// for the row solve and first column of k (event e); the first column of
// update k + 1 waits for the rest of update k (event f), whose tiles it
// overlaps; s joins s2 at the end.
template <typename T>
hipError_t potrf_t(T* C, int64_t n, int32_t* info, hipStream_t s, hipStream_t s2, hipEvent_t e, hipEvent_t f) {
    bool rest_pending = false;
    hipError_t err;
    for (int64_t kb = 0; kb < n; kb += NB) {
        const int w = (int)(n - kb < NB ? n - kb : NB);
        const int64_t rest = n - kb - w;
        const int64_t nrb = (rest + NB - 1) / NB;
        {
            ProfScope ps(ATA_KERNEL_FACTOR_PANEL, s);
            hipLaunchKernelGGL(k_chol_diag<T>, dim3(1), dim3(256), 0, s, C, kb, w, info);
            if ((err = hipGetLastError()) != hipSuccess) return err;
        }
        if (nrb == 0) continue;
        {
            ProfScope ps(ATA_KERNEL_FACTOR_PANEL, s);
            hipLaunchKernelGGL(k_chol_rows<T>, dim3((unsigned)nrb), dim3(256), 0, s, C, n, kb, w);
            if ((err = hipGetLastError()) != hipSuccess) return err;
        }
        if (!s2 || nrb == 1) {
            if (rest_pending) {
                if ((err = hipStreamWaitEvent(s, f, 0)) != hipSuccess) return err;
                rest_pending = false;
            }
            ProfScope ps(ATA_KERNEL_FACTOR_UPDATE, s);
            hipLaunchKernelGGL(k_chol_update<T>, dim3((unsigned)(nrb * (nrb + 1) / 2)), dim3(256), 0, s, C, n, kb,
                               w, (int)nrb, 0);
            if ((err = hipGetLastError()) != hipSuccess) return err;
            continue;
        }
        if (rest_pending && (err = hipStreamWaitEvent(s, f, 0)) != hipSuccess) return err;
        {
            ProfScope ps(ATA_KERNEL_FACTOR_UPDATE, s);
            hipLaunchKernelGGL(k_chol_update<T>, dim3((unsigned)nrb), dim3(256), 0, s, C, n, kb, w, (int)nrb, 1);
            if ((err = hipGetLastError()) != hipSuccess) return err;
        }
        if ((err = hipEventRecord(e, s)) != hipSuccess) return err;
        if ((err = hipStreamWaitEvent(s2, e, 0)) != hipSuccess) return err;
        {
            ProfScope ps(ATA_KERNEL_FACTOR_UPDATE, s2);
            hipLaunchKernelGGL(k_chol_update<T>, dim3((unsigned)((nrb - 1) * nrb / 2)), dim3(256), 0, s2, C, n, kb,
                               w, (int)nrb, 2);
            if ((err = hipGetLastError()) != hipSuccess) return err;
        }
        if ((err = hipEventRecord(f, s2)) != hipSuccess) return err;
        rest_pending = true;
    }
    if (rest_pending && (err = hipStreamWaitEvent(s, f, 0)) != hipSuccess) return err;
    return hipSuccess;
}

template <typename T>
hipError_t potrs_t(const T* L, int64_t n, T* B, int64_t nrhs, int64_t ldb, hipStream_t s) {
    const int64_t nblk = (n + NB - 1) / NB;
    for (int64_t k = -1; k < nblk - 1; ++k) {
        const int64_t grid = k < 0 ? 1 : nblk - k - 1;
        ProfScope ps(ATA_KERNEL_SOLVE, s);
        hipLaunchKernelGGL(k_trsv_fwd<T>, dim3((unsigned)grid), dim3(256), 0, s, L, n, B, nrhs, ldb, k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    for (int64_t k = nblk; k >= 1; --k) {
        const int64_t grid = k == nblk ? 1 : k;
        ProfScope ps(ATA_KERNEL_SOLVE, s);
        hipLaunchKernelGGL(k_trsv_bwd<T>, dim3((unsigned)grid), dim3(256), 0, s, L, n, B, nrhs, ldb, k, nblk);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t atb_t(const T* A, int64_t m, int64_t n, int64_t lda, const T* B, int64_t nrhs, int64_t ldb, T* out,
                 int64_t ldo, double* part, int64_t chunks, hipStream_t s) {
    const int64_t rows = (m + chunks - 1) / chunks;
    ProfScope ps(ATA_KERNEL_SOLVE, s);
    hipLaunchKernelGGL(k_atb_part<T>, dim3((unsigned)((n + 255) / 256), (unsigned)chunks), dim3(256), 0, s, A, m, n,
                       lda, B, nrhs, ldb, rows, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_atb_sum<T>, dim3((unsigned)((n * nrhs + 255) / 256)), dim3(256), 0, s, part, chunks, n, nrhs,
                       out, ldo);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transpose for the companion product A A^t: out (n x m, row stride m) =
// A^t for A (m x n, row stride lda), 64 x 64 tiles through LDS so that both
// the reads of A's rows and the writes of out's rows are contiguous.
// E: element type of 4 or 8 bytes (moved as raw bits).
// ---------------------------------------------------------------------------
template <typename E>
__global__ __launch_bounds__(256) void k_transpose(const E* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                   E* __restrict__ out) {
    __shared__ E tile[64][65];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * 64, r0 = (int64_t)blockIdx.y * 64;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int r = wv + 4 * u;
        if (r0 + r < m && c0 + lane < n) tile[r][lane] = A[(r0 + r) * lda + c0 + lane];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = wv + 4 * u;
        if (c0 + c < n && r0 + lane < m) out[(c0 + c) * m + r0 + lane] = tile[lane][c];
    }
}

}  // namespace

hipError_t launch_ax(bool f32, const void* A, int64_t m, int64_t n, int64_t lda, const void* X, int64_t nrhs,
                     int64_t ldx, void* out, int64_t ldo, hipStream_t s) {
    ProfScope ps(ATA_KERNEL_SOLVE, s);
    const dim3 grid((unsigned)((m + 3) / 4));
    if (f32)
        hipLaunchKernelGGL(k_ax<float>, grid, dim3(256), 0, s, (const float*)A, m, n, lda, (const float*)X, nrhs,
                           ldx, (float*)out, ldo);
    else
        hipLaunchKernelGGL(k_ax<double>, grid, dim3(256), 0, s, (const double*)A, m, n, lda, (const double*)X, nrhs,
                           ldx, (double*)out, ldo);
    return hipGetLastError();
}

hipError_t launch_transpose(int elem_bytes, const void* A, int64_t m, int64_t n, int64_t lda, void* out,
                            hipStream_t s) {
    const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 63) / 64));
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_transpose<uint64_t>, grid, dim3(256), 0, s, (const uint64_t*)A, m, n, lda,
                           (uint64_t*)out);
    else
        hipLaunchKernelGGL(k_transpose<uint32_t>, grid, dim3(256), 0, s, (const uint32_t*)A, m, n, lda,
                           (uint32_t*)out);
    return hipGetLastError();
}

hipError_t launch_potrf(bool f32, void* C, int64_t n, int32_t* info, hipStream_t s, hipStream_t s2, hipEvent_t e,
                        hipEvent_t f) {
    return f32 ? potrf_t((float*)C, n, info, s, s2, e, f) : potrf_t((double*)C, n, info, s, s2, e, f);
}

hipError_t launch_potrs(bool f32, const void* L, int64_t n, void* B, int64_t nrhs, int64_t ldb, hipStream_t s) {
    return f32 ? potrs_t((const float*)L, n, (float*)B, nrhs, ldb, s)
               : potrs_t((const double*)L, n, (double*)B, nrhs, ldb, s);
}

int64_t atb_chunks(int64_t m, int64_t n) {
    const int64_t ct = (n + 255) / 256;
    int64_t ch = (2048 + ct - 1) / ct;
    const int64_t most = (m + 255) / 256;
    if (ch > most) ch = most;
    return ch < 1 ? 1 : ch;
}

hipError_t launch_atb(bool f32, const void* A, int64_t m, int64_t n, int64_t lda, const void* B, int64_t nrhs,
                      int64_t ldb, void* out, int64_t ldo, double* part, hipStream_t s) {
    const int64_t ch = atb_chunks(m, n);
    return f32 ? atb_t((const float*)A, m, n, lda, (const float*)B, nrhs, ldb, (float*)out, ldo, part, ch, s)
               : atb_t((const double*)A, m, n, lda, (const double*)B, nrhs, ldb, (double*)out, ldo, part, ch, s);
}

}  // namespace atalib
