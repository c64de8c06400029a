// CDNA4 (gfx950) kernels of the A^t A library.
//
// FP64 products use v_mfma_f64_4x4x4_4b with its A operand broadcast to all
// four blocks, which turns the instruction into a 4 x 16 x 4 product:
//   A operand: lane l holds A[row = l & 3][k = l >> 4]
//   B operand: lane l holds B[k = l >> 4][col = l & 15]
//   result:    lane l holds D[row = l >> 4][col = l & 15]
// (measured on MI355X: this form sustains about 64 TFLOP/s, the 16x16x4 FP64
// instruction about 46 TFLOP/s).
//
// Every product here is D = X^t Y where X and Y are K x M and K x N column
// slices of the row-major A (K runs over rows of A), so both operands are
// staged in LDS as [k][column] rows copied from contiguous rows of A.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ata_plan.h"

namespace atalib {

typedef double d1_t;

__device__ __forceinline__ double mfma_f64(double a, double b, double c) {
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int64_t packed_index(int64_t r, int64_t q) { return r * (r + 1) / 2 + q; }

// ---------------------------------------------------------------------------
// Classical tile kernel: TK_SYRK (lower triangle of a diagonal block) and
// TK_GEMM (dense off-diagonal block).  128 x 128 output tile per workgroup,
// four waves of 64 x 64, K staged 16 rows at a time, double-buffered LDS.
// ---------------------------------------------------------------------------
constexpr int GT = kGemmTile;  // 128
constexpr int GK = 16;
constexpr int GPAD = 4;

__global__ void __launch_bounds__(256, 2) k_gemm_f64(const double* __restrict__ A, int64_t lda,
                                                  const DevTask* __restrict__ tasks,
                                                  const DevTerm* __restrict__ terms,
                                                  const int32_t* __restrict__ segs,
                                                  const WorkItem* __restrict__ items,
                                                  double* __restrict__ C) {
    __shared__ double Xs[2][GK][GT + GPAD];
    __shared__ double Ys[2][GK][GT + GPAD];

    const WorkItem w = items[blockIdx.x];
    const DevTask t = tasks[w.task];
    const DevTerm tx = terms[t.term_off];
    const DevTerm ty = terms[t.term_off + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int i0 = w.ti * GT, j0 = w.tj * GT;

    // staging map: thread -> row lk of the k tile, 8 consecutive columns at lc
    const int lk = tid >> 4, lc = (tid & 15) * 8;
    const int xcol = tx.col + i0 + lc;
    const int ycol = ty.col + j0 + lc;
    const int xcv = tx.cvend - xcol;  // columns valid from xcol (may be <= 0)
    const int ycv = ty.cvend - ycol;

    double acc[16][4];
#pragma unroll
    for (int a = 0; a < 16; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;

    // k-tile cursor over the segments
    const int stride = 1 + 2 * (t.nx + t.ny);
    int seg = 0, k0 = 0;
    int klen = t.nseg > 0 ? segs[t.seg_off] : 0;
    int xrow = t.nseg > 0 ? segs[t.seg_off + 1] : 0;
    int yrow = t.nseg > 0 ? segs[t.seg_off + 3] : 0;
    int ntiles = 0;
    for (int s = 0; s < t.nseg; ++s) ntiles += (segs[t.seg_off + s * stride] + GK - 1) / GK;

    double xr[8], yr[8];
    auto load = [&](int kk0, int kl, int xr0, int yr0) {
        const bool rv = (kk0 + lk) < kl;
        const double* px = A + (int64_t)(xr0 + kk0 + lk) * lda + xcol;
        const double* py = A + (int64_t)(yr0 + kk0 + lk) * lda + ycol;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            xr[e] = (rv && e < xcv) ? px[e] : 0.0;
            yr[e] = (rv && e < ycv) ? py[e] : 0.0;
        }
    };
    auto advance = [&]() {
        k0 += GK;
        if (k0 >= klen) {
            k0 = 0;
            ++seg;
            if (seg < t.nseg) {
                klen = segs[t.seg_off + seg * stride];
                xrow = segs[t.seg_off + seg * stride + 1];
                yrow = segs[t.seg_off + seg * stride + 3];
            }
        }
    };

    if (ntiles > 0) load(k0, klen, xrow, yrow);
    for (int it = 0; it < ntiles; ++it) {
        const int buf = it & 1;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            Xs[buf][lk][lc + e] = xr[e];
            Ys[buf][lk][lc + e] = yr[e];
        }
        __syncthreads();
        if (it + 1 < ntiles) {
            advance();
            load(k0, klen, xrow, yrow);
        }
#pragma unroll
        for (int ks = 0; ks < GK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double bv[4];
#pragma unroll
            for (int cf = 0; cf < 4; ++cf) bv[cf] = Ys[buf][kr][wn * 64 + cf * 16 + (lane & 15)];
#pragma unroll
            for (int rf = 0; rf < 16; ++rf) {
                const double av = Xs[buf][kr][wm * 64 + rf * 4 + (lane & 3)];
#pragma unroll
                for (int cf = 0; cf < 4; ++cf) acc[rf][cf] = mfma_f64(av, bv[cf], acc[rf][cf]);
            }
        }
    }

    // epilogue: rows of D go to C rows r0 + gi, columns to C columns q0 + gj
    const bool syrk = t.kind == TK_SYRK;
#pragma unroll
    for (int rf = 0; rf < 16; ++rf) {
        const int gi = i0 + wm * 64 + rf * 4 + (lane >> 4);
        if (gi >= t.dM) continue;
        const int64_t rowbase = packed_index((int64_t)t.r0 + gi, t.q0);
#pragma unroll
        for (int cf = 0; cf < 4; ++cf) {
            const int gj = j0 + wn * 64 + cf * 16 + (lane & 15);
            if (gj >= t.dN || (syrk && gj > gi)) continue;
            double* p = C + rowbase + gj;
            *p = t.beta ? *p + acc[rf][cf] : acc[rf][cf];
        }
    }
}

// ---------------------------------------------------------------------------
// In-tile Strassen kernel (TK_STR).  The product P = Xop^t Yop (padded M x N,
// K per segment) is split once more into quadrants; a workgroup owns the
// 64 x 64 tile at (ti, tj) of all four result quadrants, keeps the seven
// products in registers (four waves of 32 x 32 each) and combines them at the
// end.  Operand terms of higher levels are summed while staging to LDS.
// ---------------------------------------------------------------------------
constexpr int ST = kStrTile;  // 64
constexpr int SK_MAX = 16;  // k rows per LDS stage (8 when operands carry several terms)
constexpr int SPAD = 4;  // row stride = 4 mod 16 doubles: broadcast reads hit disjoint banks

template <int VAR>
__device__ __forceinline__ void left_operands(double x00, double x01, double x10, double x11, double (&o)[7]) {
    // x_ab = L_ab (M-half a, K-half b)
    if (VAR == 0) {
        o[0] = x00 + x11;
        o[1] = x10 + x11;
        o[2] = x00;
        o[3] = x11;
        o[4] = x00 + x01;
        o[5] = x10 - x00;
        o[6] = x01 - x11;
    } else {
        const double s1 = x10 + x11, s2 = s1 - x00;
        o[0] = x00;
        o[1] = x01;
        o[2] = x01 - s2;
        o[3] = x11;
        o[4] = s1;
        o[5] = s2;
        o[6] = x00 - x10;
    }
}

template <int VAR>
__device__ __forceinline__ void right_operands(double y00, double y01, double y10, double y11, double (&o)[7]) {
    // y_bc = R_bc (K-half b, N-half c)
    if (VAR == 0) {
        o[0] = y00 + y11;
        o[1] = y00;
        o[2] = y01 - y11;
        o[3] = y10 - y00;
        o[4] = y11;
        o[5] = y00 + y01;
        o[6] = y10 + y11;
    } else {
        const double t1 = y01 - y00, t2 = y11 - t1;
        o[0] = y00;
        o[1] = y10;
        o[2] = y11;
        o[3] = t2 - y10;
        o[4] = t1;
        o[5] = t2;
        o[6] = y11 - y01;
    }
}

template <int VAR>
__device__ __forceinline__ void combine_products(const double (&m)[7], double (&d)[4]) {
    if (VAR == 0) {
        d[0] = ((m[0] + m[3]) - m[4]) + m[6];
        d[1] = m[2] + m[4];
        d[2] = m[1] + m[3];
        d[3] = ((m[0] - m[1]) + m[2]) + m[5];
    } else {
        const double u2 = m[0] + m[5], u3 = u2 + m[6], u4 = u2 + m[4];
        d[0] = m[0] + m[1];
        d[1] = u4 + m[2];
        d[2] = u3 - m[3];
        d[3] = u3 + m[4];
    }
}

template <int VAR, int TMAX, int SK>
__global__ void __launch_bounds__(512, 1) k_str_f64(const double* __restrict__ A, int64_t lda,
                                                    const DevTask* __restrict__ tasks,
                                                    const DevTerm* __restrict__ terms,
                                                    const int32_t* __restrict__ segs,
                                                    const WorkItem* __restrict__ items,
                                                    double* __restrict__ C, double* __restrict__ W) {
    __shared__ double Xs[2][4][SK][ST + SPAD];
    __shared__ double Ys[2][4][SK][ST + SPAD];

    const WorkItem w = items[blockIdx.x];
    const DevTask t = tasks[w.task];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;  // 4 x 2 waves of 16 x 32
    const int MH = (t.M + 1) >> 1, NH = (t.N + 1) >> 1;
    const int i0 = w.ti * ST, j0 = w.tj * ST;
    const int stride = 1 + 2 * (t.nx + t.ny);

    // staging map: thread -> k rows lk and lk + 8, column lc (two elements per quadrant)
    const int lk = tid >> 6, lc = tid & 63;
    constexpr int KR = SK / 8;  // k rows per thread

    // Per-term column data, fixed for the whole K loop.
    int xcol[TMAX][2], ycol[TMAX][2];
    unsigned xmask[TMAX], ymask[TMAX];  // bit a: column of M-half a valid
    double xsgn[TMAX], ysgn[TMAX];
#pragma unroll
    for (int u = 0; u < TMAX; ++u) {
        xmask[u] = ymask[u] = 0u;
        xsgn[u] = ysgn[u] = 0.0;
        xcol[u][0] = xcol[u][1] = ycol[u][0] = ycol[u][1] = 0;
        if (u < t.nx) {
            const DevTerm tm = terms[t.term_off + u];
            xsgn[u] = (double)tm.sign;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                xcol[u][a] = tm.col + a * MH + i0 + lc;
                if (i0 + lc < MH && xcol[u][a] < tm.cvend) xmask[u] |= 1u << a;
            }
        }
        if (u < t.ny) {
            const DevTerm tm = terms[t.term_off + t.nx + u];
            ysgn[u] = (double)tm.sign;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                ycol[u][c] = tm.col + c * NH + j0 + lc;
                if (j0 + lc < NH && ycol[u][c] < tm.cvend) ymask[u] |= 1u << c;
            }
        }
    }

    double acc[7][4][2];
#pragma unroll
    for (int p = 0; p < 7; ++p)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[p][a][b] = 0.0;

    int ntiles = 0;
    for (int s = 0; s < t.nseg; ++s) {
        const int kh = (segs[t.seg_off + s * stride] + 1) >> 1;
        ntiles += (kh + SK - 1) / SK;
    }

    // raw term values of the next k tile: [term][quad]
    double xraw[TMAX][KR][4], yraw[TMAX][KR][4];
    int seg = 0, k0 = 0;
    int kh = t.nseg > 0 ? (segs[t.seg_off] + 1) >> 1 : 0;

    // Issue every load of the next k tile; nothing waits on them here.
    auto load = [&]() {
        const int32_t* sg = segs + t.seg_off + seg * stride;
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            const int kk = k0 + lk + 8 * r;
            const bool kv = kk < kh;
#pragma unroll
            for (int u = 0; u < TMAX; ++u) {
                if (u < t.nx) {
                    const int row0 = sg[1 + 2 * u], rvend = sg[2 + 2 * u];
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int row = row0 + b * kh + kk;
                        const bool rok = kv && row < rvend;
                        const double* pr = A + (int64_t)row * lda;
#pragma unroll
                        for (int a = 0; a < 2; ++a)
                            xraw[u][r][a * 2 + b] = (rok && ((xmask[u] >> a) & 1u)) ? pr[xcol[u][a]] : 0.0;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) xraw[u][r][q] = 0.0;
                }
                if (u < t.ny) {
                    const int row0 = sg[1 + 2 * (t.nx + u)], rvend = sg[2 + 2 * (t.nx + u)];
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int row = row0 + b * kh + kk;
                        const bool rok = kv && row < rvend;
                        const double* pr = A + (int64_t)row * lda;
#pragma unroll
                        for (int c = 0; c < 2; ++c)
                            yraw[u][r][b * 2 + c] = (rok && ((ymask[u] >> c) & 1u)) ? pr[ycol[u][c]] : 0.0;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) yraw[u][r][q] = 0.0;
                }
            }
        }
    };
    // Signed sum of the terms (fixed order) into the LDS buffer.
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < KR; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double x = 0.0, y = 0.0;
#pragma unroll
                for (int u = 0; u < TMAX; ++u) {
                    x += xsgn[u] * xraw[u][r][q];
                    y += ysgn[u] * yraw[u][r][q];
                }
                Xs[buf][q][lk + 8 * r][lc] = x;
                Ys[buf][q][lk + 8 * r][lc] = y;
            }
    };
    auto advance = [&]() {
        k0 += SK;
        if (k0 >= kh) {
            k0 = 0;
            ++seg;
            if (seg < t.nseg) kh = (segs[t.seg_off + seg * stride] + 1) >> 1;
        }
    };

    if (ntiles > 0) load();
    for (int it = 0; it < ntiles; ++it) {
        const int buf = it & 1;
        store(buf);
        __syncthreads();
        if (it + 1 < ntiles) {
            advance();
            load();
        }
#pragma unroll
        for (int ks = 0; ks < SK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double ro[2][7];
#pragma unroll
            for (int cf = 0; cf < 2; ++cf) {
                const int cc = wn * 32 + cf * 16 + (lane & 15);
                right_operands<VAR>(Ys[buf][0][kr][cc], Ys[buf][1][kr][cc], Ys[buf][2][kr][cc],
                                    Ys[buf][3][kr][cc], ro[cf]);
            }
#pragma unroll
            for (int rf = 0; rf < 4; ++rf) {
                const int rr = wm * 16 + rf * 4 + (lane & 3);
                double lo[7];
                left_operands<VAR>(Xs[buf][0][kr][rr], Xs[buf][1][kr][rr], Xs[buf][2][kr][rr],
                                   Xs[buf][3][kr][rr], lo);
#pragma unroll
                for (int p = 0; p < 7; ++p)
#pragma unroll
                    for (int cf = 0; cf < 2; ++cf) acc[p][rf][cf] = mfma_f64(lo[p], ro[cf][p], acc[p][rf][cf]);
            }
        }
    }

    // combine the seven products into the four quadrants and store
#pragma unroll
    for (int rf = 0; rf < 4; ++rf) {
        const int li = i0 + wm * 16 + rf * 4 + (lane >> 4);  // row inside a quadrant
#pragma unroll
        for (int cf = 0; cf < 2; ++cf) {
            const int lj = j0 + wn * 32 + cf * 16 + (lane & 15);
            double m[7], d[4];
#pragma unroll
            for (int p = 0; p < 7; ++p) m[p] = acc[p][rf][cf];
            combine_products<VAR>(m, d);
            if (li >= MH || lj >= NH) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gi = (q >> 1) * MH + li, gj = (q & 1) * NH + lj;
                if (gi >= t.dM || gj >= t.dN) continue;
                if (t.dst == 0) {
                    double* p = C + packed_index((int64_t)t.r0 + gi, t.q0) + gj;
                    *p = t.beta ? *p + d[q] : d[q];
                } else {
                    W[t.ws_off + (int64_t)gi * t.N + gj] = d[q];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Combination of workspace products into an off-diagonal block of packed C.
// One thread per output element; fixed summation order.
// ---------------------------------------------------------------------------
__constant__ int c_dcoef[2][7][4] = ATA_D_COEF;

__global__ void __launch_bounds__(256) k_combine_f64(const DevCombine* __restrict__ cbs, int ncb,
                                                     int64_t total, const double* __restrict__ W,
                                                     double* __restrict__ C) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int lo = 0, hi = ncb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cbs[mid].elem_off <= e) lo = mid;
        else hi = mid - 1;
    }
    const DevCombine cb = cbs[lo];
    const int64_t loc = e - cb.elem_off;
    const int i = (int)(loc / cb.N), j = (int)(loc % cb.N);
    int ii = i, jj = j, Mc = cb.M, Nc = cb.N;
    int quad[4];
    for (int l = 0; l < cb.levels; ++l) {
        const int MH = (Mc + 1) >> 1, NH = (Nc + 1) >> 1;
        const int a = ii >= MH, c = jj >= NH;
        ii -= a * MH;
        jj -= c * NH;
        quad[l] = a * 2 + c;
        Mc = MH;
        Nc = NH;
    }
    const int64_t slot_elems = (int64_t)cb.Mp * cb.Np;
    const double* base = W + cb.ws_off + (int64_t)ii * cb.Np + jj;
    double s = 0.0;
    int npaths = 1;
    for (int l = 0; l < cb.levels; ++l) npaths *= 7;
    for (int path = 0; path < npaths; ++path) {
        int rem = path, coef = 1;
        for (int l = cb.levels - 1; l >= 0; --l) {
            coef *= c_dcoef[cb.variant][rem % 7][quad[l]];
            rem /= 7;
        }
        if (coef) s += coef > 0 ? base[path * slot_elems] : -base[path * slot_elems];
    }
    double* p = C + packed_index((int64_t)cb.r0 + i, cb.q0) + j;
    *p = cb.beta ? *p + s : s;
}

template <typename T>
__global__ void k_fill_zero(T* __restrict__ p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = T(0);
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the C ABI layer)
// ---------------------------------------------------------------------------
hipError_t launch_gemm_f64(const double* A, int64_t lda, const DevTask* tasks, const DevTerm* terms,
                           const int32_t* segs, const WorkItem* items, int nitems, double* C,
                           hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gemm_f64, dim3(nitems), dim3(256), 0, s, A, lda, tasks, terms, segs, items, C);
    return hipGetLastError();
}

template <int VAR>
static void launch_str_var(int tmax, dim3 g, hipStream_t s, const double* A, int64_t lda, const DevTask* tasks,
                           const DevTerm* terms, const int32_t* segs, const WorkItem* items, double* C,
                           double* W) {
    if (tmax <= 1)
        hipLaunchKernelGGL((k_str_f64<VAR, 1, 16>), g, dim3(512), 0, s, A, lda, tasks, terms, segs, items, C, W);
    else if (tmax <= 2)
        hipLaunchKernelGGL((k_str_f64<VAR, 2, 8>), g, dim3(512), 0, s, A, lda, tasks, terms, segs, items, C, W);
    else if (tmax <= 4)
        hipLaunchKernelGGL((k_str_f64<VAR, 4, 8>), g, dim3(512), 0, s, A, lda, tasks, terms, segs, items, C, W);
    else
        hipLaunchKernelGGL((k_str_f64<VAR, 8, 8>), g, dim3(512), 0, s, A, lda, tasks, terms, segs, items, C, W);
}

// tmax: largest number of terms of either operand over the launched tasks.
hipError_t launch_str_f64(int variant, int tmax, const double* A, int64_t lda, const DevTask* tasks,
                          const DevTerm* terms, const int32_t* segs, const WorkItem* items, int nitems,
                          double* C, double* W, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (tmax > kMaxTerms) return hipErrorInvalidValue;
    if (variant == 0)
        launch_str_var<0>(tmax, dim3(nitems), s, A, lda, tasks, terms, segs, items, C, W);
    else
        launch_str_var<1>(tmax, dim3(nitems), s, A, lda, tasks, terms, segs, items, C, W);
    return hipGetLastError();
}

hipError_t launch_combine_f64(const DevCombine* cbs, int ncb, int64_t total, const double* W, double* C,
                              hipStream_t s) {
    if (ncb <= 0 || total <= 0) return hipSuccess;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_combine_f64, dim3((unsigned)blocks), dim3(256), 0, s, cbs, ncb, total, W, C);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, int64_t count, int elem_bytes, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_fill_zero<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)p, count);
    else
        hipLaunchKernelGGL(k_fill_zero<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)p, count);
    return hipGetLastError();
}

}  // namespace atalib
