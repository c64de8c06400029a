// CDNA4 (gfx950) kernels of the A^t A library.
//
// Every product here is D = X^t Y where X and Y are K x M and K x N column
// slices of the row-major A (K runs over rows of A).  The FP64 and FP32 tile
// kernels stage both operands in LDS as [k][column] rows copied from
// contiguous rows of A; the reduced-precision kernels read a transposed,
// converted copy of A made by a prepass, so that every MFMA lane loads
// k-contiguous bytes.
//
// MFMA forms (lane layouts measured on MI355X):
//  FP64  v_mfma_f64_4x4x4_4b with the A operand broadcast to all four blocks,
//        i.e. a 4 x 16 x 4 product: A lane l = A[row l&3][k l>>4],
//        B lane l = B[k l>>4][col l&15], result lane l = D[row l>>4][col l&15].
//        This form sustains about 64 TFLOP/s; the 16x16x4 FP64 form about 46.
//  FP32  v_mfma_f32_16x16x4f32: A lane l = A[row l&15][k l>>4], B as above,
//        result element e of lane l = D[row 4(l>>4)+e][col l&15].
//  BF16  v_mfma_f32_16x16x32_bf16: lane l holds 8 consecutive k of row (or
//        column) l&15 starting at k = 8(l>>4); result as FP32.
//  FP8   v_mfma_scale_f32_16x16x128_f8f6f4 (OCP e4m3 operands, unit scales):
//        lane l holds 32 consecutive k starting at k = 32(l>>4); result as FP32.
// The k assignment of the BF16/FP8 forms only has to agree between the two
// operands, which it does by construction.
#include <hip/hip_runtime.h>

#include <atomic>

#include <cstdint>
#include <type_traits>

#include "ata_kernels.h"
#include "ata_plan.h"

namespace atalib {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef int i8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t packed_index(int64_t r, int64_t q) { return r * (r + 1) / 2 + q; }

// ---------------------------------------------------------------------------
// Operand staging through raw buffer loads.  A buffer resource covers the
// valid rows of one operand slab (num_records = rows x row bytes); a load
// whose offset lies at or past num_records returns zero without touching
// memory.  This gives the zero padding of ragged quadrants and K tails
// without branches.  Offsets are 32-bit: a slab spans at most kStageRows
// rows of at most kMaxRowBytes (checked at the API).  The compiler merges
// adjacent 8-byte loads into 16-byte ones; the range check of a multi-dword
// raw buffer load applies per dword, so a pair straddling the end of a slab
// still returns its in-range half (exercised by the odd-stride tests).
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t kOOB = 0x80000000u;  // an offset past every record count used here
constexpr int kStageRows = 16;
static_assert(kStageRows * kMaxRowBytes <= (int64_t)kOOB / 2, "slab offsets must stay below kOOB");

__device__ __forceinline__ rsrc_t slab_rsrc(const void* base, int nrows, int64_t row_bytes) {
    const int bytes = nrows > 0 ? (int)(nrows * row_bytes) : 0;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T bload(rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ double bload<double>(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ float bload<float>(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

// x with its sign bit flipped when flip is set (an exact negation).
__device__ __forceinline__ double flip_sign(double x, bool flip) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x) ^ (flip ? 0x8000000000000000ull : 0ull);
    return __builtin_bit_cast(double, b);
}
__device__ __forceinline__ float flip_sign(float x, bool flip) {
    return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, x) ^ (flip ? 0x80000000u : 0u));
}

// ---------------------------------------------------------------------------
// MFMA engines for the tile kernels staged from A directly
// ---------------------------------------------------------------------------
template <typename T>
struct Eng;

template <>
struct Eng<double> {
    static constexpr int RM = 4, RN = 16, NA = 1;  // result rows, cols, elements per lane
    static constexpr int PAD = 4;  // LDS row stride = 4 mod 16 doubles: broadcast reads hit disjoint banks
    typedef double accv_t;
    __device__ static int arow(int lane) { return lane & 3; }
    __device__ static void mma(double a, double b, accv_t& c) { c = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0); }
    __device__ static double elem(const accv_t& c, int) { return c; }
    __device__ static int orow(int lane, int) { return lane >> 4; }
    __device__ static void zero(accv_t& c) { c = 0.0; }
};

template <>
struct Eng<float> {
    static constexpr int RM = 16, RN = 16, NA = 4;
    static constexpr int PAD = 16;
    typedef f4_t accv_t;
    __device__ static int arow(int lane) { return lane & 15; }
    __device__ static void mma(float a, float b, accv_t& c) { c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static double elem(const accv_t& c, int e) { return (double)c[e]; }
    __device__ static int orow(int lane, int e) { return 4 * (lane >> 4) + e; }
    __device__ static void zero(accv_t& c) { c = f4_t{0.f, 0.f, 0.f, 0.f}; }
};

// FP32 accumulators are added into FP64 every KFLUSH rows of K.
constexpr int KFLUSH = 512;

template <typename OUT>
__device__ __forceinline__ void store_out(OUT* p, int beta, double v) {
    *p = beta ? (OUT)((double)*p + v) : (OUT)v;
}

// ---------------------------------------------------------------------------
// Strassen product tiles (ATA_OPT_PRODUCT_TILES): TK_GEMM tasks whose
// operands are signed sums of up to TMAX terms (quadrant blocks of A),
// summed in term order while staging through registers; a term's columns
// past its end (padding) stage as zero.  128 x 128 output tile per
// workgroup, four waves of 64 x 64, double-buffered LDS, two workgroups per
// CU, K staged 8 rows at a time to bound the registers that hold the terms
// in flight.  (One-term tiles run on k_gemmd below.)
// ---------------------------------------------------------------------------
constexpr int GT = kGemmTile;  // 128

template <typename T, typename OUT, int TMAX>
__global__ void __launch_bounds__(256, 2) k_gemm(const T* __restrict__ A, int64_t lda,
                                                 const DevTask* __restrict__ tasks,
                                                 const DevTerm* __restrict__ terms,
                                                 const int32_t* __restrict__ segs,
                                                 const WorkItem* __restrict__ items, OUT* __restrict__ C,
                                                 double* __restrict__ W) {
    typedef Eng<T> E;
    static_assert(TMAX > 1, "multi-term operands");
    constexpr bool F32 = std::is_same<T, float>::value;
    constexpr int BR = 64 / E::RM, BC = 64 / E::RN;
    constexpr int GK = 8;                 // k rows per stage
    constexpr int EPT = GK * GT / 256;    // elements per thread, term and side
    constexpr int TPR = GT / EPT;         // threads per staged row
    __shared__ T Xs[2][GK][GT + E::PAD];
    __shared__ T Ys[2][GK][GT + E::PAD];

    const WorkItem w = items[blockIdx.x];
    const DevTask t = tasks[w.task];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int i0 = w.ti * GT, j0 = w.tj * GT;

    // staging map: thread -> row lk of the k tile, EPT consecutive columns at lc
    const int lk = tid / TPR, lc = (tid % TPR) * EPT;
    const int64_t row_bytes = lda * (int64_t)sizeof(T);
    constexpr uint32_t ES = (uint32_t)sizeof(T);
    // per term and element: byte offset inside a slab; a term's padding
    // columns get kOOB and stage as zero
    uint32_t xo[TMAX][EPT], yo[TMAX][EPT];
    T xsgn[TMAX], ysgn[TMAX];
#pragma unroll
    for (int u = 0; u < TMAX; ++u) {
        xsgn[u] = ysgn[u] = T(0);
#pragma unroll
        for (int e = 0; e < EPT; ++e) xo[u][e] = yo[u][e] = kOOB;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int nt = side == 0 ? t.nx : t.ny;
            if (u >= nt) continue;
            const DevTerm tm = terms[t.term_off + (side == 0 ? u : t.nx + u)];
            const int col = tm.col + (side == 0 ? i0 : j0) + lc;
            const uint32_t base = (uint32_t)(lk * row_bytes) + (uint32_t)col * ES;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const uint32_t off = col + e < tm.cvend ? base + e * ES : kOOB;
                if (side == 0) xo[u][e] = off;
                else yo[u][e] = off;
            }
            if (side == 0) xsgn[u] = (T)tm.sign;
            else ysgn[u] = (T)tm.sign;
        }
    }

    typename E::accv_t acc[BR][BC];
    double acc64[F32 ? BR : 1][F32 ? BC : 1][F32 ? E::NA : 1];
#pragma unroll
    for (int a = 0; a < BR; ++a)
#pragma unroll
        for (int b = 0; b < BC; ++b) E::zero(acc[a][b]);
    if (F32) {
#pragma unroll
        for (int a = 0; a < (F32 ? BR : 1); ++a)
#pragma unroll
            for (int b = 0; b < (F32 ? BC : 1); ++b)
#pragma unroll
                for (int e = 0; e < (F32 ? E::NA : 1); ++e) acc64[a][b][e] = 0.0;
    }

    // k-tile cursor over the segments: rows row_u + k for k in [kbeg, kend)
    const int stride = kSegHdr + 2 * (t.nx + t.ny);
    int seg = 0;
    int k0 = t.nseg > 0 ? segs[t.seg_off + 1] : 0;
    int kend = t.nseg > 0 ? segs[t.seg_off + 2] : 0;
    int ntiles = 0;
    for (int s = 0; s < t.nseg; ++s)
        ntiles += (segs[t.seg_off + s * stride + 2] - segs[t.seg_off + s * stride + 1] + GK - 1) / GK;

    T xr[TMAX][EPT], yr[TMAX][EPT];
    // Issue the loads of the k tile at k0: the slab of term u holds its rows
    // below both the window end and the term's row end.
    auto load = [&]() {
        const int32_t* sg = segs + t.seg_off + seg * stride;
        const int krem = kend - k0;
#pragma unroll
        for (int u = 0; u < TMAX; ++u) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int nt = side == 0 ? t.nx : t.ny;
                const int h = side == 0 ? 2 * u : 2 * (t.nx + u);
                const int row0 = u < nt ? sg[kSegHdr + h] : 0;
                const int rvend = u < nt ? sg[kSegHdr + 1 + h] : 0;
                const int base = row0 + k0;
                int nv = rvend - base < krem ? rvend - base : krem;
                nv = nv < GK ? nv : GK;
                const rsrc_t rs = slab_rsrc(A + (int64_t)base * lda, u < nt ? nv : 0, row_bytes);
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    if (side == 0) xr[u][e] = bload<T>(rs, xo[u][e]);
                    else yr[u][e] = bload<T>(rs, yo[u][e]);
                }
            }
        }
    };
    auto advance = [&]() {
        k0 += GK;
        if (k0 >= kend) {
            ++seg;
            if (seg < t.nseg) {
                k0 = segs[t.seg_off + seg * stride + 1];
                kend = segs[t.seg_off + seg * stride + 2];
            }
        }
    };

    if (ntiles > 0) load();
    for (int it = 0; it < ntiles; ++it) {
        const int buf = it & 1;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            T x = xsgn[0] * xr[0][e];
            T y = ysgn[0] * yr[0][e];
#pragma unroll
            for (int u = 1; u < TMAX; ++u) {
                x += xsgn[u] * xr[u][e];
                y += ysgn[u] * yr[u][e];
            }
            Xs[buf][lk][lc + e] = x;
            Ys[buf][lk][lc + e] = y;
        }
        __syncthreads();
        if (it + 1 < ntiles) {
            advance();
            load();
        }
        // issue priority for the MFMA section over the other workgroup's staging
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < GK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            T bv[BC];
#pragma unroll
            for (int cf = 0; cf < BC; ++cf) bv[cf] = Ys[buf][kr][wn * 64 + cf * E::RN + (lane & 15)];
#pragma unroll
            for (int rb = 0; rb < BR; ++rb) {
                const T av = Xs[buf][kr][wm * 64 + rb * E::RM + E::arow(lane)];
#pragma unroll
                for (int cf = 0; cf < BC; ++cf) E::mma(av, bv[cf], acc[rb][cf]);
            }
        }
        __builtin_amdgcn_s_setprio(0);
        if (F32 && (((it + 1) * GK) % KFLUSH == 0 || it + 1 == ntiles)) {
#pragma unroll
            for (int a = 0; a < BR; ++a)
#pragma unroll
                for (int b = 0; b < BC; ++b) {
#pragma unroll
                    for (int e = 0; e < E::NA; ++e) acc64[F32 ? a : 0][F32 ? b : 0][F32 ? e : 0] += E::elem(acc[a][b], e);
                    E::zero(acc[a][b]);
                }
        }
    }

    // epilogue: rows of D go to C rows r0 + gi, columns to C columns q0 + gj
    const bool syrk = t.kind == TK_SYRK;
#pragma unroll
    for (int rb = 0; rb < BR; ++rb) {
#pragma unroll
        for (int e = 0; e < E::NA; ++e) {
            const int gi = i0 + wm * 64 + rb * E::RM + E::orow(lane, e);
            if (gi >= t.dM) continue;
            const int64_t rowbase = packed_index((int64_t)t.r0 + gi, t.q0);
#pragma unroll
            for (int cf = 0; cf < BC; ++cf) {
                const int gj = j0 + wn * 64 + cf * E::RN + (lane & 15);
                if (gj >= t.dN || (syrk && gj > gi)) continue;
                const double v = F32 ? acc64[F32 ? rb : 0][F32 ? cf : 0][F32 ? e : 0] : E::elem(acc[rb][cf], e);
                if (t.dst == 0)
                    store_out(C + rowbase + gj, t.beta, v);
                else
                    W[t.ws_off + (int64_t)gi * t.N + gj] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Classical tile kernel with direct-to-LDS staging: the one-term tasks and
// 128 x 128 tiles of k_gemm (TK_SYRK / TK_GEMM leaves and operand-sum
// products; BATCH: tiles of several requests in one launch), two workgroups
// of four 64 x 64 waves per CU.  Operand rows are copied from global memory
// straight into LDS by buffer loads that write LDS (one dword per lane; rows
// outside the slab read as zero, columns past an operand's end feed only
// outputs that are never stored).  The copies of stage s + 1 are spread over
// the MFMA steps of stage s, so no registers hold staged data and the loop
// never waits on global memory except at the stage barrier.  Plane columns
// are XOR-swizzled by k row so that the four k rows an MFMA step reads fall
// in different LDS banks (FP64: left operand in 32-byte, right operand in
// 128-byte units; FP32: both in 64-byte units).  FP32 accumulates in FP32
// MFMA and adds into FP64 every KFLUSH rows, as k_gemm does.
// ---------------------------------------------------------------------------
// Copy of a table record addressed through a global-memory pointer, read as
// 32-bit words (the records are multiples of four bytes).
template <typename S>
__device__ __forceinline__ S load_rec(const __attribute__((address_space(1))) S* p) {
    static_assert(sizeof(S) % 4 == 0, "record size");
    S v;
    const __attribute__((address_space(1))) int32_t* q = (const __attribute__((address_space(1))) int32_t*)p;
    int32_t* d = reinterpret_cast<int32_t*>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(S) / 4); ++i) d[i] = q[i];
    return v;
}

// One 16-byte buffer load per lane into LDS at lds + 16 * lane.  (A plain
// device function: the host pass does not know the 16-byte form, which
// would otherwise fail the host-side instantiation of the kernel templates.)
__device__ __forceinline__ void lds_copy16(rsrc_t r, void* lds, uint32_t voff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds, 16, voff, 0, 0, 0);
}

template <typename T>
struct DmaCfg;
template <>
struct DmaCfg<double> {
    static constexpr int GK = 16;  // k rows per stage (64 KB of LDS, two workgroups per CU)
};
template <>
struct DmaCfg<float> {
    static constexpr int GK = 16;
};

// SPLIT: every item is part (slot mod nparts) of a K-split tile: it runs
// that share of the tile's stages and writes its raw FP64 result to tile
// slot of `part` (summed by k_tile_part_sum).
template <typename T, typename OUT, bool BATCH, bool SPLIT = false>
__global__ void __launch_bounds__(256, 2) k_gemmd(const T* __restrict__ A_, int64_t lda_,
                                                 const DevTask* __restrict__ tasks_,
                                                 const int32_t* __restrict__ segs_,
                                                 const WorkItem* __restrict__ items, OUT* __restrict__ C_,
                                                 double* __restrict__ W, const DevTerm* __restrict__ terms_,
                                                 const T* __restrict__ Aops, const BatchEntry* __restrict__ batch,
                                                 int nparts, double* __restrict__ part) {
    typedef Eng<T> E;
    constexpr bool F32 = std::is_same<T, float>::value;
    constexpr int GK = DmaCfg<T>::GK;
    static_assert(GK % 8 == 0 && GK <= 2 * kStageRows, "stage rows");
    constexpr int BR = 64 / E::RM, BC = 64 / E::RN;
    constexpr int PLANE = GK * GT;                 // elements per operand plane (k rows x 128 columns)
    constexpr int NP = GK / 4;                     // MFMA steps per stage = copy parts per stage
    constexpr int CPR = GT * (int)sizeof(T) / 256;  // 256-byte copies per plane row
    constexpr int NSL = (GK + kStageRows - 1) / kStageRows;  // slabs of at most kStageRows rows
    __shared__ __attribute__((aligned(16))) T lds[2][2][PLANE];  // [buffer][operand]

    // Table pointers typed as global memory: loads through a generic
    // pointer count as divergent (it could address per-lane memory), which
    // would put every resource built from the loaded values in a loop.
    typedef const __attribute__((address_space(1))) DevTask* TaskP;
    typedef const __attribute__((address_space(1))) DevTerm* TermP;
    typedef const __attribute__((address_space(1))) int32_t* SegP;
    const WorkItem w = items[blockIdx.x];
    const T* __restrict__ A = A_;
    OUT* __restrict__ C = C_;
    TaskP tasks = (TaskP)tasks_;
    TermP terms = (TermP)terms_;
    SegP segs = (SegP)segs_;
    int64_t lda = lda_;
    if (BATCH) {
        const BatchEntry be = batch[w.slot];
        A = (const T*)be.A;
        C = (OUT*)be.C;
        tasks = (TaskP)be.tasks;
        terms = (TermP)be.terms;
        segs = (SegP)be.segs;
        lda = be.lda;
    }
    const DevTask t = load_rec(tasks + w.task);
    if (!BATCH && t.src == 1) {  // operands from the task's operand-sum buffer
        A = Aops + t.src_off;
        lda = (int64_t)t.M + t.N;
    }
    const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int i0 = w.ti * GT, j0 = w.tj * GT;
    const int64_t row_bytes = lda * (int64_t)sizeof(T);

    // Copy role: operand cs (0: left X, 1: right Y), k rows of parity cpar.
    // Byte offset of this lane's dword per row residue (mod 4, the two of
    // this parity) and per 256-byte copy of the row.
    // FP32 (D16): 16-byte copies instead, each moving two adjacent 512-byte
    // rows (lanes 0-31 the first, 32-63 the second); the wave copies row
    // pairs 2j + cpar, whose rows r have r mod 4 = 2 cpar + (lane / 32), so
    // one offset per lane serves every copy.
    constexpr bool D16 = F32;
    const int cs = wave >> 1, cpar = wave & 1;
    const int swx = F32 ? 4 : 2, swy = 4;  // swizzle unit: 1 << swx (left) / 1 << swy (right) elements
    uint32_t doff[2][CPR];
    uint32_t doff16 = 0;
    {
        const DevTerm tm = load_rec(terms + t.term_off + (cs == 0 ? 0 : t.nx));
        const int colbase = tm.col + (cs == 0 ? i0 : j0);
        if (D16) {
            const int r4 = 2 * cpar + (lane >> 5);
            const int c = (4 * (lane & 31)) ^ (r4 << (cs == 0 ? swx : swy));  // first column of the chunk
            doff16 = (uint32_t)(colbase + c) * (uint32_t)sizeof(T);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r4 = cpar + 2 * q;
            const int sw = r4 << (cs == 0 ? swx : swy);
#pragma unroll
            for (int h = 0; h < CPR; ++h) {
                const int s = h * 64 + lane;            // dword within the row
                const int c = (F32 ? s : s >> 1) ^ sw;  // column that dword belongs to
                doff[q][h] = (uint32_t)(colbase + c) * (uint32_t)sizeof(T) + (F32 ? 0u : 4u * (uint32_t)(s & 1));
            }
        }
    }

    typename E::accv_t acc[BR][BC];
    double acc64[F32 ? BR : 1][F32 ? BC : 1][F32 ? E::NA : 1];
#pragma unroll
    for (int a = 0; a < BR; ++a)
#pragma unroll
        for (int b = 0; b < BC; ++b) {
            E::zero(acc[a][b]);
            if (F32)
#pragma unroll
                for (int e = 0; e < E::NA; ++e) acc64[F32 ? a : 0][F32 ? b : 0][F32 ? e : 0] = 0.0;
        }

    // k cursor over the segments: rows row_u + k for k in [kbeg, kend)
    const int stride = kSegHdr + 2 * (t.nx + t.ny);
    int seg = 0;
    int k0 = t.nseg > 0 ? segs[t.seg_off + 1] : 0;
    int kend = t.nseg > 0 ? segs[t.seg_off + 2] : 0;
    int ntiles = 0;
    for (int s = 0; s < t.nseg; ++s)
        ntiles += (segs[t.seg_off + s * stride + 2] - segs[t.seg_off + s * stride + 1] + GK - 1) / GK;

    // Slabs of this wave's operand for the stage at k0 (kStageRows rows each,
    // so every in-slab offset stays below kOOB): rows below both the window
    // end and the operand's row end; the rest read as zero.  Past the last
    // stage (live false) the slabs are empty and nothing is copied.
    rsrc_t rs[NSL];
    auto slab = [&](bool live) {
        const SegP sg = segs + t.seg_off + (live ? seg : 0) * stride;
        const int h = cs == 0 ? 0 : 2 * t.nx;
        const int base = (live ? sg[kSegHdr + h] : 0) + k0;
        const int rvend = live ? sg[kSegHdr + 1 + h] : 0;
        int nv = rvend - base < kend - k0 ? rvend - base : kend - k0;
        nv = nv < GK ? nv : GK;
        if (!live) nv = 0;
#pragma unroll
        for (int b = 0; b < NSL; ++b) {
            const int ns = nv - b * kStageRows;
            rs[b] = slab_rsrc(A + (int64_t)(base + b * kStageRows) * lda, ns < kStageRows ? ns : kStageRows,
                              row_bytes);
        }
    };
    // Copy part j of the stage into buffer `buf`: this wave's k rows
    // 2(2j) + cpar and 2(2j + 1) + cpar.  Nothing is copied past the last
    // stage, so no copy is in flight when the workgroup ends.  (The test also
    // keeps the copies in a block of their own, which bounds how far the
    // scheduler moves the next step's reads.)
    const int cnt = cs == 0 ? t.nx : t.ny;
    bool copying = false;  // the stage being copied exists
    auto copy_part = [&](int buf, int j) {
        if (cnt <= 0 || !copying) return;
        T* pl = lds[buf][cs];
        if constexpr (D16) {
            static_assert(GT * sizeof(T) == 512 && GK == kStageRows, "two rows per copy, one slab per stage");
            const int r = 2 * (2 * j + cpar) + (lane >> 5);  // this lane's row
            lds_copy16(rs[0], pl + 2 * (2 * j + cpar) * GT, (uint32_t)(r * row_bytes) + doff16);
            return;
        }
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
            const int r = 2 * (2 * j + ii) + cpar;
            const int q = (r >> 1) & 1;  // (r & 3) == cpar + 2 q
#pragma unroll
            for (int h = 0; h < CPR; ++h)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rs[r / kStageRows], (__attribute__((address_space(3))) void*)(pl + r * GT + h * (256 / (int)sizeof(T))),
                    4, (uint32_t)((r % kStageRows) * row_bytes) + doff[q][h], 0, 0, 0);
        }
    };
    auto advance = [&]() {
        k0 += GK;
        if (k0 >= kend) {
            ++seg;
            if (seg < t.nseg) {
                k0 = segs[t.seg_off + seg * stride + 1];
                kend = segs[t.seg_off + seg * stride + 2];
            }
        }
    };

    if constexpr (SPLIT) {
        const int tp = w.slot % nparts;
        const int s0 = (int)((int64_t)ntiles * tp / nparts), s1 = (int)((int64_t)ntiles * (tp + 1) / nparts);
        for (int u = 0; u < s0; ++u) advance();
        ntiles = s1 - s0;
    }
    if (ntiles > 0) {
        slab(true);
        copying = true;
#pragma unroll
        for (int j = 0; j < NP; ++j) copy_part(0, j);
    }
    for (int it = 0; it < ntiles; ++it) {
        const int buf = it & 1;
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of stage it have landed
        __syncthreads();                // every copy of stage it landed; stage it-1 fully read
        const bool next = it + 1 < ntiles;
        if (next) advance();
        slab(next);
        copying = next;
        const T* xp = lds[buf][0];
        const T* yp = lds[buf][1];
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < NP; ++ks) {
            const int kr = (ks * 4 + g) * GT;
            T av[BR], bv[BC];
#pragma unroll
            for (int cf = 0; cf < BC; ++cf)
                bv[cf] = yp[kr + ((wn * 64 + cf * E::RN + (lane & 15)) ^ (g << swy))];
#pragma unroll
            for (int rb = 0; rb < BR; ++rb)
                av[rb] = xp[kr + ((wm * 64 + rb * E::RM + E::arow(lane)) ^ (g << swx))];
            copy_part(buf ^ 1, ks);
#pragma unroll
            for (int rb = 0; rb < BR; ++rb)
#pragma unroll
                for (int cf = 0; cf < BC; ++cf) E::mma(av[rb], bv[cf], acc[rb][cf]);
        }
        __builtin_amdgcn_s_setprio(0);
        if (F32 && (((it + 1) * GK) % KFLUSH == 0 || it + 1 == ntiles)) {
#pragma unroll
            for (int a = 0; a < BR; ++a)
#pragma unroll
                for (int b = 0; b < BC; ++b) {
#pragma unroll
                    for (int e = 0; e < E::NA; ++e)
                        acc64[F32 ? a : 0][F32 ? b : 0][F32 ? e : 0] += E::elem(acc[a][b], e);
                    E::zero(acc[a][b]);
                }
        }
    }

    // epilogue: rows of D go to C rows r0 + gi, columns to C columns q0 + gj
    if constexpr (SPLIT) {
        double* pt = part + (int64_t)w.slot * GT * GT;
#pragma unroll
        for (int rb = 0; rb < BR; ++rb)
#pragma unroll
            for (int e = 0; e < E::NA; ++e)
#pragma unroll
                for (int cf = 0; cf < BC; ++cf)
                    pt[(wm * 64 + rb * E::RM + E::orow(lane, e)) * GT + wn * 64 + cf * E::RN + (lane & 15)] =
                        F32 ? acc64[F32 ? rb : 0][F32 ? cf : 0][F32 ? e : 0] : E::elem(acc[rb][cf], e);
        return;
    }
    const bool syrk = t.kind == TK_SYRK;
#pragma unroll
    for (int rb = 0; rb < BR; ++rb) {
#pragma unroll
        for (int e = 0; e < E::NA; ++e) {
            const int gi = i0 + wm * 64 + rb * E::RM + E::orow(lane, e);
            if (gi >= t.dM) continue;
            const int64_t rowbase = packed_index((int64_t)t.r0 + gi, t.q0);
#pragma unroll
            for (int cf = 0; cf < BC; ++cf) {
                const int gj = j0 + wn * 64 + cf * E::RN + (lane & 15);
                if (gj >= t.dN || (syrk && gj > gi)) continue;
                const double v = F32 ? acc64[F32 ? rb : 0][F32 ? cf : 0][F32 ? e : 0] : E::elem(acc[rb][cf], e);
                if (t.dst == 0)
                    store_out(C + rowbase + gj, t.beta, v);
                else
                    W[t.ws_off + (int64_t)gi * t.N + gj] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 tile kernel with 16-byte direct-to-LDS copies and 128-bit operand
// reads (k_tile): classical tiles (one term per operand: TK_SYRK / TK_GEMM
// leaves and the products of the operand-sum form) and Strassen product
// tiles whose operands are signed sums of two quadrant terms.  128 x 128
// output tile, four waves of 64 x 64, 16 k rows per stage, double-buffered
// LDS (64 KB), two workgroups per CU.
//
// Copies: one buffer load that writes LDS moves a whole 1 KB tile row (16
// bytes per lane).  The 16-byte chunks of row r sit at chunk position
// c ^ ((r & 3) << 2), so the four k rows an MFMA step reads fall in four
// different 64-byte bank groups.
//
// Operand reads: a 128-bit read gives each lane two neighbouring columns, so
// one read serves two MFMA blocks.  The FP64 4x4x4 MFMA takes the left
// operand as 4 rows x 4 k, repeated in its four lane quads (it has no
// broadcast of a single block), so the left side reads 4-row slots: slot
// (block 2q + h, row i) of a wave holds column 8q + 2i + h; the right side
// reads 16-column slots: slot (block 2u + h, column j) holds column
// 32u + 2j + h.  The epilogue maps the slots back.
//
// Two-term operands: the first term is copied into the operand's plane as
// above; the second is loaded into registers by the same wave and added into
// the plane with LDS atomic adds (x0 + s x1 with s = +-1: one rounding, as
// the sum in the product's definition) once the first has landed.  Each
// element is summed once per workgroup by the LDS unit, so the MFMA loop
// reads one plane per operand, exactly as for classical tiles, and runs no
// FP64 vector adds.  The product's overall sign is applied to the result.
// A term's columns past its end read as zero: whole chunks past the end get
// an out-of-range offset, and the one chunk that straddles the end (odd
// column counts) has its tail cleared.
// ---------------------------------------------------------------------------
typedef double d2_t __attribute__((ext_vector_type(2)));


// split: the item is part (slot mod nparts) of a K-split tile: it runs that
// share of the tile's stages and writes its raw result to tile slot of part.
template <typename OUT, int NT>
__device__ __forceinline__ void tile_body(const WorkItem w, const double* __restrict__ A_, int64_t lda_,
                                          const DevTask* __restrict__ tasks_, const DevTerm* __restrict__ terms_,
                                          const int32_t* __restrict__ segs_, OUT* __restrict__ C,
                                          double* __restrict__ W, const double* __restrict__ Aops,
                                          int nparts = 1, double* __restrict__ part = nullptr, bool split = false) {
    constexpr int GK = 16;               // k rows per stage
    static_assert(GK <= kStageRows, "one slab per stage");
    constexpr int NP = GK / 4;           // MFMA steps per stage
    constexpr int PLANE = GK * GT;       // doubles per plane
    constexpr int RPW = GK / 2;          // rows a wave copies per stage (two waves per operand)
    __shared__ __attribute__((aligned(16))) double lds[2][2][PLANE];  // [buffer][operand]

    typedef const __attribute__((address_space(1))) DevTask* TaskP;
    typedef const __attribute__((address_space(1))) DevTerm* TermP;
    typedef const __attribute__((address_space(1))) int32_t* SegP;
    const double* __restrict__ A = A_;
    int64_t lda = lda_;
    const TaskP tasks = (TaskP)tasks_;
    const TermP terms = (TermP)terms_;
    const SegP segs = (SegP)segs_;
    const DevTask t = load_rec(tasks + w.task);
    if (t.src == 1) {  // operands from the task's operand-sum buffer
        A = Aops + t.src_off;
        lda = (int64_t)t.M + t.N;
    }
    const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int i0 = w.ti * GT, j0 = w.tj * GT;
    const int64_t row_bytes = lda * (int64_t)sizeof(double);

    // Copy role: operand cs (0: left X, 1: right Y), k rows of parity cpar.
    // Per term and per row residue (r & 3 is cpar or cpar + 2): the byte
    // offset of the 16-byte chunk this lane copies, kOOB past the term's end.
    const int cs = wave >> 1, cpar = wave & 1;
    const int cnt = NT > 1 ? (cs == 0 ? t.nx : t.ny) : 1;  // terms of this wave's operand
    uint32_t doff[NT][2];
    int tail[NT];  // valid columns of the term in this tile when a chunk straddles its end, else 0
    double osgn, s1 = 1.0;  // overall sign; sign of the second term relative to the first
    {
        const DevTerm x0 = load_rec(terms + t.term_off);
        const DevTerm y0 = load_rec(terms + t.term_off + t.nx);
        osgn = (double)(x0.sign * y0.sign);
        if (NT > 1 && cnt > 1)
            s1 = (double)((cs == 0 ? x0.sign : y0.sign) *
                          load_rec(terms + t.term_off + (cs == 0 ? 1 : t.nx + 1)).sign);
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        doff[u][0] = doff[u][1] = kOOB;
        tail[u] = 0;
        if (u < cnt) {
            const DevTerm tm = load_rec(terms + t.term_off + (cs == 0 ? u : t.nx + u));
            const int colbase = tm.col + (cs == 0 ? i0 : j0);
            const int nvalid = tm.cvend - colbase;  // columns of the term from the tile start on
            if (NT > 1 && nvalid > 0 && nvalid < GT && (nvalid & 1)) tail[u] = nvalid;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int c = lane ^ ((cpar + 2 * p) << 2);  // logical chunk this lane copies
                doff[u][p] = 2 * c < nvalid ? (uint32_t)(colbase + 2 * c) * 8u : kOOB;
            }
        }
    }

    double acc[16][4];
#pragma unroll
    for (int a = 0; a < 16; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;

    // k cursor over the segments: rows row_u + k for k in [kbeg, kend)
    const int stride = kSegHdr + 2 * (t.nx + t.ny);
    int seg = 0;
    int k0 = t.nseg > 0 ? segs[t.seg_off + 1] : 0;
    int kend = t.nseg > 0 ? segs[t.seg_off + 2] : 0;
    int ntiles = 0;
    for (int s = 0; s < t.nseg; ++s)
        ntiles += (segs[t.seg_off + s * stride + 2] - segs[t.seg_off + s * stride + 1] + GK - 1) / GK;

    // Slab of each term of this wave's operand for the stage at k0: rows
    // below both the window end and the term's row end; the rest read as zero.
    rsrc_t rs[NT];
    auto slab = [&](bool live) {
        const SegP sg = segs + t.seg_off + (live ? seg : 0) * stride;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int h = 2 * ((cs == 0 ? 0 : t.nx) + u);
            const bool on = live && u < cnt;
            const int base = (on ? sg[kSegHdr + h] : 0) + k0;
            const int rvend = on ? sg[kSegHdr + 1 + h] : 0;
            int nv = rvend - base < kend - k0 ? rvend - base : kend - k0;
            nv = nv < GK ? nv : GK;
            if (!on) nv = 0;
            rs[u] = slab_rsrc(A + (int64_t)base * lda, nv, row_bytes);
        }
    };
    // Row i of this wave's rows (2 i + cpar) of the current stage: the first
    // term copied into LDS, the second loaded into registers.  Nothing is
    // copied past the last stage, so no copy is in flight when the workgroup
    // ends.
    bool copying = false;
    d2_t v1[NT > 1 ? RPW : 1];
    auto copy_row = [&](int buf, int i) {
        if (!copying) return;
        const int r = 2 * i + cpar;
        lds_copy16(rs[0], &lds[buf][cs][r * GT], (uint32_t)(r * row_bytes) + doff[0][i & 1]);
    };
    auto load_row = [&](int i) {
        if (!copying || !(NT > 1 && cnt > 1)) return;
        const int r = 2 * i + cpar;
        v1[NT > 1 ? i : 0] = __builtin_bit_cast(
            d2_t, __builtin_amdgcn_raw_buffer_load_b128(rs[NT - 1], (int)((uint32_t)(r * row_bytes) + doff[NT - 1][i & 1]),
                                                        0, 0));
    };
    auto advance = [&]() {
        k0 += GK;
        if (k0 >= kend) {
            ++seg;
            if (seg < t.nseg) {
                k0 = segs[t.seg_off + seg * stride + 1];
                kend = segs[t.seg_off + seg * stride + 2];
            }
        }
    };

    // Second terms: clear the tail of a straddling chunk of the first term in
    // the rows this wave copies (before any sum lands there), then add rows
    // [ia, ib) of the second term into the plane.  The first term's copy of
    // those rows must have landed.
    auto fix_tail = [&](int buf) {
        if (NT > 1 && tail[0] && lane < RPW) {
            const int r = 2 * lane + cpar;
            lds[buf][cs][r * GT + 2 * ((tail[0] >> 1) ^ ((r & 3) << 2)) + 1] = 0.0;
        }
    };
    auto add_rows = [&](int buf, int ia, int ib) {
        if (!(NT > 1 && cnt > 1)) return;
#pragma unroll
        for (int i = ia; i < ib; ++i) {
            const int r = 2 * i + cpar;
            d2_t v = v1[NT > 1 ? i : 0];
            if (tail[NT - 1] && (lane ^ ((r & 3) << 2)) == (tail[NT - 1] >> 1)) v[1] = 0.0;
            double* dst = &lds[buf][cs][r * GT + 2 * lane];
            __hip_atomic_fetch_add(dst, s1 * v[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(dst + 1, s1 * v[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };

    if (split) {
        const int tp = w.slot % nparts;
        const int s0 = (int)((int64_t)ntiles * tp / nparts), s1 = (int)((int64_t)ntiles * (tp + 1) / nparts);
        for (int u = 0; u < s0; ++u) advance();
        ntiles = s1 - s0;
    }
    if (ntiles > 0) {
        slab(true);
        copying = true;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            copy_row(0, i);
            load_row(i);
        }
    }
    for (int it = 0; it < ntiles; ++it) {
        const int buf = it & 1;
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies and loads of stage it have landed
        fix_tail(buf);
        add_rows(buf, 0, RPW);
        __syncthreads();  // every copy and sum of stage it is in LDS; stage it-1 fully read
        const bool next = it + 1 < ntiles;
        if (next) advance();
        slab(next);
        copying = next;
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < NP; ++ks) {
            const int kr = (ks * 4 + g) * GT;
            const int sw = g << 2;
            d2_t bv[2], av[8];
#pragma unroll
            for (int u = 0; u < 2; ++u)
                bv[u] = *(const d2_t*)&lds[buf][1][kr + 2 * ((wn * 32 + 16 * u + (lane & 15)) ^ sw)];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                av[q] = *(const d2_t*)&lds[buf][0][kr + 2 * ((wm * 32 + 4 * q + (lane & 3)) ^ sw)];
            // Every copy of the next stage goes out with the first step, so a
            // whole stage of MFMA work covers its latency.  The register loads
            // of second terms are spread over the steps (issued together they
            // would be live across the whole stage and spill).
            if (ks == 0) {
#pragma unroll
                for (int i = 0; i < RPW; ++i) copy_row(buf ^ 1, i);
            }
#pragma unroll
            for (int i = ks * (RPW / NP); i < (ks + 1) * (RPW / NP); ++i) load_row(i);
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int ha = 0; ha < 2; ++ha)
#pragma unroll
                    for (int cf = 0; cf < 4; ++cf)
                        acc[2 * q + ha][cf] =
                            __builtin_amdgcn_mfma_f64_4x4x4f64(av[q][ha], bv[cf >> 1][cf & 1], acc[2 * q + ha][cf], 0, 0, 0);
        }
        __builtin_amdgcn_s_setprio(0);
    }

    // epilogue: slot (2q + ha, row g) -> tile row 8q + 2g + ha of the wave,
    // slot (2u + hb, column j) -> tile column 32u + 2j + hb
    if (split) {
        double* pt = part + (int64_t)w.slot * GT * GT;
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int ha = 0; ha < 2; ++ha)
#pragma unroll
                for (int cf = 0; cf < 4; ++cf)
                    pt[(wm * 64 + 8 * q + 2 * g + ha) * GT + wn * 64 + 32 * (cf >> 1) + 2 * (lane & 15) + (cf & 1)] =
                        osgn * acc[2 * q + ha][cf];
        return;
    }
    const bool syrk = t.kind == TK_SYRK;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
#pragma unroll
        for (int ha = 0; ha < 2; ++ha) {
            const int gi = i0 + wm * 64 + 8 * q + 2 * g + ha;
            if (gi >= t.dM) continue;
            const int64_t rowbase = packed_index((int64_t)t.r0 + gi, t.q0);
#pragma unroll
            for (int cf = 0; cf < 4; ++cf) {
                const int gj = j0 + wn * 64 + 32 * (cf >> 1) + 2 * (lane & 15) + (cf & 1);
                if (gj >= t.dN || (syrk && gj > gi)) continue;
                const double v = osgn * acc[2 * q + ha][cf];
                if (t.dst == 0)
                    store_out(C + rowbase + gj, t.beta, v);
                else
                    W[t.ws_off + (int64_t)gi * t.N + gj] = v;
            }
        }
    }
}

template <typename OUT, int NT>
__global__ void __launch_bounds__(256, 2) k_tile(const double* __restrict__ A_, int64_t lda_,
                                                const DevTask* __restrict__ tasks_,
                                                const DevTerm* __restrict__ terms_,
                                                const int32_t* __restrict__ segs_,
                                                const WorkItem* __restrict__ items, OUT* __restrict__ C,
                                                double* __restrict__ W, const double* __restrict__ Aops) {
    tile_body<OUT, NT>(items[blockIdx.x], A_, lda_, tasks_, terms_, segs_, C, W, Aops);
}

// Persistent two-term launch: each workgroup takes items from the work queues
// until every queue is empty (at most eight probes per item, so every
// workgroup leaves the loop).  Queue x holds the items at positions x, x + 8,
// ...: the positions that a one-item-per-workgroup launch runs on XCD x, in
// the launch's longest-first order.  The queues start at zero.
template <typename OUT>
__global__ void __launch_bounds__(256, 2) k_tile_q(const double* __restrict__ A_, int64_t lda_,
                                                  const DevTask* __restrict__ tasks_,
                                                  const DevTerm* __restrict__ terms_,
                                                  const int32_t* __restrict__ segs_,
                                                  const WorkItem* __restrict__ items, OUT* __restrict__ C,
                                                  double* __restrict__ W, const double* __restrict__ Aops,
                                                  int* __restrict__ queue, int nitems) {
    __shared__ int s_item[2];
    const int home = blockIdx.x & 7;
#pragma clang loop unroll(disable)
    for (int round = 0;; ++round) {
        if (threadIdx.x == 0) {
            int got = nitems;
            for (int a = 0; a < 8; ++a) {
                const int x = (home + a) & 7;
                const int cnt = (nitems - x + 7) >> 3;
                if (cnt <= 0) continue;
                const int j = __hip_atomic_fetch_add(queue + x, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (j < cnt) {
                    got = 8 * j + x;
                    break;
                }
            }
            s_item[round & 1] = got;
        }
        __syncthreads();  // also: every wave is done with the previous item's LDS
        const int idx = __builtin_amdgcn_readfirstlane(s_item[round & 1]);
        if (idx >= nitems) break;
        tile_body<OUT, 2>(items[idx], A_, lda_, tasks_, terms_, segs_, C, W, Aops);
    }
}

// A one-term launch and its K-split last round in one grid: blocks
// [0, nmain) run the whole tiles of items, the rest the parts of tail, so
// parts start on CUs as the last whole tiles finish.
template <typename OUT>
__global__ void __launch_bounds__(256, 2) k_tile_cat(const double* __restrict__ A_, int64_t lda_,
                                                    const DevTask* __restrict__ tasks_,
                                                    const DevTerm* __restrict__ terms_,
                                                    const int32_t* __restrict__ segs_,
                                                    const WorkItem* __restrict__ items, int nmain,
                                                    const WorkItem* __restrict__ tail, OUT* __restrict__ C,
                                                    double* __restrict__ W, const double* __restrict__ Aops,
                                                    int nparts, double* __restrict__ part) {
    const int b = blockIdx.x;
    const bool split = b >= nmain;
    tile_body<OUT, 1>(split ? tail[b - nmain] : items[b], A_, lda_, tasks_, terms_, segs_, C, W, Aops, nparts, part,
                      split);
}

// Sum of the parts of the K-split tiles in part order, stored as k_tile
// stores a tile: block (li, q) covers row li of split tile q.
template <typename OUT>
__global__ void __launch_bounds__(GT) k_tile_part_sum(const DevTask* __restrict__ tasks,
                                                     const WorkItem* __restrict__ tail, int nparts,
                                                     const double* __restrict__ part, OUT* __restrict__ C,
                                                     double* __restrict__ W) {
    const int q = blockIdx.y, li = blockIdx.x, lj = threadIdx.x;
    const WorkItem w = tail[q * nparts];
    const DevTask t = tasks[w.task];
    const int gi = w.ti * GT + li, gj = w.tj * GT + lj;
    if (gi >= t.dM || gj >= t.dN || (t.kind == TK_SYRK && gj > gi)) return;
    double v = 0.0;
    for (int p = 0; p < nparts; ++p) v += part[((int64_t)(q * nparts + p) * GT + li) * GT + lj];
    if (t.dst == 0)
        store_out(C + packed_index((int64_t)t.r0 + gi, t.q0) + gj, t.beta, v);
    else
        W[t.ws_off + (int64_t)gi * t.N + gj] = v;
}

// ---------------------------------------------------------------------------
// In-tile Strassen kernel (TK_STR).  The product P = Xop^t Yop (padded M x N,
// K per segment) is split once more into quadrants; a workgroup owns the
// 64 x 64 tile at (ti, tj) of all four result quadrants and keeps the seven
// products in registers (eight waves of 16 x 32 each).  While a k tile is
// staged, each thread sums the operand terms of higher levels.  With
// single-term operands it also forms the seven left and seven right
// operands of this level from the four quadrant values it holds and writes
// them to fourteen LDS planes, which the MFMA loop reads directly; with
// multi-term operands (whose staging registers leave no room for that) it
// writes the four quadrant planes and the MFMA loop forms the sums in
// registers.  The products are combined in FP64.
// ---------------------------------------------------------------------------
constexpr int ST = kStrTile;  // 64

template <int VAR, typename T>
__device__ __forceinline__ void left_operands(T x00, T x01, T x10, T x11, T (&o)[7]) {
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
        const T s1 = x10 + x11, s2 = s1 - x00;
        o[0] = x00;
        o[1] = x01;
        o[2] = x01 - s2;
        o[3] = x11;
        o[4] = s1;
        o[5] = s2;
        o[6] = x00 - x10;
    }
}

template <int VAR, typename T>
__device__ __forceinline__ void right_operands(T y00, T y01, T y10, T y11, T (&o)[7]) {
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
        const T t1 = y01 - y00, t2 = y11 - t1;
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

template <typename T, typename OUT, int VAR, int TMAX, int SK>
__global__ void __launch_bounds__(512, 1) k_str(const T* __restrict__ A, int64_t lda,
                                                const DevTask* __restrict__ tasks,
                                                const DevTerm* __restrict__ terms,
                                                const int32_t* __restrict__ segs,
                                                const WorkItem* __restrict__ items, OUT* __restrict__ C,
                                                double* __restrict__ W) {
    typedef Eng<T> E;
    constexpr bool F32 = std::is_same<T, float>::value;
    constexpr int BR = 16 / E::RM, BC = 32 / E::RN;
    constexpr bool STAGED = TMAX == 1;  // operand sums formed while staging
    constexpr int NPL = STAGED ? 7 : 4;  // LDS planes per operand
    __shared__ T Xs[2][NPL][SK][ST + E::PAD];
    __shared__ T Ys[2][NPL][SK][ST + E::PAD];

    const WorkItem w = items[blockIdx.x];
    const DevTask t = tasks[w.task];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;  // 4 x 2 waves of 16 x 32
    const int MH = (t.M + 1) >> 1, NH = (t.N + 1) >> 1;
    const int i0 = w.ti * ST, j0 = w.tj * ST;
    const int stride = kSegHdr + 2 * (t.nx + t.ny);

    // staging map: thread -> k rows lk + 8r, column lc (one element per quadrant and row)
    const int lk = tid >> 6, lc = tid & 63;
    constexpr int KR = SK / 8;

    // Per-term column byte offsets, fixed for the whole K loop; a column
    // outside the term (quadrant padding) gets an out-of-range offset and
    // stages as zero.  Absent terms (u >= nx) have zero-row slabs.
    const int64_t row_bytes = lda * (int64_t)sizeof(T);
    uint32_t xoff[TMAX][2], yoff[TMAX][2];
    bool xneg[TMAX], yneg[TMAX];
    T xsgn[TMAX], ysgn[TMAX];
#pragma unroll
    for (int u = 0; u < TMAX; ++u) {
        xoff[u][0] = xoff[u][1] = yoff[u][0] = yoff[u][1] = kOOB;
        xneg[u] = yneg[u] = false;
        xsgn[u] = ysgn[u] = T(0);
        if (u < t.nx) {
            const DevTerm tm = terms[t.term_off + u];
            xsgn[u] = (T)tm.sign;
            xneg[u] = tm.sign < 0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int col = tm.col + a * MH + i0 + lc;
                if (i0 + lc < MH && col < tm.cvend) xoff[u][a] = (uint32_t)col * (uint32_t)sizeof(T);
            }
        }
        if (u < t.ny) {
            const DevTerm tm = terms[t.term_off + t.nx + u];
            ysgn[u] = (T)tm.sign;
            yneg[u] = tm.sign < 0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int col = tm.col + c * NH + j0 + lc;
                if (j0 + lc < NH && col < tm.cvend) yoff[u][c] = (uint32_t)col * (uint32_t)sizeof(T);
            }
        }
    }

    typename E::accv_t acc[7][BR][BC];
    double acc64[F32 ? 7 : 1][F32 ? BR : 1][F32 ? BC : 1][F32 ? E::NA : 1];
#pragma unroll
    for (int p = 0; p < 7; ++p)
#pragma unroll
        for (int a = 0; a < BR; ++a)
#pragma unroll
            for (int b = 0; b < BC; ++b) {
                E::zero(acc[p][a][b]);
                if (F32)
#pragma unroll
                    for (int e = 0; e < E::NA; ++e) acc64[F32 ? p : 0][F32 ? a : 0][F32 ? b : 0][F32 ? e : 0] = 0.0;
            }

    // per segment: K half length kh = ceil(klen / 2), window [kbeg, kend) of it
    int ntiles = 0;
    for (int s = 0; s < t.nseg; ++s)
        ntiles += (segs[t.seg_off + s * stride + 2] - segs[t.seg_off + s * stride + 1] + SK - 1) / SK;

    // raw term values of the next k tile: [term][row][quad]
    T xraw[TMAX][KR][4], yraw[TMAX][KR][4];
    int seg = 0;
    int kh = t.nseg > 0 ? (segs[t.seg_off] + 1) >> 1 : 0;
    int k0 = t.nseg > 0 ? segs[t.seg_off + 1] : 0;
    int kend = t.nseg > 0 ? segs[t.seg_off + 2] : 0;

    // Issue every load of the next k tile; nothing waits on them here.
    // Rows of half b of term u for this tile start at row0 + b kh + k0; the
    // slab holds those below both the window end and the term's row end.
    const uint32_t roff = (uint32_t)(lk * row_bytes);
    auto load = [&]() {
        const int32_t* sg = segs + t.seg_off + seg * stride;
        const int krem = kend - k0;
#pragma unroll
        for (int u = 0; u < TMAX; ++u) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int nt = side == 0 ? t.nx : t.ny;
                const int h = side == 0 ? 2 * u : 2 * (t.nx + u);
                const int row0 = u < nt ? sg[kSegHdr + h] : 0, rvend = u < nt ? sg[kSegHdr + 1 + h] : 0;
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int base = row0 + b * kh + k0;
                    int nv = rvend - base < krem ? rvend - base : krem;
                    nv = nv < SK ? nv : SK;
                    const rsrc_t rs = slab_rsrc(A + (int64_t)base * lda, u < nt ? nv : 0, row_bytes);
#pragma unroll
                    for (int r = 0; r < KR; ++r)
#pragma unroll
                        for (int a = 0; a < 2; ++a) {
                            const uint32_t off = roff + (uint32_t)(8 * r * row_bytes);
                            if (side == 0)
                                xraw[u][r][a * 2 + b] = bload<T>(rs, off + xoff[u][a]);
                            else
                                yraw[u][r][b * 2 + a] = bload<T>(rs, off + yoff[u][a]);
                        }
                }
            }
        }
    };
    // Signed sum of the terms (fixed order), then this level's seven left
    // and right operands, into the LDS buffer.
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            T x[4], y[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (TMAX == 1) {
                    x[q] = flip_sign(xraw[0][r][q], xneg[0]);
                    y[q] = flip_sign(yraw[0][r][q], yneg[0]);
                } else {
                    x[q] = xsgn[0] * xraw[0][r][q];
                    y[q] = ysgn[0] * yraw[0][r][q];
#pragma unroll
                    for (int u = 1; u < TMAX; ++u) {
                        x[q] += xsgn[u] * xraw[u][r][q];
                        y[q] += ysgn[u] * yraw[u][r][q];
                    }
                }
            }
            if constexpr (STAGED) {
                T lo[7], ro[7];
                left_operands<VAR>(x[0], x[1], x[2], x[3], lo);
                right_operands<VAR>(y[0], y[1], y[2], y[3], ro);
#pragma unroll
                for (int p = 0; p < 7; ++p) {
                    Xs[buf][p][lk + 8 * r][lc] = lo[p];
                    Ys[buf][p][lk + 8 * r][lc] = ro[p];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    Xs[buf][q][lk + 8 * r][lc] = x[q];
                    Ys[buf][q][lk + 8 * r][lc] = y[q];
                }
            }
        }
    };
    auto advance = [&]() {
        k0 += SK;
        if (k0 >= kend) {
            ++seg;
            if (seg < t.nseg) {
                kh = (segs[t.seg_off + seg * stride] + 1) >> 1;
                k0 = segs[t.seg_off + seg * stride + 1];
                kend = segs[t.seg_off + seg * stride + 2];
            }
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
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < SK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            T ro[BC][7];
#pragma unroll
            for (int cf = 0; cf < BC; ++cf) {
                const int cc = wn * 32 + cf * E::RN + (lane & 15);
                if constexpr (STAGED) {
#pragma unroll
                    for (int p = 0; p < 7; ++p) ro[cf][p] = Ys[buf][p][kr][cc];
                } else {
                    right_operands<VAR>(Ys[buf][0][kr][cc], Ys[buf][1][kr][cc], Ys[buf][2][kr][cc],
                                        Ys[buf][3][kr][cc], ro[cf]);
                }
            }
#pragma unroll
            for (int rb = 0; rb < BR; ++rb) {
                const int rr = wm * 16 + rb * E::RM + E::arow(lane);
                T lo[7];
                if constexpr (STAGED) {
#pragma unroll
                    for (int p = 0; p < 7; ++p) lo[p] = Xs[buf][p][kr][rr];
                } else {
                    left_operands<VAR>(Xs[buf][0][kr][rr], Xs[buf][1][kr][rr], Xs[buf][2][kr][rr],
                                       Xs[buf][3][kr][rr], lo);
                }
#pragma unroll
                for (int p = 0; p < 7; ++p)
#pragma unroll
                    for (int cf = 0; cf < BC; ++cf) E::mma(lo[p], ro[cf][p], acc[p][rb][cf]);
            }
        }
        __builtin_amdgcn_s_setprio(0);
        if (F32 && (((it + 1) * SK) % KFLUSH == 0 || it + 1 == ntiles)) {
#pragma unroll
            for (int p = 0; p < 7; ++p)
#pragma unroll
                for (int a = 0; a < BR; ++a)
#pragma unroll
                    for (int b = 0; b < BC; ++b) {
#pragma unroll
                        for (int e = 0; e < E::NA; ++e)
                            acc64[F32 ? p : 0][F32 ? a : 0][F32 ? b : 0][F32 ? e : 0] += E::elem(acc[p][a][b], e);
                        E::zero(acc[p][a][b]);
                    }
        }
    }

    // combine the seven products (FP64) into the four quadrants and store
#pragma unroll
    for (int rb = 0; rb < BR; ++rb) {
#pragma unroll
        for (int e = 0; e < E::NA; ++e) {
            const int li = i0 + wm * 16 + rb * E::RM + E::orow(lane, e);  // row inside a quadrant
#pragma unroll
            for (int cf = 0; cf < BC; ++cf) {
                const int lj = j0 + wn * 32 + cf * E::RN + (lane & 15);
                double m[7], d[4];
#pragma unroll
                for (int p = 0; p < 7; ++p)
                    m[p] = F32 ? acc64[F32 ? p : 0][F32 ? rb : 0][F32 ? cf : 0][F32 ? e : 0] : E::elem(acc[p][rb][cf], e);
                combine_products<VAR>(m, d);
                if (li >= MH || lj >= NH) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int gi = (q >> 1) * MH + li, gj = (q & 1) * NH + lj;
                    if (gi >= t.dM || gj >= t.dN) continue;
                    if (t.dst == 0)
                        store_out(C + packed_index((int64_t)t.r0 + gi, t.q0) + gj, t.beta, d[q]);
                    else
                        W[t.ws_off + (int64_t)gi * t.N + gj] = d[q];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Operand sums (operand-sum form): one workgroup per buffer row.  Row k of a
// record's buffer is row k of the concatenated chunk windows of its product;
// column c < M sums the X terms at column c of their quadrants, c >= M the Y
// terms at c - M, in term order and in the element type, zero where a term
// is padding (past its columns or rows).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_opsum(const T* __restrict__ A, int64_t lda,
                                               const DevTask* __restrict__ tasks,
                                               const DevTerm* __restrict__ terms,
                                               const int32_t* __restrict__ segs,
                                               const DevOpSum* __restrict__ recs, int nrec, T* __restrict__ out) {
    __shared__ int rsel;
    const int64_t g = blockIdx.x;
    if (threadIdx.x == 0) {
        int lo = 0, hi = nrec - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (recs[mid].row_off <= g) lo = mid;
            else hi = mid - 1;
        }
        rsel = lo;
    }
    __syncthreads();
    const DevOpSum rec = recs[rsel];
    const DevTask t = tasks[rec.task];
    // chunk (segment) of row k and the row inside its window
    int k = (int)(g - rec.row_off);
    const int stride = kSegHdr + 2 * (t.nx + t.ny);
    int s = 0;
    for (; s + 1 < t.nseg; ++s) {
        const int len = segs[t.seg_off + s * stride + 2] - segs[t.seg_off + s * stride + 1];
        if (k < len) break;
        k -= len;
    }
    const int32_t* sg = segs + t.seg_off + s * stride;
    const int kk = sg[1] + k;
    T* orow = out + rec.out_off + (int64_t)(g - rec.row_off) * (rec.M + rec.N);
    // Left operand (first M entries of the row), then the right one.  Terms
    // are the outer loop (uniform over the workgroup) and each thread keeps
    // the running sums of eight elements, so eight loads are in flight; every
    // element still adds its terms in term order.
    constexpr int CH = 8;
    for (int side = 0; side < 2; ++side) {
        const int nt = side == 0 ? t.nx : t.ny, u0 = side == 0 ? 0 : t.nx;
        const int width = side == 0 ? rec.M : rec.N;
        T* o = orow + (side == 0 ? 0 : rec.M);
        for (int c0 = 0; c0 < width; c0 += 256 * CH) {
            T v[CH];
            for (int u = 0; u < nt; ++u) {
                const DevTerm tm = terms[t.term_off + u0 + u];
                const int row = sg[kSegHdr + 2 * (u0 + u)] + kk;
                const bool rok = row < sg[kSegHdr + 2 * (u0 + u) + 1];
                const T sgn = (T)tm.sign;
                const T* src = A + (int64_t)row * lda + tm.col;
                T a[CH];
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    const int c = c0 + e * 256 + (int)threadIdx.x;
                    a[e] = (rok && c < width && tm.col + c < tm.cvend) ? src[c] : T(0);
                }
#pragma unroll
                for (int e = 0; e < CH; ++e) v[e] = u == 0 ? sgn * a[e] : v[e] + sgn * a[e];
            }
#pragma unroll
            for (int e = 0; e < CH; ++e) {
                const int c = c0 + e * 256 + (int)threadIdx.x;
                if (c < width) o[c] = v[e];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Combination of workspace products into an off-diagonal block of packed C.
// Each output element sums the workspace slots of its Strassen path with the
// signs of the combination formulas, over the K parts in part order, in
// FP64 (path order within a part).  One thread per element; one binary
// search per workgroup finds the block of its first element.
// ---------------------------------------------------------------------------
__constant__ int c_dcoef[2][7][4] = ATA_D_COEF;

// For one expanded level: the (at most four) products that enter result
// quadrant q, in product order, with their signs (0 pads the list).
struct QuadSlots {
    int path[2][4][4];
    int sign[2][4][4];
};
constexpr QuadSlots make_quad_slots() {
    QuadSlots t{};
    constexpr int d[2][7][4] = ATA_D_COEF;
    for (int v = 0; v < 2; ++v)
        for (int q = 0; q < 4; ++q) {
            int k = 0;
            for (int p = 0; p < 7; ++p)
                if (d[v][p][q] != 0 && k < 4) {
                    t.path[v][q][k] = p;
                    t.sign[v][q][k] = d[v][p][q];
                    ++k;
                }
        }
    return t;
}
__constant__ QuadSlots c_qslots = make_quad_slots();

template <typename OUT>
__global__ void __launch_bounds__(256) k_combine(const DevCombine* __restrict__ cbs, int ncb, int64_t total,
                                                 const double* __restrict__ W, OUT* __restrict__ C) {
    __shared__ int first;
    const int64_t e0 = (int64_t)blockIdx.x * 256;
    if (threadIdx.x == 0) {
        int lo = 0, hi = ncb - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cbs[mid].elem_off <= e0) lo = mid;
            else hi = mid - 1;
        }
        first = lo;
    }
    __syncthreads();
    const int64_t e = e0 + threadIdx.x;
    if (e >= total) return;
    int idx = first;
    while (idx + 1 < ncb && cbs[idx + 1].elem_off <= e) ++idx;
    const DevCombine& cb = cbs[idx];
    const int64_t loc = e - cb.elem_off;
    int i, j;
    if (loc < 0x100000000ll) {
        const uint32_t l32 = (uint32_t)loc, n32 = (uint32_t)cb.N;
        i = (int)(l32 / n32);
        j = (int)(l32 - (uint32_t)i * n32);
    } else {
        i = (int)(loc / cb.N);
        j = (int)(loc - (int64_t)i * cb.N);
    }
    if (cb.lower && j > i) return;
    // quadrant path of (i, j), first level in the most significant digit
    int ii = i, jj = j, Mc = cb.M, Nc = cb.N, qcode = 0;
    for (int l = 0; l < cb.levels; ++l) {
        const int MH = (Mc + 1) >> 1, NH = (Nc + 1) >> 1;
        const int a = ii >= MH, c = jj >= NH;
        ii -= a * MH;
        jj -= c * NH;
        qcode = qcode * 4 + a * 2 + c;
        Mc = MH;
        Nc = NH;
    }
    const int64_t slot_elems = (int64_t)cb.Mp * cb.Np;
    const double* base = W + cb.ws_off + (int64_t)ii * cb.Np + jj;
    double sum = 0.0;
    if (cb.levels == 1 && cb.nparts == 1) {
        // one level: load the quadrant's products together, then sum in order
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = base[c_qslots.path[cb.variant][qcode][k] * slot_elems];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int sg = c_qslots.sign[cb.variant][qcode][k];
            if (sg) sum += sg > 0 ? v[k] : -v[k];
        }
    } else {
        int npaths = 1;
        for (int l = 0; l < cb.levels; ++l) npaths *= 7;
        for (int part = 0; part < cb.nparts; ++part) {
            const double* pb = base + (int64_t)part * cb.part_stride;
            for (int path = 0; path < npaths; ++path) {
                int rem = path, qc = qcode, coef = 1;
                for (int l = 0; l < cb.levels; ++l) {  // last level first
                    coef *= c_dcoef[cb.variant][rem % 7][qc & 3];
                    rem /= 7;
                    qc >>= 2;
                }
                if (coef) sum += coef > 0 ? pb[path * slot_elems] : -pb[path * slot_elems];
            }
        }
    }
    store_out(C + packed_index((int64_t)cb.r0 + i, cb.q0) + j, cb.beta, sum);
}

template <typename T>
__global__ void k_fill_zero(T* __restrict__ p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = T(0);
}

// ---------------------------------------------------------------------------
// Reduced-precision forms: conversions
// ---------------------------------------------------------------------------
// binary32 -> bfloat16, round to nearest even (bfloat16 keeps the top 16
// bits of binary32); NaN stays NaN.
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// binary32 -> OCP FP8 e4m3 (bias 7, 3 mantissa bits, no infinities, largest
// finite 448), round to nearest even, saturating to +-448.
__device__ __forceinline__ uint8_t e4m3_rne(float x) {
    const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
    const float a = fabsf(x);
    if (!(a == a)) return (uint8_t)(sign | 0x7fu);
    if (a >= 448.0f) return (uint8_t)(sign | 0x7eu);
    if (a < 0.015625f) {  // below 2^-6: subnormal steps of 2^-9
        const float q = __builtin_rintf(a * 512.0f);  // exact scaling, then RNE
        return (uint8_t)(sign | (uint32_t)q);          // q == 8 encodes 2^-6 (exponent field 1)
    }
    int e = (int)((__float_as_uint(a) >> 23) & 0xffu) - 127;  // a = 1.f * 2^e, e in [-6, 8]
    const float mant = a * __builtin_ldexpf(1.0f, -e);         // [1, 2), exact
    float q = __builtin_rintf((mant - 1.0f) * 8.0f);           // exact scaling, then RNE
    if (q >= 8.0f) {
        q = 0.0f;
        ++e;
    }
    if (e > 8 || (e == 8 && q >= 7.0f)) return (uint8_t)(sign | 0x7eu);
    return (uint8_t)(sign | ((uint32_t)(e + 7) << 3) | (uint32_t)q);
}

__global__ void k_convert(int mode, const float* __restrict__ x, int64_t count, void* __restrict__ o0,
                          void* __restrict__ o1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float v = x[i];
    if (mode == 0) {
        const uint16_t h = bf16_rne(v);
        const float hf = __uint_as_float((uint32_t)h << 16);
        ((uint16_t*)o0)[i] = h;
        ((uint16_t*)o1)[i] = bf16_rne(v - hf);
    } else {
        ((uint8_t*)o0)[i] = e4m3_rne(v);
    }
}

// Column maxima of |A| in 256-row chunks, then power-of-two scales
// s_j = 2^floor(log2(448 / max_j)) (1 for a zero column).
// Column maxima of |A| over row chunks of 256: four columns per thread
// (16-byte loads when the row stride and base allow them).
__global__ void __launch_bounds__(256) k_colmax_part(const float* __restrict__ A, int64_t lda, int m, int n,
                                                     float* __restrict__ part) {
    const int j = (blockIdx.x * 256 + threadIdx.x) * 4;
    const int chunk = blockIdx.y;
    if (j >= n) return;
    const int r0 = chunk * 256, r1 = min(m, r0 + 256);
    float mx[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const bool vec = j + 4 <= n && (lda & 3) == 0 && (((uintptr_t)A) & 15u) == 0;
    if (vec) {
#pragma unroll 8
        for (int r = r0; r < r1; ++r) {
            const float4 v = *(const float4*)(A + (int64_t)r * lda + j);
            mx[0] = fmaxf(mx[0], fabsf(v.x));
            mx[1] = fmaxf(mx[1], fabsf(v.y));
            mx[2] = fmaxf(mx[2], fabsf(v.z));
            mx[3] = fmaxf(mx[3], fabsf(v.w));
        }
    } else {
        for (int r = r0; r < r1; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (j + q < n) mx[q] = fmaxf(mx[q], fabsf(A[(int64_t)r * lda + j + q]));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (j + q < n) part[(int64_t)chunk * n + j + q] = mx[q];
}
// Power-of-two e4m3 scale of a column whose largest magnitude is mx:
// 2^floor(log2(448 / mx)), 1 for a zero column.
__device__ __forceinline__ float e4m3_pow2_scale(float mx) {
    float s = 1.0f;
    if (mx > 0.0f) {
        // largest power of two s with s * mx <= 448: 448 / mx = f 2^e, f in [0.5, 1)
        int e;
        (void)frexpf(448.0f / mx, &e);
        s = __builtin_ldexpf(1.0f, e - 1);
        if (s * mx > 448.0f) s *= 0.5f;  // guard against the rounding of 448 / mx
    }
    return s;
}

__global__ void __launch_bounds__(256) k_colscale(const float* __restrict__ part, int nchunks, int n,
                                                  float* __restrict__ scale) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    float mx = 0.0f;
    for (int c = 0; c < nchunks; ++c) mx = fmaxf(mx, part[(int64_t)c * n + j]);
    scale[j] = e4m3_pow2_scale(mx);
}

// ---------------------------------------------------------------------------
// Column equilibration: A' = A diag(s) with s_j a power of two putting the
// largest |A_kj| of column j in [1, 2) (s_j = 1 for a zero column), and
// C = diag(s)^-1 C' diag(s)^-1 afterwards.  Multiplying by powers of two is
// exact barring underflow, so the product of A' differs from that of A only
// in rounding; fast (Strassen) products then bound every entry's error by
// the sizes of its own two columns instead of the largest columns of A.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_colmax_t(const T* __restrict__ A, int64_t lda, int m, int n,
                                                  T* __restrict__ part) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int chunk = blockIdx.y;
    if (j >= n) return;
    const int r0 = chunk * 256, r1 = min(m, r0 + 256);
    T mx = T(0);
    for (int r = r0; r < r1; ++r) mx = fmax(mx, fabs(A[(int64_t)r * lda + j]));
    part[(int64_t)chunk * n + j] = mx;
}

template <typename T>
__global__ void __launch_bounds__(256) k_eqscale(const T* __restrict__ part, int nchunks, int n,
                                                 T* __restrict__ scale) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    T mx = T(0);
    for (int c = 0; c < nchunks; ++c) mx = fmax(mx, part[(int64_t)c * n + j]);
    T s = T(1);
    if (mx > T(0) && isfinite(mx)) {
        int e;  // mx = f 2^e with f in [0.5, 1): mx 2^(1 - e) in [1, 2)
        (void)frexp(mx, &e);
        s = ldexp(T(1), 1 - e);
    }
    scale[j] = s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_scale_cols(const T* __restrict__ A, int64_t lda, int m, int n,
                                                    const T* __restrict__ scale, T* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)m * n) return;
    const int64_t r = e / n;
    const int j = (int)(e - r * n);
    out[e] = A[r * lda + j] * scale[j];
}

// C_ij / (s_i s_j) over packed lower C: one workgroup per row.
template <typename OUT, typename S>
__global__ void __launch_bounds__(256) k_descale(OUT* __restrict__ C, const S* __restrict__ scale) {
    const int i = blockIdx.x;
    const double si = 1.0 / (double)scale[i];
    OUT* row = C + packed_index(i, 0);
    for (int j = threadIdx.x; j <= i; j += 256) row[j] = (OUT)((double)row[j] * si / (double)scale[j]);
}

// Transposed, converted copy of A: out[i * ldt + k] for column i of A and
// row k (k >= m zero).  64 x 64 tiles through LDS.
template <int MODE>
__global__ void __launch_bounds__(256) k_prep_lp(const float* __restrict__ A, int64_t lda, int m, int n, int ldt,
                                                 const float* __restrict__ scale, void* __restrict__ o0,
                                                 void* __restrict__ o1) {
    // KB k values (rows of A) x 64 columns per workgroup; each lane of the
    // writing pass packs PK consecutive k of one output row into one store.
    constexpr int PK = 2;
    constexpr int KB = 64 * PK;
    __shared__ float tile[KB][65];
    const int k0 = blockIdx.x * KB, c0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    // reading pass: four consecutive columns per lane (16 rows per round),
    // every load of the lane in flight before the tile is written
    {
        const int cq = (threadIdx.x & 15) * 4, rr = threadIdx.x >> 4;
        const int c = c0 + cq;
        const bool vec = c + 4 <= n && (lda & 3) == 0 && (((uintptr_t)A) & 15u) == 0;
        float4 v[KB / 16];
#pragma unroll
        for (int u = 0; u < KB / 16; ++u) {
            const int k = k0 + rr + 16 * u;
            v[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (k < m) {
                const float* src = A + (int64_t)k * lda + c;
                if (vec) {
                    v[u] = *(const float4*)src;
                } else {
                    if (c < n) v[u].x = src[0];
                    if (c + 1 < n) v[u].y = src[1];
                    if (c + 2 < n) v[u].z = src[2];
                    if (c + 3 < n) v[u].w = src[3];
                }
            }
        }
        float4 sc = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
        if (MODE == 1) {  // exact: power-of-two scales
            if (c < n) sc.x = scale[c];
            if (c + 1 < n) sc.y = scale[c + 1];
            if (c + 2 < n) sc.z = scale[c + 2];
            if (c + 3 < n) sc.w = scale[c + 3];
        }
#pragma unroll
        for (int u = 0; u < KB / 16; ++u) {
            const int r = rr + 16 * u;
            tile[r][cq] = v[u].x * sc.x;
            tile[r][cq + 1] = v[u].y * sc.y;
            tile[r][cq + 2] = v[u].z * sc.z;
            tile[r][cq + 3] = v[u].w * sc.w;
        }
    }
    __syncthreads();
    const int kk = k0 + tx * PK;
    if (kk >= ldt) return;
    for (int i = 0; i < 16; ++i) {
        const int cl = ty + 4 * i, c = c0 + cl;
        if (c >= n) break;
        const int64_t o = (int64_t)c * ldt + kk;
        if (MODE == 0) {
            uint32_t hw = 0, lw = 0;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const float v = tile[tx * 2 + q][cl];
                const uint16_t h = bf16_rne(v);
                const float hf = __uint_as_float((uint32_t)h << 16);
                hw |= (uint32_t)h << (16 * q);
                lw |= (uint32_t)bf16_rne(v - hf) << (16 * q);
            }
            *(uint32_t*)((uint16_t*)o0 + o) = hw;
            *(uint32_t*)((uint16_t*)o1 + o) = lw;
        } else {
            const uint32_t wd = (uint32_t)e4m3_rne(tile[tx * 2][cl]) | ((uint32_t)e4m3_rne(tile[tx * 2 + 1][cl]) << 8);
            *(uint16_t*)((uint8_t*)o0 + o) = (uint16_t)wd;
        }
    }
}

// ---------------------------------------------------------------------------
// Strassen operands of the reduced-precision forms (operand-sum form): the
// signed sums of quadrant terms are formed in FP32 from A (term order, as the
// FP32 form stages them) and converted into rows of the operand copy.  One
// workgroup per 64 x 64 tile (k rows x operand columns) of a record; the M + N
// operand columns of a record become rows out_off + column, k contiguous.
//   MAXPASS: column maxima of |sum| into colmax (float bits: non-negative
//            floats order as their bit patterns), for the e4m3 scales
//   MODE 0:  bfloat16 hi = bf16(sum), lo = bf16(sum - hi)
//   MODE 1:  e4m3(sum s) with the column's power-of-two scale s from colmax,
//            which is also stored for the de-scaling epilogue
// k rows past the record's K are written as zeros up to the tile's end.
// ---------------------------------------------------------------------------
template <int MODE, bool MAXPASS>
__global__ void __launch_bounds__(256) k_opsum_lp(const float* __restrict__ A, int64_t lda,
                                                  const DevTask* __restrict__ tasks,
                                                  const DevTerm* __restrict__ terms,
                                                  const int32_t* __restrict__ segs,
                                                  const DevOpSum* __restrict__ recs, int nrec,
                                                  uint32_t* __restrict__ colmax, float* __restrict__ scale,
                                                  void* __restrict__ o0, void* __restrict__ o1, int ldt) {
    __shared__ float tile[64][65];
    __shared__ int rsel;
    const int64_t gt = blockIdx.x;
    if (threadIdx.x == 0) {
        int lo = 0, hi = nrec - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (recs[mid].row_off <= gt) lo = mid;
            else hi = mid - 1;
        }
        rsel = lo;
    }
    __syncthreads();
    const DevOpSum rec = recs[rsel];
    const DevTask t = tasks[rec.task];
    const int width = rec.M + rec.N;
    const int tiles_c = (width + 63) / 64;
    const int64_t loc = gt - rec.row_off;
    const int k0 = (int)(loc / tiles_c) * 64, c0 = (int)(loc % tiles_c) * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int stride = kSegHdr + 2 * (t.nx + t.ny);
    const int c = c0 + tx;
    const bool left = c < rec.M;
    const int nt = left ? t.nx : t.ny, u0 = left ? 0 : t.nx;
    const int cc = left ? c : c - rec.M;  // column inside the operand
    for (int r = ty; r < 64; r += 4) {
        const int k = k0 + r;
        float v = 0.0f;
        if (k < rec.K && c < width) {
            // chunk (segment) of operand row k and the row inside its window
            int kk = k, sgi = 0;
            for (; sgi + 1 < t.nseg; ++sgi) {
                const int len = segs[t.seg_off + sgi * stride + 2] - segs[t.seg_off + sgi * stride + 1];
                if (kk < len) break;
                kk -= len;
            }
            const int32_t* sg = segs + t.seg_off + sgi * stride;
            const int krow = sg[1] + kk;
            for (int u = 0; u < nt; ++u) {
                const DevTerm tm = terms[t.term_off + u0 + u];
                const int row = sg[kSegHdr + 2 * (u0 + u)] + krow;
                const bool ok = row < sg[kSegHdr + 2 * (u0 + u) + 1] && tm.col + cc < tm.cvend;
                const float a = ok ? A[(int64_t)row * lda + tm.col + cc] : 0.0f;
                const float sa = tm.sign < 0 ? -a : a;  // exact
                v = u == 0 ? sa : v + sa;
            }
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    if (MAXPASS) {
        if (threadIdx.x < 64 && c0 + (int)threadIdx.x < width) {
            float mx = 0.0f;
            for (int r = 0; r < 64; ++r) mx = fmaxf(mx, fabsf(tile[r][threadIdx.x]));
            if (mx > 0.0f) atomicMax(&colmax[rec.out_off + c0 + threadIdx.x], __float_as_uint(mx));
        }
        return;
    }
    for (int r = ty; r < 64; r += 4) {
        const int col = c0 + r, k = k0 + tx;
        if (col >= width || k >= ldt) continue;
        const float v = tile[tx][r];
        const int64_t orow = rec.out_off + col;
        const int64_t o = orow * ldt + k;
        if (MODE == 0) {
            const uint16_t h = bf16_rne(v);
            const float hf = __uint_as_float((uint32_t)h << 16);
            ((uint16_t*)o0)[o] = h;
            ((uint16_t*)o1)[o] = bf16_rne(v - hf);
        } else {
            const float sc = e4m3_pow2_scale(__uint_as_float(colmax[orow]));
            ((uint8_t*)o0)[o] = e4m3_rne(v * sc);  // exact scaling by a power of two
            if (k == 0) scale[orow] = sc;
        }
    }
}

// ---------------------------------------------------------------------------
// Reduced-precision classical tiles (TK_SYRK / TK_GEMM) on the transposed
// copy: 128 x 128 output tile, four waves of 64 x 64 (4 x 4 blocks of
// 16 x 16), FP32 MFMA accumulation.
//   MODE 0: bfloat16 split, hi^t hi + hi^t lo + lo^t hi per block; 128 k per
//           stage; the FP32 accumulators are added into FP64 every KFLUSH
//           rows (the split's accuracy is near FP32's)
//   MODE 1: e4m3, 256 k per stage; FP32 accumulation over the whole K (the
//           e4m3 rounding, about 1e-2, dwarfs it), which leaves room for two
//           workgroups per CU; result de-scaled by 1 / (s_i s_j)
// Rows of the copy are columns of A; the k range of a segment is its row range.
// ---------------------------------------------------------------------------
// Stage lengths: bfloat16 runs one workgroup per CU (its FP64 flush
// accumulators need more than half the registers), so a stage carries a
// long k range: more MFMA work per barrier and per load round trip (KFLUSH
// must be a multiple of KT); e4m3 runs two per CU with half the LDS each.
template <int MODE>
struct LpCfg;
template <>
struct LpCfg<0> {
    static constexpr int KT = 128;             // k per LDS stage (elements)
    static constexpr int EB = 2;               // bytes per element
    static constexpr int PLANES = 2;           // hi, lo
    static constexpr int ROWB = KT * EB + 16;  // LDS row stride in bytes (padded)
};
template <>
struct LpCfg<1> {
    static constexpr int KT = 256;
    static constexpr int EB = 1;
    static constexpr int PLANES = 1;
    static constexpr int ROWB = KT * EB + 16;
};

static_assert(KFLUSH % LpCfg<0>::KT == 0 && KFLUSH % LpCfg<1>::KT == 0, "flush on stage boundaries");

template <int MODE, typename OUT, bool SPLIT = false>
__global__ void __launch_bounds__(256, MODE == 1 ? 2 : 1) k_gemm_lp(const uint8_t* __restrict__ T0, const uint8_t* __restrict__ T1,
                                                    int ldt, const float* __restrict__ scale,
                                                    const DevTask* __restrict__ tasks,
                                                    const DevTerm* __restrict__ terms,
                                                    const int32_t* __restrict__ segs,
                                                    const WorkItem* __restrict__ items, OUT* __restrict__ C,
                                                    double* __restrict__ W, int nparts, double* __restrict__ part) {
    typedef LpCfg<MODE> L;
    constexpr int KT = L::KT, EB = L::EB, PL = L::PLANES, ROWB = L::ROWB;
    constexpr int ROWBYTES = KT * EB;           // bytes of one tile row per stage
    constexpr int CHUNKS = GT * ROWBYTES / 16;  // 16-byte chunks per plane and operand
    constexpr int CPT = CHUNKS / 256;           // chunks per thread per plane and operand
    __shared__ __attribute__((aligned(16))) uint8_t Xs[PL][GT * ROWB];
    __shared__ __attribute__((aligned(16))) uint8_t Ys[PL][GT * ROWB];

    const WorkItem w = items[blockIdx.x];
    const DevTask t = tasks[w.task];
    const DevTerm tx = terms[t.term_off];
    const DevTerm ty = terms[t.term_off + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int i0 = w.ti * GT, j0 = w.tj * GT;
    const int stride = kSegHdr + 2 * (t.nx + t.ny);

    constexpr bool FL = MODE == 0;  // FP64 flush accumulators
    f4_t acc[4][4];
    double acc64[FL ? 4 : 1][FL ? 4 : 1][FL ? 4 : 1];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};
            if (FL)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc64[FL ? a : 0][FL ? b : 0][FL ? e : 0] = 0.0;
        }

    int ntiles = 0;
    for (int s = 0; s < t.nseg; ++s)
        ntiles += (segs[t.seg_off + s * stride + 2] - segs[t.seg_off + s * stride + 1] + KT - 1) / KT;

    // staged chunks: [plane][operand][chunk]
    u4_t rg[PL][2][CPT];
    int seg = 0;
    int k0 = t.nseg > 0 ? segs[t.seg_off + 1] : 0;
    int klen = t.nseg > 0 ? segs[t.seg_off + 2] : 0;  // window end
    int krow = t.nseg > 0 ? segs[t.seg_off + kSegHdr] : 0;

    auto load = [&]() {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int ch = tid + 256 * c;
            const int r = ch / (ROWBYTES / 16);               // tile row
            const int kb = (ch % (ROWBYTES / 16)) * 16 / EB;  // first k of the chunk
            const int kk = k0 + kb;                            // k offset inside the segment
#pragma unroll
            for (int op = 0; op < 2; ++op) {
                const int tcol = op == 0 ? tx.col : ty.col;
                const int tend = op == 0 ? tx.cvend : ty.cvend;
                const int row = tcol + (op == 0 ? i0 : j0) + r;  // column of A = row of the copy
                const bool rv = row < tend;
                const int64_t base = (int64_t)row * ldt + krow + kk;
                const int nval = klen - kk;  // valid elements from kk
#pragma unroll
                for (int p = 0; p < PL; ++p) {
                    u4_t v = u4_t{0u, 0u, 0u, 0u};
                    if (rv && nval > 0) {
                        const uint8_t* src = (p == 0 ? T0 : T1) + base * EB;
                        if (nval >= 16 / EB && (((uintptr_t)src) & 15u) == 0) {
                            v = *(const u4_t*)src;
                        } else {
                            unsigned wd[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                            for (int q = 0; q < 16; ++q)
                                if (q / EB < nval) wd[q >> 2] |= (unsigned)src[q] << (8 * (q & 3));
                            v = u4_t{wd[0], wd[1], wd[2], wd[3]};
                        }
                    }
                    rg[p][op][c] = v;
                }
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int ch = tid + 256 * c;
            const int r = ch / (ROWBYTES / 16);
            const int off = r * ROWB + (ch % (ROWBYTES / 16)) * 16;
#pragma unroll
            for (int p = 0; p < PL; ++p) {
                *(u4_t*)(&Xs[p][off]) = rg[p][0][c];
                *(u4_t*)(&Ys[p][off]) = rg[p][1][c];
            }
        }
    };
    auto advance = [&]() {
        k0 += KT;
        if (k0 >= klen) {
            ++seg;
            if (seg < t.nseg) {
                k0 = segs[t.seg_off + seg * stride + 1];
                klen = segs[t.seg_off + seg * stride + 2];
                krow = segs[t.seg_off + seg * stride + kSegHdr];
            }
        }
    };

    if constexpr (SPLIT) {  // part (slot mod nparts) of a K-split tile: its share of the stages
        const int tp = w.slot % nparts;
        const int s0 = (int)((int64_t)ntiles * tp / nparts), s1 = (int)((int64_t)ntiles * (tp + 1) / nparts);
        for (int u = 0; u < s0; ++u) advance();
        ntiles = s1 - s0;
    }
    if (ntiles > 0) load();
    for (int it = 0; it < ntiles; ++it) {
        __syncthreads();  // previous stage fully read
        store();
        __syncthreads();
        if (it + 1 < ntiles) {
            advance();
            load();
        }
        const int rsel = lane & 15, kq = lane >> 4;
        if (MODE == 0) {
#pragma unroll
            for (int ks = 0; ks < KT / 32; ++ks) {
                const int kb = (ks * 32 + kq * 8) * EB;
                bf8_t bh[4], bl[4];
#pragma unroll
                for (int cf = 0; cf < 4; ++cf) {
                    const int rr = wn * 64 + cf * 16 + rsel;
                    bh[cf] = *(const bf8_t*)(&Ys[0][rr * ROWB + kb]);
                    bl[cf] = *(const bf8_t*)(&Ys[PL - 1][rr * ROWB + kb]);
                }
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const int rr = wm * 64 + rb * 16 + rsel;
                    const bf8_t ah = *(const bf8_t*)(&Xs[0][rr * ROWB + kb]);
                    const bf8_t al = *(const bf8_t*)(&Xs[PL - 1][rr * ROWB + kb]);
#pragma unroll
                    for (int cf = 0; cf < 4; ++cf) {
                        acc[rb][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[cf], acc[rb][cf], 0, 0, 0);
                        acc[rb][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[cf], acc[rb][cf], 0, 0, 0);
                        acc[rb][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[cf], acc[rb][cf], 0, 0, 0);
                    }
                }
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < KT / 128; ++ks) {
                const int kb = ks * 128 + kq * 32;
                i8_t bq[4];
#pragma unroll
                for (int cf = 0; cf < 4; ++cf) {
                    const int rr = wn * 64 + cf * 16 + rsel;
                    bq[cf] = *(const i8_t*)(&Ys[0][rr * ROWB + kb]);
                }
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const int rr = wm * 64 + rb * 16 + rsel;
                    const i8_t aq = *(const i8_t*)(&Xs[0][rr * ROWB + kb]);
#pragma unroll
                    for (int cf = 0; cf < 4; ++cf)
                        acc[rb][cf] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(aq, bq[cf], acc[rb][cf], 0, 0,
                                                                                      0, 0, 0, 0);
                }
            }
        }
        if (FL && (((it + 1) * KT) % KFLUSH == 0 || it + 1 == ntiles)) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc64[FL ? a : 0][FL ? b : 0][FL ? e : 0] += (double)acc[a][b][e];
                    acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};
                }
        }
    }

    if constexpr (SPLIT) {  // de-scaled FP64 partial tile (exact power-of-two scales)
        double* pt = part + (int64_t)w.slot * GT * GT;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int li = wm * 64 + rb * 16 + 4 * (lane >> 4) + e, gi = i0 + li;
                const double si = MODE == 1 && gi < t.dM ? 1.0 / (double)scale[tx.col + gi] : 1.0;
#pragma unroll
                for (int cf = 0; cf < 4; ++cf) {
                    const int lj = wn * 64 + cf * 16 + (lane & 15), gj = j0 + lj;
                    double v = FL ? acc64[FL ? rb : 0][FL ? cf : 0][FL ? e : 0] : (double)acc[rb][cf][e];
                    if (MODE == 1) v = gi < t.dM && gj < t.dN ? v * si / (double)scale[ty.col + gj] : 0.0;
                    pt[li * GT + lj] = v;
                }
            }
        return;
    }
    const bool syrk = t.kind == TK_SYRK;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int gi = i0 + wm * 64 + rb * 16 + 4 * (lane >> 4) + e;
            if (gi >= t.dM) continue;
            const int64_t rowbase = packed_index((int64_t)t.r0 + gi, t.q0);
            const double si = MODE == 1 ? 1.0 / (double)scale[tx.col + gi] : 1.0;
#pragma unroll
            for (int cf = 0; cf < 4; ++cf) {
                const int gj = j0 + wn * 64 + cf * 16 + (lane & 15);
                if (gj >= t.dN || (syrk && gj > gi)) continue;
                double v = FL ? acc64[FL ? rb : 0][FL ? cf : 0][FL ? e : 0] : (double)acc[rb][cf][e];
                if (MODE == 1) v = v * si / (double)scale[ty.col + gj];  // exact power-of-two de-scale
                if (t.dst == 0)
                    store_out(C + rowbase + gj, t.beta, v);
                else
                    W[t.ws_off + (int64_t)gi * t.N + gj] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Reduced-precision tiles with direct-to-LDS staging: the tasks of k_gemm_lp
// (classical tiles on the transposed converted copy), with every stage's rows
// of the copy moved from global memory straight into LDS by buffer loads that
// write LDS, one dword per lane, two 128-byte tile rows per copy.  The copies
// of stage s + 1 are issued while stage s is multiplied (double-buffered
// LDS), so the loop waits on global memory only at the stage barrier.  Wave w
// copies operand w / 2, tile rows [64 (w % 2), 64 (w % 2) + 64).  The copies
// need every segment window of the plan to start and end on a dword of the
// copy (checked on the host; otherwise k_gemm_lp runs).  The 16-byte chunks
// of tile row r are XOR-swizzled by (r / 2) mod 8, which puts the sixteen
// rows an MFMA operand read touches in sixteen different bank groups.
// Copies past the window end or the operand's last row get an out-of-range
// offset and write zeros.
// ---------------------------------------------------------------------------
template <int MODE>
struct LpdCfg;
template <>
struct LpdCfg<0> {  // bfloat16 hi and lo planes; FP64 flush needs the whole register file
    static constexpr int KT = 64, EB = 2, PL = 2, OCC = 1;
};
template <>
struct LpdCfg<1> {  // e4m3
    static constexpr int KT = 128, EB = 1, PL = 1, OCC = 2;
};

template <int MODE, typename OUT, bool SPLIT = false, bool B16 = false>
__global__ void __launch_bounds__(256, LpdCfg<MODE>::OCC) k_gemm_lpd(const uint8_t* __restrict__ T0,
                                                                    const uint8_t* __restrict__ T1, int ldt,
                                                                    const float* __restrict__ scale,
                                                                    const DevTask* __restrict__ tasks,
                                                                    const DevTerm* __restrict__ terms,
                                                                    const int32_t* __restrict__ segs,
                                                                    const WorkItem* __restrict__ items,
                                                                    OUT* __restrict__ C, double* __restrict__ W,
                                                                    int nparts, double* __restrict__ part) {
    typedef LpdCfg<MODE> L;
    constexpr int KT = L::KT, EB = L::EB, PL = L::PL;
    constexpr int RB = KT * EB;  // bytes of one tile row per stage
    static_assert(RB == 128, "two tile rows per 256-byte copy");
    constexpr int PLANE = GT * RB;
    constexpr int NCP = 32;  // copies per plane and wave (64 rows, two per copy)
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][PL][2][PLANE];  // [buffer][plane][operand]

    const WorkItem w = items[blockIdx.x];
    const DevTask t = tasks[w.task];
    const DevTerm tx = terms[t.term_off];
    const DevTerm ty = terms[t.term_off + 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int i0 = w.ti * GT, j0 = w.tj * GT;
    const int stride = kSegHdr + 2 * (t.nx + t.ny);
    const int64_t rowb = (int64_t)ldt * EB;  // bytes between rows of the copy

    // Copy role: operand cop, tile rows half * 64 + [0, 64).  Copy i moves
    // rows 2i (lanes 0-31) and 2i + 1 (lanes 32-63) of that range; lane
    // dword d of a row holds logical chunk (d / 4) ^ (i mod 8).  Per i mod 8:
    // the lane's byte offset inside the row block and its first k element.
    // B16: sixteen bytes per lane instead, copy i moving rows 8i to 8i + 7
    // (lane L: row 8i + L / 8, physical chunk L % 8, so logical chunk
    // (L % 8) ^ ((8i + L / 8) / 2 mod 8)); vb and ke then hold, per copy,
    // the lane's byte offset from the block's window start and first k.
    const int cop = wave >> 1, half = wave & 1;
    const int hb = lane >> 5, d = lane & 31;
    const int rl = lane >> 3;
    uint32_t vb[8];
    int ke[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if constexpr (B16) {
            const int r = 8 * q + rl;
            const int kc = (lane & 7) ^ ((r >> 1) & 7);
            vb[q] = (uint32_t)(r * rowb) + (uint32_t)(kc * 16);
            ke[q] = kc * 16 / EB;
        } else {
            const int lc = (d >> 2) ^ q;
            const int byte = lc * 16 + (d & 3) * 4;
            vb[q] = (uint32_t)(hb * rowb) + (uint32_t)byte;
            ke[q] = byte / EB;
        }
    }
    const DevTerm& tc = cop == 0 ? tx : ty;
    const int row0 = tc.col + (cop == 0 ? i0 : j0) + half * 64;  // first row of the copy this wave reads
    const int nrv = tc.cvend - row0;                              // rows of the range that exist
    const int ilim = nrv >= 64 ? NCP : (nrv - hb + 1 > 0 ? (nrv - hb + 1) / 2 : 0);  // copies with this lane's row

    constexpr bool FL = MODE == 0;  // FP64 flush accumulators
    f4_t acc[4][4];
    double acc64[FL ? 4 : 1][FL ? 4 : 1][FL ? 4 : 1];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};
            if (FL)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc64[FL ? a : 0][FL ? b : 0][FL ? e : 0] = 0.0;
        }

    int ntiles = 0;
    for (int s = 0; s < t.nseg; ++s)
        ntiles += (segs[t.seg_off + s * stride + 2] - segs[t.seg_off + s * stride + 1] + KT - 1) / KT;
    int seg = 0;
    int k0 = t.nseg > 0 ? segs[t.seg_off + 1] : 0;
    int kend = t.nseg > 0 ? segs[t.seg_off + 2] : 0;  // window end
    int krow = t.nseg > 0 ? segs[t.seg_off + kSegHdr] : 0;

    // Copies of the stage at k0 into buffer `buf` (live false: past the last
    // stage, every copy is out of range and writes zeros into the spare
    // buffer; they are waited for before the workgroup ends).
    auto copy_stage = [&](int buf, bool live) {
        const int krem = live ? kend - k0 : 0;
        const bool full = krem >= KT && nrv >= 64;  // uniform: every copy of the stage in range
#pragma unroll
        for (int p = 0; p < PL; ++p) {
            const uint8_t* base = (p == 0 ? T0 : T1) + ((int64_t)row0 * ldt + krow + k0) * EB;
            const rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(base), (short)0, 0x7fffffff,
                                                                0x00020000);
            uint8_t* dst = &lds[buf][p][cop][half * 64 * RB];
            if constexpr (B16) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const bool ok = full || (8 * i + rl < nrv && ke[i] < krem);
                    lds_copy16(rs, dst + i * 8 * RB, ok ? vb[i] : kOOB);
                }
            } else {
#pragma unroll
                for (int i = 0; i < NCP; ++i) {
                    const uint32_t off = full || (i < ilim && ke[i & 7] < krem) ? vb[i & 7] : kOOB;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rs, (__attribute__((address_space(3))) void*)(dst + 2 * i * RB), 4, off, (int)(2 * i * rowb), 0,
                        0);
                }
            }
        }
    };
    auto advance = [&]() {
        k0 += KT;
        if (k0 >= kend) {
            ++seg;
            if (seg < t.nseg) {
                k0 = segs[t.seg_off + seg * stride + 1];
                kend = segs[t.seg_off + seg * stride + 2];
                krow = segs[t.seg_off + seg * stride + kSegHdr];
            }
        }
    };
    // byte address of logical 16-byte chunk kc of tile row r inside a plane
    auto chunk = [](int r, int kc) { return r * RB + ((kc ^ ((r >> 1) & 7)) << 4); };

    if constexpr (SPLIT) {  // part (slot mod nparts) of a K-split tile: its share of the stages
        const int tp = w.slot % nparts;
        const int s0 = (int)((int64_t)ntiles * tp / nparts), s1 = (int)((int64_t)ntiles * (tp + 1) / nparts);
        for (int u = 0; u < s0; ++u) advance();
        ntiles = s1 - s0;
    }
    if (ntiles > 0) copy_stage(0, true);
    for (int it = 0; it < ntiles; ++it) {
        const int buf = it & 1;
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of stage it have landed
        __syncthreads();                // every copy of stage it landed; stage it-1 fully read
        const bool next = it + 1 < ntiles;
        if (next) advance();
        copy_stage(buf ^ 1, next);
        const int rsel = lane & 15, kq = lane >> 4;
        if (MODE == 0) {
#pragma unroll
            for (int ks = 0; ks < KT / 32; ++ks) {
                const int kc = ks * 4 + kq;
                bf8_t bh[4], bl[4];
#pragma unroll
                for (int cf = 0; cf < 4; ++cf) {
                    const int rr = wn * 64 + cf * 16 + rsel;
                    bh[cf] = *(const bf8_t*)(&lds[buf][0][1][chunk(rr, kc)]);
                    bl[cf] = *(const bf8_t*)(&lds[buf][PL - 1][1][chunk(rr, kc)]);
                }
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const int rr = wm * 64 + rb * 16 + rsel;
                    const bf8_t ah = *(const bf8_t*)(&lds[buf][0][0][chunk(rr, kc)]);
                    const bf8_t al = *(const bf8_t*)(&lds[buf][PL - 1][0][chunk(rr, kc)]);
#pragma unroll
                    for (int cf = 0; cf < 4; ++cf) {
                        acc[rb][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[cf], acc[rb][cf], 0, 0, 0);
                        acc[rb][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[cf], acc[rb][cf], 0, 0, 0);
                        acc[rb][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[cf], acc[rb][cf], 0, 0, 0);
                    }
                }
            }
        } else {
            const int kc = 2 * kq;  // 32 bytes: logical chunks kc, kc + 1
            i8_t bq[4];
#pragma unroll
            for (int cf = 0; cf < 4; ++cf) {
                const int rr = wn * 64 + cf * 16 + rsel;
                const u4_t lo = *(const u4_t*)(&lds[buf][0][1][chunk(rr, kc)]);
                const u4_t hi = *(const u4_t*)(&lds[buf][0][1][chunk(rr, kc + 1)]);
                bq[cf] = i8_t{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
            }
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int rr = wm * 64 + rb * 16 + rsel;
                const u4_t lo = *(const u4_t*)(&lds[buf][0][0][chunk(rr, kc)]);
                const u4_t hi = *(const u4_t*)(&lds[buf][0][0][chunk(rr, kc + 1)]);
                const i8_t aq = i8_t{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
#pragma unroll
                for (int cf = 0; cf < 4; ++cf)
                    acc[rb][cf] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(aq, bq[cf], acc[rb][cf], 0, 0, 0, 0,
                                                                                  0, 0);
            }
        }
        if (FL && (((it + 1) * KT) % KFLUSH == 0 || it + 1 == ntiles)) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc64[FL ? a : 0][FL ? b : 0][FL ? e : 0] += (double)acc[a][b][e];
                    acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};
                }
        }
    }

    // no copy may land after the workgroup's LDS is released
    __builtin_amdgcn_s_waitcnt(0);

    if constexpr (SPLIT) {  // de-scaled FP64 partial tile (exact power-of-two scales)
        double* pt = part + (int64_t)w.slot * GT * GT;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int li = wm * 64 + rb * 16 + 4 * (lane >> 4) + e, gi = i0 + li;
                const double si = MODE == 1 && gi < t.dM ? 1.0 / (double)scale[tx.col + gi] : 1.0;
#pragma unroll
                for (int cf = 0; cf < 4; ++cf) {
                    const int lj = wn * 64 + cf * 16 + (lane & 15), gj = j0 + lj;
                    double v = FL ? acc64[FL ? rb : 0][FL ? cf : 0][FL ? e : 0] : (double)acc[rb][cf][e];
                    if (MODE == 1) v = gi < t.dM && gj < t.dN ? v * si / (double)scale[ty.col + gj] : 0.0;
                    pt[li * GT + lj] = v;
                }
            }
        return;
    }
    const bool syrk = t.kind == TK_SYRK;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int gi = i0 + wm * 64 + rb * 16 + 4 * (lane >> 4) + e;
            if (gi >= t.dM) continue;
            const int64_t rowbase = packed_index((int64_t)t.r0 + gi, t.q0);
            const double si = MODE == 1 ? 1.0 / (double)scale[tx.col + gi] : 1.0;
#pragma unroll
            for (int cf = 0; cf < 4; ++cf) {
                const int gj = j0 + wn * 64 + cf * 16 + (lane & 15);
                if (gj >= t.dN || (syrk && gj > gi)) continue;
                double v = FL ? acc64[FL ? rb : 0][FL ? cf : 0][FL ? e : 0] : (double)acc[rb][cf][e];
                if (MODE == 1) v = v * si / (double)scale[ty.col + gj];  // exact power-of-two de-scale
                if (t.dst == 0)
                    store_out(C + rowbase + gj, t.beta, v);
                else
                    W[t.ws_off + (int64_t)gi * t.N + gj] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// e4m3 tiles of 256 x 256 (k_lp8_big): the tasks of k_gemm_lpd<1> on
// workgroup tiles four times larger, for launches with enough of them.  One
// stage of a 128 x 128 e4m3 tile is 512 MFMA cycles per wave, too short to
// cover the latency of the next stage's copies from L2 and the MALL; here a
// stage is 2048 MFMA cycles per SIMD (two waves of 32 MFMAs each) and every
// byte staged feeds twice the multiply-adds.  512 threads: eight waves of
// 128 x 64 (rows wm = wave / 4, columns wn = wave % 4), 128 k per stage,
// double-buffered LDS of 2 x 64 KB, one workgroup per CU.
//
// Copies: one 16-byte buffer load per lane that writes LDS moves eight
// 128-byte tile rows; wave w copies rows [64 (w % 4), 64 (w % 4) + 64) of
// operand w / 4.  Physical chunk p of row r holds logical chunk
// p ^ ((r / 2) mod 8) (the swizzle of k_gemm_lpd), so lane L of a copy
// fetches logical chunk (L % 8) ^ ((r / 2) mod 8) of row r = 8 i + L / 8.
// Needs every segment window of the plan on 16 elements of the copy
// (checked on the host); chunks past the window end or the operand's last
// row get an out-of-range offset and write zeros.
// ---------------------------------------------------------------------------
constexpr int BT = kBigTile;  // workgroup tile

__global__ void __launch_bounds__(512, 1) k_lp8_big(const uint8_t* __restrict__ T0, int ldt,
                                                    const float* __restrict__ scale,
                                                    const DevTask* __restrict__ tasks,
                                                    const DevTerm* __restrict__ terms,
                                                    const int32_t* __restrict__ segs,
                                                    const WorkItem* __restrict__ items, double* __restrict__ C,
                                                    double* __restrict__ W, int nparts, float* __restrict__ part) {
    constexpr int KT = 128;          // k per stage (bytes of a tile row)
    constexpr int PLANE = BT * KT;   // 32 KB
    constexpr int NCP = 8;           // copies per wave and stage (8 rows each)
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][2][PLANE];  // [buffer][operand]

    const WorkItem w = items[blockIdx.x];
    const DevTask t = tasks[w.task];
    const DevTerm tx = terms[t.term_off];
    const DevTerm ty = terms[t.term_off + 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 2, wn = wave & 3;
    const int i0 = w.ti * BT, j0 = w.tj * BT;
    const int stride = kSegHdr + 2 * (t.nx + t.ny);
    const bool syrk = t.kind == TK_SYRK;
    // waves of a diagonal tile whose 128 x 64 part lies above the diagonal
    // only copy (the other wave on their SIMD gets the MFMA unit)
    const bool idle = syrk && w.ti == w.tj && wn * 64 >= wm * 128 + 128;

    // copy role
    const int cop = wave >> 2, quarter = wave & 3;
    const DevTerm& tc = cop == 0 ? tx : ty;
    const int row0 = tc.col + (cop == 0 ? i0 : j0) + quarter * 64;  // first copy row of this wave
    const int nrv = tc.cvend - row0;                                // rows of the 64 that exist
    const int rl = lane >> 3, pc = lane & 7;                        // row in a copy, physical chunk
    uint32_t vrow[NCP];  // byte offset of this lane's chunk from row0's window start, per copy
    int kcl[NCP];        // first k of the lane's logical chunk
#pragma unroll
    for (int i = 0; i < NCP; ++i) {
        const int r = 8 * i + rl;  // row within the wave's 64 (and within the 256: quarter * 64 + r)
        const int kc = pc ^ (((quarter * 64 + r) >> 1) & 7);
        kcl[i] = kc * 16;
        vrow[i] = (uint32_t)(r * ldt + kc * 16);
    }

    f4_t acc[8][4];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};

    int ntiles = 0;
    for (int sgi = 0; sgi < t.nseg; ++sgi)
        ntiles += (segs[t.seg_off + sgi * stride + 2] - segs[t.seg_off + sgi * stride + 1] + KT - 1) / KT;
    int seg = 0;
    int k0 = t.nseg > 0 ? segs[t.seg_off + 1] : 0;
    int kend = t.nseg > 0 ? segs[t.seg_off + 2] : 0;
    int krow = t.nseg > 0 ? segs[t.seg_off + kSegHdr] : 0;

    auto copy_stage = [&](int buf, bool live) {
        const int krem = live ? kend - k0 : 0;
        const bool full = krem >= KT && nrv >= 64;
        const uint8_t* base = T0 + ((int64_t)row0 * ldt + krow + k0);
        const rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(base), (short)0, 0x7fffffff,
                                                            0x00020000);
        uint8_t* dst = &lds[buf][cop][quarter * 64 * KT];
#pragma unroll
        for (int i = 0; i < NCP; ++i) {
            const bool ok = full || (8 * i + rl < nrv && kcl[i] < krem);
            lds_copy16(rs, dst + i * 8 * KT, ok ? vrow[i] : kOOB);
        }
    };
    auto advance = [&]() {
        k0 += KT;
        if (k0 >= kend) {
            ++seg;
            if (seg < t.nseg) {
                k0 = segs[t.seg_off + seg * stride + 1];
                kend = segs[t.seg_off + seg * stride + 2];
                krow = segs[t.seg_off + seg * stride + kSegHdr];
            }
        }
    };
    auto chunk = [](int r, int kc) { return r * KT + ((kc ^ ((r >> 1) & 7)) << 4); };

    // K-split item (nparts > 1): slot = tile * nparts + part; the part runs
    // stages [part * ntiles / nparts, (part + 1) * ntiles / nparts)
    const int tq = nparts > 1 ? w.slot / nparts : 0, tp = nparts > 1 ? w.slot % nparts : 0;
    if (nparts > 1) {
        const int s0 = (int)((int64_t)ntiles * tp / nparts), s1 = (int)((int64_t)ntiles * (tp + 1) / nparts);
        for (int u = 0; u < s0; ++u) advance();
        ntiles = s1 - s0;
    }
    if (ntiles > 0) copy_stage(0, true);
    for (int it = 0; it < ntiles; ++it) {
        const int buf = it & 1;
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of stage it have landed
        __syncthreads();                // every copy of stage it landed; stage it-1 fully read
        const bool next = it + 1 < ntiles;
        if (next) advance();
        copy_stage(buf ^ 1, next);
        if (!idle) {
            const int rsel = lane & 15, kc = 2 * (lane >> 4);  // 32 bytes: logical chunks kc, kc + 1
            i8_t bq[4];
#pragma unroll
            for (int cf = 0; cf < 4; ++cf) {
                const int rr = wn * 64 + cf * 16 + rsel;
                const u4_t lo = *(const u4_t*)(&lds[buf][1][chunk(rr, kc)]);
                const u4_t hi = *(const u4_t*)(&lds[buf][1][chunk(rr, kc + 1)]);
                bq[cf] = i8_t{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
            }
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int rb = 0; rb < 8; ++rb) {
                const int rr = wm * 128 + rb * 16 + rsel;
                const u4_t lo = *(const u4_t*)(&lds[buf][0][chunk(rr, kc)]);
                const u4_t hi = *(const u4_t*)(&lds[buf][0][chunk(rr, kc + 1)]);
                const i8_t aq = i8_t{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
#pragma unroll
                for (int cf = 0; cf < 4; ++cf)
                    acc[rb][cf] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(aq, bq[cf], acc[rb][cf], 0, 0, 0, 0,
                                                                                  0, 0);
            }
            __builtin_amdgcn_s_setprio(0);
        }
    }

    // no copy may land after the workgroup's LDS is released
    __builtin_amdgcn_s_waitcnt(0);

    if (idle) return;
    if (nparts > 1) {  // raw FP32 partial tile
        float* pt = part + (int64_t)(tq * nparts + tp) * BT * BT;
#pragma unroll
        for (int rb = 0; rb < 8; ++rb)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int cf = 0; cf < 4; ++cf)
                    pt[(wm * 128 + rb * 16 + 4 * (lane >> 4) + e) * BT + wn * 64 + cf * 16 + (lane & 15)] = acc[rb][cf][e];
        return;
    }
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int gi = i0 + wm * 128 + rb * 16 + 4 * (lane >> 4) + e;
            if (gi >= t.dM) continue;
            const int64_t rowbase = packed_index((int64_t)t.r0 + gi, t.q0);
            const double si = 1.0 / (double)scale[tx.col + gi];
#pragma unroll
            for (int cf = 0; cf < 4; ++cf) {
                const int gj = j0 + wn * 64 + cf * 16 + (lane & 15);
                if (gj >= t.dN || (syrk && gj > gi)) continue;
                const double v = (double)acc[rb][cf][e] * si / (double)scale[ty.col + gj];  // exact power-of-two de-scale
                if (t.dst == 0)
                    store_out(C + rowbase + gj, t.beta, v);
                else
                    W[t.ws_off + (int64_t)gi * t.N + gj] = v;
            }
        }
    }
}

// Sum of the K parts of the split last-round tiles (FP64, in part order),
// de-scaled and stored as k_lp8_big stores: block (li, q) covers row li of
// tail tile q, one thread per column.
__global__ void __launch_bounds__(256) k_lp8_tail_sum(const float* __restrict__ scale,
                                                     const DevTask* __restrict__ tasks,
                                                     const DevTerm* __restrict__ terms,
                                                     const WorkItem* __restrict__ tail, int nparts,
                                                     const float* __restrict__ part, double* __restrict__ C,
                                                     double* __restrict__ W) {
    const int q = blockIdx.y, li = blockIdx.x, lj = threadIdx.x;
    const WorkItem w = tail[q * nparts];
    const DevTask t = tasks[w.task];
    const int gi = w.ti * BT + li, gj = w.tj * BT + lj;
    if (gi >= t.dM || gj >= t.dN || (t.kind == TK_SYRK && gj > gi)) return;
    const DevTerm tx = terms[t.term_off];
    const DevTerm ty = terms[t.term_off + 1];
    double v = 0.0;
    for (int p = 0; p < nparts; ++p) v += (double)part[((int64_t)(q * nparts + p) * BT + li) * BT + lj];
    v = v * (1.0 / (double)scale[tx.col + gi]) / (double)scale[ty.col + gj];  // exact power-of-two de-scale
    if (t.dst == 0)
        store_out(C + packed_index((int64_t)t.r0 + gi, t.q0) + gj, t.beta, v);
    else
        W[t.ws_off + (int64_t)gi * t.N + gj] = v;
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_gemm(bool f32, bool out_f64, const void* A, int64_t lda, const DevTables& tb,
                       const WorkItem* items, int nitems, void* C, double* W, hipStream_t s, const void* Aops) {
    if (nitems <= 0) return hipSuccess;
    const dim3 g(nitems), b(256);
    const BatchEntry* nb = nullptr;
    if (!f32)
        hipLaunchKernelGGL((k_gemmd<double, double, false>), g, b, 0, s, (const double*)A, lda, tb.tasks, tb.segs,
                           items, (double*)C, W, tb.terms, (const double*)Aops, nb, 1, (double*)nullptr);
    else if (out_f64)
        hipLaunchKernelGGL((k_gemmd<float, double, false>), g, b, 0, s, (const float*)A, lda, tb.tasks, tb.segs,
                           items, (double*)C, W, tb.terms, (const float*)Aops, nb, 1, (double*)nullptr);
    else
        hipLaunchKernelGGL((k_gemmd<float, float, false>), g, b, 0, s, (const float*)A, lda, tb.tasks, tb.segs,
                           items, (float*)C, W, tb.terms, (const float*)Aops, nb, 1, (double*)nullptr);
    return hipGetLastError();
}

hipError_t launch_tile(int nt, const double* A, int64_t lda, const DevTables& tb, const WorkItem* items, int nitems,
                       double* C, double* W, hipStream_t s, const double* Aops, int* queue) {
    if (nitems <= 0) return hipSuccess;
    if (nt < 1 || nt > 2) return hipErrorInvalidValue;
    const dim3 b(256);
    if (nt == 2 && queue) {
        // persistent: as many workgroups as stay resident, queues cleared first
        static std::atomic<int> resident[64];
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
        int r = resident[dev].load();
        if (r == 0) {
            int per_cu = 0, cus = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tile_q<double>, 256, 0);
            if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return e;
            r = per_cu * cus > 0 ? per_cu * cus : 1;
            resident[dev].store(r);
        }
        hipLaunchKernelGGL(k_fill_zero<int>, dim3(1), dim3(64), 0, s, queue, (int64_t)kTileQueues);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_tile_q<double>, dim3(nitems < r ? nitems : r), b, 0, s, A, lda, tb.tasks, tb.terms,
                           tb.segs, items, C, W, Aops, queue, nitems);
        return hipGetLastError();
    }
    if (nt == 1)
        hipLaunchKernelGGL((k_tile<double, 1>), dim3(nitems), b, 0, s, A, lda, tb.tasks, tb.terms, tb.segs, items, C,
                           W, Aops);
    else
        hipLaunchKernelGGL((k_tile<double, 2>), dim3(nitems), b, 0, s, A, lda, tb.tasks, tb.terms, tb.segs, items, C,
                           W, Aops);
    return hipGetLastError();
}

template <int TM>
static void launch_gemm_terms_t(bool f32, bool out_f64, dim3 g, const void* A, int64_t lda, const DevTables& tb,
                                const WorkItem* items, void* C, double* W, hipStream_t s) {
    const dim3 b(256);
    if (!f32)
        hipLaunchKernelGGL((k_gemm<double, double, TM>), g, b, 0, s, (const double*)A, lda, tb.tasks, tb.terms,
                           tb.segs, items, (double*)C, W);
    else if (out_f64)
        hipLaunchKernelGGL((k_gemm<float, double, TM>), g, b, 0, s, (const float*)A, lda, tb.tasks, tb.terms,
                           tb.segs, items, (double*)C, W);
    else
        hipLaunchKernelGGL((k_gemm<float, float, TM>), g, b, 0, s, (const float*)A, lda, tb.tasks, tb.terms,
                           tb.segs, items, (float*)C, W);
}

hipError_t launch_gemm_terms(bool f32, bool out_f64, int tmax, const void* A, int64_t lda, const DevTables& tb,
                             const WorkItem* items, int nitems, void* C, double* W, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const dim3 g(nitems);
    if (tmax <= 2)
        launch_gemm_terms_t<2>(f32, out_f64, g, A, lda, tb, items, C, W, s);
    else if (tmax <= 4)
        launch_gemm_terms_t<4>(f32, out_f64, g, A, lda, tb, items, C, W, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_gemm_batch(bool f32, bool out_f64, const BatchEntry* batch, const WorkItem* items, int nitems,
                             hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const dim3 g(nitems), b(256);
    if (!f32)
        hipLaunchKernelGGL((k_gemmd<double, double, true>), g, b, 0, s, nullptr, 0, nullptr, nullptr, items, nullptr,
                           nullptr, nullptr, nullptr, batch, 1, (double*)nullptr);
    else if (out_f64)
        hipLaunchKernelGGL((k_gemmd<float, double, true>), g, b, 0, s, nullptr, 0, nullptr, nullptr, items, nullptr,
                           nullptr, nullptr, nullptr, batch, 1, (double*)nullptr);
    else
        hipLaunchKernelGGL((k_gemmd<float, float, true>), g, b, 0, s, nullptr, 0, nullptr, nullptr, items, nullptr,
                           nullptr, nullptr, nullptr, batch, 1, (double*)nullptr);
    return hipGetLastError();
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): counter = element
// group index, key = seed; two uniform 32-bit words per normal value via the
// Box-Muller transform.
__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

template <typename T>
__global__ void k_fill_normal(T* __restrict__ p, int64_t count, uint64_t seed) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // group of 2 values
    if (2 * g >= count) return;
    uint32_t c[4] = {(uint32_t)g, (uint32_t)((uint64_t)g >> 32), 0u, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    // uniforms in (0, 1]
    const double u1 = ((double)c[0] + 1.0) * (1.0 / 4294967296.0);
    const double u2 = ((double)c[1]) * (1.0 / 4294967296.0);
    const double r = sqrt(-2.0 * log(u1));
    const double a = 6.283185307179586 * u2;
    p[2 * g] = (T)(r * cos(a));
    if (2 * g + 1 < count) p[2 * g + 1] = (T)(r * sin(a));
}

hipError_t launch_fill_normal(void* p, int64_t count, uint64_t seed, bool f64, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t groups = (count + 1) / 2;
    const int64_t blocks = (groups + 255) / 256;
    if (f64)
        hipLaunchKernelGGL(k_fill_normal<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)p, count, seed);
    else
        hipLaunchKernelGGL(k_fill_normal<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)p, count, seed);
    return hipGetLastError();
}

template <typename T, typename OUT, int VAR>
static void launch_str_t(int tmax, dim3 g, hipStream_t s, const T* A, int64_t lda, const DevTables& tb,
                         const WorkItem* items, OUT* C, double* W) {
    const dim3 b(512);
    // k rows per stage: fourteen operand planes fill most of the LDS
    constexpr int SK1 = std::is_same<T, float>::value ? 16 : 8;
    if (tmax <= 1)
        hipLaunchKernelGGL((k_str<T, OUT, VAR, 1, SK1>), g, b, 0, s, A, lda, tb.tasks, tb.terms, tb.segs, items, C, W);
    else if (tmax <= 2)
        hipLaunchKernelGGL((k_str<T, OUT, VAR, 2, 8>), g, b, 0, s, A, lda, tb.tasks, tb.terms, tb.segs, items, C, W);
    else if (tmax <= 4)
        hipLaunchKernelGGL((k_str<T, OUT, VAR, 4, 8>), g, b, 0, s, A, lda, tb.tasks, tb.terms, tb.segs, items, C, W);
    else
        hipLaunchKernelGGL((k_str<T, OUT, VAR, 8, 8>), g, b, 0, s, A, lda, tb.tasks, tb.terms, tb.segs, items, C, W);
}

template <typename T, typename OUT>
static void launch_str_v(int variant, int tmax, dim3 g, hipStream_t s, const T* A, int64_t lda, const DevTables& tb,
                         const WorkItem* items, OUT* C, double* W) {
    if (variant == 0)
        launch_str_t<T, OUT, 0>(tmax, g, s, A, lda, tb, items, C, W);
    else
        launch_str_t<T, OUT, 1>(tmax, g, s, A, lda, tb, items, C, W);
}

hipError_t launch_str(bool f32, bool out_f64, int variant, int tmax, const void* A, int64_t lda,
                      const DevTables& tb, const WorkItem* items, int nitems, void* C, double* W, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (tmax > kMaxTerms) return hipErrorInvalidValue;
    const dim3 g(nitems);
    if (!f32)
        launch_str_v<double, double>(variant, tmax, g, s, (const double*)A, lda, tb, items, (double*)C, W);
    else if (out_f64)
        launch_str_v<float, double>(variant, tmax, g, s, (const float*)A, lda, tb, items, (double*)C, W);
    else
        launch_str_v<float, float>(variant, tmax, g, s, (const float*)A, lda, tb, items, (float*)C, W);
    return hipGetLastError();
}

hipError_t launch_combine(bool out_f64, const DevCombine* cbs, int ncb, int64_t total, const double* W, void* C,
                          hipStream_t s) {
    if (ncb <= 0 || total <= 0) return hipSuccess;
    const int64_t blocks = (total + 255) / 256;
    if (out_f64)
        hipLaunchKernelGGL(k_combine<double>, dim3((unsigned)blocks), dim3(256), 0, s, cbs, ncb, total, W, (double*)C);
    else
        hipLaunchKernelGGL(k_combine<float>, dim3((unsigned)blocks), dim3(256), 0, s, cbs, ncb, total, W, (float*)C);
    return hipGetLastError();
}

hipError_t launch_gemm_split(bool f32, bool out_f64, const void* A, int64_t lda, const DevTables& tb,
                             const WorkItem* tail, int ntail, int nparts, double* part, void* C, double* W,
                             hipStream_t s, const void* Aops) {
    if (ntail <= 0 || nparts < 1) return hipSuccess;
    const dim3 g(ntail), b(256), gs(GT, ntail / nparts), bs(GT);
    const BatchEntry* nb = nullptr;
    if (!f32) {
        hipLaunchKernelGGL((k_gemmd<double, double, false, true>), g, b, 0, s, (const double*)A, lda, tb.tasks, tb.segs,
                           tail, (double*)C, W, tb.terms, (const double*)Aops, nb, nparts, part);
        hipLaunchKernelGGL(k_tile_part_sum<double>, gs, bs, 0, s, tb.tasks, tail, nparts, (const double*)part,
                           (double*)C, W);
    } else if (out_f64) {
        hipLaunchKernelGGL((k_gemmd<float, double, false, true>), g, b, 0, s, (const float*)A, lda, tb.tasks, tb.segs,
                           tail, (double*)C, W, tb.terms, (const float*)Aops, nb, nparts, part);
        hipLaunchKernelGGL(k_tile_part_sum<double>, gs, bs, 0, s, tb.tasks, tail, nparts, (const double*)part,
                           (double*)C, W);
    } else {
        hipLaunchKernelGGL((k_gemmd<float, float, false, true>), g, b, 0, s, (const float*)A, lda, tb.tasks, tb.segs,
                           tail, (float*)C, W, tb.terms, (const float*)Aops, nb, nparts, part);
        hipLaunchKernelGGL(k_tile_part_sum<float>, gs, bs, 0, s, tb.tasks, tail, nparts, (const double*)part,
                           (float*)C, W);
    }
    return hipGetLastError();
}

hipError_t launch_tile_cat(const double* A, int64_t lda, const DevTables& tb, const WorkItem* items, int nmain,
                           const WorkItem* tail, int ntail, int nparts, double* part, double* C, double* W,
                           hipStream_t s, const double* Aops) {
    if (ntail <= 0 || nparts < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tile_cat<double>), dim3(nmain + ntail), dim3(256), 0, s, A, lda, tb.tasks, tb.terms, tb.segs,
                       items, nmain, tail, C, W, Aops, nparts, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_tile_part_sum<double>), dim3(GT, ntail / nparts), dim3(GT), 0, s, tb.tasks, tail, nparts,
                       (const double*)part, C, W);
    return hipGetLastError();
}

hipError_t launch_opsum(bool f32, const void* A, int64_t lda, const DevTables& tb, const DevOpSum* recs, int nrec,
                        int64_t rows, void* out, hipStream_t s) {
    if (nrec <= 0 || rows <= 0) return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(k_opsum<float>, dim3((unsigned)rows), dim3(256), 0, s, (const float*)A, lda, tb.tasks,
                           tb.terms, tb.segs, recs, nrec, (float*)out);
    else
        hipLaunchKernelGGL(k_opsum<double>, dim3((unsigned)rows), dim3(256), 0, s, (const double*)A, lda, tb.tasks,
                           tb.terms, tb.segs, recs, nrec, (double*)out);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, int64_t count, int elem_bytes, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_fill_zero<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)p, count);
    else if (elem_bytes == 4)
        hipLaunchKernelGGL(k_fill_zero<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)p, count);
    else
        hipLaunchKernelGGL(k_fill_zero<uint8_t>, dim3((unsigned)blocks), dim3(256), 0, s, (uint8_t*)p, count);
    return hipGetLastError();
}

hipError_t launch_colscale(const float* A, int64_t lda, int m, int n, float* part, float* scale, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nch = m > 0 ? (m + 255) / 256 : 0;
    if (nch > 0) hipLaunchKernelGGL(k_colmax_part, dim3((n + 1023) / 1024, nch), dim3(256), 0, s, A, lda, m, n, part);
    hipLaunchKernelGGL(k_colscale, dim3((n + 255) / 256), dim3(256), 0, s, part, nch, n, scale);
    return hipGetLastError();
}

template <typename T>
static void launch_equilibrate_t(const T* A, int64_t lda, int m, int n, T* part, T* scale, T* out, hipStream_t s) {
    const int nch = (m + 255) / 256;
    hipLaunchKernelGGL(k_colmax_t<T>, dim3((n + 255) / 256, nch), dim3(256), 0, s, A, lda, m, n, part);
    hipLaunchKernelGGL(k_eqscale<T>, dim3((n + 255) / 256), dim3(256), 0, s, part, nch, n, scale);
    const int64_t total = (int64_t)m * n;
    hipLaunchKernelGGL(k_scale_cols<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, A, lda, m, n, scale,
                       out);
}

hipError_t launch_equilibrate(bool f32, const void* A, int64_t lda, int m, int n, void* part, void* scale, void* out,
                              hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (f32)
        launch_equilibrate_t<float>((const float*)A, lda, m, n, (float*)part, (float*)scale, (float*)out, s);
    else
        launch_equilibrate_t<double>((const double*)A, lda, m, n, (double*)part, (double*)scale, (double*)out, s);
    return hipGetLastError();
}

hipError_t launch_descale(bool f32, bool out_f64, void* C, int n, const void* scale, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (!f32)
        hipLaunchKernelGGL((k_descale<double, double>), dim3(n), dim3(256), 0, s, (double*)C, (const double*)scale);
    else if (out_f64)
        hipLaunchKernelGGL((k_descale<double, float>), dim3(n), dim3(256), 0, s, (double*)C, (const float*)scale);
    else
        hipLaunchKernelGGL((k_descale<float, float>), dim3(n), dim3(256), 0, s, (float*)C, (const float*)scale);
    return hipGetLastError();
}

hipError_t launch_prep_lp(int mode, const float* A, int64_t lda, int m, int n, int ldt, const float* scale,
                          void* out0, void* out1, hipStream_t s) {
    if (n <= 0 || ldt <= 0) return hipSuccess;
    const dim3 g((ldt + 127) / 128, (n + 63) / 64);
    if (mode == 0)
        hipLaunchKernelGGL(k_prep_lp<0>, g, dim3(256), 0, s, A, lda, m, n, ldt, scale, out0, out1);
    else
        hipLaunchKernelGGL(k_prep_lp<1>, g, dim3(256), 0, s, A, lda, m, n, ldt, scale, out0, out1);
    return hipGetLastError();
}

// Launch of the reduced-precision tiles of mode / output type / split form
// by staging path: 2 direct-to-LDS 16-byte copies, 1 dword copies,
// 0 through registers.
template <int M, typename O, bool S>
static void lp_tiles(int path, dim3 g, hipStream_t s, const uint8_t* t0, const uint8_t* t1, int ldt,
                     const float* scale, const DevTables& tb, const WorkItem* items, void* C, double* W, int nparts,
                     double* part) {
    const dim3 b(256);
    if (path == 2)
        hipLaunchKernelGGL((k_gemm_lpd<M, O, S, true>), g, b, 0, s, t0, t1, ldt, scale, tb.tasks, tb.terms, tb.segs,
                           items, (O*)C, W, nparts, part);
    else if (path == 1)
        hipLaunchKernelGGL((k_gemm_lpd<M, O, S, false>), g, b, 0, s, t0, t1, ldt, scale, tb.tasks, tb.terms, tb.segs,
                           items, (O*)C, W, nparts, part);
    else
        hipLaunchKernelGGL((k_gemm_lp<M, O, S>), g, b, 0, s, t0, t1, ldt, scale, tb.tasks, tb.terms, tb.segs, items,
                           (O*)C, W, nparts, part);
}

// Staging path for windows aligned on `align` (0: none, 1: dwords, 2: 16
// bytes) of a copy with rows of ldt elements: direct-to-LDS copies need the
// byte offsets of one 64-row copy block below 2^31.
static int lp_path(int mode, int ldt, int align) {
    const int eb = mode == 0 ? 2 : 1;
    if ((int64_t)64 * ldt * eb >= ((int64_t)1 << 31)) return 0;
    return align;
}

hipError_t launch_gemm_lp(int mode, bool out_f64, const void* T0, const void* T1, int ldt, const float* scale,
                          const DevTables& tb, const WorkItem* items, int nitems, void* C, double* W,
                          hipStream_t s, int align) {
    if (nitems <= 0) return hipSuccess;
    const dim3 g(nitems);
    const uint8_t* t0 = (const uint8_t*)T0;
    const uint8_t* t1 = (const uint8_t*)(T1 ? T1 : T0);
    const int path = lp_path(mode, ldt, align);
    if (mode == 0 && out_f64) lp_tiles<0, double, false>(path, g, s, t0, t1, ldt, scale, tb, items, C, W, 1, nullptr);
    else if (mode == 0) lp_tiles<0, float, false>(path, g, s, t0, t1, ldt, scale, tb, items, C, W, 1, nullptr);
    else if (out_f64) lp_tiles<1, double, false>(path, g, s, t0, t1, ldt, scale, tb, items, C, W, 1, nullptr);
    else lp_tiles<1, float, false>(path, g, s, t0, t1, ldt, scale, tb, items, C, W, 1, nullptr);
    return hipGetLastError();
}

hipError_t launch_lp8_big(const void* T0, int ldt, const float* scale, const DevTables& tb, const WorkItem* items,
                          int nitems, double* C, double* W, hipStream_t s, int nparts, float* part) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lp8_big, dim3(nitems), dim3(512), 0, s, (const uint8_t*)T0, ldt, scale, tb.tasks, tb.terms,
                       tb.segs, items, C, W, nparts, part);
    return hipGetLastError();
}

hipError_t launch_lp8_tail_sum(const float* scale, const DevTables& tb, const WorkItem* tail, int ntiles, int nparts,
                               const float* part, double* C, double* W, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lp8_tail_sum, dim3(kBigTile, ntiles), dim3(kBigTile), 0, s, scale, tb.tasks, tb.terms, tail,
                       nparts, part, C, W);
    return hipGetLastError();
}

hipError_t launch_gemm_lp_split(int mode, bool out_f64, const void* T0, const void* T1, int ldt, const float* scale,
                                const DevTables& tb, const WorkItem* tail, int ntail, int nparts, double* part,
                                void* C, double* W, hipStream_t s, int align) {
    if (ntail <= 0 || nparts < 1) return hipSuccess;
    const dim3 g(ntail), gs(GT, ntail / nparts), bs(GT);
    const uint8_t* t0 = (const uint8_t*)T0;
    const uint8_t* t1 = (const uint8_t*)(T1 ? T1 : T0);
    const int path = lp_path(mode, ldt, align);
    if (mode == 0 && out_f64) lp_tiles<0, double, true>(path, g, s, t0, t1, ldt, scale, tb, tail, C, W, nparts, part);
    else if (mode == 0) lp_tiles<0, float, true>(path, g, s, t0, t1, ldt, scale, tb, tail, C, W, nparts, part);
    else if (out_f64) lp_tiles<1, double, true>(path, g, s, t0, t1, ldt, scale, tb, tail, C, W, nparts, part);
    else lp_tiles<1, float, true>(path, g, s, t0, t1, ldt, scale, tb, tail, C, W, nparts, part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (out_f64)
        hipLaunchKernelGGL(k_tile_part_sum<double>, gs, bs, 0, s, tb.tasks, tail, nparts, (const double*)part,
                           (double*)C, W);
    else
        hipLaunchKernelGGL(k_tile_part_sum<float>, gs, bs, 0, s, tb.tasks, tail, nparts, (const double*)part,
                           (float*)C, W);
    return hipGetLastError();
}

hipError_t launch_opsum_lp(int mode, const float* A, int64_t lda, const DevTables& tb, const DevOpSum* recs, int nrec,
                           int64_t tiles, int64_t rows, uint32_t* colmax, float* scale, void* out0, void* out1, int ldt,
                           hipStream_t s) {
    if (nrec <= 0 || tiles <= 0) return hipSuccess;
    const dim3 g((unsigned)tiles), b(256);
    if (mode == 0) {
        hipLaunchKernelGGL((k_opsum_lp<0, false>), g, b, 0, s, A, lda, tb.tasks, tb.terms, tb.segs, recs, nrec, colmax,
                           scale, out0, out1, ldt);
    } else {
        const hipError_t e = launch_fill_zero(colmax, rows, 4, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_opsum_lp<1, true>), g, b, 0, s, A, lda, tb.tasks, tb.terms, tb.segs, recs, nrec, colmax,
                           scale, out0, out1, ldt);
        hipLaunchKernelGGL((k_opsum_lp<1, false>), g, b, 0, s, A, lda, tb.tasks, tb.terms, tb.segs, recs, nrec, colmax,
                           scale, out0, out1, ldt);
    }
    return hipGetLastError();
}

hipError_t launch_convert(int mode, const float* x, int64_t count, void* out0, void* out1, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_convert, dim3((unsigned)blocks), dim3(256), 0, s, mode, x, count, out0, out1);
    return hipGetLastError();
}

}  // namespace atalib
