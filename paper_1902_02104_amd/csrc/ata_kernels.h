// Launchers of the gfx950 kernels (defined in ata_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ata_plan.h"

namespace atalib {

// Task tables of one plan in device memory.
struct DevTables {
    const DevTask* tasks;
    const DevTerm* terms;
    const int32_t* segs;
};

// Classical tiles (TK_SYRK / TK_GEMM) on FP64 or FP32 MFMA.  out_f64 selects
// a double C for float input.
// Aops: base of the operand-sum buffers read by tasks with src == 1.
hipError_t launch_gemm(bool f32, bool out_f64, const void* A, int64_t lda, const DevTables& tb,
                       const WorkItem* items, int nitems, void* C, double* W, hipStream_t s,
                       const void* Aops = nullptr);

// FP64 tiles on 16-byte direct-to-LDS copies: nt = 1 for classical tiles
// (TK_SYRK / TK_GEMM, and products on operand-sum buffers through Aops),
// nt = 2 for Strassen product tiles with at most two terms per operand (and
// the classical tiles launched with them).  queue (nt = 2): kTileQueues ints
// of device memory, cleared by the launch, which then runs persistent
// workgroups taking the items from per-XCD work queues; null: one workgroup
// per item.
hipError_t launch_tile(int nt, const double* A, int64_t lda, const DevTables& tb, const WorkItem* items, int nitems,
                       double* C, double* W, hipStream_t s, const double* Aops = nullptr, int* queue = nullptr);

// e4m3 classical tiles of 256 x 256 (items index kBigTile tiles) on the
// transposed copy T0 (row stride ldt bytes, windows on 16 elements, 64 ldt
// below 2^31), FP64 output.
// nparts > 1: the items are K-split tiles (slot = tile * nparts + part) whose
// raw FP32 results go to part (kBigTile^2 floats per slot); then
// launch_lp8_tail_sum sums them (ntiles tiles, the first item of each tile's
// run describing it) into C.
hipError_t launch_lp8_big(const void* T0, int ldt, const float* scale, const DevTables& tb, const WorkItem* items,
                          int nitems, double* C, double* W, hipStream_t s, int nparts = 1, float* part = nullptr);
hipError_t launch_lp8_tail_sum(const float* scale, const DevTables& tb, const WorkItem* tail, int ntiles, int nparts,
                               const float* part, double* C, double* W, hipStream_t s);

// The same for a launch of k_gemmd tiles (FP32, or FP64 batched/operand-sum
// launches); C of the launch's output type.
hipError_t launch_gemm_split(bool f32, bool out_f64, const void* A, int64_t lda, const DevTables& tb,
                             const WorkItem* tail, int ntail, int nparts, double* part, void* C, double* W,
                             hipStream_t s, const void* Aops = nullptr);

// The same for the reduced-precision classical tiles (partials de-scaled).
hipError_t launch_gemm_lp_split(int mode, bool out_f64, const void* T0, const void* T1, int ldt, const float* scale,
                                const DevTables& tb, const WorkItem* tail, int ntail, int nparts, double* part,
                                void* C, double* W, hipStream_t s, int align);

// A one-term FP64 tile launch with its K-split last round in the same grid
// (the parts run as the whole tiles finish), then the sum of the parts.
hipError_t launch_tile_cat(const double* A, int64_t lda, const DevTables& tb, const WorkItem* items, int nmain,
                           const WorkItem* tail, int ntail, int nparts, double* part, double* C, double* W,
                           hipStream_t s, const double* Aops);

// Operand sums of the product tasks in `recs` (one workgroup per buffer row;
// rows = total rows of the records) into `out`, in the input type.
hipError_t launch_opsum(bool f32, const void* A, int64_t lda, const DevTables& tb, const DevOpSum* recs, int nrec,
                        int64_t rows, void* out, hipStream_t s);

// Strassen product tiles: classical tiles whose operands are signed sums of
// up to tmax terms (column padding reads as zero), written to the workspace.
hipError_t launch_gemm_terms(bool f32, bool out_f64, int tmax, const void* A, int64_t lda, const DevTables& tb,
                             const WorkItem* items, int nitems, void* C, double* W, hipStream_t s);

// Classical tiles of several requests in one launch: work item w uses
// batch[w.slot] for its matrices and tables.
hipError_t launch_gemm_batch(bool f32, bool out_f64, const BatchEntry* batch, const WorkItem* items, int nitems,
                             hipStream_t s);

// Fill count elements with i.i.d. standard normal values drawn from
// (seed, element index) by Philox4x32-10 and the Box-Muller transform.
hipError_t launch_fill_normal(void* p, int64_t count, uint64_t seed, bool f64, hipStream_t s);

// In-tile Strassen tiles (TK_STR).  tmax: most operand terms of any task.
hipError_t launch_str(bool f32, bool out_f64, int variant, int tmax, const void* A, int64_t lda,
                      const DevTables& tb, const WorkItem* items, int nitems, void* C, double* W,
                      hipStream_t s);

// Workspace combinations (FP64 workspace) into packed C.
hipError_t launch_combine(bool out_f64, const DevCombine* cbs, int ncb, int64_t total, const double* W,
                          void* C, hipStream_t s);

hipError_t launch_fill_zero(void* p, int64_t count, int elem_bytes, hipStream_t s);

// Reduced-precision forms.  The prepass writes A^t (columns of A as rows,
// rows of A along the contiguous axis, padded with zeros to ldt) converted
// to bfloat16 hi/lo planes (mode 0) or to scaled OCP e4m3 (mode 1).
// For mode 1 the per-column power-of-two scales are computed first from the
// column maxima (partial maxima per 256-row chunk in `part`).
hipError_t launch_colscale(const float* A, int64_t lda, int m, int n, float* part, float* scale,
                           hipStream_t s);
hipError_t launch_prep_lp(int mode, const float* A, int64_t lda, int m, int n, int ldt, const float* scale,
                          void* out0, void* out1, hipStream_t s);
// Strassen operands of the reduced-precision forms: the operand sums of the
// records (FP32, term order) converted into rows of the operand copy (mode 0
// bfloat16 hi/lo planes, mode 1 scaled e4m3 with per-row scales; colmax holds
// `rows` words of scratch for mode 1).  tiles: 64 x 64 conversion tiles of
// all records.
hipError_t launch_opsum_lp(int mode, const float* A, int64_t lda, const DevTables& tb, const DevOpSum* recs, int nrec,
                           int64_t tiles, int64_t rows, uint32_t* colmax, float* scale, void* out0, void* out1, int ldt,
                           hipStream_t s);
// align: 2 when every segment window of the plan starts and ends on 16
// bytes of the copy (or ends at its last row, past which the copy holds
// zeros), 1 when on dwords, else 0 (see lp_windows_aligned): the tiles stage
// through 16-byte or dword direct-to-LDS copies, or through registers.
hipError_t launch_gemm_lp(int mode, bool out_f64, const void* T0, const void* T1, int ldt,
                          const float* scale, const DevTables& tb, const WorkItem* items, int nitems,
                          void* C, double* W, hipStream_t s, int align);

// Column equilibration (power-of-two column scales into `scale`, the scaled
// copy of A into `out` with row stride n; `part` holds ceil(m/256) x n
// partial maxima) and its inverse on packed lower C.
hipError_t launch_equilibrate(bool f32, const void* A, int64_t lda, int m, int n, void* part, void* scale, void* out,
                              hipStream_t s);
hipError_t launch_descale(bool f32, bool out_f64, void* C, int n, const void* scale, hipStream_t s);

// Element conversions exposed for verification: mode 0 -> bfloat16 hi/lo
// (uint16 pairs), mode 1 -> OCP e4m3 bytes (no scaling).
hipError_t launch_convert(int mode, const float* x, int64_t count, void* out0, void* out1, hipStream_t s);

// Consumers of the packed product (ata_chol.hip), FP64 or FP32 throughout.
// Cholesky factor of packed lower C in place; info (device, may be null)
// receives the first failing column + 1 if it is still 0.  s2 (may be null):
// helper stream for the lookahead, with two events e and f; the work on s2 is
// joined back into s before the call returns.
hipError_t launch_potrf(bool f32, void* C, int64_t n, int32_t* info, hipStream_t s, hipStream_t s2, hipEvent_t e,
                        hipEvent_t f);
// L L^t X = B in place, B row-major n x nrhs with row stride ldb.
hipError_t launch_potrs(bool f32, const void* L, int64_t n, void* B, int64_t nrhs, int64_t ldb, hipStream_t s);
// out (m x nrhs, row stride ldo) = A X for A m x n (row stride lda) and X
// n x nrhs (row stride ldx), FP64 sums.
hipError_t launch_ax(bool f32, const void* A, int64_t m, int64_t n, int64_t lda, const void* X, int64_t nrhs,
                     int64_t ldx, void* out, int64_t ldo, hipStream_t s);
// out (n x m, row stride m) = A^t for A m x n with row stride lda; elements of
// elem_bytes 4 or 8.
hipError_t launch_transpose(int elem_bytes, const void* A, int64_t m, int64_t n, int64_t lda, void* out,
                            hipStream_t s);
// out = A^t B; part holds atb_chunks(m, n) x n x nrhs doubles.
int64_t atb_chunks(int64_t m, int64_t n);
hipError_t launch_atb(bool f32, const void* A, int64_t m, int64_t n, int64_t lda, const void* B, int64_t nrhs,
                      int64_t ldb, void* out, int64_t ldo, double* part, hipStream_t s);

}  // namespace atalib
