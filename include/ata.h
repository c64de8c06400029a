/*
 * ata.h - C ABI of the MI355X A^t A library (libata.so).
 *
 * Computes the lower triangle of the symmetric product C = A^t A of a
 * rectangular m x n matrix A by the ATA recursion (Section 3, Algorithm 1):
 * A is split into quadrants with m1 = ceil(m/2), m2 = floor(m/2),
 * n1 = ceil(n/2), n2 = floor(n/2); the diagonal blocks
 * C11 = A11^t A11 + A21^t A21 and C22 = A12^t A12 + A22^t A22 come from
 * recursive ATA calls whose second product is accumulated into the first, and
 * the off-diagonal block C21 = A12^t A11 + A22^t A21 from rectangular Strassen
 * products (HASA); C12 is never formed.  The recursion stops when m or n is at
 * most the cutoff (the paper uses 32) and the block is then multiplied
 * classically.
 *
 * Layout (the paper fixes neither):
 *   A        row-major, element (i, j) at A[i * lda + j], lda >= n, device
 *            memory, read only.
 *   C_lower  row-major packed lower triangle: element (i, j), j <= i, at
 *            C_lower[i * (i + 1) / 2 + j]; n (n + 1) / 2 elements, device
 *            memory, overwritten (never read).  This is also LAPACK's
 *            column-major packed upper storage of the same matrix.
 *
 * Every call is asynchronous on the given HIP stream (0 = the null stream);
 * a status of ATA_OK means the work was enqueued.  Errors raised by kernels
 * surface at the caller's next synchronisation.  Calls on different streams
 * may overlap; the plan cache is shared and thread safe.
 *
 * Return codes: 0 = ATA_OK; a negative value -k means the k-th argument is
 * invalid (LAPACK convention); positive values are runtime errors (below).
 */
#ifndef ATA_H
#define ATA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes */
#define ATA_OK 0
#define ATA_ENOMEM 1         /* device or host allocation failed */
#define ATA_EHIP 2           /* a HIP runtime call failed (see ata_last_hip_error) */
#define ATA_EUNSUPPORTED 3   /* device is not gfx950, or option not supported */
#define ATA_EWORKSPACE 4     /* caller workspace smaller than ata_workspace_bytes */
#define ATA_EREJECT 5        /* serving: request can never fit the memory budget */
#define ATA_EBUSY 6          /* serving: queue full, retry later */
#define ATA_ENOTFOUND 7      /* serving: unknown ticket */
#define ATA_EPENDING 8       /* serving: request not finished yet */

/* Arithmetic forms.  The low byte selects input type and leaf arithmetic;
 * ATA_OUT_F64 selects a double-precision C for the float-input forms. */
#define ATA_F64 0         /* A double, C double; FP64 MFMA leaves */
#define ATA_F32 1         /* A float; FP32 MFMA leaves */
#define ATA_F32_BF16X3 2  /* A float; bfloat16 split leaves: x = hi + lo,
                             hi^t hi + hi^t lo + lo^t hi, FP32 accumulation */
#define ATA_F32_FP8 3     /* A float; OCP e4m3 leaves with per-column
                             power-of-two scales, FP32 accumulation */
#define ATA_OUT_F64 0x100 /* with 1..3: C is double instead of float */

/* Strassen variants for the HASA products */
#define ATA_VARIANT_STRASSEN 0 /* Strassen 1969: 7 products, 18 additions */
#define ATA_VARIANT_WINOGRAD 1 /* Winograd 1971: 7 products, 15 additions */

/* Options for ata_ex / ata_workspace_bytes / ata_plan_info.
 * Zero-initialise, then set fields; a NULL pointer means all defaults. */
typedef struct ata_opts {
    int32_t variant;     /* ATA_VARIANT_*; default Strassen */
    int32_t max_depth;   /* Strassen levels per HASA call: -1 = unlimited
                            (the paper's rule: recurse while min(M,K,N) >
                            cutoff), 0 = classical off-diagonal products,
                            k > 0 = at most k levels.  Default when the
                            struct is NULL: ATA_DEFAULT_MAX_DEPTH. */
    int32_t flags;       /* ATA_OPT_* bits, default 0 */
    int32_t reserved;
} ata_opts;

/* ata_opts.flags: Strassen product tiles.  Without it (when an options
 * struct is given) the last Strassen level of each off-diagonal product runs
 * inside the workgroup tile (seven products in registers, combined in the
 * epilogue).  With this flag every level up to two (one for Winograd) is
 * expanded into signed operand terms instead: each of the 7^d products is a
 * classical tile whose staging sums the terms, written to the workspace and
 * combined by a separate pass.  FP64 products with at most two terms per
 * operand (one level) run in the same launch as the phase's classical tiles.
 * A NULL options struct selects this form for ATA_F64. */
#define ATA_OPT_PRODUCT_TILES 0x1
/* ata_opts.flags: with product tiles, form each product's operand sums in a
 * memory pass (the explicit sums of the paper's HASA listing) into the
 * workspace and run the products as plain classical tiles on them.  Trades
 * one pass over the operands for classical-tile efficiency of the products.
 * Implies ATA_OPT_PRODUCT_TILES. */
#define ATA_OPT_OPERAND_SUMS 0x4
/* ata_opts.flags: column equilibration.  Columns of A are scaled by powers
 * of two (each column's largest magnitude into [1, 2)) before the product
 * and C is scaled back, both exactly unless entries underflow.  The error of
 * each C_ij then scales with its own two columns, which matters for Strassen
 * levels when column sizes span many orders of magnitude.  Costs one pass
 * over A and m x n elements of workspace.  FP64 and FP32 only (the reduced-
 * precision forms scale columns themselves). */
#define ATA_OPT_EQUILIBRATE 0x2
/* ata_opts.flags: adaptive depth.  A Strassen level of an off-diagonal
 * product is taken only where it is faster than classical tiles by a cost
 * model of this library's tile kernels: tile counts of the product before and
 * after the split, the measured fractions of the MFMA peak that classical
 * tiles and Strassen tiles reach on gfx950, and the cost of the combination.
 * max_depth still caps the levels.  (The paper's HASA stops at the cutoff
 * alone; this is its adaptive stopping rule driven by measured rates.) */
#define ATA_OPT_ADAPTIVE 0x8
/* ata_opts.flags: equilibrate (as ATA_OPT_EQUILIBRATE) exactly when the plan
 * runs a Strassen level, whose error bound depends on the largest columns;
 * classical products keep each entry's error relative to its own columns
 * without it. */
#define ATA_OPT_EQUILIBRATE_AUTO 0x10

/* Defaults when the options struct is NULL: Strassen variant, at most
 * ATA_DEFAULT_MAX_DEPTH levels, flags ATA_DEFAULT_FLAGS (adaptive depth and
 * equilibration with Strassen levels), and for ATA_F64 the product-tile
 * form, the faster of the fused forms there.  A second level costs more in
 * operand-sum traffic than its 1/8 saving in multiplications on gfx950. */
#define ATA_DEFAULT_MAX_DEPTH 1
#define ATA_DEFAULT_FLAGS (ATA_OPT_ADAPTIVE | ATA_OPT_EQUILIBRATE_AUTO)
#define ATA_MAX_DEPTH_LIMIT 4 /* deepest supported Strassen level count */

/*
 * ata: C_lower = lower(A^t A) for the m x n matrix A (Algorithm 1).
 *   A        device pointer (double for ATA_F64, else float), lda >= max(n,1);
 *            rows longer than 64 MiB (lda x element bytes) give
 *            ATA_EUNSUPPORTED
 *   m, n     >= 0.  n == 0: nothing is written; m == 0: C_lower is zeroed
 *            (empty sum).
 *   C_lower  device pointer, n(n+1)/2 elements of the output type
 *   dtype    one of ATA_F64, ATA_F32, ATA_F32_BF16X3, ATA_F32_FP8, the last
 *            three optionally OR-ed with ATA_OUT_F64
 *   cutoff   > 0: base case when m <= cutoff or n <= cutoff (Algorithm 1);
 *            HASA stops at min(M, K, N) <= cutoff.  0 = tuned default for
 *            the shape.  cutoff >= min(m, n) gives one classical product.
 *   stream   hipStream_t (as void*), 0 for the null stream
 * Uses the default options (NULL ata_opts) and allocates its workspace
 * stream-ordered on `stream`: Strassen products, K-split partial tiles (of
 * launches with few tiles, and of the short last round of a launch of
 * classical tiles), operand copies of the reduced-precision forms.
 */
int ata(const void *A, int64_t m, int64_t n, int64_t lda, void *C_lower, int dtype,
        int cutoff, void *stream);

/*
 * ata_aat: the companion product C_lower = lower(A A^t), m x m packed, for
 *   the same row-major A (m x n, row stride lda >= n).  A A^t is the product
 *   of the n x m matrix A^t with itself, so the call writes A^t into a
 *   stream-ordered workspace (n x m elements, one pass over A) and runs ata
 *   on it with default options; every dtype of ata is accepted.  Argument
 *   codes as for ata (C_lower holds m (m + 1) / 2 elements).
 */
int ata_aat(const void *A, int64_t m, int64_t n, int64_t lda, void *C_lower, int dtype, int cutoff, void *stream);

/*
 * ata_ex: as ata, with options and an optional caller workspace.
 *   opts       NULL for defaults
 *   workspace  device memory of ws_bytes, or NULL: the library then
 *              allocates it stream-ordered.  Must not be used by other work
 *              until the call's work on `stream` has completed.
 */
int ata_ex(const void *A, int64_t m, int64_t n, int64_t lda, void *C_lower, int dtype, int cutoff,
           void *stream, const ata_opts *opts, void *workspace, size_t ws_bytes);

/*
 * ata_ex_noalloc: as ata_ex, for callers that cannot allocate device memory
 *   (code under HIP graph capture, tight serving loops, harnesses that forbid
 *   allocation).  It calls no hipMalloc, hipFree or other allocating routine:
 *   the plan's task tables and the whole workspace live in one fixed device
 *   array of ATA_NOALLOC_SCRATCH_BYTES per GPU, which the library holds until
 *   the process ends.  The tables are copied there (hipMemcpyAsync from host
 *   memory) on every call; the product runs with K splitting off (its
 *   partial sums would need workspace; so is the split of a short last round
 *   of tiles) and without the helper stream, so
 *   floating-point results may differ from ata_ex in rounding order only
 *   (integer-valued inputs give identical results).
 *   scratch_used  if not NULL: bytes of the array the call needs (set also
 *                 when the call is rejected for size).
 * Returns ATA_EWORKSPACE when tables plus workspace exceed the array; other
 * codes as for ata_ex.  Every call on one GPU uses that GPU's single array,
 * which keeps the last call's contents: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 */
#define ATA_NOALLOC_SCRATCH_BYTES (64u << 20)
int ata_ex_noalloc(const void *A, int64_t m, int64_t n, int64_t lda, void *C_lower, int dtype, int cutoff,
                   void *stream, const ata_opts *opts, size_t *scratch_used);

/* Bytes of device workspace ata_ex needs for this problem (0 if none;
 * classical launches of more than one round of tiles (FP64, FP32, bfloat16
 * pairs) need some for the K parts of their last round). */
int ata_workspace_bytes(int64_t m, int64_t n, int dtype, int cutoff, const ata_opts *opts,
                        size_t *bytes);

/*
 * Reduced-precision forms (ATA_F32_BF16X3, ATA_F32_FP8): the ATA recursion is
 * unchanged and the leaves run on a transposed converted copy of A.  With a
 * NULL options struct (or max_depth 0) the off-diagonal products are
 * classical.  max_depth 1 or 2 (1 for Winograd) runs HASA levels as product
 * tiles on operand sums: each product's signed sums of quadrant terms are
 * formed in FP32 from A and then converted (bfloat16 hi/lo split, or e4m3
 * with a power-of-two scale per operand column from the sums' own maxima);
 * deeper levels and ATA_OPT_EQUILIBRATE return ATA_EUNSUPPORTED.  BF16x3
 * adds its FP32 MFMA accumulators into FP64 every 512 rows; e4m3 accumulates
 * in FP32 over the whole K.  Strassen combinations and the workspace are FP64.
 * ATA_F32 leaves support Strassen levels like ATA_F64.
 */

/*
 * ata_precision_convert: the element conversions of the reduced-precision
 * forms, for verification.  x: `count` floats in device memory.
 *   ATA_F32_BF16X3: out0[i] = bfloat16 bits of x[i] rounded to nearest even
 *                   (hi), out1[i] = bits of bf16(x[i] - hi) (lo); uint16 each.
 *   ATA_F32_FP8:    out0[i] = OCP e4m3 byte of x[i], nearest even, saturated
 *                   to +-448 (no scaling applied); out1 unused.
 * Asynchronous on `stream`.
 */
int ata_precision_convert(int dtype, const float *x, int64_t count, void *out0, void *out1, void *stream);

/* Host-only description of the plan (no GPU needed). */
typedef struct ata_plan_stats {
    int64_t mults;           /* scalar multiplications of the method */
    int64_t classical_mults; /* m * n (n + 1) / 2 */
    int64_t syrk_tasks;      /* diagonal base-case blocks */
    int64_t gemm_tasks;      /* classical off-diagonal products */
    int64_t strassen_tasks;  /* in-tile Strassen products (7 leaf products each) */
    int64_t combine_tasks;   /* workspace combinations */
    int64_t work_items;      /* workgroup tiles over all launches */
    int64_t phases;          /* ordered launch groups */
    int64_t ata_depth;       /* levels of the ATA recursion */
    int64_t max_hasa_depth;  /* deepest Strassen level count */
    int64_t workspace_bytes;
    int64_t cutoff;          /* cutoff used (after resolving 0) */
    int64_t strassen_mults;  /* multiplications done by in-tile Strassen tiles */
    int64_t gemm_mults;      /* ... by classical off-diagonal tiles */
    int64_t syrk_mults;      /* ... by diagonal base-case tiles */
    int64_t combine_elems;   /* output elements formed by workspace combinations */
    int64_t lp_staging;      /* reduced-precision dtypes: how the 128 x 128 tiles stage their
                                operands, as the plan's K windows allow: 2 direct-to-LDS copies
                                of 16 bytes, 1 of dwords, 0 through registers (copy rows of
                                2^31 / 64 bytes or more always stage through registers);
                                -1 for other dtypes */
} ata_plan_stats;

int ata_plan_info(int64_t m, int64_t n, int dtype, int cutoff, const ata_opts *opts,
                  ata_plan_stats *out);

/* Default cutoff chosen for a shape when cutoff == 0: 128 when
 * min(m, n) <= 1024; otherwise 512, except 256 for float input (dtype other
 * than ATA_F64) with min(m, n) <= 4096 and m < 4 n. */
int ata_default_cutoff(int64_t m, int64_t n, int dtype);

/* Text for a status code (static storage). */
const char *ata_status_string(int status);

/* HIP error code of the last ATA_EHIP on this thread (0 if none). */
int ata_last_hip_error(void);

/* Library version as "major.minor.patch" (static storage). */
const char *ata_version(void);

/* Release cached plans, device task tables and the library's helper
 * streams (all devices).  Waits for every device holding such tables to go
 * idle first, since queued products read them.  Products of the serving
 * loop keep their own references and are not affected. */
void ata_release_caches(void);

/*
 * Kernel timing for measurement tools.  While enabled, every kernel launch the
 * library makes is bracketed by HIP events recorded on the launch's stream.
 * ata_profile_collect waits for the recorded events, writes the summed
 * duration in milliseconds and the launch count per kernel kind
 * (ATA_KERNEL_*), clears the record and returns the number of kinds written.
 * Enabling adds two event records per launch; it never synchronises.
 */
#define ATA_KERNEL_STRASSEN 0 /* in-tile Strassen tiles */
#define ATA_KERNEL_GEMM 1     /* classical off-diagonal tiles */
#define ATA_KERNEL_SYRK 2     /* diagonal base-case tiles */
#define ATA_KERNEL_COMBINE 3  /* workspace combinations */
#define ATA_KERNEL_OTHER 4    /* fills and conversions */
#define ATA_KERNEL_FACTOR_PANEL 5  /* Cholesky diagonal blocks and row solves */
#define ATA_KERNEL_FACTOR_UPDATE 6 /* Cholesky trailing updates */
#define ATA_KERNEL_SOLVE 7         /* triangular solves and A^t B */
#define ATA_KERNEL_TILES 8         /* FP64 product tiles and classical tiles of a
                                      phase in one launch */
#define ATA_KERNEL_KINDS 9
int ata_profile_enable(int on);
int ata_profile_collect(double *ms, int64_t *launches, int kinds);

/* ------------------------------------------------------------------------ */
/* Serving: a persistent loop for streams of Gram-matrix requests            */
/* ------------------------------------------------------------------------ */
/*
 * A server owns a device memory pool of `budget_bytes` and a scheduler
 * thread.  Requests are admitted in arrival order when their footprint
 * (A + packed C + workspace of their plan) fits in the free pool and fewer
 * than `max_active` requests are in flight; up to 8 queued requests behind a
 * blocked one may be admitted first if they fit.  Admitted requests run
 * concurrently on `streams` HIP streams; requests whose plan is a single
 * classical diagonal block (n or m at most the cutoff) are batched into one
 * grouped launch per scheduler pass.  A result is bit-identical whether the
 * request ran alone or in a mix: its tiles, their K order and the kernels are
 * a function of the request only.  Results stay in the pool until taken.
 * Calls are thread safe.
 */
typedef struct ata_server ata_server;

#define ATA_SRC_HOST 0   /* copy A from host memory `a` (m x n, row stride n) */
#define ATA_SRC_DEVICE 1 /* copy A from device memory `a` (row stride n) */
#define ATA_SRC_NORMAL 2 /* i.i.d. N(0,1) entries drawn on the device from `seed`
                            (Philox4x32-10 counter = element pair, Box-Muller) */

typedef struct ata_request {
    int64_t m, n;
    int32_t dtype;     /* ATA_F64 or ATA_F32 */
    int32_t cutoff;    /* 0 = default */
    int32_t max_depth; /* Strassen levels, -2 = library default */
    int32_t src;       /* ATA_SRC_* */
    const void *a;     /* source of A for ATA_SRC_HOST / ATA_SRC_DEVICE; must
                          stay valid until the request has been admitted */
    uint64_t seed;     /* ATA_SRC_NORMAL */
    int32_t keep_a;    /* 1: keep A in the pool until taken (ata_server_take
                          can copy it out); 0: free it when the product ends */
    int32_t reserved;  /* must be 0 */
} ata_request;

#define ATA_REQ_QUEUED 0
#define ATA_REQ_ADMITTED 1
#define ATA_REQ_RUNNING 2
#define ATA_REQ_DONE 3

typedef struct ata_request_info {
    int32_t state;      /* ATA_REQ_* */
    int32_t status;     /* ATA_OK or the error the request ended with */
    int64_t m, n;
    double t_submit;    /* seconds on the server's steady clock */
    double t_admit, t_launch, t_done;
    int32_t batched;    /* 1 if it ran in a grouped launch */
    int32_t stream;     /* stream index it ran on */
    int64_t footprint;  /* bytes held in the pool while in flight */
    double flops;       /* m * n * n, the classical count of the metric */
    int32_t slabs;      /* row slabs it ran in (1 unless chunked: requests
                           above 4e10 flops run in slabs of about 2e10, each
                           launched after the previous one completes) */
    int32_t reserved;
} ata_request_info;

typedef struct ata_server_stats {
    int64_t submitted, admitted, completed, rejected;
    int64_t batches;          /* grouped launches */
    int64_t batched_requests; /* requests that ran in grouped launches */
    int64_t pool_bytes, pool_in_use, pool_peak;
    int64_t queued, active;
} ata_server_stats;

#define ATA_SERVER_SIMULATE 1 /* host-only: no device memory or kernels; a
                                 request completes flops / (simulate_tflops 1e12)
                                 seconds after admission.  For scheduler tests. */
/* In simulate mode a request with src ATA_SRC_NORMAL and this seed ends with
 * status ATA_EHIP, to exercise the failure path. */
#define ATA_SERVER_SIM_FAIL_SEED 0xFFFFFFFFFFFFFFFFull

/* budget_bytes > 0; max_active >= 1; streams in [1, 16]; flags ATA_SERVER_*. */
int ata_server_create(size_t budget_bytes, int max_active, int streams, int flags, double simulate_tflops,
                      ata_server **out);
/* Queue a request.  ATA_EREJECT if its footprint exceeds the budget, negative
 * codes for invalid fields.  The ticket identifies it in the calls below. */
int ata_server_submit(ata_server *srv, const ata_request *req, uint64_t *ticket);
/* ATA_OK when done (info filled), ATA_EPENDING while queued or running. */
int ata_server_query(ata_server *srv, uint64_t ticket, ata_request_info *info);
/* Block until done or timeout_s elapses (ATA_EPENDING). */
int ata_server_wait(ata_server *srv, uint64_t ticket, double timeout_s, ata_request_info *info);
/* Copy the packed result (n(n+1)/2 elements of the request's type) to `c`
 * and, if `a` is not NULL, the request's A (m x n, row-major; it must have
 * been submitted with keep_a = 1, else -4) to `a`; both are device memory if
 * on_device, else host memory.  Either pointer may be NULL.  Then release the
 * request's pool memory.  A request that ended with an error is released by
 * this call (nothing is copied) and its error status is returned. */
int ata_server_take(ata_server *srv, uint64_t ticket, void *c, void *a, int on_device);
/* Release a finished request without copying anything. */
int ata_server_release(ata_server *srv, uint64_t ticket);
int ata_server_get_stats(ata_server *srv, ata_server_stats *out);
/* Seconds on the server's steady clock (the clock of the info timestamps). */
double ata_server_now(ata_server *srv);
/* Stop the loop after in-flight work completes and free everything. */
int ata_server_destroy(ata_server *srv);

/*
 * Normal equations of least squares.  The paper's introduction names them
 * (with projections and least squares) as a use of A^t A; these calls take
 * the packed product to a solution:  x = (A^t A)^-1 A^t b.  All four work in
 * the storage of ata's output (row-major packed lower triangle), on device
 * memory, asynchronously on `stream`, in FP64 (dtype ATA_F64) or FP32
 * (ATA_F32) arithmetic and storage throughout.  Return codes as above:
 * -k for an invalid k-th argument (a null pointer where data is needed, or a
 * pointer not aligned to its element), ATA_EUNSUPPORTED for another device or
 * n > 2^22.
 *
 * ata_potrf: Cholesky factor of the symmetric positive definite matrix in
 *   C_lower (n x n, packed), in place: on return C_lower holds L, lower
 *   triangular with positive diagonal and L L^t = C.  Right-looking in
 *   64-column blocks: per block one launch for the diagonal block, one for
 *   the rows below it and one MFMA launch for the trailing update.
 *   info: device int32 or NULL.  The call sets it to 0, and a kernel sets it
 *   to p + 1 for the first column p whose pivot is not positive (LAPACK's
 *   convention); L is then unspecified from column p on.  Read it after the
 *   stream has synchronised.
 */
int ata_potrf(void *C_lower, int64_t n, int dtype, int32_t *info, void *stream);

/*
 * ata_potrs: solve L L^t X = B in place for the factor L from ata_potrf.
 *   B: row-major n x nrhs, row stride ldb >= nrhs, overwritten by X.  One
 *   launch per 64-row block for each of the forward and back substitutions;
 *   suited to a few right-hand sides (each is solved in turn inside a block).
 */
int ata_potrs(const void *L_lower, int64_t n, void *B, int64_t nrhs, int64_t ldb, int dtype, void *stream);

/*
 * ata_atb: out = A^t B, the right-hand side of the normal equations.
 *   A: row-major m x n (row stride lda >= n); B: row-major m x nrhs (row
 *   stride ldb >= nrhs); out: row-major n x nrhs (row stride ldo >= nrhs).
 *   Sums in FP64 over fixed row chunks, then the chunks in order, so results
 *   are reproducible.  Allocates its partial sums stream-ordered on `stream`.
 */
int ata_atb(const void *A, int64_t m, int64_t n, int64_t lda, const void *B, int64_t nrhs, int64_t ldb, void *out,
            int64_t ldo, int dtype, void *stream);

/*
 * ata_normal_solve: X = (A^t A)^-1 A^t B by ata (cutoff as for ata, 0 =
 *   default; default options), ata_potrf, ata_atb and ata_potrs.  X: row-major
 *   n x nrhs (row stride ldx >= nrhs).  The packed product and the partial
 *   sums are allocated stream-ordered on `stream`.  info as for ata_potrf.
 */
int ata_normal_solve(const void *A, int64_t m, int64_t n, int64_t lda, const void *B, int64_t nrhs, int64_t ldb,
                     void *X, int64_t ldx, int dtype, int cutoff, int32_t *info, void *stream);

/*
 * ata_project: out = P B for the projection P = A (A^t A)^-1 A^t onto the
 *   column space of A, which the introduction names beside the normal
 *   equations: ata_normal_solve into a stream-ordered n x nrhs workspace,
 *   then A X (one wave per row of A, FP64 sums).  B, out: row-major
 *   m x nrhs (row strides ldb, ldo >= nrhs).  info as for ata_potrf.
 *   n = 0 gives zeros.
 */
int ata_project(const void *A, int64_t m, int64_t n, int64_t lda, const void *B, int64_t nrhs, int64_t ldb,
                void *out, int64_t ldo, int dtype, int cutoff, int32_t *info, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ATA_H */
