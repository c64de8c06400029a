// Host planner of the ATA recursion (Section 3, Algorithm 1) and the device
// task table it produces.  Shared by the host library code and the kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace atalib {

// Kinds of device tasks.
enum TaskKind : int32_t {
    TK_SYRK = 0,  // diagonal base-case block: lower triangle of X^t X
    TK_GEMM = 1,  // classical off-diagonal product X^t Y
    TK_STR = 2,   // one Strassen level done inside each workgroup tile
};

// One signed operand term: columns [col, cvend) of A are valid, the rest of
// the padded range reads as zero.  Rows are per K segment (see DevTask).
constexpr int kSegHdr = 3;

struct DevTerm {
    int32_t col;
    int32_t cvend;
    int32_t sign;
    int32_t pad;
};

// A product D (M x N, padded) = Xop^t Yop, where Xop = sum of signed X terms
// and Yop = sum of signed Y terms, both K x (M or N) slices of A.  K is a
// list of segments (row chunks of the recursion); segment s has padded length
// klen, a window [kbeg, kend) of the k it covers (of [0, klen), or of the half
// range [0, ceil(klen/2)) for TK_STR), and per term a first row and a
// valid-row end:
//   seg[seg_off + s*(kSegHdr + 2*(nx+ny))] = klen, kbeg, kend, then
//   (row, rvend) for every X term, then for every Y term.
// Windows let one product's K range be split over several workgroups.
// For TK_STR the product is split once more inside the tile: M, N and each
// klen into ceil halves, seven products, one workgroup per quadrant tile.
struct DevTask {
    int32_t kind;
    int32_t variant;   // Strassen or Winograd for TK_STR
    int32_t M, N;      // padded product dims (TK_SYRK: M == N == width)
    int32_t nx, ny;    // number of X and Y terms
    int32_t term_off;  // first X term in the term table; Y terms follow
    int32_t nseg;
    int32_t seg_off;
    int32_t dst;       // 0: packed C at (r0, q0); 1: workspace at ws_off, ld N
    int32_t beta;      // 1: accumulate into packed C, 0: overwrite
    int32_t dM, dN;    // valid destination extent (crop)
    int32_t r0, q0;    // packed-C origin: rows of D -> C rows r0.., cols q0..
    int32_t tiles_m, tiles_n;
    int32_t src;       // 0: operands are columns of A; 1: of an operand-sum buffer
    int64_t ws_off;    // element offset into the workspace
    int64_t src_off;   // src 1: element offset of the task's buffer (K rows of
                       // M + N: X columns, then Y columns)
};

// Operand sums of one product (operand-sum form): rows [0, K) of a buffer of
// row length M + N at out_off hold the product's signed sums of X terms
// (first M columns) and of Y terms (last N), zero where every term is
// padding.  `task` describes the terms and their per-chunk rows (a TK_GEMM
// task with nx, ny terms that is never launched); row_off is the record's
// first row in its launch.
struct DevOpSum {
    int32_t task;
    int32_t K, M, N;
    int64_t out_off;
    int64_t row_off;
};
// In reduced-precision plans a record describes the same sums, converted into
// the operand copy: out_off is the record's first row of the copy (its M + N
// columns become rows out_off .. out_off + M + N, k contiguous) and row_off is
// its first 64 x 64 (k x column) conversion tile in the launch.

// Combination of workspace products into an off-diagonal block of C.
// Each output element sums, over nparts K parts (slot sets part_stride
// elements apart) and over the 7^levels products, the signed workspace values.
struct DevCombine {
    int32_t M, N;       // true block extent
    int32_t levels;     // Strassen levels that were expanded into workspace slots
    int32_t variant;
    int32_t r0, q0;
    int32_t beta;
    int32_t Mp, Np;     // padded dims of one workspace slot
    int32_t nparts;     // K parts summed (1 when the K range was not split)
    int32_t lower;      // 1: write only j <= i (a diagonal block)
    int32_t pad;
    int64_t part_stride;
    int64_t ws_off;
    int64_t elem_off;   // first output element index of this block in the launch
};

// Work item of a launch: tile (ti, tj) of task `task`.  In a batched launch
// `slot` selects the request (see BatchEntry); otherwise it is 0.
struct WorkItem {
    int32_t task, ti, tj, slot;
};

// One request of a batched launch of classical tiles: its matrices and the
// device task tables of its plan.
struct BatchEntry {
    const void* A;
    void* C;
    const DevTask* tasks;
    const DevTerm* terms;
    const int32_t* segs;
    int64_t lda;
};

struct PlanOptions {
    int64_t cutoff = 32;
    int variant = 0;    // 0 Strassen, 1 Winograd
    int max_depth = 1;  // < 0: unlimited (every caller sets it)
    // K splitting: a launch with fewer workgroup tiles than split_target
    // splits long K ranges (at least split_min_k each part) over several
    // workgroups whose partial results a combination sums in part order.
    // (12 workgroups per CU: the last wave of a launch is a small fraction)
    int split_target = 6144;
    int split_min_k = 1024;
    // Where the last Strassen level of an off-diagonal product runs.  true:
    // inside each workgroup tile (TK_STR).  false: every level is expanded
    // into signed operand terms and each of the 7^d products is a classical
    // tile task (TK_GEMM with terms) writing a workspace slot, summed by a
    // combination.  Products deeper than kMaxExpandDepth levels (one for
    // Winograd) always use the in-tile form.
    bool intile = true;
    // With product tiles: form each product's operand sums in a memory pass
    // (DevOpSum) and run the products as classical tiles on those buffers.
    bool opsums = false;
    // Adaptive depth: a further Strassen level is taken only where it is
    // faster by a cost model of the tile kernels: rate_one and rate_two are
    // the measured fractions of the MFMA peak of classical tiles and of the
    // tiles of a Strassen level (product tiles or in-tile), comb the cost of
    // combining one output element in 128 x 128 x 1 tile-step units.
    // eq: cost of equilibrating one element of A, charged to a Strassen level
    // for the columns of its operands when equilibration comes with Strassen
    // levels (0 otherwise).
    bool adaptive = false;
    double rate_one = 1.0, rate_two = 1.0, comb = 0.0, eq = 0.0;
    // Accumulate: every write into C adds to what C holds (C += A^t A), for
    // sums of products over row slabs of A.
    bool accumulate = false;
    // One-term tile launches whose last round holds at most half the
    // resident workgroups run that round K-split over every CU (K splitting
    // of whole launches then stops at two rounds of tiles): 1 for the
    // FP64 tile launch of mix_items, 2 for an FP32 phase launching only
    // gemm_items or only syrk_items, 3 for the same bfloat16-pair phase (one
    // resident workgroup per CU) (0: never).
    int split_tail = 0;
    // Reduced-precision leaves: the operand sums of the Strassen products
    // (operand-sum form) are converted into rows of a separate copy instead
    // of FP32 buffers (see DevOpSum).
    bool lp = false;
};

constexpr int kMaxExpandDepth = 2;

// Launch group: everything that may run after the previous group finished.
struct Phase {
    // str: in-tile Strassen tiles; tg: Strassen product tiles (classical
    // tiles with operand terms); gemm, syrk: classical tiles of the base case
    std::vector<WorkItem> str_items, tg_items, gemm_items, syrk_items;
    // The product tiles and the classical tiles of the phase in one list, in
    // the same order rules: for kernels that run both kinds in one launch.
    std::vector<WorkItem> mix_items;
    std::vector<DevCombine> combines;
    std::vector<DevOpSum> opsums;  // run before the product tiles
    // Reduced-precision plans: the classical tasks on 256 x 256 e4m3 tiles,
    // and the tiles of a short last round split into big_tail_parts K parts
    // (slot = tile * parts + part).
    std::vector<WorkItem> big_items, big_tail;
    int big_tail_parts = 0;
    // One-term tile launches: the tiles of a short last round (taken off the
    // end of mix_items, or of the phase's one classical list for FP32) split
    // into tail_parts K parts (slot = tile * parts + part).
    std::vector<WorkItem> tail_items;
    int tail_parts = 0;
    int64_t combine_elems = 0;
    int64_t opsum_rows = 0;
    int str_tmax = 0;  // most operand terms of any TK_STR task in this phase
    int tg_tmax = 0;   // most operand terms of any product tile task
};

struct Plan {
    int64_t m = 0, n = 0;
    PlanOptions opt;
    std::vector<DevTask> tasks;
    std::vector<DevTerm> terms;
    std::vector<int32_t> segs;
    std::vector<Phase> phases;
    int64_t ws_elems = 0;
    // Work queues of the persistent two-term tile launches (kTileQueues int32
    // at this FP64 element offset of the workspace, shared by the phases in
    // turn); -1 when no phase launches two-term tiles with classical ones.
    int64_t queue_off = -1;
    // FP32 partial tiles of the split last round of e4m3 tiles (element offset
    // in the FP64 workspace; -1 when no phase splits one)
    int64_t lp_tail_off = -1;
    // FP64 partial tiles of the K-split last round of one-term tile launches
    // (element offset in the workspace; -1 when no phase splits one)
    int64_t tile_tail_off = -1;
    int64_t opsum_elems = 0;  // operand-sum buffers, in elements of A's type
    int64_t lp_ops_rows = 0;  // reduced precision: rows of the operand copy
    int64_t lp_ops_k = 0;     // ... and its longest K
    // statistics
    int64_t mults = 0;
    int64_t str_mults = 0, gemm_mults = 0, syrk_mults = 0, combine_elems = 0;
    int64_t syrk_tasks = 0, gemm_tasks = 0, str_tasks = 0, combine_tasks = 0;
    int64_t work_items = 0;
    int64_t ata_depth = 0, max_hasa_depth = 0;
    // Host-only locality record of each task (used to order work items):
    // the Strassen expansion its operands come from (-1: none) and its K part
    // after splitting.  Shorter than tasks when trailing tasks have neither.
    std::vector<int32_t> task_group, task_part;
    int32_t n_groups = 0;
};

// Tile sizes the kernels use (output tile per workgroup).
constexpr int kGemmTile = 128;  // TK_GEMM / TK_SYRK
constexpr int kTileQueues = 8;  // work queues of a persistent FP64 tile launch (one per XCD)
constexpr int kTileSlots = 512;  // resident FP64 tile workgroups (two per CU on 256 CUs)
// e4m3 classical tiles of 256 x 256 (k_lp8_big), for launches of at least
// kBigMinTiles of them (one per CU).
constexpr int kBigTile = 256;
constexpr int kBigMinTiles = 256;
constexpr int kStrTile = 64;    // TK_STR quadrant tile (4 quadrants per workgroup)
// Largest row stride in bytes: kernels address a staged slab of rows with
// 32-bit offsets.
constexpr int64_t kMaxRowBytes = (int64_t)1 << 26;
constexpr int kMaxTerms = 8;    // max terms per operand (2^(levels staged))

// Build the plan.  Throws std::invalid_argument for impossible inputs.
Plan build_plan(int64_t m, int64_t n, const PlanOptions& opt);

// Result-quadrant coefficients of the seven products, [variant][product][a*2+c]
// (Strassen 1969 and Winograd 1971; see ata_plan.cpp).  Shared by the planner
// and the combination kernel.
#define ATA_D_COEF                                                                                    \
    {                                                                                                 \
        {{1, 0, 0, 1}, {0, 0, 1, -1}, {0, 1, 0, 1}, {1, 0, 1, 0}, {-1, 1, 0, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}}, \
        {{1, 1, 1, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, -1, 0}, {0, 1, 0, 1}, {0, 1, 1, 1}, {0, 0, 1, 1}}  \
    }

// Strassen / Winograd quadrant coefficients.  For product p (0..6):
//   x_coef[v][p][a*2+b] : coefficient of L_ab (M-half a, K-half b) in the left operand
//   y_coef[v][p][b*2+c] : coefficient of R_bc (K-half b, N-half c) in the right operand
//   d_coef[v][p][a*2+c] : coefficient of the product in result quadrant D_ac
extern const int x_coef[2][7][4];
extern const int y_coef[2][7][4];
extern const int d_coef[2][7][4];

}  // namespace atalib
