// Internals of libata shared between the C ABI layer and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <vector>

#include "ata_plan.h"

namespace atalib {
namespace detail {

// Device copy of one plan's tables.
struct PhaseDev {
    int n_str = 0, n_tg = 0, n_gemm = 0, n_syrk = 0, n_cb = 0, n_ops = 0, n_mix = 0, str_tmax = 0, tg_tmax = 0;
    int n_big = 0;  // reduced-precision plans: 256 x 256 tiles of the phase's classical tasks
    int n_big_tail = 0, big_tail_parts = 0;  // ... and the K-split tiles of their last round
    int n_tail = 0, tail_parts = 0;          // FP64: K-split tiles of the last round of the mix launch
    int64_t cb_elems = 0, ops_rows = 0;
    size_t off_str = 0, off_tg = 0, off_gemm = 0, off_syrk = 0, off_cb = 0, off_ops = 0, off_mix = 0, off_big = 0,
           off_big_tail = 0, off_tail = 0;
};

struct PlanDev {
    Plan plan;
    int device = -1;
    char* blob = nullptr;          // device memory holding every table
    std::vector<char> host_blob;  // the same tables on the host
    size_t off_tasks = 0, off_terms = 0, off_segs = 0;
    std::vector<PhaseDev> phases;
    bool lp_aligned[2] = {false, false};  // reduced-precision modes: windows dword-aligned in the copy
    bool lp_aligned16 = false;            // windows on 16 elements of the copy (e4m3 256 x 256 tiles)
    bool lp_dma16[2] = {false, false};    // reduced-precision modes: windows on 16 bytes of the copy
    ~PlanDev() {
        if (blob) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(device);
            (void)hipFree(blob);
            (void)hipSetDevice(cur);
        }
    }
};

// Device workspace layout: [FP64 Strassen products][scales][column-max
// partials][converted copy plane 0][plane 1][operand-sum buffers]
// [equilibrated copy of A], each 256-byte aligned.  The scale and partial areas serve the FP8 scales or the
// equilibration scales (never both).
// Reduced-precision plans with Strassen levels add the converted operand copy
// of the products ([plane 0][plane 1] with row stride ldto), its per-row
// scales and the column-maximum scratch of the e4m3 scales.
struct WsLayout {
    size_t w = 0, scale = 0, part = 0, t0 = 0, t1 = 0, ops = 0, eqa = 0, total = 0;
    size_t t0o = 0, t1o = 0, scale_o = 0, colmax_o = 0;
    int64_t ldt = 0, ldto = 0, rows_o = 0;
    bool eq = false;
};

// Kernel timing for measurement tools (ata_profile_enable): while enabled,
// a ProfScope brackets the launches made in its lifetime with HIP events on
// the launch stream, recorded under its kernel kind (ATA_KERNEL_*).
struct ProfRec {
    int kind;
    hipEvent_t a, b;
};
extern std::mutex g_prof_mu;
extern bool g_prof_on;
extern std::vector<ProfRec> g_prof;

struct ProfScope {
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    bool on = false;
    ProfScope(int k, hipStream_t st) : kind(k), s(st) {
        {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            on = g_prof_on;
        }
        if (on && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, s);
        else
            on = false;
    }
    ~ProfScope() {
        if (!on) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof.push_back(ProfRec{kind, a, b});
    }
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;
};

int hip_fail(hipError_t e);
int check_device(int dev);       // caller holds the library mutex
int current_device_ok();         // the current device is gfx950 (locks)
void release_lookahead();        // helper streams of the Cholesky factor (waits for their devices)
bool dtype_lp(int dtype);
int elem_bytes_in(int dtype);
int elem_bytes_out(int dtype);
int64_t default_cutoff(int64_t m, int64_t n, int dtype);
WsLayout ws_layout(int64_t m, int64_t n, int dtype, int64_t ws_elems, bool equilibrate, int64_t opsum_elems,
                   int64_t lp_rows = 0, int64_t lp_k = 0);
// Internal plan flag (beside ATA_OPT_* bits): reduced-precision dtype.
constexpr int kPlanReducedPrecision = 0x10000;
// Internal plan flag: no K splitting (its partial sums need workspace).
constexpr int kPlanNoSplit = 0x20000;
// Internal plan flag: float input (the adaptive depth rule uses FP32 rates).
constexpr int kPlanF32 = 0x40000;
// Internal plan flag: accumulate into C (row slabs of one product).
constexpr int kPlanAccumulate = 0x80000;
// Internal plan flag: FP64 input (one-term tile launches split a short last
// round, see Plan::tile_tail_off).
constexpr int kPlanF64 = 0x100000;
// Internal plan flag: bfloat16-pair tiles (one resident workgroup per CU).
constexpr int kPlanBf16Pair = 0x200000;
// Equilibration in effect for a call with these option flags and this plan.
bool want_equilibrate(int flags, const Plan& P, int dtype);
int plan_flags(int flags, int dtype);
int get_plan(int64_t m, int64_t n, int64_t cutoff, int variant, int max_depth, int flags, bool need_device,
             std::shared_ptr<PlanDev>& out);
// dblob: device copy of pd.host_blob (pd.blob, or a copy the caller made)
// fork_ok: classical tiles may run on a pooled helper stream beside the
// Strassen tiles (false: everything on s).
hipError_t enqueue_product(const PlanDev& pd, const char* dblob, const WsLayout& L, const void* A, int64_t m,
                           int64_t n, int64_t lda, void* C_lower, int dtype, int variant, char* ws, hipStream_t s,
                           int dev, bool fork_ok = true);

}  // namespace detail
}  // namespace atalib
