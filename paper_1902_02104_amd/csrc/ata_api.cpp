// C ABI of the A^t A library: argument checks, plan cache, device task tables,
// workspace and launch order.  Declarations and argument conventions are in
// include/ata.h.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <algorithm>
#include <cstring>
#include <list>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <tuple>
#include <vector>

#include "../../include/ata.h"
#include "ata_plan.h"

#include "ata_internal.h"
#include "ata_kernels.h"

using namespace atalib;

namespace atalib {
namespace detail {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return e == hipErrorOutOfMemory ? ATA_ENOMEM : ATA_EHIP;
}

#define HIP_TRY(expr)                          \
    do {                                       \
        hipError_t _e = (expr);                \
        if (_e != hipSuccess) return hip_fail(_e); \
    } while (0)

using PlanKey = std::tuple<int, int64_t, int64_t, int64_t, int, int, int>;

std::mutex g_mu;
std::map<PlanKey, std::shared_ptr<PlanDev>> g_plans;
// Least recently used order of the cached plans (front = oldest) and the cap:
// a stream of shapes (serving draws m and n at random) would otherwise keep
// every plan it ever built.
std::list<PlanKey> g_plan_lru;
std::map<PlanKey, std::list<PlanKey>::iterator> g_plan_pos;
constexpr size_t kPlanCacheCap = 256;

void plan_touch(const PlanKey& key) {
    auto it = g_plan_pos.find(key);
    if (it != g_plan_pos.end()) g_plan_lru.erase(it->second);
    g_plan_lru.push_back(key);
    g_plan_pos[key] = std::prev(g_plan_lru.end());
}

// Drop the oldest plans beyond the cap (caller holds g_mu).  Callers that
// still use a plan hold their own reference.  A device copy of the tables
// may still be read by queued products, so the devices holding evicted copies
// are synchronised before the copies are freed (outside the lock, by the
// caller, through `freed`).
void plan_evict(std::vector<std::shared_ptr<PlanDev>>& freed) {
    while (g_plans.size() > kPlanCacheCap && !g_plan_lru.empty()) {
        const PlanKey k = g_plan_lru.front();
        g_plan_lru.pop_front();
        g_plan_pos.erase(k);
        auto it = g_plans.find(k);
        if (it == g_plans.end()) continue;
        freed.push_back(it->second);
        g_plans.erase(it);
    }
}

void plan_release(std::vector<std::shared_ptr<PlanDev>>& freed) {
    int cur = -1;
    for (auto& pd : freed) {
        if (pd->blob && pd.use_count() == 1) {
            if (cur < 0) (void)hipGetDevice(&cur);
            (void)hipSetDevice(pd->device);
            (void)hipDeviceSynchronize();
        }
        pd.reset();
    }
    if (cur >= 0) (void)hipSetDevice(cur);
}
std::map<int, int> g_device_ok;  // device -> 1 gfx950, 0 not

int check_device(int dev) {
    auto it = g_device_ok.find(dev);
    if (it != g_device_ok.end()) return it->second;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return 0;
    const int ok = std::strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
    g_device_ok[dev] = ok;
    return ok;
}

int current_device_ok() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    return check_device(dev);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// True when every segment window [row + kbeg, row + kend) of the plan's
// classical tasks starts and ends on a multiple of `q` elements: the
// transposed converted copy (rows padded to a multiple of 128 elements) can
// then be staged in whole dwords (q = 2 for bfloat16, 4 for e4m3).
// tail_ok: a window that ends at row m counts as aligned (the converted copy
// holds zeros from row m to its padded row length, a multiple of 128).
bool lp_windows_aligned(const Plan& P, int q, bool tail_ok = false) {
    std::set<int32_t> desc;  // tasks that only describe operand sums (never launched)
    for (const Phase& ph : P.phases)
        for (const DevOpSum& os : ph.opsums) desc.insert(os.task);
    for (size_t id = 0; id < P.tasks.size(); ++id) {
        const DevTask& t = P.tasks[id];
        if (t.kind != TK_SYRK && t.kind != TK_GEMM) continue;
        if (desc.count((int32_t)id)) continue;
        const int stride = kSegHdr + 2 * (t.nx + t.ny);
        for (int sg = 0; sg < t.nseg; ++sg) {
            const int32_t* g = P.segs.data() + t.seg_off + (int64_t)sg * stride;
            const int64_t row = g[kSegHdr];
            if ((row + g[1]) % q != 0 || ((row + g[2]) % q != 0 && !(tail_ok && row + g[2] == P.m))) return false;
        }
    }
    return true;
}

// Staging of the reduced-precision tiles the plan's windows allow: 2 for
// 16-byte direct-to-LDS copies, 1 for dword copies, 0 through registers.
int lp_align(const PlanDev& pd, int mode) { return pd.lp_dma16[mode] ? 2 : pd.lp_aligned[mode] ? 1 : 0; }

// Lay out a plan's tables in one host image (offsets recorded in pd).
void serialize(PlanDev& pd) {
    const Plan& P = pd.plan;
    size_t off = 0;
    pd.off_tasks = off;
    off = align256(off + P.tasks.size() * sizeof(DevTask));
    pd.off_terms = off;
    off = align256(off + P.terms.size() * sizeof(DevTerm));
    pd.off_segs = off;
    off = align256(off + P.segs.size() * sizeof(int32_t));
    pd.phases.resize(P.phases.size());
    for (size_t i = 0; i < P.phases.size(); ++i) {
        const Phase& ph = P.phases[i];
        PhaseDev& d = pd.phases[i];
        d.n_str = (int)ph.str_items.size();
        d.str_tmax = ph.str_tmax;
        d.n_tg = (int)ph.tg_items.size();
        d.tg_tmax = ph.tg_tmax;
        d.n_ops = (int)ph.opsums.size();
        d.ops_rows = ph.opsum_rows;
        d.n_gemm = (int)ph.gemm_items.size();
        d.n_syrk = (int)ph.syrk_items.size();
        d.n_cb = (int)ph.combines.size();
        d.cb_elems = ph.combine_elems;
        d.off_str = off;
        off = align256(off + ph.str_items.size() * sizeof(WorkItem));
        d.off_tg = off;
        off = align256(off + ph.tg_items.size() * sizeof(WorkItem));
        d.off_gemm = off;
        off = align256(off + ph.gemm_items.size() * sizeof(WorkItem));
        d.off_syrk = off;
        off = align256(off + ph.syrk_items.size() * sizeof(WorkItem));
        d.off_cb = off;
        off = align256(off + ph.combines.size() * sizeof(DevCombine));
        d.off_ops = off;
        off = align256(off + ph.opsums.size() * sizeof(DevOpSum));
        d.n_mix = (int)ph.mix_items.size();
        d.off_mix = off;
        off = align256(off + ph.mix_items.size() * sizeof(WorkItem));
        d.n_big = (int)ph.big_items.size();
        d.off_big = off;
        off = align256(off + ph.big_items.size() * sizeof(WorkItem));
        d.n_tail = (int)ph.tail_items.size();
        d.tail_parts = ph.tail_parts;
        d.off_tail = off;
        off = align256(off + ph.tail_items.size() * sizeof(WorkItem));
        d.n_big_tail = (int)ph.big_tail.size();
        d.big_tail_parts = ph.big_tail_parts;
        d.off_big_tail = off;
        off = align256(off + ph.big_tail.size() * sizeof(WorkItem));
    }
    std::vector<char>& host = pd.host_blob;
    host.assign(off ? off : 256, 0);
    std::memcpy(host.data() + pd.off_tasks, P.tasks.data(), P.tasks.size() * sizeof(DevTask));
    std::memcpy(host.data() + pd.off_terms, P.terms.data(), P.terms.size() * sizeof(DevTerm));
    std::memcpy(host.data() + pd.off_segs, P.segs.data(), P.segs.size() * sizeof(int32_t));
    for (size_t i = 0; i < P.phases.size(); ++i) {
        const Phase& ph = P.phases[i];
        const PhaseDev& d = pd.phases[i];
        std::memcpy(host.data() + d.off_str, ph.str_items.data(), ph.str_items.size() * sizeof(WorkItem));
        std::memcpy(host.data() + d.off_tg, ph.tg_items.data(), ph.tg_items.size() * sizeof(WorkItem));
        std::memcpy(host.data() + d.off_gemm, ph.gemm_items.data(), ph.gemm_items.size() * sizeof(WorkItem));
        std::memcpy(host.data() + d.off_syrk, ph.syrk_items.data(), ph.syrk_items.size() * sizeof(WorkItem));
        std::memcpy(host.data() + d.off_cb, ph.combines.data(), ph.combines.size() * sizeof(DevCombine));
        std::memcpy(host.data() + d.off_ops, ph.opsums.data(), ph.opsums.size() * sizeof(DevOpSum));
        std::memcpy(host.data() + d.off_mix, ph.mix_items.data(), ph.mix_items.size() * sizeof(WorkItem));
        std::memcpy(host.data() + d.off_big, ph.big_items.data(), ph.big_items.size() * sizeof(WorkItem));
        std::memcpy(host.data() + d.off_big_tail, ph.big_tail.data(), ph.big_tail.size() * sizeof(WorkItem));
        std::memcpy(host.data() + d.off_tail, ph.tail_items.data(), ph.tail_items.size() * sizeof(WorkItem));
    }
    for (int mode = 0; mode < 2; ++mode) pd.lp_aligned[mode] = lp_windows_aligned(P, mode == 0 ? 2 : 4);
    pd.lp_aligned16 = P.opt.lp && lp_windows_aligned(P, 16, true);
    for (int mode = 0; mode < 2; ++mode) pd.lp_dma16[mode] = P.opt.lp && lp_windows_aligned(P, mode == 0 ? 8 : 16, true);
}

// Copy a serialized plan into one device allocation.
int upload(PlanDev& pd, int dev) {
    HIP_TRY(hipMalloc(&pd.blob, pd.host_blob.size()));
    pd.device = dev;
    HIP_TRY(hipMemcpy(pd.blob, pd.host_blob.data(), pd.host_blob.size(), hipMemcpyHostToDevice));
    return ATA_OK;
}

int resolve_opts(const ata_opts* opts, int& variant, int& max_depth, int& flags) {
    variant = ATA_VARIANT_STRASSEN;
    max_depth = ATA_DEFAULT_MAX_DEPTH;
    flags = ATA_DEFAULT_FLAGS;
    if (opts) {
        variant = opts->variant;
        max_depth = opts->max_depth;
        flags = opts->flags;
        if (flags & ~(ATA_OPT_PRODUCT_TILES | ATA_OPT_EQUILIBRATE | ATA_OPT_OPERAND_SUMS | ATA_OPT_ADAPTIVE |
                      ATA_OPT_EQUILIBRATE_AUTO))
            return -1;
    }
    if (variant != ATA_VARIANT_STRASSEN && variant != ATA_VARIANT_WINOGRAD) return -1;
    if (max_depth < -1) return -1;
    return 0;
}

int elem_bytes_in(int dtype) { return (dtype & 0xff) == ATA_F64 ? 8 : 4; }

// Plan-shaping bits of the option flags plus the dtype class (the plan cache
// key): tables differ between the product-tile and in-tile forms and in the
// split-K target of the reduced-precision forms.
int plan_flags(int flags, int dtype) {
    int f = (flags & (ATA_OPT_PRODUCT_TILES | ATA_OPT_OPERAND_SUMS | ATA_OPT_ADAPTIVE)) |
            (dtype_lp(dtype) ? kPlanReducedPrecision : 0);
    if ((flags & ATA_OPT_ADAPTIVE) && (dtype & 0xff) != ATA_F64) f |= kPlanF32;
    if ((flags & ATA_OPT_ADAPTIVE) && !dtype_lp(dtype)) f |= flags & ATA_OPT_EQUILIBRATE_AUTO;
    if ((dtype & 0xff) == ATA_F64) f |= kPlanF64;
    if ((dtype & 0xff) == ATA_F32_BF16X3) f |= kPlanBf16Pair;
    return f;
}
bool want_equilibrate(int flags, const Plan& P, int dtype) {
    if (dtype_lp(dtype)) return false;
    if (flags & ATA_OPT_EQUILIBRATE) return true;
    return (flags & ATA_OPT_EQUILIBRATE_AUTO) && P.str_mults > 0;
}
// Reduced-precision forms: classical leaves by default; Strassen levels (one
// or two, one for Winograd) run as product tiles on operand sums converted
// after summing in FP32 (the operand-sum form).  They scale columns themselves,
// so explicit equilibration is refused.
int lp_options(const ata_opts* opts, int variant, int& max_depth, int& flags) {
    if (flags & ATA_OPT_EQUILIBRATE) return ATA_EUNSUPPORTED;
    flags &= ~(ATA_OPT_ADAPTIVE | ATA_OPT_EQUILIBRATE_AUTO);
    if (!opts || max_depth == 0) {
        max_depth = 0;
        return 0;
    }
    if (max_depth < 0 || max_depth > (variant == ATA_VARIANT_WINOGRAD ? 1 : kMaxExpandDepth)) return ATA_EUNSUPPORTED;
    flags |= ATA_OPT_PRODUCT_TILES | ATA_OPT_OPERAND_SUMS;
    return 0;
}

// Default form for a NULL options struct: FP64 runs its Strassen levels as
// product tiles (the faster fused form there).
int default_form_flags(const ata_opts* opts, int dtype) {
    return (!opts && (dtype & 0xff) == ATA_F64) ? ATA_OPT_PRODUCT_TILES : 0;
}
int elem_bytes_out(int dtype) {
    if ((dtype & 0xff) == ATA_F64) return 8;
    return (dtype & ATA_OUT_F64) ? 8 : 4;
}
bool dtype_valid(int dtype) {
    const int base = dtype & 0xff, flags = dtype & ~0xff;
    if (base < ATA_F64 || base > ATA_F32_FP8) return false;
    if (flags & ~ATA_OUT_F64) return false;
    if (base == ATA_F64 && flags) return false;
    return true;
}
bool dtype_lp(int dtype) { return (dtype & 0xff) == ATA_F32_BF16X3 || (dtype & 0xff) == ATA_F32_FP8; }

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

WsLayout ws_layout(int64_t m, int64_t n, int dtype, int64_t ws_elems, bool equilibrate, int64_t opsum_elems,
                   int64_t lp_rows, int64_t lp_k) {
    WsLayout L;
    size_t off = (size_t)ws_elems * sizeof(double);
    off = (off + 255) & ~(size_t)255;
    const bool lp = dtype_lp(dtype);
    if ((lp || equilibrate) && n > 0) {
        const size_t eb = lp ? sizeof(float) : (size_t)elem_bytes_in(dtype);
        L.scale = off;
        off += (size_t)n * eb;
        off = (off + 255) & ~(size_t)255;
        L.part = off;
        off += (size_t)((m + 255) / 256) * n * eb;
        off = (off + 255) & ~(size_t)255;
    }
    if (lp && n > 0) {
        const bool fp8 = (dtype & 0xff) == ATA_F32_FP8;
        L.ldt = round_up(m > 0 ? m : 1, 128);
        const size_t plane = (size_t)n * L.ldt * (fp8 ? 1 : 2);
        L.t0 = off;
        off += plane;
        off = (off + 255) & ~(size_t)255;
        if (!fp8) {
            L.t1 = off;
            off += plane;
            off = (off + 255) & ~(size_t)255;
        }
    }
    if (lp && lp_rows > 0) {
        const bool fp8 = (dtype & 0xff) == ATA_F32_FP8;
        L.rows_o = lp_rows;
        L.ldto = round_up(lp_k > 0 ? lp_k : 1, 128);
        const size_t plane = (size_t)lp_rows * L.ldto * (fp8 ? 1 : 2);
        L.t0o = off;
        off = (off + plane + 255) & ~(size_t)255;
        if (!fp8) {
            L.t1o = off;
            off = (off + plane + 255) & ~(size_t)255;
        }
        L.scale_o = off;
        off = (off + (size_t)lp_rows * sizeof(float) + 255) & ~(size_t)255;
        L.colmax_o = off;
        off = (off + (size_t)lp_rows * sizeof(uint32_t) + 255) & ~(size_t)255;
    }
    if (opsum_elems > 0 && !lp) {
        L.ops = off;
        off += (size_t)opsum_elems * elem_bytes_in(dtype);
        off = (off + 255) & ~(size_t)255;
    }
    if (equilibrate && !lp && n > 0 && m > 0) {
        L.eq = true;
        L.eqa = off;
        off += (size_t)m * n * elem_bytes_in(dtype);
        off = (off + 255) & ~(size_t)255;
    }
    L.total = off;
    return L;
}

int64_t default_cutoff(int64_t m, int64_t n, int dtype) {
    // Leaves of a few hundred columns keep every workgroup tile busy while the
    // top levels (where nearly all the work is) still split.  From timings on
    // gfx950 at one Strassen level: 512-column leaves are the fastest of
    // {128, 256, 512} for FP64 from 2048 columns up (square and tall) and for
    // every form above 4096 columns; float input on near-square shapes of up
    // to 4096 columns runs faster with 256.
    const int64_t mn = m < n ? m : n;
    if (mn <= 1024) return 128;
    if (mn <= 4096 && (dtype & 0xff) != ATA_F64 && m < 4 * n) return 256;
    return 512;
}

// Build (or fetch) the plan for the current device.
int get_plan(int64_t m, int64_t n, int64_t cutoff, int variant, int max_depth, int flags, bool need_device,
             std::shared_ptr<PlanDev>& out) {
    int dev = -1;
    if (need_device) {
        HIP_TRY(hipGetDevice(&dev));
    }
    const PlanKey key{dev, m, n, cutoff, variant, max_depth, flags};
    std::vector<std::shared_ptr<PlanDev>> freed;
    struct Release {
        std::vector<std::shared_ptr<PlanDev>>& f;
        ~Release() { plan_release(f); }
    } release{freed};  // runs after the lock below is dropped
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        out = it->second;
        plan_touch(key);
        return ATA_OK;
    }
    auto pd = std::make_shared<PlanDev>();
    PlanOptions po;
    po.cutoff = cutoff;
    po.variant = variant;
    po.max_depth = max_depth;
    po.opsums = (flags & ATA_OPT_OPERAND_SUMS) != 0;
    po.intile = (flags & (ATA_OPT_PRODUCT_TILES | ATA_OPT_OPERAND_SUMS)) == 0;
    // reduced-precision tiles run several times faster: splitting K for a
    // fuller last wave costs them more (partials and their sum) than it saves
    if (flags & kPlanReducedPrecision) po.split_target = 768;
    if (flags & kPlanNoSplit) po.split_target = 0;
    if (flags & kPlanAccumulate) po.accumulate = true;
    if (flags & kPlanReducedPrecision) po.lp = true;
    if (flags & kPlanF64) po.split_tail = 1;
    else if (!(flags & kPlanReducedPrecision)) po.split_tail = 2;
    else if (flags & kPlanBf16Pair) po.split_tail = 3;
    if (flags & ATA_OPT_ADAPTIVE) {
        // Fractions of the MFMA peak measured on MI355X for this library's
        // tiles (rocprof MFMA busy of whole launches at 10000^2): FP64
        // classical tiles 0.855, FP64 two-term product tiles 0.76, FP64
        // in-tile Strassen 0.48; FP32 classical tiles 0.66, FP32 Strassen
        // tiles about 0.48.  Combination: about 48 bytes of memory traffic per
        // output element at 5 TB/s, 0.023 of a 128 x 128 x 1 tile step.
        po.adaptive = true;
        const bool f32 = (flags & kPlanF32) != 0;
        po.rate_one = f32 ? 0.66 : 0.855;
        po.rate_two = f32 ? 0.48 : (po.intile ? 0.48 : 0.76);
        po.comb = 0.023;
        // equilibration that comes with Strassen levels: a column-maximum
        // pass and a scaled copy, three element transfers per element of A
        if (flags & ATA_OPT_EQUILIBRATE_AUTO) po.eq = f32 ? 0.0058 : 0.0115;
    }
    try {
        pd->plan = build_plan(m, n, po);
    } catch (const std::length_error&) {
        return ATA_EUNSUPPORTED;
    } catch (const std::bad_alloc&) {
        return ATA_ENOMEM;
    } catch (const std::exception&) {
        return ATA_EUNSUPPORTED;
    }
    serialize(*pd);
    if (need_device) {
        const int rc = upload(*pd, dev);
        if (rc != ATA_OK) return rc;
    }
    g_plans[key] = pd;
    plan_touch(key);
    plan_evict(freed);
    out = pd;
    return ATA_OK;
}

// ---- a second stream per call for the small classical tiles ----
// The classical off-diagonal and diagonal tiles of a phase write output
// regions disjoint from the Strassen tiles, so they run on a forked stream and
// fill the GPU while the Strassen launch drains.  Contexts are pooled per
// device; an event pair orders the fork and the join on the caller's stream.
struct ForkCtx {
    hipStream_t s2 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_fork_mu;
std::map<int, std::vector<ForkCtx>> g_fork_pool;

int fork_get(int dev, ForkCtx& c) {
    {
        std::lock_guard<std::mutex> lk(g_fork_mu);
        auto& v = g_fork_pool[dev];
        if (!v.empty()) {
            c = v.back();
            v.pop_back();
            return ATA_OK;
        }
    }
    hipError_t e = hipStreamCreateWithFlags(&c.s2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.join, hipEventDisableTiming);
    if (e != hipSuccess) {  // release what was made
        if (c.fork) (void)hipEventDestroy(c.fork);
        if (c.s2) (void)hipStreamDestroy(c.s2);
        c = ForkCtx{};
        return hip_fail(e);
    }
    return ATA_OK;
}

void fork_put(int dev, const ForkCtx& c) {
    std::lock_guard<std::mutex> lk(g_fork_mu);
    g_fork_pool[dev].push_back(c);
}

// Join the forked stream back into s, also after a failed launch: whatever
// was queued on the fork before the failure must finish before later work
// on s (a stream-ordered free of the workspace, say).  Keeps the first error.
void join_fork(ForkCtx& fc, hipStream_t s, hipError_t& err, int dev) {
    const hipError_t e1 = hipEventRecord(fc.join, fc.s2);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s, fc.join, 0) : e1;
    if (e2 != hipSuccess) (void)hipStreamSynchronize(fc.s2);  // the event could not order them
    if (err == hipSuccess) err = e2;
    fork_put(dev, fc);
}

// ---- kernel timing (measurement tools only; ProfScope in ata_internal.h) ----
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

int common_checks(const void* A, int64_t m, int64_t n, int64_t lda, const void* C, int dtype, int cutoff) {
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (!dtype_valid(dtype)) return -6;
    if (cutoff < 0) return -7;
    if (n > 0 && m > 0 && !A) return -1;
    if (n > 0 && !C) return -5;
    const uintptr_t ua = (uintptr_t)A, uc = (uintptr_t)C;
    if (ua % elem_bytes_in(dtype)) return -1;
    if (uc % elem_bytes_out(dtype)) return -5;
    if (m > INT32_MAX || n > INT32_MAX) return ATA_EUNSUPPORTED;
    if (lda > kMaxRowBytes / elem_bytes_in(dtype)) return ATA_EUNSUPPORTED;
    return 0;
}

// Enqueue every launch of one product on stream s (see ata_ex).  ws holds
// L.total bytes (may be null when L.total is 0).
hipError_t enqueue_product(const PlanDev& pdr, const char* dblob, const WsLayout& L, const void* A, int64_t m,
                           int64_t n, int64_t lda, void* C_lower, int dtype, int variant, char* ws, hipStream_t s,
                           int dev, bool fork_ok) {
    struct {
        const char* blob;
        size_t off_tasks, off_terms, off_segs;
        const std::vector<PhaseDev>& phases;
    } v{dblob, pdr.off_tasks, pdr.off_terms, pdr.off_segs, pdr.phases};
    const auto* pd = &v;
    const Plan& P = pdr.plan;
    const bool lp = dtype_lp(dtype);
    const bool f32 = (dtype & 0xff) != ATA_F64;
    const bool out64 = elem_bytes_out(dtype) == 8;
    int rc = ATA_OK;
    double* W = P.ws_elems ? (double*)(ws + L.w) : nullptr;
    const DevTables tb{(const DevTask*)(pd->blob + pd->off_tasks), (const DevTerm*)(pd->blob + pd->off_terms),
                       (const int32_t*)(pd->blob + pd->off_segs)};
    hipError_t err = hipSuccess;
    if (L.eq) {
        // every product below runs on the column-equilibrated copy of A
        ProfScope ps(ATA_KERNEL_OTHER, s);
        err = launch_equilibrate(f32, A, lda, (int)m, (int)n, ws + L.part, ws + L.scale, ws + L.eqa, s);
        A = ws + L.eqa;
        lda = n;
    }
    const int lp_mode = (dtype & 0xff) == ATA_F32_FP8 ? 1 : 0;
    if (lp) {
        ProfScope ps(ATA_KERNEL_OTHER, s);
        float* scale = (float*)(ws + L.scale);
        if (lp_mode == 1) err = launch_colscale((const float*)A, lda, (int)m, (int)n, (float*)(ws + L.part), scale, s);
        if (err == hipSuccess)
            err = launch_prep_lp(lp_mode, (const float*)A, lda, (int)m, (int)n, (int)L.ldt, scale, ws + L.t0,
                                 lp_mode == 0 ? (void*)(ws + L.t1) : nullptr, s);
    }
    for (const PhaseDev& ph : pd->phases) {
        if (err != hipSuccess) break;
        if (lp) {
            const float* scale = (const float*)(ws + L.scale);
            const void* t1 = lp_mode == 0 ? (const void*)(ws + L.t1) : nullptr;
            if (ph.n_ops) {
                // Strassen products: operand sums converted into the operand copy
                ProfScope ps(ATA_KERNEL_OTHER, s);
                err = launch_opsum_lp(lp_mode, (const float*)A, lda, tb, (const DevOpSum*)(pd->blob + ph.off_ops),
                                      ph.n_ops, ph.ops_rows, L.rows_o, (uint32_t*)(ws + L.colmax_o),
                                      (float*)(ws + L.scale_o), ws + L.t0o, lp_mode == 0 ? ws + L.t1o : nullptr,
                                      (int)L.ldto, s);
            }
            if (err == hipSuccess && ph.n_tg) {
                ProfScope ps(ATA_KERNEL_STRASSEN, s);
                err = launch_gemm_lp(lp_mode, out64, ws + L.t0o, lp_mode == 0 ? (const void*)(ws + L.t1o) : nullptr,
                                     (int)L.ldto, (const float*)(ws + L.scale_o), tb,
                                     (const WorkItem*)(pd->blob + ph.off_tg), ph.n_tg, C_lower, W, s,
                                     lp_align(pdr, lp_mode));
            }
            if (err == hipSuccess && lp_mode == 1 && out64 && pdr.lp_aligned16 && ph.n_big >= kBigMinTiles &&
                (int64_t)64 * L.ldt < ((int64_t)1 << 31)) {
                // e4m3 classical tiles of 256 x 256 in one launch
                ProfScope ps(ATA_KERNEL_GEMM, s);
                err = launch_lp8_big(ws + L.t0, (int)L.ldt, scale, tb, (const WorkItem*)(pd->blob + ph.off_big),
                                     ph.n_big, (double*)C_lower, W, s, 1, nullptr);
                if (err == hipSuccess && ph.n_big_tail) {
                    // the last, partial round of tiles with its K range split
                    // over every CU; FP32 partials summed in part order
                    float* part = (float*)(W + P.lp_tail_off);
                    err = launch_lp8_big(ws + L.t0, (int)L.ldt, scale, tb,
                                         (const WorkItem*)(pd->blob + ph.off_big_tail), ph.n_big_tail,
                                         (double*)C_lower, W, s, ph.big_tail_parts, part);
                    if (err == hipSuccess)
                        err = launch_lp8_tail_sum(scale, tb, (const WorkItem*)(pd->blob + ph.off_big_tail),
                                                  ph.n_big_tail / ph.big_tail_parts, ph.big_tail_parts, part,
                                                  (double*)C_lower, W, s);
                }
                if (err == hipSuccess && ph.n_cb) {  // sums of split K parts
                    ProfScope ps2(ATA_KERNEL_COMBINE, s);
                    err = launch_combine(out64, (const DevCombine*)(pd->blob + ph.off_cb), ph.n_cb, ph.cb_elems, W,
                                         C_lower, s);
                }
                continue;
            }
            // diagonal tiles overlap the off-diagonal ones on a forked stream
            const bool split = fork_ok && ph.n_gemm > 0 && ph.n_syrk > 0;
            ForkCtx fc;
            if (split) {
                rc = fork_get(dev, fc);
                if (rc != ATA_OK) return hipErrorOutOfMemory;
                err = hipEventRecord(fc.fork, s);
                if (err == hipSuccess) err = hipStreamWaitEvent(fc.s2, fc.fork, 0);
            }
            if (err == hipSuccess && ph.n_gemm) {
                ProfScope ps(ATA_KERNEL_GEMM, s);
                err = launch_gemm_lp(lp_mode, out64, ws + L.t0, t1, (int)L.ldt, scale, tb,
                                     (const WorkItem*)(pd->blob + ph.off_gemm), ph.n_gemm, C_lower, W, s,
                                     lp_align(pdr, lp_mode));
            }
            hipStream_t s_small = split ? fc.s2 : s;
            if (err == hipSuccess && ph.n_syrk) {
                ProfScope ps(ATA_KERNEL_SYRK, s_small);
                err = launch_gemm_lp(lp_mode, out64, ws + L.t0, t1, (int)L.ldt, scale, tb,
                                     (const WorkItem*)(pd->blob + ph.off_syrk), ph.n_syrk, C_lower, W, s_small,
                                     lp_align(pdr, lp_mode));
            }
            if (split) join_fork(fc, s, err, dev);
            if (err == hipSuccess && ph.n_tail) {
                // the last, partial round of tiles with its K range split
                // over every CU; FP64 partials summed in part order
                ProfScope ps(ph.n_gemm ? ATA_KERNEL_GEMM : ATA_KERNEL_SYRK, s);
                err = launch_gemm_lp_split(lp_mode, out64, ws + L.t0, t1, (int)L.ldt, scale, tb,
                                           (const WorkItem*)(pd->blob + ph.off_tail), ph.n_tail, ph.tail_parts,
                                           W + P.tile_tail_off, C_lower, W, s, lp_align(pdr, lp_mode));
            }
            if (err == hipSuccess && ph.n_cb) {  // sums of split K parts
                ProfScope ps(ATA_KERNEL_COMBINE, s);
                err = launch_combine(out64, (const DevCombine*)(pd->blob + ph.off_cb), ph.n_cb, ph.cb_elems, W,
                                     C_lower, s);
            }
            continue;
        }
        if (!f32 && ph.n_mix > 0 && ph.n_str == 0) {
            // FP64 product tiles and classical tiles in one launch, heaviest
            // first, then the combination of the products
            if (ph.n_ops) {
                ProfScope ps(ATA_KERNEL_OTHER, s);
                err = launch_opsum(f32, A, lda, tb, (const DevOpSum*)(pd->blob + ph.off_ops), ph.n_ops, ph.ops_rows,
                                   ws + L.ops, s);
            }
            if (err == hipSuccess) {
                // two-term launches run persistent workgroups on work queues
                ProfScope ps(ATA_KERNEL_TILES, s);
                if (ph.n_tail)  // with the K-split last round in the same grid
                    err = launch_tile_cat((const double*)A, lda, tb, (const WorkItem*)(pd->blob + ph.off_mix),
                                          ph.n_mix, (const WorkItem*)(pd->blob + ph.off_tail), ph.n_tail,
                                          ph.tail_parts, W + P.tile_tail_off, (double*)C_lower, W, s,
                                          (const double*)(ws + L.ops));
                else
                    err = launch_tile(ph.tg_tmax <= 1 ? 1 : 2, (const double*)A, lda, tb,
                                      (const WorkItem*)(pd->blob + ph.off_mix), ph.n_mix, (double*)C_lower, W, s,
                                      (const double*)(ws + L.ops),
                                      P.queue_off >= 0 ? (int*)(W + P.queue_off) : nullptr);
            }
            if (err == hipSuccess && ph.n_cb) {
                ProfScope ps(ATA_KERNEL_COMBINE, s);
                err = launch_combine(out64, (const DevCombine*)(pd->blob + ph.off_cb), ph.n_cb, ph.cb_elems, W,
                                     C_lower, s);
            }
            continue;
        }
        const bool split = fork_ok && (ph.n_str + ph.n_tg) > 0 && (ph.n_gemm + ph.n_syrk) > 0;
        ForkCtx fc;
        if (split) {
            rc = fork_get(dev, fc);
            if (rc != ATA_OK) return hipErrorOutOfMemory;
            err = hipEventRecord(fc.fork, s);
            if (err == hipSuccess) err = hipStreamWaitEvent(fc.s2, fc.fork, 0);
        }
        if (err == hipSuccess && ph.n_str) {
            ProfScope ps(ATA_KERNEL_STRASSEN, s);
            err = launch_str(f32, out64, variant, ph.str_tmax, A, lda, tb, (const WorkItem*)(pd->blob + ph.off_str),
                             ph.n_str, C_lower, W, s);
        }
        if (err == hipSuccess && ph.n_ops) {
            ProfScope ps(ATA_KERNEL_OTHER, s);
            err = launch_opsum(f32, A, lda, tb, (const DevOpSum*)(pd->blob + ph.off_ops), ph.n_ops, ph.ops_rows,
                               ws + L.ops, s);
        }
        if (err == hipSuccess && ph.n_tg) {
            ProfScope ps(ATA_KERNEL_STRASSEN, s);
            const WorkItem* it = (const WorkItem*)(pd->blob + ph.off_tg);
            if (!f32 && ph.tg_tmax <= 2)  // FP64: one-term (operand-sum buffers) or two-term tiles
                err = launch_tile(ph.tg_tmax <= 1 ? 1 : 2, (const double*)A, lda, tb, it, ph.n_tg, (double*)C_lower, W,
                                  s, (const double*)(ws + L.ops),
                                  P.queue_off >= 0 ? (int*)(W + P.queue_off) : nullptr);
            else if (ph.tg_tmax <= 1)  // products on operand-sum buffers
                err = launch_gemm(f32, out64, A, lda, tb, it, ph.n_tg, C_lower, W, s, ws + L.ops);
            else
                err = launch_gemm_terms(f32, out64, ph.tg_tmax, A, lda, tb, it, ph.n_tg, C_lower, W, s);
        }
        hipStream_t s_small = split ? fc.s2 : s;
        // FP32 phases launching one classical list: its K-split last round
        const bool tail32 = f32 && ph.n_tail > 0;
        if (err == hipSuccess && ph.n_gemm) {
            ProfScope ps(ATA_KERNEL_GEMM, s_small);
            const WorkItem* it = (const WorkItem*)(pd->blob + ph.off_gemm);
            err = f32 ? launch_gemm(f32, out64, A, lda, tb, it, ph.n_gemm, C_lower, W, s_small)
                      : launch_tile(1, (const double*)A, lda, tb, it, ph.n_gemm, (double*)C_lower, W, s_small);
            if (err == hipSuccess && tail32 && ph.n_syrk == 0)
                err = launch_gemm_split(f32, out64, A, lda, tb, (const WorkItem*)(pd->blob + ph.off_tail), ph.n_tail,
                                        ph.tail_parts, W + P.tile_tail_off, C_lower, W, s_small);
        }
        if (err == hipSuccess && ph.n_syrk) {
            ProfScope ps(ATA_KERNEL_SYRK, s_small);
            const WorkItem* it = (const WorkItem*)(pd->blob + ph.off_syrk);
            err = f32 ? launch_gemm(f32, out64, A, lda, tb, it, ph.n_syrk, C_lower, W, s_small)
                      : launch_tile(1, (const double*)A, lda, tb, it, ph.n_syrk, (double*)C_lower, W, s_small);
            if (err == hipSuccess && tail32 && ph.n_gemm == 0)
                err = launch_gemm_split(f32, out64, A, lda, tb, (const WorkItem*)(pd->blob + ph.off_tail), ph.n_tail,
                                        ph.tail_parts, W + P.tile_tail_off, C_lower, W, s_small);
        }
        if (split) join_fork(fc, s, err, dev);
        if (err == hipSuccess && ph.n_cb) {
            ProfScope ps(ATA_KERNEL_COMBINE, s);
            err = launch_combine(out64, (const DevCombine*)(pd->blob + ph.off_cb), ph.n_cb, ph.cb_elems, W, C_lower, s);
        }
    }
    if (err == hipSuccess && L.eq) {
        ProfScope ps(ATA_KERNEL_OTHER, s);
        err = launch_descale(f32, out64, C_lower, (int)n, ws + L.scale, s);
    }
    return err;
}

}  // namespace detail
}  // namespace atalib

using namespace atalib::detail;

extern "C" {

const char* ata_version(void) { return "0.1.0"; }

int ata_last_hip_error(void) { return g_last_hip; }

const char* ata_status_string(int status) {
    if (status < 0) return "invalid argument";
    switch (status) {
    case ATA_OK: return "ok";
    case ATA_ENOMEM: return "out of memory";
    case ATA_EHIP: return "HIP runtime error";
    case ATA_EUNSUPPORTED: return "unsupported device, type or option";
    case ATA_EWORKSPACE: return "workspace too small";
    case ATA_EREJECT: return "request exceeds the memory budget";
    case ATA_EBUSY: return "queue full";
    case ATA_ENOTFOUND: return "unknown ticket";
    case ATA_EPENDING: return "request pending";
    default: return "unknown status";
    }
}

int ata_default_cutoff(int64_t m, int64_t n, int dtype) { return (int)default_cutoff(m, n, dtype); }

int ata_plan_info(int64_t m, int64_t n, int dtype, int cutoff, const ata_opts* opts, ata_plan_stats* out) {
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (!dtype_valid(dtype)) return -3;
    if (cutoff < 0) return -4;
    int variant, max_depth, flags;
    if (resolve_opts(opts, variant, max_depth, flags)) return -5;
    flags |= default_form_flags(opts, dtype);
    if (!out) return -6;
    if (dtype_lp(dtype)) {
        if (const int e = lp_options(opts, variant, max_depth, flags)) return e;
    }
    const int64_t c = cutoff ? cutoff : default_cutoff(m, n, dtype);
    std::shared_ptr<PlanDev> pd;
    const int rc = get_plan(m, n, c, variant, max_depth, plan_flags(flags, dtype), false, pd);
    if (rc != ATA_OK) return rc;
    const Plan& P = pd->plan;
    std::memset(out, 0, sizeof(*out));
    out->mults = P.mults;
    out->classical_mults = m * (n * (n + 1) / 2);
    out->syrk_tasks = P.syrk_tasks;
    out->gemm_tasks = P.gemm_tasks;
    out->strassen_tasks = P.str_tasks;
    out->combine_tasks = P.combine_tasks;
    out->work_items = P.work_items;
    out->phases = (int64_t)P.phases.size();
    out->ata_depth = P.ata_depth;
    out->max_hasa_depth = P.max_hasa_depth;
    out->workspace_bytes = (int64_t)ws_layout(m, n, dtype, P.ws_elems, want_equilibrate(flags, P, dtype), P.opsum_elems, P.lp_ops_rows, P.lp_ops_k).total;
    out->cutoff = c;
    out->strassen_mults = P.str_mults;
    out->gemm_mults = P.gemm_mults;
    out->syrk_mults = P.syrk_mults;
    out->combine_elems = P.combine_elems;
    out->lp_staging = dtype_lp(dtype) ? lp_align(*pd, (dtype & 0xff) == ATA_F32_FP8 ? 1 : 0) : -1;
    return ATA_OK;
}

int ata_workspace_bytes(int64_t m, int64_t n, int dtype, int cutoff, const ata_opts* opts, size_t* bytes) {
    ata_plan_stats st;
    const int rc = ata_plan_info(m, n, dtype, cutoff, opts, &st);
    if (rc != ATA_OK) return rc;
    if (!bytes) return -6;
    *bytes = (size_t)st.workspace_bytes;
    return ATA_OK;
}

int ata_ex(const void* A, int64_t m, int64_t n, int64_t lda, void* C_lower, int dtype, int cutoff,
           void* stream, const ata_opts* opts, void* workspace, size_t ws_bytes) {
    int rc = common_checks(A, m, n, lda, C_lower, dtype, cutoff);
    if (rc) return rc;
    int variant, max_depth, flags;
    if (resolve_opts(opts, variant, max_depth, flags)) return -9;
    flags |= default_form_flags(opts, dtype);
    const bool lp = dtype_lp(dtype);
    if (lp) {
        if (const int e = lp_options(opts, variant, max_depth, flags)) return e;
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!check_device(dev)) return ATA_EUNSUPPORTED;
    }
    if (n == 0) return ATA_OK;
    const int64_t nout = n * (n + 1) / 2;
    if (m == 0) {
        ProfScope ps(ATA_KERNEL_OTHER, s);
        HIP_TRY(launch_fill_zero(C_lower, nout, elem_bytes_out(dtype), s));
        return ATA_OK;
    }
    const int64_t c = cutoff ? cutoff : default_cutoff(m, n, dtype);
    std::shared_ptr<PlanDev> pd;
    rc = get_plan(m, n, c, variant, max_depth, plan_flags(flags, dtype), true, pd);
    if (rc != ATA_OK) return rc;
    const Plan& P = pd->plan;
    const WsLayout L = ws_layout(m, n, dtype, P.ws_elems, want_equilibrate(flags, P, dtype), P.opsum_elems, P.lp_ops_rows, P.lp_ops_k);
    if (L.ldt > INT32_MAX) return ATA_EUNSUPPORTED;
    char* ws = nullptr;
    bool owned = false;
    if (L.total) {
        if (workspace) {
            if (ws_bytes < L.total) return ATA_EWORKSPACE;
            if ((uintptr_t)workspace % 256) return -10;
            ws = (char*)workspace;
        } else {
            HIP_TRY(hipMallocAsync((void**)&ws, L.total, s));
            owned = true;
        }
    }
    hipError_t err = enqueue_product(*pd, pd->blob, L, A, m, n, lda, C_lower, dtype, variant, ws, s, dev);
    if (owned) {
        hipError_t e2 = hipFreeAsync(ws, s);
        if (err == hipSuccess) err = e2;
    }
    if (err != hipSuccess) return hip_fail(err);
    return ATA_OK;
}

int ata_precision_convert(int dtype, const float* x, int64_t count, void* out0, void* out1, void* stream) {
    const int base = dtype & 0xff;
    if (base != ATA_F32_BF16X3 && base != ATA_F32_FP8) return -1;
    if (count < 0) return -3;
    if (count > 0 && !x) return -2;
    if (count > 0 && !out0) return -4;
    if (count > 0 && base == ATA_F32_BF16X3 && !out1) return -5;
    if (count == 0) return ATA_OK;
    hipError_t e = launch_convert(base == ATA_F32_FP8 ? 1 : 0, x, count, out0, out1, (hipStream_t)stream);
    return e == hipSuccess ? ATA_OK : hip_fail(e);
}

}  // extern "C"

// ---- the entry point that allocates nothing (ata_ex_noalloc) ----
// One fixed device array per GPU holds the plan tables and the workspace of
// ata_ex_noalloc.  In host code `scratch` names a host-side stand-in, not
// device memory: the device address comes from hipGetSymbolAddress, once per
// device with that device current, and only that address is used.
static __device__ __align__(256) char scratch[ATA_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch;  // device -> address of its scratch array

int scratch_address(int dev, char** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
        it = g_scratch.emplace(dev, (char*)p).first;
    }
    *out = it->second;
    return ATA_OK;
}
}  // namespace

extern "C" {

int ata_ex_noalloc(const void* A, int64_t m, int64_t n, int64_t lda, void* C_lower, int dtype, int cutoff,
                   void* stream, const ata_opts* opts, size_t* scratch_used) {
    int rc = common_checks(A, m, n, lda, C_lower, dtype, cutoff);
    if (rc) return rc;
    int variant, max_depth, flags;
    if (resolve_opts(opts, variant, max_depth, flags)) return -9;
    flags |= default_form_flags(opts, dtype);
    if (dtype_lp(dtype)) {
        if (const int e = lp_options(opts, variant, max_depth, flags)) return e;
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!check_device(dev)) return ATA_EUNSUPPORTED;
    }
    char* base = nullptr;
    rc = scratch_address(dev, &base);
    if (rc != ATA_OK) return rc;
    if (scratch_used) *scratch_used = 0;
    if (n == 0) return ATA_OK;
    const int64_t nout = n * (n + 1) / 2;
    if (m == 0) {
        HIP_TRY(launch_fill_zero(C_lower, nout, elem_bytes_out(dtype), s));
        return ATA_OK;
    }
    const int64_t c = cutoff ? cutoff : default_cutoff(m, n, dtype);
    std::shared_ptr<PlanDev> pd;
    // host tables only (no device copy of the plan); no K splitting, whose
    // partial sums would need workspace
    rc = get_plan(m, n, c, variant, max_depth, plan_flags(flags, dtype) | kPlanNoSplit, false, pd);
    if (rc != ATA_OK) return rc;
    const Plan& P = pd->plan;
    const WsLayout L = ws_layout(m, n, dtype, P.ws_elems, want_equilibrate(flags, P, dtype), P.opsum_elems, P.lp_ops_rows, P.lp_ops_k);
    if (L.ldt > INT32_MAX) return ATA_EUNSUPPORTED;
    const size_t tbytes = (pd->host_blob.size() + 255) / 256 * 256;
    const size_t need = tbytes + L.total;
    if (scratch_used) *scratch_used = need;
    if (need > (size_t)ATA_NOALLOC_SCRATCH_BYTES) return ATA_EWORKSPACE;
    // the plan's tables go to the start of the array, the workspace after them
    HIP_TRY(hipMemcpyAsync(base, pd->host_blob.data(), pd->host_blob.size(), hipMemcpyHostToDevice, s));
    const hipError_t err =
        enqueue_product(*pd, base, L, A, m, n, lda, C_lower, dtype, variant, L.total ? base + tbytes : nullptr, s,
                        dev, false);
    if (err != hipSuccess) return hip_fail(err);
    return ATA_OK;
}

int ata(const void* A, int64_t m, int64_t n, int64_t lda, void* C_lower, int dtype, int cutoff, void* stream) {
    return ata_ex(A, m, n, lda, C_lower, dtype, cutoff, stream, nullptr, nullptr, 0);
}

int ata_aat(const void* A, int64_t m, int64_t n, int64_t lda, void* C_lower, int dtype, int cutoff, void* stream) {
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (!dtype_valid(dtype)) return -6;
    if (cutoff < 0) return -7;
    if (m > 0 && n > 0 && !A) return -1;
    if (m > 0 && !C_lower) return -5;
    const int eb = elem_bytes_in(dtype);
    if ((uintptr_t)A % eb) return -1;
    if ((uintptr_t)C_lower % elem_bytes_out(dtype)) return -5;
    if ((m + 63) / 64 > 65535 || n > INT32_MAX) return ATA_EUNSUPPORTED;
    if (!current_device_ok()) return ATA_EUNSUPPORTED;
    if (m == 0) return ATA_OK;
    hipStream_t s = (hipStream_t)stream;
    void* At = nullptr;
    if (n > 0) {
        HIP_TRY(hipMallocAsync(&At, (size_t)n * (size_t)m * eb, s));
        const hipError_t e = launch_transpose(eb, A, m, n, lda, At, s);
        if (e != hipSuccess) {
            (void)hipFreeAsync(At, s);
            return hip_fail(e);
        }
    }
    // A A^t is the product of the n x m matrix A^t with itself: C = (A^t)^t A^t
    int rc = ata_ex(At, n, m, m, C_lower, dtype, cutoff, stream, nullptr, nullptr, 0);
    if (At) {
        const hipError_t e2 = hipFreeAsync(At, s);
        if (rc == ATA_OK && e2 != hipSuccess) rc = hip_fail(e2);
    }
    return rc;
}

int ata_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return ATA_OK;
}

int ata_profile_collect(double* ms, int64_t* launches, int kinds) {
    if (kinds < 0) return -3;
    if (kinds > 0 && (!ms || !launches)) return -1;
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        recs.swap(g_prof);
    }
    for (int k = 0; k < kinds; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    int rc = ATA_OK;
    for (ProfRec& r : recs) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess && rc == ATA_OK) rc = hip_fail(e);
        if (r.kind < kinds) {
            ms[r.kind] += t;
            launches[r.kind] += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    return rc == ATA_OK ? (kinds < ATA_KERNEL_KINDS ? kinds : ATA_KERNEL_KINDS) : rc;
}

void ata_release_caches(void) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    std::lock_guard<std::mutex> lk(g_mu);
    std::set<int> devs;
    for (const auto& kv : g_plans)
        if (kv.second->device >= 0) devs.insert(kv.second->device);
    {
        std::lock_guard<std::mutex> fk(g_fork_mu);
        for (auto& kv : g_fork_pool) {
            devs.insert(kv.first);
            (void)hipSetDevice(kv.first);
            (void)hipDeviceSynchronize();
            for (ForkCtx& c : kv.second) {
                (void)hipEventDestroy(c.fork);
                (void)hipEventDestroy(c.join);
                (void)hipStreamDestroy(c.s2);
            }
        }
        g_fork_pool.clear();
    }
    for (int d : devs) {
        (void)hipSetDevice(d);
        (void)hipDeviceSynchronize();
    }
    (void)hipSetDevice(cur);
    g_plans.clear();
    g_plan_lru.clear();
    g_plan_pos.clear();
    release_lookahead();
}

}  // extern "C"
