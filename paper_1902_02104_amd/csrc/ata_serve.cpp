// Serving loop: continuous batching of Gram-matrix requests on one GPU.
//
// A scheduler thread admits queued requests by memory footprint into a
// device pool, fills their A on the device, and launches them: requests whose
// plan is a single classical diagonal block go into one grouped launch per
// pass, the others run the library's normal launch sequence on one of several
// streams, so requests that arrive while others run overlap on the device.
// Completion is observed through events.  Declarations and the contract are
// in include/ata.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/ata.h"
#include "ata_internal.h"
#include "ata_kernels.h"

using namespace atalib;
using namespace atalib::detail;

namespace {

constexpr size_t kAlign = 256;
constexpr int kBypass = 8;  // queued requests that may be admitted ahead of a blocked head
// Row slabs: requests above kChunkFlops (m n^2) run in slabs of about
// kSlabFlops each, at least kMinSlabRows rows (multiples of 256).
constexpr double kChunkFlops = 4e10;
constexpr double kSlabFlops = 2e10;
constexpr int64_t kMinSlabRows = 4096;

int64_t slab_rows_for(int64_t m, int64_t n) {
    const double f = (double)m * (double)n * (double)n;
    if (f <= kChunkFlops) return 0;
    int64_t rows = (int64_t)(kSlabFlops / ((double)n * (double)n));
    rows = std::max(rows, kMinSlabRows);
    rows = (rows + 255) / 256 * 256;
    return 2 * rows <= m ? rows : 0;
}

// Simulate mode: a device-drawn request with this seed ends with ATA_EHIP
// (exercises the failure path of the scheduler without a device).
constexpr uint64_t kSimFailSeed = ATA_SERVER_SIM_FAIL_SEED;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over offsets [0, size).
class PoolAlloc {
public:
    size_t size = 0, used = 0, peak = 0;
    void init(size_t s) {
        size = s;
        used = peak = 0;
        free_.clear();
        if (s) free_[0] = s;
    }
    bool alloc(size_t bytes, size_t& off) {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rem = it->second - bytes;
                free_.erase(it);
                if (rem) free_[off + bytes] = rem;
                used += bytes;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes ? bytes : 1);
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

struct Block {
    size_t off = 0, bytes = 0;
    bool held = false;
};

struct Req {
    uint64_t id = 0;
    ata_request r{};
    int state = ATA_REQ_QUEUED;
    int status = ATA_OK;
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0, t_due = 0;
    int batched = 0, stream = -1;
    int64_t footprint = 0;
    double flops = 0;
    Block a, c, w, tb, tb_acc, tb_tail;
    std::shared_ptr<PlanDev> plan;  // host plan; its tables are copied into block tb
    WsLayout L;
    // Row slabs of a large request (the row split of the block equations:
    // C = sum over slabs of A_s^t A_s).  Slab s covers rows
    // [s slab_rows, min(m, (s + 1) slab_rows)); the first writes C (plan),
    // the others add to it (plan_acc for full slabs, plan_tail for a shorter
    // last one), each launched once the previous slab has completed, so other
    // requests' launches on the same stream run in between.
    int nslab = 1, next_slab = 0;
    int64_t slab_rows = 0;
    std::shared_ptr<PlanDev> plan_acc, plan_tail;
    WsLayout L_acc, L_tail;
    int64_t cutoff = 0;
    int variant = 0, depth = 0;
    bool small = false;
    hipEvent_t ev = nullptr;
    int batch = -1;
};

struct Batch {
    hipEvent_t ev = nullptr;
    Block tables;
    std::vector<Req*> reqs;
    std::vector<BatchEntry> entries;
    std::vector<WorkItem> items;
};

size_t elem_bytes(int dtype) { return (dtype & 0xff) == ATA_F64 ? 8 : 4; }

}  // namespace

struct ata_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    PoolAlloc pool;
    char* base = nullptr;
    int dev = 0;
    int max_active = 1, nstreams = 1, flags = 0;
    double sim_tflops = 1.0;
    std::vector<hipStream_t> streams;
    int pass = 0;
    std::deque<Req*> queue;
    std::map<uint64_t, Req*> reqs;
    std::vector<Req*> running;
    std::map<int, Batch> batches;
    int next_batch = 0;
    uint64_t next_id = 1;
    int active = 0;
    bool stop = false;
    bool kick = false;  // set by submit / take: new work or freed memory
    ata_server_stats st{};
    std::thread th;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    bool sim() const { return flags & ATA_SERVER_SIMULATE; }
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void loop();
    hipError_t launch_slab(Req* q);
    void finish(Req* q, int status, double t);
    bool admit(Req* q, int pass_stream);
    void release_block(Block& b) {
        if (b.held) {
            pool.release(b.off, b.bytes);
            b.held = false;
        }
    }
};

void ata_server::finish(Req* q, int status, double t) {
    q->state = ATA_REQ_DONE;
    q->status = status;
    q->t_done = t;
    if (!q->r.keep_a) release_block(q->a);
    release_block(q->w);
    release_block(q->tb);
    release_block(q->tb_acc);
    release_block(q->tb_tail);
    if (q->ev) {
        (void)hipEventDestroy(q->ev);
        q->ev = nullptr;
    }
    --active;
    ++st.completed;
}

// Enqueue the request's next slab (the whole product when it has one slab)
// on its stream and record its event.
hipError_t ata_server::launch_slab(Req* q) {
    const int sl = q->next_slab;
    const bool last = sl == q->nslab - 1;
    const bool tail = q->nslab > 1 && last && q->plan_tail;
    const PlanDev& pd = sl == 0 ? *q->plan : (tail ? *q->plan_tail : *q->plan_acc);
    const Block& tb = sl == 0 ? q->tb : (tail ? q->tb_tail : q->tb_acc);
    const WsLayout& L = sl == 0 ? q->L : (tail ? q->L_tail : q->L_acc);
    const int64_t r0 = (int64_t)sl * q->slab_rows;
    const int64_t rows = q->nslab == 1 ? q->r.m : std::min(q->r.m - r0, q->slab_rows);
    const size_t eb = elem_bytes(q->r.dtype);
    hipStream_t s = streams[q->stream];
    hipError_t e = enqueue_product(pd, base + tb.off, L, base + q->a.off + (size_t)r0 * q->r.n * eb, rows, q->r.n,
                                   q->r.n, base + q->c.off, q->r.dtype, q->variant,
                                   q->w.held ? base + q->w.off : nullptr, s, dev);
    if (e == hipSuccess) e = hipEventRecord(q->ev, s);
    q->next_slab = sl + 1;
    return e;
}

// Allocate the request's blocks, fill A and upload its plan.  Returns false
// (nothing held) when the pool cannot hold it now.
bool ata_server::admit(Req* q, int pass_stream) {
    const int64_t m = q->r.m, n = q->r.n;
    const size_t eb = elem_bytes(q->r.dtype);
    const size_t abytes = (size_t)m * n * eb, cbytes = (size_t)(n * (n + 1) / 2) * eb;
    Block a, c, w;
    if (!pool.alloc(abytes, a.off)) return false;
    a.bytes = abytes;
    a.held = true;
    if (!pool.alloc(cbytes, c.off)) {
        release_block(a);
        return false;
    }
    c.bytes = cbytes;
    c.held = true;
    if (q->L.total) {
        if (!pool.alloc(q->L.total, w.off)) {
            release_block(a);
            release_block(c);
            return false;
        }
        w.bytes = q->L.total;
        w.held = true;
    }
    Block tb, tba, tbt;
    const size_t tbytes = q->plan->host_blob.size();
    if (!pool.alloc(tbytes, tb.off)) {
        release_block(a);
        release_block(c);
        release_block(w);
        return false;
    }
    tb.bytes = tbytes;
    tb.held = true;
    auto more = [&](const std::shared_ptr<PlanDev>& pd, Block& b) {
        if (!pd) return true;
        if (!pool.alloc(pd->host_blob.size(), b.off)) return false;
        b.bytes = pd->host_blob.size();
        b.held = true;
        return true;
    };
    if (!more(q->plan_acc, tba) || !more(q->plan_tail, tbt)) {
        release_block(a);
        release_block(c);
        release_block(w);
        release_block(tb);
        release_block(tba);
        return false;
    }
    q->a = a;
    q->c = c;
    q->w = w;
    q->tb = tb;
    q->tb_acc = tba;
    q->tb_tail = tbt;
    q->state = ATA_REQ_ADMITTED;
    q->t_admit = now();
    ++active;
    ++st.admitted;
    if (sim()) return true;
    const Plan& P = q->plan->plan;
    // a grouped launch runs the SYRK tiles of each member whole: plans with a
    // K-split last round launch on their own
    q->small = q->nslab == 1 && P.phases.size() == 1 && P.phases[0].str_items.empty() &&
               P.phases[0].tg_items.empty() && P.phases[0].gemm_items.empty() && P.phases[0].combines.empty() &&
               P.phases[0].tail_items.empty();
    q->stream = q->small ? pass_stream : (int)((pass + q->id) % streams.size());
    hipStream_t s = streams[q->stream];
    void* A = base + q->a.off;
    // the plan's tables travel with the request (no synchronous upload)
    hipError_t e = hipMemcpyAsync(base + q->tb.off, q->plan->host_blob.data(), tbytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && q->plan_acc)
        e = hipMemcpyAsync(base + q->tb_acc.off, q->plan_acc->host_blob.data(), q->tb_acc.bytes, hipMemcpyHostToDevice,
                           s);
    if (e == hipSuccess && q->plan_tail)
        e = hipMemcpyAsync(base + q->tb_tail.off, q->plan_tail->host_blob.data(), q->tb_tail.bytes,
                           hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
    } else if (q->r.src == ATA_SRC_HOST)
        e = hipMemcpyAsync(A, q->r.a, abytes, hipMemcpyHostToDevice, s);
    else if (q->r.src == ATA_SRC_DEVICE)
        e = hipMemcpyAsync(A, q->r.a, abytes, hipMemcpyDeviceToDevice, s);
    else
        e = launch_fill_normal(A, m * n, q->r.seed, eb == 8, s);
    if (e != hipSuccess) {
        // copies already queued on s may still write the blocks: let them
        // finish before the blocks go back to the pool
        (void)hipStreamSynchronize(s);
        finish(q, hip_fail(e), now());
        release_block(q->a);
    }
    return true;
}

void ata_server::loop() {
    if (!sim()) (void)hipSetDevice(dev);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // poll in-flight work every 50 us; wake at once on new work or freed memory
        cv_work.wait_for(lk, std::chrono::microseconds(50), [&] { return stop || kick; });
        kick = false;
        if (stop && !queue.empty()) {
            // destroy: queued requests are dropped, in-flight ones finish
            for (Req* q : queue) {
                q->state = ATA_REQ_DONE;
                q->status = ATA_EBUSY;
            }
            queue.clear();
        }
        if (stop && running.empty() && batches.empty()) break;
        bool any_done = false;
        // 1. completions
        const double tnow = now();
        for (size_t i = 0; i < running.size();) {
            Req* q = running[i];
            bool done = false;
            int status = ATA_OK;
            if (sim()) {
                done = tnow >= q->t_due;
                if (done && q->r.src == ATA_SRC_NORMAL && q->r.seed == kSimFailSeed) status = ATA_EHIP;
            } else {
                const hipError_t e = hipEventQuery(q->ev);
                if (e == hipSuccess) done = true;
                else if (e != hipErrorNotReady) {
                    done = true;
                    status = hip_fail(e);
                }
            }
            if (done && status == ATA_OK && !sim() && q->next_slab < q->nslab) {
                // the previous slab has completed: queue the next one behind
                // whatever else this pass put on the stream
                const hipError_t e = launch_slab(q);
                if (e == hipSuccess) {
                    ++i;
                    continue;
                }
                status = hip_fail(e);
            }
            if (done) {
                finish(q, status, tnow);
                running[i] = running.back();
                running.pop_back();
                any_done = true;
            } else {
                ++i;
            }
        }
        for (auto it = batches.begin(); it != batches.end();) {
            const hipError_t e = hipEventQuery(it->second.ev);
            if (e == hipErrorNotReady) {
                ++it;
                continue;
            }
            const int status = e == hipSuccess ? ATA_OK : hip_fail(e);
            for (Req* q : it->second.reqs) finish(q, status, tnow);
            (void)hipEventDestroy(it->second.ev);
            release_block(it->second.tables);
            it = batches.erase(it);
            any_done = true;
        }
        // 2. admission in arrival order, with a bounded bypass of a blocked head
        ++pass;
        const int pass_stream = streams.empty() ? 0 : pass % (int)streams.size();
        std::vector<Req*> ready;
        int scanned = 0;
        for (auto it = queue.begin(); it != queue.end() && active < max_active && scanned <= kBypass;) {
            Req* q = *it;
            ++scanned;
            if (admit(q, pass_stream)) {
                it = queue.erase(it);
                if (q->state == ATA_REQ_ADMITTED) ready.push_back(q);
                else any_done = true;
            } else {
                ++it;
            }
        }
        // 3. launches
        if (!ready.empty()) {
            if (sim()) {
                for (Req* q : ready) {
                    q->state = ATA_REQ_RUNNING;
                    q->t_launch = now();
                    q->t_due = q->t_launch + q->flops / (sim_tflops * 1e12);
                    running.push_back(q);
                }
            } else {
                std::map<int, std::vector<Req*>> small_by_type;
                for (Req* q : ready) {
                    if (q->small) {
                        small_by_type[q->r.dtype].push_back(q);
                        continue;
                    }
                    hipError_t e = hipEventCreateWithFlags(&q->ev, hipEventDisableTiming);
                    if (e == hipSuccess) e = launch_slab(q);
                    q->t_launch = now();
                    if (e != hipSuccess) {
                        finish(q, hip_fail(e), now());
                        any_done = true;
                        continue;
                    }
                    q->state = ATA_REQ_RUNNING;
                    running.push_back(q);
                }
                for (auto& kv : small_by_type) {
                    std::vector<Req*>& group = kv.second;
                    Batch b;
                    for (size_t slot = 0; slot < group.size(); ++slot) {
                        Req* q = group[slot];
                        const PlanDev& pd = *q->plan;
                        const char* tb = base + q->tb.off;
                        b.entries.push_back(BatchEntry{base + q->a.off, base + q->c.off,
                                                       (const DevTask*)(tb + pd.off_tasks),
                                                       (const DevTerm*)(tb + pd.off_terms),
                                                       (const int32_t*)(tb + pd.off_segs), q->r.n});
                        for (WorkItem wi : pd.plan.phases[0].syrk_items) {
                            wi.slot = (int32_t)slot;
                            b.items.push_back(wi);
                        }
                    }
                    const size_t eb = b.entries.size() * sizeof(BatchEntry);
                    const size_t ib = b.items.size() * sizeof(WorkItem);
                    hipStream_t s = streams[pass_stream];
                    hipError_t e = hipSuccess;
                    if (!pool.alloc(align_up(eb) + ib, b.tables.off)) e = hipErrorOutOfMemory;
                    if (e == hipSuccess) {
                        b.tables.bytes = align_up(eb) + ib;
                        b.tables.held = true;
                        e = hipMemcpyAsync(base + b.tables.off, b.entries.data(), eb, hipMemcpyHostToDevice, s);
                    }
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(base + b.tables.off + align_up(eb), b.items.data(), ib,
                                           hipMemcpyHostToDevice, s);
                    const bool f32 = (kv.first & 0xff) != ATA_F64;
                    if (e == hipSuccess)
                        e = launch_gemm_batch(f32, elem_bytes_out(kv.first) == 8,
                                              (const BatchEntry*)(base + b.tables.off),
                                              (const WorkItem*)(base + b.tables.off + align_up(eb)),
                                              (int)b.items.size(), s);
                    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
                    if (e == hipSuccess) e = hipEventRecord(b.ev, s);
                    const double tl = now();
                    if (e != hipSuccess) {
                        release_block(b.tables);
                        for (Req* q : group) finish(q, hip_fail(e), tl);
                        any_done = true;
                        continue;
                    }
                    for (Req* q : group) {
                        q->state = ATA_REQ_RUNNING;
                        q->batched = 1;
                        q->t_launch = tl;
                    }
                    ++st.batches;
                    st.batched_requests += (int64_t)group.size();
                    b.reqs = group;
                    batches.emplace(next_batch++, std::move(b));
                }
            }
        }
        if (any_done) cv_done.notify_all();
    }
}

namespace {

int validate_request(const ata_request* r) {
    if (!r) return -2;
    if (r->m < 0 || r->n < 1) return -2;
    if (r->dtype != ATA_F64 && r->dtype != ATA_F32) return -2;
    if (r->cutoff < 0 || r->max_depth < -2) return -2;
    if (r->src != ATA_SRC_HOST && r->src != ATA_SRC_DEVICE && r->src != ATA_SRC_NORMAL) return -2;
    if (r->src != ATA_SRC_NORMAL && r->m > 0 && !r->a) return -2;
    if (r->reserved != 0 || (r->keep_a != 0 && r->keep_a != 1)) return -2;
    if (r->m > INT32_MAX || r->n > INT32_MAX) return ATA_EUNSUPPORTED;
    if (r->n * (r->dtype == ATA_F64 ? 8 : 4) > kMaxRowBytes) return ATA_EUNSUPPORTED;
    return 0;
}

void fill_info(const Req* q, ata_request_info* info) {
    if (!info) return;
    info->state = q->state;
    info->status = q->status;
    info->m = q->r.m;
    info->n = q->r.n;
    info->t_submit = q->t_submit;
    info->t_admit = q->t_admit;
    info->t_launch = q->t_launch;
    info->t_done = q->t_done;
    info->batched = q->batched;
    info->stream = q->stream;
    info->footprint = q->footprint;
    info->flops = q->flops;
    info->slabs = q->nslab;
    info->reserved = 0;
}

}  // namespace

extern "C" {

int ata_server_create(size_t budget_bytes, int max_active, int streams, int flags, double simulate_tflops,
                      ata_server** out) {
    if (budget_bytes == 0) return -1;
    if (max_active < 1) return -2;
    if (streams < 1 || streams > 16) return -3;
    if (flags & ~ATA_SERVER_SIMULATE) return -4;
    if ((flags & ATA_SERVER_SIMULATE) && !(simulate_tflops > 0)) return -5;
    if (!out) return -6;
    std::unique_ptr<ata_server> s(new ata_server());
    s->max_active = max_active;
    s->nstreams = streams;
    s->flags = flags;
    s->sim_tflops = simulate_tflops;
    s->pool.init(budget_bytes);
    if (!s->sim()) {
        hipError_t e = hipGetDevice(&s->dev);
        if (e != hipSuccess) return hip_fail(e);
        hipDeviceProp_t p;
        e = hipGetDeviceProperties(&p, s->dev);
        if (e != hipSuccess) return hip_fail(e);
        if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) return ATA_EUNSUPPORTED;
        e = hipMalloc((void**)&s->base, budget_bytes);
        if (e != hipSuccess) return hip_fail(e);
        for (int i = 0; i < streams; ++i) {
            hipStream_t st;
            e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e != hipSuccess) {
                for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
                (void)hipFree(s->base);
                return hip_fail(e);
            }
            s->streams.push_back(st);
        }
    }
    s->st.pool_bytes = (int64_t)budget_bytes;
    ata_server* raw = s.release();
    raw->th = std::thread([raw] { raw->loop(); });
    *out = raw;
    return ATA_OK;
}

int ata_server_submit(ata_server* srv, const ata_request* req, uint64_t* ticket) {
    if (!srv) return -1;
    int rc = validate_request(req);
    if (rc) return rc;
    if (!ticket) return -3;
    std::unique_ptr<Req> q(new Req());
    q->r = *req;
    q->variant = ATA_VARIANT_STRASSEN;
    q->depth = req->max_depth == -2 ? ATA_DEFAULT_MAX_DEPTH : req->max_depth;
    q->cutoff = req->cutoff ? req->cutoff : default_cutoff(req->m, req->n, req->dtype);
    q->flops = (double)req->m * (double)req->n * (double)req->n;
    // footprint from the host plan (no device work on the caller's thread)
    std::shared_ptr<PlanDev> hp;
    size_t wsmax = 0, tables = 0;
    if (req->m > 0) {
        q->slab_rows = slab_rows_for(req->m, req->n);
        const int64_t rows = q->slab_rows ? q->slab_rows : req->m;
        q->nslab = q->slab_rows ? (int)((req->m + rows - 1) / rows) : 1;
        if (q->slab_rows && !req->cutoff) q->cutoff = default_cutoff(rows, req->n, req->dtype);
        // the library's default depth rule for requests that leave it open;
        // the dtype class always (it selects the plan's split of short last rounds)
        const int pf = plan_flags(req->max_depth == -2 ? ATA_OPT_ADAPTIVE : 0, req->dtype);
        rc = get_plan(rows, req->n, q->cutoff, q->variant, q->depth, pf, false, hp);
        if (rc != ATA_OK) return rc;
        q->L = ws_layout(rows, req->n, req->dtype, hp->plan.ws_elems, false, hp->plan.opsum_elems);
        q->plan = hp;
        wsmax = q->L.total;
        tables = align_up(hp->host_blob.size());
        if (q->nslab > 1) {
            rc = get_plan(rows, req->n, q->cutoff, q->variant, q->depth, pf | kPlanAccumulate, false, q->plan_acc);
            if (rc != ATA_OK) return rc;
            q->L_acc = ws_layout(rows, req->n, req->dtype, q->plan_acc->plan.ws_elems, false,
                                 q->plan_acc->plan.opsum_elems);
            wsmax = std::max(wsmax, q->L_acc.total);
            tables += align_up(q->plan_acc->host_blob.size());
            const int64_t tail = req->m - (int64_t)(q->nslab - 1) * rows;
            if (tail != rows) {
                rc = get_plan(tail, req->n, q->cutoff, q->variant, q->depth, pf | kPlanAccumulate, false, q->plan_tail);
                if (rc != ATA_OK) return rc;
                q->L_tail = ws_layout(tail, req->n, req->dtype, q->plan_tail->plan.ws_elems, false,
                                      q->plan_tail->plan.opsum_elems);
                wsmax = std::max(wsmax, q->L_tail.total);
                tables += align_up(q->plan_tail->host_blob.size());
            }
        }
        // every slab's workspace layout fits in the largest one's bytes
        q->L.total = q->L_acc.total = q->L_tail.total = wsmax;
    }
    const size_t eb = elem_bytes(req->dtype);
    q->footprint = (int64_t)(align_up((size_t)req->m * req->n * eb) +
                             align_up((size_t)(req->n * (req->n + 1) / 2) * eb) + align_up(wsmax) + tables);
    std::lock_guard<std::mutex> lk(srv->mu);
    ++srv->st.submitted;
    if ((size_t)q->footprint > srv->pool.size) {
        ++srv->st.rejected;
        return ATA_EREJECT;
    }
    if (req->m == 0) {
        // empty sum: the result is zero; no device work is needed until taken
        q->state = ATA_REQ_DONE;
        q->t_submit = q->t_admit = q->t_launch = q->t_done = srv->now();
        const uint64_t id = srv->next_id++;
        q->id = id;
        *ticket = id;
        ++srv->st.completed;
        srv->reqs[id] = q.release();
        return ATA_OK;
    }
    q->id = srv->next_id++;
    q->t_submit = srv->now();
    *ticket = q->id;
    Req* raw = q.release();
    srv->reqs[raw->id] = raw;
    srv->queue.push_back(raw);
    srv->kick = true;
    srv->cv_work.notify_one();
    return ATA_OK;
}

int ata_server_query(ata_server* srv, uint64_t ticket, ata_request_info* info) {
    if (!srv) return -1;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return ATA_ENOTFOUND;
    fill_info(it->second, info);
    return it->second->state == ATA_REQ_DONE ? ATA_OK : ATA_EPENDING;
}

int ata_server_wait(ata_server* srv, uint64_t ticket, double timeout_s, ata_request_info* info) {
    if (!srv) return -1;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 0);
    for (;;) {
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end()) return ATA_ENOTFOUND;
        if (it->second->state == ATA_REQ_DONE) {
            fill_info(it->second, info);
            return ATA_OK;
        }
        if (srv->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            auto it2 = srv->reqs.find(ticket);
            if (it2 == srv->reqs.end()) return ATA_ENOTFOUND;
            fill_info(it2->second, info);
            return it2->second->state == ATA_REQ_DONE ? ATA_OK : ATA_EPENDING;
        }
    }
}

int ata_server_take(ata_server* srv, uint64_t ticket, void* c, void* a_out, int on_device) {
    const int c_on_device = on_device;
    if (!srv) return -1;
    Req* q = nullptr;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end()) return ATA_ENOTFOUND;
        q = it->second;
        if (q->state != ATA_REQ_DONE) return ATA_EPENDING;
        if (q->status != ATA_OK) {
            // a failed request is released here: its blocks go back to the pool
            const int st = q->status;
            srv->reqs.erase(it);
            srv->release_block(q->a);
            srv->release_block(q->c);
            srv->release_block(q->w);
            srv->release_block(q->tb);
            srv->release_block(q->tb_acc);
            srv->release_block(q->tb_tail);
            delete q;
            srv->kick = true;
            srv->cv_work.notify_one();
            return st;
        }
        if (a_out && q->r.m > 0 && !q->a.held) return -4;
        srv->reqs.erase(it);  // the caller now owns the request's remaining blocks
    }
    const size_t eb = elem_bytes(q->r.dtype);
    const size_t cbytes = (size_t)(q->r.n * (q->r.n + 1) / 2) * eb;
    int rc = ATA_OK;
    if (srv->sim()) {
        // no device data in simulate mode
    } else if (q->r.m == 0) {
        if (c && cbytes) {
            hipError_t e = c_on_device ? hipMemset(c, 0, cbytes) : hipSuccess;
            if (!c_on_device) std::memset(c, 0, cbytes);
            if (e != hipSuccess) rc = hip_fail(e);
        }
    } else {
        if (c) {
            hipError_t e = hipMemcpy(c, srv->base + q->c.off, cbytes,
                                     c_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
            if (e != hipSuccess) rc = hip_fail(e);
        }
        if (rc == ATA_OK && a_out) {
            hipError_t e = hipMemcpy(a_out, srv->base + q->a.off, (size_t)q->r.m * q->r.n * eb,
                                     on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
            if (e != hipSuccess) rc = hip_fail(e);
        }
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->release_block(q->a);
    srv->release_block(q->c);
    srv->release_block(q->w);
    srv->release_block(q->tb);
    srv->release_block(q->tb_acc);
    srv->release_block(q->tb_tail);
    delete q;
    srv->kick = true;
    srv->cv_work.notify_one();
    return rc;
}

int ata_server_release(ata_server* srv, uint64_t ticket) { return ata_server_take(srv, ticket, nullptr, nullptr, 0); }

int ata_server_get_stats(ata_server* srv, ata_server_stats* out) {
    if (!srv) return -1;
    if (!out) return -2;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    out->pool_in_use = (int64_t)srv->pool.used;
    out->pool_peak = (int64_t)srv->pool.peak;
    out->queued = (int64_t)srv->queue.size();
    out->active = srv->active;
    return ATA_OK;
}

double ata_server_now(ata_server* srv) { return srv ? srv->now() : 0.0; }

int ata_server_destroy(ata_server* srv) {
    if (!srv) return -1;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->th.joinable()) srv->th.join();
    for (auto& kv : srv->reqs) delete kv.second;
    srv->reqs.clear();
    if (!srv->sim()) {
        for (hipStream_t s : srv->streams) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        if (srv->base) (void)hipFree(srv->base);
    }
    delete srv;
    return ATA_OK;
}

}  // extern "C"
