// C ABI of the normal-equation consumers: Cholesky factor, triangular solves,
// A^t B, the chained least-squares solve and the projection (declared in
// ata.h).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>

#include "ata.h"
#include "ata_internal.h"
#include "ata_kernels.h"

using namespace atalib;
using namespace atalib::detail;

namespace {

constexpr int64_t kMaxOrder = int64_t(1) << 22;

bool solve_dtype(int dtype) { return dtype == ATA_F64 || dtype == ATA_F32; }

int64_t max1(int64_t x) { return x > 1 ? x : 1; }

// A device pointer must be aligned to its element (4 or 8 bytes).
bool misaligned(const void* p, int dtype) { return (uintptr_t)p % (dtype == ATA_F32 ? 4 : 8) != 0; }

#define SOLVE_TRY(expr)                            \
    do {                                           \
        hipError_t _e = (expr);                    \
        if (_e != hipSuccess) return hip_fail(_e); \
    } while (0)

// Lookahead helper of the factorization, one per device, created on first
// use and kept until ata_release_caches or the end of the process: a stream
// at the default priority and two events.  The mutex is held while a factorization is enqueued, so calls
// from several threads never interleave their event records.
struct Lookahead {
    hipStream_t s2 = nullptr;
    hipEvent_t e = nullptr, f = nullptr;
};
std::mutex g_look_mu;
std::map<int, Lookahead> g_look;

int potrf_checked(void* C, int64_t n, int dtype, int32_t* info, hipStream_t s) {
    if (info) SOLVE_TRY(launch_fill_zero(info, 1, 4, s));
    if (n == 0) return ATA_OK;
    int dev = 0;
    SOLVE_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_look_mu);
    Lookahead& la = g_look[dev];
    if (!la.s2) {
        Lookahead nl;
        SOLVE_TRY(hipStreamCreateWithFlags(&nl.s2, hipStreamNonBlocking));
        SOLVE_TRY(hipEventCreateWithFlags(&nl.e, hipEventDisableTiming));
        SOLVE_TRY(hipEventCreateWithFlags(&nl.f, hipEventDisableTiming));
        la = nl;
    }
    SOLVE_TRY(launch_potrf(dtype == ATA_F32, C, n, info, s, la.s2, la.e, la.f));
    return ATA_OK;
}

int atb_checked(const void* A, int64_t m, int64_t n, int64_t lda, const void* B, int64_t nrhs, int64_t ldb, void* out,
                int64_t ldo, int dtype, hipStream_t s) {
    if (n == 0 || nrhs == 0) return ATA_OK;
    const size_t bytes = (size_t)atb_chunks(m, n) * (size_t)n * (size_t)nrhs * sizeof(double);
    double* part = nullptr;
    SOLVE_TRY(hipMallocAsync((void**)&part, bytes, s));
    hipError_t e = launch_atb(dtype == ATA_F32, A, m, n, lda, B, nrhs, ldb, out, ldo, part, s);
    const hipError_t e2 = hipFreeAsync(part, s);
    if (e == hipSuccess) e = e2;
    return e == hipSuccess ? ATA_OK : hip_fail(e);
}

}  // namespace

void atalib::detail::release_lookahead() {
    std::lock_guard<std::mutex> lk(g_look_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_look) {
        if (!kv.second.s2) continue;
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
        (void)hipEventDestroy(kv.second.e);
        (void)hipEventDestroy(kv.second.f);
        (void)hipStreamDestroy(kv.second.s2);
    }
    g_look.clear();
    (void)hipSetDevice(cur);
}

extern "C" {

int ata_potrf(void* C_lower, int64_t n, int dtype, int32_t* info, void* stream) {
    if (n < 0) return -2;
    if (n > 0 && !C_lower) return -1;
    if (!solve_dtype(dtype)) return -3;
    if (misaligned(C_lower, dtype)) return -1;
    if ((uintptr_t)info % 4) return -4;
    if (n > kMaxOrder) return ATA_EUNSUPPORTED;
    if (!current_device_ok()) return ATA_EUNSUPPORTED;
    return potrf_checked(C_lower, n, dtype, info, (hipStream_t)stream);
}

int ata_potrs(const void* L_lower, int64_t n, void* B, int64_t nrhs, int64_t ldb, int dtype, void* stream) {
    if (n < 0) return -2;
    if (nrhs < 0) return -4;
    if (n > 0 && !L_lower) return -1;
    if (n > 0 && nrhs > 0 && !B) return -3;
    if (ldb < max1(nrhs)) return -5;
    if (!solve_dtype(dtype)) return -6;
    if (misaligned(L_lower, dtype)) return -1;
    if (misaligned(B, dtype)) return -3;
    if (n > kMaxOrder) return ATA_EUNSUPPORTED;
    if (!current_device_ok()) return ATA_EUNSUPPORTED;
    if (n == 0 || nrhs == 0) return ATA_OK;
    SOLVE_TRY(launch_potrs(dtype == ATA_F32, L_lower, n, B, nrhs, ldb, (hipStream_t)stream));
    return ATA_OK;
}

int ata_atb(const void* A, int64_t m, int64_t n, int64_t lda, const void* B, int64_t nrhs, int64_t ldb, void* out,
            int64_t ldo, int dtype, void* stream) {
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (lda < max1(n)) return -4;
    if (nrhs < 0) return -6;
    if (ldb < max1(nrhs)) return -7;
    if (ldo < max1(nrhs)) return -9;
    if (m > 0 && n > 0 && !A) return -1;
    if (m > 0 && nrhs > 0 && !B) return -5;
    if (n > 0 && nrhs > 0 && !out) return -8;
    if (!solve_dtype(dtype)) return -10;
    if (misaligned(A, dtype)) return -1;
    if (misaligned(B, dtype)) return -5;
    if (misaligned(out, dtype)) return -8;
    if (!current_device_ok()) return ATA_EUNSUPPORTED;
    return atb_checked(A, m, n, lda, B, nrhs, ldb, out, ldo, dtype, (hipStream_t)stream);
}

int ata_normal_solve(const void* A, int64_t m, int64_t n, int64_t lda, const void* B, int64_t nrhs, int64_t ldb,
                     void* X, int64_t ldx, int dtype, int cutoff, int32_t* info, void* stream) {
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (lda < max1(n)) return -4;
    if (nrhs < 0) return -6;
    if (ldb < max1(nrhs)) return -7;
    if (ldx < max1(nrhs)) return -9;
    if (m > 0 && n > 0 && !A) return -1;
    if (m > 0 && nrhs > 0 && !B) return -5;
    if (n > 0 && nrhs > 0 && !X) return -8;
    if (!solve_dtype(dtype)) return -10;
    if (cutoff < 0) return -11;
    if (misaligned(A, dtype)) return -1;
    if (misaligned(B, dtype)) return -5;
    if (misaligned(X, dtype)) return -8;
    if ((uintptr_t)info % 4) return -12;
    if (n > kMaxOrder) return ATA_EUNSUPPORTED;
    if (!current_device_ok()) return ATA_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return potrf_checked(nullptr, 0, dtype, info, s);
    const size_t cbytes = (size_t)(n * (n + 1) / 2) * (dtype == ATA_F32 ? 4 : 8);
    void* C = nullptr;
    SOLVE_TRY(hipMallocAsync(&C, cbytes, s));
    int rc = ata_ex(A, m, n, lda, C, dtype, cutoff, stream, nullptr, nullptr, 0);
    if (rc == ATA_OK) rc = potrf_checked(C, n, dtype, info, s);
    if (rc == ATA_OK) rc = atb_checked(A, m, n, lda, B, nrhs, ldb, X, ldx, dtype, s);
    if (rc == ATA_OK && nrhs > 0) {
        const hipError_t e = launch_potrs(dtype == ATA_F32, C, n, X, nrhs, ldx, s);
        if (e != hipSuccess) rc = hip_fail(e);
    }
    const hipError_t ef = hipFreeAsync(C, s);
    if (rc == ATA_OK && ef != hipSuccess) rc = hip_fail(ef);
    return rc;
}

int ata_project(const void* A, int64_t m, int64_t n, int64_t lda, const void* B, int64_t nrhs, int64_t ldb,
                void* out, int64_t ldo, int dtype, int cutoff, int32_t* info, void* stream) {
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (lda < max1(n)) return -4;
    if (nrhs < 0) return -6;
    if (ldb < max1(nrhs)) return -7;
    if (ldo < max1(nrhs)) return -9;
    if (m > 0 && n > 0 && !A) return -1;
    if (m > 0 && nrhs > 0 && !B) return -5;
    if (m > 0 && nrhs > 0 && !out) return -8;
    if (!solve_dtype(dtype)) return -10;
    if (cutoff < 0) return -11;
    if (misaligned(A, dtype)) return -1;
    if (misaligned(B, dtype)) return -5;
    if (misaligned(out, dtype)) return -8;
    if ((uintptr_t)info % 4) return -12;
    if (n > kMaxOrder || (m + 3) / 4 > INT32_MAX) return ATA_EUNSUPPORTED;
    if (!current_device_ok()) return ATA_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (m == 0 || nrhs == 0 || n == 0) {
        // no columns: the projection is zero; no rows or right-hand sides: nothing to write
        int rc = potrf_checked(nullptr, 0, dtype, info, s);
        if (rc == ATA_OK && m > 0 && nrhs > 0) {
            const hipError_t e = launch_ax(dtype == ATA_F32, A, m, 0, lda, nullptr, nrhs, nrhs, out, ldo, s);
            if (e != hipSuccess) rc = hip_fail(e);
        }
        return rc;
    }
    void* X = nullptr;
    SOLVE_TRY(hipMallocAsync(&X, (size_t)n * (size_t)nrhs * (dtype == ATA_F32 ? 4 : 8), s));
    int rc = ata_normal_solve(A, m, n, lda, B, nrhs, ldb, X, nrhs, dtype, cutoff, info, stream);
    if (rc == ATA_OK) {
        const hipError_t e = launch_ax(dtype == ATA_F32, A, m, n, lda, X, nrhs, nrhs, out, ldo, s);
        if (e != hipSuccess) rc = hip_fail(e);
    }
    const hipError_t ef = hipFreeAsync(X, s);
    if (rc == ATA_OK && ef != hipSuccess) rc = hip_fail(ef);
    return rc;
}

}  // extern "C"
