// C ABI entry points for the residual and the Jacobian-vector product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bim_common.h"
#include "vec.h"

namespace bim {

namespace {
thread_local std::string g_last_error;
}

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return BIM_OK;
    if (e == hipErrorOutOfMemory) return fail(BIM_ENOMEM, std::string(what) + ": out of device memory");
    return fail(BIM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int validate(const bim_problem *p) {
    if (!p) return fail(BIM_EINVAL, "problem is NULL");
    if (p->N < 3 || p->M < 3) return fail(BIM_EINVAL, "mesh needs N >= 3 and M >= 3");
    if ((long)p->N * p->M > (1L << 26)) return fail(BIM_EINVAL, "mesh too large");
    if (!(p->dx > 0.0) || !(p->dy > 0.0)) return fail(BIM_EINVAL, "dx and dy must be positive");
    if (!(p->froude > 0.0) || !std::isfinite(p->froude)) return fail(BIM_EINVAL, "Froude number must be positive");
    if (!std::isfinite(p->x1) || !std::isfinite(p->y1) || !std::isfinite(p->n_decay))
        return fail(BIM_EINVAL, "non-finite mesh origin or decay rate");
    if (p->half_domain && p->y1 != 0.0) return fail(BIM_EINVAL, "a half domain must start at y1 = 0");
    if (!p->beta || !p->beta_x || !p->beta_y) return fail(BIM_EINVAL, "bottom arrays must be device pointers");
    if (!std::isfinite(p->tau)) return fail(BIM_EINVAL, "surface tension must be finite");
    if (p->tau != 0.0 && p->M < 4) return fail(BIM_EINVAL, "surface tension needs M >= 4 (one-sided second y-differences)");
    return BIM_OK;
}

// Stream-ordered scratch allocation that is released when it goes out of scope.
struct Scratch {
    void *ptr = nullptr;
    hipStream_t s;
    explicit Scratch(hipStream_t st) : s(st) {}
    int alloc(size_t bytes) { return hip_check(hipMallocAsync(&ptr, bytes, s), "hipMallocAsync"); }
    ~Scratch() {
        if (ptr) (void)hipFreeAsync(ptr, s);
    }
};

// Workspace of the per-call entry points, kept per (device, stream) and grown
// on demand: successive calls on one stream reuse it in stream order.  The lock
// is held from the lookup until the call's work is enqueued, so a growth by
// another host thread (which waits for the stream before freeing) cannot free
// memory that a call is about to use.
struct StreamWorkspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mutex;
std::map<std::pair<int, hipStream_t>, StreamWorkspace> g_ws;

int stream_workspace(hipStream_t s, size_t bytes, void **out) {
    int dev = 0;
    int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    StreamWorkspace &ws = g_ws[{dev, s}];
    if (ws.bytes < bytes) {
        if (ws.ptr) {
            if ((rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
            if ((rc = hip_check(hipFree(ws.ptr), "hipFree"))) return rc;
            ws.ptr = nullptr;
            ws.bytes = 0;
        }
        if ((rc = hip_check(hipMalloc(&ws.ptr, bytes), "hipMalloc"))) return rc;
        ws.bytes = bytes;
    }
    *out = ws.ptr;
    return BIM_OK;
}

}  // namespace bim

using namespace bim;

extern "C" {

const char *bim_last_error(void) { return g_last_error.c_str(); }

const char *bim_version(void) { return "bim-mi355x 0.1"; }

static int residual_call(const bim_problem *prob, const double *u, double *F, int prec, void *stream, int linear) {
    g_last_error.clear();
    int rc = validate(prob);
    if (rc) return rc;
    if (!u || !F) return fail(BIM_EINVAL, "u and F must be device pointers");
    if (u == F) return fail(BIM_EINVAL, "F must not alias u");
    if (prec != BIM_FP64 && prec != BIM_FP32C) return fail(BIM_EINVAL, "unknown precision");
    hipStream_t s = (hipStream_t)stream;
    const Dims d(prob);
    const PairLaunch pl = pair_launch_for(prob, prec);
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    void *ws = nullptr;
    if ((rc = stream_workspace(s, residual_work_bytes(d, pl), &ws))) return rc;
    ResidualWork w;
    residual_work_carve(ws, d, pl, &w);
    return residual_enqueue(prob, u, F, prec, pl, w, s, nullptr, linear);
}

int bim_residual(const bim_problem *prob, const double *u, double *F, int prec, void *stream) {
    return residual_call(prob, u, F, prec, stream, 0);
}

int bim_residual_linear(const bim_problem *prob, const double *u, double *F, int prec, void *stream) {
    return residual_call(prob, u, F, prec, stream, 1);
}

int bim_residual_timed(const bim_problem *prob, const double *u, double *F, int prec, int iters,
                       const bim_pair_config *cfg, void *stream, double *kernel_ms, double *total_ms) {
    g_last_error.clear();
    int rc = validate(prob);
    if (rc) return rc;
    if (!u || !F || u == F) return fail(BIM_EINVAL, "u and F must be distinct device pointers");
    if (prec != BIM_FP64 && prec != BIM_FP32C) return fail(BIM_EINVAL, "unknown precision");
    if (iters < 1 || !kernel_ms || !total_ms) return fail(BIM_EINVAL, "iters >= 1 and result pointers required");
    hipStream_t s = (hipStream_t)stream;
    const Dims d(prob);
    const PairLaunch pl = cfg ? pair_launch_cfg(d, prec, *cfg) : pair_launch_for(prob, prec);
    Scratch sc(s);
    if ((rc = sc.alloc(residual_work_bytes(d, pl)))) return rc;
    ResidualWork w;
    residual_work_carve(sc.ptr, d, pl, &w);
    std::vector<hipEvent_t> ev(4 * (size_t)iters, nullptr);
    for (auto &e : ev)
        if ((rc = hip_check(hipEventCreate(&e), "hipEventCreate"))) break;
    for (int it = 0; rc == BIM_OK && it < iters; ++it) {
        hipEvent_t *e = &ev[4 * (size_t)it];
        if ((rc = hip_check(hipEventRecord(e[0], s), "hipEventRecord"))) break;
        if ((rc = residual_enqueue(prob, u, F, prec, pl, w, s, e + 1))) break;
        rc = hip_check(hipEventRecord(e[3], s), "hipEventRecord");
    }
    if (rc == BIM_OK) rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    double ksum = 0.0, tsum = 0.0;
    for (int it = 0; rc == BIM_OK && it < iters; ++it) {
        float a = 0.f, b = 0.f;
        hipEvent_t *e = &ev[4 * (size_t)it];
        if ((rc = hip_check(hipEventElapsedTime(&a, e[1], e[2]), "hipEventElapsedTime"))) break;
        if ((rc = hip_check(hipEventElapsedTime(&b, e[0], e[3]), "hipEventElapsedTime"))) break;
        ksum += a;
        tsum += b;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc) return rc;
    *kernel_ms = ksum / iters;
    *total_ms = tsum / iters;
    return BIM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free residual
namespace bim {

// Fixed device scratch of the allocation-free residual: every call on a GPU
// carves its workspace out of that GPU's copy of this array.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// Device address of `scratch` per device, looked up once per device with that
// device current (the array's name is a host-side stand-in in host code).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_addr[kMaxDevices] = {};

int scratch_address(void **out) {
    int dev = 0;
    int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return fail(BIM_EINVAL, "device index beyond the allocation-free residual's table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        if ((rc = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress"))) return rc;
        if (!ptr) return fail(BIM_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return BIM_OK;
}

}  // namespace
}  // namespace bim

extern "C" {

size_t bim_residual_noalloc_max_bytes(void) { return kNoAllocBytes; }

int bim_residual_noalloc(const bim_problem *prob, const double *u, double *F, int prec, void *stream) {
    g_last_error.clear();
    int rc = validate(prob);
    if (rc) return rc;
    if (!u || !F) return fail(BIM_EINVAL, "u and F must be device pointers");
    if (u == F) return fail(BIM_EINVAL, "F must not alias u");
    if (prec != BIM_FP64 && prec != BIM_FP32C) return fail(BIM_EINVAL, "unknown precision");
    const Dims d(prob);
    PairLaunch pl = pair_launch_for(prob, prec);
    if (residual_work_bytes(d, pl) > kNoAllocBytes) {
        // the workspace is linear in the chunk count: keep the launch's variant
        // and use the most source chunks whose partial sums still fit
        const size_t one = residual_work_bytes(d, pair_launch(d, pl.tpl, pl.unroll, 1));
        const size_t per_chunk = sizeof(double) * 2 * 2 * (size_t)d.ntg;
        if (one > kNoAllocBytes)
            return fail(BIM_EINVAL, "mesh too large for the allocation-free residual's " +
                                        std::to_string(kNoAllocBytes >> 20) + " MiB scratch");
        const long fit = 1 + (long)((kNoAllocBytes - one) / per_chunk);
        pl = pair_launch(d, pl.tpl, pl.unroll, (int)std::min<long>(fit, pl.chunks));
        while (pl.chunks > 1 && residual_work_bytes(d, pl) > kNoAllocBytes)
            pl = pair_launch(d, pl.tpl, pl.unroll, pl.chunks - 1);
    }
    void *base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    ResidualWork w;
    residual_work_carve(base, d, pl, &w);
    return residual_enqueue(prob, u, F, prec, pl, w, (hipStream_t)stream, nullptr, 0);
}

int bim_jv(const bim_problem *prob, const double *u, const double *Fu, const double *v, double h, double *Jv,
           int prec, void *stream) {
    g_last_error.clear();
    int rc = validate(prob);
    if (rc) return rc;
    if (!u || !Fu || !v || !Jv) return fail(BIM_EINVAL, "u, Fu, v and Jv must be device pointers");
    if (Jv == u || Jv == Fu || Jv == v) return fail(BIM_EINVAL, "Jv must not alias an input");
    if (prec != BIM_FP64 && prec != BIM_FP32C) return fail(BIM_EINVAL, "unknown precision");
    if (!std::isfinite(h)) return fail(BIM_EINVAL, "h must be finite");
    hipStream_t s = (hipStream_t)stream;
    const Dims d(prob);
    const PairLaunch pl = pair_launch_for(prob, prec);
    const size_t vec_bytes = ((sizeof(double) * d.nvec) + 255) & ~(size_t)255;
    const size_t red_bytes = ((sizeof(double) * reduce_parts()) + 255) & ~(size_t)255;
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    void *ws = nullptr;
    if ((rc = stream_workspace(s, residual_work_bytes(d, pl) + 2 * vec_bytes + red_bytes, &ws))) return rc;
    ResidualWork w;
    residual_work_carve(ws, d, pl, &w);
    double *uw = (double *)((char *)ws + w.bytes);
    double *Fw = (double *)((char *)uw + vec_bytes);
    double *part = (double *)((char *)Fw + vec_bytes);
    const double eps = (prec == BIM_FP64) ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23);
    if ((rc = fd_shift_enqueue(u, v, d.nvec, h, eps, part, w.scal, s))) return rc;
    if ((rc = axpy_dev_enqueue(u, v, w.scal + 2, uw, d.nvec, s))) return rc;
    if ((rc = residual_enqueue(prob, uw, Fw, prec, pl, w, s))) return rc;
    return quotient_enqueue(Fw, Fu, w.scal + 2, Jv, d.nvec, s);
}

int bim_release_workspaces(void) {
    g_last_error.clear();
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    int rc = BIM_OK, cur = 0;
    if ((rc = hip_check(hipGetDevice(&cur), "hipGetDevice"))) return rc;
    for (auto &kv : g_ws) {
        if (!kv.second.ptr) continue;
        int r2 = hip_check(hipSetDevice(kv.first.first), "hipSetDevice");
        if (r2) {
            if (!rc) rc = r2;
            continue;
        }
        // a stream destroyed by the caller cannot be waited on: wait for the device
        if (hipStreamSynchronize(kv.first.second) != hipSuccess) {
            (void)hipGetLastError();
            r2 = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        }
        if (!r2) r2 = hip_check(hipFree(kv.second.ptr), "hipFree");
        if (r2 && !rc) rc = r2;
    }
    g_ws.clear();
    const int r3 = hip_check(hipSetDevice(cur), "hipSetDevice");
    return rc ? rc : r3;
}

}  // extern "C"

// ------------------------------------------------------------------ batched residual
namespace bim {

int balanced_chunks(const Dims &d, int pairs_target) {
    // a node of a source-row visit covers nimg images
    const long pairs = (long)2 * d.M * d.N * d.nimg;
    return (int)std::max(1L, (pairs + pairs_target - 1) / pairs_target);
}

}  // namespace bim

extern "C" int bim_residual_batched(const bim_problem *probs, int count, const double *const *u, double *const *F,
                                    int prec, void *stream) {
    g_last_error.clear();
    if (count < 0 || (count > 0 && (!probs || !u || !F))) return fail(BIM_EINVAL, "bad batch arguments");
    if (count == 0) return BIM_OK;
    if (prec != BIM_FP64 && prec != BIM_FP32C) return fail(BIM_EINVAL, "unknown precision");
    int rc;
    for (int i = 0; i < count; ++i) {
        if ((rc = validate(&probs[i]))) return rc;
        if (!u[i] || !F[i] || u[i] == F[i]) return fail(BIM_EINVAL, "u[i], F[i] must be distinct device pointers");
    }
    hipStream_t s = (hipStream_t)stream;
    // one kernel variant for the batch: the tuned one of the largest problem
    int big = 0;
    for (int i = 1; i < count; ++i)
        if ((long)probs[i].N * probs[i].M > (long)probs[big].N * probs[big].M) big = i;
    const PairLaunch ref = pair_launch_for(&probs[big], prec);
    std::vector<PairLaunch> pls(count);
    std::vector<ResidualWork> ws(count);
    size_t total = 0;
    std::vector<size_t> offs(count);
    for (int i = 0; i < count; ++i) {
        const Dims d(&probs[i]);
        pls[i] = pair_launch(d, ref.tpl, ref.unroll, balanced_chunks(d, 6 * 181));
        offs[i] = total;
        total += (residual_work_bytes(d, pls[i]) + 255) & ~(size_t)255;
    }
    const size_t desc_off = total;
    total += sizeof(PairDesc) * count;
    Scratch sc(s);
    if ((rc = sc.alloc(total))) return rc;
    for (int i = 0; i < count; ++i) residual_work_carve((char *)sc.ptr + offs[i], Dims(&probs[i]), pls[i], &ws[i]);
    return residual_batched_enqueue(probs, count, u, F, prec, pls.data(), ws.data(),
                                    (PairDesc *)((char *)sc.ptr + desc_off), 0, s);
}
