// Autotuner for the all-pairs launch shape: times every supported variant on
// the caller's mesh and keeps the fastest per (N, M, half_domain, precision).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "bim_common.h"

namespace bim {

namespace {
using Key = std::tuple<int, int, int, int>;
std::mutex g_mu;
std::map<Key, bim_pair_config> g_best;
}  // namespace

PairLaunch pair_launch_for(const bim_problem *p, int prec) {
    const Dims d(p);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_best.find(Key(p->N, p->M, p->half_domain ? 1 : 0, prec));
        if (it != g_best.end())
            return pair_launch(d, it->second.targets_per_lane, it->second.unroll, it->second.rows_per_chunk);
    }
    // untuned defaults: the fastest shapes measured at 181 x 61 (FP64: 4-way
    // unroll, ~16 waves per SIMD; FP32C: 2-way unroll, ~24 waves per SIMD)
    if (prec == BIM_FP32C) return pair_launch(d, 1, 2, 0, 24576);
    return pair_launch(d, 1, 4, 0, 16384);
}

}  // namespace bim

using namespace bim;

extern "C" int bim_tune_residual(const bim_problem *prob, const double *u, int prec, void *stream,
                                 bim_pair_config *best, double *best_ms) {
    int rc = validate(prob);
    if (rc) return rc;
    if (!u) return fail(BIM_EINVAL, "u must be a device pointer");
    if (prec != BIM_FP64 && prec != BIM_FP32C) return fail(BIM_EINVAL, "unknown precision");
    const Dims d(prob);
    hipStream_t s = (hipStream_t)stream;
    double *F = nullptr;
    if ((rc = hip_check(hipMallocAsync((void **)&F, sizeof(double) * d.nvec, s), "hipMallocAsync"))) return rc;
    std::vector<bim_pair_config> cands;
    const int src_rows = 2 * d.M;
    for (int tpl : {1, 2})
        for (int unr : {2, 4, 8})
            for (long want : {8192L, 16384L, 32768L}) {
                const PairLaunch base = pair_launch(d, tpl, unr, 1);
                const long tiles = base.target_tiles;
                int chunks = (int)std::max(1L, std::min((long)src_rows, (want + tiles - 1) / tiles));
                int rpc = (src_rows + chunks - 1) / chunks;
                bim_pair_config c{tpl, unr, rpc};
                bool dup = false;
                for (auto &o : cands)
                    dup |= (o.targets_per_lane == tpl && o.unroll == unr && o.rows_per_chunk == rpc);
                if (!dup) cands.push_back(c);
            }
    bim_pair_config pick = cands[0];
    double pick_ms = 1e30;
    for (auto &c : cands) {
        double kms = 0, tms = 0;
        rc = bim_residual_timed(prob, u, F, prec, 3, &c, stream, &kms, &tms);
        if (rc) break;
        if (kms < pick_ms) {
            pick_ms = kms;
            pick = c;
        }
    }
    (void)hipFreeAsync(F, s);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_best[Key(prob->N, prob->M, prob->half_domain ? 1 : 0, prec)] = pick;
    }
    if (best) *best = pick;
    if (best_ms) *best_ms = pick_ms;
    return BIM_OK;
}
