// Lockstep JFNK for a sweep of problems of different sizes (one persistent
// all-pairs launch per round for all of them).
//
// Every round, each unfinished problem needs exactly one residual evaluation:
// its base residual, the inner base for mixed precision, the Jacobian action
// of an Arnoldi step or of a restart, or a line-search trial.  A round is
//   pre-work (batched kernels) -> batched residual(s) -> post-work (batched
//   kernels) -> one copy of every problem's small results to the host -> host
//   Newton/GMRES decisions,
// so the number of kernel launches per round does not grow with the number of
// problems.  Each problem follows the same algorithm as jfnk_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "batch.h"
#include "bim_common.h"
#include "precond.h"
#include "vec.h"

namespace bim {

namespace {

inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

enum Phase { PH_BASE, PH_INNER, PH_ARNOLDI, PH_RESTART, PH_LINESEARCH, PH_DONE };
enum Pending { PD_NONE = 0, PD_GMRES_START = 1, PD_COMBINE = 2, PD_ACCEPT = 4 };


struct Inst {
    const bim_problem *p;
    long n;
    const Precond *pc;
    PairLaunch pl;
    ResidualWork rw;
    double *u, *F, *Fin, *delta, *rhs, *V, *Z, *w, *ut, *Ft, *r, *hdev, *scal, *ydev, *part;
    int phase = PH_BASE;
    int pending = PD_NONE;
    int j = 0, cyc = 0, bt = 0, newton = 0;
    double beta0 = 0, beta = 0, fn2 = 0, finf = 0, mu = 1.0;
    std::vector<double> H, cs, sn, g, y;
    bim_jfnk_report R{};
    bool new_cycle = true;
    bool gm_first = true;
    bool inner64 = true;  // inner precision of the current Newton step (FP64 sums)
};

}  // namespace

int solve_batched_impl(const bim_problem *probs, int count, bim_precond *const *Ps_in, double *const *us,
                       const bim_jfnk_opts *o, bim_jfnk_report *reps, hipStream_t caller) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    int rc = hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
    if (rc) return rc;
    struct StreamGuard {
        hipStream_t s, caller;
        hipEvent_t *ev;
        ~StreamGuard() {
            if (*ev && hipEventRecord(*ev, s) == hipSuccess) (void)hipStreamWaitEvent(caller, *ev, 0);
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
            if (*ev) (void)hipEventDestroy(*ev);
        }
    } sg{s, caller, &ev};
    if ((rc = hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate"))) return rc;
    if ((rc = hip_check(hipEventRecord(ev, caller), "hipEventRecord"))) return rc;
    if ((rc = hip_check(hipStreamWaitEvent(s, ev, 0), "hipStreamWaitEvent"))) return rc;

    const int m = std::max(1, o->restart);
    std::vector<Inst> I(count);
    // preconditioners (caller's or built here)
    std::vector<bim_precond *> own(count, nullptr);
    struct OwnGuard {
        std::vector<bim_precond *> *v;
        ~OwnGuard() {
            for (auto *p : *v)
                if (p) precond_destroy(p);
        }
    } og{&own};
    for (int i = 0; i < count; ++i) {
        double pms = 0.0;
        const bim_precond *P = Ps_in ? Ps_in[i] : nullptr;
        if (!P && o->use_precond) {
            auto tp = std::chrono::steady_clock::now();
            if ((rc = precond_setup_ex(&probs[i], o->band_halfwidth, o->precond_storage, &own[i], s))) return rc;
            pms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp).count();
            P = own[i];
        }
        I[i].pc = o->use_precond ? precond_impl(P) : nullptr;
        I[i].R.precond_ms = pms;
    }
    // one kernel variant for all problems (the largest problem's choice), item sizes balanced
    int big = 0;
    for (int i = 1; i < count; ++i)
        if ((long)probs[i].N * probs[i].M > (long)probs[big].N * probs[big].M) big = i;
    const PairLaunch ref = pair_launch_for(&probs[big], o->inner_prec);
    // memory: per problem residual workspace + Krylov vectors; shared staging
    std::vector<size_t> off(count);
    size_t bytes = 0;
    for (int i = 0; i < count; ++i) {
        const Dims d(&probs[i]);
        I[i].p = &probs[i];
        I[i].n = d.nvec;
        I[i].pl = pair_launch(d, ref.tpl, ref.unroll, balanced_chunks(d, 6 * 181));
        off[i] = bytes;
        bytes += al256(residual_work_bytes(d, I[i].pl));
        const size_t vb = al256(sizeof(double) * d.nvec);
        bytes += vb * ((size_t)(m + 1) + m + 9);
        bytes += al256(sizeof(double) * (size_t)kBRedBlocks * (m + 1)) + al256(sizeof(double) * 3 * (m + 1)) +
                 al256(sizeof(double) * 8) + al256(sizeof(double) * (m + 1));
    }
    const size_t desc_off = bytes;
    bytes += 2 * al256(sizeof(PairDesc) * count);
    const size_t ops_off = bytes;
    const int kOpSlots = 24;
    bytes += al256(sizeof(BOp) * (size_t)count * kOpSlots) + al256(sizeof(BBand) * (size_t)count * 8) +
             al256(sizeof(BGemv) * count);
    const int kSmall = 8 + 3 * (m + 1);  // per problem: scal[8] and the Hessenberg column buffers
    const size_t stage_off = bytes;
    bytes += al256(sizeof(double) * (size_t)count * kSmall);
    void *mem = nullptr;
    if ((rc = hip_check(hipMallocAsync(&mem, bytes, s), "hipMallocAsync(batched jfnk)"))) return rc;
    struct MemGuard {
        void *p;
        hipStream_t s;
        ~MemGuard() {
            if (p) (void)hipFreeAsync(p, s);
        }
    } mg{mem, s};
    double *hstage = nullptr;
    if ((rc = hip_check(hipHostMalloc((void **)&hstage, sizeof(double) * (size_t)count * kSmall), "hipHostMalloc")))
        return rc;
    struct HostGuard {
        double *p;
        ~HostGuard() {
            if (p) (void)hipHostFree(p);
        }
    } hg{hstage};
    for (int i = 0; i < count; ++i) {
        Inst &q = I[i];
        const Dims d(q.p);
        residual_work_carve((char *)mem + off[i], d, q.pl, &q.rw);
        char *c = (char *)mem + off[i] + al256(residual_work_bytes(d, q.pl));
        auto take = [&](size_t b) {
            char *x = c;
            c += al256(b);
            return (double *)x;
        };
        const long n = q.n;
        q.V = take(sizeof(double) * n * (m + 1));
        q.Z = take(sizeof(double) * n * m);
        q.w = take(sizeof(double) * n);
        q.ut = take(sizeof(double) * n);
        q.Ft = take(sizeof(double) * n);
        q.r = take(sizeof(double) * n);
        q.F = take(sizeof(double) * n);
        q.Fin = take(sizeof(double) * n);
        q.delta = take(sizeof(double) * n);
        q.rhs = take(sizeof(double) * n);
        take(sizeof(double) * n);  // spare
        q.part = take(sizeof(double) * (size_t)kBRedBlocks * (m + 1));
        q.hdev = take(sizeof(double) * 3 * (m + 1));
        q.scal = take(sizeof(double) * 8);
        q.ydev = take(sizeof(double) * (m + 1));
        q.u = us[i];
        q.H.assign((size_t)(m + 1) * m, 0.0);
        q.cs.assign(m, 0.0);
        q.sn.assign(m, 0.0);
        q.g.assign(m + 1, 0.0);
        q.y.assign(m, 0.0);
    }
    PairDesc *desc64 = (PairDesc *)((char *)mem + desc_off);
    PairDesc *desc32 = (PairDesc *)((char *)mem + desc_off + al256(sizeof(PairDesc) * count));
    BOp *opdev = (BOp *)((char *)mem + ops_off);
    BBand *banddev = (BBand *)((char *)mem + ops_off + al256(sizeof(BOp) * (size_t)count * kOpSlots));
    BGemv *gemvdev = (BGemv *)((char *)banddev + al256(sizeof(BBand) * (size_t)count * 8));
    double *stage = (double *)((char *)mem + stage_off);

    // host-side op list builder: every batched launch gets its own slice of opdev
    std::vector<BOp> hops;
    std::vector<std::pair<size_t, int>> slices;  // (first, count)
    auto push_ops = [&](const std::vector<BOp> &v) {
        slices.push_back({hops.size(), (int)v.size()});
        hops.insert(hops.end(), v.begin(), v.end());
        return (int)slices.size() - 1;
    };
    const double eps64 = (o->fd_eps > 0) ? o->fd_eps : std::ldexp(1.0, -52);
    const double eps32 = (o->fd_eps > 0) ? o->fd_eps : std::ldexp(1.0, -23);
    const int maxh = (int)(sizeof(I[0].R.history) / sizeof(I[0].R.history[0]));
    int rounds = 0;

    auto finish_inst = [&](Inst &q, int status) {
        q.phase = PH_DONE;
        q.R.status = status;
    };

    for (;;) {
        // ---------------- gather this round's work
        std::vector<int> act;
        for (int i = 0; i < count; ++i)
            if (I[i].phase != PH_DONE) act.push_back(i);
        if (act.empty()) break;
        ++rounds;
        hops.clear();
        slices.clear();
        std::vector<BBand> hband;
        std::vector<BGemv> hgemv;
        // pending actions decided last round
        std::vector<BOp> combine, acc_u, acc_F, gm_zero, gm_rhs, gm_copy_r, gm_beta, gm_v0;
        for (int i : act) {
            Inst &q = I[i];
            if (q.pending & PD_COMBINE) combine.push_back({q.Z, nullptr, q.delta, q.ydev, nullptr, nullptr, q.n, q.n, q.j + 1, 0, 0});
            if (q.pending & PD_ACCEPT) {
                acc_u.push_back({q.ut, nullptr, q.u, nullptr, nullptr, nullptr, q.n, 0, 0, 1.0, 0.0});
                acc_F.push_back({q.Ft, nullptr, q.F, nullptr, nullptr, nullptr, q.n, 0, 0, 1.0, 0.0});
            }
            if (q.pending & PD_GMRES_START) {
                gm_rhs.push_back({q.F, nullptr, q.rhs, nullptr, nullptr, nullptr, q.n, 0, 0, -1.0, 0.0});
                gm_zero.push_back({q.F, nullptr, q.delta, nullptr, nullptr, nullptr, q.n, 0, 0, 0.0, 0.0});
                gm_copy_r.push_back({q.F, nullptr, q.r, nullptr, nullptr, nullptr, q.n, 0, 0, -1.0, 0.0});
                gm_beta.push_back({q.r, q.r, nullptr, nullptr, q.scal + 3, q.part, q.n, 0, 0, 0, 0});
                gm_v0.push_back({q.r, nullptr, q.V, q.scal + 3, nullptr, nullptr, q.n, 0, 0, 0, 0});
            }
        }
        const int sl_comb = push_ops(combine), sl_accu = push_ops(acc_u), sl_accF = push_ops(acc_F);
        const int sl_grhs = push_ops(gm_rhs), sl_gz = push_ops(gm_zero), sl_gr = push_ops(gm_copy_r),
                  sl_gb = push_ops(gm_beta), sl_gv = push_ops(gm_v0);
        // evaluation requests
        std::vector<int> eval64, eval32;  // problem indices
        std::vector<const double *> in64, in32;
        std::vector<double *> out64, out32;
        std::vector<BOp> sh_u, sh_z, sh_shift, sh_axpy, ls_axpby;
        std::vector<int> arn, rst, lsr, bas;
        for (int i : act) {
            Inst &q = I[i];
            const bool inner64 = q.inner64;
            switch (q.phase) {
                case PH_BASE:
                    eval64.push_back(i); in64.push_back(q.u); out64.push_back(q.F); bas.push_back(i);
                    break;
                case PH_INNER:
                    eval32.push_back(i); in32.push_back(q.u); out32.push_back(q.Fin);
                    break;
                case PH_ARNOLDI:
                case PH_RESTART: {
                    double *z = (q.phase == PH_ARNOLDI) ? q.Z + (size_t)q.j * q.n : q.delta;
                    if (q.phase == PH_ARNOLDI) {
                        const double *v = q.V + (size_t)q.j * q.n;
                        if (q.pc) {
                            const Precond *pc = q.pc;
                            const long nn = pc->n;
                            double *a1 = pc->scratch, *a3 = a1 + nn, *t2 = a3 + nn, *t3 = t2 + nn;
                            const double *r1 = v, *r2 = v + nn, *r3 = v + 2 * nn;
                            double *z1 = z, *z2 = z + nn, *z3 = z + 2 * nn;
                            const int M = pc->M, ss = pc->s, h = pc->h;
                            const int f = pc->storage == BIM_STORE_FP32;
                            auto arr = [&](int which) { return precond_array(pc, which); };
                            hband.push_back({arr(0), r1, nullptr, a1, M, 0, ss, 1.0, 0.0, f});   // Dinv11
                            hband.push_back({arr(5), a1, r3, t3, M, h, ss, -1.0, 1.0, f});       // B31
                            hband.push_back({arr(1), t3, nullptr, a3, M, 0, ss, 1.0, 0.0, f});   // Dinv22
                            hband.push_back({arr(3), a1, r2, t2, M, h, ss, -1.0, 1.0, f});       // B21
                            hband.push_back({arr(4), a3, t2, t2, M, h, ss, -1.0, 1.0, f});       // B23
                            hgemv.push_back({arr(7), t2, nullptr, z2, nn, (int)nn, (int)nn, 1.0, 0.0, f});  // S^-1
                            hband.push_back({arr(6), z2, a3, z3, M, h, ss, -1.0, 1.0, f});       // G
                            hband.push_back({arr(2), z2, a1, z1, M, 0, ss, -1.0, 1.0, f});       // E
                        } else {
                            ls_axpby.push_back({v, nullptr, z, nullptr, nullptr, nullptr, q.n, 0, 0, 1.0, 0.0});
                        }
                        arn.push_back(i);
                    } else {
                        rst.push_back(i);
                    }
                    sh_u.push_back({q.u, q.u, nullptr, nullptr, q.scal + 0, q.part, q.n, 0, 0, 0, 0});
                    sh_z.push_back({z, z, nullptr, nullptr, q.scal + 1, q.part + kBRedBlocks, q.n, 0, 0, 0, 0});
                    sh_shift.push_back({nullptr, nullptr, nullptr, nullptr, q.scal, nullptr, 0, 0, 0, 0.0,
                                        inner64 ? eps64 : eps32});
                    sh_axpy.push_back({q.u, z, q.ut, q.scal + 2, nullptr, nullptr, q.n, 0, 0, 0, 0});
                    if (inner64) { eval64.push_back(i); in64.push_back(q.ut); out64.push_back(q.Ft); }
                    else { eval32.push_back(i); in32.push_back(q.ut); out32.push_back(q.Ft); }
                    break;
                }
                case PH_LINESEARCH:
                    ls_axpby.push_back({q.u, q.delta, q.ut, nullptr, nullptr, nullptr, q.n, 0, 0, 1.0, q.mu});
                    eval64.push_back(i); in64.push_back(q.ut); out64.push_back(q.Ft); lsr.push_back(i);
                    break;
            }
        }
        const int sl_shu = push_ops(sh_u), sl_shz = push_ops(sh_z), sl_shift = push_ops(sh_shift),
                  sl_axpy = push_ops(sh_axpy), sl_ls = push_ops(ls_axpby);
        // post-work descriptors
        std::vector<BOp> quo, md1, or1, md2, or2, wn, vn, rs_r, rs_b, rs_v, nF2, nFi;
        int max_nv = 1;
        for (int i : arn) {
            Inst &q = I[i];
            const double *Fb = q.inner64 ? q.F : q.Fin;
            quo.push_back({q.Ft, Fb, q.w, q.scal + 2, nullptr, nullptr, q.n, 0, 0, 0, 0});
            md1.push_back({q.V, q.w, nullptr, nullptr, q.hdev, q.part, q.n, q.n, q.j + 1, 0, 0});
            or1.push_back({q.V, nullptr, q.w, q.hdev, nullptr, nullptr, q.n, q.n, q.j + 1, 0, 0});
            md2.push_back({q.V, q.w, nullptr, nullptr, q.hdev + m + 1, q.part, q.n, q.n, q.j + 1, 0, 0});
            or2.push_back({q.V, nullptr, q.w, q.hdev + m + 1, nullptr, nullptr, q.n, q.n, q.j + 1, 0, 0});
            wn.push_back({q.w, q.w, nullptr, nullptr, q.hdev + 2 * (m + 1), q.part, q.n, 0, 0, 0, 0});
            vn.push_back({q.w, nullptr, q.V + (size_t)(q.j + 1) * q.n, q.hdev + 2 * (m + 1), nullptr, nullptr, q.n, 0, 0, 0, 0});
            max_nv = std::max(max_nv, q.j + 1);
        }
        for (int i : rst) {
            Inst &q = I[i];
            const double *Fb = q.inner64 ? q.F : q.Fin;
            quo.push_back({q.Ft, Fb, q.w, q.scal + 2, nullptr, nullptr, q.n, 0, 0, 0, 0});
            rs_r.push_back({q.rhs, q.w, q.r, nullptr, nullptr, nullptr, q.n, 0, 0, 1.0, -1.0});
            rs_b.push_back({q.r, q.r, nullptr, nullptr, q.scal + 3, q.part, q.n, 0, 0, 0, 0});
            rs_v.push_back({q.r, nullptr, q.V, q.scal + 3, nullptr, nullptr, q.n, 0, 0, 0, 0});
        }
        for (int i : bas) {
            Inst &q = I[i];
            nF2.push_back({q.F, q.F, nullptr, nullptr, q.scal + 4, q.part, q.n, 0, 0, 0, 0});
            nFi.push_back({q.F, nullptr, nullptr, nullptr, q.scal + 5, q.part + 2 * kBRedBlocks, q.n, 0, 0, 0, 0});
        }
        for (int i : lsr) {
            Inst &q = I[i];
            nF2.push_back({q.Ft, q.Ft, nullptr, nullptr, q.scal + 4, q.part, q.n, 0, 0, 0, 0});
            nFi.push_back({q.Ft, nullptr, nullptr, nullptr, q.scal + 5, q.part + 2 * kBRedBlocks, q.n, 0, 0, 0, 0});
        }
        const int sl_quo = push_ops(quo), sl_md1 = push_ops(md1), sl_or1 = push_ops(or1), sl_md2 = push_ops(md2),
                  sl_or2 = push_ops(or2), sl_wn = push_ops(wn), sl_vn = push_ops(vn), sl_rsr = push_ops(rs_r),
                  sl_rsb = push_ops(rs_b), sl_rsv = push_ops(rs_v), sl_nF2 = push_ops(nF2), sl_nFi = push_ops(nFi);
        if (hops.size() > (size_t)count * kOpSlots) return fail(BIM_EINVAL, "internal: batched op buffer too small");
        if ((rc = hip_check(hipMemcpyAsync(opdev, hops.data(), sizeof(BOp) * hops.size(), hipMemcpyHostToDevice, s),
                            "copy")))
            return rc;
        if (!hgemv.empty() &&
            (rc = hip_check(hipMemcpyAsync(gemvdev, hgemv.data(), sizeof(BGemv) * hgemv.size(), hipMemcpyHostToDevice, s),
                            "copy")))
            return rc;
        auto S = [&](int k) { return opdev + slices[k].first; };
        auto C = [&](int k) { return slices[k].second; };
        // y coefficients for the combines
        for (int i : act) {
            Inst &q = I[i];
            if (q.pending & PD_COMBINE)
                if ((rc = hip_check(hipMemcpyAsync(q.ydev, q.y.data(), sizeof(double) * (q.j + 1), hipMemcpyHostToDevice, s), "copy")))
                    return rc;
        }
        // ---------------- pre-work
        if ((rc = b_combine(S(sl_comb), C(sl_comb), s))) return rc;
        if ((rc = b_axpby(S(sl_accu), C(sl_accu), s))) return rc;
        if ((rc = b_axpby(S(sl_accF), C(sl_accF), s))) return rc;
        if ((rc = b_axpby(S(sl_grhs), C(sl_grhs), s))) return rc;
        if ((rc = b_axpby(S(sl_gz), C(sl_gz), s))) return rc;
        if ((rc = b_axpby(S(sl_gr), C(sl_gr), s))) return rc;
        if ((rc = b_dot(S(sl_gb), C(sl_gb), true, s))) return rc;
        if ((rc = b_scale_inv(S(sl_gv), C(sl_gv), s))) return rc;
        // preconditioner applies, in the order of precond_apply_enqueue: hband holds 7 banded
        // products per problem (5 before the dense Schur product, 2 after); gather them stage by stage
        if (!hgemv.empty()) {
            const int napp = (int)hgemv.size(), per = 7;
            int max_rows = 0, max_groups = 0;
            for (int a = 0; a < napp; ++a) max_rows = std::max(max_rows, hgemv[a].rows);
            for (const BBand &bb : hband) max_groups = std::max(max_groups, bb.M * ((bb.s + 3) / 4));
            std::vector<BBand> gathered;
            gathered.reserve((size_t)napp * per);
            for (int stg = 0; stg < per; ++stg)
                for (int a = 0; a < napp; ++a) gathered.push_back(hband[(size_t)a * per + stg]);
            if ((rc = hip_check(hipMemcpyAsync(banddev, gathered.data(), sizeof(BBand) * gathered.size(),
                                               hipMemcpyHostToDevice, s), "copy")))
                return rc;
            for (int stg = 0; stg < 5; ++stg)
                if ((rc = b_bandmv(banddev + (size_t)stg * napp, napp, max_groups, s))) return rc;
            if ((rc = b_gemv(gemvdev, napp, max_rows, s))) return rc;
            for (int stg = 5; stg < per; ++stg)
                if ((rc = b_bandmv(banddev + (size_t)stg * napp, napp, max_groups, s))) return rc;
        }
        if ((rc = b_axpby(S(sl_ls), C(sl_ls), s))) return rc;  // unpreconditioned copies and line-search points
        if ((rc = b_dot(S(sl_shu), C(sl_shu), true, s))) return rc;
        if ((rc = b_dot(S(sl_shz), C(sl_shz), true, s))) return rc;
        if ((rc = b_shift(S(sl_shift), C(sl_shift), s))) return rc;
        if ((rc = b_axpy_dev(S(sl_axpy), C(sl_axpy), s))) return rc;
        // ---------------- batched residuals (one persistent all-pairs launch per precision)
        auto run_eval = [&](const std::vector<int> &idx, const std::vector<const double *> &in,
                            const std::vector<double *> &out, int prec, PairDesc *descs) -> int {
            if (idx.empty()) return BIM_OK;
            std::vector<bim_problem> pp;
            std::vector<PairLaunch> pls;
            std::vector<ResidualWork> ws;
            for (int i : idx) {
                pp.push_back(*I[i].p);
                pls.push_back(I[i].pl);
                ws.push_back(I[i].rw);
            }
            return residual_batched_enqueue(pp.data(), (int)idx.size(), in.data(), out.data(), prec, pls.data(),
                                            ws.data(), descs, 0, s);
        };
        // FP64 and FP32C groups use separate workspaces? They never share a problem in one round.
        if ((rc = run_eval(eval64, in64, out64, BIM_FP64, desc64))) return rc;
        if ((rc = run_eval(eval32, in32, out32, BIM_FP32C, desc32))) return rc;
        // ---------------- post-work
        if ((rc = b_quotient(S(sl_quo), C(sl_quo), s))) return rc;
        if ((rc = b_multidot(S(sl_md1), C(sl_md1), max_nv, s))) return rc;
        if ((rc = b_orth(S(sl_or1), C(sl_or1), s))) return rc;
        if ((rc = b_multidot(S(sl_md2), C(sl_md2), max_nv, s))) return rc;
        if ((rc = b_orth(S(sl_or2), C(sl_or2), s))) return rc;
        if ((rc = b_dot(S(sl_wn), C(sl_wn), true, s))) return rc;
        if ((rc = b_scale_inv(S(sl_vn), C(sl_vn), s))) return rc;
        if ((rc = b_axpby(S(sl_rsr), C(sl_rsr), s))) return rc;
        if ((rc = b_dot(S(sl_rsb), C(sl_rsb), true, s))) return rc;
        if ((rc = b_scale_inv(S(sl_rsv), C(sl_rsv), s))) return rc;
        if ((rc = b_dot(S(sl_nF2), C(sl_nF2), true, s))) return rc;
        if ((rc = b_maxabs(S(sl_nFi), C(sl_nFi), s))) return rc;
        // small results of every problem -> one pinned host copy
        {
            std::vector<BOp> gat;
            for (int i : act)
                gat.push_back({I[i].scal, I[i].hdev, stage + (size_t)i * kSmall, nullptr, nullptr, nullptr, 0, 0,
                               3 * (m + 1), 0, 0});
            BOp *gdev = opdev + hops.size();
            if (hops.size() + gat.size() > (size_t)count * kOpSlots)
                return fail(BIM_EINVAL, "internal: batched op buffer too small");
            if ((rc = hip_check(hipMemcpyAsync(gdev, gat.data(), sizeof(BOp) * gat.size(), hipMemcpyHostToDevice, s),
                                "copy")))
                return rc;
            if ((rc = b_gather(gdev, (int)gat.size(), s))) return rc;
            if ((rc = hip_check(hipMemcpyAsync(hstage, stage, sizeof(double) * (size_t)count * kSmall,
                                               hipMemcpyDeviceToHost, s), "copy")))
                return rc;
            if ((rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
        }
        // ---------------- host decisions
        for (int i : act) {
            Inst &q = I[i];
            const double *hs = hstage + (size_t)i * kSmall;
            q.pending = PD_NONE;
            auto start_newton_step = [&]() {
                // F, fn2, finf current
                const int k = q.newton;
                if (k < maxh) q.R.history[k] = q.finf;
                q.R.fnorm_inf = q.finf;
                q.R.newton_iters = k;
                if (!std::isfinite(q.fn2)) { fail(BIM_EDOMAIN, "non-finite residual"); finish_inst(q, BIM_EDOMAIN); return; }
                if (q.finf <= o->ftol) { finish_inst(q, BIM_OK); return; }
                if (k >= o->max_newton) { finish_inst(q, BIM_NOT_CONVERGED); return; }
                if (o->stall_steps > 0 && k >= o->stall_steps && k < maxh &&
                    q.finf > 0.5 * q.R.history[k - o->stall_steps]) {
                    finish_inst(q, BIM_NOT_CONVERGED);
                    return;
                }
                // FP32C inner sums, or FP64 ones once ||F||_inf <= fp64_below
                q.inner64 = (o->inner_prec == BIM_FP64) || (q.finf <= o->fp64_below);
                q.phase = q.inner64 ? PH_ARNOLDI : PH_INNER;
                q.pending |= PD_GMRES_START;
                q.j = 0;
                q.cyc = 0;
                q.gm_first = true;
                q.new_cycle = true;
            };
            switch (q.phase) {
                case PH_BASE:
                    q.fn2 = hs[4];
                    q.finf = hs[5];
                    q.R.fnorm0_inf = q.finf;
                    ++q.R.residual_evals;
                    start_newton_step();
                    break;
                case PH_INNER:
                    ++q.R.inner_residual_evals;
                    // the GMRES start was enqueued with the inner evaluation; Arnoldi next
                    q.phase = PH_ARNOLDI;
                    break;
                case PH_ARNOLDI: {
                    ++q.R.jv_evals;
                    ++q.R.gmres_iters;
                    if (q.new_cycle) {
                        q.beta = hs[3];
                        if (q.gm_first) q.beta0 = q.beta;
                        std::fill(q.g.begin(), q.g.end(), 0.0);
                        q.g[0] = q.beta;
                        q.new_cycle = false;
                        q.gm_first = false;
                    }
                    const double *hcol = hs + 8;
                    const int jj = q.j;
                    double *col = &q.H[(size_t)jj];
                    for (int a = 0; a <= jj; ++a) col[(size_t)a * m] = hcol[a] + hcol[m + 1 + a];
                    const double hn = hcol[2 * (m + 1)];
                    col[(size_t)(jj + 1) * m] = hn;
                    if (!std::isfinite(hn) || !(q.beta0 > 0.0)) {
                        if (!(q.beta0 > 0.0) && std::isfinite(q.beta0)) {  // zero right-hand side: nothing to do
                            q.phase = PH_LINESEARCH; q.mu = 1.0; q.bt = 0; break;
                        }
                        finish_inst(q, BIM_EDOMAIN);
                        break;
                    }
                    for (int a = 0; a < jj; ++a) {
                        const double x = col[(size_t)a * m], yv = col[(size_t)(a + 1) * m];
                        col[(size_t)a * m] = q.cs[a] * x + q.sn[a] * yv;
                        col[(size_t)(a + 1) * m] = -q.sn[a] * x + q.cs[a] * yv;
                    }
                    const double x = col[(size_t)jj * m], yv = col[(size_t)(jj + 1) * m];
                    const double rr = std::hypot(x, yv);
                    q.cs[jj] = rr > 0 ? x / rr : 1.0;
                    q.sn[jj] = rr > 0 ? yv / rr : 0.0;
                    col[(size_t)jj * m] = rr;
                    col[(size_t)(jj + 1) * m] = 0.0;
                    q.g[jj + 1] = -q.sn[jj] * q.g[jj];
                    q.g[jj] = q.cs[jj] * q.g[jj];
                    const double relres = std::fabs(q.g[jj + 1]) / q.beta0;
                    q.R.gmres_relres_last = relres;
                    const double rtol_q = q.inner64 ? o->gmres_rtol : std::max(o->gmres_rtol, o->fp32c_gmres_rtol);
                    const bool conv = relres <= rtol_q || hn == 0.0;
                    if (conv || jj == m - 1) {
                        const int jend = jj + 1;
                        for (int a = jend - 1; a >= 0; --a) {
                            double v = q.g[a];
                            for (int b = a + 1; b < jend; ++b) v -= q.H[(size_t)a * m + b] * q.y[b];
                            q.y[a] = v / q.H[(size_t)a * m + a];
                        }
                        q.pending |= PD_COMBINE;  // delta += Z y at the start of the next round
                        if (conv || q.cyc >= o->max_restarts) {
                            q.phase = PH_LINESEARCH;
                            q.mu = 1.0;
                            q.bt = 0;
                        } else {
                            q.phase = PH_RESTART;
                        }
                    } else {
                        q.j = jj + 1;
                    }
                    break;
                }
                case PH_RESTART: {
                    ++q.R.jv_evals;
                    q.beta = hs[3];
                    const double relres = q.beta / q.beta0;
                    q.R.gmres_relres_last = relres;
                    if (relres <= (q.inner64 ? o->gmres_rtol : std::max(o->gmres_rtol, o->fp32c_gmres_rtol))) {
                        q.phase = PH_LINESEARCH;
                        q.mu = 1.0;
                        q.bt = 0;
                    } else {
                        ++q.cyc;
                        q.j = 0;
                        q.phase = PH_ARNOLDI;
                        std::fill(q.g.begin(), q.g.end(), 0.0);
                        q.g[0] = q.beta;  // v0 = r / beta was formed on the device
                    }
                    break;
                }
                case PH_LINESEARCH: {
                    ++q.R.residual_evals;
                    const double tn2 = hs[4], tinf = hs[5];
                    if (std::isfinite(tn2) && tn2 <= (1.0 - 1e-4 * q.mu) * q.fn2) {
                        q.fn2 = tn2;
                        q.finf = tinf;
                        q.pending |= PD_ACCEPT;
                        ++q.newton;
                        const int keep = q.pending;
                        start_newton_step();
                        q.pending |= keep;
                    } else {
                        ++q.R.backtracks;
                        q.mu *= 0.5;
                        if (++q.bt > o->max_backtracks) finish_inst(q, BIM_LINESEARCH_FAIL);
                    }
                    break;
                }
                default:
                    break;
            }
        }
    }
    // make sure every accepted step was applied (the last round's pending copies)
    {
        std::vector<BOp> acc_u;
        for (int i = 0; i < count; ++i)
            if (I[i].pending & PD_ACCEPT)
                acc_u.push_back({I[i].ut, nullptr, I[i].u, nullptr, nullptr, nullptr, I[i].n, 0, 0, 1.0, 0.0});
        if (!acc_u.empty()) {
            if ((rc = hip_check(hipMemcpyAsync(opdev, acc_u.data(), sizeof(BOp) * acc_u.size(), hipMemcpyHostToDevice, s),
                                "copy")))
                return rc;
            if ((rc = b_axpby(opdev, (int)acc_u.size(), s))) return rc;
        }
        if ((rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
    }
    const double tot = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst_err = 0, worst_soft = 0;
    for (int i = 0; i < count; ++i) {
        I[i].R.time_ms = tot;
        if (reps) reps[i] = I[i].R;
        worst_err = std::min(worst_err, I[i].R.status);
        worst_soft = std::max(worst_soft, I[i].R.status);
    }
    const int worst = worst_err < 0 ? worst_err : worst_soft;
    (void)rounds;
    return worst;
}

}  // namespace bim

using namespace bim;

extern "C" int jfnk_solve_batched(const bim_problem *probs, int count, bim_precond *const *Ps, double *const *us,
                                  const bim_jfnk_opts *opts, bim_jfnk_report *reps, void *stream) {
    if (count < 0 || (count > 0 && (!probs || !us))) return fail(BIM_EINVAL, "bad batch arguments");
    if (count == 0) return BIM_OK;
    int rc;
    for (int i = 0; i < count; ++i) {
        if ((rc = validate(&probs[i]))) return rc;
        if (!us[i]) return fail(BIM_EINVAL, "u[i] must be a device pointer");
    }
    bim_jfnk_opts o;
    jfnk_default_opts(&o);
    if (opts) o = *opts;
    if (!(o.ftol > 0) || !(o.gmres_rtol > 0) || o.restart < 1 || o.restart > 30 || o.max_restarts < 0 ||
        o.max_newton < 0 || o.max_backtracks < 0 || !(o.fd_eps < 1.0) || o.stall_steps < 0 ||
        !(o.fp64_below >= 0.0) || (o.inner_prec != BIM_FP64 && o.inner_prec != BIM_FP32C) ||
        (o.precond_storage != BIM_STORE_FP64 && o.precond_storage != BIM_STORE_FP32))
        return fail(BIM_EINVAL, "invalid solver options (batched restart must be <= 30)");
    return solve_batched_impl(probs, count, Ps, us, &o, reps, (hipStream_t)stream);
}
