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
#include <cstring>
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
// Op lists of a round, in launch order (one slot per problem in each).
enum Slice {
    S_COMB, S_ACCU, S_ACCF, S_GRHS, S_GZ, S_GR, S_GB, S_GV,          // pre-work
    S_LS, S_SHU, S_SHZ, S_SHIFT, S_AXPY,                               // inputs of the evaluations
    S_QUO, S_MD1, S_OR1, S_MD2, S_OR2, S_WN, S_VN, S_RSR, S_RSB, S_RSV,  // Arnoldi and restart post-work
    S_NF2, S_NFI, S_GATHER, S_COUNT                                    // norms, results to the host
};
constexpr int kPcStages = 8;  // banded products of one preconditioner apply (plus its two triangular ones)
enum Pending { PD_NONE = 0, PD_GMRES_START = 1, PD_COMBINE = 2, PD_ACCEPT = 4 };


struct Inst {
    const bim_problem *p;
    long n;
    const Precond *pc;
    PairLaunch pl;
    ResidualWork rw;
    double *u, *F, *Fin, *delta, *rhs, *V, *Z, *w, *ut, *Ft, *r, *hdev, *scal, *part;
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
                 al256(sizeof(double) * 8);
    }
    // the round block: every descriptor of a round (op lists padded to one slot
    // per problem, preconditioner stages, pair descriptors of both precision
    // groups, GMRES combination coefficients), laid out identically in pinned
    // host memory and in device memory and moved by one copy per round
    const size_t rb_ops = 0;
    const size_t rb_bands = rb_ops + al256(sizeof(BOp) * (size_t)S_COUNT * count);
    const size_t rb_gemv = rb_bands + al256(sizeof(BBand) * (size_t)kPcStages * count);
    const size_t rb_d64 = rb_gemv + al256(sizeof(BGemv) * 2 * (size_t)count);
    const size_t rb_d32 = rb_d64 + al256(sizeof(PairDesc) * count);
    const size_t rb_y = rb_d32 + al256(sizeof(PairDesc) * count);
    const size_t rb_bytes = rb_y + al256(sizeof(double) * (size_t)count * m);
    const size_t round_off = bytes;
    bytes += rb_bytes;
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
    char *hround = nullptr;
    if ((rc = hip_check(hipHostMalloc((void **)&hstage, sizeof(double) * (size_t)count * kSmall), "hipHostMalloc")))
        return rc;
    struct HostGuard {
        void *p;
        ~HostGuard() {
            if (p) (void)hipHostFree(p);
        }
    } hg{hstage};
    if ((rc = hip_check(hipHostMalloc((void **)&hround, rb_bytes), "hipHostMalloc"))) return rc;
    HostGuard hg2{hround};
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
        q.u = us[i];
        q.H.assign((size_t)(m + 1) * m, 0.0);
        q.cs.assign(m, 0.0);
        q.sn.assign(m, 0.0);
        q.g.assign(m + 1, 0.0);
        q.y.assign(m, 0.0);
    }
    char *dround = (char *)mem + round_off;
    double *stage = (double *)((char *)mem + stage_off);
    BOp *const hops = (BOp *)(hround + rb_ops);
    BBand *const hbands = (BBand *)(hround + rb_bands);
    BGemv *const hgemv = (BGemv *)(hround + rb_gemv);
    PairDesc *const hd64 = (PairDesc *)(hround + rb_d64);
    PairDesc *const hd32 = (PairDesc *)(hround + rb_d32);
    double *const hy = (double *)(hround + rb_y);
    BOp *const dops = (BOp *)(dround + rb_ops);
    BBand *const dbands = (BBand *)(dround + rb_bands);
    BGemv *const dgemv = (BGemv *)(dround + rb_gemv);
    const PairDesc *const dd64 = (const PairDesc *)(dround + rb_d64);
    const PairDesc *const dd32 = (const PairDesc *)(dround + rb_d32);
    const double *const dy = (const double *)(dround + rb_y);
    const double eps64 = (o->fd_eps > 0) ? o->fd_eps : std::ldexp(1.0, -52);
    const double eps32 = (o->fd_eps > 0) ? o->fd_eps : std::ldexp(1.0, -23);
    const int maxh = (int)(sizeof(I[0].R.history) / sizeof(I[0].R.history[0]));
    int rounds = 0, graph_captures = 0;

    // fixed launch shapes of a round, sized for every problem taking part
    std::vector<PairLaunch> pls(count);
    std::vector<ResidualWork> rws(count);
    for (int i = 0; i < count; ++i) {
        pls[i] = I[i].pl;
        rws[i] = I[i].rw;
    }
    const BatchShape shape = residual_batched_shape(probs, count, pls.data(), 0);
    const bool has32 = o->inner_prec == BIM_FP32C;
    int max_groups = 0;
    bool has_pc = false;
    for (int i = 0; i < count; ++i)
        if (I[i].pc) {
            has_pc = true;
            max_groups = std::max(max_groups, I[i].pc->M * ((I[i].pc->s + 3) / 4));
        }
    auto OPS = [&](int slice) { return dops + (size_t)slice * count; };

    // The device work of one round, in a fixed sequence of launches whose shapes
    // do not depend on the round: every op list has one slot per problem (empty
    // slots do nothing) and the residuals cover all problems (inactive ones do
    // nothing).  With use_graphs it is captured once and replayed every round.
    auto enqueue_round = [&]() -> int {
        int q;
        if ((q = hip_check(hipMemcpyAsync(dround, hround, rb_bytes, hipMemcpyHostToDevice, s), "copy"))) return q;
        // pre-work: pending GMRES combinations, accepted steps, GMRES starts
        if ((q = b_combine(OPS(S_COMB), count, s))) return q;
        if ((q = b_axpby(OPS(S_ACCU), count, s))) return q;
        if ((q = b_axpby(OPS(S_ACCF), count, s))) return q;
        if ((q = b_axpby(OPS(S_GRHS), count, s))) return q;
        if ((q = b_axpby(OPS(S_GZ), count, s))) return q;
        if ((q = b_axpby(OPS(S_GR), count, s))) return q;
        if ((q = b_dot(OPS(S_GB), count, true, s))) return q;
        if ((q = b_scale_inv(OPS(S_GV), count, s))) return q;
        // preconditioner applies, stage by stage in the order of precond_apply_enqueue:
        // five banded products, the Schur inverse (lower triangular product,
        // block-diagonal product, upper triangular product), two banded products
        if (has_pc) {
            for (int stg = 0; stg < 5; ++stg)
                if ((q = b_bandmv(dbands + (size_t)stg * count, count, max_groups, s))) return q;
            if ((q = b_gemv_tri(dgemv, count, max_groups, s))) return q;
            if ((q = b_bandmv(dbands + (size_t)5 * count, count, max_groups, s))) return q;
            if ((q = b_gemv_tri(dgemv + count, count, max_groups, s))) return q;
            for (int stg = 6; stg < kPcStages; ++stg)
                if ((q = b_bandmv(dbands + (size_t)stg * count, count, max_groups, s))) return q;
        }
        if ((q = b_axpby(OPS(S_LS), count, s))) return q;  // unpreconditioned copies and line-search points
        if ((q = b_dot(OPS(S_SHU), count, true, s))) return q;
        if ((q = b_dot(OPS(S_SHZ), count, true, s))) return q;
        if ((q = b_shift(OPS(S_SHIFT), count, s))) return q;
        if ((q = b_axpy_dev(OPS(S_AXPY), count, s))) return q;
        // residuals: one persistent all-pairs launch per precision group
        if ((q = residual_batched_launch(dd64, count, BIM_FP64, shape, s))) return q;
        if (has32 && (q = residual_batched_launch(dd32, count, BIM_FP32C, shape, s))) return q;
        // post-work: difference quotients, two CGS passes, norms, restarts, residual norms
        if ((q = b_quotient(OPS(S_QUO), count, s))) return q;
        if ((q = b_multidot(OPS(S_MD1), count, m, s))) return q;
        if ((q = b_orth(OPS(S_OR1), count, s))) return q;
        if ((q = b_multidot(OPS(S_MD2), count, m, s))) return q;
        if ((q = b_orth(OPS(S_OR2), count, s))) return q;
        if ((q = b_dot(OPS(S_WN), count, true, s))) return q;
        if ((q = b_scale_inv(OPS(S_VN), count, s))) return q;
        if ((q = b_axpby(OPS(S_RSR), count, s))) return q;
        if ((q = b_dot(OPS(S_RSB), count, true, s))) return q;
        if ((q = b_scale_inv(OPS(S_RSV), count, s))) return q;
        if ((q = b_dot(OPS(S_NF2), count, true, s))) return q;
        if ((q = b_maxabs(OPS(S_NFI), count, s))) return q;
        // small results of every problem -> one pinned host copy
        if ((q = b_gather(OPS(S_GATHER), count, s))) return q;
        return hip_check(hipMemcpyAsync(hstage, stage, sizeof(double) * (size_t)count * kSmall,
                                        hipMemcpyDeviceToHost, s), "copy");
    };
    hipGraphExec_t round_graph = nullptr;
    struct GraphGuard {
        hipGraphExec_t *g;
        ~GraphGuard() {
            if (*g) (void)hipGraphExecDestroy(*g);
        }
    } gg{&round_graph};
    auto run_round = [&]() -> int {
        int q;
        if (!o->use_graphs) {
            if ((q = enqueue_round())) return q;
        } else {
            if (!round_graph) {
                if ((q = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture")))
                    return q;
                const int q_work = enqueue_round();
                hipGraph_t g = nullptr;
                q = hip_check(hipStreamEndCapture(s, &g), "hipStreamEndCapture");
                if (q_work || q) {
                    if (g) (void)hipGraphDestroy(g);
                    return q_work ? q_work : q;
                }
                q = hip_check(hipGraphInstantiate(&round_graph, g, nullptr, nullptr, 0), "hipGraphInstantiate");
                (void)hipGraphDestroy(g);
                if (q) return q;
                ++graph_captures;
            }
            if ((q = hip_check(hipGraphLaunch(round_graph, s), "hipGraphLaunch"))) return q;
        }
        return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    };

    auto finish_inst = [&](Inst &q, int status) {
        q.phase = PH_DONE;
        q.R.status = status;
    };
    std::vector<int> on64(count), on32(count);
    std::vector<const double *> in64(count), in32(count);
    std::vector<double *> out64(count), out32(count);

    for (;;) {
        // ---------------- gather this round's work
        std::vector<int> act;
        for (int i = 0; i < count; ++i)
            if (I[i].phase != PH_DONE) act.push_back(i);
        if (act.empty()) break;
        ++rounds;
        std::memset(hround, 0, rb_bytes);  // every slot empty
        auto put = [&](int slice, int i, const BOp &op) { hops[(size_t)slice * count + i] = op; };
        std::fill(on64.begin(), on64.end(), 0);
        std::fill(on32.begin(), on32.end(), 0);
        std::fill(in64.begin(), in64.end(), nullptr);
        std::fill(in32.begin(), in32.end(), nullptr);
        std::fill(out64.begin(), out64.end(), nullptr);
        std::fill(out32.begin(), out32.end(), nullptr);
        // pending actions decided last round
        for (int i : act) {
            Inst &q = I[i];
            if (q.pending & PD_COMBINE) {
                std::copy(q.y.begin(), q.y.begin() + (q.j + 1), hy + (size_t)i * m);
                put(S_COMB, i, {q.Z, nullptr, q.delta, dy + (size_t)i * m, nullptr, nullptr, q.n, q.n, q.j + 1, 0, 0});
            }
            if (q.pending & PD_ACCEPT) {
                put(S_ACCU, i, {q.ut, nullptr, q.u, nullptr, nullptr, nullptr, q.n, 0, 0, 1.0, 0.0});
                put(S_ACCF, i, {q.Ft, nullptr, q.F, nullptr, nullptr, nullptr, q.n, 0, 0, 1.0, 0.0});
            }
            if (q.pending & PD_GMRES_START) {
                put(S_GRHS, i, {q.F, nullptr, q.rhs, nullptr, nullptr, nullptr, q.n, 0, 0, -1.0, 0.0});
                put(S_GZ, i, {q.F, nullptr, q.delta, nullptr, nullptr, nullptr, q.n, 0, 0, 0.0, 0.0});
                put(S_GR, i, {q.F, nullptr, q.r, nullptr, nullptr, nullptr, q.n, 0, 0, -1.0, 0.0});
                put(S_GB, i, {q.r, q.r, nullptr, nullptr, q.scal + 3, q.part, q.n, 0, 0, 0, 0});
                put(S_GV, i, {q.r, nullptr, q.V, q.scal + 3, nullptr, nullptr, q.n, 0, 0, 0, 0});
            }
        }
        // evaluation requests
        std::vector<int> arn, rst, lsr, bas;
        for (int i : act) {
            Inst &q = I[i];
            const bool inner64 = q.inner64;
            switch (q.phase) {
                case PH_BASE:
                    on64[i] = 1; in64[i] = q.u; out64[i] = q.F; bas.push_back(i);
                    break;
                case PH_INNER:
                    on32[i] = 1; in32[i] = q.u; out32[i] = q.Fin;
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
                            BBand *b = hbands + i;
                            const size_t st = count;
                            b[0 * st] = {arr(0), r1, nullptr, a1, M, 0, ss, 1.0, 0.0, f};   // Dinv11
                            b[1 * st] = {arr(5), a1, r3, t3, M, h, ss, -1.0, 1.0, f};       // B31
                            b[2 * st] = {arr(1), t3, nullptr, a3, M, 0, ss, 1.0, 0.0, f};   // Dinv22
                            b[3 * st] = {arr(3), a1, r2, t2, M, h, ss, -1.0, 1.0, f};       // B21
                            b[4 * st] = {arr(4), a3, t2, t2, M, h, ss, -1.0, 1.0, f};       // B23
                            hgemv[i] = {arr(7), t2, t2, t3, nn, M, ss, 1, 1.0, 1.0, f};           // L^-1
                            b[5 * st] = {arr(8), t3, nullptr, t2, M, 0, ss, 1.0, 0.0, f};   // D^-1
                            hgemv[st + i] = {arr(7), t2, t2, z2, nn, M, ss, 2, 1.0, 1.0, f};      // V^-1
                            b[6 * st] = {arr(6), z2, a3, z3, M, h, ss, -1.0, 1.0, f};       // G
                            b[7 * st] = {arr(2), z2, a1, z1, M, 0, ss, -1.0, 1.0, f};       // E
                        } else {
                            put(S_LS, i, {v, nullptr, z, nullptr, nullptr, nullptr, q.n, 0, 0, 1.0, 0.0});
                        }
                        arn.push_back(i);
                    } else {
                        rst.push_back(i);
                    }
                    put(S_SHU, i, {q.u, q.u, nullptr, nullptr, q.scal + 0, q.part, q.n, 0, 0, 0, 0});
                    put(S_SHZ, i, {z, z, nullptr, nullptr, q.scal + 1, q.part + kBRedBlocks, q.n, 0, 0, 0, 0});
                    put(S_SHIFT, i, {nullptr, nullptr, nullptr, nullptr, q.scal, nullptr, 0, 0, 0, 0.0,
                                     inner64 ? eps64 : eps32});
                    put(S_AXPY, i, {q.u, z, q.ut, q.scal + 2, nullptr, nullptr, q.n, 0, 0, 0, 0});
                    if (inner64) { on64[i] = 1; in64[i] = q.ut; out64[i] = q.Ft; }
                    else { on32[i] = 1; in32[i] = q.ut; out32[i] = q.Ft; }
                    break;
                }
                case PH_LINESEARCH:
                    put(S_LS, i, {q.u, q.delta, q.ut, nullptr, nullptr, nullptr, q.n, 0, 0, 1.0, q.mu});
                    on64[i] = 1; in64[i] = q.ut; out64[i] = q.Ft; lsr.push_back(i);
                    break;
            }
        }
        // post-work descriptors
        for (int i : arn) {
            Inst &q = I[i];
            const double *Fb = q.inner64 ? q.F : q.Fin;
            put(S_QUO, i, {q.Ft, Fb, q.w, q.scal + 2, nullptr, nullptr, q.n, 0, 0, 0, 0});
            put(S_MD1, i, {q.V, q.w, nullptr, nullptr, q.hdev, q.part, q.n, q.n, q.j + 1, 0, 0});
            put(S_OR1, i, {q.V, nullptr, q.w, q.hdev, nullptr, nullptr, q.n, q.n, q.j + 1, 0, 0});
            put(S_MD2, i, {q.V, q.w, nullptr, nullptr, q.hdev + m + 1, q.part, q.n, q.n, q.j + 1, 0, 0});
            put(S_OR2, i, {q.V, nullptr, q.w, q.hdev + m + 1, nullptr, nullptr, q.n, q.n, q.j + 1, 0, 0});
            put(S_WN, i, {q.w, q.w, nullptr, nullptr, q.hdev + 2 * (m + 1), q.part, q.n, 0, 0, 0, 0});
            put(S_VN, i, {q.w, nullptr, q.V + (size_t)(q.j + 1) * q.n, q.hdev + 2 * (m + 1), nullptr, nullptr, q.n, 0, 0, 0, 0});
        }
        for (int i : rst) {
            Inst &q = I[i];
            const double *Fb = q.inner64 ? q.F : q.Fin;
            put(S_QUO, i, {q.Ft, Fb, q.w, q.scal + 2, nullptr, nullptr, q.n, 0, 0, 0, 0});
            put(S_RSR, i, {q.rhs, q.w, q.r, nullptr, nullptr, nullptr, q.n, 0, 0, 1.0, -1.0});
            put(S_RSB, i, {q.r, q.r, nullptr, nullptr, q.scal + 3, q.part, q.n, 0, 0, 0, 0});
            put(S_RSV, i, {q.r, nullptr, q.V, q.scal + 3, nullptr, nullptr, q.n, 0, 0, 0, 0});
        }
        for (int i : bas) {
            Inst &q = I[i];
            put(S_NF2, i, {q.F, q.F, nullptr, nullptr, q.scal + 4, q.part, q.n, 0, 0, 0, 0});
            put(S_NFI, i, {q.F, nullptr, nullptr, nullptr, q.scal + 5, q.part + 2 * kBRedBlocks, q.n, 0, 0, 0, 0});
        }
        for (int i : lsr) {
            Inst &q = I[i];
            put(S_NF2, i, {q.Ft, q.Ft, nullptr, nullptr, q.scal + 4, q.part, q.n, 0, 0, 0, 0});
            put(S_NFI, i, {q.Ft, nullptr, nullptr, nullptr, q.scal + 5, q.part + 2 * kBRedBlocks, q.n, 0, 0, 0, 0});
        }
        for (int i : act)
            put(S_GATHER, i, {I[i].scal, I[i].hdev, stage + (size_t)i * kSmall, nullptr, nullptr, nullptr, 0, 0,
                              3 * (m + 1), 0, 0});
        long tot = 0;
        if (!has32)
            for (int i = 0; i < count; ++i)
                if (on32[i]) return fail(BIM_EINVAL, "internal: FP32C evaluation in an FP64 batch");
        if ((rc = residual_batched_fill(probs, count, on64.data(), in64.data(), out64.data(), BIM_FP64, pls.data(),
                                        rws.data(), hd64, &tot)))
            return rc;
        if (has32 && (rc = residual_batched_fill(probs, count, on32.data(), in32.data(), out32.data(), BIM_FP32C,
                                                 pls.data(), rws.data(), hd32, &tot)))
            return rc;
        if ((rc = run_round())) return rc;
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
        BOp *acc = hops + (size_t)S_ACCU * count;
        std::memset(acc, 0, sizeof(BOp) * count);
        bool any = false;
        for (int i = 0; i < count; ++i)
            if (I[i].pending & PD_ACCEPT) {
                acc[i] = {I[i].ut, nullptr, I[i].u, nullptr, nullptr, nullptr, I[i].n, 0, 0, 1.0, 0.0};
                any = true;
            }
        if (any) {
            if ((rc = hip_check(hipMemcpyAsync(OPS(S_ACCU), acc, sizeof(BOp) * count, hipMemcpyHostToDevice, s),
                                "copy")))
                return rc;
            if ((rc = b_axpby(OPS(S_ACCU), count, s))) return rc;
        }
        if ((rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
    }
    // the extent of every instance's last iterate (largest elevation, smallest depth)
    std::vector<double> ext(2 * (size_t)count, 0.0);
    for (int i = 0; i < count; ++i)
        if (I[i].R.status >= BIM_OK && (size_t)2 * I[i].p->M <= (size_t)kBRedBlocks * (m + 1)) {
            if ((rc = surface_extent_enqueue(I[i].p, I[i].u, I[i].part, I[i].scal + 6, s))) return rc;
            if ((rc = hip_check(hipMemcpyAsync(&ext[2 * (size_t)i], I[i].scal + 6, sizeof(double) * 2,
                                               hipMemcpyDeviceToHost, s), "copy")))
                return rc;
        }
    if ((rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
    for (int i = 0; i < count; ++i)
        if (I[i].R.status >= BIM_OK && (size_t)2 * I[i].p->M <= (size_t)kBRedBlocks * (m + 1)) {
            I[i].R.max_zeta = ext[2 * (size_t)i];
            I[i].R.min_depth = ext[2 * (size_t)i + 1];
            if (physical_status(I[i].p, I[i].R.max_zeta, I[i].R.min_depth) != BIM_OK) I[i].R.status = BIM_UNPHYSICAL;
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
    (void)graph_captures;
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
        // each problem owns its iterate and its preconditioner's apply scratch:
        // a shared one would be written by two problems in one launch
        for (int k = 0; k < i; ++k) {
            if (us[k] == us[i]) return fail(BIM_EINVAL, "u[i] must be distinct vectors");
            if (Ps && Ps[i] && Ps[k] == Ps[i]) return fail(BIM_EINVAL, "a preconditioner appears twice in Ps");
        }
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
