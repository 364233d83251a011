// Mixed-precision form of the time step: an FP64 defect correction around
// FP32 multigrid cycles.
//
// Outer loop (FP64, finest level): r = S - N(u) and its max-norm; stop when
// max|r| <= tol.  Otherwise one FAS cycle in FP32 solves for a correction e
//     N(u + e) - N(u) = r,
// whose operator is N's linear part acting on e plus the cubic difference
//     G(e) = g(b + e; phi^k) - g(b; phi^k)
//          = 1/4 [e (b^2 + (phi^k)^2) + (b + e + phi^k)(2 b e + e^2)],
// b = phi of the current FP64 iterate rounded to FP32 (restricted to the
// coarse levels), written without cancellation.  Then u += e in FP64 (on
// levels with column tiles, inside the next defect pass).  Up to twenty FP32
// cycles run per defect, as many as the observed contraction predicts are
// needed to reach tol (one cycle is recorded as a hipGraph and replayed).  The smoother's pointwise
// 3x3 solve, the residual and all reductions run in FP64 arithmetic; only
// stored fields of the correction cycle are FP32.
#include <algorithm>
#include <cmath>
#include <utility>

#include "runtime_internal.h"

namespace pfc {

// Up to kMaxInnerCycles FP32 cycles per FP64 defect: as many as the observed
// contraction predicts are needed to bring the residual within kTolMargin of
// tol, while the predicted reduction of this defect stays above
// kMinDefectFactor: the FP32 correction cannot reduce an FP64 defect by much
// more than that (the stored correction's rounding, amplified by the
// operator), so cycles past it would be spent at that floor.  The margin
// keeps an optimistic prediction from running cycles the FP64 loop would
// not; a pessimistic one costs one more defect pass.  The floor test takes
// the contraction as at least kFloorQ: the first cycles of a step remove the
// rough part of the error at rates the later ones never reach, and a floor
// predicted from them would cut the next defect's cycles short.
constexpr int kMaxInnerCycles = 20;
constexpr double kMinDefectFactor = 1e-5;
constexpr double kTolMargin = 1.5;
constexpr double kFloorQ = 0.5;

pfc_status mixed_init(pfc_handle *H) {
    if (hipEventCreateWithFlags(&H->norm_ev, hipEventDisableTiming) != hipSuccess)
        return fail(H, PFC_ERR_HIP, "event creation failed");
    for (int l = 0; l < H->nlev; ++l) {
        Level32 &A = H->lev32[l];
        const size_t P = H->lev[l].P;
        float *e, *f, *eb;
        const bool ok = dalloc(H, &e, 3 * P) && dalloc(H, &f, 3 * P) && dalloc(H, &eb, 3 * P) &&
                        dalloc(H, &A.phk, P) && dalloc(H, &A.base, P);
        if (!ok) return fail(H, PFC_ERR_OOM, "device allocation for the FP32 hierarchy failed");
        A.e = Tri<float>{e, e + P, e + 2 * P};
        A.f = Tri<float>{f, f + P, f + 2 * P};
        A.ebar = Tri<float>{eb, eb + P, eb + 2 * P};
    }
    return PFC_OK;
}

// tau: the first sweep of a coarse level, forming the tau correction from
// I e = ebar as it smooths (launch_smooth_tau).
static void sweep32(pfc_handle *H, int l, bool tau = false) {
    Level32 &A = H->lev32[l];
    const OpParams op = op_of(H, l);
    if (H->lev[l].n <= kSmallSweepN) {  // both colours in one workgroup
        if (tau)
            launch_sweep_small_tau<float, true>(H->stream, op, 0, A.e, A.f, cst(A.ebar), A.phk,
                                                A.base);
        else
            launch_sweep_small<float, true>(H->stream, op, 0, A.e, cst(A.f), A.phk, A.base);
        return;
    }
    for (int colour = 0; colour < 2; ++colour) {
        H->begin_timed(PFC_KERNEL_SMOOTH0, l);
        if (tau)
            launch_smooth_tau<float, true>(H->stream, op, colour, 0, A.e, A.f, cst(A.ebar), A.phk,
                                           A.base);
        else
            launch_smooth<float, true>(H->stream, op, colour, 0, A.e, cst(A.f), A.phk, A.base);
        H->end_timed();
    }
}

// tau: f of level l holds I r and its iterate is still in ebar (the first
// pre-sweep, on the coarsest the solve's launch, forms the tau correction).
static void cycle32(pfc_handle *H, int l, bool fcycle, bool tau = false) {
    Level32 &A = H->lev32[l];
    if (l == H->nlev - 1) {
        H->begin_timed(PFC_KERNEL_COARSE, l);
        launch_coarse<float, true>(
            H->stream, op_of(H, l), A.e, cst(A.f), A.phk, A.base, H->lap1, H->lap3, H->minv32,
            nullptr, H->valid32, H->d_iters, nullptr,
            tau ? cst(A.ebar) : Tri<const float>{nullptr, nullptr, nullptr}, A.f);
        H->end_timed();
        return;
    }
    Level32 &B = H->lev32[l + 1];
    const Lay &LB = H->lev[l + 1].lay;
    for (int s = 0; s < H->cfg.nu1; ++s) sweep32(H, l, tau && s == 0);
    H->begin_timed(PFC_KERNEL_RESIDUAL0, l);
    if (H->lev[l].rt) {
        ResidTileArgs ra;
        ra.e32 = cst(A.e);
        ra.f32 = cst(A.f);
        ra.phk32 = A.phk;
        ra.b32 = A.base;
        ra.LC = LB;
        ra.ebar32 = B.ebar;
        ra.rr32 = B.f;
        launch_resid_tile(H->stream, RT_RESTRICT32, op_of(H, l), H->lev[l].rt_nz[RT_RESTRICT32], ra);
    } else {
        launch_resid_restrict<float, true>(H->stream, op_of(H, l), LB, cst(A.e), cst(A.f), A.phk,
                                           A.base, B.ebar, B.f);
    }
    H->end_timed();
    // a coarse level forms the tau correction in its first pre-sweep, the
    // coarsest in its solve's launch
    const bool tau_sweep = l + 1 == H->nlev - 1 || H->cfg.nu1 >= 1;
    if (!tau_sweep)
        launch_tau<float, true>(H->stream, op_of(H, l + 1), cst(B.ebar), B.f, B.e, B.phk, B.base);
    cycle32(H, l + 1, fcycle, tau_sweep);
    if (fcycle) cycle32(H, l + 1, false);
    H->begin_timed(PFC_KERNEL_PROLONG0, l);
    launch_prolong<float>(H->stream, LB, H->lev[l].lay, cst(B.e), cst(B.ebar), A.e, nullptr,
                          H->cfg.nu2 >= 1, H->lev[l].pz[1]);
    H->end_timed();
    for (int s = 0; s < H->cfg.nu2; ++s) sweep32(H, l);
}

// One FP32 cycle recorded as a graph on the handle's own stream (its
// buffers never move), replayed once per inner cycle: the cycle's ~60
// launches, mostly on small levels, go out together.  Kernel timing is not
// recorded inside it.
static pfc_status record_cycle32(pfc_handle *H) {
    const bool timing = H->timing;
    H->timing = false;
    hipError_t e = hipStreamBeginCapture(H->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        cycle32(H, 0, H->cfg.cycle == PFC_CYCLE_F);
        e = hipStreamEndCapture(H->stream, &H->mix_graph);
    }
    H->timing = timing;
    if (e == hipSuccess) e = hipGraphInstantiate(&H->mix_exec, H->mix_graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(H, e, "recording the FP32 cycle");
    return PFC_OK;
}

static pfc_status mixed_step_on(pfc_handle *H, const double *phi_prev, const double *phi_cur,
                                double *phi_next, double *mu, double *omega,
                                pfc_step_info *info);

pfc_status mixed_step(pfc_handle *H, const double *phi_prev, const double *phi_cur,
                      double *phi_next, double *mu, double *omega, pfc_step_info *info) {
    hipStream_t user;
    pfc_status st = own_stream_enter(H, &user);
    if (st != PFC_OK) return st;
    st = mixed_step_on(H, phi_prev, phi_cur, phi_next, mu, omega, info);
    const pfc_status st2 = own_stream_leave(H, user);
    return st != PFC_OK ? st : st2;
}

// The step on the handle's own stream.
static pfc_status mixed_step_on(pfc_handle *H, const double *phi_prev, const double *phi_cur,
                                double *phi_next, double *mu, double *omega,
                                pfc_step_info *info) {
    Level &A = H->lev[0];
    Level32 &A32 = H->lev32[0];
    step_begin(H, phi_prev, phi_cur, mu, omega);
    launch_to_lay<double, float>(H->stream, A.lay, phi_cur, A32.phk, 1);
    for (int l = 0; l + 1 < H->nlev; ++l)
        launch_restrict<float>(H->stream, H->lev[l].lay, H->lev[l + 1].lay, H->lev32[l].phk,
                               H->lev32[l + 1].phk);
    HIP_TRY(H, hipGetLastError());
    int c = 0;
    double rho = 0, rho0 = 0, rho_prev = 0;
    int inner_prev = 1;
    bool pending = false;  // a correction e waits to be added to u
    pfc_status status = PFC_OK;
    for (;;) {
        H->begin_timed(PFC_KERNEL_NORM0, 0);
        int cnt;
        if (A.rt) {
            ResidTileArgs ra;
            ra.f = frhs(H, 0);
            ra.phk = A.phk;
            ra.r32 = A32.f;
            ra.base32 = A32.base;
            ra.partial = H->partial;
            if (pending) {  // u2 = u + e, defect and casts of u2, in one pass
                ra.u = cst(A.u);
                ra.e = cst(A32.e);
                ra.uout = A.u2;
                cnt = launch_resid_tile(H->stream, RT_CAST_CORR, op_of(H, 0),
                                        A.rt_nz[RT_CAST_CORR], ra);
                std::swap(A.u, A.u2);
            } else {
                ra.u = cst(A.u);
                cnt = launch_resid_tile(H->stream, RT_CAST, op_of(H, 0), A.rt_nz[RT_CAST], ra);
            }
        } else {
            if (pending) launch_add_correction(H->stream, A.P, A.u, cst(A32.e));
            cnt = launch_resid_cast(H->stream, op_of(H, 0), cst(A.u), frhs(H, 0), A.phk, A32.f,
                                    A32.base, H->partial);
        }
        pending = false;
        H->end_timed();
        // the norm to the host behind an event; then the next FP32 cycles'
        // base on every level and their zero start, queued ahead of the
        // host's wait so that the device works while the host decides
        // (wasted once per step, after the last defect pass)
        launch_max_final(H->stream, H->partial, cnt, H->d_scal);
        HIP_TRY(H, hipMemcpyAsync(H->h_pin, H->d_scal, sizeof(double), hipMemcpyDeviceToHost,
                                  H->stream));
        HIP_TRY(H, hipEventRecord(H->norm_ev, H->stream));
        for (int l = 0; l + 1 < H->nlev; ++l)
            launch_restrict<float>(H->stream, H->lev[l].lay, H->lev[l + 1].lay, H->lev32[l].base,
                                   H->lev32[l + 1].base);
        launch_zero(H->stream, A32.e.a, 3 * A.P);
        HIP_TRY(H, hipGetLastError());
        HIP_TRY(H, hipEventSynchronize(H->norm_ev));
        H->collect_timings();
        rho = H->h_pin[0];
        if (c == 0) rho0 = rho;
        if (!std::isfinite(rho)) {
            status = PFC_ERR_NONFINITE;
            break;
        }
        if (rho <= H->cfg.tol) break;
        if (c >= H->cfg.max_cycles) {
            status = PFC_ERR_NOT_CONVERGED;
            break;
        }
        // FP32 cycles on this defect: as many (up to kMaxInnerCycles) as the
        // observed contraction per cycle predicts the FP64 loop would run
        // anyway before reaching tol, at least one.  Each FP64 defect pass
        // saved is a full-level FP64 read of u, f and phi^k.
        int inner = 1;
        if (rho_prev > 0 && rho < rho_prev) {
            const double q = std::pow(rho / rho_prev, 1.0 / inner_prev);
            const double qf = std::max(q, kFloorQ);
            double pred = rho * q, predf = rho * qf;
            while (inner < kMaxInnerCycles && c + inner + 1 <= H->cfg.max_cycles &&
                   pred > kTolMargin * H->cfg.tol && predf * qf > kMinDefectFactor * rho) {
                ++inner;
                pred *= q;
                predf *= qf;
            }
        }
        HIP_TRY(H, hipGetLastError());
        if (!H->mix_exec) {
            const pfc_status st2 = record_cycle32(H);
            if (st2 != PFC_OK) return st2;
        }
        for (int i = 0; i < inner; ++i) HIP_TRY(H, hipGraphLaunch(H->mix_exec, H->stream));
        pending = true;
        c += inner;
        rho_prev = rho;
        inner_prev = inner;
    }
    step_end(H, phi_next, mu, omega);
    HIP_TRY(H, hipGetLastError());
    HIP_TRY(H, hipStreamSynchronize(H->stream));
    if (info) {
        info->cycles = c;
        info->status = status;
        info->res0 = rho0;
        info->res_final = rho;
    }
    if (status != PFC_OK) fail(H, status, pfc_status_string(status));
    return status;
}

// Algorithmic HBM bytes per finest-level launch: each value the launch must
// read or write, once.  A fused FP64 sweep reads the old phi everywhere, the
// old mu and omega at colour-1 points only (colour 0's are overwritten
// unread), f (3 fields) and phi^k, and writes u: 8 + 8 + 24 + 8 + 24 = 72 B
// per point.  A half-sweep launch updates one colour: the other colour's
// three fields and its own old phi, f, phi^k and new u, i.e. 44 B per point
// of the level in FP64, and 24 B in the FP32 correction form (4 B values,
// plus the base).  The mixed form's FP64 defect pass reads u, f, phi^k and
// writes r and phi in FP32 (72 B); on column-tile levels it also reads the
// pending FP32 correction and writes u + e (108 B), which is all but the
// first pass of each step, so 108 is credited there.  In a time step the
// first component of f is phi^k itself and is read from phk (f1_phk), so
// every FP64 pass over the finest level reads 8 B per point of f fewer (4 B
// per point of the level for a half-sweep, which reads f at its own colour).
double algorithmic_bytes(const pfc_handle *H, int kernel) {
    const double P = (double)H->lev[0].P;
    const bool mixed = H->cfg.precision == PFC_MIXED;
    // variable mobility (FP64 only) reads phi* once more: 8 B/pt per pass
    const double mob = H->cfg.mobility == PFC_MOBILITY_QUADRATIC ? 8.0 : 0.0;
    const double f1 = H->f1_phk ? 8.0 : 0.0;  // f.a not streamed
    const double smooth =
        mixed ? 24.0 : (H->lev[0].fused ? 72.0 - f1 : 44.0 - 0.5 * f1) + mob;
    switch (kernel) {
        case PFC_KERNEL_SMOOTH0: return smooth * P;
        case PFC_KERNEL_RESIDUAL0: return (mixed ? 35.0 : 62.0 - f1 + mob) * P;
        // interpolation: u read and written where it is live after it (all
        // phi, colour-1 mu and omega: 2 x 2 fields' worth when a post-sweep
        // follows, else all three), plus the coarse v and ubar it forms the
        // error from (3 fields each, an eighth of the points)
        case PFC_KERNEL_PROLONG0: {
            const double fine = H->cfg.nu2 >= 1 ? 2.0 : 3.0;
            return (mixed ? 2 * 4.0 * fine + 3.0 : 2 * 8.0 * fine + 6.0) * P;
        }
        case PFC_KERNEL_NORM0:
            return (mixed ? (H->lev[0].rt ? 108.0 : 72.0) - f1 : 56.0 - f1 + mob) * P;
        // the fused sweep's 72 (80 with phi*) plus old mu and omega of the colour-0 points
        case PFC_KERNEL_SWEEP_NORM0: return H->split_norm ? (80.0 - f1 + mob) * P : 0.0;
        default: return 0.0;
    }
}

}  // namespace pfc
