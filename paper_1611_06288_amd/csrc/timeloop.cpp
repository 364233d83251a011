// Graph-driven time loop (pfc_run): many steps of scheme (1.10) with the
// cycle loop of Algorithm algorithm:FAS taken on the device.
//
// One multigrid cycle together with the stop test that precedes it (the
// residual max-norm, then the loop's decision) is recorded once as a hipGraph
// on the handle's own stream.  The decision kernel keeps the step's state in
// device memory (active, cycles, status, first and latest norm) and every
// kernel of the cycle is gated on `active`, so a replay after convergence
// does nothing.  A step launches the graph as many times as the previous step
// needed cycles, reads the 24-byte state back once, and launches one more
// replay at a time only while the step is still active.  The sequence of
// operations a step performs is therefore exactly that of pfc_step (same
// kernels, same order, same decisions), so results agree bit for bit, while
// the host round trips drop from one per cycle to one or two per step and the
// launches of a cycle go out as one graph.
//
// With the split stop test (FP64, M = 1, fused finest level) the recorded
// unit is instead: the next cycle's first finest-level pre-sweep, which also
// yields the colour-0 half of the norm of its input, then the decision on
// both halves, then the rest of the cycle, whose last post-sweep leaves the
// colour-1 half for the next replay.  A replay that stops leaves the iterate
// in the pre-sweep's input buffer, which the sweep does not write.  Before a
// step's first replay the colour-1 half is seeded with the whole-level norm.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "runtime_internal.h"

using namespace pfc;

namespace {

RunState run_state(pfc_handle *H) {
    return RunState{H->d_run, H->d_run + 1, H->d_run + 2, H->d_runres, H->d_runres + 1};
}

// The recorded cycle assumes the level iterates it was recorded with; levels
// smoothed by the fused sweep trade their two buffers once per sweep, which
// leaves them in place over a cycle only for an even sweep count.
bool graph_usable(const pfc_handle *H) {
    if (H->cfg.precision != PFC_FP64) return false;
    if (((H->cfg.nu1 + H->cfg.nu2) & 1) == 0) return true;
    for (int l = 0; l < H->nlev; ++l)
        if (H->lev[l].fused) return false;
    return true;
}

bool graph_current(const pfc_handle *H) {
    if (!H->run_exec) return false;
    for (int l = 0; l < H->nlev; ++l)
        if (H->run_key[l] != (const void *)H->lev[l].u.a) return false;
    return true;
}

pfc_status record_graph(pfc_handle *H) {
    if (H->run_exec) {
        (void)hipGraphExecDestroy(H->run_exec);
        H->run_exec = nullptr;
    }
    if (H->run_graph) {
        (void)hipGraphDestroy(H->run_graph);
        H->run_graph = nullptr;
    }
    const bool timing = H->timing;
    H->timing = false;  // no event records inside the graph
    hipError_t e = hipStreamBeginCapture(H->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        H->timing = timing;
        return hip_fail(H, e, "hipStreamBeginCapture");
    }
    H->gate = H->d_run;  // every launch below reads the active flag
    const bool fcycle = H->cfg.cycle == PFC_CYCLE_F;
    if (H->split_norm) {
        sweep64(H, 0, 1, H->cfg.nu1 >= 2);
        launch_stop_test(H->stream, H->partial, 2 * H->split_blocks, H->cfg.tol,
                         H->cfg.max_cycles, run_state(H));
        cycle64(H, 0, fcycle, kCyclePreDone | kCyclePostNorm);
    } else {
        const int cnt = enqueue_norm64(H);
        launch_stop_test(H->stream, H->partial, cnt, H->cfg.tol, H->cfg.max_cycles,
                         run_state(H));
        cycle64(H, 0, fcycle);
    }
    H->gate = nullptr;
    H->timing = timing;
    e = hipStreamEndCapture(H->stream, &H->run_graph);
    if (e != hipSuccess) return hip_fail(H, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&H->run_exec, H->run_graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(H, e, "hipGraphInstantiate");
    for (int l = 0; l < H->nlev; ++l) H->run_key[l] = H->lev[l].u.a;
    return PFC_OK;
}

// One FP64 step with the cycle loop replayed as a graph.
pfc_status graph_step(pfc_handle *H, const double *prev, const double *cur, double *next,
                      double *mu, double *om, pfc_step_info *info) {
    step_begin(H, prev, cur, mu, om);
    launch_run_reset(H->stream, run_state(H));
    if (H->split_norm) {
        unsigned long long *whole = H->partial + 2 * H->split_blocks;
        const int cnt = enqueue_norm64(H, whole);
        launch_norm_seed(H->stream, whole, cnt, H->partial + H->split_blocks, H->split_blocks);
    }
    HIP_TRY(H, hipGetLastError());
    if (!graph_current(H)) {
        const pfc_status st = record_graph(H);
        if (st != PFC_OK) return st;
    }
    int *hs = reinterpret_cast<int *>(H->h_pin + 16);  // active, cycles, status
    double *hr = H->h_pin + 20;                         // res0, res
    int launches = std::max(1, H->last_cycles);
    // a step ends after at most max_cycles + 1 stop tests
    for (int total = 0;;) {
        for (int i = 0; i < launches; ++i) HIP_TRY(H, hipGraphLaunch(H->run_exec, H->stream));
        total += launches;
        HIP_TRY(H, hipMemcpyAsync(hs, H->d_run, 3 * sizeof(int), hipMemcpyDeviceToHost, H->stream));
        HIP_TRY(H, hipMemcpyAsync(hr, H->d_runres, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                  H->stream));
        HIP_TRY(H, hipStreamSynchronize(H->stream));
        if (hs[0] == 0) break;
        if (total > H->cfg.max_cycles + 1)
            return fail(H, PFC_ERR_HIP, "time loop: the device stop test did not end the step");
        launches = 1;
    }
    const int cycles = hs[1], status = hs[2];
    const double res0 = hr[0], res = hr[1];
    step_end(H, next, mu, om);
    HIP_TRY(H, hipGetLastError());
    H->last_cycles = cycles;
    if (info) {
        info->cycles = cycles;
        info->status = status;
        info->res0 = res0;
        info->res_final = res;
    }
    if (status != PFC_OK) fail(H, status, pfc_status_string(status));
    return status;
}

}  // namespace

namespace pfc {
pfc_status own_stream_enter(pfc_handle *H, hipStream_t *user) {
    if (!H->run_stream) {
        HIP_TRY(H, hipStreamCreateWithFlags(&H->run_stream, hipStreamNonBlocking));
        HIP_TRY(H, hipEventCreateWithFlags(&H->run_ev, hipEventDisableTiming));
    }
    *user = H->stream;
    if (H->stream == H->run_stream) return PFC_OK;  // already on it
    HIP_TRY(H, hipEventRecord(H->run_ev, H->stream));
    HIP_TRY(H, hipStreamWaitEvent(H->run_stream, H->run_ev, 0));
    H->stream = H->run_stream;
    return PFC_OK;
}

pfc_status own_stream_leave(pfc_handle *H, hipStream_t user) {
    if (user == H->run_stream) return PFC_OK;
    hipError_t e = hipEventRecord(H->run_ev, H->run_stream);
    H->stream = user;
    if (e == hipSuccess) e = hipStreamWaitEvent(user, H->run_ev, 0);
    if (e != hipSuccess) return hip_fail(H, e, "own stream: hand-back");
    return PFC_OK;
}
}  // namespace pfc

extern "C" pfc_status pfc_run(pfc_handle *h, double *phi_prev, double *phi_cur, double *mu,
                              double *omega, int32_t steps, pfc_step_info *infos) {
    if (!h) return PFC_ERR_INVALID_ARG;
    if (!phi_prev || !phi_cur || !mu || !omega) return fail(h, PFC_ERR_INVALID_ARG, "NULL field pointer");
    if (phi_prev == phi_cur) return fail(h, PFC_ERR_INVALID_ARG, "phi_prev and phi_cur must differ");
    if (steps < 0) return fail(h, PFC_ERR_INVALID_ARG, "steps must be >= 0");
    if (steps == 0) return PFC_OK;
    if (!h->spare) {
        if (!dalloc(h, &h->spare, h->lev[0].P) || !dalloc(h, &h->d_run, 4) ||
            !dalloc(h, &h->d_runres, 2))
            return fail(h, PFC_ERR_OOM, "time-loop buffers");
    }
    // the loop's stream follows the caller's, and the caller's follows it at the end
    hipStream_t user;
    {
        const pfc_status st = own_stream_enter(h, &user);
        if (st != PFC_OK) return st;
    }
    const bool graph = graph_usable(h);
    double *buf[3] = {phi_prev, phi_cur, h->spare};
    int ip = 0, ic = 1, in = 2;
    pfc_status status = PFC_OK;
    for (int k = 0; k < steps; ++k) {
        pfc_step_info inf{};
        pfc_status st;
        if (graph)
            st = graph_step(h, buf[ip], buf[ic], buf[in], mu, omega, &inf);
        else if (h->cfg.precision == PFC_MIXED)
            st = mixed_step(h, buf[ip], buf[ic], buf[in], mu, omega, &inf);
        else
            st = step64(h, buf[ip], buf[ic], buf[in], mu, omega, &inf);
        if (infos) infos[k] = inf;
        // NOT_CONVERGED and NONFINITE still deliver the step's last iterate;
        // any other failure leaves the state of the previous step
        if (st == PFC_OK || st == inf.status) {
            const int op = ip;
            ip = ic;
            ic = in;
            in = op;
        }
        if (st != PFC_OK) {
            status = st;
            break;
        }
    }
    // the last two states back into the caller's buffers (a rotation of three)
    const size_t bytes = h->lev[0].P * sizeof(double);
    hipError_t e = hipSuccess;
    if (ip == 1 && ic == 2) {  // prev in phi_cur, cur in spare
        e = hipMemcpyAsync(phi_prev, phi_cur, bytes, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(phi_cur, h->spare, bytes, hipMemcpyDeviceToDevice, h->stream);
    } else if (ip == 2 && ic == 0) {  // prev in spare, cur in phi_prev
        e = hipMemcpyAsync(phi_cur, phi_prev, bytes, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(phi_prev, h->spare, bytes, hipMemcpyDeviceToDevice, h->stream);
    }
    if (e != hipSuccess) {
        (void)own_stream_leave(h, user);
        return hip_fail(h, e, "time loop: final copies");
    }
    const pfc_status st = own_stream_leave(h, user);
    return st != PFC_OK ? st : status;
}
