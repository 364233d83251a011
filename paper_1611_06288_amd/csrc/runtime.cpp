// Host runtime of the PFC multigrid solver: handle, level hierarchy, FP64
// cycle driver, time step, instrumentation and the C ABI of include/pfc.h.
//
// Algorithm (Section 5, Algorithm algorithm:FAS, with these readings): the
// loop "while residual > tolerance" runs at the finest level only and tests
// max|S - N(u)| over the three components before each cycle; a recursive call
// performs one cycle; the coarse right-hand side is N_{l+1}(I u) + I r; the
// coarse correction is I(v - I u); red-black colour (i+j+k) mod 2, colour 0
// first in every sweep; the coarsest level (n = 3 or 4) is solved exactly.
//
// The caller's fields are in natural C order; inside a call the finest level
// works on colour-split copies (converted once per step or call).
#include "pfc.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <utility>
#include <string>
#include <vector>

#include "pfc_internal.h"
#include "runtime_internal.h"

using namespace pfc;

namespace {
thread_local std::string g_create_error;
}  // namespace

namespace pfc {

bool level_sizes(int n, std::vector<int> &out) {
    out.clear();
    if (n < 4 || (n & 1) || n > kMaxN) return false;
    int m = n;
    out.push_back(m);
    while ((m & 1) == 0 && m / 2 >= 3) {
        m /= 2;
        out.push_back(m);
    }
    return m == 3 || m == 4;
}

std::string validate_config(const pfc_config *c) {
    if (!c) return "config is NULL";
    std::vector<int> sizes;
    if (!level_sizes(c->n, sizes))
        return "n must be 2^k (k >= 2) or 3*2^k (k >= 1), at most 1024, got " + std::to_string(c->n);
    if (!(c->L > 0) || !std::isfinite(c->L)) return "L must be > 0";
    if (!(c->dt > 0) || !std::isfinite(c->dt)) return "dt must be > 0";
    if (!(c->tol >= 0) || !std::isfinite(c->tol)) return "tol must be >= 0";
    if (!std::isfinite(c->eps)) return "eps must be finite";
    if (c->nu1 < 0 || c->nu2 < 0 || c->nu1 + c->nu2 < 1) return "nu1, nu2 >= 0 with nu1 + nu2 >= 1";
    if (c->max_cycles < 1) return "max_cycles must be >= 1";
    if (c->cycle != PFC_CYCLE_V && c->cycle != PFC_CYCLE_F) return "unknown cycle type";
    if (c->lin != PFC_LIN_NEWTON && c->lin != PFC_LIN_PICARD) return "unknown linearisation";
    if (c->precision != PFC_FP64 && c->precision != PFC_MIXED) return "unknown precision";
    if (c->precision == PFC_MIXED && c->lin != PFC_LIN_NEWTON)
        return "the mixed-precision form uses Newton linearisation only";
    if (c->mobility != PFC_MOBILITY_ONE && c->mobility != PFC_MOBILITY_QUADRATIC)
        return "unknown mobility";
    if (c->mobility == PFC_MOBILITY_QUADRATIC) {
        if (c->precision != PFC_FP64) return "variable mobility is available in FP64 precision only";
        if (!std::isfinite(c->mob_m0) || !std::isfinite(c->mob_m1) || !std::isfinite(c->mob_m2))
            return "mobility coefficients must be finite";
        if (!(c->mob_min > 0) || !std::isfinite(c->mob_min)) return "mob_min must be > 0";
    }
    if (c->scheme != PFC_SCHEME_CS2 && c->scheme != PFC_SCHEME_CS1) return "unknown scheme";
    if (c->scheme == PFC_SCHEME_CS1 &&
        (c->precision != PFC_FP64 || c->mobility != PFC_MOBILITY_ONE))
        return "the first-order scheme is available in FP64 with M = 1 only";
    return "";
}

// Dense Lap, Lap^2 and Lap^3 (column-major, n^3 x n^3) on the coarsest level.
void coarse_matrices(int n, double h, std::vector<double> &l1, std::vector<double> &l2,
                     std::vector<double> &l3) {
    const int P = n * n * n;
    auto id = [n](int i, int j, int k) {
        i = (i + n) % n;
        j = (j + n) % n;
        k = (k + n) % n;
        return (k * n + j) * n + i;
    };
    std::vector<double> A((size_t)P * P, 0.0);  // row-major A[r*P + c]
    const double w = 1.0 / (h * h);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const int r = id(i, j, k);
                const int nb[6] = {id(i + 1, j, k), id(i - 1, j, k), id(i, j + 1, k),
                                   id(i, j - 1, k), id(i, j, k + 1), id(i, j, k - 1)};
                for (int q = 0; q < 6; ++q) A[(size_t)r * P + nb[q]] += w;
                A[(size_t)r * P + r] -= 6.0 * w;
            }
    std::vector<double> A2((size_t)P * P, 0.0), A3((size_t)P * P, 0.0);
    for (int r = 0; r < P; ++r)
        for (int m = 0; m < P; ++m) {
            const double v = A[(size_t)r * P + m];
            if (v == 0.0) continue;
            for (int c = 0; c < P; ++c) A2[(size_t)r * P + c] += v * A[(size_t)m * P + c];
        }
    for (int r = 0; r < P; ++r)
        for (int m = 0; m < P; ++m) {
            const double v = A2[(size_t)r * P + m];
            if (v == 0.0) continue;
            for (int c = 0; c < P; ++c) A3[(size_t)r * P + c] += v * A[(size_t)m * P + c];
        }
    l1.assign((size_t)P * P, 0.0);
    l2.assign((size_t)P * P, 0.0);
    l3.assign((size_t)P * P, 0.0);
    for (int r = 0; r < P; ++r)
        for (int c = 0; c < P; ++c) {
            l1[(size_t)c * P + r] = A[(size_t)r * P + c];
            l2[(size_t)c * P + r] = A2[(size_t)r * P + c];
            l3[(size_t)c * P + r] = A3[(size_t)r * P + c];
        }
}

pfc_status fail(pfc_handle *H, pfc_status st, const std::string &msg) {
    if (H)
        H->err = msg;
    else
        g_create_error = msg;
    return st;
}

pfc_status hip_fail(pfc_handle *H, hipError_t e, const char *what) {
    return fail(H, PFC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

OpParams op_of(const pfc_handle *H, int l) {
    OpParams op{H->lev[l].lay, H->lev[l].h2inv, H->cfg.dt, H->cfg.eps};
    op.fo = H->cfg.scheme == PFC_SCHEME_CS1 ? 1 : 0;
    if (H->cfg.mobility == PFC_MOBILITY_QUADRATIC)
        op.mob = Mobility{H->lev[l].phs, H->cfg.mob_m0, H->cfg.mob_m1, H->cfg.mob_m2, H->cfg.mob_min};
    op.gate = H->gate;
    return op;
}

// Clears the two cache flags with a kernel rather than hipMemsetAsync, so
// that a caller may record the call into a graph.
__global__ void k_clear_flags(int *a, int *b) {
    if (threadIdx.x == 0) { *a = 0; *b = 0; }
}

void invalidate_coarse(pfc_handle *H) {
    k_clear_flags<<<1, 64, 0, H->stream>>>(H->valid64, H->valid32);
}

}  // namespace pfc

// ------------------------------------------------------------ timing

void pfc_handle::begin_timed(int kind, int level, double bytes) {
    cur_event = -1;
    if (!timing || kind < 0) return;
    if (kind != PFC_KERNEL_COARSE && level != 0) return;
    hipEvent_t a, b;
    if (pool.size() >= 2) {
        a = pool.back();
        pool.pop_back();
        b = pool.back();
        pool.pop_back();
    } else {
        if (hipEventCreate(&a) != hipSuccess) return;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return;
        }
    }
    (void)hipEventRecord(a, stream);
    pending.push_back(TimedLaunch{kind, a, b, bytes >= 0.0 ? bytes : algorithmic_bytes(this, kind)});
    cur_event = (int)pending.size() - 1;
}

void pfc_handle::end_timed() {
    if (cur_event < 0) return;
    (void)hipEventRecord(pending[cur_event].b, stream);
    cur_event = -1;
}

void pfc_handle::collect_timings() {
    for (auto &t : pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            t_count[t.kind] += 1;
            t_ms[t.kind] += ms;
            t_bytes[t.kind] += t.bytes;
        }
        pool.push_back(t.a);
        pool.push_back(t.b);
    }
    pending.clear();
}

pfc_handle::~pfc_handle() {
    for (auto &t : pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
    if (run_stream) (void)hipStreamSynchronize(run_stream);
    if (mix_exec) (void)hipGraphExecDestroy(mix_exec);
    if (mix_graph) (void)hipGraphDestroy(mix_graph);
    if (run_exec) (void)hipGraphExecDestroy(run_exec);
    if (run_graph) (void)hipGraphDestroy(run_graph);
    if (run_ev) (void)hipEventDestroy(run_ev);
    if (norm_ev) (void)hipEventDestroy(norm_ev);
    if (run_stream) (void)hipStreamDestroy(run_stream);
    for (void *p : allocs) (void)hipFree(p);
    if (h_pin) (void)hipHostFree(h_pin);
}

// ----------------------------------------------------- FP64 multigrid

namespace pfc {

void sweep64(pfc_handle *H, int l, int nrm, bool then_sweep, bool tau) {
    Level &A = H->lev[l];
    const OpParams op = op_of(H, l);
    if (A.fused && tau) {  // a coarse level's first sweep: two tau-forming half-sweeps from
                           // I u into the second buffer, which then becomes the iterate
        for (int colour = 0; colour < 2; ++colour)
            launch_smooth_tau<double, false>(H->stream, op, colour, H->cfg.lin == PFC_LIN_PICARD,
                                             A.u2, A.f, cst(A.ubar), A.phk, nullptr);
        std::swap(A.u, A.u2);
        return;
    }
    if (A.fused) {  // one pass, then the two iterate buffers trade places
        if (!H->split_norm || l != 0) nrm = 0;
        unsigned long long *part =
            nrm == 1 ? H->partial : (nrm == 2 ? H->partial + H->split_blocks : nullptr);
        const bool skip0 = then_sweep && nrm != 2;
        const int kind = nrm == 1 ? PFC_KERNEL_SWEEP_NORM0 : PFC_KERNEL_SMOOTH0;
        // the colour-0 mu, omega writes left out: 8 B/pt fewer
        H->begin_timed(kind, l, skip0 ? algorithmic_bytes(H, kind) - 8.0 * (double)A.P : -1.0);
        launch_sweep_fused<double, false>(H->stream, op, H->cfg.lin == PFC_LIN_PICARD, A.nz,
                                          cst(A.u), A.u2, frhs(H, l), A.phk,
                                          nullptr, nrm, part, skip0);
        H->end_timed();
        std::swap(A.u, A.u2);
        return;
    }
    const int picard = H->cfg.lin == PFC_LIN_PICARD;
    if (A.n <= kSmallSweepN) {  // both colours in one workgroup
        H->begin_timed(PFC_KERNEL_SMOOTH0, l);
        if (tau)
            launch_sweep_small_tau<double, false>(H->stream, op, picard, A.u, A.f, cst(A.ubar),
                                                  A.phk, nullptr);
        else
            launch_sweep_small<double, false>(H->stream, op, picard, A.u, frhs(H, l), A.phk,
                                              nullptr);
        H->end_timed();
        return;
    }
    for (int colour = 0; colour < 2; ++colour) {
        H->begin_timed(PFC_KERNEL_SMOOTH0, l);
        if (tau)
            launch_smooth_tau<double, false>(H->stream, op, colour, picard, A.u, A.f, cst(A.ubar),
                                             A.phk, nullptr);
        else
            launch_smooth<double, false>(H->stream, op, colour, picard, A.u, frhs(H, l), A.phk,
                                         nullptr);
        H->end_timed();
    }
}

void cycle64(pfc_handle *H, int l, bool fcycle, unsigned flags) {
    Level &A = H->lev[l];
    if (l == H->nlev - 1) {
        H->begin_timed(PFC_KERNEL_COARSE, l);
        // kCycleTauSweep: the solve applies the level's tau correction first
        launch_coarse<double, false>(
            H->stream, op_of(H, l), A.u, cst(A.f), A.phk, nullptr, H->lap1, H->lap3, H->minv64,
            nullptr, H->valid64, H->d_iters, H->lap2,
            (flags & kCycleTauSweep) ? cst(A.ubar) : Tri<const double>{nullptr, nullptr, nullptr},
            A.f);
        H->end_timed();
        return;
    }
    Level &B = H->lev[l + 1];
    for (int s = (flags & kCyclePreDone) ? 1 : 0; s < H->cfg.nu1; ++s)
        sweep64(H, l, 0, s + 1 < H->cfg.nu1, s == 0 && (flags & kCycleTauSweep));
    H->begin_timed(PFC_KERNEL_RESIDUAL0, l);
    if (A.rt) {
        ResidTileArgs ra;
        ra.u = cst(A.u);
        ra.f = frhs(H, l);
        ra.phk = A.phk;
        ra.LC = B.lay;
        ra.ubar = B.ubar;
        ra.rr = B.f;
        launch_resid_tile(H->stream, RT_RESTRICT, op_of(H, l), A.rt_nz[RT_RESTRICT], ra);
    } else {
        launch_resid_restrict<double, false>(H->stream, op_of(H, l), B.lay, cst(A.u), frhs(H, l),
                                             A.phk, nullptr, B.ubar, B.f);
    }
    H->end_timed();
    // with pre-sweeps a coarse level forms the tau correction in its first
    // sweep (two tau-forming half-sweeps, also on a fused level), which reads
    // I u where the restriction left it; the coarsest forms it in its solve's
    // launch
    const bool tau_sweep = l + 1 == H->nlev - 1 || H->cfg.nu1 >= 1;
    if (!tau_sweep)
        launch_tau<double, false>(H->stream, op_of(H, l + 1), cst(B.ubar), B.f, B.u, B.phk,
                                  nullptr);
    cycle64(H, l + 1, fcycle, tau_sweep ? kCycleTauSweep : 0u);
    if (fcycle) cycle64(H, l + 1, false);
    H->begin_timed(PFC_KERNEL_PROLONG0, l);
    launch_prolong<double>(H->stream, B.lay, A.lay, cst(B.u), cst(B.ubar), A.u, H->gate,
                           H->cfg.nu2 >= 1, A.pz[0]);
    H->end_timed();
    for (int s = 0; s < H->cfg.nu2; ++s)
        sweep64(H, l, (flags & kCyclePostNorm) && s == H->cfg.nu2 - 1 ? 2 : 0,
                s + 1 < H->cfg.nu2);
}

void restrict_phk(pfc_handle *H) {
    for (int l = 0; l + 1 < H->nlev; ++l)
        launch_restrict<double>(H->stream, H->lev[l].lay, H->lev[l + 1].lay, H->lev[l].phk,
                                H->lev[l + 1].phk);
}

// phi* of the variable mobility on every level below `from` by 8-child means.
static void restrict_phs(pfc_handle *H, int from) {
    for (int l = from; l + 1 < H->nlev; ++l)
        launch_restrict<double>(H->stream, H->lev[l].lay, H->lev[l + 1].lay, H->lev[l].phs,
                                H->lev[l + 1].phs);
    for (int l = from; l < H->nlev; ++l) H->lev[l].phs_set = true;
}

static bool mobility_on(const pfc_handle *H) { return H->cfg.mobility == PFC_MOBILITY_QUADRATIC; }

pfc_status read_norm(pfc_handle *H, int partials, double *out) {
    launch_max_final(H->stream, H->partial, partials, H->d_scal);
    HIP_TRY(H, hipGetLastError());
    HIP_TRY(H, hipMemcpyAsync(H->h_pin, H->d_scal, sizeof(double), hipMemcpyDeviceToHost,
                              H->stream));
    HIP_TRY(H, hipStreamSynchronize(H->stream));
    H->collect_timings();
    *out = H->h_pin[0];
    return PFC_OK;
}

// Per-workgroup maxima of |S - N(u)| at the finest level into dst (default
// H->partial; written to r too if r.a is set); returns their count.
static int enqueue_norm(pfc_handle *H, Tri<double> r, unsigned long long *dst = nullptr) {
    if (!dst) dst = H->partial;
    Level &A = H->lev[0];
    H->begin_timed(PFC_KERNEL_NORM0, 0);
    int cnt;
    if (A.rt && A.n >= kTileNormMinN && !r.a) {
        ResidTileArgs ra;
        ra.u = cst(A.u);
        ra.f = frhs(H, 0);
        ra.phk = A.phk;
        ra.partial = dst;
        cnt = launch_resid_tile(H->stream, RT_NORM, op_of(H, 0), A.rt_nz[RT_NORM], ra);
    } else {
        cnt = launch_resid_max<double, false>(H->stream, op_of(H, 0), cst(A.u), frhs(H, 0), A.phk,
                                              nullptr, r, dst);
    }
    H->end_timed();
    return cnt;
}

int enqueue_norm64(pfc_handle *H, unsigned long long *dst) {
    return enqueue_norm(H, Tri<double>{nullptr, nullptr, nullptr}, dst);
}

// Residual max-norm at the finest level (r.a may be null).  Synchronises.
pfc_status resid_norm64(pfc_handle *H, Tri<double> r, double *out) {
    return read_norm(H, enqueue_norm(H, r), out);
}

}  // namespace pfc

// ----------------------------------------------------- layout helpers

static void to_level0(pfc_handle *H, const double *phi, const double *mu, const double *om) {
    Level &A = H->lev[0];
    launch_to_lay<double, double>(H->stream, A.lay, phi, A.u.a, 1);
    launch_to_lay<double, double>(H->stream, A.lay, mu, A.u.b, 1);
    launch_to_lay<double, double>(H->stream, A.lay, om, A.u.c, 1);
}

static void from_level0(pfc_handle *H, double *phi, double *mu, double *om) {
    Level &A = H->lev[0];
    launch_from_lay<double, double>(H->stream, A.lay, A.u.a, phi, 1);
    launch_from_lay<double, double>(H->stream, A.lay, A.u.b, mu, 1);
    launch_from_lay<double, double>(H->stream, A.lay, A.u.c, om, 1);
}

namespace pfc {
void step_begin(pfc_handle *H, const double *phi_prev, const double *phi_cur, const double *mu,
                const double *omega) {
    Level &A = H->lev[0];
    // The coarsest level's cached Newton inverse carries over from the
    // previous step: the chord iteration rebuilds it wherever an update
    // contracts by less than 4x, so a stale inverse costs iterations, never
    // accuracy (each solve still runs to its 1e-14 update bound).
    launch_source(H->stream, op_of(H, 0), phi_cur, phi_prev, A.f);
    to_level0(H, phi_cur, mu, omega);
    launch_to_lay<double, double>(H->stream, A.lay, phi_cur, A.phk, 1);
    H->f1_phk = true;  // f.a and phk now hold the same phi^k
    restrict_phk(H);
    if (mobility_on(H)) {
        launch_phistar(H->stream, A.lay, phi_cur, phi_prev, A.phs);
        restrict_phs(H, 0);
    }
}
void step_end(pfc_handle *H, double *phi_next, double *mu, double *omega) {
    from_level0(H, phi_next, mu, omega);
}
}  // namespace pfc

// ------------------------------------------------------------- C ABI

extern "C" {

const char *pfc_status_string(pfc_status s) {
    switch (s) {
        case PFC_OK: return "ok";
        case PFC_ERR_INVALID_ARG: return "invalid argument";
        case PFC_ERR_NOT_CONVERGED: return "not converged within max_cycles";
        case PFC_ERR_NONFINITE: return "residual is not finite";
        case PFC_ERR_HIP: return "HIP runtime error";
        case PFC_ERR_OOM: return "out of memory";
        default: return "unknown status";
    }
}

const char *pfc_last_error(const pfc_handle *h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

pfc_status pfc_create(const pfc_config *cfg, void *stream, pfc_handle **out) {
    if (!out) return fail(nullptr, PFC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    const std::string why = validate_config(cfg);
    if (!why.empty()) return fail(nullptr, PFC_ERR_INVALID_ARG, why);
    pfc_handle *H = new pfc_handle();
    H->cfg = *cfg;
    H->stream = (hipStream_t)stream;
    if (hipGetDevice(&H->device) != hipSuccess) {
        delete H;
        return fail(nullptr, PFC_ERR_HIP, "hipGetDevice failed");
    }
    std::vector<int> sizes;
    level_sizes(cfg->n, sizes);
    H->nlev = (int)sizes.size();
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) device = 0;
    const bool mob = cfg->mobility == PFC_MOBILITY_QUADRATIC;
    const int slots = fused_slots(device, mob);
    int rt_slots[RT_MODES];
    for (int m = 0; m < RT_MODES; ++m) rt_slots[m] = resid_tile_slots(device, m, mob);
    const int pt_slots[2] = {prolong_tile_slots(device, false), prolong_tile_slots(device, true)};
    bool ok = true;
    for (int l = 0; l < H->nlev && ok; ++l) {
        Level &A = H->lev[l];
        A.n = sizes[l];
        A.h = cfg->L / A.n;
        A.h2inv = 1.0 / (A.h * A.h);
        A.P = (size_t)A.n * A.n * A.n;
        A.lay = make_lay(A.n, l < H->nlev - 1);
        double *u, *f, *ub;
        ok = dalloc(H, &u, 3 * A.P) && dalloc(H, &f, 3 * A.P) && dalloc(H, &ub, 3 * A.P) &&
             dalloc(H, &A.phk, A.P);
        if (ok && cfg->mobility == PFC_MOBILITY_QUADRATIC) ok = dalloc(H, &A.phs, A.P);
        if (!ok) break;
        A.u = Tri<double>{u, u + A.P, u + 2 * A.P};
        A.f = Tri<double>{f, f + A.P, f + 2 * A.P};
        A.ubar = Tri<double>{ub, ub + A.P, ub + 2 * A.P};
        A.rt = resid_tile_fits(A.lay);
        for (int m = 0; m < RT_MODES; ++m) A.rt_nz[m] = resid_tile_nz(A.n, rt_slots[m], m);
        if (l + 1 < H->nlev)
            for (int t = 0; t < 2; ++t) A.pz[t] = prolong_tile_nzr(pt_slots[t], A.n / 2, A.n);
        A.fused = l < H->nlev - 1 && fused_fits(A.n);
        if (A.fused || (l == 0 && A.rt)) {
            A.nz = fused_nz(A.n, slots);
            double *u2;
            ok = dalloc(H, &u2, 3 * A.P);
            if (!ok) break;
            A.u2 = Tri<double>{u2, u2 + A.P, u2 + 2 * A.P};
        }
    }
    ok = ok && dalloc(H, &H->partial, (size_t)3 * kMaxReduceBlocks + 16);
    if (ok) {  // the split stop test (the graph loop seeds it behind both halves)
        const Level &A = H->lev[0];
        H->split_blocks = A.fused ? fused_blocks(A.n, A.nz) : 0;
        H->split_norm = A.fused && cfg->nu1 >= 1 && cfg->nu2 >= 1 &&
                        cfg->precision == PFC_FP64 && H->split_blocks <= kMaxReduceBlocks;
    }
    ok = ok && dalloc(H, &H->d_scal, 16) && dalloc(H, &H->d_iters, 4);
    ok = ok && dalloc(H, &H->energy_part, (size_t)6 * kMaxReduceBlocks + 16);
    ok = ok && dalloc(H, &H->minv64, 64 * 64) && dalloc(H, &H->minv32, 64 * 64) &&
         dalloc(H, &H->valid64, 4) && dalloc(H, &H->valid32, 4) &&
         dalloc(H, &H->minv_adj, 64 * 64) && dalloc(H, &H->valid_adj, 4);
    std::vector<double> l1, l2, l3;
    if (ok) {
        const Level &C = H->lev[H->nlev - 1];
        coarse_matrices(C.n, C.h, l1, l2, l3);
        ok = dalloc(H, &H->lap1, l1.size()) && dalloc(H, &H->lap2, l2.size()) &&
             dalloc(H, &H->lap3, l3.size());
    }
    if (ok && hipHostMalloc((void **)&H->h_pin, 64 * sizeof(double), 0) != hipSuccess) {
        H->h_pin = nullptr;
        ok = false;
    }
    if (!ok) {
        delete H;
        return fail(nullptr, PFC_ERR_OOM, "device or pinned allocation failed");
    }
    if (hipMemcpy(H->lap1, l1.data(), l1.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(H->lap2, l2.data(), l2.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(H->lap3, l3.data(), l3.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(H->valid64, 0, sizeof(int)) != hipSuccess ||
        hipMemset(H->valid32, 0, sizeof(int)) != hipSuccess) {
        delete H;
        return fail(nullptr, PFC_ERR_HIP, "initialisation of coarse-level data failed");
    }
    if (cfg->precision == PFC_MIXED) {
        const pfc_status st = mixed_init(H);
        if (st != PFC_OK) {
            g_create_error = H->err;
            delete H;
            return st;
        }
    }
    *out = H;
    return PFC_OK;
}

pfc_status pfc_destroy(pfc_handle *h) {
    if (!h) return PFC_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(h->stream);
    delete h;
    return PFC_OK;
}

pfc_status pfc_set_stream(pfc_handle *h, void *stream) {
    if (!h) return PFC_ERR_INVALID_ARG;
    h->stream = (hipStream_t)stream;
    return PFC_OK;
}

int32_t pfc_num_levels(const pfc_handle *h) { return h ? h->nlev : 0; }

int32_t pfc_level_size(const pfc_handle *h, int32_t level) {
    if (!h || level < 0 || level >= h->nlev) return 0;
    return h->lev[level].n;
}

pfc_status pfc_init_guess(pfc_handle *h, const double *phi0, double *mu, double *omega) {
    if (!h) return PFC_ERR_INVALID_ARG;
    if (!phi0 || !mu || !omega) return fail(h, PFC_ERR_INVALID_ARG, "NULL field pointer");
    OpParams nat = op_of(h, 0);
    nat.lay = make_lay(h->lev[0].n, false);
    launch_init_guess(h->stream, nat, phi0, mu, omega);
    HIP_TRY(h, hipGetLastError());
    return PFC_OK;
}

pfc_status pfc_step(pfc_handle *h, const double *phi_prev, const double *phi_cur, double *phi_next,
                    double *mu, double *omega, pfc_step_info *info) {
    if (!h) return PFC_ERR_INVALID_ARG;
    if (!phi_prev || !phi_cur || !phi_next || !mu || !omega)
        return fail(h, PFC_ERR_INVALID_ARG, "NULL field pointer");
    if (phi_next == phi_cur || phi_next == phi_prev)
        return fail(h, PFC_ERR_INVALID_ARG, "phi_next aliases an input");
    if (h->cfg.precision == PFC_MIXED)
        return mixed_step(h, phi_prev, phi_cur, phi_next, mu, omega, info);
    return step64(h, phi_prev, phi_cur, phi_next, mu, omega, info);
}

}  // extern "C"

namespace pfc {
// One FP64 time step with the cycle loop on the host (one 8-byte read-back
// per cycle).
pfc_status step64(pfc_handle *h, const double *phi_prev, const double *phi_cur, double *phi_next,
                  double *mu, double *omega, pfc_step_info *info) {
    step_begin(h, phi_prev, phi_cur, mu, omega);
    HIP_TRY(h, hipGetLastError());
    int c = 0;
    double rho = 0, rho0 = 0;
    pfc_status status = PFC_OK;
    // With the split stop test, the norm after a cycle is completed by the next
    // cycle's first pre-sweep, launched before the decision; when the loop then
    // stops, that sweep's output is dropped (its input buffer is untouched).
    bool ahead = false;
    {
        const pfc_status st = resid_norm64(h, Tri<double>{nullptr, nullptr, nullptr}, &rho);
        if (st != PFC_OK) return st;
    }
    for (;;) {
        if (c == 0) rho0 = rho;
        if (!std::isfinite(rho)) {
            status = PFC_ERR_NONFINITE;
            break;
        }
        if (rho <= h->cfg.tol) break;
        if (c == h->cfg.max_cycles) {
            status = PFC_ERR_NOT_CONVERGED;
            break;
        }
        const bool split = h->split_norm && c + 1 < h->cfg.max_cycles;
        cycle64(h, 0, h->cfg.cycle == PFC_CYCLE_F,
                (ahead ? kCyclePreDone : 0u) | (split ? kCyclePostNorm : 0u));
        ++c;
        pfc_status st;
        if (split) {
            // the first pre-sweep of the next cycle; a second pre-sweep follows it
            // when nu1 >= 2 (and if the loop stops its output is dropped)
            sweep64(h, 0, 1, h->cfg.nu1 >= 2);
            ahead = true;
            st = read_norm(h, 2 * h->split_blocks, &rho);
        } else {
            ahead = false;
            st = resid_norm64(h, Tri<double>{nullptr, nullptr, nullptr}, &rho);
        }
        if (st != PFC_OK) return st;
    }
    if (ahead) std::swap(h->lev[0].u, h->lev[0].u2);
    step_end(h, phi_next, mu, omega);
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (info) {
        info->cycles = c;
        info->status = status;
        info->res0 = rho0;
        info->res_final = rho;
    }
    if (status != PFC_OK) fail(h, status, pfc_status_string(status));
    return status;
}
}  // namespace pfc

extern "C" {

pfc_status pfc_fas_vcycle(pfc_handle *h, double *u3, const double *f3, const double *phi_cur,
                          double *res_after) {
    if (!h) return PFC_ERR_INVALID_ARG;
    h->f1_phk = false;  // the caller's right-hand side goes into f
    if (!u3 || !f3 || !phi_cur) return fail(h, PFC_ERR_INVALID_ARG, "NULL field pointer");
    if (mobility_on(h) && !h->lev[0].phs_set)
        return fail(h, PFC_ERR_INVALID_ARG, "variable mobility: phi* not set at level 0");
    Level &A = h->lev[0];
    launch_to_lay<double, double>(h->stream, A.lay, u3, A.u.a, 3);
    launch_to_lay<double, double>(h->stream, A.lay, f3, A.f.a, 3);
    launch_to_lay<double, double>(h->stream, A.lay, phi_cur, A.phk, 1);
    restrict_phk(h);
    cycle64(h, 0, h->cfg.cycle == PFC_CYCLE_F);
    launch_from_lay<double, double>(h->stream, A.lay, A.u.a, u3, 3);
    HIP_TRY(h, hipGetLastError());
    if (res_after) {
        const pfc_status st = resid_norm64(h, Tri<double>{nullptr, nullptr, nullptr}, res_after);
        if (st != PFC_OK) return st;
    }
    return PFC_OK;
}

pfc_status pfc_energy(pfc_handle *h, const double *phi, const double *phi_prev, double *out) {
    if (!h) return PFC_ERR_INVALID_ARG;
    if (!phi || !out) return fail(h, PFC_ERR_INVALID_ARG, "NULL pointer");
    const Level &A = h->lev[0];
    launch_energy(h->stream, make_lay(A.n, false), A.h, h->cfg.eps, phi, phi_prev, h->energy_part,
                  h->d_scal);
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipMemcpyAsync(h->h_pin, h->d_scal, 3 * sizeof(double), hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    out[0] = h->h_pin[0];
    out[1] = h->h_pin[1];
    out[2] = h->h_pin[2];
    return PFC_OK;
}

// ---------------------------------------------- kernel-level entry points
// Inputs arrive in natural order; they are converted into the level's own
// buffers (its storage layout), the kernel runs there, and outputs are
// converted back.

static bool level_ok(const pfc_handle *h, int level) { return level >= 0 && level < h->nlev; }

pfc_status pfc_source(pfc_handle *h, const double *phi_prev, const double *phi_cur, double *f3) {
    if (!h) return PFC_ERR_INVALID_ARG;
    if (!phi_prev || !phi_cur || !f3) return fail(h, PFC_ERR_INVALID_ARG, "NULL pointer");
    OpParams nat = op_of(h, 0);
    nat.lay = make_lay(h->lev[0].n, false);
    const size_t P = h->lev[0].P;
    launch_source(h->stream, nat, phi_cur, phi_prev, Tri<double>{f3, f3 + P, f3 + 2 * P});
    HIP_TRY(h, hipGetLastError());
    return PFC_OK;
}

pfc_status pfc_residual(pfc_handle *h, int32_t level, const double *u3, const double *f3,
                        const double *phk, double *r3, double *maxnorm) {
    if (!h) return PFC_ERR_INVALID_ARG;
    h->f1_phk = false;  // the caller's right-hand side goes into f
    if (!level_ok(h, level) || !u3 || !f3 || !phk) return fail(h, PFC_ERR_INVALID_ARG, "bad argument");
    if (mobility_on(h) && !h->lev[level].phs_set)
        return fail(h, PFC_ERR_INVALID_ARG, "variable mobility: phi* not set at this level");
    Level &A = h->lev[level];
    launch_to_lay<double, double>(h->stream, A.lay, u3, A.u.a, 3);
    launch_to_lay<double, double>(h->stream, A.lay, f3, A.f.a, 3);
    launch_to_lay<double, double>(h->stream, A.lay, phk, A.phk, 1);
    Tri<double> r{nullptr, nullptr, nullptr};
    if (r3) r = A.ubar;
    int cnt;
    if (!r3 && A.rt && A.n >= kTileNormMinN) {  // norm only: the kernel the cycles use
        ResidTileArgs ra;
        ra.u = cst(A.u);
        ra.f = cst(A.f);
        ra.phk = A.phk;
        ra.partial = h->partial;
        cnt = launch_resid_tile(h->stream, RT_NORM, op_of(h, level), A.rt_nz[RT_NORM], ra);
    } else {
        cnt = launch_resid_max<double, false>(h->stream, op_of(h, level), cst(A.u), cst(A.f), A.phk,
                                              nullptr, r, h->partial);
    }
    if (r3) launch_from_lay<double, double>(h->stream, A.lay, A.ubar.a, r3, 3);
    HIP_TRY(h, hipGetLastError());
    double m = 0;
    const pfc_status st = read_norm(h, cnt, &m);
    if (st != PFC_OK) return st;
    if (maxnorm) *maxnorm = m;
    return PFC_OK;
}

pfc_status pfc_smooth(pfc_handle *h, int32_t level, int32_t colour, double *u3, const double *f3,
                      const double *phk) {
    if (!h) return PFC_ERR_INVALID_ARG;
    h->f1_phk = false;  // the caller's right-hand side goes into f
    if (!level_ok(h, level) || colour < 0 || colour > PFC_SWEEP_FULL || !u3 || !f3 || !phk ||
        !h->lev[level].lay.split)
        return fail(h, PFC_ERR_INVALID_ARG, "bad argument (level must be a smoothed level)");
    if (mobility_on(h) && !h->lev[level].phs_set)
        return fail(h, PFC_ERR_INVALID_ARG, "variable mobility: phi* not set at this level");
    Level &A = h->lev[level];
    launch_to_lay<double, double>(h->stream, A.lay, u3, A.u.a, 3);
    launch_to_lay<double, double>(h->stream, A.lay, f3, A.f.a, 3);
    launch_to_lay<double, double>(h->stream, A.lay, phk, A.phk, 1);
    if (colour == PFC_SWEEP_FULL)
        sweep64(h, level);
    else
        launch_smooth<double, false>(h->stream, op_of(h, level), colour,
                                     h->cfg.lin == PFC_LIN_PICARD, A.u, cst(A.f), A.phk, nullptr);
    launch_from_lay<double, double>(h->stream, A.lay, A.u.a, u3, 3);
    HIP_TRY(h, hipGetLastError());
    return PFC_OK;
}

pfc_status pfc_restrict(pfc_handle *h, int32_t level, const double *fine, double *coarse,
                        int32_t ncomp) {
    if (!h) return PFC_ERR_INVALID_ARG;
    if (!level_ok(h, level) || level + 1 >= h->nlev || !fine || !coarse || ncomp < 1 || ncomp > 3)
        return fail(h, PFC_ERR_INVALID_ARG, "bad argument");
    Level &A = h->lev[level], &B = h->lev[level + 1];
    launch_to_lay<double, double>(h->stream, A.lay, fine, A.u.a, ncomp);
    for (int c = 0; c < ncomp; ++c)
        launch_restrict<double>(h->stream, A.lay, B.lay, A.u.a + c * A.P, B.u.a + c * B.P);
    launch_from_lay<double, double>(h->stream, B.lay, B.u.a, coarse, ncomp);
    HIP_TRY(h, hipGetLastError());
    return PFC_OK;
}

pfc_status pfc_prolong_add(pfc_handle *h, int32_t level, const double *coarse_v,
                           const double *coarse_ubar, double *fine, int32_t ncomp) {
    if (!h) return PFC_ERR_INVALID_ARG;
    if (!level_ok(h, level) || level + 1 >= h->nlev || !coarse_v || !fine ||
        (ncomp != 1 && ncomp != 3))
        return fail(h, PFC_ERR_INVALID_ARG, "bad argument");
    Level &A = h->lev[level], &B = h->lev[level + 1];
    launch_to_lay<double, double>(h->stream, B.lay, coarse_v, B.u.a, ncomp);
    if (coarse_ubar) launch_to_lay<double, double>(h->stream, B.lay, coarse_ubar, B.ubar.a, ncomp);
    launch_to_lay<double, double>(h->stream, A.lay, fine, A.u.a, ncomp);
    const Tri<const double> none{nullptr, nullptr, nullptr};
    if (ncomp == 3) {
        launch_prolong<double>(h->stream, B.lay, A.lay, cst(B.u), coarse_ubar ? cst(B.ubar) : none,
                               A.u, nullptr, false, A.pz[0]);
    } else {
        launch_prolong<double>(h->stream, B.lay, A.lay, Tri<const double>{B.u.a, nullptr, nullptr},
                               Tri<const double>{coarse_ubar ? B.ubar.a : nullptr, nullptr, nullptr},
                               Tri<double>{A.u.a, nullptr, nullptr});
    }
    launch_from_lay<double, double>(h->stream, A.lay, A.u.a, fine, ncomp);
    HIP_TRY(h, hipGetLastError());
    return PFC_OK;
}

pfc_status pfc_coarse_solve(pfc_handle *h, double *u3, const double *f3, const double *phk,
                            int32_t *iters) {
    if (!h) return PFC_ERR_INVALID_ARG;
    if (!u3 || !f3 || !phk) return fail(h, PFC_ERR_INVALID_ARG, "NULL pointer");
    const int l = h->nlev - 1;
    if (mobility_on(h) && !h->lev[l].phs_set)
        return fail(h, PFC_ERR_INVALID_ARG, "variable mobility: phi* not set at the coarsest level");
    const size_t P = h->lev[l].P;
    invalidate_coarse(h);
    launch_coarse<double, false>(h->stream, op_of(h, l), Tri<double>{u3, u3 + P, u3 + 2 * P},
                                 Tri<const double>{f3, f3 + P, f3 + 2 * P}, phk, nullptr, h->lap1,
                                 h->lap3, h->minv64, nullptr, h->valid64, h->d_iters, h->lap2);
    HIP_TRY(h, hipGetLastError());
    if (iters) {
        HIP_TRY(h, hipMemcpyAsync(h->h_pin, h->d_iters, sizeof(int), hipMemcpyDeviceToHost,
                                  h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        std::memcpy(iters, h->h_pin, sizeof(int));
    }
    return PFC_OK;
}

pfc_status pfc_reset_coarse_cache(pfc_handle *h) {
    if (!h) return PFC_ERR_INVALID_ARG;
    invalidate_coarse(h);
    HIP_TRY(h, hipGetLastError());
    return PFC_OK;
}

pfc_status pfc_set_phistar(pfc_handle *h, int32_t level, const double *phs) {
    if (!h) return PFC_ERR_INVALID_ARG;
    if (!mobility_on(h)) return fail(h, PFC_ERR_INVALID_ARG, "the handle has constant mobility");
    if (!level_ok(h, level) || !phs) return fail(h, PFC_ERR_INVALID_ARG, "bad argument");
    invalidate_coarse(h);
    launch_to_lay<double, double>(h->stream, h->lev[level].lay, phs, h->lev[level].phs, 1);
    restrict_phs(h, level);
    HIP_TRY(h, hipGetLastError());
    return PFC_OK;
}

// ------------------------------------------------------- instrumentation

pfc_status pfc_timing_enable(pfc_handle *h, int32_t on) {
    if (!h) return PFC_ERR_INVALID_ARG;
    h->timing = on != 0;
    return PFC_OK;
}

pfc_status pfc_timing_reset(pfc_handle *h) {
    if (!h) return PFC_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(h->stream);
    h->collect_timings();
    for (int k = 0; k < PFC_KERNEL_COUNT; ++k) {
        h->t_count[k] = 0;
        h->t_ms[k] = 0;
        h->t_bytes[k] = 0;
    }
    return PFC_OK;
}

pfc_status pfc_timing_get(pfc_handle *h, int32_t kernel, int64_t *launches, double *total_ms,
                          double *bytes_per_launch) {
    if (!h || kernel < 0 || kernel >= PFC_KERNEL_COUNT) return PFC_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(h->stream);
    h->collect_timings();
    if (launches) *launches = h->t_count[kernel];
    if (total_ms) *total_ms = h->t_ms[kernel];
    if (bytes_per_launch)
        *bytes_per_launch = h->t_count[kernel] ? h->t_bytes[kernel] / (double)h->t_count[kernel]
                                               : algorithmic_bytes(h, kernel);
    return PFC_OK;
}

}  // extern "C"
