// Handle layout shared by the host-side translation units of the runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "pfc.h"
#include "pfc_internal.h"

namespace pfc {

constexpr int kMaxLevels = 24;

// One level of the FP64 multigrid hierarchy.  Smoothed levels are stored
// colour-split, the coarsest level in natural order.
struct Level {
    int n = 0;
    double h = 0, h2inv = 0;
    size_t P = 0;
    Lay lay{};
    Tri<double> u{nullptr, nullptr, nullptr};     // iterate
    Tri<double> f{nullptr, nullptr, nullptr};     // right-hand side
    Tri<double> ubar{nullptr, nullptr, nullptr};  // restricted fine iterate I u (scratch on level 0)
    Tri<double> u2{nullptr, nullptr, nullptr};    // second iterate buffer (fused sweeps, fused correction)
    double *phk = nullptr;                        // phi^kappa on this level
    double *phs = nullptr;                        // phi* of the variable mobility (else null)
    bool phs_set = false;                         // phs holds a field
    bool fused = false;                           // smoothed by the fused red-black sweep
    int nz = 1;                                   // its plane ranges per column
    bool rt = false;                              // residuals by column tiles
    int rt_nz[RT_MODES] = {1, 1, 1, 1, 1};        // their plane ranges, per epilogue
    int pz[2] = {0, 0};  // plane ranges of the tiled interpolation onto this level (FP64, FP32)
};

// One level of the FP32 correction cycle of the mixed-precision form.
struct Level32 {
    Tri<float> e{nullptr, nullptr, nullptr};     // correction iterate
    Tri<float> f{nullptr, nullptr, nullptr};     // right-hand side
    Tri<float> ebar{nullptr, nullptr, nullptr};  // restricted fine correction
    float *phk = nullptr;                        // phi^kappa
    float *base = nullptr;                       // FP64 iterate's phi, rounded and restricted
};

struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
    double bytes;  // the launch's algorithmic HBM bytes
};

bool level_sizes(int n, std::vector<int> &out);
std::string validate_config(const pfc_config *c);
void coarse_matrices(int n, double h, std::vector<double> &l1, std::vector<double> &l2,
                     std::vector<double> &l3);

}  // namespace pfc

struct pfc_handle {
    pfc_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    int nlev = 0;
    pfc::Level lev[pfc::kMaxLevels];
    pfc::Level32 lev32[pfc::kMaxLevels];
    std::vector<void *> allocs;
    unsigned long long *partial = nullptr;
    double *d_scal = nullptr;
    int *d_iters = nullptr;
    double *h_pin = nullptr;
    double *lap1 = nullptr, *lap2 = nullptr, *lap3 = nullptr;
    double *minv64 = nullptr, *minv32 = nullptr;  // cached coarsest Newton inverses
    int *valid64 = nullptr, *valid32 = nullptr;
    double *minv_adj = nullptr;  // cached coarsest inverse of the adjoint solve
    int *valid_adj = nullptr;
    double *energy_part = nullptr;
    // stop test split over the finest level's fused sweeps (FP64, M = 1): the
    // last post-sweep of a cycle leaves the colour-1 half of the norm in
    // partial[split_blocks .. 2 split_blocks), the next cycle's first
    // pre-sweep, run ahead of the decision, the colour-0 half in
    // partial[0 .. split_blocks)
    bool split_norm = false;
    // Set by a time step's set-up: the finest level's f.a holds phi^k, a copy
    // of phk (the first component of S is phi^k itself), so the finest-level
    // kernels read phk in its place (see frhs).  Cleared by the entry points
    // that load a caller's right-hand side into the finest level.
    bool f1_phk = false;
    int split_blocks = 0;
    // graph-driven time loop (pfc_run)
    const int *gate = nullptr;            // cycle gate, set only while its graph is recorded
    hipStream_t run_stream = nullptr;     // the loop's own stream (capturable)
    hipEvent_t run_ev = nullptr;
    hipEvent_t norm_ev = nullptr;         // the mixed form's norm copied to the host
    int *d_run = nullptr;                 // active, cycles, status of the current step
    double *d_runres = nullptr;           // res0, res of the current step
    hipGraph_t run_graph = nullptr;       // norm, stop test, one gated cycle
    hipGraphExec_t run_exec = nullptr;
    const void *run_key[pfc::kMaxLevels] = {};  // level iterates the graph was recorded with
    double *spare = nullptr;              // third phi buffer of the loop
    int last_cycles = 0;                  // cycles of the previous step (launch count guess)
    hipGraph_t mix_graph = nullptr;       // one FP32 correction cycle (mixed form)
    hipGraphExec_t mix_exec = nullptr;
    std::string err;
    // instrumentation
    bool timing = false;
    int cur_event = -1;
    std::vector<pfc::TimedLaunch> pending;
    std::vector<hipEvent_t> pool;
    int64_t t_count[PFC_KERNEL_COUNT] = {};
    double t_ms[PFC_KERNEL_COUNT] = {};
    double t_bytes[PFC_KERNEL_COUNT] = {};

    // bytes < 0: the kind's algorithmic bytes per finest-level launch
    void begin_timed(int kind, int level, double bytes = -1.0);
    void end_timed();
    void collect_timings();
    ~pfc_handle();
};

namespace pfc {
OpParams op_of(const pfc_handle *H, int l);
// flags of cycle64 (the first two at the finest level)
constexpr unsigned kCyclePreDone = 1;   // its first pre-sweep has already run (sweep64 nrm 1)
constexpr unsigned kCyclePostNorm = 2;  // its last post-sweep leaves the colour-1 norm half
constexpr unsigned kCycleTauSweep = 8;  // (coarse level) f holds I r and the
                                        // iterate is still in ubar: the first pre-sweep (the
                                        // coarsest: its solve) forms the tau correction and
                                        // reads the old values there
void cycle64(pfc_handle *H, int l, bool fcycle, unsigned flags = 0);
// Level l's right-hand side as its kernels read it.  In a time step the
// first component of the finest level's S is phi^k itself (scheme-PFC-s1),
// held bitwise in both f.a and phk; reading it from phk spares the kernels a
// second 8-byte stream per point (the fused sweep, the residual passes and
// the FP64 defect pass).
inline Tri<const double> frhs(const pfc_handle *H, int l) {
    const Level &A = H->lev[l];
    if (l == 0 && H->f1_phk) return Tri<const double>{A.phk, A.f.b, A.f.c};
    return Tri<const double>{A.f.a, A.f.b, A.f.c};
}

// One smoothing sweep of level l; nrm as in launch_sweep_fused (split_norm
// only); then_sweep: the next operation on the iterate is another sweep of
// this level (a fused sweep then leaves the dead colour-0 mu, omega
// unwritten); tau: a coarse level's first sweep forming the tau correction
// (launch_smooth_tau; on a fused level into the second buffer, which then
// becomes the iterate).
void sweep64(pfc_handle *H, int l, int nrm = 0, bool then_sweep = false,
             bool tau = false);
void restrict_phk(pfc_handle *H);
pfc_status resid_norm64(pfc_handle *H, Tri<double> r, double *out);
int enqueue_norm64(pfc_handle *H, unsigned long long *dst = nullptr);
pfc_status read_norm(pfc_handle *H, int partials, double *out);
pfc_status mixed_init(pfc_handle *H);
pfc_status step64(pfc_handle *h, const double *phi_prev, const double *phi_cur, double *phi_next,
                  double *mu, double *omega, pfc_step_info *info);
// The handle's own non-blocking stream (created on first use): recorded
// graphs need a capturable stream.  own_stream_enter makes it follow the
// caller's stream and returns that stream; own_stream_leave makes the caller's
// stream follow it again.
pfc_status own_stream_enter(pfc_handle *H, hipStream_t *user);
pfc_status own_stream_leave(pfc_handle *H, hipStream_t user);
pfc_status mixed_step(pfc_handle *H, const double *phi_prev, const double *phi_cur,
                      double *phi_next, double *mu, double *omega, pfc_step_info *info);
double algorithmic_bytes(const pfc_handle *H, int kernel);
// Finest-level set-up of one time step (source, layout conversion of the
// guess and of phi^k, phi^k hierarchy) and the conversion back.
void step_begin(pfc_handle *H, const double *phi_prev, const double *phi_cur, const double *mu,
                const double *omega);
void step_end(pfc_handle *H, double *phi_next, double *mu, double *omega);
void invalidate_coarse(pfc_handle *H);
template <typename T>
bool dalloc(pfc_handle *H, T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return false;
    H->allocs.push_back(q);
    *p = (T *)q;
    return true;
}
pfc_status fail(pfc_handle *H, pfc_status st, const std::string &msg);
pfc_status hip_fail(pfc_handle *H, hipError_t e, const char *what);
}  // namespace pfc

#define HIP_TRY(H, expr)                                                  \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) return pfc::hip_fail((H), e_, #expr);       \
    } while (0)
