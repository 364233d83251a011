// Handle layout shared by the host-side translation units of the runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "pfc.h"
#include "pfc_internal.h"

namespace pfc {

constexpr int kMaxLevels = 24;

// One level of the multigrid hierarchy (FP64 storage).  Level 0 binds the
// caller's buffers per call; coarser levels own theirs.
struct Level {
    int n = 0;
    double h = 0, h2inv = 0;
    size_t P = 0;
    Tri<double> u{nullptr, nullptr, nullptr};     // iterate
    Tri<double> f{nullptr, nullptr, nullptr};     // right-hand side
    Tri<double> ubar{nullptr, nullptr, nullptr};  // restricted fine iterate I u
    double *phk = nullptr;                        // phi^kappa on this level
};

// One level of the FP32 correction cycle of the mixed-precision form.
struct Level32 {
    Tri<float> e{nullptr, nullptr, nullptr};     // correction iterate
    Tri<float> f{nullptr, nullptr, nullptr};     // right-hand side
    Tri<float> ebar{nullptr, nullptr, nullptr};  // restricted fine correction
    float *phk = nullptr;                        // phi^kappa
    float *base = nullptr;                       // FP64 iterate's phi, rounded/restricted
};

struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
};

bool level_sizes(int n, std::vector<int> &out);
std::string validate_config(const pfc_config *c);
void coarse_matrices(int n, double h, std::vector<double> &l1, std::vector<double> &l3);

}  // namespace pfc

struct pfc_handle {
    pfc_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    int nlev = 0;
    pfc::Level lev[pfc::kMaxLevels];
    pfc::Level32 lev32[pfc::kMaxLevels];
    std::vector<void *> allocs;
    pfc::Tri<double> f0{nullptr, nullptr, nullptr};  // finest-level source
    pfc::Tri<double> r0{nullptr, nullptr, nullptr};  // finest-level FP64 residual (mixed form)
    unsigned long long *partial = nullptr;
    double *d_scal = nullptr;
    int *d_iters = nullptr;
    double *h_pin = nullptr;
    double *lap1 = nullptr, *lap3 = nullptr;
    double *energy_part = nullptr;
    std::string err;
    // instrumentation
    bool timing = false;
    int cur_event = -1;
    std::vector<pfc::TimedLaunch> pending;
    std::vector<hipEvent_t> pool;
    int64_t t_count[PFC_KERNEL_COUNT] = {0, 0, 0, 0, 0};
    double t_ms[PFC_KERNEL_COUNT] = {0, 0, 0, 0, 0};

    void begin_timed(int kind, int level);
    void end_timed();
    void collect_timings();
    ~pfc_handle();
};

namespace pfc {
void cycle64(pfc_handle *H, int l, bool fcycle);
void restrict_phk(pfc_handle *H);
pfc_status resid_norm64(pfc_handle *H, Tri<double> r, double *out);
pfc_status mixed_init(pfc_handle *H);
pfc_status mixed_step(pfc_handle *H, const double *phi_prev, const double *phi_cur,
                      double *phi_next, double *mu, double *omega, pfc_step_info *info);
double algorithmic_bytes(const pfc_handle *H, int kernel);
}  // namespace pfc
