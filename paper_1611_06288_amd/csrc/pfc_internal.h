// Internal interface between the HIP kernels (kernels.hip) and the host
// runtime (runtime.cpp).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pfc {

// Three grid functions (phi, mu, omega) of one level.
template <typename T>
struct Tri {
    T *a;  // phi (or its correction)
    T *b;  // mu
    T *c;  // omega
};

template <typename T>
inline Tri<const T> cst(Tri<T> t) { return Tri<const T>{t.a, t.b, t.c}; }

// Scalar parameters of one level's operator.
struct OpParams {
    int n;         // cells per axis on this level
    double h2inv;  // 1 / h_l^2
    double tau;    // time step
    double eps;    // epsilon
};

constexpr int kBlock = 256;

// ---- FP64 / FP32 building blocks (T = double or float; DELTA selects the
// correction form g(base + e) - g(base) of the cubic term) ----
template <typename T, bool DELTA>
void launch_smooth(hipStream_t s, const OpParams &op, int colour, int picard, Tri<T> u,
                   Tri<const T> f, const T *phk, const T *base);

template <typename T, bool DELTA>
void launch_resid_restrict(hipStream_t s, const OpParams &op, Tri<const T> u, Tri<const T> f,
                           const T *phk, const T *base, Tri<T> ubar_c, Tri<T> rr_c);

template <typename T>
void launch_restrict(hipStream_t s, int nf, const T *fine, T *coarse);

template <typename T, bool DELTA>
void launch_tau(hipStream_t s, const OpParams &opc, Tri<const T> ubar, Tri<T> f, Tri<T> u,
                const T *phk, const T *base);

template <typename T>
void launch_prolong(hipStream_t s, int nc, Tri<const T> v, Tri<const T> ubar, Tri<T> fine);

// Residual r = f - N(u) (r may have null members) and per-block maxima of |r|
// as IEEE bit patterns; returns the number of partials written.
template <typename T, bool DELTA>
int launch_resid_max(hipStream_t s, const OpParams &op, Tri<const T> u, Tri<const T> f,
                     const T *phk, const T *base, Tri<T> r, unsigned long long *partial);

void launch_max_final(hipStream_t s, const unsigned long long *partial, int count, double *out);

template <typename T, bool DELTA>
void launch_coarse(hipStream_t s, const OpParams &op, Tri<T> u, Tri<const T> f, const T *phk,
                   const T *base, const double *lap1, const double *lap3, int *iters);

void launch_source(hipStream_t s, const OpParams &op, const double *phk, const double *phkm1,
                   Tri<double> f);
void launch_init_guess(hipStream_t s, const OpParams &op, const double *phi0, double *mu,
                       double *om);

// Energy: per-block partial sums (6 per block) then a fixed-order final sum.
int energy_blocks(int n);
void launch_energy(hipStream_t s, int n, double h, double eps, const double *phi,
                   const double *phi_prev, double *partial, double *out3);

}  // namespace pfc
