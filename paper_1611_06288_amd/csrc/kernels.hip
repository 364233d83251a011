// HIP kernels (gfx950) for the FAS multigrid solve of one step of the
// second-order PFC scheme (arXiv:1611.06288, Sections 2, 3 and 5).
//
// Every kernel is a 7-point stencil, a transfer or a reduction: memory bound,
// no matrix-core work.  One thread per grid point (or per point of one
// red-black colour, or per coarse cell) on 256-thread workgroups; workgroup
// ids are remapped so that each of the 8 XCDs receives a contiguous range of
// z-planes (neighbouring planes share halo lines in that XCD's L2).
//
// Storage type T is double (FP64 path) or float (mixed-precision cycle);
// all operator arithmetic and the pointwise 3x3 solve run in FP64.
#include "pfc_internal.h"

#include <math.h>

namespace pfc {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ unsigned xcd_block() {
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned per = nb >> 3;
    if (b < (per << 3)) return (b & 7u) * per + (b >> 3);
    return b;
}

__device__ __forceinline__ int wrap_p(int i, int n) { return i == n - 1 ? 0 : i + 1; }
__device__ __forceinline__ int wrap_m(int i, int n) { return i == 0 ? n - 1 : i - 1; }

__device__ __forceinline__ size_t lin(int n, int i, int j, int k) {
    return ((size_t)k * (size_t)n + (size_t)j) * (size_t)n + (size_t)i;
}

// Offsets of the six face neighbours of (i, j, k), periodic.
struct Nbrs {
    size_t c, xp, xm, yp, ym, zp, zm;
};

__device__ __forceinline__ Nbrs nbrs(int n, int i, int j, int k) {
    Nbrs q;
    q.c = lin(n, i, j, k);
    q.xp = lin(n, wrap_p(i, n), j, k);
    q.xm = lin(n, wrap_m(i, n), j, k);
    q.yp = lin(n, i, wrap_p(j, n), k);
    q.ym = lin(n, i, wrap_m(j, n), k);
    q.zp = lin(n, i, j, wrap_p(k, n));
    q.zm = lin(n, i, j, wrap_m(k, n));
    return q;
}

template <typename T>
__device__ __forceinline__ double nsum(const T *v, const Nbrs &q) {
    return ((double)v[q.xp] + (double)v[q.xm]) + ((double)v[q.yp] + (double)v[q.ym]) +
           ((double)v[q.zp] + (double)v[q.zm]);
}

// Cubic term of the chemical potential in its second-order form,
// g(x; a) = 1/4 (x + a)(x^2 + a^2), a = phi^kappa (Section 5, N2).
// DELTA: the correction form G(e) = g(b + e; a) - g(b; a) expanded without
// cancellation, b the base iterate.
template <bool DELTA>
struct Cubic;

template <>
struct Cubic<false> {
    __device__ static __forceinline__ double g(double x, double a, double) {
        return 0.25 * (x + a) * (x * x + a * a);
    }
    __device__ static __forceinline__ double dg(double x, double a, double) {
        return 0.25 * (3.0 * x * x + 2.0 * x * a + a * a);
    }
};

template <>
struct Cubic<true> {
    __device__ static __forceinline__ double g(double e, double a, double b) {
        return 0.25 * (e * (b * b + a * a) + (b + e + a) * (2.0 * b * e + e * e));
    }
    __device__ static __forceinline__ double dg(double e, double a, double b) {
        const double x = b + e;
        return 0.25 * (3.0 * x * x + 2.0 * x * a + a * a);
    }
};

// ------------------------------------------------------------- smoothing
//
// Pointwise solve of the three equations of N(u) = f at one point with the
// six neighbours held (Section 5 smoothing scheme, M = 1):
//     phi + A mu             = r1     A = 6 tau/h^2, r1 = f1 + tau S_mu/h^2
//    -c phi + mu + B omega   = r2     B = 6/h^2,     r2 = f2 + S_om/h^2 + (lin.)
//     Dd phi + omega         = r3     Dd = 3/h^2,    r3 = f3 + S_phi/(2h^2)
// with c the linearised slope of the cubic term; eliminating omega and mu
// gives phi = (r1 - A r2 + A B r3) / (1 + A (c + B Dd)).
template <typename T, bool DELTA>
__global__ __launch_bounds__(kBlock) void k_smooth(OpParams op, int colour, int picard, Tri<T> u,
                                                   Tri<const T> f, const T *__restrict__ phk,
                                                   const T *__restrict__ base) {
    const int n = op.n, half = n >> 1;
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    const size_t total = (size_t)half * n * n;
    if (t >= total) return;
    const int m = (int)(t % half);
    const size_t rest = t / half;
    const int j = (int)(rest % n);
    const int k = (int)(rest / n);
    const int i = 2 * m + ((j + k + colour) & 1);
    const Nbrs q = nbrs(n, i, j, k);

    const double smu = nsum(u.b, q), som = nsum(u.c, q), sphi = nsum(u.a, q);
    const double phin = u.a[q.c], a = phk[q.c];
    const double b = DELTA ? (double)base[q.c] : 0.0;
    const double h2inv = op.h2inv, tau = op.tau, lin_c = 0.5 * (1.0 - op.eps);
    double c, r2;
    if (!DELTA && picard) {
        const double qq = 0.25 * (phin * phin + a * a);
        c = qq + lin_c;
        r2 = (double)f.b[q.c] + som * h2inv + qq * a;
    } else {
        const double gp = Cubic<DELTA>::dg(phin, a, b);
        c = gp + lin_c;
        r2 = (double)f.b[q.c] + som * h2inv + (Cubic<DELTA>::g(phin, a, b) - gp * phin);
    }
    const double r1 = (double)f.a[q.c] + tau * smu * h2inv;
    const double r3 = (double)f.c[q.c] + 0.5 * sphi * h2inv;
    const double A = 6.0 * tau * h2inv, B = 6.0 * h2inv, Dd = 3.0 * h2inv;
    const double phi = (r1 - A * r2 + A * B * r3) / (1.0 + A * (c + B * Dd));
    const double om = r3 - Dd * phi;
    const double mu = r2 + c * phi - B * om;
    u.a[q.c] = (T)phi;
    u.b[q.c] = (T)mu;
    u.c[q.c] = (T)om;
}

template <typename T, bool DELTA>
void launch_smooth(hipStream_t s, const OpParams &op, int colour, int picard, Tri<T> u,
                   Tri<const T> f, const T *phk, const T *base) {
    const size_t total = (size_t)(op.n / 2) * op.n * op.n;
    const unsigned blocks = (unsigned)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_smooth<T, DELTA>), dim3(blocks), dim3(kBlock), 0, s, op, colour, picard,
                       u, f, phk, base);
}

// ------------------------------------------------------------ residual

// r = f - N(u) at one point (scheme-PFC-o1..o3 with M = 1; DELTA: the
// correction operator with G in place of g).
template <typename T, bool DELTA>
__device__ __forceinline__ void resid_at(const OpParams &op, const Tri<const T> &u,
                                         const Tri<const T> &f, const T *phk, const T *base,
                                         const Nbrs &q, double &r1, double &r2, double &r3) {
    const double phi = u.a[q.c], mu = u.b[q.c], om = u.c[q.c];
    const double lmu = (nsum(u.b, q) - 6.0 * mu) * op.h2inv;
    const double lom = (nsum(u.c, q) - 6.0 * om) * op.h2inv;
    const double lphi = (nsum(u.a, q) - 6.0 * phi) * op.h2inv;
    const double a = phk[q.c];
    const double b = DELTA ? (double)base[q.c] : 0.0;
    r1 = (double)f.a[q.c] - (phi - op.tau * lmu);
    r2 = (double)f.b[q.c] - (mu - Cubic<DELTA>::g(phi, a, b) - 0.5 * (1.0 - op.eps) * phi - lom);
    r3 = (double)f.c[q.c] - (om - 0.5 * lphi);
}

__device__ __forceinline__ unsigned long long abs_bits(double v) {
    return (unsigned long long)__double_as_longlong(v) & 0x7fffffffffffffffull;
}

// Block max of non-negative IEEE bit patterns (NaN sorts above +Inf).
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v) {
    __shared__ unsigned long long red[kBlock];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const unsigned long long o = red[threadIdx.x + w];
            if (o > red[threadIdx.x]) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    return red[0];
}

template <typename T, bool DELTA>
__global__ __launch_bounds__(kBlock) void k_resid_max(OpParams op, Tri<const T> u, Tri<const T> f,
                                                      const T *__restrict__ phk,
                                                      const T *__restrict__ base, Tri<T> r,
                                                      unsigned long long *partial) {
    const int n = op.n;
    const unsigned blk = xcd_block();
    const size_t t = (size_t)blk * kBlock + threadIdx.x;
    const size_t total = (size_t)n * n * n;
    unsigned long long m = 0;
    if (t < total) {
        const int i = (int)(t % n);
        const int j = (int)((t / n) % n);
        const int k = (int)(t / ((size_t)n * n));
        const Nbrs q = nbrs(n, i, j, k);
        double r1, r2, r3;
        resid_at<T, DELTA>(op, u, f, phk, base, q, r1, r2, r3);
        if (r.a) {
            r.a[q.c] = (T)r1;
            r.b[q.c] = (T)r2;
            r.c[q.c] = (T)r3;
        }
        m = abs_bits(r1);
        const unsigned long long m2 = abs_bits(r2), m3 = abs_bits(r3);
        if (m2 > m) m = m2;
        if (m3 > m) m = m3;
    }
    m = block_max_u64(m);
    if (threadIdx.x == 0) partial[blk] = m;
}

template <typename T, bool DELTA>
int launch_resid_max(hipStream_t s, const OpParams &op, Tri<const T> u, Tri<const T> f,
                     const T *phk, const T *base, Tri<T> r, unsigned long long *partial) {
    const size_t total = (size_t)op.n * op.n * op.n;
    const unsigned blocks = (unsigned)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_resid_max<T, DELTA>), dim3(blocks), dim3(kBlock), 0, s, op, u, f, phk,
                       base, r, partial);
    return (int)blocks;
}

__global__ __launch_bounds__(1024) void k_max_final(const unsigned long long *partial, int count,
                                                    double *out) {
    __shared__ unsigned long long red[1024];
    unsigned long long m = 0;
    for (int b = threadIdx.x; b < count; b += 1024)
        if (partial[b] > m) m = partial[b];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w && red[threadIdx.x + w] > red[threadIdx.x])
            red[threadIdx.x] = red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = __longlong_as_double((long long)red[0]);
}

void launch_max_final(hipStream_t s, const unsigned long long *partial, int count, double *out) {
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(1024), 0, s, partial, count, out);
}

// ------------------------------------------------ residual + coarsening
//
// One thread per coarse cell: residual at the 8 children, then the coarse
// cell's restricted residual I r and restricted iterate I u (8-child means).
template <typename T, bool DELTA>
__global__ __launch_bounds__(kBlock) void k_resid_restrict(OpParams op, Tri<const T> u,
                                                           Tri<const T> f,
                                                           const T *__restrict__ phk,
                                                           const T *__restrict__ base,
                                                           Tri<T> ubar_c, Tri<T> rr_c) {
    const int nf = op.n, nc = nf >> 1;
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    const size_t total = (size_t)nc * nc * nc;
    if (t >= total) return;
    const int I = (int)(t % nc);
    const int J = (int)((t / nc) % nc);
    const int K = (int)(t / ((size_t)nc * nc));
    double s1 = 0, s2 = 0, s3 = 0, ua = 0, ub = 0, uc = 0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const Nbrs q = nbrs(nf, 2 * I + cx, 2 * J + cy, 2 * K + cz);
                double r1, r2, r3;
                resid_at<T, DELTA>(op, u, f, phk, base, q, r1, r2, r3);
                s1 += r1;
                s2 += r2;
                s3 += r3;
                ua += (double)u.a[q.c];
                ub += (double)u.b[q.c];
                uc += (double)u.c[q.c];
            }
    const size_t o = lin(nc, I, J, K);
    rr_c.a[o] = (T)(0.125 * s1);
    rr_c.b[o] = (T)(0.125 * s2);
    rr_c.c[o] = (T)(0.125 * s3);
    ubar_c.a[o] = (T)(0.125 * ua);
    ubar_c.b[o] = (T)(0.125 * ub);
    ubar_c.c[o] = (T)(0.125 * uc);
}

template <typename T, bool DELTA>
void launch_resid_restrict(hipStream_t s, const OpParams &op, Tri<const T> u, Tri<const T> f,
                           const T *phk, const T *base, Tri<T> ubar_c, Tri<T> rr_c) {
    const size_t nc = op.n / 2;
    const size_t total = nc * nc * nc;
    const unsigned blocks = (unsigned)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_resid_restrict<T, DELTA>), dim3(blocks), dim3(kBlock), 0, s, op, u, f,
                       phk, base, ubar_c, rr_c);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(int nf, const T *__restrict__ fine,
                                                     T *__restrict__ coarse) {
    const int nc = nf >> 1;
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    const size_t total = (size_t)nc * nc * nc;
    if (t >= total) return;
    const int I = (int)(t % nc);
    const int J = (int)((t / nc) % nc);
    const int K = (int)(t / ((size_t)nc * nc));
    double s = 0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) s += (double)fine[lin(nf, 2 * I + cx, 2 * J + cy, 2 * K + cz)];
    coarse[lin(nc, I, J, K)] = (T)(0.125 * s);
}

template <typename T>
void launch_restrict(hipStream_t s, int nf, const T *fine, T *coarse) {
    const size_t nc = nf / 2;
    const size_t total = nc * nc * nc;
    const unsigned blocks = (unsigned)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_restrict<T>), dim3(blocks), dim3(kBlock), 0, s, nf, fine, coarse);
}

// ------------------------------------------------------- tau correction
//
// Coarse right-hand side of the FAS: f_c = N_c(I u) + I r (f holds I r on
// entry); also starts the coarse iterate at I u.
template <typename T, bool DELTA>
__global__ __launch_bounds__(kBlock) void k_tau(OpParams op, Tri<const T> ubar, Tri<T> f, Tri<T> u,
                                                const T *__restrict__ phk,
                                                const T *__restrict__ base) {
    const int n = op.n;
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    const size_t total = (size_t)n * n * n;
    if (t >= total) return;
    const int i = (int)(t % n);
    const int j = (int)((t / n) % n);
    const int k = (int)(t / ((size_t)n * n));
    const Nbrs q = nbrs(n, i, j, k);
    const double phi = ubar.a[q.c], mu = ubar.b[q.c], om = ubar.c[q.c];
    const double lmu = (nsum(ubar.b, q) - 6.0 * mu) * op.h2inv;
    const double lom = (nsum(ubar.c, q) - 6.0 * om) * op.h2inv;
    const double lphi = (nsum(ubar.a, q) - 6.0 * phi) * op.h2inv;
    const double a = phk[q.c];
    const double b = DELTA ? (double)base[q.c] : 0.0;
    const double n1 = phi - op.tau * lmu;
    const double n2 = mu - Cubic<DELTA>::g(phi, a, b) - 0.5 * (1.0 - op.eps) * phi - lom;
    const double n3 = om - 0.5 * lphi;
    f.a[q.c] = (T)((double)f.a[q.c] + n1);
    f.b[q.c] = (T)((double)f.b[q.c] + n2);
    f.c[q.c] = (T)((double)f.c[q.c] + n3);
    u.a[q.c] = ubar.a[q.c];
    u.b[q.c] = ubar.b[q.c];
    u.c[q.c] = ubar.c[q.c];
}

template <typename T, bool DELTA>
void launch_tau(hipStream_t s, const OpParams &opc, Tri<const T> ubar, Tri<T> f, Tri<T> u,
                const T *phk, const T *base) {
    const size_t total = (size_t)opc.n * opc.n * opc.n;
    const unsigned blocks = (unsigned)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_tau<T, DELTA>), dim3(blocks), dim3(kBlock), 0, s, opc, ubar, f, u, phk,
                       base);
}

// ------------------------------------------------- interpolation + correction
//
// fine += P (v - ubar) (ubar may be null; fine.b null: one field only):
// cell-centred trilinear interpolation.  Along one axis
// fine cell 2I+d (d = 0, 1) takes 3/4 of coarse cell I and 1/4 of cell I-1
// (d = 0) or I+1 (d = 1), periodic; 3D weights are products.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(int nc, Tri<const T> v, Tri<const T> ubar,
                                                    Tri<T> fine) {
    const int nf = nc << 1;
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    const size_t total = (size_t)nf * nf * nf;
    if (t >= total) return;
    const int i = (int)(t % nf);
    const int j = (int)((t / nf) % nf);
    const int k = (int)(t / ((size_t)nf * nf));
    const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
    const int I1 = (i & 1) ? wrap_p(I0, nc) : wrap_m(I0, nc);
    const int J1 = (j & 1) ? wrap_p(J0, nc) : wrap_m(J0, nc);
    const int K1 = (k & 1) ? wrap_p(K0, nc) : wrap_m(K0, nc);
    const int Is[2] = {I0, I1}, Js[2] = {J0, J1}, Ks[2] = {K0, K1};
    const double w[2] = {0.75, 0.25};
    double ea = 0, eb = 0, ec = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const double ww = w[a] * w[b] * w[c];
                const size_t o = lin(nc, Is[a], Js[b], Ks[c]);
                double da = v.a[o];
                if (ubar.a) da -= (double)ubar.a[o];
                ea += ww * da;
                if (fine.b) {
                    double db = v.b[o], dc = v.c[o];
                    if (ubar.a) {
                        db -= (double)ubar.b[o];
                        dc -= (double)ubar.c[o];
                    }
                    eb += ww * db;
                    ec += ww * dc;
                }
            }
    const size_t o = lin(nf, i, j, k);
    fine.a[o] = (T)((double)fine.a[o] + ea);
    if (fine.b) {
        fine.b[o] = (T)((double)fine.b[o] + eb);
        fine.c[o] = (T)((double)fine.c[o] + ec);
    }
}

template <typename T>
void launch_prolong(hipStream_t s, int nc, Tri<const T> v, Tri<const T> ubar, Tri<T> fine) {
    const size_t nf = 2 * (size_t)nc;
    const size_t total = nf * nf * nf;
    const unsigned blocks = (unsigned)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_prolong<T>), dim3(blocks), dim3(kBlock), 0, s, nc, v, ubar, fine);
}

// ------------------------------------------------------ coarsest solve
//
// Newton's method on the coarsest level (n = 3 or 4, P = n^3 <= 64 points),
// one 64-lane wavefront, lane p owning point p.  omega and mu enter the
// system linearly, so they are eliminated exactly and Newton runs on phi:
//   F(phi) = phi - tau Lap(g(phi) + (1-eps)/2 phi) - tau/2 Lap^3 phi - b = 0,
//   b = f1 + tau Lap(f2 + Lap f3),
//   F'(phi) = I - tau Lap diag(g'(phi) + (1-eps)/2) - tau/2 Lap^3,
// then omega = f3 + Lap phi / 2 and mu = f2 + g(phi) + (1-eps)/2 phi + Lap omega.
// The Newton iterates in phi are those of Newton on the full 3P system.
// Each Newton step factorises F' (dense, column-major in LDS) by LU with
// partial pivoting.  Stops when max|delta| <= 1e-14 max(1, max|phi|) or after
// 30 iterations.  lap1 / lap3: the P x P matrices of Lap and Lap^3 (column-major).
template <typename T, bool DELTA>
__global__ __launch_bounds__(64) void k_coarse(OpParams op, Tri<T> u, Tri<const T> f,
                                               const T *__restrict__ phk,
                                               const T *__restrict__ base,
                                               const double *__restrict__ lap1,
                                               const double *__restrict__ lap3, int *iters) {
    __shared__ double Jm[64 * 64];
    __shared__ double vec[64];
    __shared__ double rhs[64];
    __shared__ double sol[64];
    __shared__ double dvec[64];
    const int n = op.n, P = n * n * n;
    const int p = threadIdx.x;
    const bool act = p < P;
    const double h2inv = op.h2inv, tau = op.tau, lc = 0.5 * (1.0 - op.eps);

    int nb[6] = {0, 0, 0, 0, 0, 0};
    if (act) {
        const int i = p % n, j = (p / n) % n, k = p / (n * n);
        nb[0] = (int)lin(n, wrap_p(i, n), j, k);
        nb[1] = (int)lin(n, wrap_m(i, n), j, k);
        nb[2] = (int)lin(n, i, wrap_p(j, n), k);
        nb[3] = (int)lin(n, i, wrap_m(j, n), k);
        nb[4] = (int)lin(n, i, j, wrap_p(k, n));
        nb[5] = (int)lin(n, i, j, wrap_m(k, n));
    }
    auto lap_lds = [&](double own) -> double {
        // vec[] holds the field; returns Lap at point p
        return ((vec[nb[0]] + vec[nb[1]]) + (vec[nb[2]] + vec[nb[3]]) + (vec[nb[4]] + vec[nb[5]]) -
                6.0 * own) * h2inv;
    };
    const double a = act ? (double)phk[p] : 0.0;
    const double bs = (DELTA && act) ? (double)base[p] : 0.0;
    const double F1 = act ? (double)f.a[p] : 0.0;
    const double F2 = act ? (double)f.b[p] : 0.0;
    const double F3 = act ? (double)f.c[p] : 0.0;
    double x = act ? (double)u.a[p] : 0.0;

    // b = f1 + tau Lap(f2 + Lap f3)
    vec[p] = F3;
    __syncthreads();
    double t = act ? lap_lds(F3) : 0.0;
    __syncthreads();
    vec[p] = F2 + t;
    __syncthreads();
    const double bp = F1 + tau * (act ? lap_lds(F2 + t) : 0.0);
    __syncthreads();

    int it;
    for (it = 1; it <= 30; ++it) {
        const double w = Cubic<DELTA>::g(x, a, bs) + lc * x;
        const double D = Cubic<DELTA>::dg(x, a, bs) + lc;
        vec[p] = w;
        __syncthreads();
        const double lw = act ? lap_lds(w) : 0.0;
        __syncthreads();
        vec[p] = x;
        __syncthreads();
        double l1 = act ? lap_lds(x) : 0.0;
        __syncthreads();
        vec[p] = l1;
        __syncthreads();
        double l2 = act ? lap_lds(l1) : 0.0;
        __syncthreads();
        vec[p] = l2;
        __syncthreads();
        const double l3 = act ? lap_lds(l2) : 0.0;
        rhs[p] = act ? -(x - tau * lw - 0.5 * tau * l3 - bp) : 0.0;
        dvec[p] = D;
        __syncthreads();
        if (act) {
            for (int qc = 0; qc < P; ++qc) {
                const size_t o = (size_t)qc * P + p;
                Jm[o] = (qc == p ? 1.0 : 0.0) - tau * lap1[o] * dvec[qc] - 0.5 * tau * lap3[o];
            }
        }
        __syncthreads();
        // LU with partial pivoting, column by column.
        for (int c = 0; c < P; ++c) {
            double val = (act && p >= c) ? fabs(Jm[(size_t)c * P + p]) : -1.0;
            int id = p;
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(val, off, 64);
                const int oid = __shfl_xor(id, off, 64);
                if (ov > val || (ov == val && oid < id)) {
                    val = ov;
                    id = oid;
                }
            }
            const int pv = id;
            if (pv != c) {
                if (act) {
                    const double tmp = Jm[(size_t)p * P + c];
                    Jm[(size_t)p * P + c] = Jm[(size_t)p * P + pv];
                    Jm[(size_t)p * P + pv] = tmp;
                }
                if (p == 0) {
                    const double tmp = rhs[c];
                    rhs[c] = rhs[pv];
                    rhs[pv] = tmp;
                }
            }
            __syncthreads();
            if (act && p > c) {
                const double lr = Jm[(size_t)c * P + p] / Jm[(size_t)c * P + c];
                Jm[(size_t)c * P + p] = lr;
                rhs[p] -= lr * rhs[c];
                for (int qc = c + 1; qc < P; ++qc) Jm[(size_t)qc * P + p] -= lr * Jm[(size_t)qc * P + c];
            }
            __syncthreads();
        }
        for (int c = P - 1; c >= 0; --c) {
            if (p == c) sol[c] = rhs[c] / Jm[(size_t)c * P + c];
            __syncthreads();
            if (act && p < c) rhs[p] -= Jm[(size_t)c * P + p] * sol[c];
            __syncthreads();
        }
        const double d = act ? sol[p] : 0.0;
        x += d;
        double dm = fabs(d), xm = fabs(x);
        for (int off = 32; off > 0; off >>= 1) {
            dm = fmax(dm, __shfl_xor(dm, off, 64));
            xm = fmax(xm, __shfl_xor(xm, off, 64));
        }
        __syncthreads();
        if (!(dm == dm)) break;  // NaN: give up, the residual test reports it
        if (dm <= 1e-14 * fmax(1.0, xm)) break;
    }
    if (it > 30) it = 30;
    vec[p] = x;
    __syncthreads();
    const double lx = act ? lap_lds(x) : 0.0;
    __syncthreads();
    const double om = F3 + 0.5 * lx;
    vec[p] = om;
    __syncthreads();
    const double lom = act ? lap_lds(om) : 0.0;
    const double mu = F2 + Cubic<DELTA>::g(x, a, bs) + lc * x + lom;
    if (act) {
        u.a[p] = (T)x;
        u.b[p] = (T)mu;
        u.c[p] = (T)om;
    }
    if (p == 0 && iters) *iters = it;
}

template <typename T, bool DELTA>
void launch_coarse(hipStream_t s, const OpParams &op, Tri<T> u, Tri<const T> f, const T *phk,
                   const T *base, const double *lap1, const double *lap3, int *iters) {
    hipLaunchKernelGGL((k_coarse<T, DELTA>), dim3(1), dim3(64), 0, s, op, u, f, phk, base, lap1,
                       lap3, iters);
}

// --------------------------------------------------------------- source

// S of (scheme-PFC-s1..s3): f1 = phk, f2 = (1-eps)/2 phk + 3 Lap phk - Lap phkm1,
// f3 = Lap phk / 2.
__global__ __launch_bounds__(kBlock) void k_source(OpParams op, const double *__restrict__ phk,
                                                   const double *__restrict__ phkm1,
                                                   Tri<double> f) {
    const int n = op.n;
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    const size_t total = (size_t)n * n * n;
    if (t >= total) return;
    const int i = (int)(t % n);
    const int j = (int)((t / n) % n);
    const int k = (int)(t / ((size_t)n * n));
    const Nbrs q = nbrs(n, i, j, k);
    const double v = phk[q.c];
    const double lk = (nsum(phk, q) - 6.0 * v) * op.h2inv;
    const double lkm1 = (nsum(phkm1, q) - 6.0 * phkm1[q.c]) * op.h2inv;
    f.a[q.c] = v;
    f.b[q.c] = 0.5 * (1.0 - op.eps) * v + 3.0 * lk - lkm1;
    f.c[q.c] = 0.5 * lk;
}

void launch_source(hipStream_t s, const OpParams &op, const double *phk, const double *phkm1,
                   Tri<double> f) {
    const size_t total = (size_t)op.n * op.n * op.n;
    const unsigned blocks = (unsigned)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_source, dim3(blocks), dim3(kBlock), 0, s, op, phk, phkm1, f);
}

__global__ __launch_bounds__(kBlock) void k_lap(OpParams op, const double *__restrict__ v,
                                                double *__restrict__ out) {
    const int n = op.n;
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    const size_t total = (size_t)n * n * n;
    if (t >= total) return;
    const int i = (int)(t % n);
    const int j = (int)((t / n) % n);
    const int k = (int)(t / ((size_t)n * n));
    const Nbrs q = nbrs(n, i, j, k);
    out[q.c] = (nsum(v, q) - 6.0 * v[q.c]) * op.h2inv;
}

// mu = phi^3 + (1-eps) phi + 2 Lap phi + Lap^2 phi, with om = Lap phi given.
__global__ __launch_bounds__(kBlock) void k_init_mu(OpParams op, const double *__restrict__ phi,
                                                    const double *__restrict__ om,
                                                    double *__restrict__ mu) {
    const int n = op.n;
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    const size_t total = (size_t)n * n * n;
    if (t >= total) return;
    const int i = (int)(t % n);
    const int j = (int)((t / n) % n);
    const int k = (int)(t / ((size_t)n * n));
    const Nbrs q = nbrs(n, i, j, k);
    const double v = phi[q.c];
    const double l2 = (nsum(om, q) - 6.0 * om[q.c]) * op.h2inv;
    mu[q.c] = v * v * v + (1.0 - op.eps) * v + 2.0 * om[q.c] + l2;
}

void launch_init_guess(hipStream_t s, const OpParams &op, const double *phi0, double *mu,
                       double *om) {
    const size_t total = (size_t)op.n * op.n * op.n;
    const unsigned blocks = (unsigned)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_lap, dim3(blocks), dim3(kBlock), 0, s, op, phi0, om);
    hipLaunchKernelGGL(k_init_mu, dim3(blocks), dim3(kBlock), 0, s, op, phi0, om, mu);
}

// --------------------------------------------------------------- energy

constexpr int kEnergyBlocks = 1024;

int energy_blocks(int n) {
    const size_t total = (size_t)n * n * n;
    const size_t b = (total + kBlock - 1) / kBlock;
    return (int)(b < (size_t)kEnergyBlocks ? b : (size_t)kEnergyBlocks);
}

// Per-block sums of phi^4, phi^2, (D phi)^2 on the cell's three forward faces
// (so every face of the periodic grid is counted once), (Lap phi)^2, the same
// face sum for phi - phi_prev, and phi.  Scaled by h^3 in the final pass.
__global__ __launch_bounds__(kBlock) void k_energy_part(int n, double hinv, double h2inv,
                                                        const double *__restrict__ phi,
                                                        const double *__restrict__ prev,
                                                        double *__restrict__ part) {
    __shared__ double red[6][kBlock];
    double s[6] = {0, 0, 0, 0, 0, 0};
    const size_t total = (size_t)n * n * n;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < total;
         t += (size_t)gridDim.x * kBlock) {
        const int i = (int)(t % n);
        const int j = (int)((t / n) % n);
        const int k = (int)(t / ((size_t)n * n));
        const Nbrs q = nbrs(n, i, j, k);
        const double v = phi[q.c];
        const double v2 = v * v;
        s[0] += v2 * v2;
        s[1] += v2;
        s[5] += v;
        const double dx = (phi[q.xp] - v) * hinv, dy = (phi[q.yp] - v) * hinv,
                     dz = (phi[q.zp] - v) * hinv;
        s[2] += dx * dx + dy * dy + dz * dz;
        const double l = (nsum(phi, q) - 6.0 * v) * h2inv;
        s[3] += l * l;
        if (prev) {
            const double w = v - prev[q.c];
            const double ex = (phi[q.xp] - prev[q.xp] - w) * hinv;
            const double ey = (phi[q.yp] - prev[q.yp] - w) * hinv;
            const double ez = (phi[q.zp] - prev[q.zp] - w) * hinv;
            s[4] += ex * ex + ey * ey + ez * ez;
        }
    }
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) part[(size_t)blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_energy_final(const double *__restrict__ part, int count,
                                                         double h, double eps,
                                                         double *__restrict__ out) {
    __shared__ double red[6][kBlock];
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < count; b += kBlock)
        for (int c = 0; c < 6; ++c) s[c] += part[(size_t)b * 6 + c];
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double h3 = h * h * h;
        const double F = h3 * (0.25 * red[0][0] + 0.5 * (1.0 - eps) * red[1][0] - red[2][0] +
                               0.5 * red[3][0]);
        out[0] = F;
        out[1] = F + 0.5 * h3 * red[4][0];
        out[2] = h3 * red[5][0];
    }
}

void launch_energy(hipStream_t s, int n, double h, double eps, const double *phi,
                   const double *phi_prev, double *partial, double *out3) {
    const int blocks = energy_blocks(n);
    hipLaunchKernelGGL(k_energy_part, dim3(blocks), dim3(kBlock), 0, s, n, 1.0 / h, 1.0 / (h * h),
                       phi, phi_prev, partial);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, s, partial, blocks, h, eps, out3);
}

// ------------------------------------------------------ instantiations

#define PFC_INST(T, DELTA)                                                                        \
    template void launch_smooth<T, DELTA>(hipStream_t, const OpParams &, int, int, Tri<T>,        \
                                          Tri<const T>, const T *, const T *);                    \
    template void launch_resid_restrict<T, DELTA>(hipStream_t, const OpParams &, Tri<const T>,    \
                                                  Tri<const T>, const T *, const T *, Tri<T>,     \
                                                  Tri<T>);                                        \
    template void launch_tau<T, DELTA>(hipStream_t, const OpParams &, Tri<const T>, Tri<T>,       \
                                       Tri<T>, const T *, const T *);                             \
    template int launch_resid_max<T, DELTA>(hipStream_t, const OpParams &, Tri<const T>,          \
                                            Tri<const T>, const T *, const T *, Tri<T>,           \
                                            unsigned long long *);                                \
    template void launch_coarse<T, DELTA>(hipStream_t, const OpParams &, Tri<T>, Tri<const T>,    \
                                          const T *, const T *, const double *, const double *,   \
                                          int *);

PFC_INST(double, false)
PFC_INST(float, true)
template void launch_restrict<double>(hipStream_t, int, const double *, double *);
template void launch_restrict<float>(hipStream_t, int, const float *, float *);
template void launch_prolong<double>(hipStream_t, int, Tri<const double>, Tri<const double>,
                                     Tri<double>);
template void launch_prolong<float>(hipStream_t, int, Tri<const float>, Tri<const float>,
                                    Tri<float>);

}  // namespace pfc
