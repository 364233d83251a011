// HIP kernels (gfx950) for the FAS multigrid solve of one step of the
// second-order PFC scheme (arXiv:1611.06288, Sections 2, 3 and 5): layouts,
// transfers (restriction, tau correction, interpolation), the coarsest-level
// solve, the source, energy sums, the FP32/FP64 conversions of the
// mixed-precision form and the batched kernels.  The smoothers live in
// smooth.hip, the column-tile residuals in residual.hip.
//
// Every kernel is a 7-point stencil, a transfer or a reduction: memory bound,
// no matrix-core work.  Smoothed levels store each field colour-split (all
// points of colour 0 = (i+j+k) even, then all of colour 1), so a red-black
// half-sweep streams only the colour it updates plus the other colour's three
// fields.  Threads walk the storage order (coalesced); workgroup ids are
// remapped so each of the 8 XCDs gets a contiguous range of z-planes, whose
// neighbours then meet in that XCD's L2.
//
// Storage type T is double (FP64 path) or float (the correction cycle of the
// mixed-precision form); operator arithmetic and the pointwise 3x3 solve run
// in FP64 in both.
#include "device_common.h"
#include "pfc.h"
#include "smooth.h"

#include <math.h>

#include <algorithm>
#include <numeric>
#include <type_traits>

namespace pfc {

// ------------------------------------------------------------------ layout

Div make_div(int d) {
    Div r{0, 0};
    if (d % 3 == 0) {
        r.three = 1;
        d /= 3;
    }
    while (d > 1) {
        d >>= 1;
        ++r.shift;
    }
    return r;
}

Lay make_lay(int n, bool split) {
    Lay l;
    l.n = n;
    l.split = split ? 1 : 0;
    l.dn = make_div(n);
    l.dh = make_div(split ? n / 2 : 1);
    return l;
}

// ------------------------------------------------------------ residual

// r = f - N(u) at one point (scheme-PFC-o1..o3 with M = 1; DELTA: the
// correction operator with G in place of g; MOB: the first equation in flux
// form with the face mobilities of op.mob).
template <typename T, bool DELTA, bool MOB = false>
__device__ __forceinline__ void resid_at(const OpParams &op, const Tri<const T> &u,
                                         const Tri<const T> &f, const T *phk, const T *base,
                                         const Off &q, double &r1, double &r2, double &r3) {
    const double phi = u.a[q.c], mu = u.b[q.c], om = u.c[q.c];
    double lmu;
    if constexpr (MOB) {
        const double *ps = op.mob.phs;
        const double pc = ps[q.c];
        const unsigned nb6[6] = {q.xp, q.xm, q.yp, q.ym, q.zp, q.zm};
        double sm = 0.0;
#pragma unroll
        for (int e = 0; e < 6; ++e)
            sm += face_mob(op.mob, pc, ps[nb6[e]]) * ((double)u.b[nb6[e]] - mu);
        lmu = sm * op.h2inv;
    } else {
        lmu = (nsum(u.b, q) - 6.0 * mu) * op.h2inv;
    }
    const double lom = (nsum(u.c, q) - 6.0 * om) * op.h2inv;
    const double lphi = (nsum(u.a, q) - 6.0 * phi) * op.h2inv;
    const double a = phk[q.c];
    const double b = DELTA ? (double)base[q.c] : 0.0;
    r1 = (double)f.a[q.c] - (phi - op.tau * lmu);
    r2 = (double)f.b[q.c] - (mu - g_of<DELTA>(op.fo, phi, a, b) - lin_of(op) * phi - lom);
    r3 = (double)f.c[q.c] - (om - w3_of(op) * lphi);
}

// Residual at the point stored at t (written to r if r.a is set); returns the
// largest |component| as an IEEE bit pattern.
template <typename T, bool DELTA, bool MOB = false>
__device__ __forceinline__ unsigned long long resid_bits(const OpParams &op, const Tri<const T> &u,
                                                         const Tri<const T> &f, const T *phk,
                                                         const T *base, const Tri<T> &r,
                                                         unsigned t) {
    int i, j, k;
    decode(op.lay, t, i, j, k);
    const Off q = offs(op.lay, i, j, k);
    double r1, r2, r3;
    resid_at<T, DELTA, MOB>(op, u, f, phk, base, q, r1, r2, r3);
    if (r.a) {
        r.a[q.c] = (T)r1;
        r.b[q.c] = (T)r2;
        r.c[q.c] = (T)r3;
    }
    return umax(abs_bits(r1), umax(abs_bits(r2), abs_bits(r3)));
}

template <typename T, bool DELTA, bool MOB>
__global__ __launch_bounds__(kBlock) void k_resid_max(OpParams op, Tri<const T> u, Tri<const T> f,
                                                      const T *__restrict__ phk,
                                                      const T *__restrict__ base, Tri<T> r,
                                                      unsigned long long *partial) {
    if (gate_closed(op.gate)) return;
    const Lay &L = op.lay;
    const unsigned total = (unsigned)npts(L);
    unsigned long long m = 0;
    for (unsigned t = xcd_block() * kBlock + threadIdx.x; t < total; t += gridDim.x * kBlock)
        m = umax(m, resid_bits<T, DELTA, MOB>(op, u, f, phk, base, r, t));
    m = block_max_u64(m);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

template <typename T, bool DELTA>
int launch_resid_max(hipStream_t s, const OpParams &op, Tri<const T> u, Tri<const T> f,
                     const T *phk, const T *base, Tri<T> r, unsigned long long *partial) {
    const unsigned blocks = reduce_blocks(npts_host(op.lay));
    if constexpr (!DELTA) {
        if (op.mob.phs) {
            hipLaunchKernelGGL((k_resid_max<T, false, true>), dim3(blocks), dim3(kBlock), 0, s, op,
                               u, f, phk, base, r, partial);
            return (int)blocks;
        }
    }
    hipLaunchKernelGGL((k_resid_max<T, DELTA, false>), dim3(blocks), dim3(kBlock), 0, s, op, u, f,
                       phk, base, r, partial);
    return (int)blocks;
}

__global__ __launch_bounds__(kBlock) void k_max_final(const unsigned long long *partial, int count,
                                                      double *out, const int *gate) {
    if (gate_closed(gate)) return;
    unsigned long long m = 0;
    for (int b = threadIdx.x; b < count; b += kBlock) m = umax(m, partial[b]);
    m = block_max_u64(m);
    if (threadIdx.x == 0) out[0] = __longlong_as_double((long long)m);
}

void launch_max_final(hipStream_t s, const unsigned long long *partial, int count, double *out,
                      const int *gate) {
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kBlock), 0, s, partial, count, out, gate);
}

// The max of partial[0 .. count) into dst[0] and zeros into dst[1 .. dcount):
// seeds one half of a split stop-test norm with a whole-level norm (max is
// exact and idempotent, so the other half's partials then change nothing).
__global__ __launch_bounds__(kBlock) void k_norm_seed(const unsigned long long *partial, int count,
                                                      unsigned long long *dst, int dcount) {
    unsigned long long m = 0;
    for (int b = threadIdx.x; b < count; b += kBlock) m = umax(m, partial[b]);
    m = block_max_u64(m);
    for (int b = threadIdx.x; b < dcount; b += kBlock) dst[b] = b == 0 ? m : 0ull;
}

void launch_norm_seed(hipStream_t s, const unsigned long long *partial, int count,
                      unsigned long long *dst, int dcount) {
    hipLaunchKernelGGL(k_norm_seed, dim3(1), dim3(kBlock), 0, s, partial, count, dst, dcount);
}

// ------------------------------------------------ stop test of the time loop

__global__ void k_run_reset(RunState st) {
    if (threadIdx.x == 0) {
        *st.active = 1;
        *st.cycles = 0;
        *st.status = 0;
        *st.res0 = 0.0;
        *st.res = 0.0;
    }
}

void launch_run_reset(hipStream_t s, RunState st) {
    hipLaunchKernelGGL(k_run_reset, dim3(1), dim3(64), 0, s, st);
}

// The decision the host loop of a time step takes before each cycle: stop on
// a non-finite norm, on norm <= tol, or when max_cycles cycles have run;
// otherwise count the cycle that follows.
__global__ __launch_bounds__(kBlock) void k_stop_test(const unsigned long long *partial,
                                                      int count, double tol, int max_cycles,
                                                      RunState st) {
    if (*st.active == 0) return;  // the same for every thread of the block
    unsigned long long m = 0;
    for (int b = threadIdx.x; b < count; b += kBlock) m = umax(m, partial[b]);
    m = block_max_u64(m);
    if (threadIdx.x != 0) return;
    const double r = __longlong_as_double((long long)m);
    const int c = *st.cycles;
    if (c == 0) *st.res0 = r;
    *st.res = r;
    if (!isfinite(r)) {
        *st.status = 3;  // PFC_ERR_NONFINITE
        *st.active = 0;
    } else if (r <= tol) {
        *st.active = 0;
    } else if (c == max_cycles) {
        *st.status = 2;  // PFC_ERR_NOT_CONVERGED
        *st.active = 0;
    } else {
        *st.cycles = c + 1;
    }
}

void launch_stop_test(hipStream_t s, const unsigned long long *partial, int count, double tol,
                      int max_cycles, RunState st) {
    hipLaunchKernelGGL(k_stop_test, dim3(1), dim3(kBlock), 0, s, partial, count, tol, max_cycles,
                       st);
}

// ------------------------------------------------ residual + coarsening
//
// One thread per coarse cell: residual at its 8 children, then the coarse
// cell's restricted residual I r and restricted iterate I u (8-child means).
template <typename T, bool DELTA, bool MOB = false>
__device__ __forceinline__ void resid_restrict_body(const OpParams &op, const Lay &LC,
                                                    Tri<const T> u, Tri<const T> f,
                                                    const T *__restrict__ phk,
                                                    const T *__restrict__ base, Tri<T> ubar_c,
                                                    Tri<T> rr_c, unsigned tn) {
    // coarse cells in natural order, so that consecutive threads read
    // consecutive fine offsets of each colour
    if (tn >= (unsigned)npts(LC)) return;
    int I, J, K;
    decode_nat(LC, tn, I, J, K);
    const unsigned t = sidx32(LC, I, J, K);
    double s1 = 0, s2 = 0, s3 = 0, ua = 0, ub = 0, uc = 0;
#pragma unroll 1
    for (int ch = 0; ch < 8; ++ch) {
        const Off q = offs(op.lay, 2 * I + (ch & 1), 2 * J + ((ch >> 1) & 1), 2 * K + (ch >> 2));
        double r1, r2, r3;
        resid_at<T, DELTA, MOB>(op, u, f, phk, base, q, r1, r2, r3);
        s1 += r1;
        s2 += r2;
        s3 += r3;
        ua += (double)u.a[q.c];
        ub += (double)u.b[q.c];
        uc += (double)u.c[q.c];
    }
    rr_c.a[t] = (T)(0.125 * s1);
    rr_c.b[t] = (T)(0.125 * s2);
    rr_c.c[t] = (T)(0.125 * s3);
    ubar_c.a[t] = (T)(0.125 * ua);
    ubar_c.b[t] = (T)(0.125 * ub);
    ubar_c.c[t] = (T)(0.125 * uc);
}

// The per-level launch: eight threads per coarse cell, one per child (child
// ch = lane & 7 in the order of resid_restrict_body), so each thread waits on
// one child's loads rather than eight in turn; the group's first lane then
// adds the eight children's values in that order, as the body does.
template <typename T, bool DELTA, bool MOB>
__global__ __launch_bounds__(kBlock) void k_resid_restrict(OpParams op, Lay LC, Tri<const T> u,
                                                           Tri<const T> f,
                                                           const T *__restrict__ phk,
                                                           const T *__restrict__ base,
                                                           Tri<T> ubar_c, Tri<T> rr_c) {
    if (gate_closed(op.gate)) return;
    const unsigned g = xcd_block() * kBlock + threadIdx.x;
    const unsigned tn = g >> 3;
    const int ch = (int)(g & 7u);
    const bool act = tn < (unsigned)npts(LC);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // r1, r2, r3, u.a, u.b, u.c of the child
    unsigned t = 0;
    if (act) {
        int I, J, K;
        decode_nat(LC, tn, I, J, K);
        t = sidx32(LC, I, J, K);
        const Off q = offs(op.lay, 2 * I + (ch & 1), 2 * J + ((ch >> 1) & 1), 2 * K + (ch >> 2));
        resid_at<T, DELTA, MOB>(op, u, f, phk, base, q, v[0], v[1], v[2]);
        v[3] = (double)u.a[q.c];
        v[4] = (double)u.b[q.c];
        v[5] = (double)u.c[q.c];
    }
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int e = 0; e < 6; ++e) s[e] += __shfl(v[e], c, 8);
    if (act && ch == 0) {
        rr_c.a[t] = (T)(0.125 * s[0]);
        rr_c.b[t] = (T)(0.125 * s[1]);
        rr_c.c[t] = (T)(0.125 * s[2]);
        ubar_c.a[t] = (T)(0.125 * s[3]);
        ubar_c.b[t] = (T)(0.125 * s[4]);
        ubar_c.c[t] = (T)(0.125 * s[5]);
    }
}

template <typename T, bool DELTA>
void launch_resid_restrict(hipStream_t s, const OpParams &op, const Lay &coarse, Tri<const T> u,
                           Tri<const T> f, const T *phk, const T *base, Tri<T> ubar_c, Tri<T> rr_c) {
    const unsigned blocks = blocks_for(8 * npts_host(coarse));
    if constexpr (!DELTA) {
        if (op.mob.phs) {
            hipLaunchKernelGGL((k_resid_restrict<T, false, true>), dim3(blocks), dim3(kBlock), 0, s,
                               op, coarse, u, f, phk, base, ubar_c, rr_c);
            return;
        }
    }
    hipLaunchKernelGGL((k_resid_restrict<T, DELTA, false>), dim3(blocks), dim3(kBlock), 0, s, op,
                       coarse, u, f, phk, base, ubar_c, rr_c);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(Lay LF, Lay LC, const T *__restrict__ fine,
                                                     T *__restrict__ coarse) {
    const unsigned tn = xcd_block() * kBlock + threadIdx.x;
    if (tn >= (unsigned)npts(LC)) return;
    int I, J, K;
    decode_nat(LC, tn, I, J, K);
    const unsigned t = sidx32(LC, I, J, K);
    double s = 0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) s += (double)fine[sidx32(LF, 2 * I + cx, 2 * J + cy, 2 * K + cz)];
    coarse[t] = (T)(0.125 * s);
}

template <typename T>
void launch_restrict(hipStream_t s, const Lay &fine, const Lay &coarse, const T *fine_v, T *coarse_v) {
    hipLaunchKernelGGL((k_restrict<T>), dim3(blocks_for(npts_host(coarse))), dim3(kBlock), 0, s,
                       fine, coarse, fine_v, coarse_v);
}

// ------------------------------------------------------- tau correction
//
// Coarse right-hand side of the FAS: f_c = N_c(I u) + I r (f holds I r on
// entry); also starts the coarse iterate at I u, unless u.a is null.
template <typename T, bool DELTA, bool MOB = false>
__device__ __forceinline__ void tau_body(const OpParams &op, Tri<const T> ubar, Tri<T> f, Tri<T> u,
                                         const T *__restrict__ phk, const T *__restrict__ base,
                                         unsigned t) {
    const Lay &L = op.lay;
    if (t >= (unsigned)npts(L)) return;
    int i, j, k;
    decode(L, t, i, j, k);
    const Off q = offs(L, i, j, k);
    const double phi = ubar.a[t], mu = ubar.b[t], om = ubar.c[t];
    double lmu;
    if constexpr (MOB) {
        const double *ps = op.mob.phs;
        const double pc = ps[q.c];
        const unsigned nb6[6] = {q.xp, q.xm, q.yp, q.ym, q.zp, q.zm};
        double sm = 0.0;
#pragma unroll
        for (int e = 0; e < 6; ++e)
            sm += face_mob(op.mob, pc, ps[nb6[e]]) * ((double)ubar.b[nb6[e]] - mu);
        lmu = sm * op.h2inv;
    } else {
        lmu = (nsum(ubar.b, q) - 6.0 * mu) * op.h2inv;
    }
    const double ls[3] = {(nsum(ubar.a, q) - 6.0 * phi) * op.h2inv, lmu,
                          (nsum(ubar.c, q) - 6.0 * om) * op.h2inv};
    // every load ahead of the first store (which may alias them as far as the
    // compiler knows); I u's own values are copied from phi, mu, om (exact)
    const double f0 = f.a[t], f1 = f.b[t], f2 = f.c[t];
    double nv[3];
    n_of_point<DELTA>(op, ls, phi, mu, om, (double)phk[t], DELTA ? (double)base[t] : 0.0, nv);
    f.a[t] = (T)(f0 + nv[0]);
    f.b[t] = (T)(f1 + nv[1]);
    f.c[t] = (T)(f2 + nv[2]);
    if (u.a) {
        u.a[t] = (T)phi;
        u.b[t] = (T)mu;
        u.c[t] = (T)om;
    }
}

template <typename T, bool DELTA, bool MOB>
__global__ __launch_bounds__(kBlock) void k_tau(OpParams op, Tri<const T> ubar, Tri<T> f, Tri<T> u,
                                                const T *__restrict__ phk,
                                                const T *__restrict__ base) {
    if (gate_closed(op.gate)) return;
    tau_body<T, DELTA, MOB>(op, ubar, f, u, phk, base, xcd_block() * kBlock + threadIdx.x);
}

template <typename T, bool DELTA>
void launch_tau(hipStream_t s, const OpParams &opc, Tri<const T> ubar, Tri<T> f, Tri<T> u,
                const T *phk, const T *base) {
    if constexpr (!DELTA) {
        if (opc.mob.phs) {
            hipLaunchKernelGGL((k_tau<T, false, true>), dim3(blocks_for(npts_host(opc.lay))),
                               dim3(kBlock), 0, s, opc, ubar, f, u, phk, base);
            return;
        }
    }
    hipLaunchKernelGGL((k_tau<T, DELTA, false>), dim3(blocks_for(npts_host(opc.lay))), dim3(kBlock),
                       0, s, opc, ubar, f, u, phk, base);
}

// ------------------------------------------------- interpolation + correction
//
// The fine x-pair of prolong_body: NC components (1: phi only, 3: all),
// UB: the coarse error is v - ubar (formed and rounded to T here) or v
// itself.  All coarse and fine values are loaded first, then added and
// stored; fine values whose store is skipped (phi0) are loaded all the same.
template <typename T, int NC, bool UB>
__device__ __forceinline__ void prolong_pair(Tri<const T> v, Tri<const T> ubar, Tri<T> fine,
                                             const unsigned (&o)[2][2][3], unsigned f0,
                                             unsigned f1, bool phi0, bool c1) {
    const T *vv[3] = {v.a, v.b, v.c};
    const T *uu[3] = {ubar.a, ubar.b, ubar.c};
    T *ff[3] = {fine.a, fine.b, fine.c};
    double e[NC][3][2][2], g0[NC], g1[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int z = 0; z < 2; ++z)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    const unsigned q = o[z][y][x];
                    // v - ubar rounded to T: what coarse_err_body stores
                    e[c][x][z][y] = UB ? (double)(T)((double)vv[c][q] - (double)uu[c][q])
                                       : (double)vv[c][q];
                }
        g0[c] = (double)ff[c][f0];
        g1[c] = (double)ff[c][f1];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double w[3];  // y/z-interpolated values at x = I-1, I, I+1
#pragma unroll
        for (int x = 0; x < 3; ++x)
            w[x] = 0.75 * (0.75 * e[c][x][0][0] + 0.25 * e[c][x][0][1]) +
                   0.25 * (0.75 * e[c][x][1][0] + 0.25 * e[c][x][1][1]);
        const bool w0 = c == 0 || !phi0 || c1, w1 = c == 0 || !phi0 || !c1;
        if (w0) ff[c][f0] = (T)(g0[c] + (0.75 * w[1] + 0.25 * w[0]));
        if (w1) ff[c][f1] = (T)(g1[c] + (0.75 * w[1] + 0.25 * w[2]));
    }
}

// fine += P (v - ubar), cell-centred trilinear: along one axis fine cell 2I+d
// (d = 0, 1) takes 3/4 of coarse cell I and 1/4 of cell I-1 (d = 0) or I+1
// (d = 1), periodic; 3D weights are products.  One thread per pair of fine
// cells (2I, j, k), (2I+1, j, k): they share the 12 coarse cells
// {I-1, I, I+1} x {J0, J1} x {K0, K1}.  Consecutive threads take consecutive
// I, so the fine accesses are unit-stride in each colour block.  phi0 (a
// smoothing sweep follows): mu and omega are corrected at the pair's colour-1
// point only, the colour-0 ones being dead until that sweep overwrites them.
template <typename T>
__device__ __forceinline__ void prolong_body(const Lay &LC, const Lay &LF, Tri<const T> v,
                                             Tri<const T> ubar, Tri<T> fine, unsigned t,
                                             bool phi0 = false) {
    const int nc = LC.n, nf = LF.n;
    if (t >= (unsigned)nc * (unsigned)nf * (unsigned)nf) return;
    const unsigned row = LC.dn.q(t);           // (k, j) fine row
    const int I = (int)(t - row * (unsigned)nc);
    const int k = (int)LF.dn.q(row);
    const int j = (int)(row - (unsigned)k * (unsigned)nf);
    const int J0 = j >> 1, K0 = k >> 1;
    const int J1 = (j & 1) ? wrap_p(J0, nc) : wrap_m(J0, nc);
    const int K1 = (k & 1) ? wrap_p(K0, nc) : wrap_m(K0, nc);
    const int Ix[3] = {wrap_m(I, nc), I, wrap_p(I, nc)};
    unsigned o[2][2][3];  // [z][y][x]
#pragma unroll
    for (int z = 0; z < 2; ++z)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int x = 0; x < 3; ++x) o[z][y][x] = sidx32(LC, Ix[x], y ? J1 : J0, z ? K1 : K0);
    const unsigned f0 = sidx32(LF, 2 * I, j, k), f1 = sidx32(LF, 2 * I + 1, j, k);
    const bool c1 = ((j + k) & 1) != 0;  // (2I, j, k) is colour 1
    // the uniform tests are taken once, so that every load of a form comes in
    // one block, ahead of the stores (which may alias them for the compiler)
    if (fine.b) {
        if (ubar.a)
            prolong_pair<T, 3, true>(v, ubar, fine, o, f0, f1, phi0, c1);
        else
            prolong_pair<T, 3, false>(v, ubar, fine, o, f0, f1, phi0, c1);
    } else {
        if (ubar.a)
            prolong_pair<T, 1, true>(v, ubar, fine, o, f0, f1, phi0, c1);
        else
            prolong_pair<T, 1, false>(v, ubar, fine, o, f0, f1, phi0, c1);
    }
}

// ubar <- v - ubar on the coarse level (the correction to interpolate).
template <typename T>
__device__ __forceinline__ void coarse_err_body(size_t P, Tri<const T> v, Tri<T> ubar, unsigned t) {
    if (t >= P) return;
    // all six loads ahead of the first store, which may alias them as far as
    // the compiler knows
    const double va = v.a[t], vb = v.b[t], vc = v.c[t];
    const double ua = ubar.a[t], ub = ubar.b[t], uc = ubar.c[t];
    ubar.a[t] = (T)(va - ua);
    ubar.b[t] = (T)(vb - ub);
    ubar.c[t] = (T)(vc - uc);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(Lay LC, Lay LF, Tri<const T> v, Tri<const T> ubar,
                                                    Tri<T> fine, const int *gate, int phi0) {
    if (gate_closed(gate)) return;
    prolong_body<T>(LC, LF, v, ubar, fine, xcd_block() * kBlock + threadIdx.x, phi0 != 0);
}

// Tiled form for colour-split fine levels with n a multiple of 64: a
// workgroup owns a 64 x 8 fine column and a range of coarse planes, and walks
// it in z.  The coarse error e = v - ubar (rounded to T, the value
// coarse_err_body stores) of three coarse planes, (32+2) x (4+2) cells each,
// sits in an LDS ring; the next coarse plane and the next plane pair's fine
// values are loaded into registers while the current pair is computed, so
// each coarse value is fetched about once per column and the load latency
// overlaps the arithmetic.  A thread updates an x-pair in both fine planes of
// a coarse plane K.  Same weights and operation order as prolong_body.  phi0
// (the cycle's interpolation, followed by a smoothing sweep): at colour-0
// points only phi is corrected, since the sweep's colour-0 half reads nothing
// else of a colour-0 point before overwriting it; mu and omega there are
// neither read nor written.
constexpr int kPX = 64, kPY = 8;
constexpr int kPCW = kPX / 2 + 2, kPCH = kPY / 2 + 2, kPCN = kPCW * kPCH;  // coarse ring plane

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_tile(Lay LC, Lay LF, Tri<const T> v,
                                                         Tri<const T> ubar, Tri<T> fine,
                                                         const int *gate, int phi0, int nzr) {
    static_assert(kPCN <= kBlock, "one coarse ring cell per thread");
    __shared__ double ce[3][3][kPCH][kPCW];  // [field][plane slot][Y][X]
    if (gate_closed(gate)) return;
    const int nc = LC.n, nf = LF.n;
    const int nbx = nf / kPX, nby = nf / kPY;
    const int b = (int)xcd_block();
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int x0 = bx * kPX, y0 = by * kPY, X0 = x0 / 2, Y0 = y0 / 2;
    const int K0 = bz * nc / nzr, K1 = (bz + 1) * nc / nzr;
    const int tid = threadIdx.x, qx = tid & 31, qy = tid >> 5;
    const int y = y0 + qy;
    auto wc = [nc](int q) { return q < 0 ? q + nc : (q >= nc ? q - nc : q); };
    auto slot = [K0](int P) { return (P - K0 + 4) % 3; };  // P >= K0 - 1
    // this thread's coarse ring cell and its error on plane P
    const int cpy = tid / kPCW, cpx = tid - cpy * kPCW;
    T cn[3];
    auto load_coarse = [&](int P) {
        if (tid < kPCN) {
            const unsigned g = sidx32(LC, wc(X0 - 1 + cpx), wc(Y0 - 1 + cpy), wc(P));
            if (ubar.a) {
                cn[0] = (T)((double)v.a[g] - (double)ubar.a[g]);
                cn[1] = (T)((double)v.b[g] - (double)ubar.b[g]);
                cn[2] = (T)((double)v.c[g] - (double)ubar.c[g]);
            } else {
                cn[0] = v.a[g];
                cn[1] = v.b[g];
                cn[2] = v.c[g];
            }
        }
    };
    auto store_coarse = [&](int P) {
        if (tid < kPCN) {
            const int s = slot(P);
            ce[0][s][cpy][cpx] = (double)cn[0];
            ce[1][s][cpy][cpx] = (double)cn[1];
            ce[2][s][cpy][cpx] = (double)cn[2];
        }
    };
    // the thread's fine values of the plane pair 2K, 2K + 1
    T fv[2][2][3];  // [dz][dx][field]
    auto load_fine = [&](int K, T (&o)[2][2][3]) {
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const unsigned g = sidx32(LF, x0 + 2 * qx + dx, y, 2 * K + dz);
                o[dz][dx][0] = fine.a[g];
                if (!phi0 || ((dx + y + dz) & 1)) {  // x0, 2 qx and 2 K are even
                    o[dz][dx][1] = fine.b[g];
                    o[dz][dx][2] = fine.c[g];
                } else {  // not read nor written back; defined for the copy below
                    o[dz][dx][1] = (T)0;
                    o[dz][dx][2] = (T)0;
                }
            }
    };
    load_coarse(K0 - 1);
    store_coarse(K0 - 1);
    load_coarse(K0);
    store_coarse(K0);
    load_coarse(K0 + 1);
    load_fine(K0, fv);
    store_coarse(K0 + 1);
    __syncthreads();
    const int cy = (y >> 1) - Y0 + 1, cy1 = (y & 1) ? cy + 1 : cy - 1, cx = qx + 1;
    for (int K = K0; K < K1; ++K) {
        T fn[2][2][3];
        if (K + 1 < K1) {
            load_coarse(K + 2);
            load_fine(K + 1, fn);
        }
        const int s1 = slot(K);
#pragma unroll
        for (int dz = 0; dz < 2; ++dz) {
            const int sz = slot(dz ? K + 1 : K - 1);  // plane K-1 for fine plane 2K, K+1 for 2K+1
#pragma unroll
            for (int fl = 0; fl < 3; ++fl) {
                double w[3];  // y/z-interpolated values at X-1, X, X+1
#pragma unroll
                for (int xx = 0; xx < 3; ++xx)
                    w[xx] = 0.75 * (0.75 * ce[fl][s1][cy][cx - 1 + xx] +
                                    0.25 * ce[fl][s1][cy1][cx - 1 + xx]) +
                            0.25 * (0.75 * ce[fl][sz][cy][cx - 1 + xx] +
                                    0.25 * ce[fl][sz][cy1][cx - 1 + xx]);
                T *ff = fl == 0 ? fine.a : (fl == 1 ? fine.b : fine.c);
                const bool c1x0 = ((y + dz) & 1) != 0;  // the pair's even-x point is colour 1
                const unsigned g0 = sidx32(LF, x0 + 2 * qx, y, 2 * K + dz);
                const unsigned g1 = sidx32(LF, x0 + 2 * qx + 1, y, 2 * K + dz);
                if (fl == 0 || !phi0 || c1x0)
                    ff[g0] = (T)((double)fv[dz][0][fl] + (0.75 * w[1] + 0.25 * w[0]));
                if (fl == 0 || !phi0 || !c1x0)
                    ff[g1] = (T)((double)fv[dz][1][fl] + (0.75 * w[1] + 0.25 * w[2]));
            }
        }
        if (K + 1 < K1) {
            __syncthreads();  // plane K-1's slot is free
            store_coarse(K + 2);
#pragma unroll
            for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx)
#pragma unroll
                    for (int fl = 0; fl < 3; ++fl) fv[dz][dx][fl] = fn[dz][dx][fl];
            __syncthreads();
        }
    }
}

// Resident workgroups of the tiled interpolation on `device` (0 if the query
// fails), for T = double and float.
int prolong_tile_slots(int device, bool fp32) {
    int occ = 0, cus = 0;
    const void *fn = fp32 ? (const void *)k_prolong_tile<float> : (const void *)k_prolong_tile<double>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kBlock, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return occ * cus;
}

// Coarse-plane ranges per column of the tiled interpolation: one resident
// wave of workgroups (a partly filled second wave costs as much as a full
// one), at most one workgroup per coarse plane of a column.
int prolong_tile_nzr(int slots, int nc, int nf) {
    if (nf % kPX != 0 || nf % kPY != 0) return 1;  // no tiled interpolation onto this level
    const int cols = (nf / kPX) * (nf / kPY);
    const int want = slots > 0 ? std::max(1, slots / cols) : 8;
    return std::max(1, std::min(want, nc));
}

template <typename T>
void launch_prolong(hipStream_t s, const Lay &coarse, const Lay &fine, Tri<const T> v,
                    Tri<const T> ubar, Tri<T> fine_u, const int *gate, bool phi0, int nzr) {
    const size_t pairs = (size_t)coarse.n * fine.n * fine.n;
    const bool tile = fine.split && fine.n % kPX == 0 && fine.n % kPY == 0;
    if (fine_u.b && tile) {
        // coarse error formed while its planes are staged (the value
        // coarse_err_body stores); ubar is left as it is
        if (nzr <= 0) nzr = prolong_tile_nzr(0, coarse.n, fine.n);
        const unsigned blocks = (unsigned)((fine.n / kPX) * (fine.n / kPY) * nzr);
        hipLaunchKernelGGL((k_prolong_tile<T>), dim3(blocks), dim3(kBlock), 0, s, coarse, fine, v,
                           ubar, fine_u, gate, phi0 ? 1 : 0, nzr);
        return;
    }
    // thread per fine pair; with ubar it forms v - ubar where it reads it
    hipLaunchKernelGGL((k_prolong<T>), dim3(blocks_for(pairs)), dim3(kBlock), 0, s, coarse, fine, v,
                       ubar, fine_u, gate, phi0 ? 1 : 0);
}

// ------------------------------------------------------ coarsest solve
//
// Exact solve of N_c(u) = f on the coarsest level (natural layout, n = 3 or
// 4, P = n^3 <= 64 points), one 64-lane wavefront, lane p owning point p.
// omega and mu enter linearly and are eliminated exactly:
//   F(phi) = phi - tau Lap(g(phi) + (1-eps)/2 phi) - tau/2 Lap^3 phi - b = 0,
//   b = f1 + tau Lap(f2 + Lap f3),
//   F'(phi) = I - tau Lap diag(g'(phi) + (1-eps)/2) - tau/2 Lap^3,
// then omega = f3 + Lap phi / 2 and mu = f2 + g(phi) + (1-eps)/2 phi + Lap omega.
// Iteration: phi <- phi - Minv F(phi) with Minv = F'(phi_0)^{-1} kept across
// calls (chord method); when an iteration contracts by less than 4x, Minv is
// rebuilt at the current iterate (which makes that step a Newton step).  The
// inverse comes from Gauss-Jordan elimination with partial pivoting in LDS.
// Stops when max|update| <= 1e-14 max(1, max|phi|) (or after 60 iterations).
// First-order scheme (op.fo): g(phi) = phi^3, (1-eps) phi, the Lap^3 term with
// tau instead of tau/2 and omega = f3 + Lap phi.
// MOB (variable mobility): the outer Lap of the first equation becomes the
// flux operator L_M = d(M D), so F(phi) = phi - tau L_M(g(phi) + (1-eps)/2 phi)
// - tau/2 L_M Lap^2 phi - b with b = f1 + tau L_M(f2 + Lap f3); its Jacobian
// uses the dense Lap^2 (lap2) for the L_M Lap^2 block.
template <typename T, bool DELTA, bool MOB = false>
__device__ __forceinline__ void coarse_body(const OpParams &op, Tri<T> u, Tri<const T> f,
                                            const T *__restrict__ phk, const T *__restrict__ base,
                                            const double *__restrict__ lap1,
                                            const double *__restrict__ lap3, double *minv,
                                            int *valid, int *iters,
                                            const double *__restrict__ lap2 = nullptr) {
    __shared__ double A[64 * 64];  // column-major: A[col * P + row]
    __shared__ double vec[64];
    __shared__ double dvec[64];
    __shared__ int perm[64];
    const int n = op.lay.n, P = n * n * n;
    const int p = threadIdx.x;
    const bool act = p < P;
    const double h2inv = op.h2inv, tau = op.tau, lc = lin_of(op), w3 = w3_of(op);

    int nb[6] = {0, 0, 0, 0, 0, 0};
    if (act) {
        const int i = p % n, j = (p / n) % n, k = p / (n * n);
        nb[0] = (k * n + j) * n + wrap_p(i, n);
        nb[1] = (k * n + j) * n + wrap_m(i, n);
        nb[2] = (k * n + wrap_p(j, n)) * n + i;
        nb[3] = (k * n + wrap_m(j, n)) * n + i;
        nb[4] = (wrap_p(k, n) * n + j) * n + i;
        nb[5] = (wrap_m(k, n) * n + j) * n + i;
    }
    // Lap of the field held in vec[] at point p (call between barriers)
    auto lap_lds = [&](double own) -> double {
        return ((vec[nb[0]] + vec[nb[1]]) + (vec[nb[2]] + vec[nb[3]]) + (vec[nb[4]] + vec[nb[5]]) -
                6.0 * own) * h2inv;
    };
    // face mobilities of point p (MOB), and L_M of the field held in vec[]
    double mf[6] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0}, msum = 6.0;
    if constexpr (MOB) {
        if (act) {
            msum = 0.0;
            for (int e = 0; e < 6; ++e) {
                mf[e] = face_mob(op.mob, op.mob.phs[p], op.mob.phs[nb[e]]);
                msum += mf[e];
            }
        }
    }
    auto lapo_lds = [&](double own) -> double {  // the first equation's outer operator
        if constexpr (MOB) {
            double sm = 0.0;
            for (int e = 0; e < 6; ++e) sm += mf[e] * (vec[nb[e]] - own);
            return sm * h2inv;
        } else {
            return lap_lds(own);
        }
    };
    const double a = act ? (double)phk[p] : 0.0;
    const double bs = (DELTA && act) ? (double)base[p] : 0.0;
    const double F1 = act ? (double)f.a[p] : 0.0;
    const double F2 = act ? (double)f.b[p] : 0.0;
    const double F3 = act ? (double)f.c[p] : 0.0;
    double x = act ? (double)u.a[p] : 0.0;

    vec[p] = F3;
    __syncthreads();
    const double t3 = act ? lap_lds(F3) : 0.0;
    __syncthreads();
    vec[p] = F2 + t3;
    __syncthreads();
    const double bp = F1 + tau * (act ? lapo_lds(F2 + t3) : 0.0);
    __syncthreads();

    // Builds Minv = F'(x)^{-1} into global memory.
    auto rebuild = [&]() {
        dvec[p] = dg_of<DELTA>(op.fo, x, a, bs) + lc;
        __syncthreads();
        if (act && !MOB) {
            // row p of F'(x); the dense Lap and Lap^3 come from global memory,
            // so their loads are issued 16 at a time ahead of the stores
            for (int q0 = 0; q0 < P; q0 += 16) {
                double l1v[16], l3v[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int q = q0 + i;
                    l1v[i] = q < P ? lap1[q * P + p] : 0.0;
                    l3v[i] = q < P ? lap3[q * P + p] : 0.0;
                }
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int q = q0 + i;
                    if (q < P)
                        A[q * P + p] =
                            (q == p ? 1.0 : 0.0) - tau * l1v[i] * dvec[q] - w3 * tau * l3v[i];
                }
            }
        }
        if constexpr (MOB) {
            if (act)
                for (int q = 0; q < P; ++q) {
                    // row p of L_M and of L_M Lap^2 (lap2 column-major: [col * P + row])
                    double lm = q == p ? -msum : 0.0, lmd2 = -msum * lap2[q * P + p];
                    for (int e = 0; e < 6; ++e) {
                        if (nb[e] == q) lm += mf[e];
                        lmd2 += mf[e] * lap2[q * P + nb[e]];
                    }
                    A[q * P + p] = (q == p ? 1.0 : 0.0) - tau * (lm * h2inv) * dvec[q] -
                                   0.5 * tau * (lmd2 * h2inv);
                }
        }
        __syncthreads();
        gj_invert(A, P, perm);
        if (act)
            for (int q = 0; q < P; ++q) minv[q * P + p] = A[q * P + p];
        __syncthreads();
    };

    bool fresh = false;
    if (!*valid) {
        rebuild();
        fresh = true;
    }
    double dprev = 0.0;
    int it;
    for (it = 1; it <= 60; ++it) {
        const double w = g_of<DELTA>(op.fo, x, a, bs) + lc * x;
        vec[p] = w;
        __syncthreads();
        const double lw = act ? lapo_lds(w) : 0.0;
        __syncthreads();
        vec[p] = x;
        __syncthreads();
        const double l1 = act ? lap_lds(x) : 0.0;
        __syncthreads();
        vec[p] = l1;
        __syncthreads();
        const double l2 = act ? lap_lds(l1) : 0.0;
        __syncthreads();
        vec[p] = l2;
        __syncthreads();
        const double l3 = act ? lapo_lds(l2) : 0.0;
        __syncthreads();
        dvec[p] = act ? (x - tau * lw - w3 * tau * l3 - bp) : 0.0;
        __syncthreads();
        double d = 0.0;
        if (act)
            for (int q = 0; q < P; ++q) d -= minv[q * P + p] * dvec[q];
        x += d;
        const double dm = wave_max(fabs(d));
        const double xm = wave_max(fabs(x));
        __syncthreads();
        if (!(dm == dm)) break;
        if (dm <= 1e-14 * fmax(1.0, xm)) break;
        if (!fresh && it > 1 && dm > 0.25 * dprev) {
            rebuild();
            fresh = true;
        } else {
            fresh = false;
        }
        dprev = dm;
    }
    if (it > 60) it = 60;
    vec[p] = x;
    __syncthreads();
    const double lx = act ? lap_lds(x) : 0.0;
    __syncthreads();
    const double om = F3 + w3 * lx;
    vec[p] = om;
    __syncthreads();
    const double lom = act ? lap_lds(om) : 0.0;
    const double mu = F2 + g_of<DELTA>(op.fo, x, a, bs) + lc * x + lom;
    if (act) {
        u.a[p] = (T)x;
        u.b[p] = (T)mu;
        u.c[p] = (T)om;
    }
    if (p == 0) {
        *valid = 1;
        if (iters) *iters = it;
    }
}

// With ubar.a set, the level's tau correction comes first: f += N(I u) with
// I u = ubar (f holds I r; written through fw, the same buffer as f) and the
// iterate starts at I u, as the tau kernel does, then a barrier.
template <typename T, bool DELTA, bool MOB>
__global__ __launch_bounds__(64) void k_coarse(OpParams op, Tri<T> u, Tri<const T> f,
                                               const T *__restrict__ phk,
                                               const T *__restrict__ base,
                                               const double *__restrict__ lap1,
                                               const double *__restrict__ lap3, double *minv,
                                               int *valid, int *iters,
                                               const double *__restrict__ lap2, Tri<const T> ubar,
                                               Tri<T> fw) {
    if (gate_closed(op.gate)) return;
    if (ubar.a) {
        for (unsigned t = threadIdx.x; t < (unsigned)npts(op.lay); t += blockDim.x)
            tau_body<T, DELTA, MOB>(op, ubar, fw, u, phk, base, t);
        __syncthreads();
    }
    coarse_body<T, DELTA, MOB>(op, u, f, phk, base, lap1, lap3, minv, valid, iters, lap2);
}

template <typename T, bool DELTA>
void launch_coarse(hipStream_t s, const OpParams &op, Tri<T> u, Tri<const T> f, const T *phk,
                   const T *base, const double *lap1, const double *lap3, double *minv, int *,
                   int *valid, int *iters, const double *lap2, Tri<const T> ubar, Tri<T> fw) {
    if constexpr (!DELTA) {
        if (op.mob.phs) {
            hipLaunchKernelGGL((k_coarse<T, false, true>), dim3(1), dim3(64), 0, s, op, u, f, phk,
                               base, lap1, lap3, minv, valid, iters, lap2, ubar, fw);
            return;
        }
    }
    hipLaunchKernelGGL((k_coarse<T, DELTA, false>), dim3(1), dim3(64), 0, s, op, u, f, phk, base,
                       lap1, lap3, minv, valid, iters, lap2, ubar, fw);
}

// --------------------------------------------------------------- source

// S of (scheme-PFC-s1..s3) from natural-layout phi^k and phi^{k-1}, written
// in layout op.lay: f1 = phk, f2 = (1-eps)/2 phk + 3 Lap phk - Lap phkm1,
// f3 = Lap phk / 2; for the first-order scheme (phk, 2 Lap phk, 0).
__global__ __launch_bounds__(kBlock) void k_source(OpParams op, Lay nat, const double *__restrict__ phk,
                                                   const double *__restrict__ phkm1,
                                                   Tri<double> f) {
    const unsigned t = xcd_block() * kBlock + threadIdx.x;
    if (t >= (unsigned)npts(nat)) return;
    int i, j, k;
    decode(nat, t, i, j, k);
    const Off q = offs(nat, i, j, k);
    const double v = phk[q.c];
    const double lk = (nsum(phk, q) - 6.0 * v) * op.h2inv;
    const double lkm1 = (nsum(phkm1, q) - 6.0 * phkm1[q.c]) * op.h2inv;
    const unsigned o = sidx32(op.lay, i, j, k);
    f.a[o] = v;
    if (op.fo) {  // first-order scheme: (phi^k, 2 Lap phi^k, 0)
        f.b[o] = 2.0 * lk;
        f.c[o] = 0.0;
    } else {
        f.b[o] = 0.5 * (1.0 - op.eps) * v + 3.0 * lk - lkm1;
        f.c[o] = 0.5 * lk;
    }
}

void launch_source(hipStream_t s, const OpParams &op, const double *phk, const double *phkm1,
                   Tri<double> f) {
    const Lay nat = make_lay(op.lay.n, false);
    hipLaunchKernelGGL(k_source, dim3(blocks_for(npts_host(nat))), dim3(kBlock), 0, s, op, nat, phk,
                       phkm1, f);
}

// phi* = 3/2 phi^k - 1/2 phi^{k-1}, the extrapolation at which the variable
// mobility is evaluated (second order in tau); t runs over storage offsets.
__global__ __launch_bounds__(kBlock) void k_phistar(Lay L, const double *__restrict__ phk,
                                                    const double *__restrict__ phkm1,
                                                    double *__restrict__ out) {
    const unsigned t = xcd_block() * kBlock + threadIdx.x;
    if (t >= (unsigned)npts(L)) return;
    int i, j, k;
    decode(L, t, i, j, k);
    const size_t nat = ((size_t)k * L.n + j) * L.n + i;
    out[t] = 1.5 * phk[nat] - 0.5 * phkm1[nat];
}

void launch_phistar(hipStream_t s, const Lay &L, const double *phk, const double *phkm1,
                    double *out) {
    hipLaunchKernelGGL(k_phistar, dim3(blocks_for(npts_host(L))), dim3(kBlock), 0, s, L, phk, phkm1,
                       out);
}

__global__ __launch_bounds__(kBlock) void k_lap(OpParams op, const double *__restrict__ v,
                                                double *__restrict__ out) {
    const Lay &L = op.lay;
    const unsigned t = xcd_block() * kBlock + threadIdx.x;
    if (t >= (unsigned)npts(L)) return;
    int i, j, k;
    decode(L, t, i, j, k);
    const Off q = offs(L, i, j, k);
    out[q.c] = (nsum(v, q) - 6.0 * v[q.c]) * op.h2inv;
}

// mu = phi^3 + (1-eps) phi + 2 Lap phi + Lap^2 phi, with om = Lap phi given.
__global__ __launch_bounds__(kBlock) void k_init_mu(OpParams op, const double *__restrict__ phi,
                                                    const double *__restrict__ om,
                                                    double *__restrict__ mu) {
    const Lay &L = op.lay;
    const unsigned t = xcd_block() * kBlock + threadIdx.x;
    if (t >= (unsigned)npts(L)) return;
    int i, j, k;
    decode(L, t, i, j, k);
    const Off q = offs(L, i, j, k);
    const double v = phi[q.c];
    const double l2 = (nsum(om, q) - 6.0 * om[q.c]) * op.h2inv;
    mu[q.c] = v * v * v + (1.0 - op.eps) * v + 2.0 * om[q.c] + l2;
}

void launch_init_guess(hipStream_t s, const OpParams &nat, const double *phi0, double *mu,
                       double *om) {
    const unsigned blocks = blocks_for(npts_host(nat.lay));
    hipLaunchKernelGGL(k_lap, dim3(blocks), dim3(kBlock), 0, s, nat, phi0, om);
    hipLaunchKernelGGL(k_init_mu, dim3(blocks), dim3(kBlock), 0, s, nat, phi0, om, mu);
}

// ------------------------------------------------------ layout conversion

template <typename S, typename D, bool TO>
__global__ __launch_bounds__(kBlock) void k_relayout(Lay L, const S *__restrict__ src,
                                                     D *__restrict__ dst, int count) {
    const unsigned t = xcd_block() * kBlock + threadIdx.x;
    const size_t P = npts(L);
    if (t >= (unsigned)P) return;
    int i, j, k;
    decode(L, t, i, j, k);  // t: storage offset in L
    const size_t nat = ((size_t)k * L.n + j) * L.n + i;
    for (int c = 0; c < count; ++c) {
        if (TO)
            dst[c * P + t] = (D)src[c * P + nat];
        else
            dst[c * P + nat] = (D)src[c * P + t];
    }
}

template <typename S, typename D>
void launch_to_lay(hipStream_t s, const Lay &lay, const S *src, D *dst, int count) {
    hipLaunchKernelGGL((k_relayout<S, D, true>), dim3(blocks_for(npts_host(lay))), dim3(kBlock), 0,
                       s, lay, src, dst, count);
}

template <typename S, typename D>
void launch_from_lay(hipStream_t s, const Lay &lay, const S *src, D *dst, int count) {
    hipLaunchKernelGGL((k_relayout<S, D, false>), dim3(blocks_for(npts_host(lay))), dim3(kBlock), 0,
                       s, lay, src, dst, count);
}

// --------------------------------------------------------------- energy

int energy_blocks(int n) { return (int)reduce_blocks((size_t)n * n * n); }

// Per-block sums of phi^4, phi^2, (D phi)^2 on the cell's three forward faces
// (so every face of the periodic grid is counted once), (Lap phi)^2, the same
// face sum for phi - phi_prev, and phi.  Scaled by h^3 in the final pass.
__global__ __launch_bounds__(kBlock) void k_energy_part(Lay L, double hinv, double h2inv,
                                                        const double *__restrict__ phi,
                                                        const double *__restrict__ prev,
                                                        double *__restrict__ part) {
    __shared__ double red[6][kBlock];
    double s[6] = {0, 0, 0, 0, 0, 0};
    const unsigned total = (unsigned)npts(L);
    for (unsigned t = blockIdx.x * kBlock + threadIdx.x; t < total; t += gridDim.x * kBlock) {
        int i, j, k;
        decode(L, t, i, j, k);
        const Off q = offs(L, i, j, k);
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

void launch_energy(hipStream_t s, const Lay &nat, double h, double eps, const double *phi,
                   const double *phi_prev, double *partial, double *out3) {
    const int blocks = energy_blocks(nat.n);
    hipLaunchKernelGGL(k_energy_part, dim3(blocks), dim3(kBlock), 0, s, nat, 1.0 / h, 1.0 / (h * h),
                       phi, phi_prev, partial);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, s, partial, blocks, h, eps, out3);
}

// ------------------------------------------------ mixed-precision helpers

__global__ __launch_bounds__(kBlock) void k_add_correction(size_t P, Tri<double> u,
                                                           Tri<const float> e) {
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    if (t >= P) return;
    u.a[t] += (double)e.a[t];
    u.b[t] += (double)e.b[t];
    u.c[t] += (double)e.c[t];
}

void launch_add_correction(hipStream_t s, size_t P, Tri<double> u, Tri<const float> e) {
    hipLaunchKernelGGL(k_add_correction, dim3(blocks_for(P)), dim3(kBlock), 0, s, P, u, e);
}

__global__ __launch_bounds__(kBlock) void k_resid_cast(OpParams op, Tri<const double> u,
                                                       Tri<const double> f,
                                                       const double *__restrict__ phk,
                                                       Tri<float> r32, float *__restrict__ base32,
                                                       unsigned long long *partial) {
    const Lay &L = op.lay;
    const unsigned total = (unsigned)npts(L);
    unsigned long long m = 0;
    for (unsigned t = xcd_block() * kBlock + threadIdx.x; t < total; t += gridDim.x * kBlock) {
        int i, j, k;
        decode(L, t, i, j, k);
        const Off q = offs(L, i, j, k);
        double r1, r2, r3;
        resid_at<double, false>(op, u, f, phk, nullptr, q, r1, r2, r3);
        r32.a[t] = (float)r1;
        r32.b[t] = (float)r2;
        r32.c[t] = (float)r3;
        base32[t] = (float)u.a[t];
        m = umax(m, umax(abs_bits(r1), umax(abs_bits(r2), abs_bits(r3))));
    }
    m = block_max_u64(m);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

int launch_resid_cast(hipStream_t s, const OpParams &op, Tri<const double> u, Tri<const double> f,
                      const double *phk, Tri<float> r32, float *base32,
                      unsigned long long *partial) {
    const unsigned blocks = reduce_blocks(npts_host(op.lay));
    hipLaunchKernelGGL(k_resid_cast, dim3(blocks), dim3(kBlock), 0, s, op, u, f, phk, r32, base32,
                       partial);
    return (int)blocks;
}

__global__ __launch_bounds__(kBlock) void k_zero(float *p, size_t count) {
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    if (t < count) p[t] = 0.0f;
}

void launch_zero(hipStream_t s, float *p, size_t count) {
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(count)), dim3(kBlock), 0, s, p, count);
}

// ----------------------------------------------------------- batched form
//
// Every multigrid phase of the batched cycle is one launch over all
// instances that take part in it.  Each instance's part of the phase (its
// "segment": half-sweep points of one colour, coarse cells, fine x-pairs or
// points) is seen as planes of work items in z, and cut into tiles of W
// consecutive items of a plane in Z consecutive planes, walked plane by
// plane, so the neighbouring planes a stencil reads are reused while they
// are still cached; the tiles of all segments form one work-list, in segment
// order.  Two schedules walk it:
//   * one tile per workgroup, the hardware dispatcher handing out tiles
//     (PERSIST = false: grid = tile count);
//   * persistent: only as many workgroups as are resident at once, each
//     taking every gridDim.x-th tile (PERSIST = true).
// A workgroup finds a tile's segment by a binary search over the segments'
// first tiles (precomputed for every tile shape) and skips tiles of
// instances whose convergence flag is cleared.  Schedule, tile shape and
// workgroup size are per phase kind, chosen by the batch's autotuner.  The
// per-item arithmetic is that of the single-instance kernels, so neither
// changes any result.

// Q items per plane and NPL planes of a segment's work (item = plane * Q +
// position), in the bodies' own item orders: a half-sweep's points of one
// colour (planes k), coarse cells and fine x-pairs in natural order (planes
// K and k), the points of a colour-split level colour-major (2n planes of
// n * n/2, else n planes of n * n), and the pointwise coarse error as one
// plane.
__host__ __device__ __forceinline__ void bseg_planes(const BSeg &g, int kind, unsigned &Q,
                                                     unsigned &NPL) {
    const unsigned n = (unsigned)g.op.lay.n, nc = (unsigned)g.lay_c.n;
    switch (kind) {
        case BK_SMOOTH: Q = n * (n / 2); NPL = n; break;
        case BK_RR: Q = nc * nc; NPL = nc; break;
        case BK_PROLONG: Q = nc * n; NPL = n; break;
        case BK_ERR: Q = nc * nc * nc; NPL = 1; break;
        default:  // BK_TAU, BK_NORM: the level's storage order
            if (g.op.lay.split) {
                Q = n * (n / 2);
                NPL = 2 * n;
            } else {
                Q = n * n;
                NPL = n;
            }
    }
}

void bseg_planes_host(const BSeg &g, int kind, unsigned &Q, unsigned &NPL) {
    bseg_planes(g, kind, Q, NPL);
}

// Segment holding work-list tile `tile` for tile shape `shape`.
__device__ __forceinline__ int bseg_of_tile(const BSeg *segs, int nseg, int kind, int shape,
                                            unsigned tile, unsigned &local) {
    int lo = 0, hi = nseg - 1;  // the last segment whose first tile is <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].first[kind][shape] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    local = tile - segs[lo].first[kind][shape];
    return lo;
}

// Item range of one tile of a segment: planes [z0, z1), positions [w0, w1).
struct TileSpan {
    unsigned Q, z0, z1, w0, w1;
};

__device__ __forceinline__ TileSpan tile_span(const BSeg &g, int kind, int shape, unsigned local) {
    const unsigned W = (unsigned)kTileMin << (shape % kWOpts), Z = 1u << (shape / kWOpts);
    unsigned Q, NPL;
    bseg_planes(g, kind, Q, NPL);
    const unsigned nw = (Q + W - 1) / W;
    const unsigned pz = local / nw, pw = local - pz * nw;
    TileSpan sp;
    sp.Q = Q;
    sp.z0 = pz * Z;
    sp.z1 = min(sp.z0 + Z, NPL);
    sp.w0 = pw * W;
    sp.w1 = min(sp.w0 + W, Q);
    return sp;
}

template <int KIND, bool PK1, bool TAU>
__device__ __forceinline__ void kb_item(const BSeg &g, unsigned i, int arg0, int arg1) {
    if constexpr (KIND == BK_SMOOTH && TAU) {  // colour as a constant: loads in one block
        if (arg0 == 0)
            smooth_body<double, false, false, false, true, 0>(g.op, 0, arg1 & 1, g.u, cst(g.f),
                                                              g.phk, nullptr, i, cst(g.ubar), g.f);
        else
            smooth_body<double, false, false, false, true, 1>(g.op, 1, arg1 & 1, g.u, cst(g.f),
                                                              g.phk, nullptr, i, cst(g.ubar), g.f);
    } else if constexpr (KIND == BK_SMOOTH) {
        smooth_body<double, false, false, PK1>(g.op, arg0, arg1 & 1, g.u, cst(g.f), g.phk, nullptr,
                                               i);
    } else if constexpr (KIND == BK_RR) {
        resid_restrict_body<double, false>(g.op, g.lay_c, cst(g.u), cst(g.f), g.phk, nullptr,
                                           g.ubarc, g.fc, i);
    } else if constexpr (KIND == BK_TAU) {
        tau_body<double, false>(g.op, cst(g.ubar), g.f, g.u, g.phk, nullptr, i);
    } else if constexpr (KIND == BK_ERR) {  // coarse error v - I u, stored over I u
        coarse_err_body<double>(npts(g.lay_c), cst(g.uc), g.ubarc, i);
    } else {  // BK_PROLONG: adds the interpolated coarse error
        prolong_body<double>(g.lay_c, g.op.lay, cst(g.ubarc),
                             Tri<const double>{nullptr, nullptr, nullptr}, g.u, i, arg0 != 0);
    }
}

// arg0, arg1: colour and picard (BK_SMOOTH); 1 when a smoothing sweep
// follows (BK_PROLONG: colour-0 mu, omega left unwritten).  PK1 (BK_SMOOTH,
// arg1 | 2): every segment's f.a is its phi^k (the finest levels), loaded once.
// TAU (BK_SMOOTH, arg1 | 4): the first sweep of coarse levels, forming the tau
// correction from I u as it smooths (smooth_body).
template <int KIND, bool PERSIST, bool PK1 = false, bool TAU = false>
__global__ __launch_bounds__(512) void kb_phase(const BSeg *segs, int nseg, unsigned ntiles,
                                                int shape, int arg0, int arg1) {
    for (unsigned t = blockIdx.x; t < ntiles; t += PERSIST ? gridDim.x : ntiles) {
        unsigned local;
        const BSeg &g = segs[bseg_of_tile(segs, nseg, KIND, shape, t, local)];
        if (!*g.active) continue;
        const TileSpan sp = tile_span(g, KIND, shape, local);
        for (unsigned z = sp.z0; z < sp.z1; ++z)
            for (unsigned r = sp.w0 + threadIdx.x; r < sp.w1; r += blockDim.x)
                kb_item<KIND, PK1, TAU>(g, z * sp.Q + r, arg0, arg1);
    }
}

// tau: each segment's tau correction first (as k_coarse with ubar set).
__global__ __launch_bounds__(64) void kb_coarse(const BSeg *segs, int nseg, int tau) {
    const int s = blockIdx.x;
    if (s >= nseg || !*segs[s].active) return;
    const BSeg &g = segs[s];
    if (tau) {
        for (unsigned t = threadIdx.x; t < (unsigned)npts(g.op.lay); t += blockDim.x)
            tau_body<double, false>(g.op, cst(g.ubar), g.f, g.u, g.phk, nullptr, t);
        __syncthreads();
    }
    coarse_body<double, false>(g.op, g.u, cst(g.f), g.phk, nullptr, g.lap1, g.lap3, g.minv, g.valid,
                               g.iters);
}

// Residual maxima of every instance's finest level, one per norm tile
// (shape kNormShape, one workgroup each, so that each instance owns a known
// range of partial[]); tiles of finished instances leave 0.
__global__ __launch_bounds__(kBlock) void kb_norm(const BSeg *segs, int nseg,
                                                  unsigned long long *partial) {
    unsigned local;
    const BSeg &g = segs[bseg_of_tile(segs, nseg, BK_NORM, kNormShape, blockIdx.x, local)];
    unsigned long long m = 0;
    if (*g.active) {
        const TileSpan sp = tile_span(g, BK_NORM, kNormShape, local);
        for (unsigned z = sp.z0; z < sp.z1; ++z)
            for (unsigned r = sp.w0 + threadIdx.x; r < sp.w1; r += blockDim.x)
                m = umax(m, resid_bits<double, false>(g.op, cst(g.u), cst(g.f), g.phk, nullptr,
                                                      Tri<double>{nullptr, nullptr, nullptr},
                                                      z * sp.Q + r));
    }
    m = block_max_u64(m);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// Stop test of every instance (one workgroup per instance): residual
// max-norm from its partials, then the rule of the single-instance driver:
// finished if the norm is at most tol (or not finite, or max_cycles cycles
// were done), otherwise one more cycle is counted.
__global__ __launch_bounds__(kBlock) void kb_update(const BSeg *segs, int nseg,
                                                    const unsigned long long *partial, BState st,
                                                    double tol, int max_cycles) {
    const int s = blockIdx.x;
    if (s >= nseg) return;
    const int i = segs[s].inst;
    const unsigned b0 = st.norm_first[s], b1 = b0 + st.norm_blocks[s];
    unsigned long long m = 0;
    for (unsigned b = b0 + threadIdx.x; b < b1; b += kBlock) m = umax(m, partial[b]);
    m = block_max_u64(m);
    if (threadIdx.x != 0 || !st.active[i]) return;
    const double r = __longlong_as_double((long long)m);
    if (st.cycles[i] == 0) st.res0[i] = r;
    st.res[i] = r;
    if (!(r <= 1.7976931348623157e308)) {  // NaN or Inf
        st.status[i] = PFC_ERR_NONFINITE;
        st.active[i] = 0;
    } else if (r <= tol) {
        st.active[i] = 0;
    } else if (st.cycles[i] == max_cycles) {
        st.status[i] = PFC_ERR_NOT_CONVERGED;
        st.active[i] = 0;
    } else {
        st.cycles[i] += 1;
    }
}

// Batched column-tiled interpolation: the tile of k_prolong_tile for one
// instance (segment) per workgroup, a PX x 8 fine column and the coarse
// planes [K0, K0 + 2^zi) of it, found through the segments' first tiles
// (BSeg::ptf).  The coarse error v - I u is formed as a coarse plane is
// staged, rounded as coarse_err_body stores it, and I u is left as it is;
// same weights and operation order as prolong_body.  phi0: colour-0 mu and
// omega are neither read nor written (a smoothing sweep follows).
template <int PX>
__global__ __launch_bounds__(4 * PX) void kb_prolong_tile(const BSeg *segs, int nseg, int zi,
                                                          int phi0) {
    constexpr int HX = PX / 2, CW = HX + 2, CH = 8 / 2 + 2, CN = CW * CH;
    static_assert(CN <= 4 * PX, "one coarse ring cell per thread");
    __shared__ double ce[3][3][CH][CW];  // [field][plane slot][Y][X]
    const unsigned tile = blockIdx.x;
    int lo = 0, hi = nseg - 1;  // the last segment whose first tile is <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].ptf[zi] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BSeg &g = segs[lo];
    if (!*g.active) return;
    const Lay &LF = g.op.lay, &LC = g.lay_c;
    const Tri<const double> v = cst(g.uc), ubar = cst(g.ubarc);
    const Tri<double> fine = g.u;
    const int nc = LC.n, nf = LF.n;
    const unsigned local = tile - g.ptf[zi];
    const int nbx = nf / PX, nby = nf / 8;
    const int bx = (int)(local % (unsigned)nbx), by = (int)((local / (unsigned)nbx) % (unsigned)nby);
    const int bz = (int)(local / (unsigned)(nbx * nby));
    const int x0 = bx * PX, y0 = by * 8, X0 = x0 / 2, Y0 = y0 / 2;
    const int K0 = bz << zi, K1 = min(K0 + (1 << zi), nc);
    const int tid = threadIdx.x, qx = tid % HX, qy = tid / HX;
    const int y = y0 + qy;
    auto wc = [nc](int q) { return q < 0 ? q + nc : (q >= nc ? q - nc : q); };
    auto slot = [K0](int P) { return (P - K0 + 4) % 3; };  // P >= K0 - 1
    const int cpy = tid / CW, cpx = tid - cpy * CW;
    double cn[3];
    auto load_coarse = [&](int P) {
        if (tid < CN) {
            const unsigned gi = sidx32(LC, wc(X0 - 1 + cpx), wc(Y0 - 1 + cpy), wc(P));
            cn[0] = v.a[gi] - ubar.a[gi];
            cn[1] = v.b[gi] - ubar.b[gi];
            cn[2] = v.c[gi] - ubar.c[gi];
        }
    };
    auto store_coarse = [&](int P) {
        if (tid < CN) {
            const int sl = slot(P);
            ce[0][sl][cpy][cpx] = cn[0];
            ce[1][sl][cpy][cpx] = cn[1];
            ce[2][sl][cpy][cpx] = cn[2];
        }
    };
    double fv[2][2][3];  // [dz][dx][field]
    auto load_fine = [&](int K, double (&o)[2][2][3]) {
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const unsigned gi = sidx32(LF, x0 + 2 * qx + dx, y, 2 * K + dz);
                o[dz][dx][0] = fine.a[gi];
                if (!phi0 || ((dx + y + dz) & 1)) {  // x0, 2 qx and 2 K are even
                    o[dz][dx][1] = fine.b[gi];
                    o[dz][dx][2] = fine.c[gi];
                } else {  // neither read nor written back
                    o[dz][dx][1] = 0.0;
                    o[dz][dx][2] = 0.0;
                }
            }
    };
    load_coarse(K0 - 1);
    store_coarse(K0 - 1);
    load_coarse(K0);
    store_coarse(K0);
    load_coarse(K0 + 1);
    load_fine(K0, fv);
    store_coarse(K0 + 1);
    __syncthreads();
    const int cy = (y >> 1) - Y0 + 1, cy1 = (y & 1) ? cy + 1 : cy - 1, cx = qx + 1;
    for (int K = K0; K < K1; ++K) {
        double fn[2][2][3];
        if (K + 1 < K1) {
            load_coarse(K + 2);
            load_fine(K + 1, fn);
        }
        const int s1 = slot(K);
#pragma unroll
        for (int dz = 0; dz < 2; ++dz) {
            const int sz = slot(dz ? K + 1 : K - 1);  // plane K-1 for fine plane 2K, K+1 for 2K+1
#pragma unroll
            for (int fl = 0; fl < 3; ++fl) {
                double w[3];  // y/z-interpolated values at X-1, X, X+1
#pragma unroll
                for (int xx = 0; xx < 3; ++xx)
                    w[xx] = 0.75 * (0.75 * ce[fl][s1][cy][cx - 1 + xx] +
                                    0.25 * ce[fl][s1][cy1][cx - 1 + xx]) +
                            0.25 * (0.75 * ce[fl][sz][cy][cx - 1 + xx] +
                                    0.25 * ce[fl][sz][cy1][cx - 1 + xx]);
                double *ff = fl == 0 ? fine.a : (fl == 1 ? fine.b : fine.c);
                const bool c1x0 = ((y + dz) & 1) != 0;  // the pair's even-x point is colour 1
                const unsigned g0 = sidx32(LF, x0 + 2 * qx, y, 2 * K + dz);
                const unsigned g1 = sidx32(LF, x0 + 2 * qx + 1, y, 2 * K + dz);
                if (fl == 0 || !phi0 || c1x0) ff[g0] = fv[dz][0][fl] + (0.75 * w[1] + 0.25 * w[0]);
                if (fl == 0 || !phi0 || !c1x0) ff[g1] = fv[dz][1][fl] + (0.75 * w[1] + 0.25 * w[2]);
            }
        }
        if (K + 1 < K1) {
            __syncthreads();  // plane K-1's slot is free
            store_coarse(K + 2);
#pragma unroll
            for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx)
#pragma unroll
                    for (int fl = 0; fl < 3; ++fl) fv[dz][dx][fl] = fn[dz][dx][fl];
            __syncthreads();
        }
    }
}

bool batch_ptile_fits(const BSeg &g) {
    return g.op.lay.split && g.op.lay.n % kBPX == 0 && g.op.lay.n % 8 == 0 && g.lay_c.n * 2 == g.op.lay.n;
}

unsigned batch_ptile_count(const BSeg &g, int zi) {
    if (!batch_ptile_fits(g)) return 0;
    const unsigned nf = (unsigned)g.op.lay.n, nc = (unsigned)g.lay_c.n, zr = 1u << zi;
    return (nf / kBPX) * (nf / 8) * ((nc + zr - 1) / zr);
}

void launch_batch_ptile(hipStream_t s, const BSeg *segs, int nseg, unsigned ntiles, int zi,
                        int phi0) {
    hipLaunchKernelGGL((kb_prolong_tile<kBPX>), dim3(std::max(ntiles, 1u)), dim3(4 * kBPX), 0, s,
                       segs, nseg, zi, phi0);
}

// Start of a time step: every instance active, counters cleared, cached
// coarsest inverses invalidated.
__global__ __launch_bounds__(kBlock) void kb_reset(BState st, int count, int **valid) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    st.active[i] = 1;
    st.cycles[i] = 0;
    st.status[i] = 0;
    st.res0[i] = 0.0;
    st.res[i] = 0.0;
    *valid[i] = 0;
}

template <int KIND, bool PK1 = false, bool TAU = false>
static void launch_kind(hipStream_t s, const BSeg *segs, int nseg, unsigned ntiles, int shape,
                        int threads, unsigned grid, int arg0, int arg1) {
    if (grid)
        hipLaunchKernelGGL((kb_phase<KIND, true, PK1, TAU>), dim3(grid), dim3(threads), 0, s, segs,
                           nseg, ntiles, shape, arg0, arg1);
    else
        hipLaunchKernelGGL((kb_phase<KIND, false, PK1, TAU>), dim3(std::max(ntiles, 1u)),
                           dim3(threads), 0, s, segs, nseg, ntiles, shape, arg0, arg1);
}

void launch_batch(hipStream_t s, int kind, const BSeg *segs, int nseg, unsigned ntiles, int shape,
                  int threads, unsigned slots, int arg0, int arg1) {
    // persistent: at most the resident workgroups, at most one per tile
    const unsigned grid = slots ? std::max(1u, std::min(slots, ntiles)) : 0u;
    switch (kind) {
        case BK_SMOOTH:
            if (arg1 & 2)
                launch_kind<BK_SMOOTH, true>(s, segs, nseg, ntiles, shape, threads, grid, arg0, arg1);
            else if (arg1 & 4)
                launch_kind<BK_SMOOTH, false, true>(s, segs, nseg, ntiles, shape, threads, grid, arg0,
                                                    arg1);
            else
                launch_kind<BK_SMOOTH>(s, segs, nseg, ntiles, shape, threads, grid, arg0, arg1);
            break;
        case BK_RR: launch_kind<BK_RR>(s, segs, nseg, ntiles, shape, threads, grid, arg0, arg1); break;
        case BK_TAU: launch_kind<BK_TAU>(s, segs, nseg, ntiles, shape, threads, grid, arg0, arg1); break;
        case BK_ERR: launch_kind<BK_ERR>(s, segs, nseg, ntiles, shape, threads, grid, arg0, arg1); break;
        case BK_PROLONG: launch_kind<BK_PROLONG>(s, segs, nseg, ntiles, shape, threads, grid, arg0, arg1); break;
        default: break;
    }
}

int batch_phase_slots(int kind, int threads, int device) {
    const void *fn = nullptr;
    switch (kind) {
        case BK_SMOOTH: fn = (const void *)kb_phase<BK_SMOOTH, true>; break;
        case BK_RR: fn = (const void *)kb_phase<BK_RR, true>; break;
        case BK_TAU: fn = (const void *)kb_phase<BK_TAU, true>; break;
        case BK_ERR: fn = (const void *)kb_phase<BK_ERR, true>; break;
        default: fn = (const void *)kb_phase<BK_PROLONG, true>; break;
    }
    int occ = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return occ * cus;
}

void launch_batch_coarse(hipStream_t s, const BSeg *segs, int nseg, int tau) {
    hipLaunchKernelGGL(kb_coarse, dim3(nseg), dim3(64), 0, s, segs, nseg, tau);
}

void launch_batch_norm(hipStream_t s, const BSeg *segs, int nseg, unsigned ntiles,
                       unsigned long long *partial, BState st, double tol, int max_cycles) {
    hipLaunchKernelGGL(kb_norm, dim3(std::max(ntiles, 1u)), dim3(kBlock), 0, s, segs, nseg, partial);
    hipLaunchKernelGGL(kb_update, dim3(nseg), dim3(kBlock), 0, s, segs, nseg,
                       (const unsigned long long *)partial, st, tol, max_cycles);
}

void launch_batch_reset(hipStream_t s, BState st, int count, int **valid) {
    hipLaunchKernelGGL(kb_reset, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, st, count,
                       valid);
}

// ------------------------------------------------------ instantiations

#define PFC_INST(T, DELTA)                                                                        \
    template void launch_resid_restrict<T, DELTA>(hipStream_t, const OpParams &, const Lay &,     \
                                                  Tri<const T>, Tri<const T>, const T *,          \
                                                  const T *, Tri<T>, Tri<T>);                     \
    template void launch_tau<T, DELTA>(hipStream_t, const OpParams &, Tri<const T>, Tri<T>,       \
                                       Tri<T>, const T *, const T *);                             \
    template int launch_resid_max<T, DELTA>(hipStream_t, const OpParams &, Tri<const T>,          \
                                            Tri<const T>, const T *, const T *, Tri<T>,           \
                                            unsigned long long *);                                \
    template void launch_coarse<T, DELTA>(hipStream_t, const OpParams &, Tri<T>, Tri<const T>,    \
                                          const T *, const T *, const double *, const double *,   \
                                          double *, int *, int *, int *, const double *,          \
                                          Tri<const T>, Tri<T>);

PFC_INST(double, false)
PFC_INST(float, true)
template void launch_restrict<double>(hipStream_t, const Lay &, const Lay &, const double *, double *);
template void launch_restrict<float>(hipStream_t, const Lay &, const Lay &, const float *, float *);
template void launch_prolong<double>(hipStream_t, const Lay &, const Lay &, Tri<const double>,
                                     Tri<const double>, Tri<double>, const int *, bool, int);
template void launch_prolong<float>(hipStream_t, const Lay &, const Lay &, Tri<const float>,
                                    Tri<const float>, Tri<float>, const int *, bool, int);
template void launch_to_lay<double, double>(hipStream_t, const Lay &, const double *, double *, int);
template void launch_from_lay<double, double>(hipStream_t, const Lay &, const double *, double *, int);
template void launch_to_lay<double, float>(hipStream_t, const Lay &, const double *, float *, int);

}  // namespace pfc
