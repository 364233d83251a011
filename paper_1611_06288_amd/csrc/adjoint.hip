// Adjoint of one time step of scheme (1.10) (M = 1), for gradients of a
// loss of phi^{k+1} with respect to phi^k, phi^{k-1} and eps.
//
// The step solution u = (phi^{k+1}, mu, omega) satisfies G = N(u) - S = 0
// (scheme-PFC-o1..o3 and scheme-PFC-s1..s3).  By the implicit-function
// theorem, with J = dN/du at u,
//     J^T lambda = (gbar_next, 0, 0),
//     gbar_cur  += -(dG/dphi^k)^T lambda
//                = lambda1 + (g_a(phi^{k+1}; phi^k) + (1-eps)/2) lambda2
//                  + 3 Lap lambda2 + Lap lambda3 / 2,
//     gbar_prev += -(dG/dphi^{k-1})^T lambda = -Lap lambda2,
//     geps      += -(dG/deps)^T lambda = -1/2 sum lambda2 (phi^{k+1} + phi^k),
// where J = [[I, -tau Lap, 0], [-D, I, -Lap], [-Lap/2, 0, I]],
// D = diag(g_phi(phi^{k+1}; phi^k) + (1-eps)/2), g_a = dg/dphi^k.
//
// J^T lambda = b is solved by linear multigrid (correction scheme) on the
// same hierarchy: red-black block Gauss-Seidel on the 3x3 point blocks of
// J^T, 8-child restriction of the residual and of D, trilinear
// interpolation of the correction, and an exact solve on the coarsest level
// after eliminating lambda2 = b2 + tau Lap lambda1 and
// lambda3 = b3 + Lap lambda2:
//     (I - tau D Lap - tau/2 Lap^3) lambda1 = b1 + D b2 + 1/2 Lap(b3 + Lap b2).
#include <cmath>

#include "device_common.h"
#include "runtime_internal.h"

namespace pfc {

// D = g_phi(phi^{k+1}; phi^k) + (1-eps)/2 from natural-layout fields into `lay`.
__global__ __launch_bounds__(kBlock) void k_adj_D(Lay lay, double eps, const double *__restrict__ phin,
                                                  const double *__restrict__ phk,
                                                  double *__restrict__ D) {
    const unsigned t = xcd_block() * kBlock + threadIdx.x;
    if (t >= (unsigned)npts(lay)) return;
    int i, j, k;
    decode_nat(lay, t, i, j, k);
    D[sidx32(lay, i, j, k)] = Cubic<false>::dg(phin[t], phk[t], 0.0) + 0.5 * (1.0 - eps);
}

// Red-black block Gauss-Seidel on J^T: at a point, with the six neighbours held,
//     lambda1 - c lambda2 + Dd lambda3 = s1 = b1 + S_l3 / (2 h^2)
//     A lambda1 + lambda2              = s2 = b2 + tau S_l1 / h^2
//     B lambda2 + lambda3              = s3 = b3 + S_l2 / h^2
// (A = 6 tau/h^2, B = 6/h^2, Dd = 3/h^2, c = D at the point).
__global__ __launch_bounds__(kBlock) void k_adj_smooth(OpParams op, int colour, Tri<double> lam,
                                                       Tri<const double> b,
                                                       const double *__restrict__ D) {
    const Lay &L = op.lay;
    const int n = L.n, hn = n >> 1;
    const unsigned H = (unsigned)((size_t)n * n * n / 2);
    const unsigned t = xcd_block() * kBlock + threadIdx.x;
    if (t >= H) return;
    const unsigned row = L.dh.q(t);
    const int m = (int)(t - row * (unsigned)hn);
    const int k = (int)L.dn.q(row);
    const int j = (int)(row - (unsigned)k * (unsigned)n);
    const int i = 2 * m + ((colour + j + k) & 1);
    const Off q = offs(L, i, j, k);
    const double s1 = b.a[q.c] + 0.5 * nsum(lam.c, q) * op.h2inv;
    const double s2 = b.b[q.c] + op.tau * nsum(lam.a, q) * op.h2inv;
    const double s3 = b.c[q.c] + nsum(lam.b, q) * op.h2inv;
    const double A = 6.0 * op.tau * op.h2inv, B = 6.0 * op.h2inv, Dd = 3.0 * op.h2inv;
    const double c = D[q.c];
    const double l1 = (s1 + (c + B * Dd) * s2 - Dd * s3) / (1.0 + A * (c + B * Dd));
    const double l2 = s2 - A * l1;
    const double l3 = s3 - B * l2;
    lam.a[q.c] = l1;
    lam.b[q.c] = l2;
    lam.c[q.c] = l3;
}

// r = b - J^T lambda at one point.
__device__ __forceinline__ void adj_resid_at(const OpParams &op, const Tri<const double> &lam,
                                             const Tri<const double> &b, const double *D,
                                             const Off &q, double &r1, double &r2, double &r3) {
    const double l1 = lam.a[q.c], l2 = lam.b[q.c], l3 = lam.c[q.c];
    const double L1 = (nsum(lam.a, q) - 6.0 * l1) * op.h2inv;
    const double L2 = (nsum(lam.b, q) - 6.0 * l2) * op.h2inv;
    const double L3 = (nsum(lam.c, q) - 6.0 * l3) * op.h2inv;
    r1 = b.a[q.c] - (l1 - D[q.c] * l2 - 0.5 * L3);
    r2 = b.b[q.c] - (l2 - op.tau * L1);
    r3 = b.c[q.c] - (l3 - L2);
}

__global__ __launch_bounds__(kBlock) void k_adj_resid_max(OpParams op, Tri<const double> lam,
                                                          Tri<const double> b,
                                                          const double *__restrict__ D,
                                                          unsigned long long *partial) {
    const Lay &L = op.lay;
    const unsigned total = (unsigned)npts(L);
    unsigned long long mx = 0;
    for (unsigned t = xcd_block() * kBlock + threadIdx.x; t < total; t += gridDim.x * kBlock) {
        int i, j, k;
        decode(L, t, i, j, k);
        const Off q = offs(L, i, j, k);
        double r1, r2, r3;
        adj_resid_at(op, lam, b, D, q, r1, r2, r3);
        mx = umax(mx, umax(abs_bits(r1), umax(abs_bits(r2), abs_bits(r3))));
    }
    mx = block_max_u64(mx);
    if (threadIdx.x == 0) partial[blockIdx.x] = mx;
}

// Coarse right-hand side b_c = I (b - J^T lambda), eight threads per coarse
// cell (one per child, child ch = (ch & 1, (ch >> 1) & 1, ch >> 2) in x, y, z),
// so each thread waits on one child's loads; the cell's eight lanes add
// their residuals in the order ch = 0..7 and the first stores b_c and clears
// the coarse iterate lam_c (the coarse problem starts from zero).
__global__ __launch_bounds__(kBlock) void k_adj_resid_restrict(OpParams op, Lay LC,
                                                               Tri<const double> lam,
                                                               Tri<const double> b,
                                                               const double *__restrict__ D,
                                                               Tri<double> bc, Tri<double> lamc) {
    const unsigned g = xcd_block() * kBlock + threadIdx.x;
    const unsigned tn = g >> 3;
    const int ch = (int)(g & 7u);
    const bool act = tn < (unsigned)npts(LC);
    double r[3] = {0.0, 0.0, 0.0};
    unsigned t = 0;
    if (act) {
        int I, J, K;
        decode_nat(LC, tn, I, J, K);
        t = sidx32(LC, I, J, K);
        const Off q = offs(op.lay, 2 * I + (ch & 1), 2 * J + ((ch >> 1) & 1), 2 * K + (ch >> 2));
        adj_resid_at(op, lam, b, D, q, r[0], r[1], r[2]);
    }
    double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int e = 0; e < 3; ++e) s[e] += __shfl(r[e], c, 8);
    if (act && ch == 0) {
        bc.a[t] = 0.125 * s[0];
        bc.b[t] = 0.125 * s[1];
        bc.c[t] = 0.125 * s[2];
        lamc.a[t] = 0.0;
        lamc.b[t] = 0.0;
        lamc.c[t] = 0.0;
    }
}

// Exact solve on the coarsest level (natural layout, P <= 64), one wavefront.
// minv caches (I - tau D Lap - tau/2 Lap^3)^{-1} while *valid is set.
__global__ __launch_bounds__(64) void k_adj_coarse(OpParams op, Tri<double> lam,
                                                   Tri<const double> b,
                                                   const double *__restrict__ D,
                                                   const double *__restrict__ lap1,
                                                   const double *__restrict__ lap3, double *minv,
                                                   int *valid) {
    __shared__ double A[64 * 64];
    __shared__ double vec[64];
    __shared__ int perm[64];
    const int n = op.lay.n, P = n * n * n;
    const int p = threadIdx.x;
    const bool act = p < P;
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
    auto lap_lds = [&](double own) -> double {
        return ((vec[nb[0]] + vec[nb[1]]) + (vec[nb[2]] + vec[nb[3]]) + (vec[nb[4]] + vec[nb[5]]) -
                6.0 * own) * op.h2inv;
    };
    const double d = act ? D[p] : 0.0;
    const double b1 = act ? b.a[p] : 0.0, b2 = act ? b.b[p] : 0.0, b3 = act ? b.c[p] : 0.0;
    if (!*valid) {
        if (act)
            for (int q = 0; q < P; ++q) {
                const int o = q * P + p;
                A[o] = (q == p ? 1.0 : 0.0) - op.tau * d * lap1[o] - 0.5 * op.tau * lap3[o];
            }
        __syncthreads();
        gj_invert(A, P, perm);
        if (act)
            for (int q = 0; q < P; ++q) minv[q * P + p] = A[q * P + p];
        __syncthreads();
    }
    // rhs = b1 + D b2 + 1/2 Lap(b3 + Lap b2)
    vec[p] = b2;
    __syncthreads();
    const double lb2 = act ? lap_lds(b2) : 0.0;
    __syncthreads();
    vec[p] = b3 + lb2;
    __syncthreads();
    const double rhs = b1 + d * b2 + 0.5 * (act ? lap_lds(b3 + lb2) : 0.0);
    __syncthreads();
    vec[p] = rhs;
    __syncthreads();
    double l1 = 0.0;
    if (act)
        for (int q = 0; q < P; ++q) l1 += minv[q * P + p] * vec[q];
    __syncthreads();
    vec[p] = l1;
    __syncthreads();
    const double l2 = b2 + op.tau * (act ? lap_lds(l1) : 0.0);
    __syncthreads();
    vec[p] = l2;
    __syncthreads();
    const double l3 = b3 + (act ? lap_lds(l2) : 0.0);
    if (act) {
        lam.a[p] = l1;
        lam.b[p] = l2;
        lam.c[p] = l3;
    }
    if (p == 0) *valid = 1;
}

__global__ __launch_bounds__(kBlock) void k_fill(double *p, size_t count, double v) {
    const size_t t = (size_t)xcd_block() * kBlock + threadIdx.x;
    if (t < count) p[t] = v;
}

// gbar_cur += lambda1 + (g_a + (1-eps)/2) lambda2 + 3 Lap lambda2 + Lap lambda3 / 2
// (natural layout; lam holds lambda in natural order).
__global__ __launch_bounds__(kBlock) void k_adj_accum_cur(OpParams nat, Tri<const double> lam,
                                                          const double *__restrict__ phin,
                                                          const double *__restrict__ phk,
                                                          double *__restrict__ gcur) {
    const Lay &L = nat.lay;
    const unsigned t = xcd_block() * kBlock + threadIdx.x;
    if (t >= (unsigned)npts(L)) return;
    int i, j, k;
    decode(L, t, i, j, k);
    const Off q = offs(L, i, j, k);
    const double l2 = lam.b[t], l3 = lam.c[t];
    const double L2 = (nsum(lam.b, q) - 6.0 * l2) * nat.h2inv;
    const double L3 = (nsum(lam.c, q) - 6.0 * l3) * nat.h2inv;
    const double x = phin[t], a = phk[t];
    const double ga = 0.25 * (x * x + 2.0 * x * a + 3.0 * a * a);
    gcur[t] += lam.a[t] + (ga + 0.5 * (1.0 - nat.eps)) * l2 + 3.0 * L2 + 0.5 * L3;
}

// gbar_prev -= Lap lambda2 (natural layout).
__global__ __launch_bounds__(kBlock) void k_adj_accum_prev(OpParams nat, const double *__restrict__ l2v,
                                                           double *__restrict__ gprev) {
    const Lay &L = nat.lay;
    const unsigned t = xcd_block() * kBlock + threadIdx.x;
    if (t >= (unsigned)npts(L)) return;
    int i, j, k;
    decode(L, t, i, j, k);
    const Off q = offs(L, i, j, k);
    gprev[t] -= (nsum(l2v, q) - 6.0 * l2v[t]) * nat.h2inv;
}

// Per-block sums of lambda2 (phi^{k+1} + phi^k); the final pass adds
// -1/2 of their fixed-order total into geps[0].
__global__ __launch_bounds__(kBlock) void k_adj_eps_part(size_t P, const double *__restrict__ l2v,
                                                         const double *__restrict__ phin,
                                                         const double *__restrict__ phk,
                                                         double *__restrict__ part) {
    __shared__ double red[kBlock];
    double s = 0.0;
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < P; t += (size_t)gridDim.x * kBlock)
        s += l2v[t] * (phin[t] + phk[t]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_adj_eps_final(const double *__restrict__ part, int count,
                                                          double *geps) {
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int b = threadIdx.x; b < count; b += kBlock) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) geps[0] += -0.5 * red[0];
}

// ------------------------------------------------------------- driver

static void fill(hipStream_t s, double *p, size_t count, double v) {
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(count)), dim3(kBlock), 0, s, p, count, v);
}

static void adj_sweep(pfc_handle *H, int l) {
    Level &A = H->lev[l];
    const OpParams op = op_of(H, l);
    for (int colour = 0; colour < 2; ++colour)
        hipLaunchKernelGGL(k_adj_smooth, dim3(blocks_for(A.P / 2)), dim3(kBlock), 0, H->stream, op,
                           colour, A.u, cst(A.f), (const double *)A.phk);
}

static void adj_cycle(pfc_handle *H, int l, bool fcycle) {
    Level &A = H->lev[l];
    if (l == H->nlev - 1) {
        hipLaunchKernelGGL(k_adj_coarse, dim3(1), dim3(64), 0, H->stream, op_of(H, l), A.u, cst(A.f),
                           (const double *)A.phk, (const double *)H->lap1,
                           (const double *)H->lap3, H->minv_adj, H->valid_adj);
        return;
    }
    Level &B = H->lev[l + 1];
    for (int s = 0; s < H->cfg.nu1; ++s) adj_sweep(H, l);
    hipLaunchKernelGGL(k_adj_resid_restrict, dim3(blocks_for(8 * B.P)), dim3(kBlock), 0, H->stream,
                       op_of(H, l), B.lay, cst(A.u), cst(A.f), (const double *)A.phk, B.f, B.u);
    adj_cycle(H, l + 1, fcycle);
    if (fcycle) adj_cycle(H, l + 1, false);
    launch_prolong<double>(H->stream, B.lay, A.lay, cst(B.u),
                           Tri<const double>{nullptr, nullptr, nullptr}, A.u, nullptr, false,
                           A.pz[0]);
    for (int s = 0; s < H->cfg.nu2; ++s) adj_sweep(H, l);
}

static pfc_status adj_norm(pfc_handle *H, double *out) {
    Level &A = H->lev[0];
    const unsigned blocks = reduce_blocks(A.P);
    hipLaunchKernelGGL(k_adj_resid_max, dim3(blocks), dim3(kBlock), 0, H->stream, op_of(H, 0),
                       cst(A.u), cst(A.f), (const double *)A.phk, H->partial);
    return read_norm(H, (int)blocks, out);
}

pfc_status adjoint_step(pfc_handle *H, const double *phi_prev, const double *phi_cur,
                        const double *phi_next, const double *gbar_next, double *gbar_cur,
                        double *gbar_prev, double *geps, double adj_tol, int32_t *cycles) {
    (void)phi_prev;  // the step's Jacobian does not depend on phi^{k-1}
    Level &A = H->lev[0];
    const size_t P = A.P;
    const Lay nat = make_lay(A.n, false);
    // D on every level (stored in the phi^k slots of the hierarchy)
    hipLaunchKernelGGL(k_adj_D, dim3(blocks_for(P)), dim3(kBlock), 0, H->stream, A.lay, H->cfg.eps,
                       phi_next, phi_cur, A.phk);
    restrict_phk(H);
    // b = (gbar_next, 0, 0), lambda = 0
    launch_to_lay<double, double>(H->stream, A.lay, gbar_next, A.f.a, 1);
    fill(H->stream, A.f.b, 2 * P, 0.0);
    fill(H->stream, A.u.a, 3 * P, 0.0);
    (void)hipMemsetAsync(H->valid_adj, 0, sizeof(int), H->stream);
    HIP_TRY(H, hipGetLastError());
    double bnorm = 0.0, rho = 0.0;
    pfc_status st = adj_norm(H, &bnorm);
    if (st != PFC_OK) return st;
    if (!std::isfinite(bnorm)) return fail(H, PFC_ERR_NONFINITE, "gbar_next is not finite");
    int c = 0;
    pfc_status status = PFC_OK;
    rho = bnorm;
    while (bnorm > 0.0 && rho > adj_tol * bnorm) {
        if (c == H->cfg.max_cycles) {
            status = PFC_ERR_NOT_CONVERGED;
            break;
        }
        adj_cycle(H, 0, H->cfg.cycle == PFC_CYCLE_F);
        ++c;
        st = adj_norm(H, &rho);
        if (st != PFC_OK) return st;
        if (!std::isfinite(rho)) {
            status = PFC_ERR_NONFINITE;
            break;
        }
    }
    if (status == PFC_OK || status == PFC_ERR_NOT_CONVERGED) {
        // lambda back to natural order (level-0 scratch), then accumulate
        launch_from_lay<double, double>(H->stream, A.lay, A.u.a, A.ubar.a, 3);
        OpParams op = op_of(H, 0);
        op.lay = nat;
        const Tri<const double> lam{A.ubar.a, A.ubar.b, A.ubar.c};
        hipLaunchKernelGGL(k_adj_accum_cur, dim3(blocks_for(P)), dim3(kBlock), 0, H->stream, op, lam,
                           phi_next, phi_cur, gbar_cur);
        hipLaunchKernelGGL(k_adj_accum_prev, dim3(blocks_for(P)), dim3(kBlock), 0, H->stream, op,
                           (const double *)A.ubar.b, gbar_prev);
        const unsigned eb = reduce_blocks(P);
        hipLaunchKernelGGL(k_adj_eps_part, dim3(eb), dim3(kBlock), 0, H->stream, P,
                           (const double *)A.ubar.b, phi_next, phi_cur, H->energy_part);
        hipLaunchKernelGGL(k_adj_eps_final, dim3(1), dim3(kBlock), 0, H->stream,
                           (const double *)H->energy_part, (int)eb, geps);
    }
    HIP_TRY(H, hipGetLastError());
    HIP_TRY(H, hipStreamSynchronize(H->stream));
    if (cycles) *cycles = c;
    if (status != PFC_OK) return fail(H, status, pfc_status_string(status));
    return PFC_OK;
}

}  // namespace pfc

extern "C" pfc_status pfc_adjoint_step(pfc_handle *h, const double *phi_prev, const double *phi_cur,
                                       const double *phi_next, const double *gbar_next,
                                       double *gbar_cur, double *gbar_prev, double *geps,
                                       double adj_tol, int32_t *cycles) {
    if (!h) return PFC_ERR_INVALID_ARG;
    if (!phi_prev || !phi_cur || !phi_next || !gbar_next || !gbar_cur || !gbar_prev || !geps)
        return pfc::fail(h, PFC_ERR_INVALID_ARG, "NULL pointer");
    if (!(adj_tol > 0.0) || !std::isfinite(adj_tol))
        return pfc::fail(h, PFC_ERR_INVALID_ARG, "adj_tol must be > 0");
    if (h->cfg.mobility != PFC_MOBILITY_ONE)
        return pfc::fail(h, PFC_ERR_INVALID_ARG, "the adjoint is derived for constant mobility");
    if (h->cfg.scheme != PFC_SCHEME_CS2)
        return pfc::fail(h, PFC_ERR_INVALID_ARG, "the adjoint is derived for scheme (1.10)");
    if (gbar_next == gbar_cur || gbar_next == gbar_prev)
        return pfc::fail(h, PFC_ERR_INVALID_ARG, "gbar_next aliases an output");
    return pfc::adjoint_step(h, phi_prev, phi_cur, phi_next, gbar_next, gbar_cur, gbar_prev, geps,
                             adj_tol, cycles);
}
