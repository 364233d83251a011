// Pointwise relaxation shared by the smoother kernels (smooth.hip) and the
// batched form (kernels.hip): the 3x3 solve at one point and the half-sweep
// update of one point in colour-split storage.
#pragma once

#include "device_common.h"

namespace pfc {

// ------------------------------------------------------------- smoothing
//
// Pointwise solve of the three equations of N(u) = f at one point with the
// six neighbours held (Section 5 smoothing scheme, M = 1):
//     phi + A mu             = r1     A = 6 tau/h^2, r1 = f1 + tau S_mu/h^2
//    -c phi + mu + B omega   = r2     B = 6/h^2,     r2 = f2 + S_om/h^2 + (lin.)
//     Dd phi + omega         = r3     Dd = 3/h^2,    r3 = f3 + S_phi/(2h^2)
// (first-order scheme: Dd = 6/h^2, r3 = f3 + S_phi/h^2).
// c is the linearised slope of the cubic term; eliminating omega and mu gives
// phi = (r1 - A r2 + A B r3) / (1 + A (c + B Dd)).
// One thread per point of colour `colour` (colour-split storage only).
template <bool DELTA>
__device__ __forceinline__ void point_solve(const OpParams &op, int picard, double phin, double a,
                                            double b, double f1, double f2, double f3, double smu,
                                            double som, double sphi, double &phi, double &mu,
                                            double &om) {
    const double h2inv = op.h2inv, tau = op.tau, lin_c = lin_of(op);
    double c, r2;
    if (!DELTA && picard) {  // second order: 1/4(phin^2 + a^2) phi; first order: phin^2 phi
        const double qq = op.fo ? phin * phin : 0.25 * (phin * phin + a * a);
        c = qq + lin_c;
        r2 = f2 + som * h2inv + (op.fo ? 0.0 : qq * a);
    } else {
        const double gp = dg_of<DELTA>(op.fo, phin, a, b);
        c = gp + lin_c;
        r2 = f2 + som * h2inv + (g_of<DELTA>(op.fo, phin, a, b) - gp * phin);
    }
    const double r1 = f1 + tau * smu * h2inv;
    const double r3 = f3 + w3_of(op) * sphi * h2inv;
    const double A = 6.0 * tau * h2inv, B = 6.0 * h2inv, Dd = (op.fo ? 6.0 : 3.0) * h2inv;
    phi = (r1 - A * r2 + A * B * r3) / (1.0 + A * (c + B * Dd));
    om = r3 - Dd * phi;
    mu = r2 + c * phi - B * om;
}

// Pointwise solve with variable mobility: the first equation becomes
// phi + A mu = r1 with A = tau msum / h^2 and r1 = f1 + tau smu / h^2, msum the
// sum of the six face mobilities, smu the sum of M_face mu_nbr.
__device__ __forceinline__ void point_solve_mob(const OpParams &op, int picard, double phin,
                                                double a, double f1, double f2, double f3,
                                                double msum, double smu, double som, double sphi,
                                                double &phi, double &mu, double &om) {
    const double h2inv = op.h2inv, tau = op.tau, lin_c = 0.5 * (1.0 - op.eps);
    double c, r2;
    if (picard) {
        const double qq = 0.25 * (phin * phin + a * a);
        c = qq + lin_c;
        r2 = f2 + som * h2inv + qq * a;
    } else {
        const double gp = Cubic<false>::dg(phin, a, 0.0);
        c = gp + lin_c;
        r2 = f2 + som * h2inv + (Cubic<false>::g(phin, a, 0.0) - gp * phin);
    }
    const double r1 = f1 + tau * smu * h2inv;
    const double r3 = f3 + 0.5 * sphi * h2inv;
    const double A = msum * tau * h2inv, B = 6.0 * h2inv, Dd = 3.0 * h2inv;
    phi = (r1 - A * r2 + A * B * r3) / (1.0 + A * (c + B * Dd));
    om = r3 - Dd * phi;
    mu = r2 + c * phi - B * om;
}

// PK1: f.a is phi^k itself (one buffer), loaded once.
// TAU (the first sweep on a coarse level): the point's right-hand side first
// takes the tau correction, f + N(I u) with I u = uo, written back through
// fw, and the old values come from uo since the level's iterate u has not been
// started at I u: colour 0 reads every neighbour and its own value there,
// colour 1 its own value and, for N(I u), its old colour-0 neighbours, while
// its solve takes the new colour-0 neighbours from u.  Same arithmetic and
// order as the tau kernel (copying I u into u) followed by two plain
// half-sweeps, so the results agree bit for bit.  TCOL: the colour as a
// compile-time constant (TAU only), so that all of a point's loads are issued
// in one block.
template <typename T, bool DELTA, bool MOB = false, bool PK1 = false, bool TAU = false,
          int TCOL = -1>
__device__ __forceinline__ void smooth_body(const OpParams &op, int colour, int picard, Tri<T> u,
                                            Tri<const T> f, const T *__restrict__ phk,
                                            const T *__restrict__ base, unsigned t,
                                            Tri<const T> uo = Tri<const T>{nullptr, nullptr, nullptr},
                                            Tri<T> fw = Tri<T>{nullptr, nullptr, nullptr}) {
    const Lay &L = op.lay;
    const int n = L.n, hn = n >> 1;
    const unsigned H = (unsigned)((size_t)n * n * n / 2);
    if (t >= H) return;
    const unsigned row = L.dh.q(t);
    const int m = (int)(t - row * (unsigned)hn);
    const int k = (int)L.dn.q(row);
    const int j = (int)(row - (unsigned)k * (unsigned)n);
    const int p = (colour + j + k) & 1;  // x parity of this point
    // other colour: same row for x-neighbours, same m for y/z neighbours
    const size_t oc = (size_t)(colour ^ 1) * H;
    const size_t own = (size_t)colour * H + t;
    const size_t rbase = oc + (size_t)row * hn;
    const size_t xm = rbase + (p ? m : (m == 0 ? hn - 1 : m - 1));
    const size_t xp = rbase + (p ? (m == hn - 1 ? 0 : m + 1) : m);
    const size_t ym = oc + ((size_t)k * n + wrap_m(j, n)) * hn + m;
    const size_t yp = oc + ((size_t)k * n + wrap_p(j, n)) * hn + m;
    const size_t zm = oc + ((size_t)wrap_m(k, n) * n + j) * hn + m;
    const size_t zp = oc + ((size_t)wrap_p(k, n) * n + j) * hn + m;

    if constexpr (TAU) {
        static_assert(!PK1 && (TCOL == 0 || TCOL == 1), "coarse levels, colour fixed");
        constexpr bool c0 = TCOL == 0;
        // own old values, phi^k, base and right-hand side, loaded ahead
        const double p0 = (double)uo.a[own], m0 = (double)uo.b[own], w0 = (double)uo.c[own];
        const double ak = (double)phk[own], bb = DELTA ? (double)base[own] : 0.0;
        const double f0 = (double)f.a[own], f1 = (double)f.b[own], f2 = (double)f.c[own];
        // the solve's neighbours: old ones (uo) for colour 0, new colour 0 (u) for colour 1
        const T *na = c0 ? uo.a : u.a, *nb = c0 ? uo.b : u.b, *nc = c0 ? uo.c : u.c;
        const double smu = ((double)nb[xp] + (double)nb[xm]) + ((double)nb[yp] + (double)nb[ym]) +
                           ((double)nb[zp] + (double)nb[zm]);
        const double som = ((double)nc[xp] + (double)nc[xm]) + ((double)nc[yp] + (double)nc[ym]) +
                           ((double)nc[zp] + (double)nc[zm]);
        const double sphi = ((double)na[xp] + (double)na[xm]) + ((double)na[yp] + (double)na[ym]) +
                            ((double)na[zp] + (double)na[zm]);
        // neighbour sums of I u for N(I u): the same values for colour 0
        double tmu = smu, tom = som, tphi = sphi;
        if constexpr (!c0) {
            tmu = ((double)uo.b[xp] + (double)uo.b[xm]) + ((double)uo.b[yp] + (double)uo.b[ym]) +
                  ((double)uo.b[zp] + (double)uo.b[zm]);
            tom = ((double)uo.c[xp] + (double)uo.c[xm]) + ((double)uo.c[yp] + (double)uo.c[ym]) +
                  ((double)uo.c[zp] + (double)uo.c[zm]);
            tphi = ((double)uo.a[xp] + (double)uo.a[xm]) + ((double)uo.a[yp] + (double)uo.a[ym]) +
                   ((double)uo.a[zp] + (double)uo.a[zm]);
        }
        double ls[3] = {(tphi - 6.0 * p0) * op.h2inv, 0.0, (tom - 6.0 * w0) * op.h2inv};
        const size_t nb6[6] = {xp, xm, yp, ym, zp, zm};
        if constexpr (MOB) {  // flux sums of the tau term (old mu) and of the solve (nb)
            const double *ps = op.mob.phs;
            const double pc = ps[own];
            double sm = 0.0;
#pragma unroll
            for (int q = 0; q < 6; ++q)
                sm += face_mob(op.mob, pc, ps[nb6[q]]) * ((double)uo.b[nb6[q]] - m0);
            ls[1] = sm * op.h2inv;
        } else {
            ls[1] = (tmu - 6.0 * m0) * op.h2inv;
        }
        double nv[3];
        n_of_point<DELTA>(op, ls, p0, m0, w0, ak, bb, nv);
        const T fa = (T)(f0 + nv[0]);
        const T fb = (T)(f1 + nv[1]);
        const T fc = (T)(f2 + nv[2]);
        double phi, mu, om;
        if constexpr (MOB) {
            const double *ps = op.mob.phs;
            const double pc = ps[own];
            double msum = 0.0, smm = 0.0;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const double mf = face_mob(op.mob, pc, ps[nb6[q]]);
                msum += mf;
                smm += mf * (double)nb[nb6[q]];
            }
            point_solve_mob(op, picard, p0, ak, (double)fa, (double)fb, (double)fc, msum, smm, som,
                            sphi, phi, mu, om);
        } else {
            point_solve<DELTA>(op, picard, p0, ak, bb, (double)fa, (double)fb, (double)fc, smu, som,
                               sphi, phi, mu, om);
        }
        fw.a[own] = fa;  // stores after every load
        fw.b[own] = fb;
        fw.c[own] = fc;
        u.a[own] = (T)phi;
        u.b[own] = (T)mu;
        u.c[own] = (T)om;
        return;
    }

    const double smu = ((double)u.b[xp] + (double)u.b[xm]) + ((double)u.b[yp] + (double)u.b[ym]) +
                       ((double)u.b[zp] + (double)u.b[zm]);
    const double som = ((double)u.c[xp] + (double)u.c[xm]) + ((double)u.c[yp] + (double)u.c[ym]) +
                       ((double)u.c[zp] + (double)u.c[zm]);
    const double sphi = ((double)u.a[xp] + (double)u.a[xm]) + ((double)u.a[yp] + (double)u.a[ym]) +
                        ((double)u.a[zp] + (double)u.a[zm]);
    double phi, mu, om;
    if constexpr (MOB) {  // flux form of the first equation (FP64 only)
        const double *ps = op.mob.phs;
        const double pc = ps[own];
        const size_t nb6[6] = {xp, xm, yp, ym, zp, zm};
        double msum = 0.0, smm = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const double mf = face_mob(op.mob, pc, ps[nb6[q]]);
            msum += mf;
            smm += mf * (double)u.b[nb6[q]];
        }
        point_solve_mob(op, picard, (double)u.a[own], (double)phk[own],
                        PK1 ? (double)phk[own] : (double)f.a[own], (double)f.b[own],
                        (double)f.c[own], msum, smm, som, sphi, phi, mu, om);
    } else {
        point_solve<DELTA>(op, picard, (double)u.a[own], (double)phk[own],
                           DELTA ? (double)base[own] : 0.0,
                           PK1 ? (double)phk[own] : (double)f.a[own], (double)f.b[own],
                           (double)f.c[own], smu, som, sphi, phi, mu, om);
    }
    u.a[own] = (T)phi;
    u.b[own] = (T)mu;
    u.c[own] = (T)om;
}

}  // namespace pfc
