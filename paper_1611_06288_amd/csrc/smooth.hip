// Smoother kernels: the red-black half-sweep (one colour per launch) and the
// fused one-pass full sweep used on large FP64 levels (Section 5 smoothing
// scheme, red-black order; arXiv:1611.06288).
#include "smooth.h"

#include <algorithm>
#include <numeric>

namespace pfc {

template <typename T, bool DELTA, bool MOB, bool PK1 = false>
__global__ __launch_bounds__(kBlock) void k_smooth(OpParams op, int colour, int picard, Tri<T> u,
                                                   Tri<const T> f, const T *__restrict__ phk,
                                                   const T *__restrict__ base) {
    if (gate_closed(op.gate)) return;
    smooth_body<T, DELTA, MOB, PK1>(op, colour, picard, u, f, phk, base,
                                    xcd_block() * kBlock + threadIdx.x);
}

template <typename T, bool DELTA>
void launch_smooth(hipStream_t s, const OpParams &op, int colour, int picard, Tri<T> u,
                   Tri<const T> f, const T *phk, const T *base) {
    const size_t H = npts_host(op.lay) / 2;
    if constexpr (!DELTA) {
        if (op.mob.phs) {  // variable mobility
            if (f.a == phk)
                hipLaunchKernelGGL((k_smooth<T, false, true, true>), dim3(blocks_for(H)), dim3(kBlock),
                                   0, s, op, colour, picard, u, f, phk, base);
            else
                hipLaunchKernelGGL((k_smooth<T, false, true>), dim3(blocks_for(H)), dim3(kBlock), 0,
                                   s, op, colour, picard, u, f, phk, base);
            return;
        }
        if (f.a == phk) {  // the first source component is phi^k itself: load it once
            hipLaunchKernelGGL((k_smooth<T, false, false, true>), dim3(blocks_for(H)), dim3(kBlock),
                               0, s, op, colour, picard, u, f, phk, base);
            return;
        }
    }
    hipLaunchKernelGGL((k_smooth<T, DELTA, false>), dim3(blocks_for(H)), dim3(kBlock), 0, s, op,
                       colour, picard, u, f, phk, base);
}

// One half-sweep of the first sweep on a coarse level, forming the tau
// correction as it goes (smooth_body, TAU): f += N(I u) at the colour's
// points, the old values read from ubar = I u.
template <typename T, bool DELTA, bool MOB, int COL>
__global__ __launch_bounds__(kBlock) void k_smooth_tau(OpParams op, int picard, Tri<T> u, Tri<T> f,
                                                       Tri<const T> ubar,
                                                       const T *__restrict__ phk,
                                                       const T *__restrict__ base) {
    if (gate_closed(op.gate)) return;
    smooth_body<T, DELTA, MOB, false, true, COL>(op, COL, picard, u,
                                                 Tri<const T>{f.a, f.b, f.c}, phk, base,
                                                 xcd_block() * kBlock + threadIdx.x, ubar, f);
}

template <typename T, bool DELTA>
void launch_smooth_tau(hipStream_t s, const OpParams &op, int colour, int picard, Tri<T> u,
                       Tri<T> f, Tri<const T> ubar, const T *phk, const T *base) {
    const size_t H = npts_host(op.lay) / 2;
    const dim3 grid(blocks_for(H)), block(kBlock);
    if constexpr (!DELTA) {
        if (op.mob.phs) {
            if (colour == 0)
                hipLaunchKernelGGL((k_smooth_tau<T, false, true, 0>), grid, block, 0, s, op, picard,
                                   u, f, ubar, phk, base);
            else
                hipLaunchKernelGGL((k_smooth_tau<T, false, true, 1>), grid, block, 0, s, op, picard,
                                   u, f, ubar, phk, base);
            return;
        }
    }
    if (colour == 0)
        hipLaunchKernelGGL((k_smooth_tau<T, DELTA, false, 0>), grid, block, 0, s, op, picard, u, f,
                           ubar, phk, base);
    else
        hipLaunchKernelGGL((k_smooth_tau<T, DELTA, false, 1>), grid, block, 0, s, op, picard, u, f,
                           ubar, phk, base);
}

template void launch_smooth_tau<double, false>(hipStream_t, const OpParams &, int, int,
                                               Tri<double>, Tri<double>, Tri<const double>,
                                               const double *, const double *);
template void launch_smooth_tau<float, true>(hipStream_t, const OpParams &, int, int, Tri<float>,
                                             Tri<float>, Tri<const float>, const float *,
                                             const float *);

// ------------------------------------------------ small-level full sweep
//
// Levels of at most kSmallSweepN^3 points: one workgroup runs both colours,
// the barrier between them standing in for a second launch (the launches of
// such levels cost more than their work).  Same per-point body and order as
// two launch_smooth calls, so the result is the same bit for bit.
constexpr int kSmallSweepThreads = 1024;

template <typename T, bool DELTA, bool MOB>
__global__ __launch_bounds__(kSmallSweepThreads) void k_sweep_small(OpParams op, int picard, Tri<T> u,
                                                                    Tri<const T> f,
                                                                    const T *__restrict__ phk,
                                                                    const T *__restrict__ base) {
    if (gate_closed(op.gate)) return;
    const unsigned H = (unsigned)(npts(op.lay) / 2);
    for (int colour = 0; colour < 2; ++colour) {
        for (unsigned t = threadIdx.x; t < H; t += blockDim.x)
            smooth_body<T, DELTA, MOB>(op, colour, picard, u, f, phk, base, t);
        __syncthreads();
    }
}

template <typename T, bool DELTA>
void launch_sweep_small(hipStream_t s, const OpParams &op, int picard, Tri<T> u, Tri<const T> f,
                        const T *phk, const T *base) {
    const size_t H = npts_host(op.lay) / 2;
    const unsigned threads =
        (unsigned)std::min<size_t>(kSmallSweepThreads, (H + 63) / 64 * 64);
    if constexpr (!DELTA) {
        if (op.mob.phs) {
            hipLaunchKernelGGL((k_sweep_small<T, false, true>), dim3(1), dim3(threads), 0, s, op,
                               picard, u, f, phk, base);
            return;
        }
    }
    hipLaunchKernelGGL((k_sweep_small<T, DELTA, false>), dim3(1), dim3(threads), 0, s, op, picard, u,
                       f, phk, base);
}

template void launch_sweep_small<double, false>(hipStream_t, const OpParams &, int, Tri<double>,
                                                Tri<const double>, const double *, const double *);
template void launch_sweep_small<float, true>(hipStream_t, const OpParams &, int, Tri<float>,
                                              Tri<const float>, const float *, const float *);

// The same, as the first sweep of a coarse level forming the tau correction
// (smooth_body, TAU).
template <typename T, bool DELTA, bool MOB>
__global__ __launch_bounds__(kSmallSweepThreads) void k_sweep_small_tau(
    OpParams op, int picard, Tri<T> u, Tri<T> f, Tri<const T> ubar, const T *__restrict__ phk,
    const T *__restrict__ base) {
    if (gate_closed(op.gate)) return;
    const unsigned H = (unsigned)(npts(op.lay) / 2);
    const Tri<const T> fc{f.a, f.b, f.c};
    for (unsigned t = threadIdx.x; t < H; t += blockDim.x)
        smooth_body<T, DELTA, MOB, false, true, 0>(op, 0, picard, u, fc, phk, base, t, ubar, f);
    __syncthreads();
    for (unsigned t = threadIdx.x; t < H; t += blockDim.x)
        smooth_body<T, DELTA, MOB, false, true, 1>(op, 1, picard, u, fc, phk, base, t, ubar, f);
    __syncthreads();
}

template <typename T, bool DELTA>
void launch_sweep_small_tau(hipStream_t s, const OpParams &op, int picard, Tri<T> u, Tri<T> f,
                            Tri<const T> ubar, const T *phk, const T *base) {
    const size_t H = npts_host(op.lay) / 2;
    const unsigned threads =
        (unsigned)std::min<size_t>(kSmallSweepThreads, (H + 63) / 64 * 64);
    if constexpr (!DELTA) {
        if (op.mob.phs) {
            hipLaunchKernelGGL((k_sweep_small_tau<T, false, true>), dim3(1), dim3(threads), 0, s, op,
                               picard, u, f, ubar, phk, base);
            return;
        }
    }
    hipLaunchKernelGGL((k_sweep_small_tau<T, DELTA, false>), dim3(1), dim3(threads), 0, s, op,
                       picard, u, f, ubar, phk, base);
}

template void launch_sweep_small_tau<double, false>(hipStream_t, const OpParams &, int,
                                                    Tri<double>, Tri<double>, Tri<const double>,
                                                    const double *, const double *);
template void launch_sweep_small_tau<float, true>(hipStream_t, const OpParams &, int, Tri<float>,
                                                  Tri<float>, Tri<const float>, const float *,
                                                  const float *);

// ------------------------------------------------- fused red-black sweep
//
// One full red-black sweep in one pass, from u_in to u_out (two buffers;
// colour-split storage).  A workgroup owns an x-y column of kFX x kFY points
// and a range [z0, z1) of planes, and walks it in z.  At step k it
//   * computes the new colour-0 values of plane k on its box plus a one-cell
//     ring in x and y (the ring cells, and the planes z0-1 and z1, belong to
//     other workgroups, which compute the same values; they are not written)
//     into a 3-plane LDS ring, reading the old colour-1 neighbours from a
//     second 3-plane LDS ring (box plus a two-cell ring) that holds every
//     old colour-1 value of the column exactly once;
//   * computes the new colour-1 values of plane k-1 on its box, whose six
//     colour-0 neighbours are all in the first ring.
// The old colour-1 plane k+2 and the own-point inputs of the next step are
// loaded into registers while step k computes, so each thread keeps its
// next loads in flight across both barriers.
// Each point sees the neighbour values of the two half-sweeps (old colour 1
// for colour 0, new colour 0 for colour 1) and the same arithmetic, so, with
// floating-point contraction off, the result is bitwise that of two
// launch_smooth calls, while each field is read and written once.
// MOB (variable mobility): phi* rides along as a fourth field of both rings
// (read-only), and the mu-sum becomes the face-mobility sum of the flux form
// in the half-sweep's neighbour order.
// NRM (M = 1, FP64) carries half of the cycle loop's stop test, max |S - N(u)|
// over the level, as per-workgroup maxima in part[blockIdx.x]:
//   NRM = 1: over the colour-0 points of the sweep's INPUT (their neighbour sums
//            are the colour-0 phase's own; old mu and omega of the box's
//            colour-0 points are read in addition, 8 B per point),
//   NRM = 2: over the colour-1 points of the sweep's OUTPUT (neighbour sums of
//            the colour-1 phase, the point's new values).
// The neighbour sums are taken in the residual kernels' order and the
// residual is formed by the same function, so the two halves together give
// bitwise the norm of the residual kernels.
// skip0: the new mu and omega of colour-0 points are not written (the next
// operation on this iterate is another fused sweep, which reads only phi of
// a colour-0 point; the colour-1 phase takes them from LDS).
constexpr int kFX = 64, kFY = 8, kFT = 256;  // column extents, threads per workgroup
constexpr int kFSl = kFX / 2 + 1;            // colour-0 ring: points per row
constexpr int kFRw = kFY + 2;                //                rows
constexpr int kFCs = kFX / 2 + 2;            // colour-1 ring: points per row
constexpr int kFCr = kFY + 4;                //                rows
constexpr int kFNr = kFSl * kFRw, kFNb = (kFX / 2) * kFY, kFNc = kFCs * kFCr;
constexpr int kFIr = (kFNr + kFT - 1) / kFT, kFIb = (kFNb + kFT - 1) / kFT,
              kFIc = (kFNc + kFT - 1) / kFT;  // items per thread in each phase

template <typename T, bool DELTA, bool MOB, int NRM, bool PK1>
__global__ __launch_bounds__(kFT) void k_sweep_fused(
    OpParams op, int picard, int nz, const T *__restrict__ ua, const T *__restrict__ ub,
    const T *__restrict__ uc, T *__restrict__ oa, T *__restrict__ ob, T *__restrict__ oc,
    const T *__restrict__ fa, const T *__restrict__ fb, const T *__restrict__ fc,
    const T *__restrict__ phk, const T *__restrict__ base, unsigned long long *__restrict__ part,
    int skip0) {
    static_assert(NRM == 0 || !DELTA, "stop-test halves: FP64 sweeps");
    constexpr int NF = MOB ? 4 : 3;         // ring fields: phi, mu, omega (, phi*)
    __shared__ T c1[NF][3][kFCr][kFCs];   // [field][plane slot][row][point] old colour 1
    __shared__ T red[NF][3][kFRw][kFSl];  // [field][plane slot][row][point] new colour 0
    __shared__ unsigned long long wmax[kFT / 64];  // NRM: per-wave maxima
    if (gate_closed(op.gate)) return;
    const double *__restrict__ ps = op.mob.phs;
    const int n = op.lay.n, hn = n >> 1;
    const unsigned un = (unsigned)n, uhn = (unsigned)hn, H = un * un * uhn;
    const int nbx = n / kFX, nby = n / kFY;
    const int b = (int)xcd_block();
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int x0 = bx * kFX, y0 = by * kFY;
    const int z0 = bz * n / nz, z1 = (bz + 1) * n / nz;
    const int tid = threadIdx.x;
    // one-step periodic wraps (every coordinate below is within one period)
    auto wn = [n](int v) { return v < 0 ? v + n : (v >= n ? v - n : v); };
    auto wh = [hn](int v) { return v < 0 ? v + hn : (v >= hn ? v - hn : v); };
    auto cslot = [z0](int p) { return (p - z0 + 3) % 3; };  // colour-1 ring slot of plane p
    auto rslot = [z0](int p) { return (p - z0 + 1) % 3; };  // colour-0 ring slot of plane p

    // old colour-1 values of one plane (box plus two-cell ring), in registers
    T cn[kFIc][NF];
    auto load_c1 = [&](int p) {
        const unsigned pw = (unsigned)wn(p);
#pragma unroll
        for (int i = 0; i < kFIc; ++i) {
            const int c = tid + i * kFT;
            if (c < kFNc) {
                const int cr = c / kFCs, cs = c - cr * kFCs;
                const unsigned g = H + (pw * un + (unsigned)wn(y0 - 2 + cr)) * uhn +
                                   (unsigned)wh(x0 / 2 - 1 + cs);
                cn[i][0] = ua[g];
                cn[i][1] = ub[g];
                cn[i][2] = uc[g];
                if constexpr (MOB) cn[i][3] = ps[g];
            }
        }
    };
    auto store_c1 = [&](int p) {
        const int s = cslot(p);
#pragma unroll
        for (int i = 0; i < kFIc; ++i) {
            const int c = tid + i * kFT;
            if (c < kFNc) {
                const int cr = c / kFCs, cs = c - cr * kFCs;
                c1[0][s][cr][cs] = cn[i][0];
                c1[1][s][cr][cs] = cn[i][1];
                c1[2][s][cr][cs] = cn[i][2];
                if constexpr (MOB) c1[3][s][cr][cs] = cn[i][3];
            }
        }
    };
    // own inputs of the colour-0 points of plane k (box plus ring)
    T ro[kFIr][MOB ? 7 : 6];
    unsigned rg[kFIr];
    T rmo[kFIr][2];  // NRM = 1: old mu, omega of the box's colour-0 points
    auto in_box = [&](int x, int y, int k) {
        return x >= x0 && x < x0 + kFX && y >= y0 && y < y0 + kFY && k >= z0 && k < z1;
    };
    auto load_red = [&](int k) {
        const unsigned kw = (unsigned)wn(k);
#pragma unroll
        for (int i = 0; i < kFIr; ++i) {
            const int q = tid + i * kFT;
            if (q < kFNr) {
                const int r = q / kFSl, sl = q - r * kFSl;
                const int y = y0 - 1 + r;
                const int x = x0 - 1 + ((x0 - 1 + y + k) & 1) + 2 * sl;
                const unsigned g = (kw * un + (unsigned)wn(y)) * uhn + (unsigned)(wn(x) >> 1);
                rg[i] = g;
                ro[i][0] = ua[g];
                ro[i][1] = phk[g];
                ro[i][2] = DELTA ? base[g] : (T)0;
                ro[i][3] = PK1 ? ro[i][1] : fa[g];
                ro[i][4] = fb[g];
                ro[i][5] = fc[g];
                if constexpr (MOB) ro[i][6] = ps[g];
                if constexpr (NRM == 1) {
                    if (in_box(x, y, k)) {
                        rmo[i][0] = ub[g];
                        rmo[i][1] = uc[g];
                    }
                }
            }
        }
    };
    // own inputs of the colour-1 points of plane kb (box); old phi comes from LDS
    T bo[kFIb][5];
    T bphi[kFIb];
    T bphs[kFIb];  // MOB: phi* of this step's colour-1 points
    auto load_black = [&](int kb) {
#pragma unroll
        for (int i = 0; i < kFIb; ++i) {
            const int q = tid + i * kFT;
            if (q < kFNb) {
                const int rb = q / (kFX / 2), s = q - rb * (kFX / 2);
                const int y = y0 + rb;
                const int x = x0 + ((x0 + y + kb + 1) & 1) + 2 * s;
                const unsigned g = H + ((unsigned)kb * un + (unsigned)y) * uhn + (unsigned)(x >> 1);
                bo[i][0] = phk[g];
                bo[i][1] = DELTA ? base[g] : (T)0;
                bo[i][2] = PK1 ? bo[i][0] : fa[g];
                bo[i][3] = fb[g];
                bo[i][4] = fc[g];
            }
        }
    };

    unsigned long long nrm = 0;  // NRM: this thread's max |r| bits
    const double h2inv = op.h2inv;
    load_c1(z0 - 2);
    store_c1(z0 - 2);
    load_c1(z0 - 1);
    store_c1(z0 - 1);
    load_c1(z0);
    load_red(z0 - 1);
    for (int k = z0 - 1; k <= z1; ++k) {
        const int kb = k - 1;  // plane of this step's colour-1 points
        store_c1(k + 1);       // its slot last held plane k-2, finished in the previous step
        if (kb >= z0) load_black(kb);
        __syncthreads();
        // colour 0, plane k
        const int sk = cslot(k), skm = cslot(k - 1), skp = cslot(k + 1), rq = rslot(k);
#pragma unroll
        for (int i = 0; i < kFIr; ++i) {
            const int q = tid + i * kFT;
            if (q < kFNr) {
                const int r = q / kFSl, sl = q - r * kFSl;
                const int y = y0 - 1 + r;
                const int x = x0 - 1 + ((x0 - 1 + y + k) & 1) + 2 * sl;
                // ring column of x and of its x-neighbours (colour-1 point m = x' >> 1)
                const int cx = (x - x0 + 2) >> 1, cxm = (x - x0 + 1) >> 1, cxp = (x - x0 + 3) >> 1;
                double s3[3];
#pragma unroll
                for (int fl = 0; fl < 3; ++fl)
                    s3[fl] = ((double)c1[fl][sk][r + 1][cxp] + (double)c1[fl][sk][r + 1][cxm]) +
                             ((double)c1[fl][sk][r + 2][cx] + (double)c1[fl][sk][r][cx]) +
                             ((double)c1[fl][skp][r + 1][cx] + (double)c1[fl][skm][r + 1][cx]);
                double phi, mu, om;
                if constexpr (MOB) {
                    const double pc = (double)ro[i][6];
                    double msum = 0.0, smm = 0.0;
                    auto face = [&](int sl3, int rr3, int cc3) {
                        const double mf = face_mob(op.mob, pc, (double)c1[3][sl3][rr3][cc3]);
                        msum += mf;
                        smm += mf * (double)c1[1][sl3][rr3][cc3];
                    };
                    face(sk, r + 1, cxp);
                    face(sk, r + 1, cxm);
                    face(sk, r + 2, cx);
                    face(sk, r, cx);
                    face(skp, r + 1, cx);
                    face(skm, r + 1, cx);
                    point_solve_mob(op, picard, (double)ro[i][0], (double)ro[i][1],
                                    (double)ro[i][3], (double)ro[i][4], (double)ro[i][5], msum,
                                    smm, s3[2], s3[0], phi, mu, om);
                    red[3][rq][r][sl] = ro[i][6];
                } else {
                    point_solve<DELTA>(op, picard, (double)ro[i][0], (double)ro[i][1],
                                       (double)ro[i][2], (double)ro[i][3], (double)ro[i][4],
                                       (double)ro[i][5], s3[1], s3[2], s3[0], phi, mu, om);
                }
                const T tphi = (T)phi, tmu = (T)mu, tom = (T)om;
                red[0][rq][r][sl] = tphi;
                red[1][rq][r][sl] = tmu;
                red[2][rq][r][sl] = tom;
                if (in_box(x, y, k)) {
                    oa[rg[i]] = tphi;
                    if (!skip0) {
                        ob[rg[i]] = tmu;
                        oc[rg[i]] = tom;
                    }
                    if constexpr (NRM == 1) {  // residual of the input at this point
                        const double p0 = (double)ro[i][0], m0 = (double)rmo[i][0],
                                     w0 = (double)rmo[i][1];
                        double ls[3] = {(s3[0] - 6.0 * p0) * h2inv, (s3[1] - 6.0 * m0) * h2inv,
                                        (s3[2] - 6.0 * w0) * h2inv};
                        if constexpr (MOB) {  // flux form, faces xp, xm, yp, ym, zp, zm
                            const double pc = (double)ro[i][6];
                            double sm6 = 0.0;
                            auto rface = [&](int sl3, int rr3, int cc3) {
                                sm6 += face_mob(op.mob, pc, (double)c1[3][sl3][rr3][cc3]) *
                                       ((double)c1[1][sl3][rr3][cc3] - m0);
                            };
                            rface(sk, r + 1, cxp);
                            rface(sk, r + 1, cxm);
                            rface(sk, r + 2, cx);
                            rface(sk, r, cx);
                            rface(skp, r + 1, cx);
                            rface(skm, r + 1, cx);
                            ls[1] = sm6 * h2inv;
                        }
                        double rr[3];
                        resid_from_lap<false>(op, ls, p0, m0, w0, (double)ro[i][3],
                                              (double)ro[i][4], (double)ro[i][5],
                                              (double)ro[i][1], 0.0, rr);
                        nrm = umax(nrm, umax(abs_bits(rr[0]), umax(abs_bits(rr[1]), abs_bits(rr[2]))));
                    }
                }
            }
        }
        // old phi of this step's colour-1 points, read before their slot is reused
        if (kb >= z0) {
            const int sb = cslot(kb);
#pragma unroll
            for (int i = 0; i < kFIb; ++i) {
                const int q = tid + i * kFT;
                if (q < kFNb) {
                    const int rb = q / (kFX / 2), s = q - rb * (kFX / 2);
                    const int x = x0 + ((x0 + y0 + rb + kb + 1) & 1) + 2 * s;
                    bphi[i] = c1[0][sb][rb + 2][(x - x0 + 2) >> 1];
                    if constexpr (MOB) bphs[i] = c1[3][sb][rb + 2][(x - x0 + 2) >> 1];
                }
            }
        }
        if (k + 2 <= z1 + 1) load_c1(k + 2);
        if (k + 1 <= z1) load_red(k + 1);
        __syncthreads();
        // colour 1, plane kb
        if (kb >= z0) {
            const int qm = rslot(kb - 1), q0 = rslot(kb), qp = rq;
#pragma unroll
            for (int i = 0; i < kFIb; ++i) {
                const int q = tid + i * kFT;
                if (q < kFNb) {
                    const int rb = q / (kFX / 2), s = q - rb * (kFX / 2);
                    const int y = y0 + rb;
                    const int x = x0 + ((x0 + y + kb + 1) & 1) + 2 * s;
                    const unsigned g =
                        H + ((unsigned)kb * un + (unsigned)y) * uhn + (unsigned)(x >> 1);
                    const int s0 = (x - x0 + 1) >> 1, sm = (x - x0) >> 1, sp = (x - x0 + 2) >> 1;
                    const int rr = rb + 1;
                    double s3[3];
#pragma unroll
                    for (int fl = 0; fl < 3; ++fl)
                        s3[fl] = ((double)red[fl][q0][rr][sp] + (double)red[fl][q0][rr][sm]) +
                                 ((double)red[fl][q0][rr + 1][s0] + (double)red[fl][q0][rr - 1][s0]) +
                                 ((double)red[fl][qp][rr][s0] + (double)red[fl][qm][rr][s0]);
                    double phi, mu, om;
                    if constexpr (MOB) {
                        const double pc = (double)bphs[i];
                        double msum = 0.0, smm = 0.0;
                        auto face = [&](int sl3, int rr3, int cc3) {
                            const double mf = face_mob(op.mob, pc, (double)red[3][sl3][rr3][cc3]);
                            msum += mf;
                            smm += mf * (double)red[1][sl3][rr3][cc3];
                        };
                        face(q0, rr, sp);
                        face(q0, rr, sm);
                        face(q0, rr + 1, s0);
                        face(q0, rr - 1, s0);
                        face(qp, rr, s0);
                        face(qm, rr, s0);
                        point_solve_mob(op, picard, (double)bphi[i], (double)bo[i][0],
                                        (double)bo[i][2], (double)bo[i][3], (double)bo[i][4],
                                        msum, smm, s3[2], s3[0], phi, mu, om);
                    } else {
                        point_solve<DELTA>(op, picard, (double)bphi[i], (double)bo[i][0],
                                           (double)bo[i][1], (double)bo[i][2], (double)bo[i][3],
                                           (double)bo[i][4], s3[1], s3[2], s3[0], phi, mu, om);
                    }
                    oa[g] = (T)phi;
                    ob[g] = (T)mu;
                    oc[g] = (T)om;
                    if constexpr (NRM == 2) {  // residual of the output at this point
                        double ls[3] = {(s3[0] - 6.0 * phi) * h2inv, (s3[1] - 6.0 * mu) * h2inv,
                                        (s3[2] - 6.0 * om) * h2inv};
                        if constexpr (MOB) {  // flux form, faces xp, xm, yp, ym, zp, zm
                            const double pc = (double)bphs[i];
                            double sm6 = 0.0;
                            auto rface = [&](int sl3, int rr3, int cc3) {
                                sm6 += face_mob(op.mob, pc, (double)red[3][sl3][rr3][cc3]) *
                                       ((double)red[1][sl3][rr3][cc3] - mu);
                            };
                            rface(q0, rr, sp);
                            rface(q0, rr, sm);
                            rface(q0, rr + 1, s0);
                            rface(q0, rr - 1, s0);
                            rface(qp, rr, s0);
                            rface(qm, rr, s0);
                            ls[1] = sm6 * h2inv;
                        }
                        double rr[3];
                        resid_from_lap<false>(op, ls, phi, mu, om, (double)bo[i][2],
                                              (double)bo[i][3], (double)bo[i][4],
                                              (double)bo[i][0], 0.0, rr);
                        nrm = umax(nrm, umax(abs_bits(rr[0]), umax(abs_bits(rr[1]), abs_bits(rr[2]))));
                    }
                }
            }
        }
    }
    if constexpr (NRM != 0) {
        nrm = block_max_u64_waves(nrm, wmax);
        if (threadIdx.x == 0) part[blockIdx.x] = nrm;
    }
}

bool fused_fits(int n) { return n % kFX == 0 && n % kFY == 0 && n >= kFusedMinN; }

int fused_slots(int device, bool mob) {
    int occ = 0, cus = 0;
    const void *fn = mob ? (const void *)k_sweep_fused<double, false, true, 0, true>
                         : (const void *)k_sweep_fused<double, false, false, 0, true>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kFT, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return occ * cus;
}

// z-split of a level: the smallest number of plane ranges for which the launch
// is a whole number of resident waves (slots workgroups each), with at least 4
// planes per range; a partly filled last wave costs as much as a full one.
int fused_nz(int n, int slots) {
    const int cols = (n / kFX) * (n / kFY);
    if (slots <= 0) return std::max(1, n / 16);
    int nz = slots / std::gcd(cols, slots);
    if (n / nz < 4) nz = std::max(1, n / 4);
    return nz;
}

int fused_blocks(int n, int nz) { return (n / kFX) * (n / kFY) * nz; }

template <typename T, bool DELTA, bool MOB, int NRM>
static void launch_fused_inst(hipStream_t s, const OpParams &op, int picard, int nz,
                              Tri<const T> uin, Tri<T> uout, Tri<const T> f, const T *phk,
                              const T *base, unsigned long long *part, int sk) {
    const unsigned blocks = (unsigned)fused_blocks(op.lay.n, nz);
    if (f.a == phk)  // the first source component is phi^k itself: load it once
        hipLaunchKernelGGL((k_sweep_fused<T, DELTA, MOB, NRM, true>), dim3(blocks), dim3(kFT), 0, s,
                           op, picard, nz, uin.a, uin.b, uin.c, uout.a, uout.b, uout.c, f.a, f.b,
                           f.c, phk, base, part, sk);
    else
        hipLaunchKernelGGL((k_sweep_fused<T, DELTA, MOB, NRM, false>), dim3(blocks), dim3(kFT), 0,
                           s, op, picard, nz, uin.a, uin.b, uin.c, uout.a, uout.b, uout.c, f.a,
                           f.b, f.c, phk, base, part, sk);
}

template <typename T, bool DELTA>
void launch_sweep_fused(hipStream_t s, const OpParams &op, int picard, int nz, Tri<const T> uin,
                        Tri<T> uout, Tri<const T> f, const T *phk, const T *base, int nrm,
                        unsigned long long *part, bool skip0) {
    const int sk = skip0 ? 1 : 0;
    if constexpr (!DELTA) {
        if (op.mob.phs) {  // variable mobility
            if (nrm == 1)
                launch_fused_inst<T, false, true, 1>(s, op, picard, nz, uin, uout, f, phk, base, part, sk);
            else if (nrm == 2)
                launch_fused_inst<T, false, true, 2>(s, op, picard, nz, uin, uout, f, phk, base, part, sk);
            else
                launch_fused_inst<T, false, true, 0>(s, op, picard, nz, uin, uout, f, phk, base, nullptr, sk);
            return;
        }
        if (nrm == 1) {
            launch_fused_inst<T, false, false, 1>(s, op, picard, nz, uin, uout, f, phk, base, part, sk);
            return;
        }
        if (nrm == 2) {
            launch_fused_inst<T, false, false, 2>(s, op, picard, nz, uin, uout, f, phk, base, part, sk);
            return;
        }
    }
    launch_fused_inst<T, DELTA, false, 0>(s, op, picard, nz, uin, uout, f, phk, base, nullptr, sk);
}

template void launch_smooth<double, false>(hipStream_t, const OpParams &, int, int, Tri<double>,
                                           Tri<const double>, const double *, const double *);
template void launch_smooth<float, true>(hipStream_t, const OpParams &, int, int, Tri<float>,
                                         Tri<const float>, const float *, const float *);
template void launch_sweep_fused<double, false>(hipStream_t, const OpParams &, int, int,
                                                Tri<const double>, Tri<double>, Tri<const double>,
                                                const double *, const double *, int,
                                                unsigned long long *, bool);

}  // namespace pfc
