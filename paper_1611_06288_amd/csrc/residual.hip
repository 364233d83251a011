// Residual kernels for large colour-split levels (n a multiple of 64):
// r = f - N(u) with N of the scheme's operator (scheme-PFC-o1..o3, M = 1), or
// of its correction form in the mixed-precision cycle (the cubic term as the
// difference G(e) = g(b + e) - g(b)), followed by one of these epilogues:
//   RT_NORM        max |r| over the level (stop test of the cycle loop),
//   RT_RESTRICT    8-child means of r and u onto the coarse level (the FAS
//                  restriction, Section 3),
//   RT_CAST        max |r|, plus r and phi rounded to FP32 (the defect and the
//                  base of the mixed-precision correction cycle),
//   RT_CAST_CORR   as RT_CAST on u + e, the FP64 iterate with the pending FP32
//                  correction added while the planes are staged; u + e is
//                  written to a second buffer (other columns read this one's
//                  u as their ring in the same launch),
//   RT_RESTRICT32  RT_RESTRICT for the FP32 correction operator.
// A workgroup owns an x-y column of kRX x rt_rows points and a range of planes and
// walks it in z.  Three planes of u (box plus a one-cell ring, all three
// fields) sit in an LDS ring; the next plane and the next step's f and phi^k
// are loaded into registers while the current plane computes, so every value
// is fetched from HBM once per column instead of up to seven times through an
// L2 that cannot hold the reuse distance.  Each thread owns an x-pair of
// points per plane.  The arithmetic and, for the restrictions, the order of
// the 8-child sums equal those of the thread-per-point kernels (and u + e that
// of the separate correction kernel), so results agree bitwise with them.
// MOB (variable mobility; RT_NORM and RT_RESTRICT): phi* is a fourth field of
// the ring and the first equation takes the face-mobility flux sum.
#include "device_common.h"

#include <algorithm>
#include <numeric>
#include <type_traits>

namespace pfc {

constexpr int kRX = 64, kRC = kRX + 2;  // column x-extent, with its ring
// Column rows and threads per workgroup: the FP32 restriction takes 16-row
// columns (its 4-byte rows are short, so the ring rows are the larger share
// of its fetches), every other mode 8 rows; one thread per x-pair of a row.
constexpr int rt_rows(int mode) { return mode == RT_RESTRICT32 ? 16 : 8; }
constexpr int rt_threads(int mode) { return 32 * rt_rows(mode); }

// PK1: the first source component is phi^k itself (one buffer), loaded once.
template <int MODE, bool MOB, bool PK1 = false>
__global__ __launch_bounds__(rt_threads(MODE)) void k_resid_tile(OpParams op, int nz,
                                                                 ResidTileArgs a) {
    constexpr int kRY = rt_rows(MODE), kRT = rt_threads(MODE);
    constexpr int kRR = kRY + 2;                                 // rows with the ring
    constexpr int kRN = kRC * kRR, kRI = (kRN + kRT - 1) / kRT;  // ring points, per thread
    constexpr bool F32 = MODE == RT_RESTRICT32;
    constexpr bool DELTA = F32;
    constexpr bool RESTRICT = MODE == RT_RESTRICT || MODE == RT_RESTRICT32;
    constexpr bool CAST = MODE == RT_CAST || MODE == RT_CAST_CORR;
    constexpr bool CORR = MODE == RT_CAST_CORR;
    using T = typename std::conditional<F32, float, double>::type;
    constexpr int NF = MOB ? 4 : 3;  // ring fields: phi, mu, omega (, phi*)
    __shared__ T t[NF][3][kRR][kRC];  // [field][plane slot][row][x]
    if (gate_closed(op.gate)) return;
    Tri<const T> u, f;
    const T *phk, *bs = nullptr;
    Tri<T> ubar, rr;
    if constexpr (F32) {
        u = a.e32;
        f = a.f32;
        phk = a.phk32;
        bs = a.b32;
        ubar = a.ebar32;
        rr = a.rr32;
    } else {
        u = a.u;
        f = a.f;
        phk = a.phk;
        ubar = a.ubar;
        rr = a.rr;
    }
    const int n = op.lay.n, hn = n >> 1;
    const unsigned un = (unsigned)n, uhn = (unsigned)hn, H = un * un * uhn;
    const int nbx = n / kRX, nby = n / kRY;
    const int b = (int)xcd_block();
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int x0 = bx * kRX, y0 = by * kRY;
    int z0, z1;
    if (RESTRICT) {  // plane pairs stay in one workgroup
        z0 = 2 * (bz * (n / 2) / nz);
        z1 = 2 * ((bz + 1) * (n / 2) / nz);
    } else {
        z0 = bz * n / nz;
        z1 = (bz + 1) * n / nz;
    }
    const int tid = threadIdx.x, qx = tid & 31, qy = tid >> 5;
    const int xe = x0 + 2 * qx, y = y0 + qy;  // this thread's points: (xe, y), (xe + 1, y)
    auto wn = [n](int v) { return v < 0 ? v + n : (v >= n ? v - n : v); };
    auto slot = [z0](int p) { return (p - z0 + 3) % 3; };  // p >= z0 - 1

    T pre[kRI][NF];
    auto load_plane = [&](int p) {
        const int pw = wn(p);
#pragma unroll
        for (int i = 0; i < kRI; ++i) {
            const int c = tid + i * kRT;
            if (c < kRN) {
                const int r = c / kRC, col = c - r * kRC;
                const int yy = wn(y0 - 1 + r), xx = wn(x0 - 1 + col);
                const unsigned g = (unsigned)((xx + yy + pw) & 1) * H +
                                   ((unsigned)pw * un + (unsigned)yy) * uhn + (unsigned)(xx >> 1);
                pre[i][0] = u.a[g];
                pre[i][1] = u.b[g];
                pre[i][2] = u.c[g];
                if constexpr (MOB) pre[i][3] = op.mob.phs[g];
                if constexpr (CORR) {
                    pre[i][0] += (double)a.e.a[g];
                    pre[i][1] += (double)a.e.b[g];
                    pre[i][2] += (double)a.e.c[g];
                }
            }
        }
    };
    auto store_plane = [&](int p) {
        const int s = slot(p);
#pragma unroll
        for (int i = 0; i < kRI; ++i) {
            const int c = tid + i * kRT;
            if (c < kRN) {
                const int r = c / kRC, col = c - r * kRC;
                t[0][s][r][col] = pre[i][0];
                t[1][s][r][col] = pre[i][1];
                t[2][s][r][col] = pre[i][2];
                if constexpr (MOB) t[3][s][r][col] = pre[i][3];
            }
        }
    };
    // f (3 fields), phi^k and (correction form) the base at the thread's two points of plane p
    auto own_index = [&](int p, int e) {
        const int x = xe + e;
        return (unsigned)((x + y + p) & 1) * H + ((unsigned)p * un + (unsigned)y) * uhn +
               (unsigned)(x >> 1);
    };
    constexpr int NO = DELTA ? 5 : 4;
    auto load_own = [&](int p, T (&o)[2][NO]) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const unsigned g = own_index(p, e);
            o[e][3] = phk[g];
            o[e][0] = PK1 ? o[e][3] : f.a[g];
            o[e][1] = f.b[g];
            o[e][2] = f.c[g];
            if constexpr (DELTA) o[e][4] = bs[g];
        }
    };

    load_plane(z0 - 1);
    store_plane(z0 - 1);
    load_plane(z0);
    store_plane(z0);
    load_plane(z0 + 1);
    T cur[2][NO];
    load_own(z0, cur);
    store_plane(z0 + 1);
    __syncthreads();

    unsigned long long m = 0;
    double sr[3] = {0.0, 0.0, 0.0}, su[3] = {0.0, 0.0, 0.0};
    const double h2inv = op.h2inv;
    for (int p = z0; p < z1; ++p) {
        T nxt[2][NO];
        if (p + 1 < z1) {
            load_plane(p + 2);
            load_own(p + 1, nxt);
        }
        const int s0 = slot(p), sm = slot(p - 1), sp = slot(p + 1), row = qy + 1;
        double r[2][3], uu[2][3];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int col = 2 * qx + e + 1;
            double ls[3];
#pragma unroll
            for (int fl = 0; fl < 3; ++fl) {
                uu[e][fl] = (double)t[fl][s0][row][col];
                const double nsum =
                    ((double)t[fl][s0][row][col + 1] + (double)t[fl][s0][row][col - 1]) +
                    ((double)t[fl][s0][row + 1][col] + (double)t[fl][s0][row - 1][col]) +
                    ((double)t[fl][sp][row][col] + (double)t[fl][sm][row][col]);
                ls[fl] = (nsum - 6.0 * uu[e][fl]) * h2inv;
            }
            const double phi = uu[e][0], mu = uu[e][1], om = uu[e][2], ak = (double)cur[e][3];
            const double bb = DELTA ? (double)cur[e][NO - 1] : 0.0;
            if constexpr (MOB) {  // flux form, faces in the order xp, xm, yp, ym, zp, zm
                const double pc = (double)t[3][s0][row][col];
                double sm6 = 0.0;
                auto face = [&](int sl3, int rw, int cl) {
                    sm6 += face_mob(op.mob, pc, (double)t[3][sl3][rw][cl]) *
                           ((double)t[1][sl3][rw][cl] - mu);
                };
                face(s0, row, col + 1);
                face(s0, row, col - 1);
                face(s0, row + 1, col);
                face(s0, row - 1, col);
                face(sp, row, col);
                face(sm, row, col);
                ls[1] = sm6 * h2inv;
            }
            resid_from_lap<DELTA>(op, ls, phi, mu, om, (double)cur[e][0], (double)cur[e][1],
                                  (double)cur[e][2], ak, bb, r[e]);
        }
        if constexpr (RESTRICT) {
            // children in the order (x, y, z) = 000, 100, 010, 110, 001, ...: this
            // row's pair, then the odd row's pair (lane + 32 of the same wave)
#pragma unroll
            for (int fl = 0; fl < 3; ++fl) {
                const double pr0 = __shfl_xor(r[0][fl], 32), pr1 = __shfl_xor(r[1][fl], 32);
                const double pu0 = __shfl_xor(uu[0][fl], 32), pu1 = __shfl_xor(uu[1][fl], 32);
                sr[fl] += r[0][fl];
                sr[fl] += r[1][fl];
                sr[fl] += pr0;
                sr[fl] += pr1;
                su[fl] += uu[0][fl];
                su[fl] += uu[1][fl];
                su[fl] += pu0;
                su[fl] += pu1;
            }
            if ((p & 1) && !(qy & 1)) {
                const unsigned c = sidx32(a.LC, xe >> 1, y >> 1, p >> 1);
                rr.a[c] = (T)(0.125 * sr[0]);
                rr.b[c] = (T)(0.125 * sr[1]);
                rr.c[c] = (T)(0.125 * sr[2]);
                ubar.a[c] = (T)(0.125 * su[0]);
                ubar.b[c] = (T)(0.125 * su[1]);
                ubar.c[c] = (T)(0.125 * su[2]);
            }
            if (p & 1) {
#pragma unroll
                for (int fl = 0; fl < 3; ++fl) sr[fl] = su[fl] = 0.0;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                m = umax(m, umax(abs_bits(r[e][0]), umax(abs_bits(r[e][1]), abs_bits(r[e][2]))));
                if constexpr (CAST) {
                    const unsigned g = own_index(p, e);
                    a.r32.a[g] = (float)r[e][0];
                    a.r32.b[g] = (float)r[e][1];
                    a.r32.c[g] = (float)r[e][2];
                    a.base32[g] = (float)uu[e][0];
                    if constexpr (CORR) {
                        a.uout.a[g] = uu[e][0];
                        a.uout.b[g] = uu[e][1];
                        a.uout.c[g] = uu[e][2];
                    }
                }
            }
        }
        __syncthreads();  // every thread is done with plane p - 1's slot
        if (p + 1 < z1) {
            store_plane(p + 2);
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
                for (int v = 0; v < NO; ++v) cur[e][v] = nxt[e][v];
        }
        __syncthreads();  // plane p + 2 visible
    }
    if constexpr (!RESTRICT) {
        m = block_max_u64(m);
        if (threadIdx.x == 0) a.partial[blockIdx.x] = m;
    }
}

bool resid_tile_fits(const Lay &L) {
    return L.split && L.n % kRX == 0 && L.n % rt_rows(RT_RESTRICT32) == 0;
}

static const void *resid_tile_fn(int mode, bool mob) {
    switch (mode) {
        case RT_RESTRICT:
            return mob ? (const void *)k_resid_tile<RT_RESTRICT, true>
                       : (const void *)k_resid_tile<RT_RESTRICT, false>;
        case RT_CAST: return (const void *)k_resid_tile<RT_CAST, false>;
        case RT_CAST_CORR: return (const void *)k_resid_tile<RT_CAST_CORR, false>;
        case RT_RESTRICT32: return (const void *)k_resid_tile<RT_RESTRICT32, false>;
        default:
            return mob ? (const void *)k_resid_tile<RT_NORM, true>
                       : (const void *)k_resid_tile<RT_NORM, false>;
    }
}

int resid_tile_slots(int device, int mode, bool mob) {
    int occ = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, resid_tile_fn(mode, mob),
                                                     rt_threads(mode), 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return occ * cus;
}

// Plane ranges per column: the smallest count for which the launch is a
// whole number of resident waves with at least 4 planes (2 plane pairs for
// the restriction) per range, within the partial-result buffer.
int resid_tile_nz(int n, int slots, int mode) {
    const int cols = (n / kRX) * (n / rt_rows(mode));
    const bool pairs = mode == RT_RESTRICT || mode == RT_RESTRICT32;
    const int units = pairs ? n / 2 : n;  // plane pairs or planes
    const int minu = pairs ? 2 : 4;
    int nz = slots > 0 ? slots / std::gcd(cols, slots) : std::max(1, units / 16);
    if (units / nz < minu) nz = std::max(1, units / minu);
    while (nz > 1 && cols * nz > kMaxReduceBlocks) nz /= 2;
    return nz;
}

int launch_resid_tile(hipStream_t s, int mode, const OpParams &op, int nz, const ResidTileArgs &a) {
    const int n = op.lay.n;
    const unsigned blocks = (unsigned)((n / kRX) * (n / rt_rows(mode)) * nz);
    const dim3 block(rt_threads(mode));
    const bool mob = op.mob.phs != nullptr;  // FP64 modes only (the FP32 cycle has M = 1)
    switch (mode) {
        case RT_RESTRICT:
            if (mob && a.f.a == a.phk)
                hipLaunchKernelGGL((k_resid_tile<RT_RESTRICT, true, true>), dim3(blocks), block,
                                   0, s, op, nz, a);
            else if (mob)
                hipLaunchKernelGGL((k_resid_tile<RT_RESTRICT, true>), dim3(blocks), block, 0, s,
                                   op, nz, a);
            else if (a.f.a == a.phk)
                hipLaunchKernelGGL((k_resid_tile<RT_RESTRICT, false, true>), dim3(blocks), block,
                                   0, s, op, nz, a);
            else
                hipLaunchKernelGGL((k_resid_tile<RT_RESTRICT, false>), dim3(blocks), block, 0,
                                   s, op, nz, a);
            break;
        case RT_CAST:
            hipLaunchKernelGGL((k_resid_tile<RT_CAST, false>), dim3(blocks), block, 0, s, op, nz,
                               a);
            break;
        case RT_CAST_CORR:
            hipLaunchKernelGGL((k_resid_tile<RT_CAST_CORR, false>), dim3(blocks), block, 0, s, op,
                               nz, a);
            break;
        case RT_RESTRICT32:
            hipLaunchKernelGGL((k_resid_tile<RT_RESTRICT32, false>), dim3(blocks), block, 0, s,
                               op, nz, a);
            break;
        default:
            if (mob)
                hipLaunchKernelGGL((k_resid_tile<RT_NORM, true>), dim3(blocks), block, 0, s, op,
                                   nz, a);
            else
                hipLaunchKernelGGL((k_resid_tile<RT_NORM, false>), dim3(blocks), block, 0, s, op,
                                   nz, a);
    }
    return (int)blocks;
}

}  // namespace pfc
