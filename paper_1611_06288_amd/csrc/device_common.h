// Device-side helpers shared by the HIP translation units: index arithmetic
// of the natural and colour-split layouts, the cubic term, reductions and the
// small dense inverse used at the coarsest level.
#pragma once

#include <math.h>

#include "pfc_internal.h"

namespace pfc {

static inline unsigned blocks_for(size_t count) { return (unsigned)((count + kBlock - 1) / kBlock); }

static inline unsigned reduce_blocks(size_t count) {
    const size_t b = (count + kBlock - 1) / kBlock;
    return (unsigned)(b < (size_t)kMaxReduceBlocks ? b : (size_t)kMaxReduceBlocks);
}

__device__ __forceinline__ unsigned xcd_block() {
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned per = nb >> 3;
    if (b < (per << 3)) return (b & 7u) * per + (b >> 3);
    return b;
}

// True when a cycle gate is set and closed (see OpParams::gate).
__device__ __forceinline__ bool gate_closed(const int *gate) { return gate && *gate == 0; }

__device__ __forceinline__ int wrap_p(int i, int n) { return i == n - 1 ? 0 : i + 1; }
__device__ __forceinline__ int wrap_m(int i, int n) { return i == 0 ? n - 1 : i - 1; }

__device__ __forceinline__ size_t npts(const Lay &L) { return (size_t)L.n * L.n * L.n; }

// Storage offset of point (i, j, k).
__device__ __forceinline__ size_t sidx(const Lay &L, int i, int j, int k) {
    const size_t n = (size_t)L.n;
    if (!L.split) return ((size_t)k * n + (size_t)j) * n + (size_t)i;
    const size_t H = n * n * n / 2;
    return (size_t)((i + j + k) & 1) * H + ((size_t)k * n + (size_t)j) * (n >> 1) + (size_t)(i >> 1);
}

// Grid point stored at offset t.
__device__ __forceinline__ void decode(const Lay &L, unsigned t, int &i, int &j, int &k) {
    const int n = L.n;
    if (!L.split) {
        const unsigned row = L.dn.q(t);
        i = (int)(t - row * (unsigned)n);
        k = (int)L.dn.q(row);
        j = (int)(row - (unsigned)k * (unsigned)n);
        return;
    }
    const unsigned H = (unsigned)((size_t)n * n * n / 2);
    const int c = t >= H ? 1 : 0;
    const unsigned r = t - (c ? H : 0u);
    const unsigned hn = (unsigned)(n >> 1);
    const unsigned row = L.dh.q(r);
    const int m = (int)(r - row * hn);
    k = (int)L.dn.q(row);
    j = (int)(row - (unsigned)k * (unsigned)n);
    i = 2 * m + ((c + j + k) & 1);
}

// Grid point number t in natural (x fastest) order, whatever the storage.
__device__ __forceinline__ void decode_nat(const Lay &L, unsigned t, int &i, int &j, int &k) {
    const unsigned row = L.dn.q(t);
    i = (int)(t - row * (unsigned)L.n);
    k = (int)L.dn.q(row);
    j = (int)(row - (unsigned)k * (unsigned)L.n);
}

// 32-bit storage offset (every level has at most 2^30 points).
__device__ __forceinline__ unsigned sidx32(const Lay &L, int i, int j, int k) {
    const unsigned n = (unsigned)L.n;
    if (!L.split) return ((unsigned)k * n + (unsigned)j) * n + (unsigned)i;
    const unsigned H = n * n * n / 2;
    return ((unsigned)((i + j + k) & 1)) * H + ((unsigned)k * n + (unsigned)j) * (n >> 1) +
           (unsigned)(i >> 1);
}

// A point and its six face neighbours, periodic, as 32-bit offsets.
struct Off {
    unsigned c, xp, xm, yp, ym, zp, zm;
};

__device__ __forceinline__ Off offs(const Lay &L, int i, int j, int k) {
    const int n = L.n;
    const int im = wrap_m(i, n), ip = wrap_p(i, n), jm = wrap_m(j, n), jp = wrap_p(j, n),
              km = wrap_m(k, n), kp = wrap_p(k, n);
    Off q;
    const unsigned un = (unsigned)n;
    if (!L.split) {
        const unsigned row = (unsigned)k * un + (unsigned)j;
        q.c = row * un + (unsigned)i;
        q.xm = row * un + (unsigned)im;
        q.xp = row * un + (unsigned)ip;
        q.ym = ((unsigned)k * un + (unsigned)jm) * un + (unsigned)i;
        q.yp = ((unsigned)k * un + (unsigned)jp) * un + (unsigned)i;
        q.zm = ((unsigned)km * un + (unsigned)j) * un + (unsigned)i;
        q.zp = ((unsigned)kp * un + (unsigned)j) * un + (unsigned)i;
        return q;
    }
    const unsigned hn = un >> 1, H = un * un * hn;
    const unsigned colour = (unsigned)((i + j + k) & 1);
    const unsigned oc = (colour ^ 1u) * H;
    const unsigned row = (unsigned)k * un + (unsigned)j;
    const unsigned m = (unsigned)(i >> 1);
    q.c = colour * H + row * hn + m;
    q.xm = oc + row * hn + (unsigned)(im >> 1);
    q.xp = oc + row * hn + (unsigned)(ip >> 1);
    q.ym = oc + ((unsigned)k * un + (unsigned)jm) * hn + m;
    q.yp = oc + ((unsigned)k * un + (unsigned)jp) * hn + m;
    q.zm = oc + ((unsigned)km * un + (unsigned)j) * hn + m;
    q.zp = oc + ((unsigned)kp * un + (unsigned)j) * hn + m;
    return q;
}

template <typename T>
__device__ __forceinline__ double nsum(const T *__restrict__ v, const Off &q) {
    return ((double)v[q.xp] + (double)v[q.xm]) + ((double)v[q.yp] + (double)v[q.ym]) +
           ((double)v[q.zp] + (double)v[q.zm]);
}

// Cubic term of the chemical potential in its second-order form,
// g(x; a) = 1/4 (x + a)(x^2 + a^2), a = phi^kappa (Section 5, N2).
// DELTA: the correction form G(e) = g(b + e; a) - g(b; a), expanded without
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

// The parts of N that differ between the two schemes (OpParams::fo).  The
// first-order convex splitting takes the cubic term as x^3 and the linear one
// as (1-eps) x in N2, and N3 = omega - Lap phi; the second-order scheme takes
// g(x; a), (1-eps)/2 x and N3 = omega - Lap phi / 2.  (The correction form of
// the mixed-precision cycle exists for the second-order scheme only.)
template <bool DELTA>
__device__ __forceinline__ double g_of(int fo, double x, double a, double b) {
    if (!DELTA && fo) return x * x * x;
    return Cubic<DELTA>::g(x, a, b);
}
template <bool DELTA>
__device__ __forceinline__ double dg_of(int fo, double x, double a, double b) {
    if (!DELTA && fo) return 3.0 * x * x;
    return Cubic<DELTA>::dg(x, a, b);
}
__device__ __forceinline__ double lin_of(const OpParams &op) {
    return op.fo ? 1.0 - op.eps : 0.5 * (1.0 - op.eps);
}
__device__ __forceinline__ double w3_of(const OpParams &op) { return op.fo ? 1.0 : 0.5; }

// Mobility on the face between two cells: M of the average of their phi*.
__device__ __forceinline__ double face_mob(const Mobility &mb, double pa, double pb) {
    const double v = 0.5 * (pa + pb);
    const double m = mb.m0 + mb.m1 * v + mb.m2 * v * v;
    return m > mb.mmin ? m : mb.mmin;
}

__device__ __forceinline__ unsigned long long abs_bits(double v) {
    return (unsigned long long)__double_as_longlong(v) & 0x7fffffffffffffffull;
}

__device__ __forceinline__ unsigned long long umax(unsigned long long a, unsigned long long b) {
    return a > b ? a : b;
}

// Block max of non-negative IEEE bit patterns (NaN sorts above +Inf, so a
// NaN residual is never lost).
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v) {
    __shared__ unsigned long long red[kBlock];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = umax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    return red[0];
}

// Block max of non-negative IEEE bit patterns through wave shuffles and one
// word per wave of LDS (wm: blockDim.x / 64 entries); for kernels whose LDS
// budget leaves no room for a per-thread array.  Every thread calls it.
__device__ __forceinline__ unsigned long long block_max_u64_waves(unsigned long long v,
                                                                  unsigned long long *wm) {
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = (unsigned long long)__double_as_longlong(
            __shfl_xor(__longlong_as_double((long long)v), off, 64));
        v = umax(v, o);
    }
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long r = wm[0];
    for (unsigned w = 1; w < blockDim.x / 64; ++w) r = umax(r, wm[w]);
    return r;
}

// r = S - N(u) at one point (M = 1) from the discrete Laplacians ls of phi, mu
// and omega there: the three equations of the scheme's operator (the cubic
// term as g, or its correction form with base bb when DELTA).  Every kernel
// that forms a point residual from Laplacians calls this, so their results
// agree bit for bit.
template <bool DELTA>
__device__ __forceinline__ void resid_from_lap(const OpParams &op, const double (&ls)[3],
                                               double phi, double mu, double om, double f0,
                                               double f1, double f2, double ak, double bb,
                                               double (&r)[3]) {
    const double tau = op.tau, lin_c = lin_of(op), w3 = w3_of(op);
    r[0] = f0 - (phi - tau * ls[1]);
    r[1] = f1 - (mu - g_of<DELTA>(op.fo, phi, ak, bb) - lin_c * phi - ls[2]);
    r[2] = f2 - (om - w3 * ls[0]);
}

// N(u) at one point from u's own values and the discrete Laplacians ls of phi,
// mu and omega there (ls[1] the flux sum where the mobility varies): the
// coarse-level term of the tau correction f_c = N_c(I u) + I r (Algorithm
// algorithm:FAS).  The tau kernel and the sweep that forms the correction as
// it smooths both call it, so their results agree bit for bit.
template <bool DELTA>
__device__ __forceinline__ void n_of_point(const OpParams &op, const double (&ls)[3], double phi,
                                           double mu, double om, double ak, double bb,
                                           double (&nv)[3]) {
    nv[0] = phi - op.tau * ls[1];
    nv[1] = mu - g_of<DELTA>(op.fo, phi, ak, bb) - lin_of(op) * phi - ls[2];
    nv[2] = om - w3_of(op) * ls[0];
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}


// In-place inverse of the P x P matrix A (column-major, A[col * P + row], in
// LDS) by Gauss-Jordan elimination with partial (row) pivoting.  Called by
// one whole 64-lane workgroup: lane p eliminates in row p and swaps entries
// of column p; perm is 64 ints of LDS.  Row interchanges are undone as column
// interchanges at the end.
__device__ __forceinline__ void gj_invert(double *A, int P, int *perm) {
    const int p = threadIdx.x;
    const bool act = p < P;
    for (int c = 0; c < P; ++c) {
        double val = (act && p >= c) ? fabs(A[c * P + p]) : -1.0;
        int id = p;
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(val, off, 64);
            const int oid = __shfl_xor(id, off, 64);
            if (ov > val || (ov == val && oid < id)) {
                val = ov;
                id = oid;
            }
        }
        const int pr = id;
        if (p == 0) perm[c] = pr;
        if (pr != c && act) {  // swap rows c and pr; lane p handles column p
            const double tmp = A[p * P + c];
            A[p * P + c] = A[p * P + pr];
            A[p * P + pr] = tmp;
        }
        __syncthreads();
        const double pinv = 1.0 / A[c * P + c];
        __syncthreads();
        if (act) A[p * P + c] = (p == c ? 1.0 : A[p * P + c]) * pinv;  // scale pivot row
        __syncthreads();
        if (act && p != c) {
            // full chunks of 16 columns take all their loads before their
            // stores (the pivot row is not written in this phase), so the LDS
            // latency is paid once per chunk; the rest goes one by one
            const double fr = A[c * P + p];
            int q0 = 0;
            for (; q0 + 16 <= P; q0 += 16) {
                double own[16], piv[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    own[i] = A[(q0 + i) * P + p];
                    piv[i] = A[(q0 + i) * P + c];
                }
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    A[(q0 + i) * P + p] = ((q0 + i == c) ? 0.0 : own[i]) - fr * piv[i];
            }
            for (int q = q0; q < P; ++q) {
                const double old = (q == c) ? 0.0 : A[q * P + p];
                A[q * P + p] = old - fr * A[q * P + c];
            }
        }
        __syncthreads();
    }
    for (int c = P - 1; c >= 0; --c) {  // undo the row swaps as column swaps
        const int pr = perm[c];
        if (pr != c && act) {
            const double tmp = A[c * P + p];
            A[c * P + p] = A[pr * P + p];
            A[pr * P + p] = tmp;
        }
        __syncthreads();
    }
}

}  // namespace pfc
