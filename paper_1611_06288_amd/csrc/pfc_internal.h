// Internal interface between the HIP kernels (kernels.hip) and the host
// runtime.  Not part of the public C ABI.
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
__host__ __device__ inline Tri<const T> cst(Tri<T> t) { return Tri<const T>{t.a, t.b, t.c}; }

// Division by n = 2^s or 3*2^s without integer divide instructions.
struct Div {
    unsigned shift;  // s
    unsigned three;  // 1 if n = 3*2^s
    __host__ __device__ unsigned q(unsigned x) const {
        x >>= shift;
        return three ? (unsigned)(((unsigned long long)x * 0xAAAAAAABull) >> 33) : x;
    }
};

Div make_div(int d);  // host: d must be 2^s or 3*2^s

// Storage of one level's fields.  Natural: C order [k][j][i].  Colour-split
// (n even): the points of colour c = (i+j+k) mod 2 are stored in block c of
// size n^3/2, row (k, j) by row, a point at position i >> 1 of its row.
struct Lay {
    int n;
    int split;
    Div dn;   // division by n
    Div dh;   // division by n/2 (split only)
};

Lay make_lay(int n, bool split);

inline size_t npts_host(const Lay &L) { return (size_t)L.n * L.n * L.n; }

// Variable mobility M(v) = max(mmin, m0 + m1 v + m2 v^2) of the first
// equation's flux form, evaluated on each face at the face average of phi*
// (phi* in the level's layout; null: M = 1).
struct Mobility {
    const double *phs = nullptr;
    double m0 = 1.0, m1 = 0.0, m2 = 0.0, mmin = 0.0;
};

// Scalar parameters of one level's operator.
struct OpParams {
    Lay lay;
    double h2inv;  // 1 / h_l^2
    double tau;    // time step
    double eps;    // epsilon
    // 1: the first-order convex-splitting scheme (N2 with phi^3 and (1-eps)
    // phi, N3 = omega - Lap phi); 0: the second-order scheme of Section 5
    int fo = 0;
    Mobility mob{};
    // Cycle gate (time loop replayed as a graph): when set and *gate == 0 the
    // cycle's kernels return at once, so cycles after convergence do nothing.
    const int *gate = nullptr;
};

constexpr int kBlock = 256;
constexpr int kMaxReduceBlocks = 16384;
constexpr int kMaxN = 1024;

// ---- building blocks; T = double or float, DELTA selects the correction
// form g(base + e) - g(base) of the cubic term ----
template <typename T, bool DELTA>
void launch_smooth(hipStream_t s, const OpParams &op, int colour, int picard, Tri<T> u,
                   Tri<const T> f, const T *phk, const T *base);

// The first half-sweep of colour `colour` on a coarse level whose iterate
// starts at I u (ubar), forming the tau correction f += N(I u) at that
// colour's points as it smooths (f holds I r on entry, I u is not copied into
// u); two calls (colour 0, then 1) equal launch_tau followed by two
// launch_smooth calls bit for bit.
template <typename T, bool DELTA>
void launch_smooth_tau(hipStream_t s, const OpParams &op, int colour, int picard, Tri<T> u,
                       Tri<T> f, Tri<const T> ubar, const T *phk, const T *base);

// One full red-black sweep in place on a level of at most kSmallSweepN^3
// points, by a single workgroup (colour 0, barrier, colour 1).  Measured:
// 3.8 us against two 2.3 us launches at 8^3, but 14 us against two 3.3 us
// launches at 16^3 (one CU then carries too much latency-bound work).
constexpr int kSmallSweepN = 8;
template <typename T, bool DELTA>
void launch_sweep_small(hipStream_t s, const OpParams &op, int picard, Tri<T> u, Tri<const T> f,
                        const T *phk, const T *base);
// The same as the first sweep of a coarse level, forming the tau correction
// (as launch_smooth_tau).
template <typename T, bool DELTA>
void launch_sweep_small_tau(hipStream_t s, const OpParams &op, int picard, Tri<T> u, Tri<T> f,
                            Tri<const T> ubar, const T *phk, const T *base);

// One full red-black sweep (colour 0 then colour 1) from uin into uout
// (distinct buffers, colour-split storage), bitwise equal to two launch_smooth
// calls; the level is cut into nz plane ranges (see fused_nz).  Instantiated
// for double only.  nrm (M = 1 only) adds half of the stop-test norm as
// per-workgroup maxima of |S - N(u)| bits in part[0 .. fused_blocks(n, nz)):
// 1 over the colour-0 points of uin, 2 over the colour-1 points of uout.
// skip0: mu and omega of colour-0 points are not written to uout (only when
// the next operation on uout is another fused sweep, which does not read them).
template <typename T, bool DELTA>
void launch_sweep_fused(hipStream_t s, const OpParams &op, int picard, int nz, Tri<const T> uin,
                        Tri<T> uout, Tri<const T> f, const T *phk, const T *base, int nrm = 0,
                        unsigned long long *part = nullptr, bool skip0 = false);
int fused_blocks(int n, int nz);  // workgroups of one fused-sweep launch
bool fused_fits(int n);           // n admits the fused sweep's column tiling
int fused_slots(int device, bool mob = false);      // resident fused-sweep workgroups on the device (0 on error)
int fused_nz(int n, int slots);   // plane ranges per column for a level of size n
constexpr int kFusedMinN = 128;  // smaller levels use the half-sweeps

// Residual of a large level by z-marching column tiles (residual.hip), with
// one of five epilogues.
enum { RT_NORM = 0, RT_RESTRICT = 1, RT_CAST = 2, RT_CAST_CORR = 3, RT_RESTRICT32 = 4, RT_MODES = 5 };
struct ResidTileArgs {
    // FP64 operator: RT_NORM, RT_RESTRICT, RT_CAST, RT_CAST_CORR
    Tri<const double> u{nullptr, nullptr, nullptr}, f{nullptr, nullptr, nullptr};
    const double *phk = nullptr;
    Tri<double> ubar{nullptr, nullptr, nullptr};  // RT_RESTRICT: I u
    Tri<double> rr{nullptr, nullptr, nullptr};    // RT_RESTRICT: I r
    Tri<float> r32{nullptr, nullptr, nullptr};    // RT_CAST*: r in FP32
    float *base32 = nullptr;                      // RT_CAST*: phi in FP32
    Tri<const float> e{nullptr, nullptr, nullptr};  // RT_CAST_CORR: correction added to u
    Tri<double> uout{nullptr, nullptr, nullptr};    // RT_CAST_CORR: u + e (distinct from u)
    // FP32 correction operator: RT_RESTRICT32
    Tri<const float> e32{nullptr, nullptr, nullptr}, f32{nullptr, nullptr, nullptr};
    const float *phk32 = nullptr, *b32 = nullptr;
    Tri<float> ebar32{nullptr, nullptr, nullptr}, rr32{nullptr, nullptr, nullptr};
    Lay LC{};                               // restrictions: the coarse level
    unsigned long long *partial = nullptr;  // RT_NORM, RT_CAST*: per-workgroup max |r|
};
bool resid_tile_fits(const Lay &L);
// The stop-test norm takes the column tiles from this size on; on a 64^3
// level each column holds a few planes and the thread-per-point norm is
// faster (7 against 11 us), while the restriction keeps the tiles there.
constexpr int kTileNormMinN = 128;
int resid_tile_slots(int device, int mode, bool mob = false);   // resident workgroups (0 on error)
int resid_tile_nz(int n, int slots, int mode);
int launch_resid_tile(hipStream_t s, int mode, const OpParams &op, int nz,
                      const ResidTileArgs &a);  // returns the workgroup count

template <typename T, bool DELTA>
void launch_resid_restrict(hipStream_t s, const OpParams &op, const Lay &coarse, Tri<const T> u,
                           Tri<const T> f, const T *phk, const T *base, Tri<T> ubar_c, Tri<T> rr_c);

template <typename T>
void launch_restrict(hipStream_t s, const Lay &fine, const Lay &coarse, const T *fine_v, T *coarse_v);

template <typename T, bool DELTA>
void launch_tau(hipStream_t s, const OpParams &opc, Tri<const T> ubar, Tri<T> f, Tri<T> u,
                const T *phk, const T *base);

// fine += P (v - ubar); ubar.a may be null; fine.b null: one field only.
// phi0: a smoothing sweep follows, so mu and omega at colour-0 points may be
// left uncorrected (they are dead until the sweep overwrites them); the tiled
// levels skip them, the others correct everything.
template <typename T>
void launch_prolong(hipStream_t s, const Lay &coarse, const Lay &fine, Tri<const T> v,
                    Tri<const T> ubar, Tri<T> fine_u, const int *gate = nullptr,
                    bool phi0 = false, int nzr = 0);
int prolong_tile_slots(int device, bool fp32);  // resident workgroups (0 on error)
int prolong_tile_nzr(int slots, int nc, int nf);  // coarse-plane ranges per column

// Residual r = f - N(u) (r.a may be null) and per-block maxima of |r| as
// IEEE bit patterns; returns the number of partials written.
template <typename T, bool DELTA>
int launch_resid_max(hipStream_t s, const OpParams &op, Tri<const T> u, Tri<const T> f,
                     const T *phk, const T *base, Tri<T> r, unsigned long long *partial);

void launch_max_final(hipStream_t s, const unsigned long long *partial, int count, double *out,
                      const int *gate = nullptr);
// dst[0] = max of partial[0 .. count), dst[1 .. dcount) = 0 (bit patterns).
void launch_norm_seed(hipStream_t s, const unsigned long long *partial, int count,
                      unsigned long long *dst, int dcount);

// Device-side stop test of the time loop: the cycle loop's decision on the
// residual max-norm before a cycle, reduced from the per-workgroup maxima
// partial[0 .. count) (IEEE bit patterns) by the same one-block launch, made
// on the GPU so that a
// replayed graph of cycles needs no host round trip.  active: cycles still
// wanted (the gate of the cycle kernels); cycles: cycles started; status: a
// pfc_status; res0/res: first and latest norm.
struct RunState {
    int *active;
    int *cycles;
    int *status;
    double *res0;
    double *res;
};
void launch_run_reset(hipStream_t s, RunState st);
void launch_stop_test(hipStream_t s, const unsigned long long *partial, int count, double tol,
                      int max_cycles, RunState st);

// Coarsest level (natural layout, n = 3 or 4).  lu/piv: cached factorisation
// of the Newton matrix (device scratch of 64*64 doubles and 64 ints), reused
// across calls while *lu_valid is set.  With ubar.a set the launch first
// applies the level's tau correction (f holds I r; fw is f writable) and
// starts u at I u = ubar, as launch_tau does.
template <typename T, bool DELTA>
void launch_coarse(hipStream_t s, const OpParams &op, Tri<T> u, Tri<const T> f, const T *phk,
                   const T *base, const double *lap1, const double *lap3, double *lu, int *piv,
                   int *lu_valid, int *iters, const double *lap2 = nullptr,
                   Tri<const T> ubar = Tri<const T>{nullptr, nullptr, nullptr},
                   Tri<T> fw = Tri<T>{nullptr, nullptr, nullptr});

// phi* = 3/2 phi^k - 1/2 phi^{k-1} from natural-layout inputs into layout L.
void launch_phistar(hipStream_t s, const Lay &L, const double *phk, const double *phkm1,
                    double *out);

// Finest-level source from natural-layout phi^k, phi^{k-1} into layout `op.lay`.
void launch_source(hipStream_t s, const OpParams &op, const double *phk, const double *phkm1,
                   Tri<double> f);
void launch_init_guess(hipStream_t s, const OpParams &nat, const double *phi0, double *mu,
                       double *om);

// Layout conversion of `count` consecutive fields between natural and `lay`
// (with a type cast).
template <typename S, typename D>
void launch_to_lay(hipStream_t s, const Lay &lay, const S *src, D *dst, int count);
template <typename S, typename D>
void launch_from_lay(hipStream_t s, const Lay &lay, const S *src, D *dst, int count);

// Energy on natural-layout fields: per-block sums, then a fixed-order final sum.
int energy_blocks(int n);
void launch_energy(hipStream_t s, const Lay &nat, double h, double eps, const double *phi,
                   const double *phi_prev, double *partial, double *out3);

// ---- mixed-precision helpers (FP64 finest level, FP32 correction) ----
// u64 += e32 on three fields (same layout, n points each).
void launch_add_correction(hipStream_t s, size_t P, Tri<double> u, Tri<const float> e);
// r = f - N(u) in FP64, per-block max-norm partials, and FP32 copies of r and
// of u.a (the base of the correction cycle).
int launch_resid_cast(hipStream_t s, const OpParams &op, Tri<const double> u, Tri<const double> f,
                      const double *phk, Tri<float> r32, float *base32,
                      unsigned long long *partial);
// Fills `count` floats with zero.
void launch_zero(hipStream_t s, float *p, size_t count);


// ---- batched form ----
enum { BK_SMOOTH = 0, BK_RR = 1, BK_TAU = 2, BK_PROLONG = 3, BK_ERR = 4, BK_NORM = 5, BK_KINDS = 6 };
// Batched tile shapes: a tile covers W consecutive work items of a plane
// (W = kTileMin << (shape % kWOpts): 64 .. 1024) in Z consecutive planes
// (Z = 1 << (shape / kWOpts): 1 .. 8), walked plane by plane; the stop
// test's norm uses shape kNormShape (W = 256, Z = 4).
constexpr int kTileMin = 64, kWOpts = 5, kZOpts = 4, kShapes = kWOpts * kZOpts;
constexpr int kNormShape = 2 + kWOpts * 2;

// One instance on one level, as seen by a batched launch.
struct BSeg {
    OpParams op;                 // this level
    Lay lay_c;                   // next coarser level (restriction, interpolation)
    Tri<double> u, f, ubar;      // this level
    Tri<double> uc, fc, ubarc;   // next coarser level
    double *phk;                 // phi^k on this level
    const double *lap1, *lap3;   // coarsest-level matrices of this instance
    double *minv;                // cached coarsest inverse
    int *valid, *iters;
    const int *active;           // the instance's convergence flag
    int inst;
    // first tile of this segment in the work-list of a launch over its list,
    // per phase kind and tile shape: segments are padded to whole tiles, so
    // a workgroup finds a tile's segment by binary search
    unsigned first[BK_KINDS][kShapes];
    // the same for the column-tiled interpolation, per coarse planes per
    // tile (1 << zi); every tile of a segment is a whole column
    unsigned ptf[kZOpts];
};

// Per-instance state of the batched stop test (device arrays).
struct BState {
    int *active, *cycles, *status;
    double *res0, *res;
    const unsigned *norm_first, *norm_blocks;  // per finest-level segment
};

// One launch of a batched phase over `ntiles` tiles of shape `shape`,
// `threads` per workgroup: one tile per workgroup (slots = 0) or
// persistent, at most `slots` workgroups walking the tiles.  arg0,
// arg1: the half-sweep's colour and picard flag (BK_SMOOTH); for BK_PROLONG
// arg0 = 1 when a smoothing sweep follows (colour-0 mu, omega left
// unwritten).
void launch_batch(hipStream_t s, int kind, const BSeg *segs, int nseg, unsigned ntiles, int shape,
                  int threads, unsigned slots, int arg0, int arg1);
// Work items of one segment as planes: Q items per plane, NPL planes (the
// item index is plane * Q + position), for the tile shapes.
void bseg_planes_host(const BSeg &g, int kind, unsigned &Q, unsigned &NPL);
// Resident workgroups of a phase kind's kernel at `threads` per workgroup.
int batch_phase_slots(int kind, int threads, int device);
void launch_batch_coarse(hipStream_t s, const BSeg *segs, int nseg, int tau);
void launch_batch_norm(hipStream_t s, const BSeg *segs, int nseg, unsigned ntiles,
                       unsigned long long *partial, BState st, double tol, int max_cycles);
void launch_batch_reset(hipStream_t s, BState st, int count, int **valid);
// Column-tiled interpolation of the batched form (fine levels whose size is a
// multiple of kBPX): a kBPX x 8 fine column and 1 << zi coarse planes of one
// instance per workgroup, the coarse error formed while staged (no
// coarse-error pass before it).  Same results as the coarse-error pass
// followed by the interpolation phase.
constexpr int kBPX = 16;
bool batch_ptile_fits(const BSeg &g);
unsigned batch_ptile_count(const BSeg &g, int zi);
void launch_batch_ptile(hipStream_t s, const BSeg *segs, int nseg, unsigned ntiles, int zi,
                        int phi0);

}  // namespace pfc
