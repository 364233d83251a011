/*
 * CPU oracle for the second-order convex-splitting PFC scheme and its FAS
 * multigrid solve.  TEST INFRASTRUCTURE ONLY: nothing in the product path may
 * link, load or call this file; only the tests, the package's smoke check and
 * the benchmark's CPU-baseline leg do.
 *
 * Plain FP64 C, written from the paper (Dong, Feng, Wang, Wise, Zhang,
 * arXiv:1611.06288):
 *   - Section 2: cell-centred periodic grid, 7-point discrete Laplacian,
 *     face differences D_x and the discrete energy F_h (PFC energy-discrete-1);
 *   - Section 3, scheme (1.10), in the form of Section 5: operator N
 *     (scheme-PFC-o1..o3) and source S (scheme-PFC-s1..s3), with mobility
 *     M = 1 or a variable mobility M(A phi*) on the cell faces (the *_m
 *     functions);
 *   - Section 1, the first-order convex splitting of the energy (convex part
 *     implicit, concave part -|grad phi|^2 explicit), as a second scheme on
 *     the same solver (the *_fo functions);
 *   - Section 5, Algorithm "Nonlinear Multigrid Method (FAS)": nonlinear
 *     red-black Gauss-Seidel smoothing with a pointwise 3x3 solve, residual,
 *     coarsening, coarse solve, correction.
 *
 * Readings where the paper is silent (also listed in the design notes):
 *   - red-black colour = (i+j+k) mod 2 with 0-based indices, colour 0 first;
 *   - restriction = mean of the 8 children; prolongation = cell-centred
 *     trilinear (weights 3/4, 1/4 per axis), both periodic;
 *   - hierarchy: halve n while n is even and n/2 >= 3; the coarsest level
 *     (n = 3 or 4) is solved by Newton's method on the full 3 n^3 system with a
 *     dense LU factorisation with partial pivoting;
 *   - the while loop of the algorithm runs at the finest level only; the
 *     residual max-norm over the three components is tested before each cycle;
 *   - local linearisation of the cubic term: Newton (default) or the paper's
 *     Picard form;
 *   - variable mobility: M(v) = max(m_min, m0 + m1 v + m2 v^2) (the paper
 *     leaves M open); its argument on a face is the face average A phi* of
 *     phi* = 3/2 phi^kappa - 1/2 phi^{kappa-1} (the system of Section 5; the
 *     smoothing formulas there print 1/2 weights, read as a misprint); coarse
 *     levels take phi* by the 8-child mean and evaluate M on their own faces.
 *
 * Loops are plain and independent within a red-black colour, so OpenMP
 * "parallel for" is used on the outer z loop where iterations are independent.
 * Reductions that sum are done per z-plane, then serially, so results do not
 * depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 2
#define ORC_NONFINITE 3
#define ORC_INVALID 1

/* ---------------------------------------------------------------- grid --- */

static inline int wrap(int i, int n) { return ((i % n) + n) % n; }

static inline size_t at(int n, int i, int j, int k)
{
    return ((size_t)wrap(k, n) * (size_t)n + (size_t)wrap(j, n)) * (size_t)n + (size_t)wrap(i, n);
}

static inline size_t npts(int n) { return (size_t)n * (size_t)n * (size_t)n; }

/* Sum of the six face neighbours of (i,j,k). */
static inline double nbr_sum(int n, const double *v, int i, int j, int k)
{
    return v[at(n, i + 1, j, k)] + v[at(n, i - 1, j, k)]
         + v[at(n, i, j + 1, k)] + v[at(n, i, j - 1, k)]
         + v[at(n, i, j, k + 1)] + v[at(n, i, j, k - 1)];
}

/* Section 2: Delta_h v = (sum of 6 neighbours - 6 v) / h^2, periodic. */
static inline double lap_at(int n, double h, const double *v, int i, int j, int k)
{
    return (nbr_sum(n, v, i, j, k) - 6.0 * v[at(n, i, j, k)]) / (h * h);
}

void orc_laplacian(int n, double h, const double *v, double *out)
{
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                out[at(n, i, j, k)] = lap_at(n, h, v, i, j, k);
}

/* Cubic term of the chemical potential, second-order form of Section 5:
 * g(phi; a) = 1/4 (phi + a)(phi^2 + a^2), a = phi^kappa. */
static inline double g_cubic(double phi, double a) { return 0.25 * (phi + a) * (phi * phi + a * a); }
static inline double g_cubic_dphi(double phi, double a) { return 0.25 * (3.0 * phi * phi + 2.0 * phi * a + a * a); }

/* ------------------------------------------------------- operator N, S --- */

/* u = [phi | mu | omega], each n^3.  out = N(u) (scheme-PFC-o1..o3, M = 1):
 *   N1 = phi - tau Delta_h mu
 *   N2 = mu - g(phi; phk) - (1-eps)/2 phi - Delta_h omega
 *   N3 = omega - 1/2 Delta_h phi                                          */
void orc_apply_N(int n, double h, double eps, double tau,
                 const double *u, const double *phk, double *out)
{
    const size_t P = npts(n);
    const double *phi = u, *mu = u + P, *om = u + 2 * P;
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t p = at(n, i, j, k);
                out[p] = phi[p] - tau * lap_at(n, h, mu, i, j, k);
                out[P + p] = mu[p] - g_cubic(phi[p], phk[p]) - 0.5 * (1.0 - eps) * phi[p]
                             - lap_at(n, h, om, i, j, k);
                out[2 * P + p] = om[p] - 0.5 * lap_at(n, h, phi, i, j, k);
            }
}

/* Source (scheme-PFC-s1..s3):
 *   S1 = phk,  S2 = (1-eps)/2 phk + 3 Delta_h phk - Delta_h phkm1,
 *   S3 = 1/2 Delta_h phk.                                                 */
void orc_source(int n, double h, double eps, const double *phk, const double *phkm1, double *f)
{
    const size_t P = npts(n);
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t p = at(n, i, j, k);
                double lk = lap_at(n, h, phk, i, j, k);
                double lkm1 = lap_at(n, h, phkm1, i, j, k);
                f[p] = phk[p];
                f[P + p] = 0.5 * (1.0 - eps) * phk[p] + 3.0 * lk - lkm1;
                f[2 * P + p] = 0.5 * lk;
            }
}

/* r = f - N(u); returns max |r| over the three components (NaN-propagating).
 * r may be NULL. */
double orc_residual(int n, double h, double eps, double tau, const double *u,
                    const double *f, const double *phk, double *r)
{
    const size_t P = npts(n);
    double *Nu = (double *)malloc(3 * P * sizeof(double));
    orc_apply_N(n, h, eps, tau, u, phk, Nu);
    double m = 0.0;
    int bad = 0;
    for (size_t p = 0; p < 3 * P; ++p) {
        double d = f[p] - Nu[p];
        if (r) r[p] = d;
        if (!isfinite(d)) bad = 1;
        if (fabs(d) > m) m = fabs(d);
    }
    free(Nu);
    return bad ? NAN : m;
}

/* ------------------------------------------------ pointwise 3x3 solve --- */

/* Solves, at one point of a level with spacing h, the three equations of N(u) = f
 * with the six neighbours held fixed and the cubic term linearised about the
 * point's current phi (Section 5, smoothing scheme):
 *     phi + a mu            = r1,   a = 6 tau / h^2
 *    -c phi + mu + b omega  = r2,   b = 6 / h^2
 *     d phi + omega         = r3,   d = 3 / h^2
 * Newton: c = g_phi(phi_n) + (1-eps)/2, r2 includes g(phi_n) - g_phi(phi_n) phi_n.
 * Picard (the paper's form): c = 1/4(phi_n^2 + phk^2) + (1-eps)/2, r2 includes
 * 1/4(phi_n^2 + phk^2) phk.  Solved by Cramer's rule. */
void orc_local_solve(double h, double eps, double tau, int picard,
                     double phin, double phk, double f1, double f2, double f3,
                     double smu, double som, double sphi,
                     double *phi_out, double *mu_out, double *om_out)
{
    const double h2 = h * h;
    const double a = 6.0 * tau / h2, b = 6.0 / h2, d = 3.0 / h2;
    double c, r2;
    if (picard) {
        double q = 0.25 * (phin * phin + phk * phk);
        c = q + 0.5 * (1.0 - eps);
        r2 = f2 + som / h2 + q * phk;
    } else {
        double gp = g_cubic_dphi(phin, phk);
        c = gp + 0.5 * (1.0 - eps);
        r2 = f2 + som / h2 + g_cubic(phin, phk) - gp * phin;
    }
    double r1 = f1 + tau * smu / h2;
    double r3 = f3 + sphi / (2.0 * h2);
    /* Cramer's rule on [[1, a, 0], [-c, 1, b], [d, 0, 1]] (phi, mu, omega). */
    double det = 1.0 + a * c + a * b * d;
    double phi = (r1 - a * r2 + a * b * r3) / det;
    double mu = r2 + c * phi - b * (r3 - d * phi);
    double om = r3 - d * phi;
    *phi_out = phi;
    *mu_out = mu;
    *om_out = om;
}

/* One red-black half-sweep of colour `colour` ((i+j+k) mod 2), in place. */
void orc_smooth_half(int n, double h, double eps, double tau, int picard, int colour,
                     double *u, const double *f, const double *phk)
{
    const size_t P = npts(n);
    double *phi = u, *mu = u + P, *om = u + 2 * P;
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                if (((i + j + k) & 1) != colour) continue;
                size_t p = at(n, i, j, k);
                double np_, nm_, no_;
                orc_local_solve(h, eps, tau, picard, phi[p], phk[p], f[p], f[P + p], f[2 * P + p],
                                nbr_sum(n, mu, i, j, k), nbr_sum(n, om, i, j, k),
                                nbr_sum(n, phi, i, j, k), &np_, &nm_, &no_);
                phi[p] = np_;
                mu[p] = nm_;
                om[p] = no_;
            }
}

void orc_sweep(int n, double h, double eps, double tau, int picard,
               double *u, const double *f, const double *phk)
{
    orc_smooth_half(n, h, eps, tau, picard, 0, u, f, phk);
    orc_smooth_half(n, h, eps, tau, picard, 1, u, f, phk);
}

/* ------------------------------------ first-order convex splitting --- */

/* The first-order convex-splitting scheme: the energy (energy-PFC) splits
 * into the convex part 1/4 phi^4 + (1-eps)/2 phi^2 + 1/2 (Delta phi)^2, taken
 * at the new time level, and the concave part -|grad phi|^2, taken at the old
 * one (Section 1):
 *   phi^{k+1} - phi^k = tau Delta_h mu,
 *   mu = (phi^{k+1})^3 + (1-eps) phi^{k+1} + 2 Delta_h phi^k + Delta_h omega,
 *   omega = Delta_h phi^{k+1}.
 * As N(u) = S with u = (phi^{k+1}, mu, omega):
 *   N1 = phi - tau Delta_h mu,                       S1 = phi^k,
 *   N2 = mu - phi^3 - (1-eps) phi - Delta_h omega,   S2 = 2 Delta_h phi^k,
 *   N3 = omega - Delta_h phi,                        S3 = 0.              */
void orc_apply_N_fo(int n, double h, double eps, double tau, const double *u, double *out)
{
    const size_t P = npts(n);
    const double *phi = u, *mu = u + P, *om = u + 2 * P;
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t p = at(n, i, j, k);
                out[p] = phi[p] - tau * lap_at(n, h, mu, i, j, k);
                out[P + p] = mu[p] - phi[p] * phi[p] * phi[p] - (1.0 - eps) * phi[p]
                             - lap_at(n, h, om, i, j, k);
                out[2 * P + p] = om[p] - lap_at(n, h, phi, i, j, k);
            }
}

void orc_source_fo(int n, double h, const double *phk, double *f)
{
    const size_t P = npts(n);
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t p = at(n, i, j, k);
                f[p] = phk[p];
                f[P + p] = 2.0 * lap_at(n, h, phk, i, j, k);
                f[2 * P + p] = 0.0;
            }
}

double orc_residual_fo(int n, double h, double eps, double tau, const double *u, const double *f,
                       double *r)
{
    const size_t P = npts(n);
    double *Nu = (double *)malloc(3 * P * sizeof(double));
    orc_apply_N_fo(n, h, eps, tau, u, Nu);
    double m = 0.0;
    int bad = 0;
    for (size_t p = 0; p < 3 * P; ++p) {
        double d = f[p] - Nu[p];
        if (r) r[p] = d;
        if (!isfinite(d)) bad = 1;
        if (fabs(d) > m) m = fabs(d);
    }
    free(Nu);
    return bad ? NAN : m;
}

/* Pointwise solve of the first-order system with the neighbours fixed:
 *     phi + a mu            = r1,   a = 6 tau / h^2
 *    -c phi + mu + b omega  = r2,   b = 6 / h^2
 *     d phi + omega         = r3,   d = 6 / h^2
 * Newton: c = 3 phi_n^2 + (1-eps), r2 includes phi_n^3 - 3 phi_n^2 phi_n;
 * Picard: phi^3 taken as phi_n^2 phi, c = phi_n^2 + (1-eps). */
void orc_local_solve_fo(double h, double eps, double tau, int picard, double phin, double f1,
                        double f2, double f3, double smu, double som, double sphi,
                        double *phi_out, double *mu_out, double *om_out)
{
    const double h2 = h * h;
    const double a = 6.0 * tau / h2, b = 6.0 / h2, d = 6.0 / h2;
    double c, r2;
    if (picard) {
        c = phin * phin + (1.0 - eps);
        r2 = f2 + som / h2;
    } else {
        double gp = 3.0 * phin * phin;
        c = gp + (1.0 - eps);
        r2 = f2 + som / h2 + phin * phin * phin - gp * phin;
    }
    double r1 = f1 + tau * smu / h2;
    double r3 = f3 + sphi / h2;
    double det = 1.0 + a * c + a * b * d;
    double phi = (r1 - a * r2 + a * b * r3) / det;
    *phi_out = phi;
    *om_out = r3 - d * phi;
    *mu_out = r2 + c * phi - b * (r3 - d * phi);
}

void orc_smooth_half_fo(int n, double h, double eps, double tau, int picard, int colour,
                        double *u, const double *f)
{
    const size_t P = npts(n);
    double *phi = u, *mu = u + P, *om = u + 2 * P;
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                if (((i + j + k) & 1) != colour) continue;
                size_t p = at(n, i, j, k);
                double np_, nm_, no_;
                orc_local_solve_fo(h, eps, tau, picard, phi[p], f[p], f[P + p], f[2 * P + p],
                                   nbr_sum(n, mu, i, j, k), nbr_sum(n, om, i, j, k),
                                   nbr_sum(n, phi, i, j, k), &np_, &nm_, &no_);
                phi[p] = np_;
                mu[p] = nm_;
                om[p] = no_;
            }
}

/* ------------------------------------------------- variable mobility --- */

typedef struct {
    double m0, m1, m2, mmin;
} orc_mobility;

static inline double mob_eval(const orc_mobility *mb, double v)
{
    double m = mb->m0 + mb->m1 * v + mb->m2 * v * v;
    return m > mb->mmin ? m : mb->mmin;
}

/* Mobility on the face between cells p and q: M(A phi*) = M((phs_p + phs_q)/2). */
static inline double face_mob(const orc_mobility *mb, const double *phs, size_t p, size_t q)
{
    return mob_eval(mb, 0.5 * (phs[p] + phs[q]));
}

/* The six face neighbours of (i,j,k) in the order +x, -x, +y, -y, +z, -z. */
static inline void nbrs(int n, int i, int j, int k, size_t q[6])
{
    q[0] = at(n, i + 1, j, k); q[1] = at(n, i - 1, j, k);
    q[2] = at(n, i, j + 1, k); q[3] = at(n, i, j - 1, k);
    q[4] = at(n, i, j, k + 1); q[5] = at(n, i, j, k - 1);
}

/* Variable-coefficient Laplacian d_x(M D_x v) + d_y(M D_y v) + d_z(M D_z v)
 * at (i,j,k): sum over the six faces of M_face (v_nbr - v) / h^2. */
static inline double lapm_at(int n, double h, const double *v, const double *phs,
                             const orc_mobility *mb, int i, int j, int k)
{
    size_t q[6], p = at(n, i, j, k);
    nbrs(n, i, j, k, q);
    double s = 0.0;
    for (int f = 0; f < 6; ++f) s += face_mob(mb, phs, p, q[f]) * (v[q[f]] - v[p]);
    return s / (h * h);
}

/* N(u) with variable mobility: N1 = phi - tau d(M D mu); N2, N3 as orc_apply_N. */
void orc_apply_N_m(int n, double h, double eps, double tau, const double *u, const double *phk,
                   const double *phs, double m0, double m1, double m2, double mmin, double *out)
{
    const orc_mobility mb = {m0, m1, m2, mmin};
    const size_t P = npts(n);
    const double *phi = u, *mu = u + P, *om = u + 2 * P;
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t p = at(n, i, j, k);
                out[p] = phi[p] - tau * lapm_at(n, h, mu, phs, &mb, i, j, k);
                out[P + p] = mu[p] - g_cubic(phi[p], phk[p]) - 0.5 * (1.0 - eps) * phi[p]
                             - lap_at(n, h, om, i, j, k);
                out[2 * P + p] = om[p] - 0.5 * lap_at(n, h, phi, i, j, k);
            }
}

double orc_residual_m(int n, double h, double eps, double tau, const double *u, const double *f,
                      const double *phk, const double *phs, double m0, double m1, double m2,
                      double mmin, double *r)
{
    const size_t P = npts(n);
    double *Nu = (double *)malloc(3 * P * sizeof(double));
    orc_apply_N_m(n, h, eps, tau, u, phk, phs, m0, m1, m2, mmin, Nu);
    double m = 0.0;
    int bad = 0;
    for (size_t p = 0; p < 3 * P; ++p) {
        double d = f[p] - Nu[p];
        if (r) r[p] = d;
        if (!isfinite(d)) bad = 1;
        if (fabs(d) > m) m = fabs(d);
    }
    free(Nu);
    return bad ? NAN : m;
}

/* Pointwise 3x3 solve with variable mobility: as orc_local_solve with the
 * first equation phi + a mu = r1, a = tau msum / h^2, r1 = f1 + tau smu / h^2,
 * where msum is the sum of the six face mobilities and smu the sum of
 * M_face mu_nbr. */
void orc_local_solve_m(double h, double eps, double tau, int picard, double phin, double phk,
                       double f1, double f2, double f3, double msum, double smu, double som,
                       double sphi, double *phi_out, double *mu_out, double *om_out)
{
    const double h2 = h * h;
    const double a = msum * tau / h2, b = 6.0 / h2, d = 3.0 / h2;
    double c, r2;
    if (picard) {
        double q = 0.25 * (phin * phin + phk * phk);
        c = q + 0.5 * (1.0 - eps);
        r2 = f2 + som / h2 + q * phk;
    } else {
        double gp = g_cubic_dphi(phin, phk);
        c = gp + 0.5 * (1.0 - eps);
        r2 = f2 + som / h2 + g_cubic(phin, phk) - gp * phin;
    }
    double r1 = f1 + tau * smu / h2;
    double r3 = f3 + sphi / (2.0 * h2);
    double det = 1.0 + a * c + a * b * d;
    double phi = (r1 - a * r2 + a * b * r3) / det;
    *phi_out = phi;
    *mu_out = r2 + c * phi - b * (r3 - d * phi);
    *om_out = r3 - d * phi;
}

void orc_smooth_half_m(int n, double h, double eps, double tau, int picard, int colour, double *u,
                       const double *f, const double *phk, const double *phs, double m0,
                       double m1, double m2, double mmin)
{
    const orc_mobility mb = {m0, m1, m2, mmin};
    const size_t P = npts(n);
    double *phi = u, *mu = u + P, *om = u + 2 * P;
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                if (((i + j + k) & 1) != colour) continue;
                size_t p = at(n, i, j, k), q[6];
                nbrs(n, i, j, k, q);
                double msum = 0.0, smu = 0.0;
                for (int f2 = 0; f2 < 6; ++f2) {
                    double mf = face_mob(&mb, phs, p, q[f2]);
                    msum += mf;
                    smu += mf * mu[q[f2]];
                }
                double np_, nm_, no_;
                orc_local_solve_m(h, eps, tau, picard, phi[p], phk[p], f[p], f[P + p], f[2 * P + p],
                                  msum, smu, nbr_sum(n, om, i, j, k), nbr_sum(n, phi, i, j, k),
                                  &np_, &nm_, &no_);
                phi[p] = np_;
                mu[p] = nm_;
                om[p] = no_;
            }
}

/* ------------------------------------------------------------ transfers --- */

/* Coarsening: coarse cell = mean of its 8 fine children.  nf = fine size. */
void orc_restrict(int nf, const double *fine, double *coarse)
{
    int nc = nf / 2;
#pragma omp parallel for
    for (int K = 0; K < nc; ++K)
        for (int J = 0; J < nc; ++J)
            for (int I = 0; I < nc; ++I) {
                double s = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            s += fine[at(nf, 2 * I + a, 2 * J + b, 2 * K + c)];
                coarse[at(nc, I, J, K)] = s / 8.0;
            }
}

/* Interpolation: fine += P e, with P cell-centred trilinear.  Along one axis
 * the fine cell 2I takes 3/4 e_I + 1/4 e_{I-1} and 2I+1 takes
 * 3/4 e_I + 1/4 e_{I+1}; the 3D weights are products.  nc = coarse size. */
void orc_prolong_add(int nc, const double *ec, double *fine)
{
    int nf = 2 * nc;
#pragma omp parallel for
    for (int k = 0; k < nf; ++k)
        for (int j = 0; j < nf; ++j)
            for (int i = 0; i < nf; ++i) {
                int I = i / 2, J = j / 2, K = k / 2;
                int si = (i % 2 == 0) ? -1 : 1;
                int sj = (j % 2 == 0) ? -1 : 1;
                int sk = (k % 2 == 0) ? -1 : 1;
                double v = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
                            v += w * ec[at(nc, I + a * si, J + b * sj, K + c * sk)];
                        }
                fine[at(nf, i, j, k)] += v;
            }
}

/* ------------------------------------------------------- coarsest solve --- */

/* Dense LU with partial pivoting, in place, then solve A x = b (b overwritten).
 * Returns 0 on success, 1 on a zero pivot. */
static int dense_solve(int m, double *A, double *b)
{
    for (int c = 0; c < m; ++c) {
        int piv = c;
        double best = fabs(A[(size_t)c * m + c]);
        for (int r = c + 1; r < m; ++r) {
            double v = fabs(A[(size_t)r * m + c]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return 1;
        if (piv != c) {
            for (int q = 0; q < m; ++q) {
                double t = A[(size_t)c * m + q];
                A[(size_t)c * m + q] = A[(size_t)piv * m + q];
                A[(size_t)piv * m + q] = t;
            }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < m; ++r) {
            double l = A[(size_t)r * m + c] / A[(size_t)c * m + c];
            A[(size_t)r * m + c] = l;
            for (int q = c + 1; q < m; ++q) A[(size_t)r * m + q] -= l * A[(size_t)c * m + q];
            b[r] -= l * b[c];
        }
    }
    for (int r = m - 1; r >= 0; --r) {
        double s = b[r];
        for (int q = r + 1; q < m; ++q) s -= A[(size_t)r * m + q] * b[q];
        b[r] = s / A[(size_t)r * m + r];
    }
    return 0;
}

/* Adds coef * Delta_h (as a matrix acting on block column `cb`) into the
 * block row `rb` of the 3P x 3P matrix J. */
static void add_lap_block(int n, double h, double coef, double *J, int rb, int cb)
{
    const int P = (int)npts(n), m = 3 * P;
    const double w = coef / (h * h);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int row = rb * P + (int)at(n, i, j, k);
                int nb[6] = {(int)at(n, i + 1, j, k), (int)at(n, i - 1, j, k),
                             (int)at(n, i, j + 1, k), (int)at(n, i, j - 1, k),
                             (int)at(n, i, j, k + 1), (int)at(n, i, j, k - 1)};
                for (int q = 0; q < 6; ++q) J[(size_t)row * m + cb * P + nb[q]] += w;
                J[(size_t)row * m + cb * P + (int)at(n, i, j, k)] -= 6.0 * w;
            }
}

/* Newton's method with a dense Jacobian on the full system N(u) = f at the
 * coarsest level.  Stops when the max-norm of the Newton update is at most
 * 1e-14 * max(1, |u|_inf), or after 30 iterations.  Returns the number of
 * iterations, or -1 on a singular Jacobian. */
int orc_coarse_solve(int n, double h, double eps, double tau, double *u,
                     const double *f, const double *phk)
{
    const int P = (int)npts(n), m = 3 * P;
    double *J = (double *)malloc((size_t)m * m * sizeof(double));
    double *r = (double *)malloc((size_t)m * sizeof(double));
    int it;
    for (it = 1; it <= 30; ++it) {
        orc_residual(n, h, eps, tau, u, f, phk, r);
        memset(J, 0, (size_t)m * m * sizeof(double));
        for (int p = 0; p < m; ++p) J[(size_t)p * m + p] = 1.0;      /* identity blocks */
        add_lap_block(n, h, -tau, J, 0, 1);                           /* dN1/dmu  = -tau Lap */
        for (int p = 0; p < P; ++p)                                   /* dN2/dphi = -D */
            J[(size_t)(P + p) * m + p] -= g_cubic_dphi(u[p], phk[p]) + 0.5 * (1.0 - eps);
        add_lap_block(n, h, -1.0, J, 1, 2);                           /* dN2/domega = -Lap */
        add_lap_block(n, h, -0.5, J, 2, 0);                           /* dN3/dphi = -Lap/2 */
        if (dense_solve(m, J, r)) { it = -1; break; }
        double dmax = 0.0, umax = 0.0;
        for (int p = 0; p < m; ++p) {
            u[p] += r[p];
            if (fabs(r[p]) > dmax) dmax = fabs(r[p]);
            if (fabs(u[p]) > umax) umax = fabs(u[p]);
        }
        if (!(dmax == dmax)) { it = -1; break; }
        if (dmax <= 1e-14 * (umax > 1.0 ? umax : 1.0)) break;
    }
    if (it > 30) it = 30;
    free(J);
    free(r);
    return it;
}

/* The coarsest-level Newton solve of the first-order system. */
int orc_coarse_solve_fo(int n, double h, double eps, double tau, double *u, const double *f)
{
    const int P = (int)npts(n), m = 3 * P;
    double *J = (double *)malloc((size_t)m * m * sizeof(double));
    double *r = (double *)malloc((size_t)m * sizeof(double));
    int it;
    for (it = 1; it <= 30; ++it) {
        orc_residual_fo(n, h, eps, tau, u, f, r);
        memset(J, 0, (size_t)m * m * sizeof(double));
        for (int p = 0; p < m; ++p) J[(size_t)p * m + p] = 1.0;
        add_lap_block(n, h, -tau, J, 0, 1);                           /* dN1/dmu  = -tau Lap */
        for (int p = 0; p < P; ++p)                                   /* dN2/dphi */
            J[(size_t)(P + p) * m + p] -= 3.0 * u[p] * u[p] + (1.0 - eps);
        add_lap_block(n, h, -1.0, J, 1, 2);                           /* dN2/domega = -Lap */
        add_lap_block(n, h, -1.0, J, 2, 0);                           /* dN3/dphi = -Lap */
        if (dense_solve(m, J, r)) { it = -1; break; }
        double dmax = 0.0, umax = 0.0;
        for (int p = 0; p < m; ++p) {
            u[p] += r[p];
            if (fabs(r[p]) > dmax) dmax = fabs(r[p]);
            if (fabs(u[p]) > umax) umax = fabs(u[p]);
        }
        if (!(dmax == dmax)) { it = -1; break; }
        if (dmax <= 1e-14 * (umax > 1.0 ? umax : 1.0)) break;
    }
    if (it > 30) it = 30;
    free(J);
    free(r);
    return it;
}

/* The coarsest-level Newton solve with variable mobility: dN1/dmu is
 * -tau times the variable-coefficient Laplacian. */
int orc_coarse_solve_m(int n, double h, double eps, double tau, double *u, const double *f,
                       const double *phk, const double *phs, double m0, double m1, double m2,
                       double mmin)
{
    const orc_mobility mb = {m0, m1, m2, mmin};
    const int P = (int)npts(n), m = 3 * P;
    double *J = (double *)malloc((size_t)m * m * sizeof(double));
    double *r = (double *)malloc((size_t)m * sizeof(double));
    int it;
    for (it = 1; it <= 30; ++it) {
        orc_residual_m(n, h, eps, tau, u, f, phk, phs, m0, m1, m2, mmin, r);
        memset(J, 0, (size_t)m * m * sizeof(double));
        for (int p = 0; p < m; ++p) J[(size_t)p * m + p] = 1.0;
        const double w = -tau / (h * h);                              /* dN1/dmu = -tau d(M D) */
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    size_t p = at(n, i, j, k), q[6];
                    nbrs(n, i, j, k, q);
                    for (int f2 = 0; f2 < 6; ++f2) {
                        double mf = face_mob(&mb, phs, p, q[f2]);
                        J[p * (size_t)m + P + q[f2]] += w * mf;
                        J[p * (size_t)m + P + p] -= w * mf;
                    }
                }
        for (int p = 0; p < P; ++p)
            J[(size_t)(P + p) * m + p] -= g_cubic_dphi(u[p], phk[p]) + 0.5 * (1.0 - eps);
        add_lap_block(n, h, -1.0, J, 1, 2);
        add_lap_block(n, h, -0.5, J, 2, 0);
        if (dense_solve(m, J, r)) { it = -1; break; }
        double dmax = 0.0, umax = 0.0;
        for (int p = 0; p < m; ++p) {
            u[p] += r[p];
            if (fabs(r[p]) > dmax) dmax = fabs(r[p]);
            if (fabs(u[p]) > umax) umax = fabs(u[p]);
        }
        if (!(dmax == dmax)) { it = -1; break; }
        if (dmax <= 1e-14 * (umax > 1.0 ? umax : 1.0)) break;
    }
    if (it > 30) it = 30;
    free(J);
    free(r);
    return it;
}

/* --------------------------------------------------------------- solver --- */

typedef struct {
    int n;            /* cells per axis on this level */
    double h;
    double *u, *f, *phk, *ubar, *r;
    double *phs;      /* phi* (variable mobility only) */
} orc_level;

typedef struct {
    int nlev;
    orc_level lev[24];
    double eps, tau, tol;
    int nu1, nu2, max_cycles, fcycle, picard;
    int coarse_iters_last;
    int mob_on;
    orc_mobility mob;
    int first_order;  /* the first-order convex-splitting scheme */
} orc_solver;

/* Level sizes: halve while even and the half is at least 3. */
int orc_num_levels(int n)
{
    int L = 1;
    while (n % 2 == 0 && n / 2 >= 3) { n /= 2; ++L; }
    return L;
}

orc_solver *orc_create(int n, double L, double eps, double tau, double tol,
                       int nu1, int nu2, int max_cycles, int fcycle, int picard)
{
    if (n < 4 || (n % 2) || L <= 0 || tau <= 0 || tol < 0 || nu1 < 0 || nu2 < 0) return NULL;
    int nl = orc_num_levels(n);
    int nc = n >> (nl - 1);
    if (nc > 4) return NULL;
    orc_solver *s = (orc_solver *)calloc(1, sizeof(orc_solver));
    s->nlev = nl;
    s->eps = eps; s->tau = tau; s->tol = tol;
    s->nu1 = nu1; s->nu2 = nu2; s->max_cycles = max_cycles;
    s->fcycle = fcycle; s->picard = picard;
    int m = n;
    for (int l = 0; l < nl; ++l) {
        size_t P = npts(m);
        s->lev[l].n = m;
        s->lev[l].h = L / m;
        s->lev[l].u = (double *)calloc(3 * P, sizeof(double));
        s->lev[l].f = (double *)calloc(3 * P, sizeof(double));
        s->lev[l].phk = (double *)calloc(P, sizeof(double));
        s->lev[l].ubar = (double *)calloc(3 * P, sizeof(double));
        s->lev[l].r = (double *)calloc(3 * P, sizeof(double));
        m /= 2;
    }
    return s;
}

void orc_destroy(orc_solver *s)
{
    if (!s) return;
    for (int l = 0; l < s->nlev; ++l) {
        free(s->lev[l].u); free(s->lev[l].f); free(s->lev[l].phk);
        free(s->lev[l].ubar); free(s->lev[l].r); free(s->lev[l].phs);
    }
    free(s);
}

/* Switches the solver to variable mobility M(v) = max(mmin, m0 + m1 v + m2 v^2). */
void orc_set_mobility(orc_solver *s, double m0, double m1, double m2, double mmin)
{
    s->mob_on = 1;
    s->mob.m0 = m0; s->mob.m1 = m1; s->mob.m2 = m2; s->mob.mmin = mmin;
    for (int l = 0; l < s->nlev; ++l)
        if (!s->lev[l].phs) s->lev[l].phs = (double *)calloc(npts(s->lev[l].n), sizeof(double));
}

/* Switches the solver to the first-order convex-splitting scheme (M = 1 only).
 * Returns 0, or -1 if variable mobility is on. */
int orc_set_first_order(orc_solver *s)
{
    if (s->mob_on) return -1;
    s->first_order = 1;
    return 0;
}

static void sweep_lev(const orc_solver *s, const orc_level *A)
{
    if (s->first_order) {
        orc_smooth_half_fo(A->n, A->h, s->eps, s->tau, s->picard, 0, A->u, A->f);
        orc_smooth_half_fo(A->n, A->h, s->eps, s->tau, s->picard, 1, A->u, A->f);
    } else if (s->mob_on) {
        const orc_mobility *m = &s->mob;
        orc_smooth_half_m(A->n, A->h, s->eps, s->tau, s->picard, 0, A->u, A->f, A->phk, A->phs,
                          m->m0, m->m1, m->m2, m->mmin);
        orc_smooth_half_m(A->n, A->h, s->eps, s->tau, s->picard, 1, A->u, A->f, A->phk, A->phs,
                          m->m0, m->m1, m->m2, m->mmin);
    } else {
        orc_sweep(A->n, A->h, s->eps, s->tau, s->picard, A->u, A->f, A->phk);
    }
}

static double resid_lev(const orc_solver *s, const orc_level *A, double *r)
{
    const orc_mobility *m = &s->mob;
    if (s->first_order) return orc_residual_fo(A->n, A->h, s->eps, s->tau, A->u, A->f, r);
    return s->mob_on ? orc_residual_m(A->n, A->h, s->eps, s->tau, A->u, A->f, A->phk, A->phs,
                                      m->m0, m->m1, m->m2, m->mmin, r)
                     : orc_residual(A->n, A->h, s->eps, s->tau, A->u, A->f, A->phk, r);
}

int orc_level_n(const orc_solver *s, int l) { return s->lev[l].n; }
int orc_levels(const orc_solver *s) { return s->nlev; }

static void restrict3(int nf, const double *fine, double *coarse)
{
    size_t Pf = npts(nf), Pc = npts(nf / 2);
    for (int c = 0; c < 3; ++c) orc_restrict(nf, fine + c * Pf, coarse + c * Pc);
}

static void cycle(orc_solver *s, int l, int fcycle)
{
    orc_level *A = &s->lev[l];
    const double eps = s->eps, tau = s->tau;
    const orc_mobility *m = &s->mob;
    if (l == s->nlev - 1) {
        s->coarse_iters_last =
            s->first_order ? orc_coarse_solve_fo(A->n, A->h, eps, tau, A->u, A->f)
            : s->mob_on ? orc_coarse_solve_m(A->n, A->h, eps, tau, A->u, A->f, A->phk, A->phs, m->m0,
                                           m->m1, m->m2, m->mmin)
                      : orc_coarse_solve(A->n, A->h, eps, tau, A->u, A->f, A->phk);
        return;
    }
    orc_level *B = &s->lev[l + 1];
    size_t Pc = npts(B->n);
    for (int q = 0; q < s->nu1; ++q) sweep_lev(s, A);
    /* residual, coarsening of residual and iterate */
    resid_lev(s, A, A->r);
    restrict3(A->n, A->u, B->ubar);
    restrict3(A->n, A->r, B->f);               /* holds I r for now */
    /* coarse right-hand side f_c = N_c(I u) + I r */
    double *Nc = (double *)malloc(3 * Pc * sizeof(double));
    if (s->first_order)
        orc_apply_N_fo(B->n, B->h, eps, tau, B->ubar, Nc);
    else if (s->mob_on)
        orc_apply_N_m(B->n, B->h, eps, tau, B->ubar, B->phk, B->phs, m->m0, m->m1, m->m2, m->mmin, Nc);
    else
        orc_apply_N(B->n, B->h, eps, tau, B->ubar, B->phk, Nc);
    for (size_t p = 0; p < 3 * Pc; ++p) B->f[p] += Nc[p];
    free(Nc);
    memcpy(B->u, B->ubar, 3 * Pc * sizeof(double));
    cycle(s, l + 1, fcycle);
    if (fcycle) cycle(s, l + 1, 0);
    /* correction u += P (v - I u) */
    double *e = (double *)malloc(3 * Pc * sizeof(double));
    for (size_t p = 0; p < 3 * Pc; ++p) e[p] = B->u[p] - B->ubar[p];
    size_t Pf = npts(A->n);
    for (int c = 0; c < 3; ++c) orc_prolong_add(B->n, e + c * Pc, A->u + c * Pf);
    free(e);
    for (int q = 0; q < s->nu2; ++q) sweep_lev(s, A);
}

/* One multigrid cycle at the finest level on a caller-supplied iterate u,
 * right-hand side f and phk (phi^kappa on the finest grid).  Returns the
 * residual max-norm after the cycle. */
double orc_cycle(orc_solver *s, double *u, const double *f, const double *phk)
{
    orc_level *A = &s->lev[0];
    size_t P = npts(A->n);
    memcpy(A->u, u, 3 * P * sizeof(double));
    memcpy(A->f, f, 3 * P * sizeof(double));
    memcpy(A->phk, phk, P * sizeof(double));
    for (int l = 0; l + 1 < s->nlev; ++l) orc_restrict(s->lev[l].n, s->lev[l].phk, s->lev[l + 1].phk);
    cycle(s, 0, s->fcycle);
    memcpy(u, A->u, 3 * P * sizeof(double));
    return resid_lev(s, A, NULL);
}

/* orc_cycle with variable mobility: phs = phi* on the finest grid. */
double orc_cycle_m(orc_solver *s, double *u, const double *f, const double *phk, const double *phs)
{
    if (!s->mob_on) return NAN;
    orc_level *A = &s->lev[0];
    memcpy(A->phs, phs, npts(A->n) * sizeof(double));
    for (int l = 0; l + 1 < s->nlev; ++l) orc_restrict(s->lev[l].n, s->lev[l].phs, s->lev[l + 1].phs);
    return orc_cycle(s, u, f, phk);
}

/* One time step of scheme (1.10).  Inputs phkm1 = phi^{kappa-1},
 * phk = phi^kappa; in/out mu, omega (initial guess, then mu^{kappa+1/2},
 * omega^{kappa+1/2}); out phi_next.  res_hist (nullable, max_cycles+1 entries)
 * receives the residual before each cycle and after the last.  Returns a
 * status; *cycles_out receives the number of cycles. */
int orc_step(orc_solver *s, const double *phkm1, const double *phk, double *phi_next,
             double *mu, double *omega, int *cycles_out, double *res_hist)
{
    orc_level *A = &s->lev[0];
    size_t P = npts(A->n);
    if (s->first_order)
        orc_source_fo(A->n, A->h, phk, A->f);
    else
        orc_source(A->n, A->h, s->eps, phk, phkm1, A->f);
    memcpy(A->phk, phk, P * sizeof(double));
    for (int l = 0; l + 1 < s->nlev; ++l) orc_restrict(s->lev[l].n, s->lev[l].phk, s->lev[l + 1].phk);
    if (s->mob_on) {  /* phi* = 3/2 phi^kappa - 1/2 phi^{kappa-1}, on every level */
        for (size_t p = 0; p < P; ++p) A->phs[p] = 1.5 * phk[p] - 0.5 * phkm1[p];
        for (int l = 0; l + 1 < s->nlev; ++l)
            orc_restrict(s->lev[l].n, s->lev[l].phs, s->lev[l + 1].phs);
    }
    memcpy(A->u, phk, P * sizeof(double));
    memcpy(A->u + P, mu, P * sizeof(double));
    memcpy(A->u + 2 * P, omega, P * sizeof(double));
    int c = 0, status = ORC_OK;
    for (;;) {
        double rho = resid_lev(s, A, NULL);
        if (res_hist) res_hist[c] = rho;
        if (!(rho == rho) || isinf(rho)) { status = ORC_NONFINITE; break; }
        if (rho <= s->tol) break;
        if (c == s->max_cycles) { status = ORC_NOT_CONVERGED; break; }
        cycle(s, 0, s->fcycle);
        ++c;
    }
    memcpy(phi_next, A->u, P * sizeof(double));
    memcpy(mu, A->u + P, P * sizeof(double));
    memcpy(omega, A->u + 2 * P, P * sizeof(double));
    if (cycles_out) *cycles_out = c;
    return status;
}

/* First-step guess consistent with a steady state:
 * mu = phi^3 + (1-eps) phi + 2 Delta_h phi + Delta_h^2 phi, omega = Delta_h phi
 * (the chemical potential of (equation-PFC), discretised). */
void orc_initial_guess(int n, double h, double eps, const double *phi0, double *mu, double *omega)
{
    size_t P = npts(n);
    orc_laplacian(n, h, phi0, omega);
    double *l2 = (double *)malloc(P * sizeof(double));
    orc_laplacian(n, h, omega, l2);
    for (size_t p = 0; p < P; ++p)
        mu[p] = phi0[p] * phi0[p] * phi0[p] + (1.0 - eps) * phi0[p] + 2.0 * omega[p] + l2[p];
    free(l2);
}

/* --------------------------------------------------------------- energy --- */

/* Discrete energy (PFC energy-discrete-1):
 *   F_h = 1/4 |phi|_4^4 + (1-eps)/2 |phi|_2^2 - |grad_h phi|_2^2 + 1/2 |Delta_h phi|_2^2,
 * with |grad_h v|^2 = h^3 * sum over all x-, y- and z-faces of (D v)^2.
 * out[0] = F_h(phi); out[1] = F_h(phi) + 1/2 |grad_h(phi - phi_prev)|^2
 * (0 contribution if phi_prev is NULL); out[2] = h^3 sum phi (mass). */
void orc_energy(int n, double h, double eps, const double *phi, const double *phi_prev, double *out)
{
    double *plane = (double *)calloc((size_t)n * 6, sizeof(double));
#pragma omp parallel for
    for (int k = 0; k < n; ++k) {
        double s4 = 0, s2 = 0, sg = 0, sl = 0, sd = 0, sm = 0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double v = phi[at(n, i, j, k)];
                s4 += v * v * v * v;
                s2 += v * v;
                sm += v;
                double dx = (phi[at(n, i + 1, j, k)] - v) / h;
                double dy = (phi[at(n, i, j + 1, k)] - v) / h;
                double dz = (phi[at(n, i, j, k + 1)] - v) / h;
                sg += dx * dx + dy * dy + dz * dz;
                double l = lap_at(n, h, phi, i, j, k);
                sl += l * l;
                if (phi_prev) {
                    double w = v - phi_prev[at(n, i, j, k)];
                    double ex = (phi[at(n, i + 1, j, k)] - phi_prev[at(n, i + 1, j, k)] - w) / h;
                    double ey = (phi[at(n, i, j + 1, k)] - phi_prev[at(n, i, j + 1, k)] - w) / h;
                    double ez = (phi[at(n, i, j, k + 1)] - phi_prev[at(n, i, j, k + 1)] - w) / h;
                    sd += ex * ex + ey * ey + ez * ez;
                }
            }
        double *q = plane + (size_t)k * 6;
        q[0] = s4; q[1] = s2; q[2] = sg; q[3] = sl; q[4] = sd; q[5] = sm;
    }
    double t[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < n; ++k)
        for (int c = 0; c < 6; ++c) t[c] += plane[(size_t)k * 6 + c];
    free(plane);
    double h3 = h * h * h;
    double F = h3 * (0.25 * t[0] + 0.5 * (1.0 - eps) * t[1] - t[2] + 0.5 * t[3]);
    out[0] = F;
    out[1] = F + 0.5 * h3 * t[4];
    out[2] = h3 * t[5];
}

/* Number of OpenMP threads the oracle's parallel loops use. */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
