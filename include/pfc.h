/*
 * pfc.h -- C ABI of the MI355X (gfx950) solver for the second-order
 * convex-splitting finite-difference scheme of the 3D phase field crystal
 * (PFC) equation, solved by FAS nonlinear multigrid.
 *
 * Paper: Dong, Feng, Wang, Wise, Zhang, "Convergence analysis and numerical
 * implementation of a second order numerical scheme for the three-dimensional
 * phase field crystal equation" (arXiv:1611.06288).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid (Section 2): cubic periodic box of side L, n cells per axis, spacing
 *   h = L/n, cell-centred values at ((i+1/2)h, (j+1/2)h, (k+1/2)h), 0-based.
 * Field layout: one FP64 array of n^3 values, C order [k][j][i] (x fastest).
 *   A "triple" is three such arrays stored back to back, [3][n][n][n], in the
 *   order (phi, mu, omega) of the unknown u of (eqn:dis-nonlinear-system).
 * Pointers: every field pointer is a DEVICE pointer on the device that was
 *   current when the handle was created; scalars returned to the caller
 *   (norms, energies, step info) are HOST pointers.  The caller owns all
 *   field buffers; the handle owns its multigrid hierarchy and scratch.
 * Streams: all work is enqueued on the hipStream_t given at creation (NULL =
 *   the default stream).  Entry points that return host scalars synchronise
 *   that stream before returning; the others return without waiting.
 * Aliasing: inputs declared const are never written.  Outputs may not alias
 *   inputs unless stated.
 * Errors: every function returns a pfc_status and never aborts; on error the
 *   outputs are unspecified unless stated; pfc_last_error() gives a message.
 * Threading: a handle is not thread-safe; distinct handles are independent.
 */
#ifndef PFC_H
#define PFC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pfc_status;
#define PFC_OK 0
#define PFC_ERR_INVALID_ARG 1   /* bad size, parameter or NULL pointer          */
#define PFC_ERR_NOT_CONVERGED 2 /* max_cycles reached; last iterate returned     */
#define PFC_ERR_NONFINITE 3     /* residual became NaN or Inf                    */
#define PFC_ERR_HIP 4           /* a HIP runtime call failed                     */
#define PFC_ERR_OOM 5           /* device or pinned-host allocation failed       */

#define PFC_FP64 0      /* every kernel in FP64                                  */
#define PFC_MIXED 1     /* FP32 multigrid cycle inside FP64 defect correction    */

#define PFC_CYCLE_V 0
#define PFC_CYCLE_F 1

#define PFC_LIN_NEWTON 0  /* pointwise Newton linearisation of the cubic term    */
#define PFC_LIN_PICARD 1  /* the Picard linearisation written in Section 5       */

#define PFC_SCHEME_CS2 0  /* second-order convex splitting, scheme (1.10)         */
#define PFC_SCHEME_CS1 1  /* first-order convex splitting (see pfc_config)       */

#define PFC_MOBILITY_ONE 0        /* M = 1, the form the convergence theorem uses */
#define PFC_MOBILITY_QUADRATIC 1  /* variable face mobility, see pfc_config       */

/* Parameters of the problem statement (Sections 2, 3, 5 and 6): grid n^3,
 * box side L, epsilon, time step (tau in Section 3, s in Section 6), residual
 * tolerance, smoothing counts nu1/nu2 of Algorithm algorithm:FAS. */
typedef struct {
    int32_t n;          /* cells per axis; n = 2^k (k >= 2) or 3*2^k (k >= 1)  */
    int32_t nu1;        /* pre-smoothing sweeps, >= 0                          */
    int32_t nu2;        /* post-smoothing sweeps, >= 0 (nu1 + nu2 >= 1)        */
    int32_t max_cycles; /* cap on cycles per time step, >= 1                   */
    int32_t cycle;      /* PFC_CYCLE_V or PFC_CYCLE_F                          */
    int32_t lin;        /* PFC_LIN_NEWTON or PFC_LIN_PICARD                    */
    int32_t precision;  /* PFC_FP64 or PFC_MIXED                               */
    int32_t mobility;   /* PFC_MOBILITY_ONE or PFC_MOBILITY_QUADRATIC          */
    double L;           /* box side, > 0                                       */
    double eps;         /* epsilon of the PFC energy (energy-PFC)              */
    double dt;          /* time step, > 0                                      */
    double tol;         /* stop when max-norm of S - N(u) (3 components) <= tol */
    /* PFC_MOBILITY_QUADRATIC: the first equation in the flux form of Section 5,
     * phi - tau [d_x(M D_x mu) + d_y(M D_y mu) + d_z(M D_z mu)] = phi^k, with
     * M = max(mob_min, mob_m0 + mob_m1 v + mob_m2 v^2) on each face and v the
     * face average A phi* of phi* = 3/2 phi^k - 1/2 phi^{k-1} (the paper leaves
     * M's form open).  mob_min > 0.  FP64 precision only; not available to the
     * adjoint and batched forms.  Ignored with PFC_MOBILITY_ONE (M = 1). */
    double mob_m0, mob_m1, mob_m2, mob_min;
    /* PFC_SCHEME_CS2 (scheme (1.10), the default) or PFC_SCHEME_CS1: the
     * first-order convex splitting of Section 1 (convex part of the energy
     * implicit, -|grad phi|^2 explicit), in the same three-field form
     *   phi - tau Lap mu = phi^k,
     *   mu - phi^3 - (1-eps) phi - Lap omega = 2 Lap phi^k,
     *   omega - Lap phi = 0
     * (phi^{k-1} unused).  FP64, M = 1; not available to the adjoint and
     * batched forms. */
    int32_t scheme;
} pfc_config;

/* Per-step report.  res0: residual max-norm before the first cycle;
 * res_final: after the last; cycles: cycles taken (0 if the guess already
 * met the tolerance). */
typedef struct {
    int32_t cycles;
    int32_t status;
    double res0;
    double res_final;
} pfc_step_info;

typedef struct pfc_handle pfc_handle;

/* Creates a solver for one grid size.  Allocates the multigrid hierarchy
 * (levels n, n/2, ... down to 3 or 4, Section 5) on the current device.
 * stream: a hipStream_t (may be NULL).  Errors: INVALID_ARG for n not of the
 * form 2^k (k >= 2) or 3*2^k (k >= 1) or above 1024 (at 1024^3 the FP64
 * hierarchy takes about 120 GiB, the mixed form about 50 GiB more), L <= 0,
 * dt <= 0, tol < 0, nu1 or nu2 < 0, nu1+nu2 == 0, max_cycles < 1, unknown
 * enum values, Picard with MIXED, variable mobility with MIXED or with
 * mob_min <= 0, the first-order scheme with MIXED or variable mobility; OOM;
 * HIP. */
pfc_status pfc_create(const pfc_config *cfg, void *stream, pfc_handle **out);
pfc_status pfc_destroy(pfc_handle *h);
pfc_status pfc_set_stream(pfc_handle *h, void *stream);
/* Number of multigrid levels and the size n_l of level l (l = 0 finest). */
int32_t pfc_num_levels(const pfc_handle *h);
int32_t pfc_level_size(const pfc_handle *h, int32_t level);

/* First-step guess for (mu, omega) from phi0 (n^3 each):
 *   omega = Delta_h phi0,
 *   mu = phi0^3 + (1-eps) phi0 + 2 Delta_h phi0 + Delta_h^2 phi0,
 * the discrete chemical potential of (equation-PFC); with it a constant
 * phi0 is an exact fixed point of the step (zero cycles). */
pfc_status pfc_init_guess(pfc_handle *h, const double *phi0, double *mu, double *omega);

/* One time step of scheme (1.10) in the form (2nd scheme-PFC-s1..s3) with
 * mobility M = 1: given phi^{k-1} = phi_prev and phi^k = phi_cur, computes
 * phi^{k+1} = phi_next, mu^{k+1/2} and omega^{k+1/2}.  mu and omega are read
 * as the initial guess and overwritten with the result; the phi guess is
 * phi_cur.  The FAS cycle of Algorithm algorithm:FAS (V or F per the config)
 * repeats until max|S - N(u)| <= tol, tested before each cycle.  In FP64 (M = 1
 * or variable mobility) on a finest level of at least 128^3 with n a multiple
 * of 64 the test
 * after a cycle is formed inside the finest sweeps (the cycle's last
 * post-sweep and the next cycle's first pre-sweep, launched before the
 * decision and dropped when the loop stops); the norm is bitwise that of
 * pfc_residual, and so are the results.  The coarsest level's cached Newton
 * inverse carries over between steps (it is rebuilt where the chord
 * iteration stops contracting).
 * For the bootstrap step pass phi_prev == phi_cur.  phi_next must not alias
 * phi_prev or phi_cur.  info (host, nullable) receives the report.
 * Returns NOT_CONVERGED after max_cycles cycles (outputs hold the last
 * iterate, info filled) and NONFINITE if the residual is NaN/Inf.
 * Synchronises the stream (one 8-byte residual read-back per cycle). */
pfc_status pfc_step(pfc_handle *h, const double *phi_prev, const double *phi_cur,
                    double *phi_next, double *mu, double *omega, pfc_step_info *info);

/* Forgets the coarsest level's cached Newton inverse (FP64 and FP32
 * copies), so that the next coarsest solve rebuilds it.  Between calls of
 * pfc_step the cache makes a step's last bits depend on the steps before it
 * (the chord iteration starts from whichever inverse the previous solve
 * left).  After this call a step's result depends on its arguments alone:
 * checkpoint-and-recompute differentiation calls it at the start of every
 * segment, in the forward pass and again in the recompute, and so
 * reproduces the forward trajectory bit for bit.  Stream-ordered (one
 * one-block kernel, no memset, so it may be recorded into a graph); does
 * not synchronise.  INVALID_ARG for a NULL handle. */
pfc_status pfc_reset_coarse_cache(pfc_handle *h);

/* Time loop: advances (phi_prev, phi_cur) = (phi^{k-1}, phi^k) by `steps`
 * steps of pfc_step, in place: on return phi_prev and phi_cur hold the last
 * two states and mu, omega the last step's chemical potential and omega (the
 * next step's guess).  phi_prev and phi_cur must be distinct buffers (for the
 * bootstrap step copy phi^0 into both).  infos (host, nullable): `steps`
 * entries.  In FP64 precision one cycle of Algorithm algorithm:FAS and the
 * residual test before it are recorded once as a hipGraph on a stream the
 * handle owns and replayed, the loop's decisions taken by a kernel; results
 * equal those of calling pfc_step `steps` times, bit for bit (a configuration
 * whose fused sweeps would not return to their buffers over a cycle, odd
 * nu1 + nu2 at n >= 128, and the mixed form run the pfc_step loop instead).
 * Per-kernel timing is not recorded by this call.  Stops at the first step
 * that fails and returns its status (NOT_CONVERGED, NONFINITE: that step's
 * last iterate is the new phi_cur).  Synchronises once or twice per step. */
pfc_status pfc_run(pfc_handle *h, double *phi_prev, double *phi_cur, double *mu, double *omega,
                   int32_t steps, pfc_step_info *infos);

/* Exactly one FP64 multigrid cycle (Algorithm algorithm:FAS, one pass of its
 * loop body at the finest level) on a caller-supplied iterate.
 * u3: triple [3][n^3] (in/out); f3: triple, right-hand side S at the finest
 * level (scheme-PFC-s1..s3 or any other); phi_cur: phi^k, n^3 (enters N).
 * res_after (host, nullable): max|f3 - N(u3)| after the cycle. Synchronises
 * if res_after is non-NULL.  With variable mobility N uses the phi* hierarchy
 * set by pfc_set_phistar (at level 0); INVALID_ARG if none was set. */
pfc_status pfc_fas_vcycle(pfc_handle *h, double *u3, const double *f3,
                          const double *phi_cur, double *res_after);

/* Discrete energy (PFC energy-discrete-1) and mass of phi (n^3):
 *   out[0] = F_h(phi) = 1/4|phi|_4^4 + (1-eps)/2 |phi|_2^2 - |grad_h phi|_2^2
 *            + 1/2 |Delta_h phi|_2^2,
 *   out[1] = out[0] + 1/2 |grad_h(phi - phi_prev)|_2^2 (the modified energy of
 *            Proposition prop:hu09; equals out[0] if phi_prev is NULL),
 *   out[2] = h^3 sum phi.
 * out is a host array of 3 doubles.  Sums are reduced in a fixed order
 * (bitwise reproducible).  Synchronises. */
pfc_status pfc_energy(pfc_handle *h, const double *phi, const double *phi_prev, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * energies and mass as pfc_energy, for any n in [4, PFC_ENERGY_STATIC_MAX_N],
 * with no handle and no allocation.  phi (and phi_prev, nullable) are DEVICE
 * pointers to n^3 FP64 values in C order on the current device, L the box
 * edge (h = L/n), eps as in the config; out3 is a DEVICE pointer to 3
 * doubles receiving (F_h, modified energy, mass) as pfc_energy's out.
 * The per-workgroup partial sums live in a 768 KiB device array of the
 * library, one per GPU, held until the process ends; its address is looked
 * up on the first call on each device (call with the stream's device
 * current).  Every call on a GPU uses that GPU's one array: calls that
 * overlap on one GPU (other streams, other host threads) race and must be
 * ordered by the caller.  Enqueued on `stream` (NULL: the null stream);
 * does not synchronise, calls no hipMalloc/hipFree, and records only kernel
 * launches (capturable).  Results are bitwise those of pfc_energy.
 * INVALID_ARG (message in pfc_last_error(NULL)) for n outside the range,
 * L <= 0, non-finite eps or NULL phi/out3. */
#define PFC_ENERGY_STATIC_MAX_N 1024
pfc_status pfc_energy_static(int32_t n, double L, double eps, const double *phi,
                             const double *phi_prev, double *out3, void *stream);

/* Adjoint of one time step (the implicit-function theorem applied to
 * G(u; phi^k, phi^{k-1}, eps) = N(u) - S = 0 of scheme-PFC-o/s).
 * Given phi_prev = phi^{k-1}, phi_cur = phi^k, phi_next = phi^{k+1} (the
 * converged step) and gbar_next = dLoss/dphi^{k+1} (n^3 each), solves
 * J^T lambda = (gbar_next, 0, 0) with J = dN/du at u = (phi^{k+1}, ., .) by
 * linear multigrid with a transposed red-black point smoother to
 * max-norm residual <= adj_tol, then ACCUMULATES
 *   gbar_cur  += -(dG/dphi^k)^T lambda,
 *   gbar_prev += -(dG/dphi^{k-1})^T lambda,
 *   geps[0]   += -(dG/deps)^T lambda        (geps: DEVICE pointer, 1 double).
 * gbar_cur and gbar_prev may be the same buffer (bootstrap step).
 * cycles (host, nullable) receives the linear cycles used.  Synchronises. */
pfc_status pfc_adjoint_step(pfc_handle *h, const double *phi_prev, const double *phi_cur,
                            const double *phi_next, const double *gbar_next,
                            double *gbar_cur, double *gbar_prev, double *geps,
                            double adj_tol, int32_t *cycles);

/* ---------------------------------------------------------------------------
 * Kernel-level entry points (single multigrid building blocks).  They act on
 * level `level` of the handle's hierarchy (size n_l = pfc_level_size, spacing
 * h_l = L/n_l) and exist so that each kernel can be checked on its own.
 * With variable mobility each of them uses the phi* stored at its level (by
 * pfc_set_phistar or by the last pfc_step) and returns INVALID_ARG while that
 * level holds none.
 * ------------------------------------------------------------------------- */

/* Variable mobility only: stores phi* (natural order, n_l^3, device) at
 * level l and its 8-child means at every coarser level, the hierarchy that
 * pfc_step builds from 3/2 phi^k - 1/2 phi^{k-1} (the face mobilities of the
 * flux form of Section 5 are M(A phi*)).  INVALID_ARG on a handle with
 * PFC_MOBILITY_ONE.  Asynchronous. */
pfc_status pfc_set_phistar(pfc_handle *h, int32_t level, const double *phs);

/* Source S of (scheme-PFC-s1..s3) at the finest level: f3 = triple
 * (phi^k, (1-eps)/2 phi^k + 3 Delta_h phi^k - Delta_h phi^{k-1}, Delta_h phi^k / 2). */
pfc_status pfc_source(pfc_handle *h, const double *phi_prev, const double *phi_cur, double *f3);

/* r3 = f3 - N_l(u3) with N of (scheme-PFC-o1..o3) at level l (M = 1, or the
 * flux form with the handle's variable mobility)
 * (phk = phi^k on that level).  r3 may be NULL; maxnorm (host, nullable)
 * receives max|r| over the three components.  Synchronises if maxnorm.
 * With r3 NULL on a colour-split level with n a multiple of 64 and at least
 * 128 the norm comes from the column-tile kernel of the stop test; it equals
 * the thread-per-point kernel's bit for bit. */
pfc_status pfc_residual(pfc_handle *h, int32_t level, const double *u3, const double *f3,
                        const double *phk, double *r3, double *maxnorm);

/* One red-black half-sweep (Section 5 smoothing scheme, red-black order) of
 * colour `colour` ((i+j+k) mod 2) at level l, in place on u3; with colour =
 * PFC_SWEEP_FULL, one full sweep (colour 0, then colour 1), the form the
 * cycles use: on levels of at least 128^3 with n a multiple of 64 it runs as
 * a single fused pass whose result equals the two half-sweeps bit for bit. */
#define PFC_SWEEP_FULL 2
pfc_status pfc_smooth(pfc_handle *h, int32_t level, int32_t colour, double *u3,
                      const double *f3, const double *phk);

/* Coarsening I_l^{l+1} of `ncomp` consecutive fields: coarse cell = mean of
 * its 8 children.  fine: ncomp x n_l^3; coarse: ncomp x n_{l+1}^3. */
pfc_status pfc_restrict(pfc_handle *h, int32_t level, const double *fine, double *coarse,
                        int32_t ncomp);

/* Interpolation I_{l+1}^l added in place: fine += P(coarse_v - coarse_ubar),
 * cell-centred trilinear (weights 3/4, 1/4 per axis), periodic; ncomp
 * consecutive fields.  coarse_ubar may be NULL (then fine += P coarse_v). */
pfc_status pfc_prolong_add(pfc_handle *h, int32_t level, const double *coarse_v,
                           const double *coarse_ubar, double *fine, int32_t ncomp);

/* Exact solve of N_c(u3) = f3 on the coarsest level (Newton's method, dense
 * LU with partial pivoting; the "solve" step of Algorithm algorithm:FAS).
 * u3 holds the start iterate and receives the solution.  iters (host,
 * nullable) receives the Newton iteration count.  Synchronises if iters. */
pfc_status pfc_coarse_solve(pfc_handle *h, double *u3, const double *f3, const double *phk,
                            int32_t *iters);

/* ---------------------------------------------------------------------------
 * Batched form: many independent simulations (own n, L, eps, dt) advanced
 * together, every phase of a cycle one launch for all instances.
 * ------------------------------------------------------------------------- */
typedef struct pfc_batch pfc_batch;

/* Creates a batch of `count` instances with configs cfgs[0..count-1] (each
 * valid for pfc_create; precision must be FP64; all share nu1, nu2, cycle,
 * lin and tol of cfgs[0]). */
pfc_status pfc_batch_create(int32_t count, const pfc_config *cfgs, void *stream, pfc_batch **out);
pfc_status pfc_batch_destroy(pfc_batch *b);
/* Loads instance i's state: phi_prev, phi_cur, mu, omega (n_i^3 each, device). */
pfc_status pfc_batch_set_state(pfc_batch *b, int32_t i, const double *phi_prev,
                               const double *phi_cur, const double *mu, const double *omega);
/* Reads instance i's state back (phi_prev, phi_cur, mu, omega; device). */
pfc_status pfc_batch_get_state(pfc_batch *b, int32_t i, double *phi_prev, double *phi_cur,
                               double *mu, double *omega);
/* Sets instance i to the first-step state of phi0 (device, n_i^3):
 * phi_prev = phi_cur = phi0 (the bootstrap phi^{-1} = phi^0) and (mu, omega)
 * as in pfc_init_guess. */
pfc_status pfc_batch_init_state(pfc_batch *b, int32_t i, const double *phi0);
/* Advances every instance by `steps` time steps of scheme (1.10).  Each
 * phase of a cycle is one launch over all instances that take part in it
 * (levels aligned from the finest), over a work-list of fixed-size tiles of
 * every instance's part of the phase, in the schedule the autotuner chose
 * (one tile per workgroup by default).  When every instance's finest size is
 * a multiple of 16, the finest levels' interpolation runs as column tiles
 * (a 16 x 8 fine column and 4 coarse planes of one instance per workgroup,
 * the coarse error staged in LDS as it is formed, no coarse-error pass);
 * otherwise as the coarse-error pass and the interpolation phase, with the
 * same results.  An instance stops cycling when its own
 * residual meets the tolerance, so it follows exactly the cycle sequence of
 * pfc_step.  One cycle plus the stop test is captured as a hipGraph on the
 * batch's own stream and replayed.  infos (host, nullable): count*steps
 * entries, instance-major.  Returns the first non-OK instance status (the
 * others still advance).  Synchronises. */
pfc_status pfc_batch_run(pfc_batch *b, int32_t steps, pfc_step_info *infos);
/* Chooses, for each batched phase kind (smoothing, residual+coarsening, tau,
 * interpolation, coarse error), its schedule and tile shape by timing every
 * combination on this batch: one tile per workgroup or persistent (as many
 * workgroups as are resident walk the work-list), 64, 128 or 256 threads per
 * workgroup, and tiles of W = 64 .. 1024 consecutive work items of a plane
 * (half-sweep points, coarse cells, fine x-pairs or points, in the level's
 * storage order) over Z = 1 .. 8 consecutive planes, walked plane by plane.
 * With cache_path (nullable) choices are read from / written to a JSON file
 * keyed by GPU architecture, instance sizes and phase.  Where the column
 * tiles apply it then times them with Z = 1, 2, 4 or 8 coarse planes per
 * tile against the chosen coarse-error pass plus interpolation and keeps the
 * faster.  chosen (host, nullable): 20 ints, (persistent, threads, W, Z) per
 * phase in that order; column tiles read (0, 64, 64, Z).
 * Results do not depend on the choice (same per-point arithmetic).  Leaves
 * the state unchanged.  Synchronises. */
pfc_status pfc_batch_autotune(pfc_batch *b, const char *cache_path, int32_t *chosen);
const char *pfc_batch_last_error(const pfc_batch *b);

/* ---------------------------------------------------------------------------
 * Instrumentation
 * ------------------------------------------------------------------------- */
#define PFC_KERNEL_SMOOTH0 0     /* finest-level smoothing sweep launches       */
#define PFC_KERNEL_RESIDUAL0 1   /* finest-level residual + coarsening          */
#define PFC_KERNEL_PROLONG0 2    /* finest-level interpolation + correction     */
#define PFC_KERNEL_NORM0 3       /* finest-level residual max-norm              */
#define PFC_KERNEL_COARSE 4      /* coarsest-level solve                        */
#define PFC_KERNEL_SWEEP_NORM0 5 /* finest-level first pre-sweep that also forms
                                    half of the stop-test norm of its input     */
#define PFC_KERNEL_COUNT 6
/* When enabled, HIP events bracket each launch of the listed kernels on the
 * handle's stream and their durations are accumulated at every host
 * synchronisation point of the handle. */
pfc_status pfc_timing_enable(pfc_handle *h, int32_t on);
/* launches and total milliseconds accumulated for `kernel` since the last
 * reset; bytes_per_launch: the kernel's algorithmic HBM bytes per launch at
 * the finest level (0 if not defined). */
pfc_status pfc_timing_get(pfc_handle *h, int32_t kernel, int64_t *launches, double *total_ms,
                          double *bytes_per_launch);
pfc_status pfc_timing_reset(pfc_handle *h);

const char *pfc_status_string(pfc_status s);
/* Message of the last error on this handle (or of the last failed create if
 * h is NULL).  Valid until the next call on the handle. */
const char *pfc_last_error(const pfc_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* PFC_H */
