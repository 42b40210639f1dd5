/*
 * hrm.h -- C-ABI of the MI355X (gfx950) library for the hot path of the
 * positivity-preserving fractional algorithm for the four-equation HRM
 * (Wong, Angel & Kiris, arXiv:2208.04488): one hyperbolic SSP-RK stage of the
 * five-equation model with PP-WCNS-IS, followed by the algebraic
 * infinite-rate thermal relaxation.
 *
 * Conventions common to every call
 *  - State arrays are caller-owned DEVICE pointers to double, laid out
 *    structure-of-arrays as W[c][z][y][x] (x fastest), interior cells only,
 *    ncell = n[0]*n[1]*n[2].  Component order is the conservative vector of
 *    Sec. 2: alpha_k rho_k (k = 0..N-1), rho u_d (d = 0..dim-1), E,
 *    alpha_k (k = 0..N-2); M = 2N + dim components.  Ghost cells do not
 *    exist in memory: boundary conditions are applied when tiles are loaded.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call only enqueues work on that stream and returns; device errors
 *    of a kernel surface at the next synchronising call.
 *  - Calls return an int status: HRM_OK, or an error code with a message
 *    readable through hrm_last_error().  No exception crosses the ABI.
 *  - Calls on one context are not thread-safe; use one context per thread.
 *    Work enqueued on one context shares its scratch (stage buffers,
 *    wavespeed partials, counters): calls on one context that run at the
 *    same time on different streams race.
 */
#ifndef HRM_H
#define HRM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HRM_MAX_SPECIES 8

/* status codes */
#define HRM_OK 0
#define HRM_EINVAL 1        /* bad sizes, EOS, stage index, aliasing, NULL pointer */
#define HRM_ENOMEM 2        /* device allocation failed */
#define HRM_EDEVICE 3       /* a HIP runtime call failed (message in hrm_last_error) */
#define HRM_EADMISSIBLE 4   /* hrm_get_diagnostics: relaxation met states outside script-G */
#define HRM_EUNSUPPORTED 5  /* (N, dim, precision, weights) combination not built */

/* boundary conditions per side (Sec. 5: extrapolation / periodic; the
 * Dirichlet inflow of the Mach-100 water jet, Sec. 5.9).  Periodic sides
 * come in pairs; a Dirichlet side needs hrm_set_boundary_state. */
#define HRM_BC_TRANSMISSIVE 0
#define HRM_BC_PERIODIC 1
#define HRM_BC_DIRICHLET 2

/* face arithmetic precision; the state, relaxation, limiter bound checks and
 * the accumulation are double in both */
#define HRM_FP64 0
#define HRM_FP32 1

/* nonlinear weights of the interpolation */
#define HRM_WEIGHTS_IS 0  /* incremental-stencil WENO weights (App. C) */
#define HRM_WEIGHTS_MLP 1 /* learned weights (not in the paper; see hrm_set_mlp); FP64, dim <= 2 */

/* grid flags */
#define HRM_NO_LIMITERS 1   /* skip the interpolation and flux limiters (Sec. 4.3.2) */
#define HRM_NO_BLEND 2      /* shock-sensor blending off: pure HCS flux (App. B) */
#define HRM_FIRST_ORDER 4   /* first-order HLLC fluxes only (Sec. 4.1.1) */
#define HRM_FUSE_RELAX 8    /* hrm_rk_stage relaxes its output in the same kernel */
#define HRM_NO_GRAPH 16     /* hrm_advance launches its kernels directly instead of replaying a graph */
/* HRM_FOUR_EQ: solve the four-equation HRM directly instead of the fractional
 * algorithm (the comparison scheme of Sec. 5.4 and App. A).  The fluxes of
 * alpha_k rho_k, rho u and E are those of the first-order HLLC solver of
 * Sec. 4.1.1 with the HRM pressure p* (eq:p_relax, the relaxed pressure of the
 * state) and the HRM sound speed (eq:4_eqn_sos) in place of the five-equation
 * ones, always in double precision; the volume fractions are not evolved (their
 * right-hand side is zero) and are the equilibrium values only where the
 * relaxation runs (HRM_FUSE_RELAX or hrm_relax), for output.  The time step of
 * hrm_compute_dt / hrm_advance uses the HRM sound speed.  Implies HRM_FIRST_ORDER;
 * the limiter, blending and weight settings have no effect. */
#define HRM_FOUR_EQ 32

/* Uniform Cartesian grid of n[0] x n[1] x n[2] cells, nodes at cell centres
 * (Sec. 4.1).  Entries beyond `dim` must be n = 1. */
typedef struct {
    int dim;               /* D = 1, 2 or 3 */
    int n[3];              /* cells per direction */
    double dx[3];          /* spacing per direction (> 0) */
    int bc_lo[3], bc_hi[3];
    int precision;         /* HRM_FP64 or HRM_FP32 */
    int weights;           /* HRM_WEIGHTS_IS */
    int flags;             /* HRM_NO_LIMITERS | HRM_NO_BLEND | HRM_FIRST_ORDER | HRM_FUSE_RELAX */
} hrm_grid;

/* Stiffened-gas species (eq:species_stiffened_EOS): gamma_k > 1, c_v,k > 0,
 * p_inf,k >= 0, q_k.  Species 0 is the liquid; species 1..N-1 must have
 * p_inf = 0 (the relaxation of Sec. 4.2 assumes one stiffened gas). */
typedef struct {
    int nspecies;          /* N >= 2 */
    double gamma[HRM_MAX_SPECIES];
    double cv[HRM_MAX_SPECIES];
    double pinf[HRM_MAX_SPECIES];
    double q[HRM_MAX_SPECIES];
} hrm_eos;

/* Tolerances and constants; hrm_default_params() fills the paper's values:
 * WENO eps 1e-15 (App. C); interpolation limiter eps 1e-10, 1e-10 and hard
 * switch 1e-11, 1e-11, 1e-9 (Sec. 4.3.2); flux limiter eps 1e-10, 1e-10,
 * 1e-8 and hard switch 1e-11, 1e-11, 1e-9 (Sec. 4.3.2); sensor C_s = 1e12,
 * q = 2 and HCS psi = 256/175 (Sec. 4.3.1). */
typedef struct {
    double eps_weno;
    double eps_i_ar, eps_i_a;
    double hs_i_ar, hs_i_a, hs_i_rc2;
    double eps_f_ar, eps_f_a, eps_f_re;
    double hs_f_ar, hs_f_a, hs_f_re;
    double Cs, qexp, psi;
} hrm_params;

/* Device-side counters, read by hrm_get_diagnostics (which synchronises). */
typedef struct {
    unsigned long long alg1;       /* interpolated partial densities blended (Alg. 1) */
    unsigned long long alg2;       /* interpolated volume fractions blended (Alg. 2) */
    unsigned long long interp_hs;  /* interpolation hard switch fired */
    unsigned long long alg3;       /* faces with theta < 1 in Alg. 3 */
    unsigned long long alg4;       /* faces with theta < 1 in Alg. 4 */
    unsigned long long flux_hs;    /* flux hard switch fired */
    unsigned long long relax_bad;  /* relaxation inputs outside script-G (left unchanged) */
    unsigned long long reserved;
} hrm_diag;

typedef struct hrm_ctx hrm_ctx;

/* Fill `p` with the paper's tolerances and constants. */
void hrm_default_params(hrm_params* p);

/* Validate grid and EOS, copy them into the context and allocate the
 * library's scratch on the current device: one M x ncell right-hand-side
 * buffer (dim > 1), two M x ncell stage buffers for hrm_advance, wavespeed
 * partials and the counters.  `params` NULL means hrm_default_params().
 * HRM_EUNSUPPORTED if a sweep launch would exceed the device's grid limits:
 * in 2D n[0] <= 4 128 705 and n[1] <= 983 025, in 3D also n[1] and n[2]
 * <= 65 535 (1D lines have no such limit).
 * On failure *out is NULL and the code says why (no message store exists). */
int hrm_create(const hrm_grid* grid, const hrm_eos* eos, const hrm_params* params, hrm_ctx** out);

/* Free the context and its scratch (synchronises the device first). */
int hrm_destroy(hrm_ctx* ctx);

/* Message of the last failed call on this context ("" if none). */
const char* hrm_last_error(const hrm_ctx* ctx);

/* Sec. 4.1.2: d_out[d] = max over cells of |u_d| + c (five-equation mixture
 * sound speed; the HRM sound speed under HRM_FOUR_EQ), d = 0..dim-1.
 * d_W: M x ncell doubles; d_out: dim doubles. */
int hrm_max_wavespeed(hrm_ctx* ctx, const double* d_W, double* d_out, void* stream);

/* Sec. 4.1.2 multi-dimensional step: tau_d = d_maxspeed[d]/dx_d,
 * dt = CFL / sum tau (or dt_fixed if > 0), sigma_d = tau_d / sum tau,
 * lambda_d = dt / (sigma_d dx_d).  If t_end > 0 the step is clipped so that
 * the device time d_slot[4] does not pass t_end, and d_slot[4] advances by dt.
 * Writes d_slot = (dt, lambda_0, lambda_1, lambda_2, t) on the device. */
int hrm_compute_dt(hrm_ctx* ctx, const double* d_maxspeed, double cfl, double dt_fixed, double t_end,
                   double* d_slot, void* stream);

/* Semi-discrete right-hand side (eq:semi_W_G_pm_eqn) of state d_W:
 *   d_L_i = - sum_d (G^{**,-}_{i+1/2} - G^{**,+}_{i-1/2}) / dx_d
 * with the limiters' lambda_d read from d_slot[1 + d].  d_L: M x ncell. */
int hrm_rhs(hrm_ctx* ctx, const double* d_W, double* d_L, const double* d_slot, void* stream);

/* One SSP-RK3 stage in Shu-Osher form (stage = 0, 1, 2; Sec. 4.4):
 *   d_Wout = a_s d_Wn + b_s (d_Ws + dt L(d_Ws)),
 *   (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3), dt = d_slot[0],
 * followed by the thermal relaxation when the grid has HRM_FUSE_RELAX.
 * d_Wout may alias d_Wn (read point-wise) but must not alias d_Ws. */
int hrm_rk_stage(hrm_ctx* ctx, int stage, const double* d_Wn, const double* d_Ws, double* d_Wout,
                 const double* d_slot, void* stream);

/* Sec. 4.2: in-place infinite-rate thermal relaxation of every cell; only the
 * volume-fraction components change.  Cells with rho(e - qbar) <= 0 are left
 * unchanged and counted in hrm_diag.relax_bad. */
int hrm_relax(hrm_ctx* ctx, double* d_W, void* stream);

/* Sec. 3: the equilibrium state of every cell as the four-equation HRM sees
 * it: the relaxed pressure p* (eq:p_relax) and temperature T*
 * (eq:T_relax_e) that the relaxation of Sec. 4.2 would reach, and the HRM
 * sound speed of eq:4_eqn_sos (the c of Sec. 5.3's acoustic experiment),
 * from alpha_k rho_k, rho u and E (the stored volume fractions are not
 * used).  d_W: M x ncell DEVICE doubles; d_p, d_T, d_c: ncell DEVICE doubles
 * each, any of them NULL to skip it (all NULL: nothing is launched).  Cells
 * with rho(e - qbar) <= 0 or no positive root get NaN in all three. */
int hrm_equilibrium_state(hrm_ctx* ctx, const double* d_W, double* d_p, double* d_T, double* d_c, void* stream);

/* Dirichlet boundary (Sec. 5.9: the left boundary of the water jet).  The
 * three ghost nodes beyond side `side` (0 low, 1 high) of dimension `dim` all
 * take a given state W_b, one per line of cells normal to that face: for the
 * line through transverse cell (i_a, i_b), a < b the two other dimensions
 * (i_a, i_b = 0 where a dimension is not used), W_b[c] is
 * d_state[c * n_a * n_b + i_a + n_a * i_b], c = 0 .. M-1 in the component
 * order of W.  The states also enter the maximum wavespeed of direction
 * `dim` (hrm_max_wavespeed, hrm_advance).  d_state is device memory of the
 * caller; it is copied into the context on `stream`, so it may be freed or
 * changed once that copy has run, and later steps see the new state.  Every
 * Dirichlet side must be set before the first hrm_rhs / hrm_rk_stage /
 * hrm_advance / hrm_max_wavespeed (HRM_EINVAL otherwise).  HRM_EINVAL if the
 * side is not Dirichlet or d_state is NULL. */
int hrm_set_boundary_state(hrm_ctx* ctx, int dim, int side, const double* d_state, void* stream);

/* Learned interpolation weights (an extension; the paper's weights are those
 * of App. C).  On a grid created with weights = HRM_WEIGHTS_MLP every
 * characteristic variable is interpolated at i+1/2 (and mirrored for the
 * right-biased value) as sum_k omega_k S_k over the three 3-point candidates
 * of the fifth-order interpolation from u_{i-2..i+2},
 *   S_l = (3u_{i-2} - 10u_{i-1} + 15u_i)/8, S_c = (-u_{i-1} + 6u_i + 3u_{i+1})/8,
 *   S_r = (3u_i + 6u_{i+1} - u_{i+2})/8,
 * omega_k proportional to d_k e^{tanh z_k} / (1e-6 + beta_k)^2, d = (1/16,
 * 10/16, 5/16): the classical fifth-order WENO weights (Jiang & Shu
 * smoothness indicators beta_k) of the normalised stencil
 * x_j = (u_j - u_i) / max_j |u_j - u_i|, each rescaled by at most e either
 * way by z = MLP(x), a 5-32-32-3 ReLU perceptron evaluated on the bfloat16
 * matrix cores with float accumulation.  Where a weight is not finite the
 * App. C value is used.  The limiters, HLLC, HCS and relaxation are
 * unchanged.
 * h_params: HOST array of 1347 floats, W1[5][32], b1[32], W2[32][32], b2[32],
 * W3[32][3], b3[3] (rows = input unit); copied (synchronises the context's
 * last stream).  Required before any operator call on such a grid. */
int hrm_set_mlp(hrm_ctx* ctx, const float* h_params);

/* The learned interpolation alone, for checking it: n stencils d_U5[i][0..4]
 * (DEVICE, doubles, u_{i-2..i+2}) -> d_val[i] (DEVICE doubles) and the
 * weights d_omega[i][0..2] (DEVICE floats), exactly as the solver evaluates
 * them.  Needs a grid with HRM_WEIGHTS_MLP after hrm_set_mlp. */
int hrm_mlp_infer(hrm_ctx* ctx, const double* d_U5, long long n, double* d_val, float* d_omega, void* stream);

/* ---- Training of the learned weights (context-free; float32 on the GPU) ----
 * Pairs come from a fine 1D ensemble (layout as hrm_batch_*, problem b owning
 * fine cells h_offsets[b] .. h_offsets[b+1]-1 of d_W, M = 2N+1 components)
 * by injection: coarse node j = fine node 2j, and the label of the coarse
 * face j+1/2 is fine node 2j+1 (cell-centred nodes).  For every problem with
 * an even fine length 2n, n >= 5, and every field of the primitive vector
 * (alpha_k rho_k, u, p, alpha_k; App. D), in that order: the left-biased
 * stencils (coarse j-2..j+2) for j = 2..n-3, then the mirrored right-biased
 * ones (coarse j+3..j-1) for j = 1..n-4.  A pair is stored normalised,
 *   x_j = (u_j - u_i) r, r = 1 / s, s = max_j |u_j - u_i|,
 *   t = (label - u_i) r,
 * with r = 0 (x = 0, t = 0: no contribution to the loss) where
 * s <= 1e-10 max_j |u_j| (variations at round-off level carry no shape) or
 * |t| > 4 (a feature the coarse stencil does not see: beyond every convex
 * combination of the candidates, whose values lie within [-3.5, 3.5]);
 * as d_X[s][0..7] = (x_0..x_4, 0, 0, 0) and d_T[s] (DEVICE floats).
 * With d_X = d_T = NULL only *nsamples is set (size query).  Otherwise
 * capacity (in samples) must hold them all.  Synchronises `stream`. */
int hrm_mlp_extract(const hrm_eos* eos, const double* d_W, long long T, int nprob, const long long* h_offsets,
                    float* d_X, float* d_T, long long capacity, long long* nsamples, void* stream);

/* Training pairs from a fine grid (grid as hrm_create takes it; only dim
 * and n are used; d_W: M x ncell DEVICE doubles, M = 2N + dim), by the
 * injection recipe of hrm_mlp_extract applied to lines of cells: for each
 * direction d < dim whose fine length n[d] = 2m is even with m >= 5, the lines
 * along d through every `stride`-th cell of each transverse dimension
 * (transverse indices 0, stride, 2 stride, ...), each line a fine 1D problem
 * of 2m cells.  Per line, for every field of the primitive vector
 * (alpha_k rho_k, u_0 .. u_{dim-1}, p, alpha_k; App. D) in that order, the
 * left-biased stencils (coarse j-2..j+2) for j = 2..m-3, then the mirrored
 * ones (coarse j+3..j-1) for j = 1..m-4; lines in direction order, then the
 * first transverse index fastest.  Normalisation, neutral pairs and the
 * output layout are those of hrm_mlp_extract.  With d_X = d_T = NULL only
 * *nsamples is set.  Asynchronous on `stream` (allocates nothing).
 * HRM_EINVAL for bad sizes or stride < 1, HRM_EUNSUPPORTED for N other than
 * 2 or 3. */
int hrm_mlp_extract_grid(const hrm_grid* grid, const hrm_eos* eos, const double* d_W, int stride, float* d_X,
                         float* d_T, long long capacity, long long* nsamples, void* stream);

/* Floats of workspace hrm_mlp_grad needs for a minibatch of `count`. */
long long hrm_mlp_grad_workspace(int count);

/* Mean squared residual over a minibatch and its gradient (float32):
 *   L = (1/count) sum_s (sum_k omega_k(x_s) S_k(x_s) - t_s)^2,
 * omega as in hrm_set_mlp (in float, without bfloat16 rounding), over the
 * samples (first + s * stride) mod nsamp, s < count, of d_X, d_T.
 * d_params: 1347 floats (layout of hrm_set_mlp, DEVICE); writes d_grad[1347]
 * and d_loss[1] (DEVICE).  Per-workgroup partial sums go to d_work (at least
 * hrm_mlp_grad_workspace(count) floats) and are reduced in a fixed order, so
 * the result is deterministic. */
int hrm_mlp_grad(const float* d_params, const float* d_X, const float* d_T, long long nsamp, long long first,
                 long long stride, int count, float* d_grad, float* d_loss, float* d_work, long long work_floats,
                 void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, training loops that must not allocate, harnesses that forbid
 * hipMalloc): hrm_mlp_grad without the workspace argument.  The
 * per-workgroup partial sums go to a fixed array in the library's device
 * memory, ceil(HRM_MLP_GRAD_NOALLOC_MAX / 64) x 1348 floats (2.8 MB), one copy
 * per device the library runs on, held until the process ends; its address on
 * the current device is looked up at the first call there (HRM_EDEVICE if
 * that fails).  The call allocates nothing and launches the kernels of
 * hrm_mlp_grad in the same order, so d_grad and d_loss equal hrm_mlp_grad's to
 * the bit.  count > HRM_MLP_GRAD_NOALLOC_MAX gives HRM_EINVAL (nothing is
 * launched).  Every entry of the array a call reads is written by that call
 * first; calls on one device that run at the same time (other streams,
 * threads or processes' contexts) share the array and race, calls on one
 * stream are ordered. */
#define HRM_MLP_GRAD_NOALLOC_MAX 32768
int hrm_mlp_grad_noalloc(const float* d_params, const float* d_X, const float* d_T, long long nsamp,
                         long long first, long long stride, int count, float* d_grad, float* d_loss, void* stream);

/* Adam step `step` (>= 1) on the 1347 parameters, all DEVICE floats:
 *   m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 *   p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
int hrm_mlp_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, int step, float lr, float beta1,
                 float beta2, float eps, void* stream);

/* `nsteps` full SSP-RK3 steps of the fractional algorithm (Sec. 4: the
 * stages of Sec. 4.1 each followed by the relaxation of Sec. 4.2) on d_W in
 * place.  Each step takes its time step from the maximum of |u_d| + c of
 * W^n (Sec. 4.1.2; into d_slot as hrm_compute_dt writes it, with the device
 * time slot[4] advanced and clipped to t_end), then runs three stages with
 * the context's stage buffers, relaxing each stage's output.  The maxima of
 * the first step are taken by a pass over d_W; those of every later step
 * by the last sweep of the step before, from the cells it has just written
 * (the same values, so the result equals nsteps calls of hrm_step to the
 * bit).  d_W (M x ncell, component-major) and d_slot (>= 5 doubles) are the
 * caller's device memory; nothing else in d_W may change during the call.
 * Unless the grid has HRM_NO_GRAPH (or timing is on), the step's launches
 * are captured once into a hipGraph on a private stream and replayed on
 * `stream` for every step with the same (d_W, d_slot, cfl, dt_fixed,
 * t_end); other arguments re-capture.  The graph holds kernel nodes only.
 * HRM_EINVAL for NULL pointers, nsteps < 0, or neither cfl nor dt_fixed
 * positive; nsteps == 0 launches nothing. */
int hrm_advance(hrm_ctx* ctx, double* d_W, int nsteps, double cfl, double dt_fixed, double t_end, double* d_slot,
                void* stream);

/* hrm_advance with nsteps = 1. */
int hrm_step(hrm_ctx* ctx, double* d_W, double cfl, double dt_fixed, double t_end, double* d_slot,
             void* stream);

/* Copy the counters to *out (synchronises the stream of the last call).
 * Returns HRM_EADMISSIBLE if relax_bad > 0, else HRM_OK. */
int hrm_get_diagnostics(hrm_ctx* ctx, hrm_diag* out);

/* Zero the counters (enqueued on `stream`, by a kernel). */
int hrm_reset_diagnostics(hrm_ctx* ctx, void* stream);

/* Opt-in kernel timing with HIP events recorded on the caller's stream
 * around each launch of the selected kinds (bit k of `mask` selects kind k).
 * For measurement only: event records add a few microseconds per launch.
 * When more than 4096 launches are pending the recording call synchronises
 * its stream to fold them into the totals. */
#define HRM_T_SWEEP_X 0    /* k_sweep, direction 0 */
#define HRM_T_SWEEP_Y 1    /* k_sweep, direction 1 */
#define HRM_T_SWEEP_Z 2    /* k_sweep, direction 2 */
#define HRM_T_WAVESPEED 3  /* wavespeed partial maxima + final reduction */
#define HRM_T_DT 4         /* time-step kernel */
#define HRM_T_RELAX 5      /* stand-alone relaxation */
#define HRM_NTIMERS 6
int hrm_set_timing(hrm_ctx* ctx, int mask);

/* Synchronise, then write the summed milliseconds and launch counts per kind
 * since the last call into ms[HRM_NTIMERS] and counts[HRM_NTIMERS]; the
 * totals restart from zero. */
int hrm_get_timing(hrm_ctx* ctx, double* ms, long long* counts);

/* ------------------------------------------------------------------------
 * Ragged ensemble of independent 1D problems (the fractional algorithm of
 * Sec. 4 applied to many shock tubes at once).  Problem b owns cells
 * offsets[b] .. offsets[b+1]-1 of one structure-of-arrays state of
 * T = offsets[nprob] cells, component-major: d_W[c * T + cell], c < M = 2N+1.
 * Both ends of every problem are transmissive.  Every problem takes its own
 * time step from its own maximum |u| + c (Sec. 4.1.2, CFL given per run) and
 * keeps its own time.  One persistent launch advances every problem by
 * `steps_per_launch` SSP-RK3 steps with the relaxation after each stage; the
 * workgroups take problems from an atomic queue, longest first. */
typedef struct hrm_batch hrm_batch;

/* Validates the EOS (as hrm_create; N = 2 or 3), offsets (offsets[0] = 0,
 * strictly increasing: every problem has at least one cell) and dx[b] > 0,
 * all HOST arrays copied at creation; precision HRM_FP64 or HRM_FP32 (face
 * arithmetic, as for grids).  Allocates two stage buffers of M x T doubles.
 * prm may be NULL (paper parameters). */
int hrm_batch_create(const hrm_eos* eos, const hrm_params* prm, int nprob, const long long* h_offsets,
                     const double* h_dx, int precision, hrm_batch** out);
int hrm_batch_destroy(hrm_batch* b);
const char* hrm_batch_last_error(const hrm_batch* b);

/* Launch shape: threads per workgroup (64, 128 or 256; one face per
 * thread, tiles of threads-1 cells), workgroups of the persistent launch,
 * and SSP-RK3 steps per launch.  Defaults 256, 3 x the device's CU count,
 * 10.  A change drops the captured graph. */
int hrm_batch_configure(hrm_batch* b, int threads, int blocks, int steps_per_launch);

/* Advance every problem of d_W (device, M x T) in place by nsteps steps, a
 * multiple of steps_per_launch.  The first call captures (queue reset,
 * persistent launch) into a hipGraph on a private stream; calls with the
 * same (d_W, cfl) replay it nsteps / steps_per_launch times on `stream`.
 * Calls on one batch must not overlap (they share the stage buffers). */
int hrm_batch_run(hrm_batch* b, double* d_W, int nsteps, double cfl, void* stream);

/* Synchronise and copy the per-problem times (sum of the steps taken since
 * creation) to h_t[nprob]. */
int hrm_batch_time(hrm_batch* b, double* h_t);

/* Per-problem end times, h_tend[nprob] on the host (copied after the work
 * already enqueued on the batch has finished).  A problem's step is clipped
 * so that its time does not pass its end time (as hrm_compute_dt clips with
 * t_end), and a problem at its end time takes no further steps, so a run of
 * enough steps brings every problem exactly to its own end time.  Values
 * <= 0 mean no end time (the default).  HRM_EINVAL for a NaN. */
int hrm_batch_set_end_times(hrm_batch* b, const double* h_tend);

/* Synchronise and copy the counters (as hrm_get_diagnostics; counts every
 * face of every problem once per stage). */
int hrm_batch_get_diagnostics(hrm_batch* b, hrm_diag* out);

#ifdef __cplusplus
}
#endif

#endif /* HRM_H */
