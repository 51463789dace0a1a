/*
 * sipf.h -- C ABI of libsipf: one time step of the SIPF-W method (stochastic interacting
 * particle-field method with weighted particles) for the 3D haptotaxis
 * reaction-diffusion-advection system, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Hu, Wang, Xin, Zhang, "A Novel Stochastic Particle-Field Algorithm for a
 * Reaction-Diffusion-Advection Cancer Invasion Model".
 *
 * Model (eq. haptotaxis-system): cell density u carried by P weighted particles (X_p, a_p)
 * (eq. u_hat); ECM v, enzyme m, oxygen w on a periodic N^3 grid of the cube [0, L)^3, nodes
 * at q h, h = L / N (eq. vmw_hat: nodal values and Fourier coefficients are equivalent).
 *
 * One step n -> n+1 (Alg. sipf-pic), all right-hand sides at time n:
 *   ubar  = sum_p a_p R_h(X_p, .)                         P2G, trilinear   (Alg. p2g)
 *   m*    = m + tau ubar,  w* = w + tau (gamma v - eta(ubar) w)   explicit reaction
 *   v'    = v exp(-alpha tau m)                            pointwise ECM update
 *   m', w'= IFFT( FFT(m*, w*) / (1 + tau (R + D |k|^2)) ) implicit spectral solves
 *                                                          (eq. k_q_tilde_update)
 *   grad v= IFFT(i k FFT(v))                               spectral gradient (eq. gradv)
 *   X'    = X + chi tau (grad v)_H(X) + sqrt(2 D_u tau) Z  Euler-Maruyama (eq. u_hat_update)
 *   a'    = a exp(tau (rho(w_H(X)) - 1))                   mass update (eq. SDE)
 * with rho(w) = 2w/(1+w), eta(u) = 2u/(1+u), G2P by K_h = h^3 R_h (Alg. g2p), and Z drawn from
 * Philox4x32-10 with counter (p, n, sim_id_lo, sim_id_hi) and key (seed_lo, seed_hi)
 * followed by Box-Muller (z1, z2 from words 0-1, z3 from words 2-3; u = (r + 1/2) 2^-32).
 *
 * Conventions for every entry point:
 *   - return 0 on success or a negative SIPF_E* code; sipf_last_error() then holds a message
 *     (thread-local, valid until the next failing call on that thread); no C++ exception
 *     crosses the ABI;
 *   - host arrays are float64, owned by the caller, read (or written) during the call only;
 *   - grid arrays are row-major [i1][i2][i3] (i3 fastest), N^3 entries; particle positions
 *     are structure-of-arrays X[0..P) = x1, X[P..2P) = x2, X[2P..3P) = x3;
 *   - with dim = 2 every N^3 below reads N^2 ([i1][i2]), every 3P reads 2P, and the gradient
 *     has two components;
 *   - the device workspace is owned by the caller (for example a torch uint8 tensor); the
 *     library owns the layout inside it and keeps all state there, so several simulations
 *     can be resident at once, each in its own workspace;
 *   - calls on one sipf_sim must not overlap; the stream given at init orders all work.
 */
#ifndef SIPF_H
#define SIPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define SIPF_OK 0
#define SIPF_EINVAL (-1) /* invalid parameter or input array                              */
#define SIPF_ENOMEM (-2) /* workspace smaller than sipf_state_bytes() or misaligned host   */
#define SIPF_EHIP (-3)   /* HIP runtime error (message names the call)                     */
#define SIPF_EPOS (-4)   /* positivity / finiteness violated (only with SIPF_FLAG_STRICT)  */

/* precision of positions, grid fields and FFTs; particle masses and all mass sums are
 * float64 in both forms */
#define SIPF_FP64 0
#define SIPF_FP32 1

/* flags (bitwise or) -- test hooks and variants of the step */
#define SIPF_FLAG_FREEZE_W 0x01u    /* keep w^{n+1} = w^n                                    */
#define SIPF_FLAG_FREEZE_V 0x02u    /* keep v^{n+1} = v^n                                    */
#define SIPF_FLAG_FREEZE_M 0x04u    /* keep m^{n+1} = m^n                                    */
#define SIPF_FLAG_NO_NOISE 0x08u    /* Wiener increments set to zero                          */
#define SIPF_FLAG_LINEAR_MASS 0x10u /* a' = a (1 + tau rho - tau), eq. u_hat_update           */
#define SIPF_FLAG_IMPLICIT_V 0x20u  /* v' = v / (1 + alpha tau m), positivity section          */
#define SIPF_FLAG_STRICT 0x40u      /* sipf_fields returns SIPF_EPOS on a violated invariant  */
#define SIPF_FLAG_EXP_DIFFUSION 0x80u   /* multiplier exp(-tau (R + D k^2)), eq. k_q_update   */
#define SIPF_FLAG_ALIASED_DIFFUSION 0x100u /* aliased positive multiplier, Lemma kernel      */

/* Parameters (eq. haptotaxis-system, eq. g_t: D = diag(0, D_m, D_w), R = diag(0, beta, 1)). */
typedef struct {
  double L;              /* period of the cube, > 0                                      */
  int32_t N;             /* grid nodes per axis: power of two in [4, 512] (2D: [4, 1024])  */
  int32_t dim;           /* 0 or 3: the 3D system; 2: the paper's two-dimensional form     *
                          * (grids N^2, positions 2P, bilinear transfers, deposit_order 2, *
                          * two Wiener components: the first two normals of the block)    */
  int64_t P;             /* particles, 0 <= P < 2^32                                      */
  double dt;             /* time step tau, 0 < dt <= 0.5 (positivity lemma)               */
  double D_u, chi, D_m, D_w, alpha, beta, gamma; /* model constants, all >= 0             */
  uint64_t seed;         /* Philox key                                                    */
  uint64_t sim_id;       /* Philox counter words 2-3: distinct per simulation              */
  uint64_t step0;        /* absolute index n of the first step (restart from a checkpoint)*/
  int32_t precision;     /* SIPF_FP64 or SIPF_FP32                                         */
  int32_t deposit_order; /* 2: trilinear assignment; 4: fourth-order assignment R_h^(4)    */
  uint32_t flags;        /* SIPF_FLAG_*                                                    */
  int32_t resort_every;  /* particle tile re-binning period in steps; 0: the library's    *
                          * default, the largest k (at most 64) with sqrt(k 2 D_u dt) <=    *
                          * 0.45 h in 3D, 2.4 h in 2D (diffusive drift within the tiles'    *
                          * LDS margins of one and four cells); the period changes only   *
                          * the summation order of the deposit                             */
  double H0;             /* low-pass filter exp(-2 pi^2 |q|^2 / H0^2) (Alg. p2g text), >= 0: *
                          * multiplies the m and w solves and the spectrum of v before its  *
                          * gradient; 0 = off (> 0 adds one half-spectrum to the workspace) */
} sipf_params;

/* Diagnostics of the current state (Lemma mass, Corollary mass, positivity lemma). */
typedef struct {
  double mass_particles; /* sum_p a_p (float64 accumulation)                               */
  double mass_grid;      /* h^3 sum_q ubar_q of the current particles                      */
  double mass_m;         /* h^3 sum_q m_q                                                  */
  double min_v, min_m, min_w, max_m, max_w;
  double min_a, max_a;
  double min_u;          /* min_q ubar_q (>= 0 for the trilinear assignment only: R_h^(4)   *
                          * has negative outer weights)                                     */
  int64_t n_nan;         /* particles with a non-finite mass or position, plus nodes with a *
                          * non-finite ubar, plus nodes with a non-finite v, m or w         */
  int64_t n_neg_m, n_neg_w;
  int64_t step;          /* absolute step index n of the state                             */
} sipf_diag;

typedef struct sipf_sim sipf_sim; /* opaque, library-owned host handle */

/* Device workspace bytes a simulation with these parameters needs (alignment 256 B).
 * Errors: SIPF_EINVAL for invalid parameters. */
int sipf_state_bytes(const sipf_params* prm, size_t* bytes);

/* Create a simulation in the caller's device workspace and upload the initial state
 * (Alg. sipf-pic initialisation: particles X0 ~ u(., 0) with masses a0; v0, m0, w0 sampled
 * at the nodes).  d_workspace: device pointer, 256-byte aligned, at least
 * sipf_state_bytes() long, owned by the caller and not used by anything else while the
 * simulation exists.  hip_stream: hipStream_t on which all later work of this simulation is
 * ordered (NULL = the default stream).  X0: 3P float64 (SoA), finite; a0: P float64, finite
 * and > 0; v0: N^3 float64, finite, >= 0; m0, w0: N^3 float64, finite (a checkpoint may hold
 * the small negative values the implicit solve allows).  Positions are wrapped into [0, L).  In SIPF_FP32
 * precision, positions and fields are rounded to float32; a0 stays float64.
 * The call is synchronous.  On success *out receives the handle.
 * Errors: SIPF_EINVAL (parameters or inputs), SIPF_ENOMEM (workspace), SIPF_EHIP. */
int sipf_init(const sipf_params* prm, void* d_workspace, size_t bytes, void* hip_stream,
              const double* X0, const double* a0, const double* v0, const double* m0,
              const double* w0, sipf_sim** out);

/* Enqueue nsteps >= 0 steps (Alg. sipf-pic loop body) on the simulation's stream; returns
 * without waiting.  The steps reduce no diagnostics: sipf_fields reduces them from the
 * state it reads.  The first call with nsteps > 0 captures the step as HIP
 * graphs (host work only; captures are serialised across threads), which later calls
 * replay.  Errors: SIPF_EINVAL, SIPF_EHIP. */
int sipf_step(sipf_sim* sim, int32_t nsteps);

/* Move a simulation to another stream (for example from the stream it was initialised on
 * to the stream its batch runs on).  Work already queued on the old stream is ordered
 * before later work on the new one; nothing waits on the host.  Errors: SIPF_EINVAL,
 * SIPF_EHIP. */
int sipf_set_stream(sipf_sim* sim, void* hip_stream);

/* Served form: enqueue nsteps steps of nsims resident simulations as one set of batched
 * launches (each kernel launch covers the work of all listed simulations).  All must share
 * the precision, deposit order and device; they run on the stream of sims[0].  Results are
 * identical to stepping each simulation alone (up to the order of floating-point atomic
 * additions).  Errors: SIPF_EINVAL (empty list, mixed precision, a repeated simulation),
 * SIPF_EHIP. */
int sipf_step_batch(sipf_sim* const* sims, int32_t nsims, int32_t nsteps);

/* Allocation-free form of sipf_step_batch, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, requirements and results as sipf_step_batch; in addition the simulations' device
 * must be the current device and nsims <= 64.  The batch's launch table (descriptors and
 * per-kernel block offsets, at most 128 KiB) lives in one library-owned device array per GPU,
 * set up when the first simulation is created on that GPU and held until the process ends;
 * the steps are launched kernel by kernel on the stream of sims[0] (no graph is instantiated,
 * nothing is allocated).  Every call on a GPU rewrites that GPU's array: calls ordered on one
 * stream are safe, calls that overlap on one GPU without ordering race on the table.
 * Errors: as sipf_step_batch, plus SIPF_EINVAL for nsims > 64, a table above the limit, or
 * a device that is not current. */
int sipf_step_batch_noalloc(sipf_sim* const* sims, int32_t nsims, int32_t nsteps);

/* Wait for the simulation's stream and copy the state to the host: any pointer may be NULL.
 * v, m, w: N^3 float64; X: 3P float64 SoA in the particle order given at init; a: P float64;
 * diag: diagnostics of the state.  With SIPF_FLAG_STRICT, returns SIPF_EPOS (after filling
 * the outputs) if a hard invariant fails: a non-finite value, ubar < 0, v <= 0, a <= 0.
 * Errors: SIPF_EHIP, SIPF_EPOS. */
int sipf_fields(sipf_sim* sim, double* v, double* m, double* w, double* X, double* a,
                sipf_diag* diag);

/* Intermediate grids of the last step, for checks of single stages: u_bar (N^3, the P2G
 * deposit of the current particles) and grad_v (3 N^3: d1 v, d2 v, d3 v of the field v
 * that drove the last push).  Either pointer may be NULL.  Synchronous.
 * Errors: SIPF_EHIP. */
int sipf_aux(sipf_sim* sim, double* u_bar, double* grad_v);

/* Profiling hook: run nsteps steps eagerly (kernel launches, not the captured graph) with HIP
 * events between the stages, and add each stage's elapsed milliseconds to stage_ms[k]
 * (caller-owned, SIPF_NUM_STAGES floats; stage order: SIPF_STAGE_*).  Synchronous.
 * Results are identical to sipf_step.  Errors: SIPF_EINVAL, SIPF_EHIP. */
#define SIPF_NUM_STAGES 8
#define SIPF_STAGE_ZFWD 0      /* reaction + forward z transforms            */
#define SIPF_STAGE_YFWD 1      /* forward y transforms                       */
#define SIPF_STAGE_XPASS 2     /* x transforms + spectral solves + d1 v      */
#define SIPF_STAGE_YINV 3      /* inverse y transforms + d2 v                */
#define SIPF_STAGE_ZINV 4      /* inverse z transforms + d3 v, field writes  */
#define SIPF_STAGE_PARTICLES 5 /* gather + push + mass update + deposit      */
#define SIPF_STAGE_FINALIZE 6  /* step index                                 */
#define SIPF_STAGE_BINNING 7   /* tile binning of the particles (when due)   */
int sipf_step_timed(sipf_sim* sim, int32_t nsteps, float* stage_ms);

/* Residual resampling (Alg. res_res) of the simulation's particles at its current step n:
 * the P weighted particles become P particles of equal mass a0 = (1/P) sum_p a_p, with
 * k_p = floor(a_p / a0) copies of particle p (in particle order) followed by
 * P - sum_p k_p particles drawn with probabilities proportional to the residuals
 * a_p - k_p a0 (in draw order).  The new particle with list index i is particle i from then
 * on (its noise stream and its place in sipf_fields' output).  Arithmetic, so that the list
 * is a function of the state alone: the mass sum is exact and rounded once to float64;
 * q_p = a_p / a0 and k_p = floor(q_p) in float64; the residual enters the draws as
 * R_p = floor((q_p - k_p) 2^32); draw j takes Philox4x32-10 words (r0, r1) at counter
 * (j, n, sim_id_lo, sim_id_hi | 2^31), key (seed_lo, seed_hi), and selects the particle whose
 * interval of the running sum of R holds floor((r0 + 2^32 r1) sum_p R_p / 2^64) (uniformly
 * over all P if every R_p is 0).  Positions are copied unchanged (in SIPF_FP32, the float32
 * positions of the state).  The deposited density is recomputed for the new particles; the
 * fields and the step index are unchanged.  Synchronous; info (may be
 * NULL) receives a0 and the two counts.  P = 0 is a no-op.
 * Errors: SIPF_EINVAL (P >= 2^31; sim_id >= 2^63; a mass negative or not finite; total mass
 * zero; largest mass outside [2^-775, 2^990) or a non-zero mass below 2^-160 of the largest:
 * the state is then unchanged), SIPF_EHIP. */
typedef struct {
  double a0;       /* mass of every particle after resampling                              */
  int64_t n_det;   /* particles placed by the deterministic copies                         */
  int64_t n_stoch; /* particles drawn                                                     */
} sipf_resample_info;
int sipf_resample(sipf_sim* sim, sipf_resample_info* info);

/* Free the host handle and the library's HIP objects (graphs, events); the workspace
 * stays the caller's.  Waits for the simulation's outstanding work.  NULL is a no-op. */
void sipf_destroy(sipf_sim* sim);

/* Message of the last failing call on this thread ("" if none). */
const char* sipf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SIPF_H */
