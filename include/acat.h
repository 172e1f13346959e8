/*
 * acat.h -- C ABI of the MI355X (gfx950) ACAT library.
 *
 * One time step of the Adaptive Compact Approximate Taylor method of
 * Carrillo, Macca, Pares, Russo and Zorio, "An order-adaptive compact
 * approximation Taylor method for systems of conservation laws"
 * (arXiv:2007.01416), for u_t + f(u)_x (+ g(u)_y) = 0 (Sec. 2, eq. of the
 * 1D system; Sec. 4, the 2D system):
 *
 *   - per interface, smoothness indicators psi^p (Sec. 3.2, minimum over the
 *     conserved components as in Sec. 3.4) choose the stencil half-width
 *     p_s = max{p in 2..P : psi^p >= theta}, or the FL-CAT2 fallback when no
 *     p qualifies (Sec. 3, admissible set and ACAT flux);
 *   - the CAT2p numerical flux is the local Taylor recursion of Sec. 2.2
 *     (centred differentiation in space and time on the 2p-point stencil in
 *     place of the Cauchy-Kovalevskaya procedure); in 2D the corner
 *     recursion of Sec. 4 on the rectangle J_q1 x J_q2 of the x- and
 *     y-interface orders;
 *   - the FL-CAT2 fallback blends CAT2 with the Rusanov flux through the
 *     superbee limiter in its speed-free min form (Sec. 3.1);
 *   - the conservative update (Sec. 2.1 conservative form; Sec. 3.3 in 1D;
 *     the unsplit 2D scheme of Sec. 4).
 *
 * Conventions
 *   - All arithmetic and all state arrays are IEEE binary64.
 *   - Arrays are DEVICE pointers unless marked "host".  States are SoA
 *     without ghost cells: 1D u[var][x], 2D u[var][y][x] (x fastest).
 *   - Interfaces: 1D has nI = nx (periodic) or nx + 1 (transmissive)
 *     interfaces; entry k is x_{i+1/2} with i = k (periodic) or i = k - 1
 *     (transmissive).  2D x-interfaces are stored [ny][nIx], y-interfaces
 *     [nIy][nx], with nIx, nIy defined the same way per direction.
 *   - The caller owns every buffer (state, workspace, decision maps) and
 *     allocates it; the library never allocates inside a step.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL is the
 *     null stream) and captures into a HIP graph: no host synchronisation,
 *     no allocation, no memset nodes.
 *   - Functions return an acat_status and never abort or throw.  Argument
 *     errors are detected on the host before any launch.  Non-finite
 *     output, or non-positive density or pressure for Euler, set bits of a
 *     device status word read by acat_device_status().
 */
#ifndef ACAT_H
#define ACAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ACAT_OK = 0,
  ACAT_ERR_NULL = -1,        /* a required pointer is NULL                     */
  ACAT_ERR_ARG = -2,         /* invalid dim/nvar/flux/P/bc/sizes/dx/dt/theta   */
  ACAT_ERR_ALIAS = -3,       /* u_in and u_out overlap                          */
  ACAT_ERR_UNSUPPORTED = -4, /* valid problem the library has no kernel for    */
  ACAT_ERR_DEVICE = -5,      /* a HIP call failed (launch or copy)              */
  ACAT_ERR_WORKSPACE = -6    /* workspace missing or smaller than required      */
} acat_status;

enum { ACAT_FLUX_ADVECTION = 0, ACAT_FLUX_BURGERS = 1, ACAT_FLUX_EULER = 2 };
enum { ACAT_BC_PERIODIC = 0, ACAT_BC_TRANSMISSIVE = 1 };

/* Variants (acat_problem.flags, bitwise or; 0 = the default method).
 *   FLO_LF / FLO_HLL: the first-order flux of the FL-CAT2 blend (Sec. 3.1) is
 *     Lax-Friedrichs (speed dx/(dim dt) per direction, so the 2D sum is the
 *     classical 2D scheme) or HLL (Davis speed estimates) instead of Rusanov;
 *     the paper's experiments compare with both (Sec. 5).  Exclusive.
 *   PSI2_MODIFIED: the modified p = 2 indicator of Sec. 3.2 (two pairs of
 *     lateral weights), which keeps order 4 at extrema lying at the midpoint
 *     of a lateral sub-interval.
 *   PSI1_ROE: scalar laws only; psi^1 from the upwind ratio chosen by the
 *     sign of Roe's speed (Sec. 3.1) instead of the min form.
 *   SQUARE_2D: 2D only; a corner whose x- and y-interface orders differ
 *     (q1 != q2) computes F on the square stencil J_q1 x J_q1 and G on
 *     J_q2 x J_q2 (the square algorithm of Sec. 4 per direction) instead of
 *     both on the rectangle J_q1 x J_q2 of the default method.  Grids of at
 *     most 2^29 corners.
 * The batched step has no variants; acat_step_adjoint rejects FLO_HLL and
 * SQUARE_2D. */
enum { ACAT_FLAG_FLO_LF = 1, ACAT_FLAG_FLO_HLL = 2, ACAT_FLAG_PSI2_MODIFIED = 4, ACAT_FLAG_PSI1_ROE = 8,
       ACAT_FLAG_SQUARE_2D = 16 };

/* Device status bits (acat_device_status): non-finite output state,
 * non-positive density or pressure (Euler), and (replay) a recorded order
 * outside 1..P, replaced by 1. */
enum { ACAT_DEV_NONFINITE = 1, ACAT_DEV_NONPHYSICAL = 2, ACAT_DEV_BAD_ORDER = 4 };

/* Problem description (host struct, passed by pointer, read at each call). */
typedef struct {
  int32_t dim;    /* 1 or 2                                                     */
  int32_t nvar;   /* advection: 1; Burgers: 1 (1D only); Euler: 3 (1D), 4 (2D)   */
  int64_t nx;     /* cells in x, >= 2 max(P, 2)                                  */
  int64_t ny;     /* cells in y (2D), >= 2 max(P, 2); ignored in 1D              */
  int32_t flux;   /* ACAT_FLUX_*                                                 */
  int32_t P;      /* largest stencil half-width: 1..6 in 1D, 1..4 in 2D          */
  int32_t bc;     /* ACAT_BC_PERIODIC (wrap) or ACAT_BC_TRANSMISSIVE (clamp)     */
  int32_t flags;  /* ACAT_FLAG_* variants, 0 for the default method              */
  double gamma;   /* Euler: ratio of specific heats (Sec. 5.3 / 5.5 EOS)         */
  double ax, ay;  /* advection speeds (f = ax u, g = ay u)                       */
  double dx, dy;  /* grid spacings (> 0)                                         */
  double eps;     /* epsilon of the lateral weights I_L, I_R (Sec. 3.2), >= 0    */
  double theta;   /* admissibility threshold: psi^p >= theta, in (0, 1]          */
} acat_problem;

/* Per-interface decisions of one step (all device pointers).  order: p_s in
 * 1..P (1 = FL-CAT2 fallback); psi1: superbee blend weight where order is 1,
 * -1 elsewhere; alpha: Rusanov speed where order is 1, -1 elsewhere.  *_y
 * are used in 2D only.  In acat_step any pointer may be NULL (not
 * recorded); in acat_step_replay and acat_step_adjoint all used pointers
 * must be set. */
typedef struct {
  int8_t* order_x;
  double* psi1_x;
  double* alpha_x;
  int8_t* order_y;
  double* psi1_y;
  double* alpha_y;
} acat_decisions;

/* Bytes of device workspace acat_step / acat_step_replay need for `prob`. */
acat_status acat_workspace_size(const acat_problem* prob, size_t* bytes /* host */);

/* u_out = one ACAT step of u_in.  The time step is *dt_dev when dt_dev is
 * not NULL (device scalar, e.g. from acat_cfl_dt), else `dt` (> 0 or 0).
 * `dec` (nullable, host struct of device pointers) records the decisions. */
acat_status acat_step(const acat_problem* prob, const double* u_in, double* u_out, double dt,
                      const double* dt_dev, void* workspace, size_t workspace_bytes,
                      const acat_decisions* dec, void* stream);

/* One step with its own CFL time step: dt_dev[0] = the time step that
 * acat_max_wave_speed + acat_cfl_dt(cfl, t_final, t_dev) would give for u_in
 * (bit for bit), computed inside the step (the classification pass reduces
 * the wave speeds; no atomics, no extra pass over u_in), then u_out = the
 * step of u_in with it.  t_dev (nullable) is advanced as in acat_cfl_dt.
 * dt_dev (device scalar) is required; cfl > 0. */
acat_status acat_step_cfl(const acat_problem* prob, const double* u_in, double* u_out, double cfl, double t_final,
                          double* t_dev, double* dt_dev, void* workspace, size_t workspace_bytes,
                          const acat_decisions* dec, void* stream);

/* ---------------------------------------------------------------------
 * Allocation-free step, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  The same step as acat_step (same kernels, same results bit
 * for bit), with the workspace taken from one fixed array of
 * ACAT_NOALLOC_SCRATCH_BYTES in the library's static device memory, one per
 * GPU, held until the process ends.  The caller still owns u_in, u_out, the
 * optional decision maps and dt_dev; the call allocates and frees nothing.
 *   - ACAT_ERR_WORKSPACE when acat_workspace_size(prob) exceeds
 *     ACAT_NOALLOC_SCRATCH_BYTES (64 MiB: e.g. 2D Euler up to about 800^2
 *     cells, 1D Euler up to about 1.4 million cells); other errors as
 *     acat_step.
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents (nothing in it needs to start at zero).  Calls that
 *     overlap on one GPU (concurrent streams, or threads) race on it: the
 *     caller serialises them.
 * --------------------------------------------------------------------- */
#define ACAT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
acat_status acat_step_noalloc(const acat_problem* prob, const double* u_in, double* u_out, double dt,
                              const double* dt_dev, const acat_decisions* dec, void* stream);

/* The same step with the decisions frozen to `dec` (orders, psi1, alpha):
 * a smooth function of u_in, the forward map differentiated by
 * acat_step_adjoint. */
acat_status acat_step_replay(const acat_problem* prob, const double* u_in, double* u_out, double dt,
                             const double* dt_dev, void* workspace, size_t workspace_bytes,
                             const acat_decisions* dec, void* stream);

/* ---------------------------------------------------------------------
 * Adjoint (reverse mode) of one step with frozen decisions.  With
 * u_out = S(u_in) the map of acat_step_replay for the same `dec` and time
 * step, ubar_in = (dS/du_in)^T ubar_out: the conservative update's
 * transpose gives the interface flux adjoints Fbar = lambda (ubar_{i+1} -
 * ubar_i) (a transmissive edge flux enters one cell only: the missing
 * term is dropped), and each interface (1D) or corner (2D) recomputes its Taylor
 * recursion (Sec. 2.2; Sec. 4) and runs it backwards, with the analytic
 * flux Jacobians and the transposed centred-difference and time-
 * extrapolation weights; the FL-CAT2 blend (Sec. 3.1) is differentiated at
 * fixed psi1 and alpha.  Contributions are summed per cell in a fixed order
 * (deterministic; no atomics).
 *   - dec: the decisions of the forward step (all used pointers set); u_in:
 *     the forward step's input state; dt / dt_dev as in acat_step.
 *   - ubar_out, ubar_in: state-shaped adjoints; ubar_in may equal ubar_out
 *     (in place) but may not partially overlap it or overlap u_in.
 *   - Every order, flux and boundary of acat_step (the transposed clamp
 *     adds the contributions of ghost reads to the edge cells); the HLL
 *     variant is not differentiated (ACAT_ERR_UNSUPPORTED).  Recorded orders outside 1..P are taken as 1
 *     and set ACAT_DEV_BAD_ORDER.
 * --------------------------------------------------------------------- */
acat_status acat_adjoint_workspace_size(const acat_problem* prob, size_t* bytes /* host */);
acat_status acat_step_adjoint(const acat_problem* prob, const double* u_in, double dt, const double* dt_dev,
                              const acat_decisions* dec, const double* ubar_out, double* ubar_in,
                              void* workspace, size_t workspace_bytes, void* stream);

/* acat_step_adjoint without its classification and list passes: the
 * order-class map and per-class corner (2D) or interface (1D) lists are
 * read from `step_workspace`, the workspace of the forward step of the same
 * u_in whose decisions `dec` holds (acat_step or acat_step_cfl recording
 * into `dec`, or acat_step_replay of `dec`; Sec. 3 order selection, the
 * lists group the items by the order the step selected).  No call may have
 * written step_workspace since that step.  Results equal acat_step_adjoint's
 * bit for bit.  The pairing is the caller's: only the sizes are checked
 * (ACAT_ERR_WORKSPACE when step_workspace_bytes < acat_workspace_size(prob));
 * a workspace of another step gives wrong results, not an error.  The
 * library reads step_workspace and does not modify it; `workspace` is the
 * adjoint workspace as in acat_step_adjoint.  For a reverse sweep over many
 * steps this keeps one step workspace per recomputed step. */
acat_status acat_step_adjoint_lists(const acat_problem* prob, const double* u_in, double dt, const double* dt_dev,
                                    const acat_decisions* dec, const double* ubar_out, double* ubar_in,
                                    const void* step_workspace, size_t step_workspace_bytes, void* workspace,
                                    size_t workspace_bytes, void* stream);

/* smax_dev[d] = max over cells of the spectral radius of the flux Jacobian
 * in direction d (d < dim): |u| (Burgers), |a| (advection), |v|+c (Euler). */
acat_status acat_max_wave_speed(const acat_problem* prob, const double* u, double* smax_dev, void* stream);

/* dt_dev[0] = CFL time step from smax_dev: 1D cfl dx / s; 2D (Sec. 5.5)
 * cfl/2 min(dx/s_x, dy/s_y).  With t_dev not NULL the step is clipped so
 * that t does not pass t_final (0 once t >= t_final) and t_dev[0] += dt. */
acat_status acat_cfl_dt(const acat_problem* prob, const double* smax_dev, double cfl, double t_final,
                        double* t_dev, double* dt_dev, void* stream);

/* ---------------------------------------------------------------------
 * Batched step: nprob independent 1D problems with one flux, each with its
 * own cell count n[b], largest half-width P[b], boundary bc[b], spacing
 * dx[b] and time step dt[b], advanced together (one classification launch,
 * one persistent flux launch over all problems and order classes, or one
 * per order class with a launch table below).  Per problem
 * the result equals acat_step bit for bit.
 *   States: SoA over the concatenated cells, u[var][coff_b + i] with
 *   coff_b = n[0] + ... + n[b-1] (total C cells: arrays of nvar * C).
 * The descriptor is a host struct of host arrays; acat_batch_init copies
 * it into the workspace once (synchronously), together with the problem
 * index of every interface and of every cell (4 bytes each); every later
 * call takes the same descriptor and workspace.
 * --------------------------------------------------------------------- */
typedef struct {
  int32_t nvar;         /* as in acat_problem (1D)                             */
  int32_t flux;
  double gamma, ax;
  double eps, theta;
  int32_t nprob;        /* >= 1                                               */
  const int64_t* n;     /* host [nprob] cells, >= max(8, 2 max(P[b], 2))      */
  const int32_t* P;     /* host [nprob] 1..4                                   */
  const int32_t* bc;    /* host [nprob] ACAT_BC_*                              */
  const double* dx;     /* host [nprob] > 0                                    */
  /* host [8] or NULL.  NULL: every order class in one persistent launch of
   * 256-thread blocks, the grid shared among the classes by their work.  A
   * table: one launch per order class p = 1..4 with the shape of entries
   * 2(p-1) and 2(p-1)+1 = waves per block (1, 2 or 4; 0 = 4) and persistent
   * blocks per CU (0 = the occupancy limit, else 1..32).  Every choice gives
   * the same results bit for bit; the autotuner chooses by timing. */
  const int32_t* launch;
} acat_batch;

acat_status acat_batch_workspace_size(const acat_batch* batch, size_t* bytes /* host */);
acat_status acat_batch_init(const acat_batch* batch, void* workspace, size_t workspace_bytes);
/* u_out = one ACAT step of every problem with dt_dev[b] (device [nprob]). */
acat_status acat_step_batched(const acat_batch* batch, const double* u_in, double* u_out, const double* dt_dev,
                              void* workspace, size_t workspace_bytes, void* stream);
/* The same step, and then dt_dev[b] = the time step that acat_batched_cfl_dt
 * (cfl) gives for u_out, bit for bit: the update pass reduces the new
 * state's wave speeds (one partial maximum per wavefront that lies inside
 * one problem, atomic maxima on the bit patterns for wavefronts that
 * straddle problems; max is exact in any order) and a last small launch
 * folds them per problem, so no extra pass over u_out is made.  dt_dev is
 * read as this step's time steps before it is overwritten; cfl > 0.  The
 * first dt_dev comes from acat_batched_cfl_dt.  Errors as acat_step_batched,
 * and ACAT_ERR_ARG for cfl <= 0 or NaN. */
acat_status acat_step_batched_cfl(const acat_batch* batch, const double* u_in, double* u_out, double* dt_dev,
                                  double cfl, void* workspace, size_t workspace_bytes, void* stream);
/* dt_dev[b] = cfl dx[b] / (max spectral radius over problem b of u). */
acat_status acat_batched_cfl_dt(const acat_batch* batch, const double* u, double cfl, double* dt_dev,
                                void* workspace, size_t workspace_bytes, void* stream);

/* Reads and clears the device status bits accumulated by steps on this
 * device (synchronises `stream`).  flags_host receives ACAT_DEV_* bits. */
acat_status acat_device_status(int32_t* flags_host, void* stream);

/* Static description of a status code. */
const char* acat_status_string(acat_status s);

/* Kernel timer.  acat_profile_enable(1) clears the record and starts
 * bracketing every kernel launch of the library with two HIP events on the
 * launch stream (launches into a capturing stream are not timed);
 * acat_profile_enable(0) clears and stops.  acat_profile_read() waits for
 * the recorded events and returns, per kernel name (at most max_kernels, in
 * order of first launch), the total time in ms and the number of launches;
 * names receives 64-byte NUL-terminated strings.  *n_kernels is the number of
 * distinct kernels recorded (may exceed max_kernels). */
acat_status acat_profile_enable(int32_t on);
acat_status acat_profile_read(int32_t max_kernels, char* names /* host [max][64] */, double* total_ms,
                              int64_t* launches, int32_t* n_kernels);

/* Measured FP64 issue rate: launches `blocks` blocks of 256 threads, each
 * thread running 16 independent chains of `iters` fused multiply-adds
 * (blocks * 256 * iters * 16 FMAs = that many times 2 flops), and writes one
 * value per thread to out[blocks * 256] (device, caller-owned; out_len
 * elements).  The caller times the launch on `stream` (events) to obtain the
 * FP64 rate at the running clock, which the roofline reports next to the
 * published peak.  ACAT_ERR_ARG if blocks is outside 1..2^20, iters < 1 or
 * out_len < blocks * 256. */
acat_status acat_fp64_fma_rate(int32_t blocks, int32_t iters, double* out, int64_t out_len, void* stream);

/* Coefficient tables the kernels use for half-width p = 1..6 (host arrays, row
 * major): g1[2p][2p] first derivatives at the nodes, gt[2p][2p] k-th time
 * derivatives at 0 (k = 0..2p-1), eta[2p] interface weights, tau[2p] the
 * (2p-1)-th derivative weights.  For inspection and tests. */
acat_status acat_coefficients(int32_t p, double* g1, double* gt, double* eta, double* tau);

#ifdef __cplusplus
}
#endif

#endif /* ACAT_H */
