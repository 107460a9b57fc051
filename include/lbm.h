/*
 * lbm.h -- C ABI of the MI355X (gfx950) implementation of the upscaled
 * Brinkman lattice Boltzmann method of J. Li and D. Brown, "Upscaled Lattice
 * Boltzmann Method for Simulations of Flows in Heterogeneous Porous Media"
 * (arXiv:1312.0195).
 *
 * All quantities are in lattice units (dx = dt = c = 1, c_s^2 = 1/3). The
 * D2Q9 populations are numbered as in Sec. 2 of the paper:
 *   0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1).
 * Fields are row-major [ny][nx] with x fastest.
 *
 * Memory ownership: every device buffer passed in is owned by the caller. The
 * library never allocates or frees device memory; scratch space comes from a
 * caller-provided workspace whose size the *_workspace_bytes functions
 * report. An lbm_handle is host memory owned by the library (freed by
 * lbm_destroy); it only refers to the caller's workspace.
 *
 * Streams and synchronisation: work is queued on the hipStream_t given at
 * set-up. Calls that return values into host memory (steps_done, mean_u)
 * synchronise that stream before they return; the others are asynchronous.
 *
 * Errors: every entry point returns an lbm_status. Parameters are checked on
 * the host before anything is launched. No exception or abort crosses the
 * ABI. lbm_last_error() gives a thread-local description of the last failure.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* invalid argument (checked on the host) */
    LBM_EDEVICE = -2,     /* a HIP call failed */
    LBM_ENOTCONV = -3,    /* step cap reached before the tolerance */
    LBM_ENONFINITE = -4,  /* NaN or Inf in the mean velocity */
    LBM_EWORKSPACE = -5   /* workspace missing, misaligned or too small */
} lbm_status;

/* Population storage of the fine-grid solver. */
enum {
    LBM_F32_SHIFTED = 0, /* FP32 deviations f_a - w_a rho0, FP64 collision arithmetic */
    LBM_F64 = 1,         /* FP64 deviations (reference-precision runs) */
    LBM_F32_FAST = 2     /* fine solver only: FP32 deviations and FP32 collision
                            arithmetic (Shan-Chen form only), written so that
                            the rounded constants bias neither mass nor
                            momentum: within 2.7e-6 of FP64 state in the
                            velocity after 20 000 steps of a 2048^2 field at
                            tau 0.8 (7.0e-6 at tau 0.53), against 2.0e-7 for
                            LBM_F32_SHIFTED; about 14% faster per step.
                            tau outside [1/2, 2] loses the exact 1 - 1/tau */
};

/* Form of the time step. Both give the same populations up to rounding (with
 * the linear f_eq the two forms are algebraically equal); they differ in cost.
 * The coarse and local solvers run the Shan-Chen form only. */
enum {
    LBM_SCHEME_SHAN_CHEN = 0, /* Sec. 2.2: Eqs. final-ueq-of-S-C, f-evolution-of-S-C */
    LBM_SCHEME_GUO = 1        /* Sec. 2.1: Eqs. f-evolution-of-Guo, ueq-of-Guo,
                                 Fi-of-Guo, f_m-depends-on-u, explicit-u-in-Guo;
                                 scalar permeability only */
};

/* Kind of permeability given per cell. */
enum {
    LBM_PERM_SCALAR = 1, /* kappa(x), Eq. f_m-depends-on-u */
    LBM_PERM_TENSOR = 4  /* [kxx, kxy, kyx, kyy](x), Eq. f_m-depends-on-u-and-tensor-k */
};

/* Parameters of one lattice (Sec. 2). tau >= 1/2 sets nu_eff = (tau - 1/2)/3;
 * nu is the viscosity in the drag term, independent of nu_eff (Eq.
 * Brinkman-like); eps is the porosity; (gx, gy) the uniform body force per
 * unit mass G, used when no per-cell force field is given. */
typedef struct {
    int32_t nx, ny;
    double tau;
    double eps;
    double nu;
    double rho0;
    double gx, gy;
    int32_t walls_y;   /* 0: periodic in y; 1: halfway bounce-back walls half a
                          cell below row 0 and above row ny-1 (x is periodic) */
    int32_t pop_dtype; /* LBM_F32_SHIFTED or LBM_F64 */
    int32_t perm_kind; /* LBM_PERM_SCALAR or LBM_PERM_TENSOR */
    int32_t scheme;    /* LBM_SCHEME_SHAN_CHEN or LBM_SCHEME_GUO (fine solver) */
} lbm_params;

typedef struct lbm_handle lbm_handle;

/* ---------------------------------------------------------------------------
 * Fine-grid solver: the time stepping of Sec. 2.2 (Eqs. feq, explicit-u-in-Guo,
 * final-ueq-of-S-C, f-evolution-of-S-C) on an nx x ny lattice.
 * ------------------------------------------------------------------------- */

/* Bytes of workspace lbm_init needs for these parameters (0 if invalid). */
size_t lbm_workspace_bytes(const lbm_params *p);

/* Set up a solver at the rest state f_a = w_a rho0.
 *   d_perm  : device FP64, [ny][nx] (scalar) or [ny][nx][4] (tensor), read
 *             once. Scalars must be > 0 (+inf means no drag); tensors must be
 *             invertible. Invalid values give LBM_EINVAL.
 *   d_force : device FP64 [ny][nx][2] per-cell G, or NULL for (gx, gy).
 *   d_ws    : device workspace of ws_bytes >= lbm_workspace_bytes(p),
 *             256-byte aligned; it must stay alive until lbm_destroy.
 * Synchronises the stream (the permeability check is read back). */
lbm_status lbm_init(lbm_handle **h, const lbm_params *p, const double *d_perm,
                    const double *d_force, void *d_ws, size_t ws_bytes, hipStream_t stream);

/* Advance up to max_steps time steps. With check_every > 0 the volume-averaged
 * flow velocity (Sec. 3, FP64 reduction) is taken every check_every steps;
 * with tol > 0 the call returns LBM_OK once the change between two checks is
 * <= tol times its norm, and LBM_ENOTCONV if max_steps pass first. tol <= 0
 * runs exactly max_steps. steps_done (may be NULL) gets the steps taken by
 * this call; mean_u (may be NULL) the mean velocity of the final state.
 * Synchronises the stream when a check runs or mean_u is requested. */
lbm_status lbm_step(lbm_handle *h, int64_t max_steps, double tol, int32_t check_every,
                    int64_t *steps_done, double mean_u[2]);

/* Flow velocity u (Eq. u-of-S-C) and density of the current state.
 *   d_u   : device FP64 [2][ny][nx] (ux plane, then uy plane)
 *   d_rho : device FP64 [ny][nx], or NULL. */
lbm_status lbm_fields(lbm_handle *h, double *d_u, double *d_rho);

/* Full populations f_a (not shifted) of the current state, device FP64
 * [9][ny][nx], pre-collision at the current time step. */
lbm_status lbm_get_populations(lbm_handle *h, double *d_f);

/* Replace the state by the populations d_f (same layout as above), e.g. to
 * resume from a checkpoint. The step counter is left unchanged. */
lbm_status lbm_set_populations(lbm_handle *h, const double *d_f);

/* Total time steps taken since lbm_init. */
int64_t lbm_steps_total(const lbm_handle *h);

void lbm_destroy(lbm_handle *h);

/* ---------------------------------------------------------------------------
 * Batched local problems: effective permeability per subdomain (Sec. 3).
 * Each patch is a periodic side x side window of the fine permeability field,
 * run from rest under G1 = (g, 0) and/or G2 = (0, g) until its own mean
 * velocity converges; then Eq. tensor-kappa gives
 *   kxx = nu ubar1_x / g, kxy = nu ubar2_x / g, kyx = nu ubar1_y / g,
 *   kyy = nu ubar2_y / g.
 * All items of one call run in one persistent launch; when a call mixes sides
 * that leave one cell per thread with larger ones, in two launches side by
 * side on streams the library owns (default priority, created on first use
 * and kept per device), forked from and joined back to `stream`, so the call
 * stays ordered on `stream` like a single launch. On a 256-CU device the two
 * streams carry complementary CU masks, the single-cell launch getting a
 * share of the CUs in proportion to its share of the cells (a multiple of 32
 * CUs, 4 per XCD), so that neither launch waits for the other's CUs.
 * ------------------------------------------------------------------------- */

typedef struct {
    double tau, eps, nu;  /* as in lbm_params */
    double g;             /* drive magnitude G_const > 0 */
    double tol;           /* relative change of the mean velocity between checks */
    int32_t check_every;  /* steps between checks, even and >= 2 */
    int64_t max_steps;    /* per-item cap (rounded up to a multiple of check_every) */
    int32_t pop_dtype;    /* LBM_F32_SHIFTED: FP32 state and arithmetic (fast);
                             LBM_F64: FP64 state and arithmetic, needed where a
                             step moves the state by less than half an FP32
                             ulp (tau near 1/2 with weak drag) */
    int32_t avg_margin;   /* oversampling (an addition to the paper, which
                             names it as a treatment for high contrast): the
                             mean velocity, for the convergence test and for
                             Eq. tensor-kappa, is taken over the inner window
                             [m, side - m)^2 only; 0 = the whole patch. Every
                             side must exceed 2 m. */
    int32_t schedule;     /* order in which the items of one side start:
                             LBM_SCHEDULE_GIVEN or LBM_SCHEDULE_COST. Results
                             do not depend on it, only the run time. */
    int32_t fp32_step_budget; /* FP32 state only (0: no budget). The FP32 state
                             is stored rebased on the item's mean momentum, so
                             a slowly relaxing but nearly uniform flow keeps
                             its precision; in a patch with nearly blocked
                             directions the non-uniform part dominates, and a
                             converged FP32 state can stop short of the fixed
                             point by a few 1e-4 of a blocked direction's own
                             small K_eff. An item that has not converged after
                             this many steps (rounded up to a check) is
                             stopped and run again from rest with FP64 state
                             (a second launch on `stream`; sides up to 45),
                             which reports its own steps and flag. Larger
                             sides finish in FP32 and get flag 3. */
} lbm_local_params;

/* Start order of the local problems. An item's step count varies by orders
 * of magnitude between patches, so a batch ends when its slowest items end.
 * LBM_SCHEDULE_COST starts the items of each side in descending order of a
 * predicted cost, ln(t_drag + t_pres) + sd(ln kappa) over the patch: a
 * permeable patch relaxes slowly, on the time scale t_drag = mean kappa /
 * (eps nu) of the drag term; a nearly impermeable one too, since where the
 * drag dominates the density diffuses with coefficient c_s^2 kappa / (eps nu),
 * t_pres = side^2 eps nu / (pi^2 c_s^2 kappa) with the geometric mean of
 * kappa; a strongly heterogeneous patch has nearly blocked directions whose
 * small velocities converge slowly. Computed by a device pre-pass and binned
 * in steps of 1/4 (ties in any order), so the long items start first and the
 * short ones fill in behind them. The largest sides of a call (those that
 * fill a workgroup with more than one cell per thread) share one queue, with
 * the prediction lowered by 2 ln(side / largest side) for their cheaper
 * steps. */
enum {
    LBM_SCHEDULE_GIVEN = 0, /* the order of the patch arrays (within a side) */
    LBM_SCHEDULE_COST = 1   /* longest predicted first */
};

/* One row of the tile table: how items of side `side` are laid out on a
 * workgroup of block_threads threads. slot_threads threads share one item
 * (each holding ceil(side^2 / slot_threads) cells, at most 4); a workgroup
 * runs block_threads / slot_threads items side by side. Items of sides not in
 * the table use the built-in choice. */
typedef struct {
    int32_t side;
    int32_t slot_threads;
} lbm_local_tile;

/* Largest patch side the local solver accepts. */
int32_t lbm_local_max_side(void);

size_t lbm_local_workspace_bytes(int32_t n_patches);

/* h_x0, h_y0, h_side, h_drive_mask: HOST int32 arrays of n_patches entries
 *   (origin of the window in the field, side in [1, lbm_local_max_side()],
 *   drive bits: 1 = x drive, 2 = y drive).
 * d_kappa_field: device FP64 [fny][fnx]; windows wrap periodically.
 * d_keff : device FP64 [n_patches][4] = kxx, kxy, kyx, kyy (entries of a
 *          skipped drive are NaN).
 * d_steps: device int32 [n_patches][2] steps taken per drive (or NULL).
 * d_flags: device int32 [n_patches][2]: 0 converged, 1 step cap reached,
 *          2 non-finite, 3 converged in FP32 state past fp32_step_budget
 *          (side too large for the FP64 re-run), -1 drive skipped (or NULL).
 * tiles/n_tiles: optional tile table (NULL/0 for the built-in one).
 * block_threads: workgroup size, 256, 512 or 1024 (0 for 1024); FP64 items
 *          run with at most 512 (tile rows asking for more are ignored), so
 *          their sides are limited to side^2 <= 4 x 512.
 * Asynchronous; the host arrays may be reused when the call returns. */
lbm_status lbm_local_keff(const lbm_local_params *lp, int32_t n_patches, const int32_t *h_x0,
                          const int32_t *h_y0, const int32_t *h_side, const int32_t *h_drive_mask,
                          const double *d_kappa_field, int32_t fnx, int32_t fny, double *d_keff,
                          int32_t *d_steps, int32_t *d_flags, const lbm_local_tile *tiles,
                          int32_t n_tiles, int32_t block_threads, void *d_ws, size_t ws_bytes,
                          hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Coarse-grid solve (Sec. 3, Sec. 4.3): the same scheme on the grid coarsened
 * by r, with the effective permeability per coarse cell. The physical rho0,
 * nu_eff, eps, nu and G are kept while dx and dt both grow by r, so in
 * lattice units tau_c = 1/2 + (tau_f - 1/2)/r, nu_c = nu_f / r,
 * kappa_c = kappa_f / r^2 and G_c = r G_f; velocities are unchanged.
 * ------------------------------------------------------------------------- */

enum { LBM_KEFF_SCALAR = 0, LBM_KEFF_TENSOR = 1 };

/* Coarse lattice parameters for a fine lattice coarsened by r (the mapping
 * above; uniform force scaled by r). */
lbm_status lbm_coarse_params(const lbm_params *fine, int32_t r, lbm_params *coarse);

size_t lbm_coarse_workspace_bytes(int32_t ncx, int32_t ncy);

/* fine     : fine-lattice parameters (nx, ny divisible by r); walls_y must be
 *            0 (the paper's coarse runs are periodic).
 * d_keff   : device FP64 [ncy][ncx][4] (kxx, kxy, kyx, kyy) in FINE lattice
 *            units, as lbm_local_keff returns them.
 * keff_mode: LBM_KEFF_SCALAR uses (kxx + kyy)/2 per cell (the scalar kappa*
 *            of Sec. 4.3), LBM_KEFF_TENSOR the full tensor (Eq.
 *            f_m-depends-on-u-and-tensor-k).
 * d_force  : device FP64 [ncy][ncx][2] G per coarse cell in FINE lattice
 *            units, or NULL for (fine->gx, fine->gy).
 * Runs from rest until the relative L2 change of the velocity field between
 * checks every check_every coarse steps is <= tol (or max_steps coarse
 * steps). d_u: device FP64 [2][ncy][ncx]; d_rho: [ncy][ncx] or NULL.
 * Synchronises the stream (steps_done is returned). */
lbm_status lbm_coarse_solve(const lbm_params *fine, int32_t r, const double *d_keff,
                            int32_t keff_mode, const double *d_force, int64_t max_steps,
                            double tol, int32_t check_every, double *d_u, double *d_rho,
                            int64_t *steps_done, void *d_ws, size_t ws_bytes,
                            hipStream_t stream);

/* Mean of every r x r block of nplanes consecutive FP64 fields [plane][ny][nx]
 * (device) into d_out [plane][ny/r][nx/r] (device), summed in FP64 in a fixed
 * order: the fine-grid quantity that a coarse cell represents (Sec. 4.3
 * compares coarse results with fine results averaged over each subdomain).
 * r must divide nx and ny. Asynchronous. */
lbm_status lbm_block_average(const double *d_in, int32_t nx, int32_t ny, int32_t nplanes, int32_t r,
                             double *d_out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Learned K_eff surrogate (an addition to the paper's method: it learns the
 * map that the local problems of Sec. 3 compute with Eq. tensor-kappa).
 *
 * Network on a periodic 32 x 32 patch of log K, with m = mean(log K):
 *   x = log K - m; a1 = relu(conv3x3(x; W1, b1))       1 -> 32 channels
 *   a2..a4 = relu(conv3x3(a; Wl, bl))                   32 -> 32 channels
 *   s = four series/parallel estimates of exp(x), as logs: the mean over rows
 *       of each row's harmonic mean; the harmonic mean over columns of each
 *       column's arithmetic mean; the same two with rows and columns exchanged
 *   z = [mean over pixels of a4, m, s] (37); h = relu(M1 z + c1) (32 hidden)
 *   prediction = M2 h + c2 + m  = (log kxx, log kyy)
 * Convolutions wrap periodically: out[y][x] = sum over taps (dy, dx) in
 * {-1,0,1}^2 of in[y + dy][x + dx] W[tap], tap = 3 (dy + 1) + (dx + 1).
 * Parameters: one FP32 vector, in this order:
 *   W1[9][32], b1[32], then for l = 2, 3, 4: Wl[9][32 ci][32 co], bl[32],
 *   M1[32][37], c1[32], M2[2][32], c2[2]          (lbm_cnn_param_count() floats)
 * The four convolutions run on BF16 MFMA with FP32 accumulation (conv1 with
 * its nine taps as the K dimension, the input and W1 rounded to BF16); the
 * features, the head, the loss, the conv1 gradients and Adam are FP32.
 * Inputs: d_logk FP32 [batch][32][32] (x fastest).
 * Symmetries: K_eff transforms with the eight symmetries of the square. A
 * symmetry code sym = t + 2 fx + 4 fy (0..7) means: output pixel (y, x) of the
 * transformed patch reads input pixel (v, u), where (u, v) = (x, y), exchanged
 * if t, then u -> 31 - u if fx and v -> 31 - v if fy; with t the network's
 * outputs are (log kyy, log kxx) of the original patch.
 * ------------------------------------------------------------------------- */

int32_t lbm_cnn_param_count(void);

/* Workspace for a batch: training != 0 adds the stored activations and
 * gradient buffers (about 256 KB per patch). It also holds the packed weights
 * and the counter from which the forward kernel's workgroups claim patches,
 * so calls that may run at the same time need workspaces of their own. */
size_t lbm_cnn_workspace_bytes(int32_t batch, int32_t training);

/* The per-patch statistics of lbm_cnn_forward's d_stats alone (same
 * arithmetic, bit-identical values), without running the network: lets a
 * caller decide which patches go to the LBM before, or while, the network
 * runs. d_logk FP32 [batch][32][32], d_stats FP32 [batch][8]. Asynchronous. */
lbm_status lbm_patch_stats(int32_t batch, const float *d_logk, float *d_stats, hipStream_t stream);

/* d_pred : FP32 [batch][2] predicted (log kxx, log kyy) of each patch, the
 *          mean over symmetry codes 0..n_sym-1 (1 <= n_sym <= 8, else
 *          LBM_EINVAL) of the network applied to the transformed patch, each
 *          mapped back to the patch's own axes. n_sym = 1: the plain network.
 * d_stats: FP32 [batch][8] per-patch mean, standard deviation and lag-1
 *          autocorrelations along x and y of log K, then the four features s
 *          (or NULL); used to flag patches outside the training distribution.
 * Asynchronous. */
lbm_status lbm_cnn_forward(const float *d_params, int32_t batch, const float *d_logk, int32_t n_sym,
                           float *d_pred, float *d_stats, void *d_ws, size_t ws_bytes, hipStream_t stream);

/* lbm_cnn_forward on at most max_workgroups workgroups (0: one per CU, as
 * lbm_cnn_forward; < 0: LBM_EINVAL). Each workgroup claims patches one at a
 * time, so fewer workgroups only lower the network's share of the device:
 * the CUs it leaves free serve work on other streams at once, e.g. the batched
 * local LBM that the surrogate path runs beside it. Results do not depend on
 * the cap. */
lbm_status lbm_cnn_forward_limited(const float *d_params, int32_t batch, const float *d_logk, int32_t n_sym,
                                   float *d_pred, float *d_stats, int32_t max_workgroups, void *d_ws,
                                   size_t ws_bytes, hipStream_t stream);

/* lbm_cnn_forward_limited with, in place of the statistics, the spread of
 * the symmetric predictions: d_spread FP32 [batch][2] gets, for log kxx and
 * log kyy, the largest minus the smallest of the n_sym predictions whose mean
 * is d_pred (0 for n_sym = 1). The symmetries of the square map a patch's
 * K_eff tensor exactly onto that of the transformed patch, so their
 * disagreement measures how far the network is from the map it learned;
 * the surrogate path sends patches with a large spread to the LBM.
 * d_pred and d_spread must not be NULL. Asynchronous. */
lbm_status lbm_cnn_forward_spread(const float *d_params, int32_t batch, const float *d_logk, int32_t n_sym,
                                  float *d_pred, float *d_spread, int32_t max_workgroups, void *d_ws,
                                  size_t ws_bytes, hipStream_t stream);

/* lbm_cnn_forward_limited without a workspace argument, for callers that
 * cannot allocate device memory during a run (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc). The call allocates
 * nothing: the packed weights and the patch counter live in a static device
 * array of the library (128 KB per device, reserved for the life of the
 * process); the first call on a device looks up its address. Inputs and
 * outputs are as in lbm_cnn_forward_limited; results are bit-identical to it.
 * Every call on one device shares that array, so calls that overlap on one
 * device (other streams, other host threads) race and must be serialised by
 * the caller; each call clears what it needs at its start. A call whose
 * scratch would exceed the reserved size returns LBM_EINVAL (the inference
 * scratch does not depend on the batch, so none does today). Asynchronous. */
lbm_status lbm_cnn_forward_noalloc(const float *d_params, int32_t batch, const float *d_logk, int32_t n_sym,
                                   float *d_pred, float *d_stats, int32_t max_workgroups, hipStream_t stream);

/* Loss = mean over the batch and both outputs of (prediction - target)^2,
 * d_target FP32 [batch][2] (log kxx, log kyy of the untransformed patch).
 * d_sym: int8 [batch] symmetry code applied to each patch (training-time
 * augmentation; NULL = none); a transposed patch is compared with the
 * exchanged target. Writes d_grad (FP32, one per parameter, may be NULL),
 * d_loss (one FP32, may be NULL) and the batch's predictions d_pred (mapped
 * back to the untransformed patch's axes, like d_target). Gradients are summed in a fixed order
 * (deterministic). Asynchronous. */
lbm_status lbm_cnn_gradients(const float *d_params, int32_t batch, const float *d_logk, const int8_t *d_sym,
                             const float *d_target, float *d_grad, float *d_loss, float *d_pred,
                             void *d_ws, size_t ws_bytes, hipStream_t stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with the
 * 1-based step count `step`) on the FP32 parameters, with the first and second
 * moments d_adam_m, d_adam_v (FP32, parameter-sized, zero before step 1).
 * d_sym as in lbm_cnn_gradients. d_loss (may be NULL) gets the batch loss
 * before the update. Asynchronous. */
lbm_status lbm_cnn_train_step(float *d_params, float *d_adam_m, float *d_adam_v, int32_t step, float lr,
                              int32_t batch, const float *d_logk, const int8_t *d_sym, const float *d_target,
                              float *d_loss, void *d_ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Three-dimensional fine grid: the same step on the D3Q19 lattice (Sec. 2:
 * three-dimensional problems use D3Q19, with their own velocities and
 * weights and the algorithm unchanged): Eqs. explicit-u-in-Guo,
 * final-ueq-of-S-C, feq and f-evolution-of-S-C with three velocity
 * components, a scalar permeability per cell and a uniform force.
 *
 * Population order, also the layout of lbm3d_get/set_populations: 0 rest;
 * 1..6: +x, -x, +y, -y, +z, -z (weight 1/18); 7..10: +x+y, -x-y, +x-y, -x+y;
 * 11..14: +x+z, -x-z, +x-z, -x+z; 15..18: +y+z, -y-z, +y-z, -y+z (1/36);
 * rest 1/3. Cells are x-fastest: index (z ny + y) nx + x.
 * ------------------------------------------------------------------------- */

typedef struct {
    int32_t nx, ny, nz;   /* (nx ny nz + 65536) x 4 B (FP32) or 8 B (FP64) below 4 GiB */
    double tau;           /* >= 1/2 */
    double eps, nu, rho0; /* as in lbm_params */
    double gx, gy, gz;    /* uniform body force per unit mass G */
    int32_t walls_z;      /* 0: periodic in z; 1: halfway bounce-back walls half a
                             cell below plane 0 and above plane nz-1 (x and y
                             are periodic) */
    int32_t pop_dtype;    /* LBM_F32_SHIFTED or LBM_F64 */
} lbm3d_params;

typedef struct lbm3d_handle lbm3d_handle;

/* Bytes of workspace lbm3d_init needs (0 if the parameters are invalid). */
size_t lbm3d_workspace_bytes(const lbm3d_params *p);

/* Set up a solver at the rest state f_a = w_a rho0.
 *   d_kappa : device FP64 [nz][ny][nx], read once; values must be > 0
 *             (+inf: no drag), else LBM_EINVAL.
 *   d_ws    : device workspace, >= lbm3d_workspace_bytes(p), 256-byte
 *             aligned, alive until lbm3d_destroy (caller-owned).
 * Synchronises the stream (the permeability check is read back). */
lbm_status lbm3d_init(lbm3d_handle **h, const lbm3d_params *p, const double *d_kappa, void *d_ws,
                      size_t ws_bytes, hipStream_t stream);

/* Advance up to max_steps steps, one launch per step. check_every, tol,
 * steps_done and mean_u (three components, FP64 volume average of the flow
 * velocity) behave as in lbm_step. */
lbm_status lbm3d_step(lbm3d_handle *h, int64_t max_steps, double tol, int32_t check_every,
                      int64_t *steps_done, double mean_u[3]);

/* Flow velocity and density of the current state.
 *   d_u   : device FP64 [3][nz][ny][nx] (u_x, u_y, u_z planes), or NULL
 *   d_rho : device FP64 [nz][ny][nx], or NULL (not both NULL). */
lbm_status lbm3d_fields(lbm3d_handle *h, double *d_u, double *d_rho);

/* Full pre-collision populations, device FP64 [19][nz][ny][nx] (order above). */
lbm_status lbm3d_get_populations(lbm3d_handle *h, double *d_f);

/* Replace the state by d_f (same layout); the step counter is kept. */
lbm_status lbm3d_set_populations(lbm3d_handle *h, const double *d_f);

int64_t lbm3d_steps_total(const lbm3d_handle *h);

void lbm3d_destroy(lbm3d_handle *h);

/* ---------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------- */

const char *lbm_status_str(lbm_status s);
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
