/*
 * grpic.h -- C ABI of libgrpic.so, the MI355X (gfx950) implementation of the
 * GRPIC particle step of Chen, Luepker & Yuan, "Introducing APERTURE: A
 * GPU-based General Relativistic Particle-in-Cell Simulation Framework"
 * (arXiv:2503.04558): field gather, generalised Boris kick, geodesic
 * predictor-corrector and Esirkepov current deposition on a 2D axisymmetric
 * Kerr-Schild (ln r, theta) grid.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: c = 1, Heaviside-Lorentz (Sec. 2.1).  Momenta u_i are the covariant
 * Kerr-Schild components per unit mass; positions are stored as a cell index
 * plus an offset in grid units.
 *
 * Grid: nr x nth cells.  Vertex i lies at ln r = lnr0 + i*dlnr (natural log),
 * vertex j at theta = j*dth with dth = pi/nth.  Every grid array (the six
 * field components, the three current components) has nr + 1 + 2*guard rows
 * of `pitch` elements; grid point (i, j) of a component lives at element
 * (i + guard)*pitch + (j + guard), rows along r, theta contiguous.  A
 * component with Yee stagger (s_r, s_th) (Sec. 2.1, Fig. Yee) stores the
 * value at (i + s_r, j + s_th):
 *   D^r, B^th, F^r : (1/2, 0)     D^th, B^r, F^th : (0, 1/2)
 *   D^ph, G^ph     : (0, 0)       B^ph            : (1/2, 1/2)
 * guard >= 2 and pitch >= nth + 1 + 2*guard are required, and a grid array
 * of (nr + 1 + 2*guard) x pitch doubles must stay below 4 GiB (the kernels
 * address grid arrays with 32-bit offsets).
 *
 * Particles (structure of arrays, one element per particle):
 *   cell  int32   i*nth + j of the cell holding the particle, -1 = removed
 *   xr,xth        offsets in the cell, xi = i + xr, eta = j + xth, in [0, 1]
 *   ur,uth,uph    covariant momenta u_r, u_th, u_ph
 *   w             macro-particle weight
 *   sp    uint8   species index into the species table
 *   phi           optional accumulated azimuth (NULL: not tracked)
 *   tag   uint64  optional identity of the particle (NULL: none); it keys
 *                 the random numbers of grpic_push_deposit_qed, so that its
 *                 draws do not depend on the order of the particles
 * Precision GRPIC_FP64: xr..w and phi are double.  GRPIC_FP32_SPLIT: xr..w are
 * float (the position keeps its integer cell exactly; fields are float too);
 * the kick and the predictor-corrector run in float on offsets from the start
 * cell, except in rows with r < 2M and in the 64-cell tiles within ~5.7
 * degrees of the axis (double there, on the same float state); the deposit
 * is evaluated in double on the stored end point and the current arrays stay
 * double.
 *
 * Current output is in flux form (the quantities eq. integral-form consumes):
 *   F^r_{i+1/2,j} = J^r A^D_r,  F^th_{i,j+1/2} = J^th A^D_th,  G^ph_{ij} = J^ph dV,
 * accumulated (+=) over all steps of a call.  Dividing by the areas A^D and
 * volumes dV (Sec. 2.3, after the deposit loop) is left to the caller.
 *
 * Memory: every array pointer is a DEVICE pointer owned by the caller; the
 * library allocates no device memory.  Workspaces are caller-provided and
 * sized by the *_bytes helpers.  Structures passed by pointer are read on the
 * host during the call only.
 *
 * Streams: every call is enqueued on `stream` (a hipStream_t, NULL = the
 * default stream) and returns once enqueued; results are valid after the
 * stream is synchronised.
 *
 * Errors: every int-returning call returns 0 on success or a negative
 * GRPIC_E* code and then enqueues nothing; grpic_last_error() returns a
 * thread-local message for the last failure.  No C++ exception crosses the
 * ABI.
 */
#ifndef GRPIC_H_
#define GRPIC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRPIC_OK 0
#define GRPIC_EINVAL (-1)   /* bad argument: NULL pointer, bad size, inconsistent grid, ... */
#define GRPIC_ERANGE (-2)   /* dt above the light-crossing time of the smallest cell        */
#define GRPIC_ENOMEM (-3)   /* caller-provided workspace too small                          */
#define GRPIC_EHIP   (-4)   /* HIP runtime or launch failure                                */

#define GRPIC_FP64 0
#define GRPIC_FP32_SPLIT 1

#define GRPIC_MAX_SPECIES 8

/* Kerr metric parameters: spin a and mass M, |a| <= M; M = a = 0 is flat
 * space (App. A, with the mass written back into z = 2Mr/rho^2 and
 * Delta = r^2 + a^2 - 2Mr). */
typedef struct {
    double a, M;
} grpic_metric;

/* Grid, see the conventions above. */
typedef struct {
    int32_t nr, nth, guard, pitch;
    double lnr0, dlnr, dth;
} grpic_grid;

/* One species: charge q, mass m.  massless != 0 marks photons, which follow
 * geodesics with u^0 = |u|/alpha and skip the Boris step (Sec. 2.2). */
typedef struct {
    double q, m;
    int32_t massless, reserved;
} grpic_species;

typedef struct {
    int64_t n;
    int32_t* cell;
    void *xr, *xth, *ur, *uth, *uph, *w;
    uint8_t* sp;
    void* phi;
    int32_t precision;   /* GRPIC_FP64 or GRPIC_FP32_SPLIT */
    int32_t reserved;
    uint64_t* tag;       /* optional particle tags (NULL: none), moved by grpic_sort */
} grpic_particles;

/* Contravariant D^i and B^i, i = r, th, ph, on the Yee stagger; double for
 * GRPIC_FP64, float for GRPIC_FP32_SPLIT. */
typedef struct {
    const void* D[3];
    const void* B[3];
} grpic_fields;

/* F^r, F^th, G^ph (double, accumulated). */
typedef struct {
    double *Fr, *Fth, *Gph;
} grpic_current;

/* Device counters, accumulated (+=) by grpic_push_deposit when non-NULL. */
#define GRPIC_CNT_OUT 0        /* particles removed at the radial edges          */
#define GRPIC_CNT_BAD 1        /* removed as non-finite or moving >= 1 cell      */
#define GRPIC_CNT_REFLECT 2    /* reflections at the axis                         */
#define GRPIC_CNT_LIVE 3       /* particle-steps taken by live particles          */
#define GRPIC_CNT_SPILL 4      /* tiled path: deposits outside the LDS window     */
#define GRPIC_NCOUNTERS 5

/*
 * grpic_push_deposit -- advance every live particle `nsteps` steps through
 * fixed fields and accumulate the current it carries.
 *
 * Per particle and step (Sec. 2.2, 2.3): CIC-interpolate D^i, B^i at x^n;
 * one full-step generalised Boris kick at x^n (eqs. boris-plus-minus, u0bar,
 * boris-scheme; the two half kicks of the Strang split bundled, as the paper
 * does); geodesic predictor (eq. geodesic-predictor) followed by `ncorr`
 * trapezoid corrector passes (eq. geodesic-corrector; the paper's default
 * is 3) on the right-hand sides of eq. particle-eom, with positions in grid
 * units; reflection at the axis (eta -> -eta or 2 nth - eta, u_th -> -u_th);
 * Esirkepov deposit of the move x^n -> x^{n+1} on the 3x3 vertex window
 * (eqs. esirkepov-decomp, j-phi-deposit, local prefix sum); a particle that
 * leaves [0, nr) in xi deposits its move into the guard vertices and is
 * removed (cell = -1).  A particle whose end point is not finite or that
 * moved one cell or more is removed without depositing (counted as BAD), and
 * so is one whose cell, offsets or species index are out of range.
 *
 * species: host array of nsp entries (1 <= nsp <= GRPIC_MAX_SPECIES).
 * parts: updated in place.  fields: read only.  J: accumulated.
 * tiling: NULL, or the tiling written by the grpic_sort call that produced
 *   the current particle order (same n and grid; checked, GRPIC_EINVAL
 *   otherwise).  With a tiling each workgroup accumulates the current of
 *   one slice of cell-sorted particles in LDS and flushes it once; particles
 *   that have drifted out of their tile's LDS window since the sort deposit
 *   straight to global memory, so results do not depend on how fresh the
 *   sort is.  Only particles live at the sort are pushed (the sort marks the
 *   rest removed); without a tiling any particle order works.  A tiled
 *   push also writes into the tiling: each launch first fills its table of
 *   r, sin(theta) and cos(theta) at the cell corners its tiles start from,
 *   and with counters each slice's live count (pushes that share a tiling
 *   must be stream-ordered, as they share the particles anyway).
 * dt > 0 must not exceed grpic_crossing_time(); ncorr in [0, 16].
 * ckpt (optional, device, ckpt_bytes >= grpic_checkpoint_bytes(n, nsteps,
 *   ckpt_every)): the particle state is saved before every step k with
 *   k % ckpt_every == 0, for grpic_push_deposit_backward (in double; a
 *   GRPIC_FP32_SPLIT state is promoted exactly; ckpt_every must divide
 *   nsteps).  NULL, 0, 0 when not needed.
 * counters: optional device int64[GRPIC_NCOUNTERS], accumulated.
 */
int grpic_push_deposit(const grpic_metric* metric, const grpic_grid* grid,
                       const grpic_species* species, int nsp,
                       grpic_particles* parts, const grpic_fields* fields, grpic_current* J,
                       void* tiling, double dt, int nsteps, int ncorr,
                       void* ckpt, size_t ckpt_bytes, int ckpt_every,
                       int64_t* counters, void* stream);

/*
 * grpic_push_deposit_vay -- grpic_push_deposit with Vay's momentum update
 * (Vay 2008) in the FIDO frame in place of the generalised Boris kick: the
 * alternative pusher of Sec. 2.2.  With h = (q/m) alpha dt / 2, v = u/gamma,
 * dot products as gamma_ij contractions and cross products with
 * e_ijk = sqrt(gamma) eps_ijk:  u' = u + h (D + v x B) + h D,  tau = h B,
 * gamma_new^2 = (sigma + sqrt(sigma^2 + 4 (tau^2 + (u'.tau)^2)))/2 with
 * sigma = 1 + u'^2 - tau^2,  t = tau/gamma_new,
 * u_new = (u' + (u'.t) t + u' x t)/(1 + t^2).  It keeps u exactly when
 * D = -v x B (the force-free drift), which the Boris kick does not.
 * Everything else (gather, geodesic predictor-corrector, boundaries,
 * deposit, tiling, counters, arguments and errors) is as in
 * grpic_push_deposit.  GRPIC_FP64 particles only (GRPIC_EINVAL otherwise);
 * no checkpoints (the adjoint differentiates the Boris kick).
 */
int grpic_push_deposit_vay(const grpic_metric* metric, const grpic_grid* grid,
                           const grpic_species* species, int nsp,
                           grpic_particles* parts, const grpic_fields* fields, grpic_current* J,
                           void* tiling, double dt, int nsteps, int ncorr,
                           int64_t* counters, void* stream);

/*
 * grpic_push_deposit_spline3 -- grpic_push_deposit with the third-order
 * shape (the spline option of Sec. 2.3) in place of CIC for both the field
 * gather and the Esirkepov deposit: the cubic B-spline W(d) = 2/3 - d^2 +
 * |d|^3/2 (|d| < 1), (2 - |d|)^3/6 (1 <= |d| < 2), 0 beyond, on the 4 x 4
 * vertices of each component's own stagger for the gather (guard rows and
 * the columns beyond the axes, which grpic_field_step keeps, are read) and
 * the 5 x 5 vertex window (lower corner floor(min xi) - 1, floor(min eta) -
 * 1) for the deposit.  Deposits beyond an axis are folded onto the mirror
 * vertex (F^r, G^ph, values kept) or theta face (F^th, sign changed), by
 * axisymmetry, so discrete charge continuity holds at every vertex with the
 * cubic charge of grpic_charge3.  Generalised Boris kick, FP64 particles,
 * no checkpoints; grid->guard >= 3 (the window's radial reach), nth >= 4.
 * tiling: NULL (one thread per particle, global atomics) or a grpic_sort
 * tiling as in grpic_push_deposit (the LDS window holds the folded 5 x 5
 * windows; moves outside it deposit to global memory).  Otherwise
 * arguments, errors and counters as in grpic_push_deposit.
 */
int grpic_push_deposit_spline3(const grpic_metric* metric, const grpic_grid* grid,
                               const grpic_species* species, int nsp,
                               grpic_particles* parts, const grpic_fields* fields, grpic_current* J,
                               void* tiling, double dt, int nsteps, int ncorr, int64_t* counters, void* stream);

/*
 * grpic_charge3 -- grpic_charge with the cubic spline shape, folded across
 * the axes like grpic_push_deposit_spline3's deposit (guard >= 3).
 */
int grpic_charge3(const grpic_grid* grid, const grpic_species* species, int nsp,
                  const grpic_particles* parts, double* Q, void* stream);

/*
 * grpic_push_deposit_qed -- one step of the monopole workload's particles
 * (Sec. 4): the push and deposit of grpic_push_deposit (FP64, Boris kick,
 * CIC; photons, the massless species, follow geodesics and carry no
 * current), then, from each particle's end point:
 *   - an e- or e+ whose FIDO Lorentz factor Gamma = sqrt(1 + gamma^ij u_i u_j)
 *     exceeds gamma_thr emits one photon of FIDO energy eps_ph along its own
 *     momentum, at its end point, with its weight; its FIDO momentum
 *     magnitude drops by eps_ph (momentum kept along the common direction);
 *   - a photon of FIDO energy eps = sqrt(gamma^ij u_i u_j) >= 2 (twice the
 *     rest energy) converts with probability P = 1 - exp(-tau dt) (eq.
 *     optical-depth) into an e- and an e+ of FIDO energy eps/2 each along its
 *     direction, at its end point, with its weight, and is removed.
 * Particles that left the grid in the step, or were removed as bad, neither
 * emit nor convert; particles created in the step are not pushed in it.
 * Random numbers: Philox4x64-10 (Salmon et al., SC'11) with counter (tag,
 * step, 0, 0) and key (seed, 0), one block per particle and step: word 0
 * gives a photon's uniform U = (x0 >> 11) 2^-53 (it converts iff U < P),
 * word 1 the tag of the emitted photon or of the e-, word 2 that of the e+.
 *
 * parts: GRPIC_FP64 with tags; parts->n is the capacity of its arrays.
 * n_used: device int64[2].  On entry n_used[0] is the number of array
 *   elements in use (every element at or beyond it must have cell = -1);
 *   the particles of [0, n_used[0]) are pushed and the created ones are
 *   written to [n_used[0], n_used[0] + created) in no particular order, so
 *   that on return n_used[0] counts them too (created particles beyond the
 *   capacity are dropped and counted).  n_used[1] is working space (its
 *   value on entry does not matter; 0 on return).  grpic_sort with
 *   n_alive_dev = n_used leaves n_used[0] right for the next step.
 * tiling: NULL, or the tiling of the grpic_sort call that produced the
 *   current order; the particles appended since that sort are pushed
 *   without the LDS window.
 * ws: NULL, or (with a tiling) a device workspace of at least
 *   grpic_qed_workspace_bytes(grid, parts->n) bytes (contents on entry do
 *   not matter).  With it each workgroup stages the particles its slice
 *   creates, and a scan places them after the others in slice order, so the
 *   step takes no same-address atomics for them (a slice's particles beyond
 *   16 are appended one atomic each); without it every wave that creates
 *   particles reserves their slots with one atomic on n_used[1].
 * step: the step number that keys the random numbers.
 * qcounters: optional device int64[GRPIC_NQCOUNTERS], accumulated.
 * Otherwise arguments and errors as in grpic_push_deposit, with nsteps = 1.
 * GRPIC_EINVAL for non-FP64 particles, no tags, species indices outside
 * the species table, a photon species that is not massless, an e- or e+
 * species that is, gamma_thr <= 1, eps_ph <= 0 or
 * eps_ph >= sqrt(gamma_thr^2 - 1) (the emitter's momentum must stay
 * positive), tau < 0 or a NULL n_used.
 */
typedef struct {
    double gamma_thr;                 /* emission threshold on Gamma               */
    double eps_ph;                    /* FIDO energy of an emitted photon          */
    double tau;                       /* conversion rate: P = 1 - exp(-tau dt)     */
    uint64_t seed;                    /* key of the random stream                  */
    int32_t electron_sp, positron_sp, photon_sp, reserved;
} grpic_qed;

#define GRPIC_QCNT_EMITTED 0          /* photons emitted                            */
#define GRPIC_QCNT_CONVERTED 1        /* photons converted into pairs               */
#define GRPIC_QCNT_DROPPED 2          /* created particles beyond the capacity      */
#define GRPIC_NQCOUNTERS 3

size_t grpic_qed_workspace_bytes(const grpic_grid* grid, int64_t n);
int grpic_push_deposit_qed(const grpic_metric* metric, const grpic_grid* grid,
                           const grpic_species* species, int nsp,
                           grpic_particles* parts, const grpic_fields* fields, grpic_current* J,
                           void* tiling, double dt, int64_t step, int ncorr, const grpic_qed* qed,
                           int64_t* n_used, void* ws, size_t ws_bytes, int64_t* counters, int64_t* qcounters,
                           void* stream);

/* Gradient outputs of grpic_push_deposit_backward (device, double). */
typedef struct {
    double *ur, *uth, *uph;          /* per particle, overwritten */
} grpic_momentum_grads;
typedef struct {
    double *D[3], *B[3];             /* grid arrays on the Yee stagger, accumulated (+=) */
} grpic_field_grads;

/*
 * grpic_push_deposit_backward -- adjoint of `nsteps` FP64 push + deposit
 * steps (not in the paper; built on its step, Sec. 2.2-2.3).
 *
 * With L = sum over the steps n and the particles of
 *   lambda_r . F^r_n + lambda_th . F^th_n + lambda_ph . G^ph_n,
 * lambda = (Fr, Fth, Gph) of `lambda` given per grid element (the cotangent
 * of the current accumulated over the steps), writes dL/du_i of every
 * particle's initial momenta to grad_u and adds dL/dD^i, dL/dB^i to
 * grad_fields.  parts: the particles at the start of the forward call (w and
 * sp are read; n, precision GRPIC_FP64); fields, dt, nsteps, ncorr (<= 8),
 * species: as in that call; ckpt: its checkpoints.  ws: device workspace of
 * grpic_backward_workspace_bytes(grid, n, ckpt_every) bytes (its contents on
 * entry do not matter).  Per particle, each
 * checkpoint segment is recomputed from its checkpoint and then reversed
 * step by step, the last step first; field gradients use FP64 atomics.
 * While a particle's cotangent is zero, steps and whole segments whose
 * deposits cannot reach a non-zero lambda entry are skipped (their
 * contribution is exactly zero), so a loss supported on a few grid rows
 * costs little for particles far from them.  ws also holds the lambda
 * support tables, hence the grid argument of grpic_backward_workspace_bytes.
 * The derivative is that of the piecewise-smooth map: where a particle's
 * CIC weights or deposit window change (cell edges), the one-sided
 * derivative of the side the trajectory lies on is taken.
 */
size_t grpic_checkpoint_bytes(int64_t n, int nsteps, int ckpt_every);
size_t grpic_backward_workspace_bytes(const grpic_grid* grid, int64_t n, int ckpt_every);
int grpic_push_deposit_backward(const grpic_metric* metric, const grpic_grid* grid,
                                const grpic_species* species, int nsp, const grpic_particles* parts,
                                const grpic_fields* fields, const grpic_current* lambda,
                                double dt, int nsteps, int ncorr, const void* ckpt, size_t ckpt_bytes,
                                int ckpt_every, void* ws, size_t ws_bytes,
                                const grpic_momentum_grads* grad_u, const grpic_field_grads* grad_fields,
                                void* stream);

/*
 * grpic_push_deposit_backward_range -- grpic_push_deposit_backward for a
 * range of the checkpointed particles and for fields that change from step
 * to step (the push + deposit steps of a PIC loop whose field solver runs
 * between them; the derivative does not pass through the field states,
 * which are inputs here).
 *
 * range->first, range->count: the particles [first, first + count) of the
 *   parts->n checkpointed ones are reversed; grad_u receives count entries
 *   (entry k for particle first + k) and ws needs only
 *   grpic_backward_workspace_bytes(grid, count, ckpt_every) bytes, so a
 *   large set can be reversed in batches with one bounded workspace (field
 *   gradients of successive batches add up).
 * range->field_step_stride: 0 (every step gathers from `fields`) or the
 *   distance in elements between the arrays of successive steps: step k of
 *   the call gathers component c from fields->D[c] + k * stride (likewise
 *   B), i.e. the fields the forward's step k saw.
 * range->grad_step_stride: 0 (field gradients summed over the steps into
 *   grad_fields) or the same distance for per-step gradient arrays.
 * grad_fields: may be NULL (no field gradients).
 * The checkpoints may come from a GRPIC_FP32_SPLIT forward (grpic_push_deposit
 * saves the float states promoted exactly to double); the reverse then
 * replays each segment in FP64 from its checkpoint, and parts must be a
 * GRPIC_FP64 view of w and sp (the other arrays are not read).
 * Otherwise arguments and errors as in grpic_push_deposit_backward; strides
 * below one grid array are rejected (GRPIC_EINVAL).
 */
typedef struct {
    int64_t first, count;
    size_t field_step_stride;
    size_t grad_step_stride;
} grpic_backward_range;
int grpic_push_deposit_backward_range(const grpic_metric* metric, const grpic_grid* grid,
                                      const grpic_species* species, int nsp, const grpic_particles* parts,
                                      const grpic_fields* fields, const grpic_current* lambda,
                                      double dt, int nsteps, int ncorr, const void* ckpt, size_t ckpt_bytes,
                                      int ckpt_every, const grpic_backward_range* range, void* ws,
                                      size_t ws_bytes, const grpic_momentum_grads* grad_u,
                                      const grpic_field_grads* grad_fields, void* stream);

/*
 * grpic_charge -- Q_ij += sum over live particles of q w S_ij(x_p), the CIC
 * charge at the vertices (rho dV; the left-hand side of eq. J-integral-eqn).
 * Used to check discrete charge continuity.  Q is a double grid array.
 */
int grpic_charge(const grpic_grid* grid, const grpic_species* species, int nsp,
                 const grpic_particles* parts, double* Q, void* stream);

/*
 * grpic_sort -- counting sort of the particles by cell (stable within a
 * cell is not promised), removed particles (cell < 0) dropped.
 *
 * in, out: particle sets of the same precision; out must hold in->n
 * particles and must not alias in; out->n is not read.  On completion the
 * first *n_alive_dev elements of out hold the live particles ordered by
 * cell; the remaining in->n - *n_alive_dev elements have cell = -1 (removed)
 * and their other fields unspecified, so out can be pushed with n = in->n.
 * cell_offsets (optional, device int64[nr*nth + 1]) receives the exclusive
 * prefix sum of the per-cell counts.  tiling (optional, device, at least
 * grpic_tiling_bytes(grid, in->n) bytes) receives the slice table that
 * grpic_push_deposit's tiled path runs on: each 64-cell tile of a grid row
 * cut into balanced slices, once of at most 256 particles (for the CIC
 * kernels) and once of at most 192 (for the cubic shape); the push must be
 * given n equal to in->n and the same grid (checked).
 * ws: device workspace of at least
 * grpic_sort_workspace_bytes() bytes.  n_alive_dev: device int64 receiving
 * the live count.  Tags move with their particles when in and out both
 * carry them (GRPIC_EINVAL if only one does).
 * Not described by the paper: particles are kept ordered by cell so that a
 * workgroup's particles share field cache lines and one LDS current window.
 */
size_t grpic_sort_workspace_bytes(const grpic_grid* grid, int64_t n);
size_t grpic_tiling_bytes(const grpic_grid* grid, int64_t n);
int grpic_sort(const grpic_grid* grid, const grpic_particles* in, grpic_particles* out,
               int64_t* cell_offsets, void* tiling, size_t tiling_bytes, void* ws, size_t ws_bytes,
               int64_t* n_alive_dev, void* stream);

/*
 * grpic_sort_noalloc -- grpic_sort for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same sort, outputs and errors, with the workspace
 * taken from a static device array of GRPIC_SORT_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends.  The call
 * allocates nothing; its scratch is cleared by kernels, not memsets.
 * GRPIC_ENOMEM if grpic_sort_workspace_bytes(grid, in->n) exceeds
 * GRPIC_SORT_SCRATCH_BYTES (2048 x 2048 grids and smaller fit).  All calls
 * on one GPU share that GPU's array: calls that overlap in time on one GPU
 * (on different streams, or from different threads without ordering) race.
 * The device is the calling thread's current device.
 */
#define GRPIC_SORT_SCRATCH_BYTES ((size_t)40 << 20)
int grpic_sort_noalloc(const grpic_grid* grid, const grpic_particles* in, grpic_particles* out,
                       int64_t* cell_offsets, void* tiling, size_t tiling_bytes, int64_t* n_alive_dev,
                       void* stream);

/*
 * Field solver (Sec. 2.1, eqs. integral-form, fld-predictor, fld-corrector,
 * Dr-axis; App. B, eqs. D-update, auxH, B-update, auxE).  GRPIC_FP64 grid
 * arrays of the layout above: the dynamic fields D^i, B^i at their Yee
 * locations, advanced in place by one step of dt.
 *
 * grpic_field_tables: writes, on the device, the inverse area elements of
 * the six components (per unit phi; 10-point Gauss quadrature of sqrt(gamma)
 * over each face), radial edge lengths, and r, sin theta, cos theta at
 * half-cell steps (from which the step forms the metric coefficients
 * alpha gamma_ij, sqrt(gamma) beta^r) into `tables` (device, at least
 * grpic_field_tables_bytes(grid) bytes, caller-owned).  The library records
 * the metric and grid the tables describe; grpic_field_step checks them.
 *
 * grpic_field_step: one step of the generalized Maxwell equations.
 *   state: the six dynamic field arrays (device, updated in place).
 *   J: the step's currents in flux form, as grpic_push_deposit accumulates
 *     them (F^r = J^r A^D_r, F^th = J^th A^D_th, G^ph = J^ph A^D_ph, areas per
 *     unit phi); NULL for vacuum.
 *   The auxiliary fields E_i, H_i are formed metric coefficients first and
 *   then averaged to their location (eqs. auxE with the 1/2 on the last
 *   term of E_ph, auxH).  A predictor X~ = X^n + dt (C(X^n) - J) is followed
 *   by ncorr (0 .. 64) passes X~ = X^n + dt ((1 - w1) C(X^n) + w1 C(X~))
 *   - dt J, w1 in [0, 1] (the paper's beta; 0.53 and 7 passes in its
 *   production runs; w1 = 1/2 is Heun's method).  D^r on the axes takes
 *   the half-cell area and only the H_ph of its own side (eq. Dr-axis, with
 *   dt on J as well); D^ph = B^th = 0 on the axes; guard rows copy the
 *   nearest physical row (zero gradient) at both radial edges.  After the
 *   step, every component at radial grid position x >= nr - damp_cells is
 *   multiplied by 1 - damp_max ((x - nr + damp_cells)/damp_cells)^2 (an
 *   outer damping layer; damp_cells = 0: none; damp_max in [0, 1]).  Last,
 *   the guard columns beyond each axis (read by the particle gather near
 *   the axis) are set from the mirrored columns by axisymmetry: (r, -theta,
 *   phi) is (r, theta, phi + pi), so the r and phi components are even and
 *   D^th, B^th odd across the axis (integer columns -m <-> m, nth + m <->
 *   nth - m; columns at j + 1/2: -m <-> m - 1, nth - 1 + m <-> nth - m).
 *   Requires nth >= 2 * guard.
 *   ws: device workspace of at least grpic_field_workspace_bytes(grid)
 *   bytes; its contents on entry do not matter.
 *   Errors: GRPIC_EINVAL for NULL arrays, dt <= 0, parameters out of range
 *   or tables not written for this metric and grid; GRPIC_ENOMEM for a small
 *   workspace.
 */
typedef struct {
    double *D[3], *B[3];                    /* D^r, D^th, D^ph; B^r, B^th, B^ph */
} grpic_field_state;

size_t grpic_field_tables_bytes(const grpic_grid* grid);
size_t grpic_field_workspace_bytes(const grpic_grid* grid);
int grpic_field_tables(const grpic_metric* metric, const grpic_grid* grid, void* tables, size_t tables_bytes,
                       void* stream);
int grpic_field_step(const grpic_metric* metric, const grpic_grid* grid, const void* tables,
                     const grpic_field_state* state, const grpic_current* J, double dt, double w1, int ncorr,
                     int damp_cells, double damp_max, void* ws, size_t ws_bytes, void* stream);

/*
 * grpic_crossing_time -- minimum over cell centres of the time light needs to
 * cross one cell, from |dxi/dt| <= (alpha sqrt(gamma^rr) + |beta^r|)/(r dlnr)
 * and |deta/dt| <= alpha sqrt(gamma^thth)/dth.  Host computation.  Returns a
 * negative value for an invalid metric or grid.
 */
double grpic_crossing_time(const grpic_metric* metric, const grpic_grid* grid);

/* Thread-local message for the last failing call ("" if none). */
const char* grpic_last_error(void);

/* Library version string. */
const char* grpic_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRPIC_H_ */
