/*
 * gpf.h -- C ABI of the MI355X (gfx950) library for the coupled
 * Grand-Potential phase-field / lattice-Boltzmann time step.
 *
 * What one step computes (paper sections / equations):
 *   1. phase fields phi_a by the grand-potential Allen-Cahn equation,
 *      Eq. (PhfGrand), with the anisotropic gradient energy, the double
 *      obstacle W of Eq. (Wpot) and the Gibbs-simplex constraint of Sec. 2.1;
 *   2. chemical potentials mu_i by Eq. (conc): h-interpolated
 *      susceptibility, the dh/dt source, and advection by the fluid velocity
 *      (the paper's modification; U = 0 in solids);
 *   3. one BGK collide + stream, Eq. (LBMEq_1) with f^eq of Eq. (f^eq) and
 *      the discrete force of Eq. (discreteForce), carrying the solutal
 *      buoyancy of Eq. (buoyancy), the drag force G_D that enforces
 *      no-slip at the diffuse solid-liquid interface and, when enabled, the
 *      shrinkage force of Eq. (shrinkage);
 *   4. staggered in the order of Algorithm phfLBM (App. A).
 * D2Q9 (Table LBM_Schemes) in 2D; D3Q19 or D3Q27 (Table LBM_Schemes) in 3D.
 * The lattice changes only the populations: the phase-field and
 * chemical-potential stencils use the 9/19-point neighbourhood throughout.
 *
 * Conventions for every call:
 *   - Return value: a gpf_status; GPF_OK = 0, negative on error.  No C++
 *     exception and no abort crosses this boundary.  gpf_last_error()
 *     returns a message for the last failing call on a context.
 *   - Field layout (host and device): [component][z][y][x], x fastest,
 *     cells = n[0] * n[1] * n[2] (n[2] = 1 in 2D).
 *   - Lattice numbering: D2Q9 as in the paper's lattice figure (0 rest,
 *     1 +x, 2 +y, 3 -x, 4 -y, 5 (+,+), 6 (-,+), 7 (-,-), 8 (+,-)); D3Q19:
 *     0 rest, 1..6 = +x,-x,+y,-y,+z,-z, then (+,+,0),(-,-,0),(+,-,0),(-,+,0),
 *     (+,0,+),(-,0,-),(+,0,-),(-,0,+),(0,+,+),(0,-,-),(0,+,-),(0,-,+);
 *     D3Q27: the D3Q19 order, then (+,+,+),(-,-,-),(+,+,-),(-,-,+),(+,-,+),
 *     (-,+,-),(-,+,+),(+,-,-).
 *   - Phases: solids first, liquid last.  n_components = K counts all
 *     species, so there are nc = K - 1 independent chemical potentials.
 *   - A context owns its device buffers; every host pointer passed in
 *     belongs to the caller and is not retained.  A context is used by one
 *     host thread at a time.
 */
#ifndef GPF_H
#define GPF_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gpf_ctx gpf_ctx;

typedef enum {
  GPF_OK = 0,
  GPF_ERR_ARG = -1,         /* NULL pointer, wrong count, unknown enum value */
  GPF_ERR_PARAM = -2,       /* physically or numerically invalid parameter */
  GPF_ERR_NOMEM = -3,       /* device allocation failed */
  GPF_ERR_DEVICE = -4,      /* a HIP call failed (message names it) */
  GPF_ERR_NONFINITE = -5,   /* health check found NaN/Inf or rho <= 0 */
  GPF_ERR_STATE = -6,       /* call not valid in the current state */
  GPF_ERR_UNSUPPORTED = -7  /* valid but not built: (dim, lattice, N, nc) outside the instances */
} gpf_status;

/* D2Q9 in 2D; D3Q19, or the paper's D3Q27 (Table LBM_Schemes), in 3D */
typedef enum { GPF_D2Q9 = 0, GPF_D3Q19 = 1, GPF_D3Q27 = 2 } gpf_lattice;
typedef enum { GPF_FP64 = 0, GPF_FP32 = 1 } gpf_precision;
typedef enum { GPF_OBSTACLE = 0, GPF_WELL = 1 } gpf_potential;
typedef enum { GPF_INIT_SEED = 0, GPF_INIT_LAMELLAE = 1, GPF_INIT_LIQUID = 2 } gpf_init_kind;

/* Fields readable with gpf_read / gpf_read_device (components per cell):
 *   GPF_PHI   N      order parameters phi^n
 *   GPF_MU    nc     chemical potentials mu^n
 *   GPF_F     Q      populations f^n after streaming (the full f, also in FP32 mode)
 *   GPF_RHO   1      sum_k f_k
 *   GPF_U     dim    lattice velocity of the last collision (advects mu in the next step)
 *   GPF_C     nc     mixture composition sum_a h_a(phi) C^a(mu)
 *   GPF_T     1      temperature T(x, n)
 *   GPF_FLAGS 1      active-phase bitmask (bit a: phase a present in the lattice neighbourhood)
 *   GPF_FPOST Q      the stored populations: post-collision f*_k - w_k rho0 of the last step,
 *                    before streaming, exactly as held on the device (checkpoint form)
 * Writable with gpf_write: GPF_PHI, GPF_MU, GPF_F, GPF_U, GPF_FPOST.  Reading
 * GPF_PHI, GPF_MU, GPF_U and GPF_FPOST and writing them back is exact in both
 * precisions, so with gpf_set_step_index a run resumes bitwise. */
typedef enum {
  GPF_PHI = 0, GPF_MU = 1, GPF_F = 2, GPF_RHO = 3, GPF_U = 4, GPF_C = 5, GPF_T = 6, GPF_FLAGS = 7,
  GPF_FPOST = 8
} gpf_field;

/* FP64 totals of gpf_reduce:
 *   GPF_SUM_SOLUTE  nc values  sum over cells of the mixture composition sum_a h_a C^a_i(mu), the
 *                              quantity Eq. (conc) conserves (flux form, zero-flux walls)
 *   GPF_SUM_MASS    1 value    sum over cells of rho = sum_k f_k, Eq. (rhovel)
 *   GPF_LOSS        1 value    L = 1/2 sum over cells and phases of (phi_a - phi^target_a)^2 against
 *                              the target of gpf_set_target (the paper has no loss: the scalar whose
 *                              parameter gradients gpf_adjoint computes) */
typedef enum { GPF_SUM_SOLUTE = 0, GPF_SUM_MASS = 1, GPF_LOSS = 2 } gpf_reduction;

typedef struct {
  int32_t dim;            /* 2 or 3 */
  int64_t n[3];           /* cells per axis; n[2] ignored in 2D */
  double dx;              /* phase-field grid spacing (the LBM runs in lattice units) */
  uint32_t periodic_mask; /* bit a set: axis a periodic, else zero-flux / no-slip walls */
} gpf_grid;

typedef struct {
  int32_t lattice;        /* gpf_lattice; must match dim */
  int32_t precision;      /* gpf_precision: FP64, or FP32 storage and arithmetic */
  int32_t potential;      /* gpf_potential: OBSTACLE (the paper) or WELL (test only) */
  double dt, eps, tau_pf; /* time step, interface parameter eps, relaxation tau of Eq. (PhfGrand) */
  double gamma[4][4];     /* interface energies gamma_ab, symmetric */
  double delta[4][4];     /* cubic anisotropy strength per pair, symmetric */
  double chi[2][2];       /* susceptibility, SPD, common to all phases: C^a = c0[a] + mT[a] (T - T_E) + chi mu */
  double c0[4][2];
  double dS[4];           /* grand potential psi^a gets + dS[a] (T - T_E) */
  double mT[4][2];        /* d c0_a / dT: the parabola centre of phase a is c0[a] + mT[a] (T - T_E),
                             the equilibrium composition moving along the App. B coexistence line
                             (slopes read as dc/dT); it makes the dT/dt term of Eq. (conc) act under
                             the pulled gradient.  All 0: compositions independent of T. */
  double T_E, T_iso;      /* eutectic / equilibrium temperature; temperature when G = 0 */
  double D[4][2];         /* diffusivity per phase and solute (solids 0 in the paper) */
  double G, V, y0;        /* frozen gradient T = T_E + G (x_pull - y0 - V n), V in cells/step */
  int32_t pull_axis;
  double tau_lb, rho0;    /* BGK relaxation time (> 1/2) and reference density */
  double gbeta[2];        /* signed products g * beta_i of Eq. (buoyancy) */
  double c_ref[2];        /* reference liquid composition of Eq. (buoyancy) */
  int32_t grav_axis, grav_sign; /* unit gravity vector = grav_sign * e_{grav_axis} */
  double h_drag, W0;      /* drag kappa = 2 nu h / W0 of G_D, nu = (tau_lb - 1/2)/3 */
  double eta[4];          /* shrinkage force G_S of Eq. (shrinkage): eta_a = (rho_a - rho_liq) / rho_liq
                             per phase (liquid 0); G_S = sum_a eta_a (phi^{n+1}_a - phi^n_a) n_a per
                             lattice step, n_a the unit normal of phi^{n+1}_a from central differences.
                             All 0: off.  gpf_adjoint refuses a context with G_S on. */
  double lid_u;           /* test only: upper wall of axis 1 moves along axis 0 (cavity) */
  int32_t init_kind;      /* gpf_init_kind */
  double init_center[3], init_radius; /* seed centre (cell units, cell i at coordinate i), radius */
  double lam_width, lam_height;       /* lamella width along x, solid height along pull_axis */
  double mu_inf[2], noise_sigma;      /* mu^0_i = mu_inf_i + sigma z(seed, cell, i) */
  int64_t frame_every;    /* moving frame of Case 2 (Sec. 3): every so many steps (0: off) the
                             front -- the largest pull-axis index of a cell with phi_liq <= 1/2 --
                             is found; if it lies beyond frame_front, every field moves down the
                             pull axis by the excess, the new far planes repeat the last one and
                             the frame origin (gpf_frame_offset) grows by it.  Needs walls on the
                             pull axis; each check synchronises. */
  int64_t frame_front;    /* pull-axis index the front is kept at, 0 <= frame_front < n[pull_axis] */
  int64_t health_every;   /* > 0: check NaN/Inf and rho <= 0 every so many steps and at the
                             end of each gpf_step call (the call then synchronises); 0: never */
  void* (*dev_alloc)(size_t bytes, void* user); /* NULL: hipMalloc; else e.g. torch's caching allocator */
  void (*dev_free)(void* ptr, void* user);
  void* alloc_user;
} gpf_params;

/* Create a simulation and its initial state (paper's problem statement:
 * grid, phases, components, material parameters; App. A Algorithm phfLBM
 * "Initialization").  Initial state: phi^0 from the 1D equilibrium profile
 * of the double obstacle, 1/2 - 1/2 sin(4 s / (pi eps)) for |s| <= pi^2 eps/8,
 * around a seed (circle/sphere) or a flat front of alternating lamellae;
 * mu^0 = mu_inf + noise_sigma * z with z standard normal from a
 * counter-based SplitMix64 + Box-Muller stream keyed by `seed`
 * (z index = cell * nc + i); f^0 = w_k rho0; U = 0.
 * n_phases: 2, 3 or 4 (four: three solids and the liquid, the paper's Case 3
 * system, built for n_components = 3 only).  n_components: 2 or 3
 * (nc = n_components - 1).
 * Errors: GPF_ERR_ARG (NULL), GPF_ERR_PARAM (tau_lb <= 1/2, dt, dx, eps,
 * tau_pf <= 0, explicit stability bound exceeded, chi not SPD, axes out of
 * range, lattice/dim mismatch), GPF_ERR_UNSUPPORTED (N, nc, dim outside the
 * built instances), GPF_ERR_NOMEM, GPF_ERR_DEVICE.  On error *out = NULL. */
int gpf_init(gpf_ctx** out, const gpf_grid* grid, int32_t n_phases, int32_t n_components,
             const gpf_params* params, uint64_t seed);

/* Launch subsequent work on this HIP stream (a hipStream_t, e.g. torch's
 * current stream); NULL selects the null stream.  The stream is not owned.
 * Not an operation of the paper: it places the passes of Algorithm phfLBM
 * (App. A) on the caller's stream.  Errors: GPF_ERR_ARG (NULL ctx). */
int gpf_set_stream(gpf_ctx* ctx, void* hip_stream);

/* Advance n >= 0 coupled steps (Algorithm phfLBM, one pass per step).
 * Asynchronous unless health_every > 0, in which case the call waits for
 * its last health check and returns GPF_ERR_NONFINITE (with the first
 * failing step in the message) when it failed. */
int gpf_step(gpf_ctx* ctx, int64_t n);

/* Like gpf_step (Algorithm phfLBM, App. A), and records HIP events around
 * each part of the step on the context's stream; kernel_ms[j] receives the
 * summed milliseconds of part j (j = 0: phase field, one kernel, or on 3D
 * grids with the bulk history the tile check and the walk of the listed
 * tiles together; 1: chemical potential + LBM), count up to n_kernels.
 * Synchronises.  For measurement only. */
int gpf_step_timed(gpf_ctx* ctx, int64_t n, double* kernel_ms, int32_t n_kernels);

/* Copy a field to caller-owned host memory as FP64 (adds w_k rho0 back to f
 * in every precision): the output step of Algorithm phfLBM (App. A), which
 * writes rho, phi, U and C, plus mu, f, T and the active-set flags.  count
 * must equal components * cells.  Synchronises.  Errors: GPF_ERR_ARG (NULL,
 * unknown field, wrong count), GPF_ERR_DEVICE. */
int gpf_read(gpf_ctx* ctx, int32_t field, double* host_dst, size_t count);

/* Copy a field to caller-owned device memory in the context's precision
 * (double or float; f as the full f): the output step of Algorithm phfLBM
 * without leaving the device.  GPF_PHI, GPF_MU, GPF_U, GPF_F only.  bytes
 * must equal components * cells * element size.  Asynchronous on the
 * context's stream.  Errors: GPF_ERR_ARG, GPF_ERR_DEVICE. */
int gpf_read_device(gpf_ctx* ctx, int32_t field, void* dev_dst, size_t bytes);

/* Overwrite a state field from FP64 host memory (GPF_PHI, GPF_MU, GPF_F as
 * the post-streaming f^n, GPF_U as the velocity of the previous step,
 * GPF_FPOST as the stored post-collision populations): the state that the
 * initialisation step of Algorithm phfLBM (App. A) sets, given by the caller
 * (tests inject states; resuming writes a checkpoint back).  Synchronises.
 * Errors: GPF_ERR_ARG (NULL, field not writable, wrong count), GPF_ERR_DEVICE. */
int gpf_write(gpf_ctx* ctx, int32_t field, const double* host_src, size_t count);

/* FP64 totals in a fixed summation order (deterministic), see gpf_reduction:
 * the solute that Eq. (conc) conserves, the mass of Eq. (rhovel), or the
 * loss against the target.  out receives nc values (GPF_SUM_SOLUTE) or one.
 * Synchronises.  Errors: GPF_ERR_ARG (NULL, unknown reduction),
 * GPF_ERR_STATE (GPF_LOSS without a target), GPF_ERR_DEVICE. */
int gpf_reduce(gpf_ctx* ctx, int32_t which, double* out);

/* gpf_reduce without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid it): the same totals in the same fixed order
 * (bitwise those of gpf_reduce), written to caller-owned device memory
 * dev_out (nc doubles for GPF_SUM_SOLUTE, else one) asynchronously on the
 * context's stream; no host synchronisation, no allocation, no memset.  The
 * partial sums live in a static device array of the library (2048 x 2
 * doubles, 32 KiB, on each GPU it runs on, until the process ends) that
 * every context on that GPU shares and that holds the last call's partials:
 * calls that overlap in time on one GPU (other streams, other host threads)
 * race on it and must be serialised by the caller.  Nothing in it needs
 * clearing: each call overwrites every partial it reads.  Must be called
 * with the context's device current.  Errors: GPF_ERR_ARG (NULL, unknown
 * reduction, more partial sums than the static array holds), GPF_ERR_STATE
 * (GPF_LOSS without a target, another device current), GPF_ERR_DEVICE. */
int gpf_reduce_noalloc(gpf_ctx* ctx, int32_t which, double* dev_out);

/* Measurement, no operation of the paper: the bandwidth (read + write GB/s)
 * that the access pattern of the population update reaches without its
 * arithmetic, the achievable side of the HBM roofline beside the published
 * peak.  pattern 0: copy of 19 FP32 arrays; 1: the D3Q19 pull out_k(P) =
 * in_k(P - c_k) (all axes periodic), one thread per cell; 2: the same pull in
 * the launch shape of the step's dominant kernel (64 x 4 tiles walking 4
 * planes).  dev_in, dev_out: caller-owned device buffers of 19 * n[0] * n[1]
 * * n[2] floats each, layout [k][z][y][x]; out is overwritten with the copied
 * or pulled values.  n[0] a multiple of 64, n[1] and n[2] multiples of 4.
 * Two untimed launches, then `reps` launches timed with HIP events on
 * `stream` (a hipStream_t; NULL: the null stream).  Synchronises.  Errors:
 * GPF_ERR_ARG (NULL, pattern, sizes), GPF_ERR_DEVICE. */
int gpf_bandwidth_probe(int32_t pattern, const void* dev_in, void* dev_out, const int64_t* n, int32_t reps,
                        void* stream, double* gbps);

/* Target phi^target of the loss GPF_LOSS: caller-owned device memory, FP64,
 * N * cells values in the layout of GPF_PHI.  The context keeps the pointer
 * (not the memory): it must stay valid until replaced or cleared (NULL, with
 * count 0).  The paper has no loss; the target is the final microstructure
 * whose parameters the adjoint inverts.  Errors: GPF_ERR_ARG (wrong count). */
int gpf_set_target(gpf_ctx* ctx, const void* dev_target, size_t count);

/* dL/dphi = phi - phi^target of the loss GPF_LOSS at the current state, FP64,
 * into caller-owned device memory of N * cells values (the seed that
 * gpf_adjoint_device takes).  Asynchronous on the context's stream.
 * Errors: GPF_ERR_ARG (NULL, wrong count), GPF_ERR_STATE (no target). */
int gpf_loss_seed_device(gpf_ctx* ctx, void* dev_seed, size_t count);

/* Change one scalar parameter between steps: "delta" (anisotropy strength
 * of the gradient energy a(phi, grad phi) of Eq. (PhfGrand), all anisotropic
 * pairs), "tau_pf" (relaxation tau of Eq. (PhfGrand)), "D" / "D1" (liquid
 * diffusivity of solute 0 / 1 in the mobility M of Eq. (conc)), "gbeta" /
 * "gbeta1" (products g beta_i of Eq. (buoyancy)): the parameters the adjoint
 * differentiates.  Re-validated like gpf_init.  Errors: GPF_ERR_ARG (unknown
 * name), GPF_ERR_PARAM (invalid value; the context is then unchanged). */
int gpf_set_param(gpf_ctx* ctx, const char* name, double value);

/* Adjoint (reverse mode of the discrete step, hand-written kernels).
 *
 * gpf_record: the current state becomes checkpoint 0 of a recording; every
 * later gpf_step stores a full-state checkpoint each `checkpoint_every`
 * steps (device memory: (N + nc + dim + Q) * cells values per checkpoint;
 * gpf_adjoint adds a tape of checkpoint_every - 1 states of
 * (N + nc + dim + 1) * cells values, two population buffers and the adjoint
 * state; with more than one segment a second tape, into which the previous
 * segment is recomputed on a second stream during the reverse of the current
 * one, when it fits: if its allocation fails the sweep runs with one tape,
 * bitwise the same results).  Checkpoint m belongs to step (start + m checkpoint_every): a state
 * restored to an earlier step and stepped again overwrites the later ones;
 * gpf_step fails with GPF_ERR_STATE at a checkpoint step before the start of
 * the recording or past the next checkpoint in sequence.
 * Errors: GPF_ERR_ARG (checkpoint_every < 1), GPF_ERR_NOMEM.
 *
 * gpf_adjoint: given dL/dphi at the current state (FP64 host array of
 * N * cells values, layout of GPF_PHI), propagates the adjoint back through
 * every step since gpf_record -- each segment between checkpoints is
 * recomputed into a tape of checkpoint_every states -- and writes the FP64
 * derivatives dL/dp for the named scalar parameters ("delta": the anisotropy
 * strength of every pair that has one; "tau_pf": the relaxation of Eq.
 * (PhfGrand); "D" / "D1": liquid diffusivity of solute 0 / 1; "gbeta" /
 * "gbeta1": buoyancy products of Eq. (buoyancy)) to grads_out[0..n_names).
 * The forward state is left unchanged.  Parameter derivatives are
 * accumulated in FP64 in a fixed order; the adjoint fields have the
 * context's precision.  Synchronises.  Errors: GPF_ERR_STATE (nothing
 * recorded), GPF_ERR_ARG (count, unknown name, more than 6 names),
 * GPF_ERR_UNSUPPORTED (shrinkage force on: eta != 0, or a moving frame),
 * GPF_ERR_NOMEM.
 *
 * gpf_adjoint_device: gpf_adjoint with dL/dphi in device memory (FP64,
 * same count and layout, e.g. a loss gradient computed on the GPU), read on
 * the library's stream; the caller keeps ownership and must not change it
 * before the call returns.  Same errors.
 *
 * gpf_adjoint_state: after gpf_adjoint, dL/d(initial recorded state) for
 * GPF_PHI, GPF_MU, GPF_U (velocity of the step before) or GPF_F (the
 * populations after streaming), FP64, components * cells values. */
int gpf_record(gpf_ctx* ctx, int64_t checkpoint_every);
int gpf_adjoint(gpf_ctx* ctx, const double* dL_dphi, size_t count, const char* const* names,
                int32_t n_names, double* grads_out);
int gpf_adjoint_device(gpf_ctx* ctx, const void* dev_dL_dphi, size_t count, const char* const* names,
                       int32_t n_names, double* grads_out);
int gpf_adjoint_state(gpf_ctx* ctx, int32_t field, double* host_dst, size_t count);

/* Step counter n of the time loop of Algorithm phfLBM (App. A); it sets the
 * time of the pulled temperature T_E + G (x - y0 - V n) of Case 2 (Sec. 3).
 * The setter is for resuming a checkpoint; n >= 0 (else GPF_ERR_ARG). */
int64_t gpf_step_index(const gpf_ctx* ctx);
int gpf_set_step_index(gpf_ctx* ctx, int64_t n);
/* Cells the moving frame of Case 2 (Sec. 3) has shifted the fields along the
 * pull axis so far (laboratory coordinate = grid index + offset; the pulled
 * temperature uses it).  The setter is for resuming a checkpoint; offset >= 0
 * (else GPF_ERR_ARG). */
int64_t gpf_frame_offset(const gpf_ctx* ctx);
int gpf_set_frame_offset(gpf_ctx* ctx, int64_t offset);
/* Error reporting and teardown (no operation of the paper).  gpf_last_error:
 * message of the last failing call on ctx (NULL ctx: of the last failed
 * gpf_init on this thread); the string belongs to the library and lives
 * until the next call on ctx.  gpf_status_string: a static name of a
 * gpf_status.  gpf_destroy: waits for the context's stream, releases every
 * device buffer (through dev_free when given) and the context; NULL is a
 * no-op. */
const char* gpf_last_error(const gpf_ctx* ctx);
const char* gpf_status_string(int status);
void gpf_destroy(gpf_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
