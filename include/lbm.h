/*
 * C ABI of the MI355X cuboid D3Q27 central-moment lattice Boltzmann step.
 *
 * Method: the 3D cuboid central-moment LB scheme (3DCCM-LBM) of Yahia,
 * Schupbach and Premnath, arXiv:2107.14774.  One step gathers the 27
 * populations of a node (streaming, Sec. 3.2), takes raw moments (App. A),
 * scales them by the grid aspect ratios r, s (App. B, eq. 59), shifts them to
 * central moments about the force-shifted velocity of eq. 12 (App. C),
 * relaxes them with the shear rate omega_nu, the bulk rate omega_xi and one
 * rate omega_hi for every higher order (1 in the paper), using the extended
 * equilibria whose
 * corrections cancel the grid-anisotropy and non-Galilean-invariant errors
 * (Sec. 2.4, eq. 38-40) with strain rates from the local system of App. D
 * (eq. 44-49), adds the body force through eq. 11c, and maps back (App. E-G).
 * Streaming is periodic or halfway bounce-back along each axis; bounce-back
 * faces may move tangentially (momentum-augmented bounce-back, Sec. 4,
 * eq. 69).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Lattice units: dx = dt = 1, dy = r, dz = s (Sec. 2.1).  Velocities and
 *   forces are in x-lengths per step.
 * - Node index n = (z * ny + y) * nx + x, x fastest.  Fields are SoA:
 *   a scalar field is n_nodes values, a vector field is [3][n_nodes].
 * - Direction order alpha = 0..26 is that of eq. 1a-c.  "Natural" population
 *   arrays are [27][n_nodes] (double unless stated), f_alpha(x, t) after
 *   streaming, i.e. the state from which eq. 12 reads rho and u.
 * - A "state" is opaque device memory of lbm_state_bytes() bytes holding one
 *   time level in the library's own layout: 27 * lbm_state_stride() elements
 *   (float, or 16-bit for the reduced-storage modes) holding deviations from
 *   the rest equilibrium w_alpha rho0 (scaled for F16), placed so that the next
 *   step can gather them (pull scheme).  The layout is blocked: every x-row is
 *   padded to a multiple of 128 nodes and cut into blocks of 128 nodes, and a
 *   block holds the 27 directions of its nodes as 27 runs of 128 elements;
 *   lbm_state_stride() is the padded node count.  Callers only allocate it and
 *   pass it between calls; lbm_import/lbm_export convert natural populations.
 * - Memory: the caller allocates every device buffer (PyTorch in the Python
 *   binding); the library never allocates or frees device memory.  The only
 *   host allocation is the handle.  All pointers to device memory must be
 *   16-byte aligned.
 * - Streams: hip_stream is a hipStream_t passed as void* (NULL = the null
 *   stream).  Every call only enqueues work and returns; no call synchronises
 *   unless its comment says so.
 * - Errors: every int-returning call returns LBM_OK (0) or a negative status;
 *   lbm_last_error() returns a thread-local message for the last failure.
 *   No C++ exception crosses the ABI.
 */
#ifndef CUBOID_LBM_H
#define CUBOID_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = -1,      /* invalid argument (sizes, rates, pointers, alignment) */
  LBM_EHIP = -2,        /* HIP runtime or launch error; message from HIP */
  LBM_ESTATE = -3,      /* handle/state misuse (e.g. NULL handle) */
  LBM_ENONFINITE = -4   /* lbm_check_sums found a NaN/Inf total */
};

enum lbm_bc { LBM_PERIODIC = 0, LBM_BOUNCEBACK = 1 };

/* Population storage.  F32 stores (f - w rho0) in float.  F16 stores
 * (f - w rho0) * sigma_alpha rounded to nearest even, sigma_alpha a power of
 * two near 1 / w_alpha (keeps the deviations in FP16's normal range).  BF16
 * stores (f - w rho0) rounded to nearest even (BF16 has FP32's exponent range).
 * BF16_SR is BF16 whose step stores round stochastically: up with probability
 * equal to the discarded fraction, from a counter-based generator keyed by the
 * node, the direction's value and the handle's step counter
 * (lbm_set_step_counter), so the rounding is unbiased where a slowly changing
 * flow would round the same way every step; init and import round to nearest.
 * Every arithmetic step is FP32. */
enum lbm_storage { LBM_F32 = 0, LBM_F16 = 1, LBM_BF16 = 2, LBM_BF16_SR = 3 };

/* Extended-equilibrium corrections (Sec. 2.4 / App. D).
 * OFF:     plain central-moment collision on the cuboid lattice;
 * LOWMACH: theta without the 3u^2 terms (last remark of Sec. 2.4);
 * LOCAL:   theta with the 3u^2 terms; the density-gradient (lambda) terms,
 *          which need a non-local finite difference, are left out;
 * FULL:    LOCAL plus the lambda terms of eq. 38-40 and the e_rho terms of
 *          the strain-rate system (App. D), with the density gradient from a
 *          density field: only lbm_step_full runs it (lbm_step and
 *          lbm_step_adjoint reject it). */
enum lbm_corr { LBM_CORR_OFF = 0, LBM_CORR_LOWMACH = 1, LBM_CORR_LOCAL = 2, LBM_CORR_FULL = 3 };

/* Moments the collision relaxes.  CENTRAL: the 3DCCM-LBM (Sec. 3.2).  RAW:
 * the raw-moment scheme of Sec. 7 (3DCRM-LBM): the same steps without the
 * frame transformation around the collision, with raw equilibria (eq. 10),
 * the same corrections, and the raw image F(-u) Phi^c of the central source
 * (eq. 11c); the strain rates of the corrections come from the same
 * non-equilibrium moments. */
enum lbm_moments_basis { LBM_CENTRAL = 0, LBM_RAW = 1 };

/* Memory layout of a state.
 * AB: two buffers; a step gathers from one and writes the other (pull), and
 *     the state holds post-collision populations placed where the next step
 *     gathers them (lbm_step's state_a / state_b).
 * AA: one buffer updated in place, half the memory.  Steps alternate between
 *     a local one (read the node's own slots, write the collided populations
 *     to the opposite-direction slots of the same node) and a shifted one
 *     (read the neighbours' opposite-direction slots, write to the
 *     neighbours' own slots); each slot is read and written by one node only.
 *     Between calls the state holds the post-stream populations in natural
 *     order (slot (a, x) = f_a(x, t)), so every step call must advance an even
 *     number of steps.  Forward steps only: lbm_step, lbm_step_forcing (not
 *     the full corrections, not the adjoint).  With walls it addresses the
 *     state through 32-bit offsets, so lbm_create returns LBM_EINVAL for a
 *     walled AA state of 4 GiB or more. */
enum lbm_layout { LBM_LAYOUT_AB = 0, LBM_LAYOUT_AA = 1 };

/* Time level of the density gradient of the full corrections (lbm_step_full). */
enum lbm_grad_mode { LBM_GRAD_EXACT = 0, LBM_GRAD_LAGGED = 1, LBM_GRAD_EXACT_DRHO = 2 };

/* Walls.  On a bounce-back axis the walls sit half a cell outside the first
 * and last node.  A population whose upstream node lies beyond a wall is the
 * node's own outgoing population of the opposite direction, plus, for a
 * moving wall, the momentum term of Sec. 4:
 *   f_a(x, t+1) = f~_abar(x, t) - [f_eq_abar - f_eq_a](rho(x, t), u_w),
 * f_eq the product-form equilibrium (eq. 9 mapped to populations), rho the
 * fluid node's density (the paper's rho_w = rho_f) and u_w the face velocity;
 * a lid moving along x gives exactly the coefficients of eq. 69.  A link that
 * leaves through two or three faces at an edge or corner takes the mean
 * velocity of the moving faces among them (zero if none moves), so a lid
 * meets the side walls without a mass source.  Faces are numbered
 * 0..5 = x-, x+, y-, y+, z-, z+. */
typedef struct lbm_params {
  int32_t nx, ny, nz;   /* grid nodes; each >= 1; >= 2 on a bounce-back axis */
  double r, s;          /* grid aspect ratios dy/dx and dz/dx (Sec. 2.1), > 0 */
  double cs2;           /* squared sound speed; <= 0 selects min(r^2, s^2)/3 (end of Sec. 2.5) */
  double omega_nu;      /* shear rate, 0 < omega_nu < 2: nu = cs2 (1/omega_nu - 1/2) (eq. 53) */
  double omega_xi;      /* bulk rate, 0 < omega_xi < 2: xi = (2 cs2/3)(1/omega_xi - 1/2) */
  double omega_hi;      /* rate of every third- and higher-order moment, 0 < omega_hi < 2
                           (App. D; the paper uses 1, the fastest kernels); other values
                           select kernels that keep the gathered populations live */
  int32_t bc_x, bc_y, bc_z; /* enum lbm_bc per axis */
  int32_t storage;      /* enum lbm_storage */
  int32_t corr;         /* enum lbm_corr */
  int32_t moments;      /* enum lbm_moments_basis */
  int32_t layout;       /* enum lbm_layout */
  double rho0;          /* reference density of the stored deviations, > 0 (usually 1) */
  double force[3];      /* uniform body force used when no force field is passed */
  double wall_velocity[6][3]; /* velocity of each face (x-, x+, y-, y+, z-, z+); must be
                                 zero on periodic axes and along the face normal */
} lbm_params;

typedef struct lbm_handle lbm_handle;

/* Relaxation rates from viscosities (eq. 53 and the bulk viscosity of
 * Sec. 2.5): omega_nu = 1 / (nu / cs2 + 1/2), omega_xi = 1 / (3 xi / (2 cs2)
 * + 1/2), the inverse of the lbm_params definitions of nu and xi.  Host-side
 * only.  LBM_EINVAL unless nu > 0, xi > 0, cs2 > 0 (all finite) and both
 * pointers are non-NULL; the rates then lie in (0, 2). */
int lbm_relaxation_rates(double nu, double xi, double cs2, double* omega_nu, double* omega_xi);

/* Validate p and create a host-side handle holding the derived constants.
 * Rejects (LBM_EINVAL): a size < 1 (or < 2 on a bounce-back axis), more than
 * 2^31 - 1 nodes, r or s <= 0, a rate outside (0, 2), a sound
 * speed that makes a rest weight <= 0 (cs2 >= min(1, r^2, s^2)), unknown enum
 * values, rho0 <= 0, a non-finite force or wall velocity, a wall velocity on
 * a periodic axis or with a component along its face normal. */
int lbm_create(const lbm_params* p, lbm_handle** out);
void lbm_destroy(lbm_handle* h);

/* Bytes of one state (27 * stride * element size) and the slots per direction
 * (the node count with every x-row padded to a multiple of 128 nodes); an
 * adjoint array (below) has 27 * stride floats. */
size_t lbm_state_bytes(const lbm_handle* h);
int64_t lbm_state_stride(const lbm_handle* h);
int64_t lbm_num_nodes(const lbm_handle* h);

/* Step counter of the handle: every step that lbm_step, lbm_step_forcing or
 * lbm_step_full launches takes the counter's value as the key of its stochastic
 * rounding (BF16_SR storage) and advances it by one; other storage ignores it.
 * lbm_create starts it at 0.  Setting it back to the value a step had makes a
 * recomputation of that step from the same state reproduce it bit for bit (the
 * adjoint's checkpoint recomputation does this).  Host-side only. */
int lbm_set_step_counter(lbm_handle* h, uint64_t counter);
uint64_t lbm_step_counter(const lbm_handle* h);

/* Thread-local description of the last error (empty string if none). */
const char* lbm_last_error(void);

/* Initial state f(x, 0) = f_eq(rho, u) (+ perturb), eq. 9 mapped to
 * populations (equivalently f_eq = Q^-1 m_eq, eq. 10 and eq. 56), computed in
 * FP64 and rounded once into the storage format.
 *   rho:     device double[n_nodes] or NULL (then rho = rho0 everywhere)
 *   u:       device double[3][n_nodes] or NULL (then u = 0)
 *   perturb: device double[27][n_nodes] added to f_eq, or NULL
 *   state:   device, lbm_state_bytes(h) bytes, written. */
int lbm_init(lbm_handle* h, void* state, const double* rho, const double* u,
             const double* perturb, void* hip_stream);

/* Write natural populations f (device double[27][n_nodes]) into a state,
 * and read them back.  lbm_export(lbm_import(f)) returns f up to the
 * rounding of the storage format. */
int lbm_import(lbm_handle* h, void* state, const double* f, void* hip_stream);
int lbm_export(lbm_handle* h, const void* state, double* f, void* hip_stream);

/* Natural populations of `count` listed nodes (a sampled lbm_export, for
 * states too large to export whole):
 *   nodes: device int64[count], node indices n = (z ny + y) nx + x; an index
 *          outside [0, n_nodes) yields NaN in all 27 of its values
 *   f:     device double[27][count], f[alpha][i] = f_alpha at nodes[i]
 * count = 0 does nothing; LBM_EINVAL for count < 0 or a NULL pointer. */
int lbm_export_nodes(lbm_handle* h, const void* state, const int64_t* nodes, int64_t count, double* f,
                     void* hip_stream);

/* Advance nsteps >= 0 collide-and-stream steps (Sec. 3.2).  The current state
 * is in state_a on entry; state_b is scratch of the same size (must differ
 * from state_a).  On return the current state is in state_a when nsteps is
 * even and in state_b when it is odd.  AA layout: state_b is not used (NULL
 * or equal to state_a), nsteps must be even (LBM_EINVAL otherwise) and the
 * state stays in state_a.
 *   force: device float[3][n_nodes] per-node body force, or NULL to use
 *          p->force for every node. */
int lbm_step(lbm_handle* h, int32_t nsteps, void* state_a, void* state_b,
             const float* force, void* hip_stream);

/* Replace the handle's uniform body force (p->force), used by every later call
 * that is given no force field.  Host-side only (no GPU work); must not run
 * concurrently with other calls on the same handle.  LBM_EINVAL if a
 * component is not finite. */
int lbm_set_force(lbm_handle* h, const double force[3]);

/* Advance nsteps >= 0 steps like lbm_step, step t using the uniform body force
 * forces[3 t .. 3 t + 2] instead of p->force (a time-dependent forcing such as
 * the pulsatile duct of Sec. 5.2, F_x = F_m cos(omega t)).
 *   forces: HOST double[nsteps][3], read before the call returns (it may be
 *           freed afterwards); LBM_EINVAL if NULL or not finite.
 * p->force is left unchanged; pass the force of the current time to
 * lbm_set_force before lbm_moments to read eq. 12's velocity at that time. */
int lbm_step_forcing(lbm_handle* h, int32_t nsteps, void* state_a, void* state_b,
                     const double* forces, void* hip_stream);

/* Density deviation rho - rho0 of every node of a state (the sum of its 27
 * gathered populations minus rho0, eq. 12), in FP32, bit-identical to the
 * density the step computes for that node.
 *   drho: device float[n_nodes], written. */
int lbm_density(lbm_handle* h, const void* state, float* drho, void* hip_stream);

/* Advance nsteps >= 0 steps with the full corrections (p->corr must be
 * LBM_CORR_FULL; LBM_EINVAL otherwise).  App. D takes the density gradient
 * from an isotropic second-order finite difference; the library uses the
 * lattice-weighted stencil grad rho (x) = (1/cs2) sum_a w_a e_a rho(x + ebar_a)
 * (w_a the rest weights, e_a the cuboid velocities), with periodic wrap and,
 * across a bounce-back wall, the boundary node's own value (its mirror
 * image).  States behave as in lbm_step.  The density fields hold rho - rho0:
 *   mode LBM_GRAD_EXACT:  before each step the density of its input state is
 *       written to drho_a and the gradient is taken from it (gradient and
 *       collision at the same time level; one more read of the state per
 *       step).  drho_b is not used and may be NULL.
 *   mode LBM_GRAD_LAGGED: drho_a holds on entry the field the first step
 *       takes its gradient from (normally lbm_density of state_a, which makes
 *       the first step exact).  Each step writes the density of its own input
 *       state into the other buffer, and the next step takes its gradient from
 *       there, one step behind.  On return the field the next call starts from
 *       is in drho_a when nsteps is even and in drho_b when it is odd, so a
 *       run split over several calls equals one call.  drho_b must differ
 *       from drho_a.
 *   drho_a, drho_b: device float[n_nodes]. */
int lbm_step_full(lbm_handle* h, int32_t nsteps, void* state_a, void* state_b,
                  const float* force, float* drho_a, float* drho_b, int32_t mode,
                  void* hip_stream);

/* Streaming only: nsteps >= 0 steps of lbm_step's gather and store with the
 * collision left out, f_a(x, t+1) = f_a(x - ebar_a, t), or f_abar(x, t) where
 * x - ebar_a lies beyond a wall (the streaming bullet of Sec. 3.2 and the
 * bounce-back of Sec. 4 with stationary walls).  It moves the step's bytes in
 * the step's access pattern with the step's launch shape (two nodes per thread
 * where the 16-bit step uses them), so its throughput is
 * the ceiling that pattern allows on the device: the reference the step's
 * memory throughput is reported against.  States behave as in lbm_step.
 * LBM_EINVAL for the AA layout, for moving walls, or state_a == state_b. */
int lbm_stream(lbm_handle* h, int32_t nsteps, void* state_a, void* state_b, void* hip_stream);

/* The adjoint step's data movement with its arithmetic left out: gathers
 * state_t as lbm_step does, reads adj_in where lbm_step_adjoint reads
 * lambda(t+1), reads force and adds it to grad_force (both optional, as in
 * lbm_step_adjoint), and writes adj_out = gathered population + that lambda
 * value at each of the node's own elements.  It moves lbm_step_adjoint's bytes
 * (without the moving-wall pass) in its access pattern, block shape and
 * occupancy, so its throughput is the ceiling that pattern allows on the
 * device: the reference the adjoint step's memory throughput is reported
 * against.  Arrays as in lbm_step_adjoint.  LBM_EINVAL for the AA layout or
 * adj_in == adj_out. */
int lbm_adjoint_stream(lbm_handle* h, const void* state_t, const float* adj_in, float* adj_out,
                       const float* force, float* grad_force, void* hip_stream);

/* Device-to-device copy of `bytes` bytes (a multiple of 16; 0 does nothing)
 * with one 16-byte non-temporal load and store per thread: the reference for
 * the read-and-write bandwidth of the device.  dst and src: device, 16-byte
 * aligned, not overlapping (LBM_EINVAL otherwise).  Needs no handle. */
int lbm_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* Observables of a state (eq. 12 / the last bullet of Sec. 3.2):
 * rho = sum f, u = (sum f e + F/2) / rho.
 *   rho:  device float[n_nodes] or NULL
 *   u:    device float[3][n_nodes] or NULL
 *   sums: device double[5] or NULL: total mass sum rho, momentum sum rho u
 *         (3), kinetic energy sum rho |u|^2 / 2, each per node (multiply by
 *         r s for a physical volume), accumulated in FP64.
 *   force: as in lbm_step. */
int lbm_moments(lbm_handle* h, const void* state, const float* force, float* rho,
                float* u, double* sums, void* hip_stream);

/* Synchronises hip_stream, copies the 5 sums to the host (out may be NULL)
 * and returns LBM_ENONFINITE if any is NaN or Inf. */
int lbm_check_sums(const double* sums_device, double* out_host, void* hip_stream);

/* ---------------------------------------------------------------- adjoint
 * The step maps a state h(t) to h(t+1) = C(S(h(t)); F): S streams (a
 * permutation of the population slots), C collides every node.  The adjoint
 * step is lambda(t) = [dh(t+1)/dh(t)]^T lambda(t+1), taken with respect to
 * the real-valued populations (the rounding of 16-bit storage is not
 * differentiated; values not scaled).  An adjoint array is float[27 * stride]
 * in the state's blocked layout, in gathered-population order: the element
 * of slot (a, x) holds the cotangent of the population that the next step
 * gathers as f_a at node x, i.e. of the slot (a, x - ebar_a), or (opp(a), x)
 * across a wall.  In this order the step stores its results at each node's
 * own slots and reads lambda(t+1) in the shape of the forward gather.
 *
 *   state_t:    the state h(t) before the step (read)
 *   adj_in:     lambda(t+1), device float[27 * stride] (read)
 *   adj_out:    lambda(t),   device float[27 * stride] (written; != adj_in)
 *   force:      as in lbm_step
 *   grad_force: device float[3][n_nodes] or NULL: += (dh(t+1)/dF)^T lambda(t+1)
 *               for a per-node force field
 *   grad_force_uniform: device double[3] or NULL: += the same summed over
 *               nodes (gradient with respect to the uniform force).
 * Moving walls (their terms depend on the node's density), the raw-moment
 * scheme and a general omega_hi are included.  The full corrections take
 * lbm_step_adjoint_full (below; LBM_EINVAL here); the AA layout has no adjoint
 * (LBM_EINVAL; also for the other adjoint entry points below). */
int lbm_step_adjoint(lbm_handle* h, const void* state_t, const float* adj_in,
                     float* adj_out, const float* force, float* grad_force,
                     double* grad_force_uniform, void* hip_stream);

/* The adjoint step of the full corrections (one step of lbm_step_full; App.
 * D's lambda and e_rho terms and the density gradient of its isotropic
 * stencil).  Arguments as in lbm_step_adjoint (the handle's corrections must
 * be LBM_CORR_FULL, LBM_EINVAL otherwise), plus fields the caller provides
 * (the library allocates nothing):
 *   drho:      device float[n_nodes]: the density field the step took its
 *              gradient from.  LBM_GRAD_EXACT: written here (the density of
 *              state_t).  LBM_GRAD_EXACT_DRHO: the exact level with drho
 *              already holding state_t's density as lbm_density or the
 *              LBM_GRAD_EXACT lbm_step_full step from state_t wrote it (read;
 *              saves the density pass).  LBM_GRAD_LAGGED: read (the density of
 *              the previous step's input, or of state_t for the first step of
 *              a run).
 *   grad_work: device float[3][n_nodes]: receives the cotangent of the step's
 *              density gradient (LBM_GRAD_LAGGED also stages the transpose of
 *              grad_pending in it during the call).
 *   grad_pending: device float[3][n_nodes] or NULL, LBM_GRAD_LAGGED only:
 *              the cotangent of the next step's gradient, which that step took
 *              from this state's density (the grad_work of the previous call
 *              of the reverse sweep); its stencil transpose is added to
 *              adj_out.  Must differ from grad_work.
 * LBM_GRAD_EXACT(_DRHO): the gradient came from state_t's own density, so its
 * cotangent flows back through the stencil into adj_out before return.
 * LBM_GRAD_LAGGED: it belongs to the state the gradient was taken from; pass
 * grad_work as grad_pending to the next call of the sweep, and after the run's
 * first step (whose gradient came from its own input) add it to lambda(0)
 * with lbm_density_adjoint. */
int lbm_step_adjoint_full(lbm_handle* h, int32_t mode, const void* state_t, const float* adj_in,
                          float* adj_out, const float* force, float* grad_force,
                          double* grad_force_uniform, float* drho, float* grad_work,
                          const float* grad_pending, void* hip_stream);

/* lbm_step_adjoint_full at the exact time level (LBM_GRAD_EXACT) without work
 * fields, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the density
 * and the gradient cotangent go to a static 64 MiB device array of the library
 * (one per device, held from library load to process exit), so the call
 * allocates nothing.  Arguments, results and errors as lbm_step_adjoint_full
 * with mode LBM_GRAD_EXACT; LBM_EINVAL if the grid needs more than the array
 * (16 B per node: at most 4,194,288 nodes).  All calls on one device share the
 * array: calls that overlap in time on one device (different streams, or
 * different host threads) race; calls on one stream are ordered and safe.  No
 * part of the array needs to start at zero. */
int lbm_step_adjoint_full_noalloc(lbm_handle* h, const void* state_t, const float* adj_in,
                                  float* adj_out, const float* force, float* grad_force,
                                  double* grad_force_uniform, void* hip_stream);

/* adj += the transpose of the full corrections' density-gradient stencil
 * applied to grad (device float[3][n_nodes], a cotangent of the gradient),
 * added to every population each node gathered (d rho / d f = 1).  adj: an
 * adjoint array (float[27 * stride], gathered-population order). */
int lbm_density_adjoint(lbm_handle* h, const float* grad, float* adj, void* hip_stream);

/* lambda(T) from cotangents of the observables of a state (the transpose of
 * lbm_moments' rho/u map):
 *   g_rho: device float[n_nodes] or NULL;  g_u: device float[3][n_nodes] or NULL
 *   adj:   device float[27 * stride], written (overwritten, not accumulated)
 *   grad_force: device float[3][n_nodes] or NULL, += d(u)/dF^T g_u (the F/2 of eq. 12). */
int lbm_moments_adjoint(lbm_handle* h, const void* state, const float* force,
                        const float* g_rho, const float* g_u, float* adj,
                        float* grad_force, void* hip_stream);

/* Cotangents of the initial fields from lambda(0) (transpose of lbm_init's
 * f_eq(rho, u) map at the given rho, u):
 *   adj:   device float[27 * stride] (read)
 *   rho, u: as in lbm_init (NULL = rho0 / zero)
 *   g_rho: device double[n_nodes] or NULL, written
 *   g_u:   device double[3][n_nodes] or NULL, written */
int lbm_init_adjoint(lbm_handle* h, const float* adj, const double* rho,
                     const double* u, double* g_rho, double* g_u, void* hip_stream);

/* Reorder an adjoint array into natural order and back: natural[alpha][n]
 * is its element of slot (alpha, n), the cotangent of the population that
 * the next step gathers as f_alpha at node n.  natural is device
 * double[27][n_nodes]. */
int lbm_adjoint_to_natural(lbm_handle* h, const float* slots, double* natural, void* hip_stream);
int lbm_adjoint_from_natural(lbm_handle* h, const double* natural, float* slots, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* CUBOID_LBM_H */
