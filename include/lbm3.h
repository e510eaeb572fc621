/*
 * lbm3.h -- C ABI of the MI355X ternary colour-gradient lattice Boltzmann library.
 *
 * The library advances three immiscible fluids on a periodic D2Q9 lattice with
 * the model of Yu, Liu, Liang and Zhang, "A versatile lattice Boltzmann model
 * for immiscible ternary fluid flows" (arXiv:1808.08555), Sec. 2.  One time step
 * computes the colour gradients of the three densities, the N-phase interfacial
 * force (Eq. 7) applied as a Guo body force (Eqs. 8-9) in the BGK collision of
 * the total distribution (Eqs. 1-3) with a harmonic-mean viscosity (Eqs. 10-11),
 * the generalized recolouring (Eq. 13) with the proposed segregation parameters
 * (Eqs. 18-20), and streaming (Eq. 22).
 *
 * Conventions shared by every call
 *   - Fluids k = 0, 1, 2 are the paper's red, green, blue ("fluid 1, 2, 3").
 *   - sigma[0] = sigma_rg (12), sigma[1] = sigma_rb (13), sigma[2] = sigma_gb (23).
 *   - Host arrays are C-contiguous float64 with x fastest:
 *       densities  rho[3][ny][nx],  velocities u[2][ny][nx],
 *       populations f[3][9][ny][nx]  (post-streaming state, direction order
 *       e_0 = (0,0), e_1 = (1,0), e_2 = (0,1), e_3 = (-1,0), e_4 = (0,-1),
 *       e_5 = (1,1), e_6 = (-1,1), e_7 = (-1,-1), e_8 = (1,-1)).
 *   - Return value: LBM3_OK (0) or a negative LBM3_E* code; a message is kept in
 *     lbm3_last_error() (per thread).  No call exits, aborts or throws.
 *   - Ownership: a handle owns all of its device memory; the caller owns every
 *     host array, which calls read or fill before they return and never keep.
 *   - Streams: work is ordered on the HIP stream given at create time (NULL =
 *     the null stream).  Only calls documented as blocking synchronise the host.
 */
#ifndef LBM3_H
#define LBM3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM3_OK = 0,
    LBM3_EINVAL = -1,      /* invalid argument, parameter or field */
    LBM3_ENOMEM = -2,      /* device or host allocation failed */
    LBM3_EDEVICE = -3,     /* a HIP runtime call failed (message names it) */
    LBM3_EUNSUPPORTED = -4,/* a feature the library does not provide (walls) */
    LBM3_ENONFINITE = -5,  /* the state holds a NaN or Inf */
    LBM3_ESTATE = -6       /* call out of order (e.g. step before init_fields) */
};

enum {
    LBM3_FP64 = 0,         /* populations stored and computed in FP64 */
    LBM3_FP32_STORAGE = 1, /* populations stored in FP32, arithmetic in FP64 */
    LBM3_FP32 = 2          /* populations stored and computed in FP32 */
};

enum { LBM3_PERIODIC = 0 };

/* Segregation law of the recolouring, Eq. (13).  Every law has the form
 * beta_kl = beta^0 (1 + s g_kl), with the host constants g_kl of lbm3_derived
 * and s a function of the node's densities:
 *   PAPER     Eqs. (18)-(20): s = C_t = min(35 rho_r rho_g rho_b / rho^3, 1),
 *             g_kl = g(X_kl) of Eq. (20);
 *   SPENCER   Eq. (15), as printed: s = 27 rho_r rho_g rho_b / rho^3 (at most 1),
 *             g_rg = 0, g_rb = sin(phi_gb) - 1, g_gb = sin(phi_rb) - 1, with phi_kl
 *             the Neumann-triangle angle of Eq. (14) (cos(phi_kl) = X_kl, clamped to
 *             [-1, 1] when no triangle exists);
 *   LECLAIRE  Eq. (16): s = C_t, g_kl = 0 for the pair of the largest phi_kl (the
 *             first in the order rg, rb, gb on ties) and sin(pi - phi_max - phi_kl) - 1
 *             for the other two; all g_kl = 0 when no triangle exists;
 *   CONSTANT  Eq. (17): beta_kl = beta^0 (all g_kl = 0). */
enum {
    LBM3_BETA_PAPER = 0,
    LBM3_BETA_SPENCER = 1,
    LBM3_BETA_LECLAIRE = 2,
    LBM3_BETA_CONSTANT = 3
};

/* How the interfacial tension enters the collision (Eq. 1):
 *   GUO           the paper's method: the force F = div T of Eq. (7) (T from the pair
 *                 sum of the colour gradients, Eq. 12 for the divergence), applied with
 *                 Guo's term of Eq. (8) and the half-force velocity of Eq. (9);
 *   PERTURBATION  the comparison method of Eqs. (4)-(5): no force; the node-local
 *                 operator Phi_i = sum_k sum_{l != k} (A_kl C_kl / 2) |G_kl|
 *                 [w_i (e_i . G_kl)^2 / |G_kl|^2 - B_i] with A_kl = A_lk = 9 sigma_kl /
 *                 (2 tau) at the node's own tau (Eqs. 10-11), B_0 = -4/27,
 *                 B_1-4 = 2/27, B_5-8 = 5/108, and u = sum_i f_i e_i / rho.  Every
 *                 launch form (one or two steps per launch, the batch when all its
 *                 instances use it); no adjoint. */
enum {
    LBM3_FORCING_GUO = 0,
    LBM3_FORCING_PERTURBATION = 1
};

/* The problem as the paper states it (Sec. 2 and the set-ups of Sec. 3):
 * lattice size, pure-fluid densities rho_k^0 (Eq. 6), interfacial tensions
 * sigma_kl (Eq. 7), per-fluid relaxation times tau_k (nu_k = (tau_k - 1/2)/3,
 * Eq. 11), reference segregation parameter beta^0 (Eq. 19), periodic
 * boundaries.  Wall wettability is reserved: the paper has no wall model. */
typedef struct {
    int32_t nx, ny;              /* 1..65535 each (device memory sets the practical limit) */
    double rho0[3];              /* > 0 (the paper validates equal densities 1) */
    double sigma[3];             /* finite, > 0 */
    double tau[3];               /* finite, > 0.5 */
    double beta0;                /* 0 selects 0.7; else finite, > 0 */
    int32_t boundary;            /* LBM3_PERIODIC only, else LBM3_EUNSUPPORTED */
    double wall_wettability[3];  /* reserved: must be 0, else LBM3_EUNSUPPORTED */
    int32_t precision;           /* LBM3_FP64 | LBM3_FP32_STORAGE | LBM3_FP32 */
    int32_t beta_law;            /* LBM3_BETA_*; 0 (the paper's law) when zero-initialised */
    int32_t forcing;             /* LBM3_FORCING_*; 0 (Guo, the paper's) when zero-initialised */
} lbm3_params;

/* Observables of the current state (the velocity is the half-force velocity of
 * Eq. 9; u_max is the maximum spurious velocity of Table 2). */
typedef struct {
    int64_t step;            /* steps taken since init_fields / set_state */
    double mass[3];          /* sum over nodes of rho_k */
    double momentum[2];      /* sum over nodes of rho u */
    double kinetic_energy;   /* sum over nodes of rho |u|^2 / 2 */
    double u_max;            /* max over nodes of |u| */
    int32_t nonfinite;       /* 1 when a density, momentum or velocity is NaN or Inf */
} lbm3_obs;

typedef struct lbm3 lbm3_t;
typedef struct lbm3_batch lbm3_batch_t;

/* Validates *p (EINVAL / EUNSUPPORTED before any device work), precomputes the
 * segregation constants of Eqs. (18)-(20) on the host in FP64 and allocates the
 * two population buffers on the current HIP device.  hip_stream: a hipStream_t
 * or NULL.  On failure *out is set to NULL. */
int lbm3_create(const lbm3_params *p, void *hip_stream, lbm3_t **out);

/* Sets the state from densities (and optionally velocities): with u == NULL
 * f_{i,k} = w_i rho_k, else f_{i,k} = (rho_k/rho) f_eq_i(rho, u) with f_eq of
 * Eq. (3).  rho: host [3][ny][nx], finite, >= 0, with rho > 0 at every node;
 * u: host [2][ny][nx] finite, or NULL.  EINVAL leaves the state unchanged.
 * Resets the step counter.  Returns after the host arrays have been copied. */
int lbm3_init_fields(lbm3_t *h, const double *rho, const double *u);

/* Sets the state from post-streaming populations f: host [3][9][ny][nx],
 * finite.  Resets the step counter. */
int lbm3_set_state(lbm3_t *h, const double *f);

/* Enqueues n >= 0 full time steps (Sec. 2: gradient, force, collision,
 * recolouring, streaming) on the handle's stream; does not wait.  ESTATE
 * before the first init_fields / set_state. */
int lbm3_step(lbm3_t *h, int64_t n);

/* Blocking.  Computes the observables of the current state into *out (may be
 * NULL) and, when non-NULL, copies the densities rho_k (host [3][ny][nx]) and
 * the post-streaming populations (host [3][9][ny][nx], converted to FP64).
 * Returns LBM3_ENONFINITE (after filling *out) when the state is not finite. */
int lbm3_observables(lbm3_t *h, lbm3_obs *out, double *rho_out, double *f_out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the observables of
 * lbm3_observables into *out (may be NULL), with the same kernels and the same
 * result bit for bit, but no densities or populations, and no allocation of any
 * kind.  Its per-workgroup partial sums live in a static device array of the
 * library (about 2 MiB, one per GPU, held until the process ends; its address is
 * looked up when the first handle on a GPU is created), which limits the launch
 * plan to 32768 workgroups (EINVAL beyond, before any device work).  Calls on one
 * GPU share that array: calls that overlap in time on one GPU (other threads or
 * other streams) race and must be serialised by the caller.  Blocking; ESTATE
 * before the first init_fields / set_state; ENONFINITE as lbm3_observables. */
int lbm3_observables_noalloc(lbm3_t *h, lbm3_obs *out);

/* Releases the handle and its device memory.  NULL is accepted. */
int lbm3_destroy(lbm3_t *h);

/* Message of the last failing call on this thread ("" if none). */
const char *lbm3_last_error(void);

/* Host-side constants the step uses for *p (validated as in lbm3_create):
 * X[p] of Eq. (18) (= cos(phi_kl) of Eq. 14) and the segregation constants
 * g[p] of p->beta_law (g(X) of Eq. 20 for the paper's law) for the pairs
 * (rg, rb, gb), and nu[k] = (tau_k - 1/2)/3.  Any output pointer may be NULL.
 * No device work. */
int lbm3_derived(const lbm3_params *p, double X[3], double g[3], double nu[3]);

/* Launch shape of the fused step's row march: threads per workgroup (64, 128,
 * 256 or 512; each workgroup owns a strip of at most threads-6 columns) and rows
 * marched per workgroup (>= 1; 0 = chosen so that the number of workgroups fits
 * the device's resident slots).  Setting a shape keeps one-step launches on the
 * march (a lattice of at most 2^20 nodes otherwise takes them on blocks, see
 * lbm3_set_steps_per_launch).  Results do not depend on the shape (bitwise).
 * get_tile returns the march's shape, with the rows actually used. */
int lbm3_set_tile(lbm3_t *h, int32_t threads, int32_t rows);
int lbm3_get_tile(const lbm3_t *h, int32_t *threads, int32_t *rows);

/* How many steps one launch advances in lbm3_step: 0 = chosen by size (two on
 * lattices of 2^19 nodes or more in FP64, of more than 2^20 in FP32 and FP32
 * storage), 1 = one, 2 = two where possible.  A two-step launch keeps the
 * intermediate state on chip (in every precision; the first step of a state loaded
 * in 27-population form runs alone) and needs a tile width (lbm3_set_tile's
 * threads) of at most 256; otherwise, and for the odd last step, a one-step launch
 * runs.  One-step launches on lattices of at most 2^20 nodes take two-dimensional
 * blocks of 28 x 12 nodes (no row march) unless lbm3_set_tile chose a shape.
 * Results do not depend on the mode or the kernel (bitwise).  EINVAL for another
 * mode. */
int lbm3_set_steps_per_launch(lbm3_t *h, int32_t mode);
/* The launch lbm3_step uses for pairs of steps: *steps = 2 with its threads per
 * workgroup and workgroup count, or *steps = 1 (and zeros) when pairs run as two
 * one-step launches.  An FP64 or FP32-storage two-step workgroup runs each step on
 * its own waves, so its threads are twice its strip width basis; FP32 uses one
 * thread per column for both steps.  Any pointer may be NULL. */
int lbm3_get_pair_launch(const lbm3_t *h, int32_t *steps, int32_t *threads, int32_t *workgroups);

/* Device pointer of the buffer that holds the current state, its element size in
 * bytes, its strides in elements and its number of planes: plane q of node (x, y)
 * is element q*plane_stride + y*row_pitch + x.  After init_fields / set_state
 * the state is the 27 populations after collision and recolouring, before
 * streaming (q = k*9 + i, nplanes = 27).  After lbm3_step (any precision) it is
 * held factored per node, nplanes = 16: f_dag_i after collision (q = i),
 * c_k = rho_k/rho (q = 9 + k) and V_k = sum_{l != k} beta_kl (rho_k rho_l / rho)
 * n_kl for k = 0, 1 (q = 12 + 2k, 13 + 2k; V_2 = -(V_0 + V_1) since the three sum
 * to zero), from which Eq. (13) gives every recoloured population as
 * c_k f_dag_i + w_i V_k . e_i.  With LBM3_FP32_STORAGE each stored value is the
 * stochastic rounding of its FP64 value.  For measurement tools; the layout is
 * not a stable API. */
int lbm3_state_buffer(const lbm3_t *h, void **dev_ptr, int32_t *elem_bytes, int64_t *plane_stride,
                      int64_t *row_pitch, int32_t *nplanes);

/* ---- batched form: many independent lattices advanced together ---------------
 * The same step (Sec. 2) on count independent periodic lattices, each with its own
 * parameters and size, all of one precision, held in one device arena.
 *
 * lbm3_batch_create: p[0..count-1] as for lbm3_create (each validated; mixed
 *   precisions or forcings give EINVAL; segregation laws may differ between
 *   instances).  hip_stream as for lbm3_create; NULL makes the batch
 *   create and own a stream (graph capture needs one).  *out is NULL on failure.
 * lbm3_batch_init_fields: instance idx (0..count-1) from host rho [3][ny][nx] and
 *   u [2][ny][nx] or NULL, as lbm3_init_fields.  Blocking.  May be called again
 *   for one instance after the batch has stepped; the others keep their state.
 * lbm3_batch_step: advances every instance by n >= 0 steps, no host sync.  Every
 *   launch covers the tiles of all instances; each run of 20 steps replays a
 *   captured hipGraph.  ESTATE while an instance is uninitialised.
 * lbm3_batch_observables: blocking; observables of instance idx into *out (may be
 *   NULL) and its densities into rho_out (host [3][ny][nx], or NULL), as
 *   lbm3_observables.
 * lbm3_batch_set_tile: size_class_side = 0 sets threads per workgroup for the
 *   whole batch (and, with rows > 0, rows for every size class); a side > 0 sets
 *   the rows of the instances with nx == side (threads must equal the batch's).
 *   Threads set this way are also the two-step launch's width (at most 256);
 *   otherwise that width is 128, or 256 when an instance is 768 or more wide.
 *   Results do not depend on the shape.
 * lbm3_batch_set_steps_per_launch: as lbm3_set_steps_per_launch, for the whole
 *   batch (0 = two when the instances hold 2^20 nodes or more in all); the
 *   two-step launch covers every instance once all hold the factored state.
 *   Results do not depend on the mode (bitwise).  EINVAL for another mode.
 * lbm3_batch_get_pair_launch: *steps = 2 with the two-step launch's threads per
 *   workgroup, rows per segment and workgroup count, or *steps = 1 (and zeros)
 *   when pairs run as two one-step launches.  Any pointer may be NULL.
 * lbm3_batch_destroy: releases everything; NULL is accepted. */
int lbm3_batch_create(const lbm3_params *p, int32_t count, void *hip_stream, lbm3_batch_t **out);
int lbm3_batch_init_fields(lbm3_batch_t *b, int32_t idx, const double *rho, const double *u);
int lbm3_batch_step(lbm3_batch_t *b, int64_t n);
int lbm3_batch_observables(lbm3_batch_t *b, int32_t idx, lbm3_obs *out, double *rho_out);
int lbm3_batch_set_tile(lbm3_batch_t *b, int32_t size_class_side, int32_t threads, int32_t rows);
int lbm3_batch_set_steps_per_launch(lbm3_batch_t *b, int32_t mode);
int lbm3_batch_get_pair_launch(const lbm3_batch_t *b, int32_t *steps, int32_t *threads, int32_t *rows,
                               int32_t *workgroups);
int lbm3_batch_destroy(lbm3_batch_t *b);

/* ---- adjoint (reverse-mode derivative) of the FP64 step ----------------------
 * lbm3_adjoint_record: from the state set by lbm3_init_fields(rho, NULL) at step 0
 *   (else ESTATE), advances the FP64 state by nsteps (as lbm3_step) and keeps a
 *   checkpoint of the state every ckpt_every steps in device memory (nsteps >= 1
 *   a multiple of ckpt_every >= 1, else EINVAL).  LBM3_EUNSUPPORTED unless the
 *   handle is LBM3_FP64 with the paper's segregation law and forcing
 *   (LBM3_BETA_PAPER, LBM3_FORCING_GUO).
 * lbm3_adjoint: given drho1_T = dL/drho_1(x, T) (host [ny][nx], finite) for the
 *   state at the end of the last recording, returns dL/dsigma in dsigma[3] (order
 *   rg, rb, gb; may be NULL) and dL/drho_k(x, 0) in drho0 (host [3][ny][nx] for
 *   the densities given to init_fields; may be NULL).  It runs a hand-written
 *   reverse sweep over the step (recolouring of Eq. 13 with Eqs. 19-20, collision
 *   with Guo forcing of Eqs. 8-9, the force of Eq. 7, the colour gradient of
 *   Eq. 12, streaming), recomputing each segment from its checkpoint.  Blocking;
 *   allocates a workspace of about 20 ckpt_every + 100 doubles per node (the
 *   checkpoints hold 18 per node each); below 2^22 nodes, where device memory
 *   allows (lbm3_adjoint_pipeline_slots), the tape and forward buffers are held
 *   twice, since the recompute of the next segment then runs on a second stream
 *   beside the reverse steps of the current one.  The reverse steps run on
 *   two-dimensional blocks where the forward's one-step launches do (at most 2^20
 *   nodes, no shape set by lbm3_set_tile, steps-per-launch mode other than 2), else
 *   on the row march; the result does not depend on which.  The
 *   forward state is left at step T.  ESTATE without a recording or after a step
 *   since it. */
int lbm3_adjoint_record(lbm3_t *h, int64_t nsteps, int32_t ckpt_every);
int lbm3_adjoint(lbm3_t *h, const double *drho1_T, double dsigma[3], double *drho0);
/* The pipeline choice of lbm3_adjoint, a pure host function (no device work): 2 slots
 * (recompute beside the reverse steps) when nodes < 2^22 and the two-slot workspace
 * ws_two_slots fits in the workspace already held plus device_free (less 1/16 in
 * reserve), else 1.  lbm3_adjoint also falls back to one slot when the two-slot
 * allocation fails.  Sizes in bytes. */
int lbm3_adjoint_pipeline_slots(int64_t nodes, uint64_t ws_two_slots, uint64_t ws_held,
                                uint64_t device_free);

/* ---- three-dimensional form (D3Q19, D3Q27) --------------------------------------
 * The step of Sec. 2 (the model is stated for DmQn lattices) on the standard D3Q19
 * lattice (c_s^2 = 1/3; w_0 = 1/3, w = 1/18 on the axis links, 1/36 on the edge links) or
 * the standard D3Q27 lattice (c_s^2 = 1/3; w_0 = 8/27, 2/27 on the axis links, 1/54 on the
 * edge links, 1/216 on the corner links): Eq. (12) as the gradient and the force
 * divergence, the stress pair sum of Eq. (7) as a 3 x 3 tensor, Guo's term and the
 * velocity of Eqs. (8)-(9), the equilibrium of Eq. (3), the recolouring of Eq. (13) with
 * any segregation law (beta_law), streaming of Eq. (22); periodic in x, y and z.  Any
 * precision (FP32 storage: each stored population the stochastic rounding of its FP64
 * value); the paper's forcing only (else LBM3_EUNSUPPORTED).  Q below is the lattice's
 * number of links, 19 or 27.
 * lbm3d_create_lattice: p as for lbm3_create (nx, ny from it), nz in 1..65535, q = 19 or
 *   27, at most 2^29 nodes (else LBM3_EINVAL); allocates the two 3Q-population state
 *   buffers (in the storage type) and a staging buffer for exports (3Q + 3 doubles per
 *   node).
 * lbm3d_create: lbm3d_create_lattice with q = 19.
 * lbm3d_init_fields: rho host [3][nz][ny][nx] (x fastest), finite, >= 0, with rho > 0 at
 *   every node; fluid at rest (f_{i,k} = w_i rho_k).  Blocking; resets the step count.
 * lbm3d_step: enqueues n >= 0 steps on the handle's stream (one launch each).
 * lbm3d_observables: blocking; masses, momentum sum rho u (Eq. 9 velocity), kinetic
 *   energy, max |u|, and when non-NULL the densities (host [3][nz][ny][nx]) and the
 *   post-streaming populations (host [3][Q][nz][ny][nx], links in the order: rest,
 *   +-x, +-y, +-z, then (+1,+1,0), (-1,-1,0), (+1,-1,0), (-1,+1,0), (+1,0,+1), (-1,0,-1),
 *   (+1,0,-1), (-1,0,+1), (0,+1,+1), (0,-1,-1), (0,+1,-1), (0,-1,+1), and for D3Q27 then
 *   (+1,+1,+1), (-1,-1,-1), (+1,+1,-1), (-1,-1,+1), (+1,-1,+1), (-1,+1,-1), (-1,+1,+1),
 *   (+1,-1,-1)).  ENONFINITE when the state is not finite.
 * lbm3d_destroy: releases everything; NULL is accepted. */
typedef struct lbm3d lbm3d_t;
typedef struct {
    int64_t step;
    double mass[3];
    double momentum[3];
    double kinetic_energy;
    double u_max;
    int32_t nonfinite;
} lbm3d_obs;
int lbm3d_create_lattice(const lbm3_params *p, int32_t nz, int32_t q, void *hip_stream, lbm3d_t **out);
int lbm3d_create(const lbm3_params *p, int32_t nz, void *hip_stream, lbm3d_t **out);
int lbm3d_init_fields(lbm3d_t *h, const double *rho);
int lbm3d_step(lbm3d_t *h, int64_t n);
int lbm3d_observables(lbm3d_t *h, lbm3d_obs *out, double *rho_out, double *f_out);
int lbm3d_destroy(lbm3d_t *h);

/* Plain device copy of nbytes (a multiple of 16) from device src to device dst on
 * hip_stream (NULL = null stream), no host sync: the bandwidth reference the
 * roofline figures are compared with.  EINVAL for NULL pointers or a bad size. */
int lbm3_device_copy(void *dst, const void *src, int64_t nbytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM3_H */
