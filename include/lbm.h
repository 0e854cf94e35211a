/*
 * lbm.h -- C ABI of the MI355X (gfx950) implementation of the fused time step of
 * the REV-scale double-distribution-function MRT lattice Boltzmann model of
 * Liu & He, "Three-dimensional multiple-relaxation-time lattice Boltzmann
 * model for convection heat transfer in porous media at the REV scale"
 * (arXiv:1611.03329).
 *
 * One lattice = one box of nx*ny*nz fluid nodes carrying
 *   - density populations f_i, D3Q19 (Sec. 3.1.2) or D3Q15 (Sec. 3.1.1), and
 *   - temperature populations g_k, D3Q7 (Sec. 3.2).
 * One time step, for every node, fuses (all on the GPU):
 *   streaming of f (Eq. 10) and g (Eq. 35) with the wall rules below;
 *   rho (Eq. 25), sigma*T (Eq. 39), buoyancy G (Eq. 5), the explicit velocity
 *   closure (Eqs. 27-28), the porous total force F (Eq. 4);
 *   the flow collision in moment space (Eq. 9) with the porosity-dependent
 *   equilibria (Eq. 21 / 15), the forcing moments (Eq. 23 / 17) and the
 *   relaxation rates (Eq. 22 / 16);
 *   the temperature collision in moment space (Eq. 34) with Eqs. 36-38, 43.
 *
 * Conventions
 *   - lattice units rho0 = dt = dx = c = 1 (Sec. 4), cs^2 = 1/3, csT^2 = varpi/3;
 *   - node (x,y,z), x fastest; linear index n = x + nx*(y + ny*z);
 *   - non-periodic faces are halfway walls at -1/2 and n-1/2 (L = n along
 *     length_axis, K = Da*L^2);
 *   - time t counts completed steps; the state at time t is the pre-collision
 *     populations f(t), g(t); fields, Nusselt numbers and totals at time t
 *     are computed from that state;
 *   - walls: halfway bounce-back for f (plus 2 w_i rho0 e_i.u_w / cs^2 for a
 *     moving wall), anti-bounce-back for an isothermal g
 *     (g_k = -g*_kbar + 2 omega_k sigma T_w), bounce-back for an adiabatic g.
 *     (The paper used non-equilibrium extrapolation, Sec. 4; these wall rules
 *     are a deliberate substitution.)  A link leaving through two wall faces
 *     takes the wall velocity of the first of them in face order.
 *
 * Threading and streams: a lattice is not thread-safe; all of its device work
 * is enqueued on the HIP stream given at creation (or lbm_set_stream).
 * Functions documented as "asynchronous" return after enqueueing; functions
 * that return host values synchronize that stream.
 *
 * Caller buffers of fields and states (lbm_fields, lbm_get_state,
 * lbm_set_state, lbm_enthalpy_fields) may be device memory of the lattice's
 * device (the device current at lbm_create; managed memory counts as device
 * memory) or host memory, pinned or pageable.  Each pointer is classified with
 * hipPointerGetAttributes before any launch: device buffers are read or
 * written by the kernels directly and the call stays asynchronous; host
 * buffers go through a device staging buffer the call allocates and frees,
 * with a stream-ordered copy, and the call then synchronizes the lattice's
 * stream before it returns.  Memory of another device, or of a kind that is
 * neither, gives LBM_ERR_INVALID_ARG with nothing enqueued.
 *
 * Errors: every function returns an lbm_status; LBM_OK is 0.  On an error the
 * lattice is unchanged unless stated; lbm_last_error() returns a thread-local
 * message describing the last failure on the calling thread.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_lattice lbm_lattice; /* opaque */
typedef struct lbm_batch lbm_batch;     /* opaque */

typedef enum { LBM_ENERGY_TEMPERATURE = 0, LBM_ENERGY_ENTHALPY = 1 } lbm_energy;

typedef enum {
  LBM_OK = 0,
  LBM_ERR_INVALID_ARG = 1,   /* bad parameter, size or pointer */
  LBM_ERR_OUT_OF_MEMORY = 2, /* device allocation failed or caller buffer too small */
  LBM_ERR_DEVICE = 3,        /* a HIP call failed */
  LBM_ERR_UNSTABLE = 4,      /* a check found a non-finite value or |u| > 0.5 (sticky) */
  LBM_ERR_UNSUPPORTED = 5    /* valid request that is not implemented */
} lbm_status;

typedef enum {
  LBM_FP64 = 0,        /* populations stored and computed in FP64 */
  LBM_FP32 = 1,        /* populations stored and computed in FP32 */
  LBM_FP16_STORAGE = 2 /* flow populations (the rest one too) stored in FP16; temperature
                          populations in FP32; arithmetic in FP32.  The FP16 stores round
                          stochastically (zero-mean error) with random bits hashed from the
                          lattice's step count, node and population: reproducible runs */
} lbm_precision;       /* in every mode populations are stored shifted by their rest state */

/* Face rules.  WALL: halfway bounce-back (u_wall: moving wall; a wall velocity
 * with a normal component makes the face an inlet).  OUTLET: open boundary at
 * rho0: the entering population is the anti-bounce-back of the leaving one to
 * twice the even part of f^eq(rho0, u), u the node's own velocity when it
 * collided.  For g, OUTFLOW is the anti-bounce-back to the node's own
 * temperature.  A link that leaves through a wall face and an open face takes
 * the wall rule. */
typedef enum { LBM_FLOW_PERIODIC = 0, LBM_FLOW_WALL = 1, LBM_FLOW_OUTLET = 3 } lbm_flow_bc;
typedef enum {
  LBM_HEAT_PERIODIC = 0,
  LBM_HEAT_ADIABATIC = 1,
  LBM_HEAT_ISOTHERMAL = 2,
  LBM_HEAT_OUTFLOW = 3
} lbm_heat_bc;

/* One face of the box.  Face order: 0 = -x, 1 = +x, 2 = -y, 3 = +y, 4 = -z, 5 = +z.
 * Opposite faces are both periodic (flow and heat) or both not. */
typedef struct {
  int32_t flow;      /* lbm_flow_bc */
  int32_t heat;      /* lbm_heat_bc */
  double T_wall;     /* isothermal wall temperature */
  double u_wall[3];  /* wall velocity of a WALL face (moving-wall bounce-back) */
} lbm_face;

/* Lattice description.  Fill with lbm_default_params() first (Sec. 4 defaults:
 * sigma = J = Gamma = 1, varpi = 1/2, s_rho = s_j = 1, s_e = s_eps = s_q = s_pi = 1.1,
 * s_m = 1.2, zeta_T = 1, zeta_e = zeta_nu = 1.2, Ma = 0.1). */
typedef struct {
  int32_t nx, ny, nz;     /* fluid nodes per axis, >= 1 */
  int32_t lattice;        /* 19 (D3Q19) or 15 (D3Q15) */
  int32_t precision;      /* lbm_precision */
  double porosity;        /* phi in (0,1] (Eqs. 2, 4) */
  double darcy;           /* Da = K/L^2 > 0 (Eq. 7) */
  double rayleigh;        /* Ra >= 0 (Eq. 7); sets g*beta = Ra nu alpha / (L^3 delta_T) */
  double prandtl;         /* Pr = nu/alpha > 0 (Eq. 7) */
  double reynolds;        /* > 0 selects the channel mapping of Eq. 51: nu = u_char L / Re */
  double u_char;          /* characteristic speed of the channel mapping */
  double mach;            /* Ma of the cavity mapping (Eq. 56) */
  double forchheimer;     /* multiplier of F_phi of Eq. 6 (1: generalized non-Darcy, 0: Brinkman) */
  double sigma, J, Gamma, varpi;  /* Eqs. 3, 7, 37 */
  double s_rho, s_e, s_eps, s_j, s_q, s_pi, s_m; /* Eqs. 16, 22 (s_pi unused by D3Q15) */
  double zeta_T, zeta_e, zeta_nu;                /* Eq. 38 */
  double s_nu_set;        /* > 0: use as s_nu instead of Eq. 56 / 51 */
  double zeta_alpha_set;  /* > 0: use as zeta_alpha instead of Eq. 56 / 51 */
  int32_t gravity_axis;   /* buoyancy acts along +axis: G_axis += g*beta*(T - T_ref) (Eq. 5) */
  int32_t length_axis;    /* L = node count along this axis */
  double T_ref;           /* T0 of Eq. 5; also the storage shift of g */
  double delta_T;         /* temperature scale of Ra and of the Nusselt numbers, > 0 */
  double accel[3];        /* constant external acceleration a of Eq. 5 */
  lbm_face face[6];
  int32_t init_axis;      /* initial T: -1 uniform T_ref, else linear along this axis ... */
  double init_T_lo;       /* ... from init_T_lo at the -1/2 face to init_T_hi at n-1/2 ... */
  double init_T_hi;
  uint64_t seed;          /* ... plus noise_amp*(2r-1), r = (SplitMix64(seed ^ n) >> 11) * 2^-53 */
  double noise_amp;
  int32_t check_interval; /* K > 0: residual check at every multiple of K steps; 0 disables */
  double init_u[3];       /* initial velocity: f = f^eq(rho0, init_u), g = g^eq(T, init_u) */
  /* ---- energy equation: LBM_ENERGY_TEMPERATURE (Sec. 3.2, default) or LBM_ENERGY_ENTHALPY
   * (App. B: effective enthalpy with solid-liquid phase change, Eqs. B4-B13).  An enthalpy
   * lattice carries only the D3Q7 populations and no flow (u = 0, the setting of the melting
   * test of Sec. 4.3); it takes FP64 or FP32, periodic / adiabatic / isothermal faces,
   * varpi, porosity, zeta_e, zeta_nu and the fields below, and check_interval 0. */
  int32_t energy;
  double c_pl, c_ps;      /* specific heats of the liquid and the solid (Eq. B2), > 0 */
  double matrix_heat;     /* rho_m c_pm / (rho_l c_pl) of the porous matrix (Eq. B4), >= 0 */
  double latent;          /* L_a >= 0 */
  double T_solidus, T_liquidus;  /* T_s <= T_l (Eq. B8) */
  double alpha_l, alpha_s;       /* effective diffusivity of each phase (Eq. B11), > 0 */
  double T_init;          /* uniform initial temperature (g = g^eq of Eq. B12 at u = 0) */
} lbm_params;

/* Derived quantities (Eqs. 6, 7, 28, 32, 41, 51, 56). */
typedef struct {
  double L, s_nu, zeta_alpha, nu_e, nu, alpha_e, alpha, K, F_phi, gbeta, l0, l1;
} lbm_derived;

/* Fills *p with the defaults above and an 8^3 D3Q19 FP64 box with all six faces
 * adiabatic no-slip walls.  Never fails for non-NULL p. */
void lbm_default_params(lbm_params* p);

/* Device bytes a lattice with these parameters needs (state, check snapshot,
 * reduction scratch).  Returns LBM_ERR_INVALID_ARG / LBM_ERR_UNSUPPORTED for
 * parameters lbm_create would reject; *bytes is 0 then. */
lbm_status lbm_required_bytes(const lbm_params* p, size_t* bytes);

/* Creates a lattice and enqueues its initialisation (f = f^eq(rho0, init_u) of
 * Eq. 24/18, g = g^eq(T_init, init_u) of Eq. 42) on `stream` (a hipStream_t; NULL = null stream).
 * dev_buf: caller-owned device memory of the current device, at least
 * lbm_required_bytes() bytes, 256-byte aligned, kept alive until lbm_destroy;
 * or NULL, in which case the library allocates (and later frees) it.  Host
 * memory or memory of another device is refused (LBM_ERR_INVALID_ARG).
 * Parameters are validated before any allocation or device work.  The
 * lattice lives on the current device; call it with that device current. */
lbm_status lbm_create(const lbm_params* p, void* dev_buf, size_t bytes, void* stream,
                      lbm_lattice** out);

/* Waits for the lattice's stream, frees what the library allocated (never the
 * caller's buffer) and the handle.  NULL is accepted. */
lbm_status lbm_destroy(lbm_lattice* h);

/* Changes the stream later calls enqueue on. The caller orders the two streams
 * (a Nusselt reduction started by lbm_nusselt_start is waited for here). */
lbm_status lbm_set_stream(lbm_lattice* h, void* stream);

/* Enqueues nsteps >= 0 fused time steps t -> t + nsteps.  When check_interval
 * K > 0 the steps that start at times n-1 and n (n a positive multiple of K)
 * also compute the residual r(n) (see lbm_residual).  Asynchronous; returns
 * LBM_ERR_UNSTABLE without enqueueing if an earlier check already found the
 * lattice unstable.  That test reads the host copy of the last check's result
 * without waiting for it: a check whose copy is still in flight is seen by the
 * first call after it has landed (at the latest after the next synchronizing
 * call, e.g. lbm_residual), so stepping may continue up to one more call past
 * an unstable check; the values are then meaningless but nothing else is
 * affected. */
lbm_status lbm_step(lbm_lattice* h, int64_t nsteps);

/* Current time t (completed steps).  Host-only, no synchronization. */
lbm_status lbm_time(const lbm_lattice* h, int64_t* t);

lbm_status lbm_derived_params(const lbm_lattice* h, lbm_derived* d);

/* Writes rho (Eq. 25), u (Eqs. 27-28) and T (Eq. 39) at the current time into
 * caller-owned buffers (device or host memory, see "Caller buffers" above) of
 * nx*ny*nz FP64 values each, x fastest.  Any pointer may be NULL to skip that
 * field.  Asynchronous for device buffers; synchronizes when one is host memory. */
lbm_status lbm_fields(lbm_lattice* h, double* rho, double* ux, double* uy, double* uz, double* T);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation): the
 * output of lbm_fields, bit for bit, with no allocation.  Same arguments,
 * layout and NULL rule as lbm_fields.  Device buffers are written directly
 * (asynchronous, as lbm_fields).  Host buffers (pinned or pageable) pass
 * through a staging array the library holds in its own device code object, 16
 * MiB per device, kept until the process ends: the lattice is processed in
 * passes of at most 16 MiB / (8 B x number of host outputs) nodes, each pass's
 * kernel followed by its copies to the host, and the call synchronizes the
 * lattice's stream before it returns.  Any lattice size is accepted: a larger
 * lattice takes more passes.  Calls no hipMalloc, hipFree or other allocating
 * routine.  Every call on a device shares that device's one array: calls that
 * overlap on one device (other threads, other streams) race and must be
 * serialized by the caller.  Errors as lbm_fields (LBM_ERR_INVALID_ARG for
 * memory of another device, LBM_ERR_UNSUPPORTED for an enthalpy lattice). */
lbm_status lbm_fields_noalloc(lbm_lattice* h, double* rho, double* ux, double* uy, double* uz, double* T);

/* Face Nusselt numbers at the current time, FP64, into host nu[6]: for every
 * isothermal face, the mean over the face's nodes of the heat that entered the
 * fluid through it during the last streaming (2 g_k - 2 omega_k sigma T_w for
 * the incoming population k of anti-bounce-back, with the wall term 2 omega_k
 * sigma T_w in the lattice's arithmetic precision, as the step applies it),
 * times L/(alpha_e delta_T): the midpoint rule for Nu_3D of Eqs. 53-55.  0 for
 * other faces.  The hot wall of a cavity reports +Nu, the cold wall -Nu.
 * Synchronizes.  After lbm_nusselt_start it collects the reduction that call
 * started instead of starting one. */
lbm_status lbm_nusselt(lbm_lattice* h, double nu[6]);

/* Starts the reduction of lbm_nusselt on the lattice's stream for the state at
 * the current time and returns without waiting; the next lbm_nusselt on the
 * lattice collects it (Eqs. 53-55, as lbm_nusselt), whatever was enqueued on
 * the stream in between.  Lets a caller that retires several lattices sharing
 * a stream start all their reductions and synchronize once.  A second start
 * before the collection replaces the first.  LBM_ERR_UNSUPPORTED for an
 * enthalpy lattice. */
lbm_status lbm_nusselt_start(lbm_lattice* h);

/* Most recent residual check: r(n) = max(|u(n) - u(n-1)|_2 / |u(n)|_2,
 * |theta(n) - theta(n-1)|_2 / |theta(n)|_2), theta = (T - T_ref)/delta_T + 1/2,
 * sums over all nodes in FP64 (a term whose denominator is 0 counts as 0 if
 * its numerator is 0).  *at_step = n, or -1 (and *r = -1) if no check has run.
 * Returns LBM_ERR_UNSTABLE if the check found the lattice unstable.
 * Synchronizes. */
lbm_status lbm_residual(lbm_lattice* h, double* r, int64_t* at_step);

/* Sum over nodes of rho and of sigma*T at the current time, FP64 (two-pass,
 * deterministic).  Synchronizes. */
lbm_status lbm_totals(lbm_lattice* h, double* mass, double* heat);

/* Copies the pre-collision state at the current time into caller-owned buffers
 * (device or host memory), FP64, layout [q][z][y][x] for f (q = 19 or 15) and
 * [7][z][y][x] for g.  Either pointer may be NULL.  Asynchronous for device
 * buffers; synchronizes when one is host memory. */
lbm_status lbm_get_state(lbm_lattice* h, double* f, double* g);

/* Replaces the state with caller-given FP64 arrays in device or host memory
 * (same layout as lbm_get_state; both required), rounding to the storage
 * precision.  The time counter is kept; the pending residual snapshot is
 * discarded.  Asynchronous for device arrays (keep them unchanged until the
 * stream has passed the copy); synchronizes when one is host memory. */
lbm_status lbm_set_state(lbm_lattice* h, const double* f, const double* g);

/* Enthalpy lattices (energy = LBM_ENERGY_ENTHALPY): temperature (Eq. B8), effective
 * enthalpy (Eq. B7) and liquid fraction (Eq. B9) at the current time into
 * caller-owned buffers (device or host memory) of nx*ny*nz FP64 values, x
 * fastest; any pointer may be NULL.  The heat capacity ratios of Eq. B4 are sigma_l = phi + (1 - phi)
 * matrix_heat and sigma_s = phi c_ps / c_pl + (1 - phi) matrix_heat, c_p,ref is
 * the harmonic mean of c_pl and c_ps (Eq. B13) and the liquidus enthalpy is
 * sigma_l c_pl T_l + phi L_a.  Walls: anti-bounce-back at T_w with the weight
 * varpi c_p,ref / 6 of Eq. B12, bounce-back at adiabatic walls.  Asynchronous
 * for device buffers; synchronizes when one is host memory.
 * LBM_ERR_UNSUPPORTED for a temperature lattice; conversely lbm_fields,
 * lbm_nusselt, lbm_totals, lbm_transfer_state and batches refuse enthalpy
 * lattices, and their lbm_get_state / lbm_set_state take f = NULL. */
lbm_status lbm_enthalpy_fields(lbm_lattice* h, double* T, double* En, double* fl);

/* Copies the current pre-collision state of src into dst, converting the
 * storage precision (e.g. an FP16-storage lattice into an FP32 one).  Both must
 * have the same lattice type, shape and rest state (varpi, sigma, T_ref); the
 * physical parameters may differ.  dst keeps its time counter; its pending
 * residual snapshot is discarded; dst must not be in a batch.  Waits for src's
 * stream if it differs from dst's, then enqueues on dst's stream. */
lbm_status lbm_transfer_state(lbm_lattice* dst, lbm_lattice* src);

/* ---------------------------------------------------------------- batches
 * A batch advances many independent lattices (members) by the same fused time
 * step of lbm_step, one kernel launch per step for a whole group of members
 * (groups: see lbm_batch_set_launch; by default one group, or two when some
 * members have moving walls or open faces and others not).  A member's
 * state after any number of steps is bit for bit the one lbm_step gives it,
 * and its residuals depend on nothing else in the batch (they are summed in a
 * fixed order set by the member's size and the block size alone).
 * Members share lattice type, precision and stream (the batch's), and the time
 * parity; lbm_batch_add takes one lbm_step of the joining lattice when its
 * parity differs.  The residual check (lbm_residual) follows the batch's own
 * step counter s: with check interval K > 0 the steps s = mK-1 and s = mK of
 * the batch compute every member's r at its own time; a member's first check
 * comes at the first such pair after it joined.  While in a batch a lattice
 * may be queried (lbm_fields, lbm_nusselt, lbm_residual, lbm_totals,
 * lbm_get_state) but not stepped, given a state or a stream of its own; the
 * queries enqueue on the batch's stream.  lbm_destroy of a member removes it
 * first.  A batch is not thread-safe. */

/* Creates an empty batch that enqueues on `stream` (hipStream_t; NULL = null
 * stream) and checks residuals every check_interval >= 0 batch steps.
 * Allocates no device memory yet. */
lbm_status lbm_batch_create(void* stream, int32_t check_interval, lbm_batch** out);

/* Waits for the batch's stream, leaves every member a plain lattice (its last
 * batch residual kept) and frees the batch.  NULL is accepted. */
lbm_status lbm_batch_destroy(lbm_batch* b);

/* Adds lattice h (not in a batch).  Returns LBM_ERR_UNSUPPORTED if its lattice
 * type or precision differs from the members'.  Synchronizes h's old stream if
 * it differs from the batch's.  May enqueue one step of h. */
lbm_status lbm_batch_add(lbm_batch* b, lbm_lattice* h);

/* Removes member h (a plain lattice again, on the batch's stream, with its
 * time and its last batch residual).  Synchronizes. */
lbm_status lbm_batch_remove(lbm_batch* b, lbm_lattice* h);

/* Number of members; member `index` in join order (removals close the gap). */
lbm_status lbm_batch_size(const lbm_batch* b, int32_t* count);
lbm_status lbm_batch_member(const lbm_batch* b, int32_t index, lbm_lattice** out);

/* Enqueues nsteps >= 0 steps of every member.  An unstable member keeps being
 * stepped (its values are then meaningless) until the caller removes it; the
 * others are unaffected.  Asynchronous, except that the first step after a
 * change of membership or launch shape, or after a member's first snapshot,
 * synchronizes once to upload the member table. */
lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps);

/* Per member, in join order, into host arrays of `count` (= the member count)
 * entries, any of them NULL to skip: the most recent residual r (-1 if none),
 * the member time it was taken at (-1), and 1 if that check found the member
 * unstable.  Synchronizes. */
lbm_status lbm_batch_residuals(lbm_batch* b, double* r, int64_t* at_step, int32_t* unstable, int32_t count);

/* Launch shape of a batch. */
typedef struct {
  int32_t block;          /* threads per tile: 64, 128 or 256 (default 256) */
  int32_t blocks_per_cu;  /* > 0: persistent grid of this many blocks per compute unit (at most
                             the tile count) whose blocks walk the tile list; 0 (default): one
                             block per tile */
  uint64_t group_bytes;   /* group size limit (0, the default: one group per wall-rule set) */
  int32_t xcd_ranges;     /* > 1: the tile list of a launch is cut into this many contiguous
                             ranges, range r taken by the blocks the hardware places on XCD r
                             (8 on MI355X), so neighbouring tiles share an L2; 0 (default):
                             hardware order */
} lbm_launch;

/* Sets the launch shape.  Whole check intervals run group by group, so a
 * group whose populations fit the last-level cache is streamed from there.
 * Results do not depend on the launch shape except through the residual's
 * summation order, which follows `block`. */
lbm_status lbm_batch_set_launch(lbm_batch* b, int32_t block, int32_t blocks_per_cu, uint64_t group_bytes,
                                int32_t xcd_ranges);

/* Chooses the launch shape by timing whole check intervals (HIP events, graph
 * replay off meanwhile): group_bytes in {0, 8, 16, 32, 64, 128, 256, 512} MiB
 * together with xcd_ranges in {0, 8}, then block in {64, 128, 256}, then
 * blocks_per_cu in {0, 4, 8}, one at a time, then the threads per tile of
 * each size class present (lbm_batch_set_class_block), one class at a time;
 * each candidate runs one untimed and three timed intervals and is scored by
 * their median, and replaces the incumbent only when its median is more than
 * 1 % lower (choices inside the timing noise keep the earlier shape); the
 * batch first steps to the start of an interval.
 * Writes the batch-wide choice to *out if non-NULL and keeps it with the
 * per-class ones (lbm_batch_class_block reads them).  The steps advance the
 * members.  Synchronizes. */
lbm_status lbm_batch_autotune(lbm_batch* b, lbm_launch* out);

/* Threads per tile (64, 128 or 256; 0: the batch's `block` of
 * lbm_batch_set_launch) for members of size class `size_class` in [0, 31]:
 * those of 2^size_class to 2^(size_class + 1) - 1 nodes.  Members whose
 * threads per tile differ launch in separate groups.  A member's state does not
 * depend on it; its residual's summation order does. */
lbm_status lbm_batch_set_class_block(lbm_batch* b, int32_t size_class, int32_t block);

/* Threads per tile the members of size class `size_class` take. */
lbm_status lbm_batch_class_block(const lbm_batch* b, int32_t size_class, int32_t* block);

/* on != 0: the residual of a check compares with the state of K steps before
 * (r = max(|u(n) - u(n-K)|_2 / |u(n)|_2, |theta(n) - theta(n-K)|_2 /
 * |theta(n)|_2)) instead of one step before; one step per interval then both
 * compares and snapshots (steps s % K == 0).  The change over K steps stands
 * out from rounding noise of the stored populations (FP16 storage) K times
 * better than the one-step change.  Only at the start of a check interval;
 * every member's next check is then its first. */
lbm_status lbm_batch_set_span(lbm_batch* b, int32_t on);

/* on != 0: whole check intervals (the K steps from a batch step s with
 * s % K == 0) are recorded once into a HIP graph and replayed; the graph is
 * recorded again when the member table outgrows its buffers or the member
 * count or launch shape changes.  Needs K > 0 and a created stream
 * (capture is impossible on the null stream): LBM_ERR_UNSUPPORTED otherwise. */
lbm_status lbm_batch_set_graph(lbm_batch* b, int32_t on);

const char* lbm_status_string(lbm_status s);
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
