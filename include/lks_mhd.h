/*
 * lks_mhd -- fused lattice-kinetic MHD time step for MI355X (gfx950).
 *
 * The method is the one of E. Yahia & K. N. Premnath, "On Boundary Conditions
 * for Lattice Kinetic Schemes for Magnetohydrodynamics Bounded by Walls with
 * Finite Electrical Conductivities" (arXiv 2112.13930):
 *   - D2Q9 BGK flow distribution f with the forcing source of Sec. V
 *     (Lorentz force J x B of Sec. II plus an external body force);
 *   - D2Q5 vector magnetic distribution g of Dellar's lattice kinetic scheme
 *     (Sec. IV), J_z from the non-equilibrium part of its first moment;
 *   - Shercliff thin-conducting-wall closures at the two channel walls
 *     (Sec. III condition): the link-based weighted bounce-back/anti-bounce-
 *     back closure (Sec. VI, moving walls App. B.1) with half-way bounce-back
 *     of f, or the on-node moment-based closure (Sec. VII, App. A, moving
 *     walls App. B.2).
 * The channel is periodic in x and bounded by walls at y = -a (row 0) and
 * y = +a (row ny-1); the imposed field B0 points along +y.
 *
 * Conventions for every entry point:
 *   - Return value: LKS_OK (0) or a negative lks_status; the reason is kept
 *     in a thread-local message returned by lks_mhd_last_error().
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are ordinary process memory.  Field arrays are FP64, row-major
 *     [ny][nx] (x fastest).  Population arrays are FP64 [19][ny][nx] with the
 *     plane order f_0..f_8, g_0x..g_4x, g_0y..g_4y and raw (not shifted)
 *     population values.
 *   - Lattice numbering: D2Q9 e = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),
 *     (-1,1),(-1,-1),(1,-1); D2Q5 e = (0,0),(1,0),(0,1),(-1,0),(0,-1).
 *   - Work is enqueued on the HIP stream given at create time; entry points
 *     documented as synchronous wait for that stream before returning.
 *   - A handle is used by one host thread at a time; separate handles are
 *     independent.  Nothing here allocates device memory except where stated.
 */
#ifndef LKS_MHD_H
#define LKS_MHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LKS_MHD_ABI_VERSION 9

typedef struct lks_mhd lks_mhd_t;             /* one channel, library-owned */
typedef struct lks_mhd_batch lks_mhd_batch_t; /* many channels, library-owned */

enum lks_bc { LKS_BC_LINK = 0, LKS_BC_MOMENT = 1 };

/* Collision operator.
 *   BGK  the paper's single-relaxation-time operators (Secs. IV and V).
 *   TRT  the two-relaxation-time form, one of the multiple-relaxation-time
 *        replacements the paper names (Secs. V and IX).  Each population
 *        splits into its parts even and odd under e -> -e, which relax at
 *        separate rates.  tau_f keeps setting the viscosity (even part of
 *        f) and tau_m the magnetic diffusivity (odd part of g), so the
 *        wall coefficients and the current J_z are unchanged.  The free
 *        rates come from the magic parameters
 *          lambda_f = (tau_f - 1/2)(tau_f_odd - 1/2),
 *          lambda_m = (tau_m_even - 1/2)(tau_m - 1/2).
 *        lambda_f = 3/16 places half-way bounce-back walls exactly for
 *        Poiseuille flow at every tau_f.
 *   MRT  multiple relaxation times: populations map to orthogonal moments,
 *        each of which relaxes at its own rate, the source's moments with
 *        the weight 1 - s/2 of their rate.  f uses the D2Q9 basis of
 *        Lallemand and Luo (Phys. Rev. E 61 (2000) 6546): rho, e, epsilon,
 *        j_x, q_x, j_y, q_y, p_xx, p_xy, with p_xx and p_xy at 1/tau_f
 *        (viscosity) and e, epsilon, q at s_fe, s_feps, s_fq.  Each
 *        component of g uses the D2Q5 basis B, Lambda_x, Lambda_y,
 *        epsilon = (-4, 1, 1, 1, 1) and d = (0, 1, -1, 1, -1) (over the
 *        rest, +x, +y, -x, -y populations), with Lambda at 1/tau_m (magnetic
 *        diffusivity) and epsilon, d at s_me, s_md.  With s_fe = s_feps =
 *        1/tau_f and s_me = s_md it is the TRT operator.  Available
 *        wherever TRT is.  In 3D, f
 *        uses the D3Q19 basis of
 *        d'Humieres et al. (Phil. Trans. R. Soc. A 360 (2002) 437): e at
 *        s_fe, epsilon and the fourth-order pi at s_feps, q and the
 *        third-order m at s_fq, the stresses at 1/tau_f; g (D3Q7, zero rest
 *        weight) relaxes its two traceless second moments at s_md (s_me has
 *        no effect there). */
enum lks_collision { LKS_BGK = 0, LKS_TRT = 1, LKS_MRT = 2 };

/* Storage precision of the populations.
 *   FP64           stored as binary64, computed in FP64, rounded to nearest.
 *   FP32           stored as binary32 and computed in FP64; each stored value
 *                  is rounded stochastically to one of its two binary32
 *                  neighbours.
 *   FP16_STORE     stored as binary16 and computed in FP32 (equilibria,
 *                  sources, the coupled u/J solve, the relaxation), rounded
 *                  stochastically to binary16.  The collision's increments
 *                  have the moments it conserves restored in FP64 (mass and
 *                  B unchanged, momentum + F) and are added to the state in
 *                  FP64, so FP32 rounding leaves no residual that slow modes
 *                  of a steady channel could integrate.  Observables and
 *                  state exchange decode in FP64.
 *   FP16_STORE_F64 stored as binary16 and computed in FP64.
 * Every population is stored as its deviation from the rest state at unit
 * density with B = (0, B0): f_alpha - w_alpha, g_alpha,x and
 * g_alpha,y - W_alpha B0.  Binary16 storage further subtracts a per-row
 * reference R[y][alpha] (FP32 values), zero until a rebase (lks_mhd_rebase)
 * moves each row's mean over x into it, so binary16 then carries only the
 * x-variation and the change since the last rebase, scaled by 2^12.  The
 * random bits of stochastic rounding are a counter-based hash of (step since
 * create or load, node, plane): a run is reproducible bit for bit and does
 * not depend on launch shape or on the other channels of a batch.
 * Steady-state reductions are FP64 in every mode. */
enum lks_precision { LKS_FP64 = 0, LKS_FP32 = 1, LKS_FP16_STORE = 2, LKS_FP16_STORE_F64 = 3 };

enum lks_status {
  LKS_OK = 0,
  LKS_EINVAL = -1,    /* invalid argument or parameter set */
  LKS_ENOMEM = -2,    /* caller buffer or pool too small */
  LKS_EDEVICE = -3,   /* a HIP call failed */
  LKS_EUNSTABLE = -4, /* a non-finite density, velocity or field appeared */
  LKS_ENOTCONV = -5   /* max_steps reached without meeting the tolerance */
};

/*
 * Physical and lattice parameters of one channel (lattice units, dx = dt = 1,
 * mu_m = 1).  Defaults that the helper lks_mhd_default_params() fills are
 * given in brackets.
 *   nx, ny      nodes; x periodic; ny >= 2 (link) or >= 3 (moment);
 *               nx * ny <= (2^31 - 1) / 19 - 8192 (19 padded planes index in 32 bits).
 *   bc          LKS_BC_LINK or LKS_BC_MOMENT.
 *   precision   lks_precision.
 *   tau_f       BGK relaxation time of f, > 1/2: nu = (tau_f - 1/2)/3 (Sec. V).
 *   tau_m       relaxation time of g, > 1/2: eta = (tau_m - 1/2)/3 (Sec. IV).
 *   ha          Hartmann number (Sec. VIII).  If finite and >= 0, the imposed
 *               field is B0 = ha * sqrt(rho0 nu eta) / a, where the half-width
 *               is a = ny/2 for link-based walls (half-way between nodes) and
 *               a = (ny-1)/2 for on-node walls.  NaN: b0 is used as given.
 *   b0          imposed field along +y; must be NaN or equal to the derived
 *               value when ha is given.
 *   c_lower,    wall conductance ratios c_w of Sec. III at y = -a and y = +a,
 *   c_upper     in [0, +INFINITY]; 0 is an insulating wall, INFINITY a
 *               perfectly conducting one.  H = a in theta and 1/(c_w a).
 *   u_lower,    wall velocities along x (App. B).
 *   u_upper
 *   fx, fy      external body force.  fx = NaN derives it from u_max through
 *               the Chang-Lundgren centreline velocity (Sec. VIII), which
 *               needs c_lower == c_upper.
 *   u_max       target centreline velocity when fx is NaN.
 *   rho0        initial density [1]; the state starts at rest at rho0 with
 *               B = (0, B0) (zero induced field).
 *   collision   lks_collision [LKS_BGK].
 *   lambda_f,   TRT magic parameters, finite and > 0 [3/16, 1/4]; ignored
 *   lambda_m    under BGK.
 *   x_walls     0: x periodic (a channel) [0].  1: an enclosure, x bounded by
 *               stationary thin conducting walls half-way outside the
 *               columns x = 0 and x = nx-1 (nx >= 2, link-based closures
 *               only; single channels, not batches), conductance ratios
 *               c_x_lower (x = 0 side) and c_x_upper in [0, INFINITY].  These
 *               walls are parallel to the imposed field, which the paper's
 *               closures do not cover: f bounces back; the induced tangential
 *               component b_y = B_y - B0 takes the theta closure with the
 *               same a as the Hartmann walls; the normal B_x anti-bounces to
 *               zero.  Links crossing a Hartmann wall at a corner take that
 *               wall's closure (with its moving-wall term).
 *   s_fe,       MRT rates of f's e, epsilon and q moments, finite in (0, 2)
 *   s_feps,     [1.64, 1.54, NaN]; NaN for s_fq takes TRT's odd rate from
 *   s_fq        lambda_f.  Ignored under BGK and TRT.
 *   s_me, s_md  MRT rates of g's epsilon and d moments, finite in (0, 2)
 *               [NaN, NaN]; NaN takes TRT's even rate from lambda_m.
 *   q_lower,    link scheme: distance of each Hartmann wall from its wall row
 *   q_upper     in (0, 1] [1/2, the paper's half-way wall].  Other values put
 *               the walls q beyond the wall rows, so that the half-width is
 *               a = (ny - 1 + q_lower + q_upper)/2, and close
 *               them by interpolated bounce-back of f (with a correction that
 *               keeps the wall impermeable), interpolated anti-bounce-back of
 *               the field components with wall value zero, and, for the
 *               tangential component at a conducting wall, a three-node
 *               closure that reduces to the paper's at q = 1/2 (single
 *               channels, not enclosures or batches; ny >= 3; a conducting
 *               wall needs c a + q + tau_m - 1 >= 1/4).
 *   nsolids,    solid bodies (lks_solid) in the channel [0]: curved walls,
 *   solids      which the paper names as future work (Sec. IX).  A fluid
 *               node's populations pulled from a solid node are closed on
 *               that link at the surface distance q (0 < q <= 1, the
 *               fraction of the link from the node): f by linear
 *               interpolated bounce-back (Bouzidi, Firdaouss and Lallemand,
 *               Phys. Fluids 13 (2001) 3452) with the surface velocity's
 *               moving-wall term, g by interpolated anti-bounce-back that
 *               holds the induced field at zero on the surface (B = (0, B0):
 *               an insulating body that field lines cross undisturbed).  At
 *               q = 1/2 this is the paper's link closure of an insulating
 *               Hartmann wall; at other q interpolated bounce-back lets a
 *               little mass through the surface.  Solid nodes hold the rest
 *               state at unit density (their observables: rho = 1, u = 0,
 *               B = (0, B0), J = 0).  Single channels in FP64 or FP32 storage,
 *               x periodic with half-way Hartmann walls (q = 1/2), nodes
 *               next to a body not on the rows 0 and ny - 1; plain launches
 *               (shape 0) only.
 */
/* Solid bodies inside a channel (curved walls), in lattice units with node
 * (i, j) at the point (i, j); x is periodic, so a circle also covers its
 * images one period away.  A node is solid if it lies strictly inside a
 * body.
 *   LKS_SOLID_DISC   solid inside the circle of centre (cx, cy), radius r
 *   LKS_SOLID_BORE   solid outside that circle
 *   LKS_SOLID_BELOW  solid where y < cy (a half-plane)
 *   LKS_SOLID_ABOVE  solid where y > cy
 * omega: a circle's surface turns at angular velocity omega
 * (counterclockwise) about its centre; u: a half-plane slides along x. */
#define LKS_MAX_SOLIDS 4
enum lks_solid_kind { LKS_SOLID_DISC = 1, LKS_SOLID_BORE = 2, LKS_SOLID_BELOW = 3,
                      LKS_SOLID_ABOVE = 4 };
typedef struct {
  int32_t kind, pad;
  double cx, cy, r;
  double omega;
  double u;
} lks_solid;

typedef struct {
  int32_t nx, ny;
  int32_t bc;
  int32_t precision;
  double tau_f, tau_m;
  double ha;
  double b0;
  double c_lower, c_upper;
  double u_lower, u_upper;
  double fx, fy;
  double u_max;
  double rho0;
  int32_t collision;
  int32_t x_walls;
  double lambda_f, lambda_m;
  double c_x_lower, c_x_upper;
  double q_lower, q_upper;
  double s_fe, s_feps, s_fq;
  double s_me, s_md;
  int32_t nsolids, pad_;
  lks_solid solids[LKS_MAX_SOLIDS];
} lks_mhd_params;

/* Lattice quantities derived from a parameter set (host FP64). */
typedef struct {
  double nu, eta, a, b0, fx, fy;
  double theta_lower, theta_upper; /* link: theta = c_w a / (tau_m - 1/2), Eq. (weightingfactor) */
  double phi_lower, phi_upper;     /* moment: c_w a / (tau_m cs2m), from Eq. (momentbasedBCslowerboundary) */
  double tau_f_odd, tau_m_even;    /* TRT: 1/2 + lambda / (tau - 1/2); BGK: tau_f, tau_m */
  double s_fe, s_feps, s_fq;       /* MRT rates in use (NaNs resolved); else the TRT/BGK rates */
  double s_me, s_md;
} lks_mhd_derived;

/* ABI version of the loaded library (LKS_MHD_ABI_VERSION). */
int lks_mhd_abi_version(void);

/* Thread-local message for the last failing call on this thread ("" if none). */
const char *lks_mhd_last_error(void);

/* Fill *p with defaults (see lks_mhd_params) for an nx x ny channel. */
void lks_mhd_default_params(lks_mhd_params *p, int32_t nx, int32_t ny);

/* Host-only validation; no device work.  LKS_EINVAL with a message if the
 * set is invalid (tau <= 1/2, c < 0 or NaN, ny too small, Ha and B0
 * inconsistent, fx NaN with unequal walls, ...). */
int lks_mhd_validate(const lks_mhd_params *p);

/* Host-only derivation of the lattice quantities; validates first. */
int lks_mhd_derive(const lks_mhd_params *p, lks_mhd_derived *out);

/* Device bytes a channel needs in the caller's buffer (two population
 * buffers, a record buffer for the residual, reduction scratch); 0 if the
 * parameters are invalid. */
size_t lks_mhd_state_bytes(const lks_mhd_params *p);

/*
 * Create a channel on the current device: the two distributions of Secs. IV
 * (D2Q5 vector field g) and V (D2Q9 flow f) on an nx x ny lattice, with the
 * parameters the paper's channel flows take (relaxation times, Hartmann
 * number and imposed field, wall conductance ratio c_w of the Shercliff
 * condition of Sec. III per wall, wall velocities of App. B, body force;
 * Sec. VIII and App. C).  dev_buf (>= lks_mhd_state_bytes, 256-byte aligned)
 * is caller-owned device memory that must outlive the handle; the library
 * carves its buffers from it and allocates no device memory.  hip_stream is
 * the hipStream_t all work is enqueued on (NULL: the default stream).  The
 * state is initialised (asynchronously) to the equilibrium at rest, density
 * rho0, B = (0, B0).  *out receives the handle.  LKS_EINVAL for invalid
 * parameters, a NULL or misaligned buffer or a NULL out; LKS_ENOMEM if bytes
 * is below lks_mhd_state_bytes; LKS_EDEVICE if a HIP call fails.
 */
int lks_mhd_create(const lks_mhd_params *p, void *dev_buf, size_t bytes,
                   void *hip_stream, lks_mhd_t **out);

/* Release the handle (device memory stays the caller's).  NULL is a no-op. */
int lks_mhd_destroy(lks_mhd_t *h);

/* Enqueue nsteps >= 0 fused time steps: pull streaming of f and g (Secs.
 * IV and V), the wall closure of the populations entering from a wall
 * (link-based, Sec. VI and App. B.1, or moment-based, Sec. VII, App. A and
 * App. B.2), the moments and the coupled solve of u and J_z (Sec. IV's
 * current from the field's non-equilibrium first moment, Sec. V's velocity
 * with half the force), the collision of f with the force source (Sec. V)
 * and of g (Sec. IV), and the store.  Asynchronous; LKS_EINVAL for a NULL
 * handle or nsteps < 0, LKS_EDEVICE if a launch fails. */
int lks_mhd_step(lks_mhd_t *h, int64_t nsteps);

/* Replay step sequences from a captured HIP graph of steps_per_graph (even,
 * >= 2) kernels when lks_mhd_step is given at least that many steps; 0
 * switches graphs off (the default).  The stream must not be the legacy
 * default stream.  Captures lazily on first use. */
int lks_mhd_set_graph(lks_mhd_t *h, int32_t steps_per_graph);

/* Launch shape of the plain step kernel (tuning): 0 = 256x1 threads in
 * hardware dispatch order; 1 = 64x4, 2 = 128x2 and 3 = 256x1 with
 * consecutive tiles kept on one XCD; 4 = 64x4 in dispatch order; 5 and 6 =
 * 256x1 threads with 2 and 4 consecutive nodes per thread and vector loads
 * and stores (LKS_EINVAL unless nx is a multiple of 2 resp. 4).  Results are
 * bitwise identical for every shape.  Default: 5 for FP16_STORE with even
 * nx, else 0. */
int lks_mhd_set_launch_shape(lks_mhd_t *h, int32_t shape);

/* Steps taken since create (or since the last load_state). */
int64_t lks_mhd_steps_done(const lks_mhd_t *h);

/*
 * Advance until the steady-state residual falls below tol (the paper runs
 * its channel flows to a steady state, Sec. VIII; the residual below is this
 * library's definition of one).  Steps go in
 * windows of K = check_every (>= 2) steps; the first step of a window
 * records phi = (u_x, B_x), the last one compares and reduces in FP64 (fixed
 * order, deterministic)
 *   R = max over phi of ||phi(n) - phi(n-K+1)||_2 / ((K-1) ||phi(n)||_2),
 * the mean change per step over the window, where phi(n) is the field the
 * step after n collides with and n = steps_done - 1.  (Averaging over the
 * window keeps the rounding noise of stochastically rounded storage, which
 * does not accumulate, from masking a steady state.)  Stops at R < tol
 * (LKS_OK), at max_steps (LKS_ENOTCONV) or on a non-finite value
 * (LKS_EUNSTABLE).  FP16_STORE states are rebased (lks_mhd_rebase) at the
 * start of every window.  Synchronous.  *steps_done and *residual (either may be
 * NULL) receive the totals reached in every case; *flow_rate (may be NULL)
 * receives sum(u_x)/nx of phi(n).
 */
int lks_mhd_run_to_steady(lks_mhd_t *h, double tol, int64_t check_every,
                          int64_t max_steps, int64_t *steps_done,
                          double *residual, double *flow_rate);

/*
 * Observables of the current state (Secs. IV and V): the density
 * rho = sum f, the velocity u from rho u = sum f e + F/2 with the force F of
 * the coupled solve, the field B = sum g and the current density J_z from
 * the non-equilibrium part of the field's first moment -- the fields the
 * next step collides with (after streaming and wall closure), in FP64.
 * Each pointer is a HOST array of nx*ny doubles, row-major [ny][nx], or NULL
 * to skip; the caller owns them.  Synchronous: waits for the handle's
 * stream, then returns with the arrays filled.  Stages the values through
 * the record buffer inside the handle's device memory (no allocation).
 * LKS_EINVAL for a NULL handle, LKS_EDEVICE if a HIP call fails.
 */
int lks_mhd_moments(lks_mhd_t *h, double *rho, double *ux, double *uy,
                    double *bx, double *by, double *jz);

/* The same observables written to DEVICE arrays of nx*ny doubles (or NULL
 * to skip), enqueued on the handle's stream.  Asynchronous. */
int lks_mhd_moments_device(lks_mhd_t *h, double *rho, double *ux, double *uy,
                           double *bx, double *by, double *jz);

/* Copy the state out to / in from a device FP64 array [19][ny][nx] of raw
 * population values (checkpoint, resume, parity tests).  load_state resets
 * steps_done to `steps`.  Asynchronous. */
int lks_mhd_save_state(lks_mhd_t *h, double *dev_pops);
int lks_mhd_load_state(lks_mhd_t *h, const double *dev_pops, int64_t steps);

/* Rebase a binary16 state: for each row y and plane alpha, move the mean
 * over x of the stored values into the row reference and re-encode the row
 * against it (stochastic rounding; the random bits hash the steps taken and
 * the node).  The populations the state decodes to change only by that
 * rounding.  A no-op for FP64 and FP32 storage.  Asynchronous. */
int lks_mhd_rebase(lks_mhd_t *h);

/* lks_mhd_step rebases a binary16 state before a step whenever steps_done is
 * a multiple of `every` (default 1000; 0 switches this off; graph replays
 * stop at those points).  run_to_steady does not apply this interval: it
 * rebases at the start of each of its windows instead.  With every = K,
 * plain stepping reproduces bit for bit the states of run_to_steady or batch
 * windows of K steps.  Ignored for FP64 and FP32 storage. */
int lks_mhd_set_rebase(lks_mhd_t *h, int64_t every);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): advance
 * a channel given as raw FP64 populations [19][ny][nx] on the device
 * (dev_pops, the plane order of lks_mhd_save_state; read and overwritten in
 * place) by nsteps >= 0 steps, step0 >= 0 being the steps the state has
 * already taken (the stochastic-rounding stream index).  The result is bit
 * for bit that of lks_mhd_create + lks_mhd_load_state(dev_pops, step0) +
 * lks_mhd_step(nsteps) + lks_mhd_save_state(dev_pops) with the same
 * parameters (plain launches, the default rebase interval of binary16).
 * The working memory (two population buffers, row references, step
 * counters) is a static 64 MiB device array of the library, one per GPU it
 * runs on, held until the process ends; nothing is allocated.  LKS_ENOMEM
 * if the channel needs more than that (about 200k nodes in FP64, 400k in
 * FP32, 700k in binary16), LKS_EINVAL for invalid parameters or arguments,
 * LKS_EDEVICE if a HIP call fails.  Asynchronous on hip_stream.  Every call
 * on one GPU uses the same array: calls that overlap on a GPU (other
 * streams, other host threads) race.
 */
int lks_mhd_advance_noalloc(const lks_mhd_params *p, double *dev_pops, int64_t step0,
                            int64_t nsteps, void *hip_stream);

/* Algorithmic HBM bytes of one step per node (19 populations read and
 * written) for a precision: 304, 152 or 76. */
int lks_mhd_bytes_per_node(int32_t precision);

/*
 * The stochastic rounding binary32 -> binary16 that the binary16 storage
 * modes apply to every stored value (the paper fixes no storage precision;
 * this is the library's own), exposed so that its bits can be checked:
 * out[i] = the binary16 bits of v[i] rounded with the random word r[i].
 * The top 13 bits of r[i] are added below binary16's last place (in the
 * subnormal range, below 2^-24) to the magnitude of v[i], which is then
 * truncated there; a carry past 65504 gives infinity.  v, r and out are
 * device arrays of n elements (0 <= n < 2^31); LKS_EINVAL for a negative or
 * too large n or a null array with n > 0, LKS_EDEVICE if the launch fails.
 * Asynchronous on hip_stream.
 */
int lks_round_binary16(const float *v, const uint32_t *r, uint16_t *out, int64_t n,
                       void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Batched channels: many independent channels of any size in one launch.   */
/* ------------------------------------------------------------------------ */

/*
 * Create a batch over a caller-owned device pool (>= 256-byte aligned).  All
 * channels share one precision (any lks_precision).
 * max_channels (1..65535) bounds the slot table.  The library allocates no device
 * memory: slot table, tile list and reduction scratch are carved from the
 * pool's front (lks_mhd_batch_overhead_bytes), channel states from the rest.
 */
size_t lks_mhd_batch_overhead_bytes(int32_t max_channels, int64_t max_nodes);
int lks_mhd_batch_create(int32_t precision, int32_t max_channels,
                         int64_t max_nodes, void *dev_pool, size_t pool_bytes,
                         void *hip_stream, lks_mhd_batch_t **out);
int lks_mhd_batch_destroy(lks_mhd_batch_t *b);

/* Device bytes one channel's state takes in the pool. */
size_t lks_mhd_batch_channel_bytes(const lks_mhd_params *p, int32_t precision);

/* Admit a channel (its precision field is ignored; the batch's is used).
 * Allocates its state from the pool (first fit) and initialises it at rest.
 * LKS_ENOMEM if the pool, the slot table or max_nodes is full.  *slot
 * receives the slot id.  Asynchronous. */
int lks_mhd_batch_admit(lks_mhd_batch_t *b, const lks_mhd_params *p,
                        int32_t *slot);

/* Remove a channel and free its pool region. */
int lks_mhd_batch_retire(lks_mhd_batch_t *b, int32_t slot);

/* Number of active channels, and the total nodes they hold. */
int32_t lks_mhd_batch_active(const lks_mhd_batch_t *b);
int64_t lks_mhd_batch_nodes(const lks_mhd_batch_t *b);

/* Tile shape used for channels of a width class (class k holds channels with
 * nx in (2^(k+2), 2^(k+3)], k = 0..6; nx <= 8 in class 0, nx > 256 in
 * class 6).  One tile is the work of one 256-thread block:
 *   tile_w in {8, 16, 32, 64, 128, 256}, tile_w * tile_h = 256: a tile_w x
 *     tile_h rectangle of the channel;
 *   tile_w = 0, tile_h in {1, 2, 4}: 256 * tile_h consecutive nodes of the
 *     channel's row-major planes (the default, with tile_h = 1). */
int lks_mhd_batch_set_tile(lks_mhd_batch_t *b, int32_t width_class,
                           int32_t tile_w, int32_t tile_h);

/* Time every candidate tile shape per width class on the current channel
 * mix (trial_steps each) and keep the fastest.  The trial steps are real
 * steps: every active channel advances by them and its steps_done grows.
 * Synchronous.  The chosen shapes are written to tiles_out[7][2] if non-NULL. */
int lks_mhd_batch_autotune(lks_mhd_batch_t *b, int32_t trial_steps,
                           int32_t *tiles_out);

/* Enqueue nsteps steps of every active channel in one persistent launch per
 * step (captured in a HIP graph of two launches when use_graph != 0).
 * Asynchronous. */
int lks_mhd_batch_step(lks_mhd_batch_t *b, int64_t nsteps, int32_t use_graph);

/* Advance nsteps >= 2 steps as one residual window (the first step records,
 * the last reduces the per-channel residual; definition as in
 * lks_mhd_run_to_steady with K = nsteps; binary16 states are rebased at the
 * window's start).  Writes
 * per-slot residuals to residuals[max_channels] and per-slot flags (1 =
 * non-finite) to unstable[max_channels] (host arrays; entries of empty slots
 * are NaN / 0).  Synchronous. */
int lks_mhd_batch_step_check(lks_mhd_batch_t *b, int64_t nsteps,
                             int32_t use_graph, double *residuals,
                             int32_t *unstable);

/* Rebase every active binary16 channel (as lks_mhd_rebase; no-op for the
 * other precisions).  Asynchronous. */
int lks_mhd_batch_rebase(lks_mhd_batch_t *b);

/* Steps the slot has taken since admission. */
int64_t lks_mhd_batch_steps_done(const lks_mhd_batch_t *b, int32_t slot);

/* Observables and state of one slot (device pointers as for one channel). */
int lks_mhd_batch_moments(lks_mhd_batch_t *b, int32_t slot, double *rho,
                          double *ux, double *uy, double *bx, double *by,
                          double *jz);
int lks_mhd_batch_save_state(lks_mhd_batch_t *b, int32_t slot,
                             double *dev_pops);

/* ------------------------------------------------------------------------ */
/* Three-dimensional channel: x and z periodic, Shercliff walls at y = 0 and */
/* y = ny - 1 (the paper's schemes, which it states extend readily to three  */
/* dimensions, Sec. IX).                                                      */
/* ------------------------------------------------------------------------ */

/*
 * Lattices: D3Q19 for f (weights 1/3, 1/18, 1/36, c_s^2 = 1/3) and D3Q7 for
 * each of the three components of g with rest weight 0 and 1/6 on the six
 * axis links (c_sm^2 = 1/3, the paper's value).  These are the weights whose
 * e_z sums give the paper's D2Q9 and D2Q5, so a z-invariant run reproduces
 * the two-dimensional scheme exactly.  Closures per component: the link-based
 * theta closure (tangential B_x, B_z; the moving-wall term on B_x only, as
 * walls move along x) and anti-bounce-back (normal B_y); the moment closure
 * takes the paper's constraint set per tangential direction (Pi_y = 0,
 * Pi_x = rho U, Pi_xx = rho (cs2 + U^2), Pi_z = 0, Pi_zz = rho cs2) and the
 * discrete Shercliff relation for B_x and B_z, sum g_y = B0 for B_y.  J has
 * three components, each from one antisymmetric pair of Lambda; u and J are
 * solved together in closed form.
 *
 * base: the two-dimensional parameter set (nx, ny, bc, tau_f, tau_m, Ha or
 * B0, c and U per wall, fx or u_max, fy, rho0; derived exactly as for one
 * channel); precision LKS_FP64 or LKS_FP32 (binary32 storage, FP64
 * arithmetic, stochastic rounding).  nz >= 1 layers; fz the body force
 * along z.  nx * ny * nz must be below 2^31, and one layer's plane of
 * nx * ny values below 2^32 bytes.
 *
 * side_walls 0: z periodic (a channel).  1: a rectangular duct, z bounded
 * by stationary thin conducting side walls half-way outside the layers
 * z = 0 and z = nz-1 (nz >= 2, link-based closures only), with conductance
 * ratios c_side_lower (z = 0 side) and c_side_upper in [0, INFINITY].  Their
 * closure per link: bounce-back for f; for the field the theta-weighted
 * Shercliff closure on the induced tangential components b_x and
 * b_y = B_y - B0 (theta = c a / (tau_m - 1/2), a the Hartmann half-width as
 * at the Hartmann walls) and anti-bounce-back to B_z = 0 for the normal one.
 * The paper treats walls normal to the field only; the side walls apply its
 * thin-wall condition to the walls parallel to it.
 */
typedef struct lks_mhd3 lks_mhd3_t;
typedef struct {
  lks_mhd_params base;
  int32_t nz;
  int32_t side_walls;
  double fz;
  double c_side_lower, c_side_upper;
} lks_mhd3_params;

/* Device bytes for create (0 and a message for invalid parameters); bytes
 * of one step per node: 37 stored planes read and written, 592 (FP64) or
 * 296 (FP32). */
size_t lks_mhd3_state_bytes(const lks_mhd3_params *p);
int lks_mhd3_bytes_per_node(int32_t precision);

/* Create over a caller-owned, 256-byte aligned device buffer; initial state
 * at rest with B = (0, B0, 0).  Asynchronous on hip_stream. */
int lks_mhd3_create(const lks_mhd3_params *p, void *dev_buf, size_t bytes,
                    void *hip_stream, lks_mhd3_t **out);
int lks_mhd3_destroy(lks_mhd3_t *h);

/* As lks_mhd_step / set_graph / steps_done / run_to_steady (residual over
 * u_x and B_x of every node; flow_rate = sum u_x / (nx nz)). */
int lks_mhd3_step(lks_mhd3_t *h, int64_t nsteps);
int lks_mhd3_set_graph(lks_mhd3_t *h, int32_t steps_per_graph);
int64_t lks_mhd3_steps_done(const lks_mhd3_t *h);
int lks_mhd3_run_to_steady(lks_mhd3_t *h, double tol, int64_t check_every,
                           int64_t max_steps, int64_t *steps_done,
                           double *residual, double *flow_rate);

/* Observables (device arrays of nx*ny*nz doubles, [z][y][x], or NULL):
 * density, velocity, field and current density J = curl B. */
int lks_mhd3_moments(lks_mhd3_t *h, double *rho, double *ux, double *uy,
                     double *uz, double *bx, double *by, double *bz,
                     double *jx, double *jy, double *jz);

/* State exchange as raw FP64 populations [40][nz][ny][nx] (device):
 * f_0..f_18 (D3Q19 order: rest; +x, +y, -x, -y; (1,1,0), (-1,1,0),
 * (-1,-1,0), (1,-1,0); +z, -z; (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1);
 * (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1)), then for B_x, B_y, B_z the seven
 * D3Q7 populations (rest, +x, +y, -x, -y, +z, -z).  The rest populations
 * of g have weight 0 and are zero; load_state ignores them.  load_state
 * resets steps_done to `steps`.  Asynchronous. */
int lks_mhd3_save_state(lks_mhd3_t *h, double *dev_pops);
int lks_mhd3_load_state(lks_mhd3_t *h, const double *dev_pops, int64_t steps);

#ifdef __cplusplus
}
#endif

#endif /* LKS_MHD_H */
