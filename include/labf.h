/*
 * labf.h -- C ABI of the MI355X (gfx950) lambda-ABF alchemical nonbonded step.
 *
 * The operation is the per-timestep work every walker of a lambda-ABF run
 * performs (Lagardere et al., "Lambda-ABF: Simplified, Portable, Accurate,
 * and Cost-effective Alchemical Free Energy Computation"):
 *   1. a cell/cluster neighbour build at r_list = r_cut + r_skin;
 *   2. the lambda-scaled nonbonded forces and the alchemical force
 *      dV/dlambda ("Alchemical pathway": soft-core LJ for lambda_v and
 *      linear scaling of electrostatics by lambda_e, decoupling; cutoff
 *      shifted-force Coulomb, or smooth PME with the reciprocal term
 *      interpolated linearly between the electrostatic end states when
 *      labf_system_desc.pme_order > 0);
 *   3. a BAOAB Langevin step of the atoms and of the extended coordinate
 *      (lambda, p_lambda) of Eq. (lambdadyn-Langevin-process), with the ABF
 *      term of Eq. (lambda-abf) and reflecting boundaries;
 *   4. accumulation of dV/dlambda into ABF bins shared by all walkers
 *      ("Orthogonal space sampling": multiple walkers sharing their
 *      mean-force estimate every K steps; "ABF parameters": linear ramp up to
 *      fullSamples), whose bin averages integrate to A(lambda).
 * The split mirrors the paper's engine/Colvars interface ("Software
 * interface"): the engine side owns coordinates and forces, the library
 * side owns lambda's mass, friction, temperature, bounds, bins and sharing.
 *
 * Conventions
 *   - Units: any consistent set.  Real units: A, fs, amu, kcal/mol, e, with
 *     accel_unit = 4.184e-4 (kcal/mol/A/amu -> A/fs^2) and coulomb_k =
 *     332.0637; reduced units: accel_unit = 1.
 *   - Arrays passed to the calls below are HOST arrays unless stated
 *     otherwise; they are copied during the call and may be freed after it.
 *     Atom arrays are in the caller's original atom order, walker w owning
 *     atoms [atom_offset[w], atom_offset[w+1]).  Vectors are AoS [N][3].
 *   - Device memory is the caller's: labf_workspace_size gives the bytes a
 *     system needs, and labf_create_system lays out every device array of
 *     the system inside the workspace the caller passes (a torch uint8
 *     tensor, say).  The library allocates no device memory for a system
 *     (only the test hooks labf_export_pairs, labf_philox and labf_probe
 *     allocate their own staging, released before they return or with the
 *     handle).  The workspace must stay allocated, and must not be touched by
 *     the caller, until labf_destroy_system returns.  Device work is
 *     asynchronous on the HIP stream passed in (NULL = default stream; the
 *     Python binding passes torch's current stream); calls that return host
 *     data synchronise that stream.  A handle is not thread-safe.
 *   - Errors: every call returns a labf_status.  Argument errors are found on
 *     the host before any device work.  Numerical faults of a walker
 *     (non-finite lambda force, neighbour skin exceeded, list or PME brick
 *     capacity exceeded) are recorded in that walker's status word
 *     (LABF_WS_*) and
 *     surface in labf_read_walker_state.  labf_last_error() describes the
 *     last failure of a handle (or of labf_create_system when passed NULL).
 *   - Positions are stored internally at the precision of the system
 *     (LABF_FP32 or LABF_FP64) offset by a power of two B >= 2L per box
 *     edge, so that every difference of two positions, and every image shift
 *     by +-L, is exact.  Box edges and inputs are rounded to that grid;
 *     labf_read_atoms returns the stored values wrapped into [0, L).
 */
#ifndef LABF_H
#define LABF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct labf_system labf_system; /* opaque; owned by the library */
typedef int32_t labf_status;

#define LABF_OK 0
#define LABF_E_ARG (-1)          /* invalid argument (detected on the host)    */
#define LABF_E_STATE (-2)        /* call not valid in the current state        */
#define LABF_E_HIP (-3)          /* HIP runtime error                          */
#define LABF_E_NONFINITE (-4)    /* non-finite value in a walker               */
#define LABF_E_SKIN (-5)         /* two largest displacements since the last rebuild exceed r_skin */
#define LABF_E_UNSUPPORTED (-6)  /* configuration not supported                */
#define LABF_E_EMPTY_BIN (-7)    /* free-energy readout with an empty bin      */
#define LABF_E_CAPACITY (-8)     /* neighbour list capacity exceeded           */

#define LABF_FP32 0              /* FP32 positions and pair terms; FP64 dV/dlambda, bins, lambda */
#define LABF_FP64 1              /* FP64 throughout                            */

#define LABF_DECOUPLE 0          /* c_x = 1 - ramp_x(lambda) (NAMD convention)  */
#define LABF_COUPLE 1            /* c_x = ramp_x(lambda) (Tinker-HP convention) */

/* soft-core form of the lambda-scaled LJ ("Alchemical pathway"; the
 * separation-shifted form is the one of the NAMD setup of the SI) */
#define LABF_SC_BEUTLER 0        /* 4 eps c (y^2 - y), y = 1/(alpha (1-c)^p + (r/sig)^6) */
#define LABF_SC_SHIFTED 1        /* 4 eps c (sig^12/s^6 - sig^6/s^3), s = r^2 + sc_shift (1-c) */

#define LABF_MODE_BATCHED 0      /* all walkers per launch, 10-step blocks replayed as HIP graphs */
#define LABF_MODE_PLAIN 1        /* one walker per launch sequence, no graph    */

/* walker status bits */
#define LABF_WS_NONFINITE 1u
#define LABF_WS_REFLECT 2u       /* lambda needed more than one reflection     */
#define LABF_WS_SKIN 4u          /* the two largest displacements since a rebuild exceed r_skin */
#define LABF_WS_CAPACITY 8u       /* a neighbour list or a PME charge-spread brick list overflowed */

/* Static description of a batch of walkers ("Software interface": the
 * engine side).  All pointers are host pointers. */
typedef struct labf_system_desc {
  int32_t n_walkers;           /* W >= 1                                          */
  int32_t precision;           /* LABF_FP32 | LABF_FP64                           */
  const int64_t *atom_offset;  /* [W+1], atom_offset[0] = 0, non-decreasing, each walker >= 1 atom */
  const double *box;           /* [W][3] orthorhombic box edges, periodic         */
  const double *pos;           /* [N][3] initial positions (wrapped into the box) */
  const double *vel;           /* [N][3] initial velocities, or NULL: Maxwell-Boltzmann at kT */
  const double *mass;          /* [N] > 0                                         */
  const double *charge;        /* [N]                                             */
  const double *sigma;         /* [N] LJ sigma (> 0 where epsilon > 0)            */
  const double *epsilon;       /* [N] LJ epsilon >= 0; Lorentz-Berthelot mixing   */
  const uint8_t *is_solute;    /* [N] 1: atom of the alchemically decoupled group */
  const double *anchor;        /* [N][3] restraint anchors, or NULL (no restraints) */
  const double *k0;            /* [N] restraint constant at lambda = 0 (NULL iff anchor NULL) */
  const double *k1;            /* [N] restraint constant at lambda = 1            */
  double r_cut;                /* pair cutoff; r_cut + r_skin < L/2 on every edge */
  double r_skin;               /* list buffer                                     */
  double kT;                   /* atom bath temperature (energy units)            */
  double gamma;                /* atom friction (1/time)                          */
  double dt;                   /* time step                                       */
  double coulomb_k;            /* Coulomb constant                                */
  double accel_unit;           /* force/mass -> acceleration factor               */
  uint64_t seed;               /* Philox4x32-10 key                               */
  int32_t rebuild_interval;    /* steps between neighbour rebuilds (>= 1; 10 typical) */
  int32_t pme_order;           /* 0: shifted-force Coulomb cut at r_cut.  4, 6 or 8: Ewald
                                  electrostatics, real-space erfc(beta r)/r pairs cut at r_cut
                                  plus smooth-PME reciprocal space with B-splines of this order
                                  (Essmann et al. 1995), self and neutralising-background terms.
                                  The alchemical group's electrostatic coupling scales the
                                  group-environment real-space pairs and the cross part of the
                                  reciprocal and background terms linearly (Section 2, alchemical
                                  pathway: many-body terms interpolated between the end values) */
  double r_skin_alch;          /* list buffer of pairs with an alchemical atom (solute atoms and
                                  atoms with k0 != k1), or 0: r_skin.  A decoupled solute has no
                                  solvent cage and can move much farther between rebuilds than the
                                  environment.  r_skin <= r_skin_alch, r_cut + r_skin_alch < L/2 */
  const double *column_width;  /* [W] x-y width of the cluster columns in units of (8/rho)^(1/3)
                                  (rho: the walker's environment atom density; 1 gives cubic
                                  8-atom clusters), or NULL: 1 for every walker; 0.5 .. 2.
                                  The tile shape that an autotuner chooses per size class */
  const int32_t *pme_dims;     /* [W][3] PME grid points per edge when pme_order > 0: multiples
                                  of 8 in [16, 256] with no prime factor above 5 (16, 24, 32,
                                  40, 48, 64, 72, 80, 96, 120, ...; else LABF_E_ARG); ignored
                                  (may be NULL) otherwise */
  double ewald_beta;           /* Ewald splitting parameter (1/length) > 0 when pme_order > 0 */
  int32_t max_bins;            /* ABF bin capacity: labf_set_lambda_params accepts n_bins up to
                                  this; 0: 1024; at most 4096 */
  int32_t list_capacity;       /* neighbour-list entries per cluster, or 0: twice the longest list
                                  estimated on the host from the initial positions plus headroom
                                  (overflow later sets LABF_WS_CAPACITY); 16 .. 2^20 */
  void *workspace;             /* DEVICE memory owned by the caller, 256-byte aligned, at least
                                  labf_workspace_size bytes (labf_create_system only; ignored by
                                  labf_workspace_size) */
  size_t workspace_bytes;      /* its size in bytes */
  const double *prune_buffer;  /* [W] b per walker, or NULL: the environment kernel evaluates, per
                                  cluster of 8 atoms, the atoms of its neighbour clusters within
                                  r_cut + b of the cluster's box, pruned after each rebuild and
                                  again whenever an atom of the walker has moved more than b/2
                                  since (a larger b prunes less often and evaluates more pairs);
                                  0 (or NULL): min(0.35, r_skin/2) in length units; else
                                  0 < b <= r_skin.  The second knob an autotuner chooses per size
                                  class.  Unused with pme_order > 0 (the real-space Ewald kernels
                                  prune the cluster lists as they evaluate them) */
} labf_system_desc;

/* Extended-lambda and ABF parameters ("Software interface" and "ABF
 * parameters": the library side; one set shared by all walkers). */
typedef struct labf_lambda_params {
  const double *lambda0;       /* [W] initial lambda in [lo, hi]                  */
  const double *p_lambda0;     /* [W] initial momenta, or NULL: Maxwell-Boltzmann */
  double m_lambda;             /* fictitious mass (energy * time^2)               */
  double gamma_lambda;         /* lambda friction (1/time)                        */
  double kT_lambda;            /* lambda bath temperature                         */
  double elec_start, elec_end; /* electrostatics ramp over [elec_start, elec_end] */
  double vdw_start, vdw_end;   /* soft-core vdW ramp over [vdw_start, vdw_end]    */
  int32_t direction;           /* LABF_DECOUPLE | LABF_COUPLE                     */
  int32_t sc_power;            /* soft-core exponent p >= 1                       */
  double sc_alpha;             /* soft-core alpha >= 0                            */
  int32_t n_bins;              /* ABF bins on [lo, hi], 1..4096                   */
  int32_t share_interval;      /* K >= 1: walkers merge their ABF samples every K steps */
  double lo, hi;               /* lambda range = reflecting boundaries            */
  int64_t full_samples;        /* bias ramp length (>= 1)                         */
  int32_t fixed_lambda;        /* 1: lambda frozen (samples still accumulated)   */
  int32_t abf_on;              /* 0: no ABF samples and no bias                   */
  int32_t sc_form;             /* LABF_SC_BEUTLER | LABF_SC_SHIFTED               */
  int32_t reserved2;           /* must be 0                                       */
  double sc_shift;             /* delta of LABF_SC_SHIFTED (length^2, >= 0)       */
} labf_lambda_params;

/* Bytes of device workspace a system of this descriptor needs (host
 * arithmetic only, no device call: the walker layout, the PME tables, the
 * neighbour-list capacity estimated from the initial positions, the ABF
 * accumulators for max_bins bins).  Validates the descriptor like
 * labf_create_system (the workspace fields are not read).  Errors:
 * LABF_E_ARG. */
labf_status labf_workspace_size(const labf_system_desc *desc, size_t *bytes);

/* Create a system: validates the descriptor on the host, lays out the
 * device arrays in desc->workspace (LABF_E_ARG if it is NULL, misaligned or
 * smaller than labf_workspace_size), uploads the atoms and builds the first
 * neighbour list on `stream`; allocates no device memory.  LABF_E_CAPACITY
 * if the initial lists exceed the list capacity.  On success *out receives
 * the handle.  On failure *out is NULL and labf_last_error(NULL) describes
 * the error. */
labf_status labf_create_system(const labf_system_desc *desc, void *stream, labf_system **out);

/* Set lambda/ABF parameters and reset lambda state: lambda = lambda0,
 * p_lambda = p_lambda0 (or Maxwell-Boltzmann draws), ABF bins emptied, the
 * next step starts a fresh BAOAB sequence.  Required before stepping.
 * n_bins must not exceed the system's max_bins (LABF_E_ARG). */
labf_status labf_set_lambda_params(labf_system *sys, const labf_lambda_params *lp, void *stream);

/* Advance every walker by n_steps >= 0 steps (asynchronous).  mode:
 * LABF_MODE_BATCHED or LABF_MODE_PLAIN; both give identical results. */
labf_status labf_step_walkers(labf_system *sys, int64_t n_steps, int32_t mode, void *stream);

/* Shared ABF accumulator (synchronous).  counts/sum/sum_sq: [n_bins]
 * (sum_sq may be NULL).  include_unshared = 1 adds the samples walkers have
 * not merged yet (share_interval > 1). */
labf_status labf_read_abf_bins(labf_system *sys, int32_t n_bins, int32_t include_unshared,
                               int64_t *counts, double *sum, double *sum_sq, void *stream);

/* Free-energy readout of the Riemann sum of bin averages (host arithmetic
 * on labf_read_abf_bins(include_unshared = 1)): grad[b] = sum_b / count_b,
 * profile[b] = A(lo + b w) - A(lo), *delta_a = A(hi) - A(lo).  Any pointer
 * may be NULL.  Returns LABF_E_EMPTY_BIN (with the outputs still written)
 * if a bin has no sample. */
labf_status labf_free_energy(labf_system *sys, double *grad, double *profile, double *delta_a,
                             void *stream);

/* Walker state (synchronous), each [W] and nullable: lambda, p_lambda (in
 * the pending form of the BAOAB sequence: the closing half-kick of the last
 * step is applied at the start of the next one), the last dV/dlambda and
 * ABF bias, status bits, and *step = steps taken since the last reset. */
labf_status labf_read_walker_state(labf_system *sys, double *lambda, double *p_lambda,
                                   double *dudl, double *bias, uint32_t *status, int64_t *step,
                                   void *stream);

/* Atom state in original order (synchronous): pos, vel [N][3] (nullable).
 * Velocities are in the pending form described above. */
labf_status labf_read_atoms(labf_system *sys, double *pos, double *vel, void *stream);

/* Replace positions and/or velocities ([N][3], nullable); rebuilds the
 * neighbour list and starts a fresh BAOAB sequence. */
labf_status labf_write_atoms(labf_system *sys, const double *pos, const double *vel, void *stream);

/* Evaluate, at the current positions and lambda, the forces [N][3], the
 * energy decomposition energy[W][5] = {environment-environment,
 * solute-solute, alchemical LJ, alchemical Coulomb, restraints} and
 * dV/dlambda [W] (synchronous; nullable outputs).  Rebuilds the list.
 * With PME the reciprocal, self and background energies of the environment's
 * own charges go to the first entry, those of the group's own charges to the
 * second, and the cross part (ce times the reciprocal cross term and the
 * background cross term) to the alchemical Coulomb entry. */
labf_status labf_compute_forces(labf_system *sys, double *forces, double *energy, double *dudl,
                                void *stream);

/* Lambda-dependent distance restraint ("Dealing with metastabilities
 * related to counterions"): between two atoms a, b of each walker,
 *   V = k/2 (d - d_min)^2  if d < d_min(lambda),  0 otherwise,
 *   d_min(lambda) = (delta/2)(1 - cos(2 pi freq lambda)),
 * d the minimum-image distance; it vanishes at lambda = 0 and 1 (freq = 1:
 * the form of the text, d_min(1/2) = delta; freq = 2: lambda doubled, as in
 * the SI script).  Adds its forces to both atoms, -k (d - d_min) d_min' to
 * dV/dlambda and its energy to the restraint part.
 *   pairs  host [W][2] walker-local atom indices, (-1, -1) for no restraint
 *          in that walker; NULL removes the restraint everywhere
 *   delta  >= 0 and < L/2 on every edge; k >= 0; freq 1 or 2
 * Errors: LABF_E_ARG (nothing changed). */
labf_status labf_set_distance_restraint(labf_system *sys, const int32_t *pairs, double delta,
                                        double k, int32_t freq, void *stream);

/* Differentiable potential energy ("Theory": the extended potential
 * V(q; lambda) whose derivatives drive the dynamics and the ABF estimator;
 * "Alchemical pathway": the lambda-scaled soft-core LJ and shifted-force
 * Coulomb terms).  For automatic differentiation (a torch.autograd.Function
 * sits on top): the forward call evaluates energies only (no forces, no
 * parameter gradient), and nothing it computes is kept for the backward
 * call, whose own kernels recompute every pair term.
 *
 * Every array argument of these two calls is a DEVICE pointer on the
 * system's GPU, read and written in the order of `stream`; the caller owns
 * them.  Each of pos, lambda, params may be NULL (keep the current value):
 *   pos     [N][3] FP64, caller order; wrapped into the box and rounded to
 *           the storage grid exactly as labf_write_atoms does
 *   lambda  [W] FP64; a value outside [lo, hi] gets the schedule's clipped
 *           couplings (no reflection is applied here)
 *   params  [S][3] FP64 (epsilon, sigma, q) of the solute atoms in increasing
 *           atom order (S = labf_info.n_solute); copied to the host and
 *           validated (finite, epsilon >= 0, sigma > 0 where epsilon > 0;
 *           LABF_E_ARG otherwise, nothing changed)
 * The given values replace the system's (velocities, lambda momenta and the
 * ABF accumulators are kept).  The neighbour structure is rebuilt when pos
 * or params are given or the atoms have moved since the last rebuild
 * (positions given: without the list-validity check); a backward call
 * with NULL pos and params after a forward call reuses the forward's lists.
 *
 * labf_energy_forward: energy[W] = total potential energy of each walker
 *   (FP64 sums; environment pair terms in the storage precision); dudl[W]
 *   = dV/dlambda of each walker (or NULL).
 * labf_energy_backward: for the upstream gradient grad_energy[W] = dL/dV_w,
 *   grad_pos[N][3]    = g_w dV_w/dx_a = -g_w F_a      (or NULL)
 *   grad_lambda[W]    = g_w dV_w/dlambda_w             (or NULL)
 *   grad_params[S][3] = g_w dV_w/d(epsilon, sigma, q)_i of solute atom i
 *                       (Lorentz-Berthelot mixing; FP64; or NULL)
 * A non-finite position gives non-finite outputs and walker status bit 1.
 * Errors: LABF_E_STATE before labf_set_lambda_params; LABF_E_ARG for NULL
 * energy / grad_energy or invalid params. */
labf_status labf_energy_forward(labf_system *sys, const double *pos, const double *lambda,
                                const double *params, double *energy, double *dudl, void *stream);
labf_status labf_energy_backward(labf_system *sys, const double *pos, const double *lambda,
                                 const double *params, const double *grad_energy,
                                 double *grad_pos, double *grad_lambda, double *grad_params,
                                 void *stream);

/* The neighbour set of walker w held by the device list: every pair (i < j,
 * walker-local indices) with |x_j - x_i|^2 < r_list^2 under the minimum
 * image, decided in FP64 as (dx*dx + dy*dy) + dz*dz.  Writes up to
 * max_pairs pairs [n][2] in lexicographic order and the total count. */
labf_status labf_export_pairs(labf_system *sys, int32_t walker, int64_t max_pairs, int64_t *pairs,
                              int64_t *n_pairs, void *stream);

/* labf_export_pairs for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same output, with the device staging in a static array
 * of LABF_EXPORT_NOALLOC_MAX_PAIRS pairs (16 MiB per GPU, held until the
 * process ends) instead of a buffer the call allocates; the host output is
 * sorted in place.  It calls no hipMalloc, hipFree or allocating routine.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (other threads, other handles) race.  Errors: LABF_E_ARG as
 * labf_export_pairs; LABF_E_CAPACITY, with *n_pairs set and nothing
 * written, if the walker has more than LABF_EXPORT_NOALLOC_MAX_PAIRS
 * pairs. */
#define LABF_EXPORT_NOALLOC_MAX_PAIRS (1 << 20)
labf_status labf_export_pairs_noalloc(labf_system *sys, int32_t walker, int64_t max_pairs,
                                      int64_t *pairs, int64_t *n_pairs, void *stream);

/* Number of unordered pairs with r < r_cut in each walker (FP64 decision),
 * counted by a separate pass over the device list (rebuilt first):
 * pairs_all[W] every pair, pairs_env[W] pairs of two environment atoms
 * (nullable).  Used to convert steps/s into pair-interactions/s. */
labf_status labf_count_pairs(labf_system *sys, int64_t *pairs_all, int64_t *pairs_env,
                             void *stream);

/* Timing pass (for roofline reporting): rebuilds the list, then runs
 * n_steps >= 1 batched steps launched one kernel at a time with HIP events
 * around each launch on `stream`.  ms[5]: ms[0] = rebuild, ms[1] = alchemical
 * kernel (average per step), ms[2] = environment kernel (average per step),
 * ms[3] = PME reciprocal space (spread, transforms, gather; average per step,
 * 0 without PME), ms[4] = pruning of the environment pair lists (average per
 * step: a full prune after the rebuild and whenever the atoms have moved far
 * enough, a test otherwise).  Advances the dynamics by n_steps like
 * labf_step_walkers. */
labf_status labf_profile_steps(labf_system *sys, int64_t n_steps, double *ms, void *stream);

/* Philox4x32-10 on the device (test hook): out[n][4] for counters ctr[n][4]
 * and key[2], all host arrays. */
labf_status labf_philox(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out,
                        void *stream);

/* Achievable-peak probe of the device (for roofline reporting): kind
 * LABF_PROBE_FP32_FMA / LABF_PROBE_FP64_FMA / LABF_PROBE_FP32_RSQ run 8
 * independent dependency chains per lane for n iterations (1 .. 1e6) on
 * 4096 blocks of 256 lanes and return lane-operations per second in *rate;
 * LABF_PROBE_TRIAD streams a[i] = b[i] + s c[i] over three device arrays of
 * n floats (n a positive multiple of 4, at most 2^30; the arrays are
 * allocated and freed by the call) and returns bytes moved (12 n per pass)
 * per second.  Timed with HIP events over 5 launches after one warm-up, on
 * `stream`; synchronous.  Errors: LABF_E_ARG for a bad kind or n. */
#define LABF_PROBE_FP32_FMA 0
#define LABF_PROBE_FP64_FMA 1
#define LABF_PROBE_FP32_RSQ 2
#define LABF_PROBE_TRIAD 3
labf_status labf_probe(int32_t kind, int64_t n, double *rate, void *stream);

/* Sizes of the device layout (for diagnostics): clusters in use, cluster
 * capacity, list entries in use, list capacity per cluster. */
typedef struct labf_info {
  int64_t n_atoms, n_slots, n_clusters, n_list_entries;
  int32_t n_walkers, list_cap, precision, uniform_lj;
  int32_t list_max_env, list_max_alch;   /* longest list of each cluster kind */
  int64_t n_solute;                      /* atoms with is_solute = 1 (S below) */
} labf_info;
labf_status labf_get_info(labf_system *sys, labf_info *info, void *stream);

void labf_destroy_system(labf_system *sys);
const char *labf_last_error(const labf_system *sys);

#ifdef __cplusplus
}
#endif
#endif
