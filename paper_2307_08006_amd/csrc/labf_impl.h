// labf_impl.h -- internal layout shared by the gfx950 kernels and the host
// runtime of the lambda-ABF alchemical nonbonded step.
//
// Layout in HBM (all walkers of a batch side by side):
//   * atoms in the caller's order: static parameters, slot_of (current slot).
//   * slots: clusters of CL = 8 atoms; walker w owns clusters
//     [cl_begin, cl_begin + cap_env + n_acl): first its environment clusters
//     (GROMACS-like columns on an x-y grid, each column sorted by z and padded
//     to a multiple of 8), then its alchemical clusters (solute atoms and
//     atoms whose restraint depends on lambda), one atom per cluster in
//     slot 0 so that their lists stay local.  Per-slot arrays are SoA.
//   * per cluster: bounding box, a list of neighbour-cluster entries
//     (cluster index | image-shift code << 26) with a fixed capacity per
//     cluster, and flags.
//   * positions are stored offset by B = 2^k >= 2L per box edge: all stored
//     positions share one exponent, so differences, and image shifts by +-L,
//     are exact in the storage precision.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace labf {

constexpr int CL = 8;                 // atoms per cluster
constexpr int SKIN_PARTS = 8;         // blocks per walker of the list-validity reduction
constexpr int WAVE = 64;              // CDNA wavefront
constexpr int SHIFT_BITS = 26;        // cluster index bits in a list entry
constexpr uint32_t CL_MASK = (1u << SHIFT_BITS) - 1u;
// Image code of a list entry: two bits per axis holding s + 1 for the box
// shift s in {-1, 0, 1} (x in bits 0-1, y in 2-3, z in 4-5).
constexpr int image_code(int sx, int sy, int sz) { return (sx + 1) | ((sy + 1) << 2) | ((sz + 1) << 4); }
constexpr int SHIFT_ZERO = image_code(0, 0, 0);  // code of the (0,0,0) image
constexpr int IMG_CODES = 64;                    // table size indexed by code
// Filler entry of a pruned list: the walker's first slot shifted by two box
// edges along every axis, farther than r_cut from any atom of the box.
constexpr uint32_t PRUNE_PAD = (uint32_t)image_code(2, 2, 2) << SHIFT_BITS;
constexpr int PDISP_SLOTS = 64;  // displacement maxima per walker (one wave reads them)
constexpr uint32_t LAMBDA_ATOM = 0xFFFFFFFFu;  // noise stream of lambda
// what an evaluation (no integration) computes
constexpr int EVAL_ALL = 0;     // forces, energy parts, dV/dlambda, solute parameter gradient
constexpr int EVAL_ENERGY = 1;  // energy parts and dV/dlambda only
constexpr int EVAL_GRAD = 2;    // forces, dV/dlambda and the solute parameter gradient

struct WalkerMeta {
  int64_t atom_begin;     // first atom (caller order)
  int64_t cl_begin;       // first cluster
  int32_t n_atoms;
  int32_t n_a;            // alchemical atoms
  int32_t cap_env;        // environment cluster capacity
  int32_t n_acl;          // alchemical clusters (= alchemical atoms; static)
  int32_t ncx, ncy;       // column grid
  int32_t col_begin;      // first entry in per-column arrays (ncx*ncy + 1 columns)
  int32_t item_begin;     // first entry of this walker in the alchemical block table
  int32_t item_cap;       // max(1, n_acl) blocks (a walker without alchemical atoms
                          // still gets one block, which runs its lambda tail)
  int32_t env_item_begin; // first entry in the environment work table
  double L[3];            // box edges
  double B[3];            // storage offset (power of two >= 2L)
  double cw[2];           // column widths
  double prune_b;         // prune buffer of the pair lists
};

// Smooth PME of one walker.  The complex grid holds the environment's charge
// density in the real part and the alchemical group's in the imaginary part,
// so that one complex transform serves both; z is the fastest index.
constexpr int PME_TILE = 4096;  // complex points per FFT block (1024 threads)
constexpr int PME_KMAX = 256;   // largest grid edge
constexpr int PME_PMAX = 8;     // largest B-spline order
constexpr int PME_BR = 8;       // grid brick edge of the charge spread (>= PME_PMAX)
constexpr int PME_PLANE = 8192; // largest K1 K2 transformed as one y-z plane in LDS
constexpr int EWTAB_N = 256;    // intervals of the FP32 real-space Ewald correction table
struct PmeWalker {
  int32_t K[3];           // grid points per edge (2^a 3^b 5^c, multiples of 8, 16 .. PME_KMAX)
  int32_t lg[3];          // log2 K, or -1 when K is not a power of two
  int8_t rad[3][8];       // radices of the mixed-radix stages (forward order), K not a power of two
  int32_t nst[3];         // number of such stages
  int32_t nl[3];          // FFT lines per block along each axis
  int32_t blk[3];         // FFT blocks along each axis
  int32_t blk_begin[3];   // first FFT block of the walker along each axis
  int32_t nbr[3];         // grid bricks per edge (K / PME_BR)
  int32_t br_begin;       // first brick of the walker
  int32_t br_cap;         // atom capacity of one brick's list
  int32_t pl_begin;       // first y-z plane block of the walker (K0 planes)
  int64_t loff;           // first brick-list entry of the walker
  int64_t goff;           // first grid point
  int64_t toff;           // first entry of the per-axis tables (K0 + K1 + K2 entries)
  double pref;            // coulomb_k / (pi V)
};

// Extended-lambda / ABF parameters as the kernels need them.
struct LamParams {
  double m_lambda, gamma_lambda, kT_lambda;
  double elec_start, elec_end, vdw_start, vdw_end;
  double sc_alpha, sc_shift;   // sc_shift: delta of the separation-shifted form
  double lo, hi, bin_w;
  double c1l, sdl;          // exp(-gamma_l dt), sqrt((1 - c1l^2) kT_l m_l)
  int64_t full_samples;
  int32_t direction, sc_power, n_bins, share_interval, fixed_lambda, abf_on;
  int32_t sc_form;             // 0: alpha (1-c)^p + (r/sig)^6; 1: r^2 + delta (1-c)
};

// Everything the kernels touch.  Pointers are device pointers.
template <typename T>
struct Dev {
  // --- sizes and scalars
  int32_t n_walkers;
  int64_t n_atoms, n_slots, n_clusters;
  int32_t list_cap;
  int32_t uniform_lj;
  double r_cut, r_list, r_list_a, dt, kT, gamma, coulomb_k, accel;
  double c1;                // exp(-gamma dt)
  uint64_t seed;
  T rc2, irc, irc2;         // r_cut^2, 1/r_cut, 1/r_cut^2 (storage precision)
  T c6, c12, ushift;        // uniform LJ: 4 eps sig^6, 4 eps sig^12, U_LJ(r_cut)
  LamParams lp;
  // --- static tables
  const WalkerMeta *meta;       // [W]
  const int32_t *atom_walker;   // [N]
  const int32_t *cl_walker;     // [C]
  const int32_t *env_table;     // [sum cap_env] -> cluster
  const int32_t *item_walker;   // [sum item_cap]
  const int32_t *alch_cluster;  // [sum item_cap] alchemical cluster of each block, or -1
  const int32_t *col_walker;    // [K] walker of each column (all walkers' columns concatenated)
  // --- caller-order atom data
  const double *a_pos0;         // [N][3] upload staging (B-offset, rounded)
  double *a_q, *a_sig, *a_eps;  // charge, sigma, epsilon (solute entries replaceable)
  const double *a_mass, *a_k0, *a_k1, *a_anchor;  // anchor [N][3]
  const int32_t *solute_atom;   // [n_solute] atoms with is_solute = 1, increasing
  int64_t n_solute;
  // lambda-dependent distance restraint (NULL tables: none)
  const int32_t *dr_partner;    // [N] the other atom of the atom's restrained pair, or -1
  const int32_t *dr_pair;       // [W][2] the walker's pair (global atom indices), or -1
  double dr_delta, dr_k;
  int32_t dr_freq;
  const uint8_t *a_sol, *a_alch;
  int32_t *slot_of, *new_slot, *col_of, *key_col, *members;
  float *disp;                  // [N] displacement since the last rebuild (rounded up)
  float *skin_part;             // [W][SKIN_PARTS][4] partial top-two displacements
  T *xref;                      // [3][N] positions at the last rebuild
  // --- per column
  int32_t *col_count, *col_fill, *col_atom0, *col_cl0;
  // --- per slot (SoA); X and V double-buffered
  T *X[2][3];
  T *V[2][3];
  T *q;                         // sqrt(coulomb_k) * charge
  T *lja, *ljb;                 // sigma/2, sqrt(eps) (per-atom mixing mode)
  T *aim;                       // accel_unit / mass
  T *nsd;                       // sqrt((1 - c1^2) kT accel_unit / mass)
  T *rk;                        // lambda-independent restraint constant
  T *anc[3];                    // restraint anchor (B-offset)
  double *q64, *sig64, *eps64, *k0_64, *k1_64;
  uint8_t *sol;                 // is_solute per slot
  int32_t *orig;                // walker-local atom index or -1
  double *fout;                 // [3][S] forces of an evaluation
  // --- per cluster
  T *bbox;                      // [C][6] lo xyz, hi xyz (storage precision: exact)
  int32_t *cl_col;              // column of an environment cluster
  int32_t *list_count;          // entries in use (environment, then alchemical)
  int32_t *list_nenv;           // environment-cluster entries of an environment list
  uint32_t *list;               // [C * list_cap]
  double *cl_energy;            // [C][2] env-env, restraint (evaluation)
  // --- pruned pair lists (per environment work-table entry): the j atoms of
  // the list's environment entries within r_cut + prune buffer of the
  // cluster box when last pruned, as (walker-relative slot | image code <<
  // SHIFT_BITS), padded with PRUNE_PAD to whole chunks of 64
  int32_t plist_cap;            // entries per cluster (a multiple of 64)
  uint32_t *plist;              // [E][plist_cap]
  int32_t *plist_n;             // [E] chunks of 64 in use; -1: stale (rebuilt list)
  T *xprune[3];                 // [3][S] positions at the last prune
  T *noise[3];                  // [3][S] Langevin normals of the coming step, drawn by the
                                //   prune kernel for the environment atoms (none with PME)
  uint32_t *pdisp;              // [2][W][PDISP_SLOTS] bits of the largest displacement since
                                // the last prune (non-negative float), spread over slots
                                // (fewer atomics per address), double-buffered like lambda
  // --- alchemical blocks (one per alchemical atom)
  double *item_force;           // [I][3] force on the block's atom
  double *item_dudl;            // [I]
  double *item_energy;          // [I][5]
  double *item_pgrad;           // [I][3] dV/d(eps, sigma, q) of the block's atom (evaluation)
  // --- per walker dynamic state
  int32_t *n_env;
  uint32_t *ticket;             // per walker
  uint32_t *gticket;            // [1]
  uint32_t *status;
  double *lambda;               // [2][W]: read [lb], written [lb ^ 1] by the tail
  double *p_lambda, *dudl, *bias;
  int64_t *step;                // [2][W], same double buffering
  int64_t *start_step;          // [1] step at which the BAOAB sequence (re)started
  double *energy;               // [W][5] evaluation output (alchemical side)
  int64_t *bin_count;           // [nbins]
  double *bin_sum, *bin_sum2;
  int64_t *loc_count;           // [W][nbins]
  double *loc_sum, *loc_sum2;
  // --- smooth PME (pme_on = 0: shifted-force Coulomb, the rest unused)
  int32_t pme_on, pme_order;
  double ewald_beta;
  T ewb, ewc;                   // beta, 2 beta / sqrt(pi) (storage precision)
  const float4 *ewtab;          // [2][EWTAB_N] cubic pieces of the real-space correction in r^2
  float ewtab_inv;              // EWTAB_N / r_cut^2
  const PmeWalker *pme;         // [W]
  const int32_t *pme_bw[3];     // walker of every FFT block along each axis
  double2 *pme_grid;            // [sum K0 K1 K2] complex grid
  const int32_t *pme_brw;       // [bricks] walker of every grid brick
  const int32_t *pme_plw;       // [planes] walker of every y-z plane (NULL: per-axis passes)
  int32_t pme_npl;              // LDS plane capacity of the y-z transform (4096 or 8192)
  int32_t *pme_bcnt;            // [bricks] atoms whose base grid point lies in the brick
  int32_t *pme_blist;           // [bricks][br_cap] their slots
  int64_t pme_nbr;              // bricks in all
  const double *pme_tab;        // [sum (K0+K1+K2)][2] exp(-pi^2 m~^2 / beta^2) |b(m)|^2, m~^2
  const int32_t *pme_perm;      // [sum (K0+K1+K2)] frequency index at each position of a forward transform
  double *pme_frc;              // [3][S] reciprocal force per slot
  double *pme_phi;              // [2][S] reciprocal potential: own group, other group
  double *pme_qs;               // [W][4] Q_E, Q_S, sum_E q^2, sum_S q^2
  // --- export / counting
  int64_t *pair_out;            // [max][2]
  unsigned long long *pair_n;   // [W] counters
  int64_t pair_max;
};

// Index ranges a launch covers (batched: everything; plain: one walker).
struct Range {
  int64_t a0, an;      // atoms
  int64_t c0, cn;      // clusters
  int64_t e0, en;      // environment work-table entries
  int64_t i0, in_;     // alchemical item slots
  int64_t k0, kn;      // per-column entries
  int32_t w0, wn;      // walkers
  int32_t pb0[3], pbn[3];  // PME FFT blocks along each axis
  int32_t pbs[3];          // the first pbs of them: walkers whose grid lengths are powers of two
  int32_t bb0, bbn;        // PME grid bricks
  int32_t pl0, pln;        // PME y-z planes
  int32_t pls;             // the first pls of them: walkers whose grid lengths are powers of two
};

// Host-side launchers (defined in labf_kernels.hip).
template <typename T>
struct Launch {
  static hipError_t rebuild(const Dev<T> &d, const Range &r, int xb, int vb, int check_disp,
                            hipStream_t s);
  // xb, vb: position/velocity buffers; lb: lambda/step buffer (flips every step)
  static hipError_t step(const Dev<T> &d, const Range &r, int xb, int vb, int lb, hipStream_t s);
  static hipError_t step_alch(const Dev<T> &d, const Range &r, int xb, int vb, int lb,
                              hipStream_t s);
  static hipError_t step_env(const Dev<T> &d, const Range &r, int xb, int vb, int lb,
                             hipStream_t s);
  // PME stepping: reciprocal force + BAOAB of the environment atoms after
  // step_env (which then only writes forces) and pme()
  static hipError_t env_integrate(const Dev<T> &d, const Range &r, int xb, int vb, int lb,
                                  hipStream_t s);
  // pruned pair lists of the environment clusters, refreshed where stale
  // (before every environment launch)
  static hipError_t prune(const Dev<T> &d, const Range &r, int xb, int lb, hipStream_t s);
  // mode: EVAL_ALL, EVAL_ENERGY or EVAL_GRAD (what an evaluation computes)
  static hipError_t eval(const Dev<T> &d, const Range &r, int xb, int vb, int lb, int mode,
                         hipStream_t s);
  static hipError_t export_pairs(const Dev<T> &d, const Range &r, int xb, int mode,
                                 hipStream_t s);
  static hipError_t init_velocities(const Dev<T> &d, int vb, hipStream_t s);
  static hipError_t gather_atoms(const Dev<T> &d, int xb, int vb, double *pos, double *vel,
                                 hipStream_t s);
  static hipError_t scatter_atoms(const Dev<T> &d, int xb, int vb, const double *pos,
                                  const double *vel, hipStream_t s);
  static hipError_t gather_forces(const Dev<T> &d, double *f, hipStream_t s);
  // differentiable energy: replace positions (caller order, unrounded),
  // lambda and solute (eps, sigma, q) from device arrays (each may be NULL)
  static hipError_t set_config(const Dev<T> &d, int xb, int lb, const double *pos,
                               const double *lam, const double *params, hipStream_t s);
  // reciprocal-space PME: spread, transforms and convolution, gather
  static hipError_t pme(const Dev<T> &d, const Range &r, int xb, int lb, hipStream_t s);
  // per-walker charge sums of the two groups (after a charge change)
  static hipError_t pme_charges(const Dev<T> &d, hipStream_t s);
  // influence-function and real-space correction tables (once, at creation)
  static hipError_t pme_tables(const Dev<T> &d, float4 *ewtab, hipStream_t s);
  // total potential energy per walker after eval()
  static hipError_t energy_total(const Dev<T> &d, double *out, hipStream_t s);
  // upstream gradient g[W] times the derivatives of the last eval()
  static hipError_t energy_grads(const Dev<T> &d, const double *g, double *gpos, double *glam,
                                 double *gpar, hipStream_t s);
};

// lam0 / p0: device arrays [W]; p0 may be NULL (Maxwell-Boltzmann draw).
template <typename T>
hipError_t launch_init_lambda(const Dev<T> &d, const double *lam0, const double *p0, int lb,
                              hipStream_t s);

hipError_t launch_philox(int64_t n, const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t s);

}  // namespace labf
