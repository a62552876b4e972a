/*
 * labf_oracle.h -- plain FP64 CPU oracle of the lambda-ABF alchemical
 * nonbonded step (Lagardere, Maurin, Adjoua, El Hage, Monmarche, Piquemal,
 * Henin: "Lambda-ABF: Simplified, Portable, Accurate, and Cost-effective
 * Alchemical Free Energy Computation").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test suite, by the
 * package smoke check and by the CPU-baseline leg of the benchmark.  The GPU
 * product path never links, loads or calls it, and it shares no code, header,
 * table or helper with the HIP path.
 *
 * Every routine is written for clarity, not speed: FP64 throughout, no
 * blocking, no fusion, no reordering beyond what the definitions state.
 */
#ifndef LABF_ORACLE_H
#define LABF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Static description of a batch of walkers plus the lambda/ABF parameters.
 * Arrays are indexed by the global atom index; walker w owns atoms
 * [atom_offset[w], atom_offset[w+1]).  Box edges are per walker. */
typedef struct orc_sys {
  int32_t n_walkers;
  int32_t pad0;
  const int64_t *atom_offset;   /* [W+1]                                   */
  const double *box;            /* [W][3] orthorhombic edges               */
  const double *mass;           /* [N]                                     */
  const double *charge;         /* [N]                                     */
  const double *sigma;          /* [N]                                     */
  const double *epsilon;        /* [N]                                     */
  const uint8_t *is_solute;     /* [N] 1 = alchemical group                */
  const double *anchor;         /* [N][3] restraint anchors or NULL        */
  const double *k0;             /* [N] restraint k at lambda=0 or NULL     */
  const double *k1;             /* [N] restraint k at lambda=1 or NULL     */
  double r_cut, r_skin, kT, gamma, dt, coulomb_k, accel_unit;
  uint64_t seed;
  /* lambda dynamics and ABF */
  double m_lambda, gamma_lambda, kT_lambda;
  double elec_start, elec_end, vdw_start, vdw_end;
  int32_t direction;            /* 0 = decoupling (c = 1 - ramp), 1 = coupling (c = ramp) */
  int32_t sc_power;             /* soft-core exponent p                    */
  double sc_alpha;              /* soft-core alpha                         */
  int32_t n_bins;
  int32_t share_interval;       /* K: walkers merge their ABF deltas every K steps */
  double lam_lo, lam_hi;
  int64_t full_samples;
  int32_t fixed_lambda;         /* 1: lambda frozen (fixed-lambda TI)      */
  int32_t abf_on;               /* 0: no samples and no bias               */
  int32_t sc_form;              /* 0: alpha (1-c)^p + (r/sig)^6 in the denominator;
                                   1: separation-shifted, r^2 -> r^2 + delta (1-c) */
  int32_t pad1;
  double sc_shift;              /* delta of the separation-shifted form (length^2) */
  /* lambda-dependent distance restraint between two atoms of each walker:
   * V = k/2 (d - d_min)^2 for d < d_min(lambda), 0 otherwise, with
   * d_min = (delta/2)(1 - cos(2 pi n lambda)); NULL pairs: none */
  const int32_t *dr_pairs;      /* [W][2] walker-local atom indices or NULL */
  double dr_delta, dr_k;
  int32_t dr_freq;              /* n (1: the text's form; 2: lambda doubled) */
  int32_t pme_on;               /* 1: Ewald electrostatics (smooth PME) instead of shifted force */
  const int32_t *pme_dims;      /* [W][3] PME grid points per edge (2^a 3^b 5^c) */
  double ewald_beta;            /* Ewald splitting parameter (1/length)    */
  int32_t pme_order;            /* B-spline order (4, 6 or 8)              */
  int32_t pad3;
} orc_sys;

/* Exact Ewald sum of point charges in an orthorhombic box (tests): real
 * space over all images within r_real, reciprocal space over all
 * |m_k| <= kmax, self and neutralising-background terms; energy and forces
 * (f may be NULL).  Units: coulomb_k q_i q_j / r. */
double orc_ewald_exact(int64_t n, const double *x, const double *q, const double *L, double beta,
                       double r_real, int32_t kmax, double coulomb_k, double *f);
/* Smooth PME reciprocal energy of one charge set (tests): order p,
 * grid K[3] (any sizes), forces added to f (may be NULL). */
double orc_spme_energy(int64_t n, const double *x, const double *q, const double *L, double beta,
                       const int32_t K[3], int32_t p, double coulomb_k, double *f);

/* d_min(lambda) and its derivative for the distance restraint. */
void orc_dmin(const orc_sys *s, double lam, double out[2]);

/* Dynamic state.  x, v: [N][3]; per-walker arrays: [W]; bins: [nbins];
 * local (not yet shared) ABF deltas: [W][nbins].  `pending` = 1 when the
 * closing half-kick of the previous step has not been applied yet. */
typedef struct orc_state {
  double *x, *v, *f;
  double *lambda, *p_lambda, *dudl, *bias;
  int64_t *bin_count;
  double *bin_sum, *bin_sum2;
  int64_t *loc_count;
  double *loc_sum, *loc_sum2;
  uint32_t *status;
  int64_t step;
  int32_t pending;
  int32_t pad0;
} orc_state;

/* Energy decomposition written by orc_evaluate (5 entries). */
enum { ORC_U_ENV = 0, ORC_U_SOLUTE = 1, ORC_U_ALCH_LJ = 2, ORC_U_ALCH_C = 3, ORC_U_RESTR = 4 };

void orc_schedule(const orc_sys *s, double lam, double out[4]);
void orc_pair_terms(double r, double sig, double eps, double qq, double cv, double ce,
                    double alpha, int32_t p, double r_cut, int32_t shift, double out[6]);
void orc_pair_terms_shifted(double r, double sig, double eps, double qq, double cv, double ce,
                            double delta, double r_cut, int32_t shift, double out[6]);
int64_t orc_neighbor_pairs(const orc_sys *s, int32_t w, const double *x, double r_list,
                           int32_t brute, int64_t max_pairs, int64_t *pairs);
int32_t orc_evaluate(const orc_sys *s, int32_t w, const double *x, double lam,
                     int32_t brute, double *f, double *u_parts, double *dudl);
int32_t orc_param_grad(const orc_sys *s, int32_t w, const double *x, double lam, double *g);
/* fs[n]: per atom, the sum of the magnitudes of its force terms (pairs,
 * reciprocal space, restraints): the scale of per-atom force errors. */
int32_t orc_force_scale(const orc_sys *s, int32_t w, const double *x, double lam, double *fs);
/* ABF bias force on lambda of walker w at lambda (bin of lambda): the ramp
 * min(1, n/fullSamples) times the bin mean, over the shared accumulator plus
 * the walker's own unshared samples; 0 for an empty bin. */
double orc_abf_bias(const orc_sys *s, const orc_state *st, int32_t w, double lam);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_normals(uint64_t seed, uint32_t atom, uint32_t step, uint32_t walker,
                 uint32_t purpose, double out[4]);
int32_t orc_init_velocities(const orc_sys *s, orc_state *st);
int32_t orc_run(const orc_sys *s, orc_state *st, int64_t n_steps, int32_t brute);
int32_t orc_full_step(const orc_sys *s, const orc_state *st, double *v_full, double *p_full);
int32_t orc_abf_readout(int32_t n_bins, double lo, double hi, const int64_t *count,
                        const double *sum, double *grad, double *profile, double *delta_a);
int32_t orc_bin_of(const orc_sys *s, double lam);

#ifdef __cplusplus
}
#endif
#endif
