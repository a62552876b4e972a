/*
 * labf_oracle.c -- plain FP64 CPU oracle of the lambda-ABF alchemical
 * nonbonded step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, by the package smoke check
 * and by the CPU-baseline leg of the benchmark; never by the product path.
 * It shares no code with the HIP path.
 *
 * What it computes, in the paper's order (section and equation names refer
 * to the lambda-ABF paper):
 *   - the alchemical schedule lambda -> (lambda_e, lambda_v), Implementation,
 *     "Alchemical pathway" (Tinker-HP convention b_v, b_e; NAMD staggered
 *     decoupling convention), and the SI lambda-schedule table;
 *   - the lambda-dependent potential V(q; lambda) of the Theory section,
 *     Eq. (lambdadyn-Hamiltonian), with soft-core Lennard-Jones (NAMD
 *     paragraph of "Alchemical pathway") and cutoff shifted-force Coulomb
 *     linearly scaled by lambda_e (same paragraph; cutoff electrostatics
 *     replaces PME here), decoupling (solute-solute terms kept at full
 *     strength);
 *   - lambda-switched harmonic restraints k(lambda) = k0 + lambda (k1 - k0)
 *     (restraint release in "Binding restraints");
 *   - Langevin dynamics of atoms and of the extended lambda coordinate,
 *     Eq. (lambdadyn-Langevin-process) with the ABF term of Eq. (lambda-abf),
 *     reflecting lambda boundaries, integrated by BAOAB (SI "Setup used for
 *     numerical results"; BAOA for lambda in "Software interface");
 *   - multiple-walker ABF on lambda: bin-averaged dV/dlambda as A'_t, linear
 *     ramp up to fullSamples ("ABF parameters"), walkers sharing their
 *     estimates every K steps ("Orthogonal space sampling");
 *   - the Riemann-sum readout of A(lambda) from the bin averages ("Adaptive
 *     Biasing Force using lambda as a collective variable").
 * Readings of points the paper leaves open are listed in the design notes
 * of the repository; each is restated where it is used below.
 */
#include "labf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ST_NONFINITE 1u
#define ORC_ST_REFLECT 2u

static inline double sq(double a) { return a * a; }

/* ---------------------------------------------------------------------------
 * Alchemical schedule ("Alchemical pathway"): each channel x in {e, v} has a
 * piecewise-linear ramp m_x(lambda) = clip((lambda - s_x)/(e_x - s_x), 0, 1).
 * Coupling direction (Tinker-HP): c_x = m_x.  Decoupling direction (NAMD):
 * c_x = 1 - m_x.  The derivative dc_x/dlambda is +-1/(e_x - s_x) on
 * [s_x, e_x) and also at lambda = e_x = hi (left derivative at the upper
 * end); zero elsewhere.
 * out = {c_e, c_v, dc_e/dlambda, dc_v/dlambda}.
 * ------------------------------------------------------------------------- */
static void channel(double lam, double s0, double s1, int coupling, double hi,
                    double *c, double *dc) {
  double m, dm;
  double w = s1 - s0;
  if (lam <= s0) {
    m = 0.0;
  } else if (lam >= s1) {
    m = 1.0;
  } else {
    m = (lam - s0) / w;
  }
  if ((lam >= s0 && lam < s1) || (lam == s1 && s1 == hi)) {
    dm = 1.0 / w;
  } else {
    dm = 0.0;
  }
  if (coupling) {
    *c = m;
    *dc = dm;
  } else {
    *c = 1.0 - m;
    *dc = -dm;
  }
}

void orc_schedule(const orc_sys *s, double lam, double out[4]) {
  double ce, dce, cv, dcv;
  channel(lam, s->elec_start, s->elec_end, s->direction == 1, s->lam_hi, &ce, &dce);
  channel(lam, s->vdw_start, s->vdw_end, s->direction == 1, s->lam_hi, &cv, &dcv);
  out[0] = ce;
  out[1] = cv;
  out[2] = dce;
  out[3] = dcv;
}

/* ---------------------------------------------------------------------------
 * Pair terms at separation r, for a pair with mixed parameters (sig, eps),
 * charge product qq (coulomb constant included) and channel couplings
 * (cv, ce).
 *
 * Soft-core LJ (Beutler form, alpha, p):
 *   s(r, c)   = 1 / (alpha (1-c)^p + (r/sig)^6)
 *   phi(r, c) = 4 eps c (s^2 - s)
 *   U_LJ      = phi(r, c) - phi(r_cut, c)        (shift at the same c)
 *   dU_LJ/dc  = psi(r) - psi(r_cut),
 *   psi       = 4 eps [(s^2 - s) + c alpha p (1-c)^(p-1) (2s - 1) s^2]
 *   F/r       = 24 eps c (2s - 1) s^2 (r/sig)^6 / r^2   (repulsive > 0)
 * Shifted-force Coulomb, linear in c_e:
 *   g(r)      = 1/r - 1/r_cut + (r - r_cut)/r_cut^2
 *   U_C       = ce qq g(r);  dU_C/dce = qq g(r)
 *   F/r       = ce qq (1/r^2 - 1/r_cut^2) / r
 * With shift = 0 the LJ potential shift is omitted (used by unit tests).
 * out = {U_LJ, dU_LJ/dc_v, (F/r)_LJ, U_C, dU_C/dc_e, (F/r)_C}.
 * ------------------------------------------------------------------------- */
static double sc_s(double r, double sig, double c, double alpha, int p) {
  double u = pow(r / sig, 6.0);
  return 1.0 / (alpha * pow(1.0 - c, (double)p) + u);
}

void orc_pair_terms(double r, double sig, double eps, double qq, double cv, double ce,
                    double alpha, int32_t p, double r_cut, int32_t shift, double out[6]) {
  int k;
  for (k = 0; k < 6; ++k) out[k] = 0.0;
  if (eps != 0.0) {
    double s = sc_s(r, sig, cv, alpha, p);
    double u = pow(r / sig, 6.0);
    double dsc = (p >= 1) ? alpha * (double)p * pow(1.0 - cv, (double)(p - 1)) : 0.0;
    double phi = 4.0 * eps * cv * (s * s - s);
    double psi = 4.0 * eps * ((s * s - s) + cv * dsc * (2.0 * s - 1.0) * s * s);
    out[2] = 24.0 * eps * cv * (2.0 * s - 1.0) * s * s * u / (r * r);
    if (shift) {
      double sc = sc_s(r_cut, sig, cv, alpha, p);
      phi -= 4.0 * eps * cv * (sc * sc - sc);
      psi -= 4.0 * eps * ((sc * sc - sc) + cv * dsc * (2.0 * sc - 1.0) * sc * sc);
    }
    out[0] = phi;
    out[1] = psi;
  }
  if (qq != 0.0) {
    double g = 1.0 / r - 1.0 / r_cut + (r - r_cut) / (r_cut * r_cut);
    out[4] = qq * g;
    if (ce != 0.0) {
      out[3] = ce * qq * g;
      out[5] = ce * qq * (1.0 / (r * r) - 1.0 / (r_cut * r_cut)) / r;
    }
  }
}

/* Separation-shifted soft-core (Zacharias, Straatsma and McCammon 1994;
 * NAMD's alchVdwShiftCoeff): the LJ distance r^2 is replaced by
 * s = r^2 + delta (1 - c) and the whole term is scaled by c,
 *   phi(r, c) = 4 eps c (sig^12 / s^6 - sig^6 / s^3),
 * i.e. c times the plain LJ at the effective distance sqrt(s).  Potential
 * shift at r_cut with the same c.  Coulomb as in orc_pair_terms.
 *   (F/r)  = -(1/r) dphi/dr = 4 eps c (12 sig^12 / s^7 - 6 sig^6 / s^4)
 *   dphi/dc = 4 eps (sig^12/s^6 - sig^6/s^3) + 4 eps c delta (6 sig^12/s^7 - 3 sig^6/s^4) */
static void shifted_lj(double r, double sig, double eps, double c, double delta, double out[3]) {
  double s = r * r + delta * (1.0 - c);
  double s6 = pow(sig, 6.0), s12 = s6 * s6;
  out[0] = 4.0 * eps * c * (s12 / pow(s, 6.0) - s6 / pow(s, 3.0));
  out[1] = 4.0 * eps * (s12 / pow(s, 6.0) - s6 / pow(s, 3.0)) +
           4.0 * eps * c * delta * (6.0 * s12 / pow(s, 7.0) - 3.0 * s6 / pow(s, 4.0));
  out[2] = 4.0 * eps * c * (12.0 * s12 / pow(s, 7.0) - 6.0 * s6 / pow(s, 4.0));
}

void orc_pair_terms_shifted(double r, double sig, double eps, double qq, double cv, double ce,
                            double delta, double r_cut, int32_t shift, double out[6]) {
  double t[3], tc[3];
  int k;
  orc_pair_terms(r, sig, 0.0, qq, cv, ce, 0.0, 1, r_cut, shift, out); /* Coulomb part */
  if (eps == 0.0) return;
  shifted_lj(r, sig, eps, cv, delta, t);
  if (shift) {
    shifted_lj(r_cut, sig, eps, cv, delta, tc);
    for (k = 0; k < 2; ++k) t[k] -= tc[k];
  }
  out[0] = t[0];
  out[1] = t[1];
  out[2] = t[2];
}

/* ---------------------------------------------------------------------------
 * Ewald electrostatics.  The Ewald split (erfc(beta r)/r pairs in real
 * space, Gaussian-screened charges in reciprocal space, minus the self
 * interaction, minus a neutralising background for a net charge) and its
 * smooth particle-mesh evaluation (Essmann, Perera, Berkowitz, Darden,
 * Lee, Pedersen 1995): charges spread on a K0 x K1 x K2 grid with cardinal
 * B-splines of order p, FFT, influence function
 *   G(m) = kC exp(-pi^2 |m~|^2 / beta^2) / (pi V |m~|^2) |b0(m0)|^2 |b1(m1)|^2 |b2(m2)|^2,
 * m~_a = m_a / L_a (m_a wrapped to [-K_a/2, K_a/2)), the grid potential
 * phi(k) = sum_m G(m) F(m) exp(+2 pi i m.k/K), energy 1/2 sum_k Q(k) phi(k),
 * force -q_i sum_k dW_i(k)/dx phi(k).
 * ------------------------------------------------------------------------- */
static const double ORC_PI = 3.14159265358979323846;

/* direct DFT of n points spaced by stride (any n): X_k = sum_j x_j exp(sign 2 pi i j k / n) */
static void dft1(double *re, double *im, int n, int64_t stride, int sign) {
  double *xr = (double *)malloc(sizeof(double) * n), *xi = (double *)malloc(sizeof(double) * n);
  int j, k;
  for (j = 0; j < n; ++j) {
    xr[j] = re[j * stride];
    xi[j] = im[j * stride];
  }
  for (k = 0; k < n; ++k) {
    double sr = 0.0, si = 0.0;
    for (j = 0; j < n; ++j) {
      /* (j k) mod n keeps the angle small and exact in the integer part */
      const double a = sign * 2.0 * ORC_PI * (double)((int64_t)j * k % n) / n;
      sr += xr[j] * cos(a) - xi[j] * sin(a);
      si += xr[j] * sin(a) + xi[j] * cos(a);
    }
    re[k * stride] = sr;
    im[k * stride] = si;
  }
  free(xr);
  free(xi);
}

/* in-place complex DFT of n points spaced by stride; sign -1: forward
 * (exp(-2 pi i j k / n)), +1: inverse without the 1/n factor.  Radix-2
 * Cooley-Tukey when n is a power of two, the direct sum otherwise. */
static void fft1(double *re, double *im, int n, int64_t stride, int sign) {
  if (n & (n - 1)) {
    dft1(re, im, n, stride, sign);
    return;
  }
  int i, j = 0, k, len;
  for (i = 1; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double t = re[i * stride];
      re[i * stride] = re[j * stride];
      re[j * stride] = t;
      t = im[i * stride];
      im[i * stride] = im[j * stride];
      im[j * stride] = t;
    }
  }
  for (len = 2; len <= n; len <<= 1) {
    double ang = sign * 2.0 * ORC_PI / len;
    for (i = 0; i < n; i += len)
      for (k = 0; k < len / 2; ++k) {
        double wr = cos(ang * k), wi = sin(ang * k);
        int64_t a = (int64_t)(i + k) * stride, b = (int64_t)(i + k + len / 2) * stride;
        double vr = re[b] * wr - im[b] * wi, vi = re[b] * wi + im[b] * wr;
        double ur = re[a], ui = im[a];
        re[a] = ur + vr;
        im[a] = ui + vi;
        re[b] = ur - vr;
        im[b] = ui - vi;
      }
  }
}

/* 3-D FFT of an array indexed (i K1 + j) K2 + k */
static void fft3(double *re, double *im, const int32_t K[3], int sign) {
  int64_t i, j;
  for (i = 0; i < K[0]; ++i)
    for (j = 0; j < K[1]; ++j) fft1(re + (i * K[1] + j) * K[2], im + (i * K[1] + j) * K[2], K[2], 1, sign);
  for (i = 0; i < K[0]; ++i)
    for (j = 0; j < K[2]; ++j) fft1(re + i * K[1] * K[2] + j, im + i * K[1] * K[2] + j, K[1], K[2], sign);
  for (i = 0; i < K[1]; ++i)
    for (j = 0; j < K[2]; ++j) fft1(re + i * K[2] + j, im + i * K[2] + j, K[0], (int64_t)K[1] * K[2], sign);
}

/* cardinal B-spline M_p(u) (support (0, p)) and its derivative */
static double bspline(double u, int p) {
  if (u <= 0.0 || u >= (double)p) return 0.0;
  if (p == 2) return 1.0 - fabs(u - 1.0);
  return (u * bspline(u, p - 1) + ((double)p - u) * bspline(u - 1.0, p - 1)) / (double)(p - 1);
}
static double dbspline(double u, int p) { return bspline(u, p - 1) - bspline(u - 1.0, p - 1); }

/* |b(m)|^2 of one axis: 1 / |sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m k / K)|^2 (p even) */
static double bmod2(int m, int K, int p) {
  double sr = 0.0, si = 0.0;
  int k;
  for (k = 0; k <= p - 2; ++k) {
    double a = 2.0 * ORC_PI * (double)m * (double)k / (double)K, M = bspline((double)(k + 1), p);
    sr += M * cos(a);
    si += M * sin(a);
  }
  return 1.0 / (sr * sr + si * si);
}

/* spline weights of one atom: grid indices idx[a][j] and weights
 * w[a][j], dw[a][j] (d/du) for j = 0..p-1 on each axis a */
static void spline_weights(const double *x, const double *L, const int32_t K[3], int p, int idx[3][8],
                           double w[3][8], double dw[3][8]) {
  int a, j;
  for (a = 0; a < 3; ++a) {
    double f = x[a] / L[a];
    double u, fr;
    int k0;
    f -= floor(f);
    u = f * K[a];
    k0 = (int)floor(u);
    fr = u - k0;
    for (j = 0; j < p; ++j) {
      int k = k0 - j;
      idx[a][j] = ((k % K[a]) + K[a]) % K[a];
      w[a][j] = bspline(fr + j, p);
      dw[a][j] = dbspline(fr + j, p);
    }
  }
}

/* influence function on the grid (index as the data) */
static void influence(const double *L, const int32_t K[3], int p, double beta, double coulomb_k, double *G) {
  double V = L[0] * L[1] * L[2];
  int i, j, k;
  for (i = 0; i < K[0]; ++i)
    for (j = 0; j < K[1]; ++j)
      for (k = 0; k < K[2]; ++k) {
        int m0 = i < K[0] / 2 ? i : i - K[0], m1 = j < K[1] / 2 ? j : j - K[1], m2 = k < K[2] / 2 ? k : k - K[2];
        double a0 = m0 / L[0], a1 = m1 / L[1], a2 = m2 / L[2];
        double m2n = a0 * a0 + a1 * a1 + a2 * a2;
        int64_t t = ((int64_t)i * K[1] + j) * K[2] + k;
        if (m2n == 0.0) {
          G[t] = 0.0;
          continue;
        }
        G[t] = coulomb_k * exp(-ORC_PI * ORC_PI * m2n / (beta * beta)) / (ORC_PI * V * m2n) *
               bmod2(i, K[0], p) * bmod2(j, K[1], p) * bmod2(k, K[2], p);
      }
}

/* grid potential phi of charges q (mask: atoms with sel[i] == want, NULL: all) */
static void spme_potential(int64_t n, const double *x, const double *q, const uint8_t *sel, int want,
                           const double *L, const int32_t K[3], int p, const double *G, double *phi,
                           double *work_im) {
  int64_t N = (int64_t)K[0] * K[1] * K[2], i, t;
  int idx[3][8];
  double w[3][8], dw[3][8];
  int a, b, c;
  memset(phi, 0, sizeof(double) * N);
  memset(work_im, 0, sizeof(double) * N);
  for (i = 0; i < n; ++i) {
    if (sel && (sel[i] != 0) != want) continue;
    if (q[i] == 0.0) continue;
    spline_weights(x + 3 * i, L, K, p, idx, w, dw);
    for (a = 0; a < p; ++a)
      for (b = 0; b < p; ++b)
        for (c = 0; c < p; ++c)
          phi[((int64_t)idx[0][a] * K[1] + idx[1][b]) * K[2] + idx[2][c]] += q[i] * w[0][a] * w[1][b] * w[2][c];
  }
  fft3(phi, work_im, K, -1);
  for (t = 0; t < N; ++t) {
    phi[t] *= G[t];
    work_im[t] *= G[t];
  }
  fft3(phi, work_im, K, +1);
}

/* sum_k W_i(k) phi(k) and its gradient for atom i */
static double spme_interp(const double *xi, const double *L, const int32_t K[3], int p, const double *phi,
                          double grad[3]) {
  int idx[3][8];
  double w[3][8], dw[3][8], v = 0.0;
  int a, b, c;
  spline_weights(xi, L, K, p, idx, w, dw);
  grad[0] = grad[1] = grad[2] = 0.0;
  for (a = 0; a < p; ++a)
    for (b = 0; b < p; ++b)
      for (c = 0; c < p; ++c) {
        double ph = phi[((int64_t)idx[0][a] * K[1] + idx[1][b]) * K[2] + idx[2][c]];
        v += w[0][a] * w[1][b] * w[2][c] * ph;
        grad[0] += dw[0][a] * w[1][b] * w[2][c] * ph * K[0] / L[0];
        grad[1] += w[0][a] * dw[1][b] * w[2][c] * ph * K[1] / L[1];
        grad[2] += w[0][a] * w[1][b] * dw[2][c] * ph * K[2] / L[2];
      }
  return v;
}

double orc_spme_energy(int64_t n, const double *x, const double *q, const double *L, double beta,
                       const int32_t K[3], int32_t p, double coulomb_k, double *f) {
  int64_t N = (int64_t)K[0] * K[1] * K[2], i;
  double *G = (double *)malloc(sizeof(double) * N), *phi = (double *)malloc(sizeof(double) * N),
         *im = (double *)malloc(sizeof(double) * N);
  double e = 0.0, g[3];
  influence(L, K, p, beta, coulomb_k, G);
  spme_potential(n, x, q, NULL, 0, L, K, p, G, phi, im);
  for (i = 0; i < n; ++i) {
    double v = spme_interp(x + 3 * i, L, K, p, phi, g);
    e += 0.5 * q[i] * v;
    if (f) {
      f[3 * i] -= q[i] * g[0];
      f[3 * i + 1] -= q[i] * g[1];
      f[3 * i + 2] -= q[i] * g[2];
    }
  }
  free(G);
  free(phi);
  free(im);
  return e;
}

double orc_ewald_exact(int64_t n, const double *x, const double *q, const double *L, double beta,
                       double r_real, int32_t kmax, double coulomb_k, double *f) {
  double V = L[0] * L[1] * L[2], e = 0.0, Q = 0.0;
  int64_t i, j;
  int nx[3], a, b, c;
  for (a = 0; a < 3; ++a) nx[a] = (int)ceil(r_real / L[a]);
  /* real space: all images within r_real */
  for (i = 0; i < n; ++i)
    for (j = 0; j < n; ++j)
      for (a = -nx[0]; a <= nx[0]; ++a)
        for (b = -nx[1]; b <= nx[1]; ++b)
          for (c = -nx[2]; c <= nx[2]; ++c) {
            double d[3], r2, r, fr;
            if (i == j && a == 0 && b == 0 && c == 0) continue;
            d[0] = x[3 * j] + a * L[0] - x[3 * i];
            d[1] = x[3 * j + 1] + b * L[1] - x[3 * i + 1];
            d[2] = x[3 * j + 2] + c * L[2] - x[3 * i + 2];
            r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < r_real * r_real)) continue;
            r = sqrt(r2);
            e += 0.5 * coulomb_k * q[i] * q[j] * erfc(beta * r) / r;
            if (f) {
              fr = coulomb_k * q[i] * q[j] * (erfc(beta * r) / r + 2.0 * beta / sqrt(ORC_PI) * exp(-beta * beta * r2)) / r2;
              f[3 * i] -= fr * d[0];
              f[3 * i + 1] -= fr * d[1];
              f[3 * i + 2] -= fr * d[2];
            }
          }
  /* reciprocal space */
  for (a = -kmax; a <= kmax; ++a)
    for (b = -kmax; b <= kmax; ++b)
      for (c = -kmax; c <= kmax; ++c) {
        double m[3], m2n, A, sr = 0.0, si = 0.0;
        if (a == 0 && b == 0 && c == 0) continue;
        m[0] = a / L[0];
        m[1] = b / L[1];
        m[2] = c / L[2];
        m2n = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
        A = exp(-ORC_PI * ORC_PI * m2n / (beta * beta)) / m2n;
        for (j = 0; j < n; ++j) {
          double ph = 2.0 * ORC_PI * (m[0] * x[3 * j] + m[1] * x[3 * j + 1] + m[2] * x[3 * j + 2]);
          sr += q[j] * cos(ph);
          si += q[j] * sin(ph);
        }
        e += coulomb_k / (2.0 * ORC_PI * V) * A * (sr * sr + si * si);
        if (f)
          for (i = 0; i < n; ++i) {
            double ph = 2.0 * ORC_PI * (m[0] * x[3 * i] + m[1] * x[3 * i + 1] + m[2] * x[3 * i + 2]);
            /* Im[conj(S) exp(2 pi i m.r_i)] */
            double s = sr * sin(ph) - si * cos(ph);
            int k;
            for (k = 0; k < 3; ++k) f[3 * i + k] += coulomb_k * 2.0 * q[i] / V * A * m[k] * s;
          }
      }
  for (i = 0; i < n; ++i) {
    e -= coulomb_k * beta / sqrt(ORC_PI) * q[i] * q[i];
    Q += q[i];
  }
  e -= coulomb_k * ORC_PI * Q * Q / (2.0 * V * beta * beta);
  return e;
}

/* ---------------------------------------------------------------------------
 * Minimum-image separation d = x_j - x_i (the neighbour-set definition):
 * d_k -= L_k * rint(d_k * (1/L_k)), 1/L_k evaluated once in FP64, rint is
 * round-half-even; r^2 = (dx*dx + dy*dy) + dz*dz with no fused operations
 * (this file is compiled with -ffp-contract=off).
 * ------------------------------------------------------------------------- */
static double min_image(const double *xi, const double *xj, const double *L,
                        const double *invL, double d[3]) {
  int k;
  for (k = 0; k < 3; ++k) {
    double dk = xj[k] - xi[k];
    dk -= L[k] * rint(dk * invL[k]);
    d[k] = dk;
  }
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* ---------------------------------------------------------------------------
 * Neighbour set: all pairs (i < j) of walker w with r^2 < r_list^2 under the
 * minimum-image separation above.  brute = 1 tests every pair; brute = 0
 * uses a cell list with n_c = floor(L / r_list) >= 3 cells per edge (falls
 * back to brute force when any edge has fewer than 3 cells).  Pairs are
 * written as walker-local indices (i, j), sorted lexicographically.
 * Returns the number of pairs (which may exceed max_pairs; only the first
 * max_pairs are stored) or -1 on an invalid request.
 * ------------------------------------------------------------------------- */
static int cmp_pair(const void *a, const void *b) {
  const int64_t *pa = (const int64_t *)a, *pb = (const int64_t *)b;
  if (pa[0] != pb[0]) return pa[0] < pb[0] ? -1 : 1;
  if (pa[1] != pb[1]) return pa[1] < pb[1] ? -1 : 1;
  return 0;
}

typedef struct {
  int nc[3];
  int64_t *head; /* first atom of each cell, -1 terminated lists */
  int64_t *next;
} cells_t;

static int cells_build(cells_t *c, const double *x, int64_t n, const double *L, double r) {
  int k;
  int64_t i, ncell;
  for (k = 0; k < 3; ++k) {
    int m = (int)floor(L[k] / r);
    while (m > 0 && L[k] / (double)m < r * (1.0 + 1e-12)) --m;
    c->nc[k] = m;
    if (m < 3) return 0;
  }
  ncell = (int64_t)c->nc[0] * c->nc[1] * c->nc[2];
  c->head = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
  c->next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (i = 0; i < ncell; ++i) c->head[i] = -1;
  /* insert in decreasing index order so each cell lists atoms ascending */
  for (i = n - 1; i >= 0; --i) {
    int ci[3];
    int64_t id;
    for (k = 0; k < 3; ++k) {
      double f = x[3 * i + k] / L[k];
      f -= floor(f);
      ci[k] = (int)floor(f * c->nc[k]);
      if (ci[k] >= c->nc[k]) ci[k] = c->nc[k] - 1;
      if (ci[k] < 0) ci[k] = 0;
    }
    id = ((int64_t)ci[0] * c->nc[1] + ci[1]) * c->nc[2] + ci[2];
    c->next[i] = c->head[id];
    c->head[id] = i;
  }
  return 1;
}

static void cells_free(cells_t *c) {
  free(c->head);
  free(c->next);
}

/* Calls visit(i, j, d, r2) once for every unordered pair (i < j) with
 * r2 < rmax^2.  Uses the cell list when possible. */
typedef void (*visit_fn)(void *ctx, int64_t i, int64_t j, const double d[3], double r2);

static void for_each_pair(const double *x, int64_t n, const double *L, double rmax,
                          int brute, visit_fn visit, void *ctx) {
  double invL[3];
  double r2max = rmax * rmax;
  int k;
  cells_t c;
  for (k = 0; k < 3; ++k) invL[k] = 1.0 / L[k];
  /* tiny walkers: scanning mostly empty cells costs more than all pairs */
  if (!brute) {
    double ncell = 1.0;
    for (k = 0; k < 3; ++k) ncell *= floor(L[k] / rmax);
    if ((double)n * (double)n < 27.0 * ncell) brute = 1;
  }
  if (!brute && cells_build(&c, x, n, L, rmax)) {
    int a, b, e;
    for (a = 0; a < c.nc[0]; ++a)
      for (b = 0; b < c.nc[1]; ++b)
        for (e = 0; e < c.nc[2]; ++e) {
          int64_t id = ((int64_t)a * c.nc[1] + b) * c.nc[2] + e;
          int da, db, de;
          /* the 27 neighbouring cells, each visited once (n_c >= 3) */
          for (da = -1; da <= 1; ++da)
            for (db = -1; db <= 1; ++db)
              for (de = -1; de <= 1; ++de) {
                int a2 = (a + da + c.nc[0]) % c.nc[0];
                int b2 = (b + db + c.nc[1]) % c.nc[1];
                int e2 = (e + de + c.nc[2]) % c.nc[2];
                int64_t id2 = ((int64_t)a2 * c.nc[1] + b2) * c.nc[2] + e2;
                int64_t i, j;
                for (i = c.head[id]; i >= 0; i = c.next[i])
                  for (j = c.head[id2]; j >= 0; j = c.next[j]) {
                    double d[3], r2;
                    if (j <= i) continue;
                    r2 = min_image(x + 3 * i, x + 3 * j, L, invL, d);
                    if (r2 < r2max) visit(ctx, i, j, d, r2);
                  }
              }
        }
    cells_free(&c);
  } else {
    int64_t i, j;
    for (i = 0; i < n; ++i)
      for (j = i + 1; j < n; ++j) {
        double d[3];
        double r2 = min_image(x + 3 * i, x + 3 * j, L, invL, d);
        if (r2 < r2max) visit(ctx, i, j, d, r2);
      }
  }
}

/* The same pairs as for_each_pair with a cell list, with the cell columns
 * (a, b) as independent chunks: visit(ctxs[a * nc[1] + b], ...) for every
 * pair whose first atom's cell lies in column (a, b), columns in parallel
 * (OpenMP).  Returns 0 without visiting anything if the box has fewer than
 * 3 cells per edge.  With one context per column, merged afterwards in
 * column order, the sums do not depend on the number of threads. */
static int cell_dims(const double *L, double r, int nc[3]) {
  int k;
  for (k = 0; k < 3; ++k) {
    int m = (int)floor(L[k] / r);
    while (m > 0 && L[k] / (double)m < r * (1.0 + 1e-12)) --m;
    nc[k] = m;
    if (m < 3) return 0;
  }
  return 1;
}

static int for_each_pair_columns(const double *x, int64_t n, const double *L, double rmax,
                                 visit_fn visit, void **ctxs) {
  double invL[3];
  double r2max = rmax * rmax;
  int k, col, ncol;
  cells_t c;
  for (k = 0; k < 3; ++k) invL[k] = 1.0 / L[k];
  if (!cells_build(&c, x, n, L, rmax)) return 0;
  ncol = c.nc[0] * c.nc[1];
#pragma omp parallel for schedule(dynamic, 1)
  for (col = 0; col < ncol; ++col) {
    int a = col / c.nc[1], b = col % c.nc[1], e;
    for (e = 0; e < c.nc[2]; ++e) {
      int64_t id = ((int64_t)a * c.nc[1] + b) * c.nc[2] + e;
      int da, db, de;
      for (da = -1; da <= 1; ++da)
        for (db = -1; db <= 1; ++db)
          for (de = -1; de <= 1; ++de) {
            int a2 = (a + da + c.nc[0]) % c.nc[0];
            int b2 = (b + db + c.nc[1]) % c.nc[1];
            int e2 = (e + de + c.nc[2]) % c.nc[2];
            int64_t id2 = ((int64_t)a2 * c.nc[1] + b2) * c.nc[2] + e2;
            int64_t i, j;
            for (i = c.head[id]; i >= 0; i = c.next[i])
              for (j = c.head[id2]; j >= 0; j = c.next[j]) {
                double d[3], r2;
                if (j <= i) continue;
                r2 = min_image(x + 3 * i, x + 3 * j, L, invL, d);
                if (r2 < r2max) visit(ctxs[col], i, j, d, r2);
              }
          }
    }
  }
  cells_free(&c);
  return 1;
}

typedef struct {
  int64_t count, max;
  int64_t *pairs;
} pair_ctx;

static void collect_pair(void *vctx, int64_t i, int64_t j, const double d[3], double r2) {
  pair_ctx *p = (pair_ctx *)vctx;
  (void)d;
  (void)r2;
  if (p->count < p->max) {
    p->pairs[2 * p->count] = i;
    p->pairs[2 * p->count + 1] = j;
  }
  p->count++;
}

int64_t orc_neighbor_pairs(const orc_sys *s, int32_t w, const double *x, double r_list,
                           int32_t brute, int64_t max_pairs, int64_t *pairs) {
  pair_ctx ctx;
  int64_t n;
  const double *L;
  int k;
  if (w < 0 || w >= s->n_walkers) return -1;
  L = s->box + 3 * w;
  for (k = 0; k < 3; ++k)
    if (!(r_list < 0.5 * L[k])) return -1;
  n = s->atom_offset[w + 1] - s->atom_offset[w];
  ctx.count = 0;
  ctx.max = max_pairs;
  ctx.pairs = pairs;
  for_each_pair(x, n, L, r_list, brute, collect_pair, &ctx);
  if (ctx.count <= max_pairs) qsort(pairs, (size_t)ctx.count, 2 * sizeof(int64_t), cmp_pair);
  return ctx.count;
}

/* ---------------------------------------------------------------------------
 * Potential, forces and dU/dlambda of one walker at (x, lambda).
 * Pair classes: alchemical iff exactly one atom is solute (decoupling:
 * solute-solute and environment-environment pairs use c = 1).  Mixing is
 * Lorentz-Berthelot.  Restraints: U = 1/2 k(lambda) |x - anchor|^2 with
 * minimum image, dU/dlambda = 1/2 (k1 - k0) |x - anchor|^2.
 * f: [n_w][3] forces (may be NULL); u_parts: [5]; dudl: scalar.
 * ------------------------------------------------------------------------- */
typedef struct {
  const orc_sys *s;
  int64_t base;
  double ce, cv, dce, dcv;
  double *f;
  double u[5];
  double dudl;
  /* optional parameter gradient: [n][3] = dU/d(eps, sigma, q) */
  double *g;
  /* optional per-atom force scale: [n] = sum over the atom's force terms of
   * their magnitudes (pairs: |f_ij|; reciprocal, restraint: |F|) */
  double *fs;
} eval_ctx;

static void eval_pair(void *vctx, int64_t i, int64_t j, const double d[3], double r2) {
  eval_ctx *c = (eval_ctx *)vctx;
  const orc_sys *s = c->s;
  int64_t gi = c->base + i, gj = c->base + j;
  double rc = s->r_cut;
  double r, sig, eps, qq, cv, ce, t[6], fr;
  int si, sj, alch;
  int k;
  if (!(r2 < rc * rc)) return;
  r = sqrt(r2);
  si = s->is_solute[gi] != 0;
  sj = s->is_solute[gj] != 0;
  alch = si != sj;
  sig = 0.5 * (s->sigma[gi] + s->sigma[gj]);
  eps = sqrt(s->epsilon[gi] * s->epsilon[gj]);
  qq = s->coulomb_k * s->charge[gi] * s->charge[gj];
  cv = alch ? c->cv : 1.0;
  ce = alch ? c->ce : 1.0;
  if (s->sc_form == 1)
    orc_pair_terms_shifted(r, sig, eps, qq, cv, ce, s->sc_shift, rc, 1, t);
  else
    orc_pair_terms(r, sig, eps, qq, cv, ce, s->sc_alpha, s->sc_power, rc, 1, t);
  if (s->pme_on) {
    /* Ewald real-space pair: qq erfc(beta r)/r, cut at r_cut, linear in ce */
    double b = s->ewald_beta, ge = erfc(b * r) / r;
    t[3] = ce * qq * ge;
    t[4] = qq * ge;
    t[5] = ce * qq * (ge + 2.0 * b / sqrt(ORC_PI) * exp(-b * b * r2)) / r2;
  }
  fr = t[2] + t[5];
  if (c->f) {
    /* d = x_j - x_i; a repulsive pair pushes i along -d */
    for (k = 0; k < 3; ++k) {
      c->f[3 * i + k] -= fr * d[k];
      c->f[3 * j + k] += fr * d[k];
    }
  }
  if (c->fs) {
    c->fs[i] += fabs(fr) * r;
    c->fs[j] += fabs(fr) * r;
  }
  if (alch) {
    c->u[ORC_U_ALCH_LJ] += t[0];
    c->u[ORC_U_ALCH_C] += t[3];
    if (c->dcv != 0.0) c->dudl += c->dcv * t[1];
    if (c->dce != 0.0) c->dudl += c->dce * t[4];
  } else if (si) {
    c->u[ORC_U_SOLUTE] += t[0] + t[3];
  } else {
    c->u[ORC_U_ENV] += t[0] + t[3];
  }
  if (c->g) {
    /* dU/d(eps_a, sigma_a, q_a) of both atoms of the pair:
     *   eps_ij = sqrt(eps_i eps_j): dU/deps_i = U_LJ / (2 eps_i)
     *   sig_ij = (sig_i + sig_j)/2: dU/dsig_i = 1/2 dU/dsig_ij,
     *     dphi/dsig = 24 eps c (2s-1) s^2 (r/sig)^6 / sig (shift included)
     *   U_C = ce k q_i q_j g(r): dU/dq_i = ce k q_j g(r)                     */
    double dsig = 0.0;
    if (eps != 0.0 && s->sc_form == 1) {
      /* d/dsig of 4 eps c (sig^12 s^-6 - sig^6 s^-3) = 4 eps c (12 sig^11 s^-6 - 6 sig^5 s^-3) */
      double sa = r * r + s->sc_shift * (1.0 - cv), sb = rc * rc + s->sc_shift * (1.0 - cv);
      dsig = 4.0 * eps * cv * ((12.0 * pow(sig, 11.0) / pow(sa, 6.0) - 6.0 * pow(sig, 5.0) / pow(sa, 3.0)) -
                               (12.0 * pow(sig, 11.0) / pow(sb, 6.0) - 6.0 * pow(sig, 5.0) / pow(sb, 3.0)));
    } else if (eps != 0.0) {
      double a = s->sc_alpha * pow(1.0 - cv, (double)s->sc_power);
      double u1 = pow(r / sig, 6.0), u2 = pow(rc / sig, 6.0);
      double s1 = 1.0 / (a + u1), s2 = 1.0 / (a + u2);
      dsig = 24.0 * eps * cv * ((2.0 * s1 - 1.0) * s1 * s1 * u1 - (2.0 * s2 - 1.0) * s2 * s2 * u2) / sig;
    }
    if (s->epsilon[gi] != 0.0) c->g[3 * i + 0] += t[0] / (2.0 * s->epsilon[gi]);
    if (s->epsilon[gj] != 0.0) c->g[3 * j + 0] += t[0] / (2.0 * s->epsilon[gj]);
    c->g[3 * i + 1] += 0.5 * dsig;
    c->g[3 * j + 1] += 0.5 * dsig;
    if (ce != 0.0) {
      double gfun = s->pme_on ? erfc(s->ewald_beta * r) / r : 1.0 / r - 1.0 / rc + (r - rc) / (rc * rc);
      c->g[3 * i + 2] += ce * s->coulomb_k * s->charge[gj] * gfun;
      c->g[3 * j + 2] += ce * s->coulomb_k * s->charge[gi] * gfun;
    }
  }
}

/* Reciprocal, self and background Ewald terms of walker w with the
 * decoupled group's electrostatics scaled linearly by ce.  With E the
 * environment charges and S the alchemical group's, the Ewald energy is
 * the quadratic form V[E+S] = V[E] + V[S] + V_x; the two end states
 * (ce = 1: V[E+S]; ce = 0: V[E] + V[S], the group decoupled but keeping
 * its own interactions) are well defined, and the energy in between is
 * their linear interpolation V[E] + V[S] + ce V_x (Section 2, alchemical
 * pathway: many-body terms interpolated between the electrostatic end
 * values).  The same split applies to the reciprocal, self (no cross part)
 * and neutralising-background terms. */
static void ewald_walker(const orc_sys *s, int32_t w, const double *x, int64_t n, double ce, double dce,
                         eval_ctx *c) {
  const double *L = s->box + 3 * w;
  const int32_t *K = s->pme_dims + 3 * w;
  int p = s->pme_order;
  int64_t N = (int64_t)K[0] * K[1] * K[2], i;
  const uint8_t *sel = s->is_solute + c->base;
  const double *q = s->charge + c->base;
  double *G = (double *)malloc(sizeof(double) * N), *phiE = (double *)malloc(sizeof(double) * N),
         *phiS = (double *)malloc(sizeof(double) * N), *im = (double *)malloc(sizeof(double) * N);
  double V = L[0] * L[1] * L[2], beta = s->ewald_beta, kC = s->coulomb_k;
  double vE = 0.0, vS = 0.0, vX = 0.0, QE = 0.0, QS = 0.0, selfE = 0.0, selfS = 0.0, bgE, bgS, bgX;
  influence(L, K, p, beta, kC, G);
  spme_potential(n, x, q, sel, 0, L, K, p, G, phiE, im);
  spme_potential(n, x, q, sel, 1, L, K, p, G, phiS, im);
  for (i = 0; i < n; ++i) {
    int solute = sel[i] != 0;
    double gE[3], gS[3], pE, pS, pown, poth;
    int k;
    pE = spme_interp(x + 3 * i, L, K, p, phiE, gE);
    pS = spme_interp(x + 3 * i, L, K, p, phiS, gS);
    if (solute) {
      vS += 0.5 * q[i] * pS;
      vX += q[i] * pE;
      QS += q[i];
      selfS += q[i] * q[i];
    } else {
      vE += 0.5 * q[i] * pE;
      QE += q[i];
      selfE += q[i] * q[i];
    }
    pown = solute ? pS : pE;
    poth = solute ? pE : pS;
    if (c->f || c->fs) {
      double fr[3];
      for (k = 0; k < 3; ++k) fr[k] = -q[i] * ((solute ? gS[k] : gE[k]) + ce * (solute ? gE[k] : gS[k]));
      if (c->f)
        for (k = 0; k < 3; ++k) c->f[3 * i + k] += fr[k];
      if (c->fs) c->fs[i] += sqrt((fr[0] * fr[0] + fr[1] * fr[1]) + fr[2] * fr[2]);
    }
    if (c->g) c->g[3 * i + 2] += pown + ce * poth - 2.0 * kC * beta / sqrt(ORC_PI) * q[i];
  }
  bgE = -ORC_PI * kC * QE * QE / (2.0 * V * beta * beta);
  bgS = -ORC_PI * kC * QS * QS / (2.0 * V * beta * beta);
  bgX = -ORC_PI * kC * QE * QS / (V * beta * beta);
  if (c->g)
    for (i = 0; i < n; ++i)
      c->g[3 * i + 2] += sel[i] ? -ORC_PI * kC * (QS + ce * QE) / (V * beta * beta)
                                : -ORC_PI * kC * (QE + ce * QS) / (V * beta * beta);
  c->u[ORC_U_ENV] += vE - kC * beta / sqrt(ORC_PI) * selfE + bgE;
  c->u[ORC_U_SOLUTE] += vS - kC * beta / sqrt(ORC_PI) * selfS + bgS;
  c->u[ORC_U_ALCH_C] += ce * (vX + bgX);
  c->dudl += dce * (vX + bgX);
  free(G);
  free(phiE);
  free(phiS);
  free(im);
}

static int eval_walker(const orc_sys *s, int32_t w, const double *x, double lam, int brute,
                       double *f, double *u_parts, double *dudl, double *g, double *fs) {
  eval_ctx c;
  int64_t n, i;
  const double *L;
  double sch[4], invL[3];
  int k;
  if (w < 0 || w >= s->n_walkers) return -1;
  L = s->box + 3 * w;
  for (k = 0; k < 3; ++k) {
    if (!(s->r_cut < 0.5 * L[k])) return -1;
    invL[k] = 1.0 / L[k];
  }
  n = s->atom_offset[w + 1] - s->atom_offset[w];
  if (s->pme_on) {
    if (!s->pme_dims || (s->pme_order != 4 && s->pme_order != 6 && s->pme_order != 8) || !(s->ewald_beta > 0.0))
      return -1;
    for (k = 0; k < 3; ++k) {
      int32_t d = s->pme_dims[3 * w + k];
      int32_t r = d;
      if (d < s->pme_order) return -1; /* before factoring: d = 0 would not end */
      while (r % 2 == 0) r /= 2;
      while (r % 3 == 0) r /= 3;
      while (r % 5 == 0) r /= 5;
      if (r != 1) return -1;
    }
  }
  memset(&c, 0, sizeof(c));
  c.s = s;
  c.base = s->atom_offset[w];
  orc_schedule(s, lam, sch);
  c.ce = sch[0];
  c.cv = sch[1];
  c.dce = sch[2];
  c.dcv = sch[3];
  c.f = f;
  c.g = g;
  c.fs = fs;
  if (f) memset(f, 0, sizeof(double) * 3 * (size_t)n);
  if (g) memset(g, 0, sizeof(double) * 3 * (size_t)n);
  if (fs) memset(fs, 0, sizeof(double) * (size_t)n);
  {
    /* walkers of 2048 atoms or more: the cell columns in parallel, each with
     * its own sums, added in column order (the same result whatever the
     * thread count); smaller ones in one sweep */
    int nc[3], done = 0;
    if (!brute && n >= 2048 && cell_dims(L, s->r_cut, nc)) {
      int ncol = nc[0] * nc[1], col, q;
      int64_t i;
      eval_ctx *cs = (eval_ctx *)calloc((size_t)ncol, sizeof(eval_ctx));
      void **ptrs = (void **)malloc(sizeof(void *) * (size_t)ncol);
      for (col = 0; col < ncol; ++col) {
        cs[col] = c;
        memset(cs[col].u, 0, sizeof(cs[col].u));
        cs[col].dudl = 0.0;
        cs[col].f = f ? (double *)calloc(3 * (size_t)n, sizeof(double)) : NULL;
        cs[col].g = g ? (double *)calloc(3 * (size_t)n, sizeof(double)) : NULL;
        cs[col].fs = fs ? (double *)calloc((size_t)n, sizeof(double)) : NULL;
        ptrs[col] = &cs[col];
      }
      done = for_each_pair_columns(x, n, L, s->r_cut, eval_pair, ptrs);
      for (col = 0; col < ncol; ++col) {
        for (q = 0; q < 5; ++q) c.u[q] += cs[col].u[q];
        c.dudl += cs[col].dudl;
        for (i = 0; i < 3 * n; ++i) {
          if (f) f[i] += cs[col].f[i];
          if (g) g[i] += cs[col].g[i];
        }
        if (fs)
          for (i = 0; i < n; ++i) fs[i] += cs[col].fs[i];
        free(cs[col].f);
        free(cs[col].g);
        free(cs[col].fs);
      }
      free(cs);
      free(ptrs);
    }
    if (!done) for_each_pair(x, n, L, s->r_cut, brute, eval_pair, &c);
  }
  if (s->pme_on) ewald_walker(s, w, x, n, c.ce, c.dce, &c);
  if (s->anchor && s->k0 && s->k1) {
    for (i = 0; i < n; ++i) {
      int64_t gi = c.base + i;
      double k0 = s->k0[gi], k1 = s->k1[gi];
      double kl, d[3], r2;
      if (k0 == 0.0 && k1 == 0.0) continue;
      kl = k0 + lam * (k1 - k0);
      r2 = min_image(s->anchor + 3 * gi, x + 3 * i, L, invL, d); /* d = x - anchor */
      c.u[ORC_U_RESTR] += 0.5 * kl * r2;
      c.dudl += 0.5 * (k1 - k0) * r2;
      if (f)
        for (k = 0; k < 3; ++k) f[3 * i + k] -= kl * d[k];
      if (fs) fs[i] += kl * sqrt(r2);
    }
  }
  if (s->dr_pairs) {
    /* lambda-dependent distance restraint ("Dealing with metastabilities
     * related to counterions"): acts only while d < d_min(lambda) */
    int32_t ia = s->dr_pairs[2 * w], ib = s->dr_pairs[2 * w + 1];
    double dm[2], d[3], r2, r;
    orc_dmin(s, lam, dm);
    r2 = min_image(x + 3 * ia, x + 3 * ib, L, invL, d); /* d = x_b - x_a */
    r = sqrt(r2);
    if (r < dm[0]) {
      double e = r - dm[0];
      c.u[ORC_U_RESTR] += 0.5 * s->dr_k * e * e;
      c.dudl += -s->dr_k * e * dm[1];
      if (f && r > 0.0)
        for (k = 0; k < 3; ++k) {
          /* dV/dx_b = k e d/r, dV/dx_a = -k e d/r */
          f[3 * ib + k] -= s->dr_k * e * d[k] / r;
          f[3 * ia + k] += s->dr_k * e * d[k] / r;
        }
      if (fs) {
        fs[ia] += fabs(s->dr_k * e);
        fs[ib] += fabs(s->dr_k * e);
      }
    }
  }
  if (u_parts)
    for (k = 0; k < 5; ++k) u_parts[k] = c.u[k];
  if (dudl) *dudl = c.dudl;
  return 0;
}

void orc_dmin(const orc_sys *s, double lam, double out[2]) {
  const double two_pi = 6.283185307179586;
  double n = (double)s->dr_freq;
  out[0] = 0.5 * s->dr_delta * (1.0 - cos(two_pi * n * lam));
  out[1] = 0.5 * s->dr_delta * two_pi * n * sin(two_pi * n * lam);
}

int32_t orc_evaluate(const orc_sys *s, int32_t w, const double *x, double lam, int32_t brute,
                     double *f, double *u_parts, double *dudl) {
  return eval_walker(s, w, x, lam, brute, f, u_parts, dudl, NULL, NULL);
}

int32_t orc_param_grad(const orc_sys *s, int32_t w, const double *x, double lam, double *g) {
  return eval_walker(s, w, x, lam, 0, NULL, NULL, NULL, g, NULL);
}

/* Per-atom force scale of walker w: the sum of the magnitudes of every
 * force term acting on the atom (|f_ij| of each pair within r_cut, the
 * magnitude of the reciprocal-space force, of each restraint force).  The
 * net force can cancel to almost nothing; an error bound relative to this
 * scale does not. */
int32_t orc_force_scale(const orc_sys *s, int32_t w, const double *x, double lam, double *fs) {
  return eval_walker(s, w, x, lam, 0, NULL, NULL, NULL, NULL, fs);
}

/* ---------------------------------------------------------------------------
 * Noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11), written from its published description:
 * ten rounds of two 32x32->64 multiplications by 0xD2511F53 and 0xCD9E8D57
 * and a word permutation, the key bumped by the Weyl constants 0x9E3779B9 and
 * 0xBB67AE85 between rounds.  Gaussian pairs come from Box-Muller in FP64
 * with u1 = (a + 1) 2^-32 in (0, 1] and u2 = b 2^-32 in [0, 1).
 * Counter = (atom, step, walker, purpose), key = (low, high words of seed).
 * Lambda noise uses atom = 0xFFFFFFFF; purpose 0 = Langevin O step,
 * purpose 1 = initial Maxwell-Boltzmann velocities.
 * ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  int r;
  for (r = 0; r < 10; ++r) {
    uint64_t p0, p1;
    uint32_t n0, n1, n2, n3;
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    n1 = (uint32_t)p1;
    n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

void orc_normals(uint64_t seed, uint32_t atom, uint32_t step, uint32_t walker, uint32_t purpose,
                 double out[4]) {
  const double two32 = 4294967296.0;
  const double two_pi = 6.283185307179586;
  uint32_t ctr[4], key[2], o[4];
  int k;
  ctr[0] = atom;
  ctr[1] = step;
  ctr[2] = walker;
  ctr[3] = purpose;
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
  orc_philox4x32_10(ctr, key, o);
  for (k = 0; k < 2; ++k) {
    double u1 = ((double)o[2 * k] + 1.0) / two32;
    double u2 = (double)o[2 * k + 1] / two32;
    double rad = sqrt(-2.0 * log(u1));
    out[2 * k] = rad * cos(two_pi * u2);
    out[2 * k + 1] = rad * sin(two_pi * u2);
  }
}

/* Maxwell-Boltzmann velocities, v = sqrt(kT a / m) xi (noise purpose 1, step 0),
 * and p_lambda = sqrt(m_lambda kT_lambda) xi (atom index 0xFFFFFFFF). */
int32_t orc_init_velocities(const orc_sys *s, orc_state *st) {
  int32_t w;
  for (w = 0; w < s->n_walkers; ++w) {
    int64_t a;
    double z[4];
    for (a = s->atom_offset[w]; a < s->atom_offset[w + 1]; ++a) {
      double sd = sqrt(s->kT * s->accel_unit / s->mass[a]);
      int k;
      orc_normals(s->seed, (uint32_t)(a - s->atom_offset[w]), 0u, (uint32_t)w, 1u, z);
      for (k = 0; k < 3; ++k) st->v[3 * a + k] = sd * z[k];
    }
    orc_normals(s->seed, 0xFFFFFFFFu, 0u, (uint32_t)w, 1u, z);
    st->p_lambda[w] = sqrt(s->m_lambda * s->kT_lambda) * z[0];
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * ABF on lambda.  Bin b = min(floor((lambda - lo)/w), nbins - 1),
 * w = (hi - lo)/nbins.  The bias force on lambda is +A'_t(lambda) (the blue
 * term of Eq. lambda-abf) with A'_t = ramp(n_b) S_b / n_b, ramp(n) =
 * min(1, n/fullSamples), 0 for an empty bin.  A walker sees the shared
 * accumulator as of the last merge plus its own unshared samples; the bias
 * of a step uses the state before that step's samples are added.
 * ------------------------------------------------------------------------- */
int32_t orc_bin_of(const orc_sys *s, double lam) {
  double w = (s->lam_hi - s->lam_lo) / (double)s->n_bins;
  int32_t b = (int32_t)floor((lam - s->lam_lo) / w);
  if (b > s->n_bins - 1) b = s->n_bins - 1;
  if (b < 0) b = 0;
  return b;
}

static double abf_bias(const orc_sys *s, const orc_state *st, int32_t w, int32_t b) {
  int64_t n = st->bin_count[b] + st->loc_count[(int64_t)w * s->n_bins + b];
  double sum = st->bin_sum[b] + st->loc_sum[(int64_t)w * s->n_bins + b];
  double ramp;
  if (n <= 0) return 0.0;
  ramp = (double)n / (double)s->full_samples;
  if (ramp > 1.0) ramp = 1.0;
  return ramp * (sum / (double)n);
}

double orc_abf_bias(const orc_sys *s, const orc_state *st, int32_t w, double lam) {
  if (w < 0 || w >= s->n_walkers) return NAN;
  return abf_bias(s, st, w, orc_bin_of(s, lam));
}

int32_t orc_abf_readout(int32_t n_bins, double lo, double hi, const int64_t *count,
                        const double *sum, double *grad, double *profile, double *delta_a) {
  double w = (hi - lo) / (double)n_bins;
  double acc = 0.0;
  int32_t b, empty = 0;
  for (b = 0; b < n_bins; ++b) {
    double g = 0.0;
    if (count[b] > 0)
      g = sum[b] / (double)count[b];
    else
      empty = 1;
    if (grad) grad[b] = g;
    if (profile) profile[b] = acc; /* A(lo + b w) - A(lo) */
    acc += g * w;
  }
  if (delta_a) *delta_a = acc;
  return empty ? -7 : 0;
}

/* ---------------------------------------------------------------------------
 * Reflecting boundaries at [lo, hi] for lambda: lambda -> 2 lo - lambda or
 * 2 hi - lambda, p_lambda -> -p_lambda.  A second reflection would be needed
 * only for a jump larger than the interval; then lambda is clamped and the
 * walker's status records it.
 * ------------------------------------------------------------------------- */
static void reflect(const orc_sys *s, double *lam, double *p, uint32_t *status) {
  if (*lam < s->lam_lo) {
    *lam = 2.0 * s->lam_lo - *lam;
    *p = -*p;
  } else if (*lam > s->lam_hi) {
    *lam = 2.0 * s->lam_hi - *lam;
    *p = -*p;
  }
  if (*lam < s->lam_lo || *lam > s->lam_hi) {
    *lam = *lam < s->lam_lo ? s->lam_lo : s->lam_hi;
    *status |= ORC_ST_REFLECT;
  }
}

static void wrap_positions(const double *L, double *x, int64_t n) {
  int64_t i;
  int k;
  for (i = 0; i < n; ++i)
    for (k = 0; k < 3; ++k) {
      double v = x[3 * i + k];
      v -= L[k] * floor(v / L[k]);
      if (v >= L[k]) v -= L[k];
      x[3 * i + k] = v;
    }
}

/* ---------------------------------------------------------------------------
 * One step of the coupled Langevin dynamics (Eq. lambda-abf), BAOAB for the
 * atoms and for (lambda, p_lambda), stored in "pending" form: a step
 *   1. evaluates F = -grad V and G = dV/dlambda at the current (x, lambda);
 *   2. ABF: every walker computes its bias from the frozen accumulator, then
 *      adds its sample (bin(lambda), G) to its unshared deltas;
 *   3. if a previous step is open, applies its closing half-kick B
 *      v += h a F/m, p += h (-G + bias);
 *   4. applies this step's B, A (x += h v, lambda += h p/m_lambda, reflect),
 *      O (v = c1 v + sqrt((1-c1^2) kT a/m) xi, same for p with gamma_lambda
 *      and m_lambda), A (and reflect, then wrap x into the box);
 *   5. every K steps merges the walkers' deltas in walker order.
 * h = dt/2, a = accel_unit, c1 = exp(-gamma dt).
 * ------------------------------------------------------------------------- */
int32_t orc_run(const orc_sys *s, orc_state *st, int64_t n_steps, int32_t brute) {
  const double h = 0.5 * s->dt;
  const double c1 = exp(-s->gamma * s->dt);
  const double c1l = exp(-s->gamma_lambda * s->dt);
  int32_t W = s->n_walkers;
  int64_t it;
  for (it = 0; it < n_steps; ++it) {
    int32_t w;
    uint32_t step = (uint32_t)st->step;
    int32_t bad = 0;
    /* 1. forces and dV/dlambda (walkers are independent: one thread each) */
    /* one walker: its pair loop runs over the cell columns in parallel
     * instead (a nested region would run on one thread) */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad) if (W > 1 && s->atom_offset[W] >= 1024)
    for (w = 0; w < W; ++w) {
      int64_t a0 = s->atom_offset[w];
      double u[5];
      if (eval_walker(s, w, st->x + 3 * a0, st->lambda[w], brute, st->f + 3 * a0, u, &st->dudl[w],
                      NULL, NULL) != 0)
        bad = 1;
      else if (!isfinite(st->dudl[w]))
        st->status[w] |= ORC_ST_NONFINITE;
    }
    if (bad) return -1;
    /* 2. ABF bias from the frozen state, then this step's samples */
    for (w = 0; w < W; ++w) {
      st->bias[w] = 0.0;
      if (s->abf_on) {
        int32_t b = orc_bin_of(s, st->lambda[w]);
        int64_t li = (int64_t)w * s->n_bins + b;
        st->bias[w] = abf_bias(s, st, w, b);
        st->loc_count[li] += 1;
        st->loc_sum[li] += st->dudl[w];
        st->loc_sum2[li] += st->dudl[w] * st->dudl[w];
      }
    }
    /* 3-4. integrate (walkers are independent) */
#pragma omp parallel for schedule(static) if (s->atom_offset[W] >= 1024)
    for (w = 0; w < W; ++w) {
      int64_t a0 = s->atom_offset[w], a1 = s->atom_offset[w + 1], a;
      const double *L = s->box + 3 * w;
      double fl = -st->dudl[w] + st->bias[w];
      double z[4];
      int k;
      for (a = a0; a < a1; ++a) {
        double im = s->accel_unit / s->mass[a];
        double sd = sqrt((1.0 - c1 * c1) * s->kT * s->accel_unit / s->mass[a]);
        orc_normals(s->seed, (uint32_t)(a - a0), step, (uint32_t)w, 0u, z);
        for (k = 0; k < 3; ++k) {
          double v = st->v[3 * a + k], x = st->x[3 * a + k], fa = st->f[3 * a + k];
          if (st->pending) v += h * fa * im;
          v += h * fa * im;
          x += h * v;
          v = c1 * v + sd * z[k];
          x += h * v;
          st->v[3 * a + k] = v;
          st->x[3 * a + k] = x;
        }
      }
      wrap_positions(L, st->x + 3 * a0, a1 - a0);
      if (!s->fixed_lambda) {
        double lam = st->lambda[w], p = st->p_lambda[w];
        double sdl = sqrt((1.0 - c1l * c1l) * s->kT_lambda * s->m_lambda);
        if (st->pending) p += h * fl;
        p += h * fl;
        lam += h * p / s->m_lambda;
        reflect(s, &lam, &p, &st->status[w]);
        orc_normals(s->seed, 0xFFFFFFFFu, step, (uint32_t)w, 0u, z);
        p = c1l * p + sdl * z[0];
        lam += h * p / s->m_lambda;
        reflect(s, &lam, &p, &st->status[w]);
        st->lambda[w] = lam;
        st->p_lambda[w] = p;
      }
    }
    st->pending = 1;
    st->step += 1;
    /* 5. share the ABF deltas every K steps, in walker order */
    if (s->abf_on && (st->step % s->share_interval) == 0) {
      int32_t b;
      for (w = 0; w < W; ++w)
        for (b = 0; b < s->n_bins; ++b) {
          int64_t li = (int64_t)w * s->n_bins + b;
          st->bin_count[b] += st->loc_count[li];
          st->bin_sum[b] += st->loc_sum[li];
          st->bin_sum2[b] += st->loc_sum2[li];
          st->loc_count[li] = 0;
          st->loc_sum[li] = 0.0;
          st->loc_sum2[li] = 0.0;
        }
    }
  }
  return 0;
}

/* Full-step velocities of the current pending state (the closing half-kick
 * applied to copies; the state is not modified).  Needs st->f and st->dudl
 * evaluated at the current positions: it evaluates them itself. */
int32_t orc_full_step(const orc_sys *s, const orc_state *st, double *v_full, double *p_full) {
  const double h = 0.5 * s->dt;
  int32_t w;
  for (w = 0; w < s->n_walkers; ++w) {
    int64_t a0 = s->atom_offset[w], a1 = s->atom_offset[w + 1], a, n = a1 - a0;
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double g = 0.0, bias = 0.0;
    int k;
    if (eval_walker(s, w, st->x + 3 * a0, st->lambda[w], 0, f, NULL, &g, NULL, NULL) != 0) {
      free(f);
      return -1;
    }
    if (s->abf_on) bias = abf_bias(s, st, w, orc_bin_of(s, st->lambda[w]));
    for (a = a0; a < a1; ++a)
      for (k = 0; k < 3; ++k) {
        double v = st->v[3 * a + k];
        if (st->pending) v += h * f[3 * (a - a0) + k] * s->accel_unit / s->mass[a];
        v_full[3 * a + k] = v;
      }
    p_full[w] = st->p_lambda[w] + (st->pending ? h * (-g + bias) : 0.0);
    free(f);
  }
  return 0;
}
