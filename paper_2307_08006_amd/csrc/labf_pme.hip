// labf_pme.hip -- smooth particle-mesh Ewald for the lambda-ABF step on gfx950:
// per-step brick lists and fixed-point charge spreading, LDS radix-2
// transforms with the influence function, the gather of potentials and
// forces, and the set-up tables (influence-function factors, the FP32
// real-space correction table, charge sums).
#include "labf_impl.h"
#include "labf_device.h"

#include <math.h>

namespace labf {

__global__ void k_pme_fill(int32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// smooth particle-mesh Ewald: reciprocal space
// ---------------------------------------------------------------------------
// The environment (E) and the alchemical group (S) each have their own
// charge density; with G the (real, even) influence function their grid
// potentials are phi_E = G * Q_E and phi_S = G * Q_S, and the decoupled
// reciprocal energy at electrostatic coupling ce is
// V_E + V_S + ce V_x, V_x = sum_k Q_S phi_E (Section 2, alchemical pathway:
// the many-body term interpolated between its electrostatic end values).
// Both densities ride in one complex grid (E real, S imaginary): one forward
// transform, the multiplication by G, one inverse transform give
// phi_E + i phi_S.  Charges are spread with B-splines of order P
// (Essmann et al. 1995) as 2^-40 fixed-point integers, so the grid does not
// depend on the order of the atomic additions.

// w[j] = M_P(f + j), dw[j] = M_P'(f + j) for j = 0..P-1 (grid point k0 - j,
// f in [0, 1)), from M_2 through M_n(u) = (u M_{n-1}(u) + (n - u) M_{n-1}(u-1)) / (n-1)
// and M_n'(u) = M_{n-1}(u) - M_{n-1}(u - 1).
template <int P>
__device__ __forceinline__ void bspline_w(double f, double (&w)[P], double (&dw)[P]) {
#pragma unroll
  for (int j = 0; j < P; ++j) w[j] = 0.0;
  w[0] = f;
  w[1] = 1.0 - f;
#pragma unroll
  for (int n = 3; n <= P; ++n) {
    if (n == P) {
      dw[0] = w[0];
#pragma unroll
      for (int j = 1; j < P; ++j) dw[j] = w[j] - w[j - 1];
    }
    const double inv = 1.0 / (double)(n - 1);
#pragma unroll
    for (int j = n - 1; j >= 0; --j) {
      const double u = f + (double)j;
      const double a = j < n - 1 ? w[j] : 0.0;
      const double b = j > 0 ? w[j - 1] : 0.0;
      w[j] = (u * a + ((double)n - u) * b) * inv;
    }
  }
}

// v in (-K, K) wrapped into [0, K)
__device__ __forceinline__ int wrapk(int v, int K) { return v < 0 ? v + K : v; }

// Grid base point k0 and offset f of one coordinate (positions are stored
// relative to B and may lie up to a list buffer outside [0, L)).
__device__ __forceinline__ int pme_axis(double x, double L, int K, double &f) {
  double g = x / L;
  g -= floor(g);
  const double u = g * (double)K;
  const double k0 = floor(u);
  f = u - k0;
  // g rounded up to 1 is the image of 0 (f = 0 there): k0 stays in [0, K)
  const int ki = (int)k0;
  return ki < K ? ki : ki - K;
}

// Charge spread, step 1 (one thread per slot): every charged atom joins the
// list of the grid brick that holds its base grid point k0.
// The lanes of a wave (slot order: a few neighbouring bricks) add to each
// brick counter once.
template <typename T>
__global__ __launch_bounds__(256) void k_pme_bin(Dev<T> d, Range r, int xb) {
  const int64_t s = r.c0 * CL + (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t key = -1;
  int w = 0, b = 0;
  if (s < (r.c0 + r.cn) * CL && d.orig[s] >= 0 && d.q64[s] != 0.0) {
    w = d.cl_walker[s / CL];
    const WalkerMeta &m = d.meta[w];
    const PmeWalker &pw = d.pme[w];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double f;
      const int k0 = pme_axis((double)d.X[xb][a][s] - m.B[a], m.L[a], pw.K[a], f);
      b = b * pw.nbr[a] + k0 / PME_BR;
    }
    key = pw.br_begin + b;
  }
  const int pos = wave_agg_add(d.pme_bcnt, key);
  if (key < 0) return;
  const PmeWalker &pw = d.pme[w];
  if (pos < pw.br_cap) d.pme_blist[pw.loff + (int64_t)b * pw.br_cap + pos] = (int32_t)s;
  else atomicOr(&d.status[w], 8u);
}

// Charge spread, step 2 (one block per brick of PME_BR^3 grid points): an
// atom with base point k0 reaches k0 - j, j < P <= PME_BR, so the brick
// receives charge only from atoms listed in itself and in the next brick
// along each axis.  Their B-spline contributions are summed in LDS as
// 2^-40 fixed-point integers (exact and order-independent) and the brick is
// written to the grid once, with no global atomics.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_pme_spread(Dev<T> d, Range r, int xb) {
  constexpr int NP = PME_BR * PME_BR * PME_BR;
  __shared__ unsigned long long acc[2][NP];
  const int bi = r.bb0 + (int)blockIdx.x;
  const int w = d.pme_brw[bi];
  const WalkerMeta &m = d.meta[w];
  const PmeWalker &pw = d.pme[w];
  const int nbx = pw.nbr[0], nby = pw.nbr[1], nbz = pw.nbr[2];
  const int lb = bi - pw.br_begin;
  const int bz = lb % nbz, by = (lb / nbz) % nby, bx = lb / (nbz * nby);
  for (int i = threadIdx.x; i < NP; i += 256) {
    acc[0][i] = 0ull;
    acc[1][i] = 0ull;
  }
  __syncthreads();
  const int ox = bx * PME_BR, oy = by * PME_BR, oz = bz * PME_BR;
  // the eight source lists as one index range
  __shared__ int sbase[9], sidx[8];
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int sb = 0; sb < 8; ++sb) {
      const int sx = (bx + (sb >> 2)) % nbx, sy = (by + ((sb >> 1) & 1)) % nby, sz = (bz + (sb & 1)) % nbz;
      const int sbi = (sx * nby + sy) * nbz + sz;
      const int n = d.pme_bcnt[pw.br_begin + sbi];
      sidx[sb] = sbi;
      sbase[sb] = tot;
      tot += n < pw.br_cap ? n : pw.br_cap;
    }
    sbase[8] = tot;
  }
  __syncthreads();
  const int ntot = sbase[8];
  // chunks of the listed atoms: first the atoms whose footprint k0 - P + 1 ..
  // k0 reaches this brick (base point at most P - 2 points past its upper
  // edge on every axis) are compacted into LDS, then every thread spreads
  // whole atoms of that list, so that waves do not idle on atoms that miss
  constexpr int CH = 1024;
  __shared__ int32_t use[CH];
  __shared__ int nuse;
  for (int c0 = 0; c0 < ntot; c0 += CH) {
    if (threadIdx.x == 0) nuse = 0;
    __syncthreads();
    for (int t = c0 + (int)threadIdx.x; t < ntot && t < c0 + CH; t += 256) {
      int sb = 0;
      while (t >= sbase[sb + 1]) ++sb;
      const int32_t s = d.pme_blist[pw.loff + (int64_t)sidx[sb] * pw.br_cap + (t - sbase[sb])];
      double f;
      bool hit = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int o = a == 0 ? ox : (a == 1 ? oy : oz);
        const int k0 = pme_axis((double)d.X[xb][a][s] - m.B[a], m.L[a], pw.K[a], f);
        hit = hit && wrapk(k0 - o, pw.K[a]) <= PME_BR + P - 2;  // k0, o in [0, K)
      }
      if (hit) use[atomicAdd(&nuse, 1)] = s;
    }
    __syncthreads();
    const int nu = nuse;
    for (int u = threadIdx.x; u < nu; u += 256) {
      const int64_t s = use[u];
      double f[3];
      int k0[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) k0[a] = pme_axis((double)d.X[xb][a][s] - m.B[a], m.L[a], pw.K[a], f[a]);
      double wt[3][P], dw[3][P];
#pragma unroll
      for (int a = 0; a < 3; ++a) bspline_w<P>(f[a], wt[a], dw[a]);
      const double q = d.q64[s];
      unsigned long long *ah = acc[d.sol[s] ? 1 : 0];
      // base point relative to the brick, in [0, K); point k0 - i lies in
      // the brick iff 0 <= dx - i < PME_BR (the wrapped alternative
      // dx - i + K is never below PME_BR, as K >= PME_BR + P - 1)
      const int dx = wrapk(k0[0] - ox, pw.K[0]), dy = wrapk(k0[1] - oy, pw.K[1]),
                dz = wrapk(k0[2] - oz, pw.K[2]);
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int lx = dx - i;
        if ((unsigned)lx >= (unsigned)PME_BR) continue;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const int ly = dy - j;
          if ((unsigned)ly >= (unsigned)PME_BR) continue;
          const double qw = q * wt[0][i] * wt[1][j];
#pragma unroll
          for (int k = 0; k < P; ++k) {
            const int lz = dz - k;
            if ((unsigned)lz >= (unsigned)PME_BR) continue;
            const long long v = __double2ll_rn(qw * wt[2][k] * 0x1p40);
            atomicAdd(ah + (lx * PME_BR + ly) * PME_BR + lz, (unsigned long long)v);
          }
        }
      }
    }
    __syncthreads();
  }
  __syncthreads();
  const int64_t K1 = pw.K[1], K2 = pw.K[2];
  for (int i = threadIdx.x; i < NP; i += 256) {
    const int lx = i / (PME_BR * PME_BR), ly = (i / PME_BR) % PME_BR, lz = i % PME_BR;
    const int64_t g = pw.goff + ((int64_t)(ox + lx) * K1 + (oy + ly)) * K2 + (oz + lz);
    d.pme_grid[g] = make_double2((double)(long long)acc[0][i] * 0x1p-40, (double)(long long)acc[1][i] * 0x1p-40);
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// DFT of R = 2, 3, 4, 5 points in place, y_j = sum_l x_l w^{jl} with
// w = exp(-2 pi i / R) (forward) or its conjugate (inverse), written out so
// that the roots are compile-time constants: cos and sin of 2 pi / 3,
// 2 pi / 5 and 4 pi / 5.
template <bool FWD, int R>
__device__ __forceinline__ void small_dft(double2 (&x)[R]) {
  // i s v for the forward transform's -i and the inverse's +i
  auto rot = [](double2 v, double s) {
    return FWD ? make_double2(s * v.y, -s * v.x) : make_double2(-s * v.y, s * v.x);
  };
  auto add = [](double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); };
  auto sub = [](double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); };
  if constexpr (R == 2) {
    const double2 a = x[0], b = x[1];
    x[0] = add(a, b);
    x[1] = sub(a, b);
  } else if constexpr (R == 3) {
    constexpr double S3 = 0.86602540378443865;  // sin(2 pi / 3)
    const double2 t1 = add(x[1], x[2]), d = sub(x[1], x[2]);
    const double2 t2 = make_double2(fma(-0.5, t1.x, x[0].x), fma(-0.5, t1.y, x[0].y));
    const double2 r = rot(d, S3);
    x[0] = add(x[0], t1);
    x[1] = add(t2, r);
    x[2] = sub(t2, r);
  } else if constexpr (R == 4) {
    const double2 a = add(x[0], x[2]), b = sub(x[0], x[2]);
    const double2 c = add(x[1], x[3]), e = rot(sub(x[1], x[3]), 1.0);
    x[0] = add(a, c);
    x[2] = sub(a, c);
    x[1] = add(b, e);
    x[3] = sub(b, e);
  } else {
    static_assert(R == 5, "radix 2, 3, 4 or 5");
    constexpr double C1 = 0.30901699437494742, C2 = -0.80901699437494742;  // cos(2 pi k / 5)
    constexpr double S1 = 0.95105651629515357, S2 = 0.58778525229247313;   // sin(2 pi k / 5)
    const double2 a1 = add(x[1], x[4]), b1 = sub(x[1], x[4]);
    const double2 a2 = add(x[2], x[3]), b2 = sub(x[2], x[3]);
    const double2 x0 = x[0];
    const double2 p1 = make_double2(fma(C2, a2.x, fma(C1, a1.x, x0.x)), fma(C2, a2.y, fma(C1, a1.y, x0.y)));
    const double2 p2 = make_double2(fma(C1, a2.x, fma(C2, a1.x, x0.x)), fma(C1, a2.y, fma(C2, a1.y, x0.y)));
    const double2 q1 = make_double2(fma(S2, b2.x, S1 * b1.x), fma(S2, b2.y, S1 * b1.y));
    const double2 q2 = make_double2(fma(-S1, b2.x, S2 * b1.x), fma(-S1, b2.y, S2 * b1.y));
    const double2 r1 = rot(q1, 1.0), r2 = rot(q2, 1.0);
    x[0] = add(x0, add(a1, a2));
    x[1] = add(p1, r1);
    x[4] = sub(p1, r1);
    x[2] = add(p2, r2);
    x[3] = sub(p2, r2);
  }
}

// One mixed-radix butterfly of a stage of radix R (span len = R m, offset
// k < m of its block; the R points m apart, mes apart in memory; tw[t] =
// exp(-2 pi i t / K), tws = K / len).  Forward (decimation in frequency):
// the R-point DFT, then output j times w_len^{jk}; inverse (decimation in
// time, stages in reverse order): input l times conj(w_len^{lk}), then the
// conjugate R-point DFT.
template <bool FWD, int R>
__device__ __forceinline__ void mr_butterfly(double2 *base, int mes, const double2 *tw, int k, int tws) {
  double2 x[R];
#pragma unroll
  for (int l = 0; l < R; ++l) x[l] = base[l * mes];
  if (!FWD) {
#pragma unroll
    for (int l = 1; l < R; ++l) x[l] = cmul(x[l], cconj(tw[l * k * tws]));
  }
  small_dft<FWD, R>(x);
  if (FWD) {
#pragma unroll
    for (int j = 1; j < R; ++j) x[j] = cmul(x[j], tw[j * k * tws]);
  }
#pragma unroll
  for (int j = 0; j < R; ++j) base[j * mes] = x[j];
}

// One stage of radix R over nl lines of length K (span len) in LDS.
template <bool FWD, int R>
__device__ __forceinline__ void mr_stage(double2 *buf, const double2 *tw, int K, int len, int nl, int ls,
                                         int es) {
  const int m = len / R, tws = K / len, per = K / R, nb = nl * per, mes = m * es;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    int t, j;
    if (es == 1) {
      t = b / per;
      j = b - t * per;
    } else {
      j = b / nl;
      t = b - j * nl;
    }
    const int blk = j / m, k = j - blk * m;
    mr_butterfly<FWD, R>(buf + t * ls + (blk * len + k) * es, mes, tw, k, tws);
  }
}

// Transforms of nl lines of length K = pw.K[ax] (not a power of two) held in
// LDS, element p of line t at buf[t * ls + p * es], by the stage plan
// pw.rad[ax] (forward: stages in order, output in the plan's digit-reversed
// order, which pme_perm maps to frequencies; inverse: stages in reverse
// order, digit-reversed input, natural output).  Ends with a barrier.
template <bool FWD>
__device__ __forceinline__ void lds_fft_mixed(double2 *buf, const double2 *tw, const PmeWalker &pw, int ax,
                                              int nl, int ls, int es) {
  const int K = pw.K[ax], ns = pw.nst[ax];
  for (int q = 0; q < ns; ++q) {
    const int st = FWD ? q : ns - 1 - q;
    int len = K;
    for (int u = 0; u < st; ++u) len /= pw.rad[ax][u];
    switch (pw.rad[ax][st]) {
      case 2: mr_stage<FWD, 2>(buf, tw, K, len, nl, ls, es); break;
      case 3: mr_stage<FWD, 3>(buf, tw, K, len, nl, ls, es); break;
      case 4: mr_stage<FWD, 4>(buf, tw, K, len, nl, ls, es); break;
      default: mr_stage<FWD, 5>(buf, tw, K, len, nl, ls, es); break;
    }
    __syncthreads();
  }
}

// One block transforms NL grid lines of length K along axis AX in LDS.
// MODE 1: forward; 2: forward, times the influence function, inverse
// (x lines); 3: inverse.  The forward transform is decimation in frequency
// (natural in, digit-reversed out: bit-reversed for the radix-2 stages of a
// power of two, the stage plan's order otherwise), the inverse decimation in
// time (digit-reversed in, natural out), so the grid holds permuted
// frequency indices between the passes and no permutation is ever done;
// pme_perm gives the frequency of each position.  Lines along z are
// contiguous; lines along y and x are taken NL (a divisor of K2) at a time
// from consecutive z so that every load and store is a run of NL
// contiguous points.  MIX = false serves walkers whose three grid lengths
// are powers of two (radix-2 stages, shifts and masks only, half the
// twiddles), MIX = true the others.
template <int AX, int MODE, bool MIX>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_pme_fft(const PmeWalker *pme, const int32_t *bw,
                                                 double2 *grid, const double *tab, const int32_t *perm,
                                                 int b0) {
  // up to PME_TILE points in lines padded by one point (NL <= PME_TILE / 16)
  __shared__ double2 buf[PME_TILE + PME_TILE / 16];
  __shared__ double2 tw[MIX ? PME_KMAX : PME_KMAX / 2];
  const int bid = b0 + (int)blockIdx.x;
  const PmeWalker &pw = pme[bw[bid]];
  const int K = pw.K[AX], lg = pw.lg[AX], NL = pw.nl[AX];
  const bool p2 = !MIX || lg >= 0;
  const int g = bid - pw.blk_begin[AX];
  const int64_t K1 = pw.K[1], K2 = pw.K[2];
  int lgnl = 0;
  if (!MIX)
    while ((1 << lgnl) < NL) ++lgnl;
  // lines of a block and their first z index (y and x lines)
  auto zsplit = [&](int &outer, int &iz0) {
    if (MIX) {
      const int gz = (int)K2 / NL;
      outer = g / gz;
      iz0 = (g - outer * gz) * NL;
    } else {
      const int lgz = pw.lg[2] - lgnl;
      outer = g >> lgz;
      iz0 = (g & ((1 << lgz) - 1)) << lgnl;
    }
  };
  int64_t base, sp;
  if (AX == 2) {
    base = (int64_t)g * NL * K;
    sp = 1;
  } else {
    int outer, iz0;
    zsplit(outer, iz0);
    base = (AX == 1 ? (int64_t)outer * K1 * K2 : (int64_t)outer * K2) + iz0;
    sp = AX == 1 ? K2 : K1 * K2;
  }
  base += pw.goff;
  for (int k = threadIdx.x; k < (MIX ? K : K >> 1); k += blockDim.x) {
    double sn, cs;
    sincospi(-2.0 * (double)k / (double)K, &sn, &cs);
    tw[k] = make_double2(cs, sn);
  }
  const int n = NL * K;
  // LDS line stride: x and y lines are loaded and stored transposed (the
  // lanes of a wave take one point of consecutive lines), so their lines are
  // padded by one point; otherwise the lanes' addresses would be K * 16 bytes
  // apart and share their LDS banks
  const int LS = AX == 2 ? K : K + 1;
  // tile element i in global order -> (line t, position pos); LDS t * LS + pos
  auto split = [&](int i, int &t, int &pos, int64_t &gi) {
    if (AX == 2) {
      if (p2) {
        t = i >> lg;
        pos = i & (K - 1);
      } else {
        t = i / K;
        pos = i - t * K;
      }
      gi = base + i;
    } else {
      if (MIX) {
        pos = i / NL;
        t = i - pos * NL;
      } else {
        pos = i >> lgnl;
        t = i & (NL - 1);
      }
      gi = base + t + pos * sp;
    }
  };
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int t, pos;
    int64_t gi;
    split(i, t, pos, gi);
    buf[t * LS + pos] = grid[gi];
  }
  __syncthreads();
  if (MODE <= 2) {
    if (p2) {
      const int nb = n >> 1, hl = lg - 1;
      for (int l = lg; l >= 1; --l) {  // span 2^l
        const int half = 1 << (l - 1), ts = 1 << (lg - l);
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
          const int t = b >> hl, j = b & ((1 << hl) - 1);
          const int k = j & (half - 1);
          const int i0 = t * LS + ((j >> (l - 1)) << l) + k, i1 = i0 + half;
          const double2 u = buf[i0], v = buf[i1];
          buf[i0] = make_double2(u.x + v.x, u.y + v.y);
          buf[i1] = cmul(make_double2(u.x - v.x, u.y - v.y), tw[k * ts]);
        }
        __syncthreads();
      }
    } else if constexpr (MIX) {
      lds_fft_mixed<true>(buf, tw, pw, AX, NL, LS, 1);
    }
  }
  if (MODE == 2) {
    // x lines (AX == 0): line t is grid column (iy, iz0 + t); each index
    // is mapped to its frequency through pme_perm
    int iy, iz0;
    zsplit(iy, iz0);
    const double *tx = tab + 2 * pw.toff, *ty = tx + 2 * pw.K[0], *tz = ty + 2 * pw.K[1];
    const int32_t *px = perm + pw.toff, *py = px + pw.K[0], *pz = py + pw.K[1];
    const int fy = py[iy];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int t = p2 ? i >> lg : i / K, pos = i - t * K;
      const int fx = px[pos], fz = pz[iz0 + t];
      const double m2 = (tx[2 * fx + 1] + ty[2 * fy + 1]) + tz[2 * fz + 1];
      const double G = (fx | fy | fz) == 0 ? 0.0 : pw.pref * (tx[2 * fx] * ty[2 * fy] * tz[2 * fz]) / m2;
      const double2 v = buf[t * LS + pos];
      buf[t * LS + pos] = make_double2(v.x * G, v.y * G);
    }
    __syncthreads();
  }
  if (MODE >= 2) {
    if (p2) {
      const int nb = n >> 1, hl = lg - 1;
      for (int l = 1; l <= lg; ++l) {
        const int half = 1 << (l - 1), ts = 1 << (lg - l);
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
          const int t = b >> hl, j = b & ((1 << hl) - 1);
          const int k = j & (half - 1);
          const int i0 = t * LS + ((j >> (l - 1)) << l) + k, i1 = i0 + half;
          const double2 u = buf[i0], w0 = tw[k * ts];
          const double2 v = cmul(buf[i1], make_double2(w0.x, -w0.y));
          buf[i0] = make_double2(u.x + v.x, u.y + v.y);
          buf[i1] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
      }
    } else if constexpr (MIX) {
      lds_fft_mixed<false>(buf, tw, pw, AX, NL, LS, 1);
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int t, pos;
    int64_t gi;
    split(i, t, pos, gi);
    grid[gi] = buf[t * LS + pos];
  }
}

// Radix-2 transforms of nl lines of length 2^lg held in LDS, element p of
// line t at buf[t * ls + p * es]; forward: decimation in frequency with
// twiddles tw[k] = exp(-2 pi i k / 2^lg); inverse: decimation in time with
// their conjugates.  Ends with a barrier.
// Consecutive threads take consecutive butterflies of a line when its
// elements are contiguous (es == 1) and consecutive lines otherwise (then
// ls == 1), so that a wave's LDS accesses are contiguous either way.
template <bool FWD>
__device__ __forceinline__ void lds_fft(double2 *buf, const double2 *tw, int lg, int nl, int ls, int es) {
  const int hl = lg - 1, nb = nl << hl;
  for (int st = 0; st < lg; ++st) {
    const int l = FWD ? lg - st : st + 1;  // span 2^l
    const int half = 1 << (l - 1), ts = 1 << (lg - l);
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      const int t = es == 1 ? b >> hl : b % nl, j = es == 1 ? b & ((1 << hl) - 1) : b / nl;
      const int k = j & (half - 1);
      const int p0 = ((j >> (l - 1)) << l) + k;
      double2 *u0 = buf + t * ls + p0 * es, *u1 = u0 + half * es;
      const double2 u = *u0, w = tw[k * ts];
      if (FWD) {
        const double2 v = *u1;
        *u0 = make_double2(u.x + v.x, u.y + v.y);
        *u1 = cmul(make_double2(u.x - v.x, u.y - v.y), w);
      } else {
        const double2 v = cmul(*u1, make_double2(w.x, -w.y));
        *u0 = make_double2(u.x + v.x, u.y + v.y);
        *u1 = make_double2(u.x - v.x, u.y - v.y);
      }
    }
    __syncthreads();
  }
}

// One block per y-z plane (fixed x) of K1 K2 <= NPL points: both transforms
// of the plane in LDS, forward (z then y) or inverse (y then z).  MIX as
// for k_pme_fft.
template <bool FWD, int NPL, bool MIX>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_pme_fft_yz(const PmeWalker *pme, const int32_t *plw,
                                                    double2 *grid, int p0) {
  __shared__ double2 buf[NPL];
  __shared__ double2 twb[MIX ? 2 * PME_KMAX : PME_KMAX];
  const int pid = p0 + (int)blockIdx.x;
  const PmeWalker &pw = pme[plw[pid]];
  const int ix = pid - pw.pl_begin;
  const int K1 = pw.K[1], K2 = pw.K[2], lg1 = pw.lg[1], lg2 = pw.lg[2];
  const int n = K1 * K2;
  // radix-2 stages use the first half of the twiddles only
  const int n1 = MIX ? K1 : K1 >> 1, n2 = MIX ? K2 : K2 >> 1;
  double2 *ty = twb, *tz = twb + n1;
  for (int k = threadIdx.x; k < n1; k += blockDim.x) {
    double sn, cs;
    sincospi(-2.0 * (double)k / (double)K1, &sn, &cs);
    ty[k] = make_double2(cs, sn);
  }
  for (int k = threadIdx.x; k < n2; k += blockDim.x) {
    double sn, cs;
    sincospi(-2.0 * (double)k / (double)K2, &sn, &cs);
    tz[k] = make_double2(cs, sn);
  }
  double2 *g = grid + pw.goff + (int64_t)ix * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) buf[i] = g[i];
  __syncthreads();
  // z lines: K1 lines, contiguous; y lines: K2 lines, stride K2
  if constexpr (!MIX) {
    if (FWD) {
      lds_fft<true>(buf, tz, lg2, K1, K2, 1);
      lds_fft<true>(buf, ty, lg1, K2, 1, K2);
    } else {
      lds_fft<false>(buf, ty, lg1, K2, 1, K2);
      lds_fft<false>(buf, tz, lg2, K1, K2, 1);
    }
  } else if (FWD) {
    if (lg2 >= 0) lds_fft<true>(buf, tz, lg2, K1, K2, 1);
    else lds_fft_mixed<true>(buf, tz, pw, 2, K1, K2, 1);
    if (lg1 >= 0) lds_fft<true>(buf, ty, lg1, K2, 1, K2);
    else lds_fft_mixed<true>(buf, ty, pw, 1, K2, 1, K2);
  } else {
    if (lg1 >= 0) lds_fft<false>(buf, ty, lg1, K2, 1, K2);
    else lds_fft_mixed<false>(buf, ty, pw, 1, K2, 1, K2);
    if (lg2 >= 0) lds_fft<false>(buf, tz, lg2, K1, K2, 1);
    else lds_fft_mixed<false>(buf, tz, pw, 2, K1, K2, 1);
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) g[i] = buf[i];
}

// One thread per slot: potentials of both groups and their gradients at the
// atom; force -q (grad phi_own + ce grad phi_other).
template <typename T, int P>
__global__ __launch_bounds__(256) void k_pme_gather(Dev<T> d, Range r, int xb, int lb) {
  const int64_t s = r.c0 * CL + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= (r.c0 + r.cn) * CL) return;
  const int64_t S = d.n_slots;
  if (d.orig[s] < 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) d.pme_frc[a * S + s] = 0.0;
    d.pme_phi[s] = 0.0;
    d.pme_phi[S + s] = 0.0;
    return;
  }
  const int w = d.cl_walker[s / CL];
  const WalkerMeta &m = d.meta[w];
  const PmeWalker &pw = d.pme[w];
  double wt[3][P], dw[3][P];
  int k0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double f;
    k0[a] = pme_axis((double)d.X[xb][a][s] - m.B[a], m.L[a], pw.K[a], f);
    bspline_w<P>(f, wt[a], dw[a]);
  }
  const double2 *gr = d.pme_grid + pw.goff;
  double pe = 0.0, ps = 0.0, ge[3] = {0.0, 0.0, 0.0}, gs[3] = {0.0, 0.0, 0.0};
  // one grid row (P points along z) per iteration keeps the loads in flight
  // few enough to avoid spilling; the x and y weights of the current row are
  // rotated into element 0 so that every array index is static
#pragma unroll 1
  for (int i = 0; i < P; ++i) {
    const int64_t ix = (int64_t)wrapk(k0[0] - i, pw.K[0]) * pw.K[1];
    double wy[P], dy[P];
#pragma unroll
    for (int t = 0; t < P; ++t) {
      wy[t] = wt[1][t];
      dy[t] = dw[1][t];
    }
#pragma unroll 1
    for (int j = 0; j < P; ++j) {
      const int64_t ixy = (ix + wrapk(k0[1] - j, pw.K[1])) * pw.K[2];
      const double wxy = wt[0][0] * wy[0], dxy = dw[0][0] * wy[0], xdy = wt[0][0] * dy[0];
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const double2 v = gr[ixy + wrapk(k0[2] - k, pw.K[2])];
        const double a = wxy * wt[2][k], bx = dxy * wt[2][k], by = xdy * wt[2][k], bz = wxy * dw[2][k];
        pe += a * v.x;
        ps += a * v.y;
        ge[0] += bx * v.x;
        gs[0] += bx * v.y;
        ge[1] += by * v.x;
        gs[1] += by * v.y;
        ge[2] += bz * v.x;
        gs[2] += bz * v.y;
      }
#pragma unroll
      for (int t = 0; t + 1 < P; ++t) {
        wy[t] = wy[t + 1];
        dy[t] = dy[t + 1];
      }
    }
#pragma unroll
    for (int t = 0; t + 1 < P; ++t) {
      wt[0][t] = wt[0][t + 1];
      dw[0][t] = dw[0][t + 1];
    }
  }
  double ce, dce;
  const LamParams &lp = d.lp;
  channel(d.lambda[lb * d.n_walkers + w], lp.elec_start, lp.elec_end, lp.direction, lp.hi, ce, dce);
  const bool so = d.sol[s] != 0;
  const double q = d.q64[s];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double sc = (double)pw.K[a] / m.L[a];
    const double own = so ? gs[a] : ge[a], oth = so ? ge[a] : gs[a];
    d.pme_frc[a * S + s] = -q * sc * (own + ce * oth);
  }
  d.pme_phi[s] = so ? ps : pe;
  d.pme_phi[S + s] = so ? pe : ps;
}

// Per-axis influence-function factors of every walker (one block per
// walker): A(m) = exp(-pi^2 m~^2 / beta^2) |b(m)|^2 and m~^2, m~ = m / L for the
// signed frequency m of natural index f, with the Euler exponential spline
// modulus |b(m)|^2 = 1 / |sum_{k=0}^{P-2} M_P(k+1) exp(2 pi i m k / K)|^2.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_pme_tables(Dev<T> d, double *tab) {
  const int w = blockIdx.x;
  const WalkerMeta &m = d.meta[w];
  const PmeWalker &pw = d.pme[w];
  double mp[P], dmp[P];
  bspline_w<P>(0.0, mp, dmp);  // mp[j] = M_P(j)
  const int n = pw.K[0] + pw.K[1] + pw.K[2];
  const double pb = 3.14159265358979323846 / d.ewald_beta;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int a = e < pw.K[0] ? 0 : (e < pw.K[0] + pw.K[1] ? 1 : 2);
    const int f = e - (a > 0 ? pw.K[0] : 0) - (a > 1 ? pw.K[1] : 0);
    const int K = pw.K[a];
    const int mm = f < K / 2 ? f : f - K;
    double re = 0.0, im = 0.0;
    for (int k = 0; k <= P - 2; ++k) {
      double sn, cs;
      sincospi(2.0 * (double)mm * (double)k / (double)K, &sn, &cs);
      re += mp[k + 1] * cs;
      im += mp[k + 1] * sn;
    }
    const double mt = (double)mm / m.L[a];
    tab[2 * (pw.toff + e)] = exp(-pb * pb * mt * mt) / (re * re + im * im);
    tab[2 * (pw.toff + e) + 1] = mt * mt;
  }
}

// Per-walker charge sums of both groups in a fixed order (one block per
// walker): Q_E, Q_S, sum_E q^2, sum_S q^2.
template <typename T>
__global__ __launch_bounds__(256) void k_pme_charges(Dev<T> d) {
  __shared__ double red[4][4];
  const int w = blockIdx.x;
  const WalkerMeta &m = d.meta[w];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < m.n_atoms; i += 256) {
    const double q = d.a_q[m.atom_begin + i];
    const int so = d.a_sol[m.atom_begin + i] ? 1 : 0;
    v[so] += q;
    v[2 + so] += q * q;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double t = wave_sum(v[k]);
    if (lane_id() == 0) red[threadIdx.x >> 6][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < 4)
    d.pme_qs[4 * w + threadIdx.x] =
        ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// gF, gE and dgF/ds at s = r^2 in FP64 (dgE/ds = -gF/2); a series in
// x^2 = beta^2 s below x = 0.1, where the closed forms cancel.
__device__ inline void ewald_g(double s, double beta, double &gf, double &ge, double &dgf) {
  const double tsp = 1.1283791670955126;  // 2 / sqrt(pi)
  const double x2 = beta * beta * s;
  if (x2 < 0.01) {
    const double b3 = beta * beta * beta;
    gf = b3 * tsp * (2.0 / 3.0 + x2 * (-2.0 / 5.0 + x2 * (1.0 / 7.0 + x2 * (-1.0 / 27.0 + x2 / 132.0))));
    ge = beta * tsp * (1.0 + x2 * (-1.0 / 3.0 + x2 * (1.0 / 10.0 + x2 * (-1.0 / 42.0 + x2 / 216.0))));
    dgf = b3 * beta * beta * tsp * (-2.0 / 5.0 + x2 * (2.0 / 7.0 + x2 * (-3.0 / 27.0 + x2 * 4.0 / 132.0)));
  } else {
    const double r = sqrt(s), x = beta * r, e = exp(-x2), ef = erf(x);
    gf = ef / (s * r) - beta * tsp * e / s;
    ge = ef / r;
    dgf = beta * tsp * e * (1.5 / (s * s) + beta * beta / s) - 1.5 * ef / (s * s * r);
  }
}

// One thread per interval: cubic Hermite pieces a0 + f (a1 + f (a2 + f a3)),
// f in [0, 1), from the values and slopes at both ends.
__global__ void k_ewald_table(double beta, double smax, float4 *tab) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= EWTAB_N) return;
  const double ds = smax / EWTAB_N;
  double f0, e0, df0, f1, e1, df1;
  ewald_g(k * ds, beta, f0, e0, df0);
  ewald_g((k + 1) * ds, beta, f1, e1, df1);
  const double g0[2] = {f0, e0}, g1[2] = {f1, e1};
  const double d0[2] = {df0 * ds, -0.5 * f0 * ds}, d1[2] = {df1 * ds, -0.5 * f1 * ds};
  for (int q = 0; q < 2; ++q) {
    const double a2 = 3.0 * (g1[q] - g0[q]) - 2.0 * d0[q] - d1[q];
    const double a3 = 2.0 * (g0[q] - g1[q]) + d0[q] + d1[q];
    tab[q * EWTAB_N + k] = make_float4((float)g0[q], (float)d0[q], (float)a2, (float)a3);
  }
}

template <typename T, int P>
static void pme_order_launch(const Dev<T> &d, const Range &r, int xb, int lb, hipStream_t s) {
  const unsigned ns = nblk(r.cn * CL, 256);
  k_pme_fill<<<nblk(r.bbn, 256), 256, 0, s>>>(d.pme_bcnt + r.bb0, r.bbn);
  k_pme_bin<T><<<ns, 256, 0, s>>>(d, r, xb);
  k_pme_spread<T, P><<<(unsigned)r.bbn, 256, 0, s>>>(d, r, xb);
  const double *tab = d.pme_tab;
  // Blocks (and planes) of walkers whose grid lengths are all powers of two
  // come first in every list: the first pbs (pls) of a range go to the
  // radix-2 instantiations, the rest to the mixed-radix ones.
  auto axis = [&](auto k2, auto km, int a) {
    if (r.pbs[a] > 0) k2<<<(unsigned)r.pbs[a], 1024, 0, s>>>(d.pme, d.pme_bw[a], d.pme_grid, tab, d.pme_perm, r.pb0[a]);
    if (r.pbn[a] > r.pbs[a])
      km<<<(unsigned)(r.pbn[a] - r.pbs[a]), 1024, 0, s>>>(d.pme, d.pme_bw[a], d.pme_grid, tab, d.pme_perm,
                                                         r.pb0[a] + r.pbs[a]);
  };
  auto planes = [&](auto k2, auto km) {
    if (r.pls > 0) k2<<<(unsigned)r.pls, 1024, 0, s>>>(d.pme, d.pme_plw, d.pme_grid, r.pl0);
    if (r.pln > r.pls) km<<<(unsigned)(r.pln - r.pls), 1024, 0, s>>>(d.pme, d.pme_plw, d.pme_grid, r.pl0 + r.pls);
  };
  // forward: y-z planes (walkers whose planes fit in LDS) or z then y lines
  // (the others), then x lines with the influence function and the inverse
  // along x, then the inverse along y and z the same two ways
  if (d.pme_npl == 4096) planes(k_pme_fft_yz<true, 4096, false>, k_pme_fft_yz<true, 4096, true>);
  else planes(k_pme_fft_yz<true, 8192, false>, k_pme_fft_yz<true, 8192, true>);
  axis(k_pme_fft<2, 1, false>, k_pme_fft<2, 1, true>, 2);
  axis(k_pme_fft<1, 1, false>, k_pme_fft<1, 1, true>, 1);
  axis(k_pme_fft<0, 2, false>, k_pme_fft<0, 2, true>, 0);
  if (d.pme_npl == 4096) planes(k_pme_fft_yz<false, 4096, false>, k_pme_fft_yz<false, 4096, true>);
  else planes(k_pme_fft_yz<false, 8192, false>, k_pme_fft_yz<false, 8192, true>);
  axis(k_pme_fft<1, 3, false>, k_pme_fft<1, 3, true>, 1);
  axis(k_pme_fft<2, 3, false>, k_pme_fft<2, 3, true>, 2);
  k_pme_gather<T, P><<<ns, 256, 0, s>>>(d, r, xb, lb);
}

template <typename T>
hipError_t Launch<T>::pme(const Dev<T> &d, const Range &r, int xb, int lb, hipStream_t s) {
  if (!d.pme_on || r.cn <= 0) return hipSuccess;
  if (d.pme_order == 4) pme_order_launch<T, 4>(d, r, xb, lb, s);
  else if (d.pme_order == 6) pme_order_launch<T, 6>(d, r, xb, lb, s);
  else pme_order_launch<T, 8>(d, r, xb, lb, s);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::pme_charges(const Dev<T> &d, hipStream_t s) {
  if (!d.pme_on) return hipSuccess;
  k_pme_charges<T><<<(unsigned)d.n_walkers, 256, 0, s>>>(d);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::pme_tables(const Dev<T> &d, float4 *ewtab, hipStream_t s) {
  if (!d.pme_on) return hipSuccess;
  k_ewald_table<<<1, EWTAB_N, 0, s>>>(d.ewald_beta, d.r_cut * d.r_cut, ewtab);
  double *tab = const_cast<double *>(d.pme_tab);
  if (d.pme_order == 4) k_pme_tables<T, 4><<<(unsigned)d.n_walkers, 256, 0, s>>>(d, tab);
  else if (d.pme_order == 6) k_pme_tables<T, 6><<<(unsigned)d.n_walkers, 256, 0, s>>>(d, tab);
  else k_pme_tables<T, 8><<<(unsigned)d.n_walkers, 256, 0, s>>>(d, tab);
  return hipGetLastError();
}

template hipError_t Launch<float>::pme(const Dev<float> &, const Range &, int, int, hipStream_t);
template hipError_t Launch<double>::pme(const Dev<double> &, const Range &, int, int, hipStream_t);
template hipError_t Launch<float>::pme_charges(const Dev<float> &, hipStream_t);
template hipError_t Launch<double>::pme_charges(const Dev<double> &, hipStream_t);
template hipError_t Launch<float>::pme_tables(const Dev<float> &, float4 *, hipStream_t);
template hipError_t Launch<double>::pme_tables(const Dev<double> &, float4 *, hipStream_t);

}  // namespace labf
