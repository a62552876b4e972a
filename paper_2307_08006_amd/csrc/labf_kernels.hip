// labf_kernels.hip -- gfx950 kernels of the lambda-ABF alchemical nonbonded step.
//
// Per step (two independent launches, run concurrently inside a HIP graph of
// 10-step blocks):
//   k_env   : environment atoms.  Environment-environment pairs in the storage
//             precision (plain LJ + shifted-force Coulomb) over a full
//             cluster-pair list (no atomics), 8 i-atoms held in scalar
//             registers against 64 j-atoms in the lanes; then the few
//             alchemical partners of the cluster (soft-core LJ at c_v(lambda),
//             Coulomb at c_e(lambda), "Alchemical pathway"); the epilogue adds
//             restraints and runs BAOAB for the cluster's atoms.
//   k_alch  : alchemical atoms (solute atoms and atoms with a lambda-dependent
//             restraint), one 256-thread block per atom, FP64: forces,
//             dV/dlambda and energies reduced in a fixed order.  The block that
//             completes a walker runs its tail: restraints, BAOAB of its
//             alchemical atoms, the ABF sample and bias, and the BAOAB step of
//             (lambda, p_lambda) with reflection (Eq. lambda-abf); the last
//             walker merges the walkers' ABF samples in walker order
//             ("Orthogonal space sampling").
// Every rebuild_interval steps the neighbour structure is rebuilt: columns
// on an x-y grid, z-sorted, cut into clusters of 8, and per-cluster lists of
// neighbour clusters within r_list = r_cut + r_skin (r_cut + r_skin_alch for
// pairs with an alchemical atom).
#include "labf_impl.h"
#include "labf_device.h"

#include <math.h>

namespace labf {

// ---------------------------------------------------------------------------
// test hook
// ---------------------------------------------------------------------------
__global__ void k_philox(int64_t n, const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t c0 = ctr[4 * i], c1 = ctr[4 * i + 1], c2 = ctr[4 * i + 2], c3 = ctr[4 * i + 3];
  philox10(c0, c1, c2, c3, k0, k1);
  out[4 * i] = c0;
  out[4 * i + 1] = c1;
  out[4 * i + 2] = c2;
  out[4 * i + 3] = c3;
}

// ---------------------------------------------------------------------------
// rebuild: columns -> z-sorted clusters -> cluster-pair lists
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// One thread per slot of the range (atoms in cluster order): wrap, finite
// check, displacement since the last rebuild, column key and column counts.
template <typename T>
__global__ void k_key(Dev<T> d, Range r, int xb, int check) {
  const int64_t s = r.c0 * CL + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int o = s < (r.c0 + r.cn) * CL ? d.orig[s] : -1;
  int64_t K = -1;
  if (o >= 0) {
    const int w = d.cl_walker[s / CL];
    const WalkerMeta &m = d.meta[w];
    const int64_t a = m.atom_begin + o;
    double x[3];
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T xw = wrap_pos<T>(d.X[xb][k][s], (T)m.B[k], (T)m.L[k]);
      x[k] = (double)xw;
      finite = finite && isfinite(x[k]);
    }
    if (!finite) atomicOr(&d.status[w], 1u);
    if (check) {
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double dd = min_image(x[k] - (double)d.xref[(int64_t)k * d.n_atoms + a], m.L[k]);
        r2 += dd * dd;
      }
      // rounded up so that the skin test stays conservative
      d.disp[a] = finite ? __double2float_ru(sqrt(r2)) : INFINITY;
    }
    // clamp in floating point before converting (non-finite or far positions)
    const double fx = fmin(fmax(floor((x[0] - m.B[0]) / m.cw[0]), 0.0), (double)(m.ncx - 1));
    const double fy = fmin(fmax(floor((x[1] - m.B[1]) / m.cw[1]), 0.0), (double)(m.ncy - 1));
    const int cx = finite ? (int)fx : 0;
    const int cy = finite ? (int)fy : 0;
    const int kc = cx * m.ncy + cy;
    const int col = d.a_alch[a] ? m.ncx * m.ncy : kc;
    d.key_col[a] = kc;
    d.col_of[a] = col;
    K = m.col_begin + col;
  }
  (void)wave_agg_add(d.col_count, K);
}

// Two largest displacements of a pair (m1 >= m2) merged with another pair.
__device__ __forceinline__ void top2_merge(float &m1, float &m2, float p1, float p2) {
  const float n2 = fmaxf(fminf(m1, p1), m1 >= p1 ? m2 : p2);
  m1 = fmaxf(m1, p1);
  m2 = n2;
}

// A pair that was farther than r_list apart at the last rebuild can have
// come within r_cut only if the displacements of its two atoms add up to
// more than the skin.  Environment pairs are tested against r_skin with the
// two largest environment displacements, pairs with an alchemical atom
// against r_skin_alch with the largest alchemical displacement plus the
// largest other one.  SKIN_PARTS blocks per walker each reduce a slice of
// its atoms to (e1, e2, a1, a2); the column scan of the walker merges them.
template <typename T>
__global__ __launch_bounds__(256) void k_skin(Dev<T> d, Range r) {
  __shared__ float sm[4][4];
  const int w = r.w0 + blockIdx.x / SKIN_PARTS, part = blockIdx.x % SKIN_PARTS;
  const WalkerMeta &m = d.meta[w];
  const int chunk = (m.n_atoms + SKIN_PARTS - 1) / SKIN_PARTS;
  const int i0 = part * chunk, i1 = min(m.n_atoms, i0 + chunk);
  float e1 = 0.f, e2 = 0.f, a1 = 0.f, a2 = 0.f;
  for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) {
    const int64_t a = m.atom_begin + i;
    const float v = d.disp[a];
    if (d.a_alch[a]) top2_merge(a1, a2, v, 0.f);
    else top2_merge(e1, e2, v, 0.f);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    top2_merge(e1, e2, __shfl_xor(e1, o, WAVE), __shfl_xor(e2, o, WAVE));
    top2_merge(a1, a2, __shfl_xor(a1, o, WAVE), __shfl_xor(a2, o, WAVE));
  }
  const int wv = threadIdx.x >> 6;
  if (lane_id() == 0) {
    sm[wv][0] = e1;
    sm[wv][1] = e2;
    sm[wv][2] = a1;
    sm[wv][3] = a2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      top2_merge(e1, e2, sm[k][0], sm[k][1]);
      top2_merge(a1, a2, sm[k][2], sm[k][3]);
    }
    float *p = d.skin_part + ((int64_t)w * SKIN_PARTS + part) * 4;
    p[0] = e1;
    p[1] = e2;
    p[2] = a1;
    p[3] = a2;
  }
}

// Merge of a walker's partial maxima and the validity flag (one thread).
template <typename T>
__device__ void skin_flag(const Dev<T> &d, int w) {
  float e1 = 0.f, e2 = 0.f, a1 = 0.f, a2 = 0.f;
  for (int part = 0; part < SKIN_PARTS; ++part) {
    const float *p = d.skin_part + ((int64_t)w * SKIN_PARTS + part) * 4;
    top2_merge(e1, e2, p[0], p[1]);
    top2_merge(a1, a2, p[2], p[3]);
  }
  const double skin = d.r_list - d.r_cut, skin_a = d.r_list_a - d.r_cut;
  const bool bad = (double)e1 + (double)e2 > skin || (double)a1 + (double)fmaxf(e1, a2) > skin_a ||
                   !(e1 <= INFINITY) || !(a1 <= INFINITY);
  if (bad) atomicOr(&d.status[w], 4u);
}

// Block-wide exclusive scan of one int per thread (256 threads).
__device__ int block_excl_scan(int v, int *sm, int &total) {
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int t = __shfl_up(inc, o, WAVE);
    if (lane >= o) inc += t;
  }
  if (lane == WAVE - 1) sm[wv] = inc;
  __syncthreads();
  int base = 0;
  for (int k = 0; k < wv; ++k) base += sm[k];
  total = sm[0] + sm[1] + sm[2] + sm[3];
  __syncthreads();
  return base + inc - v;
}

// One block per walker: cluster starts of the columns (each padded to a
// multiple of 8 atoms), atom starts of the member lists; the alchemical
// column starts at cap_env.
template <typename T>
__global__ __launch_bounds__(256) void k_scan(Dev<T> d, Range r, int check) {
  __shared__ int sm[8];
  __shared__ int run_a, run_c;
  const int w = r.w0 + blockIdx.x;
  const WalkerMeta &m = d.meta[w];
  const int ncol = m.ncx * m.ncy;
  if (threadIdx.x == 0) {
    run_a = 0;
    run_c = 0;
  }
  __syncthreads();
  for (int base = 0; base < ncol + 1; base += 256) {
    const int c = base + threadIdx.x;
    const int cnt = c <= ncol ? d.col_count[m.col_begin + c] : 0;
    const int ncl = c < ncol ? (cnt + CL - 1) / CL : 0;
    int ta, tc;
    const int ea = block_excl_scan(cnt, sm, ta);
    const int ec = block_excl_scan(ncl, sm + 4, tc);
    if (c <= ncol) {
      d.col_atom0[m.col_begin + c] = run_a + ea;
      d.col_cl0[m.col_begin + c] = c < ncol ? run_c + ec : m.cap_env;
      d.col_fill[m.col_begin + c] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      run_a += ta;
      run_c += tc;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (check) skin_flag(d, w);
    int ne = run_c;
    if (ne > m.cap_env) {
      atomicOr(&d.status[w], 8u);
      ne = m.cap_env;
    }
    d.n_env[w] = ne;
  }
}

// Member lists of the columns (slot order, one atomic per column and wave).
template <typename T>
__global__ void k_members(Dev<T> d, Range r) {
  const int64_t s = r.c0 * CL + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int o = s < (r.c0 + r.cn) * CL ? d.orig[s] : -1;
  int64_t K = -1, a = 0;
  const WalkerMeta *m = nullptr;
  if (o >= 0) {
    m = &d.meta[d.cl_walker[s / CL]];
    a = m->atom_begin + o;
    K = m->col_begin + d.col_of[a];
  }
  const int pos = wave_agg_add(d.col_fill, K);
  if (o >= 0) d.members[m->atom_begin + d.col_atom0[K] + pos] = o;
}

// One block per column: rank of each member by (z, index), alchemical atoms
// by (x-y column, z, index), computed against the column held in LDS.
// Deterministic whatever the member order.
constexpr int RANK_LDS = 1024;
template <typename T>
__global__ __launch_bounds__(256) void k_rank(Dev<T> d, Range r, int xb) {
  __shared__ T sz[RANK_LDS];
  __shared__ int sidx[RANK_LDS], skc[RANK_LDS];
  const int64_t K = r.k0 + blockIdx.x;
  if (K >= r.k0 + r.kn) return;
  const WalkerMeta &m = d.meta[d.col_walker[K]];
  const int col = (int)(K - m.col_begin);
  const int n = d.col_count[K];
  const int64_t mb = m.atom_begin + d.col_atom0[K];
  const bool alchcol = col == m.ncx * m.ncy;
  // positions are wrapped into the box only at a rebuild: sort on the wrapped
  // z, as the binning and the scatter use it
  const T *Z = d.X[xb][2];
  const T Bz = (T)m.B[2], Lz = (T)m.L[2];
  auto member = [&](int t, T &z, int &idx, int &kc) {
    idx = d.members[mb + t];
    const int64_t b = m.atom_begin + idx;
    z = wrap_pos<T>(Z[d.slot_of[b]], Bz, Lz);
    kc = alchcol ? d.key_col[b] : 0;
  };
  const bool fits = n <= RANK_LDS;
  if (fits)
    for (int t = threadIdx.x; t < n; t += blockDim.x) member(t, sz[t], sidx[t], skc[t]);
  __syncthreads();
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    T z;
    int me, kc;
    if (fits) {
      z = sz[t];
      me = sidx[t];
      kc = skc[t];
    } else {
      member(t, z, me, kc);
    }
    int rank = 0;
    for (int u = 0; u < n; ++u) {
      T zb;
      int bl, kb;
      if (fits) {
        zb = sz[u];
        bl = sidx[u];
        kb = skc[u];
      } else {
        member(u, zb, bl, kb);
      }
      const bool less = kb < kc || (kb == kc && (zb < z || (zb == z && bl < me)));
      rank += less ? 1 : 0;
    }
    // environment atoms fill their column's clusters; every alchemical atom
    // gets a cluster of its own (its list then covers the neighbourhood of
    // one point however far apart the solute atoms drift)
    d.new_slot[m.atom_begin + me] = alchcol ? (int32_t)((m.cl_begin + m.cap_env + rank) * CL)
                                            : (int32_t)((m.cl_begin + d.col_cl0[K]) * CL + rank);
  }
}

template <typename T>
__global__ void k_clear_slots(Dev<T> d, Range r, int xb_new, int vb_new) {
  const int64_t s = r.c0 * CL + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (r.c0 + r.cn) * CL) return;
  const int w = d.cl_walker[s / CL];
  const WalkerMeta &m = d.meta[w];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d.X[xb_new][k][s] = (T)(m.B[k] + 3.0 * m.L[k]);
    d.V[vb_new][k][s] = (T)0;
    d.anc[k][s] = (T)m.B[k];
  }
  d.q[s] = (T)0;
  d.lja[s] = (T)0;
  d.ljb[s] = (T)0;
  d.aim[s] = (T)0;
  d.nsd[s] = (T)0;
  d.rk[s] = (T)0;
  d.q64[s] = 0.0;
  d.sig64[s] = 1.0;
  d.eps64[s] = 0.0;
  d.k0_64[s] = 0.0;
  d.k1_64[s] = 0.0;
  d.sol[s] = 0;
  d.orig[s] = -1;
}

template <typename T>
__global__ void k_scatter(Dev<T> d, Range r, int xb_old, int vb_old, int xb_new, int vb_new) {
  const int64_t a = r.a0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= r.a0 + r.an) return;
  const int w = d.atom_walker[a];
  const WalkerMeta &m = d.meta[w];
  const int s = d.slot_of[a], s2 = d.new_slot[a];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T x = wrap_pos<T>(d.X[xb_old][k][s], (T)m.B[k], (T)m.L[k]);
    d.X[xb_new][k][s2] = x;
    d.xref[(int64_t)k * d.n_atoms + a] = x;
    d.V[vb_new][k][s2] = d.V[vb_old][k][s];
  }
  const double mass = d.a_mass[a];
  d.q[s2] = (T)(sqrt(d.coulomb_k) * d.a_q[a]);
  d.lja[s2] = (T)(0.5 * d.a_sig[a]);
  d.ljb[s2] = (T)sqrt(24.0 * d.a_eps[a]);
  d.aim[s2] = (T)(d.accel / mass);
  d.nsd[s2] = (T)sqrt((1.0 - d.c1 * d.c1) * d.kT * d.accel / mass);
  d.q64[s2] = d.a_q[a];
  d.sig64[s2] = d.a_sig[a];
  d.eps64[s2] = d.a_eps[a];
  if (d.a_k0) {
    d.k0_64[s2] = d.a_k0[a];
    d.k1_64[s2] = d.a_k1[a];
    d.rk[s2] = d.a_alch[a] ? (T)0 : (T)d.a_k0[a];
#pragma unroll
    for (int k = 0; k < 3; ++k) d.anc[k][s2] = (T)d.a_anchor[3 * a + k];
  }
  d.sol[s2] = d.a_sol[a];
  d.orig[s2] = (int32_t)(a - m.atom_begin);
  d.slot_of[a] = s2;
}

__device__ __forceinline__ bool cluster_used(const WalkerMeta &m, int ne, int64_t c) {
  const int64_t loc = c - m.cl_begin;
  return loc < ne || (loc >= m.cap_env && loc < (int64_t)m.cap_env + m.n_acl);
}

template <typename T>
__global__ void k_bbox(Dev<T> d, Range r, int xb) {
  const int64_t c = r.c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= r.c0 + r.cn) return;
  const int w = d.cl_walker[c];
  const WalkerMeta &m = d.meta[w];
  if (!cluster_used(m, d.n_env[w], c)) return;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int col = -1;
  for (int t = 0; t < CL; ++t) {
    const int64_t s = c * CL + t;
    const int o = d.orig[s];
    if (o < 0) continue;
    if (col < 0) col = d.key_col[m.atom_begin + o];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double x = (double)d.X[xb][k][s];
      lo[k] = fmin(lo[k], x);
      hi[k] = fmax(hi[k], x);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d.bbox[c * 6 + k] = (T)lo[k];  // min/max of stored coordinates: exact in T
    d.bbox[c * 6 + 3 + k] = (T)hi[k];
  }
  d.cl_col[c] = col;
}

__device__ __forceinline__ double gap1(double lo_i, double hi_i, double lo_j, double hi_j) {
  return fmax(0.0, fmax(lo_j - hi_i, lo_i - hi_j));
}

// Exclusive prefix sum across the wave and the wave total.
__device__ __forceinline__ int wave_excl_scan(int v, int &total) {
  const int lane = lane_id();
  int inc = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int t = __shfl_up(inc, o, WAVE);
    if (lane >= o) inc += t;
  }
  total = __shfl(inc, WAVE - 1, WAVE);
  return inc - v;
}

// One wave per cluster.  An environment cluster lists the environment
// clusters within r_list (its own (I, I, 0) entry first), then the
// alchemical clusters within r_list_a; an alchemical cluster lists every
// cluster within r_list_a.  The columns in range are enumerated 64 at a
// time (one lane per column, x-y gap test, cluster counts scanned across the
// wave, each flattened cluster's column noted in LDS); their clusters are
// then flattened into passes of 64 lanes, each lane testing one cluster (its
// z image nearest the box, or all three where the box is short enough for
// two to be in range), so that a pass loads 64 cluster boxes however the
// columns are filled.  Alchemical partners take one lane each, testing their
// 27 images in registers.
constexpr int LIST_TAB = 1024;  // flattened clusters per column pass with a direct column lookup
template <typename T>
__global__ __launch_bounds__(256) void k_list(Dev<T> d, Range r) {
  __shared__ int s_pre[4][WAVE + 1];
  __shared__ int s_j0[4][WAVE];
  __shared__ int s_sxy[4][WAVE];
  __shared__ uint8_t s_cidx[4][LIST_TAB];  // flattened cluster -> column lane
  const int64_t c = r.c0 + (int64_t)blockIdx.x * 4 + uni(threadIdx.x >> 6);
  if (c >= r.c0 + r.cn) return;
  const int w = d.cl_walker[c];
  const WalkerMeta &m = d.meta[w];
  const int ne = d.n_env[w];
  const int64_t loc = c - m.cl_begin;
  if (!cluster_used(m, ne, c)) return;
  const bool isA = loc >= m.cap_env;
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  double lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = d.bbox[c * 6 + k];
    hi[k] = d.bbox[c * 6 + 3 + k];
  }
  const int cap = d.list_cap;
  uint32_t *out = d.list + c * (int64_t)cap;
  // environment pairs within r_list; pairs with an alchemical atom within
  // r_list_a (an alchemical cluster lists everything with r_list_a)
  const double rl = (isA ? d.r_list_a : d.r_list) * (1.0 + 1e-7);
  const double rl2 = rl * rl;
  const double rla = d.r_list_a * (1.0 + 1e-7);
  const double rla2 = rla * rla;
  int cnt = 0, nenv = 0;
  if (!isA) {
    if (lane == 0) out[0] = (uint32_t)c | ((uint32_t)SHIFT_ZERO << SHIFT_BITS);
    cnt = 1;
  }
  const bool box_ok = lo[0] <= hi[0] && isfinite(lo[0] + lo[1] + lo[2] + hi[0] + hi[1] + hi[2]);
  if (box_ok) {
    const double tolx = 1e-9 * m.L[0] + 1e-12, toly = 1e-9 * m.L[1] + 1e-12;
    // raw column indices carry the image (-1, 0, +1 box shifts only); clamp in
    // floating point so that far or non-finite boxes cannot produce huge ranges
    auto raw = [](double v, int n) {
      return (int)fmin(fmax(floor(v), -(double)n), (double)(2 * n - 1));
    };
    const int rx0 = raw((lo[0] - rl - m.B[0]) / m.cw[0] - 1e-9, m.ncx);
    const int rx1 = raw((hi[0] + rl - m.B[0]) / m.cw[0] + 1e-9, m.ncx);
    const int ry0 = raw((lo[1] - rl - m.B[1]) / m.cw[1] - 1e-9, m.ncy);
    const int ry1 = raw((hi[1] + rl - m.B[1]) / m.cw[1] + 1e-9, m.ncy);
    const int nry = ry1 - ry0 + 1;
    const int ncols = (rx1 - rx0 + 1) * nry;
    const float inv_nry = 1.0f / (float)nry;
    for (int q0 = 0; q0 < ncols; q0 += WAVE) {
      // one lane per column: x-y gap test, cluster count and first cluster
      const int q = q0 + lane;
      int ncl = 0, j0 = 0, sxy = 0;
      if (q < ncols) {
        // q = qx nry + qy without an integer division: a float estimate of
        // the quotient, corrected by one step (q < 2^24)
        int qx = (int)((float)q * inv_nry), qy = q - qx * nry;
        if (qy < 0) {
          --qx;
          qy += nry;
        } else if (qy >= nry) {
          ++qx;
          qy -= nry;
        }
        const int rx = rx0 + qx, ry = ry0 + qy;
        // raw indices lie in [-n, 2n - 1]: one box shift at most per axis
        const int sx = rx < 0 ? -1 : (rx >= m.ncx ? 1 : 0), sy = ry < 0 ? -1 : (ry >= m.ncy ? 1 : 0);
        const int cx = rx - sx * m.ncx, cy = ry - sy * m.ncy;
        {
          const double cxl = m.B[0] + rx * m.cw[0] - tolx, cxh = m.B[0] + (rx + 1) * m.cw[0] + tolx;
          const double cyl = m.B[1] + ry * m.cw[1] - toly, cyh = m.B[1] + (ry + 1) * m.cw[1] + toly;
          const double gx = gap1(lo[0], hi[0], cxl, cxh), gy = gap1(lo[1], hi[1], cyl, cyh);
          if (gx * gx + gy * gy < rl2) {
            const int col = cx * m.ncy + cy;
            ncl = (d.col_count[m.col_begin + col] + CL - 1) / CL;
            j0 = d.col_cl0[m.col_begin + col];
            sxy = (sx + 1) * 3 + (sy + 1);
          }
        }
      }
      int tot;
      const int pre = wave_excl_scan(ncl, tot);
      s_pre[wv][lane] = pre;
      s_j0[wv][lane] = j0;
      s_sxy[wv][lane] = sxy;
      if (lane == 0) s_pre[wv][WAVE] = tot;
      for (int t = pre; t < pre + ncl && t < LIST_TAB; ++t) s_cidx[wv][t] = (uint8_t)lane;
      __builtin_amdgcn_wave_barrier();
      for (int f0 = 0; f0 < tot; f0 += WAVE) {
        const int f = f0 + lane;
        unsigned mask = 0u;
        int64_t J = 0;
        int sx = 0, sy = 0;
        if (f < tot) {
          // the column slot of flattened cluster f: looked up, else the last
          // slot whose prefix is <= f (that column has clusters)
          int a = 0;
          if (f < LIST_TAB) {
            a = s_cidx[wv][f];
          } else {
            int b = WAVE - 1;
            while (a < b) {
              const int mid = (a + b + 1) >> 1;
              if (s_pre[wv][mid] <= f) a = mid;
              else b = mid - 1;
            }
          }
          J = m.cl_begin + s_j0[wv][a] + (f - s_pre[wv][a]);
          const int code_xy = s_sxy[wv][a];
          sx = code_xy / 3 - 1;
          sy = code_xy % 3 - 1;
          const T *bj = d.bbox + J * 6;
          const double b0 = bj[0], b1 = bj[1], b2 = bj[2], b3 = bj[3], b4 = bj[4], b5 = bj[5];
          const double ox = sx * m.L[0], oy = sy * m.L[1];
          const double ax = gap1(lo[0], hi[0], b0 + ox, b3 + ox);
          const double ay = gap1(lo[1], hi[1], b1 + oy, b4 + oy);
          const double axy = ax * ax + ay * ay;
          // Two z images of the box pair can both lie within r_list only if
          // the two boxes and 2 r_list span the box length; otherwise only
          // the image whose centre lies within L/2 can (test that one).
          const bool all3 = (hi[2] - lo[2]) + (b5 - b2) + 2.0 * rl >= m.L[2] * (1.0 - 1e-6);
          const double dzc = 0.5 * ((b2 + b5) - (lo[2] + hi[2]));
          const int sn = dzc > 0.5 * m.L[2] ? -1 : (dzc < -0.5 * m.L[2] ? 1 : 0);
#pragma unroll
          for (int sz = -1; sz <= 1; ++sz) {
            if (!all3 && sz != sn) continue;
            const double oz = sz * m.L[2];
            const double az = gap1(lo[2], hi[2], b2 + oz, b5 + oz);
            bool pass = axy + az * az < rl2;
            if (!isA && J == c && sx == 0 && sy == 0 && sz == 0) pass = false;
            mask |= (pass ? 1u : 0u) << (sz + 1);
          }
        }
#pragma unroll
        for (int zs = 0; zs < 3; ++zs) {
          const bool pass = (mask >> zs) & 1u;
          const unsigned long long bal = __ballot(pass);
          if (bal == 0ull) continue;
          if (pass) {
            const int pos = cnt + __popcll(bal & ((1ull << lane) - 1ull));
            const int code = image_code(sx, sy, zs - 1);
            if (pos < cap) out[pos] = (uint32_t)J | ((uint32_t)code << SHIFT_BITS);
          }
          cnt += __popcll(bal);
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    nenv = cnt;
    // alchemical atoms (one per cluster), every image within r_list_a: an
    // environment cluster computes their forces on its own atoms, an
    // alchemical cluster its alchemical-alchemical pairs
    const int64_t A0 = m.cl_begin + m.cap_env;
    for (int t0 = 0; t0 < m.n_acl; t0 += WAVE) {
      const int t = t0 + lane;
      unsigned mask = 0u;
      int64_t J = 0;
      if (t < m.n_acl) {
        J = A0 + t;
        const T *bj = d.bbox + J * 6;
        const double b0 = bj[0], b1 = bj[1], b2 = bj[2], b3 = bj[3], b4 = bj[4], b5 = bj[5];
        if (b0 <= b3) {
          // squared box gaps per axis and image shift, then all 27 sums
          double ax2[3], ay2[3], az2[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double ox = (k - 1) * m.L[0], oy = (k - 1) * m.L[1], oz = (k - 1) * m.L[2];
            const double ax = gap1(lo[0], hi[0], b0 + ox, b3 + ox);
            const double ay = gap1(lo[1], hi[1], b1 + oy, b4 + oy);
            const double az = gap1(lo[2], hi[2], b2 + oz, b5 + oz);
            ax2[k] = ax * ax;
            ay2[k] = ay * ay;
            az2[k] = az * az;
          }
#pragma unroll
          for (int t27 = 0; t27 < 27; ++t27)
            if ((ax2[t27 / 9] + ay2[(t27 / 3) % 3]) + az2[t27 % 3] < rla2) mask |= 1u << t27;
        }
      }
      int tot;
      int pos = cnt + wave_excl_scan(__popc(mask), tot);
      for (int t27 = 0; t27 < 27; ++t27) {
        if ((mask >> t27) & 1u) {
          const int code = image_code(t27 / 9 - 1, (t27 / 3) % 3 - 1, t27 % 3 - 1);
          if (pos < cap) out[pos] = (uint32_t)J | ((uint32_t)code << SHIFT_BITS);
          ++pos;
        }
      }
      cnt += tot;
    }
  }
  if (lane == 0) {
    d.list_count[c] = cnt < cap ? cnt : cap;
    d.list_nenv[c] = nenv < cap ? nenv : cap;
    if (cnt > cap) atomicOr(&d.status[w], 8u);
    if (!isA) d.plist_n[m.env_item_begin + loc] = -1;  // prune again before use
  }
}

// ---------------------------------------------------------------------------
// dynamic pruning of the environment pair lists
// ---------------------------------------------------------------------------
// A cluster list holds whole neighbour clusters within r_list of the cluster
// box; most of their atoms lie beyond r_cut of every atom of the box.  Every
// few steps k_prune keeps, per environment cluster, the j atoms within
// r_cut + b of the box (b, the prune buffer, below the skin) in a compact
// list; k_env evaluates that list 64 atoms at a time.  Between prunes an atom
// moves at most D (the largest displacement in the walker since the prune,
// measured by the integrating kernels), so a pair inside r_cut now was
// inside r_cut + 2D then: the list stays complete while 2D <= b.  The test is
// walker-wide so that all clusters of a walker share one prune step (and one
// reference configuration); the cluster list itself stays valid while the
// displacements since the rebuild stay within the skin (the k_skin test).
// A stale list (after a rebuild) is always pruned.
constexpr int PRUNE_CPW = 1;  // clusters per wave of k_prune
constexpr int PRUNE_NP = 4;   // passes of 8 list entries gathered at once (at most 8)
template <typename T>
__global__ __launch_bounds__(256) void k_prune(Dev<T> d, Range r, int xb, int lb) {
  const int64_t nw = (r.en + PRUNE_CPW - 1) / PRUNE_CPW;  // waves in all
  const int nb = (int)((nw + 3) >> 2);
  // plain block order: the walkers that prune at a step spread over all
  // XCDs (with the XCD-aware order of k_env, a step on which a few walkers
  // prune would load only their XCDs)
  const int lblk = (int)blockIdx.x;
  if (lblk >= nb) return;
  const int64_t gw = (int64_t)lblk * 4 + uni(threadIdx.x >> 6);
  const int64_t e_first = r.e0 + gw * PRUNE_CPW;
  const int lane = lane_id();
  const int W = d.n_walkers;
  {
    // The Langevin normals of the coming step for the environment atoms,
    // four items (32 atoms) per wave at full lane width: lane -> item
    // lane / 16, atom (lane / 2) % 8, Box-Muller pair lane % 2 (z0, z1 or
    // z2 of gauss4).  Drawn here, the integrating epilogue of the
    // environment kernel only reads them.
    const int64_t e = r.e0 + gw * 4 + (lane >> 4);
    if (e < r.e0 + r.en) {
      const int64_t c = d.env_table[e];
      const int w = d.cl_walker[c];
      const int64_t s = c * CL + ((lane >> 1) & (CL - 1));
      const int32_t o = d.orig[s];
      if (c - d.meta[w].cl_begin < d.n_env[w] && o >= 0) {
        const int p = lane & 1;
        double zc, zs;
        gauss_pair(d.seed, (uint32_t)o, (uint32_t)d.step[lb * W + w], (uint32_t)w, 0u, p, zc, zs);
        if (p == 0) {
          d.noise[0][s] = (T)zc;
          d.noise[1][s] = (T)zs;
        } else {
          d.noise[2][s] = (T)zc;
        }
      }
    }
  }
  const T *X0 = d.X[xb][0], *X1 = d.X[xb][1], *X2 = d.X[xb][2];
  __shared__ T shtab[4][3][IMG_CODES];
  T *shx = shtab[threadIdx.x >> 6][0], *shy = shtab[threadIdx.x >> 6][1], *shz = shtab[threadIdx.x >> 6][2];
  int wtab = -1;    // walker of D and of the prune radius
  int wshift = -1;  // walker of the image-shift table (filled when a cluster prunes)
  float D = 0.f, half = 0.f;
  T pr2 = (T)0;
  for (int64_t e = e_first; e < e_first + PRUNE_CPW && e < r.e0 + r.en; ++e) {
    const int64_t c = d.env_table[e];
    const int w = d.cl_walker[c];
    const WalkerMeta &m = d.meta[w];
    const int64_t loc = c - m.cl_begin;
    if (loc >= d.n_env[w]) continue;
    if (w != wtab) {
      // the largest displacement since the prune, as the last step measured
      // it (maximum over the walker's slots)
      uint32_t Db = d.pdisp[((int64_t)lb * W + w) * PDISP_SLOTS + lane];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) Db = max(Db, (uint32_t)__shfl_xor((int)Db, o, WAVE));
      D = __uint_as_float(Db);
      // re-prune threshold b/2, less 1e-4 for the rounding of the box distances
      half = (float)(0.5 * m.prune_b - 1e-4);
      pr2 = (T)((d.r_cut + m.prune_b) * (d.r_cut + m.prune_b));
      wtab = w;
    }
    // the next step's integration measures into the other buffer
    if (loc == 0) d.pdisp[((int64_t)(lb ^ 1) * W + w) * PDISP_SLOTS + lane] = 0u;
    if (d.plist_n[e] >= 0 && D <= half) continue;
    if (w != wshift) {
      __builtin_amdgcn_wave_barrier();
      shx[lane] = (T)img_x(lane) * (T)m.L[0];
      shy[lane] = (T)img_y(lane) * (T)m.L[1];
      shz[lane] = (T)img_z(lane) * (T)m.L[2];
      __builtin_amdgcn_wave_barrier();
      wshift = w;
    }
    const int64_t s0 = c * CL;
    if (lane < CL) {
      d.xprune[0][s0 + lane] = X0[s0 + lane];
      d.xprune[1][s0 + lane] = X1[s0 + lane];
      d.xprune[2][s0 + lane] = X2[s0 + lane];
    }
    const T far = (T)(8.0 * m.B[0]);
    T lox = far, loy = far, loz = far, hix = -far, hiy = -far, hiz = -far;
#pragma unroll
    for (int ii = 0; ii < CL; ++ii) {
      if (d.orig[s0 + ii] >= 0) {
        lox = fmin(lox, X0[s0 + ii]);
        loy = fmin(loy, X1[s0 + ii]);
        loz = fmin(loz, X2[s0 + ii]);
        hix = fmax(hix, X0[s0 + ii]);
        hiy = fmax(hiy, X1[s0 + ii]);
        hiz = fmax(hiz, X2[s0 + ii]);
      }
    }
    const uint32_t *lst = d.list + c * (int64_t)d.list_cap;
    uint32_t *out = d.plist + e * (int64_t)d.plist_cap;
    const int cap = d.plist_cap;
    const int nenv = d.list_nenv[c];
    const int64_t ws0 = m.cl_begin * CL;
    int cnt = 0;
    // Batches of 32 entries: one coalesced load of the entries, then the
    // candidates of all four passes gathered at once (lane -> entry
    // b0 + 8 t + lane / 8, atom lane % 8 in pass t), then tested and
    // compacted pass by pass.  The cluster's own entry comes first, so its
    // atoms open the pruned list (chunk 0).  Unused slots hold positions
    // B + 3L, farther than L from every atom image: they never pass.
    // Slot offsets are 32-bit byte offsets (fewer than 2^29 slots).
    const uint32_t wsl = (uint32_t)ws0;
    for (int b0 = 0; b0 < nenv; b0 += PRUNE_NP * CL) {
      const uint32_t eb = lst[min(b0 + (lane & (PRUNE_NP * CL - 1)), nenv - 1)];
      T xj[PRUNE_NP], yj[PRUNE_NP], zj[PRUNE_NP];
      uint32_t val[PRUNE_NP];
#pragma unroll
      for (int t = 0; t < PRUNE_NP; ++t) {
        const uint32_t ent = (uint32_t)__shfl((int)eb, t * CL + (lane >> 3), WAVE);
        const uint32_t code = ent >> SHIFT_BITS;
        const uint32_t js = (ent & CL_MASK) * CL + (uint32_t)(lane & 7);
        const uint32_t bo = js * (uint32_t)sizeof(T);
        xj[t] = ld_off(X0, bo) + shx[code];
        yj[t] = ld_off(X1, bo) + shy[code];
        zj[t] = ld_off(X2, bo) + shz[code];
        val[t] = (js - wsl) | (code << SHIFT_BITS);
      }
      const bool room = cnt + PRUNE_NP * WAVE <= cap;
#pragma unroll
      for (int t = 0; t < PRUNE_NP; ++t) {
        const T gx = fmax(fmax(lox - xj[t], xj[t] - hix), (T)0);
        const T gy = fmax(fmax(loy - yj[t], yj[t] - hiy), (T)0);
        const T gz = fmax(fmax(loz - zj[t], zj[t] - hiz), (T)0);
        const bool keep = b0 + t * CL + (lane >> 3) < nenv && fma(gz, gz, fma(gy, gy, gx * gx)) < pr2;
        const unsigned long long bal = __ballot(keep);
        const int pos = cnt + lanes_below(bal);
        if (keep && (room || pos < cap)) st_off(out, (uint32_t)pos * 4u, val[t]);
        cnt += __popcll(bal);
      }
    }
    if (cnt > cap) {
      if (lane == 0) atomicOr(&d.status[w], 8u);
      cnt = cap;
    }
    // fill the last chunk
    const int nch = (cnt + WAVE - 1) / WAVE;
    const int pad = (nch - 1) * WAVE + lane;
    if (nch > 0 && pad >= cnt) out[pad] = PRUNE_PAD;
    if (lane == 0) d.plist_n[e] = nch;
  }
}

// ---------------------------------------------------------------------------
// environment pair kernel
// ---------------------------------------------------------------------------
// Per-wave LDS ring of pruned j atoms (position, scaled charge; sigma/2 and
// sqrt(24 eps) for per-atom mixing) of the real-space Ewald kernels, which
// prune their cluster lists as they go.  At most 63 + 64 entries are pending.
constexpr int RING = 128;
template <typename T, bool LB>
struct Ring {
  T x[RING], y[RING], z[RING], q[RING];
  T a[LB ? RING : 1], b[LB ? RING : 1];
  __device__ __forceinline__ void put(int k, T xj, T yj, T zj, T qj, T aj, T bj) {
    x[k] = xj;
    y[k] = yj;
    z[k] = zj;
    q[k] = qj;
    if (LB) {
      a[k] = aj;
      b[k] = bj;
    }
  }
  __device__ __forceinline__ void get(int k, T &xj, T &yj, T &zj, T &qj, T &aj, T &bj) const {
    xj = x[k];
    yj = y[k];
    zj = z[k];
    qj = q[k];
    aj = LB ? a[k] : (T)0;
    bj = LB ? b[k] : (T)0;
  }
};
// Real-space Ewald pair (qq erfc(beta r)/r, cut at r_cut) written as the
// bare Coulomb pair minus a correction: F/r = qq r^-3 - c, where c is what
// ewald_corr returns, and U = qq/r - qq gE (in ue; used by the energy
// kernels only).  FP64: c = qq r^-2 (erf(beta r)/r - (2 beta/sqrt(pi))
// exp(-beta^2 r^2)) from the library erf.  FP32: with
// gE = erf(beta r)/r and gF = erf(beta r)/r^3 - (2 beta/sqrt(pi))
// exp(-beta^2 r^2)/r^2, smooth even functions of r, c = qq gF; both are read
// from cubic Hermite pieces on EWTAB_N equal intervals of r^2 in
// [0, r_cut^2] (built in FP64, error < 2e-9 of the bare Coulomb term), so a
// pair costs a table read and three FMAs.
template <typename T>
__device__ __forceinline__ T ewald_corr(const Dev<T> &d, const float4 *, T qq, T r2, T rinv, T r2inv, T &ue) {
  const T x = d.ewb * (r2 * rinv);
  ue = qq * erfc(x) * rinv;
  return qq * r2inv * (erf(x) * rinv - d.ewc * exp(-x * x));
}

template <>
__device__ __forceinline__ float ewald_corr<float>(const Dev<float> &d, const float4 *ft, float qq, float r2,
                                                   float rinv, float r2inv, float &ue) {
  // the largest float below EWTAB_N: pairs just inside r_cut keep their
  // offset in the last interval; lanes beyond r_cut (masked) stay in range
  const float u = fminf(r2 * d.ewtab_inv, (float)EWTAB_N * 0.99999994f);
  const int k = (int)u;
  const float f = u - (float)k;
  const float4 cf = ft[k], ce = d.ewtab[EWTAB_N + k];
  const float gf = fmaf(f, fmaf(f, fmaf(f, cf.w, cf.z), cf.y), cf.x);
  const float ge = fmaf(f, fmaf(f, fmaf(f, ce.w, ce.z), ce.y), ce.x);
  ue = qq * (rinv - ge);
  return qq * gf;
}

// Coulomb F/r of a real-space Ewald pair.
template <typename T>
__device__ __forceinline__ T ewald_fr(const Dev<T> &d, T qq, T r2, T rinv, T r2inv) {
  T ue;
  return qq * rinv * r2inv - ewald_corr(d, d.ewtab, qq, r2, rinv, r2inv, ue);
}

template <typename T, bool LB, bool ENERGY, bool DIAG, bool EW, bool EONLY = false>
__device__ __forceinline__ void env_pairs(const Dev<T> &d, const T (&xi)[CL], const T (&yi)[CL],
                                          const T (&zi)[CL], const T (&qi)[CL], const T (&ai)[CL],
                                          const T (&bi)[CL], int64_t s0, T xj, T yj, T zj, T qj,
                                          T aj, T bj, int js, int vmask, T (&fx)[CL],
                                          T (&fy)[CL], T (&fz)[CL], double &eacc, const float4 *ewt) {
  const T c12x12 = (T)12 * d.c12, c6x6 = (T)6 * d.c6;
#pragma unroll
  for (int ii = 0; ii < CL; ++ii) {
    const T dx = xj - xi[ii], dy = yj - yi[ii], dz = zj - zi[ii];
    const T r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    bool in = r2 < d.rc2;
    if (DIAG) in = in && (js != (int)(s0 + ii));
    const T rinv = rsq(r2);
    const T r2inv = rinv * rinv;
    // F/r = r^-2 (L + e) - c: L the LJ part without its r^-2 factor, e = qq/r,
    // c = e / r_c^2 (shifted force) or the Ewald correction; two FMAs
    const T qq = qi[ii] * qj;
    const T e = qq * rinv;
    T g, t3 = 0, bij = 0, r6 = 0;
    if (!LB) {
      r6 = r2inv * r2inv * r2inv;
      g = fma(r6, fma(c12x12, r6, -c6x6), e);
    } else {
      const T sg = ai[ii] + aj;
      const T t = sg * sg * r2inv;
      t3 = t * t * t;
      bij = bi[ii] * bj;
      g = fma(bij * t3, fma((T)2, t3, (T)-1), e);
    }
    T uew = (T)0;
    const T c = EW ? ewald_corr(d, ewt, qq, r2, rinv, r2inv, uew) : d.irc2 * e;
    if (!EONLY) {
      T fr = fma(r2inv, g, -c);
      fr = in ? fr : (T)0;
      fx[ii] -= fr * dx;
      fy[ii] -= fr * dy;
      fz[ii] -= fr * dz;
    }
    if (ENERGY) {
      T el;
      if (!LB) {
        el = (d.c12 * r6 - d.c6) * r6 - d.ushift;
      } else {
        const T sg = ai[ii] + aj;
        const T tc = sg * sg * d.irc2;
        const T tc3 = tc * tc * tc;
        el = bij / (T)6 * ((t3 * t3 - t3) - (tc3 * tc3 - tc3));
      }
      const T rr = r2 * rinv;
      const T ec = EW ? uew : qq * (rinv - d.irc + (rr - (T)d.r_cut) * d.irc2);
      // padded i-slots share the sentinel position with padded j-slots
      eacc += (in && ((vmask >> ii) & 1)) ? 0.5 * ((double)el + (double)ec) : 0.0;
    }
  }
}

// Forces on environment atoms from alchemical atoms (storage precision):
// soft-core LJ at coupling cv with A = alpha (1 - cv)^p and shifted-force
// Coulomb at ce for solute partners, plain terms (c = 1) for the others.
// Energies and dV/dlambda of these pairs are accounted on the alchemical side.
template <typename T, bool SHIFTED, bool EW>
__device__ __forceinline__ void env_alch_pairs(const Dev<T> &d, const T (&xi)[CL],
                                               const T (&yi)[CL], const T (&zi)[CL],
                                               const T (&qi)[CL], const T (&ai)[CL],
                                               const T (&bi)[CL], T xj, T yj, T zj, T qj, T aj,
                                               T bj, bool alch, bool valid, T cv, T ce, T Asc,
                                               T Dsc, T (&fx)[CL], T (&fy)[CL], T (&fz)[CL]) {
  // soft-core: y = 1/(A + (r/sig)^6) or y = (sig^2 / (r^2 + D))^3 (separation
  // shifted, D = delta (1 - c)); F/r of the LJ part = 24 eps c (2y - 1) y g with
  // g = y (r/sig)^6 / r^2 or 1 / (r^2 + D); c = 1, A = D = 0 for plain pairs
  const T c = alch ? cv : (T)1, e = alch ? ce : (T)1, A = alch ? Asc : (T)0, D = alch ? Dsc : (T)0;
#pragma unroll
  for (int ii = 0; ii < CL; ++ii) {
    const T dx = xj - xi[ii], dy = yj - yi[ii], dz = zj - zi[ii];
    const T r2 = dx * dx + dy * dy + dz * dz;
    const bool in = valid && r2 < d.rc2;
    const T rinv = rsq(r2);
    const T r2inv = rinv * rinv;
    const T sg = ai[ii] + aj;
    T y, g;
    if (SHIFTED) {
      const T sinv = rcp(r2 + D);
      const T w = sg * sg * sinv;
      y = w * w * w;
      g = sinv;
    } else {
      const T t = r2 * rcp(sg * sg);
      const T u = t * t * t;
      y = rcp(A + u);
      g = y * u * r2inv;
    }
    const T bij = bi[ii] * bj;
    T flj = bij * c * ((T)2 * y - (T)1) * y * g;
    flj = bij != (T)0 ? flj : (T)0;
    const T fc = EW ? ewald_fr(d, e * qi[ii] * qj, r2, rinv, r2inv)
                    : e * qi[ii] * qj * rinv * (r2inv - d.irc2);
    const T fr = in ? flj + fc : (T)0;
    fx[ii] -= fr * dx;
    fy[ii] -= fr * dy;
    fz[ii] -= fr * dz;
  }
}

// Lambda-dependent distance restraint between atoms a and b (global indices):
// V = k/2 e^2 with e = d - d_min while d < d_min(lambda) = (delta/2)(1 - cos(2 pi n
// lambda)), zero otherwise ("Dealing with metastabilities related to
// counterions").  u = (x_b - x_a)/d under the minimum image; the force on a is
// k e u, on b -k e u; dV/dlambda = -k e d_min'.
struct DrTerm {
  bool on;
  double e, dm1, u[3];
};

template <typename T>
__device__ __forceinline__ DrTerm dr_term(const Dev<T> &d, const WalkerMeta &m, int xb, int64_t a,
                                          int64_t b, double lam) {
  DrTerm t = {false, 0.0, 0.0, {0.0, 0.0, 0.0}};
  const int sa = d.slot_of[a], sb = d.slot_of[b];
  double v[3], r2 = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    v[q] = min_image((double)(d.X[xb][q][sb] - d.X[xb][q][sa]), m.L[q]);
    r2 += v[q] * v[q];
  }
  const double r = sqrt(r2);
  const double ph = 6.283185307179586 * (double)d.dr_freq * lam;
  const double dmin = 0.5 * d.dr_delta * (1.0 - cos(ph));
  if (r < dmin) {
    t.on = true;
    t.e = r - dmin;
    t.dm1 = 0.5 * d.dr_delta * 6.283185307179586 * (double)d.dr_freq * sin(ph);
#pragma unroll
    for (int q = 0; q < 3; ++q) t.u[q] = r > 0.0 ? v[q] / r : 0.0;
  }
  return t;
}

// Returns the squared displacement of the new position from the position at
// the last prune (used by the environment atoms' integration only).
template <typename T>
__device__ __forceinline__ double integrate_atom(const Dev<T> &d, int64_t s, int xb, int vb, int w,
                                                 int64_t step, bool pending, const double F[3]) {
  const T h = (T)(0.5 * d.dt);
  const T c1 = (T)d.c1;
  const T im = d.aim[s], sd = d.nsd[s];
  double z[4];
  T xo[3];
  gauss4(d.seed, (uint32_t)d.orig[s], (uint32_t)step, (uint32_t)w, 0u, z);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T fa = (T)F[k];
    T v = d.V[vb][k][s];
    T x = d.X[xb][k][s];
    if (pending) v += h * fa * im;
    v += h * fa * im;
    x += h * v;
    v = c1 * v + sd * (T)z[k];
    x += h * v;
    d.V[vb][k][s] = v;
    // no wrap here: the cluster-pair list fixes the periodic image of every
    // cluster pair until the next rebuild, which wraps positions back.
    d.X[xb ^ 1][k][s] = x;
    xo[k] = x;
  }
  double r2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double u = (double)(xo[k] - d.xprune[k][s]);  // exact: one storage grid
    r2 += u * u;
  }
  return r2;
}

// One Cartesian component k of integrate_atom (same arithmetic; z is the
// normal z[k] of gauss4 rounded to T, as integrate_atom uses it): three lanes
// integrate an atom side by side.  Returns the squared displacement of this
// component from the position at the last prune.
template <typename T>
__device__ __forceinline__ double integrate_comp(const Dev<T> &d, int64_t s, int k, int xb, int vb,
                                                 bool pending, double Fk, T z) {
  const T h = (T)(0.5 * d.dt);
  const T c1 = (T)d.c1;
  const T im = d.aim[s], sd = d.nsd[s];
  // per-lane component: select the array, never index the argument block
  T *Vk = k == 0 ? d.V[vb][0] : (k == 1 ? d.V[vb][1] : d.V[vb][2]);
  const T *Xk = k == 0 ? d.X[xb][0] : (k == 1 ? d.X[xb][1] : d.X[xb][2]);
  T *Xn = k == 0 ? d.X[xb ^ 1][0] : (k == 1 ? d.X[xb ^ 1][1] : d.X[xb ^ 1][2]);
  const T *Xp = k == 0 ? d.xprune[0] : (k == 1 ? d.xprune[1] : d.xprune[2]);
  const T fa = (T)Fk;
  T v = Vk[s];
  T x = Xk[s];
  if (pending) v += h * fa * im;
  v += h * fa * im;
  x += h * v;
  v = c1 * v + sd * z;
  x += h * v;
  Vk[s] = v;
  Xn[s] = x;
  const double u = (double)(x - Xp[s]);  // exact: one storage grid
  return u * u;
}

// Largest displacement since the prune over the lanes of one walker, rounded
// up, into the buffer the next step's prune test reads (slot `slot` of the
// walker's PDISP_SLOTS: atomics on one address per walker would serialise).
// Every lane of the wave takes part; w < 0: nothing to record.
template <typename T>
__device__ __forceinline__ void record_disp(const Dev<T> &d, int lb, int w, int slot, double r2) {
  bool pend = w >= 0 && r2 > 0.0;
  unsigned long long bal = __ballot(pend);
  while (bal) {
    const int lead = __ffsll((long long)bal) - 1;
    const int wl = __shfl(w, lead, WAVE);
    double v = (pend && w == wl) ? r2 : 0.0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    if (lane_id() == lead)
      atomicMax(&d.pdisp[((int64_t)(lb ^ 1) * d.n_walkers + wl) * PDISP_SLOTS + (slot & (PDISP_SLOTS - 1))],
                __float_as_uint(__double2float_ru(sqrt(v))));
    if (w == wl) pend = false;
    bal = __ballot(pend);
  }
}

// Cross-lane sums on gfx950 without LDS: the halves of the wave swap data
// with v_permlane32_swap, the 16-lane rows with v_permlane16_swap, and lanes
// within a row exchange through DPP (row_ror:8, half-row mirror, quad
// permutations).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float halves_sum(float a, float b) {
  // lanes 0-31 get a[l] + a[l + 32], lanes 32-63 get b[l - 32] + b[l]
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float rows_sum(float a, float b) {
  // even rows (lanes 0-15, 32-47) get a summed over the row pair, odd rows b
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Transposed sum of the per-lane forces fx/fy/fz[ii] of the 8 i atoms over
// the 64 lanes: each stage halves the values a lane keeps (lanes 0-31 keep
// atoms 0-3 and lanes 32-63 atoms 4-7, then by 16-lane row, then by 8-lane
// half row), the last sums within 8 lanes; atom ii ends in lanes 8 ii ..
// 8 ii + 7.  About 50 VALU operations instead of 24 full-wave reductions.
__device__ __forceinline__ void reduce_transposed(const float (&fx)[CL], const float (&fy)[CL],
                                                  const float (&fz)[CL], float &Fx, float &Fy,
                                                  float &Fz) {
  float u[4][3];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    u[j][0] = halves_sum(fx[j], fx[j + 4]);
    u[j][1] = halves_sum(fy[j], fy[j + 4]);
    u[j][2] = halves_sum(fz[j], fz[j + 4]);
  }
  // lane in row r holds atom j + 2 r in w[j]
  float w[2][3];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) w[j][k] = rows_sum(u[j][k], u[j + 2][k]);
  const bool hi = (lane_id() & 8) != 0;
  float z[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float keep = hi ? w[1][k] : w[0][k], send = hi ? w[0][k] : w[1][k];
    z[k] = keep + dpp_f<0x128>(send);  // row_ror:8 (lane l ^ 8)
    z[k] += dpp_f<0x141>(z[k]);        // row_half_mirror (lane 7 - l within 8)
    z[k] += dpp_f<0x4E>(z[k]);         // quad_perm 2,3,0,1 (lane l ^ 2)
    z[k] += dpp_f<0xB1>(z[k]);         // quad_perm 1,0,3,2 (lane l ^ 1)
  }
  Fx = z[0];
  Fy = z[1];
  Fz = z[2];
}

// SHIFTED selects the soft-core form of the alchemical segment at compile time
// (both forms in one instantiation double the register allocation).
// The FP32 real-space Ewald forces kernel asks for at least 6 waves per SIMD
// (at most 80 VGPRs, no spills); asking 8 of any variant spills SGPRs and
// measured slower.
// EONLY (with ENERGY): energies only, no forces (the forward pass of the
// differentiable energy).
template <typename T, bool LB, bool ENERGY, bool INTEG, bool SHIFTED, bool EW, bool EONLY = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(!ENERGY && !INTEG && EW && sizeof(T) == 4 ? 6 : 1)))
void k_env(Dev<T> d, Range r, int xb, int vb, int lb) {
  static_assert(!EONLY || (ENERGY && !INTEG), "the energy-only variant evaluates energies");
  // the force half of the FP32 real-space Ewald table (4 KiB), staged in LDS
  // by the whole block before any wave leaves: one LDS read per pair
  // instead of a cached global gather
  constexpr bool EWL = EW && !ENERGY && sizeof(T) == 4;
  __shared__ float4 ewl[EWL ? EWTAB_N : 1];
  if constexpr (EWL) {
    for (int k = threadIdx.x; k < EWTAB_N; k += blockDim.x) ewl[k] = d.ewtab[k];
    __syncthreads();
  }
  const float4 *ewt = EWL ? ewl : d.ewtab;
  const int nb = (int)((r.en + 3) >> 2);
  const int lblk = xcd_block(nb);
  if (lblk >= nb) return;
  const int64_t e = r.e0 + (int64_t)lblk * 4 + uni(threadIdx.x >> 6);
  if (e >= r.e0 + r.en) return;
  const int64_t c = d.env_table[e];
  const int w = d.cl_walker[c];
  const WalkerMeta &m = d.meta[w];
  if (c - m.cl_begin >= d.n_env[w]) return;
  const int lane = lane_id();
  const int64_t s0 = c * CL;
  const T *X0 = d.X[xb][0], *X1 = d.X[xb][1], *X2 = d.X[xb][2];
  const int n = d.list_count[c];
  const int nenv = d.list_nenv[c];
  const bool need_lj = LB || (!EONLY && nenv < n);
  T xi[CL], yi[CL], zi[CL], qi[CL], ai[CL], bi[CL];
  int vmask = 0;
#pragma unroll
  for (int ii = 0; ii < CL; ++ii) {
    if (ENERGY) vmask |= (d.orig[s0 + ii] >= 0 ? 1 : 0) << ii;
    xi[ii] = X0[s0 + ii];
    yi[ii] = X1[s0 + ii];
    zi[ii] = X2[s0 + ii];
    qi[ii] = d.q[s0 + ii];
    ai[ii] = need_lj ? d.lja[s0 + ii] : (T)0;
    bi[ii] = need_lj ? d.ljb[s0 + ii] : (T)0;
  }
  T fx[CL], fy[CL], fz[CL];
#pragma unroll
  for (int ii = 0; ii < CL; ++ii) fx[ii] = fy[ii] = fz[ii] = (T)0;
  double eacc = 0.0;
  const T far = (T)(8.0 * m.B[0]);
  const uint32_t *lst = d.list + c * (int64_t)d.list_cap;
  // box shift of every image code for this wave's walker (lane = code)
  __shared__ T shtab[4][3][IMG_CODES];
  T *shx = shtab[threadIdx.x >> 6][0], *shy = shtab[threadIdx.x >> 6][1], *shz = shtab[threadIdx.x >> 6][2];
  shx[lane] = (T)img_x(lane) * (T)m.L[0];
  shy[lane] = (T)img_y(lane) * (T)m.L[1];
  shz[lane] = (T)img_z(lane) * (T)m.L[2];
  __builtin_amdgcn_wave_barrier();
  if constexpr (!EW) {
  // The pruned list, 64 j atoms per chunk (chunk 0 opens with the cluster's
  // own atoms: the self pairs are masked there).  The list streams from HBM
  // while the atoms it names are in L2: a chunk's entries are loaded two
  // chunks ahead, its atoms one chunk ahead, the gathers issued before the
  // entry loads (loads complete in order, so waiting for a gather does not
  // wait for HBM).  Two register sets take turns (no copies, which would
  // wait for loads in flight).  Slot offsets are 32-bit byte offsets (fewer
  // than 2^29 slots) so that the loads take a scalar base and a lane offset.
  const int nch = d.plist_n[e];
  typedef __attribute__((address_space(1))) const uint32_t gu32;
  gu32 *pl = (gu32 *)(d.plist + e * (int64_t)d.plist_cap);
  const uint32_t wsb = (uint32_t)(m.cl_begin * CL) * (uint32_t)sizeof(T);
  struct Jset {
    T x, y, z, q, a, b;
  };
  const int last = nch - 1;
  // each chunk's address passes an empty asm statement, so that the
  // compiler cannot match it with a later iteration's and sink the load
  auto entry = [&](int k) {
    gu32 *pk = pl + min(k, last) * WAVE;
    asm volatile("" : "+s"(pk));
    return __builtin_nontemporal_load(pk + lane);
  };
  auto gather = [&](uint32_t ent, Jset &j) {
    const int code = (int)(ent >> SHIFT_BITS);
    const uint32_t bo = wsb + (ent & CL_MASK) * (uint32_t)sizeof(T);
    j.x = ld_off(X0, bo) + shx[code];
    j.y = ld_off(X1, bo) + shy[code];
    j.z = ld_off(X2, bo) + shz[code];
    j.q = ld_off(d.q, bo);
    j.a = LB ? ld_off(d.lja, bo) : (T)0;
    j.b = LB ? ld_off(d.ljb, bo) : (T)0;
  };
  auto pairs = [&](const Jset &j) {
    env_pairs<T, LB, ENERGY, false, EW, EONLY>(d, xi, yi, zi, qi, ai, bi, s0, j.x, j.y, j.z, j.q, j.a,
                                               j.b, -1, vmask, fx, fy, fz, eacc, ewt);
  };
  if (nch > 0) {
    // chunk k sits in ja (k even) or jb (k odd); at step k the entries of
    // chunk k + 1 are in ua (k even) or ub (k odd)
    const uint32_t u0 = entry(0);
    uint32_t ua = entry(1), ub = entry(2);
    Jset ja, jb;
    gather(u0, ja);
    gather(ua, jb);
    ua = entry(3);
    const int js0 = (int)(m.cl_begin * CL + (u0 & CL_MASK));
    env_pairs<T, LB, ENERGY, true, EW, EONLY>(d, xi, yi, zi, qi, ai, bi, s0, ja.x, ja.y, ja.z, ja.q,
                                              ja.a, ja.b, js0, vmask, fx, fy, fz, eacc, ewt);
    int k = 1;
    for (; k + 1 < nch; k += 2) {
      gather(ub, ja);
      ub = entry(k + 3);
      pairs(jb);
      gather(ua, jb);
      ua = entry(k + 4);
      pairs(ja);
    }
    if (k < nch) pairs(jb);
  }
  } else {
    // Real-space Ewald: the table lookups leave the kernel latency-bound,
    // and the compact lists measured no faster than pruning the cluster
    // list on the fly, which costs no separate prune: cluster list here.
  // Candidate j atoms of list entries [e0, e0 + 8): lane -> (entry, atom).
  auto load_j = [&](int e0, T &xj, T &yj, T &zj, T &qj, T &aj, T &bj, int &js) {
    const int ee = e0 + (lane >> 3);
    xj = far;
    yj = far;
    zj = far;
    qj = (T)0;
    aj = (T)0;
    bj = (T)0;
    js = -1;
    if (ee < nenv) {
      const uint32_t ent = lst[ee];
      const int64_t J = ent & CL_MASK;
      const int code = (int)(ent >> SHIFT_BITS);
      js = (int)(J * CL + (lane & 7));
      xj = X0[js] + shx[code];
      yj = X1[js] + shy[code];
      zj = X2[js] + shz[code];
      qj = d.q[js];
      if (LB) {
        aj = d.lja[js];
        bj = d.ljb[js];
      }
    }
  };
  {
    // first 8 entries (the cluster's own entry among them) unpruned, with
    // the self pairs masked
    T xj, yj, zj, qj, aj, bj;
    int js;
    load_j(0, xj, yj, zj, qj, aj, bj, js);
    env_pairs<T, LB, ENERGY, true, EW, EONLY>(d, xi, yi, zi, qi, ai, bi, s0, xj, yj, zj, qj, aj, bj, js,
                                              vmask, fx, fy, fz, eacc, ewt);
  }
  if (nenv > CL) {
    // Remaining entries: a j atom farther than r_cut from the box of the 8
    // i atoms cannot interact with any of them, so it is dropped before the
    // pair arithmetic; survivors are compacted through a per-wave LDS ring
    // and evaluated 64 at a time.  Coordinates are exact multiples of the
    // storage grid, so the box gaps are exact and, with the same fma order as
    // r^2, the box distance never exceeds any member pair's r^2: no pair
    // inside the cutoff is dropped.
    __shared__ Ring<T, LB> ring[4];
    Ring<T, LB> &rg = ring[threadIdx.x >> 6];
    T lox = far, loy = far, loz = far, hix = -far, hiy = -far, hiz = -far;
#pragma unroll
    for (int ii = 0; ii < CL; ++ii) {
      if (d.orig[s0 + ii] >= 0) {
        lox = fmin(lox, xi[ii]);
        loy = fmin(loy, yi[ii]);
        loz = fmin(loz, zi[ii]);
        hix = fmax(hix, xi[ii]);
        hiy = fmax(hiy, yi[ii]);
        hiz = fmax(hiz, zi[ii]);
      }
    }
    int head = 0, cnt = 0;
    for (int e0 = CL; e0 < nenv; e0 += CL) {
      T xj, yj, zj, qj, aj, bj;
      int js;
      load_j(e0, xj, yj, zj, qj, aj, bj, js);
      const T gx = fmax(fmax(lox - xj, xj - hix), (T)0);
      const T gy = fmax(fmax(loy - yj, yj - hiy), (T)0);
      const T gz = fmax(fmax(loz - zj, zj - hiz), (T)0);
      const bool keep = fma(gz, gz, fma(gy, gy, gx * gx)) < d.rc2;
      const unsigned long long bal = __ballot(keep);
      if (keep) rg.put((head + cnt + lanes_below(bal)) & (RING - 1), xj, yj, zj, qj, aj, bj);
      cnt += __popcll(bal);
      if (cnt >= WAVE) {
        __builtin_amdgcn_wave_barrier();
        T x2, y2, z2, q2, a2, b2;
        rg.get((head + lane) & (RING - 1), x2, y2, z2, q2, a2, b2);
        __builtin_amdgcn_wave_barrier();
        env_pairs<T, LB, ENERGY, false, EW, EONLY>(d, xi, yi, zi, qi, ai, bi, s0, x2, y2, z2, q2, a2, b2, -1,
                                        vmask, fx, fy, fz, eacc, ewt);
        head = (head + WAVE) & (RING - 1);
        cnt -= WAVE;
      }
    }
    if (cnt > 0) {
      __builtin_amdgcn_wave_barrier();
      T x2 = far, y2 = far, z2 = far, q2 = (T)0, a2 = (T)0, b2 = (T)0;
      if (lane < cnt) rg.get((head + lane) & (RING - 1), x2, y2, z2, q2, a2, b2);
      env_pairs<T, LB, ENERGY, false, EW, EONLY>(d, xi, yi, zi, qi, ai, bi, s0, x2, y2, z2, q2, a2, b2, -1,
                                      vmask, fx, fy, fz, eacc, ewt);
    }
  }
  }
  if (!EONLY && nenv < n) {
    // alchemical partners: one atom per alchemical cluster (slot 0), 64 per pass
    const LamParams &lp = d.lp;
    double ce, dce, cv, dcv;
    channel(d.lambda[lb * d.n_walkers + w], lp.elec_start, lp.elec_end, lp.direction, lp.hi, ce, dce);
    channel(d.lambda[lb * d.n_walkers + w], lp.vdw_start, lp.vdw_end, lp.direction, lp.hi, cv, dcv);
    const T Asc = (T)(lp.sc_alpha * pow(1.0 - cv, (double)lp.sc_power));
    const T Dsc = (T)(lp.sc_shift * (1.0 - cv));
    for (int e0 = nenv; e0 < n; e0 += WAVE) {
      const int ee = e0 + lane;
      T xj = far, yj = far, zj = far, qj = (T)0, aj = (T)1, bj = (T)0;
      bool alch = false, valid = false;
      if (ee < n) {
        const uint32_t ent = lst[ee];
        const int64_t J = ent & CL_MASK;
        const int code = (int)(ent >> SHIFT_BITS);
        const int64_t js = J * CL;
        valid = d.orig[js] >= 0;
        xj = X0[js] + shx[code];
        yj = X1[js] + shy[code];
        zj = X2[js] + shz[code];
        qj = d.q[js];
        aj = d.lja[js];
        bj = d.ljb[js];
        alch = d.sol[js] != 0;
      }
      env_alch_pairs<T, SHIFTED, EW>(d, xi, yi, zi, qi, ai, bi, xj, yj, zj, qj, aj, bj, alch, valid,
                                 (T)cv, (T)ce, Asc, Dsc, fx, fy, fz);
    }
  }
  // the forces of the 8 i atoms summed over the wave: atom ii ends in
  // lanes 8 ii .. 8 ii + 7, whose first lane finishes the atom
  T Fx = (T)0, Fy = (T)0, Fz = (T)0;
  if constexpr (!EONLY) {
    if constexpr (sizeof(T) == 4) {
      reduce_transposed(fx, fy, fz, Fx, Fy, Fz);
    } else {
#pragma unroll
      for (int ii = 0; ii < CL; ++ii) {
        const T sx = wave_sum(fx[ii]), sy = wave_sum(fy[ii]), sz = wave_sum(fz[ii]);
        if ((lane >> 3) == ii) {
          Fx = sx;
          Fy = sy;
          Fz = sz;
        }
      }
    }
  }
  double eres = 0.0, dq = 0.0;
  // every lane of a group of 8 holds its atom's force sums; when stepping,
  // lanes 0-2 of the group integrate the x, y, z components side by side
  // (the restraint terms below are computed on each of them)
  const int kc = lane & 7;
  if (kc < (INTEG ? 3 : 1)) {
    const int64_t s = s0 + (lane >> 3);
    const bool valid = d.orig[s] >= 0;
    double F[3] = {(double)Fx, (double)Fy, (double)Fz};
    const T kr = d.rk[s];
    if (valid && kr != (T)0) {
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T dd0 = d.X[xb][k][s] - d.anc[k][s];
        const double dd = min_image((double)dd0, m.L[k]);
        F[k] -= (double)kr * dd;
        r2 += dd * dd;
      }
      eres = 0.5 * (double)kr * r2;
    }
    if (!EONLY && valid && d.dr_partner) {
      const int64_t a = m.atom_begin + d.orig[s];
      const int64_t b = d.dr_partner[a];
      if (b >= 0) {
        const DrTerm t = dr_term(d, m, xb, a, b, d.lambda[lb * d.n_walkers + w]);
        if (t.on)
#pragma unroll
          for (int k = 0; k < 3; ++k) F[k] += d.dr_k * t.e * t.u[k];
      }
    }
    if (EW && valid && (INTEG || ENERGY)) {
      // reciprocal-space force (the plain force launch of the PME step
      // leaves it to k_env_integrate); energy: half the atom's own-group
      // potential times its charge, minus the Ewald self term
#pragma unroll
      for (int k = 0; k < 3; ++k) F[k] += d.pme_frc[(int64_t)k * d.n_slots + s];
      if (ENERGY) {
        const double q = d.q64[s];
        eacc += 0.5 * q * d.pme_phi[s] - d.coulomb_k * d.ewald_beta * 0.56418958354775628 * q * q;
      }
    }
    if (INTEG) {
      if (valid) {
        const int64_t st = d.step[lb * d.n_walkers + w];
        const double Fk = kc == 0 ? F[0] : (kc == 1 ? F[1] : F[2]);
        T z;
        if constexpr (EW) {
          // no prune kernel with PME: draw here
          z = (T)gauss_comp(d.seed, (uint32_t)d.orig[s], (uint32_t)st, (uint32_t)w, 0u, kc);
        } else {
          z = kc == 0 ? d.noise[0][s] : (kc == 1 ? d.noise[1][s] : d.noise[2][s]);
        }
        dq = integrate_comp<T>(d, s, kc, xb, vb, st != *d.start_step, Fk, z);
      } else {
        T *Xn = kc == 0 ? d.X[xb ^ 1][0] : (kc == 1 ? d.X[xb ^ 1][1] : d.X[xb ^ 1][2]);
        const T *Xk = kc == 0 ? d.X[xb][0] : (kc == 1 ? d.X[xb][1] : d.X[xb][2]);
        Xn[s] = Xk[s];
      }
    } else if (!EONLY) {
#pragma unroll
      for (int k = 0; k < 3; ++k) d.fout[(int64_t)k * d.n_slots + s] = valid ? F[k] : 0.0;
    }
  }
  if (INTEG) {
    // the atom's squared displacement, summed in component order on lane 0
    // of its group
    const double d1 = __shfl_down(dq, 1, WAVE), d2 = __shfl_down(dq, 2, WAVE);
    dq = kc == 0 ? (dq + d1) + d2 : 0.0;
    record_disp(d, lb, w, (int)e, dq);
  }
  if (ENERGY) {
    const double et = wave_sum(eacc), er = wave_sum(eres);
    if (lane == 0) {
      d.cl_energy[c * 2] = et;
      d.cl_energy[c * 2 + 1] = er;
    }
  }
}

// ---------------------------------------------------------------------------
// alchemical kernel (FP64) and the per-walker lambda/ABF tail
// ---------------------------------------------------------------------------
struct PairOut {
  double fr, ulj, dulj, uc, duc;
  double dsig;  // dV_LJ/d(sigma_ij), shift included
  double g;     // shifted-force kernel 1/r - 1/rc + (r - rc)/rc^2
};

// Soft-core LJ at coupling c, written for both forms as phi = 4 eps c (y^2 - y):
//   form 0: y = 1 / (alpha (1-c)^p + (r/sig)^6)
//   form 1: y = sig^6 / s^3 with s = r^2 + delta (1 - c) (separation-shifted)
// so that F/r = -2 dphi/d(r^2) = 24 eps c (2y - 1) y (-dln y / d r^2) with
// -dln y/dr^2 = 3 u y / r^2 (form 0, u = (r/sig)^6) or 3 / s (form 1),
// dphi/dc = 4 eps ((y^2 - y) + c (2y - 1) dy/dc) with dy/dc = alpha p (1-c)^(p-1) y^2
// or 3 y delta / s, and dphi/dsig = 4 eps c (2y - 1) dy/dsig with
// dy/dsig = 6 u y^2 / sig or 6 y / sig.  Potential shift at r_cut with the same
// c.  Shifted-force Coulomb at ce.
struct SoftCore {
  int form, p;
  double alpha, delta;
};
// The coupling-dependent constants of the soft-core form at one c (the same
// for every pair of a walker at a step): form 1 delta (1 - c); form 0
// alpha (1 - c)^p and alpha p (1 - c)^(p - 1), hoisted out of the pair loop.
struct ScAt {
  double c, d1, A, dA;
};
__device__ __forceinline__ ScAt sc_at(const SoftCore &sc, double c) {
  ScAt a;
  a.c = c;
  a.d1 = sc.delta * (1.0 - c);
  a.A = sc.alpha * pow(1.0 - c, (double)sc.p);
  a.dA = sc.p >= 1 ? sc.alpha * (double)sc.p * pow(1.0 - c, (double)(sc.p - 1)) : 0.0;
  return a;
}

__device__ __forceinline__ void softcore_y(const SoftCore &sc, const ScAt &at, double r2,
                                           double sig2, double &y, double &dydc, double &fy,
                                           double &dys) {
  if (sc.form == 1) {
    const double s = r2 + at.d1;
    const double w = sig2 / s;
    y = w * w * w;
    dydc = 3.0 * y * sc.delta / s;
    fy = 3.0 * y / s;      // y (-dln y / d r^2)
    dys = 6.0 * y;         // sig dy/dsig
  } else {
    const double t = r2 / sig2;
    const double u = t * t * t;
    y = 1.0 / (at.A + u);
    dydc = at.dA * y * y;
    fy = 3.0 * u * y * y / r2;
    dys = 6.0 * u * y * y;
  }
}

__device__ __forceinline__ PairOut alch_pair(double r2, double sig, double eps, double qq,
                                            const ScAt &at, double ce, const SoftCore &scf,
                                            double rc, double beta) {
  PairOut o = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double r = sqrt(r2);
  const double cv = at.c;
  if (eps != 0.0) {
    const double sig2 = sig * sig;
    double y, dydc, fy, dys, yc, dycc, fyc, dysc;
    softcore_y(scf, at, r2, sig2, y, dydc, fy, dys);
    softcore_y(scf, at, rc * rc, sig2, yc, dycc, fyc, dysc);
    o.ulj = 4.0 * eps * cv * ((y * y - y) - (yc * yc - yc));
    o.dulj = 4.0 * eps * (((y * y - y) + cv * (2.0 * y - 1.0) * dydc) -
                          ((yc * yc - yc) + cv * (2.0 * yc - 1.0) * dycc));
    o.fr = 8.0 * eps * cv * (2.0 * y - 1.0) * fy;
    o.dsig = 4.0 * eps * cv * ((2.0 * y - 1.0) * dys - (2.0 * yc - 1.0) * dysc) / sig;
  }
  if (qq != 0.0) {
    // beta > 0: real-space Ewald kernel erfc(beta r)/r cut at rc
    const double g = beta > 0.0 ? erfc(beta * r) / r : 1.0 / r - 1.0 / rc + (r - rc) / (rc * rc);
    o.g = g;
    o.duc = qq * g;
    if (ce != 0.0) {
      o.uc = ce * qq * g;
      o.fr += beta > 0.0 ? ce * qq * (g + 1.1283791670955126 * beta * exp(-beta * beta * r2)) / r2
                         : ce * qq * (1.0 / r2 - 1.0 / (rc * rc)) / r;
    }
  }
  return o;
}

template <typename T, bool ENERGY, bool INTEG>
__device__ void alch_tail(const Dev<T> &d, int w, int xb, int vb, int lb) {
  const WalkerMeta &m = d.meta[w];
  const int lane = lane_id();
  const int W = d.n_walkers;
  const double lam = d.lambda[lb * W + w];
  const int64_t step = d.step[lb * W + w];
  const bool pending = step != *d.start_step;
  double gr = 0.0, ur = 0.0, g = 0.0;
  for (int t = lane; t < m.n_acl; t += WAVE) {
    const int64_t k = m.item_begin + t;
    const int64_t s = (m.cl_begin + m.cap_env + t) * CL;
    double F[3] = {d.item_force[k * 3], d.item_force[k * 3 + 1], d.item_force[k * 3 + 2]};
    g += d.item_dudl[k];
    const double k0 = d.k0_64[s], k1 = d.k1_64[s];
    if (k0 != 0.0 || k1 != 0.0) {
      const double kl = k0 + lam * (k1 - k0);
      double r2 = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double dd = min_image((double)(d.X[xb][q][s] - d.anc[q][s]), m.L[q]);
        F[q] -= kl * dd;
        r2 += dd * dd;
      }
      gr += 0.5 * (k1 - k0) * r2;
      ur += 0.5 * kl * r2;
    }
    if (d.dr_partner) {
      const int64_t a = m.atom_begin + d.orig[s];
      const int64_t b = d.dr_partner[a];
      if (b >= 0) {
        const DrTerm t = dr_term(d, m, xb, a, b, lam);
        if (t.on)
#pragma unroll
          for (int q = 0; q < 3; ++q) F[q] += d.dr_k * t.e * t.u[q];
      }
    }
    if (INTEG) {
      (void)integrate_atom<T>(d, s, xb, vb, w, step, pending, F);
    } else {
#pragma unroll
      for (int q = 0; q < 3; ++q) d.fout[(int64_t)q * d.n_slots + s] = F[q];
    }
  }
  double G = wave_sum(g) + wave_sum(gr);
  // neutralising background of the Ewald sum: -pi k Q^2 / (2 V beta^2) split
  // as E-E, S-S and the cross part, which is scaled by ce like V_x
  double bg[3] = {0.0, 0.0, 0.0}, bce = 1.0;
  if (d.pme_on) {
    const double *qs = d.pme_qs + 4 * w;
    const double f = -3.14159265358979323846 * d.coulomb_k /
                     (m.L[0] * m.L[1] * m.L[2] * d.ewald_beta * d.ewald_beta);
    bg[0] = 0.5 * f * qs[0] * qs[0];
    bg[1] = 0.5 * f * qs[1] * qs[1];
    bg[2] = f * qs[0] * qs[1];
    double dbce;
    channel(lam, d.lp.elec_start, d.lp.elec_end, d.lp.direction, d.lp.hi, bce, dbce);
    G += dbce * bg[2];
  }
  double udr = 0.0;
  if (d.dr_pair && d.dr_pair[2 * w] >= 0) {
    const DrTerm t = dr_term(d, m, xb, d.dr_pair[2 * w], d.dr_pair[2 * w + 1], lam);
    if (t.on) {
      G += -d.dr_k * t.e * t.dm1;
      udr = 0.5 * d.dr_k * t.e * t.e;
    }
  }
  if (ENERGY) {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      double e = 0.0;
      for (int t = lane; t < m.n_acl; t += WAVE) e += d.item_energy[(m.item_begin + t) * 5 + q];
      e = wave_sum(e);
      if (q == 4) e += wave_sum(ur) + udr;
      if (q == 0) e += bg[0];
      if (q == 1) e += bg[1];
      if (q == 3) e += bce * bg[2];
      if (lane == 0) d.energy[w * 5 + q] = e;
    }
  }
  if (!INTEG) {
    if (lane == 0) {
      d.dudl[w] = G;
      d.ticket[w] = 0u;
    }
    return;
  }
  const LamParams &lp = d.lp;
  // ABF: bias from the frozen accumulator, then this step's sample
  if (lane == 0) {
    double bias = 0.0;
    if (lp.abf_on) {
      int b = (int)floor((lam - lp.lo) / lp.bin_w);
      b = b > lp.n_bins - 1 ? lp.n_bins - 1 : (b < 0 ? 0 : b);
      const int64_t li = (int64_t)w * lp.n_bins + b;
      const int64_t n = d.bin_count[b] + d.loc_count[li];
      const double sum = d.bin_sum[b] + d.loc_sum[li];
      if (n > 0) {
        double ramp = (double)n / (double)lp.full_samples;
        ramp = ramp > 1.0 ? 1.0 : ramp;
        bias = ramp * (sum / (double)n);
      }
      d.loc_count[li] += 1;
      d.loc_sum[li] += G;
      d.loc_sum2[li] += G * G;
    }
    d.dudl[w] = G;
    d.bias[w] = bias;
    double l = lam, p = d.p_lambda[w];
    uint32_t st = 0u;
    if (!lp.fixed_lambda) {
      const double h = 0.5 * d.dt;
      const double fl = -G + bias;
      if (pending) p += h * fl;
      p += h * fl;
      l += h * p / lp.m_lambda;
      if (l < lp.lo) {
        l = 2.0 * lp.lo - l;
        p = -p;
      } else if (l > lp.hi) {
        l = 2.0 * lp.hi - l;
        p = -p;
      }
      if (l < lp.lo || l > lp.hi) {
        l = l < lp.lo ? lp.lo : lp.hi;
        st |= 2u;
      }
      double z[4];
      gauss4(d.seed, LAMBDA_ATOM, (uint32_t)step, (uint32_t)w, 0u, z);
      p = lp.c1l * p + lp.sdl * z[0];
      l += h * p / lp.m_lambda;
      if (l < lp.lo) {
        l = 2.0 * lp.lo - l;
        p = -p;
      } else if (l > lp.hi) {
        l = 2.0 * lp.hi - l;
        p = -p;
      }
      if (l < lp.lo || l > lp.hi) {
        l = l < lp.lo ? lp.lo : lp.hi;
        st |= 2u;
      }
    }
    if (!isfinite(G) || !isfinite(l) || !isfinite(p)) st |= 1u;
    if (st) atomicOr(&d.status[w], st);
    d.lambda[(lb ^ 1) * W + w] = l;
    d.p_lambda[w] = p;
    d.step[(lb ^ 1) * W + w] = step + 1;
    d.ticket[w] = 0u;
    __threadfence();
  }
  // last walker of the step merges the samples in walker order every K steps
  unsigned old = 0;
  if (lane == 0) old = atomicAdd(d.gticket, 1u);
  old = __shfl(old, 0, WAVE);
  if (old != (unsigned)(W - 1)) return;
  __threadfence();
  if (lp.abf_on && ((step + 1) % lp.share_interval) == 0) {
    for (int b = lane; b < lp.n_bins; b += WAVE) {
      int64_t n = d.bin_count[b];
      double s1 = d.bin_sum[b], s2 = d.bin_sum2[b];
      for (int v = 0; v < W; ++v) {
        const int64_t li = (int64_t)v * lp.n_bins + b;
        n += d.loc_count[li];
        s1 += d.loc_sum[li];
        s2 += d.loc_sum2[li];
        d.loc_count[li] = 0;
        d.loc_sum[li] = 0.0;
        d.loc_sum2[li] = 0.0;
      }
      d.bin_count[b] = n;
      d.bin_sum[b] = s1;
      d.bin_sum2[b] = s2;
    }
  }
  if (lane == 0) *d.gticket = 0u;
}

// One 256-thread block per alchemical atom: its four waves share the atom's
// neighbour list, each lane one partner per pass (FP64), and the block
// reduces force, dV/dlambda and energies in a fixed order (no atomics).  The
// block that completes a walker's set runs the walker's lambda/ABF tail.
// Stepping without PME: at most 96 VGPRs, as the environment kernel it runs beside: a
// wave of it fits where a wave of that kernel retires.
// ENERGY: the walker's energy parts (alchemical side); PGRAD: dV/d(eps,
// sigma, q) of the block's atom; INTEG: the stepping tail.
template <typename T, bool ENERGY, bool INTEG, bool PGRAD, bool EW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(INTEG && !EW ? 5 : 1)))
void k_alch(Dev<T> d, Range r, int xb, int vb, int lb) {
  constexpr int NACC = PGRAD ? 12 : (ENERGY ? 9 : 4);
  __shared__ double red[4][NACC];
  __shared__ int is_last;
  const int64_t k = r.i0 + blockIdx.x;
  if (k >= r.i0 + r.in_) return;
  const int w = d.item_walker[k];
  const int64_t c = d.alch_cluster[k];
  const WalkerMeta &m = d.meta[w];
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  const LamParams &lp = d.lp;
  double ce, dce, cv, dcv;
  const double lam = d.lambda[lb * d.n_walkers + w];
  channel(lam, lp.elec_start, lp.elec_end, lp.direction, lp.hi, ce, dce);
  channel(lam, lp.vdw_start, lp.vdw_end, lp.direction, lp.hi, cv, dcv);
  // 0-2 force, 3 dV/dlambda, 4-8 energies, 9-11 dV/d(eps, sigma, q) of atom i
  double acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q) acc[q] = 0.0;
  if (c >= 0) {
    const int64_t si = c * CL;
    const double xi = (double)d.X[xb][0][si], yi = (double)d.X[xb][1][si],
                 zi = (double)d.X[xb][2][si];
    const double qi = d.q64[si], sgi = d.sig64[si], epi = d.eps64[si];
    const int soli = d.sol[si];
    const int n = d.list_count[c];
    const double rc = d.r_cut, rc2 = rc * rc;
    const SoftCore scf = {lp.sc_form, lp.sc_power, lp.sc_alpha, lp.sc_shift};
    // soft-core constants of the alchemical pairs (c_v) and of the others (c = 1)
    double sv_d1, sv_A, sv_dA, s1_d1, s1_A, s1_dA;
    {
      const ScAt a = sc_at(scf, cv), b = sc_at(scf, 1.0);
      sv_d1 = a.d1;
      sv_A = a.A;
      sv_dA = a.dA;
      s1_d1 = b.d1;
      s1_A = b.A;
      s1_dA = b.dA;
    }
    for (int e0 = wv * CL; e0 < n; e0 += 4 * CL) {
      const int ee = e0 + (lane >> 3);
      if (ee >= n) continue;
      const uint32_t ent = d.list[c * (int64_t)d.list_cap + ee];
      const int64_t J = ent & CL_MASK;
      const int code = (int)(ent >> SHIFT_BITS);
      const int64_t js = J * CL + (lane & 7);
      if (d.orig[js] < 0 || js == si) continue;
      const double dx = ((double)d.X[xb][0][js] + img_x(code) * m.L[0]) - xi;
      const double dy = ((double)d.X[xb][1][js] + img_y(code) * m.L[1]) - yi;
      const double dz = ((double)d.X[xb][2][js] + img_z(code) * m.L[2]) - zi;
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (!(r2 < rc2)) continue;
      const int solj = d.sol[js];
      const bool alch = soli != solj;
      const double sig = 0.5 * (sgi + d.sig64[js]);
      const double eps = sqrt(epi * d.eps64[js]);
      const double qq = d.coulomb_k * qi * d.q64[js];
      ScAt at;
      at.c = alch ? cv : 1.0;
      at.d1 = alch ? sv_d1 : s1_d1;
      at.A = alch ? sv_A : s1_A;
      at.dA = alch ? sv_dA : s1_dA;
      const PairOut o = alch_pair(r2, sig, eps, qq, at, alch ? ce : 1.0, scf, rc,
                                  EW ? d.ewald_beta : 0.0);
      acc[0] -= o.fr * dx;
      acc[1] -= o.fr * dy;
      acc[2] -= o.fr * dz;
      if (alch && soli) {
        if (dcv != 0.0) acc[3] += dcv * o.dulj;
        if (dce != 0.0) acc[3] += dce * o.duc;
      }
      if (PGRAD) {
        // eps_ij = sqrt(eps_i eps_j), sig_ij = (sig_i + sig_j)/2, q_i q_j
        if (epi != 0.0) acc[9] += o.ulj / (2.0 * epi);
        acc[10] += 0.5 * o.dsig;
        acc[11] += (alch ? ce : 1.0) * d.coulomb_k * d.q64[js] * o.g;
      }
      if (ENERGY) {
        const bool isAj = (J - m.cl_begin) >= m.cap_env;
        if (!isAj || si < js) {
          if (alch) {
            acc[6] += o.ulj;
            acc[7] += o.uc;
          } else if (soli) {
            acc[5] += o.ulj + o.uc;
          } else {
            acc[4] += o.ulj + o.uc;
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NACC; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) red[wv][q] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[NACC];
#pragma unroll
    for (int q = 0; q < NACC; ++q) tot[q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
    if (EW && c >= 0) {
      // reciprocal space: force from the gather; dV/dlambda of the cross
      // term dce q phi_E for group atoms; energies and dV/dq with the self term
      const int64_t si = c * CL;
      const double q = d.q64[si], po = d.pme_phi[si], pt = d.pme_phi[d.n_slots + si];
      const bool so = d.sol[si] != 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) tot[a] += d.pme_frc[(int64_t)a * d.n_slots + si];
      if (so) tot[3] += dce * q * pt;
      const double kb = d.coulomb_k * d.ewald_beta * 0.56418958354775628;  // k beta / sqrt(pi)
      if (ENERGY) {
        const double es = 0.5 * q * po - kb * q * q;
        if (so) tot[5] += es;  // constant indices keep tot in registers
        else tot[4] += es;
        if (so) tot[7] += ce * q * pt;
      }
      if (PGRAD) {
        const double *qs = d.pme_qs + 4 * w;
        const double V = m.L[0] * m.L[1] * m.L[2];
        const double qo = so ? qs[1] : qs[0], qt = so ? qs[0] : qs[1];
        tot[11] += (po + ce * pt) - 2.0 * kb * q -
                   3.14159265358979323846 * d.coulomb_k * (qo + ce * qt) / (V * d.ewald_beta * d.ewald_beta);
      }
    }
    d.item_force[k * 3] = tot[0];
    d.item_force[k * 3 + 1] = tot[1];
    d.item_force[k * 3 + 2] = tot[2];
    d.item_dudl[k] = tot[3];
    if (ENERGY)
      for (int q = 0; q < 5; ++q) d.item_energy[k * 5 + q] = tot[4 + q];
    if (PGRAD)
      for (int q = 0; q < 3; ++q) d.item_pgrad[k * 3 + q] = tot[9 + q];
    __threadfence();
    const unsigned old = atomicAdd(&d.ticket[w], 1u);
    is_last = old == (unsigned)(m.item_cap - 1);
  }
  __syncthreads();
  if (!is_last || wv != 0) return;
  __threadfence();
  alch_tail<T, ENERGY, INTEG>(d, w, xb, vb, lb);
}

// ---------------------------------------------------------------------------
// neighbour-set export and pair counting (FP64 decision, no fused ops)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_pairs(Dev<T> d, Range r, int xb, int mode) {
  const int64_t c = r.c0 + (int64_t)blockIdx.x * 4 + uni(threadIdx.x >> 6);
  if (c >= r.c0 + r.cn) return;
  const int w = d.cl_walker[c];
  const WalkerMeta &m = d.meta[w];
  if (!cluster_used(m, d.n_env[w], c)) return;
  const bool isA = (c - m.cl_begin) >= m.cap_env;
  const int lane = lane_id();
  // environment clusters: environment entries only (alchemical pairs are
  // enumerated from the alchemical side)
  const int n = isA ? d.list_count[c] : d.list_nenv[c];
  const double lim = mode == 0 ? d.r_list * d.r_list : d.r_cut * d.r_cut;
  unsigned long long cnt = 0, cnt_env = 0;
  for (int e0 = 0; e0 < n; e0 += CL) {
    const int ee = e0 + (lane >> 3);
    if (ee >= n) continue;
    const uint32_t ent = d.list[c * (int64_t)d.list_cap + ee];
    const int64_t J = ent & CL_MASK;
    const int code = (int)(ent >> SHIFT_BITS);
    const int64_t js = J * CL + (lane & 7);
    const int oj = d.orig[js];
    if (oj < 0) continue;
    const bool isAj = (J - m.cl_begin) >= m.cap_env;
    const double xj = __dadd_rn((double)d.X[xb][0][js], img_x(code) * m.L[0]);
    const double yj = __dadd_rn((double)d.X[xb][1][js], img_y(code) * m.L[1]);
    const double zj = __dadd_rn((double)d.X[xb][2][js], img_z(code) * m.L[2]);
    for (int ii = 0; ii < CL; ++ii) {
      const int64_t si = c * CL + ii;
      const int oi = d.orig[si];
      if (oi < 0 || si == js) continue;
      const double dx = __dsub_rn(xj, (double)d.X[xb][0][si]);
      const double dy = __dsub_rn(yj, (double)d.X[xb][1][si]);
      const double dz = __dsub_rn(zj, (double)d.X[xb][2][si]);
      const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
      if (!(r2 < lim)) continue;
      const bool emit = (isA && !isAj) || oi < oj;
      if (!emit) continue;
      if (mode == 0) {
        const unsigned long long pos = atomicAdd(&d.pair_n[w], 1ull);
        if ((int64_t)pos < d.pair_max) {
          d.pair_out[2 * pos] = oi < oj ? oi : oj;
          d.pair_out[2 * pos + 1] = oi < oj ? oj : oi;
        }
      } else {
        ++cnt;
        if (!isA) ++cnt_env;
      }
    }
  }
  if (mode != 0) {
    cnt = wave_sum(cnt);
    cnt_env = wave_sum(cnt_env);
    if (lane == 0 && cnt) atomicAdd(&d.pair_n[w], cnt);
    if (lane == 0 && cnt_env) atomicAdd(&d.pair_n[d.n_walkers + w], cnt_env);
  }
}

// ---------------------------------------------------------------------------
// initialisation and caller-order transfers
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_init_vel(Dev<T> d, int vb) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= d.n_atoms) return;
  const int w = d.atom_walker[a];
  const WalkerMeta &m = d.meta[w];
  double z[4];
  gauss4(d.seed, (uint32_t)(a - m.atom_begin), 0u, (uint32_t)w, 1u, z);
  const double sd = sqrt(d.kT * d.accel / d.a_mass[a]);
  const int s = d.slot_of[a];
#pragma unroll
  for (int k = 0; k < 3; ++k) d.V[vb][k][s] = (T)(sd * z[k]);
}

template <typename T>
__global__ void k_init_lambda(Dev<T> d, const double *lam0, const double *p0, int lb) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int W = d.n_walkers;
  if (w < W) {
    d.lambda[lb * W + w] = lam0[w];
    d.lambda[(lb ^ 1) * W + w] = lam0[w];
    if (p0) {
      d.p_lambda[w] = p0[w];
    } else {
      double z[4];
      gauss4(d.seed, LAMBDA_ATOM, 0u, (uint32_t)w, 1u, z);
      d.p_lambda[w] = sqrt(d.lp.m_lambda * d.lp.kT_lambda) * z[0];
    }
    d.dudl[w] = 0.0;
    d.bias[w] = 0.0;
    d.step[w] = 0;
    d.step[W + w] = 0;
    d.ticket[w] = 0u;
    d.status[w] = 0u;
    for (int b = 0; b < d.lp.n_bins; ++b) {
      d.loc_count[(int64_t)w * d.lp.n_bins + b] = 0;
      d.loc_sum[(int64_t)w * d.lp.n_bins + b] = 0.0;
      d.loc_sum2[(int64_t)w * d.lp.n_bins + b] = 0.0;
    }
  }
  if (w == 0) {
    *d.gticket = 0u;
    *d.start_step = 0;
    for (int b = 0; b < d.lp.n_bins; ++b) {
      d.bin_count[b] = 0;
      d.bin_sum[b] = 0.0;
      d.bin_sum2[b] = 0.0;
    }
  }
}

template <typename T>
__global__ void k_gather_atoms(Dev<T> d, int xb, int vb, double *pos, double *vel) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= d.n_atoms) return;
  const WalkerMeta &m = d.meta[d.atom_walker[a]];
  const int s = d.slot_of[a];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (pos) pos[3 * a + k] = (double)wrap_pos<T>(d.X[xb][k][s], (T)m.B[k], (T)m.L[k]) - m.B[k];
    if (vel) vel[3 * a + k] = (double)d.V[vb][k][s];
  }
}

// pos: B-offset positions already rounded on the host (exact in T).
template <typename T>
__global__ void k_scatter_atoms(Dev<T> d, int xb, int vb, const double *pos, const double *vel) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= d.n_atoms) return;
  const int s = d.slot_of[a];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (pos) d.X[xb][k][s] = (T)pos[3 * a + k];
    if (vel) d.V[vb][k][s] = (T)vel[3 * a + k];
  }
}

template <typename T>
__global__ void k_gather_forces(Dev<T> d, double *f) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= d.n_atoms) return;
  const int s = d.slot_of[a];
#pragma unroll
  for (int k = 0; k < 3; ++k) f[3 * a + k] = d.fout[(int64_t)k * d.n_slots + s];
}

// ---------------------------------------------------------------------------
// differentiable energy: configuration in, total energy and gradients out
// ---------------------------------------------------------------------------
// Positions are wrapped into [0, L) and rounded to the storage grid B + x
// exactly as the host does for uploads; lambda goes to the buffer that the
// next evaluation reads.
template <typename T>
__global__ void k_set_config(Dev<T> d, int xb, int lb, const double *pos, const double *lam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos && i < d.n_atoms) {
    const WalkerMeta &m = d.meta[d.atom_walker[i]];
    const int s = d.slot_of[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double L = m.L[k], B = m.B[k];
      double v = pos[3 * i + k];
      v = v - L * floor(v / L);
      if (v >= L) v -= L;
      double X = (double)((T)B + (T)v);
      if (X >= B + L) X -= L;
      if (X < B) X += L;
      d.X[xb][k][s] = (T)X;
    }
  }
  if (lam && i < d.n_walkers) d.lambda[lb * d.n_walkers + i] = lam[i];
}

// Solute parameters (eps, sigma, q) into the caller-order atom arrays; the
// rebuild that follows derives every per-slot copy from them.
template <typename T>
__global__ void k_set_params(Dev<T> d, const double *par) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n_solute) return;
  const int a = d.solute_atom[i];
  d.a_eps[a] = par[3 * i];
  d.a_sig[a] = par[3 * i + 1];
  d.a_q[a] = par[3 * i + 2];
}

// One block per walker: environment cluster energies summed in a fixed
// order, then the alchemical-side parts.
template <typename T>
__global__ __launch_bounds__(256) void k_energy_total(Dev<T> d, double *out) {
  __shared__ double sm[4][2];
  const int w = blockIdx.x;
  const WalkerMeta &m = d.meta[w];
  const int ne = d.n_env[w];
  double ee = 0.0, er = 0.0;
  for (int c = threadIdx.x; c < ne; c += blockDim.x) {
    ee += d.cl_energy[2 * (m.cl_begin + c)];
    er += d.cl_energy[2 * (m.cl_begin + c) + 1];
  }
  ee = wave_sum(ee);
  er = wave_sum(er);
  const int wv = threadIdx.x >> 6;
  if (lane_id() == 0) {
    sm[wv][0] = ee;
    sm[wv][1] = er;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double se = ((sm[0][0] + sm[1][0]) + sm[2][0]) + sm[3][0];
    const double sr = ((sm[0][1] + sm[1][1]) + sm[2][1]) + sm[3][1];
    const double *e = d.energy + 5 * w;
    out[w] = ((((e[0] + se) + e[1]) + e[2]) + e[3]) + (e[4] + sr);
  }
}

// gpos = g_w dV/dx = -g_w F, glam = g_w dV/dlambda, gpar = g_w dV/d(eps, sigma, q).
template <typename T>
__global__ void k_energy_grads(Dev<T> d, const double *g, double *gpos, double *glam,
                               double *gpar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gpos && i < d.n_atoms) {
    const double gw = g[d.atom_walker[i]];
    const int s = d.slot_of[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) gpos[3 * i + k] = -gw * d.fout[(int64_t)k * d.n_slots + s];
  }
  if (glam && i < d.n_walkers) glam[i] = g[i] * d.dudl[i];
  if (gpar && i < d.n_solute) {
    const int a = d.solute_atom[i];
    const int w = d.atom_walker[a];
    const WalkerMeta &m = d.meta[w];
    // the t-th alchemical cluster of a walker is its t-th alchemical block
    const int64_t c = d.slot_of[a] / CL;
    const int64_t k = m.item_begin + (c - m.cl_begin - m.cap_env);
#pragma unroll
    for (int q = 0; q < 3; ++q) gpar[3 * i + q] = g[w] * d.item_pgrad[3 * k + q];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void k_fill_u64(unsigned long long *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

template <typename T>
hipError_t Launch<T>::rebuild(const Dev<T> &d, const Range &r, int xb, int vb, int check,
                              hipStream_t s) {
  if (r.an <= 0) return hipSuccess;
  k_fill_i32<<<nblk(r.kn, 256), 256, 0, s>>>(d.col_count + r.k0, r.kn, 0);
  k_key<T><<<nblk(r.cn * CL, 256), 256, 0, s>>>(d, r, xb, check);
  if (check) k_skin<T><<<(unsigned)(r.wn * SKIN_PARTS), 256, 0, s>>>(d, r);
  k_scan<T><<<(unsigned)r.wn, 256, 0, s>>>(d, r, check);
  k_members<T><<<nblk(r.cn * CL, 256), 256, 0, s>>>(d, r);
  k_rank<T><<<(unsigned)r.kn, 256, 0, s>>>(d, r, xb);
  k_clear_slots<T><<<nblk(r.cn * CL, 256), 256, 0, s>>>(d, r, xb ^ 1, vb ^ 1);
  k_scatter<T><<<nblk(r.an, 256), 256, 0, s>>>(d, r, xb, vb, xb ^ 1, vb ^ 1);
  k_bbox<T><<<nblk(r.cn, 256), 256, 0, s>>>(d, r, xb ^ 1);
  k_list<T><<<nblk(r.cn, 4), 256, 0, s>>>(d, r);
  return hipGetLastError();
}

// energy: 0 forces only, 1 forces and energies, 2 energies only
template <typename T, bool SH, bool EW>
static void env_launch_form(const Dev<T> &d, const Range &r, int xb, int vb, int lb, int energy,
                            bool integ, unsigned grid, hipStream_t s) {
  if (d.uniform_lj) {
    if (integ) k_env<T, false, false, true, SH, EW><<<grid, 256, 0, s>>>(d, r, xb, vb, lb);
    else if (energy == 2) k_env<T, false, true, false, SH, EW, true><<<grid, 256, 0, s>>>(d, r, xb, vb, lb);
    else if (energy == 1) k_env<T, false, true, false, SH, EW><<<grid, 256, 0, s>>>(d, r, xb, vb, lb);
    else k_env<T, false, false, false, SH, EW><<<grid, 256, 0, s>>>(d, r, xb, vb, lb);
  } else {
    if (integ) k_env<T, true, false, true, SH, EW><<<grid, 256, 0, s>>>(d, r, xb, vb, lb);
    else if (energy == 2) k_env<T, true, true, false, SH, EW, true><<<grid, 256, 0, s>>>(d, r, xb, vb, lb);
    else if (energy == 1) k_env<T, true, true, false, SH, EW><<<grid, 256, 0, s>>>(d, r, xb, vb, lb);
    else k_env<T, true, false, false, SH, EW><<<grid, 256, 0, s>>>(d, r, xb, vb, lb);
  }
}

template <typename T>
static void env_launch(const Dev<T> &d, const Range &r, int xb, int vb, int lb, int energy,
                       bool integ, hipStream_t s) {
  const int nb = (int)((r.en + 3) / 4);
  const unsigned grid = (unsigned)(8 * ((nb + 7) / 8));
  if (grid == 0) return;
  if (d.pme_on) {
    if (d.lp.sc_form == 1) env_launch_form<T, true, true>(d, r, xb, vb, lb, energy, integ, grid, s);
    else env_launch_form<T, false, true>(d, r, xb, vb, lb, energy, integ, grid, s);
  } else {
    if (d.lp.sc_form == 1) env_launch_form<T, true, false>(d, r, xb, vb, lb, energy, integ, grid, s);
    else env_launch_form<T, false, false>(d, r, xb, vb, lb, energy, integ, grid, s);
  }
}

// PME step, environment side: k_env writes the pair, restraint and
// distance-restraint forces (so that it can run beside the reciprocal-space
// chain); this kernel adds the reciprocal force and integrates, one thread
// per slot of the environment clusters in use (the same arithmetic, in the
// same order, as the fused epilogue of the other stepping launch).
template <typename T>
__global__ __launch_bounds__(256) void k_env_integrate(Dev<T> d, Range r, int xb, int vb, int lb) {
  const int64_t s = r.c0 * CL + (int64_t)blockIdx.x * 256 + threadIdx.x;
  int wd = -1;  // walker of a displacement to record
  double dq = 0.0;
  if (s < (r.c0 + r.cn) * CL) {
    const int64_t c = s / CL;
    const int w = d.cl_walker[c];
    const WalkerMeta &m = d.meta[w];
    if (c - m.cl_begin < d.n_env[w]) {  // not an unused or alchemical cluster
      const int64_t S = d.n_slots;
      if (d.orig[s] >= 0) {
        double F[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) F[k] = d.fout[k * S + s] + d.pme_frc[k * S + s];
        const int64_t st = d.step[lb * d.n_walkers + w];
        dq = integrate_atom<T>(d, s, xb, vb, w, st, st != *d.start_step, F);
        wd = w;
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) d.X[xb ^ 1][k][s] = d.X[xb][k][s];
      }
    }
  }
  record_disp(d, lb, wd, (int)blockIdx.x, dq);
}

// Reciprocal-space force added to the forces-only output of k_env (which
// leaves it to k_env_integrate on the stepping path): the gradient
// evaluation with PME.
template <typename T>
__global__ __launch_bounds__(256) void k_env_recip(Dev<T> d, Range r) {
  const int64_t s = r.c0 * CL + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= (r.c0 + r.cn) * CL) return;
  const int64_t c = s / CL;
  const int w = d.cl_walker[c];
  const WalkerMeta &m = d.meta[w];
  if (c - m.cl_begin >= d.n_env[w] || d.orig[s] < 0) return;
  const int64_t S = d.n_slots;
#pragma unroll
  for (int k = 0; k < 3; ++k) d.fout[k * S + s] += d.pme_frc[k * S + s];
}

// The alchemical kernel, without or with the real-space Ewald pair (the
// Ewald form compiled in only where PME is on: it raises the kernel's
// register count, which the environment kernel beside it pays for).
template <typename T, bool ENERGY, bool INTEG, bool PGRAD>
void alch_launch(const Dev<T> &d, const Range &r, int xb, int vb, int lb, hipStream_t s) {
  if (r.in_ <= 0) return;
  if (d.pme_on) k_alch<T, ENERGY, INTEG, PGRAD, true><<<(unsigned)r.in_, 256, 0, s>>>(d, r, xb, vb, lb);
  else k_alch<T, ENERGY, INTEG, PGRAD, false><<<(unsigned)r.in_, 256, 0, s>>>(d, r, xb, vb, lb);
}

template <typename T>
hipError_t Launch<T>::prune(const Dev<T> &d, const Range &r, int xb, int lb, hipStream_t s) {
  if (d.pme_on) return hipSuccess;  // the Ewald kernels prune on the fly
  const int64_t nw = (r.en + PRUNE_CPW - 1) / PRUNE_CPW;
  const int nb = (int)((nw + 3) / 4);
  const unsigned grid = (unsigned)(8 * ((nb + 7) / 8));
  if (grid > 0) k_prune<T><<<grid, 256, 0, s>>>(d, r, xb, lb);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::step(const Dev<T> &d, const Range &r, int xb, int vb, int lb,
                           hipStream_t s) {
  if (d.pme_on) {
    hipError_t e = pme(d, r, xb, lb, s);
    if (e == hipSuccess) e = step_alch(d, r, xb, vb, lb, s);
    if (e == hipSuccess) e = prune(d, r, xb, lb, s);
    if (e == hipSuccess) e = step_env(d, r, xb, vb, lb, s);
    if (e == hipSuccess) e = env_integrate(d, r, xb, vb, lb, s);
    return e;
  }
  const hipError_t e = prune(d, r, xb, lb, s);
  if (e != hipSuccess) return e;
  alch_launch<T, false, true, false>(d, r, xb, vb, lb, s);
  env_launch<T>(d, r, xb, vb, lb, 0, true, s);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::env_integrate(const Dev<T> &d, const Range &r, int xb, int vb, int lb,
                                    hipStream_t s) {
  if (!d.pme_on || r.cn <= 0) return hipSuccess;
  k_env_integrate<T><<<nblk(r.cn * CL, 256), 256, 0, s>>>(d, r, xb, vb, lb);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::step_alch(const Dev<T> &d, const Range &r, int xb, int vb, int lb,
                                hipStream_t s) {
  alch_launch<T, false, true, false>(d, r, xb, vb, lb, s);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::step_env(const Dev<T> &d, const Range &r, int xb, int vb, int lb,
                               hipStream_t s) {
  // with PME: forces only; env_integrate finishes the step
  env_launch<T>(d, r, xb, vb, lb, 0, !d.pme_on, s);
  return hipGetLastError();
}

// mode EVAL_ALL: forces, energies, dV/dlambda and the solute parameter
// gradient; EVAL_ENERGY: energies and dV/dlambda only (no forces, no
// parameter gradient); EVAL_GRAD: forces, dV/dlambda and the parameter
// gradient (no energies).
template <typename T>
hipError_t Launch<T>::eval(const Dev<T> &d, const Range &r, int xb, int vb, int lb, int mode,
                           hipStream_t s) {
  if (d.pme_on) {
    const hipError_t e = pme(d, r, xb, lb, s);
    if (e != hipSuccess) return e;
  }
  const hipError_t ep = prune(d, r, xb, lb, s);
  if (ep != hipSuccess) return ep;
  if (mode == EVAL_ENERGY) {
    alch_launch<T, true, false, false>(d, r, xb, vb, lb, s);
    env_launch<T>(d, r, xb, vb, lb, 2, false, s);
  } else if (mode == EVAL_GRAD) {
    alch_launch<T, false, false, true>(d, r, xb, vb, lb, s);
    env_launch<T>(d, r, xb, vb, lb, 0, false, s);
    if (d.pme_on && r.cn > 0) k_env_recip<T><<<nblk(r.cn * CL, 256), 256, 0, s>>>(d, r);
  } else {
    alch_launch<T, true, false, true>(d, r, xb, vb, lb, s);
    env_launch<T>(d, r, xb, vb, lb, 1, false, s);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::export_pairs(const Dev<T> &d, const Range &r, int xb, int mode,
                                   hipStream_t s) {
  k_fill_u64<<<nblk(2 * d.n_walkers, 256), 256, 0, s>>>(d.pair_n, 2 * d.n_walkers);
  if (r.cn > 0) k_pairs<T><<<nblk(r.cn, 4), 256, 0, s>>>(d, r, xb, mode);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::init_velocities(const Dev<T> &d, int vb, hipStream_t s) {
  k_init_vel<T><<<nblk(d.n_atoms, 256), 256, 0, s>>>(d, vb);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::gather_atoms(const Dev<T> &d, int xb, int vb, double *pos, double *vel,
                                   hipStream_t s) {
  k_gather_atoms<T><<<nblk(d.n_atoms, 256), 256, 0, s>>>(d, xb, vb, pos, vel);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::scatter_atoms(const Dev<T> &d, int xb, int vb, const double *pos,
                                    const double *vel, hipStream_t s) {
  k_scatter_atoms<T><<<nblk(d.n_atoms, 256), 256, 0, s>>>(d, xb, vb, pos, vel);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::set_config(const Dev<T> &d, int xb, int lb, const double *pos,
                                 const double *lam, const double *params, hipStream_t s) {
  if (params && d.n_solute > 0) {
    k_set_params<T><<<nblk(d.n_solute, 256), 256, 0, s>>>(d, params);
    if (d.pme_on) {
      const hipError_t e = pme_charges(d, s);
      if (e != hipSuccess) return e;
    }
  }
  if (pos || lam) {
    const int64_t n = pos ? (d.n_atoms > d.n_walkers ? d.n_atoms : d.n_walkers) : d.n_walkers;
    k_set_config<T><<<nblk(n, 256), 256, 0, s>>>(d, xb, lb, pos, lam);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::energy_total(const Dev<T> &d, double *out, hipStream_t s) {
  k_energy_total<T><<<(unsigned)d.n_walkers, 256, 0, s>>>(d, out);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::energy_grads(const Dev<T> &d, const double *g, double *gpos, double *glam,
                                   double *gpar, hipStream_t s) {
  int64_t n = d.n_walkers;
  if (gpos && d.n_atoms > n) n = d.n_atoms;
  if (gpar && d.n_solute > n) n = d.n_solute;
  k_energy_grads<T><<<nblk(n, 256), 256, 0, s>>>(d, g, gpos, glam, gpar);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::gather_forces(const Dev<T> &d, double *f, hipStream_t s) {
  k_gather_forces<T><<<nblk(d.n_atoms, 256), 256, 0, s>>>(d, f);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init_lambda(const Dev<T> &d, const double *lam0, const double *p0, int lb,
                              hipStream_t s) {
  k_init_lambda<T><<<nblk(d.n_walkers, 64), 64, 0, s>>>(d, lam0, p0, lb);
  return hipGetLastError();
}

hipError_t launch_philox(int64_t n, const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_philox<<<nblk(n, 256), 256, 0, s>>>(n, ctr, k0, k1, out);
  return hipGetLastError();
}

template struct Launch<float>;
template struct Launch<double>;
template hipError_t launch_init_lambda<float>(const Dev<float> &, const double *, const double *,
                                              int, hipStream_t);
template hipError_t launch_init_lambda<double>(const Dev<double> &, const double *,
                                               const double *, int, hipStream_t);

}  // namespace labf
