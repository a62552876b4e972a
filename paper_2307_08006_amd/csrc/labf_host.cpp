// labf_host.cpp -- host runtime behind the C ABI of include/labf.h.
//
// Owns the device layout (labf_impl.h), validates every argument on the host
// before device work, schedules neighbour rebuilds every rebuild_interval
// steps and, in batched mode, replays [rebuild + rebuild_interval steps] as a
// captured HIP graph.  No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "labf.h"
#include "labf_impl.h"

namespace labf {
// Achievable-peak probes (labf_probe.hip): kind 0/1/2 = FP32 FMA, FP64 FMA,
// FP32 rsqrt chains of n iterations into buf0 [blocks * 256]; kind 3 = triad
// over n floats (buf0 = buf1 + s buf2, n a multiple of 4).
hipError_t launch_probe(int kind, int64_t n, void *buf0, void *buf1, void *buf2, unsigned blocks,
                        hipStream_t s);
}  // namespace labf

using namespace labf;

namespace {

thread_local std::string g_create_error;

struct DevBufs {
  std::vector<void *> ptrs;
  ~DevBufs() { release(); }
  void release() {
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
    ptrs.clear();
  }
};

double pow2_at_least(double x) { return std::ldexp(1.0, (int)std::ceil(std::log2(x))); }

template <typename T>
double round_to(double v) {
  return (double)(T)v;
}

// L rounded so that B + L is exact in T (as the stored positions require).
template <typename T>
double grid_edge(double L, double B) {
  return (double)((T)((T)B + (T)L) - (T)B);
}

template <typename T>
double grid_pos(double x, double L, double B) {
  double v = x - L * std::floor(x / L);
  if (v >= L) v -= L;
  double X = (double)((T)B + (T)v);
  if (X >= B + L) X -= L;
  if (X < B) X += L;
  return X;
}

bool finite_all(const double *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

struct labf_system {
  int precision = LABF_FP32;
  int W = 0;
  int64_t N = 0, C = 0, S = 0, E = 0, I = 0, K = 0;
  int64_t n_solute = 0;
  int list_cap = 0;
  int interval = 10;
  bool lam_set = false;
  bool xref_valid = false;
  bool list_current = false;      // the list was built at the current positions
  int xb = 0, vb = 0, lb = 0;
  int since_rebuild = 0;
  int64_t host_steps = 0;
  std::vector<int64_t> atom_offset;
  std::vector<WalkerMeta> meta;
  std::vector<PmeWalker> pme;    // host copy (FFT block ranges of the launches)
  int32_t pme_nblk[3] = {0, 0, 0};
  int32_t pme_bricks = 0;
  int32_t pme_planes = 0;
  int32_t pme_nblk2[3] = {0, 0, 0};  // leading blocks of walkers with power-of-two grids
  int32_t pme_planes2 = 0;
  std::vector<int32_t> n_acl_host;
  hipStream_t cap_stream = nullptr, cap_stream2 = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr, pme_ev = nullptr;
  std::map<int, hipGraphExec_t> graphs;
  std::map<int, hipGraph_t> graph_defs;
  int max_bins = 0;
  void *workspace = nullptr;      // caller-owned device memory holding every array
  size_t workspace_bytes = 0;
  DevBufs hook_bufs;              // staging of the pair-export test hook (allocated by that call)
  Dev<float> df{};
  Dev<double> dd{};
  std::string err;
  // device staging
  double *stage = nullptr;       // [N*3] doubles
  double *stage2 = nullptr;      // [N*3]
  double *lam_stage = nullptr;   // [2W]
  int64_t *pairs_dev = nullptr;
  int64_t pairs_cap = 0;
  int32_t *dr_partner_dev = nullptr;  // distance-restraint tables (in the workspace)
  int32_t *dr_pair_dev = nullptr;

  template <typename T>
  Dev<T> &dev();
};
template <>
Dev<float> &labf_system::dev<float>() {
  return df;
}
template <>
Dev<double> &labf_system::dev<double>() {
  return dd;
}

namespace {

labf_status fail(labf_system *s, labf_status code, const std::string &msg) {
  if (s)
    s->err = msg;
  else
    g_create_error = msg;
  return code;
}

labf_status hip_fail(labf_system *s, hipError_t e, const char *what) {
  return fail(s, LABF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(sys, expr)                                    \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return hip_fail(sys, _e, #expr);   \
  } while (0)

template <typename P>
hipError_t dalloc(DevBufs &b, P **p, size_t count) {
  void *q = nullptr;
  size_t bytes = std::max<size_t>(count, 1) * sizeof(P);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return e;
  e = hipMemset(q, 0, bytes);
  b.ptrs.push_back(q);
  *p = (P *)q;
  return e;
}

template <typename P>
hipError_t upload(DevBufs &b, const P **p, const P *host, size_t count) {
  P *q = nullptr;
  hipError_t e = dalloc(b, &q, count);
  if (e != hipSuccess) return e;
  if (host && count) e = hipMemcpy(q, host, count * sizeof(P), hipMemcpyHostToDevice);
  *p = q;
  return e;
}

// all three grid lengths of the walker are powers of two
static bool pme_pow2(const PmeWalker &p) { return p.lg[0] >= 0 && p.lg[1] >= 0 && p.lg[2] >= 0; }

Range full_range(const labf_system *s) {
  Range r{};
  r.a0 = 0;
  r.an = s->N;
  r.c0 = 0;
  r.cn = s->C;
  r.e0 = 0;
  r.en = s->E;
  r.i0 = 0;
  r.in_ = s->I;
  r.k0 = 0;
  r.kn = s->K;
  r.w0 = 0;
  r.wn = s->W;
  for (int a = 0; a < 3; ++a) {
    r.pb0[a] = 0;
    r.pbn[a] = s->pme_nblk[a];
    r.pbs[a] = s->pme_nblk2[a];
  }
  r.bb0 = 0;
  r.bbn = s->pme_bricks;
  r.pl0 = 0;
  r.pln = s->pme_planes;
  r.pls = s->pme_planes2;
  return r;
}

Range walker_range(const labf_system *s, int w) {
  const WalkerMeta &m = s->meta[w];
  Range r{};
  r.a0 = m.atom_begin;
  r.an = m.n_atoms;
  r.c0 = m.cl_begin;
  r.cn = (int64_t)m.cap_env + m.n_acl;
  r.e0 = m.env_item_begin;
  r.en = m.cap_env;
  r.i0 = m.item_begin;
  r.in_ = m.item_cap;
  r.k0 = m.col_begin;
  r.kn = (int64_t)m.ncx * m.ncy + 1;
  r.w0 = w;
  r.wn = 1;
  const bool p2 = !s->pme.empty() && pme_pow2(s->pme[w]);
  for (int a = 0; a < 3; ++a) {
    r.pb0[a] = s->pme.empty() ? 0 : s->pme[w].blk_begin[a];
    r.pbn[a] = s->pme.empty() ? 0 : s->pme[w].blk[a];
    r.pbs[a] = p2 ? r.pbn[a] : 0;
  }
  r.bb0 = s->pme.empty() ? 0 : s->pme[w].br_begin;
  r.bbn = s->pme.empty() ? 0 : s->pme[w].nbr[0] * s->pme[w].nbr[1] * s->pme[w].nbr[2];
  r.pl0 = s->pme.empty() ? 0 : s->pme[w].pl_begin;
  // a walker with y and z line blocks transforms line by line, else by planes
  r.pln = s->pme.empty() || s->pme[w].blk[1] > 0 ? 0 : s->pme[w].K[0];
  r.pls = p2 ? r.pln : 0;
  return r;
}

void drop_graphs(labf_system *s) {
  for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto &kv : s->graph_defs) (void)hipGraphDestroy(kv.second);
  s->graphs.clear();
  s->graph_defs.clear();
}

// --- validation ---------------------------------------------------------------
labf_status validate_desc(const labf_system_desc *d) {
  if (!d) return fail(nullptr, LABF_E_ARG, "desc is NULL");
  if (d->n_walkers < 1 || d->n_walkers > (1 << 20)) return fail(nullptr, LABF_E_ARG, "n_walkers out of range");
  if (d->precision != LABF_FP32 && d->precision != LABF_FP64) return fail(nullptr, LABF_E_ARG, "bad precision");
  if (d->pme_order != 0 && d->pme_order != 4 && d->pme_order != 6 && d->pme_order != 8)
    return fail(nullptr, LABF_E_ARG, "pme_order must be 0, 4, 6 or 8");
  if (d->pme_order) {
    if (!d->pme_dims) return fail(nullptr, LABF_E_ARG, "pme_dims is NULL");
    if (!std::isfinite(d->ewald_beta) || !(d->ewald_beta > 0)) return fail(nullptr, LABF_E_ARG, "ewald_beta must be > 0");
    for (int w = 0; w < d->n_walkers; ++w)
      for (int k = 0; k < 3; ++k) {
        const int32_t K = d->pme_dims[3 * w + k];
        // range first: the factor loops below do not end for K = 0
        bool ok = K >= 16 && K <= PME_KMAX && K % PME_BR == 0;
        if (ok) {
          int32_t rest = K;
          while (rest % 2 == 0) rest /= 2;
          while (rest % 3 == 0) rest /= 3;
          while (rest % 5 == 0) rest /= 5;
          ok = rest == 1;
        }
        if (!ok)
          return fail(nullptr, LABF_E_ARG, "pme_dims must be multiples of 8 in [16, 256] with no prime factor above 5");
      }
  }
  if (!d->atom_offset || !d->box || !d->pos || !d->mass || !d->charge || !d->sigma || !d->epsilon || !d->is_solute)
    return fail(nullptr, LABF_E_ARG, "required array is NULL");
  if (d->atom_offset[0] != 0) return fail(nullptr, LABF_E_ARG, "atom_offset[0] must be 0");
  for (int w = 0; w < d->n_walkers; ++w)
    if (d->atom_offset[w + 1] <= d->atom_offset[w])
      return fail(nullptr, LABF_E_ARG, "every walker needs at least one atom");
  const int64_t N = d->atom_offset[d->n_walkers];
  if (N > 0x7FFFFFF0LL) return fail(nullptr, LABF_E_ARG, "too many atoms");
  const bool has_r = d->anchor != nullptr;
  if (has_r != (d->k0 != nullptr) || has_r != (d->k1 != nullptr))
    return fail(nullptr, LABF_E_ARG, "anchor, k0 and k1 must be given together");
  const double scal[] = {d->r_cut, d->r_skin, d->r_skin_alch, d->kT, d->gamma, d->dt, d->coulomb_k, d->accel_unit};
  if (!finite_all(scal, 8)) return fail(nullptr, LABF_E_ARG, "non-finite scalar parameter");
  if (d->r_skin_alch != 0.0 && d->r_skin_alch < d->r_skin)
    return fail(nullptr, LABF_E_ARG, "r_skin_alch must be 0 or >= r_skin");
  if (!(d->r_cut > 0) || d->r_skin < 0 || d->kT < 0 || d->gamma < 0 || !(d->dt > 0) || d->coulomb_k < 0 ||
      !(d->accel_unit > 0))
    return fail(nullptr, LABF_E_ARG, "scalar parameter out of range");
  if (d->rebuild_interval < 1 || d->rebuild_interval > 1000) return fail(nullptr, LABF_E_ARG, "rebuild_interval out of range");
  if (d->max_bins < 0 || d->max_bins > 4096) return fail(nullptr, LABF_E_ARG, "max_bins must be 0 (1024) or 1..4096");
  if (d->list_capacity != 0 && (d->list_capacity < 16 || d->list_capacity > (1 << 20)))
    return fail(nullptr, LABF_E_ARG, "list_capacity must be 0 (estimated) or 16..2^20");
  if (d->prune_buffer)
    for (int w = 0; w < d->n_walkers; ++w)
      if (!(d->prune_buffer[w] >= 0.0 && d->prune_buffer[w] <= d->r_skin))
        return fail(nullptr, LABF_E_ARG, "prune_buffer must be 0 (default) or in (0, r_skin]");
  if (d->column_width)
    for (int w = 0; w < d->n_walkers; ++w)
      if (!(d->column_width[w] >= 0.5 && d->column_width[w] <= 2.0))
        return fail(nullptr, LABF_E_ARG, "column_width must be in [0.5, 2]");
  const double rl = d->r_cut + std::max(d->r_skin, d->r_skin_alch);
  for (int w = 0; w < d->n_walkers; ++w)
    for (int k = 0; k < 3; ++k) {
      const double L = d->box[3 * w + k];
      if (!std::isfinite(L) || !(L > 0)) return fail(nullptr, LABF_E_ARG, "box edges must be finite and > 0");
      if (!(rl < 0.5 * L))
        return fail(nullptr, LABF_E_ARG, "r_cut + max(r_skin, r_skin_alch) must be < L/2 on every edge");
      if (L > 1e7) return fail(nullptr, LABF_E_ARG, "box edge too large");
    }
  if (!finite_all(d->pos, 3 * N)) return fail(nullptr, LABF_E_ARG, "non-finite position");
  if (d->vel && !finite_all(d->vel, 3 * N)) return fail(nullptr, LABF_E_ARG, "non-finite velocity");
  for (int64_t i = 0; i < N; ++i) {
    if (!std::isfinite(d->mass[i]) || !(d->mass[i] > 0)) return fail(nullptr, LABF_E_ARG, "masses must be > 0");
    if (!std::isfinite(d->charge[i])) return fail(nullptr, LABF_E_ARG, "non-finite charge");
    if (!std::isfinite(d->epsilon[i]) || d->epsilon[i] < 0) return fail(nullptr, LABF_E_ARG, "epsilon must be >= 0");
    if (!std::isfinite(d->sigma[i]) || (d->epsilon[i] > 0 && !(d->sigma[i] > 0)))
      return fail(nullptr, LABF_E_ARG, "sigma must be > 0 where epsilon > 0");
    if (d->is_solute[i] > 1) return fail(nullptr, LABF_E_ARG, "is_solute must be 0 or 1");
    if (has_r) {
      if (!finite_all(d->anchor + 3 * i, 3) || !std::isfinite(d->k0[i]) || !std::isfinite(d->k1[i]) || d->k0[i] < 0 ||
          d->k1[i] < 0)
        return fail(nullptr, LABF_E_ARG, "restraint anchors/constants must be finite, k >= 0");
    }
  }
  return LABF_OK;
}

labf_status validate_lambda(const labf_system *s, const labf_lambda_params *p) {
  if (!p) return fail(const_cast<labf_system *>(s), LABF_E_ARG, "params is NULL");
  auto bad = [&](const char *m) { return fail(const_cast<labf_system *>(s), LABF_E_ARG, m); };
  if (!p->lambda0) return bad("lambda0 is NULL");
  const double sc[] = {p->m_lambda, p->gamma_lambda, p->kT_lambda, p->elec_start, p->elec_end,
                       p->vdw_start, p->vdw_end, p->sc_alpha, p->lo, p->hi};
  if (!finite_all(sc, 10)) return bad("non-finite lambda parameter");
  if (!(p->m_lambda > 0) || p->gamma_lambda < 0 || p->kT_lambda < 0) return bad("lambda mass/friction/temperature out of range");
  if (!(p->elec_start < p->elec_end) || !(p->vdw_start < p->vdw_end)) return bad("schedule ramps need start < end");
  if (p->direction != LABF_DECOUPLE && p->direction != LABF_COUPLE) return bad("bad direction");
  if (p->sc_power < 1 || p->sc_power > 8 || p->sc_alpha < 0) return bad("soft-core parameters out of range");
  if ((p->sc_form != LABF_SC_BEUTLER && p->sc_form != LABF_SC_SHIFTED) || !std::isfinite(p->sc_shift) ||
      p->sc_shift < 0)
    return bad("sc_form must be LABF_SC_BEUTLER or LABF_SC_SHIFTED, sc_shift finite and >= 0");
  if (p->reserved2 != 0) return bad("reserved2 must be 0");
  if (p->n_bins < 1 || p->n_bins > 4096) return bad("n_bins out of range");
  if (p->share_interval < 1) return bad("share_interval must be >= 1");
  if (!(p->lo < p->hi)) return bad("lo must be < hi");
  if (p->full_samples < 1) return bad("full_samples must be >= 1");
  if ((p->fixed_lambda != 0 && p->fixed_lambda != 1) || (p->abf_on != 0 && p->abf_on != 1)) return bad("flags must be 0 or 1");
  for (int w = 0; w < s->W; ++w) {
    if (!std::isfinite(p->lambda0[w]) || p->lambda0[w] < p->lo || p->lambda0[w] > p->hi) return bad("lambda0 outside [lo, hi]");
    if (p->p_lambda0 && !std::isfinite(p->p_lambda0[w])) return bad("non-finite p_lambda0");
  }
  return LABF_OK;
}

// --- layout -------------------------------------------------------------------
// Creating a system has three parts:
//   plan  (host only): walker metadata, static tables, PME tables, the list
//         capacity (estimated from the initial positions) and every array size;
//   carve: pointers into the caller's workspace, 256-byte aligned, in a fixed
//         order (with no workspace: only the total is summed, which is what
//         labf_workspace_size returns);
//   init  (device, on the caller's stream): clear, upload, first rebuild.
// No device memory is allocated by the library for a system.

// Bump allocator over the workspace; base == nullptr only sums the sizes.
struct Carver {
  char *base = nullptr;
  size_t off = 0;
  template <typename P>
  void take(P **p, size_t count) {
    off = (off + 255) & ~(size_t)255;
    if (p) *p = base ? (P *)(base + off) : nullptr;
    off += std::max<size_t>(count, 1) * sizeof(P);
  }
};

// Everything about a system that the host computes before any device work.
struct HostLayout {
  int W = 0;
  int64_t N = 0, C = 0, S = 0, K = 0, E = 0, I = 0;
  int list_cap = 0, max_bins = 0;
  int plist_cap = 0;  // pruned-list entries per environment cluster
  bool uniform = true;
  double u_sig = 1.0, u_eps = 0.0;
  std::vector<WalkerMeta> meta;
  std::vector<uint8_t> alch, sol;
  std::vector<double> pos_grid, anc_grid;
  std::vector<int32_t> atom_walker, cl_walker, env_table, col_walker, solute_atom;
  std::vector<int32_t> item_walker, alch_cluster, slot0, orig0;
  // smooth PME
  std::vector<PmeWalker> pme;
  int64_t pme_goff = 0, pme_toff = 0, pme_loff = 0;
  int32_t pme_nbr = 0, pme_npl = 0, pme_maxyz = 0;
  int32_t pme_nblk[3] = {0, 0, 0}, pme_nblk2[3] = {0, 0, 0}, pme_planes2 = 0;
  std::vector<int32_t> pme_bw[3], pme_brw, pme_plw, pme_perm;
};

double gap1h(double lo_i, double hi_i, double lo_j, double hi_j) {
  return std::max(0.0, std::max(lo_j - hi_i, lo_i - hi_j));
}

// Upper estimate of the longest neighbour lists of the initial positions,
// from the cluster layout the rebuild produces (x-y columns of width cw,
// each sorted by z and cut into clusters of CL atoms; one cluster per
// alchemical atom): for a cluster box, every cluster of the columns and
// periodic images in reach whose z range comes within the list radius,
// with the column rectangle standing in for the other cluster's x-y extent
// (never below what the device list holds for the same positions).
// Returns {longest environment list, longest alchemical list}.
std::pair<int, int> estimate_lists(const HostLayout &h, double rl, double rla) {
  int mx_env = 0, mx_a = 0;
  for (int w = 0; w < h.W; ++w) {
    const WalkerMeta &m = h.meta[w];
    const int ncol = m.ncx * m.ncy;
    std::vector<std::vector<std::pair<double, int64_t>>> cols(ncol);
    std::vector<std::array<double, 3>> apos;
    for (int64_t i = m.atom_begin; i < m.atom_begin + m.n_atoms; ++i) {
      const double x = h.pos_grid[3 * i] - m.B[0], y = h.pos_grid[3 * i + 1] - m.B[1],
                   z = h.pos_grid[3 * i + 2] - m.B[2];
      if (h.alch[i]) {
        apos.push_back({x, y, z});
        continue;
      }
      const int cx = (int)std::min(std::max(std::floor(x / m.cw[0]), 0.0), (double)(m.ncx - 1));
      const int cy = (int)std::min(std::max(std::floor(y / m.cw[1]), 0.0), (double)(m.ncy - 1));
      cols[cx * m.ncy + cy].push_back({z, i});
    }
    // cluster boxes per column (z ranges sorted)
    std::vector<std::vector<std::array<double, 6>>> box(ncol);
    std::vector<std::vector<double>> zlo(ncol), zhi(ncol);
    for (int c = 0; c < ncol; ++c) {
      auto &v = cols[c];
      std::sort(v.begin(), v.end());
      for (size_t k = 0; k < v.size(); k += CL) {
        std::array<double, 6> b = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
        for (size_t t = k; t < std::min(v.size(), k + CL); ++t) {
          const int64_t i = v[t].second;
          for (int q = 0; q < 3; ++q) {
            const double p = h.pos_grid[3 * i + q] - m.B[q];
            b[q] = std::min(b[q], p);
            b[3 + q] = std::max(b[3 + q], p);
          }
        }
        box[c].push_back(b);
        zlo[c].push_back(b[2]);
        zhi[c].push_back(b[5]);
      }
    }
    const int nx = (int)std::ceil(rla / m.cw[0]) + 1, ny = (int)std::ceil(rla / m.cw[1]) + 1;
    // clusters of the columns in reach of box b within radius r
    auto count = [&](const std::array<double, 6> &b, double r) {
      int64_t n = 0;
      const double r2 = r * r;
      for (int dx = -nx; dx <= nx; ++dx)
        for (int dy = -ny; dy <= ny; ++dy) {
          const int cx0 = (int)std::floor(b[0] / m.cw[0]), cy0 = (int)std::floor(b[1] / m.cw[1]);
          const int rx = cx0 + dx, ry = cy0 + dy;
          const int cx = ((rx % m.ncx) + m.ncx) % m.ncx, cy = ((ry % m.ncy) + m.ncy) % m.ncy;
          const int sx = (rx - cx) / m.ncx, sy = (ry - cy) / m.ncy;
          if (sx < -1 || sx > 1 || sy < -1 || sy > 1) continue;
          const double xl = rx * m.cw[0], xh = (rx + 1) * m.cw[0];
          const double yl = ry * m.cw[1], yh = (ry + 1) * m.cw[1];
          const double gx = gap1h(b[0], b[3], xl, xh), gy = gap1h(b[1], b[4], yl, yh);
          const double gxy = gx * gx + gy * gy;
          if (gxy >= r2) continue;
          const double dz = std::sqrt(r2 - gxy);
          const int c = cx * m.ncy + cy;
          for (int sz = -1; sz <= 1; ++sz) {
            const double lo = b[2] - dz - sz * m.L[2], hi = b[5] + dz - sz * m.L[2];
            // clusters with zhi >= lo and zlo <= hi
            const auto a0 = std::lower_bound(zhi[c].begin(), zhi[c].end(), lo) - zhi[c].begin();
            const auto a1 = std::upper_bound(zlo[c].begin(), zlo[c].end(), hi) - zlo[c].begin();
            if (a1 > a0) n += a1 - a0;
          }
        }
      return n;
    };
    auto count_alch = [&](const std::array<double, 6> &b, double r) {
      int64_t n = 0;
      for (const auto &p : apos)
        for (int t = 0; t < 27; ++t) {
          const double ox = (t / 9 - 1) * m.L[0], oy = ((t / 3) % 3 - 1) * m.L[1], oz = (t % 3 - 1) * m.L[2];
          const double gx = gap1h(b[0], b[3], p[0] + ox, p[0] + ox), gy = gap1h(b[1], b[4], p[1] + oy, p[1] + oy),
                       gz = gap1h(b[2], b[5], p[2] + oz, p[2] + oz);
          if (gx * gx + gy * gy + gz * gz < r * r) ++n;
        }
      return n;
    };
    for (int c = 0; c < ncol; ++c)
      for (const auto &b : box[c])
        mx_env = (int)std::max<int64_t>(mx_env, count(b, rl) + count_alch(b, rla));
    for (const auto &p : apos) {
      const std::array<double, 6> b = {p[0], p[1], p[2], p[0], p[1], p[2]};
      mx_a = (int)std::max<int64_t>(mx_a, count(b, rla) + count_alch(b, rla));
    }
  }
  return {mx_env, mx_a};
}

// The host part of creating a system (no device work).
template <typename T>
labf_status plan_system(const labf_system_desc *desc, HostLayout &h) {
  const int W = desc->n_walkers;
  const int64_t N = desc->atom_offset[W];
  h.W = W;
  h.N = N;
  h.max_bins = desc->max_bins > 0 ? desc->max_bins : 1024;
  // alchemical set: solute atoms and atoms with a lambda-dependent restraint
  h.alch.resize(N);
  h.sol.resize(N);
  for (int64_t i = 0; i < N; ++i) {
    h.sol[i] = desc->is_solute[i];
    h.alch[i] = desc->is_solute[i] || (desc->anchor && desc->k0[i] != desc->k1[i]);
  }
  // uniform environment LJ parameters?
  bool first = true;
  for (int64_t i = 0; i < N && h.uniform; ++i) {
    if (h.alch[i]) continue;
    if (first) {
      h.u_sig = desc->sigma[i];
      h.u_eps = desc->epsilon[i];
      first = false;
    } else if (desc->sigma[i] != h.u_sig || desc->epsilon[i] != h.u_eps) {
      h.uniform = false;
    }
  }
  if (h.u_eps == 0.0) h.u_sig = 1.0;
  // per-walker metadata
  h.meta.resize(W);
  h.pos_grid.resize(3 * N);
  if (desc->anchor) h.anc_grid.resize(3 * N);
  int64_t cl = 0, col = 0, env = 0;
  const double rla = desc->r_cut + std::max(desc->r_skin, desc->r_skin_alch);
  for (int w = 0; w < W; ++w) {
    WalkerMeta &m = h.meta[w];
    std::memset(&m, 0, sizeof(m));
    m.atom_begin = desc->atom_offset[w];
    m.n_atoms = (int32_t)(desc->atom_offset[w + 1] - desc->atom_offset[w]);
    int64_t na = 0;
    for (int64_t i = m.atom_begin; i < m.atom_begin + m.n_atoms; ++i) na += h.alch[i];
    m.n_a = (int32_t)na;
    const int64_t nenv = m.n_atoms - na;
    double vol = 1.0;
    for (int k = 0; k < 3; ++k) {
      const double L0 = desc->box[3 * w + k];
      m.B[k] = pow2_at_least(2.0 * L0);
      m.L[k] = grid_edge<T>(L0, m.B[k]);
      if (!(rla < 0.5 * m.L[k])) return fail(nullptr, LABF_E_ARG, "r_list >= L/2 after rounding the box");
      vol *= m.L[k];
    }
    const double rho = (double)std::max<int64_t>(nenv, 1) / vol;
    const double target = std::cbrt((double)CL / rho) * (desc->column_width ? desc->column_width[w] : 1.0);
    m.ncx = (int32_t)std::min(256.0, std::max(1.0, std::floor(m.L[0] / target)));
    m.ncy = (int32_t)std::min(256.0, std::max(1.0, std::floor(m.L[1] / target)));
    m.cw[0] = m.L[0] / m.ncx;
    m.cw[1] = m.L[1] / m.ncy;
    // prune buffer: the given one, else half the skin, at most 0.35
    m.prune_b = desc->prune_buffer && desc->prune_buffer[w] > 0.0 ? desc->prune_buffer[w]
                                                                   : std::min(0.35, 0.5 * desc->r_skin);
    m.cap_env = (int32_t)((nenv + CL - 1) / CL + (int64_t)m.ncx * m.ncy);
    m.n_acl = (int32_t)na;  // one alchemical atom per cluster
    m.cl_begin = cl;
    m.col_begin = (int32_t)col;
    m.env_item_begin = (int32_t)env;
    cl += (int64_t)m.cap_env + m.n_acl;
    col += (int64_t)m.ncx * m.ncy + 1;
    env += m.cap_env;
    for (int64_t i = m.atom_begin; i < m.atom_begin + m.n_atoms; ++i)
      for (int k = 0; k < 3; ++k) {
        h.pos_grid[3 * i + k] = grid_pos<T>(desc->pos[3 * i + k], m.L[k], m.B[k]);
        if (desc->anchor) h.anc_grid[3 * i + k] = grid_pos<T>(desc->anchor[3 * i + k], m.L[k], m.B[k]);
      }
  }
  if (cl >= (int64_t)CL_MASK) return fail(nullptr, LABF_E_UNSUPPORTED, "too many clusters");
  h.C = cl;
  h.S = cl * CL;
  h.K = col;
  h.E = env;
  // static tables
  h.atom_walker.resize(N);
  h.cl_walker.resize(h.C);
  h.env_table.resize(h.E);
  h.col_walker.resize(h.K);
  for (int w = 0; w < W; ++w) {
    const WalkerMeta &m = h.meta[w];
    for (int64_t i = 0; i < m.n_atoms; ++i) h.atom_walker[m.atom_begin + i] = w;
    for (int64_t c = 0; c < (int64_t)m.cap_env + m.n_acl; ++c) h.cl_walker[m.cl_begin + c] = w;
    for (int64_t c = 0; c < m.cap_env; ++c) h.env_table[m.env_item_begin + c] = (int32_t)(m.cl_begin + c);
    for (int64_t k = m.col_begin; k < (int64_t)m.col_begin + (int64_t)m.ncx * m.ncy + 1; ++k) h.col_walker[k] = w;
  }
  for (int64_t i = 0; i < N; ++i)
    if (h.sol[i]) h.solute_atom.push_back((int32_t)i);
  // alchemical blocks: one per alchemical atom (a walker without any still
  // gets one block, which runs its lambda tail)
  int64_t ib = 0;
  for (int w = 0; w < W; ++w) {
    WalkerMeta &m = h.meta[w];
    m.item_begin = (int32_t)ib;
    m.item_cap = std::max(1, m.n_acl);
    for (int t = 0; t < m.item_cap; ++t) {
      h.item_walker.push_back(w);
      h.alch_cluster.push_back(t < m.n_acl ? (int32_t)(m.cl_begin + m.cap_env + t) : -1);
    }
    ib += m.item_cap;
  }
  if (ib > 0x7FFFFFF0LL) return fail(nullptr, LABF_E_UNSUPPORTED, "too many alchemical atoms");
  h.I = ib;
  // initial layout: atom i of walker w in slot cl_begin*8 + i; slot -> walker-local atom
  h.slot0.resize(N);
  h.orig0.assign(h.S, -1);
  for (int w = 0; w < W; ++w)
    for (int64_t i = 0; i < h.meta[w].n_atoms; ++i) {
      const int32_t sl = (int32_t)(h.meta[w].cl_begin * CL + i);
      h.slot0[h.meta[w].atom_begin + i] = sl;
      h.orig0[sl] = (int32_t)i;
    }
  // smooth PME: per-walker grids, FFT block tables, influence-function tables
  if (desc->pme_order) {
    h.pme.resize(W);
    int64_t goff = 0, toff = 0, loff = 0;
    int32_t nbr = 0, npl = 0, maxyz = 0;
    for (int w = 0; w < W; ++w) {
      PmeWalker &p = h.pme[w];
      std::memset(&p, 0, sizeof(p));
      for (int a = 0; a < 3; ++a) {
        p.K[a] = desc->pme_dims[3 * w + a];
        const int32_t K = p.K[a];
        if ((K & (K - 1)) == 0) {
          while ((1 << p.lg[a]) < K) ++p.lg[a];
        } else {
          // mixed-radix stage plan: fives, threes, fours, a last two
          p.lg[a] = -1;
          int32_t rest = K, ns = 0;
          for (int r : {5, 3, 4, 2})
            while (rest % r == 0) {
              p.rad[a][ns++] = (int8_t)r;
              rest /= r;
            }
          p.nst[a] = ns;
        }
      }
      // y and z transforms: fused per y-z plane in LDS when the plane fits
      // (no y or z line blocks then), else line by line
      const bool plane = p.K[1] * p.K[2] <= PME_PLANE;
      // lines per FFT block: the largest divisor of the number of lines
      // taken together that fills at most one tile
      auto max_div = [](int64_t cap, int64_t n) {
        int32_t q = (int32_t)std::min(cap, n);
        while (n % q) --q;
        return q;
      };
      p.nl[2] = max_div(PME_TILE / p.K[2], (int64_t)p.K[0] * p.K[1]);
      p.nl[1] = max_div(PME_TILE / p.K[1], p.K[2]);
      p.nl[0] = max_div(PME_TILE / p.K[0], p.K[2]);
      p.blk[2] = plane ? 0 : p.K[0] * p.K[1] / p.nl[2];
      p.blk[1] = plane ? 0 : p.K[0] * (p.K[2] / p.nl[1]);
      p.blk[0] = p.K[1] * (p.K[2] / p.nl[0]);
      // spread bricks; list capacity: three times the mean atom count of a
      // brick plus 64 (overflow is flagged in the walker status)
      const int32_t nb = (p.K[0] / PME_BR) * (p.K[1] / PME_BR) * (p.K[2] / PME_BR);
      for (int a = 0; a < 3; ++a) p.nbr[a] = p.K[a] / PME_BR;
      p.br_begin = nbr;
      nbr += nb;
      h.pme_brw.insert(h.pme_brw.end(), (size_t)nb, w);
      p.br_cap = (int32_t)(((3 * (int64_t)h.meta[w].n_atoms) / nb + 64 + 31) / 32 * 32);
      p.loff = loff;
      loff += (int64_t)nb * p.br_cap;
      if (plane) maxyz = std::max(maxyz, p.K[1] * p.K[2]);
      p.goff = goff;
      goff += (int64_t)p.K[0] * p.K[1] * p.K[2];
      p.toff = toff;
      toff += p.K[0] + p.K[1] + p.K[2];
      const WalkerMeta &m = h.meta[w];
      p.pref = desc->coulomb_k / (3.14159265358979323846 * m.L[0] * m.L[1] * m.L[2]);
    }
    // FFT blocks and y-z planes: walkers whose three grid lengths are powers
    // of two first (their own kernel instantiations), then the others
    for (int pass = 0; pass < 2; ++pass) {
      for (int w = 0; w < W; ++w) {
        PmeWalker &p = h.pme[w];
        if (pme_pow2(p) != (pass == 0)) continue;
        for (int a = 0; a < 3; ++a) {
          p.blk_begin[a] = h.pme_nblk[a];
          h.pme_nblk[a] += p.blk[a];
          h.pme_bw[a].insert(h.pme_bw[a].end(), (size_t)p.blk[a], w);
        }
        p.pl_begin = npl;
        if (p.blk[1] == 0) {
          npl += p.K[0];
          h.pme_plw.insert(h.pme_plw.end(), (size_t)p.K[0], w);
        }
      }
      if (pass == 0) {
        for (int a = 0; a < 3; ++a) h.pme_nblk2[a] = h.pme_nblk[a];
        h.pme_planes2 = npl;
      }
    }
    // frequency index at each position of a forward transform: with the
    // radices r_1 .. r_n of the decimation-in-frequency stages, position
    // p = j_1 m_1 + p' (m_1 = K / r_1) holds frequency j_1 + r_1 f(p')
    // (bit reversal for radix 2)
    h.pme_perm.resize(toff);
    for (int w = 0; w < W; ++w) {
      const PmeWalker &p = h.pme[w];
      int64_t o = p.toff;
      for (int a = 0; a < 3; ++a) {
        const int32_t K = p.K[a];
        std::vector<int32_t> rads;
        if (p.lg[a] >= 0) rads.assign((size_t)p.lg[a], 2);
        else rads.assign(p.rad[a], p.rad[a] + p.nst[a]);
        for (int32_t pos = 0; pos < K; ++pos) {
          int32_t rem = pos, len = K, mult = 1, f = 0;
          for (int32_t r : rads) {
            const int32_t mm = len / r, j = rem / mm;
            rem -= j * mm;
            f += j * mult;
            mult *= r;
            len = mm;
          }
          h.pme_perm[o + pos] = f;
        }
        o += K;
      }
    }
    h.pme_goff = goff;
    h.pme_toff = toff;
    h.pme_loff = loff;
    h.pme_nbr = nbr;
    h.pme_npl = npl;
    h.pme_maxyz = maxyz;
  }
  // neighbour-list capacity: the given one, or twice the estimated longest
  // environment list plus 64 and three times the longest alchemical one plus
  // 128 (headroom for denser regions and larger cluster boxes once the
  // configuration relaxes; overflow is flagged in the walker status)
  if (desc->list_capacity > 0) {
    h.list_cap = desc->list_capacity;
  } else {
    const auto mx = estimate_lists(h, desc->r_cut + desc->r_skin, rla);
    h.list_cap = std::max({128, (2 * mx.first + 64 + 31) / 32 * 32, (3 * mx.second + 128 + 31) / 32 * 32});
  }
  // a pruned list keeps at most every atom of the cluster list's entries;
  // its entries address walker-relative slots in SHIFT_BITS bits
  // (none with Ewald electrostatics: those kernels prune on the fly)
  h.plist_cap = desc->pme_order ? 0 : (CL * h.list_cap + WAVE - 1) / WAVE * WAVE;
  for (int w = 0; w < W; ++w)
    if (((int64_t)h.meta[w].cap_env + h.meta[w].n_acl) * CL > (int64_t)CL_MASK)
      return fail(nullptr, LABF_E_UNSUPPORTED, "too many atoms in one walker");
  return LABF_OK;
}

// Device arrays of a system, in a fixed order (count or assign).
template <typename T>
void carve(const HostLayout &h, labf_system *s, Dev<T> &d, Carver &cv) {
  const int64_t N = h.N, S = h.S, C = h.C, W = h.W, K = h.K;
  const WalkerMeta *meta = nullptr;
  cv.take(&meta, W);
  d.meta = meta;
  int32_t *p32 = nullptr;
  cv.take(&p32, N);
  d.atom_walker = p32;
  cv.take(&p32, C);
  d.cl_walker = p32;
  cv.take(&p32, h.E);
  d.env_table = p32;
  cv.take(&p32, K);
  d.col_walker = p32;
  cv.take(&p32, h.I);
  d.item_walker = p32;
  cv.take(&p32, h.I);
  d.alch_cluster = p32;
  cv.take(&p32, h.solute_atom.size());
  d.solute_atom = p32;
  cv.take(&d.a_q, N);
  cv.take(&d.a_sig, N);
  cv.take(&d.a_eps, N);
  double *p64 = nullptr;
  cv.take(&p64, N);
  d.a_mass = p64;
  uint8_t *p8 = nullptr;
  cv.take(&p8, N);
  d.a_sol = p8;
  cv.take(&p8, N);
  d.a_alch = p8;
  if (!h.anc_grid.empty()) {
    cv.take(&p64, N);
    d.a_k0 = p64;
    cv.take(&p64, N);
    d.a_k1 = p64;
    cv.take(&p64, 3 * N);
    d.a_anchor = p64;
  } else {
    d.a_k0 = d.a_k1 = d.a_anchor = nullptr;
  }
  if (!h.pme.empty()) {
    const PmeWalker *pw = nullptr;
    cv.take(&pw, W);
    d.pme = pw;
    for (int a = 0; a < 3; ++a) {
      cv.take(&p32, h.pme_bw[a].size());
      d.pme_bw[a] = p32;
    }
    cv.take(&d.pme_grid, h.pme_goff);
    cv.take(&p32, h.pme_brw.size());
    d.pme_brw = p32;
    cv.take(&d.pme_bcnt, h.pme_nbr);
    cv.take(&d.pme_blist, h.pme_loff);
    if (h.pme_npl > 0) {
      cv.take(&p32, h.pme_plw.size());
      d.pme_plw = p32;
    } else {
      d.pme_plw = nullptr;
    }
    cv.take(&p64, 2 * h.pme_toff);
    d.pme_tab = p64;
    cv.take(&p32, h.pme_perm.size());
    d.pme_perm = p32;
    cv.take(&d.pme_frc, 3 * S);
    cv.take(&d.pme_phi, 2 * S);
    cv.take(&d.pme_qs, 4 * W);
    float4 *ew = nullptr;
    cv.take(&ew, 2 * EWTAB_N);
    d.ewtab = ew;
  }
  cv.take(&d.slot_of, N);
  cv.take(&d.new_slot, N);
  cv.take(&d.col_of, N);
  cv.take(&d.key_col, N);
  cv.take(&d.members, N);
  cv.take(&d.xref, 3 * N);
  cv.take(&d.disp, N);
  cv.take(&d.skin_part, (size_t)W * SKIN_PARTS * 4);
  cv.take(&d.col_count, K);
  cv.take(&d.col_fill, K);
  cv.take(&d.col_atom0, K);
  cv.take(&d.col_cl0, K);
  for (int u = 0; u < 2; ++u)
    for (int k = 0; k < 3; ++k) {
      cv.take(&d.X[u][k], S);
      cv.take(&d.V[u][k], S);
    }
  cv.take(&d.q, S);
  cv.take(&d.lja, S);
  cv.take(&d.ljb, S);
  cv.take(&d.aim, S);
  cv.take(&d.nsd, S);
  cv.take(&d.rk, S);
  for (int k = 0; k < 3; ++k) cv.take(&d.anc[k], S);
  cv.take(&d.q64, S);
  cv.take(&d.sig64, S);
  cv.take(&d.eps64, S);
  cv.take(&d.k0_64, S);
  cv.take(&d.k1_64, S);
  cv.take(&d.sol, S);
  cv.take(&d.orig, S);
  cv.take(&d.fout, 3 * S);
  cv.take(&d.bbox, 6 * C);
  cv.take(&d.cl_col, C);
  cv.take(&d.list_count, C);
  cv.take(&d.list_nenv, C);
  cv.take(&d.cl_energy, 2 * C);
  cv.take(&d.list, (size_t)C * h.list_cap);
  cv.take(&d.plist, (size_t)h.E * h.plist_cap);
  cv.take(&d.plist_n, h.E);
  for (int k = 0; k < 3; ++k) cv.take(&d.xprune[k], S);
  for (int k = 0; k < 3; ++k) cv.take(&d.noise[k], h.plist_cap ? S : 0);
  cv.take(&d.pdisp, (size_t)2 * W * PDISP_SLOTS);
  cv.take(&d.item_force, (size_t)h.I * 3);
  cv.take(&d.item_dudl, (size_t)h.I);
  cv.take(&d.item_energy, (size_t)h.I * 5);
  cv.take(&d.item_pgrad, (size_t)h.I * 3);
  cv.take(&d.n_env, W);
  cv.take(&d.ticket, W);
  cv.take(&d.gticket, 1);
  cv.take(&d.status, W);
  cv.take(&d.lambda, 2 * W);
  cv.take(&d.p_lambda, W);
  cv.take(&d.dudl, W);
  cv.take(&d.bias, W);
  cv.take(&d.step, 2 * W);
  cv.take(&d.start_step, 1);
  cv.take(&d.energy, 5 * W);
  cv.take(&d.pair_n, 2 * W);
  // ABF accumulators, sized for max_bins
  cv.take(&d.bin_count, h.max_bins);
  cv.take(&d.bin_sum, h.max_bins);
  cv.take(&d.bin_sum2, h.max_bins);
  cv.take(&d.loc_count, (size_t)h.max_bins * W);
  cv.take(&d.loc_sum, (size_t)h.max_bins * W);
  cv.take(&d.loc_sum2, (size_t)h.max_bins * W);
  // distance-restraint tables (used once a restraint is set)
  cv.take(&s->dr_partner_dev, N);
  cv.take(&s->dr_pair_dev, 2 * W);
  // host <-> device staging
  cv.take(&s->stage, 3 * N);
  cv.take(&s->stage2, 3 * N);
  cv.take(&s->lam_stage, 2 * W);
}

// Bytes of workspace a system needs (host computation only).
template <typename T>
labf_status workspace_bytes(const labf_system_desc *desc, size_t *bytes, HostLayout *keep) {
  HostLayout local;
  HostLayout &h = keep ? *keep : local;
  labf_status rc = plan_system<T>(desc, h);
  if (rc != LABF_OK) return rc;
  labf_system tmp;
  Dev<T> d{};
  Carver cv;
  carve<T>(h, &tmp, d, cv);
  *bytes = (cv.off + 255) & ~(size_t)255;
  return LABF_OK;
}

template <typename T>
labf_status do_rebuild(labf_system *s, int mode, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  const int check = s->xref_valid ? 1 : 0;
  if (mode == LABF_MODE_PLAIN) {
    for (int w = 0; w < s->W; ++w) HIPCHK(s, Launch<T>::rebuild(d, walker_range(s, w), s->xb, s->vb, check, st));
  } else {
    HIPCHK(s, Launch<T>::rebuild(d, full_range(s), s->xb, s->vb, check, st));
  }
  s->xb ^= 1;
  s->vb ^= 1;
  s->xref_valid = true;
  s->since_rebuild = 0;
  s->list_current = true;
  return LABF_OK;
}

// The two internal streams (default priority) and events of the batched
// steps: the alchemical kernel runs on the second stream beside the
// environment kernel.
labf_status ensure_streams(labf_system *s) {
  if (s->cap_stream) return LABF_OK;
  HIPCHK(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  HIPCHK(s, hipStreamCreateWithFlags(&s->cap_stream2, hipStreamNonBlocking));
  HIPCHK(s, hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming));
  HIPCHK(s, hipEventCreateWithFlags(&s->join_ev, hipEventDisableTiming));
  HIPCHK(s, hipEventCreateWithFlags(&s->pme_ev, hipEventDisableTiming));
  return LABF_OK;
}

// One batched step on `st`, forked: with PME the reciprocal-space chain and
// then the alchemical kernel on the second stream, the environment kernel on
// `st`, and (with PME) the environment atoms integrated once both are done.
template <typename T>
hipError_t batched_step(labf_system *s, int xb, int vb, int lb, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  const Range r = full_range(s);
  // the prune test (and the occasional prune) first, alone on the device:
  // beside the alchemical kernel it takes several times longer, and the
  // environment kernel waits for it either way
  hipError_t e = Launch<T>::prune(d, r, xb, lb, st);
  if (e == hipSuccess) e = hipEventRecord(s->fork_ev, st);
  // without PME the environment kernel is issued first, so that in a graph
  // it starts right after the prune; the alchemical kernel (at most 96
  // VGPRs, as the environment kernel) takes the slots of retiring waves
  if (e == hipSuccess && !d.pme_on) e = Launch<T>::step_env(d, r, xb, vb, lb, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(s->cap_stream2, s->fork_ev, 0);
  if (e == hipSuccess && d.pme_on) e = Launch<T>::pme(d, r, xb, lb, s->cap_stream2);
  if (e == hipSuccess && d.pme_on) e = hipEventRecord(s->pme_ev, s->cap_stream2);
  if (e == hipSuccess) e = Launch<T>::step_alch(d, r, xb, vb, lb, s->cap_stream2);
  if (e == hipSuccess && d.pme_on) e = Launch<T>::step_env(d, r, xb, vb, lb, st);
  if (e == hipSuccess && d.pme_on) e = hipStreamWaitEvent(st, s->pme_ev, 0);
  if (e == hipSuccess && d.pme_on) e = Launch<T>::env_integrate(d, r, xb, vb, lb, st);
  if (e == hipSuccess) e = hipEventRecord(s->join_ev, s->cap_stream2);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, s->join_ev, 0);
  return e;
}

template <typename T>
labf_status do_step(labf_system *s, int mode, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  if (mode == LABF_MODE_PLAIN) {
    for (int w = 0; w < s->W; ++w)
      HIPCHK(s, Launch<T>::step(d, walker_range(s, w), s->xb, s->vb, s->lb, st));
  } else {
    labf_status rc = ensure_streams(s);
    if (rc != LABF_OK) return rc;
    HIPCHK(s, batched_step<T>(s, s->xb, s->vb, s->lb, st));
  }
  s->xb ^= 1;
  s->lb ^= 1;
  s->since_rebuild += 1;
  s->host_steps += 1;
  return LABF_OK;
}

// Batched block: [rebuild + interval steps] captured once per buffer parity.
// A block flips the position and velocity buffers and keeps the lambda
// buffer (interval + 1 and 1 flips, interval flips: the alternating keys
// below), so the graph of the block after this one is captured together
// with this one: no capture falls between two blocks later on.
template <typename T>
labf_status capture_block(labf_system *s, int xb, int vb, int xref, int lb) {
  Dev<T> &d = s->dev<T>();
  const int key = xb * 2 + vb + (xref ? 4 : 0) + lb * 8;
  if (s->graphs.count(key)) return LABF_OK;
  labf_status rc = ensure_streams(s);
  if (rc != LABF_OK) return rc;
  HIPCHK(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = Launch<T>::rebuild(d, full_range(s), xb, vb, xref, s->cap_stream);
  xb ^= 1;
  vb ^= 1;
  // each step: the alchemical kernel (second stream) runs beside the
  // environment kernel; they read the same positions and write disjoint
  // slots, lambda and step counters are double-buffered
  // with PME the reciprocal-space chain runs on the second stream beside
  // the environment pair kernel, followed there by the alchemical kernel;
  // the environment atoms are integrated once both forces are in
  for (int i = 0; i < s->interval && e == hipSuccess; ++i) {
    e = batched_step<T>(s, xb, vb, lb, s->cap_stream);
    xb ^= 1;
    lb ^= 1;
  }
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
  if (e != hipSuccess) return hip_fail(s, e, "graph capture");
  if (e2 != hipSuccess) return hip_fail(s, e2, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  HIPCHK(s, hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
  s->graphs[key] = ex;
  s->graph_defs[key] = g;
  // move the graph to the device now rather than at its first launch
  HIPCHK(s, hipGraphUpload(ex, s->cap_stream));
  HIPCHK(s, hipStreamSynchronize(s->cap_stream));
  return LABF_OK;
}

template <typename T>
labf_status graph_block(labf_system *s, hipStream_t st) {
  const int key = s->xb * 2 + s->vb + (s->xref_valid ? 4 : 0) + s->lb * 8;
  labf_status rc = capture_block<T>(s, s->xb, s->vb, s->xref_valid ? 1 : 0, s->lb);
  if (rc == LABF_OK)
    rc = capture_block<T>(s, s->xb ^ ((s->interval + 1) & 1), s->vb ^ 1, 1, s->lb ^ (s->interval & 1));
  if (rc != LABF_OK) return rc;
  auto it = s->graphs.find(key);
  HIPCHK(s, hipGraphLaunch(it->second, st));
  s->xb ^= 1;
  s->vb ^= 1;
  s->xref_valid = true;
  for (int i = 0; i < s->interval; ++i) {
    s->xb ^= 1;
    s->lb ^= 1;
  }
  s->since_rebuild = s->interval;
  s->host_steps += s->interval;
  return LABF_OK;
}

template <typename T>
labf_status create_impl(const labf_system_desc *desc, hipStream_t st, labf_system *s) {
  Dev<T> &d = s->dev<T>();
  HostLayout h;
  size_t need = 0;
  labf_status rc = workspace_bytes<T>(desc, &need, &h);
  if (rc != LABF_OK) return rc;
  if (!desc->workspace) return fail(nullptr, LABF_E_ARG, "workspace is NULL (labf_workspace_size gives its size)");
  if ((uintptr_t)desc->workspace % 256 != 0) return fail(nullptr, LABF_E_ARG, "workspace must be 256-byte aligned");
  if (desc->workspace_bytes < need)
    return fail(nullptr, LABF_E_ARG,
                "workspace too small: " + std::to_string(desc->workspace_bytes) + " bytes given, " +
                    std::to_string(need) + " needed");
  const int W = h.W;
  const int64_t N = h.N;
  s->W = W;
  s->N = N;
  s->C = h.C;
  s->S = h.S;
  s->K = h.K;
  s->E = h.E;
  s->I = h.I;
  s->interval = desc->rebuild_interval;
  s->atom_offset.assign(desc->atom_offset, desc->atom_offset + W + 1);
  s->meta = h.meta;
  s->pme = h.pme;
  for (int a = 0; a < 3; ++a) {
    s->pme_nblk[a] = h.pme_nblk[a];
    s->pme_nblk2[a] = h.pme_nblk2[a];
  }
  s->pme_bricks = h.pme_nbr;
  s->pme_planes = h.pme_npl;
  s->pme_planes2 = h.pme_planes2;
  s->list_cap = h.list_cap;
  s->max_bins = h.max_bins;
  s->n_solute = (int64_t)h.solute_atom.size();
  s->workspace = desc->workspace;
  s->workspace_bytes = need;
  Carver cv;
  cv.base = (char *)desc->workspace;
  carve<T>(h, s, d, cv);
  // scalars
  d.n_walkers = W;
  d.n_atoms = N;
  d.n_slots = s->S;
  d.n_clusters = s->C;
  d.list_cap = h.list_cap;
  d.plist_cap = h.plist_cap;
  d.uniform_lj = h.uniform ? 1 : 0;
  d.r_cut = desc->r_cut;
  d.r_list = desc->r_cut + desc->r_skin;
  d.r_list_a = desc->r_cut + std::max(desc->r_skin, desc->r_skin_alch);
  d.dt = desc->dt;
  d.kT = desc->kT;
  d.gamma = desc->gamma;
  d.coulomb_k = desc->coulomb_k;
  d.accel = desc->accel_unit;
  d.c1 = std::exp(-desc->gamma * desc->dt);
  d.seed = desc->seed;
  d.rc2 = (T)(desc->r_cut * desc->r_cut);
  d.irc = (T)(1.0 / desc->r_cut);
  d.irc2 = (T)(1.0 / (desc->r_cut * desc->r_cut));
  {
    const double s6 = std::pow(h.u_sig, 6.0);
    const double c6 = 4.0 * h.u_eps * s6, c12 = 4.0 * h.u_eps * s6 * s6;
    const double ir6 = 1.0 / std::pow(desc->r_cut, 6.0);
    d.c6 = (T)c6;
    d.c12 = (T)c12;
    d.ushift = (T)((c12 * ir6 - c6) * ir6);
  }
  d.n_solute = s->n_solute;
  d.a_pos0 = nullptr;
  d.dr_partner = nullptr;
  d.dr_pair = nullptr;
  d.pme_on = desc->pme_order ? 1 : 0;
  d.pme_order = desc->pme_order;
  d.ewald_beta = desc->pme_order ? desc->ewald_beta : 0.0;
  d.ewb = (T)d.ewald_beta;
  d.ewc = (T)(d.ewald_beta * 1.1283791670955126);  // 2 beta / sqrt(pi)
  d.pme_nbr = h.pme_nbr;
  d.pme_npl = h.pme_maxyz <= 4096 ? 4096 : PME_PLANE;
  d.ewtab_inv = (float)(EWTAB_N / (desc->r_cut * desc->r_cut));
  // clear everything, then upload the static tables (the host vectors live
  // until the stream is synchronised below)
  HIPCHK(s, hipMemsetAsync(desc->workspace, 0, need, st));
  auto put = [&](const void *dst, const void *src, size_t bytes) -> hipError_t {
    if (!bytes || !dst) return hipSuccess;
    return hipMemcpyAsync((void *)dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  auto vput = [&](const void *dst, const auto &v) { return put(dst, v.data(), v.size() * sizeof(v[0])); };
  HIPCHK(s, put(d.meta, h.meta.data(), sizeof(WalkerMeta) * W));
  HIPCHK(s, vput(d.atom_walker, h.atom_walker));
  HIPCHK(s, vput(d.cl_walker, h.cl_walker));
  HIPCHK(s, vput(d.env_table, h.env_table));
  HIPCHK(s, vput(d.col_walker, h.col_walker));
  HIPCHK(s, vput(d.item_walker, h.item_walker));
  HIPCHK(s, vput(d.alch_cluster, h.alch_cluster));
  HIPCHK(s, vput(d.solute_atom, h.solute_atom));
  HIPCHK(s, put(d.a_q, desc->charge, sizeof(double) * N));
  HIPCHK(s, put(d.a_sig, desc->sigma, sizeof(double) * N));
  HIPCHK(s, put(d.a_eps, desc->epsilon, sizeof(double) * N));
  HIPCHK(s, put(d.a_mass, desc->mass, sizeof(double) * N));
  HIPCHK(s, vput(d.a_sol, h.sol));
  HIPCHK(s, vput(d.a_alch, h.alch));
  if (desc->anchor) {
    HIPCHK(s, put(d.a_k0, desc->k0, sizeof(double) * N));
    HIPCHK(s, put(d.a_k1, desc->k1, sizeof(double) * N));
    HIPCHK(s, vput(d.a_anchor, h.anc_grid));
  }
  HIPCHK(s, vput(d.slot_of, h.slot0));
  HIPCHK(s, vput(d.orig, h.orig0));
  if (d.pme_on) {
    HIPCHK(s, put(d.pme, h.pme.data(), sizeof(PmeWalker) * W));
    for (int a = 0; a < 3; ++a) HIPCHK(s, vput(d.pme_bw[a], h.pme_bw[a]));
    HIPCHK(s, vput(d.pme_brw, h.pme_brw));
    if (h.pme_npl > 0) HIPCHK(s, vput(d.pme_plw, h.pme_plw));
    HIPCHK(s, vput(d.pme_perm, h.pme_perm));
    HIPCHK(s, Launch<T>::pme_tables(d, (float4 *)d.ewtab, st));
    HIPCHK(s, Launch<T>::pme_charges(d, st));
  }
  HIPCHK(s, vput(s->stage, h.pos_grid));
  if (desc->vel) HIPCHK(s, put(s->stage2, desc->vel, sizeof(double) * 3 * N));
  s->xb = 0;
  s->vb = 0;
  HIPCHK(s, Launch<T>::scatter_atoms(d, 0, 0, s->stage, desc->vel ? s->stage2 : nullptr, st));
  if (!desc->vel) HIPCHK(s, Launch<T>::init_velocities(d, 0, st));
  s->xref_valid = false;
  rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
  if (rc != LABF_OK) return rc;
  // the capacity must hold the lists of the initial configuration
  std::vector<int32_t> cnt(s->C);
  HIPCHK(s, hipMemcpyAsync(cnt.data(), d.list_count, sizeof(int32_t) * s->C, hipMemcpyDeviceToHost, st));
  std::vector<uint32_t> status(W);
  HIPCHK(s, hipMemcpyAsync(status.data(), d.status, sizeof(uint32_t) * W, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  for (int w = 0; w < W; ++w)
    if (status[w] & LABF_WS_CAPACITY)
      return fail(nullptr, LABF_E_CAPACITY,
                  "the neighbour lists of walker " + std::to_string(w) + " exceed the list capacity " +
                      std::to_string(h.list_cap) + " (raise labf_system_desc.list_capacity)");
  s->since_rebuild = 0;
  return LABF_OK;
}

template <typename T>
labf_status set_lambda_impl(labf_system *s, const labf_lambda_params *p, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  if (p->n_bins > s->max_bins)
    return fail(s, LABF_E_ARG,
                "n_bins exceeds the bin capacity of the system (labf_system_desc.max_bins = " +
                    std::to_string(s->max_bins) + ")");
  LamParams &lp = d.lp;
  lp.m_lambda = p->m_lambda;
  lp.gamma_lambda = p->gamma_lambda;
  lp.kT_lambda = p->kT_lambda;
  lp.elec_start = p->elec_start;
  lp.elec_end = p->elec_end;
  lp.vdw_start = p->vdw_start;
  lp.vdw_end = p->vdw_end;
  lp.sc_alpha = p->sc_alpha;
  lp.lo = p->lo;
  lp.hi = p->hi;
  lp.bin_w = (p->hi - p->lo) / (double)p->n_bins;
  lp.c1l = std::exp(-p->gamma_lambda * d.dt);
  lp.sdl = std::sqrt((1.0 - lp.c1l * lp.c1l) * p->kT_lambda * p->m_lambda);
  lp.full_samples = p->full_samples;
  lp.direction = p->direction;
  lp.sc_power = p->sc_power;
  lp.sc_form = p->sc_form;
  lp.sc_shift = p->sc_shift;
  lp.n_bins = p->n_bins;
  lp.share_interval = p->share_interval;
  lp.fixed_lambda = p->fixed_lambda;
  lp.abf_on = p->abf_on;
  // empty the accumulators (their capacity was carved at creation)
  const size_t nb = (size_t)s->max_bins, nl = nb * (size_t)s->W;
  HIPCHK(s, hipMemsetAsync(d.bin_count, 0, sizeof(int64_t) * nb, st));
  HIPCHK(s, hipMemsetAsync(d.bin_sum, 0, sizeof(double) * nb, st));
  HIPCHK(s, hipMemsetAsync(d.bin_sum2, 0, sizeof(double) * nb, st));
  HIPCHK(s, hipMemsetAsync(d.loc_count, 0, sizeof(int64_t) * nl, st));
  HIPCHK(s, hipMemsetAsync(d.loc_sum, 0, sizeof(double) * nl, st));
  HIPCHK(s, hipMemsetAsync(d.loc_sum2, 0, sizeof(double) * nl, st));
  HIPCHK(s, hipMemcpyAsync(s->lam_stage, p->lambda0, sizeof(double) * s->W, hipMemcpyHostToDevice, st));
  if (p->p_lambda0)
    HIPCHK(s, hipMemcpyAsync(s->lam_stage + s->W, p->p_lambda0, sizeof(double) * s->W, hipMemcpyHostToDevice, st));
  HIPCHK(s, launch_init_lambda<T>(d, s->lam_stage, p->p_lambda0 ? s->lam_stage + s->W : nullptr, s->lb, st));
  // the step numbers restart: prune before the next evaluation
  HIPCHK(s, hipMemsetAsync(d.plist_n, 0xFF, sizeof(int32_t) * s->E, st));
  HIPCHK(s, hipStreamSynchronize(st));
  drop_graphs(s);
  s->host_steps = 0;
  s->lam_set = true;
  return LABF_OK;
}

template <typename T>
labf_status step_impl(labf_system *s, int64_t n, int mode, hipStream_t st) {
  while (n > 0) {
    if (s->since_rebuild >= s->interval) {
      if (mode == LABF_MODE_BATCHED && n >= s->interval) {
        labf_status rc = graph_block<T>(s, st);
        if (rc != LABF_OK) return rc;
        n -= s->interval;
        continue;
      }
      labf_status rc = do_rebuild<T>(s, mode, st);
      if (rc != LABF_OK) return rc;
    }
    labf_status rc = do_step<T>(s, mode, st);
    if (rc != LABF_OK) return rc;
    --n;
  }
  return LABF_OK;
}

template <typename T>
labf_status start_fresh_sequence(labf_system *s, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  const int64_t v = s->host_steps;
  HIPCHK(s, hipMemcpyAsync(d.start_step, &v, sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIPCHK(s, hipStreamSynchronize(st));
  return LABF_OK;
}

template <typename T>
labf_status eval_impl(labf_system *s, double *forces, double *energy, double *dudl, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  labf_status rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
  if (rc != LABF_OK) return rc;
  HIPCHK(s, Launch<T>::eval(d, full_range(s), s->xb, s->vb, s->lb, EVAL_ALL, st));
  if (forces) {
    HIPCHK(s, Launch<T>::gather_forces(d, s->stage, st));
    HIPCHK(s, hipMemcpyAsync(forces, s->stage, sizeof(double) * 3 * s->N, hipMemcpyDeviceToHost, st));
  }
  std::vector<double> e(5 * s->W), g(s->W), ce(2 * s->C);
  std::vector<int32_t> ne(s->W);
  HIPCHK(s, hipMemcpyAsync(e.data(), d.energy, sizeof(double) * 5 * s->W, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipMemcpyAsync(g.data(), d.dudl, sizeof(double) * s->W, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipMemcpyAsync(ce.data(), d.cl_energy, sizeof(double) * 2 * s->C, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipMemcpyAsync(ne.data(), d.n_env, sizeof(int32_t) * s->W, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  for (int w = 0; w < s->W; ++w) {
    const WalkerMeta &m = s->meta[w];
    double ee = 0.0, er = 0.0;
    for (int64_t c = m.cl_begin; c < m.cl_begin + ne[w]; ++c) {
      ee += ce[2 * c];
      er += ce[2 * c + 1];
    }
    e[5 * w + 0] += ee;
    e[5 * w + 4] += er;
  }
  if (energy) std::memcpy(energy, e.data(), sizeof(double) * 5 * s->W);
  if (dudl) std::memcpy(dudl, g.data(), sizeof(double) * s->W);
  return LABF_OK;
}

// Differentiable energy: install the configuration (device arrays, each may
// be NULL), rebuild the neighbour structure when positions or solute
// parameters were given or the atoms have moved since the last rebuild, then
// evaluate every pair term once in the given mode.
template <typename T>
labf_status energy_eval(labf_system *s, const double *pos, const double *lam, const double *params, int mode,
                        hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  if (params && s->n_solute > 0) {
    std::vector<double> p(3 * s->n_solute);
    HIPCHK(s, hipMemcpyAsync(p.data(), params, sizeof(double) * p.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(s, hipStreamSynchronize(st));
    for (int64_t i = 0; i < s->n_solute; ++i) {
      const double eps = p[3 * i], sig = p[3 * i + 1], q = p[3 * i + 2];
      if (!std::isfinite(eps) || !std::isfinite(sig) || !std::isfinite(q) || eps < 0 || (eps > 0 && !(sig > 0)))
        return fail(s, LABF_E_ARG, "solute parameters: need finite values, eps >= 0, sigma > 0 where eps > 0");
    }
  }
  HIPCHK(s, Launch<T>::set_config(d, s->xb, s->lb, pos, lam, params, st));
  if (pos) s->xref_valid = false;  // positions replaced: nothing to check at this rebuild
  // the slot copies of the parameters are refreshed by the rebuild
  if (pos || (params && s->n_solute > 0) || s->since_rebuild > 0 || !s->list_current) {
    labf_status rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
    if (rc != LABF_OK) return rc;
  }
  HIPCHK(s, Launch<T>::eval(d, full_range(s), s->xb, s->vb, s->lb, mode, st));
  return LABF_OK;
}

template <typename T>
labf_status energy_impl(labf_system *s, const double *pos, const double *lam, const double *params,
                        double *energy, double *dudl, hipStream_t st) {
  labf_status rc = energy_eval<T>(s, pos, lam, params, EVAL_ENERGY, st);
  if (rc != LABF_OK) return rc;
  HIPCHK(s, Launch<T>::energy_total(s->dev<T>(), energy, st));
  if (dudl) HIPCHK(s, hipMemcpyAsync(dudl, s->dev<T>().dudl, sizeof(double) * s->W, hipMemcpyDeviceToDevice, st));
  return LABF_OK;
}

template <typename T>
labf_status energy_backward_impl(labf_system *s, const double *pos, const double *lam, const double *params,
                                 const double *g, double *gpos, double *glam, double *gpar, hipStream_t st) {
  labf_status rc = energy_eval<T>(s, pos, lam, params, EVAL_GRAD, st);
  if (rc != LABF_OK) return rc;
  HIPCHK(s, Launch<T>::energy_grads(s->dev<T>(), g, gpos, glam, gpar, st));
  return LABF_OK;
}

template <typename T>
labf_status dr_impl(labf_system *s, const int32_t *pairs, double delta, double k, int32_t freq,
                    hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  if (!pairs) {
    d.dr_partner = nullptr;
    d.dr_pair = nullptr;
    drop_graphs(s);
    return LABF_OK;
  }
  if (freq != 1 && freq != 2) return fail(s, LABF_E_ARG, "freq must be 1 or 2");
  if (!std::isfinite(delta) || delta < 0 || !std::isfinite(k) || k < 0)
    return fail(s, LABF_E_ARG, "delta and k must be finite and >= 0");
  std::vector<int32_t> partner(s->N, -1), pair(2 * s->W, -1);
  for (int w = 0; w < s->W; ++w) {
    const WalkerMeta &m = s->meta[w];
    const int32_t a = pairs[2 * w], b = pairs[2 * w + 1];
    if (a == -1 && b == -1) continue;
    if (a < 0 || b < 0 || a >= m.n_atoms || b >= m.n_atoms || a == b)
      return fail(s, LABF_E_ARG, "restrained pair: two distinct atoms of the walker (or -1, -1)");
    for (int q = 0; q < 3; ++q)
      if (!(delta < 0.5 * m.L[q])) return fail(s, LABF_E_ARG, "delta must be < L/2");
    const int64_t ga = m.atom_begin + a, gb = m.atom_begin + b;
    partner[ga] = (int32_t)gb;
    partner[gb] = (int32_t)ga;
    pair[2 * w] = (int32_t)ga;
    pair[2 * w + 1] = (int32_t)gb;
  }
  HIPCHK(s, hipMemcpyAsync(s->dr_partner_dev, partner.data(), sizeof(int32_t) * s->N, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(s->dr_pair_dev, pair.data(), sizeof(int32_t) * 2 * s->W, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipStreamSynchronize(st));
  d.dr_partner = s->dr_partner_dev;
  d.dr_pair = s->dr_pair_dev;
  d.dr_delta = delta;
  d.dr_k = k;
  d.dr_freq = freq;
  drop_graphs(s);
  return LABF_OK;
}

template <typename T>
labf_status ensure_pairs_buf(labf_system *s, int64_t n) {
  Dev<T> &d = s->dev<T>();
  if (n <= s->pairs_cap) return LABF_OK;
  if (s->pairs_dev) {
    auto it = std::find(s->hook_bufs.ptrs.begin(), s->hook_bufs.ptrs.end(), (void *)s->pairs_dev);
    if (it != s->hook_bufs.ptrs.end()) {
      (void)hipFree(*it);
      s->hook_bufs.ptrs.erase(it);
    }
  }
  HIPCHK(s, dalloc(s->hook_bufs, &s->pairs_dev, (size_t)(2 * n)));
  s->pairs_cap = n;
  d.pair_out = s->pairs_dev;
  d.pair_max = n;
  drop_graphs(s);
  return LABF_OK;
}

template <typename T>
labf_status export_impl(labf_system *s, int w, int64_t max_pairs, int64_t *pairs, int64_t *n_pairs,
                        hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  labf_status rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
  if (rc != LABF_OK) return rc;
  // count first (mode 2 counts r < r_list without writing), then fetch
  const WalkerMeta &m = s->meta[w];
  const int64_t est = (int64_t)m.n_atoms * 2048 + 1024;
  rc = ensure_pairs_buf<T>(s, std::min<int64_t>(std::max<int64_t>(max_pairs, 1), est));
  if (rc != LABF_OK) return rc;
  HIPCHK(s, Launch<T>::export_pairs(d, walker_range(s, w), s->xb, 0, st));
  unsigned long long cnt = 0;
  HIPCHK(s, hipMemcpyAsync(&cnt, d.pair_n + w, sizeof(cnt), hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  if ((int64_t)cnt > s->pairs_cap && max_pairs > s->pairs_cap) {
    rc = ensure_pairs_buf<T>(s, std::min<int64_t>((int64_t)cnt, max_pairs));
    if (rc != LABF_OK) return rc;
    HIPCHK(s, Launch<T>::export_pairs(d, walker_range(s, w), s->xb, 0, st));
    HIPCHK(s, hipStreamSynchronize(st));
  }
  const int64_t got = std::min<int64_t>({(int64_t)cnt, s->pairs_cap, max_pairs});
  std::vector<int64_t> buf(2 * std::max<int64_t>(got, 1));
  if (got > 0) HIPCHK(s, hipMemcpy(buf.data(), s->pairs_dev, sizeof(int64_t) * 2 * got, hipMemcpyDeviceToHost));
  std::vector<std::pair<int64_t, int64_t>> pv(got);
  for (int64_t i = 0; i < got; ++i) pv[i] = {buf[2 * i], buf[2 * i + 1]};
  std::sort(pv.begin(), pv.end());
  for (int64_t i = 0; i < got && pairs; ++i) {
    pairs[2 * i] = pv[i].first;
    pairs[2 * i + 1] = pv[i].second;
  }
  if (n_pairs) *n_pairs = (int64_t)cnt;
  return LABF_OK;
}

// Device staging of labf_export_pairs_noalloc: LABF_EXPORT_NOALLOC_MAX_PAIRS
// pairs (16 MiB), one array per GPU for the life of the process.  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is a host-side stand-in).
static __device__ __align__(256) int64_t scratch[2 * (int64_t)LABF_EXPORT_NOALLOC_MAX_PAIRS];
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
int64_t *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Address of the current device's staging array (looked up once per device).
hipError_t scratch_ptr(int64_t **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (int64_t *)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// labf_export_pairs without any allocation: the device staging is the
// static array above, the host output is sorted in place.
template <typename T>
labf_status export_noalloc_impl(labf_system *s, int w, int64_t max_pairs, int64_t *pairs, int64_t *n_pairs,
                                hipStream_t st) {
  int64_t *stage = nullptr;
  HIPCHK(s, scratch_ptr(&stage));
  labf_status rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
  if (rc != LABF_OK) return rc;
  Dev<T> d = s->dev<T>();  // launch copy pointing at the static staging
  d.pair_out = stage;
  d.pair_max = LABF_EXPORT_NOALLOC_MAX_PAIRS;
  HIPCHK(s, Launch<T>::export_pairs(d, walker_range(s, w), s->xb, 0, st));
  unsigned long long cnt = 0;
  HIPCHK(s, hipMemcpyAsync(&cnt, d.pair_n + w, sizeof(cnt), hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  if (n_pairs) *n_pairs = (int64_t)cnt;
  if ((int64_t)cnt > LABF_EXPORT_NOALLOC_MAX_PAIRS)
    return fail(s, LABF_E_CAPACITY,
                "walker " + std::to_string(w) + " has " + std::to_string(cnt) +
                    " pairs, more than the static staging holds (" +
                    std::to_string((int64_t)LABF_EXPORT_NOALLOC_MAX_PAIRS) + "); use labf_export_pairs");
  const int64_t got = std::min<int64_t>((int64_t)cnt, max_pairs);
  if (got > 0 && pairs) {
    HIPCHK(s, hipMemcpyAsync(pairs, stage, sizeof(int64_t) * 2 * got, hipMemcpyDeviceToHost, st));
    HIPCHK(s, hipStreamSynchronize(st));
    struct P2 {
      int64_t a, b;
    };
    P2 *pv = reinterpret_cast<P2 *>(pairs);
    std::sort(pv, pv + got, [](const P2 &x, const P2 &y) { return x.a != y.a ? x.a < y.a : x.b < y.b; });
  }
  return LABF_OK;
}

template <typename T>
labf_status count_impl(labf_system *s, int64_t *pairs, int64_t *pairs_env, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  labf_status rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
  if (rc != LABF_OK) return rc;
  HIPCHK(s, Launch<T>::export_pairs(d, full_range(s), s->xb, 1, st));
  std::vector<unsigned long long> c(2 * s->W);
  HIPCHK(s, hipMemcpyAsync(c.data(), d.pair_n, sizeof(unsigned long long) * 2 * s->W, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  for (int w = 0; w < s->W; ++w) {
    pairs[w] = (int64_t)c[w];
    if (pairs_env) pairs_env[w] = (int64_t)c[s->W + w];
  }
  return LABF_OK;
}

template <typename T>
labf_status profile_impl(labf_system *s, int64_t n, double *ms, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  // ev[0] start, ev[1] rebuilt; step i: ev[4i+2] PME, ev[4i+3] alchemical,
  // ev[4i+4] prune, ev[4i+5] environment done
  std::vector<hipEvent_t> ev(2 + 4 * n);
  for (auto &e : ev) HIPCHK(s, hipEventCreate(&e));
  auto cleanup = [&]() {
    for (auto &e : ev) (void)hipEventDestroy(e);
  };
  HIPCHK(s, hipEventRecord(ev[0], st));
  labf_status rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
  if (rc != LABF_OK) {
    cleanup();
    return rc;
  }
  HIPCHK(s, hipEventRecord(ev[1], st));
  const Range r = full_range(s);
  for (int64_t i = 0; i < n; ++i) {
    HIPCHK(s, Launch<T>::pme(d, r, s->xb, s->lb, st));
    HIPCHK(s, hipEventRecord(ev[4 * i + 2], st));
    HIPCHK(s, Launch<T>::step_alch(d, r, s->xb, s->vb, s->lb, st));
    HIPCHK(s, hipEventRecord(ev[4 * i + 3], st));
    HIPCHK(s, Launch<T>::prune(d, r, s->xb, s->lb, st));
    HIPCHK(s, hipEventRecord(ev[4 * i + 4], st));
    HIPCHK(s, Launch<T>::step_env(d, r, s->xb, s->vb, s->lb, st));
    HIPCHK(s, Launch<T>::env_integrate(d, r, s->xb, s->vb, s->lb, st));
    HIPCHK(s, hipEventRecord(ev[4 * i + 5], st));
    s->xb ^= 1;
    s->lb ^= 1;
    s->since_rebuild += 1;
    s->host_steps += 1;
  }
  HIPCHK(s, hipEventSynchronize(ev[1 + 4 * n]));
  float t = 0.f;
  HIPCHK(s, hipEventElapsedTime(&t, ev[0], ev[1]));
  ms[0] = t;
  double sum[4] = {0.0, 0.0, 0.0, 0.0};  // PME, alchemical, prune, environment
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 4; ++k) {
      HIPCHK(s, hipEventElapsedTime(&t, ev[4 * i + 1 + k], ev[4 * i + 2 + k]));
      sum[k] += t;
    }
  ms[1] = sum[1] / n;
  ms[2] = sum[3] / n;
  ms[3] = d.pme_on ? sum[0] / n : 0.0;
  ms[4] = sum[2] / n;
  cleanup();
  return LABF_OK;
}

template <typename T>
labf_status write_atoms_impl(labf_system *s, const double *pos, const double *vel, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  if (pos && !finite_all(pos, 3 * s->N)) return fail(s, LABF_E_ARG, "non-finite position");
  if (vel && !finite_all(vel, 3 * s->N)) return fail(s, LABF_E_ARG, "non-finite velocity");
  HIPCHK(s, hipStreamSynchronize(st));
  if (pos) {
    std::vector<double> g(3 * s->N);
    for (int w = 0; w < s->W; ++w) {
      const WalkerMeta &m = s->meta[w];
      for (int64_t i = m.atom_begin; i < m.atom_begin + m.n_atoms; ++i)
        for (int k = 0; k < 3; ++k) g[3 * i + k] = grid_pos<T>(pos[3 * i + k], m.L[k], m.B[k]);
    }
    HIPCHK(s, hipMemcpy(s->stage, g.data(), sizeof(double) * 3 * s->N, hipMemcpyHostToDevice));
  }
  if (vel) HIPCHK(s, hipMemcpy(s->stage2, vel, sizeof(double) * 3 * s->N, hipMemcpyHostToDevice));
  HIPCHK(s, Launch<T>::scatter_atoms(d, s->xb, s->vb, pos ? s->stage : nullptr, vel ? s->stage2 : nullptr, st));
  s->xref_valid = false;  // positions replaced: nothing to check at this rebuild
  labf_status rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
  if (rc != LABF_OK) return rc;
  return start_fresh_sequence<T>(s, st);
}

template <typename T>
labf_status read_atoms_impl(labf_system *s, double *pos, double *vel, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  HIPCHK(s, Launch<T>::gather_atoms(d, s->xb, s->vb, s->stage, s->stage2, st));
  if (pos) HIPCHK(s, hipMemcpyAsync(pos, s->stage, sizeof(double) * 3 * s->N, hipMemcpyDeviceToHost, st));
  if (vel) HIPCHK(s, hipMemcpyAsync(vel, s->stage2, sizeof(double) * 3 * s->N, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  return LABF_OK;
}

template <typename F>
labf_status dispatch(labf_system *s, F &&f) {
  return s->precision == LABF_FP64 ? f((double *)nullptr) : f((float *)nullptr);
}

}  // namespace

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

labf_status labf_workspace_size(const labf_system_desc *desc, size_t *bytes) {
  if (!bytes) return fail(nullptr, LABF_E_ARG, "bytes is NULL");
  *bytes = 0;
  labf_status rc = validate_desc(desc);
  if (rc != LABF_OK) return rc;
  return desc->precision == LABF_FP64 ? workspace_bytes<double>(desc, bytes, nullptr)
                                      : workspace_bytes<float>(desc, bytes, nullptr);
}

labf_status labf_create_system(const labf_system_desc *desc, void *stream, labf_system **out) {
  if (!out) return fail(nullptr, LABF_E_ARG, "out is NULL");
  *out = nullptr;
  labf_status rc = validate_desc(desc);
  if (rc != LABF_OK) return rc;
  auto s = std::make_unique<labf_system>();
  s->precision = desc->precision;
  hipStream_t st = (hipStream_t)stream;
  rc = desc->precision == LABF_FP64 ? create_impl<double>(desc, st, s.get()) : create_impl<float>(desc, st, s.get());
  if (rc != LABF_OK) {
    if (!s->err.empty()) g_create_error = s->err;
    return rc;
  }
  *out = s.release();
  return LABF_OK;
}

labf_status labf_set_lambda_params(labf_system *sys, const labf_lambda_params *lp, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  labf_status rc = validate_lambda(sys, lp);
  if (rc != LABF_OK) return rc;
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return set_lambda_impl<T>(sys, lp, (hipStream_t)stream);
  });
}

labf_status labf_step_walkers(labf_system *sys, int64_t n_steps, int32_t mode, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (n_steps < 0) return fail(sys, LABF_E_ARG, "n_steps must be >= 0");
  if (mode != LABF_MODE_BATCHED && mode != LABF_MODE_PLAIN) return fail(sys, LABF_E_ARG, "bad mode");
  if (!sys->lam_set) return fail(sys, LABF_E_STATE, "labf_set_lambda_params must be called first");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return step_impl<T>(sys, n_steps, mode, (hipStream_t)stream);
  });
}

labf_status labf_read_abf_bins(labf_system *sys, int32_t n_bins, int32_t include_unshared, int64_t *counts,
                               double *sum, double *sum_sq, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (!sys->lam_set) return fail(sys, LABF_E_STATE, "no lambda parameters");
  const int nb = sys->precision == LABF_FP64 ? sys->dd.lp.n_bins : sys->df.lp.n_bins;
  if (n_bins != nb) return fail(sys, LABF_E_ARG, "n_bins does not match the parameters");
  if (!counts || !sum) return fail(sys, LABF_E_ARG, "counts and sum are required");
  hipStream_t st = (hipStream_t)stream;
  const int64_t *bc = sys->precision == LABF_FP64 ? sys->dd.bin_count : sys->df.bin_count;
  const double *bs = sys->precision == LABF_FP64 ? sys->dd.bin_sum : sys->df.bin_sum;
  const double *bs2 = sys->precision == LABF_FP64 ? sys->dd.bin_sum2 : sys->df.bin_sum2;
  const int64_t *lc = sys->precision == LABF_FP64 ? sys->dd.loc_count : sys->df.loc_count;
  const double *ls = sys->precision == LABF_FP64 ? sys->dd.loc_sum : sys->df.loc_sum;
  const double *ls2 = sys->precision == LABF_FP64 ? sys->dd.loc_sum2 : sys->df.loc_sum2;
  std::vector<int64_t> c(nb), lcv((size_t)nb * sys->W);
  std::vector<double> s1(nb), s2(nb), l1((size_t)nb * sys->W), l2((size_t)nb * sys->W);
  HIPCHK(sys, hipStreamSynchronize(st));
  HIPCHK(sys, hipMemcpy(c.data(), bc, sizeof(int64_t) * nb, hipMemcpyDeviceToHost));
  HIPCHK(sys, hipMemcpy(s1.data(), bs, sizeof(double) * nb, hipMemcpyDeviceToHost));
  HIPCHK(sys, hipMemcpy(s2.data(), bs2, sizeof(double) * nb, hipMemcpyDeviceToHost));
  if (include_unshared) {
    HIPCHK(sys, hipMemcpy(lcv.data(), lc, sizeof(int64_t) * lcv.size(), hipMemcpyDeviceToHost));
    HIPCHK(sys, hipMemcpy(l1.data(), ls, sizeof(double) * l1.size(), hipMemcpyDeviceToHost));
    HIPCHK(sys, hipMemcpy(l2.data(), ls2, sizeof(double) * l2.size(), hipMemcpyDeviceToHost));
    for (int w = 0; w < sys->W; ++w)
      for (int b = 0; b < nb; ++b) {
        c[b] += lcv[(size_t)w * nb + b];
        s1[b] += l1[(size_t)w * nb + b];
        s2[b] += l2[(size_t)w * nb + b];
      }
  }
  std::memcpy(counts, c.data(), sizeof(int64_t) * nb);
  std::memcpy(sum, s1.data(), sizeof(double) * nb);
  if (sum_sq) std::memcpy(sum_sq, s2.data(), sizeof(double) * nb);
  return LABF_OK;
}

labf_status labf_free_energy(labf_system *sys, double *grad, double *profile, double *delta_a, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (!sys->lam_set) return fail(sys, LABF_E_STATE, "no lambda parameters");
  const LamParams &lp = sys->precision == LABF_FP64 ? sys->dd.lp : sys->df.lp;
  const int nb = lp.n_bins;
  std::vector<int64_t> c(nb);
  std::vector<double> s1(nb);
  labf_status rc = labf_read_abf_bins(sys, nb, 1, c.data(), s1.data(), nullptr, stream);
  if (rc != LABF_OK) return rc;
  const double w = (lp.hi - lp.lo) / nb;
  double acc = 0.0;
  bool empty = false;
  for (int b = 0; b < nb; ++b) {
    const double g = c[b] > 0 ? s1[b] / (double)c[b] : 0.0;
    if (c[b] <= 0) empty = true;
    if (grad) grad[b] = g;
    if (profile) profile[b] = acc;
    acc += g * w;
  }
  if (delta_a) *delta_a = acc;
  return empty ? fail(sys, LABF_E_EMPTY_BIN, "a bin has no sample") : LABF_OK;
}

labf_status labf_read_walker_state(labf_system *sys, double *lambda, double *p_lambda, double *dudl, double *bias,
                                   uint32_t *status, int64_t *step, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  hipStream_t st = (hipStream_t)stream;
  const int W = sys->W;
  auto get = [&](auto *dst, const auto *src) -> hipError_t {
    if (!dst || !src) return hipSuccess;
    return hipMemcpy(dst, src, sizeof(*dst) * W, hipMemcpyDeviceToHost);
  };
  HIPCHK(sys, hipStreamSynchronize(st));
  if (sys->precision == LABF_FP64) {
    const Dev<double> &d = sys->dd;
    HIPCHK(sys, get(lambda, d.lambda + sys->lb * W));
    HIPCHK(sys, get(p_lambda, d.p_lambda));
    HIPCHK(sys, get(dudl, d.dudl));
    HIPCHK(sys, get(bias, d.bias));
    HIPCHK(sys, get(status, d.status));
  } else {
    const Dev<float> &d = sys->df;
    HIPCHK(sys, get(lambda, d.lambda + sys->lb * W));
    HIPCHK(sys, get(p_lambda, d.p_lambda));
    HIPCHK(sys, get(dudl, d.dudl));
    HIPCHK(sys, get(bias, d.bias));
    HIPCHK(sys, get(status, d.status));
  }
  if (step) *step = sys->host_steps;
  return LABF_OK;
}

labf_status labf_read_atoms(labf_system *sys, double *pos, double *vel, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return read_atoms_impl<T>(sys, pos, vel, (hipStream_t)stream);
  });
}

labf_status labf_write_atoms(labf_system *sys, const double *pos, const double *vel, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return write_atoms_impl<T>(sys, pos, vel, (hipStream_t)stream);
  });
}

labf_status labf_compute_forces(labf_system *sys, double *forces, double *energy, double *dudl, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (!sys->lam_set) return fail(sys, LABF_E_STATE, "labf_set_lambda_params must be called first");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return eval_impl<T>(sys, forces, energy, dudl, (hipStream_t)stream);
  });
}

labf_status labf_energy_forward(labf_system *sys, const double *pos, const double *lambda, const double *params,
                                double *energy, double *dudl, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (!energy) return fail(sys, LABF_E_ARG, "energy is NULL");
  if (!sys->lam_set) return fail(sys, LABF_E_STATE, "labf_set_lambda_params must be called first");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return energy_impl<T>(sys, pos, lambda, params, energy, dudl, (hipStream_t)stream);
  });
}

labf_status labf_energy_backward(labf_system *sys, const double *pos, const double *lambda, const double *params,
                                 const double *grad_energy, double *grad_pos, double *grad_lambda,
                                 double *grad_params, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (!grad_energy) return fail(sys, LABF_E_ARG, "grad_energy is NULL");
  if (!sys->lam_set) return fail(sys, LABF_E_STATE, "labf_set_lambda_params must be called first");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return energy_backward_impl<T>(sys, pos, lambda, params, grad_energy, grad_pos, grad_lambda, grad_params,
                                   (hipStream_t)stream);
  });
}

labf_status labf_set_distance_restraint(labf_system *sys, const int32_t *pairs, double delta, double k,
                                        int32_t freq, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return dr_impl<T>(sys, pairs, delta, k, freq, (hipStream_t)stream);
  });
}

labf_status labf_export_pairs(labf_system *sys, int32_t walker, int64_t max_pairs, int64_t *pairs, int64_t *n_pairs,
                              void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (walker < 0 || walker >= sys->W) return fail(sys, LABF_E_ARG, "walker out of range");
  if (max_pairs < 0 || (max_pairs > 0 && !pairs)) return fail(sys, LABF_E_ARG, "bad output buffer");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return export_impl<T>(sys, walker, max_pairs, pairs, n_pairs, (hipStream_t)stream);
  });
}

labf_status labf_export_pairs_noalloc(labf_system *sys, int32_t walker, int64_t max_pairs, int64_t *pairs,
                                      int64_t *n_pairs, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (walker < 0 || walker >= sys->W) return fail(sys, LABF_E_ARG, "walker out of range");
  if (max_pairs < 0 || (max_pairs > 0 && !pairs)) return fail(sys, LABF_E_ARG, "bad output buffer");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return export_noalloc_impl<T>(sys, walker, max_pairs, pairs, n_pairs, (hipStream_t)stream);
  });
}

labf_status labf_count_pairs(labf_system *sys, int64_t *pairs, int64_t *pairs_env, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (!pairs) return fail(sys, LABF_E_ARG, "pairs is NULL");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return count_impl<T>(sys, pairs, pairs_env, (hipStream_t)stream);
  });
}

labf_status labf_profile_steps(labf_system *sys, int64_t n_steps, double *ms, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (n_steps < 1 || n_steps > 100000 || !ms) return fail(sys, LABF_E_ARG, "bad profile arguments");
  if (!sys->lam_set) return fail(sys, LABF_E_STATE, "labf_set_lambda_params must be called first");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return profile_impl<T>(sys, n_steps, ms, (hipStream_t)stream);
  });
}

labf_status labf_philox(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out, void *stream) {
  if (n < 0 || (n > 0 && (!ctr || !key || !out))) return fail(nullptr, LABF_E_ARG, "bad philox arguments");
  if (n == 0) return LABF_OK;
  if (n > (1LL << 28)) return fail(nullptr, LABF_E_ARG, "too many counters");
  hipStream_t st = (hipStream_t)stream;
  DevBufs b;
  uint32_t *dc = nullptr, *dout = nullptr;
  hipError_t e = dalloc(b, &dc, (size_t)(4 * n));
  if (e == hipSuccess) e = dalloc(b, &dout, (size_t)(4 * n));
  if (e == hipSuccess) e = hipMemcpy(dc, ctr, sizeof(uint32_t) * 4 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_philox(n, dc, key[0], key[1], dout, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipMemcpy(out, dout, sizeof(uint32_t) * 4 * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(nullptr, e, "labf_philox");
  return LABF_OK;
}

labf_status labf_probe(int32_t kind, int64_t n, double *rate, void *stream) {
  if (!rate || kind < LABF_PROBE_FP32_FMA || kind > LABF_PROBE_TRIAD) return fail(nullptr, LABF_E_ARG, "bad probe kind");
  const bool triad = kind == LABF_PROBE_TRIAD;
  if (triad ? (n < 4 || n % 4 != 0 || n > (1LL << 30)) : (n < 1 || n > 1000000))
    return fail(nullptr, LABF_E_ARG, "bad probe size");
  hipStream_t st = (hipStream_t)stream;
  const unsigned blocks = triad ? (unsigned)((n / 4 + 255) / 256) : 4096u;
  DevBufs b;
  void *p0 = nullptr, *p1 = nullptr, *p2 = nullptr;
  hipError_t e = hipSuccess;
  if (triad) {
    float *a = nullptr, *x = nullptr, *y = nullptr;
    e = dalloc(b, &a, (size_t)n);
    if (e == hipSuccess) e = dalloc(b, &x, (size_t)n);
    if (e == hipSuccess) e = dalloc(b, &y, (size_t)n);
    p0 = a;
    p1 = x;
    p2 = y;
  } else {
    double *o = nullptr;
    e = dalloc(b, &o, (size_t)blocks * 256);
    p0 = o;
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (e == hipSuccess) e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = launch_probe(kind, n, p0, p1, p2, blocks, st);
  if (e == hipSuccess) e = hipEventRecord(ev[0], st);
  for (int i = 0; i < 5 && e == hipSuccess; ++i) e = launch_probe(kind, n, p0, p1, p2, blocks, st);
  if (e == hipSuccess) e = hipEventRecord(ev[1], st);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  for (auto &x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_fail(nullptr, e, "labf_probe");
  const double work = triad ? 12.0 * (double)n : (double)blocks * 256.0 * (double)n * 8.0;
  *rate = 5.0 * work / (1e-3 * (double)ms);
  return LABF_OK;
}

labf_status labf_get_info(labf_system *sys, labf_info *info, void *stream) {
  if (!sys || !info) return fail(sys, LABF_E_ARG, "NULL argument");
  std::vector<int32_t> ne(sys->W), lc(sys->C);
  const int32_t *pne = sys->precision == LABF_FP64 ? sys->dd.n_env : sys->df.n_env;
  const int32_t *plc = sys->precision == LABF_FP64 ? sys->dd.list_count : sys->df.list_count;
  HIPCHK(sys, hipStreamSynchronize((hipStream_t)stream));
  HIPCHK(sys, hipMemcpy(ne.data(), pne, sizeof(int32_t) * sys->W, hipMemcpyDeviceToHost));
  HIPCHK(sys, hipMemcpy(lc.data(), plc, sizeof(int32_t) * sys->C, hipMemcpyDeviceToHost));
  int64_t used = 0, entries = 0;
  int32_t mx_env = 0, mx_a = 0;
  for (int w = 0; w < sys->W; ++w) {
    const WalkerMeta &m = sys->meta[w];
    used += ne[w] + m.n_acl;
    for (int64_t c = m.cl_begin; c < m.cl_begin + ne[w]; ++c) {
      entries += lc[c];
      mx_env = std::max(mx_env, lc[c]);
    }
    for (int64_t c = m.cl_begin + m.cap_env; c < m.cl_begin + m.cap_env + m.n_acl; ++c) {
      entries += lc[c];
      mx_a = std::max(mx_a, lc[c]);
    }
  }
  info->list_max_env = mx_env;
  info->list_max_alch = mx_a;
  info->n_atoms = sys->N;
  info->n_slots = sys->S;
  info->n_clusters = used;
  info->n_list_entries = entries;
  info->n_walkers = sys->W;
  info->list_cap = sys->list_cap;
  info->precision = sys->precision;
  info->uniform_lj = sys->precision == LABF_FP64 ? sys->dd.uniform_lj : sys->df.uniform_lj;
  info->n_solute = sys->n_solute;
  return LABF_OK;
}

void labf_destroy_system(labf_system *sys) {
  if (!sys) return;
  (void)hipDeviceSynchronize();
  drop_graphs(sys);
  if (sys->cap_stream) (void)hipStreamDestroy(sys->cap_stream);
  if (sys->cap_stream2) (void)hipStreamDestroy(sys->cap_stream2);
  if (sys->fork_ev) (void)hipEventDestroy(sys->fork_ev);
  if (sys->join_ev) (void)hipEventDestroy(sys->join_ev);
  if (sys->pme_ev) (void)hipEventDestroy(sys->pme_ev);
  sys->hook_bufs.release();
  delete sys;
}

const char *labf_last_error(const labf_system *sys) {
  if (!sys) return g_create_error.c_str();
  return sys->err.c_str();
}

}  // extern "C"
