// labf_host.cpp -- host runtime behind the C ABI of include/labf.h.
//
// Owns the device layout (labf_impl.h), validates every argument on the host
// before device work, schedules neighbour rebuilds every rebuild_interval
// steps and, in batched mode, replays [rebuild + rebuild_interval steps] as a
// captured HIP graph.  No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
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
  DevBufs bufs;
  DevBufs item_bufs;
  Dev<float> df{};
  Dev<double> dd{};
  std::string err;
  // device staging
  double *stage = nullptr;       // [N*3] doubles
  double *stage2 = nullptr;      // [N*3]
  double *lam_stage = nullptr;   // [2W]
  int64_t *pairs_dev = nullptr;
  int64_t pairs_cap = 0;
  int32_t *dr_partner_dev = nullptr;  // distance-restraint tables (allocated on first use)
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
template <typename T>
labf_status alloc_items(labf_system *s) {
  Dev<T> &d = s->dev<T>();
  s->item_bufs.release();
  std::vector<int32_t> item_walker, alch_cluster;
  int64_t ib = 0;
  for (int w = 0; w < s->W; ++w) {
    WalkerMeta &m = s->meta[w];
    m.item_begin = (int32_t)ib;
    m.item_cap = std::max(1, m.n_acl);
    for (int t = 0; t < m.item_cap; ++t) {
      item_walker.push_back(w);
      alch_cluster.push_back(t < m.n_acl ? (int32_t)(m.cl_begin + m.cap_env + t) : -1);
    }
    ib += m.item_cap;
  }
  if (ib > 0x7FFFFFF0LL) return fail(s, LABF_E_UNSUPPORTED, "too many alchemical atoms");
  s->I = ib;
  HIPCHK(s, upload(s->item_bufs, &d.item_walker, item_walker.data(), item_walker.size()));
  HIPCHK(s, upload(s->item_bufs, &d.alch_cluster, alch_cluster.data(), alch_cluster.size()));
  HIPCHK(s, dalloc(s->item_bufs, &d.item_force, (size_t)ib * 3));
  HIPCHK(s, dalloc(s->item_bufs, &d.item_dudl, (size_t)ib));
  HIPCHK(s, dalloc(s->item_bufs, &d.item_energy, (size_t)ib * 5));
  HIPCHK(s, dalloc(s->item_bufs, &d.item_pgrad, (size_t)ib * 3));
  HIPCHK(s, dalloc(s->item_bufs, &d.list, (size_t)s->C * s->list_cap));
  // metadata changed (item ranges)
  HIPCHK(s, hipMemcpy((void *)d.meta, s->meta.data(), sizeof(WalkerMeta) * s->W, hipMemcpyHostToDevice));
  d.list_cap = s->list_cap;
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
  return LABF_OK;
}

template <typename T>
labf_status do_step(labf_system *s, int mode, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  if (mode == LABF_MODE_PLAIN) {
    for (int w = 0; w < s->W; ++w)
      HIPCHK(s, Launch<T>::step(d, walker_range(s, w), s->xb, s->vb, s->lb, st));
  } else {
    HIPCHK(s, Launch<T>::step(d, full_range(s), s->xb, s->vb, s->lb, st));
  }
  s->xb ^= 1;
  s->lb ^= 1;
  s->since_rebuild += 1;
  s->host_steps += 1;
  return LABF_OK;
}

// Batched block: [rebuild + interval steps] captured once per buffer parity.
template <typename T>
labf_status graph_block(labf_system *s, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
  const int key = s->xb * 2 + s->vb + (s->xref_valid ? 4 : 0) + s->lb * 8;
  auto it = s->graphs.find(key);
  if (it == s->graphs.end()) {
    if (!s->cap_stream) {
      HIPCHK(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
      HIPCHK(s, hipStreamCreateWithFlags(&s->cap_stream2, hipStreamNonBlocking));
      HIPCHK(s, hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming));
      HIPCHK(s, hipEventCreateWithFlags(&s->join_ev, hipEventDisableTiming));
      HIPCHK(s, hipEventCreateWithFlags(&s->pme_ev, hipEventDisableTiming));
    }
    HIPCHK(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    int xb = s->xb, vb = s->vb, lb = s->lb;
    hipError_t e = Launch<T>::rebuild(d, full_range(s), xb, vb, s->xref_valid ? 1 : 0, s->cap_stream);
    xb ^= 1;
    vb ^= 1;
    // each step: the alchemical kernel (second stream) runs beside the
    // environment kernel; they read the same positions and write disjoint
    // slots, lambda and step counters are double-buffered
    // with PME the reciprocal-space chain runs on the second stream beside
    // the environment pair kernel, followed there by the alchemical kernel;
    // the environment atoms are integrated once both forces are in
    for (int i = 0; i < s->interval && e == hipSuccess; ++i) {
      e = hipEventRecord(s->fork_ev, s->cap_stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(s->cap_stream2, s->fork_ev, 0);
      if (e == hipSuccess && d.pme_on) e = Launch<T>::pme(d, full_range(s), xb, lb, s->cap_stream2);
      if (e == hipSuccess && d.pme_on) e = hipEventRecord(s->pme_ev, s->cap_stream2);
      if (e == hipSuccess) e = Launch<T>::step_alch(d, full_range(s), xb, vb, lb, s->cap_stream2);
      if (e == hipSuccess) e = Launch<T>::step_env(d, full_range(s), xb, vb, lb, s->cap_stream);
      if (e == hipSuccess && d.pme_on) e = hipStreamWaitEvent(s->cap_stream, s->pme_ev, 0);
      if (e == hipSuccess && d.pme_on) e = Launch<T>::env_integrate(d, full_range(s), xb, vb, lb, s->cap_stream);
      if (e == hipSuccess) e = hipEventRecord(s->join_ev, s->cap_stream2);
      if (e == hipSuccess) e = hipStreamWaitEvent(s->cap_stream, s->join_ev, 0);
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
    it = s->graphs.find(key);
  }
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
  const int W = desc->n_walkers;
  const int64_t N = desc->atom_offset[W];
  s->W = W;
  s->N = N;
  s->interval = desc->rebuild_interval;
  s->atom_offset.assign(desc->atom_offset, desc->atom_offset + W + 1);
  // alchemical set: solute atoms and atoms with a lambda-dependent restraint
  std::vector<uint8_t> alch(N), sol(N);
  for (int64_t i = 0; i < N; ++i) {
    sol[i] = desc->is_solute[i];
    alch[i] = desc->is_solute[i] || (desc->anchor && desc->k0[i] != desc->k1[i]);
  }
  // uniform environment LJ parameters?
  bool uniform = true;
  double u_sig = 1.0, u_eps = 0.0;
  bool first = true;
  for (int64_t i = 0; i < N && uniform; ++i) {
    if (alch[i]) continue;
    if (first) {
      u_sig = desc->sigma[i];
      u_eps = desc->epsilon[i];
      first = false;
    } else if (desc->sigma[i] != u_sig || desc->epsilon[i] != u_eps) {
      uniform = false;
    }
  }
  if (u_eps == 0.0) u_sig = 1.0;
  // per-walker metadata
  s->meta.resize(W);
  std::vector<double> pos_grid(3 * N), anc_grid;
  if (desc->anchor) anc_grid.resize(3 * N);
  int64_t cl = 0, col = 0, env = 0;
  const double rl = desc->r_cut + desc->r_skin;
  const double rla = desc->r_cut + std::max(desc->r_skin, desc->r_skin_alch);
  for (int w = 0; w < W; ++w) {
    WalkerMeta &m = s->meta[w];
    std::memset(&m, 0, sizeof(m));
    m.atom_begin = desc->atom_offset[w];
    m.n_atoms = (int32_t)(desc->atom_offset[w + 1] - desc->atom_offset[w]);
    int64_t na = 0;
    for (int64_t i = m.atom_begin; i < m.atom_begin + m.n_atoms; ++i) na += alch[i];
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
        pos_grid[3 * i + k] = grid_pos<T>(desc->pos[3 * i + k], m.L[k], m.B[k]);
        if (desc->anchor) anc_grid[3 * i + k] = grid_pos<T>(desc->anchor[3 * i + k], m.L[k], m.B[k]);
      }
  }
  if (cl >= (int64_t)CL_MASK) return fail(nullptr, LABF_E_UNSUPPORTED, "too many clusters");
  s->C = cl;
  s->S = cl * CL;
  s->K = col;
  s->E = env;
  // scalars
  d.n_walkers = W;
  d.n_atoms = N;
  d.n_slots = s->S;
  d.n_clusters = s->C;
  d.uniform_lj = uniform ? 1 : 0;
  d.r_cut = desc->r_cut;
  d.r_list = rl;
  d.r_list_a = rla;
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
    const double s6 = std::pow(u_sig, 6.0);
    const double c6 = 4.0 * u_eps * s6, c12 = 4.0 * u_eps * s6 * s6;
    const double ir6 = 1.0 / std::pow(desc->r_cut, 6.0);
    d.c6 = (T)c6;
    d.c12 = (T)c12;
    d.ushift = (T)((c12 * ir6 - c6) * ir6);
  }
  // static tables
  std::vector<int32_t> atom_walker(N), cl_walker(s->C), env_table(s->E);
  for (int w = 0; w < W; ++w) {
    const WalkerMeta &m = s->meta[w];
    for (int64_t i = 0; i < m.n_atoms; ++i) atom_walker[m.atom_begin + i] = w;
    for (int64_t c = 0; c < (int64_t)m.cap_env + m.n_acl; ++c) cl_walker[m.cl_begin + c] = w;
    for (int64_t c = 0; c < m.cap_env; ++c) env_table[m.env_item_begin + c] = (int32_t)(m.cl_begin + c);
  }
  DevBufs &b = s->bufs;
  HIPCHK(s, upload(b, &d.meta, s->meta.data(), W));
  HIPCHK(s, upload(b, &d.atom_walker, atom_walker.data(), N));
  HIPCHK(s, upload(b, &d.cl_walker, cl_walker.data(), s->C));
  HIPCHK(s, upload(b, &d.env_table, env_table.data(), s->E));
  {
    std::vector<int32_t> col_walker(s->K);
    for (int w = 0; w < W; ++w) {
      const WalkerMeta &m = s->meta[w];
      for (int64_t k = m.col_begin; k < (int64_t)m.col_begin + (int64_t)m.ncx * m.ncy + 1; ++k) col_walker[k] = w;
    }
    HIPCHK(s, upload(b, &d.col_walker, col_walker.data(), col_walker.size()));
  }
  for (auto pr : {std::make_pair(&d.a_q, desc->charge), std::make_pair(&d.a_sig, desc->sigma),
                  std::make_pair(&d.a_eps, desc->epsilon)}) {
    HIPCHK(s, dalloc(b, pr.first, N));
    HIPCHK(s, hipMemcpy(*pr.first, pr.second, sizeof(double) * N, hipMemcpyHostToDevice));
  }
  {
    std::vector<int32_t> solute_atom;
    for (int64_t i = 0; i < N; ++i)
      if (sol[i]) solute_atom.push_back((int32_t)i);
    s->n_solute = (int64_t)solute_atom.size();
    d.n_solute = s->n_solute;
    HIPCHK(s, upload(b, &d.solute_atom, solute_atom.data(), solute_atom.size()));
  }
  HIPCHK(s, upload(b, &d.a_mass, desc->mass, N));
  HIPCHK(s, upload(b, &d.a_sol, sol.data(), N));
  HIPCHK(s, upload(b, &d.a_alch, alch.data(), N));
  if (desc->anchor) {
    HIPCHK(s, upload(b, &d.a_k0, desc->k0, N));
    HIPCHK(s, upload(b, &d.a_k1, desc->k1, N));
    HIPCHK(s, upload(b, &d.a_anchor, anc_grid.data(), 3 * N));
  } else {
    d.a_k0 = d.a_k1 = d.a_anchor = nullptr;
  }
  // smooth PME: per-walker grids, FFT block tables, influence-function tables
  d.pme_on = desc->pme_order ? 1 : 0;
  d.pme_order = desc->pme_order;
  d.ewald_beta = desc->pme_order ? desc->ewald_beta : 0.0;
  d.ewb = (T)d.ewald_beta;
  d.ewc = (T)(d.ewald_beta * 1.1283791670955126);  // 2 beta / sqrt(pi)
  s->pme.clear();
  for (int a = 0; a < 3; ++a) s->pme_nblk[a] = s->pme_nblk2[a] = 0;
  s->pme_planes = s->pme_planes2 = 0;
  if (d.pme_on) {
    s->pme.resize(W);
    int64_t goff = 0, toff = 0, loff = 0;
    int32_t nbr = 0, npl = 0, maxyz = 0;
    std::vector<int32_t> bw[3], brw, plw;
    for (int w = 0; w < W; ++w) {
      PmeWalker &p = s->pme[w];
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
      brw.insert(brw.end(), (size_t)nb, w);
      p.br_cap = (int32_t)(((3 * (int64_t)s->meta[w].n_atoms) / nb + 64 + 31) / 32 * 32);
      p.loff = loff;
      loff += (int64_t)nb * p.br_cap;
      if (plane) maxyz = std::max(maxyz, p.K[1] * p.K[2]);
      p.goff = goff;
      goff += (int64_t)p.K[0] * p.K[1] * p.K[2];
      p.toff = toff;
      toff += p.K[0] + p.K[1] + p.K[2];
      const WalkerMeta &m = s->meta[w];
      p.pref = desc->coulomb_k / (3.14159265358979323846 * m.L[0] * m.L[1] * m.L[2]);
    }
    // FFT blocks and y-z planes: walkers whose three grid lengths are powers
    // of two first (their own kernel instantiations), then the others
    for (int pass = 0; pass < 2; ++pass) {
      for (int w = 0; w < W; ++w) {
        PmeWalker &p = s->pme[w];
        if (pme_pow2(p) != (pass == 0)) continue;
        for (int a = 0; a < 3; ++a) {
          p.blk_begin[a] = s->pme_nblk[a];
          s->pme_nblk[a] += p.blk[a];
          bw[a].insert(bw[a].end(), (size_t)p.blk[a], w);
        }
        p.pl_begin = npl;
        if (p.blk[1] == 0) {
          npl += p.K[0];
          plw.insert(plw.end(), (size_t)p.K[0], w);
        }
      }
      if (pass == 0) {
        for (int a = 0; a < 3; ++a) s->pme_nblk2[a] = s->pme_nblk[a];
        s->pme_planes2 = npl;
      }
    }
    HIPCHK(s, upload(b, &d.pme, s->pme.data(), W));
    for (int a = 0; a < 3; ++a) HIPCHK(s, upload(b, &d.pme_bw[a], bw[a].data(), bw[a].size()));
    HIPCHK(s, dalloc(b, &d.pme_grid, goff));
    HIPCHK(s, upload(b, &d.pme_brw, brw.data(), brw.size()));
    HIPCHK(s, dalloc(b, &d.pme_bcnt, nbr));
    HIPCHK(s, dalloc(b, &d.pme_blist, loff));
    d.pme_nbr = nbr;
    s->pme_bricks = nbr;
    // LDS plane capacity of the fused y-z transform (walkers whose planes fit)
    d.pme_npl = maxyz <= 4096 ? 4096 : PME_PLANE;
    if (npl > 0) {
      HIPCHK(s, upload(b, &d.pme_plw, plw.data(), plw.size()));
    } else {
      d.pme_plw = nullptr;
    }
    s->pme_planes = npl;
    double *tab = nullptr;
    HIPCHK(s, dalloc(b, &tab, 2 * toff));
    d.pme_tab = tab;
    {
      // frequency index at each position of a forward transform: with the
      // radices r_1 .. r_n of the decimation-in-frequency stages, position
      // p = j_1 m_1 + p' (m_1 = K / r_1) holds frequency j_1 + r_1 f(p')
      // (bit reversal for radix 2)
      std::vector<int32_t> perm(toff);
      for (int w = 0; w < W; ++w) {
        const PmeWalker &p = s->pme[w];
        int64_t o = p.toff;
        for (int a = 0; a < 3; ++a) {
          const int32_t K = p.K[a];
          std::vector<int32_t> rads;
          if (p.lg[a] >= 0) rads.assign((size_t)p.lg[a], 2);
          else rads.assign(p.rad[a], p.rad[a] + p.nst[a]);
          for (int32_t pos = 0; pos < K; ++pos) {
            int32_t rem = pos, len = K, mult = 1, f = 0;
            for (int32_t r : rads) {
              const int32_t m = len / r, j = rem / m;
              rem -= j * m;
              f += j * mult;
              mult *= r;
              len = m;
            }
            perm[o + pos] = f;
          }
          o += K;
        }
      }
      HIPCHK(s, upload(b, &d.pme_perm, perm.data(), perm.size()));
    }
    HIPCHK(s, dalloc(b, &d.pme_frc, 3 * s->S));
    HIPCHK(s, dalloc(b, &d.pme_phi, 2 * s->S));
    HIPCHK(s, dalloc(b, &d.pme_qs, 4 * W));
    float4 *ewtab = nullptr;
    HIPCHK(s, dalloc(b, &ewtab, 2 * EWTAB_N));
    d.ewtab = ewtab;
    d.ewtab_inv = (float)(EWTAB_N / (desc->r_cut * desc->r_cut));
    HIPCHK(s, Launch<T>::pme_tables(d, ewtab, st));
    HIPCHK(s, Launch<T>::pme_charges(d, st));
  }
  d.a_pos0 = nullptr;
  HIPCHK(s, dalloc(b, &d.slot_of, N));
  HIPCHK(s, dalloc(b, &d.new_slot, N));
  HIPCHK(s, dalloc(b, &d.col_of, N));
  HIPCHK(s, dalloc(b, &d.key_col, N));
  HIPCHK(s, dalloc(b, &d.members, N));
  HIPCHK(s, dalloc(b, &d.xref, 3 * N));
  HIPCHK(s, dalloc(b, &d.disp, N));
  HIPCHK(s, dalloc(b, &d.skin_part, (size_t)W * SKIN_PARTS * 4));
  HIPCHK(s, dalloc(b, &d.col_count, s->K));
  HIPCHK(s, dalloc(b, &d.col_fill, s->K));
  HIPCHK(s, dalloc(b, &d.col_atom0, s->K));
  HIPCHK(s, dalloc(b, &d.col_cl0, s->K));
  for (int u = 0; u < 2; ++u)
    for (int k = 0; k < 3; ++k) {
      HIPCHK(s, dalloc(b, &d.X[u][k], s->S));
      HIPCHK(s, dalloc(b, &d.V[u][k], s->S));
    }
  HIPCHK(s, dalloc(b, &d.q, s->S));
  HIPCHK(s, dalloc(b, &d.lja, s->S));
  HIPCHK(s, dalloc(b, &d.ljb, s->S));
  HIPCHK(s, dalloc(b, &d.aim, s->S));
  HIPCHK(s, dalloc(b, &d.nsd, s->S));
  HIPCHK(s, dalloc(b, &d.rk, s->S));
  for (int k = 0; k < 3; ++k) HIPCHK(s, dalloc(b, &d.anc[k], s->S));
  HIPCHK(s, dalloc(b, &d.q64, s->S));
  HIPCHK(s, dalloc(b, &d.sig64, s->S));
  HIPCHK(s, dalloc(b, &d.eps64, s->S));
  HIPCHK(s, dalloc(b, &d.k0_64, s->S));
  HIPCHK(s, dalloc(b, &d.k1_64, s->S));
  HIPCHK(s, dalloc(b, &d.sol, s->S));
  HIPCHK(s, dalloc(b, &d.orig, s->S));
  HIPCHK(s, dalloc(b, &d.fout, 3 * s->S));
  HIPCHK(s, dalloc(b, &d.bbox, 6 * s->C));
  HIPCHK(s, dalloc(b, &d.cl_col, s->C));
  HIPCHK(s, dalloc(b, &d.list_count, s->C));
  HIPCHK(s, dalloc(b, &d.list_nenv, s->C));
  HIPCHK(s, dalloc(b, &d.cl_energy, 2 * s->C));
  HIPCHK(s, dalloc(b, &d.n_env, W));
  HIPCHK(s, dalloc(b, &d.ticket, W));
  HIPCHK(s, dalloc(b, &d.gticket, 1));
  HIPCHK(s, dalloc(b, &d.status, W));
  HIPCHK(s, dalloc(b, &d.lambda, 2 * W));
  HIPCHK(s, dalloc(b, &d.p_lambda, W));
  HIPCHK(s, dalloc(b, &d.dudl, W));
  HIPCHK(s, dalloc(b, &d.bias, W));
  HIPCHK(s, dalloc(b, &d.step, 2 * W));
  HIPCHK(s, dalloc(b, &d.start_step, 1));
  HIPCHK(s, dalloc(b, &d.energy, 5 * W));
  HIPCHK(s, dalloc(b, &d.pair_n, 2 * W));
  HIPCHK(s, dalloc(b, &s->stage, 3 * N));
  HIPCHK(s, dalloc(b, &s->stage2, 3 * N));
  HIPCHK(s, dalloc(b, &s->lam_stage, 2 * W));
  // ABF arrays are (re)allocated by labf_set_lambda_params
  d.bin_count = d.loc_count = nullptr;
  d.bin_sum = d.bin_sum2 = d.loc_sum = d.loc_sum2 = nullptr;
  // initial layout: atom i of walker w in slot cl_begin*8 + i
  std::vector<int32_t> slot0(N);
  for (int w = 0; w < W; ++w)
    for (int64_t i = 0; i < s->meta[w].n_atoms; ++i)
      slot0[s->meta[w].atom_begin + i] = (int32_t)(s->meta[w].cl_begin * CL + i);
  HIPCHK(s, hipMemcpy(d.slot_of, slot0.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice));
  {
    // slot -> walker-local atom (-1: empty); the rebuilds keep it current
    std::vector<int32_t> orig0(s->S, -1);
    for (int w = 0; w < W; ++w)
      for (int64_t i = 0; i < s->meta[w].n_atoms; ++i) orig0[slot0[s->meta[w].atom_begin + i]] = (int32_t)i;
    HIPCHK(s, hipMemcpy(d.orig, orig0.data(), sizeof(int32_t) * s->S, hipMemcpyHostToDevice));
  }
  HIPCHK(s, hipMemcpy(s->stage, pos_grid.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice));
  if (desc->vel) HIPCHK(s, hipMemcpy(s->stage2, desc->vel, sizeof(double) * 3 * N, hipMemcpyHostToDevice));
  s->xb = 0;
  s->vb = 0;
  HIPCHK(s, Launch<T>::scatter_atoms(d, 0, 0, s->stage, desc->vel ? s->stage2 : nullptr, st));
  if (!desc->vel) HIPCHK(s, Launch<T>::init_velocities(d, 0, st));
  // first rebuild with a generous list capacity, then size the capacity
  s->list_cap = 1024;
  labf_status rc = alloc_items<T>(s);
  if (rc != LABF_OK) return rc;
  s->xref_valid = false;
  rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
  if (rc != LABF_OK) return rc;
  for (int attempt = 0; attempt < 4; ++attempt) {
    std::vector<int32_t> cnt(s->C);
    HIPCHK(s, hipStreamSynchronize(st));
    HIPCHK(s, hipMemcpy(cnt.data(), d.list_count, sizeof(int32_t) * s->C, hipMemcpyDeviceToHost));
    int mx_env = 0, mx_a = 0;
    for (int w = 0; w < W; ++w) {
      const WalkerMeta &m = s->meta[w];
      for (int64_t c = m.cl_begin; c < m.cl_begin + m.cap_env; ++c) mx_env = std::max(mx_env, (int)cnt[c]);
      for (int64_t c = m.cl_begin + m.cap_env; c < m.cl_begin + m.cap_env + m.n_acl; ++c)
        mx_a = std::max(mx_a, (int)cnt[c]);
    }
    const int mx = std::max(mx_env, mx_a);
    if (mx >= s->list_cap) {
      s->list_cap *= 2;  // overflowed: grow and rebuild from the same positions
    } else {
      // headroom for denser regions and larger cluster boxes once the
      // configuration relaxes; alchemical clusters (a spread-out solute) get
      // more (overflow is flagged in the walker status)
      const int want = std::max({128, ((int)(2.0 * mx_env) + 64 + 31) / 32 * 32,
                                 ((int)(3.0 * mx_a) + 128 + 31) / 32 * 32});
      if (want >= s->list_cap) break;
      s->list_cap = want;
    }
    rc = alloc_items<T>(s);
    if (rc != LABF_OK) return rc;
    s->xref_valid = false;
    rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
    if (rc != LABF_OK) return rc;
  }
  HIPCHK(s, hipStreamSynchronize(st));
  s->since_rebuild = 0;
  return LABF_OK;
}

template <typename T>
labf_status set_lambda_impl(labf_system *s, const labf_lambda_params *p, hipStream_t st) {
  Dev<T> &d = s->dev<T>();
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
  if (d.bin_count) {
    for (void *q : {(void *)d.bin_count, (void *)d.bin_sum, (void *)d.bin_sum2, (void *)d.loc_count,
                    (void *)d.loc_sum, (void *)d.loc_sum2}) {
      auto it = std::find(s->bufs.ptrs.begin(), s->bufs.ptrs.end(), q);
      if (it != s->bufs.ptrs.end()) {
        (void)hipFree(*it);
        s->bufs.ptrs.erase(it);
      }
    }
  }
  HIPCHK(s, dalloc(s->bufs, &d.bin_count, p->n_bins));
  HIPCHK(s, dalloc(s->bufs, &d.bin_sum, p->n_bins));
  HIPCHK(s, dalloc(s->bufs, &d.bin_sum2, p->n_bins));
  HIPCHK(s, dalloc(s->bufs, &d.loc_count, (size_t)p->n_bins * s->W));
  HIPCHK(s, dalloc(s->bufs, &d.loc_sum, (size_t)p->n_bins * s->W));
  HIPCHK(s, dalloc(s->bufs, &d.loc_sum2, (size_t)p->n_bins * s->W));
  HIPCHK(s, hipMemcpyAsync(s->lam_stage, p->lambda0, sizeof(double) * s->W, hipMemcpyHostToDevice, st));
  if (p->p_lambda0)
    HIPCHK(s, hipMemcpyAsync(s->lam_stage + s->W, p->p_lambda0, sizeof(double) * s->W, hipMemcpyHostToDevice, st));
  HIPCHK(s, launch_init_lambda<T>(d, s->lam_stage, p->p_lambda0 ? s->lam_stage + s->W : nullptr, s->lb, st));
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
  HIPCHK(s, Launch<T>::eval(d, full_range(s), s->xb, s->vb, s->lb, st));
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
// be NULL), rebuild, evaluate every pair term once.
template <typename T>
labf_status energy_eval(labf_system *s, const double *pos, const double *lam, const double *params,
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
  labf_status rc = do_rebuild<T>(s, LABF_MODE_BATCHED, st);
  if (rc != LABF_OK) return rc;
  HIPCHK(s, Launch<T>::eval(d, full_range(s), s->xb, s->vb, s->lb, st));
  return LABF_OK;
}

template <typename T>
labf_status energy_impl(labf_system *s, const double *pos, const double *lam, const double *params,
                        double *energy, hipStream_t st) {
  labf_status rc = energy_eval<T>(s, pos, lam, params, st);
  if (rc != LABF_OK) return rc;
  HIPCHK(s, Launch<T>::energy_total(s->dev<T>(), energy, st));
  return LABF_OK;
}

template <typename T>
labf_status energy_backward_impl(labf_system *s, const double *pos, const double *lam, const double *params,
                                 const double *g, double *gpos, double *glam, double *gpar, hipStream_t st) {
  labf_status rc = energy_eval<T>(s, pos, lam, params, st);
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
  if (!s->dr_partner_dev) {
    HIPCHK(s, dalloc(s->bufs, &s->dr_partner_dev, s->N));
    HIPCHK(s, dalloc(s->bufs, &s->dr_pair_dev, 2 * s->W));
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
    auto it = std::find(s->bufs.ptrs.begin(), s->bufs.ptrs.end(), (void *)s->pairs_dev);
    if (it != s->bufs.ptrs.end()) {
      (void)hipFree(*it);
      s->bufs.ptrs.erase(it);
    }
  }
  HIPCHK(s, dalloc(s->bufs, &s->pairs_dev, (size_t)(2 * n)));
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
  std::vector<hipEvent_t> ev(2 + 3 * n + 1);
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
  for (int64_t i = 0; i < n; ++i) {
    HIPCHK(s, Launch<T>::pme(d, full_range(s), s->xb, s->lb, st));
    HIPCHK(s, hipEventRecord(ev[2 + 3 * i], st));
    HIPCHK(s, Launch<T>::step_alch(d, full_range(s), s->xb, s->vb, s->lb, st));
    HIPCHK(s, hipEventRecord(ev[3 + 3 * i], st));
    HIPCHK(s, Launch<T>::step_env(d, full_range(s), s->xb, s->vb, s->lb, st));
    HIPCHK(s, Launch<T>::env_integrate(d, full_range(s), s->xb, s->vb, s->lb, st));
    HIPCHK(s, hipEventRecord(ev[4 + 3 * i], st));
    s->xb ^= 1;
    s->lb ^= 1;
    s->since_rebuild += 1;
    s->host_steps += 1;
  }
  HIPCHK(s, hipEventSynchronize(ev[1 + 3 * n]));
  float t = 0.f;
  HIPCHK(s, hipEventElapsedTime(&t, ev[0], ev[1]));
  ms[0] = t;
  double a = 0.0, e = 0.0, p = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    HIPCHK(s, hipEventElapsedTime(&t, ev[3 * i + 1], ev[3 * i + 2]));
    p += t;
    HIPCHK(s, hipEventElapsedTime(&t, ev[3 * i + 2], ev[3 * i + 3]));
    a += t;
    HIPCHK(s, hipEventElapsedTime(&t, ev[3 * i + 3], ev[3 * i + 4]));
    e += t;
  }
  ms[1] = a / n;
  ms[2] = e / n;
  ms[3] = d.pme_on ? p / n : 0.0;
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

labf_status labf_energy(labf_system *sys, const double *pos, const double *lambda, const double *params,
                        double *energy, void *stream) {
  if (!sys) return fail(nullptr, LABF_E_ARG, "sys is NULL");
  if (!energy) return fail(sys, LABF_E_ARG, "energy is NULL");
  if (!sys->lam_set) return fail(sys, LABF_E_STATE, "labf_set_lambda_params must be called first");
  return dispatch(sys, [&](auto *tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return energy_impl<T>(sys, pos, lambda, params, energy, (hipStream_t)stream);
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
  sys->item_bufs.release();
  sys->bufs.release();
  delete sys;
}

const char *labf_last_error(const labf_system *sys) {
  if (!sys) return g_create_error.c_str();
  return sys->err.c_str();
}

}  // extern "C"
