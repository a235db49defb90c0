// Out-of-HBM products: the operator values stay in (pinned) host memory and
// stream through a device cache managed as the paper's tree-traversal stack
// (Section II.B, Alg. 1): the terms form a data dependency tree (level 1 the
// left operator, level 2 the right operator, leaves the terms), a depth-first
// walk loads a node's operator on top of the stack, so the left operator
// stays resident for all of its right partners and allocation is a moving
// offset.  Execution is deferred (one product of a few terms would not fill
// the GPU) until the next operator does not fit (an epoch): then every
// pending term runs as one product (tns_apply_heff, accumulating into sigma)
// whose task list was built at plan time with the blocks' cache offsets, and
// the space of the nodes already left is given back.
//
// When that walk needs more than one epoch and every term's two operators fit
// in half the cache, the plan may double-buffer instead: the walk runs on half
// the cache with nothing kept from one epoch to the next, epochs alternate
// between the halves, and the copies of epoch k + 1 run on a second stream
// while epoch k's product runs (they wait only for the product of epoch k - 1,
// the last one that read their half).  That hides the copies after the first
// epoch's but needs more, smaller products, each with a fixed cost (thinner
// panels and task chunks, one more launch sequence); the plan takes the
// halves when the copy they hide exceeds the extra epochs' cost, counted as
// TT_EPOCH_ELEMS copied elements per epoch.
#include <algorithm>
#include <mutex>
#include <vector>

#include "kern.hpp"
#include "tns_internal.hpp"

namespace tns {

// Fixed cost of one more epoch in elements of copy time: 0.43 ms per product
// measured at D = 1024 (FP64, MI355X), the time of 3 M FP64 elements over the
// 57 GB/s pinned host link.
constexpr int64_t TT_EPOCH_ELEMS = 3000000;

struct TtLoad {
  int64_t host_off, cache_off, elems;  // elements of the operator value arrays
};

// Host-side plan, in the caller's host buffer: epoch records, loads, task lists.
struct TtEpoch {
  int64_t load_begin, load_end;  // loads issued before the epoch's product
  int64_t dev_off;               // its task list's build workspace in the device buffer
  int64_t ws_bytes;              // size of that workspace
};

struct TtHeader {
  int64_t n_epochs, n_loads, cache_elems, psi_dim;
  int64_t halves;  // 1: double-buffered (epoch k in half k mod 2)
  TtEpoch *epochs;
  TtLoad *loads;
  tns_tasklist *tls;  // one per epoch
};
static_assert(sizeof(TtHeader) <= 256, "TtHeader fits the plan's opaque bytes");

static inline TtHeader &tt_of(tns_ttcache_plan *p) { return *reinterpret_cast<TtHeader *>(p->opaque); }
static inline const TtHeader &tt_of(const tns_ttcache_plan *p) { return *reinterpret_cast<const TtHeader *>(p->opaque); }

// One epoch while planning: loads, resident operators (cache offset per op),
// terms to run.
struct TtPlanEpoch {
  std::vector<TtLoad> loads;
  std::vector<std::pair<int, int64_t>> resident;  // (operator, cache offset of its first element)
  std::vector<int> terms;
};

// Element range of every operator's blocks in the value array.
static void op_extents(const tns_problem *P, std::vector<int64_t> &lo, std::vector<int64_t> &hi) {
  lo.assign(P->nOps, INT64_MAX);
  hi.assign(P->nOps, -1);
  for (int b = 0; b < P->nBlk; ++b) {
    const int o = P->blk_op[b];
    lo[o] = std::min(lo[o], P->blk_off[b]);
    hi[o] = std::max(hi[o], P->blk_off[b] + (int64_t)P->blk_rows[b] * P->blk_ld[b]);
  }
  for (int o = 0; o < P->nOps; ++o)
    if (hi[o] < 0) lo[o] = hi[o] = 0;  // an operator without blocks loads nothing
}

// Depth-first walk of the dependency tree with the stack cache: level 1 the
// operator of side `lead` (0 left, 1 right) of each term, level 2 the other
// one, leaves the terms.  Entering a node loads its operator at the top of
// the stack unless it is still there; the terms are collected, not run.
// Leaving a node would let its siblings reuse the space, but the collected
// terms still read it, so the space is given back only when they run: a
// level-1 subtree whose new operators do not all fit above the stack starts
// at the bottom after the pending terms have formed an epoch, and inside a
// subtree an operator that does not fit makes an epoch and pops back to the
// level-1 operator.  Every level-1 operator is thus copied once and every
// level-2 operator at most once per parent (never more than a per-term copy),
// operators still on the stack are reused across subtrees, and a cache that
// holds everything copies each operator once and runs one product.  With
// carry false an epoch keeps nothing of the previous one (the level-1
// operator is copied again), so that consecutive epochs may use separate
// buffers.  Returns TNS_ERR_WORKSPACE when two operators of one term together
// exceed the cache.
static tns_status tt_walk(const tns_problem *P, int64_t cap, int lead, bool carry, std::vector<TtPlanEpoch> &epochs,
                          int64_t *naive, int64_t *loaded) {
  std::vector<int64_t> lo, hi;
  op_extents(P, lo, hi);
  auto size_of = [&](int o) { return o >= 0 ? (hi[o] - lo[o] + 7) / 8 * 8 : 0; };
  auto ext = [&](int o) { return o >= 0 ? hi[o] - lo[o] : 0; };
  const int32_t *first = lead ? P->term_R : P->term_L, *second = lead ? P->term_L : P->term_R;
  std::vector<int> order(P->nTerms);
  for (int t = 0; t < P->nTerms; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return first[a] != first[b] ? first[a] < first[b] : second[a] < second[b];
  });
  *naive = *loaded = 0;
  for (int t = 0; t < P->nTerms; ++t) *naive += ext(P->term_L[t]) + ext(P->term_R[t]);
  std::vector<int64_t> at(P->nOps, -1);  // cache offset of each operator on the stack
  std::vector<int> on;                   // operators on the stack
  int64_t top = 0;
  TtPlanEpoch cur;
  auto push = [&](int o) {
    at[o] = top;
    on.push_back(o);
    if (ext(o)) {
      cur.loads.push_back({lo[o], top, ext(o)});
      *loaded += ext(o);
    }
    top += size_of(o);
  };
  auto flush = [&]() {
    if (cur.terms.empty()) return;
    // one copy for operators adjacent both in host memory and in the cache
    std::vector<TtLoad> merged;
    for (auto &l : cur.loads) {
      if (!merged.empty()) {
        TtLoad &m = merged.back();
        const int64_t step = (m.elems + 7) / 8 * 8;  // its footprint: the gap up to the next is in range
        if (l.host_off == m.host_off + step && l.cache_off == m.cache_off + step) {
          m.elems = step + l.elems;
          continue;
        }
      }
      merged.push_back(l);
    }
    cur.loads.swap(merged);
    cur.resident.clear();
    for (int o : on) cur.resident.push_back({o, at[o]});
    epochs.push_back(cur);
    cur = TtPlanEpoch();
  };
  // room for operator o (o1: the level-1 operator that must stay resident)
  auto room = [&](int o, int o1) -> bool {
    if (top + size_of(o) <= cap) return true;
    bool kept = false;
    if (cur.terms.empty()) {  // nothing pending reads this epoch's copies: drop them
      bool bottom = false;
      for (auto &l : cur.loads) {
        *loaded -= l.elems;
        bottom = bottom || l.cache_off == 0;
      }
      cur.loads.clear();
      kept = carry && o1 >= 0 && at[o1] == 0 && !bottom;  // a copy made before this epoch stays valid
    } else {
      flush();
      kept = carry && o1 >= 0 && at[o1] == 0;  // its copy at the bottom stays valid
    }
    for (int x : on) at[x] = -1;
    on.clear();
    top = 0;
    if (o1 >= 0) {
      if (size_of(o1) + size_of(o) > cap) return false;
      if (kept) {
        at[o1] = 0;
        on.push_back(o1);
        top = size_of(o1);
      } else {
        push(o1);  // reloaded at the bottom
      }
    }
    return size_of(o) <= cap;
  };
  size_t i = 0;
  while (i < order.size()) {
    const int o1 = first[order[i]];
    size_t end = i;
    while (end < order.size() && first[order[end]] == o1) ++end;
    // the subtree's new operators; when they do not all fit above the stack,
    // start it at the bottom (so that o1 is never copied twice)
    int64_t need = o1 >= 0 ? size_of(o1) : 0;
    for (size_t u = i; u < end; ++u) {
      const int o2 = second[order[u]];
      if (o2 >= 0 && at[o2] < 0 && (u == i || second[order[u - 1]] != o2)) need += size_of(o2);
    }
    if (top + need > cap) {
      if (cur.terms.empty()) {
        for (auto &l : cur.loads) *loaded -= l.elems;
        cur.loads.clear();
      } else {
        flush();
      }
      for (int x : on) at[x] = -1;
      on.clear();
      top = 0;
    }
    if (o1 >= 0) {
      if (size_of(o1) > cap) return TNS_ERR_WORKSPACE;
      push(o1);
    }
    while (i < end) {
      const int o2 = second[order[i]];
      if (o2 >= 0 && at[o2] < 0) {
        if (!room(o2, o1)) return TNS_ERR_WORKSPACE;
        push(o2);
      }
      while (i < end && second[order[i]] == o2) cur.terms.push_back(order[i++]);
    }
  }
  flush();
  return TNS_OK;
}

// The sub-problem of an epoch: its terms, the blocks of its resident
// operators at their cache offsets; everything else of P.
struct TtSub {
  std::vector<int32_t> bop, bin, bout, brows, bcols, bld, tL, ta, tb, tR;
  std::vector<int64_t> boff;
  std::vector<double> tc;
  tns_problem P;
};

static void tt_sub(const tns_problem *P, const TtPlanEpoch &e, int64_t cap, TtSub &s) {
  std::vector<int64_t> lo, hi;
  op_extents(P, lo, hi);
  std::vector<int64_t> at(P->nOps, -1);
  for (auto &r : e.resident)
    if (r.first >= 0) at[r.first] = r.second;
  for (int b = 0; b < P->nBlk; ++b) {
    const int o = P->blk_op[b];
    if (at[o] < 0) continue;
    s.bop.push_back(o); s.bin.push_back(P->blk_in[b]); s.bout.push_back(P->blk_out[b]);
    s.brows.push_back(P->blk_rows[b]); s.bcols.push_back(P->blk_cols[b]); s.bld.push_back(P->blk_ld[b]);
    s.boff.push_back(at[o] + (P->blk_off[b] - lo[o]));
  }
  for (int t : e.terms) {
    s.tL.push_back(P->term_L[t]); s.ta.push_back(P->term_ma[t]); s.tb.push_back(P->term_mb[t]);
    s.tR.push_back(P->term_R[t]); s.tc.push_back(P->term_coef[t]);
  }
  s.P = *P;
  s.P.nBlk = (int32_t)s.bop.size();
  s.P.nTerms = (int32_t)s.tL.size();
  s.P.n_vals = cap;
  s.P.blk_op = s.bop.data(); s.P.blk_in = s.bin.data(); s.P.blk_out = s.bout.data();
  s.P.blk_rows = s.brows.data(); s.P.blk_cols = s.bcols.data(); s.P.blk_ld = s.bld.data();
  s.P.blk_off = s.boff.data();
  s.P.term_L = s.tL.data(); s.P.term_ma = s.ta.data(); s.P.term_mb = s.tb.data(); s.P.term_R = s.tR.data();
  s.P.term_coef = s.tc.data();
}

// The walk of the better tree: level 1 the left or the right operators,
// whichever copies fewer elements (left on a tie).
static tns_status tt_best_walk(const tns_problem *P, int64_t cap, bool carry, std::vector<TtPlanEpoch> &epochs,
                               int64_t *naive, int64_t *loaded) {
  std::vector<TtPlanEpoch> alt;
  int64_t nv2 = 0, ld2 = 0;
  tns_status s = tt_walk(P, cap, 0, carry, epochs, naive, loaded);
  const tns_status s2 = tt_walk(P, cap, 1, carry, alt, &nv2, &ld2);
  if (s2 == TNS_OK && (s != TNS_OK || ld2 < *loaded)) {
    epochs.swap(alt);
    *loaded = ld2;
    s = TNS_OK;
  }
  return s;
}

// Blocks are read at element offsets that are multiples of 8: the cache keeps
// each operator's first element at a multiple of 8 (sizes rounded up), so the
// rebased offsets stay multiples of 8 when the host ones are.
static tns_status tt_plan(const tns_problem *P, int64_t cap, int32_t mode, std::vector<TtPlanEpoch> &epochs,
                          std::vector<size_t> &ws, int64_t *naive, int64_t *loaded, bool *halves) {
  int32_t nmax = 0, maxdim = 0;
  tns_status s = validate_problem(P, &nmax, &maxdim);
  if (s != TNS_OK) return s;
  if (cap <= 0 || (mode != TNS_TT_AUTO && mode != TNS_TT_SINGLE && mode != TNS_TT_DOUBLE)) return TNS_ERR_ARG;
  const int64_t c8 = (cap / 8) * 8;
  s = tt_best_walk(P, c8, true, epochs, naive, loaded);
  if (s != TNS_OK) return s;
  *halves = false;
  const int64_t h8 = c8 / 16 * 8;  // half the cache, a multiple of 8
  if (mode != TNS_TT_SINGLE && epochs.size() > 1 && h8 > 0) {
    std::vector<TtPlanEpoch> hv;
    int64_t nv = 0, ld = 0;
    int64_t first = 0;
    const bool ok = tt_best_walk(P, h8, false, hv, &nv, &ld) == TNS_OK;
    if (ok)
      for (auto &l : hv[0].loads) first += l.elems;
    const int64_t hidden = ld - first, extra = ((int64_t)hv.size() - (int64_t)epochs.size()) * TT_EPOCH_ELEMS;
    if (ok && (mode == TNS_TT_DOUBLE || hidden > extra)) {
      for (size_t k = 1; k < hv.size(); k += 2) {  // odd epochs in the upper half
        for (auto &l : hv[k].loads) l.cache_off += h8;
        for (auto &r : hv[k].resident) r.second += h8;
      }
      epochs.swap(hv);
      *loaded = ld;
      *halves = true;
    }
  }
  if (s != TNS_OK) return s;
  ws.clear();
  for (auto &e : epochs) {
    TtSub sub;
    tt_sub(P, e, cap, sub);
    int32_t nm = 0, md = 0;
    s = validate_problem(&sub.P, &nm, &md);
    if (s != TNS_OK) return s;
    const size_t b = plan_workspace(&sub.P, nm, md, -1, false);
    if (b == 0) return TNS_ERR_SHAPE;
    ws.push_back(align_up(b, 256));
  }
  return TNS_OK;
}

template <class T>
__global__ void k_tt_zero(T *p, int64_t n) {
  GRID_STRIDE(i, n) p[i] = T(0);
}

// Copy stream and events of double-buffered products, one set per device,
// created on first use with that device current (default priority).  Every
// call on a device shares them: calls that overlap in time on one device
// must be issued on one stream.
struct TtStreams {
  hipStream_t copy = nullptr;
  hipEvent_t start = nullptr, load[2] = {nullptr, nullptr}, prod[2] = {nullptr, nullptr};
};
constexpr int TT_MAX_DEVICES = 64;
static std::mutex g_tt_mu;
static TtStreams g_tt[TT_MAX_DEVICES];

static tns_status tt_streams(hipStream_t st, TtStreams **out) {
  int dev = -1, cur = -1;
  TNS_HIP(hipStreamGetDevice(st, &dev));
  TNS_HIP(hipGetDevice(&cur));
  if (dev < 0 || dev >= TT_MAX_DEVICES) return TNS_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_tt_mu);
  TtStreams &T = g_tt[dev];
  if (!T.copy) {
    if (dev != cur) TNS_HIP(hipSetDevice(dev));
    TtStreams n;
    hipError_t e = hipStreamCreateWithFlags(&n.copy, hipStreamNonBlocking);
    hipEvent_t *evs[5] = {&n.start, &n.load[0], &n.load[1], &n.prod[0], &n.prod[1]};
    for (int i = 0; i < 5 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(evs[i], hipEventDisableTiming);
    if (dev != cur) TNS_HIP(hipSetDevice(cur));
    if (e != hipSuccess) return TNS_ERR_HIP;
    T = n;
  }
  *out = &T;
  return TNS_OK;
}

}  // namespace tns

using namespace tns;

extern "C" tns_status tns_ttcache_sizes(const tns_problem *P, int64_t cache_elems, int32_t mode, size_t *host_bytes,
                                        size_t *dev_bytes, int64_t *n_epochs) {
  if (!host_bytes || !dev_bytes) return TNS_ERR_ARG;
  std::vector<TtPlanEpoch> epochs;
  std::vector<size_t> ws;
  int64_t naive = 0, loaded = 0;
  bool halves = false;
  const tns_status s = tt_plan(P, cache_elems, mode, epochs, ws, &naive, &loaded, &halves);
  if (s != TNS_OK) return s;
  size_t nl = 0, db = 0;
  for (auto &e : epochs) nl += e.loads.size();
  for (size_t b : ws) db += b;
  *host_bytes = align_up(epochs.size() * sizeof(TtEpoch), 64) + align_up(nl * sizeof(TtLoad), 64) +
                epochs.size() * sizeof(tns_tasklist) + 64;
  *dev_bytes = db;
  if (n_epochs) *n_epochs = (int64_t)epochs.size();
  return TNS_OK;
}

extern "C" tns_status tns_ttcache_build(const tns_problem *P, int64_t cache_elems, int32_t mode, void *host_buf,
                                        size_t host_bytes, void *dev_ws, size_t dev_bytes, tns_ttcache_plan *out,
                                        hipStream_t st) {
  if (!host_buf || !dev_ws || !out) return TNS_ERR_ARG;
  std::vector<TtPlanEpoch> epochs;
  std::vector<size_t> ws;
  int64_t naive = 0, loaded = 0;
  bool halves = false;
  tns_status s = tt_plan(P, cache_elems, mode, epochs, ws, &naive, &loaded, &halves);
  if (s != TNS_OK) return s;
  size_t hb = 0, db = 0;
  int64_t ne = 0;
  s = tns_ttcache_sizes(P, cache_elems, mode, &hb, &db, &ne);
  if (s != TNS_OK) return s;
  if (host_bytes < hb || dev_bytes < db) return TNS_ERR_WORKSPACE;
  memset(out, 0, sizeof(*out));
  TtHeader &h = tt_of(out);
  char *c = reinterpret_cast<char *>(host_buf);
  h.epochs = reinterpret_cast<TtEpoch *>(c);
  c += align_up(epochs.size() * sizeof(TtEpoch), 64);
  h.loads = reinterpret_cast<TtLoad *>(c);
  size_t nl = 0;
  for (auto &e : epochs) nl += e.loads.size();
  c += align_up(nl * sizeof(TtLoad), 64);
  h.tls = reinterpret_cast<tns_tasklist *>(c);
  h.n_epochs = (int64_t)epochs.size();
  h.n_loads = (int64_t)nl;
  h.cache_elems = cache_elems;
  h.psi_dim = P->psi_off[P->nS];
  h.halves = halves ? 1 : 0;
  int64_t li = 0, doff = 0, tasks = 0, flops = 0;
  char *dws = reinterpret_cast<char *>(dev_ws);
  for (size_t k = 0; k < epochs.size(); ++k) {
    TtEpoch &E = h.epochs[k];
    E.load_begin = li;
    for (auto &l : epochs[k].loads) h.loads[li++] = l;
    E.load_end = li;
    E.dev_off = doff;
    E.ws_bytes = (int64_t)ws[k];
    TtSub sub;
    tt_sub(P, epochs[k], cache_elems, sub);
    int32_t nm = 0, md = 0;
    s = validate_problem(&sub.P, &nm, &md);
    if (s != TNS_OK) return s;
    s = build_plan(&sub.P, nm, md, nullptr, nullptr, 0, false, dws + doff, ws[k], &h.tls[k], st);
    if (s != TNS_OK) return s;
    tasks += h.tls[k].ntasks;
    flops += h.tls[k].total_flops;
    doff += (int64_t)ws[k];
  }
  out->n_epochs = h.n_epochs;
  out->n_loads = h.n_loads;
  out->loaded_elems = loaded;
  out->naive_elems = naive;
  out->ntasks = tasks;
  out->total_flops = flops;
  out->cache_elems = cache_elems;
  out->halves = h.halves;
  return TNS_OK;
}

extern "C" size_t tns_ttcache_apply_workspace_bytes(const tns_ttcache_plan *p, tns_prec prec) {
  if (!p || (prec != TNS_F64 && prec != TNS_F32)) return 0;
  const TtHeader &h = tt_of(p);
  size_t b = 256;
  for (int64_t k = 0; k < h.n_epochs; ++k) b = std::max(b, fwd_workspace(plan_of(&h.tls[k]), prec));
  return b;
}

extern "C" tns_status tns_apply_heff_streamed(const tns_ttcache_plan *p, tns_prec prec, const void *host_vals,
                                              void *cache, const void *psi, void *sigma, void *ws, size_t ws_bytes,
                                              hipStream_t st) {
  if (!p || !host_vals || !cache || !psi || !sigma || !ws) return TNS_ERR_ARG;
  if (prec != TNS_F64 && prec != TNS_F32) return TNS_ERR_ARG;
  if (ws_bytes < tns_ttcache_apply_workspace_bytes(p, prec)) return TNS_ERR_WORKSPACE;
  const TtHeader &h = tt_of(p);
  const size_t es = prec == TNS_F64 ? 8 : 4;
  const char *hv = reinterpret_cast<const char *>(host_vals);
  char *cv = reinterpret_cast<char *>(cache);
  if (h.n_epochs == 0) {  // no terms: sigma = 0
    if (h.psi_dim > 0) {
      const unsigned nb = (unsigned)std::min<int64_t>((h.psi_dim + 255) / 256, 1 << 16);
      if (prec == TNS_F64) hipLaunchKernelGGL(k_tt_zero<double>, dim3(nb), dim3(256), 0, st, (double *)sigma, h.psi_dim);
      else hipLaunchKernelGGL(k_tt_zero<float>, dim3(nb), dim3(256), 0, st, (float *)sigma, h.psi_dim);
    }
    return hipGetLastError() == hipSuccess ? TNS_OK : TNS_ERR_HIP;
  }
  if (!h.halves) {
    for (int64_t k = 0; k < h.n_epochs; ++k) {
      const TtEpoch &E = h.epochs[k];
      // the epoch's loads follow the previous epoch's product on the stream,
      // so they never overwrite operators that product still reads
      for (int64_t l = E.load_begin; l < E.load_end; ++l) {
        const TtLoad &L = h.loads[l];
        TNS_HIP(hipMemcpyAsync(cv + L.cache_off * es, hv + L.host_off * es, (size_t)L.elems * es,
                               hipMemcpyHostToDevice, st));
      }
      const tns_status s = tns_apply_heff(&h.tls[k], prec, cache, psi, sigma, k == 0 ? 0.0 : 1.0, ws, ws_bytes, st);
      if (s != TNS_OK) return s;
    }
    return TNS_OK;
  }
  // double-buffered: the copies of epoch k (half k mod 2) on the copy stream
  // after the stream's earlier work and the product of epoch k - 2, the
  // product of epoch k on `stream` after those copies; the last product waits
  // for every copy, so later work on `stream` follows the whole call
  TtStreams *T = nullptr;
  tns_status s = tt_streams(st, &T);
  if (s != TNS_OK) return s;
  TNS_HIP(hipEventRecord(T->start, st));
  TNS_HIP(hipStreamWaitEvent(T->copy, T->start, 0));
  for (int64_t k = 0; k < h.n_epochs; ++k) {
    const TtEpoch &E = h.epochs[k];
    if (k >= 2) TNS_HIP(hipStreamWaitEvent(T->copy, T->prod[k & 1], 0));
    for (int64_t l = E.load_begin; l < E.load_end; ++l) {
      const TtLoad &L = h.loads[l];
      TNS_HIP(hipMemcpyAsync(cv + L.cache_off * es, hv + L.host_off * es, (size_t)L.elems * es,
                             hipMemcpyHostToDevice, T->copy));
    }
    TNS_HIP(hipEventRecord(T->load[k & 1], T->copy));
    TNS_HIP(hipStreamWaitEvent(st, T->load[k & 1], 0));
    s = tns_apply_heff(&h.tls[k], prec, cache, psi, sigma, k == 0 ? 0.0 : 1.0, ws, ws_bytes, st);
    if (s != TNS_OK) return s;
    TNS_HIP(hipEventRecord(T->prod[k & 1], st));
  }
  return TNS_OK;
}
