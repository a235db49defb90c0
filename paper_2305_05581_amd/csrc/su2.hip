// Spin-adapted (SU(2)) two-block products (Section IV.E): the sectors of each
// block are spin multiplets, operators are tensor operators given by their
// reduced blocks, and a term couples a left and a right operator of equal rank
// to a spin scalar.  By the Wigner-Eckart theorem every task of Eq. (2) (term,
// input sector, one reduced block per side) is the U(1) task times one scalar
// that depends only on the spins of its sectors and the rank, precalculated
// here on the host; the products then run on the U(1) path's kernels unchanged.
//
// Reduced blocks use the Clebsch-Gordan convention
//   <j' m'| T_q |j m> = <j m; k q | j' m'> <j'||T||j>,
// a term is coef [T_L x T_R]^0 = coef sum_q <k q; k -q | 0 0> T_L,q T_R,-q (left
// factor first), and the wavefunction element (a, b) of sector (iL, iR) is the
// coupled state sum_mL <SL mL; SR S-mL | S S> |a SL mL> |b SR S-mL>.  The task
// scalar is then
//   W = sum_{mL, q} <SL' mL+q; SR' S-mL-q | S S> <SL mL; SR S-mL | S S>
//       <k q; k -q | 0 0> <SL mL; k q | SL' mL+q> <SR S-mL; k -q | SR' S-mL-q>
// times the fermionic sign (-1)^(p_R N_L) of moving the right factor past the
// input's left electrons.
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "kern.hpp"
#include "tns_internal.hpp"

namespace tns {

// <j1 m1; j2 m2 | j m>, every argument doubled, by Racah's closed formula.
static double cg2(int j1, int m1, int j2, int m2, int j, int m) {
  static const std::array<double, 64> fact = [] {
    std::array<double, 64> f;
    f[0] = 1.0;
    for (int i = 1; i < 64; ++i) f[i] = f[i - 1] * (double)i;
    return f;
  }();
  if (m1 + m2 != m || std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m) > j) return 0.0;
  if (((j1 + m1) & 1) || ((j2 + m2) & 1) || ((j + m) & 1)) return 0.0;
  if (j > j1 + j2 || j < std::abs(j1 - j2) || ((j1 + j2 + j) & 1)) return 0.0;
  const int a = (j1 + j2 - j) / 2, b = (j1 - j2 + j) / 2, c = (-j1 + j2 + j) / 2, d = (j1 + j2 + j) / 2 + 1;
  if (d >= 64) return NAN;
  const double pre = std::sqrt((double)(j + 1) * fact[a] * fact[b] * fact[c] / fact[d] * fact[(j1 + m1) / 2] *
                               fact[(j1 - m1) / 2] * fact[(j2 + m2) / 2] * fact[(j2 - m2) / 2] * fact[(j + m) / 2] *
                               fact[(j - m) / 2]);
  double sum = 0.0;
  for (int k = 0; k <= a; ++k) {
    const int e1 = (j1 - m1) / 2 - k, e2 = (j2 + m2) / 2 - k, e3 = (j - j2 + m1) / 2 + k, e4 = (j - j1 - m2) / 2 + k;
    if (e1 < 0 || e2 < 0) break;
    if (e3 < 0 || e4 < 0) continue;
    const double t = 1.0 / (fact[k] * fact[a - k] * fact[e1] * fact[e2] * fact[e3] * fact[e4]);
    sum += (k & 1) ? -t : t;
  }
  return pre * sum;
}

// The task scalar W of the header comment (spins doubled: sl, sr in, slp, srp
// out, s total, k rank).
static double recouple(int slp, int srp, int s, int sl, int sr, int k) {
  double w = 0.0;
  for (int ml = -sl; ml <= sl; ml += 2) {
    const double in = cg2(sl, ml, sr, s - ml, s, s);
    if (in == 0.0) continue;
    for (int q = -k; q <= k; q += 2) {
      const double x = cg2(k, q, k, -q, 0, 0) * cg2(sl, ml, k, q, slp, ml + q) * cg2(sr, s - ml, k, -q, srp, s - ml - q);
      if (x == 0.0) continue;
      w += in * x * cg2(slp, ml + q, srp, s - ml - q, s, s);
    }
  }
  return w;
}

static inline bool triangle(int a, int b, int c) { return c >= std::abs(a - b) && c <= a + b && ((a + b + c) & 1) == 0; }

struct Su2Host {
  std::vector<int32_t> psi_sec, secL, secR;
  std::vector<int64_t> psi_off;
  std::vector<tns_task> tasks;
  std::vector<int32_t> ptr;
  int32_t maxdim = 1, nmax = 1;
};

static tns_status su2_host(const tns_su2_problem *P, Su2Host &h) {
  if (!P) return TNS_ERR_ARG;
  if (P->nL <= 0 || P->nR <= 0 || P->nOps < 0 || P->nBlk < 0 || P->nTerms < 0 || P->n_vals < 0) return TNS_ERR_ARG;
  if (!P->qL || !P->dimL || !P->qR || !P->dimR) return TNS_ERR_ARG;
  if (P->nOps > 0 && (!P->op_side || !P->op_2k || !P->op_dN)) return TNS_ERR_ARG;
  if (P->nBlk > 0 && (!P->blk_op || !P->blk_in || !P->blk_out || !P->blk_rows || !P->blk_cols || !P->blk_ld ||
                      !P->blk_off))
    return TNS_ERR_ARG;
  if (P->nTerms > 0 && (!P->term_L || !P->term_R || !P->term_coef)) return TNS_ERR_ARG;
  if (P->target_2S < 0 || ((P->target_N - P->target_2S) & 1)) return TNS_ERR_QN;
  for (int side = 0; side < 2; ++side) {
    const int n = side ? P->nR : P->nL;
    const int32_t *q = side ? P->qR : P->qL, *dim = side ? P->dimR : P->dimL;
    for (int i = 0; i < n; ++i) {
      if (dim[i] <= 0 || dim[i] > MAX_DIM) return TNS_ERR_SHAPE;
      if (q[2 * i + 1] < 0 || ((q[2 * i] - q[2 * i + 1]) & 1)) return TNS_ERR_QN;
      if (i > 0 && (q[2 * i] < q[2 * i - 2] || (q[2 * i] == q[2 * i - 2] && q[2 * i + 1] <= q[2 * i - 1])))
        return TNS_ERR_QN;
      h.maxdim = std::max(h.maxdim, dim[i]);
    }
  }
  h.nmax = std::max(P->nL, P->nR);
  for (int o = 0; o < P->nOps; ++o) {
    if (P->op_side[o] != 0 && P->op_side[o] != 1) return TNS_ERR_ARG;
    if (P->op_2k[o] < 0 || P->op_2k[o] > 16 || std::abs(P->op_dN[o]) > 4) return TNS_ERR_ARG;
    if ((P->op_dN[o] - P->op_2k[o]) & 1) return TNS_ERR_QN;  // half-integer rank <=> odd electron change
  }
  // blocks: quantum numbers, shapes, layout, one block per (op, in, out)
  std::map<std::tuple<int, int, int>, int> seen;
  std::vector<std::vector<int>> by_op_in((size_t)P->nOps * h.nmax);
  for (int b = 0; b < P->nBlk; ++b) {
    const int o = P->blk_op[b];
    if (o < 0 || o >= P->nOps) return TNS_ERR_SHAPE;
    const int side = P->op_side[o], n = side ? P->nR : P->nL;
    const int32_t *q = side ? P->qR : P->qL, *dim = side ? P->dimR : P->dimL;
    const int i = P->blk_in[b], j = P->blk_out[b];
    if (i < 0 || i >= n || j < 0 || j >= n) return TNS_ERR_SHAPE;
    if (q[2 * j] != q[2 * i] + P->op_dN[o] || !triangle(q[2 * i + 1], P->op_2k[o], q[2 * j + 1])) return TNS_ERR_QN;
    if (P->blk_rows[b] != dim[j] || P->blk_cols[b] != dim[i] || P->blk_ld[b] < P->blk_cols[b]) return TNS_ERR_SHAPE;
    if (P->blk_off[b] < 0 || P->blk_off[b] % 8 != 0 || P->blk_ld[b] % 8 != 0 ||
        P->blk_off[b] + (int64_t)P->blk_rows[b] * P->blk_ld[b] > P->n_vals)
      return TNS_ERR_SHAPE;
    if (seen[std::make_tuple(o, i, j)]++) return TNS_ERR_SHAPE;
    by_op_in[(size_t)o * h.nmax + i].push_back(b);
  }
  for (int t = 0; t < P->nTerms; ++t) {
    const int oL = P->term_L[t], oR = P->term_R[t];
    if (oL < -1 || oL >= P->nOps || oR < -1 || oR >= P->nOps) return TNS_ERR_ARG;
    if ((oL >= 0 && P->op_side[oL] != 0) || (oR >= 0 && P->op_side[oR] != 1)) return TNS_ERR_ARG;
    const int kL = oL >= 0 ? P->op_2k[oL] : 0, kR = oR >= 0 ? P->op_2k[oR] : 0;
    const int nL = oL >= 0 ? P->op_dN[oL] : 0, nR = oR >= 0 ? P->op_dN[oR] : 0;
    if (kL != kR || nL + nR != 0) return TNS_ERR_QN;
    if (!std::isfinite(P->term_coef[t])) return TNS_ERR_NUMERIC;
  }
  // wavefunction sectors (iL, iR), ascending
  std::map<std::pair<int, int>, int> sec_of;
  h.psi_off.assign(1, 0);
  for (int a = 0; a < P->nL; ++a)
    for (int b = 0; b < P->nR; ++b) {
      if (P->qL[2 * a] + P->qR[2 * b] != P->target_N || !triangle(P->qL[2 * a + 1], P->qR[2 * b + 1], P->target_2S))
        continue;
      sec_of[{a, b}] = (int)h.secL.size();
      h.secL.push_back(a);
      h.secR.push_back(b);
      h.psi_sec.insert(h.psi_sec.end(), {a, 0, 0, b});
      h.psi_off.push_back(h.psi_off.back() + (int64_t)P->dimL[a] * P->dimR[b]);
    }
  const int nS = (int)h.secL.size();
  if (nS == 0) return TNS_ERR_QN;  // no sector of the target
  // tasks in (term, input sector, left block, right block) order, then stable by output sector
  std::map<std::tuple<int, int, int, int, int>, double> wcache;
  std::vector<tns_task> raw;
  const std::vector<int> ident(1, -1);
  for (int t = 0; t < P->nTerms; ++t) {
    const int oL = P->term_L[t], oR = P->term_R[t];
    const int k = oL >= 0 ? P->op_2k[oL] : 0;
    const int pR = oR >= 0 ? (std::abs(P->op_dN[oR]) & 1) : 0;
    for (int s = 0; s < nS; ++s) {
      const int iL = h.secL[s], iR = h.secR[s];
      const std::vector<int> &bl = oL >= 0 ? by_op_in[(size_t)oL * h.nmax + iL] : ident;
      const std::vector<int> &br = oR >= 0 ? by_op_in[(size_t)oR * h.nmax + iR] : ident;
      for (int lb : bl)
        for (int rb : br) {
          const int jL = lb >= 0 ? P->blk_out[lb] : iL, jR = rb >= 0 ? P->blk_out[rb] : iR;
          auto it = sec_of.find({jL, jR});
          if (it == sec_of.end()) continue;
          const int sl = P->qL[2 * iL + 1], sr = P->qR[2 * iR + 1], slp = P->qL[2 * jL + 1], srp = P->qR[2 * jR + 1];
          const auto key = std::make_tuple(slp, srp, sl, sr, k);
          auto wc = wcache.find(key);
          const double w = wc != wcache.end() ? wc->second : (wcache[key] = recouple(slp, srp, P->target_2S, sl, sr, k));
          if (!std::isfinite(w)) return TNS_ERR_SHAPE;  // spins beyond the factorial table
          if (std::fabs(w) < 1e-13) continue;
          tns_task x;
          x.out = it->second;
          x.in = s;
          x.term = t;
          x.lblk = lb;
          x.rblk = rb;
          x.alpha = (P->term_coef[t] * w) * (((pR * P->qL[2 * iL]) & 1) ? -1.0 : 1.0);
          const int64_t q = P->dimL[jL], m = P->dimL[iL], n = P->dimR[iR], r = P->dimR[jR];
          if (lb >= 0 && rb >= 0) {
            const int64_t c0 = 2 * q * n * (m + r), c1 = 2 * m * r * (n + q);
            if (c1 < c0) { x.order = 1; x.cost = c1; } else { x.order = 0; x.cost = c0; }
          } else if (lb >= 0) {
            x.order = 0; x.cost = 2 * q * m * n;
          } else if (rb >= 0) {
            x.order = 0; x.cost = 2 * m * n * r;
          } else {
            x.order = 0; x.cost = 2 * m * n;
          }
          raw.push_back(x);
        }
    }
  }
  if ((int64_t)raw.size() > INT32_MAX) return TNS_ERR_SHAPE;
  h.ptr.assign(nS + 1, 0);
  for (auto &x : raw) h.ptr[x.out + 1] += 1;
  for (int s = 0; s < nS; ++s) h.ptr[s + 1] += h.ptr[s];
  std::vector<int32_t> fill(h.ptr.begin(), h.ptr.end() - 1);
  h.tasks.resize(raw.size());
  for (auto &x : raw) h.tasks[fill[x.out]++] = x;
  return TNS_OK;
}

// The problem the U(1) schedule builder takes: sectors as they are, the
// wavefunction sectors (iL, 0, 0, iR), the reduced blocks; the explicit task
// table replaces the terms.
static tns_problem su2_generic(const tns_su2_problem *P, const Su2Host &h) {
  tns_problem G;
  memset(&G, 0, sizeof(G));
  G.nL = P->nL;
  G.nR = P->nR;
  G.nS = (int32_t)h.secL.size();
  G.nOps = 0;
  G.nBlk = P->nBlk;
  G.nTerms = 0;
  G.target_N = P->target_N;
  G.target_2Sz = P->target_2S;
  G.n_vals = std::max<int64_t>(P->n_vals, 8);
  G.qL = P->qL; G.dimL = P->dimL; G.qR = P->qR; G.dimR = P->dimR;
  G.psi_sec = h.psi_sec.data();
  G.psi_off = h.psi_off.data();
  G.blk_op = P->blk_op; G.blk_in = P->blk_in; G.blk_out = P->blk_out;
  G.blk_rows = P->blk_rows; G.blk_cols = P->blk_cols; G.blk_ld = P->blk_ld; G.blk_off = P->blk_off;
  return G;
}

}  // namespace tns

using namespace tns;

extern "C" size_t tns_su2_workspace_bytes(const tns_su2_problem *prob) {
  Su2Host h;
  if (su2_host(prob, h) != TNS_OK) return 0;
  const tns_problem G = su2_generic(prob, h);
  const size_t b = plan_workspace(&G, h.nmax, h.maxdim, (int64_t)h.tasks.size(), false);
  return b ? align_up(b, 256) : 0;
}

extern "C" tns_status tns_su2_tables(const tns_su2_problem *prob, int32_t *sec_L, int32_t *sec_R, int64_t *psi_off,
                                     int64_t cap_sectors, tns_task *tasks, int32_t *task_ptr, int64_t cap_tasks,
                                     int64_t *n_sectors, int64_t *n_tasks) {
  if (!n_sectors || !n_tasks) return TNS_ERR_ARG;
  Su2Host h;
  const tns_status s = su2_host(prob, h);
  if (s != TNS_OK) return s;
  const int64_t nS = (int64_t)h.secL.size(), nt = (int64_t)h.tasks.size();
  *n_sectors = nS;
  *n_tasks = nt;
  if (sec_L || sec_R || psi_off || task_ptr) {
    if (!sec_L || !sec_R || !psi_off || !task_ptr || cap_sectors < nS) return TNS_ERR_WORKSPACE;
    for (int64_t i = 0; i < nS; ++i) {
      sec_L[i] = h.secL[i];
      sec_R[i] = h.secR[i];
      task_ptr[i] = h.ptr[i];
    }
    for (int64_t i = 0; i <= nS; ++i) psi_off[i] = h.psi_off[i];
    task_ptr[nS] = h.ptr[nS];
  }
  if (tasks) {
    if (cap_tasks < nt) return TNS_ERR_WORKSPACE;
    for (int64_t i = 0; i < nt; ++i) tasks[i] = h.tasks[i];
  }
  return TNS_OK;
}

extern "C" tns_status tns_su2_build(const tns_su2_problem *prob, void *ws, size_t ws_bytes, tns_su2_plan *out,
                                    hipStream_t st) {
  if (!out || !ws) return TNS_ERR_ARG;
  Su2Host h;
  tns_status s = su2_host(prob, h);
  if (s != TNS_OK) return s;
  const tns_problem G = su2_generic(prob, h);
  const size_t pb = plan_workspace(&G, h.nmax, h.maxdim, (int64_t)h.tasks.size(), false);
  if (pb == 0) return TNS_ERR_SHAPE;
  if (ws_bytes < pb) return TNS_ERR_WORKSPACE;
  memset(out, 0, sizeof(*out));
  s = build_plan(&G, h.nmax, h.maxdim, h.tasks.data(), h.ptr.data(), (int64_t)h.tasks.size(), false, ws, pb, &out->tl,
                 st);
  if (s != TNS_OK) return s;
  out->n_sectors = (int64_t)h.secL.size();
  out->psi_dim = h.psi_off.back();
  out->ntasks = out->tl.ntasks;
  out->total_flops = out->tl.total_flops;
  return TNS_OK;
}
