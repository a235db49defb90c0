// Renormalisation (blocking) of block operators, the second hot spot of the
// method (Section IV.D): after a two-site step the block grows by one site
// and every operator built on it is carried over to the new, truncated basis,
//   O~_nu = U^T ( sum_t coef_t (O_t (x) m_t) ) U,
// one output per new operator (no sum over operators, unlike sigma).
//
// On the enlarged block the product state |l, s> = C_l C_s |0> sits in
// sector Q = q(l) + q(s); inside Q the product basis lists the components
// (i, s) (old sector i, site state s) in ascending order, dim(i) states each,
// and U_Q (full(Q) x keep(Q), row-major) spans the kept states.  A term
// reaches output block (Q_out <- Q_in) of nu through every old block
// B: j <- i of O_t and every site transition s -> s' of m_t with
// Q_in = q(i) + q(s), Q_out = q(j) + q(s'):
//   O~_nu[Q_out <- Q_in] += alpha  U_Qout[rows of (j, s')]^T  B  U_Qin[rows of (i, s)]
// with alpha = coef * m[s', s] * (-1)^(parity(m) N(i)) (the site factor moves
// past the old block's creators).  That is the chained product of Eq. (2)
// with the old block B as the middle factor and transposed isometry slices
// outside, so the step runs on the forward product's grouped GEMM phases:
// the host lists these tasks (levels 1-2 of the hierarchy for this step),
// the device packs B into "input sectors" and the slices U^T into
// "operator blocks", and the output sectors are the renormalised blocks.
#include <algorithm>
#include <map>
#include <vector>

#include "kern.hpp"
#include "tns_internal.hpp"

namespace tns {

// Device tables of a renormalisation plan, after the product plan's region
// of the build workspace.
struct RnTables {
  int64_t *in_src;    // [n_in] element offset of the old block in op_vals, -1 - i: identity of old sector i
  int32_t *in_ld;     // [n_in] its leading dimension
  int64_t *g_src;     // [n_g] element offset of the slice's first row in u_vals
  int32_t *g_keep;    // [n_g] keep(Q) (rows of U^T, row stride of U)
  int64_t *out_off;   // [n_out] element offset of the output block in out_vals
  int32_t *out_ld;    // [n_out] its leading dimension
  int32_t *out_tab;   // [n_out][4] new op, Q_in, Q_out, pad
};

struct RnPlan {
  int32_t n_in, n_out, n_g, nQ;
  int64_t out_elems;  // elements of out_vals
  int64_t u_need;     // elements of u_vals the isometries span
  int64_t in0;        // first input sector (0) / first output sector (n_in)
  RnTables t;
};
static_assert(sizeof(RnPlan) <= 1024, "RnPlan fits the plan's opaque bytes");

static inline RnPlan &rn_of(tns_renorm_plan *r) { return *reinterpret_cast<RnPlan *>(r->opaque); }
static inline const RnPlan &rn_of(const tns_renorm_plan *r) { return *reinterpret_cast<const RnPlan *>(r->opaque); }

// Host-side description of the generic product the step runs as.
struct RnHost {
  // generic sector table: old sectors 0..nL-1, kept enlarged sectors nL + Q
  std::vector<int32_t> q, dim;
  std::vector<int32_t> psi_sec;  // [nS][4] (row sector, 0, 0, column sector)
  std::vector<int64_t> psi_off;
  // generic blocks: transposed isometry slices, one per (Q, component)
  std::vector<int32_t> g_rows, g_cols, g_ld, g_in, g_out, g_op;
  std::vector<int64_t> g_off, g_src;
  std::vector<int32_t> g_keep;
  int64_t g_vals = 0;
  // input sectors (old blocks, identities) and output sectors
  std::vector<int64_t> in_src;
  std::vector<int32_t> in_ld;
  std::vector<int64_t> out_off;
  std::vector<int32_t> out_ld, out_tab;
  int64_t out_elems = 0, u_need = 0;
  int32_t n_in = 0, n_out = 0, maxdim = 1;
  std::vector<tns_task> tasks;
  std::vector<int32_t> ptr;
};

static bool q_less(const int32_t *a, const int32_t *b) { return a[0] < b[0] || (a[0] == b[0] && a[1] < b[1]); }

// Validation and the task table (host).  Returns a status; on success h holds
// everything the device build needs.
static tns_status rn_host(const tns_renorm_problem *R, RnHost &h) {
  if (!R) return TNS_ERR_ARG;
  if (R->nL <= 0 || R->nOps < 0 || R->nBlk < 0 || R->nQ <= 0 || R->nNew <= 0 || R->nTerms < 0 || R->n_vals < 0 ||
      R->n_u < 0)
    return TNS_ERR_ARG;
  if (!R->qL || !R->dimL || !R->qQ || !R->keep || !R->u_off) return TNS_ERR_ARG;
  if (R->nOps > 0 && (!R->op_dN || !R->op_d2Sz)) return TNS_ERR_ARG;
  if (R->nBlk > 0 && (!R->blk_op || !R->blk_in || !R->blk_out || !R->blk_rows || !R->blk_cols || !R->blk_ld ||
                      !R->blk_off))
    return TNS_ERR_ARG;
  if (R->nTerms > 0 && (!R->term_new || !R->term_op || !R->term_mono || !R->term_coef)) return TNS_ERR_ARG;
  const int nL = R->nL, nQ = R->nQ;
  for (int i = 0; i < nL; ++i) {
    if (R->dimL[i] <= 0 || R->dimL[i] > MAX_DIM) return TNS_ERR_SHAPE;
    if (i > 0 && !q_less(R->qL + 2 * (i - 1), R->qL + 2 * i)) return TNS_ERR_QN;
  }
  for (int Q = 1; Q < nQ; ++Q)
    if (!q_less(R->qQ + 2 * (Q - 1), R->qQ + 2 * Q)) return TNS_ERR_QN;
  auto find_q = [&](const int32_t *tab, int n, int N, int S) {
    int lo = 0, hi = n - 1;
    while (lo <= hi) {
      const int mid = (lo + hi) / 2;
      const int32_t *e = tab + 2 * mid;
      if (e[0] == N && e[1] == S) return mid;
      if (e[0] < N || (e[0] == N && e[1] < S)) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
  };
  // components of every enlarged sector, ascending (i, s)
  std::vector<std::vector<std::pair<int, int>>> comps(nQ);
  std::vector<int32_t> comp_q(4 * nL), comp_c(4 * nL);
  for (int i = 0; i < nL; ++i)
    for (int s = 0; s < 4; ++s) {
      const int Q = find_q(R->qQ, nQ, R->qL[2 * i] + site_N(s), R->qL[2 * i + 1] + site_2Sz(s));
      if (Q < 0) return TNS_ERR_QN;  // qQ must list every enlarged sector
      comp_q[4 * i + s] = Q;
      comp_c[4 * i + s] = (int)comps[Q].size();
      comps[Q].push_back({i, s});
    }
  // kept dimensions and isometry extents
  std::vector<int64_t> full(nQ, 0);
  for (int Q = 0; Q < nQ; ++Q) {
    if (comps[Q].empty()) return TNS_ERR_QN;  // a listed sector no component reaches
    for (auto &c : comps[Q]) full[Q] += R->dimL[c.first];
    if (R->keep[Q] <= 0 || R->keep[Q] > full[Q] || R->keep[Q] > MAX_DIM) return TNS_ERR_SHAPE;
    if (R->u_off[Q] < 0 || R->u_off[Q] + full[Q] * R->keep[Q] > R->n_u) return TNS_ERR_SHAPE;
    h.u_need = std::max<int64_t>(h.u_need, R->u_off[Q] + full[Q] * R->keep[Q]);
  }
  // old blocks
  std::vector<std::vector<int>> op_blocks(R->nOps);
  {
    std::vector<char> seen((size_t)std::max(1, R->nOps) * nL, 0);
    for (int b = 0; b < R->nBlk; ++b) {
      const int o = R->blk_op[b], i = R->blk_in[b], j = R->blk_out[b];
      if (o < 0 || o >= R->nOps || i < 0 || i >= nL || j < 0 || j >= nL) return TNS_ERR_SHAPE;
      if (R->qL[2 * j] != R->qL[2 * i] + R->op_dN[o] || R->qL[2 * j + 1] != R->qL[2 * i + 1] + R->op_d2Sz[o])
        return TNS_ERR_QN;
      if (R->blk_rows[b] != R->dimL[j] || R->blk_cols[b] != R->dimL[i] || R->blk_ld[b] < R->blk_cols[b] ||
          R->blk_ld[b] % 8 || R->blk_off[b] % 8 || R->blk_off[b] < 0 ||
          R->blk_off[b] + (int64_t)R->blk_rows[b] * R->blk_ld[b] > R->n_vals)
        return TNS_ERR_SHAPE;
      if (seen[(size_t)o * nL + i]) return TNS_ERR_SHAPE;
      seen[(size_t)o * nL + i] = 1;
      op_blocks[o].push_back(b);
    }
  }
  // terms: a new operator's terms must share one shift
  std::vector<int> nshift(2 * R->nNew, 0), nset(R->nNew, 0);
  bool any_ident = false;
  for (int t = 0; t < R->nTerms; ++t) {
    const int nu = R->term_new[t], o = R->term_op[t], m = R->term_mono[t];
    if (nu < 0 || nu >= R->nNew || o < -1 || o >= R->nOps || m < 0 || m > 15) return TNS_ERR_ARG;
    int dN, dS;
    mono_shift(m, &dN, &dS);
    if (o >= 0) { dN += R->op_dN[o]; dS += R->op_d2Sz[o]; }
    if (nset[nu] && (nshift[2 * nu] != dN || nshift[2 * nu + 1] != dS)) return TNS_ERR_QN;
    nset[nu] = 1; nshift[2 * nu] = dN; nshift[2 * nu + 1] = dS;
    any_ident |= o < 0;
  }
  // generic sector table and the transposed isometry slices
  h.q.assign(2 * (nL + nQ), 0);
  h.dim.resize(nL + nQ);
  for (int i = 0; i < nL + nQ; ++i) { h.q[2 * i] = i; h.q[2 * i + 1] = 0; }  // only the dimensions matter
  for (int i = 0; i < nL; ++i) h.dim[i] = R->dimL[i];
  for (int Q = 0; Q < nQ; ++Q) h.dim[nL + Q] = R->keep[Q];
  for (int i = 0; i < nL + nQ; ++i) h.maxdim = std::max(h.maxdim, h.dim[i]);
  std::vector<int32_t> gid(4 * nL);
  for (int Q = 0; Q < nQ; ++Q) {
    int64_t r0 = 0;
    for (auto &c : comps[Q]) {
      const int i = c.first, d = R->dimL[i];
      gid[4 * i + c.second] = (int)h.g_rows.size();
      h.g_rows.push_back(R->keep[Q]);
      h.g_cols.push_back(d);
      h.g_ld.push_back(ld8(d));
      h.g_in.push_back(i);
      h.g_out.push_back(nL + Q);
      h.g_op.push_back(0);
      h.g_off.push_back(h.g_vals);
      h.g_vals += (int64_t)R->keep[Q] * ld8(d);
      h.g_src.push_back(R->u_off[Q] + r0 * R->keep[Q]);
      h.g_keep.push_back(R->keep[Q]);
      r0 += d;
    }
  }
  // input sectors: the old blocks, then (if any term needs it) the identity of every old sector
  auto add_sector = [&](int rs, int cs) {
    h.psi_sec.push_back(rs); h.psi_sec.push_back(0); h.psi_sec.push_back(0); h.psi_sec.push_back(cs);
    const int64_t o = h.psi_off.empty() ? 0 : h.psi_off.back();
    if (h.psi_off.empty()) h.psi_off.push_back(0);
    h.psi_off.push_back(o + (int64_t)h.dim[rs] * h.dim[cs]);
  };
  for (int b = 0; b < R->nBlk; ++b) {
    add_sector(R->blk_out[b], R->blk_in[b]);
    h.in_src.push_back(R->blk_off[b]);
    h.in_ld.push_back(R->blk_ld[b]);
  }
  const int id0 = R->nBlk;
  if (any_ident)
    for (int i = 0; i < nL; ++i) {
      add_sector(i, i);
      h.in_src.push_back(-1 - (int64_t)i);
      h.in_ld.push_back(0);
    }
  h.n_in = (int32_t)h.in_src.size();
  // tasks, in (term, block, site state) order; output sector per (new op, Q_in)
  struct Raw { int32_t nu, Qin, Qout, in, lblk, rblk; double alpha; };
  std::vector<Raw> raw;
  for (int t = 0; t < R->nTerms; ++t) {
    const int nu = R->term_new[t], o = R->term_op[t], m = R->term_mono[t];
    const double coef = R->term_coef[t];
    const int pm = mono_parity(m);
    const int nb = o >= 0 ? (int)op_blocks[o].size() : nL;
    for (int k = 0; k < nb; ++k) {
      const int b = o >= 0 ? op_blocks[o][k] : -1;
      const int i = o >= 0 ? R->blk_in[b] : k, j = o >= 0 ? R->blk_out[b] : k;
      for (int s = 0; s < 4; ++s) {
        int val = 0;
        const int s2 = mono_apply(m, s, &val);
        if (s2 < 0) continue;
        const double sgn = (pm * R->qL[2 * i]) % 2 ? -1.0 : 1.0;
        Raw x;
        x.nu = nu;
        x.Qin = comp_q[4 * i + s];
        x.Qout = comp_q[4 * j + s2];
        x.in = o >= 0 ? b : id0 + i;
        x.lblk = gid[4 * j + s2];
        x.rblk = gid[4 * i + s];
        x.alpha = ((coef * (double)val) * sgn);
        raw.push_back(x);
      }
    }
  }
  std::map<std::pair<int, int>, int> out_id;  // (new op, Q_in) -> output index, ascending
  for (auto &x : raw) out_id.emplace(std::make_pair(x.nu, x.Qin), 0);
  int k = 0;
  for (auto &e : out_id) e.second = k++;
  h.n_out = k;
  h.out_tab.resize(4 * (size_t)std::max(1, k));
  h.out_off.resize(std::max(1, k));
  h.out_ld.resize(std::max(1, k));
  for (auto &e : out_id) {
    const int nu = e.first.first, Qin = e.first.second, id = e.second;
    // output block Q_out = Q_in + shift(nu)
    const int Qout = find_q(R->qQ, nQ, R->qQ[2 * Qin] + nshift[2 * nu], R->qQ[2 * Qin + 1] + nshift[2 * nu + 1]);
    h.out_tab[4 * id] = nu; h.out_tab[4 * id + 1] = Qin; h.out_tab[4 * id + 2] = Qout; h.out_tab[4 * id + 3] = 0;
  }
  for (int id = 0; id < k; ++id) {
    const int Qin = h.out_tab[4 * id + 1], Qout = h.out_tab[4 * id + 2];
    add_sector(nL + Qout, nL + Qin);
    h.out_off[id] = h.out_elems;
    h.out_ld[id] = ld8(R->keep[Qin]);
    h.out_elems += (int64_t)R->keep[Qout] * h.out_ld[id];
  }
  if (h.psi_off.empty()) h.psi_off.push_back(0);
  const int nS = h.n_in + h.n_out;
  h.ptr.assign(nS + 1, 0);
  std::vector<tns_task> tk(raw.size());
  for (size_t a = 0; a < raw.size(); ++a) {
    const Raw &x = raw[a];
    tns_task t;
    t.out = h.n_in + out_id[{x.nu, x.Qin}];
    t.in = x.in;
    t.term = x.nu;
    t.lblk = x.lblk;
    t.rblk = x.rblk;
    t.alpha = x.alpha;
    // q, m: output / input row dimensions; r, n: output / input column dimensions
    const int64_t q = R->keep[x.Qout], m = h.dim[h.psi_sec[4 * t.in]];
    const int64_t n = h.dim[h.psi_sec[4 * t.in + 3]], r = R->keep[x.Qin];
    const int64_t c0 = 2 * q * n * (m + r), c1 = 2 * m * r * (n + q);
    if (c1 < c0) { t.order = 1; t.cost = c1; } else { t.order = 0; t.cost = c0; }
    tk[a] = t;
    h.ptr[t.out + 1] += 1;
  }
  for (int s = 0; s < nS; ++s) h.ptr[s + 1] += h.ptr[s];
  std::vector<int32_t> fill(h.ptr.begin(), h.ptr.end() - 1);
  h.tasks.resize(tk.size());
  for (auto &t : tk) h.tasks[fill[t.out]++] = t;  // stable by output sector
  return TNS_OK;
}

// The generic problem (host arrays of h) the product plan is built from.
static tns_problem rn_generic(const RnHost &h, const std::vector<int32_t> &zero) {
  tns_problem P;
  memset(&P, 0, sizeof(P));
  const int ns = (int)h.dim.size();
  P.nL = P.nR = ns;
  P.nS = (int)(h.psi_off.size() - 1);
  P.nOps = 0;
  P.nBlk = (int)h.g_rows.size();
  P.nTerms = 0;
  P.n_vals = std::max<int64_t>(h.g_vals, 8);
  P.qL = P.qR = h.q.data();
  P.dimL = P.dimR = h.dim.data();
  P.psi_sec = h.psi_sec.empty() ? zero.data() : h.psi_sec.data();
  P.psi_off = h.psi_off.data();
  P.blk_op = h.g_op.data(); P.blk_in = h.g_in.data(); P.blk_out = h.g_out.data();
  P.blk_rows = h.g_rows.data(); P.blk_cols = h.g_cols.data(); P.blk_ld = h.g_ld.data();
  P.blk_off = h.g_off.data();
  return P;
}

static size_t rn_tables_bytes(const RnHost &h) {
  const size_t ni = std::max(1, h.n_in), ng = std::max<size_t>(1, h.g_rows.size()), no = std::max(1, h.n_out);
  return align_up(ni * 8, 256) + align_up(ni * 4, 256) + align_up(ng * 8, 256) + align_up(ng * 4, 256) +
         align_up(no * 8, 256) + align_up(no * 4, 256) + align_up(no * 16, 256) + 256;
}

// --- device kernels ------------------------------------------------------------------
// Input sectors <- old blocks (rows x cols from op_vals with their leading
// dimension) or identities, in the precision's vector type.
template <class T>
__global__ void k_rn_pack_in(const double *__restrict__ ops, const int64_t *__restrict__ src,
                             const int32_t *__restrict__ ld, const int64_t *__restrict__ psi_off,
                             const int32_t *__restrict__ psi_sec, const int32_t *__restrict__ dim, int n_in,
                             T *__restrict__ psi) {
  for (int s = blockIdx.x; s < n_in; s += gridDim.x) {
    const int rows = dim[psi_sec[4 * s]], cols = dim[psi_sec[4 * s + 3]];
    const int64_t o = psi_off[s], sv = src[s];
    const int l = ld[s];
    for (int64_t e = threadIdx.x; e < (int64_t)rows * cols; e += blockDim.x) {
      const int r = (int)(e / cols), c = (int)(e % cols);
      psi[o + e] = sv >= 0 ? (T)ops[sv + (int64_t)r * l + c] : (T)(r == c ? 1.0 : 0.0);
    }
  }
}

// Operator blocks <- transposed isometry slices: block g (keep x ld8(d)) holds
// U_Q[r0 + r][k] at (k, r), zeros in the padding columns; precision format
// (BF16X3 interleaved).
template <int P>
__global__ void k_rn_pack_u(const double *__restrict__ u, const int64_t *__restrict__ src,
                            const int32_t *__restrict__ keep, const int32_t *__restrict__ cols,
                            const int64_t *__restrict__ off, int ng, void *out) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int g = blockIdx.x; g < ng; g += gridDim.x) {
    const int K = keep[g], d = cols[g], ldo = ld8(d);
    const double *S = u + src[g];  // S[r * K + k]
    for (int r0 = 0; r0 < ldo; r0 += 32)
      for (int k0 = 0; k0 < K; k0 += 32) {
        for (int i = ty; i < 32; i += 8) {
          const int r = r0 + i, k = k0 + tx;
          tile[i][tx] = (r < d && k < K) ? S[(int64_t)r * K + k] : 0.0;
        }
        __syncthreads();
        for (int i = ty; i < 32; i += 8) {
          const int k = k0 + i, r = r0 + tx;
          if (k < K && r < ldo) {
            const int64_t e = off[g] + (int64_t)k * ldo + r;
            const double v = tile[tx][i];
            if constexpr (P == TNS_F64) {
              reinterpret_cast<double *>(out)[e] = v;
            } else if constexpr (P == TNS_F32) {
              reinterpret_cast<float *>(out)[e] = (float)v;
            } else {
              const float x = (float)v;
              const uint16_t hh = f32_to_bf16_rne(x);
              uint16_t *q = reinterpret_cast<uint16_t *>(out) + bfx_hi(e);
              q[0] = hh;
              q[8] = f32_to_bf16_rne(x - bf16_to_f32(hh));
            }
          }
        }
        __syncthreads();
      }
  }
}

// Output blocks <- output sectors of sigma (rows x cols) with leading
// dimension ld8(cols), padding zero.
template <class T>
__global__ void k_rn_unpack(const T *__restrict__ sigma, const int64_t *__restrict__ psi_off,
                            const int32_t *__restrict__ psi_sec, const int32_t *__restrict__ dim, int n_in,
                            int n_out, const int64_t *__restrict__ out_off, const int32_t *__restrict__ out_ld,
                            T *__restrict__ out) {
  for (int k = blockIdx.x; k < n_out; k += gridDim.x) {
    const int s = n_in + k;
    const int rows = dim[psi_sec[4 * s]], cols = dim[psi_sec[4 * s + 3]], l = out_ld[k];
    const int64_t o = psi_off[s], d = out_off[k];
    for (int64_t e = threadIdx.x; e < (int64_t)rows * l; e += blockDim.x) {
      const int r = (int)(e / l), c = (int)(e % l);
      out[d + e] = c < cols ? sigma[o + (int64_t)r * cols + c] : T(0);
    }
  }
}

template <class T>
static T *carve_dev(char *&c, size_t n) {
  T *p = reinterpret_cast<T *>(c);
  c += align_up(n * sizeof(T), 256);
  return p;
}

static size_t elem_size(tns_prec p) { return p == TNS_F64 ? 8 : 4; }

// Apply workspace: [psi | sigma | operator blocks (U^T slices) | forward product]
static size_t rn_apply_ws(const tns_renorm_plan *r, tns_prec prec) {
  const Plan &p = plan_of(&r->tl);
  const size_t es = elem_size(prec);
  const size_t gb = prec == TNS_BF16X3 ? (size_t)((p.n_vals + 7) & ~int64_t(7)) * 4 : (size_t)p.n_vals * es;
  return 2 * align_up((size_t)std::max<int64_t>(p.psi_dim, 1) * es, 256) + align_up(gb + 64, 256) +
         fwd_workspace(p, prec);
}

template <int P>
static tns_status rn_apply(const tns_renorm_plan *r, const double *ops, const double *u, void *out, char *w,
                           hipStream_t st) {
  typedef typename std::conditional<P == TNS_F64, double, float>::type T;
  const Plan &p = plan_of(&r->tl);
  const RnPlan &rp = rn_of(r);
  const size_t es = sizeof(T);
  T *psi = reinterpret_cast<T *>(w);
  w += align_up((size_t)std::max<int64_t>(p.psi_dim, 1) * es, 256);
  T *sigma = reinterpret_cast<T *>(w);
  w += align_up((size_t)std::max<int64_t>(p.psi_dim, 1) * es, 256);
  void *gvals = w;
  const size_t gb = P == TNS_BF16X3 ? (size_t)((p.n_vals + 7) & ~int64_t(7)) * 4 : (size_t)p.n_vals * es;
  w += align_up(gb + 64, 256);
  if (rp.n_in > 0)
    hipLaunchKernelGGL(k_rn_pack_in<T>, dim3(std::min(rp.n_in, 4096)), dim3(256), 0, st, ops, rp.t.in_src,
                       rp.t.in_ld, p.psi_off, p.psi_sec, p.dimL, rp.n_in, psi);
  if (rp.n_g > 0)
    hipLaunchKernelGGL(k_rn_pack_u<P>, dim3(std::min(rp.n_g, 4096)), dim3(256), 0, st, u, rp.t.g_src, rp.t.g_keep,
                       p.blk_cols, p.blk_off, rp.n_g, gvals);
  TNS_HIP(hipGetLastError());
  hipEvent_t ev[3];
  const bool timed = take_profile_events(ev);
  const tns_status s = fwd_apply(p, (tns_prec)P, gvals, psi, sigma, 0.0, w, fwd_workspace(p, (tns_prec)P), st,
                                 timed ? ev : nullptr);
  if (s != TNS_OK) return s;
  if (rp.n_out > 0)
    hipLaunchKernelGGL(k_rn_unpack<T>, dim3(std::min(rp.n_out, 4096)), dim3(256), 0, st, sigma, p.psi_off,
                       p.psi_sec, p.dimL, rp.n_in, rp.n_out, rp.t.out_off, rp.t.out_ld, (T *)out);
  return hipGetLastError() == hipSuccess ? TNS_OK : TNS_ERR_HIP;
}

}  // namespace tns

using namespace tns;

extern "C" size_t tns_renorm_workspace_bytes(const tns_renorm_problem *R) {
  RnHost h;
  if (rn_host(R, h) != TNS_OK) return 0;
  const std::vector<int32_t> zero(4, 0);
  const tns_problem P = rn_generic(h, zero);
  const size_t b = plan_workspace(&P, (int32_t)h.dim.size(), h.maxdim, (int64_t)h.tasks.size(), false);
  return b ? align_up(b, 256) + rn_tables_bytes(h) : 0;
}

extern "C" tns_status tns_renorm_build(const tns_renorm_problem *R, void *ws, size_t ws_bytes, tns_renorm_plan *out,
                                       hipStream_t st) {
  if (!out || !ws) return TNS_ERR_ARG;
  RnHost h;
  tns_status s = rn_host(R, h);
  if (s != TNS_OK) return s;
  const std::vector<int32_t> zero(4, 0);
  const tns_problem P = rn_generic(h, zero);
  const size_t pb = plan_workspace(&P, (int32_t)h.dim.size(), h.maxdim, (int64_t)h.tasks.size(), false);
  if (pb == 0) return TNS_ERR_SHAPE;
  const size_t need = align_up(pb, 256) + rn_tables_bytes(h);
  if (ws_bytes < need) return TNS_ERR_WORKSPACE;
  memset(out, 0, sizeof(*out));
  s = build_plan(&P, (int32_t)h.dim.size(), h.maxdim, h.tasks.data(), h.ptr.data(), (int64_t)h.tasks.size(), false,
                 ws, pb, &out->tl, st);
  if (s != TNS_OK) return s;
  // the tasks read only the input sectors and write only the output ones:
  // pad the former, sum the partial slots of the latter
  Plan &gp = plan_of(&out->tl);
  gp.pad_ns = h.n_in;
  gp.epi_e0 = h.psi_off[h.n_in];
  RnPlan &rp = rn_of(out);
  rp.n_in = h.n_in; rp.n_out = h.n_out; rp.n_g = (int32_t)h.g_rows.size(); rp.nQ = R->nQ;
  rp.out_elems = h.out_elems; rp.u_need = h.u_need; rp.in0 = 0;
  char *c = reinterpret_cast<char *>(ws) + align_up(pb, 256);
  rp.t.in_src = carve_dev<int64_t>(c, std::max(1, h.n_in));
  rp.t.in_ld = carve_dev<int32_t>(c, std::max(1, h.n_in));
  rp.t.g_src = carve_dev<int64_t>(c, std::max<size_t>(1, h.g_rows.size()));
  rp.t.g_keep = carve_dev<int32_t>(c, std::max<size_t>(1, h.g_rows.size()));
  rp.t.out_off = carve_dev<int64_t>(c, std::max(1, h.n_out));
  rp.t.out_ld = carve_dev<int32_t>(c, std::max(1, h.n_out));
  rp.t.out_tab = carve_dev<int32_t>(c, 4 * (size_t)std::max(1, h.n_out));
  auto put = [&](void *d, const void *src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  TNS_HIP(put(rp.t.in_src, h.in_src.data(), h.in_src.size() * 8));
  TNS_HIP(put(rp.t.in_ld, h.in_ld.data(), h.in_ld.size() * 4));
  TNS_HIP(put(rp.t.g_src, h.g_src.data(), h.g_src.size() * 8));
  TNS_HIP(put(rp.t.g_keep, h.g_keep.data(), h.g_keep.size() * 4));
  TNS_HIP(put(rp.t.out_off, h.out_off.data(), (size_t)h.n_out * 8));
  TNS_HIP(put(rp.t.out_ld, h.out_ld.data(), (size_t)h.n_out * 4));
  TNS_HIP(put(rp.t.out_tab, h.out_tab.data(), (size_t)h.n_out * 16));
  TNS_HIP(hipStreamSynchronize(st));  // the host tables above go out of scope
  out->ntasks = out->tl.ntasks;
  out->n_out_blk = h.n_out;
  out->out_elems = h.out_elems;
  out->total_flops = out->tl.total_flops;
  return TNS_OK;
}

extern "C" tns_status tns_renorm_out_table(const tns_renorm_plan *r, int32_t *blk_new, int32_t *blk_in,
                                           int32_t *blk_out, int32_t *rows, int32_t *cols, int32_t *ld,
                                           int64_t *off) {
  if (!r || !blk_new || !blk_in || !blk_out || !rows || !cols || !ld || !off) return TNS_ERR_ARG;
  const RnPlan &rp = rn_of(r);
  const Plan &p = plan_of(&r->tl);
  const int n = rp.n_out;
  if (n == 0) return TNS_OK;
  std::vector<int32_t> tab(4 * (size_t)n), sec(4 * (size_t)p.nS), dim(p.nL);
  TNS_HIP(hipMemcpy(tab.data(), rp.t.out_tab, tab.size() * 4, hipMemcpyDeviceToHost));
  TNS_HIP(hipMemcpy(ld, rp.t.out_ld, (size_t)n * 4, hipMemcpyDeviceToHost));
  TNS_HIP(hipMemcpy(off, rp.t.out_off, (size_t)n * 8, hipMemcpyDeviceToHost));
  TNS_HIP(hipMemcpy(sec.data(), p.psi_sec, sec.size() * 4, hipMemcpyDeviceToHost));
  TNS_HIP(hipMemcpy(dim.data(), p.dimL, dim.size() * 4, hipMemcpyDeviceToHost));
  for (int k = 0; k < n; ++k) {
    blk_new[k] = tab[4 * k];
    blk_in[k] = tab[4 * k + 1];
    blk_out[k] = tab[4 * k + 2];
    const int s = rp.n_in + k;
    rows[k] = dim[sec[4 * s]];
    cols[k] = dim[sec[4 * s + 3]];
  }
  return TNS_OK;
}

extern "C" size_t tns_renorm_apply_workspace_bytes(const tns_renorm_plan *r, tns_prec prec) {
  if (!r || (prec != TNS_F64 && prec != TNS_F32 && prec != TNS_BF16X3)) return 0;
  return rn_apply_ws(r, prec);
}

extern "C" tns_status tns_renormalize(const tns_renorm_plan *r, tns_prec prec, const double *op_vals,
                                      const double *u_vals, void *out_vals, void *ws, size_t ws_bytes,
                                      hipStream_t st) {
  if (!r || !op_vals || !u_vals || !out_vals || !ws) return TNS_ERR_ARG;
  if (prec != TNS_F64 && prec != TNS_F32 && prec != TNS_BF16X3) return TNS_ERR_ARG;
  if (ws_bytes < rn_apply_ws(r, prec)) return TNS_ERR_WORKSPACE;
  char *w = reinterpret_cast<char *>(ws);
  if (prec == TNS_F64) return rn_apply<TNS_F64>(r, op_vals, u_vals, out_vals, w, st);
  if (prec == TNS_F32) return rn_apply<TNS_F32>(r, op_vals, u_vals, out_vals, w, st);
  return rn_apply<TNS_BF16X3>(r, op_vals, u_vals, out_vals, w, st);
}
