// Levels 1-2 of the four-level hierarchy (Section III.A.1) on the device:
// sector lookups, the task table of Eq. (2) in canonical order, and the work
// schedule of the persistent H_eff kernel.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "tns_internal.hpp"

namespace tns {

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Exclusive scan of n int64 values into out[0..n] (out[n] = total); one
// workgroup of 1024 threads walks the array in tiles.
__global__ __launch_bounds__(1024) void k_scan_i64(const int64_t *__restrict__ in, int64_t *__restrict__ out,
                                                   int64_t n) {
  __shared__ int64_t sh[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024) {
    int64_t i = base + threadIdx.x;
    int64_t v = (i < n) ? in[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int64_t t = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < n) out[i] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

tns_status scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, in, out, n);
  return hipGetLastError() == hipSuccess ? TNS_OK : TNS_ERR_HIP;
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// lookups
// ---------------------------------------------------------------------------

__global__ void k_psi_index(Plan p) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.nS) return;
  const int32_t *e = p.psi_sec + 4 * s;
  p.psi_index[(e[0] * 4 + e[1]) * 4 + e[2]] = s;
}

__global__ void k_blk_of_out(Plan p) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= p.nBlk) return;
  p.blk_of_out[(int64_t)p.blk_op[b] * p.nmax + p.blk_out[b]] = b;
}

// ---------------------------------------------------------------------------
// task table: one wave per output sector, lanes over terms.  For an output
// sector and a term there is at most one input sector (each operator block
// and each monomial maps inputs to outputs injectively), so gathering per
// output sector in term order yields the canonical order directly.
// ---------------------------------------------------------------------------

template <bool FILL>
__global__ __launch_bounds__(256) void k_tasks(Plan p) {
  const int lane = threadIdx.x & 63;
  const int so = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (so >= p.nS) return;
  const int jL = p.psi_sec[4 * so + 0], ta = p.psi_sec[4 * so + 1];
  const int tb = p.psi_sec[4 * so + 2], jR = p.psi_sec[4 * so + 3];
  int64_t base = FILL ? p.out_ptr[so] : 0;
  int count = 0;
  for (int k0 = 0; k0 < p.nTerms; k0 += 64) {
    const int k = k0 + lane;
    bool ok = false;
    int iL = 0, iR = 0, sa = 0, sb = 0, lb = -1, rb = -1, va = 0, vb = 0, si = -1;
    int oL = -1, oR = -1, ma = 0, mb = 0;
    if (k < p.nTerms) {
      oL = p.term_L[k]; oR = p.term_R[k]; ma = p.term_ma[k]; mb = p.term_mb[k];
      ok = true;
      if (oL >= 0) {
        lb = p.blk_of_out[(int64_t)oL * p.nmax + jL];
        if (lb < 0) ok = false; else iL = p.blk_in[lb];
      } else {
        iL = jL;
      }
      if (ok) {
        sa = -1;
        for (int s = 0; s < 4; ++s) { int v; if (mono_apply(ma, s, &v) == ta) { sa = s; va = v; } }
        sb = -1;
        for (int s = 0; s < 4; ++s) { int v; if (mono_apply(mb, s, &v) == tb) { sb = s; vb = v; } }
        if (sa < 0 || sb < 0) ok = false;
      }
      if (ok) {
        if (oR >= 0) {
          rb = p.blk_of_out[(int64_t)oR * p.nmax + jR];
          if (rb < 0) ok = false; else iR = p.blk_in[rb];
        } else {
          iR = jR;
        }
      }
      if (ok) {
        si = p.psi_index[(iL * 4 + sa) * 4 + sb];
        if (si < 0 || p.psi_sec[4 * si + 3] != iR) ok = false;
      }
    }
    const uint64_t bal = __ballot(ok);
    if (FILL && ok) {
      const int rank = __popcll(bal & ((1ull << lane) - 1ull));
      tns_task t;
      t.out = so; t.in = si; t.term = k; t.lblk = lb; t.rblk = rb;
      const int Nl = p.qL[2 * iL], Na = site_N(sa), Nb = site_N(sb);
      const int pa = mono_parity(ma), pb = mono_parity(mb);
      const int pR = (oR >= 0) ? (abs(p.op_dN[oR]) & 1) : 0;
      const int e = pa * Nl + pb * (Nl + Na) + pR * (Nl + Na + Nb);
      const double sgn = (e & 1) ? -1.0 : 1.0;
      const double c = p.term_coef[k];
      t.alpha = ((c * (double)va) * (double)vb) * sgn;
      const int64_t q = p.dimL[jL], m = p.dimL[iL], n = p.dimR[iR], r = p.dimR[jR];
      if (oL >= 0 && oR >= 0) {
        const int64_t c0 = 2 * q * n * (m + r), c1 = 2 * m * r * (n + q);
        if (c1 < c0) { t.order = 1; t.cost = c1; } else { t.order = 0; t.cost = c0; }
      } else if (oL >= 0) {
        t.order = 0; t.cost = 2 * q * m * n;
      } else if (oR >= 0) {
        t.order = 0; t.cost = 2 * m * n * r;
      } else {
        t.order = 0; t.cost = 2 * m * n;
      }
      p.tasks[base + count + rank] = t;
    }
    count += __popcll(bal);
  }
  if (!FILL && lane == 0) p.scan_tmp[so] = count;
}

// Forward groups: per output sector, class-0 tasks then class-1 tasks
// (canonical order kept inside each class).  Group 2s + c holds class c of
// sector s; its output is sigma_s (c = 0) or sigma_s^T (c = 1).
__global__ __launch_bounds__(256) void k_fwd_groups(Plan p, Sched S) {
  const int lane = threadIdx.x & 63;
  const int so = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (so >= p.nS) return;
  const int t0 = p.out_ptr[so], t1 = p.out_ptr[so + 1];
  int n0 = 0;
  for (int b = t0; b < t1; b += 64) {
    const int t = b + lane;
    const int ord = (t < t1) ? p.tasks[t].order : -1;
    const uint64_t bal = __ballot(ord == 0);
    if (ord == 0) S.idx[t0 + n0 + __popcll(bal & ((1ull << lane) - 1ull))] = t;
    n0 += __popcll(bal);
  }
  int n1 = 0;
  for (int b = t0; b < t1; b += 64) {
    const int t = b + lane;
    const int ord = (t < t1) ? p.tasks[t].order : -1;
    const uint64_t bal = __ballot(ord == 1);
    if (ord == 1) S.idx[t0 + n0 + n1 + __popcll(bal & ((1ull << lane) - 1ull))] = t;
    n1 += __popcll(bal);
  }
  if (lane == 0) {
    const int q = p.dimL[p.psi_sec[4 * so]], r = p.dimR[p.psi_sec[4 * so + 3]];
    S.grp_begin[2 * so] = t0;
    S.grp_n[2 * so] = n0;
    S.grp_rows[2 * so] = q;
    S.grp_cols[2 * so] = r;
    S.grp_out[2 * so] = so;
    S.grp_mode[2 * so] = M_FWD0;
    S.grp_begin[2 * so + 1] = t0 + n0;
    S.grp_n[2 * so + 1] = n1;
    S.grp_rows[2 * so + 1] = r;
    S.grp_cols[2 * so + 1] = q;
    S.grp_out[2 * so + 1] = so;
    S.grp_mode[2 * so + 1] = M_FWD1;
  }
}

// Flops of one task evaluated in a mode (used for load balance).
__device__ inline int64_t mode_cost(const Plan &p, const tns_task &t, int mode) {
  if (mode <= M_FWD1) return t.cost;
  const int64_t q = p.dimL[p.psi_sec[4 * t.out]], r = p.dimR[p.psi_sec[4 * t.out + 3]];
  const int64_t m = p.dimL[p.psi_sec[4 * t.in]], n = p.dimR[p.psi_sec[4 * t.in + 3]];
  if (mode == M_DL) return 2 * q * r * n + 2 * q * n * m;
  if (mode == M_DR) return 2 * r * q * m + 2 * r * m * n;
  return 0;  // d psi groups carry no tasks
}

// Summed cost per group (one wave per group) and the schedule total.
__global__ __launch_bounds__(256) void k_group_cost(Plan p, Sched S) {
  const int lane = threadIdx.x & 63;
  const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (g >= S.ngroups) return;
  const int b = S.grp_begin[g], n = S.grp_n[g], mode = S.grp_mode[g];
  int64_t c = 0;
  for (int i = lane; i < n; i += 64) c += mode_cost(p, p.tasks[S.idx[b + i]], mode);
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if (lane == 0) {
    S.grp_cost[g] = c;
    atomicAdd((unsigned long long *)&S.scalars[0], (unsigned long long)c);
  }
}

// Tile extents of a group with a rows x cols output.
__device__ inline void tile_dims(const Sched &S, int rows, int cols, int *tr, int *tc) {
  if (S.tiles) {
    *tr = tile_ext_r(S.tiles, rows);
    *tc = tile_ext_c(S.tiles, cols);
  } else {
    *tr = S.tile_r;
    *tc = S.tile_c > 0 ? S.tile_c : cols;
  }
}

// Tiles (work items) of one chunk of a group with a rows x cols output.
__device__ inline int n_tiles(const Sched &S, int rows, int cols) {
  int tr, tc;
  tile_dims(S, rows, cols, &tr, &tc);
  return ((rows + tr - 1) / tr) * ((cols + tc - 1) / tc);
}

// Chunk cap unit: the number of largest tiles of the output, so that chunking
// does not depend on the tile table (partial slots stay the same).
__device__ inline int cap_tiles(const Sched &S, int rows, int cols) {
  if (!S.tiles) return n_tiles(S, rows, cols);
  return ((rows + GM - 1) / GM) * ((cols + GN - 1) / GN);
}

// Greedy task chunks per group: a chunk closes before the task that would
// push it over cap = target_item_cost * tiles (each chunk is then cut into
// output tiles, so items cost about target_item_cost each).
template <bool FILL>
__global__ void k_chunks(Plan p, Sched S) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= S.ngroups) return;
  const int n = S.grp_n[g];
  int nc = 0;
  if (n > 0) {
    // ITEMS_PER_CU items per CU on large schedules, but chunks no smaller
    // than ITEM_MIN_FLOP unless that leaves fewer than ITEMS_MIN_PER_CU per CU
    const int64_t total = S.scalars[0];
    const int64_t fine = total / ((int64_t)ITEMS_PER_CU * p.n_cu);
    const int64_t coarse = total / ((int64_t)ITEMS_MIN_PER_CU * p.n_cu);
    const int64_t floor_ = coarse < ITEM_MIN_FLOP ? coarse : ITEM_MIN_FLOP;
    const int64_t target = (fine > floor_ ? fine : floor_) + 1;
    const int64_t cap = target * cap_tiles(S, S.grp_rows[g], S.grp_cols[g]);
    const int b = S.grp_begin[g], mode = S.grp_mode[g];
    int64_t cur = 0;
    int start = b;
    bool idy = false;
    const int64_t cb = FILL ? S.grp_chunk_base[g] : 0;
    for (int i = b; i < b + n; ++i) {
      const int64_t c = mode_cost(p, p.tasks[S.idx[i]], mode);
      if (i > start && cur + c > cap) {
        if (FILL) { Chunk ch{g, start, i, 0, cur, 0, idy ? CHUNK_IDENT_Y : 0}; S.chunks[cb + nc] = ch; }
        ++nc;
        start = i;
        cur = 0;
        idy = false;
      }
      cur += c;
      if (FILL && mode <= M_FWD1) idy |= ident_y(p.tasks[S.idx[i]]);
    }
    if (FILL) { Chunk ch{g, start, b + n, 0, cur, 0, idy ? CHUNK_IDENT_Y : 0}; S.chunks[cb + nc] = ch; }
    ++nc;
  }
  if (!FILL) S.scratch[g] = nc;
}

// Per chunk: partial-slot size (rows * cols of its output) and item count.
__global__ void k_chunk_sizes(Sched S, int64_t *slot_sz, int64_t *item_n) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= S.chunks_cap) return;
  const int64_t nch = S.grp_chunk_base[S.ngroups];
  if (c >= nch) { slot_sz[c] = 0; item_n[c] = 0; return; }
  const int g = S.chunks[c].grp;
  slot_sz[c] = (int64_t)S.grp_rows[g] * S.grp_cols[g];
  item_n[c] = n_tiles(S, S.grp_rows[g], S.grp_cols[g]);
}

__global__ void k_items(Sched S) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nch = S.grp_chunk_base[S.ngroups];
  if (c >= nch) return;
  const Chunk ch = S.chunks[c];
  const int rows = S.grp_rows[ch.grp], cols = S.grp_cols[ch.grp];
  int tr, tc;
  tile_dims(S, rows, cols, &tr, &tc);
  const int ncol = (cols + tc - 1) / tc;
  const int nt = n_tiles(S, rows, cols);
  const int64_t ib = S.chunk_item_base[c];
  for (int k = 0; k < nt; ++k) {
    Item it;
    it.grp = ch.grp;
    it.p0 = (k / ncol) * tr;
    it.np = min(tr, rows - it.p0);
    it.c0 = (k % ncol) * tc;
    it.nc = min(tc, cols - it.c0);
    it.mode = S.grp_mode[ch.grp] |
              (S.tiles ? ((tail_ext(it.np, tr) / 32) << 8) | ((tail_ext(it.nc, tc) / 32) << 16) : 0) |
              ((ch.flags & CHUNK_IDENT_Y) ? ITEM_IDENT_Y : 0);
    it.tb = ch.tb;
    it.te = ch.te;
    it.slot = (int32_t)c;
    it.out = S.grp_out[ch.grp];
    it.cost = ch.cost * ((int64_t)it.np * it.nc) / ((int64_t)rows * cols);
    // the host compares the item total with items_cap after the build
    if (ib + k < S.items_cap) S.items_unsorted[ib + k] = it;
  }
}

// Chunks by descending cost (ascending key; padding last).
__global__ void k_chunk_keys(Sched S) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= S.chunks_cap) return;
  const int64_t nch = S.grp_chunk_base[S.ngroups];
  S.keys_in[c] = (c < nch) ? (~(uint64_t)S.chunks[c].cost - 1ull) : ~0ull;
  S.vals_in[c] = (int32_t)c;
}

// XCD of each chunk: boustrophedon over the cost-sorted chunks (ranks 0..nq-1
// to queues 0..nq-1, the next nq ranks back from nq-1, ...), which keeps the
// queue totals close while all row panels of a chunk share one L2.
__global__ void k_chunk_xcd(Sched S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nch = S.grp_chunk_base[S.ngroups];
  if (i >= nch) return;
  const int64_t round = i / S.nq, pos = i % S.nq;
  S.chunks[S.vals_out[i]].xcd = (int32_t)((round & 1) ? S.nq - 1 - pos : pos);
  S.chunks[S.vals_out[i]].rank = (int32_t)i;
}

// Item order: by queue, then by chunk in descending chunk cost, the tiles of
// a chunk adjacent (row-major), so that the workgroups of one XCD that run a
// chunk's tiles together share its operand panels in L2; padding sorts last.
__global__ void k_sort_keys(Sched S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.items_cap) return;
  const int64_t nit = S.chunk_item_base[S.grp_chunk_base[S.ngroups]];
  constexpr uint64_t LM = (1ull << 28) - 1;
  uint64_t key = ~0ull;
  if (i < nit) {
    const Item it = S.items_unsorted[i];
    const Chunk &ch = S.chunks[it.slot];
    key = ((uint64_t)ch.xcd << 56) | (((uint64_t)ch.rank & LM) << 28) |
          ((uint64_t)(i - S.chunk_item_base[it.slot]) & LM);
  }
  S.keys_in[i] = key;
  S.vals_in[i] = (int32_t)i;
}

// Queue bounds from the sorted keys: qbase[q] = first item of queue q.
__global__ void k_queue_bounds(Sched S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nit = S.chunk_item_base[S.grp_chunk_base[S.ngroups]];
  if (i > nit) return;
  const int prev = i == 0 ? -1 : (int)(S.keys_out[i - 1] >> 56);
  const int cur = i == nit ? S.nq : (int)(S.keys_out[i] >> 56);
  for (int q = prev + 1; q <= cur; ++q) S.qbase[q] = i;
}

__global__ void k_gather_items(Sched S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nit = S.chunk_item_base[S.grp_chunk_base[S.ngroups]];
  if (i >= nit) return;
  S.items[i] = S.items_unsorted[S.vals_out[i]];
}

__global__ void k_sched_totals(Sched S) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t nch = S.grp_chunk_base[S.ngroups];
  S.scalars[1] = nch;
  S.scalars[2] = S.chunk_item_base[nch];
  S.scalars[3] = S.slot_off[nch];
}

// --- phase-A panels ----------------------------------------------------------------
// Inner dimension K and columns N of panel G (= 2 s + class): class 0 forms
// L_k A_s (K = m, N = n), class 1 R_k A_s^T (K = n, N = m).
__device__ inline void panel_dims(const Plan &p, int G, int *K, int *N) {
  const int s = G >> 1;
  const int m = p.dimL[p.psi_sec[4 * s]], n = p.dimR[p.psi_sec[4 * s + 3]];
  *K = (G & 1) ? n : m;
  *N = (G & 1) ? m : n;
}

// Rows of T_k: the output's left dimension (class 0) or right dimension (class 1).
__device__ inline int task_t_rows(const Plan &p, const tns_task &t) {
  return t.order == 0 ? p.dimL[p.psi_sec[4 * t.out]] : p.dimR[p.psi_sec[4 * t.out + 3]];
}

__global__ void k_pan_keys(Plan p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  p.pa.keys_in[t] = 2 * p.tasks[t].in + p.tasks[t].order;
  p.pa.vals_in[t] = (int32_t)t;
}

// grp[G] = first panel-order position of panel G (from the sorted keys).
__global__ void k_pan_bounds(Plan p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  const int prev = i == 0 ? -1 : p.pa.keys_out[i - 1];
  const int cur = i == n ? p.pa.ngroups : p.pa.keys_out[i];
  for (int G = prev + 1; G <= cur; ++G) p.pa.grp[G] = i;
}

// Chunks of each panel-order position (scanned into ch afterwards); a task
// whose first factor is the identity takes no chunk: its intermediate is a
// scaled copy of the padded input sector, sized here (scanned into id_off).
__global__ void k_pan_nch(Plan p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const tns_task t = p.tasks[p.pa.idx[i]];
  const int rows = task_t_rows(p, t);
  if (ident_x(t)) {
    int K, N;
    panel_dims(p, 2 * t.in + t.order, &K, &N);
    p.pa.scratch[i] = 0;
    p.pa.id_sz[i] = (int64_t)rows * ld8(N);
  } else {
    p.pa.scratch[i] = (rows + PCH - 1) / PCH;
    p.pa.id_sz[i] = 0;
  }
}

// Per panel: first chunk, intermediate size (scanned into tb afterwards), cost.
__global__ void k_pan_sizes(Plan p) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  const Panels &A = p.pa;
  if (G > A.ngroups) return;
  A.gch[G] = A.ch[A.grp[G]];
  if (G == A.ngroups) return;
  int K, N;
  panel_dims(p, G, &K, &N);
  const int64_t nch = A.ch[A.grp[G + 1]] - A.ch[A.grp[G]];
  A.scratch[G] = nch * PCH * ld8(N);
  A.cost[G] = 2 * nch * PCH * (int64_t)N * K;
}

// Offsets of the intermediates: T_k at its chunk rows inside its panel's matrix.
__global__ void k_pan_toff(Plan p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Panels &A = p.pa;
  const int G = A.keys_out[i];
  int K, N;
  panel_dims(p, G, &K, &N);
  const int64_t ng = A.ngroups;
  p.t_off[A.idx[i]] = ident_x(p.tasks[A.idx[i]]) ? A.tb[ng] + A.id_off[i]
                                                 : A.tb[G] + (A.ch[i] - A.gch[G]) * PCH * ld8(N);
}

// Elements of all intermediates: the panels', then the identity-X copies.
__global__ void k_pan_t_total(Plan p, int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p.pa.scalars[3] = p.pa.tb[p.pa.ngroups] + p.pa.id_off[n];
}

// Phase-B segment records, one per position of the forward schedule's task
// list: T_k (class 0: output rows q, K = n; class 1: rows r, K = m) and the
// second operator block (class 0: R_k, r rows; class 1: L_k, q rows).
__global__ void k_segb(Plan p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = p.fwd.idx[i];
  const tns_task k = p.tasks[t];
  const int *so = p.psi_sec + 4 * k.out, *si = p.psi_sec + 4 * k.in;
  const int q = p.dimL[so[0]], r = p.dimR[so[3]], m = p.dimL[si[0]], nn = p.dimR[si[3]];
  SegRec s;
  s.a_off = p.t_off[t];
  s.K = k.order == 0 ? nn : m;
  s.arows = k.order == 0 ? q : r;
  s.brows = k.order == 0 ? r : q;
  const int blk = k.order == 0 ? k.rblk : k.lblk;
  s.b_off = blk >= 0 ? p.blk_off[blk] : -1;
  s.bld = blk >= 0 ? p.blk_ld[blk] : 0;
  p.segb[i] = s;
}

// Panel cost order (descending) and work queue: boustrophedon over the ranks.
__global__ void k_pan_rank_keys(Plan p) {
  const int64_t G = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Panels &A = p.pa;
  if (G >= A.ngroups) return;
  A.ikeys_in[G] = ~(uint64_t)A.cost[G];
  A.ivals_in[G] = (int32_t)G;
}
__global__ void k_pan_rank(Plan p) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Panels &A = p.pa;
  if (r >= A.ngroups) return;
  const int G = A.ivals_out[r];
  const int64_t round = r / A.nq, pos = r % A.nq;
  A.rank[G] = (int32_t)r;
  A.xcd[G] = (int32_t)((round & 1) ? A.nq - 1 - pos : pos);
}

// Work items of a panel: column tiles (extent from the tile table) x row
// pieces of whole GM-row tiles, so that an item costs about `target`.
__device__ inline void pan_split(const Plan &p, int G, int *tc, int *ncol, int *nrt, int *pieces) {
  const Panels &A = p.pa;
  int K, N;
  panel_dims(p, G, &K, &N);
  const int64_t nch = A.gch[G + 1] - A.gch[G];
  *tc = tile_ext_c(A.tiles, N);
  *ncol = nch > 0 ? (N + *tc - 1) / *tc : 0;
  *nrt = (int)((nch + PTILE_CH - 1) / PTILE_CH);
  const int64_t cost_col = 2 * (int64_t)*nrt * GM * *tc * K;
  const int64_t target = A.scalars[1];
  int64_t pc = target > 0 ? (cost_col + target - 1) / target : 1;
  if (pc > *nrt) pc = *nrt;
  *pieces = pc < 1 ? 1 : (int)pc;
}

__global__ void k_pan_total(Plan p) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  const Panels &A = p.pa;
  if (G >= A.ngroups) return;
  int K, N;
  panel_dims(p, G, &K, &N);
  const int64_t nch = A.gch[G + 1] - A.gch[G];
  if (nch == 0) return;
  const int tc = tile_ext_c(A.tiles, N), ncol = (N + tc - 1) / tc;
  const int64_t nrt = (nch + PTILE_CH - 1) / PTILE_CH;
  atomicAdd((unsigned long long *)&A.scalars[0], (unsigned long long)(2 * nrt * GM * (int64_t)tc * K * ncol));
}

// Target cost of a phase-A work item: PANEL_ITEMS_PER_CU items per CU on
// large products, but never below PANEL_ITEM_MIN_FLOP unless the product has
// fewer than PANEL_ITEMS_MIN_PER_CU items of that size per CU (small products
// keep that many items per CU, whose per-item overhead would otherwise
// dominate).
__global__ void k_pan_target(Plan p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int64_t total = p.pa.scalars[0];
    const int64_t fine = total / ((int64_t)PANEL_ITEMS_PER_CU * p.n_cu);
    const int64_t coarse = total / ((int64_t)PANEL_ITEMS_MIN_PER_CU * p.n_cu);
    const int64_t floor_ = coarse < PANEL_ITEM_MIN_FLOP ? coarse : PANEL_ITEM_MIN_FLOP;
    p.pa.scalars[1] = (fine > floor_ ? fine : floor_) + 1;
  }
}

__global__ void k_pan_count(Plan p) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  const Panels &A = p.pa;
  if (G >= A.items_cap) return;
  int tc = 0, ncol = 0, nrt = 0, pieces = 0;
  if (G < A.ngroups) pan_split(p, G, &tc, &ncol, &nrt, &pieces);
  A.scratch[G] = (int64_t)ncol * pieces;
}

__global__ void k_pan_items(Plan p) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  const Panels &A = p.pa;
  if (G >= A.ngroups) return;
  int tc, ncol, nrt, pieces, K, N;
  pan_split(p, G, &tc, &ncol, &nrt, &pieces);
  panel_dims(p, G, &K, &N);
  const int64_t nch = A.gch[G + 1] - A.gch[G], ib = A.item_base[G];
  constexpr uint64_t LM = (1ull << 28) - 1;
  for (int c = 0; c < ncol; ++c)
    for (int k = 0; k < pieces; ++k) {
      const int64_t r0 = (int64_t)k * nrt / pieces * PTILE_CH;
      int64_t r1 = (int64_t)(k + 1) * nrt / pieces * PTILE_CH;
      if (r1 > nch) r1 = nch;
      Item it;
      memset(&it, 0, sizeof(it));
      it.grp = G;
      it.p0 = (int32_t)(A.gch[G] + r0);
      it.np = (int32_t)(r1 - r0);
      it.c0 = c * tc;
      it.nc = min(tc, N - c * tc);
      it.mode = (tail_ext(it.nc, tc) / 32) << 16;
      it.cost = 2 * (r1 - r0) * PCH * (int64_t)it.nc * K;
      // the column tiles of a row piece are neighbours in the queue, so that
      // they run at the same time and share the piece's operator rows in L2
      const int64_t j = ib + (int64_t)k * ncol + c;
      A.items_unsorted[j] = it;
      A.ikeys_in[j] = ((uint64_t)A.xcd[G] << 56) | ((uint64_t)A.rank[G] << 28) | ((uint64_t)(j - ib) & LM);
      A.ivals_in[j] = (int32_t)j;
    }
}

__global__ void k_pan_pad_keys(Plan p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Panels &A = p.pa;
  if (i >= A.items_cap) return;
  if (i >= A.item_base[A.ngroups]) {
    A.ikeys_in[i] = ~0ull;
    A.ivals_in[i] = (int32_t)i;
  }
}

__global__ void k_pan_gather(Plan p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Panels &A = p.pa;
  const int64_t nit = A.item_base[A.ngroups];
  if (i > nit) return;
  if (i < nit) A.items[i] = A.items_unsorted[A.ivals_out[i]];
  const int prev = i == 0 ? -1 : (int)(A.ikeys_out[i - 1] >> 56);
  const int cur = i == nit ? A.nq : (int)(A.ikeys_out[i] >> 56);
  for (int q = prev + 1; q <= cur; ++q) A.qbase[q] = i;
  if (i == nit) A.scalars[2] = nit;
}

// Sizes of the padded copies of psi: sector s as m x ld8(n) and as its
// transpose n x ld8(m).
__global__ void k_pad_sizes(Plan p) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.nS) return;
  const int64_t m = p.dimL[p.psi_sec[4 * s]], n = p.dimR[p.psi_sec[4 * s + 3]];
  p.pp_off[s] = m * ld8((int)n);
  p.pt_off[s] = n * ld8((int)m);
}

// Backward grouping: three (key, task) entries per task -- input sector,
// left block, right block (keys offset by nS); absent entries get INT_MAX.
__global__ void k_bwd_keys(Plan p, int64_t ntasks) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntasks) return;
  const tns_task tk = p.tasks[t];
  p.bkeys_in[3 * t + 0] = tk.in;
  p.bkeys_in[3 * t + 1] = tk.lblk >= 0 ? p.nS + tk.lblk : 0x7fffffff;
  p.bkeys_in[3 * t + 2] = tk.rblk >= 0 ? p.nS + tk.rblk : 0x7fffffff;
  p.bvals_in[3 * t + 0] = (int32_t)t;
  p.bvals_in[3 * t + 1] = (int32_t)t;
  p.bvals_in[3 * t + 2] = (int32_t)t;
}

__global__ void k_bwd_count(Plan p, Sched S, int64_t nent) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nent) return;
  const int k = p.bkeys_out[e];
  if (k != 0x7fffffff) atomicAdd((unsigned long long *)&S.scratch[k], 1ull);
}

__global__ void k_bwd_groups(Plan p, Sched S) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= S.ngroups) return;
  S.grp_begin[g] = (int32_t)S.grp_chunk_base[g];  // scan of counts (reused buffer)
  S.grp_n[g] = (int32_t)(S.grp_chunk_base[g + 1] - S.grp_chunk_base[g]);
  if (g < p.nS) {
    // the tasks of input sector g: the adjoint task list's CSR; d psi runs as
    // the forward product of that list, so the group gets no work here
    S.grp_n[g] = 0;
    S.grp_rows[g] = p.dimL[p.psi_sec[4 * g]];
    S.grp_cols[g] = p.dimR[p.psi_sec[4 * g + 3]];
    S.grp_out[g] = g;
    S.grp_mode[g] = M_DPSI;
  } else {
    const int b = g - p.nS;
    S.grp_rows[g] = p.blk_rows[b];
    S.grp_cols[g] = p.blk_cols[b];
    S.grp_out[g] = b;
    S.grp_mode[g] = p.op_side[p.blk_op[b]] ? M_DR : M_DL;
  }
}

// Adjoint task j: the task at position j of the backward grouping (sorted by
// input sector, forward order inside a sector) with its sectors swapped.
// The evaluation order is chosen for the swapped shapes by the rule of the
// forward list (order 1 only if strictly cheaper); identity sides keep their
// cost (their sectors have equal dimensions).
__global__ void k_adj_tasks(Plan p, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const tns_task f = p.tasks[p.bwd.idx[j]];
  tns_task t = f;
  t.out = f.in;
  t.in = f.out;
  const int64_t q = p.dimL[p.psi_sec[4 * t.out]], r = p.dimR[p.psi_sec[4 * t.out + 3]];
  const int64_t m = p.dimL[p.psi_sec[4 * t.in]], nn = p.dimR[p.psi_sec[4 * t.in + 3]];
  t.order = 0;
  if (t.lblk >= 0 && t.rblk >= 0) {
    const int64_t c0 = 2 * q * nn * (m + r), c1 = 2 * m * r * (nn + q);
    t.order = c1 < c0 ? 1 : 0;
    t.cost = c1 < c0 ? c1 : c0;
  }
  p.adj.tasks[j] = t;
}

// CSR of the adjoint list: the backward grouping's begin of input sector s.
__global__ void k_adj_ptr(Plan p, int64_t ntasks) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > p.nS) return;
  p.adj.out_ptr[s] = s < p.nS ? p.bwd.grp_begin[s] : (int32_t)ntasks;
}

__global__ void k_copy_i32(const int32_t *a, int32_t *b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void k_i32_to_i64(const int32_t *a, int64_t *b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}
__global__ void k_i64_to_i32(const int64_t *a, int32_t *b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (int32_t)a[i];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static tns_status validate(const tns_problem *P, int32_t *nmax_out, int32_t *maxdim_out) {
  if (!P) return TNS_ERR_ARG;
  if (P->nL <= 0 || P->nR <= 0 || P->nS < 0 || P->nOps < 0 || P->nBlk < 0 || P->nTerms < 0 || P->n_vals < 0)
    return TNS_ERR_ARG;
  if (!P->qL || !P->dimL || !P->qR || !P->dimR || !P->psi_off) return TNS_ERR_ARG;
  if (P->nS > 0 && !P->psi_sec) return TNS_ERR_ARG;
  if (P->nOps > 0 && (!P->op_side || !P->op_dN || !P->op_d2Sz)) return TNS_ERR_ARG;
  if (P->nBlk > 0 && (!P->blk_op || !P->blk_in || !P->blk_out || !P->blk_rows || !P->blk_cols || !P->blk_ld ||
                      !P->blk_off))
    return TNS_ERR_ARG;
  if (P->nTerms > 0 && (!P->term_L || !P->term_ma || !P->term_mb || !P->term_R || !P->term_coef))
    return TNS_ERR_ARG;
  int32_t maxdim = 1;
  // sector dimensions 1..MAX_DIM: every block and sector matrix then holds
  // fewer than 2^31 elements (32-bit element indices inside one matrix)
  for (int i = 0; i < P->nL; ++i) {
    if (P->dimL[i] <= 0 || P->dimL[i] > MAX_DIM) return TNS_ERR_SHAPE;
    maxdim = std::max(maxdim, P->dimL[i]);
  }
  for (int i = 0; i < P->nR; ++i) {
    if (P->dimR[i] <= 0 || P->dimR[i] > MAX_DIM) return TNS_ERR_SHAPE;
    maxdim = std::max(maxdim, P->dimR[i]);
  }
  for (int i = 1; i < P->nL; ++i)
    if (P->qL[2 * i] < P->qL[2 * i - 2] || (P->qL[2 * i] == P->qL[2 * i - 2] && P->qL[2 * i + 1] <= P->qL[2 * i - 1]))
      return TNS_ERR_QN;
  for (int i = 1; i < P->nR; ++i)
    if (P->qR[2 * i] < P->qR[2 * i - 2] || (P->qR[2 * i] == P->qR[2 * i - 2] && P->qR[2 * i + 1] <= P->qR[2 * i - 1]))
      return TNS_ERR_QN;
  // wavefunction sectors: valid, conserving, strictly ascending, packed
  if (P->psi_off[0] != 0) return TNS_ERR_SHAPE;
  for (int s = 0; s < P->nS; ++s) {
    const int32_t *e = P->psi_sec + 4 * s;
    if (e[0] < 0 || e[0] >= P->nL || e[1] < 0 || e[1] > 3 || e[2] < 0 || e[2] > 3 || e[3] < 0 || e[3] >= P->nR)
      return TNS_ERR_SHAPE;
    const int N = P->qL[2 * e[0]] + site_N(e[1]) + site_N(e[2]) + P->qR[2 * e[3]];
    const int S = P->qL[2 * e[0] + 1] + site_2Sz(e[1]) + site_2Sz(e[2]) + P->qR[2 * e[3] + 1];
    if (N != P->target_N || S != P->target_2Sz) return TNS_ERR_QN;
    if (s > 0) {
      const int32_t *f = e - 4;
      const int64_t ka = ((int64_t)f[0] * 4 + f[1]) * 4 + f[2], kb = ((int64_t)e[0] * 4 + e[1]) * 4 + e[2];
      if (kb <= ka) return TNS_ERR_SHAPE;
    }
    if (P->psi_off[s + 1] - P->psi_off[s] != (int64_t)P->dimL[e[0]] * P->dimR[e[3]]) return TNS_ERR_SHAPE;
  }
  // operators and blocks
  for (int o = 0; o < P->nOps; ++o)
    if (P->op_side[o] != 0 && P->op_side[o] != 1) return TNS_ERR_ARG;
  std::vector<int> seen;  // (op, in) uniqueness
  const int nmax = std::max(P->nL, P->nR);
  seen.assign((size_t)P->nOps * nmax, 0);
  for (int b = 0; b < P->nBlk; ++b) {
    const int o = P->blk_op[b];
    if (o < 0 || o >= P->nOps) return TNS_ERR_SHAPE;
    const int side = P->op_side[o];
    const int ns = side ? P->nR : P->nL;
    const int32_t *q = side ? P->qR : P->qL;
    const int32_t *dim = side ? P->dimR : P->dimL;
    const int i = P->blk_in[b], j = P->blk_out[b];
    if (i < 0 || i >= ns || j < 0 || j >= ns) return TNS_ERR_SHAPE;
    if (q[2 * j] != q[2 * i] + P->op_dN[o] || q[2 * j + 1] != q[2 * i + 1] + P->op_d2Sz[o]) return TNS_ERR_QN;
    if (P->blk_rows[b] != dim[j] || P->blk_cols[b] != dim[i] || P->blk_ld[b] < P->blk_cols[b]) return TNS_ERR_SHAPE;
    if (P->blk_off[b] < 0 || P->blk_off[b] % 8 != 0 || P->blk_ld[b] % 8 != 0 ||
        P->blk_off[b] + (int64_t)P->blk_rows[b] * P->blk_ld[b] > P->n_vals)
      return TNS_ERR_SHAPE;
    if (seen[(size_t)o * nmax + i]++) return TNS_ERR_SHAPE;
  }
  // terms conserve (N, 2Sz)
  for (int k = 0; k < P->nTerms; ++k) {
    const int oL = P->term_L[k], oR = P->term_R[k], ma = P->term_ma[k], mb = P->term_mb[k];
    if (ma < 0 || ma > 15 || mb < 0 || mb > 15) return TNS_ERR_ARG;
    if (oL < -1 || oL >= P->nOps || oR < -1 || oR >= P->nOps) return TNS_ERR_ARG;
    if ((oL >= 0 && P->op_side[oL] != 0) || (oR >= 0 && P->op_side[oR] != 1)) return TNS_ERR_ARG;
    int dN = 0, dS = 0, a, c;
    mono_shift(ma, &a, &c); dN += a; dS += c;
    mono_shift(mb, &a, &c); dN += a; dS += c;
    if (oL >= 0) { dN += P->op_dN[oL]; dS += P->op_d2Sz[oL]; }
    if (oR >= 0) { dN += P->op_dN[oR]; dS += P->op_d2Sz[oR]; }
    if (dN != 0 || dS != 0) return TNS_ERR_QN;
  }
  *nmax_out = nmax;
  *maxdim_out = maxdim;
  return TNS_OK;
}

static int device_cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

static int device_xcd_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || n <= 0) return 1;
  return std::min(n, NQ_MAX);
}

static size_t radix_tmp_u64(int64_t n) {
  size_t tmp = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                           (const int32_t *)nullptr, (int32_t *)nullptr, (int)n);
  return tmp;
}
static size_t radix_tmp_i32(int64_t n) {
  size_t tmp = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const int32_t *)nullptr, (int32_t *)nullptr,
                                           (const int32_t *)nullptr, (int32_t *)nullptr, (int)n);
  return tmp;
}

// Carves one schedule's arrays; `idx` may be supplied by the caller.
// tile_sum: the number of output tiles of all groups at the smallest tile
// extent (32 x 32 with a tile table, tile_r rows without).  Work items are
// bounded without knowing the tasks: k_chunks closes a chunk before the task
// that would take it over cap = target x (tiles of the group at the largest
// extent), so any two consecutive chunks of a group cost more than cap, a
// group of cost c has at most 1 + 2c / cap chunks, and with target above
// total / (ITEMS_PER_CU n_cu) all groups together have at most
// tile_sum + 2 x 16 x ITEMS_PER_CU n_cu items (16 smallest tiles per
// largest one; factor 1 without a tile table).
static void layout_sched(Carve &cv, Sched &S, int32_t ngroups, int64_t ntcap, int64_t chunks_cap, int64_t tile_sum,
                         int n_cu, int tile_r, int tile_c, uint32_t tiles, int nq, bool own_idx) {
  S.ngroups = ngroups;
  S.ntcap = ntcap;
  S.chunks_cap = chunks_cap;
  S.tile_r = tile_r;
  S.tile_c = tile_c;
  S.tiles = tiles;
  const int64_t per_big = tiles ? (int64_t)(GM / 32) * (GN / 32) : 1;
  S.items_cap = std::max<int64_t>(chunks_cap, tile_sum + 2 * per_big * ITEMS_PER_CU * (int64_t)n_cu + 16);
  S.nq = nq;
  if (own_idx) S.idx = cv.take<int32_t>(ntcap);
  const size_t ng = std::max(1, ngroups);
  S.grp_begin = cv.take<int32_t>(ng); S.grp_n = cv.take<int32_t>(ng);
  S.grp_rows = cv.take<int32_t>(ng); S.grp_cols = cv.take<int32_t>(ng);
  S.grp_out = cv.take<int32_t>(ng); S.grp_mode = cv.take<int32_t>(ng);
  S.grp_cost = cv.take<int64_t>(ng); S.grp_chunk_base = cv.take<int64_t>(ng + 1);
  S.chunks = cv.take<Chunk>(chunks_cap);
  S.slot_off = cv.take<int64_t>(chunks_cap + 1);
  S.chunk_item_base = cv.take<int64_t>(chunks_cap + 1);
  S.items_unsorted = cv.take<Item>(S.items_cap);
  S.items = cv.take<Item>(S.items_cap);
  S.keys_in = cv.take<uint64_t>(S.items_cap); S.keys_out = cv.take<uint64_t>(S.items_cap);
  S.vals_in = cv.take<int32_t>(S.items_cap); S.vals_out = cv.take<int32_t>(S.items_cap);
  S.sort_tmp_bytes = radix_tmp_u64(S.items_cap);
  S.sort_tmp = cv.take<char>(S.sort_tmp_bytes + 256);
  S.qbase = cv.take<int64_t>(NQ_MAX + 1);
  if (tiles) {  // room for the narrow list (a later table may have 256-column entries)
    S.items_n = cv.take<Item>(S.items_cap);
    S.qbase_n = cv.take<int64_t>(NQ_MAX + 1);
  } else {
    S.items_n = S.items;
    S.qbase_n = S.qbase;
  }
  S.scratch = cv.take<int64_t>(std::max<int64_t>(ng, chunks_cap) + 1);
  S.scalars = cv.take<int64_t>(8);
}

// Carves the phase-A panel arrays.
static void layout_panels(Carve &cv, Panels &A, int32_t ng, int64_t ntcap, int maxdim, int n_cu, int nq,
                          uint32_t tiles) {
  A.ngroups = ng;
  A.nq = nq;
  A.ntcap = ntcap;
  A.tiles = tiles;
  // items: a panel's column tiles (smallest extent 32) plus one extra row
  // piece per PANEL_ITEMS_PER_CU share of the work
  A.items_cap = std::max<int64_t>(2 * (int64_t)PANEL_ITEMS_PER_CU * n_cu + (int64_t)ng * ((maxdim + 31) / 32) + 16, ng);
  const size_t g1 = (size_t)ng + 1;
  A.keys_in = cv.take<int32_t>(ntcap); A.keys_out = cv.take<int32_t>(ntcap);
  A.vals_in = cv.take<int32_t>(ntcap); A.idx = cv.take<int32_t>(ntcap);
  A.ch = cv.take<int64_t>(ntcap + 1);
  A.id_sz = cv.take<int64_t>(ntcap);
  A.id_off = cv.take<int64_t>(ntcap + 1);
  A.grp = cv.take<int64_t>(g1); A.gch = cv.take<int64_t>(g1); A.tb = cv.take<int64_t>(g1);
  A.cost = cv.take<int64_t>(g1);
  A.rank = cv.take<int32_t>(g1); A.xcd = cv.take<int32_t>(g1);
  A.item_base = cv.take<int64_t>(g1);
  A.items_unsorted = cv.take<Item>(A.items_cap); A.items = cv.take<Item>(A.items_cap);
  A.ikeys_in = cv.take<uint64_t>(A.items_cap); A.ikeys_out = cv.take<uint64_t>(A.items_cap);
  A.ivals_in = cv.take<int32_t>(A.items_cap); A.ivals_out = cv.take<int32_t>(A.items_cap);
  A.sort_tmp_bytes = std::max(radix_tmp_u64(A.items_cap), radix_tmp_i32(ntcap));
  A.sort_tmp = cv.take<char>(A.sort_tmp_bytes + 256);
  A.qbase = cv.take<int64_t>(NQ_MAX + 1);
  A.items_n = cv.take<Item>(A.items_cap);
  A.qbase_n = cv.take<int64_t>(NQ_MAX + 1);
  A.scratch = cv.take<int64_t>(std::max<int64_t>(std::max<int64_t>(ng, ntcap), A.items_cap) + 1);
  A.scalars = cv.take<int64_t>(8);
}

// Number of tasks of a validated problem, counted on the host with the
// enumeration rule of k_tasks (for an output sector and a term at most one
// input sector: the left block ending in the sector's left block sector, the
// site states the monomials map onto the sector's, the right block likewise,
// and that input sector present), so that the task arrays are sized exactly.
static int64_t host_task_count(const tns_problem *P, int32_t nmax) {
  std::vector<int32_t> psi_index((size_t)P->nL * 16, -1);
  for (int s = 0; s < P->nS; ++s) {
    const int32_t *e = P->psi_sec + 4 * s;
    psi_index[((size_t)e[0] * 4 + e[1]) * 4 + e[2]] = s;
  }
  std::vector<int32_t> bo((size_t)std::max(1, P->nOps) * nmax, -1);
  for (int b = 0; b < P->nBlk; ++b) bo[(size_t)P->blk_op[b] * nmax + P->blk_out[b]] = b;
  // site state reached from state s by monomial m (-1: none), per monomial
  int8_t src[16][4];
  for (int m = 0; m < 16; ++m)
    for (int t = 0; t < 4; ++t) {
      src[m][t] = -1;
      for (int u = 0; u < 4; ++u) {
        int v;
        if (mono_apply(m, u, &v) == t) src[m][t] = (int8_t)u;
      }
    }
  // terms whose two monomials reach the site states (ta, tb), per (ta, tb)
  std::vector<int32_t> site_terms[16];
  for (int k = 0; k < P->nTerms; ++k)
    for (int t = 0; t < 16; ++t)
      if (src[P->term_ma[k]][t >> 2] >= 0 && src[P->term_mb[k]][t & 3] >= 0) site_terms[t].push_back(k);
  int64_t n = 0;
  for (int so = 0; so < P->nS; ++so) {
    const int jL = P->psi_sec[4 * so], ta = P->psi_sec[4 * so + 1], tb = P->psi_sec[4 * so + 2];
    const int jR = P->psi_sec[4 * so + 3];
    for (const int32_t k : site_terms[ta * 4 + tb]) {
      const int oL = P->term_L[k], oR = P->term_R[k];
      int iL = jL, iR = jR;
      if (oL >= 0) {
        const int lb = bo[(size_t)oL * nmax + jL];
        if (lb < 0) continue;
        iL = P->blk_in[lb];
      }
      if (oR >= 0) {
        const int rb = bo[(size_t)oR * nmax + jR];
        if (rb < 0) continue;
        iR = P->blk_in[rb];
      }
      const int si = psi_index[((size_t)iL * 4 + src[P->term_ma[k]][ta]) * 4 + src[P->term_mb[k]][tb]];
      if (si < 0 || P->psi_sec[4 * si + 3] != iR) continue;
      ++n;
    }
  }
  return n;
}

// Lays out (or, with base == nullptr, sizes) the build workspace.
// ntasks_explicit >= 0: the number of tasks (of a table given by the caller,
// or the host count of the enumerated one); else counted here.
// backward: also the backward's schedules and the adjoint plan.
static size_t layout(const tns_problem *P, int32_t nmax, int32_t maxdim, int n_cu, int n_xcd, char *base,
                     Plan *pl, int64_t ntasks_explicit = -1, bool backward = true) {
  Carve cv{base, 0, 0};
  Plan p;
  memset(&p, 0, sizeof(p));
  p.nL = P->nL; p.nR = P->nR; p.nS = P->nS; p.nOps = P->nOps; p.nBlk = P->nBlk; p.nTerms = P->nTerms;
  p.nmax = nmax; p.n_cu = n_cu; p.n_vals = P->n_vals; p.maxdim = maxdim; p.tiles = TILES_DEFAULT;
  p.pad_ns = P->nS; p.epi_e0 = 0;
  p.psi_dim = P->psi_off[P->nS];
  const int64_t ntcap = std::max<int64_t>(1, ntasks_explicit >= 0 ? ntasks_explicit : host_task_count(P, nmax));
  p.qL = cv.take<int32_t>(2 * P->nL); p.dimL = cv.take<int32_t>(P->nL);
  p.qR = cv.take<int32_t>(2 * P->nR); p.dimR = cv.take<int32_t>(P->nR);
  p.psi_sec = cv.take<int32_t>(4 * (size_t)std::max(1, P->nS)); p.psi_off = cv.take<int64_t>(P->nS + 1);
  const size_t no = std::max(1, P->nOps), nb = std::max(1, P->nBlk), nt = std::max(1, P->nTerms);
  p.op_side = cv.take<int32_t>(no); p.op_dN = cv.take<int32_t>(no); p.op_d2Sz = cv.take<int32_t>(no);
  p.blk_op = cv.take<int32_t>(nb); p.blk_in = cv.take<int32_t>(nb); p.blk_out = cv.take<int32_t>(nb);
  p.blk_rows = cv.take<int32_t>(nb); p.blk_cols = cv.take<int32_t>(nb); p.blk_ld = cv.take<int32_t>(nb);
  p.blk_off = cv.take<int64_t>(nb);
  p.term_L = cv.take<int32_t>(nt); p.term_ma = cv.take<int32_t>(nt); p.term_mb = cv.take<int32_t>(nt);
  p.term_R = cv.take<int32_t>(nt); p.term_coef = cv.take<double>(nt);
  p.psi_index = cv.take<int32_t>((size_t)P->nL * 16);
  p.blk_of_out = cv.take<int32_t>(no * nmax);
  p.tasks = cv.take<tns_task>(ntcap);
  p.out_ptr = cv.take<int32_t>(P->nS + 1);
  p.scan_tmp = cv.take<int64_t>(P->nS + 1);
  p.scalars = cv.take<int64_t>(8);
  p.t_off = cv.take<int64_t>(ntcap + 1);
  p.segb = cv.take<SegRec>(ntcap);
  p.pp_off = cv.take<int64_t>(P->nS + 1);
  p.pt_off = cv.take<int64_t>(P->nS + 1);
  // forward schedule: 2 groups per sector (sigma and sigma^T of its
  // output), output tiles GM x GN at most, 32 x 32 at least
  const int64_t fchunks = 2 * (int64_t)ITEMS_PER_CU * n_cu + 4 * (int64_t)P->nS + 16;
  int64_t ftiles = 0;
  for (int s = 0; s < P->nS; ++s)
    ftiles += 2 * (int64_t)((P->dimL[P->psi_sec[4 * s]] + 31) / 32) * ((P->dimR[P->psi_sec[4 * s + 3]] + 31) / 32);
  layout_sched(cv, p.fwd, 2 * P->nS, ntcap, fchunks, ftiles, n_cu, GM, GN, TILES_DEFAULT, n_xcd, true);
  layout_panels(cv, p.pa, 2 * P->nS, ntcap, maxdim, n_cu, n_xcd, TILES_DEFAULT);
  const int64_t bent = backward ? 3 * ntcap : 0;
  Adjoint &J = p.adj;
  if (backward) {
    // backward schedule: one group per sector (d psi) and one per block (d L / d R)
    p.bkeys_in = cv.take<int32_t>(bent); p.bkeys_out = cv.take<int32_t>(bent); p.bvals_in = cv.take<int32_t>(bent);
    p.bwd.idx = cv.take<int32_t>(bent);
    p.bsort_tmp_bytes = radix_tmp_i32(bent);
    p.bsort_tmp = cv.take<char>(p.bsort_tmp_bytes + 256);
    const int32_t bgroups = P->nS + P->nBlk;
    const int64_t bchunks = 2 * (int64_t)ITEMS_PER_CU * n_cu + 2 * (int64_t)bgroups + 16;
    int64_t btiles = 0;  // row panels of the operator-block groups (the sector groups stay empty)
    for (int b = 0; b < P->nBlk; ++b) btiles += (P->blk_rows[b] + TQ - 1) / TQ;
    layout_sched(cv, p.bwd, bgroups, bent, bchunks, btiles, n_cu, TQ, 0, 0u, n_xcd, false);
    // adjoint task list (d psi of the backward) and its forward schedule
    J.tasks = cv.take<tns_task>(ntcap);
    J.out_ptr = cv.take<int32_t>(P->nS + 1);
    J.scalars = cv.take<int64_t>(8);
    J.blk_off = cv.take<int64_t>(nb);
    J.blk_ld = cv.take<int32_t>(nb);
    J.t_off = cv.take<int64_t>(ntcap + 1);
    J.segb = cv.take<SegRec>(ntcap);
    J.n_vals = 0;
    for (int b = 0; b < P->nBlk; ++b) J.n_vals += (int64_t)P->blk_cols[b] * ld8(P->blk_rows[b]);
    // the adjoint runs in FP32 / FP64 only: its lists are built narrow
    layout_sched(cv, J.fwd, 2 * P->nS, ntcap, fchunks, ftiles, n_cu, GM, GN, tiles_narrow(TILES_DEFAULT), n_xcd,
                 true);
    layout_panels(cv, J.pa, 2 * P->nS, ntcap, maxdim, n_cu, n_xcd, tiles_narrow(TILES_DEFAULT));
  }
  // counts that the sorts and item indices hold in 32 bits
  const int64_t caps[] = {bent, p.fwd.items_cap, p.bwd.items_cap, J.fwd.items_cap, p.pa.items_cap, J.pa.items_cap,
                          p.fwd.chunks_cap, p.bwd.chunks_cap};
  for (int64_t c : caps)
    if (c >= INT32_MAX) return 0;
  if (pl) *pl = p;
  return cv.off + 256;
}

template <class T>
static hipError_t up(T *dst, const T *src, size_t n, hipStream_t st) {
  if (n == 0 || !src) return hipSuccess;
  return hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, st);
}

static tns_status sched_items(Sched &S, hipStream_t st);

// Chunks, partial slots, work items and the longest-first order of a
// schedule whose groups (begin, n, rows, cols, out, mode) are set.
static tns_status finish_sched(const Plan &p, Sched &S, hipStream_t st) {
  const int B = 256;
  const int ng = S.ngroups;
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(8), 0, st, S.scalars, (int64_t)8, (int64_t)0);
  if (ng > 0) {
    hipLaunchKernelGGL(k_group_cost, dim3(nblk(ng, 4)), dim3(256), 0, st, p, S);
    hipLaunchKernelGGL(k_chunks<false>, dim3(nblk(ng, B)), dim3(B), 0, st, p, S);
    hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, S.scratch, S.grp_chunk_base, (int64_t)ng);
    hipLaunchKernelGGL(k_chunks<true>, dim3(nblk(ng, B)), dim3(B), 0, st, p, S);
  } else {
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(1), 0, st, S.grp_chunk_base, (int64_t)1, (int64_t)0);
  }
  int64_t *slot_sz = S.scratch;
  int64_t *item_n = reinterpret_cast<int64_t *>(S.keys_out);  // items_cap >= chunks_cap
  hipLaunchKernelGGL(k_chunk_sizes, dim3(nblk(S.chunks_cap, B)), dim3(B), 0, st, S, slot_sz, item_n);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, slot_sz, S.slot_off, S.chunks_cap);
  return sched_items(S, st);
}

// One item list of a schedule whose chunks and slots are set, at the table
// S.tiles into S.items / S.qbase: tiles per chunk, longest first within each
// XCD queue, queue bounds and totals (S.scalars[1..3]).
static tns_status sched_list(Sched &S, hipStream_t st) {
  const int B = 256;
  int64_t *item_n = reinterpret_cast<int64_t *>(S.keys_out);
  hipLaunchKernelGGL(k_chunk_sizes, dim3(nblk(S.chunks_cap, B)), dim3(B), 0, st, S, S.scratch, item_n);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, item_n, S.chunk_item_base, S.chunks_cap);
  hipLaunchKernelGGL(k_items, dim3(nblk(S.chunks_cap, B)), dim3(B), 0, st, S);
  hipLaunchKernelGGL(k_chunk_keys, dim3(nblk(S.chunks_cap, B)), dim3(B), 0, st, S);
  TNS_HIP(hipGetLastError());
  size_t tmp = S.sort_tmp_bytes;  // sized for items_cap >= chunks_cap entries
  TNS_HIP(hipcub::DeviceRadixSort::SortPairs(S.sort_tmp, tmp, S.keys_in, S.keys_out, S.vals_in, S.vals_out,
                                             (int)S.chunks_cap, 0, 64, st));
  hipLaunchKernelGGL(k_chunk_xcd, dim3(nblk(S.chunks_cap, B)), dim3(B), 0, st, S);
  hipLaunchKernelGGL(k_sort_keys, dim3(nblk(S.items_cap, B)), dim3(B), 0, st, S);
  TNS_HIP(hipGetLastError());
  tmp = S.sort_tmp_bytes;
  TNS_HIP(hipcub::DeviceRadixSort::SortPairs(S.sort_tmp, tmp, S.keys_in, S.keys_out, S.vals_in, S.vals_out,
                                             (int)S.items_cap, 0, 64, st));
  hipLaunchKernelGGL(k_gather_items, dim3(nblk(S.items_cap, B)), dim3(B), 0, st, S);
  hipLaunchKernelGGL(k_queue_bounds, dim3(nblk(S.items_cap + 1, B)), dim3(B), 0, st, S);
  hipLaunchKernelGGL(k_sched_totals, dim3(1), dim3(1), 0, st, S);
  TNS_HIP(hipGetLastError());
  return TNS_OK;
}

// Work items of a schedule: the list at its table and, when the table has
// 256-column entries, the list at the narrow form (items_n, qbase_n, totals
// in scalars[5..7]).  Both cover the same chunks and partial slots.
static tns_status sched_items(Sched &S, hipStream_t st) {
  if (tiles_wide(S.tiles)) {
    Sched W = S;
    W.tiles = tiles_narrow(S.tiles);
    W.items = S.items_n;
    W.qbase = S.qbase_n;
    W.scalars = S.scalars + 4;
    const tns_status s = sched_list(W, st);
    if (s != TNS_OK) return s;
  }
  return sched_list(S, st);
}

// Work items of the phase-A panels for the table p.pa.tiles into p.pa.items /
// p.pa.qbase, grouped by panel in descending panel cost inside each XCD queue.
static tns_status pan_list(const Plan &p, hipStream_t st) {
  const int B = 256;
  const Panels &A = p.pa;
  const int ng = A.ngroups;
  // scalars 0..2 (item cost total, target, items); 3 holds the intermediate
  // size written when the panels were built
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(8), 0, st, A.scalars, (int64_t)3, (int64_t)0);
  if (ng > 0) hipLaunchKernelGGL(k_pan_total, dim3(nblk(ng, B)), dim3(B), 0, st, p);
  hipLaunchKernelGGL(k_pan_target, dim3(1), dim3(1), 0, st, p);
  hipLaunchKernelGGL(k_pan_count, dim3(nblk(A.items_cap, B)), dim3(B), 0, st, p);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, A.scratch, A.item_base, (int64_t)ng);
  if (ng > 0) hipLaunchKernelGGL(k_pan_items, dim3(nblk(ng, B)), dim3(B), 0, st, p);
  hipLaunchKernelGGL(k_pan_pad_keys, dim3(nblk(A.items_cap, B)), dim3(B), 0, st, p);
  TNS_HIP(hipGetLastError());
  size_t tmp = A.sort_tmp_bytes;
  TNS_HIP(hipcub::DeviceRadixSort::SortPairs(A.sort_tmp, tmp, A.ikeys_in, A.ikeys_out, A.ivals_in, A.ivals_out,
                                             (int)A.items_cap, 0, 64, st));
  hipLaunchKernelGGL(k_pan_gather, dim3(nblk(A.items_cap + 1, B)), dim3(B), 0, st, p);
  TNS_HIP(hipGetLastError());
  return TNS_OK;
}

// Panel items at the panels' table and, when it has 256-column entries, at
// its narrow form (items_n, qbase_n, totals in scalars[4..6]).
static tns_status pan_items(const Plan &p, hipStream_t st) {
  if (tiles_wide(p.pa.tiles)) {
    Plan q = p;
    q.pa.tiles = tiles_narrow(p.pa.tiles);
    q.pa.items = p.pa.items_n;
    q.pa.qbase = p.pa.qbase_n;
    q.pa.scalars = p.pa.scalars + 4;
    const tns_status s = pan_list(q, st);
    if (s != TNS_OK) return s;
  }
  return pan_list(p, st);
}

// Phase-A panels of a built task list: panel order of the tasks, chunks,
// offsets of the intermediates (t_off), panel queues and work items.
static tns_status build_panels(const Plan &p, hipStream_t st) {
  const int B = 256;
  const Panels &A = p.pa;
  const int64_t n = p.ntasks;
  const int ng = A.ngroups;
  if (n > 0) {
    hipLaunchKernelGGL(k_pan_keys, dim3(nblk(n, B)), dim3(B), 0, st, p, n);
    size_t tmp = A.sort_tmp_bytes;
    TNS_HIP(hipcub::DeviceRadixSort::SortPairs(A.sort_tmp, tmp, A.keys_in, A.keys_out, A.vals_in, A.idx, (int)n, 0,
                                               32, st));
  }
  hipLaunchKernelGGL(k_pan_bounds, dim3(nblk(n + 1, B)), dim3(B), 0, st, p, n);
  if (n > 0) hipLaunchKernelGGL(k_pan_nch, dim3(nblk(n, B)), dim3(B), 0, st, p, n);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, A.scratch, A.ch, n);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, A.id_sz, A.id_off, n);
  hipLaunchKernelGGL(k_pan_sizes, dim3(nblk(ng + 1, B)), dim3(B), 0, st, p);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, A.scratch, A.tb, (int64_t)ng);
  if (n > 0) hipLaunchKernelGGL(k_pan_toff, dim3(nblk(n, B)), dim3(B), 0, st, p, n);
  hipLaunchKernelGGL(k_pan_t_total, dim3(1), dim3(1), 0, st, p, n);
  if (ng > 0) {
    hipLaunchKernelGGL(k_pan_rank_keys, dim3(nblk(ng, B)), dim3(B), 0, st, p);
    size_t tmp = A.sort_tmp_bytes;
    TNS_HIP(hipcub::DeviceRadixSort::SortPairs(A.sort_tmp, tmp, A.ikeys_in, A.ikeys_out, A.ivals_in, A.ivals_out,
                                               ng, 0, 64, st));
    hipLaunchKernelGGL(k_pan_rank, dim3(nblk(ng, B)), dim3(B), 0, st, p);
  }
  TNS_HIP(hipGetLastError());
  return pan_items(p, st);
}

static void read_sched(Sched &S, const int64_t *h) {
  S.total_cost = h[0];
  S.nchunks = h[1];
  S.nitems = h[2];
  S.partial_elems = h[3];
  S.nitems_n = tiles_wide(S.tiles) ? h[6] : h[2];
}

static bool sched_fits(const Sched &S) {
  return S.nchunks <= S.chunks_cap && S.nitems <= S.items_cap && S.nitems_n <= S.items_cap;
}

// Panel item counts (scalars[2], [6]) as read back from the device.
static bool pan_counts(Panels &A, int64_t n, int64_t n_narrow) {
  A.nitems = n;
  A.nitems_n = tiles_wide(A.tiles) ? n_narrow : n;
  return A.nitems <= A.items_cap && A.nitems_n <= A.items_cap;
}

Plan adjoint_plan(const Plan &p) {
  const Adjoint &J = p.adj;
  Plan q = p;
  q.tasks = J.tasks;
  q.out_ptr = J.out_ptr;
  q.scalars = J.scalars;
  q.blk_off = J.blk_off;
  q.blk_ld = J.blk_ld;
  q.blk_rows = p.blk_cols;
  q.blk_cols = p.blk_rows;
  q.blk_in = p.blk_out;
  q.blk_out = p.blk_in;
  q.t_off = J.t_off;
  q.segb = J.segb;
  q.n_vals = J.n_vals;
  q.t_elems = J.t_elems;
  q.fwd = J.fwd;
  q.pa = J.pa;
  q.tiles = J.fwd.tiles;
  return q;
}

// The adjoint task list and its forward schedule (after the backward grouping,
// whose order by input sector it takes).  boff / bld: the transposed block
// table (host memory that stays valid until the stream has synchronised).
static tns_status build_adjoint(Plan &p, const int64_t *boff, const int32_t *bld, hipStream_t st) {
  const int B = 256;
  Adjoint &J = p.adj;
  TNS_HIP(up(J.blk_off, boff, p.nBlk, st));
  TNS_HIP(up(J.blk_ld, bld, p.nBlk, st));
  if (p.ntasks > 0) hipLaunchKernelGGL(k_adj_tasks, dim3(nblk(p.ntasks, B)), dim3(B), 0, st, p, p.ntasks);
  hipLaunchKernelGGL(k_adj_ptr, dim3(nblk(p.nS + 1, B)), dim3(B), 0, st, p, p.ntasks);
  TNS_HIP(hipGetLastError());
  Plan q = adjoint_plan(p);
  if (p.nS > 0)
    hipLaunchKernelGGL(k_fwd_groups, dim3(nblk(p.nS, 4)), dim3(256), 0, st, q, q.fwd);
  TNS_HIP(hipGetLastError());
  tns_status s = finish_sched(q, q.fwd, st);
  if (s != TNS_OK) return s;
  int64_t h[8];
  TNS_HIP(hipMemcpyAsync(h, q.fwd.scalars, sizeof(h), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipStreamSynchronize(st));
  read_sched(q.fwd, h);
  if (!sched_fits(q.fwd)) return TNS_ERR_WORKSPACE;
  s = build_panels(q, st);
  if (s != TNS_OK) return s;
  if (q.ntasks > 0) hipLaunchKernelGGL(k_segb, dim3(nblk(q.ntasks, B)), dim3(B), 0, st, q, q.ntasks);
  TNS_HIP(hipGetLastError());
  int64_t ext[4];
  TNS_HIP(hipMemcpyAsync(ext, q.pa.scalars + 3, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipMemcpyAsync(ext + 1, q.pa.ch + q.ntasks, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipMemcpyAsync(ext + 2, q.pa.scalars + 2, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipMemcpyAsync(ext + 3, q.pa.scalars + 6, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipStreamSynchronize(st));
  q.pa.t_elems = ext[0];
  q.pa.nchunks = ext[1];
  if (!pan_counts(q.pa, ext[2], ext[3])) return TNS_ERR_WORKSPACE;
  J.fwd = q.fwd;
  J.pa = q.pa;
  J.t_elems = ext[0];
  return TNS_OK;
}

}  // namespace tns

using namespace tns;

tns_status tns::validate_problem(const tns_problem *P, int32_t *nmax, int32_t *maxdim) {
  return validate(P, nmax, maxdim);
}

size_t tns::plan_workspace(const tns_problem *P, int32_t nmax, int32_t maxdim, int64_t nx_explicit, bool backward) {
  return layout(P, nmax, maxdim, device_cu_count(), device_xcd_count(), nullptr, nullptr, nx_explicit, backward);
}

extern "C" tns_status tns_count_tasks(const tns_problem *prob, int64_t *ntasks) {
  if (!ntasks) return TNS_ERR_ARG;
  int32_t nmax = 0, maxdim = 0;
  const tns_status s = validate(prob, &nmax, &maxdim);
  if (s != TNS_OK) return s;
  *ntasks = host_task_count(prob, nmax);
  return TNS_OK;
}

extern "C" size_t tns_tasklist_workspace_bytes(const tns_problem *prob) {
  int32_t nmax = 0, maxdim = 0;
  if (validate(prob, &nmax, &maxdim) != TNS_OK) return 0;
  return layout(prob, nmax, maxdim, device_cu_count(), device_xcd_count(), nullptr, nullptr);
}

namespace tns {

// The plan of a validated problem in the caller's workspace.  Without xtasks
// the task table is enumerated on the device from the terms (levels 1-2);
// with xtasks (nx tasks, sorted by output sector, CSR xptr[nS + 1], host
// memory valid until the call returns) that table is taken as it stands.
// backward: also the backward grouping and the adjoint plan.
tns_status build_plan(const tns_problem *P, int32_t nmax, int32_t maxdim, const tns_task *xtasks,
                      const int32_t *xptr, int64_t nx, bool backward, void *ws, size_t ws_bytes, tns_tasklist *out,
                      hipStream_t st) {
  const int n_cu = device_cu_count(), n_xcd = device_xcd_count();
  const int64_t ntx = xtasks ? nx : host_task_count(P, nmax);
  const size_t need = layout(P, nmax, maxdim, n_cu, n_xcd, nullptr, nullptr, ntx, backward);
  if (need == 0) return TNS_ERR_SHAPE;  // schedule counts beyond 32-bit indices
  if (ws_bytes < need) return TNS_ERR_WORKSPACE;
  Plan p;
  layout(P, nmax, maxdim, n_cu, n_xcd, (char *)ws, &p, ntx, backward);
  tns_status s = TNS_OK;
  TNS_HIP(up(p.qL, P->qL, 2 * (size_t)P->nL, st));
  TNS_HIP(up(p.dimL, P->dimL, P->nL, st));
  TNS_HIP(up(p.qR, P->qR, 2 * (size_t)P->nR, st));
  TNS_HIP(up(p.dimR, P->dimR, P->nR, st));
  TNS_HIP(up(p.psi_sec, P->psi_sec, 4 * (size_t)P->nS, st));
  TNS_HIP(up(p.psi_off, P->psi_off, (size_t)P->nS + 1, st));
  TNS_HIP(up(p.op_side, P->op_side, P->nOps, st));
  TNS_HIP(up(p.op_dN, P->op_dN, P->nOps, st));
  TNS_HIP(up(p.op_d2Sz, P->op_d2Sz, P->nOps, st));
  TNS_HIP(up(p.blk_op, P->blk_op, P->nBlk, st));
  TNS_HIP(up(p.blk_in, P->blk_in, P->nBlk, st));
  TNS_HIP(up(p.blk_out, P->blk_out, P->nBlk, st));
  TNS_HIP(up(p.blk_rows, P->blk_rows, P->nBlk, st));
  TNS_HIP(up(p.blk_cols, P->blk_cols, P->nBlk, st));
  TNS_HIP(up(p.blk_ld, P->blk_ld, P->nBlk, st));
  TNS_HIP(up(p.blk_off, P->blk_off, P->nBlk, st));
  TNS_HIP(up(p.term_L, P->term_L, P->nTerms, st));
  TNS_HIP(up(p.term_ma, P->term_ma, P->nTerms, st));
  TNS_HIP(up(p.term_mb, P->term_mb, P->nTerms, st));
  TNS_HIP(up(p.term_R, P->term_R, P->nTerms, st));
  TNS_HIP(up(p.term_coef, P->term_coef, P->nTerms, st));

  const int B = 256;
  if (P->nS > 0) hipLaunchKernelGGL(k_pad_sizes, dim3(nblk(P->nS, B)), dim3(B), 0, st, p);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, p.pp_off, p.pp_off, (int64_t)P->nS);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, p.pt_off, p.pt_off, (int64_t)P->nS);
  const unsigned wblk = nblk(std::max(1, P->nS), 4);
  if (xtasks) {
    TNS_HIP(up(p.tasks, xtasks, (size_t)nx, st));
    TNS_HIP(up(p.out_ptr, xptr, (size_t)P->nS + 1, st));
  } else {
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk((int64_t)P->nL * 16, B)), dim3(B), 0, st, p.psi_index,
                       (int64_t)P->nL * 16, -1);
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk((int64_t)std::max(1, P->nOps) * nmax, B)), dim3(B), 0, st,
                       p.blk_of_out, (int64_t)std::max(1, P->nOps) * nmax, -1);
    if (P->nS > 0) hipLaunchKernelGGL(k_psi_index, dim3(nblk(P->nS, B)), dim3(B), 0, st, p);
    if (P->nBlk > 0) hipLaunchKernelGGL(k_blk_of_out, dim3(nblk(P->nBlk, B)), dim3(B), 0, st, p);
    TNS_HIP(hipGetLastError());
    // levels 1-2: task counts per output sector -> CSR -> canonical fill
    if (P->nS > 0) {
      hipLaunchKernelGGL(k_tasks<false>, dim3(wblk), dim3(256), 0, st, p);
      hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, p.scan_tmp, p.scan_tmp, (int64_t)P->nS);
      // the task arrays are sized for the host's count of the same rule;
      // the device's count must equal it before the fill writes them
      int64_t total = 0;
      TNS_HIP(hipMemcpyAsync(&total, p.scan_tmp + P->nS, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      TNS_HIP(hipStreamSynchronize(st));
      if (total != ntx) return TNS_ERR_WORKSPACE;
    } else {
      hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(1), 0, st, p.scan_tmp, (int64_t)1, (int64_t)0);
    }
    hipLaunchKernelGGL(k_i64_to_i32, dim3(nblk(P->nS + 1, B)), dim3(B), 0, st, p.scan_tmp, p.out_ptr,
                       (int64_t)P->nS + 1);
    if (P->nS > 0) hipLaunchKernelGGL(k_tasks<true>, dim3(wblk), dim3(256), 0, st, p);
  }
  if (P->nS > 0) hipLaunchKernelGGL(k_fwd_groups, dim3(wblk), dim3(256), 0, st, p, p.fwd);
  TNS_HIP(hipGetLastError());
  s = finish_sched(p, p.fwd, st);
  if (s != TNS_OK) return s;
  int64_t h[8];
  TNS_HIP(hipMemcpyAsync(h, p.fwd.scalars, sizeof(h), hipMemcpyDeviceToHost, st));
  int32_t nt32 = 0;
  TNS_HIP(hipMemcpyAsync(&nt32, p.out_ptr + P->nS, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipStreamSynchronize(st));
  p.ntasks = nt32;
  read_sched(p.fwd, h);
  if (!sched_fits(p.fwd)) return TNS_ERR_WORKSPACE;

  // phase-A panels and the offsets of the forward intermediates
  s = build_panels(p, st);
  if (s != TNS_OK) return s;
  if (p.ntasks > 0) hipLaunchKernelGGL(k_segb, dim3(nblk(p.ntasks, B)), dim3(B), 0, st, p, p.ntasks);
  TNS_HIP(hipGetLastError());

  if (!backward) {
    int64_t ext[6];
    TNS_HIP(hipMemcpyAsync(ext, p.pa.scalars + 3, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TNS_HIP(hipMemcpyAsync(ext + 1, p.pp_off + P->nS, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TNS_HIP(hipMemcpyAsync(ext + 2, p.pt_off + P->nS, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TNS_HIP(hipMemcpyAsync(ext + 3, p.pa.ch + p.ntasks, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TNS_HIP(hipMemcpyAsync(ext + 4, p.pa.scalars + 2, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TNS_HIP(hipMemcpyAsync(ext + 5, p.pa.scalars + 6, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TNS_HIP(hipStreamSynchronize(st));
    p.t_elems = p.pa.t_elems = ext[0];
    p.pp_elems = ext[1];
    p.pt_elems = ext[2];
    p.pa.nchunks = ext[3];
    if (!pan_counts(p.pa, ext[4], ext[5])) return TNS_ERR_WORKSPACE;
    p.no_backward = 1;
  } else {
  // backward grouping: stable sort of (key, task) entries by key
  const int64_t nent = 3 * p.ntasks;
  if (nent > 0) {
    hipLaunchKernelGGL(k_bwd_keys, dim3(nblk(p.ntasks, B)), dim3(B), 0, st, p, p.ntasks);
    size_t tmp = p.bsort_tmp_bytes;
    TNS_HIP(hipcub::DeviceRadixSort::SortPairs(p.bsort_tmp, tmp, p.bkeys_in, p.bkeys_out, p.bvals_in, p.bwd.idx,
                                               (int)nent, 0, 32, st));
  }
  const int bg = p.bwd.ngroups;
  hipLaunchKernelGGL(k_fill_i64, dim3(nblk(bg + 1, B)), dim3(B), 0, st, p.bwd.scratch, (int64_t)bg + 1, (int64_t)0);
  if (nent > 0) hipLaunchKernelGGL(k_bwd_count, dim3(nblk(nent, B)), dim3(B), 0, st, p, p.bwd, nent);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, p.bwd.scratch, p.bwd.grp_chunk_base, (int64_t)bg);
  if (bg > 0) hipLaunchKernelGGL(k_bwd_groups, dim3(nblk(bg, B)), dim3(B), 0, st, p, p.bwd);
  TNS_HIP(hipGetLastError());
  s = finish_sched(p, p.bwd, st);
  if (s != TNS_OK) return s;
  TNS_HIP(hipMemcpyAsync(h, p.bwd.scalars, sizeof(h), hipMemcpyDeviceToHost, st));
  int64_t ext[6];
  TNS_HIP(hipMemcpyAsync(ext, p.pa.scalars + 3, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipMemcpyAsync(ext + 1, p.pp_off + P->nS, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipMemcpyAsync(ext + 2, p.pt_off + P->nS, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipMemcpyAsync(ext + 3, p.pa.ch + p.ntasks, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipMemcpyAsync(ext + 4, p.pa.scalars + 2, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipMemcpyAsync(ext + 5, p.pa.scalars + 6, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipStreamSynchronize(st));
  read_sched(p.bwd, h);
  p.t_elems = ext[0];
  p.pp_elems = ext[1];
  p.pt_elems = ext[2];
  p.pa.t_elems = ext[0];
  p.pa.nchunks = ext[3];
  if (!sched_fits(p.bwd)) return TNS_ERR_WORKSPACE;
  if (!pan_counts(p.pa, ext[4], ext[5])) return TNS_ERR_WORKSPACE;

  // adjoint task list and schedule (d psi of the backward)
  std::vector<int64_t> toff(std::max(1, P->nBlk));
  std::vector<int32_t> tld(std::max(1, P->nBlk));
  for (int64_t b = 0, o = 0; b < P->nBlk; ++b) {
    tld[b] = ld8(P->blk_rows[b]);
    toff[b] = o;
    o += (int64_t)P->blk_cols[b] * tld[b];
  }
  s = build_adjoint(p, toff.data(), tld.data(), st);
  if (s != TNS_OK) return s;
  }

  memset(out, 0, sizeof(*out));
  out->ntasks = p.ntasks;
  out->nitems = p.fwd.nitems;
  out->nslots = p.fwd.nchunks;
  out->partial_elems = p.fwd.partial_elems;
  out->total_flops = p.fwd.total_cost;
  out->psi_dim = p.psi_dim;
  out->tasks = p.tasks;
  out->out_ptr = p.out_ptr;
  memcpy(out->opaque, &p, sizeof(p));
  return TNS_OK;
}

}  // namespace tns

extern "C" tns_status tns_build_tasklist(const tns_problem *P, void *ws, size_t ws_bytes, tns_tasklist *out,
                                         hipStream_t st) {
  if (!out || !ws) return TNS_ERR_ARG;
  int32_t nmax = 0, maxdim = 0;
  const tns_status s = validate(P, &nmax, &maxdim);
  if (s != TNS_OK) return s;
  return build_plan(P, nmax, maxdim, nullptr, nullptr, 0, true, ws, ws_bytes, out, st);
}

extern "C" tns_status tns_set_tiles(tns_tasklist *tl, uint32_t tiles, hipStream_t st) {
  if (!tl || !tiles_valid(tiles)) return TNS_ERR_ARG;
  Plan &p = plan_of(tl);
  p.fwd.tiles = tiles;
  p.pa.tiles = tiles;
  p.tiles = tiles;
  tns_status s = sched_items(p.fwd, st);
  if (s != TNS_OK) return s;
  s = pan_items(p, st);
  if (s != TNS_OK) return s;
  int64_t h[8], na[8];
  TNS_HIP(hipMemcpyAsync(h, p.fwd.scalars, sizeof(h), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipMemcpyAsync(na, p.pa.scalars, sizeof(na), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipStreamSynchronize(st));
  read_sched(p.fwd, h);
  if (!pan_counts(p.pa, na[2], na[6]) || !sched_fits(p.fwd)) return TNS_ERR_WORKSPACE;
  tl->nitems = p.fwd.nitems;
  return TNS_OK;
}

extern "C" uint32_t tns_get_tiles(const tns_tasklist *tl) { return tl ? plan_of(tl).tiles : 0u; }

extern "C" const char *tns_status_string(tns_status s) {
  switch (s) {
    case TNS_OK: return "ok";
    case TNS_ERR_ARG: return "invalid argument";
    case TNS_ERR_SHAPE: return "inconsistent shape or offset";
    case TNS_ERR_QN: return "quantum numbers not conserved";
    case TNS_ERR_WORKSPACE: return "workspace too small";
    case TNS_ERR_HIP: return "HIP runtime error";
    case TNS_ERR_NUMERIC: return "non-finite value";
    case TNS_ERR_NOT_CONVERGED: return "not converged";
  }
  return "unknown status";
}
