// Backward of sigma = H_eff psi (gradients of a loss on sigma with respect to
// psi and to the operator blocks, from the sum of Eq. (2)), the slot-sum
// epilogues shared with the forward product, element-wise operand
// conversions and the C entry points of the product.  The forward product
// itself lives in fwd.hip.
//
// d psi = sum alpha L^T G R is the forward product of the adjoint task list
// (fwd.hip's two grouped GEMM phases) on a transposed copy of the operator
// blocks.  The operator-block gradients run in one persistent fused kernel.
// Work item = (operator block, row panel of TQ rows, chunk of the tasks that
// use the block); for every task of its chunk the item computes a chained
// product on chip:
//
//   stage 1   V = X[p0:p0+TQ, :] * M[:, c0:c0+KC]      (K = K1, MFMA)
//   stage 2   acc += alpha V * Y[:, c0:c0+KC]^T          (K = KC, MFMA)
//
// over column chunks c0 of M (the Mode list in tns_internal.hpp gives X, M, Y
// of d L = G R A^T and d R = G^T L A).  The intermediate V stays in LDS and
// the sum over the task chunk in the MFMA accumulators; each item writes its
// panel into its own partial slot and an epilogue adds the slots of every
// block in a fixed order.
#include <algorithm>
#include <mutex>

#include "kern.hpp"
#include "tns_internal.hpp"

namespace tns {

constexpr int KK = 32;    // K1 step of stage 1
constexpr int CMAX = 256; // output columns held in accumulators per pass
constexpr int NWG = 256;  // threads per workgroup (4 waves)

// --- precision traits -------------------------------------------------------
template <int P> struct Prec;

template <> struct Prec<TNS_F64> {
  typedef double elem;   // global operand element
  typedef double acc;    // accumulator element
  typedef d4 accv;
  static constexpr int S = KK + 1;  // LDS row stride (elements) of k-contiguous tiles
};
template <> struct Prec<TNS_F32> {
  typedef float elem;
  typedef float acc;
  typedef f4 accv;
  static constexpr int S = KK + 2;
};

struct ApplyArgs {
  const Item *items;
  int64_t nitems;
  int32_t *queue;        // one counter per work queue
  const int64_t *qbase;  // queue q = items[qbase[q], qbase[q+1])
  int32_t nq;
  const int32_t *idx;    // grouped task indices of the schedule
  const tns_task *tasks;
  const int32_t *psi_sec, *dimL, *dimR;
  const int64_t *psi_off, *blk_off, *slot_off;
  const int32_t *blk_ld, *blk_rows, *blk_cols;
  const void *ops;       // operator values (F64: double*, F32: float*)
  const void *psi;       // psi in the same precision
  const void *grad;      // d loss / d sigma (backward modes), psi layout
  void *partial;         // acc type
  int64_t n_vals, psi_dim;
  int32_t mode_mask;     // bit m set: items of mode m are computed, others skipped
  const void *zero;      // 64 zero bytes: out-of-range loads read here
};

// Next work item of this workgroup: its own XCD's queue first, then the
// others in turn; nitems once every queue is drained.
__device__ inline int pop_item(const ApplyArgs &a) {
  const int home = blockIdx.x % a.nq;
  for (int k = 0; k < a.nq; ++k) {
    const int q = home + k < a.nq ? home + k : home + k - a.nq;
    const int64_t b = a.qbase[q], n = a.qbase[q + 1] - b;
    if (n <= 0) continue;
    const int pos = atomicAdd(a.queue + q, 1);
    if (pos < n) return (int)(b + pos);
  }
  return (int)a.nitems;
}

// Operand view of one matrix for the loaders: element (i, k) at
// base[i * si + k * sk]; identity when `ident`.
struct View {
  const void *p;  // element (0, 0), resolved in the precision of the kernel
  int32_t si, sk; // element (i, k) at p[i * si + k * sk]
  int32_t rows, cols;
  int32_t ident;  // identity operator: (i == k)
  int32_t src;    // 0 = operator values, 1 = psi, 2 = grad sigma
  int64_t off;    // element offset of (0, 0) in its array
};

// The three operands of a task in a mode (see the Mode list in
// tns_internal.hpp) and the dimensions of the mode's output matrix.
struct TaskOps {
  View X, M, Y;
  int K1, K2;
  double alpha;
};

__device__ inline View transposed(View v) {
  View t = v;
  t.rows = v.cols; t.cols = v.rows; t.si = v.sk; t.sk = v.si;
  return t;
}

__device__ inline TaskOps task_ops(const ApplyArgs &a, const tns_task &t, int mode) {
  TaskOps o;
  const int jL = a.psi_sec[4 * t.out], jR = a.psi_sec[4 * t.out + 3];
  const int iL = a.psi_sec[4 * t.in], iR = a.psi_sec[4 * t.in + 3];
  const int q = a.dimL[jL], r = a.dimR[jR], m = a.dimL[iL], n = a.dimR[iR];
  View L, R, A, G;
  L.rows = q; L.cols = m; L.ident = t.lblk < 0; L.src = 0; L.sk = 1;
  L.off = L.ident ? 0 : a.blk_off[t.lblk]; L.si = L.ident ? 0 : a.blk_ld[t.lblk];
  R.rows = r; R.cols = n; R.ident = t.rblk < 0; R.src = 0; R.sk = 1;
  R.off = R.ident ? 0 : a.blk_off[t.rblk]; R.si = R.ident ? 0 : a.blk_ld[t.rblk];
  A.rows = m; A.cols = n; A.off = a.psi_off[t.in]; A.si = n; A.sk = 1; A.ident = 0; A.src = 1;
  G.rows = q; G.cols = r; G.off = a.psi_off[t.out]; G.si = r; G.sk = 1; G.ident = 0; G.src = 2;
  if (mode == M_DL) {
    o.X = G; o.M = R; o.Y = A; o.K1 = r; o.K2 = n;
  } else {  // M_DR
    o.X = transposed(G); o.M = L; o.Y = transposed(A); o.K1 = q; o.K2 = m;
  }
  o.alpha = t.alpha;
  return o;
}

// Rows (panel dimension) and columns of the output matrix of an item: the
// operator block whose gradient it computes.
__device__ inline void out_dims(const ApplyArgs &a, const Item &it, int *rows, int *cols) {
  *rows = a.blk_rows[it.out];
  *cols = a.blk_cols[it.out];
}

// ---------------------------------------------------------------------------
// persistent kernel, FP32 / FP64
//
// Per task and per KC-wide chunk of the middle operand's columns:
//   stage 1: V (TQ x KC) = X[p0.., :] M[:, chunk], K1 stepped by KK;
//   stage 2: acc (TQ x C) += alpha V Y[:, chunk]^T, KC stepped by KS, each
//            stage-2 step staging a KS-wide slice of Y for all C <= CMAX
//            output columns so that every wave updates all its accumulators.
// Every step's global loads go to registers one step ahead (including across
// the stage boundaries and into the next chunk or task), so their latency
// overlaps the MFMA work of the current step; one LDS buffer per tile.
// ---------------------------------------------------------------------------
template <int P> struct K3;
template <> struct K3<TNS_F32> { static constexpr int KK = 32, KC = 64, KS = 4, PAD = 2; };
template <> struct K3<TNS_F64> { static constexpr int KK = 32, KC = 64, KS = 8, PAD = 1; };

// Task operands with element pointers resolved in precision T.
template <class T>
__device__ inline TaskOps task_ops_p(const ApplyArgs &a, const tns_task &t, int mode) {
  TaskOps o = task_ops(a, t, mode);
  View *vs[3] = {&o.X, &o.M, &o.Y};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    View &v = *vs[i];
    const T *b = (const T *)(v.src == 0 ? a.ops : (v.src == 1 ? a.psi : a.grad));
    v.p = b + v.off;
  }
  return o;
}

// Coordinates of thread element j of an R x CC tile walked with the
// memory-contiguous index fastest (CFAST: columns, else rows) across the
// workgroup's threads: element e = tid + NWG * j.
template <int R, int CC, bool CFAST>
__device__ inline void tile_rc(int tid, int j, int *r, int *c) {
  if constexpr (CFAST) {
    static_assert(NWG % CC == 0, "tile width must divide the workgroup");
    *r = tid / CC + j * (NWG / CC);
    *c = tid % CC;
  } else if constexpr (R <= NWG) {
    static_assert(NWG % R == 0, "tile height must divide the workgroup");
    *r = tid % R;
    *c = tid / R + j * (NWG / R);
  } else {
    static_assert(R % NWG == 0, "tile height must be a multiple of the workgroup");
    *r = tid + NWG * (j % (R / NWG));
    *c = j / (R / NWG);
  }
}

// Registers <- tile T(r, c) = v(i0 + r, k0 + c), r < R, c < CC; thread element j
// at tile_rc(tid, j), the memory-contiguous index fastest across
// threads.  KDIM selects the reduction index of the tile (0: r, 1: c): it is
// masked to zero beyond the matrix, while the other index is clamped to the
// last row/column (such values only reach accumulator rows or columns that
// are never written).  Loads are unconditional (no exec-mask branches).
template <class T, int R, int CC, int N, bool CFAST, int KDIM>
__device__ inline void tload(T *reg, const View &v, int i0, int k0, const T *zp) {
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));  // keep per-element offsets in the step (no hoisting)
  const T *p = (const T *)v.p;
  const int si = v.si, sk = v.sk, rmax = v.rows - 1, cmax = v.cols - 1;
  // the identity test is uniform: keep it outside the unrolled loops so that
  // the loads form one straight-line block (issued back to back, one wait)
  if (v.ident) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      int r, c;
      tile_rc<R, CC, CFAST>(tid, j, &r, &c);
      const int i = i0 + r, k = k0 + c;
      reg[j] = (i == k && i <= rmax && k <= cmax) ? T(1) : T(0);
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    int r, c;
    tile_rc<R, CC, CFAST>(tid, j, &r, &c);
    const int i = i0 + r, k = k0 + c;
    const bool in = KDIM == 0 ? (i <= rmax) : (k <= cmax);
    const int ic = KDIM == 0 ? i : min(i, rmax);
    const int kc = KDIM == 1 ? k : min(k, cmax);
    // select the address, not the value: nothing waits on the load here
    reg[j] = *(in ? p + (ic * si + kc * sk) : zp);
  }
}

// LDS <- registers of tload: element (r, c) at [r][c] (TRANS: [c][r]), stride S.
template <class T, int R, int CC, int N, bool CFAST, bool TRANS, int S>
__device__ inline void tstore(T *lds, const T *reg) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    int r, c;
    tile_rc<R, CC, CFAST>(tid, j, &r, &c);
    lds[TRANS ? c * S + r : r * S + c] = reg[j];
  }
}

// Stage-1 B operand of one lane: M(k0 + t, col), t < NT (k0 already holds the
// lane's k-slot group).  K index masked to zero beyond the matrix, column
// clamped; out-of-range elements read the zero region (address select).
template <class T, int NT>
__device__ inline void bload_m(T *reg, const View &v, int k0, int col, const T *zp) {
  int kb = k0;
  asm volatile("" : "+v"(kb));
  const T *p = (const T *)v.p;
  const int kmax = v.rows - 1;
  if (v.ident) {
#pragma unroll
    for (int t = 0; t < NT; ++t) reg[t] = (kb + t == col && kb + t <= kmax && col < v.cols) ? T(1) : T(0);
    return;
  }
  const T *q = p + min(col, v.cols - 1) * v.sk;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int k = kb + t;
    reg[t] = *(k <= kmax ? q + k * v.si : zp);
  }
}

// Stage-2 B operands of one lane for its column tiles u: Y(row0 + 64u,
// c + t), t < NT; Y's column (the K index) masked, rows clamped.
template <class T, int NU_, int NT>
__device__ inline void bload_y(T (*reg)[NT], const View &v, int row0, int c, const T *zp) {
  int cb = c;
  asm volatile("" : "+v"(cb));
  const T *p = (const T *)v.p;
  const int rmax = v.rows - 1, cmax = v.cols - 1;
  if (v.ident) {
#pragma unroll
    for (int u = 0; u < NU_; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        reg[u][t] = (row0 + 64 * u == cb + t && cb + t <= cmax && row0 + 64 * u <= rmax) ? T(1) : T(0);
    return;
  }
#pragma unroll
  for (int u = 0; u < NU_; ++u) {
    const T *q = p + min(row0 + 64 * u, rmax) * v.si;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int k = cb + t;
      reg[u][t] = *(k <= cmax ? q + k * v.sk : zp);
    }
  }
}

template <int P>
__global__ __launch_bounds__(NWG) void k_apply(ApplyArgs a) {
  typedef typename Prec<P>::acc T;
  typedef typename Prec<P>::accv V4;
  constexpr int KK_ = K3<P>::KK, KC_ = K3<P>::KC, KS_ = K3<P>::KS;
  constexpr int SX = KK_ + K3<P>::PAD, SV = KC_ + K3<P>::PAD;
  constexpr int NRT = TQ / 16;
  constexpr int NU = CMAX / 64;
  constexpr int NX = TQ * KK_ / NWG;
  constexpr int TM = KK_ / 4, TY = KS_ / 4;  // MFMA k-steps per stage-1 step / stage-2 slice
  static_assert(TQ % 16 == 0 && TQ <= 128 && KC_ == 64, "stage 1 maps V column tile w to wave w");
  __shared__ T xs[TQ * SX];
  __shared__ T vs[TQ * SV];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  T *part = reinterpret_cast<T *>(a.partial);
  const T *zp = reinterpret_cast<const T *>(a.zero);

  for (;;) {
    if (tid == 0) s_item = pop_item(a);
    __syncthreads();
    const int wi = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (wi >= a.nitems) break;
    const Item it = a.items[wi];
    if (!((a.mode_mask >> it.mode) & 1)) continue;
    int Rtot, Ctot;
    out_dims(a, it, &Rtot, &Ctot);
    T *slot = part + a.slot_off[it.slot];
    const int p0 = it.p0;
    for (int ct0 = 0; ct0 < Ctot; ct0 += CMAX) {
      const int Cn = min(CMAX, Ctot - ct0);
      const int njt = (Cn + 15) >> 4;
      V4 acc[NRT][NU];
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int u = 0; u < NU; ++u) acc[rt][u] = vzero<V4>();
      T xpre[NX];
      T mcur[TM], mnxt[TM];
      T ycur[NU][TY], ynxt[NU][TY];
      const int yrow0 = ct0 + w * 16 + l16;
      auto loadx = [&](const TaskOps &o, int k0) {
        if (o.X.sk == 1 || o.X.ident) tload<T, TQ, KK_, NX, true, 1>(xpre, o.X, p0, k0, zp);
        else tload<T, TQ, KK_, NX, false, 1>(xpre, o.X, p0, k0, zp);
      };
      auto storex = [&](const TaskOps &o) {
        if (o.X.sk == 1 || o.X.ident) tstore<T, TQ, KK_, NX, true, false, SX>(xs, xpre);
        else tstore<T, TQ, KK_, NX, false, false, SX>(xs, xpre);
      };

      int ti = it.tb, c0 = 0;
      TaskOps ops = task_ops_p<T>(a, a.tasks[a.idx[ti]], it.mode);
      loadx(ops, 0);
      bload_m<T, TM>(mcur, ops.M, lg * TM, w * 16 + l16, zp);
      for (;;) {
        // ---- stage 1: V[:, 16w..16w+16) = X M[:, c0 + 16w ..]; X via LDS, M direct --
        V4 vacc[NRT];
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) vacc[rt] = vzero<V4>();
        for (int k0 = 0; k0 < ops.K1; k0 += KK_) {
          __syncthreads();
          storex(ops);
          __syncthreads();
          const bool last1 = k0 + KK_ >= ops.K1;
          if (!last1) {
            loadx(ops, k0 + KK_);
            bload_m<T, TM>(mnxt, ops.M, k0 + KK_ + lg * TM, c0 + w * 16 + l16, zp);
          } else {
            bload_y<T, NU, TY>(ycur, ops.Y, yrow0, c0 + lg * TY, zp);
          }
#pragma unroll
          for (int t = 0; t < TM; ++t) {
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) vacc[rt] = mfma(xs[(rt * 16 + l16) * SX + lg * TM + t], mcur[t], vacc[rt]);
          }
          if (!last1) {
#pragma unroll
            for (int t = 0; t < TM; ++t) mcur[t] = mnxt[t];
          }
        }
        // publish alpha V (wave w: column tile w); the previous chunk's stage-2
        // reads of vs ended before this stage's barriers
        {
          const T al = (T)ops.alpha;
#pragma unroll
          for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) vs[(rt * 16 + mrow(vacc[rt], lg, v)) * SV + w * 16 + l16] = al * vacc[rt][v];
        }
        __syncthreads();
        int nc0 = c0 + KC_, nti = ti;
        if (nc0 >= ops.K2) { nti = ti + 1; nc0 = 0; }
        const bool more = nti < it.te;
        TaskOps nops = ops;
        if (more && nti != ti) nops = task_ops_p<T>(a, a.tasks[a.idx[nti]], it.mode);
        // ---- stage 2: acc += V[:, s2..] Y[:, c0 + s2 ..]^T, Y straight to registers ---
        const int send = min(KC_, ops.K2 - c0);
        for (int s2 = 0; s2 < send; s2 += KS_) {
          const bool last2 = s2 + KS_ >= send;
          if (!last2) {
            bload_y<T, NU, TY>(ynxt, ops.Y, yrow0, c0 + s2 + KS_ + lg * TY, zp);
          } else if (more) {
            loadx(nops, 0);
            bload_m<T, TM>(mcur, nops.M, lg * TM, nc0 + w * 16 + l16, zp);
          }
#pragma unroll
          for (int t = 0; t < TY; ++t) {
            T av[NRT];
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) av[rt] = vs[(rt * 16 + l16) * SV + s2 + lg * TY + t];
#pragma unroll
            for (int u = 0; u < NU; ++u)
              if (w + 4 * u < njt) {
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) acc[rt][u] = mfma(av[rt], ycur[u][t], acc[rt][u]);
              }
          }
          if (!last2) {
#pragma unroll
            for (int u = 0; u < NU; ++u)
#pragma unroll
              for (int t = 0; t < TY; ++t) ycur[u][t] = ynxt[u][t];
          }
        }
        if (!more) break;
        ti = nti;
        c0 = nc0;
        ops = nops;
      }
      // ---- write the panel into the partial slot ---------------------------------
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int jt = w + 4 * u;
          if (jt < njt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = rt * 16 + mrow(acc[rt][u], lg, v);
              const int col = ct0 + jt * 16 + l16;
              if (row < it.np && col < Ctot) {
                slot[(int64_t)(p0 + row) * Ctot + col] = acc[rt][u][v];
              }
            }
          }
        }
      __syncthreads();  // LDS reuse by the next pass / item
    }
  }
}


// ---------------------------------------------------------------------------
// epilogues: add the partial slots of every output in slot order
// ---------------------------------------------------------------------------
// psi-layout outputs (sigma, d psi): sector s owns the chunks of groups
// [gps*s, gps*s + gps) of its schedule.
template <class T>
__global__ void k_epilogue_psi(const int64_t *__restrict__ psi_off, int nS, int gps,
                               const int64_t *__restrict__ grp_chunk_base, const int64_t *__restrict__ slot_off,
                               const T *__restrict__ part, T *__restrict__ out, int64_t psi_dim, int beta,
                               int64_t e0) {
  for (int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < psi_dim;
       e += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = nS;  // s with psi_off[s] <= e < psi_off[s+1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (psi_off[mid] <= e) lo = mid; else hi = mid;
    }
    const int s = lo;
    const int64_t loc = e - psi_off[s];
    double acc = beta ? (double)out[e] : 0.0;
    const int64_t c0 = grp_chunk_base[gps * s], c1 = grp_chunk_base[gps * s + gps];
    // eight slots' loads in flight at a time, added in slot order
    for (int64_t c = c0; c < c1; c += 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = c + u < c1 ? part[slot_off[c + u] + loc] : T(0);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c + u < c1) acc += (double)v[u];
    }
    out[e] = (T)acc;
  }
}

// operator-block outputs (d L, d R): one workgroup per block, group nS + b.
template <class T>
__global__ void k_epilogue_blk(int nS, const int64_t *__restrict__ grp_chunk_base,
                               const int64_t *__restrict__ slot_off, const int64_t *__restrict__ blk_off,
                               const int32_t *__restrict__ blk_rows, const int32_t *__restrict__ blk_cols,
                               const int32_t *__restrict__ blk_ld, const T *__restrict__ part, T *__restrict__ out) {
  const int b = blockIdx.x;
  const int64_t c0 = grp_chunk_base[nS + b], c1 = grp_chunk_base[nS + b + 1];
  if (c0 == c1) return;  // unused block: stays zero
  const int rows = blk_rows[b], cols = blk_cols[b], ld = blk_ld[b];
  const int n = rows * cols;  // a block holds fewer than 2^31 elements
  T *o = out + blk_off[b];
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    double acc = 0.0;
    for (int64_t c = c0; c < c1; ++c) acc += (double)part[slot_off[c] + e];
    const int r = e / cols;
    o[(int64_t)r * ld + (e - r * cols)] = (T)acc;
  }
}

// queue counters (bytes 0..63) and the 64-byte zero region that out-of-range
// loads read (bytes 64..127)
__global__ void k_reset_head(int32_t *p) {
  if (threadIdx.x < 32) p[threadIdx.x] = 0;
}

template <class T>
__global__ void k_zero(T *p, int64_t n) {
  GRID_STRIDE(i, n) p[i] = T(0);
}

// BF16X3 operands: hi = bf16(x), lo = bf16(x - hi), interleaved (bfx_hi).
__global__ void k_split_f64(const double *__restrict__ x, int64_t n, uint16_t *__restrict__ out) {
  GRID_STRIDE(i, n) {
    const float v = (float)x[i];
    const uint16_t h = f32_to_bf16_rne(v);
    out[bfx_hi(i)] = h;
    out[bfx_hi(i) + 8] = f32_to_bf16_rne(v - bf16_to_f32(h));
  }
}

__global__ void k_f64_to_f32(const double *__restrict__ x, int64_t n, float *__restrict__ y) {
  GRID_STRIDE(i, n) y[i] = (float)x[i];
}

__global__ void k_copy_f64(const double *__restrict__ x, int64_t n, double *__restrict__ y) {
  GRID_STRIDE(i, n) y[i] = x[i];
}

// Blocks for an element-wise launch over n elements (capped; kernels stride).
static inline unsigned nb(int64_t n, int b) {
  const int64_t g = (n + b - 1) / b;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 16));
}

static size_t elem_bytes(tns_prec p) { return p == TNS_F64 ? 8 : 4; }

// Workspace of k_apply (FP64 / FP32): [queue counter | partial slots]
static size_t apply_ws(const Sched &S, tns_prec prec) {
  return 256 + align_up((size_t)std::max<int64_t>(S.partial_elems, 1) * elem_bytes(prec), 256);
}

template <class K>
static int grid_for(K kern, int n_cu) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, NWG, 0) != hipSuccess || per <= 0) per = 1;
  return per * n_cu;
}

static ApplyArgs make_args(const Plan &p, const Sched &S, const void *ops, const void *psi, const void *grad,
                           void *part, int32_t *queue) {
  ApplyArgs a;
  a.items = S.items; a.nitems = S.nitems; a.queue = queue; a.idx = S.idx; a.tasks = p.tasks;
  a.qbase = S.qbase; a.nq = S.nq;
  a.psi_sec = p.psi_sec; a.dimL = p.dimL; a.dimR = p.dimR; a.psi_off = p.psi_off; a.blk_off = p.blk_off;
  a.slot_off = S.slot_off; a.blk_ld = p.blk_ld; a.blk_rows = p.blk_rows; a.blk_cols = p.blk_cols;
  a.ops = ops; a.psi = psi; a.grad = grad; a.partial = part;
  a.n_vals = p.n_vals; a.psi_dim = p.psi_dim;
  a.mode_mask = 0x1f;
  a.zero = reinterpret_cast<const char *>(queue) + 64;
  return a;
}

static hipEvent_t g_ev_before = nullptr, g_ev_mid = nullptr, g_ev_after = nullptr;

bool take_profile_events(hipEvent_t ev[3]) {
  ev[0] = g_ev_before; ev[1] = g_ev_mid; ev[2] = g_ev_after;
  g_ev_before = g_ev_mid = g_ev_after = nullptr;
  return ev[0] && ev[1] && ev[2];
}

tns_status launch_epilogue_psi(const Plan &p, bool f64, const void *part, void *sigma, int beta, hipStream_t st) {
  const Sched &S = p.fwd;
  if (p.psi_dim <= p.epi_e0) return TNS_OK;
  const unsigned g = nb(p.psi_dim - p.epi_e0, 256);
  if (f64)
    hipLaunchKernelGGL(k_epilogue_psi<double>, dim3(g), dim3(256), 0, st, p.psi_off, p.nS, 2, S.grp_chunk_base,
                       S.slot_off, (const double *)part, (double *)sigma, p.psi_dim, beta, p.epi_e0);
  else
    hipLaunchKernelGGL(k_epilogue_psi<float>, dim3(g), dim3(256), 0, st, p.psi_off, p.nS, 2, S.grp_chunk_base,
                       S.slot_off, (const float *)part, (float *)sigma, p.psi_dim, beta, p.epi_e0);
  return hipGetLastError() == hipSuccess ? TNS_OK : TNS_ERR_HIP;
}

tns_status apply_impl(const Plan &p, tns_prec prec, const void *ops, const void *psi, void *sigma, double beta,
                      void *ws, size_t ws_bytes, hipStream_t st) {
  hipEvent_t ev[3];
  const bool timed = take_profile_events(ev);
  return fwd_apply(p, prec, ops, psi, sigma, beta, ws, ws_bytes, st, timed ? ev : nullptr);
}

// Operator values transposed block by block: block b (rows x cols, leading
// dimension bld[b], at boff[b]) becomes a cols x ld8(rows) row-major matrix at
// toff[b], its padding columns zero.  32 x 32 tiles through LDS, so that
// both the reads and the writes are row-contiguous; the gridDim.y workgroups
// of a block take every gridDim.y-th row of tiles.
template <class T>
__global__ __launch_bounds__(256) void k_transpose_blocks(const T *__restrict__ src, const int64_t *__restrict__ boff,
                                                          const int32_t *__restrict__ bld,
                                                          const int32_t *__restrict__ rows,
                                                          const int32_t *__restrict__ cols,
                                                          const int64_t *__restrict__ toff, T *__restrict__ dst,
                                                          int nblk) {
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int R = rows[b], C = cols[b], ld = bld[b], tl = ld8(R);
    const T *s = src + boff[b];
    T *d = dst + toff[b];
    for (int r0 = 32 * blockIdx.y; r0 < tl; r0 += 32 * gridDim.y)
      for (int c0 = 0; c0 < C; c0 += 32) {
        for (int i = ty; i < 32; i += 8) {
          const int r = r0 + i, c = c0 + tx;
          tile[i][tx] = (r < R && c < C) ? s[(int64_t)r * ld + c] : T(0);
        }
        __syncthreads();
        for (int i = ty; i < 32; i += 8) {
          const int c = c0 + i, r = r0 + tx;
          if (c < C && r < tl) d[(int64_t)c * tl + r] = tile[tx][i];
        }
        __syncthreads();
      }
  }
}

// Backward workspace: [k_apply: queue counter | partial slots of the
// operator-gradient schedule] [transposed operator values] [workspace of the
// adjoint forward product].
static size_t bwd_transposed_at(const Plan &p, tns_prec prec) { return apply_ws(p.bwd, prec); }
static size_t bwd_fwd_at(const Plan &p, tns_prec prec) {
  return bwd_transposed_at(p, prec) +
         align_up((size_t)std::max<int64_t>(p.adj.n_vals, 1) * elem_bytes(prec), 256);
}
static size_t bwd_workspace(const Plan &p, tns_prec prec) {
  return bwd_fwd_at(p, prec) + fwd_workspace(adjoint_plan(p), prec);
}

// d psi = sum alpha L^T G R is the forward product of the adjoint task list on
// the transposed blocks (two grouped GEMM phases); the operator gradients
// run in the fused kernel k_apply.
template <int P>
static tns_status backward_impl(const Plan &p, const void *ops, const void *psi, const void *G, void *gpsi,
                                void *gops, void *ws, hipStream_t st) {
  typedef typename Prec<P>::acc T;
  const Sched &S = p.bwd;
  char *w = reinterpret_cast<char *>(ws);
  if (gops) {
    int32_t *queue = reinterpret_cast<int32_t *>(w);
    T *part = reinterpret_cast<T *>(w + 256);
    ApplyArgs a = make_args(p, S, ops, psi, G, part, queue);
    a.mode_mask = (1 << M_DL) | (1 << M_DR);
    hipLaunchKernelGGL(k_reset_head, dim3(1), dim3(32), 0, st, queue);
    if (S.nitems > 0) hipLaunchKernelGGL(k_apply<P>, dim3(grid_for(k_apply<P>, p.n_cu)), dim3(NWG), 0, st, a);
    hipLaunchKernelGGL(k_zero<T>, dim3(nb(p.n_vals, 256)), dim3(256), 0, st, (T *)gops, p.n_vals);
    if (p.nBlk > 0)
      hipLaunchKernelGGL(k_epilogue_blk<T>, dim3(p.nBlk), dim3(256), 0, st, p.nS, S.grp_chunk_base, S.slot_off,
                         p.blk_off, p.blk_rows, p.blk_cols, p.blk_ld, (const T *)part, (T *)gops);
    TNS_HIP(hipGetLastError());
  }
  if (gpsi) {
    const tns_prec prec = (tns_prec)P;
    const Plan q = adjoint_plan(p);
    T *opsT = reinterpret_cast<T *>(w + bwd_transposed_at(p, prec));
    if (p.nBlk > 0)
      hipLaunchKernelGGL(k_transpose_blocks<T>, dim3(std::min(p.nBlk, 1 << 16), 8), dim3(256), 0, st,
                         (const T *)ops, p.blk_off, p.blk_ld, p.blk_rows, p.blk_cols, q.blk_off, opsT, p.nBlk);
    TNS_HIP(hipGetLastError());
    char *wf = w + bwd_fwd_at(p, prec);
    const tns_status s = fwd_apply(q, prec, opsT, G, gpsi, 0.0, wf, fwd_workspace(q, prec), st, nullptr);
    if (s != TNS_OK) return s;
  }
  return hipGetLastError() == hipSuccess ? TNS_OK : TNS_ERR_HIP;
}

}  // namespace tns

using namespace tns;

extern "C" size_t tns_apply_workspace_bytes(const tns_tasklist *tl, tns_prec prec) {
  if (!tl || (prec != TNS_F64 && prec != TNS_F32 && prec != TNS_BF16X3)) return 0;
  return fwd_workspace(plan_of(tl), prec);
}

extern "C" tns_status tns_prepare_operands(tns_prec prec, const double *vals64, int64_t n, void *out, hipStream_t st) {
  if (!vals64 || !out || n < 0) return TNS_ERR_ARG;
  if (n == 0) return TNS_OK;
  if (prec == TNS_F64) {
    hipLaunchKernelGGL(k_copy_f64, dim3(nb(n, 256)), dim3(256), 0, st, vals64, n, (double *)out);
  } else if (prec == TNS_F32) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(nb(n, 256)), dim3(256), 0, st, vals64, n, (float *)out);
  } else if (prec == TNS_BF16X3) {
    hipLaunchKernelGGL(k_split_f64, dim3(nb(n, 256)), dim3(256), 0, st, vals64, n, (uint16_t *)out);
  } else {
    return TNS_ERR_ARG;
  }
  return hipGetLastError() == hipSuccess ? TNS_OK : TNS_ERR_HIP;
}

extern "C" tns_status tns_apply_heff(const tns_tasklist *tl, tns_prec prec, const void *op_vals, const void *psi,
                                     void *sigma, double beta, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!tl || !op_vals || !psi || !sigma || !ws) return TNS_ERR_ARG;
  if (prec != TNS_F64 && prec != TNS_F32 && prec != TNS_BF16X3) return TNS_ERR_ARG;
  if (beta != 0.0 && beta != 1.0) return TNS_ERR_ARG;
  return apply_impl(plan_of(tl), prec, op_vals, psi, sigma, beta, ws, ws_bytes, st);
}

// --- the allocation-free product ----------------------------------------------
// Device array that stands in for the caller's workspace in
// tns_apply_heff_noalloc.  Each device holds its own copy, at its own address,
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host the name is a stand-in, not a device address): it
// passes the address hipGetSymbolAddress returns for the device.
static __device__ __align__(256) uint8_t scratch[TNS_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on the stream's device, looked up once per
// device with that device current.
static tns_status scratch_for(hipStream_t st, void **out) {
  int dev = -1, cur = -1;
  TNS_HIP(hipGetDevice(&cur));
  TNS_HIP(hipStreamGetDevice(st, &dev));
  if (dev < 0 || dev >= MAX_DEVICES) return TNS_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    if (dev != cur) TNS_HIP(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) TNS_HIP(hipSetDevice(cur));
    if (e != hipSuccess || !p) return TNS_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TNS_OK;
}

extern "C" tns_status tns_apply_heff_noalloc(const tns_tasklist *tl, tns_prec prec, const void *op_vals,
                                             const void *psi, void *sigma, double beta, hipStream_t st) {
  if (!tl || !op_vals || !psi || !sigma) return TNS_ERR_ARG;
  if (prec != TNS_F64 && prec != TNS_F32 && prec != TNS_BF16X3) return TNS_ERR_ARG;
  if (beta != 0.0 && beta != 1.0) return TNS_ERR_ARG;
  const Plan &p = plan_of(tl);
  if (fwd_workspace(p, prec) > TNS_NOALLOC_SCRATCH_BYTES) return TNS_ERR_WORKSPACE;
  void *ws = nullptr;
  const tns_status s = scratch_for(st, &ws);
  if (s != TNS_OK) return s;
  // the product clears what must start at zero (queue counters, the zero
  // region) with a kernel and writes every other byte it reads
  return apply_impl(p, prec, op_vals, psi, sigma, beta, ws, TNS_NOALLOC_SCRATCH_BYTES, st);
}

extern "C" void tns_profile_events(hipEvent_t before, hipEvent_t mid, hipEvent_t after) {
  g_ev_before = before;
  g_ev_mid = mid;
  g_ev_after = after;
}

extern "C" size_t tns_backward_workspace_bytes(const tns_tasklist *tl, tns_prec prec) {
  if (!tl || (prec != TNS_F64 && prec != TNS_F32) || plan_of(tl).no_backward) return 0;
  return bwd_workspace(plan_of(tl), prec);
}

extern "C" tns_status tns_apply_heff_backward(const tns_tasklist *tl, tns_prec prec, const void *op_vals,
                                              const void *psi, const void *grad_sigma, void *grad_psi,
                                              void *grad_ops, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!tl || !op_vals || !psi || !grad_sigma || !ws) return TNS_ERR_ARG;
  if (prec != TNS_F64 && prec != TNS_F32) return TNS_ERR_ARG;
  const Plan &p = plan_of(tl);
  if (p.no_backward) return TNS_ERR_ARG;
  if (ws_bytes < bwd_workspace(p, prec)) return TNS_ERR_WORKSPACE;
  if (!grad_psi && !grad_ops) return TNS_OK;
  if (prec == TNS_F64) return backward_impl<TNS_F64>(p, op_vals, psi, grad_sigma, grad_psi, grad_ops, ws, st);
  return backward_impl<TNS_F32>(p, op_vals, psi, grad_sigma, grad_psi, grad_ops, ws, st);
}
