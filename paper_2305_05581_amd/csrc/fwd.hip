// sigma = H_eff psi (the sum of Eq. (2), level 3 of the hierarchy of
// Section III.A.1) as two grouped GEMM phases on MFMA.
//
// Task k of output sector s' (input sector s, left block L_k, right block R_k,
// alpha_k = coefficient x Jordan-Wigner sign) contributes
//   class 0:   sigma_s'   += alpha_k (L_k A_s) R_k^T
//   class 1:   sigma_s'^T += alpha_k (R_k A_s^T) L_k^T
// (the cheaper association of the two, chosen when the task list is built).
//
// Phase A forms the intermediate of every task,
//   T_k = alpha_k X_k M_k      (class 0: X = L, M = A;  class 1: X = R, M = A^T),
// in 128 x 128 output tiles and stores it, row-major with leading dimension
// ld8(K2), in the workspace.  Phase B forms, per chunk of the task list of an
// output group,
//   slot = sum_k T_k Y_k^T     (class 0: Y = R;  class 1: Y = L)
// as one GEMM whose inner dimension runs through all tasks of the chunk, in
// 128 x 128 tiles of the group's output.  The epilogue adds the slots of each
// sector in a fixed order.  This is the batched-GEMM arrangement of Alg. 2
// (intermediates in device memory, one batched product per stage) with the
// summation over terms folded into the inner dimension of the second GEMM.
//
// Both phases run one kernel: C(i, j) = sum over segments of
// sum_k A(i, k) B(j, k) with every operand k-contiguous (rows of L, R, T and
// of the padded copies of A and A^T), staged global -> registers -> LDS with
// 16-byte loads and a double-buffered LDS pipeline, one barrier per K step.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "kern.hpp"
#include "tns_internal.hpp"

namespace tns {

constexpr int GTH = 256;  // threads per workgroup: 4 waves in a 2 x 2 grid of 64 x 64 wave tiles

// Operand: element (i, k) at p[i * ld + k] for i < rows, k < K of the
// segment; identity (i == k) when `ident`.  BF16X3: p is the high half, the
// low half lies `lo` elements further.
struct Mat {
  const void *p;
  int64_t lo;
  int32_t ld, rows, ident;
};

// Read of schedule / task metadata that no kernel of the product writes:
// through the constant address space, so that uniform reads become scalar
// loads (they do not count against the vector-memory loads in flight).
template <class T>
__device__ inline T cld(const T *p) {
  return *(const __attribute__((address_space(4))) T *)p;
}

// The fields of a work item the product kernels use, through cld.
__device__ inline Item load_item(const Item *p) {
  Item it;
  it.grp = cld(&p->grp); it.mode = cld(&p->mode); it.p0 = cld(&p->p0); it.np = cld(&p->np);
  it.tb = cld(&p->tb); it.te = cld(&p->te); it.slot = cld(&p->slot); it.out = cld(&p->out);
  it.c0 = cld(&p->c0); it.nc = cld(&p->nc); it.cost = 0;
  return it;
}

struct FwdArgs {
  const tns_task *tasks;
  int64_t ntasks;
  const int32_t *psi_sec, *dimL, *dimR;
  const int64_t *blk_off;
  const int32_t *blk_ld;
  const void *ops;  // F64 / F32 values, or BF16 hi[n] then lo at ld8-aligned offset
  int64_t ops_lo;   // element offset of the low half (BF16X3)
  const void *pp, *pt;  // padded psi (m x ld8(n)) and psi^T (n x ld8(m)) per sector
  int64_t pp_lo, pt_lo;
  const int64_t *pp_off, *pt_off;
  void *T;  // intermediates
  int64_t T_lo;
  const int64_t *t_off;
  // phase B schedule
  const Item *items;
  int64_t nitems;
  const int32_t *idx, *grp_rows, *grp_cols;
  const int64_t *slot_off, *qbase;
  void *partial;
  int32_t *queue;  // [0, 8): phase A queues, [8, 16): phase B queues
  int32_t nq;
  const void *zero;  // 64 zero bytes
  const void *ident;  // BF16X3: identity matrix maxdim x ld8(maxdim) (hi; lo `ident_lo` further)
  int64_t ident_lo;
  int32_t ident_ld;
  uint32_t tiles;     // tile table (phase A picks a task's tile from its T dimensions)
};

// --- per-precision tile parameters ---------------------------------------------
template <int P> struct FP;
template <> struct FP<TNS_F64> {
  typedef double Acc;
  typedef double E;  // element in memory and LDS
  typedef d2 V;      // 16-byte vector
  typedef d4 A4;     // MFMA accumulator
  static constexpr int BK = 16, VEC = 2, LDK = BK + 2;
};
template <> struct FP<TNS_F32> {
  typedef float Acc;
  typedef float E;
  typedef f4 V;
  typedef f4 A4;
  static constexpr int BK = 32, VEC = 4, LDK = BK + 4;
};
template <> struct FP<TNS_BF16X3> {
  typedef float Acc;
  typedef uint16_t E;
  typedef u16x8 V;
  typedef f4 A4;
  static constexpr int BK = 32, VEC = 8, LDK = BK + 8;
};

template <int P> struct __attribute__((aligned(16))) FwdSmem {
  typedef typename FP<P>::E E;
  static constexpr int NH = P == TNS_BF16X3 ? 2 : 1;  // halves per operand
  E a[2][NH][GM * FP<P>::LDK];
  E b[2][NH][GN * FP<P>::LDK];
};

// --- register-staged path (FP64, FP32): operand loads -----------------------------
// A tile has 32 NT rows (NT = 1, 2, 4 MFMA tiles per wave along it).  Thread t
// stages the vectors (row t / NV + j * RP, k-vector t % NV), j < 32 NT / RP.
template <int P> struct Stage {
  static constexpr int NV = FP<P>::BK / FP<P>::VEC;
  static constexpr int RP = GTH / NV;
  static constexpr int NL = GM / RP;
  typename FP<P>::V r[NL];
};

template <int P, int NT>
__device__ inline void stage_load(Stage<P> &s, const Mat &m, int r0, int k0, int K, const void *zero) {
  typedef typename FP<P>::E E;
  typedef typename FP<P>::V V;
  constexpr int NV = Stage<P>::NV, RP = Stage<P>::RP, VEC = FP<P>::VEC, NLX = 32 * NT / RP;
  static_assert(NLX >= 1 && 32 * NT % RP == 0, "tile rows cover whole load passes");
  if (m.ident) return;
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  const int kk = k0 + (t % NV) * VEC;
  const E *base = reinterpret_cast<const E *>(m.p);
#pragma unroll
  for (int j = 0; j < NLX; ++j) {
    const int row = r0 + t / NV + j * RP;
    const bool in = row < m.rows && kk < K;
    const E *ad = in ? base + (int64_t)row * m.ld + kk : reinterpret_cast<const E *>(zero);
    s.r[j] = *reinterpret_cast<const V *>(ad);
  }
}

template <int P, int NT>
__device__ inline void stage_store(typename FP<P>::E *lds, Stage<P> &s, const Mat &m, int r0, int k0, int K) {
  typedef typename FP<P>::E E;
  typedef typename FP<P>::V V;
  constexpr int NV = Stage<P>::NV, RP = Stage<P>::RP, VEC = FP<P>::VEC, LDK = FP<P>::LDK, NLX = 32 * NT / RP;
  const int t = threadIdx.x;
  const int kv = (t % NV) * VEC, kk = k0 + kv;
#pragma unroll
  for (int j = 0; j < NLX; ++j) {
    const int lrow = t / NV + j * RP, row = r0 + lrow;
    V h;
    if (m.ident) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) h[e] = (row == kk + e && row < m.rows && kk + e < K) ? E(1) : E(0);
    } else {
      h = s.r[j];
      if (kk + VEC > K) {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (kk + e >= K) h[e] = 0;
      }
    }
    *reinterpret_cast<V *>(&lds[lrow * LDK + kv]) = h;
  }
}

// --- MFMA on one LDS stage ------------------------------------------------------
// Wave tile (16 TM) x (16 TN) at (wm, wn); acc[i][j] is the 16 x 16 tile
// (16 i, 16 j) of it.  Lane group g = lane / 16 owns k in [g BK/4, (g+1) BK/4).
template <int P, int TM, int TN>
__device__ inline void stage_mma(const FwdSmem<P> &sm, int buf, typename FP<P>::A4 (&acc)[4][4]) {
  typedef typename FP<P>::E E;
  typedef typename FP<P>::V V;
  constexpr int LDK = FP<P>::LDK, BK = FP<P>::BK, VEC = FP<P>::VEC, KG = BK / 4;  // k per lane group
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1, l16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int h = 0; h < KG / VEC; ++h) {
    V a[TM], b[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
      a[i] = *reinterpret_cast<const V *>(&sm.a[buf][0][(wm * 16 * TM + i * 16 + l16) * LDK + g * KG + h * VEC]);
#pragma unroll
    for (int j = 0; j < TN; ++j)
      b[j] = *reinterpret_cast<const V *>(&sm.b[buf][0][(wn * 16 * TN + j * 16 + l16) * LDK + g * KG + h * VEC]);
#pragma unroll
    for (int e = 0; e < VEC; ++e)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mfma((E)a[i][e], (E)b[j][e], acc[i][j]);
  }
}

// --- segment operands -------------------------------------------------------------
template <int P>
__device__ inline Mat op_mat(const FwdArgs &g, int blk, int rows) {
  typedef typename FP<P>::E E;
  Mat m;
  m.rows = rows;
  m.lo = g.ops_lo;
  if (P == TNS_BF16X3 && blk < 0) {  // the identity as a matrix in memory
    m.p = g.ident; m.lo = g.ident_lo; m.ld = g.ident_ld; m.ident = 0;
  } else if (blk < 0) {
    m.p = g.zero; m.ld = 0; m.ident = 1;
  } else {
    m.p = reinterpret_cast<const E *>(g.ops) + cld(&g.blk_off[blk]);
    m.ld = cld(&g.blk_ld[blk]);
    m.ident = 0;
  }
  return m;
}

// Operands (A, B) and inner dimension K of task t in phase PH.
template <int P, int PH>
__device__ inline void seg_ops(const FwdArgs &g, int t, Mat &A, Mat &B, int &K, double *alpha) {
  typedef typename FP<P>::E E;
  t = __builtin_amdgcn_readfirstlane(t);  // uniform: scalar loads of the task record
  const tns_task *tp = g.tasks + t;
  const int out = cld(&tp->out), in = cld(&tp->in), order = cld(&tp->order);
  const int lblk = cld(&tp->lblk), rblk = cld(&tp->rblk);
  const int *so = g.psi_sec + 4 * out, *si = g.psi_sec + 4 * in;
  const int q = cld(&g.dimL[cld(&so[0])]), r = cld(&g.dimR[cld(&so[3])]);
  const int m = cld(&g.dimL[cld(&si[0])]), n = cld(&g.dimR[cld(&si[3])]);
  if (alpha) *alpha = cld(&tp->alpha);
  if (PH == 0) {
    if (order == 0) {  // T = L A: B(j, k) = A(k, j) = A^T(j, k)
      K = m;
      A = op_mat<P>(g, lblk, q);
      B.p = reinterpret_cast<const E *>(g.pt) + cld(&g.pt_off[in]);
      B.lo = g.pt_lo; B.ld = ld8(m); B.rows = n; B.ident = 0;
    } else {           // T = R A^T: B(j, k) = A(j, k)
      K = n;
      A = op_mat<P>(g, rblk, r);
      B.p = reinterpret_cast<const E *>(g.pp) + cld(&g.pp_off[in]);
      B.lo = g.pp_lo; B.ld = ld8(n); B.rows = m; B.ident = 0;
    }
  } else {
    const int k2 = order == 0 ? n : m;
    K = k2;
    A.p = reinterpret_cast<const E *>(g.T) + cld(&g.t_off[t]);
    A.lo = g.T_lo; A.ld = ld8(k2); A.rows = order == 0 ? q : r; A.ident = 0;
    B = order == 0 ? op_mat<P>(g, rblk, r) : op_mat<P>(g, lblk, q);
  }
}

// --- work queues --------------------------------------------------------------------
// Phase A: tasks in blocks of 4 consecutive ones, block b on queue b mod nq.
__device__ inline int64_t qa_count(int64_t ntasks, int nq, int q) {
  const int64_t per = 4 * (int64_t)nq, full = ntasks / per;
  const int64_t rest = ntasks - full * per - 4 * (int64_t)q;
  return full * 4 + (rest < 0 ? 0 : (rest > 4 ? 4 : rest));
}
__device__ inline int64_t qa_task(int nq, int q, int64_t j) { return (j / 4) * 4 * nq + 4 * q + (j % 4); }

template <int PH>
__device__ inline int pop_work(const FwdArgs &g) {
  const int home = blockIdx.x % g.nq;
  for (int k = 0; k < g.nq; ++k) {
    const int q = home + k < g.nq ? home + k : home + k - g.nq;
    if (PH == 0) {
      const int64_t n = qa_count(g.ntasks, g.nq, q);
      if (n <= 0) continue;
      const int j = atomicAdd(g.queue + q, 1);
      if (j < n) return (int)qa_task(g.nq, q, j);
    } else {
      const int64_t b = g.qbase[q], n = g.qbase[q + 1] - b;
      if (n <= 0) continue;
      const int j = atomicAdd(g.queue + 8 + q, 1);
      if (j < n) return (int)(b + j);
    }
  }
  return -1;
}

// --- the register-staged kernel ---------------------------------------------------------
// One output tile of (32 TM) x (32 TN): acc = sum over segments [sb, se) of
// A_seg B_seg^T on rows [r0, r0 + 32 TM) of A and [c0, c0 + 32 TN) of B.
template <int P, int PH, int TM, int TN>
__device__ inline void tile_gemm(const FwdArgs &g, FwdSmem<P> &sm, int sb, int se, int r0, int c0,
                                 typename FP<P>::A4 (&acc)[4][4]) {
  typedef typename FP<P>::A4 A4;
  constexpr int BK = FP<P>::BK;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = vzero<A4>();
  auto seg_task = [&](int s) { return PH == 0 ? s : cld(&g.idx[s]); };
  Mat A, B;
  int K;
  seg_ops<P, PH>(g, seg_task(sb), A, B, K, nullptr);
  Stage<P> sa, sb_;
  stage_load<P, TM>(sa, A, r0, 0, K, g.zero);
  stage_load<P, TN>(sb_, B, c0, 0, K, g.zero);
  stage_store<P, TM>(sm.a[0][0], sa, A, r0, 0, K);
  stage_store<P, TN>(sm.b[0][0], sb_, B, c0, 0, K);
  __syncthreads();
  int s = sb, k0 = 0, cur = 0;
  for (;;) {
    int ns = s, nk = k0 + BK, nK = K;
    Mat nA = A, nB = B;
    if (nk >= K) {
      ns = s + 1;
      nk = 0;
      if (ns < se) seg_ops<P, PH>(g, seg_task(ns), nA, nB, nK, nullptr);
    }
    const bool more = ns < se;
    if (more) {
      stage_load<P, TM>(sa, nA, r0, nk, nK, g.zero);
      stage_load<P, TN>(sb_, nB, c0, nk, nK, g.zero);
    }
    stage_mma<P, TM, TN>(sm, cur, acc);
    if (more) {
      stage_store<P, TM>(sm.a[cur ^ 1][0], sa, nA, r0, nk, nK);
      stage_store<P, TN>(sm.b[cur ^ 1][0], sb_, nB, c0, nk, nK);
    }
    __syncthreads();
    if (!more) break;
    cur ^= 1;
    s = ns;
    k0 = nk;
    K = nK;
    A = nA;
    B = nB;
  }
}

// Phase A, task t: every (32 TM) x (32 TN) tile of T_t, row strips in turn.
template <int P, int TM, int TN>
__device__ inline void phase_a_task(const FwdArgs &g, FwdSmem<P> &sm, int t) {
  typedef typename FP<P>::A4 A4;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1, l16 = lane & 15, lg = lane >> 4;
  Mat A, B;
  int K;
  double alpha;
  seg_ops<P, 0>(g, t, A, B, K, &alpha);
  const int rows = A.rows, cols = B.rows, ld = ld8(cols);
  typedef typename FP<P>::Acc Acc;
  Acc *Tt = reinterpret_cast<Acc *>(g.T) + cld(&g.t_off[t]);
  const Acc alf = (Acc)alpha;
  A4 acc[4][4];
  for (int r0 = 0; r0 < rows; r0 += 32 * TM)
    for (int c0 = 0; c0 < cols; c0 += 32 * TN) {
      tile_gemm<P, 0, TM, TN>(g, sm, t, t + 1, r0, c0, acc);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int col = c0 + wn * 16 * TN + j * 16 + l16;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = r0 + wm * 16 * TM + i * 16 + mrow(acc[i][j], lg, v);
            if (row < rows && col < ld) Tt[(int64_t)row * ld + col] = alf * acc[i][j][v];
          }
        }
    }
}

// Phase B, one item: its (32 TM) x (32 TN) output tile over its chunk of tasks.
template <int P, int TM, int TN>
__device__ inline void phase_b_item(const FwdArgs &g, FwdSmem<P> &sm, const Item &it, int mode) {
  typedef typename FP<P>::A4 A4;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1, l16 = lane & 15, lg = lane >> 4;
  A4 acc[4][4];
  tile_gemm<P, 1, TM, TN>(g, sm, it.tb, it.te, it.p0, it.c0, acc);
  const int R = cld(&g.grp_rows[it.grp]), C = cld(&g.grp_cols[it.grp]);
  typename FP<P>::Acc *slot = reinterpret_cast<typename FP<P>::Acc *>(g.partial) + cld(&g.slot_off[it.slot]);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = it.c0 + wn * 16 * TN + j * 16 + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = it.p0 + wm * 16 * TM + i * 16 + mrow(acc[i][j], lg, v);
        if (row < R && col < C) {
          const int64_t o = mode == M_FWD1 ? ((int64_t)col * R + row) : ((int64_t)row * C + col);
          slot[o] = acc[i][j][v];
        }
      }
    }
}

// Runs F<TM, TN> for tile extents (32 tm) x (32 tn), tm, tn in {1, 2, 4}.
#define TNS_TILE_SWITCH(tm, tn, CALL)                  \
  switch ((tm) * 8 + (tn)) {                             \
    case 9: CALL(1, 1); break;                           \
    case 10: CALL(1, 2); break;                          \
    case 12: CALL(1, 4); break;                          \
    case 17: CALL(2, 1); break;                          \
    case 18: CALL(2, 2); break;                          \
    case 20: CALL(2, 4); break;                          \
    case 33: CALL(4, 1); break;                          \
    case 34: CALL(4, 2); break;                          \
    default: CALL(4, 4); break;                          \
  }

// One work item of the register-staged path: phase A = all tiles of task
// wk, phase B = item wk of the phase-B schedule.
template <int P, int PH>
__device__ inline void fwd_item(const FwdArgs &g, FwdSmem<P> &sm, int wk) {
  if (PH == 0) {
    const tns_task *tp = g.tasks + wk;
    const int out = cld(&tp->out), in = cld(&tp->in), order = cld(&tp->order);
    const int rows = order == 0 ? cld(&g.dimL[cld(&g.psi_sec[4 * out])]) : cld(&g.dimR[cld(&g.psi_sec[4 * out + 3])]);
    const int cols = order == 0 ? cld(&g.dimR[cld(&g.psi_sec[4 * in + 3])]) : cld(&g.dimL[cld(&g.psi_sec[4 * in])]);
    const int tm = tile_ext(g.tiles, rows) / 32, tn = tile_ext(g.tiles, cols) / 32;
#define TNS_CALL_A(a, b) phase_a_task<P, a, b>(g, sm, wk)
    TNS_TILE_SWITCH(tm, tn, TNS_CALL_A)
#undef TNS_CALL_A
  } else {
    const Item it = load_item(g.items + wk);
    const int mode = it.mode & 0xff, tm = (it.mode >> 8) & 0xff, tn = (it.mode >> 16) & 0xff;
#define TNS_CALL_B(a, b) phase_b_item<P, a, b>(g, sm, it, mode)
    TNS_TILE_SWITCH(tm, tn, TNS_CALL_B)
#undef TNS_CALL_B
  }
}

// FP32: two workgroups per CU (the register budget of 256 per lane)
template <int P, int PH>
__global__ __launch_bounds__(GTH, P == TNS_F32 ? 2 : 1) void k_fwd(FwdArgs g) {
  __shared__ FwdSmem<P> sm;
  __shared__ int s_work;
  for (;;) {
    if (threadIdx.x == 0) s_work = pop_work<PH>(g);
    __syncthreads();
    // uniform: the item's metadata then comes through scalar loads, which
    // leave the vector-memory count (operand loads in flight) alone
    const int wk = __builtin_amdgcn_readfirstlane(s_work);
    __syncthreads();
    if (wk < 0) break;
    fwd_item<P, PH>(g, sm, wk);
  }
}

// --- BF16x3: direct global -> LDS loads into a ring of stages ---------------------
// A stage holds 128 x 32 tiles of A and of B, high and low halves: four
// arrays of eight 16-row chunks of 1 KB.  Row r of a chunk keeps its four
// 16-byte k-vectors at slots kv ^ bswz(r), so that the 16 rows read by one
// MFMA operand fetch fall into distinct LDS banks.  Loads go straight from
// global memory into the ring (global_load_lds, 16 bytes per lane), BNS - 1
// stages ahead of the MFMA work; a stage is consumed after a vector-memory
// count wait and one barrier.  Out-of-range rows and whole k-vectors beyond
// K read the zero region; the library's own operands (T, padded psi, the
// identity) are zero beyond K, so the k-tail of an operator row meets zeros.
typedef __bf16 bfx4 __attribute__((ext_vector_type(4)));
constexpr int BNS = 4, BBK = 32;
constexpr int BLOADS = 8;  // global_load_lds per wave and stage
__device__ inline int bswz(int r) { return (r >> 1) & 3; }
struct __attribute__((aligned(16))) BfRing {
  uint16_t s[BNS][4][GM * BBK];  // [stage][A hi, A lo, B hi, B lo][chunk * 512 + slot]
};

__device__ inline void gl_lds(const void *src, void *dst) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                   (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
}

// Waits until at most n_after stages of this wave's ring loads are in flight
// (vector-memory loads complete in order), then joins the workgroup.  No
// fence: only the LDS written by this kernel's ring loads is exchanged here.
__device__ inline void ring_sync(int n_after) {
  constexpr int E = (7 << 4) | (15 << 8);  // expcnt, lgkmcnt: no wait
  if (n_after >= 2)
    __builtin_amdgcn_s_waitcnt(E | (2 * BLOADS & 15) | ((2 * BLOADS >> 4) << 14));
  else if (n_after == 1)
    __builtin_amdgcn_s_waitcnt(E | (BLOADS & 15) | ((BLOADS >> 4) << 14));
  else
    __builtin_amdgcn_s_waitcnt(E);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}
static_assert(BNS == 4, "ring_sync covers up to two stages in flight after the awaited one");

__device__ inline void bf_issue(BfRing &rg, int buf, const Mat &A, const Mat &B, int r0, int c0, int k0, int K,
                                const void *zero) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rin = lane >> 2;
  const int k = k0 + 8 * ((lane & 3) ^ bswz(rin));
  const uint16_t *z = reinterpret_cast<const uint16_t *>(zero);
  const bool kin = k < K;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int chunk = 2 * w + h;
    const int ra = r0 + 16 * chunk + rin, rb = c0 + 16 * chunk + rin;
    const bool ia = kin && ra < A.rows, ib = kin && rb < B.rows;
    const uint16_t *pa = reinterpret_cast<const uint16_t *>(A.p) + (int64_t)ra * A.ld + k;
    const uint16_t *pb = reinterpret_cast<const uint16_t *>(B.p) + (int64_t)rb * B.ld + k;
    gl_lds(ia ? pa : z, &rg.s[buf][0][chunk * 512]);
    gl_lds(ia ? pa + A.lo : z, &rg.s[buf][1][chunk * 512]);
    gl_lds(ib ? pb : z, &rg.s[buf][2][chunk * 512]);
    gl_lds(ib ? pb + B.lo : z, &rg.s[buf][3][chunk * 512]);
  }
}

// MFMA on one ring stage for a (32 TM) x (32 TN) tile: wave (wm, wn) owns rows
// chunks wm TM + i and column chunks wn TN + j.
template <int TM, int TN>
__device__ inline void bf_mma(const BfRing &rg, int buf, f4 (&acc)[4][4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1, l16 = lane & 15, g = lane >> 4;
  const int off = (l16 * 4 + (g ^ bswz(l16))) * 8;
  u16x8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    ah[i] = *reinterpret_cast<const u16x8 *>(&rg.s[buf][0][(wm * TM + i) * 512 + off]);
    al[i] = *reinterpret_cast<const u16x8 *>(&rg.s[buf][1][(wm * TM + i) * 512 + off]);
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    bh[j] = *reinterpret_cast<const u16x8 *>(&rg.s[buf][2][(wn * TN + j) * 512 + off]);
    bl[j] = *reinterpret_cast<const u16x8 *>(&rg.s[buf][3][(wn * TN + j) * 512 + off]);
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j] = mfma_bf(al[i], bh[j], acc[i][j]);
      acc[i][j] = mfma_bf(ah[i], bl[j], acc[i][j]);
      acc[i][j] = mfma_bf(ah[i], bh[j], acc[i][j]);
    }
}

// Phase B of the BF16x3 path: one item (output tile, chunk of tasks), the
// tasks' K steps streamed through the ring.
template <int TM, int TN>
__device__ inline void bf_item_b_t(const FwdArgs &g, BfRing &rg, const Item &it, int mode) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1, l16 = lane & 15, lg = lane >> 4;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = vzero<f4>();
  int ls = it.tb, lj = 0, lK, issued = 0;
  bool ldone = false;
  Mat LA, LB;
  seg_ops<TNS_BF16X3, 1>(g, cld(&g.idx[ls]), LA, LB, lK, nullptr);
  auto issue_next = [&]() {
    bf_issue(rg, issued % BNS, LA, LB, it.p0, it.c0, lj * BBK, lK, g.zero);
    ++issued;
    if (++lj * BBK >= lK) {
      lj = 0;
      if (++ls < it.te) seg_ops<TNS_BF16X3, 1>(g, cld(&g.idx[ls]), LA, LB, lK, nullptr);
      else ldone = true;
    }
  };
  while (!ldone && issued < BNS - 1) issue_next();
  for (int s = 0; s < issued; ++s) {
    ring_sync(issued - 1 - s);
    if (!ldone) issue_next();
    bf_mma<TM, TN>(rg, s % BNS, acc);
  }
  const int R = cld(&g.grp_rows[it.grp]), C = cld(&g.grp_cols[it.grp]);
  float *slot = reinterpret_cast<float *>(g.partial) + cld(&g.slot_off[it.slot]);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = it.c0 + wn * 16 * TN + j * 16 + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = it.p0 + wm * 16 * TM + i * 16 + mrow(acc[i][j], lg, v);
        if (row < R && col < C) {
          const int64_t o = mode == M_FWD1 ? ((int64_t)col * R + row) : ((int64_t)row * C + col);
          slot[o] = acc[i][j][v];
        }
      }
    }
}

__device__ inline void bf_item_b(const FwdArgs &g, BfRing &rg, int wk) {
  const Item it = load_item(g.items + wk);
  const int mode = it.mode & 0xff, tm = (it.mode >> 8) & 0xff, tn = (it.mode >> 16) & 0xff;
#define TNS_CALL_B(a, b) bf_item_b_t<a, b>(g, rg, it, mode)
  TNS_TILE_SWITCH(tm, tn, TNS_CALL_B)
#undef TNS_CALL_B
}

__global__ __launch_bounds__(GTH) void k_fwd_bfb(FwdArgs g) {
  __shared__ BfRing rg;
  __shared__ int s_work;
  for (;;) {
    if (threadIdx.x == 0) s_work = pop_work<1>(g);
    __syncthreads();
    const int wk = __builtin_amdgcn_readfirstlane(s_work);
    __syncthreads();
    if (wk < 0) break;
    bf_item_b(g, rg, wk);
  }
}


// Phase A of the BF16x3 path.  A work item is a block of ABT consecutive
// tasks; all tiles of all its tasks form one stream of K steps, so the ring
// keeps loading across tile and task boundaries.  The MFMA operand roles are
// swapped (D = M-side x X-side^T), which gives every lane four consecutive
// columns of one row of T: the epilogue writes 8-byte groups of the high and
// low halves.
constexpr int ABT = 4;

__device__ inline int pop_block(const FwdArgs &g, int64_t nblk) {
  const int home = blockIdx.x % g.nq;
  for (int k = 0; k < g.nq; ++k) {
    const int q = home + k < g.nq ? home + k : home + k - g.nq;
    const int64_t n = nblk > q ? (nblk - 1 - q) / g.nq + 1 : 0;
    if (n <= 0) continue;
    const int j = atomicAdd(g.queue + q, 1);
    if (j < n) return (int)((int64_t)j * g.nq + q);
  }
  return -1;
}

template <int TM, int TN>
__device__ inline void bf_mma_t(const BfRing &rg, int buf, f4 (&acc)[4][4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1, l16 = lane & 15, g = lane >> 4;
  const int off = (l16 * 4 + (g ^ bswz(l16))) * 8;
  u16x8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
  for (int j = 0; j < TM; ++j) {
    ah[j] = *reinterpret_cast<const u16x8 *>(&rg.s[buf][0][(wm * TM + j) * 512 + off]);
    al[j] = *reinterpret_cast<const u16x8 *>(&rg.s[buf][1][(wm * TM + j) * 512 + off]);
  }
#pragma unroll
  for (int i = 0; i < TN; ++i) {
    bh[i] = *reinterpret_cast<const u16x8 *>(&rg.s[buf][2][(wn * TN + i) * 512 + off]);
    bl[i] = *reinterpret_cast<const u16x8 *>(&rg.s[buf][3][(wn * TN + i) * 512 + off]);
  }
  // acc[i][j]: rows = T columns wn*16*TN + 16 i + .., columns = T rows wm*16*TM + 16 j + ..
#pragma unroll
  for (int i = 0; i < TN; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) {
      acc[i][j] = mfma_bf(bl[i], ah[j], acc[i][j]);
      acc[i][j] = mfma_bf(bh[i], al[j], acc[i][j]);
      acc[i][j] = mfma_bf(bh[i], ah[j], acc[i][j]);
    }
}

// Epilogue of a phase-A BF16x3 tile: T = alpha * acc as 8-byte groups of the
// high and low halves.
template <int TM, int TN>
__device__ inline void bf_store_t(const FwdArgs &g, f4 (&acc)[4][4], int t, int r0, int c0, int rows, int ld,
                                  float alf) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1, l16 = lane & 15, lg = lane >> 4;
  uint16_t *Th = reinterpret_cast<uint16_t *>(g.T) + cld(&g.t_off[t]);
#pragma unroll
  for (int j = 0; j < TM; ++j) {
    const int row = r0 + wm * 16 * TM + j * 16 + l16;
#pragma unroll
    for (int i = 0; i < TN; ++i) {
      const int col = c0 + wn * 16 * TN + i * 16 + 4 * lg;
      if (row < rows && col < ld) {
        const f4 x = alf * acc[i][j];
        const bfx4 h = {(__bf16)x[0], (__bf16)x[1], (__bf16)x[2], (__bf16)x[3]};
        const bfx4 l = {(__bf16)(x[0] - (float)h[0]), (__bf16)(x[1] - (float)h[1]), (__bf16)(x[2] - (float)h[2]),
                        (__bf16)(x[3] - (float)h[3])};
        const int64_t o = (int64_t)row * ld + col;
        *reinterpret_cast<uint64_t *>(Th + o) = __builtin_bit_cast(uint64_t, h);
        *reinterpret_cast<uint64_t *>(Th + g.T_lo + o) = __builtin_bit_cast(uint64_t, l);
      }
      acc[i][j] = vzero<f4>();
    }
  }
}

// Phase A of the BF16x3 path: block b of ABT tasks as one stream; each task
// uses the tile extents of its T dimensions.
__device__ inline void bf_item_a(const FwdArgs &g, BfRing &rg, int b) {
  const int t_end = (int)min((int64_t)(b + 1) * ABT, g.ntasks);
  // load cursor: (task, tile row, tile column, k) in stream order
  int lt = b * ABT, lr0 = 0, lc0 = 0, lk0 = 0, lK, issued = 0, ltr, ltc;
  bool ldone = false;
  Mat LA, LB;
  auto load_task = [&]() {
    seg_ops<TNS_BF16X3, 0>(g, lt, LA, LB, lK, nullptr);
    ltr = tile_ext(g.tiles, LA.rows);
    ltc = tile_ext(g.tiles, LB.rows);
  };
  load_task();
  auto issue_next = [&]() {
    bf_issue(rg, issued % BNS, LA, LB, lr0, lc0, lk0, lK, g.zero);
    ++issued;
    if ((lk0 += BBK) < lK) return;
    lk0 = 0;
    if ((lc0 += ltc) < LB.rows) return;
    lc0 = 0;
    if ((lr0 += ltr) < LA.rows) return;
    lr0 = 0;
    if (++lt < t_end) load_task();
    else ldone = true;
  };
  while (!ldone && issued < BNS - 1) issue_next();
  // compute cursor, BNS - 1 steps behind
  int ct = b * ABT, cr0 = 0, cc0 = 0, ck0 = 0, cK, ctm, ctn;
  double alpha;
  Mat CA, CB;
  auto compute_task = [&]() {
    seg_ops<TNS_BF16X3, 0>(g, ct, CA, CB, cK, &alpha);
    ctm = tile_ext(g.tiles, CA.rows) / 32;
    ctn = tile_ext(g.tiles, CB.rows) / 32;
  };
  compute_task();
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = vzero<f4>();
  for (int s = 0; s < issued; ++s) {
    ring_sync(issued - 1 - s);
    if (!ldone) issue_next();
#define TNS_CALL_M(a, b) bf_mma_t<a, b>(rg, s % BNS, acc)
    TNS_TILE_SWITCH(ctm, ctn, TNS_CALL_M)
#undef TNS_CALL_M
    if ((ck0 += BBK) < cK) continue;
    // tile (cr0, cc0) of task ct complete
    {
      const int rows = CA.rows, ld = ld8(CB.rows);
      const float alf = (float)alpha;
#define TNS_CALL_S(a, b) bf_store_t<a, b>(g, acc, ct, cr0, cc0, rows, ld, alf)
      TNS_TILE_SWITCH(ctm, ctn, TNS_CALL_S)
#undef TNS_CALL_S
    }
    ck0 = 0;
    if ((cc0 += 32 * ctn) < CB.rows) continue;
    cc0 = 0;
    if ((cr0 += 32 * ctm) < CA.rows) continue;
    cr0 = 0;
    if (++ct < t_end) compute_task();
  }
}

__global__ __launch_bounds__(GTH) void k_fwd_bfa(FwdArgs g) {
  __shared__ BfRing rg;
  __shared__ int s_work;
  const int64_t nblk = (g.ntasks + ABT - 1) / ABT;
  for (;;) {
    if (threadIdx.x == 0) s_work = pop_block(g, nblk);
    __syncthreads();
    const int b = __builtin_amdgcn_readfirstlane(s_work);
    __syncthreads();
    if (b < 0) break;
    bf_item_a(g, rg, b);
  }
}

__global__ void k_ident_bf(uint16_t *p, int n, int ld, int64_t lo) {
  GRID_STRIDE(e, (int64_t)n * ld) {
    const int64_t i = e / ld, j = e % ld;
    p[e] = i == j ? (uint16_t)0x3f80 : (uint16_t)0;
    p[lo + e] = 0;
  }
}

// --- padded copies of psi ----------------------------------------------------------
// Sector s (m x n) to pp (m x ld8(n)) and, transposed, to pt (n x ld8(m));
// BF16X3 writes high halves and, `lo` elements further, low halves.
template <class In, int P>
__device__ inline void pad_sector(int s, const In *__restrict__ psi, const int64_t *psi_off, const int32_t *psi_sec,
                                  const int32_t *dimL, const int32_t *dimR, const int64_t *pp_off,
                                  const int64_t *pt_off, void *pp, void *pt, int64_t pp_lo, int64_t pt_lo) {
  typedef typename FP<P>::E E;
  const int m = dimL[psi_sec[4 * s]], n = dimR[psi_sec[4 * s + 3]];
  const int lm = ld8(m), ln = ld8(n);
  const In *A = psi + psi_off[s];
  E *P0 = reinterpret_cast<E *>(pp) + pp_off[s], *P1 = reinterpret_cast<E *>(pt) + pt_off[s];
  const int64_t step = (int64_t)gridDim.y * blockDim.x, e0 = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  // padded rows (zeros beyond n), then padded transposed rows (zeros beyond m)
  for (int64_t e = e0; e < (int64_t)m * ln; e += step) {
    const int i = (int)(e / ln), j = (int)(e % ln);
    if constexpr (P == TNS_BF16X3) {
      const float v = j < n ? (float)A[(int64_t)i * n + j] : 0.f;
      const uint16_t h = f32_to_bf16_rne(v);
      P0[e] = h;
      P0[pp_lo + e] = f32_to_bf16_rne(v - bf16_to_f32(h));
    } else {
      P0[e] = j < n ? (E)A[(int64_t)i * n + j] : E(0);
    }
  }
  for (int64_t e = e0; e < (int64_t)n * lm; e += step) {
    const int j = (int)(e / lm), i = (int)(e % lm);
    if constexpr (P == TNS_BF16X3) {
      const float v = i < m ? (float)A[(int64_t)i * n + j] : 0.f;
      const uint16_t h = f32_to_bf16_rne(v);
      P1[e] = h;
      P1[pt_lo + e] = f32_to_bf16_rne(v - bf16_to_f32(h));
    } else {
      P1[e] = i < m ? (E)A[(int64_t)i * n + j] : E(0);
    }
  }
}

template <class In, int P>
__global__ void k_pad_psi(const In *__restrict__ psi, const int64_t *psi_off, const int32_t *psi_sec,
                          const int32_t *dimL, const int32_t *dimR, const int64_t *pp_off, const int64_t *pt_off,
                          void *pp, void *pt, int64_t pp_lo, int64_t pt_lo) {
  pad_sector<In, P>(blockIdx.x, psi, psi_off, psi_sec, dimL, dimR, pp_off, pt_off, pp, pt, pp_lo, pt_lo);
}

// ============================================================================
// Many independent products in one launch per phase.  Instance i's arguments
// live in a device table; every XCD queue of a phase is the concatenation of
// the instances' own queue contents (instances ordered by descending cost);
// a workgroup finds (instance, local work) by binary search over the
// per-queue prefix sums and reads that instance's arguments by scalar loads.
// ============================================================================
struct InstArgs {
  FwdArgs g;
  const void *psi;  // input: double (F64) or float
  void *sigma;
  const int64_t *psi_off, *grp_chunk_base;
  int64_t psi_dim;
  int32_t nS, beta;
};
static_assert(sizeof(FwdArgs) % 8 == 0 && sizeof(InstArgs) % 8 == 0, "8-byte words");

struct BatchArgs {
  const InstArgs *tab;
  int64_t *cum;     // [2][NQ_MAX][n + 1] work prefix per phase and queue
  int32_t *queue;   // [0, 8) phase A, [8, 16) phase B
  int32_t n, nq, blocks;  // blocks: phase-A unit is a block of ABT tasks (BF16X3)
  int32_t pad_;
};

template <class T>
__device__ inline T load_words(const T *p) {
  T v;
  const uint64_t *src = reinterpret_cast<const uint64_t *>(p);
  uint64_t *dst = reinterpret_cast<uint64_t *>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 8); ++i) dst[i] = cld(src + i);
  return v;
}

__device__ inline int64_t blk_count(int64_t ntasks, int nq, int q) {
  const int64_t nblk = (ntasks + ABT - 1) / ABT;
  return nblk > q ? (nblk - 1 - q) / nq + 1 : 0;
}

// Work of instance i on queue q of phase ph (16 threads: one per (ph, q)).
__global__ void k_batch_cum(BatchArgs b) {
  const int ph = threadIdx.x / NQ_MAX, q = threadIdx.x % NQ_MAX;
  if (ph >= 2) return;
  int64_t *c = b.cum + ((int64_t)ph * NQ_MAX + q) * (b.n + 1);
  int64_t run = 0;
  for (int i = 0; i < b.n; ++i) {
    c[i] = run;
    if (q < b.nq) {
      const FwdArgs &g = b.tab[i].g;
      if (ph == 0) run += b.blocks ? blk_count(g.ntasks, b.nq, q) : qa_count(g.ntasks, b.nq, q);
      else run += g.qbase[q + 1] - g.qbase[q];
    }
  }
  c[b.n] = run;
}

// Thread 0: next (instance, work id) of phase ph, own XCD queue first.
__device__ inline void pop_batch(const BatchArgs &b, int ph, int *inst, int *wk) {
  const int home = blockIdx.x % b.nq;
  for (int k = 0; k < b.nq; ++k) {
    const int q = home + k < b.nq ? home + k : home + k - b.nq;
    const int64_t *c = b.cum + ((int64_t)ph * NQ_MAX + q) * (b.n + 1);
    const int64_t tot = c[b.n];
    if (tot <= 0) continue;
    const int j = atomicAdd(b.queue + 8 * ph + q, 1);
    if (j >= tot) continue;
    int lo = 0, hi = b.n - 1;  // last instance with c[i] <= j
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (c[mid] <= j) lo = mid; else hi = mid - 1;
    }
    const int64_t loc = j - c[lo];
    *inst = lo;
    if (ph == 1) *wk = (int)(b.tab[lo].g.qbase[q] + loc);
    else *wk = b.blocks ? (int)(loc * b.nq + q) : (int)qa_task(b.nq, q, loc);
    return;
  }
  *inst = -1;
  *wk = -1;
}

template <int P, int PH>
__global__ __launch_bounds__(GTH, P == TNS_F32 ? 2 : 1) void k_fwd_batch(BatchArgs b) {
  __shared__ FwdSmem<P> sm;
  __shared__ int s_w[2];
  for (;;) {
    if (threadIdx.x == 0) pop_batch(b, PH, &s_w[0], &s_w[1]);
    __syncthreads();
    const int inst = __builtin_amdgcn_readfirstlane(s_w[0]), wk = __builtin_amdgcn_readfirstlane(s_w[1]);
    __syncthreads();
    if (inst < 0) break;
    const FwdArgs g = load_words(&b.tab[inst].g);
    fwd_item<P, PH>(g, sm, wk);
  }
}

template <int PH>
__global__ __launch_bounds__(GTH) void k_fwd_bf_batch(BatchArgs b) {
  __shared__ BfRing rg;
  __shared__ int s_w[2];
  for (;;) {
    if (threadIdx.x == 0) pop_batch(b, PH, &s_w[0], &s_w[1]);
    __syncthreads();
    const int inst = __builtin_amdgcn_readfirstlane(s_w[0]), wk = __builtin_amdgcn_readfirstlane(s_w[1]);
    __syncthreads();
    if (inst < 0) break;
    const FwdArgs g = load_words(&b.tab[inst].g);
    if (PH == 0) bf_item_a(g, rg, wk);
    else bf_item_b(g, rg, wk);
  }
}

template <class In, int P>
__global__ void k_pad_psi_batch(const InstArgs *tab) {
  const InstArgs &a = tab[blockIdx.z];
  if ((int)blockIdx.x >= a.nS) return;
  pad_sector<In, P>(blockIdx.x, reinterpret_cast<const In *>(a.psi), a.psi_off, a.g.psi_sec, a.g.dimL, a.g.dimR,
                    a.g.pp_off, a.g.pt_off, const_cast<void *>(a.g.pp), const_cast<void *>(a.g.pt), a.g.pp_lo,
                    a.g.pt_lo);
}

// sigma_i (+)= the sum of instance i's partial slots, as k_epilogue_psi.
template <class T>
__global__ void k_epilogue_batch(const InstArgs *tab) {
  const InstArgs &a = tab[blockIdx.y];
  const int64_t *psi_off = a.psi_off, *cb = a.grp_chunk_base, *slot_off = a.g.slot_off;
  const T *part = reinterpret_cast<const T *>(a.g.partial);
  T *out = reinterpret_cast<T *>(a.sigma);
  const int nS = a.nS, beta = a.beta;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.psi_dim;
       e += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = nS;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (psi_off[mid] <= e) lo = mid; else hi = mid;
    }
    const int64_t loc = e - psi_off[lo];
    double acc = beta ? (double)out[e] : 0.0;
    const int64_t c0 = cb[2 * lo], c1 = cb[2 * lo + 2];
    for (int64_t c = c0; c < c1; ++c) acc += (double)part[slot_off[c] + loc];
    out[e] = (T)acc;
  }
}

constexpr int ARGS_PER_PUT = 3500 / (int)sizeof(InstArgs);
struct PutArgs {
  InstArgs a[ARGS_PER_PUT];
  int32_t base, n;
};
static_assert(ARGS_PER_PUT >= 1 && sizeof(PutArgs) <= 4000, "argument chunk fits the kernel argument segment");
__global__ void k_put_args(PutArgs c, InstArgs *tab) {
  if ((int)threadIdx.x < c.n) tab[c.base + threadIdx.x] = c.a[threadIdx.x];
}

// --- host side --------------------------------------------------------------------------
// BF16X3 halves: the low half of an array of n elements starts at ld8(n).
static inline int64_t lo_of(int64_t n) { return (n + 7) & ~int64_t(7); }

// Bytes of an operand array of n elements in a precision (BF16X3: both halves).
static size_t region(int64_t n, tns_prec p) {
  n = std::max<int64_t>(n, 1);
  const size_t b = p == TNS_F64 ? (size_t)n * 8 : p == TNS_F32 ? (size_t)n * 4 : (size_t)lo_of(n) * 4;
  return align_up(b + 64, 256);
}

// Identity matrix of the BF16X3 path: maxdim x ld8(maxdim).
static int64_t ident_elems(const Plan &p) { return (int64_t)p.maxdim * ld8(p.maxdim); }

// Workspace of the forward product: [queue counters, zero bytes | partial
// slots | T | padded psi | padded psi^T | (BF16X3) identity].
size_t fwd_workspace(const Plan &p, tns_prec prec) {
  return 256 + align_up((size_t)std::max<int64_t>(p.fwd.partial_elems, 1) * (prec == TNS_F64 ? 8 : 4), 256) +
         region(p.t_elems, prec) + region(p.pp_elems, prec) + region(p.pt_elems, prec) +
         (prec == TNS_BF16X3 ? region(ident_elems(p), prec) : 0);
}

// queue counters (bytes 0..63) and the 64-byte zero region that out-of-range
// loads read (bytes 64..127)
__global__ void k_reset_queues(int32_t *p) {
  if (threadIdx.x < 32) p[threadIdx.x] = 0;
}

static inline unsigned nblocks(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16));
}

template <class K>
static int grid_of(K kern, int n_cu) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, GTH, 0) != hipSuccess || per <= 0) per = 1;
  return per * n_cu;
}

// Arguments of one product whose workspace region (layout of fwd_workspace)
// starts at w.
template <int P>
static FwdArgs fwd_args(const Plan &p, const void *ops, char *w) {
  typedef typename FP<P>::Acc Acc;
  const Sched &S = p.fwd;
  const tns_prec prec = (tns_prec)P;
  char *c = w + 256;
  void *part = c;
  c += align_up((size_t)std::max<int64_t>(S.partial_elems, 1) * sizeof(Acc), 256);
  void *T = c;
  c += region(p.t_elems, prec);
  void *pp = c;
  c += region(p.pp_elems, prec);
  void *pt = c;
  c += region(p.pt_elems, prec);
  void *id = c;
  FwdArgs g;
  memset(&g, 0, sizeof(g));
  g.tasks = p.tasks; g.ntasks = p.ntasks;
  g.psi_sec = p.psi_sec; g.dimL = p.dimL; g.dimR = p.dimR;
  g.blk_off = p.blk_off; g.blk_ld = p.blk_ld;
  g.ops = ops; g.ops_lo = lo_of(p.n_vals);
  g.pp = pp; g.pt = pt; g.pp_lo = lo_of(p.pp_elems); g.pt_lo = lo_of(p.pt_elems);
  g.pp_off = p.pp_off; g.pt_off = p.pt_off;
  g.T = T; g.T_lo = lo_of(p.t_elems); g.t_off = p.t_off;
  g.items = S.items; g.nitems = S.nitems; g.idx = S.idx; g.grp_rows = S.grp_rows; g.grp_cols = S.grp_cols;
  g.slot_off = S.slot_off; g.qbase = S.qbase; g.partial = part;
  g.queue = reinterpret_cast<int32_t *>(w); g.nq = S.nq;
  g.zero = w + 64;
  g.ident = id; g.ident_lo = lo_of(ident_elems(p)); g.ident_ld = ld8(p.maxdim);
  g.tiles = p.tiles;
  return g;
}

template <int P, class In>
static tns_status fwd_launch(const Plan &p, const void *ops, const In *psi, void *sigma, int beta, char *w,
                             hipStream_t st, const hipEvent_t *ev) {
  const Sched &S = p.fwd;
  const FwdArgs g = fwd_args<P>(p, ops, w);
  hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(32), 0, st, g.queue);
  if (P == TNS_BF16X3)
    hipLaunchKernelGGL(k_ident_bf, dim3(nblocks(ident_elems(p))), dim3(256), 0, st, (uint16_t *)g.ident, p.maxdim,
                       ld8(p.maxdim), g.ident_lo);
  if (p.nS > 0)
    hipLaunchKernelGGL((k_pad_psi<In, P>), dim3(p.nS, 8), dim3(256), 0, st, psi, p.psi_off, p.psi_sec, p.dimL,
                       p.dimR, p.pp_off, p.pt_off, const_cast<void *>(g.pp), const_cast<void *>(g.pt), g.pp_lo,
                       g.pt_lo);
  if (ev) TNS_HIP(hipEventRecord(ev[0], st));
  if (p.ntasks > 0) {
    if constexpr (P == TNS_BF16X3)
      hipLaunchKernelGGL(k_fwd_bfa, dim3(grid_of(k_fwd_bfa, p.n_cu)), dim3(GTH), 0, st, g);
    else
      hipLaunchKernelGGL((k_fwd<P, 0>), dim3(grid_of(k_fwd<P, 0>, p.n_cu)), dim3(GTH), 0, st, g);
  }
  if (ev) TNS_HIP(hipEventRecord(ev[1], st));
  if (p.ntasks > 0 && S.nitems > 0) {
    if constexpr (P == TNS_BF16X3)
      hipLaunchKernelGGL(k_fwd_bfb, dim3(grid_of(k_fwd_bfb, p.n_cu)), dim3(GTH), 0, st, g);
    else
      hipLaunchKernelGGL((k_fwd<P, 1>), dim3(grid_of(k_fwd<P, 1>, p.n_cu)), dim3(GTH), 0, st, g);
  }
  if (ev) TNS_HIP(hipEventRecord(ev[2], st));
  return launch_epilogue_psi(p, P == TNS_F64, g.partial, sigma, beta, st);
}

// --- batched products -------------------------------------------------------------------
static int max_maxdim(const tns_tasklist *const *tls, int n) {
  int md = 1;
  for (int i = 0; i < n; ++i) md = std::max(md, plan_of(tls[i]).maxdim);
  return md;
}

// [queue counters, zero bytes | argument table | prefix sums | (BF16X3) shared
// identity | one forward workspace per instance]
static size_t batch_bytes(const tns_tasklist *const *tls, int n, tns_prec prec) {
  size_t b = 256 + align_up((size_t)n * sizeof(InstArgs), 256) + align_up((size_t)2 * NQ_MAX * (n + 1) * 8, 256);
  const int md = max_maxdim(tls, n);
  if (prec == TNS_BF16X3) b += region((int64_t)md * ld8(md), prec);
  for (int i = 0; i < n; ++i) b += fwd_workspace(plan_of(tls[i]), prec);
  return b;
}

template <int P>
static tns_status batch_launch(const tns_tasklist *const *tls, int n, const void *const *ops,
                               const void *const *psi, void *const *sigma, int beta, char *w, hipStream_t st,
                               const hipEvent_t *ev) {
  typedef typename FP<P>::Acc Acc;
  const tns_prec prec = (tns_prec)P;
  int32_t *queue = reinterpret_cast<int32_t *>(w);
  char *c = w + 256;
  InstArgs *tab = reinterpret_cast<InstArgs *>(c);
  c += align_up((size_t)n * sizeof(InstArgs), 256);
  int64_t *cum = reinterpret_cast<int64_t *>(c);
  c += align_up((size_t)2 * NQ_MAX * (n + 1) * 8, 256);
  const int md = max_maxdim(tls, n);
  const int64_t id_elems = (int64_t)md * ld8(md);
  void *ident = c;
  if (P == TNS_BF16X3) c += region(id_elems, prec);
  // instances by descending cost: the big ones start first, the small ones fill the tail
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) {
    return plan_of(tls[x]).fwd.total_cost > plan_of(tls[y]).fwd.total_cost;
  });
  std::vector<char *> region_of(n);
  for (int i = 0; i < n; ++i) {
    region_of[i] = c;
    c += fwd_workspace(plan_of(tls[i]), prec);
  }
  std::vector<InstArgs> args(n);
  int max_nS = 1, n_cu = 1, any_tasks = 0, any_items = 0;
  int64_t max_dim = 1;
  for (int k = 0; k < n; ++k) {
    const int i = perm[k];
    const Plan &p = plan_of(tls[i]);
    InstArgs &a = args[k];
    memset(&a, 0, sizeof(a));
    a.g = fwd_args<P>(p, ops[i], region_of[i]);
    a.g.queue = queue;
    a.g.zero = w + 64;
    a.g.ident = ident; a.g.ident_lo = lo_of(id_elems); a.g.ident_ld = ld8(md);
    a.psi = psi[i]; a.sigma = sigma[i];
    a.psi_off = p.psi_off; a.grp_chunk_base = p.fwd.grp_chunk_base;
    a.psi_dim = p.psi_dim; a.nS = p.nS; a.beta = beta;
    max_nS = std::max(max_nS, p.nS);
    max_dim = std::max(max_dim, p.psi_dim);
    n_cu = std::max(n_cu, p.n_cu);
    any_tasks |= p.ntasks > 0;
    any_items |= p.fwd.nitems > 0;
  }
  BatchArgs b;
  memset(&b, 0, sizeof(b));
  b.tab = tab; b.cum = cum; b.queue = queue; b.n = n; b.nq = plan_of(tls[0]).fwd.nq;
  b.blocks = P == TNS_BF16X3;

  hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(32), 0, st, queue);
  for (int k0 = 0; k0 < n; k0 += ARGS_PER_PUT) {
    PutArgs pa;
    memset(&pa, 0, sizeof(pa));
    pa.base = k0;
    pa.n = std::min(ARGS_PER_PUT, n - k0);
    for (int k = 0; k < pa.n; ++k) pa.a[k] = args[k0 + k];
    hipLaunchKernelGGL(k_put_args, dim3(1), dim3(64), 0, st, pa, tab);
  }
  hipLaunchKernelGGL(k_batch_cum, dim3(1), dim3(2 * NQ_MAX), 0, st, b);
  if (P == TNS_BF16X3)
    hipLaunchKernelGGL(k_ident_bf, dim3(nblocks(id_elems)), dim3(256), 0, st, (uint16_t *)ident, md, ld8(md),
                       lo_of(id_elems));
  typedef typename std::conditional<P == TNS_F64, double, float>::type In;
  hipLaunchKernelGGL((k_pad_psi_batch<In, P>), dim3(max_nS, 8, n), dim3(256), 0, st, tab);
  if (ev) TNS_HIP(hipEventRecord(ev[0], st));
  if (any_tasks) {
    if constexpr (P == TNS_BF16X3)
      hipLaunchKernelGGL(k_fwd_bf_batch<0>, dim3(grid_of(k_fwd_bf_batch<0>, n_cu)), dim3(GTH), 0, st, b);
    else
      hipLaunchKernelGGL((k_fwd_batch<P, 0>), dim3(grid_of(k_fwd_batch<P, 0>, n_cu)), dim3(GTH), 0, st, b);
  }
  if (ev) TNS_HIP(hipEventRecord(ev[1], st));
  if (any_tasks && any_items) {
    if constexpr (P == TNS_BF16X3)
      hipLaunchKernelGGL(k_fwd_bf_batch<1>, dim3(grid_of(k_fwd_bf_batch<1>, n_cu)), dim3(GTH), 0, st, b);
    else
      hipLaunchKernelGGL((k_fwd_batch<P, 1>), dim3(grid_of(k_fwd_batch<P, 1>, n_cu)), dim3(GTH), 0, st, b);
  }
  if (ev) TNS_HIP(hipEventRecord(ev[2], st));
  const unsigned gx = (unsigned)std::min<int64_t>(4096, (max_dim + 255) / 256);
  hipLaunchKernelGGL(k_epilogue_batch<Acc>, dim3(gx, n), dim3(256), 0, st, tab);
  return hipGetLastError() == hipSuccess ? TNS_OK : TNS_ERR_HIP;
}

tns_status fwd_apply(const Plan &p, tns_prec prec, const void *ops, const void *psi, void *sigma, double beta,
                     void *ws, size_t ws_bytes, hipStream_t st, const hipEvent_t *ev) {
  if (ws_bytes < fwd_workspace(p, prec)) return TNS_ERR_WORKSPACE;
  char *w = reinterpret_cast<char *>(ws);
  const int ib = beta != 0.0;
  tns_status s;
  if (prec == TNS_F64)
    s = fwd_launch<TNS_F64>(p, ops, (const double *)psi, sigma, ib, w, st, ev);
  else if (prec == TNS_F32)
    s = fwd_launch<TNS_F32>(p, ops, (const float *)psi, sigma, ib, w, st, ev);
  else
    s = fwd_launch<TNS_BF16X3>(p, ops, (const float *)psi, sigma, ib, w, st, ev);
  if (s != TNS_OK) return s;
  return hipGetLastError() == hipSuccess ? TNS_OK : TNS_ERR_HIP;
}

}  // namespace tns

using namespace tns;

// Median time (ms) of `reps` runs of `run` (which enqueues one product on st)
// after one warm-up run.
template <class F>
static tns_status time_median(F run, int reps, hipStream_t st, float *ms) {
  hipEvent_t e0, e1;
  TNS_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return TNS_ERR_HIP;
  }
  std::vector<float> t;
  tns_status s = run();
  for (int r = 0; r < reps && s == TNS_OK; ++r) {
    float x = 0.f;
    if (hipEventRecord(e0, st) != hipSuccess || (s = run()) != TNS_OK || hipEventRecord(e1, st) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&x, e0, e1) != hipSuccess) {
      if (s == TNS_OK) s = TNS_ERR_HIP;
      break;
    }
    t.push_back(x);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != TNS_OK) return s;
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return TNS_OK;
}

// Coordinate descent over the four size buckets of the tile table (largest
// dimensions first): for each bucket keep the extent (128, 64, 32) with the
// shortest median product time, the other buckets fixed.  Leaves the best
// table set on every task list.
template <class F>
static tns_status autotune(tns_tasklist *const *tls, int n, F run, hipStream_t st, uint32_t *best) {
  uint32_t cur = plan_of(tls[0]).tiles;
  static const int EXT[3] = {128, 64, 32};
  for (int b = 3; b >= 0; --b) {
    float tbest = 0.f;
    uint32_t pick = cur;
    for (int e = 0; e < 3; ++e) {
      const uint32_t cand = (cur & ~(0xffu << (8 * b))) | ((uint32_t)EXT[e] << (8 * b));
      for (int i = 0; i < n; ++i) {
        const tns_status s = tns_set_tiles(tls[i], cand, st);
        if (s != TNS_OK) return s;
      }
      float ms = 0.f;
      const tns_status s = time_median(run, 3, st, &ms);
      if (s != TNS_OK) return s;
      if (e == 0 || ms < tbest) {
        tbest = ms;
        pick = cand;
      }
    }
    cur = pick;
  }
  for (int i = 0; i < n; ++i) {
    const tns_status s = tns_set_tiles(tls[i], cur, st);
    if (s != TNS_OK) return s;
  }
  if (best) *best = cur;
  return TNS_OK;
}

static bool batch_ok(const tns_tasklist *const *tls, int n, tns_prec prec) {
  if (!tls || n <= 0) return false;
  if (prec != TNS_F64 && prec != TNS_F32 && prec != TNS_BF16X3) return false;
  for (int i = 0; i < n; ++i)
    if (!tls[i] || plan_of(tls[i]).fwd.nq != plan_of(tls[0]).fwd.nq) return false;
  return true;
}

extern "C" size_t tns_apply_batch_workspace_bytes(const tns_tasklist *const *tls, int n, tns_prec prec) {
  return batch_ok(tls, n, prec) ? batch_bytes(tls, n, prec) : 0;
}

extern "C" tns_status tns_apply_heff_batch(const tns_tasklist *const *tls, int n, tns_prec prec,
                                           const void *const *op_vals, const void *const *psi, void *const *sigma,
                                           double beta, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!batch_ok(tls, n, prec) || !op_vals || !psi || !sigma || !ws) return TNS_ERR_ARG;
  if (beta != 0.0 && beta != 1.0) return TNS_ERR_ARG;
  for (int i = 0; i < n; ++i)
    if (!op_vals[i] || !psi[i] || !sigma[i]) return TNS_ERR_ARG;
  if (ws_bytes < batch_bytes(tls, n, prec)) return TNS_ERR_WORKSPACE;
  hipEvent_t ev[3];
  const bool timed = take_profile_events(ev);
  char *w = reinterpret_cast<char *>(ws);
  const int ib = beta != 0.0;
  if (prec == TNS_F64) return batch_launch<TNS_F64>(tls, n, op_vals, psi, sigma, ib, w, st, timed ? ev : nullptr);
  if (prec == TNS_F32) return batch_launch<TNS_F32>(tls, n, op_vals, psi, sigma, ib, w, st, timed ? ev : nullptr);
  return batch_launch<TNS_BF16X3>(tls, n, op_vals, psi, sigma, ib, w, st, timed ? ev : nullptr);
}

extern "C" tns_status tns_autotune_tiles(tns_tasklist *tl, tns_prec prec, const void *op_vals, const void *psi,
                                         void *sigma, void *ws, size_t ws_bytes, uint32_t *tiles_out,
                                         hipStream_t st) {
  if (!tl || !op_vals || !psi || !sigma || !ws) return TNS_ERR_ARG;
  if (prec != TNS_F64 && prec != TNS_F32 && prec != TNS_BF16X3) return TNS_ERR_ARG;
  if (ws_bytes < fwd_workspace(plan_of(tl), prec)) return TNS_ERR_WORKSPACE;
  auto run = [&]() { return fwd_apply(plan_of(tl), prec, op_vals, psi, sigma, 0.0, ws, ws_bytes, st, nullptr); };
  tns_tasklist *one[1] = {tl};
  return autotune(one, 1, run, st, tiles_out);
}

extern "C" tns_status tns_autotune_tiles_batch(tns_tasklist *const *tls, int n, tns_prec prec,
                                               const void *const *op_vals, const void *const *psi,
                                               void *const *sigma, void *ws, size_t ws_bytes, uint32_t *tiles_out,
                                               hipStream_t st) {
  if (!batch_ok(tls, n, prec) || !op_vals || !psi || !sigma || !ws) return TNS_ERR_ARG;
  for (int i = 0; i < n; ++i)
    if (!op_vals[i] || !psi[i] || !sigma[i]) return TNS_ERR_ARG;
  if (ws_bytes < batch_bytes(tls, n, prec)) return TNS_ERR_WORKSPACE;
  auto run = [&]() { return tns_apply_heff_batch(tls, n, prec, op_vals, psi, sigma, 0.0, ws, ws_bytes, st); };
  return autotune(tls, n, run, st, tiles_out);
}
