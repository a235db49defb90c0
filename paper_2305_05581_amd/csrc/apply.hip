// Level 3 of the four-level hierarchy (Section III.A.1): sigma = H_eff psi as
// the sum of Eq. (2), executed by one persistent kernel on MFMA.
//
// Work item = (output sector, row panel of TQ rows of the panel dimension,
// chunk of tasks of one evaluation-order class).  For every task of its chunk
// the item computes a chained product on chip:
//
//   stage 1   V = X[p0:p0+TQ, :] * M[:, c0:c0+KC]      (K = K1, MFMA)
//   stage 2   acc += alpha V * Y[:, c0:c0+KC]^T          (K = KC, MFMA)
//
// over column chunks c0 of M, where for class 0, (L A) R^T, X = L, M = A and
// Y = R (acc is a row panel of sigma), and for class 1, L (A R^T), X = R,
// M = A^T and Y = L (acc is a row panel of sigma^T).  This is the summed
// batched product of Alg. 2 / Fig. 3 with the interleaved intermediate kept in
// LDS instead of global memory and the sum over the task chunk taken in the
// MFMA accumulators.  Each item writes its panel into its own partial slot;
// a second kernel adds the slots of every output sector in a fixed order.
#include <algorithm>

#include "tns_internal.hpp"

namespace tns {

// Element-wise kernels walk their array with a grid stride: operator arrays
// exceed the 2^32 work items that one dispatch can address.
#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

constexpr int KK = 32;    // K1 step of stage 1
constexpr int KC = 32;    // column chunk of M (K of stage 2)
constexpr int CMAX = 512; // output columns held in accumulators per pass
constexpr int YG = 128;   // columns of Y staged in LDS at a time
constexpr int NWG = 256;  // threads per workgroup (4 waves)

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// --- BF16 split: round to nearest even, NaN kept quiet --------------------
__host__ __device__ inline uint16_t f32_to_bf16_rne(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float x;
  memcpy(&x, &u, 4);
  return x;
}

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
template <> struct Prec<TNS_BF16X3> {
  typedef float elem;    // psi / sigma type
  typedef float acc;
  typedef f4 accv;
  static constexpr int S = KK + 8;  // bf16 elements; 80-byte rows keep 16-byte alignment
};

struct ApplyArgs {
  const Item *items;
  int64_t nitems;
  int32_t *queue;
  const int32_t *idx;    // grouped task indices of the schedule
  const tns_task *tasks;
  const int32_t *psi_sec, *dimL, *dimR;
  const int64_t *psi_off, *blk_off, *slot_off;
  const int32_t *blk_ld, *blk_rows, *blk_cols;
  const void *ops;       // F64: double*, F32: float*, BF16X3: uint16 hi[n_vals] then lo[n_vals]
  const void *psi;       // F64: double*, F32: float*, BF16X3: uint16 hi[psi_dim] then lo[psi_dim]
  const void *grad;      // d loss / d sigma (backward modes), psi layout
  void *partial;         // acc type
  int64_t n_vals, psi_dim;
  int32_t mode_mask;     // bit m set: items of mode m are computed, others skipped
  const void *zero;      // 64 zero bytes: out-of-range loads read here
};

// Operand view of one matrix for the loaders: element (i, k) at
// base[i * si + k * sk]; identity when `ident`.
struct View {
  const void *p;  // element (0, 0), resolved in the precision of the kernel
  int32_t si, sk; // element (i, k) at p[i * si + k * sk]
  int32_t rows, cols;
  int32_t ident;  // identity operator: (i == k)
  int32_t src;    // 0 = operator values, 1 = psi, 2 = grad sigma (loaders of the BF16 kernel)
  int64_t off;    // element offset of (0, 0) in its array
};

template <int P> struct Tile;

// FP32 / FP64: one LDS array per tile.
template <int P>
struct TileStore {
  typedef typename Prec<P>::acc T;
  T x[TQ * Prec<P>::S];     // X rows x K1-chunk   [i][k]
  T m[KC * Prec<P>::S];     // M chunk stored [c][k]
  T v[TQ * (KC + 2)];       // V [i][c]
  T y[YG * (KC + 2)];       // Y group [j][c]
};

struct __attribute__((aligned(16))) TileStoreBF {
  uint16_t xh[TQ * (KK + 8)], xl[TQ * (KK + 8)];
  uint16_t mh[KC * (KK + 8)], ml[KC * (KK + 8)];
  uint16_t vh[TQ * (KC + 8)], vl[TQ * (KC + 8)];
  uint16_t yh[YG * (KC + 8)], yl[YG * (KC + 8)];
};

// ---------------------------------------------------------------------------
// loaders (256 threads).  Out-of-range elements load as zero.
// ---------------------------------------------------------------------------
template <class T>
struct Bases {
  const T *ops, *psi, *grad;
};

template <class T>
__device__ inline T ld_elem(const Bases<T> &b, const View &v, int i, int k) {
  if (i >= v.rows || k >= v.cols || i < 0) return T(0);
  if (v.ident) return (i == k) ? T(1) : T(0);
  const T *base = v.src == 0 ? b.ops : (v.src == 1 ? b.psi : b.grad);
  return base[v.off + (int64_t)i * v.si + (int64_t)k * v.sk];
}

struct BF {
  uint16_t h, l;
};
__device__ inline BF ld_bf(const uint16_t *hi, const uint16_t *lo, const View &v, int i, int k) {
  BF r{0, 0};
  if (i >= v.rows || k >= v.cols || i < 0) return r;
  if (v.ident) {
    r.h = (i == k) ? (uint16_t)0x3f80 : (uint16_t)0;
    return r;
  }
  const int64_t a = v.off + (int64_t)i * v.si + (int64_t)k * v.sk;
  r.h = hi[a];
  r.l = lo[a];
  return r;
}

// Fill dst[r][c] (row stride ld) = src(r0 + r, c0 + c) for r < R, c < C with
// a thread mapping that walks the memory-contiguous index fastest.
template <class T>
__device__ inline void load_tile(T *dst, int ld, int R, int C, const Bases<T> &src, const View &v, int r0, int c0) {
  const int tid = threadIdx.x;
  const bool rowfast = (v.si == 1) && !v.ident;  // contiguous along r
  const int n = R * C;
  for (int e = tid; e < n; e += NWG) {
    int r, c;
    if (rowfast) { r = e % R; c = e / R; } else { c = e % C; r = e / C; }
    dst[r * ld + c] = ld_elem(src, v, r0 + r, c0 + c);
  }
}

__device__ inline void load_tile_bf(uint16_t *dh, uint16_t *dl, int ld, int R, int C, const uint16_t *hi,
                                    const uint16_t *lo, const View &v, int r0, int c0) {
  const int tid = threadIdx.x;
  const bool rowfast = (v.si == 1) && !v.ident;
  const int n = R * C;
  for (int e = tid; e < n; e += NWG) {
    int r, c;
    if (rowfast) { r = e % R; c = e / R; } else { c = e % C; r = e / C; }
    const BF b = ld_bf(hi, lo, v, r0 + r, c0 + c);
    dh[r * ld + c] = b.h;
    dl[r * ld + c] = b.l;
  }
}

// ---------------------------------------------------------------------------
// MFMA wrappers
// ---------------------------------------------------------------------------
__device__ inline d4 mfma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma_bf(u16x8 a, u16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                 0);
}

template <class T> __device__ inline T vzero();
template <> __device__ inline d4 vzero<d4>() { return d4{0.0, 0.0, 0.0, 0.0}; }
template <> __device__ inline f4 vzero<f4>() { return f4{0.f, 0.f, 0.f, 0.f}; }

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
  switch (mode) {
    case M_FWD0: o.X = L; o.M = A; o.Y = R; o.K1 = m; o.K2 = n; break;
    case M_FWD1: o.X = R; o.M = transposed(A); o.Y = L; o.K1 = n; o.K2 = m; break;
    case M_DPSI: o.X = transposed(L); o.M = G; o.Y = transposed(R); o.K1 = q; o.K2 = r; break;
    case M_DL: o.X = G; o.M = R; o.Y = A; o.K1 = r; o.K2 = n; break;
    default: o.X = transposed(G); o.M = L; o.Y = transposed(A); o.K1 = q; o.K2 = m; break;
  }
  o.alpha = t.alpha;
  return o;
}

// Rows (panel dimension) and columns of the output matrix of an item.
__device__ inline void out_dims(const ApplyArgs &a, const Item &it, int *rows, int *cols) {
  if (it.mode <= M_DPSI) {
    const int jL = a.psi_sec[4 * it.out], jR = a.psi_sec[4 * it.out + 3];
    const int q = a.dimL[jL], r = a.dimR[jR];
    *rows = it.mode == M_FWD1 ? r : q;
    *cols = it.mode == M_FWD1 ? q : r;
  } else {
    *rows = a.blk_rows[it.out];
    *cols = a.blk_cols[it.out];
  }
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
template <> struct K3<TNS_F32> { static constexpr int KK = 32, KC = 64, KS = 8, PAD = 2; };
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

template <int P>
__global__ __launch_bounds__(NWG) void k_apply(ApplyArgs a) {
  typedef typename Prec<P>::acc T;
  typedef typename Prec<P>::accv V4;
  constexpr int KK_ = K3<P>::KK, KC_ = K3<P>::KC, KS_ = K3<P>::KS;
  constexpr int SX = KK_ + K3<P>::PAD, SV = KC_ + K3<P>::PAD, SY = KS_ + K3<P>::PAD;
  constexpr int NRT = TQ / 16;
  constexpr int NU = CMAX / 64;
  constexpr int NX = TQ * KK_ / NWG, NM = KK_ * KC_ / NWG, NY = CMAX * KS_ / NWG;
  static_assert(TQ == 32 && KC_ == 64, "stage 1 maps V column tile w to wave w");
  __shared__ T xs[TQ * SX];
  __shared__ T ms[KC_ * SX];
  __shared__ T vs[TQ * SV];
  __shared__ T ys[CMAX * SY];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  T *part = reinterpret_cast<T *>(a.partial);
  const T *zp = reinterpret_cast<const T *>(a.zero);

  for (;;) {
    if (tid == 0) s_item = atomicAdd(a.queue, 1);
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
      T r1[NX + NM];
      T r2[NY];
      auto load1 = [&](const TaskOps &o, int c0, int k0) {
        if (o.X.sk == 1 || o.X.ident) tload<T, TQ, KK_, NX, true, 1>(r1, o.X, p0, k0, zp);
        else tload<T, TQ, KK_, NX, false, 1>(r1, o.X, p0, k0, zp);
        if (o.M.sk == 1) tload<T, KK_, KC_, NM, true, 0>(r1 + NX, o.M, k0, c0, zp);
        else tload<T, KK_, KC_, NM, false, 0>(r1 + NX, o.M, k0, c0, zp);
      };
      auto store1 = [&](const TaskOps &o) {
        if (o.X.sk == 1 || o.X.ident) tstore<T, TQ, KK_, NX, true, false, SX>(xs, r1);
        else tstore<T, TQ, KK_, NX, false, false, SX>(xs, r1);
        if (o.M.sk == 1) tstore<T, KK_, KC_, NM, true, true, SX>(ms, r1 + NX);
        else tstore<T, KK_, KC_, NM, false, true, SX>(ms, r1 + NX);
      };
      auto load2 = [&](const TaskOps &o, int c) {
        if (o.Y.sk == 1 || o.Y.ident) tload<T, CMAX, KS_, NY, true, 1>(r2, o.Y, ct0, c, zp);
        else tload<T, CMAX, KS_, NY, false, 1>(r2, o.Y, ct0, c, zp);
      };
      auto store2 = [&](const TaskOps &o) {
        if (o.Y.sk == 1 || o.Y.ident) tstore<T, CMAX, KS_, NY, true, false, SY>(ys, r2);
        else tstore<T, CMAX, KS_, NY, false, false, SY>(ys, r2);
      };

      int ti = it.tb, c0 = 0;
      TaskOps ops = task_ops_p<T>(a, a.tasks[a.idx[ti]], it.mode);
      load1(ops, 0, 0);
      for (;;) {
        // ---- stage 1 -------------------------------------------------------------
        V4 vacc[NRT];
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) vacc[rt] = vzero<V4>();
        for (int k0 = 0; k0 < ops.K1; k0 += KK_) {
          __syncthreads();
          store1(ops);
          __syncthreads();
          if (k0 + KK_ < ops.K1) load1(ops, c0, k0 + KK_);
          else load2(ops, c0);
#pragma unroll
          for (int kk = 0; kk < KK_; kk += 4) {
            const T bv = ms[(w * 16 + l16) * SX + kk + lg];
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) vacc[rt] = mfma(xs[(rt * 16 + l16) * SX + kk + lg], bv, vacc[rt]);
          }
        }
        // publish alpha V: wave w owns V column tile w (the previous chunk's
        // stage-2 reads of vs ended before the barriers of this stage 1)
        {
          const T al = (T)ops.alpha;
#pragma unroll
          for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) vs[(rt * 16 + lg * 4 + v) * SV + w * 16 + l16] = al * vacc[rt][v];
        }
        // next chunk / task, for the prefetch at the end of stage 2
        int nc0 = c0 + KC_, nti = ti;
        if (nc0 >= ops.K2) { nti = ti + 1; nc0 = 0; }
        const bool more = nti < it.te;
        TaskOps nops = ops;
        if (more && nti != ti) nops = task_ops_p<T>(a, a.tasks[a.idx[nti]], it.mode);
        // ---- stage 2 -------------------------------------------------------------
        const int send = min(KC_, ops.K2 - c0);
        for (int s2 = 0; s2 < send; s2 += KS_) {
          __syncthreads();
          store2(ops);
          __syncthreads();
          if (s2 + KS_ < send) load2(ops, c0 + s2 + KS_);
          else if (more) load1(nops, nc0, 0);
#pragma unroll
          for (int kc = 0; kc < KS_; kc += 4) {
            T av[NRT];
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) av[rt] = vs[(rt * 16 + l16) * SV + s2 + kc + lg];
#pragma unroll
            for (int u = 0; u < NU; ++u) {
              if (w + 4 * u < njt) {
                const T bv = ys[((w + 4 * u) * 16 + l16) * SY + kc + lg];
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) acc[rt][u] = mfma(av[rt], bv, acc[rt][u]);
              }
            }
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
              const int row = rt * 16 + lg * 4 + v;
              const int col = ct0 + jt * 16 + l16;
              if (row < it.np && col < Ctot) {
                const int64_t idx = it.mode == M_FWD1 ? ((int64_t)col * Rtot + p0 + row)
                                                      : ((int64_t)(p0 + row) * Ctot + col);
                slot[idx] = acc[rt][u][v];
              }
            }
          }
        }
      __syncthreads();  // LDS reuse by the next pass / item
    }
  }
}

// ---------------------------------------------------------------------------
// persistent kernel, split BF16 (three products, FP32 accumulation)
//
// Same step pipeline as k_apply; operands are (hi, lo) BF16 pairs, packed in
// registers as hi | lo << 16 and stored in separate LDS planes so that one
// 16-byte LDS read feeds an MFMA operand (8 consecutive k).
// ---------------------------------------------------------------------------
constexpr int BKK = 64, BKC = 64, BKS = 32, BPAD = 8;

__device__ inline View bview(const ApplyArgs &a, View v) {
  const uint16_t *h = (const uint16_t *)(v.src == 0 ? a.ops : a.psi);
  v.p = h + v.off;
  return v;
}

__device__ inline TaskOps task_ops_bf(const ApplyArgs &a, const tns_task &t, int mode) {
  TaskOps o = task_ops(a, t, mode);
  o.X = bview(a, o.X);
  o.M = bview(a, o.M);
  o.Y = bview(a, o.Y);
  return o;
}

// As tload, for split BF16: the lo plane sits `plane` elements after the hi
// plane of the same array.
template <int R, int CC, int N, bool CFAST, int KDIM>
__device__ inline void tload_bf(uint32_t *rh, uint32_t *rl, const View &v, int i0, int k0, int64_t plane_ops,
                                int64_t plane_psi, const uint16_t *zp) {
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const uint16_t *h = (const uint16_t *)v.p;
  const uint16_t *l = h + (v.src == 0 ? plane_ops : plane_psi);
  const int si = v.si, sk = v.sk, rmax = v.rows - 1, cmax = v.cols - 1;
  if (v.ident) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      int r, c;
      tile_rc<R, CC, CFAST>(tid, j, &r, &c);
      const int i = i0 + r, k = k0 + c;
      rh[j] = (i == k && i <= rmax && k <= cmax) ? 0x3f80u : 0u;
      rl[j] = 0u;
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
    const int off = ic * si + kc * sk;
    rh[j] = *(in ? h + off : zp);
    rl[j] = *(in ? l + off : zp);
  }
}

template <int R, int CC, int N, bool CFAST, bool TRANS, int S, int PL>
__device__ inline void tstore_bf(uint16_t *lds, const uint32_t *rh, const uint32_t *rl) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    int r, c;
    tile_rc<R, CC, CFAST>(tid, j, &r, &c);
    const int o = TRANS ? c * S + r : r * S + c;
    lds[o] = (uint16_t)rh[j];
    lds[PL + o] = (uint16_t)rl[j];
  }
}

struct __attribute__((aligned(16))) SmemBF {
  uint16_t x[2 * TQ * (BKK + BPAD)];
  uint16_t m[2 * BKC * (BKK + BPAD)];
  uint16_t v[2 * TQ * (BKC + BPAD)];
  uint16_t y[2 * CMAX * (BKS + BPAD)];
};

__global__ __launch_bounds__(NWG) void k_apply_bf16x3(ApplyArgs a) {
  constexpr int SX = BKK + BPAD, SV = BKC + BPAD, SY = BKS + BPAD;
  constexpr int PX = TQ * SX, PM = BKC * SX, PV = TQ * SV, PY = CMAX * SY;
  constexpr int NRT = TQ / 16, NU = CMAX / 64;
  constexpr int NX = TQ * BKK / NWG, NM = BKK * BKC / NWG, NY = CMAX * BKS / NWG;
  __shared__ SmemBF sm;
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  float *part = reinterpret_cast<float *>(a.partial);
  const int64_t pl_ops = a.n_vals, pl_psi = a.psi_dim;
  const uint16_t *zp = reinterpret_cast<const uint16_t *>(a.zero);

  for (;;) {
    if (tid == 0) s_item = atomicAdd(a.queue, 1);
    __syncthreads();
    const int wi = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (wi >= a.nitems) break;
    const Item it = a.items[wi];
    int Rtot, Ctot;
    out_dims(a, it, &Rtot, &Ctot);
    float *slot = part + a.slot_off[it.slot];
    const int p0 = it.p0;
    for (int ct0 = 0; ct0 < Ctot; ct0 += CMAX) {
      const int Cn = min(CMAX, Ctot - ct0);
      const int njt = (Cn + 15) >> 4;
      f4 acc[NRT][NU];
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int u = 0; u < NU; ++u) acc[rt][u] = vzero<f4>();
      uint32_t r1h[NX + NM], r1l[NX + NM];
      uint32_t r2h[NY], r2l[NY];
      auto load1 = [&](const TaskOps &o, int c0, int k0) {
        if (o.X.sk == 1 || o.X.ident) tload_bf<TQ, BKK, NX, true, 1>(r1h, r1l, o.X, p0, k0, pl_ops, pl_psi, zp);
        else tload_bf<TQ, BKK, NX, false, 1>(r1h, r1l, o.X, p0, k0, pl_ops, pl_psi, zp);
        if (o.M.sk == 1) tload_bf<BKK, BKC, NM, true, 0>(r1h + NX, r1l + NX, o.M, k0, c0, pl_ops, pl_psi, zp);
        else tload_bf<BKK, BKC, NM, false, 0>(r1h + NX, r1l + NX, o.M, k0, c0, pl_ops, pl_psi, zp);
      };
      auto store1 = [&](const TaskOps &o) {
        if (o.X.sk == 1 || o.X.ident) tstore_bf<TQ, BKK, NX, true, false, SX, PX>(sm.x, r1h, r1l);
        else tstore_bf<TQ, BKK, NX, false, false, SX, PX>(sm.x, r1h, r1l);
        if (o.M.sk == 1) tstore_bf<BKK, BKC, NM, true, true, SX, PM>(sm.m, r1h + NX, r1l + NX);
        else tstore_bf<BKK, BKC, NM, false, true, SX, PM>(sm.m, r1h + NX, r1l + NX);
      };
      auto load2 = [&](const TaskOps &o, int c) {
        if (o.Y.sk == 1 || o.Y.ident) tload_bf<CMAX, BKS, NY, true, 1>(r2h, r2l, o.Y, ct0, c, pl_ops, pl_psi, zp);
        else tload_bf<CMAX, BKS, NY, false, 1>(r2h, r2l, o.Y, ct0, c, pl_ops, pl_psi, zp);
      };
      auto store2 = [&](const TaskOps &o) {
        if (o.Y.sk == 1 || o.Y.ident) tstore_bf<CMAX, BKS, NY, true, false, SY, PY>(sm.y, r2h, r2l);
        else tstore_bf<CMAX, BKS, NY, false, false, SY, PY>(sm.y, r2h, r2l);
      };

      int ti = it.tb, c0 = 0;
      TaskOps ops = task_ops_bf(a, a.tasks[a.idx[ti]], it.mode);
      load1(ops, 0, 0);
      for (;;) {
        f4 vacc[NRT];
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) vacc[rt] = vzero<f4>();
        for (int k0 = 0; k0 < ops.K1; k0 += BKK) {
          __syncthreads();
          store1(ops);
          __syncthreads();
          if (k0 + BKK < ops.K1) load1(ops, c0, k0 + BKK);
          else load2(ops, c0);
#pragma unroll
          for (int kk = 0; kk < BKK; kk += 32) {
            const int mo = (w * 16 + l16) * SX + kk + 8 * lg;
            const u16x8 bh = *reinterpret_cast<const u16x8 *>(&sm.m[mo]);
            const u16x8 bl = *reinterpret_cast<const u16x8 *>(&sm.m[PM + mo]);
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) {
              const int xo = (rt * 16 + l16) * SX + kk + 8 * lg;
              const u16x8 ah = *reinterpret_cast<const u16x8 *>(&sm.x[xo]);
              const u16x8 al = *reinterpret_cast<const u16x8 *>(&sm.x[PX + xo]);
              vacc[rt] = mfma_bf(al, bh, vacc[rt]);
              vacc[rt] = mfma_bf(ah, bl, vacc[rt]);
              vacc[rt] = mfma_bf(ah, bh, vacc[rt]);
            }
          }
        }
        {
          const float al = (float)ops.alpha;
#pragma unroll
          for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const float x = al * vacc[rt][v];
              const uint16_t h = f32_to_bf16_rne(x);
              const int o = (rt * 16 + lg * 4 + v) * SV + w * 16 + l16;
              sm.v[o] = h;
              sm.v[PV + o] = f32_to_bf16_rne(x - bf16_to_f32(h));
            }
        }
        int nc0 = c0 + BKC, nti = ti;
        if (nc0 >= ops.K2) { nti = ti + 1; nc0 = 0; }
        const bool more = nti < it.te;
        TaskOps nops = ops;
        if (more && nti != ti) nops = task_ops_bf(a, a.tasks[a.idx[nti]], it.mode);
        const int send = min(BKC, ops.K2 - c0);
        for (int s2 = 0; s2 < send; s2 += BKS) {
          __syncthreads();
          store2(ops);
          __syncthreads();
          if (s2 + BKS < send) load2(ops, c0 + s2 + BKS);
          else if (more) load1(nops, nc0, 0);
          u16x8 ah[NRT], al[NRT];
#pragma unroll
          for (int rt = 0; rt < NRT; ++rt) {
            const int vo = (rt * 16 + l16) * SV + s2 + 8 * lg;
            ah[rt] = *reinterpret_cast<const u16x8 *>(&sm.v[vo]);
            al[rt] = *reinterpret_cast<const u16x8 *>(&sm.v[PV + vo]);
          }
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            if (w + 4 * u < njt) {
              const int yo = ((w + 4 * u) * 16 + l16) * SY + 8 * lg;
              const u16x8 bh = *reinterpret_cast<const u16x8 *>(&sm.y[yo]);
              const u16x8 bl = *reinterpret_cast<const u16x8 *>(&sm.y[PY + yo]);
#pragma unroll
              for (int rt = 0; rt < NRT; ++rt) {
                acc[rt][u] = mfma_bf(al[rt], bh, acc[rt][u]);
                acc[rt][u] = mfma_bf(ah[rt], bl, acc[rt][u]);
                acc[rt][u] = mfma_bf(ah[rt], bh, acc[rt][u]);
              }
            }
          }
        }
        if (!more) break;
        ti = nti;
        c0 = nc0;
        ops = nops;
      }
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int jt = w + 4 * u;
          if (jt < njt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = rt * 16 + lg * 4 + v;
              const int col = ct0 + jt * 16 + l16;
              if (row < it.np && col < Ctot) {
                const int64_t idx = it.mode == M_FWD1 ? ((int64_t)col * Rtot + p0 + row)
                                                      : ((int64_t)(p0 + row) * Ctot + col);
                slot[idx] = acc[rt][u][v];
              }
            }
          }
        }
      __syncthreads();
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
                               const T *__restrict__ part, T *__restrict__ out, int64_t psi_dim, int beta) {
  GRID_STRIDE(e, psi_dim) {
    int lo = 0, hi = nS;  // s with psi_off[s] <= e < psi_off[s+1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (psi_off[mid] <= e) lo = mid; else hi = mid;
    }
    const int s = lo;
    const int64_t loc = e - psi_off[s];
    double acc = beta ? (double)out[e] : 0.0;
    const int64_t c0 = grp_chunk_base[gps * s], c1 = grp_chunk_base[gps * s + gps];
    for (int64_t c = c0; c < c1; ++c) acc += (double)part[slot_off[c] + loc];
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
  const int64_t n = (int64_t)rows * cols;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    double acc = 0.0;
    for (int64_t c = c0; c < c1; ++c) acc += (double)part[slot_off[c] + e];
    out[blk_off[b] + (e / cols) * ld + (e % cols)] = (T)acc;
  }
}

// queue counter and the 64-byte zero region that out-of-range loads read
__global__ void k_reset_head(int32_t *p) {
  if (threadIdx.x < 32) p[threadIdx.x] = 0;
}

template <class T>
__global__ void k_zero(T *p, int64_t n) {
  GRID_STRIDE(i, n) p[i] = T(0);
}

__global__ void k_split_f32(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ hi, uint16_t *__restrict__ lo) {
  GRID_STRIDE(i, n) {
    const float v = x[i];
    const uint16_t h = f32_to_bf16_rne(v);
    hi[i] = h;
    lo[i] = f32_to_bf16_rne(v - bf16_to_f32(h));
  }
}

__global__ void k_split_f64(const double *__restrict__ x, int64_t n, uint16_t *__restrict__ hi,
                            uint16_t *__restrict__ lo) {
  GRID_STRIDE(i, n) {
    const float v = (float)x[i];
    const uint16_t h = f32_to_bf16_rne(v);
    hi[i] = h;
    lo[i] = f32_to_bf16_rne(v - bf16_to_f32(h));
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

// Workspace: [queue counter | partial slots | (BF16X3) psi hi, lo]
static size_t apply_ws(const Sched &S, int64_t psi_dim, tns_prec prec) {
  size_t b = 256;
  b += align_up((size_t)std::max<int64_t>(S.partial_elems, 1) * elem_bytes(prec), 256);
  if (prec == TNS_BF16X3) b += align_up((size_t)psi_dim * 2 * sizeof(uint16_t), 256);
  return b;
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
  a.psi_sec = p.psi_sec; a.dimL = p.dimL; a.dimR = p.dimR; a.psi_off = p.psi_off; a.blk_off = p.blk_off;
  a.slot_off = S.slot_off; a.blk_ld = p.blk_ld; a.blk_rows = p.blk_rows; a.blk_cols = p.blk_cols;
  a.ops = ops; a.psi = psi; a.grad = grad; a.partial = part;
  a.n_vals = p.n_vals; a.psi_dim = p.psi_dim;
  a.mode_mask = 0x1f;
  a.zero = reinterpret_cast<const char *>(queue) + 64;
  return a;
}

static hipEvent_t g_ev_before = nullptr, g_ev_after = nullptr;

tns_status apply_impl(const Plan &p, tns_prec prec, const void *ops, const void *psi, void *sigma, double beta,
                      void *ws, size_t ws_bytes, hipStream_t st) {
  hipEvent_t evb = g_ev_before, eva = g_ev_after;
  g_ev_before = g_ev_after = nullptr;
  const Sched &S = p.fwd;
  if (ws_bytes < apply_ws(S, p.psi_dim, prec)) return TNS_ERR_WORKSPACE;
  char *w = reinterpret_cast<char *>(ws);
  int32_t *queue = reinterpret_cast<int32_t *>(w);
  void *part = w + 256;
  const size_t pbytes = align_up((size_t)std::max<int64_t>(S.partial_elems, 1) * elem_bytes(prec), 256);
  ApplyArgs a = make_args(p, S, ops, psi, nullptr, part, queue);
  const int ibeta = beta != 0.0;
  hipLaunchKernelGGL(k_reset_head, dim3(1), dim3(32), 0, st, queue);
  if (prec == TNS_F64) {
    if (evb && eva) TNS_HIP(hipEventRecord(evb, st));
    if (S.nitems > 0)
      hipLaunchKernelGGL(k_apply<TNS_F64>, dim3(grid_for(k_apply<TNS_F64>, p.n_cu)), dim3(NWG), 0, st, a);
    if (evb && eva) TNS_HIP(hipEventRecord(eva, st));
    hipLaunchKernelGGL(k_epilogue_psi<double>, dim3(nb(p.psi_dim, 256)), dim3(256), 0, st, p.psi_off, p.nS, 2,
                       S.grp_chunk_base, S.slot_off, (const double *)part, (double *)sigma, p.psi_dim, ibeta);
  } else if (prec == TNS_F32) {
    if (evb && eva) TNS_HIP(hipEventRecord(evb, st));
    if (S.nitems > 0)
      hipLaunchKernelGGL(k_apply<TNS_F32>, dim3(grid_for(k_apply<TNS_F32>, p.n_cu)), dim3(NWG), 0, st, a);
    if (evb && eva) TNS_HIP(hipEventRecord(eva, st));
    hipLaunchKernelGGL(k_epilogue_psi<float>, dim3(nb(p.psi_dim, 256)), dim3(256), 0, st, p.psi_off, p.nS, 2,
                       S.grp_chunk_base, S.slot_off, (const float *)part, (float *)sigma, p.psi_dim, ibeta);
  } else {
    uint16_t *psplit = reinterpret_cast<uint16_t *>(w + 256 + pbytes);
    hipLaunchKernelGGL(k_split_f32, dim3(nb(p.psi_dim, 256)), dim3(256), 0, st, (const float *)psi, p.psi_dim,
                       psplit, psplit + p.psi_dim);
    a.psi = psplit;
    if (evb && eva) TNS_HIP(hipEventRecord(evb, st));
    if (S.nitems > 0)
      hipLaunchKernelGGL(k_apply_bf16x3, dim3(grid_for(k_apply_bf16x3, p.n_cu)), dim3(NWG), 0, st, a);
    if (evb && eva) TNS_HIP(hipEventRecord(eva, st));
    hipLaunchKernelGGL(k_epilogue_psi<float>, dim3(nb(p.psi_dim, 256)), dim3(256), 0, st, p.psi_off, p.nS, 2,
                       S.grp_chunk_base, S.slot_off, (const float *)part, (float *)sigma, p.psi_dim, ibeta);
  }
  return hipGetLastError() == hipSuccess ? TNS_OK : TNS_ERR_HIP;
}

template <int P>
static tns_status backward_impl(const Plan &p, const void *ops, const void *psi, const void *G, void *gpsi,
                                void *gops, void *ws, hipStream_t st) {
  typedef typename Prec<P>::acc T;
  const Sched &S = p.bwd;
  char *w = reinterpret_cast<char *>(ws);
  int32_t *queue = reinterpret_cast<int32_t *>(w);
  T *part = reinterpret_cast<T *>(w + 256);
  ApplyArgs a = make_args(p, S, ops, psi, G, part, queue);
  a.mode_mask = (gpsi ? (1 << M_DPSI) : 0) | (gops ? ((1 << M_DL) | (1 << M_DR)) : 0);
  hipLaunchKernelGGL(k_reset_head, dim3(1), dim3(32), 0, st, queue);
  if (S.nitems > 0) hipLaunchKernelGGL(k_apply<P>, dim3(grid_for(k_apply<P>, p.n_cu)), dim3(NWG), 0, st, a);
  if (gpsi)
    hipLaunchKernelGGL(k_epilogue_psi<T>, dim3(nb(p.psi_dim, 256)), dim3(256), 0, st, p.psi_off, p.nS, 1,
                       S.grp_chunk_base, S.slot_off, (const T *)part, (T *)gpsi, p.psi_dim, 0);
  if (gops) {
    hipLaunchKernelGGL(k_zero<T>, dim3(nb(p.n_vals, 256)), dim3(256), 0, st, (T *)gops, p.n_vals);
    if (p.nBlk > 0)
      hipLaunchKernelGGL(k_epilogue_blk<T>, dim3(p.nBlk), dim3(256), 0, st, p.nS, S.grp_chunk_base, S.slot_off,
                         p.blk_off, p.blk_rows, p.blk_cols, p.blk_ld, (const T *)part, (T *)gops);
  }
  return hipGetLastError() == hipSuccess ? TNS_OK : TNS_ERR_HIP;
}

}  // namespace tns

using namespace tns;

extern "C" size_t tns_apply_workspace_bytes(const tns_tasklist *tl, tns_prec prec) {
  if (!tl || (prec != TNS_F64 && prec != TNS_F32 && prec != TNS_BF16X3)) return 0;
  const Plan &p = plan_of(tl);
  return apply_ws(p.fwd, p.psi_dim, prec);
}

extern "C" tns_status tns_prepare_operands(tns_prec prec, const double *vals64, int64_t n, void *out, hipStream_t st) {
  if (!vals64 || !out || n < 0) return TNS_ERR_ARG;
  if (n == 0) return TNS_OK;
  if (prec == TNS_F64) {
    hipLaunchKernelGGL(k_copy_f64, dim3(nb(n, 256)), dim3(256), 0, st, vals64, n, (double *)out);
  } else if (prec == TNS_F32) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(nb(n, 256)), dim3(256), 0, st, vals64, n, (float *)out);
  } else if (prec == TNS_BF16X3) {
    uint16_t *h = (uint16_t *)out;
    hipLaunchKernelGGL(k_split_f64, dim3(nb(n, 256)), dim3(256), 0, st, vals64, n, h, h + n);
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

extern "C" void tns_profile_events(hipEvent_t before, hipEvent_t after) {
  g_ev_before = before;
  g_ev_after = after;
}

extern "C" size_t tns_backward_workspace_bytes(const tns_tasklist *tl, tns_prec prec) {
  if (!tl || (prec != TNS_F64 && prec != TNS_F32)) return 0;
  const Plan &p = plan_of(tl);
  return apply_ws(p.bwd, p.psi_dim, prec);
}

extern "C" tns_status tns_apply_heff_backward(const tns_tasklist *tl, tns_prec prec, const void *op_vals,
                                              const void *psi, const void *grad_sigma, void *grad_psi,
                                              void *grad_ops, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!tl || !op_vals || !psi || !grad_sigma || !ws) return TNS_ERR_ARG;
  if (prec != TNS_F64 && prec != TNS_F32) return TNS_ERR_ARG;
  const Plan &p = plan_of(tl);
  if (ws_bytes < apply_ws(p.bwd, p.psi_dim, prec)) return TNS_ERR_WORKSPACE;
  if (!grad_psi && !grad_ops) return TNS_OK;
  if (prec == TNS_F64) return backward_impl<TNS_F64>(p, op_vals, psi, grad_sigma, grad_psi, grad_ops, ws, st);
  return backward_impl<TNS_F32>(p, op_vals, psi, grad_sigma, grad_psi, grad_ops, ws, st);
}
