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
};

// Operand view of one matrix for the loaders: element (i, k) at
// base[i * si + k * sk]; identity when `ident`.
struct View {
  int64_t off;   // element offset
  int64_t si, sk;
  int rows, cols;
  int ident;
  int src;       // 0 = operator values, 1 = psi, 2 = grad sigma
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
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(NWG) void k_apply(ApplyArgs a) {
  typedef typename Prec<P>::acc T;
  typedef typename Prec<P>::accv V4;
  constexpr int S = Prec<P>::S;
  constexpr int SV = KC + 2;
  constexpr int NU = CMAX / 64;  // column tiles per wave
  __shared__ TileStore<P> sm;
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  Bases<T> src;
  src.ops = reinterpret_cast<const T *>(a.ops);
  src.psi = reinterpret_cast<const T *>(a.psi);
  src.grad = reinterpret_cast<const T *>(a.grad);
  T *part = reinterpret_cast<T *>(a.partial);

  for (;;) {
    if (tid == 0) s_item = atomicAdd(a.queue, 1);
    __syncthreads();
    const int wi = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (wi >= a.nitems) break;
    const Item it = a.items[wi];
    if (!((a.mode_mask >> it.mode) & 1)) continue;
    int Rtot, C;
    out_dims(a, it, &Rtot, &C);
    T *slot = part + a.slot_off[it.slot];
    for (int ct0 = 0; ct0 < C; ct0 += CMAX) {
      const int Cn = min(CMAX, C - ct0);
      const int njt = (Cn + 15) >> 4;
      V4 acc[2][NU];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int u = 0; u < NU; ++u) acc[rt][u] = vzero<V4>();

      for (int ti = it.tb; ti < it.te; ++ti) {
        const tns_task tk = a.tasks[a.idx[ti]];
        const TaskOps o = task_ops(a, tk, it.mode);
        const T alpha = (T)o.alpha;
        for (int c0 = 0; c0 < o.K2; c0 += KC) {
          // ---- stage 1: V = X[p0.., :] M[:, c0..] ------------------------
          V4 vacc = vzero<V4>();
          const int rt1 = w & 1, ct1 = w >> 1;
          for (int k0 = 0; k0 < o.K1; k0 += KK) {
            load_tile(sm.x, S, TQ, KK, src, o.X, it.p0, k0);
            // M chunk stored transposed: m[c][k] = M(k0 + k, c0 + c)
            load_tile(sm.m, S, KC, KK, src, transposed(o.M), c0, k0);
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < KK; kk += 4) {
              const T av = sm.x[(rt1 * 16 + l16) * S + kk + lg];
              const T bv = sm.m[(ct1 * 16 + l16) * S + kk + lg];
              vacc = mfma(av, bv, vacc);
            }
            __syncthreads();
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) sm.v[(rt1 * 16 + lg * 4 + v) * SV + ct1 * 16 + l16] = alpha * vacc[v];
          // ---- stage 2: acc += V Y[:, c0..]^T, Y staged YG columns at a time
          for (int g0 = 0; g0 < Cn; g0 += YG) {
            __syncthreads();
            load_tile(sm.y, SV, min(YG, (Cn - g0 + 15) & ~15), KC, src, o.Y, ct0 + g0, c0);
            __syncthreads();
#pragma unroll
            for (int kc = 0; kc < KC; kc += 4) {
              const T a0 = sm.v[(0 * 16 + l16) * SV + kc + lg];
              const T a1 = sm.v[(1 * 16 + l16) * SV + kc + lg];
#pragma unroll
              for (int u = 0; u < NU; ++u) {
                const int jt = w + 4 * u;  // global column tile within the pass
                if (jt * 16 >= g0 && jt * 16 < g0 + YG && jt < njt) {
                  const T bv = sm.y[(jt * 16 - g0 + l16) * SV + kc + lg];
                  acc[0][u] = mfma(a0, bv, acc[0][u]);
                  acc[1][u] = mfma(a1, bv, acc[1][u]);
                }
              }
            }
          }
          __syncthreads();
        }
      }
      // ---- write the panel into the partial slot -----------------------------
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int jt = w + 4 * u;
          if (jt < njt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = rt * 16 + lg * 4 + v;
              const int col = ct0 + jt * 16 + l16;
              if (row < it.np && col < C) {
                const int64_t idx = it.mode == M_FWD1 ? ((int64_t)col * Rtot + it.p0 + row)
                                                      : ((int64_t)(it.p0 + row) * C + col);
                slot[idx] = acc[rt][u][v];
              }
            }
          }
        }
    }
  }
}

// ---------------------------------------------------------------------------
// persistent kernel, split BF16 (three products, FP32 accumulation)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NWG) void k_apply_bf16x3(ApplyArgs a) {
  constexpr int S = KK + 8;
  constexpr int SV = KC + 8;
  constexpr int NU = CMAX / 64;
  __shared__ TileStoreBF sm;
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  const uint16_t *oh = reinterpret_cast<const uint16_t *>(a.ops);
  const uint16_t *ol = oh + a.n_vals;
  const uint16_t *ph = reinterpret_cast<const uint16_t *>(a.psi);
  const uint16_t *pl = ph + a.psi_dim;
  float *part = reinterpret_cast<float *>(a.partial);

  for (;;) {
    if (tid == 0) s_item = atomicAdd(a.queue, 1);
    __syncthreads();
    const int wi = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (wi >= a.nitems) break;
    const Item it = a.items[wi];
    int Rtot, C;
    out_dims(a, it, &Rtot, &C);
    float *slot = part + a.slot_off[it.slot];
    for (int ct0 = 0; ct0 < C; ct0 += CMAX) {
      const int Cn = min(CMAX, C - ct0);
      const int njt = (Cn + 15) >> 4;
      f4 acc[2][NU];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int u = 0; u < NU; ++u) acc[rt][u] = vzero<f4>();

      for (int ti = it.tb; ti < it.te; ++ti) {
        const tns_task tk = a.tasks[a.idx[ti]];
        const TaskOps o = task_ops(a, tk, it.mode);
        const float alpha = (float)o.alpha;
        for (int c0 = 0; c0 < o.K2; c0 += KC) {
          f4 vacc = vzero<f4>();
          const int rt1 = w & 1, ct1 = w >> 1;
          for (int k0 = 0; k0 < o.K1; k0 += KK) {
            load_tile_bf(sm.xh, sm.xl, S, TQ, KK, oh, ol, o.X, it.p0, k0);
            load_tile_bf(sm.mh, sm.ml, S, KC, KK, ph, pl, transposed(o.M), c0, k0);
            __syncthreads();
            const u16x8 ah = *reinterpret_cast<const u16x8 *>(&sm.xh[(rt1 * 16 + l16) * S + 8 * lg]);
            const u16x8 al = *reinterpret_cast<const u16x8 *>(&sm.xl[(rt1 * 16 + l16) * S + 8 * lg]);
            const u16x8 bh = *reinterpret_cast<const u16x8 *>(&sm.mh[(ct1 * 16 + l16) * S + 8 * lg]);
            const u16x8 bl = *reinterpret_cast<const u16x8 *>(&sm.ml[(ct1 * 16 + l16) * S + 8 * lg]);
            vacc = mfma_bf(al, bh, vacc);
            vacc = mfma_bf(ah, bl, vacc);
            vacc = mfma_bf(ah, bh, vacc);
            __syncthreads();
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float x = alpha * vacc[v];
            const uint16_t h = f32_to_bf16_rne(x);
            const uint16_t l = f32_to_bf16_rne(x - bf16_to_f32(h));
            const int idx = (rt1 * 16 + lg * 4 + v) * SV + ct1 * 16 + l16;
            sm.vh[idx] = h;
            sm.vl[idx] = l;
          }
          for (int g0 = 0; g0 < Cn; g0 += YG) {
            __syncthreads();
            load_tile_bf(sm.yh, sm.yl, SV, min(YG, (Cn - g0 + 15) & ~15), KC, oh, ol, o.Y, ct0 + g0, c0);
            __syncthreads();
            const u16x8 a0h = *reinterpret_cast<const u16x8 *>(&sm.vh[(0 * 16 + l16) * SV + 8 * lg]);
            const u16x8 a0l = *reinterpret_cast<const u16x8 *>(&sm.vl[(0 * 16 + l16) * SV + 8 * lg]);
            const u16x8 a1h = *reinterpret_cast<const u16x8 *>(&sm.vh[(1 * 16 + l16) * SV + 8 * lg]);
            const u16x8 a1l = *reinterpret_cast<const u16x8 *>(&sm.vl[(1 * 16 + l16) * SV + 8 * lg]);
#pragma unroll
            for (int u = 0; u < NU; ++u) {
              const int jt = w + 4 * u;
              if (jt * 16 >= g0 && jt * 16 < g0 + YG && jt < njt) {
                const int yo = (jt * 16 - g0 + l16) * SV + 8 * lg;
                const u16x8 bh = *reinterpret_cast<const u16x8 *>(&sm.yh[yo]);
                const u16x8 bl = *reinterpret_cast<const u16x8 *>(&sm.yl[yo]);
                acc[0][u] = mfma_bf(a0l, bh, acc[0][u]);
                acc[0][u] = mfma_bf(a0h, bl, acc[0][u]);
                acc[0][u] = mfma_bf(a0h, bh, acc[0][u]);
                acc[1][u] = mfma_bf(a1l, bh, acc[1][u]);
                acc[1][u] = mfma_bf(a1h, bl, acc[1][u]);
                acc[1][u] = mfma_bf(a1h, bh, acc[1][u]);
              }
            }
          }
          __syncthreads();
        }
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int jt = w + 4 * u;
          if (jt < njt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = rt * 16 + lg * 4 + v;
              const int col = ct0 + jt * 16 + l16;
              if (row < it.np && col < C) {
                const int64_t idx = it.mode == M_FWD1 ? ((int64_t)col * Rtot + it.p0 + row)
                                                      : ((int64_t)(it.p0 + row) * C + col);
                slot[idx] = acc[rt][u][v];
              }
            }
          }
        }
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
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= psi_dim) return;
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

__global__ void k_zero_i32(int32_t *p) { *p = 0; }

template <class T>
__global__ void k_zero(T *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

__global__ void k_split_f32(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ hi, uint16_t *__restrict__ lo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = x[i];
  const uint16_t h = f32_to_bf16_rne(v);
  hi[i] = h;
  lo[i] = f32_to_bf16_rne(v - bf16_to_f32(h));
}

__global__ void k_split_f64(const double *__restrict__ x, int64_t n, uint16_t *__restrict__ hi,
                            uint16_t *__restrict__ lo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = (float)x[i];
  const uint16_t h = f32_to_bf16_rne(v);
  hi[i] = h;
  lo[i] = f32_to_bf16_rne(v - bf16_to_f32(h));
}

__global__ void k_f64_to_f32(const double *__restrict__ x, int64_t n, float *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

__global__ void k_copy_f64(const double *__restrict__ x, int64_t n, double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

static inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

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
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, st, queue);
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
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, st, queue);
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
