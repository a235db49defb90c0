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
// and stores it, row-major with leading dimension ld8(K2), in the workspace.
// Phase B forms, per chunk of the task list of an output group,
//   slot = sum_k T_k Y_k^T     (class 0: Y = R;  class 1: Y = L)
// as one GEMM whose inner dimension runs through all tasks of the chunk.  The
// epilogue adds the slots of each sector in a fixed order.  This is the
// batched-GEMM arrangement of Alg. 2 (intermediates in device memory, one
// batched product per stage) with the summation over terms folded into the
// inner dimension of the second GEMM.
//
// Both phases compute tiles C(i, j) = sum over segments of sum_k A(i, k) B(j, k)
// with every operand k-contiguous (rows of L, R, T and of the padded copies of
// A and A^T).  Identity factors are never multiplied: an identity X makes T a
// scaled copy of the padded input sector (k_ident_T), an identity Y adds T
// into the phase-B accumulators directly.  Tiles are 32, 64 or 128 rows / columns per the
// tile table of the task list (per sector-size bucket), the last tile along a
// dimension 32, 64, 96 or 128 to fit what remains.  Operands stream from
// global memory straight into a 4-stage LDS ring (16-byte direct loads), the
// MFMA work consuming one stage per barrier.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "kern.hpp"
#include "tns_internal.hpp"

namespace tns {

// Threads per workgroup: FP32 / FP64 4 waves in a 2 x 2 grid of wave tiles,
// BF16X3 8 waves in a 2 x 4 grid (wider column tiles: fewer operand bytes per
// flop, two waves per SIMD).
template <int P> constexpr int gth() { return P == TNS_BF16X3 ? 512 : 256; }
// waves across the columns of a tile
template <int P> constexpr int wgn() { return P == TNS_BF16X3 ? 4 : 2; }

// Operand: element (i, k) at index i * ld + k for i < rows, k < K of the
// segment (BF16X3: of the interleaved halves, see bfx_hi).  Identity
// operators are matrices in memory too.
struct Mat {
  const void *p;
  int32_t ld, rows;
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
  const void *ops;  // F64 / F32 values, or BF16X3 halves interleaved (bfx_hi)
  const void *pp, *pt;  // padded psi (m x ld8(n)) and psi^T (n x ld8(m)) per sector
  const int64_t *pp_off, *pt_off;
  void *T;  // intermediates
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
  uint32_t tiles;     // tile table
  // phase-A panels
  const Item *a_items;
  const int64_t *a_qbase, *a_tb, *a_gch, *a_ch;
  const int32_t *a_idx;
  const ChunkRec *recs;  // chunk sources, written before phase A
  const SegRec *segb;    // phase-B segments, in the order of idx
};

// --- per-precision tile parameters ---------------------------------------------
template <int P> struct FP;
template <> struct FP<TNS_F64> {
  typedef double Acc;
  typedef double E;  // element in memory and LDS
  typedef d2 V;      // 16-byte vector
  typedef d4 A4;     // MFMA accumulator
};
template <> struct FP<TNS_F32> {
  typedef float Acc;
  typedef float E;
  typedef f4 V;
  typedef f4 A4;
};
template <> struct FP<TNS_BF16X3> {
  typedef float Acc;
  typedef uint16_t E;
  typedef u16x8 V;
  typedef f4 A4;
};

// --- work queues --------------------------------------------------------------------
// Phase A: panel items, phase B: the schedule's items; queue q of a phase is
// items[qbase[q], qbase[q+1]).  BF16X3 takes the lists built at the tile
// table as given (up to 256 columns per item), FP32 / FP64 those built at its
// narrow form (up to 128).
// Thread 0: next item of phase PH (own XCD queue first), -1 when drained.
template <int PH>
__device__ inline int pop_work(const FwdArgs &g) {
  const int home = blockIdx.x % g.nq;
  const int64_t *qb = PH == 0 ? g.a_qbase : g.qbase;
  for (int k = 0; k < g.nq; ++k) {
    const int q = home + k < g.nq ? home + k : home + k - g.nq;
    const int64_t b = qb[q], n = qb[q + 1] - b;
    if (n <= 0) continue;
    const int j = atomicAdd(g.queue + 8 * PH + q, 1);
    if (j < n) return (int)(b + j);
  }
  return -1;
}

// --- the LDS ring: direct global -> LDS loads, NS stages ----------------------------
// A stage holds the 128 x BK tiles of A and of B as 1 KB chunks, each the
// target of one global_load_lds_dwordx4 of a wave.  FP32 [A, B] (BK = 16) and
// FP64 [A, B] (BK = 8): arrays of 8 chunks of 16 rows x 64 bytes (4 16-byte
// k-vectors), 16 KB per stage, so that two workgroups share a CU; the
// k-vectors of row r sit at slots kv ^ ((r >> 1) & 3).  BF16X3 (BK = 32):
// chunks of 8 rows x 128 bytes, the interleaved high and low halves of 32 k,
// so that every row of a stage is one whole 128-byte line in memory; 16
// chunks for the 128 rows of A, 32 for the up to 256 rows of B; vector v of
// row r sits at slot v ^ (r & 7); 48 KB per stage, three stages, one
// workgroup of 8 waves per CU.  Either way the 16 rows read by one MFMA
// operand fetch fall into distinct LDS banks.  Loads run NS - 1 stages ahead of the MFMA
// work; a stage is consumed after a counted vector-memory wait and one
// barrier (no fence, in-flight stages stay in flight).  Out-of-range rows and
// whole k-vectors beyond K read the zero region; the library's own operands
// (T, padded psi) hold zeros beyond K, so the k-tail of an operator row
// always meets zeros.
typedef __bf16 bfx4 __attribute__((ext_vector_type(4)));
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// KS: k-halves per stage of FP32 / FP64 (each half 4 k-vectors of 16 bytes
// per row, one array of chunks per operand and half); BF16X3 uses KS = 1 and
// two halves of precision instead.
template <int P> struct RingP;
template <> struct RingP<TNS_BF16X3> { static constexpr int VEC = 8; };
template <> struct RingP<TNS_F32> { static constexpr int VEC = 4; };
template <> struct RingP<TNS_F64> { static constexpr int VEC = 2; };
template <int P, int KS> struct RingL {
  static constexpr int ARR = 2 * KS;                           // FP32 / FP64: arrays of 8 chunks
  static constexpr int CH = P == TNS_BF16X3 ? 48 : 8 * ARR;    // chunks per stage (BF16X3: A 16, B 32)
  static constexpr int LOADS = CH / 4;                         // FP32 / FP64 loads per wave and stage
  static constexpr int BK = P == TNS_BF16X3 ? 32 : KS * 4 * RingP<P>::VEC;
};
// The NS stages (2 to 5) are separate LDS arrays and every access names its
// stage at compile time (the stage loop is unrolled NS times): the compiler
// then tells the direct loads into one stage from the operand reads of
// another and does not drain the ring before each stage's reads.
template <int P, int KS> struct __attribute__((aligned(16))) Stage {
  uint8_t b[RingL<P, KS>::CH * 1024];
};
struct __attribute__((aligned(16))) NoStage {
  uint8_t b[16];
};
// Stage J of a ring of NS stages (a 16-byte placeholder when J >= NS).
template <int P, int KS, int NS, int J>
using StageJ = typename std::conditional<(J < NS), Stage<P, KS>, NoStage>::type;
template <int P, int KS, int NS> struct Ring {
  static_assert(NS >= 2 && NS <= 5, "two to five stages");
  Stage<P, KS> &s0, &s1;
  StageJ<P, KS, NS, 2> &s2;
  StageJ<P, KS, NS, 3> &s3;
  StageJ<P, KS, NS, 4> &s4;
};
template <int J, int P, int KS, int NS>
__device__ inline Stage<P, KS> &stage(Ring<P, KS, NS> &r) {
  static_assert(J < NS, "stage of the ring");
  if constexpr (J == 0) return r.s0;
  else if constexpr (J == 1) return r.s1;
  else if constexpr (J == 2) return r.s2;
  else if constexpr (J == 3) return r.s3;
  else return r.s4;
}
__device__ inline int rswz(int rin) { return (rin >> 1) & 3; }

// Output pointers as global-memory pointers: stores through them are global
// stores (not flat ones, which the compiler orders after LDS traffic).
template <class T>
__device__ inline __attribute__((address_space(1))) T *gptr(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

// Address of element e of an operand array: BF16X3 arrays interleave the
// halves (element e's high half at bfx_hi(e), its low half 8 further), so
// row starts (e a multiple of 8) map to u16 index 2 e.
template <int P>
__device__ inline const void *elem_ptr(const void *base, int64_t e) {
  typedef typename FP<P>::E E;
  if constexpr (P == TNS_BF16X3) return reinterpret_cast<const uint16_t *>(base) + 2 * e;
  else return reinterpret_cast<const E *>(base) + e;
}

__device__ inline void gl_lds(const void *src, void *dst) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                   (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
}

// Waits until at most NS - 2 stages of this wave's ring loads are in flight
// (vector-memory loads complete in order) and, with LGKM, until its LDS reads
// are complete, then joins the workgroup.  No fence: only the LDS written by
// this kernel's ring loads is exchanged here.
template <int P, int KS, int NS, bool LGKM, int NL>
__device__ inline void ring_sync() {
  constexpr int E = (7 << 4) | ((LGKM ? 0 : 15) << 8), N = (NS - 2) * NL;  // expcnt: no wait
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(E | (N & 15) | ((N >> 4) << 14));
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Waits for every ring load of this wave (before the workgroup exits).
__device__ inline void ring_drain() { __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8)); }

// Per-lane sources of the chunks a wave loads into every stage, set when a
// segment or tile starts so that issuing a stage is branch-free.  ptr[q] is
// the byte address of the lane's row at k = 0, klim[q] the row's K (0 for a
// row outside its operand, whose loads then read zeros).
// FP32 / FP64: a chunk is 16 rows x 64 bytes (4 lanes per row); q = 0, 1 the
// A chunks w and w + 4, q = 2, 3 the B chunks w and w + 4 of the 8 in each
// array.
// BF16X3 (high and low halves interleaved in groups of 8 elements, so 32 k of
// a row are 128 contiguous bytes): a chunk is 8 rows x 128 bytes (8 lanes per
// row); of the 8 waves, wave w loads rows [16 w, 16 w + 16) of A (q = u < 2:
// A chunk 2 w + u) and, with NB chunks of B per wave (B rows 64 NB), rows
// [8 NB w, 8 NB w + 8 NB) of B (q = 2 + u, u < NB: B chunk NB w + u).
template <int P> struct LoadSetT {
  static constexpr int N = P == TNS_BF16X3 ? 6 : 4;
  const char *ptr[N];
  int32_t klim[N];
};

// Rows of M from r0 on into the slots of one operand (q0 = 0: A, else B; rows
// beyond rlim read zeros): FP32 / FP64 128 rows; BF16X3 128 rows of A or
// 64 NB rows of B.
template <int P, int NB = 4>
__device__ __attribute__((always_inline)) inline void ls_mat(LoadSetT<P> &ls, int q0, const Mat &M, int r0, int rlim,
                                                             int K) {
  typedef typename FP<P>::E E;
  const int w = threadIdx.x >> 6;
  if constexpr (P == TNS_BF16X3) {
    const int rin = (threadIdx.x & 63) >> 3;
    if (q0 == 0) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int row = r0 + 16 * w + 8 * u + rin;
        ls.ptr[u] = reinterpret_cast<const char *>(M.p) + 4 * ((int64_t)row * M.ld);
        ls.klim[u] = row < rlim ? K : 0;
      }
    } else {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int row = r0 + 8 * NB * w + 8 * u + rin;
        ls.ptr[2 + u] = reinterpret_cast<const char *>(M.p) + 4 * ((int64_t)row * M.ld);
        ls.klim[2 + u] = row < rlim ? K : 0;
      }
    }
  } else {
    const int rin = (threadIdx.x & 63) >> 2, base = q0 ? 2 : 0;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int row = r0 + 16 * (w + 4 * v) + rin;
      ls.ptr[base + v] = reinterpret_cast<const char *>(reinterpret_cast<const E *>(M.p) + (int64_t)row * M.ld);
      ls.klim[base + v] = row < rlim ? K : 0;
    }
  }
}

// Stage <- one K step (k in [k0, k0 + BK)) of the chunks of ls; with live
// false every load reads the zero region.  Branch-free.  NB: BF16X3 B chunks
// per wave.
template <int P, int KS, int NB = 4>
__device__ __attribute__((always_inline)) inline void ring_issue(Stage<P, KS> &st, const LoadSetT<P> &ls, int k0,
                                                                 bool live, const void *zero) {
  typedef typename FP<P>::E E;
  static_assert(KS == 1, "one k-range per stage");
  constexpr int VEC = RingP<P>::VEC, L = RingL<P, KS>::LOADS;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const char *z = reinterpret_cast<const char *>(zero);
  if constexpr (P == TNS_BF16X3) {
    // lane: row rin of the chunk, 16-byte slot lane & 7 holding vector
    // v = slot ^ rin (v = 2 g + h: k-group g, h = 0 high, 1 low half)
    const int rin = lane >> 3, v = (lane & 7) ^ rin;
    const int k = k0 + 8 * (v >> 1);
    const int64_t boff = 4 * (int64_t)k0 + 16 * v;
#pragma unroll
    for (int u = 0; u < 2 + NB; ++u) {
      const int c = u < 2 ? 2 * w + u : 16 + NB * w + (u - 2);  // chunk of the stage (A 0..15, B 16..47)
      const bool in = live && k < ls.klim[u];
      gl_lds(in ? ls.ptr[u] + boff : z, &st.b[c * 1024]);
    }
  } else {
    const int rin = lane >> 2;
    const int k = k0 + VEC * ((lane & 3) ^ rswz(rin));
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int c = w + 4 * u;  // chunk of the stage; array h = c / 8 = u / 2
      const int q = (u / 2 >= 1 ? 2 : 0) + (u & 1);
      const bool in = live && k < ls.klim[q];
      const char *src = ls.ptr[q] + (int64_t)k * (int64_t)sizeof(E);
      gl_lds(in ? src : z, &st.b[c * 1024]);
    }
  }
}

// Byte offset in a stage of 16-byte k-vector kv of row `row` of array arr
// (FP32 / FP64 chunks of 16 rows x 64 bytes).
__device__ inline int ring_off(int arr, int row, int kv) {
  const int rin = row & 15;
  return (8 * arr + (row >> 4)) * 1024 + (rin * 4 + (kv ^ rswz(rin))) * 16;
}
// BF16X3: byte offset of vector v (2 g + h) of row `row` of operand arr
// (chunks of 8 rows x 128 bytes; row r keeps vector v at slot v ^ (r & 7), so
// the 16 rows of one MFMA operand fetch spread over the banks).
__device__ inline int ring_off_bf(int arr, int row, int v) {
  return (16 * arr + (row >> 3)) * 1024 + (row & 7) * 128 + ((v ^ (row & 7)) << 4);
}

// MFMA fragment of one 16-row tile for lane (l16, g): the 16-byte k-vector of
// k-group g (BF16X3: of both halves; FP32 / FP64: of every k-half).
template <int P, int KS> struct Frag;
template <int KS> struct Frag<TNS_BF16X3, KS> { u16x8 h, l; };
template <int KS> struct Frag<TNS_F32, KS> { f4 v[KS]; };
template <int KS> struct Frag<TNS_F64, KS> { d2 v[KS]; };

template <int P, int KS>
__device__ __attribute__((always_inline)) inline Frag<P, KS> ring_frag(const Stage<P, KS> &st, int isB, int row0, int l16, int g) {
  Frag<P, KS> f;
  const uint8_t *base = st.b;
  if constexpr (P == TNS_BF16X3) {
    f.h = *reinterpret_cast<const u16x8 *>(base + ring_off_bf(isB, row0 + l16, 2 * g));
    f.l = *reinterpret_cast<const u16x8 *>(base + ring_off_bf(isB, row0 + l16, 2 * g + 1));
  } else {
#pragma unroll
    for (int kh = 0; kh < KS; ++kh)
      f.v[kh] = *reinterpret_cast<const typename FP<P>::V *>(base + ring_off(KS * isB + kh, row0 + l16, g));
  }
  return f;
}

// acc += x y^T over the stage's k for one 16 x 16 tile (x: rows, y: columns).
template <int P, int KS, class A4>
__device__ __attribute__((always_inline)) inline void frag_mma(const Frag<P, KS> &x, const Frag<P, KS> &y, A4 &acc) {
  if constexpr (P == TNS_BF16X3) {
    acc = mfma_bf(x.l, y.h, acc);
    acc = mfma_bf(x.h, y.l, acc);
    acc = mfma_bf(x.h, y.h, acc);
  } else {
#pragma unroll
    for (int kh = 0; kh < KS; ++kh)
#pragma unroll
      for (int e = 0; e < RingP<P>::VEC; ++e) acc = mfma(x.v[kh][e], y.v[kh][e], acc);
  }
}

// One stage of MFMA for a tile of WM x WN wave tiles (WN waves across the
// columns, default wgn): wave (wm, wn) owns rows wm 16 TM + 16 i and columns
// wn 16 TN + 16 j.  SWAP: acc[i][j] holds the transposed tile (rows = B rows
// wn 16 TN + 16 i, columns = A rows wm 16 TM + 16 j).
// The operand fragments of one stage for this wave's tile.
template <int P, int KS, int TM, int TN, int WN = wgn<P>()> struct Frags {
  Frag<P, KS> a[TM], b[TN];
};

template <int P, int KS, int TM, int TN, int WN>
__device__ __attribute__((always_inline)) inline void ring_read(const Stage<P, KS> &st, Frags<P, KS, TM, TN, WN> &f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w / WN, wn = w % WN, l16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int i = 0; i < TM; ++i) f.a[i] = ring_frag<P, KS>(st, 0, wm * 16 * TM + 16 * i, l16, g);
#pragma unroll
  for (int j = 0; j < TN; ++j) f.b[j] = ring_frag<P, KS>(st, 1, wn * 16 * TN + 16 * j, l16, g);
}

template <int P, int KS, int TM, int TN, bool SWAP, int WN, int AM, int AN>
__device__ __attribute__((always_inline)) inline void ring_mma(const Frags<P, KS, TM, TN, WN> &f,
                                                               typename FP<P>::A4 (&acc)[AM][AN]) {
  if (SWAP) {
#pragma unroll
    for (int i = 0; i < TN; ++i)
#pragma unroll
      for (int j = 0; j < TM; ++j) frag_mma<P, KS>(f.b[i], f.a[j], acc[i][j]);
  } else {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) frag_mma<P, KS>(f.a[i], f.b[j], acc[i][j]);
  }
}

// Ring geometry of each (precision, phase): KS k-halves per stage, WG
// workgroups per CU, NS stages, PF register prefetch of the next stage's
// fragments.  FP32 and FP64 use four 16 KB stages at two workgroups per CU,
// BF16X3 three 48 KB stages at one.  BF16X3 phase B reads each stage's
// fragments in the step that uses them: the second fragment set of the
// prefetch does not fit its registers next to the segment bookkeeping at two
// waves per SIMD (spilled, phase B took 14.8 ms at D = 4096 against 12.7).
template <int P, int PH> struct Geo {
  static constexpr int KS = 1;
  static constexpr int WG = P == TNS_BF16X3 ? 1 : 2;
  static constexpr int NS = P == TNS_BF16X3 ? 3 : 4;
  static constexpr bool PF = !(P == TNS_BF16X3 && PH == 1);
};

// Drives the ring over one stream of K steps.  dma(stage) fills a stage
// with the load cursor's K step (zeros once the stream is exhausted) and
// adv() moves the cursor on, returning 1 for a real step and 0 past the end;
// mma(frags, J) is the MFMA work of one step, J (a compile-time constant) the
// step's position in the unrolled group of NS steps, and post() runs after
// each real step (tile completion).  Loads run NS - 1 steps ahead; step s uses stage
// s mod NS, written NS - 1 steps earlier.  Every step issues a stage and
// runs its MFMA work (past the end on zeros): the loads, the operand reads
// and the MFMA work of a step form one branch-free block that the compiler
// can interleave, and with the direct loads on every path of a loop without
// early exits the compiler keeps track of which stage each read depends on.
//
// PF (prefetch, three or four stages): the fragments of stage s + 1 are read
// into registers during step s, while the MFMA work of stage s (read one step
// earlier) runs; the slot of stage s is then free at step s and receives
// stage s + NS.  Each step waits for this wave's outstanding LDS reads before
// the barrier, so no slot is overwritten while a read of it is in flight.  NL:
// loads per wave and stage.
template <int... J, class F>
__device__ __attribute__((always_inline)) inline void static_for(std::integer_sequence<int, J...>, F &&f) {
  (f(std::integral_constant<int, J>{}), ...);
}

template <int P, int KS, int NS, bool PF, class FR, int NL, class Dma, class Adv, class Mma, class Post>
__device__ __attribute__((always_inline)) inline void ring_run(Ring<P, KS, NS> &rg, Dma &&dma, Adv &&adv, Mma &&mma,
                                                               Post &&post) {
  int issued = 0;
  static_for(std::make_integer_sequence<int, NS - 1>{}, [&](auto J) {
    dma(stage<J>(rg));
    issued += adv();
  });
  if constexpr (PF) {
    static_assert(NS == 3 || NS == 4, "prefetch alternates two fragment sets over three or four stages");
    FR f0, f1;
    ring_sync<P, KS, NS, false, NL>();
    dma(stage<NS - 1>(rg));
    issued += adv();
    ring_read(rg.s0, f0);
    auto step = [&](auto J, int s, FR &cur, FR &nxt) {
      constexpr int j = decltype(J)::value;
      ring_sync<P, KS, NS, true, NL>();
      dma(stage<j>(rg));
      ring_read(stage<(j + 1) % NS>(rg), nxt);
      mma(cur, J);
      issued += adv();
      if (s < issued) post();
    };
    // steps in groups of lcm(2, NS): the fragment sets alternate, the stages cycle
    constexpr int U = NS == 4 ? 4 : 6;
    for (int s = 0; s < issued; s += U) {
      static_for(std::make_integer_sequence<int, U>{}, [&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (i & 1) step(std::integral_constant<int, i % NS>{}, s + i, f1, f0);
        else step(std::integral_constant<int, i % NS>{}, s + i, f0, f1);
      });
    }
  } else {
    FR f;
    for (int s = 0; s < issued; s += NS) {
      static_for(std::make_integer_sequence<int, NS>{}, [&](auto J) {
        constexpr int j = decltype(J)::value;
        ring_sync<P, KS, NS, false, NL>();
        dma(stage<(j + NS - 1) % NS>(rg));
        ring_read(stage<j>(rg), f);
        mma(f, J);
        issued += adv();
        if (s + j < issued) post();
      });
    }
  }
}

// Runs CALL(TM, TN) for tile extents (32 tm) x (32 tn), tm, tn in {1, 2, 3, 4}.
#define TNS_TILE_SWITCH(tm, tn, CALL)                  \
  switch ((tm) * 8 + (tn)) {                             \
    case 9: CALL(1, 1); break;                           \
    case 10: CALL(1, 2); break;                          \
    case 11: CALL(1, 3); break;                          \
    case 12: CALL(1, 4); break;                          \
    case 17: CALL(2, 1); break;                          \
    case 18: CALL(2, 2); break;                          \
    case 19: CALL(2, 3); break;                          \
    case 20: CALL(2, 4); break;                          \
    case 25: CALL(3, 1); break;                          \
    case 26: CALL(3, 2); break;                          \
    case 27: CALL(3, 3); break;                          \
    case 28: CALL(3, 4); break;                          \
    case 33: CALL(4, 1); break;                          \
    case 34: CALL(4, 2); break;                          \
    case 35: CALL(4, 3); break;                          \
    default: CALL(4, 4); break;                          \
  }

// --- phase B: one item (output tile, chunk of tasks) ------------------------------------
// TM, TN: 16-row / 16-column MFMA tiles per wave (a workgroup tile of
// 32 TM rows x 16 TN wgn columns); ncols: the item's columns (the rest of the
// tile reads zeros and stores nothing).
template <int P, int KS, int TM, int TN, int WN = wgn<P>()>
__device__ __attribute__((always_inline)) inline void ring_item_b_t(const FwdArgs &g, Ring<P, KS, Geo<P, 1>::NS> &rg,
                                                                    const Item &it, int mode, int ncols) {
  typedef typename FP<P>::A4 A4;
  constexpr int BK = RingL<P, KS>::BK;
  constexpr int NB = (WN * TN + 3) / 4;  // BF16X3 chunks of B rows per wave
  constexpr int NL = P == TNS_BF16X3 ? 2 + NB : RingL<P, KS>::LOADS;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w / WN, wn = w % WN, l16 = lane & 15, lg = lane >> 4;
  const int cend = it.c0 + ncols;
  // FP32: the MFMA accumulators take NS steps at a time and are then added
  // into a second set (two-level summation), so that the rounding error over
  // a long inner dimension grows with the square roots of the steps per fold
  // and of the number of folds rather than with that of the whole dimension.
  constexpr bool TWO = P == TNS_F32;
  A4 acc[TM][TN], acc2[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc2[i][j] = vzero<A4>();
  int lj = 0, lK = 0;
  LoadSetT<P> LS;
  // segment records through scalar loads; the next one is fetched while the
  // current segment streams
  auto fetch = [&](int pos, SegRec &r) {
    const SegRec *q = g.segb + pos;
    r.a_off = cld(&q->a_off); r.b_off = cld(&q->b_off);
    r.K = cld(&q->K); r.arows = cld(&q->arows); r.brows = cld(&q->brows); r.bld = cld(&q->bld);
  };
  // Identity second factors (b_off < 0) contribute their intermediate T as
  // it stands: added into the accumulators here, element by element, and
  // left out of the operand stream.  Only items flagged at build time hold any.
  const bool idy = (it.mode & ITEM_IDENT_Y) != 0;
  if (idy) {
    for (int sp = it.tb; sp < it.te; ++sp) {
      SegRec r;
      fetch(sp, r);
      if (r.b_off >= 0) continue;
      const int ldT = ld8(r.K);  // T: arows x K, K = the output's columns
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int col = it.c0 + wn * 16 * TN + j * 16 + l16;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = it.p0 + wm * 16 * TM + i * 16 + mrow(acc[i][j], lg, v);
            if (row < r.arows && col < r.K && col < cend) {
              const int64_t e = r.a_off + (int64_t)row * ldT + col;
              if constexpr (P == TNS_BF16X3) {
                const uint16_t *Tu = reinterpret_cast<const uint16_t *>(g.T) + bfx_hi(e);
                acc[i][j][v] += bf16_to_f32(Tu[0]) + bf16_to_f32(Tu[8]);
              } else {
                acc[i][j][v] += reinterpret_cast<const typename FP<P>::E *>(g.T)[e];
              }
            }
          }
        }
    }
  }
  // next segment with a product at or after pos
  auto live_from = [&](int pos) {
    if (idy)
      while (pos < it.te && cld(&g.segb[pos].b_off) < 0) ++pos;
    return pos;
  };
  int seg = live_from(it.tb), nseg = it.te;
  bool ldone = seg >= it.te;  // every segment has lK >= 1
  auto load_seg = [&](const SegRec &r) {
    Mat LA, LB;
    lK = r.K;
    LA.p = elem_ptr<P>(g.T, r.a_off);
    LA.ld = ld8(r.K); LA.rows = r.arows;
    LB.p = elem_ptr<P>(g.ops, r.b_off);
    LB.ld = r.bld; LB.rows = r.brows;
    ls_mat<P, NB>(LS, 0, LA, it.p0, min(LA.rows, it.p0 + 16 * TM * (gth<P>() / 64 / WN)), lK);
    ls_mat<P, NB>(LS, 2, LB, it.c0, min(LB.rows, cend), lK);
  };
  SegRec nxt;
  if (!ldone) {
    SegRec cur;
    fetch(seg, cur);
    nseg = live_from(seg + 1);
    if (nseg < it.te) fetch(nseg, nxt);
    load_seg(cur);
  } else {  // no products: the ring runs on the zero region only
    Mat Z;
    Z.p = g.zero; Z.ld = 0; Z.rows = 0;
    ls_mat<P, NB>(LS, 0, Z, 0, 0, 0);
    ls_mat<P, NB>(LS, 2, Z, 0, 0, 0);
  }
  typedef Frags<P, KS, TM, TN, WN> FR;
  ring_run<P, KS, Geo<P, 1>::NS, Geo<P, 1>::PF, FR, NL>(
      rg, [&](Stage<P, KS> &st) { ring_issue<P, KS, NB>(st, LS, lj * BK, !ldone, g.zero); },
      [&]() -> int {
        if (ldone) return 0;
        if (++lj * BK >= lK) {
          lj = 0;
          seg = nseg;
          if (seg < it.te) {
            load_seg(nxt);
            nseg = live_from(seg + 1);
            if (nseg < it.te) fetch(nseg, nxt);
          } else {
            ldone = true;
          }
        }
        return 1;
      },
      [&](const FR &f, auto J) {
        ring_mma<P, KS, TM, TN, false>(f, acc);
        if constexpr (TWO && decltype(J)::value == Geo<P, 1>::NS - 1) {
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              acc2[i][j] += acc[i][j];
              acc[i][j] = vzero<A4>();
            }
        }
      },
      [] {});
  const int R = cld(&g.grp_rows[it.grp]), C = cld(&g.grp_cols[it.grp]);
  auto slot = gptr(reinterpret_cast<typename FP<P>::Acc *>(g.partial) + cld(&g.slot_off[it.slot]));
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = it.c0 + wn * 16 * TN + j * 16 + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = it.p0 + wm * 16 * TM + i * 16 + mrow(acc[i][j], lg, v);
        if (row < R && col < C && col < cend) {
          const int64_t o = mode == M_FWD1 ? ((int64_t)col * R + row) : ((int64_t)row * C + col);
          slot[o] = TWO ? acc2[i][j][v] + acc[i][j][v] : acc[i][j][v];
        }
      }
    }
}

// Item dispatch: BF16X3 covers up to 256 columns per tile (16 TN per wave
// over 4 waves, TN = ceil(tn / 2); 1 or 3 column tiles over 64 or 128 rows on
// 4 x 2 waves instead, 16 tn columns each); FP32 / FP64 up to 128 (16 TN per
// wave over 2 waves), which their item lists never exceed.
template <int P, int KS>
__device__ __attribute__((always_inline)) inline void ring_item_b(const FwdArgs &g, Ring<P, KS, Geo<P, 1>::NS> &rg,
                                                                  int wk) {
  const Item it = load_item(g.items + wk);
  const int mode = it.mode & 0xff, tm = (it.mode >> 8) & 0xff, tn = (it.mode >> 16) & 0xff;
  const int cw = P == TNS_BF16X3 ? (tn + 1) >> 1 : (tn < 4 ? tn : 4);
  const int ncols = P == TNS_BF16X3 ? 32 * tn : 32 * cw;
  if constexpr (P == TNS_BF16X3) {
    // 32 or 96 columns over 64 or 128 rows: 4 x 2 waves (no padding columns)
    if ((tn == 1 || tn == 3) && (tm == 2 || tm == 4)) {
      if (tm == 2) {
        if (tn == 1) ring_item_b_t<P, KS, 1, 1, 2>(g, rg, it, mode, ncols);
        else ring_item_b_t<P, KS, 1, 3, 2>(g, rg, it, mode, ncols);
      } else {
        if (tn == 1) ring_item_b_t<P, KS, 2, 1, 2>(g, rg, it, mode, ncols);
        else ring_item_b_t<P, KS, 2, 3, 2>(g, rg, it, mode, ncols);
      }
      return;
    }
  }
#define TNS_CALL_B(a, b) ring_item_b_t<P, KS, a, b>(g, rg, it, mode, ncols)
  TNS_TILE_SWITCH(tm, cw, TNS_CALL_B)
#undef TNS_CALL_B
}

// --- phase A: row tiles of a panel as one stream of K steps ---------------------------
// A panel item covers chunks [p0, p0 + np) of its panel's stacked rows (whole
// 128-row tiles) and columns [c0, c0 + ncols) of T; its row tiles share the
// right operand (the padded psi sector), and the ring keeps loading across
// tile boundaries.

// Sources of this wave's A rows in the tile starting at chunk ch, inner
// dimension K (chunks at or beyond ch_end read zeros).  FP32 / FP64: the 16
// rows of chunks ch + w and ch + w + 4 (slots 0, 1); BF16X3 (8 waves): the
// 16 rows of chunk ch + w, rows 8 u .. 8 u + 7 in slot u < 2.
template <int P>
__device__ __attribute__((always_inline)) inline void ls_chunks(const FwdArgs &g, LoadSetT<P> &ls, int ch, int ch_end,
                                                                int K) {
  const int w = threadIdx.x >> 6;
  constexpr bool BF = P == TNS_BF16X3;
  constexpr int NU = 2;
  const int rin = BF ? (threadIdx.x & 63) >> 3 : (threadIdx.x & 63) >> 2;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int c = __builtin_amdgcn_readfirstlane(BF ? ch + w : ch + w + 4 * u);  // uniform: scalar loads
    const int row = BF ? 8 * u + rin : rin;  // row inside the chunk
    ls.ptr[u] = reinterpret_cast<const char *>(g.zero);
    ls.klim[u] = 0;
    if (c < ch_end) {
      const ChunkRec *r = g.recs + c;
      const int64_t off = cld(&r->off);
      const int vr = cld(&r->vrows);
      // element index of the lane's row at k = 0
      const int64_t e = off + (int64_t)row * cld(&r->ld);
      ls.ptr[u] = reinterpret_cast<const char *>(elem_ptr<P>(g.ops, e));
      ls.klim[u] = row < vr ? K : 0;
    }
  }
}

// Epilogue of a stacked T tile starting at chunk ch (swapped accumulator:
// acc[i][j] rows = T columns c0 + wn 16 TN + 16 i + .., columns = the rows of
// chunk ch + TM wm + j; WN waves across the columns).  Row r of chunk c lies at tbase + (16 c + r) ldT;
// rows beyond the chunk's task and columns at or beyond cend are not stored.
// FP32 writes 4 consecutive columns per lane as one vector.  BF16X3: the
// lanes l and l ^ 16 hold the two halves of one 8-column group (row starts
// and cend are multiples of 8, so both store or neither); they trade 8 bytes
// so that the even lane writes the group's 8 high halves and the odd one its
// 8 low halves, each as one 16-byte store: a row's 16 columns are 64
// contiguous bytes from 4 lanes.
template <int P, int TN, int TM, int WN>
__device__ __attribute__((always_inline)) inline void ring_store_stk(const FwdArgs &g, typename FP<P>::A4 (&acc)[TN][TM],
                                                                     int ch, int ch_end, int64_t tbase, int c0,
                                                                     int cend, int ldT) {
  typedef typename FP<P>::A4 A4;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w / WN, wn = w % WN, l16 = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int j = 0; j < TM; ++j) {
    const int c = __builtin_amdgcn_readfirstlane(ch + TM * wm + j);
    if (c < ch_end) {
      const ChunkRec *r = g.recs + c;
      const int vr = cld(&r->vrows);
      const double alpha = cld(&r->alpha);
      const int64_t orow = tbase + ((int64_t)c * PCH + l16) * ldT;
      if constexpr (P == TNS_BF16X3) {
#pragma unroll
        for (int i = 0; i < TN; ++i) {
          const int col = c0 + wn * 16 * TN + i * 16 + 4 * lg;
          const f4 x = (float)alpha * acc[i][j];
          const bfx4 h = {(__bf16)x[0], (__bf16)x[1], (__bf16)x[2], (__bf16)x[3]};
          const bfx4 l = {(__bf16)(x[0] - (float)h[0]), (__bf16)(x[1] - (float)h[1]),
                          (__bf16)(x[2] - (float)h[2]), (__bf16)(x[3] - (float)h[3])};
          const uint64_t hb = __builtin_bit_cast(uint64_t, h), lb = __builtin_bit_cast(uint64_t, l);
          const bool odd = lg & 1;
          // the even lane takes its partner's high halves, the odd one its partner's low halves
          const uint64_t got = __shfl_xor((unsigned long long)(odd ? hb : lb), 16);
          if (l16 < vr && col < ldT && col < cend) {
            u64x2 v;
            v[0] = odd ? got : hb;
            v[1] = odd ? lb : got;
            // column col of the group: u16 index 2 (orow + col) is the start
            // of the group's high halves (col = 0 mod 8) or of its low halves
            // (col = 4 mod 8)
            *gptr(reinterpret_cast<u64x2 *>(reinterpret_cast<uint16_t *>(g.T) + 2 * (orow + col))) = v;
          }
        }
      } else if (l16 < vr) {
#pragma unroll
        for (int i = 0; i < TN; ++i) {
          const int col0 = c0 + wn * 16 * TN + i * 16;
          if constexpr (P == TNS_F64) {
            auto Tt = gptr(reinterpret_cast<double *>(g.T) + orow);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int col = col0 + mrow(acc[i][j], lg, v);
              if (col < ldT && col < cend) Tt[col] = alpha * acc[i][j][v];
            }
          } else {
            const int col = col0 + 4 * lg;  // FP32 / BF16 accumulators: rows 4 lg .. 4 lg + 3
            if (col < ldT && col < cend) {
              const f4 x = (float)alpha * acc[i][j];
              const int64_t o = orow + col;
              *gptr(reinterpret_cast<f4 *>(reinterpret_cast<float *>(g.T) + o)) = x;
            }
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < TN; ++i) acc[i][j] = vzero<A4>();
  }
}

// WN waves across the columns (the rest across the 128 rows, TM MFMA row
// tiles each); BF16X3 loads NB chunks of B rows per wave.
template <int P, int KS, int TN, int WN = wgn<P>()>
__device__ __attribute__((always_inline)) inline void ring_item_a_t(const FwdArgs &g, Ring<P, KS, Geo<P, 0>::NS> &rg,
                                                                    const Item &it, int ncols) {
  typedef typename FP<P>::A4 A4;
  constexpr int BK = RingL<P, KS>::BK;
  constexpr int TM = 8 * WN * 64 / gth<P>();
  constexpr int NB = (WN * TN + 3) / 4;
  constexpr int NL = P == TNS_BF16X3 ? 2 + NB : RingL<P, KS>::LOADS;
  const int cend = it.c0 + ncols;
  const int G = it.grp, sec = G >> 1, cls = G & 1;
  const int m = cld(&g.dimL[cld(&g.psi_sec[4 * sec])]), n = cld(&g.dimR[cld(&g.psi_sec[4 * sec + 3])]);
  const int K = cls ? n : m, N = cls ? m : n, ldT = ld8(N);
  Mat B;  // B(j, k) = M(k, j): class 0 A_s^T rows, class 1 A_s rows
  if (cls == 0) {
    B.p = elem_ptr<P>(g.pt, cld(&g.pt_off[sec]));
    B.ld = ld8(m); B.rows = n;
  } else {
    B.p = elem_ptr<P>(g.pp, cld(&g.pp_off[sec]));
    B.ld = ld8(n); B.rows = m;
  }
  const int ch_end = it.p0 + it.np;
  const int64_t tbase = cld(&g.a_tb[G]) - cld(&g.a_gch[G]) * PCH * ldT;
  // load cursor: (tile's first chunk, k); compute cursor NS - 1 steps behind
  int lch = it.p0, lk0 = 0, cch = it.p0, ck0 = 0;
  bool ldone = false;
  LoadSetT<P> LS;
  ls_chunks<P>(g, LS, lch, ch_end, K);
  ls_mat<P, NB>(LS, 2, B, it.c0, min(B.rows, cend), K);
  A4 acc[TN][TM];
#pragma unroll
  for (int i = 0; i < TN; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[i][j] = vzero<A4>();
  typedef Frags<P, KS, TM, TN, WN> FR;
  // the prefetch's second fragment set of the widest 4 x 2 tiles would spill
  constexpr bool PF = Geo<P, 0>::PF && !(WN == 2 && TN >= 5);
  ring_run<P, KS, Geo<P, 0>::NS, PF, FR, NL>(
      rg, [&](Stage<P, KS> &st) { ring_issue<P, KS, NB>(st, LS, lk0, !ldone, g.zero); },
      [&]() -> int {
        if (ldone) return 0;
        if ((lk0 += BK) < K) return 1;
        lk0 = 0;
        if ((lch += PTILE_CH) < ch_end) ls_chunks<P>(g, LS, lch, ch_end, K);
        else ldone = true;
        return 1;
      },
      [&](const FR &f, auto) { ring_mma<P, KS, TM, TN, true>(f, acc); },
      [&]() {
        if ((ck0 += BK) < K) return;
        ck0 = 0;
        ring_store_stk<P, TN, TM, WN>(g, acc, cch, ch_end, tbase, it.c0, cend, ldT);
        cch += PTILE_CH;
      });
}

// Item dispatch: FP32 / FP64 up to 128 columns per tile (2 x 2 waves).
// BF16X3 up to 256: an even number tn of 32-column tiles runs on 2 x 4 waves
// of 16 tn / 2 columns each, an odd one on 4 x 2 waves of 16 tn columns each
// (both without padding columns).
template <int P, int KS>
__device__ __attribute__((always_inline)) inline void ring_item_a(const FwdArgs &g, Ring<P, KS, Geo<P, 0>::NS> &rg,
                                                                  int wk) {
  const Item it = load_item(g.a_items + wk);
  const int tn = (it.mode >> 16) & 0xff;
  if constexpr (P == TNS_BF16X3) {
    const int ncols = 32 * tn;
    switch (tn) {
      case 1: ring_item_a_t<P, KS, 1, 2>(g, rg, it, ncols); break;
      case 2: ring_item_a_t<P, KS, 1, 4>(g, rg, it, ncols); break;
      case 3: ring_item_a_t<P, KS, 3, 2>(g, rg, it, ncols); break;
      case 4: ring_item_a_t<P, KS, 2, 4>(g, rg, it, ncols); break;
      case 5: case 6: ring_item_a_t<P, KS, 3, 4>(g, rg, it, ncols); break;
      default: ring_item_a_t<P, KS, 4, 4>(g, rg, it, ncols); break;
    }
  } else {
    const int cw = tn < 4 ? tn : 4;
    const int ncols = 32 * cw;
    switch (cw) {
      case 1: ring_item_a_t<P, KS, 1>(g, rg, it, ncols); break;
      case 2: ring_item_a_t<P, KS, 2>(g, rg, it, ncols); break;
      case 3: ring_item_a_t<P, KS, 3>(g, rg, it, ncols); break;
      default: ring_item_a_t<P, KS, 4>(g, rg, it, ncols); break;
    }
  }
}

// Chunk sources of the panel-order position i (one thread per task).
__device__ inline void chunk_recs_of(const FwdArgs &g, int64_t i) {
  const int t = g.a_idx[i];
  const tns_task &k = g.tasks[t];
  if (ident_x(k)) return;  // no chunks: its intermediate is a scaled copy (k_ident_T)
  const int *so = g.psi_sec + 4 * k.out;
  const int rows = k.order == 0 ? g.dimL[so[0]] : g.dimR[so[3]];
  const int blk = k.order == 0 ? k.lblk : k.rblk;
  ChunkRec *r = const_cast<ChunkRec *>(g.recs) + g.a_ch[i];
  const int64_t bo = g.blk_off[blk];
  const int ld = g.blk_ld[blk];
  for (int j = 0; j * PCH < rows; ++j) {
    ChunkRec x;
    x.off = bo + (int64_t)j * PCH * ld;
    x.ld = ld;
    x.vrows = min(PCH, rows - j * PCH);
    x.alpha = k.alpha;
    x.pad_ = 0;
    r[j] = x;
  }
}

__global__ void k_chunk_recs(FwdArgs g) {
  GRID_STRIDE(i, g.ntasks) chunk_recs_of(g, i);
}

template <int P, int PH>
__global__ __launch_bounds__(gth<P>(), (Geo<P, PH>::WG)) void k_fwd(FwdArgs g) {
  constexpr int KS = Geo<P, PH>::KS, NS = Geo<P, PH>::NS;
  __shared__ Stage<P, KS> st0, st1;
  __shared__ StageJ<P, KS, NS, 2> st2;
  __shared__ StageJ<P, KS, NS, 3> st3;
  __shared__ StageJ<P, KS, NS, 4> st4;
  Ring<P, KS, NS> rg{st0, st1, st2, st3, st4};
  int *s_work = reinterpret_cast<int *>(st0.b);  // the ring is idle between items
  for (;;) {
    ring_drain();  // the previous item's trailing (zero) loads have landed
    __syncthreads();
    if (threadIdx.x == 0) *s_work = pop_work<PH>(g);
    __syncthreads();
    // uniform: the item's metadata then comes through scalar loads, which
    // leave the vector-memory count (ring loads in flight) alone
    const int wk = __builtin_amdgcn_readfirstlane(*s_work);
    __syncthreads();
    if (wk < 0) break;
    if (PH == 0) ring_item_a<P, KS>(g, rg, wk);
    else ring_item_b<P, KS>(g, rg, wk);
  }
  ring_drain();
}

// Intermediates of the tasks whose first factor is the identity: T = alpha M
// with M the padded input sector (class 0: psi_s, m x ld8(n); class 1: its
// transpose, n x ld8(m)), which has T's shape and leading dimension, so T is
// a scaled copy of it, zero columns included.  One workgroup per task in turn.
template <int P>
__device__ inline void ident_t_of(const FwdArgs &g, int t) {
  typedef typename FP<P>::E E;
  const tns_task k = g.tasks[t];
  if (!ident_x(k)) return;
  const int m = g.dimL[g.psi_sec[4 * k.in]], n = g.dimR[g.psi_sec[4 * k.in + 3]];
  const int64_t cnt = k.order == 0 ? (int64_t)m * ld8(n) : (int64_t)n * ld8(m);
  const int64_t src = k.order == 0 ? g.pp_off[k.in] : g.pt_off[k.in];
  const E *S = reinterpret_cast<const E *>(k.order == 0 ? g.pp : g.pt);
  E *D = reinterpret_cast<E *>(g.T);
  const int64_t dst = g.t_off[t];
  for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
    if constexpr (P == TNS_BF16X3) {
      const int64_t a = bfx_hi(src + e), b = bfx_hi(dst + e);
      const float x = (float)k.alpha * (bf16_to_f32(S[a]) + bf16_to_f32(S[a + 8]));
      const uint16_t h = f32_to_bf16_rne(x);
      D[b] = h;
      D[b + 8] = f32_to_bf16_rne(x - bf16_to_f32(h));
    } else if constexpr (P == TNS_F32) {
      D[dst + e] = (float)k.alpha * S[src + e];
    } else {
      D[dst + e] = k.alpha * S[src + e];
    }
  }
}

template <int P>
__global__ void k_ident_T(FwdArgs g) {
  for (int64_t t = blockIdx.x; t < g.ntasks; t += gridDim.x) ident_t_of<P>(g, (int)t);
}

// --- padded copies of psi ----------------------------------------------------------
// Sector s (m x n) to pp (m x ld8(n)) and, transposed, to pt (n x ld8(m));
// BF16X3 writes both halves, interleaved (bfx_hi).
template <class In, int P>
__device__ inline void pad_sector(int s, const In *__restrict__ psi, const int64_t *psi_off, const int32_t *psi_sec,
                                  const int32_t *dimL, const int32_t *dimR, const int64_t *pp_off,
                                  const int64_t *pt_off, void *pp, void *pt) {
  typedef typename FP<P>::E E;
  const int m = dimL[psi_sec[4 * s]], n = dimR[psi_sec[4 * s + 3]];
  const int lm = ld8(m), ln = ld8(n);
  const In *A = psi + psi_off[s];
  E *P0 = reinterpret_cast<E *>(pp), *P1 = reinterpret_cast<E *>(pt);
  const int64_t b0 = pp_off[s], b1 = pt_off[s];
  const int64_t step = (int64_t)gridDim.y * blockDim.x, e0 = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  // padded rows (zeros beyond n), then padded transposed rows (zeros beyond m)
  for (int64_t e = e0; e < (int64_t)m * ln; e += step) {
    const int i = (int)(e / ln), j = (int)(e % ln);
    if constexpr (P == TNS_BF16X3) {
      const float v = j < n ? (float)A[(int64_t)i * n + j] : 0.f;
      const uint16_t h = f32_to_bf16_rne(v);
      P0[bfx_hi(b0 + e)] = h;
      P0[bfx_hi(b0 + e) + 8] = f32_to_bf16_rne(v - bf16_to_f32(h));
    } else {
      P0[b0 + e] = j < n ? (E)A[(int64_t)i * n + j] : E(0);
    }
  }
  for (int64_t e = e0; e < (int64_t)n * lm; e += step) {
    const int j = (int)(e / lm), i = (int)(e % lm);
    if constexpr (P == TNS_BF16X3) {
      const float v = i < m ? (float)A[(int64_t)i * n + j] : 0.f;
      const uint16_t h = f32_to_bf16_rne(v);
      P1[bfx_hi(b1 + e)] = h;
      P1[bfx_hi(b1 + e) + 8] = f32_to_bf16_rne(v - bf16_to_f32(h));
    } else {
      P1[b1 + e] = i < m ? (E)A[(int64_t)i * n + j] : E(0);
    }
  }
}

template <class In, int P>
__global__ void k_pad_psi(const In *__restrict__ psi, const int64_t *psi_off, const int32_t *psi_sec,
                          const int32_t *dimL, const int32_t *dimR, const int64_t *pp_off, const int64_t *pt_off,
                          void *pp, void *pt) {
  pad_sector<In, P>(blockIdx.x, psi, psi_off, psi_sec, dimL, dimR, pp_off, pt_off, pp, pt);
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
  int32_t n, nq;
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


// Work of instance i on queue q of phase ph (16 threads: one per (ph, q)).
__global__ void k_batch_cum(BatchArgs b) {
  const int ph = threadIdx.x / NQ_MAX, q = threadIdx.x % NQ_MAX;
  if (ph >= 2) return;
  int64_t *c = b.cum + ((int64_t)ph * NQ_MAX + q) * (b.n + 1);
  int64_t run = 0;
  for (int i = 0; i < b.n; ++i) {
    c[i] = run;
    if (q < b.nq) {
      const int64_t *qb = ph == 0 ? b.tab[i].g.a_qbase : b.tab[i].g.qbase;
      run += qb[q + 1] - qb[q];
    }
  }
  c[b.n] = run;
}

// Thread 0: next (instance, item) of phase ph, own XCD queue first.
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
    *wk = (int)((ph == 0 ? b.tab[lo].g.a_qbase : b.tab[lo].g.qbase)[q] + loc);
    return;
  }
  *inst = -1;
  *wk = -1;
}

template <int P, int PH>
__global__ __launch_bounds__(gth<P>(), (Geo<P, PH>::WG)) void k_fwd_batch(BatchArgs b) {
  constexpr int KS = Geo<P, PH>::KS, NS = Geo<P, PH>::NS;
  __shared__ Stage<P, KS> st0, st1;
  __shared__ StageJ<P, KS, NS, 2> st2;
  __shared__ StageJ<P, KS, NS, 3> st3;
  __shared__ StageJ<P, KS, NS, 4> st4;
  Ring<P, KS, NS> rg{st0, st1, st2, st3, st4};
  int *s_w = reinterpret_cast<int *>(st0.b);  // the ring is idle between items
  for (;;) {
    ring_drain();  // the previous item's trailing (zero) loads have landed
    __syncthreads();
    if (threadIdx.x == 0) pop_batch(b, PH, &s_w[0], &s_w[1]);
    __syncthreads();
    const int inst = __builtin_amdgcn_readfirstlane(s_w[0]), wk = __builtin_amdgcn_readfirstlane(s_w[1]);
    __syncthreads();
    if (inst < 0) break;
    const FwdArgs g = load_words(&b.tab[inst].g);
    if (PH == 0) ring_item_a<P, KS>(g, rg, wk);
    else ring_item_b<P, KS>(g, rg, wk);
  }
  ring_drain();
}

__global__ void k_chunk_recs_batch(const InstArgs *tab) {
  const FwdArgs &g = tab[blockIdx.y].g;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.ntasks; i += (int64_t)gridDim.x * blockDim.x)
    chunk_recs_of(g, i);
}

template <int P>
__global__ void k_ident_T_batch(const InstArgs *tab) {
  const FwdArgs &g = tab[blockIdx.y].g;
  for (int64_t t = blockIdx.x; t < g.ntasks; t += gridDim.x) ident_t_of<P>(g, (int)t);
}

template <class In, int P>
__global__ void k_pad_psi_batch(const InstArgs *tab) {
  const InstArgs &a = tab[blockIdx.z];
  if ((int)blockIdx.x >= a.nS) return;
  pad_sector<In, P>(blockIdx.x, reinterpret_cast<const In *>(a.psi), a.psi_off, a.g.psi_sec, a.g.dimL, a.g.dimR,
                    a.g.pp_off, a.g.pt_off, const_cast<void *>(a.g.pp), const_cast<void *>(a.g.pt));
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
// BF16X3 arrays of n elements hold 2 ld8(n) halves (groups of 8 high halves,
// each followed by its 8 low halves).
static inline int64_t lo_of(int64_t n) { return (n + 7) & ~int64_t(7); }

// Bytes of an operand array of n elements in a precision (BF16X3: both halves).
static size_t region(int64_t n, tns_prec p) {
  n = std::max<int64_t>(n, 1);
  const size_t b = p == TNS_F64 ? (size_t)n * 8 : p == TNS_F32 ? (size_t)n * 4 : (size_t)lo_of(n) * 4;
  return align_up(b + 64, 256);
}

// Workspace of the forward product: [queue counters, zero bytes | partial
// slots | T | padded psi | padded psi^T | chunk sources].
static size_t recs_bytes(const Plan &p) { return align_up((size_t)std::max<int64_t>(p.pa.nchunks, 1) * sizeof(ChunkRec), 256); }
size_t fwd_workspace(const Plan &p, tns_prec prec) {
  return 256 + align_up((size_t)std::max<int64_t>(p.fwd.partial_elems, 1) * (prec == TNS_F64 ? 8 : 4), 256) +
         region(p.t_elems, prec) + region(p.pp_elems, prec) + region(p.pt_elems, prec) + recs_bytes(p);
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
static int grid_of(K kern, int threads, int n_cu) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, threads, 0) != hipSuccess || per <= 0) per = 1;
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
  void *recs = c;
  FwdArgs g;
  memset(&g, 0, sizeof(g));
  g.tasks = p.tasks; g.ntasks = p.ntasks;
  g.psi_sec = p.psi_sec; g.dimL = p.dimL; g.dimR = p.dimR;
  g.blk_off = p.blk_off; g.blk_ld = p.blk_ld;
  g.ops = ops;
  g.pp = pp; g.pt = pt;
  g.pp_off = p.pp_off; g.pt_off = p.pt_off;
  g.T = T; g.t_off = p.t_off;
  // FP32 / FP64: the lists at the narrow table when the table has 256-column entries
  const bool nb = P != TNS_BF16X3 && tiles_wide(S.tiles), na = P != TNS_BF16X3 && tiles_wide(p.pa.tiles);
  g.items = nb ? S.items_n : S.items; g.nitems = nb ? S.nitems_n : S.nitems;
  g.idx = S.idx; g.grp_rows = S.grp_rows; g.grp_cols = S.grp_cols;
  g.slot_off = S.slot_off; g.qbase = nb ? S.qbase_n : S.qbase; g.partial = part;
  g.queue = reinterpret_cast<int32_t *>(w); g.nq = S.nq;
  g.zero = w + 64;
  g.tiles = p.tiles;
  g.a_items = na ? p.pa.items_n : p.pa.items; g.a_qbase = na ? p.pa.qbase_n : p.pa.qbase; g.a_tb = p.pa.tb; g.a_gch = p.pa.gch;
  g.a_ch = p.pa.ch; g.a_idx = p.pa.idx;
  g.recs = reinterpret_cast<const ChunkRec *>(recs);
  g.segb = p.segb;
  return g;
}

template <int P, class In>
static tns_status fwd_launch(const Plan &p, const void *ops, const In *psi, void *sigma, int beta, char *w,
                             hipStream_t st, const hipEvent_t *ev) {
  const Sched &S = p.fwd;
  const FwdArgs g = fwd_args<P>(p, ops, w);
  hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(32), 0, st, g.queue);
  if (p.pad_ns > 0)
    hipLaunchKernelGGL((k_pad_psi<In, P>), dim3(p.pad_ns, 8), dim3(256), 0, st, psi, p.psi_off, p.psi_sec, p.dimL,
                       p.dimR, p.pp_off, p.pt_off, const_cast<void *>(g.pp), const_cast<void *>(g.pt));
  if (p.ntasks > 0) {
    hipLaunchKernelGGL(k_chunk_recs, dim3(nblocks(p.ntasks)), dim3(256), 0, st, g);
    hipLaunchKernelGGL(k_ident_T<P>, dim3((unsigned)std::min<int64_t>(p.ntasks, 4096)), dim3(256), 0, st, g);
  }
  if (ev) TNS_HIP(hipEventRecord(ev[0], st));
  if (p.ntasks > 0)
    hipLaunchKernelGGL((k_fwd<P, 0>), dim3(grid_of(k_fwd<P, 0>, gth<P>(), p.n_cu)), dim3(gth<P>()), 0, st, g);
  if (ev) TNS_HIP(hipEventRecord(ev[1], st));
  if (p.ntasks > 0 && S.nitems > 0)
    hipLaunchKernelGGL((k_fwd<P, 1>), dim3(grid_of(k_fwd<P, 1>, gth<P>(), p.n_cu)), dim3(gth<P>()), 0, st, g);
  if (ev) TNS_HIP(hipEventRecord(ev[2], st));
  return launch_epilogue_psi(p, P == TNS_F64, g.partial, sigma, beta, st);
}

// --- batched products -------------------------------------------------------------------
// [queue counters, zero bytes | argument table | prefix sums | one forward
// workspace per instance]
static size_t batch_bytes(const tns_tasklist *const *tls, int n, tns_prec prec) {
  size_t b = 256 + align_up((size_t)n * sizeof(InstArgs), 256) + align_up((size_t)2 * NQ_MAX * (n + 1) * 8, 256);
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
  typedef typename std::conditional<P == TNS_F64, double, float>::type In;
  hipLaunchKernelGGL((k_pad_psi_batch<In, P>), dim3(max_nS, 8, n), dim3(256), 0, st, tab);
  hipLaunchKernelGGL(k_chunk_recs_batch, dim3(64, n), dim3(256), 0, st, tab);
  hipLaunchKernelGGL(k_ident_T_batch<P>, dim3(64, n), dim3(256), 0, st, tab);
  if (ev) TNS_HIP(hipEventRecord(ev[0], st));
  if (any_tasks)
    hipLaunchKernelGGL((k_fwd_batch<P, 0>), dim3(grid_of(k_fwd_batch<P, 0>, gth<P>(), n_cu)), dim3(gth<P>()), 0, st,
                       b);
  if (ev) TNS_HIP(hipEventRecord(ev[1], st));
  if (any_tasks && any_items)
    hipLaunchKernelGGL((k_fwd_batch<P, 1>), dim3(grid_of(k_fwd_batch<P, 1>, gth<P>(), n_cu)), dim3(gth<P>()), 0, st,
                       b);
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
  static const int EXT[4] = {0, 128, 64, 32};  // 0: 256 columns
  for (int b = 3; b >= 0; --b) {
    float tbest = 0.f;
    uint32_t pick = cur;
    for (int e = 0; e < 4; ++e) {
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
