// Internal declarations of the gfx950 two-site H_eff library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "../../include/tns.h"

namespace tns {

// Row-panel height of one work item of the backward's fused kernel: every
// item owns TQ rows (or fewer) of an operator block's gradient and all of its
// columns.
constexpr int TQ = 64;
// Largest sector dimension the library accepts (tns.h).
constexpr int MAX_DIM = 32768;
// Work items per compute unit the chunked schedules (phase B, backward) aim
// at on large products: shorter chunks keep the tiles of one chunk, which
// share their operand rows in L2, closer together in time.  Chunks stay at
// ITEM_MIN_FLOP or more unless that leaves fewer than ITEMS_MIN_PER_CU per CU
// (small products: few, large items; each item costs a queue atomic, a ring
// fill and drain and three barriers, which 2 per CU keep small: 64 uneven
// instances 75 -> 63-65 ms against 8 per CU).
constexpr int ITEMS_PER_CU = 32;
constexpr int ITEMS_MIN_PER_CU = 2;
constexpr int64_t ITEM_MIN_FLOP = 100000000;
// Phase-A work items per compute unit: short row pieces whose column tiles
// run side by side on one XCD, so that they share the operator rows in L2;
// never below PANEL_ITEM_MIN_FLOP unless that leaves fewer than
// PANEL_ITEMS_MIN_PER_CU items per CU.
constexpr int PANEL_ITEMS_PER_CU = 64;
constexpr int PANEL_ITEMS_MIN_PER_CU = 4;
constexpr int64_t PANEL_ITEM_MIN_FLOP = 100000000;
// Most work queues of a schedule: one per XCD (accelerator complex die, each
// with its own L2).  Workgroup b of a launch runs on XCD b mod n_xcd, since
// workgroups are dispatched to the dies round-robin.
constexpr int NQ_MAX = 8;

// Evaluation modes of a task's chained product
//   out(i, j) += alpha * sum_c (sum_k X(i, k) M(k, c)) Y(j, c)
// (q, m: output / input left dims; r, n: output / input right dims; A = psi
// input sector, G = grad of sigma output sector):
//   0  (L A) R^T        X = L,   M = A,   Y = R      out = sigma rows   (q x r)
//   1  L (A R^T)        X = R,   M = A^T, Y = L      out = sigma^T rows (r x q)
//   2  d psi = L^T G R  (labels the backward's per-sector groups, which stay
//                        empty: d psi runs as the forward product of the
//                        adjoint task list)
//   3  d L = G R A^T    X = G,   M = R,   Y = A      out = (q x m)
//   4  d R = G^T L A    X = G^T, M = L,   Y = A^T    out = (r x n)
// Modes 0 and 1 are the two classes of the forward's GEMM phases; modes 3
// and 4 run in the backward's fused kernel.
enum Mode { M_FWD0 = 0, M_FWD1 = 1, M_DPSI = 2, M_DL = 3, M_DR = 4 };

// One work item of a persistent kernel: the tile rows [p0, p0+np) x columns
// [c0, c0+nc) of the output matrix of group `grp`, entries idx[tb..te) of
// that group's task list, result into partial slot `slot` (one slot per
// chunk of a group).
struct Item {
  int32_t grp, mode, p0, np, tb, te, slot, out, c0, nc;
  int64_t cost;
};
static_assert(sizeof(Item) == 48, "Item layout");

// Largest output tile of the forward grouped GEMMs (both phases).
constexpr int GM = 128, GN = 128;

// Tile extents of the forward GEMMs chosen per dimension: a table of four
// bytes, entry b the extent used along a dimension d in bucket b = [d <= 32,
// d <= 64, d <= 128, d > 128]: 32, 64 or 128, or 0 for 256 columns (rows then
// take 128); the last tile along a dimension takes the extent tail_ext of what
// remains.  Items carry their extents in bits 8..15 (rows / 32) and 16..23
// (columns / 32) of Item::mode.
constexpr uint32_t TILES_DEFAULT = 0x00804020u;  // 32, 64, 128, 256 columns (128 rows)
__host__ __device__ inline int tile_bucket(int d) { return d <= 32 ? 0 : d <= 64 ? 1 : d <= 128 ? 2 : 3; }
__host__ __device__ inline int tile_byte(uint32_t tab, int d) { return (int)((tab >> (8 * tile_bucket(d))) & 0xffu); }
__host__ __device__ inline int tile_ext_r(uint32_t tab, int d) {
  const int e = tile_byte(tab, d);
  return e == 0 ? 128 : e;
}
__host__ __device__ inline int tile_ext_c(uint32_t tab, int d) {
  const int e = tile_byte(tab, d);
  return e == 0 ? 256 : e;
}
// Extent of the last tile along a dimension whose other tiles have extent e:
// the smallest multiple of 32 that covers the rem <= e remaining rows, so that
// only the last tile is padded, by less than 32.
__host__ __device__ inline int tail_ext(int rem, int e) {
  const int x = (rem + 31) / 32 * 32;
  return x < e ? x : e;
}
// Whether a table has 256-column entries, and its narrow form (those entries
// read as 128): the FP32 / FP64 kernels take at most 128 columns per tile, so
// schedules built at a table with 256-column entries keep a second item list
// at the narrow form for them.
__host__ __device__ inline bool tiles_wide(uint32_t tab) {
  if (tab == 0) return false;
  for (int b = 0; b < 4; ++b)
    if (((tab >> (8 * b)) & 0xffu) == 0) return true;
  return false;
}
__host__ __device__ inline uint32_t tiles_narrow(uint32_t tab) {
  uint32_t r = tab;
  for (int b = 0; b < 4; ++b)
    if (((tab >> (8 * b)) & 0xffu) == 0) r |= 0x80u << (8 * b);
  return r;
}
__host__ __device__ inline bool tiles_valid(uint32_t tab) {
  for (int b = 0; b < 4; ++b) {
    const uint32_t e = (tab >> (8 * b)) & 0xffu;
    if (e != 0 && e != 32 && e != 64 && e != 128) return false;
  }
  return true;
}

struct Chunk {
  int32_t grp, tb, te, xcd;  // xcd: queue the chunk's tiles go to
  int64_t cost;
  int32_t rank;              // position in descending cost order
  int32_t flags;             // CHUNK_IDENT_Y: some task's second factor is an identity
};
constexpr int32_t CHUNK_IDENT_Y = 1;
// Work-item mode bit: the item's chunk holds identity second factors, whose
// intermediates are added into the accumulators without a product.
constexpr int32_t ITEM_IDENT_Y = 1 << 24;

// Identity factors are not multiplied.  A task's first factor X (class 0: L,
// class 1: R) being the identity makes its intermediate T = alpha M a scaled
// copy of the padded input sector; its second factor Y (class 0: R, class 1:
// L) being the identity makes its contribution T itself.
__host__ __device__ inline bool ident_x(const tns_task &t) { return t.order == 0 ? t.lblk < 0 : t.rblk < 0; }
__host__ __device__ inline bool ident_y(const tns_task &t) { return t.order == 0 ? t.rblk < 0 : t.lblk < 0; }

// A schedule: groups of tasks that share one output matrix, cut into chunks
// (partial slots) and row panels (work items), longest item first.
struct Sched {
  int32_t ngroups, nq;  // nq: work queues (XCDs)
  int32_t tile_r, tile_c;  // item tile; tile_c == 0: all columns
  uint32_t tiles, pad2_;   // non-zero: per-dimension tile table (overrides tile_r, tile_c)
  int64_t ntcap;        // capacity of idx
  int64_t chunks_cap, items_cap;
  int64_t nchunks, nitems, partial_elems, total_cost;
  int32_t *idx;         // task indices, grouped
  int32_t *grp_begin, *grp_n, *grp_rows, *grp_cols, *grp_out, *grp_mode;
  int64_t *grp_cost, *grp_chunk_base;
  Chunk *chunks;
  int64_t *slot_off, *chunk_item_base;
  Item *items_unsorted, *items;
  uint64_t *keys_in, *keys_out;
  int32_t *vals_in, *vals_out;
  void *sort_tmp;
  size_t sort_tmp_bytes;
  int64_t *qbase;       // [NQ_MAX + 1]: queue q = items[qbase[q], qbase[q+1])
  // the same chunks' items at tiles_narrow(tiles), built when tiles_wide(tiles)
  Item *items_n;        // [items_cap]
  int64_t *qbase_n;     // [NQ_MAX + 1]
  int64_t nitems_n;
  int64_t *scratch;     // [max(ngroups, chunks_cap) + 1]
  int64_t *scalars;     // [8]: 0 total cost, 1 chunks, 2 items, 3 partial elements; 5..7: 1..3 of the narrow list
};

// Phase-A panels.  Panel 2 s + c holds the tasks with input sector s and
// evaluation class c; their intermediates T_k = alpha_k X_k M share the right
// operand M (A_s or A_s^T), so the panel is one GEMM [X_k1; X_k2; ...] M with
// the X blocks stacked along the rows.  Every task occupies whole chunks of
// PCH rows (its last chunk padded), so each chunk belongs to one task; the
// intermediates of a panel form one row-major matrix (chunk rows x ld8(N)).
constexpr int PCH = 16;
// Rows of the stacked operand per tile (chunks of a tile: GM / PCH).
constexpr int PTILE_CH = GM / PCH;

// Source of one stacked chunk, written before each product: element offset
// of the chunk's first row in the operator values (leading dimension ld);
// vrows = rows of the chunk inside its task (1..16); alpha of the task.
// Tasks whose first factor is the identity have no chunks.
struct ChunkRec {
  int64_t off;
  int32_t ld, vrows;
  double alpha;
  int64_t pad_;
};
static_assert(sizeof(ChunkRec) == 32, "ChunkRec layout");

struct Panels {
  int32_t ngroups, nq;
  uint32_t tiles, pad_;
  int64_t ntcap, items_cap;
  int64_t nchunks, nitems, t_elems;
  int32_t *keys_in, *keys_out, *vals_in, *idx;  // [ntcap]: idx = tasks in panel order
  int64_t *ch;         // [ntcap + 1] first chunk of each panel-order position (none for identity X)
  int64_t *id_sz;      // [ntcap] intermediate size of identity-X tasks (panel order), else 0
  int64_t *id_off;     // [ntcap + 1] their offsets after the panels' intermediates
  int64_t *grp;        // [ngroups + 1] first panel-order position of each panel
  int64_t *gch;        // [ngroups + 1] first chunk of each panel
  int64_t *tb;         // [ngroups + 1] element offset of each panel's intermediates
  int64_t *cost;       // [ngroups] stacked rows x N x K (balance weight)
  int32_t *rank, *xcd; // [ngroups] position by descending cost, work queue
  int64_t *item_base;  // [ngroups + 1]
  Item *items_unsorted, *items;
  uint64_t *ikeys_in, *ikeys_out;
  int32_t *ivals_in, *ivals_out;
  void *sort_tmp;
  size_t sort_tmp_bytes;
  int64_t *qbase;      // [NQ_MAX + 1]: queue q = items[qbase[q], qbase[q+1])
  // the panels' items at tiles_narrow(tiles), built when tiles_wide(tiles)
  Item *items_n;       // [items_cap]
  int64_t *qbase_n;    // [NQ_MAX + 1]
  int64_t nitems_n;
  int64_t *scratch;    // [max(ngroups, ntcap, items_cap) + 1]
  int64_t *scalars;    // [8]: total item cost, item target cost, items, intermediate elements; 4..6: 0..2 of the narrow list
};

// One segment of a phase-B work item (a task of its chunk), in the order of
// the forward schedule's task list: the intermediate T_k (element offset,
// rows, inner dimension K = its columns, leading dimension ld8(K)) and the
// operator block Y_k (element offset, or -1 for the identity; rows; leading
// dimension).  Precision-independent; one scalar load per segment switch.
struct SegRec {
  int64_t a_off, b_off;
  int32_t K, arows, brows, bld;
};
static_assert(sizeof(SegRec) == 32, "SegRec layout");

// The adjoint task list and its forward schedule.  Each task of the forward
// list, transposed (output and input sectors swapped, L and R read as L^T and
// R^T, the same alpha, the evaluation order chosen again for the swapped
// shapes), sorted by its new output sector; the backward evaluates
// d psi = sum alpha L^T G R as the forward product of this list.  Blocks are
// read from a transposed copy of the operator values: block b as a
// cols x ld8(rows) row-major matrix at blk_off[b].
struct Adjoint {
  tns_task *tasks;    // [ntcap]
  int32_t *out_ptr;   // [nS + 1] CSR over the new output sectors
  int64_t *scalars;   // [8]
  int64_t *blk_off;   // [nBlk] element offset of transposed block b
  int32_t *blk_ld;    // [nBlk] ld8(rows of block b)
  int64_t *t_off;     // [ntcap + 1] offsets of the intermediates T_k
  SegRec *segb;       // [ntcap] phase-B segment records
  int64_t n_vals;     // elements of the transposed operator copy
  int64_t t_elems;
  Sched fwd;
  Panels pa;
};

// Host-side record of everything the compute calls need; lives in
// tns_tasklist::opaque, all pointers are device pointers into the build
// workspace.
struct Plan {
  int32_t nL, nR, nS, nOps, nBlk, nTerms, nmax, n_cu;
  int32_t maxdim;        // largest sector dimension
  uint32_t tiles;        // forward tile table
  int32_t no_backward;   // 1: built without the backward's schedules
  // sectors [0, pad_ns) are padded for phase A (the task inputs), sigma is
  // written from element epi_e0 on (the task outputs): all of them for a
  // product; the input blocks and the output blocks of a generic problem
  // whose inputs and outputs are disjoint sector ranges (renormalisation)
  int32_t pad_ns;
  int64_t epi_e0;
  int64_t n_vals, psi_dim, ntasks;
  // copied tables
  int32_t *qL, *dimL, *qR, *dimR, *psi_sec;
  int64_t *psi_off;
  int32_t *op_side, *op_dN, *op_d2Sz;
  int32_t *blk_op, *blk_in, *blk_out, *blk_rows, *blk_cols, *blk_ld;
  int64_t *blk_off;
  int32_t *term_L, *term_ma, *term_mb, *term_R;
  double *term_coef;
  // lookups
  int32_t *psi_index;    // [nL*16] -> sector or -1
  int32_t *blk_of_out;   // [nOps*nmax] -> block or -1
  // task table
  tns_task *tasks;       // [ntcap]
  int32_t *out_ptr;      // [nS+1]
  int64_t *scan_tmp;     // [nS+1]
  int64_t *scalars;      // [8]
  // forward intermediates T_k = alpha X_k M_k (one per task, row-major,
  // leading dimension K2 rounded up to 8, stacked per phase-A panel) and the
  // padded copies of psi
  int64_t *t_off;        // [ntcap] element offset of T_k
  SegRec *segb;          // [ntcap] phase-B segments in the order of fwd.idx
  int64_t t_elems;
  int64_t *pp_off, *pt_off;  // [nS + 1] sector offsets: m x ld8(n) and n x ld8(m)
  int64_t pp_elems, pt_elems;
  // backward grouping keys: 3 entries per task
  int32_t *bkeys_in, *bkeys_out, *bvals_in;
  void *bsort_tmp;
  size_t bsort_tmp_bytes;
  Sched fwd, bwd;
  Panels pa;
  Adjoint adj;
};
static_assert(sizeof(Plan) <= sizeof(((tns_tasklist *)0)->opaque), "Plan too large");

inline Plan &plan_of(tns_tasklist *t) { return *reinterpret_cast<Plan *>(t->opaque); }
inline const Plan &plan_of(const tns_tasklist *t) { return *reinterpret_cast<const Plan *>(t->opaque); }

#define TNS_HIP(call)                                       \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return TNS_ERR_HIP;               \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
// Leading dimension of the library's own row-major buffers: 8 elements keep
// every row 16-byte aligned for all element types.
__host__ __device__ inline int ld8(int x) { return (x + 7) & ~7; }

// Bump allocator over a caller workspace.
struct Carve {
  char *base;
  size_t off, cap;
  template <class T>
  T *take(size_t n) {
    off = align_up(off, 256);
    T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
    off += n * sizeof(T);
    return p;
  }
};

// --- site algebra (the library's own table; see tns.h for the conventions) --
// Applies monomial m = 4u + d to site state s (bit 0 = up, bit 1 = down).
// Returns the output state or -1, and the matrix element (+-1) in *val.
__host__ __device__ inline int mono_apply(int m, int s, int *val) {
  int u = m >> 2, d = m & 3;
  int v = 1;
  // down factor acts first (it stands to the right); passing the up mode
  // (which precedes it in Jordan-Wigner order) costs (-1)^{n_up} for c+/c
  int up = s & 1, dn = (s >> 1) & 1;
  switch (d) {
    case 1: if (!dn) return -1; break;
    case 2: if (dn) return -1; dn = 1; if (up) v = -v; break;
    case 3: if (!dn) return -1; dn = 0; if (up) v = -v; break;
    default: break;
  }
  switch (u) {
    case 1: if (!up) return -1; break;
    case 2: if (up) return -1; up = 1; break;
    case 3: if (!up) return -1; up = 0; break;
    default: break;
  }
  *val = v;
  return up | (dn << 1);
}
__host__ __device__ inline int mono_parity(int m) {
  int u = m >> 2, d = m & 3;
  return ((u >= 2) + (d >= 2)) & 1;
}
__host__ __device__ inline int site_N(int s) { return (s & 1) + ((s >> 1) & 1); }
__host__ __device__ inline int site_2Sz(int s) { return (s & 1) - ((s >> 1) & 1); }
__host__ __device__ inline void mono_shift(int m, int *dN, int *d2Sz) {
  int u = m >> 2, d = m & 3;
  int du = (u == 2) ? 1 : (u == 3 ? -1 : 0);
  int dd = (d == 2) ? 1 : (d == 3 ? -1 : 0);
  *dN = du + dd;
  *d2Sz = du - dd;
}

// Plan of a validated problem (tasklist.hip): the task table enumerated on the
// device from the terms, or (xtasks) one given by the caller, sorted by output
// sector with CSR xptr; backward: with the backward's schedules.
tns_status build_plan(const tns_problem *P, int32_t nmax, int32_t maxdim, const tns_task *xtasks,
                      const int32_t *xptr, int64_t nx, bool backward, void *ws, size_t ws_bytes, tns_tasklist *out,
                      hipStream_t st);
// Host validation of a problem (shapes, ranges, quantum numbers); returns the
// largest sector count and dimension.
tns_status validate_problem(const tns_problem *P, int32_t *nmax, int32_t *maxdim);
// Build-workspace bytes of build_plan (0 when counts exceed 32-bit indices).
size_t plan_workspace(const tns_problem *P, int32_t nmax, int32_t maxdim, int64_t nx_explicit, bool backward);

// Plan of the adjoint product (the tables of p with the adjoint task list,
// block table and schedules of p.adj in place of the forward ones).
Plan adjoint_plan(const Plan &p);

// Launch helpers implemented in tasklist.hip / apply.hip / fwd.hip
tns_status scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t st);
// sigma (+)= sum of the forward partial slots of every sector (beta 0 or 1)
tns_status launch_epilogue_psi(const Plan &p, bool f64, const void *part, void *sigma, int beta, hipStream_t st);
size_t fwd_workspace(const Plan &p, tns_prec prec);
// events armed by tns_profile_events (then cleared); false when not armed
bool take_profile_events(hipEvent_t ev[3]);
// ev: null, or events recorded before phase A, between the phases and after phase B
tns_status fwd_apply(const Plan &p, tns_prec prec, const void *ops, const void *psi, void *sigma, double beta,
                     void *ws, size_t ws_bytes, hipStream_t st, const hipEvent_t *ev);

}  // namespace tns
