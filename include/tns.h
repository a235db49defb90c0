/*
 * tns.h - C ABI of the MI355X (gfx950) two-site effective-Hamiltonian library.
 *
 * The library applies sigma = H_eff psi, the matrix-vector product inside the
 * Davidson diagonalisation of the paper's DMRG method (Section III.A.2,
 * Eq. (2)): every term of the Hamiltonian, after the two single-site factors
 * are reduced to scalars, adds alpha * L_i A R_i^T into one output sector of
 * the wavefunction, A being an input sector, L_i a left-block operator block,
 * R_i a right-block operator block and alpha a precalculated scalar.  The
 * library builds the sector and task tables of the paper's four-level
 * hierarchy (Section III.A.1, levels 1-2) on the device, executes them with
 * hand-written MFMA kernels (level 3), and offers the Davidson iteration and
 * a backward pass on top.
 *
 * Conventions shared with the callers
 * -----------------------------------
 * - Quantum numbers are (N, 2Sz) pairs; sector tables are sorted ascending.
 * - Site states: 0 = empty, 1 = up, 2 = down, 3 = up-down, with (N, 2Sz) =
 *   (0,0), (1,1), (1,-1), (2,0).  Site monomials have id 4*u + d, u and d in
 *   {0: 1, 1: n, 2: c+, 3: c}, the up factor to the left; within a site the
 *   up mode precedes the down mode in Jordan-Wigner order.
 * - The product state |l, sa, sb, r> = C_l C_a C_b C_r |0>; a term
 *   c * O_L O_a O_b O_R carries the sign
 *   (-1)^(pa*Nl + pb*(Nl+Na) + pR*(Nl+Na+Nb)) with the operator parities p and
 *   the particle numbers N of the *input* state.
 * - Wavefunction sectors (iL, sa, sb, iR) are listed in ascending
 *   (iL, sa, sb) order; sector s is a dimL[iL] x dimR[iR] row-major matrix at
 *   element offset psi_off[s].  sigma has the same layout.
 * - Operator blocks are row-major matrices (rows = dimension of the output
 *   sector, cols = dimension of the input sector) at element offset blk_off
 *   with leading dimension blk_ld (>= cols) in one value array; blk_off and
 *   blk_ld are multiples of 8 and blk_off + rows * blk_ld <= n_vals, so that
 *   the kernels read every row as 16-byte vectors.  An operator has at most
 *   one block per input sector, mapping in -> in + shift.
 * - Terms are (op_L, mono_a, mono_b, op_R, coef); op id -1 is the identity.
 *
 * Ownership and errors
 * --------------------
 * The library allocates no memory: every device buffer, including the
 * workspaces whose sizes the *_workspace_bytes queries return, belongs to the
 * caller and must outlive the calls that use it.  No exception crosses the
 * ABI; every entry point returns a tns_status.  Host-side validation happens
 * before any launch, so an error status means that nothing was enqueued,
 * except for TNS_ERR_HIP (a HIP call failed; the stream state is unknown).
 * Calls are asynchronous on the given stream unless stated otherwise.
 */
#ifndef TNS_H
#define TNS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TNS_OK = 0,
  TNS_ERR_ARG = -1,           /* null pointer, negative count, bad enum       */
  TNS_ERR_SHAPE = -2,         /* inconsistent dimensions or offsets           */
  TNS_ERR_QN = -3,            /* quantum numbers not conserved                */
  TNS_ERR_WORKSPACE = -4,     /* workspace smaller than required              */
  TNS_ERR_HIP = -5,           /* a HIP runtime call failed                    */
  TNS_ERR_NUMERIC = -6,       /* non-finite value detected (Davidson)         */
  TNS_ERR_NOT_CONVERGED = -7  /* Davidson hit max_iter                        */
} tns_status;

typedef enum {
  TNS_F64 = 0,     /* FP64 operands, FP64 MFMA, FP64 accumulation                     */
  TNS_F32 = 1,     /* FP32 operands, FP32 MFMA, FP32 accumulation per output tile     */
  TNS_BF16X3 = 2   /* split BF16 operands (hi + lo), three BF16 MFMA products          */
                   /* (lo*hi + hi*lo + hi*hi) with FP32 accumulation                  */
} tns_prec;

/* One two-site problem.  All pointers are HOST pointers to small index tables
 * (read only during tns_build_tasklist, which validates them and copies them
 * into the device workspace).  Operator values are passed separately, as
 * device pointers, to the compute calls. */
typedef struct {
  int32_t nL, nR;            /* left / right block sector counts                    */
  int32_t nS;                /* wavefunction sector count                           */
  int32_t nOps, nBlk, nTerms;
  int32_t target_N, target_2Sz;
  int64_t n_vals;            /* length (elements) of the operator value array       */
  const int32_t *qL;         /* [nL][2] (N, 2Sz)                                     */
  const int32_t *dimL;       /* [nL] 1..32768                                         */
  const int32_t *qR;         /* [nR][2]                                              */
  const int32_t *dimR;       /* [nR] 1..32768                                         */
  const int32_t *psi_sec;    /* [nS][4] (iL, sa, sb, iR), ascending (iL, sa, sb)     */
  const int64_t *psi_off;    /* [nS+1]                                               */
  const int32_t *op_side;    /* [nOps] 0 = left block, 1 = right block               */
  const int32_t *op_dN;      /* [nOps] shift of N                                    */
  const int32_t *op_d2Sz;    /* [nOps] shift of 2Sz                                  */
  const int32_t *blk_op;     /* [nBlk] owning operator                               */
  const int32_t *blk_in;     /* [nBlk] input sector                                  */
  const int32_t *blk_out;    /* [nBlk] output sector (= in + shift)                  */
  const int32_t *blk_rows;   /* [nBlk] = dim(out)                                    */
  const int32_t *blk_cols;   /* [nBlk] = dim(in)                                     */
  const int32_t *blk_ld;     /* [nBlk] >= cols, multiple of 8                        */
  const int64_t *blk_off;    /* [nBlk] element offset into the value array           */
  const int32_t *term_L;     /* [nTerms] left operator or -1                         */
  const int32_t *term_ma;    /* [nTerms] site-a monomial 0..15                       */
  const int32_t *term_mb;    /* [nTerms] site-b monomial 0..15                       */
  const int32_t *term_R;     /* [nTerms] right operator or -1                        */
  const double  *term_coef;  /* [nTerms]                                             */
} tns_problem;

/* One task of the task table (Section III.A.1, level 2): 40 bytes.
 * alpha = ((coef * a) * b) * sign in FP64 (a, b = site matrix elements).
 * cost  = flops of the cheaper evaluation order of the chain L A R^T
 * (Section III.B): 2qn(m+r) for (L A) R^T, 2mr(n+q) for L (A R^T), with q, m
 * the output / input left dimensions and r, n the output / input right
 * dimensions; order = 1 only if the second is strictly cheaper.  An identity
 * side drops its product (2mnr or 2qmn; 2mn if both are identities).  The
 * table is sorted by output sector, keeping term order inside a sector. */
typedef struct {
  int32_t out, in, term, lblk, rblk, order;
  double alpha;
  int64_t cost;
} tns_task;

/* Result of tns_build_tasklist.  Counts are host values; tasks and out_ptr are
 * device views into the build workspace; `opaque` holds the library's
 * schedule (device pointers into the same workspace). */
typedef struct {
  int64_t ntasks;         /* number of tasks                                        */
  int64_t nitems;         /* work items of the persistent kernel                    */
  int64_t nslots;         /* partial-result slots                                   */
  int64_t partial_elems;  /* elements of the partial buffer                         */
  int64_t total_flops;    /* sum of task costs (algorithmic flops per application)  */
  int64_t psi_dim;        /* elements of psi / sigma                                */
  const tns_task *tasks;  /* device [ntasks]                                        */
  const int32_t *out_ptr; /* device [nS+1] CSR over output sectors                  */
  uint8_t opaque[2048];
} tns_tasklist;

/* Bytes of device workspace tns_build_tasklist needs for this problem (host
 * only, no device call except a query of the device's compute-unit count).
 * The per-task arrays are sized for the exact task count, which the host
 * counts with the device enumeration's rule (Eq. (2): a task per term and
 * output sector whose operator blocks, site monomials and input sector all
 * exist).  Returns 0 when the problem fails host validation. */
size_t tns_tasklist_workspace_bytes(const tns_problem *prob);

/* Number of tasks of Eq. (2) the problem yields (Section III.A.1, level 2),
 * counted on the host with the rule tns_build_tasklist enumerates by: one
 * task per (term, output sector) whose left block, site monomials, right
 * block and input sector all exist.  Host only, no device call; `ntasks` is
 * a host pointer.  Validation errors as tns_build_tasklist; TNS_ERR_ARG for
 * a null `ntasks`. */
tns_status tns_count_tasks(const tns_problem *prob, int64_t *ntasks);

/* Levels 1-2 of Section III.A.1 on the device: validates the problem on the
 * host (shapes, ranges, quantum-number conservation of every block and every
 * term), copies the tables into `ws`, enumerates every (term, input sector)
 * pair that yields a contribution, sorts them by output sector (term order
 * inside a sector), and builds the work schedules of the persistent kernels
 * (output row panels x task chunks, longest first) for the forward product
 * and for its backward, including the adjoint task list (every task with its
 * sectors swapped and its blocks transposed, sorted by the new output sector)
 * that the backward's d psi runs as a forward product.  Synchronises the
 * stream a few times to read counts back (the first checks the device's
 * task count against the host count the workspace was sized for:
 * TNS_ERR_WORKSPACE if they differ).
 * `ws` must stay untouched while `out` is in use. */
tns_status tns_build_tasklist(const tns_problem *prob, void *ws, size_t ws_bytes,
                              tns_tasklist *out, hipStream_t stream);

/* Device workspace bytes of tns_apply_heff for a precision. */
size_t tns_apply_workspace_bytes(const tns_tasklist *tl, tns_prec prec);

/* Convert FP64 operator values (device, n elements) into the operand format of
 * `prec`: TNS_F64 copies, TNS_F32 rounds to float (`out` = float[n]),
 * TNS_BF16X3 writes hi = bf16(x) and lo = bf16(x - hi) (round to nearest
 * even each), `out` = uint16[2 n8] with n8 = n rounded up to a multiple of 8,
 * the halves interleaved in groups of 8 elements: element e's hi at u16
 * index 2e - (e mod 8) and its lo 8 further (8 hi values, then their 8 lo
 * values), so that 32 consecutive elements of a row (rows start at multiples
 * of 8) carry both halves in 128 contiguous bytes. */
tns_status tns_prepare_operands(tns_prec prec, const double *vals64, int64_t n, void *out,
                                hipStream_t stream);

/* Level 3, Eq. (2): sigma := beta * sigma + H_eff psi for beta in {0, 1}
 * (beta = 1 is the accumulate form B := B + alpha sum L_i A R_i^T).
 * op_vals: operands from tns_prepare_operands (device).  psi, sigma: device,
 * psi_dim elements of double (TNS_F64) or float (TNS_F32, TNS_BF16X3).
 * Deterministic: every output element is summed in a fixed order. */
tns_status tns_apply_heff(const tns_tasklist *tl, tns_prec prec, const void *op_vals,
                          const void *psi, void *sigma, double beta, void *ws, size_t ws_bytes,
                          hipStream_t stream);

/* tns_apply_heff for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same product, bitwise identical to tns_apply_heff, with the workspace
 * taken from a fixed device array that the library holds on every device it
 * runs on (TNS_NOALLOC_SCRATCH_BYTES = 64 MiB each, kept until the process
 * ends) instead of a caller buffer.  The call allocates nothing and enqueues
 * the same kernels on `stream` (asynchronous); the first call on a device
 * looks the array's address up once.  TNS_ERR_WORKSPACE when the product
 * needs more than the array (tns_apply_workspace_bytes(tl, prec) >
 * TNS_NOALLOC_SCRATCH_BYTES); other errors as tns_apply_heff.  Every call on
 * one device shares that device's array: calls whose executions overlap on
 * one device (several streams, several host threads) race and give wrong
 * results; serialise them. */
#define TNS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
tns_status tns_apply_heff_noalloc(const tns_tasklist *tl, tns_prec prec, const void *op_vals, const void *psi,
                                  void *sigma, double beta, hipStream_t stream);

/* Batched form of tns_apply_heff (level 3, Eq. (2), for many independent
 * problems): sigma_i := beta * sigma_i + H_eff,i psi_i for i < n, with one
 * persistent launch per GEMM phase for all instances together (work of the
 * costliest instances first), so that small and uneven instances share the
 * device.  tls[i]: task lists built by tns_build_tasklist on this device;
 * op_vals[i], psi[i], sigma[i]: that instance's operands (device pointers, as
 * in tns_apply_heff); the pointer arrays themselves are host memory, read
 * during the call (their contents are recorded into the launch arguments, so
 * the call can be captured into a hipGraph).  Results are bitwise identical
 * to n separate tns_apply_heff calls.  TNS_ERR_ARG for null entries, n <= 0
 * or task lists built for devices with different XCD counts. */
size_t tns_apply_batch_workspace_bytes(const tns_tasklist *const *tls, int n, tns_prec prec);
tns_status tns_apply_heff_batch(const tns_tasklist *const *tls, int n, tns_prec prec,
                                const void *const *op_vals, const void *const *psi, void *const *sigma,
                                double beta, void *ws, size_t ws_bytes, hipStream_t stream);

/* Tile shapes of the two forward GEMM phases per sector-size bucket (level 3
 * work decomposition, Alg. 2's batched products; the bucket choice is this
 * library's).  `tiles` packs four bytes: byte b is the tile extent (32, 64 or
 * 128 rows/columns, or 0 for 256 columns and 128 rows) used along any output
 * dimension d of bucket b = [d <= 32, d <= 64, d <= 128, d > 128]; the last
 * tile along a dimension shrinks to the multiple of 32 that covers what
 * remains.  Default 0x00804020 (32, 64, 128, 256 columns).  BF16X3 runs
 * tiles up to 128 x 256 whole; FP32 and FP64 run a tile wider than 128
 * columns as two.  tns_set_tiles rebuilds the forward work items on the device (the
 * backward's adjoint product keeps the default table) and
 * synchronises the stream (no product may be in flight on the task list);
 * workspaces and results do not depend on the table (the sums are taken in
 * the same order).  TNS_ERR_ARG for an invalid table. */
tns_status tns_set_tiles(tns_tasklist *tl, uint32_t tiles, hipStream_t stream);
uint32_t tns_get_tiles(const tns_tasklist *tl);

/* Autotuner of the tile table: coordinate descent over the four buckets
 * (largest first), each candidate timed as the median of three products
 * (tns_apply_heff, or tns_apply_heff_batch over all instances) with HIP
 * events after a warm-up product.  Leaves the fastest table set (on every
 * task list of a batch) and returns it in *tiles_out (nullable).  Arguments
 * as for the product calls; sigma is overwritten.  Synchronous. */
tns_status tns_autotune_tiles(tns_tasklist *tl, tns_prec prec, const void *op_vals, const void *psi,
                              void *sigma, void *ws, size_t ws_bytes, uint32_t *tiles_out,
                              hipStream_t stream);
tns_status tns_autotune_tiles_batch(tns_tasklist *const *tls, int n, tns_prec prec,
                                    const void *const *op_vals, const void *const *psi, void *const *sigma,
                                    void *ws, size_t ws_bytes, uint32_t *tiles_out, hipStream_t stream);

/* Backward of tns_apply_heff (the adjoint of each task's product L A R^T of
 * Eq. (2); the paper itself only applies H_eff) for a loss with
 * G = d loss / d sigma:
 * grad_psi   = sum_tasks alpha L^T G_out R            (psi layout; nullable)
 * grad_ops   = sum_tasks alpha G_out R A^T into L,    (operator-value layout,
 *              alpha G_out^T L A into R                 padding, gaps and blocks no
 *                                                       task uses are zero; nullable)
 * A = psi_in, L and R the task's blocks (identity sides contribute no
 * operator gradient).  grad_psi is the forward product (two grouped GEMM
 * phases) of the adjoint task list on a copy of the blocks, transposed into
 * the workspace on every call; the operator gradients run in a fused
 * persistent kernel.  Both outputs are overwritten (not accumulated); sums
 * run in a fixed order, so results are bitwise reproducible.  FP32 and FP64
 * only (TNS_ERR_ARG for TNS_BF16X3); TNS_ERR_WORKSPACE when ws_bytes is below
 * tns_backward_workspace_bytes.  psi, grad_sigma, grad_psi: device, psi_dim
 * elements of the precision's type; op_vals as for tns_apply_heff. */
size_t tns_backward_workspace_bytes(const tns_tasklist *tl, tns_prec prec);
tns_status tns_apply_heff_backward(const tns_tasklist *tl, tns_prec prec, const void *op_vals,
                                   const void *psi, const void *grad_sigma, void *grad_psi,
                                   void *grad_ops, void *ws, size_t ws_bytes, hipStream_t stream);

/* Davidson iteration for the lowest eigenpair (Section III: the effective
 * Hamiltonian is diagonalised with Davidson's method).  Vectors, projections,
 * Rayleigh-Ritz, residuals and the diagonal preconditioner are FP64 on the
 * device; the matrix-vector products run in `inner` precision.  With
 * refine != 0 and inner != TNS_F64, each inner convergence is followed by an
 * FP64 product w = H x, theta = <x, w>, r = w - theta x, and the inner
 * iteration restarts from (x, w) (iterative refinement: each restarted inner
 * iteration aims at a twentieth of the last FP64 residual) until the FP64
 * residual |r| <= tol_res; acceptance never rests on the inner-precision
 * residual.  The reported energy is the FP64 Rayleigh quotient. */
typedef struct {
  int32_t max_sub;     /* subspace size before restart (<= 64)   */
  int32_t keep;        /* Ritz vectors kept at restart           */
  int32_t max_iter;    /* total products in inner precision      */
  int32_t refine;      /* FP64 residual-correction rounds        */
  double tol_res;      /* residual 2-norm                         */
  double tol_e;        /* energy change between iterations       */
  tns_prec inner;
} tns_davidson_opts;

typedef struct {
  int32_t iters, matvecs_lo, matvecs_f64;
  double res_norm;     /* final FP64 residual norm                */
  double e_lo;         /* last inner-precision Ritz value         */
} tns_davidson_info;

size_t tns_davidson_workspace_bytes(const tns_tasklist *tl, const tns_davidson_opts *opts);
/* op_vals_lo: operands for opts->inner; op_vals_f64: FP64 values (may equal
 * op_vals_lo when inner == TNS_F64).  psi_inout: FP64 start vector (device),
 * overwritten by the eigenvector.  energy: host.  One scalar readback per
 * iteration synchronises the stream. */
tns_status tns_davidson(const tns_tasklist *tl, const tns_davidson_opts *opts, const void *op_vals_lo,
                        const double *op_vals_f64, double *psi_inout, double *energy,
                        tns_davidson_info *info, void *ws, size_t ws_bytes, hipStream_t stream);

/* Renormalisation (blocking) of block operators (Section IV.D): after a
 * two-site step the block grows by one site and every operator built on it is
 * carried over to the truncated basis of the enlarged block,
 *   O~_nu = U^T ( sum over nu's terms of coef (O (x) m) ) U,
 * each new operator nu an output of its own (no sum over operators).
 * Enlarged sector Q = q(i) + q(s) (old sector i, site state s); its product
 * basis lists the components (i, s) in ascending order, dim(i) states each;
 * the product state is C_l C_s |0>, so a site factor m picks up
 * (-1)^(parity(m) N(i)) from the old block's creators.  U_Q (full(Q) x
 * keep(Q), row-major, orthonormal columns expected but not checked) spans the
 * kept states.  The step runs as the chained products of Eq. (2) with the old
 * block in the middle and transposed isometry slices outside, on the forward
 * product's grouped GEMM phases.  All pointers of the problem are HOST
 * pointers read during tns_renorm_build. */
typedef struct {
  int32_t nL;                /* sectors of the block before the step            */
  const int32_t *qL;         /* [nL][2] (N, 2Sz) ascending                       */
  const int32_t *dimL;       /* [nL] 1..32768                                    */
  int32_t nOps, nBlk;        /* its operators and their blocks, as in tns_problem */
  const int32_t *op_dN, *op_d2Sz;
  const int32_t *blk_op, *blk_in, *blk_out, *blk_rows, *blk_cols, *blk_ld;
  const int64_t *blk_off;
  int64_t n_vals;
  int32_t nQ;                /* sectors of the enlarged block                    */
  const int32_t *qQ;         /* [nQ][2] ascending: exactly the sums qL[i] + q(s)  */
  const int32_t *keep;       /* [nQ] kept states, 1 .. full(Q)                    */
  const int64_t *u_off;      /* [nQ] element offset of U_Q in the isometry array  */
  int64_t n_u;               /* elements of the isometry array                   */
  int32_t nNew, nTerms;      /* new operators; terms new op += coef (O_op (x) m)  */
  const int32_t *term_new;   /* [nTerms] 0..nNew-1                                */
  const int32_t *term_op;    /* [nTerms] old operator or -1 (identity)            */
  const int32_t *term_mono;  /* [nTerms] site monomial 0..15                      */
  const double *term_coef;   /* [nTerms]                                          */
} tns_renorm_problem;

/* A built renormalisation step: the task table of its chained products (tl,
 * views into the build workspace; its output sectors are the new blocks) and
 * the output layout.  Output block k of new operator blk_new[k] maps enlarged
 * sector blk_in[k] to blk_out[k] = blk_in[k] + shift(new op): keep(out) rows,
 * keep(in) columns, leading dimension ld8(columns), at element offset off[k]
 * of out_vals (tns_renorm_out_table). */
typedef struct {
  int64_t ntasks, n_out_blk, out_elems, total_flops;
  tns_tasklist tl;
  uint8_t opaque[1024];
} tns_renorm_plan;

/* Build workspace bytes (host only; 0 when the problem fails validation:
 * shapes, ranges, quantum numbers of every block, the enlarged sector list,
 * one shift per new operator). */
size_t tns_renorm_workspace_bytes(const tns_renorm_problem *prob);
/* Validates, lists the tasks on the host (in term, block, site-state order),
 * copies the tables into `ws` and builds the schedules on the device;
 * synchronises the stream.  `ws` must stay untouched while the plan is used. */
tns_status tns_renorm_build(const tns_renorm_problem *prob, void *ws, size_t ws_bytes, tns_renorm_plan *out,
                            hipStream_t stream);
/* Host copies of the output block table (arrays of n_out_blk entries). */
tns_status tns_renorm_out_table(const tns_renorm_plan *plan, int32_t *blk_new, int32_t *blk_in, int32_t *blk_out,
                                int32_t *rows, int32_t *cols, int32_t *ld, int64_t *off);
/* One renormalisation step: op_vals (device, FP64, the old blocks' values at
 * blk_off), u_vals (device, FP64 isometries at u_off) -> out_vals (device,
 * out_elems of double for TNS_F64, float otherwise; padding zero).  The
 * products run in `prec` (operands converted on the device on every call).
 * Asynchronous on `stream`; deterministic. */
size_t tns_renorm_apply_workspace_bytes(const tns_renorm_plan *plan, tns_prec prec);
tns_status tns_renormalize(const tns_renorm_plan *plan, tns_prec prec, const double *op_vals, const double *u_vals,
                           void *out_vals, void *ws, size_t ws_bytes, hipStream_t stream);

/* Out-of-HBM products (Section II.B, Alg. 1: tree-traversal cache).  The
 * operator values stay in host memory (pinned for asynchronous copies) and
 * stream through a device cache of cache_elems elements managed as a stack:
 * the terms form a data dependency tree (left operator, then right operator,
 * then the terms), a depth-first walk loads an operator onto the stack on
 * entering its node and pops it on leaving, so a left operator stays resident
 * for all of its right partners and allocating is moving an offset.  The terms
 * pending when the stack is full or a left subtree ends form an epoch, run as
 * one product accumulating into sigma (its task list built at plan time with
 * the blocks' cache offsets).  Each operator's blocks are loaded as the element
 * range from its first to the end of its last block.
 * tns_ttcache_sizes: host and device bytes of the plan (host only: the walk,
 * the epochs' problems and their validation); TNS_ERR_WORKSPACE when a left
 * and a right operator together exceed the cache, TNS_ERR_ARG for an unknown
 * mode.  tns_ttcache_build: builds every epoch's task list into dev_ws
 * (synchronises the stream); host_buf and dev_ws must outlive the plan; mode
 * as given to tns_ttcache_sizes.
 * Buffering (mode): when the walk needs more than one epoch and every term's
 * two operators fit in half the cache, the plan may be double-buffered
 * (halves = 1): the walk runs on half the cache, keeping nothing from one
 * epoch to the next, and epochs alternate between the halves.  TNS_TT_DOUBLE
 * takes the halves whenever they fit, TNS_TT_SINGLE never, TNS_TT_AUTO when
 * the elements copied after the first epoch (the copies the halves hide)
 * exceed 3 M per extra epoch (a product's fixed cost, measured at D = 1024 in
 * FP64).
 * tns_apply_heff_streamed: sigma := H_eff psi (FP64 or FP32; host_vals in
 * that type, the problem's value layout), one copy per load and one product
 * per epoch.  Single-buffered, all of it in order on `stream`;
 * double-buffered, the copies run on a second stream of the device (created
 * on first use, default priority, shared by all calls on the device), each
 * epoch's copies after the earlier work on `stream` and after the product of
 * two epochs before, which overlaps them with the previous epoch's product;
 * the call's last product waits for every copy.  Calls that overlap in time
 * on one device must be issued on one stream.  The sum over epochs runs in a
 * fixed order (deterministic); it differs from tns_apply_heff's order only by
 * the grouping of terms. */
enum { TNS_TT_AUTO = 0, TNS_TT_SINGLE = 1, TNS_TT_DOUBLE = 2 };
typedef struct {
  int64_t n_epochs, n_loads;
  int64_t loaded_elems;  /* operator elements copied per product                    */
  int64_t naive_elems;   /* elements a per-term load of both operators would copy   */
  int64_t ntasks, total_flops, cache_elems;
  int64_t halves;        /* 1: double-buffered                                      */
  uint8_t opaque[256];
} tns_ttcache_plan;
tns_status tns_ttcache_sizes(const tns_problem *prob, int64_t cache_elems, int32_t mode, size_t *host_bytes,
                             size_t *dev_bytes, int64_t *n_epochs);
tns_status tns_ttcache_build(const tns_problem *prob, int64_t cache_elems, int32_t mode, void *host_buf,
                             size_t host_bytes, void *dev_ws, size_t dev_bytes, tns_ttcache_plan *out,
                             hipStream_t stream);
size_t tns_ttcache_apply_workspace_bytes(const tns_ttcache_plan *plan, tns_prec prec);
tns_status tns_apply_heff_streamed(const tns_ttcache_plan *plan, tns_prec prec, const void *host_vals, void *cache,
                                   const void *psi, void *sigma, void *ws, size_t ws_bytes, hipStream_t stream);

/* Spin-adapted (SU(2)) two-block products (Section IV.E).  Each block's
 * sectors are spin multiplets q = (N, 2S), ascending, holding dim multiplets
 * (one row per multiplet: its highest-weight state M = S).  Operators are
 * tensor operators of rank k (op_2k = 2k) changing N by op_dN (odd exactly for
 * half-integer k), given by reduced blocks (out x in, rows padded to blk_ld,
 * at blk_off in the value array, both multiples of 8 elements; at most one
 * block per (op, in, out); |S_in - k| <= S_out <= S_in + k) in the
 * Clebsch-Gordan convention <j' m'| T_q |j m> = <j m; k q | j' m'> <j'||T||j>.
 * A term is coef [T_L x T_R]^0 = coef sum_q <k q; k -q | 0 0> T_L,q T_R,-q
 * (left factor first; -1 = identity, rank 0; equal ranks, opposite dN).
 * Wavefunction sectors: the pairs (iL, iR) with N_L + N_R = target_N and
 * |S_L - S_R| <= S <= S_L + S_R, ascending (iL major), each a dimL[iL] x
 * dimR[iR] row-major matrix over the coupled states
 * sum_mL <S_L mL; S_R S-mL | S S> |a S_L mL> |b S_R S-mL>.
 * Each task of Eq. (2) (term, input sector, one reduced block per side) gets
 * alpha = coef x W x (-1)^(p_R N_L): W, the precalculated recoupling scalar
 * of the sectors' spins and the rank, sum_{mL, q} <S_L' mL+q; S_R' S-mL-q|S S>
 * <S_L mL; S_R S-mL|S S> <k q; k -q|0 0> <S_L mL; k q|S_L' mL+q>
 * <S_R S-mL; k -q|S_R' S-mL-q>, and the fermionic sign of the right factor's
 * parity p_R and the input's left electrons N_L.  Tasks with W = 0 are left
 * out; the rest is the U(1) path: the plan's task list runs on
 * tns_apply_heff (every precision, operand copies from tns_prepare_operands
 * over the value array) and tns_davidson. */
typedef struct {
  int32_t nL, nR, nOps, nBlk, nTerms;
  int32_t target_N, target_2S;
  int64_t n_vals;
  const int32_t *qL, *dimL;       /* [2 nL] (N, 2S) ascending, [nL] multiplets      */
  const int32_t *qR, *dimR;       /* [2 nR], [nR]                                    */
  const int32_t *op_side;         /* [nOps] 0 left, 1 right                          */
  const int32_t *op_2k, *op_dN;   /* [nOps] twice the rank, electron change          */
  const int32_t *blk_op, *blk_in, *blk_out, *blk_rows, *blk_cols, *blk_ld;  /* [nBlk] */
  const int64_t *blk_off;         /* [nBlk]                                          */
  const int32_t *term_L, *term_R; /* [nTerms] operator or -1                         */
  const double *term_coef;        /* [nTerms]                                        */
} tns_su2_problem;

typedef struct {
  int64_t n_sectors, psi_dim, ntasks, total_flops;
  tns_tasklist tl; /* forward-only task list: tns_apply_heff, tns_davidson */
} tns_su2_plan;

/* Build workspace bytes (host only; 0 when the problem fails validation:
 * shapes, ranges, layout, quantum numbers and triangle rules of every block,
 * equal ranks and conserved N of every term, a target with no sector). */
size_t tns_su2_workspace_bytes(const tns_su2_problem *prob);
/* Host only: the wavefunction sectors (sec_L, sec_R [n_sectors], psi_off
 * [n_sectors + 1]) and the task table (tasks [n_tasks], task_ptr
 * [n_sectors + 1] CSR over output sectors, term order kept inside a sector).
 * Counts always returned; arrays written when given (all four sector arrays
 * together; TNS_ERR_WORKSPACE when a capacity is short); TNS_ERR_QN when the
 * target has no sector. */
tns_status tns_su2_tables(const tns_su2_problem *prob, int32_t *sec_L, int32_t *sec_R, int64_t *psi_off,
                          int64_t cap_sectors, tns_task *tasks, int32_t *task_ptr, int64_t cap_tasks,
                          int64_t *n_sectors, int64_t *n_tasks);
/* Validates, lists the tasks with their scalars on the host and builds the
 * schedules into `ws` on the device (synchronises the stream); `ws` must stay
 * untouched while the plan is used. */
tns_status tns_su2_build(const tns_su2_problem *prob, void *ws, size_t ws_bytes, tns_su2_plan *out,
                         hipStream_t stream);

const char *tns_status_string(tns_status s);

/* Profiling aid: when all three events are non-null, the next forward
 * product records `before` on its stream immediately before its first GEMM
 * phase (the intermediates T_k), `mid` between the two phases and `after`
 * immediately after the second (the summed products), then forgets them, so
 * that a caller can time each MFMA kernel alone.  Pass nulls to disable.
 * Not thread-safe; the events belong to the caller. */
void tns_profile_events(hipEvent_t before, hipEvent_t mid, hipEvent_t after);

/* Measurement aid: the device's MFMA throughput measured with the MFMA
 * instruction each precision's product uses (v_mfma_f64_16x16x4,
 * v_mfma_f32_16x16x4, v_mfma_f32_16x16x32_bf16), every wave running 8
 * independent accumulator chains on register operands, 32 waves per CU; best
 * of 5 timed launches after a warm-up.  *tflops receives instruction flops
 * per second (BF16X3: BF16 flops, three per algorithmic flop of a product).
 * ws: device scratch of tns_mfma_peak_workspace_bytes() bytes (0 when the
 * device cannot be queried).  Synchronous; TNS_ERR_ARG for a bad precision or
 * iters <= 0. */
size_t tns_mfma_peak_workspace_bytes(void);
tns_status tns_mfma_peak(tns_prec prec, int iters, void *ws, size_t ws_bytes, double *tflops, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* TNS_H */
