// Davidson iteration for the lowest eigenpair of H_eff on the device.
//
// Section III: the effective Hamiltonian is diagonalised iteratively with the
// Lanczos or Davidson method, the matrix-vector product being the sum of
// Eq. (2).  The paper keeps the rest of that algebra on the host; here every
// vector operation stays in HBM in FP64: projected matrix S = V^T W,
// Rayleigh-Ritz by a parallel cyclic Jacobi eigensolver in one workgroup,
// Ritz vector and residual, diagonal (Davidson) preconditioner, two passes of
// classical Gram-Schmidt, restart.  Products H v run in the inner precision;
// with an inner precision below FP64 each inner convergence is followed by an
// FP64 product (residual correction) and, when needed, a restart from it.
// All reductions are two-level with a fixed order, so a solve is
// deterministic.
#include <algorithm>
#include <cmath>

#include "tns_internal.hpp"

namespace tns {

tns_status apply_impl(const Plan &p, tns_prec prec, const void *ops, const void *psi, void *sigma, double beta,
                      void *ws, size_t ws_bytes, hipStream_t st);

constexpr int DV_MAXSUB = 64;
constexpr int DOT_BLOCKS = 1024;
constexpr int DOT_THREADS = 256;
constexpr int DOT_ROWS = 16;  // basis vectors reduced per pass

static inline unsigned nbk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// diag(H_eff): tasks whose output sector is their input sector contribute
// alpha * L_ii * R_jj at element (i, j); one workgroup per sector, tasks in
// table order.
// ---------------------------------------------------------------------------
// The sector's diagonal tasks are staged in LDS in batches (table order kept).
constexpr int DIAG_BATCH = 256;
__global__ __launch_bounds__(256) void k_diag(Plan p, const double *__restrict__ ops, double *__restrict__ d) {
  __shared__ double s_alpha[DIAG_BATCH];
  __shared__ int64_t s_loff[DIAG_BATCH], s_roff[DIAG_BATCH];
  __shared__ int s_lld[DIAG_BATCH], s_rld[DIAG_BATCH];
  __shared__ int s_n;
  const int s = blockIdx.x;
  const int iL = p.psi_sec[4 * s], iR = p.psi_sec[4 * s + 3];
  const int m = p.dimL[iL], n = p.dimR[iR];
  const int64_t base = p.psi_off[s];
  const int t0 = p.out_ptr[s], t1 = p.out_ptr[s + 1];
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) d[base + e] = 0.0;
  for (int tb = t0; tb < t1; tb += DIAG_BATCH) {
    __syncthreads();
    if (threadIdx.x == 0) {  // compact this batch's diagonal tasks, in table order
      int c = 0;
      for (int t = tb; t < min(t1, tb + DIAG_BATCH); ++t) {
        const tns_task tk = p.tasks[t];
        if (tk.in != s) continue;
        s_alpha[c] = tk.alpha;
        s_loff[c] = tk.lblk >= 0 ? p.blk_off[tk.lblk] : -1;
        s_lld[c] = tk.lblk >= 0 ? p.blk_ld[tk.lblk] : 0;
        s_roff[c] = tk.rblk >= 0 ? p.blk_off[tk.rblk] : -1;
        s_rld[c] = tk.rblk >= 0 ? p.blk_ld[tk.rblk] : 0;
        ++c;
      }
      s_n = c;
    }
    __syncthreads();
    const int nb = s_n;
    for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
      const int i = e / n, j = e % n;
      double acc = d[base + e];
      for (int c = 0; c < nb; ++c) {
        const double li = s_loff[c] >= 0 ? ops[s_loff[c] + (int64_t)i * s_lld[c] + i] : 1.0;
        const double rj = s_roff[c] >= 0 ? ops[s_roff[c] + (int64_t)j * s_rld[c] + j] : 1.0;
        acc += s_alpha[c] * li * rj;
      }
      d[base + e] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// multi-dot: out[i] = <V_i, t> for i < k, V rows of length N (stride ldv).
// Pass 1 writes per-block partials, pass 2 sums them in block order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(DOT_THREADS) void k_multidot(const double *__restrict__ V, int64_t ldv, int k0, int kn,
                                                          const double *__restrict__ t, int64_t N,
                                                          double *__restrict__ part) {
  __shared__ double red[DOT_THREADS / 64][DOT_ROWS];
  double acc[DOT_ROWS];
#pragma unroll
  for (int i = 0; i < DOT_ROWS; ++i) acc[i] = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * DOT_THREADS + threadIdx.x; e < N; e += (int64_t)gridDim.x * DOT_THREADS) {
    const double tv = t[e];
#pragma unroll
    for (int i = 0; i < DOT_ROWS; ++i)
      if (i < kn) acc[i] += V[(int64_t)(k0 + i) * ldv + e] * tv;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < DOT_ROWS; ++i) {
    double v = acc[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[w][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < kn) {
    double v = 0.0;
    for (int ww = 0; ww < DOT_THREADS / 64; ++ww) v += red[ww][threadIdx.x];
    part[(int64_t)blockIdx.x * DV_MAXSUB + k0 + threadIdx.x] = v;
  }
}

// out[i] = sum over blocks of part[b][i]: one workgroup per i, each thread a
// strided partial sum, then a fixed-order tree (deterministic).
__global__ __launch_bounds__(256) void k_reduce_parts(const double *__restrict__ part, int nblocks, int k,
                                                      double *__restrict__ out) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  if (i >= k) return;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) v += part[(int64_t)b * DV_MAXSUB + i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// x = beta x + sum_i y[i] V_i
__global__ void k_combine(const double *__restrict__ V, int64_t ldv, int k, const double *__restrict__ y,
                          double *__restrict__ x, int64_t N, int beta) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double acc = beta ? x[e] : 0.0;
  for (int i = 0; i < k; ++i) acc += y[i] * V[(int64_t)i * ldv + e];
  x[e] = acc;
}

// t = t - sum_i c[i] V_i
__global__ void k_project_out(const double *__restrict__ V, int64_t ldv, int k, const double *__restrict__ c,
                              double *__restrict__ t, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double acc = t[e];
  for (int i = 0; i < k; ++i) acc -= c[i] * V[(int64_t)i * ldv + e];
  t[e] = acc;
}

// dst = src * (1 / sqrt(nrm2[0])) ; nrm2 is a device scalar (squared norm)
__global__ void k_scale_by_rnorm(const double *__restrict__ src, double *__restrict__ dst,
                                 const double *__restrict__ nrm2, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  dst[e] = src[e] / sqrt(nrm2[0]);
}

// r = w - theta x ; theta is a device scalar
__global__ void k_residual(const double *__restrict__ w, const double *__restrict__ x, const double *__restrict__ th,
                           double *__restrict__ r, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  r[e] = w[e] - th[0] * x[e];
}

// t = r / (theta - d), denominators below 1e-12 in magnitude replaced by a
// signed 1e-12
__global__ void k_precondition(const double *__restrict__ r, const double *__restrict__ d,
                               const double *__restrict__ th, double *__restrict__ t, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double den = th[0] - d[e];
  if (fabs(den) < 1e-12) den = den < 0 ? -1e-12 : 1e-12;
  t[e] = r[e] / den;
}

__global__ void k_to_f32(const double *__restrict__ x, float *__restrict__ y, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N) y[e] = (float)x[e];
}
__global__ void k_to_f64(const float *__restrict__ x, double *__restrict__ y, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N) y[e] = (double)x[e];
}
__global__ void k_copy(const double *__restrict__ x, double *__restrict__ y, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N) y[e] = x[e];
}

// ---------------------------------------------------------------------------
// Small dense symmetric eigenproblem (k <= 64) in one workgroup: cyclic
// Jacobi with the round-robin pairing, k/2 disjoint rotations per step.
// Inputs S[k][k] (ld DV_MAXSUB); outputs eigenvalues ascending in ev[k] and
// eigenvectors as columns of Y[k][k] (ld DV_MAXSUB).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_jacobi(const double *__restrict__ S, int k, double *__restrict__ ev,
                                                double *__restrict__ Y) {
  __shared__ double A[DV_MAXSUB][DV_MAXSUB + 1];
  __shared__ double Q[DV_MAXSUB][DV_MAXSUB + 1];
  __shared__ double cs[DV_MAXSUB / 2], sn[DV_MAXSUB / 2];
  __shared__ int pp[DV_MAXSUB / 2], qq[DV_MAXSUB / 2];
  __shared__ int order[DV_MAXSUB];
  __shared__ double off, nrm;
  const int tid = threadIdx.x;
  const int n = (k + 1) & ~1;  // even size (padded with an isolated zero row)
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    A[i][j] = (i < k && j < k) ? 0.5 * (S[i * DV_MAXSUB + j] + S[j * DV_MAXSUB + i]) : 0.0;
    Q[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (tid == 0) {
      double o = 0.0, a = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          a += A[i][j] * A[i][j];
          if (i != j) o += A[i][j] * A[i][j];
        }
      off = o;
      nrm = a;
    }
    __syncthreads();
    if (off <= 1e-30 * nrm || off == 0.0) break;
    for (int step = 0; step < n - 1; ++step) {
      // round-robin pairing: position 0 fixed, others rotate
      if (tid < n / 2) {
        auto idx = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + step) % (n - 1); };
        int a = idx(tid), b = idx(n - 1 - tid);
        if (a > b) { const int t = a; a = b; b = t; }
        pp[tid] = a;
        qq[tid] = b;
        const double apq = A[a][b];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double tau = (A[b][b] - A[a][a]) / (2.0 * apq);
          const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = tid; e < (n / 2) * n; e += blockDim.x) {
        const int r = e / n, j = e % n;
        const int a = pp[r], b = qq[r];
        const double c = cs[r], s = sn[r];
        const double x = A[a][j], y = A[b][j];
        A[a][j] = c * x - s * y;
        A[b][j] = s * x + c * y;
      }
      __syncthreads();
      // columns: A <- A J, Q <- Q J
      for (int e = tid; e < (n / 2) * n; e += blockDim.x) {
        const int r = e / n, i = e % n;
        const int a = pp[r], b = qq[r];
        const double c = cs[r], s = sn[r];
        const double x = A[i][a], y = A[i][b];
        A[i][a] = c * x - s * y;
        A[i][b] = s * x + c * y;
        const double u = Q[i][a], v = Q[i][b];
        Q[i][a] = c * u - s * v;
        Q[i][b] = s * u + c * v;
      }
      __syncthreads();
    }
  }
  // sort the k genuine eigenpairs ascending (the padded index keeps value 0
  // and a unit vector outside the first k rows; it is identified by Q)
  if (tid == 0) {
    int m = 0;
    for (int j = 0; j < n; ++j) {
      if (n != k) {
        // skip the column that is the padding unit vector
        if (fabs(Q[n - 1][j]) > 0.5) continue;
      }
      order[m++] = j;
    }
    for (int i = 1; i < m; ++i) {
      const int v = order[i];
      int j = i - 1;
      while (j >= 0 && A[order[j]][order[j]] > A[v][v]) { order[j + 1] = order[j]; --j; }
      order[j + 1] = v;
    }
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e % k;
    Y[i * DV_MAXSUB + j] = Q[i][order[j]];
  }
  if (tid < k) ev[tid] = A[order[tid]][order[tid]];
}

// S[i][kk] = S[kk][i] = (<V_i, W_kk> + <W_i, V_kk>) / 2 for i <= kk.  With
// exact0, W_0 = H V_0 holds an FP64 product while the later columns of W come
// from the inner precision: the coupling of V_0 is then taken from the exact
// side alone, <W_0, V_kk> (after an FP64 correction it is about the residual
// size, below the inner precision's rounding of <V_0, W_kk>).
__global__ void k_fill_S(double *__restrict__ S, const double *__restrict__ vw, const double *__restrict__ wv,
                         int kk, int exact0) {
  const int i = threadIdx.x;
  if (i > kk) return;
  const double v = (exact0 && i == 0) ? wv[0] : 0.5 * (vw[i] + wv[i]);
  S[i * DV_MAXSUB + kk] = v;
  S[kk * DV_MAXSUB + i] = v;
}

// After a restart the projected matrix is diagonal in the kept Ritz basis.
__global__ void k_reset_S(double *__restrict__ S, const double *__restrict__ ev, int keep) {
  for (int e = threadIdx.x; e < DV_MAXSUB * DV_MAXSUB; e += blockDim.x) {
    const int i = e / DV_MAXSUB, j = e % DV_MAXSUB;
    S[e] = (i == j && i < keep) ? ev[i] : 0.0;
  }
}

// column j of Y into contiguous y
__global__ void k_col(const double *__restrict__ Y, int k, int j, double *__restrict__ y) {
  const int i = threadIdx.x;
  if (i < k) y[i] = Y[i * DV_MAXSUB + j];
}

__global__ void k_set_scalar(double *p, double v) { *p = v; }

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
struct DvWs {
  double *V, *W, *T, *x, *w, *r, *t, *d;
  float *lo_in, *lo_out;
  double *part, *S, *Y, *ev, *y, *c, *sc;  // sc: device scalars
  void *aws;
  size_t aws_bytes;
};

static size_t apply_ws_bytes(const tns_tasklist *tl, tns_prec p) { return tns_apply_workspace_bytes(tl, p); }

static size_t dv_layout(const tns_tasklist *tl, const tns_davidson_opts *o, char *base, DvWs *out) {
  const Plan &p = plan_of(tl);
  const int64_t N = p.psi_dim;
  Carve cv{base, 0, 0};
  DvWs d;
  d.V = cv.take<double>((size_t)o->max_sub * N);
  d.W = cv.take<double>((size_t)o->max_sub * N);
  d.T = cv.take<double>((size_t)o->keep * N);
  d.x = cv.take<double>(N); d.w = cv.take<double>(N); d.r = cv.take<double>(N);
  d.t = cv.take<double>(N); d.d = cv.take<double>(N);
  d.lo_in = cv.take<float>(N); d.lo_out = cv.take<float>(N);
  d.part = cv.take<double>((size_t)DOT_BLOCKS * DV_MAXSUB);
  d.S = cv.take<double>(DV_MAXSUB * DV_MAXSUB);
  d.Y = cv.take<double>(DV_MAXSUB * DV_MAXSUB);
  d.ev = cv.take<double>(DV_MAXSUB);
  d.y = cv.take<double>(DV_MAXSUB);
  d.c = cv.take<double>(2 * DV_MAXSUB);
  d.sc = cv.take<double>(16);
  d.aws_bytes = std::max(apply_ws_bytes(tl, TNS_F64), apply_ws_bytes(tl, o->inner));
  d.aws = cv.take<char>(d.aws_bytes);
  if (out) *out = d;
  return cv.off + 256;
}

static tns_status check_opts(const tns_davidson_opts *o) {
  if (!o) return TNS_ERR_ARG;
  if (o->max_sub < 2 || o->max_sub > DV_MAXSUB || o->keep < 1 || o->keep >= o->max_sub || o->max_iter < 1 ||
      o->refine < 0 || !(o->tol_res > 0) || !(o->tol_e >= 0))
    return TNS_ERR_ARG;
  if (o->inner != TNS_F64 && o->inner != TNS_F32 && o->inner != TNS_BF16X3) return TNS_ERR_ARG;
  return TNS_OK;
}

// out[0..k) = <rows of V, t>
static void multidot(const double *V, int64_t ldv, int k, const double *t, int64_t N, DvWs &d, double *out,
                     hipStream_t st) {
  for (int k0 = 0; k0 < k; k0 += DOT_ROWS)
    hipLaunchKernelGGL(k_multidot, dim3(DOT_BLOCKS), dim3(DOT_THREADS), 0, st, V, ldv, k0, std::min(DOT_ROWS, k - k0),
                       t, N, d.part);
  hipLaunchKernelGGL(k_reduce_parts, dim3(std::max(k, 1)), dim3(256), 0, st, d.part, DOT_BLOCKS, k, out);
}

// dst = H src in precision prec (src, dst FP64)
static tns_status matvec(const Plan &p, tns_prec prec, const void *ops, const double *src, double *dst, DvWs &d,
                         hipStream_t st) {
  const int64_t N = p.psi_dim;
  if (prec == TNS_F64) return apply_impl(p, TNS_F64, ops, src, dst, 0.0, d.aws, d.aws_bytes, st);
  hipLaunchKernelGGL(k_to_f32, dim3(nbk(N, 256)), dim3(256), 0, st, src, d.lo_in, N);
  tns_status s = apply_impl(p, prec, ops, d.lo_in, d.lo_out, 0.0, d.aws, d.aws_bytes, st);
  if (s != TNS_OK) return s;
  hipLaunchKernelGGL(k_to_f64, dim3(nbk(N, 256)), dim3(256), 0, st, d.lo_out, dst, N);
  return TNS_OK;
}

}  // namespace tns

using namespace tns;

extern "C" size_t tns_davidson_workspace_bytes(const tns_tasklist *tl, const tns_davidson_opts *opts) {
  if (!tl || check_opts(opts) != TNS_OK) return 0;
  return dv_layout(tl, opts, nullptr, nullptr);
}

extern "C" tns_status tns_davidson(const tns_tasklist *tl, const tns_davidson_opts *o, const void *ops_lo,
                                   const double *ops64, double *psi, double *energy, tns_davidson_info *info,
                                   void *ws, size_t ws_bytes, hipStream_t st) {
  if (!tl || !ops_lo || !ops64 || !psi || !energy || !ws) return TNS_ERR_ARG;
  tns_status s = check_opts(o);
  if (s != TNS_OK) return s;
  if (ws_bytes < dv_layout(tl, o, nullptr, nullptr)) return TNS_ERR_WORKSPACE;
  const Plan &p = plan_of(tl);
  const int64_t N = p.psi_dim;
  if (N == 0) return TNS_ERR_SHAPE;
  DvWs d;
  dv_layout(tl, o, (char *)ws, &d);
  const unsigned g = nbk(N, 256);
  const bool mixed = o->inner != TNS_F64;
  tns_davidson_info inf;
  memset(&inf, 0, sizeof(inf));

  hipLaunchKernelGGL(k_diag, dim3(std::max(1, p.nS)), dim3(256), 0, st, p, ops64, d.d);
  // V_0 = psi / |psi|
  multidot(psi, 0, 1, psi, N, d, d.sc + 0, st);
  hipLaunchKernelGGL(k_scale_by_rnorm, dim3(g), dim3(256), 0, st, psi, d.V, d.sc + 0, N);
  s = matvec(p, o->inner, ops_lo, d.V, d.W, d, st);
  if (s != TNS_OK) return s;
  inf.matvecs_lo += 1;
  int k = 1;
  double theta_prev = NAN, best_res = INFINITY;
  int stall = 0, rounds = 0;
  bool rounds_done = false;  // an FP64 correction has run
  bool w0_exact = false;     // W_0 is the FP64 product of V_0 (refinement restart)
  double r64_prev = INFINITY;
  bool accepted = false;
  // residual floor of the inner products (relative rounding of one product)
  const double eps_inner = o->inner == TNS_F32 ? 1e-6 : (o->inner == TNS_BF16X3 ? 3e-5 : 0.0);
  double h[8];
  bool done = false;
  tns_status result = TNS_OK;
  int budget = o->max_iter;
  while (!done) {
    // new row / column of S
    multidot(d.V, N, k, d.W + (int64_t)(k - 1) * N, N, d, d.c, st);
    multidot(d.W, N, k, d.V + (int64_t)(k - 1) * N, N, d, d.c + DV_MAXSUB, st);
    hipLaunchKernelGGL(k_fill_S, dim3(1), dim3(DV_MAXSUB), 0, st, d.S, d.c, d.c + DV_MAXSUB, k - 1,
                       (int)w0_exact);
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(256), 0, st, d.S, k, d.ev, d.Y);
    hipLaunchKernelGGL(k_col, dim3(1), dim3(DV_MAXSUB), 0, st, d.Y, k, 0, d.y);
    hipLaunchKernelGGL(k_combine, dim3(g), dim3(256), 0, st, d.V, N, k, d.y, d.x, N, 0);
    hipLaunchKernelGGL(k_combine, dim3(g), dim3(256), 0, st, d.W, N, k, d.y, d.w, N, 0);
    hipLaunchKernelGGL(k_residual, dim3(g), dim3(256), 0, st, d.w, d.x, d.ev, d.r, N);
    multidot(d.r, 0, 1, d.r, N, d, d.sc + 1, st);
    // correction vector, two classical Gram-Schmidt passes
    hipLaunchKernelGGL(k_precondition, dim3(g), dim3(256), 0, st, d.r, d.d, d.ev, d.t, N);
    for (int pass = 0; pass < 2; ++pass) {
      multidot(d.V, N, k, d.t, N, d, d.c, st);
      hipLaunchKernelGGL(k_project_out, dim3(g), dim3(256), 0, st, d.V, N, k, d.c, d.t, N);
    }
    multidot(d.t, 0, 1, d.t, N, d, d.sc + 2, st);
    TNS_HIP(hipGetLastError());
    // one readback per iteration: theta, |r|^2, |t|^2, theta_2
    TNS_HIP(hipMemcpyAsync(h, d.sc, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    TNS_HIP(hipMemcpyAsync(h + 3, d.ev, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    TNS_HIP(hipStreamSynchronize(st));
    const double theta = h[3], res = std::sqrt(std::max(h[1], 0.0)), tn = std::sqrt(std::max(h[2], 0.0));
    inf.iters += 1;
    inf.e_lo = theta;
    if (!std::isfinite(theta) || !std::isfinite(res)) { result = TNS_ERR_NUMERIC; break; }
    if (res < 0.9 * best_res) { best_res = res; stall = 0; } else { ++stall; }
    const double floor_res = eps_inner * std::max(1.0, std::fabs(theta));
    const bool dtheta_ok = std::isfinite(theta_prev) && std::fabs(theta - theta_prev) <= o->tol_e;
    // inner convergence: the target residual reached, or a stall of the
    // residual close to the precision floor, or breakdown of the correction.
    // The first round aims at tol_res (or the inner rounding floor).  After an
    // FP64 correction the inner iteration restarts from (x, H64 x): its
    // residual is then exact up to the inner rounding of the correction alone,
    // so it aims at a fraction of the last FP64 residual (iterative refinement).
    const double target = rounds_done ? std::max(0.5 * o->tol_res, 0.05 * r64_prev)
                                      : std::max(o->tol_res, floor_res);
    const bool conv_inner = (res <= target && dtheta_ok) ||
                            (mixed && stall >= 4 && res <= 100.0 * floor_res) ||
                            tn < 1e-10 * std::max(1.0, res);
    theta_prev = theta;
    if (conv_inner || budget <= 1) {
      if (!mixed) {
        accepted = res <= o->tol_res;
        break;
      }
      // FP64 residual correction: w64 = H x, theta64 = <x, w64>, r64 = w64 - theta64 x
      s = matvec(p, TNS_F64, ops64, d.x, d.w, d, st);
      if (s != TNS_OK) return s;
      inf.matvecs_f64 += 1;
      multidot(d.x, 0, 1, d.w, N, d, d.sc + 3, st);
      multidot(d.x, 0, 1, d.x, N, d, d.sc + 4, st);
      TNS_HIP(hipMemcpyAsync(h, d.sc + 3, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      TNS_HIP(hipStreamSynchronize(st));
      const double th64 = h[0] / h[1];
      hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, st, d.sc + 5, th64);
      hipLaunchKernelGGL(k_residual, dim3(g), dim3(256), 0, st, d.w, d.x, d.sc + 5, d.r, N);
      multidot(d.r, 0, 1, d.r, N, d, d.sc + 6, st);
      TNS_HIP(hipMemcpyAsync(h, d.sc + 6, sizeof(double), hipMemcpyDeviceToHost, st));
      TNS_HIP(hipStreamSynchronize(st));
      const double r64 = std::sqrt(std::max(h[0], 0.0));
      // Accept on the FP64 residual alone.  An energy bound r64^2 / gap would
      // need a lower bound of the gap lambda2 - lambda1; the Ritz values of
      // the (restarted, low-precision) subspace only bound lambda2 from above,
      // so the gap cannot be bounded safely from them.
      const bool ok = r64 <= o->tol_res;
      rounds_done = true;
      r64_prev = r64;
      if (ok) accepted = true;
      if (ok || rounds >= o->refine || budget <= 1) break;
      ++rounds;
      // restart the inner iteration from (x / |x|, w64 / |x|)
      hipLaunchKernelGGL(k_scale_by_rnorm, dim3(g), dim3(256), 0, st, d.x, d.V, d.sc + 4, N);
      hipLaunchKernelGGL(k_scale_by_rnorm, dim3(g), dim3(256), 0, st, d.w, d.W, d.sc + 4, N);
      hipLaunchKernelGGL(k_reset_S, dim3(1), dim3(256), 0, st, d.S, d.ev, 0);
      w0_exact = true;
      k = 1;
      best_res = INFINITY;
      stall = 0;
      theta_prev = NAN;
      continue;
    }
    --budget;
    if (k == o->max_sub) {
      // restart with the keep lowest Ritz vectors: V <- V Y[:, :keep], W <- W Y[:, :keep]
      for (int j = 0; j < o->keep; ++j) {
        hipLaunchKernelGGL(k_col, dim3(1), dim3(DV_MAXSUB), 0, st, d.Y, k, j, d.c);
        hipLaunchKernelGGL(k_combine, dim3(g), dim3(256), 0, st, d.V, N, k, d.c, d.T + (int64_t)j * N, N, 0);
      }
      for (int j = 0; j < o->keep; ++j)
        hipLaunchKernelGGL(k_copy, dim3(g), dim3(256), 0, st, d.T + (int64_t)j * N, d.V + (int64_t)j * N, N);
      for (int j = 0; j < o->keep; ++j) {
        hipLaunchKernelGGL(k_col, dim3(1), dim3(DV_MAXSUB), 0, st, d.Y, k, j, d.c);
        hipLaunchKernelGGL(k_combine, dim3(g), dim3(256), 0, st, d.W, N, k, d.c, d.T + (int64_t)j * N, N, 0);
      }
      for (int j = 0; j < o->keep; ++j)
        hipLaunchKernelGGL(k_copy, dim3(g), dim3(256), 0, st, d.T + (int64_t)j * N, d.W + (int64_t)j * N, N);
      hipLaunchKernelGGL(k_reset_S, dim3(1), dim3(256), 0, st, d.S, d.ev, o->keep);
      w0_exact = false;  // the kept columns mix inner-precision products
      k = o->keep;
      // t is orthogonal to the old span, which contains the new one
    }
    hipLaunchKernelGGL(k_scale_by_rnorm, dim3(g), dim3(256), 0, st, d.t, d.V + (int64_t)k * N, d.sc + 2, N);
    s = matvec(p, o->inner, ops_lo, d.V + (int64_t)k * N, d.W + (int64_t)k * N, d, st);
    if (s != TNS_OK) return s;
    inf.matvecs_lo += 1;
    ++k;
  }
  if (result != TNS_OK && result != TNS_ERR_NOT_CONVERGED) {
    if (info) *info = inf;
    return result;
  }
  // final FP64 Rayleigh quotient of the normalised Ritz vector
  multidot(d.x, 0, 1, d.x, N, d, d.sc + 4, st);
  hipLaunchKernelGGL(k_scale_by_rnorm, dim3(g), dim3(256), 0, st, d.x, psi, d.sc + 4, N);
  s = matvec(p, TNS_F64, ops64, psi, d.w, d, st);
  if (s != TNS_OK) return s;
  inf.matvecs_f64 += 1;
  multidot(psi, 0, 1, d.w, N, d, d.sc + 3, st);
  hipLaunchKernelGGL(k_residual, dim3(g), dim3(256), 0, st, d.w, psi, d.sc + 3, d.r, N);
  multidot(d.r, 0, 1, d.r, N, d, d.sc + 6, st);
  TNS_HIP(hipGetLastError());
  TNS_HIP(hipMemcpyAsync(h, d.sc + 3, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  TNS_HIP(hipStreamSynchronize(st));
  *energy = h[0];
  inf.res_norm = std::sqrt(std::max(h[3], 0.0));
  if (info) *info = inf;
  if (!std::isfinite(*energy)) return TNS_ERR_NUMERIC;
  if (!accepted && inf.res_norm > o->tol_res) return TNS_ERR_NOT_CONVERGED;
  return TNS_OK;
}
