// Sparse matrix-vector product on the 27-point node-block matrix, CG vector
// updates and deterministic reductions (Section 3.1: the CG iteration).
//
// The assembled matrix is stored structure-of-arrays, A[d][c][c'][node], with
// d the lattice offset (dx,dy,dz) in {-1,0,1}^3; column indices are implicit
// in the structured grid, so a row moves 27*nc*nc*8 bytes of values only.
// Dirichlet DOFs are identity rows/columns in the full numbering and hold 0 in
// every vector, which keeps every kernel free of index maps.
#include "gn_internal.h"

namespace {

constexpr int RBLK = 512;   // blocks of the fixed-shape vector reductions
constexpr int RTHR = 256;

template <int NC>
__global__ __launch_bounds__(256) void k_spmv(int NX, int NY, int NZ, const double* __restrict__ A,
                                              const double* __restrict__ x, double* __restrict__ y,
                                              double* __restrict__ part,
                                              const double* __restrict__ done) {
  __shared__ double sh[16];
  if (done && *done != 0.0) return;
  const int64_t n_node = (int64_t)NX * NY * NZ;
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dotv = 0.0;
  if (node < n_node) {
    int i = (int)(node % NX), j = (int)((node / NX) % NY), k = (int)(node / ((int64_t)NX * NY));
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    // scalar case: the assembled stencil holds exact zeros for neighbours
    // outside the grid, so their index is only clamped into range (0 * x adds
    // nothing): 27 unconditional loads, no divergent branches.  Elasticity keeps
    // the branches (its 27 x 12 unconditional loads would not fit the registers).
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
      if (NC > 1 && (k + dz < 0 || k + dz >= NZ)) continue;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        if (NC > 1 && (j + dy < 0 || j + dy >= NY)) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (NC > 1 && (i + dx < 0 || i + dx >= NX)) continue;
          const int d = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
          int64_t nb = node + dx + (int64_t)NX * (dy + (int64_t)NY * dz);
          if (NC == 1) nb = nb < 0 ? 0 : (nb >= n_node ? n_node - 1 : nb);
          double xv[NC];
#pragma unroll
          for (int c2 = 0; c2 < NC; ++c2) xv[c2] = x[nb * NC + c2];
#pragma unroll
          for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int c2 = 0; c2 < NC; ++c2)
              acc[c] += A[((int64_t)(d * NC + c) * NC + c2) * n_node + node] * xv[c2];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      y[node * NC + c] = acc[c];
      dotv += acc[c] * x[node * NC + c];
    }
  }
  if (part) {
    double s = block_sum(dotv, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
  }
}

// partial sums of (sum_j |A_ij| |x_j|)^2 over rows: the scale of the rounding
// error of any FP64 evaluation of A x, eps * || |A| |x| ||
template <int NC>
__global__ __launch_bounds__(256) void k_absmv(int NX, int NY, int NZ, const double* __restrict__ A,
                                               const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[16];
  const int64_t n_node = (int64_t)NX * NY * NZ;
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (node < n_node) {
    int i = (int)(node % NX), j = (int)((node / NX) % NY), k = (int)(node / ((int64_t)NX * NY));
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    for (int d = 0; d < 27; ++d) {
      const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
      if (i + dx < 0 || i + dx >= NX || j + dy < 0 || j + dy >= NY || k + dz < 0 || k + dz >= NZ) continue;
      const int64_t nb = node + dx + (int64_t)NX * (dy + (int64_t)NY * dz);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2)
          acc[c] += fabs(A[((int64_t)(d * NC + c) * NC + c2) * n_node + node]) * fabs(x[nb * NC + c2]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) v += acc[c] * acc[c];
  }
  double s = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_scatter_free(int64_t n_free, const int* __restrict__ f2f, const double* __restrict__ xf,
                               double* __restrict__ xfull) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_free) xfull[f2f[t]] = xf[t];
}
__global__ void k_gather_free(int64_t n_free, const int* __restrict__ f2f, const double* __restrict__ xfull,
                              double* __restrict__ xf) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_free) xf[t] = xfull[f2f[t]];
}

}  // namespace

namespace gnk {

int reduce_blocks() { return RBLK; }

void spmv_flag(const gn_problem* p, const double* x, double* y, double* part, const double* done,
               hipStream_t s) {
  dim3 grid((unsigned)((p->n_node + 255) / 256));
  GnProfScope prof(PROF_SPMV, (double)p->n_node * (27.0 * p->nc * p->nc * 8.0 + 2.0 * p->nc * 8.0), s);
  if (p->nc == 3)
    hipLaunchKernelGGL(k_spmv<3>, grid, dim3(256), 0, s, p->nn[0], p->nn[1], p->nn[2], p->d_A, x,
                       y, part, done);
  else
    hipLaunchKernelGGL(k_spmv<1>, grid, dim3(256), 0, s, p->nn[0], p->nn[1], p->nn[2], p->d_A, x,
                       y, part, done);
  GN_CHECK_LAUNCH();
}

int spmv_blocks(const gn_problem* p) { return (int)((p->n_node + 255) / 256); }

void absmv_partial(const gn_problem* p, const double* x, double* part, hipStream_t s) {
  dim3 grid((unsigned)((p->n_node + 255) / 256));
  if (p->nc == 3)
    hipLaunchKernelGGL(k_absmv<3>, grid, dim3(256), 0, s, p->nn[0], p->nn[1], p->nn[2], p->d_A, x, part);
  else
    hipLaunchKernelGGL(k_absmv<1>, grid, dim3(256), 0, s, p->nn[0], p->nn[1], p->nn[2], p->d_A, x, part);
  GN_CHECK_LAUNCH();
}

void scatter_free(const gn_problem* p, const double* xf, double* xfull, hipStream_t s) {
  GN_HIP(hipMemsetAsync(xfull, 0, sizeof(double) * p->n_dof, s));
  hipLaunchKernelGGL(k_scatter_free, dim3((unsigned)((p->n_free + 255) / 256)), dim3(256), 0, s,
                     p->n_free, p->d_free2full, xf, xfull);
  GN_CHECK_LAUNCH();
}

void gather_free(const gn_problem* p, const double* xfull, double* xf, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_free, dim3((unsigned)((p->n_free + 255) / 256)), dim3(256), 0, s,
                     p->n_free, p->d_free2full, xfull, xf);
  GN_CHECK_LAUNCH();
}

}  // namespace gnk

// ---------------------------------------------------------------------------
// CG vector kernels with device-resident scalars.
// scal layout: see enum in cg.h-like block below.
// ---------------------------------------------------------------------------
namespace {


__global__ __launch_bounds__(RTHR) void k_dot(int64_t n, const double* __restrict__ a,
                                              const double* __restrict__ b, double* __restrict__ part,
                                              const double* __restrict__ done) {
  __shared__ double sh[16];
  if (done && *done != 0.0) return;
  double v = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    v += a[t] * b[t];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// x += alpha p ; r -= alpha q ; partial r.r
__global__ __launch_bounds__(RTHR) void k_update_xr(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ p, const double* __restrict__ q,
                                                    const double* __restrict__ scal, double* __restrict__ part) {
  __shared__ double sh[16];
  if (scal[S_DONE] != 0.0) return;
  double alpha = scal[S_ALPHA];
  double v = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    x[t] += alpha * p[t];
    double rv = r[t] - alpha * q[t];
    r[t] = rv;
    v += rv * rv;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// p = z + beta p
__global__ __launch_bounds__(RTHR) void k_update_p(int64_t n, double* __restrict__ p, const double* __restrict__ z,
                                                   const double* __restrict__ scal) {
  if (scal[S_DONE] != 0.0) return;
  double beta = scal[S_BETA];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = z[t] + beta * p[t];
}

__global__ __launch_bounds__(RTHR) void k_resid(int64_t n, const double* __restrict__ b,
                                                const double* __restrict__ q, double* __restrict__ part) {
  __shared__ double sh[16];
  double v = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    double d = b[t] - q[t];
    v += d * d;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// r = b - q ; partial r.r
__global__ __launch_bounds__(RTHR) void k_sub(int64_t n, const double* __restrict__ b,
                                              const double* __restrict__ q, double* __restrict__ r,
                                              double* __restrict__ part) {
  __shared__ double sh[16];
  double v = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    double d = b[t] - q[t];
    r[t] = d;
    v += d * d;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// number of NaN / infinite entries in ncol columns of length n (leading dim ld)
__global__ void k_count_nonfinite(int64_t n, int ncol, int64_t ld, const double* __restrict__ x,
                                  unsigned* __restrict__ count) {
  unsigned c = 0;
  const int64_t tot = n * ncol;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x)
    c += isfinite(x[(t / n) * ld + t % n]) ? 0u : 1u;
  if (c) atomicAdd(count, c);
}

__global__ void k_copy(int64_t n, double* __restrict__ dst, const double* __restrict__ src,
                       const double* __restrict__ done) {
  if (done && *done != 0.0) return;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = src[t];
}


// single block: fixed-order sum of the partials, then the scalar recurrence
__global__ void k_finalize(const double* __restrict__ part, int nb, int op, double* __restrict__ scal,
                           double* __restrict__ hist, double rtol) {
  __shared__ double sh[16];
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[i];
  double s = block_sum(v, sh);
  if (threadIdx.x != 0) return;
  if (op == OP_BB) {
    scal[S_BB] = s;
    scal[S_RR] = s;
    scal[S_TOL2] = rtol * rtol * s;
    scal[S_DONE] = (s == 0.0) ? 1.0 : 0.0;
    scal[S_ITER] = 0.0;
    scal[S_BREAK] = 0.0;
    return;
  }
  if (op == OP_RESTART) {   // new residual b - A x of a restarted sequence
    scal[S_RR] = s;
    scal[S_DONE] = (s <= scal[S_TOL2] || (int)scal[S_ITER] >= (int)scal[S_MAXIT]) ? 1.0 : 0.0;
    return;
  }
  if (scal[S_DONE] != 0.0) return;
  int it = (int)scal[S_ITER];
  switch (op) {
    case OP_RZ0:
      scal[S_RZ] = s;
      break;
    case OP_ALPHA:
      scal[S_PQ] = s;
      if (!(s > 0.0)) {
        scal[S_BREAK] = 1.0;
        scal[S_DONE] = 1.0;
        scal[S_ALPHA] = 0.0;
      } else {
        scal[S_ALPHA] = scal[S_RZ] / s;
      }
      break;
    case OP_RR:
      scal[S_RR] = s;
      hist[2 * it] = scal[S_ALPHA];
      scal[S_ITER] = it + 1;
      if (s <= scal[S_TOL2] || it + 1 >= (int)scal[S_MAXIT]) scal[S_DONE] = 1.0;
      break;
    case OP_BETA: {
      double beta = s / scal[S_RZ];
      scal[S_BETA] = beta;
      scal[S_RZ] = s;
      hist[2 * (it - 1) + 1] = beta;
      break;
    }
    case OP_RZN:     // z.r of the new residual (flexible CG)
      scal[S_RZN] = s;
      break;
    case OP_BETAF: {  // s = z.q: beta = z^T (r_new - r_old) / z_old^T r_old = -alpha z.q / rz_old
      double beta = -scal[S_ALPHA] * s / scal[S_RZ];
      scal[S_BETA] = beta;
      scal[S_RZ] = scal[S_RZN];
      hist[2 * (it - 1) + 1] = beta;
      break;
    }
  }
}

}  // namespace

namespace gnk {

int scal_count() { return S_N; }

void dot_partial(int64_t n, const double* a, const double* b, double* part, const double* done,
                 hipStream_t s) {
  GnProfScope prof(PROF_VEC, 16.0 * n, s);
  hipLaunchKernelGGL(k_dot, dim3(RBLK), dim3(RTHR), 0, s, n, a, b, part, done);
  GN_CHECK_LAUNCH();
}
void finalize(const double* part, int nb, int op, double* scal, double* hist, double rtol,
              hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, part, nb, op, scal, hist, rtol);
  GN_CHECK_LAUNCH();
}
void update_xr(int64_t n, double* x, double* r, const double* p, const double* q, const double* scal,
               double* part, hipStream_t s) {
  GnProfScope prof(PROF_VEC, 48.0 * n, s);
  hipLaunchKernelGGL(k_update_xr, dim3(RBLK), dim3(RTHR), 0, s, n, x, r, p, q, scal, part);
  GN_CHECK_LAUNCH();
}
void update_p(int64_t n, double* p, const double* z, const double* scal, hipStream_t s) {
  GnProfScope prof(PROF_VEC, 24.0 * n, s);
  hipLaunchKernelGGL(k_update_p, dim3(RBLK), dim3(RTHR), 0, s, n, p, z, scal);
  GN_CHECK_LAUNCH();
}
void residual_partial(int64_t n, const double* b, const double* q, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_resid, dim3(RBLK), dim3(RTHR), 0, s, n, b, q, part);
  GN_CHECK_LAUNCH();
}
void sub_partial(int64_t n, const double* b, const double* q, double* r, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(RBLK), dim3(RTHR), 0, s, n, b, q, r, part);
  GN_CHECK_LAUNCH();
}
unsigned count_nonfinite(int64_t n, int ncol, int64_t ld, const double* x, unsigned* d_count, hipStream_t s) {
  unsigned h = 0;
  GN_HIP(hipMemsetAsync(d_count, 0, sizeof(unsigned), s));
  hipLaunchKernelGGL(k_count_nonfinite, dim3(RBLK), dim3(RTHR), 0, s, n, ncol, ld, x, d_count);
  GN_CHECK_LAUNCH();
  GN_HIP(hipMemcpyAsync(&h, d_count, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  GN_HIP(hipStreamSynchronize(s));
  return h;
}

void copy(int64_t n, double* dst, const double* src, const double* done, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(RBLK), dim3(RTHR), 0, s, n, dst, src, done);
  GN_CHECK_LAUNCH();
}

}  // namespace gnk
