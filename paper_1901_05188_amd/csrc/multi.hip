// Multi-right-hand-side PCG kernels: up to MC_K columns of one operator share
// every launch (Section 3.1: the CG iteration and M^-1_{AS,2}, applied to
// several load cases at once).  Each column keeps its own alpha, beta, residual
// and stopping flag; the operator, the local factors, Phi and the coarse factor
// are read once per launch for all columns.
//
// Layouts (full numbering as everywhere else: Dirichlet DOFs hold 0):
//   global vectors   column c at base + c * n_dof
//   local vectors    subdomain j, row r, column c at tm[(offVI_j + r) * MC_K + c]
//   coarse vectors   column c at g[c * NHP + i], NHP = NBH * TILE
//   CG scalars       column c at scal[c * S_N + ...], alpha/beta history at
//                    hist[c * hstride + ...], partial sums at part[c * pstride + ...]
//
// k_band_solve_mc: the banded forward/backward sweeps of all subdomains for
// MC_K columns on FP64 MFMA (v_mfma_f64_16x16x4f64).  One 512-thread workgroup
// per subdomain: wave (rh, kg) owns the 16 rows rh*16.. of the 32-row block row
// and the off-diagonal tiles t = kg, kg + 4, ...; the solved block rows of the
// current window live in an LDS ring of w + 1 block rows, and the next block
// row's tiles are loaded into registers while the current one is reduced.
#include "gn_internal.h"

namespace {

constexpr int MC_K = 16;    // column slots of one batch
constexpr int RBLK = 512;   // blocks of the fixed-shape vector reductions
constexpr int RTHR = 256;

typedef double gn_d4 __attribute__((ext_vector_type(4)));

__device__ inline void mc_lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ inline bool col_live(const double* scal, int c) { return scal[c * S_N + S_DONE] == 0.0; }

__device__ inline bool all_done(const double* scal, int k) {
  if (!scal) return false;
  for (int c = 0; c < k; ++c)
    if (scal[c * S_N + S_DONE] == 0.0) return false;
  return true;
}

// ---------------------------------------------------------------------------
// y_c = A x_c for the columns of one group of 4, fused partial p_c . q_c
// ---------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(256) void k_spmv_mc(int NX, int NY, int NZ, const double* __restrict__ A,
                                                 const double* __restrict__ x, double* __restrict__ y,
                                                 int64_t n_dof, int k, double* __restrict__ part, int pstride,
                                                 const double* __restrict__ scal) {
  constexpr int CB = 4;
  __shared__ double sh[16];
  const int c0 = blockIdx.y * CB;
  bool live[CB];
  bool any = false;
#pragma unroll
  for (int q = 0; q < CB; ++q) {
    live[q] = (c0 + q < k) && (!scal || col_live(scal, c0 + q));
    any |= live[q];
  }
  if (!any) return;
  const int64_t n_node = (int64_t)NX * NY * NZ;
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[CB][NC];
#pragma unroll
  for (int q = 0; q < CB; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[q][c] = 0.0;
  if (node < n_node) {
    int i = (int)(node % NX), j = (int)((node / NX) % NY), kk = (int)(node / ((int64_t)NX * NY));
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
      if (kk + dz < 0 || kk + dz >= NZ) continue;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        if (j + dy < 0 || j + dy >= NY) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (i + dx < 0 || i + dx >= NX) continue;
          const int d = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
          const int64_t nb = node + dx + (int64_t)NX * (dy + (int64_t)NY * dz);
          double a[NC][NC];
#pragma unroll
          for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int c2 = 0; c2 < NC; ++c2) a[c][c2] = A[((int64_t)(d * NC + c) * NC + c2) * n_node + node];
#pragma unroll
          for (int q = 0; q < CB; ++q) {
            if (!live[q]) continue;
            const double* xc = x + (int64_t)(c0 + q) * n_dof;
#pragma unroll
            for (int c2 = 0; c2 < NC; ++c2) {
              double xv = xc[nb * NC + c2];
#pragma unroll
              for (int c = 0; c < NC; ++c) acc[q][c] += a[c][c2] * xv;
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < CB; ++q) {
    if (!live[q]) continue;
    double dotv = 0.0;
    if (node < n_node) {
      const double* xc = x + (int64_t)(c0 + q) * n_dof;
      double* yc = y + (int64_t)(c0 + q) * n_dof;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        yc[node * NC + c] = acc[q][c];
        dotv += acc[q][c] * xc[node * NC + c];
      }
    }
    if (part) {
      double s = block_sum(dotv, sh);
      if (threadIdx.x == 0) part[(int64_t)(c0 + q) * pstride + blockIdx.x] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// per-column vector kernels: blockIdx.y is the column
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RTHR) void k_dot_mc(int64_t n, const double* __restrict__ a,
                                                 const double* __restrict__ b, double* __restrict__ part,
                                                 int pstride, const double* __restrict__ scal) {
  __shared__ double sh[16];
  const int c = blockIdx.y;
  if (scal && !col_live(scal, c)) return;
  const double* ac = a + (int64_t)c * n;
  const double* bc = b + (int64_t)c * n;
  double v = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    v += ac[t] * bc[t];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[(int64_t)c * pstride + blockIdx.x] = v;
}

__global__ __launch_bounds__(RTHR) void k_update_xr_mc(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                       const double* __restrict__ p, const double* __restrict__ q,
                                                       const double* __restrict__ scal, double* __restrict__ part,
                                                       int pstride) {
  __shared__ double sh[16];
  const int c = blockIdx.y;
  if (!col_live(scal, c)) return;
  const double alpha = scal[c * S_N + S_ALPHA];
  const int64_t o = (int64_t)c * n;
  double v = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    x[o + t] += alpha * p[o + t];
    double rv = r[o + t] - alpha * q[o + t];
    r[o + t] = rv;
    v += rv * rv;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[(int64_t)c * pstride + blockIdx.x] = v;
}

__global__ __launch_bounds__(RTHR) void k_update_p_mc(int64_t n, double* __restrict__ p, const double* __restrict__ z,
                                                      const double* __restrict__ scal) {
  const int c = blockIdx.y;
  if (!col_live(scal, c)) return;
  const double beta = scal[c * S_N + S_BETA];
  const int64_t o = (int64_t)c * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    p[o + t] = z[o + t] + beta * p[o + t];
}

__global__ __launch_bounds__(RTHR) void k_copy_mc(int64_t n, double* __restrict__ dst, const double* __restrict__ src,
                                                  const double* __restrict__ scal) {
  const int c = blockIdx.y;
  if (scal && !col_live(scal, c)) return;
  const int64_t o = (int64_t)c * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dst[o + t] = src[o + t];
}

// r_c = b_c - q_c with the partial r.r (restart from the true residual); with
// r == nullptr only the partial ||b - q||^2
__global__ __launch_bounds__(RTHR) void k_sub_mc(int64_t n, const double* __restrict__ b, const double* __restrict__ q,
                                                 double* __restrict__ r, double* __restrict__ part, int pstride,
                                                 const double* __restrict__ scal) {
  __shared__ double sh[16];
  const int c = blockIdx.y;
  if (scal && !col_live(scal, c)) return;
  const int64_t o = (int64_t)c * n;
  double v = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double d = b[o + t] - q[o + t];
    if (r) r[o + t] = d;
    v += d * d;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[(int64_t)c * pstride + blockIdx.x] = v;
}

// one block per column: fixed-order sum of the partials, then the recurrence of
// that column (same steps as the single-column finalize).  Only live columns
// take a step: a column is started (OP_BB) or restarted (OP_RESTART) by
// clearing its done flag while the others are held with theirs set.
__global__ void k_finalize_mc(const double* __restrict__ part, int pstride, int nb, int op,
                              double* __restrict__ scal_all, double* __restrict__ hist_all, int hstride,
                              double rtol) {
  __shared__ double sh[16];
  const int c = blockIdx.x;
  double* scal = scal_all + c * S_N;
  double* hist = hist_all + (int64_t)c * hstride;
  if (scal[S_DONE] != 0.0) return;
  const double* pc = part + (int64_t)c * pstride;
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += pc[i];
  double s = block_sum(v, sh);
  if (threadIdx.x != 0) return;
  if (op == OP_BB) {
    const double rt = scal[S_RTOL] > 0.0 ? scal[S_RTOL] : rtol;
    scal[S_BB] = s;
    scal[S_RR] = s;
    scal[S_TOL2] = rt * rt * s;
    scal[S_DONE] = (s == 0.0) ? 1.0 : 0.0;
    scal[S_ITER] = 0.0;
    scal[S_BREAK] = 0.0;
    return;
  }
  if (op == OP_RESTART) {
    scal[S_RR] = s;
    scal[S_DONE] = (s <= scal[S_TOL2] || (int)scal[S_ITER] >= (int)scal[S_MAXIT]) ? 1.0 : 0.0;
    return;
  }
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
  }
}

// ---------------------------------------------------------------------------
// restriction: t_j = R_j r_c for all columns (row-major, MC_K wide, zero in
// padding rows and unused columns) and g_c = Phi_j^T t_j  (Section 3.3.3)
// ---------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(256) void k_gather_mc(const SubDesc* __restrict__ subs, int NX, int NY,
                                                   const double* __restrict__ r, int64_t n_dof, int k,
                                                   double* __restrict__ tm, const double* __restrict__ Phi,
                                                   double* __restrict__ g, int NHP,
                                                   const double* __restrict__ scal) {
  constexpr int RC = 64;                     // rows per staged chunk
  __shared__ double sR[RC][MC_K + 1];
  __shared__ double sP[RC * 64];             // Phi rows of the chunk (m <= 64)
  if (all_done(scal, k)) return;
  const SubDesc& sd = subs[blockIdx.x];
  const int npad = sd.NBI * TILE;
  const int m = (Phi && g) ? sd.m : 0;
  double acc[4] = {0, 0, 0, 0};              // outputs o = threadIdx.x + 256 u: q = o / MC_K, c = o % MC_K
  double* tj = tm + sd.offVI * MC_K;
  const double* ph = Phi ? Phi + sd.offPhi : nullptr;
  for (int r0 = 0; r0 < npad; r0 += RC) {
    // read column-wise (consecutive lanes take consecutive local rows of one
    // column: runs of contiguous global DOFs), write row-wise through LDS
    for (int e = threadIdx.x; e < RC * MC_K; e += 256) {
      const int c = e / RC, rr = e % RC, row = r0 + rr;
      double v = 0.0;
      if (row < sd.nI && c < k) {
        int gn[3];
        box_global_node(sd.ilo, sd.in_, sd.permI, row / NC, gn);
        int64_t node = gn[0] + (int64_t)NX * (gn[1] + (int64_t)NY * gn[2]);
        v = r[(int64_t)c * n_dof + node * NC + row % NC];
      }
      sR[rr][c] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < RC * MC_K; e += 256) {
      const int rr = e / MC_K, c = e % MC_K, row = r0 + rr;
      if (row < npad) tj[(int64_t)row * MC_K + c] = sR[rr][c];
    }
    if (m > 0) {
      for (int e = threadIdx.x; e < RC * m; e += 256) {
        const int row = r0 + e / m;
        sP[e] = row < sd.nI ? ph[(int64_t)r0 * m + e] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = threadIdx.x + 256 * u;
        const int q = o / MC_K, c = o % MC_K;
        if (q < m) {
          double s = 0.0;
          for (int rr = 0; rr < RC; ++rr) s += sP[rr * m + q] * sR[rr][c];
          acc[u] += s;
        }
      }
    }
    __syncthreads();
  }
  if (m > 0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = threadIdx.x + 256 * u;
      const int q = o / MC_K, c = o % MC_K;
      if (q < m && c < k) g[(int64_t)c * NHP + sd.coff + q] = acc[u];
    }
  }
}

// ---------------------------------------------------------------------------
// banded forward/backward solves, MC_K columns, MFMA
// ---------------------------------------------------------------------------
template <typename FT>
__device__ inline double to_d(FT v) { return (double)v; }

template <typename FT, int SPW>
__global__ __launch_bounds__(512) void k_band_solve_mc(const SubDesc* __restrict__ subs, const FT* __restrict__ T,
                                                       const FT* __restrict__ D, const FT* __restrict__ TBk,
                                                       double* __restrict__ tm,
                                                       const FT* __restrict__ Z0, int k,
                                                       const double* __restrict__ scal) {
  extern __shared__ double ring[];           // (w + 1) block rows of TILE x MC_K
  __shared__ double red[4][TILE][MC_K];
  __shared__ double sS[TILE][MC_K];
  if (all_done(scal, k)) return;
  const SubDesc& sd = subs[blockIdx.x];
  const int NB = sd.NBI, w = sd.wI, W1 = w + 1;
  const FT* Tb = T + sd.offTI * TILE2;
  const FT* Db = D + sd.offDI * TILE2;
  double* tj = tm + sd.offVI * MC_K;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rh = wid & 1, kg = wid >> 1;
  const int lr = lane & 15, lk = lane >> 4;
  const int rb = rh * 16;
  const bool lead = kg == 0;                 // waves 0 and 1 finish each block row
  for (int e = threadIdx.x; e < W1 * TILE * MC_K; e += 512) ring[e] = 0.0;
  FT av[SPW][8];
  double dv[8], vv[4];
  gn_d4 acc[4];
#define MC_ZERO4() _Pragma("unroll") for (int u = 0; u < 4; ++u) acc[u] = gn_d4{0, 0, 0, 0};
  // forward tile of slot s at block row K: (K, t), t = kg + 4 s (the zero tile
  // if t >= w, or if the tile lies before the first block row: its stored
  // zeros are then not fetched)
#define MC_LOAD_FWD(K_)                                                                         \
  {                                                                                             \
    const int KK = (K_);                                                                        \
    _Pragma("unroll") for (int s = 0; s < SPW; ++s) {                                           \
      const int t = kg + 4 * s;                                                                 \
      const FT* tile = (t < w && KK - w + t >= 0) ? Tb + ((int64_t)KK * W1 + t) * TILE2 : Z0;   \
      _Pragma("unroll") for (int ks = 0; ks < 8; ++ks) av[s][ks] = tile[(4 * ks + lk) * TILE + rb + lr]; \
    }                                                                                           \
  }
#define MC_LOAD_DV_FWD(K_)                                                                      \
  {                                                                                             \
    const int KK = (K_);                                                                        \
    if (lead) {                                                                                 \
      const FT* dk = Db + (int64_t)KK * TILE2;                                                  \
      _Pragma("unroll") for (int ks = 0; ks < 8; ++ks) dv[ks] = to_d(dk[(4 * ks + lk) * TILE + rb + lr]); \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) vv[i] = tj[(int64_t)(KK * TILE + rb + 4 * i + lk) * MC_K + lr]; \
    }                                                                                           \
  }
  MC_LOAD_FWD(0)
  __syncthreads();
  for (int K = 0; K < NB; ++K) {
    // the diagonal tile and right-hand side of row K are loaded here and used in
    // its exchange, without a copy before a reload (a copy of registers still
    // being loaded makes the wave wait for every load in flight)
    if (lead) MC_LOAD_DV_FWD(K)
    MC_ZERO4()
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      const int t = kg + 4 * s;
      const int slot = (K - w + t + W1) % W1;
      const double* yb = ring + slot * TILE * MC_K;
#pragma unroll
      for (int ks = 0; ks < 8; ++ks)
        acc[ks & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(to_d(av[s][ks]), yb[(4 * ks + lk) * MC_K + lr],
                                                           acc[ks & 3], 0, 0, 0);
    }
    MC_LOAD_FWD(min(K + 1, NB - 1))
#pragma unroll
    for (int i = 0; i < 4; ++i)
      red[kg][rb + 4 * i + lk][lr] = (acc[0][i] + acc[1][i]) + (acc[2][i] + acc[3][i]);
    mc_lds_barrier();
    if (lead) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rb + 4 * i + lk;
        sS[row][lr] = vv[i] - ((red[0][row][lr] + red[1][row][lr]) + (red[2][row][lr] + red[3][row][lr]));
      }
    }
    mc_lds_barrier();
    if (lead) {
      MC_ZERO4()
#pragma unroll
      for (int ks = 0; ks < 8; ++ks)
        acc[ks & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(dv[ks], sS[4 * ks + lk][lr], acc[ks & 3], 0, 0, 0);
      double* yb = ring + (K % W1) * TILE * MC_K;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rb + 4 * i + lk;
        const double y = (acc[0][i] + acc[1][i]) + (acc[2][i] + acc[3][i]);
        yb[row * MC_K + lr] = y;
        tj[(int64_t)(K * TILE + row) * MC_K + lr] = y;
      }
    }
    mc_lds_barrier();
  }
#undef MC_LOAD_FWD
#undef MC_LOAD_DV_FWD
  for (int e = threadIdx.x; e < W1 * TILE * MC_K; e += 512) ring[e] = 0.0;
  // backward tile of slot s at block row K: L(K + d, K)^T, d = 1 + kg + 4 s,
  // tile d - 1 of row K of the transposed band (zero past the last block row),
  // and D_K^T in its tile w: the same contiguous lane pattern as the forward
  const FT* TBb = TBk + sd.offTI * TILE2;
#define MC_LOAD_BWD(K_)                                                                         \
  {                                                                                             \
    const int KK = (K_);                                                                        \
    _Pragma("unroll") for (int s = 0; s < SPW; ++s) {                                           \
      const int d = 1 + kg + 4 * s;                                                             \
      const FT* tile = (d <= w && KK + d < NB) ? TBb + ((int64_t)KK * W1 + (d - 1)) * TILE2 : Z0; \
      _Pragma("unroll") for (int ks = 0; ks < 8; ++ks) av[s][ks] = tile[(4 * ks + lk) * TILE + rb + lr]; \
    }                                                                                           \
  }
#define MC_LOAD_DV_BWD(K_)                                                                      \
  {                                                                                             \
    const int KK = (K_);                                                                        \
    if (lead) {                                                                                 \
      const FT* dk = TBb + ((int64_t)KK * W1 + w) * TILE2;                                      \
      _Pragma("unroll") for (int ks = 0; ks < 8; ++ks) dv[ks] = to_d(dk[(4 * ks + lk) * TILE + rb + lr]); \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) vv[i] = tj[(int64_t)(KK * TILE + rb + 4 * i + lk) * MC_K + lr]; \
    }                                                                                           \
  }
  MC_LOAD_BWD(NB - 1)
  __syncthreads();
  for (int K = NB - 1; K >= 0; --K) {
    if (lead) MC_LOAD_DV_BWD(K)
    MC_ZERO4()
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      const int d = 1 + kg + 4 * s;
      const int slot = (K + d) % W1;
      const bool inb = (d <= w) && (K + d < NB);
      const double* xb = ring + slot * TILE * MC_K;
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        const double bval = inb ? xb[(4 * ks + lk) * MC_K + lr] : 0.0;
        acc[ks & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(to_d(av[s][ks]), bval, acc[ks & 3], 0, 0, 0);
      }
    }
    MC_LOAD_BWD(max(K - 1, 0))
#pragma unroll
    for (int i = 0; i < 4; ++i)
      red[kg][rb + 4 * i + lk][lr] = (acc[0][i] + acc[1][i]) + (acc[2][i] + acc[3][i]);
    mc_lds_barrier();
    if (lead) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rb + 4 * i + lk;
        sS[row][lr] = vv[i] - ((red[0][row][lr] + red[1][row][lr]) + (red[2][row][lr] + red[3][row][lr]));
      }
    }
    mc_lds_barrier();
    if (lead) {
      MC_ZERO4()
#pragma unroll
      for (int ks = 0; ks < 8; ++ks)
        acc[ks & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(dv[ks], sS[4 * ks + lk][lr], acc[ks & 3], 0, 0, 0);
      double* xb = ring + (K % W1) * TILE * MC_K;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rb + 4 * i + lk;
        const double x = (acc[0][i] + acc[1][i]) + (acc[2][i] + acc[3][i]);
        xb[row * MC_K + lr] = x;
        tj[(int64_t)(K * TILE + row) * MC_K + lr] = x;
      }
    }
    mc_lds_barrier();
  }
#undef MC_LOAD_BWD
#undef MC_LOAD_DV_BWD
#undef MC_ZERO4
}

// ---------------------------------------------------------------------------
// coarse solve y_c = Z^T (Z g_c), Z = L_H^-1 in dense tiles; thread (i, c)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE * MC_K) void k_coarse_fwd_mc(int NBH, const double* __restrict__ Z,
                                                               const double* __restrict__ g, double* __restrict__ u,
                                                               int k, const double* __restrict__ scal) {
  if (all_done(scal, k)) return;
  const int K = blockIdx.x, i = threadIdx.x % TILE, c = threadIdx.x / TILE;
  if (c >= k) return;
  const int NHP = NBH * TILE;
  const double* gc = g + (int64_t)c * NHP;
  double acc = 0.0;
  for (int J = 0; J <= K; ++J) {
    const double* tile = Z + ((int64_t)K * NBH + J) * TILE2;
#pragma unroll 8
    for (int cc = 0; cc < TILE; ++cc) acc += tile[cc * TILE + i] * gc[J * TILE + cc];
  }
  u[(int64_t)c * NHP + K * TILE + i] = acc;
}

__global__ __launch_bounds__(TILE * MC_K) void k_coarse_bwd_mc(int NBH, const double* __restrict__ Z,
                                                               const double* __restrict__ u, double* __restrict__ y,
                                                               int k, const double* __restrict__ scal) {
  if (all_done(scal, k)) return;
  const int J = blockIdx.x, cc = threadIdx.x % TILE, c = threadIdx.x / TILE;
  if (c >= k) return;
  const int NHP = NBH * TILE;
  const double* uc = u + (int64_t)c * NHP;
  double acc = 0.0;
  for (int K = J; K < NBH; ++K) {
    const double* tile = Z + ((int64_t)K * NBH + J) * TILE2;
#pragma unroll 8
    for (int i = 0; i < TILE; ++i) acc += tile[cc * TILE + i] * uc[K * TILE + i];
  }
  y[(int64_t)c * NHP + J * TILE + cc] = acc;
}

// ---------------------------------------------------------------------------
// gather-form prolongation z_c = sum_j R_j^T (t_j + Phi_j y_j), fused r_c . z_c
// ---------------------------------------------------------------------------
struct McAxes {
  const int* cnt0; const int* cnt1; const int* cnt2;
  const int* plo0; const int* plo1; const int* plo2;
};

// t_j(row, q) += sum_e Phi_j(row, e) y(coff_j + e, q) for the MC_K columns, a
// thread per I-box row, streamed over Phi ahead of the gather
__global__ __launch_bounds__(256) void k_phi_add_mc(const SubDesc* __restrict__ subs, const double* __restrict__ Phi,
                                                    const double* __restrict__ y, int NHP, double* __restrict__ tm,
                                                    int k, const double* __restrict__ scal) {
  if (all_done(scal, k)) return;
  const SubDesc& sd = subs[blockIdx.y];
  const int row = blockIdx.x * 256 + threadIdx.x;
  const int m = sd.m;
  if (m == 0 || row >= sd.nI) return;
  const double* ph = Phi + sd.offPhi + (int64_t)row * m;
  const double* yy = y + sd.coff;
  double* tv = tm + (sd.offVI + row) * MC_K;
  double a[MC_K];
#pragma unroll
  for (int q = 0; q < MC_K; ++q) a[q] = tv[q];
  for (int e = 0; e < m; ++e) {
    const double pv = ph[e];
#pragma unroll
    for (int q = 0; q < MC_K; ++q) a[q] += pv * yy[e + (int64_t)q * NHP];
  }
#pragma unroll
  for (int q = 0; q < MC_K; ++q) tv[q] = a[q];
}

template <int NC>
__global__ __launch_bounds__(256) void k_prolong_mc(const SubDesc* __restrict__ subs, int NX, int NY, int NZ,
                                                    int P0, int P1, McAxes pa, const uint8_t* __restrict__ dir,
                                                    const double* __restrict__ tm, const double* __restrict__ Phi,
                                                    const double* __restrict__ y, int NHP,
                                                    const double* __restrict__ r, double* __restrict__ z,
                                                    int64_t n_dof, int k, double* __restrict__ part, int pstride,
                                                    const double* __restrict__ scal) {
  __shared__ double sh[16];
  if (all_done(scal, k)) return;
  const int64_t n_node = (int64_t)NX * NY * NZ;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[NC][MC_K];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int q = 0; q < MC_K; ++q) acc[c][q] = 0.0;
  if (node < n_node) {
    const int gi = (int)(node % NX), gj = (int)((node / NX) % NY), gk = (int)(node / ((int64_t)NX * NY));
    const int c0 = pa.cnt0[gi], c1 = pa.cnt1[gj], c2 = pa.cnt2[gk];
    const int p0 = pa.plo0[gi], p1 = pa.plo1[gj], p2 = pa.plo2[gk];
    for (int b2 = 0; b2 < c2; ++b2)
      for (int b1 = 0; b1 < c1; ++b1)
        for (int b0 = 0; b0 < c0; ++b0) {
          const int j = (p0 + b0) + P0 * ((p1 + b1) + P1 * (p2 + b2));
          const SubDesc& sd = subs[j];
          const int ln = box_local_node(sd.ilo, sd.in_, sd.permI, gi, gj, gk);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const int64_t row = (int64_t)ln * NC + c;
            const double* tv = tm + (sd.offVI + row) * MC_K;
#pragma unroll
            for (int q = 0; q < MC_K; ++q) acc[c][q] += tv[q];
            if (Phi && sd.m > 0) {
              const double* ph = Phi + sd.offPhi + row * sd.m;
              for (int e = 0; e < sd.m; ++e) {
                const double pv = ph[e];
                const double* yy = y + sd.coff + e;
#pragma unroll
                for (int q = 0; q < MC_K; ++q) acc[c][q] += pv * yy[(int64_t)q * NHP];
              }
            }
          }
        }
  }
  for (int q = 0; q < k; ++q) {
    if (scal && !col_live(scal, q)) continue;    // uniform over the block
    double dotv = 0.0;
    if (node < n_node) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double v = 0.0;
#pragma unroll
        for (int qq = 0; qq < MC_K; ++qq)
          if (qq == q) v = acc[c][qq];
        v = dir[node * NC + c] ? 0.0 : v;
        z[(int64_t)q * n_dof + node * NC + c] = v;
        if (r) dotv += v * r[(int64_t)q * n_dof + node * NC + c];
      }
    }
    if (part) {
      double s = block_sum(dotv, sh);
      if (threadIdx.x == 0) part[(int64_t)q * pstride + blockIdx.x] = s;
    }
  }
}

}  // namespace

namespace gnk {

int mc_width() { return MC_K; }

void spmv_mc(const gn_problem* p, const double* x, double* y, int k, double* part, int pstride,
             const double* scal, hipStream_t s) {
  dim3 grid((unsigned)((p->n_node + 255) / 256), (unsigned)((k + 3) / 4));
  GnProfScope prof(PROF_SPMV, (double)p->n_node * (27.0 * p->nc * p->nc * 8.0 + 2.0 * k * p->nc * 8.0), s);
  if (p->nc == 3)
    hipLaunchKernelGGL(k_spmv_mc<3>, grid, dim3(256), 0, s, p->nn[0], p->nn[1], p->nn[2], p->d_A, x, y,
                       p->n_dof, k, part, pstride, scal);
  else
    hipLaunchKernelGGL(k_spmv_mc<1>, grid, dim3(256), 0, s, p->nn[0], p->nn[1], p->nn[2], p->d_A, x, y,
                       p->n_dof, k, part, pstride, scal);
  GN_CHECK_LAUNCH();
}

void dot_mc(int64_t n, int k, const double* a, const double* b, double* part, int pstride, const double* scal,
            hipStream_t s) {
  GnProfScope prof(PROF_VEC, 16.0 * n * k, s);
  hipLaunchKernelGGL(k_dot_mc, dim3(RBLK, k), dim3(RTHR), 0, s, n, a, b, part, pstride, scal);
  GN_CHECK_LAUNCH();
}

void update_xr_mc(int64_t n, int k, double* x, double* r, const double* p, const double* q, const double* scal,
                  double* part, int pstride, hipStream_t s) {
  GnProfScope prof(PROF_VEC, 48.0 * n * k, s);
  hipLaunchKernelGGL(k_update_xr_mc, dim3(RBLK, k), dim3(RTHR), 0, s, n, x, r, p, q, scal, part, pstride);
  GN_CHECK_LAUNCH();
}

void update_p_mc(int64_t n, int k, double* p, const double* z, const double* scal, hipStream_t s) {
  GnProfScope prof(PROF_VEC, 24.0 * n * k, s);
  hipLaunchKernelGGL(k_update_p_mc, dim3(RBLK, k), dim3(RTHR), 0, s, n, p, z, scal);
  GN_CHECK_LAUNCH();
}

void copy_mc(int64_t n, int k, double* dst, const double* src, const double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_mc, dim3(RBLK, k), dim3(RTHR), 0, s, n, dst, src, scal);
  GN_CHECK_LAUNCH();
}

void sub_mc(int64_t n, int k, const double* b, const double* q, double* r, double* part, int pstride,
            const double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_mc, dim3(RBLK, k), dim3(RTHR), 0, s, n, b, q, r, part, pstride, scal);
  GN_CHECK_LAUNCH();
}

void finalize_mc(const double* part, int pstride, int nb, int op, int k, double* scal, double* hist,
                 int hstride, double rtol, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_mc, dim3(k), dim3(256), 0, s, part, pstride, nb, op, scal, hist, hstride, rtol);
  GN_CHECK_LAUNCH();
}

int mc_band_lds_bytes(int maxw) { return (maxw + 1) * TILE * MC_K * (int)sizeof(double); }

void precond_mc(const gn_problem* p, const gn_precond* pc, const double* r, double* z, int k, double* part,
                int pstride, const double* scal, double* tm, double* gm, double* um, double* ym, hipStream_t s) {
  if (k < 1 || k > MC_K) throw gn_error{GN_ERR_ARG, "multi-RHS batch must hold 1..16 columns"};
  if (!pc->d_LIb) throw gn_error{GN_ERR_ARG, "backward band missing"};
  const bool f32 = pc->local_prec == 32;
  const double* Phi = pc->NH > 0 ? pc->d_Phi : nullptr;
  const int NHP = pc->NBH * TILE;
  {
    GnProfScope prof(PROF_TRSV, pc->trsv_bytes_mc, s);
    if (p->nc == 3)
      hipLaunchKernelGGL(k_gather_mc<3>, dim3(pc->n_sub), dim3(256), 0, s, pc->d_sub, p->nn[0], p->nn[1], r,
                         p->n_dof, k, tm, Phi, gm, NHP, scal);
    else
      hipLaunchKernelGGL(k_gather_mc<1>, dim3(pc->n_sub), dim3(256), 0, s, pc->d_sub, p->nn[0], p->nn[1], r,
                         p->n_dof, k, tm, Phi, gm, NHP, scal);
    GN_CHECK_LAUNCH();
    const int lds = mc_band_lds_bytes(pc->maxwI);
    const int spw = (pc->maxwI + 3) / 4;
#define GN_MC(FT, S)                                                                                   \
  do {                                                                                                 \
    auto kfn = k_band_solve_mc<FT, S>;                                                                 \
    GN_HIP(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, lds));     \
    hipLaunchKernelGGL(kfn, dim3(pc->n_sub), dim3(512), lds, s, pc->d_subxI,                           \
                       (const FT*)(f32 ? (const void*)pc->d_LIf : (const void*)pc->d_LI),              \
                       (const FT*)(f32 ? (const void*)pc->d_DIf : (const void*)pc->d_DI),              \
                       (const FT*)pc->d_LIb, tm,                                                       \
                       (const FT*)(f32 ? (const void*)pc->d_zf : (const void*)pc->d_z0), k, scal);     \
  } while (0)
#define GN_MC_S(FT)                            \
  do {                                         \
    if (spw <= 1) GN_MC(FT, 1);                \
    else if (spw <= 2) GN_MC(FT, 2);           \
    else if (spw <= 3) GN_MC(FT, 3);           \
    else if (spw <= 4) GN_MC(FT, 4);           \
    else if (spw <= 5) GN_MC(FT, 5);           \
    else if (spw <= 6) GN_MC(FT, 6);           \
    else if (spw <= 8) GN_MC(FT, 8);           \
    else throw gn_error{GN_ERR_ARG, "local band wider than 32 tiles"}; \
  } while (0)
    if (f32) GN_MC_S(float); else GN_MC_S(double);
#undef GN_MC_S
#undef GN_MC
    GN_CHECK_LAUNCH();
  }
  if (pc->NH > 0 && pc->coarse_solve == 1) {
    // inexact coarse solve: one inner CG per column (finished columns skip theirs)
    const int64_t NHc = (int64_t)pc->NBH * TILE;
    for (int c = 0; c < k; ++c)
      coarse_cg(pc, gm + c * NHc, ym + c * NHc, scal ? scal + c * S_N + S_DONE : nullptr, s);
  } else if (pc->NH > 0) {
    GnProfScope prof(PROF_COARSE, (double)pc->NBH * (pc->NBH + 1) * TILE2 * 8.0, s);
    hipLaunchKernelGGL(k_coarse_fwd_mc, dim3(pc->NBH), dim3(TILE * MC_K), 0, s, pc->NBH, pc->d_Z, gm, um, k, scal);
    GN_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_coarse_bwd_mc, dim3(pc->NBH), dim3(TILE * MC_K), 0, s, pc->NBH, pc->d_Z, um, ym, k, scal);
    GN_CHECK_LAUNCH();
  }
  {
    GnProfScope prof(PROF_PROLONG, pc->prolong_bytes, s);
    if (Phi) {
      hipLaunchKernelGGL(k_phi_add_mc, dim3((unsigned)((pc->maxNBI * TILE + 255) / 256), (unsigned)pc->n_sub),
                         dim3(256), 0, s, pc->d_sub, Phi, ym, NHP, tm, k, scal);
      GN_CHECK_LAUNCH();
    }
    McAxes pa{pc->d_cnt[0], pc->d_cnt[1], pc->d_cnt[2], pc->d_plo[0], pc->d_plo[1], pc->d_plo[2]};
    dim3 grid((unsigned)((p->n_node + 255) / 256));
    const double* nophi = nullptr;   // folded into the local vectors above
    if (p->nc == 3)
      hipLaunchKernelGGL(k_prolong_mc<3>, grid, dim3(256), 0, s, pc->d_sub, p->nn[0], p->nn[1], p->nn[2],
                         pc->nparts[0], pc->nparts[1], pa, p->d_dir, tm, nophi, ym, NHP, r, z, p->n_dof, k, part,
                         pstride, scal);
    else
      hipLaunchKernelGGL(k_prolong_mc<1>, grid, dim3(256), 0, s, pc->d_sub, p->nn[0], p->nn[1], p->nn[2],
                         pc->nparts[0], pc->nparts[1], pa, p->d_dir, tm, nophi, ym, NHP, r, z, p->n_dof, k, part,
                         pstride, scal);
    GN_CHECK_LAUNCH();
  }
}

}  // namespace gnk
