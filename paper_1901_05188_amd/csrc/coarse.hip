// Inexact coarse solve (Section 3.3.3, last paragraph: for a large coarse
// space the paper solves A_H iteratively instead of factoring it, which makes
// the preconditioner vary between applications, and switches the outer Krylov
// method to a flexible one).
//
// A_H is held block-sparse: one m_j1 x m_j2 block per pair of subdomains whose
// coarse functions interact (the local-product pairs of the assembly, made
// symmetric), no dense factor and no O(N_H^2) storage.  The coarse system is
// solved by conjugate gradients preconditioned with the inverses of the
// diagonal blocks (A_H)_jj, from y = 0, until ||g - A_H y|| <= rtol ||g|| or
// maxit iterations.
//
// k_coarse_cg runs the whole inner iteration in one cooperative launch: each
// workgroup owns block rows j = blockIdx.x, blockIdx.x + G, ...; the two
// reductions of an iteration (p.q, then r.z and r.r) pass through per-workgroup
// partial sums and a grid barrier, and every workgroup adds the G partials in
// the same order, so all take the same decisions (step sizes, stopping) and
// leave the loop together.  The search direction is double-buffered: block row
// j forms p_new = z + beta p_old for its own rows and, on the fly, for the
// neighbour rows its block product reads, while the owners of those rows
// write them to the other buffer.
#include <hip/hip_cooperative_groups.h>

#include "gn_internal.h"

namespace cgr = cooperative_groups;

namespace {

constexpr int CNT = 256;     // threads: four waves; lane = row of a block row (m_j <= 64)
constexpr int CMAXM = 64;

// sum of G partials in a fixed order (the first wave; lanes stride, then a
// shuffle tree); result in every thread of the workgroup
__device__ inline double grid_sum(const double* part, int G, double* sh) {
  double v = 0.0;
  if (threadIdx.x < 64) {
    for (int i = threadIdx.x; i < G; i += 64) v += part[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (threadIdx.x == 0) *sh = v;
  }
  __syncthreads();
  v = *sh;
  __syncthreads();
  return v;
}

// block sum of one value per thread (fixed order: lanes, then waves)
__device__ inline double wg_sum(double v, double* sh4) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(CNT) void k_coarse_cg(const SubDesc* __restrict__ subs, int n_sub,
                                                   const int* __restrict__ ptr, const BsrBlock* __restrict__ blk,
                                                   const double* __restrict__ val,
                                                   const int64_t* __restrict__ dinv_off,
                                                   const double* __restrict__ dinv, const double* __restrict__ g,
                                                   double* __restrict__ y, double* __restrict__ r,
                                                   double* __restrict__ z, double* __restrict__ pA,
                                                   double* __restrict__ pB, double* __restrict__ q,
                                                   double* __restrict__ part, double rtol, int maxit,
                                                   const double* __restrict__ done, double* __restrict__ stat) {
  __shared__ double sred[CNT / 64][CMAXM];
  __shared__ double srow[CMAXM];
  __shared__ double sh4[CNT / 64];
  __shared__ double sg;
  if (done && *done != 0.0) return;          // uniform: the outer solve has finished
  cgr::grid_group grid = cgr::this_grid();
  const int G = gridDim.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double* PQ = part;
  double* RZ = part + G;
  double* RR = part + 2 * G;
  // z_j = D_j^-1 r_j for block row j (r_j staged in LDS); returns r.z and r.r of the rows
  auto precond_row = [&](int j, double& rz, double& rr) {
    const SubDesc& sd = subs[j];
    const int m = sd.m, c0 = sd.coff;
    if (threadIdx.x < m) srow[threadIdx.x] = r[c0 + threadIdx.x];
    __syncthreads();
    if (threadIdx.x < m) {
      const double* D = dinv + dinv_off[j] + (int64_t)threadIdx.x * m;
      double t = 0.0;
      for (int l = 0; l < m; ++l) t += D[l] * srow[l];
      z[c0 + threadIdx.x] = t;
      rz += srow[threadIdx.x] * t;
      rr += srow[threadIdx.x] * srow[threadIdx.x];
    }
    __syncthreads();
  };
  // ---- start: y = 0, r = g, z = D^-1 g, p_old = 0 -------------------------
  double rz_p = 0.0, gg_p = 0.0;
  for (int j = blockIdx.x; j < n_sub; j += G) {
    const SubDesc& sd = subs[j];
    if (threadIdx.x < sd.m) {
      const int i = sd.coff + threadIdx.x;
      r[i] = g[i];
      y[i] = 0.0;
      pA[i] = 0.0;
    }
    __syncthreads();
    precond_row(j, rz_p, gg_p);
  }
  double t = wg_sum(rz_p, sh4);
  double u = wg_sum(gg_p, sh4);
  if (threadIdx.x == 0) {
    RZ[blockIdx.x] = t;
    RR[blockIdx.x] = u;
  }
  grid.sync();
  double rz = grid_sum(RZ, G, &sg);
  const double gg = grid_sum(RR, G, &sg);
  const double tol2 = rtol * rtol * gg;
  double beta = 0.0;
  int it = 0;
  double* pold = pA;
  double* pnew = pB;
  if (gg > 0.0) {
    for (; it < maxit; ++it) {
      // ---- p_new = z + beta p_old, q = A_H p_new, partial p.q --------------
      double pq_p = 0.0;
      for (int j = blockIdx.x; j < n_sub; j += G) {
        const SubDesc& sd = subs[j];
        const int m = sd.m, c0 = sd.coff;
        double acc = 0.0;
        for (int b = ptr[j] + wv; b < ptr[j + 1]; b += CNT / 64) {
          const BsrBlock bk = blk[b];
          const int m2 = subs[bk.j2].m, c2 = subs[bk.j2].coff;
          if (lane < m) {
            const double* A = val + bk.off + (int64_t)lane * m2;
            for (int l = 0; l < m2; ++l) acc += A[l] * (z[c2 + l] + beta * pold[c2 + l]);
          }
        }
        if (lane < CMAXM) sred[wv][lane] = acc;
        __syncthreads();
        if (threadIdx.x < m) {
          const int i = c0 + threadIdx.x;
          const double qi = (sred[0][threadIdx.x] + sred[1][threadIdx.x]) + (sred[2][threadIdx.x] + sred[3][threadIdx.x]);
          const double pi = z[i] + beta * pold[i];
          pnew[i] = pi;
          q[i] = qi;
          pq_p += pi * qi;
        }
        __syncthreads();
      }
      t = wg_sum(pq_p, sh4);
      if (threadIdx.x == 0) PQ[blockIdx.x] = t;
      grid.sync();
      const double pq = grid_sum(PQ, G, &sg);
      if (!(pq > 0.0)) break;                // A_H not positive on p: stop with the current y
      const double alpha = rz / pq;
      // ---- y += alpha p, r -= alpha q, z = D^-1 r, partial r.z and r.r -------
      double rzn_p = 0.0, rr_p = 0.0;
      for (int j = blockIdx.x; j < n_sub; j += G) {
        const SubDesc& sd = subs[j];
        if (threadIdx.x < sd.m) {
          const int i = sd.coff + threadIdx.x;
          y[i] += alpha * pnew[i];
          r[i] -= alpha * q[i];
        }
        __syncthreads();
        precond_row(j, rzn_p, rr_p);
      }
      t = wg_sum(rzn_p, sh4);
      u = wg_sum(rr_p, sh4);
      if (threadIdx.x == 0) {
        RZ[blockIdx.x] = t;
        RR[blockIdx.x] = u;
      }
      grid.sync();
      const double rzn = grid_sum(RZ, G, &sg);
      const double rr = grid_sum(RR, G, &sg);
      beta = rzn / rz;
      rz = rzn;
      double* tmp = pold;
      pold = pnew;
      pnew = tmp;
      if (rr <= tol2) {
        ++it;
        break;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && stat) {
    stat[0] += (double)it;
    stat[1] += 1.0;
    stat[2] = fmax(stat[2], (double)it);
  }
}

// (A_H)_jj^-1 by Gauss-Jordan elimination in LDS (SPD: no pivoting), one
// workgroup per subdomain, thread t owns column t; symmetrised at the end.
// info[j] = k + 1 when pivot k is not positive.
__global__ __launch_bounds__(CMAXM) void k_block_inv(const SubDesc* __restrict__ subs, const int* __restrict__ ptr,
                                                     const BsrBlock* __restrict__ blk,
                                                     const double* __restrict__ val,
                                                     const int64_t* __restrict__ dinv_off, double* __restrict__ dinv,
                                                     int* __restrict__ info) {
  __shared__ double M[CMAXM][CMAXM + 1], X[CMAXM][CMAXM + 1];
  __shared__ double fac[CMAXM];
  __shared__ double piv;
  const int j = blockIdx.x;
  const int m = subs[j].m;
  if (m == 0) return;
  const int t = threadIdx.x;
  int64_t off = -1;
  for (int b = ptr[j]; b < ptr[j + 1]; ++b)
    if (blk[b].j2 == j) off = blk[b].off;
  if (t < m)
    for (int i = 0; i < m; ++i) {
      M[i][t] = off >= 0 ? val[off + (int64_t)i * m + t] : 0.0;
      X[i][t] = i == t ? 1.0 : 0.0;
    }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    if (t < m) fac[t] = M[t][k];
    if (t == 0) piv = M[k][k];
    __syncthreads();
    if (!(piv > 0.0)) {
      if (t == 0) info[j] = k + 1;
      return;                                  // uniform: every thread read the same pivot
    }
    if (t < m) {
      M[k][t] /= piv;
      X[k][t] /= piv;
    }
    __syncthreads();
    if (t < m)
      for (int i = 0; i < m; ++i)
        if (i != k) {
          M[i][t] -= fac[i] * M[k][t];
          X[i][t] -= fac[i] * X[k][t];
        }
    __syncthreads();
  }
  if (t < m)
    for (int i = 0; i < m; ++i) dinv[dinv_off[j] + (int64_t)i * m + t] = 0.5 * (X[i][t] + X[t][i]);
}

// blocks of the block-sparse A_H copied from the dense symmetrised assembly
// (tile (K, J) column-major at (K NBH + J) TILE2)
__global__ __launch_bounds__(256) void k_bsr_from_dense(const SubDesc* __restrict__ subs,
                                                        const BsrBlock* __restrict__ blk, int NBH,
                                                        const double* __restrict__ AH, double* __restrict__ val) {
  const BsrBlock bk = blk[blockIdx.x];
  const int m1 = subs[bk.j1].m, m2 = subs[bk.j2].m;
  const int r0 = subs[bk.j1].coff, c0 = subs[bk.j2].coff;
  for (int e = threadIdx.x; e < m1 * m2; e += blockDim.x) {
    const int row = r0 + e / m2, col = c0 + e % m2;
    val[bk.off + e] = AH[((int64_t)(row / TILE) * NBH + col / TILE) * TILE2 + (col % TILE) * TILE + row % TILE];
  }
}

}  // namespace

namespace gnk {

int coarse_cg_grid(const gn_precond* pc) {
  int dev = 0, ncu = 0, per_cu = 0;
  GN_HIP(hipGetDevice(&dev));
  GN_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  GN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_coarse_cg, CNT, 0));
  const int cap = std::max(1, ncu * std::max(per_cu, 1));
  return std::max(1, std::min(pc->n_sub, std::min(cap, ncu)));
}

void bsr_from_dense(const gn_precond* pc, const double* AH, hipStream_t s) {
  if (pc->bsr_nnz == 0) return;
  hipLaunchKernelGGL(k_bsr_from_dense, dim3((unsigned)pc->bsr_nnz), dim3(256), 0, s, pc->d_sub, pc->d_bsr_blk,
                     pc->NBH, AH, pc->d_bsr_val);
  GN_CHECK_LAUNCH();
}

void block_inverse(const gn_precond* pc, int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_block_inv, dim3((unsigned)pc->n_sub), dim3(CMAXM), 0, s, pc->d_sub, pc->d_bsr_ptr,
                     pc->d_bsr_blk, pc->d_bsr_val, pc->d_dinv_off, pc->d_dinv, info);
  GN_CHECK_LAUNCH();
}

void coarse_cg(const gn_precond* pc, const double* g, double* y, const double* done, hipStream_t s) {
  if (pc->NH == 0) return;
  const int64_t NHP = (int64_t)pc->NBH * TILE;
  double* r = pc->d_cvec;
  double* z = r + NHP;
  double* pA = z + NHP;
  double* pB = pA + NHP;
  double* q = pB + NHP;
  const SubDesc* subs = pc->d_sub;
  int n_sub = pc->n_sub;
  const int* ptr = pc->d_bsr_ptr;
  const BsrBlock* blk = pc->d_bsr_blk;
  const double* val = pc->d_bsr_val;
  const int64_t* doff = pc->d_dinv_off;
  const double* dinv = pc->d_dinv;
  double* part = pc->d_cpart;
  double rtol = pc->coarse_rtol;
  int maxit = pc->coarse_maxit;
  double* stat = pc->d_cstat;
  void* args[] = {(void*)&subs, (void*)&n_sub, (void*)&ptr, (void*)&blk, (void*)&val, (void*)&doff,
                  (void*)&dinv, (void*)&g, (void*)&y, (void*)&r, (void*)&z, (void*)&pA, (void*)&pB,
                  (void*)&q, (void*)&part, (void*)&rtol, (void*)&maxit, (void*)&done, (void*)&stat};
  GnProfScope prof(PROF_COARSE, (double)pc->bsr_nnz, s);
  GN_HIP(hipLaunchCooperativeKernel((const void*)k_coarse_cg, dim3((unsigned)pc->coarse_grid), dim3(CNT), args,
                                    0, s));
}

}  // namespace gnk
