// Application of the two-level additive Schwarz preconditioner
//   M^-1 r = sum_j R_j^T A_j^-1 R_j r + R_H^T A_H^-1 R_H r
// (Section 3.1, eqn:onelevelAS and M^-1_{AS,2}; Section 3.3.3 for the coarse
// restriction (R_H v)_i = Phi_i^T v and the prolongation R_H^T v_H).
//
// The local solves sum_j R_j^T A_j^-1 R_j r and the restriction Phi_j^T r are
//   k_local_solve_pf (local_solve.hip).
// k_coarse_units / k_coarse_rowsum: y = Z^T (Z g) with Z = L_H^-1 stored as
//   dense tiles (the coarse factor inverse; its transpose in the free upper
//   tiles), in balanced work units of at most 64 tiles of one tile row.
// k_phi_add: t_j += Phi_j y_j, streamed per subdomain.
// k_prolong: gather-form sum z = sum_j R_j^T t_j: each output DOF visits the
//   (at most 8) subdomains whose box holds it, in a fixed order, so the result
//   is deterministic without atomics; fused with the partial r.z.
#include "gn_internal.h"

namespace {

constexpr int NT = 256;

// Coarse products y = Z g (lower tiles) and y = Z^T u (upper tiles, which hold
// the transposes) in work units of at most COARSE_UNIT_TILES tiles of one tile
// row, one workgroup each, so that every workgroup streams about the same
// bytes whatever the row's length; a second launch adds the units of each row
// in a fixed order.  Thread (i, p) reads row i of the unit's tiles J = p, p+8,
// ...: 32 lanes read 256 contiguous bytes of a tile column.
template <bool UPPER>
__global__ __launch_bounds__(NT) void k_coarse_units(int NBH, const double* __restrict__ Z,
                                                     const double* __restrict__ Zdt, const int4* __restrict__ units,
                                                     const double* __restrict__ x, double* __restrict__ part,
                                                     const double* __restrict__ done) {
  __shared__ double red[8][TILE + 1];
  if (done && *done != 0.0) return;
  const int4 un = units[blockIdx.x];
  const int R = un.x;
  const int i = threadIdx.x % TILE, p = threadIdx.x / TILE;
  double acc = 0.0;
  for (int C = un.y + p; C < un.z; C += 8) {
    const double* tile = (UPPER && C == R) ? Zdt + (int64_t)R * TILE2 : Z + ((int64_t)R * NBH + C) * TILE2;
    const double* xc = x + (int64_t)C * TILE;
#pragma unroll 8
    for (int c = 0; c < TILE; ++c) acc += tile[c * TILE + i] * xc[c];
  }
  red[p][i] = acc;
  __syncthreads();
  if (threadIdx.x < TILE) {
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) sum += red[q][i];
    part[(int64_t)blockIdx.x * TILE + i] = sum;
  }
}

// y[R*TILE + i] = sum of the unit partials of row R, in unit order
__global__ __launch_bounds__(NT) void k_coarse_rowsum(int NBH, const int* __restrict__ rowstart,
                                                      const double* __restrict__ part, double* __restrict__ y,
                                                      const double* __restrict__ done) {
  if (done && *done != 0.0) return;
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= NBH * TILE) return;
  const int R = t / TILE, i = t % TILE;
  double sum = 0.0;
  for (int u = rowstart[R]; u < rowstart[R + 1]; ++u) sum += part[(int64_t)u * TILE + i];
  y[t] = sum;
}

// Z^T into the free upper tiles: (J,K) = Z(K,J)^T for K > J, Zdt[K] = Z(K,K)^T
// (blockIdx.x enumerates the lower tiles row by row)
__global__ __launch_bounds__(NT) void k_z_transpose(int NBH, double* __restrict__ Z, double* __restrict__ Zdt) {
  __shared__ double sh[TILE][TILE + 1];
  int idx = blockIdx.x;
  int K = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
  while ((int64_t)(K + 1) * (K + 2) / 2 <= idx) ++K;
  while ((int64_t)K * (K + 1) / 2 > idx) --K;
  const int J = idx - K * (K + 1) / 2;
  const double* src = Z + ((int64_t)K * NBH + J) * TILE2;
  double* dst = K == J ? Zdt + (int64_t)K * TILE2 : Z + ((int64_t)J * NBH + K) * TILE2;
  for (int e = threadIdx.x; e < TILE2; e += NT) sh[e / TILE][e % TILE] = src[e];   // sh[col][row]
  __syncthreads();
  for (int e = threadIdx.x; e < TILE2; e += NT) {
    const int col = e / TILE, row = e % TILE;   // dst(row, col) = src(col, row)
    dst[e] = sh[row][col];
  }
}

struct PartAxes {
  const int* cnt0; const int* cnt1; const int* cnt2;
  const int* plo0; const int* plo1; const int* plo2;
};

template <int NC>
__global__ __launch_bounds__(NT) void k_prolong(const SubDesc* __restrict__ subs, int NX, int NY, int NZ,
                                                int P0, int P1, PartAxes pa, const uint8_t* __restrict__ dir,
                                                const double* __restrict__ tvec, const double* __restrict__ Phi,
                                                const double* __restrict__ y, const double* __restrict__ r,
                                                double* __restrict__ z, double* __restrict__ part,
                                                const double* __restrict__ done) {
  __shared__ double sh[16];
  if (done && *done != 0.0) return;
  const int64_t n_node = (int64_t)NX * NY * NZ;
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dotv = 0.0;
  if (node < n_node) {
    int gi = (int)(node % NX), gj = (int)((node / NX) % NY), gk = (int)(node / ((int64_t)NX * NY));
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    int c0 = pa.cnt0[gi], c1 = pa.cnt1[gj], c2 = pa.cnt2[gk];
    int p0 = pa.plo0[gi], p1 = pa.plo1[gj], p2 = pa.plo2[gk];
    for (int b2 = 0; b2 < c2; ++b2)
      for (int b1 = 0; b1 < c1; ++b1)
        for (int b0 = 0; b0 < c0; ++b0) {
          int j = (p0 + b0) + P0 * ((p1 + b1) + P1 * (p2 + b2));
          const SubDesc& sd = subs[j];
          int ln = box_local_node(sd.ilo, sd.in_, sd.permI, gi, gj, gk);
          const double* tv = tvec + sd.offVI + (int64_t)ln * NC;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            double v = tv[c];
            if (Phi && sd.m > 0) {
              const double* ph = Phi + sd.offPhi + ((int64_t)ln * NC + c) * sd.m;
              const double* yy = y + sd.coff;
              for (int k = 0; k < sd.m; ++k) v += ph[k] * yy[k];
            }
            acc[c] += v;
          }
        }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double v = dir[node * NC + c] ? 0.0 : acc[c];
      z[node * NC + c] = v;
      if (r) dotv += v * r[node * NC + c];
    }
  }
  if (part) {
    double s = block_sum(dotv, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
  }
}

// t_j += Phi_j y_j on the rows of every subdomain's I box (a thread per row,
// the rows of Phi_j contiguous), ahead of the gather, which then reads t_j only:
// the same sum per (row, subdomain) in the same order as forming it inside the
// gather, streamed over Phi instead of gathered node by node.
// t_j += Phi_j y_j, one wave per 64 rows of Phi_j.  The wave's rows are one
// contiguous block of 64 m doubles: it is read with consecutive lanes on
// consecutive doubles into LDS (rows padded to m + 1 doubles), then each lane
// forms its row's sum in the order k = 0 .. m - 1 from LDS.  (Loading the rows
// lane by lane had each load instruction touch 64 addresses m doubles apart.)
constexpr int PHI_ROWS = 64;
// blockDim.x / 64 waves per workgroup, each with its own 64-row block (fewer,
// larger workgroups than one wave each)
__global__ __launch_bounds__(4 * PHI_ROWS) void k_phi_add(const SubDesc* __restrict__ subs,
                                                          const double* __restrict__ Phi,
                                                          const double* __restrict__ y, double* __restrict__ tvec,
                                                          const double* __restrict__ done) {
  extern __shared__ double sph[];   // waves x PHI_ROWS x (m + 1)
  if (done && *done != 0.0) return;
  const SubDesc& sd = subs[blockIdx.y];
  const int m = sd.m;
  const int nwv = blockDim.x / PHI_ROWS;
  if (m == 0 || (int)blockIdx.x * nwv * PHI_ROWS >= sd.nI) return;   // the whole workgroup
  const int wv = threadIdx.x / PHI_ROWS, lane = threadIdx.x % PHI_ROWS;
  const int r0 = (blockIdx.x * nwv + wv) * PHI_ROWS;
  const int nr = max(0, min(PHI_ROWS, sd.nI - r0));
  double* mys = sph + wv * PHI_ROWS * (m + 1);
  const double* ph = Phi + sd.offPhi + (int64_t)r0 * m;
  for (int e = lane; e < nr * m; e += PHI_ROWS) {
    const int r = e / m, k = e - r * m;
    mys[r * (m + 1) + k] = ph[e];
  }
  __syncthreads();
  if (lane >= nr) return;
  const double* yy = y + sd.coff;
  const double* mine = mys + lane * (m + 1);
  double v = tvec[sd.offVI + r0 + lane];
  for (int k = 0; k < m; ++k) v += mine[k] * yy[k];
  tvec[sd.offVI + r0 + lane] = v;
}

}  // namespace

namespace gnk {

int max_lds_doubles() { return 18 * 1024; }

void coarse_solve(const gn_precond* pc, const double* done, hipStream_t s) {
  if (pc->NH == 0) return;
  GnProfScope prof(PROF_COARSE, (double)pc->NBH * (pc->NBH + 1) * TILE2 * 8.0, s);
  const unsigned rs_grid = (unsigned)((pc->NBH * TILE + NT - 1) / NT);
  hipLaunchKernelGGL(k_coarse_units<false>, dim3(pc->n_cu_f), dim3(NT), 0, s, pc->NBH, pc->d_Z, pc->d_Zdt,
                     pc->d_cu_f, pc->d_g, pc->d_zpart, done);
  GN_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_coarse_rowsum, dim3(rs_grid), dim3(NT), 0, s, pc->NBH, pc->d_rs_f, pc->d_zpart, pc->d_u,
                     done);
  GN_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_coarse_units<true>, dim3(pc->n_cu_b), dim3(NT), 0, s, pc->NBH, pc->d_Z, pc->d_Zdt,
                     pc->d_cu_b, pc->d_u, pc->d_zpart, done);
  GN_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_coarse_rowsum, dim3(rs_grid), dim3(NT), 0, s, pc->NBH, pc->d_rs_b, pc->d_zpart, pc->d_y,
                     done);
  GN_CHECK_LAUNCH();
}

void z_transpose(gn_precond* pc, hipStream_t s) {
  const int64_t n = (int64_t)pc->NBH * (pc->NBH + 1) / 2;
  hipLaunchKernelGGL(k_z_transpose, dim3((unsigned)n), dim3(NT), 0, s, pc->NBH, pc->d_Z, pc->d_Zdt);
  GN_CHECK_LAUNCH();
}

int prolong_blocks(const gn_problem* p) { return (int)((p->n_node + NT - 1) / NT); }

void prolong(const gn_problem* p, const gn_precond* pc, const double* r, double* z, double* part,
             const double* done, hipStream_t s) {
  PartAxes pa{pc->d_cnt[0], pc->d_cnt[1], pc->d_cnt[2], pc->d_plo[0], pc->d_plo[1], pc->d_plo[2]};
  GnProfScope prof(PROF_PROLONG, pc->prolong_bytes, s);
  if (pc->NH > 0) {
    // four waves per workgroup while their rows fit in 64 KB of LDS
    const int nwv = sizeof(double) * 4 * PHI_ROWS * (pc->max_m + 1) <= 64 * 1024 ? 4 : 1;
    const int rows = nwv * PHI_ROWS;
    hipLaunchKernelGGL(k_phi_add, dim3((unsigned)((pc->maxNBI * TILE + rows - 1) / rows), (unsigned)pc->n_sub),
                       dim3(rows), sizeof(double) * rows * (pc->max_m + 1), s, pc->d_sub, pc->d_Phi, pc->d_y,
                       pc->d_t, done);
    GN_CHECK_LAUNCH();
  }
  const double* Phi = nullptr;   // folded into the local vectors above
  dim3 grid((unsigned)((p->n_node + NT - 1) / NT));
  if (p->nc == 3)
    hipLaunchKernelGGL(k_prolong<3>, grid, dim3(NT), 0, s, pc->d_sub, p->nn[0], p->nn[1], p->nn[2],
                       pc->nparts[0], pc->nparts[1], pa, p->d_dir, pc->d_t, Phi, pc->d_y, r, z,
                       part, done);
  else
    hipLaunchKernelGGL(k_prolong<1>, grid, dim3(NT), 0, s, pc->d_sub, p->nn[0], p->nn[1], p->nn[2],
                       pc->nparts[0], pc->nparts[1], pa, p->d_dir, pc->d_t, Phi, pc->d_y, r, z,
                       part, done);
  GN_CHECK_LAUNCH();
}

}  // namespace gnk
