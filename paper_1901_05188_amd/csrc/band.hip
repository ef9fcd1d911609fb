// Batched banded Cholesky factors of the local systems and the GenEO pencils,
// and the batched triangular solves that apply them.
//
// Section 3.1: A_j = R_j A R_j^T are the subdomain matrices of V_{h,0}(Omega_j)
// (equivalently the local assembly with homogeneous Dirichlet conditions on the
// artificial boundary); the one-level method applies A_j^-1 on every subdomain
// (eqn:onelevelAS).  Section 3.3: the local solves use a sparse direct solver.
// Here each subdomain is a box of the structured grid; numbering its nodes with
// the longest axis slowest gives a band of width (1 + n0 + n0 n1) ncomp, and the
// Cholesky factor keeps that band (no fill outside it).  The band is stored as
// TILE x TILE tiles: row block K holds tiles (K, K-w .. K), column-major inside
// a tile; the inverse of every diagonal factor tile is stored separately so the
// triangular solves only do tile matrix-vector products.
//
// One workgroup owns one subdomain (uneven sizes in one launch).
#include "gn_internal.h"

namespace {

constexpr int NT = 256;  // threads per workgroup in the band kernels

__device__ inline int64_t tile_off(int64_t offT, int K, int slot, int w) {
  return (offT + (int64_t)K * (w + 1) + slot) * TILE2;
}

// ---------------------------------------------------------------------------
// extraction of A_j = A[I_j, I_j] from the global node-block matrix
// grid: (ceil(maxNBI*TILE / NT), n_sub)
// ---------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(NT) void k_extract_local(const SubDesc* __restrict__ subs, int NX, int NY, int NZ,
                                                      const double* __restrict__ A, double* __restrict__ L) {
  const SubDesc& sd = subs[blockIdx.y];
  int r = blockIdx.x * NT + threadIdx.x;
  int nrows = sd.NBI * TILE;
  if (r >= nrows) return;
  const int w = sd.wI;
  if (r >= sd.nI) {  // padding: identity
    L[tile_off(sd.offTI, r / TILE, w, w) + (r % TILE) * TILE + (r % TILE)] = 1.0;
    return;
  }
  const int64_t n_node = (int64_t)NX * NY * NZ;
  int ln = r / NC, c = r % NC;
  int g[3];
  box_global_node(sd.ilo, sd.in_, sd.permI, ln, g);
  int64_t node = g[0] + (int64_t)NX * (g[1] + (int64_t)NY * g[2]);
  for (int d = 0; d < 27; ++d) {
    int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    int h[3] = {g[0] + dx, g[1] + dy, g[2] + dz};
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) in &= (h[a] >= sd.ilo[a] && h[a] < sd.ilo[a] + sd.in_[a]);
    if (!in) continue;
    int ln2 = box_local_node(sd.ilo, sd.in_, sd.permI, h[0], h[1], h[2]);
#pragma unroll
    for (int c2 = 0; c2 < NC; ++c2) {
      int r2 = ln2 * NC + c2;
      if (r2 > r) continue;
      double v = A[((int64_t)(d * NC + c) * NC + c2) * n_node + node];
      int K = r / TILE, J = r2 / TILE;
      L[tile_off(sd.offTI, K, J - K + w, w) + (r2 % TILE) * TILE + (r % TILE)] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// pencil P = A_N + s X A_O X on the Ibar_j box, from element matrices
// (eqm:matrixForm: A_{Omega_j} over the elements of Omega_j, A_{Omega_j^o} over
// the elements that also belong to another subdomain, X the PoU diagonal),
// Dirichlet rows and columns as identity: its lower band into L and, in the
// same pass (PE, BE not null), all of P and B = X A_O X in node-ELL planes
// (27 NC planes of npad rows from sd.offVB 27 NC) for the eigensolver's
// products.  B takes no identity: its Dirichlet rows and columns are zero
// (X vanishes there).
// ---------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(NT) void k_extract_pencil(const SubDesc* __restrict__ subs, int nex, int ney, int nez,
                                                       const double* __restrict__ Ke, const uint8_t* __restrict__ dir,
                                                       PouDev pa, double shift, double* __restrict__ L,
                                                       double* __restrict__ PE, double* __restrict__ BE) {
  const SubDesc& sd = subs[blockIdx.y];
  int r = blockIdx.x * NT + threadIdx.x;
  int nrows = sd.NBB * TILE;
  if (r >= nrows) return;
  const int w = sd.wB;
  const bool planes = PE != nullptr;
  double* pe = planes ? PE + sd.offVB * (27 * NC) : nullptr;
  double* be = planes ? BE + sd.offVB * (27 * NC) : nullptr;
  if (r >= sd.nB) {
    L[tile_off(sd.offTB, r / TILE, w, w) + (r % TILE) * TILE + (r % TILE)] = 1.0;
    if (planes)
      for (int k = 0; k < 27 * NC; ++k) pe[(int64_t)k * nrows + r] = be[(int64_t)k * nrows + r] = 0.0;
    return;
  }
  const int NX = nex + 1, NY = ney + 1;
  int ln = r / NC, c = r % NC;
  int g[3];
  box_global_node(sd.blo, sd.bn, sd.permB, ln, g);
  int64_t node = g[0] + (int64_t)NX * (g[1] + (int64_t)NY * g[2]);
  bool dr = dir[node * NC + c];
  double xr = pou_x(sd, pa, dir, NX, NY, NC, g[0], g[1], g[2], c);
  for (int d = 0; d < 27; ++d) {
    int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    int h[3] = {g[0] + dx, g[1] + dy, g[2] + dz};
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) in &= (h[a] >= sd.blo[a] && h[a] < sd.blo[a] + sd.bn[a]);
    const int ln2 = in ? box_local_node(sd.blo, sd.bn, sd.permB, h[0], h[1], h[2]) : 0;
    // the band takes the neighbours at or before row r; the planes take all
    if (!in || (ln2 * NC > r && !planes)) {
      if (planes) {
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2)
          pe[(int64_t)(d * NC + c2) * nrows + r] = be[(int64_t)(d * NC + c2) * nrows + r] = 0.0;
      }
      continue;
    }
    double vN[NC], vO[NC];
#pragma unroll
    for (int c2 = 0; c2 < NC; ++c2) vN[c2] = vO[c2] = 0.0;
    // elements containing both nodes, restricted to Omega_j
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = max(max(g[a], h[a]) - 1, sd.elo[a]);
      hi[a] = min(min(g[a], h[a]), sd.ehi[a] - 1);
    }
    for (int ez = lo[2]; ez <= hi[2]; ++ez)
      for (int ey = lo[1]; ey <= hi[1]; ++ey)
        for (int ex = lo[0]; ex <= hi[0]; ++ex) {
          int64_t e = ex + (int64_t)nex * (ey + (int64_t)ney * ez);
          int a1 = (g[0] - ex) + 2 * (g[1] - ey) + 4 * (g[2] - ez);
          int a2 = (h[0] - ex) + 2 * (h[1] - ey) + 4 * (h[2] - ez);
          bool ov = pou_overlap_elem(pa, ex, ey, ez);
          const double* row = Ke + e * (64 * NC * NC) + (int64_t)(a1 * NC + c) * (8 * NC) + a2 * NC;
#pragma unroll
          for (int c2 = 0; c2 < NC; ++c2) {
            double kv = row[c2];
            vN[c2] += kv;
            if (ov) vO[c2] += kv;
          }
        }
    int64_t node2 = h[0] + (int64_t)NX * (h[1] + (int64_t)NY * h[2]);
#pragma unroll
    for (int c2 = 0; c2 < NC; ++c2) {
      int r2 = ln2 * NC + c2;
      const double x2 = pou_x(sd, pa, dir, NX, NY, NC, h[0], h[1], h[2], c2);
      double v;
      if (dr || dir[node2 * NC + c2]) {
        v = (r2 == r) ? 1.0 : 0.0;
      } else {
        v = vN[c2] + shift * xr * x2 * vO[c2];
      }
      if (r2 <= r) {
        int K = r / TILE, J = r2 / TILE;
        L[tile_off(sd.offTB, K, J - K + w, w) + (r2 % TILE) * TILE + (r % TILE)] = v;
      }
      if (planes) {
        pe[(int64_t)(d * NC + c2) * nrows + r] = v;
        be[(int64_t)(d * NC + c2) * nrows + r] = xr != 0.0 ? vO[c2] * (xr * x2) : 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// banded Cholesky, left-looking by block rows, one workgroup per matrix
// ---------------------------------------------------------------------------
struct BandRef {
  int64_t offT, offD;
  int NB, w;
};

// ---------------------------------------------------------------------------
// Left-looking band Cholesky on FP64 matrix cores.  Block row K, tile t (column
// block J = K - w + t):
//   S = A(K,J) - sum_{t2 < t} L(K,J2) L(J,J2)^T,
//   L(K,J) = S Dinv_J^T (t < w),   L(K,K) L(K,K)^T = S, Dinv_K = L(K,K)^-1 (t = w).
// The four waves split the tile products of S (wave q takes t2 = t0 + q + 4m,
// each a full 32 x 32 product on v_mfma_f64_16x16x4f64 with the operands of the
// next product already in flight) and add their partials through LDS; the
// diagonal tile is factored and inverted by all four waves together.
// ---------------------------------------------------------------------------
typedef double bc_d4 __attribute__((ext_vector_type(4)));

__device__ inline void bc_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// RL: the finished tiles L(K, J) of the current block row are also kept in LDS
// (dynamic, w tiles with padded columns), so the X operands of the products come
// from LDS and only the Y operands (earlier block rows) stream from memory: half
// the traffic of the products, and no memory latency on the X side.
template <bool RL>
__global__ __launch_bounds__(NT) void k_band_chol_mfma(const BandRef* __restrict__ mats, double* __restrict__ T,
                                                       double* __restrict__ D, int* __restrict__ info,
                                                       double* __restrict__ TB) {
  extern __shared__ double rowL[];   // RL: w tiles, column-major with TILE + 1 stride
  __shared__ double part[4][TILE][TILE + 1];
  __shared__ double Ss[TILE][TILE + 1];
  __shared__ int fail;
  const BandRef br = mats[blockIdx.x];
  const int w = br.w, NB = br.NB;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int qr = wid & 1, qc = wid >> 1;
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  double xa0[2][8], yb0[2][8], xa1[2][8], yb1[2][8];
  bc_d4 acc[4];
#define BC_LOAD(XA, YB, T2)                                                                    \
  {                                                                                            \
    if (RL) {                                                                                  \
      /* on the diagonal Y = X; the uniform test sits outside the loads, so that */            \
      /* each case is straight-line code (not a branch around every load) */                   \
      const double* xl = rowL + (T2) * (TILE * (TILE + 1));                                    \
      _Pragma("unroll") for (int q = 0; q < 2; ++q)                                            \
        _Pragma("unroll") for (int ks = 0; ks < 8; ++ks)                                       \
          XA[q][ks] = xl[(4 * ks + lk) * (TILE + 1) + q * 16 + lr];                            \
      if (t == w) {                                                                            \
        _Pragma("unroll") for (int q = 0; q < 2; ++q)                                          \
          _Pragma("unroll") for (int ks = 0; ks < 8; ++ks) YB[q][ks] = XA[q][ks];              \
      } else {                                                                                 \
        const double* yp = T + tile_off(br.offT, J, (T2) - t + w, w);                          \
        _Pragma("unroll") for (int q = 0; q < 2; ++q)                                          \
          _Pragma("unroll") for (int ks = 0; ks < 8; ++ks)                                     \
            YB[q][ks] = yp[(4 * ks + lk) * TILE + q * 16 + lr];                                \
      }                                                                                        \
    } else {                                                                                   \
      const double* xp = T + tile_off(br.offT, K, (T2), w);                                    \
      const double* yp = (t == w) ? xp : T + tile_off(br.offT, J, (T2) - t + w, w);            \
      _Pragma("unroll") for (int q = 0; q < 2; ++q)                                            \
        _Pragma("unroll") for (int ks = 0; ks < 8; ++ks) {                                     \
          XA[q][ks] = xp[(4 * ks + lk) * TILE + q * 16 + lr];                                  \
          YB[q][ks] = yp[(4 * ks + lk) * TILE + q * 16 + lr];                                  \
        }                                                                                      \
    }                                                                                          \
  }
#define BC_MFMA(XA, YB)                                                                        \
  _Pragma("unroll") for (int ks = 0; ks < 8; ++ks)                                             \
    _Pragma("unroll") for (int q = 0; q < 4; ++q)                                              \
      acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(XA[q >> 1][ks], YB[q & 1][ks], acc[q], 0, 0, 0);
  for (int K = 0; K < NB; ++K) {
    const int t0 = max(0, w - K);
    for (int t = t0; t <= w; ++t) {
      const int J = K - w + t;
      double* tk = T + tile_off(br.offT, K, t, w);
      double aval[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = threadIdx.x + NT * u;
        aval[u] = tk[(e / TILE) * TILE + e % TILE];
      }
      double dj[8];
      if (t < w) {
        const double* Dj = D + (br.offD + J) * TILE2;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) dj[ks] = Dj[(4 * ks + lk) * TILE + qc * 16 + lr];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = bc_d4{0, 0, 0, 0};
      int t2 = t0 + wid;
      if (t2 < t) BC_LOAD(xa0, yb0, t2)
      if (t2 + 4 < t) BC_LOAD(xa1, yb1, t2 + 4)
      while (t2 < t) {
        BC_MFMA(xa0, yb0)
        if (t2 + 8 < t) BC_LOAD(xa0, yb0, t2 + 8)
        if (t2 + 4 < t) {
          BC_MFMA(xa1, yb1)
          if (t2 + 12 < t) BC_LOAD(xa1, yb1, t2 + 12)
        }
        t2 += 8;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) part[wid][(q >> 1) * 16 + 4 * i + lk][(q & 1) * 16 + lr] = acc[q][i];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = threadIdx.x + NT * u;
        const int r = e % TILE, c = e / TILE;
        Ss[r][c] = aval[u] - ((part[0][r][c] + part[1][r][c]) + (part[2][r][c] + part[3][r][c]));
      }
      __syncthreads();
      if (t < w) {
        // L(K,J) = S Dinv_J^T: quadrant (qr, qc) of this wave
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = bc_d4{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks)
          acc[ks & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ss[qr * 16 + lr][4 * ks + lk], dj[ks], acc[ks & 3], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = qr * 16 + 4 * i + lk, col = qc * 16 + lr;
          const double l = (acc[0][i] + acc[1][i]) + (acc[2][i] + acc[3][i]);
          tk[col * TILE + row] = l;
          // the transposed band (backward sweeps): block row J, slot w - t - 1
          // holds L(K, J)^T
          if (RL && TB) TB[tile_off(br.offT, J, w - t - 1, w) + row * TILE + col] = l;
          if (RL) rowL[t * (TILE * (TILE + 1)) + col * (TILE + 1) + row] = l;
        }
      } else {
        // diagonal tile: factor and inverse by elimination of [S | I] on all
        // four waves (tile_spd_eliminate), then the stores of L(K,K), Dinv_K
        // and (RL) Dinv_K^T
        double(*col)[TILE + 1] = part[0];
        double(*yr)[TILE + 1] = part[1];
        const int f = tile_spd_eliminate(Ss, col, yr, &part[2][0][0]);
        if (threadIdx.x == 0 && f != 0 && !fail) fail = K * TILE + f;
        double* dk = D + (br.offD + K) * TILE2;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = threadIdx.x + NT * u;
          const int r = e % TILE, c = e / TILE;
          double l, x;
          tile_spd_entry(col, yr, r, c, l, x);
          tk[c * TILE + r] = l;
          dk[c * TILE + r] = x;
          if (RL && TB) TB[tile_off(br.offT, K, w, w) + r * TILE + c] = x;   // slot w: Dinv_K^T
        }
      }
      __threadfence_block();
      __syncthreads();
    }
  }
#undef BC_MFMA
#undef BC_LOAD
  if (threadIdx.x == 0) info[blockIdx.x] = fail;
}

// ---------------------------------------------------------------------------
// FP64 -> FP32 copy of the local factors (mixed-precision local solves)
// ---------------------------------------------------------------------------
// Backward band of the single-column sweep: for block row K, tile d - 1
// (d = 1..w) holds L(K+d, K)^T and tile w holds D_K^T (D_K = L(K,K)^-1),
// column-major like every tile, zero where K + d is past the last block row.
// The backward sweep then reads, like the forward one, contiguous tile
// columns across the lanes.  One workgroup per (block row, subdomain).
template <typename FT>
__global__ __launch_bounds__(256) void k_band_transpose(const BandRef* __restrict__ refs, const double* __restrict__ T,
                                                       const double* __restrict__ D, FT* __restrict__ TB) {
  // each of the four waves moves one tile per round: contiguous loads into a
  // padded LDS tile, then contiguous stores of its transpose
  __shared__ double sT[4][TILE * (TILE + 1)];
  const BandRef rf = refs[blockIdx.y];
  const int K = blockIdx.x;
  if (K >= rf.NB) return;
  const int w = rf.w, W1 = w + 1;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* st = sT[wv];
  FT* out = TB + (rf.offT + (int64_t)K * W1) * TILE2;
  for (int d0 = 1; d0 <= w + 1; d0 += 4) {
    const int d = d0 + wv;
    const double* src = nullptr;
    if (d <= w && K + d < rf.NB) src = T + (rf.offT + (int64_t)(K + d) * W1 + (w - d)) * TILE2;
    if (d == w + 1) src = D + (rf.offD + (int64_t)K) * TILE2;
    if (src) {
#pragma unroll
      for (int j = 0; j < TILE2 / 64; ++j) {
        const int e = j * 64 + lane;   // source (row e % TILE, column e / TILE)
        st[(e / TILE) * (TILE + 1) + e % TILE] = src[e];
      }
    }
    __syncthreads();
    if (d <= w + 1) {
      FT* o = out + (int64_t)(d - 1) * TILE2;
#pragma unroll
      for (int j = 0; j < TILE2 / 64; ++j) {
        const int e = j * 64 + lane;   // output (row i, column rr) at rr * TILE + i
        const int i = e % TILE, rr = e / TILE;
        o[e] = src ? (FT)st[i * (TILE + 1) + rr] : (FT)0;
      }
    }
    __syncthreads();
  }
}

__global__ void k_to_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    b[t] = (float)a[t];
}

}  // namespace

namespace gnk {

void extract_local(const gn_problem* p, const gn_precond* pc, double* L, int maxNB, hipStream_t s) {
  dim3 grid((unsigned)((maxNB * TILE + NT - 1) / NT), (unsigned)pc->n_sub);
  if (p->nc == 3)
    hipLaunchKernelGGL(k_extract_local<3>, grid, dim3(NT), 0, s, pc->d_sub, p->nn[0], p->nn[1],
                       p->nn[2], p->d_A, L);
  else
    hipLaunchKernelGGL(k_extract_local<1>, grid, dim3(NT), 0, s, pc->d_sub, p->nn[0], p->nn[1],
                       p->nn[2], p->d_A, L);
  GN_CHECK_LAUNCH();
}

void extract_pencil(const gn_problem* p, const gn_precond* pc, double shift, double* L, int maxNB,
                    hipStream_t s, double* PE, double* BE) {
  if ((PE == nullptr) != (BE == nullptr)) throw gn_error{GN_ERR_ARG, "pencil planes: PE and BE go together"};
  dim3 grid((unsigned)((maxNB * TILE + NT - 1) / NT), (unsigned)pc->n_sub);
  const PouDev pa = gnh::pou_dev(p, pc);
  if (p->nc == 3)
    hipLaunchKernelGGL(k_extract_pencil<3>, grid, dim3(NT), 0, s, pc->d_sub, p->ne[0], p->ne[1],
                       p->ne[2], p->d_Ke, p->d_dir, pa, shift, L, PE, BE);
  else
    hipLaunchKernelGGL(k_extract_pencil<1>, grid, dim3(NT), 0, s, pc->d_sub, p->ne[0], p->ne[1],
                       p->ne[2], p->d_Ke, p->d_dir, pa, shift, L, PE, BE);
  GN_CHECK_LAUNCH();
}

bool band_chol(const void* d_refs, int n, int maxw, double* T, double* D, int* info, hipStream_t s, double* TB) {
  // the row tiles in LDS when they fit beside the kernel's static arrays
  // (the four partial products and the exchange tile, 41.3 KB)
  const size_t rl = sizeof(double) * (size_t)std::max(maxw, 1) * TILE * (TILE + 1);
  const size_t fixed = sizeof(double) * 5 * TILE * (TILE + 1) + 64;
  if (rl + fixed <= 160 * 1024) {
    GN_HIP(hipFuncSetAttribute((const void*)k_band_chol_mfma<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)rl));
    hipLaunchKernelGGL(k_band_chol_mfma<true>, dim3(n), dim3(NT), rl, s, (const BandRef*)d_refs, T, D, info, TB);
    GN_CHECK_LAUNCH();
    return TB != nullptr;
  }
  // (without the row in LDS the registers have no room for the transposed stores)
  hipLaunchKernelGGL(k_band_chol_mfma<false>, dim3(n), dim3(NT), 0, s, (const BandRef*)d_refs, T, D, info, nullptr);
  GN_CHECK_LAUNCH();
  return false;
}

void band_transpose(const void* d_refs, int n, int maxNB, const double* T, const double* D, void* TB, bool f32,
                    hipStream_t s) {
  dim3 grid((unsigned)maxNB, (unsigned)n);
  if (f32)
    hipLaunchKernelGGL(k_band_transpose<float>, grid, dim3(256), 0, s, (const BandRef*)d_refs, T, D, (float*)TB);
  else
    hipLaunchKernelGGL(k_band_transpose<double>, grid, dim3(256), 0, s, (const BandRef*)d_refs, T, D, (double*)TB);
  GN_CHECK_LAUNCH();
}

void to_f32(int64_t n, const double* a, float* b, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3(2048), dim3(256), 0, s, n, a, b);
  GN_CHECK_LAUNCH();
}

}  // namespace gnk
