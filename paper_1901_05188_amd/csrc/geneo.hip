// GenEO set-up kernels: batched shift-and-invert subspace iteration for the
// local generalised eigenproblems, coarse basis, coarse matrix by local
// products, and the dense tiled Cholesky of the coarse matrix.
//
// Section 3.2 (eq-geneo) and Section 3.3.2 (eqm:matrixForm): on each
// subdomain, A_{Omega_j} p = lambda X A_{Omega_j^o} X p, smallest lambda first,
// ||p||_2 = 1, solved in shift-and-invert mode with a small shift.  With
// P = A_N + s B and B = X A_O X, the pencil B p = nu P p has nu = 1/(lambda+s);
// the wanted eigenpairs are the largest nu.  All subdomains iterate in one
// batched launch per step: V <- P^-1 B V (banded triangular solves with the
// factor of P), Rayleigh-Ritz on span(P^-1 B V) with the small pencil
// (Z^T B Z, Z^T P Z) solved by Cholesky + cyclic Jacobi in LDS.
// Section 3.3.2: Phi_{i(j,k)} = X^(j) p_k^j; Section 3.3.3: A_H entries are
// the local products Phi_i^T (Atilde_{j(i)} Phi_l), nonzero only for
// overlapping subdomains.
#include "gn_internal.h"

namespace {

constexpr int NT = 256;

// ---------------------------------------------------------------------------
// B V on the Ibar box (matrix-free from element matrices), b columns
// ---------------------------------------------------------------------------
// B = X A_O X and P = A_N + s B are stored once per set-up in node-ELL form on
// the Ibar box by the pencil extraction: E[k][r], k = d*NC + c2 (27 lattice
// offsets x components), structure of arrays over the padded rows of each
// subdomain (base offVB * 27 * NC).
// out = B V for b columns. A thread computes R consecutive nodes (one
// component) of one BCW-column chunk. Consecutive nodes lie along the fastest
// local axis a0 (the box's shortest), where the neighbours of R nodes are R + 2
// consecutive rows: each of the nine neighbour lines (offsets along the two
// other axes) costs R + 2 row loads instead of 3 R.  Launched for scalar
// problems; vector problems use k_bapply_node below.
constexpr int BCW = 4;
template <int NC>
constexpr int bapply_rows() { return NC == 1 ? 4 : 2; }
// Rows of B coefficients a workgroup touches, as an upper bound: its threads
// cover at most NT / (nchunk NC) + 2 node groups of R nodes.
template <int NC>
constexpr int bapply_span(int nchunk) { return (NT / (nchunk * NC) + 2) * bapply_rows<NC>() * NC; }
template <int NC, bool LDSC>
__global__ __launch_bounds__(NT) void k_bapply(const SubDesc* __restrict__ subs, const double* __restrict__ BE,
                                               int b, const double* __restrict__ V, double* __restrict__ out,
                                               int gx, int ntot, const int* __restrict__ act) {
  constexpr int R = bapply_rows<NC>();
  extern __shared__ double sBE[];   // LDSC: the workgroup's coefficient rows, 27 NC planes of span
  // consecutive workgroups are dealt round-robin to the 8 XCDs; the 1-D grid
  // holds 8 * per workgroups and is remapped so that each XCD walks a
  // contiguous range of items (subdomain, row block): the neighbour rows of a
  // block then sit in the same XCD's L2
  const int per = (ntot + 7) / 8;
  const int lin = blockIdx.x;
  const int item = (lin % 8) * per + lin / 8;
  if (item >= ntot) return;
  const int bx = item % gx, by = item / gx;
  if (act && act[by] == 0) return;
  const SubDesc& sd = subs[by];
  const int npad = sd.NBB * TILE;
  const int nchunk = (b + BCW - 1) / BCW;
  const int tid = bx * NT + threadIdx.x;
  const int col0 = (tid % nchunk) * BCW;
  const int c = (tid / nchunk) % NC;
  const int ln0 = (tid / nchunk / NC) * R;
  const double* Vb = V + sd.offVB * b;
  const double* base = BE + sd.offVB * (27 * NC);
  // LDSC: the coefficients of the workgroup's rows are loaded once, contiguously,
  // instead of by each of the nchunk lanes that share a row
  const int span = bapply_span<NC>(nchunk);
  const int row_lo = ((bx * NT) / (nchunk * NC)) * R * NC;
  if (LDSC) {
    for (int f = threadIdx.x; f < 27 * NC * span; f += NT) {
      const int pl = f / span, rr = row_lo + f % span;
      sBE[f] = rr < npad ? base[(int64_t)pl * npad + rr] : 0.0;
    }
    __syncthreads();
  }
  if (ln0 * NC + c >= npad) return;
  // local node strides along the global axes
  int st[3];
  st[sd.permB[0]] = 1;
  st[sd.permB[1]] = sd.bn[sd.permB[0]];
  st[sd.permB[2]] = sd.bn[sd.permB[0]] * sd.bn[sd.permB[1]];
  const int nmax = sd.nB - 1;
  double acc[R][BCW];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int q = 0; q < BCW; ++q) acc[i][q] = 0.0;
  // coefficient plane of neighbour (o_x, o_y, o_z) in {0,1,2}^3: o_x + 3 o_y + 9 o_z
  const int a0 = sd.permB[0];
  const int ax1 = a0 == 0 ? 1 : 0, ax2 = a0 == 2 ? 1 : 2;
  const int s0 = a0 == 0 ? 1 : (a0 == 1 ? 3 : 9);
  const int s1 = ax1 == 0 ? 1 : 3, s2 = ax2 == 1 ? 3 : 9;
  // B = X A_O X vanishes on the core of the subdomain and on neighbours outside
  // overlap elements, and the zeros come in blocks of rows: a lane whose
  // coefficients on a line are all zero skips the line (its V loads are masked
  // off; skipping adds nothing it would not have added). A lane with a
  // zero coefficient on a line that runs adds 0 * v = +-0, which leaves its
  // sums unchanged (v is finite: row indices are clamped into the box and the
  // buffers' tails are zero). The sums run line by line, then along a0,
  // components innermost; with a0 = x that is the plane order.
#pragma unroll
  for (int yz = 0; yz < 9; ++yz) {
    const int o1 = yz % 3, o2 = yz / 3;
    const int dn = (o1 - 1) * st[ax1] + (o2 - 1) * st[ax2];
    const int dl = o1 * s1 + o2 * s2;
    double bv[R][3][NC];
    bool nz = false;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int row = (ln0 + i) * NC + c;
      const bool rin = row < npad;
      const int rowc = rin ? row : npad - 1;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2) {
          const int pl = (dl + dx * s0) * NC + c2;
          const double t = LDSC ? sBE[pl * span + (rowc - row_lo)] : base[(int64_t)pl * npad + rowc];
          bv[i][dx][c2] = rin ? t : 0.0;
          nz |= bv[i][dx][c2] != 0.0;
        }
    }
    if (!nz) continue;   // per lane: rows whose coefficients on this line are all zero load no V
    // rows of nodes ln0 - 1 .. ln0 + R on this line; out-of-box neighbours have bv = 0
    double v[R + 2][NC][BCW];
#pragma unroll
    for (int j = 0; j < R + 2; ++j)
#pragma unroll
      for (int c2 = 0; c2 < NC; ++c2) {
        const int r2 = min(max((ln0 - 1 + j + dn) * NC + c2, 0), nmax);
        // a chunk may run up to BCW - 1 columns past the row end into the next
        // row or the 64-double tail of the buffer: loads stay in bounds, stores are masked
        const double* vr = Vb + (int64_t)r2 * b + col0;
#pragma unroll
        for (int q = 0; q < BCW; ++q) v[j][c2][q] = vr[q];
      }
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2)
#pragma unroll
          for (int q = 0; q < BCW; ++q) acc[i][q] += bv[i][dx][c2] * v[i + dx][c2][q];
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int row = (ln0 + i) * NC + c;
    if (row < npad)
#pragma unroll
      for (int q = 0; q < BCW; ++q)
        if (col0 + q < b) out[sd.offVB * b + (int64_t)row * b + col0 + q] = acc[i][q];
  }
}

// out = B V for vector problems: a thread computes all NC component rows of one
// node for one CW-column chunk, so each neighbour value it loads from V feeds
// NC rows (the one-component layout above loads every neighbour value once per
// component).  Coefficients come straight from the node-ELL planes (the chunk
// lanes of a node read the same addresses; staging them in LDS instead measured
// slower, at the lower occupancy it allows); a lane whose coefficients on a
// line are all zero loads no V for it.  Every output sums over the same
// sequence (line, dx, c2) as the one-component kernel.
template <int NC, int CW>
__global__ __launch_bounds__(NT) void k_bapply_node(const SubDesc* __restrict__ subs, const double* __restrict__ BE,
                                                    int b, const double* __restrict__ V, double* __restrict__ out,
                                                    int gx, int ntot, const int* __restrict__ act) {
  const int per = (ntot + 7) / 8;
  const int lin = blockIdx.x;
  const int item = (lin % 8) * per + lin / 8;
  if (item >= ntot) return;
  const int bx = item % gx, by = item / gx;
  if (act && act[by] == 0) return;
  const SubDesc& sd = subs[by];
  const int npad = sd.NBB * TILE;
  const int nchunk = (b + CW - 1) / CW;
  const int tid = bx * NT + threadIdx.x;
  const int col0 = (tid % nchunk) * CW;
  const int ln = tid / nchunk;
  if (ln * NC >= npad) return;
  const double* Vb = V + sd.offVB * b;
  const double* base = BE + sd.offVB * (27 * NC);
  int st[3];
  st[sd.permB[0]] = 1;
  st[sd.permB[1]] = sd.bn[sd.permB[0]];
  st[sd.permB[2]] = sd.bn[sd.permB[0]] * sd.bn[sd.permB[1]];
  const int nmax = sd.nB - 1;
  double acc[NC][CW];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int q = 0; q < CW; ++q) acc[c][q] = 0.0;
  const int a0 = sd.permB[0];
  const int ax1 = a0 == 0 ? 1 : 0, ax2 = a0 == 2 ? 1 : 2;
  const int s0 = a0 == 0 ? 1 : (a0 == 1 ? 3 : 9);
  const int s1 = ax1 == 0 ? 1 : 3, s2 = ax2 == 1 ? 3 : 9;
  for (int yz = 0; yz < 9; ++yz) {
    const int o1 = yz % 3, o2 = yz / 3;
    const int dn = (o1 - 1) * st[ax1] + (o2 - 1) * st[ax2];
    const int dl = o1 * s1 + o2 * s2;
    double bv[3][NC][NC];
    bool nz = false;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int row = ln * NC + c;
      const bool rin = row < npad;
      const int rowc = rin ? row : npad - 1;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2) {
          const double t = base[(int64_t)((dl + dx * s0) * NC + c2) * npad + rowc];
          bv[dx][c][c2] = rin ? t : 0.0;
          nz |= bv[dx][c][c2] != 0.0;
        }
    }
    if (!nz) continue;   // per lane: a node whose coefficients on this line are all zero loads no V
    // nodes ln - 1, ln, ln + 1 of this line (clamped into the box: their
    // coefficients are zero where the neighbour lies outside it)
    double v[3][NC][CW];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int c2 = 0; c2 < NC; ++c2) {
        const int r2 = min(max((ln - 1 + j + dn) * NC + c2, 0), nmax);
        // a chunk may run up to CW - 1 columns past the row end into the next
        // row or the 64-double tail of the buffer: loads stay in bounds, stores are masked
        const double* vr = Vb + (int64_t)r2 * b + col0;
#pragma unroll
        for (int q = 0; q < CW; ++q) v[j][c2][q] = vr[q];
      }
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2)
#pragma unroll
          for (int q = 0; q < CW; ++q) acc[c][q] += bv[dx][c][c2] * v[dx][c2][q];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int row = ln * NC + c;
    if (row < npad)
#pragma unroll
      for (int q = 0; q < CW; ++q)
        if (col0 + q < b) out[sd.offVB * b + (int64_t)row * b + col0 + q] = acc[c][q];
  }
}

// v_mfma_f64_16x16x4f64 lane layout: A[l%16][l/16], B[l/16][l%16],
// result item j of lane l = D[4j + l/16][l%16].
typedef double gn_d4 __attribute__((ext_vector_type(4)));

// Barrier that orders LDS traffic only: global loads in flight stay in flight.
__device__ inline void geneo_lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Block solves, one wave per SIMD: four waves per workgroup (row half x tile
// parity), each wave covering NCB 16-column blocks.  Every band tile is loaded
// once per workgroup (by the wave of its row half and parity) and feeds the
// products of all NCB column blocks, and a wave has the register room for a
// prefetch P tiles deep.  The diagonal solve of a block row is split between
// the two parities: the wave pair of parity h owns column block h (NCB = 2) or
// parity 0 owns the single block (NCB = 1); the non-owner's partial sums reach
// the owner through LDS.  A workgroup takes NCB * 16 columns (csplit > 1: the
// chunk g of 16 NCB columns; siblings are n_sub workgroups apart).  Reads past
// column b take finite neighbouring values and feed only unstored outputs; ring
// slots of blocks outside the subdomain stay zero.
// ---------------------------------------------------------------------------
template <int W, int P, int NCB>
__global__ __launch_bounds__(256) void k_trsm_ring(const SubDesc* __restrict__ subs, int n_sub, int csplit, int b,
                                                    int ringlen, const double* __restrict__ T,
                                                    const double* __restrict__ D, const double* __restrict__ TBk,
                                                    const double* __restrict__ Z0, const double* Vin, double* V,
                                                    const int* __restrict__ act) {
  constexpr int WS = W / 2;                 // tile slots per wave and step
  // DEEP (P = W): the A registers hold two block rows, K and K + 1, and each
  // slot is reloaded with row K + 2 (two rows of band tiles in flight)
  constexpr bool DEEP = P == W;
  static_assert(W % 2 == 0 && (DEEP || WS % P == 0), "W / 2 must be a multiple of the prefetch depth");
  extern __shared__ double smem[];
  double* ring = smem;                      // W1 slots x TILE rows x RW columns (+16 pad)
  double* sS = smem + ringlen;              // NCB right-hand-side tiles, 32 x 16 (+1)
  double* sP = sS + NCB * (TILE * 17);      // partial sums [parity][block], 2 NCB tiles
  const SubDesc& sd = subs[blockIdx.x % n_sub];   // subdomains in the XCD-balanced order
  if (act && act[sd.id] == 0) return;
  const int c0 = csplit > 1 ? (int)(blockIdx.x / n_sub) * (16 * NCB) : 0;
  const int RW = csplit > 1 ? 16 * NCB : b; // columns held in the ring
  const int NB = sd.NBB, w = sd.wB, W1 = w + 1;
  const double* Tb = T + sd.offTB * TILE2;
  const double* Db = D + sd.offDB * TILE2;
  double* Vb = V + sd.offVB * b;            // solution (may be Vin: in place)
  const double* Vi = Vin + sd.offVB * b;    // right-hand sides
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int half = wv >> 1, rh = wv & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const int rb = rh * 16;
  // column block whose diagonal solve this wave does, or -1
  const int own = NCB == 2 ? half : (half == 0 ? 0 : -1);
  const int ocol = c0 + (own < 0 ? 0 : own) * 16 + lr;   // column of V for the owned block
  const bool ook = own >= 0 && ocol < b;
  const int olcol = (own < 0 ? 0 : own) * 16 + lr;       // its column in the ring
  for (int e = threadIdx.x; e < ringlen; e += 256) ring[e] = 0.0;
  double a[P][8];
  double dv[8], vv[4];
  gn_d4 acc[NCB][2];   // two chains per column block: consecutive products of a chain are NCB MFMAs apart
#define R2_ZERO() _Pragma("unroll") for (int q = 0; q < NCB; ++q) _Pragma("unroll") for (int u = 0; u < 2; ++u) acc[q][u] = gn_d4{0, 0, 0, 0};
  const int rstride = TILE * RW;
  // products of one block row: slots m = 0 .. WS-1 of this wave's parity, slot
  // m multiplying ring slot (SLOT0 + 2 m) mod W1; the A registers of slot m are
  // reloaded with slot m + P of the row (or of row KN past the end); DEEP: the
  // row's A registers start at BASE, slot m is reloaded with slot m of row KN
#define R2_PRODUCTS(KR, KN, SLOT0, LOADA, BASE)                                                \
  {                                                                                            \
    R2_ZERO()                                                                                  \
    int slot = (SLOT0);                                                                        \
    double bcur[NCB][8], bnxt[NCB][8];                                                         \
    _Pragma("unroll") for (int q = 0; q < NCB; ++q)                                            \
      _Pragma("unroll") for (int ks = 0; ks < 8; ++ks)                                         \
        bnxt[q][ks] = ring[slot * rstride + (4 * ks + lk) * RW + q * 16 + lr];                 \
    _Pragma("unroll") for (int m = 0; m < WS; ++m) {                                           \
      const int sl = DEEP ? (BASE) + m : m % P;                                               \
      _Pragma("unroll") for (int q = 0; q < NCB; ++q)                                          \
        _Pragma("unroll") for (int ks = 0; ks < 8; ++ks) bcur[q][ks] = bnxt[q][ks];            \
      if (m + 1 < WS) {                                                                        \
        slot += 2;                                                                             \
        while (slot >= W1) slot -= W1;                                                         \
        _Pragma("unroll") for (int q = 0; q < NCB; ++q)                                        \
          _Pragma("unroll") for (int ks = 0; ks < 8; ++ks)                                     \
            bnxt[q][ks] = ring[slot * rstride + (4 * ks + lk) * RW + q * 16 + lr];             \
      }                                                                                        \
      _Pragma("unroll") for (int ks = 0; ks < 8; ++ks)                                         \
        _Pragma("unroll") for (int q = 0; q < NCB; ++q)                                        \
          acc[q][ks & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sl][ks], bcur[q][ks], acc[q][ks & 1], 0, 0, 0); \
      __builtin_amdgcn_sched_barrier(0);                                                       \
      if (DEEP) LOADA(sl, (KN), 2 * m + half)                                                  \
      else if (m + P < WS) LOADA(sl, (KR), 2 * (m + P) + half)                                 \
      else LOADA(sl, (KN), 2 * (m + P - WS) + half)                                            \
      __builtin_amdgcn_sched_barrier(0);                                                       \
    }                                                                                          \
  }
  // exchange, diagonal solve of the owned block and the store of block row K
  // (to the ring slot K % W1 and to V); two LDS barriers for every wave
#define R2_FINISH(K)                                                                           \
  {                                                                                            \
    double psum[NCB][4];                                                                       \
    _Pragma("unroll") for (int q = 0; q < NCB; ++q)                                            \
      _Pragma("unroll") for (int i = 0; i < 4; ++i)                                            \
        psum[q][i] = acc[q][0][i] + acc[q][1][i];                                              \
    /* every wave leaves its partial sums of all blocks, the owner its right-hand */          \
    /* side; after one barrier the owner forms S = V - (P0 + P1) as it reads it */             \
    _Pragma("unroll") for (int q = 0; q < NCB; ++q)                                            \
      _Pragma("unroll") for (int i = 0; i < 4; ++i)                                            \
        sP[(half * NCB + q) * (TILE * 17) + (rb + 4 * i + lk) * 17 + lr] = psum[q][i];         \
    if (own >= 0) {                                                                            \
      _Pragma("unroll") for (int i = 0; i < 4; ++i)                                            \
        sS[own * (TILE * 17) + (rb + 4 * i + lk) * 17 + lr] = vv[i];                           \
    }                                                                                          \
    geneo_lds_barrier();                                                                       \
    if (own >= 0) {                                                                            \
      gn_d4 dq[4];                                                                             \
      _Pragma("unroll") for (int u = 0; u < 4; ++u) dq[u] = gn_d4{0, 0, 0, 0};                 \
      _Pragma("unroll") for (int ks = 0; ks < 8; ++ks) {                                       \
        const int o = (4 * ks + lk) * 17 + lr;                                                 \
        const double sk = sS[own * (TILE * 17) + o] -                                          \
                          (sP[own * (TILE * 17) + o] + sP[(NCB + own) * (TILE * 17) + o]);     \
        dq[ks & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(dv[ks], sk, dq[ks & 3], 0, 0, 0);    \
      }                                                                                        \
      double* yk = ring + ((K) % W1) * rstride;                                                \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                          \
        const int row = rb + 4 * i + lk;                                                       \
        const double y = (dq[0][i] + dq[1][i]) + (dq[2][i] + dq[3][i]);                        \
        if (ook) {                                                                             \
          yk[row * RW + olcol] = y;                                                            \
          Vb[(int64_t)((K) * TILE + row) * b + ocol] = y;                                      \
        }                                                                                      \
      }                                                                                        \
    }                                                                                          \
    geneo_lds_barrier();                                                                       \
  }
  // Band tiles hold exact zeros outside the band (row r, column c with
  // r - c > bw): a lane whose entry lies there reads the tile's entry (31, 0)
  // (forward) or (0, 31) (backward), which is zero whenever any entry is, and
  // tiles wholly before or after the matrix read the zero tile Z0, so cache
  // lines holding nothing but zeros are not fetched; the products are unchanged.
  const int bwp = sd.bwB;
  const int lrow = rb + lr - lk;            // row minus column inside the tile, less 4 ks
  // ---- forward: Y_K = Dinv_K (V_K - sum_t L(K,t) Y_{K-w+t}) ----
  // tile t of row K is L(K, K - w + t); entry (i, c) lies outside the band when
  // 32 (w - t) + i - c > bw
#define R2_FWD_TILE(K_, t_) (((t_) < w && (K_) - w + (t_) >= 0) ? Tb + ((int64_t)(K_) * W1 + (t_)) * TILE2 : Z0)
#define R2_LOAD_A_FWD(S_, K_, t_)                                                              \
  {                                                                                            \
    const double* tp = R2_FWD_TILE(K_, t_);                                                    \
    const int lim = bwp - TILE * (w - (t_));                                                   \
    _Pragma("unroll") for (int ks = 0; ks < 8; ++ks)                                           \
      a[S_][ks] = tp[(lrow - 4 * ks > lim) ? TILE - 1 : (4 * ks + lk) * TILE + rb + lr];        \
  }
#define R2_LOAD_DV_FWD(K_)                                                                     \
  {                                                                                            \
    const double* dk = Db + (int64_t)(K_) * TILE2;                                             \
    _Pragma("unroll") for (int ks = 0; ks < 8; ++ks) dv[ks] = dk[(4 * ks + lk) * TILE + rb + lr]; \
    _Pragma("unroll") for (int i = 0; i < 4; ++i)                                              \
      vv[i] = Vi[(int64_t)((K_) * TILE + rb + 4 * i + lk) * b + ocol];                          \
  }
  // the diagonal tile and right-hand side of row K are loaded just before its
  // products and used in its exchange: the products cover their latency, and
  // no register is copied before a reload (which would make the wave wait for
  // every load in flight, the next rows' band tiles included).  Ring slot of
  // tile t of row K: block K - w + t, i.e. (K + 1 + t) % W1
  if constexpr (DEEP) {
#pragma unroll
    for (int sl = 0; sl < WS; ++sl) {
      R2_LOAD_A_FWD(sl, 0, 2 * sl + half)
      R2_LOAD_A_FWD(WS + sl, min(1, NB - 1), 2 * sl + half)
    }
    __syncthreads();
    for (int K = 0; K < NB; K += 2) {
      if (own >= 0) R2_LOAD_DV_FWD(K)
      R2_PRODUCTS(K, min(K + 2, NB - 1), (K + 1 + half) % W1, R2_LOAD_A_FWD, 0)
      R2_FINISH(K)
      if (K + 1 < NB) {
        if (own >= 0) R2_LOAD_DV_FWD(K + 1)
        R2_PRODUCTS(K + 1, min(K + 3, NB - 1), (K + 2 + half) % W1, R2_LOAD_A_FWD, WS)
        R2_FINISH(K + 1)
      }
    }
  } else {
#pragma unroll
    for (int sl = 0; sl < P; ++sl) R2_LOAD_A_FWD(sl, 0, 2 * sl + half)
    __syncthreads();
    for (int K = 0; K < NB; ++K) {
      if (own >= 0) R2_LOAD_DV_FWD(K)
      R2_PRODUCTS(K, min(K + 1, NB - 1), (K + 1 + half) % W1, R2_LOAD_A_FWD, 0)
      R2_FINISH(K)
    }
  }
#undef R2_LOAD_DV_FWD
#undef R2_LOAD_A_FWD
#undef R2_FWD_TILE
  __syncthreads();
  for (int e = threadIdx.x; e < ringlen; e += 256) ring[e] = 0.0;
  // ---- backward: X_K = Dinv_K^T (Y_K - sum_d L(K+d,K)^T X_{K+d}), d = t + 1 ----
  const double* TBb = TBk + sd.offTB * TILE2;
  // tile t of row K holds L(K + t + 1, K)^T: its entry (i, c) is
  // L(K + t + 1, K)(c, i), outside the band when 32 (t + 1) + c - i > bw
#define R2_BWD_TILE(K_, t_) (((t_) < w && (K_) + (t_) + 1 < NB) ? TBb + ((int64_t)(K_) * W1 + (t_)) * TILE2 : Z0)
#define R2_LOAD_A_BWD(S_, K_, t_)                                                              \
  {                                                                                            \
    const double* tp = R2_BWD_TILE(K_, t_);                                                    \
    const int lim = bwp - TILE * ((t_) + 1);                                                   \
    _Pragma("unroll") for (int ks = 0; ks < 8; ++ks)                                           \
      a[S_][ks] = tp[(4 * ks - lrow > lim) ? (TILE - 1) * TILE : (4 * ks + lk) * TILE + rb + lr]; \
  }
#define R2_LOAD_DV_BWD(K_)                                                                     \
  {                                                                                            \
    const double* dk = TBb + ((int64_t)(K_) * W1 + w) * TILE2;                                 \
    _Pragma("unroll") for (int ks = 0; ks < 8; ++ks) dv[ks] = dk[(4 * ks + lk) * TILE + rb + lr]; \
    _Pragma("unroll") for (int i = 0; i < 4; ++i)                                              \
      vv[i] = Vb[(int64_t)((K_) * TILE + rb + 4 * i + lk) * b + ocol];                          \
  }
  // ring slot of tile t of row K: block K + 1 + t
  if constexpr (DEEP) {
#pragma unroll
    for (int sl = 0; sl < WS; ++sl) {
      R2_LOAD_A_BWD(sl, NB - 1, 2 * sl + half)
      R2_LOAD_A_BWD(WS + sl, max(NB - 2, 0), 2 * sl + half)
    }
    __syncthreads();
    for (int K = NB - 1; K >= 0; K -= 2) {
      if (own >= 0) R2_LOAD_DV_BWD(K)
      R2_PRODUCTS(K, max(K - 2, 0), (K + 1 + half) % W1, R2_LOAD_A_BWD, 0)
      R2_FINISH(K)
      if (K - 1 >= 0) {
        if (own >= 0) R2_LOAD_DV_BWD(K - 1)
        R2_PRODUCTS(K - 1, max(K - 3, 0), (K + half) % W1, R2_LOAD_A_BWD, WS)
        R2_FINISH(K - 1)
      }
    }
  } else {
#pragma unroll
    for (int sl = 0; sl < P; ++sl) R2_LOAD_A_BWD(sl, NB - 1, 2 * sl + half)
    __syncthreads();
    for (int K = NB - 1; K >= 0; --K) {
      if (own >= 0) R2_LOAD_DV_BWD(K)
      R2_PRODUCTS(K, max(K - 1, 0), (K + 1 + half) % W1, R2_LOAD_A_BWD, 0)
      R2_FINISH(K)
    }
  }
#undef R2_LOAD_DV_BWD
#undef R2_LOAD_A_BWD
#undef R2_BWD_TILE
#undef R2_FINISH
#undef R2_PRODUCTS
#undef R2_ZERO
}

// ---------------------------------------------------------------------------
// Gram matrices GP = Z^T (B V) = Z^T P Z and GB = Z^T (B Z) on FP64 matrix
// cores, and the Ritz residuals res_k = ||Z_k - nu_k V_k||^2, zz_k = ||Z_k||^2.
// Workgroup (j, g) streams rows [g*chunk, (g+1)*chunk) of subdomain j four at a
// time (the K dimension of v_mfma_f64_16x16x4f64) and writes partial Gram
// matrices and residual sums of its rows; k_small_eig adds the GRAM_SPLIT
// partials in a fixed order.  Wave wid owns the 16-row block kb = wid of both
// Gram matrices (column blocks 0..3).  Padding rows are zero in Z, BV and BZ;
// columns past b only feed output entries that are not stored.
// ---------------------------------------------------------------------------
constexpr int GRAM_SPLIT = 32;

__global__ __launch_bounds__(NT) void k_gram(const SubDesc* __restrict__ subs, int b,
                                             const double* __restrict__ Z, const double* __restrict__ BV,
                                             const double* __restrict__ BZ, const double* __restrict__ V,
                                             const double* __restrict__ nu, double* __restrict__ GPp,
                                             double* __restrict__ GBp, double* __restrict__ resp,
                                             const int* __restrict__ act) {
  __shared__ double sres[4][64], szz[4][64];
  if (act && act[blockIdx.x] == 0) return;
  const SubDesc& sd = subs[blockIdx.x];
  const int64_t base = sd.offVB * b;
  const int g = blockIdx.y;
  const int nall = sd.NBB * TILE;
  const int chunk = ((nall + GRAM_SPLIT * 16 - 1) / (GRAM_SPLIT * 16)) * 16;
  const int rlo = min(g * chunk, nall), rhi = min(rlo + chunk, nall);
  const int64_t part = (int64_t)blockIdx.x * GRAM_SPLIT + g;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int ncb = (b + 15) / 16;
  const bool active = wid < ncb;
  const int acol = min(wid * 16 + lr, 63);
  gn_d4 gp[4], gb[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) gp[q] = gb[q] = gn_d4{0, 0, 0, 0};
  if (active) {
    // rows streamed 16 at a time (4 MFMA K-steps), all loads of a step issued first;
    // padded row counts are multiples of 32
    for (int r0 = rlo; r0 < rhi; r0 += 16) {
      double a[4], bvv[4][4], bzv[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t ro = base + (int64_t)(r0 + 4 * u + lk) * b;
        a[u] = Z[ro + acol];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // column blocks past b are neither loaded nor multiplied
          int col = min(q * 16 + lr, 63);
          bvv[u][q] = q < ncb ? BV[ro + col] : 0.0;
          bzv[u][q] = q < ncb ? BZ[ro + col] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (q < ncb) {
            gp[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bvv[u][q], gp[q], 0, 0, 0);
            gb[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bzv[u][q], gb[q], 0, 0, 0);
          }
        }
    }
    double* gpo = GPp + part * b * b;
    double* gbo = GBp + part * b * b;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int row = wid * 16 + 4 * j + lk, col = q * 16 + lr;
        if (q < ncb && row < b && col < b) {
          gpo[row * b + col] = gp[q][j];
          gbo[row * b + col] = gb[q][j];
        }
      }
  }
  // residuals: lane = column, waves split the rows (nu == nullptr: formed elsewhere)
  if (!nu) return;
  const double nk = lane < b ? nu[(int64_t)blockIdx.x * b + lane] : 0.0;
  double rs = 0.0, zz = 0.0;
  if (lane < b) {
    // four rows per step, all loads of a step issued first (rows in the same order)
    const int rend = min(rhi, sd.nB);
    for (int r = rlo + wid; r < rend; r += 16) {
      double zr[4], vr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int rr = r + 4 * u;
        zr[u] = rr < rend ? Z[base + (int64_t)rr * b + lane] : 0.0;
        vr[u] = rr < rend ? V[base + (int64_t)rr * b + lane] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (r + 4 * u < rend) {
          const double d = zr[u] - nk * vr[u];
          rs += d * d;
          zz += zr[u] * zr[u];
        }
      }
    }
  }
  sres[wid][lane] = rs;
  szz[wid][lane] = zz;
  __syncthreads();
  if (threadIdx.x < b) {
    int k = threadIdx.x;
    resp[part * 2 * b + k] = sres[0][k] + sres[1][k] + sres[2][k] + sres[3][k];
    resp[part * 2 * b + b + k] = szz[0][k] + szz[1][k] + szz[2][k] + szz[3][k];
  }
}

// ---------------------------------------------------------------------------
// small generalised eigenproblem GB y = nu GP y (b <= 64), one workgroup each:
// diagonal scaling, Cholesky GP = R R^T, C = R^-1 GB R^-T, cyclic Jacobi,
// y = D R^-T w, sorted by decreasing nu; Y^T GP Y = I.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_small_eig(int b, const double* __restrict__ GPp,
                                                  const double* __restrict__ GBp, const double* __restrict__ resp,
                                                  double* __restrict__ res, double* __restrict__ Y,
                                                  double* __restrict__ nu_out, int* __restrict__ flag,
                                                  const int* __restrict__ act) {
  extern __shared__ double sm[];
  if (act && act[blockIdx.x] == 0) return;
  const int ld = b + 1;
  double* P = sm;              // b x ld
  double* C = P + b * ld;      // b x ld
  double* W = C + b * ld;      // b x ld
  __shared__ double dsc[64];
  __shared__ double cs[32], sn[32];
  __shared__ int pp[32], qq[32];
  __shared__ int order[64];
  __shared__ double offn;
  __shared__ double wred[NT / 64][2];
  const int tid = threadIdx.x;
  // sum the row-split partials of the Gram matrices and residuals (fixed order)
  {
    const double* gp = GPp + (int64_t)blockIdx.x * GRAM_SPLIT * b * b;
    const double* gb = GBp + (int64_t)blockIdx.x * GRAM_SPLIT * b * b;
    for (int e = tid; e < b * b; e += NT) {
      double sp = 0.0, sb = 0.0;
      for (int g = 0; g < GRAM_SPLIT; ++g) {
        sp += gp[(int64_t)g * b * b + e];
        sb += gb[(int64_t)g * b * b + e];
      }
      W[(e / b) * ld + e % b] = sp;
      C[(e / b) * ld + e % b] = sb;
    }
    const double* rp = resp + (int64_t)blockIdx.x * GRAM_SPLIT * 2 * b;
    for (int e = tid; e < 2 * b; e += NT) {
      double t = 0.0;
      for (int g = 0; g < GRAM_SPLIT; ++g) t += rp[g * 2 * b + e];
      res[(int64_t)blockIdx.x * 2 * b + e] = t;
    }
  }
  __syncthreads();
  if (tid < b) {
    double d = W[tid * ld + tid];
    dsc[tid] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += NT) {
    int k = e / b, l = e % b;
    double s = dsc[k] * dsc[l];
    P[k * ld + l] = 0.5 * (W[k * ld + l] + W[l * ld + k]) * s;
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += NT) {
    int k = e / b, l = e % b;
    if (k <= l) {
      double s = dsc[k] * dsc[l];
      double v = 0.5 * (C[k * ld + l] + C[l * ld + k]) * s;
      C[k * ld + l] = v;
      C[l * ld + k] = v;
    }
  }
  __syncthreads();
  // Cholesky of P (lower, in place)
  for (int k = 0; k < b; ++k) {
    if (tid == 0) {
      double d = P[k * ld + k];
      if (!(d > 1e-26)) {
        if (flag) atomicOr(flag + blockIdx.x, 1);
        d = 1e-26;
      }
      P[k * ld + k] = sqrt(d);
    }
    __syncthreads();
    double piv = P[k * ld + k];
    if (tid > k && tid < b) P[tid * ld + k] /= piv;
    __syncthreads();
    for (int e = tid; e < b * b; e += NT) {
      int rr = e / b, cc = e % b;
      if (cc > k && rr >= cc) P[rr * ld + cc] -= P[rr * ld + k] * P[cc * ld + k];
    }
    __syncthreads();
  }
  // W = R^-1 (lower triangular inverse), column per thread
  if (tid < b) {
    int cc = tid;
    for (int rr = 0; rr < b; ++rr) W[rr * ld + cc] = 0.0;
    for (int rr = cc; rr < b; ++rr) {
      double s = (rr == cc) ? 1.0 : 0.0;
      for (int k = cc; k < rr; ++k) s -= P[rr * ld + k] * W[k * ld + cc];
      W[rr * ld + cc] = s / P[rr * ld + rr];
    }
  }
  __syncthreads();
  // C <- W C W^T  (use P's strict upper part is no longer needed: reuse P as temp)
  for (int e = tid; e < b * b; e += NT) {
    int rr = e / b, cc = e % b;
    double s = 0.0;
    for (int k = 0; k <= rr; ++k) s += W[rr * ld + k] * C[k * ld + cc];
    P[rr * ld + cc] = s;   // T = W C
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += NT) {
    int rr = e / b, cc = e % b;
    double s = 0.0;
    for (int k = 0; k <= cc; ++k) s += P[rr * ld + k] * W[cc * ld + k];
    C[rr * ld + cc] = s;   // T W^T
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += NT) {
    int rr = e / b, cc = e % b;
    if (rr < cc) {
      double s = 0.5 * (C[rr * ld + cc] + C[cc * ld + rr]);
      C[rr * ld + cc] = s;
      C[cc * ld + rr] = s;
    }
  }
  // keep W = R^-1 for the back transform in P (copy), eigenvector accumulator in W
  __syncthreads();
  for (int e = tid; e < b * b; e += NT) {
    int rr = e / b, cc = e % b;
    P[rr * ld + cc] = W[rr * ld + cc];
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += NT) {
    int rr = e / b, cc = e % b;
    W[rr * ld + cc] = (rr == cc) ? 1.0 : 0.0;
  }
  __syncthreads();
  // cyclic Jacobi with round-robin pairing (b even: pad logic handles odd b)
  const int m = (b + 1) & ~1;   // players
  for (int sweep = 0; sweep < 40; ++sweep) {
    {
      // off-diagonal and diagonal squared norms: per-thread strided sums, then
      // wave shuffles and the four wave partials in a fixed order
      double off = 0.0, dn = 0.0;
      for (int e = tid; e < b * b; e += NT) {
        const int k = e / b, l = e % b;
        const double v = C[k * ld + l] * C[k * ld + l];
        if (k == l) dn += v; else off += v;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        off += __shfl_xor(off, o);
        dn += __shfl_xor(dn, o);
      }
      if ((tid & 63) == 0) {
        wred[tid >> 6][0] = off;
        wred[tid >> 6][1] = dn;
      }
      __syncthreads();
      if (tid == 0) {
        const double o4 = (wred[0][0] + wred[1][0]) + (wred[2][0] + wred[3][0]);
        const double d4 = (wred[0][1] + wred[1][1]) + (wred[2][1] + wred[3][1]);
        offn = (o4 <= 1e-32 * d4) ? 1.0 : 0.0;
      }
    }
    __syncthreads();
    if (offn != 0.0) break;
    for (int round = 0; round < m - 1; ++round) {
      if (tid < m / 2) {
        // circle method: player m-1 fixed, others rotate
        int a = (tid == 0) ? m - 1 : (round + tid) % (m - 1);
        int c2 = (round + m - 1 - tid) % (m - 1);
        if (tid == 0) c2 = round % (m - 1);
        int p = min(a, c2), q = max(a, c2);
        pp[tid] = p;
        qq[tid] = q;
        double c = 1.0, s = 0.0;
        if (q < b && p != q) {
          double apq = C[p * ld + q];
          if (apq != 0.0) {
            double app = C[p * ld + p], aqq = C[q * ld + q];
            double theta = (aqq - app) / (2.0 * apq);
            double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      // rows: C <- J^T C
      for (int e = tid; e < (m / 2) * b; e += NT) {
        int pr = e / b, col = e % b;
        int p = pp[pr], q = qq[pr];
        if (q >= b || p == q) continue;
        double c = cs[pr], s = sn[pr];
        double xp = C[p * ld + col], xq = C[q * ld + col];
        C[p * ld + col] = c * xp - s * xq;
        C[q * ld + col] = s * xp + c * xq;
      }
      __syncthreads();
      // columns: C <- C J, W <- W J
      for (int e = tid; e < (m / 2) * b; e += NT) {
        int pr = e / b, row = e % b;
        int p = pp[pr], q = qq[pr];
        if (q >= b || p == q) continue;
        double c = cs[pr], s = sn[pr];
        double xp = C[row * ld + p], xq = C[row * ld + q];
        C[row * ld + p] = c * xp - s * xq;
        C[row * ld + q] = s * xp + c * xq;
        double wp = W[row * ld + p], wq = W[row * ld + q];
        W[row * ld + p] = c * wp - s * wq;
        W[row * ld + q] = s * wp + c * wq;
      }
      __syncthreads();
    }
  }
  // sort by decreasing eigenvalue (rank sort, ties by index)
  if (tid < b) {
    double v = C[tid * ld + tid];
    int rank = 0;
    for (int k = 0; k < b; ++k) {
      double u = C[k * ld + k];
      if (u > v || (u == v && k < tid)) ++rank;
    }
    order[rank] = tid;
  }
  __syncthreads();
  // Y(:, k) = D R^-T w_{order[k]}
  double* Yb = Y + (int64_t)blockIdx.x * b * b;
  for (int e = tid; e < b * b; e += NT) {
    int rr = e / b, k = e % b;
    int src = order[k];
    double s = 0.0;
    for (int l = rr; l < b; ++l) s += P[l * ld + rr] * W[l * ld + src];   // (R^-T)(rr,l) = R^-1(l,rr)
    Yb[rr * b + k] = dsc[rr] * s;
  }
  if (tid < b) nu_out[(int64_t)blockIdx.x * b + tid] = C[order[tid] * ld + order[tid]];
}

// V = Z Y and BV = (B Z) Y (the B-image of the new block without another B
// application) on FP64 matrix cores: each wave takes 16 rows of one subdomain
// (grid.y) and all b columns, A operands straight from Z and BZ (lane group lk
// holds columns KS lk .. KS lk + KS - 1 of its row, all loaded before the
// first product), B operands
// from Y, staged in LDS once per workgroup (rows padded to b + 1 doubles, so
// the four 16-lane groups of a read hit different banks).  Columns past b are
// masked to zero on both operands, so no padding value enters a product.
template <int KS, int CB>   // K-steps and 16-column blocks covered: 4 KS >= b, 16 CB >= b
__global__ __launch_bounds__(NT) void k_vupdate(const SubDesc* __restrict__ subs, int b,
                                                const double* __restrict__ Z, const double* __restrict__ BZ,
                                                const double* __restrict__ Y, double* __restrict__ V,
                                                double* __restrict__ BV, const int* __restrict__ act) {
  __shared__ double sY[64 * 65];
  if (act && act[blockIdx.y] == 0) return;
  const SubDesc& sd = subs[blockIdx.y];
  const int nrow = sd.NBB * TILE;           // padded row counts are multiples of 32
  if (blockIdx.x * (NT / 64) * 16 >= nrow) return;   // the whole workgroup, before the barrier
  const int ldy = b + 1;
  const double* Yb = Y + (int64_t)blockIdx.y * b * b;
  for (int e = threadIdx.x; e < b * b; e += NT) sY[(e / b) * ldy + e % b] = Yb[e];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r0 = (blockIdx.x * (NT / 64) + wv) * 16;
  if (r0 >= nrow) return;                   // no barrier follows
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t arow = sd.offVB * b + (int64_t)(r0 + lr) * b;
  // the K index of step ks in lane group lk is KS lk + ks (any order of the
  // sum serves): each lane reads KS consecutive columns of its row, which the
  // compiler merges into 16-byte loads
  double za[KS], ba[KS];
  if (b == 4 * KS) {                        // full width: no column is masked
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      za[ks] = Z[arow + KS * lk + ks];
      ba[ks] = BZ[arow + KS * lk + ks];
    }
  } else {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = KS * lk + ks;
      za[ks] = k < b ? Z[arow + k] : 0.0;
      ba[ks] = k < b ? BZ[arow + k] : 0.0;
    }
  }
  gn_d4 az[CB], ab[CB];
#pragma unroll
  for (int q = 0; q < CB; ++q) az[q] = ab[q] = gn_d4{0, 0, 0, 0};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k = KS * lk + ks;
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      const int c = q * 16 + lr;
      const double y = (k < b && c < b) ? sY[k * ldy + c] : 0.0;
      az[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(za[ks], y, az[q], 0, 0, 0);
      ab[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ba[ks], y, ab[q], 0, 0, 0);
    }
  }
  const int64_t obase = sd.offVB * b + (int64_t)r0 * b;
#pragma unroll
  for (int q = 0; q < CB; ++q) {
    const int c = q * 16 + lr;
    if (c < b) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t o = obase + (int64_t)(4 * i + lk) * b + c;
        V[o] = az[q][i];
        BV[o] = ab[q][i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Chebyshev filter steps of the subspace iteration.  With T = P^-1 B (Ritz
// values nu of the block in (0, 1/s]) the unwanted part of the spectrum lies in
// [0, nu_cut], nu_cut = the smallest Ritz value of the block; the scaled
// three-term recurrence of the Chebyshev polynomials on that interval damps it
// and amplifies the wanted nu > nu_cut (per subdomain coefficients):
//   Y1 = a1 (T V - c V),   Y_{i+1} = a_i (T Y_i - c Y_i) - beta_i Y_{i-1}.
// k_cheb_first also forms the Ritz residuals of the current block from T V, in
// the same row-split layout as k_gram.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_cheb_first(const SubDesc* __restrict__ subs, int b,
                                                   const double* __restrict__ Z, const double* __restrict__ V,
                                                   const double* __restrict__ nu, const double* __restrict__ coef,
                                                   int ncoef, double* __restrict__ Y1, double* __restrict__ resp,
                                                   const int* __restrict__ act) {
  __shared__ double sres[4][64], szz[4][64];
  if (act && act[blockIdx.x] == 0) return;
  const SubDesc& sd = subs[blockIdx.x];
  const int64_t base = sd.offVB * b;
  const int g = blockIdx.y;
  const int nall = sd.NBB * TILE;
  const int chunk = ((nall + GRAM_SPLIT * 16 - 1) / (GRAM_SPLIT * 16)) * 16;
  const int rlo = min(g * chunk, nall), rhi = min(rlo + chunk, nall);
  const int64_t part = (int64_t)blockIdx.x * GRAM_SPLIT + g;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double a1 = coef[(int64_t)blockIdx.x * ncoef + 0], c = coef[(int64_t)blockIdx.x * ncoef + 1];
  const double nk = lane < b ? nu[(int64_t)blockIdx.x * b + lane] : 0.0;
  double rs = 0.0, zz = 0.0;
  if (lane < b) {
    // four rows per step, all loads of a step issued first (rows in the same order)
    for (int r = rlo + wid; r < rhi; r += 16) {
      double zr[4], vr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int rr = r + 4 * u;
        zr[u] = rr < rhi ? Z[base + (int64_t)rr * b + lane] : 0.0;
        vr[u] = rr < rhi ? V[base + (int64_t)rr * b + lane] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int rr = r + 4 * u;
        if (rr < rhi) {
          Y1[base + (int64_t)rr * b + lane] = a1 * (zr[u] - c * vr[u]);
          if (rr < sd.nB) {
            const double d = zr[u] - nk * vr[u];
            rs += d * d;
            zz += zr[u] * zr[u];
          }
        }
      }
    }
  }
  sres[wid][lane] = rs;
  szz[wid][lane] = zz;
  __syncthreads();
  if (threadIdx.x < b) {
    int k = threadIdx.x;
    resp[part * 2 * b + k] = sres[0][k] + sres[1][k] + sres[2][k] + sres[3][k];
    resp[part * 2 * b + b + k] = szz[0][k] + szz[1][k] + szz[2][k] + szz[3][k];
  }
}

// Y0 <- a (TY - c Y1) - beta Y0 in place (step i: coef[2 + 2(i-2)], coef[3 + 2(i-2)])
// Two entries per thread (a subdomain block holds an even count, 32 NBB b,
// from an even offset): 16-byte accesses; the launcher checks the buffers'
// 16-byte alignment.
typedef double gn_d2 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(NT) void k_cheb_step(const SubDesc* __restrict__ subs, int b,
                                                  const double* __restrict__ TY, const double* __restrict__ Y1,
                                                  double* __restrict__ Y0, const double* __restrict__ coef,
                                                  int ncoef, int step, const int* __restrict__ act) {
  if (act && act[blockIdx.y] == 0) return;
  const SubDesc& sd = subs[blockIdx.y];
  const int64_t n = (int64_t)sd.NBB * TILE * b;
  const int64_t e = 2 * ((int64_t)blockIdx.x * NT + threadIdx.x);
  if (e >= n) return;
  const double* cf = coef + (int64_t)blockIdx.y * ncoef;
  const double c = cf[1], a = cf[2 + 2 * step], beta = cf[3 + 2 * step];
  const int64_t o = sd.offVB * b + e;
  const gn_d2 ty = *reinterpret_cast<const gn_d2*>(TY + o);
  const gn_d2 y1 = *reinterpret_cast<const gn_d2*>(Y1 + o);
  const gn_d2 y0 = *reinterpret_cast<const gn_d2*>(Y0 + o);
  gn_d2 out;
  out[0] = a * (ty[0] - c * y1[0]) - beta * y0[0];
  out[1] = a * (ty[1] - c * y1[1]) - beta * y0[1];
  *reinterpret_cast<gn_d2*>(Y0 + o) = out;
}

// Zero-energy modes on the Ibar box of the subdomains with m_j > 0 (their
// nodes carry no Dirichlet DOF): the constant (NC = 1), or the translations
// e_x, e_y, e_z and the infinitesimal rotations e_a x (x - c) about the box
// centre c (NC = 3), at the physical node positions (ramp map included).
// Rows in the pencil's box numbering; other subdomains and padding rows zero.
template <int NC>
__global__ __launch_bounds__(NT) void k_zem_modes(const SubDesc* __restrict__ subs, const double* __restrict__ xn0,
                                                  const double* __restrict__ xn1, const double* __restrict__ xn2,
                                                  int map_kind, double mx0, double mx1, double mtan, int b,
                                                  double* __restrict__ V) {
  const SubDesc& sd = subs[blockIdx.y];
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= sd.NBB * TILE) return;
  double* out = V + sd.offVB * b + (int64_t)r * b;
  if (r >= sd.nB || sd.m == 0) {
    for (int k = 0; k < b; ++k) out[k] = 0.0;
    return;
  }
  if (NC == 1) {
    out[0] = 1.0;
    return;
  }
  int g[3];
  box_global_node(sd.blo, sd.bn, sd.permB, r / NC, g);
  const int c = r % NC;
  const double x = xn0[g[0]], y = xn1[g[1]];
  double z = xn2[g[2]];
  if (map_kind == 1) z += mtan * (fmin(fmax(x, mx0), mx1) - mx0);
  const double d0 = x - 0.5 * (xn0[sd.blo[0]] + xn0[sd.blo[0] + sd.bn[0] - 1]);
  const double d1 = y - 0.5 * (xn1[sd.blo[1]] + xn1[sd.blo[1] + sd.bn[1] - 1]);
  const double d2 = z - 0.5 * (xn2[sd.blo[2]] + xn2[sd.blo[2] + sd.bn[2] - 1]);
  out[0] = c == 0 ? 1.0 : 0.0;
  out[1] = c == 1 ? 1.0 : 0.0;
  out[2] = c == 2 ? 1.0 : 0.0;
  // e_x x d = (0, -d2, d1), e_y x d = (d2, 0, -d0), e_z x d = (-d1, d0, 0)
  out[3] = c == 0 ? 0.0 : (c == 1 ? -d2 : d1);
  out[4] = c == 0 ? d2 : (c == 1 ? 0.0 : -d0);
  out[5] = c == 0 ? -d1 : (c == 1 ? d0 : 0.0);
}

// Rayleigh quotients lambda_k = p_k^T A_N p_k / p_k^T B p_k of the b columns of
// V on each subdomain's Ibar box (eq-geneo with v = p), both energies summed
// element by element: A_N over the elements of Omega_j, B = X A_O X over those
// that also lie in another subdomain.  Every term is an element energy
// (non-negative up to rounding), so the quotient keeps the digits that
// 1/nu - s cancels when lambda is far below the shift.  Workgroup (j, chunk of
// 32 columns): the element matrices of RQ_EL elements at a time are staged in
// LDS (each read from memory once), lane c % 32 takes column c of the chunk and
// lane group c / 32 one of the staged elements; the partial energies are added
// in a fixed order.
constexpr int RQ_EL = NT / 32;
template <int NC>
__global__ __launch_bounds__(NT) void k_eig_rq(const SubDesc* __restrict__ subs, int nex, int ney,
                                               const double* __restrict__ Ke, const uint8_t* __restrict__ dir,
                                               PouDev pa, int b, const double* __restrict__ V,
                                               double* __restrict__ lam) {
  constexpr int ND = 8 * NC;
  __shared__ double sK[RQ_EL][ND * ND];
  __shared__ double sa[RQ_EL][33], sb[RQ_EL][33];
  const SubDesc& sd = subs[blockIdx.x];
  const int cl = threadIdx.x & 31, el = threadIdx.x >> 5;
  const int col = blockIdx.y * 32 + cl;
  const bool cok = col < b;
  const int NX = nex + 1, NY = ney + 1;
  const int n0 = sd.ehi[0] - sd.elo[0], n1 = sd.ehi[1] - sd.elo[1], n2 = sd.ehi[2] - sd.elo[2];
  const int nel = n0 * n1 * n2;
  const double* Vb = V + sd.offVB * b + (cok ? col : 0);
  double ea = 0.0, eb = 0.0;
  for (int t0 = 0; t0 < nel; t0 += RQ_EL) {
    __syncthreads();   // the previous batch's matrices are no longer read
    for (int f = threadIdx.x; f < RQ_EL * ND * ND; f += NT) {
      const int q = f / (ND * ND), t = t0 + q;
      double k = 0.0;
      if (t < nel) {
        const int ex = sd.elo[0] + t % n0, ey = sd.elo[1] + (t / n0) % n1, ez = sd.elo[2] + t / (n0 * n1);
        k = Ke[(ex + (int64_t)nex * (ey + (int64_t)ney * ez)) * (ND * ND) + f % (ND * ND)];
      }
      sK[q][f % (ND * ND)] = k;
    }
    __syncthreads();
    const int t = t0 + el;
    if (t >= nel || !cok) continue;
    const int ex = sd.elo[0] + t % n0, ey = sd.elo[1] + (t / n0) % n1, ez = sd.elo[2] + t / (n0 * n1);
    double pv[ND], xv[ND];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int g0 = ex + (a & 1), g1 = ey + ((a >> 1) & 1), g2 = ez + (a >> 2);
      const int rb = box_local_node(sd.blo, sd.bn, sd.permB, g0, g1, g2) * NC;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        pv[a * NC + c] = Vb[(int64_t)(rb + c) * b];
        xv[a * NC + c] = pou_x(sd, pa, dir, NX, NY, NC, g0, g1, g2, c) * pv[a * NC + c];
      }
    }
    const bool ov = pou_overlap_elem(pa, ex, ey, ez);
    const double* K = sK[el];
    double sA = 0.0, sB = 0.0;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      double kp = 0.0, kx = 0.0;
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        const double k = K[i * ND + j];
        kp += k * pv[j];
        kx += k * xv[j];
      }
      sA += pv[i] * kp;
      sB += xv[i] * kx;
    }
    ea += sA;
    if (ov) eb += sB;
  }
  sa[el][cl] = ea;
  sb[el][cl] = eb;
  __syncthreads();
  if (el == 0 && cok) {
    double ta = 0.0, tb = 0.0;
    for (int q = 0; q < RQ_EL; ++q) {
      ta += sa[q][cl];
      tb += sb[q][cl];
    }
    lam[(int64_t)blockIdx.x * b + col] = tb > 0.0 ? ta / tb : INFINITY;
  }
}

// The same quotients for scalar problems, whose element matrices (64 values)
// are read straight from memory: workgroup (j, chunk of 16 columns), lane
// c % 16 of the column chunk, 16 element lanes striding the elements of the
// box; the partial energies are added in a fixed order.
template <int NC>
__global__ __launch_bounds__(NT) void k_eig_rq_direct(const SubDesc* __restrict__ subs, int nex, int ney,
                                               const double* __restrict__ Ke, const uint8_t* __restrict__ dir,
                                               PouDev pa, int b, const double* __restrict__ V,
                                               double* __restrict__ lam) {
  constexpr int ND = 8 * NC;
  __shared__ double sa[16][17], sb[16][17];
  const SubDesc& sd = subs[blockIdx.x];
  const int cl = threadIdx.x & 15, el = threadIdx.x >> 4;
  const int col = blockIdx.y * 16 + cl;
  const int NX = nex + 1, NY = ney + 1;
  const int n0 = sd.ehi[0] - sd.elo[0], n1 = sd.ehi[1] - sd.elo[1], n2 = sd.ehi[2] - sd.elo[2];
  const int nel = n0 * n1 * n2;
  double ea = 0.0, eb = 0.0;
  if (col < b) {
    const double* Vb = V + sd.offVB * b + col;
    for (int t = el; t < nel; t += 16) {
      const int ex = sd.elo[0] + t % n0, ey = sd.elo[1] + (t / n0) % n1, ez = sd.elo[2] + t / (n0 * n1);
      double pv[ND], xv[ND];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int g0 = ex + (a & 1), g1 = ey + ((a >> 1) & 1), g2 = ez + (a >> 2);
        const int rb = box_local_node(sd.blo, sd.bn, sd.permB, g0, g1, g2) * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          pv[a * NC + c] = Vb[(int64_t)(rb + c) * b];
          xv[a * NC + c] = pou_x(sd, pa, dir, NX, NY, NC, g0, g1, g2, c) * pv[a * NC + c];
        }
      }
      const bool ov = pou_overlap_elem(pa, ex, ey, ez);
      const double* K = Ke + (ex + (int64_t)nex * (ey + (int64_t)ney * ez)) * (ND * ND);
      double sA = 0.0, sB = 0.0;
      for (int i = 0; i < ND; ++i) {
        double kp = 0.0, kx = 0.0;
#pragma unroll
        for (int j = 0; j < ND; ++j) {
          const double k = K[i * ND + j];
          kp += k * pv[j];
          kx += k * xv[j];
        }
        sA += pv[i] * kp;
        sB += xv[i] * kx;
      }
      ea += sA;
      if (ov) eb += sB;
    }
  }
  sa[el][cl] = ea;
  sb[el][cl] = eb;
  __syncthreads();
  if (el == 0 && col < b) {
    double ta = 0.0, tb = 0.0;
    for (int q = 0; q < 16; ++q) {
      ta += sa[q][cl];
      tb += sb[q][cl];
    }
    lam[(int64_t)blockIdx.x * b + col] = tb > 0.0 ? ta / tb : INFINITY;
  }
}

// Defect of the Ritz pairs in the original pencil, rho = B V - P V diag(nu)
// (P V and B V from the node-ELL products), and the correction
// V += (P^-1 rho) diag(1/nu): one inverse-iteration step in defect form, whose
// banded solve acts on the small residual only, so its backward error (of the
// order of the condition of P times the solved vector) no longer limits the
// eigenvectors.  Columns with nu ~ 0 (the null space of B) are left alone.
__global__ __launch_bounds__(NT) void k_defect(const SubDesc* __restrict__ subs, int b,
                                               const double* __restrict__ BV, const double* __restrict__ PV,
                                               const double* __restrict__ nu, double* __restrict__ rho) {
  const SubDesc& sd = subs[blockIdx.y];
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (t >= (int64_t)sd.NBB * TILE * b) return;
  const int col = (int)(t % b);
  const int64_t i = sd.offVB * b + t;
  rho[i] = BV[i] - nu[(int64_t)blockIdx.y * b + col] * PV[i];
}

__global__ __launch_bounds__(NT) void k_defect_add(const SubDesc* __restrict__ subs, int b,
                                                   const double* __restrict__ D, const double* __restrict__ nu,
                                                   double nu_min, double* __restrict__ V) {
  const SubDesc& sd = subs[blockIdx.y];
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (t >= (int64_t)sd.NBB * TILE * b) return;
  const double nk = nu[(int64_t)blockIdx.y * b + (int)(t % b)];
  const int64_t i = sd.offVB * b + t;
  if (nk > nu_min) V[i] += D[i] / nk;
}

// Ritz residual sums of one subdomain: the GRAM_SPLIT row-split partials added
// in fixed order (the same sums k_small_eig forms)
__global__ void k_resid_sum(int b, const double* __restrict__ resp, double* __restrict__ res,
                            const int* __restrict__ act) {
  if (act && act[blockIdx.x] == 0) return;
  const double* rp = resp + (int64_t)blockIdx.x * GRAM_SPLIT * 2 * b;
  for (int e = threadIdx.x; e < 2 * b; e += blockDim.x) {
    double t = 0.0;
    for (int g = 0; g < GRAM_SPLIT; ++g) t += rp[g * 2 * b + e];
    res[(int64_t)blockIdx.x * 2 * b + e] = t;
  }
}

// deterministic start block: hash of (subdomain, row, col) -> (-1, 1); zero on padding
__global__ void k_vinit(const SubDesc* __restrict__ subs, int b, double* __restrict__ V) {
  const SubDesc& sd = subs[blockIdx.y];
  int r = blockIdx.x * NT + threadIdx.x;
  if (r >= sd.NBB * TILE) return;
  for (int col = 0; col < b; ++col) {
    uint64_t h = ((uint64_t)blockIdx.y * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)r * 0xBF58476D1CE4E5B9ull) ^
                 ((uint64_t)col * 0x94D049BB133111EBull);
    h ^= h >> 31;
    h *= 0xD6E8FEB86659FD93ull;
    h ^= h >> 32;
    double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
    V[sd.offVB * b + (int64_t)r * b + col] = (r < sd.nB) ? 2.0 * u - 1.0 : 0.0;
  }
}

// unit 2-norm, largest-magnitude entry positive (lowest index on ties), first
// ncol columns: one wave per column (grid.y blocks of NT / 64 columns), lanes
// striding the rows, wave-wide shuffle reductions
__global__ __launch_bounds__(NT) void k_normalise(const SubDesc* __restrict__ subs, int b, int ncol,
                                                  double* __restrict__ V) {
  const SubDesc& sd = subs[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.y * (NT / 64) + (threadIdx.x >> 6);
  if (k >= ncol) return;                    // wave-uniform, no barrier in this kernel
  double* Vb = V + sd.offVB * b;
  double s = 0.0, mv = -1.0;
  int mi = 0x7fffffff;
  for (int r = lane; r < sd.nB; r += 64) {
    const double v = Vb[(int64_t)r * b + k];
    s += v * v;
    const double a = fabs(v);
    if (a > mv) { mv = a; mi = r; }         // rows ascend: the lowest index wins ties
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    const double a = __shfl_xor(mv, off);
    const int ai = __shfl_xor(mi, off);
    if (a > mv || (a == mv && ai < mi)) { mv = a; mi = ai; }
  }
  if (mi == 0x7fffffff) return;             // no rows
  const double sg = Vb[(int64_t)mi * b + k] < 0.0 ? -1.0 : 1.0;
  const double scale = s > 0.0 ? sg / sqrt(s) : 1.0;   // a zero column stays zero
  for (int r = lane; r < sd.nB; r += 64) Vb[(int64_t)r * b + k] *= scale;
}

// Phi_j (I-box rows x m_j, row-major) = X p on the I box
template <int NC>
__global__ __launch_bounds__(NT) void k_build_phi(const SubDesc* __restrict__ subs, int NX, int NY,
                                                  const uint8_t* __restrict__ dir, PouDev pa, int b,
                                                  const double* __restrict__ V, double* __restrict__ Phi) {
  const SubDesc& sd = subs[blockIdx.y];
  int r = blockIdx.x * NT + threadIdx.x;
  if (r >= sd.nI || sd.m == 0) return;
  int g[3];
  box_global_node(sd.ilo, sd.in_, sd.permI, r / NC, g);
  int c = r % NC;
  double x = pou_x(sd, pa, dir, NX, NY, NC, g[0], g[1], g[2], c);
  int rb = box_local_node(sd.blo, sd.bn, sd.permB, g[0], g[1], g[2]) * NC + c;
  const double* vr = V + sd.offVB * b + (int64_t)rb * b;
  double* out = Phi + sd.offPhi + (int64_t)r * sd.m;
  for (int k = 0; k < sd.m; ++k) out[k] = x * vr[k];
}

// Y_j = A Phi_j on the Ibar box (nB rows x m_j, row-major, stride b)
template <int NC>
__global__ __launch_bounds__(NT) void k_aphi(const SubDesc* __restrict__ subs, int NX, int NY, int NZ,
                                             const double* __restrict__ A, const double* __restrict__ Phi,
                                             int b, double* __restrict__ Y) {
  const SubDesc& sd = subs[blockIdx.y];
  int r = blockIdx.x * NT + threadIdx.x;
  if (r >= sd.nB || sd.m == 0) return;
  const int64_t n_node = (int64_t)NX * NY * NZ;
  int g[3];
  box_global_node(sd.blo, sd.bn, sd.permB, r / NC, g);
  int c = r % NC;
  int64_t node = g[0] + (int64_t)NX * (g[1] + (int64_t)NY * g[2]);
  double* yr = Y + sd.offVB * b + (int64_t)r * b;
  for (int k0 = 0; k0 < sd.m; k0 += 16) {   // up to 16 columns per pass over the stencil
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    for (int d = 0; d < 27; ++d) {
      int h[3] = {g[0] + d % 3 - 1, g[1] + (d / 3) % 3 - 1, g[2] + d / 9 - 1};
      bool in = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) in &= (h[a] >= sd.ilo[a] && h[a] < sd.ilo[a] + sd.in_[a]);
      if (!in) continue;
      int ln2 = box_local_node(sd.ilo, sd.in_, sd.permI, h[0], h[1], h[2]);
#pragma unroll
      for (int c2 = 0; c2 < NC; ++c2) {
        double av = A[((int64_t)(d * NC + c) * NC + c2) * n_node + node];
        const double* ph = Phi + sd.offPhi + (int64_t)(ln2 * NC + c2) * sd.m + k0;
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (k0 + q < sd.m) acc[q] += av * ph[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (k0 + q < sd.m) yr[k0 + q] = acc[q];
  }
}

// A_H block (j1, j2): sum over nodes of I_j1 cap Ibar_j2 of Phi_j1^T Y_j2, written
// into dense tiles (tile (K,J) column-major at (K*NBH + J)*TILE2)
struct Pair { int j1, j2; int lo[3], hi[3]; };

template <int NC>
__global__ __launch_bounds__(NT) void k_ah_pairs(const SubDesc* __restrict__ subs, const Pair* __restrict__ pairs,
                                                 const double* __restrict__ Phi, int b,
                                                 const double* __restrict__ Y, int NBH,
                                                 double* __restrict__ AH) {
  const Pair pr = pairs[blockIdx.x];
  const SubDesc& s1 = subs[pr.j1];
  const SubDesc& s2 = subs[pr.j2];
  const int m1 = s1.m, m2 = s2.m;
  if (m1 == 0 || m2 == 0) return;
  int n0 = pr.hi[0] - pr.lo[0], n1 = pr.hi[1] - pr.lo[1], n2 = pr.hi[2] - pr.lo[2];
  int nnodes = n0 * n1 * n2;
  // entry (k, l) of the block: a sum over the nodes of the intersection; with
  // fewer entries than threads, nsplit threads share an entry (every nsplit-th
  // node each) and their partial sums are added in a fixed order
  const int nent = m1 * m2;
  const int nsplit = nent < NT ? NT / nent : 1;
  __shared__ double red[NT];
  for (int p0 = 0; p0 < nent; p0 += NT) {
    const int pidx = p0 + threadIdx.x % (nsplit > 1 ? nent : NT), ch = nsplit > 1 ? threadIdx.x / nent : 0;
    double s = 0.0;
    if (pidx < nent && ch < nsplit) {
      const int k = pidx / m2, l = pidx % m2;
      for (int t = ch; t < nnodes; t += nsplit) {
        int gi = pr.lo[0] + t % n0, gj = pr.lo[1] + (t / n0) % n1, gk = pr.lo[2] + t / (n0 * n1);
        int l1 = box_local_node(s1.ilo, s1.in_, s1.permI, gi, gj, gk);
        int l2 = box_local_node(s2.blo, s2.bn, s2.permB, gi, gj, gk);
#pragma unroll
        for (int c = 0; c < NC; ++c)
          s += Phi[s1.offPhi + (int64_t)(l1 * NC + c) * m1 + k] * Y[s2.offVB * b + (int64_t)(l2 * NC + c) * b + l];
      }
    }
    if (nsplit > 1) {
      red[threadIdx.x] = s;
      __syncthreads();
      if (threadIdx.x < nent) {
        s = 0.0;
        for (int q = 0; q < nsplit; ++q) s += red[q * nent + threadIdx.x];
      }
    }
    if (pidx < nent && ch == 0) {
      const int k = pidx / m2, l = pidx % m2;
      int row = s1.coff + k, col = s2.coff + l;
      AH[((int64_t)(row / TILE) * NBH + col / TILE) * TILE2 + (col % TILE) * TILE + row % TILE] = s;
    }
  }
}

// symmetrise the dense tiled A_H, identity on padding rows
__global__ void k_ah_sym(int NH, int NBH, double* __restrict__ AH) {
  int64_t n = (int64_t)NBH * TILE;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  int64_t row = t / n, col = t % n;
  if (col > row) return;
  auto at = [&](int64_t r, int64_t c) -> double& {
    return AH[((r / TILE) * NBH + c / TILE) * TILE2 + (c % TILE) * TILE + r % TILE];
  };
  if (row >= NH || col >= NH) {
    double v = (row == col) ? 1.0 : 0.0;
    at(row, col) = v;
    at(col, row) = v;
    return;
  }
  double v = 0.5 * (at(row, col) + at(col, row));
  at(row, col) = v;
  at(col, row) = v;
}

// ---------------------------------------------------------------------------
// dense tiled Cholesky (right-looking) of the coarse matrix and Z = L^-1
// tiles: (K,J) at (K*NB + J)*TILE2, column-major inside a tile
// ---------------------------------------------------------------------------
__device__ inline void lds_tile(double* dst, const double* src) {
  for (int t = threadIdx.x; t < TILE2; t += NT) {
    int col = t / TILE, row = t % TILE;
    dst[col * (TILE + 1) + row] = src[t];
  }
}

// Cholesky factor L(K,K) of the diagonal tile and its inverse Dinv_K by one
// workgroup (tile_spd_eliminate).  A non-positive pivot records its index
// (first one only) in *info and is taken as 1 so the factorization runs to the
// end.
__global__ __launch_bounds__(NT) void k_potrf_tile(int NB, int K, double* __restrict__ A,
                                                   double* __restrict__ Dinv, int* __restrict__ info) {
  static_assert(NT == 256, "the tile elimination takes 256 threads");
  __shared__ double S[TILE][TILE + 1];   // S[row][column]
  __shared__ double col[TILE][TILE + 1], yr[TILE][TILE + 1], sink[NT];
  double* tk = A + ((int64_t)K * NB + K) * TILE2;
  for (int e = threadIdx.x; e < TILE2; e += NT) S[e % TILE][e / TILE] = tk[e];
  __syncthreads();
  const int f = tile_spd_eliminate(S, col, yr, sink);
  if (threadIdx.x == 0 && f != 0 && *info == 0) *info = K * TILE + f;
  double* dk = Dinv + (int64_t)K * TILE2;
  for (int e = threadIdx.x; e < TILE2; e += NT) {
    const int r = e % TILE, c = e / TILE;
    double l, x;
    tile_spd_entry(col, yr, r, c, l, x);
    tk[e] = l;
    dk[e] = x;
  }
}

// L(I,K) = A(I,K) Dinv_K^T for I = K+1+blockIdx.x
__global__ __launch_bounds__(NT) void k_trsm_tile(int NB, int K, double* __restrict__ A,
                                                  const double* __restrict__ Dinv) {
  __shared__ double X[TILE * (TILE + 1)], Dk[TILE * (TILE + 1)];
  int I = K + 1 + blockIdx.x;
  double* t = A + ((int64_t)I * NB + K) * TILE2;
  lds_tile(X, t);
  lds_tile(Dk, Dinv + (int64_t)K * TILE2);
  __syncthreads();
  const int i = threadIdx.x % TILE, c0 = threadIdx.x / TILE;
  for (int q = 0; q < 4; ++q) {
    int c = c0 + 8 * q;
    double s = 0.0;
    for (int k = 0; k < TILE; ++k) s += X[k * (TILE + 1) + i] * Dk[k * (TILE + 1) + c];
    t[c * TILE + i] = s;
  }
}

// One 16 x 16 quadrant per wave of the tile product X Y, X(r,k) at xs[k*TILE + r];
// Y(k,c) at ys[c*TILE + k] (TRANSY = false) or ys[k*TILE + c] (TRANSY = true)
template <bool TRANSY>
__device__ inline void tile_mma(const double* __restrict__ xs, const double* __restrict__ ys, int qr, int qc,
                                int lr, int lk, double out[4]) {
  gn_d4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = gn_d4{0, 0, 0, 0};
  double av[8], bv[8];
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) {
    const int k = 4 * ks + lk;
    av[ks] = xs[k * TILE + qr * 16 + lr];
    bv[ks] = TRANSY ? ys[k * TILE + qc * 16 + lr] : ys[(qc * 16 + lr) * TILE + k];
  }
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) acc[ks & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], bv[ks], acc[ks & 3], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) out[i] = (acc[0][i] + acc[1][i]) + (acc[2][i] + acc[3][i]);
}

// Explicit inverse Z = L^-1 of the coarse factor, right-looking over block
// rows K: row K is finished (Z(K,J) = -Dinv_K sum_{J<=M<K} L(K,M) Z(M,J) for
// J < K, Z(K,K) = Dinv_K), then every later row I accumulates L(I,K) Z(K,J).
// Z starts at zero and keeps the running sums in its unfinished rows.
__global__ __launch_bounds__(NT) void k_trinv_row(int NB, int K, const double* __restrict__ Dinv,
                                                  double* __restrict__ Z) {
  const int J = blockIdx.x;
  double* zt = Z + ((int64_t)K * NB + J) * TILE2;
  const double* dk = Dinv + (int64_t)K * TILE2;
  if (J == K) {
    for (int e = threadIdx.x; e < TILE2; e += NT) zt[e] = dk[e];
    return;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4, qr = wid & 1, qc = wid >> 1;
  double o[4];
  tile_mma<false>(dk, zt, qr, qc, lr, lk, o);
  __syncthreads();   // every wave has read its column block of the running sum
#pragma unroll
  for (int i = 0; i < 4; ++i) zt[(qc * 16 + lr) * TILE + qr * 16 + 4 * i + lk] = -o[i];
}

__global__ __launch_bounds__(NT) void k_trinv_update(int NB, int K, const double* __restrict__ L,
                                                     double* __restrict__ Z) {
  const int I = K + 1 + blockIdx.x / (K + 1), J = blockIdx.x % (K + 1);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4, qr = wid & 1, qc = wid >> 1;
  double o[4];
  tile_mma<false>(L + ((int64_t)I * NB + K) * TILE2, Z + ((int64_t)K * NB + J) * TILE2, qr, qc, lr, lk, o);
  double* zt = Z + ((int64_t)I * NB + J) * TILE2;
#pragma unroll
  for (int i = 0; i < 4; ++i) zt[(qc * 16 + lr) * TILE + qr * 16 + 4 * i + lk] += o[i];
}

// Panel forms of the two updates above.  The coarse factor and its inverse are
// built in panels of CPANEL tile columns (rows): inside a panel the tile steps
// run as before, restricted to the panel, and the rest of the matrix receives
// the whole panel's contribution in one pass, CPANEL tile products summed in
// the matrix-core accumulators per output tile.  Each trailing tile is then
// read and written once per panel instead of once per tile column, which is
// what bounded the tile-by-tile updates.
constexpr int CPANEL = 16;

// acc += X Y over one tile pair (the accumulating form of tile_mma)
template <bool TRANSY>
__device__ inline void tile_mma_acc(const double* __restrict__ xs, const double* __restrict__ ys, int qr, int qc,
                                    int lr, int lk, gn_d4 acc[4]) {
  double av[8], bv[8];
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) {
    const int k = 4 * ks + lk;
    av[ks] = xs[k * TILE + qr * 16 + lr];
    bv[ks] = TRANSY ? ys[k * TILE + qc * 16 + lr] : ys[(qc * 16 + lr) * TILE + k];
  }
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) acc[ks & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], bv[ks], acc[ks & 3], 0, 0, 0);
}

// A(I,J) -= sum_{k0 <= k < k1} L(I,k) L(J,k)^T over the tiles J0 <= J < J1,
// J <= I < NB, J1 - J0 <= CPANEL (the updates inside a panel; one workgroup per
// tile; blockIdx.x runs down column J0, then J0 + 1, ...: column J holds NB - J
// tiles)
__global__ __launch_bounds__(NT) void k_syrk_panel(int NB, int k0, int k1, int J0, int J1, double* __restrict__ A) {
  int idx = blockIdx.x, J = J0;
  while (J < J1 && idx >= NB - J) idx -= NB - J, ++J;   // at most CPANEL columns
  if (J >= J1) return;
  const int I = J + idx;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4, qr = wid & 1, qc = wid >> 1;
  gn_d4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = gn_d4{0, 0, 0, 0};
  for (int k = k0; k < k1; ++k)
    tile_mma_acc<true>(A + ((int64_t)I * NB + k) * TILE2, A + ((int64_t)J * NB + k) * TILE2, qr, qc, lr, lk, acc);
  double* t = A + ((int64_t)I * NB + J) * TILE2;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    t[(qc * 16 + lr) * TILE + qr * 16 + 4 * i + lk] -= (acc[0][i] + acc[1][i]) + (acc[2][i] + acc[3][i]);
}

// Trailing updates in 2 x 2 blocks of tiles: each wave owns one whole output
// tile (its four 16 x 16 quadrants), so a wave loads each operand tile once for
// four quadrant products instead of once per quadrant, and the four waves of a
// workgroup share their operand tiles through the L1 cache.
// acc[r][c][.] += X(r quadrant rows, :) Y(:, c quadrant columns) over one tile
// pair: its operands (tile_full_load), loaded ahead of the products (tile_full_mma)
template <bool TRANSY>
__device__ inline void tile_full_load(const double* __restrict__ xs, const double* __restrict__ ys, int lr, int lk,
                                      double av[2][8], double bv[2][8]) {
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) {
    const int k = 4 * ks + lk;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      av[r][ks] = xs[k * TILE + r * 16 + lr];
      bv[r][ks] = TRANSY ? ys[k * TILE + r * 16 + lr] : ys[(r * 16 + lr) * TILE + k];
    }
  }
}
// (one accumulator chain per quadrant: the four quadrants' products interleave,
// so each chain's previous product has left the pipeline when the next issues)
__device__ inline void tile_full_mma(const double av[2][8], const double bv[2][8], gn_d4 acc[2][2]) {
#pragma unroll
  for (int ks = 0; ks < 8; ++ks)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r][ks], bv[c][ks], acc[r][c], 0, 0, 0);
}
// acc += sum_{k = ka}^{kb - 1} X(k) Y(k), the operands of step k + 1 in flight
// during the products of step k (two register sets, used alternately)
template <bool TRANSY, typename XF, typename YF>
__device__ inline void tile_full_sum(int ka, int kb, XF xs, YF ys, int lr, int lk, gn_d4 acc[2][2]) {
  if (ka >= kb) return;
  double a0[2][8], b0[2][8], a1[2][8], b1[2][8];
  tile_full_load<TRANSY>(xs(ka), ys(ka), lr, lk, a0, b0);
  for (int k = ka; k < kb; k += 2) {
    if (k + 1 < kb) tile_full_load<TRANSY>(xs(k + 1), ys(k + 1), lr, lk, a1, b1);
    tile_full_mma(a0, b0, acc);
    if (k + 1 >= kb) break;
    if (k + 2 < kb) tile_full_load<TRANSY>(xs(k + 2), ys(k + 2), lr, lk, a0, b0);
    tile_full_mma(a1, b1, acc);
  }
}

// the wave's output tile t (column-major) += sgn * acc
__device__ inline void tile_store_acc(double* __restrict__ t, double sgn, int lr, int lk, gn_d4 acc[2][2]) {
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        t[(c * 16 + lr) * TILE + r * 16 + 4 * i + lk] += sgn * acc[r][c][i];
}

// A(I,J) -= sum_{k0 <= k < k1} L(I,k) L(J,k)^T for J0 <= J <= I < NB: block
// (blockIdx.x, blockIdx.y) covers I = J0 + 2 bx + (0, 1), J = J0 + 2 by + (0, 1)
// (blocks wholly above the diagonal return at once; wave = (I offset, J offset))
__global__ __launch_bounds__(NT, 2) void k_syrk_panel2(int NB, int k0, int k1, int J0, double* __restrict__ A) {
  if (blockIdx.x < blockIdx.y) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int I = J0 + 2 * (int)blockIdx.x + (wv & 1), J = J0 + 2 * (int)blockIdx.y + (wv >> 1);
  if (I >= NB || J > I) return;
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  gn_d4 acc[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[r][c] = gn_d4{0, 0, 0, 0};
  tile_full_sum<true>(
      k0, k1, [&](int k) { return A + ((int64_t)I * NB + k) * TILE2; },
      [&](int k) { return A + ((int64_t)J * NB + k) * TILE2; }, lr, lk, acc);
  tile_store_acc(A + ((int64_t)I * NB + J) * TILE2, -1.0, lr, lk, acc);
}

// Z(I,J) += sum_{max(k0,J) <= k < k1} L(I,k) Z(k,J) for I in [I0, NB), J in [0, k1):
// block (blockIdx.x, blockIdx.y) covers J = 2 bx + (0, 1), I = I0 + 2 by + (0, 1)
__global__ __launch_bounds__(NT, 2) void k_trinv_panel2(int NB, int k0, int k1, int I0, const double* __restrict__ L,
                                                     double* __restrict__ Z) {
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int J = 2 * (int)blockIdx.x + (wv & 1), I = I0 + 2 * (int)blockIdx.y + (wv >> 1);
  if (J >= k1 || I >= NB) return;
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  gn_d4 acc[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[r][c] = gn_d4{0, 0, 0, 0};
  tile_full_sum<false>(
      max(k0, J), k1, [&](int k) { return L + ((int64_t)I * NB + k) * TILE2; },
      [&](int k) { return Z + ((int64_t)k * NB + J) * TILE2; }, lr, lk, acc);
  tile_store_acc(Z + ((int64_t)I * NB + J) * TILE2, 1.0, lr, lk, acc);
}


}  // namespace

namespace gnk {

static PouDev pou_axes(const gn_precond* pc) { return gnh::pou_dev(pc->prob, pc); }

void eig_vinit(const gn_precond* pc, int b, int maxNBB, double* V, hipStream_t s) {
  hipLaunchKernelGGL(k_vinit, dim3((maxNBB * TILE + NT - 1) / NT, pc->n_sub), dim3(NT), 0, s,
                     pc->d_sub, b, V);
  GN_CHECK_LAUNCH();
}

void eig_rq(const gn_problem* p, const gn_precond* pc, int b, const double* V, double* lam, hipStream_t s) {
  if (p->nc == 3)
    hipLaunchKernelGGL(k_eig_rq<3>, dim3((unsigned)pc->n_sub, (unsigned)((b + 31) / 32)), dim3(NT), 0, s, pc->d_sub,
                       p->ne[0], p->ne[1], p->d_Ke, p->d_dir, pou_axes(pc), b, V, lam);
  else
    hipLaunchKernelGGL(k_eig_rq_direct<1>, dim3((unsigned)pc->n_sub, (unsigned)((b + 15) / 16)), dim3(NT), 0, s,
                       pc->d_sub, p->ne[0], p->ne[1], p->d_Ke, p->d_dir, pou_axes(pc), b, V, lam);
  GN_CHECK_LAUNCH();
}

void eig_defect(const gn_precond* pc, int b, int maxNBB, const double* BV, const double* PV, const double* nu,
                double* rho, hipStream_t s) {
  dim3 grid((unsigned)(((int64_t)maxNBB * TILE * b + NT - 1) / NT), pc->n_sub);
  hipLaunchKernelGGL(k_defect, grid, dim3(NT), 0, s, pc->d_sub, b, BV, PV, nu, rho);
  GN_CHECK_LAUNCH();
}

void eig_defect_add(const gn_precond* pc, int b, int maxNBB, const double* D, const double* nu, double nu_min,
                    double* V, hipStream_t s) {
  dim3 grid((unsigned)(((int64_t)maxNBB * TILE * b + NT - 1) / NT), pc->n_sub);
  hipLaunchKernelGGL(k_defect_add, grid, dim3(NT), 0, s, pc->d_sub, b, D, nu, nu_min, V);
  GN_CHECK_LAUNCH();
}

void eig_resid_sum(int n_sub, int b, const double* resp, double* res, hipStream_t s, const int* act) {
  hipLaunchKernelGGL(k_resid_sum, dim3(n_sub), dim3(128), 0, s, b, resp, res, act);
  GN_CHECK_LAUNCH();
}

void zem_modes(const gn_problem* p, const gn_precond* pc, int b, int maxNBB, double* V, hipStream_t s) {
  if (b != (p->nc == 3 ? 6 : 1)) throw gn_error{GN_ERR_ARG, "zero-energy modes: 6 columns (elasticity) or 1"};
  dim3 grid((maxNBB * TILE + NT - 1) / NT, pc->n_sub);
  const double mtan = p->map_kind == 1 ? tan(p->map_par[2]) : 0.0;
  if (p->nc == 3)
    hipLaunchKernelGGL(k_zem_modes<3>, grid, dim3(NT), 0, s, pc->d_sub, p->d_xn[0], p->d_xn[1], p->d_xn[2],
                       p->map_kind, p->map_par[0], p->map_par[1], mtan, b, V);
  else
    hipLaunchKernelGGL(k_zem_modes<1>, grid, dim3(NT), 0, s, pc->d_sub, p->d_xn[0], p->d_xn[1], p->d_xn[2],
                       p->map_kind, p->map_par[0], p->map_par[1], mtan, b, V);
  GN_CHECK_LAUNCH();
}

void eig_bapply(const gn_problem* p, const gn_precond* pc, const double* BE, int b, int maxNBB,
                const double* V, double* out, hipStream_t s, const int* act) {
  const int nchunk = (b + BCW - 1) / BCW;
  const int nc = p->nc;
  if (nc == 3) {
    // one thread per node and column chunk, all three component rows
    constexpr int CW = 8;
    const int nchunk8 = (b + CW - 1) / CW;
    const int64_t nodes = (maxNBB * TILE + 2) / 3;
    const int gx = (int)((nodes * nchunk8 + NT - 1) / NT);
    const int ntot = gx * pc->n_sub;
    hipLaunchKernelGGL((k_bapply_node<3, CW>), dim3((unsigned)(8 * ((ntot + 7) / 8))), dim3(NT), 0, s, pc->d_sub,
                       BE, b, V, out, gx, ntot, act);
    GN_CHECK_LAUNCH();
    return;
  }
  // scalar problems: threads per subdomain = node groups of R x column chunks
  constexpr int R = bapply_rows<1>();
  const int64_t nodes = maxNBB * TILE;
  const int gx = (int)((((nodes + R - 1) / R) * nchunk + NT - 1) / NT);
  const int ntot = gx * pc->n_sub;
  dim3 grid((unsigned)(8 * ((ntot + 7) / 8)));
  // coefficient rows in LDS when they fit in 48 KB (b >= 17)
  const size_t lds = sizeof(double) * 27 * bapply_span<1>(nchunk);
  if (lds <= 48 * 1024)
    hipLaunchKernelGGL((k_bapply<1, true>), grid, dim3(NT), lds, s, pc->d_sub, BE, b, V, out, gx, ntot, act);
  else
    hipLaunchKernelGGL((k_bapply<1, false>), grid, dim3(NT), 0, s, pc->d_sub, BE, b, V, out, gx, ntot, act);
  GN_CHECK_LAUNCH();
}

void eig_trsm(const gn_precond* pc, int b, const double* T, const double* D, const double* TB, const double* Vin,
              double* V, hipStream_t s, const int* act) {
  if (b > 64) throw gn_error{GN_ERR_ARG, "eigensolver block larger than 64"};
  int maxw = 0;
  for (const SubDesc& sd : pc->sub) maxw = std::max(maxw, sd.wB);
  // four-wave kernel: 32-column chunks, or 16-column ones when that ring does not fit
  {
    const int maxw1 = maxw + 1;
    int ncb2 = b <= 16 ? 1 : 2;
    int cs2 = (b + 16 * ncb2 - 1) / (16 * ncb2);
    int rw2 = cs2 > 1 ? 16 * ncb2 : b;
    int rl2 = maxw1 * TILE * rw2 + 32;
    size_t lds2 = sizeof(double) * ((size_t)rl2 + (size_t)3 * ncb2 * TILE * 17);
    if (lds2 > 160 * 1024 && ncb2 == 2) {
      ncb2 = 1;
      cs2 = (b + 15) / 16;
      rw2 = cs2 > 1 ? 16 : b;
      rl2 = maxw1 * TILE * rw2 + 32;
      lds2 = sizeof(double) * ((size_t)rl2 + (size_t)3 * TILE * 17);
    }
    // the smallest instantiated slot count W >= maxw (W / 2 a multiple of the
    // prefetch depth P): slots past the band multiply zero tiles, so a W close
    // to the band saves matrix-core work (the kernel keeps the units about two
    // thirds busy at the c5 widths)
    int W2 = 0;
    for (int wc : {6, 12, 14, 16, 18, 20, 24, 30})
      if (W2 == 0 && wc >= maxw) W2 = wc;
    if (lds2 <= 160 * 1024 && W2 > 0 && pc->d_z0 && TB) {
#define GN_R2(WV, PV, NV)                                                                             \
  do {                                                                                                \
    GN_HIP(hipFuncSetAttribute((const void*)k_trsm_ring<WV, PV, NV>,                                 \
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));               \
    hipLaunchKernelGGL((k_trsm_ring<WV, PV, NV>), dim3(pc->n_sub * cs2), dim3(256), lds2, s,         \
                       pc->d_subxB, pc->n_sub, cs2, b, rl2, T, D, TB, pc->d_z0, Vin, V, act);         \
  } while (0)
#define GN_R2W(WV, PV)                     \
  do {                                     \
    if (ncb2 == 2) GN_R2(WV, PV, 2);       \
    else GN_R2(WV, PV, 1);                 \
  } while (0)
      switch (W2) {
        case 6: GN_R2W(6, 3); break;
        case 12: GN_R2W(12, 12); break;
        case 14: GN_R2W(14, 14); break;
        case 16: GN_R2W(16, 4); break;
        case 18: GN_R2W(18, 3); break;
        case 20: GN_R2W(20, 5); break;
        case 24: GN_R2W(24, 6); break;
        default: GN_R2W(30, 3); break;
      }
#undef GN_R2W
#undef GN_R2
      GN_CHECK_LAUNCH();
      return;
    }
  }
  throw gn_error{GN_ERR_ARG, "GenEO pencil band of " + std::to_string(maxw) +
                                 " tiles is wider than the block solves take (30 tiles, or the LDS ring of " +
                                 std::to_string(b) + " columns does not fit): use more subdomains"};
}

int gram_split() { return GRAM_SPLIT; }

void eig_cheb_first(const gn_precond* pc, int b, const double* Z, const double* V, const double* nu,
                    const double* coef, int ncoef, double* Y1, double* resp, hipStream_t s, const int* act) {
  hipLaunchKernelGGL(k_cheb_first, dim3(pc->n_sub, GRAM_SPLIT), dim3(NT), 0, s, pc->d_sub, b, Z, V, nu, coef,
                     ncoef, Y1, resp, act);
  GN_CHECK_LAUNCH();
}

void eig_cheb_step(const gn_precond* pc, int b, int maxNBB, const double* TY, const double* Y1, double* Y0,
                   const double* coef, int ncoef, int step, hipStream_t s, const int* act) {
  if ((((uintptr_t)TY | (uintptr_t)Y1 | (uintptr_t)Y0) & 15) != 0)
    throw gn_error{GN_ERR_ARG, "Chebyshev step buffers not 16-byte aligned"};
  dim3 grid((unsigned)(((int64_t)maxNBB * TILE * b / 2 + NT - 1) / NT), pc->n_sub);
  hipLaunchKernelGGL(k_cheb_step, grid, dim3(NT), 0, s, pc->d_sub, b, TY, Y1, Y0, coef, ncoef, step, act);
  GN_CHECK_LAUNCH();
}

void eig_gram(const gn_precond* pc, int b, const double* Z, const double* BV, const double* BZ,
              const double* V, const double* nu, double* GPp, double* GBp, double* resp, hipStream_t s,
              const int* act) {
  hipLaunchKernelGGL(k_gram, dim3(pc->n_sub, GRAM_SPLIT), dim3(NT), 0, s, pc->d_sub, b, Z, BV, BZ, V, nu,
                     GPp, GBp, resp, act);
  GN_CHECK_LAUNCH();
}

void eig_small(int n_sub, int b, const double* GPp, const double* GBp, const double* resp, double* res,
               double* Y, double* nu, int* flag, hipStream_t s, const int* act) {
  size_t lds = sizeof(double) * 3 * b * (b + 1);
  GN_HIP(hipFuncSetAttribute((const void*)k_small_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  hipLaunchKernelGGL(k_small_eig, dim3(n_sub), dim3(NT), lds, s, b, GPp, GBp, resp, res, Y, nu, flag, act);
  GN_CHECK_LAUNCH();
}

void eig_vupdate(const gn_precond* pc, int b, int maxNBB, const double* Z, const double* BZ,
                 const double* Y, double* V, double* BV, hipStream_t s, const int* act) {
  if (b > 64) throw gn_error{GN_ERR_ARG, "eigensolver block larger than 64"};
  const int waves = maxNBB * TILE / 16;       // 16-row blocks of the largest subdomain
  const dim3 grid((waves + NT / 64 - 1) / (NT / 64), pc->n_sub);
  if (b <= 32)
    hipLaunchKernelGGL((k_vupdate<8, 2>), grid, dim3(NT), 0, s, pc->d_sub, b, Z, BZ, Y, V, BV, act);
  else
    hipLaunchKernelGGL((k_vupdate<16, 4>), grid, dim3(NT), 0, s, pc->d_sub, b, Z, BZ, Y, V, BV, act);
  GN_CHECK_LAUNCH();
}

void eig_normalise(const gn_precond* pc, int b, int ncol, double* V, hipStream_t s) {
  if (ncol <= 0 || pc->n_sub <= 0) return;
  const int cpb = NT / 64;                  // columns per workgroup
  hipLaunchKernelGGL(k_normalise, dim3(pc->n_sub, (ncol + cpb - 1) / cpb), dim3(NT), 0, s, pc->d_sub, b, ncol, V);
  GN_CHECK_LAUNCH();
}

void build_phi(const gn_problem* p, const gn_precond* pc, int b, int maxNI, const double* V,
               hipStream_t s) {
  dim3 grid((maxNI + NT - 1) / NT, pc->n_sub);
  if (p->nc == 3)
    hipLaunchKernelGGL(k_build_phi<3>, grid, dim3(NT), 0, s, pc->d_sub, p->nn[0], p->nn[1], p->d_dir,
                       pou_axes(pc), b, V, pc->d_Phi);
  else
    hipLaunchKernelGGL(k_build_phi<1>, grid, dim3(NT), 0, s, pc->d_sub, p->nn[0], p->nn[1], p->d_dir,
                       pou_axes(pc), b, V, pc->d_Phi);
  GN_CHECK_LAUNCH();
}

void aphi(const gn_problem* p, const gn_precond* pc, int b, int maxNB, double* Y, hipStream_t s) {
  dim3 grid((maxNB + NT - 1) / NT, pc->n_sub);
  if (p->nc == 3)
    hipLaunchKernelGGL(k_aphi<3>, grid, dim3(NT), 0, s, pc->d_sub, p->nn[0], p->nn[1], p->nn[2],
                       p->d_A, pc->d_Phi, b, Y);
  else
    hipLaunchKernelGGL(k_aphi<1>, grid, dim3(NT), 0, s, pc->d_sub, p->nn[0], p->nn[1], p->nn[2],
                       p->d_A, pc->d_Phi, b, Y);
  GN_CHECK_LAUNCH();
}

void ah_pairs(const gn_problem* p, const gn_precond* pc, const void* d_pairs, int npairs, int b,
              const double* Y, double* AH, hipStream_t s) {
  if (p->nc == 3)
    hipLaunchKernelGGL(k_ah_pairs<3>, dim3(npairs), dim3(NT), 0, s, pc->d_sub, (const Pair*)d_pairs,
                       pc->d_Phi, b, Y, pc->NBH, AH);
  else
    hipLaunchKernelGGL(k_ah_pairs<1>, dim3(npairs), dim3(NT), 0, s, pc->d_sub, (const Pair*)d_pairs,
                       pc->d_Phi, b, Y, pc->NBH, AH);
  GN_CHECK_LAUNCH();
  int64_t n = (int64_t)pc->NBH * TILE;
  hipLaunchKernelGGL(k_ah_sym, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, pc->NH,
                     pc->NBH, AH);
  GN_CHECK_LAUNCH();
}

int pair_size() { return (int)sizeof(Pair); }
void make_pair(void* dst, int j1, int j2, const int lo[3], const int hi[3]) {
  Pair* p = (Pair*)dst;
  p->j1 = j1;
  p->j2 = j2;
  for (int a = 0; a < 3; ++a) {
    p->lo[a] = lo[a];
    p->hi[a] = hi[a];
  }
}

// number of tiles (I, J) with J0 <= J < J1 and J <= I < NB
static int64_t trapezoid_tiles(int NB, int J0, int J1) {
  int64_t n = 0;
  for (int J = J0; J < J1; ++J) n += NB - J;
  return n;
}

// Right-looking tiled Cholesky in panels of CPANEL tile columns: inside a
// panel each column is factored (k_potrf_tile, k_trsm_tile) and updates the
// panel's later columns; then one k_syrk_panel2 launch applies the panel to
// the trailing matrix.
void dense_chol(int NB, double* A, double* Dinv, int* info, hipStream_t s) {
  for (int K0 = 0; K0 < NB; K0 += CPANEL) {
    const int K1 = std::min(NB, K0 + CPANEL);
    for (int K = K0; K < K1; ++K) {
      hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(NT), 0, s, NB, K, A, Dinv, info);
      GN_CHECK_LAUNCH();
      const int m = NB - K - 1;
      if (m > 0) {
        hipLaunchKernelGGL(k_trsm_tile, dim3(m), dim3(NT), 0, s, NB, K, A, Dinv);
        GN_CHECK_LAUNCH();
      }
      if (K + 1 < K1) {
        const int64_t nt = trapezoid_tiles(NB, K + 1, K1);
        hipLaunchKernelGGL(k_syrk_panel, dim3((unsigned)nt), dim3(NT), 0, s, NB, K, K + 1, K + 1, K1, A);
        GN_CHECK_LAUNCH();
      }
    }
    if (K1 < NB) {
      const unsigned nb2 = (unsigned)((NB - K1 + 1) / 2);
      hipLaunchKernelGGL(k_syrk_panel2, dim3(nb2, nb2), dim3(NT), 0, s, NB, K0, K1, K1, A);
      GN_CHECK_LAUNCH();
    }
  }
}

// Z = L^-1 by block rows in panels of CPANEL: each row of the panel is
// finished (k_trinv_row) and passed to the panel's later rows
// (k_trinv_update restricted to them); then one k_trinv_panel2 launch adds the
// panel's rows to the running sums of every later row.
void tri_inv(int NB, const double* L, const double* Dinv, double* Z, hipStream_t s) {
  GN_HIP(hipMemsetAsync(Z, 0, sizeof(double) * (size_t)NB * NB * TILE2, s));
  for (int K0 = 0; K0 < NB; K0 += CPANEL) {
    const int K1 = std::min(NB, K0 + CPANEL);
    for (int K = K0; K < K1; ++K) {
      hipLaunchKernelGGL(k_trinv_row, dim3(K + 1), dim3(NT), 0, s, NB, K, Dinv, Z);
      GN_CHECK_LAUNCH();
      if (K + 1 < K1) {
        hipLaunchKernelGGL(k_trinv_update, dim3((K1 - K - 1) * (K + 1)), dim3(NT), 0, s, NB, K, L, Z);
        GN_CHECK_LAUNCH();
      }
    }
    if (K1 < NB) {
      hipLaunchKernelGGL(k_trinv_panel2, dim3((unsigned)((K1 + 1) / 2), (unsigned)((NB - K1 + 1) / 2)), dim3(NT), 0,
                         s, NB, K0, K1, K1, L, Z);
      GN_CHECK_LAUNCH();
    }
  }
}

}  // namespace gnk
