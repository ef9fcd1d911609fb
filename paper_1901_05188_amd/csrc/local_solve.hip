// Local solves of the two-level additive Schwarz preconditioner: the
// sum_j R_j^T A_j^-1 R_j r of M^-1 r (Section 3.1, eqn:onelevelAS) and the
// coarse restriction (R_H r)_i = Phi_i^T r (Section 3.3.3), one workgroup per
// subdomain: k_local_solve_pf gathers r on the subdomain's node box (R_j is a
// box gather in the structured numbering), forms Phi_j^T r_j, and runs the
// forward and backward banded triangular solves with the subdomain vector held
// in LDS.  Bands too wide for its register pipeline go through the
// multi-column kernels of multi.hip with one live column.
#include <array>
#include <map>
#include <mutex>

#include "gn_internal.h"

namespace {

constexpr int NT = 256;


// The offset `off`, made to depend on `v`: loads addressed with the result are
// issued after v is computed.  It keeps a register buffer's reload behind the
// products that read the buffer's old contents; without it the reload is
// scheduled first, the old values are copied out, and each copy waits for
// every load still in flight (the memory counter retires in order), which
// leaves a single block row in flight instead of two.  The asm is empty.
__device__ inline unsigned gn_after(unsigned off, double v) {
  asm volatile("" : "+v"(off) : "v"(v));
  return off;
}

// v[l % 32] + v[32 + l % 32] in every lane l of the wave (the sum of lanes l and
// l ^ 32, bit for bit the same in both): two lane swaps between the halves of
// the wave, without the LDS crossbar that a general shuffle uses.
__device__ inline double gn_add_halves(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double lower = __builtin_bit_cast(double, ((unsigned long long)h[0] << 32) | l[0]);
  const double upper = __builtin_bit_cast(double, ((unsigned long long)h[1] << 32) | l[1]);
  return lower + upper;
}

// Barrier that orders LDS traffic only: outstanding global loads (the prefetch of
// the next block row) stay in flight across it.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Banded forward/backward solves, one subdomain per workgroup.  Thread (i, gq) owns, in every block row,
// the 4w band entries of row i in columns 4gq..4gq+3 of each off-diagonal tile
// (forward) or rows 4gq..4gq+3 of column i (backward), plus 4 entries of the
// inverse diagonal tile; the next block row's entries are loaded into registers
// while the current one is reduced, and only LDS-ordering barriers separate the
// steps.  The subdomain vector lives in LDS with w zero tiles of padding on both
// sides, so no step needs a bounds branch.  SP >= 2w register slots per buffer.
//
// Stored tiles hold exact zeros outside the band (row r, column c with
// r - c > bw) and in the upper triangle of each inverse diagonal tile.  A load
// that would only fetch such a zero is redirected: tiles wholly outside the
// matrix (the first w block rows of the forward band, the last w of the
// backward one) to the shared zero tile Z0, and single entries outside the
// band or the triangle to one fixed entry of the same tile that is itself
// zero whenever any entry of the tile is.  The products are unchanged bit for
// bit (each redirected load still reads 0), and the cache lines that hold
// nothing but zeros are never fetched.
template <typename FT, int NC, int SP, int G>
__global__ __launch_bounds__(32 * G) void k_local_solve_pf(const SubDesc* __restrict__ subs, int NX, int NY,
                                                           const double* __restrict__ r, const FT* __restrict__ T,
                                                           const FT* __restrict__ D, const FT* __restrict__ TBk,
                                                           double* __restrict__ tvec,
                                                           const double* __restrict__ Phi, double* __restrict__ g,
                                                           const double* __restrict__ done, int padw,
                                                           const FT* __restrict__ Z0) {
  constexpr int NT = 32 * G;      // threads: 32 rows x G column groups
  constexpr int CW = TILE / G;    // columns (forward) / rows (backward) per group
  extern __shared__ double smem[];
  __shared__ double red[G][TILE + 1];
  __shared__ double red2[G][TILE + 1];
  if (done && *done != 0.0) return;
  const SubDesc& sd = subs[blockIdx.x];
  const int NB = sd.NBI, w = sd.wI;
  const int npad = NB * TILE;
  double* vec = smem + padw * TILE;
  for (int e = threadIdx.x; e < padw * TILE; e += NT) {
    smem[e] = 0.0;
    vec[npad + e] = 0.0;
  }
  for (int row = threadIdx.x; row < npad; row += NT) {
    double v = 0.0;
    if (row < sd.nI) {
      int gn[3];
      box_global_node(sd.ilo, sd.in_, sd.permI, row / NC, gn);
      int64_t node = gn[0] + (int64_t)NX * (gn[1] + (int64_t)NY * gn[2]);
      v = r[node * NC + row % NC];
    }
    vec[row] = v;
  }
  __syncthreads();
  if (Phi && sd.m > 0) {
    const double* ph = Phi + sd.offPhi;
    for (int k0 = 0; k0 < sd.m; k0 += 8) {
      double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int row = threadIdx.x; row < sd.nI; row += NT) {
        double v = vec[row];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (k0 + q < sd.m) acc[q] += ph[(int64_t)row * sd.m + k0 + q] * v;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        double s = block_sum(acc[q], &red[0][0]);
        if (threadIdx.x == 0 && k0 + q < sd.m) g[sd.coff + k0 + q] = s;
      }
    }
    __syncthreads();
  }
  const int i = threadIdx.x % TILE, gq = threadIdx.x / TILE;
  const FT* Tb = T + sd.offTI * TILE2;
  const FT* Db = D + sd.offDI * TILE2;
  const int ns = CW * w;
  // zero-entry redirection (see above): the entry (row, column) of a tile sits
  // at column * TILE + row; ZR = (TILE - 1, 0), ZC = (0, TILE - 1)
  constexpr unsigned ZR = TILE - 1, ZC = (TILE - 1) * TILE;
  const int ic = i - CW * gq;          // row minus the thread's first column (row) in a tile
  const int bw = sd.bwI;
  // Two register buffers: block row K is consumed from one while the loads of
  // rows K+1 (other buffer, issued one step earlier) and K+2 (this buffer,
  // issued right after the consumption) are in flight.
  FT lv0[SP], lv1[SP], dn0[CW], dn1[CW];
  // Slots u < CW*w address band entries; the rest read a shared zero tile, so
  // every load is unconditional and the unrolled loops carry no branches.
  // ---- forward ----
  // every slot address is a uniform tile pointer plus the thread's 32-bit offset
  // inside the tile (one offset register for all slots)
  const unsigned toff = (unsigned)((CW * gq) * TILE + i);
  // forward tile t of block row K is L(K, K - w + t); its entry (i, c) lies
  // outside the band when 32 (w - t) + i - c > bw, possible for t <= 1 only
  // (32 w - bw < 32)
#define GN_LOAD_FWD_LV(K_, LV, OFF)                                                      \
  {                                                                                      \
    const int Kl = (K_);                                                                 \
    const FT* rowp = Tb + (int64_t)Kl * (w + 1) * TILE2;                                 \
    _Pragma("unroll") for (int u = 0; u < SP; ++u) {                                     \
      const int t = u / CW, q = u % CW;                                                  \
      const FT* tp = (u < ns && Kl - w + t >= 0) ? rowp + t * TILE2 : Z0;                \
      unsigned o = (OFF) + (unsigned)(q * TILE);                                         \
      if (t <= 1) o = (ic - q > bw - TILE * (w - t)) ? ZR : o;                           \
      LV[u] = tp[o];                                                                     \
    }                                                                                    \
  }
#define GN_LOAD_FWD_DN(K_, DN, OFF)                                                      \
  {                                                                                      \
    const FT* dk = Db + (int64_t)(K_) * TILE2;                                           \
    _Pragma("unroll") for (int q = 0; q < CW; ++q)                                       \
      DN[q] = dk[(q > ic) ? ZC : (OFF) + (unsigned)(q * TILE)];                          \
  }
#define GN_STEP_FWD(K_, LV, DN)                                                          \
  {                                                                                      \
    const int KK = (K_);                                                                 \
    const double* yw = vec + (KK - w) * TILE + CW * gq;                                  \
    double acc = 0.0;                                                                    \
    _Pragma("unroll") for (int u = 0; u < SP; ++u)                                       \
      acc += (double)LV[u] * yw[(u / CW) * TILE + (u % CW)];                             \
    const unsigned toffA = gn_after(toff, acc);                                          \
    GN_LOAD_FWD_LV(min(KK + 2, NB - 1), LV, toffA)                                       \
    acc = gn_add_halves(acc);   /* the wave's two column groups, same row */             \
    if ((threadIdx.x & 63) < 32) red[gq >> 1][i] = acc;                                  \
    lds_barrier();                                                                       \
    double part = 0.0;                                                                   \
    _Pragma("unroll") for (int q = 0; q < CW; ++q) {                                     \
      int c = CW * gq + q;                                                               \
      double sv = vec[KK * TILE + c];                                                    \
      _Pragma("unroll") for (int g2 = 0; g2 < G / 2; ++g2) sv -= red[g2][c];             \
      part += (double)DN[q] * sv;                                                        \
    }                                                                                    \
    const unsigned toffP = gn_after(toff, part);                                         \
    GN_LOAD_FWD_DN(min(KK + 2, NB - 1), DN, toffP)                                       \
    part = gn_add_halves(part);                                                          \
    if ((threadIdx.x & 63) < 32) red2[gq >> 1][i] = part;                                \
    lds_barrier();                                                                       \
    if (gq == 0) {                                                                       \
      double y = 0.0;                                                                    \
      _Pragma("unroll") for (int g2 = 0; g2 < G / 2; ++g2) y += red2[g2][i];             \
      vec[KK * TILE + i] = y;                                                            \
    }                                                                                    \
    lds_barrier();                                                                       \
  }
  GN_LOAD_FWD_LV(0, lv0, toff)
  GN_LOAD_FWD_DN(0, dn0, toff)
  GN_LOAD_FWD_LV(min(1, NB - 1), lv1, toff)
  GN_LOAD_FWD_DN(min(1, NB - 1), dn1, toff)
  // the scheduler may issue the two prologue groups interleaved; draining them
  // here keeps the waits inside the loop at their steady-state depth (row K's
  // loads done, row K+1's still in flight) instead of the prologue's order
  __builtin_amdgcn_s_waitcnt(0);
  // pairs of rows in the loop and an odd last row after it, so that every path
  // into the loop header has the same loads in flight
  int K = 0;
  for (; K + 1 < NB; K += 2) {
    GN_STEP_FWD(K, lv0, dn0)
    GN_STEP_FWD(K + 1, lv1, dn1)
  }
  if (K < NB) GN_STEP_FWD(K, lv0, dn0)
#undef GN_STEP_FWD
#undef GN_LOAD_FWD_LV
#undef GN_LOAD_FWD_DN
  // ---- backward ----
  // backward block row K: tile d-1 of row K of the transposed band holds
  // L(K+d, K)^T (entry (i, rr) = L(K+d, K)(rr, i)) and tile w holds D_K^T
  const FT* TBb = TBk + sd.offTI * TILE2;
  // backward tile t holds L(K + t + 1, K)^T: its entry (i, rr) is
  // L(K + t + 1, K)(rr, i), outside the band when 32 (t + 1) + rr - i > bw
#define GN_LOAD_BWD_LV(K_, LV, OFF)                                                      \
  {                                                                                      \
    const int Kl = (K_);                                                                 \
    const FT* rowp = TBb + (int64_t)Kl * (w + 1) * TILE2;                                \
    _Pragma("unroll") for (int u = 0; u < SP; ++u) {                                     \
      const int t = u / CW, q = u % CW;                                                  \
      const FT* tp = (u < ns && Kl + t + 1 < NB) ? rowp + t * TILE2 : Z0;                \
      unsigned o = (OFF) + (unsigned)(q * TILE);                                         \
      o = (q - ic > bw - TILE * (t + 1)) ? ZC : o;                                       \
      LV[u] = tp[o];                                                                     \
    }                                                                                    \
  }
#define GN_LOAD_BWD_DN(K_, DN, OFF)                                                      \
  {                                                                                      \
    const FT* dk = TBb + ((int64_t)(K_) * (w + 1) + w) * TILE2;                          \
    _Pragma("unroll") for (int q = 0; q < CW; ++q)                                       \
      DN[q] = dk[(q < ic) ? ZR : (OFF) + (unsigned)(q * TILE)];                          \
  }
#define GN_STEP_BWD(K_, LV, DN)                                                          \
  {                                                                                      \
    const int KK = (K_);                                                                 \
    const double* xw = vec + (KK + 1) * TILE + CW * gq;                                  \
    double acc = 0.0;                                                                    \
    _Pragma("unroll") for (int u = 0; u < SP; ++u)                                       \
      acc += (double)LV[u] * xw[(u / CW) * TILE + (u % CW)];                             \
    const unsigned toffA = gn_after(toff, acc);                                          \
    GN_LOAD_BWD_LV(max(KK - 2, 0), LV, toffA)                                            \
    acc = gn_add_halves(acc);   /* the wave's two column groups, same row */             \
    if ((threadIdx.x & 63) < 32) red[gq >> 1][i] = acc;                                  \
    lds_barrier();                                                                       \
    double part = 0.0;                                                                   \
    _Pragma("unroll") for (int q = 0; q < CW; ++q) {                                     \
      int rr = CW * gq + q;                                                              \
      double sv = vec[KK * TILE + rr];                                                   \
      _Pragma("unroll") for (int g2 = 0; g2 < G / 2; ++g2) sv -= red[g2][rr];            \
      part += (double)DN[q] * sv;                                                        \
    }                                                                                    \
    const unsigned toffP = gn_after(toff, part);                                         \
    GN_LOAD_BWD_DN(max(KK - 2, 0), DN, toffP)                                            \
    part = gn_add_halves(part);                                                          \
    if ((threadIdx.x & 63) < 32) red2[gq >> 1][i] = part;                                \
    lds_barrier();                                                                       \
    if (gq == 0) {                                                                       \
      double x = 0.0;                                                                    \
      _Pragma("unroll") for (int g2 = 0; g2 < G / 2; ++g2) x += red2[g2][i];             \
      vec[KK * TILE + i] = x;                                                            \
    }                                                                                    \
    lds_barrier();                                                                       \
  }
  GN_LOAD_BWD_LV(NB - 1, lv0, toff)
  GN_LOAD_BWD_DN(NB - 1, dn0, toff)
  GN_LOAD_BWD_LV(max(NB - 2, 0), lv1, toff)
  GN_LOAD_BWD_DN(max(NB - 2, 0), dn1, toff)
  __builtin_amdgcn_s_waitcnt(0);
  K = NB - 1;
  for (; K >= 1; K -= 2) {
    GN_STEP_BWD(K, lv0, dn0)
    GN_STEP_BWD(K - 1, lv1, dn1)
  }
  if (K >= 0) GN_STEP_BWD(K, lv0, dn0)
#undef GN_STEP_BWD
#undef GN_LOAD_BWD_LV
#undef GN_LOAD_BWD_DN
  __syncthreads();
  double* out = tvec + sd.offVI;
  for (int row = threadIdx.x; row < npad; row += NT) out[row] = vec[row];
}

}  // namespace

namespace gnk {

namespace {
// Launch shapes of the single-column sweep: G column groups of TILE / G
// columns; 512 threads (G = 16, two columns per thread and tile) or 1024 (G =
// 32, one column).  A shape holds sp = (TILE / G) w register slots per buffer,
// rounded up to an instantiated count.  Slot limits without spills (compiler
// resource reports): G = 16: 44 (FP64: 252 registers at 44); G = 32: 24 (FP64,
// 128 registers) or 32 (FP32).
struct PfShape {
  int G, sp, padw;
  bool ok;
};
int pf_slots(int sp) {
  return sp <= 8 ? 8 : sp <= 12 ? 12 : sp <= 16 ? 16 : sp <= 20 ? 20 : sp <= 24 ? 24 : sp <= 32 ? 32 : sp <= 40 ? 40 : 44;
}
std::vector<PfShape> pf_candidates(const gn_precond* pc) {
  std::vector<PfShape> out;
  for (int G : {16, 32}) {
    const int spmax = G == 16 ? 44 : (pc->local_prec == 32 ? 32 : 24);
    const int sp = (TILE / G) * pc->maxwI;
    if (sp > spmax) continue;
    const int spt = pf_slots(sp);
    // zero tiles on both sides of the LDS vector cover every window read: the
    // forward window starts w tiles before the row, the reads of the unused
    // slots reach spt / (TILE / G) tiles past it
    const int padw = pc->maxwI + spt / (TILE / G) + 1;
    const int stat = 2 * G * (TILE + 1);     // doubles of the static reduction arrays
    if ((pc->maxNBI + 2 * padw) * TILE + stat > 20 * 1024 - 64) continue;
    out.push_back(PfShape{G, sp, padw, true});
  }
  return out;
}
PfShape pf_shape(const gn_precond* pc) {
  if (pc->local_kernel == 1) return PfShape{16, 0, 0, false};
  if (pc->pf_G > 0) return PfShape{pc->pf_G, pc->pf_sp, pc->pf_padw, true};
  const std::vector<PfShape> c = pf_candidates(pc);
  return c.empty() ? PfShape{16, 0, 0, false} : c.front();
}

void launch_pf(const gn_problem* p, const gn_precond* pc, const PfShape& sh, const double* r, const double* done,
               hipStream_t s) {
  const bool f32 = pc->local_prec == 32;
  const double* Phi = pc->NH > 0 ? pc->d_Phi : nullptr;
  if (!pc->d_LIb) throw gn_error{GN_ERR_ARG, "backward band missing for the single-column sweep"};
  const int need_sp = sh.sp, padw = sh.padw;
  const size_t dynpf = (size_t)(pc->maxNBI + 2 * padw) * TILE * sizeof(double);
#define GN_PF(FT, NC, SPV, GV)                                                                    \
  do {                                                                                            \
    auto kfn = k_local_solve_pf<FT, NC, SPV, GV>;                                                 \
    GN_HIP(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize,      \
                               (int)dynpf));                                                      \
    hipLaunchKernelGGL(kfn, dim3(pc->n_sub), dim3(32 * GV), dynpf, s, pc->d_subxI, p->nn[0],       \
                       p->nn[1], r,                                                               \
                       (const FT*)(f32 ? (const void*)pc->d_LIf : (const void*)pc->d_LI),         \
                       (const FT*)(f32 ? (const void*)pc->d_DIf : (const void*)pc->d_DI),         \
                       (const FT*)pc->d_LIb, pc->d_t, Phi, pc->d_g, done, padw,                   \
                       (const FT*)(f32 ? (const void*)pc->d_zf : (const void*)pc->d_z0));         \
  } while (0)
#define GN_PF_SP16(FT, NC)                                \
  do {                                                    \
    if (need_sp <= 8) GN_PF(FT, NC, 8, 16);               \
    else if (need_sp <= 12) GN_PF(FT, NC, 12, 16);        \
    else if (need_sp <= 16) GN_PF(FT, NC, 16, 16);        \
    else if (need_sp <= 20) GN_PF(FT, NC, 20, 16);        \
    else if (need_sp <= 24) GN_PF(FT, NC, 24, 16);        \
    else if (need_sp <= 32) GN_PF(FT, NC, 32, 16);        \
    else if (need_sp <= 40) GN_PF(FT, NC, 40, 16);        \
    else GN_PF(FT, NC, 44, 16);                           \
  } while (0)
#define GN_PF_SP32(FT, NC)                                \
  do {                                                    \
    if (need_sp <= 8) GN_PF(FT, NC, 8, 32);               \
    else if (need_sp <= 12) GN_PF(FT, NC, 12, 32);        \
    else if (need_sp <= 16) GN_PF(FT, NC, 16, 32);        \
    else if (need_sp <= 20) GN_PF(FT, NC, 20, 32);        \
    else if (need_sp <= 24) GN_PF(FT, NC, 24, 32);        \
    else GN_PF(FT, NC, 32, 32);                           \
  } while (0)
#define GN_PF_G(FT, NC)                                   \
  do {                                                    \
    if (sh.G == 16) GN_PF_SP16(FT, NC);                   \
    else GN_PF_SP32(FT, NC);                              \
  } while (0)
  if (f32) {
    if (p->nc == 3) GN_PF_G(float, 3); else GN_PF_G(float, 1);
  } else {
    if (p->nc == 3) GN_PF_G(double, 3); else GN_PF_G(double, 1);
  }
#undef GN_PF_G
#undef GN_PF_SP32
#undef GN_PF_SP16
#undef GN_PF
  GN_CHECK_LAUNCH();
}

// Shapes chosen per process for a band shape (components, precision, band
// width, largest subdomain): every later preconditioner of that shape takes
// the same kernel, so its applications are bit-for-bit repeatable.
std::mutex g_tune_mu;
std::map<std::array<int, 4>, std::pair<int, int>> g_tune;   // key -> (G, sp)
}  // namespace

// Autotuner of the single-column sweep: when more than one shape fits the
// band, each is timed on this preconditioner's own factors (one warm-up
// launch, then the shortest of four launches timed one by one with HIP events
// on the set-up stream) and the fastest kept.
void local_solve_tune(const gn_problem* p, gn_precond* pc, hipStream_t s) {
  pc->pf_G = 0;
  if (pc->local_kernel == 1) return;
  std::vector<PfShape> cand = pf_candidates(pc);
  if (pc->local_kernel >= 3) {
    // a fixed launch shape: 512 (G = 16) or 1024 (G = 32) threads
    const int G = pc->local_kernel == 3 ? 16 : 32;
    std::vector<PfShape> keep;
    for (const PfShape& c : cand)
      if (c.G == G) keep.push_back(c);
    if (keep.empty())
      throw gn_error{GN_ERR_ARG, "local band does not fit the " + std::to_string(32 * G) +
                                     "-thread single-column sweep (local_kernel " +
                                     std::to_string(pc->local_kernel) + ")"};
    pc->pf_G = keep.front().G;
    pc->pf_sp = keep.front().sp;
    pc->pf_padw = keep.front().padw;
    return;
  }
  if (cand.empty()) return;
  const std::array<int, 4> key{p->nc, pc->local_prec, pc->maxwI, pc->maxNBI};
  PfShape best = cand.front();
  bool cached = false;
  if (pc->local_kernel == 0) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      for (const PfShape& c : cand)
        if (c.G == it->second.first) best = c;
      cached = true;
    }
  }
  if (!cached && cand.size() > 1 && pc->local_kernel == 0) {
    hipEvent_t e0, e1;
    GN_HIP(hipEventCreate(&e0));
    GN_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    for (const PfShape& c : cand) {
      launch_pf(p, pc, c, p->d_r, nullptr, s);
      float ms = 1e30f;
      for (int k = 0; k < 4; ++k) {
        GN_HIP(hipEventRecord(e0, s));
        launch_pf(p, pc, c, p->d_r, nullptr, s);
        GN_HIP(hipEventRecord(e1, s));
        GN_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        GN_HIP(hipEventElapsedTime(&t, e0, e1));
        ms = std::min(ms, t);
      }
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = {best.G, best.sp};
  }
  pc->pf_G = best.G;
  pc->pf_sp = best.sp;
  pc->pf_padw = best.padw;
}

void local_solve(const gn_problem* p, const gn_precond* pc, const double* r, const double* done,
                 hipStream_t s) {
  GnProfScope prof(PROF_TRSV, pc->trsv_bytes, s);
  const PfShape sh = pf_shape(pc);
  if (!sh.ok) throw gn_error{GN_ERR_ARG, "local band too wide for the single-column sweep kernel"};
  launch_pf(p, pc, sh, r, done, s);
}

bool pf_supported(const gn_problem* p, const gn_precond* pc) {
  (void)p;
  return pf_shape(pc).ok;
}


}  // namespace gnk
