// Internal declarations shared by the HIP translation units of libgenpcg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include <string>
#include <vector>

#include "genpcg.h"

// Band tiles are TILE x TILE, column-major inside a tile.
#define TILE 32
#define TILE2 (TILE * TILE)

// ---------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------
struct gn_error {
  gn_status code;
  std::string msg;
};
void gn_set_error(gn_status code, const std::string& msg);

#define GN_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw gn_error{e_ == hipErrorOutOfMemory ? GN_ERR_OOM : GN_ERR_DEVICE,          \
                     std::string(#call) + ": " + hipGetErrorString(e_)};              \
  } while (0)

#define GN_CHECK_LAUNCH() GN_HIP(hipGetLastError())

// device-resident CG scalars and the recurrence steps of the single-block finalize kernel;
// S_RTOL is the relative tolerance of a batched column (0: the launch argument)
// S_RZN holds z.r of the new residual while the flexible (Polak-Ribiere) beta
// waits for z.q
enum { S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_BB, S_TOL2, S_DONE, S_ITER, S_MAXIT, S_BREAK, S_RTOL, S_RZN, S_N };
enum { OP_BB = 0, OP_RZ0, OP_ALPHA, OP_RR, OP_BETA, OP_RESTART, OP_RZN, OP_BETAF };

// ---------------------------------------------------------------------------
// per-subdomain description (plain data, mirrored on the device)
// ---------------------------------------------------------------------------
struct SubDesc {
  int elo[3], ehi[3];   // element box of Omega_j: [elo, ehi)
  int ilo[3], in_[3];   // node box of V_h0(Omega_j) (local Dirichlet system): first node, count
  int blo[3], bn[3];    // node box of V_h(Omega_j) (pencil): first node, count
  int permI[3];         // axis order of the local numbering on the I box (perm[0] fastest)
  int permB[3];         // axis order on the Ibar box
  int nI, nB;           // DOFs of the boxes (nodes * ncomp)
  int NBI, wI;          // tile rows and band width in tiles, local system
  int NBB, wB;          // same for the pencil
  int64_t offTI, offTB; // offsets (in tiles) into the band storage
  int64_t offDI, offDB; // offsets (in tiles) into the inverse-diagonal storage
  int64_t offVI, offVB; // offsets (in doubles) into per-subdomain vector storage (padded)
  int m;                // number of coarse vectors
  int coff;             // first coarse index i(j, 0)
  int64_t offPhi;       // offset (doubles) of Phi_j (NBI*TILE rows x m, row-major)
  int bwI, bwB;         // half bandwidth in DOFs of the local matrix and of the pencil
  int id;               // index j of the subdomain (the reordered copies keep it)
};

// one nonzero block (A_H)_{j1,j2} of the block-sparse coarse matrix: m_j1 x m_j2
// values, row-major, at `off`
struct BsrBlock {
  int j1, j2;
  int64_t off;
};

// local DOF index <-> global node on a box with an axis permutation
__host__ __device__ inline int box_local_node(const int lo[3], const int n[3], const int perm[3],
                                              int gi, int gj, int gk) {
  int g[3] = {gi - lo[0], gj - lo[1], gk - lo[2]};
  return g[perm[0]] + n[perm[0]] * (g[perm[1]] + n[perm[1]] * g[perm[2]]);
}
__host__ __device__ inline void box_global_node(const int lo[3], const int n[3], const int perm[3],
                                                int local, int* gijk) {
  int u0 = local % n[perm[0]];
  int t = local / n[perm[0]];
  int u1 = t % n[perm[1]];
  int u2 = t / n[perm[1]];
  int g[3];
  g[perm[0]] = u0;
  g[perm[1]] = u1;
  g[perm[2]] = u2;
  gijk[0] = g[0] + lo[0];
  gijk[1] = g[1] + lo[1];
  gijk[2] = g[2] + lo[2];
}

// ---------------------------------------------------------------------------
// partition of unity X_j (Section 3.2, def:pou; Section 3.3.1)
// ---------------------------------------------------------------------------
// Per-axis tables of the tensor-product decomposition: for node index i along
// axis a, cnt[a][i] parts hold i in their I range, the first being plo[a][i];
// ecnt[a][e] parts hold element e in their element range; er0/er1[a][q] is
// the element range [er0, er1) of part q (overlap included).
struct PouDev {
  const int* cnt[3];
  const int* plo[3];
  const int* ecnt[3];
  const int* er0[3];
  const int* er1[3];
  int ne[3];
  int kind;   // 0: one over the number of subdomains; 1: smooth (distance-weighted)
};

// Element layers between node index i and the artificial ends of the element
// range [e0, e1) along one axis (ends on the physical boundary do not count).
__host__ __device__ inline int pou_dist(int i, int e0, int e1, int ne) {
  int d = 1 << 28;
  if (e0 > 0) d = i - e0 < d ? i - e0 : d;
  if (e1 < ne) d = e1 - i < d ? e1 - i : d;
  return d > 0 ? d : 0;
}

// X_j at DOF c of node (gi, gj, gk): zero off the I box of subdomain sd and on
// Dirichlet DOFs.  kind 0 gives 1 / #{subdomains whose I box holds the node};
// kind 1 weights subdomain j by the distance of the node to the artificial
// boundary of Omega_j (in element layers, the smallest over the box's
// artificial faces) and divides by the sum of those weights over all
// subdomains, so the weights fall linearly to zero across each overlap.  The
// weights are small integers, so the sums are exact.
__device__ inline double pou_x(const SubDesc& sd, const PouDev& pa, const uint8_t* dir, int NX, int NY,
                               int NC, int gi, int gj, int gk, int c) {
  if (gi < sd.ilo[0] || gi >= sd.ilo[0] + sd.in_[0] || gj < sd.ilo[1] || gj >= sd.ilo[1] + sd.in_[1] ||
      gk < sd.ilo[2] || gk >= sd.ilo[2] + sd.in_[2])
    return 0.0;
  const int64_t node = gi + (int64_t)NX * (gj + (int64_t)NY * gk);
  if (dir[node * NC + c]) return 0.0;
  if (pa.kind == 0) return 1.0 / (double)(pa.cnt[0][gi] * pa.cnt[1][gj] * pa.cnt[2][gk]);
  const int g[3] = {gi, gj, gk};
  int wj = 1 << 28;
  for (int a = 0; a < 3; ++a) {
    const int d = pou_dist(g[a], sd.elo[a], sd.ehi[a], pa.ne[a]);
    wj = d < wj ? d : wj;
  }
  double sum = 0.0;
  for (int q2 = pa.plo[2][gk]; q2 < pa.plo[2][gk] + pa.cnt[2][gk]; ++q2)
    for (int q1 = pa.plo[1][gj]; q1 < pa.plo[1][gj] + pa.cnt[1][gj]; ++q1)
      for (int q0 = pa.plo[0][gi]; q0 < pa.plo[0][gi] + pa.cnt[0][gi]; ++q0) {
        const int q[3] = {q0, q1, q2};
        int wk = 1 << 28;
        for (int a = 0; a < 3; ++a) {
          const int d = pou_dist(g[a], pa.er0[a][q[a]], pa.er1[a][q[a]], pa.ne[a]);
          wk = d < wk ? d : wk;
        }
        sum += (double)wk;
      }
  return sum > 0.0 ? (double)wj / sum : 0.0;
}

// element e lies in at least two subdomains (Omega_j^o for each subdomain holding it)
__device__ inline bool pou_overlap_elem(const PouDev& pa, int ex, int ey, int ez) {
  return pa.ecnt[0][ex] * pa.ecnt[1][ey] * pa.ecnt[2][ez] >= 2;
}

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
// One chunk of CG iterations (check_every of them) captured as a HIP graph and
// replayed by every later solve with the same chunk length and history buffer;
// every kernel of the chunk reads its scalars from device memory, so the graph
// holds no per-solve values.
struct ChunkGraph {
  hipGraphExec_t exec = nullptr;
  int chunk = 0;
  int flexible = 0;
  const double* hist = nullptr;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
};

struct gn_problem {
  int pde = 0, nc = 1;
  int ne[3] = {0, 0, 0}, nn[3] = {0, 0, 0};
  int64_t n_node = 0, n_elem = 0, n_dof = 0, n_free = 0;
  int nrhs = 1;
  int map_kind = 0;
  double map_par[3] = {0, 0, 0};
  double* d_xn[3] = {nullptr, nullptr, nullptr};
  double* d_Ke = nullptr;      // element matrices, n_elem x nd x nd (row-major)
  double* d_A = nullptr;       // node-block matrix, [27][nc][nc][n_node]
  double* d_b = nullptr;       // load, full numbering, n_dof x nrhs
  uint8_t* d_dir = nullptr;    // Dirichlet mask, full numbering
  std::vector<uint8_t> h_dir;  // the same mask on the host
  int* d_free2full = nullptr;  // n_free
  // the assembly's inputs, kept on the device for gn_reassemble (null where absent)
  int n_mat = 0;
  const double *d_mats = nullptr, *d_eang = nullptr, *d_etilt = nullptr, *d_ek = nullptr;
  const int* d_emat = nullptr;
  const double *d_body = nullptr, *d_trac = nullptr;
  // CG workspace (full numbering)
  double *d_x = nullptr, *d_r = nullptr, *d_p = nullptr, *d_q = nullptr, *d_z = nullptr;
  double* d_part = nullptr;    // block partial sums
  double* d_scal = nullptr;    // device scalars
  double* d_hist = nullptr;    // alpha/beta history
  int hist_cap = 0;
  unsigned* d_count = nullptr; // counter of the input checks
  // batched (multi-RHS) CG workspace: 16 columns of each vector, per-column
  // partial sums, scalars and alpha/beta history
  double *d_Xm = nullptr, *d_Rm = nullptr, *d_Pm = nullptr, *d_Qm = nullptr, *d_Zm = nullptr;
  double *d_partm = nullptr, *d_scalm = nullptr, *d_histm = nullptr;
  int histm_stride = 0, pstride_m = 0;
  ChunkGraph cg;               // plain-CG chunk graph
  std::vector<void*> owned;
};

struct gn_precond {
  gn_problem* prob = nullptr;
  int n_sub = 0, nparts[3] = {1, 1, 1}, overlap = 1;
  std::vector<int> cuts[3];
  std::vector<SubDesc> sub;
  SubDesc* d_sub = nullptr;
  // The same descriptors in the launch order of the one-workgroup-per-subdomain
  // band sweeps.  Workgroup q of a launch runs on XCD q mod 8 (each XCD with its
  // own L2 and share of the memory fabric), and a subdomain's sweep costs about
  // its band tile count; the natural order maps one partition column (the
  // fastest subdomain index) to each XCD, so the XCDs holding the interior
  // columns carry up to 1.4x the tiles of those holding the boundary columns.
  // xI spreads the local bands evenly over the XCDs, xB the pencil bands.
  std::vector<int> xorderI, xorderB;
  std::vector<SubDesc> subxI, subxB;
  SubDesc* d_subxI = nullptr;
  SubDesc* d_subxB = nullptr;
  int local_prec = 64;
  int local_kernel = 0;        // 0 tuned, 1 batched matrix-core kernel for single columns, 2 fixed rule
  int pf_G = 0, pf_sp = 0, pf_padw = 0;   // launch shape of the single-column sweep (0: not set)
  // per-axis node coverage (PoU counts) and part ranges for the gather-form prolongation
  int* d_cnt[3] = {nullptr, nullptr, nullptr};   // #parts whose I-range holds node index
  int* d_plo[3] = {nullptr, nullptr, nullptr};   // first such part
  int* d_ecnt[3] = {nullptr, nullptr, nullptr};  // #parts whose element range holds element
  int* d_er0[3] = {nullptr, nullptr, nullptr};   // element range [er0, er1) of each part
  int* d_er1[3] = {nullptr, nullptr, nullptr};
  int pou = 0;                                   // 0 standard, 1 smooth partition of unity
  // local factors
  double* d_LI = nullptr;    // band tiles (FP64) or nullptr
  float* d_LIf = nullptr;    // band tiles (FP32) or nullptr
  double* d_DI = nullptr;    // inverse diagonal tiles (FP64)
  float* d_DIf = nullptr;
  void* d_LIb = nullptr;     // backward band of the single-column sweep (FP64 or FP32), or nullptr
  double* d_t = nullptr;     // local vectors (sum of NBI*TILE)
  int64_t tilesI = 0, vecI = 0;
  // coarse
  int NH = 0;
  double* d_Phi = nullptr;   // concatenated Phi_j
  int64_t phi_len = 0;
  double* d_g = nullptr;     // coarse vectors (NH padded)
  double* d_u = nullptr;
  double* d_y = nullptr;
  int maxNBI = 0, maxwI = 0;
  double* d_z0 = nullptr;    // one zero tile (FP64) read by masked prefetch slots
  float* d_zf = nullptr;     // one zero tile (FP32)
  double trsv_bytes = 0.0, prolong_bytes = 0.0;
  double trsv_tile_bytes = 0.0;  // the same launch counted over whole 32 x 32 band tiles
  double trsv_bytes_mc = 0.0;  // gather + banded solves of one 16-column batch
  double* d_tm = nullptr;      // local vectors of a batch: (offVI + row) * 16 + column
  double *d_gm = nullptr, *d_um = nullptr, *d_ym = nullptr;  // coarse vectors, column * NBH*TILE
  double* d_Z = nullptr;     // L_H^-1 as dense tiles (NBH x NBH tiles): Z(K,J) for J <= K;
                             // the strictly upper tiles (J,K) hold Z(K,J)^T
  double* d_Zdt = nullptr;   // Z(K,K)^T, one tile per K
  int NBH = 0;
  int max_m = 0;             // largest m_j (rows of Phi_j hold m_j coefficients)
  // work units of the coarse products (one workgroup each): {row, first tile,
  // last tile + 1, 0}, row by row; rowstart[R] = first unit of row R
  int4* d_cu_f = nullptr;    // y = Z g: row K, tiles J in [0, K]
  int4* d_cu_b = nullptr;    // y = Z^T u: row J, tiles K in [J, NBH)
  int* d_rs_f = nullptr;
  int* d_rs_b = nullptr;
  int n_cu_f = 0, n_cu_b = 0;
  double* d_zpart = nullptr; // 32 partial sums per unit
  // inexact coarse solve (coarse_solve = 1): A_H block-sparse by subdomain
  // pairs, the inverses of its diagonal blocks, and the inner CG state
  int coarse_solve = 0;
  double coarse_rtol = 1e-4;
  int coarse_maxit = 200;
  int* d_bsr_ptr = nullptr;      // n_sub + 1: blocks of block row j at [ptr[j], ptr[j+1])
  BsrBlock* d_bsr_blk = nullptr; // block row, block column and value offset of each block
  double* d_bsr_val = nullptr;
  int64_t* d_dinv_off = nullptr; // offset of (A_H)_jj^-1 (m_j x m_j, row-major) per subdomain
  double* d_dinv = nullptr;
  double* d_cvec = nullptr;      // inner CG vectors: r, z, p (two buffers), q; NBH*TILE each
  double* d_cpart = nullptr;     // per-workgroup partial sums of the inner CG
  double* d_cstat = nullptr;     // inner iterations of the last applications (diagnostics)
  int coarse_grid = 0;           // workgroups of the cooperative inner CG launch
  int64_t bsr_nnz = 0;
  std::vector<double> lam;   // eigenvalues per subdomain (n_eval each)
  std::vector<int> lam_n;
  int n_eval = 0;
  ChunkGraph cg;               // PCG chunk graph of this preconditioner
  std::vector<void*> owned;
};

// ---------------------------------------------------------------------------
// launch helpers implemented in the kernel translation units
// ---------------------------------------------------------------------------
namespace gnk {
// fem.hip
void element_matrices(gn_problem* p, const double* d_mats, int n_mat, const int* d_emat,
                      const double* d_eang, const double* d_etilt, const double* d_ek,
                      hipStream_t s);
void assemble_matrix(gn_problem* p, hipStream_t s);
void assemble_load(const gn_problem* p, const double* d_body, const double* d_trac, int nrhs, double* d_out,
                   hipStream_t s);
// linalg.hip
void spmv_flag(const gn_problem* p, const double* x, double* y, double* part, const double* done,
               hipStream_t s);
int spmv_blocks(const gn_problem* p);
void absmv_partial(const gn_problem* p, const double* x, double* part, hipStream_t s);
void scatter_free(const gn_problem* p, const double* xf, double* xfull, hipStream_t s);
void gather_free(const gn_problem* p, const double* xfull, double* xf, hipStream_t s);
int reduce_blocks();
int scal_count();
void dot_partial(int64_t n, const double* a, const double* b, double* part, const double* done,
                 hipStream_t s);
void finalize(const double* part, int nb, int op, double* scal, double* hist, double rtol, hipStream_t s);
void update_xr(int64_t n, double* x, double* r, const double* p, const double* q, const double* scal,
               double* part, hipStream_t s);
void update_p(int64_t n, double* p, const double* z, const double* scal, hipStream_t s);
void copy(int64_t n, double* dst, const double* src, const double* done, hipStream_t s);
// NaN / infinite entries of ncol device columns (synchronises the stream)
unsigned count_nonfinite(int64_t n, int ncol, int64_t ld, const double* x, unsigned* d_count, hipStream_t s);
void residual_partial(int64_t n, const double* b, const double* q, double* part, hipStream_t s);
void sub_partial(int64_t n, const double* b, const double* q, double* r, double* part, hipStream_t s);
// band.hip
void extract_local(const gn_problem* p, const gn_precond* pc, double* L, int maxNB, hipStream_t s);
// PE, BE (both or neither): also P and B in node-ELL planes, from sd.offVB 27 nc
void extract_pencil(const gn_problem* p, const gn_precond* pc, double shift, double* L, int maxNB,
                    hipStream_t s, double* PE = nullptr, double* BE = nullptr);
// TB (may be null): also write the transposed band of the backward sweeps
// (the layout of band_transpose, FP64; block rows past the end left unwritten)
// when the row-in-LDS form runs; returns whether TB was written (otherwise
// band_transpose makes it)
bool band_chol(const void* d_refs, int n, int maxw, double* T, double* D, int* info, hipStream_t s,
               double* TB = nullptr);
void to_f32(int64_t n, const double* a, float* b, hipStream_t s);
void band_transpose(const void* d_refs, int n, int maxNB, const double* T, const double* D, void* TB, bool f32,
                    hipStream_t s);
// precond.hip
bool pf_supported(const gn_problem* p, const gn_precond* pc);
void local_solve_tune(const gn_problem* p, gn_precond* pc, hipStream_t s);
void local_solve(const gn_problem* p, const gn_precond* pc, const double* r, const double* done,
                 hipStream_t s);
void coarse_solve(const gn_precond* pc, const double* done, hipStream_t s);
// tiles per work unit of the coarse products, and the units of an NB-tile-row factor
constexpr int COARSE_UNIT_TILES = 64;
inline int64_t coarse_units(int64_t NB, bool upper) {
  int64_t n = 0;
  for (int64_t R = 0; R < NB; ++R) n += ((upper ? NB - R : R + 1) + COARSE_UNIT_TILES - 1) / COARSE_UNIT_TILES;
  return n;
}
// after tri_inv: Z^T into the upper tiles and d_Zdt (d_Zdt allocated)
void z_transpose(gn_precond* pc, hipStream_t s);
// inexact coarse solve: y = (CG on A_H, block-Jacobi) g for one column
void coarse_cg(const gn_precond* pc, const double* g, double* y, const double* done, hipStream_t s);
int coarse_cg_grid(const gn_precond* pc);
void block_inverse(const gn_precond* pc, int* info, hipStream_t s);
void bsr_from_dense(const gn_precond* pc, const double* AH, hipStream_t s);
int prolong_blocks(const gn_problem* p);
void prolong(const gn_problem* p, const gn_precond* pc, const double* r, double* z, double* part,
             const double* done, hipStream_t s);
// multi.hip (batched columns; scal == nullptr means every column is live)
int mc_width();
void spmv_mc(const gn_problem* p, const double* x, double* y, int k, double* part, int pstride,
             const double* scal, hipStream_t s);
void dot_mc(int64_t n, int k, const double* a, const double* b, double* part, int pstride, const double* scal,
            hipStream_t s);
void update_xr_mc(int64_t n, int k, double* x, double* r, const double* p, const double* q, const double* scal,
                  double* part, int pstride, hipStream_t s);
void update_p_mc(int64_t n, int k, double* p, const double* z, const double* scal, hipStream_t s);
void copy_mc(int64_t n, int k, double* dst, const double* src, const double* scal, hipStream_t s);
void sub_mc(int64_t n, int k, const double* b, const double* q, double* r, double* part, int pstride,
            const double* scal, hipStream_t s);
void finalize_mc(const double* part, int pstride, int nb, int op, int k, double* scal, double* hist,
                 int hstride, double rtol, hipStream_t s);
int mc_band_lds_bytes(int maxw);
void precond_mc(const gn_problem* p, const gn_precond* pc, const double* r, double* z, int k, double* part,
                int pstride, const double* scal, double* tm, double* gm, double* um, double* ym, hipStream_t s);
// geneo.hip
void eig_vinit(const gn_precond* pc, int b, int maxNBB, double* V, hipStream_t s);
void eig_bapply(const gn_problem* p, const gn_precond* pc, const double* BE, int b, int maxNBB,
                const double* V, double* out, hipStream_t s, const int* act = nullptr);
void eig_trsm(const gn_precond* pc, int b, const double* T, const double* D, const double* TB, const double* Vin,
              double* V, hipStream_t s, const int* act = nullptr);
int gram_split();
void eig_cheb_first(const gn_precond* pc, int b, const double* Z, const double* V, const double* nu,
                    const double* coef, int ncoef, double* Y1, double* resp, hipStream_t s,
                    const int* act = nullptr);
void eig_cheb_step(const gn_precond* pc, int b, int maxNBB, const double* TY, const double* Y1, double* Y0,
                   const double* coef, int ncoef, int step, hipStream_t s, const int* act = nullptr);
void eig_gram(const gn_precond* pc, int b, const double* Z, const double* BV, const double* BZ,
              const double* V, const double* nu, double* GPp, double* GBp, double* resp, hipStream_t s,
              const int* act = nullptr);
void eig_small(int n_sub, int b, const double* GPp, const double* GBp, const double* resp, double* res,
               double* Y, double* nu, int* flag, hipStream_t s, const int* act = nullptr);
void eig_vupdate(const gn_precond* pc, int b, int maxNBB, const double* Z, const double* BZ,
                 const double* Y, double* V, double* BV, hipStream_t s, const int* act = nullptr);
void eig_normalise(const gn_precond* pc, int b, int ncol, double* V, hipStream_t s);
void zem_modes(const gn_problem* p, const gn_precond* pc, int b, int maxNBB, double* V, hipStream_t s);
void eig_resid_sum(int n_sub, int b, const double* resp, double* res, hipStream_t s, const int* act = nullptr);
void eig_rq(const gn_problem* p, const gn_precond* pc, int b, const double* V, double* lam, hipStream_t s);
void eig_defect(const gn_precond* pc, int b, int maxNBB, const double* BV, const double* PV, const double* nu,
                double* rho, hipStream_t s);
void eig_defect_add(const gn_precond* pc, int b, int maxNBB, const double* D, const double* nu, double nu_min,
                    double* V, hipStream_t s);
void build_phi(const gn_problem* p, const gn_precond* pc, int b, int maxNI, const double* V,
               hipStream_t s);
void aphi(const gn_problem* p, const gn_precond* pc, int b, int maxNB, double* Y, hipStream_t s);
void ah_pairs(const gn_problem* p, const gn_precond* pc, const void* d_pairs, int npairs, int b,
              const double* Y, double* AH, hipStream_t s);
int pair_size();
void make_pair(void* dst, int j1, int j2, const int lo[3], const int hi[3]);
void dense_chol(int NB, double* A, double* Dinv, int* info, hipStream_t s);
void tri_inv(int NB, const double* L, const double* Dinv, double* Z, hipStream_t s);
}  // namespace gnk

// ---------------------------------------------------------------------------
// host helpers of the solve paths (api.hip)
// ---------------------------------------------------------------------------
namespace gnh {
// caching device allocator (api.hip): blocks freed with dev_free are kept for
// reuse by later allocations of about the same size; dev_free only after the
// work that used the block has finished
void* dev_alloc(size_t bytes);
void dev_free(void* p);
int64_t dev_size(const void* p);     // rounded size a live block was asked for (0 if unknown)
double dev_alloc_seconds();          // cumulative time spent in hipMalloc/hipFree
PouDev pou_dev(const gn_problem* p, const gn_precond* pc);
constexpr double kEps = 2.220446049250313e-16;
// restarts stop once b - A x is within this factor of eps || |A| |x| ||
constexpr double kFloorFactor = 1.0;
// Squared stopping level of a restarted CG sequence, relative to ||b||^2 = bb.
// Its recursive residual tracks b - A x only to within about the rounding floor
// eps || |A| |x| || (squared: floor2), so a sequence that stops at rtol leaves
// b - A x at rtol plus that drift. A restart therefore aims below rtol by the
// floor, at no less than rtol / 2. The convergence test stays rtol.
inline double restart_tol2(double rtol, double floor2, double bb) {
  const double rt = std::max(rtol - std::sqrt(floor2 / bb), 0.5 * rtol);
  return rt * rt * bb;
}
double now_s();
double absmv_norm2(gn_problem* p, const double* x, hipStream_t s);
double cond_from_hist(const double* hist, int kit);
void ensure_batch_workspace(gn_problem* p, gn_precond* pc, int maxit, hipStream_t s);
int64_t resident_bytes(const std::vector<void*>& owned);
// launch order q -> item that gives the XCDs (q mod 8) near-equal total weight:
// heaviest item first onto the least loaded XCD with a free position
std::vector<int> xcd_order(const std::vector<int64_t>& weight);
}  // namespace gnh

// ---------------------------------------------------------------------------
// slot engine of the batched solves (serve.hip): up to 16 right-hand sides of
// one operator share every launch; a slot whose column has finished takes the
// next queued column at the following chunk boundary
// ---------------------------------------------------------------------------
struct SlotColumn {
  const double* b = nullptr;   // right-hand side, free numbering (device)
  double* x = nullptr;         // solution column, free numbering (device)
  double rtol = 1e-8;
  int maxit = 1000;
  void* tag = nullptr;         // owner, handed back with the result
  int index = 0;               // column index within the owner
};
struct SlotResult {
  SlotColumn col;
  gn_solve_report rep;
  gn_status st;
};
class SlotEngine {
 public:
  SlotEngine(gn_problem* p, gn_precond* pc, int slots, int chunk, int maxit_cap, hipStream_t s);
  int slots() const { return k_; }
  int free_slots() const;
  bool busy() const;
  void admit(const SlotColumn& c);                 // needs free_slots() > 0
  void step(std::vector<SlotResult>& out);         // start admitted columns, one chunk, retire
 private:
  struct Slot {
    bool used = false, fresh = false;
    SlotColumn col;
    int restarts = 0, first_iters = -1;
    double t0 = 0.0;
    std::vector<double> fin;                       // scalars at the end of the last CG sequence
  };
  void apply_m(int op);
  void read_scal();
  void write_rows(const std::vector<int>& cols);
  void phase_begin(const std::vector<int>& cols, std::vector<int>& held);
  void phase_end(const std::vector<int>& held);
  gn_problem* p_;
  gn_precond* pc_;
  int k_, chunk_, maxit_cap_;
  hipStream_t s_;
  std::vector<Slot> slot_;
  std::vector<double> hsc_;                        // host mirror of the per-column scalars
};

// profiling of kernel groups (api.hip)
struct GnProfScope {
  int group;
  double bytes;
  hipStream_t s;
  hipEvent_t e0, e1;
  bool on;
  GnProfScope(int g, double b, hipStream_t st);
  ~GnProfScope();
};
enum { PROF_SPMV = 0, PROF_TRSV, PROF_PROLONG, PROF_COARSE, PROF_VEC, PROF_NGROUP };

// ---------------------------------------------------------------------------
// Cholesky factor and inverse of one SPD TILE x TILE tile by a workgroup of
// 256 threads: Gaussian elimination of [S | I] without pivoting, one LDS
// barrier per column.  With d_k the k-th pivot and m_rk = S_k(r, k) / d_k its
// multipliers, S_{k+1}(r, j) = S_k(r, j) - m_rk S_k(j, k) on the lower triangle
// (S_k(j, k) = S_k(k, j)), and the identity's rows take the same row
// operations, Y(r, c) -= m_rk Y(k, c), which leaves Y = Lu^-1 for the unit
// lower factor Lu of S = Lu diag(d) Lu^T.  Then L = Lu diag(d)^1/2, i.e.
// L(r, k) = S_k(r, k) / sqrt(d_k), and L^-1 = diag(d)^-1/2 Y.
// Column k of S_k and row k of Y are final once step k - 1 is done; their
// owners publish them to LDS (col[k][.], yr[k][.]) for step k.  A thread holds
// three entries of the lower triangle of S (528) and two of the strictly
// lower part of Y (496) in registers; where it has fewer it takes entry
// (0, 0), which is never published.  col and yr start as zero, with
// yr(k, k) = 1, so every step updates every entry without a test: an S entry
// (r, j) with j < k and a Y entry (r, c) with c > k or r < k read a zero factor
// and keep their value exactly; an entry already published may change
// afterwards, but only its published copy is read again.
//   S: the tile, S[r][c] (lower triangle read); col, yr: work tiles; sink: 256
//   doubles that take the stores of entries not being published.  All in LDS.
//   On return (after a barrier) col[k][r] = S_k(r, k) for r >= k and
//   yr[r][c] = Y(r, c) for c < r; tile_spd_entry forms L and L^-1 from them.
//   Returns 1 + the first step whose pivot is not positive (that pivot is
//   taken as 1 and the elimination runs to the end), or 0.
// ---------------------------------------------------------------------------
__device__ inline void tile_lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
__device__ inline int tile_spd_eliminate(const double (*S)[TILE + 1], double (*col)[TILE + 1],
                                         double (*yr)[TILE + 1], double* sink) {
  constexpr int NTH = 256, NSL = 3, NYL = 2;
  const int tid = threadIdx.x;
  int sr[NSL], sj[NSL], yrw[NYL], yc[NYL];
  double ms[NSL], my[NYL];
#pragma unroll
  for (int u = 0; u < TILE2 / NTH; ++u) {
    const int e = tid + NTH * u;
    col[e / TILE][e % TILE] = 0.0;
    yr[e / TILE][e % TILE] = (e / TILE == e % TILE) ? 1.0 : 0.0;
  }
  tile_lds_barrier();
#pragma unroll
  for (int u = 0; u < NSL + NYL; ++u) {
    const bool isS = u < NSL;
    const int f = tid + NTH * (isS ? u : u - NSL);
    const bool ok = isS ? f < TILE * (TILE + 1) / 2 : f < TILE * (TILE - 1) / 2;
    // S: f = r (r + 1) / 2 + j; Y: f = rr (rr + 1) / 2 + c with r = rr + 1
    int rr = (int)((sqrtf(8.0f * (float)f + 1.0f) - 1.0f) * 0.5f);
    if ((rr + 1) * (rr + 2) / 2 <= f) ++rr;
    if (rr * (rr + 1) / 2 > f) --rr;
    const int c = f - rr * (rr + 1) / 2;
    if (isS) {
      sr[u] = ok ? rr : 0;
      sj[u] = ok ? c : 0;
      ms[u] = S[sr[u]][sj[u]];
      if (ok && c == 0) col[0][rr] = ms[u];
    } else {
      yrw[u - NSL] = ok ? rr + 1 : 0;
      yc[u - NSL] = ok ? c : 0;
      my[u - NSL] = 0.0;
    }
  }
  tile_lds_barrier();
  int fail = 0;
  for (int k = 0; k < TILE; ++k) {
    const int k1 = k + 1 < TILE ? k + 1 : TILE - 1;
    double as[NSL], bs[NSL], ay[NYL], by[NYL];
#pragma unroll
    for (int u = 0; u < NSL; ++u) {
      as[u] = col[k][sr[u]];
      bs[u] = col[k][sj[u]];
    }
#pragma unroll
    for (int u = 0; u < NYL; ++u) {
      ay[u] = col[k][yrw[u]];
      by[u] = yr[k][yc[u]];
    }
    double d = col[k][k];
    if (!(d > 0.0)) {
      if (fail == 0) fail = k + 1;
      d = 1.0;
    }
    const double rd = 1.0 / d;
#pragma unroll
    for (int u = 0; u < NSL; ++u) {
      ms[u] -= (as[u] * rd) * bs[u];
      *(sj[u] == k + 1 ? &col[k1][sr[u]] : sink + tid) = ms[u];
    }
#pragma unroll
    for (int u = 0; u < NYL; ++u) {
      my[u] -= (ay[u] * rd) * by[u];
      *(yrw[u] == k + 1 ? &yr[k1][yc[u]] : sink + tid) = my[u];
    }
    tile_lds_barrier();
  }
  return fail;
}
// Entry (r, c) of L and of L^-1 from the results of tile_spd_eliminate (a pivot
// that was not positive is taken as 1, as there).
__device__ inline void tile_spd_entry(const double (*col)[TILE + 1], const double (*yr)[TILE + 1], int r, int c,
                                      double& l, double& x) {
  const double dc = col[c][c] > 0.0 ? col[c][c] : 1.0;
  const double dr = col[r][r] > 0.0 ? col[r][r] : 1.0;
  l = r > c ? col[c][r] / sqrt(dc) : (r == c ? sqrt(dc) : 0.0);
  x = r > c ? yr[r][c] / sqrt(dr) : (r == c ? 1.0 / sqrt(dr) : 0.0);
}

// ---------------------------------------------------------------------------
// device reduction helpers (fixed order: deterministic for a fixed launch shape)
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// sum over a block of up to 1024 threads; result valid in every thread
__device__ inline double block_sum(double v, double* sh /* >= 16 doubles */) {
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += sh[i];
  return t;
}
