/*
 * genpcg.h -- C ABI of the MI355X GenEO-preconditioned CG library.
 *
 * The library solves the Q1 finite-element system A u = b of anisotropic
 * linear elasticity or scalar diffusion (Butler et al., arXiv 1901.05188,
 * Section 2: eq:strongForm, eq-fe, eqn:fe_matrix_system; Section 6: eqn:Darcy,
 * eq-fe-darcy) by conjugate gradients (Section 3.1, eqn:KrylovSubspace)
 * preconditioned with two-level additive Schwarz (Section 3.1, eqn:onelevelAS
 * and M^-1_{AS,2}) whose coarse space is GenEO (Section 3.2, eq-geneo and the
 * coarse-space definition; Section 3.3, eqm:matrixForm and the coarse
 * assembly).
 *
 * Conventions shared by every entry point:
 *  - Structured grid of ne[0] x ne[1] x ne[2] hexahedra; node (i,j,k) has id
 *    i + (ne[0]+1)*(j + (ne[1]+1)*k); element (ex,ey,ez) has id
 *    ex + ne[0]*(ey + ne[1]*ez).
 *  - DOF vectors exchanged through the ABI use the FREE numbering: node id
 *    ascending, component fastest within a node, homogeneous Dirichlet DOFs
 *    removed.  Multi-column vectors are column-major with leading dimension
 *    ld >= n_free.
 *  - Host arrays (const pointers in the option/input structs) are read during
 *    the call and not retained.  Pointers documented as device pointers must
 *    point to device memory of the current HIP device (e.g. a torch tensor's
 *    data_ptr()) and are accessed in stream order on the given stream.
 *  - `stream` is a hipStream_t (NULL = the default stream).
 *  - Handles own their device memory until gn_destroy_*.  No C++ exception
 *    crosses the ABI.  On error *out is set to NULL, inputs are untouched, a
 *    negative status is returned and gn_last_error() describes the failure
 *    (thread-local string, valid until the next call on the same thread).
 */
#ifndef GENPCG_H
#define GENPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gn_status;
enum {
  GN_OK = 0,
  GN_WARN_MAXIT = 1,          /* solve stopped at maxit; last iterate returned   */
  GN_PENDING = 2,             /* gn_server_wait: request not finished in time    */
  GN_ERR_ARG = -1,            /* invalid argument / inconsistent sizes           */
  GN_ERR_OOM = -2,            /* device allocation failed                        */
  GN_ERR_NOT_SPD = -3,        /* a Cholesky factorisation met a non-positive pivot */
  GN_ERR_EIG_NOCONV = -4,     /* a GenEO eigensolve did not converge in eig_maxit */
  GN_ERR_COARSE_SINGULAR = -5,/* coarse matrix A_H not positive definite         */
  GN_ERR_DEVICE = -6,         /* HIP runtime error                               */
  GN_ERR_BREAKDOWN = -7       /* CG breakdown (p^T A p <= 0)                     */
};

typedef struct gn_problem gn_problem; /* device-resident A, b, element matrices */
typedef struct gn_precond gn_precond; /* local factors, coarse basis, coarse factor */

/* Tensor grid.  xn[a] holds ne[a]+1 increasing node coordinates (mm).
 * map_kind 0: identity.  map_kind 1: ramp, map_par = {x0, x1, angle}: the node
 * (x,y,z) is placed at (x, y, z + tan(angle)*(clamp(x,x0,x1) - x0)). */
typedef struct gn_grid {
  int32_t ne[3];
  const double* xn[3];
  int32_t map_kind;
  const double* map_par;
} gn_grid;

/* Material description (Section 2, eq-hooke and the ply paragraph).
 * pde 1 (elasticity): mat holds n_mat rows of 9 engineering constants
 *   (E1,E2,E3,G12,G13,G23,nu12,nu13,nu23) in MPa; elem_mat[e] selects the row;
 *   elem_angle[e] (radians, may be NULL = 0) rotates the material about +z
 *   (counter-clockwise seen from +z); elem_tilt[e] (may be NULL = 0) then tilts
 *   it about y so that the material x axis becomes (cos t, 0, sin t).
 * pde 0 (scalar diffusion): elem_k[e] > 0 is the conductivity of element e;
 *   mat/elem_mat/elem_angle/elem_tilt are ignored. */
typedef struct gn_material {
  int32_t pde;
  int32_t n_mat;
  const double* mat;
  const int32_t* elem_mat;
  const double* elem_angle;
  const double* elem_tilt;
  const double* elem_k;
} gn_material;

/* Boundary conditions and loads (Section 2, eq-boundary, eq:strongForm).
 * dirichlet[node*ncomp + c] = 1 marks a homogeneous Dirichlet DOF.
 * body (may be NULL): constant body force per element, ncomp values each.
 * traction (may be NULL): constant traction on the top face (z = max) of each
 *   top-layer element, layout [rhs][face = ex + ne[0]*ey][comp].
 * The assembled load has nrhs columns; the body force is added to each. */
typedef struct gn_loads {
  const uint8_t* dirichlet;
  const double* body;
  int32_t nrhs;
  const double* traction;
} gn_loads;

/* Assemble A (27-point node-block matrix, FP64) and b on the device
 * (eqn:fe_matrix_system, 2x2x2 Gauss).  Returns a problem handle.  The host
 * arrays are read during the call; the material and load arrays are copied to
 * the device and kept with the problem (gn_reassemble). */
gn_status gn_assemble(const gn_grid* grid, const gn_material* mat, const gn_loads* loads,
                      void* stream, gn_problem** out);

/* Assemble again, on the device, from the inputs the problem holds
 * (eqn:fe_matrix_system, the same kernels as gn_assemble): the element
 * matrices, A and b are recomputed in place, with no host array and no
 * transfer from the host.  Results equal those of gn_assemble bit for bit.
 * Synchronizes the stream.  Preconditioners built on p must not be used
 * while the call runs (they read A and the element matrices); errors:
 * GN_ERR_ARG (null problem), GN_ERR_DEVICE. */
gn_status gn_reassemble(gn_problem* p, void* stream);

/* Sizes: number of free DOFs, stored matrix entries, number of load columns. */
gn_status gn_problem_info(const gn_problem* p, int64_t* n_free, int64_t* nnz, int32_t* nrhs);

/* Copy the assembled load (n_free x nrhs, column-major, leading dim ld) into
 * the device buffer b_dev. */
gn_status gn_problem_rhs(const gn_problem* p, double* b_dev, int64_t ld, void* stream);

/* Load vectors alone, on the mesh and Dirichlet mask of p (Section 2: the
 * right-hand side of eq-fe, body force plus top-face traction, 2x2x2 and 2x2
 * Gauss as in gn_assemble), for new load cases of an assembled operator.
 * body (host, may be NULL): n_elem * ncomp values, added to every column.
 * traction (host, may be NULL): layout [rhs][face = ex + ne[0]*ey][comp].
 * b_dev (device): nrhs columns in the free numbering, leading dimension ld.
 * Temporary device memory of n_dof * nrhs doubles is allocated and freed;
 * the call returns after b_dev is written. */
gn_status gn_load_vectors(gn_problem* p, const double* body, int32_t nrhs, const double* traction,
                          double* b_dev, int64_t ld, void* stream);

/* gn_load_vectors for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments and bit-identical output, but the staged host loads and the
 * full-numbering load live in a static device workspace of 32 MiB per device
 * (held until the process ends) instead of temporary allocations; the call
 * makes no hipMalloc/hipFree.  It needs
 * 8 * (round32(n_elem * ncomp if body) + round32(nrhs * ne[0] * ne[1] * ncomp
 * if traction) + n_dof * nrhs) bytes, round32 rounding up to a multiple of 32;
 * a larger request returns GN_ERR_ARG before any device work.  Every call on a
 * device shares that device's workspace: calls that overlap in time on one
 * device (other threads, other streams) race and must be serialized by the
 * caller.  Returns after b_dev is written. */
gn_status gn_load_vectors_noalloc(gn_problem* p, const double* body, int32_t nrhs, const double* traction,
                                  double* b_dev, int64_t ld, void* stream);

/* y = A x for ncol columns (device pointers, free numbering, leading dim ld). */
gn_status gn_matvec(gn_problem* p, const double* x_dev, double* y_dev, int32_t ncol,
                    int64_t ld, void* stream);

/* Domain decomposition and GenEO options (Section 3.1: non-overlapping boxes
 * extended by `overlap` element layers; Section 3.2: m_j eigenvectors).
 * cuts[a] holds nparts[a]+1 increasing element indices from 0 to ne[a].
 * m_j = nev if nev > 0, else #{lambda < threshold} capped at nev_max (if > 0);
 * then extended while the next eigenvalue repeats the last within 1e-8
 * relative + 1e-10 absolute.  coarse = 1 builds that GenEO coarse space,
 * coarse = 0 the one-level method only, and coarse = 2 the zero-energy-mode
 * space the paper compares against (Section 5, Example 1b): on each subdomain
 * whose nodes carry no Dirichlet DOF, the kernel of its Neumann matrix
 * A_{Omega_j} (the constant for diffusion, the three translations and three
 * rotations for elasticity), times X_j; nev/threshold are then ignored and
 * gn_precond_eigenvalues reports no eigenvalues.
 * local_prec 64 stores FP64 local factors, 32 stores them in FP32 (FP64
 * factorisation, FP32 storage and triangular solves, FP64 accumulation of the
 * result).  shift > 0 is the shift-and-invert shift (Section 3.3.2; 0 = 1e-2).
 * eig_tol / eig_maxit bound the batched eigensolver (0 = defaults 1e-12 / 300):
 * it stops when every Ritz pair that enters the coarse space has
 * ||P^-1 B v - nu v|| <= eig_tol ||P^-1 B v|| and the other wanted pairs (those
 * below 1.5 x threshold, and the first one past the selection, which only fix
 * m_j through their eigenvalues) have it below sqrt(eig_tol), or when the
 * residual stays below 1e-9 without halving over 15 block solves.
 * eig_block is the subspace block size.  0 = automatic: max(32, nev + max(8,
 * nev/2)) (at most 64, and at most the smallest pencil's row count unless that
 * is below nev + max(8, nev/2)) for a fixed nev; for a threshold
 * min(32, nev_max + 8), grown by
 * 16 up to 64 and the eigensolve repeated while the eigenvalues below
 * 1.5 x threshold (plus 4 guard vectors) do not fit.  A given value must lie
 * in [nev + 5 (or 5), 64]; if it proves too small, GN_ERR_EIG_NOCONV.
 * eig_filter is the largest Chebyshev filter degree per Rayleigh-Ritz step
 * (0 = 4; 1 = plain subspace iteration); the degree ramps up 1, 2, ... from the
 * first step.
 * local_kernel selects the kernel of single-column local solves: 0 = the
 * register-pipelined sweep when the band fits it, its launch shape (512 or 1024
 * threads per subdomain) timed at set-up when both fit and the choice kept for
 * later preconditioners of the same band shape in the process; 1 = always the
 * 16-column matrix-core kernel of the batched solves; 2 = the sweep with the
 * first shape that fits, untimed; 3 / 4 = the sweep with 512 / 1024 threads
 * per subdomain (GN_ERR_ARG when the band does not fit that shape).
 * pou selects the partition of unity X_j (Section 3.2, def:pou; Section 3.3.1):
 * 0 = the standard one (one over the number of subdomains whose V_h0 holds the
 * DOF, zero on the subdomain boundary); 1 = the smoother one of Sarkis that the
 * paper also provides: subdomain j is weighted by the distance of the node to
 * the artificial boundary of Omega_j (element layers, the smallest over the
 * box's faces that are not on the physical boundary), divided by the sum of
 * those weights over all subdomains.
 * coarse_solve selects how A_H^-1 is applied (Section 3.3.3, last paragraph):
 * 0 = exactly, by the dense Cholesky factor of A_H (its explicit inverse);
 * 1 = inexactly, by conjugate gradients on the block-sparse A_H (blocks only
 * for overlapping subdomain pairs) preconditioned by the inverses of its
 * diagonal blocks, stopped at coarse_rtol (0 = 1e-4) relative residual or
 * coarse_maxit (0 = 200) iterations.  The preconditioner then varies from one
 * application to the next: solve with gn_solve_opts.flexible = 1.
 * eig_refine (0 = 1, at most 8) is the number of refinement steps in the
 * original pencil once the iteration has converged: each adds
 * P^-1 (B v - nu P v) / nu to every Ritz vector v, with B v and P v formed from
 * the element matrices, and takes a Rayleigh-Ritz step on the block. */
typedef struct gn_dd_opts {
  int32_t nparts[3];
  const int32_t* cuts[3];
  int32_t overlap;
  int32_t nev;
  double threshold;
  int32_t nev_max;
  int32_t local_prec;
  int32_t coarse;
  double shift;
  double eig_tol;
  int32_t eig_maxit;
  int32_t eig_block;
  int32_t eig_filter;
  int32_t local_kernel;
  int32_t pou;
  int32_t coarse_solve;
  double coarse_rtol;
  int32_t coarse_maxit;
  int32_t eig_refine;
} gn_dd_opts;

typedef struct gn_setup_report {
  int32_t n_sub;
  int64_t coarse_dim;
  int32_t eig_iters;         /* Rayleigh-Ritz steps of the batched eigensolver */
  int32_t max_local_n;       /* largest local system size                      */
  int32_t band_tiles;        /* band width in 32-row tiles (largest subdomain) */
  double t_local_s, t_eigen_s, t_coarse_s, t_total_s;
  int64_t hbm_bytes;         /* device bytes held by the preconditioner        */
  double eig_resid;          /* largest final relative Ritz residual of the pairs in the coarse space */
  int32_t eig_solves;        /* block solves with the pencil factors            */
  double t_alloc_s;          /* time of this call spent in hipMalloc/hipFree (freed
                                device blocks are cached and reused by later calls) */
  double apply_bytes;        /* algorithmic bytes of one single-column local-solve
                                launch: both sweeps over the factors' bands (row r
                                of a band holds min(r, bandwidth) + 1 entries), the
                                gather of r, the write of z_j and Phi_j^T r        */
  double apply_tile_bytes;   /* the same launch counted over the stored 32 x 32 band
                                tiles and inverse diagonal tiles                   */
  int32_t local_threads;     /* threads per subdomain of the single-column local
                                solve (512 or 1024); 0 when the 16-column
                                matrix-core kernel serves single columns          */
} gn_setup_report;

/* Build the preconditioner: local Dirichlet factors A_j = L_j L_j^T
 * (Section 3.1), GenEO eigenpairs of A_{Omega_j} p = lambda X A_{Omega_j^o} X p
 * (eqm:matrixForm), coarse basis Phi_{i(j,k)} = X^(j) p_k^j and coarse matrix
 * A_H = R_H A R_H^T by local products (Section 3.3.3), and its factor. */
gn_status gn_setup_geneo(gn_problem* p, const gn_dd_opts* opts, void* stream,
                         gn_precond** out, gn_setup_report* report);

/* Eigenvalues lambda_1..lambda_n of subdomain `sub` (ascending), up to cap of
 * them, into host array out; *m receives m_j, *n_avail the number computed. */
gn_status gn_precond_eigenvalues(const gn_precond* pc, int32_t sub, double* out, int32_t cap,
                                 int32_t* m, int32_t* n_avail);

/* The coarse basis (Section 3.3.2: Phi_{i(j,k)} = X^(j) p_k^j padded by zeros,
 * i(j,k) = sum_{l<j} m_l + k) copied into the host array out in the free
 * numbering: N_H columns of n_free values, column-major, leading dimension
 * ld >= n_free; *nh (may be NULL) receives N_H.  out = NULL only queries N_H.
 * Synchronizes the device.  A preconditioner without a coarse space has
 * N_H = 0. */
gn_status gn_precond_coarse_basis(const gn_precond* pc, double* out, int64_t ld, int64_t* nh);

/* z = M^-1 r for one column (device pointers, free numbering). */
gn_status gn_precond_apply(gn_precond* pc, const double* r_dev, double* z_dev, void* stream);

typedef struct gn_solve_opts {
  double rtol;          /* stop when ||r||_2 <= rtol ||b||_2                   */
  int32_t maxit;
  int32_t check_every;  /* iterations per host convergence check (0 = 8)       */
  int32_t sequential;   /* nrhs > 1: 0 = batches of up to 16 columns share every
                           launch (one pass over each local factor per iteration
                           for the whole batch, per-column alpha, beta and
                           stopping); 1 = the columns are solved one after
                           another.  Ignored for nrhs = 1.                      */
  int32_t graphs;       /* single-column solves: 1 = each chunk of check_every
                           iterations is replayed from a HIP graph captured on
                           first use (kept with the preconditioner, or with the
                           problem for plain CG, until destroyed); 0 = kernel
                           by kernel.  Same arithmetic either way.  Not used
                           while kernel profiling (gn_profile_enable) is on.    */
  int32_t flexible;     /* 1 = flexible CG: beta = z_{k+1}^T (r_{k+1} - r_k) /
                           z_k^T r_k (Polak-Ribiere), which keeps CG converging
                           when the preconditioner changes between applications,
                           as with the inexact coarse solve of Section 3.3.3
                           (gn_dd_opts.coarse_solve = 1), where the paper
                           switches to a flexible Krylov method; equal to the
                           standard beta for a fixed preconditioner.  Columns
                           are then solved one after another.                   */
} gn_solve_opts;

typedef struct gn_solve_report {
  int32_t iters;
  int32_t converged;
  double rel_res;       /* recursive residual norm / ||b||                    */
  double true_rel_res;  /* ||b - A x|| / ||b|| recomputed at exit             */
  double cond_est;      /* extreme eigenvalue ratio of the CG-Lanczos tridiagonal */
  double t_solve_s;
  int32_t iters_first;  /* iterations of the first (un-restarted) CG sequence   */
  int32_t restarts;     /* restarts from b - A x taken to meet rtol on the true residual
                           (at most 2; none once ||b - A x|| <= eps || |A| |x| ||); a
                           restarted sequence stops at max(rtol - res_floor, rtol / 2)
                           on its recursive residual, so that its drift of about
                           res_floor still leaves b - A x within rtol              */
  double res_floor;     /* eps || |A| |x| || / ||b||: rounding floor of the true
                           residual of an FP64 solution                          */
} gn_solve_report;

/* Solve A x = b by PCG with x0 = 0 for nrhs columns (device pointers, free
 * numbering, column-major, leading dim ld).  pc = NULL runs plain CG.
 * reports (host, nrhs entries) may be NULL.
 * Each column runs its own CG recurrence (Section 3.1, eqn:KrylovSubspace):
 * its own alpha, beta, stopping test and restarts, so a column's iterates do
 * not depend on the other columns of its batch beyond rounding (batched
 * columns use the MFMA block solves, single columns the scalar sweeps).
 * Returns GN_WARN_MAXIT if a column stopped at maxit, GN_ERR_BREAKDOWN if a
 * column met p^T A p <= 0; the other columns are still solved. */
gn_status gn_solve(gn_problem* p, gn_precond* pc, const double* b_dev, double* x_dev,
                   int32_t nrhs, int64_t ld, const gn_solve_opts* opts, void* stream,
                   gn_solve_report* reports);

/* Device bytes held by p and pc (pc may be NULL): assembled operator,
 * element matrices, workspaces, local factors, coarse basis and factor. */
gn_status gn_resident_bytes(const gn_problem* p, const gn_precond* pc, int64_t* bytes);

/* Resident device bytes of an operator assembled on grid (pde 0 diffusion,
 * 1 elasticity, one load column) and of its preconditioner built with opts
 * (opts may be NULL: the operator alone), including the workspace of the
 * 16-column batched solves and a history of 2000 iterations, as a request
 * server holds them (Section 3.1's decomposition sizes: subdomain boxes, band
 * widths, coarse dimension).  Computed on the host from the sizes, before any
 * assembly or set-up, for admission by footprint.  The coarse dimension is
 * taken as nev per subdomain (fixed count), nev_max (threshold: an upper
 * bound) or the mode count (zero-energy modes, every subdomain counted), and
 * the free-to-full map as if no DOF were fixed, so the figure bounds the
 * measured gn_resident_bytes from above; a fixed count whose eigenvalue
 * clusters straddle the cut can add vectors beyond nev. */
gn_status gn_footprint(const gn_grid* grid, int32_t pde, const gn_dd_opts* opts, int64_t* bytes);

/* Request server (the multi-right-hand-side path of Section 3.1 for a stream
 * of load cases): operators stay resident with their preconditioners; each
 * has its own HIP stream and a host worker thread that runs up to `slots`
 * right-hand sides in every launch (the batched kernels of gn_solve).  Each
 * column keeps its own CG recurrence, stopping test and restarts, so a
 * column's result is the same, bit for bit, whichever slot it takes and
 * whatever else is in flight.  A column that finishes frees its slot, and the
 * next queued column of that operator starts at the following check (every
 * check_every iterations) while the others keep iterating.  Operators'
 * workers run concurrently, so different operators overlap on the device.
 *  - hbm_budget: device bytes the resident operators may hold together
 *    (gn_resident_bytes after the batched workspace is allocated, or the
 *    gn_footprint estimate while a registered operator is being built); 0 =
 *    the device's total memory.  gn_server_add evicts idle server-built
 *    operators to make room and fails with GN_ERR_OOM beyond it.
 *  - slots: columns per operator batch, 1..16 (0 = 16).
 *  - check_every: CG iterations between slot updates (0 = 8).
 *  - maxit_cap: largest maxit a request may ask for (0 = 2000). */
typedef struct gn_server_opts {
  int64_t hbm_budget;
  int32_t slots;
  int32_t check_every;
  int32_t maxit_cap;
} gn_server_opts;
typedef struct gn_server gn_server;

gn_status gn_server_create(const gn_server_opts* opts, gn_server** out);

/* Register a resident operator (pc may be NULL: plain CG).  The caller keeps
 * ownership of p and pc, must have finished its own work on them, and must
 * not use them elsewhere (gn_solve, gn_precond_apply, another server) until
 * gn_server_remove returns.  *op receives the operator id, *bytes (may be
 * NULL) its footprint. */
gn_status gn_server_add(gn_server* sv, gn_problem* p, gn_precond* pc, int32_t* op, int64_t* bytes);

/* Register an operator by its description instead of built handles: the
 * host arrays of grid, mat, loads and opts are copied (nothing on the device),
 * *est_bytes (may be NULL) receives its gn_footprint estimate.  The server
 * builds it (gn_assemble + gn_setup_geneo on the operator's stream) when a
 * request for it arrives and its estimate plus 1/32 (the build's reservation,
 * replaced by the measured footprint once built) fits in the budget; while it
 * does not fit, the least recently used idle server-built operator (no queued
 * or running column) is destroyed to make room, and rebuilt when a later
 * request needs it.  Requests wait meanwhile; they fail with GN_ERR_OOM (the
 * message names the bytes) when even evicting every idle server-built operator
 * cannot make room, and with the set-up's status and message if the build
 * fails.  Registration itself returns GN_ERR_OOM when the reservation exceeds
 * the whole budget.  Right-hand sides use the operator's free numbering (the
 * mask in loads). */
gn_status gn_server_register(gn_server* sv, const gn_grid* grid, const gn_material* mat, const gn_loads* loads,
                             const gn_dd_opts* opts, int32_t* op, int64_t* est_bytes);

/* State of an operator: *resident 1 while its device data exist, *builds and
 * *evictions the number of builds and evictions so far (server-built
 * operators), *bytes its measured footprint while resident, else its estimate.
 * Any output may be NULL. */
gn_status gn_server_operator_info(gn_server* sv, int32_t op, int32_t* resident, int32_t* builds,
                                  int32_t* evictions, int64_t* bytes);

/* Finish the operator's queued and running columns, stop its worker and
 * return its footprint to the budget (a server-built operator's device data
 * are destroyed). */
gn_status gn_server_remove(gn_server* sv, int32_t op);

/* Queue nrhs right-hand sides of operator op (device pointers, free
 * numbering, column-major with leading dimension ld; x0 = 0).  b_dev must be
 * complete on the device when this is called, no pending work may access
 * x_dev, and both must stay allocated and untouched until gn_server_wait has
 * returned the ticket (the operator's worker writes x_dev on its own stream).  Returns at once;
 * *ticket identifies the request. */
gn_status gn_server_submit(gn_server* sv, int32_t op, const double* b_dev, double* x_dev, int32_t nrhs,
                           int64_t ld, double rtol, int32_t maxit, int64_t* ticket);

/* Wait up to timeout_s seconds (< 0: no limit) for a request.  When it has
 * finished: x_dev is complete, reports (host, nrhs entries, may be NULL) and
 * *latency_s (submit to the last column's completion, may be NULL) are
 * filled, the ticket is released and the request's status is returned
 * (worst over its columns, as gn_solve).  Otherwise GN_PENDING. */
gn_status gn_server_wait(gn_server* sv, int64_t ticket, double timeout_s, gn_solve_report* reports,
                         double* latency_s);

/* Finish every queued request, stop all workers and free the server (the
 * operators stay with the caller). */
void gn_server_destroy(gn_server* sv);

/* Per-kernel timing with HIP events on the library's launch stream.  enable=1
 * starts recording every launch of the named kernel group ("spmv", "trsv",
 * "prolong", "coarse", "vec"); gn_profile_read returns the summed milliseconds,
 * the number of launches and the algorithmic bytes those launches move. */
gn_status gn_profile_enable(int32_t enable);
gn_status gn_profile_read(const char* group, double* total_ms, int64_t* launches, double* bytes);

/* Device memory of the library: blocks freed by gn_destroy_*, by the end of
 * gn_setup_geneo (its temporaries) and by gn_load_vectors are kept by the
 * process and reused by later allocations of about the same size (repeated
 * set-ups then allocate nothing new).  gn_trim_memory synchronises the device
 * and returns every such idle block to the runtime; *released (may be NULL)
 * receives the bytes returned.  Blocks held by live handles are untouched. */
gn_status gn_trim_memory(int64_t* released);

void gn_destroy_problem(gn_problem* p);
void gn_destroy_precond(gn_precond* pc);
const char* gn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GENPCG_H */
