// Host orchestration behind the C ABI declared in include/genpcg.h.
//
// gn_assemble     : Section 2 (eq-fe, eqn:fe_matrix_system) on the device.
// gn_setup_geneo  : Section 3.1 (overlapping boxes, A_j), Section 3.2 (PoU,
//                   eq-geneo, coarse space), Section 3.3 (eqm:matrixForm,
//                   coarse assembly by local products, coarse factor).
// gn_solve        : Section 3.1 (preconditioned CG, x0 = 0), with the
//                   CG-Lanczos condition estimate the tables report.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "gn_internal.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;
void gn_set_error(gn_status code, const std::string& msg) {
  (void)code;
  g_last_error = msg;
}
extern "C" const char* gn_last_error(void) { return g_last_error.c_str(); }

#define GN_TRY try {
#define GN_CATCH                                                  \
  }                                                               \
  catch (const gn_error& e) {                                     \
    gn_set_error(e.code, e.msg);                                  \
    return e.code;                                                \
  }                                                               \
  catch (const std::bad_alloc&) {                                 \
    gn_set_error(GN_ERR_OOM, "host allocation failed");           \
    return GN_ERR_OOM;                                            \
  }                                                               \
  catch (...) {                                                   \
    gn_set_error(GN_ERR_DEVICE, "unexpected exception");          \
    return GN_ERR_DEVICE;                                         \
  }

static void argfail(const std::string& m) { throw gn_error{GN_ERR_ARG, m}; }

// ---------------------------------------------------------------------------
// device memory: a caching allocator
// ---------------------------------------------------------------------------
// Set-up allocates and frees many GB per call (pencil bands, block vectors,
// coarse matrix); fresh hipMalloc/hipFree of that much memory took from
// milliseconds to seconds from one call to the next.  Freed blocks therefore
// stay with the process, keyed by their rounded size, and an allocation takes
// the smallest cached block of at least its size and at most 1/8 larger.  A
// failed hipMalloc returns every cached block to the runtime and tries once
// more.  Callers free a block only after the work that used it has finished
// (a stream or device synchronisation), so a reused block is idle.
namespace {
std::mutex g_pool_mu;
std::multimap<size_t, void*> g_pool_free;   // rounded size -> idle block
std::map<void*, size_t> g_pool_size;        // every live or idle block -> its size
std::map<void*, size_t> g_pool_used;        // live blocks -> the rounded size asked for
size_t g_pool_cached = 0;
double g_pool_alloc_s = 0.0;                // seconds spent in hipMalloc/hipFree

size_t pool_round(size_t bytes) {
  if (bytes < ((size_t)1 << 20)) return (bytes + 511) & ~(size_t)511;
  return (bytes + ((size_t)1 << 21) - 1) & ~(((size_t)1 << 21) - 1);
}

size_t pool_trim_locked() {
  size_t n = 0;
  const auto t0 = std::chrono::steady_clock::now();
  for (auto& kv : g_pool_free) {
    (void)hipFree(kv.second);
    g_pool_size.erase(kv.second);
    n += kv.first;
  }
  g_pool_free.clear();
  g_pool_cached = 0;
  g_pool_alloc_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return n;
}
}  // namespace

void* gnh::dev_alloc(size_t bytes) {
  const size_t sz = pool_round(std::max(bytes, (size_t)1));
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pool_free.lower_bound(sz);
  if (it != g_pool_free.end() && it->first <= sz + sz / 8) {
    void* p = it->second;
    g_pool_cached -= it->first;
    g_pool_free.erase(it);
    g_pool_used[p] = sz;
    return p;
  }
  void* p = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    pool_trim_locked();
    e = hipMalloc(&p, sz);
  }
  g_pool_alloc_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw gn_error{e == hipErrorOutOfMemory ? GN_ERR_OOM : GN_ERR_DEVICE,
                   "device allocation of " + std::to_string(sz) + " bytes: " + hipGetErrorString(e)};
  }
  g_pool_size[p] = sz;
  g_pool_used[p] = sz;
  return p;
}

void gnh::dev_free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pool_size.find(p);
  if (it == g_pool_size.end()) return;
  g_pool_used.erase(p);
  g_pool_free.emplace(it->second, p);
  g_pool_cached += it->second;
}

// the rounded size a live block was asked for (a reused idle block may be up
// to 1/8 larger; that slack is the pool's, not the handle's)
int64_t gnh::dev_size(const void* p) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pool_used.find(const_cast<void*>(p));
  return it == g_pool_used.end() ? 0 : (int64_t)it->second;
}

double gnh::dev_alloc_seconds() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  return g_pool_alloc_s;
}

extern "C" gn_status gn_trim_memory(int64_t* released) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  (void)hipDeviceSynchronize();
  const size_t n = pool_trim_locked();
  if (released) *released = (int64_t)n;
  return GN_OK;
}

template <typename T>
static T* dalloc(std::vector<void*>& owned, size_t count) {
  void* p = gnh::dev_alloc(std::max(count, (size_t)1) * sizeof(T));
  owned.push_back(p);
  return (T*)p;
}
static void dfree_all(std::vector<void*>& owned) {
  for (void* p : owned) gnh::dev_free(p);
  owned.clear();
}
template <typename T>
static T* upload(std::vector<void*>& owned, const T* h, size_t count, hipStream_t s) {
  T* d = dalloc<T>(owned, count);
  GN_HIP(hipMemcpyAsync(d, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}
std::vector<int> gnh::xcd_order(const std::vector<int64_t>& weight) {
  constexpr int X = 8;
  const int n = (int)weight.size();
  std::vector<int> byw(n);
  for (int j = 0; j < n; ++j) byw[j] = j;
  std::stable_sort(byw.begin(), byw.end(), [&](int a, int c) { return weight[a] > weight[c]; });
  std::vector<std::vector<int>> on(X);
  std::vector<int64_t> load(X, 0);
  for (int j : byw) {
    int best = -1;
    for (int x = 0; x < X; ++x) {
      const int cap = x < n ? (n - 1 - x) / X + 1 : 0;   // positions q < n with q % X == x
      if ((int)on[x].size() < cap && (best < 0 || load[x] < load[best])) best = x;
    }
    on[best].push_back(j);
    load[best] += weight[j];
  }
  std::vector<int> order(n);
  for (int x = 0; x < X; ++x)
    for (size_t i = 0; i < on[x].size(); ++i) order[i * X + x] = on[x][i];
  return order;
}
// device copies of the descriptors: natural order and the two XCD-balanced orders
static void upload_descs(gn_precond* pc, hipStream_t s) {
  const int n = pc->n_sub;
  for (int q = 0; q < n; ++q) {
    pc->subxI[q] = pc->sub[pc->xorderI[q]];
    pc->subxB[q] = pc->sub[pc->xorderB[q]];
  }
  GN_HIP(hipMemcpyAsync(pc->d_sub, pc->sub.data(), sizeof(SubDesc) * n, hipMemcpyHostToDevice, s));
  GN_HIP(hipMemcpyAsync(pc->d_subxI, pc->subxI.data(), sizeof(SubDesc) * n, hipMemcpyHostToDevice, s));
  GN_HIP(hipMemcpyAsync(pc->d_subxB, pc->subxB.data(), sizeof(SubDesc) * n, hipMemcpyHostToDevice, s));
}
PouDev gnh::pou_dev(const gn_problem* p, const gn_precond* pc) {
  PouDev d;
  for (int a = 0; a < 3; ++a) {
    d.cnt[a] = pc->d_cnt[a];
    d.plo[a] = pc->d_plo[a];
    d.ecnt[a] = pc->d_ecnt[a];
    d.er0[a] = pc->d_er0[a];
    d.er1[a] = pc->d_er1[a];
    d.ne[a] = p->ne[a];
  }
  d.kind = pc->pou;
  return d;
}
double gnh::now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
using gnh::now_s;

int64_t gnh::resident_bytes(const std::vector<void*>& owned) {
  int64_t t = 0;
  for (void* q : owned) t += gnh::dev_size(q);
  return t;
}

// ---------------------------------------------------------------------------
// kernel-group profiling with HIP events
// ---------------------------------------------------------------------------
namespace {
struct ProfRec {
  int group;
  double bytes;
  hipEvent_t e0, e1;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
double g_prof_ms[PROF_NGROUP] = {0};
double g_prof_bytes[PROF_NGROUP] = {0};
int64_t g_prof_n[PROF_NGROUP] = {0};
const char* g_prof_names[PROF_NGROUP] = {"spmv", "trsv", "prolong", "coarse", "vec"};

void prof_drain() {
  for (auto& r : g_prof_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
      g_prof_ms[r.group] += ms;
      g_prof_bytes[r.group] += r.bytes;
      g_prof_n[r.group] += 1;
    }
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  g_prof_pending.clear();
}
}  // namespace

GnProfScope::GnProfScope(int g, double b, hipStream_t st) : group(g), bytes(b), s(st), on(false) {
  if (!g_prof_on) return;
  if (hipEventCreate(&e0) != hipSuccess) return;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return;
  }
  (void)hipEventRecord(e0, s);
  on = true;
}
GnProfScope::~GnProfScope() {
  if (!on) return;
  (void)hipEventRecord(e1, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_pending.push_back(ProfRec{group, bytes, e0, e1});
}

extern "C" gn_status gn_profile_enable(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_drain();
  g_prof_on = enable != 0;
  for (int i = 0; i < PROF_NGROUP; ++i) g_prof_ms[i] = g_prof_bytes[i] = 0.0, g_prof_n[i] = 0;
  return GN_OK;
}

extern "C" gn_status gn_profile_read(const char* group, double* total_ms, int64_t* launches,
                                     double* bytes) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_drain();
  for (int i = 0; i < PROF_NGROUP; ++i) {
    if (group && std::strcmp(group, g_prof_names[i]) == 0) {
      if (total_ms) *total_ms = g_prof_ms[i];
      if (launches) *launches = g_prof_n[i];
      if (bytes) *bytes = g_prof_bytes[i];
      return GN_OK;
    }
  }
  gn_set_error(GN_ERR_ARG, "unknown profile group");
  return GN_ERR_ARG;
}

// ---------------------------------------------------------------------------
// assembly
// ---------------------------------------------------------------------------
// Element matrices, A and b from the inputs held on the device (eqn:fe_matrix_system).
static void assemble_on_device(gn_problem* p, hipStream_t s) {
  gnk::element_matrices(p, p->d_mats, p->n_mat, p->d_emat, p->d_eang, p->d_etilt, p->d_ek, s);
  gnk::assemble_matrix(p, s);
  gnk::assemble_load(p, p->d_body, p->d_trac, p->nrhs, p->d_b, s);
  GN_HIP(hipStreamSynchronize(s));
}

extern "C" gn_status gn_assemble(const gn_grid* grid, const gn_material* mat, const gn_loads* loads,
                                 void* stream, gn_problem** out) {
  if (out) *out = nullptr;
  gn_problem* p = nullptr;
  GN_TRY
  if (!grid || !mat || !loads || !out) argfail("null argument");
  hipStream_t s = (hipStream_t)stream;
  for (int a = 0; a < 3; ++a) {
    if (grid->ne[a] < 1) argfail("ne must be >= 1 on every axis");
    if (!grid->xn[a]) argfail("missing node coordinates");
    for (int i = 0; i < grid->ne[a]; ++i)
      if (!(grid->xn[a][i + 1] > grid->xn[a][i])) argfail("node coordinates must increase");
  }
  if (mat->pde != 0 && mat->pde != 1) argfail("pde must be 0 (diffusion) or 1 (elasticity)");
  if (grid->map_kind != 0 && grid->map_kind != 1) argfail("map_kind must be 0 or 1");
  if (grid->map_kind == 1 && !grid->map_par) argfail("ramp map needs map_par");
  if (!loads->dirichlet) argfail("missing Dirichlet mask");
  if (loads->nrhs < 1) argfail("nrhs must be >= 1");
  p = new gn_problem();
  p->pde = mat->pde;
  p->nc = mat->pde == 1 ? 3 : 1;
  for (int a = 0; a < 3; ++a) {
    p->ne[a] = grid->ne[a];
    p->nn[a] = grid->ne[a] + 1;
  }
  p->n_node = (int64_t)p->nn[0] * p->nn[1] * p->nn[2];
  p->n_elem = (int64_t)p->ne[0] * p->ne[1] * p->ne[2];
  p->n_dof = p->n_node * p->nc;
  if (p->n_dof >= (int64_t)1 << 31) argfail("problem too large for 32-bit DOF indices");
  p->nrhs = loads->nrhs;
  p->map_kind = grid->map_kind;
  if (grid->map_kind == 1)
    for (int a = 0; a < 3; ++a) p->map_par[a] = grid->map_par[a];
  const int nc = p->nc;
  // host-side validation of element data
  if (p->pde == 1) {
    if (!mat->mat || !mat->elem_mat || mat->n_mat < 1) argfail("elasticity needs materials");
    for (int m = 0; m < mat->n_mat; ++m) {
      const double* c = mat->mat + 9 * m;
      for (int k = 0; k < 6; ++k)
        if (!(c[k] > 0.0)) argfail("moduli must be positive");
    }
    for (int64_t e = 0; e < p->n_elem; ++e)
      if (mat->elem_mat[e] < 0 || mat->elem_mat[e] >= mat->n_mat) argfail("elem_mat out of range");
  } else {
    if (!mat->elem_k) argfail("diffusion needs elem_k");
    for (int64_t e = 0; e < p->n_elem; ++e)
      if (!(mat->elem_k[e] > 0.0) || !std::isfinite(mat->elem_k[e])) argfail("elem_k must be positive");
  }
  if (loads->body)
    for (int64_t i = 0; i < p->n_elem * nc; ++i)
      if (!std::isfinite(loads->body[i])) argfail("non-finite body force");
  if (loads->traction)
    for (int64_t i = 0; i < (int64_t)loads->nrhs * p->ne[0] * p->ne[1] * nc; ++i)
      if (!std::isfinite(loads->traction[i])) argfail("non-finite traction");
  // free numbering
  std::vector<int> f2f;
  f2f.reserve((size_t)p->n_dof);
  for (int64_t d = 0; d < p->n_dof; ++d)
    if (!loads->dirichlet[d]) f2f.push_back((int)d);
  p->n_free = (int64_t)f2f.size();
  if (p->n_free == 0) argfail("no free DOFs");
  for (int a = 0; a < 3; ++a) p->d_xn[a] = upload(p->owned, grid->xn[a], (size_t)p->nn[a], s);
  p->d_dir = upload(p->owned, loads->dirichlet, (size_t)p->n_dof, s);
  p->h_dir.assign(loads->dirichlet, loads->dirichlet + p->n_dof);
  p->d_free2full = upload(p->owned, f2f.data(), f2f.size(), s);
  const int nd = 8 * nc;
  p->d_Ke = dalloc<double>(p->owned, (size_t)p->n_elem * nd * nd);
  p->d_A = dalloc<double>(p->owned, (size_t)p->n_node * 27 * nc * nc);
  p->d_b = dalloc<double>(p->owned, (size_t)p->n_dof * p->nrhs);
  // the inputs stay on the device with the problem (gn_reassemble)
  if (p->pde == 1) {
    p->n_mat = mat->n_mat;
    p->d_mats = upload(p->owned, mat->mat, (size_t)9 * mat->n_mat, s);
    p->d_emat = upload(p->owned, mat->elem_mat, (size_t)p->n_elem, s);
    if (mat->elem_angle) p->d_eang = upload(p->owned, mat->elem_angle, (size_t)p->n_elem, s);
    if (mat->elem_tilt) p->d_etilt = upload(p->owned, mat->elem_tilt, (size_t)p->n_elem, s);
  } else {
    p->d_ek = upload(p->owned, mat->elem_k, (size_t)p->n_elem, s);
  }
  if (loads->body) p->d_body = upload(p->owned, loads->body, (size_t)p->n_elem * nc, s);
  if (loads->traction)
    p->d_trac = upload(p->owned, loads->traction, (size_t)loads->nrhs * p->ne[0] * p->ne[1] * nc, s);
  assemble_on_device(p, s);
  // CG workspace
  p->d_x = dalloc<double>(p->owned, (size_t)p->n_dof);
  p->d_r = dalloc<double>(p->owned, (size_t)p->n_dof);
  p->d_p = dalloc<double>(p->owned, (size_t)p->n_dof);
  p->d_q = dalloc<double>(p->owned, (size_t)p->n_dof);
  p->d_z = dalloc<double>(p->owned, (size_t)p->n_dof);
  int nb = std::max(std::max(gnk::spmv_blocks(p), gnk::reduce_blocks()), gnk::prolong_blocks(p));
  p->d_part = dalloc<double>(p->owned, (size_t)nb);
  p->d_scal = dalloc<double>(p->owned, 64);
  p->d_count = dalloc<unsigned>(p->owned, 1);
  GN_HIP(hipMemsetAsync(p->d_p, 0, sizeof(double) * p->n_dof, s));
  GN_HIP(hipMemsetAsync(p->d_scal, 0, sizeof(double) * 64, s));
  GN_HIP(hipStreamSynchronize(s));
  *out = p;
  return GN_OK;
  }
  catch (const gn_error& e) {
    if (p) { dfree_all(p->owned); delete p; }
    gn_set_error(e.code, e.msg);
    return e.code;
  }
  catch (...) {
    if (p) { dfree_all(p->owned); delete p; }
    gn_set_error(GN_ERR_DEVICE, "unexpected exception in gn_assemble");
    return GN_ERR_DEVICE;
  }
}

extern "C" gn_status gn_reassemble(gn_problem* p, void* stream) {
  if (!p) {
    gn_set_error(GN_ERR_ARG, "null problem");
    return GN_ERR_ARG;
  }
  try {
    assemble_on_device(p, (hipStream_t)stream);
    return GN_OK;
  } catch (const gn_error& e) {
    gn_set_error(e.code, e.msg);
    return e.code;
  } catch (...) {
    gn_set_error(GN_ERR_DEVICE, "unexpected exception in gn_reassemble");
    return GN_ERR_DEVICE;
  }
}

extern "C" gn_status gn_problem_info(const gn_problem* p, int64_t* n_free, int64_t* nnz, int32_t* nrhs) {
  if (!p) {
    gn_set_error(GN_ERR_ARG, "null problem");
    return GN_ERR_ARG;
  }
  if (n_free) *n_free = p->n_free;
  if (nnz) *nnz = p->n_node * 27 * p->nc * p->nc;
  if (nrhs) *nrhs = p->nrhs;
  return GN_OK;
}

extern "C" gn_status gn_problem_rhs(const gn_problem* p, double* b_dev, int64_t ld, void* stream) {
  GN_TRY
  if (!p || !b_dev) argfail("null argument");
  if (ld < p->n_free) argfail("ld < n_free");
  hipStream_t s = (hipStream_t)stream;
  for (int c = 0; c < p->nrhs; ++c) gnk::gather_free(p, p->d_b + (int64_t)c * p->n_dof, b_dev + c * ld, s);
  return GN_OK;
  GN_CATCH
}

extern "C" gn_status gn_load_vectors(gn_problem* p, const double* body, int32_t nrhs, const double* traction,
                                     double* b_dev, int64_t ld, void* stream) {
  GN_TRY
  if (!p || !b_dev) argfail("null argument");
  if (nrhs < 1 || ld < p->n_free) argfail("bad nrhs/ld");
  hipStream_t s = (hipStream_t)stream;
  const int nc = p->nc;
  if (body)
    for (int64_t i = 0; i < p->n_elem * nc; ++i)
      if (!std::isfinite(body[i])) argfail("non-finite body force");
  if (traction)
    for (int64_t i = 0; i < (int64_t)nrhs * p->ne[0] * p->ne[1] * nc; ++i)
      if (!std::isfinite(traction[i])) argfail("non-finite traction");
  std::vector<void*> tmp;
  try {
    const double *d_body = nullptr, *d_trac = nullptr;
    if (body) d_body = upload(tmp, body, (size_t)p->n_elem * nc, s);
    if (traction) d_trac = upload(tmp, traction, (size_t)nrhs * p->ne[0] * p->ne[1] * nc, s);
    double* d_full = dalloc<double>(tmp, (size_t)p->n_dof * nrhs);
    gnk::assemble_load(p, d_body, d_trac, nrhs, d_full, s);
    for (int c = 0; c < nrhs; ++c) gnk::gather_free(p, d_full + (int64_t)c * p->n_dof, b_dev + c * ld, s);
    GN_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    dfree_all(tmp);
    throw;
  }
  dfree_all(tmp);
  return GN_OK;
  GN_CATCH
}

// ---------------------------------------------------------------------------
// load vectors without allocation: the staging of the host loads and the
// full-numbering load live in a static device array
// ---------------------------------------------------------------------------
#define GN_SCRATCH_DOUBLES ((size_t)4 << 20)     // 32 MiB per device
static __device__ __align__(256) double scratch[GN_SCRATCH_DOUBLES];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {nullptr};
// device address of this device's copy of `scratch` (looked up once per device)
double* scratch_address() {
  int dev = 0;
  GN_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw gn_error{GN_ERR_DEVICE, "device index beyond the static workspace table"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    GN_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = (double*)ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" gn_status gn_load_vectors_noalloc(gn_problem* p, const double* body, int32_t nrhs,
                                             const double* traction, double* b_dev, int64_t ld, void* stream) {
  GN_TRY
  if (!p || !b_dev) argfail("null argument");
  if (nrhs < 1 || ld < p->n_free) argfail("bad nrhs/ld");
  hipStream_t s = (hipStream_t)stream;
  const int nc = p->nc;
  const int64_t nbody = body ? p->n_elem * nc : 0;
  const int64_t ntrac = traction ? (int64_t)nrhs * p->ne[0] * p->ne[1] * nc : 0;
  auto pad = [](int64_t n) { return (n + 31) / 32 * 32; };
  const int64_t need = pad(nbody) + pad(ntrac) + p->n_dof * nrhs;
  if (need > (int64_t)GN_SCRATCH_DOUBLES)
    argfail("load vectors need " + std::to_string(need * 8) + " bytes of workspace; the static workspace holds " +
            std::to_string(GN_SCRATCH_DOUBLES * 8) + " (use gn_load_vectors)");
  for (int64_t i = 0; i < nbody; ++i)
    if (!std::isfinite(body[i])) argfail("non-finite body force");
  for (int64_t i = 0; i < ntrac; ++i)
    if (!std::isfinite(traction[i])) argfail("non-finite traction");
  double* ws = scratch_address();
  double* d_body = body ? ws : nullptr;
  double* d_trac = traction ? ws + pad(nbody) : nullptr;
  double* d_full = ws + pad(nbody) + pad(ntrac);   // every entry is written by the load kernel
  if (body) GN_HIP(hipMemcpyAsync(d_body, body, sizeof(double) * nbody, hipMemcpyHostToDevice, s));
  if (traction) GN_HIP(hipMemcpyAsync(d_trac, traction, sizeof(double) * ntrac, hipMemcpyHostToDevice, s));
  gnk::assemble_load(p, d_body, d_trac, nrhs, d_full, s);
  for (int c = 0; c < nrhs; ++c) gnk::gather_free(p, d_full + (int64_t)c * p->n_dof, b_dev + c * ld, s);
  GN_HIP(hipStreamSynchronize(s));
  return GN_OK;
  GN_CATCH
}

extern "C" gn_status gn_matvec(gn_problem* p, const double* x_dev, double* y_dev, int32_t ncol,
                               int64_t ld, void* stream) {
  GN_TRY
  if (!p || !x_dev || !y_dev) argfail("null argument");
  if (ncol < 1 || ld < p->n_free) argfail("bad ncol/ld");
  hipStream_t s = (hipStream_t)stream;
  for (int c = 0; c < ncol; ++c) {
    gnk::scatter_free(p, x_dev + c * ld, p->d_p, s);
    gnk::spmv_flag(p, p->d_p, p->d_q, nullptr, nullptr, s);
    gnk::gather_free(p, p->d_q, y_dev + c * ld, s);
  }
  return GN_OK;
  GN_CATCH
}

// ---------------------------------------------------------------------------
// decomposition + GenEO set-up
// ---------------------------------------------------------------------------
namespace {

struct BandRefH {
  int64_t offT, offD;
  int NB, w;
};

void axis_perm(const int n[3], int perm[3]) {
  perm[0] = 0, perm[1] = 1, perm[2] = 2;
  std::stable_sort(perm, perm + 3, [&](int a, int b) { return n[a] < n[b]; });
}

int band_width_dofs(const int n[3], const int perm[3], int nc) {
  int64_t d0 = n[perm[0]], d1 = n[perm[1]];
  return (int)((1 + d0 + d0 * d1) * nc + nc - 1);
}

// eigenvalues of a symmetric tridiagonal matrix by Sturm bisection
void tridiag_extremes(const std::vector<double>& d, const std::vector<double>& e, double* lo, double* hi) {
  int n = (int)d.size();
  double gl = 1e300, gu = -1e300;
  for (int i = 0; i < n; ++i) {
    double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    gl = std::min(gl, d[i] - r);
    gu = std::max(gu, d[i] + r);
  }
  auto count_below = [&](double x) {
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
      double e2 = i > 0 ? e[i - 1] * e[i - 1] : 0.0;
      q = d[i] - x - (i > 0 ? e2 / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  auto kth = [&](int k) {  // k-th smallest (0-based)
    double a = gl, b = gu;
    for (int it = 0; it < 200; ++it) {
      double m = 0.5 * (a + b);
      if (count_below(m) > k) b = m; else a = m;
      if (b - a <= 1e-15 * std::max(std::fabs(a), std::fabs(b))) break;
    }
    return 0.5 * (a + b);
  };
  *lo = kth(0);
  *hi = kth(n - 1);
}

}  // namespace

// Overlapping decomposition on the host (Section 3.1): per-axis element ranges
// of the parts extended by the overlap, their V_h0 (I) node ranges, coverage
// counts, and the subdomain descriptors with their band widths and storage
// offsets.  Shared by the set-up and by the a-priori footprint.
struct DdPlan {
  std::vector<int> eR0[3], eR1[3], iR0[3], iR1[3];
  std::vector<int> cnt[3], plo[3], ec[3];
  std::vector<SubDesc> sub;
  int64_t offTI = 0, offDI = 0, offVI = 0, offTB = 0, offDB = 0, offVB = 0;
  int maxNBI = 0, maxNBB = 0, maxNI = 0, maxNB = 0, maxw = 0, maxwB = 0;
};

static DdPlan plan_decomposition(const int ne_[3], int nc, const gn_dd_opts* o) {
  for (int a = 0; a < 3; ++a) {
    if (o->nparts[a] < 1) argfail("nparts must be >= 1");
    if (!o->cuts[a]) argfail("missing cuts");
    if (o->cuts[a][0] != 0 || o->cuts[a][o->nparts[a]] != ne_[a]) argfail("cuts must span 0..ne");
    for (int q = 0; q < o->nparts[a]; ++q)
      if (o->cuts[a][q + 1] <= o->cuts[a][q]) argfail("cuts must increase");
  }
  const int n_sub = o->nparts[0] * o->nparts[1] * o->nparts[2];
  if (n_sub > 1 && o->overlap < 1) argfail("overlap must be >= 1");
  const int O = std::max(o->overlap, 0);
  DdPlan pl;
  for (int a = 0; a < 3; ++a) {
    const int P = o->nparts[a], ne = ne_[a];
    pl.cnt[a].assign(ne + 1, 0);
    pl.plo[a].assign(ne + 1, -1);
    pl.ec[a].assign(ne, 0);
    for (int q = 0; q < P; ++q) {
      const int e0 = std::max(0, o->cuts[a][q] - O), e1 = std::min(ne, o->cuts[a][q + 1] + O);
      const int i0 = e0 + (e0 > 0 ? 1 : 0), i1 = e1 - (e1 < ne ? 1 : 0);   // inclusive node range
      pl.eR0[a].push_back(e0);
      pl.eR1[a].push_back(e1);
      pl.iR0[a].push_back(i0);
      pl.iR1[a].push_back(i1);
      for (int i = i0; i <= i1; ++i) {
        if (pl.cnt[a][i] == 0) pl.plo[a][i] = q;
        ++pl.cnt[a][i];
      }
      for (int e = e0; e < e1; ++e) ++pl.ec[a][e];
    }
    for (int i = 0; i <= ne; ++i)
      if (pl.cnt[a][i] == 0) argfail("a node lies in no subdomain interior: overlap too small");
    for (int i = 0; i <= ne; ++i)
      if (pl.cnt[a][i] > 0)
        for (int q = pl.plo[a][i]; q < pl.plo[a][i] + pl.cnt[a][i]; ++q)
          if (i < pl.iR0[a][q] || i > pl.iR1[a][q]) argfail("non-contiguous subdomain cover");
  }
  pl.sub.resize(n_sub);
  for (int r = 0; r < o->nparts[2]; ++r)
    for (int q = 0; q < o->nparts[1]; ++q)
      for (int pp = 0; pp < o->nparts[0]; ++pp) {
        const int j = pp + o->nparts[0] * (q + o->nparts[1] * r);
        SubDesc& sd = pl.sub[j];
        std::memset(&sd, 0, sizeof(sd));
        sd.id = j;
        const int idx[3] = {pp, q, r};
        for (int a = 0; a < 3; ++a) {
          sd.elo[a] = pl.eR0[a][idx[a]];
          sd.ehi[a] = pl.eR1[a][idx[a]];
          sd.ilo[a] = pl.iR0[a][idx[a]];
          sd.in_[a] = pl.iR1[a][idx[a]] - pl.iR0[a][idx[a]] + 1;
          sd.blo[a] = sd.elo[a];
          sd.bn[a] = sd.ehi[a] - sd.elo[a] + 1;
        }
        axis_perm(sd.in_, sd.permI);
        axis_perm(sd.bn, sd.permB);
        sd.nI = sd.in_[0] * sd.in_[1] * sd.in_[2] * nc;
        sd.nB = sd.bn[0] * sd.bn[1] * sd.bn[2] * nc;
        sd.NBI = (sd.nI + TILE - 1) / TILE;
        sd.NBB = (sd.nB + TILE - 1) / TILE;
        sd.bwI = std::min(sd.nI - 1, band_width_dofs(sd.in_, sd.permI, nc));
        sd.bwB = std::min(sd.nB - 1, band_width_dofs(sd.bn, sd.permB, nc));
        sd.wI = std::max(std::min(sd.NBI - 1, (band_width_dofs(sd.in_, sd.permI, nc) + TILE - 1) / TILE), 0);
        sd.wB = std::max(std::min(sd.NBB - 1, (band_width_dofs(sd.bn, sd.permB, nc) + TILE - 1) / TILE), 0);
        // the single-column sweep finds entries outside the band only in its two
        // outermost band tiles, which needs 32 w - bw < 32
        if (TILE * sd.wI - sd.bwI > TILE - 1 || sd.bwI < 0)
          throw gn_error{GN_ERR_DEVICE, "band planner: inconsistent band width in tiles"};
        sd.offTI = pl.offTI;
        sd.offDI = pl.offDI;
        sd.offVI = pl.offVI;
        sd.offTB = pl.offTB;
        sd.offDB = pl.offDB;
        sd.offVB = pl.offVB;
        pl.offTI += (int64_t)sd.NBI * (sd.wI + 1);
        pl.offDI += sd.NBI;
        pl.offVI += (int64_t)sd.NBI * TILE;
        pl.offTB += (int64_t)sd.NBB * (sd.wB + 1);
        pl.offDB += sd.NBB;
        pl.offVB += (int64_t)sd.NBB * TILE;
        pl.maxNBI = std::max(pl.maxNBI, sd.NBI);
        pl.maxNBB = std::max(pl.maxNBB, sd.NBB);
        pl.maxNI = std::max(pl.maxNI, sd.nI);
        pl.maxNB = std::max(pl.maxNB, sd.nB);
        pl.maxw = std::max(pl.maxw, sd.wI);
        pl.maxwB = std::max(pl.maxwB, sd.wB);
      }
  return pl;
}

// Resident device bytes of an operator and its preconditioner from the sizes
// alone (no device work): every allocation that gn_assemble, gn_setup_geneo,
// the first solve (history of maxit iterations) and the batched workspace make
// and keep, each rounded as the allocator rounds it.  The mask is unknown
// here, so the free-to-full map is counted for every DOF; m_j is nev (fixed
// count), nev_max (threshold: an upper bound) or the mode count (zero-energy
// modes, every subdomain taken as floating).
static int64_t estimate_footprint(const int ne[3], int nc, const gn_dd_opts* o, int nrhs, int maxit,
                                  bool batched) {
  int64_t t = 0;
  auto add = [&](int64_t bytes) { t += (int64_t)pool_round((size_t)std::max<int64_t>(bytes, 1)); };
  const int64_t nn[3] = {ne[0] + 1, ne[1] + 1, ne[2] + 1};
  const int64_t n_node = nn[0] * nn[1] * nn[2], n_elem = (int64_t)ne[0] * ne[1] * ne[2];
  const int64_t n_dof = n_node * nc, nd = 8 * nc;
  const int KC = gnk::mc_width();
  // problem
  for (int a = 0; a < 3; ++a) add(nn[a] * 8);
  add(n_dof);
  add(n_dof * 4);
  add(n_elem * nd * nd * 8);
  add(n_node * 27 * nc * nc * 8);
  add(n_dof * nrhs * 8);
  // the assembly's inputs kept with the problem, every optional array counted
  if (nc == 3) {
    add(9 * 8);            // material rows (a few)
    add(n_elem * 4);       // element material ids
    add(n_elem * 8);       // ply angles
    add(n_elem * 8);       // tilts
  } else {
    add(n_elem * 8);       // conductivities
  }
  add(n_elem * nc * 8);                         // body force
  add((int64_t)nrhs * ne[0] * ne[1] * nc * 8);  // top-face tractions
  for (int v = 0; v < 5; ++v) add(n_dof * 8);
  const int64_t pstride = std::max<int64_t>((n_node + 255) / 256, gnk::reduce_blocks());
  add(pstride * 8);
  add(64 * 8);
  add(4);
  add((2 * (int64_t)maxit + 2) * 8);
  if (batched) {
    for (int v = 0; v < 5; ++v) add(n_dof * KC * 8);
    add(pstride * KC * 8);
    add((int64_t)S_N * KC * 8);
    add((2 * (int64_t)maxit + 2) * KC * 8);
  }
  if (!o) return t;
  // preconditioner
  const DdPlan pl = plan_decomposition(ne, nc, o);
  const int n_sub = (int)pl.sub.size();
  for (int a = 0; a < 3; ++a) {
    add(nn[a] * 4);
    add(nn[a] * 4);
    add((int64_t)ne[a] * 4);
    add((int64_t)o->nparts[a] * 4);
    add((int64_t)o->nparts[a] * 4);
  }
  for (int c = 0; c < 3; ++c) add((int64_t)std::max(n_sub, 1) * (int64_t)sizeof(SubDesc));
  const int64_t fb = o->local_prec == 32 ? 4 : 8;
  add(pl.offTI * TILE2 * fb);                 // backward (transposed) band
  add(pl.offTI * TILE2 * fb);                 // forward band
  add(pl.offDI * TILE2 * fb);                 // inverse diagonal tiles
  add(pl.offVI * 8);
  add(TILE2 * 8);
  add(TILE2 * 4);
  int64_t NH = 0, phi = 0;
  if (o->coarse != 0 && n_sub > 1) {
    const int m = o->coarse == 2 ? (nc == 3 ? 6 : 1) : (o->nev > 0 ? o->nev : o->nev_max);
    for (const SubDesc& sd : pl.sub) {
      NH += m;
      phi += (int64_t)sd.nI * m;
    }
  }
  const int64_t NBH = (NH + TILE - 1) / TILE;
  if (NH > 0) {
    add(phi * 8);
    if (o->coarse_solve == 1) {
      // block-sparse A_H over the interacting subdomain pairs, inverted diagonal
      // blocks, inner CG vectors and partial sums
      const int m = (int)(NH / n_sub);
      int64_t blocks = 0;
      for (int j1 = 0; j1 < n_sub; ++j1)
        for (int j2 = 0; j2 < n_sub; ++j2) {
          bool hit12 = true, hit21 = true;
          for (int a = 0; a < 3; ++a) {
            const SubDesc &s1 = pl.sub[j1], &s2 = pl.sub[j2];
            hit12 &= std::min(s1.ilo[a] + s1.in_[a], s2.blo[a] + s2.bn[a]) > std::max(s1.ilo[a], s2.blo[a]);
            hit21 &= std::min(s2.ilo[a] + s2.in_[a], s1.blo[a] + s1.bn[a]) > std::max(s2.ilo[a], s1.blo[a]);
          }
          blocks += (hit12 || hit21) ? 1 : 0;
        }
      add((int64_t)(n_sub + 1) * 4);
      add(blocks * (int64_t)sizeof(BsrBlock));
      add(blocks * m * m * 8);
      add((int64_t)n_sub * 8);
      add((int64_t)n_sub * m * m * 8);
      add(5 * NBH * TILE * 8);
      add(3 * 256 * 8);
      add(4 * 8);
    } else {
      // Z (Z^T in its upper tiles), the transposed diagonal tiles, the unit
      // tables and row starts of the coarse products, their partial sums
      add(NBH * NBH * TILE2 * 8);
      add(NBH * TILE2 * 8);
      const int64_t uf = gnk::coarse_units(NBH, false), ub = gnk::coarse_units(NBH, true);
      add(uf * (int64_t)sizeof(int4));
      add(ub * (int64_t)sizeof(int4));
      add((NBH + 1) * 4);
      add((NBH + 1) * 4);
      add(std::max(uf, ub) * TILE * 8);
    }
    for (int v = 0; v < 3; ++v) add(NBH * TILE * 8);
  }
  if (batched) {
    add(pl.offVI * KC * 8);
    for (int v = 0; v < 3; ++v) add(std::max<int64_t>(NBH, 1) * TILE * KC * 8);
  }
  return t;
}

extern "C" gn_status gn_footprint(const gn_grid* grid, int32_t pde, const gn_dd_opts* opts, int64_t* bytes) {
  GN_TRY
  if (!grid || !bytes) argfail("null argument");
  if (pde != 0 && pde != 1) argfail("pde must be 0 (diffusion) or 1 (elasticity)");
  for (int a = 0; a < 3; ++a)
    if (grid->ne[a] < 1) argfail("ne must be >= 1 on every axis");
  if (opts && opts->local_prec != 64 && opts->local_prec != 32) argfail("local_prec must be 64 or 32");
  *bytes = estimate_footprint(grid->ne, pde == 1 ? 3 : 1, opts, 1, 2000, true);
  return GN_OK;
  GN_CATCH
}

extern "C" gn_status gn_setup_geneo(gn_problem* p, const gn_dd_opts* o, void* stream, gn_precond** out,
                                    gn_setup_report* rep) {
  if (out) *out = nullptr;
  gn_precond* pc = nullptr;
  std::vector<void*> tmp;
  GN_TRY
  if (!p || !o || !out) argfail("null argument");
  hipStream_t s = (hipStream_t)stream;
  const double t0 = now_s();
  const double ta0 = gnh::dev_alloc_seconds();
  const int nc = p->nc;
  for (int a = 0; a < 3; ++a) {
    if (o->nparts[a] < 1) argfail("nparts must be >= 1");
    if (!o->cuts[a]) argfail("missing cuts");
  }
  const int n_sub = o->nparts[0] * o->nparts[1] * o->nparts[2];
  if (n_sub > 1 && o->overlap < 1) argfail("overlap must be >= 1");
  if (o->local_prec != 64 && o->local_prec != 32) argfail("local_prec must be 64 or 32");
  const int O = std::max(o->overlap, 0);
  const double shift = o->shift > 0 ? o->shift : 1e-2;
  const double eig_tol = o->eig_tol > 0 ? o->eig_tol : 1e-12;
  if (o->eig_refine < 0 || o->eig_refine > 8) argfail("eig_refine must lie in [0, 8]");
  const int eig_refine = o->eig_refine > 0 ? o->eig_refine : 1;
  const int eig_maxit = o->eig_maxit > 0 ? o->eig_maxit : 300;
  if (o->eig_filter < 0 || o->eig_filter > 8) argfail("eig_filter must lie in [0, 8]");
  if (o->coarse < 0 || o->coarse > 2) argfail("coarse must be 0, 1 or 2");
  if (o->coarse == 1 && o->nev <= 0 && !(o->threshold > 0)) argfail("coarse space needs nev > 0 or threshold > 0");
  if (o->coarse == 1 && o->nev > 48) argfail("nev must be <= 48");
  if (o->coarse == 1 && o->nev <= 0 && (o->nev_max <= 0 || o->nev_max > 48))
    argfail("threshold mode needs 0 < nev_max <= 48");
  pc = new gn_precond();
  pc->prob = p;
  pc->n_sub = n_sub;
  pc->overlap = O;
  pc->local_prec = o->local_prec;
  if (o->pou < 0 || o->pou > 1) argfail("pou must be 0 (standard) or 1 (smooth)");
  pc->pou = o->pou;
  if (o->coarse_solve < 0 || o->coarse_solve > 1) argfail("coarse_solve must be 0 (exact) or 1 (inexact CG)");
  if (o->coarse_rtol < 0 || o->coarse_maxit < 0) argfail("coarse_rtol and coarse_maxit must not be negative");
  pc->coarse_solve = o->coarse_solve;
  pc->coarse_rtol = o->coarse_rtol > 0 ? o->coarse_rtol : 1e-4;
  pc->coarse_maxit = o->coarse_maxit > 0 ? o->coarse_maxit : 200;
  if (o->local_kernel < 0 || o->local_kernel > 4) argfail("local_kernel must lie in [0, 4]");
  pc->local_kernel = o->local_kernel;
  for (int a = 0; a < 3; ++a) {
    pc->nparts[a] = o->nparts[a];
    pc->cuts[a].assign(o->cuts[a], o->cuts[a] + o->nparts[a] + 1);
  }
  const DdPlan plan = plan_decomposition(p->ne, nc, o);
  for (int a = 0; a < 3; ++a) {
    pc->d_cnt[a] = upload(pc->owned, plan.cnt[a].data(), plan.cnt[a].size(), s);
    pc->d_plo[a] = upload(pc->owned, plan.plo[a].data(), plan.plo[a].size(), s);
    pc->d_ecnt[a] = upload(pc->owned, plan.ec[a].data(), plan.ec[a].size(), s);
    pc->d_er0[a] = upload(pc->owned, plan.eR0[a].data(), plan.eR0[a].size(), s);
    pc->d_er1[a] = upload(pc->owned, plan.eR1[a].data(), plan.eR1[a].size(), s);
  }
  pc->sub = plan.sub;
  const int64_t offTI = plan.offTI, offDI = plan.offDI, offVI = plan.offVI, offTB = plan.offTB,
                offDB = plan.offDB, offVB = plan.offVB;
  const int maxNBI = plan.maxNBI, maxNBB = plan.maxNBB, maxNI = plan.maxNI, maxNB_ = plan.maxNB, maxw = plan.maxw;
  (void)offVB;
  pc->tilesI = offTI;
  pc->vecI = offVI;
  pc->maxNBI = maxNBI;
  pc->maxwI = maxw;
  pc->d_sub = upload(pc->owned, pc->sub.data(), pc->sub.size(), s);
  {
    std::vector<int64_t> wI(n_sub), wB(n_sub);
    for (int j = 0; j < n_sub; ++j) {
      wI[j] = (int64_t)pc->sub[j].NBI * (pc->sub[j].wI + 1);
      wB[j] = (int64_t)pc->sub[j].NBB * (pc->sub[j].wB + 1);
    }
    pc->xorderI = gnh::xcd_order(wI);
    pc->xorderB = gnh::xcd_order(wB);
    pc->subxI.resize(n_sub);
    pc->subxB.resize(n_sub);
    pc->d_subxI = dalloc<SubDesc>(pc->owned, (size_t)std::max(n_sub, 1));
    pc->d_subxB = dalloc<SubDesc>(pc->owned, (size_t)std::max(n_sub, 1));
    upload_descs(pc, s);
  }
  int* d_info = dalloc<int>(tmp, (size_t)std::max(n_sub, 1) + 64);
  GN_HIP(hipMemsetAsync(d_info, 0, sizeof(int) * (n_sub + 64), s));
  std::vector<int> info(n_sub + 64);

  // ---- local Dirichlet factors -------------------------------------------
  double* LI = dalloc<double>(tmp, (size_t)offTI * TILE2);
  double* DI = dalloc<double>(tmp, (size_t)offDI * TILE2);
  GN_HIP(hipMemsetAsync(LI, 0, sizeof(double) * (size_t)offTI * TILE2, s));
  gnk::extract_local(p, pc, LI, maxNBI, s);
  std::vector<BandRefH> refs(n_sub);
  for (int j = 0; j < n_sub; ++j) refs[j] = BandRefH{pc->sub[j].offTI, pc->sub[j].offDI, pc->sub[j].NBI, pc->sub[j].wI};
  BandRefH* d_refs = upload(tmp, refs.data(), refs.size(), s);
  // transposed backward band: the backward sweeps stream it like the forward
  // ones; FP64 factors write it as they are computed, FP32 ones convert later
  if (o->local_prec == 32) pc->d_LIb = dalloc<float>(pc->owned, (size_t)offTI * TILE2);
  else pc->d_LIb = dalloc<double>(pc->owned, (size_t)offTI * TILE2);
  const bool tb_done = gnk::band_chol(d_refs, n_sub, pc->maxwI, LI, DI, d_info, s,
                                      o->local_prec == 32 ? nullptr : (double*)pc->d_LIb);
  GN_HIP(hipMemcpyAsync(info.data(), d_info, sizeof(int) * n_sub, hipMemcpyDeviceToHost, s));
  GN_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < n_sub; ++j)
    if (info[j]) throw gn_error{GN_ERR_NOT_SPD, "local matrix of subdomain " + std::to_string(j) +
                                                    " not positive definite (row " + std::to_string(info[j] - 1) + ")"};
  if (!tb_done) gnk::band_transpose(d_refs, n_sub, maxNBI, LI, DI, pc->d_LIb, o->local_prec == 32, s);
  if (o->local_prec == 32) {
    pc->d_LIf = dalloc<float>(pc->owned, (size_t)offTI * TILE2);
    pc->d_DIf = dalloc<float>(pc->owned, (size_t)offDI * TILE2);
    gnk::to_f32((int64_t)offTI * TILE2, LI, pc->d_LIf, s);
    gnk::to_f32((int64_t)offDI * TILE2, DI, pc->d_DIf, s);
  } else {
    // keep the FP64 factor: move ownership from tmp to pc
    tmp.erase(std::remove(tmp.begin(), tmp.end(), (void*)LI), tmp.end());
    tmp.erase(std::remove(tmp.begin(), tmp.end(), (void*)DI), tmp.end());
    pc->owned.push_back(LI);
    pc->owned.push_back(DI);
    pc->d_LI = LI;
    pc->d_DI = DI;
  }
  pc->d_t = dalloc<double>(pc->owned, (size_t)offVI);
  GN_HIP(hipMemsetAsync(pc->d_t, 0, sizeof(double) * offVI, s));
  pc->d_z0 = dalloc<double>(pc->owned, TILE2);
  pc->d_zf = dalloc<float>(pc->owned, TILE2);
  GN_HIP(hipMemsetAsync(pc->d_z0, 0, sizeof(double) * TILE2, s));
  GN_HIP(hipMemsetAsync(pc->d_zf, 0, sizeof(float) * TILE2, s));
  GN_HIP(hipStreamSynchronize(s));
  const double t1 = now_s();
  double t2 = t1, t3 = t1;
  int eig_iters = 0, eig_solves = 0;
  double eig_resid = 0.0;

  // ---- GenEO eigenproblems -------------------------------------------------
  pc->NH = 0;
  if (o->coarse != 0 && n_sub > 1) {
    // columns per subdomain of the basis buffer V (eigen block or mode count)
    int b = 0, maxm = 0;
    double *V = nullptr, *Z = nullptr;
    if (o->coarse == 2) {
      // zero-energy modes: the kernel of the Neumann matrix A_{Omega_j} on the
      // Ibar_j box, present when no node of the box carries a Dirichlet DOF
      b = nc == 3 ? 6 : 1;
      int coff = 0;
      for (int j = 0; j < n_sub; ++j) {
        SubDesc& sd = pc->sub[j];
        bool floating = true;
        for (int k = 0; k < sd.bn[2] && floating; ++k)
          for (int jj = 0; jj < sd.bn[1] && floating; ++jj)
            for (int i = 0; i < sd.bn[0] && floating; ++i) {
              const int64_t node = (sd.blo[0] + i) + (int64_t)p->nn[0] * ((sd.blo[1] + jj) +
                                   (int64_t)p->nn[1] * (sd.blo[2] + k));
              for (int c = 0; c < nc; ++c) floating &= p->h_dir[node * nc + c] == 0;
            }
        sd.m = floating ? b : 0;
        sd.coff = coff;
        coff += sd.m;
        maxm = std::max(maxm, sd.m);
      }
      pc->NH = coff;
      pc->n_eval = 0;
      pc->lam.clear();
      pc->lam_n.assign(n_sub, 0);
      const size_t vlen = (size_t)offVB * b;
      V = dalloc<double>(tmp, vlen + 64);
      Z = dalloc<double>(tmp, vlen + 64);
      GN_HIP(hipMemsetAsync(V, 0, sizeof(double) * (vlen + 64), s));
      upload_descs(pc, s);
      gnk::zem_modes(p, pc, b, maxNBB, V, s);
      if (maxm > 0) gnk::eig_normalise(pc, b, maxm, V, s);
    } else {
    const bool fixed = o->nev > 0;
    const int guard = 8;
    // block size: fixed m_j plus a guard band; threshold mode starts at 32 and
    // grows by 16 (to 64) when the eigenvalues below 1.5 x threshold do not fit
    // (a block of up to 32 columns costs the block solves the same matrix-core
    // work as one of 17: fixed counts take at least 32, which converges in
    // fewer steps)
    b = fixed ? std::min(64, std::max(32, o->nev + std::max(guard, o->nev / 2))) : std::min(32, o->nev_max + guard);
    if (fixed) {
      // never more vectors than the smallest pencil has rows
      int min_nb = 1 << 30;
      for (const SubDesc& sd : pc->sub) min_nb = std::min(min_nb, sd.nB);
      b = std::max(std::min(b, min_nb), std::min(64, o->nev + std::max(guard, o->nev / 2)));
    }
    if (o->eig_block > 0) {
      const int need = (fixed ? o->nev : 0) + 1 + guard / 2;
      if (o->eig_block < need || o->eig_block > 64)
        argfail("eig_block must lie in [" + std::to_string(need) + ", 64]");
      b = o->eig_block;
    }
    bool block_short = false;   // a wanted set reached the guard band of the block
    double* LB = dalloc<double>(tmp, (size_t)offTB * TILE2);
    double* DB = dalloc<double>(tmp, (size_t)offDB * TILE2);
    GN_HIP(hipMemsetAsync(LB, 0, sizeof(double) * (size_t)offTB * TILE2, s));
    // B = X A_O X for the iteration's products and P = A_N + s B for the
    // refinement's, in node-ELL planes, from the same pass over the element
    // matrices as the pencil's band
    double* BE = dalloc<double>(tmp, (size_t)offVB * 27 * nc);
    double* PE = dalloc<double>(tmp, (size_t)offVB * 27 * nc);
    gnk::extract_pencil(p, pc, shift, LB, maxNBB, s, PE, BE);
    for (int j = 0; j < n_sub; ++j) refs[j] = BandRefH{pc->sub[j].offTB, pc->sub[j].offDB, pc->sub[j].NBB, pc->sub[j].wB};
    GN_HIP(hipMemcpyAsync(d_refs, refs.data(), sizeof(BandRefH) * n_sub, hipMemcpyHostToDevice, s));
    GN_HIP(hipMemsetAsync(d_info, 0, sizeof(int) * n_sub, s));
    int maxwB = 0;
    for (const SubDesc& sd : pc->sub) maxwB = std::max(maxwB, sd.wB);
    // the pencils' transposed bands (backward sweeps of the block solves) are
    // written by the factorization as it goes
    double* TBB = dalloc<double>(tmp, (size_t)offTB * TILE2);
    const bool tbb_done = gnk::band_chol(d_refs, n_sub, maxwB, LB, DB, d_info, s, TBB);
    GN_HIP(hipMemcpyAsync(info.data(), d_info, sizeof(int) * n_sub, hipMemcpyDeviceToHost, s));
    GN_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < n_sub; ++j)
      if (info[j]) throw gn_error{GN_ERR_NOT_SPD, "GenEO pencil of subdomain " + std::to_string(j) + " not definite"};
    if (!tbb_done) gnk::band_transpose(d_refs, n_sub, maxNBB, LB, DB, TBB, false, s);

    const bool auto_block = o->eig_block <= 0;
    std::vector<double> h_nu;
    int solves_prev = 0;   // block solves of earlier attempts with a smaller block
    for (;;) {
      const size_t vlen = (size_t)offVB * b;
      // 64 doubles of tail padding: the matrix-core solve reads whole 16-column
      // blocks past column b of the last row (those values are masked out)
      V = dalloc<double>(tmp, vlen + 64);
      Z = dalloc<double>(tmp, vlen + 64);
      double* BV = dalloc<double>(tmp, vlen + 64);
      double* BZ = dalloc<double>(tmp, vlen + 64);
      for (double* t : {V, Z, BV, BZ}) GN_HIP(hipMemsetAsync(t + vlen, 0, sizeof(double) * 64, s));
      const int gsplit = gnk::gram_split();
      double* GP = dalloc<double>(tmp, (size_t)n_sub * gsplit * b * b);
      double* GB = dalloc<double>(tmp, (size_t)n_sub * gsplit * b * b);
      double* resp = dalloc<double>(tmp, (size_t)n_sub * gsplit * 2 * b);
      double* Y = dalloc<double>(tmp, (size_t)n_sub * b * b);
      double* nu = dalloc<double>(tmp, (size_t)n_sub * b);
      double* res = dalloc<double>(tmp, (size_t)n_sub * 2 * b);
      GN_HIP(hipMemsetAsync(nu, 0, sizeof(double) * n_sub * b, s));
      GN_HIP(hipMemsetAsync(d_info, 0, sizeof(int) * n_sub, s));
      gnk::eig_vinit(pc, b, maxNBB, V, s);
      h_nu.assign((size_t)n_sub * b, 0.0);
      std::vector<double> h_res((size_t)n_sub * 2 * b);
      std::vector<double> worst_hist;
      bool converged = false;
      gnk::eig_bapply(p, pc, BE, b, maxNBB, V, BV, s);
      // Chebyshev-filtered subspace iteration: outer iteration it applies a filter
      // of degree d = min(dmax, it + 1) in T = P^-1 B (d block solves), then one
      // Rayleigh-Ritz step; d = 1 is plain subspace iteration
      const int dmax = o->eig_filter > 0 ? o->eig_filter : 4;
      const int ncoef = std::max(2, 2 * dmax - 2);
      double *A1 = nullptr, *B1 = nullptr, *d_coef = nullptr;
      if (dmax > 1) {
        A1 = dalloc<double>(tmp, vlen + 64);
        B1 = dalloc<double>(tmp, vlen + 64);
        for (double* t : {A1, B1}) GN_HIP(hipMemsetAsync(t + vlen, 0, sizeof(double) * 64, s));
        d_coef = dalloc<double>(tmp, (size_t)n_sub * ncoef);
      }
      std::vector<double> h_coef((size_t)n_sub * ncoef, 0.0);
      std::vector<int> solves_hist;
      int solves = 0;
      // Subdomains whose wanted pairs have all converged are locked: the
      // iteration's kernels skip them (h_act[j] = 0 on the host, d_act on the
      // device), so their Ritz pairs stay those that passed the test, and the
      // last iterations cost only what the slowest subdomains need.  Their
      // residual figures and guard-band test are kept from that check.
      std::vector<int> h_act(n_sub, 1);
      std::vector<double> j_worst(n_sub, 0.0), j_strict(n_sub, 0.0);
      std::vector<char> j_short(n_sub, 0);
      int* d_act = dalloc<int>(tmp, n_sub);
      GN_HIP(hipMemcpyAsync(d_act, h_act.data(), sizeof(int) * n_sub, hipMemcpyHostToDevice, s));
      // convergence of the Ritz pairs pnu whose residuals are in h_res
      auto check = [&](const std::vector<double>& pnu) -> bool {
        bool all = true;
        block_short = false;
        double worst = 0.0;          // largest scaled residual over the wanted pairs
        double strict_worst = 0.0;   // largest relative residual of the coarse-space pairs
        for (int j = 0; j < n_sub; ++j) {
          if (!h_act[j]) {
            worst = std::max(worst, j_worst[j]);
            strict_worst = std::max(strict_worst, j_strict[j]);
            block_short |= j_short[j] != 0;
            continue;
          }
          bool jall = true, jshort = false;
          double jworst = 0.0, jstrict = 0.0;
          // wanted pairs: nev+1 (fixed) or those below 1.5*threshold plus one (capped)
          int nw;
          if (fixed) {
            nw = std::min(b - guard / 2, o->nev + 1);
          } else {
            nw = 0;
            for (int k = 0; k < b; ++k) {
              double nk = pnu[(size_t)j * b + k];
              double lam = nk > 0 ? 1.0 / nk - shift : 1e300;
              if (lam < 1.5 * o->threshold) nw = k + 1;
            }
            if (std::min(nw + 1, o->nev_max + 1) > b - guard / 2) jshort = true;
            nw = std::min(std::min(nw + 1, o->nev_max + 1), b - guard / 2);
          }
          // pairs whose eigenvectors enter the coarse space (m_j of them, with a
          // generous cluster margin) need the full residual tolerance; the others
          // only decide m_j through their eigenvalues, whose error is of the order
          // of the squared residual, so sqrt(eig_tol) suffices for them
          auto lam_of = [&](int k) {
            double nk = pnu[(size_t)j * b + k];
            return nk > 0 ? 1.0 / nk - shift : 1e300;
          };
          int nin = 0;
          if (fixed) {
            nin = std::min(o->nev, nw);
          } else {
            while (nin < nw && lam_of(nin) < o->threshold) ++nin;
            nin = std::min(nin, o->nev_max);
          }
          while (nin > 0 && nin < nw && lam_of(nin) - lam_of(nin - 1) <= 1e-6 * std::fabs(lam_of(nin - 1)) + 1e-8)
            ++nin;
          for (int k = 0; k < nw; ++k) {
            double nk = pnu[(size_t)j * b + k];
            double rs = h_res[(size_t)j * 2 * b + k], zz = h_res[(size_t)j * 2 * b + b + k];
            if (nk <= 1e-12 / shift) continue;      // null space of B: lambda = inf
            double rel = zz > 0 ? std::sqrt(rs / zz) : 0.0;
            // scaled so that the tolerance of every pair reads as eig_tol
            const double scaled = k < nin ? rel : rel * (eig_tol / std::sqrt(eig_tol));
            if (!(scaled <= eig_tol)) jall = false;
            if (!(scaled <= jworst)) jworst = std::isfinite(scaled) ? std::max(jworst, scaled) : 1e300;
            if (k < nin && std::isfinite(rel)) jstrict = std::max(jstrict, rel);
          }
          j_worst[j] = jworst;
          j_strict[j] = jstrict;
          j_short[j] = jshort;
          worst = std::max(worst, jworst);
          strict_worst = std::max(strict_worst, jstrict);
          block_short |= jshort;
          if (!jall) all = false;
          else h_act[j] = 0;
        }
        GN_HIP(hipMemcpyAsync(d_act, h_act.data(), sizeof(int) * n_sub, hipMemcpyHostToDevice, s));
        worst_hist.push_back(worst);
        solves_hist.push_back(solves);
        eig_resid = strict_worst;
        // accept a residual that has reached the rounding floor: no halving over
        // the last 15 block solves once it is below 1e-9
        bool stagnated = false;
        if (solves > 20 && worst <= 1e-9) {
          for (size_t q = worst_hist.size(); q-- > 0;)
            if (solves_hist[q] <= solves - 15) {
              stagnated = worst > 0.5 * worst_hist[q];
              break;
            }
        }
        return all || stagnated;
      };
      for (int it = 0; it < eig_maxit; ++it) {
        const int d = std::min(dmax, it + 1);
        // Z = T V = P^-1 B V
        gnk::eig_trsm(pc, b, LB, DB, TBB, BV, Z, s, d_act);
        ++solves;
        if (d == 1) {
          // Rayleigh-Ritz on span(Z): P Z = B V, so Z^T P Z = Z^T (B V)
          gnk::eig_bapply(p, pc, BE, b, maxNBB, Z, BZ, s, d_act);
          gnk::eig_gram(pc, b, Z, BV, BZ, V, nu, GP, GB, resp, s, d_act);
        } else {
          // filter interval [0, nu_cut] per subdomain, nu_cut = smallest Ritz value
          // of the last Rayleigh-Ritz step; scaled so that nu = 1/s maps to 1
          const double nuref = 1.0 / shift;
          for (int j = 0; j < n_sub; ++j) {
            double nucut = h_nu[(size_t)j * b + b - 1];
            nucut = std::min(std::max(nucut, 1e-12 * nuref), 0.5 * nuref);
            const double e = 0.5 * nucut, c = 0.5 * nucut;
            const double s1 = e / (nuref - c);
            double* cf = &h_coef[(size_t)j * ncoef];
            cf[0] = s1 / e;
            cf[1] = c;
            double sig = s1;
            for (int i = 2; i < d; ++i) {
              const double sn = 1.0 / (2.0 / s1 - sig);
              cf[2 + 2 * (i - 2)] = 2.0 * sn / e;
              cf[3 + 2 * (i - 2)] = sig * sn;
              sig = sn;
            }
          }
          GN_HIP(hipMemcpyAsync(d_coef, h_coef.data(), sizeof(double) * h_coef.size(), hipMemcpyHostToDevice, s));
          // Y1 = a1 (Z - c V), with the Ritz residuals of the current block
          gnk::eig_cheb_first(pc, b, Z, V, nu, d_coef, ncoef, A1, resp, s, d_act);
          // Z = T V gives the residuals of the current pairs (those of the last
          // Rayleigh-Ritz step): stop here when they have converged
          gnk::eig_resid_sum(n_sub, b, resp, res, s, d_act);
          GN_HIP(hipMemcpyAsync(h_res.data(), res, sizeof(double) * h_res.size(), hipMemcpyDeviceToHost, s));
          GN_HIP(hipStreamSynchronize(s));
          eig_solves = solves_prev + solves;
          if (check(h_nu)) {
            converged = true;
            eig_iters = it;
            break;
          }
          double *Y0 = V, *BY0 = BV, *Yc = A1, *BYc = B1;
          gnk::eig_bapply(p, pc, BE, b, maxNBB, Yc, BYc, s, d_act);
          for (int i = 2; i < d; ++i) {
            gnk::eig_trsm(pc, b, LB, DB, TBB, BYc, Z, s, d_act);
            ++solves;
            gnk::eig_cheb_step(pc, b, maxNBB, Z, Yc, Y0, d_coef, ncoef, i - 2, s, d_act);   // Y0 <- Y_i
            gnk::eig_bapply(p, pc, BE, b, maxNBB, Y0, BY0, s, d_act);
            std::swap(Y0, Yc);
            std::swap(BY0, BYc);
          }
          // W = T Y_{d-1}: Rayleigh-Ritz on span(W) with P W = B Y_{d-1}
          gnk::eig_trsm(pc, b, LB, DB, TBB, BYc, Z, s, d_act);
          ++solves;
          gnk::eig_bapply(p, pc, BE, b, maxNBB, Z, BZ, s, d_act);
          gnk::eig_gram(pc, b, Z, BYc, BZ, nullptr, nullptr, GP, GB, nullptr, s, d_act);
        }
        gnk::eig_small(n_sub, b, GP, GB, resp, res, Y, nu, nullptr, s, d_act);
        gnk::eig_vupdate(pc, b, maxNBB, Z, BZ, Y, V, BV, s, d_act);
        GN_HIP(hipMemcpyAsync(h_res.data(), res, sizeof(double) * h_res.size(), hipMemcpyDeviceToHost, s));
        // residuals refer to the Ritz pairs of the previous iteration (h_nu before this copy)
        std::vector<double> prev_nu = h_nu;
        GN_HIP(hipMemcpyAsync(h_nu.data(), nu, sizeof(double) * h_nu.size(), hipMemcpyDeviceToHost, s));
        GN_HIP(hipStreamSynchronize(s));
        eig_iters = it + 1;
        eig_solves = solves_prev + solves;
        if (it == 0 || d > 1) continue;   // filtered steps check right after their first solve
        if (check(prev_nu)) {
          converged = true;
          break;
        }
      }
      if (!converged)
        throw gn_error{GN_ERR_EIG_NOCONV, "GenEO eigensolver did not converge in " + std::to_string(eig_maxit) +
                                              " iterations"};
      if (block_short && auto_block && b < 64) {
        b = std::min(64, b + 16);   // more eigenvalues below 1.5 x threshold than the block holds
        solves_prev = eig_solves;
        continue;
      }
      if (block_short)
        throw gn_error{GN_ERR_EIG_NOCONV, "GenEO eigensolver block of " + std::to_string(b) +
                                              " vectors too small for the eigenvalues below 1.5 x threshold "
                                              "(raise eig_block)"};
      {
        // Refinement in the original pencil.  The iteration applies
        // T = P^-1 B through the banded factor, whose backward error, amplified
        // by the condition of P, limits how well the Ritz vectors can match the
        // pencil's eigenvectors.  One inverse-iteration step in defect form
        // (V += P^-1 (B V - P V diag(nu)) diag(1/nu), with P V and B V from
        // P = A_N + s B and B themselves) passes only the small defect through
        // the solve; a last Rayleigh-Ritz step on span(V) then forms its Gram
        // matrices V^T P V and V^T B V from the same exact products.
        // Further steps (eig_refine) shrink the error components of the block
        // again by the ratio of the wanted to the unwanted nu.
        for (int step = 0; step < eig_refine; ++step) {
          gnk::eig_bapply(p, pc, PE, b, maxNBB, V, Z, s);       // Z = P V
          gnk::eig_bapply(p, pc, BE, b, maxNBB, V, BV, s);      // BV = B V
          gnk::eig_defect(pc, b, maxNBB, BV, Z, nu, BZ, s);     // BZ = B V - P V diag(nu)
          gnk::eig_trsm(pc, b, LB, DB, TBB, BZ, Z, s);          // Z = P^-1 (defect)
          ++eig_solves;
          gnk::eig_defect_add(pc, b, maxNBB, Z, nu, 1e-12 / shift, V, s);
          gnk::eig_bapply(p, pc, PE, b, maxNBB, V, Z, s);       // Z = P V
          gnk::eig_bapply(p, pc, BE, b, maxNBB, V, BV, s);      // BV = B V
          gnk::eig_gram(pc, b, V, Z, BV, nullptr, nullptr, GP, GB, nullptr, s);
          gnk::eig_small(n_sub, b, GP, GB, resp, res, Y, nu, nullptr, s);
          gnk::eig_vupdate(pc, b, maxNBB, V, BV, Y, Z, BZ, s);  // Z = V Y, BZ = (B V) Y
          std::swap(V, Z);
        }
        GN_HIP(hipMemcpyAsync(h_nu.data(), nu, sizeof(double) * h_nu.size(), hipMemcpyDeviceToHost, s));
        GN_HIP(hipStreamSynchronize(s));
      }
      break;
    }
    // V now holds the Ritz vectors of the last Rayleigh-Ritz step (h_nu).  Each
    // eigenvalue is reported as the Rayleigh quotient p^T A_N p / p^T B p of its
    // Ritz vector, summed from element energies: 1/nu - s would lose about
    // log10(s / lambda) digits to cancellation when lambda is far below s.
    std::vector<double> h_rq((size_t)n_sub * b);
    {
      double* d_rq = dalloc<double>(tmp, (size_t)n_sub * b);
      gnk::eig_rq(p, pc, b, V, d_rq, s);
      GN_HIP(hipMemcpyAsync(h_rq.data(), d_rq, sizeof(double) * h_rq.size(), hipMemcpyDeviceToHost, s));
      GN_HIP(hipStreamSynchronize(s));
    }
    pc->n_eval = b;
    pc->lam.assign((size_t)n_sub * b, 0.0);
    pc->lam_n.assign(n_sub, b);
    int coff = 0;
    for (int j = 0; j < n_sub; ++j) {
      std::vector<double> lam(b);
      for (int k = 0; k < b; ++k) {
        const double nk = h_nu[(size_t)j * b + k], rq = h_rq[(size_t)j * b + k];
        lam[k] = nk > 1e-12 / shift ? (std::isfinite(rq) ? rq : 1.0 / nk - shift) : INFINITY;
        pc->lam[(size_t)j * b + k] = lam[k];
      }
      int finite = 0;
      for (int k = 0; k < b; ++k)
        if (std::isfinite(lam[k])) ++finite;
      int m;
      if (fixed) {
        m = std::min(o->nev, finite);
      } else {
        m = 0;
        for (int k = 0; k < b; ++k)
          if (lam[k] < o->threshold) ++m;
        if (o->nev_max > 0) m = std::min(m, o->nev_max);
      }
      int cap = std::max(o->nev_max > 0 ? o->nev_max : finite, m);
      cap = std::min(cap, b - 1);
      while (m > 0 && m < std::min(cap, finite) && lam[m] - lam[m - 1] <= 1e-8 * std::fabs(lam[m - 1]) + 1e-10) ++m;
      pc->sub[j].m = m;
      pc->sub[j].coff = coff;
      coff += m;
      maxm = std::max(maxm, m);
    }
    pc->NH = coff;
    gnk::eig_normalise(pc, b, maxm, V, s);
    }
    t2 = now_s();
    // ---- coarse basis, coarse matrix, coarse factor ------------------------
    if (pc->NH > 0) {
      int64_t phi = 0;
      pc->max_m = 0;
      for (int j = 0; j < n_sub; ++j) pc->max_m = std::max(pc->max_m, pc->sub[j].m);
      for (int j = 0; j < n_sub; ++j) {
        pc->sub[j].offPhi = phi;
        phi += (int64_t)pc->sub[j].nI * pc->sub[j].m;
      }
      pc->phi_len = phi;
      upload_descs(pc, s);
      pc->d_Phi = dalloc<double>(pc->owned, (size_t)phi);
      gnk::build_phi(p, pc, b, maxNI, V, s);
      gnk::aphi(p, pc, b, maxNB_, Z, s);
      // pairs (j1, j2) with I_j1 cap Ibar_j2 nonempty
      std::vector<std::pair<int, int>> pair_list;
      std::vector<char> pbuf;
      int np = 0;
      const int psz = gnk::pair_size();
      for (int j1 = 0; j1 < n_sub; ++j1)
        for (int j2 = 0; j2 < n_sub; ++j2) {
          const SubDesc &a1 = pc->sub[j1], &a2 = pc->sub[j2];
          if (a1.m == 0 || a2.m == 0) continue;
          int lo[3], hi[3];
          bool ok = true;
          for (int a = 0; a < 3; ++a) {
            lo[a] = std::max(a1.ilo[a], a2.blo[a]);
            hi[a] = std::min(a1.ilo[a] + a1.in_[a], a2.blo[a] + a2.bn[a]);
            ok &= hi[a] > lo[a];
          }
          if (!ok) continue;
          pbuf.resize((size_t)(np + 1) * psz);
          gnk::make_pair(pbuf.data() + (size_t)np * psz, j1, j2, lo, hi);
          pair_list.emplace_back(j1, j2);
          ++np;
        }
      char* d_pairs = upload(tmp, pbuf.data(), pbuf.size(), s);
      pc->NBH = (pc->NH + TILE - 1) / TILE;
      const size_t ahlen = (size_t)pc->NBH * pc->NBH * TILE2;
      double* AH = dalloc<double>(tmp, ahlen);
      double* DH = dalloc<double>(tmp, (size_t)pc->NBH * TILE2);
      GN_HIP(hipMemsetAsync(AH, 0, sizeof(double) * ahlen, s));
      gnk::ah_pairs(p, pc, d_pairs, np, b, Z, AH, s);
      if (pc->coarse_solve == 0) {
        GN_HIP(hipMemsetAsync(d_info + n_sub, 0, sizeof(int), s));
        gnk::dense_chol(pc->NBH, AH, DH, d_info + n_sub, s);
        int hinfo = 0;
        GN_HIP(hipMemcpyAsync(&hinfo, d_info + n_sub, sizeof(int), hipMemcpyDeviceToHost, s));
        GN_HIP(hipStreamSynchronize(s));
        if (hinfo) throw gn_error{GN_ERR_COARSE_SINGULAR, "coarse matrix not positive definite"};
        pc->d_Z = dalloc<double>(pc->owned, ahlen);
        gnk::tri_inv(pc->NBH, AH, DH, pc->d_Z, s);
        // Z^T in the upper tiles and the work units of the coarse products
        pc->d_Zdt = dalloc<double>(pc->owned, (size_t)pc->NBH * TILE2);
        gnk::z_transpose(pc, s);
        for (int upper = 0; upper < 2; ++upper) {
          std::vector<int4> units;
          std::vector<int> rowstart(pc->NBH + 1, 0);
          for (int R = 0; R < pc->NBH; ++R) {
            rowstart[R] = (int)units.size();
            const int c0 = upper ? R : 0, c1 = upper ? pc->NBH : R + 1;
            for (int c = c0; c < c1; c += gnk::COARSE_UNIT_TILES)
              units.push_back(int4{R, c, std::min(c1, c + gnk::COARSE_UNIT_TILES), 0});
          }
          rowstart[pc->NBH] = (int)units.size();
          if ((int64_t)units.size() != gnk::coarse_units(pc->NBH, upper != 0))
            throw gn_error{GN_ERR_DEVICE, "coarse unit table size mismatch"};
          (upper ? pc->n_cu_b : pc->n_cu_f) = (int)units.size();
          (upper ? pc->d_cu_b : pc->d_cu_f) = upload(pc->owned, units.data(), units.size(), s);
          (upper ? pc->d_rs_b : pc->d_rs_f) = upload(pc->owned, rowstart.data(), rowstart.size(), s);
        }
        pc->d_zpart = dalloc<double>(pc->owned, (size_t)std::max(pc->n_cu_f, pc->n_cu_b) * TILE);
      } else {
        // inexact coarse solve: A_H kept block-sparse (the symmetric closure of
        // the interacting pairs), the diagonal blocks inverted
        if (maxm > 64) argfail("inexact coarse solve needs at most 64 vectors per subdomain");
        std::vector<std::vector<int>> nbr(n_sub);
        for (const auto& pr : pair_list) {
          nbr[pr.first].push_back(pr.second);
          nbr[pr.second].push_back(pr.first);
        }
        std::vector<int> ptr(n_sub + 1, 0);
        std::vector<BsrBlock> blk;
        std::vector<int64_t> doff(n_sub, 0);
        int64_t off = 0, dsz = 0;
        for (int j = 0; j < n_sub; ++j) {
          std::sort(nbr[j].begin(), nbr[j].end());
          nbr[j].erase(std::unique(nbr[j].begin(), nbr[j].end()), nbr[j].end());
          for (int j2 : nbr[j]) {
            blk.push_back(BsrBlock{j, j2, off});
            off += (int64_t)pc->sub[j].m * pc->sub[j2].m;
          }
          ptr[j + 1] = (int)blk.size();
          doff[j] = dsz;
          dsz += (int64_t)pc->sub[j].m * pc->sub[j].m;
        }
        pc->bsr_nnz = (int64_t)blk.size();
        pc->d_bsr_ptr = upload(pc->owned, ptr.data(), ptr.size(), s);
        pc->d_bsr_blk = upload(pc->owned, blk.data(), std::max<size_t>(blk.size(), 1), s);
        pc->d_bsr_val = dalloc<double>(pc->owned, (size_t)std::max<int64_t>(off, 1));
        pc->d_dinv_off = upload(pc->owned, doff.data(), doff.size(), s);
        pc->d_dinv = dalloc<double>(pc->owned, (size_t)std::max<int64_t>(dsz, 1));
        gnk::bsr_from_dense(pc, AH, s);
        GN_HIP(hipMemsetAsync(d_info, 0, sizeof(int) * n_sub, s));
        gnk::block_inverse(pc, d_info, s);
        GN_HIP(hipMemcpyAsync(info.data(), d_info, sizeof(int) * n_sub, hipMemcpyDeviceToHost, s));
        GN_HIP(hipStreamSynchronize(s));
        for (int j = 0; j < n_sub; ++j)
          if (info[j]) throw gn_error{GN_ERR_COARSE_SINGULAR, "diagonal block of the coarse matrix not positive definite"};
        pc->coarse_grid = gnk::coarse_cg_grid(pc);
        pc->d_cvec = dalloc<double>(pc->owned, (size_t)5 * pc->NBH * TILE);
        pc->d_cpart = dalloc<double>(pc->owned, (size_t)3 * pc->coarse_grid);
        pc->d_cstat = dalloc<double>(pc->owned, 4);
        GN_HIP(hipMemsetAsync(pc->d_cvec, 0, sizeof(double) * 5 * pc->NBH * TILE, s));
        GN_HIP(hipMemsetAsync(pc->d_cstat, 0, sizeof(double) * 4, s));
      }
      pc->d_g = dalloc<double>(pc->owned, (size_t)pc->NBH * TILE);
      pc->d_u = dalloc<double>(pc->owned, (size_t)pc->NBH * TILE);
      pc->d_y = dalloc<double>(pc->owned, (size_t)pc->NBH * TILE);
      GN_HIP(hipMemsetAsync(pc->d_g, 0, sizeof(double) * pc->NBH * TILE, s));
      GN_HIP(hipMemsetAsync(pc->d_u, 0, sizeof(double) * pc->NBH * TILE, s));
      GN_HIP(hipMemsetAsync(pc->d_y, 0, sizeof(double) * pc->NBH * TILE, s));
    }
    GN_HIP(hipStreamSynchronize(s));
    t3 = now_s();
  } else {
    upload_descs(pc, s);
  }
  // launch shape of the single-column local solves (timed when several fit)
  gnk::local_solve_tune(p, pc, s);
  GN_HIP(hipStreamSynchronize(s));
  dfree_all(tmp);
  // algorithmic bytes of one preconditioner application (for the roofline report)
  {
    const double fb = pc->local_prec == 32 ? 4.0 : 8.0;
    double tb = 0.0, tbt = 0.0, pb = 0.0;
    for (const SubDesc& sd : pc->sub) {
      // algorithmic: the forward sweep reads the factor's band once (row r holds
      // min(r, bw) + 1 entries), the backward sweep reads it once more; the
      // gather reads r on I_j, z_j is written, Phi_j is read for the restriction
      double entries = 0.0;
      for (int r = 0; r < sd.nI; ++r) entries += (double)std::min(r, sd.bwI) + 1.0;
      const double vec = (double)sd.nI * 8.0 * 2.0 + (double)sd.nI * sd.m * 8.0;
      tb += 2.0 * entries * fb + vec;
      // as stored: whole band tiles (lower-triangle tiles touched) and inverse diagonals
      double tiles = 0.0;
      for (int K = 0; K < sd.NBI; ++K) tiles += std::min(K, sd.wI);
      tbt += 2.0 * (tiles + sd.NBI) * TILE2 * fb + vec;
      pb += (double)sd.nI * 8.0 + (double)sd.nI * sd.m * 8.0;
    }
    pc->trsv_bytes = tb;
    pc->trsv_tile_bytes = tbt;
    pc->prolong_bytes = pb + (double)p->n_dof * 8.0 * 2.0;
    // batched: the band is read once for all 16 columns; the gather writes the
    // 16-wide local vectors, which both sweeps read and write once more
    double tbm = 0.0;
    for (const SubDesc& sd : pc->sub) {
      double tiles = 0.0;
      for (int K = 0; K < sd.NBI; ++K) tiles += std::min(K, sd.wI);
      tbm += 2.0 * (tiles + sd.NBI) * TILE2 * fb + (double)sd.NBI * TILE * 16.0 * 8.0 * 5.0 +
             (double)sd.nI * sd.m * 8.0;
    }
    pc->trsv_bytes_mc = tbm;
  }
  int64_t hb = 0;
  hb += (int64_t)pc->tilesI * TILE2 * (pc->local_prec == 32 ? 4 : 8) * (pc->d_LIb ? 2 : 1);
  hb += (int64_t)pc->sub.size() * 0;
  hb += pc->phi_len * 8 + (int64_t)pc->NBH * pc->NBH * TILE2 * 8 + pc->vecI * 8;
  if (rep) {
    rep->n_sub = n_sub;
    rep->coarse_dim = pc->NH;
    rep->eig_iters = eig_iters;
    rep->eig_solves = eig_solves;
    rep->max_local_n = maxNI;
    rep->band_tiles = maxw;
    rep->t_local_s = t1 - t0;
    rep->t_eigen_s = t2 - t1;
    rep->t_coarse_s = t3 - t2;
    rep->t_total_s = now_s() - t0;
    rep->t_alloc_s = gnh::dev_alloc_seconds() - ta0;
    rep->apply_bytes = pc->trsv_bytes;
    rep->apply_tile_bytes = pc->trsv_tile_bytes;
    rep->local_threads = gnk::pf_supported(p, pc) ? 32 * pc->pf_G : 0;
    rep->hbm_bytes = hb;
    rep->eig_resid = eig_resid;
  }
  *out = pc;
  return GN_OK;
  }
  catch (const gn_error& e) {
    dfree_all(tmp);
    if (pc) { dfree_all(pc->owned); delete pc; }
    gn_set_error(e.code, e.msg);
    return e.code;
  }
  catch (...) {
    dfree_all(tmp);
    if (pc) { dfree_all(pc->owned); delete pc; }
    gn_set_error(GN_ERR_DEVICE, "unexpected exception in gn_setup_geneo");
    return GN_ERR_DEVICE;
  }
}

extern "C" gn_status gn_precond_eigenvalues(const gn_precond* pc, int32_t sub, double* out, int32_t cap,
                                            int32_t* m, int32_t* n_avail) {
  if (!pc || sub < 0 || sub >= pc->n_sub) {
    gn_set_error(GN_ERR_ARG, "bad precond/subdomain");
    return GN_ERR_ARG;
  }
  int n = pc->lam.empty() ? 0 : pc->n_eval;
  if (m) *m = pc->sub[sub].m;
  if (n_avail) *n_avail = n;
  if (out)
    for (int k = 0; k < std::min(n, (int)cap); ++k) out[k] = pc->lam[(size_t)sub * pc->n_eval + k];
  return GN_OK;
}

extern "C" gn_status gn_precond_coarse_basis(const gn_precond* pc, double* out, int64_t ld, int64_t* nh) {
  GN_TRY
  if (!pc) argfail("null argument");
  const gn_problem* p = pc->prob;
  if (nh) *nh = pc->NH;
  if (!out || pc->NH == 0) return GN_OK;
  if (ld < p->n_free) argfail("ld must be >= n_free");
  std::vector<double> phi((size_t)pc->phi_len);
  std::vector<int> f2f((size_t)p->n_free);
  GN_HIP(hipDeviceSynchronize());
  GN_HIP(hipMemcpy(phi.data(), pc->d_Phi, sizeof(double) * phi.size(), hipMemcpyDeviceToHost));
  GN_HIP(hipMemcpy(f2f.data(), p->d_free2full, sizeof(int) * f2f.size(), hipMemcpyDeviceToHost));
  std::vector<int64_t> full2free((size_t)p->n_dof, -1);
  for (int64_t i = 0; i < p->n_free; ++i) full2free[f2f[i]] = i;
  for (int64_t c = 0; c < pc->NH; ++c) std::fill(out + c * ld, out + c * ld + p->n_free, 0.0);
  const int nc = p->nc;
  for (int j = 0; j < pc->n_sub; ++j) {
    const SubDesc& sd = pc->sub[j];
    for (int row = 0; row < sd.nI; ++row) {
      int g[3];
      box_global_node(sd.ilo, sd.in_, sd.permI, row / nc, g);
      const int64_t node = g[0] + (int64_t)p->nn[0] * (g[1] + (int64_t)p->nn[1] * g[2]);
      const int64_t f = full2free[node * nc + row % nc];
      if (f < 0) continue;   // Dirichlet DOF: Phi is zero there
      for (int k = 0; k < sd.m; ++k) out[(sd.coff + k) * ld + f] = phi[sd.offPhi + (int64_t)row * sd.m + k];
    }
  }
  return GN_OK;
  GN_CATCH
}

static void ensure_batch_precond(gn_precond* pc, hipStream_t s);

// z = M^-1 r on full-numbering device vectors
static void precond_full(gn_problem* p, gn_precond* pc, const double* r, double* z, double* part,
                         const double* done, hipStream_t s) {
  if (gnk::pf_supported(p, pc)) {
    gnk::local_solve(p, pc, r, done, s);
    if (pc->coarse_solve == 1) gnk::coarse_cg(pc, pc->d_g, pc->d_y, done, s);
    else gnk::coarse_solve(pc, done, s);
    gnk::prolong(p, pc, r, z, part, done, s);
  } else {
    // bands too wide for the single-column register pipeline: the batched
    // kernels with one live column (done sits at S_DONE of the scalar block)
    ensure_batch_precond(pc, s);
    gnk::precond_mc(p, pc, r, z, 1, part, 0, done ? done - S_DONE : nullptr, pc->d_tm, pc->d_gm, pc->d_um,
                    pc->d_ym, s);
  }
}

extern "C" gn_status gn_precond_apply(gn_precond* pc, const double* r_dev, double* z_dev, void* stream) {
  GN_TRY
  if (!pc || !r_dev || !z_dev) argfail("null argument");
  gn_problem* p = pc->prob;
  hipStream_t s = (hipStream_t)stream;
  gnk::scatter_free(p, r_dev, p->d_r, s);
  precond_full(p, pc, p->d_r, p->d_z, nullptr, nullptr, s);
  gnk::gather_free(p, p->d_z, z_dev, s);
  GN_HIP(hipStreamSynchronize(s));
  return GN_OK;
  GN_CATCH
}

// ---------------------------------------------------------------------------
// PCG
// ---------------------------------------------------------------------------

// || |A| |x| ||^2 for one full-numbering vector: eps times its square root is
// the rounding floor of b - A x for any FP64 x near x (attainable accuracy)
double gnh::absmv_norm2(gn_problem* p, const double* x, hipStream_t s) {
  const int nb = gnk::spmv_blocks(p);
  std::vector<double> part(nb);
  gnk::absmv_partial(p, x, p->d_part, s);
  GN_HIP(hipMemcpyAsync(part.data(), p->d_part, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  GN_HIP(hipStreamSynchronize(s));
  double t = 0.0;
  for (double v : part) t += v;
  return t;
}
using gnh::kEps;
using gnh::kFloorFactor;
using gnh::absmv_norm2;

// CG-Lanczos tridiagonal of the first kit steps: T_ii = 1/a_i + b_{i-1}/a_{i-1},
// T_{i,i+1} = sqrt(b_i)/a_i; returns its extreme eigenvalue ratio
double gnh::cond_from_hist(const double* hist, int kit) {
  if (kit <= 0) return 1.0;
  std::vector<double> d(kit), e(std::max(kit - 1, 0));
  for (int i = 0; i < kit; ++i) {
    double a = hist[2 * i];
    d[i] = 1.0 / a + (i > 0 ? hist[2 * (i - 1) + 1] / hist[2 * (i - 1)] : 0.0);
    if (i + 1 < kit) e[i] = std::sqrt(std::max(hist[2 * i + 1], 0.0)) / a;
  }
  double lo, hi;
  tridiag_extremes(d, e, &lo, &hi);
  return lo > 0 ? hi / lo : INFINITY;
}

using gnh::cond_from_hist;

// batched workspace for up to 16 columns, allocated on first use
void gnh::ensure_batch_workspace(gn_problem* p, gn_precond* pc, int maxit, hipStream_t s) {
  const int KC = gnk::mc_width();
  const int64_t n = p->n_dof;
  if (!p->d_Xm) {
    p->d_Xm = dalloc<double>(p->owned, (size_t)n * KC);
    p->d_Rm = dalloc<double>(p->owned, (size_t)n * KC);
    p->d_Pm = dalloc<double>(p->owned, (size_t)n * KC);
    p->d_Qm = dalloc<double>(p->owned, (size_t)n * KC);
    p->d_Zm = dalloc<double>(p->owned, (size_t)n * KC);
    for (double* v : {p->d_Xm, p->d_Rm, p->d_Pm, p->d_Qm, p->d_Zm})
      GN_HIP(hipMemsetAsync(v, 0, sizeof(double) * n * KC, s));
    p->pstride_m = std::max(std::max(gnk::spmv_blocks(p), gnk::reduce_blocks()), gnk::prolong_blocks(p));
    p->d_partm = dalloc<double>(p->owned, (size_t)p->pstride_m * KC);
    p->d_scalm = dalloc<double>(p->owned, (size_t)S_N * KC);
  }
  if (p->histm_stride < 2 * maxit + 2) {
    if (p->d_histm) {
      GN_HIP(hipStreamSynchronize(s));
      gnh::dev_free(p->d_histm);
      p->owned.erase(std::remove(p->owned.begin(), p->owned.end(), (void*)p->d_histm), p->owned.end());
    }
    p->histm_stride = 2 * maxit + 2;
    p->d_histm = dalloc<double>(p->owned, (size_t)p->histm_stride * KC);
  }
  if (pc) ensure_batch_precond(pc, s);
}

static void ensure_batch_precond(gn_precond* pc, hipStream_t s) {
  if (pc->d_tm) return;
  const int KC = gnk::mc_width();
  pc->d_tm = dalloc<double>(pc->owned, (size_t)pc->vecI * KC);
  GN_HIP(hipMemsetAsync(pc->d_tm, 0, sizeof(double) * pc->vecI * KC, s));
  const size_t nh = (size_t)std::max(pc->NBH, 1) * TILE * KC;
  pc->d_gm = dalloc<double>(pc->owned, nh);
  pc->d_um = dalloc<double>(pc->owned, nh);
  pc->d_ym = dalloc<double>(pc->owned, nh);
  for (double* v : {pc->d_gm, pc->d_um, pc->d_ym}) GN_HIP(hipMemsetAsync(v, 0, sizeof(double) * nh, s));
}

extern "C" gn_status gn_solve(gn_problem* p, gn_precond* pc, const double* b_dev, double* x_dev,
                              int32_t nrhs, int64_t ld, const gn_solve_opts* opts, void* stream,
                              gn_solve_report* reports) {
  GN_TRY
  if (!p || !b_dev || !x_dev || !opts) argfail("null argument");
  if (nrhs < 1 || ld < p->n_free) argfail("bad nrhs/ld");
  if (!(opts->rtol > 0) || opts->maxit < 1) argfail("rtol > 0 and maxit >= 1 required");
  if (pc && pc->prob != p) argfail("preconditioner built for another problem");
  hipStream_t s = (hipStream_t)stream;
  if (gnk::count_nonfinite(p->n_free, nrhs, ld, b_dev, p->d_count, s) != 0)
    argfail("right-hand side holds NaN or infinite entries");
  const int chunk = opts->check_every > 0 ? opts->check_every : 8;
  const int64_t n = p->n_dof;
  if (p->hist_cap < 2 * opts->maxit + 2) {
    if (p->d_hist) {
      GN_HIP(hipStreamSynchronize(s));
      gnh::dev_free(p->d_hist);
      p->owned.erase(std::remove(p->owned.begin(), p->owned.end(), (void*)p->d_hist), p->owned.end());
    }
    p->d_hist = dalloc<double>(p->owned, (size_t)2 * opts->maxit + 2);
    p->hist_cap = 2 * opts->maxit + 2;
  }
  double* scal = p->d_scal;
  const double* done = scal + S_DONE;
  gn_status ret = GN_OK;
  // flexible CG (a preconditioner that varies between applications: the
  // inexact coarse solve) runs the columns one after another
  const int flex = opts->flexible != 0 ? 1 : 0;
  if (nrhs > 1 && !opts->sequential && !flex) {
    // up to 16 columns share every launch; a finished column's slot takes the
    // next column at the following chunk boundary
    const double tstart = now_s();
    SlotEngine eng(p, pc, std::min(gnk::mc_width(), (int)nrhs), chunk, opts->maxit, s);
    std::vector<SlotResult> res;
    int next = 0;
    while (next < nrhs || eng.busy()) {
      while (next < nrhs && eng.free_slots() > 0) {
        SlotColumn c;
        c.b = b_dev + next * ld;
        c.x = x_dev + next * ld;
        c.rtol = opts->rtol;
        c.maxit = opts->maxit;
        c.index = next++;
        eng.admit(c);
      }
      res.clear();
      eng.step(res);
      for (const SlotResult& r : res) {
        if (reports) reports[r.col.index] = r.rep;
        if (r.st < 0 && ret >= 0) ret = r.st;
        else if (r.st > 0 && ret == GN_OK) ret = r.st;
      }
    }
    if (reports)
      for (int c = 0; c < nrhs; ++c) reports[c].t_solve_s = now_s() - tstart;
    return ret;
  }
  const int nbs = gnk::spmv_blocks(p), nbr = gnk::reduce_blocks(), nbp = gnk::prolong_blocks(p);
  for (int col = 0; col < nrhs; ++col) {
    const double tstart = now_s();
    // r = b (x0 = 0), x = 0
    gnk::scatter_free(p, b_dev + col * ld, p->d_r, s);
    GN_HIP(hipMemsetAsync(p->d_x, 0, sizeof(double) * n, s));
    double maxit_d = (double)opts->maxit;
    GN_HIP(hipMemcpyAsync(scal + S_MAXIT, &maxit_d, sizeof(double), hipMemcpyHostToDevice, s));
    gnk::dot_partial(n, p->d_r, p->d_r, p->d_part, nullptr, s);
    gnk::finalize(p->d_part, nbr, OP_BB, scal, p->d_hist, opts->rtol, s);
    if (pc) {
      precond_full(p, pc, p->d_r, p->d_z, p->d_part, done, s);
      gnk::finalize(p->d_part, nbp, OP_RZ0, scal, p->d_hist, opts->rtol, s);
    } else {
      gnk::copy(n, p->d_z, p->d_r, done, s);
      gnk::dot_partial(n, p->d_r, p->d_z, p->d_part, done, s);
      gnk::finalize(p->d_part, nbr, OP_RZ0, scal, p->d_hist, opts->rtol, s);
    }
    gnk::copy(n, p->d_p, p->d_z, done, s);
    double hs[16];
    int iters = 0;
    // one chunk of iterations; kernels of finished solves return at once
    auto launch_chunk = [&](hipStream_t st) {
      for (int k = 0; k < chunk; ++k) {
        gnk::spmv_flag(p, p->d_p, p->d_q, p->d_part, done, st);
        gnk::finalize(p->d_part, nbs, OP_ALPHA, scal, p->d_hist, opts->rtol, st);
        gnk::update_xr(n, p->d_x, p->d_r, p->d_p, p->d_q, scal, p->d_part, st);
        gnk::finalize(p->d_part, nbr, OP_RR, scal, p->d_hist, opts->rtol, st);
        if (pc && flex) {
          // Polak-Ribiere beta: z.r of the new residual, then z.q (r_new - r_old = -alpha q)
          precond_full(p, pc, p->d_r, p->d_z, p->d_part, done, st);
          gnk::finalize(p->d_part, nbp, OP_RZN, scal, p->d_hist, opts->rtol, st);
          gnk::dot_partial(n, p->d_z, p->d_q, p->d_part, done, st);
          gnk::finalize(p->d_part, nbr, OP_BETAF, scal, p->d_hist, opts->rtol, st);
        } else if (pc) {
          precond_full(p, pc, p->d_r, p->d_z, p->d_part, done, st);
          gnk::finalize(p->d_part, nbp, OP_BETA, scal, p->d_hist, opts->rtol, st);
        } else {
          gnk::copy(n, p->d_z, p->d_r, done, st);
          gnk::dot_partial(n, p->d_r, p->d_z, p->d_part, done, st);
          gnk::finalize(p->d_part, nbr, OP_BETA, scal, p->d_hist, opts->rtol, st);
        }
        gnk::update_p(n, p->d_p, p->d_z, scal, st);
      }
    };
    // the cooperative launch of the inexact coarse solve is issued kernel by kernel
    const bool use_graph = opts->graphs != 0 && !g_prof_on && !(pc && pc->coarse_solve == 1);
    ChunkGraph& cg = pc ? pc->cg : p->cg;
    auto run_chunk = [&]() {
      if (!use_graph) {
        launch_chunk(s);
        return;
      }
      if (!cg.exec || cg.chunk != chunk || cg.hist != p->d_hist || cg.flexible != flex) {
        // capture on a private stream (the caller's may be the null stream),
        // replay on the caller's
        cg.release();
        hipStream_t cs = nullptr;
        GN_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          try {
            launch_chunk(cs);
          } catch (...) {
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            (void)hipStreamDestroy(cs);
            throw;
          }
          e = hipStreamEndCapture(cs, &g);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&cg.exec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
          cg.exec = nullptr;
          throw gn_error{GN_ERR_DEVICE, std::string("CG chunk graph capture: ") + hipGetErrorString(e)};
        }
        cg.chunk = chunk;
        cg.hist = p->d_hist;
        cg.flexible = flex;
      }
      GN_HIP(hipGraphLaunch(cg.exec, s));
    };
    auto iterate = [&]() {
      bool fin = false;
      while (!fin) {
        run_chunk();
        GN_HIP(hipMemcpyAsync(hs, scal, sizeof(double) * S_N, hipMemcpyDeviceToHost, s));
        GN_HIP(hipStreamSynchronize(s));
        iters = (int)hs[S_ITER];
        fin = hs[S_DONE] != 0.0;
      }
    };
    // ||b - A x||^2, leaving A x in q and b (full numbering) in z
    std::vector<double> part(nbr);
    double floor2 = 0.0;   // (eps || |A| |x| ||)^2
    auto true_residual = [&]() {
      floor2 = kEps * kEps * absmv_norm2(p, p->d_x, s);
      gnk::spmv_flag(p, p->d_x, p->d_q, nullptr, nullptr, s);
      gnk::scatter_free(p, b_dev + col * ld, p->d_z, s);
      gnk::residual_partial(n, p->d_z, p->d_q, p->d_part, s);
      GN_HIP(hipMemcpyAsync(part.data(), p->d_part, sizeof(double) * nbr, hipMemcpyDeviceToHost, s));
      GN_HIP(hipStreamSynchronize(s));
      double t = 0.0;
      for (double v : part) t += v;
      return t;
    };
    iterate();
    const int first_iters = iters;
    double tr = true_residual();
    // the recursive residual drifts from b - A x (attainable accuracy of CG):
    // restart from the current iterate with the true residual, at most twice,
    // unless b - A x already sits at the rounding floor of FP64 x
    int restarts = 0;
    const double tol2 = hs[S_TOL2];   // rtol^2 ||b||^2
    double tol2r = 0.0;
    for (; restarts < 2 && hs[S_BREAK] == 0.0 && hs[S_BB] > 0.0 && tr > tol2 &&
           tr > kFloorFactor * kFloorFactor * floor2 && iters < opts->maxit;
         ++restarts) {
      gnk::sub_partial(n, p->d_z, p->d_q, p->d_r, p->d_part, s);   // r = b - A x
      gnk::finalize(p->d_part, nbr, OP_RESTART, scal, p->d_hist, opts->rtol, s);
      tol2r = gnh::restart_tol2(opts->rtol, floor2, hs[S_BB]);
      GN_HIP(hipMemcpyAsync(scal + S_TOL2, &tol2r, sizeof(double), hipMemcpyHostToDevice, s));
      if (pc) {
        precond_full(p, pc, p->d_r, p->d_z, p->d_part, done, s);
        gnk::finalize(p->d_part, nbp, OP_RZ0, scal, p->d_hist, opts->rtol, s);
      } else {
        gnk::copy(n, p->d_z, p->d_r, done, s);
        gnk::dot_partial(n, p->d_r, p->d_z, p->d_part, done, s);
        gnk::finalize(p->d_part, nbr, OP_RZ0, scal, p->d_hist, opts->rtol, s);
      }
      gnk::copy(n, p->d_p, p->d_z, done, s);
      iterate();
      tr = true_residual();
    }
    const double tsolve = now_s() - tstart;
    double bb = hs[S_BB], rr = hs[S_RR];
    const int kit = first_iters;   // the CG-Lanczos estimate uses the first (unrestarted) sequence
    std::vector<double> hist((size_t)2 * std::max(kit, 1));
    if (kit > 0)
      GN_HIP(hipMemcpyAsync(hist.data(), p->d_hist, sizeof(double) * 2 * kit, hipMemcpyDeviceToHost, s));
    gnk::gather_free(p, p->d_x, x_dev + col * ld, s);
    GN_HIP(hipStreamSynchronize(s));
    bool conv = bb == 0.0 || rr <= tol2;
    if (hs[S_BREAK] != 0.0) ret = GN_ERR_BREAKDOWN;
    else if (!conv && ret == GN_OK) ret = GN_WARN_MAXIT;
    if (reports) {
      gn_solve_report& R = reports[col];
      R.iters = iters;
      R.converged = conv ? 1 : 0;
      R.rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
      R.true_rel_res = bb > 0 ? std::sqrt(tr / bb) : 0.0;
      R.res_floor = bb > 0 ? std::sqrt(floor2 / bb) : 0.0;
      R.t_solve_s = tsolve;
      R.iters_first = first_iters;
      R.restarts = restarts;
      R.cond_est = cond_from_hist(hist.data(), kit);
    }
  }
  return ret;
  GN_CATCH
}

extern "C" void gn_destroy_problem(gn_problem* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  p->cg.release();
  dfree_all(p->owned);
  delete p;
}

extern "C" void gn_destroy_precond(gn_precond* pc) {
  if (!pc) return;
  (void)hipDeviceSynchronize();
  pc->cg.release();
  dfree_all(pc->owned);
  delete pc;
}
