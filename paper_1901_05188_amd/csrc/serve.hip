// Batched right-hand sides and the request server (host code).
//
// SlotEngine: the CG iteration of Section 3.1 (eqn:KrylovSubspace) with the
// preconditioner M^-1_{AS,2} for up to 16 right-hand sides of one operator.
// Every launch serves all slots; each column keeps its own alpha, beta,
// stopping test and restarts (the scalars of column c sit at scal[c * S_N]).
// A column moves through: admitted -> started (x = 0, r = b, z = M^-1 r,
// p = z) -> CG chunks -> finished (true residual b - A x) -> restarted from
// b - A x (at most twice, while above the tolerance and above the FP64
// rounding floor) or retired (x copied out, report filled).  A retired
// column frees its slot, and the next queued column starts at the following
// chunk boundary while the other slots keep iterating.  Starting or
// restarting columns holds the running ones by setting their done flags for
// the few launches of that phase, so the batched kernels, which skip done
// columns, touch only the columns being started.  The arithmetic of a column
// is independent of its slot and of what the other slots hold.
//
// gn_server: resident operators, each with its own HIP stream and worker
// thread driving a SlotEngine; requests (a group of right-hand sides of one
// operator) are queued per operator and their columns enter slots as these
// free up.  Work of different operators overlaps on the device.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "gn_internal.h"

using gnh::kEps;
using gnh::kFloorFactor;
using gnh::now_s;

// ---------------------------------------------------------------------------
// SlotEngine
// ---------------------------------------------------------------------------
SlotEngine::SlotEngine(gn_problem* p, gn_precond* pc, int slots, int chunk, int maxit_cap, hipStream_t s)
    : p_(p), pc_(pc), k_(slots), chunk_(chunk), maxit_cap_(maxit_cap), s_(s) {
  if (slots < 1 || slots > gnk::mc_width()) throw gn_error{GN_ERR_ARG, "slots must lie in 1..16"};
  if (chunk < 1 || maxit_cap < 1) throw gn_error{GN_ERR_ARG, "chunk and maxit must be >= 1"};
  gnh::ensure_batch_workspace(p, pc, maxit_cap, s);
  slot_.resize(k_);
  hsc_.assign((size_t)k_ * S_N, 0.0);
  for (int c = 0; c < k_; ++c) hsc_[(size_t)c * S_N + S_DONE] = 1.0;   // a free slot is done
  GN_HIP(hipMemcpyAsync(p->d_scalm, hsc_.data(), sizeof(double) * k_ * S_N, hipMemcpyHostToDevice, s));
  GN_HIP(hipStreamSynchronize(s));
}

int SlotEngine::free_slots() const {
  int f = 0;
  for (const Slot& sl : slot_) f += sl.used ? 0 : 1;
  return f;
}

bool SlotEngine::busy() const {
  for (const Slot& sl : slot_)
    if (sl.used) return true;
  return false;
}

void SlotEngine::admit(const SlotColumn& c) {
  if (c.maxit > maxit_cap_) throw gn_error{GN_ERR_ARG, "maxit above the engine's cap"};
  for (Slot& sl : slot_) {
    if (sl.used) continue;
    sl = Slot();
    sl.used = true;
    sl.fresh = true;
    sl.col = c;
    return;
  }
  throw gn_error{GN_ERR_ARG, "no free slot"};
}

void SlotEngine::read_scal() {
  GN_HIP(hipMemcpyAsync(hsc_.data(), p_->d_scalm, sizeof(double) * k_ * S_N, hipMemcpyDeviceToHost, s_));
  GN_HIP(hipStreamSynchronize(s_));
}

// The host mirror is exact here (read after the last launch that could change it).
void SlotEngine::phase_begin(const std::vector<int>& cols, std::vector<int>& held) {
  held.clear();
  std::vector<char> in(k_, 0);
  for (int c : cols) in[c] = 1;
  for (int c = 0; c < k_; ++c) {
    double& d = hsc_[(size_t)c * S_N + S_DONE];
    if (in[c]) {
      d = 0.0;
    } else if (slot_[c].used && d == 0.0) {
      d = 1.0;
      held.push_back(c);
    }
  }
  GN_HIP(hipMemcpyAsync(p_->d_scalm, hsc_.data(), sizeof(double) * k_ * S_N, hipMemcpyHostToDevice, s_));
}

void SlotEngine::phase_end(const std::vector<int>& held) {
  read_scal();
  if (held.empty()) return;
  for (int c : held) hsc_[(size_t)c * S_N + S_DONE] = 0.0;
  GN_HIP(hipMemcpyAsync(p_->d_scalm, hsc_.data(), sizeof(double) * k_ * S_N, hipMemcpyHostToDevice, s_));
  GN_HIP(hipStreamSynchronize(s_));
}

// z = M^-1 r for the live columns, then the r.z step of the recurrence
void SlotEngine::apply_m(int op) {
  gn_problem* p = p_;
  const int64_t n = p->n_dof;
  const int ps = p->pstride_m, hs = p->histm_stride;
  if (pc_) {
    gnk::precond_mc(p, pc_, p->d_Rm, p->d_Zm, k_, p->d_partm, ps, p->d_scalm, pc_->d_tm, pc_->d_gm, pc_->d_um,
                    pc_->d_ym, s_);
    gnk::finalize_mc(p->d_partm, ps, gnk::prolong_blocks(p), op, k_, p->d_scalm, p->d_histm, hs, 0.0, s_);
  } else {
    gnk::copy_mc(n, k_, p->d_Zm, p->d_Rm, p->d_scalm, s_);
    gnk::dot_mc(n, k_, p->d_Rm, p->d_Zm, p->d_partm, ps, p->d_scalm, s_);
    gnk::finalize_mc(p->d_partm, ps, gnk::reduce_blocks(), op, k_, p->d_scalm, p->d_histm, hs, 0.0, s_);
  }
}

void SlotEngine::step(std::vector<SlotResult>& out) {
  gn_problem* p = p_;
  const int64_t n = p->n_dof;
  const int ps = p->pstride_m, hs = p->histm_stride;
  const int nbs = gnk::spmv_blocks(p), nbr = gnk::reduce_blocks();
  double *X = p->d_Xm, *R = p->d_Rm, *P = p->d_Pm, *Q = p->d_Qm, *Z = p->d_Zm;
  double *part = p->d_partm, *scal = p->d_scalm, *hist = p->d_histm;
  std::vector<int> held;

  // 1. start the admitted columns: x = 0, r = b, ||b||^2, z = M^-1 r, p = z
  std::vector<int> J;
  for (int c = 0; c < k_; ++c)
    if (slot_[c].used && slot_[c].fresh) J.push_back(c);
  if (!J.empty()) {
    const double t = now_s();
    for (int c : J) {
      Slot& sl = slot_[c];
      GN_HIP(hipMemsetAsync(X + c * n, 0, sizeof(double) * n, s_));
      gnk::scatter_free(p, sl.col.b, R + c * n, s_);
      double* h = &hsc_[(size_t)c * S_N];
      std::fill(h, h + S_N, 0.0);
      h[S_MAXIT] = (double)sl.col.maxit;
      h[S_RTOL] = sl.col.rtol;
      sl.fresh = false;
      sl.t0 = t;
    }
    phase_begin(J, held);
    gnk::dot_mc(n, k_, R, R, part, ps, scal, s_);
    gnk::finalize_mc(part, ps, nbr, OP_BB, k_, scal, hist, hs, 0.0, s_);
    apply_m(OP_RZ0);
    gnk::copy_mc(n, k_, P, Z, scal, s_);
    phase_end(held);
  }

  // 2. one chunk of CG iterations for the live columns
  bool live = false;
  for (int c = 0; c < k_; ++c) live |= slot_[c].used && hsc_[(size_t)c * S_N + S_DONE] == 0.0;
  if (live) {
    for (int it = 0; it < chunk_; ++it) {
      gnk::spmv_mc(p, P, Q, k_, part, ps, scal, s_);
      gnk::finalize_mc(part, ps, nbs, OP_ALPHA, k_, scal, hist, hs, 0.0, s_);
      gnk::update_xr_mc(n, k_, X, R, P, Q, scal, part, ps, s_);
      gnk::finalize_mc(part, ps, nbr, OP_RR, k_, scal, hist, hs, 0.0, s_);
      apply_m(OP_BETA);
      gnk::update_p_mc(n, k_, P, Z, scal, s_);
    }
    read_scal();
  }

  // 3. columns whose CG sequence ended: ||b - A x||^2 (A x left in Q, b in Z)
  std::vector<int> F;
  for (int c = 0; c < k_; ++c)
    if (slot_[c].used && hsc_[(size_t)c * S_N + S_DONE] != 0.0) F.push_back(c);
  if (F.empty()) return;
  std::vector<double> floor2(k_, 0.0), tr(k_, 0.0), hpart((size_t)ps * k_);
  for (int c : F) floor2[c] = kEps * kEps * gnh::absmv_norm2(p, X + c * n, s_);
  gnk::spmv_mc(p, X, Q, k_, nullptr, ps, nullptr, s_);
  for (int c : F) gnk::scatter_free(p, slot_[c].col.b, Z + c * n, s_);
  gnk::sub_mc(n, k_, Z, Q, nullptr, part, ps, nullptr, s_);
  GN_HIP(hipMemcpyAsync(hpart.data(), part, sizeof(double) * ps * k_, hipMemcpyDeviceToHost, s_));
  GN_HIP(hipStreamSynchronize(s_));
  std::vector<int> again, retire;
  for (int c : F) {
    double t = 0.0;
    for (int i = 0; i < nbr; ++i) t += hpart[(size_t)c * ps + i];
    tr[c] = t;
    Slot& sl = slot_[c];
    const double* h = &hsc_[(size_t)c * S_N];
    if (sl.first_iters < 0) sl.first_iters = (int)h[S_ITER];
    sl.fin.assign(h, h + S_N);
    // the recursive residual drifts from b - A x (attainable accuracy of CG):
    // restart from b - A x unless it meets the tolerance or sits at the
    // rounding floor eps || |A| |x| || of an FP64 solution
    const double tol2 = sl.col.rtol * sl.col.rtol * h[S_BB];
    const bool re = sl.restarts < 2 && h[S_BREAK] == 0.0 && h[S_BB] > 0.0 && t > tol2 &&
                    t > kFloorFactor * kFloorFactor * floor2[c] && (int)h[S_ITER] < (int)h[S_MAXIT];
    // a restarted sequence stops below rtol (uploaded with the scalars by phase_begin)
    if (re) hsc_[(size_t)c * S_N + S_TOL2] = gnh::restart_tol2(sl.col.rtol, floor2[c], h[S_BB]);
    (re ? again : retire).push_back(c);
  }
  if (!again.empty()) {
    phase_begin(again, held);
    gnk::sub_mc(n, k_, Z, Q, R, part, ps, scal, s_);   // r = b - A x
    gnk::finalize_mc(part, ps, nbr, OP_RESTART, k_, scal, hist, hs, 0.0, s_);
    apply_m(OP_RZ0);
    gnk::copy_mc(n, k_, P, Z, scal, s_);
    phase_end(held);
    for (int c : again) ++slot_[c].restarts;
  }
  if (retire.empty()) return;
  std::vector<std::vector<double>> hh(retire.size());
  for (size_t i = 0; i < retire.size(); ++i) {
    const int c = retire[i];
    Slot& sl = slot_[c];
    gnk::gather_free(p, X + c * n, sl.col.x, s_);
    hh[i].assign((size_t)2 * std::max(sl.first_iters, 1), 0.0);
    if (sl.first_iters > 0)
      GN_HIP(hipMemcpyAsync(hh[i].data(), hist + (int64_t)c * hs, sizeof(double) * 2 * sl.first_iters,
                            hipMemcpyDeviceToHost, s_));
  }
  GN_HIP(hipStreamSynchronize(s_));
  const double tnow = now_s();
  for (size_t i = 0; i < retire.size(); ++i) {
    const int c = retire[i];
    Slot& sl = slot_[c];
    const double* h = sl.fin.data();
    const double bb = h[S_BB], rr = h[S_RR];
    const bool conv = bb == 0.0 || rr <= sl.col.rtol * sl.col.rtol * bb;
    SlotResult r;
    r.col = sl.col;
    r.st = h[S_BREAK] != 0.0 ? GN_ERR_BREAKDOWN : (conv ? GN_OK : GN_WARN_MAXIT);
    gn_solve_report& Rp = r.rep;
    std::memset(&Rp, 0, sizeof(Rp));
    Rp.iters = (int)h[S_ITER];
    Rp.converged = conv ? 1 : 0;
    Rp.rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    Rp.true_rel_res = bb > 0 ? std::sqrt(tr[c] / bb) : 0.0;
    Rp.res_floor = bb > 0 ? std::sqrt(floor2[c] / bb) : 0.0;
    Rp.t_solve_s = tnow - sl.t0;
    Rp.iters_first = sl.first_iters;
    Rp.restarts = sl.restarts;
    Rp.cond_est = gnh::cond_from_hist(hh[i].data(), sl.first_iters);
    out.push_back(r);
    sl = Slot();   // free; its done flag stays set on the device and in the mirror
  }
}

// ---------------------------------------------------------------------------
// gn_server
// ---------------------------------------------------------------------------
namespace {

struct Request {
  int op = -1;
  int nrhs = 0;
  int remaining = 0;
  double t_submit = 0.0, t_done = 0.0;
  gn_status st = GN_OK;
  std::string msg;   // why the request failed (empty: it did not)
  bool done = false;
  std::vector<gn_solve_report> rep;
};

// Host copy of an operator's description (gn_server_register): the server
// builds the operator from it when a request needs it and the budget allows,
// and may destroy and rebuild it later.
struct Spec {
  int ne[3] = {0, 0, 0};
  std::vector<double> xn[3];
  int map_kind = 0;
  double map_par[3] = {0, 0, 0};
  int pde = 0, n_mat = 0;
  std::vector<double> mat, elem_angle, elem_tilt, elem_k, body, traction;
  std::vector<int32_t> elem_mat;
  std::vector<uint8_t> dirichlet;
  int nrhs = 1;
  gn_dd_opts dd{};
  std::vector<int32_t> cuts[3];
};

struct Operator {
  int id = -1;
  gn_problem* p = nullptr;
  gn_precond* pc = nullptr;
  hipStream_t s = nullptr;
  int64_t bytes = 0;        // measured footprint while resident (budget share)
  int64_t est = 0;          // a-priori footprint (server-built operators)
  int64_t n_free = 0;
  std::unique_ptr<Spec> spec;   // set: the server builds, evicts and rebuilds the operator
  bool resident = true;
  bool building = false;
  bool evict_req = false;
  double last_use = 0.0;
  int builds = 0, evictions = 0;
  std::deque<SlotColumn> queue;
  std::thread worker;
  bool stop = false;
  bool failed = false;
  int inflight = 0;   // columns queued or in slots
};

}  // namespace

struct gn_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_mem;
  int device = 0;
  int slots = 16, chunk = 8, maxit_cap = 2000;
  int64_t budget = 0, used = 0;
  std::vector<std::unique_ptr<Operator>> ops;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_ticket = 1;
};

static void merge_status(gn_status& into, gn_status st) {
  if (st < 0 && into >= 0) into = st;
  else if (st > 0 && into == GN_OK) into = st;
}

// finish every column of op that is queued or in flight with status st (lock held)
static void fail_operator(gn_server* sv, Operator& o, gn_status st, const std::string& msg = std::string()) {
  const int op = o.id;
  o.failed = true;
  o.queue.clear();
  for (auto& kv : sv->reqs) {
    Request& q = *kv.second;
    if (q.op != op || q.done) continue;
    merge_status(q.st, st);
    if (q.msg.empty()) q.msg = msg;
    q.remaining = 0;
    q.done = true;
    q.t_done = now_s();
  }
  o.inflight = 0;
  sv->cv_done.notify_all();
  sv->cv_mem.notify_all();
}

// Reserve `need` bytes of the budget for operator self (lock held): while they
// do not fit, ask the least recently used idle server-built operator to evict
// itself and wait for the memory to come back.  Returns false when even
// evicting every idle server-built operator cannot make room (the resident
// caller-registered operators and the busy ones hold the rest).
static bool reserve_budget(gn_server* sv, std::unique_lock<std::mutex>& lk, Operator* self, int64_t need) {
  for (;;) {
    if (self && self->stop) return false;
    if (sv->used + need <= sv->budget) {
      sv->used += need;
      return true;
    }
    int64_t fixed = 0;    // resident caller-registered operators: never evicted
    Operator* victim = nullptr;
    bool pending = false; // memory that will come back: evictions, builds, busy server-built operators
    for (auto& up : sv->ops) {
      Operator* o = up.get();
      if (!o || o == self) continue;
      if (!o->spec) {
        if (o->resident) fixed += o->bytes;
        continue;
      }
      if (o->building || o->evict_req) {
        pending = true;
        continue;
      }
      if (!o->resident) continue;
      if (o->queue.empty() && o->inflight == 0) {
        if (!victim || o->last_use < victim->last_use) victim = o;
      } else {
        pending = true;
      }
    }
    if (fixed + need > sv->budget) return false;
    if (victim) {
      victim->evict_req = true;
      sv->cv_work.notify_all();
    } else if (!pending) {
      return false;
    }
    sv->cv_mem.wait(lk);
  }
}

// Build a server-registered operator on its own stream (lock not held).
static gn_status build_operator(Operator& o, std::string& err) {
  const Spec& sp = *o.spec;
  gn_grid g{};
  for (int a = 0; a < 3; ++a) {
    g.ne[a] = sp.ne[a];
    g.xn[a] = sp.xn[a].data();
  }
  g.map_kind = sp.map_kind;
  g.map_par = sp.map_par;
  gn_material m{};
  m.pde = sp.pde;
  m.n_mat = sp.n_mat;
  m.mat = sp.mat.empty() ? nullptr : sp.mat.data();
  m.elem_mat = sp.elem_mat.empty() ? nullptr : sp.elem_mat.data();
  m.elem_angle = sp.elem_angle.empty() ? nullptr : sp.elem_angle.data();
  m.elem_tilt = sp.elem_tilt.empty() ? nullptr : sp.elem_tilt.data();
  m.elem_k = sp.elem_k.empty() ? nullptr : sp.elem_k.data();
  gn_loads l{};
  l.dirichlet = sp.dirichlet.data();
  l.body = sp.body.empty() ? nullptr : sp.body.data();
  l.nrhs = sp.nrhs;
  l.traction = sp.traction.empty() ? nullptr : sp.traction.data();
  gn_dd_opts dd = sp.dd;
  for (int a = 0; a < 3; ++a) dd.cuts[a] = sp.cuts[a].data();
  gn_problem* p = nullptr;
  gn_precond* pc = nullptr;
  gn_status st = gn_assemble(&g, &m, &l, o.s, &p);
  if (st == GN_OK) {
    gn_setup_report rep{};
    st = gn_setup_geneo(p, &dd, o.s, &pc, &rep);
    if (st != GN_OK) gn_destroy_problem(p);
  }
  if (st != GN_OK) {
    err = gn_last_error();
    return st;
  }
  o.p = p;
  o.pc = pc;
  return GN_OK;
}

static void worker_main(gn_server* sv, Operator* op_ptr) {
  Operator& o = *op_ptr;
  (void)hipSetDevice(sv->device);
  std::unique_ptr<SlotEngine> eng;
  auto make_engine = [&]() -> bool {
    try {
      eng.reset(new SlotEngine(o.p, o.pc, sv->slots, sv->chunk, sv->maxit_cap, o.s));
      return true;
    } catch (const gn_error& e) {
      std::lock_guard<std::mutex> lk(sv->mu);
      fail_operator(sv, o, e.code, e.msg);
      return false;
    }
  };
  if (o.resident && !make_engine()) return;
  std::vector<SlotResult> res;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] {
        return o.stop || !o.queue.empty() || (eng && eng->busy()) || (o.evict_req && o.queue.empty());
      });
      const bool busy = eng && eng->busy();
      if (o.stop && o.queue.empty() && !busy) return;   // stop requested and drained
      if (o.evict_req && o.queue.empty() && !busy) {
        // evict: free the operator's device memory; it is rebuilt on demand
        lk.unlock();
        eng.reset();
        (void)hipStreamSynchronize(o.s);
        gn_destroy_precond(o.pc);
        gn_destroy_problem(o.p);
        lk.lock();
        o.pc = nullptr;
        o.p = nullptr;
        sv->used -= o.bytes;
        o.bytes = 0;
        o.resident = false;
        o.evict_req = false;
        ++o.evictions;
        sv->cv_mem.notify_all();
        continue;
      }
      o.evict_req = false;
      if (!o.resident) {
        // admission: the operator is built once its a-priori footprint fits
        // the estimate counts nev vectors per subdomain; cluster completion
        // can add a few (0.1 % of the bytes on the laminate catalogue), so the
        // build reserves 1/32 more and settles on the measured footprint
        o.building = true;
        const int64_t reserve = o.est + o.est / 32;
        if (!reserve_budget(sv, lk, &o, reserve)) {
          o.building = false;
          fail_operator(sv, o, GN_ERR_OOM,
                        "operator " + std::to_string(o.id) + " needs " + std::to_string(reserve) +
                            " bytes to build (estimate + 1/32); the budget of " + std::to_string(sv->budget) +
                            " bytes cannot make room for it");
          o.failed = false;          // later requests may fit once others are removed
          continue;
        }
        lk.unlock();
        std::string err;
        const gn_status st = build_operator(o, err);
        int64_t measured = 0;
        if (st == GN_OK) {
          try {
            gnh::ensure_batch_workspace(o.p, o.pc, sv->maxit_cap, o.s);
            GN_HIP(hipStreamSynchronize(o.s));
            measured = gnh::resident_bytes(o.p->owned) + gnh::resident_bytes(o.pc->owned);
          } catch (const gn_error& e) {
            lk.lock();
            sv->used -= reserve;
            o.building = false;
            fail_operator(sv, o, e.code, e.msg);
            return;
          }
        }
        lk.lock();
        sv->used -= reserve;
        o.building = false;
        if (st != GN_OK) {
          gn_set_error(st, err);
          fail_operator(sv, o, st, err);
          return;
        }
        sv->used += measured;
        o.bytes = measured;
        o.resident = true;
        ++o.builds;
        sv->cv_mem.notify_all();
        lk.unlock();
        if (!make_engine()) return;
        lk.lock();
      }
      while (!o.queue.empty() && eng->free_slots() > 0) {
        eng->admit(o.queue.front());
        o.queue.pop_front();
      }
      o.last_use = now_s();
    }
    res.clear();
    gn_status err = GN_OK;
    std::string err_msg;
    try {
      eng->step(res);
    } catch (const gn_error& e) {
      err = e.code;
      err_msg = e.msg;
    } catch (...) {
      err = GN_ERR_DEVICE;
      err_msg = "unexpected exception in the solve loop";
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    if (err != GN_OK) {
      fail_operator(sv, o, err, err_msg);
      return;
    }
    const double t = now_s();
    for (const SlotResult& r : res) {
      Request& q = *(Request*)r.col.tag;
      q.rep[r.col.index] = r.rep;
      merge_status(q.st, r.st);
      --o.inflight;
      if (--q.remaining == 0) {
        q.done = true;
        q.t_done = t;
      }
    }
    o.last_use = t;
    if (!res.empty()) {
      sv->cv_done.notify_all();
      if (o.inflight == 0) sv->cv_mem.notify_all();   // an idle operator can now be evicted
    }
  }
}

#define SV_TRY try {
#define SV_CATCH                                   \
  }                                                \
  catch (const gn_error& e) {                      \
    gn_set_error(e.code, e.msg);                   \
    return e.code;                                 \
  }                                                \
  catch (...) {                                    \
    gn_set_error(GN_ERR_DEVICE, "unexpected exception"); \
    return GN_ERR_DEVICE;                          \
  }

extern "C" gn_status gn_server_create(const gn_server_opts* opts, gn_server** out) {
  SV_TRY
  if (!out) throw gn_error{GN_ERR_ARG, "null argument"};
  *out = nullptr;
  std::unique_ptr<gn_server> sv(new gn_server());
  GN_HIP(hipGetDevice(&sv->device));
  size_t fr = 0, tot = 0;
  GN_HIP(hipMemGetInfo(&fr, &tot));
  sv->budget = (int64_t)tot;
  if (opts) {
    if (opts->slots < 0 || opts->slots > gnk::mc_width()) throw gn_error{GN_ERR_ARG, "slots must lie in 0..16"};
    if (opts->hbm_budget < 0 || opts->check_every < 0 || opts->maxit_cap < 0)
      throw gn_error{GN_ERR_ARG, "negative option"};
    if (opts->slots > 0) sv->slots = opts->slots;
    if (opts->check_every > 0) sv->chunk = opts->check_every;
    if (opts->maxit_cap > 0) sv->maxit_cap = opts->maxit_cap;
    if (opts->hbm_budget > 0) sv->budget = opts->hbm_budget;
  }
  *out = sv.release();
  return GN_OK;
  SV_CATCH
}

extern "C" gn_status gn_resident_bytes(const gn_problem* p, const gn_precond* pc, int64_t* bytes) {
  SV_TRY
  if (!p || !bytes) throw gn_error{GN_ERR_ARG, "null argument"};
  if (pc && pc->prob != p) throw gn_error{GN_ERR_ARG, "preconditioner built for another problem"};
  *bytes = gnh::resident_bytes(p->owned) + (pc ? gnh::resident_bytes(pc->owned) : 0);
  return GN_OK;
  SV_CATCH
}

extern "C" gn_status gn_server_add(gn_server* sv, gn_problem* p, gn_precond* pc, int32_t* op, int64_t* bytes) {
  SV_TRY
  if (!sv || !p || !op) throw gn_error{GN_ERR_ARG, "null argument"};
  if (pc && pc->prob != p) throw gn_error{GN_ERR_ARG, "preconditioner built for another problem"};
  std::unique_lock<std::mutex> lk(sv->mu);
  for (auto& o : sv->ops)
    if (o && o->p == p) throw gn_error{GN_ERR_ARG, "problem already served"};
  // the batched workspace is part of the resident footprint: allocate it now
  gnh::ensure_batch_workspace(p, pc, sv->maxit_cap, nullptr);
  GN_HIP(hipStreamSynchronize(nullptr));
  const int64_t b = gnh::resident_bytes(p->owned) + (pc ? gnh::resident_bytes(pc->owned) : 0);
  if (bytes) *bytes = b;
  // idle server-built operators are evicted to make room if needed
  if (!reserve_budget(sv, lk, nullptr, b))
    throw gn_error{GN_ERR_OOM, "operator footprint exceeds the server's remaining HBM budget"};
  std::unique_ptr<Operator> o(new Operator());
  o->p = p;
  o->pc = pc;
  o->bytes = b;
  o->n_free = p->n_free;
  o->last_use = now_s();
  GN_HIP(hipStreamCreateWithFlags(&o->s, hipStreamNonBlocking));
  const int id = (int)sv->ops.size();
  o->id = id;
  Operator* raw = o.get();
  sv->ops.push_back(std::move(o));
  raw->worker = std::thread(worker_main, sv, raw);
  *op = id;
  return GN_OK;
  SV_CATCH
}

extern "C" gn_status gn_server_register(gn_server* sv, const gn_grid* grid, const gn_material* mat,
                                        const gn_loads* loads, const gn_dd_opts* opts, int32_t* op,
                                        int64_t* est_bytes) {
  SV_TRY
  if (!sv || !grid || !mat || !loads || !opts || !op) throw gn_error{GN_ERR_ARG, "null argument"};
  std::unique_ptr<Spec> sp(new Spec());
  int64_t n_elem = 1, n_node = 1;
  for (int a = 0; a < 3; ++a) {
    if (grid->ne[a] < 1 || !grid->xn[a]) throw gn_error{GN_ERR_ARG, "bad grid"};
    sp->ne[a] = grid->ne[a];
    sp->xn[a].assign(grid->xn[a], grid->xn[a] + grid->ne[a] + 1);
    n_elem *= grid->ne[a];
    n_node *= grid->ne[a] + 1;
  }
  sp->map_kind = grid->map_kind;
  if (grid->map_kind == 1) {
    if (!grid->map_par) throw gn_error{GN_ERR_ARG, "ramp map needs map_par"};
    for (int a = 0; a < 3; ++a) sp->map_par[a] = grid->map_par[a];
  }
  if (mat->pde != 0 && mat->pde != 1) throw gn_error{GN_ERR_ARG, "pde must be 0 or 1"};
  const int nc = mat->pde == 1 ? 3 : 1;
  sp->pde = mat->pde;
  sp->n_mat = mat->n_mat;
  auto copy_d = [](std::vector<double>& dst, const double* src, int64_t n) {
    if (src) dst.assign(src, src + n);
  };
  if (mat->pde == 1) {
    if (!mat->mat || !mat->elem_mat || mat->n_mat < 1) throw gn_error{GN_ERR_ARG, "elasticity needs materials"};
    copy_d(sp->mat, mat->mat, 9 * (int64_t)mat->n_mat);
    sp->elem_mat.assign(mat->elem_mat, mat->elem_mat + n_elem);
    copy_d(sp->elem_angle, mat->elem_angle, n_elem);
    copy_d(sp->elem_tilt, mat->elem_tilt, n_elem);
  } else {
    if (!mat->elem_k) throw gn_error{GN_ERR_ARG, "diffusion needs elem_k"};
    copy_d(sp->elem_k, mat->elem_k, n_elem);
  }
  if (!loads->dirichlet || loads->nrhs < 1) throw gn_error{GN_ERR_ARG, "bad loads"};
  sp->dirichlet.assign(loads->dirichlet, loads->dirichlet + n_node * nc);
  copy_d(sp->body, loads->body, n_elem * nc);
  sp->nrhs = loads->nrhs;
  copy_d(sp->traction, loads->traction, (int64_t)loads->nrhs * grid->ne[0] * grid->ne[1] * nc);
  sp->dd = *opts;
  for (int a = 0; a < 3; ++a) {
    if (opts->nparts[a] < 1 || !opts->cuts[a]) throw gn_error{GN_ERR_ARG, "bad cuts"};
    sp->cuts[a].assign(opts->cuts[a], opts->cuts[a] + opts->nparts[a] + 1);
    sp->dd.cuts[a] = nullptr;
  }
  int64_t est = 0;
  if (gn_footprint(grid, mat->pde, opts, &est) != GN_OK) throw gn_error{GN_ERR_ARG, gn_last_error()};
  int64_t n_free = 0;
  for (uint8_t d : sp->dirichlet) n_free += d ? 0 : 1;
  if (n_free == 0) throw gn_error{GN_ERR_ARG, "no free DOFs"};
  std::lock_guard<std::mutex> lk(sv->mu);
  // a build reserves the estimate plus 1/32 (see the worker's admission step)
  if (est + est / 32 > sv->budget)
    throw gn_error{GN_ERR_OOM, "operator footprint " + std::to_string(est) + " bytes (+1/32 build margin) exceeds the server's HBM budget of " + std::to_string(sv->budget) + " bytes"};
  std::unique_ptr<Operator> o(new Operator());
  o->spec = std::move(sp);
  o->resident = false;
  o->est = est;
  o->n_free = n_free;
  GN_HIP(hipStreamCreateWithFlags(&o->s, hipStreamNonBlocking));
  const int id = (int)sv->ops.size();
  o->id = id;
  Operator* raw = o.get();
  sv->ops.push_back(std::move(o));
  raw->worker = std::thread(worker_main, sv, raw);
  *op = id;
  if (est_bytes) *est_bytes = est;
  return GN_OK;
  SV_CATCH
}

extern "C" gn_status gn_server_operator_info(gn_server* sv, int32_t op, int32_t* resident, int32_t* builds,
                                             int32_t* evictions, int64_t* bytes) {
  SV_TRY
  if (!sv) throw gn_error{GN_ERR_ARG, "null argument"};
  std::lock_guard<std::mutex> lk(sv->mu);
  if (op < 0 || op >= (int)sv->ops.size() || !sv->ops[op]) throw gn_error{GN_ERR_ARG, "unknown operator"};
  const Operator& o = *sv->ops[op];
  if (resident) *resident = o.resident ? 1 : 0;
  if (builds) *builds = o.builds;
  if (evictions) *evictions = o.evictions;
  if (bytes) *bytes = o.resident ? o.bytes : o.est;
  return GN_OK;
  SV_CATCH
}

// stop the worker of op after its queued and running columns (lock not held)
static void retire_operator(gn_server* sv, int op) {
  Operator* o = nullptr;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    o = sv->ops[op].get();
    if (!o) return;
    o->stop = true;
  }
  sv->cv_work.notify_all();
  sv->cv_mem.notify_all();
  if (o->worker.joinable()) o->worker.join();
  std::lock_guard<std::mutex> lk(sv->mu);
  (void)hipStreamSynchronize(o->s);
  if (o->spec && o->resident) {
    gn_destroy_precond(o->pc);
    gn_destroy_problem(o->p);
  }
  (void)hipStreamDestroy(o->s);
  if (o->resident) sv->used -= o->bytes;
  sv->ops[op].reset();
  sv->cv_mem.notify_all();
}

extern "C" gn_status gn_server_remove(gn_server* sv, int32_t op) {
  SV_TRY
  if (!sv) throw gn_error{GN_ERR_ARG, "null argument"};
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (op < 0 || op >= (int)sv->ops.size() || !sv->ops[op]) throw gn_error{GN_ERR_ARG, "unknown operator"};
  }
  retire_operator(sv, op);
  return GN_OK;
  SV_CATCH
}

extern "C" gn_status gn_server_submit(gn_server* sv, int32_t op, const double* b_dev, double* x_dev, int32_t nrhs,
                                      int64_t ld, double rtol, int32_t maxit, int64_t* ticket) {
  SV_TRY
  if (!sv || !b_dev || !x_dev || !ticket) throw gn_error{GN_ERR_ARG, "null argument"};
  std::lock_guard<std::mutex> lk(sv->mu);
  if (op < 0 || op >= (int)sv->ops.size() || !sv->ops[op]) throw gn_error{GN_ERR_ARG, "unknown operator"};
  Operator& o = *sv->ops[op];
  if (o.failed) throw gn_error{GN_ERR_DEVICE, "operator's worker stopped after an error"};
  if (nrhs < 1 || ld < o.n_free) throw gn_error{GN_ERR_ARG, "bad nrhs/ld"};
  if (!(rtol > 0.0) || maxit < 1 || maxit > sv->maxit_cap)
    throw gn_error{GN_ERR_ARG, "rtol > 0 and 1 <= maxit <= maxit_cap required"};
  std::unique_ptr<Request> q(new Request());
  q->op = op;
  q->nrhs = nrhs;
  q->remaining = nrhs;
  q->t_submit = now_s();
  q->rep.assign(nrhs, gn_solve_report());
  for (int c = 0; c < nrhs; ++c) {
    SlotColumn col;
    col.b = b_dev + c * ld;
    col.x = x_dev + c * ld;
    col.rtol = rtol;
    col.maxit = maxit;
    col.tag = q.get();
    col.index = c;
    o.queue.push_back(col);
  }
  o.inflight += nrhs;
  const int64_t t = sv->next_ticket++;
  sv->reqs.emplace(t, std::move(q));
  *ticket = t;
  sv->cv_work.notify_all();
  return GN_OK;
  SV_CATCH
}

extern "C" gn_status gn_server_wait(gn_server* sv, int64_t ticket, double timeout_s, gn_solve_report* reports,
                                    double* latency_s) {
  SV_TRY
  if (!sv) throw gn_error{GN_ERR_ARG, "null argument"};
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) throw gn_error{GN_ERR_ARG, "unknown ticket"};
  Request* q = it->second.get();
  if (timeout_s < 0) {
    sv->cv_done.wait(lk, [&] { return q->done; });
  } else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return q->done; })) {
    return GN_PENDING;
  }
  if (reports) std::copy(q->rep.begin(), q->rep.end(), reports);
  if (latency_s) *latency_s = q->t_done - q->t_submit;
  const gn_status st = q->st;
  const std::string msg = q->msg.empty() ? std::string("request failed on the device") : q->msg;
  sv->reqs.erase(it);
  if (st < 0) gn_set_error(st, msg.c_str());
  return st;
  SV_CATCH
}

extern "C" void gn_server_destroy(gn_server* sv) {
  if (!sv) return;
  for (int op = 0; op < (int)sv->ops.size(); ++op) retire_operator(sv, op);
  delete sv;
}
