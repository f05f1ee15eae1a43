// Pools of resident simulations: host analysis of many meshes, admission
// into groups (one concatenated device mesh each) under a device-memory
// budget, batched steps of any subset, and the request loop that serves
// step requests with continuous batching (a group steps every simulation
// with a queued request; requests arriving meanwhile join its next batch;
// groups step concurrently on their own streams).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/qnsim.h"
#include "ctx.hpp"

using namespace qn;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct PoolSim {
  qnsim* c = nullptr;        // analyzed host context (mesh, factor); no device state
  int group = -1;            // -1: staged
  int slot = -1;             // position in its group
  bool removed = false;
  bool admitting = false;    // staged, its group is being built by a commit
  bool has_force = false;    // its slice of the group's force array is set
  std::vector<double> force; // host copy of that force (n x 3, caller order)
  int64_t est_bytes = 0;     // device-memory estimate
  std::vector<double> x0, v0;  // initial state until admitted
};

struct PoolGroup {
  DeviceMesh D;
  std::vector<int> ids;      // pool ids in group order
  std::vector<int> cv0;      // first caller vertex of each member in xs / vs
  double* xs = nullptr;      // states of the members, concatenated n x 3
  double* vs = nullptr;
  double* fx = nullptr;      // external forces, as xs (allocated on the first force set)
  int64_t bytes = 0;
  int live = 0;              // members not removed
  bool busy = false;         // a step is running
  bool repacking = false;    // a commit is rebuilding it without its removed members (it
                             // keeps serving; the members' host data stays meanwhile)
  int trials = 0;            // line-search trials per cycle from the tuner (0: the pool's)
};

struct Request {
  int64_t ticket;
  int sim;
  double t_submit;
  std::shared_ptr<const std::vector<double>> force;  // this step's own f_ext, or null
};

struct Done {
  int rc;
  qnsim_stats st;
  double latency;
};

}  // namespace

struct qnsim_pool {
  qnsim_options opt;
  double h = 0.0;
  int64_t budget = 0, used = 0;
  int64_t steps_done = 0, batches_done = 0;
  std::vector<PoolSim> sims;
  std::vector<std::unique_ptr<PoolGroup>> groups;
  // a commit is building groups outside the lock; commits, time-step
  // changes and tuning wait for it (one administrative change at a time)
  bool admin_busy = false;
  std::mutex mu;
  std::condition_variable cv;
  std::string last_error;
  // request loop
  std::vector<std::thread> lanes;
  bool serving = false, stopping = false;
  std::deque<Request> queue;
  std::unordered_map<int64_t, Done> done;
  int64_t next_ticket = 1;
};

namespace {

int pfail(qnsim_pool* p, int code, const std::string& msg) {
  p->last_error = msg;
  return code;
}

StepParams pool_params(const qnsim_pool* p) {
  StepParams s;
  s.iterations = p->opt.iterations;
  s.history = p->opt.history;
  s.max_halvings = p->opt.max_halvings;
  s.budget = p->opt.trials_per_cycle;
  s.graph = p->opt.step_graph;
  s.direction = p->opt.direction;
  s.cheb_delay = p->opt.cheb_delay;
  s.cheb_rho = p->opt.cheb_rho;
  s.gamma = p->opt.gamma;
  s.backtrack = p->opt.backtrack;
  for (int i = 0; i < 3; ++i) s.grav[i] = p->opt.gravity[i];
  s.h = p->h;
  return s;
}

void stats_of(const SimStat& t, qnsim_stats* s) {
  s->iterations_run = t.iters;
  s->ls_trials = t.trials;
  s->ls_exhausted = t.exhausted;
  s->lbfgs_skipped = t.skipped;
  s->fallbacks = t.fallbacks;
  s->reserved = 0;
  s->g_first = t.g_first;
  s->g_last = t.g_last;
  s->grad_norm_first = std::sqrt(t.gnorm2_first);
  s->grad_norm_last = NAN;
}

// Device bytes of one simulation in a group (the allocations of the upload
// and of dev_alloc, plus its state arrays).
int64_t estimate_bytes(const qnsim* c, int history) {
  const Factor& F = c->factor;
  const int64_t n = c->n, nf = c->nf, T = c->T, slots = history + 1;
  int64_t packed = 0, vp = 0;
  for (const Supernode& S : F.sn) {
    packed += (int64_t)S.ncol * (S.ncol + 1) / 2 + (int64_t)S.nbelow * S.ncol;
    vp += 3 * (int64_t)(S.ncol + S.nbelow) * 4;  // update layers (a few per supernode)
  }
  int64_t b = 0;
  b += T * (16 + 72 + 8 + 4 + 4 + 8 + 8);           // tv, Bm, vol, tmat, tperm, psi, lc_idx
  b += n * (8 + 4 + 4 + 4 * 24 + 2 * 24);           // mass, vperm, vsim, x0 v0 y X, state
  b += nf * (24 * 5 + 2 * slots * 24 + 4 * 8 + 3 * 28);  // G d r q z, S/T rings, partials
  b += 2 * packed * 8 + vp * 8;                     // forward/backward blocks, layers
  b += (int64_t)F.rows.size() * 8 + (int64_t)F.sn.size() * 64 * 8;  // rows, rel, items
  b += (T / 256 + nf / 64 + 3 * nf / 256 + 16) * (32 + 8 * 60);     // block tables, partials
  b += sizeof(Ctl) + sizeof(SimStat) + 64;
  return b + b / 16;
}

// One simulation described by d, analyzed on the host for the pool's h.
int analyze_one(const qnsim_pool* p, const qnsim_mesh_desc& d, PoolSim& out, std::string& err) {
  qnsim_options o = p->opt;
  qnsim_t* c = nullptr;
  int rc = qnsim_create(&o, &c);
  if (rc) { err = "invalid options"; return rc; }
  auto bail = [&](int code) {
    err = qnsim_last_error(c);
    qnsim_destroy(c);
    return code;
  };
  if ((rc = qnsim_set_mesh(c, d.n_verts, d.rest_xyz, d.n_tets, d.tets))) return bail(rc);
  if (d.n_pinned > 0 && (rc = qnsim_set_pinned(c, d.n_pinned, d.pinned))) return bail(rc);
  if ((rc = qnsim_set_materials(c, d.n_mat, d.mats, d.tet_mat))) return bail(rc);
  if ((rc = qnsim_analyze(c, p->h))) return bail(rc);
  const size_t n3 = 3 * (size_t)d.n_verts;
  out.x0.assign(n3, 0.0);
  out.v0.assign(n3, 0.0);
  for (size_t i = 0; i < n3; ++i) {
    out.x0[i] = d.x0 ? d.x0[i] : d.rest_xyz[i];
    out.v0[i] = d.v0 ? d.v0[i] : 0.0;
    if (!std::isfinite(out.x0[i]) || !std::isfinite(out.v0[i])) {
      err = "non-finite initial state";
      qnsim_destroy(c);
      return QNSIM_E_NONFINITE;
    }
  }
  out.c = c;
  out.est_bytes = estimate_bytes(c, p->opt.history);
  return QNSIM_OK;
}

void free_group(PoolGroup& g) {
  if (g.xs) (void)hipFree(g.xs);
  if (g.vs) (void)hipFree(g.vs);
  if (g.fx) (void)hipFree(g.fx);
  g.xs = g.vs = g.fx = nullptr;
  dev_free(g.D);
}

// What a commit needs to build one group, taken from the pool's tables under
// the lock so that the build itself runs without it: the members' pool ids,
// their analysed host contexts (which stay put while the pool grows) and
// their initial states (moved out of the staged records, moved back on a
// failure).
struct GroupBuild {
  std::vector<int> ids;
  std::vector<const qnsim*> cs;
  std::vector<std::vector<double>> x0, v0;
  std::unique_ptr<PoolGroup> g;
  int rc = QNSIM_OK;
  std::string err;
};

// Uploads the members of b as one group (factored for h); returns 0 or an
// error code. Touches no pool table: runs without the pool lock, while other
// groups step on their own (non-blocking) streams.
int build_group(const qnsim_options& opt, double h, GroupBuild& b) {
  auto g = std::make_unique<PoolGroup>();
  int n = 0;
  for (const qnsim* c : b.cs) {
    g->cv0.push_back(n);
    n += c->n;
  }
  if (hipSetDevice(opt.device) != hipSuccess) {
    b.err = "hipSetDevice failed";
    return QNSIM_E_DEVICE;
  }
  int rc = upload_sims(b.cs, opt, h, g->D, b.err);
  if (rc) { free_group(*g); return rc; }
  const size_t bytes = 3 * (size_t)n * sizeof(double);
  if (hipMalloc((void**)&g->xs, bytes) != hipSuccess || hipMalloc((void**)&g->vs, bytes) != hipSuccess) {
    free_group(*g);
    b.err = "state allocation failed";
    return QNSIM_E_NOMEM;
  }
  for (size_t k = 0; k < b.cs.size(); ++k) {
    const size_t off = 3 * (size_t)g->cv0[k];
    if (hipMemcpy(g->xs + off, b.x0[k].data(), b.x0[k].size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->vs + off, b.v0[k].data(), b.v0[k].size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      free_group(*g);
      b.err = "state upload failed";
      return QNSIM_E_DEVICE;
    }
  }
  g->ids = b.ids;
  g->live = (int)b.ids.size();
  g->bytes = (int64_t)g->D.bytes + 2 * (int64_t)bytes;
  b.g = std::move(g);
  return QNSIM_OK;
}

// A group rebuilt without its removed members (their device memory is
// returned to the budget): the live members' host contexts and their slots
// in the old group. The old group keeps serving while the new one is built;
// their states (and forces) are copied over on the device when it replaces
// the old one.
struct Repack {
  int gi = -1;
  std::vector<int> ids, old_slots;
  std::vector<const qnsim*> cs;
  bool refactored = false;   // the pool's h differs from the analysed one
  std::unique_ptr<PoolGroup> g;
  int rc = QNSIM_OK;
  std::string err;
};

// Builds r.g from r's live members (mesh, factor, empty state arrays); reads
// only their host contexts, which stay while the old group is marked
// repacking. Runs without the lock.
int build_repack(const qnsim_options& opt, double h, int elem_tile, Repack& r) {
  auto g = std::make_unique<PoolGroup>();
  int n = 0;
  for (const qnsim* c : r.cs) {
    g->cv0.push_back(n);
    n += c->n;
  }
  if (hipSetDevice(opt.device) != hipSuccess) { r.err = "hipSetDevice failed"; return QNSIM_E_DEVICE; }
  qnsim_options o = opt;
  o.elem_tile = elem_tile;
  int rc = upload_sims(r.cs, o, h, g->D, r.err);
  // host factor values belong to an earlier h after a time-step change
  if (!rc && r.refactored) rc = dev_refactor_mesh(r.cs, g->D, h, nullptr, r.err);
  if (rc) { free_group(*g); return rc; }
  const size_t bytes = 3 * (size_t)n * sizeof(double);
  if (hipMalloc((void**)&g->xs, bytes) != hipSuccess || hipMalloc((void**)&g->vs, bytes) != hipSuccess) {
    free_group(*g);
    r.err = "state allocation failed";
    return QNSIM_E_NOMEM;
  }
  g->ids = r.ids;
  g->bytes = (int64_t)g->D.bytes + 2 * (int64_t)bytes;
  r.g = std::move(g);
  return QNSIM_OK;
}

// Moves the members' states (and forces) from the old group into the
// rebuilt one on the device; the old group is not stepping (the caller
// holds the lock and waited for it).
int repack_states(const PoolGroup& old, PoolGroup& g, const Repack& r, std::string& err) {
  size_t n = 0;
  for (const qnsim* c : r.cs) n += (size_t)c->n;
  const size_t bytes = 3 * n * sizeof(double);
  if (old.fx && !g.fx) {  // the first force was set while the group was rebuilt
    if (hipMalloc((void**)&g.fx, bytes) != hipSuccess) {
      g.fx = nullptr;
      err = "force allocation failed";
      return QNSIM_E_NOMEM;
    }
    g.bytes += (int64_t)bytes;
  }
  hipStream_t st = (hipStream_t)g.D.stream;
  hipError_t e = hipSuccess;
  for (size_t k = 0; k < r.cs.size() && e == hipSuccess; ++k) {
    const size_t dst = 3 * (size_t)g.cv0[k], src = 3 * (size_t)old.cv0[r.old_slots[k]];
    const size_t nb = 3 * (size_t)r.cs[k]->n * sizeof(double);
    e = hipMemcpyAsync(g.xs + dst, old.xs + src, nb, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(g.vs + dst, old.vs + src, nb, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && g.fx)
      e = hipMemcpyAsync(g.fx + dst, old.fx + src, nb, hipMemcpyDeviceToDevice, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    err = std::string("state copy failed: ") + hipGetErrorString(e);
    return QNSIM_E_DEVICE;
  }
  return QNSIM_OK;
}

// The group's force array (zeroed) on first use; called with the pool lock held.
int ensure_force_array(qnsim_pool* p, PoolGroup& g, std::string& err) {
  if (g.fx) return QNSIM_OK;
  const size_t all = 3 * (size_t)g.D.n * sizeof(double);
  if (hipMalloc((void**)&g.fx, all) != hipSuccess) {
    g.fx = nullptr;
    err = "force allocation failed";
    return QNSIM_E_NOMEM;
  }
  if (hipMemsetAsync(g.fx, 0, all, (hipStream_t)g.D.stream) != hipSuccess) {
    err = "force clear failed";
    return QNSIM_E_DEVICE;
  }
  g.bytes += (int64_t)all;
  p->used += (int64_t)all;
  return QNSIM_OK;
}

// Writes the force of member `slot` (caller order; null: zero) into the
// group's force array, on the group's stream.
int write_force(PoolGroup& g, int slot, int n, const double* f, std::string& err) {
  double* dst = g.fx + 3 * (size_t)g.cv0[slot];
  const size_t bytes = 3 * (size_t)n * sizeof(double);
  hipStream_t st = (hipStream_t)g.D.stream;
  const hipError_t e = f ? hipMemcpyAsync(dst, f, bytes, hipMemcpyHostToDevice, st)
                         : hipMemsetAsync(dst, 0, bytes, st);
  if (e != hipSuccess) { err = hipGetErrorString(e); return QNSIM_E_DEVICE; }
  return QNSIM_OK;
}

// One batched step of the listed members of group g (slots), on its stream.
// Called without the pool lock; the group is marked busy by the caller.
int step_group(qnsim_pool* p, PoolGroup& g, const std::vector<int>& slots,
               std::vector<SimStat>& st, std::string& err) {
  if (hipSetDevice(p->opt.device) != hipSuccess) { err = "hipSetDevice failed"; return QNSIM_E_DEVICE; }
  std::vector<int> run(g.D.S, 0);
  for (int s : slots) run[s] = 1;
  int rc = dev_set_run(g.D, run.data(), g.D.stream, err);
  if (rc) return rc;
  StepParams prm = pool_params(p);
  if (g.trials > 0) prm.budget = g.trials;
  rc = dev_step(g.D, prm, g.xs, g.vs, g.fx, g.xs, g.vs, g.D.stream, false, err);
  if (rc) return rc;
  st.resize(slots.size());
  for (size_t i = 0; i < slots.size(); ++i) st[i] = g.D.stat_host[slots[i]];
  return QNSIM_OK;
}

int resident(const qnsim_pool* p, int id) {
  return id >= 0 && id < (int)p->sims.size() && !p->sims[id].removed && p->sims[id].group >= 0;
}

// Request loop of one lane.
void lane_main(qnsim_pool* p) {
  (void)hipSetDevice(p->opt.device);
  std::unique_lock<std::mutex> lk(p->mu);
  for (;;) {
    // the group of the oldest queued request that is not stepping
    int gi = -1;
    for (const Request& r : p->queue) {
      const int g = p->sims[r.sim].group;
      if (g >= 0 && !p->groups[g]->busy) { gi = g; break; }
    }
    if (gi < 0) {
      if (p->stopping && p->queue.empty()) return;
      p->cv.wait(lk);
      continue;
    }
    PoolGroup& g = *p->groups[gi];
    std::vector<Request> batch;
    std::vector<int> slots;
    std::vector<char> taken(g.ids.size(), 0);
    for (auto it = p->queue.begin(); it != p->queue.end();) {
      const int sim = it->sim;
      if (p->sims[sim].group == gi && !taken[p->sims[sim].slot]) {
        taken[p->sims[sim].slot] = 1;
        slots.push_back(p->sims[sim].slot);
        batch.push_back(*it);
        it = p->queue.erase(it);
      } else {
        ++it;
      }
    }
    // requests with their own force: the group's force array takes it for
    // this step, and the simulation's own force (or zero) afterwards
    // (copied under the lock: the pool's tables may grow while it steps)
    struct OwnForce {
      int slot, n;
      std::shared_ptr<const std::vector<double>> req;
      std::vector<double> keep;  // the simulation's own force; empty: none
    };
    std::vector<OwnForce> own;
    for (const Request& r : batch)
      if (r.force) {
        const PoolSim& s = p->sims[r.sim];
        own.push_back(OwnForce{s.slot, s.c->n, r.force, s.has_force ? s.force : std::vector<double>()});
      }
    std::string err;
    int rc = own.empty() ? QNSIM_OK : ensure_force_array(p, g, err);
    g.busy = true;
    lk.unlock();
    std::vector<SimStat> st;
    for (size_t k = 0; k < own.size() && !rc; ++k)
      rc = write_force(g, own[k].slot, own[k].n, own[k].req->data(), err);
    if (!rc) rc = step_group(p, g, slots, st, err);
    for (size_t k = 0; k < own.size() && g.fx; ++k) {
      std::string e2;
      const int r2 = write_force(g, own[k].slot, own[k].n,
                                 own[k].keep.empty() ? nullptr : own[k].keep.data(), e2);
      if (r2 && !rc) { rc = r2; err = e2; }
    }
    if (!own.empty() && g.fx && hipStreamSynchronize((hipStream_t)g.D.stream) != hipSuccess && !rc) {
      rc = QNSIM_E_DEVICE;
      err = "force restore failed";
    }
    const double t_end = now_s();
    lk.lock();
    g.busy = false;
    for (size_t i = 0; i < batch.size(); ++i) {
      Done d;
      d.rc = rc;
      std::memset(&d.st, 0, sizeof(d.st));
      if (!rc) stats_of(st[i], &d.st);
      d.latency = t_end - batch[i].t_submit;
      p->done[batch[i].ticket] = d;
    }
    if (rc) p->last_error = err;
    else { p->steps_done += (int64_t)batch.size(); p->batches_done += 1; }
    p->cv.notify_all();
  }
}

}  // namespace

extern "C" {

int qnsim_pool_create(const qnsim_options* opts, double h, int64_t budget_bytes,
                      qnsim_pool_t** out) {
  if (!out || !(h > 0.0) || !std::isfinite(h) || budget_bytes <= 0) return QNSIM_E_INVALID;
  qnsim_options o;
  if (opts) o = *opts;
  else qnsim_options_default(&o);
  // a level launch of a group serves every simulation in it, so merging
  // levels (or a dense top block) would only add bytes
  o.dense_top = 0;
  o.level_merge = 0;
  o.device_factor = 0;
  qnsim_t* probe = nullptr;  // option validation as for a single context
  int rc = qnsim_create(&o, &probe);
  if (rc) return rc;
  qnsim_destroy(probe);
  qnsim_pool* p = new (std::nothrow) qnsim_pool();
  if (!p) return QNSIM_E_NOMEM;
  p->opt = o;
  p->h = h;
  p->budget = budget_bytes;
  *out = p;
  return QNSIM_OK;
}

void qnsim_pool_destroy(qnsim_pool_t* p) {
  if (!p) return;
  qnsim_pool_serve_stop(p);
  for (auto& g : p->groups)
    if (g) free_group(*g);
  for (PoolSim& s : p->sims)
    if (s.c) qnsim_destroy(s.c);
  delete p;
}

int qnsim_pool_add(qnsim_pool_t* p, int32_t n, const qnsim_mesh_desc* descs, int32_t* ids) {
  if (!p) return QNSIM_E_INVALID;
  if (n <= 0 || !descs || !ids) return pfail(p, QNSIM_E_INVALID, "need n > 0 descriptions and ids");
  std::vector<PoolSim> made(n);
  std::vector<int> rcs(n, 0);
  std::vector<std::string> errs(n);
  {
    // host analysis in parallel; the dense kernels inside share one thread pool
    const int nt = std::max(1, std::min<int>(n, std::min(16, (int)std::thread::hardware_concurrency())));
    std::vector<std::thread> th;
    std::mutex qm;
    int next = 0;
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&]() {
        for (;;) {
          int i;
          {
            std::lock_guard<std::mutex> g(qm);
            i = next++;
          }
          if (i >= n) return;
          try {
            rcs[i] = analyze_one(p, descs[i], made[i], errs[i]);
          } catch (const std::bad_alloc&) {
            rcs[i] = QNSIM_E_NOMEM;
            errs[i] = "host allocation failed";
          }
        }
      });
    for (auto& t : th) t.join();
  }
  for (int i = 0; i < n; ++i)
    if (rcs[i]) {
      for (PoolSim& s : made)
        if (s.c) qnsim_destroy(s.c);
      return pfail(p, rcs[i], "simulation " + std::to_string(i) + ": " + errs[i]);
    }
  std::lock_guard<std::mutex> lk(p->mu);
  for (int i = 0; i < n; ++i) {
    ids[i] = (int)p->sims.size();
    p->sims.push_back(std::move(made[i]));
  }
  return QNSIM_OK;
}

int qnsim_pool_commit(qnsim_pool_t* p, int32_t max_group_sims, int32_t* n_admitted) {
  if (!p) return QNSIM_E_INVALID;
  if (n_admitted) *n_admitted = 0;
  std::unique_lock<std::mutex> lk(p->mu);
  p->cv.wait(lk, [&] { return !p->admin_busy; });
  // 1. plan under the lock. Groups whose removed members hold at least half
  //    of their memory are repacked (rebuilt with the live members while
  //    the old group keeps serving them); the memory that frees counts for
  //    the admission. Then staged simulations in id order while the budget
  //    allows, max_group_sims per group.
  std::vector<Repack> repacks;
  std::vector<int> repack_tile;
  int64_t freed = 0;
  for (int gi = 0; gi < (int)p->groups.size(); ++gi) {
    PoolGroup& g = *p->groups[gi];
    if (g.live == 0 || g.live == (int)g.ids.size() || g.repacking) continue;
    int64_t dead = 0, all = 0;
    for (int id : g.ids) {
      all += p->sims[id].est_bytes;
      if (p->sims[id].removed) dead += p->sims[id].est_bytes;
    }
    if (2 * dead < all) continue;
    Repack r;
    r.gi = gi;
    for (size_t k = 0; k < g.ids.size(); ++k) {
      const PoolSim& m = p->sims[g.ids[k]];
      if (m.removed) continue;
      r.ids.push_back(g.ids[k]);
      r.old_slots.push_back((int)k);
      r.cs.push_back(m.c);
      r.refactored = r.refactored || m.c->factor_on_device;
    }
    g.repacking = true;
    freed += dead;
    repack_tile.push_back(g.D.elem_tile);
    repacks.push_back(std::move(r));
  }
  std::vector<std::vector<int>> plan;
  std::vector<int> cur;
  int64_t room = p->budget - p->used + freed;
  for (int id = 0; id < (int)p->sims.size(); ++id) {
    const PoolSim& s = p->sims[id];
    if (s.removed || s.group >= 0 || s.admitting) continue;
    if (s.est_bytes > room) continue;  // stays staged
    room -= s.est_bytes;
    cur.push_back(id);
    if (max_group_sims > 0 && (int)cur.size() >= max_group_sims) {
      plan.push_back(cur);
      cur.clear();
    }
  }
  if (!cur.empty()) plan.push_back(cur);
  if (plan.empty() && repacks.empty()) return QNSIM_OK;
  std::vector<GroupBuild> builds(plan.size());
  for (size_t b = 0; b < plan.size(); ++b) {
    builds[b].ids = plan[b];
    for (int id : plan[b]) {
      PoolSim& s = p->sims[id];
      s.admitting = true;
      builds[b].cs.push_back(s.c);
      builds[b].x0.push_back(std::move(s.x0));
      builds[b].v0.push_back(std::move(s.v0));
    }
  }
  p->admin_busy = true;
  const qnsim_options opt = p->opt;
  const double h = p->h;
  lk.unlock();
  // 2. build and upload outside the lock: serving lanes keep picking and
  //    stepping resident groups (those being repacked included) meanwhile;
  //    repacks first, and they replace their old groups (whose memory is
  //    freed) before the new groups allocate
  int rc = QNSIM_OK;
  std::string err;
  for (size_t k = 0; k < repacks.size(); ++k) {
    Repack& r = repacks[k];
    try {
      r.rc = build_repack(opt, h, repack_tile[k], r);
    } catch (const std::bad_alloc&) {
      r.rc = QNSIM_E_NOMEM;
      r.err = "host allocation failed";
    }
  }
  if (!repacks.empty()) {
    std::vector<std::unique_ptr<PoolGroup>> dead;
    lk.lock();
    for (Repack& r : repacks) {
      p->cv.wait(lk, [&] { return !p->groups[r.gi]->busy; });
      PoolGroup& old = *p->groups[r.gi];
      old.repacking = false;
      if (!r.rc && old.live > 0) r.rc = repack_states(old, *r.g, r, r.err);
      if (r.rc || old.live == 0) {
        if (r.g) free_group(*r.g);
        if (r.rc) {  // the old group stays as it was
          if (!rc) { rc = r.rc; err = "repack: " + r.err; }
          continue;
        }
        // every member was removed while the group was rebuilt
        p->used -= old.bytes;
        free_group(old);
        for (int id : old.ids)
          if (p->sims[id].c) { qnsim_destroy(p->sims[id].c); p->sims[id].c = nullptr; }
        continue;
      }
      r.g->live = old.live;
      r.g->trials = old.trials;
      p->used += r.g->bytes - old.bytes;
      std::vector<char> kept(p->sims.size(), 0);
      for (int id : r.ids) kept[id] = 1;
      for (int id : old.ids) {  // members removed before the repack leave for good
        PoolSim& m = p->sims[id];
        if (!kept[id] && m.c) { qnsim_destroy(m.c); m.c = nullptr; }
      }
      for (size_t k = 0; k < r.ids.size(); ++k) p->sims[r.ids[k]].slot = (int)k;
      dead.push_back(std::move(p->groups[r.gi]));
      p->groups[r.gi] = std::move(r.g);
    }
    p->cv.notify_all();
    lk.unlock();
    for (auto& g : dead) free_group(*g);  // no lane holds a replaced group
  }
  bool failed = false;
  for (GroupBuild& b : builds) {
    if (failed) { b.rc = QNSIM_E_STATE; continue; }
    try {
      b.rc = build_group(opt, h, b);
    } catch (const std::bad_alloc&) {
      b.rc = QNSIM_E_NOMEM;
      b.err = "host allocation failed";
    }
    failed = b.rc != QNSIM_OK;
  }
  // 3. publish the new groups under the lock
  lk.lock();
  int admitted = 0;
  for (GroupBuild& b : builds) {
    if (b.rc) {
      // not admitted: the simulations stay staged with their initial state
      for (size_t k = 0; k < b.ids.size(); ++k) {
        PoolSim& s = p->sims[b.ids[k]];
        s.admitting = false;
        s.x0 = std::move(b.x0[k]);
        s.v0 = std::move(b.v0[k]);
        if (s.removed && s.c) { qnsim_destroy(s.c); s.c = nullptr; }
      }
      if (!rc && b.rc != QNSIM_E_STATE) { rc = b.rc; err = b.err; }
      continue;
    }
    const int gi = (int)p->groups.size();
    for (size_t k = 0; k < b.ids.size(); ++k) {
      PoolSim& s = p->sims[b.ids[k]];
      s.admitting = false;
      s.group = gi;
      s.slot = (int)k;
      if (s.removed) b.g->live--;  // removed while its group was built
    }
    p->used += b.g->bytes;
    admitted += b.g->live;
    p->groups.push_back(std::move(b.g));
    if (p->groups.back()->live == 0) {  // every member removed meanwhile
      p->used -= p->groups.back()->bytes;
      free_group(*p->groups.back());
      for (int id : b.ids)
        if (p->sims[id].c) { qnsim_destroy(p->sims[id].c); p->sims[id].c = nullptr; }
    }
  }
  p->admin_busy = false;
  if (n_admitted) *n_admitted = admitted;
  p->cv.notify_all();
  return rc ? pfail(p, rc, err) : QNSIM_OK;
}

int qnsim_pool_remove(qnsim_pool_t* p, int32_t id) {
  if (!p) return QNSIM_E_INVALID;
  std::unique_lock<std::mutex> lk(p->mu);
  if (id < 0 || id >= (int)p->sims.size() || p->sims[id].removed)
    return pfail(p, QNSIM_E_INVALID, "unknown simulation id");
  PoolSim& s = p->sims[id];
  for (const Request& r : p->queue)
    if (r.sim == id) return pfail(p, QNSIM_E_STATE, "simulation has queued requests");
  s.removed = true;
  if (s.admitting) return QNSIM_OK;  // the commit building its group drops it
  if (s.group >= 0) {
    // the group is looked up again after the wait: a repack may replace it
    // and a concurrent add may move the simulation records
    p->cv.wait(lk, [&] { return !p->groups[p->sims[id].group]->busy; });
    PoolGroup& g = *p->groups[p->sims[id].group];
    // a group being repacked is freed by the commit once its build is done
    // (the build reads the members' host data)
    if (--g.live == 0 && !g.repacking) {
      p->used -= g.bytes;
      free_group(g);
      // the members' host data served the group's refactorisation
      for (int id2 : g.ids)
        if (p->sims[id2].removed && p->sims[id2].c) {
          qnsim_destroy(p->sims[id2].c);
          p->sims[id2].c = nullptr;
        }
    }
    return QNSIM_OK;  // a member's host data stays while its group is resident
  }
  if (s.c) { qnsim_destroy(s.c); s.c = nullptr; }
  return QNSIM_OK;
}

int qnsim_pool_step(qnsim_pool_t* p, int32_t n, const int32_t* ids, qnsim_stats* stats) {
  if (!p) return QNSIM_E_INVALID;
  if (n < 0 || (n > 0 && !ids)) return pfail(p, QNSIM_E_INVALID, "bad id list");
  std::unique_lock<std::mutex> lk(p->mu);
  if (p->serving) return pfail(p, QNSIM_E_STATE, "the request loop is running");
  // wait until no listed simulation's group is stepping or being repacked
  p->cv.wait(lk, [&] {
    for (int i = 0; i < n; ++i)
      if (resident(p, ids[i]) && p->groups[p->sims[ids[i]].group]->busy) return false;
    return true;
  });
  std::vector<std::vector<int>> slots(p->groups.size());
  std::vector<std::vector<int>> where(p->groups.size());  // index into ids
  std::vector<char> seen(p->sims.size(), 0);
  for (int i = 0; i < n; ++i) {
    if (!resident(p, ids[i])) return pfail(p, QNSIM_E_INVALID, "id " + std::to_string(ids[i]) + " is not resident");
    if (seen[ids[i]]++) return pfail(p, QNSIM_E_INVALID, "repeated id");
    const PoolSim& s = p->sims[ids[i]];
    slots[s.group].push_back(s.slot);
    where[s.group].push_back(i);
  }
  // The groups are taken by pointer while the lock is held: a concurrent
  // commit may grow p->groups (moving its elements, not the groups).
  std::vector<int> gl;
  std::vector<PoolGroup*> gp;
  for (int g = 0; g < (int)p->groups.size(); ++g)
    if (!slots[g].empty()) {
      gl.push_back(g);
      gp.push_back(p->groups[g].get());
      gp.back()->busy = true;
    }
  lk.unlock();
  std::vector<int> rcs(gl.size(), 0);
  std::vector<std::string> errs(gl.size());
  std::vector<std::vector<SimStat>> st(gl.size());
  if (gl.size() == 1) {
    rcs[0] = step_group(p, *gp[0], slots[gl[0]], st[0], errs[0]);
  } else {
    std::vector<std::thread> th;
    for (size_t k = 0; k < gl.size(); ++k)
      th.emplace_back([&, k]() { rcs[k] = step_group(p, *gp[k], slots[gl[k]], st[k], errs[k]); });
    for (auto& t : th) t.join();
  }
  lk.lock();
  int rc = 0;
  for (size_t k = 0; k < gl.size(); ++k) {
    gp[k]->busy = false;
    if (rcs[k] && !rc) { rc = rcs[k]; p->last_error = errs[k]; }
    if (!rcs[k] && stats)
      for (size_t j = 0; j < where[gl[k]].size(); ++j) stats_of(st[k][j], &stats[where[gl[k]][j]]);
  }
  if (!rc) { p->steps_done += n; p->batches_done += (int64_t)gl.size(); }
  p->cv.notify_all();
  return rc;
}

static int state_copy(qnsim_pool* p, int id, double* xh, double* vh, const double* xin,
                      const double* vin) {
  std::unique_lock<std::mutex> lk(p->mu);
  if (!resident(p, id)) return pfail(p, QNSIM_E_INVALID, "id is not resident");
  p->cv.wait(lk, [&] { return !resident(p, id) || !p->groups[p->sims[id].group]->busy; });
  if (!resident(p, id)) return pfail(p, QNSIM_E_INVALID, "id was removed");
  const PoolSim& s = p->sims[id];
  PoolGroup& g = *p->groups[s.group];
  const size_t off = 3 * (size_t)g.cv0[s.slot], bytes = 3 * (size_t)s.c->n * sizeof(double);
  hipStream_t st = (hipStream_t)g.D.stream;
  hipError_t e = hipSuccess;
  if (xin) {
    e = hipMemcpyAsync(g.xs + off, xin, bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(g.vs + off, vin, bytes, hipMemcpyHostToDevice, st);
  } else {
    e = hipMemcpyAsync(xh, g.xs + off, bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(vh, g.vs + off, bytes, hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return pfail(p, QNSIM_E_DEVICE, hipGetErrorString(e));
  return QNSIM_OK;
}

int qnsim_pool_get_state(qnsim_pool_t* p, int32_t id, double* x, double* v) {
  if (!p || !x || !v) return QNSIM_E_INVALID;
  return state_copy(p, id, x, v, nullptr, nullptr);
}

int qnsim_pool_set_state(qnsim_pool_t* p, int32_t id, const double* x, const double* v) {
  if (!p || !x || !v) return QNSIM_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!resident(p, id)) return pfail(p, QNSIM_E_INVALID, "id is not resident");
    const size_t n3 = 3 * (size_t)p->sims[id].c->n;
    for (size_t i = 0; i < n3; ++i)
      if (!std::isfinite(x[i]) || !std::isfinite(v[i])) return pfail(p, QNSIM_E_NONFINITE, "non-finite state");
  }
  return state_copy(p, id, nullptr, nullptr, x, v);
}

int qnsim_pool_set_force(qnsim_pool_t* p, int32_t id, const double* f_ext) {
  if (!p) return QNSIM_E_INVALID;
  std::unique_lock<std::mutex> lk(p->mu);
  if (!resident(p, id)) return pfail(p, QNSIM_E_INVALID, "id is not resident");
  PoolSim& s = p->sims[id];
  const size_t n3 = 3 * (size_t)s.c->n;
  if (f_ext)
    for (size_t i = 0; i < n3; ++i)
      if (!std::isfinite(f_ext[i])) return pfail(p, QNSIM_E_NONFINITE, "non-finite force");
  p->cv.wait(lk, [&] { return !resident(p, id) || !p->groups[p->sims[id].group]->busy; });
  if (!resident(p, id)) return pfail(p, QNSIM_E_INVALID, "id was removed");
  PoolSim& s2 = p->sims[id];  // records may have moved during the wait
  PoolGroup& g = *p->groups[s2.group];
  if (!f_ext && !s2.has_force) return QNSIM_OK;
  if (hipSetDevice(p->opt.device) != hipSuccess) return pfail(p, QNSIM_E_DEVICE, "hipSetDevice failed");
  std::string err;
  int rc = ensure_force_array(p, g, err);
  if (!rc) rc = write_force(g, s2.slot, s2.c->n, f_ext, err);
  if (!rc && hipStreamSynchronize((hipStream_t)g.D.stream) != hipSuccess) {
    rc = QNSIM_E_DEVICE;
    err = "force copy failed";
  }
  if (rc) return pfail(p, rc, err);
  s2.has_force = f_ext != nullptr;
  if (f_ext) s2.force.assign(f_ext, f_ext + n3);
  else std::vector<double>().swap(s2.force);
  return QNSIM_OK;
}

int qnsim_pool_serve_start(qnsim_pool_t* p, int32_t lanes) {
  if (!p) return QNSIM_E_INVALID;
  if (lanes < 1 || lanes > 8) return pfail(p, QNSIM_E_INVALID, "lanes must be 1..8");
  std::lock_guard<std::mutex> lk(p->mu);
  if (p->serving) return pfail(p, QNSIM_E_STATE, "the request loop is already running");
  for (auto& g : p->groups)
    if (g->busy) return pfail(p, QNSIM_E_STATE, "a step is running");
  p->serving = true;
  p->stopping = false;
  for (int i = 0; i < lanes; ++i) p->lanes.emplace_back(lane_main, p);
  return QNSIM_OK;
}

int qnsim_pool_submit(qnsim_pool_t* p, int32_t id, int64_t* ticket) {
  if (!p || !ticket) return QNSIM_E_INVALID;
  std::lock_guard<std::mutex> lk(p->mu);
  if (!p->serving || p->stopping) return pfail(p, QNSIM_E_STATE, "the request loop is not running");
  if (!resident(p, id)) return pfail(p, QNSIM_E_INVALID, "id is not resident");
  const int64_t t = p->next_ticket++;
  p->queue.push_back(Request{t, id, now_s(), nullptr});
  *ticket = t;
  p->cv.notify_all();
  return QNSIM_OK;
}

int qnsim_pool_submit_force(qnsim_pool_t* p, int32_t id, const double* f_ext, int64_t* ticket) {
  if (!p || !ticket) return QNSIM_E_INVALID;
  std::shared_ptr<std::vector<double>> f;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!resident(p, id)) return pfail(p, QNSIM_E_INVALID, "id is not resident");
    if (f_ext) {
      const size_t n3 = 3 * (size_t)p->sims[id].c->n;
      for (size_t i = 0; i < n3; ++i)
        if (!std::isfinite(f_ext[i])) return pfail(p, QNSIM_E_NONFINITE, "non-finite force");
      f = std::make_shared<std::vector<double>>(f_ext, f_ext + n3);
    }
  }
  std::lock_guard<std::mutex> lk(p->mu);
  if (!p->serving || p->stopping) return pfail(p, QNSIM_E_STATE, "the request loop is not running");
  if (!resident(p, id)) return pfail(p, QNSIM_E_INVALID, "id is not resident");
  const int64_t t = p->next_ticket++;
  p->queue.push_back(Request{t, id, now_s(), f});
  *ticket = t;
  p->cv.notify_all();
  return QNSIM_OK;
}

int qnsim_pool_wait(qnsim_pool_t* p, int64_t ticket, double timeout_s, qnsim_stats* stats,
                    double* latency_s) {
  if (!p) return QNSIM_E_INVALID;
  std::unique_lock<std::mutex> lk(p->mu);
  if (ticket <= 0 || ticket >= p->next_ticket) return pfail(p, QNSIM_E_STATE, "unknown ticket");
  auto ready = [&] { return p->done.count(ticket) > 0; };
  if (timeout_s < 0) {
    p->cv.wait(lk, [&] { return ready() || (!p->serving && p->queue.empty()); });
  } else {
    p->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
  }
  auto it = p->done.find(ticket);
  if (it == p->done.end()) return pfail(p, QNSIM_E_STATE, "request not done (time-out or unknown ticket)");
  const Done d = it->second;
  p->done.erase(it);
  if (d.rc) return d.rc;
  if (stats) *stats = d.st;
  if (latency_s) *latency_s = d.latency;
  return QNSIM_OK;
}

int qnsim_pool_serve_stop(qnsim_pool_t* p) {
  if (!p) return QNSIM_E_INVALID;
  std::vector<std::thread> lanes;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->serving) return QNSIM_OK;
    p->stopping = true;
    lanes.swap(p->lanes);
    p->cv.notify_all();
  }
  for (auto& t : lanes) t.join();
  std::lock_guard<std::mutex> lk(p->mu);
  p->serving = false;
  p->stopping = false;
  p->cv.notify_all();
  return QNSIM_OK;
}

int qnsim_pool_status(qnsim_pool_t* p, int32_t id, int32_t* status, int32_t* group) {
  if (!p || !status) return QNSIM_E_INVALID;
  std::lock_guard<std::mutex> lk(p->mu);
  if (id < 0 || id >= (int)p->sims.size()) return pfail(p, QNSIM_E_INVALID, "unknown simulation id");
  const PoolSim& s = p->sims[id];
  *status = s.removed ? QNSIM_SIM_REMOVED : s.group >= 0 ? QNSIM_SIM_RESIDENT : QNSIM_SIM_STAGED;
  if (group) *group = s.removed ? -1 : s.group;
  return QNSIM_OK;
}

int qnsim_pool_get_info(qnsim_pool_t* p, qnsim_pool_info* info) {
  if (!p || !info) return QNSIM_E_INVALID;
  std::lock_guard<std::mutex> lk(p->mu);
  std::memset(info, 0, sizeof(*info));
  for (const PoolSim& s : p->sims) {
    if (s.removed) continue;
    if (s.group >= 0) {
      info->sims_resident++;
      info->nnz_L += s.c->factor.nnz_exact;
      info->n_free += s.c->nf;
      info->n_tets += s.c->T;
    } else {
      info->sims_staged++;
    }
  }
  for (auto& g : p->groups)
    if (g->live > 0) info->groups++;
  info->groups_made = (int32_t)p->groups.size();
  info->serving = p->serving ? 1 : 0;
  info->budget_bytes = p->budget;
  info->used_bytes = p->used;
  info->steps_done = p->steps_done;
  info->batches_done = p->batches_done;
  return QNSIM_OK;
}

int qnsim_pool_set_h(qnsim_pool_t* p, double h, double* device_ms) {
  if (!p) return QNSIM_E_INVALID;
  if (!(h > 0.0) || !std::isfinite(h)) return pfail(p, QNSIM_E_INVALID, "h must be positive");
  std::unique_lock<std::mutex> lk(p->mu);
  if (p->serving) return pfail(p, QNSIM_E_STATE, "the request loop is running");
  p->cv.wait(lk, [&] {
    if (p->admin_busy) return false;
    for (auto& g : p->groups)
      if (g && g->busy) return false;
    return true;
  });
  const double h_old = p->h;
  double total = 0.0;
  std::string err;
  // resident groups: A refactored on the device, group by group; on a
  // failure the groups already done go back to the previous h
  std::vector<int> done;
  for (int gi = 0; gi < (int)p->groups.size(); ++gi) {
    PoolGroup& g = *p->groups[gi];
    if (g.live == 0) continue;
    std::vector<const qnsim*> members;
    for (int id : g.ids) members.push_back(p->sims[id].c);
    double ms = 0.0;
    int rc = dev_refactor_mesh(members, g.D, h, &ms, err);
    if (rc) {
      for (int gj : done) {
        PoolGroup& g2 = *p->groups[gj];
        std::vector<const qnsim*> m2;
        for (int id : g2.ids) m2.push_back(p->sims[id].c);
        std::string e2;
        (void)dev_refactor_mesh(m2, g2.D, h_old, nullptr, e2);
      }
      return pfail(p, rc, err);
    }
    total += ms;
    done.push_back(gi);
  }
  // staged simulations: host analysis for the new h
  for (PoolSim& s : p->sims)
    if (!s.removed && s.group < 0 && s.c) {
      int rc = qnsim_analyze(s.c, h);
      if (rc) return pfail(p, rc, std::string("staged simulation: ") + qnsim_last_error(s.c));
    }
  for (PoolSim& s : p->sims)
    if (s.c && s.group >= 0) {
      s.c->h = h;
      s.c->factor_on_device = true;  // the host factor values belong to the old h
    }
  p->h = h;
  if (device_ms) *device_ms = total;
  return QNSIM_OK;
}

int qnsim_pool_tune(qnsim_pool_t* p, int32_t candidates, int32_t reps, int32_t n_groups,
                    int32_t* tiles, double* step_ms, int32_t* trials, double* trials_ms) {
  if (!p) return QNSIM_E_INVALID;
  if (candidates == 0) candidates = 7;
  if (candidates < 0 || candidates > 7)
    return pfail(p, QNSIM_E_INVALID, "candidates: a mask of bits 1 (128), 2 (256), 4 (512)");
  if (reps < 1 || reps > 1000 || n_groups < 0 || (n_groups > 0 && !tiles))
    return pfail(p, QNSIM_E_INVALID, "reps must be 1..1000 and tiles given for n_groups > 0");
  std::unique_lock<std::mutex> lk(p->mu);
  if (p->serving) return pfail(p, QNSIM_E_STATE, "the request loop is running");
  p->cv.wait(lk, [&] {
    if (p->admin_busy) return false;
    for (auto& g : p->groups)
      if (g && g->busy) return false;
    return true;
  });
  for (int gi = 0; gi < n_groups; ++gi) {
    tiles[gi] = 0;
    if (trials) trials[gi] = 0;
    for (int k = 0; k < 3; ++k) {
      if (step_ms) step_ms[3 * gi + k] = NAN;
      if (trials_ms) trials_ms[3 * gi + k] = NAN;
    }
  }
  std::string err;
  for (int gi = 0; gi < (int)p->groups.size(); ++gi) {
    PoolGroup& g = *p->groups[gi];
    if (g.live == 0) continue;
    if (hipSetDevice(p->opt.device) != hipSuccess) return pfail(p, QNSIM_E_DEVICE, "hipSetDevice failed");
    std::vector<const qnsim*> members;
    bool refactored = false;
    for (int id : g.ids) {
      members.push_back(p->sims[id].c);
      refactored = refactored || p->sims[id].c->factor_on_device;
    }
    // the steps being timed run on a copy of the members' states
    const size_t bytes = 3 * (size_t)g.D.n * sizeof(double);
    double *tx = nullptr, *tvl = nullptr;
    if (hipMalloc((void**)&tx, bytes) != hipSuccess || hipMalloc((void**)&tvl, bytes) != hipSuccess) {
      if (tx) (void)hipFree(tx);
      return pfail(p, QNSIM_E_NOMEM, "tuning state allocation failed");
    }
    StepParams prm = pool_params(p);
    if (g.trials > 0) prm.budget = g.trials;
    // ms per batched step of all members on mesh D from the members' states
    auto timed = [&](DeviceMesh& D, const StepParams& P, double* ms) -> int {
      hipStream_t st = (hipStream_t)D.stream;
      std::vector<int> all(D.S, 1);
      int r = dev_set_run(D, all.data(), D.stream, err);
      if (!r && (hipMemcpyAsync(tx, g.xs, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                 hipMemcpyAsync(tvl, g.vs, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)) {
        err = "tuning state copy failed";
        r = QNSIM_E_DEVICE;
      }
      // one untimed step (graph capture), then reps timed steps
      if (!r) r = dev_step(D, P, tx, tvl, nullptr, tx, tvl, D.stream, false, err);
      const double t0 = now_s();
      for (int k = 0; k < reps && !r; ++k)
        r = dev_step(D, P, tx, tvl, nullptr, tx, tvl, D.stream, false, err);
      *ms = (now_s() - t0) * 1e3 / reps;
      return r;
    };
    DeviceMesh spare, cand;  // the fastest rebuilt mesh so far, the one being timed
    int best_tile = g.D.elem_tile;
    double best_ms = INFINITY;
    int rc = QNSIM_OK;
    for (int k = 0; k < 3 && !rc; ++k) {
      if (!(candidates & (1 << k))) continue;
      const int tile = kElemTiles[k];
      DeviceMesh* D = &g.D;
      if (tile != g.D.elem_tile) {
        qnsim_options o = p->opt;
        o.elem_tile = tile;
        rc = upload_sims(members, o, p->h, cand, err);
        // host factor values belong to an earlier h after a time-step change
        if (!rc && refactored) rc = dev_refactor_mesh(members, cand, p->h, nullptr, err);
        if (rc) break;
        D = &cand;
      }
      double ms = 0.0;
      rc = timed(*D, prm, &ms);
      if (rc) break;
      if (step_ms && gi < n_groups) step_ms[3 * gi + k] = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best_tile = tile;
        if (D == &cand) std::swap(spare, cand);
      }
      dev_free(cand);
    }
    if (!rc && best_tile != g.D.elem_tile) {
      const int64_t old = (int64_t)g.D.bytes;
      std::swap(g.D, spare);
      p->used += (int64_t)g.D.bytes - old;
      g.bytes += (int64_t)g.D.bytes - old;
    }
    dev_free(cand);
    dev_free(spare);
    // then the line-search trials per cycle with the kept tile
    if (!rc && trials) {
      int best_b = prm.budget;
      best_ms = INFINITY;
      for (int b = 1; b <= 3 && !rc; ++b) {
        StepParams pb = prm;
        pb.budget = b;
        double ms = 0.0;
        rc = timed(g.D, pb, &ms);
        if (!rc && trials_ms && gi < n_groups) trials_ms[3 * gi + b - 1] = ms;
        if (!rc && ms < best_ms) { best_ms = ms; best_b = b; }
      }
      if (!rc) g.trials = best_b;
    }
    (void)hipFree(tx);
    (void)hipFree(tvl);
    if (rc) return pfail(p, rc, err);
    if (gi < n_groups) {
      tiles[gi] = g.D.elem_tile;
      if (trials) trials[gi] = g.trials > 0 ? g.trials : p->opt.trials_per_cycle;
    }
  }
  return QNSIM_OK;
}

int qnsim_pool_time_kernel(qnsim_pool_t* p, int32_t group, int32_t kernel, int32_t reps,
                           double* avg_ms) {
  if (!p || !avg_ms || reps < 1 || kernel < QNSIM_KERNEL_ELEMENT || kernel > QNSIM_KERNEL_SOLVE)
    return QNSIM_E_INVALID;
  std::unique_lock<std::mutex> lk(p->mu);
  if (p->serving) return pfail(p, QNSIM_E_STATE, "the request loop is running");
  if (group < 0 || group >= (int)p->groups.size() || p->groups[group]->live == 0)
    return pfail(p, QNSIM_E_INVALID, "no such group");
  PoolGroup& g = *p->groups[group];
  if (g.busy) return pfail(p, QNSIM_E_STATE, "the group is stepping");
  g.busy = true;
  lk.unlock();
  std::string err;
  std::vector<int> all(g.D.S, 1);
  int rc = dev_set_run(g.D, all.data(), g.D.stream, err);
  if (!rc) rc = dev_time_kernel(g.D, kernel, reps, avg_ms, err);
  lk.lock();
  g.busy = false;
  p->cv.notify_all();
  return rc ? pfail(p, rc, err) : QNSIM_OK;
}

const char* qnsim_pool_last_error(const qnsim_pool_t* p) { return p ? p->last_error.c_str() : ""; }

}  // extern "C"
