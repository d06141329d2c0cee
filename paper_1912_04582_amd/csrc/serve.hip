// Serving: continuous batching of independent solves on one device.
//
// Requests that share N, precision and whether their mesh has faces off the
// coordinate axes (which selects the expansion kernels) are the instances of
// one batched state (a cohort), so a step of a cohort is one set of launches
// over the cells of all its requests.  A worker thread
//   1. admits queued requests, in arrival order among those that fit,
//      whenever their estimated device memory fits what the running cohorts
//      leave of the budget (a request that could never fit is refused at
//      submit).  Admitted requests join the cohort of their kind at its next
//      step boundary: the cohort is rebuilt with its running requests and
//      the new ones, the running ones' Tucker states and kept eigenbases
//      copied over device to device, so they continue exactly where they
//      were.  With no cohort of their kind they form a new one (own
//      sub-context, default-priority stream and state);
//   2. keeps one step in flight per cohort, with the residual and the numeric
//      flag of every instance copied back; a cohort whose step has completed
//      gets its next step at once, without waiting for the other cohorts;
//   3. retires a request whose residual fell below its tolerance, that
//      reached its step limit, or whose cells turned non-finite: its
//      macroparameters are copied out and its instance is frozen (moments
//      and rounding skip its cells from the next step on).  A cohort's
//      memory returns to the budget when its last request retires or when
//      it is rebuilt (during a rebuild the old and new states coexist).
// Instances never exchange data and every kernel's arithmetic on a cell is
// the same whichever cells share its launch, so a request's result does not
// depend on the requests served beside it.
// Times are seconds since the server was created.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>

#include "tk_runtime.h"

namespace {

struct ServeReq {
  uint64_t ticket = 0;
  std::vector<int32_t> fl, fr;
  std::vector<double> fn, fa, vol, ctr, macro;
  std::vector<tk_bc> bc;
  tk_mesh_desc desc{};
  tk_params params{};
  int32_t max_steps = 0;
  double res_tol = 0.0;
  size_t bytes = 0;
  bool oblique = false;  // a face off the coordinate axes
  double t_arrive = 0, t_admit = -1, t_done = -1;
  tk_status status = TK_PENDING;
  int32_t steps = 0;
  double residual = INFINITY;
  std::vector<double> macro_out;
};

// Requests stepped by one batched state; owned by the worker thread.
struct Cohort {
  tk_ctx* ctx = nullptr;
  std::vector<tk_mesh*> meshes;
  tk_state* st = nullptr;
  std::vector<ServeReq*> mem;  // instance k = mem[k]
  std::vector<char> live;
  int n_live = 0;
  double* h_res = nullptr;     // pinned [instances]
  int* h_flag = nullptr;       // pinned [instances]
  hipEvent_t ev = nullptr;     // end of the step in flight
  bool inflight = false;
  tk_status step_status = TK_OK;
  size_t bytes = 0;
};

}  // namespace

struct tk_server {
  tk_ctx* parent = nullptr;
  size_t budget = 0;
  size_t in_use = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  uint64_t next = 1;
  std::map<uint64_t, std::unique_ptr<ServeReq>> reqs;
  std::deque<uint64_t> queue;
  std::vector<std::unique_ptr<Cohort>> cohorts;  // worker thread only
  std::vector<ServeReq*> pending;  // admitted, waiting for a running cohort of their kind
  int64_t stats[4] = {0, 0, 0, 0};  // cohorts, cohort steps, request steps, largest cohort
  std::chrono::steady_clock::time_point t0;
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void release(Cohort* c) {
  if (c->st) tk_state_destroy(c->st);
  for (tk_mesh* m : c->meshes) tk_mesh_destroy(m);
  if (c->ev) (void)hipEventDestroy(c->ev);
  if (c->ctx) tk_ctx_destroy(c->ctx);
  if (c->h_res) (void)hipHostFree(c->h_res);
  if (c->h_flag) (void)hipHostFree(c->h_flag);
  c->st = nullptr;
  c->meshes.clear();
  c->ev = nullptr;
  c->ctx = nullptr;
  c->h_res = nullptr;
  c->h_flag = nullptr;
}

// migrated: the first requests of c->mem, whose states (and face
// estimates) the caller copies in from their previous cohort
tk_status form(int device, Cohort* c, int migrated = 0) {
  const int n = (int)c->mem.size();
  for (ServeReq* r : c->mem) c->bytes += r->bytes;
  tk_status s = tk_ctx_create(device, c->bytes + (256u << 20), nullptr, &c->ctx);
  std::vector<tk_params> params;
  std::vector<const double*> macros;
  for (int k = 0; k < n && s == TK_OK; ++k) {
    tk_mesh* m = nullptr;
    s = tk_mesh_load(c->ctx, &c->mem[k]->desc, &m);
    if (s == TK_OK) c->meshes.push_back(m);
    params.push_back(c->mem[k]->params);
    macros.push_back(c->mem[k]->macro.data());
  }
  if (s == TK_OK)
    s = state_create_served(c->ctx, n, (const tk_mesh* const*)c->meshes.data(), params.data(), macros.data(),
                            &c->st, migrated);
  // one rounding pass per step (pass-size trials would serialise the mix)
  if (s == TK_OK) s = tk_state_set_chunk(c->st, c->st->chunk_max);
  if (s == TK_OK && (hipHostMalloc((void**)&c->h_res, sizeof(double) * n) != hipSuccess ||
                     hipHostMalloc((void**)&c->h_flag, sizeof(int) * n) != hipSuccess ||
                     hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess))
    s = TK_EDEVICE;
  c->live.assign(n, 1);
  c->n_live = n;
  return s;
}

// Requests that can share a batched state: the same N and precision, and
// the same face kind (which selects the expansion kernels).
bool same_kind(const ServeReq* a, const ServeReq* b) {
  return a->params.N == b->params.N && a->params.precision == b->params.precision && a->oblique == b->oblique;
}

struct Out {
  ServeReq* r;
  tk_status status;
  bool finished, stepped;
  double residual;
  std::vector<double> macro;
};

// Outcome of a cohort's completed step for each of its running requests;
// the requests that finish are frozen in the state.
void collect(Cohort* c, std::vector<Out>& outs) {
  const size_t first = outs.size();
  bool copy = false;
  for (size_t k = 0; k < c->mem.size(); ++k) {
    if (!c->live[k]) continue;
    ServeReq* r = c->mem[k];
    Out o{r, TK_PENDING, false, false, r->residual, {}};
    if (c->step_status != TK_OK) {
      o.status = c->step_status;
      o.finished = true;
    } else {
      o.stepped = true;
      o.residual = c->h_res[k];
      if (c->h_flag[k]) {
        o.status = TK_ENUMERIC;
        o.finished = true;
      } else if (o.residual < r->res_tol || r->steps + 1 >= r->max_steps) {
        o.status = TK_OK;
        o.finished = true;
        copy = true;
      }
    }
    outs.push_back(std::move(o));
  }
  if (copy) {
    std::vector<double> all((size_t)c->st->nc * 8);
    const tk_status s = tk_moments(c->st, all.data());
    for (size_t i = first; i < outs.size(); ++i) {
      Out& o = outs[i];
      if (!o.finished || o.status != TK_OK) continue;
      if (s != TK_OK) {
        o.status = s;
        continue;
      }
      const size_t k = std::find(c->mem.begin(), c->mem.end(), o.r) - c->mem.begin();
      const size_t a = (size_t)c->st->inst_off[k], b = (size_t)c->st->inst_off[k + 1];
      o.macro.assign(all.begin() + 8 * a, all.begin() + 8 * b);
    }
  }
  for (size_t i = first; i < outs.size(); ++i) {
    if (!outs[i].finished) continue;
    const size_t k = std::find(c->mem.begin(), c->mem.end(), outs[i].r) - c->mem.begin();
    c->live[k] = 0;
    --c->n_live;
    if (c->n_live > 0 && state_freeze_instance(c->st, (int)k) != TK_OK) c->step_status = TK_EDEVICE;
  }
}

void worker_loop(tk_server* srv) {
  (void)hipSetDevice(srv->parent->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    if (srv->stop) break;
    // 1. admission by memory, in arrival order among those that fit; one
    // cohort per (N, precision, oblique) of the admitted requests
    std::vector<ServeReq*> adm;
    for (auto it = srv->queue.begin(); it != srv->queue.end();) {
      ServeReq* r = srv->reqs[*it].get();
      if (srv->in_use + r->bytes > srv->budget) {
        ++it;
        continue;
      }
      it = srv->queue.erase(it);
      srv->in_use += r->bytes;
      r->t_admit = srv->now();
      adm.push_back(r);
    }
    srv->pending.insert(srv->pending.end(), adm.begin(), adm.end());
    if (!srv->pending.empty()) {
      lk.unlock();
      // one group per kind, in arrival order
      std::vector<std::vector<ServeReq*>> groups;
      for (ServeReq* r : srv->pending) {
        std::vector<ServeReq*>* g = nullptr;
        for (auto& x : groups)
          if (same_kind(x[0], r)) g = &x;
        if (!g) {
          groups.emplace_back();
          g = &groups.back();
        }
        g->push_back(r);
      }
      std::vector<ServeReq*> waiting;
      std::vector<std::unique_ptr<Cohort>> made, failed;
      std::vector<std::pair<Cohort*, std::unique_ptr<Cohort>>> merged;  // old cohort, its replacement
      for (auto& g : groups) {
        Cohort* idle = nullptr;
        bool busy = false;
        for (auto& c : srv->cohorts) {
          if (!same_kind(c->mem[0], g[0]) || c->n_live == 0 || c->step_status != TK_OK) continue;
          if (c->inflight) busy = true;
          else if (!idle) idle = c.get();
        }
        if (!idle && busy) {
          // join a running cohort of this kind when its step completes
          waiting.insert(waiting.end(), g.begin(), g.end());
          continue;
        }
        std::unique_ptr<Cohort> c(new Cohort());
        std::vector<int> from;  // instance of the old cohort each migrated request had
        if (idle)
          for (size_t k = 0; k < idle->mem.size(); ++k)
            if (idle->live[k]) {
              c->mem.push_back(idle->mem[k]);
              from.push_back((int)k);
            }
        c->mem.insert(c->mem.end(), g.begin(), g.end());
        tk_status s = form(srv->parent->device, c.get(), (int)from.size());
        for (size_t k = 0; k < from.size() && s == TK_OK; ++k)
          s = state_copy_instance(c->st, (int)k, idle->st, from[k]);
        if (s == TK_OK && !from.empty() && hipStreamSynchronize(c->ctx->stream) != hipSuccess) s = TK_EDEVICE;
        if (s == TK_OK) {
          if (idle) merged.emplace_back(idle, std::move(c));
          else made.push_back(std::move(c));
          continue;
        }
        release(c.get());
        if (idle) {
          // the running requests stay where they were; the new ones alone
          std::unique_ptr<Cohort> a(new Cohort());
          a->mem = g;
          s = form(srv->parent->device, a.get());
          if (s == TK_OK) {
            made.push_back(std::move(a));
            continue;
          }
          release(a.get());
          c.reset(new Cohort());
          c->mem = g;
        }
        c->step_status = s;
        failed.push_back(std::move(c));
      }
      std::vector<std::unique_ptr<Cohort>> old;
      lk.lock();
      srv->pending = waiting;
      const double t = srv->now();
      for (auto& c : failed)
        for (ServeReq* r : c->mem) {
          r->status = c->step_status;
          r->t_done = t;
          srv->in_use -= r->bytes;
        }
      for (auto& m : merged) {
        // the replaced cohort's retired requests' memory returns to the budget
        size_t live = 0;
        for (size_t k = 0; k < m.first->mem.size(); ++k)
          if (m.first->live[k]) live += m.first->mem[k]->bytes;
        srv->in_use -= m.first->bytes - live;
        for (auto& c : srv->cohorts)
          if (c.get() == m.first) {
            old.push_back(std::move(c));
            c = std::move(m.second);
            srv->stats[0] += 1;
            srv->stats[3] = std::max<int64_t>(srv->stats[3], (int64_t)c->mem.size());
            break;
          }
      }
      for (auto& c : made) {
        srv->stats[0] += 1;
        srv->stats[3] = std::max<int64_t>(srv->stats[3], (int64_t)c->mem.size());
        srv->cohorts.push_back(std::move(c));
      }
      if (!old.empty()) {
        lk.unlock();
        for (auto& c : old) release(c.get());
        lk.lock();
      }
    }
    if (srv->cohorts.empty()) {
      srv->cv.wait(lk, [&] { return srv->stop || !srv->queue.empty(); });
      continue;
    }
    lk.unlock();
    // 2. a step in flight for every cohort
    for (auto& c : srv->cohorts) {
      if (c->inflight) continue;
      c->inflight = true;
      if (c->step_status != TK_OK) continue;  // retired below with that status
      std::lock_guard<std::recursive_mutex> g(c->ctx->mu);
      tk_status s = state_step_residual_async(c->st, c->h_res, c->h_flag);
      if (s == TK_OK && hipEventRecord(c->ev, c->ctx->stream) != hipSuccess) s = TK_EDEVICE;
      c->step_status = s;  // an enqueue error retires the cohort's requests below
    }
    // 3. the cohorts whose step has completed (polled: none waits for another)
    std::vector<Cohort*> ready;
    for (;;) {
      for (auto& c : srv->cohorts) {
        if (c->step_status != TK_OK) {
          ready.push_back(c.get());
          continue;
        }
        const hipError_t q = hipEventQuery(c->ev);
        if (q == hipSuccess) {
          ready.push_back(c.get());
        } else if (q != hipErrorNotReady) {
          c->step_status = TK_EDEVICE;
          ready.push_back(c.get());
        }
      }
      if (!ready.empty()) break;
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    std::vector<Out> outs;
    int64_t stepped = 0;
    for (Cohort* c : ready) {
      if (c->step_status == TK_OK) stepped += 1;
      collect(c, outs);
      c->inflight = false;
    }
    // results are published to pollers under the lock only
    std::vector<std::unique_ptr<Cohort>> done;
    lk.lock();
    const double t = srv->now();
    srv->stats[1] += stepped;
    for (Out& o : outs) {
      ServeReq* r = o.r;
      if (o.stepped) {
        r->steps += 1;
        srv->stats[2] += 1;
      }
      r->residual = o.residual;
      if (!o.finished) continue;
      r->macro_out = std::move(o.macro);
      r->t_done = t;
      r->status = o.status;
    }
    for (auto it = srv->cohorts.begin(); it != srv->cohorts.end();) {
      if ((*it)->n_live > 0) {
        ++it;
        continue;
      }
      srv->in_use -= (*it)->bytes;
      done.push_back(std::move(*it));
      it = srv->cohorts.erase(it);
    }
    if (!done.empty()) {
      lk.unlock();
      for (auto& c : done) release(c.get());
      lk.lock();
    }
  }
}

}  // namespace

extern "C" {

tk_status tk_serve_create(tk_ctx* ctx, size_t hbm_budget, tk_server** out) {
  if (!ctx || !out) return TK_EINVAL;
  *out = nullptr;
  if (ctx->device < 0) return ctx_fail(ctx, TK_EDEVICE, "serve: host-only context");
  std::unique_ptr<tk_server> s(new tk_server());
  s->parent = ctx;
  s->budget = hbm_budget ? hbm_budget : ctx->budget;
  s->t0 = std::chrono::steady_clock::now();
  tk_server* p = s.get();
  p->worker = std::thread(worker_loop, p);
  *out = s.release();
  return TK_OK;
}

tk_status tk_serve_submit(tk_server* srv, const tk_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket || !req->macro) return TK_EINVAL;
  const tk_mesh_desc& d = req->mesh;
  if (d.n_cells <= 0 || d.n_faces <= 0 || !d.face_left || !d.face_right || !d.face_normal || !d.face_area ||
      !d.cell_volume || d.n_bc < 0 || (d.n_bc > 0 && !d.bc) || req->max_steps < 1)
    return TK_EINVAL;
  std::unique_ptr<ServeReq> r(new ServeReq());
  const int nc = d.n_cells, nf = d.n_faces;
  r->fl.assign(d.face_left, d.face_left + nf);
  r->fr.assign(d.face_right, d.face_right + nf);
  r->fn.assign(d.face_normal, d.face_normal + 3 * (size_t)nf);
  r->fa.assign(d.face_area, d.face_area + nf);
  r->vol.assign(d.cell_volume, d.cell_volume + nc);
  if (d.cell_center) r->ctr.assign(d.cell_center, d.cell_center + 3 * (size_t)nc);
  r->bc.assign(d.bc, d.bc + d.n_bc);
  r->macro.assign(req->macro, req->macro + 5 * (size_t)nc);
  r->desc = d;
  r->desc.face_left = r->fl.data();
  r->desc.face_right = r->fr.data();
  r->desc.face_normal = r->fn.data();
  r->desc.face_area = r->fa.data();
  r->desc.cell_volume = r->vol.data();
  r->desc.cell_center = d.cell_center ? r->ctr.data() : nullptr;
  r->desc.bc = r->bc.data();
  r->params = req->params;
  r->max_steps = req->max_steps;
  r->res_tol = req->residual_tol;
  // served states lay every cell out for the largest rank cap
  tk_params pm = req->params;
  pm.rank_cap = tk::kMaxCap;
  r->bytes = state_bytes_estimate(nc, pm, false, nc);
  for (int f = 0; f < nf && !r->oblique; ++f) r->oblique = face_axis(&r->fn[3 * (size_t)f]) < 0;
  std::lock_guard<std::mutex> g(srv->mu);
  if (srv->stop) return TK_EBUSY;
  if (r->bytes > srv->budget) return TK_ENOMEM;
  r->ticket = srv->next++;
  r->t_arrive = srv->now();
  *ticket = r->ticket;
  srv->queue.push_back(r->ticket);
  srv->reqs[r->ticket] = std::move(r);
  srv->cv.notify_all();
  return TK_OK;
}

tk_status tk_serve_poll(tk_server* srv, uint64_t ticket, tk_result* res) {
  if (!srv || !res) return TK_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return TK_ENOTFOUND;
  ServeReq* r = it->second.get();
  res->status = r->status;
  res->steps = r->steps;
  res->residual = r->residual;
  res->t_arrive = r->t_arrive;
  res->t_admit = r->t_admit;
  res->t_done = r->t_done;
  if (r->status != TK_PENDING && res->macro_out && !r->macro_out.empty())
    std::memcpy(res->macro_out, r->macro_out.data(), sizeof(double) * r->macro_out.size());
  return r->status;
}

tk_status tk_serve_stats(tk_server* srv, int64_t* out4) {
  if (!srv || !out4) return TK_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  for (int i = 0; i < 4; ++i) out4[i] = srv->stats[i];
  return TK_OK;
}

tk_status tk_serve_destroy(tk_server* srv) {
  if (!srv) return TK_EINVAL;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    srv->cv.notify_all();
  }
  if (srv->worker.joinable()) srv->worker.join();
  for (auto& c : srv->cohorts) release(c.get());
  delete srv;
  return TK_OK;
}

}  // extern "C"
