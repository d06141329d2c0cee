// Serving: continuous batching of independent solves on one device.
//
// Each admitted request gets its own sub-context (own default-priority HIP
// stream), mesh and Tucker state, so requests never share numerical work
// and a result is the same alone or in a mix.  A worker thread
//   1. admits queued requests, in arrival order, whenever the estimated
//      device memory of the request fits what the running ones leave of
//      the budget (a request that could never fit is refused at submit);
//   2. enqueues one step, with its residual, for every running request on
//      that request's stream, so their kernels overlap on the device;
//   3. waits for the streams, retires the requests whose residual fell below
//      their tolerance or that reached their step limit (macroparameters
//      copied out), and frees their memory for the next admissions.
// Times are seconds since the server was created.
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
  double t_arrive = 0, t_admit = -1, t_done = -1;
  tk_status status = TK_PENDING;
  int32_t steps = 0;
  double residual = INFINITY;
  std::vector<double> macro_out;
  tk_ctx* ctx = nullptr;
  tk_mesh* mesh = nullptr;
  tk_state* st = nullptr;
  double* h_res = nullptr;
  int* h_flag = nullptr;
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
  std::vector<ServeReq*> running;
  std::chrono::steady_clock::time_point t0;
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void release(ServeReq* r) {
  if (r->st) tk_state_destroy(r->st);
  if (r->mesh) tk_mesh_destroy(r->mesh);
  if (r->ctx) tk_ctx_destroy(r->ctx);
  if (r->h_res) (void)hipHostFree(r->h_res);
  if (r->h_flag) (void)hipHostFree(r->h_flag);
  r->st = nullptr;
  r->mesh = nullptr;
  r->ctx = nullptr;
  r->h_res = nullptr;
  r->h_flag = nullptr;
}

tk_status admit(tk_server* srv, ServeReq* r) {
  tk_status s = tk_ctx_create(srv->parent->device, r->bytes + (256u << 20), nullptr, &r->ctx);
  if (s == TK_OK) s = tk_mesh_load(r->ctx, &r->desc, &r->mesh);
  if (s == TK_OK) s = tk_state_init(r->ctx, r->mesh, &r->params, r->macro.data(), &r->st);
  // one rounding pass per step (no pass-size trials: each request runs alone
  // on its stream and its trial steps would serialise the mix)
  if (s == TK_OK) s = tk_state_set_chunk(r->st, r->st->chunk_max);
  if (s == TK_OK && (hipHostMalloc((void**)&r->h_res, sizeof(double)) != hipSuccess ||
                     hipHostMalloc((void**)&r->h_flag, sizeof(int)) != hipSuccess))
    s = TK_EDEVICE;
  return s;
}

void worker_loop(tk_server* srv) {
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    if (srv->stop) break;
    // 1. admission by memory, in arrival order among those that fit
    for (auto it = srv->queue.begin(); it != srv->queue.end();) {
      ServeReq* r = srv->reqs[*it].get();
      if (srv->in_use + r->bytes > srv->budget) {
        ++it;
        continue;
      }
      it = srv->queue.erase(it);
      srv->in_use += r->bytes;
      r->t_admit = srv->now();
      lk.unlock();
      const tk_status s = admit(srv, r);
      lk.lock();
      if (s != TK_OK) {
        release(r);
        r->status = s;
        r->t_done = srv->now();
        srv->in_use -= r->bytes;
      } else {
        srv->running.push_back(r);
      }
    }
    if (srv->running.empty()) {
      srv->cv.wait(lk, [&] { return srv->stop || !srv->queue.empty(); });
      continue;
    }
    std::vector<ServeReq*> run = srv->running;
    lk.unlock();
    // 2. one step of every running request, overlapped across streams
    std::vector<tk_status> st(run.size(), TK_OK);
    for (size_t i = 0; i < run.size(); ++i) {
      std::lock_guard<std::recursive_mutex> g(run[i]->ctx->mu);
      st[i] = state_step_residual_async(run[i]->st, run[i]->h_res, run[i]->h_flag);
    }
    // 3. completion; results are published to pollers under the lock only
    struct Out {
      ServeReq* r;
      tk_status status;
      bool finished;
      double residual;
      std::vector<double> macro;
    };
    std::vector<Out> outs;
    outs.reserve(run.size());
    for (size_t i = 0; i < run.size(); ++i) {
      ServeReq* r = run[i];
      Out o{r, TK_PENDING, false, r->residual, {}};
      if (st[i] == TK_OK && hipStreamSynchronize(r->ctx->stream) != hipSuccess) st[i] = TK_EDEVICE;
      if (st[i] != TK_OK) {
        o.status = st[i];
        o.finished = true;
      } else {
        o.residual = *r->h_res;
        const int steps = r->steps + 1;
        if (*r->h_flag) {
          o.status = TK_ENUMERIC;
          o.finished = true;
        } else if (o.residual < r->res_tol || steps >= r->max_steps) {
          o.macro.resize((size_t)r->desc.n_cells * 8);
          o.status = tk_moments(r->st, o.macro.data());
          o.finished = true;
        }
      }
      outs.push_back(std::move(o));
    }
    lk.lock();
    const double t = srv->now();
    for (size_t i = 0; i < outs.size(); ++i) {
      Out& o = outs[i];
      ServeReq* r = o.r;
      if (st[i] == TK_OK) r->steps += 1;
      r->residual = o.residual;
      if (!o.finished) continue;
      r->macro_out = std::move(o.macro);
      r->t_done = t;
      r->status = o.status;
      release(r);
      srv->in_use -= r->bytes;
      srv->running.erase(std::find(srv->running.begin(), srv->running.end(), r));
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
  r->bytes = state_bytes_estimate(nc, req->params, false, nc);
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

tk_status tk_serve_destroy(tk_server* srv) {
  if (!srv) return TK_EINVAL;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    srv->cv.notify_all();
  }
  if (srv->worker.joinable()) srv->worker.join();
  for (auto& kv : srv->reqs) release(kv.second.get());
  delete srv;
  return TK_OK;
}

}  // extern "C"
