// Host side of the tk library: contexts, meshes, states, the step driver
// and the C ABI entry points (declared in tk.h).
//
// Mesh data follow the finite-volume form of the method (eq. ode_system):
// per face its two cells, unit normal and area, per cell its volume.  Each
// cell gets up to six face slots naming what lies on the far side and the
// slot's outward orientation, with coefficient dt A / V.  The time step is
// dt = cfl / max_i (D_i + nu_i^0), D_i = xi_max / (2 V_i) sum_l A_l ||e_l||_1,
// the positivity bound of the explicit scheme (eq. expl-scheme-final),
// with nu^0 taken from the initial macroparameters.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>

#include "tk_internal.h"
#include "tk_runtime.h"

namespace tk {
const char* kKernelNames[KID_COUNT] = {"moments", "expand", "gram", "eig", "project", "init",
                                       "plain_moments", "plain_step", "residual", "rround", "lusgs"};
}

using namespace tk;

// ---------------------------------------------------------------------------
// Scratch of tk_round_tucker_noalloc: device memory that the library never
// allocates at run time.  Every GPU that loads the library holds its own
// copy of this array until the process ends.  In host code the name is only
// a host-side stand-in: kernels and copies take the device address that
// hipGetSymbolAddress returns for the current device (scratch_lookup).

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.
static hipError_t scratch_lookup(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// context helpers

tk_status ctx_fail(tk_ctx* ctx, tk_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

tk_status ctx_hip(tk_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return TK_OK;
  return ctx_fail(ctx, e == hipErrorOutOfMemory ? TK_ENOMEM : TK_EDEVICE,
                  std::string(what) + ": " + hipGetErrorString(e));
}

void* ctx_alloc(tk_ctx* ctx, size_t bytes, tk_status* st) {
  *st = TK_OK;
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~size_t(255);
  if (ctx->used + bytes > ctx->budget) {
    *st = ctx_fail(ctx, TK_ENOMEM, "allocation of " + std::to_string(bytes) + " bytes exceeds the budget");
    return nullptr;
  }
  void* p = nullptr;
  if (ctx->alloc.alloc) {
    p = ctx->alloc.alloc(ctx->alloc.user, bytes);
    if (!p) {
      *st = ctx_fail(ctx, TK_ENOMEM, "the caller's allocator returned no memory for " + std::to_string(bytes) + " bytes");
      return nullptr;
    }
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      *st = ctx_hip(ctx, e, "hipMalloc");
      return nullptr;
    }
  }
  ctx->used += bytes;
  ctx->sizes[p] = bytes;
  return p;
}

void ctx_free(tk_ctx* ctx, void* p) {
  if (!p) return;
  auto it = ctx->sizes.find(p);
  if (it != ctx->sizes.end()) {
    ctx->used -= it->second;
    ctx->sizes.erase(it);
  }
  if (ctx->alloc.alloc) ctx->alloc.free(ctx->alloc.user, p);
  else (void)hipFree(p);
}

void prof_begin(tk_ctx* ctx, int kid, hipEvent_t* ev, hipStream_t q = nullptr) {
  *ev = nullptr;
  if (!ctx->prof) return;
  if (ctx->ev_pool.empty()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    ctx->ev_pool.push_back(e);
  }
  *ev = ctx->ev_pool.back();
  ctx->ev_pool.pop_back();
  (void)hipEventRecord(*ev, q ? q : ctx->stream);
  (void)kid;
}

void prof_end(tk_ctx* ctx, int kid, hipEvent_t start, hipStream_t q = nullptr) {
  if (!ctx->prof || !start) return;
  hipEvent_t e;
  if (ctx->ev_pool.empty()) {
    if (hipEventCreate(&e) != hipSuccess) return;
  } else {
    e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
  }
  (void)hipEventRecord(e, q ? q : ctx->stream);
  ctx->pending.push_back({kid, start, e});
}

void prof_harvest(tk_ctx* ctx) {
  for (auto& p : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->prof_ms[p.kid] += ms;
      ctx->prof_n[p.kid] += 1;
    }
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.clear();
}

// ---------------------------------------------------------------------------
// mesh

static tk_status mesh_build(tk_ctx* ctx, const tk_mesh_desc* d, tk_mesh* m) {
  std::string err;
  const tk_status s = tk::mesh_build_host(d, m, &err);
  return s == TK_OK ? TK_OK : ctx_fail(ctx, s, err);
}

// ---------------------------------------------------------------------------
// state

static const int kSupportedN[] = {16, 24, 32, 48};

static tk_status check_params(tk_ctx* ctx, const tk_params* p) {
  bool okN = false;
  for (int n : kSupportedN) okN |= (p->N == n);
  if (!okN) return ctx_fail(ctx, TK_EINVAL, "params: N must be 16, 24, 32 or 48");
  if (p->rank_cap < 1 || p->rank_cap > kMaxCap || p->rank_cap > p->N)
    return ctx_fail(ctx, TK_EINVAL, "params: rank_cap must be in 1..16 and <= N");
  if (!(p->xi_max > 0) || !(p->R_g > 0) || !(p->m > 0) || !(p->Kn > 0) || !(p->cfl > 0) || !(p->tol >= 0) ||
      !(p->Pr > 0))
    return ctx_fail(ctx, TK_EINVAL, "params: xi_max, R_g, m, Kn, cfl, Pr must be positive and tol >= 0");
  if (p->precision != TK_FP64 && p->precision != TK_MIXED)
    return ctx_fail(ctx, TK_EINVAL, "params: precision must be TK_FP64 or TK_MIXED");
  return TK_OK;
}

static double collision_freq(const tk_params& p, double n, double T) {
  return p.m * n * p.R_g * T / (0.5 * p.Kn * std::pow(T, p.omega));
}

void state_free(tk_state* st) {
  tk_ctx* ctx = st->ctx;
  for (int p = 0; p < 2; ++p)
    if (st->gexec[p]) (void)hipGraphExecDestroy(st->gexec[p]);
  st->gexec[0] = st->gexec[1] = nullptr;
  for (hipEvent_t e : st->tune_ev) (void)hipEventDestroy(e);
  st->tune_ev.clear();
  if (st->ev_fork) (void)hipEventDestroy(st->ev_fork);
  if (st->ev_join) (void)hipEventDestroy(st->ev_join);
  if (st->q2) (void)hipStreamDestroy(st->q2);
  st->ev_fork = st->ev_join = nullptr;
  st->q2 = nullptr;
  for (void* p : st->allocs) ctx_free(ctx, p);
  st->allocs.clear();
  if (st->h_rcnt) (void)hipHostFree(st->h_rcnt);
  st->h_rcnt = nullptr;
}

static void* st_alloc(tk_state* st, size_t bytes, tk_status* s) {
  void* p = ctx_alloc(st->ctx, bytes, s);
  if (p) st->allocs.push_back(p);
  return p;
}

DevState state_dev(const tk_state* st) {
  DevState d;
  d.n_cells = st->nc;
  d.N = st->N;
  d.CS = st->CS;
  d.inst = st->d_inst;
  d.ip = st->d_ip;
  d.slot_nb = st->d_slot_nb;
  d.slot_kind = st->d_slot_kind;
  d.slot_axis = st->d_slot_axis;
  d.slot_sig = st->d_slot_sig;
  d.slot_coef = st->d_slot_coef;
  d.bc_fac = st->d_bc_fac;
  d.core = st->core[st->cur];
  d.fac = st->fac[st->cur];
  d.rank = st->rank[st->cur];
  d.core_n = st->core[st->cur ^ 1];
  d.fac_n = st->fac[st->cur ^ 1];
  d.rank_n = st->rank[st->cur ^ 1];
  d.macro = st->d_macro;
  d.nu = st->d_nu;
  d.nw = st->d_nw;
  d.flag = st->d_flag;
  d.slot_nrm = st->d_slot_nrm;
  d.slot_est = st->d_slot_est;
  d.est_core = st->d_est_core;
  d.est_fac = st->d_est_fac;
  d.est_rank = st->d_est_rank;
  d.cells = nullptr;
  d.cells_n = nullptr;
  return d;
}

DevPlain plain_dev(const tk_state* st) {
  DevPlain d;
  d.n_cells = st->nc;
  d.N = st->N;
  d.inst = st->d_inst;
  d.ip = st->d_ip;
  d.slot_nb = st->d_slot_nb;
  d.slot_kind = st->d_slot_kind;
  d.slot_axis = st->d_slot_axis;
  d.slot_sig = st->d_slot_sig;
  d.slot_coef = st->d_slot_coef;
  d.bc_fac = st->d_bc_fac;
  d.slot_nrm = st->d_slot_nrm;
  d.f = st->pf[st->cur];
  d.f_n = st->pf[st->cur ^ 1];
  d.macro = st->d_macro;
  d.nu = st->d_nu;
  d.nw = st->d_nw;
  d.flag = st->d_flag;
  return d;
}

size_t state_bytes_estimate(int nc, const tk_params& p, bool plain, int chunk) {
  // the allocations of state_create for one instance (slot tables, macros,
  // Tucker buffers, eigenbases, rounding workspaces), rounded up by 10%
  const size_t N = p.N, CS = std::max(4, p.rank_cap);
  const size_t tsz = p.precision == TK_MIXED ? 4 : 8;
  size_t b = (size_t)nc * (4 + kSlots * (4 + 3 + 8) + 8 + 8 * 8 * 3 + 8 + 8 * kSlots);
  if (plain) {
    b += 2 * (size_t)nc * N * N * N * tsz;
  } else {
    const size_t ch = std::min<size_t>((size_t)nc, (size_t)chunk);
    b += 2 * (size_t)nc * (CS * CS * CS + 3 * CS * N) * 8 + 2 * (size_t)nc * 3 * 4;
    b += (size_t)nc * 3 * N * N * 8;                      // warm-start eigenbases
    b += (size_t)nc * (4 + 4 + 12);                       // rounding lists, basis validity
    b += ch * (N * N * N * tsz + 3 * N * N * 8 + 8);      // X, Gram workspaces, the expansion's cell lists
    if (p.precision == TK_FP64) b += ch * 3 * N * N * 8;  // first-pass bases
    b += (size_t)nc * kSlots * (3 * 8 + 4);               // oblique slots
    b += (size_t)nc * 3 * (kEstCap * kEstCap * kEstCap + 3 * kEstCap * N) * 8 / 2;  // estimates
  }
  return b + b / 10 + (64u << 20);
}

static tk_status state_create(tk_ctx* ctx, int count, const tk_mesh* const* meshes, const tk_params* params,
                              const double* const* macros, bool plain, tk_state** out, bool served = false,
                              int est_skip = 0) {
  if (!ctx || !out || count <= 0 || !meshes || !params || !macros) return ctx_fail(ctx, TK_EINVAL, "state: null argument");
  *out = nullptr;
  if (ctx->device < 0) return ctx_fail(ctx, TK_EDEVICE, "state: host-only context");
  const int N = params[0].N;
  const int prec = params[0].precision;
  int CS = 4, nc = 0, nbc = 0;
  for (int k = 0; k < count; ++k) {
    tk_status s = check_params(ctx, &params[k]);
    if (s != TK_OK) return s;
    if (params[k].N != N || params[k].precision != prec)
      return ctx_fail(ctx, TK_EINVAL, "state: all instances of a batch share N and precision");
    if (!meshes[k] || !macros[k]) return ctx_fail(ctx, TK_EINVAL, "state: null mesh or macro");
    CS = std::max(CS, params[k].rank_cap);
    nc += meshes[k]->n_cells;
    nbc += (int)meshes[k]->bc.size();
  }
  // a server's states share one layout, so that instances can move between
  // them (state_copy_instance)
  if (served) CS = kMaxCap;
  std::unique_ptr<tk_state> st(new tk_state());
  st->ctx = ctx;
  st->N = N;
  st->CS = CS;
  st->mixed = (prec == TK_MIXED);
  st->plain = plain;
  st->nc = nc;
  st->ninst = count;
  st->params.assign(params, params + count);
  st->meshes.assign(meshes, meshes + count);
  // host tables
  std::vector<int> inst(nc), slot_nb((size_t)nc * kSlots);
  std::vector<int8_t> slot_kind((size_t)nc * kSlots), slot_axis((size_t)nc * kSlots), slot_sig((size_t)nc * kSlots);
  std::vector<double> slot_coef((size_t)nc * kSlots), vol(nc), bc_fac((size_t)std::max(nbc, 1) * 3 * N, 0.0);
  std::vector<double> macro5((size_t)nc * 5);
  std::vector<InstParams> ip(count);
  std::vector<double> slot_nrm((size_t)nc * kSlots * 3, 0.0);
  std::vector<int> slot_est((size_t)nc * kSlots, -1);
  std::vector<double> est_nrm;   // normals of the oblique faces
  std::vector<int> est_inst;     // owning instance of each estimate
  bool oblique = false;
  for (int k = 0; k < count; ++k) oblique |= meshes[k]->oblique;
  st->inst_off.assign(count + 1, 0);
  st->est_off.assign(count + 1, 0);
  int c0 = 0, b0 = 0;
  for (int k = 0; k < count; ++k) {
    const tk_mesh* m = meshes[k];
    const int est_start = (int)est_inst.size();
    const tk_params& p = params[k];
    const double dxi = 2.0 * p.xi_max / (N - 1);
    // time step of this instance
    double dmax = 0.0;
    for (int c = 0; c < m->n_cells; ++c) {
      const double* mc = macros[k] + 5 * (size_t)c;
      for (int a = 0; a < 5; ++a)
        if (!std::isfinite(mc[a])) return ctx_fail(ctx, TK_ENUMERIC, "state: non-finite initial macroparameter");
      if (!(mc[0] > 0.0) || !(mc[4] > 0.0)) return ctx_fail(ctx, TK_ENUMERIC, "state: initial n or T not positive");
      double l1 = 0.0;
      for (int s = 0; s < kSlots; ++s) l1 += m->slot_l1[(size_t)c * kSlots + s];
      const double D = p.xi_max / (2.0 * m->volume[c]) * l1;
      dmax = std::max(dmax, D + collision_freq(p, mc[0], mc[4]));
    }
    const double dt = p.cfl / dmax;
    InstParams& P = ip[k];
    P.xi_min = -p.xi_max;
    P.dxi = dxi;
    P.dt = dt;
    P.Rg = p.R_g;
    P.m = p.m;
    P.Pr = p.Pr;
    P.omega = p.omega;
    P.Kn = p.Kn;
    P.tol = p.tol;
    P.cap = p.rank_cap;
    P.frozen = 0;
    std::vector<int> face_est(m->oblique ? m->n_faces : 0, -1);
    for (int c = 0; c < m->n_cells; ++c) {
      const int g = c0 + c;
      inst[g] = k;
      vol[g] = m->volume[c];
      std::memcpy(&macro5[5 * (size_t)g], macros[k] + 5 * (size_t)c, 5 * sizeof(double));
      for (int s = 0; s < kSlots; ++s) {
        const size_t src = (size_t)c * kSlots + s, dst = (size_t)g * kSlots + s;
        const int8_t kind = m->slot_kind[src];
        slot_kind[dst] = kind;
        slot_axis[dst] = m->slot_axis[src];
        slot_sig[dst] = m->slot_sig[src];
        slot_coef[dst] = dt * m->slot_area[src] / m->volume[c];
        slot_nb[dst] = (kind == SK_INTERIOR) ? m->slot_nb[src] + c0 : (kind == SK_NONE ? -1 : m->slot_nb[src] + b0);
        for (int a = 0; a < 3; ++a) slot_nrm[3 * dst + a] = m->slot_nrm[3 * src + a];
        if (kind != SK_NONE && m->slot_axis[src] < 0) {
          const int j = m->slot_face[src];
          if (face_est[j] < 0) {
            face_est[j] = (int)est_inst.size();
            est_inst.push_back(k);
            for (int a = 0; a < 3; ++a) est_nrm.push_back(m->face_normal[3 * (size_t)j + a]);
          }
          slot_est[dst] = face_est[j];
        }
      }
    }
    // rank-1 boundary Maxwellian factors
    for (size_t b = 0; b < m->bc.size(); ++b) {
      const tk_bc& bc = m->bc[b];
      double n = 0, T = 0, u[3] = {0, 0, 0};
      if (bc.kind == TK_BC_INFLOW) {
        n = bc.n; T = bc.T; u[0] = bc.u[0]; u[1] = bc.u[1]; u[2] = bc.u[2];
        if (!(n > 0) || !(T > 0)) return ctx_fail(ctx, TK_EINVAL, "state: inflow n and T must be positive");
      } else if (bc.kind == TK_BC_WALL) {
        n = 1.0; T = bc.T_w;
        if (!(T > 0)) return ctx_fail(ctx, TK_EINVAL, "state: wall temperature must be positive");
      } else {
        continue;
      }
      const double amp = std::cbrt(n) / std::sqrt(2.0 * M_PI * p.R_g * T);
      for (int a = 0; a < 3; ++a)
        for (int i = 0; i < N; ++i) {
          const double x = -p.xi_max + i * dxi - u[a];
          bc_fac[((size_t)(b0 + b) * 3 + a) * N + i] = amp * std::exp(-x * x / (2.0 * p.R_g * T));
        }
    }
    st->inst_off[k] = c0;
    st->est_off[k] = est_start;
    c0 += m->n_cells;
    b0 += (int)m->bc.size();
  }
  st->est_off[count] = (int)est_inst.size();
  st->inst_off[count] = c0;
  st->ip_host = ip;
  // chunk of cells processed per rounding pass
  const size_t tsz = st->mixed ? 4 : 8;
  const size_t per = (size_t)N * N * N * tsz + 3 * (size_t)N * N * 8;
  size_t ws = std::min<size_t>(ctx->budget / 4, (size_t)4 << 30);
  st->chunk = (int)std::max<size_t>(1, std::min<size_t>(nc, ws / per));
  st->chunk_max = st->chunk;
  // device allocations
  tk_status s = TK_OK;
  tk_state* S = st.get();
#define ALLOC(ptr, type, n)                                                    \
  do {                                                                         \
    S->ptr = (type*)st_alloc(S, sizeof(type) * (size_t)(n), &s);               \
    if (!S->ptr) { state_free(S); return s; }                                  \
  } while (0)
  ALLOC(d_inst, int, nc);
  ALLOC(d_ip, InstParams, count);
  ALLOC(d_slot_nb, int, (size_t)nc * kSlots);
  ALLOC(d_slot_kind, int8_t, (size_t)nc * kSlots);
  ALLOC(d_slot_axis, int8_t, (size_t)nc * kSlots);
  ALLOC(d_slot_sig, int8_t, (size_t)nc * kSlots);
  ALLOC(d_slot_coef, double, (size_t)nc * kSlots);
  ALLOC(d_bc_fac, double, (size_t)std::max(nbc, 1) * 3 * N);
  ALLOC(d_vol, double, nc);
  ALLOC(d_inst_off, int, count + 1);
  ALLOC(d_macro, double, (size_t)nc * 8);
  ALLOC(d_macro_prev, double, (size_t)nc * 8);
  ALLOC(d_nu, double, nc);
  ALLOC(d_nw, double, (size_t)nc * kSlots);
  ALLOC(d_flag, int, count);
  ALLOC(d_resid, double, count);
  ALLOC(d_macro5, double, (size_t)nc * 5);
  const int n_est = (int)est_inst.size();
  S->oblique = oblique;
  S->served = served;
  S->n_est = n_est;
  if (oblique) {
    ALLOC(d_slot_nrm, double, (size_t)nc * kSlots * 3);
    ALLOC(d_slot_est, int, (size_t)nc * kSlots);
    ALLOC(d_est_core, double, (size_t)std::max(n_est, 1) * kEstCap * kEstCap * kEstCap);
    ALLOC(d_est_fac, double, (size_t)std::max(n_est, 1) * 3 * kEstCap * N);
    ALLOC(d_est_rank, int, (size_t)std::max(n_est, 1) * 3);
  }
  if (plain) {
    for (int b = 0; b < 2; ++b) {
      S->pf[b] = st_alloc(S, tsz * (size_t)nc * N * N * N, &s);
      if (!S->pf[b]) { state_free(S); return s; }
    }
  } else {
    for (int b = 0; b < 2; ++b) {
      ALLOC(core[b], double, (size_t)nc * CS * CS * CS);
      ALLOC(fac[b], double, (size_t)nc * 3 * CS * N);
      ALLOC(rank[b], int, (size_t)nc * 3);
    }
    S->X = st_alloc(S, per * 0 + (size_t)S->chunk * N * N * N * tsz, &s);
    if (!S->X) { state_free(S); return s; }
    ALLOC(G, double, (size_t)S->chunk * 3 * N * N);
    // cells of a pass left to later expansion launches (ranks beyond the
    // small LDS layout, oblique sources beyond the one-stage budgets): two
    // lists and their counters, since the oblique expansion hands cells on twice
    ALLOC(ob_list, int, 2 * (size_t)S->chunk);
    ALLOC(ob_n, int, 2);
    if (!S->mixed) ALLOC(Wb, double, (size_t)S->chunk * 3 * N * N);
    ALLOC(Wkeep, double, (size_t)nc * 3 * N * N);
    ALLOC(d_wvalid, int, (size_t)nc * 3);
    ALLOC(d_rstats, unsigned long long, 8);
    // the factor-space kernel takes or leaves each cell by itself (a cell
    // with an oblique face goes to the N-basis passes)
    S->rspace_ok = N <= 32;
    S->rspace = S->rspace_ok;
    if (S->rspace_ok) {
      ALLOC(d_rlistD, int, nc);
      ALLOC(d_rcnt, int, 1);
      if (hipHostMalloc((void**)&S->h_rcnt, sizeof(int), 0) != hipSuccess) {
        S->h_rcnt = nullptr;
        state_free(S);
        return ctx_fail(ctx, TK_EDEVICE, "state: pinned host word");
      }
      *S->h_rcnt = 0;
    }
    // optional second workspace: only if it fits what the budget leaves
    // (with a margin), so that no error is recorded when it does not
    const size_t ch = (size_t)S->chunk;
    const size_t need = ch * N * N * N * tsz + ch * 3 * N * N * 8 * (S->mixed ? 1 : 2) + 2 * ch * 4 + 4096;
    if (nc > 1 && !served && ctx->used + need + (64u << 20) <= ctx->budget) {
      tk_status s2 = TK_OK;
      S->X2 = st_alloc(S, ch * N * N * N * tsz, &s2);
      if (S->X2) S->G2 = (double*)st_alloc(S, ch * 3 * N * N * 8, &s2);
      if (S->G2 && !S->mixed) S->Wb2 = (double*)st_alloc(S, ch * 3 * N * N * 8, &s2);
      if (S->G2 && (S->mixed || S->Wb2)) S->ob_list2 = (int*)st_alloc(S, 2 * ch * 4, &s2);
      if (S->ob_list2) S->ob_n2 = (int*)st_alloc(S, 2 * 4, &s2);
      if (S->ob_n2 && hipStreamCreate(&S->q2) != hipSuccess) S->q2 = nullptr;
      if (S->q2 && (hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming) != hipSuccess ||
                    hipEventCreateWithFlags(&S->ev_join, hipEventDisableTiming) != hipSuccess)) {
        if (S->ev_fork) (void)hipEventDestroy(S->ev_fork);
        S->ev_fork = nullptr;
        (void)hipStreamDestroy(S->q2);
        S->q2 = nullptr;
      }
      if (!S->q2) S->X2 = nullptr;  // the pieces are released with the state
    }
  }
#undef ALLOC
  hipStream_t q = ctx->stream;
  hipError_t e = hipSuccess;
  auto up = [&](void* dst, const void* src, size_t n) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, q);
  };
  up(S->d_inst, inst.data(), sizeof(int) * nc);
  up(S->d_ip, ip.data(), sizeof(InstParams) * count);
  up(S->d_slot_nb, slot_nb.data(), sizeof(int) * slot_nb.size());
  up(S->d_slot_kind, slot_kind.data(), slot_kind.size());
  up(S->d_slot_axis, slot_axis.data(), slot_axis.size());
  up(S->d_slot_sig, slot_sig.data(), slot_sig.size());
  up(S->d_slot_coef, slot_coef.data(), sizeof(double) * slot_coef.size());
  up(S->d_bc_fac, bc_fac.data(), sizeof(double) * bc_fac.size());
  up(S->d_vol, vol.data(), sizeof(double) * nc);
  up(S->d_inst_off, st->inst_off.data(), sizeof(int) * (count + 1));
  up(S->d_macro5, macro5.data(), sizeof(double) * macro5.size());
  if (oblique) {
    up(S->d_slot_nrm, slot_nrm.data(), sizeof(double) * slot_nrm.size());
    up(S->d_slot_est, slot_est.data(), sizeof(int) * slot_est.size());
  }
  if (e == hipSuccess) e = hipMemsetAsync(S->d_flag, 0, sizeof(int) * count, q);
  if (e == hipSuccess) e = hipMemsetAsync(S->d_nw, 0, sizeof(double) * (size_t)nc * kSlots, q);
  if (e == hipSuccess) e = hipMemsetAsync(S->d_macro, 0, sizeof(double) * (size_t)nc * 8, q);
  if (e != hipSuccess) { state_free(S); return ctx_hip(ctx, e, "state upload"); }
  S->cur = 0;
  if (plain) {
    e = launch_plain_init(plain_dev(S), S->d_macro5, S->mixed, q);
  } else {
    // zero both buffers' padding, then the rank-1 Maxwellians
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
      e = hipMemsetAsync(S->core[b], 0, sizeof(double) * (size_t)nc * CS * CS * CS, q);
      if (e == hipSuccess) e = hipMemsetAsync(S->fac[b], 0, sizeof(double) * (size_t)nc * 3 * CS * N, q);
      if (e == hipSuccess) e = hipMemsetAsync(S->rank[b], 0, sizeof(int) * (size_t)nc * 3, q);
    }
    if (e == hipSuccess) e = launch_init_maxwell(state_dev(S), S->d_macro5, q);
    if (e == hipSuccess) e = launch_identity_basis(N, (size_t)nc * 3, S->Wkeep, q);
    if (e == hipSuccess) e = launch_fill_int(S->d_wvalid, (size_t)nc * 3, 1, q);
    if (e == hipSuccess) e = hipMemsetAsync(S->d_rstats, 0, 8 * sizeof(unsigned long long), q);
    if (e == hipSuccess && oblique && n_est > st->est_off[std::min(est_skip, count)]) {
      // |xi . e| estimate of every oblique face: truncated HOSVD of the exact
      // tensor, mode ranks <= kEstCap, singular values <= kEstDrop sigma_1 dropped
      const size_t per_face = (size_t)N * N * N * 8 + 3 * (size_t)N * N * 8;
      const size_t avail = ctx->budget > ctx->used ? ctx->budget - ctx->used : 0;
      const int fch = (int)std::max<size_t>(1, std::min<size_t>(2048, avail / 2 / per_face));
      tk_status s2 = TK_OK;
      double* d_nrm = (double*)ctx_alloc(ctx, sizeof(double) * 3 * n_est, &s2);
      double* d_X = d_nrm ? (double*)ctx_alloc(ctx, sizeof(double) * (size_t)fch * N * N * N, &s2) : nullptr;
      double* d_Gm = d_X ? (double*)ctx_alloc(ctx, sizeof(double) * (size_t)fch * 3 * N * N, &s2) : nullptr;
      if (!d_Gm) {
        ctx_free(ctx, d_nrm); ctx_free(ctx, d_X);
        state_free(S);
        return s2;
      }
      e = hipMemcpyAsync(d_nrm, est_nrm.data(), sizeof(double) * est_nrm.size(), hipMemcpyHostToDevice, q);
      // the estimates of the first est_skip instances are copied in by the
      // caller (state_copy_instance)
      int f0 = st->est_off[std::min(est_skip, count)];
      while (f0 < n_est && e == hipSuccess) {
        const int cnt = std::min(fch, n_est - f0);
        // every instance of a state shares N; the velocity grid is per instance:
        // one launch covers consecutive faces on the same grid
        const InstParams& P0 = ip[est_inst[f0]];
        int cnt2 = 1;
        while (cnt2 < cnt && ip[est_inst[f0 + cnt2]].dxi == P0.dxi) ++cnt2;
        e = launch_absxi(N, cnt2, d_nrm + 3 * (size_t)f0, P0.xi_min, P0.dxi, d_X, q);
        if (e == hipSuccess) e = launch_gram(N, cnt2, d_X, 0, d_Gm, q);
        if (e == hipSuccess)
          e = launch_eig(N, cnt2, d_Gm, nullptr, nullptr, f0, 0.0, kEstCap, kEstCap, S->d_est_fac, S->d_est_rank,
                         nullptr, nullptr, nullptr, 1e-15, 1e-18, q, kEstDrop);
        if (e == hipSuccess)
          e = launch_project(N, cnt2, d_X, 0, f0, kEstCap, S->d_est_fac, S->d_est_rank, S->d_est_core, q);
        f0 += cnt2;
      }
      if (e == hipSuccess) e = hipStreamSynchronize(q);
      ctx_free(ctx, d_nrm); ctx_free(ctx, d_X); ctx_free(ctx, d_Gm);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(q);
  if (e != hipSuccess) { state_free(S); return ctx_hip(ctx, e, "state init"); }
  state_tune_begin(S);
  *out = st.release();
  return TK_OK;
}

// Key of the pass-size choice: states of one key run the same kernels on
// the same amount of work.
static std::string tune_key(const tk_state* st) {
  return std::to_string(st->N) + (st->mixed ? "m" : "d") + (st->oblique ? "o" : "a") + std::to_string(st->CS) +
         "/" + std::to_string(st->nc) + "/" + std::to_string(st->chunk_max);
}

// Candidate pass sizes: the allocated maximum, fixed sizes below it, and
// the size whose FP32/FP64 workspace fits 192 MiB (the expansion is then
// read back by the Gram and projection kernels from the 256 MiB last-level
// cache rather than HBM).
// Pass-size trials: ordinary steps first, so that the ranks (and with them
// the cost of every kernel) resemble a running state rather than the
// rank-1 start, then kTuneReps timed steps per candidate in cycles over the
// candidates, alternately in ascending and descending order, compared by
// their mean: step costs still drift as ranks grow, and the alternation
// gives every candidate the same mean position in the sequence.
constexpr int kTuneSkip = 16;
constexpr int kTuneReps = 4;

// candidate index of trial step t (nc candidates)
static int tune_index(int t, int nc) {
  const int cyc = t / nc, pos = t % nc;
  return (cyc & 1) ? nc - 1 - pos : pos;
}

static std::vector<int> chunk_candidates(const tk_state* st) {
  const size_t x = (size_t)st->N * st->N * st->N * (st->mixed ? 4 : 8);
  std::vector<int> c = {st->chunk_max, 16384, 12288, 8192, 6144, 4096, 2048,
                        (int)std::max<size_t>(256, (192u << 20) / x)};
  std::vector<int> out;
  for (int v : c)
    if (v <= st->chunk_max && v >= 256 && std::find(out.begin(), out.end(), v) == out.end()) out.push_back(v);
  std::sort(out.begin(), out.end());
  return out;
}

void state_tune_begin(tk_state* st) {
  st->tune = 0;
  if (st->plain) return;
  auto it = st->ctx->tuned_chunk.find(tune_key(st));
  if (it != st->ctx->tuned_chunk.end()) {
    st->chunk = it->second;
    return;
  }
  st->tune_cand = chunk_candidates(st);
  if (st->tune_cand.size() > 1) {
    st->tune = 1;
    st->tune_step = 0;
    st->tune_skip = kTuneSkip;
  }
}

static void tune_events_free(tk_state* st) {
  for (hipEvent_t e : st->tune_ev) (void)hipEventDestroy(e);
  st->tune_ev.clear();
}

// one explicit step of every instance of the state
static tk_status state_step_once(tk_state* st) {
  tk_ctx* ctx = st->ctx;
  hipStream_t q = ctx->stream;
  hipError_t e;
  hipEvent_t ev;
  if (st->plain) {
    DevPlain d = plain_dev(st);
    prof_begin(ctx, KID_PLAIN_MOM, &ev);
    e = launch_plain_moments(d, st->mixed, q);
    prof_end(ctx, KID_PLAIN_MOM, ev);
    if (e != hipSuccess) return ctx_hip(ctx, e, "plain moments");
    prof_begin(ctx, KID_PLAIN_STEP, &ev);
    e = launch_plain_step(d, st->mixed, q);
    prof_end(ctx, KID_PLAIN_STEP, ev);
    if (e != hipSuccess) return ctx_hip(ctx, e, "plain step");
    st->cur ^= 1;
    return TK_OK;
  }
  DevState d = state_dev(st);
  prof_begin(ctx, KID_MOMENTS, &ev);
  e = launch_moments(d, q);
  prof_end(ctx, KID_MOMENTS, ev);
  if (e != hipSuccess) return ctx_hip(ctx, e, "moments");
  // rounding in the space of the concatenated factors: the cells it leaves
  // (their concatenated ranks or core too large for its layouts) are listed
  // for the N-basis passes below; an eager step reads their count back, a
  // captured or served step runs passes over every cell that end at the
  // list's count
  int dense_n = st->nc;
  if (st->rspace) {
    prof_begin(ctx, KID_RROUND, &ev);
    e = launch_rround(d, st->d_rlistD, st->d_rcnt, st->d_wvalid, st->d_rstats, q);
    prof_end(ctx, KID_RROUND, ev);
    if (e != hipSuccess) return ctx_hip(ctx, e, "rounding in factor space");
    d.cells = st->d_rlistD;
    d.cells_n = st->d_rcnt;
    if (!st->capturing && !st->served) {
      e = hipMemcpyAsync(st->h_rcnt, st->d_rcnt, sizeof(int), hipMemcpyDeviceToHost, q);
      if (e == hipSuccess) e = hipStreamSynchronize(q);
      if (e != hipSuccess) return ctx_hip(ctx, e, "rounding list count");
      dense_n = *st->h_rcnt;
      st->dense_total += dense_n;
    }
  } else if (!st->capturing) {
    st->dense_total += st->nc;
  }
  // odd passes on the second stream with the second workspace: the passes
  // are independent (each reads the current state and writes its own cells
  // of the next one), and a stream reuses its workspace only after its
  // previous pass
  const bool dual = st->X2 && st->q2 && !st->capturing && !st->one_stream;
  if (dual) {
    e = hipEventRecord(st->ev_fork, q);
    if (e == hipSuccess) e = hipStreamWaitEvent(st->q2, st->ev_fork, 0);
    if (e != hipSuccess) return ctx_hip(ctx, e, "fork");
  }
  // on an error, order the second stream's work before later context-stream
  // work all the same
  auto fail = [&](const char* what) -> tk_status {
    if (dual && hipEventRecord(st->ev_join, st->q2) == hipSuccess) (void)hipStreamWaitEvent(q, st->ev_join, 0);
    return ctx_hip(ctx, e, what);
  };
  int pass = 0;
  for (int c0 = 0; c0 < dense_n; c0 += st->chunk, ++pass) {
    const int cnt = std::min(st->chunk, dense_n - c0);
    const bool two = dual && (pass & 1);
    hipStream_t sq = two ? st->q2 : q;
    void* X = two ? st->X2 : st->X;
    double* G = two ? st->G2 : st->G;
    double* Wb = two ? st->Wb2 : st->Wb;
    int* obl = two ? st->ob_list2 : st->ob_list;
    int* obn = two ? st->ob_n2 : st->ob_n;
    prof_begin(ctx, KID_EXPAND, &ev, sq);
    e = launch_expand(d, c0, cnt, X, st->mixed, st->oblique ? 1 : 0, obl, obn, sq);
    prof_end(ctx, KID_EXPAND, ev, sq);
    if (e != hipSuccess) return fail("expand");
    prof_begin(ctx, KID_GRAM, &ev, sq);
    e = launch_gram(st->N, cnt, X, st->mixed, G, sq, c0, d.cells_n);
    prof_end(ctx, KID_GRAM, ev, sq);
    if (e != hipSuccess) return fail("gram");
    prof_begin(ctx, KID_EIG, &ev, sq);
    if (st->mixed) {
      // warm start from the kept basis over the full matrix (no leading-block
      // shortcut: accepting a block whose complement carries up to 1e-3 of
      // the truncation budget moved the end-of-run macroparameters by 4e-4
      // against the FP64 path on the channel, against 4.6e-5 without it)
      e = launch_eig(st->N, cnt, G, st->d_inst, st->d_ip, c0, 0.0, 0, st->CS, d.fac_n, d.rank_n, nullptr,
                     nullptr, st->Wkeep, 1e-12, 1e-13, sq, 0.0, d.cells, d.cells_n, st->d_wvalid);
    } else {
      // FP64 path: first basis, Gram of the rotated unfoldings, final basis
      e = launch_eig(st->N, cnt, G, st->d_inst, st->d_ip, c0, 0.0, 0, st->CS, d.fac_n, d.rank_n, nullptr, Wb,
                     st->Wkeep, 1e-15, 1e-18, sq, 0.0, d.cells, d.cells_n, st->d_wvalid);
      if (e == hipSuccess) e = launch_gram_rot(st->N, cnt, X, 0, Wb, G, sq, c0, d.cells_n);
      if (e == hipSuccess)
        e = launch_eig(st->N, cnt, G, st->d_inst, st->d_ip, c0, 0.0, 0, st->CS, d.fac_n, d.rank_n, Wb, nullptr,
                       nullptr, 1e-15, 1e-18, sq, 0.0, d.cells, d.cells_n, nullptr);
    }
    prof_end(ctx, KID_EIG, ev, sq);
    if (e != hipSuccess) return fail("eig");
    prof_begin(ctx, KID_PROJECT, &ev, sq);
    e = launch_project(st->N, cnt, X, st->mixed, c0, st->CS, d.fac_n, d.rank_n, d.core_n, sq, d.cells, d.cells_n);
    prof_end(ctx, KID_PROJECT, ev, sq);
    if (e != hipSuccess) return fail("project");
  }
  if (dual) {
    e = hipEventRecord(st->ev_join, st->q2);
    if (e == hipSuccess) e = hipStreamWaitEvent(q, st->ev_join, 0);
    if (e != hipSuccess) return ctx_hip(ctx, e, "join");
  }
  st->cur ^= 1;
  st->warm = true;
  return TK_OK;
}

// A step replayed from the graph captured for the current buffer parity.
static tk_status state_step_graph(tk_state* st) {
  tk_ctx* ctx = st->ctx;
  hipStream_t q = ctx->stream;
  const int p = st->cur;
  hipError_t e = hipSuccess;
  if (!st->gexec[p] || st->gchunk[p] != st->chunk) {
    if (st->gexec[p]) (void)hipGraphExecDestroy(st->gexec[p]);
    st->gexec[p] = nullptr;
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return ctx_hip(ctx, e, "graph capture");
    st->capturing = true;  // one stream inside the graph
    const tk_status s = state_step_once(st);
    st->capturing = false;
    e = hipStreamEndCapture(q, &g);
    st->cur = p;
    if (s != TK_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&st->gexec[p], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) return ctx_hip(ctx, e, "graph instantiate");
    st->gchunk[p] = st->chunk;
  }
  e = hipGraphLaunch(st->gexec[p], q);
  if (e != hipSuccess) return ctx_hip(ctx, e, "graph launch");
  st->cur ^= 1;
  return TK_OK;
}

// One step: a timed trial while the pass size is being chosen, a graph
// replay when enabled, else eager launches.
// The step with intermediate roundings: per pass of cells, each face slot's
// flux term expanded and rounded into its buffer (tolerance and cap of the
// cell's instance), then the cell's own terms plus the rounded face terms
// expanded and rounded into the next state.  Every cell on the N-basis path,
// one stream; the FP64 path refines each basis with a second eigensolver pass.
static tk_status state_step_faces(tk_state* st) {
  tk_ctx* ctx = st->ctx;
  hipStream_t q = ctx->stream;
  hipEvent_t ev;
  hipError_t e;
  DevState d = state_dev(st);
  prof_begin(ctx, KID_MOMENTS, &ev);
  e = launch_moments(d, q);
  prof_end(ctx, KID_MOMENTS, ev);
  if (e != hipSuccess) return ctx_hip(ctx, e, "moments");
  const int nc = st->nc, N = st->N, CS = st->CS;
  const int mx = st->mixed ? 1 : 0;
  // face slot l's buffers
  auto fcore = [&](int l) { return st->d_face_core + (size_t)l * nc * CS * CS * CS; };
  auto ffac = [&](int l) { return st->d_face_fac + (size_t)l * nc * 3 * CS * N; };
  auto frank = [&](int l) { return st->d_face_rank + (size_t)l * nc * 3; };
  FaceStates fs;
  for (int l = 0; l < kSlots; ++l) {
    fs.core[l] = fcore(l);
    fs.fac[l] = ffac(l);
    fs.rank[l] = frank(l);
  }
  auto round_into = [&](int c0, int cnt, double* fac_o, int* rank_o, double* core_o) -> tk_status {
    prof_begin(ctx, KID_GRAM, &ev);
    e = launch_gram(N, cnt, st->X, mx, st->G, q);
    prof_end(ctx, KID_GRAM, ev);
    if (e != hipSuccess) return ctx_hip(ctx, e, "gram");
    prof_begin(ctx, KID_EIG, &ev);
    if (mx) {
      e = launch_eig(N, cnt, st->G, st->d_inst, st->d_ip, c0, 0.0, 0, CS, fac_o, rank_o, nullptr, nullptr, nullptr,
                     1e-12, 1e-13, q);
    } else {
      e = launch_eig(N, cnt, st->G, st->d_inst, st->d_ip, c0, 0.0, 0, CS, fac_o, rank_o, nullptr, st->Wb, nullptr,
                     1e-15, 1e-18, q);
      if (e == hipSuccess) e = launch_gram_rot(N, cnt, st->X, 0, st->Wb, st->G, q);
      if (e == hipSuccess)
        e = launch_eig(N, cnt, st->G, st->d_inst, st->d_ip, c0, 0.0, 0, CS, fac_o, rank_o, st->Wb, nullptr, nullptr,
                       1e-15, 1e-18, q);
    }
    prof_end(ctx, KID_EIG, ev);
    if (e != hipSuccess) return ctx_hip(ctx, e, "eig");
    prof_begin(ctx, KID_PROJECT, &ev);
    e = launch_project(N, cnt, st->X, mx, c0, CS, fac_o, rank_o, core_o, q);
    prof_end(ctx, KID_PROJECT, ev);
    return e == hipSuccess ? TK_OK : ctx_hip(ctx, e, "project");
  };
  tk_status s = TK_OK;
  for (int c0 = 0; c0 < nc && s == TK_OK; c0 += st->chunk) {
    const int cnt = std::min(st->chunk, nc - c0);
    for (int l = 0; l < kSlots && s == TK_OK; ++l) {
      prof_begin(ctx, KID_EXPAND, &ev);
      e = launch_face_term(d, c0, cnt, st->X, mx, l, q);
      prof_end(ctx, KID_EXPAND, ev);
      if (e != hipSuccess) return ctx_hip(ctx, e, "face term");
      s = round_into(c0, cnt, ffac(l), frank(l), fcore(l));
    }
    if (s != TK_OK) break;
    prof_begin(ctx, KID_EXPAND, &ev);
    e = launch_face_sum(d, fs, c0, cnt, st->X, mx, q);
    prof_end(ctx, KID_EXPAND, ev);
    if (e != hipSuccess) return ctx_hip(ctx, e, "face sum");
    s = round_into(c0, cnt, d.fac_n, d.rank_n, d.core_n);
  }
  if (s != TK_OK) return s;
  if (!st->capturing) st->dense_total += nc;
  st->cur ^= 1;
  return TK_OK;
}

static tk_status state_step(tk_state* st) {
  tk_ctx* ctx = st->ctx;
  if (st->face_round) return state_step_faces(st);
  if (st->tune == 1 && st->tune_skip > 0) {
    --st->tune_skip;
    return state_step_once(st);
  }
  if (st->tune == 1) {
    const int nc = (int)st->tune_cand.size();
    st->chunk = st->tune_cand[tune_index(st->tune_step, nc)];
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return ctx_fail(ctx, TK_EDEVICE, "event");
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return ctx_fail(ctx, TK_EDEVICE, "event");
    }
    st->tune_ev.push_back(a);
    st->tune_ev.push_back(b);
    (void)hipEventRecord(a, ctx->stream);
    const tk_status s = state_step_once(st);
    (void)hipEventRecord(b, ctx->stream);
    if (s != TK_OK) return s;
    if (++st->tune_step == kTuneReps * nc) {
      // the mean of the timings per candidate
      std::vector<float> best(nc, 0.f);
      hipError_t e = hipEventSynchronize(b);
      for (int k = 0; e == hipSuccess && k < kTuneReps * nc; ++k) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, st->tune_ev[2 * k], st->tune_ev[2 * k + 1]);
        best[tune_index(k, nc)] += ms;
      }
      tune_events_free(st);
      st->tune = 0;
      if (e != hipSuccess) return ctx_hip(ctx, e, "pass-size timing");
      const int i = (int)(std::min_element(best.begin(), best.end()) - best.begin());
      st->chunk = st->tune_cand[i];
      ctx->tuned_chunk[tune_key(st)] = st->chunk;
    }
    return TK_OK;
  }
  if (st->use_graph && st->warm && !ctx->prof && !st->plain) return state_step_graph(st);
  return state_step_once(st);
}

tk_status state_moments_now(tk_state* st) {
  hipError_t e;
  if (st->plain) e = launch_plain_moments(plain_dev(st), st->mixed, st->ctx->stream);
  else e = launch_moments(state_dev(st), st->ctx->stream);
  return ctx_hip(st->ctx, e, "moments");
}

// ---------------------------------------------------------------------------
// LU-SGS implicit iteration (eq. linear-system times dt, diagonal of eq.
// diagonal_term with the bound of eq. xin-one-rank-approx, divided in rank-1
// form as eq. one_rank_division): sweep order by a greedy colouring of the
// face graph (cells in index order, smallest colour no earlier neighbour
// has), so each colour is one set of passes of independent cells.

static tk_status lu_setup(tk_state* st) {
  tk_ctx* ctx = st->ctx;
  const int nc = st->nc, N = st->N, CS = st->CS;
  std::vector<std::vector<int>> nbrs(nc);
  for (int k = 0; k < st->ninst; ++k) {
    const tk_mesh* m = st->meshes[k];
    const int off = st->inst_off[k];
    for (int c = 0; c < m->n_cells; ++c)
      for (int s = 0; s < kSlots; ++s) {
        const size_t sl = (size_t)c * kSlots + s;
        if (m->slot_kind[sl] != SK_INTERIOR) continue;
        const int g = off + c, nb = off + m->slot_nb[sl];
        if (nb != g) nbrs[g].push_back(nb);
      }
  }
  std::vector<int> col(nc, -1);
  int ncol = 0;
  for (int i = 0; i < nc; ++i) {
    std::vector<char> taken(nbrs[i].size() + 1, 0);
    for (int m : nbrs[i])
      if (col[m] >= 0 && col[m] < (int)taken.size()) taken[col[m]] = 1;
    int c = 0;
    while (taken[c]) ++c;
    col[i] = c;
    ncol = std::max(ncol, c + 1);
  }
  std::vector<int> fw, bw;
  st->lu_off.assign(ncol + 1, 0);
  st->lu_boff.assign(ncol + 1, 0);
  std::vector<int> cnt(ncol, 0), bcnt(ncol, 0);
  for (int k = 0; k < ncol; ++k) {
    for (int i = 0; i < nc; ++i) {
      if (col[i] != k) continue;
      fw.push_back(i);
      bool later = false;
      for (int m : nbrs[i]) later = later || col[m] > k;
      if (later) bw.push_back(i);
    }
    st->lu_off[k + 1] = (int)fw.size();
    st->lu_boff[k + 1] = (int)bw.size();
    cnt[k] = st->lu_off[k + 1] - st->lu_off[k];
    bcnt[k] = st->lu_boff[k + 1] - st->lu_boff[k];
  }
  // (p, Q) of the mode-1 unfolding of |xi| per instance
  std::vector<double> pq((size_t)st->ninst * (N + N * N), 0.0);
  for (int k = 0; k < st->ninst; ++k) {
    const InstParams& P = st->ip_host[k];
    std::vector<double> S((size_t)N * N * N);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j)
        for (int l = 0; l < N; ++l) {
          const double x = P.xi_min + i * P.dxi, y = P.xi_min + j * P.dxi, z = P.xi_min + l * P.dxi;
          S[((size_t)i * N + j) * N + l] = std::sqrt(x * x + y * y + z * z);
        }
    double* p = pq.data() + (size_t)k * (N + N * N);
    double* Q = p + N;
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      for (int o = 0; o < N * N; ++o) s += S[(size_t)i * N * N + o];
      p[i] = s;
      for (int i2 = 0; i2 < N; ++i2) {
        double q = 0.0;
        for (int o = 0; o < N * N; ++o) q += S[(size_t)i * N * N + o] * S[(size_t)i2 * N * N + o];
        Q[i * N + i2] = q;
      }
    }
  }
  tk_status s = TK_OK;
  auto take = [&](size_t bytes) -> void* { return s == TK_OK ? st_alloc(st, std::max<size_t>(bytes, 4), &s) : nullptr; };
  st->d_lu_col = (int*)take(sizeof(int) * nc);
  st->d_lu_cells = (int*)take(sizeof(int) * nc);
  st->d_lu_bcells = (int*)take(sizeof(int) * bw.size());
  st->d_lu_cnt = (int*)take(sizeof(int) * ncol);
  st->d_lu_bcnt = (int*)take(sizeof(int) * ncol);
  st->d_df_core = (double*)take(sizeof(double) * (size_t)nc * CS * CS * CS);
  st->d_df_fac = (double*)take(sizeof(double) * (size_t)nc * 3 * CS * N);
  st->d_df_rank = (int*)take(sizeof(int) * (size_t)nc * 3);
  st->d_lu_dinv = (double*)take(sizeof(double) * (size_t)nc * (N + 1));
  st->d_lu_pq = (double*)take(sizeof(double) * pq.size());
  if (s != TK_OK) return s;
  hipError_t e = hipMemcpy(st->d_lu_col, col.data(), sizeof(int) * nc, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(st->d_lu_cells, fw.data(), sizeof(int) * nc, hipMemcpyHostToDevice);
  if (e == hipSuccess && !bw.empty())
    e = hipMemcpy(st->d_lu_bcells, bw.data(), sizeof(int) * bw.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(st->d_lu_cnt, cnt.data(), sizeof(int) * ncol, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(st->d_lu_bcnt, bcnt.data(), sizeof(int) * ncol, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(st->d_lu_pq, pq.data(), sizeof(double) * pq.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return ctx_hip(ctx, e, "LU-SGS set-up");
  st->lu_ready = true;
  return TK_OK;
}

// One LU-SGS iteration: moments, rank-1 diagonals, forward sweep (df* by
// colour, ascending), backward sweep (df by colour, descending, only cells
// with a later neighbour), commit f + df into the next buffers.  Every stage
// is an N-basis FP64 rounding of the stage's expanded tensor.
static tk_status state_lu_iteration(tk_state* st) {
  tk_ctx* ctx = st->ctx;
  hipStream_t q = ctx->stream;
  hipEvent_t ev;
  hipError_t e;
  DevState d = state_dev(st);
  prof_begin(ctx, KID_MOMENTS, &ev);
  e = launch_moments(d, q);
  prof_end(ctx, KID_MOMENTS, ev);
  if (e != hipSuccess) return ctx_hip(ctx, e, "moments");
  prof_begin(ctx, KID_LU, &ev);
  e = launch_lu_diag(d, st->d_lu_pq, st->d_lu_dinv, q);
  prof_end(ctx, KID_LU, ev);
  if (e != hipSuccess) return ctx_hip(ctx, e, "LU-SGS diagonal");
  LuArgs lu{st->d_df_core, st->d_df_fac, st->d_df_rank, st->d_lu_col, 0, st->d_lu_dinv};
  void* X = st->X;
  const int mx = st->mixed ? 1 : 0;
  // one stage over the listed cells (cells == nullptr: every cell), rounded
  // into (fac_o, rank_o, core_o): on the FP64 path two eigensolver passes
  // (first basis, Gram of the rotated unfoldings), on the mixed path one
  // pass over the FP32 stage tensor with its thresholds
  auto stage = [&](int kind, int count, const int* cells, const int* cells_n, double* fac_o, int* rank_o,
                   double* core_o) -> tk_status {
    DevState ds = d;
    ds.cells = cells;
    ds.cells_n = cells_n;
    for (int c0 = 0; c0 < count; c0 += st->chunk) {
      const int cnt = std::min(st->chunk, count - c0);
      prof_begin(ctx, KID_LU, &ev);
      e = launch_lu_expand(ds, lu, kind, c0, cnt, X, mx, q);
      prof_end(ctx, KID_LU, ev);
      if (e != hipSuccess) return ctx_hip(ctx, e, "LU-SGS stage");
      prof_begin(ctx, KID_GRAM, &ev);
      e = launch_gram(st->N, cnt, X, mx, st->G, q, c0, cells_n);
      prof_end(ctx, KID_GRAM, ev);
      if (e != hipSuccess) return ctx_hip(ctx, e, "gram");
      prof_begin(ctx, KID_EIG, &ev);
      if (mx) {
        e = launch_eig(st->N, cnt, st->G, st->d_inst, st->d_ip, c0, 0.0, 0, st->CS, fac_o, rank_o, nullptr, nullptr,
                       nullptr, 1e-12, 1e-13, q, 0.0, cells, cells_n, nullptr);
      } else {
        e = launch_eig(st->N, cnt, st->G, st->d_inst, st->d_ip, c0, 0.0, 0, st->CS, fac_o, rank_o, nullptr, st->Wb,
                       nullptr, 1e-15, 1e-18, q, 0.0, cells, cells_n, nullptr);
        if (e == hipSuccess) e = launch_gram_rot(st->N, cnt, X, 0, st->Wb, st->G, q, c0, cells_n);
        if (e == hipSuccess)
          e = launch_eig(st->N, cnt, st->G, st->d_inst, st->d_ip, c0, 0.0, 0, st->CS, fac_o, rank_o, st->Wb, nullptr,
                         nullptr, 1e-15, 1e-18, q, 0.0, cells, cells_n, nullptr);
      }
      prof_end(ctx, KID_EIG, ev);
      if (e != hipSuccess) return ctx_hip(ctx, e, "eig");
      prof_begin(ctx, KID_PROJECT, &ev);
      e = launch_project(st->N, cnt, X, mx, c0, st->CS, fac_o, rank_o, core_o, q, cells, cells_n);
      prof_end(ctx, KID_PROJECT, ev);
      if (e != hipSuccess) return ctx_hip(ctx, e, "project");
    }
    return TK_OK;
  };
  const int ncol = (int)st->lu_off.size() - 1;
  tk_status s = TK_OK;
  for (int k = 0; k < ncol && s == TK_OK; ++k) {
    lu.colour = k;
    s = stage(LU_FORWARD, st->lu_off[k + 1] - st->lu_off[k], st->d_lu_cells + st->lu_off[k], st->d_lu_cnt + k,
              st->d_df_fac, st->d_df_rank, st->d_df_core);
  }
  for (int k = ncol - 1; k >= 0 && s == TK_OK; --k) {
    lu.colour = k;
    s = stage(LU_BACKWARD, st->lu_boff[k + 1] - st->lu_boff[k], st->d_lu_bcells + st->lu_boff[k],
              st->d_lu_bcnt + k, st->d_df_fac, st->d_df_rank, st->d_df_core);
  }
  if (s == TK_OK) s = stage(LU_COMMIT, st->nc, nullptr, nullptr, d.fac_n, d.rank_n, d.core_n);
  if (s != TK_OK) return s;
  st->cur ^= 1;
  return TK_OK;
}

tk_status state_steps(tk_state* st, int nsteps, double* residual, bool wait, bool lusgs) {
  tk_ctx* ctx = st->ctx;
  hipStream_t q = ctx->stream;
  tk_status s;
  for (int k = 0; k < nsteps; ++k) {
    if (residual && k == nsteps - 1) {
      if ((s = state_moments_now(st)) != TK_OK) return s;
      hipError_t e = hipMemcpyAsync(st->d_macro_prev, st->d_macro, sizeof(double) * (size_t)st->nc * 8,
                                    hipMemcpyDeviceToDevice, q);
      if (e != hipSuccess) return ctx_hip(ctx, e, "macro copy");
    }
    if ((s = lusgs ? state_lu_iteration(st) : state_step(st)) != TK_OK) return s;
  }
  if (!wait) return TK_OK;
  if ((s = state_moments_now(st)) != TK_OK) return s;
  if (residual && nsteps > 0) {
    hipError_t e = launch_residual(st->d_macro_prev, st->d_macro, st->d_vol, st->d_inst_off, st->ninst, st->d_resid, q);
    if (e == hipSuccess)
      e = hipMemcpyAsync(residual, st->d_resid, sizeof(double) * st->ninst, hipMemcpyDeviceToHost, q);
    if (e != hipSuccess) return ctx_hip(ctx, e, "residual");
  }
  std::vector<int> flag(st->ninst, 0);
  hipError_t e = hipMemcpyAsync(flag.data(), st->d_flag, sizeof(int) * st->ninst, hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipStreamSynchronize(q);
  if (e != hipSuccess) return ctx_hip(ctx, e, "step sync");
  prof_harvest(ctx);
  for (int k = 0; k < st->ninst; ++k)
    if (flag[k] && !st->ip_host[k].frozen)
      return ctx_fail(ctx, TK_ENUMERIC, "a cell of instance " + std::to_string(k) + " has non-positive or non-finite n or T");
  return TK_OK;
}

// One step with the residuals and the numeric flags copied asynchronously to
// host memory (h_res[n_instances], h_flag[n_instances]); the caller
// synchronises the stream.
tk_status state_create_served(tk_ctx* ctx, int count, const tk_mesh* const* meshes, const tk_params* params,
                              const double* const* macros, tk_state** out, int est_skip) {
  if (!ctx) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  return state_create(ctx, count, meshes, params, macros, false, out, true, est_skip);
}

// Copies the current Tucker state of instance ks of src (its cells' cores,
// factors and ranks, the kept eigenbases with their validity, and the
// |xi . e| estimates of its oblique faces) over instance kd of dst: the same
// mesh and parameters, N, precision and layout (CS).  Enqueued on dst's
// context stream after src's pending work; dst then continues that instance
// exactly where src left it.
tk_status state_copy_instance(tk_state* dst, int kd, tk_state* src, int ks) {
  if (!dst || !src || kd < 0 || kd >= dst->ninst || ks < 0 || ks >= src->ninst || dst->plain || src->plain)
    return TK_EINVAL;
  const int n = src->inst_off[ks + 1] - src->inst_off[ks];
  if (n != dst->inst_off[kd + 1] - dst->inst_off[kd] || dst->N != src->N || dst->CS != src->CS ||
      dst->mixed != src->mixed)
    return ctx_fail(dst->ctx, TK_EINVAL, "copy instance: different shapes");
  const size_t a = (size_t)src->inst_off[ks], b = (size_t)dst->inst_off[kd];
  const size_t N = dst->N, CS = dst->CS;
  hipStream_t q = dst->ctx->stream;
  hipError_t e = hipStreamSynchronize(src->ctx->stream);
  auto cp = [&](void* d, const void* s, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(d, s, bytes, hipMemcpyDeviceToDevice, q);
  };
  cp(dst->core[dst->cur] + b * CS * CS * CS, src->core[src->cur] + a * CS * CS * CS, sizeof(double) * n * CS * CS * CS);
  cp(dst->fac[dst->cur] + b * 3 * CS * N, src->fac[src->cur] + a * 3 * CS * N, sizeof(double) * n * 3 * CS * N);
  cp(dst->rank[dst->cur] + b * 3, src->rank[src->cur] + a * 3, sizeof(int) * n * 3);
  cp(dst->Wkeep + b * 3 * N * N, src->Wkeep + a * 3 * N * N, sizeof(double) * n * 3 * N * N);
  cp(dst->d_wvalid + b * 3, src->d_wvalid + a * 3, sizeof(int) * n * 3);
  const int ne = src->est_off[ks + 1] - src->est_off[ks];
  if (ne != dst->est_off[kd + 1] - dst->est_off[kd]) return ctx_fail(dst->ctx, TK_EINVAL, "copy instance: faces differ");
  if (ne > 0) {
    const size_t ea = (size_t)src->est_off[ks], eb = (size_t)dst->est_off[kd];
    const size_t E3 = (size_t)kEstCap * kEstCap * kEstCap, EF = 3 * (size_t)kEstCap * N;
    cp(dst->d_est_core + eb * E3, src->d_est_core + ea * E3, sizeof(double) * ne * E3);
    cp(dst->d_est_fac + eb * EF, src->d_est_fac + ea * EF, sizeof(double) * ne * EF);
    cp(dst->d_est_rank + eb * 3, src->d_est_rank + ea * 3, sizeof(int) * ne * 3);
  }
  return ctx_hip(dst->ctx, e, "copy instance");
}

// Stops stepping instance k of a state from the next step on (enqueued on
// the context stream): moments and factor-space rounding skip its cells, so
// its macroparameters stay as they were.  The N-basis passes reach only the
// cells that factor-space rounding lists, so on states with that rounding no
// kernel reads or writes the instance's Tucker data any more.
tk_status state_freeze_instance(tk_state* st, int k) {
  if (!st || k < 0 || k >= st->ninst) return TK_EINVAL;
  st->ip_host[k].frozen = 1;
  const hipError_t e = hipMemcpyAsync(st->d_ip + k, &st->ip_host[k], sizeof(InstParams), hipMemcpyHostToDevice,
                                      st->ctx->stream);
  return ctx_hip(st->ctx, e, "freeze instance");
}

tk_status state_step_residual_async(tk_state* st, double* h_res, int* h_flag) {
  tk_ctx* ctx = st->ctx;
  hipStream_t q = ctx->stream;
  tk_status s;
  if ((s = state_moments_now(st)) != TK_OK) return s;
  hipError_t e = hipMemcpyAsync(st->d_macro_prev, st->d_macro, sizeof(double) * (size_t)st->nc * 8,
                                hipMemcpyDeviceToDevice, q);
  if (e != hipSuccess) return ctx_hip(ctx, e, "macro copy");
  if ((s = state_step(st)) != TK_OK) return s;
  if ((s = state_moments_now(st)) != TK_OK) return s;
  e = launch_residual(st->d_macro_prev, st->d_macro, st->d_vol, st->d_inst_off, st->ninst, st->d_resid, q);
  if (e == hipSuccess) e = hipMemcpyAsync(h_res, st->d_resid, sizeof(double) * st->ninst, hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipMemcpyAsync(h_flag, st->d_flag, sizeof(int) * st->ninst, hipMemcpyDeviceToHost, q);
  return ctx_hip(ctx, e, "residual");
}

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

tk_status tk_ctx_create(int32_t device, size_t hbm_budget, void* hip_stream, tk_ctx** out) {
  return tk_ctx_create_ex(device, hbm_budget, hip_stream, nullptr, out);
}

tk_status tk_ctx_create_ex(int32_t device, size_t hbm_budget, void* hip_stream, const tk_alloc_fns* alloc,
                           tk_ctx** out) {
  if (!out) return TK_EINVAL;
  if (alloc && (!alloc->alloc || !alloc->free)) return TK_EINVAL;
  *out = nullptr;
  if (device == -1) {
    // host-only context: mesh loading and validation, no device work
    std::unique_ptr<tk_ctx> c(new tk_ctx());
    c->device = -1;
    *out = c.release();
    return TK_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TK_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return TK_EDEVICE;
  std::unique_ptr<tk_ctx> c(new tk_ctx());
  c->device = device;
  size_t freeb = 0, total = 0;
  if (hipMemGetInfo(&freeb, &total) != hipSuccess) return TK_EDEVICE;
  c->budget = hbm_budget ? hbm_budget : (size_t)(0.9 * (double)freeb);
  if (scratch_lookup(device, &c->scratch) != hipSuccess) return TK_EDEVICE;
  if (alloc) c->alloc = *alloc;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
    c->own_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return TK_EDEVICE;
    c->own_stream = true;
  }
  *out = c.release();
  return TK_OK;
}

tk_status tk_ctx_destroy(tk_ctx* ctx) {
  if (!ctx) return TK_EINVAL;
  if (ctx->device < 0) {
    delete ctx;
    return TK_OK;
  }
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto& p : ctx->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return TK_OK;
}

const char* tk_last_error(const tk_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

tk_status tk_sync(tk_ctx* ctx) {
  if (!ctx) return TK_EINVAL;
  if (ctx->device < 0) return TK_OK;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  tk_status s = ctx_hip(ctx, hipStreamSynchronize(ctx->stream), "sync");
  prof_harvest(ctx);
  return s;
}

tk_status tk_prof_enable(tk_ctx* ctx, int32_t on) {
  if (!ctx) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  ctx->prof = on != 0;
  return TK_OK;
}

tk_status tk_prof_get(tk_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches) {
  if (!ctx || !kernel) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  prof_harvest(ctx);
  for (int k = 0; k < KID_COUNT; ++k)
    if (std::strcmp(kernel, kKernelNames[k]) == 0) {
      if (total_ms) *total_ms = ctx->prof_ms[k];
      if (launches) *launches = ctx->prof_n[k];
      return TK_OK;
    }
  return ctx_fail(ctx, TK_ENOTFOUND, std::string("unknown kernel family ") + kernel);
}

tk_status tk_prof_eig(tk_ctx* ctx, int64_t* out4, int32_t reset) {
  if (!ctx || !out4) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  if (ctx->device < 0) return ctx_fail(ctx, TK_EDEVICE, "host-only context");
  unsigned long long v[4];
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = eig_stats(v, reset != 0);
  if (e != hipSuccess) return ctx_hip(ctx, e, "eig stats");
  for (int i = 0; i < 4; ++i) out4[i] = (int64_t)v[i];
  return TK_OK;
}

tk_status tk_prof_reset(tk_ctx* ctx) {
  if (!ctx) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  prof_harvest(ctx);
  for (int k = 0; k < KID_COUNT; ++k) { ctx->prof_ms[k] = 0.0; ctx->prof_n[k] = 0; }
  return TK_OK;
}

tk_status tk_mesh_load(tk_ctx* ctx, const tk_mesh_desc* desc, tk_mesh** out) {
  if (!ctx || !out) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  *out = nullptr;
  std::unique_ptr<tk_mesh> m(new tk_mesh());
  m->ctx = ctx;
  tk_status s = mesh_build(ctx, desc, m.get());
  if (s != TK_OK) return s;
  *out = m.release();
  return TK_OK;
}

tk_status tk_mesh_destroy(tk_mesh* mesh) {
  if (!mesh) return TK_EINVAL;
  delete mesh;
  return TK_OK;
}

tk_status tk_state_init(tk_ctx* ctx, const tk_mesh* mesh, const tk_params* params, const double* macro,
                        tk_state** out) {
  if (!ctx) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  return state_create(ctx, 1, &mesh, params, &macro, false, out);
}

tk_status tk_state_init_batch(tk_ctx* ctx, int32_t count, const tk_mesh* const* meshes, const tk_params* params,
                              const double* const* macros, tk_state** out) {
  if (!ctx) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  return state_create(ctx, count, meshes, params, macros, false, out);
}

tk_status tk_plain_init(tk_ctx* ctx, const tk_mesh* mesh, const tk_params* params, const double* macro,
                        tk_state** out) {
  if (!ctx) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  return state_create(ctx, 1, &mesh, params, &macro, true, out);
}

tk_status tk_state_destroy(tk_state* st) {
  if (!st) return TK_EINVAL;
  tk_ctx* ctx = st->ctx;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  (void)hipStreamSynchronize(ctx->stream);
  state_free(st);
  delete st;
  return TK_OK;
}

tk_status tk_state_info(const tk_state* st, int32_t* n_cells, int32_t* n_instances) {
  if (!st) return TK_EINVAL;
  if (n_cells) *n_cells = st->nc;
  if (n_instances) *n_instances = st->ninst;
  return TK_OK;
}

tk_status tk_state_dt(const tk_state* st, int32_t inst, double* dt) {
  if (!st || !dt || inst < 0 || inst >= st->ninst) return TK_EINVAL;
  *dt = st->ip_host[inst].dt;
  return TK_OK;
}

// ---- checkpoints -------------------------------------------------------------
namespace {

struct CkptLayout {
  size_t ip, core, fac, rank, wkeep, wvalid, f, total;
};

CkptLayout ckpt_layout(const tk_state* st) {
  CkptLayout L{};
  size_t o = sizeof(CkptHeader);
  L.ip = o;
  o += sizeof(tk::InstParams) * st->ninst;
  const size_t nc = st->nc, N = st->N, CS = st->CS;
  if (st->plain) {
    L.f = o;
    o += nc * N * N * N * (st->mixed ? 4 : 8);
  } else {
    L.core = o;
    o += nc * CS * CS * CS * sizeof(double);
    L.fac = o;
    o += nc * 3 * CS * N * sizeof(double);
    L.rank = o;
    o += nc * 3 * sizeof(int);
    L.wkeep = o;
    o += nc * 3 * N * N * sizeof(double);
    L.wvalid = o;
    o += nc * 3 * sizeof(int);
  }
  L.total = o;
  return L;
}

}  // namespace

tk_status tk_state_checkpoint(tk_state* st, void* buf, size_t bytes, size_t* needed) {
  if (!st) return TK_EINVAL;
  tk_ctx* ctx = st->ctx;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  const CkptLayout L = ckpt_layout(st);
  if (needed) *needed = L.total;
  if (!buf) return TK_OK;
  if (bytes < L.total) return ctx_fail(ctx, TK_EINVAL, "checkpoint buffer too small");
  unsigned char* b = static_cast<unsigned char*>(buf);
  CkptHeader h{};
  std::memcpy(h.magic, "TKCKPT2", 8);
  h.N = st->N;
  h.CS = st->CS;
  h.nc = st->nc;
  h.ninst = st->ninst;
  h.mixed = st->mixed ? 1 : 0;
  h.plain = st->plain ? 1 : 0;
  h.warm = st->warm ? 1 : 0;
  std::memcpy(b, &h, sizeof(h));
  std::memcpy(b + L.ip, st->ip_host.data(), sizeof(tk::InstParams) * st->ninst);
  hipStream_t q = ctx->stream;
  const size_t nc = st->nc, N = st->N, CS = st->CS;
  hipError_t e = hipStreamSynchronize(q);
  if (st->plain) {
    if (e == hipSuccess) e = hipMemcpy(b + L.f, st->pf[st->cur], L.total - L.f, hipMemcpyDeviceToHost);
  } else {
    if (e == hipSuccess)
      e = hipMemcpy(b + L.core, st->core[st->cur], nc * CS * CS * CS * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
      e = hipMemcpy(b + L.fac, st->fac[st->cur], nc * 3 * CS * N * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(b + L.rank, st->rank[st->cur], nc * 3 * sizeof(int), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
      e = hipMemcpy(b + L.wkeep, st->Wkeep, nc * 3 * N * N * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(b + L.wvalid, st->d_wvalid, nc * 3 * sizeof(int), hipMemcpyDeviceToHost);
  }
  return ctx_hip(ctx, e, "checkpoint copy");
}

tk_status tk_state_restore(tk_state* st, const void* buf, size_t bytes) {
  if (!st || !buf) return TK_EINVAL;
  tk_ctx* ctx = st->ctx;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  const CkptLayout L = ckpt_layout(st);
  const unsigned char* b = static_cast<const unsigned char*>(buf);
  CkptHeader want{};
  want.N = st->N;
  want.CS = st->CS;
  want.nc = st->nc;
  want.ninst = st->ninst;
  want.mixed = st->mixed ? 1 : 0;
  want.plain = st->plain ? 1 : 0;
  std::string err;
  if (ckpt_check_header(buf, bytes, want, L.total, &err) != TK_OK) return ctx_fail(ctx, TK_EINVAL, err);
  std::vector<tk::InstParams> ip(st->ninst);
  std::memcpy(ip.data(), b + L.ip, sizeof(tk::InstParams) * st->ninst);
  for (int k = 0; k < st->ninst; ++k)
    if (ip[k].cap != st->ip_host[k].cap || ip[k].dxi != st->ip_host[k].dxi || ip[k].xi_min != st->ip_host[k].xi_min)
      return ctx_fail(ctx, TK_EINVAL, "restore: checkpoint of different instance parameters");
  hipStream_t q = ctx->stream;
  const size_t nc = st->nc, N = st->N, CS = st->CS;
  // ranks index the factor and core layouts in every kernel: a buffer with
  // ranks outside 1..CS is refused before anything reaches the device
  std::vector<int> rk;
  if (!st->plain) {
    rk.resize(nc * 3);
    std::memcpy(rk.data(), b + L.rank, nc * 3 * sizeof(int));
    if (ckpt_check_ranks(rk.data(), rk.size(), st->CS, &err) != TK_OK) return ctx_fail(ctx, TK_EINVAL, err);
  }
  hipError_t e = hipStreamSynchronize(q);
  if (e == hipSuccess) e = hipMemcpy(st->d_ip, ip.data(), sizeof(tk::InstParams) * st->ninst, hipMemcpyHostToDevice);
  if (st->plain) {
    if (e == hipSuccess) e = hipMemcpy(st->pf[st->cur], b + L.f, L.total - L.f, hipMemcpyHostToDevice);
  } else {
    if (e == hipSuccess)
      e = hipMemcpy(st->core[st->cur], b + L.core, nc * CS * CS * CS * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(st->fac[st->cur], b + L.fac, nc * 3 * CS * N * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(st->rank[st->cur], rk.data(), nc * 3 * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(st->Wkeep, b + L.wkeep, nc * 3 * N * N * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(st->d_wvalid, b + L.wvalid, nc * 3 * sizeof(int), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return ctx_hip(ctx, e, "restore copy");
  // the face coefficients dt A / V carry the checkpoint's dt
  bool same_dt = true;
  for (int k = 0; k < st->ninst; ++k) same_dt = same_dt && ip[k].dt == st->ip_host[k].dt;
  if (!same_dt) {
    std::vector<double> coef((size_t)st->nc * kSlots);
    for (int k = 0; k < st->ninst; ++k) {
      const tk_mesh* m = st->meshes[k];
      const double dt = ip[k].dt;
      for (int c = 0; c < m->n_cells; ++c)
        for (int sl = 0; sl < kSlots; ++sl) {
          const size_t src = (size_t)c * kSlots + sl, dst = ((size_t)st->inst_off[k] + c) * kSlots + sl;
          coef[dst] = dt * m->slot_area[src] / m->volume[c];
        }
    }
    e = hipMemcpy(st->d_slot_coef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return ctx_hip(ctx, e, "restore face coefficients");
  }
  st->ip_host = ip;
  CkptHeader h;
  std::memcpy(&h, b, sizeof(h));
  st->warm = h.warm != 0;
  return TK_OK;
}

tk_status tk_state_set_chunk(tk_state* st, int32_t cells) {
  if (!st) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(st->ctx->mu);
  if (cells < 0 || cells > st->chunk_max)
    return ctx_fail(st->ctx, TK_EINVAL, "pass size must be 0 (choose) or 1.." + std::to_string(st->chunk_max));
  tune_events_free(st);
  if (cells == 0) {
    state_tune_begin(st);
  } else {
    st->tune = 0;
    st->chunk = cells;
  }
  return TK_OK;
}

tk_status tk_state_chunk(const tk_state* st, int32_t* cells, int32_t* max_cells) {
  if (!st) return TK_EINVAL;
  if (cells) *cells = st->chunk;
  if (max_cells) *max_cells = st->chunk_max;
  return TK_OK;
}

tk_status tk_state_tune(tk_state* st, int32_t* steps_run) {
  if (!st) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(st->ctx->mu);
  int n = 0;
  if (steps_run) *steps_run = 0;
  while (st->tune == 1 && n < 256) {
    const tk_status s = state_step(st);
    if (s != TK_OK) return s;
    ++n;
    if (steps_run) *steps_run = n;
  }
  return ctx_hip(st->ctx, hipStreamSynchronize(st->ctx->stream), "tune sync");
}

tk_status tk_state_use_graph(tk_state* st, int32_t on) {
  if (!st) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(st->ctx->mu);
  st->use_graph = on != 0;
  return TK_OK;
}

tk_status tk_state_streams(tk_state* st, int32_t two, int32_t* available) {
  if (!st) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(st->ctx->mu);
  const bool have = st->X2 && st->q2;
  if (available) *available = have ? 1 : 0;
  if (two >= 0) st->one_stream = two == 0;
  return TK_OK;
}

tk_status tk_state_rounding(tk_state* st, int32_t factor_space, int64_t* counts) {
  if (!st) return TK_EINVAL;
  tk_ctx* ctx = st->ctx;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  if (factor_space > 0 && !st->rspace_ok)
    return ctx_fail(ctx, TK_EINVAL, "rounding in factor space needs N <= 32 and a Tucker state");
  if (factor_space >= 0) {
    st->rspace = factor_space > 0;
    // the graphs captured for the other path
    for (int p = 0; p < 2; ++p) {
      if (st->gexec[p]) (void)hipGraphExecDestroy(st->gexec[p]);
      st->gexec[p] = nullptr;
    }
  }
  if (counts) {
    for (int i = 0; i < 4; ++i) counts[i] = 0;
    if (st->d_rstats) {
      unsigned long long v[8];
      hipError_t e = hipStreamSynchronize(ctx->stream);
      if (e == hipSuccess) e = hipMemcpy(v, st->d_rstats, sizeof(v), hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemset(st->d_rstats, 0, sizeof(v));
      if (e != hipSuccess) return ctx_hip(ctx, e, "rounding counters");
      counts[0] = (int64_t)v[0];
      counts[2] = (int64_t)v[2];
      counts[3] = (int64_t)v[1];
    }
    counts[1] = st->dense_total;
    st->dense_total = 0;
  }
  return TK_OK;
}

tk_status tk_moments(tk_state* st, double* out) {
  if (!st || !out) return TK_EINVAL;
  tk_ctx* ctx = st->ctx;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  tk_status s = state_moments_now(st);
  if (s != TK_OK) return s;
  hipError_t e = hipMemcpyAsync(out, st->d_macro, sizeof(double) * (size_t)st->nc * 8, hipMemcpyDeviceToHost,
                                ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return ctx_hip(ctx, e, "moments copy");
}

tk_status tk_step(tk_state* st, int32_t nsteps, double* residual) {
  if (!st || nsteps < 0) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(st->ctx->mu);
  return state_steps(st, nsteps, residual, true);
}

tk_status tk_lusgs(tk_state* st, int32_t iters, double* residual) {
  if (!st || iters < 0) return TK_EINVAL;
  tk_ctx* ctx = st->ctx;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  if (st->plain || st->oblique || st->N > 32)
    return ctx_fail(ctx, TK_EINVAL, "LU-SGS runs on Tucker states with N <= 32 and axis-aligned faces");
  if (!st->lu_ready) {
    const tk_status s = lu_setup(st);
    if (s != TK_OK) return s;
  }
  return state_steps(st, iters, residual, true, true);
}

tk_status tk_state_face_rounding(tk_state* st, int32_t on) {
  if (!st) return TK_EINVAL;
  tk_ctx* ctx = st->ctx;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  if (st->plain || st->served)
    return ctx_fail(ctx, TK_EINVAL, "intermediate rounding runs on Tucker states outside a server");
  if (on && !st->d_face_core) {
    const size_t nc = st->nc, CS = st->CS, N = st->N;
    tk_status s = TK_OK;
    double* core = (double*)st_alloc(st, sizeof(double) * kSlots * nc * CS * CS * CS, &s);
    double* fac = s == TK_OK ? (double*)st_alloc(st, sizeof(double) * kSlots * nc * 3 * CS * N, &s) : nullptr;
    int* rank = s == TK_OK ? (int*)st_alloc(st, sizeof(int) * kSlots * nc * 3, &s) : nullptr;
    if (s != TK_OK) return s;
    st->d_face_core = core;
    st->d_face_fac = fac;
    st->d_face_rank = rank;
  }
  st->face_round = on != 0;
  return TK_OK;
}

tk_status tk_step_async(tk_state* st, int32_t nsteps) {
  if (!st || nsteps < 0) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(st->ctx->mu);
  return state_steps(st, nsteps, nullptr, false);
}

tk_status tk_state_ranks(tk_state* st, int32_t* ranks, double* mean_compression) {
  if (!st) return TK_EINVAL;
  tk_ctx* ctx = st->ctx;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  if (st->plain) return ctx_fail(ctx, TK_EINVAL, "plain state has no ranks");
  std::vector<int> r((size_t)st->nc * 3);
  hipError_t e = hipMemcpyAsync(r.data(), st->rank[st->cur], sizeof(int) * r.size(), hipMemcpyDeviceToHost,
                                ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return ctx_hip(ctx, e, "ranks copy");
  if (ranks) std::memcpy(ranks, r.data(), sizeof(int) * r.size());
  if (mean_compression) {
    const double N = st->N;
    double acc = 0.0;
    for (int c = 0; c < st->nc; ++c) {
      const double r1 = r[3 * c], r2 = r[3 * c + 1], r3 = r[3 * c + 2];
      acc += (r1 * r2 * r3 + N * (r1 + r2 + r3)) / (N * N * N);
    }
    *mean_compression = acc / st->nc;
  }
  return TK_OK;
}

tk_status tk_state_export(tk_state* st, int32_t cell, tk_tucker* out) {
  if (!st || !out || cell < 0 || cell >= st->nc || !out->core) return TK_EINVAL;
  tk_ctx* ctx = st->ctx;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  if (st->plain) return ctx_fail(ctx, TK_EINVAL, "plain state has no Tucker form");
  const int N = st->N, CS = st->CS;
  std::vector<double> core((size_t)CS * CS * CS), fac((size_t)3 * CS * N);
  int r[3];
  hipStream_t q = ctx->stream;
  hipError_t e = hipMemcpyAsync(r, st->rank[st->cur] + 3 * (size_t)cell, sizeof(r), hipMemcpyDeviceToHost, q);
  if (e == hipSuccess)
    e = hipMemcpyAsync(core.data(), st->core[st->cur] + (size_t)cell * CS * CS * CS, sizeof(double) * core.size(),
                       hipMemcpyDeviceToHost, q);
  if (e == hipSuccess)
    e = hipMemcpyAsync(fac.data(), st->fac[st->cur] + (size_t)cell * 3 * CS * N, sizeof(double) * fac.size(),
                       hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipStreamSynchronize(q);
  if (e != hipSuccess) return ctx_hip(ctx, e, "export copy");
  out->N = N;
  for (int a = 0; a < 3; ++a) out->r[a] = r[a];
  for (int k3 = 0; k3 < r[2]; ++k3)
    for (int k2 = 0; k2 < r[1]; ++k2)
      for (int k1 = 0; k1 < r[0]; ++k1)
        out->core[k1 + r[0] * (k2 + r[1] * k3)] = core[k1 + CS * (k2 + CS * k3)];
  for (int a = 0; a < 3; ++a) {
    if (!out->U[a]) return ctx_fail(ctx, TK_EINVAL, "export: null factor buffer");
    for (int k = 0; k < r[a]; ++k)
      for (int i = 0; i < N; ++i) out->U[a][i + N * k] = fac[((size_t)a * CS + k) * N + i];
  }
  return TK_OK;
}

tk_status tk_round_tucker(tk_ctx* ctx, int32_t count, const tk_tucker* in, double tol, int32_t cap,
                          tk_tucker* out) {
  if (!ctx || count < 0 || (count > 0 && (!in || !out))) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  if (count == 0) return TK_OK;
  if (ctx->device < 0) return ctx_fail(ctx, TK_EDEVICE, "round: host-only context");
  const int N = in[0].N;
  bool okN = false;
  for (int n : kSupportedN) okN |= (N == n && n <= 32);
  if (!okN) return ctx_fail(ctx, TK_EINVAL, "round: N must be 16, 24 or 32");
  if (cap < 1 || cap > kMaxCap || cap > N || !(tol >= 0)) return ctx_fail(ctx, TK_EINVAL, "round: bad tol or cap");
  int CSi = 1;
  for (int k = 0; k < count; ++k) {
    if (in[k].N != N) return ctx_fail(ctx, TK_EINVAL, "round: all tensors share N");
    for (int a = 0; a < 3; ++a) {
      if (in[k].r[a] < 1 || in[k].r[a] > N) return ctx_fail(ctx, TK_EINVAL, "round: a rank exceeds N");
      if (in[k].r[a] > kMaxCap) return ctx_fail(ctx, TK_EINVAL, "round: input ranks above 16 are not supported");
      CSi = std::max(CSi, in[k].r[a]);
    }
  }
  const int CSo = cap;
  std::vector<double> core((size_t)count * CSi * CSi * CSi, 0.0), fac((size_t)count * 3 * CSi * N, 0.0);
  std::vector<int> rk((size_t)count * 3);
  for (int k = 0; k < count; ++k) {
    const tk_tucker& t = in[k];
    for (int a = 0; a < 3; ++a) rk[3 * k + a] = t.r[a];
    for (int k3 = 0; k3 < t.r[2]; ++k3)
      for (int k2 = 0; k2 < t.r[1]; ++k2)
        for (int k1 = 0; k1 < t.r[0]; ++k1)
          core[(size_t)k * CSi * CSi * CSi + k1 + CSi * (k2 + CSi * k3)] = t.core[k1 + t.r[0] * (k2 + t.r[1] * k3)];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < t.r[a]; ++c)
        for (int i = 0; i < N; ++i) fac[(((size_t)k * 3 + a) * CSi + c) * N + i] = t.U[a][i + N * c];
  }
  tk_status s = TK_OK;
  std::vector<void*> mem;
  auto A = [&](size_t b) -> void* {
    void* p = ctx_alloc(ctx, b, &s);
    if (p) mem.push_back(p);
    return p;
  };
  double* d_core = (double*)A(sizeof(double) * core.size());
  double* d_fac = d_core ? (double*)A(sizeof(double) * fac.size()) : nullptr;
  int* d_rk = d_fac ? (int*)A(sizeof(int) * rk.size()) : nullptr;
  double* d_X = d_rk ? (double*)A(sizeof(double) * (size_t)count * N * N * N) : nullptr;
  double* d_G = d_X ? (double*)A(sizeof(double) * (size_t)count * 3 * N * N) : nullptr;
  double* d_fo = d_G ? (double*)A(sizeof(double) * (size_t)count * 3 * CSo * N) : nullptr;
  int* d_ro = d_fo ? (int*)A(sizeof(int) * (size_t)count * 3) : nullptr;
  double* d_co = d_ro ? (double*)A(sizeof(double) * (size_t)count * CSo * CSo * CSo) : nullptr;
  double* d_W = d_co ? (double*)A(sizeof(double) * (size_t)count * 3 * N * N) : nullptr;
  auto cleanup = [&]() { for (void* p : mem) ctx_free(ctx, p); };
  if (!d_W) { cleanup(); return s; }
  hipStream_t q = ctx->stream;
  hipError_t e = hipMemcpyAsync(d_core, core.data(), sizeof(double) * core.size(), hipMemcpyHostToDevice, q);
  if (e == hipSuccess) e = hipMemcpyAsync(d_fac, fac.data(), sizeof(double) * fac.size(), hipMemcpyHostToDevice, q);
  if (e == hipSuccess) e = hipMemcpyAsync(d_rk, rk.data(), sizeof(int) * rk.size(), hipMemcpyHostToDevice, q);
  if (e == hipSuccess) e = launch_expand_plain(N, count, CSi, d_core, d_fac, d_rk, d_X, q);
  if (e == hipSuccess) e = launch_gram(N, count, d_X, 0, d_G, q);
  if (e == hipSuccess) e = launch_eig(N, count, d_G, nullptr, nullptr, 0, tol, cap, CSo, d_fo, d_ro, nullptr, d_W, nullptr, 1e-15, 1e-18, q);
  if (e == hipSuccess) e = launch_gram_rot(N, count, d_X, 0, d_W, d_G, q);
  if (e == hipSuccess) e = launch_eig(N, count, d_G, nullptr, nullptr, 0, tol, cap, CSo, d_fo, d_ro, d_W, nullptr, nullptr, 1e-15, 1e-18, q);
  if (e == hipSuccess) e = launch_project(N, count, d_X, 0, 0, CSo, d_fo, d_ro, d_co, q);
  std::vector<double> co((size_t)count * CSo * CSo * CSo), fo((size_t)count * 3 * CSo * N);
  std::vector<int> ro((size_t)count * 3);
  if (e == hipSuccess) e = hipMemcpyAsync(co.data(), d_co, sizeof(double) * co.size(), hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipMemcpyAsync(fo.data(), d_fo, sizeof(double) * fo.size(), hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipMemcpyAsync(ro.data(), d_ro, sizeof(int) * ro.size(), hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipStreamSynchronize(q);
  cleanup();
  if (e != hipSuccess) return ctx_hip(ctx, e, "round");
  for (int k = 0; k < count; ++k) {
    tk_tucker& t = out[k];
    if (!t.core || !t.U[0] || !t.U[1] || !t.U[2]) return ctx_fail(ctx, TK_EINVAL, "round: null output buffer");
    t.N = N;
    for (int a = 0; a < 3; ++a) t.r[a] = ro[3 * k + a];
    for (int k3 = 0; k3 < t.r[2]; ++k3)
      for (int k2 = 0; k2 < t.r[1]; ++k2)
        for (int k1 = 0; k1 < t.r[0]; ++k1)
          t.core[k1 + t.r[0] * (k2 + t.r[1] * k3)] = co[(size_t)k * CSo * CSo * CSo + k1 + CSo * (k2 + CSo * k3)];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < t.r[a]; ++c)
        for (int i = 0; i < N; ++i) t.U[a][i + N * c] = fo[(((size_t)k * 3 + a) * CSo + c) * N + i];
  }
  return TK_OK;
}

tk_status tk_round(tk_state* st, double tol, int32_t cap) {
  if (!st) return TK_EINVAL;
  tk_ctx* ctx = st->ctx;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  if (st->plain) return ctx_fail(ctx, TK_EINVAL, "round: a plain state has no Tucker form");
  const int N = st->N, CS = st->CS;
  if (N > 32) return ctx_fail(ctx, TK_EINVAL, "round: N must be 16, 24 or 32");
  if (!(tol >= 0) || cap < 1 || cap > CS) return ctx_fail(ctx, TK_EINVAL, "round: tol must be >= 0 and cap in 1..the storage cap");
  // passes of cells whose FP64 work space (N^3 tensor, three Grams, three
  // first-pass bases) fits half of what the budget leaves, at most 4096
  const size_t nn = (size_t)N * N;
  const size_t per = sizeof(double) * (nn * N + 6 * nn);
  const size_t avail = ctx->budget > ctx->used ? ctx->budget - ctx->used : 0;
  const int pass = (int)std::min<size_t>({(size_t)st->nc, avail / 2 / per, (size_t)4096});
  if (pass < 1) return ctx_fail(ctx, TK_ENOMEM, "round: no room for the work space");
  tk_status s = TK_OK;
  double* X = (double*)ctx_alloc(ctx, (size_t)pass * nn * N * sizeof(double), &s);
  double* G = X ? (double*)ctx_alloc(ctx, (size_t)pass * 3 * nn * sizeof(double), &s) : nullptr;
  double* W = G ? (double*)ctx_alloc(ctx, (size_t)pass * 3 * nn * sizeof(double), &s) : nullptr;
  if (!W) {
    ctx_free(ctx, X);
    ctx_free(ctx, G);
    return s;
  }
  hipStream_t q = ctx->stream;
  const double* core = st->core[st->cur];
  const double* fac = st->fac[st->cur];
  const int* rank = st->rank[st->cur];
  double* core_n = st->core[st->cur ^ 1];
  double* fac_n = st->fac[st->cur ^ 1];
  int* rank_n = st->rank[st->cur ^ 1];
  const size_t c3 = (size_t)CS * CS * CS, cf = (size_t)3 * CS * N;
  hipError_t e = hipSuccess;
  for (int c0 = 0; c0 < st->nc && e == hipSuccess; c0 += pass) {
    const int n = std::min(pass, st->nc - c0);
    e = launch_expand_plain(N, n, CS, core + c0 * c3, fac + c0 * cf, rank + 3 * (size_t)c0, X, q);
    if (e == hipSuccess) e = launch_gram(N, n, X, 0, G, q);
    if (e == hipSuccess)
      e = launch_eig(N, n, G, nullptr, nullptr, 0, tol, cap, CS, fac_n + c0 * cf, rank_n + 3 * (size_t)c0, nullptr,
                     W, nullptr, 1e-15, 1e-18, q);
    if (e == hipSuccess) e = launch_gram_rot(N, n, X, 0, W, G, q);
    if (e == hipSuccess)
      e = launch_eig(N, n, G, nullptr, nullptr, 0, tol, cap, CS, fac_n + c0 * cf, rank_n + 3 * (size_t)c0, W,
                     nullptr, nullptr, 1e-15, 1e-18, q);
    if (e == hipSuccess) e = launch_project(N, n, X, 0, 0, CS, fac_n + c0 * cf, rank_n + 3 * (size_t)c0, core_n + c0 * c3, q);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(q);
  ctx_free(ctx, X);
  ctx_free(ctx, G);
  ctx_free(ctx, W);
  if (e != hipSuccess) return ctx_hip(ctx, e, "round");
  st->cur ^= 1;
  return TK_OK;
}

tk_status tk_round_tucker_noalloc(tk_ctx* ctx, int32_t N, int32_t count, int32_t in_cap, const double* core_in,
                                  const double* fac_in, const int32_t* rank_in, double tol, int32_t cap,
                                  double* core_out, double* fac_out, int32_t* rank_out) {
  if (!ctx || count < 0) return TK_EINVAL;
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  if (ctx->device < 0) return ctx_fail(ctx, TK_EDEVICE, "round (no allocation): host-only context");
  if (!ctx->scratch) return ctx_fail(ctx, TK_EDEVICE, "round (no allocation): scratch array not set up");
  if (N != 16 && N != 24 && N != 32) return ctx_fail(ctx, TK_EINVAL, "round (no allocation): N must be 16, 24 or 32");
  if (in_cap < 1 || in_cap > kMaxCap || in_cap > N)
    return ctx_fail(ctx, TK_EINVAL, "round (no allocation): in_cap must be in 1..16 and <= N");
  if (cap < 1 || cap > kMaxCap || cap > N || !(tol >= 0))
    return ctx_fail(ctx, TK_EINVAL, "round (no allocation): bad tol or cap");
  if (count == 0) return TK_OK;
  if (!core_in || !fac_in || !rank_in || !core_out || !fac_out || !rank_out)
    return ctx_fail(ctx, TK_EINVAL, "round (no allocation): null buffer");
  // per tensor: the expanded N^3 tensor, three Grams and three first-pass bases
  const size_t nn = (size_t)N * N;
  const size_t per = sizeof(double) * (nn * N + 6 * nn);
  const int pass = (int)std::min<size_t>((size_t)count, kScratchBytes / per);
  if (pass < 1) return ctx_fail(ctx, TK_EINVAL, "round (no allocation): one tensor exceeds the scratch array");
  double* X = static_cast<double*>(ctx->scratch);
  double* G = X + (size_t)pass * nn * N;
  double* W = G + (size_t)pass * 3 * nn;
  const size_t ci = (size_t)in_cap * in_cap * in_cap, co = (size_t)cap * cap * cap;
  hipStream_t q = ctx->stream;
  hipError_t e = hipSuccess;
  for (int p0 = 0; p0 < count && e == hipSuccess; p0 += pass) {
    const int n = std::min(pass, count - p0);
    double* fo = fac_out + (size_t)p0 * 3 * cap * N;
    int* ro = rank_out + 3 * (size_t)p0;
    e = launch_expand_plain(N, n, in_cap, core_in + (size_t)p0 * ci, fac_in + (size_t)p0 * 3 * in_cap * N,
                            rank_in + 3 * (size_t)p0, X, q);
    if (e == hipSuccess) e = launch_gram(N, n, X, 0, G, q);
    if (e == hipSuccess)
      e = launch_eig(N, n, G, nullptr, nullptr, 0, tol, cap, cap, fo, ro, nullptr, W, nullptr, 1e-15, 1e-18, q);
    if (e == hipSuccess) e = launch_gram_rot(N, n, X, 0, W, G, q);
    if (e == hipSuccess)
      e = launch_eig(N, n, G, nullptr, nullptr, 0, tol, cap, cap, fo, ro, W, nullptr, nullptr, 1e-15, 1e-18, q);
    if (e == hipSuccess) e = launch_project(N, n, X, 0, 0, cap, fo, ro, core_out + (size_t)p0 * co, q);
  }
  return ctx_hip(ctx, e, "round (no allocation)");
}

}  // extern "C"
