// Host-side objects behind the opaque handles of tk.h.
#pragma once

#include <string>
#include <vector>

#include "tk_internal.h"

struct tk_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0;
  size_t used = 0;
  std::map<void*, size_t> sizes;
  // device memory from the caller's allocator (alloc.alloc == nullptr: hipMalloc)
  tk_alloc_fns alloc = {nullptr, nullptr, nullptr};
  // device address of this device's copy of the no-allocation rounding
  // scratch array (runtime.hip), looked up once per device at context set-up
  void* scratch = nullptr;
  std::string err;
  std::recursive_mutex mu;
  // per-kernel-family timing
  bool prof = false;
  struct Pending {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[tk::KID_COUNT] = {};
  int64_t prof_n[tk::KID_COUNT] = {};
  // rounding-pass sizes chosen by timing, per state shape
  std::map<std::string, int> tuned_chunk;
};

struct tk_state {
  tk_ctx* ctx = nullptr;
  int N = 0, CS = 0;
  bool mixed = false, plain = false;
  int nc = 0, ninst = 0;
  int chunk = 1;      // cells per rounding pass in use
  int chunk_max = 1;  // allocated
  // pass-size tuning: 0 fixed, 1 tuning; the trial steps and their events
  int tune = 0;
  int tune_step = 0;
  int tune_skip = 0;  // untimed steps left before the trials
  std::vector<int> tune_cand;
  std::vector<hipEvent_t> tune_ev;
  // graph replay of a step, one graph per buffer parity
  bool use_graph = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int gchunk[2] = {0, 0};
  std::vector<tk_params> params;
  std::vector<const tk_mesh*> meshes;
  std::vector<int> inst_off;
  std::vector<int> est_off;  // first |xi . e| estimate of each instance (oblique faces, instance order)
  std::vector<tk::InstParams> ip_host;
  std::vector<void*> allocs;
  // device tables
  int* d_inst = nullptr;
  tk::InstParams* d_ip = nullptr;
  int* d_slot_nb = nullptr;
  int8_t* d_slot_kind = nullptr;
  int8_t* d_slot_axis = nullptr;
  int8_t* d_slot_sig = nullptr;
  double* d_slot_coef = nullptr;
  double* d_bc_fac = nullptr;
  double* d_vol = nullptr;
  int* d_inst_off = nullptr;
  double* d_macro = nullptr;
  double* d_macro_prev = nullptr;
  double* d_macro5 = nullptr;
  double* d_nu = nullptr;
  double* d_nw = nullptr;
  int* d_flag = nullptr;
  double* d_resid = nullptr;
  // Tucker state, double buffered
  double* core[2] = {nullptr, nullptr};
  double* fac[2] = {nullptr, nullptr};
  int* rank[2] = {nullptr, nullptr};
  int cur = 0;
  // rounding workspaces
  void* X = nullptr;
  double* G = nullptr;
  int* ob_list = nullptr;  // [2][chunk] cells of a pass left to later expansion launches
  int* ob_n = nullptr;     // [2] their counts
  // second workspace and stream: odd passes of a step run there, so one
  // pass's eigensolves overlap the next pass's expansion (allocated only
  // when the budget leaves room; not used while timing kernels or capturing)
  void* X2 = nullptr;
  double* G2 = nullptr;
  double* Wb2 = nullptr;
  int* ob_list2 = nullptr;
  int* ob_n2 = nullptr;
  hipStream_t q2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool capturing = false;
  bool one_stream = false;  // tk_state_streams(st, 0): all passes on the context stream
  // oblique faces: per-slot outward normal and index of the |xi.e| estimate
  bool oblique = false;
  int n_est = 0;
  double* d_slot_nrm = nullptr;
  int* d_slot_est = nullptr;
  double* d_est_core = nullptr;  // [n_est][6^3]
  double* d_est_fac = nullptr;   // [n_est][3][6][N]
  int* d_est_rank = nullptr;     // [n_est][3]
  // rounding in the space of the concatenated factors (axis-aligned faces,
  // N <= 32): the cells it leaves to the N-basis passes and their count,
  // per-cell-and-mode validity of the kept N-basis eigenbases, counters,
  // and a pinned word for that count, read back each eager step
  bool rspace = false;
  bool rspace_ok = false;  // the state supports it
  bool served = false;     // a server's state: no second workspace, eager steps never wait on the host
  int* d_rlistD = nullptr;
  int* d_rcnt = nullptr;
  int* d_wvalid = nullptr;
  unsigned long long* d_rstats = nullptr;
  int* h_rcnt = nullptr;
  long long dense_total = 0;  // cells rounded on the N-basis path (eager steps)
  // LU-SGS (set up on first use): sweep colour of every cell, the cells of
  // each colour (forward) and those of each colour with a later neighbour
  // (backward), the increments df* / df in the state layout, the rank-1
  // inverse diagonals and (p, Q) of |xi| per instance
  bool lu_ready = false;
  std::vector<int> lu_off, lu_boff;
  int* d_lu_col = nullptr;
  int* d_lu_cells = nullptr;
  int* d_lu_bcells = nullptr;
  int* d_lu_cnt = nullptr;
  int* d_lu_bcnt = nullptr;
  double* d_df_core = nullptr;
  double* d_df_fac = nullptr;
  int* d_df_rank = nullptr;
  double* d_lu_dinv = nullptr;
  double* d_lu_pq = nullptr;
  // intermediate rounding of the face terms (set up on first use): the
  // rounded flux term of every face slot, six state-layout buffers
  bool face_round = false;
  double* d_face_core = nullptr;  // [6][nc][CS^3]
  double* d_face_fac = nullptr;   // [6][nc][3][CS][N]
  int* d_face_rank = nullptr;     // [6][nc][3]
  double* Wb = nullptr;     // first-pass bases of the FP64 refinement
  double* Wkeep = nullptr;  // [nc][3][N][N] previous full eigenbases (warm start)
  bool warm = false;        // Wkeep holds real bases (after the first step)
  // plain comparator storage
  void* pf[2] = {nullptr, nullptr};
};

// shared helpers (runtime.hip)
tk_status ctx_fail(tk_ctx* ctx, tk_status st, const std::string& msg);
tk_status ctx_hip(tk_ctx* ctx, hipError_t e, const char* what);
void* ctx_alloc(tk_ctx* ctx, size_t bytes, tk_status* st);
void ctx_free(tk_ctx* ctx, void* p);
tk_status state_steps(tk_state* st, int nsteps, double* residual, bool wait, bool lusgs = false);
size_t state_bytes_estimate(int nc, const tk_params& p, bool plain, int chunk);
void state_tune_begin(tk_state* st);
tk_status state_step_residual_async(tk_state* st, double* h_res, int* h_flag);
// est_skip: the |xi . e| estimates of the first est_skip instances are not
// computed (state_copy_instance brings them from a state that has them)
tk_status state_create_served(tk_ctx* ctx, int count, const tk_mesh* const* meshes, const tk_params* params,
                              const double* const* macros, tk_state** out, int est_skip = 0);
tk_status state_freeze_instance(tk_state* st, int k);
tk_status state_copy_instance(tk_state* dst, int kd, tk_state* src, int ks);
