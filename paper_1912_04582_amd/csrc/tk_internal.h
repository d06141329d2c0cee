// Internal declarations of the tk library (device layouts, kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tk.h"
#include "tk_host.h"

namespace tk {

constexpr int kEstCap = 6;   // mode ranks of the |xi.e| estimate on oblique faces
constexpr double kEstDrop = 1e-14;  // estimate: drop singular values <= kEstDrop sigma_1

// Per-instance parameters, device resident (one entry per instance).
struct InstParams {
  double xi_min, dxi;
  double dt, Rg, m, Pr, omega, Kn, tol;
  int cap;
  int frozen;  // 1: the instance is no longer stepped (a retired served request)
};

// Device views used by the step kernels.  Factor storage: fac[cell][a][k][i]
// (column k of mode a, N contiguous); core storage: core[cell][k1 + CS (k2 +
// CS k3)] with CS the state's storage cap; ranks rank[cell][3].
struct DevState {
  int n_cells;
  int N;
  int CS;                  // storage cap (max over instances)
  const int* inst;         // [nc]
  const InstParams* ip;    // [n_inst]
  const int* slot_nb;      // [nc][6] neighbour cell, or global bc index
  const int8_t* slot_kind; // [nc][6]
  const int8_t* slot_axis; // [nc][6]
  const int8_t* slot_sig;  // [nc][6] outward orientation along the axis
  const double* slot_coef; // [nc][6] dt * A / V
  const double* bc_fac;    // [n_bc][3][N] rank-1 boundary Maxwellian factors
  // state, current buffer
  const double* core;
  const double* fac;
  const int* rank;
  // state, next buffer
  double* core_n;
  double* fac_n;
  int* rank_n;
  // per-cell macro (n,u1,u2,u3,T,q1,q2,q3), collision frequency, wall ghosts
  double* macro;
  double* nu;
  double* nw;      // [nc][6]
  int* flag;       // numeric error flag per instance
  // oblique faces (slot_axis < 0): outward normal, estimate index and data
  const double* slot_nrm;  // [nc][6][3]
  const int* slot_est;     // [nc][6]
  const double* est_core;  // [n_est][kEstCap^3]
  const double* est_fac;   // [n_est][3][kEstCap][N]
  const int* est_rank;     // [n_est][3]
  // N-basis rounding over a device-side cell list: pass-local cell k is
  // cells[c0 + k], and a pass ends at *cells_n (nullptr: cells c0 + k)
  const int* cells;
  const int* cells_n;
};

// Intermediate rounding: the rounded flux term of every face slot, each in the
// state layout (core [nc][CS^3], factors [nc][3][CS][N], ranks [nc][3]).
struct FaceStates {
  const double* core[kSlots];
  const double* fac[kSlots];
  const int* rank[kSlots];
};

// LU-SGS sweeps: the increments (state layout) of the cells already swept,
// the sweep colour of every cell and the rank-1 inverse diagonal.
struct LuArgs {
  const double* core;  // [nc][CS^3]
  const double* fac;   // [nc][3][CS][N]
  const int* rank;     // [nc][3]
  const int* col;      // [nc]
  int colour;          // colour of the cells of the launch
  const double* dinv;  // [nc][N + 1]: 1 / u(i) for i < N, then 1 / sigma
};
enum LuStage { LU_FORWARD = 0, LU_BACKWARD = 1, LU_COMMIT = 2 };

// Kernel families (names used by the profiler interface).
enum KernelId { KID_MOMENTS = 0, KID_EXPAND, KID_GRAM, KID_EIG, KID_PROJECT, KID_INIT, KID_PLAIN_MOM,
                KID_PLAIN_STEP, KID_RESID, KID_RROUND, KID_LU, KID_COUNT };
extern const char* kKernelNames[KID_COUNT];

// ---- launchers (each enqueues on `s`) -------------------------------------
hipError_t launch_init_maxwell(const DevState& d, const double* macro5, hipStream_t s);
hipError_t launch_moments(const DevState& d, hipStream_t s);
// oblique: list/list_n hold the cells of the pass left to the general path
// (device memory for `count` cells and a counter)
hipError_t launch_expand(const DevState& d, int c0, int count, void* X, int mixed, int oblique, int* list,
                         int* list_n, hipStream_t s);
// c0/cells_n: workgroups whose c0 + k reaches *cells_n exit (device-side cell lists)
hipError_t launch_gram(int N, int count, const void* X, int mixed, double* G, hipStream_t s, int c0 = 0,
                       const int* cells_n = nullptr);
// eig of Grams [count][3][N][N]; writes factors/ranks of cells c0.. into the
// next buffers (tol/cap per instance via inst/ip, or the overrides when
// inst == nullptr)
hipError_t launch_eig(int N, int count, const double* G, const int* inst, const InstParams* ip, int c0,
                      double tol_override, int cap_override, int CS, double* fac_n, int* rank_n,
                      const double* Win, double* Wout, double* Wkeep, double rel_thr, double abs_fac,
                      hipStream_t s, double drop = 0.0, const int* cells = nullptr, const int* cells_n = nullptr,
                      int* wvalid = nullptr);
hipError_t eig_stats(unsigned long long* out, bool reset);
// |xi . e| on the full grid for `count` unit normals (FP64), for the estimate
hipError_t launch_absxi(int N, int count, const double* normals, double xi_min, double dxi, double* X,
                        hipStream_t s);
// set `count` N x N bases to the identity (cold start of the warm-started eigensolver)
hipError_t launch_identity_basis(int N, size_t count, double* W, hipStream_t s);
// Gram of the rotated unfoldings: G2_a = (W_a^T A_(a)) (W_a^T A_(a))^T
hipError_t launch_gram_rot(int N, int count, const void* X, int mixed, const double* W, double* G2,
                           hipStream_t s, int c0 = 0, const int* cells_n = nullptr);
hipError_t launch_project(int N, int count, const void* X, int mixed, int c0, int CS, const double* fac_n,
                          const int* rank_n, double* core_n, hipStream_t s, const int* cells = nullptr,
                          const int* cells_n = nullptr);
// Intermediate rounding of the face terms: X = the contribution of face slot
// `slot` to the update (zero for cells without that slot), or the sum of the
// cell's own terms and the rounded face terms fs
hipError_t launch_face_term(const DevState& d, int c0, int count, void* X, int mixed, int slot, hipStream_t s);
hipError_t launch_face_sum(const DevState& d, const FaceStates& fs, int c0, int count, void* X, int mixed,
                           hipStream_t s);
// Rounding in the space of the concatenated factors, fused with the term
// assembly (axis-aligned faces, rank-1 neighbourhoods): every cell of d is
// tried; the cells it leaves go to listD/nD for the N-basis path.
// wvalid[3 c + a] = 0 for the cells rounded here.  stats (nullable, 8
// counters): [0] cells rounded, [1] their FP64 operations, [2] their Jacobi
// sweeps.
hipError_t launch_rround(const DevState& d, int* listD, int* nD, int* wvalid, unsigned long long* stats,
                         hipStream_t s);
// p[0..n) = v
hipError_t launch_fill_int(int* p, size_t n, int v, hipStream_t s);
// Rank-1 truncated HOSVD u (x) u (x) u sigma of every cell's LU-SGS diagonal
// (1 + dt nu) 1 + (dt / (2 V)) (sum_l A_l) |xi|; pq[inst] = (p, Q) of |xi|'s
// mode-1 unfolding S: p = S 1 (N values), Q = S S^T (N x N)
hipError_t launch_lu_diag(const DevState& d, const double* pq, double* dinv, hipStream_t s);
// LU-SGS stage of `count` cells (d.cells / d.cells_n from c0) into X (FP64,
// or FP32 when mixed):
// forward  X = D^-1 (dt R + sum_{lower far cells} b_l o df*_m)
// backward X = df*_i + D^-1 sum_{upper far cells} b_l o df_m
// commit   X = f_i + df_i
hipError_t launch_lu_expand(const DevState& d, const LuArgs& lu, int stage, int c0, int count, void* X, int mixed,
                            hipStream_t s);
// generic expansion of `count` Tucker tensors given in the state layout into X (fp64)
hipError_t launch_expand_plain(int N, int count, int CS, const double* core, const double* fac,
                               const int* rank, double* X, hipStream_t s);
hipError_t launch_residual(const double* macro_old, const double* macro_new, const double* vol,
                           const int* inst_off, int n_inst, double* out, hipStream_t s);

// plain full-tensor comparator
struct DevPlain {
  int n_cells;
  int N;
  const int* inst;
  const InstParams* ip;
  const int* slot_nb;
  const int8_t* slot_kind;
  const int8_t* slot_axis;
  const int8_t* slot_sig;
  const double* slot_coef;
  const double* bc_fac;
  const double* slot_nrm;  // [nc][6][3] outward normals (faces off the axes), or nullptr
  const void* f;   // [nc][N^3] float or double
  void* f_n;
  double* macro;
  double* nu;
  double* nw;
  int* flag;
};
hipError_t launch_plain_init(const DevPlain& d, const double* macro5, int mixed, hipStream_t s);
hipError_t launch_plain_moments(const DevPlain& d, int mixed, hipStream_t s);
hipError_t launch_plain_step(const DevPlain& d, int mixed, hipStream_t s);

}  // namespace tk
