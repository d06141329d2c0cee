// Term assembly: the full update f* = f + dt R of one cell on the N^3 grid,
// written to a workspace for the rounding kernels.
//
// With P_out = (xi_n + |xi_n|)/2 and P_in = (xi_n - |xi_n|)/2 for the
// outward normal of every face (eq. exact-flux in gather form, Alg. 1
// steps 2-9), an axis-aligned face with outward normal s e_a contributes
// the row scalings max(s xi_a, 0) (own cell) and min(s xi_a, 0) (far
// side).  Hence
//
//   f* = w o f  +  dt nu f_S  +  sum_l b_l o g_l,
//   w(i)   = 1 - dt nu - sum_l (dt A_l / V) max(s_l xi_{a_l}, 0)
//   b_l(i) = (dt A_l / V) max(-s_l xi_{a_l}, 0)  (a function of one index)
//
// where g_l is the neighbour's Tucker state or the boundary ghost.  Every
// source (the cell, f_S, the six far sides) is expanded from its Tucker
// form by three mode products, G x3 U3 -> x2 U2 -> x1 U1, staged through
// LDS; the last product accumulates straight into registers: in the fibre
// form each thread owns whole mode-1 fibres of f*, in the matrix-core form
// (k_expand_pipe at N = 32, FP32) each wave owns 32 x 32 tiles.
// f_S is built directly in Tucker form with mode ranks 4: columns
// m_a(xi) (xi - u_a)^k, k = 0..3, and a 4x4x4 core with 13 non-zeros
// (the expansion of f_M [1 + A_s (q.v)(v^2/(2 R_g T) - 5/2)]).
#include "tk_internal.h"

namespace tk {

namespace {

constexpr int KC = 4;  // rank-1 chunk of the staged mode products

// Workgroups per cell of the axis-aligned expansion.
template <int N>
struct ExpandSplit {
  static constexpr int S = 1;
};
template <>
struct ExpandSplit<32> {
  static constexpr int S = 2;
};

// Y = G x3 U3 of one staged source, all r1 x r2 x N entries, into LDS.
template <int N, int BLOCK, typename T>
__device__ inline void y_stage(const T* sU, const T* sG, T* sY, int r1, int r2, int r3, int CS) {
  const T* U3 = sU + 2 * CS * N;
  for (int o = threadIdx.x; o < r1 * r2 * N; o += BLOCK) {
    const int i3 = o % N, t = o / N, k2 = t % r2, j = t / r2;
    T sacc = 0;
    const T* g = sG + j + r1 * k2;
    for (int k3 = 0; k3 < r3; ++k3) sacc += g[r1 * r2 * k3] * U3[k3 * N + i3];
    sY[o] = sacc;
  }
}

// Mode-2 and mode-1 products of one source whose Y is in LDS, for the
// thread's own fibres: z_j = sum_k2 U2[i2,k2] Y[j,k2,i3], acc += U1[:,j] z_j.
template <int N, typename T, int FIB>
__device__ inline void fibre_products(T (&acc)[FIB][N], const T* sU, const T* sY, int r1, int r2, int CS,
                                      const int (&pf)[FIB]) {
  const T* U1 = sU;
  const T* U2 = sU + CS * N;
  for (int j = 0; j < r1; ++j) {
    T z[FIB];
#pragma unroll
    for (int f = 0; f < FIB; ++f) {
      const int i2 = pf[f] % N, i3 = pf[f] / N;
      const T* y = sY + j * r2 * N + i3;
      T sacc = 0;
      for (int k2 = 0; k2 < r2; ++k2) sacc += U2[k2 * N + i2] * y[k2 * N];
      z[f] = sacc;
    }
    const T* u = U1 + j * N;
#pragma unroll
    for (int i1 = 0; i1 < N; ++i1) {
      const T uv = u[i1];
#pragma unroll
      for (int f = 0; f < FIB; ++f) acc[f][i1] += uv * z[f];
    }
  }
}

// One source into the fibre accumulators: Y = G x3 U3 (all r1 x r2 x N in
// LDS), then each thread forms z_j = sum_k2 U2[i2,k2] Y[j,k2,i3] for its own
// fibres and adds U1[:,j] z_j.  One barrier between Y and its use; the
// caller separates sources with a barrier before restaging.
template <int N, int BLOCK, typename T, int FIB>
__device__ inline void expand_fibres(T (&acc)[FIB][N], const T* sU, const T* sG, T* sY, int r1, int r2, int r3,
                                     int CS, const int (&pf)[FIB]) {
  y_stage<N, BLOCK, T>(sU, sG, sY, r1, r2, r3, CS);
  __syncthreads();
  fibre_products<N, T, FIB>(acc, sU, sY, r1, r2, CS, pf);
}

// Stage a state-layout Tucker tensor into LDS.  rev_axis: mode whose rows
// are reversed (symmetry ghost), scale_axis / sc: row scaling of one mode,
// gsc: core scale.
template <int N, int BLOCK, typename T>
__device__ inline void stage_state(const double* core, const double* fac, int CS, int c, int r1, int r2,
                                   int r3, int rev_axis, int scale_axis, const T* sc, double gsc, T* sU,
                                   T* sG) {
  const int tid = threadIdx.x;
  const int rr[3] = {r1, r2, r3};
  for (int o = tid; o < 3 * CS * N; o += BLOCK) {
    const int a = o / (CS * N), rem = o % (CS * N), k = rem / N, i = rem % N;
    if (k >= rr[a]) continue;
    const int is = (a == rev_axis) ? (N - 1 - i) : i;
    T v = (T)fac[((size_t)c * 3 + a) * CS * N + k * N + is];
    if (a == scale_axis) v *= sc[i];
    sU[o] = v;
  }
  for (int o = tid; o < r1 * r2 * r3; o += BLOCK) {
    const int k1 = o % r1, t = o / r1, k2 = t % r2, k3 = t / r2;
    sG[o] = (T)(core[(size_t)c * CS * CS * CS + k1 + CS * (k2 + CS * k3)] * gsc);
  }
}

// LU: the forward LU-SGS stage instead of the explicit update: the cell's
// own coefficient loses its 1 (dt R instead of f + dt R), the increments
// df* of the far cells swept earlier are added as further far sides, and the
// sum is divided by the rank-1 diagonal.
template <int N, int BLOCK, typename T, bool LU = false>
__global__ __launch_bounds__(BLOCK) void k_expand(DevState d, int c0, T* X, LuArgs lu) {
  // SPLIT workgroups share a cell, each expanding every source but only its
  // share of the fibres (more, smaller workgroups per CU)
  constexpr int SPLIT = ExpandSplit<N>::S;
  constexpr int FIB = N * N / (BLOCK * SPLIT);
  static_assert(FIB * BLOCK * SPLIT == N * N, "fibres must tile the workgroups");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int CS = d.CS;
  T* sxi = smem;                  // N
  T* sd = sxi + N;                // 3 N   own-cell outflow tables d_a
  T* sb = sd + 3 * N;             // N     row scaling of the current source
  T* sU = sb + N;                 // 3 CS N
  T* sG = sU + 3 * CS * N;        // CS^3
  T* sY = sG + CS * CS * CS;      // CS CS N
  T* sFU = sY + CS * CS * N;      // 3 CS N   f_S factors
  T* sFG = sFU + 3 * CS * N;      // 64       f_S core
  const int cb = blockIdx.x / SPLIT, part = blockIdx.x % SPLIT;
  if (d.cells && c0 + cb >= *d.cells_n) return;
  const int c = d.cells ? d.cells[c0 + cb] : c0 + cb;
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const double nu = d.nu[c];
  int pf[FIB];
#pragma unroll
  for (int f = 0; f < FIB; ++f) pf[f] = tid + BLOCK * (part * FIB + f);

  for (int i = tid; i < N; i += BLOCK) {
    const double x = P.xi_min + i * P.dxi;
    sxi[i] = (T)x;
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
      for (int l = 0; l < kSlots; ++l) {
        const int8_t kind = d.slot_kind[kSlots * c + l];
        if (kind == SK_NONE || d.slot_axis[kSlots * c + l] != a) continue;
        s -= d.slot_coef[kSlots * c + l] * fmax((double)d.slot_sig[kSlots * c + l] * x, 0.0);
      }
      sd[a * N + i] = (T)s;
    }
  }
  // f_S in Tucker form, scaled by dt nu, staged before the accumulators are
  // live (its FP64 set-up would otherwise share their registers)
  {
    const double* M = d.macro + 8 * (size_t)c;
    const double n = M[0], T0 = M[4];
    const double RT = P.Rg * T0;
    const double amp = cbrt(n) / sqrt(2.0 * M_PI * RT);
    const double beta = 1.0 / (2.0 * RT);
    const double As = 2.0 * (1.0 - P.Pr) / (5.0 * P.m * n * RT * RT);
    for (int o = tid; o < 3 * N; o += BLOCK) {
      const int a = o / N, i = o % N;
      const double v = P.xi_min + i * P.dxi - M[1 + a];
      const double base = amp * exp(-v * v * beta);
      sFU[a * CS * N + 0 * N + i] = (T)base;
      sFU[a * CS * N + 1 * N + i] = (T)(base * v);
      sFU[a * CS * N + 2 * N + i] = (T)(base * v * v);
      sFU[a * CS * N + 3 * N + i] = (T)(base * v * v * v);
    }
    if (tid == 0) {
      for (int o = 0; o < 64; ++o) sFG[o] = 0;
      const double sc = P.dt * nu;
      sFG[0] = (T)sc;
      for (int a = 0; a < 3; ++a) {
        const double qa = M[5 + a];
        int st = (a == 0) ? 1 : (a == 1 ? 4 : 16);
        sFG[1 * st] += (T)(sc * -2.5 * As * qa);
        sFG[3 * st] += (T)(sc * As * beta * qa);
        for (int b2 = 0; b2 < 3; ++b2) {
          if (b2 == a) continue;
          const int sb2 = (b2 == 0) ? 1 : (b2 == 1 ? 4 : 16);
          sFG[1 * st + 2 * sb2] += (T)(sc * As * beta * qa);
        }
      }
    }
  }
  const int r1 = d.rank[3 * c], r2 = d.rank[3 * c + 1], r3 = d.rank[3 * c + 2];
  stage_state<N, BLOCK, T>(d.core, d.fac, CS, c, r1, r2, r3, -1, -1, sb, 1.0, sU, sG);
  __syncthreads();

  T acc[FIB][N];
#pragma unroll
  for (int f = 0; f < FIB; ++f)
#pragma unroll
    for (int i = 0; i < N; ++i) acc[f][i] = 0;
  expand_fibres<N, BLOCK, T, FIB>(acc, sU, sG, sY, r1, r2, r3, CS, pf);
  __syncthreads();
  {
    const T cterm = (T)((LU ? 0.0 : 1.0) - P.dt * nu);
#pragma unroll
    for (int f = 0; f < FIB; ++f) {
      const T dd = cterm + sd[N + pf[f] % N] + sd[2 * N + pf[f] / N];
#pragma unroll
      for (int i = 0; i < N; ++i) acc[f][i] *= (sd[i] + dd);
    }
  }
  expand_fibres<N, BLOCK, T, FIB>(acc, sFU, sFG, sY, 4, 4, 4, CS, pf);
  __syncthreads();

  // far sides of the six faces
  for (int l = 0; l < kSlots; ++l) {
    const int8_t kind = d.slot_kind[kSlots * c + l];
    if (kind == SK_NONE) continue;
    const int ax = d.slot_axis[kSlots * c + l];
    const double sg = (double)d.slot_sig[kSlots * c + l];
    const double coef = d.slot_coef[kSlots * c + l];
    const int nb = d.slot_nb[kSlots * c + l];
    for (int i = tid; i < N; i += BLOCK) sb[i] = (T)(coef * fmax(-sg * (P.xi_min + i * P.dxi), 0.0));
    __syncthreads();
    int q1 = 1, q2 = 1, q3 = 1;
    if (kind == SK_INTERIOR || kind == SK_OUTFLOW || kind == SK_SYM) {
      const int src = (kind == SK_INTERIOR) ? nb : c;
      q1 = d.rank[3 * src];
      q2 = d.rank[3 * src + 1];
      q3 = d.rank[3 * src + 2];
      stage_state<N, BLOCK, T>(d.core, d.fac, CS, src, q1, q2, q3, kind == SK_SYM ? ax : -1, ax, sb, 1.0,
                               sU, sG);
    } else {
      const double gsc = (kind == SK_WALL) ? d.nw[kSlots * c + l] : 1.0;
      const double* bf = d.bc_fac + (size_t)nb * 3 * N;
      for (int o = tid; o < 3 * N; o += BLOCK) {
        const int a = o / N, i = o % N;
        T v = (T)bf[o];
        if (a == ax) v *= sb[i];
        sU[a * CS * N + i] = v;
      }
      if (tid == 0) sG[0] = (T)gsc;
    }
    __syncthreads();
    expand_fibres<N, BLOCK, T, FIB>(acc, sU, sG, sY, q1, q2, q3, CS, pf);
    __syncthreads();
  }
  if constexpr (LU) {
    for (int l = 0; l < kSlots; ++l) {
      if (d.slot_kind[kSlots * c + l] != SK_INTERIOR) continue;
      const int nb = d.slot_nb[kSlots * c + l];
      if (lu.col[nb] >= lu.colour) continue;
      const int ax = d.slot_axis[kSlots * c + l];
      const double sg = (double)d.slot_sig[kSlots * c + l];
      const double coef = d.slot_coef[kSlots * c + l];
      for (int i = tid; i < N; i += BLOCK) sb[i] = (T)(coef * fmax(-sg * (P.xi_min + i * P.dxi), 0.0));
      __syncthreads();
      const int q1 = lu.rank[3 * nb], q2 = lu.rank[3 * nb + 1], q3 = lu.rank[3 * nb + 2];
      stage_state<N, BLOCK, T>(lu.core, lu.fac, CS, nb, q1, q2, q3, -1, ax, sb, 1.0, sU, sG);
      __syncthreads();
      expand_fibres<N, BLOCK, T, FIB>(acc, sU, sG, sY, q1, q2, q3, CS, pf);
      __syncthreads();
    }
    const double* di = lu.dinv + (size_t)c * (N + 1);
    for (int i = tid; i < N; i += BLOCK) sb[i] = (T)di[i];
    __syncthreads();
    const T isg = (T)di[N];
#pragma unroll
    for (int f = 0; f < FIB; ++f) {
      const T w = sb[pf[f] % N] * sb[pf[f] / N] * isg;
#pragma unroll
      for (int i = 0; i < N; ++i) acc[f][i] *= sb[i] * w;
    }
  }

  T* out = X + (size_t)cb * N * N * N;
#pragma unroll
  for (int f = 0; f < FIB; ++f)
#pragma unroll
    for (int i = 0; i < N; ++i) out[(size_t)pf[f] * N + i] = acc[f][i];
}

// ---------------------------------------------------------------------------
// The same assembly with the sources software-pipelined.  The cell's face
// records and the far cells' ranks are read once, by one thread per face,
// into LDS; each source is staged into one of two LDS buffers, and the
// global loads of the next source are issued before the current source's
// fibre products, so their latency is hidden behind arithmetic.  Used when
// two buffers leave room for two workgroups per CU.  At N = 32 in FP32 the
// last two mode products run on the matrix cores (tile_products): the
// fibre form reads all of U1[:, j] from LDS for every 32 FMAs of a wave,
// which on the CU's shared LDS takes about twice the time of the FMAs.

enum : int { SRC_STATE = 0, SRC_FS = 1, SRC_BC = 2 };

// one source: its kind, the cell or boundary index, ranks, the reversed
// axis (symmetry ghost), the scaled axis with b(i) = coef max(-sig xi_i, 0)
// and the core scale
struct ExpSrc {
  int type, idx, q1, q2, q3, rev, sax;
  double coef, sig, gsc;
};

// this thread's share of a source's global data: one value per mode factor
// (threads below q_a N), the first core value, or one boundary factor value
struct ExpPre {
  double f0, f1, f2, g;
};

template <int N>
__device__ inline int fac_index(int tid, int rev_axis, int a) {
  const int i = tid % N;
  return (tid / N) * N + ((a == rev_axis) ? (N - 1 - i) : i);
}

template <int N>
__device__ inline void src_prefetch(const DevState& d, const ExpSrc& e, ExpPre& p) {
  const int tid = threadIdx.x;
  const int CS = d.CS;
  p.f0 = p.f1 = p.f2 = p.g = 0.0;
  if (e.type == SRC_STATE) {
    const double* fa = d.fac + (size_t)e.idx * 3 * CS * N;
    if (tid < e.q1 * N) p.f0 = fa[fac_index<N>(tid, e.rev, 0)];
    if (tid < e.q2 * N) p.f1 = fa[CS * N + fac_index<N>(tid, e.rev, 1)];
    if (tid < e.q3 * N) p.f2 = fa[2 * CS * N + fac_index<N>(tid, e.rev, 2)];
    if (tid < e.q1 * e.q2 * e.q3) {
      const int k1 = tid % e.q1, t = tid / e.q1, k2 = t % e.q2, k3 = t / e.q2;
      p.g = d.core[(size_t)e.idx * CS * CS * CS + k1 + CS * (k2 + CS * k3)];
    }
  } else if (e.type == SRC_BC) {
    if (tid < 3 * N) p.f0 = d.bc_fac[(size_t)e.idx * 3 * N + tid];
  }
}

template <int N, int BLOCK, typename T>
__device__ inline void src_store(const DevState& d, const InstParams& P, const ExpSrc& e, const ExpPre& p, T* sU,
                                 T* sG, int LS) {
  const int tid = threadIdx.x;
  const int CS = d.CS;
  auto scale = [&](int i) -> T { return (T)(e.coef * fmax(-e.sig * (P.xi_min + i * P.dxi), 0.0)); };
  if (e.type == SRC_STATE) {
    const double fv[3] = {p.f0, p.f1, p.f2};
    const int qq[3] = {e.q1, e.q2, e.q3};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (tid < qq[a] * N) {
        T v = (T)fv[a];
        if (a == e.sax) v *= scale(tid % N);
        sU[a * LS * N + tid] = v;
      }
    }
    const int nq = e.q1 * e.q2 * e.q3;
    if (tid < nq) sG[tid] = (T)(p.g * 1.0);
    for (int o = tid + BLOCK; o < nq; o += BLOCK) {
      const int k1 = o % e.q1, t = o / e.q1, k2 = t % e.q2, k3 = t / e.q2;
      sG[o] = (T)(d.core[(size_t)e.idx * CS * CS * CS + k1 + CS * (k2 + CS * k3)] * 1.0);
    }
  } else if (e.type == SRC_BC) {
    if (tid < 3 * N) {
      const int a = tid / N, i = tid % N;
      T v = (T)p.f0;
      if (a == e.sax) v *= scale(i);
      sU[a * LS * N + i] = v;
    }
    if (tid == 0) sG[0] = (T)e.gsc;
  }
}

typedef float v16f __attribute__((ext_vector_type(16)));

// Orders the LDS accesses of one wavefront's lanes (a wave's LDS
// instructions execute in order; this keeps the compiler from moving them
// across the point).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Y = G x3 U3 of one staged source at the wave's two i3 (i3a, i3a + 1), all
// j < r1, k2 < r2, into the wave's own LDS slice wy[(j r2 + k2) 2 + t]
// (the same sums, in the same order, as y_stage); no workgroup barrier.
__device__ inline void wave_y(const float* sU, const float* sG, float* wy, int r1, int r2, int r3, int LS, int lane,
                              int i3a) {
  constexpr int N = 32;
  const float* U3 = sU + 2 * LS * N;
  const int E = 2 * r1 * r2;
  for (int o = lane; o < E; o += 64) {
    const int t = o & 1, jk = o >> 1, k2 = jk % r2, j = jk / r2;
    float sacc = 0.f;
    const float* g = sG + j + r1 * k2;
    for (int k3 = 0; k3 < r3; ++k3) sacc += g[r1 * r2 * k3] * U3[k3 * N + i3a + t];
    wy[o] = sacc;
  }
}

// Last two mode products of one source on the matrix cores (N = 32, FP32):
// for the wave's tiles X[i1, i2, i3] (i3 = i3a, i3a + 1; all i1, i2),
//   X^T[i2, i1] += sum_j Z_j[i2, i3] U1[i1, j],  Z_j = U2 Y_j,
// two values of j per v_mfma_f32_32x32x2f32.  Lane l supplies the A value
// at row l % 32, k = l / 32 (z of j = j0 + l / 32 at i2 = l % 32, formed by
// the lane itself from the wave's Y slice) and the B value at k = l / 32,
// column l % 32 (U1[l % 32, j]); it holds D rows 8 (v / 4) + 4 (l / 32) +
// v % 4 of column l % 32.
__device__ inline void tile_products(v16f& t0, v16f& t1, const float* sU, const float* wy, int r1, int r2, int LS,
                                     int li, int hi) {
  constexpr int N = 32;
  const float* U1 = sU;
  const float* U2 = sU + LS * N;
  for (int j0 = 0; j0 < r1; j0 += 2) {
    const int j = j0 + hi;
    float z0 = 0.f, z1 = 0.f, u1 = 0.f;
    if (j < r1) {
      const float* y = wy + 2 * j * r2;
      for (int k2 = 0; k2 < r2; ++k2) {
        const float u2 = U2[k2 * N + li];
        const float2 yy = *reinterpret_cast<const float2*>(y + 2 * k2);
        z0 += u2 * yy.x;
        z1 += u2 * yy.y;
      }
      u1 = U1[j * N + li];
    }
    t0 = __builtin_amdgcn_mfma_f32_32x32x2f32(z0, u1, t0, 0, 0, 0);
    t1 = __builtin_amdgcn_mfma_f32_32x32x2f32(z1, u1, t1, 0, 0, 0);
  }
}

// RB > 0: LDS laid out for ranks up to RB (more workgroups per CU); a cell
// with a larger rank among its sources is appended to `list` and left to a
// second launch.  LIST: 0 every cell of the pass, 1 as 0 with that
// hand-off, 2 only the cells in `list` (the count in *list_n).
template <int N, int BLOCK, typename T, bool MF, int RB, int LIST>
__global__ __launch_bounds__(BLOCK, RB > 0 ? 6 : 1) void k_expand_pipe(DevState d, int c0, T* X, int* list,
                                                                       int* list_n) {
  constexpr int SPLIT = ExpandSplit<N>::S;
  constexpr int FIB = N * N / (BLOCK * SPLIT);
  static_assert(FIB * BLOCK * SPLIT == N * N, "fibres must tile the workgroups");
  static_assert(BLOCK >= N * kMaxCap && BLOCK >= 3 * N, "one factor value per thread and mode");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ ExpSrc s_slot[kSlots];     // per face, as stored
  __shared__ ExpSrc s_src[2 + kSlots];  // own cell, f_S, then the used faces
  __shared__ int s_ns;
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int LS = RB > 0 ? RB : d.CS;                     // rank extent of the LDS layout
  const int GS = (LS * LS * LS + 1) & ~1;                // core extent, even so Y stays 8-byte aligned
  const int BUF = 3 * LS * N + GS + (MF ? 0 : LS * LS * N);  // sU, sG (and sY) of one buffer
  T* sd = smem;                   // 3 N   own-cell outflow tables d_a
  T* sFU = sd + 3 * N;            // 3 LS N   f_S factors
  T* sFG = sFU + 3 * LS * N;      // 64       f_S core
  T* sB = sFG + 64;               // two buffers
  T* sWY = sB + 2 * BUF;          // MF: per wave 2 LS LS values of Y
  const int part = blockIdx.x % SPLIT;
  int cb = blockIdx.x / SPLIT;
  if constexpr (LIST == 2) {
    if (cb >= *list_n) return;
    cb = list[cb];
  } else {
    if (d.cells && c0 + cb >= *d.cells_n) return;
  }
  const int c = d.cells ? d.cells[c0 + cb] : c0 + cb;
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const double nu = d.nu[c];
  int pf[FIB];
#pragma unroll
  for (int f = 0; f < FIB; ++f) pf[f] = tid + BLOCK * (part * FIB + f);

  // face records: one thread per slot, each one round of loads (plus the
  // far cell's ranks)
  if (tid < kSlots) {
    const size_t sl = (size_t)kSlots * c + tid;
    const int kind = d.slot_kind[sl];
    ExpSrc e;
    e.type = -1;
    e.idx = d.slot_nb[sl];
    e.q1 = e.q2 = e.q3 = 1;
    e.rev = -1;
    e.sax = d.slot_axis[sl];
    e.coef = d.slot_coef[sl];
    e.sig = (double)d.slot_sig[sl];
    e.gsc = 1.0;
    if (kind == SK_INTERIOR || kind == SK_OUTFLOW || kind == SK_SYM) {
      e.type = SRC_STATE;
      if (kind != SK_INTERIOR) e.idx = c;
      if (kind == SK_SYM) e.rev = e.sax;
      e.q1 = d.rank[3 * e.idx];
      e.q2 = d.rank[3 * e.idx + 1];
      e.q3 = d.rank[3 * e.idx + 2];
    } else if (kind != SK_NONE) {
      e.type = SRC_BC;
      if (kind == SK_WALL) e.gsc = d.nw[sl];
    }
    s_slot[tid] = e;
  }
  if (tid == 0) {
    ExpSrc e;
    e.type = SRC_STATE;
    e.idx = c;
    e.q1 = d.rank[3 * c];
    e.q2 = d.rank[3 * c + 1];
    e.q3 = d.rank[3 * c + 2];
    e.rev = e.sax = -1;
    e.coef = e.sig = 0.0;
    e.gsc = 1.0;
    s_src[0] = e;
    e.type = SRC_FS;
    e.q1 = e.q2 = e.q3 = 4;
    s_src[1] = e;
  }
  // the own cell's data, in flight while f_S is set up
  ExpPre pre;
  {
    ExpSrc own;
    own.type = SRC_STATE;
    own.idx = c;
    own.q1 = d.rank[3 * c];
    own.q2 = d.rank[3 * c + 1];
    own.q3 = d.rank[3 * c + 2];
    own.rev = own.sax = -1;
    own.coef = own.sig = 0.0;
    own.gsc = 1.0;
    src_prefetch<N>(d, own, pre);
  }
  // f_S in Tucker form, scaled by dt nu
  {
    const double* M = d.macro + 8 * (size_t)c;
    const double n = M[0], T0 = M[4];
    const double RT = P.Rg * T0;
    const double amp = cbrt(n) / sqrt(2.0 * M_PI * RT);
    const double beta = 1.0 / (2.0 * RT);
    const double As = 2.0 * (1.0 - P.Pr) / (5.0 * P.m * n * RT * RT);
    for (int o = tid; o < 3 * N; o += BLOCK) {
      const int a = o / N, i = o % N;
      const double v = P.xi_min + i * P.dxi - M[1 + a];
      const double base = amp * exp(-v * v * beta);
      sFU[a * LS * N + 0 * N + i] = (T)base;
      sFU[a * LS * N + 1 * N + i] = (T)(base * v);
      sFU[a * LS * N + 2 * N + i] = (T)(base * v * v);
      sFU[a * LS * N + 3 * N + i] = (T)(base * v * v * v);
    }
    if (tid == 0) {
      for (int o = 0; o < 64; ++o) sFG[o] = 0;
      const double sc = P.dt * nu;
      sFG[0] = (T)sc;
      for (int a = 0; a < 3; ++a) {
        const double qa = M[5 + a];
        int st = (a == 0) ? 1 : (a == 1 ? 4 : 16);
        sFG[1 * st] += (T)(sc * -2.5 * As * qa);
        sFG[3 * st] += (T)(sc * As * beta * qa);
        for (int b2 = 0; b2 < 3; ++b2) {
          if (b2 == a) continue;
          const int sb2 = (b2 == 0) ? 1 : (b2 == 1 ? 4 : 16);
          sFG[1 * st + 2 * sb2] += (T)(sc * As * beta * qa);
        }
      }
    }
  }
  __syncthreads();
  if constexpr (LIST == 1) {
    // every source must fit the RB layout; otherwise hand the cell over
    int qm = max(s_src[0].q1, max(s_src[0].q2, s_src[0].q3));
    for (int l = 0; l < kSlots; ++l)
      if (s_slot[l].type == SRC_STATE) qm = max(qm, max(s_slot[l].q1, max(s_slot[l].q2, s_slot[l].q3)));
    if (qm > RB) {
      if (tid == 0 && part == 0) list[atomicAdd(list_n, 1)] = cb;
      return;
    }
  }
  // compact the source list (unused slots dropped), the own-cell outflow
  // tables, and the own cell into buffer 0
  if (tid == 0) {
    int n = 2;
    for (int l = 0; l < kSlots; ++l)
      if (s_slot[l].type >= 0) s_src[n++] = s_slot[l];
    s_ns = n;
  }
  for (int i = tid; i < N; i += BLOCK) {
    const double x = P.xi_min + i * P.dxi;
    for (int a = 0; a < 3; ++a) {
      double sacc = 0.0;
      for (int l = 0; l < kSlots; ++l) {
        const ExpSrc& e = s_slot[l];
        if (e.type < 0 || e.sax != a) continue;
        sacc -= e.coef * fmax(e.sig * x, 0.0);
      }
      sd[a * N + i] = (T)sacc;
    }
  }
  src_store<N, BLOCK, T>(d, P, s_src[0], pre, sB, sB + 3 * LS * N, LS);
  __syncthreads();
  if constexpr (!MF) {
    y_stage<N, BLOCK, T>(sB, sB + 3 * LS * N, sB + 3 * LS * N + GS, s_src[0].q1, s_src[0].q2, s_src[0].q3, LS);
    __syncthreads();
  }

  // VALU path: whole mode-1 fibres per thread.  MFMA path (MF): each wave
  // owns the 32 x 32 tiles (i2 x i1) of two consecutive i3.
  T acc[FIB][N];
  v16f t0, t1;
  const int lane = tid & 63, li = lane & 31, hi = lane >> 5;
  const int i3a = 2 * (part * (BLOCK / 64) + (tid >> 6));
  if constexpr (MF) {
#pragma unroll
    for (int v = 0; v < 16; ++v) t0[v] = t1[v] = 0.f;
  } else {
#pragma unroll
    for (int f = 0; f < FIB; ++f)
#pragma unroll
      for (int i = 0; i < N; ++i) acc[f][i] = 0;
  }
  const int ns = s_ns;
  for (int sidx = 0; sidx < ns; ++sidx) {
    T* cur = sB + (sidx & 1) * BUF;
    T* nxt = sB + ((sidx + 1) & 1) * BUF;
    const ExpSrc& e = s_src[sidx];
    const bool more = sidx + 1 < ns;
    if (more) src_prefetch<N>(d, s_src[sidx + 1], pre);
    const T* su = e.type == SRC_FS ? sFU : cur;
    const T* sy = cur + 3 * LS * N + GS;
    if constexpr (MF) {
      float* wy = reinterpret_cast<float*>(sWY) + (tid >> 6) * 2 * LS * LS;
      if (e.type == SRC_FS)
        wave_y((const float*)sFU, (const float*)sFG, wy, 4, 4, 4, LS, lane, i3a);
      else
        wave_y((const float*)cur, (const float*)(cur + 3 * LS * N), wy, e.q1, e.q2, e.q3, LS, lane, i3a);
      wave_sync();
      tile_products(t0, t1, (const float*)su, wy, e.q1, e.q2, LS, li, hi);
    } else {
      fibre_products<N, T, FIB>(acc, su, sy, e.q1, e.q2, LS, pf);
    }
    if (sidx == 0) {
      const T cterm = (T)(1.0 - P.dt * nu);
      if constexpr (MF) {
        // tile element v of this lane: i1 = li, i2 = 8 (v / 4) + 4 hi + v % 4
        const T s0 = sd[li];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int i2 = 8 * (v / 4) + 4 * hi + v % 4;
          const T da = cterm + sd[N + i2] + sd[2 * N + i3a];
          const T db = cterm + sd[N + i2] + sd[2 * N + i3a + 1];
          t0[v] *= (s0 + da);
          t1[v] *= (s0 + db);
        }
      } else {
#pragma unroll
        for (int f = 0; f < FIB; ++f) {
          const T dd = cterm + sd[N + pf[f] % N] + sd[2 * N + pf[f] / N];
#pragma unroll
          for (int i = 0; i < N; ++i) acc[f][i] *= (sd[i] + dd);
        }
      }
    }
    if (more) {
      const ExpSrc& en = s_src[sidx + 1];
      src_store<N, BLOCK, T>(d, P, en, pre, nxt, nxt + 3 * LS * N, LS);
      __syncthreads();
      if constexpr (!MF) {
        if (en.type == SRC_FS)
          y_stage<N, BLOCK, T>(sFU, sFG, nxt + 3 * LS * N + GS, 4, 4, 4, LS);
        else
          y_stage<N, BLOCK, T>(nxt, nxt + 3 * LS * N, nxt + 3 * LS * N + GS, en.q1, en.q2, en.q3, LS);
        __syncthreads();
      }
    }
  }

  T* out = X + (size_t)cb * N * N * N;
  if constexpr (MF) {
    // rows of 32 consecutive i1 per half-wave: coalesced 128-byte stores
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i2 = 8 * (v / 4) + 4 * hi + v % 4;
      out[((size_t)i3a * N + i2) * N + li] = t0[v];
      out[((size_t)(i3a + 1) * N + i2) * N + li] = t1[v];
    }
  } else {
#pragma unroll
    for (int f = 0; f < FIB; ++f)
#pragma unroll
      for (int i = 0; i < N; ++i) out[(size_t)pf[f] * N + i] = acc[f][i];
  }
}

// ---------------------------------------------------------------------------
// Meshes with faces off the coordinate axes.  There P_out and P_in of such a
// face depend on all three velocity indices (xi_n = n.xi is rank 2 by
// Lemma 1, the |xi_n| estimate has mode ranks <= 6), so the flux weights are
// evaluated per grid node:
//   f* = W o f + dt nu f_S + sum_l B_l o g_l,
//   W   = 1 - dt nu + sum_l a_l (xi_n,l + est_l),   B_l = a_l (xi_n,l - est_l),
//   a_l = -dt A_l / (2 V)
// (axis-aligned faces keep their separable form).  Each thread holds one
// mode-1 fibre per pass in three register arrays: the accumulator, a weight
// (W or B_l, from the estimate's expansion) and the far side's expansion.

template <int N, int BLOCK, typename T>
__device__ inline void expand_pass(T (&acc)[N], const T* sU, const T* sG, T* sY, T* sZ, int r1, int r2, int r3,
                                   int CSL, int pbase) {
  const T* U1 = sU;
  const T* U2 = sU + CSL * N;
  const T* U3 = sU + 2 * CSL * N;
  const int tid = threadIdx.x;
  for (int kb = 0; kb < r1; kb += KC) {
    const int kc = min(KC, r1 - kb);
    for (int o = tid; o < kc * r2 * N; o += BLOCK) {
      const int i3 = o % N, t = o / N, k2 = t % r2, j = t / r2;
      T s = 0;
      const T* g = sG + (kb + j) + r1 * k2;
      for (int k3 = 0; k3 < r3; ++k3) s += g[r1 * r2 * k3] * U3[k3 * N + i3];
      sY[(j * r2 + k2) * N + i3] = s;
    }
    __syncthreads();
    for (int o = tid; o < kc * BLOCK; o += BLOCK) {
      const int j = o / BLOCK, q = o % BLOCK, pp = pbase + q;
      const int i2 = pp % N, i3 = pp / N;
      T s = 0;
      const T* y = sY + j * r2 * N + i3;
      for (int k2 = 0; k2 < r2; ++k2) s += U2[k2 * N + i2] * y[k2 * N];
      sZ[o] = s;
    }
    __syncthreads();
    for (int j = 0; j < kc; ++j) {
      const T z = sZ[j * BLOCK + tid];
      const T* u = U1 + (kb + j) * N;
#pragma unroll
      for (int i1 = 0; i1 < N; ++i1) acc[i1] += u[i1] * z;
    }
    __syncthreads();
  }
}

// Stage a Tucker tensor stored with factor stride CSsrc into the LDS layout
// with stride CSL (rows of mode rev reversed, mode `ax` scaled by
// coef * max(-sg xi, 0) when coef != 0, core scaled by gsc).
template <int N, int BLOCK, typename T>
__device__ inline void stage_any(const double* core, const double* fac, int CSsrc, size_t id, const int (&rr)[3],
                                 int rev, int ax, double coef, double sg, double xi_min, double dxi, double gsc,
                                 int CSL, T* sU, T* sG) {
  const int tid = threadIdx.x;
  for (int o = tid; o < 3 * CSL * N; o += BLOCK) {
    const int a = o / (CSL * N), rem = o % (CSL * N), k = rem / N, i = rem % N;
    if (k >= rr[a]) continue;
    const int is = (a == rev) ? (N - 1 - i) : i;
    double v = fac[(id * 3 + a) * CSsrc * N + (size_t)k * N + is];
    if (a == ax && coef != 0.0) v *= coef * fmax(-sg * (xi_min + i * dxi), 0.0);
    sU[o] = (T)v;
  }
  for (int o = tid; o < rr[0] * rr[1] * rr[2]; o += BLOCK) {
    const int k1 = o % rr[0], t = o / rr[0], k2 = t % rr[1], k3 = t / rr[1];
    sG[o] = (T)(core[id * CSsrc * CSsrc * CSsrc + k1 + CSsrc * (k2 + CSsrc * k3)] * gsc);
  }
}


// ---- fast path: every source staged once per cell ---------------------------
// Sources: the cell, f_S, and per face slot the far side (state or ghost)
// followed, on an oblique face, by its |xi.e| estimate.  Each is kept in LDS
// as its mode-1 and mode-2 factors and Y = G x3 U3 (r1 x r2 x N); G and U3
// pass through a scratch area source by source.  The fibre passes then need
// no barrier: per fibre and per half of mode 1 a thread expands the cell,
// f_S, each far side and each estimate into registers and combines them
// node by node.
constexpr int kObSrcMax = 2 + 2 * kSlots;
enum ObRole : int { OB_OWN = 0, OB_FS = 1, OB_FAR_AXIS = 2, OB_FAR_OBL = 3, OB_EST = 4 };

struct ObTab {
  int n;
  int role[kObSrcMax], slot[kObSrcMax];
  int r[kObSrcMax][3];
  int offU[kObSrcMax], offY[kObSrcMax];
  int tmp;   // offset of the scratch area (G and U3 of one source)
  int need;  // floats in use from the start of the source area
};

// Halves of mode 1 a thread expands at once: at most 96 bytes of fibre per
// register array.
template <int N, typename T>
constexpr int ob_halves() {
  int h = 1;
  while ((N * (int)sizeof(T)) / h > 96 || N % h) ++h;
  return h;
}

// Expand source s of the table over nodes [i0, i0 + NH) of fibre (i2, i3),
// adding into out.
template <int N, int NH, typename T>
__device__ inline void ob_fibre(const ObTab& tb, int s, const T* src, int i2, int i3, int i0, T (&out)[NH]) {
  const int r1 = tb.r[s][0], r2 = tb.r[s][1];
  const T* U1 = src + tb.offU[s];
  const T* U2 = U1 + r1 * N;
  const T* Y = src + tb.offY[s];
  for (int j = 0; j < r1; ++j) {
    T z = 0;
    const T* y = Y + j * r2 * N + i3;
    for (int k2 = 0; k2 < r2; ++k2) z += U2[k2 * N + i2] * y[k2 * N];
    const T* u = U1 + j * N + i0;
#pragma unroll
    for (int i = 0; i < NH; ++i) out[i] += u[i] * z;
  }
}

template <int N, int BLOCK, typename T>
__device__ void ob_fast(const DevState& d, int c, T* Xc, const T* sxi, const T* sd, T* src, const ObTab& tb,
                        const double (&nrm)[kSlots][3]) {
  constexpr int NPASS = N * N / BLOCK;
  constexpr int H = ob_halves<N, T>();
  constexpr int NH = N / H;
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const double nu = d.nu[c];
  const double* M = d.macro + 8 * (size_t)c;
  const int CS = d.CS;
  // ---- staging, source by source: U1, U2 to their slots, G and U3 to the
  // scratch area, then Y = G x3 U3
  for (int s = 0; s < tb.n; ++s) {
    const int role = tb.role[s], l = tb.slot[s];
    const int r1 = tb.r[s][0], r2 = tb.r[s][1], r3 = tb.r[s][2];
    T* U = src + tb.offU[s];        // U1 (r1 N), U2 (r2 N)
    T* G = src + tb.tmp;            // r1 r2 r3
    T* U3 = G + r1 * r2 * r3;       // r3 N
    const int nU = (r1 + r2 + r3) * N;
    int kind = 0, ax = -1, nb = 0;
    double coef = 0.0, sg = 0.0, gsc = 1.0;
    if (role == OB_FAR_AXIS || role == OB_FAR_OBL || role == OB_EST) {
      kind = d.slot_kind[kSlots * c + l];
      ax = d.slot_axis[kSlots * c + l];
      nb = d.slot_nb[kSlots * c + l];
      coef = d.slot_coef[kSlots * c + l];
      sg = (double)d.slot_sig[kSlots * c + l];
      if (kind == SK_WALL) gsc = d.nw[kSlots * c + l];
    }
    // f_S parameters
    const double n0 = M[0], T0 = M[4];
    const double RT = P.Rg * T0;
    const double amp = cbrt(n0) / sqrt(2.0 * M_PI * RT);
    const double beta = 1.0 / (2.0 * RT);
    const double As = 2.0 * (1.0 - P.Pr) / (5.0 * P.m * n0 * RT * RT);
    for (int o = tid; o < nU; o += BLOCK) {
      int a, k, i;
      if (o < r1 * N) { a = 0; k = o / N; i = o % N; }
      else if (o < (r1 + r2) * N) { a = 1; k = (o - r1 * N) / N; i = o % N; }
      else { a = 2; k = (o - (r1 + r2) * N) / N; i = o % N; }
      double v;
      if (role == OB_OWN) {
        v = d.fac[((size_t)c * 3 + a) * CS * N + (size_t)k * N + i];
      } else if (role == OB_FS) {
        const double x = P.xi_min + i * P.dxi - M[1 + a];
        v = amp * exp(-x * x * beta);
        for (int q = 0; q < k; ++q) v *= x;
      } else if (role == OB_EST) {
        const int e = d.slot_est[kSlots * c + l];
        v = d.est_fac[(((size_t)e * 3 + a) * kEstCap + k) * N + i];
      } else if (kind == SK_INTERIOR || kind == SK_OUTFLOW || kind == SK_SYM) {
        const int sc = (kind == SK_INTERIOR) ? nb : c;
        const int is = (kind == SK_SYM && a == ax) ? (N - 1 - i) : i;
        v = d.fac[((size_t)sc * 3 + a) * CS * N + (size_t)k * N + is];
        if (role == OB_FAR_AXIS && a == ax) v *= coef * fmax(-sg * (P.xi_min + i * P.dxi), 0.0);
      } else {
        v = d.bc_fac[((size_t)nb * 3 + a) * N + i];
        if (role == OB_FAR_AXIS && a == ax) v *= coef * fmax(-sg * (P.xi_min + i * P.dxi), 0.0);
      }
      if (a < 2) U[o] = (T)v;
      else U3[o - (r1 + r2) * N] = (T)v;
    }
    for (int o = tid; o < r1 * r2 * r3; o += BLOCK) {
      const int k1 = o % r1, t = o / r1, k2 = t % r2, k3 = t / r2;
      double g;
      if (role == OB_OWN) {
        g = d.core[(size_t)c * CS * CS * CS + k1 + CS * (k2 + CS * k3)];
      } else if (role == OB_FS) {
        // 13 non-zeros of the f_S core (Proposition 1), times dt nu
        const int kk[3] = {k1, k2, k3};
        int nz = 0, which = -1;
        for (int a = 0; a < 3; ++a)
          if (kk[a]) { ++nz; which = a; }
        g = 0.0;
        if (nz == 0) {
          g = 1.0;
        } else if (nz == 1) {
          if (kk[which] == 1) g = -2.5 * As * M[5 + which];
          else if (kk[which] == 3) g = As * beta * M[5 + which];
        } else if (nz == 2) {
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
              if (a != b && kk[a] == 1 && kk[b] == 2 && kk[3 - a - b] == 0) g = As * beta * M[5 + a];
        }
        g *= P.dt * nu;
      } else if (role == OB_EST) {
        const int e = d.slot_est[kSlots * c + l];
        g = d.est_core[(size_t)e * kEstCap * kEstCap * kEstCap + k1 + kEstCap * (k2 + kEstCap * k3)];
      } else if (kind == SK_INTERIOR || kind == SK_OUTFLOW || kind == SK_SYM) {
        const int sc = (kind == SK_INTERIOR) ? nb : c;
        g = d.core[(size_t)sc * CS * CS * CS + k1 + CS * (k2 + CS * k3)];
      } else {
        g = gsc;
      }
      G[o] = (T)g;
    }
    __syncthreads();
    T* Y = src + tb.offY[s];
    for (int o = tid; o < r1 * r2 * N; o += BLOCK) {
      const int i3 = o % N, t = o / N, k2 = t % r2, j = t / r2;
      T acc = 0;
      const T* g = G + j + r1 * k2;
      for (int k3 = 0; k3 < r3; ++k3) acc += g[r1 * r2 * k3] * U3[k3 * N + i3];
      Y[o] = acc;
    }
    __syncthreads();
  }
  // ---- fibre passes
  const T c1 = (T)(1.0 - P.dt * nu);
  for (int pass = 0; pass < NPASS; ++pass) {
    const int p = pass * BLOCK + tid;
    const int i2 = p % N, i3 = p / N;
    const T base = c1 + sd[N + i2] + sd[2 * N + i3];
    T* out = Xc + (size_t)p * N;
    for (int h = 0; h < H; ++h) {
      const int i0 = h * NH;
      T own[NH], acc[NH];
#pragma unroll
      for (int i = 0; i < NH; ++i) own[i] = 0;
      ob_fibre<N, NH, T>(tb, 0, src, i2, i3, i0, own);
#pragma unroll
      for (int i = 0; i < NH; ++i) acc[i] = (base + sd[i0 + i]) * own[i];
      ob_fibre<N, NH, T>(tb, 1, src, i2, i3, i0, acc);
      for (int s = 2; s < tb.n; ++s) {
        const int role = tb.role[s];
        if (role == OB_FAR_AXIS) {
          ob_fibre<N, NH, T>(tb, s, src, i2, i3, i0, acc);
        } else if (role == OB_FAR_OBL) {
          // W gains a_l (xi_n + est), the far side is weighted by
          // a_l (xi_n - est): acc += a_l (xi_n (own + g) + est (own - g))
          const int l = tb.slot[s];
          T g[NH], e[NH];
#pragma unroll
          for (int i = 0; i < NH; ++i) { g[i] = 0; e[i] = 0; }
          ob_fibre<N, NH, T>(tb, s, src, i2, i3, i0, g);
          ob_fibre<N, NH, T>(tb, s + 1, src, i2, i3, i0, e);
          const T al = (T)(-0.5 * d.slot_coef[kSlots * c + l]);
          const T n1 = (T)nrm[l][0];
          const T x23 = (T)(nrm[l][1] * (double)sxi[i2] + nrm[l][2] * (double)sxi[i3]);
#pragma unroll
          for (int i = 0; i < NH; ++i) {
            const T xn = n1 * sxi[i0 + i] + x23;
            acc[i] += al * (xn * (own[i] + g[i]) + e[i] * (own[i] - g[i]));
          }
          ++s;  // the estimate was consumed with its face
        }
      }
#pragma unroll
      for (int i = 0; i < NH; ++i) out[i0 + i] = acc[i];
    }
  }
}

// Source table of cell c and the floats it needs after the tables; built by
// one thread.
__device__ inline void ob_table(const DevState& d, int c, int N, ObTab& tb) {
  int off = 0, n = 0, tmp = 0;
  auto add = [&](int role, int slot, int r1, int r2, int r3) {
    tb.role[n] = role;
    tb.slot[n] = slot;
    tb.r[n][0] = r1; tb.r[n][1] = r2; tb.r[n][2] = r3;
    tb.offU[n] = off;
    off += (r1 + r2) * N;
    tb.offY[n] = off;
    off += r1 * r2 * N;
    const int t = r1 * r2 * r3 + r3 * N;
    if (t > tmp) tmp = t;
    ++n;
  };
  add(OB_OWN, -1, d.rank[3 * c], d.rank[3 * c + 1], d.rank[3 * c + 2]);
  add(OB_FS, -1, 4, 4, 4);
  for (int l = 0; l < kSlots; ++l) {
    const int kind = d.slot_kind[kSlots * c + l];
    if (kind == SK_NONE) continue;
    const bool obl = d.slot_axis[kSlots * c + l] < 0;
    int q[3] = {1, 1, 1};
    if (kind == SK_INTERIOR || kind == SK_OUTFLOW || kind == SK_SYM) {
      const int sc = (kind == SK_INTERIOR) ? d.slot_nb[kSlots * c + l] : c;
      for (int a = 0; a < 3; ++a) q[a] = d.rank[3 * sc + a];
    }
    add(obl ? OB_FAR_OBL : OB_FAR_AXIS, l, q[0], q[1], q[2]);
    if (obl) {
      const int e = d.slot_est[kSlots * c + l];
      add(OB_EST, l, d.est_rank[3 * e], d.est_rank[3 * e + 1], d.est_rank[3 * e + 2]);
    }
  }
  tb.n = n;
  tb.tmp = off;
  tb.need = off + tmp;
}

// Per-cell tables of both paths: the velocity nodes, the separable
// (axis-aligned) outflow tables and the outward normals of the face slots.
template <int N, int BLOCK, typename T>
__device__ inline void ob_tables(const DevState& d, int c, T* sxi, T* sd, double (&nrm)[kSlots][3]) {
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  // outward normals (the table exists only on states with oblique faces;
  // they are read for oblique slots only)
  if (d.slot_nrm && tid < kSlots * 3) nrm[tid / 3][tid % 3] = d.slot_nrm[(size_t)kSlots * 3 * c + tid];
  for (int i = tid; i < N; i += BLOCK) {
    const double x = P.xi_min + i * P.dxi;
    sxi[i] = (T)x;
    for (int a = 0; a < 3; ++a) {
      double sum = 0.0;
      for (int l = 0; l < kSlots; ++l) {
        const int8_t kind = d.slot_kind[kSlots * c + l];
        if (kind == SK_NONE || d.slot_axis[kSlots * c + l] != a) continue;
        sum -= d.slot_coef[kSlots * c + l] * fmax((double)d.slot_sig[kSlots * c + l] * x, 0.0);
      }
      sd[a * N + i] = (T)sum;
    }
  }
}

// f_S of the macroparameters M (Tucker form, ranks 4: factors base v^k,
// k = 0..3, the 13 non-zero core entries of the Shakhov correction), core
// scaled by `scale`, staged into the LDS layout with factor stride CSL.
template <int N, int BLOCK, typename T>
__device__ inline void stage_fs_any(const double* M, const InstParams& P, double scale, int CSL, T* sU, T* sG) {
  const int tid = threadIdx.x;
  const double n = M[0], T0 = M[4];
  const double RT = P.Rg * T0;
  const double amp = cbrt(n) / sqrt(2.0 * M_PI * RT);
  const double beta = 1.0 / (2.0 * RT);
  const double As = 2.0 * (1.0 - P.Pr) / (5.0 * P.m * n * RT * RT);
  for (int o = tid; o < 3 * N; o += BLOCK) {
    const int a = o / N, i = o % N;
    const double v = P.xi_min + i * P.dxi - M[1 + a];
    const double bse = amp * exp(-v * v * beta);
    sU[a * CSL * N + 0 * N + i] = (T)bse;
    sU[a * CSL * N + 1 * N + i] = (T)(bse * v);
    sU[a * CSL * N + 2 * N + i] = (T)(bse * v * v);
    sU[a * CSL * N + 3 * N + i] = (T)(bse * v * v * v);
  }
  for (int o = tid; o < 64; o += BLOCK) {
    const int k[3] = {o & 3, (o >> 2) & 3, o >> 4};
    double g = 0.0;
    int nz = 0, which = -1;
    for (int a = 0; a < 3; ++a)
      if (k[a]) { ++nz; which = a; }
    if (nz == 0) {
      g = 1.0;
    } else if (nz == 1) {
      if (k[which] == 1) g = -2.5 * As * M[5 + which];
      else if (k[which] == 3) g = As * beta * M[5 + which];
    } else if (nz == 2) {
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          if (a != b && k[a] == 1 && k[b] == 2 && k[3 - a - b] == 0) g = As * beta * M[5 + a];
    }
    sG[o] = (T)(scale * g);
  }
}

// General path (any ranks): sources restaged for every pass of fibres.
template <int N, int BLOCK, typename T>
__device__ void ob_slow(const DevState& d, const int c, T* Xc, T* smem) {
  constexpr int NPASS = N * N / BLOCK;
  static_assert(NPASS * BLOCK == N * N, "passes must tile the fibres");
  const int CS = d.CS;
  const int CSL = CS > kEstCap ? CS : kEstCap;
  T* sxi = smem;                  // N
  T* sd = sxi + N;                // 3 N   separable (axis-aligned) outflow tables
  T* sU = sd + 3 * N;             // 3 CSL N
  T* sG = sU + 3 * CSL * N;       // CSL^3
  T* sY = sG + CSL * CSL * CSL;   // KC CSL N
  T* sZ = sY + KC * CSL * N;      // KC BLOCK
  __shared__ double s_nrm[kSlots][3];
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const double nu = d.nu[c];
  ob_tables<N, BLOCK, T>(d, c, sxi, sd, s_nrm);
  __syncthreads();
  const double* M = d.macro + 8 * (size_t)c;
  for (int pass = 0; pass < NPASS; ++pass) {
    const int pbase = pass * BLOCK;
    const int p = pbase + tid;
    const int i2 = p % N, i3 = p / N;
    T acc[N], w[N], tmp[N];
    // ---- own-cell weight W
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] = 0;
    for (int l = 0; l < kSlots; ++l) {
      const int8_t kind = d.slot_kind[kSlots * c + l];
      if (kind == SK_NONE || d.slot_axis[kSlots * c + l] >= 0) continue;
      const int e = d.slot_est[kSlots * c + l];
      const int rr[3] = {d.est_rank[3 * e], d.est_rank[3 * e + 1], d.est_rank[3 * e + 2]};
      const double al = -0.5 * d.slot_coef[kSlots * c + l];
      stage_any<N, BLOCK, T>(d.est_core, d.est_fac, kEstCap, (size_t)e, rr, -1, -1, 0.0, 0.0, P.xi_min, P.dxi, al,
                             CSL, sU, sG);
      __syncthreads();
      expand_pass<N, BLOCK, T>(w, sU, sG, sY, sZ, rr[0], rr[1], rr[2], CSL, pbase);
    }
    {
      const T base = (T)(1.0 - P.dt * nu) + sd[N + i2] + sd[2 * N + i3];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double xn = 0.0;
        for (int l = 0; l < kSlots; ++l) {
          const int8_t kind = d.slot_kind[kSlots * c + l];
          if (kind == SK_NONE || d.slot_axis[kSlots * c + l] >= 0) continue;
          const double al = -0.5 * d.slot_coef[kSlots * c + l];
          xn += al * (s_nrm[l][0] * (double)sxi[i] + s_nrm[l][1] * (double)sxi[i2] + s_nrm[l][2] * (double)sxi[i3]);
        }
        w[i] += base + sd[i] + (T)xn;
      }
    }
    // ---- the cell itself, times W
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = 0;
    {
      const int rr[3] = {d.rank[3 * c], d.rank[3 * c + 1], d.rank[3 * c + 2]};
      stage_any<N, BLOCK, T>(d.core, d.fac, CS, (size_t)c, rr, -1, -1, 0.0, 0.0, P.xi_min, P.dxi, 1.0, CSL, sU, sG);
      __syncthreads();
      expand_pass<N, BLOCK, T>(acc, sU, sG, sY, sZ, rr[0], rr[1], rr[2], CSL, pbase);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] *= w[i];
    // ---- f_S, scaled by dt nu
    stage_fs_any<N, BLOCK, T>(M, P, P.dt * nu, CSL, sU, sG);
    __syncthreads();
    expand_pass<N, BLOCK, T>(acc, sU, sG, sY, sZ, 4, 4, 4, CSL, pbase);
    // ---- far sides
    for (int l = 0; l < kSlots; ++l) {
      const int8_t kind = d.slot_kind[kSlots * c + l];
      if (kind == SK_NONE) continue;
      const int ax = d.slot_axis[kSlots * c + l];
      const double sg = (double)d.slot_sig[kSlots * c + l];
      const double coef = d.slot_coef[kSlots * c + l];
      const int nb = d.slot_nb[kSlots * c + l];
      const bool obl = ax < 0;
      if (obl) {
        // B_l = a_l (xi_n - est_l) into w
        const int e = d.slot_est[kSlots * c + l];
        const int rr[3] = {d.est_rank[3 * e], d.est_rank[3 * e + 1], d.est_rank[3 * e + 2]};
        const double al = -0.5 * coef;
#pragma unroll
        for (int i = 0; i < N; ++i) w[i] = 0;
        stage_any<N, BLOCK, T>(d.est_core, d.est_fac, kEstCap, (size_t)e, rr, -1, -1, 0.0, 0.0, P.xi_min, P.dxi, -al,
                               CSL, sU, sG);
        __syncthreads();
        expand_pass<N, BLOCK, T>(w, sU, sG, sY, sZ, rr[0], rr[1], rr[2], CSL, pbase);
#pragma unroll
        for (int i = 0; i < N; ++i)
          w[i] += (T)(al * (s_nrm[l][0] * (double)sxi[i] + s_nrm[l][1] * (double)sxi[i2] +
                            s_nrm[l][2] * (double)sxi[i3]));
#pragma unroll
        for (int i = 0; i < N; ++i) tmp[i] = 0;
      }
      // the far side, row-scaled on axis-aligned faces, plain on oblique ones
      const double rc = obl ? 0.0 : coef;
      if (kind == SK_INTERIOR || kind == SK_OUTFLOW || kind == SK_SYM) {
        const int src = (kind == SK_INTERIOR) ? nb : c;
        const int rr[3] = {d.rank[3 * src], d.rank[3 * src + 1], d.rank[3 * src + 2]};
        stage_any<N, BLOCK, T>(d.core, d.fac, CS, (size_t)src, rr, kind == SK_SYM ? ax : -1, ax, rc, sg, P.xi_min,
                               P.dxi, 1.0, CSL, sU, sG);
        __syncthreads();
        if (obl) expand_pass<N, BLOCK, T>(tmp, sU, sG, sY, sZ, rr[0], rr[1], rr[2], CSL, pbase);
        else expand_pass<N, BLOCK, T>(acc, sU, sG, sY, sZ, rr[0], rr[1], rr[2], CSL, pbase);
      } else {
        const double gsc = (kind == SK_WALL) ? d.nw[kSlots * c + l] : 1.0;
        const double* bf = d.bc_fac + (size_t)nb * 3 * N;
        for (int o = tid; o < 3 * N; o += BLOCK) {
          const int a = o / N, i = o % N;
          double v = bf[o];
          if (a == ax && !obl) v *= coef * fmax(-sg * (P.xi_min + i * P.dxi), 0.0);
          sU[a * CSL * N + i] = (T)v;
        }
        if (tid == 0) sG[0] = (T)gsc;
        __syncthreads();
        if (obl) expand_pass<N, BLOCK, T>(tmp, sU, sG, sY, sZ, 1, 1, 1, CSL, pbase);
        else expand_pass<N, BLOCK, T>(acc, sU, sG, sY, sZ, 1, 1, 1, CSL, pbase);
      }
      if (obl) {
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] += tmp[i] * w[i];
      }
    }
    T* out = Xc + (size_t)p * N;
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = acc[i];
  }
}

// Cells whose sources fit the LDS budget take the one-stage path; the others
// are listed for k_expand_obl_general.
template <int N, int BLOCK, typename T>
__global__ __launch_bounds__(BLOCK) void k_expand_obl(DevState d, int c0, T* X, int lds_floats, int* list,
                                                      int* list_n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  T* sxi = smem;      // N
  T* sd = sxi + N;    // 3 N
  __shared__ double s_nrm[kSlots][3];
  __shared__ ObTab s_tab;
  if (d.cells && c0 + (int)blockIdx.x >= *d.cells_n) return;
  const int c = d.cells ? d.cells[c0 + blockIdx.x] : c0 + blockIdx.x;
  ob_tables<N, BLOCK, T>(d, c, sxi, sd, s_nrm);
  if (threadIdx.x == 0) ob_table(d, c, N, s_tab);
  __syncthreads();
  if (s_tab.need > lds_floats - 4 * N) {
    if (threadIdx.x == 0) list[atomicAdd(list_n, 1)] = blockIdx.x;
    return;
  }
  ob_fast<N, BLOCK, T>(d, c, X + (size_t)blockIdx.x * N * N * N, sxi, sd, sd + 3 * N, s_tab, s_nrm);
}

// The one-stage path with a larger LDS budget (one workgroup per CU) over the
// cells an earlier launch listed (pass-local indices in / in_n); the cells
// that still do not fit go to list / list_n.
template <int N, int BLOCK, typename T>
__global__ __launch_bounds__(BLOCK) void k_expand_obl_listed(DevState d, int c0, T* X, int lds_floats,
                                                             const int* in, const int* in_n, int* list,
                                                             int* list_n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  T* sxi = smem;      // N
  T* sd = sxi + N;    // 3 N
  __shared__ double s_nrm[kSlots][3];
  __shared__ ObTab s_tab;
  const int n = *in_n;
  for (int b = blockIdx.x; b < n; b += gridDim.x) {
    const int bi = in[b];
    const int c = d.cells ? d.cells[c0 + bi] : c0 + bi;
    ob_tables<N, BLOCK, T>(d, c, sxi, sd, s_nrm);
    if (threadIdx.x == 0) ob_table(d, c, N, s_tab);
    __syncthreads();
    if (s_tab.need > lds_floats - 4 * N) {
      if (threadIdx.x == 0) list[atomicAdd(list_n, 1)] = bi;
    } else {
      ob_fast<N, BLOCK, T>(d, c, X + (size_t)bi * N * N * N, sxi, sd, sd + 3 * N, s_tab, s_nrm);
    }
    __syncthreads();  // the tables are rewritten for the next cell
  }
}

template <int N, int BLOCK, typename T>
__global__ __launch_bounds__(BLOCK) void k_expand_obl_general(DevState d, int c0, T* X, const int* list,
                                                              const int* list_n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int n = *list_n;
  for (int b = blockIdx.x; b < n; b += gridDim.x) {
    const int bi = list[b];
    ob_slow<N, BLOCK, T>(d, d.cells ? d.cells[c0 + bi] : c0 + bi, X + (size_t)bi * N * N * N, smem);
    __syncthreads();
  }
}

__global__ void k_zero_count(int* p) { *p = 0; }

template <int N>
struct OblShape;
template <> struct OblShape<16> { static constexpr int B = 256; };
template <> struct OblShape<24> { static constexpr int B = 288; };
template <> struct OblShape<32> { static constexpr int B = 512; };
template <> struct OblShape<48> { static constexpr int B = 384; };

// ---- intermediate rounding of the face terms ---------------------------------
// The variant of the step that rounds each face's flux term on its own before
// the sum (the paper's placement of roundings after the rank-raising
// operations).  k_face_term expands the contribution of face slot l to the
// update, E_l = -(dt A_l / V) (P_out o f + P_in o g): on an axis-aligned face
// P_out = max(s xi_a, 0), P_in = min(s xi_a, 0); on an oblique one
// P_out/in = (xi_n +- est_l) / 2 with the |xi.e| estimate.  k_face_sum expands
// (1 - dt nu) f + dt nu f_S + sum_l E~_l from the rounded face terms.  Both use
// the general (any rank) staging of the oblique path; a cell without slot l
// gets E_l = 0.

// far side g of face slot l staged (the neighbour, the cell itself, the cell
// with the face axis reversed, or the rank-1 boundary Maxwellian)
template <int N, int BLOCK, typename T>
__device__ inline void stage_far(const DevState& d, int c, int l, const InstParams& P, int CSL, T* sU, T* sG,
                                 int (&q)[3]) {
  const int kind = d.slot_kind[kSlots * c + l];
  const int ax = d.slot_axis[kSlots * c + l];
  const int nb = d.slot_nb[kSlots * c + l];
  if (kind == SK_INTERIOR || kind == SK_OUTFLOW || kind == SK_SYM) {
    const int src = (kind == SK_INTERIOR) ? nb : c;
    q[0] = d.rank[3 * src];
    q[1] = d.rank[3 * src + 1];
    q[2] = d.rank[3 * src + 2];
    stage_any<N, BLOCK, T>(d.core, d.fac, d.CS, (size_t)src, q, kind == SK_SYM ? ax : -1, -1, 0.0, 0.0, P.xi_min,
                           P.dxi, 1.0, CSL, sU, sG);
  } else {
    q[0] = q[1] = q[2] = 1;
    const double gsc = (kind == SK_WALL) ? d.nw[kSlots * c + l] : 1.0;
    const double* bf = d.bc_fac + (size_t)nb * 3 * N;
    for (int o = threadIdx.x; o < 3 * N; o += BLOCK) sU[(o / N) * CSL * N + o % N] = (T)bf[o];
    if (threadIdx.x == 0) sG[0] = (T)gsc;
  }
}

template <int N, int BLOCK, typename T>
__global__ __launch_bounds__(BLOCK) void k_face_term(DevState d, int c0, T* X, int l) {
  constexpr int NPASS = N * N / BLOCK;
  static_assert(NPASS * BLOCK == N * N, "passes must tile the fibres");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int CS = d.CS;
  const int CSL = CS > kEstCap ? CS : kEstCap;
  T* sU = smem;                   // 3 CSL N
  T* sG = sU + 3 * CSL * N;       // CSL^3
  T* sY = sG + CSL * CSL * CSL;   // KC CSL N
  T* sZ = sY + KC * CSL * N;      // KC BLOCK
  __shared__ double s_nrm[3];
  const int cb = blockIdx.x;
  if (d.cells && c0 + cb >= *d.cells_n) return;
  const int c = d.cells ? d.cells[c0 + cb] : c0 + cb;
  const int tid = threadIdx.x;
  T* Xc = X + (size_t)cb * N * N * N;
  const int kind = d.slot_kind[kSlots * c + l];
  if (kind == SK_NONE) {
    for (int o = tid; o < N * N * N; o += BLOCK) Xc[o] = 0;
    return;
  }
  const InstParams P = d.ip[d.inst[c]];
  const int ax = d.slot_axis[kSlots * c + l];
  const double sg = (double)d.slot_sig[kSlots * c + l];
  const double cf = -d.slot_coef[kSlots * c + l];
  // outward normal of an oblique face (the table exists only on states with
  // oblique faces)
  if (ax < 0 && tid < 3) s_nrm[tid] = d.slot_nrm[((size_t)kSlots * c + l) * 3 + tid];
  const int rc[3] = {d.rank[3 * c], d.rank[3 * c + 1], d.rank[3 * c + 2]};
  for (int pass = 0; pass < NPASS; ++pass) {
    const int pbase = pass * BLOCK;
    const int p = pbase + tid;
    const int i2 = p % N, i3 = p / N;
    T f[N], g[N];
#pragma unroll
    for (int i = 0; i < N; ++i) f[i] = g[i] = 0;
    stage_any<N, BLOCK, T>(d.core, d.fac, CS, (size_t)c, rc, -1, -1, 0.0, 0.0, P.xi_min, P.dxi, 1.0, CSL, sU, sG);
    __syncthreads();
    expand_pass<N, BLOCK, T>(f, sU, sG, sY, sZ, rc[0], rc[1], rc[2], CSL, pbase);
    int q[3];
    stage_far<N, BLOCK, T>(d, c, l, P, CSL, sU, sG, q);
    __syncthreads();
    expand_pass<N, BLOCK, T>(g, sU, sG, sY, sZ, q[0], q[1], q[2], CSL, pbase);
    T* out = Xc + (size_t)p * N;
    if (ax >= 0) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int ia = ax == 0 ? i : (ax == 1 ? i2 : i3);
        const double x = sg * (P.xi_min + ia * P.dxi);
        out[i] = (T)cf * ((T)fmax(x, 0.0) * f[i] + (T)fmin(x, 0.0) * g[i]);
      }
    } else {
      T e[N];
#pragma unroll
      for (int i = 0; i < N; ++i) e[i] = 0;
      const int ei = d.slot_est[kSlots * c + l];
      const int re[3] = {d.est_rank[3 * ei], d.est_rank[3 * ei + 1], d.est_rank[3 * ei + 2]};
      stage_any<N, BLOCK, T>(d.est_core, d.est_fac, kEstCap, (size_t)ei, re, -1, -1, 0.0, 0.0, P.xi_min, P.dxi, 1.0,
                             CSL, sU, sG);
      __syncthreads();
      expand_pass<N, BLOCK, T>(e, sU, sG, sY, sZ, re[0], re[1], re[2], CSL, pbase);
      const double x2 = s_nrm[1] * (P.xi_min + i2 * P.dxi) + s_nrm[2] * (P.xi_min + i3 * P.dxi);
      const T h = (T)(0.5 * cf);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const T xn = (T)(s_nrm[0] * (P.xi_min + i * P.dxi) + x2);
        out[i] = h * ((xn + e[i]) * f[i] + (xn - e[i]) * g[i]);
      }
    }
  }
}

template <int N, int BLOCK, typename T>
__global__ __launch_bounds__(BLOCK) void k_face_sum(DevState d, FaceStates fs, int c0, T* X) {
  constexpr int NPASS = N * N / BLOCK;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int CS = d.CS;
  const int CSL = CS > kEstCap ? CS : kEstCap;
  T* sU = smem;
  T* sG = sU + 3 * CSL * N;
  T* sY = sG + CSL * CSL * CSL;
  T* sZ = sY + KC * CSL * N;
  const int cb = blockIdx.x;
  if (d.cells && c0 + cb >= *d.cells_n) return;
  const int c = d.cells ? d.cells[c0 + cb] : c0 + cb;
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const double nu = d.nu[c];
  const double* M = d.macro + 8 * (size_t)c;
  const int rc[3] = {d.rank[3 * c], d.rank[3 * c + 1], d.rank[3 * c + 2]};
  T* Xc = X + (size_t)cb * N * N * N;
  for (int pass = 0; pass < NPASS; ++pass) {
    const int pbase = pass * BLOCK;
    T acc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = 0;
    stage_any<N, BLOCK, T>(d.core, d.fac, CS, (size_t)c, rc, -1, -1, 0.0, 0.0, P.xi_min, P.dxi, 1.0 - P.dt * nu,
                           CSL, sU, sG);
    __syncthreads();
    expand_pass<N, BLOCK, T>(acc, sU, sG, sY, sZ, rc[0], rc[1], rc[2], CSL, pbase);
    stage_fs_any<N, BLOCK, T>(M, P, P.dt * nu, CSL, sU, sG);
    __syncthreads();
    expand_pass<N, BLOCK, T>(acc, sU, sG, sY, sZ, 4, 4, 4, CSL, pbase);
    for (int l = 0; l < kSlots; ++l) {
      if (d.slot_kind[kSlots * c + l] == SK_NONE) continue;
      const int q[3] = {fs.rank[l][3 * c], fs.rank[l][3 * c + 1], fs.rank[l][3 * c + 2]};
      stage_any<N, BLOCK, T>(fs.core[l], fs.fac[l], CS, (size_t)c, q, -1, -1, 0.0, 0.0, P.xi_min, P.dxi, 1.0, CSL,
                             sU, sG);
      __syncthreads();
      expand_pass<N, BLOCK, T>(acc, sU, sG, sY, sZ, q[0], q[1], q[2], CSL, pbase);
    }
    T* out = Xc + (size_t)(pbase + tid) * N;
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = acc[i];
  }
}

template <int N, typename T>
size_t face_lds(int CS) {
  const int CSL = CS > kEstCap ? CS : kEstCap;
  return sizeof(T) * (3 * (size_t)CSL * N + (size_t)CSL * CSL * CSL + (size_t)KC * CSL * N + (size_t)KC * OblShape<N>::B);
}

template <int N, typename T>
hipError_t launch_face_term_t(const DevState& d, int c0, int count, void* X, int slot, hipStream_t s) {
  constexpr int B = OblShape<N>::B;
  const size_t sh = face_lds<N, T>(d.CS);
  auto k = k_face_term<N, B, T>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(count), dim3(B), sh, s, d, c0, (T*)X, slot);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t launch_face_sum_t(const DevState& d, const FaceStates& fs, int c0, int count, void* X, hipStream_t s) {
  constexpr int B = OblShape<N>::B;
  const size_t sh = face_lds<N, T>(d.CS);
  auto k = k_face_sum<N, B, T>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(count), dim3(B), sh, s, d, fs, c0, (T*)X);
  return hipGetLastError();
}


template <int N, typename T>
hipError_t launch_expand_obl_t(const DevState& d, int c0, int count, void* X, int* list, int* list_n,
                               hipStream_t s) {
  constexpr int B = OblShape<N>::B;
  // one-stage path of low-rank cells: two workgroups per CU
  const size_t fast = (size_t)76 * 1024;
  auto kf = k_expand_obl<N, B, T>;
  hipError_t e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fast);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, list_n);
  hipLaunchKernelGGL(kf, dim3(count), dim3(B), fast, s, d, c0, (T*)X, (int)(fast / sizeof(T)), list, list_n);
  // the listed cells through the one-stage path with one workgroup's worth of
  // LDS per CU (list entries from `count` on, second counter), then the
  // cells left, any ranks, through the restaging path
  int* list2 = list + count;
  int* list2_n = list_n + 1;
  const size_t big = (size_t)150 * 1024;
  auto kb = k_expand_obl_listed<N, B, T>;
  e = hipFuncSetAttribute((const void*)kb, hipFuncAttributeMaxDynamicSharedMemorySize, (int)big);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, list2_n);
  hipLaunchKernelGGL(kb, dim3(count < 512 ? count : 512), dim3(B), big, s, d, c0, (T*)X, (int)(big / sizeof(T)),
                     (const int*)list, (const int*)list_n, list2, list2_n);
  const int CSL = d.CS > kEstCap ? d.CS : kEstCap;
  const size_t slow = sizeof(T) * (4 * N + 3 * CSL * N + CSL * CSL * CSL + KC * CSL * N + KC * B);
  auto ks = k_expand_obl_general<N, B, T>;
  e = hipFuncSetAttribute((const void*)ks, hipFuncAttributeMaxDynamicSharedMemorySize, (int)slow);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ks, dim3(count < 1024 ? count : 1024), dim3(B), slow, s, d, c0, (T*)X, list2, list2_n);
  return hipGetLastError();
}

// Plain expansion of state-layout Tucker tensors (rounding test hook).
template <int N, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_expand_plain(int CS, const double* core, const double* fac,
                                                        const int* rank, double* X) {
  constexpr int FIB = N * N / BLOCK;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* smem = reinterpret_cast<double*>(smem_raw);
  double* sU = smem;
  double* sG = sU + 3 * CS * N;
  double* sY = sG + CS * CS * CS;  // CS CS N
  const int c = blockIdx.x;
  int pf[FIB];
#pragma unroll
  for (int f = 0; f < FIB; ++f) pf[f] = threadIdx.x + BLOCK * f;
  // ranks clamped to 1..CS, so that device-resident ranks outside that range
  // (never produced by this library) keep every access inside the layout
  auto clampr = [CS](int r) { return r < 1 ? 1 : (r > CS ? CS : r); };
  const int r1 = clampr(rank[3 * c]), r2 = clampr(rank[3 * c + 1]), r3 = clampr(rank[3 * c + 2]);
  stage_state<N, BLOCK, double>(core, fac, CS, c, r1, r2, r3, -1, -1, nullptr, 1.0, sU, sG);
  __syncthreads();
  double acc[FIB][N];
#pragma unroll
  for (int f = 0; f < FIB; ++f)
#pragma unroll
    for (int i = 0; i < N; ++i) acc[f][i] = 0;
  expand_fibres<N, BLOCK, double, FIB>(acc, sU, sG, sY, r1, r2, r3, CS, pf);
  double* out = X + (size_t)c * N * N * N;
#pragma unroll
  for (int f = 0; f < FIB; ++f)
#pragma unroll
    for (int i = 0; i < N; ++i) out[(size_t)pf[f] * N + i] = acc[f][i];
}

template <int N>
struct ExpandShape;
template <> struct ExpandShape<16> { static constexpr int B = 256; };
template <> struct ExpandShape<24> { static constexpr int B = 576; };
template <> struct ExpandShape<32> { static constexpr int B = 512; };
template <> struct ExpandShape<48> { static constexpr int B = 768; };

// rank bound of the small-LDS expansion launch
constexpr int kExpRB = 8;

template <int N, typename T>
hipError_t launch_expand_t(const DevState& d, int c0, int count, void* X, int* list, int* list_n, hipStream_t s) {
  constexpr int B = ExpandShape<N>::B;
  const int CS = d.CS;
  constexpr bool MF = (N == 32 && B == 512 && ExpandSplit<N>::S == 2 && sizeof(T) == 4);
  const dim3 grid(count * ExpandSplit<N>::S);
  // LDS of k_expand_pipe for rank extent LS: tables, f_S, two buffers and,
  // on the MFMA path, each wave's Y slice instead of a shared Y
  auto pipe_lds = [&](int LS) -> size_t {
    const size_t b = 3 * LS * N + ((LS * LS * LS + 1) & ~1) + (MF ? 0 : LS * LS * N);
    return sizeof(T) * (3 * N + 3 * LS * N + 64 + 2 * b + (MF ? (B / 64) * 2 * LS * LS : 0));
  };
  if (CS > kExpRB && list && list_n && pipe_lds(CS) <= (size_t)150 * 1024) {
    // cells whose sources all have ranks <= kExpRB: a small LDS layout, three
    // workgroups per CU; the rest through the full layout, from the list
    constexpr int RB = kExpRB;
    const size_t ss = pipe_lds(RB);
    const size_t sl = pipe_lds(CS);
    auto kf = k_expand_pipe<N, B, T, MF, RB, 1>;
    auto kl = k_expand_pipe<N, B, T, MF, 0, 2>;
    hipError_t e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ss);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)kl, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sl);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, list_n);
    hipLaunchKernelGGL(kf, grid, dim3(B), ss, s, d, c0, (T*)X, list, list_n);
    hipLaunchKernelGGL(kl, grid, dim3(B), sl, s, d, c0, (T*)X, list, list_n);
    return hipGetLastError();
  }
  const size_t sp = pipe_lds(CS);
  if (sp <= 80 * 1024) {
    // two buffers still leave room for two workgroups per CU
    auto k = k_expand_pipe<N, B, T, MF, 0, 0>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sp);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, grid, dim3(B), sp, s, d, c0, (T*)X, (int*)nullptr, (int*)nullptr);
    return hipGetLastError();
  }
  const size_t sh = sizeof(T) * (N + 3 * N + N + 3 * CS * N + CS * CS * CS + CS * CS * N + 3 * CS * N + 64);
  auto k = k_expand<N, B, T>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(count * ExpandSplit<N>::S), dim3(B), sh, s, d, c0, (T*)X, LuArgs{});
  return hipGetLastError();
}

// LU-SGS backward stage and commit of one cell each (fibre form, in the
// workspace type T: FP64, or FP32 on the mixed path): backward
// X = df*_i + D^-1 sum_{upper far cells} b_l o df_m, with b_l the explicit
// step's far-side row scaling; commit X = f_i + df_i.
template <int N, int BLOCK, typename T>
__global__ __launch_bounds__(BLOCK) void k_lu_combine(DevState d, LuArgs lu, int c0, T* X, int stage) {
  constexpr int FIB = N * N / BLOCK;
  static_assert(FIB * BLOCK == N * N, "fibres must tile the workgroup");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int CS = d.CS;
  T* sU = smem;                  // 3 CS N
  T* sG = sU + 3 * CS * N;       // CS^3
  T* sY = sG + CS * CS * CS;     // CS CS N
  T* sb = sY + CS * CS * N;      // N
  const int cb = blockIdx.x;
  if (d.cells && c0 + cb >= *d.cells_n) return;
  const int c = d.cells ? d.cells[c0 + cb] : c0 + cb;
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  int pf[FIB];
#pragma unroll
  for (int f = 0; f < FIB; ++f) pf[f] = tid + BLOCK * f;
  T acc[FIB][N];
#pragma unroll
  for (int f = 0; f < FIB; ++f)
#pragma unroll
    for (int i = 0; i < N; ++i) acc[f][i] = (T)0;
  if (stage == LU_BACKWARD) {
    for (int l = 0; l < kSlots; ++l) {
      if (d.slot_kind[kSlots * c + l] != SK_INTERIOR) continue;
      const int nb = d.slot_nb[kSlots * c + l];
      if (lu.col[nb] <= lu.colour) continue;
      const int ax = d.slot_axis[kSlots * c + l];
      const double sg = (double)d.slot_sig[kSlots * c + l];
      const double coef = d.slot_coef[kSlots * c + l];
      for (int i = tid; i < N; i += BLOCK) sb[i] = (T)(coef * fmax(-sg * (P.xi_min + i * P.dxi), 0.0));
      __syncthreads();
      const int q1 = lu.rank[3 * nb], q2 = lu.rank[3 * nb + 1], q3 = lu.rank[3 * nb + 2];
      stage_state<N, BLOCK, T>(lu.core, lu.fac, CS, nb, q1, q2, q3, -1, ax, sb, 1.0, sU, sG);
      __syncthreads();
      expand_fibres<N, BLOCK, T, FIB>(acc, sU, sG, sY, q1, q2, q3, CS, pf);
      __syncthreads();
    }
    const double* di = lu.dinv + (size_t)c * (N + 1);
    for (int i = tid; i < N; i += BLOCK) sb[i] = (T)di[i];
    __syncthreads();
    const T isg = (T)di[N];
#pragma unroll
    for (int f = 0; f < FIB; ++f) {
      const T w = sb[pf[f] % N] * sb[pf[f] / N] * isg;
#pragma unroll
      for (int i = 0; i < N; ++i) acc[f][i] *= sb[i] * w;
    }
  } else {
    const int r1 = d.rank[3 * c], r2 = d.rank[3 * c + 1], r3 = d.rank[3 * c + 2];
    stage_state<N, BLOCK, T>(d.core, d.fac, CS, c, r1, r2, r3, -1, -1, nullptr, 1.0, sU, sG);
    __syncthreads();
    expand_fibres<N, BLOCK, T, FIB>(acc, sU, sG, sY, r1, r2, r3, CS, pf);
    __syncthreads();
  }
  // the cell's own increment (df* in the backward stage, df in the commit)
  const int q1 = lu.rank[3 * c], q2 = lu.rank[3 * c + 1], q3 = lu.rank[3 * c + 2];
  stage_state<N, BLOCK, T>(lu.core, lu.fac, CS, c, q1, q2, q3, -1, -1, nullptr, 1.0, sU, sG);
  __syncthreads();
  expand_fibres<N, BLOCK, T, FIB>(acc, sU, sG, sY, q1, q2, q3, CS, pf);
  T* out = X + (size_t)cb * N * N * N;
#pragma unroll
  for (int f = 0; f < FIB; ++f)
#pragma unroll
    for (int i = 0; i < N; ++i) out[(size_t)pf[f] * N + i] = acc[f][i];
}

// The rank-1 truncated HOSVD of D = a 1 + b |xi| (a = 1 + dt nu, b = (dt /
// (2 V)) sum_l A_l): by the symmetry of |xi| in the three velocity axes the
// three factors are one vector u, the leading eigenvector of the mode-1
// Gram a^2 N^2 1 1^T + a b (1 p^T + p 1^T) + b^2 Q, found by power
// iteration from the positive start (the Gram is positive, so u is); the
// core is D x u x u x u = a (sum u)^3 + b sum |xi|(i,j,k) u_i u_j u_k.  One
// wavefront per cell.
__device__ inline double lu_wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <int N>
__global__ __launch_bounds__(64) void k_lu_diag(DevState d, const double* pq, double* dinv) {
  __shared__ double sp[N], sQ[N * N], su[N];
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const int k = d.inst[c];
  const InstParams P = d.ip[k];
  const double* pk = pq + (size_t)k * (N + N * N);
  for (int o = lane; o < N + N * N; o += 64) {
    if (o < N) sp[o] = pk[o];
    else sQ[o - N] = pk[o];
  }
  double b = 0.0;
  if (lane < kSlots && d.slot_kind[kSlots * c + lane] != SK_NONE) b = 0.5 * d.slot_coef[kSlots * c + lane];
  b = lu_wave_sum(b);
  const double a = 1.0 + P.dt * d.nu[c];
  const double t = b / a;
  double u = lane < N ? 1.0 / sqrt((double)N) : 0.0;
  wave_sync();
  for (int it = 0; it < 200; ++it) {
    if (lane < N) su[lane] = u;
    wave_sync();
    const double s1 = lu_wave_sum(u);
    const double pu = lu_wave_sum(lane < N ? sp[lane] * u : 0.0);
    double v = 0.0;
    if (lane < N) {
      double qu = 0.0;
      for (int j = 0; j < N; ++j) qu += sQ[lane * N + j] * su[j];
      v = (double)(N * N) * s1 + t * (pu + s1 * sp[lane]) + t * t * qu;
    }
    v /= sqrt(lu_wave_sum(v * v));
    const double moved = lu_wave_sum(fabs(v - u) > 1e-16 ? 1.0 : 0.0);
    wave_sync();
    u = v;
    if (moved == 0.0) break;
  }
  if (lane < N) su[lane] = u;
  wave_sync();
  double acc = 0.0;
  for (int o = lane; o < N * N; o += 64) {
    const int i = o / N, j = o % N;
    const double xi = P.xi_min + i * P.dxi, xj = P.xi_min + j * P.dxi;
    double sk = 0.0;
    for (int q = 0; q < N; ++q) {
      const double xk = P.xi_min + q * P.dxi;
      sk += sqrt(xi * xi + xj * xj + xk * xk) * su[q];
    }
    acc += su[i] * su[j] * sk;
  }
  const double s3 = lu_wave_sum(acc);
  const double s1 = lu_wave_sum(u);
  const double sigma = a * s1 * s1 * s1 + b * s3;
  double* out = dinv + (size_t)c * (N + 1);
  if (lane < N) out[lane] = 1.0 / u;
  if (lane == 0) out[N] = 1.0 / sigma;
}

template <int N, typename T>
hipError_t launch_lu_t(const DevState& d, const LuArgs& lu, int stage, int c0, int count, T* X, hipStream_t s) {
  constexpr int B = ExpandShape<N>::B;
  const int CS = d.CS;
  if (stage == LU_FORWARD) {
    const size_t sh = sizeof(T) * (N + 3 * N + N + 3 * CS * N + CS * CS * CS + CS * CS * N + 3 * CS * N + 64);
    auto k = k_expand<N, B, T, true>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(count * ExpandSplit<N>::S), dim3(B), sh, s, d, c0, X, lu);
    return hipGetLastError();
  }
  const size_t sh = sizeof(T) * (3 * CS * N + CS * CS * CS + CS * CS * N + N);
  auto k = k_lu_combine<N, B, T>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(count), dim3(B), sh, s, d, lu, c0, X, stage);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_expand(const DevState& d, int c0, int count, void* X, int mixed, int oblique, int* list,
                         int* list_n, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (oblique) {
    if (mixed) {
      switch (d.N) {
        case 16: return launch_expand_obl_t<16, float>(d, c0, count, X, list, list_n, s);
        case 24: return launch_expand_obl_t<24, float>(d, c0, count, X, list, list_n, s);
        case 32: return launch_expand_obl_t<32, float>(d, c0, count, X, list, list_n, s);
        case 48: return launch_expand_obl_t<48, float>(d, c0, count, X, list, list_n, s);
      }
    } else {
      switch (d.N) {
        case 16: return launch_expand_obl_t<16, double>(d, c0, count, X, list, list_n, s);
        case 24: return launch_expand_obl_t<24, double>(d, c0, count, X, list, list_n, s);
        case 32: return launch_expand_obl_t<32, double>(d, c0, count, X, list, list_n, s);
        case 48: return launch_expand_obl_t<48, double>(d, c0, count, X, list, list_n, s);
      }
    }
    return hipErrorInvalidValue;
  }
  if (mixed) {
    switch (d.N) {
      case 16: return launch_expand_t<16, float>(d, c0, count, X, list, list_n, s);
      case 24: return launch_expand_t<24, float>(d, c0, count, X, list, list_n, s);
      case 32: return launch_expand_t<32, float>(d, c0, count, X, list, list_n, s);
      case 48: return launch_expand_t<48, float>(d, c0, count, X, list, list_n, s);
    }
  } else {
    switch (d.N) {
      case 16: return launch_expand_t<16, double>(d, c0, count, X, list, list_n, s);
      case 24: return launch_expand_t<24, double>(d, c0, count, X, list, list_n, s);
      case 32: return launch_expand_t<32, double>(d, c0, count, X, list, list_n, s);
      // the axis-face kernels' FP64 layouts do not fit the LDS at N = 48: the
      // general path of oblique meshes (separable tables for axis faces)
      case 48: return launch_expand_obl_t<48, double>(d, c0, count, X, list, list_n, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_face_term(const DevState& d, int c0, int count, void* X, int mixed, int slot, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (slot < 0 || slot >= kSlots) return hipErrorInvalidValue;
  if (mixed) {
    switch (d.N) {
      case 16: return launch_face_term_t<16, float>(d, c0, count, X, slot, s);
      case 24: return launch_face_term_t<24, float>(d, c0, count, X, slot, s);
      case 32: return launch_face_term_t<32, float>(d, c0, count, X, slot, s);
      case 48: return launch_face_term_t<48, float>(d, c0, count, X, slot, s);
    }
  } else {
    switch (d.N) {
      case 16: return launch_face_term_t<16, double>(d, c0, count, X, slot, s);
      case 24: return launch_face_term_t<24, double>(d, c0, count, X, slot, s);
      case 32: return launch_face_term_t<32, double>(d, c0, count, X, slot, s);
      case 48: return launch_face_term_t<48, double>(d, c0, count, X, slot, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_face_sum(const DevState& d, const FaceStates& fs, int c0, int count, void* X, int mixed,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (mixed) {
    switch (d.N) {
      case 16: return launch_face_sum_t<16, float>(d, fs, c0, count, X, s);
      case 24: return launch_face_sum_t<24, float>(d, fs, c0, count, X, s);
      case 32: return launch_face_sum_t<32, float>(d, fs, c0, count, X, s);
      case 48: return launch_face_sum_t<48, float>(d, fs, c0, count, X, s);
    }
  } else {
    switch (d.N) {
      case 16: return launch_face_sum_t<16, double>(d, fs, c0, count, X, s);
      case 24: return launch_face_sum_t<24, double>(d, fs, c0, count, X, s);
      case 32: return launch_face_sum_t<32, double>(d, fs, c0, count, X, s);
      case 48: return launch_face_sum_t<48, double>(d, fs, c0, count, X, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_lu_expand(const DevState& d, const LuArgs& lu, int stage, int c0, int count, void* X, int mixed,
                            hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (mixed) {
    switch (d.N) {
      case 16: return launch_lu_t<16, float>(d, lu, stage, c0, count, (float*)X, s);
      case 24: return launch_lu_t<24, float>(d, lu, stage, c0, count, (float*)X, s);
      case 32: return launch_lu_t<32, float>(d, lu, stage, c0, count, (float*)X, s);
    }
  } else {
    switch (d.N) {
      case 16: return launch_lu_t<16, double>(d, lu, stage, c0, count, (double*)X, s);
      case 24: return launch_lu_t<24, double>(d, lu, stage, c0, count, (double*)X, s);
      case 32: return launch_lu_t<32, double>(d, lu, stage, c0, count, (double*)X, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_lu_diag(const DevState& d, const double* pq, double* dinv, hipStream_t s) {
  if (d.n_cells <= 0) return hipSuccess;
  switch (d.N) {
    case 16: hipLaunchKernelGGL(k_lu_diag<16>, dim3(d.n_cells), dim3(64), 0, s, d, pq, dinv); break;
    case 24: hipLaunchKernelGGL(k_lu_diag<24>, dim3(d.n_cells), dim3(64), 0, s, d, pq, dinv); break;
    case 32: hipLaunchKernelGGL(k_lu_diag<32>, dim3(d.n_cells), dim3(64), 0, s, d, pq, dinv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_expand_plain(int N, int count, int CS, const double* core, const double* fac,
                               const int* rank, double* X, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const size_t sh = sizeof(double) * (3 * CS * N + CS * CS * CS + CS * CS * N);
#define TK_XP(NN, BB)                                                                                       \
  do {                                                                                                      \
    auto k = k_expand_plain<NN, BB>;                                                                        \
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh); \
    if (e != hipSuccess) return e;                                                                          \
    hipLaunchKernelGGL(k, dim3(count), dim3(BB), sh, s, CS, core, fac, rank, X);                            \
  } while (0)
  switch (N) {
    case 16: TK_XP(16, 256); break;
    case 24: TK_XP(24, 288); break;
    case 32: TK_XP(32, 512); break;
    default: return hipErrorInvalidValue;
  }
#undef TK_XP
  return hipGetLastError();
}

}  // namespace tk
