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
// LDS in chunks of the first rank index; the last product accumulates
// straight into registers: each thread owns whole mode-1 fibres of f*.
// f_S is built directly in Tucker form with mode ranks 4: columns
// m_a(xi) (xi - u_a)^k, k = 0..3, and a 4x4x4 core with 13 non-zeros
// (the expansion of f_M [1 + A_s (q.v)(v^2/(2 R_g T) - 5/2)]).
#include "tk_internal.h"

namespace tk {

namespace {

constexpr int KC = 4;  // rank-1 chunk of the staged mode products

// One source into the fibre accumulators: Y = G x3 U3 (all r1 x r2 x N in
// LDS), then each thread forms z_j = sum_k2 U2[i2,k2] Y[j,k2,i3] for its own
// fibres and adds U1[:,j] z_j.  One barrier between Y and its use; the
// caller separates sources with a barrier before restaging.
template <int N, int BLOCK, typename T, int FIB>
__device__ inline void expand_fibres(T (&acc)[FIB][N], const T* sU, const T* sG, T* sY, int r1, int r2, int r3,
                                     int CS, const int (&pf)[FIB]) {
  const T* U1 = sU;
  const T* U2 = sU + CS * N;
  const T* U3 = sU + 2 * CS * N;
  const int tid = threadIdx.x;
  for (int o = tid; o < r1 * r2 * N; o += BLOCK) {
    const int i3 = o % N, t = o / N, k2 = t % r2, j = t / r2;
    T sacc = 0;
    const T* g = sG + j + r1 * k2;
    for (int k3 = 0; k3 < r3; ++k3) sacc += g[r1 * r2 * k3] * U3[k3 * N + i3];
    sY[o] = sacc;
  }
  __syncthreads();
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

template <int N, int BLOCK, typename T>
__global__ __launch_bounds__(BLOCK) void k_expand(DevState d, int c0, T* X) {
  constexpr int FIB = N * N / BLOCK;
  static_assert(FIB * BLOCK == N * N, "fibres must tile the block");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int CS = d.CS;
  T* sxi = smem;                  // N
  T* sd = sxi + N;                // 3 N   own-cell outflow tables d_a
  T* sb = sd + 3 * N;             // N     row scaling of the current source
  T* sU = sb + N;                 // 3 CS N
  T* sG = sU + 3 * CS * N;        // CS^3
  T* sY = sG + CS * CS * CS;      // CS CS N
  const int c = c0 + blockIdx.x;
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const double nu = d.nu[c];
  int pf[FIB];
#pragma unroll
  for (int f = 0; f < FIB; ++f) pf[f] = tid + BLOCK * f;

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
    const T cterm = (T)(1.0 - P.dt * nu);
#pragma unroll
    for (int f = 0; f < FIB; ++f) {
      const T dd = cterm + sd[N + pf[f] % N] + sd[2 * N + pf[f] / N];
#pragma unroll
      for (int i = 0; i < N; ++i) acc[f][i] *= (sd[i] + dd);
    }
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
      sU[a * CS * N + 0 * N + i] = (T)base;
      sU[a * CS * N + 1 * N + i] = (T)(base * v);
      sU[a * CS * N + 2 * N + i] = (T)(base * v * v);
      sU[a * CS * N + 3 * N + i] = (T)(base * v * v * v);
    }
    for (int o = tid; o < 64; o += BLOCK) sG[o] = 0;
    __syncthreads();
    if (tid == 0) {
      const double s = P.dt * nu;
      sG[0] = (T)s;
      for (int a = 0; a < 3; ++a) {
        const double qa = M[5 + a];
        int st = (a == 0) ? 1 : (a == 1 ? 4 : 16);
        sG[1 * st] += (T)(s * -2.5 * As * qa);
        sG[3 * st] += (T)(s * As * beta * qa);
        for (int b = 0; b < 3; ++b) {
          if (b == a) continue;
          const int sb2 = (b == 0) ? 1 : (b == 1 ? 4 : 16);
          sG[1 * st + 2 * sb2] += (T)(s * As * beta * qa);
        }
      }
    }
    __syncthreads();
    expand_fibres<N, BLOCK, T, FIB>(acc, sU, sG, sY, 4, 4, 4, CS, pf);
    __syncthreads();
  }

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

  T* out = X + (size_t)blockIdx.x * N * N * N;
#pragma unroll
  for (int f = 0; f < FIB; ++f)
#pragma unroll
    for (int i = 0; i < N; ++i) out[(size_t)pf[f] * N + i] = acc[f][i];
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

template <int N, int BLOCK, typename T>
__global__ __launch_bounds__(BLOCK) void k_expand_obl(DevState d, int c0, T* X) {
  constexpr int NPASS = N * N / BLOCK;
  static_assert(NPASS * BLOCK == N * N, "passes must tile the fibres");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int CS = d.CS;
  const int CSL = CS > kEstCap ? CS : kEstCap;
  T* sxi = smem;                  // N
  T* sd = sxi + N;                // 3 N   separable (axis-aligned) outflow tables
  T* sU = sd + 3 * N;             // 3 CSL N
  T* sG = sU + 3 * CSL * N;       // CSL^3
  T* sY = sG + CSL * CSL * CSL;   // KC CSL N
  T* sZ = sY + KC * CSL * N;      // KC BLOCK
  __shared__ double s_nrm[kSlots][3];
  const int c = c0 + blockIdx.x;
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const double nu = d.nu[c];
  if (tid < kSlots * 3) s_nrm[tid / 3][tid % 3] = d.slot_nrm[(size_t)kSlots * 3 * c + tid];
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
    {
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
        sG[o] = (T)(P.dt * nu * g);
      }
      __syncthreads();
      expand_pass<N, BLOCK, T>(acc, sU, sG, sY, sZ, 4, 4, 4, CSL, pbase);
    }
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
    T* out = X + (size_t)blockIdx.x * N * N * N + (size_t)p * N;
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = acc[i];
  }
}

template <int N>
struct OblShape;
template <> struct OblShape<16> { static constexpr int B = 256; };
template <> struct OblShape<24> { static constexpr int B = 288; };
template <> struct OblShape<32> { static constexpr int B = 512; };
template <> struct OblShape<48> { static constexpr int B = 384; };

template <int N, typename T>
hipError_t launch_expand_obl_t(const DevState& d, int c0, int count, void* X, hipStream_t s) {
  constexpr int B = OblShape<N>::B;
  const int CSL = d.CS > kEstCap ? d.CS : kEstCap;
  const size_t sh = sizeof(T) * (4 * N + 3 * CSL * N + CSL * CSL * CSL + KC * CSL * N + KC * B);
  auto k = k_expand_obl<N, B, T>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(count), dim3(B), sh, s, d, c0, (T*)X);
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
  const int r1 = rank[3 * c], r2 = rank[3 * c + 1], r3 = rank[3 * c + 2];
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
template <> struct ExpandShape<24> { static constexpr int B = 288; };
template <> struct ExpandShape<32> { static constexpr int B = 512; };
template <> struct ExpandShape<48> { static constexpr int B = 768; };

template <int N, typename T>
hipError_t launch_expand_t(const DevState& d, int c0, int count, void* X, hipStream_t s) {
  constexpr int B = ExpandShape<N>::B;
  const int CS = d.CS;
  const size_t sh = sizeof(T) * (N + 3 * N + N + 3 * CS * N + CS * CS * CS + CS * CS * N);
  auto k = k_expand<N, B, T>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(count), dim3(B), sh, s, d, c0, (T*)X);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_expand(const DevState& d, int c0, int count, void* X, int mixed, int oblique, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (oblique) {
    if (mixed) {
      switch (d.N) {
        case 16: return launch_expand_obl_t<16, float>(d, c0, count, X, s);
        case 24: return launch_expand_obl_t<24, float>(d, c0, count, X, s);
        case 32: return launch_expand_obl_t<32, float>(d, c0, count, X, s);
        case 48: return launch_expand_obl_t<48, float>(d, c0, count, X, s);
      }
    } else {
      switch (d.N) {
        case 16: return launch_expand_obl_t<16, double>(d, c0, count, X, s);
        case 24: return launch_expand_obl_t<24, double>(d, c0, count, X, s);
        case 32: return launch_expand_obl_t<32, double>(d, c0, count, X, s);
      }
    }
    return hipErrorInvalidValue;
  }
  if (mixed) {
    switch (d.N) {
      case 16: return launch_expand_t<16, float>(d, c0, count, X, s);
      case 24: return launch_expand_t<24, float>(d, c0, count, X, s);
      case 32: return launch_expand_t<32, float>(d, c0, count, X, s);
      case 48: return launch_expand_t<48, float>(d, c0, count, X, s);
    }
  } else {
    switch (d.N) {
      case 16: return launch_expand_t<16, double>(d, c0, count, X, s);
      case 24: return launch_expand_t<24, double>(d, c0, count, X, s);
      case 32: return launch_expand_t<32, double>(d, c0, count, X, s);
    }
  }
  return hipErrorInvalidValue;
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
