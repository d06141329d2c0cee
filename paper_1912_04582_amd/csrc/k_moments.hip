// Macroparameters of every cell from its Tucker state, plus the wall ghost
// densities, and the rank-1 Maxwellian initial state.
//
// Moments (Alg. 2, its moment part) are Op5 convolutions: per mode the factor
// columns are summed against 1-D weights (1, xi, xi^2 and the central
// powers (xi - u_a)^p, p <= 3), then the core is contracted with those
// sums.  T uses central second moments (equal to Alg. 2's raw form in
// exact arithmetic, better conditioned for fast flows).  The collision
// frequency is nu = p / mu(T), p = m n R_g T, mu = (Kn / 2) T^omega.
//
// Wall ghosts (diffuse reflection, eq. wall-bc-f with the impermeability
// condition): n_w = -<P_out, f> / <P_in, f_w1> with P_out = max(s xi_a, 0)
// and P_in = min(s xi_a, 0) on a wall whose outward normal is s e_a, f_w1
// the unit-density wall Maxwellian.
#include "tk_internal.h"

namespace tk {

namespace {

constexpr int kMomThreads = 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The cell's core, held by the wave: entry o = lane + 64 m in register slot
// m (with its packed indices) for m < kMomGR, cores beyond that read from
// global memory.  Keeping it out of LDS leaves room for more cells per CU.
constexpr int kMomGR = 8;

struct CoreRegs {
  double g[kMomGR];
  int k[kMomGR];  // k1 | k2 << 8 | k3 << 16
  const double* G;  // the cell's core in global memory (layout k1 + CS (k2 + CS k3))
  int r1, r2, tot, CS;
};

__device__ inline void core_load(CoreRegs& R, const double* G, int r1, int r2, int r3, int CS) {
  R.G = G;
  R.r1 = r1;
  R.r2 = r2;
  R.tot = r1 * r2 * r3;
  R.CS = CS;
#pragma unroll
  for (int m = 0; m < kMomGR; ++m) {
    const int o = threadIdx.x + kMomThreads * m;
    R.g[m] = 0.0;
    R.k[m] = 0;
    if (o < R.tot) {
      const int k1 = o % r1, t = o / r1, k2 = t % r2, k3 = t / r2;
      R.g[m] = G[k1 + CS * (k2 + CS * k3)];
      R.k[m] = k1 | (k2 << 8) | (k3 << 16);
    }
  }
}

// sum_k G[k1, k2, k3] s1[k1] s2[k2] s3[k3] over the core entries in the
// order o = k1 + r1 (k2 + r2 k3), reduced over the wave
__device__ inline double contract(const CoreRegs& R, const double* s1, const double* s2, const double* s3) {
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < kMomGR; ++m) {
    const int o = threadIdx.x + kMomThreads * m;
    if (o < R.tot) {
      const int kk = R.k[m];
      acc += R.g[m] * s1[kk & 255] * s2[(kk >> 8) & 255] * s3[kk >> 16];
    }
  }
  for (int o = threadIdx.x + kMomThreads * kMomGR; o < R.tot; o += kMomThreads) {
    const int k1 = o % R.r1, t = o / R.r1, k2 = t % R.r2, k3 = t / R.r2;
    acc += R.G[k1 + R.CS * (k2 + R.CS * k3)] * s1[k1] * s2[k2] * s3[k3];
  }
  return wave_sum(acc);
}

template <int N>
__global__ __launch_bounds__(kMomThreads, 4) void k_moments(DevState d) {
  extern __shared__ double smem[];
  const int CS = d.CS;
  double* sU = smem;                 // [3][CS][N]
  double* sS = sU + 3 * CS * N;      // weighted sums [3][8][CS]
  double* sxi = sS + 3 * 8 * CS;     // [N]
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  if (P.frozen) return;  // macroparameters kept as they were
  const int r1 = d.rank[3 * c], r2 = d.rank[3 * c + 1], r3 = d.rank[3 * c + 2];
  const int rr[3] = {r1, r2, r3};
  for (int o = tid; o < N; o += kMomThreads) sxi[o] = P.xi_min + o * P.dxi;
  for (int a = 0; a < 3; ++a)
    for (int o = tid; o < rr[a] * N; o += kMomThreads)
      sU[a * CS * N + o] = d.fac[((size_t)c * 3 + a) * CS * N + o];
  CoreRegs sG;
  core_load(sG, d.core + (size_t)c * CS * CS * CS, r1, r2, r3, CS);
  __syncthreads();
  // raw weighted sums: sS[a][p][k] = dxi * sum_i U_a[k][i] xi_i^p, p = 0, 1, 2
  for (int o = tid; o < 3 * 3 * CS; o += kMomThreads) {
    const int k = o % CS, p = (o / CS) % 3, a = o / (3 * CS);
    double s = 0.0;
    if (k < rr[a]) {
      const double* u = sU + a * CS * N + k * N;
      #pragma unroll 4
      for (int i = 0; i < N; ++i) {
        const double x = sxi[i];
        s += u[i] * (p == 0 ? 1.0 : (p == 1 ? x : x * x));
      }
    }
    sS[(a * 8 + p) * CS + k] = s * P.dxi;
  }
  __syncthreads();
  auto S = [&](int a, int p) { return sS + (a * 8 + p) * CS; };
  const double n = contract(sG, S(0, 0), S(1, 0), S(2, 0));
  double u[3];
  u[0] = contract(sG, S(0, 1), S(1, 0), S(2, 0)) / n;
  u[1] = contract(sG, S(0, 0), S(1, 1), S(2, 0)) / n;
  u[2] = contract(sG, S(0, 0), S(1, 0), S(2, 1)) / n;
  __syncthreads();
  // central weighted sums: slots p = 3..5 hold (xi - u_a)^1..3
  for (int o = tid; o < 3 * 3 * CS; o += kMomThreads) {
    const int k = o % CS, p = (o / CS) % 3 + 1, a = o / (3 * CS);
    double s = 0.0;
    if (k < rr[a]) {
      const double* uu = sU + a * CS * N + k * N;
      #pragma unroll 4
      for (int i = 0; i < N; ++i) {
        const double v = sxi[i] - u[a];
        s += uu[i] * (p == 1 ? v : (p == 2 ? v * v : v * v * v));
      }
    }
    sS[(a * 8 + 2 + p) * CS + k] = s * P.dxi;
  }
  __syncthreads();
  auto C = [&](int a, int p) { return p == 0 ? S(a, 0) : sS + (a * 8 + 2 + p) * CS; };
  const double c2 = contract(sG, C(0, 2), C(1, 0), C(2, 0)) +
                    contract(sG, C(0, 0), C(1, 2), C(2, 0)) +
                    contract(sG, C(0, 0), C(1, 0), C(2, 2));
  const double T = c2 / (3.0 * n * P.Rg);
  double q[3];
  for (int a = 0; a < 3; ++a) {
    const double* w[3];
    for (int b = 0; b < 3; ++b) w[b] = C(b, 0);
    w[a] = C(a, 3);
    double acc = contract(sG, w[0], w[1], w[2]);
    for (int b = 0; b < 3; ++b) {
      if (b == a) continue;
      for (int e = 0; e < 3; ++e) w[e] = C(e, 0);
      w[a] = C(a, 1);
      w[b] = C(b, 2);
      acc += contract(sG, w[0], w[1], w[2]);
    }
    q[a] = 0.5 * P.m * acc;
  }
  const double p = P.m * n * P.Rg * T;
  const double nu = (P.Kn == INFINITY) ? 0.0 : p / (0.5 * P.Kn * pow(T, P.omega));
  if (tid == 0) {
    double* M = d.macro + 8 * (size_t)c;
    M[0] = n; M[1] = u[0]; M[2] = u[1]; M[3] = u[2]; M[4] = T;
    M[5] = q[0]; M[6] = q[1]; M[7] = q[2];
    d.nu[c] = nu;
    const bool ok = (n > 0.0) && (T > 0.0) && isfinite(n) && isfinite(T) && isfinite(u[0]) &&
                    isfinite(u[1]) && isfinite(u[2]) && isfinite(q[0]) && isfinite(q[1]) &&
                    isfinite(q[2]);
    if (!ok) atomicOr(&d.flag[d.inst[c]], 1);
  }
  // wall ghost densities
  for (int l = 0; l < kSlots; ++l) {
    if (d.slot_kind[kSlots * c + l] != SK_WALL) continue;
    const int a = d.slot_axis[kSlots * c + l];
    const double sg = (double)d.slot_sig[kSlots * c + l];
    __syncthreads();
    double* sw = sS + (a * 8 + 7) * CS;  // scratch slot 7 of mode a
    for (int k = tid; k < CS; k += kMomThreads) {
      double s = 0.0;
      if (k < rr[a]) {
        const double* uu = sU + a * CS * N + k * N;
        #pragma unroll 4
        for (int i = 0; i < N; ++i) s += uu[i] * fmax(sg * sxi[i], 0.0);
      }
      sw[k] = s;
    }
    __syncthreads();
    const double* w[3] = {S(0, 0), S(1, 0), S(2, 0)};
    w[a] = sw;
    const double num = contract(sG, w[0], w[1], w[2]) / P.dxi / P.dxi;
    const double* fw = d.bc_fac + (size_t)d.slot_nb[kSlots * c + l] * 3 * N;
    double den = 1.0;
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
      for (int i = tid; i < N; i += kMomThreads)
        s += fw[b * N + i] * (b == a ? fmin(sg * sxi[i], 0.0) : 1.0);
      den *= wave_sum(s);
    }
    if (tid == 0) d.nw[kSlots * c + l] = -num / den;
  }
}

__global__ __launch_bounds__(64) void k_init_maxwell(DevState d, const double* macro5) {
  const int c = blockIdx.x;
  const int N = d.N, CS = d.CS;
  const InstParams P = d.ip[d.inst[c]];
  const double n = macro5[5 * (size_t)c], T = macro5[5 * (size_t)c + 4];
  const double amp = cbrt(n) / sqrt(2.0 * M_PI * P.Rg * T);
  const double inv = 1.0 / (2.0 * P.Rg * T);
  double* core = const_cast<double*>(d.core) + (size_t)c * CS * CS * CS;
  double* fac = const_cast<double*>(d.fac) + (size_t)c * 3 * CS * N;
  for (int o = threadIdx.x; o < CS * CS * CS; o += 64) core[o] = (o == 0) ? 1.0 : 0.0;
  for (int o = threadIdx.x; o < 3 * CS * N; o += 64) {
    const int a = o / (CS * N), rem = o % (CS * N), k = rem / N, i = rem % N;
    double v = 0.0;
    if (k == 0) {
      const double x = P.xi_min + i * P.dxi - macro5[5 * (size_t)c + 1 + a];
      v = amp * exp(-x * x * inv);
    }
    fac[o] = v;
  }
  if (threadIdx.x < 3) const_cast<int*>(d.rank)[3 * c + threadIdx.x] = 1;
}

}  // namespace

hipError_t launch_init_maxwell(const DevState& d, const double* macro5, hipStream_t s) {
  if (d.n_cells == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_maxwell, dim3(d.n_cells), dim3(64), 0, s, d, macro5);
  return hipGetLastError();
}

hipError_t launch_moments(const DevState& d, hipStream_t s) {
  if (d.n_cells == 0) return hipSuccess;
  const size_t sh = sizeof(double) * (3 * d.CS * d.N + 3 * 8 * d.CS + d.N);
  switch (d.N) {
    case 16: hipLaunchKernelGGL(k_moments<16>, dim3(d.n_cells), dim3(kMomThreads), sh, s, d); break;
    case 24: hipLaunchKernelGGL(k_moments<24>, dim3(d.n_cells), dim3(kMomThreads), sh, s, d); break;
    case 32: hipLaunchKernelGGL(k_moments<32>, dim3(d.n_cells), dim3(kMomThreads), sh, s, d); break;
    case 48: hipLaunchKernelGGL(k_moments<48>, dim3(d.n_cells), dim3(kMomThreads), sh, s, d); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tk
