// The paper's baseline discrete velocity method on full N^3 tensors (Alg. 1
// and Alg. 2 on the grid values, no rounding): the comparator the Tucker
// step is measured against.  Moments are FP64 sums over the tensor; the
// update streams the cell and its six far sides once (HBM-bound).
//
// Also: the per-instance steady-state residual
// max(||n' - n|| / ||n||, ||T' - T|| / ||T||) with cell-volume weighted
// 2-norms, reduced in a fixed order (one workgroup per instance).
#include "tk_internal.h"

namespace tk {

namespace {

constexpr int kPM = 256;

__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// moments of full tensors; also the six directional half fluxes used by
// the wall ghosts (sum max(+-xi_a, 0) f)
template <int N, typename T>
__global__ __launch_bounds__(kPM) void k_plain_moments(DevPlain d) {
  __shared__ double red[kPM / 64];
  const int c = blockIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const T* f = (const T*)d.f + (size_t)c * N * N * N;
  double s0 = 0, s1[3] = {0, 0, 0}, hp[3] = {0, 0, 0}, hm[3] = {0, 0, 0};
  for (int e = threadIdx.x; e < N * N * N; e += kPM) {
    const int i = e % N, j = (e / N) % N, k = e / (N * N);
    const double v = (double)f[e];
    const double x[3] = {P.xi_min + i * P.dxi, P.xi_min + j * P.dxi, P.xi_min + k * P.dxi};
    s0 += v;
    for (int a = 0; a < 3; ++a) {
      s1[a] += x[a] * v;
      hp[a] += fmax(x[a], 0.0) * v;
      hm[a] += fmax(-x[a], 0.0) * v;
    }
  }
  const double w3 = P.dxi * P.dxi * P.dxi;
  const double n = block_sum(s0, red) * w3;
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = block_sum(s1[a], red) * w3 / n;
  double H[6];
  for (int a = 0; a < 3; ++a) { H[a] = block_sum(hp[a], red); H[3 + a] = block_sum(hm[a], red); }
  double c2 = 0, q[3] = {0, 0, 0};
  for (int e = threadIdx.x; e < N * N * N; e += kPM) {
    const int i = e % N, j = (e / N) % N, k = e / (N * N);
    const double v = (double)f[e];
    const double x[3] = {P.xi_min + i * P.dxi - u[0], P.xi_min + j * P.dxi - u[1], P.xi_min + k * P.dxi - u[2]};
    const double v2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    c2 += v2 * v;
    for (int a = 0; a < 3; ++a) q[a] += x[a] * v2 * v;
  }
  const double T0 = block_sum(c2, red) * w3 / (3.0 * n * P.Rg);
  for (int a = 0; a < 3; ++a) q[a] = 0.5 * P.m * block_sum(q[a], red) * w3;
  const double p = P.m * n * P.Rg * T0;
  const double nu = p / (0.5 * P.Kn * pow(T0, P.omega));
  if (threadIdx.x == 0) {
    double* M = d.macro + 8 * (size_t)c;
    M[0] = n; M[1] = u[0]; M[2] = u[1]; M[3] = u[2]; M[4] = T0;
    M[5] = q[0]; M[6] = q[1]; M[7] = q[2];
    d.nu[c] = nu;
    if (!(n > 0.0) || !(T0 > 0.0) || !isfinite(n) || !isfinite(T0)) atomicOr(d.flag, 1);
    for (int l = 0; l < kSlots; ++l) {
      if (d.slot_kind[kSlots * c + l] != SK_WALL) continue;
      const int a = d.slot_axis[kSlots * c + l];
      const int sg = d.slot_sig[kSlots * c + l];
      const double num = (sg > 0) ? H[a] : H[3 + a];
      const double* fw = d.bc_fac + (size_t)d.slot_nb[kSlots * c + l] * 3 * N;
      double den = 1.0;
      for (int b = 0; b < 3; ++b) {
        double s = 0.0;
        for (int i = 0; i < N; ++i) s += fw[b * N + i] * (b == a ? fmin(sg * (P.xi_min + i * P.dxi), 0.0) : 1.0);
        den *= s;
      }
      d.nw[kSlots * c + l] = -num / den;
    }
  }
}

// One thread updates EPT consecutive grid nodes of one cell; the per-cell
// constants (f_S parameters, face coefficients) are computed once per
// workgroup.  Reads the cell and its six far sides once per node.
template <int N, typename T>
__global__ __launch_bounds__(kPM) void k_plain_step(DevPlain d) {
  constexpr int NE = N * N * N;
  constexpr int EPT = 4;
  __shared__ double s_c[16];
  __shared__ double s_coef[kSlots];
  __shared__ int s_nb[kSlots];
  __shared__ int8_t s_kind[kSlots], s_axis[kSlots], s_sig[kSlots];
  const int c = blockIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  if (threadIdx.x == 0) {
    const double* M = d.macro + 8 * (size_t)c;
    const double nu = d.nu[c];
    const double RT = P.Rg * M[4];
    s_c[0] = M[0] / pow(2.0 * M_PI * RT, 1.5);               // f_M amplitude
    s_c[1] = 1.0 / (2.0 * RT);                               // 1 / (2 R_g T)
    s_c[2] = 2.0 * (1.0 - P.Pr) / (5.0 * P.m * M[0] * RT * RT);  // A_s
    s_c[3] = P.dt * nu;
    for (int a = 0; a < 3; ++a) { s_c[4 + a] = M[1 + a]; s_c[7 + a] = M[5 + a]; }
    for (int l = 0; l < kSlots; ++l) {
      s_kind[l] = d.slot_kind[kSlots * c + l];
      s_axis[l] = d.slot_axis[kSlots * c + l];
      s_sig[l] = d.slot_sig[kSlots * c + l];
      s_coef[l] = d.slot_coef[kSlots * c + l];
      s_nb[l] = d.slot_nb[kSlots * c + l];
    }
  }
  __syncthreads();
  const int e0 = (blockIdx.y * kPM + threadIdx.x) * EPT;
  if (e0 >= NE) return;
  const T* f = (const T*)d.f;
  const double amp = s_c[0], ib = s_c[1], As = s_c[2], dtnu = s_c[3];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = e0 + q;
    const int idx[3] = {e % N, (e / N) % N, e / (N * N)};
    const double x[3] = {P.xi_min + idx[0] * P.dxi, P.xi_min + idx[1] * P.dxi, P.xi_min + idx[2] * P.dxi};
    const double own = (double)f[(size_t)c * NE + e];
    const double v[3] = {x[0] - s_c[4], x[1] - s_c[5], x[2] - s_c[6]};
    const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double qv = s_c[7] * v[0] + s_c[8] * v[1] + s_c[9] * v[2];
    const double fs = amp * exp(-v2 * ib) * (1.0 + As * qv * (v2 * ib - 2.5));
    double w = 1.0 - dtnu;
    double acc = dtnu * fs;
    for (int l = 0; l < kSlots; ++l) {
      const int8_t kind = s_kind[l];
      if (kind == SK_NONE) continue;
      const int a = s_axis[l];
      const double sg = (double)s_sig[l];
      const double coef = s_coef[l];
      w -= coef * fmax(sg * x[a], 0.0);
      const double b = coef * fmax(-sg * x[a], 0.0);
      if (b == 0.0) continue;
      const int nb = s_nb[l];
      double g;
      if (kind == SK_INTERIOR) {
        g = (double)f[(size_t)nb * NE + e];
      } else if (kind == SK_OUTFLOW) {
        g = own;
      } else if (kind == SK_SYM) {
        int r[3] = {idx[0], idx[1], idx[2]};
        r[a] = N - 1 - r[a];
        g = (double)f[(size_t)c * NE + r[0] + N * (r[1] + N * r[2])];
      } else {
        const double* bf = d.bc_fac + (size_t)nb * 3 * N;
        g = bf[idx[0]] * bf[N + idx[1]] * bf[2 * N + idx[2]];
        if (kind == SK_WALL) g *= d.nw[kSlots * c + l];
      }
      acc += b * g;
    }
    ((T*)d.f_n)[(size_t)c * NE + e] = (T)(w * own + acc);
  }
}

template <int N, typename T>
__global__ __launch_bounds__(256) void k_plain_init(DevPlain d, const double* macro5) {
  constexpr int NE = N * N * N;
  const int c = blockIdx.x;
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= NE) return;
  const InstParams P = d.ip[d.inst[c]];
  const double* m = macro5 + 5 * (size_t)c;
  const int idx[3] = {e % N, (e / N) % N, e / (N * N)};
  const double RT = P.Rg * m[4];
  double v2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double v = P.xi_min + idx[a] * P.dxi - m[1 + a];
    v2 += v * v;
  }
  // the same rank-1 product as the Tucker initial state
  const double amp = cbrt(m[0]) / sqrt(2.0 * M_PI * RT);
  double val = 1.0;
  for (int a = 0; a < 3; ++a) {
    const double v = P.xi_min + idx[a] * P.dxi - m[1 + a];
    val *= amp * exp(-v * v / (2.0 * RT));
  }
  (void)v2;
  ((T*)d.f)[(size_t)c * NE + e] = (T)val;
}

__global__ __launch_bounds__(256) void k_residual(const double* mo, const double* mn, const double* vol,
                                                  const int* off, double* out) {
  __shared__ double red[4];
  const int inst = blockIdx.x;
  const int a = off[inst], b = off[inst + 1];
  double dn = 0, nn = 0, dT = 0, TT = 0;
  for (int c = a + threadIdx.x; c < b; c += 256) {
    const double V = vol[c];
    const double n0 = mo[8 * (size_t)c], n1 = mn[8 * (size_t)c];
    const double T0 = mo[8 * (size_t)c + 4], T1 = mn[8 * (size_t)c + 4];
    dn += V * (n1 - n0) * (n1 - n0);
    nn += V * n0 * n0;
    dT += V * (T1 - T0) * (T1 - T0);
    TT += V * T0 * T0;
  }
  dn = block_sum(dn, red);
  nn = block_sum(nn, red);
  dT = block_sum(dT, red);
  TT = block_sum(TT, red);
  if (threadIdx.x == 0) out[inst] = fmax(sqrt(dn / nn), sqrt(dT / TT));
}

}  // namespace

#define TK_PLAIN_DISPATCH(KERNEL, GRID, BLK, ...)                                     \
  do {                                                                                \
    if (mixed) {                                                                      \
      switch (d.N) {                                                                  \
        case 16: hipLaunchKernelGGL((KERNEL<16, float>), GRID, BLK, 0, s, __VA_ARGS__); break; \
        case 24: hipLaunchKernelGGL((KERNEL<24, float>), GRID, BLK, 0, s, __VA_ARGS__); break; \
        case 32: hipLaunchKernelGGL((KERNEL<32, float>), GRID, BLK, 0, s, __VA_ARGS__); break; \
        case 48: hipLaunchKernelGGL((KERNEL<48, float>), GRID, BLK, 0, s, __VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                         \
      }                                                                               \
    } else {                                                                          \
      switch (d.N) {                                                                  \
        case 16: hipLaunchKernelGGL((KERNEL<16, double>), GRID, BLK, 0, s, __VA_ARGS__); break; \
        case 24: hipLaunchKernelGGL((KERNEL<24, double>), GRID, BLK, 0, s, __VA_ARGS__); break; \
        case 32: hipLaunchKernelGGL((KERNEL<32, double>), GRID, BLK, 0, s, __VA_ARGS__); break; \
        case 48: hipLaunchKernelGGL((KERNEL<48, double>), GRID, BLK, 0, s, __VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                         \
      }                                                                               \
    }                                                                                 \
  } while (0)

hipError_t launch_plain_init(const DevPlain& d, const double* macro5, int mixed, hipStream_t s) {
  if (d.n_cells == 0) return hipSuccess;
  const int ne = d.N * d.N * d.N;
  dim3 grid(d.n_cells, (ne + 255) / 256);
  TK_PLAIN_DISPATCH(k_plain_init, grid, dim3(256), d, macro5);
  return hipGetLastError();
}

hipError_t launch_plain_moments(const DevPlain& d, int mixed, hipStream_t s) {
  if (d.n_cells == 0) return hipSuccess;
  TK_PLAIN_DISPATCH(k_plain_moments, dim3(d.n_cells), dim3(kPM), d);
  return hipGetLastError();
}

hipError_t launch_plain_step(const DevPlain& d, int mixed, hipStream_t s) {
  if (d.n_cells == 0) return hipSuccess;
  const int ne = d.N * d.N * d.N;
  dim3 grid(d.n_cells, (ne + 4 * kPM - 1) / (4 * kPM));
  TK_PLAIN_DISPATCH(k_plain_step, grid, dim3(kPM), d);
  return hipGetLastError();
}

hipError_t launch_residual(const double* macro_old, const double* macro_new, const double* vol,
                           const int* inst_off, int n_inst, double* out, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual, dim3(n_inst), dim3(256), 0, s, macro_old, macro_new, vol, inst_off, out);
  return hipGetLastError();
}

}  // namespace tk
