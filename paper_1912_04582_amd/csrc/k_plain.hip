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

// One workgroup updates a chunk of one cell's grid nodes.  Per-cell 1-D
// tables are built once per workgroup: the Maxwellian factors of f_S
// (f_M = m_1(i1) m_2(i2) m_3(i3)), the separable outflow weight
// d_a(i) = -sum_{faces on axis a} (dt A/V) max(s xi_i, 0) and each face's
// inflow scaling b_l(i) = (dt A/V) max(-s xi_i, 0); per node only
// polynomial arithmetic remains (in the storage precision).
template <int N, typename T>
__global__ __launch_bounds__(kPM) void k_plain_step(DevPlain d) {
  constexpr int NE = N * N * N;
  constexpr int EPT = 4;
  __shared__ T s_m[3][N];       // Maxwellian 1-D factors
  __shared__ T s_v[3][N];       // xi_i - u_a
  __shared__ T s_d[3][N];       // separable own-cell weights
  __shared__ T s_b[kSlots][N];  // inflow scalings of the six faces
  __shared__ T s_c[8];
  __shared__ int s_nb[kSlots];
  __shared__ int8_t s_kind[kSlots], s_axis[kSlots];
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const double* M = d.macro + 8 * (size_t)c;
  if (tid < kSlots) {
    s_kind[tid] = d.slot_kind[kSlots * c + tid];
    s_axis[tid] = d.slot_axis[kSlots * c + tid];
    s_nb[tid] = d.slot_nb[kSlots * c + tid];
  }
  const double RT = P.Rg * M[4];
  const double nu = d.nu[c];
  for (int o = tid; o < 3 * N; o += kPM) {
    const int a = o / N, i = o % N;
    const double x = P.xi_min + i * P.dxi;
    const double v = x - M[1 + a];
    s_m[a][i] = (T)(cbrt(M[0]) / sqrt(2.0 * M_PI * RT) * exp(-v * v / (2.0 * RT)));
    s_v[a][i] = (T)v;
    double w = 0.0;
    for (int l = 0; l < kSlots; ++l) {
      if (d.slot_kind[kSlots * c + l] == SK_NONE || d.slot_axis[kSlots * c + l] != a) continue;
      w -= d.slot_coef[kSlots * c + l] * fmax((double)d.slot_sig[kSlots * c + l] * x, 0.0);
    }
    s_d[a][i] = (T)w;
  }
  for (int o = tid; o < kSlots * N; o += kPM) {
    const int l = o / N, i = o % N;
    const int8_t kind = d.slot_kind[kSlots * c + l];
    double b = 0.0;
    if (kind != SK_NONE) {
      const int a = d.slot_axis[kSlots * c + l];
      const double x = P.xi_min + i * P.dxi;
      b = d.slot_coef[kSlots * c + l] * fmax(-(double)d.slot_sig[kSlots * c + l] * x, 0.0);
      if (kind == SK_WALL) b *= d.nw[kSlots * c + l];
      (void)a;
    }
    s_b[l][i] = (T)b;
  }
  if (tid == 0) {
    s_c[0] = (T)(1.0 - P.dt * nu);                                  // 1 - dt nu
    s_c[1] = (T)(P.dt * nu);                                        // dt nu
    s_c[2] = (T)(2.0 * (1.0 - P.Pr) / (5.0 * P.m * M[0] * RT * RT));  // A_s
    s_c[3] = (T)(1.0 / (2.0 * RT));                                 // beta
    for (int a = 0; a < 3; ++a) s_c[4 + a] = (T)M[5 + a];            // q
  }
  __syncthreads();
  const int e0 = (blockIdx.y * kPM + tid) * EPT;
  if (e0 >= NE) return;
  const T* f = (const T*)d.f;
  T* fo = (T*)d.f_n;
  const T c1 = s_c[0], dtnu = s_c[1], As = s_c[2], beta = s_c[3];
  const T q0 = s_c[4], q1 = s_c[5], q2 = s_c[6];
#pragma unroll
  for (int qn = 0; qn < EPT; ++qn) {
    const int e = e0 + qn;
    const int i1 = e % N, i2 = (e / N) % N, i3 = e / (N * N);
    const int idx[3] = {i1, i2, i3};
    const T own = f[(size_t)c * NE + e];
    const T v1 = s_v[0][i1], v2 = s_v[1][i2], v3 = s_v[2][i3];
    const T vv = v1 * v1 + v2 * v2 + v3 * v3;
    const T fs = s_m[0][i1] * s_m[1][i2] * s_m[2][i3] *
                 ((T)1 + As * (q0 * v1 + q1 * v2 + q2 * v3) * (beta * vv - (T)2.5));
    T acc = (c1 + s_d[0][i1] + s_d[1][i2] + s_d[2][i3]) * own + dtnu * fs;
#pragma unroll
    for (int l = 0; l < kSlots; ++l) {
      const int8_t kind = s_kind[l];
      if (kind == SK_NONE) continue;
      const int a = s_axis[l];
      const T b = s_b[l][idx[a]];
      if (b == (T)0) continue;
      T g;
      if (kind == SK_INTERIOR) {
        g = f[(size_t)s_nb[l] * NE + e];
      } else if (kind == SK_OUTFLOW) {
        g = own;
      } else if (kind == SK_SYM) {
        int r[3] = {i1, i2, i3};
        r[a] = N - 1 - r[a];
        g = f[(size_t)c * NE + r[0] + N * (r[1] + N * r[2])];
      } else {
        const double* bf = d.bc_fac + (size_t)s_nb[l] * 3 * N;
        g = (T)(bf[i1] * bf[N + i2] * bf[2 * N + i3]);
      }
      acc += b * g;
    }
    fo[(size_t)c * NE + e] = acc;
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
