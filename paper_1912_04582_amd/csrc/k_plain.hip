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

// Four consecutive grid nodes along mode 1 (one 16- or 32-byte access).
// N/2 is a multiple of 4 for every supported N, so a group never straddles
// xi_1 = 0 and the mode-1 upwind choice is the same for its four nodes.
template <typename T>
struct Quad {
  T v[4];
};
template <typename T>
__device__ inline Quad<T> load_quad(const T* p) {
  Quad<T> q;
  if constexpr (sizeof(T) == 4) {
    const float4 x = *(const float4*)p;
    q.v[0] = x.x; q.v[1] = x.y; q.v[2] = x.z; q.v[3] = x.w;
  } else {
    const double2 x = *(const double2*)p, y = *(const double2*)(p + 2);
    q.v[0] = x.x; q.v[1] = x.y; q.v[2] = y.x; q.v[3] = y.y;
  }
  return q;
}
template <typename T>
__device__ inline void store_quad(T* p, const Quad<T>& q) {
  if constexpr (sizeof(T) == 4) {
    *(float4*)p = make_float4(q.v[0], q.v[1], q.v[2], q.v[3]);
  } else {
    *(double2*)p = make_double2(q.v[0], q.v[1]);
    *(double2*)(p + 2) = make_double2(q.v[2], q.v[3]);
  }
}

// Moments of full tensors in one pass over the cell: raw sums of
// xi^p f up to total order 3 (19 FP64 accumulators: order 0, 1, 2, the
// three int xi_a |xi|^2 f, and the six half sums of max(+-xi_a, 0) f used
// by the wall ghosts).  The central quantities follow algebraically:
//   n T 3R_g = S_aa - n|u|^2,
//   2 q_a / m = S3_a - 2 sum_b u_b S_ab - u_a S_bb + 2 u_a |u|^2 S_0.
// Each thread reduces its four mode-1 nodes to 1-D partial sums first.
template <int N, typename T>
__global__ __launch_bounds__(kPM) void k_plain_moments(DevPlain d) {
  constexpr int Q = N / 4, NG = N * N * N / 4, NA = 19;
  __shared__ double red[kPM / 64][NA];
  const int c = blockIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const T* f = (const T*)d.f + (size_t)c * N * N * N;
  double A[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) A[i] = 0.0;
  for (int g = threadIdx.x; g < NG; g += kPM) {
    const int i0 = 4 * (g % Q), j = (g / Q) % N, k = g / (Q * N);
    const Quad<T> q = load_quad(f + 4 * (size_t)g);
    double p0 = 0, p1 = 0, p2 = 0, p3 = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double x = P.xi_min + (i0 + t) * P.dxi, v = (double)q.v[t];
      const double xv = x * v, xxv = x * xv;
      p0 += v; p1 += xv; p2 += xxv; p3 += x * xxv;
    }
    const double y = P.xi_min + j * P.dxi, z = P.xi_min + k * P.dxi;
    const double r2 = y * y + z * z;
    A[0] += p0;
    A[1] += p1; A[2] += y * p0; A[3] += z * p0;
    A[4] += p2; A[5] += y * y * p0; A[6] += z * z * p0;
    A[7] += y * p1; A[8] += z * p1; A[9] += y * z * p0;
    A[10] += p3 + r2 * p1; A[11] += y * (p2 + r2 * p0); A[12] += z * (p2 + r2 * p0);
    const double x0 = P.xi_min + i0 * P.dxi;
    if (x0 > 0.0) A[13] += p1; else A[16] -= p1;
    if (y > 0.0) A[14] += y * p0; else A[17] -= y * p0;
    if (z > 0.0) A[15] += z * p0; else A[18] -= z * p0;
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    double v = A[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (l == 0) red[w][i] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double S[NA];
  for (int i = 0; i < NA; ++i) {
    S[i] = 0.0;
    for (int ww = 0; ww < kPM / 64; ++ww) S[i] += red[ww][i];
  }
  const double w3 = P.dxi * P.dxi * P.dxi;
  const double n = S[0] * w3;
  const double u[3] = {S[1] / S[0], S[2] / S[0], S[3] / S[0]};
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double Str = S[4] + S[5] + S[6];
  const double T0 = (Str - S[0] * uu) * w3 / (3.0 * n * P.Rg);
  // symmetric second-moment matrix S_ab
  const double M2[3][3] = {{S[4], S[7], S[8]}, {S[7], S[5], S[9]}, {S[8], S[9], S[6]}};
  double q[3];
  for (int a = 0; a < 3; ++a) {
    const double ub = u[0] * M2[a][0] + u[1] * M2[a][1] + u[2] * M2[a][2];
    q[a] = 0.5 * P.m * (S[10 + a] - 2.0 * ub - u[a] * Str + 2.0 * u[a] * uu * S[0]) * w3;
  }
  const double p = P.m * n * P.Rg * T0;
  const double nu = p / (0.5 * P.Kn * pow(T0, P.omega));
  double* M = d.macro + 8 * (size_t)c;
  M[0] = n; M[1] = u[0]; M[2] = u[1]; M[3] = u[2]; M[4] = T0;
  M[5] = q[0]; M[6] = q[1]; M[7] = q[2];
  d.nu[c] = nu;
  if (!(n > 0.0) || !(T0 > 0.0) || !isfinite(n) || !isfinite(T0)) atomicOr(&d.flag[d.inst[c]], 1);
  for (int s = 0; s < kSlots; ++s) {
    if (d.slot_kind[kSlots * c + s] != SK_WALL) continue;
    const int a = d.slot_axis[kSlots * c + s];
    const int sg = d.slot_sig[kSlots * c + s];
    const double num = (sg > 0) ? S[13 + a] : S[16 + a];
    const double* fw = d.bc_fac + (size_t)d.slot_nb[kSlots * c + s] * 3 * N;
    double den = 1.0;
    for (int b = 0; b < 3; ++b) {
      double sum = 0.0;
      for (int i = 0; i < N; ++i) sum += fw[b * N + i] * (b == a ? fmin(sg * (P.xi_min + i * P.dxi), 0.0) : 1.0);
      den *= sum;
    }
    d.nw[kSlots * c + s] = -num / den;
  }
}

// Groups of four mode-1 nodes handled by one thread in the step kernel, and
// the number of such groups per thread in one workgroup.
constexpr int kPlainGroups = 8;

template <int N>
constexpr int plain_blocks_per_cell() {
  return (N * N * N / 4 + kPM * kPlainGroups - 1) / (kPM * kPlainGroups);
}

// One workgroup updates a contiguous range of one cell's grid nodes, four
// mode-1 nodes per thread access.  Per-cell 1-D tables are built once per
// workgroup: the Maxwellian factors of f_S (f_M = m_1(i1) m_2(i2) m_3(i3)),
// the separable outflow weight d_a(i) = -sum_{faces on axis a} (dt A/V)
// max(s xi_i, 0), each face's inflow scaling b_l(i) = (dt A/V)
// max(-s xi_i, 0), and the rank-1 factors of inflow and wall ghosts; per
// node only polynomial arithmetic remains, in the storage precision.
// Workgroups are numbered so that each XCD (eight of them, dispatched
// round-robin) walks a contiguous range of cells and finds the mode-1
// neighbours of its cells in its own L2.
template <int N, typename T>
__global__ __launch_bounds__(kPM) void k_plain_step(DevPlain d, int total) {
  constexpr int NE = N * N * N, Q = N / 4, NG = NE / 4;
  constexpr int BPC = plain_blocks_per_cell<N>();
  __shared__ T s_m[3][N];       // Maxwellian 1-D factors
  __shared__ T s_v[3][N];       // xi_i - u_a
  __shared__ T s_d[3][N];       // separable own-cell weights
  __shared__ T s_b[kSlots][N];  // inflow scalings of the six faces
  __shared__ T s_g[kSlots][3][N];  // rank-1 inflow / wall ghost factors
  __shared__ T s_c[8];
  __shared__ T s_x[N];             // xi_i
  __shared__ T s_n[kSlots][3];     // outward normals of faces off the axes
  __shared__ T s_a[kSlots];        // their dt A / V
  __shared__ int s_nb[kSlots];
  __shared__ int8_t s_kind[kSlots], s_axis[kSlots];
  const int pb = blockIdx.x;
  const int full = total & ~7;
  const int lb = pb < full ? (pb & 7) * (full >> 3) + (pb >> 3) : pb;
  const int c = lb / BPC, part = lb % BPC;
  const int tid = threadIdx.x;
  const InstParams P = d.ip[d.inst[c]];
  const double* M = d.macro + 8 * (size_t)c;
  if (tid < kSlots) {
    s_kind[tid] = d.slot_kind[kSlots * c + tid];
    s_axis[tid] = d.slot_axis[kSlots * c + tid];
    s_nb[tid] = d.slot_nb[kSlots * c + tid];
    s_a[tid] = (T)d.slot_coef[kSlots * c + tid];
    for (int a = 0; a < 3; ++a)
      s_n[tid][a] = (d.slot_nrm && s_axis[tid] < 0) ? (T)d.slot_nrm[3 * (kSlots * c + tid) + a] : (T)0;
  }
  for (int i = tid; i < N; i += kPM) s_x[i] = (T)(P.xi_min + i * P.dxi);
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
      const double x = P.xi_min + i * P.dxi;
      b = d.slot_coef[kSlots * c + l] * fmax(-(double)d.slot_sig[kSlots * c + l] * x, 0.0);
      if (kind == SK_WALL) b *= d.nw[kSlots * c + l];
      if (kind == SK_INFLOW || kind == SK_WALL) {
        const double* bf = d.bc_fac + (size_t)d.slot_nb[kSlots * c + l] * 3 * N;
        for (int a = 0; a < 3; ++a) s_g[l][a][i] = (T)bf[a * N + i];
      }
    }
    s_b[l][i] = (T)b;
  }
  if (tid == 0) {
    s_c[0] = (T)(1.0 - P.dt * nu);                                    // 1 - dt nu
    s_c[1] = (T)(P.dt * nu);                                          // dt nu
    s_c[2] = (T)(2.0 * (1.0 - P.Pr) / (5.0 * P.m * M[0] * RT * RT));  // A_s
    s_c[3] = (T)(1.0 / (2.0 * RT));                                   // beta
    for (int a = 0; a < 3; ++a) s_c[4 + a] = (T)M[5 + a];              // q
  }
  __syncthreads();
  const T* f = (const T*)d.f;
  T* fo = (T*)d.f_n;
  const T c1 = s_c[0], dtnu = s_c[1], As = s_c[2], beta = s_c[3];
  const T q0 = s_c[4], q1 = s_c[5], q2 = s_c[6];
  const int g_end = min(NG, (part + 1) * kPM * kPlainGroups);
  for (int g = part * kPM * kPlainGroups + tid; g < g_end; g += kPM) {
    const int i0 = 4 * (g % Q), j = (g / Q) % N, k = g / (Q * N);
    const size_t base = (size_t)c * NE + 4 * (size_t)g;
    const Quad<T> own = load_quad(f + base);
    const T v2 = s_v[1][j], v3 = s_v[2][k];
    const T m23 = s_m[1][j] * s_m[2][k];
    const T vv23 = v2 * v2 + v3 * v3, qv23 = q1 * v2 + q2 * v3;
    const T w23 = c1 + s_d[1][j] + s_d[2][k];
    Quad<T> acc;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T v1 = s_v[0][i0 + t];
      const T fs = s_m[0][i0 + t] * m23 * ((T)1 + As * (q0 * v1 + qv23) * (beta * (v1 * v1 + vv23) - (T)2.5));
      acc.v[t] = (w23 + s_d[0][i0 + t]) * own.v[t] + dtnu * fs;
    }
#pragma unroll
    for (int l = 0; l < kSlots; ++l) {
      const int8_t kind = s_kind[l];
      if (kind == SK_NONE) continue;
      const int a = s_axis[l];
      if (a < 0) {
        // a face off the coordinate axes (interior, outflow or free-stream
        // inflow): the exact upwind split of xi_n = xi . n per node
        const T n0 = s_n[l][0], coef = s_a[l];
        const T x23 = s_n[l][1] * s_x[j] + s_n[l][2] * s_x[k];
        Quad<T> g4;
        if (kind == SK_INTERIOR) {
          g4 = load_quad(f + (size_t)s_nb[l] * NE + 4 * (size_t)g);
        } else if (kind == SK_OUTFLOW) {
          g4 = own;
        } else {
          const T g23 = s_g[l][1][j] * s_g[l][2][k];
#pragma unroll
          for (int t = 0; t < 4; ++t) g4.v[t] = s_g[l][0][i0 + t] * g23;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const T x = n0 * s_x[i0 + t] + x23;
          acc.v[t] += x > (T)0 ? -coef * x * own.v[t] : -coef * x * g4.v[t];
        }
        continue;
      }
      T b[4];
      if (a == 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t) b[t] = s_b[l][i0 + t];
      } else {
        const T bb = s_b[l][a == 1 ? j : k];
#pragma unroll
        for (int t = 0; t < 4; ++t) b[t] = bb;
      }
      if (b[0] == (T)0 && b[1] == (T)0 && b[2] == (T)0 && b[3] == (T)0) continue;
      Quad<T> g4;
      if (kind == SK_INTERIOR) {
        g4 = load_quad(f + (size_t)s_nb[l] * NE + 4 * (size_t)g);
      } else if (kind == SK_OUTFLOW) {
        g4 = own;
      } else if (kind == SK_SYM) {
        if (a == 0) {
          const Quad<T> r = load_quad(f + (size_t)c * NE + (N - 4 - i0) + N * (j + N * k));
#pragma unroll
          for (int t = 0; t < 4; ++t) g4.v[t] = r.v[3 - t];
        } else if (a == 1) {
          g4 = load_quad(f + (size_t)c * NE + i0 + N * ((N - 1 - j) + N * k));
        } else {
          g4 = load_quad(f + (size_t)c * NE + i0 + N * (j + N * (N - 1 - k)));
        }
      } else {
        const T g23 = s_g[l][1][j] * s_g[l][2][k];
#pragma unroll
        for (int t = 0; t < 4; ++t) g4.v[t] = s_g[l][0][i0 + t] * g23;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) acc.v[t] += b[t] * g4.v[t];
    }
    store_quad(fo + base, acc);
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
  int bpc = 0;
  switch (d.N) {
    case 16: bpc = plain_blocks_per_cell<16>(); break;
    case 24: bpc = plain_blocks_per_cell<24>(); break;
    case 32: bpc = plain_blocks_per_cell<32>(); break;
    case 48: bpc = plain_blocks_per_cell<48>(); break;
    default: return hipErrorInvalidValue;
  }
  const long long total = (long long)d.n_cells * bpc;
  if (total > 0x7fffffffLL) return hipErrorInvalidValue;
  TK_PLAIN_DISPATCH(k_plain_step, dim3((unsigned)total), dim3(kPM), d, (int)total);
  return hipGetLastError();
}

hipError_t launch_residual(const double* macro_old, const double* macro_new, const double* vol,
                           const int* inst_off, int n_inst, double* out, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual, dim3(n_inst), dim3(256), 0, s, macro_old, macro_new, vol, inst_off, out);
  return hipGetLastError();
}

}  // namespace tk
