// Mode Gram matrices G_a = A_(a) A_(a)^T of the full update tensor, the
// first stage of the truncated HOSVD (Op4: the left singular subspace of
// each unfolding, eq. svd).  FP64 on the matrix cores: one wavefront per
// (cell, mode) accumulates 16x16 blocks with v_mfma_f64_16x16x4f64 over
// the N^2 columns of the unfolding; only blocks on or above the diagonal
// are computed and mirrored.
#include "tk_internal.h"

namespace tk {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline double ld(const T* p) { return (double)*p; }

template <int N, typename T>
__global__ __launch_bounds__(64) void k_gram(const T* X, double* G) {
  constexpr int NB = (N + 15) / 16;  // 16-row blocks
  constexpr int NP = NB * (NB + 1) / 2;
  const int cell = blockIdx.x / 3;
  const int mode = blockIdx.x % 3;
  const int lane = threadIdx.x;
  const int ii = lane & 15;  // row within block (A) / column within block (B)
  const int kk = lane >> 4;  // k within the 4-wide step
  const T* x = X + (size_t)cell * N * N * N;
  v4d acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = v4d{0.0, 0.0, 0.0, 0.0};
  // row r of the unfolding, column col -> linear index of the tensor
  auto addr = [&](int r, int col) -> int {
    if (mode == 0) return r + N * col;
    if (mode == 1) return (col % N) + N * r + N * N * (col / N);
    return col + N * N * r;
  };
  for (int c0 = 0; c0 < N * N; c0 += 4) {
    const int col = c0 + kk;
    double v[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int r = 16 * b + ii;
      v[b] = (r < N) ? ld(x + addr(r, col)) : 0.0;
    }
    int p = 0;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
      for (int bj = bi; bj < NB; ++bj) {
        acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[bi], v[bj], acc[p], 0, 0, 0);
        ++p;
      }
  }
  double* g = G + ((size_t)cell * 3 + mode) * N * N;
  int p = 0;
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = bi; bj < NB; ++bj) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // D layout of v_mfma_f64_16x16x4f64: lane holds rows lane/16 + 4 r
        // of column lane%16
        const int i = 16 * bi + kk + 4 * r;
        const int j = 16 * bj + ii;
        if (i < N && j < N && (bi != bj || i <= j)) {
          g[i * N + j] = acc[p][r];
          g[j * N + i] = acc[p][r];
        }
      }
      ++p;
    }
}

// G2 = (W^T A_(a)) (W^T A_(a))^T for one (cell, mode) per workgroup, FP64
// vector arithmetic over chunks of CH unfolding columns.  W holds the
// first-pass basis as rows: W[k][i] is entry i of basis vector k.
template <int N, typename T>
__global__ __launch_bounds__(256) void k_gram_rot(const T* X, const double* Wb, double* G2) {
  constexpr int CH = 64;
  constexpr int PER = (N * N + 255) / 256;
  __shared__ double W[N * N];
  __shared__ double Ac[N * (CH + 1)];
  __shared__ double Bc[N * (CH + 1)];
  const int m = blockIdx.x;
  const int cell = m / 3, mode = m % 3;
  const int tid = threadIdx.x;
  const T* x = X + (size_t)cell * N * N * N;
  for (int o = tid; o < N * N; o += 256) W[o] = Wb[(size_t)m * N * N + o];
  double acc[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) acc[t] = 0.0;
  auto addr = [&](int r, int col) -> int {
    if (mode == 0) return r + N * col;
    if (mode == 1) return (col % N) + N * r + N * N * (col / N);
    return col + N * N * r;
  };
  for (int c0 = 0; c0 < N * N; c0 += CH) {
    __syncthreads();
    for (int o = tid; o < N * CH; o += 256) {
      const int i = o / CH, c = o % CH;
      Ac[i * (CH + 1) + c] = (double)x[addr(i, c0 + c)];
    }
    __syncthreads();
    for (int o = tid; o < N * CH; o += 256) {
      const int k = o / CH, c = o % CH;
      double v = 0.0;
      for (int i = 0; i < N; ++i) v += W[k * N + i] * Ac[i * (CH + 1) + c];
      Bc[k * (CH + 1) + c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int o = tid + 256 * t;
      if (o < N * N) {
        const int i = o / N, j = o % N;
        double v = 0.0;
        for (int c = 0; c < CH; ++c) v += Bc[i * (CH + 1) + c] * Bc[j * (CH + 1) + c];
        acc[t] += v;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int o = tid + 256 * t;
    if (o < N * N) G2[(size_t)m * N * N + o] = acc[t];
  }
}

}  // namespace

hipError_t launch_gram_rot(int N, int count, const void* X, int mixed, const double* W, double* G2,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  dim3 grid(3 * count), blk(256);
  if (mixed) {
    const float* x = (const float*)X;
    switch (N) {
      case 16: hipLaunchKernelGGL((k_gram_rot<16, float>), grid, blk, 0, s, x, W, G2); break;
      case 24: hipLaunchKernelGGL((k_gram_rot<24, float>), grid, blk, 0, s, x, W, G2); break;
      case 32: hipLaunchKernelGGL((k_gram_rot<32, float>), grid, blk, 0, s, x, W, G2); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const double* x = (const double*)X;
    switch (N) {
      case 16: hipLaunchKernelGGL((k_gram_rot<16, double>), grid, blk, 0, s, x, W, G2); break;
      case 24: hipLaunchKernelGGL((k_gram_rot<24, double>), grid, blk, 0, s, x, W, G2); break;
      case 32: hipLaunchKernelGGL((k_gram_rot<32, double>), grid, blk, 0, s, x, W, G2); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_gram(int N, int count, const void* X, int mixed, double* G, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  dim3 grid(3 * count), blk(64);
  if (mixed) {
    const float* x = (const float*)X;
    switch (N) {
      case 16: hipLaunchKernelGGL((k_gram<16, float>), grid, blk, 0, s, x, G); break;
      case 24: hipLaunchKernelGGL((k_gram<24, float>), grid, blk, 0, s, x, G); break;
      case 32: hipLaunchKernelGGL((k_gram<32, float>), grid, blk, 0, s, x, G); break;
      case 48: hipLaunchKernelGGL((k_gram<48, float>), grid, blk, 0, s, x, G); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const double* x = (const double*)X;
    switch (N) {
      case 16: hipLaunchKernelGGL((k_gram<16, double>), grid, blk, 0, s, x, G); break;
      case 24: hipLaunchKernelGGL((k_gram<24, double>), grid, blk, 0, s, x, G); break;
      case 32: hipLaunchKernelGGL((k_gram<32, double>), grid, blk, 0, s, x, G); break;
      case 48: hipLaunchKernelGGL((k_gram<48, double>), grid, blk, 0, s, x, G); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace tk
