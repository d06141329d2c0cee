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

// four consecutive values (16-byte aligned for float, two 16-byte loads for double)
__device__ inline void ld4(const float* p, double (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ inline void ld4(const double* p, double (&o)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}

template <int N, typename T>
__global__ __launch_bounds__(192) void k_gram(const T* X, double* G, int c0, const int* cells_n) {
  constexpr int NB = (N + 15) / 16;  // 16-row blocks
  constexpr int NP = NB * (NB + 1) / 2;
  // one workgroup per cell, one wavefront per mode: the three waves read the
  // same tensor at the same time, on the same CU
  const int cell = blockIdx.x;
  if (cells_n && c0 + cell >= *cells_n) return;
  const int mode = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
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
  if (mode == 0) {
    // rows (i1) contiguous: the 16 lanes of a k-group read 16 consecutive values
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
  } else {
    // columns contiguous: each lane loads 4 consecutive columns of its row at
    // once and feeds them to 4 successive MFMA steps (the Gram sums over all
    // columns, so their order across steps is free)
    for (int c0 = 0; c0 < N * N; c0 += 16) {
      const int col = c0 + 4 * kk;
      double v[NB][4];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int r = 16 * b + ii;
        double t4[4];
        ld4(x + addr(r < N ? r : 0, col), t4);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[b][q] = (r < N) ? t4[q] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int p = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
          for (int bj = bi; bj < NB; ++bj) {
            acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[bi][q], v[bj][q], acc[p], 0, 0, 0);
            ++p;
          }
      }
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

// All three Grams of one cell per workgroup, with the cell's tensor staged
// once in LDS.  Padded strides (i2 stride N+1, i3 stride N(N+1)+1) keep the
// 16 rows of an MFMA fragment on distinct banks for every unfolding.  Each
// of the 8 wavefronts accumulates every 16x16 block over 1/8 of the
// unfolding's columns; the partial blocks are summed in a fixed order.
constexpr int kGramLdsThreads = 512;

template <int N, typename T>
__global__ __launch_bounds__(kGramLdsThreads) void k_gram_lds(const T* X, double* G) {
  constexpr int NB = (N + 15) / 16;
  constexpr int NP = NB * (NB + 1) / 2;
  constexpr int S2 = N + 1;
  constexpr int S3 = N * S2 + 1;
  constexpr int NW = kGramLdsThreads / 64;
  constexpr int KS = N * N / 4;  // 4-column steps per unfolding
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sx = reinterpret_cast<T*>(smem_raw);
  const int cell = blockIdx.x;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int ii = lane & 15, kk = lane >> 4;
  const T* x = X + (size_t)cell * N * N * N;
  for (int o = tid; o < N * N * N; o += kGramLdsThreads) {
    const int i1 = o % N, i2 = (o / N) % N, i3 = o / (N * N);
    sx[i1 + S2 * i2 + S3 * i3] = x[o];
  }
  __syncthreads();
  v4d acc[3][NP];
#pragma unroll
  for (int md = 0; md < 3; ++md)
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[md][p] = v4d{0.0, 0.0, 0.0, 0.0};
  const int k0 = (KS * wave) / NW, k1 = (KS * (wave + 1)) / NW;
  for (int ks = k0; ks < k1; ++ks) {
    const int col = 4 * ks + kk;
    const int ca = col % N, cb = col / N;
#pragma unroll
    for (int md = 0; md < 3; ++md) {
      double v[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int r = 16 * b + ii;
        const int rr = (r < N) ? r : 0;  // padding rows read a valid element, then zero it
        int a;
        if (md == 0) a = rr + S2 * ca + S3 * cb;       // row i1, column (i2, i3)
        else if (md == 1) a = ca + S2 * rr + S3 * cb;  // row i2, column (i1, i3)
        else a = ca + S2 * cb + S3 * rr;               // row i3, column (i1, i2)
        const double val = (double)sx[a];
        v[b] = (r < N) ? val : 0.0;
      }
      int p = 0;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NB; ++bj) {
          acc[md][p] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[bi], v[bj], acc[md][p], 0, 0, 0);
          ++p;
        }
    }
  }
  __syncthreads();  // the tensor is no longer needed: reuse LDS for partials
  double* part = reinterpret_cast<double*>(smem_raw);  // [NW][3][NP][4][64]
#pragma unroll
  for (int md = 0; md < 3; ++md)
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) part[(((size_t)wave * 3 + md) * NP + p) * 256 + r * 64 + lane] = acc[md][p][r];
  __syncthreads();
  double* g = G + (size_t)cell * 3 * N * N;
  for (int o = tid; o < 3 * NP * 256; o += kGramLdsThreads) {
    const int l = o & 63, r = (o >> 6) & 3, p = (o >> 8) % NP, md = (o >> 8) / NP;
    double sum = 0.0;
    for (int w = 0; w < NW; ++w) sum += part[(((size_t)w * 3 + md) * NP + p) * 256 + r * 64 + l];
    // pair index p -> (bi, bj)
    int bi = 0, rem = p;
    while (rem >= NB - bi) { rem -= NB - bi; ++bi; }
    const int bj = bi + rem;
    const int i = 16 * bi + (l >> 4) + 4 * r;
    const int j = 16 * bj + (l & 15);
    if (i < N && j < N && (bi != bj || i <= j)) {
      g[(size_t)md * N * N + i * N + j] = sum;
      g[(size_t)md * N * N + j * N + i] = sum;
    }
  }
}

template <int N, typename T>
constexpr size_t gram_lds_bytes() {
  constexpr int NB = (N + 15) / 16;
  constexpr int NP = NB * (NB + 1) / 2;
  constexpr size_t a = sizeof(T) * (size_t)N * (N * (N + 1) + 1);
  constexpr size_t b = sizeof(double) * (size_t)(kGramLdsThreads / 64) * 3 * NP * 256;
  return a > b ? a : b;
}

// G2 = (W^T A_(a)) (W^T A_(a))^T for one (cell, mode) per workgroup, FP64
// vector arithmetic over chunks of CH unfolding columns.  W holds the
// first-pass basis as rows: W[k][i] is entry i of basis vector k.
template <int N, typename T>
__global__ __launch_bounds__(256) void k_gram_rot(const T* X, const double* Wb, double* G2, int c0,
                                                   const int* cells_n) {
  constexpr int CH = N >= 48 ? 32 : 64;  // keeps the static LDS within 64 KB at N = 48
  constexpr int PER = (N * N + 255) / 256;
  __shared__ double W[N * N];
  __shared__ double Ac[N * (CH + 1)];
  __shared__ double Bc[N * (CH + 1)];
  const int m = blockIdx.x;
  const int cell = m / 3, mode = m % 3;
  if (cells_n && c0 + cell >= *cells_n) return;
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
                           hipStream_t s, int c0, const int* cells_n) {
  if (count <= 0) return hipSuccess;
  dim3 grid(3 * count), blk(256);
  if (mixed) {
    const float* x = (const float*)X;
    switch (N) {
      case 16: hipLaunchKernelGGL((k_gram_rot<16, float>), grid, blk, 0, s, x, W, G2, c0, cells_n); break;
      case 24: hipLaunchKernelGGL((k_gram_rot<24, float>), grid, blk, 0, s, x, W, G2, c0, cells_n); break;
      case 32: hipLaunchKernelGGL((k_gram_rot<32, float>), grid, blk, 0, s, x, W, G2, c0, cells_n); break;
      case 48: hipLaunchKernelGGL((k_gram_rot<48, float>), grid, blk, 0, s, x, W, G2, c0, cells_n); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const double* x = (const double*)X;
    switch (N) {
      case 16: hipLaunchKernelGGL((k_gram_rot<16, double>), grid, blk, 0, s, x, W, G2, c0, cells_n); break;
      case 24: hipLaunchKernelGGL((k_gram_rot<24, double>), grid, blk, 0, s, x, W, G2, c0, cells_n); break;
      case 32: hipLaunchKernelGGL((k_gram_rot<32, double>), grid, blk, 0, s, x, W, G2, c0, cells_n); break;
      case 48: hipLaunchKernelGGL((k_gram_rot<48, double>), grid, blk, 0, s, x, W, G2, c0, cells_n); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <int N, typename T>
hipError_t launch_gram_lds_t(int count, const void* X, double* G, hipStream_t s) {
  constexpr size_t sh = gram_lds_bytes<N, T>();
  static_assert(sh <= 160 * 1024, "tensor must fit the LDS");
  auto k = k_gram_lds<N, T>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(count), dim3(kGramLdsThreads), sh, s, (const T*)X, G);
  return hipGetLastError();
}

hipError_t launch_gram(int N, int count, const void* X, int mixed, double* G, hipStream_t s, int c0,
                       const int* cells_n) {
  if (count <= 0) return hipSuccess;
  dim3 grid(count), blk(192);
  if (mixed) {
    const float* x = (const float*)X;
    switch (N) {
      case 16: hipLaunchKernelGGL((k_gram<16, float>), grid, blk, 0, s, x, G, c0, cells_n); break;
      case 24: hipLaunchKernelGGL((k_gram<24, float>), grid, blk, 0, s, x, G, c0, cells_n); break;
      case 32: hipLaunchKernelGGL((k_gram<32, float>), grid, blk, 0, s, x, G, c0, cells_n); break;
      case 48: hipLaunchKernelGGL((k_gram<48, float>), grid, blk, 0, s, x, G, c0, cells_n); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const double* x = (const double*)X;
    switch (N) {
      case 16: hipLaunchKernelGGL((k_gram<16, double>), grid, blk, 0, s, x, G, c0, cells_n); break;
      case 24: hipLaunchKernelGGL((k_gram<24, double>), grid, blk, 0, s, x, G, c0, cells_n); break;
      case 32: hipLaunchKernelGGL((k_gram<32, double>), grid, blk, 0, s, x, G, c0, cells_n); break;
      case 48: hipLaunchKernelGGL((k_gram<48, double>), grid, blk, 0, s, x, G, c0, cells_n); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace tk
