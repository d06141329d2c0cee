// Core of the rounded tensor: C = A x1 W1^T x2 W2^T x3 W3^T (the last step of
// the truncated HOSVD, Op1/Op4), with W_a the kept eigenvectors of the mode
// Gram matrices.  One workgroup per cell walks the mode-3 slices of A:
// Q = W1^T A(:,:,i3), T = Q W2, then C(:,:,k3) += T W3(i3,k3).  FP64
// accumulation whatever the storage type of A.
#include "tk_internal.h"

namespace tk {

namespace {

constexpr int kProjThreads = 256;

template <int N, typename T>
__global__ __launch_bounds__(kProjThreads) void k_project(const T* X, int c0, int CS, const double* fac_n,
                                                         const int* rank_n, double* core_n, const int* cells,
                                                         const int* cells_n, int lo) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sS = reinterpret_cast<double*>(smem_raw);  // N*N slice
  double* sW = sS + N * N;                             // 3 * CS * N
  double* sQ = sW + 3 * CS * N;                        // CS * N
  double* sT = sQ + CS * N;                            // CS * CS
  const int cl = blockIdx.x;
  if (cells && c0 + cl >= *cells_n) return;
  const int cell = cells ? cells[c0 + cl] : c0 + cl;
  const int tid = threadIdx.x;
  const int r1 = rank_n[3 * cell], r2 = rank_n[3 * cell + 1], r3 = rank_n[3 * cell + 2];
  // cells whose larger rank of modes 1 and 2 is <= lo went through k_project_fib
  if ((r1 > r2 ? r1 : r2) <= lo) return;
  for (int o = tid; o < 3 * CS * N; o += kProjThreads)
    sW[o] = fac_n[(size_t)cell * 3 * CS * N + o];
  constexpr int MAXC = kMaxCap * kMaxCap * kMaxCap / kProjThreads;
  double acc[MAXC];
#pragma unroll
  for (int m = 0; m < MAXC; ++m) acc[m] = 0.0;
  const int tot = r1 * r2 * r3;
  const T* x = X + (size_t)cl * N * N * N;
  const double* W1 = sW;
  const double* W2 = sW + CS * N;
  const double* W3 = sW + 2 * CS * N;
  for (int i3 = 0; i3 < N; ++i3) {
    __syncthreads();
    for (int o = tid; o < N * N; o += kProjThreads) sS[o] = (double)x[(size_t)i3 * N * N + o];
    __syncthreads();
    // Q[k1][i2] = sum_i1 W1[k1][i1] S[i1 + N i2]
    for (int o = tid; o < r1 * N; o += kProjThreads) {
      const int i2 = o % N, k1 = o / N;
      double s = 0.0;
      for (int i1 = 0; i1 < N; ++i1) s += W1[k1 * N + i1] * sS[i1 + N * i2];
      sQ[k1 * N + i2] = s;
    }
    __syncthreads();
    // T[k1 + r1 k2] = sum_i2 Q[k1][i2] W2[k2][i2]
    for (int o = tid; o < r1 * r2; o += kProjThreads) {
      const int k1 = o % r1, k2 = o / r1;
      double s = 0.0;
      for (int i2 = 0; i2 < N; ++i2) s += sQ[k1 * N + i2] * W2[k2 * N + i2];
      sT[o] = s;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MAXC; ++m) {
      const int o = tid + kProjThreads * m;
      if (o < tot) {
        const int k12 = o % (r1 * r2), k3 = o / (r1 * r2);
        acc[m] += sT[k12] * W3[k3 * N + i3];
      }
    }
  }
  double* out = core_n + (size_t)cell * CS * CS * CS;
  for (int o = tid; o < CS * CS * CS; o += kProjThreads) {
    const int k1 = o % CS, t = o / CS, k2 = t % CS, k3 = t / CS;
    if (k1 >= r1 || k2 >= r2 || k3 >= r3) out[o] = 0.0;
  }
#pragma unroll
  for (int m = 0; m < MAXC; ++m) {
    const int o = tid + kProjThreads * m;
    if (o < tot) {
      const int k1 = o % r1, t = o / r1, k2 = t % r2, k3 = t / r2;
      out[k1 + CS * (k2 + CS * k3)] = acc[m];
    }
  }
}

// Variant for tensors whose first mode product fits the LDS: every thread
// reads whole mode-1 fibres (N contiguous values, coalesced across the
// workgroup) once, Y1 = W1^T A is kept in LDS, then Y2 = Y1 x2 W2^T and
// C = Y2 x3 W3^T; two barriers in total.  The LDS is laid out for ranks up
// to `cap` in modes 1 and 2.  A launch takes the cells whose larger rank of
// modes 1 and 2 lies in (lo, hi]; launches over consecutive rank tiers
// cover every cell once, the low tiers with room for several workgroups per
// CU.
template <int N, typename T>
__global__ __launch_bounds__(kProjThreads) void k_project_fib(const T* X, int c0, int CS, const double* fac_n,
                                                             const int* rank_n, double* core_n, int cap,
                                                             int lo, int hi, const int* cells,
                                                             const int* cells_n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sW = reinterpret_cast<double*>(smem_raw);    // 3 CS N
  double* sY2 = sW + 3 * CS * N;                       // cap cap N
  T* sY1 = reinterpret_cast<T*>(sY2 + cap * cap * N);  // cap N^2
  const int cl = blockIdx.x;
  if (cells && c0 + cl >= *cells_n) return;
  const int cell = cells ? cells[c0 + cl] : c0 + cl;
  const int tid = threadIdx.x;
  const int r1 = rank_n[3 * cell], r2 = rank_n[3 * cell + 1], r3 = rank_n[3 * cell + 2];
  const int r12 = r1 > r2 ? r1 : r2;
  if (r12 <= lo || r12 > hi) return;
  for (int o = tid; o < 3 * CS * N; o += kProjThreads) sW[o] = fac_n[(size_t)cell * 3 * CS * N + o];
  __syncthreads();
  const T* x = X + (size_t)cl * N * N * N;
  const double* W1 = sW;
  const double* W2 = sW + CS * N;
  const double* W3 = sW + 2 * CS * N;
  for (int p = tid; p < N * N; p += kProjThreads) {
    T f[N];
#pragma unroll
    for (int i = 0; i < N; ++i) f[i] = x[(size_t)p * N + i];
    for (int k1 = 0; k1 < r1; ++k1) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) s += W1[k1 * N + i] * (double)f[i];
      sY1[k1 * N * N + p] = (T)s;
    }
  }
  __syncthreads();
  // Y2[k1][k2][i3] = sum_i2 W2[k2][i2] Y1[k1][i2 + N i3]
  for (int o = tid; o < r1 * r2 * N; o += kProjThreads) {
    const int i3 = o % N, t = o / N, k2 = t % r2, k1 = t / r2;
    double s = 0.0;
    for (int i2 = 0; i2 < N; ++i2) s += W2[k2 * N + i2] * (double)sY1[k1 * N * N + i2 + N * i3];
    sY2[(k1 * r2 + k2) * N + i3] = s;
  }
  __syncthreads();
  double* out = core_n + (size_t)cell * CS * CS * CS;
  for (int o = tid; o < CS * CS * CS; o += kProjThreads) {
    const int k1 = o % CS, t = o / CS, k2 = t % CS, k3 = t / CS;
    double s = 0.0;
    if (k1 < r1 && k2 < r2 && k3 < r3) {
      const double* y = sY2 + (k1 * r2 + k2) * N;
      for (int i3 = 0; i3 < N; ++i3) s += W3[k3 * N + i3] * y[i3];
    }
    out[o] = s;
  }
}

template <int N, typename T>
size_t project_fib_bytes(int CS, int cap) {
  return sizeof(double) * (3 * (size_t)CS * N + (size_t)cap * cap * N) + sizeof(T) * (size_t)cap * N * N;
}

// rank tiers of the projection launches: (0, 6], (6, 9], (9, cap]
constexpr int kProjTier[2] = {6, 9};
// largest LDS layout of k_project_fib (one workgroup per CU); the tiers
// above it (large N and caps) go through the slice kernel
constexpr size_t kProjFibMax = (size_t)150 * 1024;

template <int N, typename T>
hipError_t launch_project_t(int count, const void* X, int c0, int CS, const double* fac_n, const int* rank_n,
                            double* core_n, hipStream_t s, const int* cells, const int* cells_n) {
  auto k = k_project_fib<N, T>;
  int lo = 0;
  bool attr = false;
  for (int t = 0; t <= 2 && lo < CS; ++t) {
    const int hi = (t < 2 && kProjTier[t] < CS) ? kProjTier[t] : CS;
    const size_t sh = project_fib_bytes<N, T>(CS, hi);
    if (sh > kProjFibMax) break;
    if (!attr) {
      // the largest layout this call launches
      size_t top = sh;
      for (int u = t + 1, l2 = hi; u <= 2 && l2 < CS; ++u) {
        const int h2 = (u < 2 && kProjTier[u] < CS) ? kProjTier[u] : CS;
        const size_t s2 = project_fib_bytes<N, T>(CS, h2);
        if (s2 > kProjFibMax) break;
        top = s2;
        l2 = h2;
      }
      const hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)top);
      if (e != hipSuccess) return e;
      attr = true;
    }
    hipLaunchKernelGGL(k, dim3(count), dim3(kProjThreads), sh, s, (const T*)X, c0, CS, fac_n, rank_n, core_n, hi,
                       lo, hi, cells, cells_n);
    lo = hi;
  }
  if (lo < CS) {
    const size_t sh = sizeof(double) * (N * N + 3 * CS * N + CS * N + CS * CS);
    hipLaunchKernelGGL((k_project<N, T>), dim3(count), dim3(kProjThreads), sh, s, (const T*)X, c0, CS, fac_n,
                       rank_n, core_n, cells, cells_n, lo);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_project(int N, int count, const void* X, int mixed, int c0, int CS, const double* fac_n,
                          const int* rank_n, double* core_n, hipStream_t s, const int* cells,
                          const int* cells_n) {
  if (count <= 0) return hipSuccess;
  if (mixed) {
    switch (N) {
      case 16: return launch_project_t<16, float>(count, X, c0, CS, fac_n, rank_n, core_n, s, cells, cells_n);
      case 24: return launch_project_t<24, float>(count, X, c0, CS, fac_n, rank_n, core_n, s, cells, cells_n);
      case 32: return launch_project_t<32, float>(count, X, c0, CS, fac_n, rank_n, core_n, s, cells, cells_n);
      case 48: return launch_project_t<48, float>(count, X, c0, CS, fac_n, rank_n, core_n, s, cells, cells_n);
    }
  } else {
    switch (N) {
      case 16: return launch_project_t<16, double>(count, X, c0, CS, fac_n, rank_n, core_n, s, cells, cells_n);
      case 24: return launch_project_t<24, double>(count, X, c0, CS, fac_n, rank_n, core_n, s, cells, cells_n);
      case 32: return launch_project_t<32, double>(count, X, c0, CS, fac_n, rank_n, core_n, s, cells, cells_n);
      case 48: return launch_project_t<48, double>(count, X, c0, CS, fac_n, rank_n, core_n, s, cells, cells_n);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace tk
