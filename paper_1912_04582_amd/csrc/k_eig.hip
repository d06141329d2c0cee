// Symmetric eigen-decomposition of the mode Gram matrices and the
// truncation rule of the rounding (Op4 / Op1: ||A - B||_F <= eps ||A||_F).
//
// One workgroup per N x N matrix runs cyclic Jacobi with the parallel
// round-robin ordering (N/2 disjoint rotations per round, N-1 rounds per
// sweep) in LDS, until no off-diagonal element exceeds both
// rel_thr sqrt(|a_pp a_qq|) and abs_fac trace, the latter capped at 1e-2 of
// the truncation budget (FP64 path 1e-15 and 1e-18; mixed path 1e-12 and
// 1e-13: the FP32 term assembly leaves noise among the smallest directions
// whose couplings to the kept ones hover near a lower floor, so every step
// re-rotated them for nothing).  The discarded energy is read from the
// diagonal of an orthonormal rotation of G, so the error bound holds at any
// convergence level; the
// thresholds only decide how close to optimal the kept subspace is.
// Eigenvalues of G_a are the
// squared singular values of the mode-a unfolding (eq. svd).  The kept rank
// is the smallest r >= 1 whose discarded eigenvalues sum to at most
// eps^2 trace / 3, capped; the kept eigenvectors (sorted by decreasing
// eigenvalue) become the new factor, each column's largest-magnitude entry
// made positive.
//
// Warm start: a cell's Gram changes little from one time step to the next,
// so the full eigenbasis of the previous step is kept per cell and mode
// (`Wkeep`); the matrix is first rotated into it (A = W^T G W, V = W, two
// N x N products on the FP64 matrix cores) and Jacobi then only removes the
// small off-diagonal remainder.  Rounds in
// which no pair needs a rotation skip the update passes; convergence is
// checked by a parallel scan of the off-diagonal elements before each sweep.
//
// Accuracy: a Gram matrix formed in FP64 carries errors of order
// eps ||A||^2, which move the kept subspace by eps sigma_1^2 / sigma_r.  The
// FP64 path therefore runs a second pass: the unfolding is rotated by the
// first basis W, B = W^T A_(a), the Gram of B (whose errors scale with its
// row norms) is diagonalised again and the final vectors are W V'.  For
// that pass the kernel takes the first basis as `Win`; with `Wout` it
// returns the full sorted basis instead of the truncated factor.
//
// Basis layouts (Wkeep, Win, Wout): vector k, entry i at [k N + i].
#include "tk_internal.h"
#include "tk_jacobi.h"

namespace tk {

namespace {

constexpr int kEigThreads = 256;

typedef double v4d __attribute__((ext_vector_type(4)));

// Warm-start rotation A <- V^T G V (G held in A) on the FP64 matrix cores,
// v_mfma_f64_16x16x4f64 on 16x16 blocks: lane (ii, kk) feeds row ii /
// column ii of the operands at k0 + kk and holds rows kk + 4r of column ii
// of the result.  Each wavefront takes blocks (bi, bj >= bi) of the result:
// it first forms column block bj of T = G V in registers, whose layout is
// that of the second product's right operand (rows 16b + 4r + kk, column
// ii), then accumulates V^T T over those rows.  The results are written
// after every wavefront has read G, mirrored so that A stays exactly
// symmetric.  Rows and columns beyond N read as zero and are not written;
// N is a multiple of 4.
template <int N, int LD>
__device__ void warm_rotate(double* A, const double* V) {
  static_assert(N % 4 == 0, "k steps of 4");
  constexpr int NB = (N + 15) / 16;
  constexpr int NU = NB * (NB + 1) / 2;
  constexpr int NW = kEigThreads / 64;
  constexpr int MT = (NU + NW - 1) / NW;
  const int wave = threadIdx.x >> 6;
  const int ii = threadIdx.x & 15, kk = (threadIdx.x >> 4) & 3;
  v4d res[MT];
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int t = wave + u * NW;
    res[u] = v4d{0.0, 0.0, 0.0, 0.0};
    if (t >= NU) continue;
    int bi = 0, rest = t;
    while (rest >= NB - bi) {
      rest -= NB - bi;
      ++bi;
    }
    const int bj = bi + rest;
    const int row = 16 * bi + ii, col = 16 * bj + ii;
    v4d tm[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int gr = 16 * b + ii;
      v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int k0 = 0; k0 < N; k0 += 4) {
        const int k = k0 + kk;
        const double a = gr < N ? A[gr * LD + k] : 0.0;
        const double v = col < N ? V[k * LD + col] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, v, acc, 0, 0, 0);
      }
      tm[b] = acc;
    }
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (16 * b + 4 * r >= N) continue;
        const int k = 16 * b + 4 * r + kk;
        const double a = row < N ? V[k * LD + row] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, tm[b][r], acc, 0, 0, 0);
      }
    res[u] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int t = wave + u * NW;
    if (t >= NU) continue;
    int bi = 0, rest = t;
    while (rest >= NB - bi) {
      rest -= NB - bi;
      ++bi;
    }
    const int bj = bi + rest;
    const int col = 16 * bj + ii;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * bi + kk + 4 * r;
      if (i < N && col < N && (bi != bj || i <= col)) {
        A[i * LD + col] = res[u][r];
        A[col * LD + i] = res[u][r];
      }
    }
  }
  __syncthreads();
}

// The truncation rule on one wavefront (all 64 lanes call it, n <= 64):
// lane k reads the k-th largest eigenvalue, the discarded tail is summed
// from the smallest one upward in the same order as a serial loop, its
// terms broadcast from the lanes' registers, so the result is bitwise that
// of the serial rule.  Returns the rank r >= 1, capped.
__device__ int choose_rank_wave(const double* lam, int stride, const int* order, int n, double thr, double drop,
                                int cap) {
  const int wl = threadIdx.x & 63;
  const double lk = wl < n ? lam[order[wl] * stride] : 0.0;
  int r = n;
  if (drop > 0.0) {
    const double l0 = __shfl(lk, 0, 64);
    r = __popcll(__ballot(wl < n && lk > drop * drop * l0));
  } else if (!(0.0 > thr)) {  // a negative budget keeps every vector
    double tail = 0.0;
    for (int k = n - 1; k >= 1; --k) {
      const int lo = __builtin_amdgcn_readlane(__double2loint(lk), k);
      const int hi = __builtin_amdgcn_readlane(__double2hiint(lk), k);
      tail += __hiloint2double(hi, lo);
      if (tail <= thr)
        r = k;
      else
        break;
    }
  }
  if (r > cap) r = cap;
  if (r < 1) r = 1;
  return r;
}

}  // namespace

// Eigensolver statistics: [1] matrices solved, [2] Jacobi sweeps run ([0]
// and [3] stay zero).
__device__ unsigned long long g_eig_stats[4];

namespace {

// LDS holds the matrix and the basis (2 N (N + 1) doubles): eight
// workgroups per CU up to N = 32 (64 registers; two spilled at N = 32),
// four at N = 48.
template <int N>
__global__ __launch_bounds__(kEigThreads) __attribute__((amdgpu_waves_per_eu(N >= 48 ? 4 : 8))) void k_eig(const double* Gm, const int* inst, const InstParams* ip,
                                                     int c0, double tol_o, int cap_o, int CS, double* fac_n,
                                                     int* rank_n, const double* Win, double* Wout, double* Wkeep,
                                                     double rel_thr, double abs_fac, double drop,
                                                     const int* cells, const int* cells_n, int* wvalid) {
  constexpr int NT = kEigThreads;
  constexpr int LD = N + 1;
  constexpr int NH = N / 2;
  __shared__ double A[N * LD];
  __shared__ double V[N * LD];
  __shared__ double cs[NH], sn[NH], tt[NH];
  __shared__ int pp[NH], qq[NH];
  __shared__ int order[N];
  __shared__ int flag[2], s_conv;
  __shared__ int s_rank;
  const int m = blockIdx.x;
  const int cl = m / 3, mode = m % 3;
  // a pass over a device-side cell list ends at its count
  if (cells && c0 + cl >= *cells_n) return;
  const int cell = cells ? cells[c0 + cl] : c0 + cl;
  const int lane = threadIdx.x;
  const double* g = Gm + (size_t)m * N * N;
  double* wk = Wkeep ? Wkeep + ((size_t)cell * 3 + mode) * N * N : nullptr;
  // the kept basis is a usable warm start unless the cell was last rounded
  // in the space of its concatenated factors (it is written again below)
  // (one flag per cell and mode, read and written only by this workgroup)
  const double* wr = (wk && (!wvalid || wvalid[3 * cell + mode])) ? wk : nullptr;
  double tol = tol_o;
  int cap = cap_o;
  if (inst) {
    const InstParams P = ip[inst[cell]];
    tol = P.tol;
    cap = P.cap;
  }
  // the matrix and the previous basis (V[i][j]: entry i of vector j), both
  // requested before either is used
  {
    constexpr int PER = (N * N + NT - 1) / NT;
    double ga[PER], wa[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int o = lane + t * NT;
      if (o < N * N) {
        ga[t] = g[o];
        wa[t] = wr ? wr[o] : (((o / N) == (o % N)) ? 1.0 : 0.0);
      }
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int o = lane + t * NT;
      if (o < N * N) {
        A[(o / N) * LD + o % N] = ga[t];
        V[(o % N) * LD + o / N] = wa[t];
      }
    }
  }
  __syncthreads();
  // trace, reduced by every wave
  double tot = 0.0;
  {
    const int d = lane & 63;
    if (d < N) tot = A[d * LD + d];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
  }
  const double thr = tol * tol * tot / 3.0;
  // off-diagonal floor: abs_fac of the trace, but never above 1e-2 of the
  // truncation budget: a coupling that small moves at most its square over
  // the eigenvalue gap across the cut (far below the budget), and turns the
  // smallest kept directions by at most 1e-2 radian
  const double abs_thr = thr > 0.0 ? fmin(abs_fac * fabs(tot), 1e-2 * thr) : abs_fac * fabs(tot);
  // full warm start: A <- V^T G V
  if (wr) warm_rotate<N, LD>(A, V);
  if (lane == 0) atomicAdd(&g_eig_stats[1], 1ull);
  jacobi<NT, NH>(A, LD, V, LD, N, N, rel_thr, abs_thr, cs, sn, tt, pp, qq, flag, &s_conv, &g_eig_stats[2]);
  sort_desc<NT>(A, LD + 1, N, order);
  if (wk) {
    for (int o = lane; o < N * N; o += NT) {
      const int kk = o / N, i = o % N;
      wk[o] = V[i * LD + order[kk]];
    }
    if (wvalid && lane == 0) wvalid[3 * cell + mode] = 1;
  }
  if (Wout) {
    // full sorted basis (premultiplied by Win when given), no truncation
    double* out = Wout + (size_t)m * N * N;
    for (int o = lane; o < N * N; o += NT) {
      const int kk = o / N, i = o % N, j = order[kk];
      double v;
      if (Win) {
        const double* w = Win + (size_t)m * N * N;
        v = 0.0;
        for (int t = 0; t < N; ++t) v += w[t * N + i] * V[t * LD + j];
      } else {
        v = V[i * LD + j];
      }
      out[o] = v;
    }
    return;
  }
  if (lane < 64) {
    const int r = choose_rank_wave(A, LD + 1, order, N, thr, drop, cap);
    if (lane == 0) {
      s_rank = r;
      rank_n[3 * cell + mode] = r;
    }
  }
  __syncthreads();
  const int r = s_rank;
  // one wavefront per output column: the kept vectors (premultiplied by Win
  // when given) with their canonical sign, largest-magnitude entry positive
  // (the first on ties; a NaN entry never counts as largest), then zeros
  double* out = fac_n + ((size_t)cell * 3 + mode) * CS * N;
  const int wl = lane & 63;
  for (int c = lane >> 6; c < CS; c += NT / 64) {
    if (c < r) {
      const int j = order[c];
      double v = 0.0;
      if (wl < N) {
        if (Win) {
          const double* w = Win + (size_t)m * N * N;
          for (int t = 0; t < N; ++t) v += w[t * N + wl] * V[t * LD + j];
        } else {
          v = V[wl * LD + j];
        }
      }
      const double av = fabs(v);
      double key = (wl < N && av == av) ? av : -1.0;
      int idx = wl;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ok = __shfl_xor(key, off, 64);
        const int oi = __shfl_xor(idx, off, 64);
        if (ok > key || (ok == key && oi < idx)) {
          key = ok;
          idx = oi;
        }
      }
      const double sg = (__shfl(v, idx, 64) < 0.0) ? -1.0 : 1.0;
      if (wl < N) out[c * N + wl] = sg * v;
    } else if (wl < N) {
      out[c * N + wl] = 0.0;
    }
  }
}

__global__ void k_absxi(int N, const double* nrm, double xi_min, double dxi, double* X) {
  const int f = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * N * N) return;
  const int i1 = e % N, i2 = (e / N) % N, i3 = e / (N * N);
  const double* n = nrm + 3 * (size_t)f;
  X[(size_t)f * N * N * N + e] =
      fabs(n[0] * (xi_min + i1 * dxi) + n[1] * (xi_min + i2 * dxi) + n[2] * (xi_min + i3 * dxi));
}

__global__ void k_identity_basis(int N, size_t count, double* W) {
  const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= count * N * N) return;
  const int r = (int)(o % ((size_t)N * N));
  W[o] = (r / N == r % N) ? 1.0 : 0.0;
}

}  // namespace

hipError_t launch_eig(int N, int count, const double* G, const int* inst, const InstParams* ip, int c0,
                      double tol_override, int cap_override, int CS, double* fac_n, int* rank_n,
                      const double* Win, double* Wout, double* Wkeep, double rel_thr, double abs_fac,
                      hipStream_t s, double drop, const int* cells, const int* cells_n, int* wvalid) {
  if (count <= 0) return hipSuccess;
  dim3 grid(3 * count), blk(kEigThreads);
#define TK_EIG(NN) hipLaunchKernelGGL(k_eig<NN>, grid, blk, 0, s, G, inst, ip, c0, tol_override, cap_override, CS, \
                                      fac_n, rank_n, Win, Wout, Wkeep, rel_thr, abs_fac, drop, \
                                      cells, cells_n, wvalid)
  switch (N) {
    case 16: TK_EIG(16); break;
    case 24: TK_EIG(24); break;
    case 32: TK_EIG(32); break;
    case 48: TK_EIG(48); break;
    default: return hipErrorInvalidValue;
  }
#undef TK_EIG
  return hipGetLastError();
}

hipError_t launch_identity_basis(int N, size_t count, double* W, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const size_t tot = count * N * N;
  hipLaunchKernelGGL(k_identity_basis, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, N, count, W);
  return hipGetLastError();
}

}  // namespace tk

namespace tk {
hipError_t launch_absxi(int N, int count, const double* normals, double xi_min, double dxi, double* X,
                        hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int ne = N * N * N;
  hipLaunchKernelGGL(k_absxi, dim3((ne + 255) / 256, count), dim3(256), 0, s, N, normals, xi_min, dxi, X);
  return hipGetLastError();
}
}  // namespace tk

namespace tk {
hipError_t eig_stats(unsigned long long* out, bool reset) {
  hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_eig_stats), sizeof(unsigned long long) * 4);
  if (e == hipSuccess && reset) {
    unsigned long long z[4] = {0, 0, 0, 0};
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_eig_stats), z, sizeof(z));
  }
  return e;
}
}  // namespace tk
