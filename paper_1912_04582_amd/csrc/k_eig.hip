// Symmetric eigen-decomposition of the mode Gram matrices and the
// truncation rule of the rounding (Op4 / Op1: ||A - B||_F <= eps ||A||_F).
//
// One workgroup per N x N matrix runs cyclic Jacobi with the parallel
// round-robin ordering (N/2 disjoint rotations per round, N-1 rounds per
// sweep) in LDS, until no off-diagonal element exceeds both
// rel_thr sqrt(|a_pp a_qq|) and abs_fac trace (FP64 path 1e-15 and 1e-18;
// mixed path 1e-12 and 1e-16, far below its FP32 term assembly).  Eigenvalues of G_a are the
// squared singular values of the mode-a unfolding (eq. svd).  The kept rank
// is the smallest r >= 1 whose discarded eigenvalues sum to at most
// eps^2 trace / 3, capped; the kept eigenvectors (sorted by decreasing
// eigenvalue) become the new factor, each column's largest-magnitude entry
// made positive.
//
// Warm start: a cell's Gram changes little from one time step to the next,
// so the full eigenbasis of the previous step is kept per cell and mode
// (`Wkeep`); the matrix is first rotated into it (A = W^T G W, V = W) and
// Jacobi then only removes the small off-diagonal remainder.  Rounds in
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

namespace tk {

namespace {

constexpr int kEigThreads = 256;

template <int N>
__global__ __launch_bounds__(kEigThreads) void k_eig(const double* Gm, const int* inst, const InstParams* ip,
                                                     int c0, double tol_o, int cap_o, int CS, double* fac_n,
                                                     int* rank_n, const double* Win, double* Wout, double* Wkeep,
                                                     double rel_thr, double abs_fac, double drop) {
  constexpr int NT = kEigThreads;
  constexpr int LD = N + 1;
  constexpr int NH = N / 2;
  constexpr int NBLK = NH * (NH + 1) / 2;
  __shared__ double A[N * LD];
  __shared__ double V[N * LD];
  __shared__ double Tm[N * LD];
  __shared__ double cs[NH], sn[NH], tt[NH];
  __shared__ int pp[NH], qq[NH];
  __shared__ int bi_[NBLK], bj_[NBLK];
  __shared__ int order[N];
  __shared__ int flag[2], s_conv;
  __shared__ double s_tot;
  __shared__ int s_rank;
  const int m = blockIdx.x;
  const int cl = m / 3, mode = m % 3;
  const int cell = c0 + cl;
  const int lane = threadIdx.x;
  const double* g = Gm + (size_t)m * N * N;
  double* wk = Wkeep ? Wkeep + ((size_t)cell * 3 + mode) * N * N : nullptr;
  for (int o = lane; o < N * N; o += NT) {
    const int i = o / N, j = o % N;
    A[i * LD + j] = g[o];
    // V[i][j]: entry i of vector j
    V[i * LD + j] = wk ? wk[j * N + i] : ((i == j) ? 1.0 : 0.0);
  }
  for (int b = lane; b < NBLK; b += NT) {
    int I = 0, rem = b;
    while (rem >= NH - I) { rem -= NH - I; ++I; }
    bi_[b] = I;
    bj_[b] = I + rem;
  }
  __syncthreads();
  if (lane == 0) {
    double t = 0.0;
    for (int i = 0; i < N; ++i) t += A[i * LD + i];
    s_tot = t;
  }
  if (wk) {
    // A <- V^T A V through Tm = A V
    for (int o = lane; o < N * N; o += NT) {
      const int i = o / N, j = o % N;
      double s = 0.0;
      for (int k = 0; k < N; ++k) s += A[i * LD + k] * V[k * LD + j];
      Tm[i * LD + j] = s;
    }
    __syncthreads();
    for (int o = lane; o < N * N; o += NT) {
      const int i = o / N, j = o % N;
      if (j < i) continue;
      double s = 0.0;
      for (int k = 0; k < N; ++k) s += V[k * LD + i] * Tm[k * LD + j];
      A[i * LD + j] = s;
      A[j * LD + i] = s;
    }
  }
  __syncthreads();
  const double abs_thr = abs_fac * fabs(s_tot);
  for (int sweep = 0; sweep < 40; ++sweep) {
    // converged when no off-diagonal element exceeds the rotation threshold
    if (lane == 0) {
      s_conv = 1;
      flag[0] = 0;
      flag[1] = 0;
    }
    __syncthreads();
    for (int o = lane; o < N * N; o += NT) {
      const int i = o / N, j = o % N;
      if (j <= i) continue;
      const double apq = A[i * LD + j];
      if (fabs(apq) > fmax(rel_thr * sqrt(fabs(A[i * LD + i] * A[j * LD + j])), abs_thr)) s_conv = 0;
    }
    __syncthreads();
    if (s_conv) break;
    for (int r = 0; r < N - 1; ++r) {
      // flag[r & 1]: some pair of round r rotates.  The other flag is cleared
      // for the next round; its readers (round r - 1) have all passed that
      // round's last barrier, or read a value that is already 0.
      const int f = r & 1;
      if (lane < NH) {
        int p, q;
        if (lane == 0) {
          p = 0;
          q = 1 + r % (N - 1);
        } else {
          p = 1 + (r + lane) % (N - 1);
          q = 1 + (r + N - 1 - lane) % (N - 1);
        }
        if (p > q) { const int t = p; p = q; q = t; }
        const double app = A[p * LD + p], aqq = A[q * LD + q], apq = A[p * LD + q];
        double c = 1.0, s = 0.0, t = 0.0;
        if (fabs(apq) > fmax(rel_thr * sqrt(fabs(app * aqq)), abs_thr) && apq != 0.0) {
          const double th = (aqq - app) / (2.0 * apq);
          if (fabs(th) > 1e150) {
            t = 0.5 / th;
          } else {
            t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          }
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
          flag[f] = 1;
        }
        pp[lane] = p; qq[lane] = q; cs[lane] = c; sn[lane] = s; tt[lane] = t;
      }
      if (lane == 0) flag[f ^ 1] = 0;
      __syncthreads();
      if (!flag[f]) continue;
      for (int b = lane; b < NBLK; b += NT) {
        const int I = bi_[b], J = bj_[b];
        if (I == J) {
          const double t = tt[I];
          if (t != 0.0) {
            const int pI = pp[I], qI = qq[I];
            const double apq = A[pI * LD + qI];
            A[pI * LD + pI] -= t * apq;
            A[qI * LD + qI] += t * apq;
            A[pI * LD + qI] = 0.0;
            A[qI * LD + pI] = 0.0;
          }
        } else {
          const double sI = sn[I], sJ = sn[J];
          if (sI == 0.0 && sJ == 0.0) continue;
          const int pI = pp[I], qI = qq[I], pJ = pp[J], qJ = qq[J];
          const double cI = cs[I], cJ = cs[J];
          const double a = A[pI * LD + pJ], bb = A[pI * LD + qJ];
          const double cc = A[qI * LD + pJ], dd = A[qI * LD + qJ];
          const double a1 = cJ * a - sJ * bb, b1 = sJ * a + cJ * bb;
          const double c1 = cJ * cc - sJ * dd, d1 = sJ * cc + cJ * dd;
          const double a2 = cI * a1 - sI * c1, c2 = sI * a1 + cI * c1;
          const double b2 = cI * b1 - sI * d1, d2 = sI * b1 + cI * d1;
          A[pI * LD + pJ] = a2; A[pJ * LD + pI] = a2;
          A[pI * LD + qJ] = b2; A[qJ * LD + pI] = b2;
          A[qI * LD + pJ] = c2; A[pJ * LD + qI] = c2;
          A[qI * LD + qJ] = d2; A[qJ * LD + qI] = d2;
        }
      }
      for (int it = lane; it < N * NH; it += NT) {
        const int row = it % N, J = it / N;
        const double c = cs[J], s = sn[J];
        if (s == 0.0) continue;
        const int p = pp[J], q = qq[J];
        const double v1 = V[row * LD + p], v2 = V[row * LD + q];
        V[row * LD + p] = c * v1 - s * v2;
        V[row * LD + q] = s * v1 + c * v2;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // sort eigenvalues, descending (stable on ties); the identity order first so
  // that every entry stays a valid index even if a value is not a number
  if (lane < N) order[lane] = lane;
  __syncthreads();
  if (lane < N) {
    const double li = A[lane * LD + lane];
    int pos = 0;
    for (int j = 0; j < N; ++j) {
      const double lj = A[j * LD + j];
      pos += (lj > li) || (lj == li && j < lane);
    }
    if (pos < N) order[pos] = lane;
  }
  __syncthreads();
  if (wk) {
    for (int o = lane; o < N * N; o += NT) {
      const int k = o / N, i = o % N;
      wk[o] = V[i * LD + order[k]];
    }
  }
  if (Wout) {
    // full sorted basis (premultiplied by Win when given), no truncation
    double* out = Wout + (size_t)m * N * N;
    for (int o = lane; o < N * N; o += NT) {
      const int k = o / N, i = o % N, j = order[k];
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
  if (lane == 0) {
    double tol = tol_o;
    int cap = cap_o;
    if (inst) {
      const InstParams P = ip[inst[cell]];
      tol = P.tol;
      cap = P.cap;
    }
    double tot = 0.0;
    for (int i = 0; i < N; ++i) tot += A[order[i] * LD + order[i]];
    const double thr = tol * tol * tot / 3.0;
    int r = N;
    if (drop > 0.0) {
      // keep singular values above drop * sigma_1 (eigenvalues above drop^2 lambda_1)
      const double l0 = A[order[0] * LD + order[0]];
      r = 0;
      for (int k = 0; k < N; ++k)
        if (A[order[k] * LD + order[k]] > drop * drop * l0) ++r;
    } else {
      // smallest r >= 1 with sum_{k >= r} lambda_k <= thr
      double tail = 0.0;
      for (int k = N - 1; k >= 1; --k) {
        tail += A[order[k] * LD + order[k]];
        if (tail <= thr) r = k;
        else break;
      }
    }
    if (r > cap) r = cap;
    if (r < 1) r = 1;
    s_rank = r;
    rank_n[3 * cell + mode] = r;
  }
  __syncthreads();
  const int r = s_rank;
  double* out = fac_n + ((size_t)cell * 3 + mode) * CS * N;
  double* vec = Tm;
  for (int k = 0; k < CS; ++k) {
    if (k < r) {
      const int j = order[k];
      for (int i = lane; i < N; i += NT) {
        double v;
        if (Win) {
          const double* w = Win + (size_t)m * N * N;
          v = 0.0;
          for (int t = 0; t < N; ++t) v += w[t * N + i] * V[t * LD + j];
        } else {
          v = V[i * LD + j];
        }
        vec[i] = v;
      }
      __syncthreads();
      // canonical sign: largest-magnitude entry positive (first on ties)
      if (lane == 0) {
        double best = -1.0;
        int bi = 0;
        for (int i = 0; i < N; ++i) {
          const double v = fabs(vec[i]);
          if (v > best) { best = v; bi = i; }
        }
        cs[0] = (vec[bi] < 0.0) ? -1.0 : 1.0;
      }
      __syncthreads();
      const double sg = cs[0];
      for (int i = lane; i < N; i += NT) out[k * N + i] = sg * vec[i];
      __syncthreads();
    } else {
      for (int i = lane; i < N; i += NT) out[k * N + i] = 0.0;
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
                      hipStream_t s, double drop) {
  if (count <= 0) return hipSuccess;
  dim3 grid(3 * count), blk(kEigThreads);
#define TK_EIG(NN) hipLaunchKernelGGL(k_eig<NN>, grid, blk, 0, s, G, inst, ip, c0, tol_override, cap_override, CS, \
                                      fac_n, rank_n, Win, Wout, Wkeep, rel_thr, abs_fac, drop)
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
