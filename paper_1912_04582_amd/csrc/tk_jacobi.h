// Symmetric eigen-decomposition by parallel cyclic Jacobi in LDS, the
// descending sort of the eigenvalues and the truncation rule of the rounding
// (Op4 / Op1), shared by the N-basis eigensolver (k_eig.hip) and the rounding
// in the space of the concatenated factors (k_rround.hip).
//
// Truncation rule: the rank of a mode is the smallest r >= 1 whose
// discarded eigenvalues (squared singular values of the unfolding, eq. svd)
// sum to at most eps^2 ||A||_F^2 / 3, then capped; this keeps
// ||A - B||_F <= eps ||A||_F when no cap applies.
#pragma once

#include <hip/hip_runtime.h>

namespace tk {
namespace {

// Parallel cyclic Jacobi on the n x n symmetric matrix A (leading dimension
// lda; n even), rotations accumulated into the columns of V (nv rows,
// leading dimension ldv).  Round-robin ordering: n/2 disjoint pairs per
// round, n-1 rounds per sweep; a pair rotates when |a_pq| exceeds both
// rel_thr sqrt(|a_pp a_qq|) and abs_thr.  Convergence is checked by a
// parallel scan of the off-diagonal elements before each sweep; `sweeps`
// (nullable) counts the sweeps run, which are also returned.  All threads of
// the block call it.
template <int NT, int NHMAX>
__device__ int jacobi(double* A, int lda, double* V, int ldv, int nv, int n, double rel_thr, double abs_thr,
                       double* cs, double* sn, double* tt, int* pp, int* qq, int* flag, int* conv,
                       unsigned long long* sweeps) {
  // the (I, J) pair blocks of the update, tabulated once per call
  __shared__ unsigned char b_i[NHMAX * (NHMAX + 1) / 2], b_j[NHMAX * (NHMAX + 1) / 2];
  const int lane = threadIdx.x;
  const int nh = n / 2;
  const int nblk = nh * (nh + 1) / 2;
  for (int b = lane; b < nblk; b += NT) {
    int I = 0, rem = b;
    while (rem >= nh - I) { rem -= nh - I; ++I; }
    b_i[b] = (unsigned char)I;
    b_j[b] = (unsigned char)(I + rem);
  }
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    if (lane == 0) {
      *conv = 1;
      flag[0] = 0;
      flag[1] = 0;
    }
    __syncthreads();
    for (int o = lane; o < n * n; o += NT) {
      const int i = o / n, j = o % n;
      if (j <= i) continue;
      const double apq = A[i * lda + j];
      if (fabs(apq) > fmax(rel_thr * sqrt(fabs(A[i * lda + i] * A[j * lda + j])), abs_thr)) *conv = 0;
    }
    __syncthreads();
    if (*conv) break;
    if (sweeps && lane == 0) atomicAdd(sweeps, 1ull);
    for (int r = 0; r < n - 1; ++r) {
      // flag[r & 1]: some pair of round r rotates.  The other flag is cleared
      // for the next round; its readers (round r - 1) have all passed that
      // round's last barrier, or read a value that is already 0.
      const int f = r & 1;
      if (lane < nh) {
        // round-robin pair of this lane in round r (no integer division:
        // both indices wrap at most once)
        int p, q;
        if (lane == 0) {
          p = 0;
          q = 1 + r;
        } else {
          int x = r + lane;
          if (x >= n - 1) x -= n - 1;
          int y = r + n - 1 - lane;
          if (y >= n - 1) y -= n - 1;
          p = 1 + x;
          q = 1 + y;
        }
        if (p > q) { const int t = p; p = q; q = t; }
        const double app = A[p * lda + p], aqq = A[q * lda + q], apq = A[p * lda + q];
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
      for (int b = lane; b < nblk; b += NT) {
        const int I = b_i[b], J = b_j[b];
        if (I == J) {
          const double t = tt[I];
          if (t != 0.0) {
            const int pI = pp[I], qI = qq[I];
            const double apq = A[pI * lda + qI];
            A[pI * lda + pI] -= t * apq;
            A[qI * lda + qI] += t * apq;
            A[pI * lda + qI] = 0.0;
            A[qI * lda + pI] = 0.0;
          }
        } else {
          const double sI = sn[I], sJ = sn[J];
          if (sI == 0.0 && sJ == 0.0) continue;
          const int pI = pp[I], qI = qq[I], pJ = pp[J], qJ = qq[J];
          const double cI = cs[I], cJ = cs[J];
          const double a = A[pI * lda + pJ], bb = A[pI * lda + qJ];
          const double cc = A[qI * lda + pJ], dd = A[qI * lda + qJ];
          const double a1 = cJ * a - sJ * bb, b1 = sJ * a + cJ * bb;
          const double c1 = cJ * cc - sJ * dd, d1 = sJ * cc + cJ * dd;
          const double a2 = cI * a1 - sI * c1, c2 = sI * a1 + cI * c1;
          const double b2 = cI * b1 - sI * d1, d2 = sI * b1 + cI * d1;
          A[pI * lda + pJ] = a2; A[pJ * lda + pI] = a2;
          A[pI * lda + qJ] = b2; A[qJ * lda + pI] = b2;
          A[qI * lda + pJ] = c2; A[pJ * lda + qI] = c2;
          A[qI * lda + qJ] = d2; A[qJ * lda + qI] = d2;
        }
      }
      for (int it = lane; it < nv * nh; it += NT) {
        const int row = it % nv, J = it / nv;
        const double c = cs[J], s = sn[J];
        if (s == 0.0) continue;
        const int p = pp[J], q = qq[J];
        const double v1 = V[row * ldv + p], v2 = V[row * ldv + q];
        V[row * ldv + p] = c * v1 - s * v2;
        V[row * ldv + q] = s * v1 + c * v2;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  return sweep;
}

// Sum of v over the 64 lanes of a wavefront by DPP lane moves (quad
// permutations, row rotations, then row broadcasts into the upper rows), in
// a fixed order; every lane receives the total (read from lane 63).
template <int CTRL, int RMASK>
__device__ inline double dpp_move(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, RMASK, 0xF, false);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, RMASK, 0xF, false);
  return __hiloint2double(h2, l2);
}

__device__ inline double wave_sum_dpp(double v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124, 0xF>(v);  // row_ror:4
  v += dpp_move<0x128, 0xF>(v);  // row_ror:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Orders the LDS accesses of one wavefront: its earlier stores are visible
// to its later loads from any lane (no workgroup barrier).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same parallel cyclic Jacobi (round-robin pairs, the same rotation
// formula and thresholds, each element updated by the same arithmetic) run
// by a single wavefront on its own matrix, synchronised within the wave only,
// so that several waves of a workgroup diagonalise their matrices at once.
// b_i/b_j: per-wave tables of NHMAX (NHMAX + 1) / 2 bytes; cs..qq: NHMAX
// entries.  Returns the sweeps run.
template <int NHMAX>
__device__ int jacobi_wave(double* A, int lda, double* V, int ldv, int nv, int n, double rel_thr, double abs_thr,
                           double* cs, double* sn, double* tt, int* pp, int* qq, unsigned char* b_i,
                           unsigned char* b_j) {
  const int lane = threadIdx.x & 63;
  const int nh = n / 2;
  const int nblk = nh * (nh + 1) / 2;
  for (int b = lane; b < nblk; b += 64) {
    int I = 0, rem = b;
    while (rem >= nh - I) { rem -= nh - I; ++I; }
    b_i[b] = (unsigned char)I;
    b_j[b] = (unsigned char)(I + rem);
  }
  wave_sync();
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    int big = 0;
    for (int o = lane; o < n * n; o += 64) {
      const int i = o / n, j = o % n;
      if (j <= i) continue;
      const double apq = A[i * lda + j];
      if (fabs(apq) > fmax(rel_thr * sqrt(fabs(A[i * lda + i] * A[j * lda + j])), abs_thr)) big = 1;
    }
    if (!__any(big)) break;
    for (int r = 0; r < n - 1; ++r) {
      int rot = 0;
      if (lane < nh) {
        int p, q;
        if (lane == 0) {
          p = 0;
          q = 1 + r;
        } else {
          int x = r + lane;
          if (x >= n - 1) x -= n - 1;
          int y = r + n - 1 - lane;
          if (y >= n - 1) y -= n - 1;
          p = 1 + x;
          q = 1 + y;
        }
        if (p > q) { const int t = p; p = q; q = t; }
        const double app = A[p * lda + p], aqq = A[q * lda + q], apq = A[p * lda + q];
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
          rot = 1;
        }
        pp[lane] = p; qq[lane] = q; cs[lane] = c; sn[lane] = s; tt[lane] = t;
      }
      if (!__any(rot)) continue;
      wave_sync();
      for (int b = lane; b < nblk; b += 64) {
        const int I = b_i[b], J = b_j[b];
        if (I == J) {
          const double t = tt[I];
          if (t != 0.0) {
            const int pI = pp[I], qI = qq[I];
            const double apq = A[pI * lda + qI];
            A[pI * lda + pI] -= t * apq;
            A[qI * lda + qI] += t * apq;
            A[pI * lda + qI] = 0.0;
            A[qI * lda + pI] = 0.0;
          }
        } else {
          const double sI = sn[I], sJ = sn[J];
          if (sI == 0.0 && sJ == 0.0) continue;
          const int pI = pp[I], qI = qq[I], pJ = pp[J], qJ = qq[J];
          const double cI = cs[I], cJ = cs[J];
          const double a = A[pI * lda + pJ], bb = A[pI * lda + qJ];
          const double cc = A[qI * lda + pJ], dd = A[qI * lda + qJ];
          const double a1 = cJ * a - sJ * bb, b1 = sJ * a + cJ * bb;
          const double c1 = cJ * cc - sJ * dd, d1 = sJ * cc + cJ * dd;
          const double a2 = cI * a1 - sI * c1, c2 = sI * a1 + cI * c1;
          const double b2 = cI * b1 - sI * d1, d2 = sI * b1 + cI * d1;
          A[pI * lda + pJ] = a2; A[pJ * lda + pI] = a2;
          A[pI * lda + qJ] = b2; A[qJ * lda + pI] = b2;
          A[qI * lda + pJ] = c2; A[pJ * lda + qI] = c2;
          A[qI * lda + qJ] = d2; A[qJ * lda + qI] = d2;
        }
      }
      for (int it = lane; it < nv * nh; it += 64) {
        const int row = it % nv, J = it / nv;
        const double c = cs[J], s = sn[J];
        if (s == 0.0) continue;
        const int p = pp[J], q = qq[J];
        const double v1 = V[row * ldv + p], v2 = V[row * ldv + q];
        V[row * ldv + p] = c * v1 - s * v2;
        V[row * ldv + q] = s * v1 + c * v2;
      }
      wave_sync();
    }
  }
  wave_sync();
  return sweep;
}

// Descending order of n <= 64 values d[0..n) (stable on ties) into order[],
// by one wavefront; the identity first, so that every entry stays a valid
// index even when comparisons fail (non-finite values).
__device__ inline void sort_desc_wave(const double* d, int stride, int n, int* order) {
  const int lane = threadIdx.x & 63;
  if (lane < n) order[lane] = lane;
  wave_sync();
  if (lane < n) {
    const double li = d[lane * stride];
    int pos = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = d[j * stride];
      pos += (lj > li) || (lj == li && j < lane);
    }
    if (pos < n) order[pos] = lane;
  }
  wave_sync();
}

// Descending order of the n values d[0..n) (stable on ties) into order[];
// the identity first so every entry stays a valid index.
template <int NT>
__device__ void sort_desc(const double* d, int stride, int n, int* order) {
  const int lane = threadIdx.x;
  for (int i = lane; i < n; i += NT) order[i] = i;
  __syncthreads();
  for (int i = lane; i < n; i += NT) {
    const double li = d[i * stride];
    int pos = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = d[j * stride];
      pos += (lj > li) || (lj == li && j < i);
    }
    if (pos < n) order[pos] = i;
  }
  __syncthreads();
}

// The truncation rule: smallest r >= 1 with extra + sum_{k >= r} lam_k <= thr
// (lam sorted descending, n of them), or with drop > 0 the count of values
// above drop^2 lam_0; then capped.
__device__ inline int choose_rank(const double* lam, int stride, const int* order, int n, double extra, double thr,
                                  double drop, int cap) {
  int r = n;
  if (drop > 0.0) {
    const double l0 = lam[order[0] * stride];
    r = 0;
    for (int k = 0; k < n; ++k)
      if (lam[order[k] * stride] > drop * drop * l0) ++r;
  } else {
    double tail = extra;
    if (tail > thr) return cap < n ? cap : n;  // the discarded block alone exceeds the budget
    for (int k = n - 1; k >= 1; --k) {
      tail += lam[order[k] * stride];
      if (tail <= thr) r = k;
      else break;
    }
  }
  if (r > cap) r = cap;
  if (r < 1) r = 1;
  return r;
}

}  // namespace
}  // namespace tk
