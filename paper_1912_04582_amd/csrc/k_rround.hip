// Rounding in the space of the concatenated factors (Op4 as the paper
// describes Tucker rounding: QR of the factors, the core multiplied by the
// R factors, SVDs of the small core's unfoldings), fused with the term
// assembly of one explicit step, one workgroup per cell.
//
// The update f* = f + dt R of a cell on axis-aligned faces is a sum of
// Tucker terms (eq. exact-flux in gather form, Alg. 1 steps 2-9; Op2 sums,
// Op3 products with rank-1 row scalings):
//
//   f* = (1 - dt nu) f + sum_a d_a o_a f + dt nu f_S + sum_l b_l o_{a_l} g_l,
//   d_a(i) = -sum_{l on axis a} (dt A_l / V) max(s_l xi_i, 0),
//   b_l(i) = (dt A_l / V) max(-s_l xi_i, 0),
//
// where o_a scales the rows of mode a, f_S is the rank-4 S-model
// equilibrium (Alg. 2 steps 10-11, Proposition 1) and g_l the far side of
// face l (neighbour state or boundary ghost).  Per mode a the factor of the
// sum is the concatenation Ucat_a = [U_a, d_a U_a, F_a, far sides] with
// r0_a = 2 r_a + 4 + sum_l q_l,a columns; its core is block-sparse.
//
// Steps per cell:
//  1. Ucat_a in LDS (the own factor, its scaled copy, the f_S columns
//     m_a (xi - u_a)^k, the far sides with their row scaling and, for a
//     symmetry ghost, the reversed velocity index).
//  2. Ucat_a = Q_a R_a by classical Gram-Schmidt with one
//     re-orthogonalisation, one wavefront per mode.  A column whose
//     component outside the span of the previous ones is at most 1e-13 of
//     its norm adds no basis vector (its R column still holds its
//     coordinates): m_a <= r0_a basis vectors remain, and the tensor
//     changes by at most that fraction of each term.
//  3. The small core G' = sum_t G_t x_1 R_1[:, cols] x_2 R_2[:, cols]
//     x_3 R_3[:, cols] (m_1 x m_2 x m_3) in LDS.  The rounded tensor is then
//     G' x_a Q_a, and its mode-a singular values are those of G'_(a).
//  4. Per mode: the Gram G'_(a) G'_(a)^T (FP64) is diagonalised by Jacobi,
//     G' is rotated by the eigenvectors, and the Gram of the rotated
//     unfolding is diagonalised again (a Gram formed in FP64 moves small
//     singular directions by eps sigma_1^2 / sigma_r; the second pass has
//     errors that scale with its own rows), after which G' is rotated
//     again.  The rank rule of the truncated HOSVD (T-HOSVD, independent
//     per mode) is applied to the eigenvalues.
//  5. Factors Q_a V_a[:, kept] with the canonical sign (largest-magnitude
//     entry positive), core = the kept block of the rotated G'.
//
// FP64 throughout on both precision paths (on this device FP64 and FP32
// vector arithmetic without packed instructions retire at the same rate).
// A cell that does not fit a tier's layout (r0_a or a source rank above the
// tier's bounds, an oblique face, or m_1 m_2 m_3 above its core capacity)
// is appended to `next` and left to the next tier or the N-basis path.
#include "tk_internal.h"
#include "tk_jacobi.h"

namespace tk {

namespace {

constexpr int kRThreads = 256;
constexpr double kQrDrop = 1e-13;  // Gram-Schmidt: relative norm below which a column adds no vector

// far side of one face slot
struct RSide {
  int type;  // 0 state of cell idx, 1 boundary Maxwellian idx
  int idx;
  int q[3];
  int rev;   // reversed axis (symmetry ghost) or -1
  int sax;   // scaled axis
  double coef, sig, gsc;
  int off[3];  // first column per mode
};

template <int N, int RM>
struct RLds {
  static constexpr int U = 3 * RM * N;                    // Ucat, then Q
  static constexpr int R = 3 * RM * RM;                   // R, then the rotations V
  static constexpr int A = (RM * (RM + 1) > N * RM) ? RM * (RM + 1) : N * RM;  // Jacobi matrix / W
  static constexpr int V = RM * (RM + 1);                 // Jacobi vectors
};

template <int N, int RM, int GM, int QM>
constexpr size_t rround_lds_bytes() {
  return sizeof(double) * (RLds<N, RM>::U + RLds<N, RM>::R + GM + RLds<N, RM>::A + RLds<N, RM>::V + QM * QM * QM);
}

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One cell; returns false (uniformly) when the cell is left to the next tier.
template <int N, int RM, int GM, int QM>
__device__ bool rround_cell(const DevState& d, int c, double* smem, unsigned long long* sweeps) {
  constexpr int NT = kRThreads;
  constexpr int LDA = RM + 1;
  double* sU = smem;
  double* sR = sU + RLds<N, RM>::U;
  double* sG = sR + RLds<N, RM>::R;
  double* sA = sG + GM;
  double* sV = sA + RLds<N, RM>::A;
  double* sC = sV + RLds<N, RM>::V;
  __shared__ RSide s_side[kSlots];
  __shared__ int s_ns, s_ok, s_r[3], s_r0[3], s_m[3], s_nr[3];
  __shared__ signed char s_src[3][RM], s_k[3][RM];  // column source (0 own, 1 own scaled, 2 f_S, 3+l far) and index
  __shared__ double s_d[3][N], s_fb[3][N], s_fv[3][N];  // d_a, f_S base and xi - u_a
  __shared__ double s_c1[3][RM], s_c2[3][RM];
  __shared__ double s_lam[3][RM];
  __shared__ int s_order[3][RM];
  __shared__ double s_sign[3][kMaxCap];
  __shared__ double s_fs[64];
  __shared__ double s_cs[RM / 2], s_sn[RM / 2], s_tt[RM / 2];
  __shared__ int s_pp[RM / 2], s_qq[RM / 2], s_flag[2], s_conv;
  __shared__ double s_tr;
  const int tid = threadIdx.x;
  const int CS = d.CS;
  const InstParams P = d.ip[d.inst[c]];
  const double nu = d.nu[c];

  // ---- sources, column tables, eligibility (one thread) ----------------------
  if (tid == 0) {
    int ok = 1;
    int r[3];
    for (int a = 0; a < 3; ++a) r[a] = d.rank[3 * c + a];
    int ns = 0;
    int off[3];
    for (int a = 0; a < 3; ++a) off[a] = 2 * r[a] + 4;
    for (int a = 0; a < 3; ++a) ok &= (r[a] <= QM) ? 1 : 0;
    for (int l = 0; l < kSlots && ok; ++l) {
      const size_t sl = (size_t)kSlots * c + l;
      const int kind = d.slot_kind[sl];
      if (kind == SK_NONE) continue;
      const int ax = d.slot_axis[sl];
      if (ax < 0) { ok = 0; break; }
      RSide e;
      e.rev = -1;
      e.sax = ax;
      e.coef = d.slot_coef[sl];
      e.sig = (double)d.slot_sig[sl];
      e.gsc = 1.0;
      const int nb = d.slot_nb[sl];
      if (kind == SK_INTERIOR || kind == SK_OUTFLOW || kind == SK_SYM) {
        e.type = 0;
        e.idx = (kind == SK_INTERIOR) ? nb : c;
        if (kind == SK_SYM) e.rev = ax;
        for (int a = 0; a < 3; ++a) e.q[a] = d.rank[3 * e.idx + a];
      } else {
        e.type = 1;
        e.idx = nb;
        e.q[0] = e.q[1] = e.q[2] = 1;
        if (kind == SK_WALL) e.gsc = d.nw[sl];
      }
      for (int a = 0; a < 3; ++a) {
        ok &= (e.q[a] <= QM) ? 1 : 0;
        e.off[a] = off[a];
        off[a] += e.q[a];
      }
      s_side[ns++] = e;
    }
    for (int a = 0; a < 3; ++a) ok &= (off[a] <= RM) ? 1 : 0;
    if (ok) {
      for (int a = 0; a < 3; ++a) {
        s_r[a] = r[a];
        s_r0[a] = off[a];
        int col = 0;
        for (int k = 0; k < r[a]; ++k) { s_src[a][col] = 0; s_k[a][col++] = (signed char)k; }
        for (int k = 0; k < r[a]; ++k) { s_src[a][col] = 1; s_k[a][col++] = (signed char)k; }
        for (int k = 0; k < 4; ++k) { s_src[a][col] = 2; s_k[a][col++] = (signed char)k; }
        for (int l = 0; l < ns; ++l)
          for (int k = 0; k < s_side[l].q[a]; ++k) { s_src[a][col] = (signed char)(3 + l); s_k[a][col++] = (signed char)k; }
      }
    }
    s_ns = ns;
    s_ok = ok;
  }
  __syncthreads();
  if (!s_ok) return false;
  const int ns = s_ns;

  // ---- 1-D tables: d_a, f_S factors ---------------------------------------
  const double* M = d.macro + 8 * (size_t)c;
  const double n0 = M[0], T0 = M[4];
  const double RT = P.Rg * T0;
  const double beta = 1.0 / (2.0 * RT);
  for (int o = tid; o < 3 * N; o += NT) {
    const int a = o / N, i = o % N;
    const double x = P.xi_min + i * P.dxi;
    double s = 0.0;
    for (int l = 0; l < kSlots; ++l) {
      const size_t sl = (size_t)kSlots * c + l;
      if (d.slot_kind[sl] == SK_NONE || d.slot_axis[sl] != a) continue;
      s -= d.slot_coef[sl] * fmax((double)d.slot_sig[sl] * x, 0.0);
    }
    s_d[a][i] = s;
    const double v = x - M[1 + a];
    s_fv[a][i] = v;
    s_fb[a][i] = cbrt(n0) / sqrt(2.0 * M_PI * RT) * exp(-v * v * beta);
  }
  if (tid == 0) {
    // f_S core (4x4x4, k1 + 4 k2 + 16 k3), scaled by dt nu: the expansion of
    // f_M [1 + A_s (q.v)(v^2 / (2 R_g T) - 5/2)] in the columns m_a v_a^k
    const double As = 2.0 * (1.0 - P.Pr) / (5.0 * P.m * n0 * RT * RT);
    const double sc = P.dt * nu;
    for (int o = 0; o < 64; ++o) s_fs[o] = 0.0;
    s_fs[0] = sc;
    for (int a = 0; a < 3; ++a) {
      const double qa = M[5 + a];
      const int st = (a == 0) ? 1 : (a == 1 ? 4 : 16);
      s_fs[1 * st] += sc * -2.5 * As * qa;
      s_fs[3 * st] += sc * As * beta * qa;
      for (int b2 = 0; b2 < 3; ++b2) {
        if (b2 == a) continue;
        const int sb2 = (b2 == 0) ? 1 : (b2 == 1 ? 4 : 16);
        s_fs[1 * st + 2 * sb2] += sc * As * beta * qa;
      }
    }
  }
  __syncthreads();

  // ---- 1. concatenated factors ---------------------------------------------
  for (int o = tid; o < 3 * RM * N; o += NT) {
    const int a = o / (RM * N), rem = o % (RM * N), col = rem / N, i = rem % N;
    if (col >= s_r0[a]) continue;
    const int src = s_src[a][col], k = s_k[a][col];
    double v;
    if (src <= 1) {
      v = d.fac[((size_t)c * 3 + a) * CS * N + k * N + i];
      if (src == 1) v *= s_d[a][i];
    } else if (src == 2) {
      const double w = s_fv[a][i];
      v = s_fb[a][i];
      for (int p = 0; p < k; ++p) v *= w;
    } else {
      const RSide& e = s_side[src - 3];
      const double x = P.xi_min + i * P.dxi;
      if (e.type == 0) {
        const int is = (a == e.rev) ? (N - 1 - i) : i;
        v = d.fac[((size_t)e.idx * 3 + a) * CS * N + k * N + is];
      } else {
        v = d.bc_fac[((size_t)e.idx * 3 + a) * N + i];
      }
      if (a == e.sax) v *= e.coef * fmax(-e.sig * x, 0.0);
    }
    sU[o] = v;
  }
  __syncthreads();

  // ---- 2. Gram-Schmidt (CGS2 with dropping), wave a handles mode a ---------
  {
    const int wave = tid >> 6, lane = tid & 63;
    const int a = wave < 3 ? wave : 0;
    const bool act = wave < 3;
    double* Ua = sU + a * RM * N;
    double* Ra = sR + a * RM * RM;
    int m = 0;
    const int r0 = s_r0[a];
    const int jmax = max(s_r0[0], max(s_r0[1], s_r0[2]));
    for (int j = 0; j < jmax; ++j) {
      const bool colj = act && j < r0;
      // (i) coefficients against the current basis and the column norm
      double un = 0.0;
      if (colj) {
        if (lane < m) {
          double s = 0.0;
          for (int i = 0; i < N; ++i) s += Ua[lane * N + i] * Ua[j * N + i];
          s_c1[a][lane] = s;
        }
        const double uj = lane < N ? Ua[j * N + lane] : 0.0;
        un = sqrt(wsum(uj * uj));
      }
      __syncthreads();
      double vl = 0.0;
      if (colj && lane < N) {
        double v = Ua[j * N + lane];
        for (int k = 0; k < m; ++k) v -= Ua[k * N + lane] * s_c1[a][k];
        vl = v;
        Ua[j * N + lane] = v;
      }
      __syncthreads();
      // (ii) re-orthogonalisation
      if (colj && lane < m) {
        double s = 0.0;
        for (int i = 0; i < N; ++i) s += Ua[lane * N + i] * Ua[j * N + i];
        s_c2[a][lane] = s;
      }
      __syncthreads();
      if (colj) {
        if (lane < N)
          for (int k = 0; k < m; ++k) vl -= Ua[k * N + lane] * s_c2[a][k];
        const double vn = sqrt(wsum(vl * vl));
        const bool keep = (vn > kQrDrop * un) && (m < N) && (m < RM);
        // R column j: coordinates in the basis, rows beyond it zero
        if (lane < RM) {
          double rv = 0.0;
          if (lane < m) rv = s_c1[a][lane] + s_c2[a][lane];
          else if (lane == m && keep) rv = vn;
          Ra[j * RM + lane] = rv;
        }
        if (keep) {
          if (lane < N) Ua[m * N + lane] = vl / vn;
          ++m;
        }
      }
      __syncthreads();
    }
    if (act && lane == 0) s_m[a] = m;
  }
  __syncthreads();
  const int m1 = s_m[0], m2 = s_m[1], m3 = s_m[2];
  if (m1 * m2 * m3 > GM || m1 * m2 * m3 == 0) return false;

  // ---- 3. small core G' = sum_t G_t x_a R_a[:, cols_t] ----------------------
  const int mt = m1 * m2 * m3;
  for (int o = tid; o < mt; o += NT) sG[o] = 0.0;
  const int r1 = s_r[0], r2 = s_r[1], r3 = s_r[2];
  const double* R1 = sR;
  const double* R2 = sR + RM * RM;
  const double* R3 = sR + 2 * RM * RM;
  for (int t = 0; t < 5 + ns; ++t) {
    int q1, q2, q3, o1, o2, o3;
    __syncthreads();  // the previous term's core is no longer read
    if (t <= 3) {
      // own state: (1 - dt nu) f with columns [U], then d_a o_a f with the
      // scaled columns in mode a
      q1 = r1; q2 = r2; q3 = r3;
      o1 = (t == 1) ? r1 : 0;
      o2 = (t == 2) ? r2 : 0;
      o3 = (t == 3) ? r3 : 0;
      const double gs = (t == 0) ? 1.0 - P.dt * nu : 1.0;
      for (int o = tid; o < q1 * q2 * q3; o += NT) {
        const int k1 = o % q1, tt = o / q1, k2 = tt % q2, k3 = tt / q2;
        sC[o] = gs * d.core[(size_t)c * CS * CS * CS + k1 + CS * (k2 + CS * k3)];
      }
    } else if (t == 4) {
      q1 = q2 = q3 = 4;
      o1 = 2 * r1; o2 = 2 * r2; o3 = 2 * r3;
      for (int o = tid; o < 64; o += NT) sC[o] = s_fs[o];
    } else {
      const RSide& e = s_side[t - 5];
      q1 = e.q[0]; q2 = e.q[1]; q3 = e.q[2];
      o1 = e.off[0]; o2 = e.off[1]; o3 = e.off[2];
      if (e.type == 0) {
        for (int o = tid; o < q1 * q2 * q3; o += NT) {
          const int k1 = o % q1, tt = o / q1, k2 = tt % q2, k3 = tt / q2;
          sC[o] = d.core[(size_t)e.idx * CS * CS * CS + k1 + CS * (k2 + CS * k3)];
        }
      } else if (tid == 0) {
        sC[0] = e.gsc;
      }
    }
    __syncthreads();
    for (int p = tid; p < m2 * m3; p += NT) {
      const int i2 = p % m2, i3 = p / m2;
      double z[QM];
#pragma unroll
      for (int k1 = 0; k1 < QM; ++k1) z[k1] = 0.0;
      for (int k3 = 0; k3 < q3; ++k3) {
        const double w3 = R3[(o3 + k3) * RM + i3];
        for (int k2 = 0; k2 < q2; ++k2) {
          const double w23 = w3 * R2[(o2 + k2) * RM + i2];
          const double* g = sC + q1 * (k2 + q2 * k3);
#pragma unroll
          for (int k1 = 0; k1 < QM; ++k1)
            if (k1 < q1) z[k1] += g[k1] * w23;
        }
      }
      double* gp = sG + m1 * p;
      for (int i1 = 0; i1 < m1; ++i1) {
        double s = gp[i1];
#pragma unroll
        for (int k1 = 0; k1 < QM; ++k1)
          if (k1 < q1) s += R1[(o1 + k1) * RM + i1] * z[k1];
        gp[i1] = s;
      }
    }
  }
  __syncthreads();

  // ---- 4. per mode: two Jacobi passes, G' rotated by both ------------------
  const int mm[3] = {m1, m2, m3};
  const int st[3] = {1, m1, m1 * m2};
  for (int a = 0; a < 3; ++a) {
    const int ma = mm[a];
    const int na = ma + (ma & 1);
    const int b = (a == 0) ? 1 : 0, cc = (a == 2) ? 1 : 2;  // the other two modes
    const int mb = mm[b], mc = mm[cc], sb = st[b], sc2 = st[cc], sa = st[a];
    double* Va = sR + a * RM * RM;  // V_a(p, k) at Va[k * RM + p]
    for (int pass = 0; pass < 2; ++pass) {
      // Gram of the mode-a unfolding of (the rotated) G'
      for (int o = tid; o < na * na; o += NT) {
        const int p = o / na, q = o % na;
        if (q < p) continue;
        double s = 0.0;
        if (p < ma && q < ma) {
          for (int jc = 0; jc < mc; ++jc)
            for (int jb = 0; jb < mb; ++jb) {
              const int e0 = jb * sb + jc * sc2;
              s += sG[e0 + p * sa] * sG[e0 + q * sa];
            }
        }
        sA[p * LDA + q] = s;
        sA[q * LDA + p] = s;
        sV[p * LDA + q] = (p == q) ? 1.0 : 0.0;
        sV[q * LDA + p] = (p == q) ? 1.0 : 0.0;
      }
      __syncthreads();
      if (tid < 64) {
        const double v = tid < ma ? sA[tid * LDA + tid] : 0.0;
        const double tr = wsum(v);
        if (tid == 0) s_tr = tr;
      }
      __syncthreads();
      const double tr = s_tr;
      const double thr = P.tol * P.tol * tr / 3.0;
      const double abs_thr = thr > 0.0 ? fmin(1e-18 * fabs(tr), 1e-4 * thr) : 1e-18 * fabs(tr);
      jacobi<NT, RM / 2>(sA, LDA, sV, LDA, na, na, 1e-15, abs_thr, s_cs, s_sn, s_tt, s_pp, s_qq, s_flag, &s_conv,
                         sweeps);
      // rotate G' in mode a: G'(.., p, ..) <- sum_q V(q, p) G'(.., q, ..)
      for (int f = tid; f < mb * mc; f += NT) {
        const int jb = f % mb, jc = f / mb;
        double* g = sG + jb * sb + jc * sc2;
        double x[RM];
#pragma unroll
        for (int q = 0; q < RM; ++q) x[q] = (q < ma) ? g[q * sa] : 0.0;
        for (int p = 0; p < ma; ++p) {
          double s = 0.0;
#pragma unroll
          for (int q = 0; q < RM; ++q)
            if (q < ma) s += sV[q * LDA + p] * x[q];
          g[p * sa] = s;
        }
      }
      if (pass == 0) {
        for (int o = tid; o < ma * ma; o += NT) {
          const int p = o % ma, k = o / ma;
          Va[k * RM + p] = sV[p * LDA + k];
        }
      } else {
        // eigenvalues of the second pass; V_a <- V_a (first pass) x V (second)
        if (tid < ma) s_lam[a][tid] = sA[tid * LDA + tid];
        __syncthreads();
        for (int o = tid; o < ma * ma; o += NT) {
          const int p = o % ma, k = o / ma;
          double s = 0.0;
          for (int q = 0; q < ma; ++q) s += Va[q * RM + p] * sV[q * LDA + k];
          sA[p * LDA + k] = s;
        }
        __syncthreads();
        for (int o = tid; o < ma * ma; o += NT) {
          const int p = o % ma, k = o / ma;
          Va[k * RM + p] = sA[p * LDA + k];
        }
      }
      __syncthreads();
    }
    // rank of mode a from the second pass's eigenvalues
    sort_desc<NT>(&s_lam[a][0], 1, ma, &s_order[a][0]);
    if (tid == 0) {
      double tr = 0.0;
      for (int p = 0; p < ma; ++p) tr += s_lam[a][p];
      const double thr = P.tol * P.tol * tr / 3.0;
      s_nr[a] = choose_rank(&s_lam[a][0], 1, &s_order[a][0], ma, 0.0, thr, 0.0, P.cap);
    }
    __syncthreads();
  }

  // ---- 5. factors Q_a V_a[:, kept] with canonical signs, core --------------
  for (int a = 0; a < 3; ++a) {
    const int ma = mm[a], ra = s_nr[a];
    const double* Qa = sU + a * RM * N;
    const double* Va = sR + a * RM * RM;
    // W(i, k) at sA[k * N + i]
    for (int o = tid; o < ra * N; o += NT) {
      const int k = o / N, i = o % N;
      const int j = s_order[a][k];
      double s = 0.0;
      for (int p = 0; p < ma; ++p) s += Qa[p * N + i] * Va[j * RM + p];
      sA[o] = s;
    }
    __syncthreads();
    if (tid < ra) {
      double best = -1.0;
      int bi = 0;
      for (int i = 0; i < N; ++i) {
        const double v = fabs(sA[tid * N + i]);
        if (v > best) { best = v; bi = i; }
      }
      s_sign[a][tid] = (sA[tid * N + bi] < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    double* out = d.fac_n + ((size_t)c * 3 + a) * CS * N;
    for (int o = tid; o < ra * N; o += NT) out[o] = s_sign[a][o / N] * sA[o];
    __syncthreads();
  }
  const int n1 = s_nr[0], n2 = s_nr[1], n3 = s_nr[2];
  for (int o = tid; o < n1 * n2 * n3; o += NT) {
    const int k1 = o % n1, tt = o / n1, k2 = tt % n2, k3 = tt / n2;
    const int e = s_order[0][k1] + m1 * (s_order[1][k2] + m2 * s_order[2][k3]);
    d.core_n[(size_t)c * CS * CS * CS + k1 + CS * (k2 + CS * k3)] =
        s_sign[0][k1] * s_sign[1][k2] * s_sign[2][k3] * sG[e];
  }
  if (tid < 3) d.rank_n[3 * c + tid] = s_nr[tid];
  __syncthreads();
  return true;
}

// One launch of a tier: cells 0..nc-1 (list == nullptr, one workgroup per
// cell) or the cells of `list` (grid-stride over *list_n).  Cells the tier
// cannot take are appended to next; cells it rounds lose their N-basis warm
// start (wvalid[3 c + a] = 0: the kept eigenbasis of the N-basis path
// predates this step).
template <int N, int RM, int GM, int QM>
__global__ __launch_bounds__(kRThreads) void k_rround(DevState d, const int* list, const int* list_n, int* next,
                                                      int* next_n, int* wvalid, unsigned long long* stats) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* smem = reinterpret_cast<double*>(smem_raw);
  const int n = list ? *list_n : d.n_cells;
  for (int b = blockIdx.x; b < n; b += gridDim.x) {
    const int c = list ? list[b] : b;
    const bool done = rround_cell<N, RM, GM, QM>(d, c, smem, stats ? stats + 2 : nullptr);
    if (threadIdx.x == 0) {
      if (done) {
        if (wvalid) wvalid[3 * c] = wvalid[3 * c + 1] = wvalid[3 * c + 2] = 0;
        if (stats) atomicAdd(stats, 1ull);
      } else {
        next[atomicAdd(next_n, 1)] = c;
      }
    }
    __syncthreads();
  }
}

__global__ void k_rround_zero(int* a, int* b) {
  *a = 0;
  *b = 0;
}

// tiers: rank-1 neighbourhoods (r0 <= 12), then r0 <= 24 with source ranks <= 8
template <int N>
hipError_t launch_rround_t(const DevState& d, int* listM, int* nM, int* listD, int* nD, int* wvalid,
                           unsigned long long* stats, hipStream_t s) {
  auto kS = k_rround<N, 12, 12 * 12 * 12, 4>;
  auto kM = k_rround<N, 24, 4096, 8>;
  const size_t shS = rround_lds_bytes<N, 12, 12 * 12 * 12, 4>();
  const size_t shM = rround_lds_bytes<N, 24, 4096, 8>();
  hipError_t e = hipFuncSetAttribute((const void*)kS, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shS);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)kM, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shM);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rround_zero, dim3(1), dim3(1), 0, s, nM, nD);
  hipLaunchKernelGGL(kS, dim3(d.n_cells), dim3(kRThreads), shS, s, d, (const int*)nullptr, (const int*)nullptr, listM,
                     nM, wvalid, stats);
  const int gM = d.n_cells < 1024 ? d.n_cells : 1024;
  hipLaunchKernelGGL(kM, dim3(gM), dim3(kRThreads), shM, s, d, (const int*)listM, (const int*)nM, listD, nD, wvalid,
                     stats ? stats + 4 : nullptr);
  return hipGetLastError();
}

__global__ void k_fill_int(int* p, size_t n, int v) {
  const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o < n) p[o] = v;
}

}  // namespace

hipError_t launch_fill_int(int* p, size_t n, int v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_rround(const DevState& d, int* listM, int* nM, int* listD, int* nD, int* wvalid,
                         unsigned long long* stats, hipStream_t s) {
  if (d.n_cells <= 0) return hipSuccess;
  switch (d.N) {
    case 16: return launch_rround_t<16>(d, listM, nM, listD, nD, wvalid, stats, s);
    case 24: return launch_rround_t<24>(d, listM, nM, listD, nD, wvalid, stats, s);
    case 32: return launch_rround_t<32>(d, listM, nM, listD, nD, wvalid, stats, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace tk
