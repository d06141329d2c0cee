// Rounding in the space of the concatenated factors (Op4 as the paper
// describes Tucker rounding: QR of the factors, the core multiplied by the
// R factors, SVDs of the small core's unfoldings), fused with the term
// assembly of one explicit step, one workgroup of four wavefronts per cell.
//
// The update f* = f + dt R of a cell on axis-aligned faces is a sum of
// Tucker terms (eq. exact-flux in gather form, Alg. 1, the flux part; Op2 sums,
// Op3 products with rank-1 row scalings):
//
//   f* = (1 - dt nu) f + sum_a d_a o_a f + dt nu f_S + sum_l b_l o_{a_l} g_l,
//   d_a(i) = -sum_{l on axis a} (dt A_l / V) max(s_l xi_i, 0),
//   b_l(i) = (dt A_l / V) max(-s_l xi_i, 0),
//
// where o_a scales the rows of mode a, f_S is the rank-4 S-model
// equilibrium (Alg. 2, Proposition 1) and g_l the far side of
// face l (neighbour state or boundary ghost).  Per mode a the factor of the
// sum is the concatenation Ucat_a = [U_a, d_a U_a, F_a, far sides] with
// r0_a = 2 r_a + 4 + sum_l q_l,a columns; its core is block-sparse.
//
// Steps per cell:
//  1. Face records by one lane per slot; column tables, 1-D tables (d_a,
//     the f_S columns m_a (xi - u_a)^k) and the term cores staged in LDS.
//  2. Wavefront a loads the columns of Ucat_a (row i in lane i, with the row
//     scaling of each far side and, for a symmetry ghost, the reversed
//     velocity index) and factors Ucat_a = Q_a R_a by classical
//     Gram-Schmidt with one re-orthogonalisation, sums over the rows by DPP
//     wave reductions.  A column whose component outside the span of the
//     previous ones is at most 1e-13 of its norm adds no basis vector (its R
//     column still holds its coordinates): m_a <= r0_a vectors remain, and
//     the tensor changes by at most that fraction of each term.
//  3. The small core G' = sum_t G_t x_1 R_1[:, cols] x_2 R_2[:, cols]
//     x_3 R_3[:, cols] (m_1 x m_2 x m_3) in LDS, each thread owning mode-1
//     fibres.  The update is G' x_a Q_a, and its mode-a singular values
//     are those of G'_(a).
//  4. Wavefront a forms the Gram G'_(a) G'_(a)^T (FP64; its sums are short,
//     m_b m_c products, which keeps the small kept directions accurate to
//     the FP64 parity bar in one pass) and diagonalises it by Jacobi; the
//     rank rule of the truncated HOSVD (T-HOSVD, modes independent) is
//     applied to its eigenvalues.
//  5. G' is rotated by the eigenvectors in every mode; the factors are
//     Q_a V_a[:, kept] with the canonical sign (largest-magnitude entry
//     positive, the first on ties), the core is the kept block.
//
// FP64 throughout on both precision paths (on this device FP64 and FP32
// vector arithmetic without packed instructions retire at the same rate).
// The layout takes cells whose own state and far sides all have rank 1
// (r0_a <= 12); a cell with a higher rank around it, an oblique face, or a
// core above the layout's capacity is appended to `next` for the N-basis
// path.
#include "tk_internal.h"
#include "tk_jacobi.h"

namespace tk {

namespace {

constexpr int kRThreads = 256;
constexpr double kQrDrop = 1e-13;  // Gram-Schmidt: relative norm below which a column adds no vector


template <int N, int RM, int GM, int SC>
struct RLds {
  static constexpr int LDU = N + 1;                       // column stride of Ucat / Q (odd: no bank conflicts)
  static constexpr int LDA = RM + 1;                      // Jacobi matrices
  static constexpr int U = 3 * RM * LDU;                  // Ucat, then Q
  static constexpr int R0 = 3 * RM * RM;                  // R (until the core is assembled)
  static constexpr int AV = 6 * RM * LDA;                 // per mode: Gram A_a, eigenvectors V_a
  static constexpr int R = R0 > AV ? R0 : AV;             // R, then A/V
  static constexpr int G = GM;                            // core G'
  static constexpr int C = SC;                            // staged term cores
  static constexpr int total = U + R + G + C;
};

template <int N, int RM, int GM, int QM, int SC>
constexpr size_t rround_lds_bytes() {
  return sizeof(double) * RLds<N, RM, GM, SC>::total;
}

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double mt_of(const int (&mm)[3]) { return (double)mm[0] * mm[1] * mm[2]; }

// far side of one face slot, as read by its lane
struct RSlot {
  int kind, axis, nb, q[3];
  double coef, sig, gsc;
};

// One cell; returns false (uniformly) when the cell is left to the next tier.
// *flops (thread 0) receives the cell's FP64 operation count: 2 per
// multiply-add of the Gram-Schmidt passes, core assembly, Grams, Jacobi
// sweeps (10 n per rotation of an n x n matrix, both sides and the vectors),
// rotations and output products; index arithmetic and tables not counted.
// Layout of the core G' in LDS: entry (i1, i2, i3) at i1 + L1 (i2 + L2 i3)
// with L1, L2 the first two sizes rounded up to odd numbers, so that the
// mode-wise Gram reads of one wave fall on different banks.
template <int N, int RM, int GM, int QM, int SC>
__device__ bool rround_cell(const DevState& d, int c, double* smem, unsigned long long* sweeps, double* flops) {
  using L = RLds<N, RM, GM, SC>;
  constexpr int NT = kRThreads;
  constexpr int LDU = L::LDU, LDA = L::LDA;
  double* sU = smem;
  double* sR = sU + L::U;
  double* sG = sR + L::R;
  double* sC = sG + L::G;
  __shared__ RSlot s_slot[kSlots];
  __shared__ int s_ns, s_ok, s_r[3], s_r0[3], s_m[3], s_nr[3];
  __shared__ int s_side[kSlots], s_off[kSlots][3], s_coff[2 + kSlots];  // used slots, column offsets, core offsets
  __shared__ signed char s_src[3][RM], s_k[3][RM];  // column source (0 own, 1 own scaled, 2 f_S, 3+s far side s) and index
  __shared__ double s_d[3][N], s_fb[3][N], s_fv[3][N];  // d_a, f_S base and xi - u_a
  __shared__ double s_c1[3][RM], s_c2[3][RM];
  __shared__ double s_lam[3][RM];
  __shared__ int s_order[3][RM];
  __shared__ double s_sign[3][kMaxCap];
  __shared__ double s_cs[3][RM / 2], s_sn[3][RM / 2], s_tt[3][RM / 2];
  __shared__ int s_pp[3][RM / 2], s_qq[3][RM / 2];
  __shared__ unsigned char s_bi[3][(RM / 2) * (RM / 2 + 1) / 2], s_bj[3][(RM / 2) * (RM / 2 + 1) / 2];
  __shared__ double s_fl[4];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int CS = d.CS;
  const InstParams P = d.ip[d.inst[c]];
  const double nu = d.nu[c];

  // ---- face records (one lane per slot), then sources and columns --------
  if (tid < kSlots) {
    const size_t sl = (size_t)kSlots * c + tid;
    RSlot e;
    e.kind = d.slot_kind[sl];
    e.axis = d.slot_axis[sl];
    e.nb = d.slot_nb[sl];
    e.coef = d.slot_coef[sl];
    e.sig = (double)d.slot_sig[sl];
    e.gsc = 1.0;
    e.q[0] = e.q[1] = e.q[2] = 1;
    if (e.kind == SK_INTERIOR || e.kind == SK_OUTFLOW || e.kind == SK_SYM) {
      const int src = (e.kind == SK_INTERIOR) ? e.nb : c;
      for (int a = 0; a < 3; ++a) e.q[a] = d.rank[3 * src + a];
    } else if (e.kind == SK_WALL) {
      e.gsc = d.nw[sl];
    }
    s_slot[tid] = e;
  } else if (tid == 64) {
    for (int a = 0; a < 3; ++a) s_r[a] = d.rank[3 * c + a];
  }
  __syncthreads();
  if (tid == 0) {
    int ok = 1, ns = 0, off[3];
    for (int a = 0; a < 3; ++a) {
      off[a] = 2 * s_r[a] + 4;
      ok &= (s_r[a] <= QM) ? 1 : 0;
    }
    int coff = s_r[0] * s_r[1] * s_r[2];  // staged cores: own, f_S, far sides
    s_coff[0] = 0;
    s_coff[1] = coff;
    coff += 64;
    for (int l = 0; l < kSlots; ++l) {
      const RSlot& e = s_slot[l];
      if (e.kind == SK_NONE) continue;
      if (e.axis < 0) ok = 0;
      for (int a = 0; a < 3; ++a) {
        ok &= (e.q[a] <= QM) ? 1 : 0;
        s_off[ns][a] = off[a];
        off[a] += e.q[a];
      }
      s_coff[2 + ns] = coff;
      coff += e.q[0] * e.q[1] * e.q[2];
      s_side[ns++] = l;
    }
    for (int a = 0; a < 3; ++a) ok &= (off[a] <= RM) ? 1 : 0;
    ok &= (coff <= SC) ? 1 : 0;
    if (ok) {
      for (int a = 0; a < 3; ++a) {
        s_r0[a] = off[a];
        int col = 0;
        for (int k = 0; k < s_r[a]; ++k) { s_src[a][col] = 0; s_k[a][col++] = (signed char)k; }
        for (int k = 0; k < s_r[a]; ++k) { s_src[a][col] = 1; s_k[a][col++] = (signed char)k; }
        for (int k = 0; k < 4; ++k) { s_src[a][col] = 2; s_k[a][col++] = (signed char)k; }
        for (int t = 0; t < ns; ++t)
          for (int k = 0; k < s_slot[s_side[t]].q[a]; ++k) {
            s_src[a][col] = (signed char)(3 + t);
            s_k[a][col++] = (signed char)k;
          }
      }
    }
    s_ns = ns;
    s_ok = ok;
  }
  __syncthreads();
  if (!s_ok) return false;
  const int ns = s_ns;
  const int r1 = s_r[0], r2 = s_r[1], r3 = s_r[2];

  // ---- 1-D tables (d_a, f_S columns), f_S core and the staged term cores --
  const double* M = d.macro + 8 * (size_t)c;
  const double n0 = M[0], T0 = M[4];
  const double RT = P.Rg * T0;
  const double beta = 1.0 / (2.0 * RT);
  for (int o = tid; o < 3 * N; o += NT) {
    const int a = o / N, i = o % N;
    const double x = P.xi_min + i * P.dxi;
    double s = 0.0;
    for (int l = 0; l < kSlots; ++l) {
      const RSlot& e = s_slot[l];
      if (e.kind == SK_NONE || e.axis != a) continue;
      s -= e.coef * fmax(e.sig * x, 0.0);
    }
    s_d[a][i] = s;
    const double v = x - M[1 + a];
    s_fv[a][i] = v;
    s_fb[a][i] = cbrt(n0) / sqrt(2.0 * M_PI * RT) * exp(-v * v * beta);
  }
  {
    // own core (unscaled), then the far sides' cores (scaled by the wall
    // density where the far side is a wall)
    const int no = r1 * r2 * r3;
    for (int o = tid; o < no; o += NT) {
      const int k1 = o % r1, tt = o / r1, k2 = tt % r2, k3 = tt / r2;
      sC[o] = d.core[(size_t)c * CS * CS * CS + k1 + CS * (k2 + CS * k3)];
    }
    for (int t = 0; t < ns; ++t) {
      const RSlot& e = s_slot[s_side[t]];
      double* dst = sC + s_coff[2 + t];
      if (e.kind == SK_INTERIOR || e.kind == SK_OUTFLOW || e.kind == SK_SYM) {
        const int src = (e.kind == SK_INTERIOR) ? e.nb : c;
        const int q1 = e.q[0], q2 = e.q[1], nq = e.q[0] * e.q[1] * e.q[2];
        for (int o = tid; o < nq; o += NT) {
          const int k1 = o % q1, tt = o / q1, k2 = tt % q2, k3 = tt / q2;
          dst[o] = d.core[(size_t)src * CS * CS * CS + k1 + CS * (k2 + CS * k3)];
        }
      } else if (tid == 0) {
        dst[0] = e.gsc;
      }
    }
    if (tid == 64) {
      // f_S core (4x4x4, k1 + 4 k2 + 16 k3), scaled by dt nu: the expansion of
      // f_M [1 + A_s (q.v)(v^2 / (2 R_g T) - 5/2)] in the columns m_a v_a^k
      double* fs = sC + s_coff[1];
      const double As = 2.0 * (1.0 - P.Pr) / (5.0 * P.m * n0 * RT * RT);
      const double sc = P.dt * nu;
      for (int o = 0; o < 64; ++o) fs[o] = 0.0;
      fs[0] = sc;
      for (int a = 0; a < 3; ++a) {
        const double qa = M[5 + a];
        const int st = (a == 0) ? 1 : (a == 1 ? 4 : 16);
        fs[1 * st] += sc * -2.5 * As * qa;
        fs[3 * st] += sc * As * beta * qa;
        for (int b2 = 0; b2 < 3; ++b2) {
          if (b2 == a) continue;
          const int sb2 = (b2 == 0) ? 1 : (b2 == 1 ? 4 : 16);
          fs[1 * st + 2 * sb2] += sc * As * beta * qa;
        }
      }
    }
  }
  __syncthreads();

  // ---- 1-2. concatenated factors and their Gram-Schmidt QR, wave a on mode a:
  // lane i holds row i of Ucat_a in registers (the kept basis vectors are
  // compacted into the leading slots), classical Gram-Schmidt with one
  // re-orthogonalisation, sums across the rows by DPP wave reductions
  static_assert(RM <= 12, "the register Gram-Schmidt holds at most 12 columns per lane");
  if (wave < 3) {
    const int a = wave;
    const int r0 = s_r0[a];
    const int i = lane < N ? lane : N - 1;
    const bool row = lane < N;
    const double x = P.xi_min + i * P.dxi;
    double U[RM];
#pragma unroll
    for (int col = 0; col < RM; ++col) {
      double v = 0.0;
      if (col < r0 && row) {
        const int src = s_src[a][col], k = s_k[a][col];
        if (src <= 1) {
          v = d.fac[((size_t)c * 3 + a) * CS * N + k * N + i];
          if (src == 1) v *= s_d[a][i];
        } else if (src == 2) {
          const double w = s_fv[a][i];
          v = s_fb[a][i];
          for (int p = 0; p < k; ++p) v *= w;
        } else {
          const RSlot& e = s_slot[s_side[src - 3]];
          if (e.kind == SK_INTERIOR || e.kind == SK_OUTFLOW || e.kind == SK_SYM) {
            const int srcc = (e.kind == SK_INTERIOR) ? e.nb : c;
            const int is = (e.kind == SK_SYM && a == e.axis) ? (N - 1 - i) : i;
            v = d.fac[((size_t)srcc * 3 + a) * CS * N + k * N + is];
          } else {
            v = d.bc_fac[((size_t)e.nb * 3 + a) * N + i];
          }
          if (a == e.axis) v *= e.coef * fmax(-e.sig * x, 0.0);
        }
      }
      U[col] = v;
    }
    double* Ra = sR + a * RM * RM;
    int m = 0;
    double qrf = 0.0;
    for (int j = 0; j < r0; ++j) {
      double u = 0.0;
#pragma unroll
      for (int k = 0; k < RM; ++k)
        if (k == j) u = U[k];
      const double un = sqrt(wave_sum_dpp(u * u));
      double c1[RM], c2[RM];
      double v = u;
#pragma unroll
      for (int k = 0; k < RM; ++k) {
        c1[k] = 0.0;
        if (k < m) c1[k] = wave_sum_dpp(U[k] * u);
      }
#pragma unroll
      for (int k = 0; k < RM; ++k)
        if (k < m) v -= U[k] * c1[k];
#pragma unroll
      for (int k = 0; k < RM; ++k) {
        c2[k] = 0.0;
        if (k < m) c2[k] = wave_sum_dpp(U[k] * v);
      }
#pragma unroll
      for (int k = 0; k < RM; ++k)
        if (k < m) v -= U[k] * c2[k];
      if (!row) v = 0.0;
      const double vn = sqrt(wave_sum_dpp(v * v));
      qrf += 8.0 * m * N + 4.0 * N;
      const bool keep = (vn > kQrDrop * un) && (m < N) && (m < RM);
      // R column j: coordinates in the basis, rows beyond it zero
      double rv = 0.0;
#pragma unroll
      for (int k = 0; k < RM; ++k) {
        if (lane == k && k < m) rv = c1[k] + c2[k];
        if (lane == k && k == m && keep) rv = vn;
      }
      if (lane < RM) Ra[j * RM + lane] = rv;
      if (keep) {
        const double q = v / vn;
#pragma unroll
        for (int k = 0; k < RM; ++k)
          if (k == m) U[k] = q;
        ++m;
      }
    }
    // the basis into LDS for the output factors
    double* Ua = sU + a * RM * LDU;
#pragma unroll
    for (int k = 0; k < RM; ++k)
      if (k < m && row) Ua[k * LDU + lane] = U[k];
    if (lane == 0) {
      s_m[a] = m;
      s_fl[a] = qrf;
    }
  }
  __syncthreads();
  const int m1 = s_m[0], m2 = s_m[1], m3 = s_m[2];
  const int L1 = m1 | 1, L2 = m2 | 1;
  const int gsize = L1 * L2 * m3;
  if (gsize > GM || m1 * m2 * m3 == 0) return false;

  // ---- 3. small core G' = sum_t G_t x_a R_a[:, cols_t] ----------------------
  double fl = s_fl[0] + s_fl[1] + s_fl[2];
  const double* R1 = sR;
  const double* R2 = sR + RM * RM;
  const double* R3 = sR + 2 * RM * RM;
  for (int p = tid; p < m2 * m3; p += NT) {
    const int i2 = p % m2, i3 = p / m2;
    double acc[RM];
#pragma unroll
    for (int i1 = 0; i1 < RM; ++i1) acc[i1] = 0.0;
    for (int t = 0; t < 5 + ns; ++t) {
      int q1, q2, q3, o1, o2, o3;
      const double* g;
      double gs = 1.0;
      if (t <= 3) {
        // own state: (1 - dt nu) f with columns [U], then d_a o_a f with the
        // scaled columns in mode a
        q1 = r1; q2 = r2; q3 = r3;
        o1 = (t == 1) ? r1 : 0;
        o2 = (t == 2) ? r2 : 0;
        o3 = (t == 3) ? r3 : 0;
        g = sC;
        if (t == 0) gs = 1.0 - P.dt * nu;
      } else if (t == 4) {
        q1 = q2 = q3 = 4;
        o1 = 2 * r1; o2 = 2 * r2; o3 = 2 * r3;
        g = sC + s_coff[1];
      } else {
        const RSlot& e = s_slot[s_side[t - 5]];
        q1 = e.q[0]; q2 = e.q[1]; q3 = e.q[2];
        o1 = s_off[t - 5][0]; o2 = s_off[t - 5][1]; o3 = s_off[t - 5][2];
        g = sC + s_coff[2 + t - 5];
      }
      double z[QM];
#pragma unroll
      for (int k1 = 0; k1 < QM; ++k1) z[k1] = 0.0;
      for (int k3 = 0; k3 < q3; ++k3) {
        const double w3 = R3[(o3 + k3) * RM + i3];
        for (int k2 = 0; k2 < q2; ++k2) {
          const double w23 = w3 * R2[(o2 + k2) * RM + i2];
          const double* gk = g + q1 * (k2 + q2 * k3);
#pragma unroll
          for (int k1 = 0; k1 < QM; ++k1)
            if (k1 < q1) z[k1] += gk[k1] * w23;
        }
      }
#pragma unroll
      for (int k1 = 0; k1 < QM; ++k1)
        if (k1 < q1) z[k1] *= gs;
#pragma unroll
      for (int i1 = 0; i1 < RM; ++i1) {
        if (i1 < m1) {
          double s = acc[i1];
#pragma unroll
          for (int k1 = 0; k1 < QM; ++k1)
            if (k1 < q1) s += R1[(o1 + k1) * RM + i1] * z[k1];
          acc[i1] = s;
        }
      }
    }
#pragma unroll
    for (int i1 = 0; i1 < RM; ++i1)
      if (i1 < m1) sG[i1 + L1 * (i2 + L2 * i3)] = acc[i1];
  }
  if (tid == 0) {
    for (int t = 0; t < 5 + ns; ++t) {
      int q1, q2, q3;
      if (t <= 3) { q1 = r1; q2 = r2; q3 = r3; }
      else if (t == 4) { q1 = q2 = q3 = 4; }
      else { const RSlot& e = s_slot[s_side[t - 5]]; q1 = e.q[0]; q2 = e.q[1]; q3 = e.q[2]; }
      fl += 2.0 * m2 * m3 * ((double)q1 * q2 * q3 + (double)q2 * q3 + (double)q1 + (double)m1 * q1);
    }
  }
  __syncthreads();

  // ---- 4. per mode on its own wave: Gram of the unfolding, Jacobi, rank -----
  const int mm[3] = {m1, m2, m3};
  const int st[3] = {1, L1, L1 * L2};
  if (wave < 3) {
    const int a = wave;
    const int ma = mm[a];
    const int na = ma + (ma & 1);
    const int b = (a == 0) ? 1 : 0, cc = (a == 2) ? 1 : 2;  // the other two modes
    const int mb = mm[b], mc = mm[cc], sb = st[b], sc2 = st[cc], sa = st[a];
    double* A = sR + a * 2 * RM * LDA;
    double* V = A + RM * LDA;
    for (int o = lane; o < na * na; o += 64) {
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
      A[p * LDA + q] = s;
      A[q * LDA + p] = s;
      V[p * LDA + q] = (p == q) ? 1.0 : 0.0;
      V[q * LDA + p] = (p == q) ? 1.0 : 0.0;
    }
    wave_sync();
    const double tr = wsum(lane < ma ? A[lane * LDA + lane] : 0.0);
    const double thr = P.tol * P.tol * tr / 3.0;
    const double abs_thr = thr > 0.0 ? fmin(1e-18 * fabs(tr), 1e-4 * thr) : 1e-18 * fabs(tr);
    const int nsw = jacobi_wave<RM / 2>(A, LDA, V, LDA, na, na, 1e-15, abs_thr, s_cs[a], s_sn[a], s_tt[a],
                                        s_pp[a], s_qq[a], s_bi[a], s_bj[a]);
    if (lane < ma) s_lam[a][lane] = A[lane * LDA + lane];
    wave_sync();
    sort_desc_wave(&s_lam[a][0], 1, ma, &s_order[a][0]);
    if (lane == 0) {
      double t2 = 0.0;
      for (int p = 0; p < ma; ++p) t2 += s_lam[a][p];
      s_nr[a] = choose_rank(&s_lam[a][0], 1, &s_order[a][0], ma, 0.0, P.tol * P.tol * t2 / 3.0, 0.0, P.cap);
      s_fl[a] = (double)(na + 1) * mt_of(mm) + 5.0 * nsw * na * (double)na * (na - 1) + 2.0 * ma * mt_of(mm);
      if (sweeps) atomicAdd(sweeps, (unsigned long long)nsw);
    }
  }
  __syncthreads();
  fl += s_fl[0] + s_fl[1] + s_fl[2];

  // ---- 5. core of the kept directions: G' rotated by V_a in every mode ------
  for (int a = 0; a < 3; ++a) {
    const int ma = mm[a];
    const int b = (a == 0) ? 1 : 0, cc = (a == 2) ? 1 : 2;
    const int mb = mm[b], mc = mm[cc], sb = st[b], sc2 = st[cc], sa = st[a];
    const double* V = sR + a * 2 * RM * LDA + RM * LDA;
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
          if (q < ma) s += V[q * LDA + p] * x[q];
        g[p * sa] = s;
      }
    }
    __syncthreads();
    fl += 2.0 * ma * (double)(m1 * m2 * m3);
  }
  // factors Q_a V_a[:, kept], each wave its mode, one column at a time: the
  // canonical sign makes the column's largest-magnitude entry (the first on
  // ties) positive
  if (wave < 3) {
    const int a = wave;
    const int ma = mm[a], ra = s_nr[a];
    const double* Qa = sU + a * RM * LDU;
    const double* V = sR + a * 2 * RM * LDA + RM * LDA;
    double* out = d.fac_n + ((size_t)c * 3 + a) * CS * N;
    for (int k = 0; k < ra; ++k) {
      const int j = s_order[a][k];
      double w = 0.0;
      if (lane < N)
        for (int p = 0; p < ma; ++p) w += Qa[p * LDU + lane] * V[p * LDA + j];
      double bv = lane < N ? fabs(w) : -1.0;
      int bi = lane;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      const double sg = (__shfl(w, bi, 64) < 0.0) ? -1.0 : 1.0;
      if (lane < N) out[k * N + lane] = sg * w;
      if (lane == 0) s_sign[a][k] = sg;
    }
    if (lane == 0) s_fl[a] = 2.0 * N * ma * ra;
  }
  __syncthreads();
  fl += s_fl[0] + s_fl[1] + s_fl[2];
  const int n1 = s_nr[0], n2 = s_nr[1], n3 = s_nr[2];
  for (int o = tid; o < n1 * n2 * n3; o += NT) {
    const int k1 = o % n1, tt = o / n1, k2 = tt % n2, k3 = tt / n2;
    d.core_n[(size_t)c * CS * CS * CS + k1 + CS * (k2 + CS * k3)] =
        s_sign[0][k1] * s_sign[1][k2] * s_sign[2][k3] *
        sG[s_order[0][k1] * st[0] + s_order[1][k2] * st[1] + s_order[2][k3] * st[2]];
  }
  if (tid < 3) d.rank_n[3 * c + tid] = s_nr[tid];
  if (tid == 0) *flops = fl;
  __syncthreads();
  return true;
}

// One launch of a tier: cells 0..nc-1 (list == nullptr, one workgroup per
// cell) or the cells of `list` (grid-stride over *list_n).  Cells the tier
// cannot take are appended to next; cells it rounds lose their N-basis warm
// start (wvalid[3 c + a] = 0: the kept eigenbasis of the N-basis path
// predates this step).
template <int N, int RM, int GM, int QM, int SC>
// Four workgroups per CU (at most 128 VGPRs, a few spilled): the per-cell
// chains of reductions and barriers are latency-bound, and a fourth
// workgroup hides more of that latency than the spills cost (14.3 against
// 15.8 ms per step over the channel run's first 180 steps).
__global__ __launch_bounds__(kRThreads, 4) void k_rround(DevState d, const int* list, const int* list_n, int* next,
                                                      int* next_n, int* wvalid, unsigned long long* stats) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* smem = reinterpret_cast<double*>(smem_raw);
  const int n = list ? *list_n : d.n_cells;
  for (int b = blockIdx.x; b < n; b += gridDim.x) {
    const int c = list ? list[b] : b;
    if (d.ip[d.inst[c]].frozen) continue;  // neither rounded nor listed
    double fl = 0.0;
    const bool done = rround_cell<N, RM, GM, QM, SC>(d, c, smem, stats ? stats + 2 : nullptr, &fl);
    if (threadIdx.x == 0) {
      if (done) {
        if (wvalid) wvalid[3 * c] = wvalid[3 * c + 1] = wvalid[3 * c + 2] = 0;
        if (stats) {
          atomicAdd(stats, 1ull);
          atomicAdd(stats + 1, (unsigned long long)fl);
        }
      } else {
        next[atomicAdd(next_n, 1)] = c;
      }
    }
    __syncthreads();
  }
}

__global__ void k_zero_count(int* a) { *a = 0; }

// Cells whose own state and far sides all have rank 1 (r0 <= 12 per mode): a
// 13 x 13 x 12 core layout and 128 staged core values (34 KB of LDS, four
// workgroups per CU).  The others are listed for the N-basis path.
template <int N>
hipError_t launch_rround_t(const DevState& d, int* listD, int* nD, int* wvalid, unsigned long long* stats,
                           hipStream_t s) {
  auto k = k_rround<N, 12, 13 * 13 * 12, 4, 128>;
  const size_t sh = rround_lds_bytes<N, 12, 13 * 13 * 12, 4, 128>();
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, nD);
  hipLaunchKernelGGL(k, dim3(d.n_cells), dim3(kRThreads), sh, s, d, (const int*)nullptr, (const int*)nullptr, listD,
                     nD, wvalid, stats);
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

hipError_t launch_rround(const DevState& d, int* listD, int* nD, int* wvalid, unsigned long long* stats,
                         hipStream_t s) {
  if (d.n_cells <= 0) return hipSuccess;
  switch (d.N) {
    case 16: return launch_rround_t<16>(d, listD, nD, wvalid, stats, s);
    case 24: return launch_rround_t<24>(d, listD, nD, wvalid, stats, s);
    case 32: return launch_rround_t<32>(d, listD, nD, wvalid, stats, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace tk
