"""Tucker-format algebra for 3-D tensors (oracle; test infrastructure only).

A Tucker tensor is A(i1,i2,i3) = sum_k G(k1,k2,k3) U1(i1,k1) U2(i2,k2) U3(i3,k3)
(Section "Tensor decompositions", Tucker format).  The operations are the
five the paper lists for the tensorised method:

  Op1 `hosvd`      full tensor -> Tucker with ||A-B||_F <= eps ||A||_F
                   (truncated higher-order SVD, de Lathauwer et al.)
  Op2 `add`        element-wise sum: block-diagonal core, concatenated
                   factors (eq. element_wise_sum)
  Op3 `hadamard`   element-wise product: Kronecker product of cores and of
                   factor rows
  Op4 `round`      recompression of a Tucker tensor: QR of the factors,
                   core times the R factors, SVDs of the core unfoldings
                   (Oseledets' Tucker rounding)
  Op5 `convolve`   sum_i A(i) w1(i1) w2(i2) w3(i3) via S_a = U_a^T w_a

plus Lemma 1 (`lemma1`: w1 + w2 + w3 has Tucker rank 2) and the exact
division by a rank-1 tensor (eq. one_rank_division).

Truncation rule (reading of the paper's "ranks determined by eps"):
independent per-mode SVDs (T-HOSVD); the rank of mode a is the smallest
r >= 1 whose discarded squared singular values sum to at most
eps^2 ||A||_F^2 / 3, then capped.  This guarantees the Frobenius bound of
Op1 when no cap applies.  Kept singular vectors are sign-canonicalised
(largest-magnitude entry positive, first such entry on ties).
"""

import numpy as np


class Tucker:
    __slots__ = ("G", "U")

    def __init__(self, G, U):
        self.G = np.asarray(G, dtype=np.float64)
        self.U = [np.asarray(u, dtype=np.float64) for u in U]
        if self.G.ndim != 3 or len(self.U) != 3:
            raise ValueError("3-D Tucker tensors only")
        for a in range(3):
            if self.U[a].ndim != 2 or self.U[a].shape[1] != self.G.shape[a]:
                raise ValueError("factor/core rank mismatch")

    @property
    def ranks(self):
        return tuple(self.G.shape)

    @property
    def shape(self):
        return tuple(u.shape[0] for u in self.U)

    def copy(self):
        return Tucker(self.G.copy(), [u.copy() for u in self.U])

    def scaled(self, s):
        return Tucker(self.G * s, [u.copy() for u in self.U])


def mode_product(A, M, mode):
    """(A x_mode M)[.., i, ..] = sum_k M[i, k] A[.., k, ..]."""
    return np.moveaxis(np.tensordot(M, A, axes=(1, mode)), 0, mode)


def unfold(A, mode):
    return np.moveaxis(A, mode, 0).reshape(A.shape[mode], -1)


def full(t):
    """Expand a Tucker tensor to its N1 x N2 x N3 array."""
    A = t.G
    for a in range(3):
        A = mode_product(A, t.U[a], a)
    return A


def choose_rank(sig2, total, eps, cap):
    """Smallest r >= 1 with sum_{k>=r} sig2[k] <= eps^2 total / 3, capped."""
    thr = eps * eps * total / 3.0
    sig2 = np.asarray(sig2, dtype=np.float64)
    n = sig2.shape[0]
    r = n
    for cand in range(1, n + 1):
        if sig2[cand:].sum() <= thr:
            r = cand
            break
    return max(1, min(int(cap), r))


def canonicalise(t):
    """Flip kept columns so each one's largest-magnitude entry is positive."""
    G = t.G.copy()
    U = [u.copy() for u in t.U]
    for a in range(3):
        for k in range(U[a].shape[1]):
            col = U[a][:, k]
            i = int(np.argmax(np.abs(col)))
            if col[i] < 0:
                U[a][:, k] = -col
                sl = [slice(None)] * 3
                sl[a] = k
                G[tuple(sl)] *= -1.0
    return Tucker(G, U)


def _hosvd_bases(A, eps, cap, drop_rel=None):
    W, sig = [], []
    for a in range(3):
        Ua, s, _ = np.linalg.svd(unfold(A, a), full_matrices=False)
        s2 = s * s
        r = choose_rank(s2, s2.sum(), eps, cap)
        if drop_rel is not None:
            keep = int(np.sum(s > drop_rel * s[0])) if s[0] > 0 else 1
            r = max(1, min(r, keep))
        W.append(Ua[:, :r])
        sig.append(s)
    return W, sig


def hosvd(A, eps, cap, drop_rel=None, return_sigma=False):
    """Op1: truncated HOSVD of a full 3-D array (LAPACK SVD per unfolding)."""
    A = np.asarray(A, dtype=np.float64)
    W, sig = _hosvd_bases(A, eps, cap, drop_rel)
    G = A
    for a in range(3):
        G = mode_product(G, W[a].T, a)
    t = canonicalise(Tucker(G, W))
    return (t, sig) if return_sigma else t


def add(a, b):
    """Op2: element-wise sum; ranks add, core is block diagonal."""
    ra, rb = a.ranks, b.ranks
    G = np.zeros(tuple(x + y for x, y in zip(ra, rb)))
    G[:ra[0], :ra[1], :ra[2]] = a.G
    G[ra[0]:, ra[1]:, ra[2]:] = b.G
    return Tucker(G, [np.hstack([a.U[k], b.U[k]]) for k in range(3)])


def hadamard(a, b):
    """Op3: element-wise product; ranks multiply.

    Column k = kA * rB + kB of the result's factor holds the row-wise
    product U^A(:,kA) U^B(:,kB); the core is the Kronecker product.
    """
    G = np.kron(a.G, b.G)
    U = []
    for k in range(3):
        ua, ub = a.U[k], b.U[k]
        U.append((ua[:, :, None] * ub[:, None, :]).reshape(ua.shape[0], -1))
    return Tucker(G, U)


def convolve(t, w1, w2, w3):
    """Op5: sum_i A(i1,i2,i3) w1(i1) w2(i2) w3(i3) in O(n r^3)."""
    s = [t.U[0].T @ w1, t.U[1].T @ w2, t.U[2].T @ w3]
    return float(np.einsum("abc,a,b,c->", t.G, s[0], s[1], s[2]))


def lemma1(w1, w2, w3):
    """Lemma 1: w1(i1) + w2(i2) + w3(i3) as a Tucker tensor of ranks 2.

    Factors [w_a, 1]; the only non-zero core entries sit where exactly one
    index selects the w column (0-based (0,1,1), (1,0,1), (1,1,0)).
    """
    G = np.zeros((2, 2, 2))
    G[0, 1, 1] = G[1, 0, 1] = G[1, 1, 0] = 1.0
    U = [np.stack([np.asarray(w, float), np.ones(len(w))], 1) for w in (w1, w2, w3)]
    return Tucker(G, U)


def divide_rank1(t, d1, d2, d3):
    """Exact division by the rank-1 tensor d1(i1) d2(i2) d3(i3)."""
    return Tucker(t.G.copy(), [t.U[0] / d1[:, None], t.U[1] / d2[:, None], t.U[2] / d3[:, None]])


def round(t, eps, cap):  # noqa: A001 - the paper's name for Op4
    """Op4: Tucker rounding (QR of factors, core x R, SVD of core unfoldings)."""
    return round_sum([t], eps, cap)


def round_sum(terms, eps, cap):
    """Op4 applied to the Op2-sum of `terms`, without forming its core.

    The sum's factors are the concatenated term factors, U_a = Q_a R_a; its
    core is block diagonal, so core x_a R_a is the sum over terms of
    G_t x_1 R_1[:, cols_t] x_2 R_2[:, cols_t] x_3 R_3[:, cols_t].  The rest
    is the T-HOSVD of that small core, mapped back through Q.
    """
    Q, R = [], []
    for a in range(3):
        Ucat = np.hstack([t.U[a] for t in terms])
        q, r = np.linalg.qr(Ucat, mode="reduced")
        Q.append(q)
        R.append(r)
    shape = tuple(q.shape[1] for q in Q)
    Gp = np.zeros(shape)
    off = [0, 0, 0]
    for t in terms:
        blk = t.G
        for a in range(3):
            ra = t.ranks[a]
            blk = mode_product(blk, R[a][:, off[a]:off[a] + ra], a)
        Gp += blk
        for a in range(3):
            off[a] += t.ranks[a]
    W, _ = _hosvd_bases(Gp, eps, cap)
    G = Gp
    for a in range(3):
        G = mode_product(G, W[a].T, a)
    return canonicalise(Tucker(G, [Q[a] @ W[a] for a in range(3)]))


def tucker_rank1(u1, u2, u3, scale=1.0):
    return Tucker(np.full((1, 1, 1), float(scale)),
                  [np.asarray(u1, float)[:, None], np.asarray(u2, float)[:, None],
                   np.asarray(u3, float)[:, None]])
