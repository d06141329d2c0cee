"""Pins of the oracle's Tucker algebra against brute force and theorems."""

import os

import numpy as np
import pytest

from oracle import tucker as tk

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_tucker(rng, N=(6, 5, 7), r=(2, 3, 2)):
    G = rng.standard_normal(r)
    U = [rng.standard_normal((N[a], r[a])) for a in range(3)]
    return tk.Tucker(G, U)


def brute_full(t):
    # element by element, independent of the mode-product code
    N = t.shape
    out = np.zeros(N)
    for i in range(N[0]):
        for j in range(N[1]):
            for k in range(N[2]):
                s = 0.0
                for a in range(t.ranks[0]):
                    for b in range(t.ranks[1]):
                        for c in range(t.ranks[2]):
                            s += t.G[a, b, c] * t.U[0][i, a] * t.U[1][j, b] * t.U[2][k, c]
                out[i, j, k] = s
    return out


def test_full_matches_elementwise_definition():
    rng = np.random.default_rng(0)
    t = rand_tucker(rng)
    np.testing.assert_allclose(tk.full(t), brute_full(t), rtol=0, atol=1e-12)


def test_op2_sum():
    rng = np.random.default_rng(1)
    a, b = rand_tucker(rng), rand_tucker(rng, r=(1, 2, 4))
    c = tk.add(a, b)
    assert c.ranks == (3, 5, 6)
    np.testing.assert_allclose(tk.full(c), tk.full(a) + tk.full(b), rtol=0, atol=1e-13)


def test_op3_hadamard_and_index_map():
    rng = np.random.default_rng(2)
    a, b = rand_tucker(rng), rand_tucker(rng, r=(3, 1, 2))
    c = tk.hadamard(a, b)
    assert c.ranks == (6, 3, 4)
    np.testing.assert_allclose(tk.full(c), tk.full(a) * tk.full(b), rtol=0, atol=1e-12)
    # factor column kA*rB + kB is the row-wise product of U^A(:,kA), U^B(:,kB)
    rB = b.ranks[0]
    for kA in range(a.ranks[0]):
        for kB in range(rB):
            np.testing.assert_array_equal(c.U[0][:, kA * rB + kB], a.U[0][:, kA] * b.U[0][:, kB])


def test_op5_convolution():
    rng = np.random.default_rng(3)
    t = rand_tucker(rng)
    w = [rng.standard_normal(n) for n in t.shape]
    ref = np.einsum("ijk,i,j,k->", brute_full(t), *w)
    assert abs(tk.convolve(t, *w) - ref) <= 1e-12 * max(1.0, abs(ref))


def test_lemma1_matches_paper_core_and_sum():
    rows = np.loadtxt(os.path.join(GOLDEN, "lemma1_core.txt"))
    rng = np.random.default_rng(4)
    w = [rng.standard_normal(n) for n in (5, 6, 7)]
    t = tk.lemma1(*w)
    assert t.ranks == (2, 2, 2)
    G = np.zeros((2, 2, 2))
    for k1, k2, k3, v in rows:
        G[int(k1) - 1, int(k2) - 1, int(k3) - 1] = v
    np.testing.assert_array_equal(t.G, G)
    ref = w[0][:, None, None] + w[1][None, :, None] + w[2][None, None, :]
    np.testing.assert_allclose(tk.full(t), ref, rtol=0, atol=1e-14)


def test_rank1_division_exact():
    rng = np.random.default_rng(5)
    t = rand_tucker(rng)
    d = [rng.uniform(0.5, 2.0, n) for n in t.shape]
    q = tk.divide_rank1(t, *d)
    D = d[0][:, None, None] * d[1][None, :, None] * d[2][None, None, :]
    np.testing.assert_allclose(tk.full(q), tk.full(t) / D, rtol=1e-13, atol=1e-13)


def test_hosvd_eckart_young_matrix_case():
    # an N1 x N2 x 1 tensor: T-HOSVD truncation of mode 1 is the matrix
    # truncated SVD, whose Frobenius error is the discarded singular values
    rng = np.random.default_rng(6)
    M = rng.standard_normal((9, 8)) @ np.diag(0.5 ** np.arange(8)) @ rng.standard_normal((8, 8))
    A = M[:, :, None]
    t, sig = tk.hosvd(A, 0.0, 3, return_sigma=True)
    s = np.linalg.svd(M, compute_uv=False)
    err = np.linalg.norm(tk.full(t) - A)
    assert t.ranks[0] == 3 and t.ranks[1] == 3
    # both modes truncated to 3: error equals the matrix tail (same subspace)
    assert abs(err - np.sqrt((s[3:] ** 2).sum())) <= 1e-12 * np.linalg.norm(M)


@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-4])
def test_hosvd_error_bounds(eps):
    rng = np.random.default_rng(7)
    x = np.linspace(-3, 3, 12)
    A = np.exp(-(x[:, None, None] - 0.3 * x[None, :, None] * x[None, None, :] / 3) ** 2)
    A += 1e-3 * rng.standard_normal(A.shape)
    t, sig = tk.hosvd(A, eps, 12, return_sigma=True)
    err2 = np.linalg.norm(tk.full(t) - A) ** 2
    tails = [float((sig[a][t.ranks[a]:] ** 2).sum()) for a in range(3)]
    assert max(tails) <= err2 * (1 + 1e-10) + 1e-24
    assert err2 <= sum(tails) * (1 + 1e-10) + 1e-24
    assert np.sqrt(err2) <= eps * np.linalg.norm(A) * (1 + 1e-12)
    # each rank is the smallest that meets its share of the bound
    for a in range(3):
        r = t.ranks[a]
        if r > 1:
            assert float((sig[a][r - 1:] ** 2).sum()) > eps ** 2 * np.linalg.norm(A) ** 2 / 3


def test_hosvd_keeps_exact_low_rank():
    rng = np.random.default_rng(8)
    t0 = rand_tucker(rng, N=(8, 8, 8), r=(2, 3, 2))
    A = tk.full(t0)
    t = tk.hosvd(A, 1e-12, 8)
    assert t.ranks == (2, 3, 2)
    np.testing.assert_allclose(tk.full(t), A, rtol=0, atol=1e-13 * np.abs(A).max())
    for a in range(3):
        np.testing.assert_allclose(t.U[a].T @ t.U[a], np.eye(t.ranks[a]), atol=1e-13)
        # sign canonical: largest-magnitude entry of every column positive
        for k in range(t.ranks[a]):
            col = t.U[a][:, k]
            assert col[np.argmax(np.abs(col))] > 0


def test_op4_rounding_equals_hosvd_of_full():
    rng = np.random.default_rng(9)
    x = np.linspace(-2, 2, 10)
    terms = [tk.hosvd(np.exp(-(x[:, None, None] - c) ** 2 - (x[None, :, None] * c) ** 2
                             - x[None, None, :] ** 2 * (1 + c)), 0.0, 4) for c in (0.1, 0.5, 0.9)]
    terms.append(rand_tucker(rng, N=(10, 10, 10), r=(2, 2, 2)).scaled(1e-3))
    A = sum(tk.full(t) for t in terms)
    for eps, cap in ((1e-3, 10), (1e-6, 10), (1e-6, 3)):
        r1 = tk.round_sum(terms, eps, cap)
        r2 = tk.hosvd(A, eps, cap)
        assert r1.ranks == r2.ranks
        np.testing.assert_allclose(tk.full(r1), tk.full(r2), rtol=0, atol=1e-12 * np.abs(A).max())
        # single-tensor Op4 on the Op2 sum gives the same
        s = terms[0]
        for t in terms[1:]:
            s = tk.add(s, t)
        r3 = tk.round(s, eps, cap)
        np.testing.assert_allclose(tk.full(r3), tk.full(r2), rtol=0, atol=1e-12 * np.abs(A).max())


def test_truncation_mass_error_bound():
    rng = np.random.default_rng(10)
    A = rng.standard_normal((8, 8, 8)) * np.exp(-np.arange(8))[:, None, None]
    t = tk.hosvd(A, 1e-2, 8)
    D = tk.full(t) - A
    assert abs(D.sum()) <= 8 ** 1.5 * np.linalg.norm(D) + 1e-15


def test_choose_rank_rule():
    s2 = np.array([1.0, 1e-2, 1e-4, 1e-6, 0.0])
    tot = s2.sum()
    assert tk.choose_rank(s2, tot, 0.0, 10) == 4      # only exact zeros dropped
    assert tk.choose_rank(s2, tot, 1.0, 10) == 1
    thr = (s2[2:].sum() * 3 / tot) ** 0.5              # tail from index 2 exactly at the threshold
    assert tk.choose_rank(s2, tot, thr * (1 + 1e-9), 10) == 2
    assert tk.choose_rank(s2, tot, thr * (1 - 1e-9), 10) == 3
    assert tk.choose_rank(s2, tot, 0.0, 2) == 2
