"""Pins of the FP64 HOOI oracle against facts fixed by the paper and by linear
algebra (not against the oracle's own formulas)."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import hooi as O


def _rng(seed):
    return np.random.default_rng(seed)


def _ttm_loops(X, A, n):
    """TTM by its element-wise definition: Z[..k..] = sum_l A[k,l] X[..l..]."""
    shape = list(X.shape)
    out_shape = shape.copy()
    out_shape[n] = A.shape[0]
    Z = np.zeros(out_shape)
    for idx in itertools.product(*[range(s) for s in out_shape]):
        k = idx[n]
        s = 0.0
        for l in range(shape[n]):
            src = list(idx)
            src[n] = l
            s += A[k, l] * X[tuple(src)]
        Z[idx] = s
    return Z


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 4, 2), (5, 1, 3), (4, 3)])
def test_ttm_matches_elementwise_definition(shape):
    g = _rng(1)
    X = g.standard_normal(shape)
    for n in range(len(shape)):
        A = g.standard_normal((3, shape[n]))
        np.testing.assert_allclose(O.ttm(X, A, n), _ttm_loops(X, A, n), rtol=1e-13, atol=1e-13)


def test_ttm_is_matrix_product_on_unfolding():
    # Sec. 2.1: Z = X x_n A is realised as A @ X_(n), read back as Z_(n).
    g = _rng(2)
    X = g.standard_normal((4, 5, 6, 3))
    for n in range(4):
        A = g.standard_normal((2, X.shape[n]))
        Z = O.ttm(X, A, n)
        np.testing.assert_allclose(O.unfold(Z, n), A @ O.unfold(X, n), rtol=1e-13, atol=1e-13)
        assert Z.shape[n] == 2 and Z.size == 2 * X.size // X.shape[n]


def test_ttm_identity_and_unit_mode():
    g = _rng(3)
    X = g.standard_normal((3, 1, 4))
    for n in range(3):
        np.testing.assert_array_equal(O.ttm(X, np.eye(X.shape[n]), n), X)
    A = g.standard_normal((5, 1))
    Z = O.ttm(X, A, 1)
    np.testing.assert_allclose(Z, A[None, :, 0, None] * X[:, 0:1, :], rtol=1e-15)


def test_ttm_chain_commutes():
    # Sec. 2.1: (T x_{n1} A1) x_{n2} A2 = (T x_{n2} A2) x_{n1} A1.
    g = _rng(4)
    T = g.standard_normal((5, 6, 7))
    A1 = g.standard_normal((2, 5))
    A2 = g.standard_normal((3, 7))
    left = O.ttm(O.ttm(T, A1, 0), A2, 2)
    right = O.ttm(O.ttm(T, A2, 2), A1, 0)
    np.testing.assert_allclose(left, right, rtol=1e-12, atol=1e-12)


def test_lead_spans_leading_singular_subspace():
    # leading eigenvectors of the Gram = leading left singular vectors (SVD).
    g = _rng(5)
    Y = g.standard_normal((9, 4, 5))
    for n in range(3):
        K = 3
        F, w = O.lead(Y, n, K)
        U, s, _ = np.linalg.svd(O.unfold(Y, n), full_matrices=False)
        np.testing.assert_allclose(F @ F.T, U[:, :K] @ U[:, :K].T, atol=1e-12)
        np.testing.assert_allclose(w, s[:K] ** 2, rtol=1e-12)
        assert np.all(np.diff(w) <= 0)
        np.testing.assert_allclose(F.T @ F, np.eye(K), atol=1e-13)
        # sign rule: largest-magnitude entry of every column is positive
        for j in range(K):
            assert F[np.argmax(np.abs(F[:, j])), j] > 0


def test_matrix_case_is_truncated_svd():
    # N = 2: HOSVD/HOOI reach the Eckart-Young optimum, err = tail of singular values.
    g = _rng(6)
    M = g.standard_normal((12, 9))
    k = 4
    s = np.linalg.svd(M, compute_uv=False)
    expect = math.sqrt(np.sum(s[k:] ** 2)) / np.linalg.norm(M)
    F = O.hosvd(M, (k, k))
    G = O.new_core(M, F)
    assert abs(O.rel_error_explicit(M, G, F) - expect) < 1e-13
    F2, G2, _ = O.hooi_step(M, F, (k, k))
    assert abs(O.rel_error_explicit(M, G2, F2) - expect) < 1e-13


def test_planted_exact_rank_recovered_to_roundoff():
    T, info = synth.planted((10, 11, 12), (3, 4, 2), noise=0.0, dtype="f64", cfg=90)
    F = O.hosvd(T, (3, 4, 2))
    G = O.new_core(T, F)
    assert O.rel_error_explicit(T, G, F) < 1e-13
    for n in range(3):
        U = info["factors"][n]
        np.testing.assert_allclose(F[n] @ F[n].T, U @ U.T, atol=1e-12)
    F, G, errs = O.hooi(T, (3, 4, 2), 2, F0=F)
    assert max(errs) < 1e-13


def test_norm_identity_with_orthonormal_factors():
    # ||T||^2 = ||G||^2 + ||T - G x F||^2 when every F_n has orthonormal columns.
    g = _rng(7)
    T = g.standard_normal((6, 7, 5))
    K = (3, 2, 4)
    F = [np.linalg.qr(g.standard_normal((T.shape[n], K[n])))[0] for n in range(3)]
    G = O.new_core(T, F)
    e = O.rel_error_explicit(T, G, F)
    nT2 = float(np.sum(T * T))
    assert abs(nT2 - (float(np.sum(G * G)) + e * e * nT2)) < 1e-12 * nT2
    assert abs(O.rel_error_identity(nT2, G) - e) < 1e-12


def test_core_norm_equals_gram_trace_for_every_mode():
    # ||T x_j F_j^T (all j)||^2 = trace(F_n^T S_n F_n), S_n = Gram of T x_{j!=n} F_j^T.
    g = _rng(8)
    T = g.standard_normal((5, 6, 4, 3))
    K = (2, 3, 2, 2)
    F = [np.linalg.qr(g.standard_normal((T.shape[n], K[n])))[0] for n in range(4)]
    G = O.new_core(T, F)
    g2 = float(np.sum(G * G))
    for n in range(4):
        S = O.gram(O.chain_except(T, F, n), n)
        assert abs(np.trace(F[n].T @ S @ F[n]) - g2) < 1e-12 * g2


def test_hooi_error_monotone_on_planted_tensor():
    T, _ = synth.planted((16, 16, 16), (4, 4, 4), noise=1e-3, noise_kind="abs", dtype="f64",
                         cfg=91)
    F, G, errs = O.hooi(T, (4, 4, 4), 6)
    e0 = O.rel_error_explicit(T, O.new_core(T, O.hosvd(T, (4, 4, 4))), O.hosvd(T, (4, 4, 4)))
    seq = [e0] + errs
    for a, b in zip(seq, seq[1:]):
        assert b <= a + 1e-12


def test_gauss_seidel_variant_never_increases_error():
    # Classical ALS form: each mode update minimises the error given the others.
    for seed in range(6):
        g = _rng(100 + seed)
        T = g.standard_normal((5, 6, 4))
        K = (2, 3, 2)
        F = O.hosvd(T, K)
        prev = O.rel_error_explicit(T, O.new_core(T, F), F)
        for _ in range(4):
            F, G = O.hooi_step_gauss_seidel(T, F, K)
            e = O.rel_error_explicit(T, G, F)
            assert e <= prev + 1e-12
            prev = e


def test_tree_leaves_equal_any_chain_order():
    # A leaf Y_n depends only on the set of modes multiplied (commutativity).
    g = _rng(9)
    T = g.standard_normal((4, 5, 3, 6))
    F = [np.linalg.qr(g.standard_normal((T.shape[n], 2)))[0] for n in range(4)]
    for n in range(4):
        ref = O.chain_except(T, F, n)
        others = [j for j in range(4) if j != n]
        for perm in itertools.permutations(others):
            Y = T
            for j in perm:
                Y = O.ttm(Y, F[j].T, j)
            np.testing.assert_allclose(Y, ref, rtol=1e-12, atol=1e-12)


def test_leaf_entries_by_definition():
    g = _rng(10)
    T = g.standard_normal((4, 5, 3, 6))
    F = [g.standard_normal((T.shape[n], 2)) for n in range(4)]
    for n in range(4):
        Y = O.chain_except(T, F, n)
        idx = [tuple(int(g.integers(0, s)) for s in Y.shape) for _ in range(7)]
        np.testing.assert_allclose(O.leaf_entries(T, F, n, idx), [Y[i] for i in idx],
                                   rtol=1e-12, atol=1e-12)


def test_bf16_upcast_exact():
    bits = np.array([0x3F80, 0xC000, 0x0000, 0x3E80, 0x7F7F], dtype=np.uint16)
    np.testing.assert_array_equal(O.as_f64(bits, "bf16"),
                                  [1.0, -2.0, 0.0, 0.25, float(np.float32(3.3895314e38))])


# ---------------------------------------------------------------------------
# STHOSVD (initial decomposition, Sec. 1 and Sec. 2.2)
# ---------------------------------------------------------------------------
def test_sthosvd_two_modes_equals_truncated_svd():
    """N = 2: the first step is the leading K left singular vectors of T, the
    second the leading K right singular vectors of U_K^T T = Sigma_K V_K^T:
    both factors span the truncated SVD's subspaces, and the error is the
    Eckart-Young tail sqrt(sum_{i>K} sigma_i^2) / ||T||."""
    g = np.random.default_rng(4)
    T = g.standard_normal((30, 22))
    K = (5, 5)
    F, G, disc = O.sthosvd(T, K)
    U, sv, Vt = np.linalg.svd(T)
    assert np.linalg.norm(F[0] @ F[0].T - U[:, :5] @ U[:, :5].T, 2) < 1e-12
    assert np.linalg.norm(F[1] @ F[1].T - Vt[:5].T @ Vt[:5], 2) < 1e-12
    e = O.rel_error_explicit(T, G, F)
    assert abs(e - np.sqrt(np.sum(sv[5:] ** 2)) / np.linalg.norm(T)) < 1e-12
    # the second step discards nothing: U_K^T T has rank K
    assert abs(disc[1]) < 1e-10 * np.sum(sv ** 2)


def test_sthosvd_recovers_planted_tensor():
    L, K = (14, 12, 10, 9), (3, 4, 2, 3)
    T, info = synth.planted(L, K, noise=0.0, dtype="f64", cfg=90)
    for order in (None, (3, 1, 0, 2)):
        F, G, disc = O.sthosvd(T, K, order=order)
        for n in range(4):
            U = info["factors"][n]
            assert np.linalg.norm(F[n] @ F[n].T - U @ U.T, 2) < 1e-10
        assert O.rel_error_explicit(T, G, F) < 1e-13


def test_sthosvd_error_is_sum_of_discarded_energy():
    """The residual of STHOSVD splits into the parts each step removes, and
    they are mutually orthogonal: ||T - G x F||^2 = sum of the discarded
    eigenvalue tails of the sequential Grams (exact, any order); each tail is
    at most the tail of the original unfolding, so the error is at most the
    HOSVD bound sqrt(sum_n tail_n(T_(n)))."""
    g = np.random.default_rng(12)
    T = g.standard_normal((11, 9, 8, 7))
    K = (4, 3, 5, 2)
    nT2 = float(np.sum(T * T))
    for order in (None, (2, 0, 3, 1)):
        F, G, disc = O.sthosvd(T, K, order=order)
        e = O.rel_error_explicit(T, G, F)
        assert abs(e * e * nT2 - sum(disc)) < 1e-10 * nT2
        assert abs(O.rel_error_identity(nT2, G) - e) < 1e-10
        tails = []
        for n in range(4):
            w = np.sort(np.linalg.eigvalsh(O.gram(T, n)))[::-1]
            tails.append(float(np.sum(w[K[n]:])))
        assert e * e * nT2 <= sum(tails) * (1 + 1e-12)
        # the factors are orthonormal and the core is T projected on them
        for n in range(4):
            assert np.abs(F[n].T @ F[n] - np.eye(K[n])).max() < 1e-13
        assert np.allclose(G, O.new_core(T, F), atol=1e-12 * np.sqrt(nT2))
