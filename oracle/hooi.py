"""FP64 CPU oracle for one HOOI invocation -- test infrastructure only.

Everything here is float64 NumPy, written from the paper's definitions:

* TTM (Sec. 2.1, "Tensor-Times-Matrix Multiplication"): Z = X x_n A applies
  the K x L_n matrix A to every mode-n fiber; Z has length K along mode n.
* TTM-chain (Sec. 2.1): multiply along several distinct modes, in any order.
* HOOI (Sec. 2.2, Fig. 2 "HOOI Procedure"), Jacobi form: for every mode n,
  Z = T x_{j != n} F_j^T with the *input* factors, then F~_n = leading K_n left
  singular vectors of Z_(n); after all modes, the new core
  G~ = T x_1 F~_1^T ... x_N F~_N^T.
* The singular vectors come from the Gram matrix Z_(n) Z_(n)^T followed by a
  symmetric eigensolver (Sec. 5, Gram + EVD).
* Error: normalised root-mean-square difference between T and the recovered
  tensor (Sec. 2.2); read as ||T - G x_1 F_1 ... x_N F_N||_F / ||T||_F.

Readings of points the paper leaves open (each listed in the design notes):
  - the per-mode chain runs in ascending mode order (any order is equal by
    commutativity);
  - eigenvalues are taken in descending order, eigenvectors get a sign rule:
    the largest-magnitude entry of each column (lowest index on ties) is made
    positive;
  - the unfolding's column order is row-major (last mode fastest); the Gram
    matrix does not depend on it.
"""
from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# Sec. 2.1: tensor basics
# --------------------------------------------------------------------------
def as_f64(T_stored: np.ndarray, dtype: str) -> np.ndarray:
    """Exact float64 upcast of a stored tensor ("f64", "f32", "f16" or "bf16" bits)."""
    if dtype == "bf16":
        b = np.asarray(T_stored, dtype=np.uint16)
        return (b.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    return np.asarray(T_stored, dtype=np.float64)


def ttm(X: np.ndarray, A: np.ndarray, n: int) -> np.ndarray:
    """Z = X x_n A for a K x L_n matrix A (Sec. 2.1, TTM).

    Every mode-n fiber x of X is replaced by A @ x.  Viewing X (row-major) as a
    stack of A_n matrices of size L_n x B_n (A_n = product of the lengths before
    mode n, B_n = product after), each such matrix M becomes A @ M.
    """
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    shape = X.shape
    if A.ndim != 2 or A.shape[1] != shape[n]:
        raise ValueError(f"ttm: matrix {A.shape} does not match mode {n} of {shape}")
    a = int(np.prod(shape[:n], dtype=np.int64))
    b = int(np.prod(shape[n + 1:], dtype=np.int64))
    Z = np.matmul(A, X.reshape(a, shape[n], b))
    return Z.reshape(shape[:n] + (A.shape[0],) + shape[n + 1:])


def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding X_(n): L_n x (|X|/L_n), columns are the mode-n fibers (Sec. 2.1)."""
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def chain_except(T: np.ndarray, F, n: int) -> np.ndarray:
    """Naive TTM-chain of Fig. 2: T x_j F_j^T over every mode j != n, ascending j."""
    Y = T
    for j in range(T.ndim):
        if j != n:
            Y = ttm(Y, np.asarray(F[j]).T, j)
    return Y


# --------------------------------------------------------------------------
# Sec. 2.2 / Sec. 5: leading singular vectors through the Gram matrix
# --------------------------------------------------------------------------
def gram(Y: np.ndarray, n: int) -> np.ndarray:
    """S = Y_(n) Y_(n)^T (Sec. 5: Gram matrix before the eigen-decomposition)."""
    M = unfold(Y, n)
    return M @ M.T


def sign_rule(V: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of each column positive (first index on ties)."""
    V = np.array(V, dtype=np.float64, copy=True)
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V


def leading_eigvecs(S: np.ndarray, K: int):
    """Leading K eigenpairs of a symmetric S, eigenvalues descending, sign rule applied."""
    w, V = np.linalg.eigh(S)
    order = np.argsort(-w, kind="stable")[:K]
    return sign_rule(V[:, order]), w[order]


def lead(Y: np.ndarray, n: int, K: int):
    """Leading K left singular vectors of Y_(n) (via Gram + EVD) and the Gram eigenvalues."""
    return leading_eigvecs(gram(Y, n), K)


# --------------------------------------------------------------------------
# Fig. 2: one HOOI invocation, its start, core and error
# --------------------------------------------------------------------------
def hosvd(T: np.ndarray, K) -> list:
    """HOSVD start: F_n = leading K_n left singular vectors of T_(n)."""
    return [lead(T, n, int(K[n]))[0] for n in range(T.ndim)]


def sthosvd(T: np.ndarray, K, order=None):
    """Sequentially truncated HOSVD, the initial decomposition of Sec. 1 and
    Sec. 2.2: modes are processed one after another (ascending unless `order`
    is given); mode n takes the leading K_n left singular vectors of the
    current tensor's mode-n unfolding and truncates the tensor along n
    before the next mode.  Returns (F, G, discarded) with G the truncated
    tensor (the core) and discarded[i] the sum of the eigenvalues of the
    i-th step's Gram beyond the K_n leading ones (the energy that step
    removes)."""
    N = T.ndim
    order = list(range(N)) if order is None else [int(n) for n in order]
    if sorted(order) != list(range(N)):
        raise ValueError(f"order {order} is not a permutation of the modes")
    F = [None] * N
    Y = np.asarray(T, dtype=np.float64)
    discarded = []
    for n in order:
        S = gram(Y, n)
        w = np.linalg.eigvalsh(S)
        Fn, wn = leading_eigvecs(S, int(K[n]))
        discarded.append(float(np.sum(w) - np.sum(wn)))
        F[n] = Fn
        Y = ttm(Y, Fn.T, n)
    return F, Y, discarded


def new_core(T: np.ndarray, F) -> np.ndarray:
    """G = T x_1 F_1^T x_2 ... x_N F_N^T (Fig. 2, new core)."""
    G = T
    for n in range(T.ndim):
        G = ttm(G, np.asarray(F[n]).T, n)
    return G


def reconstruct(G: np.ndarray, F) -> np.ndarray:
    """Recovered tensor Z = G x_1 F_1 ... x_N F_N (Sec. 2.2)."""
    Z = G
    for n in range(G.ndim):
        Z = ttm(Z, F[n], n)
    return Z


def rel_error_explicit(T: np.ndarray, G: np.ndarray, F) -> float:
    """||T - G x_1 F_1 ... x_N F_N||_F / ||T||_F."""
    R = T - reconstruct(G, F)
    return float(np.linalg.norm(R.reshape(-1)) / np.linalg.norm(T.reshape(-1)))


def rel_error_identity(normT2: float, G: np.ndarray) -> float:
    """sqrt(max(||T||^2 - ||G||^2, 0)) / ||T||, valid for orthonormal factors."""
    g2 = float(np.dot(G.reshape(-1), G.reshape(-1)))
    return math.sqrt(max(normT2 - g2, 0.0) / normT2)


def hooi_step(T: np.ndarray, F, K):
    """One HOOI invocation, Jacobi form (every chain uses the input factors).

    Returns (F_new, G_new, leaves) where leaves[n] = T x_{j != n} F_j^T.
    """
    leaves = [chain_except(T, F, n) for n in range(T.ndim)]
    F_new = [lead(leaves[n], n, int(K[n]))[0] for n in range(T.ndim)]
    return F_new, new_core(T, F_new), leaves


def hooi_step_gauss_seidel(T: np.ndarray, F, K):
    """Gauss-Seidel HOOI (oracle-only variant): mode n already uses F~_1..F~_{n-1}.

    This is the classical alternating least-squares form whose error is
    non-increasing; kept to contrast with the Jacobi form of Fig. 2.
    """
    F = [np.asarray(f, dtype=np.float64) for f in F]
    for n in range(T.ndim):
        F[n] = lead(chain_except(T, F, n), n, int(K[n]))[0]
    return F, new_core(T, F)


def hooi(T: np.ndarray, K, iters: int, F0=None):
    """HOSVD (or F0) start, then `iters` Jacobi HOOI invocations.

    Returns (F, G, errs) with errs[t] the explicit relative error after t+1
    invocations.
    """
    F = hosvd(T, K) if F0 is None else [np.asarray(f, dtype=np.float64) for f in F0]
    errs = []
    G = None
    for _ in range(iters):
        F, G, _ = hooi_step(T, F, K)
        errs.append(rel_error_explicit(T, G, F))
    return F, G, errs


# --------------------------------------------------------------------------
# Single entries by definition (for sampled checks on full-size tensors)
# --------------------------------------------------------------------------
def leaf_entries(T: np.ndarray, F, n: int, index_list) -> np.ndarray:
    """Entries of Y_n = T x_{j != n} F_j^T, each computed from its definition.

    index_list holds tuples (k_1, .., l_n, .., k_N).  For one entry the slice of
    T at l_n along mode n is contracted, mode by mode, with the column k_j of F_j.
    """
    out = np.empty(len(index_list), dtype=np.float64)
    N = T.ndim
    for e, idx in enumerate(index_list):
        X = np.take(T, int(idx[n]), axis=n).astype(np.float64)
        # remaining axes are the modes j != n in ascending order
        for j in reversed([j for j in range(N) if j != n]):
            axis = j if j < n else j - 1
            X = np.tensordot(X, np.asarray(F[j], dtype=np.float64)[:, int(idx[j])],
                             axes=([axis], [0]))
        out[e] = float(X)
    return out
