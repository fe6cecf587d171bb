"""Independent FP64 references for the diffusion vectors -- TEST INFRASTRUCTURE.

Plain numpy / scipy definitions, used to pin the step-by-step oracle:

* PPR  f = alpha (I - (1-alpha) A D^-1)^-1 s                (Eq. (2))
* Katz x* = (I - beta A)^-1 s                                 (Eq. (3))
* HK   f = exp(-tau (I - A D^-1)) s and its Taylor truncation  (Sec. 2, "Heat Kernel")
* truncated Neumann series (what LocalGD computes when every nonzero residual
  is active) and the Chebyshev residual polynomial (what LocalCH computes in
  the same limit; Sec. 3.3).
* eigenvalue bounds of A.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
import scipy.sparse as sp


def dense_adjacency(row_ptr, col_idx):
    n = len(row_ptr) - 1
    A = np.zeros((n, n))
    for u in range(n):
        for e in range(row_ptr[u], row_ptr[u + 1]):
            A[col_idx[e], u] += 1.0
    return A


def sparse_adjacency(row_ptr, col_idx):
    n = len(row_ptr) - 1
    data = np.ones(len(col_idx))
    return sp.csr_matrix((data, np.asarray(col_idx), np.asarray(row_ptr)), shape=(n, n))


def degrees(row_ptr):
    return np.diff(np.asarray(row_ptr, dtype=np.int64)).astype(np.float64)


def seed_vector(n, seed_idx, seed_val=None):
    s = np.zeros(n)
    idx = np.atleast_1d(seed_idx)
    s[idx] = 1.0 if seed_val is None else np.atleast_1d(seed_val)
    return s


def walk_matrix(A):
    """M = A D^-1 (column-stochastic on nodes of positive degree)."""
    d = A.sum(axis=0)
    with np.errstate(divide="ignore"):
        inv = np.where(d > 0, 1.0 / d, 0.0)
    return A * inv[None, :]


def ppr_exact(A, alpha, s):
    n = A.shape[0]
    return alpha * np.linalg.solve(np.eye(n) - (1.0 - alpha) * walk_matrix(A), s)


def katz_exact(A, beta, s):
    n = A.shape[0]
    return np.linalg.solve(np.eye(n) - beta * A, s)


def hk_expm(A, tau, s):
    n = A.shape[0]
    return scipy.linalg.expm(-tau * (np.eye(n) - walk_matrix(A))) @ s


def hk_taylor(A, tau, K, s):
    """f_K = sum_{k<=K} e^{-tau} tau^k / k! M^k s."""
    M = walk_matrix(A)
    v = np.asarray(s, dtype=np.float64).copy()
    f = np.zeros_like(v)
    for k in range(K + 1):
        f += math.exp(-tau) * tau**k / math.factorial(k) * v
        v = M @ v
    return f


def neumann_ppr(A, alpha, s, T):
    """alpha * sum_{k<T} ((1-alpha) A D^-1)^k s."""
    M = (1.0 - alpha) * walk_matrix(A)
    v = alpha * np.asarray(s, dtype=np.float64)
    x = np.zeros_like(v)
    for _ in range(T):
        x += v
        v = M @ v
    return x


def neumann_katz(A, beta, s, T):
    """sum_{k<T} beta^k A^k s."""
    v = np.asarray(s, dtype=np.float64).copy()
    x = np.zeros_like(v)
    for _ in range(T):
        x += v
        v = beta * (A @ v)
    return x


def chebyshev_polynomial(t, z):
    """T_t(z) by its defining three-term recursion (Sec. 3.3)."""
    if t == 0:
        return np.ones_like(z)
    a, b = np.ones_like(z), z
    for _ in range(t - 1):
        a, b = b, 2.0 * z * b - a
    return b


def chebyshev_residual(Q, r0, mu, L, t):
    """Residual of t Chebyshev steps on Q x = b from x = 0:
    r_t = T_t((L+mu-2Q)/(L-mu)) r0 / T_t((L+mu)/(L-mu)), by eigendecomposition of Q
    (Q is similar to a symmetric matrix for both PPR and Katz)."""
    w, V = np.linalg.eig(Q)
    w = w.real
    V = V.real
    z = (L + mu - 2.0 * w) / (L - mu)
    scale = chebyshev_polynomial(t, np.array([(L + mu) / (L - mu)]))[0]
    coef = np.linalg.solve(V, r0)
    return V @ (chebyshev_polynomial(t, z) / scale * coef)


def adjacency_eig_bounds(A):
    w = np.linalg.eigvalsh(A)
    return float(w[0]), float(w[-1])


def lambda_bounds_power(row_ptr, col_idx, iters=100):
    """Bounds on the largest adjacency eigenvalue for graphs too large for a dense
    eigensolver (the Katz settings of Sec. 5 need beta * lambda_max < 1): power
    iteration on A + I from the all-ones vector.  Lower bound: the Rayleigh
    quotient v'Av / v'v.  Upper bound: the Collatz-Wielandt value max_u (Av)_u / v_u,
    which bounds the Perron root of a nonnegative matrix from above for any
    positive v.  Isolated nodes are excluded from the maximum (their ratio is 0)."""
    A = sparse_adjacency(row_ptr, col_idx)
    n = A.shape[0]
    v = np.ones(n)
    lo, hi = 0.0, float("inf")
    for _ in range(iters):
        Av = A @ v
        lo = max(lo, float(v @ Av) / float(v @ v))
        hi = min(hi, float(np.max(Av / v)))
        y = Av + v
        v = y / np.linalg.norm(y)
        v = np.maximum(v, 1e-300)
    return lo, hi


def global_ppr(row_ptr, col_idx, alpha, s, tol=1e-14, max_iter=100000):
    """Global FP64 Richardson on the whole graph until ||r||_1 < tol ||s||_1."""
    A = sparse_adjacency(row_ptr, col_idx)
    d = degrees(row_ptr)
    inv = np.where(d > 0, 1.0 / np.maximum(d, 1), 0.0)
    r = alpha * np.asarray(s, dtype=np.float64)
    x = np.zeros_like(r)
    target = tol * np.abs(s).sum()
    for _ in range(max_iter):
        x += r
        r = (1.0 - alpha) * (A @ (inv * r))
        if np.abs(r).sum() < target:
            break
    return x
