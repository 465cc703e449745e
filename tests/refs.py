"""Independent reference computations used to pin the oracle.

None of these routines calls the oracle: they compute the quantities the
oracle must reproduce by other routes (explicit DFT matrices, direct circular
convolution loops, dense solves, brute-force enumeration, projected gradient).
"""
from __future__ import annotations

import itertools

import numpy as np


def dft_matrix(n: int, sign: int = -1) -> np.ndarray:
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


def naive_dft2(x: np.ndarray) -> np.ndarray:
    """Unnormalised 2-D DFT from its definition, by two explicit DFT matrices."""
    ph, pw = x.shape[-2:]
    return dft_matrix(ph) @ x @ dft_matrix(pw).T


def circ_conv2(d: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Circular convolution on z's grid: out[m,n] = sum_ab d[a,b] z[(m-a)%Ph, (n-b)%Pw]."""
    ph, pw = z.shape
    out = np.zeros((ph, pw))
    for a in range(d.shape[0]):
        for b in range(d.shape[1]):
            out += d[a, b] * np.roll(np.roll(z, a, axis=0), b, axis=1)
    return out


def toeplitz_operator(filt: np.ndarray, shape) -> np.ndarray:
    """Matrix T(d) with T(d) vec(z) = vec(d (*) z) (circular, row-major vec), built by loops."""
    ph, pw = shape
    P = ph * pw
    T = np.zeros((P, P))
    for col in range(P):
        e = np.zeros(P)
        e[col] = 1.0
        T[:, col] = circ_conv2(filt, e.reshape(shape)).ravel()
    return T


def code_shift_matrix(z: np.ndarray, filt_shape) -> np.ndarray:
    """Matrix A with A vec(d) = vec(d (*) z) for filters of shape filt_shape."""
    mh, mw = filt_shape
    cols = []
    for a in range(mh):
        for b in range(mw):
            cols.append(np.roll(np.roll(z, a, axis=0), b, axis=1).ravel())
    return np.stack(cols, axis=1)


def lasso_objective(A, x, u, lam):
    r = x - A @ u
    return 0.5 * float(r @ r) + lam * float(np.abs(u).sum())


def brute_force_lasso(A: np.ndarray, x: np.ndarray, lam: float, tol: float = 1e-10):
    """Global minimiser of 1/2||x - A u||^2 + lam ||u||_1 by enumerating sign patterns.

    For every assignment of {-1, 0, +1} to the unknowns the KKT system on the
    active set is solved; consistent candidates are kept and the best returned.
    Returns (u, objective, n_optimal_candidates).
    """
    n = A.shape[1]
    best_u, best_f = np.zeros(n), lasso_objective(A, x, np.zeros(n), lam)
    for pattern in itertools.product((-1, 0, 1), repeat=n):
        s = np.array(pattern, dtype=float)
        act = np.nonzero(s)[0]
        if act.size == 0:
            continue
        As = A[:, act]
        M = As.T @ As
        try:
            ua = np.linalg.solve(M, As.T @ x - lam * s[act])
        except np.linalg.LinAlgError:
            continue
        if np.any(np.sign(ua) != s[act]):
            continue
        u = np.zeros(n)
        u[act] = ua
        g = A.T @ (x - A @ u)
        inact = np.setdiff1d(np.arange(n), act)
        if inact.size and np.max(np.abs(g[inact])) > lam + tol:
            continue
        f = lasso_objective(A, x, u, lam)
        if f < best_f:
            best_u, best_f = u, f
    return best_u, best_f


def project_ball(v: np.ndarray) -> np.ndarray:
    n = np.linalg.norm(v)
    return v / max(n, 1.0)


def fista_ball(As, xs, K: int, m2: int, iters: int = 20000):
    """Projected accelerated gradient for min_d sum_i 1/2||x_i - A_i d||^2, ||d_k|| <= 1.

    ``d`` stacks K filters of m2 taps; returns d of shape (K, m2).
    """
    Q = sum(A.T @ A for A in As)
    c = sum(A.T @ x for A, x in zip(As, xs))
    L = np.linalg.eigvalsh(Q)[-1]
    d = np.zeros(K * m2)
    y = d.copy()
    tk = 1.0
    for _ in range(iters):
        g = Q @ y - c
        dn = (y - g / L).reshape(K, m2)
        dn = np.stack([project_ball(r) for r in dn]).ravel()
        tn = 0.5 * (1 + np.sqrt(1 + 4 * tk * tk))
        y = dn + ((tk - 1) / tn) * (dn - d)
        d, tk = dn, tn
    return d.reshape(K, m2)
