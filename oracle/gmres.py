"""Restarted GMRES with right diagonal (Jacobi) preconditioning.

Test infrastructure only. The paper uses an iterative solver with a
diagonal preconditioner, stopped when the relative root-mean-square residual
falls below a tolerance (Section 2.2); it does not name the method. We take
GMRES(m) (Saad & Schultz 1986) with x0 = 0, right preconditioning
A D^-1 u = b, x = D^-1 u, D = diag(Z), modified Gram-Schmidt Arnoldi and
Givens rotations, stopped on ||b - A x|| / ||b|| <= tol (the relative RMS
residual is this same ratio). A zero right-hand side returns x = 0.
"""

from __future__ import annotations

import numpy as np


def gmres(apply_a, b: np.ndarray, diag: np.ndarray, tol: float, restart: int = 100,
          max_iter: int = 10_000, x0=None):
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    bnorm = np.linalg.norm(b)
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    hist = []
    if bnorm == 0.0:
        return x, dict(iters=0, resid=0.0, history=hist, converged=True)
    dinv = 1.0 / diag
    its = 0
    while True:
        r = b - apply_a(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta / bnorm <= tol or its >= max_iter:
            return x, dict(iters=its, resid=beta / bnorm, history=hist, converged=beta / bnorm <= tol)
        m = restart
        V = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        V[0] = r / beta
        g[0] = beta
        j_end = 0
        for j in range(m):
            w = apply_a(dinv * V[j])
            its += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            # previous rotations, then a new one that zeroes H[j+1, j]:
            # Q_i = [[conj(c_i), conj(s_i)], [-s_i, c_i]]
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, c = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            cs[j], sn[j] = (a / den, c / den) if den != 0 else (1.0, 0.0)
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            j_end = j + 1
            if abs(g[j + 1]) / bnorm <= tol or its >= max_iter or H[j, j] == 0:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + dinv * (V[:j_end].T @ y)
