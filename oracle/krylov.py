"""GMRES and flexible GMRES (FGMRES) in FP64.

Readings where the paper is silent: Arnoldi orthogonalisation is classical
Gram-Schmidt applied twice (CGS2); the small least-squares problem is solved
with complex Givens rotations; the starting guess of the coarse GMRES is zero.
The outer solver is right-preconditioned FGMRES(m) (Saad's flexible GMRES,
which the paper names as the outer method, Sec. 2) with a true-residual
recomputation after each restart cycle.
"""
import numpy as np


def _dot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def _norm(a):
    return float(np.sqrt(np.real(_dot(a, a))))


def givens(a, b):
    """(c, s) with [[c, s], [-conj(s), c]] @ [a, b] = [r, 0], c real."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, 1.0 + 0.0j
    rho = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    c = abs(a) / rho
    s = (a / abs(a)) * np.conj(b) / rho
    return c, s


def _arnoldi_step(V, w, j):
    h = np.zeros(j + 2, dtype=np.complex128)
    for _ in range(2):
        hh = np.array([_dot(V[i], w) for i in range(j + 1)])
        for i in range(j + 1):
            w = w - hh[i] * V[i]
        h[:j + 1] += hh
    h[j + 1] = _norm(w)
    return h, w


def _least_squares_update(H, cs, g, h, j):
    for i in range(j):
        c, s = cs[i]
        t = c * h[i] + s * h[i + 1]
        h[i + 1] = -np.conj(s) * h[i] + c * h[i + 1]
        h[i] = t
    c, s = givens(h[j], h[j + 1])
    cs.append((c, s))
    h[j] = c * h[j] + s * h[j + 1]
    h[j + 1] = 0.0
    g[j + 1] = -np.conj(s) * g[j]
    g[j] = c * g[j]
    H[:j + 1, j] = h[:j + 1]


def _back_solve(H, g, k):
    y = np.zeros(k, dtype=np.complex128)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
    return y


def gmres(apply, b, maxiter, tol=None):
    """GMRES from x0 = 0; stops after maxiter steps or at ||r|| <= tol ||b||.

    Returns (x, iterations, estimated residual norm).
    """
    beta = _norm(b)
    if beta == 0.0:
        return np.zeros_like(b), 0, 0.0
    V = [b / beta]
    H = np.zeros((maxiter + 1, maxiter), dtype=np.complex128)
    g = np.zeros(maxiter + 1, dtype=np.complex128)
    g[0] = beta
    cs = []
    k = 0
    for j in range(maxiter):
        w = apply(V[j])
        h, w = _arnoldi_step(V, w, j)
        hnext = h[j + 1]
        _least_squares_update(H, cs, g, h, j)
        k = j + 1
        if hnext == 0.0:
            break
        V.append(w / hnext)
        if tol is not None and abs(g[j + 1]) <= tol * beta:
            break
    y = _back_solve(H, g, k)
    x = np.zeros_like(b)
    for i in range(k):
        x = x + y[i] * V[i]
    return x, k, float(abs(g[k]))


def fgmres(apply, precond, b, tol, restart, maxiter, x0=None):
    """Right-preconditioned FGMRES(restart) for apply(x) = b.

    Stops when the true residual ||b - apply(x)|| <= tol ||b|| (checked after
    every restart cycle, and whenever the Arnoldi estimate says so) or after
    maxiter preconditioned steps.  Returns (x, iterations, true relative
    residual history per cycle).
    """
    bnorm = _norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply(x)
    hist = [_norm(r) / bnorm]
    it = 0
    while hist[-1] > tol and it < maxiter:
        beta = _norm(r)
        V = [r / beta]
        Z = []
        m = min(restart, maxiter - it)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        cs = []
        k = 0
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            h, w = _arnoldi_step(V, apply(z), j)
            hnext = h[j + 1]
            _least_squares_update(H, cs, g, h, j)
            k = j + 1
            it += 1
            if hnext == 0.0 or abs(g[j + 1]) <= tol * bnorm:
                break
            V.append(w / hnext)
        y = _back_solve(H, g, k)
        for i in range(k):
            x = x + y[i] * Z[i]
        r = b - apply(x)
        hist.append(_norm(r) / bnorm)
    return x, it, hist
