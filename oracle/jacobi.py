"""Brute-force one-sided (Hestenes) Jacobi SVD in pure Python loops, for tiny matrices.

Test infrastructure only.  It is an independent route to the exact SVD (Sec. 2.1, Eq. 1) used to pin
the reference when l = min(m, n), where Algorithm 4 must return the exact singular values.
"""
import math
import numpy as np


def jacobi_svd(A, tol=1e-15, max_sweeps=60):
    """Return (U, s, V) with A = U diag(s) V^T, s descending; A is m x n with m >= n."""
    W = [list(map(float, row)) for row in np.asarray(A, dtype=np.float64).T]   # columns of A
    n = len(W)
    m = len(W[0]) if n else 0
    if m < n:
        raise ValueError("jacobi_svd expects m >= n")
    J = [[1.0 if i == j else 0.0 for i in range(n)] for j in range(n)]      # columns of V
    for _ in range(max_sweeps):
        rotated = False
        for p in range(n - 1):
            for q in range(p + 1, n):
                alpha = sum(x * x for x in W[p])
                beta = sum(x * x for x in W[q])
                gamma = sum(x * y for x, y in zip(W[p], W[q]))
                if gamma == 0.0 or abs(gamma) <= tol * math.sqrt(alpha * beta):
                    continue
                rotated = True
                zeta = (beta - alpha) / (2.0 * gamma)
                t = math.copysign(1.0, zeta) / (abs(zeta) + math.sqrt(1.0 + zeta * zeta))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = c * t
                for vec in (W, J):
                    xp, xq = vec[p], vec[q]
                    vec[p] = [c * a - s * b for a, b in zip(xp, xq)]
                    vec[q] = [s * a + c * b for a, b in zip(xp, xq)]
        if not rotated:
            break
    sig = [math.sqrt(sum(x * x for x in col)) for col in W]
    order = sorted(range(n), key=lambda j: -sig[j])
    s = np.array([sig[j] for j in order])
    V = np.array([J[j] for j in order]).T
    U = np.zeros((m, n))
    for out, j in enumerate(order):
        if sig[j] > 0:
            U[:, out] = np.array(W[j]) / sig[j]
    return U, s, V
