"""Algorithm 2 (the earlier single-pass algorithm the paper compares against, Sec. 2.3), plain
FP64.  Test infrastructure only: it exists so the accuracy study of Sec. 4.1 can be repeated on
the reference side; the GPU path does not implement it.
"""
import numpy as np

from .pca import _qr_nonneg, apply_sign_convention


def alg2_single_pass(A, Omega, Omega_t, k, want_u=True):
    """Algorithm 2: Y = A Omega and Y~ = A^T Omega~ from one pass; Q = orth(Y), Q~ = orth(Y~);
    B solves Omega~^T Q B = Y~^T Q~ (least squares when Omega~^T Q is not square); svd(B) gives
    S, and U = Q U~, V = Q~ V~.  Omega is n x l and Omega~ is m x l2 (l2 >= l)."""
    A = np.asarray(A, dtype=np.float64)
    Y = A @ Omega
    Yt = A.T @ Omega_t
    Q, _ = _qr_nonneg(Y)
    Qt, _ = _qr_nonneg(Yt)
    M = Omega_t.T @ Q
    rhs = Yt.T @ Qt
    B = np.linalg.lstsq(M, rhs, rcond=None)[0]
    Ub, s, Vbt = np.linalg.svd(B, full_matrices=False)
    kk = min(k, len(s))
    S = np.zeros(k)
    S[:kk] = s[:kk]
    V = np.zeros((A.shape[1], k))
    V[:, :kk] = Qt @ Vbt[:kk].T
    U = None
    if want_u:
        U = np.zeros((A.shape[0], k))
        U[:, :kk] = Q @ Ub[:, :kk]
    U, V = apply_sign_convention(U, V)
    return S, U, V
