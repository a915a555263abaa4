"""Error measures between two truncated SVDs.

Test infrastructure only.  The paper reports the maximum error of the computed singular values and,
for principal components, an infinity-norm difference and correlation coefficients (Sec. 4.1-4.2).
Reading: relative singular-value error per index, and the largest principal-angle sine between the
computed and the reference subspaces, which does not depend on column signs or on rotations within
clusters of equal singular values.
"""
import numpy as np


def rel_sigma_error(S, S_ref):
    """|S_j - S_ref_j| / S_ref_j elementwise (0 where both are 0)."""
    S = np.asarray(S, np.float64)
    S_ref = np.asarray(S_ref, np.float64)
    den = np.where(S_ref != 0, np.abs(S_ref), 1.0)
    return np.abs(S - S_ref) / den


def sin_theta_max(X_ref, X):
    """sin of the largest principal angle between span(X_ref) and span(X) (both orthonormal)."""
    X_ref = np.asarray(X_ref, np.float64)
    X = np.asarray(X, np.float64)
    R = X - X_ref @ (X_ref.T @ X)
    if R.size == 0:
        return 0.0
    return float(np.linalg.norm(R, 2))


def column_cosines(X_ref, X):
    """|cos| between matching columns."""
    num = np.abs(np.sum(np.asarray(X_ref) * np.asarray(X), axis=0))
    den = np.linalg.norm(X_ref, axis=0) * np.linalg.norm(X, axis=0)
    return num / np.where(den > 0, den, 1.0)
