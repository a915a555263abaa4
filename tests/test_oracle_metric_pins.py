"""Pins of the oracle's error measures and of its sign convention.

The paper reports singular-value errors and compares principal components by their difference and
correlation (Sec. 4.1-4.2); every subspace assertion of the GPU tests and of the benchmark goes
through ``sin_theta_max``, so it must be shown to measure what it claims, not only to return small
numbers.  The pins use configurations whose principal angles are known in closed form: two
subspaces spanned by q_i and cos(t_i) q_i + sin(t_i) q_(k+i) for orthonormal q have exactly the
principal angles t_i.  The sign convention (a reading: the paper leaves signs open) is pinned by
hand-made vectors, including ties.
"""
import inspect
import textwrap

import numpy as np
import pytest

import oracle
from oracle import metrics as M
from oracle import pca as P


def _orthonormal(n, k, seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    return q


def _rotated_pair(n, k, angles, seed):
    """(X_ref, X): orthonormal n x k bases whose principal angles are exactly `angles` (padded with
    zeros to k)."""
    Q = _orthonormal(n, 2 * k, seed)
    t = np.zeros(k)
    t[:len(angles)] = angles
    X_ref = Q[:, :k]
    X = Q[:, :k] * np.cos(t) + Q[:, k:] * np.sin(t)
    return X_ref, X


# ---------------------------------------------------------------- sin_theta_max -------------------
def _check_sin_theta(fn):
    """Every closed-form fact about the largest principal angle; returns True when all hold."""
    ok = True
    X_ref, _ = _rotated_pair(60, 5, [], 1)
    ok &= fn(X_ref, X_ref) < 1e-14                                  # equal spans
    for angles in ([0.3], [0.7, 0.2], [np.pi / 2 - 1e-3, 0.1, 0.05], [1e-6]):
        X_ref, X = _rotated_pair(80, 6, angles, 2)
        ok &= abs(fn(X_ref, X) - np.sin(max(angles))) < 1e-13      # largest angle
        ok &= abs(fn(X, X_ref) - np.sin(max(angles))) < 1e-13      # symmetric for equal dims
    # invariant to column signs and to any rotation within either span
    X_ref, X = _rotated_pair(50, 4, [0.4, 0.1], 3)
    R = _orthonormal(4, 4, 4)
    s0 = np.sin(0.4)
    ok &= abs(fn(X_ref, X * np.array([1, -1, -1, 1])) - s0) < 1e-13
    ok &= abs(fn(X_ref @ R, X @ R.T) - s0) < 1e-13
    # one basis vector swapped for an orthogonal one: the angle is pi/2
    Q = _orthonormal(40, 6, 5)
    ok &= abs(fn(Q[:, :3], np.column_stack([Q[:, 0], Q[:, 1], Q[:, 5]])) - 1.0) < 1e-13
    # a lower-dimensional subspace inside the reference has angle 0
    ok &= fn(Q[:, :4], Q[:, 1:3]) < 1e-14
    return bool(ok)


def test_sin_theta_max_closed_forms():
    """sin of the largest principal angle: 0 for equal spans, sin(t) for a planted rotation by t,
    symmetric, invariant to signs and in-span rotations, 1 for an orthogonal replacement."""
    assert _check_sin_theta(oracle.sin_theta_max)


def test_sin_theta_max_against_svd_definition():
    """The principal-angle cosines are the singular values of X_ref^T X (Bjorck-Golub); the
    largest sine is sqrt(1 - min cos^2), computed here from scipy's subspace_angles."""
    from scipy.linalg import subspace_angles
    rng = np.random.default_rng(6)
    for k in (1, 3, 10):
        A = np.linalg.qr(rng.standard_normal((100, k)))[0]
        B = np.linalg.qr(A + 0.05 * rng.standard_normal((100, k)))[0]
        ref = np.sin(np.max(subspace_angles(A, B)))
        assert abs(oracle.sin_theta_max(A, B) - ref) < 1e-12


def test_rel_sigma_error_values():
    """|S - S_ref| / S_ref, with 0 where both vanish and the absolute error where S_ref = 0."""
    e = oracle.rel_sigma_error([1.1, 2.0, 0.0, 0.5], [1.0, 4.0, 0.0, 0.0])
    assert np.allclose(e, [0.1, 0.5, 0.0, 0.5], rtol=0, atol=1e-15)


def test_column_cosines_values():
    X = np.array([[1.0, 0.0], [0.0, 2.0]])
    Y = np.array([[-3.0, 1.0], [0.0, 1.0]])
    assert np.allclose(oracle.column_cosines(X, Y), [1.0, 1 / np.sqrt(2)], atol=1e-15)


# ---------------------------------------------------------------- sign convention -----------------
def _check_signs(fn):
    """The reading: flip (u_j, v_j) together so the largest-|.| entry of v_j is positive, the
    lowest index deciding ties; zero columns are left alone."""
    V = np.array([[0.1, -0.5, 0.5, 0.0, -0.2],
                  [-0.9, 0.5, -0.5, 0.0, 0.2],
                  [0.3, 0.1, 0.2, 0.0, 0.1]])
    U = np.arange(1.0, 16.0).reshape(3, 5)
    U2, V2 = fn(U, V)
    want = np.array([-1.0, -1.0, 1.0, 1.0, -1.0])   # col 0: -0.9 wins; cols 1, 2, 4: ties
    ok = np.array_equal(V2, V * want) and np.array_equal(U2, U * want)
    ok &= np.array_equal(V, np.array([[0.1, -0.5, 0.5, 0.0, -0.2], [-0.9, 0.5, -0.5, 0.0, 0.2],
                                      [0.3, 0.1, 0.2, 0.0, 0.1]]))     # inputs not modified
    U3, V3 = fn(U2, V2)                                                 # idempotent
    ok &= np.array_equal(V3, V2) and np.array_equal(U3, U2)
    _, V4 = fn(None, -V)                                                # U optional
    ok &= np.array_equal(V4, V2)
    return bool(ok)


def test_sign_convention_rule():
    assert _check_signs(oracle.apply_sign_convention)


# ---------------------------------------------------------------- planted mistakes ----------------
_METRIC_MUTATIONS = {
    "frobenius_norm": (M.sin_theta_max, "np.linalg.norm(R, 2)", "np.linalg.norm(R)"),
    "no_projection": (M.sin_theta_max, "R = X - X_ref @ (X_ref.T @ X)", "R = X_ref.T @ X"),
    "always_zero": (M.sin_theta_max, "return float(np.linalg.norm(R, 2))", "return 0.0"),
    "transposed_projector": (M.sin_theta_max, "X_ref @ (X_ref.T @ X)", "X_ref @ (X.T @ X_ref)"),
}
_SIGN_MUTATIONS = {
    "signed_argmax": (P.apply_sign_convention, "np.argmax(np.abs(col))", "np.argmax(col)"),
    "last_index_on_ties": (P.apply_sign_convention, "p = int(np.argmax(np.abs(col)))",
                           "p = len(col) - 1 - int(np.argmax(np.abs(col[::-1])))"),
    "u_not_flipped": (P.apply_sign_convention, "U[:, j] = -U[:, j]", "U[:, j] = U[:, j]"),
    "inverted_rule": (P.apply_sign_convention, "if col[p] < 0:", "if col[p] > 0:"),
}


def _mutant(fn, old, new):
    src = textwrap.dedent(inspect.getsource(fn))
    assert old in src, old
    ns = dict(inspect.getmodule(fn).__dict__)
    exec(src.replace(old, new), ns)
    return ns[fn.__name__]


def _caught(check, fn):
    """A mutant is caught when a pin fails or the mutant cannot even run the pins."""
    try:
        return not check(fn)
    except (ValueError, IndexError, TypeError):
        return True


@pytest.mark.parametrize("name", sorted(_METRIC_MUTATIONS))
def test_metric_pins_catch_planted_mistakes(name):
    fn, old, new = _METRIC_MUTATIONS[name]
    assert _caught(_check_sin_theta, _mutant(fn, old, new))


@pytest.mark.parametrize("name", sorted(_SIGN_MUTATIONS))
def test_sign_pins_catch_planted_mistakes(name):
    fn, old, new = _SIGN_MUTATIONS[name]
    assert _caught(_check_signs, _mutant(fn, old, new))
