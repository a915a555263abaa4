"""Singular-value spectra for synthetic test matrices.

Index j runs from 1.  The five "Type" spectra are the ones of the paper's accuracy study
(Sec. 4.1); the others are the decays of the workload recipes.
"""
import numpy as np


def paper_type_spectrum(kind: int, count: int) -> np.ndarray:
    """Spectrum Type 1..5 of Sec. 4.1, first ``count`` values, descending."""
    j = np.arange(1, count + 1, dtype=np.float64)
    if kind == 1:
        s = np.where(j <= 20, 10.0 ** (-4.0 * (j - 1) / 19.0),
                     1e-4 / np.maximum(j - 20, 1) ** 0.1)
    elif kind == 2:
        s = j ** -2.0
    elif kind == 3:
        s = j ** -3.0
    elif kind == 4:
        s = np.exp(-j / 7.0)
    elif kind == 5:
        s = 10.0 ** (-j / 10.0)
    else:
        raise ValueError(f"unknown spectrum type {kind}")
    return s


def exp_spectrum(count: int, scale: float) -> np.ndarray:
    """sigma_j = exp(-j/scale)."""
    j = np.arange(1, count + 1, dtype=np.float64)
    return np.exp(-j / scale)


def inv_spectrum(count: int) -> np.ndarray:
    """sigma_j = 1/j."""
    return 1.0 / np.arange(1, count + 1, dtype=np.float64)


def inv_floor_spectrum(count: int, knee: int = 200, floor: float = 1e-4) -> np.ndarray:
    """sigma_j = 1/j for j <= knee, then a constant floor."""
    j = np.arange(1, count + 1, dtype=np.float64)
    return np.where(j <= knee, 1.0 / j, floor)


def inv_square_spectrum(count: int) -> np.ndarray:
    """sigma_j = j^-2."""
    return np.arange(1, count + 1, dtype=np.float64) ** -2.0


def noisy_spectrum(sigma: np.ndarray, noise_std: float, seed: int) -> np.ndarray:
    """|sigma_j + noise_std * N(0,1)|, re-sorted descending.

    The noise acts on the singular values (not on the entries), so the spectrum of the matrix built
    from the result stays exactly known.
    """
    rng = np.random.default_rng(seed)
    s = np.abs(np.asarray(sigma, dtype=np.float64) + noise_std * rng.standard_normal(len(sigma)))
    return np.sort(s)[::-1].copy()
