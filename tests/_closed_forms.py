"""Closed forms used as references where the oracle cannot run (test
infrastructure; no arithmetic of the method itself)."""
from __future__ import annotations

import numpy as np


def path_laplacian_expm(m: int, t: float) -> np.ndarray:
    """e^{-t L} for the Laplacian of a path of m nodes (unit weights, degree 1
    at both ends), from its exact eigenbasis: eigenvalues 2 - 2 cos(pi k / m)
    with eigenvectors cos(pi k (j + 1/2) / m), k = 0 .. m-1."""
    k = np.arange(m)[None, :]
    j = np.arange(m)[:, None]
    V = np.cos(np.pi * k * (j + 0.5) / m)
    V[:, 0] *= np.sqrt(1.0 / m)
    V[:, 1:] *= np.sqrt(2.0 / m)
    lam = 2.0 - 2.0 * np.cos(np.pi * np.arange(m) / m)
    return (V * np.exp(-t * lam)[None, :]) @ V.T


def unit_grid_expm_row(P: np.ndarray, cols: int, i: int) -> np.ndarray:
    """Row i of e^{-t L} for the unit 5-point grid Laplacian of a rows x cols
    grid numbered row-major: L = L_rows (x) I + I (x) L_cols, the two terms
    commute, so e^{-t L} = e^{-t L_rows} (x) e^{-t L_cols}.  P is the path
    exponential of the (square) grid side."""
    y, x = divmod(i, cols)
    return np.outer(P[y], P[x]).ravel()
