"""Independent FP64 route for gap-free Toeplitz blocks (test infrastructure).

Levinson-Durbin recursion (the paper cites Levinson and Durbin for adapting
the operator to a segment, Sec. II.B item 6) gives the prediction-error
variances E_k of the symmetric positive-definite Toeplitz matrix, so that
det C = prod E_k, and the first column x of C^-1 (C x = e1).

The Gohberg-Semencul formula (Sec. III.A.3) writes
    C^-1 = (1/x1) (L_x L_x^T - R_x^T R_x)
with L_x lower-triangular Toeplitz with first column x and R_x strictly
upper-triangular Toeplitz with first row (0, x_n, ..., x_2).  Hence
    r^T C^-1 r = (||L_x^T r||^2 - ||R_x r||^2) / x1,
and each Toeplitz product is evaluated by circulant embedding of length
m >= 2n - 1 and FFTs (eq:toeplitz_fft).  No Cholesky factor is used.
"""
from __future__ import annotations

import numpy as np


def levinson_durbin(acf: np.ndarray):
    """Solve the Yule-Walker system for a symmetric PD Toeplitz matrix of size n.

    Returns (a, E): a are the order-(n-1) predictor coefficients with a[0] = 1,
    and E[k], k = 0..n-1, the prediction-error variance of order k, so that
    log det C = sum_k log E_k.
    """
    r = np.asarray(acf, dtype=np.float64)
    n = len(r)
    a = np.zeros(n)
    a[0] = 1.0
    E = np.empty(n)
    E[0] = r[0]
    for k in range(1, n):
        # reflection coefficient from the order-(k-1) predictor
        acc = r[k] + np.dot(a[1:k], r[k - 1:0:-1])
        kappa = -acc / E[k - 1]
        a_prev = a[:k].copy()
        a[1:k] = a_prev[1:k] + kappa * a_prev[k - 1:0:-1]
        a[k] = kappa
        E[k] = E[k - 1] * (1.0 - kappa * kappa)
    return a, E


def logdet_toeplitz(acf: np.ndarray) -> float:
    """log det of the SPD Toeplitz matrix of ``acf`` via Levinson-Durbin: sum log E_k."""
    _, E = levinson_durbin(acf)
    return float(np.sum(np.log(E)))


def first_column(acf: np.ndarray) -> np.ndarray:
    """x = C^-1 e1.  The augmented Yule-Walker system of the order-(n-1) predictor
    a = (1, a_1, ..., a_{n-1}) reads C a = E_{n-1} e1, hence x = a / E_{n-1}."""
    a, E = levinson_durbin(acf)
    return a / E[-1]


def toeplitz_matvec(col: np.ndarray, row: np.ndarray, v: np.ndarray) -> np.ndarray:
    """T v for the Toeplitz matrix with first column ``col`` and first row ``row``.

    Circulant embedding (eq:toeplitz_fft): m >= 2n - 1, c = (col, 0..., row[n-1..1]),
    T v = P_n F^-1[F(c) . F(v zero-padded to m)].  v may be [n] or [k, n].
    """
    n = len(col)
    m = 1 << int(np.ceil(np.log2(2 * n - 1)))
    c = np.zeros(m)
    c[:n] = col
    c[m - n + 1:] = row[1:][::-1]
    Fc = np.fft.fft(c)
    V = np.fft.fft(v, m, axis=-1)
    return np.real(np.fft.ifft(Fc * V, axis=-1))[..., :n]


def gs_quadratic_form(acf: np.ndarray, R: np.ndarray) -> np.ndarray:
    """r^T C^-1 r for each row r of R by the Gohberg-Semencul formula."""
    x = first_column(acf)
    n = len(x)
    zeros = np.zeros(n)
    # L_x^T r : L_x^T is upper Toeplitz with first row x, first column (x1, 0, ...)
    col_LT = np.zeros(n); col_LT[0] = x[0]
    u = toeplitz_matvec(col_LT, x, R)
    # R_x r : strictly upper Toeplitz with first row (0, x_n, ..., x_2), first column 0
    row_R = np.concatenate([[0.0], x[:0:-1]])
    v = toeplitz_matvec(zeros, row_R, R)
    return (np.sum(u * u, axis=-1) - np.sum(v * v, axis=-1)) / x[0]
