"""Plain FP64 definition of the likelihood (test infrastructure; see package docstring).

Definitions followed (paper Sec. II):
  * Covariance of wide-sense-stationary noise: C_ij = rho(|i - j|), a symmetric
    Toeplitz matrix built from the autocorrelation function rho (Sec. II, the
    Toeplitz definition).
  * Inner product <s, h> = s^T C^-1 h (eqn:ip) and the exact Gaussian
    likelihood ln L = const - 1/2 <d - h, d - h> (eqn:lik).
  * Whitened form: C = L L^T with lower-triangular L, whitening operator
    W = L^-1, r = W (d - h), ln L = -1/2 r^T r + const (Sec. II.A,
    eq:td_innerprod_whitened, eq:td_like_whitened).
  * Time segments: the covariance of a segment is the Toeplitz matrix of the
    ACF truncated to the segment length (Sec. II.B item 1); disjoint segments
    are independent blocks.
  * Data gaps: excluded samples are dropped from the model (Sec. II.B item 2).
    Reading: the retained samples have the marginal Gaussian law, covariance
    C[keep, keep]; values at excluded samples are ignored.
  * Multi-detector likelihood: per-detector log-likelihoods are summed
    (Sec. II.B item 3).
  * The triangular solve is the paper's CDL evaluation (Sec. III.A, the
    solve_triangular call).
  * Constant (the paper writes "const"): -1/2 log det C - (N_eff/2) log 2 pi with
    N_eff the number of retained samples over all segments.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg as sla

LOG2PI = float(np.log(2.0 * np.pi))


def retained_indices(N: int, gap_mask: Optional[np.ndarray] = None,
                     segments: Optional[Sequence[Tuple[int, int]]] = None) -> List[np.ndarray]:
    """Per segment, the sorted absolute indices of retained samples (gap_mask == 0)."""
    if segments is None:
        segments = [(0, N)]
    out = []
    for off, length in segments:
        idx = np.arange(off, off + length)
        if gap_mask is not None:
            idx = idx[np.asarray(gap_mask)[off:off + length] == 0]
        out.append(idx)
    return out


def segment_covariance(acf: np.ndarray, offset: int, length: int, idx: np.ndarray) -> np.ndarray:
    """C_s = Toeplitz(acf[:length]) restricted to rows/cols idx - offset (Sec. II, II.B)."""
    T = sla.toeplitz(np.asarray(acf[:length], dtype=np.float64))
    loc = np.asarray(idx) - offset
    return T[np.ix_(loc, loc)]


@dataclasses.dataclass
class Factor:
    """Cholesky factors of each segment block: C_s = L_s L_s^T (lower)."""
    N: int
    segments: List[Tuple[int, int]]
    idx: List[np.ndarray]
    L: List[np.ndarray]
    logdet: float
    n_eff: int


def factor(acf: np.ndarray, N: int, gap_mask: Optional[np.ndarray] = None,
           segments: Optional[Sequence[Tuple[int, int]]] = None) -> Factor:
    """Factor every segment block once (one-time O(N^3) cost, Sec. III.A.2).

    log det C = sum over blocks of 2 sum log diag(L_s).
    Raises numpy.linalg.LinAlgError if a block is not positive definite.
    """
    segs = [(0, N)] if segments is None else [tuple(map(int, s)) for s in segments]
    idxs = retained_indices(N, gap_mask, segs)
    Ls, logdet, n_eff = [], 0.0, 0
    for (off, length), idx in zip(segs, idxs):
        if len(idx) == 0:
            Ls.append(np.zeros((0, 0)))
            continue
        C = segment_covariance(acf, off, length, idx)
        L = sla.cholesky(C, lower=True)
        Ls.append(L)
        logdet += 2.0 * float(np.sum(np.log(np.diag(L))))
        n_eff += len(idx)
    return Factor(N, segs, idxs, Ls, logdet, n_eff)


def whiten(f: Factor, X: np.ndarray) -> np.ndarray:
    """W x restricted to retained samples, segments concatenated: r_s = L_s^-1 x[idx_s].

    X: [..., N] (one vector or one row per template).  Returns [..., N_eff].
    """
    X = np.asarray(X, dtype=np.float64)
    parts = []
    for idx, L in zip(f.idx, f.L):
        if len(idx) == 0:
            continue
        rhs = X[..., idx]
        sol = sla.solve_triangular(L, rhs.reshape(-1, len(idx)).T, lower=True)
        parts.append(sol.T.reshape(rhs.shape))
    return np.concatenate(parts, axis=-1)


def quad_forms(f: Factor, R: np.ndarray) -> np.ndarray:
    """q = r^T C^-1 r = ||W r||^2 for each row of R (eqn:ip via eq:td_innerprod_whitened)."""
    w = whiten(f, R)
    return np.sum(w * w, axis=-1)


def loglik(f: Factor, d: np.ndarray, H: np.ndarray) -> np.ndarray:
    """Per-template log-likelihood of one detector, constants included.

    logL_b = -1/2 ||W (d - h_b)||^2 - 1/2 log det C - (N_eff/2) log 2 pi.
    """
    d = np.asarray(d, dtype=np.float64)
    H = np.atleast_2d(np.asarray(H, dtype=np.float64))
    q = quad_forms(f, d[None, :] - H)
    return -0.5 * q - 0.5 * f.logdet - 0.5 * f.n_eff * LOG2PI


def loglik_network(factors: Sequence[Factor], ds: Sequence[np.ndarray], H: np.ndarray) -> np.ndarray:
    """Network log-likelihood: sum of per-detector logL (Sec. II.B item 3); same H in every detector."""
    total = None
    for f, d in zip(factors, ds):
        x = loglik(f, d, H)
        total = x if total is None else total + x
    return total
