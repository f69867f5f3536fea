"""Synthetic workload generators (inputs only; no likelihood arithmetic).

Paper context: data model d = h + n with wide-sense-stationary Gaussian noise
whose covariance is the Toeplitz matrix of the ACF (Sec. II); the benchmark
shapes are fs = 4096 Hz and N = 16384 (4 s, Sec. III.B.1), two detectors
(Sec. V), segments and gaps (Sec. II.B items 1-2).  The real strain data,
Welch PSDs and NRSur7dq4 waveforms the paper uses are not available; the
analytic PSD and the Newtonian-like chirp below stand in for them.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

FS = 4096.0                 # sample rate [Hz]
PSD_GRID = 2 ** 20          # one fixed irfft length for every N ("recompute and truncate")
EPS_PRIMARY = 1e-6          # nugget added to lag 0 after normalisation (primary)
EPS_STRESS = 1e-8           # stress nugget (kappa ~ 3e8)
SEED_BASE = 260306010       # workload k uses SEED_BASE + k
F_LO, F_HI = 20.0, 2048.0   # PSD support [Hz]; zero below F_LO


def analytic_psd(f: np.ndarray) -> np.ndarray:
    """One-sided PSD S(f) = (f/30)^-4 + 1 + (f/300)^2 on [20, 2048] Hz, 0 elsewhere."""
    f = np.asarray(f, dtype=np.float64)
    s = np.zeros_like(f)
    band = (f >= F_LO) & (f <= F_HI)
    fb = f[band]
    s[band] = (fb / 30.0) ** -4 + 1.0 + (fb / 300.0) ** 2
    return s


_GRID_CACHE = {}


def _grid():
    if "R" not in _GRID_CACHE:
        f = np.fft.rfftfreq(PSD_GRID, 1.0 / FS)
        S = analytic_psd(f)
        R = np.fft.irfft(S, PSD_GRID)
        _GRID_CACHE["f"] = f
        _GRID_CACHE["S"] = S
        _GRID_CACHE["R"] = R
    return _GRID_CACHE["f"], _GRID_CACHE["S"], _GRID_CACHE["R"]


def make_acf(n_lags: int, eps: float = EPS_PRIMARY) -> np.ndarray:
    """ACF rho[0..n_lags-1] of the analytic PSD, normalised so rho[0] = 1, plus ``eps`` at lag 0.

    The PSD is sampled on one fixed rfft grid of length 2^20 for every N, inverted
    with an inverse real FFT, truncated to the requested number of lags and
    normalised by lag 0 (Sec. II.B item 6: ACF from a PSD by inverse FFT, then
    truncated to the segment).  The literal recipe has about 1% of its spectrum
    exactly zero (below 20 Hz) and its Toeplitz matrices are numerically
    singular for N >= 2048, so a nugget ``eps`` is added to lag 0 after
    normalisation; ``eps`` is part of the input, never added by the library.
    """
    if n_lags > PSD_GRID // 2:
        raise ValueError("n_lags exceeds half the PSD grid")
    _, _, R = _grid()
    acf = R[:n_lags] / R[0]
    acf = acf.copy()
    acf[0] += eps
    return acf


def eig_bounds(eps: float = EPS_PRIMARY) -> Tuple[float, float]:
    """Bounds (lo, hi) on every eigenvalue of any covariance built from ``make_acf(n, eps)``.

    toeplitz(make_acf(n, eps)), n <= 2^19, is the leading block of the 2^20 circulant whose
    eigenvalues are S_k / R[0] + eps (see ``stationary_noise``), and a gapped covariance
    C[keep, keep] is a principal submatrix of that block.  By Cauchy interlacing every
    eigenvalue lies in [min_k S_k / R[0] + eps, max_k S_k / R[0] + eps]; min_k S_k = 0
    (the band below 20 Hz), so lo = eps.  hi / lo bounds the condition number.
    """
    _, S, R = _grid()
    return float(S.min() / R[0] + eps), float(S.max() / R[0] + eps)


def stationary_noise(rng: np.random.Generator, n: int, count: int,
                     eps: float = EPS_PRIMARY) -> np.ndarray:
    """``count`` independent length-``n`` draws from N(0, toeplitz(make_acf(n, eps))).

    Circulant embedding on the 2^20 grid: the circulant whose first column is the
    periodic normalised autocovariance plus ``eps`` at lag 0 has eigenvalues
    S_k / R[0] + eps >= 0, and its leading n x n block is exactly the Toeplitz
    covariance of ``make_acf``.  Hence these draws have exactly the law of
    L z with C = L L^T and z ~ N(0, I) (the paper's noise recipe), without
    factoring C.  Each complex FFT yields two independent real draws.
    """
    _, S, R = _grid()
    lam_half = S / R[0] + eps                      # rfft-grid eigenvalues
    lam = np.concatenate([lam_half, lam_half[-2:0:-1]])  # full Hermitian grid
    scale = np.sqrt(lam / PSD_GRID)
    out = np.empty((count, n), dtype=np.float64)
    k = 0
    while k < count:
        z = rng.standard_normal(PSD_GRID) + 1j * rng.standard_normal(PSD_GRID)
        x = np.fft.fft(scale * z)
        out[k] = x.real[:n]
        if k + 1 < count:
            out[k + 1] = x.imag[:n]
        k += 2
    return out


def chirp(n: int, f0, tc, phi0, amp) -> np.ndarray:
    """Newtonian-like chirp templates, one row per parameter set.

    t_j = j / fs; x = 1 - t/tc; f(t) = f0 x^(-3/8); amplitude amp * x^(-1/4);
    phase phi0 + 2 pi f0 tc (8/5) (1 - x^(5/8)) (the exact integral of f).
    The frequency is capped at 1024 Hz by ending the signal sharply at
    t_cap = tc (1 - (f0/1024)^(8/3)); a Tukey(0.1) window over all n samples
    tapers the start.  Broadcasts over parameter arrays.
    """
    from scipy.signal.windows import tukey
    f0 = np.atleast_1d(np.asarray(f0, np.float64))[:, None]
    tc = np.atleast_1d(np.asarray(tc, np.float64))[:, None]
    phi0 = np.atleast_1d(np.asarray(phi0, np.float64))[:, None]
    amp = np.atleast_1d(np.asarray(amp, np.float64))[:, None]
    t = (np.arange(n, dtype=np.float64) / FS)[None, :]
    tcap = tc * (1.0 - (f0 / 1024.0) ** (8.0 / 3.0))
    x = np.clip(1.0 - t / tc, 1e-300, None)
    h = amp * x ** -0.25 * np.cos(phi0 + 2.0 * np.pi * f0 * tc * 1.6 * (1.0 - x ** 0.625))
    h = np.where(t > tcap, 0.0, h)
    return h * tukey(n, 0.1)[None, :]


def whittle_snr2(h: np.ndarray) -> np.ndarray:
    """Band-limited frequency-domain (Whittle) optimal SNR^2 of each row of ``h``.

    SNR^2 = (1/M) sum_k |H_k|^2 / lambda(f_k) over the bins with 20 <= f <= 2048 Hz,
    both signs of frequency, with H the length-M FFT of the zero-padded row
    (M = next power of two >= 2n) and lambda(f) = S(f)/R[0] the per-sample
    spectrum of the normalised noise.  This is the conventional matched-filter
    SNR of the analysis band; it is used only to set template amplitudes and is
    not the time-domain quantity the library evaluates.
    """
    h = np.atleast_2d(h)
    n = h.shape[1]
    m = 1 << int(np.ceil(np.log2(2 * n)))
    _, _, R = _grid()
    f = np.fft.rfftfreq(m, 1.0 / FS)
    S = analytic_psd(f)
    band = S > 0
    w = np.where(band, 2.0, 0.0)
    w[-1] = np.where(band[-1], 1.0, 0.0)     # Nyquist bin counted once
    inv = np.where(band, R[0] / np.where(band, S, 1.0), 0.0) * w
    out = np.empty(h.shape[0])
    for i in range(0, h.shape[0], 256):
        Hk = np.fft.rfft(h[i:i + 256], m, axis=1)
        out[i:i + 256] = (np.abs(Hk) ** 2 * inv[None, :]).sum(1) / m
    return out


def draw_gaps(rng: np.random.Generator, n: int, count: int,
              lmin: int = 64, lmax: int = 512) -> List[Tuple[int, int]]:
    """``count`` disjoint gaps (start, length), lengths U{lmin..lmax}, starts U{0..n-len}.

    Redrawn until pairwise disjoint with at least one retained sample between
    any two gaps.  Sorted by start.
    """
    if count == 0:
        return []
    while True:
        lens = rng.integers(lmin, lmax + 1, size=count)
        starts = np.array([rng.integers(0, n - L + 1) for L in lens])
        order = np.argsort(starts)
        s, L = starts[order], lens[order]
        ok = all(s[i] + L[i] < s[i + 1] for i in range(count - 1))
        if ok:
            return [(int(a), int(b)) for a, b in zip(s, L)]


def gap_mask_from(n: int, gaps: Sequence[Tuple[int, int]]) -> np.ndarray:
    """uint8 mask of length n, 1 = excluded sample."""
    m = np.zeros(n, dtype=np.uint8)
    for s, L in gaps:
        m[s:s + L] = 1
    return m


@dataclasses.dataclass
class Instance:
    """One analysis instance: n_det detectors sharing a template bank.

    acf: float64[N] (nugget included); masks: per detector uint8[N] or None;
    segments: list of (offset, length) or None (one segment [0, N));
    d: float64[n_det, N]; H: float64[B, N] (same templates in every detector).
    """
    N: int
    acf: np.ndarray
    masks: List[Optional[np.ndarray]]
    segments: Optional[List[Tuple[int, int]]]
    d: np.ndarray
    H: np.ndarray
    eps: float

    @property
    def n_det(self) -> int:
        return self.d.shape[0]

    @property
    def B(self) -> int:
        return self.H.shape[0]


@dataclasses.dataclass
class Workload:
    name: str
    instances: List[Instance]
    requests: Optional[dict] = None


def _template_params(rng, n, count):
    T = n / FS
    f0 = rng.uniform(20.0, 40.0, count)
    tc = rng.uniform(0.8 * T, T, count)
    phi0 = rng.uniform(0.0, 2.0 * np.pi, count)
    snr = rng.uniform(8.0, 30.0, count)
    return f0, tc, phi0, snr


def _scaled_chirps(n, f0, tc, phi0, snr, n_det):
    """Chirps with network (band-limited Whittle) SNR = ``snr``; same h in every detector."""
    h = chirp(n, f0, tc, phi0, np.ones_like(f0))
    s2 = whittle_snr2(h) * n_det
    return h * (snr / np.sqrt(s2))[:, None]


def _streams(k):
    root = np.random.default_rng(SEED_BASE + k)
    return dict(zip(["gaps", "noise", "injection", "templates", "requests"], root.spawn(5)))


def _instance(st, n, n_det, n_gaps, B, eps, rows=None):
    acf = make_acf(n, eps)
    masks = []
    for _ in range(n_det):                      # gap positions drawn per detector
        g = draw_gaps(st["gaps"], n, n_gaps) if n_gaps else []
        masks.append(gap_mask_from(n, g) if g else None)
    noise = stationary_noise(st["noise"], n, n_det, eps)
    p = _template_params(st["injection"], n, 1)
    inj = _scaled_chirps(n, *p, n_det)[0]
    d = noise + inj[None, :]
    pt = _template_params(st["templates"], n, B)
    if rows is not None:  # only these template rows (same draws as the full bank)
        pt = tuple(np.asarray(x)[rows] for x in pt)
    H = _scaled_chirps(n, *pt, n_det)
    return Instance(N=n, acf=acf, masks=masks, segments=None, d=d, H=H, eps=eps)


def c1_workload(eps: float = EPS_PRIMARY, B: int = 32) -> Workload:
    """Plain FP64, one detector, N = 1024, 32 templates perturbed +-10% around the injection.

    Injection: f0 = 30 Hz, tc = 0.9 T, phi0 = 1 rad, SNR 15.  Each template
    multiplies tc, phi0 and the amplitude by (1 + u), u ~ U[-0.1, 0.1].
    """
    st = _streams(0)
    n = 1024
    T = n / FS
    acf = make_acf(n, eps)
    noise = stationary_noise(st["noise"], n, 1, eps)
    h_unit = chirp(n, 30.0, 0.9 * T, 1.0, 1.0)
    a_inj = 15.0 / np.sqrt(whittle_snr2(h_unit)[0])
    d = noise + a_inj * h_unit
    u = st["templates"].uniform(-0.1, 0.1, size=(3, B))
    H = chirp(n, np.full(B, 30.0), 0.9 * T * (1 + u[0]), 1.0 * (1 + u[1]), a_inj * (1 + u[2]))
    return Workload("C1", [Instance(n, acf, [None], None, d, H, eps)])


def c2_workload(eps: float = EPS_PRIMARY, B: int = 4096, n: int = 16384, rows=None) -> Workload:
    """Two detectors x N = 16384 (4 s), independent noise, 4096 templates per launch.

    ``rows`` selects a subset of the template bank (same draws as the full bank)."""
    st = _streams(1)
    return Workload("C2", [_instance(st, n, 2, 0, B, eps, rows)])


def c3_workload(eps: float = EPS_PRIMARY, B: int = 8192, n: int = 32768, rows=None) -> Workload:
    """One detector, N = 32768 (8 s), exactly 3 gaps of 64-512 samples, 8192 templates."""
    st = _streams(2)
    return Workload("C3", [_instance(st, n, 1, 3, B, eps, rows)])


def c4_workload(eps: float = EPS_PRIMARY, n_inst: int = 64, B: int = 256,
                nmin: int = 2048, nmax: int = 32768) -> Workload:
    """64 ragged instances: N ~ U{2048..32768}, 0-2 gaps per detector, 1-2 detectors, 256 templates."""
    st = _streams(3)
    shape_rng = st["requests"]
    insts = []
    for _ in range(n_inst):
        n = int(shape_rng.integers(nmin, nmax + 1))
        n_det = int(shape_rng.integers(1, 3))
        n_gaps = int(shape_rng.integers(0, 3))
        insts.append(_instance(st, n, n_det, n_gaps, B, eps))
    return Workload("C4", insts)


def c5_workload(eps: float = EPS_PRIMARY, n_datasets: int = 32, duration_s: float = 10.0,
                rate_hz: float = 20000.0, n_walkers: int = 512,
                sizes=(4096, 8192, 16384, 32768, 65536), bank: int = 256) -> Workload:
    """32 resident single-detector datasets and a Poisson request trace.

    Dataset k has N = sizes[k mod 5].  Each request picks a dataset U{0..31},
    a template count U{1..64}, a walker U{0..511}; inter-arrival gaps are
    exponential with mean 1/rate.  Templates of a request are rows of the
    dataset's template bank (``bank`` rows, drawn like C2's templates), taken
    cyclically from a random start row.
    """
    st = _streams(4)
    insts = [_instance(st, sizes[k % len(sizes)], 1, 0, bank, eps) for k in range(n_datasets)]
    req = _requests(st["requests"], rate_hz, duration_s, n_datasets, n_walkers, bank)
    return Workload("C5", insts, req)


def _requests(r, rate_hz, duration_s, n_datasets, n_walkers, bank):
    n_req = int(rate_hz * duration_s)
    arrivals = np.cumsum(r.exponential(1.0 / rate_hz, n_req))
    return dict(t=arrivals, dataset=r.integers(0, n_datasets, n_req),
                count=r.integers(1, 65, n_req), walker=r.integers(0, n_walkers, n_req),
                start=r.integers(0, bank, n_req))


def c5_requests(rate_hz: float, duration_s: float, n_datasets: int = 32, n_walkers: int = 512,
                bank: int = 256, trace: int = 1) -> dict:
    """Another Poisson request trace over the C5 datasets (same law as c5_workload's),
    from its own seeded stream: one trace per offered load of a load sweep."""
    r = np.random.default_rng([SEED_BASE + 4, 1000 + trace])
    return _requests(r, rate_hz, duration_s, n_datasets, n_walkers, bank)


def make_workload(k: int, **kw) -> Workload:
    return [c1_workload, c2_workload, c3_workload, c4_workload, c5_workload][k](**kw)


def random_rhs_case(seed: int, n: int, n_det: int, n_gaps: int, B: int, eps: float = EPS_PRIMARY,
                    segments: Optional[List[Tuple[int, int]]] = None) -> Instance:
    """Small seeded instance for parity tests (same laws as the workloads, any size)."""
    root = np.random.default_rng(seed)
    st = dict(zip(["gaps", "noise", "injection", "templates", "requests"], root.spawn(5)))
    inst = _instance(st, n, n_det, n_gaps, B, eps)
    inst.segments = segments
    return inst
