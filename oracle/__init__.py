"""FP64 CPU reference implementation of the time-domain Gaussian log-likelihood.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links or
executes this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; both sides receive the same seeded inputs from ``synth``.

Contents
  tdlik  -- the plain definition: Toeplitz covariance restricted to retained
            samples of each segment, FP64 Cholesky, triangular solve, log-det
            and the full log-likelihood with its constant.
  gsce   -- an independent route for gap-free Toeplitz blocks: Levinson-Durbin
            recursion (C x = e1 and log det) and the Gohberg-Semencul quadratic
            form evaluated with circulant-embedded FFT Toeplitz products.
  snr    -- matched-filter and effective SNR from the same inner product.
  acf    -- autocovariance estimates from strain: direct correlation, and a
            Welch PSD followed by its inverse Fourier transform.

Pinning: every function here is checked by ``tests/test_oracle_pins.py``
against closed forms (white noise, AR(1), gapped AR(1)), brute force at 50
digits for N <= 48, Leibniz determinants for N <= 6, the independent
Levinson/Gohberg-Semencul route and statistical properties of whitened noise.
"""
from .tdlik import (  # noqa: F401
    LOG2PI, retained_indices, segment_covariance, Factor, factor, whiten,
    loglik, loglik_network, quad_forms,
)
from . import acf, gsce, snr  # noqa: F401
