"""Seeded synthetic inputs shaped like the paper's workloads.

This module builds *inputs only*: the noise autocorrelation (ACF) from an
analytic one-sided PSD, stationary Gaussian noise with that ACF, chirp
templates, gap masks and the five benchmark workloads.  It contains none of
the likelihood arithmetic (no covariance factorisation, no triangular solve,
no quadratic form), so it can feed both the FP64 reference implementation in
``oracle/`` and the HIP library without coupling them.

Readings of under-specified points are fixed here once (see the docstrings):
the PSD grid and regularisation nugget, the noise law, the chirp phase and
cut-off, the SNR convention for template amplitudes and the gap law.
"""
from .workloads import (  # noqa: F401
    FS, PSD_GRID, EPS_PRIMARY, EPS_STRESS, SEED_BASE,
    analytic_psd, make_acf, eig_bounds, stationary_noise, chirp, whittle_snr2,
    draw_gaps, gap_mask_from, Instance, Workload, make_workload,
    c1_workload, c2_workload, c3_workload, c4_workload, c5_workload, c5_requests,
    random_rhs_case,
)
