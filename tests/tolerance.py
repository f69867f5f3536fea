"""FP64 comparison bound shared by the GPU tests (no likelihood arithmetic).

Two FP64 evaluations of logL = -q/2 + const differ through the rounding of the
factorisation and of the solve.  A backward-stable Cholesky solve computes the exact
quadratic form of a perturbed covariance C + dC with |dC| <= c u |C|, which moves
q = r^T C^-1 r by at most c u kappa(C) q (first order).  logL moves by half of that
on each side, so two evaluations differ by at most c u kappa(C) q; c = 1 is used (the
n-dependence of the worst-case backward-error constant is not seen in practice), plus
1e-6 absolute for the summation order of the constant terms.  kappa(C) is bounded by
the input's eigenvalue range (synth.eig_bounds for the synthetic ACFs), q is the
oracle's quadratic form summed over detectors.
"""
import numpy as np

U = 2.0 ** -53          # FP64 unit roundoff
ABS = 1e-6              # summation order of log det and the constant
LOG2PI = np.log(2.0 * np.pi)


def kappa_synth(eps):
    import synth
    lo, hi = synth.eig_bounds(eps)
    return hi / lo


def kappa_exact(acf, n):
    """Condition number of toeplitz(acf[:n]) by eigenvalues (small n only)."""
    import scipy.linalg
    ev = np.linalg.eigvalsh(scipy.linalg.toeplitz(np.asarray(acf)[:n]))
    return float(ev[-1] / ev[0])


def q_of(loglik, factors):
    """Quadratic forms behind oracle log-likelihoods: q = -2 (logL - sum of constants)."""
    c = sum(-0.5 * f.logdet - 0.5 * f.n_eff * LOG2PI for f in factors)
    return -2.0 * (np.asarray(loglik) - c)


def tol_f64(q, kappa, scale=1.0):
    """|dlogL| bound between two FP64 evaluations (scale = 10 for the less stable forms:
    Gohberg-Semencul's difference of two quadratic forms and the explicit inverse)."""
    return scale * (ABS + kappa * U * np.abs(q))


def tol_terms(q, dh, hh, kappa, scale=1.0):
    """Bound for the inner products <d,h>, <h,h> of two FP64 evaluations: both come from
    quadratic forms of r = d - h, of h and of d (q, <h,h>, <d,d> = q + 2<d,h> - <h,h>),
    each with the bound above."""
    q, dh, hh = (np.abs(np.asarray(x)) for x in (q, dh, hh))
    return tol_f64(q + (q + 2.0 * dh + hh) + hh, kappa, scale)
