"""The free-streaming kernel I(x) (eq. (I.def), Appendix C), FP64.

I(X) is the Fourier transform of the unperturbed momentum distribution, normalised so
that I(0) = 1; for relic neutrinos it depends only on x = X T_nu0 with X = k (s - s')/m.
The method uses the rational fit of Appendix C, eq. (fit); the paper states that the exact
function gives the same results. The exact alternating series of Appendix C is kept here
only so that tests can pin the fit against it.
"""
import numpy as np

from .background import ZETA3


def I_fit(x):
    """eq. (fit): (1 + 0.0168 x^2 + 0.0407 x^4) / (1 + 2.1734 x^2 + 1.6787 x^4.1811 + 0.1467 x^8)."""
    x = np.asarray(x, dtype=np.float64)
    x2 = x * x
    num = 1.0 + 0.0168 * x2 + 0.0407 * x2 * x2
    den = 1.0 + 2.1734 * x2 + 1.6787 * np.power(x, 4.1811) + 0.1467 * x2 ** 4
    return num / den


def I_series(x, n_terms=4000):
    """Exact I(x) = 4/(3 zeta(3)) sum_{n>=1} (-1)^{n+1} n/(n^2+x^2)^2 (Appendix C).

    The alternating tail is summed with the average of two consecutive partial sums,
    which for this monotone series brings the truncation error to O(N^-4).
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = np.arange(1, n_terms + 2, dtype=np.float64)[:, None]
    terms = np.where(n % 2 == 1, 1.0, -1.0) * n / (n * n + x[None, :] ** 2) ** 2
    partial = np.cumsum(terms, axis=0)
    s = 0.5 * (partial[-1] + partial[-2])
    return 4.0 / (3.0 * ZETA3) * s
