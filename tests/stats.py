"""Statistical comparison helpers for the tests (3-sigma rule with a
multiple-comparison allowance)."""
import numpy as np
from scipy import stats as _st


def allowed_failures(n_bins: int, p_fail: float = 0.0027, quantile: float = 0.999) -> int:
    """Number of bins allowed outside 3 sigma: the 99.9 % quantile of
    Binomial(n_bins, 0.0027)."""
    return int(_st.binom.ppf(quantile, n_bins, p_fail))


def three_sigma(m1, s1, m2=None, s2=None, truth=None, min_sigma=0.0, dof=None):
    """Per-bin |m1 - m2| <= 3 sqrt(s1^2 + s2^2) (or against an exact ``truth``).
    dof: the standard errors come from that many degrees of freedom (batches
    - 1), so a bin's z follows Student's t and the allowance uses its tail
    P(|t| > 3) instead of the normal 0.0027.  Returns (n_fail, n_allowed,
    worst z)."""
    m1 = np.asarray(m1, float)
    s1 = np.asarray(s1, float)
    if truth is not None:
        diff = m1 - np.asarray(truth, float)
        sig = s1
    else:
        diff = m1 - np.asarray(m2, float)
        sig = np.sqrt(s1 ** 2 + np.asarray(s2, float) ** 2)
    sig = np.maximum(sig, min_sigma)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = np.where(sig > 0, np.abs(diff) / sig, np.where(diff == 0, 0.0, np.inf))
    n_fail = int(np.sum(z > 3.0))
    p_fail = 0.0027 if dof is None else float(2.0 * _st.t.sf(3.0, dof))
    return n_fail, allowed_failures(z.size, p_fail), float(np.max(z)) if z.size else 0.0
