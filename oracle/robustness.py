"""Force-outlier count of one configuration (test oracle).

Test infrastructure only. The paper measures the robustness of a model by the
number of force values that lie more than five standard deviations from the
rest during a simulation (Sec. 1, Fig. 1; Sec. 3.2). It gives no formula; this
project's reading (R20): over the 3N force components F_k of one
configuration, the mean mu and the population standard deviation sigma
(divisor 3N); an outlier is a component with |F_k - mu| > nsigma * sigma.
"""
from __future__ import annotations

import numpy as np


def force_outliers(forces, nsigma: float = 5.0) -> int:
    """Number of components of forces[N, 3] farther than nsigma sigma from the mean."""
    f = np.asarray(forces, dtype=np.float64).reshape(-1)
    mu = f.mean()
    sigma = np.sqrt(((f - mu) ** 2).mean())
    return int(np.count_nonzero(np.abs(f - mu) > nsigma * sigma))
