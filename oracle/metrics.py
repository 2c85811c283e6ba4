"""Error metrics and exact sums (TEST INFRASTRUCTURE)."""
import math

import numpy as np


def l1_error(numerical, averaged_exact, dV):
    """L1 = dV * sum_i |N_i - <A(x_i)>| (paper section 3, equation "l1_error")."""
    return float(dV * np.abs(np.asarray(numerical) - np.asarray(averaged_exact)).sum())


def fitted_order(ns, errs):
    """Least-squares slope of log(err) against log(1/n)."""
    x = np.log(1.0 / np.asarray(ns, dtype=np.float64))
    y = np.log(np.asarray(errs, dtype=np.float64))
    return float(np.polyfit(x, y, 1)[0])


def exact_sum(a):
    """Correctly rounded sum of all entries (math.fsum)."""
    return math.fsum(np.asarray(a, dtype=np.float64).ravel().tolist())


def field_rel_linf(gpu, ref):
    """max|g - o| / max|o| (normwise relative L-infinity)."""
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max()
    return float(np.abs(np.asarray(gpu, dtype=np.float64) - ref).max() / den) if den > 0 else \
        float(np.abs(np.asarray(gpu, dtype=np.float64)).max())


def field_rel_l1(gpu, ref):
    """sum|g - o| / sum|o| (relative L1 over the whole field)."""
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).sum()
    num = np.abs(np.asarray(gpu, dtype=np.float64) - ref).sum()
    return float(num / den) if den > 0 else float(num)
