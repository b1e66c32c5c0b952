"""Kato-Temple bounds on the eigenvalue error of Ritz pairs whose slice
counts are exact (shared by the GPU tests at workload scale)."""
import numpy as np


def kato_temple(lam, res_abs, lo, hi):
    """Upper bounds of |lam_k - lambda| for the eigenvalue lambda nearest to
    each Ritz value (lam ascending, every eigenvalue in [lo, hi) accounted for
    by the exact counts, res_abs = ||r_k||_2; the eigenvalues outside lie
    below lo or at or above hi)."""
    out = np.full(len(lam), np.inf)
    for k in range(len(lam)):
        gaps = [lam[k] - lo if k == 0 else lam[k] - lam[k - 1] - res_abs[k - 1]]
        gaps.append(hi - lam[k] if k + 1 == len(lam) else lam[k + 1] - lam[k] - res_abs[k + 1])
        gap = min(gaps) - res_abs[k]
        if gap > 0:
            out[k] = res_abs[k] ** 2 / gap
    return out
