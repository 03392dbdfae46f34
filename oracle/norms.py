"""Error norms of Sec. VI (oracle, test infrastructure only).

relative_norms: eq. (relative_norms), L1 = sum|e| / sum|s_ana|,
L2 = sqrt(sum e^2) / sqrt(sum s_ana^2), Linf = max|e| / max|s_ana|.
absolute_norms: eq. (norms), for an analytic field that is zero everywhere.
"""
import numpy as np


def relative_norms(s_num, s_ana):
    s_num = np.asarray(s_num, dtype=np.float64)
    s_ana = np.asarray(s_ana, dtype=np.float64)
    e = s_num - s_ana
    return (
        np.sum(np.abs(e)) / np.sum(np.abs(s_ana)),
        np.sqrt(np.sum(e * e)) / np.sqrt(np.sum(s_ana * s_ana)),
        np.max(np.abs(e)) / np.max(np.abs(s_ana)),
    )


def absolute_norms(e):
    e = np.asarray(e, dtype=np.float64)
    return np.sum(np.abs(e)), np.sqrt(np.sum(e * e)), np.max(np.abs(e))
