"""Comparison rules shared by the GPU parity tests.

Tolerance on the per-variable measure M_i = -k_i of one step (teacher-forced,
so the oracle and the GPU see the same residual data):

    |M_gpu - M_ref| <= 1e-4 * max(|M_ref|, s_t),   s_t = 1e-3 * max_k |M_ref,k|

(1e-4 relative, with a floor at 1e-3 of the step's largest measure because the
most exogenous candidates can have M = 0 exactly).  The GPU's choice must be
the oracle's argmax unless the oracle's best-versus-runner-up gap is within
2e-4 * max(k_(2), s_t) (a near-tie, where either choice is accepted).
"""
import numpy as np

REL = 1e-4
FLOOR = 1e-3


def measure_close(m_gpu, m_ref):
    """Boolean mask of entries within tolerance (arrays over active variables)."""
    m_gpu = np.asarray(m_gpu, dtype=np.float64)
    m_ref = np.asarray(m_ref, dtype=np.float64)
    s_t = FLOOR * np.max(np.abs(m_ref)) if m_ref.size else 0.0
    return np.abs(m_gpu - m_ref) <= REL * np.maximum(np.abs(m_ref), s_t)


def near_tie(m_ref, a, b):
    """True when the oracle cannot tell columns a and b apart at the tolerance."""
    m_ref = np.asarray(m_ref, dtype=np.float64)
    fin = m_ref[np.isfinite(m_ref)]
    s_t = FLOOR * np.max(np.abs(fin)) if fin.size else 0.0
    ka, kb = -m_ref[a], -m_ref[b]
    return abs(ka - kb) <= 2 * REL * max(max(ka, kb), s_t)


def check_step(meas_gpu_row, meas_ref_row, chosen):
    """Check one step (rows indexed by original id, NaN = inactive).

    Returns (n_bad_measures, choice_ok)."""
    act = np.isfinite(meas_ref_row)
    assert np.array_equal(act, np.isfinite(meas_gpu_row)), "active sets differ"
    ids = np.flatnonzero(act)
    close = measure_close(meas_gpu_row[ids], meas_ref_row[ids])
    ref_best = ids[np.argmax(meas_ref_row[ids])]
    choice_ok = chosen == ref_best or near_tie(meas_ref_row, chosen, ref_best)
    return int((~close).sum()), bool(choice_ok)


# The library's FP64 tie resolution: at an FP32-path step, when 2..16 active
# variables have k <= k_best (1 + 4e-3) + 1e-12 (k = -M from the FP32
# measures), the choice among them is made from their k recomputed in FP64.
TIE_REL, TIE_ABS, TIE_MAX = 4e-3, 1e-12, 16


def choice_ok(row, chosen):
    """(ok, resolved): the chosen variable is the step's FP32 argmax (ties to
    the smallest id), or the step is a near-tie the FP64 resolution decided
    and the choice lies within its band.  row: measures by original id (NaN =
    inactive)."""
    ids = np.flatnonzero(np.isfinite(row))
    best = row[ids].max()
    first = ids[np.flatnonzero(row[ids] == best)[0]]
    if chosen == first:
        return True, False
    lim = -best * (1.0 + TIE_REL) + TIE_ABS
    band = ids[-row[ids] <= lim]
    return (2 <= band.size <= TIE_MAX and chosen in band), True
