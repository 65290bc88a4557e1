"""Time-series statistics for Monte Carlo observables (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle.py``).

Thermal averages over the measurement phase follow the paper's Monte Carlo
paragraph (equilibrate, then average) and Eq. (2) (magnetisation per spin).
Error bars use the blocking transformation of Flyvbjerg and Petersen
(J. Chem. Phys. 91, 461 (1989)): pairwise averaging of the series until the
variance-of-the-mean estimate stops growing.
"""
from __future__ import annotations

import numpy as np


def blocking_error(x) -> float:
    """Standard error of the mean of a correlated series by repeated pairwise
    blocking; the estimate is the maximum over levels with at least 32 blocks
    (a conservative plateau)."""
    x = np.asarray(x, dtype=np.float64)
    best = 0.0
    while x.size >= 32:
        n = x.size
        var = x.var(ddof=1) if n > 1 else 0.0
        err = np.sqrt(var / n)
        best = max(best, err)
        m = n // 2
        x = 0.5 * (x[0:2 * m:2] + x[1:2 * m:2])
    if best == 0.0 and x.size > 1:
        best = float(np.sqrt(x.var(ddof=1) / x.size))
    return float(best)


def binder_jackknife_error(m2, m4, n_blocks: int = 32) -> float:
    """Error of U4 = 1 - <m^4>/(3 <m^2>^2) by the delete-one-block jackknife
    (Efron 1982; blocks long compared with the autocorrelation time):
    B = min(n_blocks, n) contiguous blocks, record i in block floor(B i / n);
    U4 re-evaluated with each block left out; error^2 = (B-1)/B * sum of
    squared deviations of those values from their mean."""
    m2 = np.asarray(m2, dtype=np.float64)
    m4 = np.asarray(m4, dtype=np.float64)
    n = m2.size
    B = min(n_blocks, n)
    if B < 2:
        return 0.0
    block = (np.arange(n, dtype=np.int64) * B) // n
    u = np.empty(B)
    for b in range(B):
        keep = block != b
        u[b] = 1.0 - m4[keep].mean() / (3.0 * m2[keep].mean() ** 2)
    return float(np.sqrt((B - 1) / B * np.sum((u - u.mean()) ** 2)))


def series_summary(records, n_sites: int, T: float):
    """From per-sweep records (rows {Mx, My, Mz (sums), E_exch, E_anis, ...})
    compute means and blocked errors of |m|, m^2, m^4, E/N and the derived
    Binder cumulant U4 = 1 - <m^4>/(3 <m^2>^2), specific heat and
    susceptibility (fluctuation formulas, k_B = 1)."""
    r = np.asarray(records, dtype=np.float64)
    m_vec = r[:, 0:3] / n_sites
    m2 = np.einsum("ij,ij->i", m_vec, m_vec)
    mabs = np.sqrt(m2)
    m4 = m2 * m2
    E = r[:, 3] + r[:, 4]
    e = E / n_sites
    out = {}
    for name, s in (("abs_m", mabs), ("m2", m2), ("m4", m4), ("e", e)):
        out[name] = float(s.mean())
        out[name + "_err"] = blocking_error(s)
    out["U4"] = 1.0 - out["m4"] / (3.0 * out["m2"] ** 2)
    out["U4_err"] = binder_jackknife_error(m2, m4)
    if T > 0 and np.isfinite(T):
        out["C"] = float((np.mean(E * E) - np.mean(E) ** 2) / (n_sites * T * T))
        out["chi"] = float(n_sites * (out["m2"] - out["abs_m"] ** 2) / T)
    return out
