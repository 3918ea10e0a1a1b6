"""Autocorrelation statistics of Markov-chain measurement series (test infrastructure only).

tau_int with Sokal's automatic windowing (Madras & Sokal, J. Stat. Phys. 50,
109 (1988)): rho(t) = C(t)/C(0) with C(t) = (1/n) sum_{s=0}^{n-1-t} d_s d_{s+t},
d the deviations from the chain mean; tau(M) = 1/2 + sum_{t=1}^{M} rho(t);
the window M is the smallest with M >= c tau(M).  The standard error of the
mean over chains treats chains as independent, each with variance
C(0) 2 tau / n.

Pinned by the AR(1) closed form tau_int = (1 + phi) / (2 (1 - phi)) and by
i.i.d. data (tau_int = 1/2).
"""
import numpy as np


def tau_int(series, c=5.0):
    x = np.asarray(series, dtype=np.float64)
    n = len(x)
    d = x - x.mean()
    c0 = float(d @ d) / n
    tau = 0.5
    if c0 == 0.0:
        return tau
    for M in range(1, n):
        tau += float(d[:n - M] @ d[M:]) / n / c0
        if M >= c * tau:
            break
    return tau


def chain_stats(series2d, c=5.0):
    x = np.asarray(series2d, dtype=np.float64)
    taus = np.array([tau_int(row, c) for row in x])
    n = x.shape[1]
    var = np.array([np.mean((row - row.mean()) ** 2) for row in x])
    err = np.sqrt(np.sum(var * 2 * taus / n)) / x.shape[0]
    return taus, float(x.mean(axis=1).mean()), float(err)
