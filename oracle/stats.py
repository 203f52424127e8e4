"""Binning error analysis and integrated autocorrelation time.  Test
infrastructure only.

* binning (the standard binning analysis named in Sec. II B): the standard
  error of the mean from bins of 2^k consecutive samples, for every k that
  leaves at least ``min_bins`` bins; the estimate is the largest value over
  the levels.
* tau_int by automatic windowing (Sokal): tau(W) = 1/2 + sum_{t=1..W} rho(t),
  W the smallest window with W >= c tau(W), c = 5.  ESS = n / (2 tau_int).
Parity unpinned by the paper (it reports no autocorrelation times); pinned in
the tests by the closed form of an AR(1) process.
"""
import numpy as np


def binning_levels(x, min_bins=16):
    x = np.asarray(x, dtype=float)
    out = []
    b = 1
    while len(x) // b >= min_bins:
        nb = len(x) // b
        m = x[:nb * b].reshape(nb, b).mean(axis=1)
        out.append((b, m.std(ddof=1) / np.sqrt(nb)))
        b *= 2
    return out


def binning_error(x, min_bins=16):
    lv = binning_levels(x, min_bins)
    if not lv:
        x = np.asarray(x, dtype=float)
        return float(x.std(ddof=1) / np.sqrt(max(len(x), 1)))
    return float(max(e for _, e in lv))


def autocorr(x):
    x = np.asarray(x, dtype=float)
    n = len(x)
    y = x - x.mean()
    f = np.fft.rfft(y, 2 * n)
    ac = np.fft.irfft(f * np.conj(f))[:n] / n
    return ac / ac[0] if ac[0] > 0 else np.zeros(n)


def tau_int(x, c=5.0):
    rho = autocorr(x)
    tau = 0.5
    for W in range(1, len(rho)):
        tau += rho[W]
        if W >= c * tau:
            return float(max(tau, 0.5))
    return float(max(tau, 0.5))


def ess(x, c=5.0):
    return len(x) / (2.0 * tau_int(x, c))


def mean_err(x):
    x = np.asarray(x, dtype=float)
    return float(x.mean()), binning_error(x)
