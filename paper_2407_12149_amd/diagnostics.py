"""Chain diagnostics: integrated autocorrelation time and effective sample rate.

The integrated autocorrelation time (IACT) follows the paper's normalisation
tau = 1 + 2 sum_{t>=1} rho(t) (Sec. 4.3, eq. tau_int_definition), estimated with
Wolff's automatic windowing (U. Wolff, "Monte Carlo errors with less errors",
Comput. Phys. Commun. 156 (2004), Sec. 3.3), as the paper does in Sec. 5.3.2.
Wolff states his estimate as 1/2 + sum rho, i.e. half of the paper's value.
"""
import numpy as np


def autocovariance(z):
    """Gamma(t) = 1/(N-t) sum_m (z_m - zbar)(z_{m+t} - zbar), t = 0..N-1 (Sec. 5.3.2)."""
    z = np.asarray(z, dtype=np.float64)
    n = z.size
    d = z - z.mean()
    size = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(d, size)
    acf = np.fft.irfft(f * np.conj(f), size)[:n]
    return acf / (n - np.arange(n))


def iact_wolff(z, stau=1.5):
    """Return (tau, dtau, W): IACT in the paper's normalisation, its error
    estimate tau * sqrt(2 (2W+1)/N), and the summation window W."""
    z = np.asarray(z, dtype=np.float64)
    n = z.size
    if n < 4:
        raise ValueError("series too short")
    gamma = autocovariance(z)
    if gamma[0] <= 0.0:
        return 1.0, 0.0, 0
    rho = gamma / gamma[0]
    tint = 0.5
    window = n - 1
    for w in range(1, n):
        tint += rho[w]
        if tint <= 0.5:
            window = w
            break
        tau_w = stau / np.log((2.0 * tint + 1.0) / (2.0 * tint - 1.0))
        g = np.exp(-w / tau_w) - tau_w / np.sqrt(w * n)
        if g < 0.0:
            window = w
            break
    tint = 0.5 + rho[1:window + 1].sum()
    tau = 2.0 * tint
    dtau = tau * np.sqrt(2.0 * (2 * window + 1) / n)
    return float(tau), float(dtau), int(window)


def effective_samples_per_second(nsamples, nchains, seconds, tau):
    """ESS/s = samples x chains / (tau x wall time): the inverse of the paper's
    time per independent sample (Sec. 5.2)."""
    return nsamples * nchains / (tau * seconds)
