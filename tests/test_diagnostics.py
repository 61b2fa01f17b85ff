"""Pins of the IACT estimator (Wolff automatic windowing, paper normalisation)."""
import numpy as np

from paper_2407_12149_amd import diagnostics


def ar1(phi, n, seed):
    rng = np.random.default_rng(seed)
    e = rng.normal(size=n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - phi ** 2)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    return x


def test_iact_of_ar1_matches_closed_form():
    """AR(1) with coefficient phi has rho(t) = phi^t, so tau = 1 + 2 sum phi^t
    = (1 + phi)/(1 - phi)."""
    for phi, seed in [(0.0, 1), (0.3, 2), (0.6, 3), (0.9, 4)]:
        x = ar1(phi, 200_000, seed)
        tau, dtau, window = diagnostics.iact_wolff(x)
        want = (1 + phi) / (1 - phi)
        assert abs(tau - want) < 4 * dtau + 0.01, (phi, tau, want, dtau)
        assert window >= 1


def test_autocovariance_definition():
    rng = np.random.default_rng(0)
    z = rng.normal(size=257)
    g = diagnostics.autocovariance(z)
    d = z - z.mean()
    for t in (0, 1, 5, 100, 256):
        assert np.isclose(g[t], (d[: z.size - t] * d[t:]).sum() / (z.size - t))


def test_ess_rate():
    assert diagnostics.effective_samples_per_second(1000, 8, 2.0, 1.25) == 3200.0
