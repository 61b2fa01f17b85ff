"""Input generators: the 3D log-normal coefficient and the sensor layout of
the posterior workloads (host only)."""
import numpy as np

from paper_2407_12149_amd import workloads


def test_lognormal_faces_3d_layout_and_statistics():
    """Face arrays of the three axes in the face_midpoints layout; log a has
    the requested variance and a correlation that decays like the
    squared-exponential covariance exp(-r^2 / (2 l^2))."""
    n, corr, var = 31, 0.1, 1.0
    logs = []
    for seed in range(6):
        face = workloads.lognormal_faces_fft3(n, corr, var, seed=seed)
        assert face.shape == (3 * (n + 1) * n * n,)
        assert np.all(face > 0)
        logs.append(np.log(face[: (n + 1) * n * n].reshape(n, n, n + 1)))  # x faces [z][y][x]
    g = np.stack(logs)
    # variance of the face values (means of two node values at distance h:
    # var * (1 + rho(h)) / 2, with rho(h) = exp(-h^2 / (2 l^2)))
    h = 1.0 / (n + 1)
    expect = var * (1.0 + np.exp(-h * h / (2 * corr * corr))) / 2.0
    assert abs(g.var() / expect - 1.0) < 0.25
    # correlation at lag 3 faces along x against the model (same averaging
    # on both sides cancels to first order)
    a, b = g[..., :-3].ravel(), g[..., 3:].ravel()
    rho = np.corrcoef(a, b)[0, 1]
    model = np.exp(-(3 * h) ** 2 / (2 * corr * corr))
    assert abs(rho - model) < 0.1


def test_lognormal_faces_3d_seeded():
    a = workloads.lognormal_faces_fft3(15, 0.1, 1.0, seed=3)
    b = workloads.lognormal_faces_fft3(15, 0.1, 1.0, seed=3)
    c = workloads.lognormal_faces_fft3(15, 0.1, 1.0, seed=4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_patch_sensors_3d_are_volume_means():
    n, m = 15, 10
    ptr, idx, val = workloads.patch_sensors(n, 3, m, seed=5)
    assert ptr.shape == (m + 1,) and ptr[-1] == 27 * m
    assert np.allclose(val, 1.0 / 27)
    for j in range(m):
        sites = idx[ptr[j]:ptr[j + 1]]
        x, y, z = sites % n, (sites // n) % n, sites // (n * n)
        # a 3 x 3 x 3 block of distinct nodes inside the grid
        assert len(set(sites.tolist())) == 27
        for c in (x, y, z):
            assert c.max() - c.min() == 2 and c.min() >= 0 and c.max() <= n - 1


def test_operator_weights_reduce_to_multilinear():
    """The operator-dependent transfer of learned.operator_weights equals
    multilinear interpolation for a = 1 and kappa = 0 (the collapsed 5-point
    stencil of -Laplace gives 1/2 on edges and 1/4 at cell centres), and
    stays a convex-like weighting for a rough log-normal field."""
    from paper_2407_12149_amd import learned
    n = 31
    cfg = dict(n=n, kappa2=0.0)
    face = workloads.face_array(n, 2, lambda x, y: 0.0 * x)
    w = learned.operator_weights(cfg, face).reshape(-1, 9)
    ml = np.array([0.25, 0.5, 0.25, 0.5, 1.0, 0.5, 0.25, 0.5, 0.25])
    assert np.abs(w - ml).max() <= 1e-15
    rough = workloads.lognormal_faces_fft(n, 2, 0.05, 2.0, seed=3)
    w = learned.operator_weights(dict(n=n, kappa2=1.0), rough).reshape(-1, 9)
    assert np.all(w > 0) and np.all(w <= 1.0 + 1e-12)
