"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module only draws inputs (coefficient fields, sensor layouts, data,
quantity-of-interest weights); it holds none of the sampler's arithmetic.

Workloads follow the paper's experimental set-up (Sec. 5.1): unit square or
cube, homogeneous Dirichlet data, interior-node unknowns, point observations
averaged over small patches with diagonal noise covariance, and a linear
quantity of interest averaged over a central region.
"""
import numpy as np

# --------------------------------------------------------------------------
# grid helpers
# --------------------------------------------------------------------------


def sites(n, dim):
    return n ** dim


def level_ns(n, levels):
    out = [n]
    for _ in range(levels - 1):
        out.append((out[-1] - 1) // 2)
    return out[::-1]  # coarsest first


def face_midpoints(n, dim, k):
    """Coordinates of the faces normal to axis k, in the layout of the face
    arrays: axis k has n+1 entries (face between nodes f and f+1 sits at
    (f + 1/2) h), the other axes n entries (node i at i h), x fastest."""
    h = 1.0 / (n + 1)
    axes = []
    for j in range(dim):
        if j == k:
            axes.append((np.arange(n + 1) + 0.5) * h)
        else:
            axes.append(np.arange(1, n + 1) * h)
    # meshgrid with x fastest: build in reversed axis order, C-order
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    return [g for g in grids[::-1]]  # list x, y, (z), each shape (..., x)


def face_array(n, dim, log_a):
    """Concatenate a(x) = exp(log_a(x)) at the faces of every axis."""
    parts = []
    for k in range(dim):
        xs = face_midpoints(n, dim, k)
        parts.append(np.exp(log_a(*xs)).reshape(-1))
    return np.concatenate(parts)


# --------------------------------------------------------------------------
# coefficient fields
# --------------------------------------------------------------------------


def fourier_log_field(dim, nmodes=64, amplitude=1.0, max_wave=4, seed=1):
    """log a = amplitude sqrt(2/K) sum_k cos(2 pi w_k.x + phi_k), w_k uniform in
    {-W..W}^d minus 0, phi_k uniform in [0, 2 pi): pointwise std = amplitude."""
    rng = np.random.default_rng(seed)
    waves = []
    while len(waves) < nmodes:
        w = rng.integers(-max_wave, max_wave + 1, size=dim)
        if np.any(w != 0):
            waves.append(w)
    waves = np.array(waves, dtype=np.float64)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    c = amplitude * np.sqrt(2.0 / nmodes)

    def log_a(*xs):
        out = np.zeros_like(xs[0])
        for w, ph in zip(waves, phases):
            arg = ph + 2.0 * np.pi * sum(w[j] * xs[j] for j in range(dim))
            out += np.cos(arg)
        return c * out

    return log_a


def gaussian_log_field(dim, corr_len, variance, seed, nfeatures=1024):
    """Random-Fourier-feature Gaussian field with squared-exponential
    covariance variance * exp(-|r|^2 / (2 corr_len^2)):
    log a = sqrt(2 variance / K) sum_k cos(omega_k.x + phi_k), omega ~ N(0, I/corr_len^2)."""
    rng = np.random.default_rng(seed)
    omega = rng.normal(0.0, 1.0 / corr_len, size=(nfeatures, dim))
    phases = rng.uniform(0.0, 2.0 * np.pi, size=nfeatures)
    c = np.sqrt(2.0 * variance / nfeatures)

    def log_a(*xs):
        out = np.zeros_like(xs[0])
        for chunk in range(0, nfeatures, 64):
            for w, ph in zip(omega[chunk:chunk + 64], phases[chunk:chunk + 64]):
                out += np.cos(ph + sum(w[j] * xs[j] for j in range(dim)))
        return c * out

    return log_a


def lognormal_faces_fft(n, dim, corr_len, variance, seed):
    """Face coefficients a = exp(g) of a stationary Gaussian field g with
    squared-exponential covariance variance * exp(-|r|^2 / (2 corr_len^2)),
    synthesised spectrally on a periodic grid of spacing h/2 covering the
    unit cube twice over (so that the periodisation is negligible), then read
    at the face midpoints.  2D only (the 3D workloads use gaussian_log_field)."""
    if dim != 2:
        raise ValueError("spectral synthesis is provided for 2D")
    h = 1.0 / (n + 1)
    m = 4 * (n + 1)  # grid of spacing h/2 over a periodic box of side 2
    rng = np.random.default_rng(seed)
    k = np.fft.fftfreq(m, d=h / 2) * 2.0 * np.pi
    kx, ky = np.meshgrid(k, k, indexing="ij")
    # spectral density of the squared-exponential covariance in 2D
    spec = variance * 2.0 * np.pi * corr_len ** 2 * np.exp(-0.5 * corr_len ** 2 * (kx ** 2 + ky ** 2))
    box = m * (h / 2)
    amp = np.sqrt(spec / box ** 2) * m * m
    noise = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
    field = np.real(np.fft.ifft2(amp * noise))
    # grid point (a, b) sits at (a h/2, b h/2): node i at 2i, face f + 1/2 at 2f + 1
    gxy = field.T  # index [y][x]
    per = (n + 1) * n
    ax = np.exp(gxy[2 * np.arange(1, n + 1)][:, 2 * np.arange(n + 1) + 1])  # [y node][x face]
    ay = np.exp(gxy[2 * np.arange(n + 1) + 1][:, 2 * np.arange(1, n + 1)])  # [y face][x node]
    out = np.concatenate([ax.reshape(-1), ay.reshape(-1)])
    assert out.size == 2 * per
    return out


def lognormal_faces_fft3(n, corr_len, variance, seed, box=1.5):
    """3D face coefficients a = exp(g) of a stationary Gaussian field g with
    squared-exponential covariance variance * exp(-|r|^2 / (2 corr_len^2)),
    synthesised spectrally at the nodes (spacing h, periodic box of side
    `box` > 1 + a few correlation lengths), with the face value between two
    nodes exp((g_i + g_j) / 2).  Face arrays as in face_midpoints."""
    import scipy.fft
    h = 1.0 / (n + 1)
    m = int(np.ceil(box / h))
    rng = np.random.default_rng(seed)
    k = np.fft.fftfreq(m, d=h) * 2.0 * np.pi
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    # spectral density of the squared-exponential covariance in 3D
    spec = variance * (2.0 * np.pi * corr_len ** 2) ** 1.5 * np.exp(-0.5 * corr_len ** 2 * k2)
    del k2
    side = m * h
    amp = np.sqrt(spec / side ** 3) * float(m) ** 3
    del spec
    noise = rng.normal(size=(m, m, m)) + 1j * rng.normal(size=(m, m, m))
    g = np.real(scipy.fft.ifftn(amp * noise, workers=8))[: n + 2, : n + 2, : n + 2]
    del noise, amp
    g = np.ascontiguousarray(g.transpose(2, 1, 0))  # index [z][y][x], node i at i h
    inner = slice(1, n + 1)
    ax = np.exp(0.5 * (g[inner, inner, : n + 1] + g[inner, inner, 1 : n + 2]))  # [z][y][x face]
    ay = np.exp(0.5 * (g[inner, : n + 1, inner] + g[inner, 1 : n + 2, inner]))  # [z][y face][x]
    az = np.exp(0.5 * (g[: n + 1, inner, inner] + g[1 : n + 2, inner, inner]))  # [z face][y][x]
    return np.concatenate([ax.reshape(-1), ay.reshape(-1), az.reshape(-1)])


# --------------------------------------------------------------------------
# observations, data and quantity of interest
# --------------------------------------------------------------------------


def patch_sensors(n, dim, m, seed):
    """m sensors, each the mean over the 3^dim nodes centred at a node drawn
    uniformly without replacement among nodes at least 2 from the boundary.
    Returns CSR over observations (ptr[m+1], fine site index, weight)."""
    rng = np.random.default_rng(seed)
    inner = n - 2  # centres i_k in 2..n-1
    if inner < 1:
        raise ValueError("grid too small for 3-point patches")
    total = inner ** dim
    if m > total:
        raise ValueError("more sensors than admissible centres")
    flat = rng.choice(total, size=m, replace=False)
    ptr = np.zeros(m + 1, dtype=np.int64)
    idx, val = [], []
    w = 1.0 / 3 ** dim
    for j, f in enumerate(flat):
        c = []
        for _ in range(dim):
            c.append(2 + f % inner)
            f //= inner
        for t in range(3 ** dim):
            rem, lin, mult = t, 0, 1
            for k in range(dim):
                off = rem % 3 - 1
                rem //= 3
                lin += (c[k] + off - 1) * mult
                mult *= n
            idx.append(lin)
            val.append(w)
        ptr[j + 1] = len(idx)
    return ptr, np.array(idx, dtype=np.int32), np.array(val, dtype=np.float64)


def ball_sensors(n, dim, m, radius, seed):
    """m sensors, each the mean over the nodes x_i with |x_i - c_j| <= radius
    (the ball averages of Sec. 5.1.2, eq. observations, in nodal
    quadrature), centres c_j drawn uniformly in [2 radius, 1 - 2 radius]^dim.
    At a fixed radius the functional does not change with h, unlike a patch
    of a fixed number of nodes.  Returns CSR over observations."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (n + 1)
    centres = rng.uniform(2 * radius, 1 - 2 * radius, size=(m, dim))
    ptr = np.zeros(m + 1, dtype=np.int64)
    idx, val = [], []
    for j, c in enumerate(centres):
        lo = [max(1, int(np.ceil((c[k] - radius) / h))) for k in range(dim)]
        hi = [min(n, int(np.floor((c[k] + radius) / h))) for k in range(dim)]
        axes = [np.arange(lo[k], hi[k] + 1) for k in range(dim)]
        grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
        pts = np.stack([g.reshape(-1) for g in grids], axis=1)
        d2 = ((pts * h - c) ** 2).sum(axis=1)
        pts = pts[d2 <= radius ** 2]
        if len(pts) == 0:  # coarse grid: the nearest node
            pts = np.clip(np.rint(c / h), 1, n).astype(int)[None, :]
        lin = np.zeros(len(pts), dtype=np.int64)
        for k in range(dim - 1, -1, -1):
            lin = lin * n + (pts[:, k] - 1)
        order = np.argsort(lin)
        idx.extend(lin[order].tolist())
        val.extend([1.0 / len(pts)] * len(pts))
        ptr[j + 1] = len(idx)
    return ptr, np.array(idx, dtype=np.int32), np.array(val, dtype=np.float64)


def observed_values(m, seed, low=1.0, high=4.0):
    """Fixed observed values in [1, 4], as in the paper's posterior set-up."""
    return np.random.default_rng(seed).uniform(low, high, size=m)


def subcube_qoi(n, dim, lo=0.25, hi=0.75):
    """F_i = 1/count on nodes with every coordinate in [lo, hi] (inclusive)."""
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    inside = (x >= lo - 1e-12) & (x <= hi + 1e-12)
    mask = inside
    for _ in range(dim - 1):
        mask = np.multiply.outer(inside, mask)
    F = mask.astype(np.float64).reshape(-1)
    return F / F.sum()


# --------------------------------------------------------------------------
# the benchmark configurations
# --------------------------------------------------------------------------


def config(name):
    """Problem description for a named workload: grid, levels, shift, coefficient
    field, sensors and their noise, chains and QoI weights, all seeded."""
    if name == "prior63":
        n, dim = 63, 2
        return dict(name=name, dim=dim, n=n, levels=4, kappa2=100.0, face_coef=None,
                    obs=None, y=None, nchains=1, nsamples=2000, seed=0,
                    F=subcube_qoi(n, dim))
    if name == "posterior1023":
        n, dim, m = 1023, 2, 64
        face = face_array(n, dim, fourier_log_field(dim, nmodes=64, amplitude=1.0, seed=1))
        ptr, idx, val = patch_sensors(n, dim, m, seed=2)
        gamma = np.full(m, 0.01 ** 2)
        return dict(name=name, dim=dim, n=n, levels=7, kappa2=100.0, face_coef=face,
                    obs=(ptr, idx, val, gamma), y=observed_values(m, seed=3), nchains=8,
                    nsamples=10000, seed=0, F=subcube_qoi(n, dim))
    if name == "learned511":
        # learned prolongation: 511^2, lognormal a (correlation length 0.05,
        # variance 2), kappa = 1, prior; fields 0..1999 train, 2000.. held out
        n, dim = 511, 2
        return dict(name=name, dim=dim, n=n, levels=7, kappa2=1.0, corr_len=0.05, variance=2.0,
                    train_fields=2000, test_fields=200, field_seed0=1000, nchains=1,
                    nsamples=10000, burn_in=1000, seed=0, F=subcube_qoi(n, dim))
    if name == "posterior255":
        # full posterior at scale: 255^3, lognormal a (correlation length 0.1,
        # variance 1), 256 sensors averaging 3^3 nodes, Gamma = 0.005^2 I,
        # 64 chains, kappa = 1 (the paper's 3D correlation length 1/kappa = 1)
        n, dim, m = 255, 3, 256
        face = lognormal_faces_fft3(n, 0.1, 1.0, seed=4)
        ptr, idx, val = patch_sensors(n, dim, m, seed=5)
        gamma = np.full(m, 0.005 ** 2)
        return dict(name=name, dim=dim, n=n, levels=6, kappa2=1.0, face_coef=face,
                    obs=(ptr, idx, val, gamma), y=observed_values(m, seed=6), nchains=64,
                    nsamples=5000, seed=0, F=subcube_qoi(n, dim))
    if name == "batched512":
        # 512 prior chains of five shapes, kappa = 5, constant coefficient
        shapes = [(2, 127, 5, 103), (2, 255, 6, 103), (2, 511, 7, 102), (3, 63, 4, 102),
                  (3, 127, 5, 102)]
        parts = [dict(dim=d, n=n, levels=lv, kappa2=25.0, face_coef=None, obs=None, y=None,
                      nchains=c, F=subcube_qoi(n, d)) for d, n, lv, c in shapes]
        return dict(name=name, parts=parts, nsamples=5000, seed=0)
    raise KeyError(name)
