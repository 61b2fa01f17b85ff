"""Pins of the oracle's operators: fine FD matrix, prolongation, Galerkin
hierarchy, observation restriction, colouring and coarsest factor."""
import numpy as np
import pytest

import oracle
from paper_2407_12149_amd import workloads


def tridiag(n):
    return 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)


def kron_all(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def laplace_dense(n, dim):
    """h^2 (-Delta_h) as a Kronecker sum (textbook), x fastest."""
    eye = np.eye(n)
    total = 0
    for k in range(dim):
        factors = [eye] * dim
        factors[dim - 1 - k] = tridiag(n)  # kron order: last factor is x
        total = total + kron_all(factors)
    return total


@pytest.mark.parametrize("dim,n", [(2, 7), (2, 15), (3, 7)])
def test_fine_operator_constant_coefficient(dim, n):
    h = 1.0 / (n + 1)
    kappa2 = 100.0
    o = oracle.Oracle(dim, n, 1, kappa2)
    A = o.dense(0, 0)
    want = h ** dim * (kappa2 * np.eye(n ** dim) + laplace_dense(n, dim) / h ** 2)
    assert np.allclose(A, want, rtol=1e-14, atol=1e-14 * np.abs(want).max())


def difference_operator(n, dim, k):
    """Map nodal values (zero Dirichlet) to differences across the faces normal
    to axis k, in the face-array layout; D1 is (n+1) x n with rows e_{f+1}-e_f."""
    d1 = np.zeros((n + 1, n))
    for f in range(n + 1):
        if f < n:
            d1[f, f] = 1.0
        if f >= 1:
            d1[f, f - 1] = -1.0
    factors = []
    for j in range(dim - 1, -1, -1):
        factors.append(d1 if j == k else np.eye(n))
    return kron_all(factors)


@pytest.mark.parametrize("dim,n", [(2, 7), (3, 3)])
def test_fine_operator_divergence_form(dim, n):
    """A = s (kappa^2 I + h^-2 sum_k D_k^T diag(a_k) D_k): the discrete
    -div(a grad) in divergence form with face coefficients (Sec. 5.1.1)."""
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(3)
    per = (n + 1) * n ** (dim - 1)
    face = np.exp(rng.normal(size=dim * per))
    o = oracle.Oracle(dim, n, 1, 2.5, face_coef=face)
    A = o.dense(0, 0)
    want = 2.5 * np.eye(n ** dim)
    for k in range(dim):
        D = difference_operator(n, dim, k)
        want = want + D.T @ np.diag(face[k * per:(k + 1) * per]) @ D / h ** 2
    want *= h ** dim
    assert np.allclose(A, want, rtol=1e-13, atol=1e-13 * np.abs(want).max())
    assert np.allclose(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0


def test_face_layout_matches_generator():
    """workloads.face_array and the oracle agree on the face layout: a field
    a(x, y) = 1 + x gives x-face values at (f + 1/2) h."""
    n, dim = 7, 2
    face = workloads.face_array(n, dim, lambda x, y: np.log(1.0 + x + 0 * y))
    per = (n + 1) * n
    ax = face[:per].reshape(n, n + 1)
    h = 1.0 / (n + 1)
    assert np.allclose(ax[3], 1.0 + (np.arange(n + 1) + 0.5) * h)
    ay = face[per:].reshape(n + 1, n)
    assert np.allclose(ay[:, 2], 1.0 + 3 * h)


def test_prolongation_is_multilinear():
    """P = P1 (x) P1 (x) ... with the 1D linear interpolation [1/2, 1, 1/2]
    (Sec. 3.1: canonical prolongation for nested multilinear spaces)."""
    for dim, n in [(2, 15), (3, 7)]:
        o = oracle.Oracle(dim, n, 2, 1.0)
        nc = (n - 1) // 2
        p1 = np.zeros((n, nc))
        for j in range(nc):
            p1[2 * j + 1, j] = 1.0
            p1[2 * j, j] = 0.5
            p1[2 * j + 2, j] = 0.5
        want = kron_all([p1] * dim)
        assert np.array_equal(o.dense(1, 1), want)


@pytest.mark.parametrize("dim,n,levels", [(2, 15, 3), (3, 7, 2)])
def test_galerkin_hierarchy(dim, n, levels):
    """A_{l-1} = P^T A_l P and B_{l-1} = P^T B_l (eq. A_ell_1_B_ell_1), coarse
    stencils at most 3^dim wide, all symmetric positive definite."""
    rng = np.random.default_rng(1)
    per = (n + 1) * n ** (dim - 1)
    face = np.exp(rng.normal(size=dim * per))
    o = oracle.Oracle(dim, n, levels, 4.0, face_coef=face)
    ptr, idx, val = workloads.patch_sensors(n, dim, 3, seed=4)
    o.set_obs(ptr, idx, val, np.full(3, 1e-3))
    for l in range(levels - 1, 0, -1):
        A = o.dense(l, 0)
        P = o.dense(l, 1)
        Ac = o.dense(l - 1, 0)
        assert np.allclose(Ac, P.T @ A @ P, rtol=1e-13, atol=1e-13 * np.abs(Ac).max())
        assert np.allclose(o.dense(l - 1, 2), P.T @ o.dense(l, 2), atol=1e-15)
        assert (np.count_nonzero(Ac, axis=1) <= 3 ** dim).all()
        assert np.linalg.eigvalsh(Ac).min() > 0
    # At_l = A_l + B_l Gamma^-1 B_l^T on every level
    for l in range(levels):
        B = o.dense(l, 2)
        assert np.allclose(o.dense(l, 6), o.dense(l, 0) + B @ B.T / 1e-3)


def test_observation_matrix_is_patch_mean():
    n, dim = 15, 2
    ptr, idx, val = workloads.patch_sensors(n, dim, 5, seed=9)
    o = oracle.Oracle(dim, n, 2, 1.0)
    o.set_obs(ptr, idx, val, np.ones(5))
    B = o.dense(1, 2)
    assert np.allclose(B.sum(axis=0), 1.0)
    assert ((B > 0).sum(axis=0) == 9).all()


@pytest.mark.parametrize("dim,n,levels", [(2, 15, 3), (3, 7, 2)])
def test_colouring_decouples(dim, n, levels):
    """Sites of one colour never couple, on every level (5/7-point fine and
    9/27-point Galerkin stencils alike)."""
    o = oracle.Oracle(dim, n, levels, 1.0)
    for l in range(levels):
        A = o.dense(l, 0)
        col = o.dense(l, 7)
        same = col[:, None] == col[None, :]
        np.fill_diagonal(same, False)
        assert not np.any(A[same] != 0.0)
        # colour is the parity vector of the 1-based coordinates
        nl = o.level_n(l)
        idx = np.arange(nl ** dim)
        want = np.zeros_like(idx)
        for k in range(dim):
            ik = (idx // nl ** k) % nl + 1
            want |= (ik & 1) << k
        assert np.array_equal(col.astype(int), want)


def test_coarse_cholesky_factor():
    n, dim = 15, 2
    o = oracle.Oracle(dim, n, 2, 3.0)
    ptr, idx, val = workloads.patch_sensors(n, dim, 4, seed=1)
    o.set_obs(ptr, idx, val, np.full(4, 0.01))
    U = o.dense(0, 5)
    assert np.allclose(np.tril(U, -1), 0.0)
    At0 = o.dense(0, 6)
    assert np.allclose(U.T @ U, At0, rtol=1e-13, atol=1e-13 * np.abs(At0).max())


def test_invalid_problems_rejected():
    with pytest.raises(ValueError):
        oracle.Oracle(2, 10, 2, 1.0)  # n not 2^k - 1
    with pytest.raises(ValueError):
        oracle.Oracle(4, 7, 2, 1.0)
    with pytest.raises(ValueError):
        oracle.Oracle(2, 7, 4, 1.0)  # too many levels
    with pytest.raises(ValueError):
        oracle.Oracle(2, 7, 2, -1e4)  # not SPD -> Cholesky fails
