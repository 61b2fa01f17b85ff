"""Pins of the learned-prolongation reference (oracle/pnet.py)."""
import numpy as np
from scipy import signal

import oracle
from oracle import pnet
from paper_2407_12149_amd import workloads


def test_equal_outputs_give_multilinear_prolongation():
    """softplus(o) = 1 everywhere reproduces the multilinear P of the C oracle."""
    n, nc = 15, 7
    o = np.full((9, nc, nc), np.log(np.expm1(1.0)))
    w = pnet.normalize(o, nc)
    ref = oracle.Oracle(2, n, 2, 1.0).dense(1, 1)  # fine x coarse
    P = np.zeros((n * n, nc * nc))
    for Jy in range(1, nc + 1):
        for Jx in range(1, nc + 1):
            for t in range(9):
                dx, dy = t % 3 - 1, t // 3 - 1
                P[(2 * Jx + dx - 1) + n * (2 * Jy + dy - 1), (Jx - 1) + nc * (Jy - 1)] = w[Jy - 1, Jx - 1, t]
    assert np.allclose(P, ref, atol=1e-15)


def test_partition_of_unity_with_ghosts():
    rng = np.random.default_rng(0)
    nc = 7
    o = rng.normal(size=(9, nc, nc))
    w = pnet.normalize(o, nc)
    n = 2 * nc + 1
    rows = np.zeros((n + 2, n + 2))
    for Jy in range(1, nc + 1):
        for Jx in range(1, nc + 1):
            for t in range(9):
                dx, dy = t % 3 - 1, t // 3 - 1
                rows[2 * Jy + dy, 2 * Jx + dx] += w[Jy - 1, Jx - 1, t]
    # interior fine nodes away from the boundary receive weights summing to 1
    assert np.allclose(rows[2:n, 2:n], 1.0)
    assert (w > 0).all()


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(3, 6, 5))
    W = rng.normal(size=(2, 3, 9))
    b = rng.normal(size=2)
    out = pnet.conv3x3(X, W, b)
    for o in range(2):
        want = b[o] + sum(signal.correlate2d(X[c], W[o, c].reshape(3, 3), mode="same") for c in range(3))
        assert np.allclose(out[o], want)


def test_features_of_a_smooth_field():
    """log a = x + 2 y: every feature is the face midpoint's x + 2 y."""
    n = 15
    nc = 7
    h = 1.0 / (n + 1)
    faces = workloads.face_array(n, 2, lambda x, y: x + 2 * y)
    X = pnet.features(faces, n)
    Jx, Jy = 3, 5
    # channel 0: x-face 2Jx-2 (at (2Jx-2+1/2) h) in fine row 2Jy-1
    assert np.isclose(X[0, Jy - 1, Jx - 1], (2 * Jx - 1.5) * h + 2 * (2 * Jy - 1) * h)
    # channel 12: y-face 2Jy-2 (at (2Jy-1.5) h) in fine column 2Jx-1
    assert np.isclose(X[12, Jy - 1, Jx - 1], (2 * Jx - 1) * h + 2 * (2 * Jy - 1.5) * h)
    assert X.shape == (24, nc, nc)


def crop_problem(seed=3, n=31):
    faces = workloads.lognormal_faces_fft(n, 2, 0.1, 1.0, seed=seed)
    rng = np.random.default_rng(seed)
    errors = rng.normal(size=(2, n * n))
    return faces, errors


def test_coarse_correction_alone_is_the_missed_energy_fraction():
    """Without smoothers: L = 1 - g^T A_c^{-1} g / e^T A e, in (0, 1), and 0
    for errors in the range of P (T is the A-orthogonal projector onto the
    complement of range(P))."""
    n, nc, cw = 31, 15, 15
    faces, errors = crop_problem()
    rng = np.random.default_rng(4)
    w = pnet.normalize(rng.normal(size=(9, nc, nc)), nc)
    loss, _ = pnet.crop_loss_grad(faces, n, 1.0, w, errors, [(1, 1)], cw, smooth=False)
    A = pnet.fine_operator_dense(faces, n, 1.0, 1, 1, 2 * cw + 1)
    P = pnet.crop_prolongation(w, 1, 1, cw)
    want = 0.0
    for e in errors:
        g = P.T @ A @ e
        want += 1.0 - g @ np.linalg.solve(P.T @ A @ P, g) / (e @ A @ e)
    assert abs(loss - want / len(errors)) <= 1e-12 and 0.0 < loss < 1.0
    v = rng.normal(size=cw * cw)
    e = np.zeros((n, n))
    e[0:2 * cw + 1, 0:2 * cw + 1] = (P @ v).reshape(2 * cw + 1, 2 * cw + 1)
    l0, _ = pnet.crop_loss_grad(faces, n, 1.0, w, [e.reshape(-1)], [(1, 1)], cw, smooth=False)
    assert abs(l0) < 1e-12


def test_red_black_sweeps_are_the_gauss_seidel_splitting():
    """The sweep equals I - M^{-1} A with M the lower triangle of A in
    red-then-black order (textbook Gauss-Seidel), the backward sweep is the
    A-adjoint of the forward one, and both contract in the A-norm."""
    n, cw = 31, 15
    faces, errors = crop_problem()
    fw = 2 * cw + 1
    A = pnet.fine_operator_dense(faces, n, 1.0, 1, 1, fw)
    red, black = pnet.red_black_masks(1, 1, fw)
    perm = np.concatenate([np.flatnonzero(red), np.flatnonzero(black)])
    Ap = A[np.ix_(perm, perm)]
    M = np.tril(Ap)
    S_perm = np.eye(fw * fw) - np.linalg.solve(M, Ap)
    inv = np.argsort(perm)
    S_ref = S_perm[np.ix_(inv, inv)]
    Sf = np.column_stack([pnet.gs_sweep(A, np.eye(fw * fw)[:, j], (red, black)) for j in range(fw * fw)])
    Sb = pnet.gs_sweep(A, np.eye(fw * fw), (black, red))  # all columns at once
    assert np.allclose(Sf, S_ref, atol=1e-13)
    assert np.allclose(A @ Sb, Sf.T @ A, atol=1e-12)
    e = errors[0].reshape(n, n)[:fw, :fw].reshape(-1)
    assert (Sf @ e) @ A @ (Sf @ e) < e @ A @ e


def test_two_grid_loss_is_a_contraction_factor():
    """0 < ||S_b T S_f e||_A^2 / ||e||_A^2 < 1, and below the loss of the
    coarse correction alone for the same errors (smoothing only helps)."""
    n, nc, cw = 31, 15, 15
    faces, errors = crop_problem()
    w = pnet.normalize(np.full((9, nc, nc), np.log(np.expm1(1.0))), nc)
    l2, _ = pnet.crop_loss_grad(faces, n, 1.0, w, errors, [(1, 1)], cw)
    l1, _ = pnet.crop_loss_grad(faces, n, 1.0, w, errors, [(1, 1)], cw, smooth=False)
    assert 0.0 < l2 < l1 < 1.0


def test_gradient_matches_finite_differences():
    n = 31
    faces, errors = crop_problem(seed=5)
    theta = pnet.init_params(2)
    theta = theta + np.random.default_rng(6).normal(scale=0.05, size=theta.size)
    loss, grad = pnet.loss_and_grad(theta, faces, n, 1.0, errors, [(1, 1)])
    rng = np.random.default_rng(7)
    idx = rng.choice(theta.size, size=12, replace=False)
    idx = np.concatenate([idx, [theta.size - 1, theta.size - 5]])  # two output biases
    for k in idx:
        eps = 1e-5
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        lp, _ = pnet.loss_and_grad(tp, faces, n, 1.0, errors, [(1, 1)])
        lm, _ = pnet.loss_and_grad(tm, faces, n, 1.0, errors, [(1, 1)])
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grad[k]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (k, fd, grad[k])
