"""GPU parity of the learned-prolongation network against the FP64 reference.

The network runs in FP32 on the device (features, convolutions, ReLU) and
FP64 from its outputs on (softplus, normalisation, two-grid loss, crop
Cholesky).  The reference is FP64 throughout, fed the same FP32 parameters.
Tolerances: the weights are held, entry by entry, to twice a first-order
bound of the FP32 rounding in the network (weight_error_bound below), and to
1e-5 of the largest weight overall.  The loss and the gradient move
linearly with the weight errors (relative size ~3e-7 for an FP32 emulation
of the same network); the loss, a ratio of FP64 quadratic forms with
relative sensitivity below 1, is held to 1e-7 relative, and the gradient,
which passes three more FP32 products (back-propagation) and sums over every
coarse node, to 1e-5 of its norm.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import pnet as ref
from paper_2407_12149_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def fields(n, count, seed0):
    return [workloads.lognormal_faces_fft(n, 2, 0.1, 1.0, seed=seed0 + k) for k in range(count)]


def params(seed, noise):
    th = ref.init_params(seed)
    th = th + np.random.default_rng(seed + 100).normal(scale=noise, size=th.size)
    return th.astype(np.float32)


def test_param_count_matches_reference():
    from paper_2407_12149_amd import mgmc
    assert mgmc.mgmc_pnet_param_count() == ref.nparams()


U32 = 2.0 ** -24  # unit roundoff of FP32


LAMBDA = 6.0  # probabilistic bound holds with probability >= 1 - 2 exp(-18) per sum


def sum_bound(k):
    """Probabilistic bound on the relative rounding of a k-term FP32 sum
    (Higham and Mary, SIAM J. Sci. Comput. 2019): |fl(s) - s| <= lambda sqrt(k) u
    sum |terms| with probability >= 1 - 2 exp(-lambda^2 (1 - u)^2 / 2)."""
    return LAMBDA * np.sqrt(k) * U32


def weight_error_bound(theta, faces, n):
    """First-order bound on |w_FP32 path - w| from the FP32 rounding of the
    features and of every convolution sum (sum_bound), carried through the
    next layers with |W|, ReLU (1-Lipschitz), softplus (slope sigma(o)) and
    the normalisation w = rho / Z (relative errors add)."""
    nc = (n - 1) // 2
    W1, b1, W2, b2, W3, b3 = ref.unpack(theta)
    X = ref.features(faces, n)
    a, da = X, U32 * np.abs(X)
    for W, b, relu in ((W1, b1, True), (W2, b2, True), (W3, b3, False)):
        z = ref.conv3x3(a, W, b)
        k = W.shape[1] * 9 + 1
        dz = sum_bound(k) * (ref.conv3x3(np.abs(a), np.abs(W), np.abs(b))) + \
            ref.conv3x3(da, np.abs(W), np.zeros_like(b))
        a, da = (np.maximum(z, 0.0) if relu else z), dz
    o, do = a, da
    rho = ref.softplus(o)
    drho = do / (1.0 + np.exp(-(o + do)))
    w = ref.normalize(o, nc)
    dw = np.zeros_like(w)
    for Jy in range(1, nc + 1):
        for Jx in range(1, nc + 1):
            for t in range(9):
                if t == 4:
                    continue
                dx, dy = t % 3 - 1, t // 3 - 1
                Z, dZ = 0.0, 0.0
                for Ky, ey in ref.covering(2 * Jy + dy, nc):
                    for Kx, ex in ref.covering(2 * Jx + dx, nc):
                        if 1 <= Kx <= nc and 1 <= Ky <= nc:
                            u = (ex + 1) + 3 * (ey + 1)
                            Z += rho[u, Ky - 1, Kx - 1]
                            dZ += drho[u, Ky - 1, Kx - 1]
                        else:
                            Z += 1.0
                r = rho[t, Jy - 1, Jx - 1]
                dw[Jy - 1, Jx - 1, t] = w[Jy - 1, Jx - 1, t] * (drho[t, Jy - 1, Jx - 1] / r + dZ / Z)
    return w.reshape(nc * nc, 9), dw.reshape(nc * nc, 9)


def test_weights_match_reference():
    from paper_2407_12149_amd import mgmc
    n, nc, b = 63, 31, 3
    log(f"[pnet] weights n={n} batch={b}")
    th = params(1, 0.05)
    faces = fields(n, b, 10)
    net = mgmc.PNet(n, max_batch=b, params=th)
    w = net.weights(torch.tensor(np.stack(faces), device="cuda")).cpu().numpy()
    torch.cuda.synchronize()
    for k in range(b):
        want = ref.prolongation_weights(th.astype(np.float64), faces[k], n)
        _, bound = weight_error_bound(th.astype(np.float64), faces[k], n)
        err = np.abs(w[k] - want)
        ratio = (err / (bound + 1e-15)).max()
        log(f"[pnet] field {k}: weight rel err {err.max() / np.abs(want).max():.2e}, "
            f"error / first-order FP32 bound <= {ratio:.3f}")
        assert (err <= 2.0 * bound + 1e-14).all()
        # the bound is worst-case in sign; an FP32 emulation of the same
        # network (numpy float32, same summation order) stays below 3e-7
        assert err.max() <= 1e-5 * np.abs(want).max()
    net.close()


def test_initial_network_is_multilinear():
    """Zero weights and the initial output bias give equal rho: multilinear P."""
    from paper_2407_12149_amd import mgmc
    n, nc = 31, 15
    th = ref.init_params(0) * 0.0
    th[-9:] = np.log(np.expm1(1.0))
    net = mgmc.PNet(n, params=th.astype(np.float32))
    w = net.weights(torch.tensor(fields(n, 1, 3)[0], device="cuda")).cpu().numpy()[0]
    P = oracle.Oracle(2, n, 2, 1.0).dense(1, 1)
    for J in range(nc * nc):
        Jx, Jy = 1 + J % nc, 1 + J // nc
        for t in range(9):
            fx, fy = 2 * Jx + t % 3 - 1, 2 * Jy + t // 3 - 1
            assert abs(w[J, t] - P[(fx - 1) + n * (fy - 1), J]) <= 1e-6
    net.close()


def test_loss_and_gradient_match_reference():
    from paper_2407_12149_amd import mgmc
    n, nc, b, K = 63, 31, 2, 2
    log(f"[pnet] loss/grad n={n} batch={b} errors={K}")
    th = params(2, 0.05)
    faces = fields(n, b, 20)
    rng = np.random.default_rng(5)
    errs = rng.normal(size=(b, K, n * n))
    crops = [(1 + 15 * cx, 1 + 15 * cy) for cy in range(nc // 15) for cx in range(nc // 15)]
    want_l, want_g = 0.0, np.zeros(ref.nparams())
    for k in range(b):
        l, g = ref.loss_and_grad(th.astype(np.float64), faces[k], n, 2.0, errs[k], crops)
        want_l += l / b
        want_g += g / b
    net = mgmc.PNet(n, max_batch=b, max_errors=K, params=th)
    got_l, got_g = net.loss_grad(torch.tensor(np.stack(faces), device="cuda"),
                                 torch.tensor(errs, device="cuda"), 2.0)
    log(f"[pnet] loss {got_l:.12f} vs {want_l:.12f}")
    assert abs(got_l - want_l) <= 1e-7 * abs(want_l)
    gerr = np.linalg.norm(got_g - want_g) / np.linalg.norm(want_g)
    log(f"[pnet] gradient rel err {gerr:.2e}")
    assert gerr <= 1e-5
    net.close()


def test_training_reduces_the_loss():
    from paper_2407_12149_amd import mgmc
    n, b, K = 63, 2, 4
    log(f"[pnet] training n={n} batch={b}")
    faces = torch.tensor(np.stack(fields(n, b, 40)), device="cuda")
    errs = torch.tensor(np.random.default_rng(9).normal(size=(b, K, n * n)), device="cuda")
    net = mgmc.PNet(n, max_batch=b, max_errors=K, params=ref.init_params(4).astype(np.float32))
    first = net.train_step(faces, errs, 1.0, 3e-3)
    for _ in range(40):
        last = net.train_step(faces, errs, 1.0, 3e-3)
    log(f"[pnet] loss {first:.5f} -> {last:.5f}")
    assert np.isfinite(last) and last < first
    net.close()


def test_learned_weights_drive_the_sampler():
    """Weights produced by the network, fed back as prolong_w, give the same
    chain on the device and in the oracle."""
    from paper_2407_12149_amd import mgmc
    n = 63
    log(f"[pnet] sampler with learned P n={n}")
    face = fields(n, 1, 60)[0]
    net = mgmc.PNet(n, params=params(7, 0.1))
    w = net.weights(torch.tensor(face, device="cuda")).cpu().numpy()[0]
    net.close()
    prob = dict(dim=2, n=n, levels=3, kappa2=10.0, face_coef=face, prolong_w=w.reshape(-1),
                nchains=2, seed=4)
    o = oracle.Oracle(2, n, 3, 10.0, face_coef=face, prolong_w=w.reshape(-1), seed=4)
    ref_tr = [o.chain(np.zeros(n * n), 0, 3, chain=c, traj=True)[2] for c in range(2)]
    s = mgmc.Sampler(prob)
    for k in range(3):
        s.sample(k, 1, want_qoi=False)
        torch.cuda.synchronize()
        got = s.theta.cpu().numpy()
        for c in range(2):
            want = ref_tr[c][k]
            e = np.abs(got[c] - want).max() / np.abs(want).max()
            assert e <= 1e-10, (k, c, e)
    s.close()
