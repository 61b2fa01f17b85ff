"""mgmc_sample_noalloc against mgmc_sample through the C ABI: the same kernels
with their per-call scratch in the static device array, so the results are
bit-identical; two calls in a row, the second on a smaller problem."""
import numpy as np
import pytest

from paper_2407_12149_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def one_case(n, levels, nchains, beta, nsamples, precision):
    from paper_2407_12149_amd import mgmc
    face = workloads.face_array(n, 2, workloads.fourier_log_field(2, nmodes=8, seed=3))
    prob = dict(dim=2, n=n, levels=levels, kappa2=50.0, face_coef=face, nchains=nchains, seed=1,
                precision=precision)
    ptr, idx, val = workloads.patch_sensors(n, 2, beta, seed=2)
    obs = (ptr, idx, val, np.full(beta, 1e-3))
    y = workloads.observed_values(beta, seed=4)
    F = torch.tensor(workloads.subcube_qoi(n, 2), device="cuda")
    # f_L = B Gamma^{-1} y as an explicit right-hand side for both entry points
    f = np.zeros(n * n)
    for j in range(beta):
        f[idx[ptr[j]:ptr[j + 1]]] += val[ptr[j]:ptr[j + 1]] * y[j] / 1e-3
    rhs = torch.tensor(f, device="cuda")
    out = {}
    for name in ("sample", "noalloc"):
        s = mgmc.Sampler(prob, obs=obs)
        q = torch.zeros(nsamples, nchains, dtype=torch.float64, device="cuda")
        with torch.cuda.stream(s.stream):
            fn = mgmc.mgmc_sample if name == "sample" else mgmc.mgmc_sample_noalloc
            fn(s.ctx, 0, nsamples, s.theta, rhs, F, q)
        s.stream.synchronize()
        out[name] = (s.theta.clone(), q.clone())
        s.close()
    assert torch.equal(out["sample"][0], out["noalloc"][0])
    assert torch.equal(out["sample"][1], out["noalloc"][1])


def test_noalloc_matches_sample_twice():
    print("[noalloc] 127^2 x 8 chains, beta 6, fp64", flush=True)
    one_case(127, 5, 8, 6, 4, "fp64")
    print("[noalloc] 63^2 x 3 chains, beta 3, fp32", flush=True)
    one_case(63, 4, 3, 3, 3, "fp32")


def test_noalloc_rejects_oversized_scratch():
    """20000 chains and 16 observations need qnb * 20000 + 2 * 16 * 20000 >
    2^19 doubles of scratch: refused before any launch."""
    from paper_2407_12149_amd import mgmc
    n, beta, nch = 31, 16, 20000
    ptr, idx, val = workloads.patch_sensors(n, 2, beta, seed=2)
    s = mgmc.Sampler(dict(dim=2, n=n, levels=3, kappa2=50.0, nchains=nch),
                     obs=(ptr, idx, val, np.full(beta, 1e-3)))
    with pytest.raises(mgmc.MGMCError) as ei:
        mgmc.mgmc_sample_noalloc(s.ctx, 0, 1, s.theta)
    assert ei.value.status == mgmc.MGMC_EINVAL
    s.close()
