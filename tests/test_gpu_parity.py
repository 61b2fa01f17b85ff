"""GPU parity: the HIP library against the CPU oracle, element by element.

Every case runs the same problem, seed and chain ids through both and
compares chain states after every update (relative to the largest oracle
entry) and the QoI series.  FP64 tolerance 1e-10: both sides evaluate the
same formulas in FP64 and differ only by rounding order (fused multiply-add,
device vs host libm, the algebraically equal Woodbury and coarse-solve
forms of the library), which the contracting V-cycle does not amplify.
"""
import concurrent.futures as cf
import sys

import numpy as np
import pytest

import oracle
from paper_2407_12149_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def make_problem(dim, n, levels, kappa2, face=None, beta=0, gamma=1e-3, seed=0, nchains=2,
                 chain_offset=0, prolong_w=None, nu1=1, nu2=1, precision="fp64", obs_seed=1):
    prob = dict(dim=dim, n=n, levels=levels, kappa2=kappa2, face_coef=face, nchains=nchains,
                chain_offset=chain_offset, seed=seed, prolong_w=prolong_w, nu1=nu1, nu2=nu2,
                precision=precision)
    obs = None
    if beta:
        ptr, idx, val = workloads.patch_sensors(n, dim, beta, seed=obs_seed)
        obs = (ptr, idx, val, np.full(beta, gamma))
    return prob, obs


def oracle_for(prob, obs, y=None, rhs=None):
    o = oracle.Oracle(prob["dim"], prob["n"], prob["levels"], prob["kappa2"],
                      face_coef=prob.get("face_coef"), prolong_w=prob.get("prolong_w"),
                      nu1=prob.get("nu1", 1), nu2=prob.get("nu2", 1), seed=prob.get("seed", 0))
    if obs is not None:
        o.set_obs(*obs)
    if y is not None:
        o.set_posterior_rhs(y)
    elif rhs is not None:
        o.set_rhs(rhs)
    return o


def oracle_runs(o, prob, nsamples, F=None, m0=0, theta0=None, traj=True):
    """Trajectories of every chain, one thread per chain (ctypes releases the GIL)."""
    N = prob["n"] ** prob["dim"]
    ids = [prob.get("chain_offset", 0) + c for c in range(prob["nchains"])]

    def one(k):
        t0 = np.zeros(N) if theta0 is None else theta0[k]
        return o.chain(t0, m0, nsamples, chain=ids[k], F=F, traj=traj)

    with cf.ThreadPoolExecutor(max_workers=min(8, len(ids))) as ex:
        return list(ex.map(one, range(len(ids))))


def rel_err(got, want):
    return np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)


def check_stepwise(prob, obs, nsamples, y=None, rhs=None, F=None, label="", tiled=True,
                   variant=None, cpb=None, levels=None, fused=None, options=None):
    from paper_2407_12149_amd import mgmc
    log(f"[parity] {label} dim={prob['dim']} n={prob['n']} levels={prob['levels']} "
        f"beta={0 if obs is None else len(obs[0]) - 1} chains={prob['nchains']} tiled={tiled}")
    o = oracle_for(prob, obs, y=y, rhs=rhs)
    ref = oracle_runs(o, prob, nsamples, F=F)
    s = mgmc.Sampler(prob, obs=obs)
    s.set_option(mgmc.MGMC_OPT_TILED_SWEEPS, 1 if tiled else 0)
    if variant is not None:
        s.set_option(mgmc.MGMC_OPT_SWEEP_VARIANT, variant)
    if cpb is not None:
        s.set_option(mgmc.MGMC_OPT_CHAINS_PER_BLOCK, cpb)
    if levels is not None:
        from paper_2407_12149_amd import autotune
        autotune.apply(s, levels)
    if fused is not None:
        s.set_option(mgmc.MGMC_OPT_COARSE_FUSED, int(fused))
    for opt, val in (options or {}).items():
        s.set_option(opt, val)
    Fd = None if F is None else torch.tensor(F, device="cuda")
    rhsd = None if rhs is None else torch.tensor(rhs, device="cuda")
    worst = 0.0
    for k in range(nsamples):
        if y is not None:
            q = s.posterior_sample(y, k, 1, F=Fd)
        else:
            q = s.sample(k, 1, rhs=rhsd, F=Fd)
        torch.cuda.synchronize()
        got = s.theta.cpu().numpy()
        for c in range(prob["nchains"]):
            e = rel_err(got[c], ref[c][2][k])
            worst = max(worst, e)
            assert e <= TOL, f"{label}: sample {k} chain {c}: rel err {e:.3e}"
            if F is not None:
                qw = ref[c][1][k]
                assert abs(q[0, c].item() - qw) <= TOL * max(np.abs(ref[c][1]).max(), 1e-300)
    s.close()
    log(f"[parity] {label}: worst relative state error {worst:.2e}")
    return worst


@pytest.mark.parametrize("tiled", [True, False])
def test_prior_2d_stepwise(tiled):
    prob, obs = make_problem(2, 63, 4, 100.0, nchains=2)
    check_stepwise(prob, obs, 8, F=workloads.subcube_qoi(63, 2), label="prior 63^2", tiled=tiled)


@pytest.mark.parametrize("tiled", [True, False])
def test_posterior_2d_variable_stepwise(tiled):
    n = 127
    face = workloads.face_array(n, 2, workloads.fourier_log_field(2, nmodes=32, seed=4))
    prob, obs = make_problem(2, n, 4, 100.0, face=face, beta=8, gamma=1e-4, nchains=3)
    y = workloads.observed_values(8, seed=5)
    check_stepwise(prob, obs, 5, y=y, F=workloads.subcube_qoi(n, 2), label="posterior 127^2",
                   tiled=tiled)


@pytest.mark.parametrize("variant,cpb", [(0, 0), (1, 0), (1, 4), (2, 3), (2, 0), (3, 0), (4, 0), (4, 3)])
def test_posterior_2d_many_tiles_many_chains(variant, cpb):
    """255^2 spans several sweep tiles in both directions with a ragged last
    tile; 9 chains exercise chain groups per block (ragged when cpb = 4)."""
    n = 255
    face = workloads.face_array(n, 2, workloads.fourier_log_field(2, nmodes=8, seed=2))
    prob, obs = make_problem(2, n, 5, 30.0, face=face, beta=5, gamma=1e-3, nchains=9)
    y = workloads.observed_values(5, seed=6)
    check_stepwise(prob, obs, 2, y=y, F=workloads.subcube_qoi(n, 2),
                   label=f"posterior 255^2 variant {variant} cpb {cpb}", variant=variant, cpb=cpb)


@pytest.mark.parametrize("fused", [3, 1, 0])
def test_bottom_levels_fused_or_per_level(fused):
    """The levels up to 63^2 (fused 3) or up to 15^2 (fused 1) as one launch
    (one workgroup per chain, LDS resident), or level by level (0): all follow
    the oracle; 2 pre- and 3 post-sweeps exercise the sweep counts inside the
    fused bottom."""
    n = 255
    face = workloads.face_array(n, 2, workloads.fourier_log_field(2, nmodes=8, seed=5))
    prob, obs = make_problem(2, n, 6, 30.0, face=face, beta=6, gamma=1e-3, nchains=3, nu1=2, nu2=3)
    y = workloads.observed_values(6, seed=9)
    check_stepwise(prob, obs, 2, y=y, label=f"posterior 255^2 fused bottom {fused}", fused=fused)


@pytest.mark.parametrize("form", [1, 2, 0])
def test_low_rank_step_forms(form):
    """The low-rank step (ragged 16-chain tile with 19 chains, beta not a
    multiple of 4): 1 = one launch from the sweep's snapshot of the
    observation sites with the FP64 MFMA product, 2 = separate B^T theta
    launch and MFMA product, 0 = vector FMA product."""
    n = 127
    face = workloads.face_array(n, 2, workloads.fourier_log_field(2, nmodes=8, seed=6))
    prob, obs = make_problem(2, n, 4, 30.0, face=face, beta=7, gamma=1e-3, nchains=19)
    y = workloads.observed_values(7, seed=10)
    from paper_2407_12149_amd import mgmc
    check_stepwise(prob, obs, 2, y=y, label=f"posterior 127^2 x 19 low-rank form {form}",
                   options={mgmc.MGMC_OPT_LOWRANK_MFMA: form})


@pytest.mark.parametrize("width", [4, 5])
def test_low_rank_snapshot_wide_sensors(width):
    """Sensors averaging width x width nodes (16 or 25 weights per observation
    on the finest level, more slots on coarser ones), so the snapshot takes
    its wider slot layouts."""
    n = 127
    face = workloads.face_array(n, 2, workloads.fourier_log_field(2, nmodes=8, seed=12))
    prob, _ = make_problem(2, n, 4, 30.0, face=face, nchains=5)
    rng = np.random.default_rng(20 + width)
    m = 9
    ptr, idx, val = [0], [], []
    for _ in range(m):
        x0, y0 = rng.integers(1, n - width, size=2)
        for dy in range(width):
            for dx in range(width):
                idx.append((x0 + dx - 1) + n * (y0 + dy - 1))
                val.append(1.0 / width ** 2)
        ptr.append(len(idx))
    obs = (np.array(ptr, dtype=np.int64), np.array(idx, dtype=np.int32), np.array(val), np.full(m, 1e-3))
    y = workloads.observed_values(m, seed=13)
    check_stepwise(prob, obs, 2, y=y, label=f"posterior 127^2 {width}x{width} sensors")


def test_low_rank_snapshot_with_lds_tiled_sweeps():
    """The snapshot of the observation sites written by the LDS-tiled sweep
    form (tile height 32) on every level, 70 observations across tiles."""
    n = 255
    face = workloads.face_array(n, 2, workloads.fourier_log_field(2, nmodes=8, seed=7))
    prob, obs = make_problem(2, n, 5, 30.0, face=face, beta=70, gamma=1e-3, nchains=3)
    y = workloads.observed_values(70, seed=11)
    check_stepwise(prob, obs, 2, y=y, label="posterior 255^2 beta 70 tiled sweeps",
                   levels=[None, [0, 0], [0, 0], [0, 0], [0, 0]])


def test_per_level_kernel_forms():
    """A different sweep form and chain grouping on every level."""
    n = 255
    face = workloads.face_array(n, 2, workloads.fourier_log_field(2, nmodes=8, seed=4))
    prob, obs = make_problem(2, n, 5, 30.0, face=face, beta=4, gamma=1e-3, nchains=7)
    y = workloads.observed_values(4, seed=8)
    check_stepwise(prob, obs, 2, y=y, label="posterior 255^2 mixed per-level forms",
                   levels=[None, [2, 3], [0, 0], [1, 5], [2, 1]])


def test_prior_3d_stepwise():
    prob, obs = make_problem(3, 15, 3, 1.0, nchains=2)
    check_stepwise(prob, obs, 4, F=workloads.subcube_qoi(15, 3), label="prior 15^3")


def test_posterior_3d_variable_stepwise():
    n = 31
    face = workloads.face_array(n, 3, workloads.gaussian_log_field(3, 0.1, 1.0, seed=8, nfeatures=64))
    prob, obs = make_problem(3, n, 3, 1.0, face=face, beta=6, gamma=2.5e-5, nchains=2)
    y = workloads.observed_values(6, seed=9)
    check_stepwise(prob, obs, 3, y=y, F=workloads.subcube_qoi(n, 3), label="posterior 31^3")


def test_single_level_is_cholesky_sampler():
    prob, obs = make_problem(2, 15, 1, 10.0, beta=3, gamma=1e-2, nchains=3)
    y = workloads.observed_values(3, seed=1)
    check_stepwise(prob, obs, 3, y=y, label="one level 15^2")


@pytest.mark.parametrize("tiled", [True, False])
def test_user_prolongation_weights(tiled):
    n = 63
    nc = 31
    rng = np.random.default_rng(3)
    w = rng.uniform(0.2, 1.0, size=(nc * nc, 9))
    prob, obs = make_problem(2, n, 3, 50.0, nchains=2, prolong_w=w.reshape(-1))
    check_stepwise(prob, obs, 4, label="user P 63^2", tiled=tiled)


def test_user_prolongation_weights_posterior():
    """User weights on the finest transfer with observations (the low-rank
    term of the restricted right-hand side through the user weights)."""
    n = 63
    nc = 31
    rng = np.random.default_rng(4)
    w = rng.uniform(0.2, 1.0, size=(nc * nc, 9))
    prob, obs = make_problem(2, n, 3, 50.0, beta=5, gamma=1e-3, nchains=3, prolong_w=w.reshape(-1))
    y = workloads.observed_values(5, seed=12)
    check_stepwise(prob, obs, 3, y=y, label="user P 63^2 posterior")


def test_more_sweeps_and_rhs():
    n = 31
    rng = np.random.default_rng(0)
    rhs = rng.normal(size=n * n)
    prob, obs = make_problem(2, n, 3, 10.0, nchains=2, nu1=2, nu2=3)
    check_stepwise(prob, obs, 4, rhs=rhs, label="nu=(2,3) with rhs 31^2")


def test_ragged_chain_offset():
    prob, obs = make_problem(2, 31, 3, 10.0, nchains=5, chain_offset=7, beta=2, gamma=1e-2)
    y = workloads.observed_values(2, seed=2)
    check_stepwise(prob, obs, 2, y=y, label="5 chains offset 7")


def test_prior63_full_run_qoi_series():
    """The 63^2 prior workload: one chain, 2000 updates, QoI series and final state."""
    from paper_2407_12149_amd import mgmc
    cfg = workloads.config("prior63")
    prob, obs = make_problem(2, 63, 4, cfg["kappa2"], nchains=1)
    log("[parity] prior63 2000 samples")
    o = oracle_for(prob, obs)
    th, qw, _ = o.chain(np.zeros(63 * 63), 0, cfg["nsamples"], chain=0, F=cfg["F"])
    s = mgmc.Sampler(prob)
    q = s.sample(0, cfg["nsamples"], F=torch.tensor(cfg["F"], device="cuda"))
    torch.cuda.synchronize()
    assert rel_err(s.theta.cpu().numpy()[0], th) <= TOL
    assert np.abs(q[:, 0].cpu().numpy() - qw).max() <= TOL * np.abs(qw).max()
    s.close()


def test_posterior1023_sampled_parity():
    """Full-size 1023^2 posterior workload (7 levels, 64 sensors, 8 chains) in the
    launch configuration the benchmark times: the first two updates of every
    chain against the oracle."""
    from paper_2407_12149_amd import mgmc
    cfg = workloads.config("posterior1023")
    prob = dict(dim=2, n=1023, levels=7, kappa2=cfg["kappa2"], face_coef=cfg["face_coef"],
                nchains=8, seed=0)
    log("[parity] posterior1023 8 chains x 2 samples")
    o = oracle_for(prob, cfg["obs"], y=cfg["y"])
    ref = oracle_runs(o, prob, 2, F=cfg["F"], traj=False)
    s = mgmc.Sampler(prob, obs=cfg["obs"])
    s.set_graph(True)
    q = s.posterior_sample(cfg["y"], 0, 2, F=torch.tensor(cfg["F"], device="cuda"))
    torch.cuda.synchronize()
    got = s.theta.cpu().numpy()
    for c in range(8):
        e = rel_err(got[c], ref[c][0])
        assert e <= TOL, f"chain {c}: {e:.3e}"
        assert np.abs(q[:, c].cpu().numpy() - ref[c][1]).max() <= TOL * np.abs(ref[c][1]).max()
    s.close()


def _run(prob, obs, y, m0, nsamples, theta0=None, graph=False):
    from paper_2407_12149_amd import mgmc
    s = mgmc.Sampler(prob, obs=obs)
    if theta0 is not None:
        s.theta.copy_(theta0)
    s.set_graph(graph)
    if y is None:
        s.sample(m0, nsamples)
    else:
        s.posterior_sample(y, m0, nsamples)
    torch.cuda.synchronize()
    out = s.theta.clone()
    s.close()
    return out


def test_counter_based_chunking_graph_and_determinism():
    prob, obs = make_problem(2, 63, 4, 20.0, beta=4, gamma=1e-3, nchains=3)
    y = workloads.observed_values(4, seed=3)
    log("[property] chunking / graph / determinism")
    full = _run(prob, obs, y, 0, 6)
    again = _run(prob, obs, y, 0, 6)
    assert torch.equal(full, again)
    half = _run(prob, obs, y, 0, 3)
    rest = _run(prob, obs, y, 3, 3, theta0=half)
    assert torch.equal(full, rest)
    graph = _run(prob, obs, y, 0, 6, graph=True)
    assert torch.equal(full, graph)
    # chain c with offset k reproduces chain k + c
    p2 = dict(prob, nchains=1, chain_offset=2)
    one = _run(p2, obs, y, 0, 6)
    assert torch.equal(one[0], full[2])


def test_posterior_without_observations_is_state_error():
    from paper_2407_12149_amd import mgmc
    prob, _ = make_problem(2, 15, 2, 1.0)
    s = mgmc.Sampler(prob)
    with pytest.raises(mgmc.MGMCError) as ei:
        s.posterior_sample(np.zeros(2), 0, 1)
    assert ei.value.status == mgmc.MGMC_ESTATE
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dma_tiles_match_register_form(precision):
    """Form 4 brings each chain's state tile and coarse patch into LDS by DMA
    and otherwise runs form 1's arithmetic, so the states agree bit for bit
    (9 chains in groups of 3 and of 9: odd groups end on either buffer)."""
    n = 255
    face = workloads.face_array(n, 2, workloads.fourier_log_field(2, nmodes=8, seed=3))
    prob, obs = make_problem(2, n, 5, 30.0, face=face, beta=5, gamma=1e-3, nchains=9,
                             precision=precision)
    y = workloads.observed_values(5, seed=7)
    from paper_2407_12149_amd import mgmc
    states = {}
    for variant, cpb in ((1, 3), (4, 3), (4, 9)):
        log(f"[dma] {precision} variant {variant} cpb {cpb}")
        s = mgmc.Sampler(prob, obs=obs)
        s.set_option(mgmc.MGMC_OPT_SWEEP_VARIANT, variant)
        s.set_option(mgmc.MGMC_OPT_CHAINS_PER_BLOCK, cpb)
        s.posterior_sample(y, 0, 3)
        torch.cuda.synchronize()
        states[(variant, cpb)] = s.theta.clone()
        s.close()
    ref = states[(1, 3)]
    for key, th in states.items():
        assert torch.equal(th, ref), f"{precision} {key}: max diff {(th - ref).abs().max().item():.3e}"


def test_fp32_tracks_fp64_on_common_random_numbers():
    """FP32 sweeps and noise draw from the same Philox counters and the same
    53-bit uniforms as FP64, so the chains stay close (paired
    common-random-number comparison) to the per-site bound derived in
    tests/test_gpu_oracle_paths.py, 144 u (max|theta| + max|f| / A_ii), over
    50 updates."""
    n = 127
    face = workloads.face_array(n, 2, workloads.fourier_log_field(2, nmodes=16, seed=1))
    prob64, obs = make_problem(2, n, 5, 100.0, face=face, beta=8, gamma=1e-4, nchains=2)
    prob32 = dict(prob64, precision="fp32")
    y = workloads.observed_values(8, seed=4)
    F = torch.tensor(workloads.subcube_qoi(n, 2), device="cuda")
    from paper_2407_12149_amd import mgmc
    log("[fp32] paired run 127^2")
    s64 = mgmc.Sampler(prob64, obs=obs)
    s32 = mgmc.Sampler(prob32, obs=obs)
    q64 = s64.posterior_sample(y, 0, 50, F=F)
    q32 = s32.posterior_sample(y, 0, 50, F=F)
    torch.cuda.synchronize()
    scale = q64.abs().max().item()
    dq = (q64 - q32).abs().max().item() / scale
    rel = ((s64.theta - s32.theta.double()).abs() / s64.theta.abs().max()).flatten()
    med = rel.median().item()
    p999 = rel.quantile(0.999).item() if rel.numel() < 16_000_000 else rel.max().item()
    log(f"[fp32] qoi rel diff {dq:.2e}; state rel diff median {med:.2e} "
        f"p99.9 {p999:.2e} max {rel.max().item():.2e}")
    from test_gpu_oracle_paths import fp32_bound, posterior_rhs
    o = oracle_for(prob64, obs)
    bound = fp32_bound(s64.theta.abs().max().item(), posterior_rhs(n, 2, obs, y), o.dense(4, 8))
    diff = (s64.theta - s32.theta.double()).abs().max().item()
    log(f"[fp32] max site difference {diff:.2e}, bound {bound:.2e}")
    assert med <= 1e-6
    assert diff <= bound
    s64.close()
    s32.close()



def test_fp32_3d_chain_groups_track_fp64():
    """3D FP32 prolongation and residual restriction give each thread a group
    of chains (by size: one group of all 5 chains on the 127^3 level, groups
    of 2, 2 and 1 on its 63^3 coarse level); the paired FP64 run (one chain
    per thread) must track it as in 2D, chain by chain, to the derived FP32
    bound."""
    n = 127
    face = workloads.face_array(n, 3, workloads.gaussian_log_field(3, 0.1, 1.0, seed=3, nfeatures=64))
    prob64, obs = make_problem(3, n, 5, 1.0, face=face, beta=6, gamma=2.5e-5, nchains=5)
    prob32 = dict(prob64, precision="fp32")
    y = workloads.observed_values(6, seed=5)
    F = torch.tensor(workloads.subcube_qoi(n, 3), device="cuda")
    from paper_2407_12149_amd import mgmc
    log("[fp32] paired run 127^3, 5 chains")
    s64 = mgmc.Sampler(prob64, obs=obs)
    s32 = mgmc.Sampler(prob32, obs=obs)
    q64 = s64.posterior_sample(y, 0, 10, F=F)
    q32 = s32.posterior_sample(y, 0, 10, F=F)
    torch.cuda.synchronize()
    for c in range(prob64["nchains"]):
        dth = (s64.theta[c] - s32.theta[c].double()).abs()
        rel = (dth / s64.theta[c].abs().max()).flatten()
        med = rel.median().item()
        # the last QoI of the pair differs by at most sum_i |F_i| |dtheta_i|
        # of the final states (both reductions accumulate in FP64)
        dq = abs(q64[-1, c].item() - q32[-1, c].item())
        bound = (F.abs() * dth).sum().item()
        slack = 1e-12 * (F.abs() * s64.theta[c].abs()).sum().item()
        log(f"[fp32] chain {c}: last qoi diff {dq:.2e} (bound {bound:.2e}); state rel diff "
            f"median {med:.2e} max {rel.max().item():.2e}")
        assert dq <= bound + slack
        assert med <= 1e-6
        from test_gpu_oracle_paths import fp32_bound, posterior_rhs
        if c == 0:
            diag = oracle_for(prob64, obs).dense(4, 8)
            frhs = posterior_rhs(n, 3, obs, y)
        tol = fp32_bound(s64.theta[c].abs().max().item(), frhs, diag)
        assert dth.max().item() <= tol
    s64.close()
    s32.close()

def test_batch_graph_equals_individual_runs():
    """Contexts of different sizes and dimensions advanced as branches of one
    graph give bitwise the same chains and QoI as separate runs."""
    from paper_2407_12149_amd import mgmc
    log("[batch] 3 contexts, graph branches")
    specs = [make_problem(2, 127, 5, 25.0, nchains=3),
             make_problem(2, 63, 4, 25.0, nchains=2, beta=3, gamma=1e-3),
             make_problem(3, 15, 3, 25.0, nchains=2)]
    specs[0][0]["precision"] = "fp32"
    y = workloads.observed_values(3, seed=1)
    Fs = [torch.tensor(workloads.subcube_qoi(p["n"], p["dim"]), device="cuda") for p, _ in specs]
    ref = []
    for (p, o), F in zip(specs, Fs):
        s = mgmc.Sampler(p, obs=o)
        q = s.posterior_sample(y, 0, 5, F=F) if o is not None else s.sample(0, 5, F=F)
        torch.cuda.synchronize()
        ref.append((s.theta.clone(), q.clone()))
        s.close()
    samplers = [mgmc.Sampler(p, obs=o) for p, o in specs]
    samplers[1].posterior_sample(y, 0, 0)  # bind the data y
    b = mgmc.Batch(samplers, updates_per_launch=2)
    qs = b.sample(0, 5, Fs=Fs)
    torch.cuda.synchronize()
    for (th, q), s, qb in zip(ref, samplers, qs):
        assert torch.equal(th, s.theta)
        assert torch.equal(q, qb)
    b.close()
    for s in samplers:
        s.close()


def test_autotune_picks_and_caches(tmp_path):
    from paper_2407_12149_amd import autotune, mgmc
    prob, obs = make_problem(2, 255, 6, 25.0, nchains=4)
    log("[autotune] 255^2 x 4")
    s = mgmc.Sampler(prob)
    cache = str(tmp_path / "tune.json")
    best = autotune.autotune(s, cache_path=cache, updates=2)
    assert not best["cached"] and best["ms"] > 0
    again = autotune.autotune(s, cache_path=cache)
    assert again["cached"] and again["levels"] == best["levels"]
    s.close()
    # the tuned options keep oracle parity
    log(f"[autotune] per-level choice {best['levels']}")
    prob2 = dict(prob, nchains=4)
    check_stepwise(prob2, None, 2, label="tuned 255^2", levels=best["levels"])
