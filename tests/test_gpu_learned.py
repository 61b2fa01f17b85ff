"""What the trained prolongation network gains over multilinear P, and
what any transfer could gain on this workload.

Trains the network with the library's own kernels on seeded log-normal
fields (correlation length 0.05, variance 2, kappa = 1, as the learned
prolongation workload, at 255^2 to keep the test short), then compares on
held-out fields: the two-grid loss, and the IACT of the MGMC chains with
learned and with multilinear P.  Whatever P, the target stays the same
(test_learned_weights_drive_the_sampler checks the chains against the
oracle), so only efficiency can change.
"""
import sys

import numpy as np
import pytest

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


def test_training_gain_on_held_out_fields():
    from paper_2407_12149_amd import learned
    cfg = dict(workloads.config("learned511"))
    n = 255
    cfg.update(n=n, levels=6, F=workloads.subcube_qoi(n, 2))
    log(f"[learned] n={n}: 32 training fields, 4 held out")
    host = learned.fields(cfg, 0, 32)
    faces = torch.as_tensor(host, device="cuda")
    errs = torch.stack([learned.chain_errors(cfg, host[k], 4, seed=1000 + k) for k in range(32)])
    hold_host = learned.fields(cfg, cfg["train_fields"], 4)
    hold = torch.as_tensor(hold_host, device="cuda")
    herr = torch.stack([learned.chain_errors(cfg, hold_host[k], 4, seed=5000 + k) for k in range(4)])
    base = learned.mean_loss(cfg, learned.multilinear_params(), hold, herr)
    params, hist = learned.train(cfg, faces, errs, 200, batch=4, lr=1e-3)
    after = learned.mean_loss(cfg, params, hold, herr)
    log(f"[learned] held-out two-grid loss: multilinear {base:.6f}, learned {after:.6f}")
    assert np.isfinite(after) and after < base
    res = learned.evaluate(cfg, hold_host, params, nchains=8, nsamples=2000, burn=200,
                           operator=True)
    ml = np.array([r["multilinear"]["iact"] for r in res])
    le = np.array([r["learned"]["iact"] for r in res])
    op = np.array([r["operator"]["iact"] for r in res])
    log(f"[learned] held-out IACT: multilinear {ml.mean():.4f}, learned {le.mean():.4f}, "
        f"operator-dependent {op.mean():.4f}")
    assert not any(r["fallback"] for r in res)
    # What a better transfer can gain here: Dendy's operator-dependent P,
    # which adapts to the coefficient exactly, changes the IACT by less than
    # 2% on these well-resolved fields (12 fields at 511^2: 0.09% +- 0.04%),
    # so no trained P can gain more on this workload ...
    headroom = ml / op
    assert np.all(np.abs(headroom - 1.0) < 0.02), headroom
    # ... and the trained network, which starts from multilinear P, must not
    # lose against it beyond the paired spread of the fields
    d = le - ml
    assert d.mean() <= 3 * d.std(ddof=1) / np.sqrt(len(d)) + 0.01 * ml.mean(), d
