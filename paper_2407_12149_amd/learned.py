"""Learned prolongation workflow on the GPU: training data from the plain
sampler, training with the library's own network kernels, and evaluation
against multilinear prolongation by integrated autocorrelation time.

Any full-rank prolongation with Galerkin coarse operators leaves the target
invariant (Sec. 4.2; transfers are not unique, Sec. 3.1), so the learned
weights can only change the mixing speed; multilinear P is the fallback
whenever the network yields non-finite weights.

Training errors are states of the plain (multilinear) MGMC prior chain on each
training field: with mean zero a state is its own error, drawn from the target
N(0, A^{-1}).  The loss is the two-grid error reduction
||S_b T S_f e||_A^2 / ||e||_A^2 on 15 x 15 coarse crops (see
mgmc_pnet_loss_grad in include/mgmc.h); the smoothers matter: the coarse
correction T alone can be improved by weights that slow the V-cycle down.

Command line (writes a parameter file the benchmark and tests can load):

    python -m paper_2407_12149_amd.learned train --out weights.npy [--fields 400 ...]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import diagnostics, mgmc, workloads

NPARAM_SHAPES = [(16, 24, 9), (16,), (16, 16, 9), (16,), (9, 16, 9), (9,)]


def init_params(seed):
    """Random hidden layers and a zero output layer whose bias makes
    softplus = 1: training starts from multilinear interpolation exactly."""
    rng = np.random.default_rng(seed)
    out = []
    for s in NPARAM_SHAPES:
        if len(s) == 3 and s[0] != 9:
            out.append(rng.normal(0.0, 1.0 / np.sqrt(s[1] * 9), size=s))
        else:
            out.append(np.zeros(s))
    out[5][:] = np.log(np.expm1(1.0))
    return np.concatenate([a.reshape(-1) for a in out]).astype(np.float32)


def field(cfg, k):
    """Face coefficients of field k of a learned-prolongation workload."""
    return workloads.lognormal_faces_fft(cfg["n"], 2, cfg["corr_len"], cfg["variance"],
                                         seed=cfg["field_seed0"] + k)


def fields(cfg, start, count, workers=8):
    """Fields start .. start+count-1 (threads: the FFTs release the GIL)."""
    import concurrent.futures as cf
    if count <= 2 or workers <= 1:
        return np.stack([field(cfg, start + k) for k in range(count)])
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return np.stack(list(ex.map(lambda k: field(cfg, start + k), range(count))))


def problem(cfg, face, prolong_w=None, nchains=1, seed=0, precision="fp64"):
    return dict(dim=2, n=cfg["n"], levels=cfg["levels"], kappa2=cfg["kappa2"], face_coef=face,
                prolong_w=prolong_w, nchains=nchains, seed=seed, precision=precision)


def chain_errors(cfg, face, nerr, burn=4, seed=0):
    """nerr states of the plain (multilinear) MGMC prior chain on this field,
    one chain per error, after `burn` updates: with mean zero a state is its
    own error, drawn from the target N(0, A^{-1})."""
    import torch
    s = mgmc.Sampler(problem(cfg, face, nchains=nerr, seed=seed))
    s.sample(0, burn, want_qoi=False)
    torch.cuda.synchronize()
    out = s.theta.detach().clone()
    s.close()
    return out


def train(cfg, faces, errors, steps, batch=4, lr=2e-3, params=None, log=None, seed=0):
    """Adam on the two-grid loss over minibatches of (field, its errors).
    faces: device [F][2 (n+1) n]; errors: device [F][K][n*n].  Returns the
    parameters and the loss history."""
    import torch
    n = cfg["n"]
    F, K = faces.shape[0], errors.shape[1]
    net = mgmc.PNet(n, max_batch=batch, max_errors=K,
                    params=init_params(seed) if params is None else params)
    rng = np.random.default_rng(seed + 17)
    hist = []
    for it in range(steps):
        pick = torch.as_tensor(rng.choice(F, size=min(batch, F), replace=False), device=faces.device)
        loss = net.train_step(faces[pick], errors[pick], cfg["kappa2"], lr)
        hist.append(loss)
        if log and (it % 50 == 0 or it == steps - 1):
            log(f"[learned] step {it} loss {loss:.5f}")
    p = net.params()
    net.close()
    return p, hist


def mean_loss(cfg, params, faces, errors):
    """Two-grid loss of a parameter set averaged over the given fields (no update)."""
    n = cfg["n"]
    net = mgmc.PNet(n, max_batch=1, max_errors=errors.shape[1], params=params)
    tot = 0.0
    for k in range(faces.shape[0]):
        loss, _ = net.loss_grad(faces[k:k + 1], errors[k:k + 1], cfg["kappa2"], want_grad=False)
        tot += loss
    net.close()
    return tot / faces.shape[0]


def multilinear_params():
    """Parameters whose network output is constant: multilinear P exactly."""
    p = np.zeros(sum(int(np.prod(s)) for s in NPARAM_SHAPES), dtype=np.float32)
    p[-9:] = np.log(np.expm1(1.0))
    return p


def prolong_weights(cfg, params, face):
    """Learned weights of the finest transfer (prolong_w layout), or None when
    the network gives a non-finite value (multilinear fallback)."""
    import torch
    net = mgmc.PNet(cfg["n"], params=params)
    w = net.weights(torch.as_tensor(face, device="cuda")).cpu().numpy()[0]
    net.close()
    return w.reshape(-1) if np.all(np.isfinite(w)) else None


def evaluate(cfg, faces_host, params, nchains=4, nsamples=2000, burn=500, precision="fp64",
             log=None, operator=False):
    """IACT and ESS/s of multilinear vs learned P on each field (QoI = mean
    over the central sub-square), both samplers of a field run as branches
    of one batch.  Returns a list of per-field dicts."""
    import torch
    F = torch.as_tensor(cfg["F"], device="cuda")
    res = []
    for k, face in enumerate(faces_host):
        w = prolong_weights(cfg, params, face) if params is not None else None
        row = {"field": k, "fallback": w is None}
        cands = [("multilinear", None), ("learned", w)]
        if operator:
            cands.append(("operator", operator_weights(cfg, face)))
        for name, pw in cands:
            s = mgmc.Sampler(problem(cfg, face, prolong_w=pw, nchains=nchains, seed=k,
                                     precision=precision))
            s.set_graph(True)
            s.sample(0, burn, want_qoi=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            q = s.sample(burn, nsamples, F=F)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            qs = q.cpu().numpy()
            taus = [diagnostics.iact_wolff(qs[:, c])[0] for c in range(nchains)]
            tau = float(np.mean(taus))
            row[name] = {"iact": tau, "ms_per_step": sec * 1e3 / nsamples,
                         "ess_per_s": nsamples * nchains / (tau * sec)}
            s.close()
        if log:
            log(f"[learned] field {k}: iact multilinear {row['multilinear']['iact']:.3f} "
                f"learned {row['learned']['iact']:.3f}"
                + (f" operator {row['operator']['iact']:.3f}" if operator else ""))
        res.append(row)
    return res


def operator_weights(cfg, face):
    """Operator-dependent ("black box", Dendy 1982) weights of the finest
    transfer in the prolong_w layout, from the 5-point operator
    s (kappa^2 - div(a grad)) of this field: a fine node between two coarse
    nodes along x takes -A_(i, toward J) / (A_ii + A_(i,S) + A_(i,N)) (the
    stencil collapsed across the other axis), likewise along y, and a node at
    a cell centre -(A_(i,x-edge) P(x-edge node, J) + A_(i,y-edge) P(y-edge
    node, J)) / A_ii.  For a = 1 and kappa h -> 0 these are the multilinear
    weights.  A reference transfer that adapts to the coefficient without
    training: the headroom an operator-aware P could give."""
    n = cfg["n"]
    nc = (n - 1) // 2
    h = 1.0 / (n + 1)
    s = h * h
    per = (n + 1) * n
    ax = face[:per].reshape(n, n + 1)      # [y][x face]
    ay = face[per:2 * per].reshape(n + 1, n)  # [y face][x]
    ih2 = 1.0 / (h * h)
    # stencil of fine node (x, y), 1-based coordinates
    def W(x, y): return -s * ih2 * ax[y - 1, x - 1]
    def E(x, y): return -s * ih2 * ax[y - 1, x]
    def S(x, y): return -s * ih2 * ay[y - 1, x - 1]
    def N(x, y): return -s * ih2 * ay[y, x - 1]
    def C(x, y): return s * (cfg["kappa2"] + ih2 * (ax[y - 1, x - 1] + ax[y - 1, x] + ay[y - 1, x - 1] + ay[y, x - 1]))
    J1, J2 = np.meshgrid(np.arange(1, nc + 1), np.arange(1, nc + 1), indexing="xy")
    J1, J2 = J1.reshape(-1), J2.reshape(-1)
    w = np.zeros((nc * nc, 9))
    edge = {}
    for dx in (-1, 1):  # x-edge nodes 2J + (dx, 0)
        x, y = 2 * J1 + dx, 2 * J2
        toward = W(x, y) if dx == 1 else E(x, y)
        edge[(dx, 0)] = -toward / (C(x, y) + S(x, y) + N(x, y))
    for dy in (-1, 1):  # y-edge nodes 2J + (0, dy)
        x, y = 2 * J1, 2 * J2 + dy
        toward = S(x, y) if dy == 1 else N(x, y)
        edge[(0, dy)] = -toward / (C(x, y) + W(x, y) + E(x, y))
    for (dx, dy), v in edge.items():
        w[:, (dx + 1) + 3 * (dy + 1)] = v
    w[:, 4] = 1.0
    for dx in (-1, 1):
        for dy in (-1, 1):
            x, y = 2 * J1 + dx, 2 * J2 + dy
            ax_e = W(x, y) if dx == 1 else E(x, y)  # coupling to the y-edge node 2J + (0, dy)
            ay_e = S(x, y) if dy == 1 else N(x, y)  # coupling to the x-edge node 2J + (dx, 0)
            w[:, (dx + 1) + 3 * (dy + 1)] = -(ax_e * edge[(0, dy)] + ay_e * edge[(dx, 0)]) / C(x, y)
    return w.reshape(-1)


def save_params(path, params, meta=None):
    np.save(path, np.asarray(params, dtype=np.float32), allow_pickle=False)
    if meta is not None:
        with open(os.path.splitext(path)[0] + ".json", "w") as fh:
            json.dump(meta, fh, indent=1, sort_keys=True)


def load_params(path):
    p = np.load(path, allow_pickle=False)
    if p.dtype != np.float32 or p.ndim != 1:
        raise ValueError("parameter file must hold a float32 vector")
    return p


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train"])
    ap.add_argument("--workload", default="learned511")
    ap.add_argument("--out", required=True)
    ap.add_argument("--fields", type=int, default=400, help="training fields (of the workload's 2000)")
    ap.add_argument("--errors", type=int, default=4, help="chain states per field")
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--holdout", type=int, default=8, help="held-out fields scored by the loss")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    import torch

    def log(msg):
        print(msg, flush=True)

    cfg = workloads.config(args.workload)
    n = cfg["n"]
    log(f"[learned] generating {args.fields} training fields of {n}^2")
    t0 = time.perf_counter()
    host = fields(cfg, 0, args.fields)
    faces = torch.as_tensor(host, device="cuda")
    log(f"[learned] fields done in {time.perf_counter() - t0:.1f} s; drawing chain errors")
    errs = torch.empty((args.fields, args.errors, n * n), dtype=torch.float64, device="cuda")
    for k in range(args.fields):
        errs[k] = chain_errors(cfg, host[k], args.errors, seed=1000 + k)
        if k % 50 == 0:
            log(f"[learned] errors for field {k}")
    hold_host = fields(cfg, cfg["train_fields"], args.holdout)
    hold = torch.as_tensor(hold_host, device="cuda")
    herr = torch.stack([chain_errors(cfg, hold_host[k], args.errors, seed=5000 + k)
                        for k in range(args.holdout)])
    base = mean_loss(cfg, multilinear_params(), hold, herr)
    log(f"[learned] held-out loss with multilinear P: {base:.5f}")
    params, hist = train(cfg, faces, errs, args.steps, batch=args.batch, lr=args.lr, log=log,
                         seed=args.seed)
    after = mean_loss(cfg, params, hold, herr)
    log(f"[learned] held-out loss with learned P: {after:.5f}")
    meta = {"workload": args.workload, "fields": args.fields, "errors": args.errors,
            "steps": args.steps, "batch": args.batch, "lr": args.lr, "seed": args.seed,
            "holdout_loss_multilinear": base, "holdout_loss_learned": after,
            "train_loss_first": hist[0], "train_loss_last": hist[-1]}
    save_params(args.out, params, meta)
    log(json.dumps(meta))
    return 0


if __name__ == "__main__":
    sys.exit(main())
