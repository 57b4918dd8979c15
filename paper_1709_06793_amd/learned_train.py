"""Training and evaluation of the learned smoothing correction.

Training data: for each coefficient field (lognormal, random sigma and
correlation length drawn from the field's seed) on the 6-tet Kuhn cube, a
random right-hand side, the FP64 solution u* (V-cycles to 1e-12), then plain
V(2,2) Chebyshev cycles from u = 0; at the start of each of the first cycles
the pair (r = f - A u, e = u* - u) is kept in FP32.  The network is trained
with Adam on the energy of the error after one learned step,
L = e1^T A e1 / e^T A e, e1 = e - D^{-1}(omega r + s c); every loss and
gradient is computed by the library's kernels (forward, scaled apply,
backward), the optimizer step by the library's host code.

Evaluation: FP32-in-FP64 solves to a relative residual of 1e-8 with the
learned smoother on the finest level against the same solve with the network
switched off (zero weights: plain damped Jacobi steps) and against plain
Chebyshev smoothing, per-cycle contraction and fallback events.
"""
import time

import numpy as np

from . import hhg


def make_field_context(level, seed, mesh_fn, torch):
    """Context with the lognormal field of `seed` (sigma ~ U(0.5,2), l_c ~ U(0.05,0.3))
    and a random right-hand side drawn from the same stream."""
    from hhg_inputs import lognormal_params, lognormal_k
    X, T = mesh_fn()
    ctx = hhg.Context(X, T, level)
    xyz, dirichlet = ctx.node_coords(level)
    prm = lognormal_params(seed)
    ctx.set_coefficient(lognormal_k(xyz, prm))
    f = prm["rng"].uniform(-1, 1, xyz.shape[0])
    f[dirichlet] = 0.0
    fd = ctx.from_canonical(level, torch.tensor(f, device="cuda"))
    return ctx, fd, prm


def generate_samples(level, seeds, mesh_fn, torch, cycles=5, noise=3, log=None):
    """[(ctx, [(r32, e32), ...], f), ...] for the given field seeds: `cycles`
    pairs from plain V-cycles (smooth errors) and `noise` pairs with a uniform
    random error (rough errors, as the smoother sees after a coarse-grid
    correction); every pair satisfies r = A e."""
    out = []
    for q, seed in enumerate(seeds):
        ctx, f, prm = make_field_context(level, seed, mesh_fn, torch)
        us = ctx.vector(level)
        ctx.solve(level, f, us, mode=hhg.SOLVE_F64, tol=1e-12, max_iter=200)
        u = ctx.vector(level)
        pairs = []
        for _ in range(cycles):
            r32 = ctx.vector(level, torch.float32)
            e32 = ctx.vector(level, torch.float32)
            ctx.training_pair(level, f, u, us, r32, e32)
            pairs.append((r32, e32))
            ctx.vcycle(level, f, u, 2, 2, hhg.CHEBYSHEV)
        zero = ctx.vector(level)
        n_nodes = ctx.sizes(level)["n_nodes"]
        for _ in range(noise):
            # u = -e (consistent, 0 on Dirichlet slots), u* = 0, f = 0: r = A e
            e = prm["rng"].uniform(-1, 1, n_nodes)
            mu = ctx.from_canonical(level, torch.tensor(-e, device="cuda"))
            r32 = ctx.vector(level, torch.float32)
            e32 = ctx.vector(level, torch.float32)
            ctx.training_pair(level, zero, mu, zero, r32, e32)
            pairs.append((r32, e32))
        out.append((ctx, pairs, f))
        if log and (q + 1) % 16 == 0:
            log(f"samples: {q + 1}/{len(seeds)} fields")
    return out


def init_weights(seed=0):
    """Glorot-uniform layers 1-2, zero biases, zero output layer (c = 0 at start)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(hhg.LEARNED_NPARAM, dtype=np.float32)
    a1 = np.sqrt(6.0 / 48.0)
    w[:512] = rng.uniform(-a1, a1, 512)
    a2 = np.sqrt(6.0 / 32.0)
    w[528:784] = rng.uniform(-a2, a2, 256)
    return w


def train(data, level, epochs=20, lr=2e-3, seed=0, w0=None, log=None):
    """Adam on the one-step energy loss; returns (weights, per-epoch mean loss)."""
    w = init_weights(seed) if w0 is None else np.array(w0, dtype=np.float32)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    rng = np.random.default_rng(seed + 1)
    items = [(ci, pi) for ci in range(len(data)) for pi in range(len(data[ci][1]))]
    hist = []
    t = 0
    for ep in range(epochs):
        order = rng.permutation(len(items))
        tot = 0.0
        t0 = time.time()
        for idx in order:
            ci, pi = items[idx]
            ctx, pairs = data[ci][:2]
            r, e = pairs[pi]
            ctx.learned_set_weights(w)
            loss, g = ctx.learned_loss_grad(level, r, e)
            if not np.all(np.isfinite(g)):
                continue
            t += 1
            hhg.adam_update(w, m, v, g, t, lr=lr)
            tot += loss
        hist.append(tot / len(items))
        if log:
            log(f"epoch {ep}: mean one-step energy ratio {hist[-1]:.5f} ({time.time() - t0:.1f} s)")
    return w, hist


def mean_loss(data, level, w):
    tot, n = 0.0, 0
    for ctx, pairs, _ in data:
        ctx.learned_set_weights(w)
        for r, e in pairs:
            loss, _ = ctx.learned_loss_grad(level, r, e)
            tot += loss
            n += 1
    return tot / n


def evaluate(ctx, f, level, w, torch, tol=1e-8, max_iter=200, margin=1.05):
    """FP32-in-FP64 solves with the learned smoother, with the network off
    (damped Jacobi steps) and with plain Chebyshev; returns the stats dicts.
    The learned solve runs with the library's fallback (a cycle that does not
    reduce the residual switches the solve to Chebyshev, and with margin > 0
    so does one that contracts worse than margin x the plain cycle measured
    from the same iterate); the network-off reference never falls back."""
    res = {}
    u = ctx.vector(level)
    res["chebyshev"] = ctx.solve(level, f, u, mode=hhg.SOLVE_MIXED, tol=tol, max_iter=max_iter)
    for name, wv, rate, margin in (("learned", w, 1.0, margin), ("network_off", np.zeros_like(w), 1e30, 0.0)):
        ctx.learned_set_weights(wv)
        ctx.learned_set_fallback(rate, margin)
        u = ctx.vector(level)
        res[name] = ctx.solve(level, f, u, mode=hhg.SOLVE_LEARNED, tol=tol, max_iter=max_iter)
    return res


# ---------------------------------------------------------------- full training / evaluation runs
WEIGHTS_PATH = __import__("os").path.join(__import__("os").path.dirname(__file__), "learned_weights.json")


def save_weights(w, path, meta):
    import json
    with open(path, "w") as fh:
        json.dump({"nparam": int(w.size), "weights": [float(x) for x in w], "meta": meta}, fh)


def load_weights(path=WEIGHTS_PATH):
    """Trained parameters shipped with the package (float32, 817 values)."""
    import json
    with open(path) as fh:
        d = json.load(fh)
    w = np.asarray(d["weights"], dtype=np.float32)
    if w.size != hhg.LEARNED_NPARAM:
        raise ValueError(f"{path}: {w.size} parameters, expected {hhg.LEARNED_NPARAM}")
    return w, d.get("meta", {})


def evaluate_fields(level, seeds, w, torch, mesh_fn, tol=1e-8, log=None):
    """Learned vs Chebyshev vs network-off solves on one context per mesh,
    re-used across fields (set_coefficient per field)."""
    from hhg_inputs import lognormal_params, lognormal_k
    X, T = mesh_fn()
    ctx = hhg.Context(X, T, level)
    xyz, dirichlet = ctx.node_coords(level)
    out = []
    for q, seed in enumerate(seeds):
        prm = lognormal_params(seed)
        ctx.set_coefficient(lognormal_k(xyz, prm))
        f = prm["rng"].uniform(-1, 1, xyz.shape[0])
        f[dirichlet] = 0.0
        fd = ctx.from_canonical(level, torch.tensor(f, device="cuda"))
        res = evaluate(ctx, fd, level, w, torch, tol=tol)
        u = ctx.vector(level)
        res["f64"] = ctx.solve(level, fd, u, mode=hhg.SOLVE_F64, tol=tol, max_iter=200)
        res["seed"] = seed
        res["sigma"] = float(prm["sigma"])
        res["corr_len"] = float(prm["corr_len"])
        out.append(res)
        if log:
            log(f"eval field {seed}: iterations learned {res['learned']['iterations']} chebyshev "
                f"{res['chebyshev']['iterations']} off {res['network_off']['iterations']}; seconds learned "
                f"{res['learned']['seconds']:.3f} chebyshev {res['chebyshev']['seconds']:.3f} "
                f"f64 {res['f64']['seconds']:.3f}; fallback {res['learned']['fallback']}")
    return out


def summarize(results):
    def col(name, key):
        return np.array([r[name][key] for r in results], dtype=float)
    s = {"fields": len(results)}
    for name in ("learned", "chebyshev", "network_off", "f64"):
        s[name] = {"mean_iterations": float(col(name, "iterations").mean()),
                   "mean_seconds": float(col(name, "seconds").mean()),
                   "median_rho": float(np.median(col(name, "rho"))),
                   "max_rel_residual": float(col(name, "rel_residual").max()),
                   "fallbacks": int(col(name, "fallback").sum())}
    s["learned_fewer_iterations_than_chebyshev"] = int((col("learned", "iterations") < col("chebyshev", "iterations")).sum())
    s["learned_faster_than_chebyshev"] = int((col("learned", "seconds") < col("chebyshev", "seconds")).sum())
    s["learned_faster_than_f64"] = int((col("learned", "seconds") < col("f64", "seconds")).sum())
    return s


def main(argv=None):
    """python -m paper_1709_06793_amd.learned_train {train,eval} ...

    train: fields 100..355 (256) on the 6-tet Kuhn cube at level 6, Adam on
    the one-step energy loss, weights written to learned_weights.json.
    eval: held-out fields 1000..1031 at level 8, learned vs Chebyshev vs
    network-off (all FP32-in-FP64) and plain FP64 solves to 1e-8."""
    import argparse
    import json
    import sys
    import torch
    from hhg_inputs import kuhn_cube
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["train", "eval"])
    ap.add_argument("--level", type=int, default=None)
    ap.add_argument("--first-seed", type=int, default=None)
    ap.add_argument("--fields", type=int, default=None)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=WEIGHTS_PATH)
    ap.add_argument("--weights", default=WEIGHTS_PATH)
    ap.add_argument("--json", default=None, help="write the evaluation records here")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    torch.cuda.set_device(0)
    if a.what == "train":
        level = a.level or 6
        s0 = 100 if a.first_seed is None else a.first_seed
        nf = a.fields or 256
        t0 = time.time()
        data = generate_samples(level, list(range(s0, s0 + nf)), kuhn_cube, torch, log=log)
        log(f"samples ready: {nf} fields, {sum(len(p) for _, p, _ in data)} pairs ({time.time() - t0:.1f} s)")
        w, hist = train(data, level, epochs=a.epochs, lr=a.lr, log=log)
        meta = {"level": level, "fields": [s0, s0 + nf - 1], "epochs": a.epochs, "lr": a.lr,
                "loss_history": [float(h) for h in hist], "mesh": "6-tet Kuhn unit cube",
                "pairs_per_field": "5 V(2,2)-cycle pairs + 3 random-error pairs"}
        save_weights(w, a.out, meta)
        log(json.dumps({"trained": a.out, "final_loss": hist[-1], "seconds": time.time() - t0}))
        return 0
    level = a.level or 8
    s0 = 1000 if a.first_seed is None else a.first_seed
    nf = a.fields or 32
    w, meta = load_weights(a.weights)
    res = evaluate_fields(level, list(range(s0, s0 + nf)), w, torch, kuhn_cube, log=log)
    summ = summarize(res)
    if a.json:
        with open(a.json, "w") as fh:
            json.dump({"summary": summ, "fields": res, "weights_meta": meta}, fh, indent=1)
    log(json.dumps(summ))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
