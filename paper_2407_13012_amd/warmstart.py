"""Learned warm starts for QAOA angle optimisation.

Pipeline (every numerical step runs in the HIP library):

1. ``build_dataset``: the batched engine optimises the depth-p angles of many
   small random weighted MaxCut graphs (n ~ U{10..20}) with on-device Adam
   from the linear ramp, producing (graph, gamma*, beta*) pairs.
2. ``train``: the message-passing network (qaoa_mpnn_*) is fitted to those
   angles with its own GPU forward/backward kernels and Adam.
3. ``evaluate``: on held-out graphs the library's L-BFGS (each evaluation one
   qaoa_gradient call) is run from the linear ramp ("plain") and from the
   network's prediction ("learned"; the ramp is also evaluated and the better
   of the two starts is used, both evaluations counted).  Reported: mean
   approximation ratio E / max C of both, and the gradient evaluations each
   needs to reach the plain run's final ratio minus a tolerance.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, List, Optional

import numpy as np

from ._binding import QaoaBatch, QaoaHandle, QaoaMpnn, qaoa_lbfgs_minimize
from .batch_tune import cost_maxima, options_of, ramp_angles, save_dataset, tune

HERE = os.path.dirname(os.path.abspath(__file__))


class _Graph:
    """Minimal MaxCut record (n, edges, weights) rebuilt from a saved dataset."""

    def __init__(self, n, edges, weights):
        self.n = int(n)
        self.edges = edges
        self.weights = weights

    @property
    def m(self):
        return int(self.edges.shape[0])

    def weight_array(self):
        return np.ones(self.m) if self.weights is None else self.weights


def graphs_of(ds: Dict) -> List[_Graph]:
    off = ds["edge_offsets"]
    return [_Graph(ds["n"][i], ds["edges"][off[i]:off[i + 1]], ds["weights"][off[i]:off[i + 1]])
            for i in range(len(ds["n"]))]


def build_dataset(graphs, p: int, steps: int, tuned: bool = True, log=print) -> Dict:
    """Optimise every graph's angles with the batched engine; returns the dataset arrays."""
    opts = options_of(tune(graphs, p, log=log)) if tuned else {}
    g0, b0 = ramp_angles(len(graphs), p)
    t0 = time.perf_counter()
    with QaoaBatch(graphs, p, steps=steps, **opts) as b:
        gam, bet, e0, e1 = b.run(g0, b0)
    dt = time.perf_counter() - t0
    log(f"[warmstart] batched engine: {len(graphs)} graphs x {steps} Adam steps at p={p} in {dt:.1f} s")
    cmax = cost_maxima(graphs)
    return dict(graphs=graphs, gamma=gam, beta=bet, e_first=e0, e_last=e1, cmax=cmax, seconds=dt)


def train(graphs, gamma, beta, p: int, epochs: int = 30, batch: int = 256, lr: float = 2e-3,
          seed: int = 0, val_frac: float = 0.1, theta0=None, log=print, log_every: int = 1,
          select: str = "last"):
    """Fit the network to (graphs -> gamma, beta).  Returns (params, history): the
    parameters after the last epoch, or with select="best" those of the epoch
    with the lowest validation loss."""
    from qaoa_inputs import mpnn_init_params  # seeded initial weights (inputs, no network arithmetic)
    rng = np.random.default_rng(seed)
    G = len(graphs)
    order = rng.permutation(G)
    nval = max(1, int(val_frac * G))
    val, tr = order[:nval], order[nval:]
    theta = mpnn_init_params(p, seed).astype(np.float32) if theta0 is None else theta0
    hist = []
    with QaoaMpnn(p, theta) as m:
        vg = [graphs[i] for i in val]
        base, _ = m.loss_grad(vg, gamma[val], beta[val], want_grad=False)
        hist.append({"epoch": 0, "val_loss": base})
        best_val, best_params, best_epoch = base, m.get_params(), 0
        t0 = time.perf_counter()
        for ep in range(1, epochs + 1):
            rng.shuffle(tr)
            losses = []
            # cosine learning-rate decay over the epochs
            lr_ep = lr * 0.5 * (1 + np.cos(np.pi * (ep - 1) / epochs))
            for s in range(0, len(tr), batch):
                idx = tr[s:s + batch]
                losses.append(m.train_step([graphs[i] for i in idx], gamma[idx], beta[idx], lr=lr_ep))
            vl, _ = m.loss_grad(vg, gamma[val], beta[val], want_grad=False)
            hist.append({"epoch": ep, "train_loss": float(np.mean(losses)), "val_loss": vl})
            if vl < best_val:  # keep the parameters with the lowest validation loss
                best_val, best_params, best_epoch = vl, m.get_params(), ep
            if ep % log_every == 0 or ep == epochs:
                log(f"[warmstart] epoch {ep}: train {np.mean(losses):.3e} val {vl:.3e}")
        secs = time.perf_counter() - t0
        last_params = m.get_params()
    return (best_params if select == "best" else last_params), {
        "history": hist, "train_seconds": secs, "train_graphs": int(len(tr)), "val_graphs": int(nval),
        "best_epoch": best_epoch, "best_val_loss": best_val, "selected": select}


class _Reached(Exception):
    """Raised inside an L-BFGS evaluation to stop the run once E reaches its target."""


def _lbfgs_counted(h: QaoaHandle, x0, p: int, max_iter: int, gtol: float, stop_at: Optional[float] = None):
    """L-BFGS on -E from x0.  Returns (E_final, E after every evaluation, seconds
    from the start to the end of every evaluation).  With stop_at the run ends
    at the first evaluation whose E reaches it (E_final is then that E)."""
    trace, times = [], []
    t0 = time.perf_counter()

    def fun(x):
        E, dg, db = h.gradient(x[:p], x[p:])
        trace.append(E)
        times.append(time.perf_counter() - t0)
        if stop_at is not None and E >= stop_at:
            raise _Reached()
        return -E, -np.concatenate([dg, db])

    try:
        _, f, _, _ = qaoa_lbfgs_minimize(fun, x0, max_iter=max_iter, gtol=gtol, ftol=1e-12,
                                         max_evals=4 * max_iter)
        E_final = -f
    except _Reached:
        E_final = trace[-1]
    return E_final, np.asarray(trace), np.asarray(times)


def evals_to_reach(trace: np.ndarray, target: float) -> Optional[int]:
    best = np.maximum.accumulate(trace)
    hit = np.nonzero(best >= target)[0]
    return int(hit[0]) + 1 if hit.size else None


def evaluate(params, graphs, p: int, tol: float = 0.005, max_iter: int = 200, gtol: float = 1e-6,
             learned_until_target: bool = False, log=print) -> Dict:
    """Plain (ramp) vs learned starts under the same L-BFGS; see the module docstring.

    The plain run always runs to convergence (its final ratio defines the
    target).  With learned_until_target the learned run stops at the first
    evaluation that reaches the target (time-to-ratio); otherwise it also runs
    to convergence and its final ratio is reported."""
    g_ramp, b_ramp = ramp_angles(1, p)
    x_ramp = np.concatenate([g_ramp[0], b_ramp[0]])
    t0 = time.perf_counter()
    with QaoaMpnn(p, params) as m:
        pg, pb = m.predict(graphs)
    t_predict = time.perf_counter() - t0
    rows = []
    t_plain = t_learned = t_plain_target = t_learned_target = 0.0
    for i, g in enumerate(graphs):
        with QaoaHandle.maxcut(g.n, g.edges, g.weights) as h:
            cmax = h.cost_extrema()[1]
            E_plain, tr_plain, tm_plain = _lbfgs_counted(h, x_ramp, p, max_iter, gtol)
            r_plain = E_plain / cmax
            target = (r_plain - tol) * cmax
            t0 = time.perf_counter()
            x_learn = np.concatenate([pg[i], pb[i]])
            E_l0 = h.evaluate(pg[i], pb[i])
            E_r0 = h.evaluate(g_ramp[0], b_ramp[0])
            t_starts = time.perf_counter() - t0
            start = x_learn if E_l0 >= E_r0 else x_ramp
            if max(E_l0, E_r0) >= target:
                E_learn, tr_learn, tm_learn = max(E_l0, E_r0), np.zeros(0), np.zeros(0)
                if not learned_until_target:
                    E_learn, tr_learn, tm_learn = _lbfgs_counted(h, start, p, max_iter, gtol)
            else:
                E_learn, tr_learn, tm_learn = _lbfgs_counted(
                    h, start, p, max_iter, gtol, stop_at=target if learned_until_target else None)
        t_plain += float(tm_plain[-1])
        t_learned += t_starts + (float(tm_learn[-1]) if tm_learn.size else 0.0)
        r_learn = E_learn / cmax
        n_plain = evals_to_reach(tr_plain, target)
        n_learn = evals_to_reach(np.concatenate([[max(E_l0, E_r0)], tr_learn]), target)
        t_plain_target += float(tm_plain[n_plain - 1])
        if n_learn is None:
            t_learned_target += t_starts + float(tm_learn[-1])
        else:
            t_learned_target += t_starts + (float(tm_learn[n_learn - 2]) if n_learn >= 2 else 0.0)
        rows.append(dict(n=g.n, cmax=cmax, r_plain=r_plain, r_learned=r_learn, r_start_learned=E_l0 / cmax,
                         r_start_ramp=E_r0 / cmax, evals_plain=len(tr_plain), evals_plain_to_target=n_plain,
                         evals_learned_to_target=(None if n_learn is None else n_learn + 1),
                         evals_learned=len(tr_learn) + 2, used_learned_start=bool(E_l0 >= E_r0)))
        if log and (i % 32 == 0 or i == len(graphs) - 1):
            log(f"[warmstart] eval {i + 1}/{len(graphs)}: r_plain {r_plain:.4f} r_learned {r_learn:.4f}")

    def tot(k, full=None):
        # a run that never reaches the target is charged all of its evaluations
        return int(sum(r[k] if r[k] is not None else r[full] for r in rows if r[k] is not None or full))
    reached = [r for r in rows if r["evals_learned_to_target"] is not None]
    return {
        "graphs": len(rows), "p": p, "tolerance": tol, "learned_until_target": learned_until_target,
        "mean_ratio_plain": float(np.mean([r["r_plain"] for r in rows])),
        "mean_ratio_learned": float(np.mean([r["r_learned"] for r in rows])),
        "mean_start_ratio_ramp": float(np.mean([r["r_start_ramp"] for r in rows])),
        "mean_start_ratio_learned": float(np.mean([r["r_start_learned"] for r in rows])),
        "total_evals_plain": tot("evals_plain"),
        "total_evals_plain_to_target": tot("evals_plain_to_target", "evals_plain"),
        "total_evals_learned_to_target": tot("evals_learned_to_target", "evals_learned"),
        "learned_reached_target": len(reached),
        "seconds_plain": t_plain, "seconds_learned": t_learned + t_predict, "seconds_predict": t_predict,
        "seconds_plain_to_target": t_plain_target, "seconds_learned_to_target": t_learned_target + t_predict,
        "rows": rows,
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default="warmstart_out")
    ap.add_argument("--train-graphs", type=int, default=4096)
    ap.add_argument("--select", choices=["last", "best"], default="last")
    ap.add_argument("--train-steps", type=int, default=300)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--min-ratio", type=float, default=0.5)
    ap.add_argument("--eval-graphs", type=int, default=512)
    ap.add_argument("--eval-n", type=int, default=24)
    ap.add_argument("--max-iter", type=int, default=200)
    args = ap.parse_args(argv)
    import qaoa_inputs as qi
    os.makedirs(args.out, exist_ok=True)

    def log(msg):
        print(msg, flush=True)

    graphs = qi.batched_family(args.train_graphs)
    ds = build_dataset(graphs, args.p, args.train_steps, log=log)
    save_dataset(os.path.join(args.out, f"dataset_p{args.p}.npz"), graphs, args.p, ds["gamma"], ds["beta"],
                 ds["e_first"], ds["e_last"], ds["cmax"],
                 meta={"adam_steps": args.train_steps, "engine_seconds": ds["seconds"]})
    cm = np.maximum(ds["cmax"], 1e-9)
    log(f"[warmstart] dataset median ratio {np.median(ds['e_last'] / cm):.4f} "
        f"(start {np.median(ds['e_first'] / cm):.4f})")
    # graphs whose optimisation stayed poor (tiny max C, or a run that did not
    # reach min_ratio) carry little information about good angles
    ratio = ds["e_last"] / np.maximum(ds["cmax"], 1e-9)
    keep = np.nonzero(ratio >= args.min_ratio)[0]
    log(f"[warmstart] training on {keep.size} of {len(graphs)} graphs (final ratio >= {args.min_ratio})")
    params, info = train([graphs[i] for i in keep], ds["gamma"][keep], ds["beta"][keep], args.p,
                         epochs=args.epochs, batch=args.batch, lr=args.lr, log=log,
                         log_every=max(1, args.epochs // 20), select=args.select)
    np.save(os.path.join(args.out, f"mpnn_p{args.p}.npy"), params)
    ev_graphs = qi.warmstart_eval_graphs(args.eval_graphs, args.eval_n)
    res = evaluate(params, ev_graphs, args.p, max_iter=args.max_iter, log=log)
    res["training"] = info
    res["dataset"] = {"graphs": len(graphs), "adam_steps": args.train_steps, "engine_seconds": ds["seconds"],
                      "median_ratio_start": float(np.median(ds["e_first"] / np.maximum(ds["cmax"], 1e-9))),
                      "median_ratio_final": float(np.median(ds["e_last"] / np.maximum(ds["cmax"], 1e-9))),
                      "training_graphs_kept": int(keep.size)}
    with open(os.path.join(args.out, "warmstart_eval.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    summary = {k: v for k, v in res.items() if k != "rows"}
    log(json.dumps(summary))
    return 0


if __name__ == "__main__":
    sys.exit(main())
