"""Autotuner and dataset driver for the batched engine (qaoa_batch_*).

The engine's launch is shaped by a few knobs that only measurement can settle
on a given device:

* the fusion depth of the mixer passes per qubit count n (``group_by_n``):
  a layer of an n-qubit instance, n > 12, is applied as one low pass of 12
  qubits plus ceil((n - 12) / k) high passes of at most k qubits each, so
  smaller k means more, narrower passes over the slot;
* the register budget of the engine kernel (``waves_per_simd``, 1 or 2);
* the number of persistent workgroups (``workgroups``);
* the largest n run LDS-resident (``resident_max_n``, 0 or 12): instances of
  at most 12 qubits are one tile, and may either stream through their slot
  between passes within the main launch or keep both vectors in LDS in a
  second launch of one workgroup per compute unit.

``tune`` times short runs of the actual batch (a couple of Adam steps per
instance) over these candidates, keeps the fastest, and caches the choice in a
JSON file keyed by the device and the batch's size histogram and depth.
All arithmetic runs in the HIP library; this module only picks options, times
calls and moves results.
"""
from __future__ import annotations

import json
import os
import time
from collections import Counter
from typing import Dict, Optional, Sequence

import numpy as np

from ._binding import QaoaBatch, QaoaHandle

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning", "batch_mi355x.json")
DEPTHS = (4, 6, 8, 10)


def device_key() -> str:
    """Architecture and CU count (the marketing name depends on the host's
    device-id tables, so it is left out)."""
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "").split(":")[0]
    return f"{arch}|cu{props.multi_processor_count}"


def batch_key(graphs, p: int) -> str:
    hist = Counter(int(g.n) for g in graphs)
    return f"p{p};" + ",".join(f"{n}:{hist[n]}" for n in sorted(hist))


def _time_run(graphs, p, g0, b0, steps, **opt) -> float:
    import torch
    with QaoaBatch(graphs, p, steps=steps, **opt) as b:
        b.run(g0, b0)  # warm-up (first launch, graph upload)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(g0, b0)
        return time.perf_counter() - t0


def ramp_angles(count: int, p: int):
    """Linear-ramp start angles gamma_i = i/p, beta_i = 1 - i/p (i = 1..p), per instance."""
    i = np.arange(1, p + 1, dtype=np.float64)
    return np.tile(i / p, (count, 1)), np.tile(1.0 - i / p, (count, 1))


def tune(graphs: Sequence, p: int, cache: Optional[str] = DEFAULT_CACHE, probe_steps: int = 2,
         force: bool = False, log=None) -> Dict:
    """Return the fastest measured options for this batch (from the cache when
    present).  The result is a dict of QaoaBatch keyword arguments plus the
    timings that chose it under "measured"."""
    import torch
    log = log or (lambda *a: None)
    dkey, bkey = device_key(), batch_key(graphs, p)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
        hit = table.get(dkey, {}).get(bkey)
        if hit is not None and not force and "resident_max_n" in hit:
            return hit
    measured = {"depth": {}, "launch": {}, "resident": {}}
    ns = sorted({int(g.n) for g in graphs})
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    group_by_n = {}
    # 1) fusion depth per n > 12, on that n's instances alone
    for n in ns:
        if n <= 12:
            continue
        sub = [g for g in graphs if g.n == n][: 2 * cus]
        g0, b0 = ramp_angles(len(sub), p)
        best, best_t = 10, None
        seen = set()
        for k in sorted(DEPTHS, reverse=True):
            passes = -(-(n - 12) // k)  # equal pass counts give the same (balanced) plan
            if passes in seen:
                continue
            seen.add(passes)
            t = _time_run(sub, p, g0, b0, probe_steps, max_group=k)
            measured["depth"][f"{n}:{k}"] = t
            log(f"[tune] n={n} depth={k}: {1e3 * t:.2f} ms")
            if best_t is None or t < best_t:
                best, best_t = k, t
        group_by_n[n] = best
    # 2) register budget and persistent grid size on the whole batch
    g0, b0 = ramp_angles(len(graphs), p)
    best = None
    for wpe in (1, 2):
        for wg in (cus, 2 * cus):
            t = _time_run(graphs, p, g0, b0, probe_steps, waves_per_simd=wpe, workgroups=wg,
                          group_by_n=group_by_n, resident_max_n=0)
            measured["launch"][f"wpe{wpe}:wg{wg}"] = t
            log(f"[tune] waves_per_simd={wpe} workgroups={wg}: {1e3 * t:.2f} ms")
            if best is None or t < best[0]:
                best = (t, wpe, wg)
    # 3) one-tile instances streamed within that launch or LDS-resident after it
    resident = 0
    if min(ns) <= 12:
        t_res = _time_run(graphs, p, g0, b0, probe_steps, waves_per_simd=best[1], workgroups=best[2],
                          group_by_n=group_by_n, resident_max_n=12)
        measured["resident"] = {"0": best[0], "12": t_res}
        log(f"[tune] resident_max_n=12: {1e3 * t_res:.2f} ms (streamed: {1e3 * best[0]:.2f} ms)")
        resident = 12 if t_res < best[0] else 0
    choice = {"group_by_n": {str(k): v for k, v in group_by_n.items()}, "waves_per_simd": best[1],
              "workgroups": best[2], "resident_max_n": resident, "probe_steps": probe_steps,
              "measured": measured}
    if cache:
        table.setdefault(dkey, {})[bkey] = choice
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return choice


def options_of(choice: Dict) -> Dict:
    """QaoaBatch keyword arguments of a tuning result."""
    return {"group_by_n": {int(k): int(v) for k, v in choice["group_by_n"].items()},
            "waves_per_simd": int(choice["waves_per_simd"]), "workgroups": int(choice["workgroups"]),
            "resident_max_n": int(choice.get("resident_max_n", 0))}


def cost_maxima(graphs) -> np.ndarray:
    """max_z C(z) of every graph, from the library's cost diagonal reduction."""
    out = np.empty(len(graphs))
    for i, g in enumerate(graphs):
        with QaoaHandle.maxcut(g.n, g.edges, g.weights) as h:
            out[i] = h.cost_extrema()[1]
    return out


def save_dataset(path: str, graphs, p: int, gamma, beta, e_first, e_last, cmax=None, meta=None):
    """Write the (graph, gamma*, beta*) dataset as a plain .npz (no pickled objects)."""
    n = np.asarray([g.n for g in graphs], dtype=np.int32)
    m = np.asarray([g.m for g in graphs], dtype=np.int64)
    off = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum(m, out=off[1:])
    edges = np.concatenate([np.asarray(g.edges, np.int32).reshape(-1, 2) for g in graphs])
    w = np.concatenate([g.weight_array() for g in graphs])
    arrays = dict(n=n, edge_offsets=off, edges=edges, weights=w, p=np.int32(p),
                  gamma=np.asarray(gamma), beta=np.asarray(beta), e_first=np.asarray(e_first),
                  e_last=np.asarray(e_last))
    if cmax is not None:
        arrays["cmax"] = np.asarray(cmax)
    if meta is not None:
        arrays["meta"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    np.savez_compressed(path, **arrays)


def load_dataset(path: str) -> Dict:
    """Inverse of save_dataset (numpy.load without pickles)."""
    with np.load(path, allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    if "meta" in d:
        d["meta"] = json.loads(bytes(d["meta"]).decode())
    return d
