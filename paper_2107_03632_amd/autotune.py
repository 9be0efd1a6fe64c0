"""Autotuner for the mixed-order weights batch.

Times every candidate of the three forms on a given node set and keeps
the fastest: the one persistent launch (blocks per compute unit, tile size
per order), one persistent launch per order (blocks per compute unit of
each order's launch), and one launch per order of the single-order kernels
with a block per list entry (no parameters).  The tuning only changes speed, never results.  The choice is saved to
batch_tuning.json next to the library, which the binding applies whenever
the library is loaded.

    python -m paper_2107_03632_amd.autotune          # 1M-node {2,4,6} batch
"""

from __future__ import annotations

import itertools
import json
import sys
import time

import numpy as np
import torch

from . import binding as rb
from . import nodes

# one launch: blocks per compute unit (the K = 84 body's 40 KB of LDS
# keeps four resident; more queue behind them) and stencils per tile
CANDIDATES = {
    "blocks_per_cu": [2, 3, 4, 6, 8],
    "gpt2": [1, 2, 4],
    "gpt4": [1, 2, 4],
    "gpt6": [1, 2],
}
# one launch per order: blocks per compute unit for m = 2, 4, 6
ORDER_CANDIDATES = {
    "bpc2": [8, 12, 16],
    "bpc4": [8, 12, 16],
    "bpc6": [3, 4, 6],
}


def _time_ms(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune_batch(x, y, nbr, order, reps: int = 3, candidates=CANDIDATES,
               order_candidates=ORDER_CANDIDATES) -> dict:
    """Time each candidate setting of both forms; apply and return the
    fastest."""
    table = []
    keys = list(candidates)
    for vals in itertools.product(*(candidates[k] for k in keys)):
        c = dict(zip(keys, vals))
        rb.batch_tuning_set(c["blocks_per_cu"], [c["gpt2"], c["gpt4"], c["gpt6"]], 0)
        ms = _time_ms(lambda: rb.rbffd_weights(x, y, nbr, order=order), reps)
        table.append({**c, "per_order": 0, "ms": ms})
    best1 = min(table, key=lambda r: r["ms"])
    okeys = list(order_candidates)
    for vals in itertools.product(*(order_candidates[k] for k in okeys)):
        c = dict(zip(okeys, vals))
        rb.batch_tuning_set(best1["blocks_per_cu"], [best1["gpt2"], best1["gpt4"], best1["gpt6"]],
                            1, [c["bpc2"], c["bpc4"], c["bpc6"]])
        ms = _time_ms(lambda: rb.rbffd_weights(x, y, nbr, order=order), reps)
        table.append({**c, "per_order": 1, "ms": ms})
    rb.batch_tuning_set(best1["blocks_per_cu"], [best1["gpt2"], best1["gpt4"], best1["gpt6"]], 2)
    ms = _time_ms(lambda: rb.rbffd_weights(x, y, nbr, order=order), reps)
    table.append({"per_order": 2, "ms": ms})
    best = min(table, key=lambda r: r["ms"])
    best2 = min((r for r in table if r["per_order"] == 1), key=lambda r: r["ms"])
    choice = {"blocks_per_cu": best1["blocks_per_cu"],
              "groups_per_tile": [best1["gpt2"], best1["gpt4"], best1["gpt6"]],
              "per_order": best["per_order"],
              "order_blocks_per_cu": [best2["bpc2"], best2["bpc4"], best2["bpc6"]]}
    rb.batch_tuning_set(choice["blocks_per_cu"], choice["groups_per_tile"], choice["per_order"],
                        choice["order_blocks_per_cu"])
    return {"choice": choice, "ms": best["ms"], "one_launch_ms": best1["ms"],
            "per_order_ms": best2["ms"], "per_order_block_per_entry_ms": ms, "table": table}


def main(argv=None) -> int:
    dev = torch.device("cuda:0")
    ns = nodes.workload("square_1m_mixed")
    X = torch.as_tensor(ns.x, device=dev)
    Y = torch.as_tensor(ns.y, device=dev)
    O = torch.as_tensor(ns.order, device=dev)
    nbr = rb.rbffd_knn(X, Y, 56)
    t0 = time.time()
    res = tune_batch(X, Y, nbr, O)
    res["workload"] = "1M-node square, per-node order uniform on {2,4,6}, n = 12/30/56"
    res["device"] = torch.cuda.get_device_name(dev)
    res["seconds"] = time.time() - t0
    out = argv[0] if argv else rb.TUNING_PATH
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({"choice": res["choice"], "ms": res["ms"]}))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
