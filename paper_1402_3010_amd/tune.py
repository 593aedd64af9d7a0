"""Tune the self-join on the named synthetic workloads and store the choices.

    python -m paper_1402_3010_amd.tune c3 c4 [--out paper_1402_3010_amd/tuning/gfx950.json]

For each workload the index is built as the benchmark builds it (the
screened join for c4), and apss_autotune times every tile variant and range
width of the join kernel at the workload's first threshold, then the number
of ranges per work item; the choice is merged into the JSON file, which the
benchmark reads back.
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_OUT = os.path.join(HERE, "tuning", "gfx950.json")
SCREEN_DIMS = {"c4": 4096}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+")
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--budget-ms", type=float, default=0.0)
    args = ap.parse_args()
    import numpy as np
    import torch

    import paper_1402_3010_amd as apss
    from synth.corpus import CONFIGS, make_corpus, spec_for

    apss.load()
    for name in args.configs:
        V = make_corpus(spec_for(name))
        t = np.float32(CONFIGS[name]["t"][0])
        dev = (V.n, V.m, torch.from_numpy(V.row_ptr).cuda(), torch.from_numpy(V.col).cuda(),
               torch.from_numpy(V.val).cuda())
        for sd in sorted({0, SCREEN_DIMS.get(name, 0)}):
            ix = apss.Index.build(dev, t, screen_dims=sd)
            t0 = time.perf_counter()
            r = ix.autotune(t, budget_ms=args.budget_ms, cache=args.out)
            print("%s t=%.2f screen_dims=%d: variant %d, range %d rows, %d ranges per item, %.1f ms (%d tried, %.1f s)"
                  % (name, t, sd, r["variant"], r["range_rows"], r["range_group"], r["ms"], r["tried"],
                     time.perf_counter() - t0), flush=True)
            ix.close()
        del dev, V


if __name__ == "__main__":
    main()
