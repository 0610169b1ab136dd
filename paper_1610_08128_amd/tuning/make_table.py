"""Write the tuning table shipped for MI355X (tuning/mi355x.txt) on a GPU.

Times the autotuner's candidate launch settings on the benchmark's
workloads and keeps the fastest per size class:

* the 3D 7-point 128^3 grid (one large graph, team kernel settings);
* the 2D 5-point 64x64 grid (one small graph: the one-work-group engine
  against small teams);
* the 32 x 500,000 strip (the asynchronous search's round length);
* the batch of 512 graphs (batched-call settings).

Every candidate is checked to give the same permutation.  Usage::

    python -m paper_1610_08128_amd.tuning.make_table [out.txt]
"""

from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "mi355x.txt")


def main(out: str = TABLE) -> str:
    from paper_1610_08128_amd import inputs, tune

    t0 = time.time()
    table = tune.autotune_single([inputs.config(1)], reps=3)
    print(f"3D grid done ({time.time() - t0:.1f} s)", flush=True)
    table = tune.autotune_single([inputs.config(0)], candidates=tune.SMALL_CANDIDATES, reps=5,
                                 table=table)
    print(f"2D grid done ({time.time() - t0:.1f} s)", flush=True)
    table = tune.autotune_single([inputs.config(2)], candidates=tune.LONG_CANDIDATES, reps=2,
                                 table=table)
    print(f"strip done ({time.time() - t0:.1f} s)", flush=True)
    table = tune.autotune_batched([inputs.batch_graphs(512, seed=4)], reps=7, table=table)
    print(f"batch done ({time.time() - t0:.1f} s)", flush=True)
    table.save(out, header="MI355X (gfx950), one GPU; workloads: 128^3 3D grid, 64x64 2D grid, "
                           "32x500,000 strip, 512-graph batch\nregenerate: python -m "
                           "paper_1610_08128_amd.tuning.make_table")
    return out


if __name__ == "__main__":
    print(main(*sys.argv[1:]))
