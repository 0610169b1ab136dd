"""Autotuner for the ordering's launch parameters.

The ordering's results do not depend on its launch parameters; only the time
does. Those parameters are:

- the team shape: work-groups per team and threads per work-group;
- the narrow-level cutoff below which one work-group walks the levels alone;
- the component-size cutoff below which a component gets a single
  work-group;
- the threads of those single-work-group teams;
- how many large-component teams run at once;
- the labelling sub-team, the asynchronous search's round length and the
  rebalance interval of the level-synchronous passes;
- the engine (the persistent team kernel or the one-work-group LDS engine).

The tuner times candidate settings on caller-supplied representative graphs
(or batches) and keeps the fastest per size class in a table. It checks that
every candidate returned the same permutation.  The table is a text file the
library itself reads (rcm_options.tuning_file or RCM_TUNING_FILE; format in
include/rcm.h, rcm_tuning_options): one line per size class with its
options, and the measured times as comments.

Usage::

    table = autotune_single([g1, g2])            # inputs.Graph objects
    table.save("rcm_tuning.txt")
    perm, stats = rcm.order(rowptr, colidx, tuning_file="rcm_tuning.txt")
"""

from __future__ import annotations

import json
import math
import time
from dataclasses import dataclass, field
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

from . import rcm

# Large single graphs: team shape, labelling sub-team, round length of the
# asynchronous search, rebalance interval of the level-synchronous passes,
# and the width below which one work-group walks a level alone (0 = the
# library's 256).
SINGLE_CANDIDATES: List[Dict[str, int]] = [
    dict(mode=1, team_size=w, block_threads=256, label_team=lt, search_round=sr,
         rebalance_levels=rb, narrow_cutoff=nc)
    for w in (128, 256)
    for lt in (64, 96, 128)
    for sr in (12, 16, 24)
    for rb in (4, 8)
    for nc in (0, 128, 160)
]

# Long narrow graphs (the strip): the round length of the asynchronous
# search, which sets how many round barriers its narrow frontier meets.
LONG_CANDIDATES: List[Dict[str, int]] = [
    dict(mode=1, search_round=sr) for sr in (16, 32, 64, 128)]

# Small single graphs: the one-work-group engine against teams of the
# persistent kernel.
SMALL_CANDIDATES: List[Dict[str, int]] = (
    [dict(mode=2)] +
    [dict(mode=1, team_size=w, block_threads=256, narrow_cutoff=nc, label_team=w)
     for w in (16, 64) for nc in (64, 256)])

# The first candidate is the library's automatic batch layout (no options:
# a batch of many large components, none of them very large, gets teams of
# 4 over every resident work-group); setting team_size or max_teams turns
# that rule off.
BATCH_CANDIDATES: List[Dict[str, int]] = [dict()] + [
    dict(small_cutoff=sc, small_threads=st, team_size=w, max_teams=mt)
    for sc in (1 << 15, 1 << 16, 1 << 17)
    for st in (256, 512)
    for (w, mt) in ((4, 64), (8, 32), (16, 16))
]


def size_class(n: int, nnz: int, graphs: int = 1) -> str:
    """Key of a tuning entry: call kind, floor(log2) of the vertex count, and
    the mean row length rounded half to even (the library computes the same
    key)."""
    kind = "batch" if graphs > 1 else "single"
    lg = max(n, 1).bit_length() - 1
    deg = int(round(nnz / max(n, 1)))
    return f"{kind}:n2^{lg}:d{deg}"


@dataclass
class TuningTable:
    entries: Dict[str, Dict[str, int]] = field(default_factory=dict)
    timings: Dict[str, Dict[str, float]] = field(default_factory=dict)

    def options_for(self, n: int, nnz: int, graphs: int = 1) -> Dict[str, int]:
        """Options of the exact size class, else of the nearest class of the
        same kind and row length, else of the nearest of the same kind,
        else {} (the library's defaults).  As in the library, the engine
        (mode) comes only from the exact class, and mode 2 (the
        one-work-group engine where the graph fits) is what auto does
        anyway, so it is not passed on."""
        key = size_class(n, nnz, graphs)
        if key in self.entries:
            return {k: v for k, v in self.entries[key].items() if not (k == "mode" and v == 2)}
        kind, lg, deg = key.split(":")
        lg_v, deg_v = int(lg[3:]), int(deg[1:])
        best, best_d = None, None
        for k in self.entries:
            k_kind, k_lg, k_deg = k.split(":")
            if k_kind != kind:
                continue
            d = abs(int(k_lg[3:]) - lg_v) + 4 * abs(int(k_deg[1:]) - deg_v)
            if best_d is None or d < best_d:
                best, best_d = k, d
        if best is None:
            return {}
        return {k: v for k, v in self.entries[best].items() if k != "mode"}

    def save(self, path: str, header: str = "") -> None:
        """The library's text format; the measured times (ms per candidate)
        follow each entry as comments."""
        with open(path, "w") as f:
            f.write("# Reverse Cuthill-McKee launch options per size class, written by "
                    "paper_1610_08128_amd/tune.py\n")
            for line in header.splitlines():
                f.write(f"# {line}\n")
            for key in sorted(self.entries):
                opts = " ".join(f"{k}={int(v)}" for k, v in sorted(self.entries[key].items()))
                f.write(f"{key} {opts}\n")
                for cand, ms in sorted(self.timings.get(key, {}).items(), key=lambda kv: kv[1]):
                    f.write(f"#   {ms:10.4f} ms  {cand}\n")

    @classmethod
    def load(cls, path: str) -> "TuningTable":
        entries: Dict[str, Dict[str, int]] = {}
        with open(path) as f:
            for line in f:
                line = line.split("#", 1)[0].split()
                if not line:
                    continue
                entries[line[0]] = {k: int(v) for k, v in (t.split("=", 1) for t in line[1:])}
        return cls(entries=entries)


def _time_calls(call, reps: int) -> float:
    """Median wall time of `reps` calls after one warm-up call (the median,
    not the best: a batched call's time can be bimodal)."""
    import torch

    call()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        call()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return float(np.median(times))


def autotune_single(graphs: Iterable, candidates: Optional[Sequence[Dict[str, int]]] = None,
                    reps: int = 3, table: Optional[TuningTable] = None) -> TuningTable:
    """Time every candidate on every graph (one call per graph, device
    resident, caller-sized workspace); the fastest candidate of each size
    class is kept.  Raises if two candidates disagree on a permutation."""
    import torch

    cands = list(candidates or SINGLE_CANDIDATES)
    table = table or TuningTable()
    per_class: Dict[str, Dict[int, float]] = {}
    for g in graphs:
        rp = torch.from_numpy(np.ascontiguousarray(g.rowptr)).cuda()
        ci = torch.from_numpy(np.ascontiguousarray(g.colidx)).cuda()
        ws = torch.empty(max(rcm.workspace_bytes(g.n, g.nnz), 1), dtype=torch.uint8,
                         device=rp.device)
        ref = None
        key = size_class(g.n, g.nnz)
        for i, opts in enumerate(cands):
            out = {}

            def call(opts=opts, out=out):
                out["perm"], _ = rcm.order(rp, ci, workspace=ws, **opts)

            t = _time_calls(call, reps)
            perm = out["perm"].cpu().numpy()
            if ref is None:
                ref = perm
            elif not np.array_equal(ref, perm):
                raise RuntimeError(f"candidate {opts} changed the permutation of {g.name}")
            per_class.setdefault(key, {}).setdefault(i, 0.0)
            per_class[key][i] += t
    for key, times in per_class.items():
        best = min(times, key=times.get)
        table.entries[key] = dict(cands[best])
        table.timings[key] = {json.dumps(cands[i], sort_keys=True): round(t * 1e3, 4)
                              for i, t in times.items()}
    return table


def autotune_batched(batches: Iterable, candidates: Optional[Sequence[Dict[str, int]]] = None,
                     reps: int = 5, table: Optional[TuningTable] = None) -> TuningTable:
    """Like autotune_single for batched calls; each batch is a list of
    graphs ordered in one rcm_order_batched call."""
    import torch

    from . import inputs

    cands = list(candidates or BATCH_CANDIDATES)
    table = table or TuningTable()
    per_class: Dict[str, Dict[int, float]] = {}
    for graphs in batches:
        vo, no, rp_h, ci_h = inputs.concat_batch(graphs)
        rp = torch.from_numpy(rp_h).cuda()
        ci = torch.from_numpy(ci_h).cuda()
        G, N, NNZ = len(graphs), int(vo[-1]), int(no[-1])
        ws = torch.empty(max(rcm.batched_workspace_bytes(G, N, NNZ), 1), dtype=torch.uint8,
                         device=rp.device)
        ref = None
        key = size_class(N, NNZ, G)
        for i, opts in enumerate(cands):
            out = {}

            def call(opts=opts, out=out):
                out["perm"], _ = rcm.order_batched(vo, no, rp, ci, workspace=ws, **opts)

            t = _time_calls(call, reps)
            perm = out["perm"].cpu().numpy()
            if ref is None:
                ref = perm
            elif not np.array_equal(ref, perm):
                raise RuntimeError(f"candidate {opts} changed a batched permutation")
            per_class.setdefault(key, {}).setdefault(i, 0.0)
            per_class[key][i] += t
    for key, times in per_class.items():
        best = min(times, key=times.get)
        table.entries[key] = dict(cands[best])
        table.timings[key] = {json.dumps(cands[i], sort_keys=True): round(t * 1e3, 4)
                              for i, t in times.items()}
    return table
