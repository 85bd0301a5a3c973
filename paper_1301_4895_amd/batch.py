"""Batched runs of an uneven mix of nuclei, volumes and time extents.

Lanes of one nucleus and one volume form a group; every group is cut into
launch chunks of at most ``chunk`` lanes (the items of the batch).  The
library's scheduler spreads the items over concurrent graph branches
(longest first), every branch gets one set of buffers sized for the largest
of its items, and the whole batch is recorded once into one HIP graph
(mb_batch_create) and launched with one call.  The autotuner picks the
launch settings of every nucleus and the number of branches.
"""
from __future__ import annotations

import time

import torch

from . import binding as B


class BatchRunner:
    """groups: list of dicts with keys
         tl        uploaded TermList (shared by groups of one nucleus)
         props     device tensor [lanes][V][n_src][12][12] (u = d)
         props_s   the strange propagator, same layout (term lists with a
                   Lambda only; optional otherwise)
         sink_w    complex128 [n_src][V] device tensor or None
         scale_exp int32 [lanes] device tensor or None
         precision the group's precision mode (optional; default the
                   runner's ``precision``)
    After ``launch`` + synchronisation, ``corr[g]`` holds the correlators of
    group g ([lanes][n_delta][n_alpha] complex128) and ``exp[g]`` their
    scale exponents."""

    def __init__(self, groups, precision, n_branches=4, chunk=256):
        self.groups = groups
        self.precision = precision
        self.chunk = chunk
        dev = groups[0]["props"].device
        self.corr, self.exp, self.items = [], [], []
        for g in groups:
            lanes = g["props"].shape[0]
            c = g["tl"].counts()
            self.corr.append(torch.empty((lanes, c["n_delta"], c["n_alpha"]), dtype=torch.complex128,
                                         device=dev))
            self.exp.append(torch.empty(lanes, dtype=torch.int32, device=dev))
            sink = None if g.get("sink_w") is None else torch.view_as_real(g["sink_w"])
            for b0 in range(0, lanes, chunk):
                b1 = min(lanes, b0 + chunk)
                p = B.problem(b1 - b0, g["props"].shape[1], g["props"][b0:b1], g["props"][b0:b1],
                              g.get("precision", precision),
                              sink, None if g.get("scale_exp") is None else g["scale_exp"][b0:b1],
                              None if g.get("props_s") is None else g["props_s"][b0:b1])
                self.items.append(dict(tl=g["tl"], prob=p, corr=self.corr[-1][b0:b1],
                                       exp=self.exp[-1][b0:b1]))
        self.batch = None
        self.record(n_branches)

    def record(self, n_branches):
        """(Re)assigns the items to n_branches branches, allocates one buffer
        set per branch and records the graph."""
        if self.batch is not None:
            self.batch.close()
            self.batch = None
            self.bufs = None
            torch.cuda.empty_cache()
        self.n_branches = n_branches
        br, self.cost = B.batch_plan([it["tl"] for it in self.items], [it["prob"] for it in self.items],
                                     n_branches)
        need = [[0, 0, 0] for _ in range(n_branches)]
        for it, k in zip(self.items, br):
            it["branch"] = k
            for j, v in enumerate(B.workspace_query(it["tl"], it["prob"])):
                need[k][j] = max(need[k][j], v)
        dev = self.items[0]["corr"].device
        self.bufs = [[torch.empty(max(v, 1), dtype=torch.uint8, device=dev) for v in n] for n in need]
        for it in self.items:
            it["blocks"], it["blocks_ws"], it["contract_ws"] = self.bufs[it["branch"]]
        self.batch = B.Batch(self.items, n_branches)
        return self

    def launch(self, stream=None):
        self.batch.launch(stream)

    def kernel_count(self):
        return self.batch.kernel_count()

    def workspace_bytes(self):
        return sum(t.numel() for b in self.bufs for t in b)

    def run_eager(self, stream=None):
        """The same items one after the other through the single calls (the
        reference order for checking the graph)."""
        for it in self.items:
            B.make_blocks(it["tl"], it["prob"], it["blocks"], it["blocks_ws"], stream)
            B.contract_correlator(it["tl"], it["prob"], it["blocks"], it["corr"], it["exp"], it["contract_ws"],
                                  stream)

    def tune_branches(self, candidates=(1, 2, 4), reps=3, log=None):
        """Times the recorded graph for every branch count and keeps the
        fastest.  Returns {n_branches: ms}."""
        times = {}
        for nb in candidates:
            self.record(nb)
            self.launch()
            torch.cuda.synchronize()
            ms = []
            for _ in range(reps):
                t0 = time.perf_counter()
                self.launch()
                torch.cuda.synchronize()
                ms.append((time.perf_counter() - t0) * 1e3)
            times[nb] = min(ms)
            if log:
                log(f"[batch] {nb} branches: {times[nb]:.2f} ms")
        best = min(times, key=times.get)
        if best != self.n_branches:
            self.record(best)
        return times


def tune_nuclei(groups, precision, chunk=256, cache=None, key=None, log=None, committed_first=True):
    """Launch settings of every distinct term list: the committed ones for
    this key (paper_1301_4895_amd/tuned.json) when present and
    committed_first, else the autotuner on the largest of its groups (the
    settings do not depend on the volume), in the group's precision mode
    (its "precision" entry, else ``precision``).  Returns {id(tl):
    (settings, source)}."""
    from . import autotune
    from .runner import Runner
    best = {}
    for g in sorted(groups, key=lambda g: -g["props"].shape[0]):
        tl = g["tl"]
        if id(tl) in best:
            continue
        n = min(chunk, g["props"].shape[0])
        prec = g.get("precision", precision)
        k = None if key is None else f"{key}|{g['name']}|{prec}|{n}"
        fixed = autotune.committed(k) if (committed_first and k) else None
        if fixed is not None:
            autotune.apply(tl, fixed)
            best[id(tl)] = (fixed, "committed")
            continue
        r = Runner(tl, g["props"][:n], g["props"][:n], prec, g.get("sink_w"),
                   None if g.get("scale_exp") is None else g["scale_exp"][:n])
        best[id(tl)] = (autotune.tune(tl, r, key=k, cache=cache, log=log), "autotuned")
        del r
        torch.cuda.empty_cache()
    return best
