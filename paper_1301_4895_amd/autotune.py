"""Autotuner for the recursion-step launches.

For every step of a term list it times the candidate launch settings exposed
by ``mb_term_list_tune`` -- the kernel (direct gathers, or block rows staged
in LDS), passthrough spin parts per thread, lanes per wavefront, outputs
per wavefront, splits in flight per wavefront and LDS
reserved per workgroup (which caps resident workgroups, hence operands in
flight per L2) -- on the caller's own buffers, keeps the fastest, and records
the choice in a JSON cache keyed by workload, precision, lanes and device.
Results of the method do not depend on the settings.

The choices the benchmark times are kept in ``tuned.json`` beside this file
(read only: ``committed`` and ``apply``), so that the timed launch settings
are the ones the full-size parity tests run; ``tune`` writes only to a cache
file the caller names.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import binding as B

LDS_CANDIDATES = (0, 16384)
COMMITTED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
TILES = (64, 16)


CACHE_VERSION = "v5"


def _candidates(npass, nsingle):
    """(kernel, pass group, LDS bytes, lane tile, splits in flight, outputs per
    wavefront, two-phase)."""
    pgs = [pg for pg in (1, 2, 3, 6) if npass % pg == 0]
    direct = [(0, pg, 0, t, u, 1, 0) for pg in pgs for t in TILES for u in (1, 2)]
    capped = [(0, pg, lds, t, 0, 1, 0) for pg in pgs for t in TILES for lds in LDS_CANDIDATES if lds]
    grouped = [(0, pg, 0, 64, 0, gr, 0) for pg in pgs if pg <= 3 for gr in (2, 4)]
    staged = [(1, pg, 0, 16, 0, 1, 0) for pg in (1, 2, 3) if npass % pg == 0]
    two = [(0, pg, 0, t, u, 1, 1) for pg in pgs for t in TILES for u in (1, 2)] if nsingle > 1 else []
    return direct + capped + grouped + staged + two


def _apply(tl, s, kernel, pg, lds, tile, unroll, group, two_phase=0):
    tl.tune(s, B.MB_TUNE_KERNEL, kernel)
    tl.tune(s, B.MB_TUNE_PASS_GROUP, pg)
    tl.tune(s, B.MB_TUNE_LDS_BYTES, lds)
    tl.tune(s, B.MB_TUNE_LANE_TILE, tile)
    tl.tune(s, B.MB_TUNE_UNROLL, unroll)
    tl.tune(s, B.MB_TUNE_GROUP, group)
    tl.tune(s, B.MB_TUNE_TWO_PHASE, two_phase)


def _device_arch():
    if torch.cuda.is_available():
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return "gfx950"


def full_key(key):
    return f"{key}|{_device_arch()}|{CACHE_VERSION}"


def committed(key):
    """The committed launch settings of a workload key ("c3|mixed|768"), or
    None: {step: (kernel, pass_group, lds_bytes, lane_tile, unroll, group,
    two_phase, ms)}."""
    if not os.path.exists(COMMITTED):
        return None
    table = json.load(open(COMMITTED))
    v = table.get(full_key(key))
    return None if v is None else {int(s): tuple(x) for s, x in v.items()}


def apply(tl, best):
    """Sets every step's launch settings from a {step: settings} table
    (step 0: the blocks kernel, (MB_TUNE_BLOCKS value, ms))."""
    tl.tune(0, B.MB_TUNE_BLOCKS, int(best[0][0]) if 0 in best else 0)
    for s, v in best.items():
        if s > 0:
            _apply(tl, s, *v[:7])


def _time_blocks(runner, reps):
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        runner.run_blocks()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return min(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))


def _npass_nsingle(tl, c, s):
    """Passthrough spin parts of step s (spin parts of the other species)
    and the added baryon's single-flavour quark count (d of a proton, u of
    a neutron; a Lambda step has no pair split: 1)."""
    added = c["path"][s]
    kP = sum(1 for t in c["path"][:s + 1] if t == 0)
    kN = sum(1 for t in c["path"][:s + 1] if t == 1)
    kL = s + 1 - kP - kN
    k_added = (kP, kN, kL)[added]
    npass = c["n_spin"][s] // math.comb(_base(tl, added), k_added)
    nsingle = (kP + 2 * kN + kL) if added == 0 else (2 * kP + kN + kL) if added == 1 else 1
    return npass, nsingle


def _time_step(tl, runner, step, reps, stream):
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        B.contract_step(tl, runner.p, runner.blocks, step, runner.corr, runner.exp, runner.cws,
                        stream.cuda_stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return min(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))


def tune(tl: B.TermList, runner, key: str | None = None, cache: str | None = None, reps: int = 2,
         log=None):
    """Tunes every step on ``runner``'s buffers.
    Returns {step: (kernel, pass_group, lds_bytes, lane_tile, unroll, group, two_phase, ms)}."""
    c = tl.counts()
    fkey = full_key(key) if key else None
    if cache and fkey and os.path.exists(cache):
        table = json.load(open(cache))
        if fkey not in table and log:
            log(f"[autotune] {fkey} not in {cache}: tuning")
        if fkey in table:
            best = {int(s): tuple(v) for s, v in table[fkey].items()}
            apply(tl, best)
            return best
    stream = torch.cuda.current_stream()
    # two-phase candidates only where their partials fit in the free device
    # memory (with a margin); the workspace for the largest of them is
    # allocated once (a reallocation would drop the stages the timed steps read)
    lanes = (runner.batch + 63) // 64 * 64
    elem = 16 if runner.p.precision == B.MB_FP64 else 8
    free = torch.cuda.mem_get_info()[0] - (8 << 30)
    two_ok = {}
    for s in range(1, c["n_stages"]):
        nsingle = _npass_nsingle(tl, c, s)[1]
        two_ok[s] = nsingle > 1 and nsingle * c["n_req"][s] * lanes * elem <= free
    for s in range(1, c["n_stages"]):
        tl.tune(s, B.MB_TUNE_TWO_PHASE, int(two_ok[s]))
    runner.ensure_workspace()
    for s in range(1, c["n_stages"]):
        tl.tune(s, B.MB_TUNE_TWO_PHASE, 0)
    best = {}
    # the blocks: matrix cores (where the shape has that kernel) or the
    # register-tiled vector-unit kernel
    bres = []
    for kern in ((0, 2) if c["n_xi"] <= 12 else (2,)):
        tl.tune(0, B.MB_TUNE_BLOCKS, kern)
        runner.run_blocks()
        bres.append((_time_blocks(runner, reps), kern))
    bms, bk = min(bres)
    tl.tune(0, B.MB_TUNE_BLOCKS, bk)
    best[0] = (bk, bms)
    if log:
        log("[autotune] blocks: " + ", ".join(f"{'vector' if k == 2 else 'matrix'}={m:.3f}ms" for m, k in bres))
    # bring every stage to a valid state once
    runner.run_blocks()
    for s in range(c["n_stages"] + 1):
        B.contract_step(tl, runner.p, runner.blocks, s, runner.corr, runner.exp, runner.cws,
                        stream.cuda_stream)
    torch.cuda.synchronize()
    for s in range(1, c["n_stages"]):
        # the step reads stage s-1, written by the previous step: rerun it first
        B.contract_step(tl, runner.p, runner.blocks, s - 1, runner.corr, runner.exp, runner.cws,
                        stream.cuda_stream)
        npass, nsingle = _npass_nsingle(tl, c, s)
        results = []
        for cand in _candidates(npass, nsingle if two_ok[s] else 1):
            _apply(tl, s, *cand)
            runner.ensure_workspace()
            try:
                results.append((_time_step(tl, runner, s, reps, stream),) + cand)
            except B.MBError as e:
                # no kernel for this setting and step (refused before any launch)
                if e.code != B.MB_EUNSUPPORTED:
                    raise
        ms, *cand = min(results)
        _apply(tl, s, *cand)
        runner.ensure_workspace()
        best[s] = tuple(cand) + (ms,)
        if log:
            log(f"[autotune] step {s}: " + ", ".join(
                f"{'lds' if k else 'dir'}/pg{g}/lds{l}/t{t}/u{u}/g{gr}{'/2ph' if tp else ''}={m:.2f}ms"
                for m, k, g, l, t, u, gr, tp in sorted(results)[:4]))
    if cache and fkey:
        table = json.load(open(cache)) if os.path.exists(cache) else {}
        table[fkey] = {str(s): list(v) for s, v in best.items()}
        json.dump(table, open(cache, "w"), indent=1)
    return best


def _base(tl, species):
    """Size of the sink base set of a species (0 proton, 1 neutron, 2 Lambda)."""
    d = (tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2)[:, species] if species < 2
         else tl.export(B.MB_EXPORT_DELTA_L))
    m = 0
    for v in d:
        m |= int(v)
    return bin(m).count("1")
