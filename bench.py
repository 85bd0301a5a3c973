#!/usr/bin/env python3
"""Throughput of the recursive multibaryon correlator path on one MI355X.

One step = blocks + recursion + final sum for every (problem, timeslice) lane
of the workload, propagators already resident in HBM.  The metric is
correlator timeslices per second for the mixed-precision path, with the
plain FP64 path timed on the same inputs, the relative error between them,
per-kernel times from HIP events on the launch stream, the roofline of the
dominant kernel and the oracle timed on a bounded sample on the host.

  python bench.py [--config all|c3+c4|c1|c2|c3|c4|c5] [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Workloads: synthetic propagators shaped like the paper's (Sec. 7 nuclei).
CONFIGS = {
    "c1": dict(workload="p+n NR, all components, L=4 T=8, 1 problem, complex128",
               nP=1, nN=1, rel=False, nsrc=1, spins=None, L=4, T=8, nprob=1, c128=True),
    "c2": dict(workload="4He NR (0,1,0,1), L=16 T=32, 8 problems, complex128",
               nP=2, nN=2, rel=False, nsrc=1, spins=(0, 1, 0, 1), L=16, T=32, nprob=8, c128=True),
    "c3": dict(workload="4He relativistic, all 36x36 spin components, L=24 T=48, 16 problems, complex64",
               nP=2, nN=2, rel=True, nsrc=1, spins=None, L=24, T=48, nprob=16, c128=False),
    "c4": dict(workload="8Be NR, two sources, (0,1,2,3,0,1,2,3), L=32 T=64, 16 problems, complex64",
               nP=4, nN=4, rel=False, nsrc=2, spins=(0, 1, 2, 3, 0, 1, 2, 3), L=32, T=64, nprob=16,
               c128=False),
    # beyond the paper's tables: a hypernucleus (third flavour, one Lambda
    # after the nucleons) and five neutrons on three sources
    "h5": dict(workload="Lambda + 4He relativistic, spins (0,1,0,1; 0), L=24 T=48, 16 problems, complex64, "
                        "strange propagator with m = 0.6",
               nP=2, nN=2, nLam=1, rel=True, nsrc=1, spins=(0, 1, 0, 1, 0), L=24, T=48, nprob=16, c128=False),
    "n5": dict(workload="5 neutrons NR, three sources, (0,3,1,4,2), L=16 T=32, 2 problems, complex64",
               nP=0, nN=5, rel=False, nsrc=3, spins=(0, 3, 1, 4, 2), L=16, T=32, nprob=2, c128=False),
}
M_DECAY = 0.5
M_DECAY_S = 0.6   # strange propagators decay faster (heavier quark)
NEXT = ["h5", "n5"]   # reported under next_workloads; tuned only when committed settings exist

# The uneven batch: 64 problems drawn by seed from four nuclei, L in
# {16, 24, 32}, T in {32, 64, 96}, complex64 propagators, 2^k(t) rescale.
MIX_TYPES = [
    dict(name="p+n NR all", nP=1, nN=1, rel=False, nsrc=1, spins=None),
    dict(name="3He NR all", nP=2, nN=1, rel=False, nsrc=1, spins=None),
    dict(name="4He rel all", nP=2, nN=2, rel=True, nsrc=1, spins=None),
    dict(name="8Be NR 2src", nP=4, nN=4, rel=False, nsrc=2, spins=(0, 1, 2, 3, 0, 1, 2, 3)),
]
MIX_SEED, MIX_N, MIX_STREAM0 = 2013, 64, 1000

# library precision modes: tuning-table labels and the storage they stand for
TUNE_LABEL = {0: "fp64", 1: "mixed", 2: "mixed-f32b"}
STORAGE = {0: "f64", 1: "f32 stages, f64 blocks", 2: "f32 stages, f32 block copies for the steps, f64 blocks"}


def mixed_precision(tl, args, cfg):
    """The mixed mode of a workload: float block copies (MB_MIXED_F32B) for a
    list of all spin components (many outputs per lane, whose error stays
    far below 1e-6 with them), else MB_MIXED (one spin component: the
    cancellation in it lifts the coherent rounding of the block copies above
    1e-6); --mixed-storage forces one."""
    from paper_1301_4895_amd import binding as B
    want = ("f32b" if cfg["spins"] is None else "f32") if args.mixed_storage == "auto" else args.mixed_storage
    return B.MB_MIXED if want == "f32" else B.MB_MIXED_F32B


def mix_groups(dev, types=None, n=MIX_N, seed=MIX_SEED):
    """Groups (nucleus, L) of the uneven batch with device propagators; the
    propagators of problem p are dataset stream MIX_STREAM0 + p (one problem
    of its own T).  Returns (groups, term lists by type, problem list)."""
    import numpy as np
    import torch

    from paper_1301_4895_amd import binding as B
    from synth.gpu import fill_props
    from synth.props import mix_problems, momentum_phase
    probs = mix_problems(seed, n, len(MIX_TYPES))
    types = sorted({t for t, _, _ in probs}) if types is None else types
    tls = {}
    for t in types:
        m = MIX_TYPES[t]
        tls[t] = (B.TermList(m["nP"], m["nN"], m["rel"], m["nsrc"], all_components=True) if m["spins"] is None
                  else B.TermList.spin_state(m["nP"], m["nN"], m["rel"], m["nsrc"], m["spins"]))
        tls[t].upload(dev)
    groups = []
    for t in types:
        for L in sorted({L for tt, L, _ in probs if tt == t}):
            members = [(p, T) for p, (tt, LL, T) in enumerate(probs) if tt == t and LL == L]
            lanes = sum(T for _, T in members)
            nsrc = MIX_TYPES[t]["nsrc"]
            V = L ** 3
            props = torch.empty((lanes, V, nsrc, 12, 12), dtype=torch.complex64, device=dev)
            kexp, units, off = [], [], 0
            for p, T in members:
                per = max(1, (1 << 31) // (V * nsrc * 144))
                for b0 in range(0, T, per):
                    b1 = min(T, b0 + per)
                    fill_props(props[off + b0:off + b1], seed=seed, stream_id=MIX_STREAM0 + p, V=V, nsrc=nsrc,
                               T=T, first_bt=b0, m=M_DECAY)
                kexp += [int(math.floor(M_DECAY * t_ / math.log(2.0) + 0.5)) for t_ in range(T)]
                units += [(p, t_, T) for t_ in range(T)]
                off += T
            sink = None
            if nsrc == 2:
                sink = torch.from_numpy(np.stack([np.ones(V, np.complex128), momentum_phase(L, 1)])).to(dev)
            groups.append(dict(name=f"{MIX_TYPES[t]['name']} L={L}", type=t, L=L, tl=tls[t], props=props,
                               sink_w=sink, scale_exp=torch.tensor(kexp, dtype=torch.int32, device=dev),
                               units=units))
    return groups, tls, probs
VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (no packed FP32)
HBM_PEAK_GBS = 8000.0
MFMA_F64_PEAK_TFLOPS = 78.6  # FP64 matrix (dense)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    """Hash of the recursion-step sources: the measured traffic of a step is
    only reported while these are unchanged."""
    h = hashlib.sha256()
    for f in ("contract.hip", "contract_impl.h", "contract_f32.hip", "contract_f32b.hip", "contract_f64.hip",
              "contract_f32_m6.hip", "contract_f64_m6.hip", "kernels.h"):
        h.update(open(os.path.join(ROOT, "paper_1301_4895_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def error_report(mixed, fp64, sigma=None):
    """Mixed against FP64, per lane (leading axis of each array in the lists):
    the relative Frobenius norm over the lane's components, the largest
    relative error of its components of at least 1e-3 of its largest, and,
    with the library's error estimates (sigma per component), how the
    measured deviation compares with them."""
    import numpy as np
    per_lane, comp = [], []
    ratio, dev_over_sig = [], 0.0
    for i, (a, b) in enumerate(zip(mixed, fp64)):
        a2, b2 = a.reshape(a.shape[0], -1), b.reshape(b.shape[0], -1)
        d = np.abs(a2 - b2)
        per_lane.append(np.linalg.norm(d, axis=1) / np.linalg.norm(b2, axis=1))
        ref = np.abs(b2)
        big = ref >= 1e-3 * ref.max(axis=1, keepdims=True)
        comp.append(np.where(big, d / np.where(big, ref, 1.0), 0.0).max(axis=1))
        if sigma is not None:
            sg = sigma[i].reshape(sigma[i].shape[0], -1)
            ratio.append(np.linalg.norm(sg, axis=1) / np.maximum(np.linalg.norm(d, axis=1), 1e-300))
            dev_over_sig = max(dev_over_sig, float((d / np.maximum(sg, 1e-300)).max()))
    per_lane, comp = np.concatenate(per_lane), np.concatenate(comp)
    out = dict(median=float(np.median(per_lane)), p99=float(np.quantile(per_lane, 0.99)), max=float(per_lane.max()),
               componentwise_max=float(comp.max()), componentwise_median=float(np.median(comp)),
               componentwise_threshold="components >= 1e-3 of the lane's largest")
    if sigma is not None:
        ratio = np.concatenate(ratio)
        out["error_estimate"] = dict(
            sigma_over_deviation_per_lane=dict(min=float(ratio.min()), median=float(np.median(ratio)),
                                               max=float(ratio.max())),
            max_component_deviation_in_sigmas=dev_over_sig)
    return out


def run_workload(name, args):
    """Times one workload on both paths; returns its summary."""
    import numpy as np
    import torch

    from paper_1301_4895_amd import binding as B
    from paper_1301_4895_amd.runner import Runner
    from synth.gpu import fill_props
    from synth.props import momentum_phase

    cfg = CONFIGS[name]
    dev = torch.device("cuda:0")
    V, T, nprob, nsrc = cfg["L"] ** 3, cfg["T"], cfg["nprob"], cfg["nsrc"]
    nlam = cfg.get("nLam", 0)
    lanes = nprob * T
    t0 = time.time()
    if cfg["spins"] is None:
        tl = B.TermList(cfg["nP"], cfg["nN"], cfg["rel"], nsrc, all_components=True, n_Lambda=nlam)
    else:
        tl = B.TermList.spin_state(cfg["nP"], cfg["nN"], cfg["rel"], nsrc, cfg["spins"], n_Lambda=nlam)
    tl.upload(dev)
    counts = tl.counts()
    t_list = time.time() - t0
    log(f"[bench] {name}: term list {counts['n_lambda']} ops, built+uploaded in {t_list:.1f}s")

    cdt = torch.complex128 if cfg["c128"] else torch.complex64
    props = torch.empty((lanes, V, nsrc, 12, 12), dtype=cdt, device=dev)
    chunk_gen = max(1, (1 << 31) // (V * nsrc * 144))
    for b0 in range(0, lanes, chunk_gen):
        fill_props(props[b0:b0 + chunk_gen], seed=2013, stream_id=0, V=V, nsrc=nsrc, T=T, first_bt=b0,
                   m=M_DECAY)
    props_s = None
    if nlam:
        props_s = torch.empty_like(props)
        for b0 in range(0, lanes, chunk_gen):
            fill_props(props_s[b0:b0 + chunk_gen], seed=2013, stream_id=1, V=V, nsrc=nsrc, T=T, first_bt=b0,
                       m=M_DECAY_S)
    kexp = torch.tensor([int(math.floor(M_DECAY * (b % T) / math.log(2.0) + 0.5)) for b in range(lanes)],
                        dtype=torch.int32, device=dev)
    sink = None
    if nsrc >= 2:
        # sink function s' of source s': zero momentum, then one and two units along x3
        w = np.stack([np.ones(V, np.complex128)] + [momentum_phase(cfg["L"], p) for p in range(1, nsrc)])
        sink = torch.from_numpy(w).to(dev)
    nbytes = props.numel() * props.element_size() * (2 if nlam else 1)
    log(f"[bench] propagators {nbytes / 1e9:.1f} GB generated")

    chunk = lanes if args.chunk <= 0 else min(args.chunk, lanes)   # default: one launch for all lanes
    assert lanes % chunk == 0
    nchunk = lanes // chunk
    A = cfg["nP"] + cfg["nN"] + nlam
    steps_idx = list(range(A + 1))
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    results = {}
    outs = {}
    tuning = {}
    applied = {}
    mixed = mixed_precision(tl, args, cfg)
    for prec_name, prec in [("mixed", mixed), ("fp64", B.MB_FP64)]:
        if args.only and prec_name != args.only:
            continue
        r = Runner(tl, props[:chunk], props[:chunk], prec, sink, kexp[:chunk],
                   props_s=None if props_s is None else props_s[:chunk])
        tuning[prec_name] = None
        from paper_1301_4895_amd import autotune
        key = f"{name}|{TUNE_LABEL[prec]}|{chunk}"
        if name in NEXT and autotune.committed(key) is None and not args.retune:
            tuning[prec_name] = {"source": "library defaults (not tuned)"}
        elif not args.no_autotune:
            best = None if args.retune else autotune.committed(key)
            source = "committed (paper_1301_4895_amd/tuned.json)"
            if best is not None:
                autotune.apply(tl, best)
                r.ensure_workspace()
                log(f"[bench] {name} {prec_name}: committed launch settings")
            else:
                best = autotune.tune(tl, r, key=key, cache=args.tune_cache, log=log)
                source = "autotuned in this run"
            applied[prec_name] = best
            tuning[prec_name] = {"source": source, "steps": {
                str(k): {"kernel": "lds-staged" if v[0] else "direct", "pass_group": v[1],
                         "lds_bytes": v[2], "lane_tile": v[3], "unroll": v[4],
                         "outputs_per_wave": v[5], "two_phase": v[6], "ms_when_tuned": round(v[7], 3)}
                for k, v in best.items() if k > 0},
                "blocks_kernel": "vector units" if best.get(0, (0,))[0] == 2 else "matrix cores (automatic)"}
        corr_all = torch.empty((lanes,) + tuple(r.corr.shape[1:]), dtype=torch.complex128, device=dev)
        ev = {}

        def one_pass(record):
            for c in range(nchunk):
                sl = slice(c * chunk, (c + 1) * chunk)
                r.set_props(props[sl], props[sl], kexp[sl], None if props_s is None else props_s[sl])
                evs = [torch.cuda.Event(enable_timing=True) for _ in range(A + 3)] if record else None
                if record:
                    evs[0].record(stream)
                B.make_blocks(tl, r.p, r.blocks, r.bws, sh)
                if record:
                    evs[1].record(stream)
                for s in steps_idx:
                    B.contract_step(tl, r.p, r.blocks, s, r.corr, r.exp, r.cws, sh)
                    if record:
                        evs[2 + s].record(stream)
                corr_all[sl].copy_(r.corr)
                if record:
                    ev.setdefault("chunks", []).append(evs)

        for _ in range(args.warmup):
            one_pass(False)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(args.steps):
            one_pass(True)
        stop.record(stream)
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(stop)
        # per-kernel times
        names = ["blocks"] + [f"step{s}" for s in steps_idx]
        ktime = {n: 0.0 for n in names}
        for evs in ev["chunks"]:
            for i, n in enumerate(names):
                ktime[n] += evs[i].elapsed_time(evs[i + 1])
        nlaunch = args.steps * nchunk
        kavg = {n: ktime[n] / nlaunch for n in names}
        ms_per_step = total_ms / args.steps
        results[prec_name] = dict(ms_per_step=ms_per_step, value=lanes / (ms_per_step / 1e3),
                                  kernel_avg_ms=kavg)
        outs[prec_name] = corr_all.cpu().numpy()
        log(f"[bench] {prec_name}: {ms_per_step:.2f} ms/step, {lanes / (ms_per_step / 1e3):.1f} timeslices/s, "
            f"kernels(avg ms/launch of {chunk} lanes): " +
            ", ".join(f"{n}={kavg[n]:.3f}" for n in names))
        del r
        torch.cuda.empty_cache()

    err = None
    err_stats = None
    if "mixed" in outs and "fp64" in outs:
        # one untimed mixed pass with the library's error estimates (err_out),
        # in the timed launch settings; its correlators must be the timed ones
        sig = torch.empty((lanes,) + tuple(outs["mixed"].shape[1:]), dtype=torch.float64)
        same = True
        if "mixed" in applied:
            from paper_1301_4895_amd import autotune
            autotune.apply(tl, applied["mixed"])
        re = Runner(tl, props[:chunk], props[:chunk], mixed, sink, kexp[:chunk], err_estimate=True,
                    props_s=None if props_s is None else props_s[:chunk])
        for c in range(nchunk):
            sl = slice(c * chunk, (c + 1) * chunk)
            re.set_props(props[sl], props[sl], kexp[sl], None if props_s is None else props_s[sl])
            corr, _ = re.run()
            torch.cuda.synchronize()
            same = same and bool(np.array_equal(corr.cpu().numpy(), outs["mixed"][sl]))
            sig[sl] = re.err[..., 0].cpu()
        del re
        torch.cuda.empty_cache()
        err_stats = error_report([outs["mixed"]], [outs["fp64"]], [sig.numpy()])
        err_stats["error_estimate"]["correlators_identical_to_timed_run"] = same
        err = err_stats["max"]
        log(f"[bench] rel err mixed vs fp64 over {lanes} lanes: median {err_stats['median']:.2e} "
            f"p99 {err_stats['p99']:.2e} max {err:.3e}; componentwise max {err_stats['componentwise_max']:.2e}; "
            f"estimate/deviation {err_stats['error_estimate']['sigma_over_deviation_per_lane']}")

    main_name = "mixed" if "mixed" in results else "fp64"
    res = results[main_name]
    # dominant kernel: the recursion step with the largest time
    step_names = [f"step{s}" for s in range(1, A)]
    dom = max(step_names, key=lambda n: res["kernel_avg_ms"][n])
    s = int(dom[4:])
    flops = counts["n_lambda_step"][s] * 8.0 * chunk
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        t = json.load(open(tf))
        key = f"{name}:{main_name}:{dom}"
        # the counters were taken with each workload's own mixed mode (the
        # default --mixed-storage auto) and the current step sources
        if (t.get("kernel_hash") == kernel_hash() and key in t.get("bytes_per_launch", {})
                and (main_name != "mixed" or args.mixed_storage == "auto")):
            traffic = t["bytes_per_launch"][key]
    from paper_1301_4895_amd import autotune
    prec = mixed if main_name == "mixed" else B.MB_FP64
    sp = counts["path"][s]
    nxi = counts["n_xi"]
    rows = nxi ** 3 if sp == 2 else nxi * (nxi - 1) // 2 * nxi
    per_row = (autotune._base(tl, sp) + 1) // 2 * 16 if prec == B.MB_MIXED_F32B else counts["n_psi"] * 16
    roofline = step_roofline(flops, counts["n_req"][s - 1], counts["n_req"][s], 16 if prec == B.MB_FP64 else 8,
                             rows * per_row, chunk, res["kernel_avg_ms"][dom], traffic)
    roofline["kernel"] = f"recursion {dom} ({('proton', 'neutron', 'Lambda')[sp]} added)"
    roofline["blocks"] = blocks_roofline(cfg, counts, chunk, res["kernel_avg_ms"]["blocks"])

    return dict(name=name, cfg=cfg, lanes=lanes, V=V, counts=counts, chunk=chunk, results=results,
                main=main_name, err=err, err_stats=err_stats, roofline=roofline, tuning=tuning, t_list=t_list,
                storage=STORAGE[mixed if main_name == "mixed" else B.MB_FP64])


def run_mix(args):
    """The uneven batch as one graph launch per step, mixed and FP64."""
    import numpy as np
    import torch

    from paper_1301_4895_amd import binding as B
    from paper_1301_4895_amd.batch import BatchRunner, tune_nuclei
    dev = torch.device("cuda:0")
    c5_chunk = args.chunk if args.chunk > 0 else 256   # lanes per batch item
    t0 = time.time()
    groups, tls, probs = mix_groups(dev)
    lanes = sum(g["props"].shape[0] for g in groups)
    log(f"[bench] mix: {len(probs)} problems, {len(groups)} groups, {lanes} lanes, "
        f"{sum(g['props'].numel() * 8 for g in groups) / 1e9:.1f} GB of propagators ({time.time() - t0:.1f}s)")
    results, outs, tuning = {}, {}, {}
    for prec_name, prec in [("mixed", B.MB_MIXED), ("fp64", B.MB_FP64)]:
        if args.only and prec_name != args.only:
            continue
        # every group in the leg's mode; the mixed leg picks per nucleus as
        # the single workloads do
        for g in groups:
            g["precision"] = prec if prec == B.MB_FP64 else mixed_precision(g["tl"], args, MIX_TYPES[g["type"]])
        sources = None
        if not args.no_autotune:
            tuned = tune_nuclei(groups, prec, c5_chunk, cache=args.tune_cache, key="c5", log=log,
                                committed_first=not args.retune)
            sources = sorted({src for _, src in tuned.values()})
        br = BatchRunner(groups, prec, n_branches=4, chunk=c5_chunk)
        times = br.tune_branches(log=log) if not args.no_autotune else None
        tuning[prec_name] = dict(branches=br.n_branches, graph_ms_by_branches=times, launch_settings=sources)
        for _ in range(args.warmup):
            br.launch()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(args.steps):
            br.launch()
        stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / args.steps
        results[prec_name] = dict(ms_per_step=ms, value=lanes / (ms / 1e3), kernel_avg_ms={},
                                  kernels_per_graph=br.kernel_count())
        outs[prec_name] = [c.cpu().numpy() for c in br.corr]
        log(f"[bench] mix {prec_name}: {ms:.2f} ms per graph launch ({br.kernel_count()} kernels, "
            f"{br.n_branches} branches), {lanes / (ms / 1e3):.1f} timeslices/s")
        br.batch.close()
        del br
        torch.cuda.empty_cache()
    err = err_stats = None
    if len(outs) == 2:
        err_stats = error_report(outs["mixed"], outs["fp64"])
        err = err_stats["max"]
        log(f"[bench] mix rel err mixed vs fp64: median {err_stats['median']:.2e} max {err:.3e}, "
            f"componentwise max {err_stats['componentwise_max']:.2e}")
    main_name = "mixed" if "mixed" in results else "fp64"
    cfg = dict(workload=f"uneven batch: {len(probs)} problems drawn by seed {MIX_SEED} from "
                        f"{', '.join(m['name'] for m in MIX_TYPES)}; L in {{16,24,32}}, T in {{32,64,96}}; "
                        f"complex64, one graph launch")
    storage = STORAGE[B.MB_FP64]
    if main_name == "mixed":
        storage = "; ".join(f"{m['name']}: {STORAGE[mixed_precision(tls[t], args, m)]}"
                            for t, m in enumerate(MIX_TYPES) if t in tls)
    return dict(name="c5", cfg=cfg, lanes=lanes, V=None, counts=dict(n_lambda=None), chunk=c5_chunk,
                results=results, main=main_name, err=err, err_stats=err_stats, roofline=None, tuning=tuning,
                t_list=0.0, storage=storage)


def step_roofline(flops, n_in, n_out, elem, block_bytes_per_lane, lanes, ms, traffic=None):
    """The roofline object of a recursion step launch from its algorithmic
    work: `flops` per launch against the vector peak, and the algorithmic
    bytes (the previous stage's n_in components read once, the new stage's
    n_out written once, elem bytes each, and the added species' block
    entries read once, per lane) against HBM; the bound is the roof with the
    larger fraction, whose achieved rate and fraction are reported.  The
    measured HBM traffic (bytes per launch, or None) goes beside them: its
    rate, HBM fraction and ratio to the algorithmic bytes."""
    sec = ms / 1e3
    alg_bytes = ((n_in + n_out) * elem + block_bytes_per_lane) * lanes
    tflops = flops / sec / 1e12
    alu_frac = tflops / VALU_PEAK_TFLOPS
    hbm_frac = alg_bytes / sec / 1e9 / HBM_PEAK_GBS
    out = dict(bound="alu", achieved=round(tflops, 3), peak=VALU_PEAK_TFLOPS, unit="TFLOP/s",
               frac=round(alu_frac, 4), traffic=traffic, flops_per_launch=flops,
               algorithmic_bytes_per_launch=alg_bytes, hbm_frac_algorithmic=round(hbm_frac, 4),
               launch_ms=round(ms, 4))
    if hbm_frac > alu_frac:
        out.update(bound="hbm", achieved=round(alg_bytes / sec / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                   frac=round(hbm_frac, 4), alu_frac=round(alu_frac, 4))
    if traffic is not None:
        # measured HBM traffic (FETCH_SIZE x calibration + WRITE_SIZE; FETCH_SIZE
        # counts every L2 request to the memory fabric, MALL hits included)
        out.update(measured_traffic_gbps=round(traffic / sec / 1e9, 1),
                   hbm_frac_measured_traffic=round(traffic / sec / 1e9 / HBM_PEAK_GBS, 4),
                   traffic_over_algorithmic=round(traffic / alg_bytes, 2))
    return out


def blocks_roofline(cfg, counts, chunk, ms):
    """The blocks call (site sums on FP64 MFMA, finish, lane exponents) against
    its binding roof.  Algorithmic flops per site, symmetric diquark (u = d):
    the contraction 3 colours x (rows psi x xi1) x (xi2 <= xi3 pairs) and
    the diquark 3 colours x pairs x (2 eps terms x the nonzero C gamma_5
    entries: 4 relativistic, 2 nonrelativistic) complex FMAs, 8 flops each
    (104 832 per site for 4He relativistic, 97 344 for 8Be with two sources,
    8 064 for nonrelativistic one-source nuclei).  Bytes: the propagator
    entries the blocks need, (3 D)^2 per source and site (the rows and
    columns of the active spins), each read once.  The bound is the roof
    with the longer ideal time; both fractions are reported.  With a Lambda
    its block adds the same contraction over all n_xi^2 ordered (u, d)
    pairs and their diquarks, and the strange propagator's entries.  Three
    sources run the site sums on the vector units (bound "alu", the same
    FP64 peak)."""
    V = cfg["L"] ** 3
    npsi, nxi = counts["n_psi"], counts["n_xi"]
    D = 4 if cfg["rel"] else 2
    npair = nxi * (nxi + 1) // 2
    ncg5 = 4 if cfg["rel"] else 2
    per_site = 8.0 * 3 * npair * (npsi * nxi + 2 * ncg5)
    nflav = 1
    if cfg.get("nLam"):
        per_site += 8.0 * 3 * nxi * nxi * (npsi * nxi + 2 * ncg5)
        nflav = 2
    flops = chunk * V * per_site
    nbytes = chunk * V * cfg["nsrc"] * (3 * D) ** 2 * (16 if cfg["c128"] else 8) * nflav
    t_mfma, t_hbm = flops / (MFMA_F64_PEAK_TFLOPS * 1e12), nbytes / (HBM_PEAK_GBS * 1e9)
    tflops = flops / (ms / 1e3) / 1e12
    gbs = nbytes / (ms / 1e3) / 1e9
    out = dict(flops_per_site=per_site, bytes_per_site=nbytes / (chunk * V), launch_ms=round(ms, 4),
               mfma_frac=round(tflops / MFMA_F64_PEAK_TFLOPS, 4), hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
               ideal_ms_mfma=round(t_mfma * 1e3, 4), ideal_ms_hbm=round(t_hbm * 1e3, 4))
    if t_mfma >= t_hbm:
        out.update(bound="alu" if cfg["nsrc"] == 3 else "mfma", achieved=round(tflops, 3),
                   peak=MFMA_F64_PEAK_TFLOPS, unit="TFLOP/s", frac=out["mfma_frac"])
    else:
        out.update(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=out["hbm_frac"])
    return out


def summary(w):
    res = w["results"][w["main"]]
    fp = w["results"].get("fp64")
    return {
        "value": round(res["value"], 2),
        "ms_per_step": round(res["ms_per_step"], 3),
        "config": {"workload": w["cfg"]["workload"], "lanes": w["lanes"], "V": w["V"],
                   "n_lambda": w["counts"]["n_lambda"], "lanes_per_launch": w["chunk"], "precision": w["main"],
                   "storage": w["storage"]},
        "fp64": ({"value": round(fp["value"], 2), "ms_per_step": round(fp["ms_per_step"], 3),
                  "speedup_mixed_over_fp64": round(res["value"] / fp["value"], 3)}
                 if fp is not None and w["main"] == "mixed" else None),
        "max_rel_err_mixed_vs_fp64": w["err"],
        "rel_err_mixed_vs_fp64_per_lane": w["err_stats"],
        "kernel_avg_ms": {k: round(v, 4) for k, v in res["kernel_avg_ms"].items()},
        "roofline": w["roofline"],
        "term_list_build_s": round(w["t_list"], 2),
        "autotune": w["tuning"],
        "kernels_per_graph": res.get("kernels_per_graph"),
    }


def calibrate_copy():
    """A plain device copy of known size (1 GiB, three times), the yardstick
    for the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied 3 x {n} bytes", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="all", choices=sorted(CONFIGS) + ["all", "c3+c4", "c5"],
                    help="workload; all (default) times 4He relativistic (the reported value), 8Be NR, the "
                         "uneven batch and 4He NR; c3+c4 only the first two")
    ap.add_argument("--chunk", type=int, default=0,
                    help="lanes per launch (default: every lane of the workload in one launch; batch items of at most 256 lanes for c5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None)
    ap.add_argument("--mixed-storage", choices=["auto", "f32b", "f32"], default="auto",
                    help="mixed path: float stages and float block copies for the steps (f32b), float "
                         "stages and double blocks (f32), or per term list (auto: f32b for lists of all spin "
                         "components, f32 for one spin state)")
    ap.add_argument("--no-autotune", action="store_true", help="library default launch settings")
    ap.add_argument("--retune", action="store_true",
                    help="autotune every step in this run instead of using the committed settings")
    ap.add_argument("--tune-cache", default=None, help="JSON file of tuned launch settings (read/write)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(lanes are independent, so whole launches of lanes would go to each GPU)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    names = {"all": ["c3", "c4", "c5", "c2"] + NEXT, "c3+c4": ["c3", "c4"]}.get(args.config, [args.config])
    ws = []
    for n in names:
        ws.append(run_mix(args) if n == "c5" else run_workload(n, args))
        import torch
        torch.cuda.empty_cache()
    first = summary(ws[0])
    cpu = None
    if not args.no_cpu_baseline and names[0] != "c5":
        cpu = cpu_baseline(ws[0]["cfg"], names[0])

    line = {
        "metric": "correlator timeslices/s (4He rel., 8Be NR): mixed vs FP64 GPU, rel err<=1e-6",
        "value": first["value"],
        "unit": "timeslices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": first["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # both paths multiply and add in double; the mixed path stores the
        # recursion stages (and, by default, the blocks the steps read) in float
        "dtype": "f64",
        "data": "synthetic",
        "config": first["config"],
    }
    for k in ("fp64", "max_rel_err_mixed_vs_fp64", "rel_err_mixed_vs_fp64_per_lane", "kernel_avg_ms",
              "roofline"):
        line[k] = first[k]
    line["cpu_baseline"] = cpu
    for k in ("term_list_build_s", "autotune"):
        line[k] = first[k]
    nxt = [w for n, w in zip(names[1:], ws[1:]) if n in NEXT]
    for key, w in zip(("second_workload", "third_workload", "fourth_workload"),
                      [w for n, w in zip(names[1:], ws[1:]) if n not in NEXT]):
        line[key] = summary(w)
    if nxt:
        line["next_workloads"] = {w["name"]: summary(w) for w in nxt}
    print(json.dumps(line), flush=True)


def cpu_baseline(cfg, name):
    """The oracle on a bounded sample of one timeslice: its brute-force blocks
    over a slice of the sites and its correlator for a few (sink set, source
    set) pairs, scaled to one full timeslice of the workload."""
    import numpy as np

    from oracle import oracle as O
    from synth import props as SP
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = min(16, avail)   # the host share of one GPU
    O.set_threads(threads)
    host = dict(cpu_count=os.cpu_count(), available_to_process=avail, threads_used=threads)
    V = cfg["L"] ** 3
    D = 4 if cfg["rel"] else 2
    if cfg["nP"] + cfg["nN"] > 4:
        return {"value": None, "unit": "timeslices/s", "cores": threads, "host": host, "kind": "oracle",
                "sample": "infeasible: the oracle's permutation sum has n_u! n_d! = (12!)^2 terms per "
                          "component for 8Be"}
    nsite = V
    S = SP.props(2013, 0, cfg["nprob"], cfg["T"], V, cfg["nsrc"], M_DECAY, np.complex128, probs=[0],
                 ts=[1])[0, 0]
    t = time.time()
    fP, fN = O.blocks(cfg["rel"], cfg["nsrc"], S[:nsite], S[:nsite], None, 2.0)
    t_blocks_sample = time.time() - t
    req = (O.all_components_request(cfg["nP"], cfg["nN"], D, cfg["nsrc"]) if cfg["spins"] is None
           else O.spin_state_request(cfg["nP"], cfg["nN"], cfg["spins"]))
    types = [0] * cfg["nP"] + [1] * cfg["nN"]
    dsets = O.delta_sets(cfg["nP"], cfg["nN"], req)
    nL = {a: len(O.L_for_alpha(cfg["rel"], cfg["nsrc"], cfg["nP"], cfg["nN"], a)[0]) for a in req["alphas"]}
    # 12 (sink set, source set) pairs spread over the requested ones
    npairs = min(12, len(dsets) * len(req["alphas"]))
    sample_pairs = [(dsets[(7 * i) % len(dsets)], req["alphas"][(11 * i) % len(req["alphas"])])
                    for i in range(npairs)]
    t = time.time()
    nl_sample = 0
    for d, a in sample_pairs:
        um, dm, cf = O.L_for_alpha(cfg["rel"], cfg["nsrc"], cfg["nP"], cfg["nN"], a)
        O.corr_from_L(types, O._bits(d[0]) + O._bits(d[1]), fP, fN, um, dm, cf)
        nl_sample += len(um)
    t_pairs = time.time() - t
    # the permutation sums cost about the same per L entry for every pair
    nl_total = len(dsets) * sum(nL.values())
    per_ts = t_blocks_sample * V / nsite + t_pairs * nl_total / nl_sample
    # the same oracle on one thread, on a smaller sample: blocks on 1/16 of
    # the sites and 2 of the pairs, scaled the same way
    O.set_threads(1)
    ns1 = max(1, V // 16)
    t = time.time()
    fP1, fN1 = O.blocks(cfg["rel"], cfg["nsrc"], S[:ns1], S[:ns1], None, 2.0)
    t_b1 = time.time() - t
    t = time.time()
    nl1 = 0
    for d, a in sample_pairs[:2]:
        um, dm, cf = O.L_for_alpha(cfg["rel"], cfg["nsrc"], cfg["nP"], cfg["nN"], a)
        O.corr_from_L(types, O._bits(d[0]) + O._bits(d[1]), fP1, fN1, um, dm, cf)
        nl1 += len(um)
    t_p1 = time.time() - t
    O.set_threads(threads)
    per_ts1 = t_b1 * V / ns1 + t_p1 * nl_total / nl1
    return {"value": 1.0 / per_ts, "unit": "timeslices/s", "cores": threads, "host": host, "kind": "oracle",
            "sample": (f"one timeslice: oracle blocks on {nsite} of {V} sites ({t_blocks_sample:.1f}s), "
                       f"scaled by {V / nsite:.2f}; oracle correlator for {len(sample_pairs)} of "
                       f"{len(dsets)}x{len(req['alphas'])} component pairs ({nl_sample} L entries, "
                       f"{t_pairs:.1f}s), scaled by the {nl_total} L entries of all pairs"),
            "seconds_measured": round(t_blocks_sample + t_pairs, 2),
            "single_thread": {"value": 1.0 / per_ts1, "unit": "timeslices/s", "cores": 1,
                              "sample": (f"oracle blocks on {ns1} of {V} sites ({t_b1:.1f}s), correlator for 2 "
                                         f"component pairs ({nl1} L entries, {t_p1:.1f}s), scaled as above"),
                              "seconds_measured": round(t_b1 + t_p1, 2)}}


if __name__ == "__main__":
    main()
