"""Batched runs (mb_batch_*): uneven mixes of nuclei, volumes and lane counts
recorded into one HIP graph with concurrent branches.

  * small mix: every lane of the FP64 graph against the oracle (1e-12), the
    mixed graph against FP64 (1e-6), graph against the single calls
    (identical bits: same kernels, same launch settings), several replays
    with other work in between;
  * the full uneven batch (64 problems drawn by seed, L in {16,24,32}, T in
    {32,64,96}): mixed against FP64 on every lane (1e-6), graph against the
    single calls, and both paths against the oracle on sampled p+n, 3He and
    4He relativistic lanes.
Correlator comparisons are element by element (tests.gpu_helpers.assert_close).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from bench import M_DECAY, MIX_SEED, MIX_STREAM0, MIX_TYPES, mix_groups
from oracle import oracle as O
from paper_1301_4895_amd import binding as B
from paper_1301_4895_amd.batch import BatchRunner
from synth import props as SP
from tests.gpu_helpers import assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _oracle_lane(tl, m, S, w, k):
    dsets = tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2)
    asets = tl.export(B.MB_EXPORT_ALPHA).reshape(-1, 2)
    req = dict(sinkP=int(np.bitwise_or.reduce(dsets[:, 0])), sinkN=int(np.bitwise_or.reduce(dsets[:, 1])),
               alphas=[tuple(map(int, a)) for a in asets])
    Cd = O.correlators(m["rel"], m["nsrc"], m["nP"], m["nN"], req, S, S, w, 2.0 ** int(k))
    out = np.zeros((len(dsets), len(asets)), np.complex128)
    for i, d in enumerate(map(tuple, dsets.tolist())):
        for j, a in enumerate(map(tuple, asets.tolist())):
            out[i, j] = Cd[(d, a)]
    return out


def _oracle_pairs(tl, m, S, k, pairs):
    """Oracle correlators of a few (sink set, source set) pairs, for nuclei
    whose full set of pairs is too slow for the permutation sum."""
    dsets = tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2)
    asets = tl.export(B.MB_EXPORT_ALPHA).reshape(-1, 2)
    fP, fN = O.blocks(m["rel"], m["nsrc"], S, S, None, 2.0 ** int(k))
    types = [0] * m["nP"] + [1] * m["nN"]
    out = {}
    for i, j in pairs:
        d, a = tuple(map(int, dsets[i])), tuple(map(int, asets[j]))
        um, dm, cf = O.L_for_alpha(m["rel"], m["nsrc"], m["nP"], m["nN"], a)
        out[(i, j)] = O.corr_from_L(types, O._bits(d[0]) + O._bits(d[1]), fP, fN, um, dm, cf)
    return out


def _mixed_sigma(groups, chunk=256):
    """The library's estimated standard deviation of the rounding error of
    every mixed correlator of every group (single calls with err_out, in the
    group's mixed mode "mixed", default MB_MIXED; the correlators are those
    of the graph)."""
    from paper_1301_4895_amd.runner import Runner
    out = []
    for g in groups:
        lanes = g["props"].shape[0]
        parts = []
        for b0 in range(0, lanes, chunk):
            b1 = min(lanes, b0 + chunk)
            r = Runner(g["tl"], g["props"][b0:b1], g["props"][b0:b1], g.get("mixed", B.MB_MIXED), g.get("sink_w"),
                       None if g.get("scale_exp") is None else g["scale_exp"][b0:b1], err_estimate=True)
            r.run()
            torch.cuda.synchronize()
            parts.append(r.err[..., 0].cpu().numpy())
            del r
        out.append(np.concatenate(parts))
        torch.cuda.empty_cache()
    return out


def _small_groups():
    """p+n NR (V=27, 70 lanes: two chunks of 64 and 6), 3He NR (V=8, 5
    lanes), 4He relativistic (V=8, 3 lanes), and p+n again at V=64 (17
    lanes) sharing its term list."""
    spec = [(0, 3, 70), (1, 2, 5), (2, 2, 3), (0, 4, 17)]
    tls, groups = {}, []
    for gi, (t, L, lanes) in enumerate(spec):
        m = MIX_TYPES[t]
        if t not in tls:
            tls[t] = B.TermList(m["nP"], m["nN"], m["rel"], m["nsrc"], all_components=True)
            tls[t].upload(DEV)
        V = L ** 3
        S = SP.props(77, 50 + gi, 1, lanes, V, 1, M_DECAY, np.complex128)[0]
        k = np.array([int(math.floor(M_DECAY * t_ / math.log(2.0) + 0.5)) for t_ in range(lanes)], np.int32)
        groups.append(dict(name=f"g{gi}", type=t, L=L, tl=tls[t], props=torch.from_numpy(S).to(DEV),
                           sink_w=None, scale_exp=torch.from_numpy(k).to(DEV), host=S, k=k))
    return groups, tls


def test_small_mix_graph_vs_oracle_and_single_calls():
    groups, tls = _small_groups()
    res = {}
    for prec in (B.MB_FP64, B.MB_MIXED):
        br = BatchRunner(groups, prec, n_branches=3, chunk=64)
        assert br.kernel_count() > 0
        br.launch()
        torch.cuda.synchronize()
        graph = [c.cpu().numpy() for c in br.corr]
        gexp = [e.cpu().numpy() for e in br.exp]
        # replays with other device work in between give the same bits
        for rep in range(3):
            for c in br.corr:
                c.zero_()
            x = torch.randn(1 << 20, device=DEV)
            (x * 2).sum().item()
            br.launch()
            torch.cuda.synchronize()
            for g, c in enumerate(br.corr):
                assert np.array_equal(c.cpu().numpy(), graph[g]), (prec, rep, g)
        # the single calls, one after the other, give the same bits
        for c in br.corr:
            c.zero_()
        br.run_eager()
        torch.cuda.synchronize()
        for g, c in enumerate(br.corr):
            assert np.array_equal(c.cpu().numpy(), graph[g]), (prec, "eager", g)
        res[prec] = graph
        for g, grp in enumerate(groups):
            assert np.array_equal(gexp[g], 3 * (MIX_TYPES[grp["type"]]["nP"] + MIX_TYPES[grp["type"]]["nN"])
                                  * grp["k"])
        br.batch.close()
    O.set_threads(8)
    for g, grp in enumerate(groups):
        m = MIX_TYPES[grp["type"]]
        lanes = grp["host"].shape[0]
        check = range(lanes) if lanes <= 8 else sorted({0, 1, 63, 64, lanes - 1} & set(range(lanes)))
        for b in check:
            if m["rel"] and m["nP"] + m["nN"] == 4:
                got = res[B.MB_FP64][g][b]
                for (i, j), ref in _oracle_pairs(grp["tl"], m, grp["host"][b], grp["k"][b],
                                                 [(0, 0), (14, 21), (35, 7)]).items():
                    assert abs(got[i, j] - ref) <= 1e-12 * abs(ref), (g, b, i, j)
                continue
            ref = _oracle_lane(grp["tl"], m, grp["host"][b], None, grp["k"][b])
            assert_close(res[B.MB_FP64][g][b], ref, 1e-12, (g, b))
    sig = _mixed_sigma(groups)
    for g, grp in enumerate(groups):
        assert_close(res[B.MB_MIXED][g], res[B.MB_FP64][g], 1e-6, (g, "mixed vs fp64"), sigma=sig[g])


def test_batch_rejects_shared_buffers_across_branches():
    groups, tls = _small_groups()
    br = BatchRunner(groups[:2], B.MB_FP64, n_branches=2, chunk=64)
    items = br.items
    # put two items on different branches but give them the same workspace
    bad = [dict(it) for it in items[:2]]
    bad[0]["branch"], bad[1]["branch"] = 0, 1
    bad[1]["contract_ws"] = bad[0]["contract_ws"]
    bad[1]["blocks"] = bad[0]["blocks"]
    bad[1]["blocks_ws"] = bad[0]["blocks_ws"]
    with pytest.raises(B.MBError) as e:
        B.Batch(bad, 2)
    assert e.value.code == B.MB_EINVAL
    with pytest.raises(B.MBError):
        B.Batch(bad, 1)   # branch index out of range
    br.batch.close()


def test_full_uneven_batch():
    """In the launch settings and precision modes the benchmark times (the
    committed table, keyed like bench.py's C5 run; the mixed leg with float
    block copies for the all-component nuclei)."""
    import argparse

    from bench import mixed_precision
    from paper_1301_4895_amd.batch import tune_nuclei
    groups, tls, probs = mix_groups(torch.device(DEV))
    assert sum(g["props"].shape[0] for g in groups) == sum(T for _, _, T in probs)
    auto = argparse.Namespace(mixed_storage="auto")
    for g in groups:
        g["mixed"] = mixed_precision(g["tl"], auto, MIX_TYPES[g["type"]])
    assert {g["mixed"] for g in groups} == {B.MB_MIXED, B.MB_MIXED_F32B}
    res = {}
    for prec in (B.MB_MIXED, B.MB_FP64):
        for g in groups:
            g["precision"] = g["mixed"] if prec == B.MB_MIXED else prec
        tuned = tune_nuclei(groups, prec, 256, key="c5")
        print(prec, {src for _, src in tuned.values()}, flush=True)
        br = BatchRunner(groups, prec, n_branches=4, chunk=256)
        br.launch()
        torch.cuda.synchronize()
        res[prec] = [c.cpu().numpy() for c in br.corr]
        if prec == B.MB_MIXED:
            for c in br.corr:
                c.zero_()
            br.run_eager()
            torch.cuda.synchronize()
            for g, c in enumerate(br.corr):
                assert np.array_equal(c.cpu().numpy(), res[prec][g]), groups[g]["name"]
        br.batch.close()
        del br
        torch.cuda.empty_cache()
    sig = _mixed_sigma(groups)
    for g, grp in enumerate(groups):
        assert np.all(np.isfinite(res[B.MB_MIXED][g])), grp["name"]
        assert_close(res[B.MB_MIXED][g], res[B.MB_FP64][g], 1e-6, (grp["name"], "mixed vs fp64"), sigma=sig[g])
    # both paths against the oracle on sampled lanes: every component of p+n
    # and 3He lanes, a few (sink set, source set) pairs of 4He relativistic
    # lanes (its full permutation sum per lane is too slow at these volumes)
    import os
    O.set_threads(min(16, os.cpu_count() or 1))
    for g, grp in enumerate(groups):
        if grp["type"] not in (0, 1, 2):
            continue
        m = MIX_TYPES[grp["type"]]
        lanes = (0, len(grp["units"]) - 1) if grp["type"] != 2 else (len(grp["units"]) // 2,)
        for lane in lanes:
            p, t, T = grp["units"][lane]
            S = SP.props(MIX_SEED, MIX_STREAM0 + p, 1, T, grp["L"] ** 3, 1, M_DECAY, np.complex64,
                         probs=[0], ts=[t])[0, 0].astype(np.complex128)
            k = int(math.floor(M_DECAY * t / math.log(2.0) + 0.5))
            if grp["type"] == 2:
                for (i, j), ref in _oracle_pairs(grp["tl"], m, S, k, [(0, 0), (14, 21), (35, 7)]).items():
                    assert abs(ref) > 0
                    assert abs(res[B.MB_FP64][g][lane, i, j] - ref) <= 1e-12 * abs(ref), (grp["name"], lane, i, j)
                    assert abs(res[B.MB_MIXED][g][lane, i, j] - ref) <= max(1e-6 * abs(ref), 6 * sig[g][lane, i, j]), \
                        (grp["name"], lane, i, j)
                continue
            ref = _oracle_lane(grp["tl"], m, S, None, k)
            assert_close(res[B.MB_FP64][g][lane], ref, 1e-12, (grp["name"], lane))
            assert_close(res[B.MB_MIXED][g][lane], ref, 1e-6, (grp["name"], lane), sigma=sig[g][lane])


def test_batch_with_a_lambda_and_three_sources():
    """One graph holding a hypernucleus (Lambda + n, all components), a
    three-source nucleus (three neutrons, one per source) and p+n: the FP64
    graph equals the single calls bit for bit and the oracle within 1e-12 on
    every lane; the mixed graph equals its single calls and FP64 within
    1e-6 or 6 estimated sigma."""
    from paper_1301_4895_amd.runner import Runner
    tl_l = B.TermList(0, 1, False, 1, all_components=True, n_Lambda=1)
    tl_3 = B.TermList.spin_state(0, 3, False, 3, (0, 2, 4))
    tl_pn = B.TermList(1, 1, False, 1, all_components=True)
    specs = [("lambda", tl_l, 27, 1, 21), ("three", tl_3, 8, 3, 9), ("pn", tl_pn, 27, 1, 12)]
    groups = []
    rng = np.random.default_rng(3)
    for gi, (name, tl, V, nsrc, lanes) in enumerate(specs):
        tl.upload(DEV)
        S = SP.props(91, 60 + gi, 1, lanes, V, nsrc, M_DECAY, np.complex128)[0]
        Ss = SP.props(91, 70 + gi, 1, lanes, V, nsrc, 0.6, np.complex128)[0] if name == "lambda" else None
        w = (rng.normal(size=(nsrc, V)) + 1j * rng.normal(size=(nsrc, V))) if nsrc > 1 else None
        k = np.array([int(math.floor(M_DECAY * t_ / math.log(2.0) + 0.5)) for t_ in range(lanes)], np.int32)
        groups.append(dict(name=name, tl=tl, props=torch.from_numpy(S).to(DEV),
                           props_s=None if Ss is None else torch.from_numpy(Ss).to(DEV),
                           sink_w=None if w is None else torch.from_numpy(w).to(DEV),
                           scale_exp=torch.from_numpy(k).to(DEV), host=S, host_s=Ss, w=w, k=k, nsrc=nsrc))
    res = {}
    for prec in (B.MB_FP64, B.MB_MIXED):
        br = BatchRunner(groups, prec, n_branches=2, chunk=16)
        br.launch()
        torch.cuda.synchronize()
        graph = [c.cpu().numpy() for c in br.corr]
        for c in br.corr:
            c.zero_()
        br.run_eager()
        torch.cuda.synchronize()
        for g, c in enumerate(br.corr):
            assert np.array_equal(c.cpu().numpy(), graph[g]), (prec, groups[g]["name"])
        res[prec] = graph
        br.batch.close()
        del br
        torch.cuda.empty_cache()
    for gi, g in enumerate(groups):
        sig = []
        for b0 in range(0, g["props"].shape[0], 16):
            b1 = min(g["props"].shape[0], b0 + 16)
            r = Runner(g["tl"], g["props"][b0:b1], g["props"][b0:b1], B.MB_MIXED, g["sink_w"],
                       g["scale_exp"][b0:b1], err_estimate=True,
                       props_s=None if g["props_s"] is None else g["props_s"][b0:b1])
            r.run()
            torch.cuda.synchronize()
            sig.append(r.err[..., 0].cpu().numpy())
            del r
        assert_close(res[B.MB_MIXED][gi], res[B.MB_FP64][gi], 1e-6, g["name"], sigma=np.concatenate(sig))
    O.set_threads(8)
    for gi, g in enumerate(groups):
        tl = g["tl"]
        d2 = tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2)
        a2 = tl.export(B.MB_EXPORT_ALPHA).reshape(-1, 2)
        for lane in range(g["props"].shape[0]):
            sc = 2.0 ** int(g["k"][lane])
            if g["name"] == "lambda":
                dl = np.concatenate([d2, tl.export(B.MB_EXPORT_DELTA_L)[:, None]], 1)
                al = np.concatenate([a2, tl.export(B.MB_EXPORT_ALPHA_L)[:, None]], 1)
                req = O.hyperon_request_all(0, 1, 2, 1)
                Cd = O.hyperon_correlators(False, 1, 0, 1, req, g["host"][lane], g["host"][lane],
                                           g["host_s"][lane], None, sc)
            else:
                dl, al = d2, a2
                nP = 1 if g["name"] == "pn" else 0
                nN = 1 if g["name"] == "pn" else 3
                req = dict(sinkP=int(np.bitwise_or.reduce(d2[:, 0])), sinkN=int(np.bitwise_or.reduce(d2[:, 1])),
                           alphas=[tuple(map(int, a)) for a in a2])
                Cd = O.correlators(False, g["nsrc"], nP, nN, req, g["host"][lane], g["host"][lane], g["w"], sc)
            ref = np.array([[Cd[(tuple(map(int, d)), tuple(map(int, a)))] for a in al] for d in dl])
            assert_close(res[B.MB_FP64][gi][lane], ref, 1e-12, (g["name"], lane))
