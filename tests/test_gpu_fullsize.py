"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (every lane of the workload in one launch: 768 lanes for 4He, 1024 for
8Be; device-generated propagators, 2^k(t) rescale).

The oracle checks sampled lanes one by one:
  * 4He relativistic, all components, V = 24^3: blocks of three lanes (every
    entry) and their correlators for a few (sink set, source set) pairs;
  * 8Be nonrelativistic with two sources, V = 32^3: blocks of one lane, and
    the full correlator through the two-source factorisation on disjoint
    regions (a property that holds at any size; the 8Be permutation sum
    itself is beyond the oracle).
FP64 path: 1e-12 relative; mixed paths (float stages with double blocks,
MB_MIXED, and for the all-component 4He, where the benchmark times it, also
float block copies, MB_MIXED_F32B): 1e-6 relative, element by element.

Every run uses the launch settings the benchmark times: the committed table
paper_1301_4895_amd/tuned.json (or, where it has no entry for the
workload, the autotuner run on the test's own buffers), so that the kernel
instantiations that are timed are the ones checked against the oracle here.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from bench import CONFIGS, M_DECAY, TUNE_LABEL
from oracle import oracle as O
from paper_1301_4895_amd import autotune
from paper_1301_4895_amd import binding as B
from paper_1301_4895_amd.runner import Runner
from synth import props as SP
from tests.gpu_helpers import assert_close, check_lane_exponent, lib_blocks, oracle_blocks_lib_layout

pytestmark = pytest.mark.gpu

SEED = 2013

# The site sums of the blocks have 3V terms (41 472 at L = 24, 98 304 at
# L = 32); the double rounding of either side (library or oracle) is about
# 2^-53 sqrt(3V) times the largest entry, a few 1e-15 of it, so element by
# element the relative bound 1e-12 applies from 1e-2 of the largest entry.
BLOCKS_SIGNIFICANT = 1e-2


def all_lanes(cfg):
    return cfg["nprob"] * cfg["T"]


def kexp(lanes, T):
    return np.array([int(math.floor(M_DECAY * (b % T) / math.log(2.0) + 0.5)) for b in range(lanes)], np.int32)


def device_props(cfg, lanes):
    from synth.gpu import fill_props
    V, T, nsrc = cfg["L"] ** 3, cfg["T"], cfg["nsrc"]
    p = torch.empty((lanes, V, nsrc, 12, 12), dtype=torch.complex64, device="cuda")
    fill_props(p, seed=SEED, stream_id=0, V=V, nsrc=nsrc, T=T, first_bt=0, m=M_DECAY)
    return p


def host_lane(cfg, lane):
    T = cfg["T"]
    return SP.props(SEED, 0, cfg["nprob"], T, cfg["L"] ** 3, cfg["nsrc"], M_DECAY, np.complex64,
                    probs=[lane // T], ts=[lane % T])[0, 0].astype(np.complex128)


def lane_blocks(r, tl, lane):
    """Stored blocks [species][psi][block quark index] of one lane and its
    exponent."""
    blk, e = lib_blocks(r, tl)
    out, ee = blk[..., lane].cpu().numpy(), int(e[lane])
    check_lane_exponent(out, ee)
    return out, ee


def bench_runner(name, tl, props, prec, sink, k):
    """A Runner with the launch settings bench.py times for this workload
    (mixed: with the error estimates, which read the stages and leave the
    correlators unchanged)."""
    lanes = props.shape[0]
    r = Runner(tl, props, props, prec, sink, k, err_estimate=prec != B.MB_FP64)
    key = f"{name}|{TUNE_LABEL[prec]}|{lanes}"
    best = autotune.committed(key)
    if best is None:
        best = autotune.tune(tl, r, key=None)
    else:
        autotune.apply(tl, best)
    r.ensure_workspace()
    return r, best


@pytest.fixture(scope="module")
def oracle_threads():
    import os
    O.set_threads(min(16, os.cpu_count() or 1))
    yield


def test_4he_relativistic_full_size(oracle_threads):
    cfg = CONFIGS["c3"]
    V = cfg["L"] ** 3
    tl = B.TermList(2, 2, True, 1, all_components=True)
    lanes = all_lanes(cfg)
    props = device_props(cfg, lanes)
    k = torch.from_numpy(kexp(lanes, cfg["T"])).cuda()
    out, sig = {}, {}
    check_lanes = (3, 197, 700)
    mixed = (B.MB_MIXED, B.MB_MIXED_F32B)
    for prec in (B.MB_FP64,) + mixed:
        r, best = bench_runner("c3", tl, props, prec, None, k)
        print(f"c3 {TUNE_LABEL[prec]} launch settings {best}", flush=True)
        corr, _ = r.run()
        torch.cuda.synchronize()
        blocks = {lane: lane_blocks(r, tl, lane) for lane in check_lanes} if prec == B.MB_FP64 else None
        if prec != B.MB_FP64:
            sig[prec] = r.err[..., 0].cpu().numpy()
        out[prec] = (corr.cpu().numpy(), blocks)
        del r, corr
    # the device buffers go before any check (a failing check keeps this frame)
    del props, k
    torch.cuda.empty_cache()
    # mixed against FP64, every lane, element by element
    for prec in mixed:
        assert_close(out[prec][0], out[B.MB_FP64][0], 1e-6, f"c3 {TUNE_LABEL[prec]} vs fp64", sigma=sig[prec])
    dsets = tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2)
    asets = tl.export(B.MB_EXPORT_ALPHA).reshape(-1, 2)
    pairs = [(i, j) for i in (0, 14, 35) for j in (0, 21)] + [(7, 33), (28, 5)]
    for lane in check_lanes:
        S = host_lane(cfg, lane)
        kk = int(kexp(lanes, cfg["T"])[lane])
        fP, fN = O.blocks(True, 1, S, S, None, 2.0 ** kk)
        got_blocks, e = out[B.MB_FP64][1][lane]
        ref_blocks = oracle_blocks_lib_layout(fP, fN) * 2.0 ** -e
        for sp in range(2):
            assert_close(got_blocks[sp], ref_blocks[sp], 1e-12, ("blocks", lane, sp),
                         significant=BLOCKS_SIGNIFICANT)
        for i, j in pairs:
            d, a = tuple(map(int, dsets[i])), tuple(map(int, asets[j]))
            um, dm, cf = O.L_for_alpha(True, 1, 2, 2, a)
            ref = O.corr_from_L([0, 0, 1, 1], O._bits(d[0]) + O._bits(d[1]), fP, fN, um, dm, cf)
            assert abs(ref) > 0
            # the timed instantiations of both paths against the oracle
            assert abs(out[B.MB_FP64][0][lane, i, j] - ref) <= 1e-12 * abs(ref), (lane, i, j)
            for prec in mixed:
                assert abs(out[prec][0][lane, i, j] - ref) <= max(1e-6 * abs(ref), 6 * sig[prec][lane, i, j]), \
                    (prec, lane, i, j)


def test_8be_two_sources_full_size(oracle_threads):
    cfg = CONFIGS["c4"]
    L = cfg["L"]
    V = L ** 3
    tl = B.TermList.spin_state(4, 4, False, 2, (0, 1, 2, 3, 0, 1, 2, 3))
    lanes = all_lanes(cfg)
    props = device_props(cfg, lanes)
    k = torch.from_numpy(kexp(lanes, cfg["T"])).cuda()
    w = np.stack([np.ones(V, np.complex128), SP.momentum_phase(L, 1)])
    # blocks of one lane of the benchmark inputs, every entry
    r, _ = bench_runner("c4", tl, props, B.MB_FP64, torch.from_numpy(w).cuda(), k)
    r.run_blocks()
    torch.cuda.synchronize()
    lane = 877
    got_blocks, e = lane_blocks(r, tl, lane)
    del r
    S = host_lane(cfg, lane)
    fP, fN = O.blocks(False, 2, S, S, w, 2.0 ** int(kexp(lanes, cfg["T"])[lane]))
    ref_blocks = oracle_blocks_lib_layout(fP, fN) * 2.0 ** -e
    for sp in range(2):
        assert_close(got_blocks[sp], ref_blocks[sp], 1e-12, ("blocks", lane, sp), significant=BLOCKS_SIGNIFICANT)
    # correlators through the factorisation: source 0 and sink function 0 live
    # on x3 < L/2, source 1 and sink function 1 on x3 >= L/2
    x3 = np.arange(V) // (L * L)
    low = torch.from_numpy(x3 < L // 2).cuda()
    props[:, ~low, 0] = 0    # source 0 vanishes on the upper half
    props[:, low, 1] = 0     # source 1 vanishes on the lower half
    wr = w.copy()
    wr[0, x3 >= L // 2] = 0
    wr[1, x3 < L // 2] = 0
    res = {}
    mixed = (B.MB_MIXED,)
    for prec in (B.MB_FP64,) + mixed:
        rr, best = bench_runner("c4", tl, props, prec, torch.from_numpy(wr).cuda(), k)
        print(f"c4 {TUNE_LABEL[prec]} launch settings {best}", flush=True)
        corr, _ = rr.run()
        torch.cuda.synchronize()
        res[prec] = corr.cpu().numpy()[:, 0, 0]
        del rr, corr
    # the device buffers go before any check (a failing check keeps this frame)
    del props, k, low
    torch.cuda.empty_cache()
    req = O.spin_state_request(2, 2, (0, 1, 0, 1))
    for lane in (0, 130, 611, 1023):
        S = host_lane(cfg, lane)
        S[x3 >= L // 2, 0] = 0   # same regions as on the device
        S[x3 < L // 2, 1] = 0
        sc = 2.0 ** int(kexp(lanes, cfg["T"])[lane])
        c0 = O.correlators(False, 1, 2, 2, req, S[:, :1], S[:, :1], wr[:1], sc)[((3, 3), (3, 3))]
        c1 = O.correlators(False, 1, 2, 2, req, S[:, 1:], S[:, 1:], wr[1:], sc)[((3, 3), (3, 3))]
        ref = c0 * c1
        assert abs(ref) > 0
        assert abs(res[B.MB_FP64][lane] - ref) <= 1e-12 * abs(ref), lane
        for prec in mixed:
            assert abs(res[prec][lane] - ref) <= 1e-6 * abs(ref), (prec, lane)


def test_5n_three_sources_full_size(oracle_threads):
    """Five neutrons on three sources at the benchmark's size and launch
    settings (64 lanes, V = 16^3): the blocks of one lane against the oracle,
    then the correlator through the three-region factorisation (source s
    and sink function s on the planes of region s): nn(source 0) x
    nn(source 1) x n(source 2), each from the oracle, on sampled lanes."""
    cfg = CONFIGS["n5"]
    L = cfg["L"]
    V = L ** 3
    tl = B.TermList.spin_state(0, 5, False, 3, cfg["spins"])
    lanes = all_lanes(cfg)
    props = device_props(cfg, lanes)
    k = torch.from_numpy(kexp(lanes, cfg["T"])).cuda()
    w = np.stack([np.ones(V, np.complex128), SP.momentum_phase(L, 1), SP.momentum_phase(L, 2)])
    r, _ = bench_runner("n5", tl, props, B.MB_FP64, torch.from_numpy(w).cuda(), k)
    r.run_blocks()
    torch.cuda.synchronize()
    lane = 37
    got_blocks, e = lane_blocks(r, tl, lane)
    del r
    S = host_lane(cfg, lane)
    fP, fN = O.blocks(False, 3, S, S, w, 2.0 ** int(kexp(lanes, cfg["T"])[lane]))
    ref_blocks = oracle_blocks_lib_layout(fP, fN) * 2.0 ** -e
    for sp in range(2):
        assert_close(got_blocks[sp], ref_blocks[sp], 1e-12, ("blocks", lane, sp), significant=BLOCKS_SIGNIFICANT)
    region = np.minimum(np.arange(V) // (L * L) // 6, 2)
    reg = torch.from_numpy(region).cuda()
    wr = w.copy()
    for s in range(3):
        props[:, reg != s, s] = 0
        wr[s, region != s] = 0
    res, sig = {}, None
    for prec in (B.MB_FP64, B.MB_MIXED):
        rr, best = bench_runner("n5", tl, props, prec, torch.from_numpy(wr).cuda(), k)
        print(f"n5 {'mixed' if prec else 'fp64'} launch settings {best}", flush=True)
        corr, _ = rr.run()
        torch.cuda.synchronize()
        res[prec] = corr.cpu().numpy()[:, 0, 0]
        if prec == B.MB_MIXED:
            sig = rr.err[:, 0, 0, 0].cpu().numpy()
        del rr, corr
    del props, k, reg
    torch.cuda.empty_cache()
    nn, n1 = O.spin_state_request(0, 2, (0, 1)), O.spin_state_request(0, 1, (0,))
    for lane in (0, 40, 63):
        S = host_lane(cfg, lane)
        for s in range(3):
            S[region != s, s] = 0
        sc = 2.0 ** int(kexp(lanes, cfg["T"])[lane])
        c0 = O.correlators(False, 1, 0, 2, nn, S[:, :1], S[:, :1], wr[:1], sc)[((0, 3), (0, 3))]
        c1 = O.correlators(False, 1, 0, 2, nn, S[:, 1:2], S[:, 1:2], wr[1:2], sc)[((0, 3), (0, 3))]
        c2 = O.correlators(False, 1, 0, 1, n1, S[:, 2:], S[:, 2:], wr[2:], sc)[((0, 1), (0, 1))]
        ref = c0 * c1 * c2
        assert abs(ref) > 0
        assert abs(res[B.MB_FP64][lane] - ref) <= 1e-12 * abs(ref), lane
        assert abs(res[B.MB_MIXED][lane] - ref) <= max(1e-6 * abs(ref), 6 * sig[lane]), lane


def test_lambda_4he_full_size():
    """Lambda + 4He (relativistic, spins (0,1,0,1; 0)) at the benchmark's
    size and launch settings (768 lanes, V = 24^3), with u != d: exchanging
    the u and d propagators maps the proton operator to minus the
    neutron's and the Lambda to minus itself at sink and source, so for this
    spin state (the same indices for protons and neutrons) the correlator
    is unchanged -- every lane of the timed FP64 path, 1e-12; the mixed path
    against FP64 element by element (1e-6 or 6 estimated sigma)."""
    from synth.gpu import fill_props

    from bench import M_DECAY_S
    cfg = CONFIGS["h5"]
    V, T = cfg["L"] ** 3, cfg["T"]
    lanes = all_lanes(cfg)
    tl = B.TermList.spin_state(2, 2, True, 1, cfg["spins"], n_Lambda=1)
    P = []
    for stream, m in ((0, M_DECAY), (2, M_DECAY), (1, M_DECAY_S)):
        x = torch.empty((lanes, V, 1, 12, 12), dtype=torch.complex64, device="cuda")
        fill_props(x, seed=SEED, stream_id=stream, V=V, nsrc=1, T=T, first_bt=0, m=m)
        P.append(x)
    k = torch.from_numpy(kexp(lanes, T)).cuda()
    out = {}
    for prec in (B.MB_FP64, B.MB_MIXED):
        key = f"h5|{TUNE_LABEL[prec]}|{lanes}"
        best = autotune.committed(key)
        got = []
        for u, d in ((0, 1), (1, 0)):
            if prec != B.MB_FP64 and (u, d) == (1, 0):
                continue   # the mirror is checked on the FP64 path
            r = Runner(tl, P[u], P[d], prec, None, k, err_estimate=prec != B.MB_FP64, props_s=P[2])
            if best is None:
                best = autotune.tune(tl, r, key=None)
            else:
                autotune.apply(tl, best)
            r.ensure_workspace()
            corr, _ = r.run()
            torch.cuda.synchronize()
            got.append((corr.cpu().numpy(), None if prec == B.MB_FP64 else r.err[..., 0].cpu().numpy()))
            del r, corr
        out[prec] = got
    del P, k
    torch.cuda.empty_cache()
    (a, _), (b, _) = out[B.MB_FP64]
    assert_close(a, b, 1e-12, "h5 u <-> d mirror")
    (m, sig), = out[B.MB_MIXED]
    assert_close(m, a, 1e-6, "h5 mixed vs fp64", sigma=sig)
