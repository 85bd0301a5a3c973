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
FP64 path: 1e-12 relative; mixed path: 1e-6 relative.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from bench import CONFIGS, M_DECAY
from oracle import oracle as O
from paper_1301_4895_amd import binding as B
from paper_1301_4895_amd.runner import Runner
from synth import props as SP
from tests.gpu_helpers import check_lane_exponent, lib_blocks, oracle_blocks_lib_layout, rel_err

pytestmark = pytest.mark.gpu

SEED = 2013


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
    out = {}
    for prec in (B.MB_FP64, B.MB_MIXED):
        r = Runner(tl, props, props, prec, None, k)
        corr, _ = r.run()
        torch.cuda.synchronize()
        out[prec] = (corr.cpu().numpy(), r)
    dsets = tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2)
    asets = tl.export(B.MB_EXPORT_ALPHA).reshape(-1, 2)
    pairs = [(i, j) for i in (0, 14, 35) for j in (0, 21)]
    for lane in (3, 197, 700):
        S = host_lane(cfg, lane)
        kk = int(kexp(lanes, cfg["T"])[lane])
        fP, fN = O.blocks(True, 1, S, S, None, 2.0 ** kk)
        got_blocks, e = lane_blocks(out[B.MB_FP64][1], tl, lane)
        ref_blocks = oracle_blocks_lib_layout(fP, fN) * 2.0 ** -e
        assert rel_err(got_blocks, ref_blocks) <= 1e-12
        for i, j in pairs:
            d, a = tuple(map(int, dsets[i])), tuple(map(int, asets[j]))
            um, dm, cf = O.L_for_alpha(True, 1, 2, 2, a)
            ref = O.corr_from_L([0, 0, 1, 1], O._bits(d[0]) + O._bits(d[1]), fP, fN, um, dm, cf)
            assert abs(ref) > 0
            assert abs(out[B.MB_FP64][0][lane, i, j] - ref) <= 1e-12 * abs(ref), (lane, i, j)
        # mixed against FP64 on the whole lane
        assert rel_err(out[B.MB_MIXED][0][lane], out[B.MB_FP64][0][lane]) <= 1e-6


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
    r = Runner(tl, props, props, B.MB_FP64, torch.from_numpy(w).cuda(), k)
    r.run_blocks()
    torch.cuda.synchronize()
    lane = 877
    S = host_lane(cfg, lane)
    fP, fN = O.blocks(False, 2, S, S, w, 2.0 ** int(kexp(lanes, cfg["T"])[lane]))
    got_blocks, e = lane_blocks(r, tl, lane)
    ref_blocks = oracle_blocks_lib_layout(fP, fN) * 2.0 ** -e
    assert rel_err(got_blocks, ref_blocks) <= 1e-12
    del r
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
    for prec in (B.MB_FP64, B.MB_MIXED):
        rr = Runner(tl, props, props, prec, torch.from_numpy(wr).cuda(), k)
        corr, _ = rr.run()
        torch.cuda.synchronize()
        res[prec] = corr.cpu().numpy()[:, 0, 0]
        del rr
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
        assert abs(res[B.MB_MIXED][lane] - ref) <= 1e-6 * abs(ref), lane
