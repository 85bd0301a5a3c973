"""The two small workloads at their full sizes, as bench.py runs them
(device-generated propagators, 2^k(t) rescale, every lane in one launch):

  * p+n NR, all components, L=4 T=8, one problem, complex128: every lane of
    the FP64 path against the oracle (1e-12), mixed against FP64 (1e-6);
    element by element (tests.gpu_helpers.assert_close);
  * 4He NR (0,1,0,1), L=16 T=32, 8 problems, complex128: mixed against FP64
    on all 256 lanes, FP64 against the oracle on sampled lanes.
"""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from bench import CONFIGS, M_DECAY
from oracle import oracle as O
from paper_1301_4895_amd import binding as B
from paper_1301_4895_amd.runner import Runner
from synth import props as SP
from tests.gpu_helpers import assert_close

pytestmark = pytest.mark.gpu

SEED = 2013


def _run(name, lanes_checked):
    cfg = CONFIGS[name]
    V, T, nsrc = cfg["L"] ** 3, cfg["T"], cfg["nsrc"]
    lanes = cfg["nprob"] * T
    tl = (B.TermList(cfg["nP"], cfg["nN"], cfg["rel"], nsrc, all_components=True) if cfg["spins"] is None
          else B.TermList.spin_state(cfg["nP"], cfg["nN"], cfg["rel"], nsrc, cfg["spins"]))
    from synth.gpu import fill_props
    props = torch.empty((lanes, V, nsrc, 12, 12), dtype=torch.complex128, device="cuda")
    fill_props(props, seed=SEED, stream_id=0, V=V, nsrc=nsrc, T=T, first_bt=0, m=M_DECAY)
    kexp = np.array([int(math.floor(M_DECAY * (b % T) / math.log(2.0) + 0.5)) for b in range(lanes)], np.int32)
    k = torch.from_numpy(kexp).cuda()
    out, sig = {}, []
    for prec in (B.MB_FP64, B.MB_MIXED):
        chunks = []
        for b0 in range(0, lanes, 256):
            r = Runner(tl, props[b0:b0 + 256], props[b0:b0 + 256], prec, None, k[b0:b0 + 256],
                       err_estimate=prec == B.MB_MIXED)
            corr, ex = r.run()
            torch.cuda.synchronize()
            assert np.array_equal(ex.cpu().numpy(), 3 * (cfg["nP"] + cfg["nN"]) * kexp[b0:b0 + 256])
            chunks.append(corr.cpu().numpy())
            if prec == B.MB_MIXED:
                sig.append(r.err[..., 0].cpu().numpy())
            del r
        out[prec] = np.concatenate(chunks)
    assert_close(out[B.MB_MIXED], out[B.MB_FP64], 1e-6, "mixed vs fp64", sigma=np.concatenate(sig))
    dsets = tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2)
    asets = tl.export(B.MB_EXPORT_ALPHA).reshape(-1, 2)
    req = dict(sinkP=int(np.bitwise_or.reduce(dsets[:, 0])), sinkN=int(np.bitwise_or.reduce(dsets[:, 1])),
               alphas=[tuple(map(int, a)) for a in asets])
    O.set_threads(min(16, os.cpu_count() or 1))
    for lane in lanes_checked(lanes):
        S = SP.props(SEED, 0, cfg["nprob"], T, V, nsrc, M_DECAY, np.complex128, probs=[lane // T],
                     ts=[lane % T])[0, 0]
        Cd = O.correlators(cfg["rel"], nsrc, cfg["nP"], cfg["nN"], req, S, S, None, 2.0 ** int(kexp[lane]))
        ref = np.array([[Cd[(tuple(map(int, d)), tuple(map(int, a)))] for a in asets] for d in dsets])
        assert_close(out[B.MB_FP64][lane], ref, 1e-12, lane)


def test_pn_nonrelativistic_small_workload():
    _run("c1", lambda n: range(n))


def test_4he_nonrelativistic_workload():
    _run("c2", lambda n: (0, 31, 100, 255))
