"""Systems with one Lambda hyperon (third quark flavour s) on an MI355X:
the HIP path through the C ABI against the oracle.

The Lambda is the baryon form of Sec. 1 with (q1, q2, q3) = (s, u, d) and
the nucleons' Gamma matrices, added after the nucleons.  Checks: the Lambda
block against the oracle's (1e-12); correlators of the FP64 path against
the oracle (1e-12) for a single Lambda, Lambda + n, Lambda + p, the
hypertriton and Lambda + 3H, with one or two sources, u = d and u != d;
the mixed path against FP64 (1e-6, or within 6 of the library's estimated
standard deviations); every launch setting a Lambda step accepts; the
isospin mirror (u <-> d exchanges proton and neutron) at a larger volume;
and Lambda + 4He on two sources through the factorisation into the
oracle's one-source 4He and Lambda correlators (Sec. 6).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1301_4895_amd import binding as B
from paper_1301_4895_amd.runner import Runner
from tests.gpu_helpers import (assert_close, check_lane_exponent, host_props, lib_blocks, lib_lambda_block,
                               oracle_blocks_lib_layout)

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _tl(rel, nsrc, nP, nN, spins):
    if spins is None:
        return B.TermList(nP, nN, rel, nsrc, all_components=True, n_Lambda=1)
    return B.TermList.spin_state(nP, nN, rel, nsrc, spins, n_Lambda=1)


def _inputs(seed, nl, V, nsrc, dtype, same_ud, s_is_u=False, with_sink=True):
    Su = host_props(seed, 0, nl, 1, V, nsrc, dtype)[:, 0]
    Sd = Su if same_ud else host_props(seed, 1, nl, 1, V, nsrc, dtype)[:, 0]
    Ss = Su if s_is_u else host_props(seed, 2, nl, 1, V, nsrc, dtype)[:, 0]
    rng = np.random.default_rng(seed)
    w = (rng.normal(size=(nsrc, V)) + 1j * rng.normal(size=(nsrc, V))) if with_sink else None
    k = rng.integers(-3, 4, size=nl).astype(np.int32)
    return Su, Sd, Ss, w, k


def _runner(tl, Su, Sd, Ss, w, k, precision, err=False):
    tu = torch.from_numpy(np.ascontiguousarray(Su)).to(DEV)
    td = tu if Sd is Su else torch.from_numpy(np.ascontiguousarray(Sd)).to(DEV)
    ts = tu if Ss is Su else td if Ss is Sd else torch.from_numpy(np.ascontiguousarray(Ss)).to(DEV)
    tw = None if w is None else torch.from_numpy(np.ascontiguousarray(w)).to(DEV)
    r = Runner(tl, tu, td, precision, tw, torch.from_numpy(k).to(DEV), err_estimate=err, props_s=ts)
    return r


def _run(tl, Su, Sd, Ss, w, k, precision):
    r = _runner(tl, Su, Sd, Ss, w, k, precision, err=precision == B.MB_MIXED)
    corr, ex = r.run()
    torch.cuda.synchronize()
    sig = None if precision != B.MB_MIXED else r.err[..., 0].cpu().numpy()
    return r, corr.cpu().numpy(), ex.cpu().numpy(), sig


def _oracle(tl, rel, nsrc, nP, nN, Su, Sd, Ss, w, k):
    dl = np.concatenate([tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2), tl.export(B.MB_EXPORT_DELTA_L)[:, None]], 1)
    al = np.concatenate([tl.export(B.MB_EXPORT_ALPHA).reshape(-1, 2), tl.export(B.MB_EXPORT_ALPHA_L)[:, None]], 1)
    req = dict(sinkP=int(np.bitwise_or.reduce(dl[:, 0])), sinkN=int(np.bitwise_or.reduce(dl[:, 1])),
               sinkL=int(np.bitwise_or.reduce(dl[:, 2])), alphas=[tuple(map(int, a)) for a in al])
    c = O.hyperon_correlators(rel, nsrc, nP, nN, req, Su.astype(np.complex128), Sd.astype(np.complex128),
                              Ss.astype(np.complex128), w, 2.0 ** int(k))
    return np.array([[c[(tuple(map(int, d)), tuple(map(int, a)))] for a in al] for d in dl])


@pytest.mark.parametrize("kernel", [0, 2])
@pytest.mark.parametrize("rel,nsrc", [(False, 1), (True, 1), (False, 2)])
@pytest.mark.parametrize("same_ud,s_is_u", [(True, False), (False, False), (True, True)])
@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_lambda_block_matches_oracle(rel, nsrc, same_ud, s_is_u, dtype, kernel):
    V, nl = 27, 3
    Su, Sd, Ss, w, k = _inputs(61, nl, V, nsrc, dtype, same_ud, s_is_u)
    tl = _tl(rel, nsrc, 0, 1, None)
    tl.tune(0, B.MB_TUNE_BLOCKS, kernel)
    for prec in (B.MB_FP64, B.MB_MIXED):
        r = _runner(tl, Su, Sd, Ss, w, k, prec)
        r.run_blocks()
        torch.cuda.synchronize()
        blk, e = lib_blocks(r, tl)
        fl = lib_lambda_block(r, tl)
        blk, e, fl = blk.cpu().numpy(), e.cpu().numpy(), fl.cpu().numpy()
        for b in range(nl):
            check_lane_exponent(np.concatenate([blk[..., b].ravel(), fl[..., b].ravel()]), int(e[b]))
            S = [X[b].astype(np.complex128) for X in (Su, Sd, Ss)]
            fP, fN = O.blocks(rel, nsrc, S[0], S[1], w, 2.0 ** int(k[b]))
            fL = O.blocks_lambda(rel, nsrc, *S, w, 2.0 ** int(k[b]))
            ref = oracle_blocks_lib_layout(fP, fN) * 2.0 ** -int(e[b])
            for sp in range(2):
                assert_close(blk[sp, :, :, b], ref[sp], 1e-12, (prec, sp, b))
            assert_close(fl[:, :, b], fL.reshape(fL.shape[0], -1) * 2.0 ** -int(e[b]), 1e-12, (prec, "L", b))


LAMBDA_CASES = [
    # rel, nsrc, nP, nN, spins, V, lanes, same_ud
    (False, 1, 0, 0, None, 27, 3, False),          # a single Lambda
    (True, 1, 0, 0, None, 8, 2, True),
    (False, 1, 0, 1, None, 27, 3, True),           # Lambda + n, all components
    (False, 1, 0, 1, None, 8, 2, False),           # u != d
    (False, 1, 1, 0, None, 8, 2, True),            # Lambda + p
    (True, 1, 1, 0, (1, 2), 8, 1, False),          # relativistic, one spin component
    (False, 1, 1, 1, None, 8, 2, True),            # hypertriton
    (False, 1, 1, 2, (0, 0, 1, 1), 8, 1, True),    # Lambda + 3H
    (False, 2, 0, 1, (1, 2), 8, 2, True),          # two sources
    (False, 2, 1, 1, None, 8, 1, False),
]


@pytest.mark.parametrize("rel,nsrc,nP,nN,spins,V,nl,same_ud", LAMBDA_CASES)
def test_lambda_correlators_match_oracle(rel, nsrc, nP, nN, spins, V, nl, same_ud):
    Su, Sd, Ss, w, k = _inputs(70 + nP + 3 * nN + nsrc, nl, V, nsrc, np.complex128, same_ud)
    tl = _tl(rel, nsrc, nP, nN, spins)
    _, c64, ex, _ = _run(tl, Su, Sd, Ss, w, k, B.MB_FP64)
    assert np.array_equal(ex, 3 * (nP + nN + 1) * k)
    for b in range(nl):
        assert_close(c64[b], _oracle(tl, rel, nsrc, nP, nN, Su[b], Sd[b], Ss[b], w, k[b]), 1e-12, b)
    _, c32, ex32, sig = _run(tl, Su, Sd, Ss, w, k, B.MB_MIXED)
    assert np.array_equal(ex32, ex)
    assert_close(c32, c64, 1e-6, "mixed vs fp64", sigma=sig)


@pytest.mark.parametrize("precision,tol", [(B.MB_FP64, 1e-12), (B.MB_MIXED, 1e-6)])
def test_lambda_launch_settings_keep_results(precision, tol):
    """Every setting the Lambda step accepts (passthrough group, lane tile,
    splits in flight, grouped outputs) gives the same correlators; the
    LDS-staged kernel and the two-phase step are refused for it before any
    launch (MB_EUNSUPPORTED)."""
    rel, nsrc, nP, nN, V, nl = False, 1, 1, 1, 8, 70
    Su, Sd, Ss, w, k = _inputs(81, nl, V, nsrc, np.complex64, True)
    tl = _tl(rel, nsrc, nP, nN, None)
    _, ref, _, _ = _run(tl, Su, Sd, Ss, w, k, B.MB_FP64)
    last = tl.counts()["n_stages"] - 1
    assert tl.counts()["n_spin"][last] == 8   # 4 passthrough (proton, neutron) parts x 2 Lambda indices
    for pg, tile, unroll, group in [(1, 64, 1, 1), (2, 16, 2, 1), (2, 64, 2, 1), (1, 16, 1, 1), (1, 64, 0, 2),
                                    (2, 64, 0, 4), (0, 64, 0, 1)]:
        tl.tune(last, B.MB_TUNE_PASS_GROUP, pg)
        tl.tune(last, B.MB_TUNE_LANE_TILE, tile)
        tl.tune(last, B.MB_TUNE_UNROLL, unroll)
        tl.tune(last, B.MB_TUNE_GROUP, group)
        _, got, _, sig = _run(tl, Su, Sd, Ss, w, k, precision)
        assert_close(got, ref, tol, (pg, tile, unroll, group), sigma=sig)
    tl.tune(last, B.MB_TUNE_GROUP, 1)
    for what in (B.MB_TUNE_KERNEL, B.MB_TUNE_TWO_PHASE):
        tl.tune(last, what, 1)
        with pytest.raises(B.MBError) as e:
            _run(tl, Su, Sd, Ss, w, k, precision)
        assert e.value.code == B.MB_EUNSUPPORTED
        tl.tune(last, what, 0)


def test_lambda_isospin_mirror_at_larger_volume():
    """u <-> d maps the proton operator to minus the neutron's and the Lambda
    to minus itself, at sink and source alike (the oracle pins this on small
    inputs): C_{Lambda n}(S_u, S_d, S_s) = C_{Lambda p}(S_d, S_u, S_s)
    component by component, here at V = 16^3 with 64 lanes, and the same for
    the hypertriton with its proton and neutron indices exchanged."""
    V, nl = 16 ** 3, 64
    Su, Sd, Ss, w, k = _inputs(91, nl, V, 1, np.complex64, False)
    for prec, tol in [(B.MB_FP64, 1e-12), (B.MB_MIXED, 1e-6)]:
        tn = _tl(False, 1, 0, 1, None)
        tp = _tl(False, 1, 1, 0, None)
        _, cn, _, sn = _run(tn, Su, Sd, Ss, w, k, prec)
        _, cp, _, sp_ = _run(tp, Sd, Su, Ss, w, k, prec)
        # the same sink and source sets, neutron masks in place of proton masks
        assert np.array_equal(tn.export(B.MB_EXPORT_DELTA).reshape(-1, 2)[:, ::-1],
                              tp.export(B.MB_EXPORT_DELTA).reshape(-1, 2))
        assert_close(cn, cp, tol if prec == B.MB_FP64 else 2e-6, prec,
                     sigma=None if sn is None else np.hypot(sn, sp_))
    t3 = _tl(False, 1, 1, 1, None)
    _, a, _, _ = _run(t3, Su, Sd, Ss, w, k, B.MB_FP64)
    _, b, _, _ = _run(t3, Sd, Su, Ss, w, k, B.MB_FP64)
    dl = np.concatenate([t3.export(B.MB_EXPORT_DELTA).reshape(-1, 2), t3.export(B.MB_EXPORT_DELTA_L)[:, None]], 1)
    al = np.concatenate([t3.export(B.MB_EXPORT_ALPHA).reshape(-1, 2), t3.export(B.MB_EXPORT_ALPHA_L)[:, None]], 1)
    di = {tuple(d): i for i, d in enumerate(dl.tolist())}
    ai = {tuple(x): i for i, x in enumerate(al.tolist())}
    pd = [di[(d[1], d[0], d[2])] for d in dl.tolist()]
    pa = [ai[(x[1], x[0], x[2])] for x in al.tolist()]
    assert_close(a, b[:, pd][:, :, pa], 1e-12, "hypertriton mirror")


def test_lambda_4he_two_source_factorisation():
    """Lambda + 4He (nonrelativistic): the 4He from source 0 and the Lambda
    from source 1, each source and its sink function on its own half of the
    sites (Sec. 6): the correlator is the product of the oracle's one-source
    4He correlator and the single-Lambda closed form.  psi = 2 alpha + s:
    protons and neutrons {0, 2}, the Lambda 1."""
    V = 16
    half = V // 2
    S = [host_props(95, j, 1, 1, V, 2, np.complex128)[0, 0].copy() for j in range(3)]
    for X in S:
        X[half:, 0] = 0
        X[:half, 1] = 0
    rng = np.random.default_rng(5)
    w = np.zeros((2, V), np.complex128)
    w[0, :half] = rng.normal(size=half) + 1j * rng.normal(size=half)
    w[1, half:] = rng.normal(size=half) + 1j * rng.normal(size=half)
    tl = _tl(False, 2, 2, 2, (0, 2, 0, 2, 1))
    k = np.array([1], np.int32)
    for prec, tol in [(B.MB_FP64, 1e-12), (B.MB_MIXED, 1e-6)]:
        _, corr, ex, sig = _run(tl, S[0][None], S[1][None], S[2][None], w, k, prec)
        assert ex[0] == 15
        req = O.spin_state_request(2, 2, (0, 1, 0, 1))
        c4 = O.correlators(False, 1, 2, 2, req, S[0][:, :1], S[1][:, :1], w[:1], 2.0)[((3, 3), (3, 3))]
        cl = O.lambda_closed(False, S[0][:, 1:], S[1][:, 1:], S[2][:, 1:], w[1:], 2.0, 0, 0)
        ref = np.array([[c4 * cl]])
        assert abs(ref[0, 0]) > 0
        assert_close(corr[0], ref, tol, prec, sigma=None if sig is None else sig[0])
