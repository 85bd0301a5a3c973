"""The float-block mixed mode (MB_MIXED_F32B) on an MI355X, through the C ABI.

Its recursion steps read float copies of the scaled blocks; stages are
stored in float as in MB_MIXED and every product and sum is formed in
double.  Checks: the copies are the double entries rounded to nearest (bit
for bit, every species, the Lambda's included); correlators within 1e-6 of
the FP64 path (element by element, or within 6 of the library's estimated
standard deviations, or of the first-order bound where one component per
lane is asked for) and of the oracle; the error estimate (err_out), which
adds the rounding of the block copies, bounds the measured deviation; every
launch setting the mode accepts gives the same correlators, and the
LDS-staged kernel, which it has no form of, is refused before any launch;
three sources with up to six sink indices per species.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1301_4895_amd import binding as B
from paper_1301_4895_amd.runner import Runner
from tests.gpu_helpers import assert_close, host_props

pytestmark = pytest.mark.gpu

DEV = "cuda"

CASES = [
    (False, 1, 2, 2, (0, 1, 0, 1), 512, 64, np.complex128),             # 4He NR
    (True, 1, 2, 2, None, 216, 64, np.complex64),                        # 4He rel, all components
    (False, 2, 4, 4, (0, 1, 2, 3, 0, 1, 2, 3), 512, 64, np.complex64),  # 8Be NR, two sources
]


def _tl(rel, nsrc, nP, nN, spins, n_Lambda=0):
    if spins is None:
        return B.TermList(nP, nN, rel, nsrc, all_components=True, n_Lambda=n_Lambda)
    return B.TermList.spin_state(nP, nN, rel, nsrc, spins, n_Lambda=n_Lambda)


def _inputs(seed, nl, V, nsrc, dtype, with_sink):
    Su = host_props(seed, 0, nl, 1, V, nsrc, dtype)[:, 0]
    rng = np.random.default_rng(seed)
    w = (rng.normal(size=(nsrc, V)) + 1j * rng.normal(size=(nsrc, V))) if with_sink else None
    k = rng.integers(-3, 4, size=nl).astype(np.int32)
    return Su, w, k


def _runner(tl, Su, w, k, prec, err=False, Ss=None):
    tu = torch.from_numpy(np.ascontiguousarray(Su)).to(DEV)
    tw = None if w is None else torch.from_numpy(np.ascontiguousarray(w)).to(DEV)
    ts = None if Ss is None else torch.from_numpy(np.ascontiguousarray(Ss)).to(DEV)
    return Runner(tl, tu, tu, prec, tw, torch.from_numpy(k).to(DEV), err_estimate=err, props_s=ts)


def _accept(err, spins):
    """The sigma of assert_close: the estimated standard deviation, or for
    one-component outputs a sixth of the first-order bound (a rounded block
    copy enters many splits of one output coherently, beyond sigma's
    independence model)."""
    return err[..., 0] if spins is None else err[..., 1] / 6


def _run(tl, Su, w, k, prec, Ss=None):
    """Correlators and (mixed modes) the estimated (sigma, bound) per output."""
    r = _runner(tl, Su, w, k, prec, err=prec != B.MB_FP64, Ss=Ss)
    corr, _ = r.run()
    torch.cuda.synchronize()
    return corr.cpu().numpy(), (None if prec == B.MB_FP64 else r.err.cpu().numpy())


def _bases(tl):
    """Sink base sets (sorted spin indices) of proton, neutron and Lambda."""
    d = tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2)
    m = [int(np.bitwise_or.reduce(d[:, 0])), int(np.bitwise_or.reduce(d[:, 1]))]
    m.append(int(np.bitwise_or.reduce(tl.export(B.MB_EXPORT_DELTA_L))) if tl.counts().get("n_Lambda") else 0)
    return [[i for i in range(32) if x >> i & 1] for x in m]


def test_block_copies_are_the_rounded_entries():
    """The float copies after the exponents (padded to 256 bytes), species by
    species: block entry (y, psi_of_pos[2j + h]) of lane b rounded to nearest
    at complex float h of pair ((y * Bp/16 + b/16) * P + j) * 16 + b % 16,
    P = ceil(M / 2) position pairs of the species' M base-set positions,
    the odd tail zero."""
    nl, V = 70, 27
    Su, w, k = _inputs(5, nl, V, 1, np.complex64, False)
    Ss = host_props(5, 2, nl, 1, V, 1, np.complex64)[:, 0]
    for tl, s in ((_tl(True, 1, 2, 2, None), None), (_tl(False, 1, 2, 1, (0, 1, 1, 0), n_Lambda=1), Ss),
                  (_tl(False, 2, 1, 1, (0, 3, 1), n_Lambda=1), None)):
        if s is None and tl.counts().get("n_Lambda"):
            s = Su
        r = _runner(tl, Su, w, k, B.MB_MIXED_F32B, Ss=s)
        r.run()
        torch.cuda.synchronize()
        c = tl.counts()
        nxi, npsi = c["n_xi"], c["n_psi"]
        Bp = (nl + 63) // 64 * 64
        nyq = nxi * (nxi - 1) // 2 * nxi
        rows = [nyq, nyq, nxi ** 3 if c.get("n_Lambda") else 0]
        raw = r.blocks.cpu().numpy()
        d0, off = 0, sum(rows) * npsi * Bp * 16
        off += (4 * Bp + 255) // 256 * 256
        for sp, base in enumerate(_bases(tl)):
            n = rows[sp] * npsi * Bp * 16
            dbl = raw[d0:d0 + n].view(np.complex128).reshape(rows[sp], Bp // 16, npsi, 16)
            d0 += n
            P = (len(base) + 1) // 2
            exp = np.zeros((rows[sp], Bp // 16, P, 16, 2), np.complex64)
            for q, psi in enumerate(base):
                exp[:, :, q // 2, :, q % 2] = dbl[:, :, psi, :].astype(np.complex64)
            nb = rows[sp] * Bp * P * 16
            got = raw[off:off + nb].view(np.complex64).reshape(exp.shape)
            off += (nb + 255) // 256 * 256
            assert np.array_equal(got.view(np.uint32), exp.view(np.uint32)), (sp, base)
            assert nb == 0 or np.count_nonzero(got) > 0
        assert off == r.blocks.numel()


@pytest.mark.parametrize("rel,nsrc,nP,nN,spins,V,nl,dtype", CASES)
def test_float_blocks_match_fp64(rel, nsrc, nP, nN, spins, V, nl, dtype):
    Su, w, k = _inputs(9, nl, V, nsrc, dtype, nsrc >= 2)
    tl = _tl(rel, nsrc, nP, nN, spins)
    c64, _ = _run(tl, Su, w, k, B.MB_FP64)
    cm, _ = _run(tl, Su, w, k, B.MB_MIXED)
    cb, eb = _run(tl, Su, w, k, B.MB_MIXED_F32B)
    assert_close(cb, c64, 1e-6, "float blocks vs fp64", sigma=_accept(eb, spins))
    # the float copies are what the steps read: the results differ from MB_MIXED
    assert not np.array_equal(cb, cm)


def test_float_blocks_match_oracle():
    """4He nonrelativistic (one spin state) with u != d against the oracle."""
    nl, V = 2, 27
    Su = host_props(17, 0, nl, 1, V, 1, np.complex64)[:, 0]
    Sd = host_props(17, 1, nl, 1, V, 1, np.complex64)[:, 0]
    k = np.array([0, 2], np.int32)
    tl = _tl(False, 1, 2, 2, (0, 1, 0, 1))
    r = Runner(tl, torch.from_numpy(Su).to(DEV), torch.from_numpy(Sd).to(DEV), B.MB_MIXED_F32B, None,
               torch.from_numpy(k).to(DEV), err_estimate=True)
    corr, _ = r.run()
    torch.cuda.synchronize()
    got = corr.cpu().numpy()
    sig = _accept(r.err.cpu().numpy(), (0, 1, 0, 1))
    dsets = tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2)
    asets = tl.export(B.MB_EXPORT_ALPHA).reshape(-1, 2)
    req = dict(sinkP=int(np.bitwise_or.reduce(dsets[:, 0])), sinkN=int(np.bitwise_or.reduce(dsets[:, 1])),
               alphas=[tuple(map(int, a)) for a in asets])
    ref = np.zeros_like(got)
    for b in range(nl):
        Cd = O.correlators(False, 1, 2, 2, req, Su[b].astype(np.complex128), Sd[b].astype(np.complex128), None,
                           2.0 ** int(k[b]))
        for i, d in enumerate(map(tuple, dsets.tolist())):
            for j, a in enumerate(map(tuple, asets.tolist())):
                ref[b, i, j] = Cd[(d, a)]
    assert_close(got, ref, 1e-6, "float blocks vs oracle", sigma=sig)


def test_float_blocks_with_a_lambda():
    nl, V = 64, 64
    Su, w, k = _inputs(33, nl, V, 2, np.complex64, True)
    Ss = host_props(33, 2, nl, 1, V, 2, np.complex64)[:, 0]
    tl = _tl(False, 2, 1, 1, (0, 1, 2), n_Lambda=1)
    c64, _ = _run(tl, Su, w, k, B.MB_FP64, Ss=Ss)
    cb, eb = _run(tl, Su, w, k, B.MB_MIXED_F32B, Ss=Ss)
    assert_close(cb, c64, 1e-6, "float blocks vs fp64 (Lambda + p + n)", sigma=_accept(eb, (0, 1, 2)))


@pytest.mark.parametrize("two_phase", [0, 1])
@pytest.mark.parametrize("rel,nsrc,nP,nN,spins,V,nl,dtype", CASES)
def test_error_estimate_covers_the_float_block_deviation(rel, nsrc, nP, nN, spins, V, nl, dtype, two_phase):
    """Every component within its first-order bound of the FP64 result; for
    all-component lists also within 6 estimated standard deviations, and per
    lane the estimated deviation is neither below a sixth nor above 100
    times the measured one (one-component outputs: sigma underestimates the
    coherent block-copy rounding, so only the bound is asserted there)."""
    Su, w, k = _inputs(9, nl, V, nsrc, dtype, nsrc >= 2)
    tl = _tl(rel, nsrc, nP, nN, spins)
    for s in range(1, tl.counts()["n_stages"]):
        tl.tune(s, B.MB_TUNE_TWO_PHASE, two_phase)
    c64, _ = _run(tl, Su, w, k, B.MB_FP64)
    r = _runner(tl, Su, w, k, B.MB_MIXED_F32B, err=True)
    r.err_all.fill_(float("nan"))
    corr, _ = r.run()
    torch.cuda.synchronize()
    cb, eb = corr.cpu().numpy(), r.err.cpu().numpy()
    # the error estimate does not change the correlators
    plain = _runner(tl, Su, w, k, B.MB_MIXED_F32B)
    assert np.array_equal(plain.run()[0].cpu().numpy(), cb)
    d = np.abs(cb - c64)
    sigma, bound = eb[..., 0], eb[..., 1]
    assert np.all(np.isfinite(sigma)) and np.all(np.isfinite(bound))
    assert np.all(d <= bound), float((d / bound).max())
    assert np.all(sigma > 0)
    nd = np.sqrt((d ** 2).reshape(nl, -1).sum(1))
    ns = np.sqrt((sigma ** 2).reshape(nl, -1).sum(1))
    ratio = ns / nd
    print(f"sigma/deviation per lane: min {ratio.min():.3g} median {np.median(ratio):.3g} max {ratio.max():.3g}")
    if spins is None:
        assert np.all(d <= 6 * sigma), float((d / sigma).max())
        assert ratio.min() >= 1 / 6 and ratio.max() <= 100, (ratio.min(), ratio.max())


@pytest.mark.parametrize("rel,nsrc,nP,nN,spins,V,nl", [
    (True, 1, 2, 2, None, 27, 64),
    (False, 2, 2, 2, (0, 2, 0, 2), 8, 70),
    (False, 2, 4, 4, (0, 1, 2, 3, 0, 1, 2, 3), 8, 20),
])
def test_float_block_launch_settings_keep_results(rel, nsrc, nP, nN, spins, V, nl):
    """Direct kernel (tiles, passthrough groups, splits in flight, two-phase)
    and grouped kernel give the same correlators; the LDS-staged kernel,
    which stages double rows, is refused before any launch."""
    Su, w, k = _inputs(13, nl, V, nsrc, np.complex64, nsrc >= 2)
    tl = _tl(rel, nsrc, nP, nN, spins)
    ref, _ = _run(tl, Su, w, k, B.MB_FP64)
    nst = tl.counts()["n_stages"]
    for kern, pg, tile, unroll, group, two in [
            (0, 1, 16, 1, 1, 0), (0, 3, 16, 2, 1, 0), (0, 6, 64, 2, 1, 0), (0, 2, 64, 1, 1, 0),
            (0, 1, 64, 0, 2, 0), (0, 3, 64, 0, 4, 0), (0, 6, 64, 2, 1, 1), (0, 1, 16, 2, 1, 1),
            (1, 1, 16, 0, 1, 0)]:
        for s in range(1, nst):
            tl.tune(s, B.MB_TUNE_KERNEL, kern)
            tl.tune(s, B.MB_TUNE_UNROLL, unroll)
            tl.tune(s, B.MB_TUNE_GROUP, group)
            tl.tune(s, B.MB_TUNE_TWO_PHASE, two)
            try:
                tl.tune(s, B.MB_TUNE_PASS_GROUP, pg)
            except B.MBError:
                tl.tune(s, B.MB_TUNE_PASS_GROUP, 1)
            tl.tune(s, B.MB_TUNE_LANE_TILE, tile)
            tl.tune(s, B.MB_TUNE_LDS_BYTES, 0)
        if kern == 1:
            with pytest.raises(B.MBError) as ei:
                _run(tl, Su, w, k, B.MB_MIXED_F32B)
            assert ei.value.code == B.MB_EUNSUPPORTED
            continue
        got, e = _run(tl, Su, w, k, B.MB_MIXED_F32B)
        assert_close(got, ref, 1e-6, (kern, pg, tile, unroll, group, two), sigma=_accept(e, spins))


@pytest.mark.parametrize("nP,nN,spins,nl,V", [
    (1, 2, (0, 1, 5), 20, 8),             # at most two sink indices per species
    (0, 5, (0, 3, 1, 4, 2), 64, 64),      # five neutrons: five sink indices (odd: a padded pair)
    (0, 3, None, 8, 8),                   # three neutrons, all components: six sink indices
])
def test_three_sources(nP, nN, spins, nl, V):
    """Three sources, including the steps with five and six sink indices per
    species, against FP64 (element by element within 1e-6, or the bound or
    6 sigma) and within the first-order bound."""
    Su, w, k = _inputs(3, nl, V, 3, np.complex64, True)
    tl = _tl(False, 3, nP, nN, spins)
    c64, _ = _run(tl, Su, w, k, B.MB_FP64)
    cb, eb = _run(tl, Su, w, k, B.MB_MIXED_F32B)
    assert_close(cb, c64, 1e-6, "float blocks vs fp64 (three sources)", sigma=_accept(eb, spins))
    assert np.all(np.abs(cb - c64) <= eb[..., 1])


def test_projected_and_side_outputs():
    """Projected lists (one output per lane) and side nuclei (final sums of
    earlier stages) read the float-block stages like the main output: every
    output within its first-order bound of FP64, and element by element
    within 1e-6 (or the bound)."""
    from tests.spin_weights import sparse_weights
    nl, V = 3, 27
    Su, w, k = _inputs(91, nl, V, 1, np.complex64, False)
    full = B.TermList(2, 1, False, 1, all_components=True)
    cf = full.counts()
    W = sparse_weights((cf["n_delta"], cf["n_alpha"]), 7, 0.3)
    for tl in (B.TermList(2, 1, False, 1, all_components=True, proj=W),
               B.TermList(2, 1, False, 1, all_components=True, sides=[(0, None), (1, None)])):
        res = {}
        for prec in (B.MB_FP64, B.MB_MIXED_F32B):
            r = _runner(tl, Su, w, k, prec, err=True)
            r.run()
            torch.cuda.synchronize()
            res[prec] = (r.out.cpu().numpy(), r.err_all.cpu().numpy())
        got, ref = res[B.MB_MIXED_F32B][0], res[B.MB_FP64][0]
        bound = res[B.MB_MIXED_F32B][1][:, 1]
        d = np.abs(got - ref)
        assert np.all(d <= bound), float((d / bound).max())
        assert_close(got.reshape(nl, -1), ref.reshape(nl, -1), 1e-6, "float blocks vs fp64",
                     sigma=(bound / 6).reshape(nl, -1))
        assert np.all(res[B.MB_FP64][1] == 0)
