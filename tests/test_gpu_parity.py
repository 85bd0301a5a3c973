"""Parity of the HIP path (through the C ABI) with the oracle, on an MI355X.

Every input is seeded and synthetic (synth.props).  Tolerances:
  * FP64 path vs oracle: 1e-12 relative, blocks and correlators;
  * mixed path vs FP64 path and vs oracle: 1e-6 relative.
Every comparison is per lane and element by element (tests.gpu_helpers.
assert_close): the Frobenius norm over the lane's components, every
component of at least 1e-3 of the lane's largest within tol of itself, and
every other component (exact zeros included) within tol of the largest.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1301_4895_amd import binding as B
from paper_1301_4895_amd.runner import Runner
from tests.gpu_helpers import assert_close, check_lane_exponent, host_props, lib_blocks, oracle_blocks_lib_layout

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _tl(rel, nsrc, nP, nN, spins):
    if spins is None:
        return B.TermList(nP, nN, rel, nsrc, all_components=True)
    return B.TermList.spin_state(nP, nN, rel, nsrc, spins)


def _inputs(seed, nlanes, V, nsrc, dtype, same_ud, with_sink, rng_k=True):
    Su = host_props(seed, 0, nlanes, 1, V, nsrc, dtype)[:, 0]
    Sd = Su if same_ud else host_props(seed, 1, nlanes, 1, V, nsrc, dtype)[:, 0]
    rng = np.random.default_rng(seed)
    w = None
    if with_sink:
        w = rng.normal(size=(nsrc, V)) + 1j * rng.normal(size=(nsrc, V))
    k = rng.integers(-3, 4, size=nlanes).astype(np.int32) if rng_k else np.zeros(nlanes, np.int32)
    return Su, Sd, w, k


def _run(tl, Su, Sd, w, k, precision):
    tu = torch.from_numpy(np.ascontiguousarray(Su)).to(DEV)
    td = tu if Sd is Su else torch.from_numpy(np.ascontiguousarray(Sd)).to(DEV)
    tw = None if w is None else torch.from_numpy(np.ascontiguousarray(w)).to(DEV)
    tk = torch.from_numpy(k).to(DEV)
    r = Runner(tl, tu, td, precision, tw, tk)
    corr, ex = r.run()
    torch.cuda.synchronize()
    blk, e = lib_blocks(r, tl)
    blocks = blk[..., :len(Su)].cpu().numpy()
    e = e[:len(Su)].cpu().numpy()
    for b in range(len(Su)):
        check_lane_exponent(blocks[..., b], int(e[b]))
    return (blocks, e), corr.cpu().numpy(), ex.cpu().numpy()


def _mixed(tl, Su, Sd, w, k):
    """Mixed-path correlators and the library's estimated standard deviation
    of each one's rounding error (err_out[..., 0])."""
    tu = torch.from_numpy(np.ascontiguousarray(Su)).to(DEV)
    td = tu if Sd is Su else torch.from_numpy(np.ascontiguousarray(Sd)).to(DEV)
    tw = None if w is None else torch.from_numpy(np.ascontiguousarray(w)).to(DEV)
    r = Runner(tl, tu, td, B.MB_MIXED, tw, torch.from_numpy(k).to(DEV), err_estimate=True)
    corr, _ = r.run()
    torch.cuda.synchronize()
    return corr.cpu().numpy(), r.err[..., 0].cpu().numpy()


def _oracle_corr(tl, rel, nsrc, nP, nN, Su, Sd, w, k):
    """Oracle correlators in the library's [delta][alpha] order, one lane."""
    dsets = tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2)
    asets = tl.export(B.MB_EXPORT_ALPHA).reshape(-1, 2)
    req = dict(sinkP=int(np.bitwise_or.reduce(dsets[:, 0])), sinkN=int(np.bitwise_or.reduce(dsets[:, 1])),
               alphas=[tuple(map(int, a)) for a in asets])
    Cd = O.correlators(rel, nsrc, nP, nN, req, Su.astype(np.complex128), Sd.astype(np.complex128), w,
                       2.0 ** int(k))
    out = np.zeros((len(dsets), len(asets)), np.complex128)
    for i, d in enumerate(map(tuple, dsets.tolist())):
        for j, a in enumerate(map(tuple, asets.tolist())):
            out[i, j] = Cd[(d, a)]
    return out


# --------------------------------------------------------------------- inputs

def test_device_generator_matches_host():
    from synth.gpu import fill_props
    for dt, tdt in [(np.complex128, torch.complex128), (np.complex64, torch.complex64)]:
        host = host_props(7, 3, 2, 3, 5, 2, dt).reshape(6, 5, 2, 12, 12)
        dev = torch.empty((4, 5, 2, 12, 12), dtype=tdt, device=DEV)
        fill_props(dev, 7, 3, 5, 2, 3, 1)          # units 1..4 of a (2 problems x 3 t) set
        assert np.array_equal(dev.cpu().numpy(), host[1:5])


# --------------------------------------------------------------------- blocks

@pytest.mark.parametrize("kernel", [0, 2])
@pytest.mark.parametrize("rel,nsrc", [(False, 1), (True, 1), (False, 2), (False, 3)])
@pytest.mark.parametrize("same_ud", [True, False])
@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_blocks_match_oracle(rel, nsrc, same_ud, dtype, kernel):
    """Blocks of both site-sum kernels (MB_TUNE_BLOCKS 0: matrix cores where
    the shape has them, 2: register-tiled vector units) against the
    oracle's."""
    V, nl = 27, 3
    Su, Sd, w, k = _inputs(11, nl, V, nsrc, dtype, same_ud, with_sink=nsrc >= 2 or rel)
    tl = _tl(rel, nsrc, 1, 1, None)
    tl.tune(0, B.MB_TUNE_BLOCKS, kernel)
    for prec, tol in [(B.MB_FP64, 1e-12), (B.MB_MIXED, 1e-12)]:
        (blocks, e), _, _ = _run(tl, Su, Sd, w, k, prec)
        for b in range(nl):
            fP, fN = O.blocks(rel, nsrc, Su[b].astype(np.complex128), Sd[b].astype(np.complex128), w,
                              2.0 ** int(k[b]))
            ref = oracle_blocks_lib_layout(fP, fN) * 2.0 ** -int(e[b])
            for sp in range(2):
                assert_close(blocks[sp, :, :, b], ref[sp], tol, (prec, sp, b))


# --------------------------------------------------------------------- correlators

CORR_CASES = [
    # rel, nsrc, nP, nN, spins, V, lanes, same_ud
    (False, 1, 1, 1, None, 64, 4, True),          # p+n, the small configuration
    (False, 1, 1, 1, None, 8, 2, False),          # p+n with u != d
    (False, 1, 2, 0, None, 8, 2, True),           # pp
    (False, 1, 0, 2, None, 8, 2, True),           # nn
    (False, 1, 2, 1, None, 8, 2, True),           # 3He
    (False, 1, 1, 2, None, 8, 2, False),          # 3H, u != d
    (False, 1, 2, 2, (0, 1, 0, 1), 27, 2, True),  # 4He NR
    (False, 1, 1, 0, None, 8, 2, False),          # single proton
    (True, 1, 1, 1, None, 8, 1, True),            # p+n relativistic, all components
    (True, 1, 1, 2, (0, 0, 1), 8, 1, True),       # 3H relativistic
    (True, 1, 2, 2, (0, 1, 0, 1), 8, 1, True),    # 4He relativistic
    (False, 2, 1, 1, None, 8, 2, True),           # p+n, two sources
    (False, 2, 2, 2, (0, 2, 0, 2), 8, 1, True),   # 4He NR, two sources
    (False, 2, 0, 3, (0, 1, 2), 8, 1, True),      # 3n, two sources
    (False, 3, 1, 1, None, 8, 2, True),           # p+n, three sources (Sec. 6)
    (False, 3, 0, 3, (0, 2, 4), 8, 1, True),      # 3n, one neutron per source
    (False, 3, 1, 2, (0, 1, 5), 8, 2, False),     # 3H, three sources, u != d
    (False, 3, 2, 2, (0, 4, 1, 5), 8, 1, True),   # 4He, three sources
]


@pytest.mark.parametrize("rel,nsrc,nP,nN,spins,V,nl,same_ud", CORR_CASES)
def test_correlators_fp64_match_oracle(rel, nsrc, nP, nN, spins, V, nl, same_ud):
    Su, Sd, w, k = _inputs(5 + nP + 3 * nN, nl, V, nsrc, np.complex128, same_ud, with_sink=nsrc >= 2)
    tl = _tl(rel, nsrc, nP, nN, spins)
    _, corr, ex = _run(tl, Su, Sd, w, k, B.MB_FP64)
    A = nP + nN
    assert np.array_equal(ex, 3 * A * k)
    for b in range(nl):
        ref = _oracle_corr(tl, rel, nsrc, nP, nN, Su[b], Sd[b], w, k[b])
        assert_close(corr[b], ref, 1e-12, b)


def test_pauli_zero_with_identical_sink_functions():
    # 4He with two sources and the same sink function on both: the two rows
    # with equal alpha coincide and the antisymmetrised product vanishes.
    V, nl = 8, 1
    Su, Sd, _, k = _inputs(3, nl, V, 2, np.complex128, True, False)
    tl = _tl(False, 2, 2, 2, (0, 1, 0, 1))
    _, corr, _ = _run(tl, Su, Sd, None, k, B.MB_FP64)
    tl2 = _tl(False, 2, 2, 2, (0, 2, 0, 2))
    _, corr2, _ = _run(tl2, Su, Sd, None, k, B.MB_FP64)
    assert abs(corr[0, 0, 0]) <= 1e-12 * abs(corr2[0, 0, 0])


def test_8be_two_source_factorisation():
    """8Be (NR, two sources) on disjoint regions equals the product of two
    one-source 4He correlators, each from the oracle (Sec. 6)."""
    V = 8
    half = V // 2
    S = host_props(21, 0, 1, 1, V, 2, np.complex128)[0, 0].copy()
    S[half:, 0] = 0
    S[:half, 1] = 0
    rng = np.random.default_rng(4)
    w = np.zeros((2, V), np.complex128)
    w[0, :half] = rng.normal(size=half) + 1j * rng.normal(size=half)
    w[1, half:] = rng.normal(size=half) + 1j * rng.normal(size=half)
    tl = _tl(False, 2, 4, 4, (0, 1, 2, 3, 0, 1, 2, 3))
    k = np.array([1], np.int32)
    _, corr, _ = _run(tl, S[None], S[None], w, k, B.MB_FP64)
    req = O.spin_state_request(2, 2, (0, 1, 0, 1))
    c0 = O.correlators(False, 1, 2, 2, req, S[:, :1], S[:, :1], w[:1], 2.0)[((3, 3), (3, 3))]
    c1 = O.correlators(False, 1, 2, 2, req, S[:, 1:], S[:, 1:], w[1:], 2.0)[((3, 3), (3, 3))]
    assert abs(c0 * c1) > 0
    assert abs(corr[0, 0, 0] - c0 * c1) <= 1e-12 * abs(c0 * c1)


def test_five_neutrons_three_source_factorisation():
    """Five neutrons on three sources, each source and its sink function on
    its own region of sites (Sec. 6): the correlator is the product of the
    oracle's one-source correlators of the regions (nn, nn, n).  Spin sets
    psi = chi = {0, 3, 1, 4, 2}, psi = 3 alpha + s."""
    V = 24
    region = np.arange(V) // 8
    S = host_props(23, 0, 1, 1, V, 3, np.complex128)[0, 0].copy()
    rng = np.random.default_rng(6)
    w = np.zeros((3, V), np.complex128)
    for s in range(3):
        S[region != s, s] = 0
        w[s, region == s] = rng.normal(size=8) + 1j * rng.normal(size=8)
    tl = _tl(False, 3, 0, 5, (0, 3, 1, 4, 2))
    k = np.array([1], np.int32)
    _, corr, ex = _run(tl, S[None], S[None], w, k, B.MB_FP64)
    assert ex[0] == 15
    nn = O.spin_state_request(0, 2, (0, 1))
    n1 = O.spin_state_request(0, 1, (0,))
    one = lambda s, req, key: O.correlators(False, 1, 0, len(O._bits(key)), req, S[:, s:s + 1], S[:, s:s + 1],
                                            w[s:s + 1], 2.0)[((0, key), (0, key))]
    ref = one(0, nn, 3) * one(1, nn, 3) * one(2, n1, 1)
    assert abs(ref) > 0
    assert abs(corr[0, 0, 0] - ref) <= 1e-12 * abs(ref)
    c32, sig = _mixed(tl, S[None], S[None], w, k)
    assert_close(c32, corr, 1e-6, "mixed vs fp64", sigma=sig)


# --------------------------------------------------------------------- mixed precision

MIXED_CASES = [
    (False, 1, 2, 2, (0, 1, 0, 1), 512, 64, np.complex128),    # 4He NR (C2 kind)
    (True, 1, 2, 2, None, 216, 64, np.complex64),               # 4He rel, all components (C3 kind)
    (False, 2, 4, 4, (0, 1, 2, 3, 0, 1, 2, 3), 512, 64, np.complex64),  # 8Be NR (C4 kind)
    (False, 3, 0, 5, (0, 3, 1, 4, 2), 64, 64, np.complex64),   # 5n, three sources
]


@pytest.mark.parametrize("rel,nsrc,nP,nN,spins,V,nl,dtype", MIXED_CASES)
def test_mixed_matches_fp64(rel, nsrc, nP, nN, spins, V, nl, dtype):
    Su, Sd, w, k = _inputs(9, nl, V, nsrc, dtype, True, with_sink=nsrc >= 2)
    tl = _tl(rel, nsrc, nP, nN, spins)
    _, c64, _ = _run(tl, Su, Sd, w, k, B.MB_FP64)
    c32, sig = _mixed(tl, Su, Sd, w, k)
    assert_close(c32, c64, 1e-6, "mixed vs fp64", sigma=sig)


@pytest.mark.parametrize("precision,tol", [(B.MB_FP64, 1e-12), (B.MB_MIXED, 1e-6)])
@pytest.mark.parametrize("rel,nsrc,nP,nN,spins,V,nl", [
    (True, 1, 2, 2, None, 27, 64),                       # n_xi = 12: two pair-row ranges
    (False, 2, 2, 2, (0, 2, 0, 2), 8, 70),               # two sources, ragged lanes
    (False, 1, 2, 1, None, 27, 33),                      # n_xi = 6: one pair-row range
    (False, 2, 4, 4, (0, 1, 2, 3, 0, 1, 2, 3), 8, 20),   # 8Be: every step kind
    (False, 3, 1, 2, (0, 1, 5), 8, 20),                  # three sources: six sink indices per species
])
def test_launch_tuning_keeps_results(precision, tol, rel, nsrc, nP, nN, spins, V, nl):
    """Every launch setting the autotuner may pick -- direct or LDS-staged
    kernel, passthrough group, lane tile, LDS cap -- gives the same
    correlators (up to summation order).  Steps with more than four sink
    indices per species have the direct kernel with one passthrough part
    per thread only; the library refuses the other settings there
    (MB_EUNSUPPORTED, before any launch)."""
    Su, Sd, w, k = _inputs(13, nl, V, nsrc, np.complex64, True, with_sink=nsrc >= 2)
    tl = _tl(rel, nsrc, nP, nN, spins)
    _, ref, _ = _run(tl, Su, Sd, w, k, B.MB_FP64)
    # with 2^k, k up to 3, an eight-baryon correlator reaches ~1e50: far beyond
    # float, which the per-lane block exponents keep out of the float stages
    assert np.all(np.isfinite(ref))
    nst = tl.counts()["n_stages"]
    for kern, pg, tile, lds, unroll, group, two in [
            (0, 1, 16, 0, 1, 1, 0), (0, 2, 64, 16384, 0, 1, 0), (0, 3, 16, 0, 2, 1, 0), (0, 3, 64, 0, 1, 1, 0),
            (0, 6, 64, 0, 2, 1, 0), (0, 6, 16, 0, 1, 1, 0), (0, 1, 64, 0, 2, 1, 0), (0, 1, 64, 0, 0, 2, 0),
            (0, 2, 64, 0, 0, 4, 0), (0, 3, 64, 0, 0, 4, 0), (1, 1, 16, 0, 0, 1, 0), (1, 2, 16, 0, 0, 1, 0),
            (1, 3, 16, 0, 0, 1, 0),
            # two-phase steps (partials per single index, then their sum)
            (0, 6, 64, 0, 2, 1, 1), (0, 3, 16, 0, 1, 1, 1), (0, 1, 64, 0, 1, 1, 1), (0, 2, 64, 0, 0, 1, 1),
            (0, 1, 16, 0, 2, 1, 1)]:
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
            tl.tune(s, B.MB_TUNE_LDS_BYTES, lds)
        try:
            if precision == B.MB_MIXED:
                got, sig = _mixed(tl, Su, Sd, w, k)
            else:
                _, got, _ = _run(tl, Su, Sd, w, k, precision)
                sig = None
        except B.MBError as e:
            if nsrc < 3 or e.code != B.MB_EUNSUPPORTED or (kern == 0 and group == 1 and pg == 1):
                raise
            continue
        assert_close(got, ref, tol, (kern, pg, tile, lds, unroll, group, two), sigma=sig)


@pytest.mark.parametrize("nl", [150, 500, 520])
def test_workgroup_mapping_covers_every_lane(nl):
    """Lane counts whose lane tiles number fewer than 8, a multiple of 8, or
    neither (the workgroup-to-XCD assignment of the recursion kernels has a
    case for each): every lane of one large batch equals the same lane run
    in batches of at most 64 lanes (one or four tiles), exactly, for every
    lane tile and output grouping; two lanes are also checked against the
    oracle."""
    rel, nsrc, nP, nN, spins, V = False, 1, 2, 2, (0, 1, 0, 1), 8
    Su, Sd, w, k = _inputs(17, nl, V, nsrc, np.complex128, True, with_sink=False)
    tl = _tl(rel, nsrc, nP, nN, spins)
    nst = tl.counts()["n_stages"]
    for tile, group in [(16, 1), (64, 1), (64, 2), (64, 4)]:
        for s in range(1, nst):
            tl.tune(s, B.MB_TUNE_KERNEL, 0)
            tl.tune(s, B.MB_TUNE_UNROLL, 0)
            tl.tune(s, B.MB_TUNE_GROUP, group)
            tl.tune(s, B.MB_TUNE_PASS_GROUP, 1)
            tl.tune(s, B.MB_TUNE_LANE_TILE, tile)
            tl.tune(s, B.MB_TUNE_LDS_BYTES, 0)
        _, full, _ = _run(tl, Su, Sd, w, k, B.MB_FP64)
        parts = []
        for i in range(0, nl, 64):
            su = Su[i:i + 64]   # one array for both flavours, as in the full batch
            parts.append(_run(tl, su, su, w, k[i:i + 64], B.MB_FP64)[1])
        chunked = np.concatenate(parts)
        assert np.array_equal(full, chunked), (tile, group, np.argwhere(full != chunked)[:4])
    for b in (0, nl - 1):
        ref = _oracle_corr(tl, rel, nsrc, nP, nN, Su[b], Sd[b], w, k[b])
        assert_close(full[b], ref, 1e-12, b)


# --------------------------------------------------------------------- projection (Sec. 5)

PROJ_CASES = [
    # rel, nsrc, nP, nN, V, lanes, weights
    (False, 1, 1, 1, 27, 3, "deuteron"),   # p+n, spin 1, m = 0
    (False, 1, 2, 1, 8, 2, "sparse"),      # 3He
    (True, 1, 1, 1, 8, 1, "sparse"),       # p+n relativistic
    (False, 2, 1, 1, 8, 2, "sparse"),      # p+n, two sources
    (False, 3, 1, 1, 8, 1, "sparse"),      # p+n, three sources
]


@pytest.mark.parametrize("rel,nsrc,nP,nN,V,nl,kind", PROJ_CASES)
def test_projected_correlator_matches_oracle(rel, nsrc, nP, nN, V, nl, kind):
    """The projected correlator C_M (one value per lane, eq. CM_final) equals
    sum W[delta][alpha] C(delta; alpha) with C from the oracle, and with C
    from the unprojected library path; the error bound is relative to
    sum |W| |C|, the size of the terms of the projection."""
    from tests.spin_weights import deuteron_weights, sparse_weights
    Su, Sd, w, k = _inputs(31 + nP + nN, nl, V, nsrc, np.complex128, True, with_sink=nsrc >= 2)
    full = B.TermList(nP, nN, rel, nsrc, all_components=True)
    cf = full.counts()
    W = (deuteron_weights(full) if kind == "deuteron"
         else sparse_weights((cf["n_delta"], cf["n_alpha"]), 3 * nP + nN + nsrc, 0.3))
    tl = B.TermList(nP, nN, rel, nsrc, all_components=True, proj=W)
    assert tl.counts()["projected"]
    _, cfull, _ = _run(full, Su, Sd, w, k, B.MB_FP64)
    refs = [_oracle_corr(full, rel, nsrc, nP, nN, Su[b], Sd[b], w, k[b]) for b in range(nl)]
    for prec, tol in [(B.MB_FP64, 1e-12), (B.MB_MIXED, 1e-6)]:
        _, cp, ex = _run(tl, Su, Sd, w, k, prec)
        assert cp.shape == (nl, 1, 1)
        assert np.array_equal(ex, 3 * (nP + nN) * k)
        for b in range(nl):
            R = refs[b]
            scale = (np.abs(W) * np.abs(R)).sum()
            assert scale > 0
            assert abs(cp[b, 0, 0] - (W * R).sum()) <= tol * scale, (prec, b)
            assert abs(cp[b, 0, 0] - (W * cfull[b]).sum()) <= tol * scale, (prec, b)


# --------------------------------------------------------------------- smaller nuclei on the path (Sec. 7)

SIDE_CASES = [
    # rel, nsrc, nP, nN, sides (stage, source sets), V, lanes
    (False, 1, 2, 1, [(0, None), (1, None)], 8, 2),   # 3He with p and pp
    (False, 1, 2, 2, [(2, None)], 8, 2),              # 4He NR with 3H
    (True, 1, 1, 1, [(0, None)], 8, 1),               # p+n relativistic with n
    (False, 2, 1, 1, [(0, None)], 8, 2),              # p+n, two sources, with n
]


@pytest.mark.parametrize("rel,nsrc,nP,nN,sides,V,nl", SIDE_CASES)
def test_side_nuclei_match_oracle(rel, nsrc, nP, nN, sides, V, nl):
    """Correlators of the smaller nuclei on the path, read from the shared
    stages, match the oracle's Wick contraction of each smaller nucleus; the
    main correlator matches the list without side nuclei."""
    Su, Sd, w, k = _inputs(41 + nP + nN, nl, V, nsrc, np.complex128, True, with_sink=nsrc >= 2)
    tl = B.TermList(nP, nN, rel, nsrc, all_components=True, sides=sides)
    main = B.TermList(nP, nN, rel, nsrc, all_components=True)
    c = tl.counts()
    _, cmain, _ = _run(main, Su, Sd, w, k, B.MB_FP64)
    tu = torch.from_numpy(np.ascontiguousarray(Su)).to(DEV)
    tw = None if w is None else torch.from_numpy(np.ascontiguousarray(w)).to(DEV)
    tk = torch.from_numpy(k).to(DEV)
    refs = []
    for i, (stage, _) in enumerate(sides):
        _, alphas, *_ = tl.side(i)
        kP = sum(1 for t in c["path"][:stage + 1] if t == 0)
        kN = stage + 1 - kP
        dsets = tl.export(B.MB_EXPORT_SPIN, stage).reshape(-1, 2)
        req = dict(sinkP=int(np.bitwise_or.reduce(dsets[:, 0])), sinkN=int(np.bitwise_or.reduce(dsets[:, 1])),
                   alphas=[tuple(map(int, a)) for a in alphas])
        per_lane = []
        for b in range(nl):
            ref = O.correlators(rel, nsrc, kP, kN, req, Su[b], Sd[b], w, 2.0 ** int(k[b]))
            per_lane.append(np.array([[ref[(tuple(map(int, d)), tuple(map(int, a)))] for a in alphas]
                                      for d in dsets]))
        refs.append(per_lane)
    for prec, tol in [(B.MB_FP64, 1e-12), (B.MB_MIXED, 1e-6)]:
        r = Runner(tl, tu, tu, prec, tw, tk, err_estimate=prec == B.MB_MIXED)
        corr, ex = r.run()
        torch.cuda.synchronize()
        assert np.array_equal(ex.cpu().numpy(), 3 * (nP + nN) * k)
        got_main = corr.cpu().numpy()
        sig_all = r.err_all[:, 0].cpu().numpy() if prec == B.MB_MIXED else None
        nmain = got_main.size
        assert_close(got_main, cmain, tol, (prec, "main"),
                     sigma=None if sig_all is None else sig_all[:nmain].reshape(got_main.shape))
        off = nmain
        for i in range(len(sides)):
            got = r.side_corr[i].cpu().numpy()
            sg = None if sig_all is None else sig_all[off:off + got.size].reshape(got.shape)
            off += got.size
            assert_close(got, np.array(refs[i]), tol, (prec, "side", i), sigma=sg)


# --------------------------------------------------------------------- recursion orders (Sec. 7)

@pytest.mark.parametrize("rel,nsrc,nP,nN,spins,order,V,nl", [
    (False, 1, 2, 1, None, 0b101, 8, 2),              # 3He as P N P
    (False, 1, 2, 2, (0, 1, 0, 1), 0b1010, 27, 2),    # 4He NR as N P N P
    (True, 1, 1, 2, (0, 0, 1), 0b010, 8, 1),          # 3H relativistic as N P N
    (False, 2, 2, 2, (0, 2, 0, 2), 0b0110, 8, 1),     # 4He NR, two sources, as N P P N
])
def test_interleaved_order_matches_oracle(rel, nsrc, nP, nN, spins, order, V, nl):
    """A recursion that alternates the species (every step kind reached from
    stages of mixed content) gives the oracle's correlators and those of the
    default order, in both precision modes."""
    Su, Sd, w, k = _inputs(51 + order, nl, V, nsrc, np.complex128, True, with_sink=nsrc >= 2)
    ref_tl = _tl(rel, nsrc, nP, nN, spins)
    if spins is None:
        tl = B.TermList(nP, nN, rel, nsrc, all_components=True, path=B.MB_PATH_EXPLICIT, order=order)
    else:
        tl = B.TermList.spin_state(nP, nN, rel, nsrc, spins, path=B.MB_PATH_EXPLICIT, order=order)
    assert tl.counts()["path"] == [0 if (order >> i) & 1 else 1 for i in range(nP + nN)]
    _, cref, _ = _run(ref_tl, Su, Sd, w, k, B.MB_FP64)
    for prec, tol in [(B.MB_FP64, 1e-12), (B.MB_MIXED, 1e-6)]:
        _, corr, ex = _run(tl, Su, Sd, w, k, prec)
        assert np.array_equal(ex, 3 * (nP + nN) * k)
        sig = _mixed(tl, Su, Sd, w, k)[1] if prec == B.MB_MIXED else None
        assert_close(corr, cref, tol, (prec, "default order"), sigma=sig)
        if prec == B.MB_FP64:
            for b in range(nl):
                ref = _oracle_corr(tl, rel, nsrc, nP, nN, Su[b], Sd[b], w, k[b])
                assert_close(corr[b], ref, 1e-12, b)


# --------------------------------------------------------------------- saved term lists

def test_loaded_term_list_contracts_identically(tmp_path):
    """A term list written to a file and read back gives bit-identical
    correlators to the one built in memory, in both precision modes."""
    Su, Sd, w, k = _inputs(61, 3, 8, 1, np.complex128, True, with_sink=False)
    tl = B.TermList(2, 1, False, 1, all_components=True, sides=[(1, None)])
    f = tmp_path / "list.mbt"
    tl.save(f)
    back = B.TermList.load(f)
    for prec in (B.MB_FP64, B.MB_MIXED):
        _, a, ea = _run(tl, Su, Sd, w, k, prec)
        _, b, eb = _run(back, Su, Sd, w, k, prec)
        assert np.array_equal(a, b) and np.array_equal(ea, eb), prec


# --------------------------------------------------------------------- paired stage layout

@pytest.mark.parametrize("rel,nsrc,nP,nN,spins,V,nl", [
    (True, 1, 2, 2, None, 8, 70),                          # 4He relativistic: pairs of passthrough parts
    (False, 2, 2, 2, (0, 2, 0, 2), 8, 64),                # pairs of input sets (neutron steps, one passthrough)
    (False, 2, 4, 4, (0, 1, 2, 3, 0, 1, 2, 3), 8, 66),    # 8Be: every step kind
])
def test_paired_stage_layout_is_bit_identical(rel, nsrc, nP, nN, spins, V, nl):
    """Float stages stored with neighbouring spin parts paired per lane (read
    with one 16-byte load by the direct kernel with 64-lane tiles or the
    grouped kernel) give exactly the correlators of the plain layout with
    the same kernels: every output keeps its sum order."""
    Su, Sd, w, k = _inputs(71, nl, V, nsrc, np.complex64, True, with_sink=nsrc >= 2)
    tl = _tl(rel, nsrc, nP, nN, spins)
    nst = tl.counts()["n_stages"]
    _, ref, _ = _run(tl, Su, Sd, w, k, B.MB_FP64)
    # (pass group, outputs per wave, two-phase), 64-lane tiles
    for pg, group, two in [(3, 1, 0), (2, 1, 0), (6, 1, 0), (1, 1, 0), (1, 2, 0), (1, 4, 0), (6, 1, 1), (1, 1, 1)]:
        res = []
        for paired in (0, 1):
            for s in range(1, nst):
                tl.tune(s, B.MB_TUNE_KERNEL, 0)
                tl.tune(s, B.MB_TUNE_GROUP, group)
                tl.tune(s, B.MB_TUNE_TWO_PHASE, two)
                tl.tune(s, B.MB_TUNE_LANE_TILE, 64)
                tl.tune(s, B.MB_TUNE_LDS_BYTES, 0)
                tl.tune(s, B.MB_TUNE_UNROLL, 0)
                tl.tune(s, B.MB_TUNE_PAIRED, paired)
                try:
                    tl.tune(s, B.MB_TUNE_PASS_GROUP, pg)
                except B.MBError:
                    tl.tune(s, B.MB_TUNE_PASS_GROUP, 1)
            got, sig = _mixed(tl, Su, Sd, w, k)
            res.append(got)
        assert np.array_equal(res[0], res[1]), (pg, group, two)
        assert_close(res[1], ref, 1e-6, (pg, group, two), sigma=sig)


# --------------------------------------------------------------------- error estimates (err_out)

@pytest.mark.parametrize("two_phase", [0, 1])
@pytest.mark.parametrize("rel,nsrc,nP,nN,spins,V,nl,dtype", MIXED_CASES)
def test_error_estimate_covers_the_mixed_deviation(rel, nsrc, nP, nN, spins, V, nl, dtype, two_phase):
    """err_out of the mixed path against the measured deviation of the mixed
    correlators from the FP64 ones (eq. C_final outputs): every component
    lies within its first-order bound and within 6 estimated standard
    deviations; per lane, the estimated deviation (norm over the lane's
    components) is neither below a sixth nor above 100 times the measured
    one.  The FP64 path reports zeros."""
    Su, Sd, w, k = _inputs(9, nl, V, nsrc, dtype, True, with_sink=nsrc >= 2)
    tl = _tl(rel, nsrc, nP, nN, spins)
    for s in range(1, tl.counts()["n_stages"]):
        tl.tune(s, B.MB_TUNE_TWO_PHASE, two_phase)   # partials rounded to float too
    tu = torch.from_numpy(np.ascontiguousarray(Su)).to(DEV)
    tw = None if w is None else torch.from_numpy(np.ascontiguousarray(w)).to(DEV)
    tk = torch.from_numpy(k).to(DEV)
    out = {}
    for prec in (B.MB_FP64, B.MB_MIXED):
        r = Runner(tl, tu, tu, prec, tw, tk, err_estimate=True)
        r.err_all.fill_(float("nan"))
        corr, _ = r.run()
        torch.cuda.synchronize()
        out[prec] = (corr.cpu().numpy(), r.err.cpu().numpy())
    c64, e64 = out[B.MB_FP64]
    c32, e32 = out[B.MB_MIXED]
    assert np.all(e64 == 0)
    # the correlators are those of the run without error estimates
    _, plain, _ = _run(tl, Su, Sd, w, k, B.MB_MIXED)
    assert np.array_equal(plain, c32)
    d = np.abs(c32 - c64)
    sigma, bound = e32[..., 0], e32[..., 1]
    assert np.all(np.isfinite(sigma)) and np.all(np.isfinite(bound))
    assert np.all(d <= bound), float((d / bound).max())
    assert np.all(d <= 6 * sigma), float((d / sigma).max())
    nd = np.sqrt((d ** 2).reshape(nl, -1).sum(1))
    ns = np.sqrt((sigma ** 2).reshape(nl, -1).sum(1))
    ratio = ns / nd
    print(f"sigma/deviation per lane: min {ratio.min():.3g} median {np.median(ratio):.3g} max {ratio.max():.3g}; "
          f"bound/deviation max {(bound / np.maximum(d, 1e-300)).max():.3g}")
    assert ratio.min() >= 1 / 6 and ratio.max() <= 100, (ratio.min(), ratio.max())


def test_error_estimate_of_projected_and_side_outputs():
    """Projected lists (one output per lane, the estimates summed over the
    sink sets) and side nuclei (their own final sums) get estimates too."""
    Su, Sd, w, k = _inputs(91, 3, 27, 1, np.complex64, True, with_sink=False)
    from tests.spin_weights import sparse_weights
    full = B.TermList(2, 1, False, 1, all_components=True)
    cf = full.counts()
    W = sparse_weights((cf["n_delta"], cf["n_alpha"]), 7, 0.3)
    for tl in (B.TermList(2, 1, False, 1, all_components=True, proj=W),
               B.TermList(2, 1, False, 1, all_components=True, sides=[(0, None), (1, None)])):
        tu = torch.from_numpy(np.ascontiguousarray(Su)).to(DEV)
        tk = torch.from_numpy(k).to(DEV)
        res = {}
        for prec in (B.MB_FP64, B.MB_MIXED):
            r = Runner(tl, tu, tu, prec, None, tk, err_estimate=True)
            r.run()
            torch.cuda.synchronize()
            res[prec] = (r.out.cpu().numpy(), r.err_all.cpu().numpy())
        d = np.abs(res[B.MB_MIXED][0] - res[B.MB_FP64][0])
        sigma, bound = res[B.MB_MIXED][1][:, 0], res[B.MB_MIXED][1][:, 1]
        assert np.all(res[B.MB_FP64][1] == 0)
        assert np.all(d <= bound) and np.all(d <= 6 * sigma)
        assert (sigma > 0).mean() > 0.5
