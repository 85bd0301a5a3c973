"""Helpers shared by the GPU tests: inputs, oracle blocks in library layout."""
import numpy as np

from oracle import oracle as O
from synth import props as SP


def pairs(n):
    return [(a, b) for b in range(n) for a in range(b)]


def oracle_blocks_lib_layout(fP, fN):
    """Oracle blocks antisymmetrised and laid out like the library:
    [species][psi][block quark index]."""
    npsi, nxi = fP.shape[0], fP.shape[1]
    pr = pairs(nxi)
    npair = len(pr)
    out = np.zeros((2, npsi, npair * nxi), np.complex128)
    for i, (a, b) in enumerate(pr):
        for c in range(nxi):
            out[0, :, i * nxi + c] = fP[:, a, b, c] - fP[:, b, a, c]
            out[1, :, c * npair + i] = fN[:, a, c, b] - fN[:, b, c, a]
    return out


def host_props(seed, stream, nprob, T, V, nsrc, dtype, probs=None, ts=None):
    return SP.props(seed, stream, nprob, T, V, nsrc, 0.5, dtype, probs, ts)


def rel_err(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


SIGNIFICANT = 1e-3   # components at least this fraction of the largest are compared relatively


NSIGMA = 6.0        # a mixed-path component may also lie within this many estimated standard deviations


def component_err(got, ref, sigma=None, significant=SIGNIFICANT):
    """Element-wise error of one lane's correlators (any shape): the largest
    |got - ref| / |ref| over the components with |ref| >= SIGNIFICANT * max
    |ref|, and the largest |got - ref| / max |ref| over the others (exact
    zeros included).  With sigma (the library's estimated standard deviation
    of each component's float-storage rounding error), components with
    |got - ref| <= NSIGMA * sigma count as exact."""
    got, ref = np.ravel(got), np.ravel(ref)
    scale = np.abs(ref).max()
    d = np.abs(got - ref)
    if sigma is not None:
        d = np.where(d <= NSIGMA * np.ravel(sigma), 0.0, d)
    if scale == 0:
        return 0.0, float(d.max())
    big = np.abs(ref) >= significant * scale
    rel = float((d[big] / np.abs(ref[big])).max())
    small = float(d[~big].max() / scale) if (~big).any() else 0.0
    return rel, small


def assert_close(got, ref, tol, what="", sigma=None, significant=SIGNIFICANT):
    """Parity of correlators, lane by lane (leading axis): the relative
    Frobenius norm over a lane's components is at most tol, every component
    with |ref| >= SIGNIFICANT * max |ref| of its lane is within tol |ref|,
    and every other component (exact zeros included) within tol * max |ref|.

    sigma (mixed path against FP64 or the oracle): the standard deviations
    the library estimates for the rounding error of each component (err_out
    [..., 0] of mb_contract_correlator).  A component then also passes when
    it lies within NSIGMA of them: float storage of the stages gives a
    component that is small through cancellation an error of order
    2^-24 times the size of its terms, which a relative bound of 1e-6 on
    the component cannot hold.  The norm bound likewise also passes when
    the lane's deviation is within NSIGMA of the root sum of squares of its
    sigmas (a lane whose few components all cancel, e.g. a single spin
    component).
    significant: the fraction of the lane's largest component from which the
    relative bound applies (default SIGNIFICANT).
    Returns the worst (norm, significant, small) errors."""
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape, what)
    if sigma is not None:
        sigma = np.asarray(sigma)
        assert sigma.shape == ref.shape, (sigma.shape, ref.shape, what)
    if got.ndim <= 2:
        got, ref = got[None], ref[None]
        sigma = None if sigma is None else sigma[None]
    worst = [0.0, 0.0, 0.0]
    for b in range(len(ref)):
        assert np.abs(ref[b]).max() > 0, (what, b, "all-zero reference")
        n = rel_err(got[b], ref[b])
        if sigma is not None and np.linalg.norm(np.ravel(got[b] - ref[b])) <= NSIGMA * np.linalg.norm(sigma[b]):
            n = 0.0
        rel, small = component_err(got[b], ref[b], None if sigma is None else sigma[b], significant)
        assert n <= tol and rel <= tol and small <= tol, (what, b, n, rel, small, tol)
        worst = [max(worst[0], n), max(worst[1], rel), max(worst[2], small)]
    return tuple(worst)


def lib_blocks(r, tl):
    """The library's blocks of a Runner as [species][psi][block quark index]
    [lane] (complex, as stored) and the per-lane exponents e (stored blocks =
    blocks * 2^-e)."""
    import torch
    c = tl.counts()
    nxi, npsi = c["n_xi"], c["n_psi"]
    nyq = nxi * (nxi - 1) // 2 * nxi
    Bp = (r.batch + 63) // 64 * 64
    n = 2 * nyq * npsi * Bp * 16
    blk = (r.blocks[:n].view(torch.complex128).view(2, nyq, Bp // 16, npsi, 16).permute(0, 3, 1, 2, 4)
           .reshape(2, npsi, nyq, Bp))
    nl = nxi ** 3 * npsi * Bp * 16 if c.get("n_Lambda") else 0
    e = r.blocks[n + nl:n + nl + 4 * Bp].view(torch.int32)
    return blk, e


def lib_lambda_block(r, tl):
    """The Lambda block of a Runner as [psi][block quark index][lane]."""
    import torch
    c = tl.counts()
    nxi, npsi = c["n_xi"], c["n_psi"]
    nyq = nxi * (nxi - 1) // 2 * nxi
    Bp = (r.batch + 63) // 64 * 64
    n = 2 * nyq * npsi * Bp * 16
    nyl = nxi ** 3
    return (r.blocks[n:n + nyl * npsi * Bp * 16].view(torch.complex128).view(nyl, Bp // 16, npsi, 16)
            .permute(2, 0, 1, 3).reshape(npsi, nyl, Bp))


def check_lane_exponent(blk_lane, e):
    """The stored blocks of a lane have their largest |Re|, |Im| in [1/2, 1)."""
    m = max(np.abs(blk_lane.real).max(), np.abs(blk_lane.imag).max())
    assert (m == 0 and e == 0) or 0.5 <= m < 1.0, (m, e)
