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
    e = r.blocks[n:n + 4 * Bp].view(torch.int32)
    return blk, e


def check_lane_exponent(blk_lane, e):
    """The stored blocks of a lane have their largest |Re|, |Im| in [1/2, 1)."""
    m = max(np.abs(blk_lane.real).max(), np.abs(blk_lane.imag).max())
    assert (m == 0 and e == 0) or 0.5 <= m < 1.0, (m, e)
