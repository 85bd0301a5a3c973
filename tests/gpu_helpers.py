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
