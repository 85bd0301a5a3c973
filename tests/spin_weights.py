"""Real weights of spin projections (Sec. 5) for the tests: over the sink
sets (rows) and source sets (columns) a term list exports."""
import math

import numpy as np

from paper_1301_4895_amd import binding as B


def sparse_weights(shape, seed, density=0.2):
    """Real weights with many zeros; every value is a multiple of 1/4, so
    that sums of integer coefficients times weights are exact in any order."""
    rng = np.random.default_rng(seed)
    w = rng.choice([-2.0, -1.0, -0.5, 0.25, 0.5, 1.0, 1.5], size=shape)
    w[rng.random(shape) >= density] = 0.0
    w.flat[rng.integers(w.size)] = 1.0   # at least one nonzero weight
    return w


def deuteron_weights(tl):
    """Spin-1, m = 0 projection of p+n with nonrelativistic operators, one
    source: (|up down> + |down up>) / sqrt(2) at the sink and the source;
    the weights are products of the two amplitudes (1/2 each)."""
    def amp(sets):
        v = np.zeros(len(sets))
        for i, (p, n) in enumerate(sets):
            if (int(p), int(n)) in ((1, 2), (2, 1)):
                v[i] = math.sqrt(0.5)
        return v
    d = amp(tl.export(B.MB_EXPORT_DELTA).reshape(-1, 2))
    a = amp(tl.export(B.MB_EXPORT_ALPHA).reshape(-1, 2))
    return np.outer(d, a)
