"""Reference (oracle) for the recursive multibaryon correlator method.

Guenther, Toth, Varnhorst, "A recursive approach to determine correlation
functions in multibaryon systems", arXiv:1301.4895.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of the benchmark are the only users.  The heavy loops live in
``oracle.c`` (plain C99, double precision); this module marshals arguments and
composes them into the quantities the paper defines.  Nothing here imports the
HIP package, and the HIP package never imports this.

Conventions (the paper leaves them open; see the readings in the design notes):
  * quark index xi = N_s*(3*spin + colour) + source, baryon index
    psi/chi = N_s*alpha + source (sink function at the sink);
  * nonrelativistic operators keep spins 0, 1 only (Dirac representation,
    Sec. 7), so quark indices run over 3*D*N_s values and baryon indices over
    D*N_s values, with D = 4 (relativistic) or 2;
  * baryon order inside a correlator: protons, then neutrons, then the
    Lambda, each group in ascending spin index; the same order at sink and
    source;
  * the Lambda operator is the baryon form of Sec. 1 (eq. C_baryons) with
    (q1, q2, q3) = (s, u, d) and the nucleons' Gamma_1, Gamma_2;
  * propagators S[x][s][row][kappa] complex128, row the sink spin-colour,
    kappa the source spin-colour of source s.
"""
from __future__ import annotations

import ctypes as C
import itertools
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_lib = None

PROTON, NEUTRON, LAMBDA = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c into liborc.so with the system C compiler."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = C.CDLL(_SO)
        _lib.orc_bound_P.restype = C.c_ulonglong
        _lib.orc_bound_Q.restype = C.c_ulonglong
        _lib.orc_L_uca.restype = C.c_long
        _lib.orc_req_stage.restype = C.c_long
        _lib.orc_lambda_stage.restype = C.c_long
    return _lib


def set_threads(n: int):
    """Threads for the oracle's parallel loops (each output is one thread's
    sum, so results do not depend on the count)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _ints(seq):
    return np.ascontiguousarray(np.asarray(seq, dtype=np.int32))


# --------------------------------------------------------------------------
# Dirac algebra and G tensors (Sec. 2 eq. def_g, Sec. 6 eq. G_tilde, Sec. 7)

def dirac():
    """gamma^0..gamma^3, gamma_5, C as a (6,4,4) complex array."""
    out = np.zeros((6, 4, 4), np.complex128)
    lib().orc_dirac(_p(out))
    return out


def gamma(rel: bool):
    """(Gamma_1, Gamma_2) of the relativistic or nonrelativistic nucleon."""
    g1 = np.zeros((4, 4), np.complex128)
    g2 = np.zeros((4, 4), np.complex128)
    lib().orc_gamma(int(rel), _p(g1), _p(g2))
    return g1, g2


def g_nonzero(rel: bool, nsrc: int, chi: int):
    """Nonzero entries of G-tilde(chi; xi1, xi2, xi3): (xi[n,3], value[n])."""
    cap = (12 * nsrc) ** 3
    xi = np.zeros((cap, 3), np.int32)
    val = np.zeros(cap, np.complex128)
    n = lib().orc_g_nonzero(int(rel), nsrc, chi, _p(xi), _p(val), cap)
    return xi[:n].copy(), val[:n].copy()


# --------------------------------------------------------------------------
# Blocks (Sec. 2, Sec. 6)

def blocks(rel, nsrc, Su, Sd, sinkw=None, scale=1.0, D=None):
    """Full proton and neutron blocks f[psi][xi1][xi2][xi3] (Sec. 2).

    Su, Sd: complex128 [V][nsrc][12][12]; sinkw: complex128 [nsrc][V] or None
    (zero momentum, s(x) = 1); scale multiplies every propagator entry.
    Returns (fP, fN) of shape (D*nsrc, 3*D*nsrc, 3*D*nsrc, 3*D*nsrc).
    """
    D = D or (4 if rel else 2)
    Su = np.ascontiguousarray(Su, np.complex128)
    Sd = np.ascontiguousarray(Sd, np.complex128)
    V = Su.shape[0]
    assert Su.shape == (V, nsrc, 12, 12) and Sd.shape == Su.shape
    npsi, nxi = D * nsrc, 3 * D * nsrc
    fP = np.zeros((npsi, nxi, nxi, nxi), np.complex128)
    fN = np.zeros_like(fP)
    if sinkw is not None:
        sinkw = np.ascontiguousarray(sinkw, np.complex128)
        assert sinkw.shape == (nsrc, V)
    lib().orc_blocks(int(rel), nsrc, npsi, nxi, V, _p(Su), _p(Sd),
                     _p(sinkw) if sinkw is not None else None,
                     C.c_double(scale), _p(fP), _p(fN))
    return fP, fN


def blocks_lambda(rel, nsrc, Su, Sd, Ss, sinkw=None, scale=1.0, D=None):
    """Full Lambda block fL[psi][xi_s][xi_u][xi_d]: the baryon form of
    Sec. 1 with (q1, q2, q3) = (s, u, d), same conventions as blocks()."""
    D = D or (4 if rel else 2)
    Su, Sd, Ss = (np.ascontiguousarray(S, np.complex128) for S in (Su, Sd, Ss))
    V = Su.shape[0]
    assert Su.shape == (V, nsrc, 12, 12) and Sd.shape == Su.shape and Ss.shape == Su.shape
    npsi, nxi = D * nsrc, 3 * D * nsrc
    fL = np.zeros((npsi, nxi, nxi, nxi), np.complex128)
    if sinkw is not None:
        sinkw = np.ascontiguousarray(sinkw, np.complex128)
        assert sinkw.shape == (nsrc, V)
    lib().orc_blocks_lambda(int(rel), nsrc, npsi, nxi, V, _p(Su), _p(Sd), _p(Ss),
                            _p(sinkw) if sinkw is not None else None, C.c_double(scale), _p(fL))
    return fL


def antisym_blocks(fP, fN):
    """Antisymmetrised blocks (Sec. 4: all permutations of the same-flavour
    slots, without normalisation) as dictionaries keyed by
    (psi, u-mask, d-mask)."""
    npsi, nxi = fP.shape[0], fP.shape[1]
    outP, outN = {}, {}
    for psi in range(npsi):
        for a in range(nxi):
            for b in range(a + 1, nxi):
                for c in range(nxi):
                    # proton: u slots 1, 2
                    outP[(psi, (1 << a) | (1 << b), 1 << c)] = fP[psi, a, b, c] - fP[psi, b, a, c]
                    # neutron: d slots 1, 3
                    outN[(psi, 1 << c, (1 << a) | (1 << b))] = fN[psi, a, c, b] - fN[psi, b, c, a]
    return outP, outN


# --------------------------------------------------------------------------
# The tensor L (Sec. 2 eq. tensor_L)

def L_uca(rel, nsrc, types, chis, with_s=False):
    """L(alpha; z) on sorted index sets, by explicit permutations (Sec. 2).

    types/chis: per baryon in order (LAMBDA for a Lambda).  Returns (umask,
    dmask, coef) arrays of the nonzero entries, or (umask, dmask, smask,
    coef) with with_s, ascending in (umask, dmask, smask)."""
    t, c = _ints(types), _ints(chis)
    nb = len(t)
    cap = 1 << 22
    um = np.zeros(cap, np.uint32)
    dm = np.zeros(cap, np.uint32)
    sm = np.zeros(cap, np.uint32)
    cf = np.zeros(cap, np.int64)
    n = lib().orc_L_uca(int(rel), nsrc, nb, _p(t), _p(c), _p(um), _p(dm), _p(sm), _p(cf), C.c_long(cap))
    assert n <= cap
    if with_s:
        return um[:n].copy(), dm[:n].copy(), sm[:n].copy(), cf[:n].copy()
    assert not sm[:n].any()
    return um[:n].copy(), dm[:n].copy(), cf[:n].copy()


# --------------------------------------------------------------------------
# Correlator (Sec. 2 eq. f_L_contr) and independent closed forms

def corr_from_L(types, psis, fP, fN, um, dm, coef, fL=None, sm=None):
    """C = sum_z L(alpha; z) W(delta; z) with the permutation sum W (fL and
    the s masks sm for a system with a Lambda)."""
    t, ps = _ints(types), _ints(psis)
    out = np.zeros(1, np.complex128)
    um = np.ascontiguousarray(um, np.uint32)
    dm = np.ascontiguousarray(dm, np.uint32)
    coef = np.ascontiguousarray(coef, np.int64)
    fP = np.ascontiguousarray(fP)
    fN = np.ascontiguousarray(fN)
    assert (LAMBDA in list(t)) == (fL is not None)
    fL = None if fL is None else np.ascontiguousarray(fL)
    sm = None if sm is None else np.ascontiguousarray(sm, np.uint32)
    lib().orc_corr(len(t), _p(t), _p(ps), fP.shape[0], fP.shape[1], _p(fP), _p(fN),
                   _p(fL) if fL is not None else None, C.c_long(len(um)), _p(um), _p(dm),
                   _p(sm) if sm is not None else None, _p(coef), _p(out))
    return complex(out[0])


def proton_closed(rel, Su, Sd, sinkw=None, scale=1.0, delta=0, alpha=0):
    """Single proton two-point function by direct Wick contraction."""
    Su = np.ascontiguousarray(Su, np.complex128)
    Sd = np.ascontiguousarray(Sd, np.complex128)
    V = Su.shape[0]
    assert Su.shape[1] == 1
    out = np.zeros(1, np.complex128)
    w = None if sinkw is None else np.ascontiguousarray(sinkw, np.complex128).reshape(-1)
    lib().orc_proton_closed(int(rel), V, _p(Su), _p(Sd), _p(w) if w is not None else None,
                            C.c_double(scale), delta, alpha, _p(out))
    return complex(out[0])


def wick_literal(rel, nsrc, types, psis, chis, Su, Sd, sinkw=None, scale=1.0, Ss=None):
    """Literal Wick contraction of <prod B prod Bbar> (tiny systems only);
    Ss is the strange propagator of a system with a Lambda."""
    Su = np.ascontiguousarray(Su, np.complex128)
    Sd = np.ascontiguousarray(Sd, np.complex128)
    Ss = None if Ss is None else np.ascontiguousarray(Ss, np.complex128)
    V = Su.shape[0]
    t, ps, ch = _ints(types), _ints(psis), _ints(chis)
    assert (LAMBDA in list(t)) == (Ss is not None)
    out = np.zeros(1, np.complex128)
    w = None if sinkw is None else np.ascontiguousarray(sinkw, np.complex128)
    lib().orc_wick_literal(int(rel), nsrc, len(t), _p(t), _p(ps), _p(ch), V, _p(Su), _p(Sd),
                           _p(Ss) if Ss is not None else None, _p(w) if w is not None else None,
                           C.c_double(scale), _p(out))
    return complex(out[0])


def lambda_closed(rel, Su, Sd, Ss, sinkw=None, scale=1.0, delta=0, alpha=0):
    """Single Lambda two-point function by direct Wick contraction (the s,
    u and d quarks each meet their own source quark: one term)."""
    Su, Sd, Ss = (np.ascontiguousarray(S, np.complex128) for S in (Su, Sd, Ss))
    V = Su.shape[0]
    assert Su.shape[1] == 1
    out = np.zeros(1, np.complex128)
    w = None if sinkw is None else np.ascontiguousarray(sinkw, np.complex128).reshape(-1)
    lib().orc_lambda_closed(int(rel), V, _p(Su), _p(Sd), _p(Ss), _p(w) if w is not None else None,
                            C.c_double(scale), delta, alpha, _p(out))
    return complex(out[0])


# --------------------------------------------------------------------------
# Required components and operation lists (Sec. 3, 4, 5)

def req_stage(final, shape):
    """All components of `shape` = (kP, kN, ku, kd) that are sub-tuples of a
    final component (rows of four masks).  Sorted unique (m, 4) uint32."""
    fin = np.ascontiguousarray(final, np.uint32).reshape(-1, 4)
    n = lib().orc_req_stage(C.c_long(len(fin)), _p(fin), *[int(s) for s in shape], None, C.c_long(0))
    out = np.zeros((max(n, 1), 4), np.uint32)
    lib().orc_req_stage(C.c_long(len(fin)), _p(fin), *[int(s) for s in shape], _p(out), C.c_long(n))
    return out[:n]


def lambda_stage(zs, added, xs, rows=False):
    """Operation list of one recursion step (eq. recr_F): every split of
    every required output into (x, y).  Returns the count, or with
    rows=True an int64 (n, 6) array (z index, x index, y spin mask, y u
    mask, y d mask, sign)."""
    zs = np.ascontiguousarray(zs, np.uint32).reshape(-1, 4)
    xs = np.ascontiguousarray(xs, np.uint32).reshape(-1, 4)
    n = lib().orc_lambda_stage(C.c_long(len(zs)), _p(zs), int(added), C.c_long(len(xs)), _p(xs),
                               None, C.c_long(0))
    if n < 0:
        raise ValueError("an operand is missing from the previous stage")
    if not rows:
        return n
    out = np.zeros((max(n, 1), 6), np.int64)
    lib().orc_lambda_stage(C.c_long(len(zs)), _p(zs), int(added), C.c_long(len(xs)), _p(xs),
                           _p(out), C.c_long(n))
    return out[:n]


def bound_P(D, nsrc, nP, nN):
    return int(lib().orc_bound_P(D, nsrc, nP, nN))


def bound_Q(D, nsrc, added, nP, nN):
    return int(lib().orc_bound_Q(D, nsrc, int(added), nP, nN))


# --------------------------------------------------------------------------
# Composition: nucleus, path, spin requests

def path(nP, nN):
    """Order in which baryons are added: all baryons of the more numerous
    species first (Sec. 7); on a tie, neutrons first."""
    first = NEUTRON if nN >= nP else PROTON
    second = PROTON if first == NEUTRON else NEUTRON
    nf = nN if first == NEUTRON else nP
    ns = nP if first == NEUTRON else nN
    return [first] * nf + [second] * ns


def _mask(idx):
    m = 0
    for i in idx:
        m |= 1 << i
    return m


def _bits(m):
    return [i for i in range(32) if m >> i & 1]


def all_components_request(nP, nN, D, nsrc):
    """'All independent spinor components' (Tables 1-3): every sink set over
    the D*N_s baryon indices; at the source, with one source every set, with
    several sources the sets that put min(n, D) baryons of a species on
    source 0 (any spins), min(rest, D) on source 1, and so on."""
    nb = D * nsrc
    sinkP = (1 << nb) - 1
    sinkN = (1 << nb) - 1

    def src_sets(n):
        if nsrc == 1:
            return [_mask(c) for c in itertools.combinations(range(nb), n)]
        counts, left = [], n
        for s in range(nsrc):
            counts.append(min(left, D))
            left -= counts[-1]
        per_source = [itertools.combinations([nsrc * a + s for a in range(D)], counts[s]) for s in range(nsrc)]
        return sorted(_mask(sum(cs, ())) for cs in itertools.product(*[list(p) for p in per_source]))

    alphas = [(p, n) for p in src_sets(nP) for n in src_sets(nN)]
    return dict(sinkP=sinkP, sinkN=sinkN, alphas=alphas)


def spin_state_request(nP, nN, spins):
    """Single spin component (Sec. 8): the listed indices, protons first,
    used both at the sink and at the source."""
    pm = _mask(spins[:nP])
    nm = _mask(spins[nP:nP + nN])
    assert bin(pm).count("1") == nP and bin(nm).count("1") == nN
    return dict(sinkP=pm, sinkN=nm, alphas=[(pm, nm)])


def delta_sets(nP, nN, req):
    """Sink index sets of the request: every nP-subset of the sink proton
    base set times every nN-subset of the neutron base set."""
    ps = [_mask(c) for c in itertools.combinations(_bits(req["sinkP"]), nP)]
    ns = [_mask(c) for c in itertools.combinations(_bits(req["sinkN"]), nN)]
    return [(p, n) for p in ps for n in ns]


def L_for_alpha(rel, nsrc, nP, nN, alpha):
    """L(alpha; z) for an alpha set (protons first, ascending)."""
    types = [PROTON] * nP + [NEUTRON] * nN
    chis = _bits(alpha[0]) + _bits(alpha[1])
    return L_uca(rel, nsrc, types, chis)


def term_list(rel, nsrc, nP, nN, req, with_ops=False):
    """Everything the recursion needs, from the definitions: L per alpha set,
    the final required set, the required sets at every stage (sub-tuples)
    and the operation counts (or lists) of every step."""
    D = 4 if rel else 2
    Ls = {}
    U = set()
    for a in req["alphas"]:
        um, dm, cf = L_for_alpha(rel, nsrc, nP, nN, a)
        Ls[a] = {(int(u), int(d)): int(c) for u, d, c in zip(um, dm, cf)}
        U.update(Ls[a].keys())
    U = sorted(U)
    dsets = delta_sets(nP, nN, req)
    final = np.array([(p, n, u, d) for (p, n) in dsets for (u, d) in U], np.uint32).reshape(-1, 4)
    final = final[np.lexsort(final.T[::-1])]
    seq = path(nP, nN)
    shapes = []
    kp = kn = 0
    for t in seq:
        if t == PROTON:
            kp += 1
        else:
            kn += 1
        shapes.append((kp, kn, 2 * kp + kn, kp + 2 * kn))
    reqs = []
    for i, sh in enumerate(shapes):
        reqs.append(final if i == len(shapes) - 1 else req_stage(final, sh))
    ops = []
    for i in range(1, len(seq)):
        ops.append(lambda_stage(reqs[i], seq[i], reqs[i - 1], rows=with_ops))
    n_ops = sum(len(o) if with_ops else o for o in ops)
    return dict(L=Ls, U=U, dsets=dsets, path=seq, shapes=shapes, req=reqs,
                ops=ops, n_lambda=int(n_ops), D=D)


def correlators(rel, nsrc, nP, nN, req, Su, Sd, sinkw=None, scale=1.0, tl=None):
    """C[delta set, alpha set] for one timeslice by eq. f_L_contr, with the
    blocks by their definition.  Returns a dict keyed by (delta, alpha)."""
    D = 4 if rel else 2
    fP, fN = blocks(rel, nsrc, Su, Sd, sinkw, scale, D=D)
    types = [PROTON] * nP + [NEUTRON] * nN
    out = {}
    for a in req["alphas"]:
        if tl is not None:
            L = tl["L"][a]
            um = np.array([k[0] for k in L], np.uint32)
            dm = np.array([k[1] for k in L], np.uint32)
            cf = np.array([L[k] for k in L], np.int64)
        else:
            um, dm, cf = L_for_alpha(rel, nsrc, nP, nN, a)
        for d in delta_sets(nP, nN, req):
            psis = _bits(d[0]) + _bits(d[1])
            out[(d, a)] = corr_from_L(types, psis, fP, fN, um, dm, cf)
    return out


# --------------------------------------------------------------------------
# Systems with one Lambda (the baryon form of Sec. 1 with (s, u, d) slots),
# added after the nucleons: the generalisation of Sec. 3-4 to a third quark
# flavour and a third baryon species.

def _src_sets(n, D, nsrc):
    """The source sets of all_components_request for n baryons of one
    species."""
    nb = D * nsrc
    if nsrc == 1:
        return [_mask(c) for c in itertools.combinations(range(nb), n)]
    counts, left = [], n
    for s in range(nsrc):
        counts.append(min(left, D))
        left -= counts[-1]
    per_source = [itertools.combinations([nsrc * a + s for a in range(D)], counts[s]) for s in range(nsrc)]
    return sorted(_mask(sum(cs, ())) for cs in itertools.product(*[list(p) for p in per_source]))


def hyperon_request_all(nP, nN, D, nsrc):
    """All components of a system of nP protons, nN neutrons and one Lambda:
    every sink set, and the source sets of all_components_request per
    species (the Lambda on source 0)."""
    full = (1 << (D * nsrc)) - 1
    alphas = [(p, n, l) for p in _src_sets(nP, D, nsrc) for n in _src_sets(nN, D, nsrc)
              for l in _src_sets(1, D, nsrc)]
    return dict(sinkP=full if nP else 0, sinkN=full if nN else 0, sinkL=full, alphas=alphas)


def hyperon_request_spin(nP, nN, spins):
    """One spin component: protons, neutrons, then the Lambda's index."""
    pm, nm, lm = _mask(spins[:nP]), _mask(spins[nP:nP + nN]), _mask(spins[nP + nN:nP + nN + 1])
    assert bin(pm).count("1") == nP and bin(nm).count("1") == nN and bin(lm).count("1") == 1
    return dict(sinkP=pm, sinkN=nm, sinkL=lm, alphas=[(pm, nm, lm)])


def hyperon_delta_sets(nP, nN, req):
    """Sink sets (P set, N set, Lambda index), proton rank major, then the
    neutron rank, then the Lambda's."""
    ps = [_mask(c) for c in itertools.combinations(_bits(req["sinkP"]), nP)]
    ns = [_mask(c) for c in itertools.combinations(_bits(req["sinkN"]), nN)]
    ls = [1 << b for b in _bits(req["sinkL"])]
    return [(p, n, l) for p in ps for n in ns for l in ls]


def hyperon_L(rel, nsrc, nP, nN, alpha):
    """L(alpha; z) on sorted (u, d, s) sets of the system (Sec. 2)."""
    types = [PROTON] * nP + [NEUTRON] * nN + [LAMBDA]
    chis = _bits(alpha[0]) + _bits(alpha[1]) + _bits(alpha[2])
    return L_uca(rel, nsrc, types, chis, with_s=True)


def _sgn_group(x, y):
    """sgn(x|y) of Sec. 3 for one group: -1 to the number of pairs i in x,
    j in y with i > j."""
    return -1 if sum(bin(x >> (j + 1)).count("1") for j in _bits(y)) % 2 else 1


def hyperon_term_list(rel, nsrc, nP, nN, req, with_ops=False):
    """term_list for nP protons, nN neutrons and one Lambda added last:
    components are (P set, N set, Lambda set, u, d, s); the stages before
    the Lambda hold nucleon components only (4-tuples as in term_list).
    The Lambda step's operations split every final component z into x (a
    nucleon component) and y = (the Lambda's spin, one u, one d, the s
    index) with sign sgn(x_u|y_u) sgn(x_d|y_d)."""
    D = 4 if rel else 2
    Ls, U = {}, set()
    for a in req["alphas"]:
        um, dm, sm, cf = hyperon_L(rel, nsrc, nP, nN, a)
        Ls[a] = {(int(u), int(d), int(x)): int(c) for u, d, x, c in zip(um, dm, sm, cf)}
        U.update(Ls[a].keys())
    U = sorted(U)
    dsets = hyperon_delta_sets(nP, nN, req)
    final = np.array([(p, n, l, u, d, x) for (p, n, l) in dsets for (u, d, x) in U], np.uint32).reshape(-1, 6)
    final = final[np.lexsort(final.T[::-1])]
    seq = path(nP, nN) if nP + nN else []
    shapes, kp, kn = [], 0, 0
    for t in seq:
        kp += t == PROTON
        kn += t == NEUTRON
        shapes.append((kp, kn, 2 * kp + kn, kp + 2 * kn))
    nuc_final = np.unique(final[:, [0, 1, 3, 4]], axis=0) if seq else None
    reqs = [req_stage(nuc_final, sh) for sh in shapes] + [final]
    ops = []
    for i in range(1, len(seq)):
        ops.append(lambda_stage(reqs[i], seq[i], reqs[i - 1], rows=with_ops))
    if seq:
        xs = reqs[-2]
        xindex = {tuple(map(int, r)): i for i, r in enumerate(xs)}
        rows = []
        for iz, (p, n, l, u, d, x) in enumerate(final.tolist()):
            for yu in _bits(u):
                for yd in _bits(d):
                    xk = (p, n, u & ~(1 << yu), d & ~(1 << yd))
                    sg = _sgn_group(xk[2], 1 << yu) * _sgn_group(xk[3], 1 << yd)
                    rows.append((iz, xindex[xk], l, 1 << yu, 1 << yd, x, sg))
        ops.append(np.array(rows, np.int64).reshape(-1, 7) if with_ops else len(rows))
    n_ops = sum(len(o) if with_ops else o for o in ops)
    return dict(L=Ls, U=U, dsets=dsets, path=seq + [LAMBDA], shapes=shapes, req=reqs, ops=ops,
                n_lambda=int(n_ops), D=D)


def hyperon_correlators(rel, nsrc, nP, nN, req, Su, Sd, Ss, sinkw=None, scale=1.0):
    """C[delta set, alpha set] of the system by eq. f_L_contr with the blocks
    by their definition, keyed by (delta, alpha) triples."""
    D = 4 if rel else 2
    fP, fN = blocks(rel, nsrc, Su, Sd, sinkw, scale, D=D)
    fL = blocks_lambda(rel, nsrc, Su, Sd, Ss, sinkw, scale, D=D)
    types = [PROTON] * nP + [NEUTRON] * nN + [LAMBDA]
    out = {}
    for a in req["alphas"]:
        um, dm, sm, cf = hyperon_L(rel, nsrc, nP, nN, a)
        for d in hyperon_delta_sets(nP, nN, req):
            psis = _bits(d[0]) + _bits(d[1]) + _bits(d[2])
            out[(d, a)] = corr_from_L(types, psis, fP, fN, um, dm, cf, fL=fL, sm=sm)
    return out


def rescale_exponent(t: int, m: float) -> int:
    """k(t) = round(m t / ln 2): the propagators of timeslice t are read
    multiplied by 2**k(t), which undoes their decay exp(-m t) up to a factor
    in [2**-0.5, 2**0.5] and is exact in binary floating point."""
    return int(math.floor(m * t / math.log(2.0) + 0.5))
