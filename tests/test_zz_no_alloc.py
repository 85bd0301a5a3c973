"""mb_make_blocks_noalloc (the site-chunk partial sums in the library's fixed
device scratch) against mb_make_blocks (caller workspace), through the C ABI:
two calls in a row on the same GPU, the second with a smaller input, each
giving exactly the blocks of the workspace call (same kernels, same
chunking).  Runs alone in a fresh process and after the other tests."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1301_4895_amd import binding as B
from tests.gpu_helpers import host_props

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _blocks_both_ways(tl, Su, Sd, w, k, precision):
    tu = torch.from_numpy(np.ascontiguousarray(Su)).to(DEV)
    td = tu if Sd is Su else torch.from_numpy(np.ascontiguousarray(Sd)).to(DEV)
    tw = None if w is None else torch.view_as_real(torch.from_numpy(np.ascontiguousarray(w)).to(DEV))
    tk = torch.from_numpy(k).to(DEV)
    p = B.problem(len(Su), Su.shape[1], tu, td, precision, tw, tk)
    nb, nbw, _ = B.workspace_query(tl, p)
    assert nbw <= B.MB_NOALLOC_SCRATCH_BYTES
    ref = torch.empty(nb, dtype=torch.uint8, device=DEV)
    ws = torch.empty(nbw, dtype=torch.uint8, device=DEV)
    got = torch.full((nb,), 0xA5, dtype=torch.uint8, device=DEV)   # garbage the call must overwrite
    B.make_blocks(tl, p, ref, ws)
    B.make_blocks_noalloc(tl, p, got)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("rel,nsrc,same_ud,dtype,shapes", [
    (True, 1, True, np.complex64, [(125, 40), (27, 7)]),           # relativistic, u = d
    (False, 2, False, np.complex128, [(64, 33), (8, 3)]),          # two sources, u != d, sink functions
    (False, 1, True, np.complex128, [(216, 70), (27, 5)]),         # nonrelativistic, one source
])
def test_noalloc_blocks_match_workspace_blocks(rel, nsrc, same_ud, dtype, shapes):
    tl = B.TermList(1, 1, rel, nsrc, all_components=True)
    rng = np.random.default_rng(5)
    for call, (V, nl) in enumerate(shapes):
        Su = host_props(81 + call, 0, nl, 1, V, nsrc, dtype)[:, 0]
        Sd = Su if same_ud else host_props(81 + call, 1, nl, 1, V, nsrc, dtype)[:, 0]
        w = (rng.normal(size=(nsrc, V)) + 1j * rng.normal(size=(nsrc, V))) if nsrc == 2 else None
        k = rng.integers(-2, 3, size=nl).astype(np.int32)
        # MB_MIXED_F32B: the float block copies after the exponents too
        for prec in (B.MB_FP64, B.MB_MIXED, B.MB_MIXED_F32B):
            got, ref = _blocks_both_ways(tl, Su, Sd, w, k, prec)
            assert np.array_equal(got, ref), (call, V, nl, prec)


def test_noalloc_rejects_problems_beyond_the_scratch():
    # relativistic blocks of 2048 lanes on 64^3 sites need ~245 MB of partial sums
    tl = B.TermList(1, 1, True, 1, all_components=True)
    t = torch.empty((1,), dtype=torch.complex64, device=DEV)
    p = B.problem(2048, 64 ** 3, t, t, B.MB_MIXED)
    _, nbw, _ = B.workspace_query(tl, p)
    assert nbw > B.MB_NOALLOC_SCRATCH_BYTES
    with pytest.raises(B.MBError) as e:
        B.make_blocks_noalloc(tl, p, t)
    assert e.value.code == B.MB_ENOWORKSPACE
