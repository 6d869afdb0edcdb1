"""The allocation-free bitvector -> sparse conversion against the allocating
one, through the C ABI: two calls in a row on the same GPU (the second with a
smaller input, so stale scratch from the first would show), a ragged tail,
and the size limit."""
import numpy as np
import pytest

from gpu_util import say, torch_dev

pytestmark = pytest.mark.gpu


def _bits(n, density, seed):
    rng = np.random.default_rng(seed)
    member = rng.random(n) < density
    W = (n + 63) // 64
    padded = np.zeros(W * 64, bool)
    padded[:n] = member
    # junk above n in the last word must be ignored
    padded[n:] = True
    words = np.packbits(padded.reshape(W, 64)[:, ::-1], axis=1).view(">u8").ravel()
    return member, words.astype(np.uint64)


def _convert(gi, fn, n, words):
    torch, dev = torch_dev()
    bv = torch.from_numpy(words.view(np.int64).copy()).to(dev)
    ids = torch.full((n + 1,), -7, dtype=torch.int32, device=dev)
    cnt = torch.full((1,), -7, dtype=torch.int32, device=dev)
    fn(n, bv, ids, cnt)
    torch.cuda.synchronize()
    c = int(cnt.cpu().item())
    return c, ids.cpu().numpy()


def test_noalloc_matches_allocating_conversion():
    import paper_1805_00923_amd as gi
    for n, dens, seed in [(1_000_003, 0.3, 1), (70_001, 0.05, 2), (1, 1.0, 3), (64, 0.5, 4)]:
        say("noalloc bitvec_to_sparse n=%d density=%g seed=%d" % (n, dens, seed))
        member, words = _bits(n, dens, seed)
        c_ref, ids_ref = _convert(gi, gi.bitvec_to_sparse, n, words)
        c, ids = _convert(gi, gi.bitvec_to_sparse_noalloc, n, words)
        assert c == c_ref == int(member.sum())
        assert np.array_equal(ids[:c], ids_ref[:c_ref])
        assert np.array_equal(ids[:c], np.flatnonzero(member).astype(np.int32))
        assert (ids[c:] == -7).all()


def test_noalloc_limit_refused_before_device_work():
    import paper_1805_00923_amd as gi
    n = 64 * gi.NOALLOC_MAX_WORDS + 1
    torch, dev = torch_dev()
    small = torch.zeros(4, dtype=torch.int64, device=dev)
    with pytest.raises(gi.GiError) as e:
        gi.bitvec_to_sparse_noalloc(n, small, small, small)
    assert e.value.status == gi.GI_ERR_UNSUPPORTED
    assert "at most" in str(e.value)
