"""fgs_sort_pairs_noalloc (the pair sort on the library's static scratch)
against fgs_sort_pairs (the same sort on a caller workspace), both through the
C ABI: several calls in a row, each smaller than the one before, so that every
later call runs over the scratch contents an earlier call left."""
import numpy as np
import pytest
import torch

from paper_2602_09999_amd import _lib as L
from paper_2602_09999_amd import binding as B

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)


def _pairs(n, key_bytes, key_bits, seed):
    rng = np.random.default_rng(seed)
    utype = np.uint16 if key_bytes == 2 else np.uint32
    keys = rng.integers(0, 1 << (8 * key_bytes), n, dtype=np.uint64).astype(utype)
    itype = np.int16 if key_bytes == 2 else np.int32
    return keys, torch.from_numpy(keys.view(itype).copy()).cuda(), torch.arange(n, dtype=torch.int32, device="cuda")


# (key bytes, key bits, n): the largest accepted size first, then smaller ones
CALLS = [(4, 32, L.FGS_SORT_NOALLOC_MAX_PAIRS), (4, 31, 300_007), (2, 13, 70_001), (2, 16, 4_097), (4, 20, 5)]


def test_noalloc_sort_equals_workspace_sort():
    for call, (kb, bits, n) in enumerate(CALLS):
        say("no-alloc sort call", call, "key bytes", kb, "bits", bits, "n", n)
        keys, dk, dv = _pairs(n, kb, bits, seed=call)
        ka, va = dk.clone(), dv.clone()
        B.sort_pairs(ka, va, bits)
        kb_, vb = dk.clone(), dv.clone()
        B.sort_pairs_noalloc(kb_, vb, bits)
        torch.cuda.synchronize()
        assert torch.equal(ka, kb_) and torch.equal(va, vb), f"call {call}"
        mask = (1 << bits) - 1
        perm = np.argsort(keys.astype(np.uint64) & np.uint64(mask), kind="stable")
        assert np.array_equal(vb.cpu().numpy(), perm.astype(np.int32)), f"call {call}"


def test_noalloc_sort_rejects_more_pairs_than_its_scratch():
    n = L.FGS_SORT_NOALLOC_MAX_PAIRS + 1
    k = torch.zeros(n, dtype=torch.int32, device="cuda")
    v = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(L.FasterGSError) as e:
        B.sort_pairs_noalloc(k, v, 32)
    assert e.value.status == L.FGS_ERR_INVALID_ARGUMENT
    B.sort_pairs_noalloc(k[:0], v[:0], 8)  # empty: nothing to do
