"""The device radix sort through the C ABI (fgs_sort_pairs) against numpy's
stable argsort: bit-exact keys and values, equal keys in input order.

Sizes span the three ways a pass scans its digit histogram: one workgroup per
digit (up to 2048 blocks of 4096 keys), one flat scan whose blocks add up the
partial sums before them (up to 2048 partial sums), and a flat scan over
scanned partial sums (beyond; 16-bit keys with a 7-bit digit reach it above
67M keys, 32-bit keys with 8-bit digits above 33.6M), with ragged tails."""
import numpy as np
import pytest
import torch

import paper_2602_09999_amd.binding as B

pytestmark = pytest.mark.gpu

CASES = [
    # (key bytes, key bits, n, distinct keys or None for the full range)
    (2, 13, 1, None),
    (2, 13, 4095, None),
    (2, 13, 4097, 7),
    (2, 16, 1_000_003, None),
    (2, 9, 300_007, None),        # digits 4 + 5 (16-bit keys: the narrower digit first)
    (2, 15, 500_009, 20_000),     # digits 7 + 8
    (4, 9, 300_007, None),        # digits 5 + 4 (32-bit keys: the narrower digit last)
    (2, 13, 9_000_001, None),     # flat scan, direct partial sums
    (2, 13, 70_000_017, 6_700),   # flat scan over scanned partial sums (7-bit pass)
    (4, 31, 5, None),
    (4, 32, 1_000_001, 3),
    (4, 31, 8_388_609, None),     # 2049 blocks: flat scan
    (4, 32, 34_000_003, None),    # flat scan over scanned partial sums
    (4, 20, 2_000_000, None),
]


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("key_bytes,key_bits,n,distinct", CASES)
def test_sort_pairs_matches_stable_sort(key_bytes, key_bits, n, distinct):
    say("sort", key_bytes, key_bits, n, distinct)
    rng = np.random.default_rng(n + key_bits)
    width = 8 * key_bytes
    utype = np.uint16 if key_bytes == 2 else np.uint32
    if distinct is None:
        keys = rng.integers(0, 1 << width, n, dtype=np.uint64).astype(utype)
    else:
        keys = rng.integers(0, distinct, n, dtype=np.uint64).astype(utype)
    if key_bits < width:
        # random bits above key_bits are carried along, never sorted by
        high = rng.integers(0, 1 << (width - key_bits), n, dtype=np.uint64) << np.uint64(key_bits)
        keys = (keys.astype(np.uint64) & np.uint64((1 << key_bits) - 1) | high).astype(utype)
    mask = utype((1 << key_bits) - 1)
    perm = np.argsort(keys & mask, kind="stable")
    itype = torch.int16 if key_bytes == 2 else torch.int32
    dk = torch.from_numpy(keys.view(np.int16 if key_bytes == 2 else np.int32)).cuda()
    dv = torch.arange(n, dtype=torch.int32, device="cuda")
    assert dk.dtype == itype
    B.sort_pairs(dk, dv, key_bits)
    torch.cuda.synchronize()
    got_k = dk.cpu().numpy().view(utype)
    got_v = dv.cpu().numpy()
    assert np.array_equal(got_v, perm.astype(np.int32))
    assert np.array_equal(got_k, keys[perm])


def test_sort_pairs_rejects_bad_arguments():
    k = torch.zeros(16, dtype=torch.int16, device="cuda")
    v = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError):
        B.sort_pairs(k, v, 17)
    with pytest.raises(TypeError):
        B.sort_pairs(k.float(), v, 8)
    B.sort_pairs(k[:0], v[:0], 8)  # empty: nothing to do
