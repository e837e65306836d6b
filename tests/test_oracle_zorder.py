"""Pins of the z-order oracle (oracle/zorder32.py) against definitions that
do not share its code: closed-form codes, an inverse, the octree order the
Morton code is defined to produce, quantisation end points and stability."""
import numpy as np

from oracle import zorder32 as Z


def test_interleave_closed_forms():
    # x in bit 0, y in bit 1, z in bit 2, then the next bit of each
    assert Z.interleave(np.array([1]), np.array([0]), np.array([0]))[0] == 1
    assert Z.interleave(np.array([0]), np.array([1]), np.array([0]))[0] == 2
    assert Z.interleave(np.array([0]), np.array([0]), np.array([1]))[0] == 4
    assert Z.interleave(np.array([1]), np.array([1]), np.array([1]))[0] == 7
    assert Z.interleave(np.array([2]), np.array([0]), np.array([0]))[0] == 8
    assert Z.interleave(np.array([0]), np.array([0]), np.array([512]))[0] == 1 << 29
    full = np.array([1023])
    assert Z.interleave(full, full, full)[0] == (1 << 30) - 1


def test_interleave_is_a_bijection_with_its_inverse():
    rng = np.random.default_rng(0)
    q = rng.integers(0, 1024, size=(3, 5000)).astype(np.uint32)
    c = Z.interleave(q[0], q[1], q[2])
    assert np.array_equal(np.stack(Z.deinterleave(c)), q)
    codes = rng.integers(0, 1 << 30, size=5000).astype(np.uint32)
    assert np.array_equal(Z.interleave(*Z.deinterleave(codes)), codes)


def _octree_order(cells, depth):
    """Cells of a 2^depth grid listed by recursive subdivision: octant index
    (x half) + 2 (y half) + 4 (z half), coarsest level first."""
    if depth == 0 or len(cells) <= 1:
        return list(cells)
    half = 1 << (depth - 1)
    out = []
    for octant in range(8):
        sub = [c for c in cells if ((c[0] >= half) == bool(octant & 1)) and ((c[1] >= half) == bool(octant & 2))
               and ((c[2] >= half) == bool(octant & 4))]
        sub = [(x % half, y % half, z % half, x, y, z) for (x, y, z) in sub]
        rec = _octree_order([s[:3] for s in sub], depth - 1)
        back = {s[:3]: s[3:] for s in sub}
        out += [back[r] for r in rec]
    return out


def test_code_order_is_the_octree_traversal():
    cells = [(x, y, z) for x in range(8) for y in range(8) for z in range(8)]
    ref = _octree_order(cells, 3)
    q = np.array(cells, np.uint32).T
    order = np.argsort(Z.interleave(q[0], q[1], q[2]), kind="stable")
    assert [cells[i] for i in order] == ref


def test_quantisation_end_points_and_degenerate_box():
    m = np.array([[0.0, 1.0, 0.5, 0.25], [2.0, 2.0, 2.0, 2.0], [-1.0, -1.0, -1.0, -0.5]], np.float32)
    q = Z.quantize32(m)
    # x spans the cube side 1: 0 -> 0, 1 -> clamped 1023, 0.5 -> 512, 0.25 -> 256
    assert q[0].tolist() == [0, 1023, 512, 256]
    assert q[1].tolist() == [0, 0, 0, 0]             # zero extent on y
    assert q[2].tolist() == [0, 0, 0, 512]
    assert not Z.quantize32(np.ones((3, 5), np.float32)).any()
    assert Z.zorder_permutation(np.zeros((3, 0), np.float32)).size == 0


def test_permutation_is_stable_and_sorted():
    rng = np.random.default_rng(3)
    m = rng.integers(0, 4, size=(3, 2000)).astype(np.float32)   # many equal codes
    perm = Z.zorder_permutation(m)
    assert np.array_equal(np.sort(perm), np.arange(2000))
    codes = Z.morton_codes(m)[perm]
    assert np.all(np.diff(codes.astype(np.int64)) >= 0)
    same = np.diff(codes.astype(np.int64)) == 0
    assert np.all(np.diff(perm.astype(np.int64))[same] > 0), "ties must keep the index order"
