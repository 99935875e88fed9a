"""Oracle pins for the variant readings (other readings of passages the
paper leaves ambiguous): footnote 1's integer sphere rule, inlet masking,
and 26-connected trapping."""
import math

import numpy as np
import pytest

import oracle
from paper_2101_03240_amd import synth
from tests import _golden


def _case(seed, solid_inlets=False):
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in rng.integers(4, 14, size=3))
    if seed % 3 == 0:
        shape = (1,) + shape[1:]
    img = (rng.random(shape) < rng.uniform(0.6, 0.95)).astype(np.uint8)
    img.flat[int(rng.integers(img.size))] = 0
    inl = np.zeros(shape, np.uint8)
    if solid_inlets:
        inl = (rng.random(shape) < 0.08).astype(np.uint8)
    else:
        inl[0] = 1
    return img, inl


def _paint_integer_brute(img, cs, M):
    """seq by definition under the integer rule: min step over centres c with
    |v - c|^2 <= floor(sqrt(M))^2, pore voxels only."""
    seq = np.where(img > 0, 0, -1).astype(np.int64)
    best = np.full(img.shape, np.iinfo(np.int64).max)
    grid = np.indices(img.shape).reshape(3, -1).T
    for c in np.argwhere(cs > 0):
        k = int(cs[tuple(c)])
        R = math.isqrt(int(M[k - 1]))
        d2 = ((grid - c) ** 2).sum(1).reshape(img.shape)
        hit = (d2 <= R * R) & (img > 0)
        best = np.where(hit, np.minimum(best, k), best)
    return np.where((img > 0) & (best < np.iinfo(np.int64).max), best, seq)


@pytest.mark.parametrize("seed", range(10))
def test_integer_ball_by_definition(seed):
    img, inl = _case(seed)
    r = oracle.invade(img, inl, integer_ball=True)
    lit = oracle.invade(img, inl, integer_ball=True, literal=True)
    assert r["K"] == lit["K"]
    np.testing.assert_array_equal(r["seq"], lit["seq"])
    np.testing.assert_array_equal(r["M"], lit["M"])
    np.testing.assert_array_equal(r["seq"], _paint_integer_brute(img, r["centre_step"], r["M"]))
    # the selection does not depend on the sphere rule
    d = oracle.invade(img, inl)
    np.testing.assert_array_equal(r["centre_step"], d["centre_step"])
    np.testing.assert_array_equal(r["M"], d["M"])


def test_integer_ball_differs_where_expected():
    # all pore except the eight corners of the central 3x3x3 cube: the centre
    # has dt2 = 3 (nearest solid at offset (1, 1, 1)) and is the first centre
    # from a single inlet there. The strict ball {|o|^2 < 3} paints the centre,
    # its 6 face and 12 edge neighbours (19); the integer ball, radius
    # floor(sqrt(3)) = 1, paints {|o|^2 <= 1}: the centre and 6 faces (7)
    img = np.ones((5, 5, 5), np.uint8)
    for x in (1, 3):
        for y in (1, 3):
            for z in (1, 3):
                img[x, y, z] = 0
    inl = np.zeros_like(img)
    inl[2, 2, 2] = 1
    assert oracle.edt(img)[2, 2, 2] == 3
    s = oracle.invade(img, inl, max_steps=1)
    i = oracle.invade(img, inl, max_steps=1, integer_ball=True)
    assert s["M"][0] == 3 and i["M"][0] == 3
    assert (s["seq"] == 1).sum() == 19 and (i["seq"] == 1).sum() == 7


def test_mask_inlets_fixture():
    # a row whose only inlet voxel is solid: the literal reading seeds its pore
    # neighbour, the masked reading seeds nothing
    img = np.array([[[0, 1, 1, 1, 0]]], np.uint8)
    inl = np.array([[[1, 0, 0, 0, 0]]], np.uint8)
    lit = oracle.invade(img, inl)
    msk = oracle.invade(img, inl, mask_inlets=True)
    assert lit["K"] >= 1 and lit["seq"][0, 0, 1] == 1
    assert msk["K"] == 0
    np.testing.assert_array_equal(msk["seq"], np.where(img > 0, 0, -1))


@pytest.mark.parametrize("seed", range(8))
def test_mask_inlets_candidate_equals_literal(seed):
    img, inl = _case(seed, solid_inlets=True)
    r = oracle.invade(img, inl, mask_inlets=True)
    lit = oracle.invade(img, inl, mask_inlets=True, literal=True)
    assert r["K"] == lit["K"]
    np.testing.assert_array_equal(r["seq"], lit["seq"])
    # masking the inlets by pore beforehand is the same thing
    r2 = oracle.invade(img, (inl & img).astype(np.uint8))
    np.testing.assert_array_equal(r["seq"], r2["seq"])


@pytest.mark.parametrize("seed", range(4))
def test_mask_inlets_mio_invariant(seed):
    img, inl = _case(seed + 20, solid_inlets=True)
    r = oracle.invade(img, inl, mask_inlets=True)
    dt2 = oracle.edt(img)
    cs, M, K = r["centre_step"], r["M"], r["K"]
    for t in sorted(set(int(x) for x in dt2[dt2 > 0]))[::-1][:6]:
        below = np.nonzero(M < t)[0]
        kstar = int(below[0]) + 1 if below.size else K + 1
        np.testing.assert_array_equal((cs > 0) & (cs < kstar), oracle.mio_kept(img, inl, dt2, t, mask_inlets=True))


def test_trap26_fixture():
    g = _golden.load("trap_2d_diagonal.txt")
    seq = _golden.as_volume(g["seq"]).astype(np.int32)
    out = _golden.as_volume(g["outlets"]).astype(np.uint8)
    np.testing.assert_array_equal(oracle.trap(seq, out, conn=6)["trapped"], _golden.as_volume(g["trapped6"]))
    np.testing.assert_array_equal(oracle.trap(seq, out, conn=26)["trapped"], _golden.as_volume(g["trapped26"]))
    np.testing.assert_array_equal(oracle.trap_brute(seq, out, conn=26), _golden.as_volume(g["trapped26"]))


@pytest.mark.parametrize("seed", range(8))
def test_trap26_union_find_equals_definition(seed):
    img, inl = _case(seed)
    r = oracle.invade(img, inl)
    out = np.zeros_like(img)
    out[-1] = 1
    t = oracle.trap(r["seq"], out, conn=26)
    np.testing.assert_array_equal(t["trapped"], oracle.trap_brute(r["seq"], out, conn=26))
    # more connections never trap more
    t6 = oracle.trap(r["seq"], out, conn=6)
    assert not (t["trapped"] & ~t6["trapped"].astype(bool)).any()
