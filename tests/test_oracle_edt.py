"""Pins for the oracle's distance transform (Section 2.1, Figure 2(b)).

The oracle's separable EDT is pinned to (1) the definition by brute force on
every 2D 4x4 image and on random 3D images, (2) closed forms, and (3) SciPy's
exact Euclidean distance transform, squared and rounded. The brute force is
itself pinned by the closed forms.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi
from hypothesis import given, settings, strategies as st

import oracle


def _all_4x4():
    bits = np.arange(1 << 16, dtype=np.uint32)[:, None]
    return ((bits >> np.arange(16, dtype=np.uint32)) & 1).astype(np.uint8).reshape(-1, 1, 4, 4)


def test_edt_exhaustive_2d_4x4_matches_brute_force():
    imgs = _all_4x4()
    for img in imgs:
        if img.all():
            with pytest.raises(oracle.OracleError) as e:
                oracle.edt(img)
            assert e.value.code == oracle.ENOSOLID
            continue
        np.testing.assert_array_equal(oracle.edt(img), oracle.edt_brute(img))


@pytest.mark.parametrize("shape,s", [((5, 6, 7), (2, 3, 4)), ((1, 9, 4), (0, 0, 3)), ((7, 1, 1), (6, 0, 0))])
def test_single_solid_voxel_closed_form(shape, s):
    img = np.ones(shape, np.uint8)
    img[s] = 0
    g = np.indices(shape)
    want = sum((g[i] - s[i]) ** 2 for i in range(3)).astype(np.uint32)
    np.testing.assert_array_equal(oracle.edt(img), want)
    np.testing.assert_array_equal(oracle.edt_brute(img), want)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_half_space_closed_form(axis):
    shape = (6, 7, 8)
    img = np.ones(shape, np.uint8)
    sl = [slice(None)] * 3
    sl[axis] = 0
    img[tuple(sl)] = 0
    want = (np.indices(shape)[axis] ** 2).astype(np.uint32)
    np.testing.assert_array_equal(oracle.edt(img), want)
    np.testing.assert_array_equal(oracle.edt_brute(img), want)


def test_two_solids_closed_form():
    img = np.ones((1, 1, 11), np.uint8)
    img[0, 0, 2] = 0
    img[0, 0, 9] = 0
    z = np.arange(11)
    want = np.minimum((z - 2) ** 2, (z - 9) ** 2).astype(np.uint32).reshape(1, 1, 11)
    np.testing.assert_array_equal(oracle.edt(img), want)


def test_border_is_not_solid():
    img = np.ones((3, 3, 3), np.uint8)
    img[1, 1, 1] = 0
    d = oracle.edt(img)
    assert d[0, 0, 0] == 3  # corner: distance to the centre solid, not to the border


@settings(max_examples=40, deadline=None)
@given(st.tuples(st.integers(1, 16), st.integers(1, 16), st.integers(1, 16)),
       st.floats(0.3, 0.97), st.integers(0, 2**31 - 1))
def test_random_3d_matches_brute_force(shape, porosity, seed):
    rng = np.random.default_rng(seed)
    img = (rng.random(shape) < porosity).astype(np.uint8)
    if img.all():
        img.flat[rng.integers(img.size)] = 0
    np.testing.assert_array_equal(oracle.edt(img), oracle.edt_brute(img))


@pytest.mark.parametrize("seed", range(6))
def test_matches_scipy_exact_edt(seed):
    rng = np.random.default_rng(100 + seed)
    shape = tuple(int(s) for s in rng.integers(10, 40, size=3))
    img = (rng.random(shape) < rng.uniform(0.6, 0.995)).astype(np.uint8)
    img.flat[0] = 0
    want = np.rint(ndi.distance_transform_edt(img) ** 2).astype(np.uint32)
    np.testing.assert_array_equal(oracle.edt(img), want)


def test_point_query_matches_full_transform():
    rng = np.random.default_rng(7)
    img = (rng.random((20, 17, 23)) < 0.9).astype(np.uint8)
    img[3, 3, 3] = 0
    d = oracle.edt(img)
    for _ in range(300):
        x, y, z = (int(rng.integers(0, n)) for n in img.shape)
        assert oracle.edt_at(img, x, y, z) == d[x, y, z]
