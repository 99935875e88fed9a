"""Oracle pins for the saturation map and the trapping-aware curves
(Sections 2.2.1-2.2.3, Figure 5 left)."""
import numpy as np
import pytest

import oracle
from paper_2101_03240_amd import synth
from tests import _golden


def test_pocket_fixture():
    g = _golden.load("sat_1d_pocket.txt")
    seq = _golden.as_volume(g["seq"]).astype(np.int32)
    M = g["M"].reshape(-1).astype(np.uint32)
    s = oracle.steps(seq, M, c0=2.0)
    np.testing.assert_array_equal(s["sat"] * 4, g["sat_num"].reshape(-1))
    np.testing.assert_array_equal(oracle.satmap(seq, s["sat"]).reshape(-1) * 4, g["satmap_num"].reshape(-1))
    out = np.zeros_like(seq, dtype=np.uint8)
    out[0, 0, -1] = 1
    t = oracle.trap(seq, out)
    np.testing.assert_array_equal(t["seq_trapped"].reshape(-1), g["seq_trapped"].reshape(-1))
    Ma = oracle.remap_steps(seq, t["seq_trapped"], M, t["K_after"])
    np.testing.assert_array_equal(Ma, g["M_after"].reshape(-1))
    sa = oracle.steps(t["seq_trapped"], Ma, c0=2.0)
    np.testing.assert_array_equal(sa["sat"] * 4, g["sat_after_num"].reshape(-1))
    np.testing.assert_array_equal(oracle.satmap(t["seq_trapped"], sa["sat"]).reshape(-1) * 4,
                                  g["satmap_after_num"].reshape(-1))
    np.testing.assert_allclose(sa["pc"], [2 / 3, 1.0, 2.0], rtol=1e-15)


def _case(seed):
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in rng.integers(6, 20, size=3))
    img = synth.overlapping_spheres(shape, r2=int(rng.integers(3, 12)), porosity=float(rng.uniform(0.55, 0.8)),
                                    seed=seed)
    if img.all():
        img.flat[0] = 0
    inl = synth.face_mask(shape, 0, 0)
    out = synth.face_mask(shape, 0, shape[0] - 1)
    return img, inl, out


@pytest.mark.parametrize("seed", range(6))
def test_threshold_of_the_map_is_the_configuration(seed):
    img, inl, out = _case(seed)
    r = oracle.invade(img, inl)
    s = oracle.steps(r["seq"], r["M"])
    m = oracle.satmap(r["seq"], s["sat"])
    assert ((m == -1) == (img == 0)).all()
    assert ((m == 0) == ((img != 0) & (r["seq"] == 0))).all()
    for k in np.unique(r["seq"][r["seq"] > 0])[:: max(1, r["K"] // 15)]:
        np.testing.assert_array_equal((m > 0) & (m <= s["sat"][k - 1]), (r["seq"] >= 1) & (r["seq"] <= k))


@pytest.mark.parametrize("seed", range(6))
def test_trapped_curve(seed):
    img, inl, out = _case(seed)
    r = oracle.invade(img, inl)
    t = oracle.trap(r["seq"], out)
    Ma = oracle.remap_steps(r["seq"], t["seq_trapped"], r["M"], t["K_after"])
    # the surviving steps, as a set, in increasing order, keep their radii
    alive = np.unique(r["seq"][(r["seq"] > 0) & (t["trapped"] == 0)])
    np.testing.assert_array_equal(Ma, r["M"][alive - 1])
    sa = oracle.steps(t["seq_trapped"], Ma)
    n_pore = int((img != 0).sum())
    invaded = int((r["seq"] > 0).sum())
    trapped = int(t["trapped"].sum())
    if t["K_after"]:
        assert sa["sat"][-1] == (invaded - trapped) / n_pore
        assert (np.diff(sa["sat"]) > 0).all()  # every surviving step keeps at least one voxel
    m = oracle.satmap(t["seq_trapped"], sa["sat"])
    assert ((m > 0) == ((r["seq"] > 0) & (t["trapped"] == 0))).all()


def test_remap_rejects_inconsistent_labels():
    seq = np.array([[[1, 2, 3]]], np.int32)
    bad = np.array([[[1, 1, 2]]], np.int32)  # two original steps in one re-ranked step
    with pytest.raises(Exception):
        oracle.remap_steps(seq, bad, np.array([9, 4, 1], np.uint32), 2)


def test_compare_opening_fixture():
    g = _golden.load("compare_1d.txt")
    sat_T = g["sat_T_x6"].reshape(-1) / 6.0
    sm = (g["satmap_x6"].reshape(-1) / 6.0).reshape(1, 1, -1)
    c = oracle.compare_opening(sm, g["mio_r2"].reshape(1, 1, -1), g["T"].reshape(-1), sat_T,
                               trapped=g["trapped"].reshape(1, 1, -1))
    np.testing.assert_array_equal(c["disagree"], g["disagree"].reshape(-1))
    np.testing.assert_array_equal(c["mio_trapped"], g["mio_trapped"].reshape(-1))


def test_compare_opening_identical_configurations():
    # an opening that holds exactly IBIP's configuration at every level agrees
    # everywhere: levels = the distinct saturations l_0 < l_1 < ..., T[i] =
    # n - i, and a voxel with satmap l_j first held at level j (mio_r2 = T[j])
    img, inl, out = _case(2)
    r = oracle.invade(img, inl)
    s = oracle.steps(r["seq"], r["M"])
    m = oracle.satmap(r["seq"], s["sat"])
    levels = np.unique(m[m > 0])
    n = len(levels)
    T = np.arange(n, 0, -1).astype(np.uint32)
    r2 = np.where(m > 0, T[np.searchsorted(levels, m)], 0).astype(np.uint32) if n else np.zeros(img.shape, np.uint32)
    c = oracle.compare_opening(m, r2, T, levels)
    assert (c["disagree"] == 0).all()
    # shifting the opening one level later disagrees by exactly the voxels of each next level
    c2 = oracle.compare_opening(m, r2, T, np.concatenate([levels[1:], [2.0]])[: n])
    np.testing.assert_array_equal(c2["disagree"][:-1], [int((m == lv).sum()) for lv in levels[1:]])
