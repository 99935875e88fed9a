"""Pins for the oracle's trapping (Section 2.2.3) and MIO drainage (2.4.1).

Trapping: the union-find reverse sweep is checked against one breadth-first
search per invaded voxel (the definition), a hand-worked fixture, and the
special cases fixed by the definition (every pore voxel an outlet: nothing
trapped; no outlet: every invaded voxel trapped; more outlets never trap
more). MIO: erosion read from the distance transform is checked against a
voxel-by-voxel erosion with the ball, a hand-worked fixture, and the
per-voxel definition of the opening.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_2101_03240_amd import synth
from tests import _golden


def test_golden_1d_pocket():
    g = _golden.load("trap_1d_pocket.txt")
    seq = _golden.as_volume(g["seq"])
    r = oracle.trap(seq, _golden.as_volume(g["outlets"]))
    np.testing.assert_array_equal(r["trapped"], _golden.as_volume(g["trapped"]))
    np.testing.assert_array_equal(r["seq_trapped"], _golden.as_volume(g["seq_trapped"]))
    assert r["K_after"] == int(g["K_after"].ravel()[0])
    np.testing.assert_array_equal(oracle.trap_brute(seq, _golden.as_volume(g["outlets"])),
                                  _golden.as_volume(g["trapped"]))


def test_golden_2d_throat_nothing_trapped():
    g = _golden.load("ibip_2d_throat.txt")
    seq = _golden.as_volume(g["seq"]).astype(np.int32)
    r = oracle.trap(seq, _golden.as_volume(g["outlets"]))
    np.testing.assert_array_equal(r["trapped"], _golden.as_volume(g["trapped"]))


def _invaded_case(rng, max_side=10):
    shape = tuple(int(s) for s in rng.integers(2, max_side + 1, size=3))
    img = (rng.random(shape) < rng.uniform(0.55, 0.9)).astype(np.uint8)
    img.flat[int(rng.integers(img.size))] = 0
    inl = synth.face_mask(shape, 0, 0)
    out = synth.face_mask(shape, 0, shape[0] - 1)
    r = oracle.invade(img, inl)
    return img, out, r["seq"]


@settings(max_examples=60, deadline=None)
@given(st.integers(0, 2**31 - 1))
def test_union_find_matches_breadth_first_search(seed):
    rng = np.random.default_rng(seed)
    img, out, seq = _invaded_case(rng)
    if rng.random() < 0.3:
        out = (rng.random(seq.shape) < 0.1).astype(np.uint8)
    r = oracle.trap(seq, out)
    np.testing.assert_array_equal(r["trapped"], oracle.trap_brute(seq, out))


@settings(max_examples=40, deadline=None)
@given(st.integers(0, 2**31 - 1))
def test_random_sequences_match_breadth_first_search(seed):
    """Arbitrary step labels (not from an invasion) exercise every branch."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in rng.integers(1, 8, size=3))
    seq = rng.integers(-1, 6, size=shape).astype(np.int32)
    out = (rng.random(shape) < 0.2).astype(np.uint8)
    r = oracle.trap(seq, out)
    np.testing.assert_array_equal(r["trapped"], oracle.trap_brute(seq, out))


def test_special_cases():
    rng = np.random.default_rng(3)
    img, out, seq = _invaded_case(rng, max_side=12)
    all_pore = (seq >= 0).astype(np.uint8)
    r = oracle.trap(seq, all_pore)
    assert not r["trapped"].any()
    none = np.zeros_like(all_pore)
    r = oracle.trap(seq, none)
    np.testing.assert_array_equal(r["trapped"].astype(bool), seq > 0)
    assert r["K_after"] == 0 and (r["seq_trapped"][seq >= 0] == 0).all()


def test_more_outlets_never_trap_more_and_rerank_is_contiguous():
    rng = np.random.default_rng(11)
    for _ in range(10):
        img, out, seq = _invaded_case(rng)
        extra = out | (rng.random(seq.shape) < 0.05).astype(np.uint8)
        a = oracle.trap(seq, out)
        b = oracle.trap(seq, extra)
        assert (b["trapped"] <= a["trapped"]).all()
        assert (a["trapped"].astype(bool) <= (seq > 0)).all()
        st_ = a["seq_trapped"]
        vals = np.unique(st_[st_ > 0])
        np.testing.assert_array_equal(vals, np.arange(1, a["K_after"] + 1))
        # re-ranking keeps the order of the surviving steps
        keep = (seq > 0) & (a["trapped"] == 0)
        order_a = np.argsort(seq[keep], kind="stable")
        assert (np.diff(st_[keep][order_a]) >= 0).all()
        np.testing.assert_array_equal(st_ == -1, seq == -1)


def test_golden_2d_throat_mio():
    g = _golden.load("ibip_2d_throat.txt")
    img = _golden.as_volume(g["image"])
    inl = _golden.as_volume(g["inlets"])
    T = g["mio_T"].ravel().astype(np.uint32)
    for brute in (False, True):
        m = oracle.mio(img, inl, T, brute_erosion=brute)
        np.testing.assert_array_equal(m["mio_r2"], _golden.as_volume(g["mio_r2"]))
        np.testing.assert_array_equal(m["mio_sat"], g["mio_sat_num"].ravel() / int(g["n_pore"].ravel()[0]))


@settings(max_examples=25, deadline=None)
@given(st.integers(0, 2**31 - 1))
def test_mio_erosion_from_dt_equals_ball_erosion(seed):
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in rng.integers(2, 11, size=3))
    img = (rng.random(shape) < rng.uniform(0.6, 0.95)).astype(np.uint8)
    img.flat[int(rng.integers(img.size))] = 0
    inl = synth.face_mask(shape, int(rng.integers(3)), 0)
    T = np.array(sorted(set(int(t) for t in rng.integers(1, 20, size=5)), reverse=True), np.uint32)
    a = oracle.mio(img, inl, T, brute_erosion=False)
    b = oracle.mio(img, inl, T, brute_erosion=True)
    np.testing.assert_array_equal(a["mio_r2"], b["mio_r2"])
    np.testing.assert_array_equal(a["mio_sat"], b["mio_sat"])


def test_mio_matches_per_voxel_definition():
    """mio_r2[v] = largest T_i such that some kept centre c at T_i has
    |v - c|^2 < T_i (0 if none)."""
    img = synth.overlapping_spheres((16, 15, 14), r2=9, porosity=0.6, seed=5)
    inl = synth.face_mask(img.shape, 0, 0)
    dt2 = oracle.edt(img)
    T = np.array(sorted(set(int(t) for t in np.unique(dt2[img > 0])), reverse=True), np.uint32)
    m = oracle.mio(img, inl, T)
    g = np.indices(img.shape).reshape(3, -1).T
    want = np.zeros(img.size, np.uint32)
    for t in T[::-1]:  # ascending, so larger T overwrite
        kept = np.argwhere(oracle.mio_kept(img, inl, dt2, int(t)))
        if kept.size == 0:
            continue
        hit = np.zeros(img.size, bool)
        for c in kept:
            hit |= ((g - c) ** 2).sum(1) < t
        want[hit] = t
    np.testing.assert_array_equal(m["mio_r2"].ravel(), want)
