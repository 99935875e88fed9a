"""Pins for the oracle's invasion loop (Section 2.1; Sections 2.2.1-2.2.2).

Two oracle implementations pin each other: the literal loop (whole-image
cross dilation and rescan every step, as Figure 2(e)-(l) describes) and the
candidate-set loop. Both are pinned to hand-traced fixtures, and the
candidate-set loop to invariants fixed by the paper and by the mathematics:
every inserted sphere lies in pore space; a configuration is ``seq <= N``
with first write winning; the invaded set before the first step whose
inserted radius drops below R equals the MIO opening seed set at R (the
envelope of peak pressures equals the pressure-based curve, Sections 2.2.2,
3.1.1); saturation rises monotonically from 0 to the reachable fraction.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi
from hypothesis import given, settings, strategies as st

import oracle
from paper_2101_03240_amd import synth
from tests import _golden

CROSS = ndi.generate_binary_structure(3, 1)


def _q0(img, inlets):
    return (ndi.binary_dilation(inlets.astype(bool), structure=CROSS) | inlets.astype(bool)) & (img > 0)


def _check_golden_invasion(g, r):
    img = _golden.as_volume(g["image"])
    np.testing.assert_array_equal(oracle.edt(img), _golden.as_volume(g["dt2"]))
    np.testing.assert_array_equal(r["seq"], _golden.as_volume(g["seq"]))
    np.testing.assert_array_equal(r["rad2"], _golden.as_volume(g["rad2"]))
    np.testing.assert_array_equal(r["centre_step"], _golden.as_volume(g["centre_step"]))
    np.testing.assert_array_equal(r["M"], g["M"].ravel())


@pytest.mark.parametrize("literal", [False, True])
def test_golden_2d_throat(literal):
    g = _golden.load("ibip_2d_throat.txt")
    img = _golden.as_volume(g["image"])
    inl = _golden.as_volume(g["inlets"])
    r = oracle.invade(img, inl, literal=literal)
    _check_golden_invasion(g, r)
    s = oracle.steps(r["seq"], r["M"], c0=2.0)
    np.testing.assert_array_equal(s["n_new"], g["n_new"].ravel())
    n_pore = int(g["n_pore"].ravel()[0])
    np.testing.assert_array_equal(s["sat"], g["sat_num"].ravel() / n_pore)
    # Washburn: Pc = 2 sigma / r with sigma = 1, r = sqrt(M)
    np.testing.assert_array_equal(s["pc"], 2.0 / np.sqrt(g["M"].ravel().astype(np.float64)))
    assert s["pc"][2] == 2.0 and s["pc"][0] == 1.0


@pytest.mark.parametrize("literal", [False, True])
def test_golden_1d_blind_pores(literal):
    g = _golden.load("ibip_1d_blind.txt")
    img = _golden.as_volume(g["image"])
    r = oracle.invade(img, _golden.as_volume(g["inlets"]), literal=literal)
    _check_golden_invasion(g, r)


def test_max_steps_truncates_the_sequence():
    g = _golden.load("ibip_2d_throat.txt")
    img = _golden.as_volume(g["image"])
    inl = _golden.as_volume(g["inlets"])
    full = oracle.invade(img, inl)
    for k in range(1, 8):
        r = oracle.invade(img, inl, max_steps=k)
        assert r["K"] == k
        want = np.where(full["seq"] > k, 0, full["seq"])
        np.testing.assert_array_equal(r["seq"], want)
        np.testing.assert_array_equal(r["M"], full["M"][:k])


def test_no_inlet_means_no_step():
    img = np.ones((4, 4, 4), np.uint8)
    img[0, 0, 0] = 0
    r = oracle.invade(img, np.zeros_like(img))
    assert r["K"] == 0 and (r["seq"][img > 0] == 0).all()


def test_no_solid_is_an_error():
    img = np.ones((3, 3, 3), np.uint8)
    with pytest.raises(oracle.OracleError) as e:
        oracle.invade(img, synth.face_mask(img.shape))
    assert e.value.code == oracle.ENOSOLID


def _all_4x4():
    bits = np.arange(1 << 16, dtype=np.uint32)[:, None]
    return ((bits >> np.arange(16, dtype=np.uint32)) & 1).astype(np.uint8).reshape(-1, 1, 4, 4)


def test_exhaustive_2d_4x4_literal_equals_candidate_set():
    inl = np.zeros((1, 4, 4), np.uint8)
    inl[0, 0, :] = 1
    for img in _all_4x4():
        if img.all():
            continue
        a = oracle.invade(img, inl, literal=True)
        b = oracle.invade(img, inl, literal=False)
        assert a["K"] == b["K"]
        np.testing.assert_array_equal(a["seq"], b["seq"])
        np.testing.assert_array_equal(a["rad2"], b["rad2"])
        np.testing.assert_array_equal(a["centre_step"], b["centre_step"])
        np.testing.assert_array_equal(a["M"], b["M"])


def _random_case(rng, max_side=12):
    shape = tuple(int(s) for s in rng.integers(1, max_side + 1, size=3))
    img = (rng.random(shape) < rng.uniform(0.5, 0.95)).astype(np.uint8)
    img.flat[int(rng.integers(img.size))] = 0
    kind = rng.integers(3)
    if kind == 0:
        inl = synth.face_mask(shape, int(rng.integers(3)), 0)
    elif kind == 1:  # an interior inlet (evaporation-like, Section 2.1)
        inl = np.zeros(shape, np.uint8)
        inl[tuple(int(s) // 2 for s in shape)] = 1
    else:  # a random mask, possibly on solid voxels
        inl = (rng.random(shape) < 0.05).astype(np.uint8)
    return img, inl


@settings(max_examples=60, deadline=None)
@given(st.integers(0, 2**31 - 1))
def test_random_3d_literal_equals_candidate_set(seed):
    rng = np.random.default_rng(seed)
    img, inl = _random_case(rng)
    a = oracle.invade(img, inl, literal=True)
    b = oracle.invade(img, inl, literal=False)
    assert a["K"] == b["K"]
    for k in ("seq", "rad2", "centre_step", "M"):
        np.testing.assert_array_equal(a[k], b[k])


@settings(max_examples=40, deadline=None)
@given(st.integers(0, 2**31 - 1))
def test_random_3d_selection_alone_equals_full_loop(seed):
    """The candidate-set loop without sphere insertion selects the same
    centres with the same M (insertion never feeds back into selection)."""
    rng = np.random.default_rng(seed)
    img, inl = _random_case(rng)
    a = oracle.invade(img, inl)
    b = oracle.invade(img, inl, paint=False)
    assert a["K"] == b["K"] and b["seq"] is None
    np.testing.assert_array_equal(a["centre_step"], b["centre_step"])
    np.testing.assert_array_equal(a["M"], b["M"])
    # and on a literal-loop run truncated by max_steps
    c = oracle.invade(img, inl, max_steps=3, literal=True)
    d = oracle.invade(img, inl, max_steps=3, paint=False)
    assert c["K"] == d["K"]
    np.testing.assert_array_equal(c["centre_step"], d["centre_step"])


def _paint_by_definition(shape, cs, M):
    """seq[v] = min over popped c with |v - c|^2 < M[step(c)] of step(c)."""
    seq = np.zeros(shape, np.int64)
    g = np.indices(shape).reshape(3, -1).T
    best = np.full(g.shape[0], np.iinfo(np.int64).max)
    for c in np.argwhere(cs > 0):
        k = cs[tuple(c)]
        d2 = ((g - c) ** 2).sum(1)
        hit = d2 < M[k - 1]
        best[hit] = np.minimum(best[hit], k)
    seq.flat[:] = np.where(best == np.iinfo(np.int64).max, 0, best)
    return seq


def _frontier_definition_check(img, inl, r, dt2):
    """M_k = max of dt2 over F_k and C_k = its argmax set, with
    F_k = ((inlets U C_<k) dilated by a cross) & pore - C_<k."""
    cs = r["centre_step"]
    base = inl.astype(bool)
    for k in range(1, r["K"] + 1):
        popped = (cs > 0) & (cs < k)
        F = (ndi.binary_dilation(base | popped, structure=CROSS) | base | popped) & (img > 0) & ~popped
        assert F.any()
        m = dt2[F].max()
        assert m == r["M"][k - 1]
        np.testing.assert_array_equal(F & (dt2 == m), cs == k)
    popped = cs > 0
    F = (ndi.binary_dilation(base | popped, structure=CROSS) | base | popped) & (img > 0) & ~popped
    assert not F.any()


@pytest.mark.parametrize("seed", range(4))
def test_small_3d_against_definitions(seed):
    rng = np.random.default_rng(seed)
    img = synth.overlapping_spheres((14, 13, 12), r2=5, porosity=0.6, seed=seed)
    inl = synth.face_mask(img.shape, 0, 0)
    r = oracle.invade(img, inl)
    dt2 = oracle.edt(img)
    _frontier_definition_check(img, inl, r, dt2)
    np.testing.assert_array_equal(r["seq"][img > 0], _paint_by_definition(img.shape, r["centre_step"], r["M"])[img > 0])
    del rng


@pytest.fixture(scope="module")
def c1():
    img = synth.config_image("spheres64")
    inl = synth.face_mask(img.shape, 0, 0)
    return img, inl, oracle.invade(img, inl), oracle.edt(img)


def test_c1_generator_is_stable(c1):
    img = c1[0]
    assert synth.sha256(img) == "74e54c71a849e9801ddfd41327501c713f01f2bb7d2de4ecc9055b0a7630e89c"


def test_c1_basic_invariants(c1):
    img, inl, r, dt2 = c1
    seq, cs, M, K = r["seq"], r["centre_step"], r["M"], r["K"]
    assert K == M.shape[0] > 0
    np.testing.assert_array_equal(seq == -1, img == 0)  # nothing painted on solid
    inv = seq > 0
    np.testing.assert_array_equal(r["rad2"][inv], M[seq[inv] - 1])
    assert (r["rad2"][~inv] == 0).all()
    popped = cs > 0
    np.testing.assert_array_equal(dt2[popped], M[cs[popped] - 1])
    assert (seq[popped] <= cs[popped]).all()  # a centre lies inside its own sphere
    # every centre is a seed or touches an earlier centre
    q0 = _q0(img, inl)
    earlier = np.zeros_like(popped)
    for ax in range(3):
        for s in (-1, 1):
            nb = np.roll(cs, s, axis=ax)
            sl = [slice(None)] * 3
            sl[ax] = 0 if s == 1 else -1
            nb[tuple(sl)] = 0
            earlier |= (nb > 0) & (nb < cs)
    assert (q0 | earlier)[popped].all()
    # reachable pore (6-connected to Q0) is exactly what gets popped
    lab, _ = ndi.label(img > 0, structure=CROSS)
    reach = np.isin(lab, np.unique(lab[q0]))
    np.testing.assert_array_equal(popped, reach)


def test_c1_mio_seed_set_invariant(c1):
    """For every squared radius T: the centres popped before the first step
    with M_k < T are exactly the MIO kept set at T (eroded pore connected to
    the inlets), and the configuration at that point contains the MIO
    opening at T."""
    img, inl, r, dt2 = c1
    cs, M, seq = r["centre_step"], r["M"], r["seq"]
    for T in np.unique(dt2[img > 0]):
        below = np.nonzero(M < T)[0]
        kstar = int(below[0]) + 1 if below.size else r["K"] + 1
        ibip = (cs > 0) & (cs < kstar)
        kept = oracle.mio_kept(img, inl, dt2, int(T))
        np.testing.assert_array_equal(ibip, kept)
    T = np.array(sorted(set(int(t) for t in np.unique(dt2[img > 0])[::7]), reverse=True), dtype=np.uint32)
    mio = oracle.mio(img, inl, T)
    for t in T:
        below = np.nonzero(M < t)[0]
        kstar = int(below[0]) + 1 if below.size else r["K"] + 1
        conf = (seq > 0) & (seq < kstar)
        assert (conf | ~(mio["mio_r2"] == t)).all()


def test_c1_saturation_and_pc(c1):
    img, inl, r, dt2 = c1
    s = oracle.steps(r["seq"], r["M"], c0=oracle.washburn_c0(0.07, 0.3, 2e-6))
    sat = s["sat"]
    assert (np.diff(sat) >= 0).all() and sat[0] > 0
    assert sat[-1] == (r["seq"] > 0).sum() / (img > 0).sum()
    assert s["n_new"].sum() == (r["seq"] > 0).sum()
    c0 = 2 * 0.07 * np.cos(0.3) / 2e-6
    np.testing.assert_allclose(s["pc"] * np.sqrt(r["M"].astype(np.float64)), c0, rtol=1e-15)
