"""Equal-saturation comparison of IBIP with the opening on the GPU against the
oracle (Section 3.1.1, Figures 8 and 9): the hand-worked fixture, random maps
over both the LDS-binned and the HBM path, and the whole 2D validation on
synthetic 500 x 500 images (blurred noise and overlapping disks), with and
without trapping."""
import numpy as np
import pytest

import oracle
from paper_2101_03240_amd import synth
from tests import _golden

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ibip = pytest.importorskip("paper_2101_03240_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _d(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)


def test_fixture(dev):
    g = _golden.load("compare_1d.txt")
    sat_T = g["sat_T_x6"].reshape(-1) / 6.0
    sm = (g["satmap_x6"].reshape(-1) / 6.0).reshape(1, 1, -1)
    c = ibip.compare_opening(_d(sm, dev), _d(_i32(g["mio_r2"].reshape(1, 1, -1)), dev), g["T"].reshape(-1),
                             sat_T, trapped=_d(g["trapped"].reshape(1, 1, -1).astype(np.uint8), dev))
    np.testing.assert_array_equal(c["disagree"].cpu().numpy(), g["disagree"].reshape(-1))
    np.testing.assert_array_equal(c["mio_trapped"].cpu().numpy(), g["mio_trapped"].reshape(-1))


@pytest.mark.parametrize("n_levels", [1, 7, 2048, 2049, 5000])
def test_random_maps(dev, n_levels):
    # random maps that hit the level values exactly, fall between them and
    # lie beyond the last; solid (-1), uninvaded (0) and r2 = 0 voxels
    rng = np.random.default_rng(n_levels)
    shape = (3, 41, 67)
    T = np.sort(rng.choice(np.arange(1, 4 * n_levels + 2), size=n_levels, replace=False))[::-1].astype(np.uint32)
    sat_T = np.sort(rng.uniform(0.0, 1.0, size=n_levels))
    sat_T[rng.integers(0, n_levels, size=n_levels // 3)] = sat_T[0]  # repeated saturations
    sat_T.sort()
    pick = rng.integers(0, n_levels, size=shape)
    sm = np.where(rng.random(shape) < 0.5, sat_T[pick], rng.uniform(0.0, 1.0, size=shape))
    sm[rng.random(shape) < 0.1] = -1.0
    sm[rng.random(shape) < 0.1] = 0.0
    r2 = np.where(rng.random(shape) < 0.5, T[pick], rng.integers(0, 4 * n_levels + 4, size=shape)).astype(np.uint32)
    r2[rng.random(shape) < 0.1] = 0
    tr = (rng.random(shape) < 0.2).astype(np.uint8)
    ref = oracle.compare_opening(sm, r2, T, sat_T, trapped=tr)
    c = ibip.compare_opening(_d(sm, dev), _d(_i32(r2), dev), T.tolist(), sat_T.tolist(), trapped=_d(tr, dev))
    np.testing.assert_array_equal(c["disagree"].cpu().numpy(), ref["disagree"])
    np.testing.assert_array_equal(c["mio_trapped"].cpu().numpy(), ref["mio_trapped"])
    c0 = ibip.compare_opening(_d(sm, dev), _d(_i32(r2), dev), T.tolist(), sat_T.tolist())
    np.testing.assert_array_equal(c0["disagree"].cpu().numpy(), ref["disagree"])
    assert (c0["mio_trapped"].cpu().numpy() == 0).all()


def test_rejects_bad_levels(dev):
    sm = _d(np.zeros((1, 1, 4)), dev)
    r2 = _d(np.zeros((1, 1, 4), np.int32), dev)
    with pytest.raises(ibip.IbipError):
        ibip.compare_opening(sm, r2, [4, 4], [0.1, 0.2])  # radii not decreasing
    with pytest.raises(ibip.IbipError):
        ibip.compare_opening(sm, r2, [4, 1], [0.3, 0.2])  # saturations decreasing
    with pytest.raises(ibip.IbipError):
        ibip.compare_opening(sm, r2, [4, 0], [0.1, 0.2])  # radius zero


def _image(kind):
    if kind == "noise":
        return synth.blurred_noise((1, 500, 500), sigma=4.0, porosity=0.6, seed=11)
    return synth.overlapping_spheres((1, 500, 500), r2=144, porosity=0.6, seed=12)


@pytest.mark.parametrize("kind", ["noise", "disks"])
@pytest.mark.parametrize("integer_ball", [False, True])
def test_validation_2d(dev, kind, integer_ball):
    """The Figure 8/9 pipeline on a 500 x 500 image with a resolution of one
    pixel: IBIP from the left edge, its saturation map, the opening at the
    squared radii of IBIP's own steps, trapping against the right edge, and
    the per-level comparison -- every stage against the oracle."""
    img = _image(kind)
    inl = synth.face_mask(img.shape, axis=1, index=0)
    out = synth.face_mask(img.shape, axis=1, index=img.shape[1] - 1)
    ro = oracle.invade(img, inl, integer_ball=integer_ball)
    so = oracle.steps(ro["seq"], ro["M"])
    mo = oracle.satmap(ro["seq"], so["sat"])
    T = np.unique(ro["M"])[::-1].astype(np.uint32)
    T = T[T >= 1]
    po = oracle.mio(img, inl, T)
    to = oracle.trap(ro["seq"], out)
    ref = oracle.compare_opening(mo, po["mio_r2"], T, po["mio_sat"], trapped=to["trapped"])

    r = ibip.invade(_d(img, dev), _d(inl, dev), integer_ball=integer_ball)
    np.testing.assert_array_equal(r["seq"].cpu().numpy(), ro["seq"])
    s = ibip.saturation(r["seq"], r["M"])
    np.testing.assert_array_equal(s["satmap"].cpu().numpy(), mo)
    p = ibip.opening_drainage(_d(img, dev), _d(inl, dev), T.tolist())
    np.testing.assert_array_equal(p["mio_r2"].cpu().numpy().view(np.uint32), po["mio_r2"])
    np.testing.assert_array_equal(np.asarray(p["mio_sat"]), po["mio_sat"])
    t = ibip.trap(r["seq"], _d(out, dev), seq_trapped=False)
    np.testing.assert_array_equal(t["trapped"].cpu().numpy(), to["trapped"])
    c = ibip.compare_opening(s["satmap"], p["mio_r2"], T.tolist(), p["mio_sat"], trapped=t["trapped"])
    np.testing.assert_array_equal(c["disagree"].cpu().numpy(), ref["disagree"])
    np.testing.assert_array_equal(c["mio_trapped"].cpu().numpy(), ref["mio_trapped"])
    # both methods end on the same pixels: at the smallest level (a ball of
    # one voxel) the opening holds every inlet-connected pore pixel, which is
    # what IBIP has invaded when it stops (the bound on the levels before is
    # pinned on the oracle alone, with its decomposition)
    n_pore = int(img.sum())
    assert T[-1] == 1 and ref["disagree"][-1] == 0
    print(f"{kind} integer_ball={integer_ball}: levels {len(T)}, max disagreement {int(ref['disagree'].max())} "
          f"of {n_pore} pore pixels, opening pixels left trapped by IBIP up to {int(ref['mio_trapped'].max())}")
