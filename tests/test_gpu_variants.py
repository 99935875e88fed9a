"""Variant readings on the GPU against the oracle's: footnote 1's integer
sphere rule, inlet masking (invasion and opening seeds), 26-connected
trapping."""
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


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _case(seed, solid_inlets=False):
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in rng.integers(5, 40, size=3))
    if seed % 4 == 0:
        shape = (1,) + shape[1:]
    if seed % 2:
        img = synth.overlapping_spheres(shape, r2=int(rng.integers(3, 20)), porosity=float(rng.uniform(0.5, 0.8)),
                                        seed=seed)
    else:
        img = (rng.random(shape) < rng.uniform(0.6, 0.95)).astype(np.uint8)
    if img.all():
        img.flat[0] = 0
    if solid_inlets:
        inl = (rng.random(shape) < 0.05).astype(np.uint8)
    else:
        inl = synth.face_mask(shape, int(rng.integers(3)), 0)
    return img, inl


def _same_as_oracle(g, r):
    assert g["K"] == r["K"]
    np.testing.assert_array_equal(g["seq"].cpu().numpy(), r["seq"])
    np.testing.assert_array_equal(_u32(g["rad2"]), r["rad2"])
    np.testing.assert_array_equal(g["centre_step"].cpu().numpy(), r["centre_step"])
    np.testing.assert_array_equal(_u32(g["M"]), r["M"])


@pytest.mark.parametrize("seed", range(8))
def test_integer_ball(dev, seed):
    img, inl = _case(seed)
    g = ibip.invade(_d(img, dev), _d(inl, dev), integer_ball=True)
    _same_as_oracle(g, oracle.invade(img, inl, integer_ball=True))


def test_integer_ball_fixture(dev):
    img = np.ones((5, 5, 5), np.uint8)
    for x in (1, 3):
        for y in (1, 3):
            for z in (1, 3):
                img[x, y, z] = 0
    inl = np.zeros_like(img)
    inl[2, 2, 2] = 1
    s = ibip.invade(_d(img, dev), _d(inl, dev), max_steps=1)
    i = ibip.invade(_d(img, dev), _d(inl, dev), max_steps=1, integer_ball=True)
    assert int((s["seq"] == 1).sum()) == 19 and int((i["seq"] == 1).sum()) == 7


@pytest.mark.parametrize("seed", range(8))
def test_mask_inlets(dev, seed):
    img, inl = _case(seed + 10, solid_inlets=True)
    g = ibip.invade(_d(img, dev), _d(inl, dev), mask_inlets=True)
    _same_as_oracle(g, oracle.invade(img, inl, mask_inlets=True))
    dt2 = oracle.edt(img)
    vals = sorted(set(int(v) for v in dt2[dt2 > 0]), reverse=True)[:6]
    T = [v for v in vals if v >= 1]
    m = ibip.opening_drainage(_d(img, dev), _d(inl, dev), T, mask_inlets=True)
    r = oracle.mio(img, inl, np.array(T, np.uint32), mask_inlets=True)
    np.testing.assert_array_equal(_u32(m["mio_r2"]), r["mio_r2"])
    np.testing.assert_array_equal(np.array(m["mio_sat"]), r["mio_sat"])


def test_mask_inlets_fixture(dev):
    img = np.array([[[0, 1, 1, 1, 0]]], np.uint8)
    inl = np.array([[[1, 0, 0, 0, 0]]], np.uint8)
    assert ibip.invade(_d(img, dev), _d(inl, dev))["K"] >= 1
    g = ibip.invade(_d(img, dev), _d(inl, dev), mask_inlets=True)
    assert g["K"] == 0
    np.testing.assert_array_equal(g["seq"].cpu().numpy(), np.where(img > 0, 0, -1))


def test_trap26_fixture(dev):
    gd = _golden.load("trap_2d_diagonal.txt")
    seq = _golden.as_volume(gd["seq"]).astype(np.int32)
    out = _golden.as_volume(gd["outlets"]).astype(np.uint8)
    t6 = ibip.trap(_d(seq, dev), _d(out, dev))
    t26 = ibip.trap(_d(seq, dev), _d(out, dev), connectivity=26)
    np.testing.assert_array_equal(t6["trapped"].cpu().numpy(), _golden.as_volume(gd["trapped6"]))
    np.testing.assert_array_equal(t26["trapped"].cpu().numpy(), _golden.as_volume(gd["trapped26"]))


@pytest.mark.parametrize("seed", range(8))
def test_trap26(dev, seed):
    img, inl = _case(seed + 20)
    r = oracle.invade(img, inl)
    out = synth.face_mask(img.shape, 0, img.shape[0] - 1)
    t = ibip.trap(_d(r["seq"], dev), _d(out, dev), connectivity=26)
    o = oracle.trap(r["seq"], out, conn=26)
    np.testing.assert_array_equal(t["trapped"].cpu().numpy(), o["trapped"])
    np.testing.assert_array_equal(t["seq_trapped"].cpu().numpy(), o["seq_trapped"])
    assert t["K_after"] == o["K_after"]


@pytest.mark.timeout(300)
def test_trap26_packing200(dev):
    img = synth.config_image("packing200")
    inl = synth.face_mask(img.shape, 0, 0)
    out = synth.face_mask(img.shape, 0, img.shape[0] - 1)
    g = ibip.invade(_d(img, dev), _d(inl, dev))
    t = ibip.trap(g["seq"], _d(out, dev), connectivity=26)
    o = oracle.trap(g["seq"].cpu().numpy(), out, conn=26)
    np.testing.assert_array_equal(t["trapped"].cpu().numpy(), o["trapped"])
    np.testing.assert_array_equal(t["seq_trapped"].cpu().numpy(), o["seq_trapped"])


def test_readings_do_not_leak(dev):
    img, inl = _case(3, solid_inlets=True)
    a = ibip.invade(_d(img, dev), _d(inl, dev))
    ibip.invade(_d(img, dev), _d(inl, dev), integer_ball=True, mask_inlets=True)
    b = ibip.invade(_d(img, dev), _d(inl, dev))
    assert torch.equal(a["seq"], b["seq"])
    _same_as_oracle(b, oracle.invade(img, inl))
