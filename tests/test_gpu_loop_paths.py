"""GPU parity of the step loop's forms (Section 2.1), bit for bit against the
oracle, on images built so that every step has a chosen number of centres.

A flat channel one voxel thick (solid above and below in z) has the same
distance value, 1, at every pore voxel, so from an inlet column the invasion
floods one column per step: after the first step (the inlet column and the
next, both seeds) every step pops exactly `width` centres, all of them pushed
by the step before. Widths around 10/11, 21/22, 64/65 and
128/129 take the wave-0 run with one and two passes of (centre, direction)
pairs, the wave-0 steps of three or more passes, and the steps run by all
waves. A long tube of constant radius gives long runs whose centres each
step lists for the next, and step limits that land inside such a run.
"""
import numpy as np
import pytest

import oracle
from paper_2101_03240_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ibip = pytest.importorskip("paper_2101_03240_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _check(img, inl, dev, max_steps=0):
    g = ibip.invade(torch.from_numpy(img).to(dev), torch.from_numpy(inl).to(dev), max_steps=max_steps)
    r = oracle.invade(img, inl, max_steps=max_steps)
    assert g["K"] == r["K"]
    np.testing.assert_array_equal(g["seq"].cpu().numpy(), r["seq"])
    np.testing.assert_array_equal(g["rad2"].cpu().numpy().view(np.uint32), r["rad2"])
    np.testing.assert_array_equal(g["centre_step"].cpu().numpy(), r["centre_step"])
    np.testing.assert_array_equal(g["M"].cpu().numpy().view(np.uint32), r["M"])
    return r


def _channel(width, length=40):
    img = np.zeros((length, width + 2, 3), np.uint8)
    img[:, 1:width + 1, 1] = 1
    return img


@pytest.mark.parametrize("width", [1, 10, 11, 21, 22, 64, 65, 128, 129, 300])
def test_steps_of_fixed_size(dev, width):
    img = _channel(width)
    inl = synth.face_mask(img.shape, 0, 0)
    r = _check(img, inl, dev)
    # the first step pops the inlet column and the next (both seeds), every
    # later step one column
    cs = r["centre_step"][:, 1:width + 1, 1]
    assert r["K"] == img.shape[0] - 1
    assert all(np.unique(cs[x]).tolist() == [max(x, 1)] for x in range(img.shape[0]))


@pytest.mark.parametrize("max_steps", [1, 2, 37, 1023, 1024, 1025])
def test_step_limit_inside_a_run(dev, max_steps):
    # a tube of radius 2 along x: the flood runs at one distance value
    X, Y, Z = 1500, 7, 7
    v = np.indices((Y, Z))
    disk = (v[0] - 3) ** 2 + (v[1] - 3) ** 2 <= 4
    img = np.zeros((X, Y, Z), np.uint8)
    img[:, disk] = 1
    inl = synth.face_mask(img.shape, 0, 0)
    _check(img, inl, dev, max_steps=max_steps)


def test_descending_chambers(dev):
    # chambers of decreasing radius joined by throats, entered from the
    # largest: after each chamber the maximum falls to older, lower slices
    X, Y, Z = 120, 25, 25
    v = np.indices((X, Y, Z))
    pore = np.zeros((X, Y, Z), bool)
    cx = 10
    for rad in (10, 8, 7, 5, 4, 3):
        pore |= (v[0] - cx) ** 2 + (v[1] - 12) ** 2 + (v[2] - 12) ** 2 <= rad * rad
        nxt = cx + rad + 2
        pore[cx:nxt + 1, 11:14, 11:14] = True  # throat to the next chamber
        cx = nxt + (rad - 1)
    img = pore.astype(np.uint8)
    inl = np.zeros_like(img)
    inl[10, 12, 12] = 1
    _check(img, inl, dev)


def test_batch_of_fixed_size_steps(dev):
    # the same channels in one batched call: every job's loop in its own workgroup
    widths = [1, 10, 11, 21, 22, 64, 65, 128, 129]
    imgs = [_channel(w, length=30 + 3 * i) for i, w in enumerate(widths)]
    inls = [synth.face_mask(im.shape, 0, 0) for im in imgs]
    res = ibip.invade_batch([torch.from_numpy(im).to(dev) for im in imgs],
                            [torch.from_numpy(i).to(dev) for i in inls])
    for im, inl, g in zip(imgs, inls, res):
        r = oracle.invade(im, inl)
        assert g["K"] == r["K"]
        np.testing.assert_array_equal(g["seq"].cpu().numpy(), r["seq"])
        np.testing.assert_array_equal(g["centre_step"].cpu().numpy(), r["centre_step"])
        np.testing.assert_array_equal(g["M"].cpu().numpy().view(np.uint32), r["M"])
