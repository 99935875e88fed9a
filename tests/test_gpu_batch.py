"""Batches of uneven images give exactly the per-image results (the batch
pattern of the invasion loop: one launch runs every job's step loop)."""
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


def _d(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _jobs(seed, n):
    rng = np.random.default_rng(seed)
    imgs, inls = [], []
    for i in range(n):
        shape = tuple(int(s) for s in rng.integers(4, 48, size=3))
        if i % 5 == 0:
            shape = (1,) + shape[1:]
        kind = i % 3
        if kind == 0:
            img = synth.overlapping_spheres(shape, r2=int(rng.integers(2, 20)), porosity=float(rng.uniform(0.5, 0.8)),
                                            seed=i)
        elif kind == 1 and min(shape) >= 8:
            img = synth.blurred_noise(shape, sigma=2.0, porosity=float(rng.uniform(0.4, 0.7)), seed=i)
        else:
            img = (rng.random(shape) < 0.7).astype(np.uint8)
        if img.all():
            img.flat[0] = 0
        inl = synth.face_mask(shape, int(rng.integers(3)), 0)
        imgs.append(img)
        inls.append(inl)
    return imgs, inls


@pytest.mark.parametrize("seed", [0, 1])
def test_batch_equals_single_runs(dev, seed):
    imgs, inls = _jobs(seed, 23)
    out = ibip.invade_batch([_d(a, dev) for a in imgs], [_d(a, dev) for a in inls], sat=True)
    for img, inl, b in zip(imgs, inls, out):
        s = ibip.invade(_d(img, dev), _d(inl, dev))
        assert b["status"] == 0
        assert b["K"] == s["K"]
        assert torch.equal(b["seq"], s["seq"])
        assert torch.equal(b["rad2"], s["rad2"])
        assert torch.equal(b["centre_step"], s["centre_step"])
        assert torch.equal(b["M"], s["M"])
        assert torch.equal(b["sat"], s["sat"])


def test_batch_against_oracle(dev):
    imgs, inls = _jobs(7, 9)
    out = ibip.invade_batch([_d(a, dev) for a in imgs], [_d(a, dev) for a in inls])
    for img, inl, b in zip(imgs, inls, out):
        r = oracle.invade(img, inl)
        assert b["K"] == r["K"]
        np.testing.assert_array_equal(b["seq"].cpu().numpy(), r["seq"])
        np.testing.assert_array_equal(b["M"].cpu().numpy().view(np.uint32), r["M"])


def test_batch_failed_job_and_step_limits(dev):
    imgs, inls = _jobs(3, 6)
    imgs.insert(2, np.ones((9, 9, 9), np.uint8))  # no solid
    inls.insert(2, synth.face_mask((9, 9, 9)))
    limits = [0, 5, 0, 17, 0, 1, 3]
    out = ibip.invade_batch([_d(a, dev) for a in imgs], [_d(a, dev) for a in inls], max_steps=limits,
                            raise_on_error=False)
    assert out[2]["status"] == -3
    for i, (img, inl, b) in enumerate(zip(imgs, inls, out)):
        if i == 2:
            continue
        assert b["status"] == 0
        r = oracle.invade(img, inl, max_steps=limits[i])
        assert b["K"] == r["K"]
        np.testing.assert_array_equal(b["seq"].cpu().numpy(), r["seq"])
    with pytest.raises(ibip.IbipError):
        ibip.invade_batch([_d(a, dev) for a in imgs], [_d(a, dev) for a in inls])
