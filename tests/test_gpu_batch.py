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


@pytest.mark.skip(reason="the persistent batch launch with shared wide steps that this test was written for hung "
                         "on the GPU twice (its first batch call never returned) and its code path was taken out; "
                         "the launch parameters it passes no longer exist")
@pytest.mark.parametrize("tuning", [
    {"batch_wide": 128, "batch_workgroups": 0, "batch_chunk_rounds": 1},
    {"batch_wide": 128, "batch_workgroups": 5, "batch_chunk_rounds": 2},
    {"batch_wide": 300, "batch_workgroups": 2, "batch_chunk_rounds": 1},
    {"batch_wide": 128, "batch_workgroups": 40, "batch_chunk_rounds": 3},
])
def test_batch_shared_wide_steps(dev, tuning):
    """Steps above a low threshold run as shared wide steps (the job's
    workgroup with the workgroups that have no job left, in chunks of 1024
    to 3072 centres); fewer workgroups than jobs make workgroups take several
    jobs one after the other. Every result equals the oracle; a job without
    solid fails alone and a step limit holds."""
    rng = np.random.default_rng(7)
    imgs, inls, lims = [], [], []
    for i in range(9):
        L = int(rng.integers(40, 90))
        if i % 2:
            img = synth.blurred_noise((L, L + 3, L - 5), sigma=3.0, porosity=0.6, seed=50 + i)
        else:
            img = synth.overlapping_spheres((L, L - 2, L + 4), r2=16, porosity=0.65, seed=50 + i)
        imgs.append(img)
        inls.append(synth.face_mask(img.shape, 0, 0))
        lims.append(0 if i != 4 else 57)
    imgs.append(np.ones((20, 20, 24), np.uint8))  # no solid: ENOSOLID
    inls.append(synth.face_mask(imgs[-1].shape, 0, 0))
    lims.append(0)
    out = ibip.invade_batch([_d(a, dev) for a in imgs], [_d(a, dev) for a in inls], max_steps=lims,
                            raise_on_error=False, tuning=tuning)
    assert out[-1]["status"] == -3
    for img, inl, lim, b in zip(imgs[:-1], inls[:-1], lims[:-1], out[:-1]):
        r = oracle.invade(img, inl, max_steps=lim)
        assert b["status"] == 0
        assert b["K"] == r["K"]
        np.testing.assert_array_equal(b["seq"].cpu().numpy(), r["seq"])
        np.testing.assert_array_equal(b["rad2"].cpu().numpy().view(np.uint32), r["rad2"])
        np.testing.assert_array_equal(b["centre_step"].cpu().numpy(), r["centre_step"])
        np.testing.assert_array_equal(b["M"].cpu().numpy().view(np.uint32), r["M"])
    # the context's own tuning is back to what it was
    assert ibip.get_tuning() == {"batch_wide": 0, "batch_workgroups": 0, "batch_chunk_rounds": 0}


def _wide_jobs():
    rng = np.random.default_rng(7)
    imgs, inls, lims = [], [], []
    for i in range(9):
        L = int(rng.integers(40, 90))
        if i % 2:
            img = synth.blurred_noise((L, L + 3, L - 5), sigma=3.0, porosity=0.6, seed=50 + i)
        else:
            img = synth.overlapping_spheres((L, L - 2, L + 4), r2=16, porosity=0.65, seed=50 + i)
        imgs.append(img)
        inls.append(synth.face_mask(img.shape, 0, 0))
        lims.append(0 if i != 4 else 57)
    return imgs, inls, lims


@pytest.mark.parametrize("tuning", [
    {"batch_wide": 128},
    {"batch_wide": 300, "edt_tile_y": 64, "edt_tile_x": 16},
    {"batch_wide": 2000, "edt_tile_y": 64},
    {"batch_wide": -1, "edt_tile_x": 16},
])
def test_batch_continued_wide_steps(dev, tuning):
    """A job's step above the threshold stops its loop in the batched launch;
    the host runs that step over the whole GPU and the job's loop continues
    in launches of its own, stopping again at every later such step (a low
    threshold makes that happen hundreds of times per job). Every result
    equals the oracle; a job without solid fails alone; a step limit holds;
    the EDT tile widths change nothing."""
    imgs, inls, lims = _wide_jobs()
    imgs.append(np.ones((20, 20, 24), np.uint8))  # no solid: ENOSOLID
    inls.append(synth.face_mask(imgs[-1].shape, 0, 0))
    lims.append(0)
    print("batch tuning", tuning, flush=True)
    before = ibip.get_tuning()
    out = ibip.invade_batch([_d(a, dev) for a in imgs], [_d(a, dev) for a in inls], max_steps=lims,
                            raise_on_error=False, tuning=tuning)
    assert out[-1]["status"] == -3
    for img, inl, lim, b in zip(imgs[:-1], inls[:-1], lims[:-1], out[:-1]):
        r = oracle.invade(img, inl, max_steps=lim)
        assert b["status"] == 0
        assert b["K"] == r["K"]
        np.testing.assert_array_equal(b["seq"].cpu().numpy(), r["seq"])
        np.testing.assert_array_equal(b["rad2"].cpu().numpy().view(np.uint32), r["rad2"])
        np.testing.assert_array_equal(b["centre_step"].cpu().numpy(), r["centre_step"])
        np.testing.assert_array_equal(b["M"].cpu().numpy().view(np.uint32), r["M"])
    # the context's own tuning is back to what it was
    assert ibip.get_tuning() == before


def test_tuning_rejects_unknown_tile_widths(dev):
    ibip.set_tuning({"edt_tile_y": 64, "edt_tile_x": 16, "batch_wide": 5})
    with pytest.raises(ibip.IbipError):
        ibip.set_tuning({"edt_tile_y": 48})
    with pytest.raises(ibip.IbipError):
        ibip.set_tuning({"edt_tile_x": 64})
    assert ibip.get_tuning() == {"edt_tile_y": 64, "edt_tile_x": 16, "batch_wide": 5}
    ibip.set_tuning(None)
    assert ibip.get_tuning() == {"edt_tile_y": 0, "edt_tile_x": 0, "batch_wide": 0}


def test_setup_graph_replays(dev):
    """The batch's setup is captured into graphs (one per batch stream) for
    its buffers and replayed while the same batch comes back: A (9 jobs)
    twice (a capture, then a replay), a single-image call, B (5 jobs, fewer
    than the streams) twice, three rounds, every result equal
    to the single runs; then new contents in A's input buffers, which a
    capture and a replay of A must both read."""
    imgs_a, inls_a = _jobs(11, 9)
    imgs_b, inls_b = _jobs(12, 5)
    da = [_d(a, dev) for a in imgs_a]
    ia = [_d(a, dev) for a in inls_a]
    db = [_d(a, dev) for a in imgs_b]
    ib = [_d(a, dev) for a in inls_b]
    want_a = [ibip.invade(x, y) for x, y in zip(da, ia)]
    want_b = [ibip.invade(x, y) for x, y in zip(db, ib)]

    def check(out, want):
        for b, s in zip(out, want):
            assert b["status"] == 0 and b["K"] == s["K"]
            assert torch.equal(b["seq"], s["seq"]) and torch.equal(b["rad2"], s["rad2"])
            assert torch.equal(b["centre_step"], s["centre_step"]) and torch.equal(b["M"], s["M"])

    for rnd in range(3):
        check(ibip.invade_batch(da, ia), want_a)  # a capture
        check(ibip.invade_batch(da, ia), want_a)  # a replay
        ibip.invade(da[0], ia[0])
        torch.cuda.synchronize()
        check(ibip.invade_batch(db, ib), want_b)
        check(ibip.invade_batch(db, ib), want_b)
    # the same buffers with new contents: the replay reads them
    flip = [torch.from_numpy(np.flip(a, axis=-1).copy()).to(dev) for a in imgs_a]
    for x, y in zip(da, flip):
        x.copy_(y)
    want_f = [ibip.invade(x, y) for x, y in zip(da, ia)]
    check(ibip.invade_batch(da, ia), want_f)
    check(ibip.invade_batch(da, ia), want_f)
