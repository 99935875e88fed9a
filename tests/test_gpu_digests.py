"""GPU parity at the full benchmark sizes against the oracle's stored digests.

The oracle's results for the 512^3 blurred-noise image, the 96 images of the
uneven batch and the smallest serving request above 512 voxels a side
(515^3, whose lines are longer than the EDT's LDS tiles) were computed on
the CPU by tests/golden/make_digests.py and stored as SHA-256 digests of
every output array plus a short hash per x-slab. Here the same seeded inputs
are generated again (their own SHA-256 is checked first), run through
ibip_invade, ibip_invade_batch and the server in the configurations the
benchmark uses, trapped with ibip_trap, and every output is compared with
the digests: bit for bit (sequence, radii, centres, per-step radii, counts
and saturation; trapped mask, re-ranked sequence), and Pc to 1e-12 relative
against the oracle's formula on the same radii. A mismatch names the array
and the first x-slab that differs.
"""
import concurrent.futures as cf
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_2101_03240_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ibip = pytest.importorskip("paper_2101_03240_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _load(case):
    with open(os.path.join(GOLDEN, f"digests_{case}.json")) as f:
        return json.load(f)


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _slabs(a):
    a = np.ascontiguousarray(a)
    return [hashlib.blake2b(a[x].tobytes(), digest_size=4).hexdigest() for x in range(a.shape[0])]


def _np(t, dtype):
    return np.ascontiguousarray(t.cpu().numpy()).view(dtype)


def _check_array(what, name, got, entry):
    got = np.ascontiguousarray(got).view(np.dtype(entry["dtype"]))
    if _sha(got) == entry["sha256"]:
        return
    msg = f"{what}: {name} differs from the oracle"
    if "slabs" in entry:
        want = [entry["slabs"][8 * i:8 * i + 8] for i in range(len(entry["slabs"]) // 8)]
        have = _slabs(got)
        bad = [x for x in range(len(want)) if want[x] != have[x]]
        if bad:
            msg += f"; first differing x-slab x = {bad[0]} of {len(want)} ({len(bad)} slabs differ)"
    pytest.fail(msg)


def _check_image(what, img, d):
    assert list(img.shape) == d["shape"], (what, img.shape)
    assert synth.sha256(img) == d["image_sha256"], \
        f"{what}: the generator made another image than the one the digests were taken on"


def _check_trap(what, seq_d, L, d, dev):
    out = torch.from_numpy(synth.face_mask(tuple(d["shape"]), 0, L - 1)).to(dev)
    t = ibip.trap(seq_d, out)
    assert t["K_after"] == d["K_after"], (what, t["K_after"], d["K_after"])
    _check_array(what, "trapped", _np(t["trapped"], np.uint8), d["arrays"]["trapped"])
    _check_array(what, "seq_trapped", _np(t["seq_trapped"], np.int32), d["arrays"]["seq_trapped"])


def _check_invade(what, r, d, full_steps=True):
    assert r["K"] == d["K"], (what, r["K"], d["K"])
    seq = _np(r["seq"], np.int32)
    _check_array(what, "seq", seq, d["arrays"]["seq"])
    _check_array(what, "rad2", _np(r["rad2"], np.uint32), d["arrays"]["rad2"])
    _check_array(what, "centre_step", _np(r["centre_step"], np.int32), d["arrays"]["centre_step"])
    M = _np(r["M"], np.uint32)
    _check_array(what, "M", M, d["steps"]["M"])
    if full_steps:
        _check_array(what, "n_new", _np(r["n_new"], np.int64), d["steps"]["n_new"])
        _check_array(what, "sat", _np(r["sat"], np.float64), d["steps"]["sat"])
        # seq and M equal the oracle's, so this is the oracle's Pc
        want = oracle.steps(seq, M, c0=2.0)["pc"]
        np.testing.assert_allclose(_np(r["pc"], np.float64), want, rtol=1e-12, atol=0)
    return seq


@pytest.mark.timeout(600)
def test_noise512_digests(dev):
    d = _load("noise512")
    print("digests: noise512 (512^3 blurred noise) through ibip_invade and ibip_trap", flush=True)
    img = synth.config_image("noise512")
    _check_image("noise512", img, d)
    inl = synth.face_mask(img.shape, 0, 0)
    r = ibip.invade(torch.from_numpy(img).to(dev), torch.from_numpy(inl).to(dev))
    _check_invade("noise512", r, d)
    _check_trap("noise512", r["seq"], img.shape[0], d, dev)


@pytest.mark.timeout(600)
def test_serve515_digests(dev):
    """The serving path (and the plain call) on a 515^3 request: rows of
    Z % 8 != 0 and lines longer than 512 voxels take the EDT's untiled passes."""
    d = _load("serve515")
    specs = synth.serve_specs(256)
    j = min((s.L, j) for j, s in enumerate(specs) if s.L > 512)[1]
    s = specs[j]
    print(f"digests: serving request {j} ({s.L}^3) through the server, ibip_invade and ibip_trap", flush=True)
    img = synth.blurred_noise((s.L,) * 3, sigma=s.sigma, porosity=s.porosity, seed=s.seed)
    _check_image("serve515", img, d)
    img_d = torch.from_numpy(img).to(dev)
    inl_d = torch.from_numpy(synth.face_mask(img.shape, 0, 0)).to(dev)
    with ibip.Server(dev, hbm_budget_bytes=8 << 30, max_inflight=4) as srv:
        r = srv.wait(srv.submit(img_d, inl_d))
        assert r["status"] == 0
        _check_invade("serve515 (server)", r, d, full_steps=False)
    del r
    r = ibip.invade(img_d, inl_d)
    _check_invade("serve515 (ibip_invade)", r, d)
    _check_trap("serve515", r["seq"], s.L, d, dev)


def _batch_image(i):
    return synth.image_for_spec(synth.batch_specs(96)[i])


@pytest.mark.timeout(900)
def test_batch96_digests(dev):
    """All 96 images of the uneven batch (sides 32..192) in one
    ibip_invade_batch call, as the benchmark runs it."""
    d = _load("batch96")
    print("digests: batch96 generating 96 images", flush=True)
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        imgs = list(ex.map(_batch_image, range(96)))
    for i, (img, e) in enumerate(zip(imgs, d["images"])):
        _check_image(f"batch96[{i}]", img, e)
    print("digests: batch96 through ibip_invade_batch", flush=True)
    d_imgs = [torch.from_numpy(a).to(dev) for a in imgs]
    d_inls = [torch.from_numpy(synth.face_mask(a.shape, 0, 0)).to(dev) for a in imgs]
    out = ibip.invade_batch(d_imgs, d_inls)
    for i, (r, e) in enumerate(zip(out, d["images"])):
        assert r["status"] == 0, (i, r["status"])
        _check_invade(f"batch96[{i}]", r, e, full_steps=False)
    print("digests: batch96 trapping", flush=True)
    for i, (r, e) in enumerate(zip(out, d["images"])):
        _check_trap(f"batch96[{i}]", r["seq"], e["shape"][0], e, dev)
