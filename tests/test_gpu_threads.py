"""Calls from two host threads, each on its own stream (each thread gets its
own library context), give the results of the same calls made one after the
other."""
import concurrent.futures as cf

import numpy as np
import pytest

from paper_2101_03240_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ibip = pytest.importorskip("paper_2101_03240_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_two_threads_two_streams(dev):
    a = synth.overlapping_spheres((48, 40, 56), r2=9, porosity=0.7, seed=11)
    b = synth.blurred_noise((40, 48, 64), sigma=3.0, porosity=0.55, seed=12)
    da, db = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    ia = torch.from_numpy(synth.face_mask(a.shape)).to(dev)
    ib = torch.from_numpy(synth.face_mask(b.shape)).to(dev)
    T = [30, 20, 12, 6, 3, 1]
    ref_a = ibip.invade(da, ia)
    ref_b = ibip.opening_drainage(db, ib, T)
    ref_c = ibip.invade(db, ib)
    torch.cuda.synchronize()
    side = torch.cuda.Stream(device=dev)

    def other():
        with torch.cuda.stream(side):
            m = ibip.opening_drainage(db, ib, T)
            c = ibip.invade(db, ib)
            side.synchronize()
            return m, c

    with cf.ThreadPoolExecutor(max_workers=1) as ex:
        for _ in range(3):
            fut = ex.submit(other)
            ra = ibip.invade(da, ia)
            m, c = fut.result()
            torch.cuda.synchronize()
            assert torch.equal(ra["seq"], ref_a["seq"]) and ra["K"] == ref_a["K"]
            assert torch.equal(m["mio_r2"], ref_b["mio_r2"]) and m["mio_sat"] == ref_b["mio_sat"]
            assert torch.equal(c["seq"], ref_c["seq"]) and torch.equal(c["M"], ref_c["M"])

