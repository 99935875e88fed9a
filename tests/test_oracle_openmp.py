"""The oracle built with OpenMP (the benchmark's data-parallel CPU baseline:
the distance transform's lines and the x-planes of large spheres split over
threads) gives exactly the plain build's results. It runs in a child process
with 4 threads; the plain results come from this process."""
import json
import os
import subprocess
import sys
import tempfile

import numpy as np

import oracle
from paper_2101_03240_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import hashlib, json, sys
sys.path.insert(0, ROOT)
import numpy as np
import oracle
from tests.test_oracle_openmp import cases
out = {"threads": oracle.threads(), "digests": []}
for img, inl, outl in cases():
    r = oracle.invade(img, inl)
    t = oracle.trap(r["seq"], outl)
    arrs = [oracle.edt(img), r["seq"], r["rad2"], r["centre_step"], r["M"], t["trapped"], t["seq_trapped"]]
    out["digests"].append([hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest() for a in arrs])
print(json.dumps(out))
"""


def cases():
    """Images with spheres large enough (radius >= 8) for the threaded insertion."""
    v = np.indices((40, 44, 48))
    ball = ((v[0] - 20) ** 2 + (v[1] - 22) ** 2 + (v[2] - 24) ** 2 < 17 ** 2)
    chan = (v[0] < 20) & ((v[1] - 22) ** 2 + (v[2] - 24) ** 2 < 9)
    imgs = [(ball | chan).astype(np.uint8),
            synth.overlapping_spheres((30, 26, 34), r2=9, porosity=0.7, seed=4),
            synth.blurred_noise((1, 90, 70), sigma=5.0, porosity=0.6, seed=5)]
    for img in imgs:
        img.flat[0] = 0
        yield img, synth.face_mask(img.shape, 0, 0) if img.shape[0] > 1 else synth.face_mask(img.shape, 1, 0), \
            synth.face_mask(img.shape, 0, img.shape[0] - 1) if img.shape[0] > 1 else \
            synth.face_mask(img.shape, 1, img.shape[1] - 1)


def test_openmp_build_equals_plain_build():
    import hashlib
    want = []
    mmax = 0
    for img, inl, outl in cases():
        r = oracle.invade(img, inl)
        mmax = max(mmax, int(r["M"].max()))
        t = oracle.trap(r["seq"], outl)
        arrs = [oracle.edt(img), r["seq"], r["rad2"], r["centre_step"], r["M"], t["trapped"], t["seq_trapped"]]
        want.append([hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest() for a in arrs])
    assert mmax >= 64  # some sphere takes the threaded insertion (radius >= 8)
    with tempfile.TemporaryDirectory() as tmp:
        lib = oracle.build_openmp(os.path.join(tmp, "libibip_oracle_omp.so"))
        env = dict(os.environ, IBIP_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
        p = subprocess.run([sys.executable, "-c", SCRIPT.replace("ROOT", repr(ROOT))], env=env, capture_output=True,
                           text=True, timeout=600, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-4000:]
    got = json.loads(p.stdout.strip().splitlines()[-1])
    assert got["threads"] == 4
    assert got["digests"] == want
