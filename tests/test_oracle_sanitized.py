"""The oracle built with AddressSanitizer and UndefinedBehaviourSanitizer runs
every entry point on small images (2D and 3D, every variant reading, the
error paths) without a memory error or undefined behaviour. The sanitized
library runs in a child process with the sanitizer runtime preloaded."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, ROOT)
import numpy as np
import oracle
from paper_2101_03240_amd import synth
rng = np.random.default_rng(0)
cases = [synth.overlapping_spheres((12, 10, 14), r2=4, porosity=0.6, seed=1),
         synth.overlapping_spheres((1, 17, 23), r2=9, porosity=0.55, seed=2),
         (rng.random((5, 1, 9)) < 0.7).astype(np.uint8), np.zeros((3, 4, 5), np.uint8)]
for img in cases:
    if img.any():
        img.flat[0] = 0
    inl = synth.face_mask(img.shape, 2, 0)
    out = synth.face_mask(img.shape, 2, img.shape[2] - 1)
    d = oracle.edt(img)
    assert (d == oracle.edt_brute(img)).all()
    assert oracle.edt_at(img, 0, 0, 0) == d[0, 0, 0]
    for lit in (False, True):
        for ib in (False, True):
            for mk in (False, True):
                r = oracle.invade(img, inl, literal=lit, integer_ball=ib, mask_inlets=mk)
                r2 = oracle.invade(img, inl, max_steps=2, literal=lit, integer_ball=ib, mask_inlets=mk)
    s = oracle.steps(r["seq"], r["M"])
    oracle.satmap(r["seq"], s["sat"])
    for conn in (6, 26):
        t = oracle.trap(r["seq"], out, conn=conn)
        assert (t["trapped"] == oracle.trap_brute(r["seq"], out, conn=conn)).all()
    st, ka = oracle.rerank(r["seq"], t["trapped"])
    oracle.remap_steps(r["seq"], t["seq_trapped"], r["M"], t["K_after"])
    T = np.array([9, 5, 2, 1], np.uint32)
    for be in (False, True):
        for mk in (False, True):
            oracle.mio(img, inl, T, brute_erosion=be, mask_inlets=mk)
    oracle.mio_kept(img, inl, d, 2)
# the error paths
try:
    oracle.invade(np.ones((4, 4, 4), np.uint8), synth.face_mask((4, 4, 4), 0, 0))
except oracle.OracleError:
    pass
print("sanitized oracle ok")
"""


def test_oracle_under_asan_and_ubsan():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime")
    with tempfile.TemporaryDirectory() as tmp:
        lib = oracle.build_sanitized(os.path.join(tmp, "libibip_oracle_asan.so"))
        env = dict(os.environ, IBIP_ORACLE_LIB=lib, LD_PRELOAD=asan,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([sys.executable, "-c", SCRIPT.replace("ROOT", repr(ROOT))], env=env, capture_output=True,
                           text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
