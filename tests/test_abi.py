"""The C ABI library loads and exports every function include/*.h declares
(no GPU needed: nothing is called)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2101_03240_amd import library_path

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(ibip_\w+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary_calls():
    d = _declared()
    for name in ("ibip_edt", "ibip_invade", "ibip_get_steps", "ibip_trap", "ibip_opening_drainage",
                 "ibip_ctx_create", "ibip_ctx_destroy", "ibip_last_error"):
        assert name in d


def test_library_exports_every_declared_symbol():
    if not os.path.exists(library_path()):
        pytest.fail("libibip_hip.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(library_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
