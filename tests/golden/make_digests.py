"""Writes the oracle's digests of the full-size workloads to tests/golden/.

The CPU oracle needs minutes per 512^3 image, too long for a GPU test, so its
results at the benchmark sizes are computed here once and stored as digests:
SHA-256 of every output array, plus a short hash of each x-slab of the
per-voxel arrays so that a mismatch can be located. Only ``oracle`` (the
results) and ``paper_2101_03240_amd.synth`` (the seeded inputs, whose own
SHA-256 is stored too) are used.

    python tests/golden/make_digests.py noise512   # 512^3 blurred noise
    python tests/golden/make_digests.py serve515   # the smallest serving request above 512 voxels a side
    python tests/golden/make_digests.py batch96    # the 96 images of the uneven batch

Per case: the invasion (seq, rad2, centre_step, M, n_new, sat; Section 2.1,
Sections 2.2.1-2.2.2) from the inlet face x = 0 and the trapping with
re-ranking (trapped, seq_trapped; Section 2.2.3) against the outlet face
x = L - 1.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2101_03240_amd import synth  # noqa: E402

VOXEL_ARRAYS = ("seq", "rad2", "centre_step", "trapped", "seq_trapped")
STEP_ARRAYS = ("M", "n_new", "sat")


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def slab_hashes(a: np.ndarray) -> str:
    """8 hex digits (BLAKE2b, 4 bytes) per x-slab, concatenated."""
    a = np.ascontiguousarray(a)
    return "".join(hashlib.blake2b(a[x].tobytes(), digest_size=4).hexdigest() for x in range(a.shape[0]))


def serve_case():
    """The smallest request of the 256-request serving stream whose side
    exceeds 512 (lines longer than the EDT's LDS tiles), generated on the host."""
    specs = synth.serve_specs(256)
    j = min((s.L, j) for j, s in enumerate(specs) if s.L > 512)[1]
    return j, specs[j]


def image_of(case: str, i: int = 0) -> tuple[np.ndarray, str]:
    if case == "noise512":
        return synth.config_image("noise512"), "synth.config_image('noise512')"
    if case == "serve515":
        j, s = serve_case()
        return (synth.blurred_noise((s.L,) * 3, sigma=s.sigma, porosity=s.porosity, seed=s.seed),
                f"synth.blurred_noise(({s.L},)*3, sigma={s.sigma}, porosity=serve_specs(256)[{j}].porosity, "
                f"seed={s.seed})")
    if case == "batch96":
        return synth.image_for_spec(synth.batch_specs(96)[i]), f"synth.image_for_spec(synth.batch_specs(96)[{i}])"
    raise ValueError(case)


def digest_one(img: np.ndarray, slabs=VOXEL_ARRAYS) -> dict:
    L = img.shape[0]
    inl = synth.face_mask(img.shape, 0, 0)
    out = synth.face_mask(img.shape, 0, L - 1)
    r = oracle.invade(img, inl)
    s = oracle.steps(r["seq"], r["M"])
    t = oracle.trap(r["seq"], out)
    arrays = {"seq": r["seq"], "rad2": r["rad2"], "centre_step": r["centre_step"],
              "trapped": t["trapped"], "seq_trapped": t["seq_trapped"]}
    d = {"shape": list(img.shape), "image_sha256": sha(img), "K": int(r["K"]), "K_after": int(t["K_after"]),
         "invaded": int((r["seq"] > 0).sum()), "n_trapped": int(t["trapped"].sum()),
         "pore": int((img > 0).sum()), "arrays": {}, "steps": {}}
    for name, a in arrays.items():
        e = {"dtype": str(a.dtype), "sha256": sha(a)}
        if name in slabs:
            e["slabs"] = slab_hashes(a)
        d["arrays"][name] = e
    steps = {"M": r["M"], "n_new": s["n_new"], "sat": s["sat"]}
    for name, a in steps.items():
        d["steps"][name] = {"dtype": str(a.dtype), "sha256": sha(a)}
    return d


def _batch_item(i: int) -> dict:
    img, recipe = image_of("batch96", i)
    d = digest_one(img, slabs=("seq", "trapped"))
    d["recipe"] = recipe
    return d


def main(case: str) -> None:
    t0 = time.time()
    if case == "batch96":
        with cf.ProcessPoolExecutor(max_workers=int(os.environ.get("DIGEST_WORKERS", "4"))) as ex:
            items = list(ex.map(_batch_item, range(96)))
        doc = {"case": case, "inlets": "face x = 0", "outlets": "face x = L - 1", "images": items}
    else:
        img, recipe = image_of(case)
        doc = {"case": case, "inlets": "face x = 0", "outlets": "face x = L - 1", "recipe": recipe,
               **digest_one(img)}
    doc["oracle_seconds"] = round(time.time() - t0, 1)
    path = os.path.join(HERE, f"digests_{case}.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print("wrote", path, f"in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    for c in sys.argv[1:] or ["noise512", "serve515", "batch96"]:
        main(c)
