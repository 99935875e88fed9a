"""Autotuner for the library's launch parameters (``ibip_tuning``).

Results never depend on these parameters, only speed does:

* ``edt_tile_y`` / ``edt_tile_x``: z columns per LDS tile of the exact EDT's
  passes y (32 or 64) and x (16 or 32), chosen per size class of the image
  (largest side up to 96, 256 and 512; longer lines take the untiled passes);
* ``batch_wide``: the step size above which a batch job leaves the batched
  launch and continues with its wide steps over the whole GPU (never, or
  32768 / 131072 / 524288 centres);
* ``serve_wide``: the same threshold for the server's jobs (2048, 8192,
  32768 centres, or never).

``python -m paper_2101_03240_amd.autotune`` times every candidate on seeded
synthetic images of each class on the current GPU (HIP-event kernel time for
the EDT, wall time for the batch and the server) and writes the fastest to
``tuning_cache.json`` beside this file, with every measured time. Each
parameter keeps the library's default (the first candidate) unless another
is faster by more than a margin: ``MARGIN`` for the batch and the server,
whose wall times vary by a few per cent from run to run, ``MARGIN_EDT`` for
the EDT's kernel times; a choice inside that spread is not a gain. The
binding applies the cached choice of an image's size class to each call when
the cache was written on the same GPU architecture.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")

CLASSES = (("small", 96), ("medium", 256), ("large", 512), ("xlarge", 1 << 30))
EDT_TILES = [(32, 32), (32, 16), (64, 32), (64, 16)]
BATCH_WIDE = [-1, 32768, 131072, 524288]
SERVE_WIDE = [8192, 2048, 32768, -1]
MARGIN = 0.05
MARGIN_EDT = 0.02


def pick(times: dict, default: str, margin: float = 0.0) -> str:
    """The fastest candidate, or `default` unless the fastest beats it by more
    than `margin` (a fraction of the default's time)."""
    best = min(times, key=times.get)
    return best if times[best] < (1.0 - margin) * times[default] else default


def size_class(shape) -> str:
    m = max(int(x) for x in shape)
    for name, top in CLASSES:
        if m <= top:
            return name
    return CLASSES[-1][0]


def _log(*a):
    print("autotune:", *a, file=sys.stderr, flush=True)


def tune_edt(dev, reps: int = 20) -> dict:
    import torch

    import paper_2101_03240_amd as ibip
    from paper_2101_03240_amd import synth

    sides = {"small": 96, "medium": 256, "large": 512}
    out = {}
    for cls, L in sides.items():
        img = synth.blurred_noise_device((L, L, L), 6.0, 0.55, 0, dev)
        times = {}
        for ty, tx in EDT_TILES:
            ibip.set_tuning({"edt_tile_y": ty, "edt_tile_x": tx})
            for _ in range(3):
                ibip.edt(img)
            torch.cuda.synchronize()
            ibip.reset_timing()
            ibip.enable_timing(True)
            for _ in range(reps):
                ibip.edt(img)
            torch.cuda.synchronize()
            ibip.enable_timing(False)
            times[f"{ty}x{tx}"] = ibip.get_timing()["edt_ms"] / reps
        ibip.set_tuning(None)
        best = pick(times, "%dx%d" % EDT_TILES[0], MARGIN_EDT)
        ty, tx = (int(v) for v in best.split("x"))
        out[cls] = {"edt_tile_y": ty, "edt_tile_x": tx, "side": L, "ms": times}
        _log("edt", cls, L, best, {k: round(v, 4) for k, v in times.items()})
        del img
    return out


def _batch_images(n: int):
    import concurrent.futures as cf

    from paper_2101_03240_amd import synth

    specs = synth.batch_specs(96)[:n]
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(synth.image_for_spec, specs))


def tune_batch(dev, n: int = 96, reps: int = 3) -> dict:
    import torch

    import paper_2101_03240_amd as ibip
    from paper_2101_03240_amd import synth

    imgs = _batch_images(n)
    d_imgs = [torch.from_numpy(a).to(dev) for a in imgs]
    d_inls = [torch.from_numpy(synth.face_mask(a.shape, 0, 0)).to(dev) for a in imgs]
    times = {}
    for w in BATCH_WIDE:
        ibip.invade_batch(d_imgs, d_inls, tuning={"batch_wide": w})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ibip.invade_batch(d_imgs, d_inls, tuning={"batch_wide": w})
        torch.cuda.synchronize()
        times[str(w)] = 1e3 * (time.perf_counter() - t0) / reps
    best = pick(times, str(BATCH_WIDE[0]), MARGIN)
    _log("batch_wide", best, {k: round(v, 2) for k, v in times.items()})
    return {"batch_wide": int(best), "images": n, "ms": times}


def tune_serve(dev, sides=(192, 320, 448, 576), reps: int = 1) -> dict:
    import torch

    import paper_2101_03240_amd as ibip
    from paper_2101_03240_amd import synth

    imgs = [synth.blurred_noise_device((L, L, L), 6.0, 0.55, 2000 + i, dev) for i, L in enumerate(sides)]
    inls = []
    for a in imgs:
        m = torch.zeros_like(a)
        m[0] = 1
        inls.append(m)
    torch.cuda.synchronize()
    times = {}
    for w in SERVE_WIDE:
        with ibip.Server(dev, hbm_budget_bytes=32 << 30, max_inflight=len(imgs)) as srv:
            srv.set_tuning({"batch_wide": w})
            srv.wait(srv.submit(imgs[0], inls[0]))
            t0 = time.perf_counter()
            for _ in range(reps):
                tickets = [srv.submit(a, b) for a, b in zip(imgs, inls)]
                for t in tickets:
                    srv.wait(t)
            times[str(w)] = 1e3 * (time.perf_counter() - t0) / reps
    best = pick(times, str(SERVE_WIDE[0]), MARGIN)
    _log("serve_wide", best, {k: round(v, 2) for k, v in times.items()})
    return {"serve_wide": int(best), "sides": list(sides), "ms": times}


def main() -> int:
    import argparse

    import torch

    ap = argparse.ArgumentParser(description="time the launch-parameter candidates and write the cache")
    ap.add_argument("--out", default=CACHE, help="where to write the cache (default: beside this file)")
    args = ap.parse_args()

    if not torch.cuda.is_available():
        print("autotune needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    arch = torch.cuda.get_device_properties(dev).gcnArchName
    doc = {"arch": arch, "written": time.strftime("%Y-%m-%d %H:%M:%S"),
           "margin": MARGIN, "margin_edt": MARGIN_EDT,
           "edt": tune_edt(dev), "batch": tune_batch(dev), "serve": tune_serve(dev)}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    _log("wrote", args.out)
    return 0


def load(arch: str) -> dict | None:
    """The cache's choices when it was written on `arch`, else None."""
    if not os.path.exists(CACHE):
        return None
    try:
        with open(CACHE) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        return None
    return doc if doc.get("arch", "").split(":")[0] == arch.split(":")[0] else None


if __name__ == "__main__":
    sys.exit(main())
