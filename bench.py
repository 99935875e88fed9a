#!/usr/bin/env python3
"""Throughput of the image-based invasion percolation hot path on one MI355X.

One step = the whole path over one synthetic image already resident in HBM:
exact squared EDT, the invasion loop (steps, sphere insertion, per-step
saturation and capillary pressure) and defender trapping. The default workload
is the 512^3 blurred-noise image (invasion + trapping). On the 200^3 packing
(and the 64^3 spheres) a step also runs the pressure-based morphological-
opening drainage at 25 radii used for the equal-saturation comparison; the
opening needs only the image and the inlets, so it runs from a second host
thread on a second stream while the invasion (whose step loop occupies one
compute unit) and the trapping run. The reported value is invaded voxels per
second of wall time over the timed steps.

Outside the timed region the default run also reports the equal-saturation
comparison with the opening on the 200^3 packing (trapping off) and the EDT
alone at 512^3, and times the CPU oracle on a thin slab of the same image.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload noise512]

Prints ONE JSON line. Only one GPU is supported: --gpus N with N > 1 exits with
a message.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "invaded voxels/s (full sequence+trapping), EDT GB/s; batched vs plain, bit-exact"
HBM_PEAK_GBPS = 8000.0

WORKLOADS = {
    "spheres64": "64^3 overlapping balls (radius 4, Poisson centres, porosity 0.65, seed 0); inlets x=0, "
                 "outlets x=63; invade + trap + MIO at 25 radii",
    "packing200": "200^3 sphere packing (lognormal radii mean 12 sd 3 voxels, porosity ~0.40, seed 0); "
                  "inlets x=0, outlets x=199; invade + trap + MIO at 25 radii",
    "noise512": "512^3 Gaussian-blurred noise (sigma 6, porosity 0.55, seed 0); inlets x=0, outlets x=511; "
                "invade + trap",
    "opening512": "the opening drainage alone (Section 2.4.1: erosion at T, trim to the inlet-connected part, "
                  "ball dilation) on the 512^3 blurred-noise image at one squared radius T = the median of dt2 over "
                  "the pore; library time over 5 calls",
    "edt768": "the exact squared EDT alone (passes z, y, x; lines of 768 voxels) on 768^3 Gaussian-blurred noise "
              "(sigma 6, porosity 0.55, seed 0, generated on the device), kernel time over 20 calls",
    "edt512": "the exact squared EDT alone (passes z, y, x) on 512^3 Gaussian-blurred noise (sigma 6, porosity "
              "0.55, seed 0, generated on the device), kernel time over 20 calls",
    "serve": "continuous-batching server: blurred-noise requests (sigma 6, porosity U[0.45, 0.65], side "
             "log-uniform in 64..768, seeds 1000+j), inlets x=0; a closed loop at fixed depth gives the "
             "sustained capacity, then Poisson arrivals at 0.7x that rate give the latency from arrival to result",
    "batch96": "96 images of uneven size, sides uniform in 32..192 (even: sphere packings with radii scaled to "
               "the side, odd: blurred noise), porosity uniform in 0.35..0.70, seeds 0..95; inlets x=0; "
               "invade of every image in one batched call vs one call per image",
}

OPENING_BYTES_PER_VOXEL = 25  # the ball dilation: 17 B (three EDT passes) + 8 B (threshold read, output)
# Algorithmic bytes per unit of work for each phase.
EDT_BYTES_PER_VOXEL = 5          # read 1 B image, write 4 B dt2 (the floor)
EDT_BUDGET_BYTES_PER_VOXEL = 17  # three passes: 1+2, 2+4, 4+4
LOOP_BYTES_PER_CENTRE = 20       # push 4 + pop 4 + state write 4 + claim 4 + key read 4
PAINT_BYTES_PER_PORE = 12        # read state 4 + key 4, write seq 4
TRAP_BYTES_PER_VOXEL = 14        # read seq 4 + outlets 1, W 4 + write W 4, trapped 1
MIO_BYTES_PER_VOXEL_RADIUS = 13  # EDT of the kept set 5 + read K map 4 + update 4


def thresholds_for(dt2_max: int, n: int = 25) -> list[int]:
    """T_i = max(1, ceil((r_max i / n)^2)), i = n..1, deduplicated, r_max = sqrt(max dt2)."""
    rmax = math.sqrt(dt2_max)
    return sorted({max(1, math.ceil((rmax * i / n) ** 2)) for i in range(1, n + 1)}, reverse=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(img, with_mio: bool) -> dict:
    """The CPU oracle (single-threaded C) on a bounded slab of the same image:
    48 x-planes of a 512^2 cross-section, 128 of a 200^2 one (10-20 s)."""
    import numpy as np

    import oracle
    from paper_2101_03240_amd import synth

    X = img.shape[0]
    L = min(X, 128 if img.shape[1] * img.shape[2] <= 200 * 200 else 48)
    sl = np.ascontiguousarray(img[:L])
    inl = synth.face_mask(sl.shape, 0, 0)
    out = synth.face_mask(sl.shape, 0, L - 1)
    t0 = time.perf_counter()
    r = oracle.invade(sl, inl)
    oracle.trap(r["seq"], out)
    what = "invade + trap"
    if with_mio:
        dt2 = oracle.edt(sl)
        T = thresholds_for(int(dt2.max()))
        oracle.mio(sl, inl, np.array(T, np.uint32))
        what += f" + MIO at {len(T)} radii"
    dt = time.perf_counter() - t0
    invaded = int((r["seq"] > 0).sum())
    return {"value": invaded / dt, "unit": "invaded voxels/s", "cores": 1, "kind": "oracle",
            "cpu": cpu_model(), "host_threads": os.cpu_count(),
            "sample": f"slab x<{L} of the same image ({L}x{img.shape[1]}x{img.shape[2]}), inlets x=0, "
                      f"outlets x={L - 1}: {what} in {dt:.1f} s, {invaded} invaded voxels, one thread"}


CPU_PARALLEL_CHILD = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle
from paper_2101_03240_amd import synth
sl = np.load(sys.argv[2])
inl = synth.face_mask(sl.shape, 0, 0)
out = synth.face_mask(sl.shape, 0, sl.shape[0] - 1)
t0 = time.perf_counter()
r = oracle.invade(sl, inl)
oracle.trap(r["seq"], out)
dt = time.perf_counter() - t0
print(json.dumps({"s": dt, "invaded": int((r["seq"] > 0).sum()), "threads": oracle.threads()}))
"""


def cpu_parallel_baseline(img) -> dict:
    """The same oracle source built with OpenMP (its distance transform's
    lines and the x-planes of large spheres split over the host's threads;
    the selection loop and trapping stay serial), on the same slab as
    cpu_baseline, in a child process that loads that build."""
    import subprocess
    import tempfile

    import numpy as np

    import oracle

    lib = oracle.OPENMP_LIB if os.path.exists(oracle.OPENMP_LIB) else oracle.build_openmp()
    X = img.shape[0]
    L = min(X, 128 if img.shape[1] * img.shape[2] <= 200 * 200 else 48)
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "slab.npy")
        np.save(path, np.ascontiguousarray(img[:L]))
        p = subprocess.run([sys.executable, "-c", CPU_PARALLEL_CHILD, ROOT, path], capture_output=True, text=True,
                           env=dict(os.environ, IBIP_ORACLE_LIB=lib), timeout=600)
    if p.returncode != 0:
        raise RuntimeError("cpu parallel baseline failed: " + p.stderr[-2000:])
    r = json.loads(p.stdout.strip().splitlines()[-1])
    return {"value": r["invaded"] / r["s"], "unit": "invaded voxels/s", "threads": r["threads"],
            "kind": "oracle built with OpenMP", "cpu": cpu_model(),
            "sample": f"slab x<{L} of the same image ({L}x{img.shape[1]}x{img.shape[2]}), inlets x=0, "
                      f"outlets x={L - 1}: invade + trap in {r['s']:.1f} s, {r['invaded']} invaded voxels, "
                      f"EDT lines and the x-planes of spheres of radius >= 8 on {r['threads']} threads, the "
                      f"selection loop and trapping serial"}


def edt_alone(dev, L: int = 512, reps: int = 20) -> dict:
    """The exact EDT alone (passes z, y, x) on an L^3 blurred-noise image
    (sigma 6, porosity 0.55, seed 0, generated on the device), kernel time
    from the library's own events over `reps` calls, against HBM."""
    import torch

    import paper_2101_03240_amd as ibip
    from paper_2101_03240_amd import synth

    img = synth.blurred_noise_device((L, L, L), 6.0, 0.55, 0, dev)
    for _ in range(3):
        ibip.edt(img)
    torch.cuda.synchronize()
    ibip.reset_timing()
    ibip.enable_timing(True)
    for _ in range(reps):
        ibip.edt(img)
    torch.cuda.synchronize()
    ibip.enable_timing(False)
    ms = ibip.get_timing()["edt_ms"] / reps
    ibip.reset_timing()
    n = L ** 3
    floor = EDT_BYTES_PER_VOXEL * n / (ms * 1e-3) / 1e9
    budget = EDT_BUDGET_BYTES_PER_VOXEL * n / (ms * 1e-3) / 1e9
    traffic = measured_traffic("edt", f"edt{L}")
    del img
    return {"bound": "hbm", "kernel": f"edt alone (passes z, y, x), {L}^3 blurred noise",
            "achieved": floor, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": floor / HBM_PEAK_GBPS,
            "traffic": traffic, "avg_launch_ms": ms, "budget_gbps": budget, "budget_frac": budget / HBM_PEAK_GBPS,
            "measured_gbps": traffic / (ms * 1e-3) / 1e9 if traffic else None,
            "measured_frac": traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS if traffic else None}


def opening_alone(dev, reps: int = 5) -> dict:
    """The opening drainage alone on the 512^3 blurred-noise image at one
    squared radius (the median of dt2 over the pore), library time (HIP
    events on its stream) per call, against HBM at 25 B per voxel for the
    ball dilation (three EDT passes, the threshold read and the output)."""
    import torch

    import paper_2101_03240_amd as ibip
    from paper_2101_03240_amd import synth

    img = make_image("noise512")
    img_d = torch.from_numpy(img).to(dev)
    inl_d = torch.from_numpy(synth.face_mask(img.shape, 0, 0)).to(dev)
    d = ibip.edt(img_d)
    T = int(torch.median(d[d > 0].to(torch.int64)).item())
    for _ in range(2):
        ibip.opening_drainage(img_d, inl_d, [T])
    torch.cuda.synchronize()
    ibip.reset_timing()
    ibip.enable_timing(True)
    for _ in range(reps):
        m = ibip.opening_drainage(img_d, inl_d, [T])
    torch.cuda.synchronize()
    ibip.enable_timing(False)
    ms = ibip.get_timing()["mio_ms"] / reps
    ibip.reset_timing()
    n = img.size
    gbps = OPENING_BYTES_PER_VOXEL * n / (ms * 1e-3) / 1e9
    traffic = measured_traffic("opening", "opening512")
    return {"bound": "hbm", "kernel": "opening drainage at one radius (K-map, capped EDT, first-write epilogue)",
            "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
            "traffic": traffic, "avg_launch_ms": ms, "T": T, "mio_sat": m["mio_sat"][0],
            "measured_gbps": traffic / (ms * 1e-3) / 1e9 if traffic else None}


def eqsat_report(dev) -> dict:
    """Equal-saturation comparison of IBIP with the opening on the 200^3
    packing, trapping off (Section 3.1.1, Figures 6 and 8), from the GPU path:
    the opening at the 25 radii T_i, IBIP's saturation map, the per-level
    symmetric difference, its split 2a + gap (a: voxels IBIP holds through
    balls larger than the opening's; gap: IBIP's step granularity at equal
    count), and the peak-pressure envelope: IBIP's saturation just before its
    first step below T_i against the opening's saturation at T_i."""
    import numpy as np
    import torch

    import paper_2101_03240_amd as ibip
    from paper_2101_03240_amd import synth

    img = synth.config_image("packing200")
    img_d = torch.from_numpy(img).to(dev)
    inl_d = torch.from_numpy(synth.face_mask(img.shape, 0, 0)).to(dev)
    T = thresholds_for(int(ibip.edt(img_d).max().item()))
    r = ibip.invade(img_d, inl_d)
    s = ibip.saturation(r["seq"], r["M"])
    m = ibip.opening_drainage(img_d, inl_d, T)
    c = ibip.compare_opening(s["satmap"], m["mio_r2"], T, m["mio_sat"])
    dis = c["disagree"].cpu().numpy()
    M = r["M"].cpu().numpy().view(np.uint32).astype(np.int64)
    cum = np.cumsum(r["n_new"].cpu().numpy())
    n_pore = int(img.sum())
    lv = []
    for i, t in enumerate(T):
        mcount = int(round(m["mio_sat"][i] * n_pore))
        keq = int(np.searchsorted(cum, mcount, side="right"))
        gap = mcount - (int(cum[keq - 1]) if keq else 0)
        below = np.nonzero(M < t)[0]
        kstar = int(below[0]) + 1 if below.size else len(M) + 1
        env = (int(cum[kstar - 2]) if kstar >= 2 else 0) - mcount
        lv.append((int(t), int(dis[i]), (int(dis[i]) - gap) // 2, gap, env))
    worst = max(lv, key=lambda x: x[1])
    return {"image": "packing200 (200^3 sphere packing), inlets x=0, trapping off, 25 radii",
            "pore_voxels": n_pore, "levels": len(T),
            "max_disagreement": worst[1], "max_disagreement_frac": worst[1] / n_pore, "at_T": worst[0],
            "larger_balls_a": worst[2], "granularity_gap": worst[3],
            "max_larger_balls_frac": max(x[2] for x in lv) / n_pore,
            "max_envelope_excess": max(x[4] for x in lv), "max_envelope_excess_frac": max(x[4] for x in lv) / n_pore,
            "per_level": [{"T": x[0], "disagree": x[1], "a": x[2], "gap": x[3], "envelope_excess": x[4]} for x in lv]}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none for this workload or the kernel's
    source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f).get("kernels", {}).get(kernel)
    if not t:
        return None
    srcs = t.get("sources") or {t["source"]: t["source_sha256"]}
    for src, digest in srcs.items():
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return float(t["traffic_bytes_per_launch"])


def _spec_image(i):
    from paper_2101_03240_amd import synth
    sp = synth.batch_specs(96)[i]
    return synth.image_for_spec(sp)


def batch_images(n: int = 96):
    """The uneven-size batch, generated in a process pool."""
    import concurrent.futures as cf
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_spec_image, range(n)))


def run_batch(args) -> int:
    import numpy as np
    import torch

    import paper_2101_03240_amd as ibip
    from paper_2101_03240_amd import synth

    dev = torch.device("cuda:0")
    print("batch96: generating 96 images", file=sys.stderr, flush=True)
    imgs = batch_images(96)
    print("batch96: images generated", file=sys.stderr, flush=True)
    d_imgs = [torch.from_numpy(a).to(dev) for a in imgs]
    d_inls = [torch.from_numpy(synth.face_mask(a.shape, 0, 0)).to(dev) for a in imgs]
    n_vox = int(sum(a.size for a in imgs))

    tuning = json.loads(args.tuning) if args.tuning else None

    def batched():
        return ibip.invade_batch(d_imgs, d_inls, tuning=tuning)

    def plain():
        return [ibip.invade(a, b) for a, b in zip(d_imgs, d_inls)]

    for _ in range(args.warmup):
        batched()
        plain()
    b = batched()
    p = plain()
    exact = all(torch.equal(x["seq"], y["seq"]) and torch.equal(x["rad2"], y["rad2"]) and x["K"] == y["K"]
                and torch.equal(x["M"], y["M"]) for x, y in zip(b, p))
    invaded = int(sum(int((x["seq"] > 0).sum().item()) for x in b))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batched()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain()
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / args.steps
    res = {
        "metric": METRIC, "value": invaded / tb, "unit": "invaded voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * tb, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "batch96", "description": WORKLOADS["batch96"], "images": len(imgs),
                   "voxels": n_vox, "invaded_voxels": invaded, "parallelism": "single GPU",
                   "tuning": tuning if tuning is not None else
                   ibip.cached_tuning(max((a.shape for a in imgs), key=max), batch=True)},
        "batched_vs_plain": {"batched_ms": 1e3 * tb, "plain_ms": 1e3 * tp, "speedup": tp / tb,
                             "bit_exact": bool(exact), "plain_value": invaded / tp},
    }
    print(json.dumps(res), flush=True)
    del np
    return 0


def run_serve(args) -> int:
    import queue
    import threading

    import numpy as np
    import torch

    import paper_2101_03240_amd as ibip
    from paper_2101_03240_amd import synth

    dev = torch.device("cuda:0")
    specs = synth.serve_specs(args.requests)
    imgs, inls = [], []
    for j, sp in enumerate(specs):
        L = sp.L
        imgs.append(synth.blurred_noise_device((L, L, L), sp.sigma, sp.porosity, sp.seed, dev))
        m = torch.zeros((L, L, L), dtype=torch.uint8, device=dev)
        m[0] = 1
        inls.append(m)
        if (j + 1) % 16 == 0:
            print(f"serve: {j + 1} of {len(specs)} requests generated", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    vox = np.array([x.numel() for x in imgs], dtype=np.float64)
    print(f"serve: {len(imgs)} requests generated, {vox.sum() / 1e9:.2f} G voxels", file=sys.stderr, flush=True)
    srv = ibip.Server(dev, hbm_budget_bytes=int(args.serve_budget_gb * (1 << 30)), max_inflight=args.inflight,
                      lookahead=args.lookahead)
    if args.tuning:
        srv.set_tuning(json.loads(args.tuning))
    small = np.argsort(vox)[:min(8, len(imgs))]
    for i in small[: args.warmup * 4]:
        srv.wait(srv.submit(imgs[i], inls[i]))

    def collect(q, out):
        while True:
            item = q.get()
            if item is None:
                return
            i, t = item
            r = srv.wait(t)
            out[i] = (r["status"], r["latency_ms"], r["K"], int((r["seq"] > 0).sum().item()))
            if len(out) % 32 == 0:
                print(f"serve: {len(out)} results", file=sys.stderr, flush=True)

    def run(arrivals):
        q, out = queue.Queue(), {}
        th = threading.Thread(target=collect, args=(q, out))
        th.start()
        t0 = time.perf_counter()
        depth = args.depth
        inflight = []
        for i in range(len(imgs)):
            if arrivals is None:
                # closed loop: keep `depth` requests outstanding
                while len(inflight) >= depth:
                    inflight = [j for j in inflight if j not in out]
                    if len(inflight) >= depth:
                        time.sleep(0.0002)
            else:
                dt = t0 + arrivals[i] - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            q.put((i, srv.submit(imgs[i], inls[i])))
            inflight.append(i)
        q.put(None)
        th.join()
        return time.perf_counter() - t0, out

    wall_c, res_c = run(None)
    print(f"serve: closed loop {wall_c:.2f} s", file=sys.stderr, flush=True)
    rate = 0.7 * len(imgs) / wall_c
    arr = np.cumsum(np.random.default_rng(7).exponential(1.0 / rate, size=len(imgs)))
    arr -= arr[0]
    wall_p, res_p = run(arr)
    print(f"serve: poisson {wall_p:.2f} s", file=sys.stderr, flush=True)
    st = srv.stats()
    # a few requests again, alone, must give the same result
    exact = True
    for i in list(small[:3]) + [int(np.argmax(vox))][: args.check_large]:
        t = srv.submit(imgs[i], inls[i])
        r = srv.wait(t)
        a = ibip.invade(imgs[i], inls[i])
        exact &= r["K"] == a["K"] and torch.equal(r["seq"], a["seq"]) and torch.equal(r["M"], a["M"])
    srv.close()
    ok = all(v[0] == 0 for v in list(res_c.values()) + list(res_p.values()))
    lat_c = np.array([res_c[i][1] for i in range(len(imgs))])
    lat_p = np.array([res_p[i][1] for i in range(len(imgs))])
    invaded = float(sum(res_c[i][3] for i in range(len(imgs))))
    res = {
        "metric": METRIC, "value": invaded / wall_c, "unit": "invaded voxels/s", "n_gpus": 1,
        "steps": 1, "warmup": args.warmup, "ms_per_step": 1e3 * wall_c, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "serve", "description": WORKLOADS["serve"], "requests": len(imgs),
                   "voxels": float(vox.sum()), "max_inflight": args.inflight, "hbm_budget_gb": args.serve_budget_gb,
                   "closed_loop_depth": args.depth, "parallelism": "single GPU",
                   "tuning": srv.tuning},
        "serve": {"capacity_jobs_per_s": len(imgs) / wall_c, "capacity_voxels_per_s": vox.sum() / wall_c,
                  "closed_loop_p50_ms": float(np.percentile(lat_c, 50)),
                  "closed_loop_p99_ms": float(np.percentile(lat_c, 99)),
                  "poisson_rate_jobs_per_s": rate, "poisson_jobs_per_s": len(imgs) / wall_p,
                  "poisson_voxels_per_s": vox.sum() / wall_p,
                  "poisson_p50_ms": float(np.percentile(lat_p, 50)),
                  "poisson_p99_ms": float(np.percentile(lat_p, 99)),
                  "peak_running": int(st["peak_running"]), "peak_pool_gb": st["peak_bytes"] / 2 ** 30,
                  "all_ok": bool(ok), "alone_equals_mix": bool(exact)},
    }
    print(json.dumps(res), flush=True)
    return 0


def make_image(name: str):
    from paper_2101_03240_amd import synth
    return synth.config_image(name, seed=0)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="noise512", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-eqsat", action="store_true",
                    help="skip the equal-saturation comparison on the 200^3 packing")
    ap.add_argument("--no-edt512", action="store_true", help="skip the EDT-alone measurement at 512^3")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB before the workload, as a reference "
                         "for hardware traffic counters")
    ap.add_argument("--requests", type=int, default=64, help="serve: number of requests")
    ap.add_argument("--inflight", type=int, default=16, help="serve: execution slots")
    ap.add_argument("--lookahead", type=int, default=8, help="serve: admission window")
    ap.add_argument("--depth", type=int, default=32, help="serve: outstanding requests in the closed loop")
    ap.add_argument("--serve-budget-gb", type=float, default=96.0, help="serve: HBM pool for job scratch")
    ap.add_argument("--check-large", type=int, default=0, help="serve: also rerun the largest request alone")
    ap.add_argument("--tuning", default="",
                    help="launch parameters as JSON (keys edt_tile_y, edt_tile_x, batch_wide) for the batch, the "
                         "server or the single-image workloads")
    ap.add_argument("--hw-queues", type=int, default=-1,
                    help="hardware queues per process for the HIP runtime (0: its default)")
    args = ap.parse_args()
    if args.hw_queues < 0:
        # the batch and the server spread work over 8 and 16 streams, whose
        # kernels serialise when they share a hardware queue
        args.hw_queues = 16 if args.workload in ("batch96", "serve") else 0
    if args.hw_queues:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(args.hw_queues, 32))
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent images would shard one per GPU)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2101_03240_amd as ibip
    from paper_2101_03240_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.workload == "batch96":
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)
    dev = torch.device("cuda:0")
    if args.copy_probe_mb > 0:
        src = torch.ones(args.copy_probe_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.tuning:
        ibip.set_tuning(json.loads(args.tuning))
    if args.workload == "opening512":
        e = opening_alone(dev)
        print(json.dumps({
            "metric": METRIC, "value": e["achieved"], "unit": "GB/s", "n_gpus": 1, "steps": 5, "warmup": 2,
            "ms_per_step": e["avg_launch_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32", "data": "synthetic",
            "config": {"workload": "opening512", "description": WORKLOADS["opening512"], "shape": [512, 512, 512],
                       "parallelism": "single GPU"},
            "roofline": e}), flush=True)
        return 0
    if args.workload in ("edt512", "edt768"):
        L = int(args.workload[3:])
        e = edt_alone(dev, L)
        print(json.dumps({
            "metric": METRIC, "value": e["achieved"], "unit": "GB/s", "n_gpus": 1, "steps": 20, "warmup": 3,
            "ms_per_step": e["avg_launch_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32", "data": "synthetic",
            "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "shape": [L, L, L],
                       "parallelism": "single GPU"},
            "roofline": e}), flush=True)
        return 0
    print(f"bench: generating {args.workload}", file=sys.stderr, flush=True)
    img = make_image(args.workload)
    with_mio = args.workload in ("packing200", "spheres64")
    inl = synth.face_mask(img.shape, 0, 0)
    out = synth.face_mask(img.shape, 0, img.shape[0] - 1)
    img_d = torch.from_numpy(img).to(dev)
    inl_d = torch.from_numpy(inl).to(dev)
    out_d = torch.from_numpy(out).to(dev)
    dt2_max = int(ibip.edt(img_d).max().item())
    T = thresholds_for(dt2_max)
    n_vox = img.size
    n_pore = int(img.sum())

    import concurrent.futures as cf
    side_pool = cf.ThreadPoolExecutor(max_workers=1)  # one host thread, its own context and stream
    side = torch.cuda.Stream(device=dev)

    def opening():
        with torch.cuda.stream(side):
            return ibip.opening_drainage(img_d, inl_d, T)

    def on_side(fn):
        return side_pool.submit(fn).result()

    def step():
        fut = side_pool.submit(opening) if with_mio else None
        r = ibip.invade(img_d, inl_d)
        t = ibip.trap(r["seq"], out_d)
        m = fut.result() if fut is not None else None
        return r, t, m

    print("bench: warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        r, t, m = step()
    torch.cuda.synchronize()
    r, t, m = step()
    invaded = int((r["seq"] > 0).sum().item())
    K = r["K"]

    ibip.reset_timing()
    ibip.enable_timing(True)
    on_side(lambda: (ibip.reset_timing(), ibip.enable_timing(True)))
    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"bench: {1e3 * elapsed / args.steps:.1f} ms per step", file=sys.stderr, flush=True)
    ibip.enable_timing(False)
    tm = ibip.get_timing()
    ts = on_side(ibip.get_timing)
    on_side(lambda: ibip.enable_timing(False))
    side_pool.shutdown()
    tm["mio_ms"] += ts["mio_ms"]
    tm["relax_sweeps"] += ts["relax_sweeps"]

    ms_per_step = 1e3 * elapsed / args.steps
    value = invaded * args.steps / elapsed
    S = args.steps
    # per-phase kernels and their algorithmic traffic per launch
    phases = {
        "edt (3 passes, inside invade)": (tm["edt_ms"] / S, EDT_BYTES_PER_VOXEL * n_vox, S),
        "step loop (single-workgroup kernel)": (
            tm["loop_kernel_ms"] / max(tm["loop_launches"], 1),
            # centres of the steps this kernel ran (the wide steps' centres go to k_wide)
            LOOP_BYTES_PER_CENTRE * (tm["popped"] - tm["wide_centres"]) / max(tm["loop_launches"], 1),
            tm["loop_launches"]),
        "sphere insertion": (tm["paint_ms"] / S, PAINT_BYTES_PER_PORE * n_pore, S),
        "trapping": (tm["trap_ms"] / S, TRAP_BYTES_PER_VOXEL * n_vox, S),
    }
    if with_mio:
        phases["opening drainage"] = (tm["mio_ms"] / S, MIO_BYTES_PER_VOXEL_RADIUS * n_vox * len(T), S)
    totals = {k: v[0] * v[2] for k, v in phases.items()}
    dom = max(totals, key=totals.get)
    d_ms, d_bytes, d_launches = phases[dom]
    achieved = d_bytes / (d_ms * 1e-3) / 1e9 if d_ms > 0 else 0.0
    edt_ms = tm["edt_ms"] / S
    edt_gbps = EDT_BYTES_PER_VOXEL * n_vox / (edt_ms * 1e-3) / 1e9 if edt_ms > 0 else 0.0
    edt_budget = EDT_BUDGET_BYTES_PER_VOXEL * n_vox / (edt_ms * 1e-3) / 1e9 if edt_ms > 0 else 0.0
    edt_traffic = measured_traffic("edt", args.workload)
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "invaded voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "shape": list(img.shape), "pore_voxels": n_pore, "invaded_voxels": invaded,
                   "invasion_steps": K, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(dom, args.workload),
                     "avg_launch_ms": d_ms, "launches": int(d_launches)},
        "edt_roofline": {"bound": "hbm", "kernel": "edt (passes z, y, x of the invasion's EDT)",
                         "achieved": edt_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": edt_gbps / HBM_PEAK_GBPS, "traffic": edt_traffic,
                         "avg_launch_ms": edt_ms, "budget_gbps": edt_budget,
                         "budget_frac": edt_budget / HBM_PEAK_GBPS,
                         "measured_gbps": edt_traffic / (edt_ms * 1e-3) / 1e9 if edt_traffic and edt_ms > 0 else None},
        "phases_ms_per_step": {
            "edt": tm["edt_ms"] / S, "setup": tm["setup_ms"] / S, "loop": tm["loop_ms"] / S,
            "loop_kernel": tm["loop_kernel_ms"] / S, "wide_kernel": tm["wide_kernel_ms"] / S,
            "paint": tm["paint_ms"] / S, "steps": tm["steps_ms"] / S, "trap": tm["trap_ms"] / S,
            "mio": tm["mio_ms"] / S},
        "loop": {"us_per_invasion_step": 1e3 * tm["loop_ms"] / max(tm["steps"], 1),
                 # the loop's time outside its kernels: host synchronisation, state copies and
                 # relaunches around the wide steps
                 "host_overhead_ms_per_call": (tm["loop_ms"] - tm["loop_kernel_ms"] - tm["wide_kernel_ms"]) / S,
                 "host_overhead_us_per_launch": 1e3 * (tm["loop_ms"] - tm["loop_kernel_ms"] - tm["wide_kernel_ms"])
                 / max(tm["loop_launches"], 1),
                 "invasion_steps_per_s": tm["steps"] / (tm["loop_ms"] * 1e-3) if tm["loop_ms"] > 0 else 0.0,
                 "loop_launches_per_call": tm["loop_launches"] / S, "wide_launches_per_call": tm["wide_launches"] / S,
                 "wide_centres_per_call": tm["wide_centres"] / S,
                 "ns_per_wide_centre": 1e6 * tm["wide_kernel_ms"] / max(tm["wide_centres"], 1),
                 "relax_sweeps_per_step": tm["relax_sweeps"] / S},
    }
    # the latency the loop's steps are bound by: one claim (a returning
    # atomic) per step at least, from L2 (a 256 KiB chain), from the
    # memory-side cache (64 MiB) or from HBM (1 GiB)
    lat = {f"{name}_ns": ibip.probe_claim_latency(span, 20000)
           for name, span in (("l2", 256 << 10), ("mall", 64 << 20), ("hbm", 1 << 30))}
    us_step = res["loop"]["us_per_invasion_step"]
    res["loop"]["claim_round_trip"] = lat
    # how many L2 claim round trips one step takes
    res["loop"]["step_in_l2_claim_round_trips"] = 1e3 * us_step / lat["l2_ns"]
    # the EDT alone at the 512^3 size, where it is not dominated by launches
    if with_mio:
        res["config"]["mio_radii"] = len(T)
        res["config"]["overlap"] = "the opening drainage runs on a second stream during invade + trap"
    if not args.no_edt512:
        print("bench: edt alone at 512^3", file=sys.stderr, flush=True)
        res["edt512_roofline"] = edt_alone(dev)
    if not args.no_eqsat:
        print("bench: equal-saturation comparison on the 200^3 packing", file=sys.stderr, flush=True)
        res["equal_saturation_packing200"] = eqsat_report(dev)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle on a slab)", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(img, with_mio)
        print("bench: cpu data-parallel baseline (OpenMP build of the oracle on the slab)", file=sys.stderr,
              flush=True)
        res["cpu_parallel_baseline"] = cpu_parallel_baseline(img)
    print(json.dumps(res), flush=True)
    del np
    return 0


if __name__ == "__main__":
    sys.exit(main())
