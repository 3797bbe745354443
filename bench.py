#!/usr/bin/env python3
"""Throughput of the shift-and-stack search on one GPU.

One step is the whole path on one synthetic stack already resident in HBM:
likelihood planes (kb_make_psi_phi), the trajectory search (kb_search) and the
final per-pixel top-k (kb_topk).  Default workload: 15 images of 4096 x 4096
over 3 nights, 600 velocities, K = 50 (about 1e10 trajectories).

Prints one JSON line with trajectory-image evaluations per second
(N * H * W * V per step / step time), the search kernel's fraction of the HBM
gather roofline (8 bytes of psi/phi per evaluation against 8 TB/s) and the
FP64 oracle's throughput on the host cores for context.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_TIE_F32 = 8.0
# The search kernel's sources: a counter profile is valid only for these bytes.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1901_02492_amd", "csrc", f)
                  for f in ("kbmi_device.h", "kbmi_search.hip")]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "search_kernel_survey_15x4096x4096_v600_k50.md")


def measured_traffic():
    """HBM bytes per search launch from the committed counter profile, or None
    if the profile is missing or was taken on a different kernel source."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(f, "rb").read())
        src = h.hexdigest()
    except OSError:
        return None
    fields = dict(line.strip().split(":", 1) for line in text.splitlines()
                  if line.strip().startswith(("kernel_source_sha256:",
                                              "traffic_bytes_per_launch:")))
    if fields.get("kernel_source_sha256", "").strip() != src:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_stack(workload):
    from paper_1901_02492_amd import synth
    if workload == "survey":
        return synth.survey_stack()
    if workload == "small":
        return synth.small_stack()
    raise SystemExit(f"unknown workload {workload}")


# --- CPU baseline: the FP64 oracle on crops of the same stack ---------------
_CPU_STACK = None


def _oracle_crop(arg):
    import oracle
    y0, x0, c = arg
    s = _CPU_STACK
    sl = (slice(None), slice(y0, y0 + c), slice(x0, x0 + c))
    t0 = time.perf_counter()
    oracle.search(s.img[sl], s.var[sl], s.mask[sl], s.t, s.psf, s.vel, s.k)
    return time.perf_counter() - t0


def cpu_baseline(s, crop=224):
    """Run the oracle on one crop per worker process (all images, all velocities)."""
    global _CPU_STACK
    _CPU_STACK = s
    n, h, w = s.img.shape
    workers = max(1, min(16, os.cpu_count() or 1))
    c = min(crop, h, w)
    rng = np.random.default_rng(0)
    args = [(int(rng.integers(0, h - c + 1)), int(rng.integers(0, w - c + 1)), c)
            for _ in range(workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        per = pool.map(_oracle_crop, args)
    wall = time.perf_counter() - t0
    tie = workers * n * c * c * s.vel.shape[0]
    return {"value": tie / wall, "unit": "trajectory-image evals/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{workers} crops of {c}x{c} start pixels (all {n} images, all "
                      f"{s.vel.shape[0]} velocities, K={s.k}), one FP64 numpy oracle process "
                      f"per crop; wall {wall:.1f} s, per-crop {min(per):.1f}-{max(per):.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="survey", choices=["survey", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (to scale HBM "
                         "byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the search runs on a single device "
              "(pass --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "copies": 2}), flush=True)
        return

    t0 = time.perf_counter()
    s = make_stack(args.workload)
    n, h, w = s.img.shape
    nv = s.vel.shape[0]
    log(f"workload {s.name}: generated in {time.perf_counter() - t0:.1f} s")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(s)
        log(f"cpu baseline {cpu['value']:.3e} TIE/s on {cpu['cores']} cores")

    import torch
    from paper_1901_02492_amd import lib
    lib.load()
    dev = torch.device("cuda:0")
    img = torch.from_numpy(s.img).to(dev)
    var = torch.from_numpy(s.var).to(dev)
    mask = torch.from_numpy(s.mask).to(dev)
    planes = torch.empty((n, h, w, 2), dtype=torch.float32, device=dev)
    cand = lib.alloc_candidates(h, w, s.k, dev)
    res = lib.alloc_candidates(h, w, s.k, dev)
    ws = lib.alloc_workspace(n, h, w, nv, dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    log("inputs resident on the device")

    def step(ev=None):
        lib.make_psi_phi(img, var, mask, s.psf, out=planes)
        if ev is not None:
            ev[0].record(stream)
        lib.search(planes, s.t, s.vel, s.k, out=cand, workspace=ws)
        if ev is not None:
            ev[1].record(stream)
        lib.topk(cand, s.k, n, out=res)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"{args.warmup} warmup steps done")

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    search_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    log(f"{args.steps} timed steps: {ms_step:.2f} ms/step, search kernel {search_ms:.2f} ms")

    tie = s.tie
    achieved = BYTES_PER_TIE_F32 * tie / (search_ms * 1e-3) / 1e9
    out = {
        "metric": "trajectory-image evals/s",
        "value": tie / (ms_step * 1e-3),
        "unit": "trajectory-image evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": s.name, "n_img": n, "h": h, "w": w, "n_vel": nv, "k": s.k,
                   "trajectories": h * w * nv, "tie_per_step": tie,
                   "step": "kb_make_psi_phi + kb_search + kb_topk"},
        "roofline": {"bound": "hbm", "kernel": "search_kernel", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(), "search_ms": search_ms,
                     "bytes_per_tie": BYTES_PER_TIE_F32},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
