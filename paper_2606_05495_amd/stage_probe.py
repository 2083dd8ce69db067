"""Launch each stage kernel of a template back to back (for rocprofv3 kernel
traces and hardware-counter runs), plus a plain device copy of known size
that calibrates the byte counters.

    python -m paper_2606_05495_amd.stage_probe --side 1024 --reps 50
"""
from __future__ import annotations

import argparse
import json

import numpy as np


def _copy_us(torch, nbytes, reps):
    """A plain device copy moving the same bytes (half read, half written)."""
    half = max(16, nbytes // 2)
    a = torch.empty(half, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(10):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    return round(e0.elapsed_time(e1) * 1e3 / reps, 3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pipeline", default="gauss_sobel", choices=["gauss_sobel", "box_hist", "scan", "hotspot"])
    ap.add_argument("--steps", type=int, default=4, help="hotspot: steps per job")
    ap.add_argument("--side", type=int, default=1024)
    ap.add_argument("--n", type=int, default=1 << 21)
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--copy-mib", type=int, default=64)
    args = ap.parse_args()
    import torch
    from paper_2606_05495_amd import synth
    from paper_2606_05495_amd.runtime import Context, pinned

    ctx = Context(mode="set", workers=1, slots=2)
    if args.pipeline == "scan":
        tid = ctx.define("scan", max_n=args.n)
        data = synth.scan_input(0, 0, args.n).view(np.uint8)
    elif args.pipeline == "hotspot":
        tid = ctx.define("hotspot", width=args.side, height=args.side, max_n=args.steps)
        t0, p = synth.hotspot_input(0, 0, args.side, args.side)
        data = np.concatenate([t0.ravel(), p.ravel()]).view(np.uint8)
    elif args.pipeline == "box_hist":
        tid = ctx.define("box_hist", width=args.side, height=args.side)
        data = synth.box_image(0, 0, args.side, args.side).ravel()
    else:
        tid = ctx.define("gauss_sobel", width=args.side, height=args.side)
        data = synth.normal_image(0, 0, args.side, args.side).view(np.uint8).ravel()
    ib, ob = ctx.in_bytes(tid), ctx.out_bytes(tid)
    tin, nin = pinned(ib)
    nin[:] = data
    tout, _ = pinned(max(ob, 64))
    for _ in range(4):
        ctx.submit(tid, host_in=tin.data_ptr(), in_bytes=ib, host_out=tout.data_ptr(), out_bytes=ob)
    ctx.drain()
    out = {}
    for i, (name, nbytes) in enumerate(ctx.stage_info(tid)):
        us = ctx.time_stage(tid, i, 0, args.reps)
        out[name] = {"avg_us": round(us, 3), "bytes": int(nbytes), "GBps": round(nbytes / us / 1e3, 1),
                     "copy_same_bytes_us": _copy_us(torch, int(nbytes), args.reps)}
    # calibration: a plain device-to-device copy of known size
    n = args.copy_mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        b.copy_(a)
    torch.cuda.synchronize()
    out["calibration_copy_bytes"] = n
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
