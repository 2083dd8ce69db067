"""Per-stage kernel timing against the HBM roofline (and the launch loops that
rocprofv3 kernel traces and counter runs read).

Every slot of an 8-worker template first runs one job: one batch graph of
8 x slots chains, chain i in slot i / 8 of worker i % 8.  Each stage is then
timed with HIP events around `reps` back-to-back launches, two ways:

* cold: launch r works on slot r mod (8 x slots).  The slots together hold far
  more than the 256 MB of last-level cache, so each launch reads its operands
  from HBM and its writes go back to HBM;
* warm: every launch on one slot, whose operands stay cached when they fit
  (the figure the first measurements reported).

Beside each stage: a plain device copy moving the same bytes (half read, half
written), cold (rotating over 1 GiB): the library's reference copy kernel (one
16-byte word per thread), the bandwidth the memory system gives at that
transfer size; and the runtime's device-to-device copy (hipMemcpy's blit
kernel), cold and warm (one buffer pair).  A last plain copy of known size
calibrates the byte counters of counter runs.

    python -m paper_2606_05495_amd.stage_probe --side 1024 --reps 100
"""
from __future__ import annotations

import argparse
import json

import numpy as np

WORKERS = 8


def cold_copy_us(torch, half, reps, span=1 << 30):
    """Mean time of a device copy of `half` bytes, copy r taking source and
    destination slice r mod k of two buffers of about span / 2 bytes each."""
    k = max(2, (span // 2) // max(half, 1))
    a = torch.empty(k * half, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.fill_(0)
    for r in range(min(k, 16)):
        b[r * half:(r + 1) * half].copy_(a[r * half:(r + 1) * half])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        i = (r * 7 + 3) % k  # stride through the slices so neighbours are not reused
        b[i * half:(i + 1) * half].copy_(a[i * half:(i + 1) * half])
    e1.record()
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    del a, b
    return us


def warm_copy_us(torch, half, reps):
    """Mean time of a device copy of `half` bytes between one buffer pair."""
    a = torch.empty(max(16, half), dtype=torch.uint8, device="cuda")
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
    return e0.elapsed_time(e1) * 1e3 / reps


def _inputs(args, slots):
    """Eight seeded inputs, cycled over the 8 x slots jobs."""
    from paper_2606_05495_amd import synth
    n = WORKERS * slots
    if args.pipeline == "scan":
        base = [synth.scan_input(0, k, args.n).view(np.uint8) for k in range(8)]
    elif args.pipeline == "hotspot":
        base = []
        for k in range(8):
            t0, p = synth.hotspot_input(0, k, args.height or args.side, args.side)
            base.append(np.concatenate([t0.ravel(), p.ravel()]).view(np.uint8))
    elif args.pipeline == "box_hist":
        base = [synth.box_image(0, k, args.height or args.side, args.side).ravel() for k in range(8)]
    else:
        base = [synth.normal_image(0, k, args.height or args.side, args.side).view(np.uint8).ravel() for k in range(8)]
    return [base[k % 8] for k in range(n)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pipeline", default="gauss_sobel", choices=["gauss_sobel", "box_hist", "scan", "hotspot"])
    ap.add_argument("--steps", type=int, default=4, help="hotspot: steps per job")
    ap.add_argument("--side", type=int, default=1024, help="image / grid width (and height, unless --height)")
    ap.add_argument("--height", type=int, default=0, help="image / grid height (default: --side)")
    ap.add_argument("--n", type=int, default=1 << 21)
    ap.add_argument("--reps", type=int, default=100)
    ap.add_argument("--slots", type=int, default=0,
                    help="slots per worker (0: enough for about 1 GiB of slots, at least 2)")
    ap.add_argument("--copy-mib", type=int, default=64)
    ap.add_argument("--cold-only", action="store_true",
                    help="time the cold loops only (no warm loops, no same-bytes copies): for counter runs, where "
                         "each stage's dispatches are then the batch's 8 x slots followed by its cold loop")
    args = ap.parse_args()
    import torch
    from paper_2606_05495_amd import _abi as A
    from paper_2606_05495_amd.runtime import Context, pinned

    def template(ctx):
        if args.pipeline == "scan":
            return ctx.define("scan", max_n=args.n)
        if args.pipeline == "hotspot":
            return ctx.define("hotspot", width=args.side, height=args.height or args.side, max_n=args.steps)
        if args.pipeline == "box_hist":
            return ctx.define("box_hist", width=args.side, height=args.height or args.side)
        return ctx.define("gauss_sobel", width=args.side, height=args.height or args.side)

    slots = args.slots
    if slots <= 0:
        probe = Context(mode="batch", workers=1, slots=1, batch_size=1)
        slot_bytes, _ = A.set_template_footprint(probe.cfg, probe.templates[template(probe)])
        probe.close()
        slots = int(min(64, max(2, -(-(1 << 30) // (WORKERS * slot_bytes)))))
    ctx = Context(mode="batch", workers=WORKERS, slots=slots, batch_size=WORKERS * slots)
    tid = template(ctx)
    ib, ob = ctx.in_bytes(tid), ctx.out_bytes(tid)
    data = _inputs(args, slots)
    n = len(data)
    tin, nin = pinned(ib * n)
    for k, d in enumerate(data):
        nin[k * ib:(k + 1) * ib] = d
    ostride = (max(ob, 64) + 255) // 256 * 256
    tout, _ = pinned(ostride * n)
    arr = ctx.job_array(n)
    j = np.arange(n, dtype=np.uint64)
    arr["host_in"] = tin.data_ptr() + j * np.uint64(ib)
    arr["in_bytes"] = ib
    arr["host_out"] = tout.data_ptr() + j * np.uint64(ostride)
    arr["out_bytes"] = ob
    ctx.submit_many(tid, arr)  # one batch graph: every slot runs one job
    ctx.drain()
    out = {"slots": WORKERS * slots, "reps": args.reps}
    # one untimed pass over every stage first: the device leaves the idle
    # state of the set-up above before the first timed loop
    for i in range(len(ctx.stage_info(tid))):
        ctx.time_stage(tid, i, -1, args.reps)
    for i, (name, nbytes) in enumerate(ctx.stage_info(tid)):
        cold = ctx.time_stage(tid, i, -1, args.reps)
        if name in out:  # a repeated stage (the thermal grid's steps): the last one keeps the plain name
            out[name + "@%d" % (i - 1)] = out.pop(name)
        out[name] = {"bytes": int(nbytes), "cold_us": round(cold, 3), "cold_GBps": round(nbytes / cold / 1e3, 1)}
        if args.cold_only:
            continue
        warm = ctx.time_stage(tid, i, 0, args.reps)
        half = max(16, (int(nbytes) // 2 + 15) // 16 * 16)
        out[name].update({"warm_us": round(warm, 3), "warm_GBps": round(nbytes / warm / 1e3, 1),
                          "copy_cold_us": round(ctx.time_device_copy(2 * half, args.reps), 3),
                          "runtime_copy_cold_us": round(cold_copy_us(torch, half, args.reps), 3),
                          "copy_warm_us": round(warm_copy_us(torch, half, args.reps), 3)})
    ctx.close()
    # calibration: a plain device-to-device copy of known size
    nc = args.copy_mib << 20
    a = torch.empty(nc, dtype=torch.uint8, device="cuda")
    b = torch.empty(nc, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        b.copy_(a)
    torch.cuda.synchronize()
    out["calibration_copy_bytes"] = nc
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
