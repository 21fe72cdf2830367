"""Fixed workloads for rocprofv3 runs, and the summariser for their output.

    python -m paper_2104_01253_amd.profile_run run --workload qr [--reps 2]

Workloads: qr and qr32 (2,000,000 x 100 QR, FP64 or FP32-stored basis), qr2pass,
arnoldi (128^3 stencil, n = 100), gmres and gmres32 (GMRES(50) at 128^3 to 1e-8,
FP64 or FP32-stored basis), batched (128 Krylov-Schur instances).
    python -m paper_2104_01253_amd.profile_run summarize --fetch DIR --write DIR \\
        --trace DIR --out profiles/<name>

`run` executes the named workload `reps` times plus one plain device copy of
`COPY_BYTES` bytes (torch's copy kernel) that calibrates the FETCH_SIZE /
WRITE_SIZE counters.  `summarize` reads rocprofv3's CSV output (counter
collection and kernel stats) and writes <out>.md, a short text summary, and
<out>.json, the per-kernel HBM bytes per launch (calibrated), keyed by a hash of
the kernel sources so that a stale measurement is not reused.  bench.py reads
the QR workload's record from profiles/traffic.json, a copy of that summary's
JSON.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 1 << 30     # 1 GiB read + 1 GiB written


def run(workload: str, reps: int, tuning=None):
    import torch
    sys.path.insert(0, ROOT)
    from paper_2104_01253_amd import binding, synth
    torch.cuda.set_device(0)
    ctx = binding.Context(0)
    for key, value in (tuning or {}).items():
        if value is not None:
            ctx.set_tuning(getattr(binding, key), value)
    if workload in ("qr", "qr32"):
        m, n = 2_000_000, 100
        B = binding.colmajor_from_numpy(synth.tall_skinny(m, n, 8.0))
        Q = binding.colmajor_empty(m, n, dtype=torch.float32 if workload == "qr32" else None)
        for _ in range(reps):
            _, rc, _ = ctx.qr(B, Q)
            assert rc == 0
    elif workload == "qr2pass":
        m, n = 2_000_000, 100
        B = binding.colmajor_from_numpy(synth.tall_skinny(m, n, 8.0))
        Q = binding.colmajor_empty(m, n)
        ctx.set_qr_schedule(False)
        for _ in range(reps):
            _, rc, _ = ctx.qr(B, Q)
            assert rc == 0
    elif workload == "arnoldi":
        prob, b = synth.gmres_cd3d(128)
        op = binding.stencil_op(prob.grid, prob.D, prob.vel)
        bd = torch.from_numpy(b).cuda()
        Q = binding.colmajor_empty(prob.m, 101)
        for _ in range(reps):
            _, rc, _ = ctx.arnoldi(op, bd, 100, Q)
            assert rc == 0
    elif workload in ("gmres", "gmres32"):
        if workload == "gmres32":
            ctx.set_basis_precision(32)
        prob, b = synth.gmres_cd3d(128)
        op = binding.stencil_op(prob.grid, prob.D, prob.vel)
        bd = torch.from_numpy(b).cuda()
        x = torch.zeros(prob.m, dtype=torch.float64, device="cuda")
        for _ in range(reps):
            x.zero_()
            rc, _ = ctx.gmres(op, bd, x, restart=50, rtol=1e-8)
            assert rc == 0
    elif workload == "batched":
        # the batched Krylov-Schur family (2-D grids n_x in 48..256, basis 60, keep 20,
        # 10 eigenvalues), 128 instances so that the trace stays small
        count = 128
        probs = synth.ks_instances(count, seed=4)
        descs = [binding.stencil2d(p.grid, p.D, p.vel) for p in probs]
        import numpy as np
        v0 = torch.from_numpy(np.concatenate([synth.normal_vector(p.m, 1000 + i)
                                              for i, p in enumerate(probs)])).cuda()
        for _ in range(reps):
            _, rc, _ = ctx.krylov_schur_batched(descs, v0, 10, 60, 20, 1e-8, 300, use_graph=True)
            assert rc == 0
    else:
        raise SystemExit(f"unknown workload {workload}")
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    print(f"profile_run {workload} done", flush=True)


def _rows(d, pattern):
    out = []
    for f in glob.glob(os.path.join(d, "**", pattern), recursive=True):
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


# kernel name fragments -> the kernel classes of dcgs2_profile_read
CLASSES = (("fused_qr_kernel", "fused_qr"), ("reduce_mv_kernel", "reduce"), ("reduce_kernel", "reduce"),
           ("update_slab_kernel", "update"), ("update_kernel", "update"),
           ("project_norm_kernel", "project_norm"), ("scale_col_kernel", "scale"),
           ("stencil_kernel", "spmv"), ("csr_kernel", "spmv"), ("tsgemm_kernel", "tsgemm"),
           ("finish_kernel", "finish"), ("bschur_kernel", "dense_schur"),
           ("btruncate_kernel", "truncate"), ("bscale_kernel", "scale"))


def _short(name: str) -> str:
    for key, cls in CLASSES:
        if key in name:
            return cls
    return "other"


def _dispatches(d, counter):
    """[(dispatch id, kernel name, grid size, counter value in KiB)] of one counter run."""
    out = []
    for r in _rows(d, "*counter_collection.csv"):
        if r.get("Counter_Name") == counter:
            out.append((int(r["Dispatch_Id"]), r.get("Kernel_Name", ""), int(r.get("Grid_Size", 0)),
                        float(r["Counter_Value"])))
    return out


def _calibrated(d, counter):
    """Per kernel class: (dispatches, bytes per launch) with the counter scaled so that
    the calibration copy (the largest copy-kernel dispatch, COPY_BYTES read and
    written) reads exactly COPY_BYTES; and the scale itself."""
    rows = _dispatches(d, counter)
    copies = [r for r in rows if "copyBuffer" in r[1]]      # hipMemcpy device-to-device
    cal = max(copies, key=lambda r: r[3]) if copies else None
    scale = COPY_BYTES / (cal[3] * 1024.0) if cal and cal[3] > 0 else 1.0
    per = {}
    for _, name, _, v in rows:
        k = _short(name)
        if k == "other":
            continue
        n, tot = per.get(k, (0, 0.0))
        per[k] = (n + 1, tot + v * 1024.0 * scale)
    return {k: (n, tot / n) for k, (n, tot) in per.items()}, scale


def summarize(fetch_dir, write_dir, trace_dir, out, command,
              sources=("kernels.hip", "device_common.h")):
    fetch, fscale = _calibrated(fetch_dir, "FETCH_SIZE")
    write, wscale = _calibrated(write_dir, "WRITE_SIZE")
    stats = {}
    for r in _rows(trace_dir, "*kernel_stats.csv"):
        k = _short(r["Name"])
        s = stats.setdefault(k, [0, 0.0])
        s[0] += int(r["Calls"])
        s[1] += float(r["TotalDurationNs"])
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        n = max(fetch.get(k, (0, 0.0))[0], write.get(k, (0, 0.0))[0], 1)
        fb = fetch.get(k, (0, 0.0))[1]
        wb = write.get(k, (0, 0.0))[1]
        kernels[k] = {"dispatches": n, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                      "bytes_per_launch": fb + wb}
        if k in stats:
            kernels[k]["trace_launches"] = stats[k][0]
            kernels[k]["avg_duration_us"] = stats[k][1] / max(stats[k][0], 1) / 1e3
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(HERE, "csrc", f), "rb").read())
    rec = {"kernel_source_sha256_16": h.hexdigest()[:16], "kernel_sources": list(sources),
           "calibration": {"copy_bytes": COPY_BYTES, "fetch_scale": fscale, "write_scale": wscale},
           "command": command, "kernels": kernels}
    os.makedirs(os.path.dirname(out) or ".", exist_ok=True)
    with open(out + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
    with open(out + ".md", "w") as fh:
        fh.write(f"# {os.path.basename(out)}\n\n")
        fh.write(f"commands:\n\n```\n{command}\n```\n\n")
        fh.write(f"Counter calibration: a device copy of {COPY_BYTES} bytes read and written; "
                 f"FETCH_SIZE scale {fscale:.4f}, WRITE_SIZE scale {wscale:.4f}.\n\n")
        fh.write("| kernel class | dispatches | HBM read MB/launch | HBM write MB/launch | "
                 "avg duration us (kernel trace) | measured GB/s |\n|---|---|---|---|---|---|\n")
        for k, v in kernels.items():
            us = v.get("avg_duration_us", float("nan"))
            gbs = v["bytes_per_launch"] / (us * 1e-6) / 1e9 if us == us and us > 0 else float("nan")
            fh.write(f"| {k} | {v['dispatches']} | {v['fetch_bytes_per_launch']/1e6:.2f} | "
                     f"{v['write_bytes_per_launch']/1e6:.2f} | {us:.1f} | {gbs:.0f} |\n")
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="qr")
    r.add_argument("--reps", type=int, default=1)
    r.add_argument("--fused-waves", type=int, default=None)
    r.add_argument("--reduce-grid", type=int, default=None)
    r.add_argument("--fused-min-j", type=int, default=None)
    r.add_argument("--fused-pair-slots", type=int, default=None)
    r.add_argument("--batch-dense", type=int, default=None,
                   help="batched workload: 0 dense restart work on the GPU, 1 on the host")
    s = sub.add_parser("summarize")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--trace", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--command", default="")
    s.add_argument("--sources", default="kernels.hip,device_common.h",
                   help="comma-separated csrc files whose hash keys the record")
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.workload, a.reps, {"TUNE_FUSED_WAVES": a.fused_waves,
                                 "TUNE_REDUCE_GRID": a.reduce_grid,
                                 "TUNE_FUSED_MIN_J": a.fused_min_j,
                                 "TUNE_FUSED_PAIR_SLOTS": a.fused_pair_slots,
                                 "TUNE_BATCH_DENSE": a.batch_dense})
    else:
        summarize(a.fetch, a.write, a.trace, a.out, a.command, tuple(a.sources.split(",")))


if __name__ == "__main__":
    main()
