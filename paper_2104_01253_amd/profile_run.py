"""Fixed workloads for rocprofv3 runs, and the summariser for their output.

    python -m paper_2104_01253_amd.profile_run run --workload qr [--reps 2]
    python -m paper_2104_01253_amd.profile_run summarize --fetch DIR --write DIR \\
        --trace DIR --out profiles/<name>

`run` executes the named workload `reps` times plus one plain device copy of
`COPY_BYTES` bytes (torch's copy kernel) that calibrates the FETCH_SIZE /
WRITE_SIZE counters.  `summarize` reads rocprofv3's CSV output (counter
collection and kernel stats) and writes a short text summary and
profiles/traffic.json (per-kernel HBM bytes per launch, calibrated, keyed by a
hash of kernels.hip so a stale measurement is not reused).
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


def run(workload: str, reps: int):
    import torch
    sys.path.insert(0, ROOT)
    from paper_2104_01253_amd import binding, synth
    torch.cuda.set_device(0)
    ctx = binding.Context(0)
    if workload == "qr":
        m, n = 2_000_000, 100
        B = binding.colmajor_from_numpy(synth.tall_skinny(m, n, 8.0))
        Q = binding.colmajor_empty(m, n)
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
    elif workload == "gmres":
        prob, b = synth.gmres_cd3d(128)
        op = binding.stencil_op(prob.grid, prob.D, prob.vel)
        bd = torch.from_numpy(b).cuda()
        x = torch.zeros(prob.m, dtype=torch.float64, device="cuda")
        for _ in range(reps):
            x.zero_()
            rc, _ = ctx.gmres(op, bd, x, restart=50, rtol=1e-8)
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


def _short(name: str) -> str:
    for key in ("fused_qr_kernel", "reduce_kernel", "update_kernel", "project_norm_kernel",
                "scale_col_kernel", "stencil_kernel", "csr_kernel", "tsgemm_kernel"):
        if key in name:
            return key
    if "copy" in name.lower() or "elementwise" in name.lower():
        return "torch_copy"
    return name[:60]


def _counter(d, counter):
    """Sum of `counter` per short kernel name and dispatch count."""
    per, disp = {}, {}
    for r in _rows(d, "*counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        k = _short(r.get("Kernel_Name", ""))
        per[k] = per.get(k, 0.0) + float(r["Counter_Value"])
        disp.setdefault(k, set()).add(r.get("Dispatch_Id"))
    return per, {k: len(v) for k, v in disp.items()}


def summarize(fetch_dir, write_dir, trace_dir, out, command):
    fetch, nf = _counter(fetch_dir, "FETCH_SIZE")
    write, nw = _counter(write_dir, "WRITE_SIZE")
    # copy calibration: the copy kernel moves COPY_BYTES in and COPY_BYTES out
    cf = fetch.get("torch_copy", 0.0) * 1024.0
    cw = write.get("torch_copy", 0.0) * 1024.0
    fscale = COPY_BYTES / cf if cf > 0 else 1.0
    wscale = COPY_BYTES / cw if cw > 0 else 1.0
    stats = {}
    for r in _rows(trace_dir, "*kernel_stats.csv"):
        k = _short(r["Name"])
        s = stats.setdefault(k, [0, 0.0])
        s[0] += int(r["Calls"])
        s[1] += float(r["TotalDurationNs"])
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        if k == "torch_copy":
            continue
        n = max(nf.get(k, 0), nw.get(k, 0), 1)
        fb = fetch.get(k, 0.0) * 1024.0 * fscale / n
        wb = write.get(k, 0.0) * 1024.0 * wscale / n
        kernels[k] = {"dispatches": n, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                      "bytes_per_launch": fb + wb}
        if k in stats:
            kernels[k]["avg_duration_us"] = stats[k][1] / max(stats[k][0], 1) / 1e3
    src = open(os.path.join(HERE, "csrc", "kernels.hip"), "rb").read()
    rec = {"kernel_source_sha256_16": hashlib.sha256(src).hexdigest()[:16],
           "calibration": {"copy_bytes": COPY_BYTES, "fetch_scale": fscale, "write_scale": wscale},
           "command": command, "kernels": kernels}
    os.makedirs(os.path.dirname(out) or ".", exist_ok=True)
    with open(out + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
    with open(out + ".md", "w") as fh:
        fh.write(f"# {os.path.basename(out)}\n\ncommand: `{command}`\n\n")
        fh.write(f"copy calibration: FETCH scale {fscale:.4f}, WRITE scale {wscale:.4f}\n\n")
        fh.write("| kernel | dispatches | fetch MB/launch | write MB/launch | avg us |\n|---|---|---|---|---|\n")
        for k, v in kernels.items():
            fh.write(f"| {k} | {v['dispatches']} | {v['fetch_bytes_per_launch']/1e6:.2f} | "
                     f"{v['write_bytes_per_launch']/1e6:.2f} | {v.get('avg_duration_us', float('nan')):.1f} |\n")
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="qr")
    r.add_argument("--reps", type=int, default=1)
    s = sub.add_parser("summarize")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--trace", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--command", default="")
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.workload, a.reps)
    else:
        summarize(a.fetch, a.write, a.trace, a.out, a.command)


if __name__ == "__main__":
    main()
