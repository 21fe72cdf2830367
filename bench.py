"""Benchmark of the DCGS2 hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-legs]

Headline workload (one bench "step"): the left-looking DCGS2 QR of the
tall-skinny B = G diag(logspace(0,-8,100)) V, m = 2,000,000 x n = 100, FP64,
resident in HBM -- 100 DCGS2 columns (steps) per factorisation.  `value` is DCGS2
steps (columns) per second over the K timed factorisations.

Also reported (not `value`): the DCGS2 Arnoldi expansion at m = 128^3 = 2,097,152
with n = 100 (3-D convection-diffusion matvec), restarted GMRES(50) on the same
operator to a 1e-8 true relative residual (time-to-solution, FP64 and FP32-stored
basis), one Krylov-Schur solve, batched Krylov-Schur over 512 operators, batched
GMRES over 128 systems against the single-instance solver, GMRES from the learned
initial guess against x0 = 0, the per-kernel roofline figures measured with HIP
events around each launch, and the FP64 oracle timed on the host (the whole QR
factorisation, and a two-cycle sample of its GMRES).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, published
METRIC = "DCGS2 Arnoldi steps/s + HBM GB/s (m=2M,n=100); GMRES time-to-1e-8 vs FP64"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
TRAFFIC_FILE_Q32 = os.path.join(ROOT, "profiles", "traffic_q32.json")
TRAFFIC_FILE_ARNOLDI = os.path.join(ROOT, "profiles", "arnoldi_128cube_n100.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2104_01253_amd", "csrc", f)
               for f in ("kernels.hip", "device_common.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sources of the path's kernels (a counter record is only used when
    it was taken with exactly these sources)."""
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, record: str = TRAFFIC_FILE):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when the kernels changed since the counters were taken."""
    try:
        t = json.load(open(record))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("kernels", {}).get(kernel, {}).get("bytes_per_launch")


def timed(torch, fn, steps):
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1000.0


def kernel_roof(st, traffic=None):
    """Algorithmic GB/s of one kernel class (bytes per launch over its mean duration),
    with the counter-measured HBM bytes per launch when a record for these kernels
    exists."""
    avg_ms = st["total_ms"] / max(st["launches"], 1)
    bytes_per_launch = st["bytes"] / max(st["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {"launches": st["launches"], "avg_launch_us": round(avg_ms * 1e3, 2),
            "alg_bytes_per_launch": bytes_per_launch, "achieved": round(achieved, 1),
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic}


def roofline(prof, record=TRAFFIC_FILE):
    kern = {k: v for k, v in prof.items() if not k.startswith("phase_")}
    dom = max(kern.items(), key=lambda kv: kv[1]["total_ms"])
    name, st = dom
    avg_ms = st["total_ms"] / max(st["launches"], 1)
    bytes_per_launch = st["bytes"] / max(st["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    tr = measured_traffic(name, record)
    return name, {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": tr,
        "kernel": name, "launches": st["launches"], "avg_launch_us": round(avg_ms * 1e3, 2),
        "alg_bytes_per_launch": bytes_per_launch,
    }


def cpu_model() -> str:
    """The host CPU's model name, family/model/stepping numbers and logical CPU count
    (Linux), for the CPU baseline's context (a virtual machine may report only the
    product family as its name)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if ":" in line:
                    k, v = line.split(":", 1)
                    info.setdefault(k.strip(), v.strip())
    except OSError:
        pass
    name = info.get("model name", "unknown")
    fam = "/".join(info.get(k, "?") for k in ("cpu family", "model", "stepping"))
    return f"{name} (family/model/stepping {fam}, {os.cpu_count()} logical CPUs)"


def cpu_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_gmres_sample(cycles=2):
    """The oracle's GMRES(50) (oracle.gmres.gmres_dcgs2, unmodified) on the 128^3 GMRES
    workload for its first `cycles` restart cycles: iterations per second on the host,
    and the time to 1e-8 projected from that rate and the oracle's own iteration count
    (tests/golden/gmres50_128cube.json, written by a script that runs only the oracle;
    every cycle sweeps the same basis sizes, so the first cycles' rate holds for all)."""
    from oracle import operators as ops
    from oracle.gmres import gmres_dcgs2
    from paper_2104_01253_amd import synth
    prob, b = synth.gmres_cd3d(128)
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    t0 = time.perf_counter()
    _, info = gmres_dcgs2(A, b, restart=50, rtol=1e-8, max_iters=50 * cycles)
    dt = time.perf_counter() - t0
    rate = info["iters"] / dt
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "gmres50_128cube.json")))
    iters = golden["fp64"]["iters"]
    return {"iters_per_s": round(rate, 2), "oracle_iters_to_1e-8": iters,
            "projected_time_to_1e-8_s": round(iters / rate, 2), "cores": int(cpu_threads()),
            "sample": f"the first {cycles} restart cycles ({info['iters']} iterations, "
                      f"{dt:.1f} s) of the oracle's GMRES(50) at 128^3"}


def cpu_baseline(B, n):
    """The FP64 oracle (oracle.gram_schmidt.dcgs2_qr, unmodified) on the whole of B."""
    from oracle import gram_schmidt as gs
    cores = cpu_threads()
    m = B.shape[0]
    t0 = time.perf_counter()
    gs.dcgs2_qr(B)
    dt = time.perf_counter() - t0
    return {"value": round(n / dt, 3), "unit": "steps/s", "cores": int(cores),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"one full factorization of the same B ({m} x {n}) by "
                      f"oracle.gram_schmidt.dcgs2_qr (NumPy/BLAS fp64), {dt:.2f} s"}


def calibration(torch, nbytes=1_600_000_000):
    """Achievable HBM rates on this device for the roofline's context: a device copy
    (read + write) and a streaming read (sum) over nbytes of FP64."""
    x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    t_copy = timed(torch, lambda: y.copy_(x), 5) / 5
    x.sum()
    t_read = timed(torch, lambda: x.sum(), 5) / 5
    del x, y
    torch.cuda.empty_cache()
    return {"copy_gbps": round(2 * nbytes / t_copy / 1e9, 1),
            "read_gbps": round(nbytes / t_read / 1e9, 1), "bytes": nbytes}


def row_block_leg(torch, ctx, binding, B, n, rows=250_000, steps=20):
    """The same factorisation on the first `rows` rows of B: one GPU's row block when
    the m = 2,000,000 problem is split eight ways (without the per-step all-reduce
    such a split adds).  Reports the wall time, the time inside the streaming
    kernels (HIP events) and the rest: finishing kernels and launch gaps, the fixed
    per-step costs that grow in weight as the row block shrinks."""
    Bs = binding.colmajor_from_numpy(np.ascontiguousarray(B[:rows]))
    Qs = binding.colmajor_empty(rows, n)

    def once():
        _, rc, _ = ctx.qr(Bs, Qs)
        assert rc == binding.OK, rc
    for _ in range(3):
        once()
    T = timed(torch, once, steps) / steps
    ctx.profile(True)
    ctx.profile_read(reset=True)
    once()
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    stream_ms = sum(v["total_ms"] for v in prof.values())
    alg = sum(v["bytes"] for v in prof.values())
    del Bs, Qs
    return {"m": rows, "n": n, "ms": round(T * 1e3, 3), "steps_per_s": round(n / T, 1),
            "hbm_gbps": round(alg / T / 1e9, 1), "streaming_kernels_ms": round(stream_ms, 3),
            "finish_and_gaps_ms": round(T * 1e3 - stream_ms, 3)}


def batched_ks_leg(torch, ctx, binding, synth, count=512, tune_count=64):
    """Batched Krylov-Schur: `count` 2-D convection-diffusion operators, n_x ~ U{48..256},
    v ~ U(0,50)^2, 10 largest-magnitude eigenvalues, basis 60, keep 20, tol 1e-8.  The
    rows per reduction workgroup are first autotuned on the first `tune_count`
    instances (the restart's dense work stays on host threads)."""
    from paper_2104_01253_amd import autotune
    probs = synth.ks_instances(count, seed=4)
    descs = [binding.stencil2d(p.grid, p.D, p.vel) for p in probs]
    v0s = [synth.normal_vector(p.m, 1000 + i) for i, p in enumerate(probs)]
    v0 = torch.from_numpy(np.concatenate(v0s)).cuda()
    vt = torch.from_numpy(np.concatenate(v0s[:tune_count])).cuda()
    torch.cuda.synchronize()
    key = binding.TUNE_BATCH_REDUCE_ROWS
    best, _, _ = autotune.tune(
        ctx, lambda: ctx.krylov_schur_batched(descs[:tune_count], vt, 10, 60, 20, 1e-8, 300),
        reps=1, candidates={key: autotune.BATCHED_CANDIDATES[key]})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rc, infos = ctx.krylov_schur_batched(descs, v0, 10, 60, 20, 1e-8, 300, use_graph=True)
    dt = time.perf_counter() - t0
    st = [i["status"] for i in infos]
    rs = [i["restarts"] for i in infos]
    return {"instances": count, "time_s": round(dt, 3), "converged": st.count(0),
            "restarts_max": max(rs), "restarts_mean": round(float(np.mean(rs)), 2),
            "matvecs_total": int(sum(i["matvecs"] for i in infos)),
            "instances_per_s": round(count / dt, 2), "status": rc,
            "batch_reduce_rows": best[key]}


def batched_gmres_leg(torch, ctx, binding, synth, count=128):
    """Batched GMRES: `count` 2-D convection-diffusion systems of uneven size (grids
    32..128 per side) and restart length (20..60), v ~ U(0,30)^2, b ~ U(0,1), to a 1e-8
    true relative residual: time to solve them all in one batch (autotuned rows per
    reduction workgroup), against the single-instance FP64 gmres_solve looping over the
    same systems on the same GPU."""
    from paper_2104_01253_amd import autotune
    inst = synth.gmres_batched_instances(count)
    descs = [binding.stencil2d(p.grid, p.D, p.vel) for p, _, _ in inst]
    rs = [r for _, r, _ in inst]
    bd = torch.from_numpy(np.concatenate([b for _, _, b in inst])).cuda()
    x = torch.zeros_like(bd)

    def batch():
        x.zero_()
        return ctx.gmres_batched(descs, rs, bd, x, rtol=1e-8)
    key = binding.TUNE_BATCH_REDUCE_ROWS
    default = ctx.get_tuning(key)
    best, _, _ = autotune.tune(ctx, batch, reps=1,
                               candidates={key: autotune.BATCHED_CANDIDATES[key]})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, infos = batch()
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    ctx.set_tuning(key, default)
    xs, off, t_single, it_single = [], 0, 0.0, 0
    for (p, r, b), d in zip(inst, descs):
        op = binding.stencil_op(p.grid, p.D, p.vel)
        bi = bd[off:off + p.m]
        xi = torch.zeros(p.m, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rci, ii = ctx.gmres(op, bi, xi, restart=r, rtol=1e-8)
        t_single += time.perf_counter() - t1
        it_single += ii["iters"]
        off += p.m
    its = [i["iters"] for i in infos]
    return {"instances": count, "rows": int(sum(p.m for p, _, _ in inst)),
            "time_to_1e-8_s": round(tb, 4), "single_instance_loop_s": round(t_single, 4),
            "speedup_vs_single": round(t_single / tb, 2),
            "converged": sum(i["status"] == 0 for i in infos),
            "iters_total": int(sum(its)), "iters_max": int(max(its)),
            "iters_total_single": int(it_single),
            "max_relres_true": max(i["relres_true"] for i in infos),
            "batch_reduce_rows": best[key], "status": rc}


def learned_guess_leg(torch, ctx, binding, synth, count=16):
    """GMRES(50) to 1e-8 on held-out instances of the 256 x 256 variable-coefficient
    family, from x0 = 0 and from the trained network's guess (inference and the
    guard included in the timed region)."""
    from paper_2104_01253_amd import guess
    if not os.path.exists(guess.DEFAULT_WEIGHTS):
        return {"status": "no trained weights"}
    model = guess.GuessModel(ctx, max_batch=count)
    model.load(guess.DEFAULT_WEIGHTS)
    probs = synth.varcoef_instances(count, seed=777, n=guess.N)
    rows = []
    for p in probs:
        b = torch.from_numpy(synth.varcoef_rhs(p)).cuda()
        prm = torch.from_numpy(guess.params_of(p)).cuda()
        dop = guess.DeviceOp(p)
        _, rc0, i0, t_zero = guess.solve(ctx, p, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x0 = model.predict(b[None], prm[None])[0].contiguous()
        kept, ratio = ctx.guess_guard(dop.op, b, x0, 10.0)
        t_inf = time.perf_counter() - t0
        _, rc1, i1, t_g = guess.solve(ctx, p, b, x0=x0)
        rows.append((t_zero, t_inf + t_g, i0["iters"], i1["iters"], kept, ratio, rc0, rc1))
    a = np.array([r[:4] for r in rows], dtype=float)
    return {"instances": count, "zero_guess_s_mean": round(float(a[:, 0].mean()), 4),
            "learned_guess_s_mean": round(float(a[:, 1].mean()), 4),
            "speedup": round(float(a[:, 0].sum() / a[:, 1].sum()), 3),
            "iters_zero_mean": float(a[:, 2].mean()), "iters_guess_mean": float(a[:, 3].mean()),
            "guesses_kept": int(sum(r[4] for r in rows)),
            "residual_ratio_mean": round(float(np.mean([r[5] for r in rows])), 3),
            "status": [int(r[7]) for r in rows]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=2_000_000)
    ap.add_argument("--n", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-legs", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the path would shard by row blocks with one small all-reduce per step); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_01253_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    m, n = args.m, args.n
    log(f"[bench] generating B {m} x {n}, kappa ~ 1e8")
    B = synth.tall_skinny(m, n, 8.0)
    Bd = binding.colmajor_from_numpy(B)
    Qd = binding.colmajor_empty(m, n)
    ctx = binding.Context(0)

    def qr_once():
        _, rc, _ = ctx.qr(Bd, Qd)
        assert rc == binding.OK, rc

    log(f"[bench] warmup {args.warmup} (+ autotuning of the launch shapes)")
    for _ in range(args.warmup):
        qr_once()
    tuned = {}
    # the launch shapes are tuned for the QR; the Arnoldi, GMRES and Krylov-Schur legs
    # below run with the library's defaults again
    keys = (binding.TUNE_FUSED_WAVES, binding.TUNE_REDUCE_GRID, binding.TUNE_FUSED_MIN_J,
            binding.TUNE_FUSED_PAIR_SLOTS)
    defaults = {k: ctx.get_tuning(k) for k in keys}
    if not args.no_tune:
        from paper_2104_01253_amd import autotune
        # the one-pass crossover is fixed at J = 4, the measured optimum (fused passes
        # from J = 2-4 are fastest at this shape), so that the counter records taken at
        # the same setting describe the timed launches
        cands = dict(autotune.CANDIDATES)
        cands[binding.TUNE_FUSED_MIN_J] = (4,)
        best, best_ms, _ = autotune.tune(ctx, qr_once, reps=1, candidates=cands, refine=4)
        names = {binding.TUNE_FUSED_WAVES: "fused_waves", binding.TUNE_REDUCE_GRID: "reduce_grid",
                 binding.TUNE_FUSED_MIN_J: "fused_min_j",
                 binding.TUNE_FUSED_PAIR_SLOTS: "fused_pair_slots"}
        tuned = {names[k]: v for k, v in best.items()}
        log(f"[bench] autotuned {tuned} ({best_ms:.2f} ms)")
    log(f"[bench] timing {args.steps} factorizations")
    T = timed(torch, qr_once, args.steps)
    ms_per_step = T / args.steps * 1e3
    value = n * args.steps / T
    # kernel durations: the same K factorizations again with HIP events around each launch
    ctx.profile(True)
    ctx.profile_read(reset=True)
    T_prof = timed(torch, qr_once, args.steps)
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    prof = {k: v for k, v in prof.items() if v["launches"] > 0}
    dom, roof = roofline(prof)
    alg_bytes_step = sum(v["bytes"] for v in prof.values()) / args.steps
    log(f"[bench] qr {ms_per_step:.3f} ms/factorization, {value:.1f} steps/s; "
        f"dominant {dom} {roof['achieved']} GB/s")
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"dcgs2_qr: B = G diag(logspace(0,-8,{n})) V, m={m}, n={n}, "
                               "fp64, resident in HBM; one step = one factorization",
                   "m": m, "n": n, "cond": 1e8, "launch_shapes": tuned},
        "hbm_gbps_step": round(alg_bytes_step / (ms_per_step * 1e-3) / 1e9, 1),
        "alg_bytes_per_step": alg_bytes_step,
        "profiled_ms_per_step": round(T_prof / args.steps * 1e3, 4),
        "kernels": {k: {"launches": v["launches"], "avg_us": round(v["total_ms"] / v["launches"] * 1e3, 2),
                        "gbps": round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1) if v["total_ms"] > 0 else None}
                    for k, v in prof.items()},
        "roofline": roof,
    }
    if not args.no_legs:
        # the comparator (Alg. cgs2, three reductions per column) on the same B
        def cgs2_once():
            _, rc, _ = ctx.cgs2_qr(Bd, Qd)
            assert rc == binding.OK, rc
        cgs2_once()
        Tc = timed(torch, cgs2_once, 3) / 3
        out["cgs2_qr"] = {"steps_per_s": round(n / Tc, 1), "ms": round(Tc * 1e3, 3),
                          "dcgs2_speedup": round(Tc / (ms_per_step * 1e-3), 3)}
        # the column-by-column MGS comparator (n(n+1)/2 reductions), once
        mgs_once = lambda: ctx.mgs_qr(Bd, Qd)
        Tm = timed(torch, mgs_once, 1)
        out["mgs_qr"] = {"steps_per_s": round(n / Tm, 1), "ms": round(Tm * 1e3, 3),
                         "dcgs2_speedup": round(Tm / (ms_per_step * 1e-3), 3)}
        # FP32-stored basis, FP64 reductions (same B)
        Q32 = binding.colmajor_empty(m, n, dtype=torch.float32)

        def q32_once():
            _, rc, _ = ctx.qr(Bd, Q32)
            assert rc == binding.OK, rc
        q32_once()
        T32 = timed(torch, q32_once, 3) / 3
        ctx.profile(True)
        ctx.profile_read(reset=True)
        q32_once()
        p32 = {k: v for k, v in ctx.profile_read(reset=True).items() if v["launches"] > 0}
        ctx.profile(False)
        _, roof32 = roofline(p32, TRAFFIC_FILE_Q32)
        b32 = sum(v["bytes"] for v in p32.values())
        out["qr_fp32_basis"] = {"steps_per_s": round(n / T32, 1), "ms": round(T32 * 1e3, 3),
                                "hbm_gbps": round(b32 / T32 / 1e9, 1), "roofline": roof32}
        del Q32
        log(f"[bench] cgs2 {out['cgs2_qr']}, mgs {out['mgs_qr']}, fp32 basis {out['qr_fp32_basis']}")
        out["qr_row_block_250k"] = row_block_leg(torch, ctx, binding, B, n)
        log(f"[bench] one GPU's row block of an 8-way split {out['qr_row_block_250k']}")
    del Bd, Qd
    torch.cuda.empty_cache()
    for k, v in defaults.items():
        ctx.set_tuning(k, v)

    if not args.no_legs:
        prob, b = synth.gmres_cd3d(128)
        op = binding.stencil_op(prob.grid, prob.D, prob.vel)
        bd = torch.from_numpy(b).cuda()
        Qa = binding.colmajor_empty(prob.m, n + 1)

        def arn_once():
            _, rc, _ = ctx.arnoldi(op, bd, n, Qa)
            assert rc == binding.OK, rc
        arn_once()
        Ta = timed(torch, arn_once, 3) / 3
        ctx.profile(True)
        ctx.profile_read(reset=True)
        arn_once()
        pa = ctx.profile_read(reset=True)
        ctx.profile(False)
        abytes = sum(v["bytes"] for v in pa.values())
        # per kernel, as the paper reports its two orthogonalisation kernels (MvTransMv,
        # the reduction, and MvTimesMatAddMv, the update) separately (Sec. 7)
        out["arnoldi_128cube_n100"] = {
            "steps_per_s": round(n / Ta, 1), "ms": round(Ta * 1e3, 3),
            "hbm_gbps": round(abytes / Ta / 1e9, 1),
            "roofline_by_kernel": {"bound": "hbm", "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                   **{k: kernel_roof(v, measured_traffic(k, TRAFFIC_FILE_ARNOLDI))
                                      for k, v in pa.items() if v["launches"] > 0}}}
        del Qa
        x = torch.zeros(prob.m, dtype=torch.float64, device="cuda")

        def gm_once():
            x.zero_()
            return ctx.gmres(op, bd, x, restart=50, rtol=1e-8)
        gm_once()
        t0 = time.perf_counter()
        rc, info = gm_once()
        tg = time.perf_counter() - t0
        # algorithmic bytes of the same solve's expansion kernels (the per-cycle solution
        # update and residual, about 2 % more, are not counted), over the unprofiled
        # wall time
        ctx.profile(True)
        ctx.profile_read(reset=True)
        gm_once()
        gbytes = sum(v["bytes"] for v in ctx.profile_read(reset=True).values())
        ctx.profile(False)
        out["gmres50_128cube_fp64"] = {"time_to_1e-8_s": round(tg, 4), "iters": info["iters"],
                                       "cycles": info["cycles"], "relres_true": info["relres_true"],
                                       "expansion_gbps": round(gbytes / tg / 1e9, 1),
                                       "expansion_gb_per_iter": round(gbytes / max(info["iters"], 1) / 1e9, 3),
                                       "status": rc}
        ctx.set_basis_precision(32)
        gm_once()
        t0 = time.perf_counter()
        rc, info = gm_once()
        tg32 = time.perf_counter() - t0
        ctx.set_basis_precision(64)
        out["gmres50_128cube_fp32_basis"] = {"time_to_1e-8_s": round(tg32, 4), "iters": info["iters"],
                                             "relres_true": info["relres_true"], "status": rc,
                                             "speedup_vs_fp64": round(tg / tg32, 3)}
        ks = synth.cd2d(128, vel=(25.0, 40.0))
        kop = binding.stencil_op(ks.grid, ks.D, ks.vel)
        v0 = torch.from_numpy(synth.normal_vector(ks.m, 1)).cuda()
        t0 = time.perf_counter()
        ev, rc, kinfo = ctx.krylov_schur(kop, v0, nev=10, ncv=60, keep=20, tol=1e-8)
        out["krylov_schur_128sq"] = {"time_s": round(time.perf_counter() - t0, 4),
                                     "restarts": kinfo["restarts"], "matvecs": kinfo["matvecs"],
                                     "status": rc}
        log(f"[bench] legs: arnoldi {out['arnoldi_128cube_n100']}, gmres {out['gmres50_128cube_fp64']}")
        out["krylov_schur_batched_512"] = batched_ks_leg(torch, ctx, binding, synth)
        log(f"[bench] batched KS {out['krylov_schur_batched_512']}")
        out["gmres_batched_128"] = batched_gmres_leg(torch, ctx, binding, synth)
        log(f"[bench] batched GMRES {out['gmres_batched_128']}")
        out["gmres50_learned_guess_256sq"] = learned_guess_leg(torch, ctx, binding, synth)
        log(f"[bench] learned guess {out['gmres50_learned_guess_256sq']}")

    out["roofline"]["achievable"] = calibration(torch)
    # the dominant kernel against what a plain streaming read reaches on this device
    out["roofline"]["frac_of_read"] = round(out["roofline"]["achieved"] /
                                            out["roofline"]["achievable"]["read_gbps"], 4)
    log(f"[bench] calibration {out['roofline']['achievable']}")
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(B, n)
        if not args.no_legs:
            out["cpu_baseline"]["gmres50_128cube"] = cpu_gmres_sample()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
