"""Autotuner for the launch shapes of libdcgs2 (workgroups per reduction pass,
wavefronts per one-pass QR workgroup).

The knobs change launch shapes only -- never the arithmetic, and the result is
deterministic for each setting -- so the tuner times each candidate on the
caller's own workload and keeps the fastest.  Timing uses HIP events on the
context's stream through torch.

    best = autotune.tune(ctx, lambda: ctx.qr(B, Q))
    best = autotune.tune(ctx, lambda: ctx.krylov_schur_batched(descs, v0, 10, 60, 20, 1e-8, 300),
                         reps=1, candidates=autotune.BATCHED_CANDIDATES)
"""
from __future__ import annotations

import itertools

from . import binding

CANDIDATES = {
    binding.TUNE_REDUCE_GRID: (0, 512, 1024),
    binding.TUNE_FUSED_MIN_J: (0, 4, 8, 16),
    binding.TUNE_FUSED_PAIR_SLOTS: (16, 8, 5, 0),
}

# Knobs of krylov_schur_batched: rows per workgroup of an instance's reduction
# passes, and where the restart's dense work runs (1 host threads, 0 the GPU).
BATCHED_CANDIDATES = {
    binding.TUNE_BATCH_REDUCE_ROWS: (8192, 4096, 2048, 1024),
    binding.TUNE_BATCH_DENSE: (1, 0),
}


def _time(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(ctx: "binding.Context", fn, reps: int = 2, candidates=None, verbose=False,
         refine: int = 0, refine_reps: int = 5):
    """Try every combination of the knobs, leave the fastest set on ctx and return
    (settings dict, best ms, all timings).  With refine > 1 the `refine` fastest
    combinations of the sweep are timed again over `refine_reps` calls each and the
    fastest of those is kept, so that run-to-run noise of a short sweep does not pick
    the setting."""
    import torch
    cands = candidates or CANDIDATES
    keys = list(cands)
    timings = []
    for combo in itertools.product(*(cands[k] for k in keys)):
        for k, v in zip(keys, combo):
            ctx.set_tuning(k, v)
        ms = _time(torch, fn, reps)
        timings.append((dict(zip(keys, combo)), ms))
        if verbose:
            print("autotune", dict(zip(keys, combo)), f"{ms:.3f} ms", flush=True)
    ranked = sorted(timings, key=lambda t: t[1])
    best, best_ms = ranked[0]
    if refine > 1:
        finals = []
        for settings, _ in ranked[:refine]:
            for k, v in settings.items():
                ctx.set_tuning(k, v)
            finals.append((settings, _time(torch, fn, refine_reps)))
            if verbose:
                print("autotune refine", settings, f"{finals[-1][1]:.3f} ms", flush=True)
        best, best_ms = min(finals, key=lambda t: t[1])
    for k, v in best.items():
        ctx.set_tuning(k, v)
    return best, best_ms, timings
