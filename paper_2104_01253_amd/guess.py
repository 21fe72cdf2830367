"""Learned initial guess for GMRES on the variable-coefficient convection-diffusion
family: data generation, training and inference on the device.

    python -m paper_2104_01253_amd.guess train --count 4096 --out <weights.npz>

Pipeline for one instance (every numeric step is a libdcgs2 kernel; this module
marshals arguments, assembles the operator's CSR arrays and batches samples):

  features  f = [R(b)/s, xi, v/10, 0...]       (dcgs2_guess_features)
  network   y = MLP(f)                          (dcgs2_mlp_forward, FP32 matrix cores)
  guess     x0 = (s / gain) P(y)                (dcgs2_guess_prolong)
  fallback  x0 = 0 unless ||b - A x0|| < 10 ||b||   (dcgs2_guess_guard)

Training data are GMRES(50) solutions of seeded instances of the family
(solved by this library); the targets are R(x)/s, the loss the mean squared
error, the optimiser Adam.
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np

from . import binding, synth

N, NC = 256, 32
NPARAM = len(synth.KL_MODES) + 2            # xi and the two velocity components
FDIM = NC * NC + 16                         # features padded to a multiple of 16
WIDTHS = (FDIM, 512, 512, NC * NC)
# Targets are gain R(x)/s: with s the RMS of R(b) they have an RMS near 1/70 on this
# family, so gain = 64 brings them to order one, the scale of a He-initialised
# network's outputs (unscaled targets leave the network at its initial output).
GAIN = 64.0
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                               "guess_mlp_256.npz")


# ---- operator of the family -----------------------------------------------------------
def diffusion(prob, x, y):
    """D(x, y) = exp(sum_k xi_k a_k phi_k(x, y)) with the family's KL modes."""
    s = np.zeros(np.broadcast(x, y).shape)
    for (p, q), xi in zip(synth.KL_MODES, prob.xi):
        s = s + xi / (p * p + q * q) * 2.0 * np.sin(p * np.pi * x) * np.sin(q * np.pi * y)
    return np.exp(s)


def diffusion_grid(prob, tx, ty):
    """diffusion() on the tensor grid [iy, ix] = (tx[ix], ty[iy]) (the same values,
    element by element: the modes are separable, so the sines are taken on the axes)."""
    s = np.zeros((ty.shape[0], tx.shape[0]))
    for (p, q), xi in zip(synth.KL_MODES, prob.xi):
        s = s + (xi / (p * p + q * q) * 2.0 * np.sin(p * np.pi * tx))[None, :] \
            * np.sin(q * np.pi * ty)[:, None]
    return np.exp(s)


def varcoef_csr(prob):
    """CSR arrays (rowptr int32, colind int32, val float64) of -div(D grad u) + v.grad u:
    face-centred diffusion, central convection, Dirichlet, x fastest, columns sorted."""
    n = prob.n
    h = 1.0 / (n + 1)
    t = np.arange(1, n + 1) * h
    De = diffusion_grid(prob, t + h / 2, t)            # [iy, ix]
    Dw = diffusion_grid(prob, t - h / 2, t)
    Dn = diffusion_grid(prob, t, t + h / 2)
    Ds = diffusion_grid(prob, t, t - h / 2)
    vx, vy = prob.vel
    ih2 = 1.0 / (h * h)
    cx = vx / (2.0 * h)
    cy = vy / (2.0 * h)
    # neighbour order by column index: south, west, centre, east, north
    vals = np.stack([-Ds * ih2 - cy, -Dw * ih2 - cx, (De + Dw + Dn + Ds) * ih2,
                     -De * ih2 + cx, -Dn * ih2 + cy], axis=-1)        # [iy, ix, 5]
    iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    r = iy * n + ix
    cols = np.stack([r - n, r - 1, r, r + 1, r + n], axis=-1)
    ok = np.stack([iy > 0, ix > 0, np.ones_like(ix, bool), ix < n - 1, iy < n - 1], axis=-1)
    counts = ok.reshape(-1, 5).sum(axis=1)
    rowptr = np.zeros(n * n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(counts)
    return rowptr, cols.reshape(-1, 5)[ok.reshape(-1, 5)].astype(np.int32), \
        vals.reshape(-1, 5)[ok.reshape(-1, 5)].astype(np.float64)


def params_of(prob) -> np.ndarray:
    return np.array(list(prob.xi) + [prob.vel[0] / 10.0, prob.vel[1] / 10.0], dtype=np.float32)


class DeviceOp:
    """CSR operator of one instance on the device (keeps its tensors alive)."""

    def __init__(self, prob, device="cuda"):
        import torch
        rp, ci, va = varcoef_csr(prob)
        self.rowptr = torch.from_numpy(rp).to(device)
        self.colind = torch.from_numpy(ci).to(device)
        self.val = torch.from_numpy(va).to(device)
        self.op = binding.csr_op(self.rowptr, self.colind, self.val)


# ---- model ----------------------------------------------------------------------------
def he_init(widths, seed):
    g = synth.rng(seed)
    return [(g.standard_normal((a, b)) * np.sqrt(2.0 / a), np.zeros(b))
            for a, b in zip(widths[:-1], widths[1:])]


class GuessModel:
    def __init__(self, ctx: binding.Context, max_batch=256, widths=WIDTHS, seed=0):
        self.ctx = ctx
        self.mlp = binding.MLP(ctx, widths, max_batch)
        self.mlp.set_params(self.mlp.pack(he_init(widths, seed)))

    def predict(self, b, prm):
        """b: CUDA float64 (count, N*N); prm: CUDA float32 (count, NPARAM) -> x0 (count, N*N)."""
        feat, scale = self.ctx.guess_features(b, prm, N, NC, FDIM)
        y = self.mlp.forward(feat)
        return self.ctx.guess_prolong(y, scale, N, NC, GAIN)

    def save(self, path, **meta):
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        np.savez(path, params=self.mlp.get_params(), widths=np.array(self.mlp.widths),
                 **{k: np.asarray(v) for k, v in meta.items()})

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            if tuple(int(w) for w in z["widths"]) != tuple(self.mlp.widths):
                raise ValueError("weights file has other layer widths")
            self.mlp.set_params(z["params"])


# ---- data and training ------------------------------------------------------------------
def solve(ctx, prob, b_dev, x0=None, rtol=1e-8, restart=50, max_iters=20000):
    """GMRES(restart) on one instance; returns (x, rc, info, seconds)."""
    import torch
    dop = DeviceOp(prob, b_dev.device)
    x = torch.zeros_like(b_dev) if x0 is None else x0.clone()
    # the inputs are ready on torch's stream (the library runs on its own); other
    # threads' solver streams are not waited for
    torch.cuda.current_stream().synchronize()
    t0 = time.perf_counter()
    rc, info = ctx.gmres(dop.op, b_dev, x, restart=restart, rtol=rtol, max_iters=max_iters)
    return x, rc, info, time.perf_counter() - t0


def generate(ctx, count, seed, rtol=1e-5, max_iters=6000, log=None, workers=1):
    """Features and targets of the solved instances among `count` seeded ones
    (device tensors, in instance order).  An instance whose GMRES(50) does not reach
    rtol within max_iters iterations is left out (restarted GMRES can stagnate on
    this family); the coarse targets need far less accuracy than rtol.

    workers > 1 solves contiguous slices of the instances concurrently, each in a host
    thread of its own with a context on a stream of its own (default priority; the
    thread's torch work runs on the same stream): one 256 x 256 solve fills only a
    small part of the GPU.  The result does not depend on the number of workers."""
    import threading
    import torch
    probs = synth.varcoef_instances(count, seed=seed, n=N)
    workers = max(1, min(int(workers), count))
    rows = [None] * count                   # (features, targets) or None, per instance
    iters = [0] * count
    done = [0]
    lock = threading.Lock()
    errors = []

    def run(lo, hi, c, stream=None):
        try:
            torch.cuda.set_device(0)
            if stream is not None:
                with torch.cuda.stream(stream):
                    solve_range(lo, hi, c)
            else:
                solve_range(lo, hi, c)
        except Exception as e:              # re-raised in the calling thread
            errors.append(e)

    def solve_range(lo, hi, c):
        for i in range(lo, hi):
            p = probs[i]
            b = torch.from_numpy(synth.varcoef_rhs(p)).cuda()
            prm = torch.from_numpy(params_of(p)).cuda()
            x, rc, info, _ = solve(c, p, b, rtol=rtol, max_iters=max_iters)
            iters[i] = info["iters"]
            if rc == binding.OK:
                f, sc = c.guess_features(b[None], prm[None], N, NC, FDIM)
                rows[i] = (f[0].clone(), c.guess_targets(x[None], sc, N, NC, GAIN)[0].clone())
            with lock:
                done[0] += 1
                if log and done[0] % 256 == 0:
                    kept = sum(r is not None for r in rows)
                    log(f"solved {done[0]}/{count}: kept {kept}, median "
                        f"{int(np.median([t for t in iters if t]))} iterations")

    if workers == 1:
        run(0, count, ctx)
    else:
        bounds = [count * w // workers for w in range(workers + 1)]
        streams = [torch.cuda.Stream() for _ in range(workers)]
        ctxs = [binding.Context(0, stream=st.cuda_stream) for st in streams]
        try:
            ts = [threading.Thread(target=run, args=(bounds[w], bounds[w + 1], ctxs[w],
                                                     streams[w]))
                  for w in range(workers)]
            for t in ts:
                t.start()
            for t in ts:
                t.join()
            torch.cuda.synchronize()
        finally:
            for c in ctxs:
                c.close()
    if errors:
        raise errors[0]
    keep = [r for r in rows if r is not None]
    if not keep:
        return (torch.empty((0, FDIM), dtype=torch.float32, device="cuda"),
                torch.empty((0, NC * NC), dtype=torch.float32, device="cuda"))
    out = (torch.stack([r[0] for r in keep]).contiguous(),
           torch.stack([r[1] for r in keep]).contiguous())
    torch.cuda.synchronize()                # before the per-stream rows are freed
    return out


def validate(model, vf, vt):
    """Relative error ||MLP(vf) - vt|| / ||vt|| on a held-out set (chunks of max_batch)."""
    num = den = 0.0
    for s in range(0, vf.shape[0], model.mlp.max_batch):
        y = model.mlp.forward(vf[s:s + model.mlp.max_batch].contiguous())
        t = vt[s:s + model.mlp.max_batch]
        num += float(((y - t) ** 2).sum())
        den += float((t ** 2).sum())
    return (num / max(den, 1e-300)) ** 0.5


def train(model, feats, targs, epochs=60, batch=256, lr=1e-3, seed=0, log=None, val=None):
    """Adam on minibatches; with val = (features, targets) the parameters with the
    lowest validation error (checked every 10 epochs) are kept."""
    import torch
    g = synth.rng(seed)
    count = feats.shape[0]
    hist = []
    best = (float("inf"), None)
    for ep in range(epochs):
        perm = torch.from_numpy(g.permutation(count)).cuda()
        tot, nb = 0.0, 0
        step_lr = lr if ep < int(0.7 * epochs) else 0.1 * lr     # one decay step at 70 %
        for s in range(0, count - batch + 1, batch):
            idx = perm[s:s + batch]
            X = feats.index_select(0, idx).contiguous()
            T = targs.index_select(0, idx).contiguous()
            tot += model.mlp.loss_grad(X, T)
            model.mlp.adam(step_lr)
            nb += 1
        hist.append(tot / max(nb, 1))
        if ep % 10 == 9 or ep == epochs - 1:
            msg = f"epoch {ep + 1}: train mse {hist[-1]:.4e}"
            if val is not None:
                err = validate(model, *val)
                if err < best[0]:
                    best = (err, model.mlp.get_params())
                msg += f", validation relative error {err:.4f}"
            if log:
                log(msg)
    if best[1] is not None:
        model.mlp.set_params(best[1])
    return hist


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--count", type=int, default=4096)
    t.add_argument("--val", type=int, default=256)
    t.add_argument("--epochs", type=int, default=150)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=100)
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--workers", type=int, default=4, help="concurrent solver threads")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)

    def log(msg):
        print(msg, flush=True)

    ctx = binding.Context(0)
    model = GuessModel(ctx)
    t0 = time.perf_counter()
    feats, targs = generate(ctx, a.count, a.seed, log=log, workers=a.workers)
    vf, vt = generate(ctx, a.val, a.seed + 1, log=log, workers=a.workers)
    log(f"data: {time.perf_counter() - t0:.1f} s")
    hist = train(model, feats, targs, a.epochs, lr=a.lr, log=log, val=(vf, vt))
    rel = validate(model, vf, vt)
    log(f"kept parameters: validation relative error {rel:.4f} "
        f"({feats.shape[0]} training and {vf.shape[0]} validation instances)")
    model.save(a.out, train_mse=hist[-1], val_rel=rel, count=a.count, kept=feats.shape[0],
               seed=a.seed, epochs=a.epochs, gain=GAIN)
    log(f"saved {a.out}")


if __name__ == "__main__":
    main()
