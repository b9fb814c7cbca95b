"""Train and evaluate the K-step surrogate against the plain stepper.

Data: trajectories of the plain stepper itself (the batched persistent kernel)
on 256x256 grids from seeded random / circle / star starts with m in {4,5,6};
a snapshot every K = 100 steps up to T = 2000 gives 20 (phi_k, phi_{k+1})
pairs per trajectory, all kept in HBM.

Training: mini-batches of pairs, MSE of phi + U(phi) against phi_{k+1}, Adam;
forward, backward and update all run in libac's BF16-MFMA kernels.

Inference to T with judge and fallback: each K-block the surrogate advances
every trusted grid; the plain stepper advances the same grids from the same
states (the judge compares the two: interface error <= h and RMS <= l2_bar;
every block by default, a rotating sample as an option) and every grid that
has failed once (the fallback), all in one masked batched launch.  Time-to-T
includes the judge and the fallback.

  python -m paper_2105_09671_amd.sur_train --out weights.npz [--trajectories 4096] [--steps 3000]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import api, workloads
from .surrogate import K_STEPS, Surrogate

HW = 256
L2_BAR = 0.05


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def grids_for(seeds):
    gs = [workloads.surrogate_grid(s, HW) for s in seeds]
    return gs, [workloads.surrogate_initial(g) for g in gs]


def make_trajectories(seeds, blocks: int = 20) -> torch.Tensor:
    """[len(seeds), blocks + 1, HW, HW] FP32 snapshots every K_STEPS steps."""
    gs, fields = grids_for(seeds)
    b = api.Batch(fields, [(g.h, g.dt, g.eps) for g in gs])
    state = b.phi.view(len(seeds), HW, HW)
    out = torch.empty(len(seeds), blocks + 1, HW, HW, dtype=torch.float32, device="cuda")
    out[:, 0] = state
    for k in range(1, blocks + 1):
        b.step(K_STEPS)
        out[:, k] = state
    torch.cuda.synchronize()
    return out


def init_weights(seed: int, n: int) -> np.ndarray:
    """He-uniform conv weights (sqrt(6/fan_in)), zero biases, head at 0.1x, drawn
    with the seeded SplitMix64 input generator (layer order of the network)."""
    from . import inputs
    layers = [(1, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3), (64, 128, 3), (128, 64, 1),
              (128, 64, 3), (64, 32, 1), (64, 32, 3), (32, 1, 1)]
    parts = []
    for li, (cin, cout, k) in enumerate(layers):
        u = inputs.uniform01(seed, 500 + li, cout * k * k * cin)
        scale = math.sqrt(6.0 / (cin * k * k)) * (0.1 if li == len(layers) - 1 else 1.0)
        parts += [scale * (2 * u - 1), np.zeros(cout)]
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == n
    return w


def training_pairs(kinds, blocks: int):
    """(trajectory, block) pairs used for training: every block of every
    trajectory except the first block of a random start -- from raw noise the
    outcome after K steps is set by the exact noise amplified (spinodal
    growth), which no local map can predict; the judge falls back there."""
    return np.array([(t, k) for t, kd in enumerate(kinds) for k in range(blocks)
                     if not (kd == "random" and k == 0)], dtype=np.int64)


def train(data: torch.Tensor, steps: int, batch: int = 32, lr: float = 1e-3, seed: int = 0,
          net: Surrogate | None = None, log_every: int = 500, kinds=None):
    """Adam on MSE of random (trajectory, block) pairs; cosine-decayed lr."""
    ntraj, nb = data.shape[0], data.shape[1] - 1
    pairs = training_pairs(kinds or ["circle"] * ntraj, nb)
    if net is None:
        net = Surrogate(batch, HW)
        net.set_weights(init_weights(seed, net.n))
    rng = np.random.RandomState(seed)
    x = torch.empty(batch, HW, HW, device="cuda")
    y = torch.empty_like(x)
    hist = []
    t0 = time.perf_counter()
    for it in range(steps):
        sel = pairs[rng.randint(0, len(pairs), batch)]
        ti = torch.from_numpy(sel[:, 0]).cuda()
        ki = torch.from_numpy(sel[:, 1]).cuda()
        x.copy_(data[ti, ki])
        y.copy_(data[ti, ki + 1])
        a = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * it / max(steps, 1))))
        loss = net.train_step(x, y, a)
        if it % log_every == 0 or it == steps - 1:
            lv = float(loss.item())
            hist.append((it, lv))
            log("train step %d loss %.3e lr %.2e (%.1f s)" % (it, lv, a, time.perf_counter() - t0))
    torch.cuda.synchronize()
    return net, hist, time.perf_counter() - t0


def validate(net: Surrogate, data: torch.Tensor, kinds) -> dict:
    """Mean squared error of phi + U(phi) against the stepper, per kind and block."""
    out = {}
    nb = data.shape[1] - 1
    B = net.batch_max
    pred = torch.empty(B, HW, HW, device="cuda")
    for kd in sorted(set(kinds)):
        idx = [i for i, x in enumerate(kinds) if x == kd]
        row = []
        for k in range(nb):
            se, n = 0.0, 0
            for s in range(0, len(idx), B):
                sub = torch.tensor(idx[s:s + B], device="cuda")
                x = data[sub, k].contiguous()
                net.infer(x, pred[:len(sub)])
                se += float(((pred[:len(sub)] - data[sub, k + 1]) ** 2).sum().item())
                n += len(sub) * HW * HW
            row.append(se / n)
        out[kd] = row
    return out


# FLOPs of one forward pass on a 256 x 256 grid (2 per multiply-add), the two
# 1x1 layers counted at the low resolution where they are evaluated
FORWARD_FLOP = 2 * sum(ci * co * k * k * (HW // f) ** 2 for ci, co, k, f in [
    (1, 32, 3, 1), (32, 32, 3, 1), (32, 64, 3, 2), (64, 64, 3, 2), (64, 128, 3, 4),
    (128, 64, 1, 4), (128, 64, 3, 2), (64, 32, 1, 2), (64, 32, 3, 1), (32, 1, 1, 1)])


def forward_rate(net: Surrogate, n: int, reps: int = 3) -> dict:
    """Time the inference forward pass alone on n grids: ms per call and TFLOP/s."""
    x = torch.zeros(n, HW, HW, device="cuda")
    y = torch.empty_like(x)
    B = net.batch_max
    for s in range(0, n, B):
        net.infer(x[s:s + B], y[s:s + B])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        for s in range(0, n, B):
            net.infer(x[s:s + B], y[s:s + B])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"grids": n, "ms": round(ms, 3), "TFLOPs": round(n * FORWARD_FLOP / ms / 1e9, 1),
            "flop_per_grid": FORWARD_FLOP}


def evaluate(net: Surrogate, seeds, T_blocks: int = 20, sample_every: int = 1,
             l2_bar: float = L2_BAR, return_state: bool = False) -> dict:
    """Surrogate + judge + fallback to T versus the plain stepper, on held-out seeds.

    Per K-block the surrogate predicts every trusted grid.  The judged grids
    -- every trusted grid when sample_every == 1 (the default), else every grid
    in the first block and then a rotating 1/sample_every of the trusted ones --
    are also advanced by the plain stepper from the same state (the judge), in
    one masked batched launch together with every untrusted grid (the
    fallback).  A judged prediction within interface error h and RMS l2_bar of
    the plain result is kept; otherwise the plain result is kept and the grid
    is untrusted (stepped plainly) from then on.  With sample_every > 1 the
    predictions of unjudged blocks are taken unchecked.  Time-to-T includes the
    surrogate, the judge and the fallback.  The final states are compared with
    a plain run to T (per grid: interface error and RMS)."""
    if sample_every < 1:
        raise ValueError("sample_every must be >= 1")
    gs, fields = grids_for(seeds)
    params = [(g.h, g.dt, g.eps) for g in gs]
    N = len(seeds)
    h = gs[0].h
    # plain reference to T (also the accuracy reference), timed
    plain = api.Batch(fields, params)
    plain.step(K_STEPS * T_blocks)                      # builds the plan + graph
    torch.cuda.synchronize()
    for v, f in zip(plain.views(), fields):
        v.copy_(torch.from_numpy(f).float())
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    plain.step(K_STEPS * T_blocks)
    s1.record()
    torch.cuda.synchronize()
    plain_ms = s0.elapsed_time(s1)
    ref_T = plain.phi.view(N, HW, HW).clone()
    del plain

    fb = api.Batch(fields, params)
    state = fb.phi.view(N, HW, HW)
    active = torch.zeros(N, dtype=torch.int32, device="cuda")
    fb.step_masked(K_STEPS, active)                     # builds the plan; steps nothing
    pred = torch.empty_like(state)
    B = net.batch_max
    net.infer(state[:min(N, B)].contiguous(), pred[:min(N, B)])     # warm-up
    # warm-up of the other calls the timed loop makes (first-use costs: module
    # loading, the judge's workspace), on scratch copies
    dev_ = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).cuda()
    scratch = state[:min(N, B)].clone()
    api.judge2d(pred[:len(scratch)].contiguous(), scratch, h)
    scratch.index_copy_(0, dev_(np.arange(len(scratch))), pred.index_select(0, dev_(np.arange(len(scratch)))))
    del scratch
    torch.cuda.synchronize()
    # book-keeping on the host: which grids are trusted, judged, stepped
    trusted = np.ones(N, dtype=bool)
    sur_blocks = np.zeros(N, dtype=np.int64)           # surrogate predictions kept, per grid
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).cuda()
    judged, judged_fail = 0, 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(T_blocks):
        tidx = np.nonzero(trusted)[0]
        nt = len(tidx)
        if sample_every == 1 or k == 0:
            spos = np.arange(nt)
        else:
            spos = np.arange(k % sample_every, nt, sample_every)
        kpos = np.setdiff1d(np.arange(nt), spos)
        samp = tidx[spos]
        if nt == N:
            x, out = state, pred                        # every grid trusted: no gather
        elif nt:
            x = state.index_select(0, dev(tidx))
            out = torch.empty_like(x)
        for s in range(0, nt, B):
            net.infer(x[s:s + B], out[s:s + B])
        act = ~trusted
        act[samp] = True
        active.copy_(torch.from_numpy(act.astype(np.int32)))
        fb.step_masked(K_STEPS, active)                 # plain: judged + untrusted, in place
        if len(samp):
            iface, l2 = api.judge2d(out.index_select(0, dev(spos)), state.index_select(0, dev(samp)), h)
            ok = ((iface <= h) & (l2 <= l2_bar)).cpu().numpy()
            judged += len(samp)
            judged_fail += int((~ok).sum())
            trusted[samp[~ok]] = False
            keep = spos[ok]                             # accepted predictions replace the judge's state
            if len(keep):
                state.index_copy_(0, dev(tidx[keep]), out.index_select(0, dev(keep)))
                sur_blocks[tidx[keep]] += 1
        if len(kpos):
            state.index_copy_(0, dev(tidx[kpos]), out.index_select(0, dev(kpos)))
            sur_blocks[tidx[kpos]] += 1
    e1.record()
    torch.cuda.synchronize()
    sur_ms = e0.elapsed_time(e1)
    iface_T, l2_T = api.judge2d(state.contiguous(), ref_T, h)
    iface_T, l2_T = iface_T.cpu().numpy(), l2_T.cpu().numpy()
    kinds = [g.kind for g in gs]
    ok_T = (iface_T <= h) & (l2_T <= l2_bar)
    by_kind = {kd: {"final_ok": float(np.mean(ok_T[[i for i, x in enumerate(kinds) if x == kd]])),
                    "trusted_at_T": float(np.mean(trusted[[i for i, x in enumerate(kinds) if x == kd]]))}
               for kd in sorted(set(kinds))}
    res = {"grids": N, "T_steps": K_STEPS * T_blocks, "plain_ms": round(plain_ms, 3),
           "surrogate_ms": round(sur_ms, 3), "speedup": round(plain_ms / sur_ms, 4),
           "forward": forward_rate(net, N),
           "surrogate_grid_blocks": int(sur_blocks.sum()), "grid_blocks": N * T_blocks,
           "judged": judged, "judged_failures": judged_fail, "sample_every": sample_every,
           "final_ok_fraction": float(np.mean(ok_T)), "by_kind": by_kind,
           "final_iface_max_over_h": float(np.max(np.minimum(iface_T / h, 1e9))),
           "final_iface_median_over_h": float(np.median(np.minimum(iface_T / h, 1e9))),
           "final_l2_max": float(np.max(l2_T)), "final_l2_median": float(np.median(l2_T))}
    if return_state:
        res["state"], res["ref_T"] = state.clone(), ref_T
        res["per_grid"] = {"iface": iface_T, "l2": l2_T, "trusted": trusted.copy(),
                           "surrogate_blocks": sur_blocks, "kinds": kinds}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="", help="weights file (.npz) to write")
    ap.add_argument("--trajectories", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=30000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval", type=int, default=256, help="held-out grids (seeds 100000..)")
    ap.add_argument("--init", default="", help="start from these weights (.npz)")
    ap.add_argument("--evaluate-only", action="store_true",
                    help="skip training: evaluate the weights given by --init")
    args = ap.parse_args()
    if args.evaluate_only:
        ev = Surrogate(min(256, args.eval), HW)
        ev.set_weights(np.load(args.init)["weights"])
        print(json.dumps(evaluate(ev, list(range(100000, 100000 + args.eval)))), flush=True)
        return
    t0 = time.perf_counter()
    seeds = list(range(args.trajectories))
    kinds = [workloads.surrogate_grid(s, HW).kind for s in seeds]
    data = make_trajectories(seeds)
    log("trajectories %s in %.1f s" % (tuple(data.shape), time.perf_counter() - t0))
    net = None
    if args.init:
        net = Surrogate(args.batch, HW)
        net.set_weights(np.load(args.init)["weights"])
    net, hist, tsec = train(data, args.steps, args.batch, args.lr, net=net, kinds=kinds)
    del data
    w = net.get_weights()
    vseeds = list(range(200000, 200064))
    vkinds = [workloads.surrogate_grid(s, HW).kind for s in vseeds]
    vdata = make_trajectories(vseeds)
    val = validate(net, vdata, vkinds)
    del vdata
    log("validation MSE per kind and block: %s" % json.dumps(
        {k: ["%.2e" % v for v in row] for k, row in val.items()}))
    np.savez(args.out, weights=w, history=np.array(hist), steps=args.steps,
             trajectories=args.trajectories, batch=args.batch, lr=args.lr, train_seconds=tsec)
    log("saved %s (%d params, %.1f s of training)" % (args.out, w.size, tsec))
    ev = Surrogate(min(256, args.eval), HW)
    ev.set_weights(w)
    res = evaluate(ev, list(range(100000, 100000 + args.eval)))
    res["train_seconds"] = round(tsec, 2)
    res["final_loss"] = hist[-1][1]
    res["validation_mse"] = val
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
