"""Train the warm-start network on GPU-generated pattern pairs.

Training set: synthetic pairs of 256 x 256 px (FCC bands, pattern centre
(0.5, 0.5, 0.7), 1e4 counts with Poisson noise), misorientation uniform in
0-12 degrees about a random axis, symmetric strain with components uniform
in +-2e-3; the label is the exact shift field of Eq. (2) at the 64 x 64
coarse grid (full-resolution px).  Loss: mean squared endpoint error; Adam,
batch 64.  Evaluation pairs come from a disjoint seed range.

Every step runs in the library (ebsd_gen_pairs, ebsd_cnn_train_step); this
script only schedules them.

    python -m paper_1907_05993_amd.train_cnn --pairs 200000 --out weights.bin

A run can be cut into pieces (--time-limit) and continued (--resume): the
checkpoint (--checkpoint, NumPy .npz written with allow_pickle off) holds the
parameters, Adam's moments and step count, the global step and the position
in the epoch's shuffled order; the learning-rate schedule is a function of the
global step (cosine from --lr to --lr-final over --total-steps), so a resumed
run continues the same schedule.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

TRAIN_CID, EVAL_CID = 100, 101


def log(msg):
    print(msg, flush=True)


def make_specs(cid, start, n, mis=(0.0, 12.0), strain=2e-3):
    from . import synth as S
    return [S.make_spec(cid, start + i, 256, 256, mis_deg=mis, strain=strain) for i in range(n)]


def init_params(seed=0):
    """He-normal 3x3 weights [3][3][cin][cout], zero biases, head N(0, 1/128);
    flat in the library's parameter order."""
    rng = np.random.default_rng(seed)
    convs = [(2, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128), (128, 256), (256, 256),
             (384, 128), (128, 128)]
    parts = []
    for ci, co in convs:
        parts.append(rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), size=9 * ci * co))
        parts.append(np.zeros(co))
    parts.append(rng.normal(0.0, math.sqrt(1.0 / 128), size=256))
    parts.append(np.zeros(2))
    return np.concatenate(parts).astype(np.float32)


def evaluate(net, specs, batch, E):
    """Endpoint errors of the network field against the labels (px, full res),
    and the misfit of the Eq. (2) fit to it that decides the warm start's
    fallback (RMS over the grid points inside the ROI ring, full-res px)."""
    import torch
    errs, mis = [], []
    reg = E.Registrar(E.Params(levels=3, iters=(0, 0, 0), sigma_px=1.0, roi_size=64, n_roi=20, warm_start=2,
                               fallback_residual_px=1e9))
    reg.set_model(net)
    for i in range(0, len(specs), batch):
        ref, test, label = E.gen_pairs(specs[i:i + batch])
        out = net.forward(ref, test)
        d = (out - label).double()
        errs.append(torch.sqrt((d ** 2).sum(-1)).reshape(d.shape[0], -1).cpu().numpy())
        mis.append(reg.register(ref, test, want_field=False)["warm_misfit"].cpu().numpy())
    reg.close()
    e = np.concatenate(errs)
    m = np.concatenate(mis)
    per_pair = np.sqrt((e ** 2).mean(axis=1))
    return {"rms_epe_px": float(np.sqrt((e ** 2).mean())), "median_epe_px": float(np.median(e)),
            "p95_epe_px": float(np.percentile(e, 95)), "pairs_rms_gt_0.5px": float((per_pair > 0.5).mean()),
            "misfit_median_px": float(np.median(m)), "misfit_p95_px": float(np.percentile(m, 95)),
            "pairs_misfit_le_0.5px": float((m <= 0.5).mean())}


def save_checkpoint(path, net, step, epoch, pos):
    params = net.get_params()
    m, v, adam_step = net.get_optimizer()
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=params, adam_m=m, adam_v=v, adam_step=np.int64(adam_step), step=np.int64(step),
             epoch=np.int64(epoch), pos=np.int64(pos))
    os.replace(tmp, path)


def load_checkpoint(path, net):
    with np.load(path, allow_pickle=False) as z:
        net.set_params(z["params"])
        net.set_optimizer(z["adam_m"], z["adam_v"], int(z["adam_step"]))
        return int(z["step"]), int(z["epoch"]), int(z["pos"])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=200000, help="training pairs per epoch")
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=None,
                    help="cosine decay of the learning rate to this value over --total-steps (default: constant)")
    ap.add_argument("--total-steps", type=int, default=0,
                    help="length of the cosine schedule in steps (default: all epochs)")
    ap.add_argument("--eval", type=int, default=2048)
    ap.add_argument("--init", default=None, help="start from a parameter file (fresh optimizer)")
    ap.add_argument("--resume", default=None, help="continue from a checkpoint (.npz)")
    ap.add_argument("--checkpoint", default=None, help="checkpoint file written during and after the run")
    ap.add_argument("--checkpoint-every", type=float, default=120.0, help="seconds between checkpoints")
    ap.add_argument("--out", required=True)
    ap.add_argument("--time-limit", type=float, default=0.0, help="stop training after this many seconds")
    ap.add_argument("--log-every", type=float, default=20.0, help="seconds between progress lines")
    args = ap.parse_args(argv)

    t0 = time.time()
    train_specs = make_specs(TRAIN_CID, 0, args.pairs)
    eval_specs = make_specs(EVAL_CID, 0, args.eval)
    log(f"[train] {len(train_specs)} training and {len(eval_specs)} evaluation specs in {time.time() - t0:.1f} s")

    import torch
    from . import ebsd as E
    net = E.Cnn(max_batch=args.batch)
    step, ep0, pos0 = 0, 0, 0
    if args.resume:
        step, ep0, pos0 = load_checkpoint(args.resume, net)
        log(f"[train] resumed {args.resume}: step {step}, epoch {ep0}, position {pos0}")
    elif args.init:
        net.load(args.init)
    else:
        net.set_params(init_params(0))
    ev0 = evaluate(net, eval_specs[:256], args.batch, E)
    log(f"[train] before: {ev0}")

    steps_per_epoch = args.pairs // args.batch
    total = args.total_steps or steps_per_epoch * args.epochs
    t_train = time.time()
    last = last_ck = t_train
    losses = []
    stop = False
    step0 = step
    ep, pos = ep0, pos0
    for ep in range(ep0, args.epochs):
        order = np.random.default_rng(1000 + ep).permutation(steps_per_epoch)
        start_pos = pos0 if ep == ep0 else 0
        for pos in range(start_pos, steps_per_epoch):
            b = order[pos]
            specs = train_specs[b * args.batch:(b + 1) * args.batch]
            ref, test, label = E.gen_pairs(specs)
            lr = args.lr
            if args.lr_final is not None:
                frac = min(1.0, step / max(1, total))
                lr = args.lr_final + 0.5 * (args.lr - args.lr_final) * (1.0 + math.cos(math.pi * frac))
            losses.append(net.train_step(ref, test, label, lr=lr))
            step += 1
            now = time.time()
            if now - last >= args.log_every:
                last = now
                log(f"[train] epoch {ep} step {step} loss(last 50) {np.mean(losses[-50:]):.4f} lr {lr:.2e} "
                    f"{(step - step0) / (now - t_train):.1f} steps/s")
            if args.checkpoint and now - last_ck >= args.checkpoint_every:
                last_ck = now
                save_checkpoint(args.checkpoint, net, step, ep, pos + 1)
            if (args.time_limit and now - t_train > args.time_limit) or (args.total_steps and step >= total):
                stop = True
                break
        if stop:
            break
    else:
        ep, pos = args.epochs, -1
    dt = time.time() - t_train
    log(f"[train] {step - step0} steps ({(step - step0) * args.batch} pairs) in {dt:.1f} s, "
        f"{(step - step0) / max(dt, 1e-9):.2f} steps/s; global step {step}")
    if args.checkpoint:
        save_checkpoint(args.checkpoint, net, step, ep, pos + 1)
    net.save(args.out)
    ev = evaluate(net, eval_specs, args.batch, E)
    log(f"[train] after: {ev}")
    log(f"[train] saved {args.out}")
    return ev


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
