"""Train the learned form's network on pairs the method itself generates.

    python -m paper_1203_4874_amd.train_mlp [--pairs 20000] [--holdout 2000] [--out DIR] [--eval-only]
                                            [--checkpoint FILE [--resume]]

Data (seeded, synthetic): 256 x 256 Gaussian-sum scenes, kernel sizes k1, k2
drawn independently from {5, 7, ..., 15} (uniform entries, sum 1, coprime),
noise sigma in {0, 1e-3, 1e-2} in equal shares, S = 2 max(k1, k2), FP32
frames.  Every pair goes through the library's batched deblurring call with
diagnostics on, which returns each sample's spectrum features, null vector
and the averaged kernel spectra.  Targets come from the true kernels:

  * w*: the inverse sine of the angle between the sample's null vector and
    the true kernel slices at that sample, divided by its geometric mean over
    the frame's 2S samples, clipped to [0.1, 10] (a compressed confidence:
    the network's error in log w then moves a weight by a bounded factor);
  * tau*: S times the noise-to-signal ratio of the frame's averaged spectra
    against the true spectra (after the best complex scale), floored at
    1e-12 -- a ridge strength in the units of the assembly's normal matrix.

The network (32 -> 128 -> 128 -> 2, BF16 on the matrix cores) is trained with
the library's own forward / backward / Adam kernels on (features, (log w*,
log tau*)).  The held-out pairs are then deblurred with and without the
network and both kernel errors against the truth are reported (the learned
call includes the noise gate, which keeps the plain kernels on frames with a
noise floor, and the judge that keeps them when the plain method's objective
prefers them).  --eval-only redoes that comparison for the committed network.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

SIZES = (5, 7, 9, 11, 13, 15)
NOISES = (0.0, 1e-3, 1e-2)
SEED = 1004
FRAME = 256


def make_pair(idx: int):
    """One seeded pair of the training set (host, numpy)."""
    r = synth.rng_for(SEED, 0, idx)
    k1, k2 = (int(v) for v in r.choice(SIZES, 2, replace=True))
    noise = NOISES[idx % 3]
    L = synth.gaussian_scene(r, FRAME, FRAME)
    K1, K2 = synth.draw_coprime_pair(r, k1, k2, "uniform")
    B1, B2 = synth.blur_pair(synth.rng_for(SEED, 1, idx), L, K1, K2, noise)
    return dict(B1=B1.astype(np.float32), B2=B2.astype(np.float32), K1=K1, K2=K2, noise=noise,
                S=2 * max(k1, k2))


def true_slices(K1, K2, S):
    """Per-sample true null vectors x* = (u*: k2, v*: k1) of both passes.
    Pass X sample j evaluates along y at w_j; pass Y sample i along x."""
    w = np.exp(-2j * np.pi * np.arange(S) / S)
    out = []
    for axis in (0, 1):
        xs = []
        for j in range(S):
            p2 = (w[j] ** np.arange(K2.shape[axis]))
            p1 = (w[j] ** np.arange(K1.shape[axis]))
            u = p2 @ K2 if axis == 0 else K2 @ p2
            v = p1 @ K1 if axis == 0 else K1 @ p1
            xs.append(np.concatenate([u, v]))
        out.append(xs)
    return out


def true_spectra(K, S):
    """Khat*[i][j] = sum_{y,x} K[y][x] w_j^y w_i^x."""
    k = K.shape[0]
    F = np.exp(-2j * np.pi * np.outer(np.arange(S), np.arange(k)) / S)
    return F @ K.T @ F.T


def targets(diag, K1, K2):
    """(features [2S][32], targets [2S][2]) of one frame from its diagnostics."""
    S, n = diag["S"], diag["n"]
    xs = true_slices(K1, K2, S)
    sin2 = np.zeros((2, S))
    for p in range(2):
        for j in range(S):
            x = diag["sample_vec"][p, j]
            t = xs[p][j]
            c = abs(np.vdot(t, x)) ** 2 / (np.vdot(x, x).real * np.vdot(t, t).real)
            sin2[p, j] = max(1.0 - c, 1e-10)
    w = 1.0 / np.sqrt(sin2)
    w = np.clip(w / np.exp(np.mean(np.log(w))), 0.1, 10.0)
    num = den = 0.0
    for c, K in enumerate((K1, K2)):
        Kt = true_spectra(K, S)
        Kg = diag["khat"][c]
        num += np.vdot(Kt, Kg)
        den += np.vdot(Kt, Kt).real
    scale = num / den
    err = sum(np.linalg.norm(diag["khat"][c] - scale * true_spectra(K, S)) ** 2 for c, K in enumerate((K1, K2)))
    ref = sum(np.linalg.norm(scale * true_spectra(K, S)) ** 2 for K in (K1, K2))
    tau = max(err / ref, 1e-12) * S
    X = diag["sample_features"].reshape(2 * S, 32)
    T = np.stack([np.log(w.reshape(-1)), np.full(2 * S, np.log(tau))], 1)
    return X.astype(np.float32), T.astype(np.float32)


def run_pairs(P, torch, dev, pairs, mlp=None, chunk=128):
    """Deblur pairs grouped by S; returns per-pair (diag, K1, K2) in order."""
    out = [None] * len(pairs)
    groups = {}
    for i, p in enumerate(pairs):
        groups.setdefault(p["S"], []).append(i)
    for S, idx in sorted(groups.items()):
        for c0 in range(0, len(idx), chunk):
            ids = idx[c0:c0 + chunk]
            frames = [(torch.as_tensor(pairs[i]["B1"], device=dev), torch.as_tensor(pairs[i]["B2"], device=dev),
                       FRAME, FRAME) for i in ids]
            kmax = max(max(pairs[i]["K1"].shape[0], pairs[i]["K2"].shape[0]) for i in ids)
            d = P.Deblurrer(FRAME + kmax - 1, FRAME + kmax - 1, kmax, 1, len(ids), P.Precision.MIXED, samples=S,
                            device=dev, diag=True)
            pb = d.prepare_batch(frames, lam=1e-4, mlp=mlp)
            st = pb.run(check=False)
            torch.cuda.synchronize()
            raw = d.diag.cpu().numpy()
            sz = P.diag_size()
            for t, i in enumerate(ids):
                dg = P.decode_diag(raw[t * sz:(t + 1) * sz]) if st[t] == 0 else None
                out[i] = (dg, pb.K1s[t].cpu().numpy(), pb.K2s[t].cpu().numpy())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--holdout", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_1203_4874_amd", "weights"))
    ap.add_argument("--eval-only", action="store_true",
                    help="skip training: compare the committed network with the plain method on the held-out pairs")
    ap.add_argument("--checkpoint", default="",
                    help="file (.npz) for the training state after every epoch (weights, Adam moments, step)")
    ap.add_argument("--resume", action="store_true", help="continue from --checkpoint")
    args = ap.parse_args()

    # the generator processes are forked before anything touches the GPU
    import multiprocessing as mp
    ex = ProcessPoolExecutor(max_workers=args.workers, mp_context=mp.get_context("fork"))
    list(ex.map(abs, range(4 * args.workers)))

    import torch
    import paper_1203_4874_amd as P
    dev = torch.device("cuda:0")
    P.lib()
    total = args.pairs + args.holdout
    if args.eval_only:
        with ex:
            hold = list(ex.map(make_pair, range(args.pairs, total), chunksize=32))
        blob = P.load_mlp(os.path.join(args.out, "cbp_mlp.npz"), device=dev)
        holdout_report(P, torch, dev, hold, blob, args.out, None)
        return
    t0 = time.time()
    Xs, Ts = [], []
    chunk = 2000
    with ex:
        # training pairs, generated and consumed chunk by chunk (only features and targets are kept)
        for c0 in range(0, args.pairs, chunk):
            ids = list(range(c0, min(c0 + chunk, args.pairs)))
            pairs = list(ex.map(make_pair, ids, chunksize=32))
            res = run_pairs(P, torch, dev, pairs)
            for p, (dg, _, _) in zip(pairs, res):
                if dg is None:
                    continue
                X, T = targets(dg, p["K1"], p["K2"])
                Xs.append(X)
                Ts.append(T)
            print(f"[train] features of {ids[-1] + 1}/{args.pairs} pairs ({time.time() - t0:.0f} s)", flush=True)
        hold = list(ex.map(make_pair, range(args.pairs, total), chunksize=32))
    X = np.concatenate(Xs)
    T = np.concatenate(Ts)
    ok = np.isfinite(X).all(1) & np.isfinite(T).all(1)
    X, T = X[ok], T[ok]
    print(f"[train] {X.shape[0]} sample rows", flush=True)

    rng = np.random.default_rng(SEED)
    init = rng.standard_normal(P.MlpState.param_count()).astype(np.float32)
    # He-normal layers, zero biases (packed order W1, b1, W2, b2, W3, b3)
    o = 0
    for rows, cols, gain in ((128, 32, 2.0), (128, 128, 2.0), (2, 128, 0.02)):
        init[o:o + rows * cols] *= np.sqrt(gain / cols)
        o += rows * cols
        init[o:o + rows] = 0.0
        o += rows
    # output biases at the targets' centre: w = softplus(o1) = 1, o2 = mean log tau*
    init[-2] = np.log(np.e - 1.0)
    init[-1] = float(np.mean(T[:, 1]))
    st = P.MlpState(args.batch, dev)
    st.set_params(init)
    Xd = torch.as_tensor(X, device=dev)
    Td = torch.as_tensor(T, device=dev)
    nrow = X.shape[0]
    steps_per_epoch = max(1, nrow // args.batch)
    step = 0
    first_epoch = 0
    if args.resume and args.checkpoint and os.path.exists(args.checkpoint):
        with np.load(args.checkpoint, allow_pickle=False) as z:
            st.load_state(z["state"])
            step, first_epoch = int(z["step"]), int(z["epoch"]) + 1
        print(f"[train] resumed after epoch {first_epoch} (step {step})", flush=True)
    t0 = time.time()
    for ep in range(first_epoch, args.epochs):
        perm = torch.randperm(nrow, device=dev, generator=torch.Generator(device=dev).manual_seed(ep))
        tot = 0.0
        for b in range(steps_per_epoch):
            ids = perm[b * args.batch:(b + 1) * args.batch]
            xb, tb = Xd[ids].contiguous(), Td[ids].contiguous()
            step += 1
            lr = args.lr * (0.05 + 0.95 * 0.5 * (1 + np.cos(np.pi * step / (args.epochs * steps_per_epoch))))
            loss = st.train_step(xb, tb, lr, step)
            tot += float(loss.item()) if b % 16 == 0 else 0.0
        print(f"[train] epoch {ep + 1}/{args.epochs}: loss ~{tot / max(1, (steps_per_epoch + 15) // 16):.4f} "
              f"({time.time() - t0:.0f} s)", flush=True)
        if args.checkpoint:
            tmp = args.checkpoint + ".tmp.npz"
            np.savez(tmp, state=st.save_state().cpu().numpy(), step=step, epoch=ep)
            os.replace(tmp, args.checkpoint)
    params = st.get_params().cpu().numpy()
    blob = st.export()
    os.makedirs(args.out, exist_ok=True)
    np.savez(os.path.join(args.out, "cbp_mlp.npz"), params=params,
             note=np.array("learned-form network; packed W1, b1, W2, b2, W3, b3 (FP32)"))

    holdout_report(P, torch, dev, hold, blob, args.out, int(nrow))


def holdout_report(P, torch, dev, hold, blob, out, rows_trained):
    """Held-out comparison, plain vs learned route (noise gate and judge
    included), kernel rel-L2 against the truth per noise level; written to
    holdout.json."""
    plain = run_pairs(P, torch, dev, hold)
    learn = run_pairs(P, torch, dev, hold, mlp=blob)
    rows = []
    for p, a, b in zip(hold, plain, learn):
        if a[0] is None or b[0] is None:
            continue
        def err(K1, K2):
            return max(np.linalg.norm(K1 - p["K1"]) / np.linalg.norm(p["K1"]),
                       np.linalg.norm(K2 - p["K2"]) / np.linalg.norm(p["K2"]))
        rows.append((p["noise"], err(a[1], a[2]), err(b[1], b[2]), 1.0 if b[0]["flags"] & 16 else 0.0))
    rows = np.array(rows)
    summary = {}
    for nz in NOISES:
        sel = rows[rows[:, 0] == nz]
        summary[str(nz)] = dict(pairs=int(sel.shape[0]), plain_median=float(np.median(sel[:, 1])),
                                learned_median=float(np.median(sel[:, 2])),
                                plain_mean=float(np.mean(sel[:, 1])), learned_mean=float(np.mean(sel[:, 2])),
                                learned_better_fraction=float(np.mean(sel[:, 2] < sel[:, 1])),
                                plain_kept_fraction=float(np.mean(sel[:, 3])))
    if rows_trained is not None:
        summary["rows"] = rows_trained
    summary["note"] = ("learned route = network weights, noise gate (plain kernels on frames with a noise floor) "
                       "and judge; plain_kept_fraction = frames where the plain kernels were returned")
    print(json.dumps(summary), flush=True)
    with open(os.path.join(out, "holdout.json"), "w") as fh:
        json.dump(summary, fh, indent=1)

if __name__ == "__main__":
    main()
