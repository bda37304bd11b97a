"""Benchmark: deblurred Mpixel/s of the CBP hot path (kernel recovery + two-channel
Fourier division) on one MI355X.

Workload: one 480x640 grayscale frame per step (smooth scene of 40 anisotropic
Gaussians + 0.1 texture), coprime 9x9 / 11x11 kernels (Gaussian sigma 2 + 0.2
uniform, sum 1), additive noise sigma 1e-3, lambda 1e-4, S = 11.  Inputs are
generated on the host, copied to the device once and resident in HBM before
the timed region.  The headline `value` is the mixed form (FP32 frames and FFT,
FP64 kernel recovery); the plain FP64 form is timed the same way and reported
beside it, each with its PSNR against the FP64 oracle's latent.

A step is one cbp_deblur call (every kernel of the path).  W untimed warm-up
steps, then exactly K timed steps between two device synchronisations.  A
second pass of K steps records HIP events around every kernel (on the stream
the kernels run on) for the per-kernel averages and the roofline line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--batch-frames", type=int, default=64,
                    help="frames of the 720p batching workload reported beside the headline (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--colour-frames", type=int, default=8,
                    help="frames of the 1080p colour workload (one batch; 0 = skip)")
    ap.add_argument("--colour-steps", type=int, default=20)
    ap.add_argument("--forms", default="mixed,fp64,mfma32,bf16,learned",
                    help="comma-separated forms of the single-frame workload (mixed is always run)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 256 MiB (counter calibration runs)")
    return ap.parse_args()


def psnr(a, b, peak=1.0):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(peak * peak / mse)


def source_hash(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1203_4874_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# Algorithmic cost of each kernel for one frame of this workload.  Bytes: the
# minimum HBM traffic of the kernel's own inputs and outputs.  FLOPs: the FP64
# arithmetic of the kernel's algorithm, counted as real operations (a complex
# multiply-add is 8, a double-double complex multiply-add about 40).
def eig_flops(n, refine_steps, invit=3, bisect_probes=64 * 8):
    """One Hermitian smallest-eigenvector solve of order n: Householder
    tridiagonalisation (16/3 n^3), Sturm multisection (about 5 n per probe),
    the LDL^T factors of T - sigma I (4 n), `invit` inverse iterations on T
    (forward and backward substitution on a complex vector and its norm,
    about 16 n each), x = Q D y with the reflectors applied one by one (a dot
    and an axpy per reflector, 8 n^2) and `refine_steps` Newton corrections
    (a double-double Gram mat-vec, 40 n^2, two reflector sweeps, 16 n^2, and
    a tridiagonal solve)."""
    return 16.0 / 3.0 * n ** 3 + bisect_probes * 5 * n + 4 * n + invit * 16 * n + 8 * n * n \
        + refine_steps * (56 * n * n + 16 * n)


def kernel_models(H1, W1, H2, W2, m, n, k1, k2, S, Py, Px, esize, refine_sample, refine_scale):
    hx = Px // 2 + 1
    N = k1 + k2
    cplx = 2 * esize
    pix_in = (H1 * W1 + H2 * W2)
    # cofactor grids P, Q for both kernels (S*S*k complex MACs each), the
    # scale system (|P|^2, |Q|^2 sums and the cross sums), the 2S solve, the
    # averaged spectra and the two-stage S x S inverse DFT cropped to k x k
    fin = sum(2 * S * S * k * 8 + (S * S * k + S * k * k) * 8 * 2 for k in (k1, k2)) \
        + 2 * 2 * S * S * 3 + 2 * S * S * 8 + eig_flops(2 * S, refine_scale) + 2 * S * S * 14
    models = {
        "fold_cols": dict(bound="hbm", bytes=pix_in * esize + 8 * S * (W1 + W2)),
        "eval_rows": dict(bound="hbm", bytes=pix_in * esize + 16 * S * (H1 + H2)),
        "row_fft_fwd": dict(bound="hbm", bytes=pix_in * esize + cplx * hx * (H1 + H2)),
        "col_fft_filter": dict(bound="hbm", bytes=cplx * hx * (H1 + H2) + cplx * hx * m),
        "row_fft_inv": dict(bound="hbm", bytes=cplx * hx * m + esize * m * n),
        "sample_eig": dict(bound="alu", flops=2 * S * eig_flops(N, refine_sample), peak=FP64_PEAK_TFLOPS),
        "scale_assemble": dict(bound="alu", flops=fin, peak=FP64_PEAK_TFLOPS),
    }
    return models


def bench_batch(P, torch, dev, orc, args):
    """The batching form: N moving-blob 720x1280 frames with per-frame uneven
    kernels 7..15, noise 1e-3, lambda 1e-4, FP32 frames (mixed form), all
    frames in one work-list launch per phase, launch shapes from the
    autotuner, replayed as one HIP graph per call."""
    import synth
    nf = args.batch_frames
    t0 = time.perf_counter()
    fr = list(synth.config3_frames(nframes=nf))
    print(f"[bench] batch workload generated ({nf} frames, {time.perf_counter() - t0:.1f} s)", file=sys.stderr,
          flush=True)
    frames = [(torch.as_tensor(f["B1"].astype(np.float32), device=dev),
               torch.as_tensor(f["B2"].astype(np.float32), device=dev), f["m"], f["n"]) for f in fr]
    d = P.Deblurrer(734, 1294, 15, 1, nf, P.Precision.MIXED)
    tune = d.prepare_batch(frames, lam=1e-4, flags=P.Flags.AUTOTUNE)
    tune.run()
    torch.cuda.synchronize()
    tuned = P.last_tuning()
    out = {}
    for name, flags in (("graph", P.Flags.GRAPH), ("eager", 0)):
        pb = d.prepare_batch(frames, lam=1e-4, flags=flags)
        for _ in range(2):
            pb.run(check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            pb.run(check=False)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.batch_steps
        out[name] = dict(ms_per_batch=ms, value=nf * 720 * 1280 / 1e6 / (ms / 1e3))
        print(f"[bench] batch {name}: {ms:.3f} ms per {nf}-frame batch", file=sys.stderr, flush=True)
        if name == "graph":
            keep = pb
    with P.profile() as prof:
        pe = d.prepare_batch(frames, lam=1e-4)
        for _ in range(3):
            pe.run(check=False)
        torch.cuda.synchronize()
    phases = {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof.result.items()}
    # accuracy on sampled frames (oracle, outside the timed region)
    errs, ps, pt = [], [], []
    for f in (0, nf // 2, nf - 1):
        h = fr[f]
        B1 = h["B1"].astype(np.float32).astype(np.float64)
        B2 = h["B2"].astype(np.float32).astype(np.float64)
        Lo, R1, R2 = orc.deblur(B1, B2, h["m"], h["n"], 0, 1e-4)
        K1 = keep.K1s[f].cpu().numpy()
        K2 = keep.K2s[f].cpu().numpy()
        L = keep.latents[f].double().cpu().numpy()
        errs.append(max(float(np.linalg.norm(K1 - R1) / np.linalg.norm(R1)),
                        float(np.linalg.norm(K2 - R2) / np.linalg.norm(R2))))
        ps.append(psnr(L, Lo))
        pt.append(psnr(L, h["L"]))
    return dict(workload=f"{nf} x 720x1280 moving-blob frames, per-frame coprime kernels 7..15 (uneven), "
                         "noise 1e-3, lambda 1e-4, FP32 frames (mixed form)",
                metric="deblurred Mpixel/s", value=out["graph"]["value"], unit="Mpixel/s",
                ms_per_batch=out["graph"]["ms_per_batch"], eager=out["eager"], tuning=tuned,
                phases_us_per_batch=phases, sampled_frames=[0, nf // 2, nf - 1],
                kernel_rel_l2_vs_oracle_max=max(errs), psnr_vs_oracle_db_min=min(ps),
                psnr_vs_truth_db_min=min(pt))


def _colour_frame(f):
    """One frame of the 1080p colour workload as FP32 frames (pool worker)."""
    import synth
    h = synth.config5_frame(f)
    return dict(B1=h["B1"].astype(np.float32), B2=h["B2"].astype(np.float32), K1=h["K1"], K2=h["K2"],
                L=h["L"].astype(np.float32), m=h["m"], n=h["n"], S=h["S"], lam=h["lam"])


def bench_colour(P, torch, dev, orc, args, host, blob):
    """Colour batching: one batch of 1080x1920 RGB frames (channels share one
    kernel pair from the channel-summed Grams; per-channel division), one
    15x15 / 17x17 pair, noise 5e-3, lambda 1e-4, FP32 frames, replayed as one
    HIP graph; the plain mixed form and the learned form.  Per-batch latency
    percentiles over repeated calls; accuracy on frame 0 against the truth
    and the oracle's colour route."""
    nf = len(host)
    m, n = host[0]["m"], host[0]["n"]
    frames = [(torch.as_tensor(h["B1"], device=dev), torch.as_tensor(h["B2"], device=dev), m, n) for h in host]
    H = max(max(h["B1"].shape[1], h["B2"].shape[1]) for h in host)
    W = max(max(h["B1"].shape[2], h["B2"].shape[2]) for h in host)
    d = P.Deblurrer(H, W, H - m + 1, 3, nf, P.Precision.MIXED)
    h0 = host[0]
    Lo, R1, R2 = orc.deblur(h0["B1"].astype(np.float64), h0["B2"].astype(np.float64), m, n, 0, h0["lam"])
    out = {}
    for form, mlp in (("mixed", None), ("learned", blob)):
        if form == "learned" and mlp is None:
            continue
        pb = d.prepare_batch(frames, lam=h0["lam"], flags=P.Flags.GRAPH, mlp=mlp)
        for _ in range(2):
            pb.run(check=False)
        torch.cuda.synchronize()
        times = []
        for _ in range(args.colour_steps):
            t0 = time.perf_counter()
            pb.run(check=False)
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0))
        ms = np.array(times)
        p50 = float(np.percentile(ms, 50))
        K1 = pb.K1s[0].cpu().numpy()
        K2 = pb.K2s[0].cpu().numpy()
        L = pb.latents[0].double().cpu().numpy()
        kt = max(float(np.linalg.norm(K1 - h0["K1"]) / np.linalg.norm(h0["K1"])),
                 float(np.linalg.norm(K2 - h0["K2"]) / np.linalg.norm(h0["K2"])))
        ko = max(float(np.linalg.norm(K1 - R1) / np.linalg.norm(R1)),
                 float(np.linalg.norm(K2 - R2) / np.linalg.norm(R2)))
        out[form] = dict(value=nf * m * n / 1e6 / (p50 / 1e3), channel_value=3 * nf * m * n / 1e6 / (p50 / 1e3),
                         ms_per_batch_p50=p50, ms_per_batch_p99=float(np.percentile(ms, 99)),
                         kernel_rel_l2_vs_truth=kt, kernel_rel_l2_vs_plain_oracle=ko,
                         psnr_vs_truth_db_min=min(psnr(L[c], h0["L"][c]) for c in range(3)),
                         psnr_vs_plain_oracle_db_min=min(psnr(L[c], Lo[c]) for c in range(3)))
        print(f"[bench] colour {form}: p50 {p50:.3f} ms per {nf}-frame batch", file=sys.stderr, flush=True)
    return dict(workload=f"{nf} x 1080x1920 RGB frames (moving blobs, channel gains + texture), one coprime "
                         "15x15/17x17 pair, noise 5e-3, lambda 1e-4, FP32 frames, batch of "
                         f"{nf} as one HIP graph", metric="deblurred Mpixel/s (RGB pixel counted once)",
                unit="Mpixel/s", forms=out, steps=args.colour_steps)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)

    colour_host = None
    if args.colour_frames > 0:
        # generated in forked workers before anything touches the GPU
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        t0 = time.perf_counter()
        with ProcessPoolExecutor(max_workers=min(8, args.colour_frames), mp_context=mp.get_context("fork")) as ex:
            colour_host = list(ex.map(_colour_frame, range(args.colour_frames)))
        print(f"[bench] colour workload generated ({args.colour_frames} frames, {time.perf_counter() - t0:.1f} s)",
              file=sys.stderr, flush=True)

    import torch
    import synth
    import paper_1203_4874_amd as P

    dev = torch.device("cuda:0")
    P.lib()
    c = synth.config2()
    m, n, lam = c["m"], c["n"], c["lam"]
    H1, W1 = c["B1"].shape
    H2, W2 = c["B2"].shape
    k1, k2, S = c["K1"].shape[0], c["K2"].shape[0], c["S"]

    blob = P.load_mlp(device=dev) if os.path.exists(P.WEIGHTS) else None
    forms = {}
    for name, npd, tdt, prec in (("mixed", np.float32, torch.float32, P.Precision.MIXED),
                                 ("fp64", np.float64, torch.float64, P.Precision.FP64),
                                 ("mfma32", np.float32, torch.float32, P.Precision.MFMA32),
                                 ("bf16", np.float32, torch.float32, P.Precision.BF16),
                                 ("learned", np.float32, torch.float32, P.Precision.MIXED)):
        if name == "learned" and blob is None:
            continue
        if name != "mixed" and name not in args.forms.split(","):
            continue
        B1 = c["B1"].astype(npd)
        B2 = c["B2"].astype(npd)
        b1 = torch.as_tensor(B1, device=dev)
        b2 = torch.as_tensor(B2, device=dev)
        d = P.Deblurrer(max(H1, H2), max(W1, W2), max(k1, k2), precision=prec, device=dev)
        out = torch.empty((m, n), dtype=tdt, device=dev)
        K1 = torch.empty((k1, k1), dtype=torch.float64, device=dev)
        K2 = torch.empty((k2, k2), dtype=torch.float64, device=dev)
        forms[name] = dict(B1=B1, B2=B2, b1=b1, b2=b2, d=d, out=out, K1=K1, K2=K2,
                           mlp=blob if name == "learned" else None)

    def step(f):
        f["d"].deblur(f["b1"], f["b2"], m, n, lam=lam, out=f["out"], K1=f["K1"], K2=f["K2"], mlp=f["mlp"])

    results = {}
    for name, f in forms.items():
        for _ in range(args.warmup):
            step(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(f)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms = 1e3 * dt / args.steps
        print(f"[bench] {name}: {args.steps} steps in {dt:.3f} s ({ms:.4f} ms/step)", file=sys.stderr, flush=True)
        # per-kernel timing pass (HIP events on the call's stream)
        with P.profile() as prof:
            for _ in range(args.steps):
                step(f)
            torch.cuda.synchronize()
        phases = {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof.result.items()}
        results[name] = dict(ms=ms, phases_us=phases)

    # the headline form replayed as one HIP graph per call (the library captures
    # the call's launch sequence once and replays it)
    f = forms["mixed"]
    for _ in range(args.warmup):
        f["d"].deblur(f["b1"], f["b2"], m, n, lam=lam, out=f["out"], K1=f["K1"], K2=f["K2"], flags=P.Flags.GRAPH)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f["d"].deblur(f["b1"], f["b2"], m, n, lam=lam, out=f["out"], K1=f["K1"], K2=f["K2"], flags=P.Flags.GRAPH)
    torch.cuda.synchronize()
    gms = 1e3 * (time.perf_counter() - t0) / args.steps
    print(f"[bench] mixed, graph replay: {gms:.4f} ms/step", file=sys.stderr, flush=True)

    # accuracy of each form against the FP64 oracle (outside the timed regions)
    from oracle import cbp as orc
    Lo, R1, R2 = orc.deblur(c["B1"], c["B2"], m, n, S, lam)
    for name, f in forms.items():
        step(f)
        torch.cuda.synchronize()
        L = f["out"].double().cpu().numpy()
        kr = float(np.linalg.norm(f["K1"].cpu().numpy() - R1) / np.linalg.norm(R1))
        kr2 = float(np.linalg.norm(f["K2"].cpu().numpy() - R2) / np.linalg.norm(R2))
        kt = float(np.linalg.norm(f["K1"].cpu().numpy() - c["K1"]) / np.linalg.norm(c["K1"]))
        kt2 = float(np.linalg.norm(f["K2"].cpu().numpy() - c["K2"]) / np.linalg.norm(c["K2"]))
        results[name].update(psnr_vs_oracle=psnr(L, Lo), psnr_vs_truth=psnr(L, c["L"]),
                             kernel_rel_l2_vs_oracle=max(kr, kr2), kernel_rel_l2_vs_truth=max(kt, kt2))

    mpix = m * n / 1e6
    main_form = results["mixed"]
    value = mpix / (main_form["ms"] / 1e3)

    # roofline of the dominant kernel of the headline form
    ph = {k: v for k, v in main_form["phases_us"].items() if v}
    dom = max(ph, key=ph.get)
    Py, Px = orc.smooth7(max(H1, H2)), orc.smooth7(max(W1, W2))
    # refinement step counts of the solves (diag run, outside the timed regions)
    f = forms["mixed"]
    dd = P.Deblurrer(max(H1, H2), max(W1, W2), max(k1, k2), precision=P.Precision.MIXED, device=dev, diag=True)
    dd.deblur(f["b1"], f["b2"], m, n, lam=lam, out=f["out"], K1=f["K1"], K2=f["K2"])
    dg = dd.read_diag()
    models = kernel_models(H1, W1, H2, W2, m, n, k1, k2, S, Py, Px, 4,
                           dg["refine_sample"], dg["refine_scale"])
    roof = None
    if dom in models:
        mdl = models[dom]
        t = ph[dom] * 1e-6
        if mdl["bound"] == "hbm":
            ach = mdl["bytes"] / t / 1e9
            roof = dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=ach / HBM_PEAK_GBS, algorithmic_bytes=mdl["bytes"])
        else:
            ach = mdl["flops"] / t / 1e12
            roof = dict(kernel=dom, bound="alu", achieved=ach, peak=mdl["peak"], unit="TFLOP/s",
                        frac=ach / mdl["peak"], algorithmic_flops=mdl["flops"])
        roof["avg_us"] = ph[dom]
        if dom == "scale_assemble":
            roof["launch"] = "one 64-lane workgroup per frame (a single solve of order 2S)"
        elif dom == "sample_eig":
            roof["launch"] = f"{2 * S} workgroups of 64 lanes (one solve of order k1+k2 each)"
        roof["traffic"] = None
        tf = os.path.join(ROOT, "profiles", "traffic.json")
        if os.path.exists(tf):
            with open(tf) as fh:
                tr = json.load(fh)
            ent = tr.get(dom)
            if ent and ent.get("source_hash") == source_hash(ent.get("sources", [])):
                roof["traffic"] = ent.get("bytes_per_launch")
    else:
        roof = dict(kernel=dom, bound="alu", achieved=None, peak=None, unit=None, frac=None, traffic=None,
                    avg_us=ph[dom])

    # every kernel's fraction of its own bound, for the stage split
    kern_roof = {}
    for k, v in ph.items():
        if k in models:
            mdl = models[k]
            if mdl["bound"] == "hbm":
                kern_roof[k] = dict(bound="hbm", GBs=mdl["bytes"] / (v * 1e-6) / 1e9,
                                    frac=mdl["bytes"] / (v * 1e-6) / 1e9 / HBM_PEAK_GBS)
            else:
                kern_roof[k] = dict(bound="alu", TFLOPs=mdl["flops"] / (v * 1e-6) / 1e12,
                                    frac=mdl["flops"] / (v * 1e-6) / 1e12 / mdl["peak"])

    cpu = None
    if not args.no_cpu_baseline:
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count() or 1
        reps, t0 = 0, time.perf_counter()
        while True:
            orc.deblur(c["B1"], c["B2"], m, n, S, lam)
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        cpu = dict(value=reps * mpix / el, unit="Mpixel/s", cores=int(threads), kind="oracle",
                   sample=f"{reps} repetitions of the same 480x640 frame (FP64 NumPy/SciPy oracle, {el:.1f} s)")

    # PCIe-inclusive rate of the headline form: frames from pinned host
    # memory, the latent back to pinned host memory, in every step
    f = forms["mixed"]
    h1 = torch.from_numpy(np.ascontiguousarray(f["B1"])).pin_memory()
    h2 = torch.from_numpy(np.ascontiguousarray(f["B2"])).pin_memory()
    hL = torch.empty((m, n), dtype=torch.float32).pin_memory()

    def pstep():
        f["b1"].copy_(h1, non_blocking=True)
        f["b2"].copy_(h2, non_blocking=True)
        step(f)
        hL.copy_(f["out"], non_blocking=True)

    for _ in range(args.warmup):
        pstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pstep()
    torch.cuda.synchronize()
    pms = 1e3 * (time.perf_counter() - t0) / args.steps
    pcie = dict(value=mpix / (pms / 1e3), unit="Mpixel/s", ms_per_step=pms,
                note="frames H2D from pinned host memory and the latent D2H, inside every step")

    batched = None
    if args.batch_frames > 0:
        batched = bench_batch(P, torch, dev, orc, args)
    colour = None
    if colour_host:
        colour = bench_colour(P, torch, dev, orc, args, colour_host, blob)

    if args.copy_calibration:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()

    line = {
        "metric": "deblurred Mpixel/s (kernel recovery + deconv), mixed form, PSNR vs FP64 oracle reported",
        "value": value,
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_form["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (frames, FFT, division) + f64 (evaluation, Gram, eigen-solves, scale fix)",
        "data": "synthetic",
        "config": {"workload": "480x640 grayscale frame, coprime 9x9/11x11 kernels, noise 1e-3, lambda 1e-4, S=11",
                   "frames_per_step": 1, "blurred": [[H1, W1], [H2, W2]], "fft_grid": [Py, Px]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "psnr_vs_oracle_db": main_form["psnr_vs_oracle"],
        "psnr_vs_truth_db": main_form["psnr_vs_truth"],
        "kernel_rel_l2_vs_oracle": main_form["kernel_rel_l2_vs_oracle"],
        "phases_us": main_form["phases_us"],
        "phases_roofline": kern_roof,
        "plain_fp64": None if "fp64" not in results else {
            "value": mpix / (results["fp64"]["ms"] / 1e3), "ms_per_step": results["fp64"]["ms"],
            "psnr_vs_oracle_db": results["fp64"]["psnr_vs_oracle"],
            "kernel_rel_l2_vs_oracle": results["fp64"]["kernel_rel_l2_vs_oracle"],
            "phases_us": results["fp64"]["phases_us"]},
        "precision_forms": {k: {"value": mpix / (results[k]["ms"] / 1e3), "ms_per_step": results[k]["ms"],
                                "psnr_vs_oracle_db": results[k]["psnr_vs_oracle"],
                                "kernel_rel_l2_vs_oracle": results[k]["kernel_rel_l2_vs_oracle"],
                                "phases_us": results[k]["phases_us"]}
                            for k in ("mfma32", "bf16") if k in results},
        "learned": None if "learned" not in results else {
            "value": mpix / (results["learned"]["ms"] / 1e3), "ms_per_step": results["learned"]["ms"],
            "kernel_rel_l2_vs_truth": results["learned"]["kernel_rel_l2_vs_truth"],
            "plain_kernel_rel_l2_vs_truth": results["mixed"]["kernel_rel_l2_vs_truth"],
            "psnr_vs_truth_db": results["learned"]["psnr_vs_truth"],
            "plain_psnr_vs_truth_db": results["mixed"]["psnr_vs_truth"],
            "phases_us": results["learned"]["phases_us"]},
        "graph_replay": {"value": mpix / (gms / 1e3), "ms_per_step": gms,
                         "note": "the headline form with the call captured once and replayed as a HIP graph"},
        "pcie_inclusive": pcie,
        "batched_720p": batched,
        "colour_1080p": colour,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
