"""Benchmark: deblurred Mpixel/s of the CBP hot path (kernel recovery + two-channel
Fourier division) on one MI355X.

Headline workload: a stream of 300 RGB frames of 1080x1920 (a moving-blob
surveillance scene, per-channel gains and texture), one coprime 15x15 / 17x17
kernel pair for every frame, additive noise sigma 5e-3, lambda 1e-4, S = 17.
The stream cycles through U (default 24) generated frames; every one of the
300 frames has its own device buffers, resident in HBM before the timed
region.  Frames are deblurred in batches of 8 (one cbp_deblur_batch call per
batch, each replayed as a HIP graph); channels share one kernel pair and the
latent is divided channel by channel.  The headline `value` is the mixed form
(FP32 frames, FFT and division; FP64 evaluation, double-double Gram, FP64
eigen-solves and scale fix); the plain FP64 form is timed the same way and
reported beside it, each with its kernel error and PSNR against the FP64
oracle on sampled frames.

A step is one batch (one call over 8 frames: every kernel of the path).  All
batches of the stream are captured once before timing; then W untimed warm-up
steps and exactly K timed steps (step i runs batch i mod 38) between two
device synchronisations.  A profiled pass (HIP events around every kernel on
the call's stream, eager launches) gives the per-kernel averages for the
roofline line.  A real-time pass replays the stream at 30 frames per second
arrival (a batch starts when its last frame has arrived) for per-frame
arrival-to-output latency percentiles.

Also reported: the form the workload names (learned weights + BF16 Gram),
the 480x640 single-frame workload (every precision form), the 64-frame 720p
batching workload, and the CPU oracle on sampled frames of the stream.

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
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X FP64 matrix cores (dense)
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=38, help="timed batch steps (38 = the 300-frame stream once)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=300, help="frames of the 1080p RGB stream")
    ap.add_argument("--unique-frames", type=int, default=24, help="generated frames the stream cycles through")
    ap.add_argument("--batch", type=int, default=8, help="frames per call (one HIP graph per batch)")
    ap.add_argument("--fps", type=float, default=30.0, help="arrival rate of the real-time pass (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=4, help="stream frames the oracle runs on")
    ap.add_argument("--precision", default="mfma64", choices=["mixed", "mfma64"],
                    help="Gram form of the headline: double-double on the vector units or FP64 matrix cores")
    ap.add_argument("--forms", default="fp64,mixed,learned_mfma64",
                    help="comma-separated extra forms on the stream (fp64, mixed, mfma64, learned, learned_mfma64, "
                         "learned_bf16)")
    ap.add_argument("--single-steps", type=int, default=100,
                    help="steps of the 480x640 single-frame workload (0 = skip)")
    ap.add_argument("--batch-frames", type=int, default=64,
                    help="frames of the 720p batching workload (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--workers", type=int, default=16, help="host processes generating the stream's frames")
    ap.add_argument("--no-autotune", action="store_true", help="default launch shapes for the stream")
    ap.add_argument("--lanes", type=int, default=3,
                    help="streams the stream's batches alternate on (each with its own workspace): one "
                         "batch's kernel recovery overlaps the previous batches' FFT passes")
    ap.add_argument("--only-timing", action="store_true",
                    help="stop after the timed steps (kernel-trace runs: the last W + K dispatches of each kernel "
                         "are the timed graph replays)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 256 MiB (counter calibration runs)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def psnr(a, b, peak=1.0):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(peak * peak / mse)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def source_hash(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1203_4874_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def traffic_for(phase, workload):
    """Calibrated HBM bytes per launch of a kernel on a workload, from the
    committed counter summary, while the kernel's sources are unchanged."""
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tf):
        return None
    with open(tf) as fh:
        tr = json.load(fh)
    ent = tr.get(f"{phase}@{workload}")
    if ent and ent.get("source_hash") == source_hash(ent.get("sources", [])):
        return ent.get("bytes_per_launch")
    return None


# Algorithmic cost of each kernel for one frame of the single-frame workload.
# Bytes: the minimum HBM traffic of the kernel's own inputs and outputs.
# FLOPs: the FP64 arithmetic of the kernel's algorithm, counted as real
# operations (a complex multiply-add is 8, a double-double one about 40).
def eig_flops(n, refine_steps, invit=3, bisect_probes=64 * 8):
    """One Hermitian smallest-eigenvector solve of order n: Householder
    tridiagonalisation (16/3 n^3), Sturm multisection (about 5 n per probe),
    the LDL^T factors of T - sigma I (4 n), `invit` inverse iterations,
    x = Q D y with the reflectors applied one by one (8 n^2) and
    `refine_steps` Newton corrections (a double-double Gram mat-vec, 40 n^2,
    two reflector sweeps, 16 n^2, and a solve)."""
    return 16.0 / 3.0 * n ** 3 + bisect_probes * 5 * n + 4 * n + invit * 16 * n + 8 * n * n \
        + refine_steps * (56 * n * n + 16 * n)


def kernel_models(H1, W1, H2, W2, m, n, k1, k2, S, Py, Px, esize, refine_sample, refine_scale):
    hx = Px // 2 + 1
    N = k1 + k2
    cplx = 2 * esize
    pix_in = (H1 * W1 + H2 * W2)
    fin = sum(2 * S * S * k * 8 + (S * S * k + S * k * k) * 8 * 2 for k in (k1, k2)) \
        + 2 * 2 * S * S * 3 + 2 * S * S * 8 + eig_flops(2 * S, refine_scale) + 2 * S * S * 14
    # a deblurring call's row pass reads the frames once: it also folds the
    # columns (the fold's output, S rows per frame) and writes the row
    # evaluation; its first launch only writes the FP64 twiddle table of the
    # kernels' row DFTs (Px entries)
    return {
        "fold_cols": dict(bound="hbm", bytes=16 * Px),
        "eval_cols": dict(bound="hbm", bytes=8 * S * (W1 + W2) + 16 * S * (W1 + W2)),
        "row_fft_fwd": dict(bound="hbm", bytes=pix_in * esize + cplx * hx * (H1 + H2) + 8 * S * (W1 + W2)
                            + 16 * S * (H1 + H2)),
        "col_fft_filter": dict(bound="hbm", bytes=cplx * hx * (H1 + H2) + cplx * hx * m),
        "row_fft_inv": dict(bound="hbm", bytes=cplx * hx * m + esize * m * n),
        "sample_eig": dict(bound="alu", flops=2 * S * eig_flops(N, refine_sample), peak=FP64_PEAK_TFLOPS),
        "scale_assemble": dict(bound="alu", flops=fin, peak=FP64_PEAK_TFLOPS),
    }


# ---------------------------------------------------------------- the 1080p RGB stream

def _colour_frame(f):
    """Frame f of the 1080p colour workload as FP32 frames (pool worker)."""
    import synth
    h = synth.config5_frame(f)
    return dict(B1=h["B1"].astype(np.float32), B2=h["B2"].astype(np.float32), K1=h["K1"], K2=h["K2"],
                L=h["L"].astype(np.float32), m=h["m"], n=h["n"], S=h["S"], lam=h["lam"], noise=h["noise"])


class Stream:
    """The stream's frames in HBM (one buffer pair and one latent per frame)
    and its batches, prepared once (argument marshalling, graph capture)."""

    def __init__(self, P, torch, dev, host, nframes, batch, dtype, precision, flags, mlp=None, autotune=True,
                 lanes=1):
        self.P, self.torch = P, torch
        self.nframes, self.batch = nframes, batch
        U = len(host)
        m, n = host[0]["m"], host[0]["n"]
        self.m, self.n = m, n
        src1 = [torch.as_tensor(h["B1"], device=dev).to(dtype) for h in host]
        src2 = [torch.as_tensor(h["B2"], device=dev).to(dtype) for h in host]
        self.b1 = [src1[f % U].clone() for f in range(nframes)]
        self.b2 = [src2[f % U].clone() for f in range(nframes)]
        del src1, src2
        self.out = [torch.empty((3, m, n), dtype=dtype, device=dev) for _ in range(nframes)]
        H = max(max(h["B1"].shape[1], h["B2"].shape[1]) for h in host)
        W = max(max(h["B1"].shape[2], h["B2"].shape[2]) for h in host)
        # `lanes` streams, each with its own workspace: batch i runs on lane
        # i mod lanes, so one batch's kernel recovery (a few one-wave solves)
        # can share the chip with the previous batch's streaming passes
        self.lanes = [torch.cuda.current_stream()] + [torch.cuda.Stream(device=dev) for _ in range(lanes - 1)]
        self.ds = [P.Deblurrer(H, W, H - m + 1, 3, batch, precision, device=dev) for _ in range(lanes)]
        self.d = self.ds[0]
        self.starts = list(range(0, nframes, batch))
        self.batches = []
        for i, s in enumerate(self.starts):
            fr = range(s, min(s + batch, nframes))
            pairs = [(self.b1[f], self.b2[f], m, n) for f in fr]
            self.batches.append(self.ds[i % lanes].prepare_batch(pairs, lam=host[0]["lam"],
                                                                 outs=[self.out[f] for f in fr], flags=flags,
                                                                 mlp=mlp))
        if autotune:
            # the launch shapes of each batch class (full batches, the shorter
            # last one) searched once; later calls of the class use them
            for pb in sorted({len(b.pairs): b for b in self.batches}.values(), key=lambda b: len(b.pairs)):
                keep = pb.flags
                pb.flags = (keep & ~P.Flags.GRAPH) | P.Flags.AUTOTUNE
                pb.run(check=True)
                pb.flags = keep
            self.tuning = P.last_tuning()
        torch.cuda.synchronize()

    def frames_in(self, i):
        b = i % len(self.batches)
        return min(self.starts[b] + self.batch, self.nframes) - self.starts[b]

    def run(self, i):
        # the inputs are resident before any batch runs; a lane's batches reuse its
        # workspace in stream order
        b = i % len(self.batches)
        self.batches[b].run(stream=self.lane_of(b), check=False)

    def lane_of(self, b):
        return self.lanes[b % len(self.lanes)]

    def kernels(self, f):
        pb = self.batches[f // self.batch]
        j = f - self.starts[f // self.batch]
        return pb.K1s[j].cpu().numpy(), pb.K2s[j].cpu().numpy()


def time_stream(torch, s, warmup, steps):
    for i in range(len(s.batches)):          # capture every batch's graph (untimed)
        s.run(i)
    torch.cuda.synchronize()
    for i in range(warmup):
        s.run(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        s.run(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    frames = sum(s.frames_in(i) for i in range(steps))
    return dict(seconds=dt, frames=frames, ms_per_step=1e3 * dt / steps,
                value=frames * s.m * s.n / 1e6 / dt)


def profile_stream(P, torch, s, nb):
    """Per-kernel averages (us per launch) over nb full batches run eagerly
    on one stream (no overlap between batches, so every phase's events time
    its launch alone)."""
    P_flags = [pb.flags for pb in s.batches]
    for pb in s.batches:
        pb.flags = 0
    with P.profile() as prof:
        for i in range(nb):
            s.batches[i % len(s.batches)].run(stream=s.lanes[0], check=False)
        torch.cuda.synchronize()
    for pb, fl in zip(s.batches, P_flags):
        pb.flags = fl
    return {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof.result.items()}


def arrival_pass(torch, s, fps):
    """Replay the stream with frame f arriving at f / fps seconds: batch b is
    launched once its last frame has arrived, on its lane's stream (after the
    lane's earlier batches).  Returns per-frame arrival-to-output latencies (ms)
    and per-batch launch-to-output times (ms)."""
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    ends = [torch.cuda.Event(enable_timing=True) for _ in s.batches]
    launch = []
    e0.record()
    t0 = time.perf_counter()
    for b, st in enumerate(s.starts):
        last = min(st + s.batch, s.nframes) - 1
        due = t0 + last / fps
        while True:
            now = time.perf_counter()
            if now >= due:
                break
            time.sleep(min(0.002, due - now))
        launch.append(time.perf_counter() - t0)
        s.run(b)
        ends[b].record(s.lane_of(b))
    torch.cuda.synchronize()
    done = [e0.elapsed_time(e) / 1e3 for e in ends]       # seconds after t0 (device clock)
    lat = []
    for b, st in enumerate(s.starts):
        for f in range(st, min(st + s.batch, s.nframes)):
            lat.append(1e3 * (done[b] - f / fps))
    proc = [1e3 * (done[b] - launch[b]) for b in range(len(s.starts))]
    return np.array(lat), np.array(proc)


def copy_calibration(torch, dev):
    """A plain 256 MiB device copy (five launches) whose counter readings
    scale the kernels' FETCH_SIZE / WRITE_SIZE to bytes."""
    a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()


# ---------------------------------------------------------------- secondary workloads

def bench_single(P, torch, dev, orc, args, blob):
    """One 480x640 grayscale frame per call, every precision form."""
    import synth
    c = synth.config2()
    m, n, lam = c["m"], c["n"], c["lam"]
    H1, W1 = c["B1"].shape
    H2, W2 = c["B2"].shape
    k1, k2, S = c["K1"].shape[0], c["K2"].shape[0], c["S"]
    Lo, R1, R2 = orc.deblur(c["B1"], c["B2"], m, n, S, lam)
    res = {}
    for name, npd, tdt, prec in (("mixed", np.float32, torch.float32, P.Precision.MIXED),
                                 ("fp64", np.float64, torch.float64, P.Precision.FP64),
                                 ("mfma64", np.float32, torch.float32, P.Precision.MFMA64),
                                 ("mfma32", np.float32, torch.float32, P.Precision.MFMA32),
                                 ("bf16", np.float32, torch.float32, P.Precision.BF16),
                                 ("learned", np.float32, torch.float32, P.Precision.MIXED)):
        if name == "learned" and blob is None:
            continue
        mlp = blob if name == "learned" else None
        b1 = torch.as_tensor(c["B1"].astype(npd), device=dev)
        b2 = torch.as_tensor(c["B2"].astype(npd), device=dev)
        d = P.Deblurrer(max(H1, H2), max(W1, W2), max(k1, k2), precision=prec, device=dev)
        out = torch.empty((m, n), dtype=tdt, device=dev)
        K1 = torch.empty((k1, k1), dtype=torch.float64, device=dev)
        K2 = torch.empty((k2, k2), dtype=torch.float64, device=dev)

        def step():
            d.deblur(b1, b2, m, n, lam=lam, out=out, K1=K1, K2=K2, mlp=mlp)

        for _ in range(10):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.single_steps):
            step()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.single_steps
        with P.profile() as prof:
            for _ in range(args.single_steps):
                step()
            torch.cuda.synchronize()
        phases = {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof.result.items()}
        L = out.double().cpu().numpy()
        Kg1, Kg2 = K1.cpu().numpy(), K2.cpu().numpy()
        res[name] = dict(value=m * n / 1e6 / (ms / 1e3), ms_per_step=ms,
                         kernel_rel_l2_vs_oracle=max(rel(Kg1, R1), rel(Kg2, R2)),
                         kernel_rel_l2_vs_truth=max(rel(Kg1, c["K1"]), rel(Kg2, c["K2"])),
                         psnr_vs_oracle_db=psnr(L, Lo), psnr_vs_truth_db=psnr(L, c["L"]), phases_us=phases)
        log(f"single {name}: {ms:.4f} ms/frame")
    # per-kernel fractions of the mixed form
    Py, Px = orc.smooth7(max(H1, H2)), orc.smooth7(max(W1, W2))
    models = kernel_models(H1, W1, H2, W2, m, n, k1, k2, S, Py, Px, 4, 2, 2)
    kr = {}
    for k, v in res["mixed"]["phases_us"].items():
        if v and k in models:
            mdl = models[k]
            if mdl["bound"] == "hbm":
                kr[k] = dict(bound="hbm", frac=mdl["bytes"] / (v * 1e-6) / 1e9 / HBM_PEAK_GBS)
            else:
                kr[k] = dict(bound="alu", frac=mdl["flops"] / (v * 1e-6) / 1e12 / mdl["peak"])
    return dict(workload="480x640 grayscale frame, coprime 9x9/11x11 kernels, noise 1e-3, lambda 1e-4, S=11, "
                         "one cbp_deblur call per frame", forms=res, phases_roofline_mixed=kr)


def bench_batch(P, torch, dev, orc, args):
    """The batching form: N moving-blob 720x1280 frames with per-frame uneven
    kernels 7..15, noise 1e-3, lambda 1e-4, FP32 frames (the headline's form), all
    frames in one work-list launch per phase, launch shapes from the
    autotuner, replayed as one HIP graph per call."""
    import synth
    nf = args.batch_frames
    t0 = time.perf_counter()
    fr = list(synth.config3_frames(nframes=nf))
    log(f"720p batch workload generated ({nf} frames, {time.perf_counter() - t0:.1f} s)")
    frames = [(torch.as_tensor(f["B1"].astype(np.float32), device=dev),
               torch.as_tensor(f["B2"].astype(np.float32), device=dev), f["m"], f["n"]) for f in fr]
    prec = P.Precision.MFMA64 if args.precision == "mfma64" else P.Precision.MIXED
    d = P.Deblurrer(734, 1294, 15, 1, nf, prec)
    tune = d.prepare_batch(frames, lam=1e-4, flags=P.Flags.AUTOTUNE)
    tune.run()
    torch.cuda.synchronize()
    tuned = P.last_tuning()
    pb = d.prepare_batch(frames, lam=1e-4, flags=P.Flags.GRAPH)
    for _ in range(2):
        pb.run(check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        pb.run(check=False)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.batch_steps
    log(f"720p batch graph: {ms:.3f} ms per {nf}-frame batch")
    with P.profile() as prof:
        pe = d.prepare_batch(frames, lam=1e-4)
        for _ in range(3):
            pe.run(check=False)
        torch.cuda.synchronize()
    phases = {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof.result.items()}
    errs, ps, pt = [], [], []
    for f in (0, nf // 2, nf - 1):
        h = fr[f]
        B1 = h["B1"].astype(np.float32).astype(np.float64)
        B2 = h["B2"].astype(np.float32).astype(np.float64)
        Lo, R1, R2 = orc.deblur(B1, B2, h["m"], h["n"], 0, 1e-4)
        L = pb.latents[f].double().cpu().numpy()
        errs.append(max(rel(pb.K1s[f].cpu().numpy(), R1), rel(pb.K2s[f].cpu().numpy(), R2)))
        ps.append(psnr(L, Lo))
        pt.append(psnr(L, h["L"]))
    byts = sum(4 * (f["B1"].size + f["B2"].size + f["m"] * f["n"]) for f in fr)
    return dict(workload=f"{nf} x 720x1280 moving-blob frames, per-frame coprime kernels 7..15 (uneven), "
                         f"noise 1e-3, lambda 1e-4, FP32 frames ({args.precision} form), one call, autotuned, "
                         "HIP graph",
                metric="deblurred Mpixel/s", value=nf * 720 * 1280 / 1e6 / (ms / 1e3), unit="Mpixel/s",
                ms_per_batch=ms, tuning=tuned, phases_us_per_batch=phases,
                hbm_frac_end_to_end=byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                sampled_frames=[0, nf // 2, nf - 1], kernel_rel_l2_vs_oracle_max=max(errs),
                psnr_vs_oracle_db_min=min(ps), psnr_vs_truth_db_min=min(pt))


def bench_encoder_multilevel(P, torch, dev, host, args, orc=None):
    """The encoder on the GPU (kernel pairs drawn per frame, both streams
    blurred) and the multi-level workload (Sec. 3): the first stream frame's
    private stream without b least significant bits, decoded by the path."""
    h = host[0]
    m, n = h["m"], h["n"]
    k1, k2 = h["K1"].shape[0], h["K2"].shape[0]
    L = torch.as_tensor(h["L"], device=dev)                        # (3, m, n) FP32
    nf = 8
    K1s, K2s, att, _ = P.draw_kernel_pairs(1005, 0, nf, k1, k2, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    K1s, K2s, att, _ = P.draw_kernel_pairs(1005, 0, nf, k1, k2, device=dev)
    torch.cuda.synchronize()
    draw_ms = 1e3 * (time.perf_counter() - t0)
    b1 = torch.empty((3, m + k1 - 1, n + k1 - 1), dtype=torch.float32, device=dev)
    b2 = torch.empty((3, m + k2 - 1, n + k2 - 1), dtype=torch.float32, device=dev)
    for _ in range(3):
        P.encode(L, K1s[0], K2s[0], b1, b2)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for f in range(reps):
        P.encode(L, K1s[f % nf], K2s[f % nf], b1, b2)
    torch.cuda.synchronize()
    enc_ms = 1e3 * (time.perf_counter() - t0) / reps
    log(f"encoder: {draw_ms:.2f} ms for {nf} kernel pairs, {enc_ms:.3f} ms per 1080p RGB frame pair")
    # multi-level: the latent of frame 0 encoded on the GPU with a drawn 5 x 5 / 7 x 7
    # pair (no sensor noise), both streams at 8 bits, b low bits of the
    # private one dropped, decoded by the mixed form
    mk1, mk2 = 5, 7
    P1, P2, _, _ = P.draw_kernel_pairs(1005, 1, 1, mk1, mk2, device=dev)
    e1, e2 = P.encode(L, P1[0], P2[0])
    d = P.Deblurrer(e2.shape[1], e2.shape[2], mk2, 3, 1, P.Precision.MIXED, device=dev)
    d1 = P.dequantize(P.quantize(e1, 0))
    T1, T2 = P1[0].cpu().numpy(), P2[0].cpu().numpy()
    levels = []
    for b in range(0, 5):
        d2 = P.dequantize(P.quantize(e2, b))
        Lr, R1, R2 = d.deblur(d1, d2, m, n, lam=h["lam"])
        torch.cuda.synchronize()
        Lh = Lr.double().cpu().numpy()
        levels.append(dict(dropped_bits=b,
                           psnr_vs_truth_db=min(psnr(Lh[c], h["L"][c]) for c in range(3)),
                           kernel_rel_l2_vs_truth=max(rel(R1.cpu().numpy(), T1), rel(R2.cpu().numpy(), T2))))
        if orc is not None and b in (0, 2):
            # the oracle decodes the same 8-bit streams (outside any timed region)
            Lo, O1, O2 = orc.deblur(d1.double().cpu().numpy(), d2.double().cpu().numpy(), m, n, 0, h["lam"])
            levels[-1].update(kernel_rel_l2_vs_oracle=max(rel(R1.cpu().numpy(), O1), rel(R2.cpu().numpy(), O2)),
                              psnr_vs_oracle_db=min(psnr(Lh[c], Lo[c]) for c in range(3)))
        log(f"multi-level: {b} bits dropped -> PSNR {levels[-1]['psnr_vs_truth_db']:.2f} dB")
    return dict(encoder=dict(workload=f"{nf} kernel pairs {k1}x{k1}/{k2}x{k2} drawn and checked per frame; "
                                      "1080x1920 RGB latent blurred into both streams (FP32)",
                             draw_ms_per_batch=draw_ms, attempts=[int(a) for a in att],
                             blur_ms_per_frame=enc_ms, blur_mpixel_per_s=m * n / 1e3 / enc_ms),
                multilevel=dict(workload="latent of stream frame 0 (1080x1920 RGB) encoded on the GPU with a "
                                         "drawn 5x5/7x7 pair, no sensor noise; public stream at 8 bits, private "
                                         "stream without b least significant bits, decoded by the mixed form, "
                                         "lambda 1e-4", levels=levels))


# ---------------------------------------------------------------- main

def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    U = max(1, min(args.unique_frames, args.frames))

    # the stream's frames are generated in forked workers before anything touches the GPU
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=max(1, min(args.workers, U)), mp_context=mp.get_context("fork")) as ex:
        host = list(ex.map(_colour_frame, range(U)))
    log(f"stream: {U} distinct 1080p RGB frames generated in {time.perf_counter() - t0:.1f} s")

    import torch
    import paper_1203_4874_amd as P
    from oracle import cbp as orc

    dev = torch.device("cuda:0")
    P.lib()
    blob = P.load_mlp(device=dev) if os.path.exists(P.WEIGHTS) else None
    m, n = host[0]["m"], host[0]["n"]
    H1, W1 = host[0]["B1"].shape[1:]
    H2, W2 = host[0]["B2"].shape[1:]
    k1, k2 = host[0]["K1"].shape[0], host[0]["K2"].shape[0]
    S = host[0]["S"]
    bytes_frame = 4 * 3 * (H1 * W1 + H2 * W2 + m * n)          # read B1, B2 and write L, FP32, all channels
    nb = (args.frames + args.batch - 1) // args.batch

    # ---- headline: the mixed form on the stream
    t0 = time.perf_counter()
    head_prec = P.Precision.MFMA64 if args.precision == "mfma64" else P.Precision.MIXED
    main_s = Stream(P, torch, dev, host, args.frames, args.batch, torch.float32, head_prec, P.Flags.GRAPH,
                    autotune=not args.no_autotune, lanes=args.lanes)
    log(f"stream in HBM ({args.frames} frames, {time.perf_counter() - t0:.1f} s)")
    tm = time_stream(torch, main_s, args.warmup, args.steps)
    log(f"{args.precision}: {args.steps} steps in {tm['seconds']:.4f} s ({tm['ms_per_step']:.3f} ms per "
        f"{args.batch}-frame step)")
    if args.only_timing:
        if args.copy_calibration:
            copy_calibration(torch, dev)
        print(json.dumps({"metric": "deblurred Mpixel/s", "value": tm["value"], "unit": "Mpixel/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": tm["ms_per_step"],
                          "launch_shapes": getattr(main_s, "tuning", None), "note": "timing only"}))
        return
    phases = profile_stream(P, torch, main_s, min(nb, 8))
    lat = proc = None
    if args.fps > 0:
        lat, proc = arrival_pass(torch, main_s, args.fps)
        log(f"arrival pass: p50 {np.percentile(lat, 50):.1f} ms, p99 {np.percentile(lat, 99):.1f} ms")

    # sampled frames of the stream against the oracle (outside the timed regions)
    samples = sorted(set(int(round(x)) for x in np.linspace(0, args.frames - 1, max(1, args.cpu_frames))))
    orc_res = {}
    t0 = time.perf_counter()
    for f in samples:
        h = host[f % U]
        orc_res[f] = orc.deblur(h["B1"].astype(np.float64), h["B2"].astype(np.float64), m, n, 0, h["lam"])
    cpu_el = time.perf_counter() - t0
    threads = blas_threads()
    single = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits
        h = host[samples[0] % U]
        with threadpool_limits(1):
            t0 = time.perf_counter()
            orc.deblur(h["B1"].astype(np.float64), h["B2"].astype(np.float64), m, n, 0, h["lam"])
            single = time.perf_counter() - t0
    log(f"oracle: {len(samples)} frames in {cpu_el:.1f} s")

    def accuracy(s):
        ek, ps, pt, kt = [], [], [], []
        for f in samples:
            Lo, R1, R2 = orc_res[f]
            h = host[f % U]
            K1, K2 = s.kernels(f)
            L = s.out[f].double().cpu().numpy()
            ek.append(max(rel(K1, R1), rel(K2, R2)))
            kt.append(max(rel(K1, h["K1"]), rel(K2, h["K2"])))
            ps.append(min(psnr(L[c], Lo[c]) for c in range(3)))
            pt.append(min(psnr(L[c], h["L"][c]) for c in range(3)))
        return dict(sampled_frames=samples, kernel_rel_l2_vs_oracle_max=max(ek), psnr_vs_oracle_db_min=min(ps),
                    kernel_rel_l2_vs_truth_max=max(kt), psnr_vs_truth_db_min=min(pt))

    acc_main = accuracy(main_s)
    main_s_tuning = getattr(main_s, "tuning", None)

    # roofline: algorithmic bytes of one launch (the frames of one batch) over
    # the dominant kernel's average launch time, and over the whole step
    ph = {k: v for k, v in phases.items() if v}
    dom = max(ph, key=ph.get)
    per_launch = bytes_frame * args.batch
    ach = per_launch / (ph[dom] * 1e-6) / 1e9
    roof = dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                traffic=traffic_for(dom, "stream_1080p_rgb_batch8"), avg_us=ph[dom],
                algorithmic_bytes_per_launch=per_launch,
                launch=f"one launch per phase over the {args.batch} frames of a batch (3 channels each)",
                end_to_end=dict(achieved=per_launch / (tm["ms_per_step"] * 1e-3) / 1e9,
                                frac=per_launch / (tm["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                note="the same bytes over the whole step (every kernel of the path)"))
    if args.precision == "mfma64" and ph.get("gram"):
        # the MFMA64 Gram against the FP64 matrix-core peak: issued = the
        # v_mfma_f64_16x16x4f64 tiles it runs (2048 flops each: one per 16 x 16
        # lag-correlation tile and 64 rows), useful = the four columns of R
        # = M^T M it needs (4 x 2N x L real MACs per sample, pass and channel)
        def tiles(ka, kb):
            kk = [kb, ka, kb, ka]
            return sum(((14 + kk[a]) >> 4) - (0 if a == b else -((kk[b] + 14) >> 4)) + 1
                       for a in range(4) for b in range(a, 4))
        N = k1 + k2
        issued = useful = 0.0
        for l1, l2 in ((W1, W2), (H1, H2)):
            steps = (max(l1, l2) + 63) // 64
            issued += args.batch * S * 3 * tiles(k1, k2) * steps * 2048.0
            useful += args.batch * S * 3 * 4 * 2 * N * (l1 + k2 - 1) * 2.0
        t = ph["gram"] * 1e-6
        roof["gram_mfma"] = dict(kernel="gram", bound="mfma", unit="TFLOP/s", peak=FP64_MFMA_PEAK_TFLOPS,
                                 avg_us=ph["gram"], issued=issued / t / 1e12, useful=useful / t / 1e12,
                                 frac_issued=issued / t / 1e12 / FP64_MFMA_PEAK_TFLOPS,
                                 frac_useful=useful / t / 1e12 / FP64_MFMA_PEAK_TFLOPS,
                                 tiles_per_64_rows=tiles(k1, k2))

    # ---- the other forms on the stream
    extra = {}
    forms = [f for f in args.forms.split(",") if f]
    del main_s
    torch.cuda.empty_cache()
    for name in forms:
        if name.startswith("learned") and blob is None:
            continue
        if name == args.precision:
            continue
        if name == "fp64":
            s = Stream(P, torch, dev, host, args.frames, args.batch, torch.float64, P.Precision.FP64, P.Flags.GRAPH,
                       lanes=args.lanes)
        elif name in ("mixed", "mfma64"):
            s = Stream(P, torch, dev, host, args.frames, args.batch, torch.float32,
                       P.Precision.MFMA64 if name == "mfma64" else P.Precision.MIXED, P.Flags.GRAPH,
                       autotune=not args.no_autotune, lanes=args.lanes)
        elif name == "learned_mfma64":
            s = Stream(P, torch, dev, host, args.frames, args.batch, torch.float32, P.Precision.MFMA64, P.Flags.GRAPH,
                       mlp=blob, lanes=args.lanes)
        elif name == "learned_bf16":
            s = Stream(P, torch, dev, host, args.frames, args.batch, torch.float32, P.Precision.BF16, P.Flags.GRAPH,
                       mlp=blob, lanes=args.lanes)
        elif name == "learned":
            s = Stream(P, torch, dev, host, args.frames, args.batch, torch.float32, P.Precision.MIXED, P.Flags.GRAPH,
                       mlp=blob, lanes=args.lanes)
        else:
            continue
        t = time_stream(torch, s, args.warmup, args.steps)
        log(f"{name}: {t['ms_per_step']:.3f} ms per step")
        extra[name] = dict(value=t["value"], ms_per_step=t["ms_per_step"], **accuracy(s))
        del s
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = dict(value=len(samples) * m * n / 1e6 / cpu_el, unit="Mpixel/s", cores=int(threads), kind="oracle",
                   sample=f"frames {samples} of the stream (1080x1920 RGB), FP64 NumPy/SciPy oracle, "
                          f"{cpu_el:.1f} s",
                   single_thread=dict(value=m * n / 1e6 / single, seconds_per_frame=single),
                   host_cpu=cpu_model(), host_logical_cpus=os.cpu_count())

    enc_ml = bench_encoder_multilevel(P, torch, dev, host, args, orc)
    single_res = bench_single(P, torch, dev, orc, args, blob) if args.single_steps > 0 else None
    batched = bench_batch(P, torch, dev, orc, args) if args.batch_frames > 0 else None

    if args.copy_calibration:
        copy_calibration(torch, dev)

    line = {
        "metric": f"deblurred Mpixel/s (kernel recovery + deconv), {args.precision} form, PSNR vs FP64 oracle "
                  "reported",
        "value": tm["value"],
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tm["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (frames, FFT, division) + f64 (evaluation, Gram, eigen-solves, scale fix)"
                 + (", Gram on FP64 matrix cores" if args.precision == "mfma64" else ""),
        "data": "synthetic",
        "config": {"workload": f"stream of {args.frames} x 1080x1920 RGB frames (moving blobs, channel gains + "
                               f"texture) cycled from {U} generated frames, one coprime 15x15/17x17 pair, "
                               "noise 5e-3, lambda 1e-4, S=17, HIP-graph batches of "
                               f"{args.batch} frames, inputs resident in HBM",
                   "frames": args.frames, "unique_frames": U, "frames_per_step": args.batch,
                   "lanes": args.lanes,
                   "pixels_per_frame": m * n, "channels": 3, "blurred": [[H1, W1], [H2, W2]],
                   "kernels": [k1, k2], "samples": S,
                   "launch_shapes": None if args.no_autotune else main_s_tuning,
                   "fft_grid": [orc.smooth7(max(H1, H2)), orc.smooth7(max(W1, W2))]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "channel_mpixel_per_s": 3 * tm["value"],
        "accuracy": acc_main,
        "latency_ms": None if lat is None else {
            "arrival_fps": args.fps,
            "frame_p50": float(np.percentile(lat, 50)), "frame_p99": float(np.percentile(lat, 99)),
            "batch_p50": float(np.percentile(proc, 50)), "batch_p99": float(np.percentile(proc, 99)),
            "note": "frame: arrival to output, including the wait for its batch to fill; "
                    "batch: launch to output"},
        "phases_us_per_launch": phases,
        "plain_fp64": extra.get("fp64"),
        "other_forms": {k: v for k, v in extra.items() if k != "fp64"},
        "encoder": enc_ml["encoder"],
        "multilevel": enc_ml["multilevel"],
        "single_frame_480x640": single_res,
        "batched_720p": batched,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
