"""GPU parity of the batching form: many frames of uneven sizes and kernel
sizes in one work-list launch per phase, the HIP-graph replay, and the
autotuned launch shapes, all through the C ABI.

Bars: a batched frame equals the same frame deblurred alone, bit for bit
(same kernels, same per-item arithmetic); graph replays equal eager calls bit
for bit; autotuned shapes (which change summation orders) meet the oracle
tolerances of the precision form (kernel rel-L2 <= 1e-3 mixed, <= 1e-6 FP64;
latent PSNR >= 60 dB against the oracle's latent).
"""

import numpy as np
import pytest

import synth
from oracle import cbp as orc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def to_dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=_dev())


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def psnr(a, b, peak=1.0):
    mse = float(np.mean((np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(peak * peak / mse)


@pytest.fixture(scope="module")
def P():
    import paper_1203_4874_amd as P
    P.lib()
    return P


def uneven_frames(seed, shapes, npd, noise=0.0):
    """(b1, b2, m, n) device tuples plus host copies, one coprime uniform pair per frame."""
    out, host = [], []
    for f, (m, n, k1, k2) in enumerate(shapes):
        r = synth.rng_for(seed, f)
        L = synth.gaussian_scene(r, m, n) if m * n > 4000 else r.random((m, n))
        K1, K2 = synth.draw_coprime_pair(r, k1, k2, "uniform")
        B1, B2 = synth.blur_pair(synth.rng_for(seed, 100 + f), L, K1, K2, noise)
        B1, B2 = B1.astype(npd), B2.astype(npd)
        dt = torch.float32 if npd is np.float32 else torch.float64
        out.append((to_dev(B1, dt), to_dev(B2, dt), m, n))
        host.append(dict(B1=B1.astype(np.float64), B2=B2.astype(np.float64), L=L, K1=K1, K2=K2, m=m, n=n))
    return out, host


SHAPES = [(40, 50, 3, 5), (96, 128, 9, 7), (31, 77, 7, 4), (120, 90, 15, 13), (64, 64, 5, 5),
          (17, 23, 2, 1), (80, 200, 11, 9)]


def _deblurrer(P, frames, precision, batch):
    H = max(max(b1.shape[-2], b2.shape[-2]) for b1, b2, _, _ in frames)
    W = max(max(b1.shape[-1], b2.shape[-1]) for b1, b2, _, _ in frames)
    k = max(max(b1.shape[-2], b2.shape[-2]) - m + 1 for b1, b2, m, _ in frames)
    return P.Deblurrer(H, W, k, 1, batch, precision)


@pytest.mark.parametrize("npd,prec,ktol", [(np.float32, 1, 1e-3), (np.float64, 0, 1e-6)])
def test_uneven_batch_equals_single_and_oracle(P, npd, prec, ktol):
    frames, host = uneven_frames(901, SHAPES, npd, noise=0.0)
    d = _deblurrer(P, frames, prec, len(frames))
    Ls, K1s, K2s, st = d.deblur_batch(frames, lam=0.0)
    torch.cuda.synchronize()
    assert st == [0] * len(frames)
    one = _deblurrer(P, frames, prec, 1)
    for (b1, b2, m, n), L, K1, K2, h in zip(frames, Ls, K1s, K2s, host):
        L1, J1, J2 = one.deblur(b1, b2, m, n)
        torch.cuda.synchronize()
        assert torch.equal(L1, L) and torch.equal(J1, K1) and torch.equal(J2, K2), (m, n)
        Lo, R1, R2 = orc.deblur(h["B1"], h["B2"], m, n, 0, 0.0)
        e = max(rel(K1.cpu().numpy(), R1), rel(K2.cpu().numpy(), R2))
        p = psnr(L.cpu().numpy(), Lo)
        print(f"frame {m}x{n} k=({h['K1'].shape[0]},{h['K2'].shape[0]}): kernel rel-L2 {e:.2e}, PSNR {p:.1f} dB")
        assert e <= ktol
        assert p >= 60


@pytest.mark.parametrize("nb", [1, 2, 3, 4])
def test_small_batches_equal_single(P, nb):
    """Calls of up to three frames carry their work-list head in the first
    launch's arguments, larger ones upload it: both give each frame the bits
    of the same frame deblurred alone, and a graph of a small call replays
    them."""
    frames, _ = uneven_frames(905, SHAPES[:nb], np.float32, noise=1e-3)
    d = _deblurrer(P, frames, 1, len(frames))
    Ls, K1s, K2s, st = d.deblur_batch(frames, lam=1e-4)
    torch.cuda.synchronize()
    assert st == [0] * nb
    one = _deblurrer(P, frames, 1, 1)
    for (b1, b2, m, n), L, K1, K2 in zip(frames, Ls, K1s, K2s):
        L1, J1, J2 = one.deblur(b1, b2, m, n, lam=1e-4)
        torch.cuda.synchronize()
        assert torch.equal(L1, L) and torch.equal(J1, K1) and torch.equal(J2, K2), (nb, m, n)
    if nb == 2:
        eager = d.prepare_batch(frames, lam=1e-4)
        g = d.prepare_batch(frames, lam=1e-4, flags=P.Flags.GRAPH)
        eager.run()
        torch.cuda.synchronize()
        ref = [(L.clone(), K1.clone()) for L, K1 in zip(eager.latents, eager.K1s)]
        for rep in range(3):
            for L in g.latents:
                L.zero_()
            g.run()
            torch.cuda.synchronize()
            for (L, K1), (Lr, K1r) in zip(zip(g.latents, g.K1s), ref):
                assert torch.equal(L, Lr) and torch.equal(K1, K1r), rep
            eager.run()
            torch.cuda.synchronize()


@pytest.mark.parametrize("npd", [np.float32, np.float64])
def test_kernel_only_call_equals_deblur_kernels(P, npd):
    """cbp_recover_kernels evaluates rows in k_eval_rows; cbp_deblur takes the
    same evaluation from its row FFT kernel.  Both give the same bits."""
    frames, _ = uneven_frames(77, [(96, 128, 9, 7), (60, 61, 4, 6)], npd, noise=1e-3)
    prec = 1 if npd is np.float32 else 0
    d = _deblurrer(P, frames, prec, 1)
    for b1, b2, m, n in frames:
        A1, A2 = d.recover_kernels(b1, b2, m, n)
        A1, A2 = A1.clone(), A2.clone()
        _, B1k, B2k = d.deblur(b1, b2, m, n, lam=1e-4)
        torch.cuda.synchronize()
        assert torch.equal(A1, B1k) and torch.equal(A2, B2k)


def test_graph_replays_equal_eager(P):
    frames, host = uneven_frames(903, SHAPES[:5], np.float32, noise=1e-3)
    d = _deblurrer(P, frames, 1, len(frames))
    eager = d.prepare_batch(frames, lam=1e-4)
    eager.run()
    torch.cuda.synchronize()
    ref = [(L.clone(), K1.clone(), K2.clone()) for L, K1, K2 in zip(eager.latents, eager.K1s, eager.K2s)]
    g = d.prepare_batch(frames, lam=1e-4, flags=P.Flags.GRAPH)
    for rep in range(3):
        for L in g.latents:
            L.zero_()
        g.run()
        torch.cuda.synchronize()
        for (L, K1, K2), (Lr, K1r, K2r) in zip(zip(g.latents, g.K1s, g.K2s), ref):
            assert torch.equal(L, Lr) and torch.equal(K1, K1r) and torch.equal(K2, K2r), rep
        eager.run()  # the program's own eager work between replays
        torch.cuda.synchronize()
    # new frame contents behind the same pointers: the replay reads them
    b1, b2, m, n = frames[1]
    b1.mul_(0.5)
    b2.mul_(0.5)
    g.run()
    eager.run()
    torch.cuda.synchronize()
    assert torch.equal(g.latents[1], eager.latents[1]) and torch.equal(g.K1s[1], eager.K1s[1])
    h = host[1]
    Lo, R1, _ = orc.deblur(h["B1"] * 0.5, h["B2"] * 0.5, m, n, 0, 1e-4)
    assert rel(g.K1s[1].cpu().numpy(), R1) <= 1e-3


def test_graph_replays_with_dynamic_column_items(P):
    """A batch whose column pass has more strips than workgroups hands them
    out from counters in the workspace head, which every call (and every
    replay of its graph) starts from zero: replays equal the eager call bit
    for bit, and a frame of the batch equals the same frame alone (one strip
    per workgroup, no counters)."""
    shapes = [(720, 1280, 7, 9)] * 6
    frames, host = uneven_frames(907, shapes, np.float32, noise=1e-3)
    d = _deblurrer(P, frames, 1, len(frames))
    eager = d.prepare_batch(frames, lam=1e-4)
    eager.run()
    torch.cuda.synchronize()
    ref = [(L.clone(), K1.clone()) for L, K1 in zip(eager.latents, eager.K1s)]
    g = d.prepare_batch(frames, lam=1e-4, flags=P.Flags.GRAPH)
    for rep in range(3):
        for L in g.latents:
            L.zero_()
        g.run()
        torch.cuda.synchronize()
        for (L, K1), (Lr, K1r) in zip(zip(g.latents, g.K1s), ref):
            assert torch.equal(L, Lr) and torch.equal(K1, K1r), rep
        eager.run()
        torch.cuda.synchronize()
    one = _deblurrer(P, frames[:1], 1, 1)
    b1, b2, m, n = frames[2]
    L1, J1, _ = one.deblur(b1, b2, m, n, lam=1e-4)
    torch.cuda.synchronize()
    assert torch.equal(L1, ref[2][0]) and torch.equal(J1, ref[2][1])
    h = host[2]
    Lo, R1, _ = orc.deblur(h["B1"], h["B2"], m, n, 0, 1e-4)
    assert rel(J1.cpu().numpy(), R1) <= 1e-3
    assert psnr(L1.cpu().numpy(), Lo) >= 60


def test_graph_single_frame_call(P):
    c = synth.config2()
    b1 = to_dev(c["B1"].astype(np.float32), torch.float32)
    b2 = to_dev(c["B2"].astype(np.float32), torch.float32)
    d = P.Deblurrer(490, 650, 11, precision=P.Precision.MIXED)
    La, K1a, _ = d.deblur(b1, b2, 480, 640, lam=1e-4)
    La, K1a = La.clone(), K1a.clone()
    out = torch.zeros_like(La)
    K1 = torch.zeros((9, 9), dtype=torch.float64, device=_dev())
    K2 = torch.zeros((11, 11), dtype=torch.float64, device=_dev())
    for _ in range(3):   # capture, then replays
        out.zero_()
        Lb, K1b, _ = d.deblur(b1, b2, 480, 640, lam=1e-4, out=out, K1=K1, K2=K2, flags=P.Flags.GRAPH)
        torch.cuda.synchronize()
        assert torch.equal(La, Lb) and torch.equal(K1a, K1b)


def test_autotuned_batch_meets_oracle(P):
    # six frames: a batch class of its own (the tuned choice applies to its class only)
    frames, host = uneven_frames(905, SHAPES[:6], np.float32, noise=0.0)
    d = _deblurrer(P, frames, 1, len(frames))
    pb = d.prepare_batch(frames, lam=0.0, flags=P.Flags.AUTOTUNE)
    pb.run()
    torch.cuda.synchronize()
    t = P.last_tuning()
    print("autotuned:", t)
    assert t is not None and t["ms"] > 0
    first = [(L.clone(), K1.clone()) for L, K1 in zip(pb.latents, pb.K1s)]
    plain = d.prepare_batch(frames, lam=0.0)   # same class: the stored choice applies without the flag
    plain.run()
    torch.cuda.synchronize()
    for (L, K1), L2, K12, h in zip(first, plain.latents, plain.K1s, host):
        assert torch.equal(L, L2) and torch.equal(K1, K12)
        Lo, R1, R2 = orc.deblur(h["B1"], h["B2"], h["m"], h["n"], 0, 0.0)
        assert rel(K1.cpu().numpy(), R1) <= 1e-3
        assert psnr(L.cpu().numpy(), Lo) >= 60


def test_batch_over_one_launch_chunk(P):
    """More frames than one launch holds (256): the batch is split."""
    shapes = [(16 + f % 9, 20 + f % 7, 2 + f % 3, 1 + f % 4) for f in range(260)]
    frames, host = uneven_frames(907, shapes, np.float64)
    d = _deblurrer(P, frames, 0, len(frames))
    Ls, K1s, K2s, st = d.deblur_batch(frames)
    torch.cuda.synchronize()
    assert st == [0] * len(frames)
    one = _deblurrer(P, frames, 0, 1)
    for f in list(range(0, 260, 37)) + [255, 256, 259]:
        b1, b2, m, n = frames[f]
        L1, J1, _ = one.deblur(b1, b2, m, n)
        torch.cuda.synchronize()
        assert torch.equal(L1, Ls[f]) and torch.equal(J1, K1s[f]), f
        h = host[f]
        Lo, R1, _ = orc.deblur(h["B1"], h["B2"], m, n, 0, 0.0)
        assert rel(K1s[f].cpu().numpy(), R1) <= 1e-6


def test_batch_skips_invalid_frames(P):
    frames, _ = uneven_frames(909, SHAPES[:3], np.float64)
    b1, b2, m, n = frames[1]
    bad = list(frames)
    bad[1] = (b1, b2[:, :-1], m, n)          # W1 - W2 != H1 - H2
    d = _deblurrer(P, frames, 0, 3)
    with pytest.raises(P.CbpError) as e:
        d.deblur_batch(bad)
    assert e.value.status == 2
    pb = d.prepare_batch(bad)
    st = pb.run(check=False)
    torch.cuda.synchronize()
    assert st == [0, 2, 0]
    one = _deblurrer(P, frames, 0, 1)
    for f in (0, 2):
        L1, _, _ = one.deblur(*frames[f])
        torch.cuda.synchronize()
        assert torch.equal(L1, pb.latents[f])


def test_surveillance_batch_720p_sampled(P):
    """The batching workload at full frame size: 720x1280 moving-blob frames,
    per-frame uneven kernels 7..15, noise 1e-3, lambda 1e-4, FP32 frames,
    one graph per batch (the benchmark's launch configuration), 16 frames;
    three frames checked against the oracle."""
    fr = list(synth.config3_frames(nframes=16))
    frames = [(to_dev(f["B1"].astype(np.float32), torch.float32), to_dev(f["B2"].astype(np.float32), torch.float32),
               f["m"], f["n"]) for f in fr]
    d = P.Deblurrer(734, 1294, 15, 1, len(frames), P.Precision.MIXED)
    pb = d.prepare_batch(frames, lam=1e-4, flags=P.Flags.GRAPH)
    st = pb.run()
    torch.cuda.synchronize()
    assert st == [0] * len(frames)
    for f in (0, 7, 15):
        h = fr[f]
        B1 = h["B1"].astype(np.float32).astype(np.float64)
        B2 = h["B2"].astype(np.float32).astype(np.float64)
        Lo, R1, R2 = orc.deblur(B1, B2, h["m"], h["n"], 0, 1e-4)
        e = max(rel(pb.K1s[f].cpu().numpy(), R1), rel(pb.K2s[f].cpu().numpy(), R2))
        p = psnr(pb.latents[f].cpu().numpy(), Lo)
        print(f"720p frame {f} k=({h['K1'].shape[0]},{h['K2'].shape[0]}): kernel rel-L2 {e:.2e}, PSNR vs oracle {p:.1f} dB")
        assert e <= 1e-3
        assert p >= 60
