"""GPU parity of colour frames: one kernel pair per frame from the channels'
summed per-sample Grams, latent divided channel by channel, against the
oracle's colour route (stacked sample matrices, per-channel division) on the
same seeded frames.  Bars: kernels rel-L2 <= 1e-6 (FP64) / 1e-3 (mixed),
latent PSNR vs the oracle's latent >= 60 dB in every channel; a batch of
colour frames equals the single calls bit for bit."""

import numpy as np
import pytest

import synth
from oracle import cbp as orc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def P():
    import paper_1203_4874_amd as P
    P.lib()
    return P


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)


def _colour(seed, m, n, k1, k2, noise):
    r = synth.rng_for(seed, m, n)
    K1, K2 = synth.draw_coprime_pair(r, k1, k2, "uniform")
    gains = synth.rng_for(seed, 1).uniform(0.5, 1.0, 3)
    L = synth.gaussian_scene(synth.rng_for(seed, 2), m, n)
    Ls = np.stack([g * L + 0.05 * synth.rng_for(seed, 3, c).random((m, n)) for c, g in enumerate(gains)])
    B = [synth.blur_pair(synth.rng_for(seed, 4, c), Ls[c], K1, K2, noise) for c in range(3)]
    return np.stack([b[0] for b in B]), np.stack([b[1] for b in B]), K1, K2


@pytest.mark.parametrize("dtype,kt,lt", [(torch.float64, 1e-6, 60.0), (torch.float32, 1e-3, 60.0)])
@pytest.mark.parametrize("m,n,k1,k2,noise", [(64, 80, 5, 7, 1e-3), (41, 57, 6, 3, 0.0)])
def test_colour_deblur_matches_oracle(P, dtype, kt, lt, m, n, k1, k2, noise):
    B1, B2, _, _ = _colour(11 + k1, m, n, k1, k2, noise)
    if dtype == torch.float32:
        B1 = B1.astype(np.float32).astype(np.float64)
        B2 = B2.astype(np.float32).astype(np.float64)
    lam = 1e-4 if noise else 0.0
    Lo, R1, R2 = orc.deblur(B1, B2, m, n, 0, lam)
    b1 = torch.as_tensor(B1, dtype=dtype, device=_dev())
    b2 = torch.as_tensor(B2, dtype=dtype, device=_dev())
    k = max(k1, k2)
    prec = P.Precision.FP64 if dtype == torch.float64 else P.Precision.MIXED
    d = P.Deblurrer(m + k - 1, n + k - 1, k, 3, 1, prec)
    print(f"[case] colour {m}x{n} k=({k1},{k2}) noise {noise} {dtype}", flush=True)
    L, K1, K2 = d.deblur(b1, b2, m, n, lam=lam)
    torch.cuda.synchronize()
    L = L.double().cpu().numpy()
    e = max(rel(K1.cpu().numpy(), R1), rel(K2.cpu().numpy(), R2))
    ps = [psnr(L[c], Lo[c]) for c in range(3)]
    print(f"colour {m}x{n} k=({k1},{k2}) noise {noise} {dtype}: kernel rel-L2 {e:.2e}, "
          f"PSNR per channel {', '.join(f'{p:.1f}' for p in ps)} dB")
    assert L.shape == (3, m, n)
    assert e <= kt and min(ps) >= lt


def test_colour_batch_equals_single_calls(P):
    frames = [_colour(31, 48, 60, 4, 6, 1e-3), _colour(32, 56, 40, 7, 5, 1e-3)]
    shapes = [(48, 60), (56, 40)]
    dev = _dev()
    pairs = [(torch.as_tensor(f[0], dtype=torch.float64, device=dev),
              torch.as_tensor(f[1], dtype=torch.float64, device=dev), m, n) for f, (m, n) in zip(frames, shapes)]
    d = P.Deblurrer(62, 65, 7, 3, 2, P.Precision.FP64)
    print("[case] colour batch of 2", flush=True)
    Ls, K1s, K2s, st = d.deblur_batch(pairs, lam=1e-4)
    torch.cuda.synchronize()
    assert list(st) == [0, 0]
    for i, (b1, b2, m, n) in enumerate(pairs):
        H, W = max(b1.shape[1], b2.shape[1]), max(b1.shape[2], b2.shape[2])
        ds = P.Deblurrer(H, W, H - m + 1, 3, 1, P.Precision.FP64)
        L, K1, K2 = ds.deblur(b1, b2, m, n, lam=1e-4)
        torch.cuda.synchronize()
        assert torch.equal(L, Ls[i]) and torch.equal(K1, K1s[i]) and torch.equal(K2, K2s[i])
        Lo, R1, R2 = orc.deblur(frames[i][0], frames[i][1], m, n, 0, 1e-4)
        assert max(rel(K1.cpu().numpy(), R1), rel(K2.cpu().numpy(), R2)) <= 1e-6


def test_colour_1080p_frame_matches_oracle(P):
    """One frame of the 1080p colour stream at its full size: 1080x1920 RGB,
    one coprime 15x15 / 17x17 pair, noise 5e-3, lambda 1e-4, FP32 frames
    (mixed form), in the launch configuration the benchmark times (a batch
    call replayed as a HIP graph), against the oracle's colour route on the
    same FP32 values."""
    h = synth.config5_frame(0)
    B1 = h["B1"].astype(np.float32)
    B2 = h["B2"].astype(np.float32)
    m, n = h["m"], h["n"]
    dev = _dev()
    b1 = torch.as_tensor(B1, device=dev)
    b2 = torch.as_tensor(B2, device=dev)
    H, W = max(B1.shape[1], B2.shape[1]), max(B1.shape[2], B2.shape[2])
    d = P.Deblurrer(H, W, H - m + 1, 3, 1, P.Precision.MIXED)
    print("[case] 1080x1920 RGB frame, k=(15,17), mixed, graph replay", flush=True)
    pb = d.prepare_batch([(b1, b2, m, n)], lam=h["lam"], flags=P.Flags.GRAPH)
    pb.run()
    pb.run()
    torch.cuda.synchronize()
    L = pb.latents[0].double().cpu().numpy()
    Lo, R1, R2 = orc.deblur(B1.astype(np.float64), B2.astype(np.float64), m, n, 0, h["lam"])
    e = max(rel(pb.K1s[0].cpu().numpy(), R1), rel(pb.K2s[0].cpu().numpy(), R2))
    ps = [psnr(L[c], Lo[c]) for c in range(3)]
    print(f"1080p RGB: kernel rel-L2 vs oracle {e:.2e}, PSNR per channel {', '.join(f'{p:.1f}' for p in ps)} dB")
    assert L.shape == (3, m, n)
    assert e <= 1e-3 and min(ps) >= 60.0
