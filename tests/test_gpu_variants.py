"""GPU parity of the paper-faithful variants (CBP_FLAG_DIVIDE_B1,
CBP_FLAG_SCALE_K1, CBP_FLAG_ONE_AXIS) against oracle/variants.py, through
the C ABI.  Tolerances as for the default method: kernels rel-L2 <= 1e-6 in
the FP64 form, <= 1e-3 in the mixed form; latents against the oracle's
latent of the same variant at >= 60 dB (and max |diff| <= 1e-8 for the FP64
noiseless case).
"""


import numpy as np
import pytest

import synth
from oracle import variants as ov

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


def run(P, B1, B2, m, n, S, lam, flags, dtype):
    dev = _dev()
    b1 = torch.as_tensor(np.ascontiguousarray(B1), dtype=dtype, device=dev)
    b2 = torch.as_tensor(np.ascontiguousarray(B2), dtype=dtype, device=dev)
    k = max(b1.shape[-2], b2.shape[-2]) - m + 1
    prec = P.Precision.FP64 if dtype == torch.float64 else P.Precision.MIXED
    d = P.Deblurrer(max(b1.shape[-2], b2.shape[-2]), max(b1.shape[-1], b2.shape[-1]), k, precision=prec,
                    samples=S, device=dev, diag=True)
    print(f"variant flags {flags}: frames {tuple(b1.shape)} {dtype} S {S} lambda {lam}", flush=True)
    L, K1, K2 = d.deblur(b1, b2, m, n, lam, flags=flags)
    torch.cuda.synchronize()
    return (L.double().cpu().numpy(), K1.cpu().numpy(), K2.cpu().numpy(), d.read_diag(),
            b1.double().cpu().numpy(), b2.double().cpu().numpy())


CASES = {
    "divide_b1": (lambda P: P.Flags.DIVIDE_B1, "both", "single"),
    "scale_k1": (lambda P: P.Flags.SCALE_K1, "k1", "two"),
    "one_axis": (lambda P: P.Flags.ONE_AXIS, "one_axis", "two"),
    "scale_k1+divide_b1": (lambda P: P.Flags.SCALE_K1 | P.Flags.DIVIDE_B1, "k1", "single"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_variants_fp64_noiseless(P, name):
    fl, scale, division = CASES[name]
    c = synth.config1()
    S = 6 if scale == "one_axis" else 5
    lam = 1e-6 if division == "single" else 0.0
    L, K1, K2, dg, B1, B2 = run(P, c["B1"], c["B2"], 64, 64, S, lam, fl(P), torch.float64)
    Lo, R1, R2 = ov.deblur(B1, B2, 64, 64, S, lam, scale, division)
    assert rel(K1, R1) <= 1e-6 and rel(K2, R2) <= 1e-6
    assert rel(K1, c["K1"]) <= 1e-6
    assert np.max(np.abs(L - Lo)) <= 1e-8


@pytest.mark.parametrize("name", list(CASES))
def test_variants_mixed_noisy(P, name):
    """480 x 640 workload frame (FP32, noise 1e-3, 9 x 9 / 11 x 11)."""
    fl, scale, division = CASES[name]
    c = synth.config2()
    S = 12 if scale == "one_axis" else 11
    L, K1, K2, dg, B1, B2 = run(P, c["B1"], c["B2"], 480, 640, S, c["lam"], fl(P), torch.float32)
    Lo, R1, R2 = ov.deblur(B1, B2, 480, 640, S, c["lam"], scale, division)
    e = max(rel(K1, R1), rel(K2, R2))
    print(f"  kernel rel-L2 vs oracle {e:.2e}, latent PSNR vs oracle {psnr(L, Lo):.1f} dB", flush=True)
    assert e <= 1e-3
    assert psnr(L, Lo) >= 60.0


@pytest.mark.parametrize("k1,k2,S", [(7, 5, 7), (5, 7, 7), (4, 4, 9), (3, 6, 8)])
def test_one_axis_uneven_and_oversampled(P, k1, k2, S):
    r = synth.rng_for(31, k1, k2, S)
    Lt = synth.uniform_scene(r, 37, 45)
    K1, K2 = synth.draw_coprime_pair(r, k1, k2, "uniform", sample_counts=(S,))
    B1, B2 = synth.blur_pair(r, Lt, K1, K2, 0.0)
    L, G1, G2, dg, B1d, B2d = run(P, B1, B2, 37, 45, S, 0.0, P.Flags.ONE_AXIS, torch.float64)
    Lo, R1, R2 = ov.deblur(B1d, B2d, 37, 45, S, 0.0, "one_axis", "two")
    assert rel(G1, R1) <= 1e-6 and rel(G2, R2) <= 1e-6 and rel(G1, K1) <= 1e-6
    assert np.max(np.abs(L - Lo)) <= 1e-8
    assert dg["kernel_outside"][0] < 1e-12


def test_variant_flag_validation(P):
    c = synth.config1()
    dev = _dev()
    b1 = torch.as_tensor(c["B1"], device=dev)
    b2 = torch.as_tensor(c["B2"], device=dev)
    d = P.Deblurrer(68, 68, 5, precision=P.Precision.FP64, samples=5, device=dev)
    with pytest.raises(P.CbpError) as e:          # S = k1 = k2: no support equation
        d.deblur(b1, b2, 64, 64, 0.0, flags=P.Flags.ONE_AXIS)
    assert e.value.status == 1
    with pytest.raises(P.CbpError) as e:          # two scale fixes at once
        d.deblur(b1, b2, 64, 64, 0.0, flags=P.Flags.ONE_AXIS | P.Flags.SCALE_K1)
    assert e.value.status == 1


def test_variant_batch_equals_single_calls(P):
    """A batch with a variant flag equals its single-frame calls bit for bit."""
    dev = _dev()
    frames = []
    for s in range(2):
        r = synth.rng_for(41, s)
        Lt = synth.uniform_scene(r, 50, 60)
        K1, K2 = synth.draw_coprime_pair(r, 5, 7, "uniform", sample_counts=(8,))
        B1, B2 = synth.blur_pair(r, Lt, K1, K2, 1e-3)
        frames.append((torch.as_tensor(B1, dtype=torch.float32, device=dev),
                       torch.as_tensor(B2, dtype=torch.float32, device=dev), 50, 60))
    fl = P.Flags.ONE_AXIS | P.Flags.DIVIDE_B1
    d = P.Deblurrer(56, 66, 7, 1, 2, P.Precision.MIXED, samples=8, device=dev)
    Ls, K1s, K2s, st = d.deblur_batch(frames, 1e-4, flags=fl)
    torch.cuda.synchronize()
    assert list(st) == [0, 0]
    for f, (b1, b2, m, n) in enumerate(frames):
        one = P.Deblurrer(56, 66, 7, 1, 1, P.Precision.MIXED, samples=8, device=dev)
        L, K1, K2 = one.deblur(b1, b2, m, n, 1e-4, flags=fl)
        torch.cuda.synchronize()
        assert torch.equal(L, Ls[f]) and torch.equal(K1, K1s[f]) and torch.equal(K2, K2s[f])
