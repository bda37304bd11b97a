"""GPU failure paths: inputs the method cannot solve give their diagnostic
flag and finite outputs, through the C ABI.

  * a pair that is not coprime (K2 = K1 (x) f, Sec. 3 requires coprime
    kernels): every per-sample null space has dimension >= 2, so the sample
    Grams have no clear null direction -> CBP_DIAG_SAMPLE_WEAK;
  * a non-finite pixel: the evaluations, Grams and kernel estimates are
    non-finite -> CBP_DIAG_NONFINITE, both kernels returned as zeros and a
    zero latent;
  * an all-zero frame pair: every Gram is zero and the kernel estimate sums
    to zero or is not a number -> CBP_DIAG_KERNEL_ZERO (or NONFINITE), zero
    kernels and latent;
  * a learned-form network blob with a foreign header -> CBP_DIAG_BAD_NETWORK
    and unit weights, i.e. the plain kernels.
Every case is an ordinary input the kernels handle with bounded loops; none
faults or hangs the GPU.
"""

import numpy as np
import pytest

import synth
from oracle import learned as orl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NONFINITE, SAMPLE_WEAK, SCALE_WEAK, KERNEL_ZERO, FALLBACK, BAD_NETWORK = 1, 2, 4, 8, 16, 32


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def P():
    import paper_1203_4874_amd as P
    P.lib()
    return P


def _run(P, B1, B2, m, n, dtype=torch.float64, lam=0.0, mlp=None):
    k = max(B1.shape[-2], B2.shape[-2]) - m + 1
    prec = P.Precision.FP64 if dtype == torch.float64 else P.Precision.MIXED
    d = P.Deblurrer(max(B1.shape[-2], B2.shape[-2]), max(B1.shape[-1], B2.shape[-1]), k, precision=prec, diag=True)
    b1 = torch.as_tensor(B1, dtype=dtype, device=_dev())
    b2 = torch.as_tensor(B2, dtype=dtype, device=_dev())
    L, K1, K2 = d.deblur(b1, b2, m, n, lam=lam, mlp=mlp)
    torch.cuda.synchronize()
    return L.double().cpu().numpy(), K1.cpu().numpy(), K2.cpu().numpy(), d.read_diag()


def test_non_coprime_pair_flags_weak_samples(P):
    r = synth.rng_for(501)
    m, n = 40, 44
    L = r.random((m, n))
    K1 = synth.uniform_kernel(r, 4)
    f = np.array([[1.0, 0.5], [0.25, 1.0]])
    K2 = synth.full_conv2d(K1, f)
    K2 /= K2.sum()                            # K2 = K1 (x) f: a common factor of degree (3, 3)
    B1, B2 = synth.full_conv2d(L, K1), synth.full_conv2d(L, K2)
    print("[case] non-coprime 4x4 / 5x5 pair, 40x44, FP64", flush=True)
    Lg, G1, G2, dg = _run(P, B1, B2, m, n)
    print(f"flags {dg['flags']}, lambda1 / scale min "
          f"{np.min(dg['sample_lambda1'] / dg['sample_scale']):.2e}")
    assert dg["flags"] & SAMPLE_WEAK
    assert np.all(np.isfinite(Lg)) and np.all(np.isfinite(G1)) and np.all(np.isfinite(G2))


@pytest.mark.parametrize("dtype,lam", [(torch.float64, 0.0), (torch.float32, 1e-4)])
def test_nonfinite_pixel_gives_flag_and_zero_outputs(P, dtype, lam):
    c = synth.config1()
    B1 = c["B1"].copy()
    B1[17, 23] = np.nan
    print(f"[case] NaN pixel in B1, config-1 frame, {dtype}", flush=True)
    Lg, G1, G2, dg = _run(P, B1, c["B2"], c["m"], c["n"], dtype, lam)
    print(f"flags {dg['flags']}")
    assert dg["flags"] & NONFINITE
    assert np.all(G1 == 0.0) and np.all(G2 == 0.0)
    assert np.all(Lg == 0.0)
    B2 = c["B2"].copy()
    B2[0, 0] = np.inf
    print(f"[case] inf pixel in B2, config-1 frame, {dtype}", flush=True)
    Lg, G1, G2, dg = _run(P, c["B1"], B2, c["m"], c["n"], dtype, lam)
    assert dg["flags"] & NONFINITE and np.all(Lg == 0.0) and np.all(G1 == 0.0)


@pytest.mark.parametrize("dtype,lam", [(torch.float64, 0.0), (torch.float32, 1e-4)])
def test_all_zero_frames_give_flag_and_zero_outputs(P, dtype, lam):
    m, n, k1, k2 = 30, 34, 5, 6
    B1 = np.zeros((m + k1 - 1, n + k1 - 1))
    B2 = np.zeros((m + k2 - 1, n + k2 - 1))
    print(f"[case] all-zero frames {m}x{n} k=({k1},{k2}), {dtype}", flush=True)
    Lg, G1, G2, dg = _run(P, B1, B2, m, n, dtype, lam)
    print(f"flags {dg['flags']}")
    assert dg["flags"] & (KERNEL_ZERO | NONFINITE)
    assert np.all(G1 == 0.0) and np.all(G2 == 0.0) and np.all(Lg == 0.0)


def test_foreign_network_blob_falls_back_to_unit_weights(P):
    r = synth.rng_for(503)
    m, n = 48, 52
    L = synth.gaussian_scene(r, m, n)
    K1, K2 = synth.draw_coprime_pair(r, 5, 6, "uniform")
    B1, B2 = synth.blur_pair(synth.rng_for(503, 1), L, K1, K2, 1e-3)
    p = orl.init_params(np.random.default_rng(5))
    blob = P.mlp_blob_from_params(orl.pack(p).astype(np.float32), _dev())
    bad = blob.clone()
    bad[0] ^= 0xFF                            # first byte of the magic number
    print("[case] learned form with a corrupted blob header", flush=True)
    _, A1, A2, _ = _run(P, B1, B2, m, n, torch.float32, 1e-4)
    _, G1, G2, dg = _run(P, B1, B2, m, n, torch.float32, 1e-4, mlp=bad)
    print(f"flags {dg['flags']}, weights {dg['sample_weights'][:3]}, tau {dg['sample_weights'][-1]}")
    assert dg["flags"] & BAD_NETWORK
    S = dg["S"]
    assert np.all(dg["sample_weights"][:2 * S] == 1.0) and dg["sample_weights"][2 * S] == 0.0
    # unit weights and tau = 0: the learned assembly is the plain one
    e = max(np.linalg.norm(G1 - A1) / np.linalg.norm(A1), np.linalg.norm(G2 - A2) / np.linalg.norm(A2))
    assert e <= 1e-9
    # the intact blob raises no such flag
    _, _, _, dg = _run(P, B1, B2, m, n, torch.float32, 1e-4, mlp=blob)
    assert not dg["flags"] & BAD_NETWORK
