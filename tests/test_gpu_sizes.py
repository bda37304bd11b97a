"""GPU parity of blind kernel-size estimation (cbp_estimate_kernel_sizes)
against the oracle (oracle/sizes.py), through the C ABI.

Both sides take the decision from their own FP64 scores, so the cases keep a
clear margin; the bar:
  * the estimate (k1, k2) and its flags are identical;
  * per-sample ratios s = lambda_min / lambda_max agree within
    5e-14 + 1e-7 s (the GPU rounds the double-double Gram to FP64 and
    brackets the eigenvalues by Sturm multisection to ~1e-14 of lambda_max);
  * candidate scores agree within the ratio bound carried into the log10
    median, 1e-6 + (5e-14 / s + 1e-7) / ln 10 decades at the smaller score s.
"""

import numpy as np
import pytest

import synth
from oracle import sizes as osz

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


def pair(k1, k2, m, n, noise=0.0, seed=7, channels=0):
    r = synth.rng_for(seed, k1, k2, m)
    K1, K2 = synth.draw_coprime_pair(r, k1, k2, "uniform")
    if channels:
        Ls = [synth.uniform_scene(r, m, n) for _ in range(channels)]
        B = [synth.blur_pair(r, L, K1, K2, noise) for L in Ls]
        return np.stack([b[0] for b in B]), np.stack([b[1] for b in B])
    return synth.blur_pair(r, synth.uniform_scene(r, m, n), K1, K2, noise)


def compare(P, B1, B2, kmin, kmax, step=1, S=0, dtype=torch.float64):
    dev = _dev()
    b1 = torch.as_tensor(np.ascontiguousarray(B1), dtype=dtype, device=dev)
    b2 = torch.as_tensor(np.ascontiguousarray(B2), dtype=dtype, device=dev)
    print(f"sizes: frames {tuple(b1.shape)} / {tuple(b2.shape)} {dtype}, search {kmin}..{kmax} step {step} "
          f"S {S}", flush=True)
    g = P.estimate_kernel_sizes(b1, b2, kmin, kmax, step, S, ratios=True)
    o = osz.estimate_sizes(b1.double().cpu().numpy(), b2.double().cpu().numpy(), kmin, kmax, step, S)
    assert g["candidates"] == o["candidates"]
    assert g["S"] == o["S"]
    assert (g["k1"], g["k2"], g["flags"]) == (o["k1"], o["k2"], o["flags"]), (g["scores"], o["scores"])
    assert np.all(np.abs(g["ratios"] - o["ratios"]) <= 5e-14 + 1e-7 * o["ratios"])
    # the ratio bound carried into the log10 median: (5e-14 / s + 1e-7) / ln 10 decades
    s_low = 10.0 ** np.minimum(g["scores"], o["scores"])
    assert np.all(np.abs(g["scores"] - o["scores"]) <= 1e-6 + (5e-14 / s_low + 1e-7) / np.log(10.0))
    return g


@pytest.mark.parametrize("k1,k2,m,n", [(5, 5, 40, 46), (7, 5, 33, 41), (4, 9, 36, 30), (1, 3, 20, 25),
                                       (12, 11, 40, 52), (16, 16, 48, 40)])
def test_sizes_match_oracle_and_truth(P, k1, k2, m, n):
    B1, B2 = pair(k1, k2, m, n)
    g = compare(P, B1, B2, 1, 20)
    assert (g["k1"], g["k2"]) == (k1, k2)


@pytest.mark.parametrize("k", [9, 13, 25])
def test_paper_odd_search_9_to_25(P, k):
    B1, B2 = pair(k, k, 30, 34)
    g = compare(P, B1, B2, 9, 25, 2)
    assert g["candidates"] == list(range(9, 26, 2))
    assert (g["k1"], g["k2"]) == (k, k)


def test_wrong_size_ranges(P):
    """A search that misses the true size: below it nothing is singular, above
    it the first candidate already is; both flagged, both as the oracle."""
    B1, B2 = pair(9, 9, 30, 34)
    g = compare(P, B1, B2, 3, 8)
    assert g["flags"] == P.SIZE_NONE_SINGULAR and g["k1"] == 8
    g = compare(P, B1, B2, 11, 16)
    assert g["flags"] == P.SIZE_FIRST_SINGULAR and g["k1"] == 11


def test_shared_factor_and_colour(P):
    r = synth.rng_for(3, 1)
    L = synth.uniform_scene(r, 36, 40)
    G1, G2 = synth.draw_coprime_pair(r, 5, 4, "uniform")
    F = synth.uniform_kernel(r, 3)
    B1 = synth.full_conv2d(L, synth.full_conv2d(G1, F))
    B2 = synth.full_conv2d(L, synth.full_conv2d(G2, F))
    g = compare(P, B1, B2, 1, 12)
    assert (g["k1"], g["k2"]) == (5, 4)           # the cofactors of the common factor
    C1, C2 = pair(6, 4, 30, 33, channels=3)
    g = compare(P, C1, C2, 1, 10, S=7)
    assert (g["k1"], g["k2"]) == (6, 4)


def test_fp32_frames_and_noise(P):
    """FP32 frames (the oracle reads the same float32 values) and a mildly
    noisy pair whose scores both sides compute alike."""
    B1, B2 = pair(7, 9, 60, 64)
    compare(P, B1, B2, 1, 14, dtype=torch.float32)
    N1, N2 = pair(5, 6, 64, 72, noise=1e-6)
    g = compare(P, N1, N2, 1, 12)
    assert (g["k1"], g["k2"]) == (5, 6)


def test_bench_sized_frame(P):
    """A 480x640 frame of the single-frame workload's shape with 9 x 9 / 11 x 11
    uniform kernels, the candidates 5..16 and S = 11."""
    B1, B2 = pair(9, 11, 480, 640, seed=11)
    g = compare(P, B1, B2, 5, 16, S=11, dtype=torch.float32)
    assert (g["k1"], g["k2"]) == (9, 11)
