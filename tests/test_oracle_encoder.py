"""Pins of the encoder oracle (oracle/encoder.py): the counter-based
generator, the kernel draws and their coprimality rule, the blur, and the
multi-level 8-bit streams.

What fixes the expected values:
  * Philox4x64-10 against NumPy's own implementation (numpy.random.Philox,
    which advances its counter by one before each block of four words);
  * the blur against scipy.signal.convolve2d and, on integer inputs, exact
    polynomial multiplication (SymPy);
  * the Sylvester ratios against the input generator's independent SVD of
    the explicit Sylvester matrices (synth.sylvester_margin: ratio =
    margin^2), and a pair with a common factor (ratio at the rounding level);
  * the 8-bit streams by integer identities: 255 levels round-trip, the
    dropped bits are zero, values clamp to 0..255.
"""

import json
import os

import numpy as np
import pytest
from scipy import signal

import synth
from oracle import encoder as enc
from oracle import exact

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("counter,key", [((5, 7, 9, 11), (123, 456)), ((0, 0, 0, 0), (0, 0)),
                                         ((2 ** 64 - 1, 3, 0, 0), (2 ** 64 - 1, 2 ** 63)),
                                         ((12, 1, 3, 0), (1005, 17))])
def test_philox_matches_numpy(counter, key):
    # numpy's generator produces the block of counter + 1 first (a 256-bit counter)
    v = (sum(int(w) << (64 * i) for i, w in enumerate(counter)) - 1) % 2 ** 256
    prev = np.array([(v >> (64 * i)) & (2 ** 64 - 1) for i in range(4)], dtype=np.uint64)
    g = np.random.Philox(counter=prev, key=np.array(key, dtype=np.uint64))
    want = [int(x) for x in g.random_raw(4)]
    assert enc.philox4x64(counter, key) == want


def test_kernel_draw_words_and_normalisation():
    K = enc.kernel_draw(1005, 3, 2, 1, 5)
    assert K.shape == (5, 5) and np.all(K > 0)
    assert abs(K.sum() - 1.0) < 1e-15
    # the first four entries come from the block at counter (0, stream, attempt, 0)
    g = np.random.Philox(counter=np.array([2 ** 64 - 1, 1, 1, 0], dtype=np.uint64),
                         key=np.array([1005, 3], dtype=np.uint64))       # numpy steps to (0, 2, 1, 0)
    raw = [int(x) for x in g.random_raw(4)]
    u = np.array([((w >> 11) + 0.5) * 2.0 ** -53 for w in raw])
    full = np.array([((w >> 11) + 0.5) * 2.0 ** -53
                     for e in range(25) for w in [enc.philox4x64((e // 4, 2, 1, 0), (1005, 3))[e % 4]]])
    assert np.array_equal(full[:4], u)
    assert np.allclose(K.ravel() * full.sum(), full, rtol=1e-14, atol=0)
    # streams, attempts and frames give different kernels; the same inputs the same bits
    assert not np.allclose(K, enc.kernel_draw(1005, 3, 1, 1, 5))
    assert not np.allclose(K, enc.kernel_draw(1005, 3, 2, 0, 5))
    assert not np.allclose(K, enc.kernel_draw(1005, 4, 2, 1, 5))
    assert np.array_equal(K, enc.kernel_draw(1005, 3, 2, 1, 5))


@pytest.mark.parametrize("k1,k2,S", [(5, 5, 5), (7, 4, 7), (3, 9, 12), (1, 4, 4), (2, 2, 3)])
def test_sylvester_ratios_match_the_generators_svd(k1, k2, S):
    r = synth.rng_for(77, k1, k2)
    K1, K2 = synth.uniform_kernel(r, k1), synth.uniform_kernel(r, k2)
    rat = enc.sylvester_ratios(K1, K2, S)
    margin = synth.sylvester_margin(K1, K2, (S,))
    if k1 == 1 or k2 == 1:
        assert np.all(rat == 1.0) or np.min(rat) > 0.0
    else:
        assert abs(np.min(rat) - margin ** 2) <= 1e-9 * margin ** 2 + 1e-15


def test_common_factor_is_rejected():
    r = synth.rng_for(78, 1)
    F = synth.uniform_kernel(r, 3)
    K1 = synth.full_conv2d(synth.uniform_kernel(r, 3), F)
    K2 = synth.full_conv2d(synth.uniform_kernel(r, 4), F)
    rat = enc.sylvester_ratios(K1, K2, 6)
    assert np.max(rat) < 1e-20


def test_draw_pair_rule(monkeypatch):
    K1, K2, a = enc.draw_pair(1005, 0, 15, 17)
    assert a >= 0 and np.min(enc.sylvester_ratios(K1, K2, 17)) > enc.SYLV_MIN
    assert np.array_equal(K1, enc.kernel_draw(1005, 0, 1, a, 15))
    # the redraw loop: attempts whose pair fails are skipped
    calls = []

    def fake(A, B, S):
        calls.append(1)
        return np.full((2, S), 0.0 if len(calls) <= 2 else 1.0)
    monkeypatch.setattr(enc, "sylvester_ratios", fake)
    K1, K2, a = enc.draw_pair(9, 1, 4, 5)
    assert a == 2 and np.array_equal(K2, enc.kernel_draw(9, 1, 2, 2, 5))
    monkeypatch.setattr(enc, "sylvester_ratios", lambda A, B, S: np.zeros((2, S)))
    assert enc.draw_pair(9, 1, 4, 5)[2] == -1


def test_blur_matches_library_and_exact_products():
    r = np.random.default_rng(5)
    L = r.random((23, 31))
    K = r.random((6, 6))
    assert np.allclose(enc.blur(L, K), signal.convolve2d(L, K, mode="full"), rtol=1e-13, atol=1e-13)
    g = json.load(open(os.path.join(HERE, "golden", "tiny_integer_case.json")))
    Li, K2i = np.array(g["L"]), np.array(g["K2"])
    ex = exact.exact_blur(Li.astype(object), K2i.astype(object)).astype(np.int64)
    assert np.array_equal(enc.blur(Li.astype(np.float64), K2i.astype(np.float64)), ex)
    C = np.stack([L, 2 * L])
    assert np.allclose(enc.blur(C, K)[1], 2 * enc.blur(L, K))


def test_quantize_levels():
    q = np.arange(256, dtype=np.uint8)
    B = enc.dequantize(q)
    assert B.dtype == np.float32
    assert np.array_equal(enc.quantize(B), q)                    # every level round-trips
    for b in range(9):
        qb = enc.quantize(B, b)
        assert np.array_equal(qb, q & ((0xFF << b) & 0xFF))
        assert np.all(qb.astype(np.int64) % (1 << b) == 0)
    assert np.array_equal(enc.quantize(np.array([-0.3, 1.7, 0.999], np.float32)), [0, 255, 255])
    assert enc.quantize(np.array([25.6 / 255, 25.4 / 255], np.float64)).tolist() == [26, 25]
