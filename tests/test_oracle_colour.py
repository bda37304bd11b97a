"""Pins of the oracle's colour-frame path (CPU).

Colour frames share one kernel pair: each sample's null vector comes from the
channels' sample matrices stacked (equivalently, the sum of the channels'
Gram matrices), and the latent is divided channel by channel.  The pins:
  * exact recovery of the true kernels from noiseless colour frames whose
    channels hold different scenes, also when one channel is blank (a route
    that used only one channel fails this);
  * three identical channels give the single-channel kernels;
  * a one-channel colour frame gives the grey-frame result bit for bit;
  * the stacked sample matrix's Gram is the sum of the channels' Grams;
  * the per-channel division with the true kernels is an exact inverse.
"""

import numpy as np

import synth
from oracle import cbp as orc


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _colour_pair(seed, m, n, k1, k2, blank=None, noise=0.0):
    r = synth.rng_for(seed, m, n)
    K1, K2 = synth.draw_coprime_pair(r, k1, k2, "uniform")
    Ls, B1s, B2s = [], [], []
    for c in range(3):
        L = synth.uniform_scene(synth.rng_for(seed, 7, c), m, n)
        if blank == c:
            L = np.zeros_like(L)
        B1, B2 = synth.blur_pair(synth.rng_for(seed, 8, c), L, K1, K2, noise)
        Ls.append(L)
        B1s.append(B1)
        B2s.append(B2)
    return np.stack(Ls), np.stack(B1s), np.stack(B2s), K1, K2


def test_noiseless_colour_frames_give_the_true_kernels():
    L, B1, B2, K1, K2 = _colour_pair(5, 40, 52, 5, 4)
    R1, R2 = orc.recover_kernels(B1, B2, 40, 52)
    assert rel(R1, K1) <= 1e-8 and rel(R2, K2) <= 1e-8
    Lr = orc.deconvolve(B1, B2, R1, R2, 40, 52, 0.0)
    assert Lr.shape == (3, 40, 52)
    assert np.abs(Lr - L).max() <= 1e-6


def test_blank_channel_does_not_break_recovery():
    _, B1, B2, K1, K2 = _colour_pair(6, 36, 44, 4, 5, blank=0)
    assert np.abs(B1[0]).max() == 0.0
    R1, R2 = orc.recover_kernels(B1, B2, 36, 44)
    assert rel(R1, K1) <= 1e-8 and rel(R2, K2) <= 1e-8
    # the blank channel alone carries nothing: its Grams are zero
    EX1, _ = orc.unit_circle_eval(B1[0], 5)
    assert np.abs(EX1).max() == 0.0


def test_identical_channels_give_the_grey_kernels():
    c = synth.config1()
    B1, B2 = c["B1"], c["B2"]
    G1, G2 = orc.recover_kernels(B1, B2, 64, 64)
    C1, C2 = orc.recover_kernels(np.stack([B1] * 3), np.stack([B2] * 3), 64, 64)
    assert rel(C1, G1) <= 1e-9 and rel(C2, G2) <= 1e-9


def test_one_channel_colour_frame_equals_grey_frame():
    _, B1, B2, _, _ = _colour_pair(7, 30, 34, 3, 5, noise=1e-3)
    G = orc.deblur(B1[1], B2[1], 30, 34, 0, 1e-4)
    C = orc.deblur(B1[1:2], B2[1:2], 30, 34, 0, 1e-4)
    assert np.array_equal(C[1], G[1]) and np.array_equal(C[2], G[2])
    assert np.array_equal(C[0][0], G[0])


def test_stacked_gram_is_the_channel_sum():
    _, B1, B2, _, _ = _colour_pair(8, 24, 28, 4, 3, noise=1e-2)
    S = 4
    ev1 = [orc.unit_circle_eval(B1[c], S) for c in range(3)]
    ev2 = [orc.unit_circle_eval(B2[c], S) for c in range(3)]
    for j in range(S):
        A = np.vstack([orc.sample_matrix(ev1[c][0][j], ev2[c][0][j], 4, 3) for c in range(3)])
        Gs = sum(orc.sample_gram(ev1[c][0][j], ev2[c][0][j], 4, 3) for c in range(3))
        assert np.abs(A.conj().T @ A - Gs).max() <= 1e-12 * np.abs(Gs).max()
