"""The learned form's training targets (paper_1203_4874_amd/train_mlp.py):
on noiseless pairs the true kernel slices it builds are the method's exact
per-sample null vectors (pinned against the oracle's), and the true spectra
are the oracle's averaged spectra up to one complex scale."""

import numpy as np

import synth
from oracle import cbp as orc
from paper_1203_4874_amd import train_mlp as tm


def test_true_slices_are_the_noiseless_null_vectors():
    r = synth.rng_for(5)
    L = r.random((40, 44))
    K1, K2 = synth.draw_coprime_pair(r, 5, 4, "uniform")
    B1, B2 = synth.full_conv2d(L, K1), synth.full_conv2d(L, K2)
    S = 10
    _, _, f = orc.recover_kernels(B1, B2, 40, 44, S, full=True)
    xs = tm.true_slices(K1, K2, S)
    for p, (U, V) in enumerate(((f["XU"], f["XV"]), (f["YU"], f["YV"]))):
        for j in range(S):
            x = np.concatenate([U[j], V[j]])
            t = xs[p][j]
            c = abs(np.vdot(t, x)) ** 2 / (np.vdot(x, x).real * np.vdot(t, t).real)
            assert 1.0 - c <= 1e-10, (p, j, c)
    # the averaged spectra are the true ones times one complex number
    for c, K in enumerate((K1, K2)):
        Kt = tm.true_spectra(K, S)
        P, Q = f["P"][c], f["Q"][c]
        Kh = 0.5 * (f["a"][None, :] * P + f["b"][:, None] * Q)
        s = np.vdot(Kt, Kh) / np.vdot(Kt, Kt)
        assert np.abs(Kh - s * Kt).max() <= 1e-9 * np.abs(Kh).max()


def test_pairs_are_seeded_and_shaped():
    a = tm.make_pair(7)
    b = tm.make_pair(7)
    assert np.array_equal(a["B1"], b["B1"]) and a["S"] == 2 * max(a["K1"].shape[0], a["K2"].shape[0])
    assert a["B1"].dtype == np.float32 and a["B1"].shape[0] == tm.FRAME + a["K1"].shape[0] - 1
