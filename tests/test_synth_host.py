"""Host checks of the seeded input generators (no method arithmetic here)."""

import numpy as np

import synth


def test_blob_frame_equals_the_sequence():
    seq = list(synth.blob_sequence(77, 5, 40, 56))
    for f in (0, 1, 4):
        assert np.array_equal(synth.blob_frame(77, f, 40, 56), seq[f])


def test_config5_frame_shapes_and_shared_kernels():
    a = synth.config5_frame(0, m=30, n=44)
    b = synth.config5_frame(3, m=30, n=44)
    assert a["B1"].shape == (3, 30 + 14, 44 + 14) and a["B2"].shape == (3, 30 + 16, 44 + 16)
    assert np.array_equal(a["K1"], b["K1"]) and np.array_equal(a["K2"], b["K2"])
    assert abs(a["K1"].sum() - 1) < 1e-12 and abs(a["K2"].sum() - 1) < 1e-12
    assert not np.array_equal(a["L"][0], a["L"][1])
