"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point declared in include/cbp.h, the diag record layout matches the
binding, the workspace size is monotone, and host-side validation returns
its error codes before any device work (the pointers passed here are never
dereferenced)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_1203_4874_amd as P
    if not os.path.exists(P.library_path):
        pytest.fail("libcbp.so is not built (run python -m paper_1203_4874_amd.build)")
    return P


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cbp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cbp_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(P):
    L = P.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(P._SIGS), "binding signatures must cover exactly the header"


def test_version_status_and_diag_layout(P):
    L = P.lib()
    assert L.cbp_version().decode().count(".") == 2
    assert L.cbp_status_string(0) == b"ok"
    assert L.cbp_status_string(5) == b"workspace too small"
    assert L.cbp_diag_size() == ctypes.sizeof(P.CbpDiag)


def test_workspace_size_monotone_and_invalid(P):
    a = P.workspace_size(490, 650, 11)
    assert a > 0
    assert P.workspace_size(720, 1300, 15) > a
    # a batch holds every frame plus a head of frame descriptors and item prefix sums
    assert 3 * a < P.workspace_size(490, 650, 11, batch=4) <= 4 * a
    assert P.workspace_size(490, 650, 33) == 0
    assert P.workspace_size(0, 650, 11) == 0


def _img(ptr, dtype, h, w, c=1):
    return P_.CbpImage(ptr, dtype, h, w, c, w, h * w)


def test_host_validation_codes(P):
    global P_
    P_ = P
    L = P.lib()
    i1, i2 = _img(0x1000, 0, 488, 648), _img(0x2000, 0, 490, 650)
    lat = _img(0x3000, 0, 480, 640)
    o = P.CbpOptions()
    o.precision = P.Precision.MIXED
    call = lambda a, b, c, opts: L.cbp_deblur(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), None, None,
                                              ctypes.byref(opts))
    assert call(i1, i2, lat, o) == 5                       # no workspace
    assert call(i1, i2, _img(0x3000, 0, 481, 640), o) == 2  # latent inconsistent with frames
    assert call(i1, _img(0x2000, 0, 490, 651), lat, o) == 2  # H1-H2 != W1-W2
    assert call(i1, i2, _img(0x3000, 1, 480, 640), o) == 1  # latent dtype differs
    o.samples = 5                                           # S < max k
    assert call(i1, i2, lat, o) == 1
    o.samples = 0
    o.lambda_ = -1.0
    assert call(i1, i2, lat, o) == 1
    o.lambda_ = 0.0
    o.precision = P.Precision.FP64                          # FP64 form needs FP64 frames
    assert call(i1, i2, lat, o) == 1
    o.precision = P.Precision.BF16                          # matrix-core forms take FP32 frames
    assert call(i1, i2, lat, o) == 5                        # (accepted; no workspace)
    assert call(_img(0x1000, 1, 488, 648), _img(0x2000, 1, 490, 650), _img(0x3000, 1, 480, 640), o) == 1
    wide = (_img(0x1000, 0, 480 + 19, 640 + 19), _img(0x2000, 0, 480 + 15, 640 + 15))   # k1 + k2 = 36 > 32
    assert call(wide[0], wide[1], lat, o) == 6
    o.precision = P.Precision.MFMA32
    assert call(wide[0], wide[1], lat, o) == 6
    assert call(i1, i2, lat, o) == 5
    o.precision = P.Precision.MIXED
    o.learned = 1                                           # the learned form needs its network blob
    assert call(i1, i2, lat, o) == 1
    o.learned = 0
    big = _img(0x1000, 0, 488 + 40, 648 + 40)               # k = 41 > 32
    assert call(big, _img(0x2000, 0, 490 + 40, 650 + 40), _img(0x3000, 0, 480, 640), o) == 2
    assert call(_img(0, 0, 488, 648), i2, lat, o) == 1      # null data pointer
    assert L.cbp_deblur(None, ctypes.byref(i2), ctypes.byref(lat), None, None, ctypes.byref(o)) == 1
    o.flags = 64                                            # unknown option flag
    assert call(i1, i2, lat, o) == 1
    o.flags = 0


def test_batch_host_validation(P):
    """Per-frame statuses of cbp_deblur_batch come from host checks; a batch
    whose every frame is invalid returns before any HIP call."""
    global P_
    P_ = P
    L = P.lib()
    o = P.CbpOptions()
    o.precision = P.Precision.MIXED
    n = 3
    I1 = (P.CbpImage * n)(_img(0x1000, 0, 488, 648), _img(0x1000, 0, 488, 648), _img(0, 0, 488, 648))
    I2 = (P.CbpImage * n)(_img(0x2000, 0, 490, 651), _img(0x2000, 1, 490, 650), _img(0x2000, 0, 490, 650))
    IO = (P.CbpImage * n)(_img(0x3000, 0, 480, 640), _img(0x3000, 0, 480, 640), _img(0x3000, 0, 480, 640))
    st = (ctypes.c_int * n)()
    r = L.cbp_deblur_batch(n, I1, I2, IO, None, None, st, ctypes.byref(o))
    assert list(st) == [2, 1, 1]      # H1-H2 != W1-W2; dtypes differ; null data pointer
    assert r == 2                     # the first failure
    assert L.cbp_deblur_batch(0, I1, I2, IO, None, None, st, ctypes.byref(o)) == 1
    t = P.CbpTuning()
    assert L.cbp_last_tuning(None) == 1


def test_noalloc_host_validation(P):
    """cbp_deblur_noalloc rejects, before any HIP call, the flags that would
    allocate (graphs, the autotuner) and frames whose workspace exceeds the
    library's scratch; the scratch bound is the stated 48 MiB and the mixed
    1080p grayscale frame it is sized for fits it."""
    global P_
    P_ = P
    L = P.lib()
    limit = P.noalloc_scratch_bytes()
    assert limit == 48 << 20
    assert P.workspace_size(1096, 1936, 17, 1, 1, P.Precision.MIXED) <= limit
    o = P.CbpOptions()
    o.precision = P.Precision.MIXED
    call = lambda a, b, c, opts: L.cbp_deblur_noalloc(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), None,
                                                      None, ctypes.byref(opts))
    i1, i2 = _img(0x1000, 0, 488, 648), _img(0x2000, 0, 490, 650)
    lat = _img(0x3000, 0, 480, 640)
    for f in (P.Flags.GRAPH, P.Flags.AUTOTUNE):
        o.flags = f
        assert call(i1, i2, lat, o) == 6
    o.flags = 0
    assert call(i1, i2, _img(0x3000, 0, 481, 640), o) == 2   # the usual shape checks come first
    # a 1080p RGB frame needs ~132 MiB of workspace: too large for the scratch
    big1, big2 = _img(0x1000, 0, 1094, 1934, 3), _img(0x2000, 0, 1096, 1936, 3)
    assert call(big1, big2, _img(0x3000, 0, 1080, 1920, 3), o) == 5
    assert b"scratch" in L.cbp_last_error()
    assert L.cbp_deblur_noalloc(None, ctypes.byref(i2), ctypes.byref(lat), None, None, ctypes.byref(o)) == 1


def test_size_estimation_host_validation(P):
    """cbp_estimate_kernel_sizes: host-side errors before any HIP call."""
    global P_
    P_ = P
    L = P.lib()
    o = P.CbpOptions()
    o.precision = P.Precision.FP64
    se = P.CbpSizeSearch(1, 16, 1, 0)
    i1, i2 = _img(0x1000, 1, 50, 60), _img(0x2000, 1, 48, 58)
    call = lambda a, b, s, opts, res=0x4000: L.cbp_estimate_kernel_sizes(
        ctypes.byref(a), ctypes.byref(b), ctypes.byref(s), res, None, ctypes.byref(opts))
    assert call(i1, i2, se, o) == 5                                    # no workspace
    assert call(i1, _img(0x2000, 1, 48, 59), se, o) == 2               # H1 - H2 != W1 - W2
    assert call(i1, i2, P.CbpSizeSearch(0, 16, 1, 0), o) == 1          # kmin < 1
    assert call(i1, i2, P.CbpSizeSearch(5, 4, 1, 0), o) == 1           # kmax < kmin
    assert call(i1, i2, P.CbpSizeSearch(1, 16, 0, 0), o) == 1          # step < 1
    assert call(i1, i2, P.CbpSizeSearch(1, 16, 1, 33), o) == 1         # S > 32
    assert call(i1, i2, P.CbpSizeSearch(40, 50, 1, 0), o) == 2         # no candidate fits
    assert call(i1, i2, se, o, res=None) == 1                          # no result buffer
    assert call(_img(0x1000, 0, 50, 60), i2, se, o) == 1               # dtypes differ
    o.precision = P.Precision.MFMA32
    assert call(_img(0x1000, 0, 50, 60), _img(0x2000, 0, 48, 58), se, o) == 1   # dd Gram forms only
    o.precision = P.Precision.FP64
    ws = lambda *a: L.cbp_size_workspace_size(*a[:4], ctypes.byref(a[4]), ctypes.byref(o))
    assert ws(50, 60, 1, 2, se) > 0
    assert ws(50, 60, 1, 2, P.CbpSizeSearch(1, 16, 0, 0)) == 0
    assert ws(50, 60, 3, 2, se) > ws(50, 60, 1, 2, se)


def test_encoder_host_validation(P):
    """Encoder and 8-bit stream entry points: host-side errors before any HIP call."""
    global P_
    P_ = P
    L = P.lib()
    assert L.cbp_draw_kernel_pairs(1, 0, 0, 5, 5, 0, 0x1000, 0x2000, 0x3000, None, None) == 1    # no frame
    assert L.cbp_draw_kernel_pairs(1, 0, 4, 0, 5, 0, 0x1000, 0x2000, 0x3000, None, None) == 2    # k < 1
    assert L.cbp_draw_kernel_pairs(1, 0, 4, 5, 33, 0, 0x1000, 0x2000, 0x3000, None, None) == 2   # k > 32
    assert L.cbp_draw_kernel_pairs(1, 0, 4, 5, 5, 33, 0x1000, 0x2000, 0x3000, None, None) == 1   # S > 32
    assert L.cbp_draw_kernel_pairs(1, -1, 4, 5, 5, 0, 0x1000, 0x2000, 0x3000, None, None) == 1   # frame0 < 0
    assert L.cbp_draw_kernel_pairs(1, 0, 4, 5, 5, 0, None, 0x2000, 0x3000, None, None) == 1
    lat = _img(0x1000, 0, 40, 50)
    enc = lambda l, k1, k2, b1, b2: L.cbp_encode(ctypes.byref(l), 0x5000, k1, 0x6000, k2, ctypes.byref(b1),
                                                 ctypes.byref(b2), None)
    assert enc(lat, 5, 3, _img(0x2000, 0, 45, 54), _img(0x3000, 0, 42, 52)) == 2     # B1 height != m + k1 - 1
    assert enc(lat, 5, 3, _img(0x2000, 1, 44, 54), _img(0x3000, 0, 42, 52)) == 1     # dtype differs
    assert enc(lat, 40, 3, _img(0x2000, 0, 79, 89), _img(0x3000, 0, 42, 52)) == 2    # k > 32
    q8 = P.CbpImage(0x7000, 2, 40, 50, 1, 50, 2000)
    assert L.cbp_quantize(ctypes.byref(lat), ctypes.byref(q8), 9, None) == 1         # drop_bits > 8
    assert L.cbp_quantize(ctypes.byref(lat), ctypes.byref(lat), 0, None) == 1        # dst must be 8-bit
    assert L.cbp_quantize(ctypes.byref(lat), ctypes.byref(P.CbpImage(0x7000, 2, 41, 50, 1, 50, 2050)), 0,
                          None) == 2
    assert L.cbp_dequantize(ctypes.byref(lat), ctypes.byref(lat), None) == 1        # src must be 8-bit
    # an 8-bit image is not a frame of the deblurring entry points
    o = P.CbpOptions()
    o.precision = P.Precision.MIXED
    assert L.cbp_deblur(ctypes.byref(q8), ctypes.byref(q8), ctypes.byref(lat), None, None, ctypes.byref(o)) == 1
