"""The allocation-free entry point (cbp_deblur_noalloc) against cbp_deblur.

Both run the same kernels with the same launch shapes on the same frame, so
the latent and the kernels must agree bit for bit (the workspace's address
and its previous contents do not enter any result).  Two calls in a row, the
second on a smaller frame of another dtype, check that the shared scratch
keeps nothing a later call depends on.  The device's free memory is the same
before and after the calls (the entry point allocates nothing).
"""

import ctypes

import numpy as np
import pytest

import synth

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


def _case(P, cfg, dtype, lam):
    dev = _dev()
    b1 = torch.as_tensor(np.ascontiguousarray(cfg["B1"]), dtype=dtype, device=dev)
    b2 = torch.as_tensor(np.ascontiguousarray(cfg["B2"]), dtype=dtype, device=dev)
    m, n = cfg["m"], cfg["n"]
    k1, k2 = cfg["K1"].shape[0], cfg["K2"].shape[0]
    ref = P.Deblurrer(max(b1.shape[-2], b2.shape[-2]), max(b1.shape[-1], b2.shape[-1]), max(k1, k2),
                      precision=P._precision_of(b1), device=dev, diag=True)
    out = torch.empty((m, n), dtype=dtype, device=dev)
    K1 = torch.empty((k1, k1), dtype=torch.float64, device=dev)
    K2 = torch.empty((k2, k2), dtype=torch.float64, device=dev)
    diag = torch.zeros(P.diag_size(), dtype=torch.uint8, device=dev)
    return dict(b1=b1, b2=b2, m=m, n=n, lam=lam, ref=ref, out=out, K1=K1, K2=K2, diag=diag)


def test_noalloc_equals_deblur_on_two_calls():
    import paper_1203_4874_amd as P
    P.lib()
    big = synth.config2(noise=1e-3)                    # 480 x 640, 9 x 9 / 11 x 11, FP32 frames
    small = synth.config1()                            # 64 x 64, 5 x 5, FP64 frames
    cases = [_case(P, big, torch.float32, big["lam"]), _case(P, small, torch.float64, 0.0)]
    refs = []
    for c in cases:
        refs.append(c["ref"].deblur(c["b1"], c["b2"], c["m"], c["n"], c["lam"]))
        c["out"].fill_(float("nan"))
        c["K1"].fill_(float("nan"))
        c["K2"].fill_(float("nan"))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    # two calls in a row on the shared scratch, the second on the smaller frame
    for c in cases:
        P.deblur_noalloc(c["b1"], c["b2"], c["out"], c["K1"], c["K2"], lam=c["lam"], diag=c["diag"])
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    for c, (L0, R1, R2) in zip(cases, refs):
        print(f"noalloc {tuple(c['b1'].shape)} {c['b1'].dtype}: latent max |diff| "
              f"{float((c['out'] - L0).abs().max()):.3e}", flush=True)
        assert torch.equal(c["out"], L0)
        assert torch.equal(c["K1"], R1)
        assert torch.equal(c["K2"], R2)
        d_ref = P.decode_diag(c["ref"].diag.cpu().numpy())
        d_na = P.decode_diag(c["diag"].cpu().numpy())
        assert d_na["flags"] == d_ref["flags"]
        assert np.array_equal(d_na["khat"], d_ref["khat"])
    assert free1 == free0


def test_noalloc_rejects_oversized_frame_and_flags():
    import paper_1203_4874_amd as P
    L = P.lib()
    dev = _dev()
    # a 1080p RGB pair needs ~132 MiB of workspace, more than the 48 MiB scratch
    b1 = torch.zeros((3, 1094, 1934), dtype=torch.float32, device=dev)
    b2 = torch.zeros((3, 1096, 1936), dtype=torch.float32, device=dev)
    out = torch.empty((3, 1080, 1920), dtype=torch.float32, device=dev)
    with pytest.raises(P.CbpError) as e:
        P.deblur_noalloc(b1, b2, out, None, None)
    assert e.value.status == 5
    i1, i2, io = P._image(b1[0]), P._image(b2[0]), P._image(out[0])
    o = P.CbpOptions()
    o.precision = P.Precision.MIXED
    o.flags = P.Flags.GRAPH
    assert L.cbp_deblur_noalloc(ctypes.byref(i1), ctypes.byref(i2), ctypes.byref(io), None, None,
                                ctypes.byref(o)) == 6
