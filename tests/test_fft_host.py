"""The HIP path's Stockham butterflies (csrc/fft_core.h stockham_read, the
in-place pass order of the kernels), compiled for the host with g++ and run
through tests/host/fft_driver.cpp, against numpy.fft."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("fft") / "fft_driver")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1203_4874_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "fft_driver.cpp"), "-o", exe], check=True)
    return exe


def run(exe, x, direction, order=0, with9=0):
    inp = f"{len(x)} {direction} {order} {with9}\n" + "\n".join(f"{float(v.real)!r} {float(v.imag)!r}" for v in x)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([complex(*map(float, line.split())) for line in out.strip().split("\n")])


@pytest.mark.parametrize("with9", [0, 1])
@pytest.mark.parametrize("order", [0, 1, 2])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7, 8, 9, 12, 18, 27, 35, 49, 64, 81, 490, 672, 735, 1120, 1296,
                               1792, 1944, 2048])
def test_stockham_matches_numpy(driver, N, order, with9):
    """Every radix pass order the autotuner may pick, with and without the
    radix-9 passes of the row plans, computes the same DFT."""
    r = np.random.default_rng(N)
    x = r.standard_normal(N) + 1j * r.standard_normal(N)
    y = run(driver, x, -1, order, with9)
    assert np.abs(y - np.fft.fft(x)).max() <= 1e-14 * max(1.0, np.abs(np.fft.fft(x)).max())
    z = run(driver, x, +1, order, with9)
    assert np.abs(z - N * np.fft.ifft(x)).max() <= 1e-14 * max(1.0, np.abs(N * np.fft.ifft(x)).max())


@pytest.fixture(scope="module")
def sanitized_driver(tmp_path_factory):
    """The same driver built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code: the butterflies, the plans and the index splits)."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("fft_san") / "fft_driver_san")
    r = subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "paper_1203_4874_amd", "csrc"),
                        os.path.join(ROOT, "tests", "host", "fft_driver.cpp"), "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    return exe


@pytest.mark.parametrize("N", [1, 2, 9, 49, 81, 490, 1120, 1944, 2048])
def test_sanitized_butterflies(sanitized_driver, N):
    """Every pass order with and without radix 9 under ASan / UBSan: no
    out-of-bounds access, overflow or other undefined behaviour, and the
    same transform."""
    r = np.random.default_rng(N + 3)
    x = r.standard_normal(N) + 1j * r.standard_normal(N)
    for order in (0, 1, 2):
        for with9 in (0, 1):
            y = run(sanitized_driver, x, -1, order, with9)
            assert np.abs(y - np.fft.fft(x)).max() <= 1e-14 * max(1.0, np.abs(np.fft.fft(x)).max())


def test_non_smooth_size_has_no_plan(driver):
    out = subprocess.run([driver], input="11 -1 0 0\n" + "0 0\n" * 11, capture_output=True, text=True)
    assert "BADPLAN" in out.stdout


def test_radix_constants():
    """The odd-radix cosines / sines written in csrc/common.h."""
    import re
    import mpmath as mp
    mp.mp.dps = 30
    src = open(os.path.join(ROOT, "paper_1203_4874_amd", "csrc", "common.h")).read()
    vals = dict(re.findall(r"static constexpr double (\w+) = (-?[0-9.]+);", src))
    for R in (3, 5, 7, 9):
        for k in range(1, (R - 1) // 2 + 1):
            c = vals.get(f"c{R}_{k}")
            s = vals.get(f"s{R}_{k}")
            if c is not None:
                assert abs(mp.mpf(c) - mp.cos(2 * mp.pi * k / R)) < 1e-19
            if s is not None:
                assert abs(mp.mpf(s) - mp.sin(2 * mp.pi * k / R)) < 1e-19
    assert abs(mp.mpf(vals["r2_2"]) - mp.sqrt(0.5)) < 1e-19


def test_float_reciprocal_index_split_is_exact():
    """fft_core.h splits t = f nb + j and j = q Ns + k with
    floor((a + 1/2) * fl(1/b)) in FP32; exhaustive over every pass of every
    7-smooth size up to 2048, with up to 16 transforms per launch."""
    def smooth(n):
        for p in (2, 3, 5, 7):
            while n % p == 0:
                n //= p
        return n == 1
    f32 = np.float32
    for N in (n for n in range(2, 2049) if smooth(n)):
        for R in (2, 3, 4, 5, 7, 8, 9):
            if N % R:
                continue
            nb = N // R
            t = np.arange(nb * 16, dtype=np.int64)
            q = ((t.astype(f32) + f32(0.5)) * (f32(1.0) / f32(nb))).astype(np.int64)
            assert np.array_equal(q, t // nb), (N, R)
            for Ns in {d for d in range(1, N + 1) if N % (d * R) == 0}:
                j = np.arange(nb, dtype=np.int64)
                q2 = ((j.astype(f32) + f32(0.5)) * (f32(1.0) / f32(Ns))).astype(np.int64)
                assert np.array_equal(q2, j // Ns), (N, R, Ns)
