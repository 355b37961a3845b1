"""The AMG hierarchy build of libsstep (its host side, csrc/amg.hip) on the
CPU: compiled with AddressSanitizer and UndefinedBehaviorSanitizer on the
host code (no GPU call is made) and compared with the oracle's hierarchy.

Bars: the level sizes and every row's aggregate equal the oracle's (integer
work on the same values: the fine level exactly, the coarse levels through
Galerkin sums that differ by rounding, which the tie rule of the second
aggregation pass keeps from deciding); the prolongators, restrictions and
coarse operators to 1e-12 of their largest entry; the coarse inverse to
1e-10.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg
from paper_2501_03743_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("needs hipcc")
    exe = str(tmp_path_factory.mktemp("amg") / "amg_host_check")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address,undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2501_03743_amd", "csrc"),
           "-o", exe, os.path.join(ROOT, "tests", "amg_host_check.hip")]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def _read_csr(buf, off):
    n, m, z = np.frombuffer(buf, np.int64, 3, off)
    off += 24
    rp = np.frombuffer(buf, np.int64, n + 1, off)
    off += 8 * (n + 1)
    ci = np.frombuffer(buf, np.int32, z, off)
    off += 4 * z
    v = np.frombuffer(buf, np.float64, z, off)
    off += 8 * z
    return sp.csr_matrix((v, ci, rp), shape=(n, m)), off


def _rel(a, b):
    return abs(a - b).max() / max(abs(b).max(), 1e-300)


@pytest.mark.parametrize("kind,shape,max_coarse,max_levels",
                         [("2d5", (64, 64), 64, 10), ("3d7", (24, 20, 18), 64, 10),
                          ("3d7", (33, 31, 29), 64, 10), ("2d5", (37, 29), 64, 10),
                          ("3d7", (14, 13, 12), 64, 2)])
def test_host_hierarchy_equals_oracle(driver, tmp_path, kind, shape, max_coarse, max_levels):
    rp, ci, v = wl.stencil_csr(kind, shape)
    n = rp.size - 1
    src, out = str(tmp_path / "A.bin"), str(tmp_path / "H.bin")
    with open(src, "wb") as f:
        f.write(struct.pack("qq", n, ci.size))
        f.write(rp.astype(np.int32).tobytes() + ci.astype(np.int32).tobytes() +
                v.astype(np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([driver, src, out, str(max_coarse), str(max_levels)], env=env,
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    S = sp.csr_matrix((v, ci, rp), shape=(n, n))
    H = amg.Hierarchy(S, max_coarse=max_coarse, max_levels=max_levels)
    buf = open(out, "rb").read()
    levels = int(np.frombuffer(buf, np.int64, 1, 0)[0])
    off = 8
    assert levels == len(H.A), (levels, H.sizes)
    for l in range(levels - 1):
        agg = np.frombuffer(buf, np.int64, H.A[l].shape[0], off)
        off += 8 * agg.size
        assert np.array_equal(agg, H.aggs[l]), l
        P, off = _read_csr(buf, off)
        R, off = _read_csr(buf, off)
        Ac, off = _read_csr(buf, off)
        assert P.shape == H.P[l].shape and Ac.shape == H.A[l + 1].shape
        assert _rel(P, H.P[l]) <= 1e-12 and _rel(R, H.R[l]) <= 1e-12, l
        assert _rel(Ac, H.A[l + 1]) <= 1e-12, l
    nc = H.A[-1].shape[0]
    inv = np.frombuffer(buf, np.float64, nc * nc, off).reshape(nc, nc)
    assert np.max(np.abs(inv - H.coarse)) <= 1e-10 * np.max(np.abs(H.coarse))
