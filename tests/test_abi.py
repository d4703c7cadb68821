"""The C ABI on the host: the shared library loads, exports every entry point
declared in include/exageo.h, and its host-only logic (workspace sizing,
argument checks before any launch) behaves as documented.  No GPU needed."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exageo.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(exageo_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1908_06936_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libexageo.so not built")
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("exageo_matern_cov", "exageo_loglik", "exageo_loglik_grad", "exageo_mle"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, f"not exported: {missing}"


def test_binding_list_matches_header():
    from paper_1908_06936_amd import _lib

    assert sorted(_lib.EXPORTS) == declared_functions()


def test_workspace_bytes_host_only(lib):
    from paper_1908_06936_amd._lib import FP64, MIXED

    ws = lib.exageo_workspace_bytes
    assert ws(0, 768, FP64, 0) == 0  # invalid n
    assert ws(1000, 100, FP64, 0) == 0  # ts not a multiple of 128
    a = ws(40000, 768, FP64, 0)
    g = ws(40000, 768, FP64, 1)
    m = ws(40000, 768, MIXED, 0)
    assert a > 0 and g > a
    nt = (40000 + 767) // 768
    tiles = nt * (nt + 1) // 2 * 768 * 768 * 8
    assert tiles <= a < 1.3 * tiles  # the FP64 tiles dominate
    # 4-byte off-diagonal slots plus an FP64 pool for up to half of the
    # off-diagonal tiles, plus the panel copies: about the FP64 size
    assert 0.9 * a < m < 1.25 * a


def test_workspace_of_the_fisher_information(lib):
    # the derivative matrices take one buffer of lower tiles each (npad^2 / 2
    # doubles), two without a nugget and three with one, plus a strip of about
    # npad^2 / 8 doubles; kriging borrows the gradient plan's staging buffer
    from paper_1908_06936_amd._lib import FP64, MIXED

    ws = lib.exageo_workspace_bytes
    for n, ts in ((40000, 768), (90000, 768), (10000, 512)):
        nt = (n + ts - 1) // ts
        low = nt * (nt + 1) // 2 * ts * ts * 8
        npad2 = (nt * ts) ** 2 * 8
        g = ws(n, ts, FP64, 1)
        f2, f3 = ws(n, ts, FP64, 2), ws(n, ts, FP64, 3)
        w = nt if nt < 8 else (nt + 7) // 8  # strip: w tile rows of the derivative matrix
        strip = w * nt * ts * ts * 8
        parts = -(-(nt * (nt + 1) // 2 * (ts // 128) ** 2 * 9 * 8) // 256) * 256
        assert f2 - g == 2 * low + strip + parts + 256
        assert strip <= npad2 / 6
        assert f3 - f2 == low
    assert ws(1000, 256, FP64, 4) == 0 and ws(1000, 256, 7, 1) == 0


def test_entry_points_reject_bad_arguments_before_any_launch(lib):
    from paper_1908_06936_amd._lib import EINVAL

    out = ctypes.c_void_p()
    assert lib.exageo_create(ctypes.byref(out), 0, 100, None) == EINVAL  # ts not a multiple of 128
    assert lib.exageo_create(None, 0, 768, None) == EINVAL
    ll = ctypes.c_double()
    theta = (ctypes.c_double * 3)(1.0, 0.1, 0.5)
    assert lib.exageo_loglik(None, 10, None, None, None, theta, 0, ctypes.byref(ll), None) == EINVAL
    assert lib.exageo_set_mixed_policy(None, 3.0) == EINVAL
    assert lib.exageo_set_mixed_fp64_band(None, 1.0) == EINVAL
    assert lib.exageo_set_mixed_bf16_block(None, 256) == EINVAL
    assert lib.exageo_last_error(None) == b"null context"


def test_no_silent_cpu_path_without_a_gpu():
    # the product path needs the GPU: without one it raises instead of falling back
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import paper_1908_06936_amd as exa

    with pytest.raises(RuntimeError):
        exa.Context(ts=768)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def test_tile_index_reciprocal_is_exact_in_range():
    # The mixed FP64 LAUUM takes the tile index k / ts as the high half of
    # k m, m = floor(2^32 / ts) + 1, and the entry points keep k ts < 2^32.
    # a m / 2^32 never falls below a / ts and is nondecreasing in a, so the
    # quotient is exact on a whole block [q ts, q ts + ts - 1] once it is exact
    # at the block's last element: check that element for every q in range,
    # for every tile size the library accepts.
    import numpy as np

    src = open(os.path.join(ROOT, "paper_1908_06936_amd", "csrc", "common.h")).read()
    assert "m((uint32_t)(0x100000000ull / (uint64_t)d + 1))" in src and "__umulhi(a, m)" in src
    for d in range(128, 4097, 128):
        m = (1 << 32) // d + 1
        assert m < (1 << 32)
        amax = ((1 << 32) - 1) // d  # largest a with a d < 2^32
        q = np.arange(0, amax // d + 1, dtype=np.uint64)
        a = np.minimum(q * np.uint64(d) + np.uint64(d - 1), np.uint64(amax))
        got = (a * np.uint64(m)) >> np.uint64(32)
        assert np.array_equal(got, a // np.uint64(d)), d


def test_profile_summaries_state_runnable_commands():
    # every committed rocprofv3 summary gives the command that made it; the
    # profiled program is the committed bench.py and every option it passes
    # is one bench.py still accepts
    prof = os.path.join(ROOT, "profiles")
    bench_src = open(os.path.join(ROOT, "bench.py")).read()
    accepted = set(re.findall(r'add_argument\("(--[a-z0-9-]+)"', bench_src))
    files = sorted(f for f in os.listdir(prof) if f.endswith((".md", ".txt")))
    assert files
    for f in files:
        cmds = re.findall(r"rocprofv3 [^\n`]*", open(os.path.join(prof, f)).read())
        assert cmds, f
        for c in cmds:
            prog = c.split(" -- ", 1)[1].split()
            assert prog[0] == "python3" and prog[1].endswith("/bench.py"), (f, c)
            for opt in (a for a in prog[2:] if a.startswith("--")):
                assert opt in accepted, (f, opt)
