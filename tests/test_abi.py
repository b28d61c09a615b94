"""The C ABI library loads and exports every entry point include/mantra.h
declares (no GPU needed: nothing here calls into the device)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mantra.h")
LIB = os.path.join(ROOT, "paper_2304_08356_amd", "libmantra.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mantra_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for want in ("mantra_graph_create", "mantra_estimate", "mantra_submit", "mantra_poll",
                 "mantra_count_pairs", "mantra_run"):
        assert want in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2304_08356_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2304_08356_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared())


def test_exports_are_plain_c(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    syms = set(re.findall(r"\b(mantra_[a-z_]+)\b", out))
    assert set(declared()) <= syms


def test_no_device_gives_an_error_not_a_fallback(lib):
    """Without a GPU the graph constructor must fail loudly."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2304_08356_amd import Graph, MantraError
    import numpy as np
    with pytest.raises(MantraError):
        Graph(3, np.array([0, 1]), np.array([1, 2]), np.array([1, 2]))


def test_output_array_checks():
    """Caller-given output arrays must be writeable contiguous float64 of the
    exact size; None means a fresh zeroed array."""
    import numpy as np
    import paper_2304_08356_amd as pk
    a = np.zeros(5)
    assert pk.Graph._out_array(a, 5, "x") is a
    fresh = pk.Graph._out_array(None, 3, "x")
    assert fresh.dtype == np.float64 and fresh.shape == (3,) and not fresh.any()
    ro = np.zeros(5)
    ro.setflags(write=False)
    for bad in (np.zeros(4), np.zeros(5, dtype=np.float32), np.zeros((5, 1)), np.zeros(10)[::2], ro, [0.0] * 5):
        with pytest.raises(ValueError):
            pk.Graph._out_array(bad, 5, "x")
