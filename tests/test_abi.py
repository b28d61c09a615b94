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
