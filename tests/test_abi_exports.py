"""The built library loads and exports every entry point include/qmc.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qmc.h")
LIB = os.path.join(ROOT, "paper_2002_07401_amd", "libqmc_jagp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qmc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("qmc_eval_batch", "qmc_propose_move", "qmc_accept_move", "qmc_forces"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.qmc_abi_version.restype = ctypes.c_int32
    hdr = open(HEADER).read()
    version = int(re.search(r"#define QMC_ABI_VERSION (\d+)", hdr).group(1))
    assert lib.qmc_abi_version() == version


def test_binding_names_match_header():
    from paper_2002_07401_amd import binding
    assert sorted(binding.FUNCTIONS) == declared_functions()
