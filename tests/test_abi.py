"""CPU checks of the C ABI: the library loads and exports every symbol that
include/sip.h declares; the header and the binding agree.  No compute calls."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sip.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sip_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1303_4538_amd import build, sip
    if not os.path.exists(sip.LIB_PATH):
        build.build()
    return sip.LIB_PATH


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("sip_factor", "sip_iterate", "sip_solve", "sip_batch_submit", "sip_batch_poll"):
        assert n in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sip_[a-z_0-9]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_lists_all(libpath):
    from paper_1303_4538_amd import sip
    L = sip.lib()
    assert L.sip_abi_version() == 1
    assert L.sip_status_str(sip.SIP_EBREAKDOWN) == b"SIP_EBREAKDOWN"
    assert sorted(sip.EXPORTS) == declared_functions()
    for n in declared_functions():
        assert hasattr(L, n)


def test_struct_layouts_match_header():
    from paper_1303_4538_amd import sip
    # sip_problem: 3 int32, pad, 7 pointers, double, int32 (+pad)
    assert ctypes.sizeof(sip.Problem) == 4 * 3 + 4 + 8 * 7 + 8 + 8
    assert ctypes.sizeof(sip.Info) == 24
    # sip_block_problem: sip_problem, 3 int32 (+pad), 3 pointers
    assert ctypes.sizeof(sip.BlockProblem) == ctypes.sizeof(sip.Problem) + 12 + 4 + 24
