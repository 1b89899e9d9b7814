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
    # sip_request: id, sip_problem, b, x, x0, rtol, max_iter, retain, stream
    assert ctypes.sizeof(sip.Request) == 8 + ctypes.sizeof(sip.Problem) + 24 + 8 + 8 + 8
    assert sip.Request.stream.offset == ctypes.sizeof(sip.Request) - 8


def test_host_side_argument_checks(libpath):
    """Bad arguments come back as SIP_EINVAL from host-side checks, before
    any device call (the coefficient pointers below are never dereferenced)."""
    from paper_1303_4538_amd import sip
    L = sip.lib()

    def problem(ni, nj, nk, alpha=0.92, precision=1, storage=0):
        p = sip.Problem()
        p.ni, p.nj, p.nk = ni, nj, nk
        for d in range(7):
            p.a[d] = 0x100000 + 64 * d
        p.alpha, p.precision, p.storage = alpha, precision, storage
        return p

    h = ctypes.c_void_p()
    cases = [problem(0, 4, 4), problem(4, 4, 4, alpha=1.5), problem(4, 4, 4, alpha=float("nan")),
             problem(4, 4, 4, alpha=-0.1), problem(4, 4, 4, precision=3),
             problem(4, 4, 4, storage=2), problem(4, 4, 4, precision=2, storage=1),
             problem(1024, 1024, 300)]           # more than 2^28 cells in the tile-sheared layout
    for p in cases:
        assert L.sip_factor(ctypes.byref(p), None, ctypes.byref(h)) == sip.SIP_EINVAL
    p = problem(4, 4, 4)
    p.a[3] = None
    assert L.sip_factor(ctypes.byref(p), None, ctypes.byref(h)) == sip.SIP_EINVAL
    # multi-block domains: cut planes and precision
    for cuts, prec in ((([0, 4], [0, 4], [0, 3]), 1), (([0, 2, 2, 4], [0, 4], [0, 4]), 1),
                       (([1, 4], [0, 4], [0, 4]), 1), (([0, 4], [0, 4], [0, 4]), 2)):
        bp = sip.BlockProblem()
        bp.domain = problem(4, 4, 4, precision=prec)
        arrs = [(ctypes.c_int32 * len(c))(*c) for c in cuts]
        for d in range(3):
            bp.nb[d] = len(cuts[d]) - 1
            bp.cuts[d] = ctypes.cast(arrs[d], ctypes.POINTER(ctypes.c_int32))
        assert L.sip_blocks_factor(ctypes.byref(bp), None, ctypes.byref(h)) == sip.SIP_EINVAL
    # NULL handles and counts
    assert L.sip_iterate(None, None, None, 1, None, None) == sip.SIP_EINVAL
    assert L.sip_solve_multi(None, 2, None, None, 1e-8, 10, None, None) == sip.SIP_EINVAL
    assert L.sip_blocks_solve(None, None, None, 1e-8, 10, None, None) == sip.SIP_EINVAL
    cfg = sip.ServerConfig()
    cfg.max_slots, cfg.epoch_iters, cfg.max_queue = 0, 4, 16
    assert L.sip_server_create(ctypes.byref(cfg), ctypes.byref(h)) == sip.SIP_EINVAL
    assert L.sip_last_error() == b"bad server configuration"


def test_tuning_table_round_trip(libpath, tmp_path):
    """sip_tune_load / sip_tune_save are host only: a table written by hand
    loads, saves back entry for entry, and a malformed file merges nothing."""
    import json
    from paper_1303_4538_amd import sip
    entries = [dict(ni=256, nj=256, nk=256, precision=1, symmetric=0, phases=2, poll=2),
               dict(ni=17, nj=9, nk=5, precision=2, symmetric=0, phases=3, poll=1),
               dict(ni=512, nj=512, nk=256, precision=0, symmetric=1, phases=1, poll=2),
               dict(ni=40, nj=40, nk=40, precision=1, symmetric=0, phases=2, poll=3)]
    old_format = dict(ni=24, nj=24, nk=24, precision=1, symmetric=0, phases=3)   # no poll: the default 2
    src = tmp_path / "tune.jsonl"
    src.write_text("\n".join(json.dumps(e) for e in entries + [old_format]) + "\n\n")
    sip.sip_tune_load(src)
    out = tmp_path / "saved.jsonl"
    sip.sip_tune_save(out)
    saved = [json.loads(line) for line in out.read_text().splitlines() if line.strip()]
    for e in entries + [dict(old_format, poll=2)]:
        assert e in saved
    # a later entry for the same key wins
    src.write_text(json.dumps(dict(entries[0], phases=3)) + "\n")
    sip.sip_tune_load(src)
    sip.sip_tune_save(out)
    saved = [json.loads(line) for line in out.read_text().splitlines()]
    assert dict(entries[0], phases=3) in saved and entries[0] not in saved
    # bad lines: nothing of the file is merged
    for bad in ('{"ni": 8, "nj": 8, "nk": 8, "precision": 1, "symmetric": 0, "phases": 4}',
                '{"ni": 0, "nj": 8, "nk": 8, "precision": 1, "symmetric": 0, "phases": 2}',
                '{"ni": 8, "nj": 8, "nk": 8, "precision": 5, "symmetric": 0, "phases": 2}',
                '{"ni": 8, "nj": 8, "nk": 8, "precision": 1, "phases": 2}',
                '{"ni": 8, "nj": 8, "nk": 8, "precision": 1, "symmetric": 0, "phases": 2, "poll": 4}',
                '{"ni": 8, "nj": 8, "nk": 8, "precision": 1, "symmetric": 0, "phases": 2, "poll": 0}',
                'not json'):
        f = tmp_path / "bad.jsonl"
        f.write_text(json.dumps(dict(ni=9, nj=9, nk=9, precision=1, symmetric=0, phases=2)) + "\n" + bad + "\n")
        with pytest.raises(sip.SipError) as e:
            sip.sip_tune_load(f)
        assert e.value.status == sip.SIP_EINVAL
    sip.sip_tune_save(out)
    assert all(e["ni"] != 9 for e in map(json.loads, out.read_text().splitlines()))
    with pytest.raises(sip.SipError):
        sip.sip_tune_load(tmp_path / "missing.jsonl")


def test_server_stats_length_matches_header():
    import re
    from paper_1303_4538_amd import sip
    hdr = open(os.path.join(ROOT, "include", "sip.h")).read()
    n = int(re.search(r"#define SIP_SERVER_NSTATS (\d+)", hdr).group(1))
    src = open(sip.__file__).read()
    assert f"(ctypes.c_uint64 * {n})()" in src
