"""The C-ABI library on the host, with no GPU call.

It loads, it exports every function include/lagrom.h declares (with C
linkage), the Python binding names exactly those functions, and the host-only
entry points (time-window logic, eq. sample_window and eq. window_sample)
agree with the oracle.
"""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from oracle.windows import window_columns, windows_by_samples

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lagrom.h")


def header_functions(path=HEADER):
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = "\n".join(l for l in src.splitlines() if not l.lstrip().startswith("#"))
    src = src.replace('extern "C" {', " ")
    # drop struct / enum bodies
    while True:
        s2 = re.sub(r"\{[^{}]*\}", " ", src)
        if s2 == src:
            break
        src = s2
    names = []
    for stmt in src.split(";"):
        stmt = " ".join(stmt.split())
        if not stmt or stmt.startswith("typedef") or stmt.startswith("enum"):
            continue
        m = re.match(r"^(?:[A-Za-z_]\w*[\s\*]+)+?\**([A-Za-z_]\w*)\s*\(", stmt)
        if m:
            names.append(m.group(1))
    return names


@pytest.fixture(scope="module")
def so_path():
    from paper_2104_11404_amd import lib

    if not os.path.exists(lib.LIB_PATH):
        from paper_2104_11404_amd import build

        build.build()
    return lib.LIB_PATH


def test_header_parse_finds_the_entry_points():
    names = header_functions()
    for n in ("fom_force", "rom_build_basis", "rom_sample_deim", "rom_step", "rom_create", "lh_problem_create",
              "lh_last_error"):
        assert n in names
    assert len(names) == len(set(names))


def test_library_exports_every_declared_function(so_path):
    out = subprocess.run(["nm", "-D", "--defined-only", so_path], capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if len(l.split()) >= 3 and l.split()[1] == "T"}
    missing = [n for n in header_functions() if n not in exported]
    assert not missing, missing
    so = C.CDLL(so_path)
    for n in header_functions():
        assert getattr(so, n, None) is not None, n


def test_binding_covers_the_header_exactly(so_path):
    from paper_2104_11404_amd import lib

    assert sorted(lib.exported_symbols()) == sorted(header_functions())
    assert lib.missing_symbols(so_path) == []


def test_last_error_is_a_string(so_path):
    from paper_2104_11404_amd import lib

    assert isinstance(lib.load(so_path).lh_last_error(), bytes)


def test_window_logic_matches_oracle(so_path):
    from paper_2104_11404_amd import pipeline

    ta = list(np.cumsum([0.0] + list(np.random.default_rng(0).uniform(0.5, 1.5, 37))))
    tb = list(np.cumsum([0.0] + list(np.random.default_rng(1).uniform(0.5, 1.5, 41))))
    tb = [x * ta[-1] / tb[-1] for x in tb]
    for ns in (2, 4, 6, 10, 22, 200):
        T = pipeline.windows_by_samples([ta, tb], ns)
        assert T == windows_by_samples([ta, tb], ns)

        class Tr:
            t = ta

        first, ncol = pipeline.window_columns(ta, T)
        cols = window_columns(Tr, T)
        assert len(cols) == len(T)
        for w, c in enumerate(cols):
            assert ncol[w] == len(c)
            idx = [2 * (i - 1) + 1 if k == "init" else i for k, i in c]
            assert idx == list(range(first[w], first[w] + ncol[w]))


def test_window_logic_rejects_bad_arguments(so_path):
    from paper_2104_11404_amd import lib, pipeline

    with pytest.raises(lib.LagromError):
        pipeline.windows_by_samples([[0.0, 1.0, 2.0]], 1)


def test_idw_weights_of_the_library_match_the_oracle():
    """lh_idw_weights (host only) against the oracle's eq. interpolate_os weights."""
    from oracle import rom as R
    from paper_2104_11404_amd import lib
    for params, mu in (([0.8, 1.0, 1.2], 0.9), ([0.8, 1.0, 1.2], 1.2), ([0.8, 1.0, 1.2], 1.37),
                       ([[0.0, 0.0], [2.0, 0.0], [0.5, 1.5]], [1.0, 3.0])):
        for r in (1.0, 2.0, 3.5):
            np.testing.assert_allclose(lib.idw_weights(params, mu, r), R.idw_weights(params, mu, r), rtol=1e-14)


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes mirror of a header struct has the C size and the C offset of each field (a host
    program built from include/lagrom.h with g++ prints them)."""
    import shutil
    import subprocess

    from paper_2104_11404_amd import lib

    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("needs g++ and the HIP headers")
    pairs = {"lh_problem_desc": lib.ProblemDesc, "lh_fom_run_desc": lib.FomRunDesc,
             "lh_fom_run_stats": lib.FomRunStats, "lh_window_desc": lib.WindowDesc,
             "lh_instance_desc": lib.InstanceDesc, "lh_mlp_desc": lib.MlpDesc, "lh_rom_state": lib.RomState}
    lines = ["#include <cstdio>", "#include <cstddef>", '#include "lagrom.h"', "int main() {"]
    for cname, cls in pairs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run([gxx, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", inc, str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            c, f, v = ln.split()
            got[(c, f)] = int(v)
    for cname, cls in pairs.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
