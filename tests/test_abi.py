"""Host-side checks of the C ABI: the library loads and exports every function
include/ftgcr.h declares, the header and the ctypes binding agree on struct
layouts, and the input generators produce what the configurations state.
No GPU calls."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2103_07210_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ftgcr.h")
LIB = os.path.join(ROOT, "paper_2103_07210_amd", "libftgcr.so")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ftgcr_[a-z_A-Z]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2103_07210_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_exports_every_declared_function(lib):
    names = _declared_functions()
    assert len(names) >= 13
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2103_07210_amd import ftgcr
    assert sorted(ftgcr.EXPORTED) == names


def test_default_options_and_create_errors_without_gpu(lib):
    from paper_2103_07210_amd import ftgcr
    lib.ftgcr_default_options.argtypes = [ctypes.POINTER(ftgcr.Options)]
    o = ftgcr.Options()
    lib.ftgcr_default_options(ctypes.byref(o))
    assert o.ft == 1 and o.poll_steps == 16 and o.max_steps == 100000
    assert o.inner_tol == 3e-5 and o.hist_cap == 65536
    assert o.batch_levels_per_block == 0 and o.levels_per_block == 0
    assert o.order_stencil == ftgcr.ORDER_AUTO and o.order_dir == ftgcr.ORDER_AUTO
    # the batch autotuner validates before any device call
    lib.ftgcr_autotune_batch.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    assert lib.ftgcr_autotune_batch(None, 0, None, None, 3, 8, None) == ftgcr.E_INVALID
    lib.ftgcr_get_tiling.argtypes = [ctypes.c_void_p] * 5
    assert lib.ftgcr_get_tiling(None, None, None, None, None) == ftgcr.E_INVALID
    # argument validation happens before any device call
    lib.ftgcr_create.argtypes = [ctypes.POINTER(ftgcr.Grid), ctypes.POINTER(ftgcr.Coeffs), ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.ftgcr_last_error.argtypes = [ctypes.c_void_p]
    lib.ftgcr_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    c = ftgcr.Coeffs(1.57, 0.52, 0.5, 0.35, 0.3, 1e-3)
    assert lib.ftgcr_create(ctypes.byref(ftgcr.Grid(2, 4, 4, 1.0)), ctypes.byref(c), 1, 0, 3, None,
                            ctypes.byref(h)) == ftgcr.E_INVALID
    assert b"nlon" in lib.ftgcr_last_error(None)
    assert lib.ftgcr_create(ctypes.byref(ftgcr.Grid(8, 4, 97, 1.0)), ctypes.byref(c), 1, 0, 3, None,
                            ctypes.byref(h)) == ftgcr.E_UNSUPPORTED
    assert lib.ftgcr_create(ctypes.byref(ftgcr.Grid(8, 4, 4, 1.0)), ctypes.byref(c), 1, 0, 17, None,
                            ctypes.byref(h)) == ftgcr.E_INVALID
    assert lib.ftgcr_create(ctypes.byref(ftgcr.Grid(8, 4, 4, 1.0)), ctypes.byref(c), 2, 0, 3, None,
                            ctypes.byref(h)) == ftgcr.E_INVALID
    assert b"precond" in lib.ftgcr_last_error(None)
    assert not h.value


def test_struct_layouts_match_header(tmp_path):
    """Compile a probe against include/ftgcr.h and compare sizes and field
    offsets with the ctypes mirrors of the binding."""
    import subprocess
    from paper_2103_07210_amd import ftgcr
    mirrors = {"ftgcr_grid": ftgcr.Grid, "ftgcr_coeffs": ftgcr.Coeffs, "ftgcr_options": ftgcr.Options,
               "ftgcr_fault_event": ftgcr.FaultEvent, "ftgcr_fault_plan": ftgcr.FaultPlan,
               "ftgcr_detect_rec": ftgcr.DetectRec, "ftgcr_stats": ftgcr.Stats,
               "ftgcr_kernel_time": ftgcr.KernelTime}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            if fname.endswith('_') and fname.startswith('pad'):
                continue
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            if fname.startswith("pad"):
                continue
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_generators_follow_the_configurations():
    r = I.rhs(I.C1, 1)
    assert r.shape == (8, 32, 64) and r.min() >= -1 and r.max() <= 1
    np.testing.assert_array_equal(r, I.rhs(I.C1, 1))
    plans = I.campaign_plans(I.Problem(32, 16, 8), count=60, seed0=1000)
    n = 32 * 16 * 8
    sizes = {p[0].count for p in plans}
    assert sizes == {1, int(np.ceil(0.01 * n)), int(np.ceil(0.1 * n))}
    for p in plans:
        ev = p[0]
        assert 1 <= ev.step <= 20 and 0 <= ev.bit <= 63 and 0 <= ev.vec <= 3
        idx = ev.indices()
        assert idx.min() >= 0 and idx.max() < n and len(set(idx.tolist())) == idx.size
    ens = I.ensemble(64, seed=4)
    assert len(ens) == 64 and sum(1 for m in ens if m.plan) == 6
    assert {(m.problem.nx, m.problem.ny, m.problem.nz) for m in ens} <= set(I.C4_SIZES)
    assert all(0.2 <= m.problem.hill_amp <= 1.0 for m in ens)
    blk = I.block_plan(I.C5)[0]
    assert blk.count == int(np.ceil(0.1 * I.C5.n)) and blk.start + blk.count <= I.C5.n


def _header_enum(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"typedef enum \{([^}]*)\}\s*" + name + ";", text)
    assert m, name
    return {k.strip(): int(v) for k, v in (item.split("=") for item in m.group(1).split(","))}


def test_fault_targets_agree_with_header_and_oracle():
    """The vector codes of fault events: header enum, the generators' codes
    and the oracle header's codes are the same numbers (plans go to both)."""
    hdr = _header_enum("ftgcr_vec")
    assert hdr == {"FTGCR_V_X": 0, "FTGCR_V_R": 1, "FTGCR_V_P": 2, "FTGCR_V_AP": 3, "FTGCR_V_E": 4}
    assert I.VEC_NAMES == {"x": 0, "r": 1, "p": 2, "ap": 3, "e": 4}
    otext = open(os.path.join(ROOT, "oracle", "ftgcr_oracle.h")).read()
    m = re.search(r"enum \{ (ORC_V_X = 0[^}]*)\}", otext)
    codes = {k.strip(): int(v) for k, v in (item.split("=") for item in m.group(1).split(","))}
    assert list(codes.values()) == list(hdr.values())
