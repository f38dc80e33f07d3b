"""Host-side checks of the C-ABI library: it loads, exports what include/*.h declare,
and its host-only entry points (node counts, coordinates, argument errors) agree with
the oracle's grid.  No GPU compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.ark import tableau_float
from oracle.grid import Grid
from paper_2306_02526_amd import hps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^HPS_API[^;(]*?\b(\w+)\s*\(", text, flags=re.M))
    return sorted(names)


def test_header_declarations_match_binding():
    assert _declared() == sorted(hps.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = hps.lib()
    for name in _declared():
        assert hasattr(L, name), name
    # nothing else of the implementation leaks into the dynamic symbol table
    out = os.popen(f"nm -D --defined-only {hps.LIB_PATH}").read()
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert exported == set(_declared())


@pytest.mark.parametrize("n1,n2,p", [(1, 1, 3), (4, 4, 8), (8, 2, 11), (64, 64, 16), (2, 16, 24)])
def test_node_counts_match_oracle(n1, n2, p):
    g = hps.make_grid(0, n1 * 0.25, -1, -1 + n2 * 0.25, n1, n2, p)
    N, n_int, n_iface, n_bdry = hps.hps_num_nodes(g)
    og = Grid(0, n1 * 0.25, -1, -1 + n2 * 0.25, n1, n2, p)
    assert N == og.N and n_int == og.n_int
    assert n_bdry == 2 * (p - 2) * (n1 + n2) and n_iface == og.n_edge - n_bdry


@pytest.mark.parametrize("n1,n2,p", [(2, 2, 5), (4, 2, 8), (1, 4, 12)])
def test_node_coordinates_match_oracle(n1, n2, p):
    g = hps.make_grid(0.5, 0.5 + n1 * 0.3, 0, n2 * 0.3, n1, n2, p)
    x, y = hps.hps_nodes(g)
    ox, oy = Grid(0.5, 0.5 + n1 * 0.3, 0, n2 * 0.3, n1, n2, p).coordinates()
    assert np.abs(x - ox).max() < 1e-15 and np.abs(y - oy).max() < 1e-15


@pytest.mark.parametrize("bad", [dict(n1=3), dict(p=2), dict(p=25), dict(x1=0.0), dict(y1=5.0)])
def test_invalid_grids_are_rejected(bad):
    args = dict(x0=0.0, x1=1.0, y0=0.0, y1=1.0, n1=4, n2=4, p=8)
    args.update(bad)
    g = hps.make_grid(**args)
    with pytest.raises(hps.HPSError) as e:
        hps.hps_num_nodes(g)
    assert e.value.code == -1 and len(str(e.value)) > 12


def test_null_handles_are_rejected():
    L = hps.lib()
    assert L.hps_op_bytes(None, None) == -1
    assert L.ark_stage_solves_per_step(None) == -1
    L.hps_free(None)
    L.ark_free(None)
    out = ctypes.c_void_p()
    assert L.hps_build(None, None, 1.0, 0, None, ctypes.byref(out)) == -1
    assert L.ark_step_burgers(None, None, 0.0, None, None, None, None, None) == -1


@pytest.mark.parametrize("flags", [64, -1, 128 | hps.HPS_FP32_IR, hps.HPS_IR_STRICT, hps.HPS_TEST_FP32_SKEW,
                                   hps.HPS_IR_STRICT | hps.HPS_WIDE_TILES, hps.HPS_AUTOTUNE | hps.HPS_WIDE_TILES])
def test_unknown_build_flags_are_rejected(flags):
    """Only HPS_FP32_IR, HPS_WIDE_TILES, HPS_UNIFORM_COEFFS, HPS_AUTOTUNE (not with
    HPS_WIDE_TILES) and, with HPS_FP32_IR, HPS_IR_STRICT and HPS_TEST_FP32_SKEW may be set;
    the check comes before any device use."""
    g = hps.make_grid(0.0, 1.0, 0.0, 1.0, 2, 2, 6)
    fake = ctypes.c_void_p(4096)
    co = hps.HpsCoeffs(fake, fake, fake, fake, fake)
    out = ctypes.c_void_p()
    L = hps.lib()
    assert L.hps_build(ctypes.byref(g), ctypes.byref(co), 1e-2, flags, None, ctypes.byref(out)) == -1
    assert b"flags" in L.hps_last_error()


@pytest.mark.parametrize("name", ["ark436l2sa", "ark548l2sa"])
def test_product_tableau_equals_oracle_tableau(name):
    """The product's tableaux (written separately from the oracle's) equal the oracle's
    pinned ones in every double."""
    import oracle.ark as oark
    from paper_2306_02526_amd import tableau as ptab
    a = getattr(ptab, name)()
    b = tableau_float(getattr(oark, name)())
    for k in ("A", "Ahat", "b", "bhat", "c"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    assert a["s"] == b["s"] and a["gamma"] == b["gamma"]


def test_binding_structs_match_header_layout(tmp_path):
    """Sizes and field offsets of every struct in include/*.h, as gcc lays them out, equal
    the ctypes structures of the binding."""
    import subprocess
    structs = {"hps_grid": hps.HpsGrid, "hps_coeffs": hps.HpsCoeffs, "hps_info": hps.HpsInfo,
               "ark_tableau": hps.ArkTableau, "ark_g": hps.ArkG, "srv_config": hps.SrvConfig,
               "srv_job": hps.SrvJob, "srv_status": hps.SrvStatus, "srv_stats": hps.SrvStats}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "hps_batch.h"', '#include "hps_serve.h"',
             "int main(void) {"]
    expect = []
    for cname, py in structs.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(py))
        for fname, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {fname}));')
            expect.append(getattr(py, fname).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == expect


def test_batched_and_server_argument_errors():
    """Argument checks that return before any device call."""
    L = hps.lib()
    assert L.hps_solve_batched(None, 1, None, None, None, None, None, None) == -1
    assert L.hps_solve_batched(None, -1, None, None, None, None, None, None) == -1
    assert L.hps_solve_batched(None, 0, None, None, None, None, None, None) == 0
    assert L.ark_step_batched(None, 2, None, None, None, None, None, None, None) == -1
    assert L.srv_submit(None, None, None, None) == -1
    assert L.srv_poll(None, 0, None) == -1
