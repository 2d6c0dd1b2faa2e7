"""CPU-side checks of the C-ABI library: it loads, exports every declared entry point, and its
host-only entry point (workspace sizing) validates descriptors.  No compute call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2210_15668_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\([^;]*\)\s*;", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def fx():
    from paper_2210_15668_amd import ferrox
    if not os.path.exists(ferrox.LIB_PATH):
        pytest.fail("libferrox.so is not built; run __graft_entry__.build()")
    return ferrox


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("init_stack", "tdgl_step", "poisson_solve", "run_steps", "stack_workspace_bytes",
              "get_field", "set_field", "destroy_stack", "last_error"):
        assert n in names, names


def test_library_exports_every_declared_symbol(fx):
    lib = fx.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    bound = {s[0] for s in fx.SIGNATURES}
    assert set(declared_functions()) == bound


def test_unet_sizes_are_host_only_and_validated(fx):
    lib = fx.lib()
    from oracle import unet_ref
    assert lib.unet_num_params() == unet_ref.num_params()
    assert lib.unet_workspace_bytes(128, 128, 60, 0) > 0
    assert lib.unet_workspace_bytes(128, 128, 60, 1) > lib.unet_workspace_bytes(128, 128, 60, 0)
    for bad in [(126, 128, 60), (128, 128, 62), (0, 4, 4), (4, 4, 2)]:
        assert lib.unet_workspace_bytes(*bad, 0) == 0
        assert fx.lib().last_error().decode() != ""


def test_binding_struct_matches_header_layout(fx, tmp_path):
    """Every binding struct has the C struct's size and every field its offset, as the C
    compiler lays out include/ferrox.h."""
    import subprocess
    pairs = [("fx_stack_desc", fx.StackDesc), ("fx_solve_info", fx.SolveInfo), ("fx_run_info", fx.RunInfo),
             ("fx_batch_info", fx.BatchInfo), ("fx_tune_info", fx.TuneInfo)]
    cname = {"lam": "lambda"}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ferrox.h"', 'int main(void) {']
    for ct, py in pairs:
        lines.append(f'printf("{ct} sizeof %zu\\n", sizeof({ct}));')
        for f, _ in py._fields_:
            c = cname.get(f, f)
            lines.append(f'printf("{ct} {f} %zu\\n", offsetof({ct}, {c}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for ct, py in pairs:
        assert got[(ct, "sizeof")] == ctypes.sizeof(py), ct
        for f, _ in py._fields_:
            assert got[(ct, f)] == getattr(py, f).offset, (ct, f)


def test_workspace_sizing_and_validation(fx):
    good = W.mfism_large()
    n = fx.workspace_bytes(good)
    # at least: the P ping-pong and phi backup (2 full grids) plus e, r on the finest level
    assert n >= 8 * (2 * good.ncell + 2 * good.n_active())
    mixed = good.copy(prec=W.PREC_MIXED)
    assert fx.workspace_bytes(mixed) < n
    bad = [
        good.copy(h=0.0),
        good.copy(gamma=-1.0),
        good.copy(pbc=7),
        good.copy(max_cycles=0),
        good.copy(T=0.0),
    ]
    mat = good.plane_mat.copy()
    mat[60] = W.METAL                     # metal inside the device
    bad.append(good.copy(plane_mat=mat))
    mat = good.plane_mat.copy()
    f0, f1 = good.fe_range()
    mat[f0:f1 - 2] = W.DE                 # ferroelectric of 2 planes
    bad.append(good.copy(plane_mat=mat))
    for b in bad:
        assert fx.workspace_bytes(b) == 0
        assert fx.lib().last_error().decode() != ""
