"""The ctypes mirrors of the ABI structs against the C header, and those of the oracle
against its header (CPU): a small C program built with the host compiler prints sizeof and
offsetof of every member the binding declares, so a member added, moved or resized on one
side only fails here instead of as wrong values."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2607_13507_amd import lpic as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [("lpic_grid", L.Grid), ("lpic_laser", L.Laser), ("lpic_fields", L.Fields),
         ("lpic_species", L.Species), ("lpic_tiling", L.Tiling), ("lpic_options", L.Options),
         ("lpic_stats", L.Stats), ("lpic_pml", L.Pml), ("lpic_plasma", L.Plasma),
         ("lpic_tune_space", L.TuneSpace), ("lpic_tune_report", L.TuneReport),
         ("lpic_qed_params", L.QedParams), ("lpic_qed_buffer", L.QedBuffer)]


def _layout(tmp_path, header, pairs, include_dirs):
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{header}"',
             'int main(void) {']
    expect = []
    for cname, cls in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(cls))
        for f in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {f[0]}));')
            expect.append(getattr(cls, f[0]).offset)
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = [a for d in include_dirs for a in ("-I", d)]
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", *inc, "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)], text=True).split()]
    assert got == expect


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_binding_structs_match_the_header(tmp_path):
    _layout(tmp_path, "lpic.h", PAIRS, [os.path.join(ROOT, "include"), "/opt/rocm/include"])


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_structs_match_its_header(tmp_path):
    import oracle as O
    pairs = [("orc_pml", O.Pml), ("orc_grid", O.Grid), ("orc_laser", O.Laser),
             ("orc_fields", O.Fields), ("orc_species", O.Species)]
    _layout(tmp_path, "oracle.h", pairs, [os.path.join(ROOT, "oracle")])
