"""The ctypes mirrors of the C-ABI structs match include/wcsdp.h field by field.

A small C program built with the host compiler prints sizeof and the offset of
every field of each struct; the Python binding's ctypes.Structure classes must
agree, so that a field added on one side only fails here rather than
corrupting the options or statistics a caller reads.
"""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2407_14013_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "sdp_problem": L.SdpProblem,
    "sdp_options": L.SdpOptions,
    "sdp_inner_stats": L.SdpInnerStats,
    "sdp_step_stats": L.SdpStepStats,
    "sdp_adjoint_stats": L.SdpAdjointStats,
    "sdp_batch_tune": L.SdpBatchTune,
    "sdp_result": L.SdpResult,
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "wcsdp.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    layout = {}
    for line in out.splitlines():
        s, f, v = line.split()
        layout[(s, f)] = int(v)
    return layout


@pytest.mark.parametrize("cname", sorted(STRUCTS))
def test_struct_layout_matches_header(c_layout, cname):
    cls = STRUCTS[cname]
    assert C.sizeof(cls) == c_layout[(cname, "sizeof")]
    for field, _ in cls._fields_:
        assert getattr(cls, field).offset == c_layout[(cname, field)], field
