"""The C-ABI library loads and exports every symbol include/*.h declares, and
the ctypes struct layouts match the C header (no GPU needed)."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

from paper_1708_07954_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(hdr).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(dba_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("dba_create", "dba_set_problem", "dba_iterate", "dba_residuals", "dba_get_params"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(binding.EXPORTS) <= set(_declared_functions())


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dba.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(dba_options),'
                   ' sizeof(dba_problem_desc), sizeof(dba_residual_report),'
                   ' offsetof(dba_options, persistent), offsetof(dba_residual_report, iteration),'
                   ' offsetof(dba_options, block_points), offsetof(dba_options, camera_model),'
                   ' offsetof(dba_options, local_solver), offsetof(dba_options, block_cameras),'
                   ' offsetof(dba_options, segment_schedule));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(binding.dba_options), ctypes.sizeof(binding.dba_problem_desc),
            ctypes.sizeof(binding.dba_residual_report), binding.dba_options.persistent.offset,
            binding.dba_residual_report.iteration.offset, binding.dba_options.block_points.offset,
            binding.dba_options.camera_model.offset, binding.dba_options.local_solver.offset,
            binding.dba_options.block_cameras.offset, binding.dba_options.segment_schedule.offset]
    assert got == want


def test_default_options_need_no_gpu():
    o = binding.make_options()
    assert o.lm_steps == 5 and o.lm_lambda0 == 1e-3 and o.rb_mu == 10.0 and o.rb_tau == 2.0
