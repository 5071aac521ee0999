"""The C-ABI library: it loads, exports every declared symbol, and its record
layouts match the header (checked by compiling the header with gcc)."""
import os
import subprocess

import numpy as np
import pytest

import paper_1304_3771_amd as dv
from paper_1304_3771_amd import devirt as binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1304_3771_amd import build
        build.build(force=True)
    return dv.lib()


def test_exports_every_declared_function(lib):
    names = dv.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_binding_covers_the_header():
    declared = set(dv.header_functions())
    bound = set(binding._SIGS) | {"devirt_last_error"}
    assert declared == bound


def test_record_layouts_match_header(tmp_path):
    prog = tmp_path / "sizes.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "devirt.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(devirt_request), sizeof(devirt_result),
         sizeof(devirt_fault), sizeof(devirt_xlat), sizeof(devirt_config), sizeof(devirt_stats),
         sizeof(devirt_server_cfg), sizeof(devirt_completion));
  printf("%zu %zu %zu %zu\n", offsetof(devirt_request, dir), offsetof(devirt_request, tag),
         offsetof(devirt_xlat, page_shift), offsetof(devirt_completion, t_done_ns));
  printf("%zu %zu %zu %zu\n", sizeof(devirt_map), offsetof(devirt_map, gpa), offsetof(devirt_map, flags),
         sizeof(devirt_server_stats));
  return 0;
}
''')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    a, b, c = subprocess.check_output([str(exe)]).decode().split("\n")[:3]
    sizes = list(map(int, a.split()))
    offs = list(map(int, b.split()))
    import ctypes
    assert list(map(int, c.split())) == [dv.MAP_DTYPE.itemsize, dv.MAP_DTYPE.fields["gpa"][1],
                                         dv.MAP_DTYPE.fields["flags"][1], ctypes.sizeof(binding.ServerStats)]
    import ctypes
    assert sizes == [dv.REQUEST_DTYPE.itemsize, dv.RESULT_DTYPE.itemsize, dv.FAULT_DTYPE.itemsize,
                     dv.XLAT_DTYPE.itemsize, ctypes.sizeof(binding.Config), ctypes.sizeof(binding.Stats),
                     ctypes.sizeof(binding.ServerCfg), ctypes.sizeof(binding.Completion)]
    assert offs == [dv.REQUEST_DTYPE.fields["dir"][1], dv.REQUEST_DTYPE.fields["tag"][1],
                    dv.XLAT_DTYPE.fields["page_shift"][1], binding.COMPLETION_DTYPE.fields["t_done_ns"][1]]


def test_generator_request_layout_is_the_abi_layout():
    from workload import REQ_DTYPE
    assert REQ_DTYPE == dv.REQUEST_DTYPE


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_1304_3771_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower(), f"{f} mentions the oracle"


def test_open_without_a_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(dv.DevirtError) as e:
        dv.Context(0)
    assert e.value.rc < 0


def test_library_is_built_for_gfx950(lib):
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", binding.LIB_PATH], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout
    assert np.uint8(0) == 0
