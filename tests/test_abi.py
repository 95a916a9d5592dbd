"""CPU checks of the C ABI: the library loads, exports every entry point that
include/scw.h declares, and the ctypes structures have the C layout."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2404_07293_amd import _native as N

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "scw.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(scw_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = N.load()
    declared = _declared_functions()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(N.SIGNATURES), "binding and header disagree"


def _c_layout():
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "scw.h"
#define F(T, f) printf("%s %s %zu\n", #T, #f, offsetof(T, f));
int main(void) {
  F(scw_problem, nx) F(scw_problem, px) F(scw_problem, n) F(scw_problem, lambda)
  F(scw_problem, n_top) F(scw_problem, n_bot_im) F(scw_problem, U) F(scw_problem, inc_ex)
  F(scw_problem, inc_ey) F(scw_problem, inc_nx) F(scw_problem, pw_u) F(scw_problem, pw_ex)
  F(scw_problem, pw_ey) F(scw_problem, route) F(scw_problem, eig)
  F(scw_grid, fx) F(scw_grid, z_begin) F(scw_grid, z_end)
  F(scw_solution_info, M) F(scw_solution_info, min_abs_sz)
  F(scw_solution_info, connection_rcond) F(scw_solution_info, assembly_device_ms)
  F(scw_solution_info, boundary_seconds)
  F(scw_synth_config, modal_rows) F(scw_synth_config, transform)
  F(scw_synth_config, fft_radix) F(scw_synth_config, tiles)
  F(scw_tune_report, n_candidates) F(scw_tune_report, default_ms) F(scw_tune_report, best_ms)
  F(scw_tune_report, config) F(scw_tune_report, batch_radix)
  F(scw_tune_report, batch_blocks_per_cu) F(scw_tune_report, batch_chunk)
  F(scw_slice, axis) F(scw_slice, position) F(scw_slice, n) F(scw_slice, fz)
  F(scw_slice, z_begin) F(scw_slice, z_end)
  F(scw_plane_wave, u) F(scw_plane_wave, v) F(scw_plane_wave, ex) F(scw_plane_wave, ey)
  printf("size scw_plane_wave %zu\n", sizeof(scw_plane_wave));
  printf("size scw_slice %zu\n", sizeof(scw_slice));
  printf("enum route stable %d\nenum route connection %d\n", SCW_ROUTE_STABLE, SCW_ROUTE_CONNECTION);
  printf("enum route stable_device %d\nenum route connection_device %d\n",
         SCW_ROUTE_STABLE_DEVICE, SCW_ROUTE_CONNECTION_DEVICE);
  printf("size scw_problem %zu\nsize scw_grid %zu\nsize scw_solution_info %zu\n",
         sizeof(scw_problem), sizeof(scw_grid), sizeof(scw_solution_info));
  printf("size scw_synth_config %zu\nsize scw_tune_report %zu\n",
         sizeof(scw_synth_config), sizeof(scw_tune_report));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    return out.split("\n")


def test_ctypes_structures_match_c_layout():
    rename = {"lambda": "lam"}
    types = {"scw_problem": N.ScwProblem, "scw_grid": N.ScwGrid,
             "scw_solution_info": N.ScwSolutionInfo, "scw_synth_config": N.ScwSynthConfig,
             "scw_tune_report": N.ScwTuneReport, "scw_slice": N.ScwSlice,
             "scw_plane_wave": N.ScwPlaneWave}
    for line in _c_layout():
        if not line:
            continue
        if line.startswith("enum route "):
            _, _, name, value = line.split()
            assert N.ROUTE[name] == int(value), line
            continue
        a, b, c = line.split()
        if a == "size":
            assert ctypes.sizeof(types[b]) == int(c), line
        else:
            field = getattr(types[a], rename.get(b, b))
            assert field.offset == int(c), line


def test_create_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    lib = N.load()
    h = ctypes.c_void_p()
    rc = lib.scw_create(ctypes.byref(h), 0, 0)
    assert rc == -3
    assert b"hipGetDeviceCount" in lib.scw_last_error()
    assert lib.scw_create(None, 0, 0) == -1


def test_null_arguments_rejected_without_touching_the_gpu():
    lib = N.load()
    assert lib.scw_solve(None, None, None) == -1
    assert lib.scw_synthesize(None, None, None, 1, None, None) == -1
    assert lib.scw_solution_info_get(None, None) == -1
    assert lib.scw_synthesis_bytes(None, None, 1) == 0.0
    assert lib.scw_synthesis_configure(None, None) == -1
    assert lib.scw_tune_synthesis(None, None, None, 1, None, None, 5, None) == -1
    assert lib.scw_batch_tune(None, None, None, 3, None) == -1
    assert lib.scw_batch_configure(None, 16, 4, 1) == -1
    assert lib.scw_synthesize_slice(None, None, None, 1, None, None) == -1
    assert lib.scw_synthesize_image(None, None, None, 1, 0.5, None, None, None) == -1
    assert lib.scw_synthesize_filtered(None, None, None, 1, None, None, None, None) == -1
    assert lib.scw_solve_illuminations(None, None, 0, None, None) == -1
    assert lib.scw_synthesize_illuminations(None, None, None, 1, None, None) == -1
    assert lib.scw_sur_set_compute(None, 1) == -1
