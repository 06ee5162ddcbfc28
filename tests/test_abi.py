"""The C ABI library loads on the host and exports what include/chhs.h declares.

No device work: only calls that validate arguments on the host before any
HIP call are made here.
"""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chhs.h")


def _ensure_built():
    from paper_1611_02967_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


@pytest.fixture(scope="module")
def binding():
    _ensure_built()
    from paper_1611_02967_amd import chhs
    return chhs


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chhs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for required in ("chhs_init", "chhs_step", "chhs_fas_vcycle", "chhs_energy_mass"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_ensure_built())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol(binding):
    assert set(declared_functions()) <= set(binding._SIGS)


def test_struct_layouts_match_the_c_compiler(binding):
    """sizeof/offsetof as gcc sees the header equal the ctypes mirrors."""
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "chhs.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(chhs_problem), sizeof(chhs_opts), sizeof(chhs_stats));
  printf("%zu %zu %zu %zu %zu %zu %zu\n", offsetof(chhs_problem, h), offsetof(chhs_opts, tol), offsetof(chhs_opts, smoother), offsetof(chhs_opts, autotune), offsetof(chhs_opts, order), offsetof(chhs_opts, tile_threads), offsetof(chhs_opts, tile_rows));
  printf("%zu %zu %zu\n", offsetof(chhs_stats, res), offsetof(chhs_stats, max_abs_phi), offsetof(chhs_stats, res0));
  printf("%zu %zu %zu\n", offsetof(chhs_opts, nu1_coarse), offsetof(chhs_opts, prolong), offsetof(chhs_opts, inner_cycles));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as tmp:
        src = os.path.join(tmp, "layout.c")
        exe = os.path.join(tmp, "layout")
        open(src, "w").write(prog)
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    want = [ctypes.sizeof(binding.chhs_problem), ctypes.sizeof(binding.chhs_opts),
            ctypes.sizeof(binding.chhs_stats),
            binding.chhs_problem.h.offset, binding.chhs_opts.tol.offset,
            binding.chhs_opts.smoother.offset, binding.chhs_opts.autotune.offset,
            binding.chhs_opts.order.offset, binding.chhs_opts.tile_threads.offset,
            binding.chhs_opts.tile_rows.offset,
            binding.chhs_stats.res.offset, binding.chhs_stats.max_abs_phi.offset,
            binding.chhs_stats.res0.offset,
            binding.chhs_opts.nu1_coarse.offset, binding.chhs_opts.prolong.offset,
            binding.chhs_opts.inner_cycles.offset]
    assert got == want


def test_workspace_bytes_rejects_invalid_problems(binding):
    o = binding.chhs_default_opts()
    good = binding.make_problem((64, 64), 1 / 64, 0.05, 1.0, 1e-3)
    assert binding.chhs_workspace_bytes([good], o) > 0
    bad = [
        binding.make_problem((64, 64), 1 / 64, 0.05, 1.0, 0.0),     # dt = 0
        binding.make_problem((64, 64), 1 / 64, 0.0, 1.0, 1e-3),     # eps = 0
        binding.make_problem((64, 64), 1 / 64, 0.05, -1.0, 1e-3),   # gamma < 0
        binding.make_problem((64, 64), 0.0, 0.05, 1.0, 1e-3),       # h = 0
        binding.make_problem((34, 34), 1 / 34, 0.05, 1.0, 1e-3),    # coarsest 17 > 8
        binding.make_problem((3, 3), 1 / 3, 0.05, 1.0, 1e-3),       # a single level
        binding.make_problem((64, 4), 1 / 64, 0.05, 1.0, 1e-3),     # coarsest 32 x 2
    ]
    for p in bad:
        assert binding.chhs_workspace_bytes([p], o) == 0
    assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(tol=0.0)) == 0
    assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(nu1=0, nu2=0)) == 0
    # the first-order step: FP64 only; orders other than 0, 1, 2 are rejected
    assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(order=1)) > 0
    assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(order=1, precision=1)) == 0
    assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(order=3)) == 0
    assert binding.chhs_default_opts().order == 2
    # tile block sizes and heights: 0 (by the tile count) or one of the kernels' sizes
    o = binding.chhs_default_opts()
    assert o.tile_threads == 0 and o.tile_rows == 0
    for nt in (256, 512, 1024):
        assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(tile_threads=nt)) > 0
    for nt in (128, 768, -1):
        assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(tile_threads=nt)) == 0
    for rows in (4, 8, 16):
        assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(tile_rows=rows)) > 0
    for rows in (2, 32, -4):
        assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(tile_rows=rows)) == 0
    # 32 rows: the FP32 finest level of the mixed path only
    assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(tile_rows=32,
                                                                          precision=1)) > 0
    # smoother 4 (fused 3D step on every level): the 3D second-order scheme only
    cube = binding.make_problem((32, 32, 32), 1 / 32, 0.05, 1.0, 1e-3)
    assert binding.chhs_workspace_bytes([cube], binding.chhs_default_opts(smoother=4)) > 0
    assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(smoother=4)) == 0
    assert binding.chhs_workspace_bytes([cube], binding.chhs_default_opts(smoother=4, order=1)) == 0
    assert binding.chhs_workspace_bytes([cube], binding.chhs_default_opts(smoother=5)) == 0
    # sweeps below the finest level (0 = as on the finest) and the prolongation
    d = binding.chhs_default_opts()
    assert d.nu1_coarse == 0 and d.nu2_coarse == 0 and d.prolong == 0
    assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(nu1_coarse=3, nu2_coarse=1,
                                                                          prolong=1)) > 0
    for bad_opts in (dict(nu1_coarse=-1), dict(nu2_coarse=-2), dict(prolong=2), dict(prolong=-1)):
        assert binding.chhs_workspace_bytes([good], binding.chhs_default_opts(**bad_opts)) == 0


def test_sizes_beyond_32_bit_indexing_are_rejected_on_the_host(binding):
    """Kernels address a field with a 32-bit byte offset and packed caller
    arrays with int offsets: an instance of 2^29 cells or more (an FP64 field of
    4 GiB) and a batch of more than 2^31 - 1 cells are refused before any
    table is built or any device work is enqueued."""
    o = binding.chhs_default_opts()
    below = binding.make_problem((256, 1024, 1024), 1 / 1024, 0.05, 1.0, 1e-3)   # 2^28 cells
    at = binding.make_problem((512, 1024, 1024), 1 / 1024, 0.05, 1.0, 1e-3)     # 2^29 cells
    wide = binding.make_problem((768, 1024, 1024), 1 / 1024, 0.05, 1.0, 1e-3)   # 768 = 3 * 2^8
    assert binding.chhs_workspace_bytes([below], o) > 0
    assert binding.chhs_workspace_bytes([at], o) == 0
    assert binding.chhs_workspace_bytes([wide], o) == 0
    # eight instances of 2^28 cells: each passes alone, together they hold
    # 2^31 cells, one more than int offsets reach (refused before the tables)
    assert binding.chhs_workspace_bytes([below] * 8, o) == 0
    arr = (binding.chhs_problem * 1)(at)
    handle = ctypes.c_void_p()
    rc = binding._lib.chhs_init(arr, 1, ctypes.byref(o), ctypes.c_void_p(1 << 20), 1 << 62, None,
                                ctypes.byref(handle))
    assert rc == binding.CHHS_E_INVAL and not handle.value


def test_workspace_accounts_for_every_level(binding):
    """11 arrays per coarse level and 8 on the finest, 256-byte aligned."""
    o = binding.chhs_default_opts()
    p = binding.make_problem((64, 64), 1 / 64, 0.05, 1.0, 1e-3)
    n = binding.chhs_workspace_bytes([p], o)
    cells = [64 * 64 // 4 ** l for l in range(6)]
    arrays = 8 * ((cells[0] * 8 + 255) // 256 * 256)
    arrays += sum(11 * ((c * 8 + 255) // 256 * 256) for c in cells[1:])
    assert n >= arrays


def test_init_rejects_bad_arguments_on_the_host(binding):
    o = binding.chhs_default_opts()
    p = binding.make_problem((64, 64), 1 / 64, 0.05, 1.0, 1e-3)
    arr = (binding.chhs_problem * 1)(p)
    handle = ctypes.c_void_p()
    # NULL workspace
    rc = binding._lib.chhs_init(arr, 1, ctypes.byref(o), None, 1 << 20, None, ctypes.byref(handle))
    assert rc == binding.CHHS_E_INVAL and not handle.value
    # workspace too small (pointer never dereferenced: size is checked first)
    rc = binding._lib.chhs_init(arr, 1, ctypes.byref(o), ctypes.c_void_p(1 << 20), 16, None,
                                ctypes.byref(handle))
    assert rc == binding.CHHS_E_NOMEM and not handle.value
    # misaligned workspace
    rc = binding._lib.chhs_init(arr, 1, ctypes.byref(o), ctypes.c_void_p((1 << 20) + 8), 1 << 30,
                                None, ctypes.byref(handle))
    assert rc == binding.CHHS_E_INVAL


def test_strerror_covers_every_code(binding):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert binding.chhs_strerror(code) != "unknown error code"
    assert binding.chhs_strerror(-99) == "unknown error code"


def test_entry_points_reject_null_context(binding):
    assert binding._lib.chhs_fas_vcycle(None, None) == binding.CHHS_E_INVAL
    assert binding._lib.chhs_step(None, None, None, None, None, 1, None) == binding.CHHS_E_INVAL
    assert binding._lib.chhs_step_log(None, None, None, None, None, 1, None) == binding.CHHS_E_INVAL
    assert binding._lib.chhs_energy_mass(None, None, None, None) == binding.CHHS_E_INVAL
    assert binding._lib.chhs_graph_count(None, None) == binding.CHHS_E_INVAL
    assert binding._lib.chhs_set_timing(None, 0) == binding.CHHS_E_INVAL
    assert binding._lib.chhs_tune_sweeps(None, None, None, None, None, None) == binding.CHHS_E_INVAL
    assert binding._lib.chhs_get_opts(None, None) == binding.CHHS_E_INVAL
    binding._lib.chhs_destroy(None)
