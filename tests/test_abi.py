"""CPU-side checks of the C ABI: every declared symbol is exported, and the
host-only helpers and argument checks behave as documented (no GPU calls)."""
import ctypes
import glob
import os
import re

import pytest

from paper_1801_01134_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DECL = re.compile(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\*?\s*(spc_\w+)\s*\(", re.M)


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        with open(h) as f:
            names |= set(DECL.findall(f.read()))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_symbols()
    for must in ("spc_beta_count", "spc_csr_to_beta", "spc_beta_to_csr", "spc_plan_create",
                 "spc_spmv_beta"):
        assert must in names


@pytest.mark.parametrize("name", declared_symbols())
def test_symbol_exported(name):
    L = B.lib()
    assert hasattr(L, name), f"{name} declared in include/ but not exported"


def test_host_helpers():
    L = B.lib()
    assert L.spc_status_string(0) == b"SPC_OK"
    assert L.spc_status_string(-2) == b"SPC_ERR_UNSUPPORTED_SHAPE"
    assert [L.spc_shape_index(r, c) for r, c in B.SHAPES] == list(range(6))
    assert L.spc_shape_index(3, 3) == -2
    pad = 512
    assert L.spc_mask_bytes(1, 8, 1) == 8 + pad and L.spc_mask_bytes(1, 8, 8) == 8 + pad
    assert L.spc_mask_bytes(1, 8, 9) == 16 + pad
    assert L.spc_mask_bytes(4, 8, 3) == 16 + pad and L.spc_mask_bytes(2, 8, 4) == 8 + pad
    assert L.spc_mask_bytes(1, 8, 0) == pad
    assert L.spc_mask_bytes(5, 5, 1) == -1
    assert L.spc_version() >= 10000


def test_argument_errors_before_any_launch():
    L = B.lib()
    nb = ctypes.c_int64()
    # unsupported shape, negative sizes, null outputs: refused on the host
    assert L.spc_beta_count(3, 3, 4, 4, None, None, None, ctypes.byref(nb), None) == -2
    assert L.spc_beta_count(1, 8, -1, 4, None, None, None, ctypes.byref(nb), None) == -1
    assert L.spc_beta_count(1, 8, 4, 4, None, None, None, ctypes.byref(nb), None) == -1
    assert L.spc_beta_count(1, 8, 1 << 31, 4, None, None, None, ctypes.byref(nb), None) == -5
    v = B.BetaView(3, 3, 1, 0, 4, 4, 0, 0, None, None, None, None)
    h = ctypes.c_void_p()
    assert L.spc_plan_create(ctypes.byref(v), None, ctypes.byref(h), None) == -2
    v = B.BetaView(1, 8, 7, 0, 4, 4, 0, 0, None, None, None, None)
    assert L.spc_plan_create(ctypes.byref(v), None, ctypes.byref(h), None) == -1
    v = B.BetaView(1, 8, 1, 0, 4, 4, 2, 2, 16, 32, 12, 64)   # misaligned masks pointer
    assert L.spc_plan_create(ctypes.byref(v), None, ctypes.byref(h), None) == -1
    assert b"aligned" in L.spc_last_error()
    assert L.spc_spmv_beta(None, None, None, None, 0, None) == -1
    assert L.spc_plan_destroy(None) == 0


def test_plan_parameters_checked_on_the_host():
    """Plan parameters are validated before any device call (the pointers of
    this view are never dereferenced)."""
    L = B.lib()
    h = ctypes.c_void_p()
    v = B.BetaView(2, 4, 1, 0, 8, 8, 16, 4, 4096, 8192, 16384, 32768)
    for bad in (dict(cu_groups=1), dict(cu_groups=9), dict(cu_groups=-1),
                dict(mode=1, tile_bits=2048, cu_groups=2), dict(mode=5), dict(mode=-1),
                dict(mode=3, wave_tiles=2), dict(mode=3, pipeline=1), dict(mode=3, wave_chunks=3),
                dict(wave_chunks=5), dict(mode=1, tile_bits=1000), dict(pipeline=-1),
                dict(mode=1, tile_bits=2048, pipeline=1), dict(tile_order=2), dict(tile_order=-1)):
        p = B.PlanParams(**bad)
        assert L.spc_plan_create(ctypes.byref(v), ctypes.byref(p), ctypes.byref(h), None) == -1, bad
        assert not h.value
    # value lanes exist for beta(1,8) only
    p = B.PlanParams(mode=4)
    assert L.spc_plan_create(ctypes.byref(v), ctypes.byref(p), ctypes.byref(h), None) == -2
    assert not h.value


def test_kernel_classes_and_output_counts_on_the_host():
    L = B.lib()
    # classes: the six shapes, then the test kernels of beta(1,8) and beta(2,4)
    assert [L.spc_class_shape(k) for k in range(8)] == [0, 1, 2, 3, 4, 5, 0, 1]
    assert L.spc_class_shape(8) == -1 and L.spc_class_shape(-1) == -1
    assert [L.spc_class_mode(k) for k in range(8)] == [-1] * 6 + [2, 2]
    assert L.spc_selector_n_classes(None, 0) == 0
    # the network takes 6 or 8 outputs; any other count is refused before a launch
    assert L.spc_mlp_targets(None, 0, 7, None, None) == -1
    assert L.spc_mlp_targets(None, 0, 6, None, None) == 0
    assert L.spc_mlp_infer(None, None, None, None, 0, 8, None, None, None) == -1   # null parameters
    sel = ctypes.c_void_p()
    assert L.spc_selector_create(ctypes.byref(sel)) == 0
    one = (ctypes.c_double * 7)(*([1.0] * 7))
    assert L.spc_selector_fit_interp(sel, 1, 7, one, one, 1) == -1     # 7 classes
    assert L.spc_selector_fit_interp(sel, 1, 8, (ctypes.c_double * 8)(*([2.0] * 8)),
                                     (ctypes.c_double * 8)(*([3.0] * 8)), 0) == 0
    assert L.spc_selector_n_classes(sel, 0) == 8 and L.spc_selector_n_classes(sel, 1) == 0
    assert L.spc_selector_destroy(sel) == 0


def test_batch_parameter_counts_on_the_host():
    L = B.lib()
    out = ctypes.c_void_p()
    v = (B.BetaView * 2)()
    # n_params must be 0, 1 or count; count >= 1
    assert L.spc_batch_create(2, v, None, 1, ctypes.byref(out), None) == -1
    assert L.spc_batch_create(0, v, None, 0, ctypes.byref(out), None) == -1
    p = (B.PlanParams * 2)()
    assert L.spc_batch_create(2, v, p, 3, ctypes.byref(out), None) == -1
