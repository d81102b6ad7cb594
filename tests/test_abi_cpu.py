"""CPU checks of the boundary: the library loads, exports every symbol include/spt.h declares
with the binding's signature table, and host-side argument checks fire without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "spt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spt_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1809_09175_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def test_every_declared_symbol_is_exported_and_bound(lib):
    from paper_1809_09175_amd import _lib
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.SIGNATURES) == names


def test_status_strings_and_version(lib):
    assert lib.spt_version() >= 100
    for code in range(-7, 1):
        assert lib.spt_status_string(code)
    assert b"unknown" in lib.spt_status_string(-99)


def test_host_argument_checks(lib):
    dims = (ctypes.c_int64 * 3)(10, 20, 30)
    assert lib.spt_tensor_workspace_bytes(3, dims, 1000, 1) > 0
    assert lib.spt_tensor_workspace_bytes(1, dims, 1000, 1) == 0      # order < 2
    assert lib.spt_tensor_workspace_bytes(6, dims, 1000, 1) == 0      # order > 5
    assert lib.spt_tensor_workspace_bytes(3, dims, -1, 1) == 0
    assert lib.spt_tensor_workspace_bytes(3, dims, 1000, 2) == 0      # BF16 values
    h = ctypes.c_void_p()
    # null output handle, misaligned / short workspace: rejected before any GPU call
    assert lib.spt_tensor_create(None, 3, dims, 0, None, None, 1, None, 0, None) == -1
    assert lib.spt_tensor_create(ctypes.byref(h), 3, dims, 0, None, None, 1,
                                 ctypes.c_void_p(0x1001), 1 << 20, None) == -5
    assert lib.spt_mttkrp(None, 0, 8, None, 1, None, None, None, None, None) == -1
    assert lib.spt_cp_workspace_bytes(None, 8) == 0
    assert lib.spt_f32_to_bf16(None, None, -1, None) == -1
    assert lib.spt_stream_triad(None, None, None, ctypes.c_float(1.0), -5, None) == -1
    # generalized-CP entry points: null tensor / loss, bad loss kind, bad sizes and steps
    assert lib.spt_gcp_fused(None, 8, None, 1, 0, None, None, None, None, None) == -1
    assert lib.spt_gcp_forward(None, 8, None, 1, 4, None, None, None, None, 0, None) == -1
    assert lib.spt_gcp_sample(None, 1, 0, 4, 4, None, None, None, 1, None) == -1
    assert lib.spt_adam_step(None, None, None, None, 10, 1, 1e-3, 0.9, 0.999, 1e-8, 0,
                             float("-inf"), None) == -1                   # step t = 0
    assert lib.spt_adam_step(None, None, None, None, 0, 2, 1e-3, 0.9, 0.999, 1e-8, 1,
                             float("-inf"), None) == -1                   # BF16 not supported
    assert lib.spt_adam_step(None, None, None, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, 1,
                             float("-inf"), None) == 0                    # empty: nothing to do
    assert lib.spt_scale_values(None, None, 5, 1, None, None) == -1
    # sorted copies: null tensor for either order; the size query answers 0
    assert lib.spt_tensor_sorted_copy_bytes(None, -1, 0) == 0
    assert lib.spt_tensor_sorted_copy_bytes(None, 0, 1) == 0
    assert lib.spt_tensor_sort_copy(None, -1, 1, None, 0, None) == -1
    assert lib.spt_cp_fit_after_mode(None, 0, 8, None, 1, None, None, None, 0, None, None,
                                     None) == -1


def test_workspace_accounting_matches_section5_storage():
    """The permutations cost one P-vector of ordinals per mode (Sec. 6: total (s_r+2 d s_o) P
    with the keys); the workspace holds the records, d permutations and d sorted keys."""
    from paper_1809_09175_amd import _lib
    lib = _lib.load()
    P = 1 << 20
    dims = (ctypes.c_int64 * 3)(1000, 1000, 1000)
    ws = lib.spt_tensor_workspace_bytes(3, dims, P, 1)
    records = 16 * P
    perms_and_keys = 2 * 3 * 4 * P
    sort_scratch = 2 * 4 * P
    assert records + perms_and_keys + sort_scratch <= ws < records + perms_and_keys + sort_scratch + (8 << 20)


def test_paper_block_size_table_matches_golden():
    """spt_paper_block_sizes reproduces Tab. sizes (tests/golden/paper_tab_sizes.txt)."""
    from paper_1809_09175_amd import _lib
    lib = _lib.load()
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_tab_sizes.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append(tuple(int(x) for x in line.split()))
    for lo, hi, vs, fbs in rows:
        for R in range(lo, (hi or lo + 200) + 1):
            v = ctypes.c_int()
            f = ctypes.c_int()
            assert lib.spt_paper_block_sizes(R, ctypes.byref(v), ctypes.byref(f)) == 0
            assert (v.value, f.value) == (vs, fbs), R
    # at most four columns per thread, as the paper states for its choices
    for R in range(1, 300):
        v = ctypes.c_int()
        f = ctypes.c_int()
        lib.spt_paper_block_sizes(R, ctypes.byref(v), ctypes.byref(f))
        assert f.value <= 4 * v.value


def test_batch_config_queries():
    from paper_1809_09175_amd import _lib
    lib = _lib.load()
    assert lib.spt_batch_workspace_bytes(0) == 0
    assert lib.spt_batch_workspace_bytes(64) >= 64 * 64
    assert lib.spt_batch_supported_tune(3, 1, 2, 8, 4) == 1      # F32, permuted, 8 x 4
    assert lib.spt_batch_supported_tune(3, 0, 2, 8, 4) == 0      # F64 not batched
    assert lib.spt_batch_supported_tune(4, 1, 2, 8, 4) == 0      # 3-way only
