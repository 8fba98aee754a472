"""Host-side checks of the C ABI: the library loads and exports every symbol
include/fasttracks.h declares, and host-only entry points behave (no GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fasttracks.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ft_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("ft_create", "ft_set_sfts", "ft_set_velocities", "ft_eval_templates",
                 "ft_toplist"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2411_18370_amd import fasttracks
    if not os.path.exists(fasttracks.LIB_PATH):
        from paper_2411_18370_amd import build
        build.build()
    lib = C.CDLL(fasttracks.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(fasttracks.EXPORTS) <= set(_declared())


def test_host_only_entry_points():
    from paper_2411_18370_amd import fasttracks as ft
    ft.load()
    assert ft.ft_tile_count() >= 4
    names = [ft.ft_tile_name(i) for i in range(1, ft.ft_tile_count() + 1)]
    assert all(n.startswith("L") for n in names)
    assert ft.ft_tile_name(0) == "" and ft.ft_tile_name(10_000) == ""
    assert ft.load().ft_status_string(-3) == b"FT_E_RANGE"


def test_struct_layouts_match_header():
    from paper_2411_18370_amd import fasttracks as ft
    assert C.sizeof(ft.ft_bank) == 88
    assert C.sizeof(ft.ft_eval_opts) == 40
    assert ft.ft_eval_opts.statistic.offset == 28 and ft.ft_eval_opts.weights.offset == 32
    assert C.sizeof(ft.ft_candidate) == 72
    assert ft.ft_candidate.s64.offset == 56
    assert C.sizeof(ft.ft_tune_entry) == 32
    assert C.sizeof(ft.ft_box_partition) == 32 and C.sizeof(ft.ft_box_result) == 32
    assert ft.BOX_DTYPE.itemsize == 32 and ft.ft_box_result.s64.offset == 16


def test_null_arguments_are_rejected_without_a_device():
    from paper_2411_18370_amd import fasttracks as ft
    lib = ft.load()
    assert lib.ft_create(None, 0, None) == ft.FT_E_INVALID
    assert lib.ft_set_sfts(None, 1, None, None, 1800.0, 0, 1, None, None) == ft.FT_E_INVALID
    assert lib.ft_set_velocities(None, None) == ft.FT_E_INVALID
    assert lib.ft_sync(None) == ft.FT_E_INVALID
    assert lib.ft_tune_clear(None) == ft.FT_E_INVALID
    assert lib.ft_tune_report(None, None, 0, None, None) == ft.FT_E_INVALID
    assert lib.ft_lib_sincos(None, None, 0, None, None) == ft.FT_E_INVALID
    assert lib.ft_q_sample(None, None, 0, None, None, None, None) == ft.FT_E_INVALID
    assert lib.ft_gen_binary_bank(None, None, 0, 0, 0, None, None, None, None, None) == ft.FT_E_INVALID
    assert lib.ft_eval_binary_random(None, None, 0, 0, 0.0, None, None) == ft.FT_E_INVALID
    assert lib.ft_set_arms(None, None) == ft.FT_E_INVALID
    assert lib.ft_binary_cos_mode(None, 0, None) == ft.FT_E_INVALID
    assert lib.ft_eval_binary_boxes(None, None, 0, 0, 0.0, None, None, None, None) == ft.FT_E_INVALID
    assert lib.ft_toplist_number_count(None, 0, None, None, None) == ft.FT_E_INVALID
    assert C.sizeof(ft.ft_binary_region) == 96


def test_oracle_and_library_share_no_code():
    """The oracle neither imports nor links the GPU library, and vice versa."""
    import glob
    for p in glob.glob(os.path.join(ROOT, "oracle", "*")):
        if p.endswith((".py", ".c", ".h")):
            txt = open(p).read()
            assert "fasttracks" not in txt.replace("libfasttracks", "") or p.endswith("__init__.py")
            assert "csrc" not in txt
    for p in glob.glob(os.path.join(ROOT, "paper_2411_18370_amd", "**", "*"), recursive=True):
        if p.endswith((".py", ".cpp", ".hip", ".h")):
            txt = open(p).read()
            assert "import oracle" not in txt and "from oracle" not in txt, p
            assert "ft_oracle" not in txt, p
