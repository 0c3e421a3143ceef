"""The C-ABI library loads and exports every entry point its header declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "sbpfdtd.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(sbp_[a-z_0-9]+)\s*\(", text))
    names.discard("sbp_alloc_fn")
    names.discard("sbp_free_fn")
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sbp_create", "sbp_add_block", "sbp_set_face_bc", "sbp_connect", "sbp_add_source",
                     "sbp_add_probe", "sbp_finalize", "sbp_step", "sbp_read_field", "sbp_read_energy",
                     "sbp_read_probe", "sbp_save_state", "sbp_load_state", "sbp_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2206_00638_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the Python binding covers the same names
    assert set(declared_functions()) == set(binding.SIGNATURES)


def test_null_context_is_rejected_without_gpu():
    from paper_2206_00638_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.lib()
    assert lib.sbp_step(None, 1) == binding.SBP_EINVAL
    assert lib.sbp_last_error(None) == b"null context"
