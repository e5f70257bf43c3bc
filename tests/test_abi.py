"""The C-ABI library loads and exports every function declared in
include/gpumcd.h (no compute calls: this runs without a GPU)."""
import os

import pytest

from paper_1101_1245_amd import gpumcd as G


def test_library_exports_every_declared_symbol():
    if not os.path.exists(G.LIB_PATH):
        pytest.fail("libgpumcd.so is not built; run __graft_entry__.build()")
    L = G.lib()
    names = G.header_symbols()
    assert {"gmc_create", "gmc_load_tables", "gmc_load_phantom", "gmc_run_beam"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_no_device_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(G.GpumcdError):
        G.Context(0)
