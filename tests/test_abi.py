"""The C-ABI library loads and exports every entry point declared in
include/dqmc.h; host-side validation works without a GPU."""
import os
import re

import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "dqmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dqmc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("dqmc_create", "dqmc_sweep", "dqmc_replay", "dqmc_get_green", "dqmc_measure", "dqmc_destroy"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    p = pytest.importorskip("paper_2609_14668_amd")
    try:
        lib = p.load()
    except ImportError:
        pytest.skip("libdqmc.so not built")
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_workspace_size_and_validation():
    p = pytest.importorskip("paper_2609_14668_amd")
    try:
        p.load()
    except ImportError:
        pytest.skip("libdqmc.so not built")
    small = p.dqmc_workspace_size(workloads.plain_L3())
    big = p.dqmc_workspace_size(workloads.plain_L12(1))
    assert 0 < small < big
    bad = workloads.plain_L3()
    bad[0]["beta"] = 3.05          # beta/dtau not an integer
    with pytest.raises(p.DqmcError):
        p.dqmc_workspace_size(bad)
    bad = workloads.plain_L3()
    bad[0]["L"] = 17               # prime factor the FFT does not support
    with pytest.raises(p.DqmcError):
        p.dqmc_workspace_size(bad)
    bad = workloads.plain_L3()
    bad[0]["n_stab"] = 7           # must divide M = 30
    with pytest.raises(p.DqmcError):
        p.dqmc_workspace_size(bad)


def test_status_strings():
    p = pytest.importorskip("paper_2609_14668_amd")
    try:
        lib = p.load()
    except ImportError:
        pytest.skip("libdqmc.so not built")
    assert lib.dqmc_status_string(0) == b"ok"
    assert b"invalid" in lib.dqmc_status_string(-1)
