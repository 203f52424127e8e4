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


def test_tau_integrals_host_entry_point():
    """dqmc_tau_integrals (host arithmetic only) against the oracle's
    integrals: trapezoid and least-squares polynomial fits, and its argument
    checks."""
    p = pytest.importorskip("paper_2609_14668_amd")
    try:
        p.load()
    except ImportError:
        pytest.skip("libdqmc.so not built")
    import numpy as np
    from oracle import tau
    rng = np.random.default_rng(4)
    for n, dt in ((91, 0.1), (11, 0.2), (2, 0.05)):
        t = dt * np.arange(n)
        c = 0.3 * np.exp(-2.0 * t) + 0.05 + 0.01 * rng.standard_normal(n)
        for deg in [None] + [k for k in (1, 3, 6, 9) if k < n]:
            got = p.tau_integrals(c, dt, 648, -1 if deg is None else deg)
            ref = tau.tau_integrals(c, dt, 648, deg)
            np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-15)
    for bad in ((np.ones(1), 0.1, 8, -1), (np.ones(5), 0.0, 8, -1), (np.ones(5), 0.1, 0, -1),
                (np.ones(5), 0.1, 8, 5), (np.ones(20), 0.1, 8, 13)):
        with pytest.raises(p.DqmcError):
            p.tau_integrals(*bad)
