"""The C-ABI library loads on the CPU host and exports every symbol include/gempe.h declares.

No compute call is made here (there is no GPU); only host-side argument checks that return
before anything touches the device.
"""
import ctypes
import os
import re

import pytest

from paper_2011_03479_amd import gempe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "gempe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(gempe_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gempe.LIB_PATH):
        pytest.fail("libgempe.so is not built (run python -m paper_2011_03479_amd.build)")
    return gempe.load()


def test_header_matches_binding_list():
    assert header_functions() == sorted(gempe.ABI_SYMBOLS)


def test_every_declared_symbol_is_exported(lib):
    for name in header_functions():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_params_default_and_status_strings(lib):
    p = gempe.params_default()
    assert (p.mu, p.sigma, p.precision, p.near_k, p.flags) == (1.5, 1.0, gempe.GEMPE_FP32, 9.0, 0)
    assert ctypes.sizeof(gempe.gempe_params) == 40
    for s in range(0, -8, -1):
        assert gempe.status_string(s) not in ("", "unknown status")
    assert gempe.status_string(42) == "unknown status"


def test_host_side_argument_checks(lib):
    out = ctypes.c_void_p()
    assert lib.gempe_graph_create(10, 0, None, None, None, 0, None, None) == gempe.GEMPE_ERR_ARG
    assert lib.gempe_graph_create(0, 0, None, None, None, 0, None, ctypes.byref(out)) == gempe.GEMPE_ERR_ARG
    assert lib.gempe_graph_create(10, 3, None, None, None, 0, None, ctypes.byref(out)) == gempe.GEMPE_ERR_GRAPH
    assert lib.gempe_graph_create(3, 8, None, None, None, 0, None, ctypes.byref(out)) == gempe.GEMPE_ERR_GRAPH
    assert "nnz" in gempe.last_error()
    # the graph's device memory is the caller's: size query, then the workspace checks run
    # on the host before anything touches the (here fake, never dereferenced) pointers
    need = lib.gempe_graph_workspace_bytes(1000, 20000)
    assert need >= 8 * 1001 + 2 * 4 * 20000 + 8 * 2 * 10000
    assert lib.gempe_graph_workspace_bytes(0, 0) == 0 and lib.gempe_graph_workspace_bytes(10, 3) == 0
    fake = ctypes.c_void_p(0x1000)
    assert lib.gempe_graph_create(1000, 20000, fake, fake, None, need, None, ctypes.byref(out)) == \
        gempe.GEMPE_ERR_ARG
    assert "workspace" in gempe.last_error()
    assert lib.gempe_graph_create(1000, 20000, fake, fake, ctypes.c_void_p(0x1010), need, None,
                                  ctypes.byref(out)) == gempe.GEMPE_ERR_ARG
    assert "aligned" in gempe.last_error()
    assert lib.gempe_graph_create(1000, 20000, fake, fake, fake, need - 1, None, ctypes.byref(out)) == \
        gempe.GEMPE_ERR_NOMEM
    assert out.value is None
    p = gempe.params_default()
    assert lib.gempe_workspace_bytes(None, 2, ctypes.byref(p)) == 0
    assert lib.gempe_loss_grad(None, 2, None, None, None, None, None, None, 0, ctypes.byref(p), None) == \
        gempe.GEMPE_ERR_ARG
    assert lib.gempe_embed(None, 2, None, 1, ctypes.c_float(0.1), None, None, 0, ctypes.byref(p), None) == \
        gempe.GEMPE_ERR_ARG
    # flags: GEMPE_F_REVERSE_TILES is the only known bit (the footprint query runs the
    # problem checks on the host and answers 0 for a rejected problem)
    pf = gempe.params_default(flags=gempe.GEMPE_F_REVERSE_TILES)
    assert lib.gempe_job_footprint(1000, 10000, 2, 10, ctypes.byref(pf)) > 0
    for bad in (2, 0x80000000):
        pf = gempe.params_default(flags=bad)
        assert lib.gempe_job_footprint(1000, 10000, 2, 10, ctypes.byref(pf)) == 0
        assert "flag" in gempe.last_error()
    assert lib.gempe_graph_num_edges(None) == -1 and lib.gempe_graph_num_vertices(None) == -1
    assert lib.gempe_graph_destroy(None) == gempe.GEMPE_ERR_ARG


def test_server_structs_and_host_checks(lib):
    assert ctypes.sizeof(gempe.gempe_job_desc) == 4 + 4 + 8 + 3 * 8 + 4 + 4 + 40 + 8 + 8 + 8
    assert ctypes.sizeof(gempe.gempe_job_info) == 16 + 24 + 8
    p = gempe.params_default()
    # footprints are pure host arithmetic: graph + X + history + workspace, monotone in n
    f1 = lib.gempe_job_footprint(1000, 10000, 2, 200, ctypes.byref(p))
    f2 = lib.gempe_job_footprint(2000, 10000, 2, 200, ctypes.byref(p))
    assert 0 < f1 < f2
    assert f1 >= 1000 * 2 * 4 * 6 + 8 * 1001 + 4 * 10000 * 2 + 8 * 201
    assert lib.gempe_job_footprint(1, 0, 2, 200, ctypes.byref(p)) == 0
    assert lib.gempe_job_footprint(1000, 10000, 0, 200, ctypes.byref(p)) == 0
    out = ctypes.c_void_p()
    assert lib.gempe_server_create(1 << 20, 0, ctypes.byref(out)) == gempe.GEMPE_ERR_ARG
    assert lib.gempe_server_create(1 << 20, 4, None) == gempe.GEMPE_ERR_ARG
    assert lib.gempe_server_submit(None, None, None) == gempe.GEMPE_ERR_ARG
    assert lib.gempe_server_destroy(None) == gempe.GEMPE_ERR_ARG


def test_sweep_launch_bound_is_checked_on_the_host(lib):
    """The FP32 sweeps launch a workgroup per tile; a problem whose launch would exceed
    HIP's 2^32 work-items is refused on the host (GEMPE_ERR_UNSUPPORTED through every
    entry point; the job footprint query answers 0) instead of failing at launch."""
    p = gempe.params_default()
    for n, d in ((741_000, 32), (2_900_000, 16), (5_900_000, 2), (100_000, 128)):
        assert lib.gempe_job_footprint(n, 2 * n, d, 1, ctypes.byref(p)) > 0, (n, d)
    for n, d in ((742_000, 32), (1_000_000, 128), (3_000_000, 16), (6_000_000, 3), (2_000_000_000, 2)):
        assert lib.gempe_job_footprint(n, 2 * n, d, 1, ctypes.byref(p)) == 0, (n, d)
        assert "too large" in gempe.last_error()
