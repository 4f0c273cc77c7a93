"""Host-side checks of the C ABI that need no GPU: the library loads, exports every function
the header declares, and the host-only dry run validates designs and sizes workspaces."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2604_02624_amd import dpx, workloads as wk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpx.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(dpx_[a-z_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dpx.LIB_PATH):
        pytest.fail("libdpx.so is not built (run python -m paper_2604_02624_amd.build)")
    return dpx.load_library()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for f in ("dpx_plan_create", "dpx_plan_destroy", "dpx_forward", "dpx_loss", "dpx_backward",
              "dpx_last_error", "dpx_plan_query", "dpx_plan_layout"):
        assert f in names


def test_binding_matches_the_header_constants_and_option_layout():
    """Status codes and dpx_opts field order as the header declares them."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    codes = dict((name, int(v)) for name, v in re.findall(r"\b(DPX_(?:OK|E_[A-Z]+))\s*=\s*(\d+)", src))
    assert codes == {name: code for code, name in dpx.STATUS_NAMES.items()}
    body = re.search(r"typedef struct dpx_opts \{(.*?)\} dpx_opts;", src, flags=re.S).group(1)
    fields = re.findall(r"\b(int32_t|int64_t)\s+(\w+);", body)
    ctype = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64}
    assert [(n, ctype[t]) for t, n in fields] == list(dpx.COpts._fields_)


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(dpx.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), f"{name} declared in dpx.h but not exported"
    assert b"gfx950" in lib.dpx_version()


def _query(designs, **kw):
    return dpx.plan_query(designs, **kw)


def test_query_workspace_of_the_large_workload(lib):
    d = wk.make_workload(1)["designs"][0]
    b = _query([d])
    N, M, K, W, F = 64, 128, 2, 6, 32
    spec = W * N * M * 8
    ck = (K - 1) * W * N * N * 8            # layer 0's field is rebuilt from u_in and h
    assert b >= spec + ck + W * F * F * 8


def test_query_checkpoint_slab_of_the_first_layer(lib):
    """Without an input gap the field after the first layer is not stored (one slab of W N^2
    complex less); with one it is, in store and recompute modes alike."""
    d = wk.make_workload(1)["designs"][0]
    N, W = d["n"], d["n_wl"]
    gap = dict(d, z_in=10e-6)
    assert _query([gap]) - _query([d]) == W * N * N * 8
    rec = dict(checkpoint_mode=1, wl_chunk=2)
    assert _query([gap], **rec) - _query([d], **rec) == 2 * N * N * 8
    one = dict(d, layers=1, z=d["z"][:1])
    assert _query([dict(one, z_in=10e-6)]) - _query([one]) == W * N * N * 8


def test_query_store_vs_recompute_memory(lib):
    d = wk.make_design(n=512, layers=4, wl=np.linspace(450e-9, 750e-9, 4096), n_mat=1.5, dx=3e-7,
                       z=3e-5, fov=64)
    store = _query([d])
    rec = _query([d], checkpoint_mode=1, wl_chunk=64)
    assert store > 32 * 2 ** 30            # 24 GiB of checkpoints and 16 GiB of spectra
    assert rec < 2 * 2 ** 30
    assert store < 288e9                    # fits one MI355X
    two = _query([d], streams=2)            # two lanes of quarter-size chunks: 8 GiB of spectra
    assert store - two >= 8 * 2 ** 30       # instead of 16 GiB for the whole workload at once


def test_query_counts_transfer_tables(lib):
    d = wk.make_workload(1)["designs"][0]           # N 64, M 128, 2 layers with one gap length
    off = _query([d], transfer_table=1)
    on = _query([d], transfer_table=2)
    assert on - off == 1 * d["n_wl"] * 65 * 65 * 8
    d2 = dict(d)
    d2["z"] = np.array([d["z"][0], 2 * d["z"][0]])   # two gap lengths: two tables
    assert _query([d2], transfer_table=2) - _query([d2], transfer_table=1) == 2 * d["n_wl"] * 65 * 65 * 8
    with pytest.raises(dpx.DpxError):
        _query([d], transfer_table=3)


@pytest.mark.parametrize("field,value,status", [
    ("n", 63, dpx.DPX_E_ARG),
    ("n", 0, dpx.DPX_E_ARG),
    ("layers", 0, dpx.DPX_E_ARG),
    ("fov", 65, dpx.DPX_E_ARG),
    ("fov", 31, dpx.DPX_E_ARG),
    ("bin", 3, dpx.DPX_E_ARG),
    ("pad", 3, dpx.DPX_E_ARG),
    ("dx", -1.0, dpx.DPX_E_ARG),
    ("dx", float("nan"), dpx.DPX_E_ARG),
    ("n", 80, dpx.DPX_E_UNSUPPORTED),
    ("n_wl", 0, dpx.DPX_E_ARG),
])
def test_query_rejects_bad_designs(lib, field, value, status):
    d = dict(wk.make_workload(1)["designs"][0])
    d[field] = value
    with pytest.raises(dpx.DpxError) as e:
        _query([d])
    assert e.value.status == status
    assert len(str(e.value)) > 12


def test_query_rejects_bad_arrays(lib):
    d = dict(wk.make_workload(1)["designs"][0])
    d["wl"] = d["wl"].copy()
    d["wl"][2] = 0.0
    with pytest.raises(dpx.DpxError) as e:
        _query([d])
    assert e.value.status == dpx.DPX_E_ARG and "wl[2]" in str(e.value)
    d = dict(wk.make_workload(1)["designs"][0])
    d["z"] = np.array([1e-5, -1e-6])
    with pytest.raises(dpx.DpxError):
        _query([d])
    d = dict(wk.make_workload(1)["designs"][0])
    d["kappa"] = -np.ones(6)
    with pytest.raises(dpx.DpxError):
        _query([d])


def test_query_rejects_bad_options(lib):
    d = wk.make_workload(1)["designs"][0]
    with pytest.raises(dpx.DpxError):
        _query([d], checkpoint_mode=2)
    with pytest.raises(dpx.DpxError):
        _query([d], force_variant=5)
    with pytest.raises(dpx.DpxError):
        _query([d], schedule=3)
    with pytest.raises(dpx.DpxError):
        _query([d], small_path=2)
    assert _query([d], schedule=2) > 0
    with pytest.raises(dpx.DpxError) as e:
        _query([d], schedule=2, checkpoint_mode=1)
    assert e.value.status == dpx.DPX_E_UNSUPPORTED


def test_null_plan_and_pointers_are_errors(lib):
    assert lib.dpx_forward(None, None, None, None, None) == dpx.DPX_E_ARG
    assert b"plan" in lib.dpx_last_error()
    assert lib.dpx_backward(None, None, None, None, None, None) == dpx.DPX_E_ARG
    assert lib.dpx_loss(None, None, None, None, None, None) == dpx.DPX_E_ARG
    assert lib.dpx_plan_destroy(None) == dpx.DPX_OK


def test_every_workload_is_accepted(lib):
    for cfg in (1, 3, 4, 5):
        w = wk.make_workload(cfg)
        assert _query(w["designs"]) > 0
