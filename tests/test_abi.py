"""CPU checks of the C ABI: the library builds, loads and exports every
function include/tri.h declares; host-side argument handling that needs no
device (null context, status strings)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "tri.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def T():
    import paper_1812_01178_amd as T
    if not os.path.exists(T.LIB_PATH):
        from paper_1812_01178_amd import build
        build.build()
    T.lib()
    return T


def test_header_declares_the_four_solves():
    names = declared_functions()
    for f in ("tri_pdd_solve", "tri_ppt_solve", "adi_sweep", "poisson_wavenumber_solve"):
        assert f in names


def test_library_exports_every_declared_symbol(T):
    out = subprocess.run(["nm", "-D", "--defined-only", T.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    assert sorted(T.EXPORTED) == declared_functions()


def test_library_is_gfx950_code(T):
    """The embedded code object targets gfx950 (bundle id in .hip_fatbin)."""
    blob = open(T.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_null_context_and_status_strings(T):
    L = T.lib()
    assert L.tri_pdd_solve(None, None, None, 0, None, 4, 0, 0, None) == T.TRI_E_ARG
    assert L.tri_sync_status(None) == T.TRI_E_ARG
    assert L.tri_plan_execute(None) == T.TRI_E_ARG
    assert T.tri_status_string(T.TRI_E_SHAPE).startswith("invalid shape")
    assert T.tri_status_string(99) == "unknown status"
    assert L.tri_plan_item_partitions(None, 0) == -1
    assert L.tri_plan_launch_count(None) == -1
    assert L.tri_stream_copy(None, None, None, 0) == T.TRI_E_ARG
    assert L.tri_set_pdd_tolerance(None, 1e-12) == T.TRI_E_ARG
    assert L.tri_reserve(None, 64, 4, 1) == T.TRI_E_ARG
    # the pressure-step entry points refuse a null context before anything else
    assert L.spanwise_rfft(None, None, None, 4, 8) == T.TRI_E_ARG
    assert L.spanwise_irfft(None, None, None, 4, 8) == T.TRI_E_ARG
    assert L.streamwise_dct(None, None, 8, 1) == T.TRI_E_ARG
    assert L.streamwise_idct(None, None, 8, 1) == T.TRI_E_ARG
    assert L.projection_divergence_rfft(None, None, None, None, 1.0, None, 4, 4, 8) == T.TRI_E_ARG
    assert L.projection_correct(None, None, None, None, None, None, 1.0, 4, 4, 8) == T.TRI_E_ARG
    assert L.projection_step(None, None, None, None, 1.0, None, None, None, None, None, 4, 4, 8, 1) == T.TRI_E_ARG
    assert L.projection3d_divergence_rfft(None, None, None, None, 1.0, None, 1.0, None, 4, 4, 8) == T.TRI_E_ARG
    assert L.projection3d_correct(None, None, None, None, None, None, 1.0, None, 1.0, 4, 4, 8) == T.TRI_E_ARG
    assert L.projection3d_step(None, None, None, None, 1.0, None, 1.0, None, None, None, None, None, None,
                               4, 4, 8, 1) == T.TRI_E_ARG
    assert L.poisson_shifted_solve(None, None, 4, 4, 4, None, None, None, None, 1, T.TRI_PPT) == T.TRI_E_ARG
