"""The C ABI library: it loads, exports every function include/deepscatter.h
declares, and rejects bad arguments on the host before touching a device."""
import ctypes as C
import os
import re

import pytest

import paper_1709_05418_amd as ds

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")

pytestmark = pytest.mark.skipif(not os.path.exists(ds.LIB_PATH),
                                reason="libdeepscatter.so not built")


def declared_functions():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if fn.endswith(".h"):
            txt = open(os.path.join(HEADER_DIR, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(ds_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert "ds_predict" in names and "ds_cloud_create" in names
    lib = C.CDLL(ds.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_param_count_without_device():
    assert "gfx950" in ds.ds_version()
    assert ds.ds_net_param_count(10, 200, 3) == 1_296_601
    assert ds.ds_net_param_count(6, 64, 3) == 140_993
    assert ds.ds_net_param_count(0, 200, 3) == -1
    assert ds.ds_net_param_count(10, 300, 3) == -1


def test_null_and_bad_arguments_are_rejected_before_any_launch():
    L = ds.lib()
    out = C.c_void_p()
    amin = (C.c_float * 3)(-0.5, -0.5, -0.5)
    assert L.ds_cloud_create(None, None, 0, 8, 8, 8, 1.0, amin, 0.125, 3, None, 2,
                             C.byref(out)) == -1
    assert "NULL" in ds.ds_last_error()
    assert L.ds_predict(None, None, None, 1, None, None, None, 10, None, None, None) == -1
    assert L.ds_gather(None, None, None, None, None, 4, 0, None, None) == -1
    assert L.ds_net_create(None, None, C.byref(out)) == -1
    assert L.ds_lights_create(None, 1, None, None, C.byref(out)) == -1
    assert L.ds_render_mc_lights(None, None, None, None, None, None, 4, 1, 0, None, None) == -1
    assert L.ds_first_hits_lights(None, None, None, None, 1, None, None, 4, 0, 0, None, None,
                                  None, None, None, None) == -1
    assert L.ds_render_rpnn_lights(None, None, None, 1, None, None, 1, None, None, 4, 1, 0, 0,
                                   None, None, None, None) == -1
    assert L.ds_light_table(0, None, None, None) == -1
    assert L.ds_net_create_mlp(None, 1, 1, None, C.byref(out)) == -1
    assert L.ds_phase_create(None, 4, None, 0.0, C.byref(out)) == -1
    assert L.ds_phase_build(1, None, 0.0, None, None, None, None) == -1
    assert L.ds_phase_destroy(None) == 0
    assert ds.ds_net_param_count_mlp(10, [200] * 22 + [1]) == 1_294_801
    assert ds.ds_net_param_count_mlp(10, [400, 400, 200, 200, 200, 1]) == 1_222_001
    assert ds.ds_net_param_count_mlp(10, [200, 2]) == -1    # the output must be scalar
    assert ds.ds_net_param_count_mlp(0, [1]) == -1
    assert L.ds_lights_destroy(None) == 0
    # destroying NULL handles is a no-op
    assert L.ds_destroy(None) == 0 and L.ds_cloud_destroy(None) == 0 and L.ds_net_destroy(None) == 0


def test_create_without_a_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    out = C.c_void_p()
    st = ds.lib().ds_create(0, None, C.byref(out))
    assert st < 0 and ds.ds_last_error()
