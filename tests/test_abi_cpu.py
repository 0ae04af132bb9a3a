"""CPU checks of the C ABI: the library loads without a GPU and exports every entry point
that include/dss.h declares; the binding's parameter struct matches the header's layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dss.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dss_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("dss_create", "dss_set_particles", "dss_build_neighbours", "dss_compute_forces", "dss_step",
              "dss_read_stress", "dss_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2108_01013_amd import dss
    lib = dss.load_library()
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(dss.EXPORTS) == declared()


def test_status_strings_without_gpu():
    from paper_2108_01013_amd import dss
    lib = dss.load_library()
    assert lib.dss_status_string(0) == b"ok"
    assert lib.dss_status_string(3) == b"capacity exceeded"
    assert lib.dss_status_string(99) == b"unknown status"


def test_params_struct_layout():
    from paper_2108_01013_amd import dss
    # 3 + 15 doubles, 4 int32, then the 2 doubles of the rolling spring and 2 of the wave
    assert ctypes.sizeof(dss.Params) == 18 * 8 + 4 * 4 + 4 * 8
    assert dss.Params.precision.offset == 18 * 8
    assert dss.Params.k_roll.offset == 18 * 8 + 4 * 4
    assert ctypes.sizeof(dss.Tuning) == 2 * 8 + 6 * 4 and dss.Tuning.sized.offset == 24
    assert dss.Tuning.queue_cap.offset == 32 and dss.Tuning.adj_cap.offset == 36
    assert ctypes.sizeof(dss.Info) == 8 + 8 + 12 + 4 + 8 + 8 + 4 + 4 + 8


def test_create_rejects_bad_params_without_touching_the_device():
    from paper_2108_01013_amd import dss, synth
    lib = dss.load_library()
    p = dss.make_params(synth.default_params([10.0, 10.0, 10.0], dt=-1.0))
    h = ctypes.c_void_p()
    assert lib.dss_create(ctypes.byref(p), None, ctypes.byref(h)) == 1
    assert not h.value


def test_create_batch_rejects_mixed_physics_without_touching_the_device():
    from paper_2108_01013_amd import dss, synth
    lib = dss.load_library()
    a = synth.default_params([10.0, 10.0, 10.0])
    b = synth.default_params([12.0, 11.0, 13.0], shear_rate=3.0)      # allowed to differ
    c = synth.default_params([10.0, 10.0, 10.0], eta0=2.0)            # not allowed
    h = ctypes.c_void_p()
    arr = (dss.Params * 2)(dss.make_params(a), dss.make_params(c))
    assert lib.dss_create_batch(arr, 2, None, ctypes.byref(h)) == 1
    assert not h.value
    arr = (dss.Params * 2)(dss.make_params(a), dss.make_params(b))
    assert lib.dss_create_batch(arr, 0, None, ctypes.byref(h)) == 1
    assert ctypes.sizeof(dss.BoxInfo) == 8 + 8 + 12 + 4 + 8 + 8 + 4 + 4 + 24 + 8 + 8 + 8


@pytest.mark.parametrize("over", [dict(wave_amp=2.0, wave_n=0.5), dict(wave_amp=2.0, wave_n=0.0),
                                  dict(kr=-1.0), dict(mu_r=-0.1)])
def test_create_rejects_bad_extension_params_without_touching_the_device(over):
    from paper_2108_01013_amd import dss, synth
    lib = dss.load_library()
    p = dss.make_params(synth.default_params([10.0, 10.0, 10.0], **over))
    h = ctypes.c_void_p()
    assert lib.dss_create(ctypes.byref(p), None, ctypes.byref(h)) == 1
    assert not h.value
