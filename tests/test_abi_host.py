"""CPU-only checks of the C ABI: the library loads, exports every declared
entry point, and rejects invalid configurations before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tvolap.h")
LIB = os.path.join(ROOT, "paper_2310_00319_amd", "libtvolap.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tvolap_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtvolap.so not built (run python -m paper_2310_00319_amd.build)")
    from paper_2310_00319_amd import _lib
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tvolap_create", "tvolap_set_ir", "tvolap_select_ir", "tvolap_process_block",
                     "tvolap_reset", "tvolap_destroy", "tvolap_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_declares_every_exported_symbol():
    from paper_2310_00319_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_functions()


def _cfg(**kw):
    from paper_2310_00319_amd._lib import TvolapConfig
    c = TvolapConfig()
    c.hop, c.n_channels, c.n_inputs, c.max_taps, c.n_slots, c.spectra_dtype = 128, 2, 2, 1000, 1, 0
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("kw,msg", [
    (dict(hop=100), "hop"),
    (dict(hop=32), "hop"),
    (dict(n_channels=0), ">= 1"),
    (dict(n_slots=0), ">= 1"),
    (dict(max_taps=0), ">= 1"),
    (dict(spectra_dtype=7), "spectra_dtype"),
    (dict(n_inputs=1), "n_inputs != n_channels"),
])
def test_create_rejects_invalid_config_without_device(lib, kw, msg):
    h = ctypes.c_void_p(1234)
    rc = lib.tvolap_create(ctypes.byref(_cfg(**kw)), ctypes.byref(h))
    assert rc == -1
    assert h.value is None
    assert msg in lib.tvolap_last_error(None).decode()


def test_create_rejects_bad_maps(lib):
    h = ctypes.c_void_p()
    bad_map = (ctypes.c_int32 * 2)(0, 5)
    cfg = _cfg(n_inputs=1)
    cfg.input_of_channel = ctypes.cast(bad_map, ctypes.POINTER(ctypes.c_int32))
    assert lib.tvolap_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    taps = (ctypes.c_int32 * 2)(10, 2000)
    cfg = _cfg()
    cfg.taps_of_channel = ctypes.cast(taps, ctypes.POINTER(ctypes.c_int32))
    assert lib.tvolap_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert "taps_of_channel" in lib.tvolap_last_error(None).decode()


@pytest.mark.parametrize("n_out,bus,msg", [
    (3, None, "n_outputs must be in"),
    (-1, None, "n_outputs must be in"),
    (1, None, "output_of_channel is NULL"),
    (2, (0, 2), "output_of_channel value out of range"),
    (2, (1, 1), "every output needs at least one channel"),
])
def test_create_rejects_bad_mixdown(lib, n_out, bus, msg):
    h = ctypes.c_void_p()
    cfg = _cfg(n_outputs=n_out)
    if bus is not None:
        arr = (ctypes.c_int32 * 2)(*bus)
        cfg.output_of_channel = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
    assert lib.tvolap_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert h.value is None
    assert msg in lib.tvolap_last_error(None).decode()


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.tvolap_create(None, ctypes.byref(h)) == -1
    assert lib.tvolap_create(ctypes.byref(_cfg()), None) == -1
    assert lib.tvolap_destroy(None) == 0
    assert lib.tvolap_process_block(None, None, 0, None, 0, None) == -1
    assert lib.tvolap_set_irs(None, 0, None, 1) == -1
    assert lib.tvolap_configure_batch(None, 0, 0, 0, 0, 0, 0) == -1
    assert lib.tvolap_version().decode().startswith("tvolap")


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2310_00319_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h", ".hpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f


def test_build_retries_a_failed_unit_once_then_reports(monkeypatch, tmp_path):
    """build(): a unit whose compile fails under the parallel pass is compiled
    once more on its own; a unit that fails twice raises."""
    from paper_2310_00319_amd import build as b
    calls = []

    def fake_run(cmd, verbose):
        calls.append(cmd[-1])
        name = os.path.basename(cmd[-1])
        if name == "tvolap_capi.o" and calls.count(cmd[-1]) == 1:
            raise RuntimeError("device compiler aborted")
        if name == "tvolap_dispatch.o" and fail_twice:
            raise RuntimeError("bad source")

    monkeypatch.setattr(b, "_run", fake_run)
    monkeypatch.setattr(b, "OBJ", str(tmp_path / "obj"))
    monkeypatch.setattr(b, "LIB", str(tmp_path / "lib.so"))
    monkeypatch.setattr(b.os, "replace", lambda a, c: None)
    fail_twice = False
    b.build(jobs=2)
    capi = [c for c in calls if c.endswith("tvolap_capi.o")]
    assert len(capi) == 2                                     # failed once, retried alone
    assert calls[-1].endswith("lib.so.tmp")                   # then linked
    calls.clear()
    fail_twice = True
    with pytest.raises(RuntimeError, match="bad source"):
        b.build(jobs=2)
    assert not any(c.endswith("lib.so.tmp") for c in calls)  # no link after a second failure
