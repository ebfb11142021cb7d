"""The C-ABI library loads, exports every entry point include/mkf.h
declares, and rejects bad arguments before touching the GPU.  CPU only: no
call here launches device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mkf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mkf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("mkf_create", "mkf_destroy", "mkf_load_geometry", "mkf_load_hits", "mkf_seed",
              "mkf_find", "mkf_get_tracks", "mkf_fit", "mkf_propagate", "mkf_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1811_04141_amd import mkf
    lib = C.CDLL(mkf.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(mkf.EXPORTS) == set(declared_functions())


def test_struct_layouts_match_header():
    from paper_1811_04141_amd import mkf
    # mkf_layer: 11 x 4 bytes; mkf_config: 6 floats, 2 ints, 6 floats, flags
    assert C.sizeof(mkf.Layer) == 44
    assert C.sizeof(mkf.Config) == 4 * (6 + 2 + 6 + 1)
    assert C.sizeof(mkf.Track) == 4 * 5 + 4 + 4 * 27 + 32 + 4 * 32
    # mkf_region: eta bounds, a count and MKF_MAX_PLAN layer ids
    assert C.sizeof(mkf.Region) == 4 * 3 + 4 * 32
    assert C.sizeof(mkf.MaterialInfo) == 4 * 6
    assert C.sizeof(mkf.Field) == 4 * 5
    # mkf_train_cfg: int64, 2 int32, float, padding, uint64, 7 floats, 2 int32
    assert C.sizeof(mkf.TrainCfg) == 72
    assert mkf.TrainCfg.first_step.offset == 60 and mkf.TrainCfg.n_steps.offset == 64


def test_host_side_argument_errors():
    from paper_1811_04141_amd import mkf
    from synth import FindConfig
    lib = mkf.lib
    h = C.c_void_p()
    assert lib.mkf_create(None, None, C.byref(h)) == mkf.MKF_E_ARG
    assert b"NULL" in lib.mkf_last_error(None)
    bad = mkf.make_config(FindConfig(n_cand=9))
    assert lib.mkf_create(C.byref(bad), None, C.byref(h)) == mkf.MKF_E_ARG
    bad = mkf.make_config(FindConfig(chi2_cut=-1.0))
    assert lib.mkf_create(C.byref(bad), None, C.byref(h)) == mkf.MKF_E_ARG
    bad = mkf.make_config(FindConfig(init_var=(1, 1, 1, 0, 1, 1)))
    assert lib.mkf_create(C.byref(bad), None, C.byref(h)) == mkf.MKF_E_ARG
    assert lib.mkf_create(C.byref(mkf.make_config(FindConfig())), None, None) == mkf.MKF_E_ARG
    bad = mkf.make_config(FindConfig(), flags=16)  # no such flag
    assert lib.mkf_create(C.byref(bad), None, C.byref(h)) == mkf.MKF_E_ARG
    assert b"flag" in lib.mkf_last_error(None)
    lib.mkf_destroy(None)  # NULL is accepted
    assert lib.mkf_find(None) == mkf.MKF_E_ARG
    assert lib.mkf_load_geometry(None, None, 0) == mkf.MKF_E_ARG
    assert lib.mkf_get_stats(None, None) == mkf.MKF_E_ARG
    assert lib.mkf_backward_fit(None, None, None, None, None) == mkf.MKF_E_ARG
    assert lib.mkf_smooth(None, None, None, None) == mkf.MKF_E_ARG
    assert lib.mkf_make_seeds(None, None, 0, None, None, None) == mkf.MKF_E_ARG
    assert lib.mkf_find_duplicates(None, 0.5, None, None) == mkf.MKF_E_ARG
    assert lib.mkf_clean_seeds(None, None, None, None) == mkf.MKF_E_ARG
    assert lib.mkf_load_steering(None, None, 0) == mkf.MKF_E_ARG
    assert lib.mkf_load_material(None, None, None, None) == mkf.MKF_E_ARG
    assert lib.mkf_load_field(None, None) == mkf.MKF_E_ARG


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib
    import paper_1811_04141_amd.mkf as m
    monkeypatch.setattr(m, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        m._load()
