"""The C ABI library builds, loads, exports every symbol include/pm_nu.h declares, and
rejects bad arguments on the host (CPU; no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_1209_0461_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pm_nu.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_nu_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1209_0461_amd import build
        build.build()
    return binding.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), f"{n} declared in pm_nu.h but not exported"


def test_binding_covers_the_header():
    assert set(_declared()) == set(binding.SIGNATURES)


def test_default_config(lib):
    cfg = binding.pm_nu_default_config()
    assert (cfg.n_mesh, cfg.n_boxes, cfg.n_kbins, cfg.substeps, cfg.iterations) == (32, 1, 32, 8, 1)
    assert cfg.deconvolve == 1 and cfg.n_species == 3 and cfg.omega_m == 0.3


@pytest.mark.parametrize("field,value", [("n_mesh", 100), ("n_mesh", 1024), ("n_mesh", 4),
                                         ("n_kbins", 0), ("n_kbins", 1025), ("substeps", 0),
                                         ("box_size", -1.0), ("max_history", 1),
                                         ("response_mode", 5), ("n_particles", 0),
                                         ("iterations", 0)])
def test_bad_config_is_rejected_before_touching_a_device(lib, field, value):
    cfg = binding.pm_nu_default_config()
    setattr(cfg, field, value)
    with pytest.raises(binding.PMNuError) as e:
        binding.pm_nu_init(cfg, [0.3])
    assert e.value.code == -1
    assert field.split("_")[-1] in str(e.value) or "must" in str(e.value)


def test_null_context_is_an_error(lib):
    assert lib.pm_nu_deposit(None, None) == -1
    assert lib.pm_nu_response(None, 1.0) == -1
    assert b"NULL" in lib.pm_nu_last_error()
    # the switches between fused and separate FFT passes, like every other setter
    for setter in (lib.pm_nu_set_forward_zy, lib.pm_nu_set_inverse_xy, lib.pm_nu_set_inverse_yz,
                   lib.pm_nu_set_keep_density):
        assert setter(None, 1) == -1
    lib.pm_nu_destroy(None)   # ignored


def test_blob_size(lib):
    assert binding.pm_nu_surrogate_blob_floats() == 35329 + 4 * 16 + 2


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        binding.load_library(str(tmp_path / "nope.so"))
