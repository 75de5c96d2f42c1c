"""The C-ABI library loads and exports every function include/mpmc.h declares
(no compute calls: this runs without a GPU)."""
import ctypes

import numpy as np
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpmc.h")
LIB = os.path.join(ROOT, "paper_2402_00016_amd", "libmpmc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpmc_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ["mpmc_apply_M", "mpmc_gmres_poly", "mpmc_apply_poly", "mpmc_deflate",
              "mpmc_level_estimate", "mpmc_solve"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmpmc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmpmc.so not built")
def test_binding_declares_every_symbol():
    from paper_2402_00016_amd import mpmc
    assert set(declared_functions()) == set(mpmc._SIGS)


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2402_00016_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", src, flags=re.M), f
                assert "oracle/" not in src and "liboracle" not in src, f


def test_driver_identity_weights_match_oracle():
    from oracle import net as ON
    from paper_2402_00016_amd import driver, mpmc
    w = driver.net_identity_weights()
    assert w.size == mpmc.mpmc_net_n_params() == ON.n_params()
    assert np.array_equal(w, ON.identity_theta())


def test_sweep_relative_variance_definitions():
    """eq. 3 (ratio of configuration-averaged variances) and eq. 4 (base-10
    log average) on two configurations with hand-computed values."""
    from paper_2402_00016_amd import sweep
    per = [{"ns": 10.0, 4: 1.0}, {"ns": 1000.0, 4: 10.0}]
    row = sweep.summarize(per, [4])[0]
    assert abs(row["rel_var"] - (11.0 / 2) / (1010.0 / 2)) < 1e-15
    assert abs(row["log_avg_rel_var"] - 10 ** -1.5) < 1e-15
    assert abs(sweep.sample_var([1.0, 3.0]) - 2.0) < 1e-15
