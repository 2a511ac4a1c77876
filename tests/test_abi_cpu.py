"""CPU-side checks of the C ABI: the built library loads and exports every
function include/pifcm.h declares; no GPU computation is run."""
import ctypes as ct
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_boundary():
    from paper_2002_01981_amd import header_symbols
    names = header_symbols()
    for required in ("ifcm_solve", "swarm_evaluate", "ifcm_backward", "pifcm_create",
                     "pifcm_destroy", "pifcm_last_error", "pifcm_normalize", "pifcm_fcm_init",
                     "pifcm_tune", "pifcm_set_stream"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2002_01981_amd import header_symbols
    from paper_2002_01981_amd.abi import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.fail("libpifcm.so is not built (run python paper_2002_01981_amd/build.py)")
    lib = ct.CDLL(LIB_PATH)
    missing = [s for s in header_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_null_context_is_rejected_without_touching_a_gpu():
    from paper_2002_01981_amd.abi import PIFCM_E_INVALID, load_library
    lib = load_library()
    assert lib.pifcm_last_error(None) == b""
    assert lib.ifcm_solve(None, None, None, 0.0, 0.0, None, None, None, None, None, None, None,
                          None) == PIFCM_E_INVALID
    assert lib.swarm_evaluate(None, None, 0, None, None, 0, None, None, None, None, None,
                              0) == PIFCM_E_INVALID
    assert lib.pifcm_create(0, None, None) == PIFCM_E_INVALID


def test_product_does_not_reference_the_oracle():
    """The product package and its C sources never import, include or load
    the oracle."""
    pkg = os.path.join(ROOT, "paper_2002_01981_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "pifcm_oracle" not in text and "liboracle" not in text, f


def test_build_entry_reaches_both_build_functions(monkeypatch):
    """__graft_entry__.build() calls the oracle's and the library's build
    functions (stubbed here so that nothing is compiled)."""
    import importlib
    import sys

    sys.path.insert(0, ROOT)
    entry = importlib.import_module("__graft_entry__")
    calls = []
    monkeypatch.setattr(importlib.import_module("oracle.build"), "build",
                        lambda *a, **k: calls.append("oracle"))
    monkeypatch.setattr(importlib.import_module("paper_2002_01981_amd.build"), "build",
                        lambda *a, **k: calls.append("lib"))
    entry.build()
    assert calls == ["oracle", "lib"]
