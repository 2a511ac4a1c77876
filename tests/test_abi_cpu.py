"""CPU-side checks of the C ABI: the built library loads and exports every
function include/pifcm.h declares; no GPU computation is run."""
import ctypes as ct
import os

import numpy as np
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


# ------------------------------------------------- argument checks of the binding
class _NoLibrary:
    """Stands in for the loaded library: any call is a test failure marker."""

    def __getattr__(self, name):
        raise _Reached(name)


class _Reached(Exception):
    pass


@pytest.fixture()
def bare_ctx(monkeypatch):
    """A Context whose library refuses every call, with CPU tensors taken as
    device tensors, so the binding's own checks run without a GPU."""
    from paper_2002_01981_amd import abi
    monkeypatch.setattr(abi, "_is_device", lambda t: True)
    ctx = abi.Context.__new__(abi.Context)
    ctx.lib = _NoLibrary()
    ctx.h = None
    return ctx


def _vol(shape=(3, 4, 5)):
    import torch
    return torch.zeros(shape, dtype=torch.float32)


def _u(n, C=4, dtype=None):
    import torch
    return torch.zeros((n, C), dtype=dtype or torch.float32)


def test_binding_rejects_bad_buffers_before_the_library(bare_ctx):
    import torch

    from paper_2002_01981_amd import Params
    p = Params(C=4)
    x = _vol()
    n = x.numel()
    c = [0.1, 0.4, 0.6, 0.9]
    bad = [
        lambda: bare_ctx.ifcm_solve(x, p, 0.1, 0.2, c, U_in=_u(n - 1)),
        lambda: bare_ctx.ifcm_solve(x, p, 0.1, 0.2, c, U_in=_u(n, 3)),
        lambda: bare_ctx.ifcm_solve(x, p, 0.1, 0.2, c, U_out=_u(n + 1)),
        lambda: bare_ctx.ifcm_solve(x, p, 0.1, 0.2, c[:3]),
        lambda: bare_ctx.ifcm_solve(x, p, 0.1, 0.2, c, U_in=_u(n).t()),
        lambda: bare_ctx.ifcm_solve_noalloc(x, p, 0.1, 0.2, c, U_in=_u(n - 1)),
        lambda: bare_ctx.ifcm_solve_noalloc(x, p, 0.1, 0.2, c, U_out=_u(n + 1)),
        lambda: bare_ctx.ifcm_solve_slab(x, 0, 1, p, 0.1, 0.2, c, _u(2 * n)),
        lambda: bare_ctx.swarm_evaluate([x, x], p, np.zeros((3, 2)), np.zeros((2, 4)), [_u(n)]),
        lambda: bare_ctx.swarm_evaluate([x, x], p, np.zeros((3, 5, 2)), np.zeros((2, 4)),
                                        [_u(n), _u(n)]),
        lambda: bare_ctx.swarm_evaluate([x, x], p, np.zeros((2, 5, 3)), np.zeros((2, 4)),
                                        [_u(n), _u(n)]),
        lambda: bare_ctx.swarm_evaluate([x, _vol((2, 2, 2))], p, np.zeros((5, 2)),
                                        np.zeros((2, 4)), [_u(n), _u(n)]),
        lambda: bare_ctx.swarm_evaluate([x], p, np.zeros((5, 2)), np.zeros(3), [_u(n)]),
        lambda: bare_ctx.ifcm_backward(x, p, 0.1, 0.2, c, _u(n - 4), 5, 5),
        lambda: bare_ctx.pifcm_normalize(x, out=torch.zeros(n + 1)),
    ]
    for i, call in enumerate(bad):
        with pytest.raises(ValueError):
            call()
    for call in (lambda: bare_ctx.ifcm_solve(x, p, 0.1, 0.2, c, U_in=_u(n, dtype=torch.float64)),
                 lambda: bare_ctx.ifcm_backward(x, p, 0.1, 0.2, c, _u(n, dtype=torch.float16), 5, 5)):
        with pytest.raises(TypeError):
            call()


def test_binding_passes_well_formed_buffers_to_the_library(bare_ctx):
    """The same calls with consistent buffers reach the library."""
    from paper_2002_01981_amd import Params
    p = Params(C=4)
    x = _vol()
    y = _vol((2, 3, 7))
    c = [0.1, 0.4, 0.6, 0.9]
    good = [
        ("ifcm_solve", lambda: bare_ctx.ifcm_solve(x, p, 0.1, 0.2, c, U_in=_u(x.numel()))),
        ("ifcm_solve_slab", lambda: bare_ctx.ifcm_solve_slab(x, 0, 1, p, 0.1, 0.2, c, _u(x.numel()))),
        ("swarm_evaluate", lambda: bare_ctx.swarm_evaluate(
            [x, y], p, np.zeros((2, 5, 2)), np.zeros((2, 4)), [_u(x.numel()), _u(y.numel())])),
        ("ifcm_backward", lambda: bare_ctx.ifcm_backward(x, p, 0.1, 0.2, c, _u(x.numel()), 5, 5)),
    ]
    for name, call in good:
        with pytest.raises(_Reached) as e:
            call()
        assert str(e.value) == name
