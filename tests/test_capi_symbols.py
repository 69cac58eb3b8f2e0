"""The C-ABI library loads and exports every symbol include/*.h declares;
the Python binding wraps each of them (no compute calls: no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(mcv_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def libpath():
    path = os.path.join(ROOT, "paper_1811_09711_amd", "libmcv.so")
    if not os.path.exists(path):
        from paper_1811_09711_amd import build
        build.build()
    return path


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("mcv_create_integrator", "mcv_sample_iteration", "mcv_refine", "mcv_result",
                     "mcv_unweight", "mcv_destroy", "mcv_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(libpath):
    import torch  # noqa: F401  (same HIP runtime as the binding)
    lib = ctypes.CDLL(libpath)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_symbol(libpath):
    from paper_1811_09711_amd import mcv
    assert set(mcv._SIGNATURES) == set(_declared())
    assert mcv.lib().mcv_version().startswith(b"mcv")
    assert isinstance(mcv.lib().mcv_last_error(), bytes)  # "" or the last failure on this thread


def test_oracle_and_library_share_no_code():
    """The oracle is plain C with its own header; the HIP sources never
    include or import it and it never includes theirs."""
    csrc = os.path.join(ROOT, "paper_1811_09711_amd")
    for path in glob.glob(os.path.join(csrc, "**", "*"), recursive=True):
        if path.endswith((".hip", ".h", ".py", ".cpp")):
            text = open(path).read()
            assert "oracle" not in re.sub(r"(//|#).*", "", text).lower() or path.endswith("build.py"), path
    for path in glob.glob(os.path.join(ROOT, "oracle", "*")):
        if path.endswith((".c", ".h", ".py")):
            text = open(path).read()
            assert "paper_1811_09711_amd" not in text and "mcv_device" not in text, path
