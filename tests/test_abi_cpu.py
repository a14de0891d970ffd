"""CPU-side checks of the C ABI library: it loads, and it exports every
symbol that include/lbm.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2207_06043_amd", "liblbmib.so")
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:lbm|ib)_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2207_06043_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_every_declared_symbol():
    from paper_2207_06043_amd import EXPORTS
    assert sorted(EXPORTS) == _declared()


def test_product_path_has_no_fallback(monkeypatch, tmp_path):
    """Without the built library the package refuses to run."""
    import paper_2207_06043_amd._abi as abi
    monkeypatch.setattr(abi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(abi, "_lib", None)
    with pytest.raises(ImportError):
        abi.load_library()
