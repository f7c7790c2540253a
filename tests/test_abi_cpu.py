"""Host-side checks of the C ABI that need no GPU: the library loads and exports every
function include/ibsn.h declares, and the binding declares the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibsn.h")
LIB = os.path.join(ROOT, "paper_2603_07156_amd", "libibsn.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ibsn_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared()
    for required in ("ibsn_solve", "ibsn_subproblem_eval", "ibsn_sparsify", "ibsn_hvp"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libibsn.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2603_07156_amd import ibsn
    assert sorted(ibsn.EXPORTS) == declared()


def test_no_oracle_import_in_product():
    """The product path never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2603_07156_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "ibsn_oracle" not in text, f
