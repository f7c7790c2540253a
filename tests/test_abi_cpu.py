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
    text = re.sub(r"/\*.*?\*/", " ", open(HEADER).read(), flags=re.S)   # comments out
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



def test_struct_layouts_match_header(tmp_path):
    """sizeof and field offsets of the option and report structs, compiled from the header
    with the host C compiler, equal those of the ctypes binding."""
    import shutil
    import subprocess
    from paper_2603_07156_amd import ibsn
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    fields_o = [f for f, _ in ibsn.Options._fields_]
    fields_r = [f for f, _ in ibsn.Report._fields_]
    fields_t = [f for f, _ in ibsn.IterRecord._fields_]
    nl = "\\n"
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "ibsn.h"', "int main(void) {",
           f'printf("%zu %zu %zu{nl}", sizeof(ibsn_options), sizeof(ibsn_report), '
           'sizeof(ibsn_iter_record));']
    src += [f'printf("%zu{nl}", offsetof(ibsn_options, {f}));' for f in fields_o]
    src += [f'printf("%zu{nl}", offsetof(ibsn_report, {f}));' for f in fields_r]
    src += [f'printf("%zu{nl}", offsetof(ibsn_iter_record, {f}));' for f in fields_t]
    src += ["return 0; }"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", inc, str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    so, sr, stt = int(out[0]), int(out[1]), int(out[2])
    offs = [int(x) for x in out[3:]]
    assert so == ctypes.sizeof(ibsn.Options) and sr == ctypes.sizeof(ibsn.Report)
    assert stt == ctypes.sizeof(ibsn.IterRecord)
    no, nr = len(fields_o), len(fields_r)
    assert offs[:no] == [getattr(ibsn.Options, f).offset for f in fields_o]
    assert offs[no:no + nr] == [getattr(ibsn.Report, f).offset for f in fields_r]
    assert offs[no + nr:] == [getattr(ibsn.IterRecord, f).offset for f in fields_t]


def test_constants_match_header(tmp_path):
    """The binding's mode and kind constants equal the header's enumerators, compiled from
    the header with the host C compiler."""
    import shutil
    import subprocess
    from paper_2603_07156_amd import ibsn
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = {"IBSN_OK": ibsn.IBSN_OK, "IBSN_WARN_MAXITER": ibsn.IBSN_WARN_MAXITER,
             "IBSN_NOALLOC_MAX_M": ibsn.NOALLOC_MAX_M, "IBSN_COST_POINTS": ibsn.IBSN_COST_POINTS,
             "IBSN_PREC_F64": ibsn.PREC_F64, "IBSN_PREC_MIXED": ibsn.PREC_MIXED,
             "IBSN_CG_AUTO": ibsn.CG_AUTO, "IBSN_CG_LAUNCHES": ibsn.CG_LAUNCHES,
             "IBSN_CG_PERSISTENT": ibsn.CG_PERSISTENT, "IBSN_CG_SINGLE": ibsn.CG_SINGLE,
             "IBSN_CG_PIPE": ibsn.CG_PIPE, "IBSN_CSC_AUTO": ibsn.CSC_AUTO,
             "IBSN_CSC_ENTRY": ibsn.CSC_ENTRY, "IBSN_CSC_BLOCK": ibsn.CSC_BLOCK}
    nl = "\\n"
    src = ['#include <stdio.h>', '#include "ibsn.h"', "int main(void) {"]
    src += [f'printf("%lld{nl}", (long long)({k}));' for k in pairs]
    src += ["return 0; }"]
    c = tmp_path / "consts.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "consts"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert [int(x) for x in out] == list(pairs.values())
