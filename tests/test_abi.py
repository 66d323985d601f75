"""The C-ABI library builds, loads and exports every symbol include/tkc.h
declares.  No compute call runs here (no GPU in the CPU suite)."""
import os
import re
import subprocess

import pytest

from conftest import ROOT, hip_available

HEADER = os.path.join(ROOT, "include", "tkc.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tkc_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["tkc_ctx_create", "tkc_graph_upload", "tkc_topk_closeness", "tkc_graph_free",
                 "tkc_server_create", "tkc_server_submit", "tkc_server_result", "tkc_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1704_01077_amd import tkc
    out = subprocess.run(["nm", "-D", "--defined-only", tkc.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (tkc_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    assert set(tkc.EXPORTS) == set(declared())


def test_binding_names_match_abi():
    from paper_1704_01077_amd import tkc
    for n in declared():
        assert hasattr(tkc, n), n
    assert tkc.tkc_version().startswith("tkc")


def test_header_compiles_as_c():
    src = '#include "tkc.h"\nint main(void){ tkc_stats s; (void)s; return TKC_OK; }\n'
    r = subprocess.run(["gcc", "-x", "c", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                        "-fsyntax-only", "-"], input=src, text=True, capture_output=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.skipif(hip_available(), reason="checks the no-device error path")
def test_no_device_is_a_clean_error():
    from paper_1704_01077_amd import tkc
    with pytest.raises(tkc.TkcError) as e:
        tkc.tkc_ctx_create(0, None)
    assert e.value.code == tkc.TKC_EDEVICE


@pytest.mark.parametrize("struct", ["tkc_stats", "tkc_tuning"])
def test_struct_layout_matches_header(struct):
    """sizeof and every field offset seen by C equal the ctypes mirror."""
    from paper_1704_01077_amd import tkc
    import ctypes
    mirror = getattr(tkc, struct)
    fields = [f for f, _ in mirror._fields_]
    body = 'printf("%zu", sizeof({s}));'.format(s=struct)
    body += "".join(' printf(" %zu", offsetof({s}, {f}));'.format(s=struct, f=f) for f in fields)
    src = ('#include <stdio.h>\n#include <stddef.h>\n#include "tkc.h"\n'
           'int main(void){ %s return 0; }\n' % body)
    exe = "/tmp/tkc_sizeof_%s_%d" % (struct, os.getpid())
    subprocess.run(["gcc", "-x", "c", "-I", os.path.dirname(HEADER), "-o", exe, "-"], input=src, text=True,
                   check=True)
    out = [int(x) for x in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    os.unlink(exe)
    assert out[0] == ctypes.sizeof(mirror)
    assert out[1:] == [getattr(mirror, f).offset for f in fields]


def test_missing_library_fails_loudly(tmp_path):
    """Without libtkc.so the binding refuses to import: there is no other
    path to an answer."""
    import shutil
    import sys
    pkg = tmp_path / "paper_1704_01077_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1704_01077_amd", "tkc.py"), pkg / "tkc.py")
    (pkg / "__init__.py").write_text("")
    p = subprocess.run([sys.executable, "-c", "import paper_1704_01077_amd.tkc"], cwd=str(tmp_path),
                       capture_output=True, text=True)
    assert p.returncode != 0
    assert "ImportError" in p.stderr and "libtkc.so is not built" in p.stderr


def test_product_never_reaches_the_oracle():
    """The package (binding, build script, HIP and C++ sources) names no part
    of the oracle: no import, no include, no library, no fallback."""
    pkg = os.path.join(ROOT, "paper_1704_01077_amd")
    pat = re.compile(r"\boracle\b|liboracle|oracle_[a-z]+\(")
    hits = []
    for d, _, files in os.walk(pkg):
        if "_build" in d or "__pycache__" in d:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                for i, line in enumerate(open(os.path.join(d, f)), 1):
                    if pat.search(line):
                        hits.append("%s:%d: %s" % (f, i, line.strip()))
    assert not hits, hits
