"""Host-side checks of the C ABI: the library loads and exports every symbol
include/qcams.h declares, and the binding's ctypes layouts equal the header's
C layouts (compiled here with gcc).  No GPU calls."""
import ctypes as C
import os
import subprocess
import tempfile

import pytest

import paper_2304_02731_amd as Q
from paper_2304_02731_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def built():
    if B.is_stale():
        B.build()
    return Q.LIB_PATH


def test_exports_every_declared_symbol(built):
    names = Q.exported_names()
    for must in ("qcams_init_conditions", "qcams_propagate", "qcams_classify",
                 "qcams_cross_sections", "qcams_create", "qcams_levels"):
        assert must in names
    lib = C.CDLL(built)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True).stdout
    defined = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(names) <= defined


def test_struct_layouts_match_header():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "qcams.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(qcams_pair), sizeof(qcams_system),
         sizeof(qcams_params), sizeof(qcams_instance), sizeof(qcams_state), sizeof(qcams_outcome));
  printf("%zu %zu %zu %zu\n", offsetof(qcams_params, fixed_step), offsetof(qcams_params, max_steps),
         offsetof(qcams_instance, n_traj), offsetof(qcams_instance, seed));
  printf("%d %d %d %d\n", QCAMS_NF, QCAMS_NS, QCAMS_XS_STRIDE, QCAMS_VMAX);
  return 0; }
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        lines = subprocess.check_output([exe], text=True).split("\n")
    sizes = [int(x) for x in lines[0].split()]
    assert sizes == [C.sizeof(Q.Pair), C.sizeof(Q.System), C.sizeof(Q.Params),
                     C.sizeof(Q.Instance), C.sizeof(Q.StateC), C.sizeof(Q.OutcomeC)]
    offs = [int(x) for x in lines[1].split()]
    assert offs == [Q.Params.fixed_step.offset, Q.Params.max_steps.offset,
                    Q.Instance.n_traj.offset, Q.Instance.seed.offset]
    assert [int(x) for x in lines[2].split()] == [Q.NF, Q.NS, Q.XS_STRIDE, Q.VMAX]


def test_header_documents_each_call():
    """Every declared entry point carries a comment block with its contract."""
    txt = open(os.path.join(ROOT, "include", "qcams.h")).read()
    import re
    for n in Q.exported_names():
        m = re.search(r"^(int|void|const char \*)\s*" + n + r"\(", txt, flags=re.M)
        assert m, n
        before = txt[:m.start()].rstrip()
        assert before.endswith("*/"), n


def test_binding_refuses_without_library(monkeypatch):
    """No CPU fallback: the binding raises when the library is absent."""
    monkeypatch.setattr(Q.qcams, "LIB_PATH", "/nonexistent/libqcams.so")
    monkeypatch.setattr(Q.qcams, "_lib", None)
    with pytest.raises(Q.QcamsError):
        Q.qcams.lib()
