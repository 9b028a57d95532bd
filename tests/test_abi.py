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


def test_system_resolve_against_the_oracle(built):
    """Row a1 through the C ABI, on the CPU: qcams_system_resolve converts
    masses in atomic mass units to electron masses, the LJ pair given by its
    depth and minimum (eps, r_m) to (Cn, Cm) and the Morse pair given by its
    harmonic frequency to its range parameter, as the oracle's own
    conversions do (CODATA 2018 mass unit; Sec. 3.1-3.2)."""
    import oracle as orc
    import qcams_workloads as W
    mixed = W.mixed_system()
    hh = W.Pair("morse", {"De": 0.1745, "re": 1.40, "we": 0.0200749568})
    cah = W.Pair("morse", {"De": 0.0625, "re": 3.78, "alpha": 0.62})
    h2ca_we = W.System((1.008, 1.008, 40.078), (hh, cah, hh), "H2+Ca, Morse by w_e")
    for system in (mixed, W.h2ca_system(), h2ca_we):
        r = Q.resolve_system(system)
        o = orc.make_system(system)
        assert r.mass_unit == Q.MASS_ME
        for i in range(3):
            assert r.mass[i] == pytest.approx(o.mass[i], rel=1e-15)
            assert r.pair[i].kind == o.pair[i].kind
            assert (r.pair[i].n, r.pair[i].m) == (o.pair[i].n, o.pair[i].m)
            for k in range(3):
                assert r.pair[i].p[k] == pytest.approx(o.pair[i].p[k], rel=1e-14), (i, k)
    # the mixed surface's LJ 12-6 pair (eps 0.02, r_m 4): C12 = 335544.32, C6 = 163.84
    r = Q.resolve_system(mixed)
    assert r.pair[0].p[0] == pytest.approx(335544.32, rel=1e-15)
    assert r.pair[0].p[1] == pytest.approx(163.84, rel=1e-15)
    # electron masses pass through unchanged
    r = Q.resolve_system(mixed, masses_me=[1.0, 2.0, 3.0])
    assert list(r.mass) == [1.0, 2.0, 3.0]


def test_system_resolve_rejects_bad_input(built):
    import qcams_workloads as W
    s = Q.make_system(W.h2ca_system())
    s.mass_unit = 7
    out = Q.System()
    assert Q.lib().qcams_system_resolve(C.byref(s), C.byref(out)) == Q.EINVAL
    assert b"unit" in Q.lib().qcams_last_error(None)
    bad = W.System((1.0, 1.0, 1.0), (W.Pair("lj", {"n": 6, "m": 12, "eps": 0.1, "rm": 3.0}),) * 3)
    with pytest.raises(Q.QcamsError, match="LJ"):
        Q.resolve_system(bad)
    with pytest.raises(Q.QcamsError, match="mass"):
        Q.resolve_system(W.h2ca_system(), masses_me=[1.0, -2.0, 3.0])


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
