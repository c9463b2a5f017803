"""CPU tests of the native library: exported symbols, argument validation and
structure parity (host hierarchy of libdh2 vs the oracle, bit-exact)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle.structure import build_structure
from paper_1809_04384_amd import dh2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = dh2.load()
    header = open(os.path.join(ROOT, "include", "dh2.h")).read()
    declared = set(re.findall(r"\b(dh2_[a-z_]+)\s*\(", header))
    assert declared == set(dh2.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name


def test_batch_entry_points_reject_bad_arguments_without_gpu():
    import ctypes
    lib = dh2.load()
    b = ctypes.c_void_p()
    assert lib.dh2_batch_create(None, None, None, 1, 0, None, ctypes.byref(b)) == 1
    assert b.value is None
    assert lib.dh2_batch_create(None, None, None, 1, 1, None, None) == 1
    assert lib.dh2_batch_run(None) == 1
    lib.dh2_batch_free(None)


def test_build_many_rejects_bad_arguments_without_gpu():
    import ctypes
    lib = dh2.load()
    out = (ctypes.c_void_p * 2)()
    assert lib.dh2_build_many(0, None, None, None, None, None, None, None, 0, out) == 1
    assert lib.dh2_build_many(2, None, None, None, None, None, None, None, 0, out) == 1
    assert out[0] is None and out[1] is None


def test_build_rejects_bad_arguments_without_gpu():
    V, T = synth.sphere_octahedral(2)
    bad = [dict(kappa=-1.0), dict(order=0), dict(eta=0.0), dict(leafsize=0), dict(tol=-1.0)]
    base = dict(kappa=1.0, order=3, eta=1.0, leafsize=8, tol=1e-6)
    for b in bad:
        p = dict(base, **b)
        with pytest.raises(dh2.Dh2Error) as e:
            dh2.Handle(V, T, p["kappa"], p["order"], p["eta"], p["leafsize"], p["tol"])
        assert e.value.status == 1
    # unknown precision / norm codes are rejected before any device work
    for kw in (dict(precision=7), dict(norm=5), dict(norm=-1)):
        with pytest.raises(dh2.Dh2Error) as e:
            dh2.Handle(V, T, 1.0, 3, 1.0, 8, 1e-6, **kw)
        assert e.value.status == 1
    T2 = T.copy()
    T2[3, 1] = len(V) + 5
    with pytest.raises(dh2.Dh2Error) as e:
        dh2.Handle(V, T2, 1.0, 3, 1.0, 8, 1e-6)
    assert e.value.status == 2
    T3 = T.copy()
    T3[0, 1] = T3[0, 0]
    with pytest.raises(dh2.Dh2Error) as e:
        dh2.Plan(V, T3, 1.0, 3, 1.0, 8)
    assert e.value.status == 2


@pytest.mark.parametrize("name", ["dir512", "sphere2k", "dir2k", "cube768", "cube1200dir"])
def test_structure_parity_with_oracle(name):
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    st = build_structure(V, T, w.kappa, w.eta, w.leaf, w.eta1)
    ex = dh2.Plan(V, T, w.kappa, w.order, w.eta, w.leaf, w.eta1).export()
    assert np.array_equal(ex["perm"], st.perm)
    assert np.array_equal(ex["first"], st.first)
    assert np.array_equal(ex["size"], st.size)
    assert np.array_equal(ex["level"], st.level)
    assert np.array_equal(ex["parent"], st.parent)
    assert np.array_equal(ex["box"][:, :3], st.lo) and np.array_equal(ex["box"][:, 3:], st.hi)
    nd = [len(d) for d in st.dirs]
    assert ex["level_ndirs"].tolist() == nd
    assert np.array_equal(ex["dirs"], np.vstack(st.dirs))
    off = 0
    for l in range(st.depth + 1):
        sd = ex["sd"][off:off + nd[l]]
        if l < st.depth:
            assert np.array_equal(sd, st.sd[l])
        off += nd[l]
    assert [tuple(r) for r in ex["adm"].tolist()] == [tuple(map(int, a)) for a in st.adm]
    assert [tuple(r) for r in ex["near"].tolist()] == [tuple(map(int, a)) for a in st.near]


@pytest.mark.slow
def test_structure_parity_sphere32k():
    w = synth.WORKLOADS["sphere32k"]
    V, T = synth.make_mesh(w)
    st = build_structure(V, T, w.kappa, w.eta, w.leaf, w.eta1)
    ex = dh2.Plan(V, T, w.kappa, w.order, w.eta, w.leaf, w.eta1).export()
    assert np.array_equal(ex["perm"], st.perm)
    assert [tuple(r) for r in ex["adm"].tolist()] == [tuple(map(int, a)) for a in st.adm]
    assert [tuple(r) for r in ex["near"].tolist()] == [tuple(map(int, a)) for a in st.near]


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of dh2_options and dh2_stats have the sizes and field
    offsets of the C declarations (compiled here with the host compiler)."""
    import subprocess
    fields_s = [f for f, _ in dh2.Stats._fields_]
    fields_o = [f for f, _ in dh2.Options._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "dh2.h"', "int main(void) {",
           'printf("%zu %zu\\n", sizeof(dh2_stats), sizeof(dh2_options));']
    for f in fields_s:
        src.append('printf("s %s %%zu\\n", offsetof(dh2_stats, %s));' % (f, f))
    for f in fields_o:
        src.append('printf("o %s %%zu\\n", offsetof(dh2_options, %s));' % (f, f))
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, stdout=subprocess.PIPE, text=True).stdout.split("\n")
    size_s, size_o = map(int, out[0].split())
    assert size_s == ctypes.sizeof(dh2.Stats)
    assert size_o == ctypes.sizeof(dh2.Options)
    for line in out[1:]:
        if not line:
            continue
        kind, name, off = line.split()
        cls = dh2.Stats if kind == "s" else dh2.Options
        assert getattr(cls, name).offset == int(off), (kind, name)
