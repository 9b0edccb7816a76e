"""The C-ABI library on the host (no GPU): it loads, exports every symbol that
include/fnlh.h declares, validates meshes and options, and builds valid colour orderings
and permutations."""
import os
import re

import numpy as np
import pytest

from oracle import ordering
from paper_2404_01407_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    from paper_2404_01407_amd import fnlh
    return fnlh


def test_exports_every_declared_symbol(F):
    hdr = open(os.path.join(ROOT, "include", "fnlh.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"\b(fnlh_[a-z_0-9]+)\s*\(", hdr))
    assert {"fnlh_create", "fnlh_relax", "fnlh_residual", "fnlh_assemble_jacobian", "fnlh_set_harmonics"} <= names
    for n in sorted(names):
        assert hasattr(F.LIB, n), n
    assert "gfx950" in F.version()


def test_struct_layouts_match_header(F, tmp_path):
    """Size and every field offset of the ctypes mirrors equal what a C compiler makes
    of include/fnlh.h."""
    import ctypes as C
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"fnlh_mesh": F.Mesh, "fnlh_options": F.Options, "fnlh_relax_opts": F.RelaxOpts,
               "fnlh_sys_report": F.Report, "fnlh_kernel_stats": F.KernelStats,
               "fnlh_gmres_opts": F.GmresOpts, "fnlh_gmres_report": F.GmresReport,
               "fnlh_tune_result": F.TuneResult}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fnlh.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ['  printf("params %d\\n", (int)FNLH_NN_PARAMS);', "  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            *key, val = ln.split()
            got[" ".join(key)] = int(val)
    for cname, py in structs.items():
        assert got[f"{cname} size"] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[f"{cname} {fname}"] == getattr(py, fname).offset, (cname, fname)
    assert got["params"] == F.NN_PARAMS


@pytest.mark.parametrize("shape", [(16, 8, 4), (7, 5, 3), (3, 2, 2)])
def test_bipartite_ordering_and_permutation(F, shape):
    m = synth.passage_block(*shape, 36, seed=2)
    col, perm, nc = F.order_mesh(m)
    assert nc == 2 and ordering.is_valid(col, m.edges)
    n = m.n_cells
    # colour-major internal numbering: each colour starts on a 64-row boundary
    assert len(np.unique(perm)) == n
    for c in range(nc):
        rows = np.sort(perm[col == c])
        assert rows[-1] - rows[0] + 1 == rows.size
        assert rows[0] % 64 == 0
    assert perm[col == 0].max() < perm[col == 1].min()


def test_greedy_ordering_with_triangles(F):
    m = synth.multi_row(6, 8, 4, n_blades=(36, 60, 48), seed=5)
    col, perm, nc = F.order_mesh(m)
    assert nc >= 3 and ordering.is_valid(col, m.edges)
    with pytest.raises(F.FnlhError) as e:
        F.order_mesh(m, ordering="bipartite")
    assert e.value.code == F.E_MESH


def test_user_ordering(F):
    m = synth.chain(10)
    nat = np.arange(10)
    col, perm, nc = F.order_mesh(m, ordering="user", user_colour=nat)
    assert nc == 10 and np.array_equal(col, nat)
    bad = np.zeros(10, np.int32)
    with pytest.raises(F.FnlhError) as e:
        F.order_mesh(m, ordering="user", user_colour=bad)
    assert e.value.code == F.E_MESH


def test_ordering_deterministic(F):
    m = synth.passage_block(9, 7, 5, 36, seed=4)
    a = F.order_mesh(m)
    b = F.order_mesh(m)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _bad(m, **kw):
    for k, v in kw.items():
        setattr(m, k, v)
    return m


@pytest.mark.parametrize("mutate,code", [
    ("self_loop", -2), ("out_of_range", -2), ("duplicate", -2), ("volume", -2), ("zone", -2),
    ("bface", -2), ("nan_area", -2),
])
def test_mesh_validation(F, mutate, code):
    m = synth.passage_block(4, 3, 2, 36, seed=1)
    if mutate == "self_loop":
        m.edges[3, 1] = m.edges[3, 0]
    elif mutate == "out_of_range":
        m.edges[5, 0] = m.n_cells
    elif mutate == "duplicate":
        m.edges = np.concatenate([m.edges, m.edges[2:3, ::-1]])
        m.area = np.concatenate([m.area, -m.area[2:3]])
    elif mutate == "volume":
        m.volume[7] = 0.0
    elif mutate == "zone":
        m.zone[1] = 5
    elif mutate == "bface":
        m.bface_cell[0] = -1
    elif mutate == "nan_area":
        m.area[0, 1] = np.nan
    with pytest.raises(F.FnlhError) as e:
        F.order_mesh(m)
    assert e.value.code == code


def test_create_rejects_bad_mesh_before_touching_device(F):
    m = synth.passage_block(4, 3, 2, 36, seed=1)
    m.volume[0] = -1.0
    with pytest.raises(F.FnlhError) as e:
        F.Context(m)
    assert e.value.code == F.E_MESH
    assert "volume" in str(e.value)


def test_bad_options(F):
    import ctypes as C
    m = synth.passage_block(4, 3, 2, 36, seed=1)
    arrs = F._MeshArrays(m)
    o = F.Options(7, 0, 0, 0, None, 0, 0)
    rc = F.LIB.fnlh_order_mesh(C.byref(arrs.s), C.byref(o), None, None, None)
    assert rc == F.E_ARG
    o = F.Options(0, 0, 3, 0, None, 0, 0)   # USER without colours
    assert F.LIB.fnlh_order_mesh(C.byref(arrs.s), C.byref(o), None, None, None) == F.E_ARG
