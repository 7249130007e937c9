"""CPU-side checks of the C ABI library: it loads, exports every declared
symbol, and its host stencil builder reproduces the oracle's stencils."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2312_17042_amd import cteno as T
from paper_2312_17042_amd import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "cteno.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cteno_[a-z0-9_]+)\s*\(", src)) - {"cteno_alloc_fn", "cteno_free_fn"})


def test_library_exports_every_declared_symbol():
    L = T.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(T.exported_symbols())


def test_invalid_arguments_are_reported():
    m = W.split_jitter_mesh(8, 8, seed=1)
    sch = T.make_scheme(physics=T.EULER, degree=7)
    with pytest.raises(T.CtenoError) as e:
        T.stencils_host(m.xy, m.tri, m.box, m.bc, sch)
    assert e.value.status == T.ERR_INVALID
    bad = W.split_jitter_mesh(8, 8, seed=1)
    bad.xy = bad.xy.copy()
    bad.xy[bad.tri[0, 1]] = bad.xy[bad.tri[0, 0]]      # degenerate triangle
    with pytest.raises(T.CtenoError) as e:
        T.stencils_host(bad.xy, bad.tri, bad.box, bad.bc, T.make_scheme(physics=T.EULER, degree=3))
    assert e.value.status == T.ERR_MESH
    with pytest.raises(T.CtenoError) as e:                # empty mesh
        T.stencils_host(m.xy, m.tri[:0], m.box, m.bc, T.make_scheme(physics=T.EULER, degree=3))
    assert e.value.status == T.ERR_INVALID and "empty" in str(e.value)
    # beyond the cell limit (2^28, the inflow row field of a face code): the
    # descriptor claims that many cells over small arrays; the builder refuses
    # it before reading them, and the outputs may be NULL
    d = T.mesh_desc(m.xy, m.tri, m.box, m.bc)
    d.n_cells = 1 << 28
    with pytest.raises(T.CtenoError) as e:
        T._check(T.lib().cteno_stencils_host(ctypes.byref(d), ctypes.byref(T.make_scheme(physics=T.EULER, degree=3)),
                                             None, None, None))
    assert e.value.status == T.ERR_INVALID and "2^28" in str(e.value)


def test_inflow_data_is_checked():
    """Prescribed-state sides: unphysical states, unknown kinds and switches
    on periodic sides are refused before anything is built."""
    sch = T.make_scheme(physics=T.EULER, degree=3)
    m = W.split_jitter_mesh(8, 4, (0, 1, 0, 0.5), seed=1, bc=(T.INFLOW, 2, 1, 1))
    good = W.constant_inflow(W.prim_to_cons(1.0, 2.0, 0.0, 1.0))
    T.stencils_host(m.xy, m.tri, m.box, m.bc, sch, good)
    for bnd, bc in [(W.constant_inflow((1.0, 0.0, 0.0, -1.0)), m.bc),           # negative energy
                    (W.Boundary(), m.bc),                                      # zero density
                    (good, (4, 2, 1, 1)),                                      # unknown kind
                    (W.Boundary(behind=good.behind, ahead=good.ahead, split_kind=(0, 0, 5, 0)), m.bc)]:
        with pytest.raises(T.CtenoError) as e:
            T.stencils_host(m.xy, m.tri, m.box, bc, sch, bnd)
        assert e.value.status == T.ERR_INVALID
    per = W.split_jitter_mesh(8, 8, seed=1)
    sw = W.Boundary(split_kind=(W.WALL, 0, 0, 0), split_at=(0.5, 0, 0, 0))
    with pytest.raises(T.CtenoError) as e:
        T.stencils_host(per.xy, per.tri, per.box, per.bc, sch, sw)
    assert "periodic" in str(e.value)


@pytest.mark.parametrize("case", ["adv", "vortex", "sod", "r2", "sod_r4", "r5", "adv_r6"])
def test_host_stencils_equal_oracle(case):
    if case == "adv":
        m, deg, phys = W.split_jitter_mesh(20, 20, seed=1), 2, O.ADVECTION
    elif case == "vortex":
        m, deg, phys = W.split_jitter_mesh(40, 40, (0, 10, 0, 10), seed=2), 3, O.EULER
    elif case == "sod":
        m, deg, phys = W.split_jitter_mesh(40, 10, (0, 1, 0, 0.25), seed=3, bc=(2, 2, 1, 1)), 3, O.EULER
    elif case == "r2":
        m, deg, phys = W.split_jitter_mesh(12, 12, seed=4), 2, O.EULER
    elif case == "sod_r4":
        m, deg, phys = W.split_jitter_mesh(40, 10, (0, 1, 0, 0.25), seed=3, bc=(2, 2, 1, 1)), 4, O.EULER
    elif case == "r5":
        m, deg, phys = W.split_jitter_mesh(24, 24, seed=7), 5, O.EULER
    else:
        m, deg, phys = W.split_jitter_mesh(24, 24, seed=8), 6, O.ADVECTION
    o = O.Oracle.from_mesh(m, physics=phys, degree=deg)
    oc, od, on = o.stencils()
    lc, ld, ln = T.stencils_host(m.xy, m.tri, m.box, m.bc, T.make_scheme(physics=phys, degree=deg))
    assert np.array_equal(np.sort(oc, axis=1), lc)
    assert np.array_equal(on, ln)
    assert od.shape == ld.shape
    assert np.array_equal(od, ld)
