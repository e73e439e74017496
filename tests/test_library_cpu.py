"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point the header declares, compiles the workloads' programs and
rejects malformed instances before touching a device."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import synthetic as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2504_12037_amd import _lib as L
    return L


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = L.lib()
    hdr = open(os.path.join(ROOT, "include", "tnvan.h")).read()
    declared = set(re.findall(r"\b(tnvan_[a-z_]+)\s*\(", hdr))
    assert len(declared) >= 13
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(L.EXPORTS)


def test_plan_statistics_of_the_workloads():
    L = _lib()
    c1 = L.plan(S.c1_small_lattice())
    assert c1[0] == 8 and c1[1] == 2 and c1[4] == 4 and c1[5] == 12
    c2 = L.plan(S.c2_lattice())
    # three strips of 16 rows, row-transfer messages over <= 5 spins
    assert c2[0] == 48 and c2[1] == 5 and c2[4] == 32 and c2[5] == 224
    c3 = L.plan(S.c3_sk())
    assert c3[0] == 2 and c3[1] == 8 and c3[4] == 48 and c3[5] == 16
    c4 = L.plan(S.c4_rrg())
    assert c4[1] <= 10 and c4[4] + c4[5] == 256


def _build(inst, max_width=14):
    L = _lib()
    keep = []
    c = L.make_cinstance(inst, keep)
    opt = L.COptions(1, max_width, 1, 0, 0)
    h = C.c_void_p()
    code = L.lib().tnvan_build_network(C.byref(c), 1, C.byref(opt), C.byref(h))
    return code, L.lib().tnvan_last_error().decode()


def _mod(inst, **kw):
    d = dict(n=inst.n, edges=inst.edges, J=inst.J, h=inst.h, beta=inst.beta,
             width_set=inst.width_set, order=inst.order, group_ptr=inst.group_ptr,
             hidden=inst.hidden)
    d.update(kw)
    return S.Instance(**d)


@pytest.mark.parametrize("case", ["dup_edge", "self_loop", "order_overlap",
                                  "not_partition", "nan_J", "neg_beta",
                                  "nan_h", "bad_groups", "big_group"])
def test_invalid_instances_are_rejected(case):
    base = S.c1_small_lattice()
    if case == "dup_edge":
        inst = _mod(base, edges=np.vstack([base.edges, base.edges[:1]]),
                    J=np.append(base.J, 0.5))
    elif case == "self_loop":
        inst = _mod(base, edges=np.vstack([base.edges, [[3, 3]]]), J=np.append(base.J, 1.0))
    elif case == "order_overlap":
        o = base.order.copy()
        o[0] = base.width_set[0]
        inst = _mod(base, order=o)
    elif case == "not_partition":
        inst = _mod(base, order=base.order[:-1], group_ptr=None)
    elif case == "nan_J":
        J = base.J.copy()
        J[2] = np.nan
        inst = _mod(base, J=J)
    elif case == "neg_beta":
        inst = _mod(base, beta=-1.0)
    elif case == "nan_h":
        h = base.h.copy()
        h[0] = np.inf
        inst = _mod(base, h=h)
    elif case == "bad_groups":
        inst = _mod(base, group_ptr=np.array([0, 5, 11], np.int32))
    else:
        inst = _mod(base, group_ptr=np.array([0, 12], np.int32))
    code, msg = _build(inst)
    assert code == 1, (code, msg)
    assert msg


def test_width_limit_is_enforced():
    inst = S.c4_rrg()
    code, msg = _build(inst, max_width=6)
    assert code == 2 and "width" in msg


def test_grouped_step_with_foreign_inputs_is_rejected():
    # single-spin elimination of a ladder, but grouped two-by-two across rungs
    base = S.lattice_2d(4, seed=0)
    inst = S.lattice_column_split(base, [2], row_groups=False)
    gp = np.array([0, 2, 4] + list(range(5, 13)), np.int32)
    code, msg = _build(_mod(inst, group_ptr=gp))
    assert code == 1 and "group" in msg
