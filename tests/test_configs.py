"""The workload files under configs/ build the same instances as the
generators the tests and the benchmark use (CPU)."""

import os

import numpy as np
import pytest

import synthetic as S
from synthetic import config as C


def _same(a, b):
    assert a.n == b.n and a.beta == b.beta and a.hidden == b.hidden
    for f in ("edges", "J", "h", "width_set", "order"):
        assert np.array_equal(np.asarray(getattr(a, f)), np.asarray(getattr(b, f))), f
    assert (a.group_ptr is None) == (b.group_ptr is None)
    if a.group_ptr is not None:
        assert np.array_equal(a.group_ptr, b.group_ptr)


def test_every_config_loads():
    names = sorted(f[:-5] for f in os.listdir(C.CONFIG_DIR) if f.endswith(".json"))
    assert {"c1", "c2", "c3", "c4", "c5"} <= set(names)
    for name in names:
        cfg = C.load(name)
        assert cfg["name"] == name
        opts = C.net_options(cfg)
        assert opts["precision"] in ("fp64", "fp32", "bf16")
        if cfg["instances"][0]["kind"] not in ("rrg_planned", "mixed_batch"):
            insts, counts = C.instances(cfg)
            assert len(insts) == len(counts) and all(b > 0 for b in counts)


@pytest.mark.parametrize("name,want,B", [
    ("c1", lambda: [S.c1_small_lattice(16)], [1024]),
    ("c2", lambda: [S.c2_lattice(b, 256) for b in (0.5, 1.0, 2.0)], [8192] * 3),
    ("c3", lambda: [S.c3_sk(b, 128) for b in (0.5, 1.0, 1.5)], [2048] * 3),
    ("c4", lambda: [S.c4_rrg()], [4096]),
])
def test_configs_match_the_generators(name, want, B):
    insts, counts = C.instances(name)
    ref = want()
    assert counts == B and len(insts) == len(ref)
    for a, b in zip(insts, ref):
        _same(a, b)


def test_mixed_batch_config():
    # one instance of each of the seven kinds (the file asks for all 64)
    cfg = C.load("c5")
    assert cfg["instances"][0]["count"] == 64
    cfg["instances"][0]["count"] = 7
    insts, counts = C.instances(cfg)
    ref = S.mixed_batch_instances(7)
    assert counts == S.mixed_batch_sizes(ref)
    for a, b in zip(insts, ref):
        _same(a, b)
    assert C.net_options("c5")["flags"] == 8 | 4
