"""Workload files: configs/<name>.json -> instances, sample counts and net
options.

A file names the instances (kind and generator parameters, all seeded), the
samples per instance, the precision and flags of the net and the training
settings of Algorithm 1.  This module only reads them and calls the seeded
generators of this package (and, for planned instances, the library's
width-set planner); it holds none of the method's arithmetic.
"""

from __future__ import annotations

import json
import os
from typing import List, Tuple

import numpy as np

from . import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CONFIG_DIR = os.path.join(ROOT, "configs")


def config_path(name: str) -> str:
    return name if name.endswith(".json") else os.path.join(CONFIG_DIR, name + ".json")


def load(name: str) -> dict:
    with open(config_path(name)) as f:
        return json.load(f)


def _instance(spec: dict) -> List[I.Instance]:
    kind = spec["kind"]
    if kind == "lattice":
        beta = spec["beta"]
        if beta == "critical":
            beta = 0.5 * float(np.log(1.0 + np.sqrt(2.0)))
        base = I.lattice_2d(spec["L"], seed=spec["seed"], beta=float(beta),
                            ferro=bool(spec.get("ferro", False)),
                            h_var=float(spec.get("h_var", 0.0)))
        return [I.lattice_column_split(base, spec["width_columns"], hidden=spec.get("hidden", 0))]
    if kind == "sk":
        return [I.sherrington_kirkpatrick(spec["n"], seed=spec["seed"], beta=float(spec["beta"]),
                                          n_width=spec["n_width"],
                                          group_size=spec["group_size"],
                                          hidden=spec.get("hidden", 0))]
    if kind == "rrg":
        return [I.random_regular(spec["n"], spec["d"], seed=spec["seed"], beta=float(spec["beta"]),
                                 h_var=float(spec["h_var"]), width_limit=spec["width_limit"],
                                 hidden=spec.get("hidden", 0))]
    if kind == "mixed_batch":
        return I.mixed_batch_instances(spec["count"], hidden=spec["hidden"],
                                       base_seed=spec["base_seed"])
    if kind == "rrg_planned":
        from paper_2504_12037_amd import plan_width_set
        e = I.random_regular_edges(spec["n"], spec["d"], np.random.default_rng(spec["graph_seed"]))
        W, order, _, _ = plan_width_set(spec["n"], e, spec["w_u"])
        J = np.random.default_rng(spec["coupling_seed"]).choice([-1.0, 1.0], len(e))
        h = np.random.default_rng(spec["field_seed"]).normal(0.0, np.sqrt(spec["h_var"]), spec["n"])
        return [I.Instance(spec["n"], e.astype(np.int32), J, h, float(spec["beta"]),
                           W.astype(np.int32), order.astype(np.int32), None,
                           spec.get("hidden", 0), f"rrg{spec['n']}_wu{spec['w_u']}")]
    raise ValueError(f"unknown instance kind {kind!r}")


def instances(cfg) -> Tuple[List[I.Instance], List[int]]:
    """(instances, samples per instance) of a config (dict or name)."""
    if isinstance(cfg, str):
        cfg = load(cfg)
    insts = []
    for spec in cfg["instances"]:
        insts.extend(_instance(spec))
    if cfg["samples"] == "per_instance":
        counts = I.mixed_batch_sizes(insts)
    else:
        counts = [int(cfg["samples"])] * len(insts)
    return insts, counts


FLAG_BITS = {"lds_chain": 1, "profile": 2, "graph": 4, "split_bf16": 8, "check_finite": 16,
             "markers": 32}


def net_options(cfg) -> dict:
    """Keyword arguments of paper_2504_12037_amd.Net for a config."""
    if isinstance(cfg, str):
        cfg = load(cfg)
    flags = 0
    for f in cfg.get("flags", []):
        flags |= FLAG_BITS[f]
    return {"precision": cfg["precision"], "flags": flags,
            "max_width": int(cfg.get("max_width", 14)), "seed": int(cfg["train"]["seed"])}
