"""Algorithm 1 driver with a per-step JSON-lines log.

    from paper_2504_12037_amd import Net
    from paper_2504_12037_amd.train import train
    history = train(net, n_samples, lr=1e-2, steps=1000, log="run.jsonl")

Each iteration is one tnvan_free_energy_step call (sample from q, contract
logZ_R, F_q and the REINFORCE weights, the gradient of q, Adam); the
library does all of it.  Every ``every`` steps the driver waits for the
step and writes one JSON object per line:

    step        steps taken so far (the net's step counter of instance 0)
    F_q         per instance, the batch mean of f (Eq. 9)
    stderr      its standard error
    F_q_per_spin, Etilde, lnq_over_beta   per instance
    grad_norm   per instance, the REINFORCE gradient's 2-norm (every
                ``grad_every`` logged steps; null otherwise)
    rel_gap     per instance, (F_q - F) / |F| when exact free energies are
                passed in ``exact_F``
    wall_s      seconds since the first step

This is the F_q-against-epoch record the paper plots for its runs
(Sec. 4, Fig. 3(b)).  The returned list holds the same records.
"""

from __future__ import annotations

import json
import math
import time
from typing import Optional, Sequence

import torch


def train(net, n_samples, lr: float, steps: int, log: Optional[str] = None, every: int = 1,
          grad_every: int = 0, exact_F: Optional[Sequence[float]] = None) -> list:
    counts = n_samples if not isinstance(n_samples, int) else [n_samples] * len(net.instances)
    n_inst = len(net.instances)
    stats = torch.empty(n_inst, 4, dtype=torch.float64, device="cuda")
    history = []
    out = open(log, "a") if log else None
    step0 = net.get_step(0)
    t0 = time.perf_counter()
    logged = 0
    try:
        for it in range(1, steps + 1):
            net.free_energy_step(counts, lr, stats=stats)
            if it % every and it != steps:
                continue
            st = stats.cpu().numpy()
            rec = {"step": step0 + it,
                   "F_q": [float(v) for v in st[:, 0]],
                   "stderr": [float(v) for v in st[:, 1]],
                   "F_q_per_spin": [float(st[k, 0]) / net.n[k] for k in range(n_inst)],
                   "Etilde": [float(v) for v in st[:, 2]],
                   "lnq_over_beta": [float(v) for v in st[:, 3]],
                   "grad_norm": None,
                   "wall_s": time.perf_counter() - t0}
            if grad_every and logged % grad_every == 0:
                rec["grad_norm"] = [float(torch.linalg.vector_norm(net.get_state(k, 1)))
                                    for k in range(n_inst)]
            if exact_F is not None:
                rec["rel_gap"] = [(rec["F_q"][k] - exact_F[k]) / abs(exact_F[k])
                                  if exact_F[k] is not None and math.isfinite(exact_F[k]) else None
                                  for k in range(n_inst)]
            history.append(rec)
            logged += 1
            if out:
                out.write(json.dumps(rec) + "\n")
                out.flush()
    finally:
        if out:
            out.close()
    return history
