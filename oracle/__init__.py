"""FP64 CPU oracle for the TNVAN hot path.  TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct reference that the HIP
library is checked against.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library: it reads the same seeded inputs
(couplings, fields, beta, width set, order, spins, uniforms, parameters) and
recomputes everything with numpy in float64.

Modules
  ising     energy split and the conditional log-partition function of the
            remainder (Sec. 2, Eqs. 1-4): brute force and log-domain variable
            elimination, plus the reverse pass giving marginals/correlations
  made      the masked autoregressive network (Sec. 3, Eqs. 6-8): logits,
            ancestral sampling, log q and its backward
  objective variational free energy and REINFORCE weights (Eqs. 9-10), Adam,
            exact enumeration over small width sets, the training loop of
            Algorithm 1
  philox    Philox4x32-10 counter-based generator (Salmon et al., SC'11)
  magnetisation
            conditional law of the remainder's magnetisation given s_W and
            the importance-weighted susceptibility estimator (Sec. 3)

Parity status of every function is listed in its module header.
"""

from . import ising, made, magnetisation, objective, philox  # noqa: F401
