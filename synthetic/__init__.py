"""Seeded synthetic inputs shared by the oracle and the GPU path.

Everything here is an *input*: coupling graphs and their random couplings and
fields, width sets, elimination orders and row groupings, spin batches,
uniform random numbers and initial network parameters.  No part of the
method's arithmetic (Boltzmann weights, partition functions, network
evaluation, gradients) lives here; the oracle and the HIP library each
implement that on their own.
"""

from .instances import (  # noqa: F401
    Instance,
    lattice_2d,
    lattice_column_split,
    lattice_auto_split,
    sherrington_kirkpatrick,
    random_regular,
    mixed_batch_instances,
    mixed_batch_sizes,
    paper_configs,
    c1_small_lattice,
    c2_lattice,
    c3_sk,
    c4_rrg,
    c4_small_copies,
)
from .planner import (  # noqa: F401
    elimination_scopes,
    min_fill_order,
    order_width,
    greedy_width_set,
)
from . import config  # noqa: F401
from .draws import (  # noqa: F401
    uniform_spins,
    uniforms,
    made_init,
    made_param_count,
    split_params,
)
