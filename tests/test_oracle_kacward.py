"""Pins of the Kac-Ward oracle (exact ln Z of planar zero-field Ising models)
against brute-force enumeration: square lattices with ferromagnetic and
Gaussian couplings at several temperatures, and a triangulated lattice (turns
of 45, 90 and 135 degrees), all small enough to enumerate."""

import numpy as np
import pytest

import synthetic as S
from oracle import ising as OI
from oracle import kacward as K
from synthetic import instances as SI


@pytest.mark.parametrize("L,ferro,beta", [(3, True, 0.44), (4, True, 0.3), (4, True, 1.0),
                                          (4, False, 0.7), (3, False, 2.0)])
def test_kac_ward_square_lattice_matches_brute_force(L, ferro, beta):
    inst = S.lattice_2d(L, seed=3 + L, beta=beta, ferro=ferro)
    want = OI.logz_full_bruteforce(inst)
    got = K.logz_planar(inst.n, inst.edges, inst.J, beta, K.lattice_xy(L))
    assert abs(got - want) <= 1e-10 * max(1.0, abs(want))


def test_kac_ward_triangulated_lattice_matches_brute_force():
    # square lattice plus one diagonal per plaquette: still planar with
    # straight edges, and turns that are not multiples of 90 degrees
    L = 4
    e = [tuple(x) for x in SI.lattice_edges(L)]
    e += [(r * L + c, (r + 1) * L + c + 1) for r in range(L - 1) for c in range(L - 1)]
    e = np.asarray(e, np.int32)
    J = np.random.default_rng(9).standard_normal(e.shape[0])
    beta = 0.8
    inst = SI.Instance(L * L, e, J, np.zeros(L * L), beta, np.zeros(0, np.int32),
                       np.arange(L * L, dtype=np.int32))
    want = OI.logz_full_bruteforce(inst)
    got = K.logz_planar(inst.n, e, J, beta, K.lattice_xy(L))
    assert abs(got - want) <= 1e-10 * max(1.0, abs(want))


def test_kac_ward_high_temperature_limit():
    # beta = 0: Z = 2^N
    L = 5
    e = SI.lattice_edges(L)
    got = K.logz_planar(L * L, e, np.ones(e.shape[0]), 0.0, K.lattice_xy(L))
    assert abs(got - L * L * np.log(2.0)) <= 1e-12
