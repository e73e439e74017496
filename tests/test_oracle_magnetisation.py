"""Pins of the oracle for the remainder's magnetisation moments and the
susceptibility estimator (Sec. 3: magnetisation and susceptibility from the
trained network's samples) against closed forms, invariants, independent
oracle routines and full enumeration."""

import numpy as np
import pytest

import synthetic as S
from oracle import ising as I
from oracle import magnetisation as M
from oracle import objective as O
from test_oracle_ising import random_instance


def _chain(n, seed, beta, field=0.0):
    # an open chain of n remainder spins plus one isolated width-set spin
    rng = np.random.default_rng(seed)
    edges = np.stack([np.arange(1, n), np.arange(2, n + 1)], 1).astype(np.int32)
    J = rng.standard_normal(n - 1)
    h = np.zeros(n + 1)
    h[1:] = field
    return S.Instance(n + 1, edges, J, h, beta, np.zeros(1, np.int32),
                      np.arange(1, n + 1, dtype=np.int32), None, 0, "chain")


def _chain_variance(J, beta):
    # zero field: <r_i r_j> = prod_{k=i}^{j-1} tanh(beta J_k), <r_i> = 0
    t = np.tanh(beta * np.asarray(J))
    n = len(J) + 1
    var = float(n)
    for i in range(n):
        p = 1.0
        for j in range(i + 1, n):
            p *= t[j - 1]
            var += 2 * p
    return var


def test_beta_zero_is_independent_spins():
    inst = random_instance(14, 0.3, 2, 5, beta=0.0)
    s = S.uniform_spins(6, 5, 3)
    for fn in (M.remainder_magnetisation_bruteforce, M.remainder_magnetisation):
        mean, var = fn(inst, s)
        np.testing.assert_allclose(mean, 0.0, atol=1e-12)
        np.testing.assert_allclose(var, 9.0, atol=1e-11)


def test_isolated_remainder_spins_closed_form():
    # W = one side of a bipartite graph: every R spin sees only W spins and
    # its field, so M_R is a sum of independent spins with effective fields f
    rng = np.random.default_rng(4)
    nw, nr = 5, 7
    edges = np.array([(w, nw + r) for w in range(nw) for r in range(nr)
                      if rng.random() < 0.6], np.int32)
    inst = S.Instance(nw + nr, edges, rng.standard_normal(len(edges)),
                      0.4 * rng.standard_normal(nw + nr), 0.9,
                      np.arange(nw, dtype=np.int32),
                      np.arange(nw, nw + nr, dtype=np.int32), None, 0, "bip")
    s = S.uniform_spins(12, nw, 5)
    f = I.Split(inst).fields_on_r(s)[:, nw:]
    t = np.tanh(inst.beta * f)
    for fn in (M.remainder_magnetisation_bruteforce, M.remainder_magnetisation):
        mean, var = fn(inst, s)
        np.testing.assert_allclose(mean, t.sum(1), atol=1e-12)
        np.testing.assert_allclose(var, (1 - t * t).sum(1), atol=1e-12)


@pytest.mark.parametrize("beta", [0.3, 1.0, 2.5])
def test_open_chain_closed_form(beta):
    # small enough for brute force, and far beyond it for the elimination
    s = np.ones((1, 1), np.int8)
    for n in (12, 90):
        inst = _chain(n, 5, beta)
        want = _chain_variance(inst.J, beta)
        fns = [M.remainder_magnetisation] + ([M.remainder_magnetisation_bruteforce]
                                             if n <= 16 else [])
        for fn in fns:
            mean, var = fn(inst, s)
            assert abs(mean[0]) < 1e-10
            assert abs(var[0] - want) < 1e-9 * want


def test_distribution_matches_enumeration():
    # the whole law of M_R, not only its first two moments
    inst = random_instance(15, 0.35, 7, 4, beta=0.8)
    s = S.uniform_spins(9, 4, 8)
    lp = M.remainder_magnetisation_distribution(inst, s)
    sp = I.Split(inst)
    nr = len(sp.R)
    Jrr, _ = I._r_quadratic(sp)
    f = sp.fields_on_r(s)[:, sp.R]
    r = I._all_configs(nr)
    expo = inst.beta * (np.einsum("ci,ij,cj->c", r, Jrr, r)[None, :] + f @ r.T)
    p = np.exp(expo - I._logsumexp(expo, axis=1)[:, None])
    k = ((1 - r) / 2).sum(1).astype(int)
    want = np.zeros((s.shape[0], nr + 1))
    for c in range(r.shape[0]):
        want[:, k[c]] += p[:, c]
    np.testing.assert_allclose(np.exp(lp), want, atol=1e-13)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_elimination_against_bruteforce(seed):
    inst = random_instance(16, 0.3, seed, 5, beta=1.1, hfield=0.5, order_seed=seed + 1)
    s = S.uniform_spins(10, 5, seed)
    m1, v1 = M.remainder_magnetisation_bruteforce(inst, s)
    m2, v2 = M.remainder_magnetisation(inst, s)
    np.testing.assert_allclose(m2, m1, atol=1e-11)
    np.testing.assert_allclose(v2, v1, atol=1e-10)


def test_global_flip_without_fields():
    inst = random_instance(14, 0.35, 21, 4, beta=0.9, hfield=0.0)
    s = S.uniform_spins(8, 4, 22)
    mean, var = M.remainder_magnetisation(inst, s)
    mf, vf = M.remainder_magnetisation(inst, -s)
    np.testing.assert_allclose(mf, -mean, atol=1e-11)
    np.testing.assert_allclose(vf, var, atol=1e-10)


def test_mean_is_the_sum_of_the_marginals():
    # against the reverse pass of the plain elimination (an independent
    # routine), on a lattice remainder beyond enumeration
    inst = S.lattice_column_split(S.lattice_2d(8, seed=9, beta=0.7, h_var=0.2), [5])
    s = S.uniform_spins(6, inst.n_width, 23)
    mean, _ = M.remainder_magnetisation(inst, s)
    _, mag, _, _ = I.marginals_elimination(inst, s)
    np.testing.assert_allclose(mean, mag[:, inst.order].sum(1), atol=1e-10)


@pytest.mark.parametrize("big", [False, True])
def test_variance_is_the_second_field_derivative(big):
    # v_R = d^2 logZ_R / d(beta H)^2 for a uniform field H on R, by a central
    # second difference of logZ_R (brute force, or elimination at |R| = 56)
    if big:
        inst = S.lattice_column_split(S.lattice_2d(8, seed=9, beta=0.7, h_var=0.2), [5])
        lz = I.logz_r_elimination
    else:
        inst = random_instance(14, 0.35, 31, 4, beta=0.8, hfield=0.3)
        lz = I.logz_r_bruteforce
    s = S.uniform_spins(5, inst.n_width, 32)
    mean, var = M.remainder_magnetisation(inst, s)
    d = 1e-3
    vals = []
    for k in (-1, 0, 1):
        h = np.array(inst.h, dtype=np.float64).copy()
        h[inst.order] += k * d
        vals.append(lz(S.Instance(inst.n, inst.edges, inst.J, h, inst.beta, inst.width_set,
                                  inst.order, inst.group_ptr, 0), s))
    b = inst.beta
    fd1 = (vals[2] - vals[0]) / (2 * d) / b
    fd2 = (vals[2] - 2 * vals[1] + vals[0]) / (d * d) / (b * b)
    # truncation of the central differences: d^2 / 6 times the third
    # cumulant of M_R (first), d^2 / 12 times the fourth (second)
    np.testing.assert_allclose(mean, fd1, rtol=2e-5, atol=2e-5)
    np.testing.assert_allclose(var, fd2, rtol=2e-4, atol=2e-4)


@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0])
def test_susceptibility_exact_under_full_enumeration(beta):
    # every width-set configuration once, with a uniform q: the weights are
    # the exact W-marginal of p, so the estimator equals the moments of p
    # by enumerating all 2^N states
    inst = random_instance(13, 0.35, 41, 5, beta=beta, hfield=0.3)
    sW = O.all_width_states(5).astype(np.int8)
    logq = np.full(sW.shape[0], -5 * np.log(2))
    m, m2, chi, ess = M.susceptibility(inst, sW, logq)
    c = I._all_configs(inst.n)
    e = I.energy(inst, c)
    lw = -beta * e
    p = np.exp(lw - I._logsumexp(lw, axis=0))
    Mf = c.sum(1)
    want_m, want_m2 = p @ Mf, p @ (Mf * Mf)
    assert abs(m - want_m / inst.n) < 1e-12
    assert abs(m2 - want_m2 / inst.n ** 2) < 1e-12
    assert abs(chi - beta * (want_m2 - want_m ** 2) / inst.n) < 1e-11
    assert 1.0 <= ess <= sW.shape[0] + 1e-9
