"""Pins of the FP64 oracle for the conditional partition function (Sec. 2,
Eqs. 1-4) against closed forms, invariants and brute force."""

import numpy as np
import pytest

import synthetic as S
from oracle import ising as I


def random_instance(n, p, seed, nw, beta=0.8, hfield=0.3, order_seed=None):
    rng = np.random.default_rng(seed)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n)
             if rng.random() < p]
    edges = np.asarray(edges, np.int32).reshape(-1, 2)
    J = rng.standard_normal(edges.shape[0])
    h = hfield * rng.standard_normal(n)
    perm = rng.permutation(n)
    W = np.sort(perm[:nw]).astype(np.int32)
    R = perm[nw:]
    if order_seed is not None:
        R = np.random.default_rng(order_seed).permutation(R)
    return S.Instance(n, edges, J, h, beta, W, R.astype(np.int32), None, 0,
                      f"er{n}_{seed}")


def chain(n, seed, beta, with_w=False):
    rng = np.random.default_rng(seed)
    edges = np.stack([np.arange(n - 1), np.arange(1, n)], 1).astype(np.int32)
    J = rng.standard_normal(n - 1)
    return S.Instance(n, edges, J, np.zeros(n), beta, np.zeros(0, np.int32),
                      np.arange(n, dtype=np.int32), None, 0, "chain")


def test_energy_split_sums_to_energy():
    inst = random_instance(12, 0.4, 1, 4)
    rng = np.random.default_rng(0)
    s = (2 * rng.integers(0, 2, (20, 4)) - 1).astype(np.int8)
    r = (2 * rng.integers(0, 2, (20, 8)) - 1).astype(np.int8)
    e1, e2 = I.energy_split(inst, s, r)
    full = np.zeros((20, 12))
    full[:, inst.width_set] = s
    full[:, inst.order] = r
    # direct definition of E written as a plain loop over edges and spins
    E = np.zeros(20)
    for (a, b), j in zip(inst.edges, inst.J):
        E -= j * full[:, a] * full[:, b]
    for v in range(12):
        E -= inst.h[v] * full[:, v]
    np.testing.assert_allclose(e1 + e2, E, atol=1e-12)
    np.testing.assert_allclose(I.e1_energy(inst, s), e1, atol=1e-12)


def test_beta_zero_counts_states():
    inst = random_instance(14, 0.3, 2, 5, beta=0.0)
    s = S.uniform_spins(6, 5, 3)
    nr = 9
    np.testing.assert_allclose(I.logz_r_bruteforce(inst, s), nr * np.log(2),
                               atol=1e-12)
    np.testing.assert_allclose(I.logz_r_elimination(inst, s), nr * np.log(2),
                               atol=1e-12)


@pytest.mark.parametrize("beta", [0.3, 1.0, 2.5])
def test_open_chain_closed_form(beta):
    inst = chain(12, 5, beta)
    s = np.zeros((1, 0), np.int8)
    want = 12 * np.log(2) + np.sum(np.log(np.cosh(beta * inst.J)))
    assert abs(I.logz_r_bruteforce(inst, s)[0] - want) < 1e-11
    assert abs(I.logz_r_elimination(inst, s)[0] - want) < 1e-11


def test_chain_with_boundary_fields_transfer_matrix():
    # the 4x1 strip of the 4x4 workload: a chain of 4 R spins, each coupled
    # to W spins; summed with 2x2 transfer matrices (textbook method)
    inst = S.c1_small_lattice()
    s = S.uniform_spins(16, 4, 11)
    sp = I.Split(inst)
    f = sp.fields_on_r(s)
    b = inst.beta
    # strip 1 = column 1 = vertices 0, 4, 8, 12 (vertical bonds)
    col = [0, 4, 8, 12]
    eid = {tuple(e): k for k, e in enumerate(inst.edges.tolist())}
    lz_strip = np.zeros(16)
    for bi in range(16):
        vec = np.array([np.exp(b * f[bi, col[0]]), np.exp(-b * f[bi, col[0]])])
        for a, c in zip(col[:-1], col[1:]):
            Jv = inst.J[eid[(a, c)]]
            K = np.array([[np.exp(b * Jv), np.exp(-b * Jv)],
                          [np.exp(-b * Jv), np.exp(b * Jv)]])
            D = np.diag([np.exp(b * f[bi, c]), np.exp(-b * f[bi, c])])
            vec = vec @ K @ D
        lz_strip[bi] = np.log(vec.sum())
    # strip 2 (columns 3-4, a 4x2 ladder) by brute force over its 8 spins
    lad = [2, 3, 6, 7, 10, 11, 14, 15]
    cfg = I._all_configs(8)
    lz_lad = np.zeros(16)
    for bi in range(16):
        ex = np.zeros(cfg.shape[0])
        for (a, c), j in zip(inst.edges, inst.J):
            if a in lad and c in lad:
                ex += b * j * cfg[:, lad.index(a)] * cfg[:, lad.index(c)]
        for k, v in enumerate(lad):
            ex += b * f[bi, v] * cfg[:, k]
        lz_lad[bi] = np.log(np.sum(np.exp(ex)))
    want = lz_strip + lz_lad
    np.testing.assert_allclose(I.logz_r_bruteforce(inst, s), want, atol=1e-11)
    np.testing.assert_allclose(I.logz_r_elimination(inst, s), want, atol=1e-11)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_elimination_matches_bruteforce(seed):
    inst = random_instance(16, 0.35, seed, 4 + seed)
    s = S.uniform_spins(9, inst.n_width, seed)
    np.testing.assert_allclose(I.logz_r_elimination(inst, s),
                               I.logz_r_bruteforce(inst, s), atol=1e-11)


def test_order_independence():
    a = random_instance(16, 0.35, 7, 5, order_seed=1)
    b = random_instance(16, 0.35, 7, 5, order_seed=2)
    assert not np.array_equal(a.order, b.order)
    s = S.uniform_spins(5, 5, 0)
    np.testing.assert_allclose(I.logz_r_elimination(a, s),
                               I.logz_r_elimination(b, s), atol=1e-11)


def test_gauge_invariance():
    inst = random_instance(15, 0.4, 9, 5)
    s = S.uniform_spins(8, 5, 4)
    base = I.logz_r_bruteforce(inst, s)
    e1 = I.e1_energy(inst, s)
    for v in [int(inst.width_set[1]), int(inst.order[3])]:
        J2 = inst.J.copy()
        touch = (inst.edges[:, 0] == v) | (inst.edges[:, 1] == v)
        J2[touch] *= -1
        h2 = inst.h.copy()
        h2[v] *= -1
        s2 = s.copy()
        if v in inst.width_set:
            s2[:, list(inst.width_set).index(v)] *= -1
        g = S.Instance(inst.n, inst.edges, J2, h2, inst.beta, inst.width_set,
                       inst.order)
        np.testing.assert_allclose(I.logz_r_bruteforce(g, s2), base, atol=1e-11)
        np.testing.assert_allclose(I.logz_r_elimination(g, s2), base, atol=1e-11)
        np.testing.assert_allclose(I.e1_energy(g, s2), e1, atol=1e-12)


def test_global_flip_without_fields():
    inst = S.c1_small_lattice()
    s = S.uniform_spins(16, 4, 2)
    np.testing.assert_allclose(I.logz_r_elimination(inst, s),
                               I.logz_r_elimination(inst, -s), atol=1e-11)


@pytest.mark.parametrize("maker", ["c1", "er"])
def test_slice_sum_identity(maker):
    # Eq. 3: summing exp(-beta E_1 + logZ_R) over every width-set state
    # gives the full partition function
    inst = S.c1_small_lattice() if maker == "c1" else random_instance(14, 0.4, 3, 6)
    nw = inst.n_width
    k = np.arange(2 ** nw)[:, None]
    s = (1 - 2 * ((k >> np.arange(nw)[None, :]) & 1)).astype(np.int8)
    lz = I.logz_r_elimination(inst, s)
    e1 = I.e1_energy(inst, s)
    tot = np.logaddexp.reduce(-inst.beta * e1 + lz)
    assert abs(tot - I.logz_full_bruteforce(inst)) < 1e-10


def test_marginals_elimination_vs_bruteforce():
    for seed in range(3):
        inst = random_instance(15, 0.4, 20 + seed, 4)
        s = S.uniform_spins(6, 4, seed)
        lz, mag, corr, e2 = I.marginals_elimination(inst, s)
        m2, c2, e22 = I.marginals_bruteforce(inst, s)
        np.testing.assert_allclose(lz, I.logz_r_bruteforce(inst, s), atol=1e-11)
        np.testing.assert_allclose(mag, m2, atol=1e-11)
        np.testing.assert_allclose(corr, c2, atol=1e-11)
        np.testing.assert_allclose(e2, e22, atol=1e-10)
        assert np.all(np.abs(mag) <= 1 + 1e-12) and np.all(np.abs(corr) <= 1 + 1e-12)


def _with(inst, J=None, h=None, beta=None):
    return S.Instance(inst.n, inst.edges, inst.J if J is None else J,
                      inst.h if h is None else h,
                      inst.beta if beta is None else beta,
                      inst.width_set, inst.order)


def test_vjp_finite_differences_and_euler():
    inst = random_instance(14, 0.4, 31, 4)
    s = S.uniform_spins(5, 4, 8)
    g = np.array([0.3, -1.2, 0.7, 0.1, 2.0])
    dh, dJ, db = I.logz_r_vjp(inst, s, g)
    eps = 1e-4

    def L(i):
        return float(g @ I.logz_r_bruteforce(i, s))
    for e in range(0, inst.n_edges, 3):
        Jp, Jm = inst.J.copy(), inst.J.copy()
        Jp[e] += eps
        Jm[e] -= eps
        fd = (L(_with(inst, J=Jp)) - L(_with(inst, J=Jm))) / (2 * eps)
        assert abs(fd - dJ[e]) < 1e-6
    for v in range(inst.n):
        hp, hm = inst.h.copy(), inst.h.copy()
        hp[v] += eps
        hm[v] -= eps
        fd = (L(_with(inst, h=hp)) - L(_with(inst, h=hm))) / (2 * eps)
        assert abs(fd - dh[v]) < 1e-6
    fd = (L(_with(inst, beta=inst.beta + eps)) - L(_with(inst, beta=inst.beta - eps))) / (2 * eps)
    assert abs(fd - db) < 1e-6
    # Euler identity of a function homogeneous in (beta J, beta h)
    assert abs(inst.beta * db - (inst.J @ dJ + inst.h @ dh)) < 1e-9


def test_marginals_vanish_at_beta_zero():
    inst = random_instance(14, 0.4, 5, 4, beta=0.0)
    s = S.uniform_spins(4, 4, 1)
    _, mag, corr, e2 = I.marginals_elimination(inst, s)
    sp = I.Split(inst)
    assert np.abs(mag).max() < 1e-12
    assert np.abs(corr[:, sp.rr + sp.wr]).max() < 1e-12
    assert np.abs(e2).max() < 1e-12


def test_rrg_small_copies_elimination():
    for inst in S.c4_small_copies():
        s = S.uniform_spins(4, inst.n_width, 5)
        lz, mag, corr, e2 = I.marginals_elimination(inst, s)
        m2, c2, e22 = I.marginals_bruteforce(inst, s)
        np.testing.assert_allclose(lz, I.logz_r_bruteforce(inst, s), atol=1e-11)
        np.testing.assert_allclose(mag, m2, atol=1e-10)
        np.testing.assert_allclose(corr, c2, atol=1e-10)
