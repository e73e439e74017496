"""Moments of p from samples of q (self-normalised importance weights, the
remainder's conditional moments from the adjoint) through the C ABI, against
brute force (full enumeration of W with a uniform q, where the estimate is
exact) and against the oracle's estimator on oracle-drawn samples."""

import numpy as np
import pytest

import synthetic as S
from oracle import ising as OI
from oracle import made as OM
from oracle import objective as OO
from oracle import philox as OP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-4}


def _net(insts, prec, **kw):
    from paper_2504_12037_amd import Net
    return Net(insts, precision=prec, **kw)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().reshape(-1)


@pytest.mark.parametrize("prec,flags", [("fp64", 0), ("fp32", 0), ("fp32", 8)])
def test_observables_exact_under_full_enumeration(prec, flags):
    inst = S.c1_small_lattice()
    nw = inst.n_width
    x = np.arange(1 << nw)[:, None]
    sw = (1 - 2 * ((x >> np.arange(nw)[None, :]) & 1)).astype(np.int8)
    print(f"\n[obs] 4x4 full enumeration prec={prec} flags={flags}", flush=True)
    net = _net([inst], prec, flags=flags)
    mag, corr, ess = net.observables(_dev(sw), torch.zeros(sw.shape[0]), sw.shape[0])
    torch.cuda.synchronize()
    n = inst.n
    y = np.arange(1 << n)[:, None]
    full = (1 - 2 * ((y >> np.arange(n)[None, :]) & 1)).astype(np.float64)
    e = OI.energy(inst, full)
    p = np.exp(-inst.beta * (e - e.min()))
    p /= p.sum()
    ed = np.asarray(inst.edges).reshape(-1, 2)
    np.testing.assert_allclose(mag.cpu().numpy(), p @ full, atol=TOL[prec])
    np.testing.assert_allclose(corr.cpu().numpy(), p @ (full[:, ed[:, 0]] * full[:, ed[:, 1]]),
                               atol=TOL[prec])
    _, _, ess_o = OO.observables(inst, sw, np.zeros(sw.shape[0]))
    assert abs(ess.cpu().numpy()[0] - ess_o) <= 1e-6 * ess_o


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_observables_match_the_oracle_estimator(prec):
    # two instances in one call (offsets), samples and ln q drawn by the
    # oracle's MADE from seeded uniforms
    insts = [S.lattice_column_split(S.lattice_2d(8, seed=14, h_var=0.1), [5], hidden=16),
             S.c4_small_copies()[2]]
    Bs = [300, 200]
    spins, logqs = [], []
    for k, inst in enumerate(insts):
        n, H = inst.n_width, inst.hidden
        th = S.made_init(n, H, 40 + k).astype(np.float64)
        u = OP.sampler_uniforms(5, 0, k, Bs[k], n)
        s, lq, _ = OM.sample(th, u, n, H)
        spins.append(s.astype(np.int8))
        logqs.append(lq)
    print(f"\n[obs] oracle samples prec={prec}", flush=True)
    net = _net(insts, prec)
    mag, corr, ess = net.observables(_dev(np.concatenate([s.reshape(-1) for s in spins])),
                                     torch.from_numpy(np.concatenate(logqs)), Bs)
    torch.cuda.synchronize()
    mag, corr, ess = mag.cpu().numpy(), corr.cpu().numpy(), ess.cpu().numpy()
    vo = eo = 0
    for k, inst in enumerate(insts):
        m_o, c_o, ess_o = OO.observables(inst, spins[k], logqs[k])
        ne = len(inst.edges)
        np.testing.assert_allclose(mag[vo:vo + inst.n], m_o, atol=TOL[prec])
        np.testing.assert_allclose(corr[eo:eo + ne], c_o, atol=TOL[prec])
        assert abs(ess[k] - ess_o) <= 1e-3 * ess_o
        assert np.all(np.abs(mag[vo:vo + inst.n]) <= 1 + 1e-12)
        vo += inst.n
        eo += ne
