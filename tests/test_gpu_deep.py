"""Deeper masked networks (D - 1 hidden-to-hidden tanh layers after the
first) through the C ABI against the FP64 oracle: ancestral sampling given
uniforms and from the Philox stream, ln q, one training iteration of
Algorithm 1 (statistics, REINFORCE gradient, Adam) and its graph replay, on
nets that mix deeper and one-layer instances."""

import numpy as np
import pytest

import synthetic as S
from oracle import ising as OI
from oracle import made as OM
from oracle import objective as OO
from oracle import philox as OP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TIE = 1e-6


def _net(insts, prec, **kw):
    from paper_2504_12037_amd import Net
    return Net(insts, precision=prec, **kw)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().reshape(-1)


def _deep(inst, H, D):
    inst.hidden = H
    inst.depth = D
    return inst


def _theta(n, H, D, seed, noise):
    th = S.made_init(n, H, seed, depth=D)
    return (th + noise * np.random.default_rng(seed).standard_normal(th.shape)).astype(np.float32)


def _check_spins(theta, u, n, H, D, s_gpu):
    """Oracle sampling with the GPU's spin forced at near-ties only."""
    B = u.shape[0]
    force = np.zeros((B, n), np.int8)
    s_o, lq_o, p = OM.sample(theta.astype(np.float64), u, n, H, depth=D)
    tie = np.abs(p - u) < TIE
    if tie.any():
        force[tie] = s_gpu[tie]
        s_o, lq_o, p = OM.sample(theta.astype(np.float64), u, n, H, force=force, depth=D)
    assert np.array_equal(s_o, s_gpu), np.argwhere(s_o != s_gpu)[:5]
    return int(tie.sum())


def _mixed():
    # a depth-3 and a depth-2 instance beside a one-layer one and one with
    # no hidden layer (H = 0)
    return [_deep(S.c1_small_lattice(), 16, 3),
            _deep(S.lattice_column_split(S.lattice_2d(8, seed=1), [5]), 24, 2),
            _deep(S.c4_small_copies()[0], 8, 1),
            _deep(S.lattice_column_split(S.lattice_2d(6, seed=4), [3]), 0, 1)]


def test_parameter_count_and_refusals():
    from paper_2504_12037_amd import TnvanError
    insts = _mixed()
    net = _net(insts, "fp32")
    for k, inst in enumerate(insts):
        assert net.param_count(k) == OM.param_count(inst.n_width, inst.hidden,
                                                    inst.depth if inst.hidden else 1)
    with pytest.raises(TnvanError):
        _net([_deep(S.c1_small_lattice(), 16, 5)], "fp32")
    with pytest.raises(TnvanError):
        # a deeper network needs |W| <= 256
        big = S.lattice_column_split(S.lattice_2d(40, seed=1), [5, 10, 15, 20, 25, 30, 35])
        _net([_deep(big, 8, 2)], "fp32")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deep_sampler_parity_given_uniforms(prec):
    # every instance |W| <= 128 and H <= 64: 16 lanes per sample
    _sampler_parity(_mixed(), [301, 257, 64, 130], prec)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_deep_sampler_parity_one_wave_per_sample(prec):
    # an instance with H above 64: a wave per sample for the whole net
    insts = [_deep(S.lattice_column_split(S.lattice_2d(8, seed=1), [5]), 80, 2),
             _deep(S.c1_small_lattice(), 16, 3)]
    _sampler_parity(insts, [129, 64], prec)


def _sampler_parity(insts, Bs, prec):
    print(f"\n[deep sample] prec={prec} H={[i.hidden for i in insts]}", flush=True)
    net = _net(insts, prec)
    thetas, us = [], []
    for k, inst in enumerate(insts):
        n, H, D = inst.n_width, inst.hidden, inst.depth
        thetas.append(_theta(n, H, D, 3 + k, 0.5))
        net.set_params(k, torch.from_numpy(thetas[-1]))
        us.append(S.uniforms(Bs[k], n, 11 + k))
    sp, lq = net.sample(Bs, _dev(np.concatenate([u.reshape(-1) for u in us])))
    sp, lq = sp.cpu().numpy(), lq.cpu().numpy()
    so = lo = 0
    tol = 1e-10 if prec == "fp64" else 2e-4
    for k, inst in enumerate(insts):
        n, H, D = inst.n_width, inst.hidden, inst.depth
        s = sp[so:so + Bs[k] * n].reshape(Bs[k], n)
        ties = _check_spins(thetas[k], us[k], n, H, D, s)
        lq_o = OM.logq(thetas[k].astype(np.float64), s, n, H, D)
        print(f"  instance {k}: n={n} H={H} D={D} ties={ties} "
              f"ln q err {np.abs(lq[lo:lo + Bs[k]] - lq_o).max():.2e}", flush=True)
        assert np.abs(lq[lo:lo + Bs[k]] - lq_o).max() <= tol * max(1, n / 8)
        so += Bs[k] * n
        lo += Bs[k]


@pytest.mark.parametrize("H", [24, 80])
def test_deep_sampler_philox_stream(H):
    # H = 24: 16 lanes per sample; H = 80: a wave per sample
    inst = _deep(S.lattice_column_split(S.lattice_2d(8, seed=1), [5]), H, 3)
    n, D, B = inst.n_width, 3, 500
    theta = _theta(n, H, D, 4, 0.3)
    net = _net([inst], "fp32", seed=0x1234_5678_9ABC)
    net.set_params(0, torch.from_numpy(theta))
    sp, _ = net.sample(B)
    u = OP.sampler_uniforms(0x1234_5678_9ABC, 0, 0, B, n)
    _check_spins(theta, u, n, H, D, sp.cpu().numpy().reshape(B, n))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deep_free_energy_step_parity(prec):
    # one iteration of Algorithm 1 on the mixed net: the GPU's spins equal
    # the oracle's from the Philox stream, and its statistics, REINFORCE
    # gradient and Adam step follow the oracle's on those spins
    insts = _mixed()
    Bs = [512, 256, 128, 200]
    seed, lr = 77, 1e-2
    net = _net(insts, prec, seed=seed)
    thetas = []
    for k, inst in enumerate(insts):
        thetas.append(_theta(inst.n_width, inst.hidden, inst.depth, 5 + k, 0.4))
        net.set_params(k, torch.from_numpy(thetas[-1]))
    spins = torch.empty(sum(b * i.n_width for b, i in zip(Bs, insts)), dtype=torch.int8,
                        device="cuda")
    print(f"\n[deep step] prec={prec}", flush=True)
    stats, _ = net.free_energy_step(Bs, lr, spins_out=spins)
    torch.cuda.synchronize()
    sp_all, st_all = spins.cpu().numpy(), stats.cpu().numpy()
    off = 0
    tol = 1e-9 if prec == "fp64" else 2e-5
    for k, (inst, b) in enumerate(zip(insts, Bs)):
        n, H, D = inst.n_width, inst.hidden, inst.depth
        sp = sp_all[off:off + b * n].reshape(b, n)
        off += b * n
        _check_spins(thetas[k], OP.sampler_uniforms(seed, 0, k, b, n), n, H, D, sp)
        th64 = thetas[k].astype(np.float64)
        lq = OM.logq(th64, sp, n, H, D)
        lz = (OI.logz_r_bruteforce if len(inst.order) <= 16 else OI.logz_r_elimination)(inst, sp)
        f, st = OO.free_energy_terms(inst, sp, lq, lz)
        np.testing.assert_allclose(st_all[k], st, atol=tol * 10, rtol=tol)
        g = OM.logq_backward(th64, sp, OO.reinforce_weights(f), n, H, D)
        g_gpu = net.get_state(k, 1).cpu().numpy()
        err = np.abs(g_gpu - g).max()
        print(f"  instance {k}: D={D} gradient err {err:.2e} of {np.abs(g).max():.2e}",
              flush=True)
        assert err <= 1e-7 + (1e-10 if prec == "fp64" else 1e-4) * np.abs(g).max()
        th1, _, _ = OO.adam_step(th64, g_gpu.astype(np.float64), np.zeros_like(th64),
                                 np.zeros_like(th64), 1, lr)
        np.testing.assert_allclose(net.get_params(k).cpu().numpy(), th1, atol=1e-6, rtol=0)
        if H > 0 and n >= 2:
            M1, M2, M0 = OM.masks(n, H)
            MH = OM.hidden_mask(n, H)
            mask = OM.pack(M1, np.ones(H), M2, np.ones(n), M0, [(MH, np.ones(H))] * (D - 1))
            assert np.all(g_gpu[mask == 0] == 0)


def test_deep_training_step_graph_replay():
    # replays of the recorded step equal an identical eager net bit for bit
    from paper_2504_12037_amd import Net
    insts = _mixed()[:2]
    Bs = [256, 300]
    nets = [_net(insts, "fp32", seed=21), _net(insts, "fp32", seed=21, flags=Net.FLAG_GRAPH)]
    for net in nets:
        for k, inst in enumerate(insts):
            net.set_params(k, torch.from_numpy(_theta(inst.n_width, inst.hidden, inst.depth,
                                                      30 + k, 0.2)))
    stats = [torch.empty(len(insts), 4, dtype=torch.float64, device="cuda") for _ in nets]
    spins = [torch.empty(sum(b * i.n_width for b, i in zip(Bs, insts)), dtype=torch.int8,
                         device="cuda") for _ in nets]
    for it in range(5):
        print(f"\n[deep graph] iteration {it}", flush=True)
        for net, st, sp in zip(nets, stats, spins):
            net.free_energy_step(Bs, 1e-2, stats=st, spins_out=sp)
        torch.cuda.synchronize()
        assert torch.equal(stats[0], stats[1]), it
        assert torch.equal(spins[0], spins[1]), it
    for k in range(len(insts)):
        assert torch.equal(nets[0].get_params(k), nets[1].get_params(k))
