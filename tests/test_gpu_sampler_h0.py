"""The one-layer sampler (H = 0, Eq. 7 as the whole network; Table 1's
depth-1 setting) for width sets too large for the matrix-core sampler:
spins and ln q against the oracle's ancestral sampling, given uniforms and
on the Philox stream, for |W| spanning every register layout (70, 200, 300,
512) and an uneven two-instance batch."""

import numpy as np
import pytest

import synthetic as S
from oracle import made as OM
from oracle import philox as OP
from synthetic import instances as SI

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TIE = 1e-6


def _chain_instance(nw, seed):
    # a path of nw + 4 spins with W = the first nw: the contraction is tiny,
    # the sampler sees |W| = nw
    n = nw + 4
    rng = np.random.default_rng(seed)
    e = np.stack([np.arange(n - 1), np.arange(1, n)], 1).astype(np.int32)
    return SI.Instance(n, e, rng.standard_normal(n - 1), np.zeros(n), 0.7,
                       np.arange(nw, dtype=np.int32), np.arange(nw, n, dtype=np.int32),
                       None, 0, f"path{n}")


def _theta(n, seed):
    th = S.made_init(n, 0, seed)
    return (th + 0.3 * np.random.default_rng(seed).standard_normal(th.shape)).astype(np.float32)


def _check(theta, u, n, s_gpu, lq_gpu, prec):
    B = u.shape[0]
    s_o, _, p = OM.sample(theta.astype(np.float64), u, n, 0)
    tie = np.abs(p - u) < TIE
    if tie.any():
        force = np.zeros((B, n), np.int8)
        force[tie] = s_gpu[tie]
        s_o, _, p = OM.sample(theta.astype(np.float64), u, n, 0, force=force)
    assert np.array_equal(s_o, s_gpu), np.argwhere(s_o != s_gpu)[:5]
    lq_o = OM.logq(theta.astype(np.float64), s_gpu, n, 0)
    tol = 1e-10 if prec == "fp64" else 2e-4
    assert np.abs(lq_gpu - lq_o).max() <= tol * max(1, n / 8)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("nw", [70, 200, 300, 512])
def test_one_layer_sampler_given_uniforms(nw, prec):
    from paper_2504_12037_amd import Net
    inst = _chain_instance(nw, nw)
    B = 203
    print(f"\n[sample-h0] n={nw} prec={prec} B={B}", flush=True)
    theta = _theta(nw, 5 + nw)
    net = Net([inst], precision=prec)
    net.set_params(0, torch.from_numpy(theta))
    u = S.uniforms(B, nw, 13)
    sp, lq = net.sample(B, torch.from_numpy(u).cuda().reshape(-1))
    _check(theta, u, nw, sp.cpu().numpy().reshape(B, nw), lq.cpu().numpy(), prec)


def test_one_layer_sampler_philox_stream_two_instances():
    # uneven batch (333 and 130 samples; 130 is not a multiple of the four
    # samples of a block), two widths in one launch, Philox uniforms
    from paper_2504_12037_amd import Net
    insts = [_chain_instance(150, 1), _chain_instance(300, 2)]
    Bs = [333, 130]
    seed = 0x2468_ACE0_1357
    print("\n[sample-h0] two instances, Philox", flush=True)
    net = Net(insts, precision="fp32", seed=seed)
    thetas = [_theta(i.n_width, 20 + k) for k, i in enumerate(insts)]
    for k, th in enumerate(thetas):
        net.set_params(k, torch.from_numpy(th))
    sp, lq = net.sample(Bs)
    sp, lq = sp.cpu().numpy(), lq.cpu().numpy()
    so = bo = 0
    for k, inst in enumerate(insts):
        n, B = inst.n_width, Bs[k]
        u = OP.sampler_uniforms(seed, 0, k, B, n)
        _check(thetas[k], u, n, sp[so:so + B * n].reshape(B, n), lq[bo:bo + B], "fp32")
        so += B * n
        bo += B


@pytest.mark.parametrize("prec,nw", [("fp32", 200), ("fp64", 70), ("fp32", 300)])
def test_one_layer_training_step_parity(prec, nw):
    # one step: Philox draws, F_q statistics, the REINFORCE gradient from
    # the conditionals the sampler stored, and Adam, against the oracle
    from oracle import ising as OI
    from oracle import objective as OO
    from paper_2504_12037_amd import Net
    inst = _chain_instance(nw, 40 + nw)
    B, seed, lr = 517, 91, 1e-2
    print(f"\n[step-h0] n={nw} prec={prec} B={B}", flush=True)
    theta = _theta(nw, 7 + nw)
    net = Net([inst], precision=prec, seed=seed)
    net.set_params(0, torch.from_numpy(theta))
    spins = torch.empty(B * nw, dtype=torch.int8, device="cuda")
    stats, _ = net.free_energy_step(B, lr, spins_out=spins)
    torch.cuda.synchronize()
    sp = spins.cpu().numpy().reshape(B, nw)
    u = OP.sampler_uniforms(seed, 0, 0, B, nw)
    th64 = theta.astype(np.float64)
    s_o, _, p = OM.sample(th64, u, nw, 0)
    tie = np.abs(p - u) < TIE
    if tie.any():
        force = np.zeros((B, nw), np.int8)
        force[tie] = sp[tie]
        s_o, _, _ = OM.sample(th64, u, nw, 0, force=force)
    assert np.array_equal(s_o, sp)
    lq = OM.logq(th64, sp, nw, 0)
    lz = OI.logz_r_bruteforce(inst, sp)
    f, st = OO.free_energy_terms(inst, sp, lq, lz)
    g = OM.logq_backward(th64, sp, OO.reinforce_weights(f), nw, 0)
    tol = 1e-9 if prec == "fp64" else 2e-5
    np.testing.assert_allclose(stats.cpu().numpy()[0], st, atol=tol * 10 * max(1, nw / 64),
                               rtol=tol)
    g_gpu = net.get_state(0, 1).cpu().numpy()
    assert np.abs(g_gpu - g).max() <= 1e-6 + 1e-4 * np.abs(g).max()
    th1, _, _ = OO.adam_step(th64, g_gpu.astype(np.float64), np.zeros_like(th64),
                             np.zeros_like(th64), 1, lr)
    np.testing.assert_allclose(net.get_params(0).cpu().numpy(), th1, atol=1e-6, rtol=0)
    M1, M2, M0 = OM.masks(nw, 0)
    mask = OM.pack(M1, np.ones(0), M2, np.ones(nw), M0)
    assert np.all(g_gpu[mask == 0] == 0)


def test_one_layer_training_step_graph_replay():
    # the one-layer step (columns of W0, sampler, stored conditionals, rows,
    # sums, Adam) recorded once and replayed, against an identical eager net,
    # with eager work on another batch shape between replays
    from paper_2504_12037_amd import Net
    insts = [_chain_instance(200, 61), _chain_instance(90, 62)]
    Bs = [300, 129]
    nets = [Net(insts, precision="fp32", seed=5),
            Net(insts, precision="fp32", seed=5, flags=Net.FLAG_GRAPH)]
    for net in nets:
        for k, inst in enumerate(insts):
            net.set_params(k, torch.from_numpy(_theta(inst.n_width, 70 + k)))
    stats = [torch.empty(2, 4, dtype=torch.float64, device="cuda") for _ in nets]
    spins = [torch.empty(sum(b * i.n_width for b, i in zip(Bs, insts)), dtype=torch.int8,
                         device="cuda") for _ in nets]
    for it in range(6):
        print(f"\n[graph-h0] iteration {it}", flush=True)
        for net, st, sp in zip(nets, stats, spins):
            net.free_energy_step(Bs, 1e-2, stats=st, spins_out=sp)
        torch.cuda.synchronize()
        assert torch.equal(stats[0], stats[1]), it
        assert torch.equal(spins[0], spins[1]), it
        if it == 2:
            sp_o, _ = nets[1].sample([17, 5])
            torch.cuda.synchronize()
            assert sp_o.numel() == 17 * 200 + 5 * 90
    for k in range(len(insts)):
        assert torch.equal(nets[0].get_params(k), nets[1].get_params(k))
