"""GPU parity of the sampler (Eq. 8), the Philox stream, and one full
training iteration of Algorithm 1 (sample -> contract -> F_q and REINFORCE
-> Adam) against the FP64 oracle, through the C ABI."""

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


def _theta(n, H, seed, noise):
    th = S.made_init(n, H, seed)
    return (th + noise * np.random.default_rng(seed).standard_normal(th.shape)).astype(np.float32)


def _check_spins(theta, u, n, H, s_gpu):
    """Oracle sampling with the GPU's spin forced at near-ties only."""
    B = u.shape[0]
    force = np.zeros((B, n), np.int8)
    s_o, lq_o, p = OM.sample(theta.astype(np.float64), u, n, H)
    tie = np.abs(p - u) < TIE
    if tie.any():
        force[tie] = s_gpu[tie]
        s_o, lq_o, p = OM.sample(theta.astype(np.float64), u, n, H, force=force)
    assert np.array_equal(s_o, s_gpu), np.argwhere(s_o != s_gpu)[:5]
    return int(tie.sum()), lq_o


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["c1", "c2", "c3", "h0"])
def test_sampler_parity_given_uniforms(case, prec):
    inst = {"c1": lambda: S.c1_small_lattice(16), "c2": lambda: S.c2_lattice(1.0, 256),
            "c3": lambda: S.c3_sk(1.0, 128),
            "h0": lambda: S.lattice_column_split(S.lattice_2d(8, seed=1), [5], hidden=0)}[case]()
    n, H = inst.n_width, inst.hidden
    B = 777
    print(f"\n[sample] case={case} prec={prec} n={n} H={H} B={B}", flush=True)
    theta = _theta(n, H, 3, 0.5)
    net = _net([inst], prec)
    net.set_params(0, torch.from_numpy(theta))
    u = S.uniforms(B, n, 11)
    sp, lq = net.sample(B, _dev(u))
    sp = sp.cpu().numpy().reshape(B, n)
    ties, _ = _check_spins(theta, u, n, H, sp)
    lq_o = OM.logq(theta.astype(np.float64), sp, n, H)
    tol = 1e-10 if prec == "fp64" else 2e-4
    assert np.abs(lq.cpu().numpy() - lq_o).max() <= tol * max(1, n / 8)


def test_sampler_philox_stream():
    inst = S.c2_lattice(1.0, 64)
    n, H, B = 32, 64, 1000
    theta = _theta(n, H, 4, 0.3)
    net = _net([inst], "fp32", seed=0x1234_5678_9ABC)
    net.set_params(0, torch.from_numpy(theta))
    sp, _ = net.sample(B)
    sp = sp.cpu().numpy().reshape(B, n)
    u = OP.sampler_uniforms(0x1234_5678_9ABC, 0, 0, B, n)
    _check_spins(theta, u, n, H, sp)


@pytest.mark.parametrize("prec,split", [("fp64", False), ("fp32", False), ("fp32", True)])
def test_free_energy_step_parity(prec, split):
    from paper_2504_12037_amd import Net
    inst = S.c1_small_lattice(16)
    n, H, B = 4, 16, 1024
    seed, lr = 77, 1e-2
    theta = _theta(n, H, 5, 0.4)
    net = _net([inst], prec, seed=seed, flags=Net.FLAG_SPLIT_BF16 if split else 0)
    net.set_params(0, torch.from_numpy(theta))
    spins = torch.empty(B * n, dtype=torch.int8, device="cuda")
    stats, _ = net.free_energy_step(B, lr, spins_out=spins)
    torch.cuda.synchronize()
    sp = spins.cpu().numpy().reshape(B, n)
    u = OP.sampler_uniforms(seed, 0, 0, B, n)
    _check_spins(theta, u, n, H, sp)
    th64 = theta.astype(np.float64)
    lq = OM.logq(th64, sp, n, H)
    lz = OI.logz_r_bruteforce(inst, sp)
    f, st = OO.free_energy_terms(inst, sp, lq, lz)
    g = OM.logq_backward(th64, sp, OO.reinforce_weights(f), n, H)
    st_gpu = stats.cpu().numpy()[0]
    tol = 1e-9 if prec == "fp64" else 2e-5
    np.testing.assert_allclose(st_gpu, st, atol=tol * 10, rtol=tol)
    g_gpu = net.get_state(0, 1).cpu().numpy()
    assert np.abs(g_gpu - g).max() <= 1e-6 + 1e-4 * np.abs(g).max()
    th1, _, _ = OO.adam_step(th64, g_gpu.astype(np.float64), np.zeros_like(th64),
                             np.zeros_like(th64), 1, lr)
    np.testing.assert_allclose(net.get_params(0).cpu().numpy(), th1, atol=1e-6, rtol=0)
    # masked entries never move
    M1, M2, M0 = OM.masks(n, H)
    mask = OM.pack(M1, np.ones(H), M2, np.ones(n), M0)
    assert np.all(g_gpu[mask == 0] == 0)


def test_free_energy_step_multi_instance_and_training():
    insts = [S.c1_small_lattice(16), S.c3_sk(1.0, 32),
             S.lattice_column_split(S.lattice_2d(8, seed=2), [5], hidden=32)]
    Bs = [512, 256, 384]
    net = _net(insts, "fp32", seed=9)
    thetas = []
    for k, inst in enumerate(insts):
        th = _theta(inst.n_width, inst.hidden, 10 + k, 0.2)
        thetas.append(th)
        net.set_params(k, torch.from_numpy(th))
    spins = torch.empty(sum(b * i.n_width for b, i in zip(Bs, insts)), dtype=torch.int8,
                        device="cuda")
    stats, _ = net.free_energy_step(Bs, 1e-2, spins_out=spins)
    sp_all = spins.cpu().numpy()
    st_all = stats.cpu().numpy()
    off = 0
    for k, (inst, b) in enumerate(zip(insts, Bs)):
        n, H = inst.n_width, inst.hidden
        sp = sp_all[off:off + b * n].reshape(b, n)
        off += b * n
        u = OP.sampler_uniforms(9, 0, k, b, n)
        _check_spins(thetas[k], u, n, H, sp)
        lq = OM.logq(thetas[k].astype(np.float64), sp, n, H)
        lz = (OI.logz_r_bruteforce if len(inst.order) <= 16 else OI.logz_r_elimination)(inst, sp)
        _, st = OO.free_energy_terms(inst, sp, lq, lz)
        np.testing.assert_allclose(st_all[k], st, atol=2e-4, rtol=2e-5)
    # a short training run on the 4x4 workload lowers the exact F_q and stays
    # above the exact free energy (Eq. 5)
    inst = insts[0]
    net1 = _net([inst], "fp32", seed=3)
    th0 = S.made_init(4, 16, 0)
    net1.set_params(0, torch.from_numpy(th0))
    Fq0, _ = OO.exact_fq_and_grad(inst, th0.astype(np.float64), 16)
    for _ in range(60):
        net1.free_energy_step(256, 1e-2)
    th1 = net1.get_params(0).cpu().numpy().astype(np.float64)
    Fq1, _ = OO.exact_fq_and_grad(inst, th1, 16)
    F = OO.exact_free_energy(inst)
    assert F - 1e-9 <= Fq1 < Fq0


def test_free_energy_step_graph_replay():
    # the training step recorded once and replayed: every replay must equal
    # the eager step of an identical net; eager work on other batch shapes
    # (which moves the net's tables) runs between the replays
    from paper_2504_12037_amd import Net
    insts = [S.c1_small_lattice(16), S.lattice_column_split(S.lattice_2d(8, seed=2), [5], hidden=32),
             S.c2_lattice(1.0, 64)]
    Bs = [256, 384, 512]
    nets = [_net(insts, "fp32", seed=21), _net(insts, "fp32", seed=21, flags=Net.FLAG_GRAPH)]
    for net in nets:
        for k, inst in enumerate(insts):
            net.set_params(k, torch.from_numpy(_theta(inst.n_width, inst.hidden, 30 + k, 0.2)))
    stats = [torch.empty(len(insts), 4, dtype=torch.float64, device="cuda") for _ in nets]
    spins = [torch.empty(sum(b * i.n_width for b, i in zip(Bs, insts)), dtype=torch.int8,
                         device="cuda") for _ in nets]
    other = S.uniform_spins(100, insts[2].n_width, 5)
    for it in range(8):
        print(f"\n[graph] iteration {it}", flush=True)
        for net, st, sp in zip(nets, stats, spins):
            net.free_energy_step(Bs, 1e-2, stats=st, spins_out=sp)
        torch.cuda.synchronize()
        assert torch.equal(stats[0], stats[1]), (it, stats[0], stats[1])
        assert torch.equal(spins[0], spins[1])
        if it % 3 == 1:
            # eager work on another batch shape between replays
            lz = nets[1].logz(_dev(np.concatenate([S.uniform_spins(7, insts[0].n_width, 1).reshape(-1),
                                                   S.uniform_spins(9, insts[1].n_width, 2).reshape(-1),
                                                   other.reshape(-1)])), [7, 9, 100])
            torch.cuda.synchronize()
            assert torch.isfinite(lz).all()
    for k in range(len(insts)):
        assert torch.equal(nets[0].get_params(k), nets[1].get_params(k))


@pytest.mark.parametrize("graph,split,Bs", [(False, False, (512, 256)), (True, False, (512, 256)),
                                             (False, True, (512, 256)), (False, True, (300, 77))])
def test_training_steps_track_the_oracle(graph, split, Bs):
    # several iterations of Algorithm 1 on the GPU beside the FP64 oracle's
    # own run from the same start (its own spins, logZ, gradients and Adam
    # state).  Between steps the optimiser keeps the sampler's packed tables
    # current; a parameter upload in the middle restarts instance 0 (new
    # parameters, moments and step counter) and must take effect at once,
    # also for a recorded step.
    from paper_2504_12037_amd import Net
    insts = [S.c1_small_lattice(16),
             S.lattice_column_split(S.lattice_2d(12, seed=6), [5, 9], hidden=32)]
    Bs = list(Bs)
    seed, lr = 41, 1e-2
    net = _net(insts, "fp32", seed=seed, flags=(Net.FLAG_GRAPH if graph else 0) |
               (Net.FLAG_SPLIT_BF16 if split else 0))
    ora = []

    def restart(k, th):
        net.set_params(k, torch.from_numpy(th))
        z = np.zeros(th.shape, np.float64)
        if k < len(ora):
            ora[k] = [th.astype(np.float64), z, z.copy(), 0]
        else:
            ora.append([th.astype(np.float64), z, z.copy(), 0])

    for k, inst in enumerate(insts):
        restart(k, _theta(inst.n_width, inst.hidden, 60 + k, 0.2))
    spins = torch.empty(sum(b * i.n_width for b, i in zip(Bs, insts)), dtype=torch.int8,
                        device="cuda")
    stats = torch.empty(len(insts), 4, dtype=torch.float64, device="cuda")
    ties = 0
    for it in range(6):
        if it == 3:
            restart(0, _theta(insts[0].n_width, insts[0].hidden, 70, 0.3))
        print(f"\n[train] graph={graph} split={split} iteration {it}", flush=True)
        net.free_energy_step(Bs, lr, stats=stats, spins_out=spins)
        torch.cuda.synchronize()
        sp_all, st_all = spins.cpu().numpy(), stats.cpu().numpy()
        off = 0
        for k, (inst, b) in enumerate(zip(insts, Bs)):
            n, H = inst.n_width, inst.hidden
            sp = sp_all[off:off + b * n].reshape(b, n)
            off += b * n
            th, m, v, t = ora[k]
            u = OP.sampler_uniforms(seed, t, k, b, n)
            nt, lq = _check_spins(th, u, n, H, sp)
            ties += nt
            lz = (OI.logz_r_bruteforce if len(inst.order) <= 16 else OI.logz_r_elimination)(inst, sp)
            f, st = OO.free_energy_terms(inst, sp, lq, lz)
            np.testing.assert_allclose(st_all[k], st, atol=2e-4, rtol=2e-5)
            g = OM.logq_backward(th, sp, OO.reinforce_weights(f), n, H)
            g_gpu = net.get_state(k, 1).cpu().numpy()
            assert np.abs(g_gpu - g).max() <= 1e-6 + 1e-4 * np.abs(g).max(), (it, k)
            th, m, v = OO.adam_step(th, g, m, v, t + 1, lr)
            ora[k] = [th, m, v, t + 1]
            d = np.abs(net.get_params(k).cpu().numpy() - th).max()
            print(f"[train] it={it} inst={k} max|theta_gpu - theta_oracle|={d:.2e}", flush=True)
            assert d <= 1e-4, (it, k, d)
    print(f"[train] near-ties adopted: {ties}", flush=True)


def test_packed_tables_after_training_equal_a_fresh_pack():
    # the sampler after optimiser steps (tables written by the optimiser)
    # equals, bit for bit, the sampler of a net given the same parameters
    # (tables packed from scratch), on the same uniforms
    insts = [S.c1_small_lattice(16),
             S.lattice_column_split(S.lattice_2d(12, seed=6), [5, 9], hidden=32)]
    Bs = [300, 200]
    a = _net(insts, "fp32", seed=5)
    for k, inst in enumerate(insts):
        a.set_params(k, torch.from_numpy(_theta(inst.n_width, inst.hidden, 80 + k, 0.2)))
    for _ in range(3):
        a.free_energy_step(Bs, 2e-2)
    b = _net(insts, "fp32", seed=5)
    for k in range(len(insts)):
        b.set_params(k, a.get_params(k))
    u = _dev(np.concatenate([S.uniforms(bb, i.n_width, 90 + k).reshape(-1)
                             for k, (bb, i) in enumerate(zip(Bs, insts))]))
    sa, la = a.sample(Bs, u)
    sb, lb = b.sample(Bs, u)
    torch.cuda.synchronize()
    assert torch.equal(sa, sb) and torch.equal(la, lb)


def test_reinforce_gradient_full_width_split_products():
    # the 16x16 lattice workload's network (|W| = 32, H = 256) with
    # split-BF16 products: one step's statistics and REINFORCE gradient
    # against the oracle on the step's own samples
    from paper_2504_12037_amd import Net
    inst = S.c2_lattice(1.0)
    n, H, B = 32, 256, 2048
    seed, lr = 19, 1e-3
    theta = _theta(n, H, 6, 0.05)
    net = _net([inst], "fp32", seed=seed, flags=Net.FLAG_SPLIT_BF16)
    net.set_params(0, torch.from_numpy(theta))
    spins = torch.empty(B * n, dtype=torch.int8, device="cuda")
    print("\n[split-grad] C2 network, 2048 samples", flush=True)
    stats, _ = net.free_energy_step(B, lr, spins_out=spins)
    torch.cuda.synchronize()
    sp = spins.cpu().numpy().reshape(B, n)
    u = OP.sampler_uniforms(seed, 0, 0, B, n)
    _, lq = _check_spins(theta, u, n, H, sp)
    lz = OI.logz_r_elimination(inst, sp)
    f, st = OO.free_energy_terms(inst, sp, lq, lz)
    np.testing.assert_allclose(stats.cpu().numpy()[0], st, atol=2e-4, rtol=2e-5)
    g = OM.logq_backward(theta.astype(np.float64), sp, OO.reinforce_weights(f), n, H)
    g_gpu = net.get_state(0, 1).cpu().numpy()
    err = np.abs(g_gpu - g).max() / np.abs(g).max()
    print(f"[split-grad] max |g_gpu - g| / max |g| = {err:.2e}", flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("prec,split", [("fp32", True), ("fp32", False), ("fp64", False)])
def test_training_with_an_instance_left_empty(prec, split):
    # an instance with no samples in some steps keeps its parameters, Adam
    # moments and step counter, and gets a zero statistics row; its next real
    # step is the oracle's next Adam step (bias corrections of step t + 1)
    from paper_2504_12037_amd import Net
    insts = [S.c1_small_lattice(16),
             S.lattice_column_split(S.lattice_2d(12, seed=6), [5, 9], hidden=32)]
    seed, lr = 43, 1e-2
    net = _net(insts, prec, seed=seed, flags=Net.FLAG_SPLIT_BF16 if split else 0)
    ora = []
    for k, inst in enumerate(insts):
        th = _theta(inst.n_width, inst.hidden, 90 + k, 0.2)
        net.set_params(k, torch.from_numpy(th))
        z = np.zeros(th.shape, np.float64)
        ora.append([th.astype(np.float64), z, z.copy(), 0])
    stats = torch.empty(len(insts), 4, dtype=torch.float64, device="cuda")
    for it, Bs in enumerate([(256, 128), (256, 0), (192, 0), (256, 160)]):
        print(f"\n[train-empty] prec={prec} split={split} iteration {it} B={Bs}", flush=True)
        spins = torch.empty(max(1, sum(b * i.n_width for b, i in zip(Bs, insts))),
                            dtype=torch.int8, device="cuda")
        stats.fill_(np.nan)
        net.free_energy_step(list(Bs), lr, stats=stats, spins_out=spins)
        torch.cuda.synchronize()
        sp_all, st_all = spins.cpu().numpy(), stats.cpu().numpy()
        off = 0
        for k, (inst, b) in enumerate(zip(insts, Bs)):
            n, H = inst.n_width, inst.hidden
            th, m, v, t = ora[k]
            if b == 0:
                assert np.all(st_all[k] == 0.0), st_all[k]
            else:
                sp = sp_all[off:off + b * n].reshape(b, n)
                off += b * n
                u = OP.sampler_uniforms(seed, t, k, b, n)
                _, lq = _check_spins(th, u, n, H, sp)
                lz = (OI.logz_r_bruteforce if len(inst.order) <= 16
                      else OI.logz_r_elimination)(inst, sp)
                f, st = OO.free_energy_terms(inst, sp, lq, lz)
                np.testing.assert_allclose(st_all[k], st, atol=2e-4, rtol=2e-5)
                g = OM.logq_backward(th, sp, OO.reinforce_weights(f), n, H)
                th, m, v = OO.adam_step(th, g, m, v, t + 1, lr)
                ora[k] = [th, m, v, t + 1]
            d = np.abs(net.get_params(k).cpu().numpy() - th).max()
            dm = np.abs(net.get_state(k, 2).cpu().numpy() - m).max()
            assert d <= 1e-4 and dm <= 1e-5, (it, k, d, dm)


@pytest.mark.parametrize("graph", [False, True])
def test_nonfinite_free_energy_is_reported(graph):
    # one NaN parameter makes every f_b of its instance NaN: with
    # TNVAN_FLAG_CHECK_FINITE the step reports TNVAN_E_NONFINITE (eager and
    # replayed), the flag clears, and finite parameters step normally again
    from paper_2504_12037_amd import Net, TnvanError
    insts = [S.c1_small_lattice(16), S.lattice_column_split(S.lattice_2d(8, seed=2), [5], hidden=16)]
    Bs = [256, 128]
    flags = Net.FLAG_CHECK_FINITE | (Net.FLAG_GRAPH if graph else 0)
    net = _net(insts, "fp32", seed=5, flags=flags)
    good = [_theta(i.n_width, i.hidden, 20 + k, 0.1) for k, i in enumerate(insts)]
    for k, th in enumerate(good):
        net.set_params(k, torch.from_numpy(th))
    for _ in range(3):
        net.free_energy_step(Bs, 1e-3)
    bad = good[1].copy()
    n1, H1 = insts[1].n_width, insts[1].hidden
    bad[H1 * n1 + H1 + n1 * H1] = np.nan      # b2[0], the first logit's bias
    net.set_params(1, torch.from_numpy(bad))
    print(f"\n[nonfinite] graph={graph}", flush=True)
    for _ in range(2):      # eager (and recorded), then replayed
        with pytest.raises(TnvanError) as e:
            net.free_energy_step(Bs, 1e-3)
        assert e.value.code == 6 and "instance 1" in str(e.value)
    net.set_params(1, torch.from_numpy(good[1]))
    stats, _ = net.free_energy_step(Bs, 1e-3)
    assert np.all(np.isfinite(stats.cpu().numpy()))
    # without the flag the step does not look
    plain = _net(insts, "fp32", seed=5)
    for k, th in enumerate(good):
        plain.set_params(k, torch.from_numpy(th))
    plain.set_params(1, torch.from_numpy(bad))
    st2, _ = plain.free_energy_step(Bs, 1e-3)
    assert np.isnan(st2.cpu().numpy()[1, 0])


@pytest.mark.parametrize("prec,split", [("fp32", True), ("fp64", False)])
def test_checkpoint_and_resume_bit_for_bit(prec, split):
    # Algorithm 1 resumed from a checkpoint (parameters, Adam moments, step
    # counter) in a new net continues exactly as the uninterrupted run
    from paper_2504_12037_amd import Net
    insts = [S.c1_small_lattice(16),
             S.lattice_column_split(S.lattice_2d(12, seed=6), [5, 9], hidden=32)]
    Bs = [384, 256]
    fl = Net.FLAG_SPLIT_BF16 if split else 0
    a = _net(insts, prec, seed=77, flags=fl)
    for k, inst in enumerate(insts):
        a.set_params(k, torch.from_numpy(_theta(inst.n_width, inst.hidden, 40 + k, 0.2)))
    for _ in range(3):
        a.free_energy_step(Bs, 1e-2)
    ck = a.checkpoint()
    assert [c[3] for c in ck] == [3, 3]
    b = _net(insts, prec, seed=77, flags=fl)
    b.restore(ck)
    print(f"\n[resume] prec={prec} split={split}", flush=True)
    for it in range(3):
        sa, _ = a.free_energy_step(Bs, 1e-2)
        sb, _ = b.free_energy_step(Bs, 1e-2)
        torch.cuda.synchronize()
        assert torch.equal(sa, sb), it
    for k in range(len(insts)):
        for which in (0, 2, 3):
            assert torch.equal(a.get_state(k, which), b.get_state(k, which)), (k, which)
        assert a.get_step(k) == b.get_step(k) == 6


def test_c1_as_configured_fp64_training():
    # the 4x4 workload as specified: FP64 path, 1024 samples, hidden 16,
    # 200 Adam steps at lr 1e-3; the exact F_q of the trained network
    # (enumeration of its 16 width-set states) lies between F (2^16-state
    # enumeration, Eq. 5) and the exact F_q it started from
    inst = S.c1_small_lattice(16)
    net = _net([inst], "fp64", seed=1)
    th0 = S.made_init(4, 16, 3)
    net.set_params(0, torch.from_numpy(th0))
    stats = torch.empty(1, 4, dtype=torch.float64, device="cuda")
    print("\n[c1] 200 FP64 training steps", flush=True)
    for _ in range(200):
        net.free_energy_step(1024, 1e-3, stats=stats)
    th = net.get_params(0).cpu().numpy().astype(np.float64)
    F = OO.exact_free_energy(inst)
    Fq0, _ = OO.exact_fq_and_grad(inst, th0.astype(np.float64), 16)
    Fq1, _ = OO.exact_fq_and_grad(inst, th, 16)
    print(f"[c1] F = {F:.6f}, exact F_q {Fq0:.6f} -> {Fq1:.6f}", flush=True)
    assert F - 1e-12 <= Fq1 < Fq0
    assert net.get_step(0) == 200
    # the last batch estimate is within 5 standard errors of the exact F_q
    st = stats.cpu().numpy()[0]
    assert abs(st[0] - Fq1) <= 5 * st[1] + 1e-9
