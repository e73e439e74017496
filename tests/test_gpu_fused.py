"""logZ and its adjoint in one call (tnvan_logz_and_backward) and the
training step with the adjoint of its own samples
(tnvan_free_energy_step_adjoint), through the C ABI.

Where the net allows a single contraction (FP32, every instance on the
register-resident chain kernels) logZ comes from the adjoint's forward pass,
which does the forward kernel's arithmetic step for step; elsewhere the two
calls are made in turn.  Either way the results must equal those of the
separate calls bit for bit, and logZ is also checked against the oracle."""

import numpy as np
import pytest

import synthetic as S
from oracle import ising as OI

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 1e-3}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().reshape(-1)


def _net(insts, prec, **kw):
    from paper_2504_12037_amd import Net
    return Net(insts, precision=prec, **kw)


CASES = {
    "c1": lambda: [S.c1_small_lattice()],
    "c2_b2": lambda: [S.c2_lattice(2.0)],
    "lat8_field": lambda: [S.lattice_column_split(S.lattice_2d(8, seed=9, h_var=0.2), [5])],
    "c3_b1": lambda: [S.c3_sk(1.0)],
    "c4": lambda: [S.c4_small_copies()[0]],
    "mixed": lambda: [S.c1_small_lattice(), S.c4_small_copies()[1],
                      S.lattice_column_split(S.lattice_2d(8, seed=3), [5])],
    "chains3": lambda: [S.c2_lattice(0.5, 64), S.c1_small_lattice(16),
                        S.lattice_column_split(S.lattice_2d(8, seed=4), [5], hidden=32)],
}


def _oracle_logz(inst, spins):
    if len(inst.order) <= 16:
        return OI.logz_r_bruteforce(inst, spins)
    return OI.logz_r_elimination(inst, spins)


@pytest.mark.parametrize("flags", [0, 1, 8])
@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16"])
@pytest.mark.parametrize("case", list(CASES))
def test_logz_and_backward_equals_separate_calls(case, prec, flags):
    insts = CASES[case]()
    Bs = [229 + 37 * k for k in range(len(insts))]
    print(f"\n[fused] case={case} prec={prec} flags={flags} B={Bs}", flush=True)
    spins = [S.uniform_spins(b, i.n_width, 40 + k) for k, (b, i) in enumerate(zip(Bs, insts))]
    flat = _dev(np.concatenate([s.reshape(-1) for s in spins]))
    g = _dev(np.random.default_rng(sum(Bs)).standard_normal(sum(Bs)))
    net = _net(insts, prec, flags=flags)
    lz, dh, dJ, db = net.logz_and_backward(flat, g, Bs)
    lz1 = net.logz(flat, Bs)
    dh1, dJ1, db1 = net.backward(flat, g, Bs)
    torch.cuda.synchronize()
    assert torch.equal(lz, lz1), (lz - lz1).abs().max().item()
    assert torch.equal(dh, dh1) and torch.equal(dJ, dJ1) and torch.equal(db, db1)
    # and logZ against the oracle (first 64 samples of each instance)
    got = lz.cpu().numpy()
    off = 0
    for inst, b, s in zip(insts, Bs, spins):
        want = _oracle_logz(inst, s[:64])
        assert np.abs(got[off:off + 64] - want).max() / inst.n <= TOL[prec]
        off += b


def test_logz_and_backward_full_size():
    # the benchmark workload at its full batch in one call: logZ equals the
    # separate forward bit for bit, sampled outputs against the oracle
    insts = [S.c2_lattice(b) for b in (0.5, 1.0, 2.0)]
    B = 8192
    sp = S.uniform_spins(3 * B, 32, 102)
    flat = _dev(sp)
    g = torch.full((3 * B,), 1.0 / B, dtype=torch.float64, device="cuda")
    net = _net(insts, "fp32")
    lz, dh, dJ, db = net.logz_and_backward(flat, g, [B] * 3)
    lz1 = net.logz(flat, [B] * 3)
    dh1, dJ1, db1 = net.backward(flat, g, [B] * 3)
    torch.cuda.synchronize()
    assert torch.equal(lz, lz1)
    assert torch.equal(dh, dh1) and torch.equal(dJ, dJ1) and torch.equal(db, db1)
    got = lz.cpu().numpy()
    idx = np.random.default_rng(5).choice(B, 32, replace=False)
    for k, inst in enumerate(insts):
        want = OI.logz_r_elimination(inst, sp[k * B + idx])
        assert np.abs(got[k * B + idx] - want).max() / inst.n <= TOL["fp32"]


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("case", ["chains3", "mixed"])
def test_free_energy_step_adjoint_equals_step_then_backward(case, graph, split):
    from paper_2504_12037_amd import Net
    insts = CASES[case]()
    Bs = [256, 128, 384][:len(insts)]
    print(f"\n[step-adjoint] case={case} graph={graph} split={split} B={Bs}", flush=True)
    sf = Net.FLAG_SPLIT_BF16 if split else 0
    nets = [_net(insts, "fp32", seed=33, flags=sf),
            _net(insts, "fp32", seed=33, flags=sf | (Net.FLAG_GRAPH if graph else 0))]
    for net in nets:
        for k, inst in enumerate(insts):
            th = S.made_init(inst.n_width, inst.hidden, 50 + k).astype(np.float32)
            net.set_params(k, torch.from_numpy(th))
    nB = sum(Bs)
    nsp = sum(b * i.n_width for b, i in zip(Bs, insts))
    g = torch.cat([torch.full((b,), 1.0 / b, dtype=torch.float64, device="cuda") for b in Bs])
    stats = [torch.empty(len(insts), 4, dtype=torch.float64, device="cuda") for _ in nets]
    spins = [torch.empty(nsp, dtype=torch.int8, device="cuda") for _ in nets]
    adj = (g, torch.empty(sum(i.n for i in insts), dtype=torch.float64, device="cuda"),
           torch.empty(sum(i.n_edges for i in insts), dtype=torch.float64, device="cuda"),
           torch.empty(len(insts), dtype=torch.float64, device="cuda"))
    for it in range(4):
        print(f"[step-adjoint] iteration {it}", flush=True)
        nets[0].free_energy_step(Bs, 1e-2, stats=stats[0], spins_out=spins[0])
        dh0, dJ0, db0 = nets[0].backward(spins[0], g, Bs)
        nets[1].free_energy_step(Bs, 1e-2, stats=stats[1], spins_out=spins[1], adjoint=adj)
        torch.cuda.synchronize()
        assert torch.equal(spins[0], spins[1]), it
        assert torch.equal(stats[0], stats[1]), (it, stats[0], stats[1])
        assert torch.equal(dh0, adj[1]) and torch.equal(dJ0, adj[2][:dJ0.numel()])
        assert torch.equal(db0, adj[3])
    for k in range(len(insts)):
        assert torch.equal(nets[0].get_params(k), nets[1].get_params(k))
    # the step's logZ against the oracle: F_q's energy part uses it, so check
    # one instance's logZ of the last sampled spins directly
    sp = spins[1][:Bs[0] * insts[0].n_width].cpu().numpy().reshape(Bs[0], insts[0].n_width)
    lz = nets[1].logz(spins[1], Bs).cpu().numpy()[:Bs[0]]
    want = _oracle_logz(insts[0], sp[:48])
    assert np.abs(lz[:48] - want).max() / insts[0].n <= TOL["fp32"]


def test_profile_mask_times_only_the_chosen_kernels():
    from paper_2504_12037_amd import Net
    insts = [S.c2_lattice(1.0, 64)]
    net = _net(insts, "fp32", seed=3, flags=Net.FLAG_PROFILE)
    net.profile_only(["chain_bwd_2"])
    g = torch.full((512,), 1.0 / 512, dtype=torch.float64, device="cuda")
    adj = (g, torch.empty(insts[0].n, dtype=torch.float64, device="cuda"),
           torch.empty(insts[0].n_edges, dtype=torch.float64, device="cuda"),
           torch.empty(1, dtype=torch.float64, device="cuda"))
    for _ in range(2):
        net.free_energy_step(512, 1e-3, adjoint=adj)
    torch.cuda.synchronize()
    tot, n = net.kernel_time("chain_bwd_2")
    assert n == 2 and tot > 0
    assert net.kernel_time("sample") == (0.0, 0)
    assert net.kernel_time("made_grad") == (0.0, 0)
