"""Auxiliary subsystems on the GPU: roctx phase markers change nothing, the
per-step JSON-lines log of the training driver, repeated runs equal bit for
bit, the autotuner's cache path from the environment."""

import json
import os

import numpy as np
import pytest

import synthetic as S
from oracle import objective as OO

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _nets(insts, **kw):
    from paper_2504_12037_amd import Net
    return Net(insts, **kw)


def _setup(net, insts, seed=3):
    for k, inst in enumerate(insts):
        net.set_params(k, torch.from_numpy(S.made_init(inst.n_width, inst.hidden, seed + k)))


@pytest.mark.parametrize("prec,flags", [("fp32", 8), ("fp64", 0)])
def test_markers_change_nothing_and_runs_repeat_bit_for_bit(prec, flags):
    from paper_2504_12037_amd import Net
    insts = [S.c1_small_lattice(16), S.lattice_column_split(S.lattice_2d(8, seed=2), [5], hidden=32),
             S.c4_small_copies()[0]]
    Bs = [256, 300, 77]
    print(f"\n[aux] prec={prec} flags={flags}", flush=True)
    nets = [_nets(insts, precision=prec, seed=5, flags=flags | Net.FLAG_MARKERS),
            _nets(insts, precision=prec, seed=5, flags=flags),
            _nets(insts, precision=prec, seed=5, flags=flags)]
    sp = torch.from_numpy(np.concatenate([S.uniform_spins(b, i.n_width, 9 + k).reshape(-1)
                                          for k, (b, i) in enumerate(zip(Bs, insts))])).cuda()
    g = torch.from_numpy(np.random.default_rng(1).standard_normal(sum(Bs))).cuda()
    outs, stats = [], []
    for net in nets:
        _setup(net, insts)
        outs.append([t.clone() for t in net.logz_and_backward(sp, g, Bs)])
        st = torch.empty(len(insts), 4, dtype=torch.float64, device="cuda")
        for _ in range(3):
            net.free_energy_step(Bs, 1e-2, stats=st)
        stats.append(st.clone())
    torch.cuda.synchronize()
    for k in (1, 2):
        for a, b in zip(outs[0], outs[k]):
            assert torch.equal(a, b)
        assert torch.equal(stats[0], stats[k])
        for q in range(len(insts)):
            assert torch.equal(nets[0].get_params(q), nets[k].get_params(q))


def test_training_log_jsonl(tmp_path):
    from paper_2504_12037_amd.train import train
    inst = S.c1_small_lattice(16)
    log = tmp_path / "run.jsonl"
    F = OO.exact_free_energy(inst)
    net = _nets([inst], precision="fp32", seed=11)
    ref = _nets([inst], precision="fp32", seed=11)
    _setup(net, [inst])
    _setup(ref, [inst])
    hist = train(net, 512, lr=1e-2, steps=12, log=str(log), every=3, grad_every=2, exact_F=[F])
    lines = [json.loads(x) for x in open(log)]
    assert lines == hist and [r["step"] for r in lines] == [3, 6, 9, 12]
    assert lines[0]["grad_norm"] is not None and lines[1]["grad_norm"] is None
    assert lines[2]["grad_norm"][0] > 0
    # the logged statistics are those of the net's own steps
    st = torch.empty(1, 4, dtype=torch.float64, device="cuda")
    for it in range(12):
        ref.free_energy_step(512, 1e-2, stats=st)
        if (it + 1) % 3 == 0:
            rec = lines[(it + 1) // 3 - 1]
            assert rec["F_q"][0] == float(st[0, 0]) and rec["stderr"][0] == float(st[0, 1])
            assert abs(rec["F_q_per_spin"][0] - float(st[0, 0]) / inst.n) < 1e-15
    # Eq. 5 on the sampled F_q, within its noise
    for rec in lines:
        assert rec["F_q"][0] >= F - 5 * rec["stderr"][0] - 1e-9
        assert rec["rel_gap"][0] == pytest.approx((rec["F_q"][0] - F) / abs(F))
    assert net.get_step(0) == 12


def test_autotune_cache_from_the_environment(tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("TNVAN_AUTOTUNE_CACHE", str(cache))
    inst = S.c4_small_copies()[1]
    net = _nets([inst], precision="fp32")
    B = 200
    sp = torch.from_numpy(S.uniform_spins(B, inst.n_width, 4)).cuda().reshape(-1)
    g = torch.full((B,), 1.0 / B, dtype=torch.float64, device="cuda")
    net.autotune(sp, g, B)
    assert cache.exists() and json.loads(cache.read_text())
