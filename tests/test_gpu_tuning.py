"""Launch shapes and the autotuner (tnvan_set_tuning, tnvan_autotune)
through the C ABI.

A launch shape changes how the samples are tiled, not what is computed per
sample: logZ must be the same bit for bit under every shape, and the
adjoint (whose batch sums run in tile order) must meet the error model of
adjtol.py against the oracle.  The autotuner must apply its choice, report
it, and read it back from its cache."""

import json

import numpy as np
import pytest

import synthetic as S
from adjtol import check_vjp
from oracle import ising as OI

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().reshape(-1)


def _mixed():
    # a general-step instance (random regular graph with fields) and a
    # lattice on the register-resident chain kernels
    return [S.c4_small_copies(limit=3)[2], S.c4_rrg(),
            S.lattice_column_split(S.lattice_2d(8, seed=4, h_var=0.1), [5])]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_every_launch_shape_keeps_parity(prec):
    from paper_2504_12037_amd import Net
    insts = _mixed()
    Bs = [300, 517, 1000]
    sp = [S.uniform_spins(b, i.n_width, 31 + k) for k, (b, i) in enumerate(zip(Bs, insts))]
    flat = _dev(np.concatenate([x.reshape(-1) for x in sp]))
    g = np.concatenate([np.random.default_rng(k).standard_normal(b) for k, b in enumerate(Bs)])
    net = Net(insts, precision=prec)
    ref = net.logz(flat, Bs).clone()
    wants = [OI.logz_r_vjp(inst, s, g[sum(Bs[:k]):sum(Bs[:k + 1])])
             for k, (inst, s) in enumerate(zip(insts, sp))]
    shapes = [dict(general_tile_fwd=t, general_tile_bwd=u, chain_groups=c)
              for t, u, c in [(1, 1, 1), (4, 2, 2), (16, 8, 1), (64, 64, 2), (2, 32, 0)]]
    from paper_2504_12037_amd import TnvanError
    tried = 0
    for sh in shapes:
        print(f"\n[tuning] prec={prec} {sh}", flush=True)
        before = net.get_tuning()
        try:
            net.set_tuning(**sh)
        except TnvanError as e:
            # a tile whose LDS part does not fit: refused, nothing changed
            assert e.code == 1 and net.get_tuning() == before
            continue
        tried += 1
        got = net.get_tuning()
        for k in ("general_tile_fwd", "general_tile_bwd"):
            assert got[k] == sh[k]
        assert torch.equal(net.logz(flat, Bs), ref)
        dh, dJ, db = (x.cpu().numpy() for x in net.backward(flat, _dev(g), Bs))
        ho = eo = so = 0
        for k, (inst, b) in enumerate(zip(insts, Bs)):
            check_vjp((dh[ho:ho + inst.n], dJ[eo:eo + inst.n_edges], db[k]), wants[k], inst,
                      g[so:so + b], prec, (sh, k))
            ho += inst.n
            eo += inst.n_edges
            so += b
    assert tried >= 3


def test_set_tuning_refuses_bad_shapes():
    from paper_2504_12037_amd import Net, TnvanError
    net = Net([S.c4_rrg()], precision="fp32")
    before = net.get_tuning()
    for bad in (dict(general_tile_fwd=3), dict(general_tile_bwd=128), dict(chain_groups=3)):
        with pytest.raises(TnvanError):
            net.set_tuning(**bad)
    assert net.get_tuning() == before


def test_autotune_applies_and_caches(tmp_path):
    from paper_2504_12037_amd import Net
    insts = _mixed()
    Bs = [256, 4096, 2048]
    sp = [S.uniform_spins(b, i.n_width, 61 + k) for k, (b, i) in enumerate(zip(Bs, insts))]
    flat = _dev(np.concatenate([x.reshape(-1) for x in sp]))
    g = _dev(np.concatenate([np.full(b, 1.0 / b) for b in Bs]))
    cache = tmp_path / "tune.json"
    net = Net(insts, precision="fp32", flags=Net.FLAG_SPLIT_BF16)
    print("\n[autotune] timing", flush=True)
    chosen = net.autotune(flat, g, Bs, cache_path=cache)
    print(f"[autotune] chosen {chosen}", flush=True)
    got = net.get_tuning()
    assert got == chosen
    assert chosen["kinds"] == 3
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.startswith("gfx950") and "fp32+split" in key
    # results after tuning, against the oracle
    lz = net.logz(flat, Bs).cpu().numpy()
    off = 0
    for inst, b, s in zip(insts, Bs, sp):
        want = OI.logz_r_elimination(inst, s[:40])
        assert np.abs(lz[off:off + 40] - want).max() / inst.n <= 1e-5
        off += b
    # a second net of the same signature takes the cached shapes
    net2 = Net(insts, precision="fp32", flags=Net.FLAG_SPLIT_BF16)
    again = net2.autotune(flat, g, Bs, cache_path=cache)
    for k in ("general_tile_fwd", "general_tile_bwd", "chain_groups"):
        if val[k]:
            assert again[k] == val[k]
    assert json.loads(cache.read_text()) == entries


def _uneven():
    # lattices of three chain widths, random regular graphs (general steps)
    # and an empty instance, with uneven batches
    insts = [S.c2_lattice(1.0, 32), S.c1_small_lattice(16), S.c4_rrg(),
             S.lattice_column_split(S.lattice_2d(8, seed=4, h_var=0.1), [5], hidden=16),
             S.c4_small_copies(limit=3)[3], S.lattice_column_split(S.lattice_2d(12, seed=8), [5, 9], hidden=16)]
    for i in insts:
        if not i.hidden:
            i.hidden = 8
    return insts, [1000, 333, 517, 0, 129, 2048]


@pytest.mark.parametrize("prec,split", [("fp32", True), ("fp32", False), ("bf16", False), ("fp64", False)])
def test_persistent_launches_equal_per_tile_launches(prec, split):
    # every (instance, tile or chain, sample group) item writes only its own
    # outputs, so the persistent work-queue launches give the same logZ and
    # adjoint bit for bit; called repeatedly (the queue counters reset)
    from paper_2504_12037_amd import Net
    insts, Bs = _uneven()
    sp = [S.uniform_spins(b, i.n_width, 140 + k) for k, (b, i) in enumerate(zip(Bs, insts))]
    flat = _dev(np.concatenate([x.reshape(-1) for x in sp]))
    g = _dev(np.concatenate([np.random.default_rng(k).standard_normal(b) for k, b in enumerate(Bs)]))
    fl = Net.FLAG_SPLIT_BF16 if split else 0
    ref_net = Net(insts, precision=prec, flags=fl)
    ref = [x.clone() for x in ref_net.logz_and_backward(flat, g, Bs)]
    ref_f = ref_net.logz(flat, Bs).clone()
    net = Net(insts, precision=prec, flags=fl)
    net.set_tuning(launch_mode=2)
    assert net.get_tuning()["launch_mode"] == 2
    print(f"\n[persistent] prec={prec} split={split}", flush=True)
    for rep in range(3):
        out = net.logz_and_backward(flat, g, Bs)
        for a, b in zip(out, ref):
            assert torch.equal(a, b), rep
        assert torch.equal(net.logz(flat, Bs), ref_f)
    lz = ref_f.cpu().numpy()
    off = 0
    for inst, b, s in zip(insts, Bs, sp):
        if b:
            want = OI.logz_r_elimination(inst, s[:24])
            tol = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 1e-3}[prec]
            assert np.abs(lz[off:off + 24] - want).max() / inst.n <= tol
        off += b


def test_persistent_training_step_replayed():
    # the recorded training step with the adjoint in persistent launches,
    # replayed, equals the eager per-tile step bit for bit
    from paper_2504_12037_amd import Net
    insts, Bs = _uneven()
    runs = []
    for mode, flags in ((1, 0), (2, Net.FLAG_GRAPH)):
        net = Net(insts, precision="fp32", seed=4, flags=Net.FLAG_SPLIT_BF16 | flags)
        net.set_tuning(launch_mode=mode)
        for q, inst in enumerate(insts):
            net.set_params(q, torch.from_numpy(S.made_init(inst.n_width, inst.hidden, 30 + q)))
        g = torch.cat([torch.full((b,), 1.0 / max(b, 1), dtype=torch.float64, device="cuda")
                       for b in Bs])
        adj = (g,) + net._adjoint_out(None)
        res = []
        for it in range(4):
            print(f"\n[persistent-step] mode={mode} it={it}", flush=True)
            st, _ = net.free_energy_step(Bs, 1e-2, adjoint=adj)
            res.append([st.clone()] + [a.clone() for a in adj[1:]])
        torch.cuda.synchronize()
        runs.append(res)
    for it, (a, b) in enumerate(zip(runs[0], runs[1])):
        for x, y in zip(a, b):
            assert torch.equal(x, y), it


def _wide16():
    # random 3-regular graph, n = 100, planned at w_u = 16: single-spin steps
    # of up to 16-spin scopes, whose arenas are in device memory
    from paper_2504_12037_amd import plan_width_set
    from synthetic import instances as SI
    e = SI.random_regular_edges(100, 3, np.random.default_rng(3))
    W, order, width, _ = plan_width_set(100, e, 16)
    assert width == 16
    rng = np.random.default_rng(8)
    return S.Instance(100, e.astype(np.int32), rng.choice([-1.0, 1.0], len(e)),
                      rng.normal(0.0, 0.3, 100), 0.7, W.astype(np.int32),
                      order.astype(np.int32), None, 0, "rrg100_wu16")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_arena_limit_runs_the_batch_in_chunks(prec):
    # a 1 MiB limit leaves one resident workgroup, which takes every tile in
    # turn: the same per-tile arithmetic in the same tile order, so logZ and
    # the adjoint are unchanged bit for bit
    from paper_2504_12037_amd import Net
    inst = _wide16()
    B = 300
    sp = S.uniform_spins(B, inst.n_width, 41)
    flat = _dev(sp)
    g = _dev(np.random.default_rng(7).standard_normal(B))
    outs = []
    for lim in (0, 1):
        print(f"\n[arena-limit] prec={prec} limit={lim}", flush=True)
        net = Net([inst], precision=prec, max_width=20)
        net.set_tuning(arena_limit_mib=lim)
        assert net.get_tuning()["arena_limit_mib"] == lim
        outs.append([net.logz(flat, B).clone()] +
                    [x.clone() for x in net.logz_and_backward(flat, g, B)])
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    want = OI.logz_r_elimination(inst, sp[:6], chunk=1)
    tol = {"fp64": 1e-10, "fp32": 1e-5}[prec]
    assert np.abs(outs[0][0].cpu().numpy()[:6] - want).max() / inst.n <= tol
