"""The adjoint of one-tile chains split between two waves (forward pass of
the first ceil(T/2) steps on one, the backward vectors of the others on the
second, joined at the meeting step by out . R = 1) through the C ABI against
the FP64 oracle: chains of 1, 2, 3, 4 and 5 steps with fields, in one net
with uneven batches and partial sample groups, in every product form; the
persistent launch, where one wave takes both roles in turn, equals the
two-wave launch bit for bit."""

import numpy as np
import pytest

import synthetic as S
from adjtol import check_vjp
from oracle import ising as OI
from synthetic.instances import Instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 1e-3}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().reshape(-1)


def _row(n, seed):
    # a path of n spins, W = the even ones: every R spin is a one-row strip
    rng = np.random.default_rng(seed)
    e = np.array([(i, i + 1) for i in range(n - 1)], np.int32)
    W = np.arange(0, n, 2, dtype=np.int32)
    R = np.arange(1, n, 2, dtype=np.int32)
    return Instance(n, e, rng.standard_normal(len(e)), rng.normal(0.0, 0.5, n), 0.8, W, R,
                    np.arange(len(R) + 1, dtype=np.int32), 8, f"path{n}")


def _short():
    return [S.lattice_column_split(S.lattice_2d(2, seed=3, h_var=0.3), [1], hidden=8),
            S.lattice_column_split(S.lattice_2d(3, seed=4, h_var=0.3), [2], hidden=8),
            S.lattice_column_split(S.lattice_2d(5, seed=5, beta=1.5, h_var=0.2), [3], hidden=8),
            S.c1_small_lattice(8),
            _row(7, 6)]


BS = [37, 100, 257, 16, 50]


@pytest.mark.parametrize("gk", ["inv", "rand"])
@pytest.mark.parametrize("path", ["split", "fp32", "bf16"])
def test_short_one_tile_chains_against_the_oracle(path, gk):
    from paper_2504_12037_amd import Net
    insts = _short()
    prec = "bf16" if path == "bf16" else "fp32"
    flags = Net.FLAG_PROFILE | (Net.FLAG_SPLIT_BF16 if path == "split" else 0)
    net = Net(insts, precision=prec, flags=flags)
    sp = [S.uniform_spins(b, i.n_width, 60 + k) for k, (b, i) in enumerate(zip(BS, insts))]
    flat = _dev(np.concatenate([x.reshape(-1) for x in sp]))
    rng = np.random.default_rng(9)
    g = np.concatenate([np.full(b, 1.0 / b) if gk == "inv" else rng.standard_normal(b) for b in BS])
    print(f"\n[split adjoint] path={path} g={gk}", flush=True)
    lz, dh, dJ, db = (x.cpu().numpy() for x in net.logz_and_backward(flat, _dev(g), BS))
    assert net.kernel_time("chain_bwd_1")[1] > 0
    so = ho = eo = 0
    for q, (inst, b, s) in enumerate(zip(insts, BS, sp)):
        want_lz = OI.logz_r_bruteforce(inst, s)
        assert np.abs(lz[so:so + b] - want_lz).max() / inst.n <= TOL[prec], q
        mag, corr, e2 = OI.marginals_bruteforce(inst, s)
        want = OI.logz_r_vjp(inst, s, g[so:so + b], marg=(mag, corr, e2))
        check_vjp((dh[ho:ho + inst.n], dJ[eo:eo + inst.n_edges], db[q]), want, inst,
                  g[so:so + b], path, inst.name)
        so += b
        ho += inst.n
        eo += inst.n_edges


@pytest.mark.parametrize("path", ["split", "fp32"])
def test_one_wave_persistent_equals_two_wave_launch(path):
    from paper_2504_12037_amd import Net
    insts = _short()
    flags = Net.FLAG_SPLIT_BF16 if path == "split" else 0
    sp = [S.uniform_spins(b, i.n_width, 70 + k) for k, (b, i) in enumerate(zip(BS, insts))]
    flat = _dev(np.concatenate([x.reshape(-1) for x in sp]))
    g = _dev(np.random.default_rng(2).standard_normal(sum(BS)))
    outs = []
    for mode in (1, 2):
        print(f"\n[split adjoint] path={path} launch_mode={mode}", flush=True)
        net = Net(insts, precision="fp32", flags=flags)
        net.set_tuning(launch_mode=mode)
        outs.append([x.clone() for x in net.logz_and_backward(flat, g, BS)])
    torch.cuda.synchronize()
    for a, b in zip(*outs):
        assert torch.equal(a, b)
