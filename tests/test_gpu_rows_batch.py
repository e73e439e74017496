"""The REINFORCE rows of every instance in one launch per class of LDS need
(parameters staged in LDS up to 40 KB, up to 80 KB, up to the block limit,
and read from global memory above it) through the C ABI: one training step
on a net with an instance in each class and uneven batches whose last block
is partial, gradient of Eq. (10) against the FP64 oracle per instance.  The
same step's spins pin the general sampler with its parameters read from
global memory (one round of samples per block) against the oracle's Eq. (8)
given the Philox uniforms."""

import numpy as np
import pytest

import synthetic as S
from oracle import ising as OI
from oracle import made as OM
from oracle import objective as OO
from oracle import philox as OP
from synthetic.instances import Instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _path(nw, H, seed):
    # a path of 2 nw spins, W = the even ones (nw of them), every R spin a
    # one-row strip
    n = 2 * nw
    rng = np.random.default_rng(seed)
    e = np.array([(i, i + 1) for i in range(n - 1)], np.int32)
    W = np.arange(0, n, 2, dtype=np.int32)
    R = np.arange(1, n, 2, dtype=np.int32)
    return Instance(n, e, rng.standard_normal(len(e)), rng.normal(0.0, 0.5, n), 0.7, W, R,
                    np.arange(len(R) + 1, dtype=np.int32), H, f"path{n}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_rows_of_every_lds_class_against_the_oracle(prec):
    from paper_2504_12037_amd import Net
    # |W| = 8, 40, 96, 120 with 128 hidden units: about 22 KB, 60 KB, 154 KB
    # and 200 KB of parameters and rows in FP32
    insts = [_path(8, 128, 1), _path(40, 128, 2), _path(96, 128, 3), _path(120, 128, 4)]
    Bs = [37, 300, 513, 100]
    seed, lr = 21, 1e-3
    net = Net(insts, precision=prec, seed=seed)
    thetas = []
    for k, inst in enumerate(insts):
        th = S.made_init(inst.n_width, inst.hidden, 30 + k)
        th = (th + 0.1 * np.random.default_rng(k).standard_normal(th.shape)).astype(np.float32)
        thetas.append(th)
        net.set_params(k, torch.from_numpy(th))
    spins = torch.empty(sum(b * i.n_width for b, i in zip(Bs, insts)), dtype=torch.int8,
                        device="cuda")
    print(f"\n[rows batch] prec={prec} widths={[i.n_width for i in insts]} B={Bs}", flush=True)
    stats, _ = net.free_energy_step(Bs, lr, spins_out=spins)
    torch.cuda.synchronize()
    sp_all = spins.cpu().numpy()
    off = 0
    for k, (inst, b) in enumerate(zip(insts, Bs)):
        n, H = inst.n_width, inst.hidden
        sp = sp_all[off:off + b * n].reshape(b, n)
        off += b * n
        th64 = thetas[k].astype(np.float64)
        # the sampler: the oracle's draws from the same uniforms, with the
        # GPU's spin forced only where the conditional is within 1e-6 of
        # the uniform (FP32 against FP64 rounding)
        u = OP.sampler_uniforms(seed, 0, k, b, n)
        s_o, _, pr = OM.sample(th64, u, n, H)
        tie = np.abs(pr - u) < 1e-6
        if tie.any():
            force = np.zeros((b, n), np.int8)
            force[tie] = sp[tie]
            s_o, _, pr = OM.sample(th64, u, n, H, force=force)
        assert np.array_equal(s_o, sp), (inst.name, np.argwhere(s_o != sp)[:5])
        lq = OM.logq(th64, sp, n, H)
        lz = OI.logz_r_elimination(inst, sp)
        f, _ = OO.free_energy_terms(inst, sp, lq, lz)
        g = OM.logq_backward(th64, sp, OO.reinforce_weights(f), n, H)
        g_gpu = net.get_state(k, 1).cpu().numpy().astype(np.float64)
        err = np.abs(g_gpu - g).max()
        # the gradient is held in FP32: in FP64 nets one rounding of it
        bar = (1e-12 + 2.0 ** -24 * np.abs(g).max()) if prec == "fp64" else \
            (1e-6 + 1e-4 * np.abs(g).max())
        assert err <= bar, (inst.name, err, bar)
        M1, M2, M0 = OM.masks(n, H)
        mask = OM.pack(M1, np.ones(H), M2, np.ones(n), M0)
        assert np.all(g_gpu[mask == 0] == 0), inst.name


def test_rows_beyond_the_lds_limit_are_refused():
    # FP64 rows of |W| = 700 with H = 16 need 16 x (2 x 701 + 17) x 8 bytes
    # of LDS per block (about 182 KB), above the block limit: the step is
    # refused before any rows launch, with the sizes in the message
    from paper_2504_12037_amd import Net
    from paper_2504_12037_amd._lib import TnvanError
    net = Net([_path(700, 16, 5)], precision="fp64", seed=3)
    print("\n[rows batch] |W| = 700 FP64, expecting a refusal", flush=True)
    with pytest.raises(TnvanError, match="LDS"):
        net.free_energy_step([64], 1e-3)
