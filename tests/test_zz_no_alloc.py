"""The allocation-free conditional log-partition call
(tnvan_logz_batch_noalloc) against tnvan_logz_batch, through the C ABI.

Both run the same kernels on the same inputs, so the results must agree bit
for bit; sampled outputs are also checked against the oracle.  Two calls in a
row, the second with a smaller batch (the static scratch keeps the first
call's contents), and the size and net checks that turn a call away before
any work is queued."""

import numpy as np
import pytest

import synthetic as S
from oracle import ising as OI

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().reshape(-1)


def _spins(insts, Bs, seed):
    sp = [S.uniform_spins(b, i.n_width, seed + k) for k, (b, i) in enumerate(zip(Bs, insts))]
    return sp, _dev(np.concatenate([s.reshape(-1) for s in sp]))


@pytest.mark.parametrize("prec,flags", [("fp32", 8), ("fp32", 0), ("bf16", 0)])
def test_noalloc_logz_equals_logz_batch(prec, flags):
    from paper_2504_12037_amd import Net
    insts = [S.c2_lattice(b) for b in (0.5, 1.0, 2.0)] + [S.c1_small_lattice()]
    net = Net(insts, precision=prec, flags=flags)
    tol = {"fp32": 1e-5, "bf16": 1e-3}[prec]
    for call, Bs in enumerate([[8192, 8192, 8192, 1024], [1000, 0, 37, 5]]):
        print(f"\n[no-alloc] prec={prec} flags={flags} call={call} B={Bs}", flush=True)
        sp, flat = _spins(insts, Bs, 60 + 10 * call)
        out = torch.full((sum(Bs),), np.nan, dtype=torch.float64, device="cuda")
        got = net.logz_noalloc(flat, Bs, out)
        ref = net.logz(flat, Bs)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (got - ref).abs().max().item()
        lz = got.cpu().numpy()
        off = 0
        for inst, b, s in zip(insts, Bs, sp):
            idx = np.arange(0, b, max(1, b // 24))
            if b:
                want = (OI.logz_r_bruteforce if len(inst.order) <= 16 else
                        OI.logz_r_elimination)(inst, s[idx])
                assert np.abs(lz[off + idx] - want).max() / inst.n <= tol
            off += b


def test_noalloc_refuses_what_it_cannot_hold():
    from paper_2504_12037_amd import Net, TnvanError
    insts = [S.c2_lattice(1.0)]
    net = Net(insts, precision="fp32")
    big = 40000   # 40000 samples x (4 x 224 + 8 x 14 + 8 x 3) bytes > 32 MiB
    flat = torch.ones(big * 32, dtype=torch.int8, device="cuda")
    out = torch.empty(big, dtype=torch.float64, device="cuda")
    with pytest.raises(TnvanError) as e:
        net.logz_noalloc(flat, [big], out)
    assert e.value.code == 1
    # a net with general (non-chain) steps: refused
    rrg = Net([S.c4_small_copies()[0]], precision="fp32")
    sp = torch.ones(4 * S.c4_small_copies()[0].n_width, dtype=torch.int8, device="cuda")
    with pytest.raises(TnvanError) as e:
        rrg.logz_noalloc(sp, [4], out)
    assert e.value.code == 5
    # and the refused calls left the array usable
    Bs = [513]
    sp, flat = _spins(insts, Bs, 3)
    got = net.logz_noalloc(flat, Bs, out)
    assert torch.equal(got, net.logz(flat, Bs))
