"""The paper's 40x40 open-boundary ferromagnet (Sec. 4, Fig. 2) at the
critical temperature, trained with Table 1's settings (one masked layer,
batch 1000, 1000 steps, learning rate 0.01), against the exact free energy
from the Kac-Ward determinant.  W = columns 7, 14, 21, 28 and 35 (|W| = 200,
strips of at most 6 columns, contracted row by row)."""

import numpy as np
import pytest

import synthetic as S
from adjtol import check_vjp
from oracle import kacward as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BETA_C = 0.5 * np.log(1.0 + np.sqrt(2.0))


def test_lattice40_ferromagnet_at_tc_against_kac_ward():
    from paper_2504_12037_amd import Net
    L = 40
    inst = S.lattice_column_split(S.lattice_2d(L, seed=0, beta=BETA_C, ferro=True),
                                  [7, 14, 21, 28, 35], hidden=0)
    F_exact = -K.logz_planar(inst.n, inst.edges, inst.J, BETA_C, K.lattice_xy(L)) / BETA_C
    print(f"\n[paper-scale] 40x40 ferromagnet, beta_c, |W|={inst.n_width}, "
          f"exact F/N={F_exact / inst.n:.8f}", flush=True)
    net = Net([inst], precision="fp32", flags=Net.FLAG_SPLIT_BF16)
    stats = torch.empty(1, 4, device="cuda", dtype=torch.float64)
    seen = []
    for s in range(1000):
        net.free_energy_step(1000, 0.01, stats=stats)
        if s % 100 == 99:
            Fq, se = (float(v) for v in stats.cpu().numpy()[0, :2])
            seen.append((Fq, se))
            print(f"  step {s + 1}: rel err {(Fq - F_exact) / abs(F_exact):.3e}", flush=True)
    # the variational bound F_q >= F, up to the batch estimate's noise
    for Fq, se in seen:
        assert Fq >= F_exact - 5 * se
    # the paper's order of accuracy at T_c
    Fq, _ = seen[-1]
    assert (Fq - F_exact) / abs(F_exact) <= 3e-4


@pytest.mark.parametrize("split", [False, True])
def test_lattice40_logz_and_adjoint_wide_width_set(split):
    # |W| = 200 (beyond the adjoint's 128-bit spin mask): the forward runs
    # the register-resident chain kernels with the unary factors read from
    # the spin bytes, the adjoint the LDS-staged ones; Gaussian couplings and
    # fields, against the oracle's elimination and its reverse pass
    from oracle import ising as OI
    from paper_2504_12037_amd import Net
    inst = S.lattice_column_split(S.lattice_2d(40, seed=21, beta=0.6, h_var=0.1),
                                  [7, 14, 21, 28, 35])
    B = 67
    print(f"\n[paper-scale] 40x40 Gaussian, |W|={inst.n_width}, split={split}", flush=True)
    spins = S.uniform_spins(B, inst.n_width, 3)
    net = Net([inst], precision="fp32", flags=Net.FLAG_SPLIT_BF16 if split else 0)
    sp = torch.from_numpy(spins).cuda().reshape(-1)
    lz = net.logz(sp, B).cpu().numpy()
    assert np.abs(lz - OI.logz_r_elimination(inst, spins)).max() / inst.n <= 1e-5
    g = np.random.default_rng(4).standard_normal(B)
    got = net.backward(sp, torch.from_numpy(g).cuda(), B)
    check_vjp([x.cpu().numpy() for x in got], OI.logz_r_vjp(inst, spins, g), inst, g,
              "split" if split else "fp32", "lattice40")
