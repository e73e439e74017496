"""Benchmark of the TNVAN hot path on one MI355X.

Workload: 16x16 open-boundary Gaussian spin glass (J ~ N(0,1), seed 2, h = 0)
at beta in {0.5, 1.0, 2.0} (three instances in one net), width set = columns
6 and 11 (32 spins), remainder = strips 16x5 / 16x4 / 16x5 contracted row by
row, masked network of hidden width 256, 8192 samples per instance.

One step is one pass of the whole hot path over one batch, in one call
(tnvan_free_energy_step_adjoint): ancestral sampling (Philox uniforms), the
batched conditional log Z together with its adjoint (g_b = 1/B, giving
magnetisations, correlations and internal energy; one contraction, whose
forward pass yields log Z), E_1 / F_q / the REINFORCE weights in FP64, the
log-prob pass and the REINFORCE gradient, and the Adam update.  `value` is
samples per second of that step (3 x 8192 samples per step), inputs resident
in HBM.

The metric's own rate, the forward + adjoint
alone (tnvan_logz_and_backward), is breakdown.fwd_adj_samples_per_s, beside
the plain FP64 path on the same inputs.

The breakdown also measures the other workloads, each forward + adjoint per
path with its error against the oracle:
  c1   4x4 lattice, FP64 training (200 Adam steps, lr 1e-3, 1024 samples,
       hidden 16), exact F_q of the trained network against the 2^16-state F
  c2   the step's lattices with FP32 products and in the BF16 precision
  c3   SK N = 64 (beta 0.5, 1, 1.5; 48-spin width set, 2048 samples each)
  c4   random 3-regular N = 256, +-J, Gaussian fields, 4096 samples
  c5   64 uneven instances (lattices L = 8..24, random regular graphs
       N = 64..256, 512-4096 samples each, 122,880 in all), forward +
       adjoint and the training step replayed from a HIP graph
plus a roofline line for the dominant kernel and the oracle timed on the
host cores.  Every use of the oracle (the timed CPU baseline and every error
against it) is in the oracle leg at the end (--no-cpu-baseline skips it and
leaves the errors null).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("conditional logZ samples/s (fwd+adjoint) at |dlogZ|/N<=1e-5 vs plain FP64 path")
BETAS = (0.5, 1.0, 2.0)
B = 8192
HIDDEN = 256
PROFILE_EVERY = 4      # timed steps per step whose dominant kernel is timed by events
NW = 32
# Algorithmic flops per sample (one multiply-add = 2).  Remainder
# contraction in the pairwise form: per row transition, one 2x2 mix per
# vertical bond over the 2^w row states plus the diagonal horizontal bonds
# and fields; 15 transitions and a closing sum per 16-row strip:
#   two 16x5 strips: 2 * (15 * (4*5*32 + 32*2) + 32) = 21184
#   one 16x4 strip:       15 * (4*4*16 + 16*2) + 16  =  4336
# forward 25520; the adjoint is twice the forward (reverse sweep plus the
# per-step correlation sums), so forward + adjoint = 76560.  The adjoint
# kernels run the forward pass too and it yields log Z, so their count is
# forward + adjoint.
FWD_STRIP5 = 21184
FWD_STRIP4 = 4336
FWD_FLOPS = FWD_STRIP5 + FWD_STRIP4
# masked network (|W| = 32, H = 256): forward 2 * 2 * 32 * 256 = 32768 flops
# (the two masked products, dense count), backward about twice that
MADE_FWD = 2 * 2 * NW * HIDDEN
MADE_GRAD = 3 * MADE_FWD
SAMPLE_FLOPS = 2 * HIDDEN * NW + NW * NW
# per-kernel algorithmic flops per sample of the batch (every launch covers
# all three instances)
KERNEL_FLOPS = {
    "chain_fwd_2": FWD_STRIP5, "chain_fwd_1": FWD_STRIP4,
    "chain_bwd_2": 3 * FWD_STRIP5, "chain_bwd_1": 3 * FWD_STRIP4,
    "made_grad": MADE_GRAD, "sample": SAMPLE_FLOPS,
}
KERNEL_NAMES = {
    "chain_fwd_2": "rchain_fwd_kernel<{mode}, 2, 2>", "chain_fwd_1": "rchain_fwd_kernel<{mode}, 1, 2>",
    "chain_bwd_2": "rchain_bwd_kernel<2, {split}, {kk}>", "chain_bwd_1": "rchain_meet_kernel<{split}>",
    "made_grad": "mgrad_kernel<2, 16>", "sample": "msample_kernel<2, false>",
}
PEAK_FP32 = 157.3e12       # MI355X FP32 (vector and 16x16x4 matrix), published
PEAK_FP64 = 78.6e12        # MI355X FP64 (vector and matrix), published
PEAK_BF16 = 2.5e15         # MI355X BF16 dense matrix, published


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-samples", type=int, default=24576,
                   help="oracle samples per instance for cpu_baseline")
    p.add_argument("--fp32-products", action="store_true",
                   help="FP32 matrix-core products in the chain kernels (default: split BF16)")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="run one plain device copy of MIB MiB first (counter calibration)")
    p.add_argument("--checkpoint-every", type=int, default=0, metavar="K",
                   help="adjoint checkpoint interval of the step's net (0: the default, 1)")
    p.add_argument("--markers", action="store_true",
                   help="roctx phase ranges on the step's net (for rocprofv3 --marker-trace)")
    p.add_argument("--quick", action="store_true",
                   help="the timed step and its roofline line only (no breakdown, no "
                        "CPU baseline); for counter runs")
    return p.parse_args()


def event_time(fn, iters, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(iters):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / iters


def cpu_baseline(insts, n_samples):
    """The oracle (numpy FP64 log-domain elimination and its reverse pass)
    on a bounded sample of the same workload, on this host's cores."""
    import synthetic as S
    from oracle import ising as OI
    t0 = time.perf_counter()
    for k, inst in enumerate(insts):
        spins = S.uniform_spins(n_samples, inst.n_width, 4242 + k)
        OI.marginals_elimination(inst, spins, chunk=8192)
    dt = time.perf_counter() - t0
    n_samples *= len(insts)
    cores = len(os.sched_getaffinity(0))
    threads = os.environ.get("OMP_NUM_THREADS", "unset")
    return {"value": n_samples / dt, "unit": "samples/s", "cores": cores,
            "kind": "oracle",
            "sample": (f"{n_samples} samples (every beta of the workload), forward + "
                       f"reverse pass (numpy FP64, BLAS threads OMP_NUM_THREADS="
                       f"{threads}; elementwise numpy is single-threaded), "
                       f"{dt:.1f} s")}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy calibration), or None when
    there is none or the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_c2_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for src in fields.get("sources", "").split():
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if not fields.get("sources") or h.hexdigest() != fields.get("sources_sha256"):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def fwd_adj(net, flat, counts, iters, st, g=None, tune=None):
    """Time tnvan_logz_and_backward with g_b = 1/B (per instance); returns
    (seconds per call, logz, (dh, dJ, dbeta)) of the last call, on the host.
    With tune (a dict), the call is timed with the default launch shapes,
    then the autotuner picks shapes on this batch and the call is timed
    again; tune receives both times and the choice, and the returned time
    is the tuned one."""
    import torch
    if g is None:
        g = torch.cat([torch.full((b,), 1.0 / max(b, 1), dtype=torch.float64, device="cuda")
                       for b in counts])
    logz = torch.empty(max(1, sum(counts)), dtype=torch.float64, device="cuda")
    out = net._adjoint_out(None)
    fa = lambda: net.logz_and_backward(flat, g, counts, logz_out=logz, out=out)
    for _ in range(2):
        fa()
    t = event_time(fa, iters, st)
    if tune is not None:
        tune["default_s"] = t
        tune["default_shapes"] = net.get_tuning()
        t0 = time.perf_counter()
        tune["chosen"] = net.autotune(flat, g, counts)
        tune["tuning_s"] = time.perf_counter() - t0
        for _ in range(2):
            fa()
        t = event_time(fa, iters, st)
        tune["tuned_s"] = t
    fa()
    torch.cuda.synchronize()
    return t, logz[:sum(counts)].cpu().numpy(), tuple(x.cpu().numpy() for x in out)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the batch of samples is independent and would shard by sample, "
              "but no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)
    import torch

    import synthetic as S
    from paper_2504_12037_amd import Net

    torch.cuda.set_device(0)
    st = torch.cuda.current_stream()
    # the workload file of the step (configs/c2.json)
    from synthetic import config as SC
    insts, counts = SC.instances("c2")
    assert counts == [B] * len(BETAS) and [i.beta for i in insts] == list(BETAS)
    assert all(i.hidden == HIDDEN for i in insts)
    nI = len(insts)
    nw = insts[0].n_width
    iters = max(5, args.steps)
    keep = {}          # GPU results the oracle leg checks
    if args.calibrate_copy > 0:
        # a plain copy of known size: the HBM traffic counters of every kernel
        # are scaled by what they read for it
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # eager launches; the library records HIP events around the launches of
    # the dominant kernel of the step (the 2-tile adjoint chain kernel, by the
    # rocprofv3 statistics) and of no other kernel, in every PROFILE_EVERY-th
    # timed step: each timed launch adds two event records to the stream,
    # which serialise the queue around it (about 10 us per step)
    # FP32 path with split-BF16 products in the chain kernels (three BF16
    # matrix-core products per FP32 product; the breakdown reports the logZ
    # error this leaves against the oracle), unless --fp32-products
    split = args.precision == "fp32" and not args.fp32_products
    net = Net(insts, precision=args.precision, seed=2024,
              flags=Net.FLAG_PROFILE | (Net.FLAG_SPLIT_BF16 if split else 0) |
              (Net.FLAG_MARKERS if args.markers else 0),
              checkpoint_every=args.checkpoint_every)
    net.profile_only(["chain_bwd_2"])
    for k in range(nI):
        net.set_params(k, torch.from_numpy(S.made_init(nw, HIDDEN, 7 + k)))
    spins = torch.empty(nI * B * nw, dtype=torch.int8, device="cuda")
    stats = torch.empty(nI, 4, dtype=torch.float64, device="cuda")
    g = torch.full((nI * B,), 1.0 / B, dtype=torch.float64, device="cuda")
    dh = torch.empty(sum(i.n for i in insts), dtype=torch.float64, device="cuda")
    dJ = torch.empty(sum(i.n_edges for i in insts), dtype=torch.float64, device="cuda")
    db = torch.empty(nI, dtype=torch.float64, device="cuda")

    def step():
        net.free_energy_step(counts, 1e-3, stats=stats, spins_out=spins, adjoint=(g, dh, dJ, db))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for k in Net.KERNELS:
        net.kernel_time(k)          # drop the warm-up launches
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for i in range(args.steps):
        net.profile_only(["chain_bwd_2"] if i % PROFILE_EVERY == 0 else [])
        step()
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    value = nI * B / (ms / 1e3)
    # per-kernel device time over the timed region (HIP events recorded by the
    # library on the launch stream around each launch)
    ktime = {}
    for k in Net.KERNELS:
        tot, n = net.kernel_time(k)
        if n:
            ktime[k] = (tot, n)

    if args.quick:
        quick_line(args, value, ms, ktime, nI, split, wall)
        return

    # ---- C2: forward + adjoint alone, this path and the others, same inputs
    sp_np = S.uniform_spins(nI * B, nw, 102)
    sp_fix = torch.from_numpy(sp_np).cuda().reshape(-1)
    keep["c2_spins"] = sp_np
    tune_c2 = {}
    t_fa, lz, adj = fwd_adj(net, sp_fix, counts, iters, st, tune=tune_c2)
    keep["c2"] = {"run": (lz, adj)}
    logz = torch.empty(nI * B, dtype=torch.float64, device="cuda")
    out = (dh, dJ, db)
    t_bwd = event_time(lambda: net.backward(sp_fix, g, counts, out=out), iters, st)
    t_fwd = event_time(lambda: net.logz(sp_fix, counts, out=logz), iters, st)
    c2_paths = {}
    for pname, prec, flags in (("fp64", "fp64", 0), ("fp32_products", "fp32", 0),
                               ("bf16", "bf16", 0), ("split_bf16", "fp32", Net.FLAG_SPLIT_BF16)):
        if prec == args.precision and (flags != 0) == split:
            continue
        n2 = Net(insts, precision=prec, flags=flags)
        t2, lz2, adj2 = fwd_adj(n2, sp_fix, counts, iters, st)
        keep["c2"][pname] = (lz2, adj2)
        c2_paths[pname] = {"fwd_adj_s": t2, "fwd_adj_samples_per_s": nI * B / t2}
        del n2
    # the adjoint checkpoint interval k: time of the forward + adjoint call
    # and of the dominant kernel per k (same results bit for bit)
    ck_k = {}
    if args.precision != "fp64":
        for kk in (1, 2, 4, 8):
            nk = Net(insts, precision=args.precision, flags=Net.FLAG_PROFILE |
                     (Net.FLAG_SPLIT_BF16 if split else 0), checkpoint_every=kk)
            nk.profile_only(["chain_bwd_2"])
            tk, _, _ = fwd_adj(nk, sp_fix, counts, iters, st)
            ktot, kn = nk.kernel_time("chain_bwd_2")
            ck_k[kk] = {"fwd_adj_s": tk, "chain_bwd_2_avg_s": ktot / max(kn, 1),
                        "checkpoint_bytes_per_launch": 2 * nI * B * 2 * 16 * 4 * ((16 + kk - 1) // kk)}
            del nk
    t_fa64 = c2_paths["fp64"]["fwd_adj_s"] if "fp64" in c2_paths else t_fa
    lz64 = keep["c2"].get("fp64", (lz, None))[0]
    err64 = float(np.abs(lz - lz64).max() / insts[0].n)

    # ---- C1: plain FP64 training on the 4x4 lattice (Algorithm 1)
    c1 = S.c1_small_lattice(hidden=16)
    net1 = Net([c1], precision="fp64", seed=1)
    net1.set_params(0, torch.from_numpy(S.made_init(4, 16, 3)))
    st1 = torch.empty(1, 4, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(200):
        net1.free_energy_step(1024, 1e-3, stats=st1)
    torch.cuda.synchronize()
    t_c1 = (time.perf_counter() - t0) / 200
    keep["c1_theta"] = net1.get_params(0).cpu().numpy()
    keep["c1_last_Fq"] = float(st1.cpu().numpy()[0, 0])
    del net1

    # ---- C3: SK N = 64, dense 256 x 256 steps (LDS-staged chain kernels)
    c3 = [S.c3_sk(b) for b in (0.5, 1.0, 1.5)]
    B3 = 2048
    sp3 = S.uniform_spins(3 * B3, 48, 103)
    keep["c3_spins"] = sp3
    flat3 = torch.from_numpy(sp3).cuda().reshape(-1)
    c3_paths = {}
    keep["c3"] = {}
    for pname, prec in (("fp32", "fp32"), ("bf16", "bf16"), ("fp64", "fp64")):
        n3 = Net(c3, precision=prec)
        tn = {}
        t3, lz3, adj3 = fwd_adj(n3, flat3, [B3] * 3, iters, st, tune=tn)
        keep["c3"][pname] = (lz3, adj3)
        c3_paths[pname] = {"fwd_adj_s": t3, "fwd_adj_samples_per_s": 3 * B3 / t3, "tuning": tn}
        if pname == "fp32":
            c3_flops = n3.info(0)[3]
        del n3

    # ---- C4: random 3-regular N = 256 (general single-spin steps)
    c4 = S.c4_rrg()
    B4 = 4096
    sp4 = S.uniform_spins(B4, c4.n_width, 104)
    keep["c4_spins"] = sp4
    flat4 = torch.from_numpy(sp4).cuda().reshape(-1)
    c4_paths = {}
    keep["c4"] = {}
    for pname, prec in (("fp32", "fp32"), ("fp64", "fp64")):
        n4 = Net([c4], precision=prec)
        tn = {}
        t4, lz4, adj4 = fwd_adj(n4, flat4, [B4], iters, st, tune=tn)
        keep["c4"][pname] = (lz4, adj4)
        c4_paths[pname] = {"fwd_adj_s": t4, "fwd_adj_samples_per_s": B4 / t4, "tuning": tn}
        if pname == "fp32":
            c4_flops = n4.info(0)[3]
        del n4

    # ---- C5: 64 uneven instances in one net
    c5 = S.mixed_batch_instances()
    B5 = S.mixed_batch_sizes(c5)
    sp5 = [S.uniform_spins(b, i.n_width, 900 + k) for k, (b, i) in enumerate(zip(B5, c5))]
    keep["c5_spins"] = sp5
    flat5 = torch.from_numpy(np.concatenate([x.reshape(-1) for x in sp5])).cuda()
    c5_paths = {}
    keep["c5"] = {}
    for pname, prec, flags in (("split_bf16", "fp32", Net.FLAG_SPLIT_BF16), ("bf16", "bf16", 0),
                               ("fp64", "fp64", 0)):
        n5 = Net(c5, precision=prec, flags=flags | (Net.FLAG_GRAPH if prec != "fp64" else 0))
        tn = {}
        t5, lz5, _ = fwd_adj(n5, flat5, B5, 3, st, tune=tn)
        keep["c5"][pname] = lz5
        c5_paths[pname] = {"fwd_adj_s": t5, "fwd_adj_samples_per_s": sum(B5) / t5, "tuning": tn}
        if prec != "fp64":
            for k, inst in enumerate(c5):
                n5.set_params(k, torch.from_numpy(S.made_init(inst.n_width, inst.hidden, 7 + k)))
            st5 = torch.empty(len(c5), 4, dtype=torch.float64, device="cuda")
            g5 = torch.cat([torch.full((b,), 1.0 / b, dtype=torch.float64, device="cuda")
                            for b in B5])
            a5 = (g5,) + n5._adjoint_out(None)
            s5 = lambda: n5.free_energy_step(B5, 1e-3, stats=st5, adjoint=a5)
            for _ in range(2):
                s5()        # eager, then recorded; replays after
            t_s5 = event_time(s5, 3, st)
            c5_paths[pname].update({"train_step_graph_s": t_s5,
                                    "train_step_samples_per_s": sum(B5) / t_s5})
        del n5

    # exact slicing (every width-set configuration contracted as one sample,
    # Eqs. 3-4): a 12x12 Gaussian lattice with W = columns 5 and 9 (|W| = 24,
    # 16.8M configurations), timed on this path; logZ also by the FP64 path
    inst_x = S.lattice_column_split(S.lattice_2d(12, seed=6), [5, 9])
    netx = Net([inst_x], precision=args.precision, flags=Net.FLAG_SPLIT_BF16 if split else 0)
    outx = torch.empty(2, dtype=torch.float64, device="cuda")
    netx.exact_free_energy(0, out=outx)
    torch.cuda.synchronize()
    t_x = event_time(lambda: netx.exact_free_energy(0, out=outx), 2, st)
    lzx, Fx = (float(v) for v in outx.cpu().numpy())
    netx64 = Net([inst_x], precision="fp64")
    lzx64 = float(netx64.exact_free_energy(0).cpu().numpy()[0])
    del netx, netx64

    # moments of p from samples of q (self-normalised importance weights and
    # the adjoint's conditional moments): the step's network and batch
    sp_o, lq_o = net.sample(counts)
    obs = lambda: net.observables(sp_o, lq_o, counts)
    _, _, ess_o = obs()
    torch.cuda.synchronize()
    t_obs = event_time(obs, 5, st)
    ess_o = [float(v) for v in ess_o.cpu().numpy()]

    # magnetisation moments and susceptibility of p from the same samples:
    # the remainder's conditional mean and variance by the second-order
    # Taylor contraction, then the importance-weighted moments
    sus = lambda: net.susceptibility(sp_o, lq_o, counts)
    out_sus = sus().cpu().numpy()
    t_sus = event_time(sus, 5, st)
    mom = lambda: net.remainder_moments(sp_o, counts)
    _, mean_m, var_m = mom()
    torch.cuda.synchronize()
    t_mom = event_time(mom, 5, st)
    keep["moments"] = (sp_o.cpu().numpy().reshape(nI * B, nw), mean_m.cpu().numpy(),
                       var_m.cpu().numpy())

    # deeper masked networks: the training step of the step's lattices with
    # H = 64 at depth 1, 2 and 3 (depth 1 on the one-layer kernels, the others
    # on the deep sampler and rows kernels)
    deep = {}
    for D in (1, 2, 3):
        insts_d = [S.c2_lattice(b, 64) for b in BETAS]
        for i_d in insts_d:
            i_d.depth = D
        nd = Net(insts_d, precision=args.precision, seed=5,
                 flags=Net.FLAG_SPLIT_BF16 if split else 0)
        for k in range(nI):
            nd.set_params(k, torch.from_numpy(S.made_init(nw, 64, 7 + k, depth=D)))
        std = torch.empty(nI, 4, dtype=torch.float64, device="cuda")
        fd = lambda: nd.free_energy_step(counts, 1e-3, stats=std)
        fd()
        fd()
        t_d = event_time(fd, 5, st)
        deep[str(D)] = {"ms_per_step": 1e3 * t_d, "samples_per_s": nI * B / t_d,
                        "params_per_instance": nd.param_count(0)}
        del nd

    # the width-set planner (host only, Sec. 2 dynamic slicing) on the
    # paper's graph sizes: a 40x40 lattice and an n = 1000, d = 3 random
    # regular graph at w_u = 20 with the tree kept, an n = 300, d = 4 random
    # regular graph at w_u = 20 with the tree rebuilt after every pick
    from paper_2504_12037_amd import plan_width_set
    from synthetic import instances as SI
    plans = {}
    for pname, pn, pe, pw, prg in [
            ("lattice40_wu20", 1600, SI.lattice_edges(40), 20, False),
            ("rrg1000d3_wu20", 1000, SI.random_regular_edges(1000, 3, np.random.default_rng(9)), 20, False),
            ("rrg300d4_wu20_regreedy", 300, SI.random_regular_edges(300, 4, np.random.default_rng(7)), 20, True)]:
        t0 = time.perf_counter()
        Wp, _, wp, _ = plan_width_set(pn, pe, pw, regreedy=prg)
        plans[pname] = {"s": time.perf_counter() - t0, "width_set": int(Wp.shape[0]), "width": wp}

    # the paper's 40x40 ferromagnet at the critical temperature (Fig. 2)
    # with Table 1's settings: one masked layer, batch 1000, 1000 steps,
    # learning rate 0.01; W = columns 7, 14, 21, 28, 35 (|W| = 200)
    beta_c = 0.5 * float(np.log(1.0 + np.sqrt(2.0)))
    inst40 = S.lattice_column_split(S.lattice_2d(40, seed=0, beta=beta_c, ferro=True),
                                    [7, 14, 21, 28, 35], hidden=0)
    net40 = Net([inst40], precision=args.precision, flags=Net.FLAG_SPLIT_BF16 if split else 0)
    st40 = torch.empty(1, 4, device="cuda", dtype=torch.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(1000):
        net40.free_energy_step(1000, 0.01, stats=st40)
    torch.cuda.synchronize()
    t40 = (time.perf_counter() - t0) / 1000
    F40 = [float(v) / inst40.n for v in st40.cpu().numpy()[0, :2]]
    del net40

    # the paper's n = 1000, d = 3 random regular graph with a batch of 10000
    # at w_u = 20 (Sec. 4, Fig. 3(b)): W and the order from the planner
    # (|W| near the paper's 139 at that bound), message scopes up to 20 on
    # the wide single-spin steps; logZ and forward + adjoint on this path
    e1k = SI.random_regular_edges(1000, 3, np.random.default_rng(9))
    W1k, o1k, w1k, _ = plan_width_set(1000, e1k, 20)
    inst1k = S.Instance(1000, e1k.astype(np.int32),
                        np.random.default_rng(1).choice([-1.0, 1.0], len(e1k)),
                        np.random.default_rng(2).normal(0.0, np.sqrt(0.1), 1000), 0.5,
                        W1k.astype(np.int32), o1k.astype(np.int32), None, 0, "rrg1000_wu20")
    p1k = "fp64" if args.precision == "fp64" else "fp32"
    net1k = Net([inst1k], precision=p1k, max_width=20)
    B1k = 10000
    sp1k_np = S.uniform_spins(B1k, inst1k.n_width, 105)
    sp1k = torch.from_numpy(sp1k_np).cuda().reshape(-1)
    lz1k = torch.empty(B1k, dtype=torch.float64, device="cuda")
    net1k.logz(sp1k, B1k, out=lz1k)
    torch.cuda.synchronize()
    t_l1k = event_time(lambda: net1k.logz(sp1k, B1k, out=lz1k), 1, st)
    t_fa1k, lzf1k, _ = fwd_adj(net1k, sp1k, [B1k], 1, st)
    keep["rrg1000"] = (inst1k, sp1k_np[:2], lzf1k[:2])
    rrg1k = {"workload": "random 3-regular n=1000, +-J, h ~ N(0,0.1), beta 0.5, w_u = 20 "
                         f"(|W| = {inst1k.n_width}, message scope {w1k}), 10000 samples, {p1k}",
             "logz_s": t_l1k, "fwd_adj_s": t_fa1k, "logz_samples_per_s": B1k / t_l1k,
             "fwd_adj_samples_per_s": B1k / t_fa1k}
    del net1k

    # the dominant kernel's live timing (none on paths without it, e.g. FP64)
    roofline = roofline_line(ktime, nI, split, args.checkpoint_every)
    # call-level rooflines of the other workloads: algorithmic flops of the
    # forward + adjoint call (three times the forward) per second
    c3_alg = 3 * 2 * 65536          # [256] x [256, 256] per sample, forward x 3
    c4_alg = 3 * c4_flops
    for pth, d in c3_paths.items():
        pk = {"fp32": PEAK_FP32, "bf16": PEAK_BF16, "fp64": PEAK_FP64}[pth]
        d["roofline_call"] = {"bound": "mfma", "achieved_TFLOPs": c3_alg * d["fwd_adj_samples_per_s"] / 1e12,
                              "peak_TFLOPs": pk / 1e12,
                              "frac": c3_alg * d["fwd_adj_samples_per_s"] / pk}
    for pth, d in c4_paths.items():
        pk = {"fp32": PEAK_FP32, "fp64": PEAK_FP64}[pth]
        d["roofline_call"] = {"bound": "alu", "achieved_TFLOPs": c4_alg * d["fwd_adj_samples_per_s"] / 1e12,
                              "peak_TFLOPs": pk / 1e12,
                              "frac": c4_alg * d["fwd_adj_samples_per_s"] / pk}
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32+bf16x3" if split else
                  {"fp32": "f32", "fp64": "f64", "bf16": "bf16"}[args.precision]),
        "data": "synthetic",
        "config": {"workload": "16x16 OBC Gaussian spin glass, W = columns 6,11, "
                               "beta in {0.5,1,2}, 8192 samples each, MADE H=256",
                   "global_batch": nI * B, "instances": nI, "parallelism": "single GPU"},
        "value_is": ("samples/s of the whole training step (sample, logZ with its adjoint, "
                     "F_q, REINFORCE, Adam); the forward + adjoint alone is "
                     "breakdown.fwd_adj_samples_per_s"),
        "roofline": roofline,
        "breakdown": {
            "fwd_adj_samples_per_s": nI * B / t_fa,
            "fwd_adj_fp64_path_samples_per_s": nI * B / t_fa64,
            "speedup_vs_fp64_path": t_fa64 / t_fa,
            "logz_fwd_s": t_fwd, "logz_bwd_s": t_bwd, "fwd_adj_s": t_fa,
            "fwd_adj_fp64_s": t_fa64,
            "max_abs_dlogZ_per_N_vs_oracle": None,
            "max_abs_dlogZ_per_N_vs_fp64_path": err64,
            "adjoint_max_err_over_max_entry_vs_oracle": None,
            "c2_other_paths": c2_paths,
            "checkpoint_every": ck_k,
            "tuning": tune_c2,
            "wall_s_timed_region": wall,
            "c1": {"workload": "4x4 Gaussian lattice (seed 1), W = column 2, FP64 path, "
                               "200 Adam steps, lr 1e-3, 1024 samples, MADE H=16",
                   "ms_per_step": 1e3 * t_c1, "samples_per_s": 1024 / t_c1,
                   "last_batch_F_q": keep["c1_last_Fq"]},
            "c3": {"workload": "SK N=64, J ~ N(0,1/64) (seed 3), beta 0.5/1/1.5, |W| = 48, "
                               "R = 16 spins in two groups of 8, 2048 samples each",
                   "algorithmic_flops_per_sample_fwd_adj": c3_alg, "paths": c3_paths,
                   "speedup_fp32_vs_fp64": c3_paths["fp64"]["fwd_adj_s"] / c3_paths["fp32"]["fwd_adj_s"]},
            "c4": {"workload": "random 3-regular N=256, +-J, h ~ N(0,0.1) (seed 4), greedy "
                               f"width limit 10 (|W| = {c4.n_width}), 4096 samples",
                   "algorithmic_flops_per_sample_fwd_adj": c4_alg, "paths": c4_paths,
                   "speedup_fp32_vs_fp64": c4_paths["fp64"]["fwd_adj_s"] / c4_paths["fp32"]["fwd_adj_s"]},
            "c5": {"workload": "64 instances: lattices L in {8,12,16,24}, random 3-regular "
                               "N in {64,128,256}, 512-4096 samples each",
                   "samples": sum(B5), "paths": c5_paths},
            "exact_slicing": {"workload": "12x12 OBC Gaussian lattice (seed 6), W = columns 5,9, beta 1",
                              "configurations": 1 << inst_x.n_width, "s": t_x,
                              "configurations_per_s": (1 << inst_x.n_width) / t_x,
                              "logZ": lzx, "F": Fx,
                              "abs_dlogZ_per_N_vs_fp64_path": abs(lzx - lzx64) / inst_x.n},
            "observables": {"workload": "the step's network and batch (samples of q)",
                            "s": t_obs, "samples_per_s": nI * B / t_obs,
                            "effective_sample_size": ess_o},
            "susceptibility": {"workload": "the step's network and batch (samples of q)",
                               "s": t_sus, "samples_per_s": nI * B / t_sus,
                               "remainder_moments_s": t_mom,
                               "m_per_spin": [float(v) for v in out_sus[:, 0]],
                               "chi": [float(v) for v in out_sus[:, 2]],
                               "effective_sample_size": [float(v) for v in out_sus[:, 3]]},
            "deep_made": {"workload": "the step's 16x16 lattices, MADE H=64 at depth 1/2/3, "
                                      "training step (sample, logZ, F_q, REINFORCE, Adam)",
                          "depth": deep},
            "planner": plans,
            "lattice40_ferro_tc": {"workload": "40x40 OBC ferromagnet at beta_c, W = columns "
                                               "7,14,21,28,35, one masked layer, batch 1000, "
                                               "1000 steps, lr 0.01",
                                   "ms_per_step": 1e3 * t40, "F_q_per_spin": F40[0],
                                   "stderr_per_spin": F40[1]},
            "rrg1000_wu20": rrg1k,
            "kernel_avg_us": {kname(k, split, args.checkpoint_every): 1e6 * t / n
                              for k, (t, n) in ktime.items()},
        },
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(insts, args.cpu_samples)
        oracle_checks(res["breakdown"], keep, insts, c3, c4, c5, B5)
    print(json.dumps(res), flush=True)


def kname(k, split, ck=1):
    return KERNEL_NAMES.get(k, k).format(split=str(split).lower(), mode=2 if split else 0,
                                         kk=str(ck > 1).lower())


def roofline_line(ktime, nI, split, ck=1):
    """The dominant kernel's live timing against its peak (None on paths
    without it, e.g. FP64)."""
    if "chain_bwd_2" not in ktime:
        return None
    dom = "chain_bwd_2"
    dom_avg = ktime[dom][0] / ktime[dom][1]
    achieved = KERNEL_FLOPS[dom] * nI * B / dom_avg
    # the peak of the units the products run on: BF16 dense for split
    # products (three BF16 products per algorithmic FP32 product, so at most
    # a third of it is attainable), FP32 matrix otherwise
    peak = PEAK_BF16 if split else PEAK_FP32
    return {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": measured_traffic(dom) if ck <= 1 else None,
            "kernel": kname(dom, split, ck), "kernel_avg_s": dom_avg, "kernel_launches_timed": ktime[dom][1],
            "flops_per_launch": KERNEL_FLOPS[dom] * nI * B,
            "peak_units": "bf16 dense, 3 products per flop" if split else "fp32 matrix"}


def quick_line(args, value, ms, ktime, nI, split, wall):
    print(json.dumps({"metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f32+bf16x3" if split else args.precision, "data": "synthetic",
                      "config": {"workload": "16x16 OBC Gaussian spin glass, W = columns 6,11, "
                                             "beta in {0.5,1,2}, 8192 samples each, MADE H=256",
                                 "global_batch": nI * B, "instances": nI,
                                 "parallelism": "single GPU"},
                      "roofline": roofline_line(ktime, nI, split, args.checkpoint_every),
                      "quick": True,
                      "checkpoint_every": args.checkpoint_every or 1,
                      "wall_s_timed_region": wall}), flush=True)


def oracle_checks(bd, keep, insts, c3, c4, c5, B5):
    """The oracle leg's errors: every GPU result kept above against the FP64
    oracle on the same inputs (per-sample logZ error per spin; adjoint error
    relative to the largest entry, with g_b = 1/B)."""
    import synthetic as S
    from oracle import ising as OI
    from oracle import objective as OO

    def vjp_err(inst, spins, adj, k=0):
        Bk = spins.shape[0]
        wdh, wdJ, wdb = OI.logz_r_vjp(inst, spins, np.full(Bk, 1.0 / Bk))
        dh, dJ, db = adj
        eh = np.abs(dh[k * inst.n:(k + 1) * inst.n] - wdh).max()
        eJ = np.abs(dJ[k * inst.n_edges:(k + 1) * inst.n_edges] - wdJ).max()
        return float(max(eh, eJ) / max(np.abs(wdh).max(), np.abs(wdJ).max()))

    # C2, full batch of every beta
    sp = keep["c2_spins"]
    nI = len(insts)
    want = [OI.logz_r_elimination(inst, sp[k * B:(k + 1) * B]) for k, inst in enumerate(insts)]
    for pname, (lz, adj) in keep["c2"].items():
        e = max(float(np.abs(lz[k * B:(k + 1) * B] - want[k]).max() / inst.n)
                for k, inst in enumerate(insts))
        ea = max(vjp_err(inst, sp[k * B:(k + 1) * B], adj, k) for k, inst in enumerate(insts))
        if pname == "run":
            bd["max_abs_dlogZ_per_N_vs_oracle"] = e
            bd["adjoint_max_err_over_max_entry_vs_oracle"] = ea
        else:
            bd["c2_other_paths"][pname]["max_abs_dlogZ_per_N_vs_oracle"] = e
            bd["c2_other_paths"][pname]["adjoint_max_err_over_max_entry_vs_oracle"] = ea
    # C1: exact F_q of the trained network (enumeration of q) against F
    c1 = S.c1_small_lattice(hidden=16)
    Fq, _ = OO.exact_fq_and_grad(c1, keep["c1_theta"].astype(np.float64), 16)
    F = OO.exact_free_energy(c1)
    bd["c1"].update({"exact_F_q_after_training": Fq, "exact_F": F,
                     "relative_gap": (Fq - F) / abs(F)})
    # C3, full batch (brute force over the 2^16 remainder states)
    sp3 = keep["c3_spins"]
    B3 = sp3.shape[0] // 3
    want3 = [OI.logz_r_bruteforce(inst, sp3[k * B3:(k + 1) * B3]) for k, inst in enumerate(c3)]
    for pname, (lz, adj) in keep["c3"].items():
        d = bd["c3"]["paths"][pname]
        d["max_abs_dlogZ_per_N_vs_oracle"] = max(
            float(np.abs(lz[k * B3:(k + 1) * B3] - want3[k]).max() / inst.n)
            for k, inst in enumerate(c3))
    # C4, full batch logZ and the adjoint
    sp4 = keep["c4_spins"]
    want4 = OI.logz_r_elimination(c4, sp4)
    for pname, (lz, adj) in keep["c4"].items():
        d = bd["c4"]["paths"][pname]
        d["max_abs_dlogZ_per_N_vs_oracle"] = float(np.abs(lz - want4).max() / c4.n)
        d["adjoint_max_err_over_max_entry_vs_oracle"] = vjp_err(c4, sp4, adj)
    # magnetisation moments: 64 samples of every instance of the step's
    # batch against the oracle's count-resolved elimination, relative to
    # the raw second moment of M_R
    from oracle import magnetisation as MG
    sp_m, mean_m, var_m = keep["moments"]
    em = 0.0
    for k, inst in enumerate(insts):
        idx = k * B + np.arange(0, B, B // 64)
        mo, vo = MG.remainder_magnetisation(inst, sp_m[idx])
        s2 = vo + mo * mo + 1.0
        em = max(em, float(np.max(np.abs(mean_m[idx] - mo) / np.sqrt(s2))),
                 float(np.max(np.abs(var_m[idx] - vo) / s2)))
    bd["susceptibility"]["moments_max_err_over_second_moment_vs_oracle_64_per_instance"] = em
    # the n = 1000 graph at w_u = 20: two samples by the oracle's elimination
    inst1k, sp1k, lz1k = keep["rrg1000"]
    want1k = OI.logz_r_elimination(inst1k, sp1k, chunk=1)
    bd["rrg1000_wu20"]["max_abs_dlogZ_per_N_vs_oracle_2_samples"] = float(
        np.abs(lz1k - want1k).max() / inst1k.n)
    # C5, 16 samples of every instance
    off = np.concatenate([[0], np.cumsum(B5)])
    want5 = [OI.logz_r_elimination(inst, keep["c5_spins"][k][:16]) for k, inst in enumerate(c5)]
    for pname, lz in keep["c5"].items():
        bd["c5"]["paths"][pname]["max_abs_dlogZ_per_N_vs_oracle_16_per_instance"] = max(
            float(np.abs(lz[off[k]:off[k] + 16] - want5[k]).max() / inst.n)
            for k, inst in enumerate(c5))


if __name__ == "__main__":
    main()
