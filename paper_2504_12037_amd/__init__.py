"""TNVAN hot path on MI355X: Python face of libtnvan.so.

    net = Net(instances, precision="fp32")
    logz = net.logz(spins, n_samples)              # Eqs. 3-4, per sample
    dh, dJ, dbeta = net.backward(spins, g, n_samples)
    spins, logq = net.sample(n_samples, uniforms)  # Eq. 8
    stats, spins = net.free_energy_step(n_samples, lr)   # Algorithm 1

Tensors are torch tensors on the current HIP device; the current torch
stream is handed to the library.  ``LogZ`` wraps logz/backward as a
torch.autograd.Function returning gradients for (J, h, beta).
"""

from __future__ import annotations

import ctypes as C
from typing import Sequence

import torch

from . import _lib
from ._lib import TnvanError, plan, plan_width_set  # noqa: F401

__all__ = ["Net", "LogZ", "plan", "plan_width_set", "TnvanError"]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Net:
    """One or more compiled instances sharing a device program."""

    def __init__(self, instances: Sequence, precision: str = "fp32",
                 max_width: int = 14, seed: int = 0, flags: int = 0,
                 checkpoint_every: int = 0):
        L = _lib.lib()
        self.instances = list(instances)
        self.precision = precision
        keep = []
        arr = (_lib.CInstance * len(self.instances))()
        for k, inst in enumerate(self.instances):
            arr[k] = _lib.make_cinstance(inst, keep)
        opt = _lib.COptions(_lib._PREC[precision], int(max_width), 1, int(flags), int(seed),
                            int(checkpoint_every))
        h = C.c_void_p()
        _lib.check(L.tnvan_build_network(arr, len(self.instances), C.byref(opt),
                                         C.byref(h)))
        self._h = h
        self.nw = [int(len(i.width_set)) for i in self.instances]
        self.n = [int(i.n) for i in self.instances]
        self.ne = [int(len(i.edges)) for i in self.instances]
        # the couplings, fields and inverse temperatures the tables were
        # compiled from (LogZ checks its arguments against them)
        import numpy as np
        self.couplings = (
            torch.from_numpy(np.concatenate([np.asarray(i.J, np.float64).reshape(-1)
                                             for i in self.instances])),
            torch.from_numpy(np.concatenate([np.zeros(i.n) if i.h is None else
                                             np.asarray(i.h, np.float64).reshape(-1)
                                             for i in self.instances])),
            torch.tensor([float(i.beta) for i in self.instances], dtype=torch.float64))

    def __del__(self):
        h = getattr(self, "_h", None)
        lib = getattr(_lib, "_lib", None)
        if h is not None and h.value and lib is not None:
            lib.tnvan_free_network(h)
            self._h = None

    # ---------------------------------------------------------------- helpers
    def _counts(self, n_samples):
        if isinstance(n_samples, int):
            n_samples = [n_samples] * len(self.instances)
        arr = (C.c_int64 * len(self.instances))(*[int(b) for b in n_samples])
        return arr, [int(b) for b in n_samples]

    @property
    def logq_dtype(self):
        return torch.float64 if self.precision == "fp64" else torch.float32

    def info(self, inst: int = 0):
        out = (C.c_int64 * 6)()
        _lib.check(_lib.lib().tnvan_program_info(self._h, inst, out))
        return tuple(int(x) for x in out)

    # kernel ids of tnvan_kernel_time (built with flags=FLAG_PROFILE)
    KERNELS = {"chain_fwd_1": 0, "chain_fwd_2": 1, "chain_fwd_4": 2, "chain_bwd_1": 3,
               "chain_bwd_2": 4, "sample": 5, "made_grad": 6, "chain_fwd_all": 7,
               "chain_bwd_all": 8}
    FLAG_LDS_CHAIN = 1
    FLAG_PROFILE = 2
    FLAG_GRAPH = 4
    FLAG_SPLIT_BF16 = 8
    FLAG_CHECK_FINITE = 16
    FLAG_MARKERS = 32

    def profile_only(self, kernels):
        """Time only these kernels (names or ids of KERNELS) from now on."""
        mask = 0
        for k in kernels:
            mask |= 1 << (self.KERNELS[k] if isinstance(k, str) else int(k))
        _lib.check(_lib.lib().tnvan_profile_mask(self._h, mask))

    def kernel_time(self, kernel):
        """(total seconds, launches) of one kernel since the previous read."""
        k = self.KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        ms = C.c_double()
        n = C.c_int64()
        _lib.check(_lib.lib().tnvan_kernel_time(self._h, k, C.byref(ms), C.byref(n)))
        return ms.value / 1e3, int(n.value)

    # ---------------------------------------------------------- launch shapes
    def get_tuning(self) -> dict:
        """Launch shapes in effect (tnvan_get_tuning) as a dict."""
        t = _lib.CTuning()
        _lib.check(_lib.lib().tnvan_get_tuning(self._h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **shapes):
        """Request launch shapes (general_tile_fwd, general_tile_bwd,
        chain_groups, checkpoint_every, launch_mode, arena_limit_mib; 0 or
        absent = default rule)."""
        t = _lib.CTuning()
        for k, v in shapes.items():
            if k not in _lib.CTuning.FIELDS:
                raise KeyError(k)
            setattr(t, k, int(v))
        _lib.check(_lib.lib().tnvan_set_tuning(self._h, C.byref(t)))

    def autotune(self, spins: torch.Tensor, grad: torch.Tensor, n_samples,
                 cache_path: str = None) -> dict:
        """tnvan_autotune on this batch: times the candidate launch shapes,
        applies the fastest and returns it (JSON cache at cache_path, or at
        $TNVAN_AUTOTUNE_CACHE when that is set and cache_path is None)."""
        import os
        if cache_path is None:
            cache_path = os.environ.get("TNVAN_AUTOTUNE_CACHE") or None
        arr, counts = self._counts(n_samples)
        spins = spins.to(device="cuda").contiguous()
        grad = grad.to(device="cuda", dtype=torch.float64).contiguous()
        logz = torch.empty(max(1, sum(counts)), device="cuda", dtype=torch.float64)
        dh, dJ, db = self._adjoint_out(None)
        t = _lib.CTuning()
        path = None if cache_path is None else str(cache_path).encode()
        _lib.check(_lib.lib().tnvan_autotune(self._h, arr, _ptr(spins), _ptr(grad), _ptr(logz),
                                             _ptr(dh), _ptr(dJ), _ptr(db), path, C.byref(t),
                                             _stream()))
        return t.as_dict()

    def param_count(self, inst: int = 0) -> int:
        n = C.c_int64()
        _lib.check(_lib.lib().tnvan_param_count(self._h, inst, C.byref(n)))
        return n.value

    def set_params(self, inst: int, theta: torch.Tensor):
        t = theta.to(device="cuda", dtype=torch.float32).contiguous()
        assert t.numel() == self.param_count(inst)
        _lib.check(_lib.lib().tnvan_set_params(self._h, inst, _ptr(t), _stream()))
        torch.cuda.current_stream().synchronize()

    def get_params(self, inst: int = 0) -> torch.Tensor:
        t = torch.empty(self.param_count(inst), device="cuda", dtype=torch.float32)
        _lib.check(_lib.lib().tnvan_get_params(self._h, inst, _ptr(t), _stream()))
        return t

    def get_state(self, inst: int, which: int) -> torch.Tensor:
        """0 params, 1 last gradient, 2 Adam m, 3 Adam v (float32)."""
        t = torch.empty(self.param_count(inst), device="cuda", dtype=torch.float32)
        _lib.check(_lib.lib().tnvan_get_state(self._h, inst, which, _ptr(t), _stream()))
        return t

    def set_state(self, inst: int, which: int, value: torch.Tensor):
        """0 params (moments and step counter kept), 2 Adam m, 3 Adam v."""
        t = value.to(device="cuda", dtype=torch.float32).contiguous()
        assert t.numel() == self.param_count(inst)
        _lib.check(_lib.lib().tnvan_set_state(self._h, inst, which, _ptr(t), _stream()))
        torch.cuda.current_stream().synchronize()

    def get_step(self, inst: int = 0) -> int:
        v = C.c_int32()
        _lib.check(_lib.lib().tnvan_get_step(self._h, inst, C.byref(v), _stream()))
        return int(v.value)

    def set_step(self, inst: int, step: int):
        _lib.check(_lib.lib().tnvan_set_step(self._h, inst, int(step), _stream()))

    def checkpoint(self) -> list:
        """Per instance (params, Adam m, Adam v, step) on the host."""
        return [(self.get_state(k, 0).cpu(), self.get_state(k, 2).cpu(),
                 self.get_state(k, 3).cpu(), self.get_step(k))
                for k in range(len(self.instances))]

    def restore(self, ckpt: list):
        """Resume from checkpoint() (bit for bit)."""
        for k, (p, m, v, t) in enumerate(ckpt):
            self.set_state(k, 0, p)
            self.set_state(k, 2, m)
            self.set_state(k, 3, v)
            self.set_step(k, t)
        torch.cuda.current_stream().synchronize()

    # ----------------------------------------------------------- entry points
    def sample(self, n_samples, uniforms: torch.Tensor = None):
        arr, counts = self._counts(n_samples)
        tot = sum(b * w for b, w in zip(counts, self.nw))
        spins = torch.empty(max(tot, 1), device="cuda", dtype=torch.int8)
        logq = torch.empty(max(sum(counts), 1), device="cuda", dtype=self.logq_dtype)
        if uniforms is not None:
            uniforms = uniforms.to(device="cuda").contiguous()
            assert uniforms.dtype == torch.float32 and uniforms.numel() == tot
        _lib.check(_lib.lib().tnvan_sample(self._h, arr, _ptr(uniforms), _ptr(spins),
                                           _ptr(logq), _stream()))
        return spins[:tot], logq[:sum(counts)]

    def logz(self, spins: torch.Tensor, n_samples, out: torch.Tensor = None,
             e1: bool = False):
        """logZ_R per sample (float64 device tensor); with e1=True also
        E_1(s_W) per sample: returns (logz, e1)."""
        arr, counts = self._counts(n_samples)
        spins = spins.to(device="cuda").contiguous()
        assert spins.dtype == torch.int8
        assert spins.numel() == sum(b * w for b, w in zip(counts, self.nw))
        if out is None:
            out = torch.empty(max(sum(counts), 1), device="cuda", dtype=torch.float64)
        e = torch.empty(max(sum(counts), 1), device="cuda", dtype=torch.float64) if e1 else None
        _lib.check(_lib.lib().tnvan_logz_batch(self._h, arr, _ptr(spins), _ptr(out), _ptr(e),
                                               _stream()))
        if e1:
            return out[:sum(counts)], e[:sum(counts)]
        return out[:sum(counts)]

    def set_couplings(self, inst: int, J, h, beta: float):
        """tnvan_set_couplings: new couplings [n_edges], fields [n] (or None)
        and inverse temperature of instance ``inst``; the tables are compiled
        again, the parameters of q and the optimiser state stay."""
        import numpy as np
        Jn = np.ascontiguousarray(np.asarray(J, dtype=np.float64).reshape(-1))
        assert Jn.size == self.ne[inst]
        hn = None
        if h is not None:
            hn = np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(-1))
            assert hn.size == self.n[inst]
        ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        _lib.check(_lib.lib().tnvan_set_couplings(self._h, int(inst), ptr(Jn), ptr(hn),
                                                  float(beta)))
        e0, n0 = sum(self.ne[:inst]), sum(self.n[:inst])
        Jt, ht, bt = self.couplings
        Jt[e0:e0 + Jn.size] = torch.from_numpy(Jn)
        ht[n0:n0 + self.n[inst]] = 0.0 if hn is None else torch.from_numpy(hn)
        bt[inst] = float(beta)

    def logz_noalloc(self, spins: torch.Tensor, n_samples, out: torch.Tensor):
        """tnvan_logz_batch_noalloc: logz into ``out`` (a float64 device
        tensor of at least sum(n_samples) entries) with the library's static
        scratch; the call itself allocates nothing."""
        arr, counts = self._counts(n_samples)
        assert spins.is_cuda and spins.dtype == torch.int8 and spins.is_contiguous()
        assert spins.numel() >= sum(b * w for b, w in zip(counts, self.nw))
        assert out.is_cuda and out.dtype == torch.float64 and out.numel() >= sum(counts)
        _lib.check(_lib.lib().tnvan_logz_batch_noalloc(self._h, arr, _ptr(spins), _ptr(out),
                                                       _stream()))
        return out[:sum(counts)]

    def observables(self, spins: torch.Tensor, logq: torch.Tensor, n_samples):
        """(mag [sum n], corr [sum E], ess [n_inst]) device float64 tensors:
        <sigma_i>_p and <sigma_i sigma_j>_p estimated from samples of q
        (self-normalised importance weights) and the effective sample size."""
        arr, counts = self._counts(n_samples)
        spins = spins.to(device="cuda").contiguous()
        logq = logq.to(device="cuda", dtype=self.logq_dtype).contiguous()
        assert spins.dtype == torch.int8 and logq.numel() == sum(counts)
        mag = torch.empty(sum(self.n), device="cuda", dtype=torch.float64)
        corr = torch.empty(max(sum(self.ne), 1), device="cuda", dtype=torch.float64)
        ess = torch.empty(len(counts), device="cuda", dtype=torch.float64)
        _lib.check(_lib.lib().tnvan_observables(self._h, arr, _ptr(spins), _ptr(logq), _ptr(mag),
                                                _ptr(corr), _ptr(ess), _stream()))
        return mag, corr[:sum(self.ne)], ess

    def remainder_moments(self, spins: torch.Tensor, n_samples):
        """(logz, mean, var) device float64 tensors [sum n_samples]: ln Z_R,
        <M_R | s_W> and Var(M_R | s_W) per sample (tnvan_remainder_moments)."""
        arr, counts = self._counts(n_samples)
        spins = spins.to(device="cuda").contiguous()
        assert spins.dtype == torch.int8
        assert spins.numel() == sum(b * w for b, w in zip(counts, self.nw))
        out = [torch.empty(max(sum(counts), 1), device="cuda", dtype=torch.float64)
               for _ in range(3)]
        _lib.check(_lib.lib().tnvan_remainder_moments(self._h, arr, _ptr(spins), _ptr(out[0]),
                                                      _ptr(out[1]), _ptr(out[2]), _stream()))
        return tuple(t[:sum(counts)] for t in out)

    def susceptibility(self, spins: torch.Tensor, logq: torch.Tensor, n_samples):
        """[n_inst, 4] device float64: <M>/N, <M^2>/N^2, chi = beta N
        (<M^2>/N^2 - (<M>/N)^2) and the effective sample size, estimated
        from samples of q (tnvan_susceptibility)."""
        arr, counts = self._counts(n_samples)
        spins = spins.to(device="cuda").contiguous()
        logq = logq.to(device="cuda", dtype=self.logq_dtype).contiguous()
        assert spins.dtype == torch.int8 and logq.numel() == sum(counts)
        out = torch.empty(len(counts), 4, device="cuda", dtype=torch.float64)
        _lib.check(_lib.lib().tnvan_susceptibility(self._h, arr, _ptr(spins), _ptr(logq),
                                                   _ptr(out), _stream()))
        return out

    def exact_free_energy(self, inst: int = 0, out: torch.Tensor = None):
        """(logZ, F) of one instance by slicing over all 2^|W| width-set
        configurations (device float64 tensor [2]; the net's batch is left
        at one pass of that instance)."""
        if out is None:
            out = torch.empty(2, device="cuda", dtype=torch.float64)
        _lib.check(_lib.lib().tnvan_exact_free_energy(self._h, int(inst), _ptr(out), _stream()))
        return out

    def backward(self, spins: torch.Tensor, grad: torch.Tensor, n_samples, out=None):
        arr, counts = self._counts(n_samples)
        spins = spins.to(device="cuda").contiguous()
        grad = grad.to(device="cuda", dtype=torch.float64).contiguous()
        assert grad.numel() == sum(counts)
        if out is None:
            dh = torch.empty(sum(self.n), device="cuda", dtype=torch.float64)
            dJ = torch.empty(max(sum(self.ne), 1), device="cuda", dtype=torch.float64)
            db = torch.empty(len(self.instances), device="cuda", dtype=torch.float64)
        else:
            dh, dJ, db = out
        _lib.check(_lib.lib().tnvan_logz_backward(self._h, arr, _ptr(spins), _ptr(grad),
                                                  _ptr(dh), _ptr(dJ), _ptr(db),
                                                  _stream()))
        return dh, dJ[:sum(self.ne)], db

    def _adjoint_out(self, out):
        if out is not None:
            return out
        return (torch.empty(sum(self.n), device="cuda", dtype=torch.float64),
                torch.empty(max(sum(self.ne), 1), device="cuda", dtype=torch.float64),
                torch.empty(len(self.instances), device="cuda", dtype=torch.float64))

    def logz_and_backward(self, spins: torch.Tensor, grad: torch.Tensor, n_samples,
                          logz_out: torch.Tensor = None, out=None):
        """logz(spins) and backward(spins, grad) in one call (one contraction
        where the net allows it); returns (logz, dh, dJ, dbeta)."""
        arr, counts = self._counts(n_samples)
        spins = spins.to(device="cuda").contiguous()
        assert spins.dtype == torch.int8
        assert spins.numel() == sum(b * w for b, w in zip(counts, self.nw))
        grad = grad.to(device="cuda", dtype=torch.float64).contiguous()
        assert grad.numel() == sum(counts)
        if logz_out is None:
            logz_out = torch.empty(max(sum(counts), 1), device="cuda", dtype=torch.float64)
        dh, dJ, db = self._adjoint_out(out)
        _lib.check(_lib.lib().tnvan_logz_and_backward(self._h, arr, _ptr(spins), _ptr(grad),
                                                      _ptr(logz_out), _ptr(dh), _ptr(dJ),
                                                      _ptr(db), _stream()))
        return logz_out[:sum(counts)], dh, dJ[:sum(self.ne)], db

    def free_energy_step(self, n_samples, lr: float, stats: torch.Tensor = None,
                         spins_out: torch.Tensor = None, adjoint=None):
        """One training step.  With adjoint=(grad, dh, dJ, dbeta) (device
        float64 tensors; grad per sample, set before the call) the adjoint of
        the sampled spins is computed in the same call."""
        arr, counts = self._counts(n_samples)
        if stats is None:
            stats = torch.empty(len(self.instances), 4, device="cuda", dtype=torch.float64)
        if adjoint is None:
            _lib.check(_lib.lib().tnvan_free_energy_step(self._h, arr, float(lr), _ptr(stats),
                                                         _ptr(spins_out), _stream()))
        else:
            grad, dh, dJ, db = adjoint
            assert grad.dtype == torch.float64 and grad.is_contiguous()
            assert grad.numel() == sum(counts)
            _lib.check(_lib.lib().tnvan_free_energy_step_adjoint(
                self._h, arr, float(lr), _ptr(stats), _ptr(spins_out), _ptr(grad), _ptr(dh),
                _ptr(dJ), _ptr(db), _stream()))
        return stats, spins_out


class LogZ(torch.autograd.Function):
    """logZ_R(s_W) per sample as a differentiable function of (J, h, beta).

        logz = LogZ.apply(J, h, beta, spins, net, n_samples)

    J [sum E], h [sum N] and beta [n_inst] are the couplings, fields and
    inverse temperatures of the net's instances, concatenated in instance
    order.  Where an instance's values differ from those its tables hold
    (compared in the caller's dtype, i.e. the held values rounded to it),
    tnvan_set_couplings compiles that instance again with the values passed
    (as float64) before the forward.  The
    forward is tnvan_logz_batch, the backward tnvan_logz_backward with the
    incoming gradient as g_b, returning (dJ, dh, dbeta) = (beta sum g <x x>,
    beta sum g <r>, -sum g <E_2>) (Eqs. 3-4 differentiated).
    """

    @staticmethod
    def forward(ctx, J, h, beta, spins, net: Net, n_samples):
        got = [t.detach().to("cpu").reshape(-1) for t in (J, h, beta)]
        for name, g, held in zip(("J", "h", "beta"), got, net.couplings):
            if g.shape != held.shape:
                raise ValueError(f"LogZ: {name} has {g.numel()} entries, the net "
                                 f"holds {held.numel()}")
        e0 = n0 = 0
        for k in range(len(net.instances)):
            sl = [slice(e0, e0 + net.ne[k]), slice(n0, n0 + net.n[k]), slice(k, k + 1)]
            if any(not torch.equal(g[s], held[s].to(g.dtype))
                   for g, held, s in zip(got, net.couplings, sl)):
                net.set_couplings(k, got[0][sl[0]].double().numpy(),
                                  got[1][sl[1]].double().numpy(), float(got[2][k]))
            e0 += net.ne[k]
            n0 += net.n[k]
        ctx.net = net
        ctx.n_samples = n_samples
        ctx.meta = [(t.dtype, t.device, t.shape) for t in (J, h, beta)]
        ctx.save_for_backward(spins)
        return net.logz(spins, n_samples).clone()

    @staticmethod
    def backward(ctx, g):
        (spins,) = ctx.saved_tensors
        dh, dJ, db = ctx.net.backward(spins, g.contiguous(), ctx.n_samples)
        out = [t.to(dtype=dt, device=dev).reshape(shape)
               for t, (dt, dev, shape) in zip((dJ, dh, db), ctx.meta)]
        return out[0], out[1], out[2], None, None, None
