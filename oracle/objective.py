"""Oracle for the variational objective and its optimisation.

TEST INFRASTRUCTURE ONLY.

  Etilde(s) = E_1(s) - logZ_R(s) / beta                         (Eq. 4)
  F_q = E_{s~q}[Etilde(s) + ln q(s) / beta]                      (Eq. 9)
  grad F_q = E_{s~q}[(Etilde + ln q / beta) grad ln q(s)]        (Eq. 10)

The batch estimator uses f_b = Etilde(s_b) + ln q(s_b) / beta, F_q = mean f,
and subtracts the batch mean as a baseline (it leaves the expectation of the
estimator unchanged because E_q[grad ln q] = 0): the per-sample REINFORCE
weight is w_b = (f_b - mean f) / B.  The update is Adam (Kingma & Ba 2015)
with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 (the paper says gradient
descent, Algorithm 1 step (d)).

Functions and what pins them (tests/test_oracle_objective.py):
  free_energy_terms   Eq. 9 written out; pinned at beta = 0.5 and 2 by
                      Eq. 5's equality case (q = the W-marginal of p from
                      a full enumeration of Eq. 1 makes every f_b equal
                      -ln Z / beta, its standard error zero, and Etilde
                      equal -(ln p_W + ln Z) / beta), by the KL identity
                      beta (F_q - F) = KL(q | p_W) for a network q, and its
                      standard error by the spread of F_q over 400
                      independent batches
  exact_fq_and_grad   enumeration of all 2^|W| width-set states; pinned by
                      the KL identity of Eq. 5 at beta = 0.5 and 2 and the
                      bound F_q >= F; the exact gradient by central finite
                      differences of the exact F_q, and the sampled
                      REINFORCE estimator is checked against it
                      statistically (beta = 0.5, 1, 2)
  adam_step           pinned by the closed form of the first step
                      (update = lr * g / (|g| + eps)) and a hand-computed
                      second step
  train               Algorithm 1 (sample -> contract -> loss/grad -> update)
  observables         <sigma_i>_p and <sigma_i sigma_j>_p estimated from
                      samples of q by self-normalised importance weights;
                      pinned by the full enumeration of W with uniform q,
                      where the estimate is exact (brute-force moments)
"""

from __future__ import annotations

import numpy as np

from . import ising, made, philox


def free_energy_terms(inst, spins, logq, logz_r):
    """Per-sample f_b and the batch statistics (F_q, stderr, <Etilde>,
    <ln q>/beta)."""
    beta = float(inst.beta)
    e1 = ising.e1_energy(inst, spins)
    et = e1 - np.asarray(logz_r, np.float64) / beta
    f = et + np.asarray(logq, np.float64) / beta
    B = f.shape[0]
    Fq = float(np.mean(f))
    se = float(np.std(f, ddof=1) / np.sqrt(B)) if B > 1 else 0.0
    return f, np.array([Fq, se, float(np.mean(et)),
                        float(np.mean(np.asarray(logq, np.float64) / beta))])


def reinforce_weights(f: np.ndarray) -> np.ndarray:
    f = np.asarray(f, np.float64)
    return (f - f.mean()) / f.shape[0]


def adam_step(theta, grad, m, v, t: int, lr: float, b1=0.9, b2=0.999,
              eps=1e-8):
    """One Adam update; t is the 1-based step number.  Returns new
    (theta, m, v)."""
    g = np.asarray(grad, np.float64)
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def all_width_states(nw: int) -> np.ndarray:
    k = np.arange(2 ** nw, dtype=np.int64)[:, None]
    return (1 - 2 * ((k >> np.arange(nw)[None, :]) & 1)).astype(np.int8)


def exact_free_energy(inst) -> float:
    """F = -ln Z / beta by enumerating all 2^n states (Eq. 1)."""
    return -ising.logz_full_bruteforce(inst) / float(inst.beta)


def exact_fq_and_grad(inst, theta, H: int, logz_fn=None):
    """Exact F_q = sum_s q(s) [Etilde(s) + ln q(s)/beta] over all 2^|W|
    states and its exact gradient, sum_s q(s) f(s) grad ln q(s)."""
    nw = int(inst.width_set.shape[0])
    s = all_width_states(nw)
    lz = (logz_fn or ising.logz_r_elimination)(inst, s)
    lq = made.logq(theta, s, nw, H)
    q = np.exp(lq)
    f = ising.e1_energy(inst, s) - lz / inst.beta + lq / inst.beta
    Fq = float(np.sum(q * f))
    grad = made.logq_backward(theta, s, q * f, nw, H)
    return Fq, grad


def train(inst, theta0, H: int, steps: int, B: int, lr: float, seed: int,
          inst_index: int = 0, logz_fn=None, record=False):
    """Algorithm 1: per epoch sample with Philox uniforms, contract, form
    F_q and the REINFORCE gradient, apply Adam.  Returns the final theta
    and the per-step statistics [steps, 4]."""
    nw = int(inst.width_set.shape[0])
    theta = np.asarray(theta0, np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    stats = []
    lzf = logz_fn or ising.logz_r_elimination
    for t in range(steps):
        u = philox.sampler_uniforms(seed, t, inst_index, B, nw)
        s, lq, _ = made.sample(theta, u, nw, H)
        lz = lzf(inst, s)
        f, st = free_energy_terms(inst, s, lq, lz)
        w = reinforce_weights(f)
        g = made.logq_backward(theta, s, w, nw, H)
        theta, m, v = adam_step(theta, g, m, v, t + 1, lr)
        stats.append(st)
    return theta, np.asarray(stats)


def observables(inst, spins, logq, marg=None):
    """Moments of the Boltzmann distribution p (Eq. 1) from samples of q.

    The W-marginal of p is p(s_W) = exp(-beta E_1(s_W)) Z_R(s_W) / Z, so the
    weight of a sample is p/q up to a constant: exp(-beta f_b) with f_b of
    Eq. 9 (free_energy_terms).  Normalised, w_b = exp(-beta f_b) / sum.
    Each moment is the weighted mean of its conditional expectation given
    s_W: s_i on W vertices, s_i s_j on W-W edges, and the conditional
    marginals and correlations of the remainder (marginals_elimination)
    elsewhere.  Returns (mag [n], corr [E], ess) with the effective sample
    size ess = 1 / sum w_b^2.
    """
    beta = float(inst.beta)
    s = np.asarray(spins)
    if marg is None:
        lz, mag, corr, _ = ising.marginals_elimination(inst, s)
    else:
        lz, mag, corr = marg
    f, _ = free_energy_terms(inst, s, logq, lz)
    lw = -beta * f
    w = np.exp(lw - lw.max())
    w /= w.sum()
    sp = ising.Split(inst)
    sf = s.astype(np.float64)
    m = w @ mag
    for i, v in enumerate(sp.W):
        m[v] = w @ sf[:, i]
    c = w @ corr          # W-W edges: s_a s_b already
    return m, c, float(1.0 / np.sum(w * w))
