"""Error model of the adjoint's batch sums, shared by the GPU parity tests.

Every output of the adjoint is a weighted batch sum of per-sample
conditional moments m_b of the remainder (magnetisations and edge
correlations, |m_b| <= 1):

    dh_i = beta sum_b g_b <r_i>_b,   dJ_e = beta sum_b g_b <x_i x_j>_b,
    dbeta = -sum_b g_b <E_2>_b.

Write the error of one per-sample moment as eps_b = mu + eta_b: a part mu
shared by the samples (a systematic rounding bias) and a part eta_b that
varies from sample to sample, both at most delta in size.  Weighted by g,
the error of an entry is beta (mu sum_b g_b + sum_b g_b eta_b).  The first
term is at most beta delta |sum g|; the second is a sum of terms with
independent signs, at most beta delta sqrt(sum g^2) per standard deviation,
taken here at four.  So each entry obeys

    |error| <= beta delta (|sum g| + 4 sqrt(sum g^2)),

which for g = 1/B is about beta delta, and for random-sign g grows like
sqrt(B), as the entries themselves do.  <E_2>_b is a sum over the
remainder's edges and fields, so dbeta takes the same bound with beta
replaced by sum |J_e| + sum |h_i|.

delta per sample, from the arithmetic of each path (measured errors, in the
design notes, sit 10-40x below these):
  fp64   1e-11   FP64 messages over at most a few hundred steps
  fp32   5e-6    FP32 messages: unit round-off 6e-8 over 16-step chains of
                 32-term products, in relative terms; moments are ratios of
                 two such contractions
  bf16   5e-6    the BF16 precision rounds only the forward products; its
                 adjoint runs on the FP32 tables
  split  1e-4    split-BF16 products keep about 16 bits of each operand
                 (relative error 2^-16 = 1.5e-5 per product before the
                 dropped lo*lo term), over 16 steps
"""

import numpy as np

DELTA = {"fp64": 1e-11, "fp32": 5e-6, "bf16": 5e-6, "split": 1e-4}


def weight_factor(g):
    g = np.asarray(g, np.float64)
    return abs(float(g.sum())) + 4.0 * float(np.sqrt((g * g).sum()))


def vjp_tolerances(inst, g, path):
    """(tolerance of dh and dJ entries, tolerance of dbeta)."""
    w = DELTA[path] * weight_factor(g)
    h = np.zeros(inst.n) if inst.h is None else np.asarray(inst.h)
    jscale = float(np.abs(inst.J).sum() + np.abs(h).sum())
    return float(inst.beta) * w, jscale * w


def check_vjp(got, want, inst, g, path, what=""):
    """Assert the adjoint's (dh, dJ, dbeta) against the oracle's under the
    error model; returns the largest entry error relative to the largest
    entry (for reports)."""
    dh, dJ, db = (np.asarray(x, np.float64) for x in got)
    wdh, wdJ, wdb = (np.asarray(x, np.float64) for x in want)
    tol, tol_b = vjp_tolerances(inst, g, path)
    eh = float(np.abs(dh - wdh).max()) if dh.size else 0.0
    eJ = float(np.abs(dJ - wdJ).max()) if dJ.size else 0.0
    eb = float(np.abs(np.asarray(db).reshape(-1) - np.asarray(wdb).reshape(-1)).max())
    assert eh <= tol, (what, "dh", eh, tol)
    assert eJ <= tol, (what, "dJ", eJ, tol)
    assert eb <= tol_b, (what, "dbeta", eb, tol_b)
    big = max(float(np.abs(wdh).max()) if wdh.size else 0.0,
              float(np.abs(wdJ).max()) if wdJ.size else 0.0, 1e-300)
    return max(eh, eJ) / big
