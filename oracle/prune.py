"""Contribution-based pruning (Sec. 3.3), in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring): a plain statement of the pruning
step for the tests, ``smoke()`` and the CPU baseline; the product path never imports it.

At every training iteration each Gaussian's opacity o_g and largest scale s_max(g) are
compared with their tau-quantiles over all Gaussians.  A Gaussian under both quantiles is
a pruning candidate of that iteration (the intersection of the opacity and the scale
candidate sets) and gains one vote.  A Gaussian whose votes exceed I_prune * v is removed.
Appendix C (additional implementation details) sets I_prune = 1000, v = 0.6 and tau = 0.2.

Readings (the paper leaves these open):
* Q_tau is the quantile that interpolates linearly between the order statistics around
  position tau (N - 1) of the sorted values (0-based), the usual default of array libraries.
* o_g is the sigmoid of the stored opacity logit and s_max(g) the exponential of the largest
  stored log-scale.
* Votes count within one pruning interval: removal is tested once per interval of I_prune
  iterations, on the votes of that interval, and the survivors' votes then start again
  from zero (a Gaussian goes when its votes exceed the bound within an interval).
* Survivors keep their order.

Table 4 ablates the two criteria: ``criteria`` selects opacity alone, scale alone or both.

Parity pins: ``tests/test_oracle_prune.py`` (rank counts, hand-computed fixtures with ties,
an independent library quantile, special cases, the vote bound).
"""
import numpy as np

__all__ = ["prune_opacity", "prune_max_scale", "quantile", "prune_candidates", "prune_vote",
           "prune_survivors", "PRUNE_TAU", "PRUNE_INTERVAL", "PRUNE_V"]

PRUNE_TAU = 0.2          # Appendix C: the redundancy threshold tau
PRUNE_INTERVAL = 1000    # Appendix C: I_prune
PRUNE_V = 0.6            # Appendix C: vote threshold v


def prune_opacity(opacity_logit):
    """o_g = sigmoid(logit) (Sec. 3.3; the stored parameter is the logit)."""
    x = np.asarray(opacity_logit, dtype=np.float64)
    return 1.0 / (1.0 + np.exp(-x))


def prune_max_scale(log_scale):
    """s_max(g) = max over the three axes of exp(log-scale) (Sec. 3.3); log_scale is [3][N]."""
    return np.exp(np.max(np.asarray(log_scale, dtype=np.float64), axis=0))


def quantile(x, tau):
    """Q_tau(x): linear interpolation between the sorted values at positions k and k + 1,
    k = floor(tau (N - 1)), weight tau (N - 1) - k (the reading stated above)."""
    s = np.sort(np.asarray(x, dtype=np.float64))
    h = float(tau) * (len(s) - 1)
    k = int(np.floor(h))
    if k + 1 >= len(s):
        return s[k]
    return s[k] + (h - k) * (s[k + 1] - s[k])


def prune_candidates(opacity_logit, log_scale, tau=PRUNE_TAU, criteria="both"):
    """C_prune = C_opacity and C_scale: o_g < Q_tau(o) and s_max(g) < Q_tau(s_max) (Sec. 3.3).
    ``criteria`` "opacity" or "scale" keeps one of the two sets alone (Table 4's ablation)."""
    if criteria not in ("both", "opacity", "scale"):
        raise ValueError(f"unknown criteria {criteria!r}")
    o = prune_opacity(opacity_logit)
    s = prune_max_scale(log_scale)
    if o.size == 0:
        return np.zeros(0, dtype=bool)
    c_opacity = o < quantile(o, tau)
    c_scale = s < quantile(s, tau)
    if criteria == "opacity":
        return c_opacity
    if criteria == "scale":
        return c_scale
    return c_opacity & c_scale


def prune_vote(votes, opacity_logit, log_scale, tau=PRUNE_TAU, criteria="both"):
    """V^(t+1) = V^(t) + 1[g in C_prune^(t)] (Sec. 3.3)."""
    cand = prune_candidates(opacity_logit, log_scale, tau, criteria)
    return np.asarray(votes) + cand.astype(np.asarray(votes).dtype)


def prune_survivors(votes, interval=PRUNE_INTERVAL, v=PRUNE_V):
    """Indices of the Gaussians kept at the end of an interval: not (V_g > I_prune * v) (Sec. 3.3),
    in ascending order."""
    return np.nonzero(~(np.asarray(votes, dtype=np.float64) > interval * v))[0]
