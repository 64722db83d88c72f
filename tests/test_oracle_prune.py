"""Pins of the pruning oracle (Sec. 3.3) against what the definitions fix: counts below a
quantile from the ranks, hand-computed cases with ties, a library quantile, textbook special
cases, brute force over ranks for the candidate sets, and the vote bound of Appendix C."""
import math

import numpy as np
import pytest

import oracle as O

P = O.prune


def _below_count_distinct(n, tau):
    """Distinct values: Q_tau lies strictly between the k-th and (k+1)-th smallest when tau (N - 1)
    has a fractional part (k + 1 values below it), else it is the k-th (k values below)."""
    h = tau * (n - 1)
    k = math.floor(h)
    return k + 1 if h > k else k


@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 10, 97, 1000])
@pytest.mark.parametrize("tau", [0.0, 0.1, 0.2, 0.25, 0.5, 0.75, 0.9, 1.0])
def test_values_below_quantile_from_ranks(n, tau):
    x = np.random.default_rng(n).permutation(n).astype(np.float64) * 0.37 - 5.0
    assert int((x < P.quantile(x, tau)).sum()) == _below_count_distinct(n, tau)


@pytest.mark.parametrize("tau,q,below", [
    (0.4, 1.0, 0),     # position 2.0: the third value (1), nothing is strictly below it
    (0.5, 1.5, 3),     # position 2.5: halfway between 1 and 2
    (0.7, 2.0, 3),     # position 3.5: between two 2s
    (0.9, 2.5, 5),     # position 4.5: halfway between 2 and 3
    (1.0, 3.0, 5),
    (0.0, 1.0, 0),
])
def test_quantile_with_ties_by_hand(tau, q, below):
    x = np.array([2.0, 1.0, 3.0, 1.0, 2.0, 1.0])        # sorted: 1 1 1 2 2 3
    assert P.quantile(x, tau) == pytest.approx(q, abs=1e-15)
    assert int((x < P.quantile(x, tau)).sum()) == below


@pytest.mark.parametrize("seed", range(4))
def test_quantile_equals_library_linear_quantile(seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=int(rng.integers(2, 5000)))
    for tau in (0.0, 0.2, 0.37, 0.5, 0.999, 1.0):
        assert P.quantile(x, tau) == pytest.approx(float(np.quantile(x, tau, method="linear")), rel=1e-14, abs=1e-14)


def test_special_cases():
    x = np.array([4.0, -1.0, 7.0, 2.0, 9.0])
    assert P.quantile(x, 0.0) == -1.0 and P.quantile(x, 1.0) == 9.0 and P.quantile(x, 0.5) == 4.0   # min, max, median
    z = np.zeros(3, np.float32)
    assert not P.prune_candidates(z, np.zeros((3, 3), np.float32), 0.5).any()    # all equal: nothing below
    assert P.prune_candidates(np.zeros(0, np.float32), np.zeros((3, 0), np.float32)).shape == (0,)
    assert not P.prune_candidates(np.ones(1, np.float32), np.ones((3, 1), np.float32)).any()


def _brute_candidates(logit, log_scale, tau):
    """Candidate test from ranks in the stored parameters (sigmoid and exp are increasing):
    x_g < Q_tau <=> x_g <= x_(k) if Q_tau is strictly between x_(k) and x_(k+1), else x_g < x_(k)."""
    n = logit.size
    h = tau * (n - 1)
    k = math.floor(h)

    def below(x):
        s = sorted(float(v) for v in x)
        xk = s[k]
        inclusive = h > k and k + 1 < n and s[k + 1] > xk
        return np.array([(v <= xk) if inclusive else (v < xk) for v in map(float, x)])

    smax = np.array([max(float(log_scale[0, g]), float(log_scale[1, g]), float(log_scale[2, g])) for g in range(n)])
    return below(logit) & below(smax)


@pytest.mark.parametrize("seed", range(6))
def test_candidates_equal_rank_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 60))
    logit = rng.normal(0, 1.5, n).astype(np.float32)
    ls = rng.normal(-3.5, 0.5, (3, n)).astype(np.float32)
    if seed % 2:                                   # ties at the quantile
        logit[: n // 2] = logit[0]
        ls[:, : n // 3] = ls[:, :1]
    for tau in (0.0, 0.2, 0.5, 0.8, 1.0):
        np.testing.assert_array_equal(P.prune_candidates(logit, ls, tau), _brute_candidates(logit, ls, tau))


def test_candidates_need_both_criteria_and_the_largest_axis():
    n = 20
    logit = np.arange(n, dtype=np.float32)                 # opacity increases with g
    ls = np.zeros((3, n), np.float32)
    ls[1] = -np.arange(n, dtype=np.float32)                # largest log-scale decreases ...
    ls[0] = -100.0
    ls[2] = -100.0 + np.arange(n, dtype=np.float32)        # ... smallest axis increases
    # low opacity = small g, low largest scale = large g: disjoint, so no candidate
    assert not P.prune_candidates(logit, ls, 0.3).any()
    # the same order for both: the low-opacity set
    ls2 = np.stack([np.arange(n, dtype=np.float32)] * 3)
    got = np.nonzero(P.prune_candidates(logit, ls2, 0.3))[0]
    np.testing.assert_array_equal(got, np.arange(_below_count_distinct(n, 0.3)))



def test_single_criterion_ablations():
    """Table 4's ablation: opacity alone and scale alone are the rank-count sets of one attribute;
    both is their intersection."""
    rng = np.random.default_rng(7)
    n = 200
    logit = (rng.permutation(n) * 0.05 - 5.0).astype(np.float32)        # distinct, inside sigmoid's range
    ls = rng.normal(-3.0, 0.5, (3, n)).astype(np.float32)
    for tau in (0.2, 0.5):
        want = _below_count_distinct(n, tau)
        co = P.prune_candidates(logit, ls, tau, "opacity")
        cs = P.prune_candidates(logit, ls, tau, "scale")
        assert int(co.sum()) == want and int(cs.sum()) == want
        np.testing.assert_array_equal(co, logit < np.sort(logit)[want])  # the `want` smallest logits
        np.testing.assert_array_equal(P.prune_candidates(logit, ls, tau), co & cs)
    with pytest.raises(ValueError):
        P.prune_candidates(logit, ls, 0.2, "neither")


def test_votes_and_the_removal_bound():
    votes = np.array([0, 599, 600, 601, 1000], np.uint32)
    # I_prune * v = 600 (Appendix C): 600 votes stay, 601 go
    np.testing.assert_array_equal(P.prune_survivors(votes, 1000, 0.6), [0, 1, 2])
    np.testing.assert_array_equal(P.prune_survivors(votes, 10, 0.55), [0])    # 5.5: more than 5.5 is 6 and up
    logit = np.array([-3.0, 2.0, -2.0, 1.0, 0.5], np.float32)
    ls = np.array([[-5.0, 1.0, -4.0, 0.0, -1.0]] * 3, np.float32)
    v = np.zeros(5, np.uint32)
    for _ in range(7):
        v = P.prune_vote(v, logit, ls, 0.5)
    # tau = 0.5 over 5 values: the median; below it in both: Gaussians 0 and 2
    np.testing.assert_array_equal(v, [7, 0, 7, 0, 0])
    np.testing.assert_array_equal(P.prune_survivors(v, 10, 0.7), [0, 1, 2, 3, 4])    # 7 votes: not more than 7
    np.testing.assert_array_equal(P.prune_survivors(v, 10, 0.6), [1, 3, 4])          # more than 6


def test_appendix_settings():
    assert (P.PRUNE_TAU, P.PRUNE_INTERVAL, P.PRUNE_V) == (0.2, 1000, 0.6)
