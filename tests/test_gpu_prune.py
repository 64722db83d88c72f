"""Contribution-based pruning (Sec. 3.3) through the C ABI against the FP64 oracle, bit for bit:
candidate flags and votes over several iterations (random attributes, ties at the quantile,
signed zeros, all-equal and tiny inputs, up to the 1M-Gaussian scene), the survivors' indices
and counts, the reset votes, and the gathered attribute planes."""
import numpy as np
import pytest
import torch

import mgs_data
import oracle as O
from gpu_helpers import say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(300)]
P = O.prune


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11531_amd as M
    from paper_2603_11531_amd import prune
    M._lib.lib()
    return prune


def _attrs(n, seed, ties=False, zeros=False):
    rng = np.random.default_rng(seed)
    logit = rng.normal(0.0, 1.5, n).astype(np.float32)
    ls = rng.normal(-3.5, 0.5, (3, n)).astype(np.float32)
    if ties and n > 4:
        # many copies of the values at and near the 0.2 / 0.5 quantiles
        s = np.sort(logit)
        for q in (0.2, 0.5):
            v = s[int(q * (n - 1))]
            logit[rng.choice(n, n // 8, replace=False)] = v
        m = np.sort(ls.max(axis=0))[int(0.2 * (n - 1))]
        ls[:, rng.choice(n, n // 8, replace=False)] = m
    if zeros and n > 4:
        logit[rng.choice(n, n // 3, replace=False)] = 0.0
        logit[rng.choice(n, n // 3, replace=False)] = -0.0
    return logit, ls


def _gpu_candidates(M, logit, ls, tau, criteria="both"):
    pr = M.Pruner(logit.size, tau=tau, criteria=criteria)
    cand = torch.zeros(max(logit.size, 1), dtype=torch.uint8, device="cuda")
    lt, lst = torch.from_numpy(logit).cuda(), torch.from_numpy(np.ascontiguousarray(ls)).cuda()
    pr.vote(lt, lst, cand)
    torch.cuda.synchronize()
    return cand[:logit.size].cpu().numpy().astype(bool), pr.votes[:logit.size].cpu().numpy()


@pytest.mark.parametrize("n", [1, 2, 5, 1000, 4097, 100_003])
@pytest.mark.parametrize("kind", ["random", "ties", "zeros"])
def test_candidates_equal_oracle(M, n, kind):
    logit, ls = _attrs(n, n + len(kind), ties=kind == "ties", zeros=kind == "zeros")
    for tau in (0.0, 0.2, 0.5, 0.73, 1.0):
        say(f"test_candidates_equal_oracle n={n} kind={kind} tau={tau}")
        got, votes = _gpu_candidates(M, logit, ls, tau)
        want = P.prune_candidates(logit, ls, tau)
        assert np.array_equal(got, want), f"{int((got != want).sum())} flags differ"
        assert np.array_equal(votes, want.astype(np.int32))



@pytest.mark.parametrize("criteria", ["opacity", "scale"])
def test_single_criterion_ablation_equals_oracle(M, criteria):
    """Table 4's ablation: one criterion alone, on random attributes and with ties."""
    for n, ties in ((5000, False), (20_001, True)):
        logit, ls = _attrs(n, 77 + n, ties=ties)
        for tau in (0.2, 0.6):
            say(f"test_single_criterion_ablation_equals_oracle {criteria} n={n} tau={tau}")
            got, _ = _gpu_candidates(M, logit, ls, tau, criteria)
            assert np.array_equal(got, P.prune_candidates(logit, ls, tau, criteria))


def test_all_equal_and_constant_axes(M):
    n = 3000
    logit = np.full(n, 0.7, np.float32)
    ls = np.full((3, n), -2.0, np.float32)
    for tau in (0.0, 0.2, 1.0):
        got, _ = _gpu_candidates(M, logit, ls, tau)
        assert not got.any()
    ls[0, ::2] = -1.0               # largest axis differs from the others for every second Gaussian
    logit[::3] = -1.0
    got, _ = _gpu_candidates(M, logit, ls, 0.5)
    assert np.array_equal(got, P.prune_candidates(logit, ls, 0.5))


def test_votes_over_iterations_and_compaction_match_oracle(M):
    """An interval of 12 iterations of slowly changing attributes (as during training), then
    pruning at I_prune = 12, v = 0.5: votes, survivors, reset votes and gathered planes."""
    say("test_votes_over_iterations_and_compaction_match_oracle")
    scene = mgs_data.make_scene_uniform(50_000, 3)
    pr = M.Pruner(50_000, tau=0.2, interval=12, v=0.5)
    want = np.zeros(50_000, np.int64)
    for it in range(12):
        sc = mgs_data.perturb_scene(scene, 100 + it, mean_sd=0.0, opac_sd=0.3)
        logit = np.ascontiguousarray(sc["opacity_logit"], np.float32)
        noise = np.random.default_rng(200 + it).normal(0.0, 0.05, (3, 50_000)).astype(np.float32)
        ls = np.ascontiguousarray(sc["log_scale"], np.float32) + noise
        pr.vote(torch.from_numpy(logit).cuda(), torch.from_numpy(ls).cuda())
        want = P.prune_vote(want, logit, ls, 0.2)
    torch.cuda.synchronize()
    assert np.array_equal(pr.votes.cpu().numpy(), want)
    keep = P.prune_survivors(want, 12, 0.5)
    say(f"  max votes {int(want.max())}, survivors {keep.size} of 50000")
    assert 0 < keep.size < 50_000
    tens = {k: torch.from_numpy(np.ascontiguousarray(scene[k], np.float32)).cuda() for k in mgs_data_keys()}
    out, kept = pr.prune(tens)
    assert np.array_equal(kept.cpu().numpy(), keep)
    for k, t in out.items():
        assert np.array_equal(t.cpu().numpy(), np.ascontiguousarray(scene[k], np.float32)[..., keep]), k
    assert pr.n == keep.size and int(pr.votes.abs().sum()) == 0


def mgs_data_keys():
    return ("mean", "log_scale", "quat", "opacity_logit", "sh")


@pytest.mark.parametrize("n", [0, 1, 4095, 4096, 4097, 300_001])
def test_compaction_equals_oracle_survivors(M, n):
    say(f"test_compaction_equals_oracle_survivors n={n}")
    rng = np.random.default_rng(n)
    votes = rng.integers(0, 1001, n).astype(np.int32)
    votes[rng.random(n) < 0.3] = 600          # at the bound: kept
    votes[rng.random(n) < 0.1] = 601          # just over: pruned
    pr = M.Pruner(n)
    if n:
        pr.votes[:n] = torch.from_numpy(votes).cuda()
    idx, cnt = pr.compact()
    torch.cuda.synchronize()
    keep = P.prune_survivors(votes, 1000, 0.6)
    m = int(cnt.cpu()[0])
    assert m == keep.size
    assert np.array_equal(idx[:m].cpu().numpy(), keep)
    if n:
        assert int(pr.votes[:n].abs().sum()) == 0


def test_full_scene_candidates(M):
    """The 1M-Gaussian unbounded scene (tau = 0.2, Appendix C)."""
    say("test_full_scene_candidates")
    scene, _, _, _ = mgs_data.make_config("unbounded", seed=0)
    logit = np.ascontiguousarray(scene["opacity_logit"], np.float32)
    ls = np.ascontiguousarray(scene["log_scale"], np.float32)
    got, _ = _gpu_candidates(M, logit, ls, 0.2)
    want = P.prune_candidates(logit, ls, 0.2)
    say(f"  candidates {int(want.sum())} of {want.size}")
    assert np.array_equal(got, want)


def test_argument_checks(M):
    from paper_2603_11531_amd import _lib as L
    pr = M.Pruner(10)
    x = torch.zeros(10, device="cuda")
    with pytest.raises(L.MgsError):
        L.check(L.lib().mgs_prune_vote(L.ptr(x), L.ptr(x), 10, 1.5, 3, L.ptr(pr.ws), pr.ws.numel() * 4,
                                       L.ptr(pr.votes), None, L.stream_ptr()))
    with pytest.raises(L.MgsError):
        L.check(L.lib().mgs_prune_vote(L.ptr(x), L.ptr(x), 10, 0.2, 3, L.ptr(pr.ws), 16, L.ptr(pr.votes), None,
                                       L.stream_ptr()))


def test_training_continues_on_the_pruned_scene(M):
    """Pruning inside a training loop: three iterations of render, L1 loss, backward and a small
    gradient step, each followed by the vote (checked against the oracle's votes on the same
    parameter values); at the interval's end the pruned scene is the oracle's survivors in order,
    renders bit-identically to the scene indexed by them, and trains on (backward runs)."""
    say("test_training_continues_on_the_pruned_scene")
    from paper_2603_11531_amd.autograd import render
    scene = mgs_data.make_scene_uniform(3000, 9)
    cam = mgs_data.look_at((0.2, -0.1, -4.0), width=96, height=80, f=96.0)
    keys = mgs_data_keys()
    params = {k: torch.tensor(np.ascontiguousarray(scene[k], np.float32), device="cuda", requires_grad=True)
              for k in keys}
    target = torch.full((3, 80, 96), 0.25, device="cuda")
    pr = M.Pruner(3000, tau=0.2, interval=3, v=0.5)
    want = np.zeros(3000, np.int64)
    for it in range(3):
        for p in params.values():
            p.grad = None
        (render(params, cam) - target).abs().mean().backward()
        with torch.no_grad():
            for k in ("opacity_logit", "log_scale"):
                params[k] -= 50.0 * params[k].grad
        pr.vote(params["opacity_logit"].detach(), params["log_scale"].detach())
        want = P.prune_vote(want, params["opacity_logit"].detach().cpu().numpy(),
                            params["log_scale"].detach().cpu().numpy(), 0.2)
    torch.cuda.synchronize()
    assert np.array_equal(pr.votes.cpu().numpy(), want)
    keep = P.prune_survivors(want, 3, 0.5)
    say(f"  survivors {keep.size} of 3000")
    assert 0 < keep.size < 3000
    host = {k: p.detach().cpu().numpy() for k, p in params.items()}
    pruned, kept = pr.prune({k: p.detach() for k, p in params.items()})
    assert np.array_equal(kept.cpu().numpy(), keep)
    pruned = {k: t.requires_grad_(True) for k, t in pruned.items()}
    indexed = {k: torch.tensor(np.ascontiguousarray(host[k][..., keep]), device="cuda") for k in keys}
    img = render(pruned, cam)
    assert torch.equal(img.detach(), render(indexed, cam))
    (img - target).abs().mean().backward()
    assert pruned["mean"].grad.shape == (3, keep.size) and torch.isfinite(pruned["mean"].grad).all()


def test_schedule_prunes_at_interval_ends_and_stops(M):
    """Pruner.step: votes every iteration below `until`, prunes at each interval's end (the
    oracle's survivors of that interval, votes restarting at zero), nothing from `until` on."""
    say("test_schedule_prunes_at_interval_ends_and_stops")
    scene = mgs_data.make_scene_uniform(8000, 13)
    t = {k: torch.tensor(np.ascontiguousarray(scene[k], np.float32), device="cuda") for k in mgs_data_keys()}
    pr = M.Pruner(8000, tau=0.3, interval=2, v=0.5)
    host = {k: np.ascontiguousarray(scene[k], np.float32) for k in mgs_data_keys()}
    votes = np.zeros(8000, np.int64)
    sizes = []
    for it in range(6):
        t, kept = pr.step(it, t, until=4)
        if it < 4:
            votes = P.prune_vote(votes, host["opacity_logit"], host["log_scale"], 0.3)
        if it in (1, 3):
            keep = P.prune_survivors(votes, 2, 0.5)
            assert kept is not None and np.array_equal(kept.cpu().numpy(), keep)
            host = {k: v[..., keep] for k, v in host.items()}
            votes = np.zeros(keep.size, np.int64)
        else:
            assert kept is None
        sizes.append(pr.n)
        assert np.array_equal(t["sh"].cpu().numpy(), host["sh"])
    torch.cuda.synchronize()
    say(f"  sizes {sizes}")
    assert sizes[0] == 8000 and sizes[1] < 8000 and sizes[3] < sizes[1] and sizes[3] == sizes[5]
