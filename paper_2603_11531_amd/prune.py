"""Contribution-based pruning (Sec. 3.3) through the C ABI.

Every training iteration, ``Pruner.vote`` adds a vote to each Gaussian whose opacity and
largest scale both lie under their tau-quantiles.  At the end of a pruning interval,
``Pruner.prune`` removes the Gaussians with more than I_prune * v votes from every attribute
tensor and starts the next interval's votes from zero.  The defaults are Appendix C's
settings.  All work runs in libmgs.so's kernels; this module only holds the buffers.
"""
import ctypes as C
import math

import torch

from . import _lib as L

TAU, INTERVAL, V = 0.2, 1000, 0.6   # Appendix C: tau, I_prune, v
UNTIL = 25_000                      # Appendix C: pruning only during the first 25k iterations


class Pruner:
    """Vote counts (device uint32, stored as int32) and the pruning workspace for n Gaussians."""

    CRITERIA = {"both": L.MGS_PRUNE_BOTH, "opacity": L.MGS_PRUNE_OPACITY, "scale": L.MGS_PRUNE_SCALE}

    def __init__(self, n, tau=TAU, interval=INTERVAL, v=V, criteria="both", device="cuda"):
        """``criteria``: "both" (Sec. 3.3), or "opacity" / "scale" alone (Table 4's ablation)."""
        if criteria not in self.CRITERIA:
            raise ValueError(f"criteria must be one of {sorted(self.CRITERIA)}")
        self.tau, self.interval, self.v, self.device = float(tau), int(interval), float(v), device
        self.criteria = self.CRITERIA[criteria]
        self._resize(int(n))

    def _resize(self, n):
        self.n = n
        nb = C.c_size_t()
        L.check(L.lib().mgs_prune_workspace(n, C.byref(nb)))
        self.ws = torch.empty(max(1, (nb.value + 255) // 256 * 64), dtype=torch.float32, device=self.device)
        self.votes = torch.zeros(max(n, 1), dtype=torch.int32, device=self.device)
        self.keep_index = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        self.n_keep = torch.zeros(1, dtype=torch.int32, device=self.device)

    @property
    def max_votes(self):
        """floor(I_prune * v): integer votes exceed I_prune * v exactly when they exceed this."""
        return int(math.floor(self.interval * self.v))

    def vote(self, opacity_logit, log_scale, candidates=None, stream=None):
        """One iteration's votes from opacity_logit [n] and log_scale [3][n] (device float32).
        ``candidates`` (uint8 [n]) receives the iteration's candidate flags when given."""
        if opacity_logit.numel() != self.n or log_scale.shape != (3, self.n):
            raise ValueError(f"expected opacity_logit [{self.n}] and log_scale [3, {self.n}]")
        if not (opacity_logit.is_contiguous() and log_scale.is_contiguous()):
            raise ValueError("opacity_logit / log_scale must be contiguous")
        if candidates is not None and (candidates.dtype != torch.uint8 or candidates.numel() < self.n):
            raise ValueError("candidates must be uint8 with n entries")
        L.check(L.lib().mgs_prune_vote(L.ptr(opacity_logit), L.ptr(log_scale), self.n, self.tau, self.criteria,
                                       L.ptr(self.ws),
                                       self.ws.numel() * 4, L.ptr(self.votes), L.ptr(candidates),
                                       L.stream_ptr(stream)))

    def compact(self, stream=None):
        """The survivors' indices (ascending, in keep_index) and their count (n_keep, device);
        resets the votes."""
        L.check(L.lib().mgs_prune_compact(L.ptr(self.votes), self.n, self.max_votes, L.ptr(self.ws),
                                          self.ws.numel() * 4, L.ptr(self.keep_index), L.ptr(self.n_keep),
                                          L.stream_ptr(stream)))
        return self.keep_index, self.n_keep

    def gather(self, t, m, stream=None):
        """Rows [.., n] of t at keep_index[:m] as a new tensor [.., m] (one kernel per tensor); m is
        the survivor count of the last compact()."""
        if t.shape[-1] != self.n or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"expected a contiguous float32 tensor with last dimension {self.n}")
        planes = 1 if t.dim() == 1 else int(math.prod(t.shape[:-1]))
        out = torch.empty(t.shape[:-1] + (m,), dtype=torch.float32, device=t.device)
        if m > 0:
            L.check(L.lib().mgs_gather_planes(L.ptr(t), self.n, planes, L.ptr(self.keep_index), L.ptr(self.n_keep),
                                              m, L.ptr(out), m, L.stream_ptr(stream)))
        return out

    def prune(self, tensors, stream=None):
        """End of a pruning interval: returns ({name: tensor without the pruned Gaussians}, kept
        index tensor) for every [.., n] float32 tensor of ``tensors``; the next interval's votes
        start from zero for the survivors.  Reads the survivor count back to the host."""
        self.compact(stream)
        (torch.cuda.current_stream() if stream is None else stream).synchronize()
        m = int(self.n_keep.cpu()[0])
        out = {k: self.gather(t, m, stream) for k, t in tensors.items()}
        kept = self.keep_index[:m].clone()
        self._resize(m)
        return out, kept

    def step(self, iteration, tensors, until=UNTIL, stream=None):
        """Appendix C's schedule for training iteration ``iteration`` (0-based): below ``until``,
        vote on tensors["opacity_logit"] / tensors["log_scale"], and at the end of every pruning
        interval prune every tensor.  Returns (tensors, kept index or None): the pruned tensors
        at an interval's end, else the same tensors."""
        if iteration >= until:
            return tensors, None
        self.vote(tensors["opacity_logit"], tensors["log_scale"], stream=stream)
        if (iteration + 1) % self.interval:
            return tensors, None
        return self.prune(tensors, stream=stream)
