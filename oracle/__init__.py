"""FP64 CPU oracle for the Mobile-GS order-independent render pass.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
statement of what the render pass computes, written from the paper
(Mobile-GS, arXiv 2603.11531): Eq. 2 and Eq. 3 (Sec. 3.1) for the
order-independent blend, Eq. 4 for the view-dependent enhancement MLP, and
Eq. 11 (Appendix B) for the sorted alpha-blend comparison path, and the
codebook decode of vector-quantised attributes (Sec. 3.2, ``oracle.nvq``) and the
contribution-based pruning step (Sec. 3.3, ``oracle.prune``).  It shares no
code with the HIP path and imports nothing from it.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path never does.

Every function states the passage it follows; where the paper is silent or
ambiguous, the reading taken is stated beside the code that applies it.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, textbook special cases or brute force,
except what the paper leaves unspecified (fidelity of the readings to the
authors' unreleased code), which is parity unpinned by nature.
"""
from .render import *  # noqa: F401,F403
from .render import __all__  # noqa: F401
from . import nvq  # noqa: F401
from . import prune  # noqa: F401
