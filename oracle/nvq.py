"""Decode of vector-quantised Gaussian attributes (test infrastructure; a lookup, so exact).

Neural vector quantization (Sec. 3.2, and the implementation details in the appendix):
the per-Gaussian attribute vector is cut into K sub-vectors, each quantised with its own
codebook of B codewords; the deployed renderer keeps only the codes and the codebooks
(the group MLPs that refine the codewords are applied once, to the codebooks, so the
per-frame decode is a lookup).  The paper uses five groups and B = 2^10 (codebook-size
study).  Reading taken here (the paper does not list the grouping): positions stay
float32, and the 20 other attributes, in the order

    [log_scale(3), quat(4) (w, x, y, z), opacity_logit, sh(12) (plane 3k + ch)]

are cut into five consecutive sub-vectors of four values:

    group 0 = log_scale 0..2, quat w      group 1 = quat x, y, z, opacity_logit
    group 2 = sh 0..3                     group 3 = sh 4..7        group 4 = sh 8..11

decode() returns a scene dict in the layout of mgs_data scenes, which the rest of the
oracle renders unchanged.
"""
from __future__ import annotations

import numpy as np

GROUPS, DIM = 5, 4


def decode(codes, codebooks, mean):
    """codes [5][N] integer, codebooks [5][B][4], mean [3][N] -> scene dict (float32 arrays).

    Attribute value j of group g of Gaussian i is codebooks[g][codes[g][i]][j].
    """
    codes = np.asarray(codes)
    cb = np.asarray(codebooks, np.float32)
    assert codes.shape[0] == GROUPS and cb.shape[0] == GROUPS and cb.shape[2] == DIM
    n = codes.shape[1]
    rows = np.empty((n, GROUPS * DIM), np.float32)
    for g in range(GROUPS):
        rows[:, g * DIM:(g + 1) * DIM] = cb[g][codes[g].astype(np.int64)]
    return dict(mean=np.ascontiguousarray(mean, np.float32),
                log_scale=np.ascontiguousarray(rows[:, 0:3].T),
                quat=np.ascontiguousarray(rows[:, 3:7].T),
                opacity_logit=np.ascontiguousarray(rows[:, 7]),
                sh=np.ascontiguousarray(rows[:, 8:20].T))
