"""Iteration diagnostics of a PTP run from its retirement record (host-side
bookkeeping; no arithmetic of the method).

The band of iteration k (paper Sec. 4.2) is [i_k, j_k] with j_k = min(k,
rho - 1) (Eq. upper_band) and i_k the first topleset not yet retired before
iteration k; the retirement record (the last iteration that updated each
topleset, as ``Plan.schedule()`` returns it) therefore fixes the whole band
sequence.  These are the quantities of the paper's band figures (vertices
and toplesets updated per iteration, dynamic band against the fixed half
band of Sec. 6)."""
from __future__ import annotations

import numpy as np


def band_trace(retire, offsets, K):
    """Per iteration k = 1..K: lo (first topleset of the band), j (last),
    toplesets (j - lo + 1) and vertices (|B_k|).  retire[rho], offsets[rho+1]
    (topleset starts, as ``Plan.order()`` returns them)."""
    retire = np.asarray(retire, np.int64)
    offsets = np.asarray(offsets, np.int64)
    rho = retire.shape[0]
    ks = np.arange(1, K + 1)
    j = np.minimum(ks, rho - 1)
    # lo_k = 1 + number of toplesets r >= 1 retired before iteration k
    done = np.where(retire[1:] >= 0, retire[1:], np.iinfo(np.int64).max)
    srt = np.sort(done)
    lo = 1 + np.searchsorted(srt, ks, side="left")
    lo = np.minimum(lo, j)
    return {"k": ks, "lo": lo, "j": j, "toplesets": j - lo + 1,
            "vertices": offsets[j + 1] - offsets[lo]}


def updates(retire, offsets, K) -> int:
    """U = sum over k of |B_k| (Eq. n_operations without the constant)."""
    return int(band_trace(retire, offsets, K)["vertices"].sum())
