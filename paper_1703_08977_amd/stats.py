"""Error bars from one run: the delete-one-group jackknife over walker blocks.

he_fk_propagate leaves in its workspace the per-block partial rows
[G][n_samples][8] whose merge is the sample table; each block's rows cover a
fixed set of walkers, so groups of blocks are independent sub-ensembles.  The
grouping, the merge of rows and the replicas are computed by the library
(he_fk_energy_blocks); this module only forwards the call.
"""
from __future__ import annotations

import numpy as np

from .api import he_fk_energy_blocks


def jackknife(partials: np.ndarray, dt_sample: float, e_ref: float, method: str = "window", n_groups: int = 32,
              fit_w=None):
    """(estimate from all walkers, jackknife standard error) of an he_fk_energy estimator."""
    return he_fk_energy_blocks(partials, dt_sample, e_ref, method, n_groups, fit_w)
