"""Error bars from one run: delete-one-group jackknife over walker blocks.

he_fk_propagate leaves in its workspace the per-block partial rows
[G][n_samples][8] whose merge is the sample table; each block's rows cover a
fixed set of walkers, so groups of blocks are independent sub-ensembles.
Merging of rows here is the same rescale-to-the-larger-maximum rule as on
the device; the energy of each replica comes from he_fk_energy.
"""
from __future__ import annotations

import numpy as np

from .api import he_fk_energy


def merge_rows(rows: np.ndarray) -> np.ndarray:
    """Merge partial rows along axis 0: [k, ns, 8] -> [ns, 8]."""
    rows = np.asarray(rows, dtype=np.float64)
    m = rows[:, :, 0].max(axis=0)
    mm = np.where(np.isfinite(m), m, 0.0)
    scale = np.where(np.isfinite(rows[:, :, 0]), np.exp(rows[:, :, 0] - mm[None, :]), 0.0)
    out = np.zeros(rows.shape[1:])
    out[:, 0] = m
    out[:, 1] = (rows[:, :, 1] * scale).sum(axis=0)
    out[:, 2] = (rows[:, :, 2] * scale).sum(axis=0)
    out[:, 3] = (rows[:, :, 3] * scale * scale).sum(axis=0)
    out[:, 4:7] = rows[:, :, 4:7].sum(axis=0)
    return out


def jackknife(partials: np.ndarray, dt_sample: float, e_ref: float, method: str = "window", n_groups: int = 32):
    """(estimate from all walkers, jackknife standard error) of an he_fk_energy estimator (first value)."""
    G = partials.shape[0]
    n_groups = max(2, min(n_groups, G))
    groups = np.array_split(np.arange(G), n_groups)
    grows = np.stack([merge_rows(partials[g]) for g in groups])
    full = merge_rows(grows)
    e_all = he_fk_energy(full, dt_sample, e_ref, method)[0][0]
    reps = np.array([he_fk_energy(merge_rows(np.delete(grows, i, axis=0)), dt_sample, e_ref, method)[0][0]
                     for i in range(n_groups)])
    var = (n_groups - 1) / n_groups * np.sum((reps - reps.mean()) ** 2)
    return float(e_all), float(np.sqrt(var))
