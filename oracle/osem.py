"""FP64 oracle of the OSEM initialisation (Sec. IV-C: the SDP-BSREM runs on
clinical data start from 2 iterations of OSEM with 24 subsets).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``; shares no code with the
HIP path.

Ordered-subsets EM of Hudson and Larkin (the paper's reference for it), with
the subsets of the reconstruction (interleaved angles, processed 1..M): for
subset i,
    f_j <- f_j * (A_i^T (y_i / (A_i f + r_i)))_j / (A_i^T 1)_j,
and f_j unchanged where the subset sensitivity (A_i^T 1)_j is zero.
"""
from __future__ import annotations

import numpy as np

from . import back, forward, img_shape, sino_shape


def subset_sensitivity(g, subset):
    """A_i^T 1 (subset 1..M; 0 = every ray)."""
    return _back_ones(g, subset)


def _back_ones(g, subset):
    return back(g, np.ones(sino_shape(g)), subset)


def osem_subiteration(g, f, y, r, subset, sens=None):
    """One OSEM update with subset `subset`; returns the new image."""
    f = np.asarray(f, np.float64).reshape(img_shape(g))
    y = np.asarray(y, np.float64).reshape(sino_shape(g))
    r = np.asarray(r, np.float64).reshape(sino_shape(g))
    s = _back_ones(g, subset) if sens is None else sens
    q = forward(g, f, subset)
    ratio = np.zeros_like(q)
    M = g.n_subsets
    sel = np.zeros(q.shape, bool)
    if subset == 0:
        sel[...] = True
    else:
        sel[:, (subset - 1)::M, :] = True
    ratio[sel] = y[sel] / (q[sel] + r[sel])
    b = back(g, ratio, subset)
    out = f.copy()
    pos = s > 0
    out[pos] = f[pos] * b[pos] / s[pos]
    return out


def osem(g, f0, y, r, n_iter):
    """n_iter OSEM iterations (M subiterations each) from f0."""
    M = g.n_subsets
    sens = [_back_ones(g, i) for i in range(1, M + 1)]
    f = np.asarray(f0, np.float64).reshape(img_shape(g)).copy()
    for _ in range(n_iter):
        for i in range(1, M + 1):
            f = osem_subiteration(g, f, y, r, i, sens[i - 1])
    return f
