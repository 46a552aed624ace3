"""FP64 oracle of the gradient-consistency diagnostic (Sec. IV-B, "Comparison
of Gradient Consistency", Fig. 2).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: imported by ``tests/``
and nothing in the product package.  Built on the oracle's own projector,
penalty and gradient-magnitude routines; shares no code with the HIP path.

Definitions followed:
- subset objective (Sec. II-B):
  Phi_i(f) = <A_i f, 1> - <ln(A_i f + gamma_i), g_i> + (beta/M) R(f);
  its gradient A_i^T (1 - g_i / (A_i f + gamma_i)) + (beta/M) grad R(f).
  subset = 0 means every ray and the full weight beta (Phi itself).
- smooth and variable areas: I_s = {j : grad(f)_j < 0.01 mean(f)},
  I_v = {j : grad(f)_j > 0.2 mean(f)}, grad the Matlab-style gradient
  magnitude of the smoothness measure (Sec. III-B).
- angle theta(v1, v2) = arccos(<v1, v2> / (|v1| |v2|)) of the two vectors
  restricted to the area.
- sequence: after subiteration (k, i) has produced f^{k,i}, the gradient
  h^{k,i} = grad Phi_i(f^{k,i}); theta_{k,i} is the angle between h^{k,i-1}
  and h^{k,i} on I_s^{k,i} (areas taken from f^{k,i}); h^{k,0} =
  grad Phi_M(f^{k,0}) (Phi_0 := Phi_M), which for k >= 1 is h^{k-1,M}.
  theta_k is the mean of theta_{k,i} over i = 1..M; the same on I_v gives
  the tilde sequence.
"""
from __future__ import annotations

import math

import numpy as np

from . import back, forward, grad_mag, img_shape, rdp_grad, rdp_value

SMOOTH_FRAC, VAR_FRAC = 0.01, 0.2


def subset_objective(g, f, y, r, subset, beta, gamma_R, eps):
    """Phi_i(f) from its definition (subset 0: Phi(f))."""
    M = g.n_subsets
    q = forward(g, f, subset)
    sel = _subset_rows(g, subset)
    qs, ys, rs = q[sel], _sino(g, y)[sel], _sino(g, r)[sel]
    w = beta if subset == 0 else beta / M
    return float(np.sum(qs) - np.sum(ys * np.log(qs + rs)) + w * rdp_value(g, f, gamma_R, eps))


def subset_gradient(g, f, y, r, subset, beta, gamma_R, eps):
    """grad Phi_i(f) = A_i^T (1 - y / (A_i f + r)) + (beta/M) grad R(f)."""
    M = g.n_subsets
    q = forward(g, f, subset)
    sel = _subset_rows(g, subset)
    ratio = np.zeros_like(q)
    ratio[sel] = 1.0 - _sino(g, y)[sel] / (q[sel] + _sino(g, r)[sel])
    w = beta if subset == 0 else beta / M
    return back(g, ratio, subset) + w * rdp_grad(g, f, gamma_R, eps)


def _sino(g, x):
    from . import sino_shape
    return np.asarray(x, np.float64).reshape(sino_shape(g))


def _subset_rows(g, subset):
    """Boolean mask of the sinogram entries of a subset (interleaved angles:
    angle a belongs to subset (a mod M) + 1)."""
    from . import sino_shape
    shp = sino_shape(g)
    sel = np.zeros(shp, dtype=bool)
    if subset == 0:
        sel[...] = True
    else:
        sel[:, (subset - 1)::g.n_subsets, :] = True
    return sel


def areas(g, f, smooth_frac=SMOOTH_FRAC, var_frac=VAR_FRAC):
    """(I_s, I_v) as boolean images."""
    gm = grad_mag(g, f)
    m = float(np.mean(np.asarray(f, np.float64)))
    return gm < smooth_frac * m, gm > var_frac * m


def angle(v1, v2):
    """theta(v1, v2) in radians; NaN when either vector is zero or empty."""
    v1 = np.asarray(v1, np.float64).ravel()
    v2 = np.asarray(v2, np.float64).ravel()
    n1, n2 = float(np.dot(v1, v1)), float(np.dot(v2, v2))
    if n1 == 0.0 or n2 == 0.0:
        return math.nan
    c = float(np.dot(v1, v2)) / math.sqrt(n1 * n2)
    return math.acos(max(-1.0, min(1.0, c)))


def gradient_angles(g, h_prev, h_cur, f, smooth_frac=SMOOTH_FRAC, var_frac=VAR_FRAC):
    """(theta on I_s, theta on I_v, |I_s|, |I_v|) with the areas of f."""
    s, v = areas(g, f, smooth_frac, var_frac)
    hp = np.asarray(h_prev, np.float64).reshape(img_shape(g))
    hc = np.asarray(h_cur, np.float64).reshape(img_shape(g))
    return angle(hp[s], hc[s]), angle(hp[v], hc[v]), int(s.sum()), int(v.sum())


def consistency_sequence(recon, n_iter):
    """Run n_iter iterations of the oracle reconstruction ``recon`` (an
    ``oracle.Recon`` at the start of an iteration) and return
    (theta[k][i], theta_tilde[k][i]) in radians."""
    g, p = recon.g, recon.p
    M = g.n_subsets
    h_prev = subset_gradient(g, recon.f, recon.y, recon.r, M, p.beta, p.gamma_R, p.eps)
    th, tt = [], []
    for _ in range(n_iter):
        row_s, row_v = [], []
        for i in range(1, M + 1):
            recon.subiteration()
            h = subset_gradient(g, recon.f, recon.y, recon.r, i, p.beta, p.gamma_R, p.eps)
            a_s, a_v, _, _ = gradient_angles(g, h_prev, h, recon.f)
            row_s.append(a_s)
            row_v.append(a_v)
            h_prev = h
        th.append(row_s)
        tt.append(row_v)
    return th, tt
