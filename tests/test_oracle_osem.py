"""Pins of the oracle's OSEM (Hudson-Larkin; the initialisation of Sec. IV-C):
the count identity of the EM step, the fixed point on consistent data, the
monotone likelihood of MLEM (one subset), agreement with MLEM written on the
brute-force clipped system matrix, and positivity."""
import numpy as np
import pytest

from tests.test_oracle_method import dense_A, g2, g3


def data(orc, g, seed=0, bg=1.0):
    rng = np.random.default_rng(seed)
    f_true = rng.uniform(0.5, 3.0, orc.n_voxels(g))
    q = orc.forward(g, f_true).reshape(-1)
    y = rng.poisson(q + bg).astype(float)
    r = np.full(y.size, bg)
    return f_true, y, r


@pytest.mark.parametrize("dim", [2, 3])
def test_em_count_identity(orc, dim):
    """sum_j (A_i^T 1)_j f_new_j = sum_{rows of subset i} (A_i f)_i y_i / ((A_i f)_i + r_i)."""
    from oracle import osem as O
    g = g2(orc) if dim == 2 else g3(orc)
    _, y, r = data(orc, g)
    rng = np.random.default_rng(5)
    f = rng.uniform(0.2, 2.0, orc.n_voxels(g)).reshape(orc.img_shape(g))
    for i in range(1, g.n_subsets + 1):
        s = O.subset_sensitivity(g, i)
        fn = O.osem_subiteration(g, f, y, r, i)
        q = orc.forward(g, f, i).reshape(-1)
        rows = np.zeros(orc.sino_shape(g), bool)
        rows[:, (i - 1)::g.n_subsets, :] = True
        rows = rows.reshape(-1)
        rhs = np.sum(q[rows] * y[rows] / (q[rows] + r[rows]))
        assert np.sum(s * fn) == pytest.approx(rhs, rel=1e-12)


def test_fixed_point_on_consistent_data(orc):
    from oracle import osem as O
    g = g2(orc)
    f_true, _, r = data(orc, g)
    y = orc.forward(g, f_true).reshape(-1) + r        # noise-free, consistent
    f = f_true.reshape(orc.img_shape(g))
    for i in range(1, g.n_subsets + 1):
        fn = O.osem_subiteration(g, f, y, r, i)
        assert np.max(np.abs(fn - f)) <= 1e-12 * np.max(f)


def test_mlem_likelihood_monotone_and_dense(orc):
    """One subset: OSEM is MLEM, whose Poisson likelihood never decreases
    (its negative, the fidelity, never increases); and it equals MLEM written
    on the brute-force system matrix."""
    from oracle import osem as O
    g = g2(orc, n=6, na=8, nr=9, M=1)
    _, y, r = data(orc, g, 3)
    A = dense_A(orc, g)
    f = np.ones(orc.n_voxels(g))
    fd = f.copy()
    prev = orc.fidelity(g, f, y, r)
    s = A.sum(axis=0)
    for _ in range(15):
        f = O.osem(g, f, y, r, 1).reshape(-1)
        cur = orc.fidelity(g, f, y, r)
        assert cur <= prev + 1e-9 * abs(prev)
        prev = cur
        fd = np.where(s > 0, fd * (A.T @ (y / (A @ fd + r))) / np.where(s > 0, s, 1.0), fd)
        assert np.max(np.abs(f - fd)) <= 1e-10 * np.max(fd)


def test_positivity_and_zero_pixels(orc):
    from oracle import osem as O
    g = g2(orc)
    _, y, r = data(orc, g, 9)
    f = np.ones(orc.img_shape(g))
    f[2, 3] = 0.0
    out = O.osem(g, f, y, r, 3)
    assert out[2, 3] == 0.0
    assert (out >= 0).all() and (out[f > 0] > 0).all()
