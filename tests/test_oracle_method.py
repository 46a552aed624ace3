"""Pins of the oracle's SDP-BSREM arithmetic against what the paper and the
mathematics fix: finite differences, homogeneity (Euler) identities, the
Hessian's null vector, numpy's gradient, the scalar-sequence limits of the
proof of thm:SpecificSDPs, the MLEM special case, and convergence to an
independently computed minimiser on tiny dense problems."""
import math

import numpy as np
import pytest


def g2(orc, n=8, na=12, nr=13, v=2.0, M=3):
    return orc.geom(dict(dim=2, nx=n, ny=n, vx=v, vy=v, n_angles=na, n_radial=nr, ds=v, n_subsets=M))


def g3(orc, n=5, nz=4, na=6, nr=9, M=2):
    return orc.geom(dict(dim=3, nx=n, ny=n, nz=nz, vx=2.0, vy=2.0, vz=3.0, n_angles=na,
                         n_radial=nr, ds=2.0, n_rings=nz, max_ring_diff=2, ring_pitch=3.0,
                         det_radius=50.0, n_subsets=M))


def dense_A(orc, g):
    """System matrix by brute-force clipping (no Siddon trace involved)."""
    P, nv = orc.n_planes(g), orc.n_voxels(g)
    nz = g.nz if g.dim == 3 else 1
    A = np.zeros((P * g.n_angles * g.n_radial, nv))
    row = 0
    for p in range(P):
        for a in range(g.n_angles):
            for b in range(g.n_radial):
                for iz in range(nz):
                    for iy in range(g.ny):
                        for ix in range(g.nx):
                            A[row, (iz * g.ny + iy) * g.nx + ix] = orc.chord_clip(g, p, a, b, ix, iy, iz)
                row += 1
    return A


def base_params(orc, **kw):
    p = dict(mode="BSREM", beta=0.0, gamma_R=2.0, eps=1e-12, t_clip=1e-4, U=1e9, lambda0=1.0,
             a=1e-9, rho=3.0, delta1=2.0, delta2=2.0, nu1=0.5, nu2=2.0, J0=3, J1=1000)
    p.update(kw)
    return orc.params(p)


# ---------------------------------------------------------------- fidelity F

def test_fidelity_gradient_fd_and_identity(orc):
    g = g2(orc)
    rng = np.random.default_rng(0)
    f = rng.uniform(0.5, 2.0, 64)
    A = dense_A(orc, g)
    y = rng.poisson(A @ f + 1.0).astype(float)
    r = np.full(y.size, 1.0)
    q = orc.forward(g, f).reshape(-1)
    grad = orc.back(g, 1.0 - y / (q + r)).reshape(-1)        # A^T(1 - g/(Af + gamma))
    h = 1e-6
    for j in (0, 9, 27, 63):
        e = np.zeros(64); e[j] = h
        fd = (orc.fidelity(g, f + e, y, r) - orc.fidelity(g, f - e, y, r)) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-7 * max(1.0, abs(grad[j])) + 1e-6
    assert math.isclose(grad @ f, q.sum() - (y * q / (q + r)).sum(), rel_tol=1e-12)


# ---------------------------------------------------------------- RDP

@pytest.mark.parametrize("dim", [2, 3])
def test_rdp_euler_identity_and_fd(orc, dim):
    g = g2(orc) if dim == 2 else g3(orc)
    nv = orc.n_voxels(g)
    rng = np.random.default_rng(1)
    f = rng.uniform(0.0, 3.0, nv)
    f[::7] = 0.0
    gR, eps = 2.0, 1e-3
    R = orc.rdp_value(g, f, gR, eps)
    grad = orc.rdp_grad(g, f, gR, eps).reshape(-1)
    # each pair term is 1-homogeneous in u = f + eps/2  =>  sum_j u_j dR/df_j = R
    assert math.isclose(((f + eps / 2) * grad).sum(), R, rel_tol=1e-12)
    h = 1e-6
    for j in rng.choice(np.flatnonzero(f > 0.1), 6, replace=False):
        e = np.zeros(nv); e[j] = h
        fd = (orc.rdp_value(g, f + e, gR, eps) - orc.rdp_value(g, f - e, gR, eps)) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-6 * max(1.0, abs(grad[j]))


def test_rdp_constant_image(orc):
    g = g3(orc)
    f = np.full(orc.n_voxels(g), 2.5)
    assert orc.rdp_value(g, f, 2.0, 1e-12) == 0.0
    assert not orc.rdp_grad(g, f, 2.0, 1e-12).any()


def test_rdp_neighbourhood_counts_ordered_pairs(orc):
    """8 in-image neighbours in 2D: a single hot pixel in the interior gives
    8 pair terms counted twice (j->k and k->j)."""
    g = g2(orc, n=5)
    f = np.zeros(25); f[12] = 1.0
    eps, gR = 1e-12, 0.0
    # each of the 16 ordered pairs contributes 1^2 / (1 + eps)
    assert math.isclose(orc.rdp_value(g, f, gR, eps), 16 / (1 + eps), rel_tol=1e-14)
    f2 = np.zeros(25); f2[0] = 1.0              # corner: 3 neighbours
    assert math.isclose(orc.rdp_value(g, f2, gR, eps), 6 / (1 + eps), rel_tol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_rdp_hessian(orc, dim):
    g = g2(orc) if dim == 2 else g3(orc)
    nv = orc.n_voxels(g)
    rng = np.random.default_rng(2)
    f = rng.uniform(0.2, 3.0, nv)
    gR, eps = 2.0, 1e-2
    # Hessian_R: null vector 2f + eps
    Hn = orc.rdp_hess_apply(g, f, gR, eps, 2 * f + eps).reshape(-1)
    scale = np.abs(orc.rdp_hess_apply(g, f, gR, eps, np.ones(nv))).max() * (2 * f + eps).max()
    assert np.abs(Hn).max() <= 1e-13 * scale
    # Hessian-vector product equals the finite difference of the gradient
    x = rng.normal(0, 1, nv)
    h = 1e-6
    fd = (orc.rdp_grad(g, f + h * x, gR, eps) - orc.rdp_grad(g, f - h * x, gR, eps)).reshape(-1) / (2 * h)
    Hx = orc.rdp_hess_apply(g, f, gR, eps, x).reshape(-1)
    assert np.abs(fd - Hx).max() <= 1e-6 * np.abs(Hx).max()
    assert x @ Hx >= 0.0


def test_grad_mag_matches_numpy_gradient(orc):
    """numpy.gradient with edge_order=1 is the Matlab gradient (central inside,
    one-sided at the edges, unit spacing)."""
    rng = np.random.default_rng(3)
    g = g2(orc, n=9)
    f = rng.uniform(0, 1, (9, 9))
    gy, gx = np.gradient(f, edge_order=1)
    assert np.allclose(orc.grad_mag(g, f), np.hypot(gx, gy), rtol=1e-15, atol=1e-15)
    g = g3(orc, n=6, nz=4)
    f = rng.uniform(0, 1, (4, 6, 6))
    gz, gy, gx = np.gradient(f, edge_order=1)
    assert np.allclose(orc.grad_mag(g, f), np.sqrt(gx ** 2 + gy ** 2 + gz ** 2), rtol=1e-15, atol=1e-15)


# ---------------------------------------------------------------- scalars

def test_nesterov_sequence_limits(orc):
    """Proof of thm:SpecificSDPs: t_{k,i} > (kM+i)/2, alpha -> 2,
    k (2 - alpha_{k,i}) -> 3/M; alpha_{0,1} = 1."""
    M = 24
    t = 1.0
    alphas = []
    J = 0
    K = 100000
    for k in range(K + 1):
        for i in range(1, M + 1):
            J += 1
            tn = orc.nesterov_next(t)
            if J > 1:
                assert t > J / 2.0
            alpha = 1.0 + (t - 1.0) / tn
            if k == 0 and i == 1:
                assert alpha == 1.0
            # identity 2 - alpha = 1/(2 t' (sqrt(1+4t^2) + 2t)) + 3/(2 t')  (printed with 4t)
            ident = 1.0 / (2 * tn * (math.sqrt(1 + 4 * t * t) + 2 * t)) + 3.0 / (2 * tn)
            assert math.isclose(2.0 - alpha, ident, rel_tol=1e-9, abs_tol=1e-15)
            if k == K:
                alphas.append(alpha)
            t = tn
    for a in alphas:
        assert abs(K * (2.0 - a) - 3.0 / M) <= 2e-4


def test_km_sequence_limits(orc):
    p = base_params(orc, rho=2.2, delta1=0.1, delta2=1.6)
    M = 28
    assert math.isclose(orc.km_alpha(p, 1), 1.6 / 0.1, rel_tol=1e-15)    # alpha_{0,1} = delta2/delta1
    K = 10 ** 6
    for i in (1, 7, 28):
        a = orc.km_alpha(p, K * M + i)
        assert abs(K * (2.2 - a) - (2.2 * 0.1 - 1.6) / M) <= 1e-4


def test_relaxation_conditions(orc):
    """condition (iv): sum lambda_k diverges, sum lambda_k^2 converges."""
    p = base_params(orc, lambda0=1.6, a=0.25)
    lam = np.array([orc.relax(p, k) for k in range(200000)])
    assert lam[0] == 1.6
    s1, s2 = np.cumsum(lam), np.cumsum(lam ** 2)
    assert s1[-1] > 1.8 * s1[len(s1) // 200]          # logarithmic growth
    K = len(s2)
    # tail of sum lambda^2 bounded by the integral lambda0^2 / (a^2 k) -> 0
    assert s2[-1] - s2[K // 2] <= 1.6 ** 2 / 0.25 ** 2 * (2.0 / K)


# ---------------------------------------------------------------- nu

def test_nu_schedule_and_bounds(orc):
    g = g2(orc, n=10, na=12, nr=15, M=3)
    rng = np.random.default_rng(4)
    A = dense_A(orc, g)
    ftrue = rng.uniform(0.5, 3.0, 100)
    y = rng.poisson(A @ ftrue + 0.5).astype(float)
    r = np.full(y.size, 0.5)
    f0 = np.ones(100)
    p = base_params(orc, mode="P2", beta=0.1, nu1=0.7, nu2=1.9, J0=2, J1=7, a=0.3)
    rec = orc.Recon(g, p, f0, y, r)
    nus = [rec.subiteration(want_nu=True) for _ in range(12)]
    assert np.all(nus[0] == 1.0) and np.all(nus[1] == 1.0)            # J <= J0
    # constant image at J = 1? no: J = 3 is the first adaptive one; f is not constant any more
    for J in range(3, 8):
        nu = nus[J - 1]
        assert nu.min() >= 0.7 and nu.max() <= 1.9
        assert not np.all(nu == nu[0])
    for J in range(8, 13):
        assert np.array_equal(nus[J - 1], nus[6])                      # frozen at J1 = 7


def test_nu_of_constant_image(orc):
    """constant f => grad = 0 => mu = 0.01 everywhere => nu = clamp(1, nu1, nu2)."""
    g = g2(orc, n=6, na=6, nr=9, M=2)
    y = np.ones(orc.n_bins(g)); r = np.ones_like(y)
    for lo, hi, expect in ((0.6, 1.25, 1.0), (1.3, 2.1, 1.3), (0.2, 0.8, 0.8)):
        p = base_params(orc, mode="P2", nu1=lo, nu2=hi, J0=0, J1=10)
        rec = orc.Recon(g, p, np.full(36, 2.0), y, r)
        nu = rec.subiteration(want_nu=True)
        assert np.allclose(nu, expect, rtol=1e-14, atol=0)


# ---------------------------------------------------------------- one full step

def test_mlem_special_case(orc):
    """M = 1, beta = 0, lambda = 1, alpha = nu = 1, U huge: one BSREM step is
    exactly the MLEM update f+ = f A^T(g/(Af+gamma)) / A^T 1 (Shepp-Vardi)."""
    g = g2(orc, n=8, na=10, nr=13, M=1)
    rng = np.random.default_rng(5)
    A = dense_A(orc, g)
    f = rng.uniform(0.5, 2.0, 64)
    y = rng.poisson(A @ f * 3 + 1.0).astype(float)
    r = rng.uniform(0.5, 1.5, y.size)
    p = base_params(orc)
    rec = orc.Recon(g, p, f, y, r)
    rec.subiteration()
    s = A.sum(axis=0)
    q = A @ f
    mlem = f * (A.T @ (y / (q + r))) / s
    assert np.abs(rec.f - mlem).max() <= 1e-13 * mlem.max()
    # count identity of the MLEM step
    assert math.isclose(s @ rec.f, (y * q / (q + r)).sum(), rel_tol=1e-13)


def test_iterates_stay_positive_and_in_box(orc):
    g = g2(orc, n=10, na=12, nr=15, M=4)
    rng = np.random.default_rng(6)
    A = dense_A(orc, g)
    ftrue = np.zeros(100); ftrue[rng.choice(100, 40, replace=False)] = rng.uniform(1, 5, 40)
    y = rng.poisson(A @ ftrue + 0.2).astype(float)
    r = np.full(y.size, 0.2)
    U = 3.0
    for mode in ("BSREM", "M1", "M2", "P1", "P2"):
        p = base_params(orc, mode=mode, beta=0.05, U=U, lambda0=1.0, a=0.2, rho=4.0,
                        delta1=2.0, delta2=2.0, nu1=0.8, nu2=2.2, J0=3, J1=30)
        rec = orc.Recon(g, p, np.ones(100), y, r)
        for _ in range(60):
            rec.subiteration()
            assert rec.f.min() > 0.0 and rec.f.max() < U


# ---------------------------------------------------------------- convergence

def _tiny_problem(orc, seed, n=6, M=3, na=9, nr=11, U=None):
    g = g2(orc, n=n, na=na, nr=nr, M=M, v=2.0)
    rng = np.random.default_rng(seed)
    A = dense_A(orc, g)
    ftrue = rng.uniform(0.5, 4.0, n * n)
    y = rng.poisson(5 * A @ ftrue + 1.0).astype(float)
    r = np.full(y.size, 1.0)
    return g, A, y, r


def _minimiser(A, y, r, beta, gR, eps, orc, g, U):
    """Independent minimiser of Phi over [0, U]^q: scipy L-BFGS-B on the
    closed forms of F (eq:FidelityTerm) with the oracle's R."""
    from scipy.optimize import minimize
    nv = A.shape[1]

    def fun(f):
        q = A @ f
        F = q.sum() - (y * np.log(q + r)).sum()
        Rv = orc.rdp_value(g, f, gR, eps)
        gradF = A.T @ (1 - y / (q + r))
        return F + beta * Rv, gradF + beta * orc.rdp_grad(g, f, gR, eps).reshape(-1)

    res = minimize(fun, np.ones(nv), jac=True, method="L-BFGS-B", bounds=[(0, U)] * nv,
                   options=dict(maxiter=20000, ftol=1e-16, gtol=1e-12, maxcor=50))
    return res.x


@pytest.mark.parametrize("mode", ["BSREM", "M1", "M2", "P1", "P2"])
def test_converges_to_independent_minimiser(orc, mode):
    """thm:SpecificSDPs on a tiny problem: every variant approaches the unique
    minimiser of Phi over B; KKT residual and distance shrink; Phi settles."""
    g, A, y, r = _tiny_problem(orc, 7)
    beta, gR, eps = 0.5, 2.0, 1e-12
    U = 1e4
    fstar = _minimiser(A, y, r, beta, gR, eps, orc, g, U)
    P = dict(BSREM=dict(a=0.05), M1=dict(a=0.05), M2=dict(a=0.05, rho=2.0, delta1=1.0, delta2=1.0),
             P1=dict(a=0.05, nu1=0.8, nu2=1.6), P2=dict(a=0.05, rho=2.0, delta1=1.0, delta2=1.0,
                                                        nu1=0.8, nu2=1.6))[mode]
    p = base_params(orc, mode=mode, beta=beta, U=U, lambda0=0.5, J0=3, J1=150, **P)
    f = np.ones(A.shape[1])
    errs = []
    for chunk in (200, 800, 3000):
        f, obj = orc.reconstruct(g, p, f, y, r, chunk)
        p.J0, p.J1 = -1, -1          # schedule already past J1 after the first chunk
        errs.append(np.linalg.norm(f.reshape(-1) - fstar) / np.linalg.norm(fstar))
    assert errs[2] < errs[0]
    assert errs[2] < 2e-3, errs


def test_converges_to_upper_bound_branch(orc):
    """U below the unconstrained optimum: the minimiser sits on f_j = U and the
    (U - f)/p branch of eq:preconditioner lets the iterates approach U itself,
    not U - t.  t is made large so that the difference is visible."""
    g, A, y, r = _tiny_problem(orc, 8, M=1)
    beta, gR, eps = 0.2, 2.0, 1e-12
    free = _minimiser(A, y, r, beta, gR, eps, orc, g, 1e6)
    U = 0.7 * free.max()
    fstar = _minimiser(A, y, r, beta, gR, eps, orc, g, U)
    assert (fstar >= U - 1e-9).sum() >= 1
    p = base_params(orc, mode="BSREM", beta=beta, U=U, t_clip=0.02 * U, lambda0=0.5, a=0.01)
    f, _ = orc.reconstruct(g, p, np.ones(A.shape[1]), y, r, 3000)
    f = f.reshape(-1)
    at = fstar >= U - 1e-9
    assert np.all(f[at] > U - 0.005 * U)
    assert np.linalg.norm(f - fstar) / np.linalg.norm(fstar) < 2e-3


def test_objective_decreases_to_minimum(orc):
    g, A, y, r = _tiny_problem(orc, 9, M=3)
    beta, gR, eps = 0.5, 2.0, 1e-12
    fstar = _minimiser(A, y, r, beta, gR, eps, orc, g, 1e4)
    q = A @ fstar
    phistar = q.sum() - (y * np.log(q + r)).sum() + beta * orc.rdp_value(g, fstar, gR, eps)
    p = base_params(orc, mode="P2", beta=beta, U=1e4, lambda0=0.5, a=0.05, rho=2.0, delta1=1.0,
                    delta2=1.0, nu1=0.8, nu2=1.6, J0=3, J1=150)
    f, obj = orc.reconstruct(g, p, np.ones(36), y, r, 2000)
    assert obj[-1] >= phistar - 1e-9 * abs(phistar)
    assert abs(obj[-1] - phistar) <= 1e-8 * abs(phistar)
    assert np.all(np.diff(obj[200:]) <= 1e-9 * abs(phistar))


# ---------------------------------------------------------------- default U


@pytest.mark.parametrize("dim", [2, 3])
def test_default_U_by_hand(orc, dim):
    """The default box bound (the paper only proves U exists, eq:BoundedSet)
    is 1e3 max(max f0, (sum y - sum r)_+ / sum_j (A^T 1)_j), the sensitivity
    summed over every ray, computed here from the brute-force matrix: each
    branch of the max, and the clipped count excess."""
    g = g2(orc, n=6, na=8, nr=9, M=4) if dim == 2 else g3(orc, n=4, nz=3, na=4, nr=7, M=2)
    A = dense_A(orc, g)
    s_tot = A.sum()                      # sum_j (A^T 1)_j over every ray of every subset
    rng = np.random.default_rng(17)
    nb, nv = A.shape
    r = rng.uniform(0.5, 1.5, nb)
    # count excess dominates: (sum y - sum r) / sum s exceeds max f0
    f0 = rng.uniform(0.1, 0.5, nv)
    y = rng.uniform(20.0, 40.0, nb)
    chat = (y.sum() - r.sum()) / s_tot
    assert chat > f0.max()
    assert abs(orc.default_U(g, f0, y, r) - 1e3 * chat) <= 1e-12 * 1e3 * chat
    # max f0 dominates
    f0b = f0.copy()
    f0b[3] = 10.0 * chat
    assert orc.default_U(g, f0b, y, r) == 1e3 * f0b.max()
    # fewer counts than background: the excess is clipped at 0
    y0 = 0.1 * r
    assert orc.default_U(g, f0, y0, r) == 1e3 * f0.max()
