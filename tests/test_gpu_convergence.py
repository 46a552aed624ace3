"""The convergence comparison of Sec. IV-B (Figs. 3-6) on a small case, run
through the C ABI: the trajectories are finite, the objective of every
algorithm falls, BSREM approaches f_inf (its NRMSD falls), and the reach
table is consistent with the trajectories.  The driver's outputs are also
compared with the FP64 oracle run on the same data: the objective after
every iteration, f_inf and each algorithm's final image, the NRMSD per ROI
and the iterations-to-reach table."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASE = dict(phantom="ellipse", n=64, M=12, count_level="high", modes=("BSREM", "P1", "P2"), n_iter=8,
            ref_iter=300, seed=5, targets=(2, 4))


def test_convergence_small_case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_07886_amd import convergence
    print("[gpu-convergence] ellipse 64^2, M=12, BSREM/P1/P2, 8 iterations, f_inf 300", flush=True)
    case = convergence.run_case(**CASE)
    assert math.isfinite(case["phi_inf"])
    for mode, d in case["modes"].items():
        phi = d["objective"]
        assert len(phi) == 8 and all(math.isfinite(v) for v in phi), mode
        assert phi[-1] < phi[0], mode
        assert phi[-1] >= case["phi_inf"] - 1e-6 * abs(case["phi_inf"]), mode
        g = d["nrmsd"]["global"]
        assert all(math.isfinite(v) for v in g), mode
        if mode == "BSREM":
            assert g[-1] < g[0]
        assert d["ms_per_iteration"] > 0
    for K, per in case["iterations_to_reach_bsrem"].items():
        assert per["BSREM"] <= int(K)
        for mode, k in per.items():
            if k is not None:
                target = case["modes"]["BSREM"]["objective"][int(K) - 1]
                assert case["modes"][mode]["objective"][k - 1] <= target
    s = convergence.summary(case)
    assert set(s) == {"BSREM", "P1", "P2"}


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def test_convergence_against_oracle(orc):
    """The same small case on data built by the oracle (its projection of
    the phantom, the counts model, its default U), against the oracle's own
    trajectories on those data.  Tolerances as for the reconstruction
    trajectories: the stated 1e-6 (objective) and 1e-4 (image), or 5x the
    method's own FP32-noise spread where that is larger; an image whose
    tolerance that rule widens beyond 1e-2 (P2 here: spread 0.11) is recorded,
    not asserted, and its NRMSD is not compared."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_07886_amd import convergence
    from parity_record import record
    from synth import configs, phantoms
    from test_gpu_parity import IMG_PARITY_LIMIT, TOL_IMG, TOL_OBJ, intrinsic_spread, rel
    desc, img, rois, rng = convergence.make_data(CASE["phantom"], CASE["n"], CASE["M"], configs.TC_HIGH,
                                                 CASE["seed"])
    g = orc.geom(desc)
    Af = orc.forward(g, img)
    y, r, _ = phantoms.simulate_sdp_counts(Af, configs.TC_HIGH, rng, configs.SF, configs.RF)
    y, r = f32(y), f32(r)
    ones = np.ones(orc.img_shape(g))
    U = orc.default_U(g, ones, y, r)
    print("[gpu-convergence] driver on oracle-built data", flush=True)
    case = convergence.run_case(**CASE, data=dict(y=y, r=r, U=U), keep_images=True)
    # f_inf = BSREM(24) after ref_iter iterations, and its objective
    p24 = configs.params_2d(24, 1e7, mode="BSREM", U=U)
    g24 = orc.geom(dict(desc, n_subsets=24))
    finf_o, _ = orc.reconstruct(g24, orc.params(p24), ones, y, r, CASE["ref_iter"], want_obj=False)
    phi_inf_o = orc.objective(g24, finf_o, y, r, p24["beta"], p24["gamma_R"], p24["eps"])
    e_inf = rel(case["images"]["f_inf"], finf_o)
    eo_inf = abs(case["phi_inf"] - phi_inf_o) / abs(phi_inf_o)
    print(f"[gpu-convergence] f_inf rel-L2 {e_inf:.2e}, phi_inf rel {eo_inf:.2e}", flush=True)
    record("convergence", "f_inf BSREM(24) 300 iterations", image_rel_l2=e_inf, objective_rel=eo_inf)
    assert e_inf <= TOL_IMG and eo_inf <= TOL_OBJ
    traj_o = {}
    for mode, d in case["modes"].items():
        p = d["params"]
        fo, objo = orc.reconstruct(g, orc.params(p), ones, y, r, CASE["n_iter"])
        traj_o[mode] = objo[1:]
        w = phantoms.Workload(desc=desc, f_true=img, y=y, r=r, f0=ones, U=U)
        # the objective's spread after every iteration (the early iterations
        # of the relaxed modes are the most sensitive)
        s_img, s_obj = intrinsic_spread(orc, w, p, CASE["n_iter"], per_iteration=True)
        tol_img = max(TOL_IMG, 5 * s_img)
        tol_obj = [max(TOL_OBJ, 5 * v) for v in s_obj]
        eos = [abs(a - b) / abs(b) for a, b in zip(d["objective"], objo[1:])]
        e = rel(case["images"][mode], fo)
        worst = max(range(len(eos)), key=lambda k: eos[k] / tol_obj[k])
        print(f"[gpu-convergence] {mode}: objective trace, worst iteration {worst + 1}: rel {eos[worst]:.2e} "
              f"(tol {tol_obj[worst]:.1e}); image {e:.2e} (tol {tol_img:.1e})", flush=True)
        img_asserted = tol_img <= IMG_PARITY_LIMIT
        record("convergence", f"ellipse 64^2 M=12 {mode}", n_iter=CASE["n_iter"], objective_trace_rel=eos,
               objective_tol=tol_obj, objective_spread=s_obj, image_rel_l2=e, image_tol=tol_img,
               image_spread=s_img, image_asserted=img_asserted)
        assert all(a <= b for a, b in zip(eos, tol_obj)), (mode, eos, tol_obj)
        if not img_asserted:
            continue            # the trajectory itself is that sensitive: objective only
        assert e <= tol_img, mode
        # NRMSD per ROI of the final iterate against f_inf, from the oracle's images
        for roi, vals in d["nrmsd"].items():
            m = None if roi == "global" else rois[roi]
            no = convergence.nrmsd(fo, finf_o, m)
            assert abs(vals[-1] - no) <= 1e-3 * max(no, 1e-3), (mode, roi, vals[-1], no)
    # iterations to reach BSREM's objective after K iterations: the oracle's
    # table, except where the oracle's own objective lies within tolerance of
    # the target (a decision FP32 may take either way)
    for K, per in case["iterations_to_reach_bsrem"].items():
        target = traj_o["BSREM"][int(K) - 1]
        for mode, k in per.items():
            ko = convergence.iterations_to_reach(traj_o[mode], target)
            near = any(abs(v - target) <= 5 * TOL_OBJ * abs(target) for v in traj_o[mode])
            assert k == ko or near, (K, mode, k, ko)
