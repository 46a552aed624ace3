"""The convergence comparison of Sec. IV-B on a small case, run through the
C ABI: the trajectories are finite, the objective of every algorithm falls,
BSREM approaches f_inf (its NRMSD falls), and the reach table is
consistent with the trajectories."""
import math

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_convergence_small_case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_07886_amd import convergence
    print("[gpu-convergence] ellipse 64^2, M=12, BSREM/P1/P2, 8 iterations, f_inf 300", flush=True)
    case = convergence.run_case("ellipse", n=64, M=12, count_level="high", modes=("BSREM", "P1", "P2"),
                                n_iter=8, ref_iter=300, seed=5, targets=(2, 4))
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
