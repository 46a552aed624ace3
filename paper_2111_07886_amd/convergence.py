"""Convergence comparison of the preconditioners on the paper's 2D simulation
set-up (Sec. IV-A/IV-B, Figs. 3-6), run on the GPU path.

The data follow the paper's model: the phantom is projected through the same
system matrix used to reconstruct (Sec. IV-A) -- with ``full_model`` the
paper's own (32 sub-rays per bin, Gaussian PSF of FWHM 6.59 mm, water
attenuation 0.096 / cm over the phantom's support), otherwise one line per
bin --, trues are scaled to the total count TC, scatter is a smoothed
projection with SF = 0.25, randoms are uniform with RF = 0.25, and the counts
are Poisson.  Phantoms: the uniform phantom of Fig. 1b (synth.phantoms), and
a seeded ellipse phantom with hot lesions standing in for the brain phantom,
which is not available.

Figures of merit (Sec. IV-A): the objective Phi(f^k) after every iteration and
the NRMSD sqrt(sum_ROI (f^k - f_inf)^2) / sqrt(sum_ROI f_inf^2), with f_inf the
image after 1000 iterations of BSREM with 24 subsets.  From them: the
iterations each algorithm needs to reach the objective that BSREM reaches in K
iterations (the paper's "same objective function value" comparison), and the
NRMSD per ROI after a fixed number of iterations.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import Geometry, State

GEOM_2D = dict(n_angles=288, n_radial=367, fov_mm=300.0)   # Sec. IV-A: 288 angles, 300 mm FOV


def nrmsd(f, f_inf, mask=None):
    """ROI-based NRMSD of Sec. IV-A (whole image when mask is None)."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(f_inf, dtype=np.float64)
    if mask is not None:
        f, g = f[mask], g[mask]
    return float(np.sqrt(np.sum((f - g) ** 2)) / np.sqrt(np.sum(g ** 2)))


def iterations_to_reach(phi, target):
    """First iteration (1-based) whose objective is <= target, or None."""
    for k, v in enumerate(phi, start=1):
        if v <= target:
            return k
    return None


def make_data(phantom: str, n: int, M: int, TC: float, seed: int):
    """Geometry descriptor, phantom activity, counts and background."""
    from synth import configs, phantoms
    n_r = GEOM_2D["n_radial"] if n == 256 else 2 * int(math.ceil(n / math.sqrt(2))) + 3
    desc = configs.desc_2d(n, GEOM_2D["n_angles"], n_r, GEOM_2D["fov_mm"] / n, M)
    rng = np.random.default_rng(seed)
    if phantom == "uniform":
        img, rois = phantoms.uniform_phantom_2d(n)
    else:
        w = phantoms.make_2d(desc, seed=seed, n_ell=12, counts=1e6, bg_frac=0.0, hot_lesions=4)
        img, rois = w.f_true / w.f_true.max(), {"body": w.f_true > 0}
    return desc, img, rois, rng


def full_model_geometry(desc, img):
    """The paper's system model for a 2D descriptor: sub-rays, PSF, and the
    attenuation factors of water over the phantom's support."""
    from synth import configs
    d = dict(desc, n_subrays=configs.N_SUBRAYS, psf_fwhm=configs.PSF_FWHM_MM)
    mu = torch.tensor(np.where(np.asarray(img) > 0, configs.MU_WATER_PER_MM, 0.0), dtype=torch.float32,
                      device="cuda")
    g0 = Geometry(d)
    att = g0.attenuation_factors(mu).cpu().numpy()
    g0.close()
    return d, att


def run_case(phantom="uniform", n=256, M=24, count_level="high", modes=("BSREM", "P1", "P2"), n_iter=100,
             ref_iter=1000, seed=21, targets=(10, 20, 50), full_model=False, data=None, keep_images=False):
    """One data set, the given algorithms for n_iter iterations each, against
    f_inf = BSREM(24) after ref_iter iterations.

    data: None (simulate: the phantom projected by this geometry, then the
    counts model of simulate_sdp_counts), or a dict with the counts ``y``,
    the background ``r`` (numpy, natural layout) and the bound ``U`` to
    reconstruct instead.  keep_images: the result also holds ``f_inf`` and
    each mode's final image (numpy) under ``images``."""
    from synth import configs
    TC = configs.TC_HIGH if count_level == "high" else configs.TC_LOW
    desc, img, rois, rng = make_data(phantom, n, M, TC, seed)
    att = None
    if full_model:
        desc, att = full_model_geometry(desc, img)
    G = Geometry(desc, att=att)
    dev = torch.device("cuda")
    if data is None:
        Af = G.forward(torch.tensor(img, dtype=torch.float32, device=dev)).cpu().double().numpy()
        from synth import phantoms
        y_np, r_np, scale = phantoms.simulate_sdp_counts(Af, TC, rng, configs.SF, configs.RF)
    else:
        y_np, r_np = data["y"], data["r"]
    y = torch.tensor(np.asarray(y_np).reshape(G.sino_shape), dtype=torch.float32, device=dev)
    r = torch.tensor(np.asarray(r_np).reshape(G.sino_shape), dtype=torch.float32, device=dev)
    ones = torch.ones(G.img_shape, dtype=torch.float32, device=dev)
    U = G.default_U(ones, y, r) if data is None else float(data["U"])

    def params(mode, m):
        if phantom == "uniform" and m == 24 and mode in ("BSREM", "P1", "P2") and count_level == "high":
            p = configs.params_2d_uniform(mode, U=U)
        else:
            p = configs.params_2d(m, 1e7 if count_level == "high" else 1e5, mode=mode, U=U)
        return p

    # f_inf: BSREM with 24 subsets (same data; its own 24-subset geometry)
    G24 = G if M == 24 else Geometry(dict(desc, n_subsets=24), att=att)
    f_inf = ones.clone()
    st = State(G24, params("BSREM", 24))
    st.run(f_inf, y, r, ref_iter)
    torch.cuda.synchronize()
    f_inf_np = f_inf.cpu().double().numpy()
    phi_inf = G24.objective(params("BSREM", 24), f_inf, y, r)
    st.close()

    out = {"phantom": phantom, "n": n, "subsets": M, "counts": count_level, "TC": TC, "U": U,
           "system_model": "32 sub-rays, PSF 6.59 mm, attenuation" if full_model else "one line per bin",
           "f_inf_iterations": ref_iter, "phi_inf": phi_inf, "modes": {}}
    for mode in modes:
        p = params(mode, M)
        # time per iteration (no objective evaluations)
        f = ones.clone()
        st = State(G, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.run(f, y, r, n_iter)
        torch.cuda.synchronize()
        ms_it = 1e3 * (time.perf_counter() - t0) / n_iter
        st.close()
        # trajectory: objective and NRMSD after every iteration
        f = ones.clone()
        st = State(G, p)
        phi, nr = [], {"global": []}
        for k in rois:
            nr[k] = []
        for _ in range(n_iter):
            phi.append(st.run(f, y, r, 1, want_objective=True)[0])
            fh = f.cpu().double().numpy()
            nr["global"].append(nrmsd(fh, f_inf_np))
            for k, m in rois.items():
                nr[k].append(nrmsd(fh, f_inf_np, m))
        st.close()
        out["modes"][mode] = {"params": p, "ms_per_iteration": ms_it, "objective": phi, "nrmsd": nr}
        if keep_images:
            out.setdefault("images", {"f_inf": f_inf_np})[mode] = f.cpu().double().numpy()
    # iterations to reach BSREM's objective after K iterations
    if "BSREM" in out["modes"]:
        ref = out["modes"]["BSREM"]["objective"]
        reach = {}
        for K in targets:
            if K <= len(ref):
                reach[str(K)] = {mode: iterations_to_reach(d["objective"], ref[K - 1])
                                 for mode, d in out["modes"].items()}
        out["iterations_to_reach_bsrem"] = reach
    return out


def summary(case):
    """Compact view: per mode, iterations to reach BSREM(K)'s objective, the
    speed-up K / iterations (and the same in elapsed GPU time), and the final
    NRMSD."""
    s = {}
    reach = case.get("iterations_to_reach_bsrem", {})
    for mode, d in case["modes"].items():
        row = {"ms_per_iteration": round(d["ms_per_iteration"], 3),
               "nrmsd_global_final": round(d["nrmsd"]["global"][-1], 5)}
        ms_ref = case["modes"]["BSREM"]["ms_per_iteration"] if "BSREM" in case["modes"] else None
        for K, per in reach.items():
            k = per.get(mode)
            row[f"iters_to_bsrem{K}"] = k
            row[f"speedup_at_bsrem{K}"] = round(int(K) / k, 3) if k else None
            # elapsed-time version (the paper's figures plot the objective against time)
            row[f"time_speedup_at_bsrem{K}"] = \
                round(int(K) * ms_ref / (k * d["ms_per_iteration"]), 3) if k and ms_ref else None
        for roi, v in d["nrmsd"].items():
            if roi != "global":
                row[f"nrmsd_{roi}_final"] = round(v[-1], 5)
        s[mode] = row
    return s


def main(argv=None):
    import argparse
    import json
    import os
    ap = argparse.ArgumentParser(description="convergence comparison of BSREM and the SDP preconditioners (2D)")
    ap.add_argument("--phantom", default="uniform", choices=["uniform", "ellipse"])
    ap.add_argument("--subsets", type=int, default=24)
    ap.add_argument("--counts", default="high", choices=["high", "low"])
    ap.add_argument("--modes", default="BSREM,P1,P2")
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--ref-iters", type=int, default=1000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seed", type=int, default=21)
    ap.add_argument("--out", default=None, help="write the full trajectories as JSON here")
    ap.add_argument("--full-model", action="store_true",
                    help="the paper's system model: 32 sub-rays per bin, PSF, water attenuation")
    a = ap.parse_args(argv)
    case = run_case(a.phantom, a.n, a.subsets, a.counts, tuple(a.modes.split(",")), a.iters, a.ref_iters, a.seed,
                    full_model=a.full_model)
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as fh:
            json.dump(case, fh)
    head = {k: case[k] for k in ("phantom", "n", "subsets", "counts", "TC", "U", "system_model", "f_inf_iterations",
                                 "phi_inf")}
    print(json.dumps({"case": head, "summary": summary(case)}), flush=True)


if __name__ == "__main__":
    main()
