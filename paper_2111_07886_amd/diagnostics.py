"""Gradient-consistency diagnostic of Sec. IV-B (Fig. 2), on the GPU path.

Along an SDP-BSREM run, after subiteration (k, i) has produced f^{k,i}, the
subset gradient h^{k,i} = grad Phi_i(f^{k,i}) is taken; theta_{k,i} is the
angle between h^{k,i-1} and h^{k,i} restricted to the smooth area of f^{k,i}
(grad(f)_j < 0.01 mean f) and theta~_{k,i} the same on the variable area
(grad(f)_j > 0.2 mean f), with h^{k,0} = grad Phi_M(f^{k,0}) (Phi_0 := Phi_M).
theta_k and theta~_k are the means over the M subiterations of iteration k.
"""
from __future__ import annotations

import math

import torch

from . import Geometry, State


def gradient_consistency(geom: Geometry, params: dict, f, y, r, n_iter: int, smooth_frac=0.01, var_frac=0.2,
                         state: State | None = None):
    """Advance f (in place) by n_iter iterations and return a dict with the
    per-subiteration angles (radians) on both areas, the area sizes and the
    per-iteration means.  ``state`` (optional) must sit at the start of an
    iteration; a fresh one is made from ``params`` otherwise."""
    M = geom.desc["n_subsets"]
    own = state is None
    st = State(geom, params) if own else state
    if st.position()[1] != 1:
        raise ValueError("the state must be at the start of an iteration")
    h_prev = geom.subset_gradient(params, f, y, r, M)
    h_cur = torch.empty_like(h_prev)
    th, tt, ns, nv = [], [], [], []
    for _ in range(n_iter):
        rs, rv, cs, cv = [], [], [], []
        for i in range(1, M + 1):
            st.subiteration(f, y, r)
            geom.subset_gradient(params, f, y, r, i, out=h_cur)
            a_s, a_v, c_s, c_v = geom.gradient_angles(h_prev, h_cur, f, smooth_frac, var_frac)
            rs.append(a_s)
            rv.append(a_v)
            cs.append(c_s)
            cv.append(c_v)
            h_prev, h_cur = h_cur, h_prev
        th.append(rs)
        tt.append(rv)
        ns.append(cs)
        nv.append(cv)
    if own:
        st.close()

    def mean(row):
        v = [x for x in row if not math.isnan(x)]
        return sum(v) / len(v) if v else math.nan

    return {"theta": th, "theta_tilde": tt, "n_smooth": ns, "n_variable": nv,
            "theta_mean": [mean(r) for r in th], "theta_tilde_mean": [mean(r) for r in tt]}


def main(argv=None):
    """Fig. 2 set-up on the synthetic stand-ins: P1 and P2 with 24 subsets on
    high-count data of the 256^2 ellipse phantom (the brain phantom is not
    available); prints the per-iteration mean angles in degrees."""
    import argparse
    import json
    import numpy as np
    from synth import configs
    from .convergence import make_data
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--phantom", default="ellipse", choices=["uniform", "ellipse"])
    ap.add_argument("--modes", default="P1,P2")
    ap.add_argument("--subsets", type=int, default=24)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--seed", type=int, default=21)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    from synth import phantoms
    desc, img, _, rng = make_data(a.phantom, 256, a.subsets, configs.TC_HIGH, a.seed)
    G = Geometry(desc)
    Af = G.forward(torch.tensor(img, dtype=torch.float32, device="cuda")).cpu().double().numpy()
    y_np, r_np, _ = phantoms.simulate_sdp_counts(Af, configs.TC_HIGH, rng, configs.SF, configs.RF)
    y = torch.tensor(y_np, dtype=torch.float32, device="cuda")
    r = torch.tensor(r_np, dtype=torch.float32, device="cuda")
    res = {}
    for mode in a.modes.split(","):
        f = torch.ones(G.img_shape, dtype=torch.float32, device="cuda")
        U = G.default_U(f, y, r)
        p = configs.params_2d(a.subsets, 1e7, mode=mode, U=U)
        d = gradient_consistency(G, p, f, y, r, a.iters)
        res[mode] = d
        deg = 180.0 / math.pi
        print(json.dumps({"mode": mode,
                          "theta_mean_deg": [round(x * deg, 3) for x in d["theta_mean"]],
                          "theta_tilde_mean_deg": [round(x * deg, 3) for x in d["theta_tilde_mean"]],
                          "smooth_frac_of_image": float(np.mean(d["n_smooth"][-1])) / f.numel(),
                          "variable_frac_of_image": float(np.mean(d["n_variable"][-1])) / f.numel()}),
              flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh)


if __name__ == "__main__":
    main()
