#!/usr/bin/env python3
"""Benchmark of the SDP-BSREM hot path on one MI355X.

Default workload: the fully 3D reconstruction (200x200x64 volume, 224 angles x
281 bins x 1744 span-1 planes, 64 rings with ring difference <= 15, 28
interleaved subsets, SDP-P2 with the Table III non-TOF row, seeded ellipsoid
phantom, 5e8 counts, 30 % randoms + scatter).  One step = one full
iteration: 28 subiterations (forward projection + ratio, back-projection +
RDP/smoothness stencil, preconditioned update).  The FP64 objective, which no
subiteration needs, is timed on its own (config.objective_ms).  Inputs are
resident in HBM before timing.

The same run measures the metric's batched and served half: 96 uneven 2D
reconstructions advanced by one captured launch per batched subiteration
against the same requests one at a time ("batched"), and a Poisson arrival
trace served by the continuous-batching server against the plain path
("served", recons/s with p50/p99 latency).  --workload c2 / c1 / c2full give
the 2D single-request lines, c4 / c5 the two legs alone.

Prints ONE JSON line (metric, value = subiterations/s, roofline of the
dominant kernel, CPU oracle baselines).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def progress(msg):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"# {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)
WORKLOADS = {
    "c2": "2D SDP-P2, 256x256 image (1.171875 mm), 288 angles x 367 bins, 24 subsets, 5e6 counts, "
          "20% background; step = 1 iteration (24 subiterations); the FP64 objective is timed on its own",
    "c1": "2D SDP-P2, 64x64 image (2 mm), 60 angles x 95 bins, 4 subsets, 1e5 counts, 10% background; "
          "step = 1 iteration (4 subiterations); the FP64 objective is timed on its own",
    "c2full": "2D SDP-P2 with the full system model (32 sub-rays per bin, Gaussian PSF FWHM 6.59 mm, water "
              "attenuation over the object's support), 256x256 image (1.171875 mm), 288 angles x 367 bins, "
              "24 subsets, 5e6 counts, 20% background; step = 1 iteration (24 subiterations); the FP64 objective is timed on its own",
    "c3": "3D SDP-P2, 200x200x64 volume (1.5x1.5x3 mm), 224 angles x 281 bins x 1744 span-1 planes "
          "(64 rings, |d| <= 15), 28 subsets, 5e8 counts, 30% background; step = 1 iteration "
          "(28 subiterations); the FP64 objective is timed on its own",
}
# 3D: three launches per subiteration (the penalty gradient and mu run as
# extra blocks of the back-projector's launch)
KERNELS = {0: "k_fp3 (forward projection + Poisson ratio)",
           1: "k_bp3 (back-projection; RDP gradient and mu blocks in the same launch)",
           2: "k_upd3 (G = b + (beta/M) grad R, nu, S, relaxed step, P_t; z-fastest copy)"}
# 2D: two launches per subiteration (the update is fused into the back-projection)
KERNELS_2D = {0: "k_fp_px (forward projection + Poisson ratio; snapshot of f and mu)",
              1: "k_bp (back-projection + RDP gradient + nu, S, relaxed step, P_t)"}
# 2D with the PSF: the events bracket the blur launches with the projectors
KERNELS_2D_PSF = {0: "k_blur2 + k_fp_px (PSF blur of f; sub-ray forward projection + ratio; snapshot, mu)",
                  1: "k_bp + k_blur2 + k_upd2 (sub-ray back-projection; PSF blur; RDP gradient + update)"}


def kernel_source_hash():
    """Hash of the device sources with comments and whitespace removed: a
    stored traffic measurement stays valid across comment-only edits."""
    import re
    h = hashlib.sha256()
    for name in ("kernels.hip", "kernels3d.hip", "devutil.h", "raygeom.h"):
        with open(os.path.join(ROOT, "paper_2111_07886_amd", "csrc", name), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


# kernel-name prefixes of the per-subiteration launches, by kernel index
TRAFFIC_KERNELS = {2: {0: "void petos::k_fp_px<", 1: "void petos::k_bp<"},
                   3: {0: "petos::k_fp3(", 1: "void petos::k_bp3<", 2: "petos::k_upd3("}}
COPY_BYTES = 64 * 1024 * 1024 * 4      # the --calibrate-copy transfer


def stored_traffic(workload, mode, shapes, kernel):
    """Memory-side bytes per launch of `kernel` (0 forward, 1 back, 2 3D
    update) from profiles/traffic_<workload>.json, or None.  The counts were
    taken with the default projector shapes (counter runs take --no-autotune)
    in one algorithm mode: they hold while the kernel sources, the shapes and
    the mode are the same."""
    tpath = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(tpath):
        return None
    t = json.load(open(tpath))
    if (t.get("kernel_source") == kernel_source_hash() and t.get("shapes") == "default"
            and t.get("mode") == mode and shapes["current"] == shapes["default"]
            and str(kernel) in t.get("bytes_per_launch", {})):
        return t["bytes_per_launch"][str(kernel)]
    return None


def traffic_from_pmc(fetch_csv, write_csv, dim):
    """Measured memory-side bytes per launch from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
    same counter reads for the plain copy of COPY_BYTES (--calibrate-copy);
    the median over the launches of each kernel's most launched variant (the
    per-subiteration one: the autotuner's trial shapes run a few times)."""
    import collections
    import csv
    import statistics

    def per_kernel(path):
        rows = list(csv.DictReader(open(path)))
        copy = max(float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"])
        scale = COPY_BYTES / (copy * 1024.0)
        out = {}
        for k, prefix in TRAFFIC_KERNELS[dim].items():
            by_name = collections.defaultdict(list)
            for r in rows:
                if r["Kernel_Name"].startswith(prefix):
                    by_name[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0 * scale)
            if by_name:
                out[k] = statistics.median(max(by_name.values(), key=len))
        return out, scale

    fetch, sf = per_kernel(fetch_csv)
    write, sw = per_kernel(write_csv)
    return {str(k): int(fetch[k] + write.get(k, 0.0)) for k in fetch}, {"fetch": sf, "write": sw}


# MI355X on-chip ceilings (256 CUs of 4 SIMDs, 8 XCDs of 16 L2 channels, at
# 2.4 GHz): a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles;
# the LDS returns 128 bytes per clock per CU; an L2 channel takes one
# request per clock
CLOCK_HZ = 2.4e9
VALU_WAVE_INSTR_PEAK = 256 * 4 * CLOCK_HZ / 4          # 614.4e9 wave64 instructions / s
LDS_PEAK_BYTES = 256 * 128 * CLOCK_HZ                  # 78.6e12 B/s
L2_REQ_PEAK = 8 * 16 * CLOCK_HZ                        # 307.2e9 requests / s
COUNTERS = ["SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_LDS", "SQ_INSTS_LDS_LOAD_BANDWIDTH",
            "TCC_HIT_sum", "TCC_MISS_sum", "SQ_INSTS_SALU", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64",
            "SQ_INSTS_VALU_MUL_F64", "SQ_LDS_BANK_CONFLICT", "SQ_WAVES", "GRBM_GUI_ACTIVE"]


def counters_from_pmc(csv_paths, dim):
    """Per-launch medians of the rocprofv3 --pmc counters in csv_paths for
    each kernel of the per-subiteration launches (its most launched variant),
    keyed by kernel index as in TRAFFIC_KERNELS."""
    import collections
    import csv
    import statistics
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            vals[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = {}
    for k, prefix in TRAFFIC_KERNELS[dim].items():
        names = [n for n in vals if n.startswith(prefix)]
        if not names:
            continue
        main = max(names, key=lambda n: max(len(v) for v in vals[n].values()))
        out[str(k)] = {c: statistics.median(v) for c, v in vals[main].items()}
    return out


def stored_counters(workload, mode, shapes, kernel):
    """Per-launch counters of `kernel` from profiles/counters_<workload>.json
    while the kernel sources, the shapes and the mode are those profiled."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if (t.get("kernel_source") == kernel_source_hash() and t.get("shapes") == "default"
            and t.get("mode") == mode and shapes["current"] == shapes["default"]):
        return t.get("per_launch", {}).get(str(kernel))
    return None


def onchip_ceilings(c, avg_us, traffic):
    """Fractions of the on-chip ceilings one launch reaches, from its
    counters c (per launch) and its duration: VALU issue, LDS bandwidth, L2
    request rate, and the counted HBM bytes against 8 TB/s."""
    t = avg_us * 1e-6
    out = {}
    if traffic is not None:
        out["hbm_counted"] = {"achieved_GBs": round(traffic / t / 1e9, 1), "peak_GBs": HBM_PEAK_GBS,
                              "frac": round(traffic / t / 1e9 / HBM_PEAK_GBS, 4)}
    if c is None:
        return out or None
    if "SQ_INSTS_VALU" in c:
        r = c["SQ_INSTS_VALU"] / t
        out["valu_issue"] = {"achieved_G_instr_s": round(r / 1e9, 1), "peak_G_instr_s": VALU_WAVE_INSTR_PEAK / 1e9,
                             "frac": round(r / VALU_WAVE_INSTR_PEAK, 4)}
        if "SQ_INSTS_VALU_FMA_F32" in c:
            out["valu_issue"]["fma_f32_share"] = round(c["SQ_INSTS_VALU_FMA_F32"] / c["SQ_INSTS_VALU"], 4)
    if "SQ_INSTS_LDS_LOAD_BANDWIDTH" in c:
        r = 64.0 * c["SQ_INSTS_LDS_LOAD_BANDWIDTH"] / t
        out["lds_load"] = {"achieved_TBs": round(r / 1e12, 2), "peak_TBs": round(LDS_PEAK_BYTES / 1e12, 1),
                           "frac": round(r / LDS_PEAK_BYTES, 4)}
    if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c:
        req = c["TCC_HIT_sum"] + c["TCC_MISS_sum"]
        out["l2_requests"] = {"achieved_G_req_s": round(req / t / 1e9, 1), "peak_G_req_s": L2_REQ_PEAK / 1e9,
                              "frac": round(req / t / L2_REQ_PEAK, 4), "hit_rate": round(c["TCC_HIT_sum"] / req, 4)}
    return out


# FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA x 2 (packed
# FP32) x 2.4 GHz = 157.3 TFLOP/s, the published figure; the kernels are
# built without packed FP32, which halves what they can issue (78.6)
FP32_VECTOR_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2 * CLOCK_HZ / 1e12
FP32_UNPACKED_PEAK_TFLOPS = FP32_VECTOR_PEAK_TFLOPS / 2


def algorithmic_flops(kernel, nnz_sub, rays_sub, q, osem=False):
    """Floating-point work one 3D launch must do: one FMA (2 flops) per
    nonzero in either projector; the Poisson ratio (add, divide, subtract)
    per ray; the penalty blocks of the back-projector's launch (not in OSEM)
    26 neighbour terms of 10 flops plus the gradient magnitude and mu (about
    280 per voxel); the update (kernel 2) about 14 per voxel (G, nu, S,
    step, P_t)."""
    if kernel == 0:
        return 2.0 * nnz_sub + 3.0 * rays_sub
    if kernel == 1:
        return 2.0 * nnz_sub + (0.0 if osem else 280.0 * q)
    return 14.0 * q


def algorithmic_bytes(kernel, nnz_sub, rays_sub, q, dim=3, osem=False, psf=False):
    """Bytes one launch must move (A is computed on the fly, never stored).
    3D, three launches: forward: 4 B image gather per nonzero + read y, r
    and write w per ray; back: 4 B w gather per nonzero + stage w once per
    ray + write A_i^T w per voxel, and its penalty blocks read f and write
    grad R and mu; update: read f, A_i^T w, grad R, mu, p and write f:
    8 nnz + 16 rays + 40 q per subiteration.  2D, two launches: forward + pixel pass (read f, write its
    snapshot and mu), and back-projection + update (read the snapshot, mu, p,
    write f): 8 nnz + 16 rays + 32 q.  OSEM has no mu, p or penalty but reads
    the subset sensitivity: 2D forward + pixel pass 8 q, back + update 12 q;
    3D back 4 q, update 20 q (f, G, s_i in; f and its z copy out)."""
    if psf and dim == 2 and not osem:
        # + the blur of f (read f, write its blur) before the forward projector;
        # the back-projection is written, blurred (read, write) and read again
        return 4.0 * nnz_sub + (12.0 * rays_sub + 20.0 * q if kernel == 0 else 4.0 * rays_sub + 32.0 * q)
    if osem:
        if dim == 2:
            return 4.0 * nnz_sub + (12.0 * rays_sub + 8.0 * q if kernel == 0 else 4.0 * rays_sub + 12.0 * q)
        if kernel == 0:
            return 4.0 * nnz_sub + 12.0 * rays_sub
        if kernel == 1:
            return 4.0 * nnz_sub + 4.0 * rays_sub + 4.0 * q
        return 20.0 * q
    if dim == 2:
        if kernel == 0:
            return 4.0 * nnz_sub + 12.0 * rays_sub + 12.0 * q
        return 4.0 * nnz_sub + 4.0 * rays_sub + 20.0 * q
    if kernel == 0:
        return 4.0 * nnz_sub + 12.0 * rays_sub
    if kernel == 1:
        return 4.0 * nnz_sub + 4.0 * rays_sub + 16.0 * q
    return 24.0 * q


def cpu_baseline_osem(w, budget_s=12.0):
    """The FP64 OSEM oracle on the same workload: subiterations from f0 until
    ~budget_s of CPU work is done."""
    import oracle
    from oracle import osem as O
    oracle.build(force=False)
    att = getattr(w, "att", None)
    g = oracle.geom(dict(w.desc, att=None if att is None else att.astype("float64")))
    M = w.desc["n_subsets"]
    sens = [O.subset_sensitivity(g, i) for i in range(1, M + 1)]
    f = w.f0
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and n < 50 * M:
        i = n % M + 1
        f = O.osem_subiteration(g, f, w.y_f32, w.r_f32, i, sens[i - 1])
        n += 1
    dt = time.perf_counter() - t0
    return {"value": round(n / dt, 3), "unit": "subiterations/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first {n} OSEM subiterations of the same workload from f0 (subset sensitivities "
                      f"precomputed), FP64 oracle, {dt:.1f} s wall", "host": host_cpu()}


def cpu_baseline(w, p, budget_s=12.0):
    """The FP64 oracle, as it stands, on the same workload: subiterations from
    f0 until ~budget_s of CPU work is done.  Like the GPU's timed region it
    evaluates no objective (the paper's Table I subiteration only)."""
    import oracle
    if p["mode"] == "OSEM":
        return cpu_baseline_osem(w, budget_s), None
    oracle.build(force=False)
    att = getattr(w, "att", None)
    g = oracle.geom(dict(w.desc, att=None if att is None else att.astype("float64")))
    rec = oracle.Recon(g, oracle.params(p), w.f0, w.y_f32, w.r_f32)
    M = w.desc["n_subsets"]
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and n < 50 * M and (n == 0 or budget_s > 0):
        rec.subiteration()
        n += 1
    dt = time.perf_counter() - t0
    out = {"value": round(n / dt, 3), "unit": "subiterations/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": f"first {n} subiterations of the same workload from f0 (no objective evaluations, as in "
                     f"the GPU's timed region), FP64 C oracle, {dt:.1f} s wall"}
    out["one_thread"] = one_thread_rate(g, p, w, n / dt)
    out["host"] = host_cpu()
    return out, rec


def host_cpu():
    """The host the oracle ran on: logical CPUs visible and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu": model}


def one_thread_rate(g, p, w, rate_all, budget_s=4.0):
    """The same oracle on one host thread, from f0, for about budget_s (at
    least one subiteration; skipped where one would take over 20 s)."""
    import oracle
    nt = oracle.num_threads()
    if nt > 1 and nt / rate_all > 20.0:
        return None
    oracle.set_num_threads(1)
    try:
        rec = oracle.Recon(g, oracle.params(p), w.f0, w.y_f32, w.r_f32)
        n = 0
        t0 = time.perf_counter()
        while n == 0 or time.perf_counter() - t0 < budget_s:
            rec.subiteration()
            n += 1
        dt = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(nt)
    return {"value": round(n / dt, 3), "unit": "subiterations/s", "sample": f"first {n} subiterations, {dt:.1f} s"}


def one_step_error(rec, geom, p, w):
    """Error of the GPU path against the oracle where the baseline stopped:
    one GPU subiteration and one oracle subiteration from the oracle's own
    state (iterate cast to FP32, position, Nesterov t, frozen nu); rel-L2."""
    import numpy as np
    import torch

    import paper_2111_07886_amd as pet
    fin = np.asarray(rec.f, dtype=np.float32).astype(np.float64)
    ref = rec.clone_with(fin)
    ref.frozen = np.asarray(rec.frozen, dtype=np.float32).astype(np.float64)
    ref.subiteration()
    st = pet.State(geom, p)
    nu = None
    if rec.st.have_frozen:
        nu = torch.tensor(ref.frozen.reshape(geom.img_shape), dtype=torch.float32, device="cuda")
    st.seek(rec.st.k, rec.st.i, rec.st.t_nest, nu)
    fg = torch.tensor(fin.reshape(geom.img_shape), dtype=torch.float32, device="cuda")
    st.subiteration(fg, torch.tensor(w.y_f32, dtype=torch.float32, device="cuda").reshape(geom.sino_shape),
                    torch.tensor(w.r_f32, dtype=torch.float32, device="cuda").reshape(geom.sino_shape))
    torch.cuda.synchronize()
    st.close()
    g = fg.cpu().double().numpy().reshape(-1)
    o = ref.image().reshape(-1)
    return float(np.linalg.norm(g - o) / np.linalg.norm(o)), int(rec.st.k), int(rec.st.i)


def oracle_recons_rate(items, budget_s=15.0, note=""):
    """The FP64 oracle, as it stands, on a bounded sample of reconstruction
    requests: (geometry descriptor, params, f0, y, r, n_iter) items taken in
    order, subiteration by subiteration (no objective evaluations, as in the
    GPU's timed region), until ~budget_s of CPU work is done.  A request cut
    short counts by the fraction of its subiterations done."""
    import oracle
    oracle.build(force=False)
    done, subs, started = 0.0, 0, 0
    t0 = time.perf_counter()
    for desc, p, f0, y, r, n_iter in items:
        if time.perf_counter() - t0 >= budget_s:
            break
        started += 1
        g = oracle.geom(desc)
        rec = oracle.Recon(g, oracle.params(p), f0, y, r)
        total = n_iter * desc["n_subsets"]
        k = 0
        while k < total and time.perf_counter() - t0 < budget_s:
            rec.subiteration()
            k += 1
        done += k / total
        subs += k
    dt = time.perf_counter() - t0
    return {"value": round(done / dt, 4), "unit": "recons/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{note}: {started} requests started, {done:.2f} reconstructions' worth ({subs} "
                      f"subiterations, no objective) in {dt:.1f} s, FP64 C oracle",
            "subiterations_per_s": round(subs / dt, 3), "host": host_cpu()}


def calibrate_copy(dev):
    """A plain device copy of COPY_BYTES, the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the same process."""
    import torch
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def bench_batched(args, cpu=True):
    """96 uneven 2D reconstructions (10 iterations each): one batch, one
    captured step per subiteration, vs the same requests one at a time."""
    import numpy as np
    import torch

    import paper_2111_07886_amd as pet
    from synth import configs

    specs = configs.c4_specs()
    progress("batched: generating 96 requests")
    reqs = [configs.c4_workload(sp) for sp in specs]
    dev = torch.device("cuda:0")
    geoms, ys, rs = [], [], []
    for w, p, n in reqs:
        G = pet.Geometry(w.desc)
        if not args.no_autotune:
            pet.autotune(G)
        geoms.append(G)
        ys.append(torch.tensor(w.y, dtype=torch.float32, device=dev))
        rs.append(torch.tensor(w.r, dtype=torch.float32, device=dev))
    n_sub = sum(n * w.desc["n_subsets"] for w, _, n in reqs)
    bytes_total = 0.0
    for (w, p, n), G in zip(reqs, geoms):
        M = w.desc["n_subsets"]
        bytes_total += n * (8.0 * G.nnz(0) + 16.0 * G.n_bins + 32.0 * M * G.n_voxels)
    params = [p for _, p, _ in reqs]
    iters = [n for _, _, n in reqs]
    if getattr(args, "calibrate_copy", False):
        calibrate_copy(dev)
    # warm-up (graph capture, caches)
    progress("batched: geometries ready, timing")
    fs = [torch.tensor(w.f0, dtype=torch.float32, device=dev) for w, _, _ in reqs]
    pet.reconstruct_batch(geoms, params, fs, ys, rs, [1] * len(reqs))
    fs = [torch.tensor(w.f0, dtype=torch.float32, device=dev) for w, _, _ in reqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pet.reconstruct_batch(geoms, params, fs, ys, rs, iters)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    fs2 = [torch.tensor(w.f0, dtype=torch.float32, device=dev) for w, _, _ in reqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for G, p, f, y, r, n in zip(geoms, params, fs2, ys, rs, iters):
        pet.reconstruct(G, p, f, y, r, n)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(fs, fs2))
    cpu_base = None
    if cpu:
        progress("batched: oracle sample")
        # every 8th request (a spread of sizes), data as the GPU sees them (FP32)
        f32 = lambda t: t.cpu().double().numpy()
        items = [(w.desc, p, w.f0, f32(ys[k]), f32(rs[k]), n) for k, (w, p, n) in enumerate(reqs) if k % 8 == 0]
        cpu_base = oracle_recons_rate(items, note="every 8th of the 96 batched requests")
    return {"metric": "recons/s", "value": round(len(reqs) / tb, 3), "unit": "recons/s", "n_gpus": 1,
            "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * tb, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "batched: 96 uneven 2D SDP-P2 reconstructions (64..320 px, 60..360 angles, "
                                   "4..32 subsets, 1e5..1e7 counts), 10 iterations each; step = all 96 to the end",
                       "subiterations": n_sub, "subiterations_per_s": round(n_sub / tb, 1),
                       "plain_one_at_a_time_s": round(tp, 4), "plain_recons_per_s": round(len(reqs) / tp, 3),
                       "speedup_vs_plain": round(tp / tb, 3), "batched_equals_plain_bitwise": same},
            "roofline": {"bound": "hbm", "achieved": round(bytes_total / tb / 1e9, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(bytes_total / tb / 1e9 / HBM_PEAK_GBS, 5), "traffic": None,
                         "kernel": "whole batched step (all kernels), algorithmic bytes 8 nnz + 16 rays + 32 q "
                                   "per subiteration"},
            "cpu_baseline": cpu_base}


def bench_served(args, cpu=True):
    """Poisson arrivals (200 req/s) of 2D (128..320 px) and 3D (128x128x32)
    requests, 30 iterations each: the continuous-batching server vs the same
    trace served one request at a time (FIFO) by pet_os_reconstruct."""
    import tempfile

    import numpy as np
    import torch

    import paper_2111_07886_amd as pet
    from synth import configs, phantoms

    # the server and the plain path take the same autotuned shapes for a
    # geometry (the tuning result is timed, so it may differ run to run)
    os.environ["PET_OS_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="petos_tune_"), "tune.txt")
    trace = configs.c5_trace(n_requests=args.requests)
    dev = torch.device("cuda:0")
    reqs = []
    progress(f"served: generating {len(trace)} requests")
    for qi, q in enumerate(trace):
        if qi % 50 == 49:
            progress(f"served: {qi + 1} requests generated")
        d = q["desc"]
        if d["dim"] == 3:
            w = phantoms.make_3d(d, seed=q["seed"], n_ell=11, counts=q["counts"], bg_uniform=0.1, bg_scatter=0.1)
            p = configs.params_3d(U=w.U)
        else:
            w = phantoms.make_2d(d, seed=q["seed"], n_ell=8, counts=q["counts"], bg_frac=0.2)
            p = configs.params_2d(d["n_subsets"], q["counts"], U=w.U)
        y = torch.tensor(w.y, dtype=torch.float32, device=dev)
        r = torch.tensor(w.r, dtype=torch.float32, device=dev)
        f0 = torch.tensor(w.f0, dtype=torch.float32, device=dev)
        reqs.append((w.desc, p, q["n_iter"], q["arrival_s"], f0, y, r))
    # geometry caches warm in both paths: every distinct geometry once
    keys = {}
    for desc, p, n, at, f0, y, r in reqs:
        keys.setdefault(json.dumps(desc, sort_keys=True), (desc, p, f0, y, r))
    S = pet.Server(64 << 30, args.slots)
    for desc, p, f0, y, r in keys.values():
        S.wait(S.submit(desc, p, f0.clone(), y, r, 1))
    plain_geoms = {}
    for k, (desc, p, f0, y, r) in keys.items():
        G = pet.Geometry(desc)
        if not args.no_autotune:
            pet.autotune(G)
        plain_geoms[k] = G
    torch.cuda.synchronize()

    def pct(v, q):
        return float(np.percentile(np.asarray(v), q))

    # served
    progress("served: geometries warm, serving the trace")
    fs = [f0.clone() for *_, f0, y, r in reqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = []
    for (desc, p, n, at, f0, y, r), f in zip(reqs, fs):
        dt = at - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(S.submit(desc, p, f, y, r, n))
    res = [S.wait(t) for t in tickets]
    st = S.stats()
    S.close()
    lat_s = [r_["t_finish"] - r_["t_submit"] for r_ in res]
    span_s = max(r_["t_finish"] for r_ in res) - min(r_["t_submit"] for r_ in res)
    ok = sum(r_["status"] == 0 for r_ in res)
    # plain: one at a time, arrival order, same arrival times
    progress("served: the same trace one request at a time")
    fs2 = [f0.clone() for *_, f0, y, r in reqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat_p, fin = [], []
    for (desc, p, n, at, f0, y, r), f in zip(reqs, fs2):
        dt = at - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        pet.reconstruct(plain_geoms[json.dumps(desc, sort_keys=True)], p, f, y, r, n)
        torch.cuda.synchronize()
        now = time.perf_counter() - t0
        lat_p.append(now - at)
        fin.append(now)
    span_p = fin[-1] - reqs[0][3]
    same = sum(torch.equal(a, b) for a, b in zip(fs, fs2))
    n = len(reqs)
    cpu_base = None
    if cpu:
        progress("served: oracle sample")
        f32 = lambda t: t.cpu().double().numpy()
        items = [(desc, p, f32(f0), f32(y), f32(r), nn) for k, (desc, p, nn, at, f0, y, r) in enumerate(reqs)
                 if k % 20 == 0]
        cpu_base = oracle_recons_rate(items, note="every 20th request of the arrival trace, one at a time")
    out = {"metric": "served recons/s", "value": round(n / span_s, 3), "unit": "recons/s", "n_gpus": 1,
           "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * span_s, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"served: {n} requests, Poisson arrivals at 200/s, 98% 2D (128..320 px) / "
                                  f"2% 3D (128x128x32, 180x185x424 planes), 30 iterations each",
                      "completed": ok, "p50_latency_ms": round(1e3 * pct(lat_s, 50), 2),
                      "p99_latency_ms": round(1e3 * pct(lat_s, 99), 2), "slots": args.slots,
                      "max_active": st["max_active"],
                      "plain_recons_per_s": round(n / span_p, 3),
                      "plain_p50_latency_ms": round(1e3 * pct(lat_p, 50), 2),
                      "plain_p99_latency_ms": round(1e3 * pct(lat_p, 99), 2),
                      "results_equal_to_plain": f"{same}/{n}"},
           "roofline": None, "cpu_baseline": cpu_base}
    return out


def bench_gradcons(args):
    """Gradient-consistency diagnostic (Sec. IV-B, Fig. 2) riding along the
    reconstruction: every subiteration is followed by grad Phi_i at the new
    iterate and the two angles.  value = such subiterations per second; the
    plain rate of the same workload is reported beside it.  The per-kernel
    durations of the diagnostic come from rocprofv3 (the entry points are
    synchronous calls that allocate their scratch, so HIP events around them
    would include host time)."""
    import torch

    import paper_2111_07886_amd as pet
    from paper_2111_07886_amd.diagnostics import gradient_consistency
    from synth import configs

    three = args.workload == "gradcons3"
    w, p, _ = (configs.c3 if three else configs.c2)()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    y = torch.tensor(w.y, dtype=torch.float32, device=dev).contiguous()
    r = torch.tensor(w.r, dtype=torch.float32, device=dev).contiguous()
    w.att = None
    if getattr(w, "mu", None) is not None:
        # attenuation factors of the geometry's own rays through the mu map
        g0 = pet.Geometry(w.desc)
        w.att = g0.attenuation_factors(torch.tensor(w.mu, dtype=torch.float32, device=dev)).cpu().numpy()
        g0.close()
    geom = pet.Geometry(w.desc, att=w.att)
    if not args.no_autotune:
        # the library's own tuner: projector shapes timed on the first subset
        pet.autotune(geom)
    M = w.desc["n_subsets"]
    steps = max(1, args.steps if not three else min(args.steps, 3))
    f = torch.tensor(w.f0, dtype=torch.float32, device=dev).contiguous()
    st = pet.State(geom, p)
    gradient_consistency(geom, p, f, y, r, 1, state=st)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = gradient_consistency(geom, p, f, y, r, steps, state=st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st.close()
    f = torch.tensor(w.f0, dtype=torch.float32, device=dev).contiguous()
    st = pet.State(geom, p)
    st.run(f, y, r, 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st.run(f, y, r, steps)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t1
    st.close()
    deg = 180.0 / 3.141592653589793
    res = {
        "metric": "subiterations/s (with the gradient-consistency diagnostic)",
        "value": round(steps * M / elapsed, 2),
        "unit": "subiterations/s",
        "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": round(1e3 * elapsed / steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "gradient consistency along SDP-P2 on " + WORKLOADS["c3" if three else "c2"].split(";")[0]
                               + "; step = 1 iteration, each subiteration followed by grad Phi_i and the two angles",
                   "plain_subiterations_per_s": round(steps * M / plain, 2),
                   "theta_mean_deg_last": round(out["theta_mean"][-1] * deg, 4),
                   "theta_tilde_mean_deg_last": round(out["theta_tilde_mean"][-1] * deg, 4)},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default projector shapes (the served workload's server still tunes its "
                         "2D geometries)")
    ap.add_argument("--workload", default="c3",
                    choices=["c3", "c2", "c1", "c2full", "c4", "c5", "gradcons", "gradcons3"],
                    help="c3 (default: the benchmark line, with the batched and served legs); c1 / c2 / c2full "
                         "for the 2D single-request measurements; c4 / c5 for the batched / served legs alone")
    ap.add_argument("--no-batched", action="store_true", help="c3: leave out the batched leg (c4)")
    ap.add_argument("--no-served", action="store_true", help="c3: leave out the served leg (c5)")
    ap.add_argument("--requests", type=int, default=400, help="c5: requests taken from the arrival trace")
    ap.add_argument("--slots", type=int, default=128, help="c5: requests the server runs at once")
    ap.add_argument("--mode", default=None, choices=["BSREM", "M1", "M2", "P1", "P2", "OSEM"],
                    help="c1/c2/c3: run this algorithm instead of the workload's SDP-P2 (OSEM: the "
                         "initialisation of Sec. IV-C)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (for PMC byte-counter scaling)")
    ap.add_argument("--counters-from", nargs="+", metavar="PMC_CSV",
                    help="write profiles/counters_<workload>.json from rocprofv3 --pmc counter CSVs of this "
                         "workload run with --no-autotune (the default projector shapes), and exit")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<workload>.json from two rocprofv3 --pmc counter CSVs "
                         "(FETCH_SIZE, WRITE_SIZE) of this workload run with --calibrate-copy --no-autotune "
                         "(the default projector shapes), and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "runs on one GPU only: sharding across GPUs is designed but neither "
                                   "built nor measured", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.counters_from:
        dim = 3 if args.workload == "c3" else 2
        out = {"workload": args.workload, "mode": args.mode or "P2", "kernel_source": kernel_source_hash(),
               "shapes": "default", "per_launch": counters_from_pmc(args.counters_from, dim),
               "note": "rocprofv3 --pmc counters per launch (median over the launches of each kernel's "
                       "per-subiteration variant), runs with the default projector shapes (--no-autotune)"}
        path = os.path.join(ROOT, "profiles", f"counters_{args.workload}.json")
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print(json.dumps(out))
        return
    if args.traffic_from:
        dim = 3 if args.workload == "c3" else 2
        per, scale = traffic_from_pmc(args.traffic_from[0], args.traffic_from[1], dim)
        out = {"workload": args.workload, "mode": args.mode or "P2", "kernel_source": kernel_source_hash(),
               "shapes": "default",
               "bytes_per_launch": per, "counter_scale": scale,
               "note": "memory-side bytes (FETCH_SIZE + WRITE_SIZE) per launch, median over the launches of "
                       "each kernel's per-subiteration variant, scaled by the counters of a plain 256 MiB copy; "
                       "counter runs with the default projector shapes (--no-autotune)"}
        path = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print(json.dumps(out))
        return
    if args.workload == "c4":
        print(json.dumps(bench_batched(args, cpu=not args.no_cpu_baseline)), flush=True)
        return
    if args.workload == "c5":
        print(json.dumps(bench_served(args, cpu=not args.no_cpu_baseline)), flush=True)
        return
    if args.workload in ("gradcons", "gradcons3"):
        return bench_gradcons(args)

    import numpy as np
    import torch

    import paper_2111_07886_amd as pet
    from synth import configs

    progress(f"{args.workload}: generating the workload")
    w, p, _ = {"c1": configs.c1, "c2": configs.c2, "c3": configs.c3, "c2full": configs.c2_full}[args.workload]()
    progress(f"{args.workload}: workload ready")
    if args.mode == "OSEM":
        p = pet.osem_params(p["beta"], p["gamma_R"], p["eps"])
    elif args.mode:
        p = dict(p, mode=args.mode)
    p = dict(p, objective_every=1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    f = torch.tensor(w.f0, dtype=torch.float32, device=dev).contiguous()
    y = torch.tensor(w.y, dtype=torch.float32, device=dev).contiguous()
    r = torch.tensor(w.r, dtype=torch.float32, device=dev).contiguous()
    w.y_f32 = y.cpu().double().numpy()
    w.r_f32 = r.cpu().double().numpy()
    w.att = None
    if getattr(w, "mu", None) is not None:
        # attenuation factors of the geometry's own rays through the mu map
        g0 = pet.Geometry(w.desc)
        w.att = g0.attenuation_factors(torch.tensor(w.mu, dtype=torch.float32, device=dev)).cpu().numpy()
        g0.close()
    geom = pet.Geometry(w.desc, att=w.att)
    if not args.no_autotune:
        # the library's own tuner: projector shapes timed on the first subset
        pet.autotune(geom)
    shapes = geom.shapes()
    M = w.desc["n_subsets"]
    state = pet.State(geom, p)

    if args.calibrate_copy:
        calibrate_copy(dev)

    # warm-up, then exactly `steps` timed iterations bracketed by synchronisation
    # the timed steps are subiterations only: the objective (not part of a
    # subiteration) is timed on its own below
    state.run(f, y, r, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    state.run(f, y, r, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    progress(f"{args.workload}: {args.steps} timed steps in {elapsed:.3f} s")
    sub_per_s = args.steps * M / elapsed
    # the FP64 objective of the iterate, as a state evaluates it after an
    # iteration (device time of one more iteration with and without it)
    obj_ms = None
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    obj = state.run(f, y, r, 1, want_objective=True)
    ev[1].record()
    state.run(f, y, r, 1)
    ev[2].record()
    torch.cuda.synchronize()
    obj_ms = max(0.0, ev[0].elapsed_time(ev[1]) - ev[1].elapsed_time(ev[2]))

    # the spread of the step time: HIP events around each of `steps` more
    # steps (outside the timed region)
    sev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    sev[0].record()
    for k in range(args.steps):
        state.run(f, y, r, 1)
        sev[k + 1].record()
    torch.cuda.synchronize()
    step_ms = sorted(sev[k].elapsed_time(sev[k + 1]) for k in range(args.steps))

    def pct(v, q):
        return v[min(len(v) - 1, int(round(q * (len(v) - 1))))]

    step_spread = {"p10": round(pct(step_ms, 0.1), 4), "p50": round(pct(step_ms, 0.5), 4),
                   "p90": round(pct(step_ms, 0.9), 4), "n": len(step_ms)}

    # per-kernel device time: HIP events on the launch stream around every
    # launch of one kernel, over a pass of the same steps (kept out of the
    # timed region above so that the events do not perturb it)
    nnz_sub = geom.nnz(0) / M
    rays_sub = geom.n_bins / M
    q = geom.n_voxels
    per_kernel = {}
    dim = w.desc["dim"]
    psf = dim == 2 and w.desc.get("psf_fwhm", 0.0) > 0.0
    names = (KERNELS_2D_PSF if psf else KERNELS_2D) if dim == 2 else KERNELS
    if not args.no_profile:
        for k in names:
            state.profile(k)
            state.run(f, y, r, min(args.steps, 10))
            ms, n = state.profile_read()
            state.profile(-1)
            if n:
                per_kernel[k] = dict(avg_us=1e3 * ms / n, launches=n,
                                     bytes=algorithmic_bytes(k, nnz_sub, rays_sub, q, dim,
                                                             osem=p["mode"] == "OSEM", psf=psf))
    roofline = None
    if per_kernel:
        dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_us"])
        roofline = roofline_of(per_kernel, dom, names, dim, nnz_sub, rays_sub, q,
                               stored_traffic(args.workload, p["mode"], shapes, dom),
                               stored_counters(args.workload, p["mode"], shapes, dom),
                               osem=p["mode"] == "OSEM")

    del state
    cpu, parity = None, None
    if not args.no_cpu_baseline:
        progress(f"{args.workload}: oracle baseline")
        cpu, rec = cpu_baseline(w, p)
        if rec is not None:
            e, k_at, i_at = one_step_error(rec, geom, p, w)
            parity = {"one_subiteration_rel_l2": e, "at_k": k_at, "at_i": i_at,
                      "what": "one GPU subiteration vs one FP64 oracle subiteration from the oracle's state "
                              "where the CPU baseline stopped (FP32-cast iterate)"}

    out = {
        "metric": "subiterations/s",
        "value": round(sub_per_s, 2),
        "unit": "subiterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] if not args.mode else
                   WORKLOADS[args.workload].replace("SDP-P2", "OSEM" if args.mode == "OSEM" else "SDP-" + args.mode),
                   "subsets": M, "nnz_per_subset": int(nnz_sub), "rays_per_subset": int(rays_sub),
                   "voxels": q, "autotuned": not args.no_autotune, "shapes": shapes["current"],
                   "attenuation": w.att is not None,
                   "objective_last": obj[-1] if obj else None,
                   "objective_ms": None if obj_ms is None else round(obj_ms, 4),
                   "step_ms_spread": step_spread},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    if args.workload == "c3":
        # the metric's batched and served half, measured in the same run
        if not args.no_batched:
            out["batched"] = leg_summary(bench_batched(args, cpu=not args.no_cpu_baseline))
            progress(f"batched leg done: {out['batched']['recons_per_s']} recons/s")
        if not args.no_served:
            out["served"] = leg_summary(bench_served(args, cpu=not args.no_cpu_baseline))
            progress(f"served leg done: {out['served']['recons_per_s']} recons/s")
    print(json.dumps(out), flush=True)


def roofline_of(per_kernel, dom, names, dim, nnz_sub, rays_sub, q, traffic, counters, osem=False):
    """The roofline record of the dominant kernel `dom`.  2D: HBM-bound,
    achieved = its algorithmic bytes over its average launch.  3D: the
    projectors' gathers are served by LDS and L2, not HBM (their algorithmic
    byte rate exceeds what HBM delivers), so the bound is the VALU: achieved
    = algorithmic flops over the launch against FP32 FMA issue; the byte
    rate is kept under its own key.  `ceilings`: what the launch reaches of
    each on-chip ceiling, from the counters on record and the same
    duration."""
    K = per_kernel[dom]
    t = K["avg_us"] * 1e-6
    rate_gbs = K["bytes"] / t / 1e9
    common = {"traffic": traffic, "kernel": names[dom], "avg_launch_us": round(K["avg_us"], 3),
              "algorithmic_bytes_per_launch": int(K["bytes"]),
              "per_kernel_us": {names[k].split(" (")[0]: round(v["avg_us"], 3) for k, v in per_kernel.items()},
              "ceilings": onchip_ceilings(counters, K["avg_us"], traffic)}
    if dim == 3:
        fl = algorithmic_flops(dom, nnz_sub, rays_sub, q, osem=osem)
        achieved = fl / t / 1e12
        out = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(FP32_VECTOR_PEAK_TFLOPS, 1),
               "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 5),
               "frac_of_unpacked_fp32": round(achieved / FP32_UNPACKED_PEAK_TFLOPS, 5),
               "algorithmic_flops_per_launch": int(fl),
               "algorithmic_bytes_GBs": round(rate_gbs, 1)}
    else:
        out = {"bound": "hbm", "achieved": round(rate_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(rate_gbs / HBM_PEAK_GBS, 5)}
    out.update(common)
    return out


def leg_summary(line):
    """The batched or served measurement as keys of the benchmark line."""
    c = line["config"]
    out = {"workload": c["workload"], "recons_per_s": line["value"], "wall_s": round(line["ms_per_step"] / 1e3, 4)}
    for k in ("subiterations_per_s", "plain_recons_per_s", "speedup_vs_plain", "batched_equals_plain_bitwise",
              "p50_latency_ms", "p99_latency_ms", "plain_p50_latency_ms", "plain_p99_latency_ms", "slots",
              "max_active", "completed", "results_equal_to_plain"):
        if k in c:
            out[k] = c[k]
    if "speedup_vs_plain" not in out and "plain_recons_per_s" in c:
        out["speedup_vs_plain"] = round(line["value"] / c["plain_recons_per_s"], 3)
    if line.get("roofline"):
        out["roofline"] = line["roofline"]
    out["cpu_baseline"] = line.get("cpu_baseline")
    return out


if __name__ == "__main__":
    main()
