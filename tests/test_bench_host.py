"""Host-side logic of bench.py (no GPU): the one-GPU contract, the
algorithmic byte model, the memory-side traffic from PMC counter CSVs, the
kernel-source key of stored traffic, and the oracle baseline record."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    saved = sys.argv
    sys.argv = ["bench.py"]
    try:
        import bench as b
    finally:
        sys.argv = saved
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


@pytest.mark.parametrize("osem", [False, True])
def test_byte_model_totals(bench, osem):
    """Per subiteration the launches move 8 nnz + 16 rays + 32 q bytes in 2D
    and 8 nnz + 16 rays + 40 q in 3D, whose back-projector's penalty blocks
    read f and write grad R and mu, and whose update reads the back-projection
    and grad R (OSEM: no mu, p or penalty, but the subset sensitivity; 2D
    8 nnz + 16 rays + 20 q, 3D 8 nnz + 16 rays + 24 q)."""
    nnz, rays, q = 1_001_276.0, 4404.0, 65536.0
    two = sum(bench.algorithmic_bytes(k, nnz, rays, q, dim=2, osem=osem) for k in (0, 1))
    three = sum(bench.algorithmic_bytes(k, nnz, rays, q, dim=3, osem=osem) for k in (0, 1, 2))
    if not osem:
        assert two == 8 * nnz + 16 * rays + 32 * q
        assert three == 8 * nnz + 16 * rays + 40 * q
    else:
        assert two == 8 * nnz + 16 * rays + 20 * q
        assert three == 8 * nnz + 16 * rays + 24 * q
    # the full model adds the blur of f and of the back-projection
    full = sum(bench.algorithmic_bytes(k, nnz, rays, q, dim=2, psf=True) for k in (0, 1))
    assert full == 8 * nnz + 16 * rays + 52 * q


def _pmc_csv(path, counter, rows):
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for i, (name, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val})


def test_traffic_from_counters(bench, tmp_path):
    """Counters scaled by what they read for the plain copy, the median over
    the most launched variant of each kernel (trial shapes left out)."""
    copy_kib = bench.COPY_BYTES / 1024.0
    fp = "void petos::k_fp_px<64, false>(petos::GeoK, petos::FPArgs, petos::PxArgs, int)"
    bp = "void petos::k_bp<petos::Tile<8, 8, 4>, false, false>(petos::GeoK, petos::BPArgs)"
    trial = "void petos::k_bp<petos::Tile<16, 16, 1>, false, false>(petos::GeoK, petos::BPArgs)"
    # FETCH_SIZE reads half of the copy's bytes (x2), WRITE_SIZE all of them (x1)
    _pmc_csv(tmp_path / "f.csv", "FETCH_SIZE",
             [("__amd_rocclr_copyBuffer", copy_kib / 2), (fp, 100.0), (fp, 110.0), (fp, 120.0),
              (bp, 200.0), (bp, 210.0), (bp, 220.0), (trial, 9999.0)])
    _pmc_csv(tmp_path / "w.csv", "WRITE_SIZE",
             [("__amd_rocclr_copyBuffer", copy_kib), (fp, 10.0), (fp, 10.0), (fp, 10.0),
              (bp, 20.0), (bp, 20.0), (bp, 20.0), (trial, 1.0), (trial, 1.0)])
    per, scale = bench.traffic_from_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 2)
    assert scale == {"fetch": 2.0, "write": 1.0}
    assert per["0"] == int((2 * 110.0 + 10.0) * 1024)
    assert per["1"] == int((2 * 210.0 + 20.0) * 1024)


def test_source_key_ignores_comments(bench, tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2111_07886_amd" / "csrc"
    csrc.mkdir(parents=True)
    names = ("kernels.hip", "kernels3d.hip", "devutil.h", "raygeom.h")
    for n in names:
        (csrc / n).write_text("int f(int x) { return x + 1; }  // one\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    k0 = bench.kernel_source_hash()
    (csrc / "kernels.hip").write_text("/* header */\nint f(int x)\n{\n    return x + 1;  // other words\n}\n")
    assert bench.kernel_source_hash() == k0
    (csrc / "kernels.hip").write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash() != k0


def test_cpu_baseline_record(bench):
    """The oracle leg on the 64x64 case: rate, host threads, the one-thread
    rate and the oracle state handed to the parity check."""
    import oracle
    from synth import configs
    oracle.build(force=False)
    w, p, _ = configs.c1()
    w.y_f32 = w.y.astype("float32").astype("float64")
    w.r_f32 = w.r.astype("float32").astype("float64")
    out, rec = bench.cpu_baseline(w, p, budget_s=0.5)
    assert out["kind"] == "oracle" and out["unit"] == "subiterations/s" and out["value"] > 0
    assert out["cores"] == oracle.num_threads() >= 1
    one = out["one_thread"]
    assert one is not None and one["value"] > 0
    assert oracle.num_threads() == out["cores"]       # the thread count is restored
    assert rec is not None and rec.st.k * w.desc["n_subsets"] + rec.st.i - 1 >= 1
    assert out["host"]["nproc"] >= 1 and "cpu" in out["host"]


def test_stored_traffic_needs_same_sources_shapes_and_mode(bench, tmp_path, monkeypatch):
    """The counted bytes of a kernel are reported only for the sources, the
    default shapes and the algorithm mode they were counted with."""
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "k1")
    rec = {"workload": "c2", "mode": "P2", "kernel_source": "k1", "shapes": "default",
           "bytes_per_launch": {"0": 111, "1": 222}}
    (tmp_path / "profiles" / "traffic_c2.json").write_text(json.dumps(rec))
    dflt = {"fp_seg": 64, "bp_kind": 1}
    same = {"current": dict(dflt), "default": dict(dflt)}
    assert bench.stored_traffic("c2", "P2", same, 1) == 222
    assert bench.stored_traffic("c2", "P2", same, 2) is None          # kernel not counted
    assert bench.stored_traffic("c2", "OSEM", same, 1) is None        # other mode
    tuned = {"current": dict(dflt, fp_seg=16), "default": dict(dflt)}
    assert bench.stored_traffic("c2", "P2", tuned, 1) is None         # other shapes
    assert bench.stored_traffic("c3", "P2", same, 1) is None          # nothing stored
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "k2")
    assert bench.stored_traffic("c2", "P2", same, 1) is None          # sources changed


def test_counters_and_onchip_ceilings(bench, tmp_path):
    """Per-launch counters are the medians over the most launched variant of
    each kernel; the ceilings divide them by the launch's duration against
    the chip's VALU issue (256 CUs x 4 SIMDs, a wave64 instruction every 4
    cycles at 2.4 GHz), LDS (128 B per clock per CU) and L2 request
    (8 x 16 channels, one per clock) rates."""
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    bp = "void petos::k_bp3<64, 20>(petos::GeoK, petos::BP3Args, int)"
    trial = "void petos::k_bp3<32, 20>(petos::GeoK, petos::BP3Args, int)"
    _pmc_csv(a, "SQ_INSTS_VALU", [(bp, 100.0), (bp, 300.0), (bp, 200.0), (trial, 7.0)])
    _pmc_csv(b, "TCC_HIT_sum", [(bp, 90.0), (bp, 90.0), (bp, 90.0)])
    with open(b, "a", newline="") as fh:
        w = csv.writer(fh)
        for i in range(3):
            w.writerow([10 + i, bp, "TCC_MISS_sum", 10.0])
    per = bench.counters_from_pmc([str(a), str(b)], 3)
    assert per["1"] == {"SQ_INSTS_VALU": 200.0, "TCC_HIT_sum": 90.0, "TCC_MISS_sum": 10.0}
    assert bench.VALU_WAVE_INSTR_PEAK == 614.4e9
    assert abs(bench.LDS_PEAK_BYTES - 78.6432e12) < 1e6 and bench.L2_REQ_PEAK == 307.2e9
    c = {"SQ_INSTS_VALU": 614.4e3, "SQ_INSTS_VALU_FMA_F32": 153.6e3, "SQ_INSTS_LDS_LOAD_BANDWIDTH": 1e6,
         "TCC_HIT_sum": 2.4576e5, "TCC_MISS_sum": 6.144e4}
    out = bench.onchip_ceilings(c, 2.0, 8e6)          # a 2 us launch
    assert abs(out["valu_issue"]["frac"] - 0.5) < 1e-9 and out["valu_issue"]["fma_f32_share"] == 0.25
    assert abs(out["lds_load"]["achieved_TBs"] - 32.0) < 1e-9
    assert abs(out["l2_requests"]["frac"] - 0.5) < 1e-9 and out["l2_requests"]["hit_rate"] == 0.8
    assert out["hbm_counted"]["achieved_GBs"] == 4000.0 and out["hbm_counted"]["frac"] == 0.5
    assert bench.onchip_ceilings(None, 2.0, None) is None


def test_roofline_bound_by_dimension(bench):
    """2D: the dominant kernel's algorithmic bytes over its launch against
    8 TB/s.  3D: the gathers are served on chip, so the record is the VALU
    bound: 2 flops per nonzero (and, in the back-projector's launch, ~280
    per voxel for its penalty blocks, none in OSEM) over the launch against
    the published FP32 vector peak (157.3 TFLOP/s; 78.6 without packed
    FP32), with the byte rate under its own key."""
    assert abs(bench.FP32_VECTOR_PEAK_TFLOPS - 157.2864) < 1e-9
    assert abs(bench.FP32_UNPACKED_PEAK_TFLOPS - 78.6432) < 1e-9
    names = {0: "k_fp3 (x)", 1: "k_bp3 (y)"}
    nnz, rays, q = 1e9, 4e6, 2.5e6
    per = {0: {"avg_us": 100.0, "bytes": bench.algorithmic_bytes(0, nnz, rays, q, 3)},
           1: {"avg_us": 400.0, "bytes": bench.algorithmic_bytes(1, nnz, rays, q, 3)}}
    r3 = bench.roofline_of(per, 1, names, 3, nnz, rays, q, None, None, osem=True)
    assert r3["bound"] == "alu" and r3["unit"] == "TFLOP/s"
    assert abs(r3["achieved"] - 2e9 / 400e-6 / 1e12) < 1e-3            # 5 TFLOP/s
    assert abs(r3["frac"] - 5.0 / 157.2864) < 1e-5
    assert abs(r3["algorithmic_bytes_GBs"] - (4 * nnz + 4 * rays + 16 * q) / 400e-6 / 1e9) < 0.1
    r3p = bench.roofline_of(per, 1, names, 3, nnz, rays, q, None, None)
    assert abs(r3p["algorithmic_flops_per_launch"] - (2 * nnz + 280 * q)) < 1.0
    assert r3["kernel"] == "k_bp3 (y)" and r3["traffic"] is None
    per2 = {1: {"avg_us": 10.0, "bytes": 5e6}}
    r2 = bench.roofline_of(per2, 1, {1: "k_bp (z)"}, 2, nnz, rays, q, 4e6, None)
    assert r2["bound"] == "hbm" and r2["achieved"] == 500.0 and r2["frac"] == 0.0625
    assert r2["ceilings"]["hbm_counted"]["achieved_GBs"] == 400.0
