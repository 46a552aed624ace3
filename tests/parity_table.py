"""Tabulate the parity records of a GPU test run (the JSON lines that the
parity tests append to the file named by PET_OS_PARITY_RECORD) as the
Markdown table kept under profiles/.

    python tests/parity_table.py RECORDS.jsonl profiles/parity_trajectories.md "<command>"
"""
import json
import sys


def table(rows, command):
    traj = [r for r in rows if r["kind"] == "trajectory"]
    step = [r for r in rows if r["kind"] == "stepwise"]
    out = ["# GPU parity against the FP64 oracle: trajectories and stepwise cases", "",
           "Written by `tests/parity_table.py` from the records of one GPU test run:", "",
           "```", command, "```", "",
           "Trajectory rule: image rel-L2 tolerance = max(1e-4, 5 x the method's own FP32-noise spread), "
           "asserted where that stays <= 1e-2; objective relative tolerance = max(1e-6, 5 x its spread), "
           "always asserted.  \"face value\" = the stated tolerance applied unchanged.", "",
           "## Trajectories (the configured iterations from f0)", "",
           "| case | iterations | image rel-L2 | image spread | image tol | image | objective rel | "
           "objective spread | objective tol | objective |",
           "|---|---:|---:|---:|---:|---|---:|---:|---:|---|"]
    for r in traj:
        img = ("asserted, face value" if r["image_face_value"] else "asserted, widened") if r["image_asserted"] \
            else "recorded only"
        obj = "face value" if r["objective_face_value"] else "widened"
        out.append(f"| {r['label']} | {r['n_iter']} | {r['image_rel_l2']:.2e} | {r['image_spread']:.2e} | "
                   f"{r['image_tol']:.1e} | {img} | {r['objective_rel']:.2e} | {r['objective_spread']:.2e} | "
                   f"{r['objective_tol']:.1e} | {obj} |")
    n = len(traj)
    n_img = sum(r["image_asserted"] for r in traj)
    n_img_face = sum(r["image_asserted"] and r["image_face_value"] for r in traj)
    n_obj_face = sum(r["objective_face_value"] for r in traj)
    out += ["", f"{n_img} of {n} trajectories have their image asserted ({n_img_face} at the stated 1e-4); "
                f"all {n} their objective ({n_obj_face} at the stated 1e-6).", "",
            "## Stepwise (one GPU subiteration from the oracle's state against one oracle subiteration)", "",
            "| case | samples | worst rel-L2 | tolerance | voxels entering on the upper branch of S | "
            "U - t clamps (oracle / GPU / differing) |",
            "|---|---:|---:|---:|---:|---:|"]
    for r in step:
        clamps = (f"{r['clamp_hi']} / {r.get('clamp_hi_gpu', '–')} / {r.get('clamp_hi_differ', '–')}"
                  if "clamp_hi" in r else "–")
        out.append(f"| {r['label']} | {r['samples']} | {r['worst_rel_l2']:.2e} | {r['tol']:.0e} | "
                   f"{r.get('upper', '–')} | {clamps} |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    rows = [json.loads(l) for l in open(sys.argv[1]) if l.strip()]
    open(sys.argv[2], "w").write(table(rows, sys.argv[3]))
