"""Records of the GPU parity tests: each trajectory and stepwise case appends
one JSON line (errors, the method's own noise spread, the tolerance applied)
to the file named by PET_OS_PARITY_RECORD, when that variable is set."""
import json
import os


def record(kind: str, label: str, **values) -> None:
    path = os.environ.get("PET_OS_PARITY_RECORD")
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "a") as fh:
        fh.write(json.dumps(dict(kind=kind, label=label, **values), sort_keys=True) + "\n")
