"""Host logic of the continuous-batching server, on its host-only simulated
executor (no GPU): arrival-order admission, slot and memory-budget limits,
continuous joining, cancellation, validation, and injected failures that hit
only the requests they concern."""
import time

import pytest

from synth import configs


@pytest.fixture(scope="module")
def pet():
    import os
    import paper_2111_07886_amd as pet
    if not os.path.exists(pet.LIB_PATH):
        from paper_2111_07886_amd import build
        build.build()
    return pet


def req(n=64, M=4, na=None):
    import math
    na = na or max(2 * M, (int(1.125 * n) // M) * M)
    nr = 2 * int(math.ceil(n / math.sqrt(2))) + 3
    return configs.desc_2d(n, na, nr, 300.0 / n, M), configs.params_2d(M, 1e6)


def test_all_complete_with_slot_limit(pet):
    S = pet.Server(1 << 40, 4, simulate=True, step_us=200)
    tickets = []
    for k in range(20):
        d, p = req(64 + 16 * (k % 5), M=4 + (k % 3) * 4)
        tickets.append(S.submit(d, p, n_iter=1 + k % 3))
    res = [S.wait(t) for t in tickets]
    assert all(r["status"] == 0 for r in res)
    st = S.stats()
    assert st["max_active"] <= 4 and st["active"] == 0 and st["queued"] == 0
    # arrival order: admissions are monotone in ticket order
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)
    # continuous batching: some request is admitted before an earlier one finishes
    assert any(res[k]["t_admit"] < res[j]["t_finish"] for j in range(5) for k in range(j + 1, 20))
    for r, (k, t) in zip(res, enumerate(tickets)):
        assert r["subiterations"] == (1 + k % 3) * (4 + (k % 3) * 4)
    S.close()


def test_budget_limits_and_rejects(pet):
    d, p = req(128, M=8)
    # bytes one running request holds, its geometry included
    S = pet.Server(1 << 40, 16, simulate=True, step_us=5000)
    t = S.submit(d, p, n_iter=2)
    while S.stats()["active"] == 0:
        time.sleep(0.001)
    per = S.stats()["bytes_in_use"]
    S.wait(t)
    geo = S.stats()["bytes_in_use"]
    S.close()
    assert 0 < geo < per
    # a budget that fits the geometry and two requests
    S = pet.Server(geo + int(2.5 * (per - geo)), 16, simulate=True, step_us=300)
    ts = [S.submit(d, p, n_iter=2) for _ in range(6)]
    res = [S.wait(t) for t in ts]
    assert all(r["status"] == 0 for r in res)
    assert S.stats()["max_active"] == 2
    big, pb = req(2048, M=8)
    t = S.submit(big, pb, n_iter=1)
    r = S.wait(t)
    assert r["status"] == -4 and "budget" in r["message"]
    S.close()


def test_invalid_requests_rejected_synchronously(pet):
    S = pet.Server(1 << 30, 2, simulate=True)
    d, p = req()
    with pytest.raises(pet.PetOSError) as e:
        S.submit(dict(d, n_subsets=0), p)
    assert e.value.code == -1
    with pytest.raises(pet.PetOSError):
        S.submit(d, dict(p, eps=-1.0))
    with pytest.raises(pet.PetOSError):
        S.submit(d, p, n_iter=0)
    with pytest.raises(pet.PetOSError):
        S.wait(12345)
    S.close()


def test_cancel_queued_and_running(pet):
    S = pet.Server(1 << 40, 1, simulate=True, step_us=2000)
    d, p = req(64, M=4)
    a = S.submit(d, p, n_iter=50)
    b = S.submit(d, p, n_iter=1)
    time.sleep(0.02)
    S.cancel(b)                   # still queued behind a
    S.cancel(a)                   # running
    ra, rb = S.wait(a), S.wait(b)
    assert ra["status"] == -6 and 0 < ra["subiterations"] < 200
    assert rb["status"] == -6 and rb["subiterations"] == 0
    c = S.submit(d, p, n_iter=1)
    assert S.wait(c)["status"] == 0
    S.close()


def test_wait_timeout(pet):
    S = pet.Server(1 << 40, 1, simulate=True, step_us=5000)
    d, p = req(64, M=4)
    t = S.submit(d, p, n_iter=5)
    with pytest.raises(pet.PetOSError) as e:
        S.wait(t, timeout_us=1000)
    assert e.value.code == -6
    assert S.wait(t)["status"] == 0
    S.close()


def test_injected_admission_failure_hits_one_request(pet):
    S = pet.Server(1 << 40, 2, simulate=True, step_us=100)
    S.inject("admit_oom", 1)
    d, p = req(64, M=4)
    ts = [S.submit(d, p, n_iter=1) for _ in range(4)]
    res = [S.wait(t) for t in ts]
    assert [r["status"] for r in res] == [-2, 0, 0, 0]
    S.close()


def test_bad_data_fails_only_its_request(pet):
    """A request whose data fail the admission check of Sec. II-A (here an
    injected r <= 0) ends with INVALID_ARG; requests queued before and after
    it, and those running beside it, complete."""
    S = pet.Server(1 << 40, 2, simulate=True, step_us=500)
    d, p = req(64, M=4)
    a = S.submit(d, p, n_iter=3)
    while S.stats()["active"] == 0:
        time.sleep(0.001)
    S.inject("bad_data", 1)
    ts = [S.submit(d, p, n_iter=1) for _ in range(3)]
    ra = S.wait(a)
    res = [S.wait(t) for t in ts]
    assert ra["status"] == 0 and ra["subiterations"] == 12
    assert [r["status"] for r in res] == [-1, 0, 0]
    assert "r:" in res[0]["message"] and res[0]["subiterations"] == 0
    st = S.stats()
    assert st["active"] == 0 and st["queued"] == 0
    S.close()


def test_injected_step_failure_fails_running_only(pet):
    S = pet.Server(1 << 40, 4, simulate=True, step_us=5000)
    d, p = req(64, M=4)
    first = [S.submit(d, p, n_iter=3) for _ in range(2)]
    time.sleep(0.01)
    S.inject("step_failure", 1)
    res = [S.wait(t) for t in first]
    assert all(r["status"] == -3 for r in res)
    later = [S.submit(d, p, n_iter=1) for _ in range(3)]
    assert all(S.wait(t)["status"] == 0 for t in later)
    S.close()


def test_injected_nan_objective(pet):
    S = pet.Server(1 << 40, 2, simulate=True, step_us=100)
    S.inject("nan_objective", 1)
    d, p = req(64, M=4)
    a = S.submit(d, p, n_iter=1, want_objective=True)
    ra = S.wait(a)
    b = S.submit(d, p, n_iter=1, want_objective=True)
    rb = S.wait(b)
    assert ra["status"] == -5
    assert rb["status"] == 0 and rb["objective"] == -1.0
    S.close()


def test_geometry_cache_reuse_and_eviction(pet):
    S = pet.Server(1 << 40, 2, simulate=True, step_us=50)
    d, p = req(64, M=4)
    for _ in range(3):
        S.wait(S.submit(d, p, n_iter=1))
    assert S.stats()["geometries_cached"] == 1
    d2, p2 = req(80, M=4)
    S.wait(S.submit(d2, p2, n_iter=1))
    assert S.stats()["geometries_cached"] == 2
    S.close()


def req3d(n=32, nz=8, M=4):
    import math
    nr = 2 * int(math.ceil(n / math.sqrt(2))) + 3
    return configs.desc_3d(n, nz, 4 * M, nr, 300.0 / n, 3.0, nz, 3, M), configs.params_3d()


def test_lanes_by_class(pet):
    """2D and 3D requests run in lanes of their own: a 3D request waiting for
    memory does not hold back the 2D requests queued behind it, and each class
    is admitted in its own arrival order."""
    d2, p2 = req(64, M=4)
    d3, p3 = req3d(48, 16)
    S = pet.Server(1 << 40, 16, simulate=True, step_us=2000)
    one2 = S.submit(d2, p2, n_iter=1)
    while S.stats()["active"] == 0:
        time.sleep(0.001)
    per2 = S.stats()["bytes_in_use"]
    S.wait(one2)
    g2 = S.stats()["bytes_in_use"]          # the cached 2D geometry
    r2 = per2 - g2
    t3 = S.submit(d3, p3, n_iter=1)
    while S.stats()["active"] == 0:
        time.sleep(0.001)
    per3 = S.stats()["bytes_in_use"]        # the 3D request, its geometry and the cached 2D one
    S.wait(t3)
    S.close()
    assert per3 > 3 * per2
    # room for the 3D request alone, or for 2D requests, not for the 3D one beside a 2D one
    S = pet.Server(per3 + r2 // 2, 16, simulate=True, step_us=2000)
    a = S.submit(d2, p2, n_iter=20)          # long, holds memory
    b = S.submit(d3, p3, n_iter=1)           # cannot fit until a leaves
    c = S.submit(d2, p2, n_iter=1)           # fits beside a
    ra, rb, rc = S.wait(a), S.wait(b), S.wait(c)
    S.close()
    assert ra["status"] == rc["status"] == 0
    assert rb["status"] == 0
    assert rc["t_admit"] < rb["t_admit"] and rc["t_finish"] < ra["t_finish"]
    assert rb["t_admit"] >= ra["t_finish"] - 1e-3        # b waited for a's memory
