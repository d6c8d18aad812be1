"""Admission policy of the serving loop, replayed on the host
(cnmf_server_simulate runs the server's own BlockArena and pick_admission
code without a GPU)."""
import numpy as np
import pytest

from paper_1505_04650_amd import _lib as L

torch = pytest.importorskip("torch")

api = pytest.importorskip("paper_1505_04650_amd.api")

G = 256  # arena granule


def rnd(b):
    return (np.asarray(b, dtype=np.int64) + G - 1) // G * G


def _check_invariants(arr, nbytes, svc, budget, max_inflight, adm, done, peak):
    n = len(arr)
    rb = rnd(np.maximum(nbytes, 1))
    for i in range(n):
        if rb[i] > budget // G * G:
            assert adm[i] == -1 and done[i] == -1
            continue
        assert adm[i] >= arr[i] - 1e-12
        assert abs(done[i] - (adm[i] + svc[i])) < 1e-9
    ok = adm >= 0
    # at every admission instant: concurrency and memory within bounds
    for t in np.unique(adm[ok]):
        live = ok & (adm <= t) & (done > t)
        assert live.sum() <= max_inflight
        assert rb[live].sum() <= budget
    assert peak <= budget


def test_random_load_respects_budget_and_slots():
    g = np.random.default_rng(0)
    n = 400
    arr = np.cumsum(g.exponential(0.5, n))
    nbytes = (g.lognormal(16, 1.0, n)).astype(np.uint64)
    svc = g.uniform(1, 20, n)
    budget = int(np.sort(nbytes)[-1] * 3)
    adm, done, peak = api.simulate_admission(arr, nbytes, svc, budget, 16)
    _check_invariants(arr, nbytes.astype(np.int64), svc, budget, 16, adm, done, peak)
    assert (adm >= 0).all()
    assert peak > budget // 3   # the arena is actually used


def test_oversized_request_is_rejected_others_run():
    arr = np.array([0.0, 1.0, 2.0])
    nbytes = np.array([1000, 10 ** 9, 1000], dtype=np.uint64)
    svc = np.array([5.0, 5.0, 5.0])
    adm, done, peak = api.simulate_admission(arr, nbytes, svc, 10 ** 6, 4)
    assert adm[1] == -1 and done[1] == -1
    assert adm[0] == 0.0 and adm[2] == 2.0


def test_fifo_when_everything_fits():
    g = np.random.default_rng(1)
    n = 200
    arr = np.cumsum(g.exponential(1.0, n))
    nbytes = np.full(n, 4096, dtype=np.uint64)
    svc = g.uniform(5, 30, n)
    adm, done, _ = api.simulate_admission(arr, nbytes, svc, 1 << 30, 8)
    # slots are the only limit: admission order is arrival order
    assert np.all(np.diff(adm) >= -1e-12)


def test_large_head_is_not_starved_by_small_requests():
    # budget 100 units; a stream of small requests (10 units, 10 ms each)
    # arriving every 1 ms keeps the arena busy; a 90-unit request arriving
    # at t = 5 must be admitted once the running small ones drain
    U = 1 << 20
    small_t = np.arange(0.0, 200.0, 1.0)
    arr = np.sort(np.concatenate([small_t, [5.0]]))
    big = int(np.searchsorted(arr, 5.0, side="right")) - 1
    nbytes = np.full(len(arr), 10 * U, dtype=np.uint64)
    nbytes[big] = 90 * U
    svc = np.full(len(arr), 10.0)
    adm, done, peak = api.simulate_admission(arr, nbytes, svc, 100 * U, 64)
    _check_invariants(arr, nbytes.astype(np.int64), svc, 100 * U, 64, adm, done, peak)
    # small requests may pass it only while the head stays covered, so it
    # waits at most one service time of what was already running
    assert adm[big] <= 5.0 + 10.0 + 1e-9
    # it did wait (the arena was busy) and others were admitted meanwhile
    assert adm[big] > 5.0


def test_bypass_is_bounded():
    # a head that can never be covered while others keep arriving would let
    # at most 64 later requests pass before the queue waits for it
    U = 1 << 20
    n = 300
    arr = np.arange(n, dtype=np.float64) * 0.1
    nbytes = np.full(n, 1 * U, dtype=np.uint64)
    nbytes[0] = 60 * U
    nbytes[1] = 50 * U          # running first...
    arr[0], arr[1] = 0.05, 0.0  # ...so the 60-unit request waits behind it
    order = np.argsort(arr, kind="stable")
    arr, nbytes = arr[order], nbytes[order]
    svc = np.full(n, 1000.0)
    adm, done, peak = api.simulate_admission(arr, nbytes, svc, 100 * U, 1000)
    head = int(np.where(nbytes == 60 * U)[0][0])
    passed = np.sum((adm >= 0) & (adm < adm[head]) & (np.arange(n) > head))
    assert passed <= 64
    _check_invariants(arr, nbytes.astype(np.int64), svc, 100 * U, 1000, adm, done, peak)


def test_simulate_argument_checks():
    lib = L.load()
    assert api.simulate_admission([], [], [], 1 << 20, 4)[2] == 0
    with pytest.raises(L.CnmfError):
        api.simulate_admission([1.0, 0.0], [1, 1], [1.0, 1.0], 1 << 20, 4)  # unsorted
    with pytest.raises(L.CnmfError):
        api.simulate_admission([0.0], [1], [1.0], 1 << 20, 0)
    assert lib.cnmf_server_last_error()
