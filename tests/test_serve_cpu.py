"""Scheduler and admission logic of the evaluation server, on the CPU.

The server runs in dry-run mode: no device work, a batch "takes" its GP
operation count divided by a configured rate, outputs are not written.
That lets the host force the failure paths: over-budget requests, a full
queue, cancellation, time-outs, memory-bounded admission."""
import threading
import time

import numpy as np
import pytest

import paper_1601_00221_amd as gp
import synth

N = 10000
FAKE_X, FAKE_Y, FAKE_OUT = 0x10000, 0x20000, 0x30000   # never dereferenced in dry-run mode


def server(**kw):
    kw.setdefault("dry_run", True)
    s = gp.Server(**kw)
    ds = s.add_dataset(FAKE_X, FAKE_Y, n_feat=4, n_cases=N)
    return s, ds


def job(ds, n_prog=16, seed=0, size=20):
    rng = synth.rng_for(seed)
    pop = synth.ptc2_population(rng, n_prog, synth.BASIC, 4, 3, size, 0.2)
    j = gp.make_job(pop, ds, "mse", None)
    j.out = FAKE_OUT
    return j


def test_single_request_completes():
    s, ds = server(dry_run_gpops=1e10)
    t = s.submit(job(ds))
    assert s.wait(t, 5_000_000) == gp.GP_OK
    assert s.poll(t)
    st = s.stats()
    assert st["completed"] == 1 and st["bytes_in_flight"] == 0 and st["p50_us"] > 0
    s.close()


def test_over_budget_request_is_rejected():
    s, ds = server(memory_budget=4096, dry_run_gpops=1e10)
    rc, _ = s.try_submit(job(ds))
    assert rc == gp.GP_E_NOMEM
    assert "budget" in gp.last_error()
    assert s.stats()["rejected"] == 1
    s.close()


def test_queue_full_and_cancel():
    # 1 GPop/s: the first batch runs for a long time; the queue fills up
    s, ds = server(max_queue=3, n_streams=1, max_batch=1, dry_run_gpops=1e6)
    first = s.submit(job(ds, seed=1))
    time.sleep(0.05)
    queued = [s.submit(job(ds, seed=2 + i)) for i in range(3)]
    rc, _ = s.try_submit(job(ds, seed=9))
    assert rc == gp.GP_E_AGAIN
    assert s.cancel(queued[0]) == gp.GP_OK
    assert s.cancel(first) == gp.GP_E_AGAIN          # already admitted
    assert s.wait(queued[0], 0) != gp.GP_OK           # cancelled tickets do not report success
    assert s.wait(queued[1], 1000) == gp.GP_E_TIMEOUT
    st = s.stats()
    assert st["cancelled"] == 1 and st["queue_depth"] >= 1
    s.close()                                          # cancels the rest, drains the running batch
    assert s._h is None


def test_unknown_dataset_and_bad_program():
    s, ds = server(dry_run_gpops=1e10)
    j = job(ds)
    j.dataset = 7
    rc, _ = s.try_submit(j)
    assert rc == gp.GP_E_NOTFOUND
    bad = gp.make_job(synth.trees_from_lists([(np.array([synth.ADD], np.int32), np.zeros(1, np.float32))]),
                      ds, "mse", None)
    bad.out = FAKE_OUT
    rc, _ = s.try_submit(bad)
    assert rc == gp.GP_E_INVAL
    rc = gp.lib().gp_serve_wait(s._h, 12345, 0)
    assert rc == gp.GP_E_NOTFOUND
    s.close()


def test_memory_bounded_admission_never_exceeds_budget():
    # measure one request's footprint while it runs (1e6 GPop/s: it runs a while)
    probe, dsp = server(dry_run_gpops=1e6)
    tk = probe.submit(job(dsp, seed=0))
    time.sleep(0.02)
    need = probe.stats()["bytes_in_flight"]
    assert need > 0
    probe.close()
    budget = 3 * need + need // 2        # room for three requests, not four
    s, ds = server(memory_budget=budget, n_streams=8, max_batch=64, dry_run_gpops=2e8)
    tickets = [s.submit(job(ds, seed=0)) for i in range(24)]
    peak, peak_q = 0, 0
    while True:
        st = s.stats()
        peak = max(peak, st["bytes_in_flight"])
        peak_q = max(peak_q, st["queue_depth"])
        if st["completed"] == 24:
            break
        time.sleep(0.0005)
    assert peak <= budget
    assert peak >= 2 * need              # admission did run requests side by side
    assert peak_q > 0                    # and held others back
    assert all(s.wait(t, 0) == gp.GP_OK for t in tickets)
    s.close()


def test_continuous_batching_fuses_arrivals():
    s, ds = server(n_streams=2, max_batch=64, dry_run_gpops=5e7)
    tickets = []
    for i in range(40):
        tickets.append(s.submit(job(ds, seed=i)))
    for t in tickets:
        assert s.wait(t, 10_000_000) == gp.GP_OK
    st = s.stats()
    assert st["completed"] == 40
    assert st["mean_batch"] > 1.5          # arrivals during a launch were fused
    s.close()


def test_launch_slots_on_one_hip_stream():
    """Two launch slots sharing one HIP stream (the next batch queued behind
    the running one) complete every request; a negative count is refused."""
    s, ds = server(n_streams=2, hip_streams=1, max_batch=8, dry_run_gpops=5e7)
    tickets = [s.submit(job(ds, seed=i)) for i in range(24)]
    for t in tickets:
        assert s.wait(t, 10_000_000) == gp.GP_OK
    assert s.stats()["completed"] == 24
    s.close()
    with pytest.raises(gp.GPError):
        gp.Server(dry_run=True, hip_streams=-1)


def test_one_launch_per_request_baseline_mode():
    s, ds = server(batching=False, dry_run_gpops=1e9)
    tickets = [s.submit(job(ds, seed=i)) for i in range(6)]
    for t in tickets:
        assert s.wait(t, 10_000_000) == gp.GP_OK
    st = s.stats()
    assert st["batches"] == 6 and st["mean_batch"] == 1.0
    s.close()


def test_concurrent_submitters():
    s, ds = server(dry_run_gpops=1e9)
    errors = []

    def run(k):
        try:
            for i in range(10):
                t = s.submit(job(ds, seed=100 * k + i, n_prog=4))
                if s.wait(t, 10_000_000) != gp.GP_OK:
                    errors.append((k, i))
                s.release(t)
        except Exception as e:  # pragma: no cover
            errors.append(e)

    th = [threading.Thread(target=run, args=(k,)) for k in range(8)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errors
    assert s.stats()["completed"] == 80
    s.close()


def test_release_forgets_finished_tickets():
    s, ds = server(dry_run_gpops=1e10)
    t = s.submit(job(ds))
    assert s.wait(t, -1) == gp.GP_OK
    assert s.release(t) == gp.GP_OK
    assert s.release(t) == gp.GP_E_NOTFOUND
    s.close()
