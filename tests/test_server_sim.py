"""The serving runtime's scheduling, admission and failure handling on the CPU
(dry-run executor: no GPU is touched and batches complete after a fixed
delay), through the C ABI."""
import threading
import time

import numpy as np
import pytest

import paper_2411_01919_amd as pp
from paper_2411_01919_amd import _native as N

W, H = 128, 96
K = (100.0, 100.0, 64.0, 48.0)


def _server(**kw):
    cfg = dict(hbm_budget_bytes=64 << 20, max_batch=8, lanes=2, staging_frames=64, dry_run_us=20000)
    cfg.update(kw)
    return pp.Server(**cfg)


def _frame(k=0):
    return np.full((H, W), 1000 + k, np.uint16)


def _open(s, sid=0, w=W, h=H, **rk):
    rc = pp.RansacConfig(max_planes=12, hyps=256, min_inliers=50, **rk)
    s.open_stream(sid, w, h, K, pp.DiffuseConfig(10), rc)


def _drain(s, tickets, sid=0, timeout_s=10.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets) and time.time() - t0 < timeout_s:
        for t in tickets:
            if t in out:
                continue
            r = s.poll(t, sid, timeout_us=2000, labels=False)
            if r is not None:
                out[t] = r
    assert len(out) == len(tickets)
    return out


def _wait_launches(s, n, timeout_s=5.0):
    """Until the scheduler has started n batches (a launch is counted when it starts)."""
    t_end = time.time() + timeout_s
    while s.stats()["launches"] < n and time.time() < t_end:
        time.sleep(0.0005)
    assert s.stats()["launches"] == n


def _frame_bytes():
    # one frame's arena block (inputs, outputs, scratch); read back from the stats of a lone frame
    s = _server()
    _open(s)
    t = s.submit(0, _frame(), 0)
    time.sleep(0.005)
    peak = s.stats()["hbm_peak"]
    _drain(s, [t])
    s.close()
    return peak


def test_admission_respects_the_hbm_budget():
    fb = _frame_bytes()
    assert fb > W * H * 60
    s = _server(hbm_budget_bytes=2 * fb + fb // 2, lanes=4, max_batch=8)
    _open(s)
    ts = [s.submit(0, _frame(k), k) for k in range(10)]
    res = _drain(s, ts)
    st = s.stats()
    assert st["completed"] == 10 and st["hbm_peak"] <= 2 * fb + fb // 2
    assert st["hbm_in_use"] == 0 and st["queued"] == 0
    assert st["mean_batch"] <= 2.0 + 1e-9  # never more than two frames resident
    assert all(r["latency_us"] > 0 for r in res.values())
    s.close()


def test_a_frame_that_can_never_fit_is_rejected_at_open():
    s = _server(hbm_budget_bytes=1 << 20)
    with pytest.raises(pp.PPError) as e:
        _open(s, w=640, h=480)
    assert e.value.status == N.PP_E_BUDGET
    s.close()


def test_backpressure_when_staging_is_full():
    s = _server(staging_frames=3, dry_run_us=50000)
    _open(s)
    ts = [s.submit(0, _frame(k), k) for k in range(3)]
    assert s.try_submit(0, _frame(9), 9) is None
    assert s.stats()["rejected"] == 1
    first = None
    while first is None:
        first = s.poll(ts[0], 0, timeout_us=100000, labels=False)
    assert s.try_submit(0, _frame(10), 10) is not None  # a slot came back with the poll
    s.close()


def test_close_cancels_queued_frames_and_lets_launched_ones_finish():
    fb = _frame_bytes()
    s = _server(hbm_budget_bytes=fb + fb // 2, lanes=1, max_batch=1, dry_run_us=100000)
    _open(s)
    ts = [s.submit(0, _frame(k), k) for k in range(4)]
    _wait_launches(s, 1)  # the first frame is launched, the others wait for memory
    s.close_stream(0)
    with pytest.raises(pp.PPError) as e:
        s.submit(0, _frame(), 99)
    assert e.value.status == N.PP_E_CLOSED
    done = s.poll(ts[0], 0, timeout_us=2_000_000, labels=False)
    assert done is not None and done["frame_id"] == 0
    for t in ts[1:]:
        with pytest.raises(pp.PPError) as e:
            s.poll(t, 0, timeout_us=0, labels=False)
        assert e.value.status == N.PP_E_CLOSED
    assert s.stats()["cancelled"] == 3
    s.close()


def test_frames_arriving_during_a_batch_start_on_another_lane():
    s = _server(lanes=2, dry_run_us=100000)
    _open(s)
    t0 = s.submit(0, _frame(0), 0)
    _wait_launches(s, 1)  # lane 0 is busy with frame 0
    t1 = s.submit(0, _frame(1), 1)
    r1 = s.poll(t1, 0, timeout_us=1_000_000, labels=False)
    r0 = s.poll(t0, 0, timeout_us=1_000_000, labels=False)
    assert r0 is not None and r1 is not None
    # frame 1 did not wait for frame 0's batch to finish
    assert r1["latency_us"] < 170000
    assert s.stats()["launches"] == 2
    s.close()


def test_frames_waiting_together_share_a_batch():
    s = _server(lanes=1, dry_run_us=200000, max_batch=16)
    _open(s)
    frames = [_frame(k) for k in range(9)]
    t0 = s.submit(0, frames[0], 0)
    # frame 0's batch holds the only lane; the rest queue behind it and leave together
    _wait_launches(s, 1)
    ts = [s.submit(0, frames[k], k) for k in range(1, 9)]
    _drain(s, [t0] + ts)
    st = s.stats()
    assert st["launches"] == 2 and abs(st["mean_batch"] - 4.5) < 1e-9
    s.close()


def test_latency_percentiles():
    s = _server(dry_run_us=5000, lanes=4)
    _open(s)
    ts = []
    for k in range(40):
        ts.append(s.submit(0, _frame(k), k))
        time.sleep(0.001)
    res = _drain(s, ts)
    st = s.stats()
    lat = np.array([r["latency_us"] for r in res.values()])
    assert st["completed"] == 40
    assert 0 < st["p50_us"] <= st["p99_us"] <= st["max_us"]
    assert abs(st["max_us"] - lat.max()) < 1.0
    assert st["p50_us"] >= 5000
    s.close()


def test_concurrent_submitters_on_several_streams():
    s = _server(dry_run_us=2000, lanes=3, max_batch=32, staging_frames=128)
    for sid in range(4):
        _open(s, sid)
    results = {}
    errors = []

    def cam(sid):
        try:
            ts = [s.submit(sid, _frame(k), 1000 * sid + k) for k in range(50)]
            results[sid] = _drain(s, ts, sid)
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    th = [threading.Thread(target=cam, args=(sid,)) for sid in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors
    for sid in range(4):
        assert sorted(r["frame_id"] for r in results[sid].values()) == [1000 * sid + k for k in range(50)]
        assert all(r["stream_id"] == sid for r in results[sid].values())
    assert s.stats()["completed"] == 200
    s.close()


def test_invalid_server_calls():
    with pytest.raises(pp.PPError):
        pp.Server(lanes=9, dry_run_us=1000)
    s = _server()
    _open(s)
    with pytest.raises(pp.PPError) as e:
        _open(s)  # stream ids are unique
    assert e.value.status == N.PP_E_INVAL
    h = N.lib()
    res = N.Result()
    assert h.pp_poll(s.h, 12345, res, 0) == N.PP_E_INVAL
    t = N.c_u64()
    assert h.pp_submit(s.h, 77, np.zeros((H, W), np.uint16).ctypes.data, 0, t) == N.PP_E_INVAL
    s.close()


def _poll_status(s, t, sid=0, timeout_s=5.0):
    """The status a ticket's poll ends with (PP_OK or the error)."""
    t_end = time.time() + timeout_s
    while time.time() < t_end:
        try:
            if s.poll(t, sid, timeout_us=2000, labels=False) is not None:
                return N.PP_OK
        except pp.PPError as e:
            return e.status
    raise AssertionError("ticket never finished")


def test_a_failed_batch_poisons_the_server_and_reset_recovers():
    """An executor failure (the third batch, injected in the dry run) fails
    that batch's frames and every frame not yet completed with PP_E_HIP, and
    poisons the server: submits return PP_E_HIP.  pp_server_reset then fails
    what is left, frees the arena, and the server completes new frames."""
    s = _server(max_batch=2, lanes=1, dry_run_us=50000, dry_run_fail_batch=3)  # all 10 queued before it fails
    _open(s)
    ts = [s.submit(0, _frame(k), k) for k in range(10)]
    st = [_poll_status(s, t) for t in ts]
    assert st[:4] == [N.PP_OK] * 4            # batches 1 and 2
    assert all(v == N.PP_E_HIP for v in st[4:])  # batch 3 failed, the rest never ran
    with pytest.raises(pp.PPError) as e:
        s.submit(0, _frame(), 99)
    assert e.value.status == N.PP_E_HIP
    assert "injected failure" in N.lib().pp_server_last_error(s.h).decode()
    s.reset()
    stats = s.stats()
    assert stats["hbm_in_use"] == 0 and stats["queued"] == 0 and stats["in_flight"] == 0
    ts = [s.submit(0, _frame(k), 100 + k) for k in range(5)]
    assert all(_poll_status(s, t) == N.PP_OK for t in ts)
    assert s.stats()["completed"] == 4 + 5
    s.close()


def test_reset_of_a_healthy_server_cancels_unfinished_frames_and_keeps_results():
    """Reset with frames in every state: completed results stay pollable,
    frames queued or on the (simulated) device end with PP_E_CLOSED, and the
    server runs new frames afterwards."""
    s = _server(max_batch=1, lanes=1, dry_run_us=30000)
    _open(s)
    done = s.submit(0, _frame(0), 0)
    t_end = time.time() + 10.0
    while s.stats()["completed"] < 1 and time.time() < t_end:  # the first batch has completed
        time.sleep(0.001)
    assert s.stats()["completed"] == 1
    rest = [s.submit(0, _frame(k), k) for k in range(1, 5)]
    _wait_launches(s, 2)
    s.reset()
    assert _poll_status(s, done) == N.PP_OK
    assert all(_poll_status(s, t) == N.PP_E_CLOSED for t in rest)
    t = s.submit(0, _frame(7), 7)
    assert _poll_status(s, t) == N.PP_OK
    s.close()


def test_failure_injection_needs_the_dry_run():
    with pytest.raises(pp.PPError):
        pp.Server(hbm_budget_bytes=64 << 20, dry_run_us=0, dry_run_fail_batch=1)
    with pytest.raises(pp.PPError):
        pp.Server(hbm_budget_bytes=64 << 20, dry_run_us=100, dry_run_fail_batch=-1)
