"""Serving loop on the CPU: queueing, memory-based admission, slots,
continuous batching, failure handling and shutdown rules, driven through the
C ABI with the library's timed fake backend (no GPU)."""
import ctypes as C
import time

import pytest

import paper_1407_2089_amd as vr
from paper_1407_2089_amd.synth import Cam

FAKE = 0x7f0000000000  # never dereferenced: the fake backend renders nothing
CAM = Cam("perspective", (10, 20, 30), (0, 0, -1), (0, 1, 0), 0.8, 1.0, 1.0, 30.0)


def desc():
    return vr.vr_volume_desc(32, 32, 16, 1, 4, vr.VR_U8, 8, (C.c_float * 3)(1, 1, 1),
                             (C.c_float * 3)(0, 0, 0), (C.c_int32 * 3)(0, 0, 0))


@pytest.fixture
def served():
    d = desc()
    need = vr.vr_volume_storage_bytes(d)
    holder = {}

    def make(budget, slots=2, ns_per_ray=0.0, fail_width=-1, max_batch=32, launch_ms=0.0):
        ctx = vr.vr_init(-1, budget + need)
        vol = vr.vr_create_volume(ctx, d, FAKE, need)
        vr.vr_test_fake_backend(ctx, slots, ns_per_ray, fail_width, max_batch, launch_ms)
        holder["ctx"], holder["vol"] = ctx, vol
        return ctx, vol

    yield make
    ctx, vol = holder["ctx"], holder["vol"]
    wait_idle(ctx, holder.get("tickets", []), 30.0)
    vr.vr_destroy_volume(vol)
    vr.vr_shutdown(ctx)


def req(vol, w, h, stereo=True, frame=0):
    return vr.make_request(vol, frame, CAM, w, h, stereo, 1.0, 0.99, FAKE)


def wait(ctx, tickets, timeout=20.0):
    t0 = time.time()
    infos = {}
    for t in tickets:
        while True:
            i = vr.vr_poll(ctx, t)
            if i.state >= 2:
                infos[t] = i
                break
            if time.time() - t0 > timeout:
                raise TimeoutError(f"ticket {t} stuck in state {i.state}")
            time.sleep(0.0005)
    return infos


def wait_idle(ctx, tickets, timeout):
    try:
        wait(ctx, tickets, timeout)
    except Exception:
        pass


OUT = lambda w, h, eyes=2: w * h * eyes * 16  # output bytes the loop accounts


def test_all_tickets_complete_with_ordered_timestamps(served):
    ctx, vol = served(1 << 30, slots=2, ns_per_ray=50.0)
    ts = [vr.vr_submit(ctx, req(vol, 64 + 8 * k, 48)) for k in range(20)]
    infos = wait(ctx, ts)
    for t in ts:
        i = infos[t]
        assert i.state == 2 and i.err == 0
        assert 0 < i.t_arrive_ns <= i.t_admit_ns <= i.t_start_ns <= i.t_done_ns
        assert i.samples == i.rays  # the fake backend composites one sample per ray
    assert infos[ts[3]].rays == (64 + 24) * 48 * 2
    assert len(set(ts)) == 20


def test_start_stamp_is_the_device_span_before_completion(served):
    # a lone 400 x 250 stereo request "runs" 200000 rays x 1000 ns = 200 ms:
    # its start stamp lies that span before its completion stamp
    ctx, vol = served(1 << 30, slots=1, ns_per_ray=1000.0)
    t = vr.vr_submit(ctx, req(vol, 400, 250))
    i = wait(ctx, [t])[t]
    span = i.t_done_ns - i.t_start_ns
    assert 0.2e9 <= span <= 0.2e9 + 0.05e9, span
    assert i.t_admit_ns <= i.t_start_ns


def test_poll_and_submit_do_not_wait_for_a_slow_launch(served):
    # each launch takes 400 ms of the serving thread; meanwhile submit and
    # poll answer at once (the loop does not hold its lock across a launch)
    ctx, vol = served(1 << 30, slots=1, launch_ms=400.0)
    a = vr.vr_submit(ctx, req(vol, 16, 16))
    while vr.vr_poll(ctx, a).state == 0:
        time.sleep(0.0005)
    t0 = time.perf_counter()
    more = []
    for _ in range(20):
        assert vr.vr_poll(ctx, a).state in (1, 2)
        more.append(vr.vr_submit(ctx, req(vol, 16, 16)))
    dt = time.perf_counter() - t0
    assert dt < 0.1, dt
    wait(ctx, [a] + more)


def test_late_arrival_is_admitted_while_first_batch_runs(served):
    # slot 0 is busy for ~300 ms with a big request; a request submitted after
    # it starts gets slot 1 at once and finishes long before the big one.
    ctx, vol = served(1 << 30, slots=2, ns_per_ray=1000.0)
    big = vr.vr_submit(ctx, req(vol, 500, 300))
    while vr.vr_poll(ctx, big).state == 0:
        time.sleep(0.0005)
    late = vr.vr_submit(ctx, req(vol, 10, 10))
    infos = wait(ctx, [big, late])
    assert infos[late].t_admit_ns < infos[big].t_done_ns
    assert infos[late].t_done_ns < infos[big].t_done_ns


def test_memory_budget_serialises_admission(served):
    # the budget holds one 200x100 stereo output at a time: with two free
    # slots the second request must still wait for the first to complete
    ctx, vol = served(OUT(200, 100) + 1000, slots=2, ns_per_ray=2000.0)
    a = vr.vr_submit(ctx, req(vol, 200, 100))
    b = vr.vr_submit(ctx, req(vol, 200, 100))
    infos = wait(ctx, [a, b])
    assert infos[b].t_admit_ns >= infos[a].t_done_ns


def test_request_larger_than_budget_fails_alone(served):
    ctx, vol = served(OUT(100, 100), slots=1, ns_per_ray=10.0)
    big = vr.vr_submit(ctx, req(vol, 200, 200))
    ok = vr.vr_submit(ctx, req(vol, 100, 100))
    infos = wait(ctx, [big, ok])
    assert infos[big].state == 3 and infos[big].err == vr.VR_ERR_OUT_OF_MEMORY
    assert infos[ok].state == 2


def test_failed_batch_marks_its_tickets_and_serving_goes_on(served):
    ctx, vol = served(1 << 30, slots=1, ns_per_ray=100.0, fail_width=13, max_batch=1)
    ts = [vr.vr_submit(ctx, req(vol, w, 20)) for w in (40, 13, 41, 13, 42)]
    infos = wait(ctx, ts)
    states = [infos[t].state for t in ts]
    assert states == [2, 3, 2, 3, 2]
    assert infos[ts[1]].err == vr.VR_ERR_DEVICE
    later = vr.vr_submit(ctx, req(vol, 30, 30))
    assert wait(ctx, [later])[later].state == 2


def test_batches_respect_max_batch(served):
    ctx, vol = served(1 << 30, slots=1, ns_per_ray=3000.0, max_batch=4)
    first = vr.vr_submit(ctx, req(vol, 100, 100))  # occupies the slot ~60 ms
    while vr.vr_poll(ctx, first).state == 0:
        time.sleep(0.0005)
    ts = [vr.vr_submit(ctx, req(vol, 8, 8)) for _ in range(10)]
    infos = wait(ctx, [first] + ts)
    groups = {}
    for t in ts:
        groups.setdefault(infos[t].t_admit_ns, []).append(t)
    sizes = sorted(len(g) for g in groups.values())
    assert sizes == [2, 4, 4]
    assert min(infos[t].t_admit_ns for t in ts) >= infos[first].t_done_ns


def test_queue_full_returns_busy(served):
    ctx, vol = served(1 << 34, slots=1, ns_per_ray=1000.0, max_batch=32)
    block = vr.vr_submit(ctx, req(vol, 600, 500, stereo=False))  # ~300 ms
    while vr.vr_poll(ctx, block).state == 0:
        time.sleep(0.0005)
    ok, busy = [], False
    for _ in range(5000):
        try:
            ok.append(vr.vr_submit(ctx, req(vol, 1, 1, stereo=False)))
        except vr.VrError as e:
            assert e.status == vr.VR_ERR_BUSY
            busy = True
            break
    assert busy and len(ok) >= 4096
    wait(ctx, [block] + ok, 60.0)


def test_ticket_lifecycle_and_shutdown_rules(served):
    ctx, vol = served(1 << 30, slots=1, ns_per_ray=2000.0)
    t = vr.vr_submit(ctx, req(vol, 150, 100))
    with pytest.raises(vr.VrError) as e:
        vr.vr_release(ctx, t)
    assert e.value.status == vr.VR_ERR_BUSY
    with pytest.raises(vr.VrError) as e:
        vr.vr_destroy_volume(vol)
    assert e.value.status == vr.VR_ERR_BUSY
    with pytest.raises(vr.VrError) as e:
        vr.vr_shutdown(ctx)
    assert e.value.status == vr.VR_ERR_BUSY
    wait(ctx, [t])
    vr.vr_release(ctx, t)
    with pytest.raises(vr.VrError) as e:
        vr.vr_poll(ctx, t)
    assert e.value.status == vr.VR_ERR_NOT_FOUND
    with pytest.raises(vr.VrError) as e:
        vr.vr_poll(ctx, 987654321)
    assert e.value.status == vr.VR_ERR_NOT_FOUND


def test_invalid_submission_is_rejected(served):
    ctx, vol = served(1 << 30)
    r = req(vol, 10, 10)
    r.frame = 9
    with pytest.raises(vr.VrError) as e:
        vr.vr_submit(ctx, r)
    assert e.value.status == vr.VR_ERR_INVALID_ARG
