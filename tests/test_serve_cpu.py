"""The serving scheduler on the CPU (fake backend, virtual clock): admission
order and HBM budget, continuous batching, failure isolation."""
import pytest

import paper_2209_08241_amd as bn

PX = 640 * 480
SLOT = ((12 * PX + 255) // 256 * 256 + (PX + 255) // 256 * 256 + 4352)  # device-input slot


def fake(budget, **kw):
    kw.setdefault("fake_ns_per_pixel", 1.0)      # 1 ms per 1 Mpix
    kw.setdefault("fake_launch_ns", 10_000.0)
    return bn.Server(budget, backend="fake", **kw)


def submit_dev(s, H=480, W=640):
    # device-resident input: the fake backend never dereferences it
    return s.submit(0x1000, 500.0, 500.0, W / 2, H / 2, host=False, height=H, width=W)


def states(s, ids):
    return [s.query(i)["state"] for i in ids]


def test_admission_is_fifo_and_bounded_by_budget():
    with fake(3 * SLOT + 100, max_batch=8, max_batches_in_flight=1) as s:
        ids = [submit_dev(s) for _ in range(6)]
        s.progress()
        st = states(s, ids)
        assert st[:3] == [bn.REQ_RUNNING] * 3       # zero-copy inputs are ready at once
        assert st[3:] == [bn.REQ_PENDING] * 3
        assert s.stats()["bytes_in_use"] <= 3 * SLOT + 100
        s.fake_advance(1.0)
        s.progress()
        assert states(s, ids)[:3] == [bn.REQ_DONE] * 3
        assert states(s, ids)[3:] == [bn.REQ_PENDING] * 3   # budget still held
        s.release(ids[0])              # released requests are forgotten
        s.progress()
        assert states(s, ids[3:]) == [bn.REQ_RUNNING, bn.REQ_PENDING, bn.REQ_PENDING]
        for i in ids[1:3]:
            s.release(i)
        s.progress()
        # one launch is in flight (max_batches_in_flight=1): the next two wait, ready
        assert states(s, ids[4:]) == [bn.REQ_READY] * 2
        s.fake_advance(1.0)
        s.progress()
        assert states(s, ids[3:]) == [bn.REQ_DONE, bn.REQ_RUNNING, bn.REQ_RUNNING]
        st = s.stats()
        assert st["peak_bytes_in_use"] <= 3 * SLOT + 100


def test_head_of_line_request_is_not_overtaken():
    big = 13 * 4096 * 3072 + 4608       # one 4096x3072 slot
    with fake(int(1.5 * big), max_batch=8) as s:
        a = submit_dev(s, 3072, 4096)      # takes most of the budget
        b = submit_dev(s, 3072, 4096)      # does not fit next to a
        c = submit_dev(s)                  # small, would fit, but comes after b
        s.progress()
        assert states(s, [a, b, c]) == [bn.REQ_RUNNING, bn.REQ_PENDING, bn.REQ_PENDING]
        s.fake_advance(1.0)
        s.progress()
        s.release(a)
        s.progress()
        assert states(s, [b, c])[0] == bn.REQ_RUNNING


def test_request_larger_than_budget_is_rejected():
    with fake(SLOT) as s:
        with pytest.raises(bn.BnError) as e:
            submit_dev(s, 3072, 4096)
        assert e.value.status == bn.BN_ERR_OOM


def test_continuous_batching_admits_while_running():
    with fake(SLOT * 64, max_batch=4, max_batches_in_flight=1) as s:
        first = [submit_dev(s) for _ in range(3)]
        s.progress()
        assert all(q == bn.REQ_RUNNING for q in states(s, first))
        b1 = s.query(first[0])["batch"]
        # arrivals during the first launch are admitted and queued
        later = [submit_dev(s) for _ in range(6)]
        s.progress()
        assert states(s, later) == [bn.REQ_READY] * 6
        s.fake_advance(0.01)       # first launch: 10 us + 3 * 0.3072 ms
        s.progress()
        assert states(s, first) == [bn.REQ_DONE] * 3
        info = [s.query(i) for i in later]
        assert [x["state"] for x in info[:4]] == [bn.REQ_RUNNING] * 4   # max_batch = 4
        assert [x["state"] for x in info[4:]] == [bn.REQ_READY] * 2
        assert info[0]["batch"] != b1 and info[0]["batch_size"] == 4
        s.fake_advance(0.01)
        s.progress()
        assert states(s, later[4:]) == [bn.REQ_RUNNING] * 2
        s.fake_advance(0.01)
        s.progress()
        assert states(s, later) == [bn.REQ_DONE] * 6
        st = s.stats()
        assert st["batches"] == 3 and st["max_batch_seen"] == 4 and st["completed"] == 9


def test_timestamps_follow_the_virtual_clock():
    with fake(SLOT * 8, max_batch=8, fake_copy_gbs=1.0) as s:
        s.fake_advance(1.0)
        import numpy as np
        rid = s.submit(0x2000, 500.0, 500.0, 320.0, 240.0, host=True, height=480, width=640)
        s.progress()
        assert s.query(rid)["state"] == bn.REQ_ADMITTED       # host input: copy in flight
        s.fake_advance(4 * PX / 1e9 + 1e-9)                     # 1.2 ms at 1 GB/s
        s.progress()
        s.fake_advance(10e-6 + PX * 1e-9 + 1e-9)
        s.progress()
        info = s.query(rid)
        assert info["state"] == bn.REQ_DONE
        assert info["t_submit"] == 1.0 and info["t_admit"] == 1.0
        assert info["t_submit"] <= info["t_launch"] <= info["t_done"]
        assert abs(info["t_done"] - (1.0 + 4 * PX / 1e9 + 10e-6 + PX * 1e-9)) < 1e-6


def test_a_failed_request_does_not_affect_the_others():
    with fake(SLOT * 16, max_batch=8) as s:
        ids = [submit_dev(s) for _ in range(5)]
        s.fake_fail(ids[2])
        s.progress()
        s.fake_advance(1.0)
        s.progress()
        st = states(s, ids)
        assert st[2] == bn.REQ_FAILED
        assert [q for k, q in enumerate(st) if k != 2] == [bn.REQ_DONE] * 4
        assert s.query(ids[2])["status"] == bn.BN_ERR_DEVICE
        for i in ids:
            s.release(i)
        stats = s.stats()
        assert stats["failed"] == 1 and stats["completed"] == 4 and stats["bytes_in_use"] == 0


def test_argument_errors():
    with pytest.raises(bn.BnError):
        bn.Server(0, backend="fake")
    with pytest.raises(bn.BnError):
        bn.Server(SLOT, max_batch=0, backend="fake")
    with fake(SLOT * 4) as s:
        with pytest.raises(bn.BnError):
            s.submit(0x1000, -1.0, 500.0, 1.0, 1.0, host=False, height=4, width=4)
        rid = submit_dev(s)
        with pytest.raises(bn.BnError):       # not done yet
            s.release(rid)
        with pytest.raises(bn.BnError) as e:  # the fake backend is driven by progress()
            s.wait(rid, 0.01)
        assert e.value.status == bn.BN_ERR_UNSUPPORTED
