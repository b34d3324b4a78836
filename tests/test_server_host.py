"""Serving-loop semantics on the CPU, with the server's dry-run executor (no
GPU work; each batch takes a fixed time per Mpixel and finds no blobs):
admission by footprint, queue limits, batching, tickets and statistics."""
import time

import numpy as np
import pytest

import paper_2010_08486_amd as dog

PRM = dog.Params(1.0, 30.0, 1.6, 0.05, 0.5)


def _frames(n, H=64, W=64):
    return [np.full((H, W), i, np.float32) for i in range(n)]


def test_all_requests_complete_with_latency_stats():
    with dog.Server(PRM, dry_run=True, dry_run_us_per_mpx=2000.0, slots=2, max_batch_frames=4) as sv:
        tickets = [sv.submit(f) for f in _frames(20)]
        sv.drain()
        st = sv.stats()
        assert st["submitted"] == 20 and st["completed"] == 20 and st["failed"] == 0
        assert st["queued"] == 0 and st["running"] == 0 and st["reserved_bytes"] == 0
        assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
        for t in tickets:
            blobs, info = sv.wait(t)
            assert len(blobs) == 0 and info["status"] == 0
            assert info["t_done_ns"] >= info["t_arrive_ns"] > 0
        with pytest.raises(dog.DogError) as e:
            sv.poll(tickets[0])            # already taken
        assert e.value.code == dog.DOG_ENOTFOUND


def test_requests_arriving_while_busy_are_batched():
    # one slot, slow service: a burst queues up behind the first launch and
    # is taken in batches of up to max_batch_frames
    with dog.Server(PRM, dry_run=True, dry_run_us_per_mpx=50000.0, slots=1,
                    max_batch_frames=8) as sv:
        for f in _frames(17, 256, 256):
            sv.submit(f)
        sv.drain()
        st = sv.stats()
        assert st["completed"] == 17
        assert st["batches"] < 17 and st["mean_batch_frames"] > 1.5


def test_poll_is_nonblocking():
    with dog.Server(PRM, dry_run=True, dry_run_us_per_mpx=2e6, slots=1) as sv:
        t = sv.submit(_frames(1, 512, 512)[0])     # ~0.5 s of service
        assert sv.poll(t) is None
        blobs, info = sv.wait(t)
        assert info["status"] == 0


def test_admission_budget_bounds_work_in_flight():
    one = dog.footprint(PRM, [(256, 256)])
    # room for one 256x256 frame at a time, although two slots are idle
    with dog.Server(PRM, dry_run=True, dry_run_us_per_mpx=20000.0, slots=2,
                    hbm_budget_bytes=one + one // 2) as sv:
        for f in _frames(6, 256, 256):
            sv.submit(f)
        sv.drain()
        st = sv.stats()
        assert st["completed"] == 6
        assert st["peak_reserved_bytes"] <= one + one // 2
        assert st["mean_batch_frames"] == 1.0
        with pytest.raises(dog.DogError) as e:
            sv.submit(np.zeros((1024, 1024), np.float32))   # larger than the whole budget
        assert e.value.code == dog.DOG_ENOMEM
        assert sv.stats()["rejected"] == 1


def test_queue_capacity_rejects_with_busy():
    with dog.Server(PRM, dry_run=True, dry_run_us_per_mpx=1e6, slots=1, max_batch_frames=1,
                    queue_capacity=3) as sv:
        codes = []
        for f in _frames(12, 256, 256):
            try:
                sv.submit(f)
                codes.append(0)
            except dog.DogError as e:
                codes.append(e.code)
        assert dog.DOG_EBUSY in codes
        assert codes.count(0) <= 1 + 1 + 3          # running + dispatching + queued
        sv.drain()


def test_batching_window_groups_requests():
    with dog.Server(PRM, dry_run=True, dry_run_us_per_mpx=1000.0, slots=1, max_batch_frames=4,
                    max_wait_ms=200.0) as sv:
        for f in _frames(4):
            sv.submit(f)
        sv.drain()
        st = sv.stats()
        assert st["batches"] == 1 and st["mean_batch_frames"] == 4.0


def test_invalid_server_arguments():
    with pytest.raises(dog.DogError):
        dog.Server(dog.Params(sigma_min=0.0), dry_run=True)
    with dog.Server(PRM, dry_run=True) as sv:
        with pytest.raises(dog.DogError):
            sv.submit(np.zeros((0, 4), np.float32))


def test_pixel_cap_bounds_batch_size():
    # 1024x1024 frames: the default cap of 2^20 pixels gives one frame per
    # batch; a negative cap lets max_batch_frames decide
    with dog.Server(PRM, dry_run=True, dry_run_us_per_mpx=20000.0, slots=1,
                    max_batch_frames=8) as sv:
        for f in _frames(9, 1024, 1024):
            sv.submit(f)
        sv.drain()
        st = sv.stats()
        assert st["completed"] == 9 and st["batches"] == 9
    with dog.Server(PRM, dry_run=True, dry_run_us_per_mpx=20000.0, slots=1,
                    max_batch_frames=8, max_batch_pixels=-1) as sv:
        for f in _frames(9, 1024, 1024):
            sv.submit(f)
        sv.drain()
        st = sv.stats()
        assert st["completed"] == 9 and st["batches"] <= 3
    # a frame larger than the cap still runs, alone
    with dog.Server(PRM, dry_run=True, slots=1, max_batch_pixels=1000) as sv:
        t = sv.submit(_frames(1, 64, 64)[0])
        blobs, info = sv.wait(t)
        assert info["status"] == 0
