"""Host logic of the serving loop (no GPU): job shapes and admission."""
import threading

import numpy as np
import pytest

from paper_2410_11184_amd import serve


def test_job_shape():
    assert serve.job_shape(1, 256, 32768) == (1, 128)
    assert serve.job_shape(128, 256, 32768) == (1, 128)
    assert serve.job_shape(129, 256, 32768) == (2, 256)
    assert serve.job_shape(512, 32768, 32768) == (512, 512)
    assert serve.job_shape(3, 32768, 32768) == (4, 4)
    with pytest.raises(ValueError):
        serve.job_shape(1, 100, 32768)
    with pytest.raises(ValueError):
        serve.job_shape(40000, 2, 32768)         # would need more ciphertexts than n


def _server(budget, bytes_per_ct, max_jobs=8):
    s = object.__new__(serve.SoftmaxServer)
    s.slots = 2048
    s.budget = budget
    s.bytes_per_ct = bytes_per_ct
    s.max_jobs = max_jobs
    s.pending = []
    s.in_flight = 0.0
    s.variant = 1
    s.exclusive = 0
    s.softmax_kw = {}
    s.lock = threading.Condition()
    return s


def _req(rid, V, n, M=8.0):
    return serve.Request(rid, np.zeros((V, n)), M, float(rid))


def test_admission_takes_the_oldest_shape_fifo():
    s = _server(budget=100, bytes_per_ct=1)
    s.pending = [_req(0, 10, 16), _req(1, 5, 32), _req(2, 100, 16), _req(3, 1, 16, M=4.0), _req(4, 128, 16)]
    batch, cost = s._admit()
    # shape of request 0: n = 16, m = 1 (10 * 16 <= 2048), M = 8
    assert [r.rid for r in batch] == [0, 2, 4]
    assert cost == 3
    assert [r.rid for r in s.pending] == [1, 3]


def test_admission_respects_the_memory_budget():
    s = _server(budget=10, bytes_per_ct=4)
    s.pending = [_req(i, 10, 16) for i in range(5)]
    batch, cost = s._admit()
    assert len(batch) == 2 and cost == 8          # a third job would exceed 10
    s.in_flight = cost
    batch2, _ = s._admit()
    assert batch2 == []                           # waits for memory while work runs
    s.in_flight = 0
    batch3, _ = s._admit()
    assert len(batch3) == 2


def test_oversized_request_runs_alone_when_idle():
    s = _server(budget=1, bytes_per_ct=4)
    s.pending = [_req(0, 10, 16), _req(1, 10, 16)]
    batch, cost = s._admit()
    assert [r.rid for r in batch] == [0] and cost == 4


def test_latency_stats():
    rs = [_req(i, 1, 16) for i in range(100)]
    for i, r in enumerate(rs):
        r.t_done = r.t_arrival + (i + 1) / 100.0
    st = serve.latency_stats(rs)
    assert abs(st["p50_s"] - 0.505) < 1e-9 and st["max_s"] == 1.0


def test_variant_choice_by_dimension_and_range():
    s = _server(budget=100, bytes_per_ct=1)
    # version B up to n = 16384 while its k (the Theorem's, one more from
    # n = 4096) stays within five squarings; Algorithm SM otherwise
    assert s._variant(256, 128.0) == 1
    assert s._variant(4096, 128.0) == 1          # k = 4 + 1
    assert s._variant(16384, 128.0) == 1         # k = 4 + 1
    assert s._variant(32768, 128.0) == 0         # beyond the dimension bound
    assert s._variant(256, 256.0) == 0           # k = 6
    assert s._variant(16384, 64.0) == 1          # k = 3 + 1
    assert s._variant(8192, 256.0) == 0          # k = 5 + 1
    s.softmax_kw = {"k": 6}                     # a k given by the caller counts
    assert s._variant(256, 128.0) == 0
    s.softmax_kw = {}
    s.variant = 0
    assert s._variant(256, 128.0) == 0
