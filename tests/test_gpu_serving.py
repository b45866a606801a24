"""GPU tests of the batched sort of separate arrays and of the
continuous-batching server: every result equals the oracle's, and equals
the same request sorted alone (alone-vs-mix, tolerance 0)."""
import time

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1206_3511_amd import intsort as I
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 100, 256, 257, 2048, 2049, 8192, 8193, 16384, 16385, 50_000, 200_003, 0]


def _requests(seed, count, sizes=None):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = sizes[i % len(sizes)] if sizes is not None else int(rng.integers(1, 300_000))
        dist = int(rng.integers(0, 7))
        keys = workloads.config2_keys(dist, n, 5000 + seed * 1000 + i)
        if rng.integers(0, 2):
            keys = (keys.astype(np.uint64) << np.uint64(int(rng.integers(0, 33)))) | keys.astype(np.uint64)
        reqs.append(keys)
    return reqs


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_batched_sort_separate_arrays(dtype):
    arrays = [a.astype(dtype) for a in _requests(1, len(SIZES), SIZES)]
    ins = [dev(a) for a in arrays if a.size]
    outs = I.batched_sort(ins)
    for a, o in zip([a for a in arrays if a.size], outs):
        np.testing.assert_array_equal(host(o), oracle.radix_lsd(a).keys)
    # in place
    ins2 = [dev(a) for a in arrays if a.size]
    I.batched_sort(ins2, outputs=ins2)
    for a, o in zip([a for a in arrays if a.size], ins2):
        np.testing.assert_array_equal(host(o), np.sort(a))


def _serve(reqs, budget, max_batch, slots, spacing_s=0.0):
    srv = I.Server(0, budget_bytes=budget, max_batch=max_batch, slots=slots)
    ins = [dev(a) for a in reqs]
    outs = [torch.empty_like(t) for t in ins]
    torch.cuda.synchronize()
    tickets = []
    for a, b in zip(ins, outs):
        tickets.append(srv.submit(a, b))
        if spacing_s:
            time.sleep(spacing_s)
    srv.drain()
    done = dict(srv.completed())
    assert set(done) == set(tickets)
    assert all(v >= 0 for v in done.values())
    res = [host(o) for o in outs]
    srv.close()
    return res


def test_server_alone_vs_mix_and_oracle():
    reqs = _requests(2, 60)
    mixed = _serve(reqs, budget=16 << 30, max_batch=64, slots=2, spacing_s=0.0005)
    for a, got in zip(reqs, mixed):
        alone = host(I.sort(dev(a)))
        assert got.tobytes() == alone.tobytes()           # alone == in the mix, exactly
        np.testing.assert_array_equal(got, oracle.radix_lsd(a).keys)


def test_server_budget_queueing_and_plain_path():
    reqs = _requests(3, 24, sizes=[100_000, 30_000, 5000])
    # room for about two requests at a time: the rest wait and are admitted
    # as memory frees up
    tight = _serve(reqs, budget=4 << 20, max_batch=16, slots=2)
    plain = _serve(reqs, budget=64 << 30, max_batch=1, slots=1)
    for a, t, p in zip(reqs, tight, plain):
        ref = oracle.radix_lsd(a).keys
        np.testing.assert_array_equal(t, ref)
        np.testing.assert_array_equal(p, ref)


def test_server_rejects_over_budget():
    srv = I.Server(0, budget_bytes=1 << 20, max_batch=4, slots=1)
    a = torch.zeros(1 << 20, dtype=torch.uint32, device="cuda:0")
    with pytest.raises(I.IntsortError) as e:
        srv.submit(a, torch.empty_like(a))
    assert e.value.status == I.ERR_OVER_BUDGET
    srv.close()


def test_server_failed_launch_reports_and_keeps_serving():
    """A batch whose launch fails finishes its requests as failed (poll and
    completed report INTSORT_ERR_HIP, drain reports it once) and the server
    goes on serving: later requests equal the oracle's sort."""
    # one key type: max_batch bounds the arrays of each key type in a batch
    reqs = [workloads.config2_keys(i % 7, n, 9000 + i).astype(np.uint32)
            for i, n in enumerate([3000, 40_000, 1, 17_000] * 2)]
    ins = [dev(a) for a in reqs]
    outs = [torch.zeros_like(t) for t in ins]
    torch.cuda.synchronize()
    # plain path: one request per launch, in arrival order, so the first
    # two launches carry the first two requests
    srv = I.Server(0, budget_bytes=64 << 30, max_batch=1, slots=1)
    srv.fail_next_launches(2)
    tickets = [srv.submit(a, b) for a, b in zip(ins[:5], outs[:5])]
    with pytest.raises(I.IntsortError) as e:
        srv.drain()
    assert e.value.status == I.ERR_HIP
    srv.drain()                                  # reported once: the next drain is clean
    with pytest.raises(I.ServerRequestsFailed) as e:
        srv.completed()
    assert sorted(e.value.tickets) == tickets[:2]
    assert sorted(t for t, _ in e.value.results) == tickets
    assert srv.failed == set(tickets[:2])
    for t in tickets[:2]:                        # forgotten once poll and completed reported them
        with pytest.raises(I.IntsortError) as e:
            srv.poll(t)
        assert e.value.status == I.ERR_INVALID_ARGUMENT
    for o in outs[:2]:                           # an injected failure enqueues nothing
        assert not host(o).any()
    for a, o in zip(reqs[2:5], outs[2:5]):
        np.testing.assert_array_equal(host(o), oracle.radix_lsd(a).keys)
    # the server keeps serving: nothing else fails
    more = [srv.submit(a, b) for a, b in zip(ins[5:], outs[5:])]
    srv.drain()
    assert sorted(t for t, _ in srv.completed()) == more
    for a, o in zip(reqs[5:], outs[5:]):
        np.testing.assert_array_equal(host(o), oracle.radix_lsd(a).keys)
    # a failure while batching fails whole batches, never a request that ran
    srv.close()
    srv = I.Server(0, budget_bytes=64 << 30, max_batch=8, slots=2)
    srv.fail_next_launches(1)
    outs = [torch.zeros_like(t) for t in ins]
    torch.cuda.synchronize()
    tickets = [srv.submit(a, b) for a, b in zip(ins, outs)]
    with pytest.raises(I.IntsortError):
        srv.drain()
    done = srv.completed(raise_on_failure=False)
    assert sorted(t for t, _ in done) == tickets
    assert 1 <= len(srv.failed) <= 8
    for t, a, o in zip(tickets, reqs, outs):
        if t not in srv.failed:
            np.testing.assert_array_equal(host(o), oracle.radix_lsd(a).keys)
    srv.close()


def test_server_submit_from_several_threads():
    """Four host threads submit, poll and collect completions at once (the
    server serialises its calls); every request comes back sorted and every
    ticket is reported by exactly one completed() call."""
    import threading
    srv = I.Server(0, budget_bytes=8 << 30, max_batch=16, slots=2)
    per = 24
    reqs = [[workloads.config2_keys(i % 7, 1000 + 997 * i + 50_000 * t, 700 + 100 * t + i).astype(np.uint32)
             for i in range(per)] for t in range(4)]
    ins = [[dev(a) for a in r] for r in reqs]
    outs = [[torch.empty_like(x) for x in r] for r in ins]
    torch.cuda.synchronize()
    tickets = [[] for _ in range(4)]
    reported = [[] for _ in range(4)]
    errors = []
    # completed() forgets the finished tickets it lists, whichever thread
    # submitted them: every thread polls its own before any collects them
    polled = threading.Barrier(4, timeout=60)

    def work(t):
        try:
            for a, b in zip(ins[t], outs[t]):
                tickets[t].append(srv.submit(a, b))
            for tk in tickets[t]:
                while not srv.poll(tk)[0]:
                    time.sleep(0.0002)
            polled.wait()
            reported[t].extend(tk for tk, _ in srv.completed())
        except Exception as e:   # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert not errors and not any(th.is_alive() for th in threads)
    srv.drain()
    done = [t for r in reported for t in r] + [t for t, _ in srv.completed()]
    allt = [x for r in tickets for x in r]
    assert sorted(done) == sorted(allt) and len(set(allt)) == 4 * per
    for t in range(4):
        for a, o in zip(reqs[t], outs[t]):
            np.testing.assert_array_equal(host(o), np.sort(a))
    srv.close()
