"""Graph capture: sort calls recorded once into a HIP graph and replayed.
Every replay is checked against the oracle on the data the input buffers hold
at that moment; between replays the program does its own eager work (new
input data, other sorts on the same context, synchronizations), and each
replay must still produce the exact result."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1206_3511_amd import intsort as I
from gpu_util import host

pytestmark = pytest.mark.gpu


def _fill(dst: torch.Tensor, a: np.ndarray, stream):
    with torch.cuda.stream(stream):
        dst.copy_(torch.from_numpy(a).to(dst.device, non_blocking=False))
    stream.synchronize()


@pytest.mark.parametrize("algo,n", [("radix", 1_000_003), ("radix", 40_000_000), ("bucket", 1_000_003)])
def test_graph_replays_plain_sort(algo, n):
    print(f"graph plain {algo} n={n}", flush=True)
    s = torch.cuda.Stream()
    keys = torch.empty(n, dtype=torch.uint32, device="cuda:0")
    out = torch.empty_like(keys)
    _fill(keys, workloads.config2_keys(0, n, seed=1), s)
    g = I.capture(lambda: I.sort(keys, algo=algo, out=out), s)
    for rep, dist in enumerate((0, 6, 3, 1)):
        a = workloads.config2_keys(dist, n, seed=10 + rep)
        _fill(keys, a, s)
        # eager work of the program's own between replays, on the same context
        other = torch.from_numpy(workloads.config2_keys(2, 50_000, seed=rep)).to("cuda:0")
        np.testing.assert_array_equal(host(I.sort(other)), np.sort(other.cpu().numpy()))
        g.launch(s)
        s.synchronize()
        np.testing.assert_array_equal(host(out), oracle.radix_lsd(a, r=8).keys)
    assert I.device_error(0, s) == 0
    assert I.device_error(0) == 0
    g.close()


def test_graph_replays_segmented_sort():
    print("graph segmented", flush=True)
    s = torch.cuda.Stream()
    keys_h, offsets = workloads.segmented_keys(num_segments=300, seed=9, lo=16, base=4096)
    keys = torch.from_numpy(keys_h).to("cuda:0")
    offs = torch.from_numpy(offsets.view(np.int64)).to("cuda:0")
    out = torch.empty_like(keys)
    g = I.capture(lambda: I.segmented_sort(keys, offs, out_keys=out), s)
    rng = np.random.default_rng(3)
    for rep in range(3):
        a = rng.integers(0, 1 << 32, keys_h.size, dtype=np.uint64).astype(np.uint32)
        if rep == 1:
            a >>= np.uint32(20)          # a small range: most digit passes skipped
        _fill(keys, a, s)
        g.launch(s)
        s.synchronize()
        ref, _ = oracle.segmented(a, offsets, algo="radix")
        np.testing.assert_array_equal(host(out), ref)
    g.close()


def test_graph_pairs_and_second_graph():
    """Two graphs on one context (a key-value sort and a key sort of another
    size) replayed alternately."""
    print("graph pairs", flush=True)
    s = torch.cuda.Stream()
    n1, n2 = 300_001, 2_000_003
    k1 = torch.empty(n1, dtype=torch.uint64, device="cuda:0")
    v1 = torch.arange(n1, dtype=torch.int32, device="cuda:0").view(torch.uint32)
    ok1, ov1 = torch.empty_like(k1), torch.empty_like(v1)
    k2 = torch.empty(n2, dtype=torch.uint32, device="cuda:0")
    o2 = torch.empty_like(k2)
    _fill(k1, np.zeros(n1, dtype=np.uint64), s)
    _fill(k2, np.zeros(n2, dtype=np.uint32), s)
    g1 = I.capture(lambda: I.sort_pairs(k1, v1, out_keys=ok1, out_vals=ov1), s)
    g2 = I.capture(lambda: I.sort(k2, out=o2), s)
    rng = np.random.default_rng(4)
    for rep in range(2):
        a1 = rng.integers(0, 1 << 40, n1, dtype=np.uint64)
        a1[::3] = a1[1]
        a2 = rng.integers(0, 1 << 32, n2, dtype=np.uint64).astype(np.uint32)
        _fill(k1, a1, s)
        _fill(k2, a2, s)
        g1.launch(s)
        g2.launch(s)
        s.synchronize()
        ref = oracle.radix_lsd(a1, np.arange(n1, dtype=np.uint32), r=8)
        np.testing.assert_array_equal(host(ok1), ref.keys)
        np.testing.assert_array_equal(host(ov1), ref.vals)
        np.testing.assert_array_equal(host(o2), oracle.radix_lsd(a2, r=8).keys)
    g1.close()
    g2.close()
