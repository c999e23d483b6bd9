"""Capture of library calls in a HIP graph.

Every entry point only enqueues kernels on the caller's stream: nothing is
allocated, no memory is set by the runtime and the host never waits inside
a call.  A caller can therefore capture a whole sequence of calls once and
replay it with new inputs copied into the same buffers.  Each test replays
its graph several times, with eager work and synchronisations between the
replays, and checks every replay against the oracle and the eager call."""
import numpy as np
import pytest
import torch

import oracle
from paper_1105_6040_amd import _native as N
from paper_1105_6040_amd import api, inputs

pytestmark = pytest.mark.gpu


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def capture(fn):
    """Run fn once eagerly on a side stream (as torch's graph capture
    expects), then capture it into a graph."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def workspace(op, kt, vals, n, nseg=0):
    return torch.empty(max(1, N.workspace_size(op, kt, vals, n, nseg)), dtype=torch.uint8, device="cuda")


def test_graph_replay_of_paper_method():
    """The paper's 10^5-key method with p = 4 parts (sort_segmented, then
    merge_runs) captured once, replayed for five new inputs."""
    k0, p = inputs.paper_small(0)
    n = k0.size
    toff = api.part_offsets(n, p, "cuda")
    kin = torch.from_numpy(k0).cuda()
    s_out, m_out = torch.empty_like(kin), torch.empty_like(kin)
    ws_s = workspace(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, n, p)
    ws_m = workspace(N.MS_OP_MERGE_RUNS, N.MS_KEY_I32, False, n, p)

    def method():
        api.sort_segmented(kin, toff, keys_out=s_out, ws=ws_s)
        api.merge_runs(s_out, toff, keys_out=m_out, ws=ws_m)

    g = capture(method)
    for r in range(5):
        k = inputs.keys("i32", n, "uniform" if r % 2 == 0 else "few", seed=100 + r)
        kin.copy_(torch.from_numpy(k))
        g.replay()
        got = host(m_out)
        eager = host(api.sort_keys(torch.from_numpy(k).cuda()))
        assert np.array_equal(got, oracle.paper_method(k, p)), r
        assert np.array_equal(got, eager), r


def test_graph_replay_of_pairs_and_segments():
    """A whole-list sort_pairs (decoupled look-back, persistent workgroups,
    atomic tile tickets cleared by a kernel at the start of every call) and
    a segmented sort of many segments, captured in one graph, replayed for
    three new inputs."""
    n = 300_000
    lengths = np.array([0, 5, 70_000, 1, 64, 9_000, 8_192, 40_000, 17, 172_721], dtype=np.int64)
    assert lengths.sum() == n
    off = inputs.offsets_from_lengths(lengths)
    toff = torch.from_numpy(off).cuda()
    kin = torch.empty(n, dtype=torch.uint32, device="cuda")
    vin = torch.from_numpy(np.arange(n, dtype=np.uint32)).cuda()
    ko, vo, so = torch.empty_like(kin), torch.empty_like(vin), torch.empty_like(kin)
    ws_p = workspace(N.MS_OP_SORT_PAIRS, N.MS_KEY_U32, True, n)
    ws_s = workspace(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_U32, False, n, lengths.size)

    def work():
        api.sort_pairs(kin, vin, ko, vo, ws=ws_p)
        api.sort_segmented(kin, toff, keys_out=so, ws=ws_s)

    kin.copy_(torch.from_numpy(inputs.keys("u32", n, "uniform", seed=7)))
    g = capture(work)
    v = np.arange(n, dtype=np.uint32)
    for r in range(3):
        k = inputs.keys("u32", n, ("uniform", "few", "sorted")[r], seed=200 + r)
        kin.copy_(torch.from_numpy(k))
        g.replay()
        ek, ev = oracle.sort(k, v)
        assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), r
        assert np.array_equal(host(so), oracle.sort_segmented(k, off)), r
        api.sort_keys(torch.from_numpy(k).cuda())  # eager work between replays
        torch.cuda.synchronize()
