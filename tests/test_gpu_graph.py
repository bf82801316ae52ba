"""The library's calls only enqueue kernels on the caller's stream (no
allocation, no memset, no synchronisation), so a forward + backward step and
a binary32 forward can be captured into a HIP graph and replayed.  Every
replay, with the program's own eager work and synchronisations between
replays, matches the eager result bitwise, also after new inputs are copied
into the captured buffers."""
import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


def _cols(x, dev, dtype=None):
    import torch
    out = [torch.from_numpy(np.ascontiguousarray(x[:, k])).to(dev) for k in range(x.shape[1])]
    return [t.to(dtype) for t in out] if dtype is not None else out


def test_step_graph_replay():
    import torch

    import paper_2511_00292_amd as eig3
    dev = torch.device("cuda:0")
    n, ns = 4096 + 77, 2048 + 5
    c = w.differentiation_batch(n, seed=61)
    a, g = _cols(c["a"], dev), _cols(c["g"], dev)
    s32 = _cols(w.stress_tensors_f32(ns, seed=62)["s"], dev)
    lam = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3)]
    grad = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(9)]
    l32 = [torch.empty(ns, dtype=torch.float32, device=dev) for _ in range(3)]
    outs = lam + grad + l32

    def step():
        eig3.eig3_eigvals(a, "general", "double_word", "soa", out=lam)
        eig3.eig3_eigvals_backward(a, g, "general", "double_word", out=grad)
        eig3.eig3_eigvals(s32, "symmetric", "double_word", "soa", out=l32)

    def eager():
        step()
        torch.cuda.synchronize()
        return [x.clone() for x in outs]

    ref = eager()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(4):
        for x in outs:
            x.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, (x, r) in enumerate(zip(outs, ref)):
            assert torch.equal(x, r), (rep, k)
    # new inputs in the captured buffers: a replay computes on them
    c2 = w.differentiation_batch(n, seed=63)
    for dst, src in zip(a, _cols(c2["a"], dev)):
        dst.copy_(src)
    for dst, src in zip(g, _cols(c2["g"], dev)):
        dst.copy_(src)
    ref2 = eager()
    for x in outs:
        x.fill_(float("nan"))
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    assert not torch.equal(ref2[0], ref[0])
    for k, (x, r) in enumerate(zip(outs, ref2)):
        assert torch.equal(x, r), ("new inputs", k)
