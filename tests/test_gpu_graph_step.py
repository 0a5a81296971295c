"""The overlapped c2 step, and its build + merge part, each captured as one
HIP graph: every replay must write exactly what an eager run writes, with
eager runs and synchronisations between the replays (the bench times these
replays)."""
import pytest
import torch

import bench
from helpers import say


@pytest.mark.gpu
@pytest.mark.parametrize("workload", ["c2"])  # the step's index needs 64-bit keys
def test_step_graph_replays_match_eager(gpu, workload):
    say("graph step", workload)
    d = bench.make_workload(workload)
    pipe = bench.Pipeline(gpu, d, torch.device("cuda:0"))
    pipe.step()
    torch.cuda.synchronize()
    pipe.check()
    pipe.nu = int(pipe.cnt[2].item())
    pipe.make_lookups()
    pipe.step_concurrent()
    torch.cuda.synchronize()
    want = bench.step_outputs(pipe)
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=cap):
        pipe.step_concurrent()
    torch.cuda.synchronize()
    for r in range(4):
        # scribble over the outputs so that a replay that writes nothing fails
        for t in (pipe.m, *pipe.p, pipe.idx, pipe.d2, pipe.lrank, pipe.brank):
            t.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        got = bench.step_outputs(pipe)
        for i, (a, b) in enumerate(zip(got, want)):
            assert torch.equal(a, b), (workload, r, i)
        pipe.check()
        pipe.step()  # eager work between replays
        torch.cuda.synchronize()
    assert torch.equal(pipe.lrank, pipe.brank) and torch.equal(pipe.lfound, pipe.bfound)


@pytest.mark.gpu
def test_build_merge_graph_replays_match_eager(gpu):
    say("graph build+merge c2")
    d = bench.make_workload("c2")
    pipe = bench.Pipeline(gpu, d, torch.device("cuda:0"))
    pipe.build_merge_concurrent()
    torch.cuda.synchronize()
    pipe.check()
    want = bench.step_outputs(pipe, full=False)
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=cap):
        pipe.build_merge_concurrent()
    torch.cuda.synchronize()
    for r in range(4):
        for t in (pipe.ka, pipe.kb, pipe.ca, pipe.cb, pipe.m, pipe.cnt):
            t.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        got = bench.step_outputs(pipe, full=False)
        for i, (a, b) in enumerate(zip(got, want)):
            assert torch.equal(a, b), (r, i)
        pipe.check()
        pipe.build_merge()  # eager work between replays
        torch.cuda.synchronize()
