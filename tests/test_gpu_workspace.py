"""Caller-owned workspaces and graph capture of the single-problem calls:
life_plan_scratch_bytes, life_dsc_ws / life_wc_ws / life_sbbnnls_step_ws (one
plan serving two streams at once, each with its own scratch), and one
life_sbbnnls_step captured in a hipGraph and replayed.  Every result is compared
bitwise with the same call on the plan's own workspace (same kernels, same
summation orders), and the plan's products with the FP64 oracle."""
import ctypes

import numpy as np
import pytest

from conftest import relerr

torch = pytest.importorskip("torch")
from paper_1905_06234_amd import life  # noqa: E402
from test_gpu_parity import _np, _signal, _t, dev, problem  # noqa: E402,F401

pytestmark = pytest.mark.gpu


def test_scratch_bytes_and_rejects(dev):
    c, op, plan = problem("mid", dev)
    n = plan.scratch_bytes()
    # at least the SBB vectors: two signals and six weight vectors
    assert n >= 4 * (2 * plan.n_signal + 6 * c.n_fascicles)
    D, w = _t(c.D, dev), _t(c.w0, dev)
    y = torch.empty(plan.n_signal, dtype=torch.float32, device=dev)
    small = torch.empty(n - 256, dtype=torch.uint8, device=dev)
    with pytest.raises(life.LifeError) as e:
        plan.dsc(D, w, y, scratch=small)
    assert e.value.status == 1
    big = torch.empty(n + 512, dtype=torch.uint8, device=dev)
    with pytest.raises(life.LifeError) as e:
        plan.dsc(D, w, y, scratch=big[1:n + 1])     # not 256-byte aligned
    assert e.value.status == 1


def test_ws_calls_equal_plan_workspace(dev):
    c, op, plan = problem("mid", dev)
    D, w = _t(c.D, dev), _t(c.w0, dev)
    yv = _t(c.noise, dev)
    scratch = plan.new_scratch(dev)
    scratch.fill_(0xFF)                              # garbage: every region is written before it is read
    y0, y1 = plan.dsc(D, w).clone(), plan.dsc(D, w, scratch=scratch)
    g0, g1 = plan.wc(D, yv).clone(), plan.wc(D, yv, scratch=scratch)
    assert torch.equal(y0, y1) and torch.equal(g0, g1)
    assert relerr(_np(y1), op.dsc(c.w0)) <= 1e-5
    assert relerr(_np(g1), op.wc(c.noise)) <= 1e-5
    b = _t(_signal("mid", op, c), dev)
    wa, wb = w.clone(), w.clone()
    sa, sb = life.new_state(dev), life.new_state(dev)
    for _ in range(3):
        plan.sbbnnls_step(D, b, wa, sa)
        plan.sbbnnls_step(D, b, wb, sb, scratch=scratch)
    assert torch.equal(wa, wb) and torch.equal(sa, sb)


def test_one_plan_two_streams(dev):
    """Two streams run DSC, WC and SBB steps on one plan at the same time, each with
    its own scratch and inputs; every output equals the serial run bitwise."""
    c, op, plan = problem("mid", dev)
    rng = np.random.default_rng(5)
    D = _t(c.D, dev)
    b = _t(_signal("mid", op, c), dev)
    inputs = []
    for k in range(2):
        inputs.append((_t(rng.random(c.n_fascicles), dev), _t(rng.standard_normal(plan.n_signal), dev)))
    # serial reference on the plan's workspace
    ref = []
    for w, yv in inputs:
        ww, st = w.clone(), life.new_state(dev)
        y, g = plan.dsc(D, w).clone(), plan.wc(D, yv).clone()
        for _ in range(4):
            plan.sbbnnls_step(D, b, ww, st)
        ref.append((y, g, ww, st))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    scratch = [plan.new_scratch(dev), plan.new_scratch(dev)]
    outs = []
    for k, (w, yv) in enumerate(inputs):
        outs.append((torch.empty_like(ref[k][0]), torch.empty_like(ref[k][1]), w.clone(), life.new_state(dev)))
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    for rep in range(3):
        # interleave the enqueues so the two streams' kernels overlap on the device
        for k in range(2):
            w, yv = inputs[k]
            y, g, _, _ = outs[k]
            plan.dsc(D, w, y, stream=streams[k], scratch=scratch[k])
            plan.wc(D, yv, g, stream=streams[k], scratch=scratch[k])
        if rep == 0:
            for _ in range(4):
                for k in range(2):
                    _, _, ww, st = outs[k]
                    plan.sbbnnls_step(D, b, ww, st, stream=streams[k], scratch=scratch[k])
    torch.cuda.synchronize()
    for k in range(2):
        for got, want in zip(outs[k], ref[k]):
            assert torch.equal(got, want), k


def test_single_step_graph_replay_matches_eager(dev):
    """One life_sbbnnls_step captured in a hipGraph and replayed five times (the
    parity gate alternates on the device): every replay equals the eager
    iteration bitwise, with eager work and synchronizations between replays."""
    c, op, plan = problem("mid", dev)
    D = _t(c.D, dev)
    b = _t(_signal("mid", op, c), dev)
    w0 = _t(c.w0, dev)
    w_e, st_e = w0.clone(), life.new_state(dev)
    eager = []
    for _ in range(5):
        plan.sbbnnls_step(D, b, w_e, st_e)
        torch.cuda.synchronize()
        eager.append((w_e.clone(), st_e.clone()))
    w_g, st_g = w0.clone(), life.new_state(dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        w_tmp, st_tmp = w0.clone(), life.new_state(dev)
        plan.sbbnnls_step(D, b, w_tmp, st_tmp)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.sbbnnls_step(D, b, w_g, st_g)
    torch.cuda.synchronize()
    w_g.copy_(w0)
    st_g.copy_(life.new_state(dev))
    for i in range(5):
        graph.replay()
        torch.cuda.synchronize()
        _ = (w_g * 2.0).sum().item()
        assert torch.equal(w_g, eager[i][0]), i
        assert torch.equal(st_g, eager[i][1]), i
        assert life.read_state(st_g)["iter"] == i + 1


def test_scratch_symbol_reports_size(dev):
    c, op, plan = problem("tiny", dev)
    n = ctypes.c_uint64()
    assert life.load().life_plan_scratch_bytes(plan._h, ctypes.byref(n)) == 0
    assert n.value == plan.scratch_bytes() and n.value % 256 == 0
    assert life.load().life_plan_scratch_bytes(plan._h, None) == 1
