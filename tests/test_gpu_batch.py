"""GPU parity of batched plans (life_plan_batch, life_sbbnnls_step_batch): the
union of uneven instances sharing one dictionary, checked instance by instance
against the FP64 oracle (normwise relative error <= 1e-5), plus hipGraph replay
and the schedule tuner."""
import numpy as np
import pytest

import oracle
import synth
from conftest import relerr

torch = pytest.importorskip("torch")
from paper_1905_06234_amd import life  # noqa: E402
from test_gpu_parity import _np, _t, dev  # noqa: E402,F401

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _instances():
    b = synth.make_batch(3, seed=5, scale=0.02)
    r = synth.random_coo(96, 1057, 300, 80, 900, seed=11)
    rng = np.random.default_rng(12)
    nf = r.n_fascicles + 5                       # five fascicles that cross no voxel
    r = synth.Connectome(name="r", n_theta=96, n_atoms=1057, n_voxels=r.n_voxels, n_fascicles=nf,
                         atom=r.atom, voxel=r.voxel, fascicle=r.fascicle, phi=r.phi, D=b[0].D,
                         w0=rng.random(nf).astype(np.float32), w_true=rng.random(nf).astype(np.float32),
                         noise=r.noise, grid=r.grid,
                         voxel_xyz=rng.integers(0, 9, (r.n_voxels, 3)).astype(np.int16))
    return b[:2] + [r] + b[2:]


@pytest.fixture(scope="module")
def batch(dev):
    inst = _instances()
    print(f"[batch] {len(inst)} instances, nnz {[c.nnz for c in inst]}", flush=True)
    plan = life.Plan.batch(inst)
    ops = [oracle.Operator.from_connectome(c) for c in inst]
    bs = [oracle.noisy_signal(op, c.w_true, c.noise).astype(np.float32) for op, c in zip(ops, inst)]
    yield inst, ops, plan, bs
    plan.close()


def _split(x, off, width=1):
    return [x[off[k] * width:off[k + 1] * width] for k in range(len(off) - 1)]


def test_batch_dsc_wc_parity(batch, dev):
    inst, ops, plan, _ = batch
    assert plan.n_inst == len(inst)
    rng = np.random.default_rng(41)
    w = [rng.random(c.n_fascicles).astype(np.float32) for c in inst]
    D = _t(inst[0].D, dev)
    y = _np(plan.dsc(D, _t(np.concatenate(w), dev)))
    for k, (op, yk) in enumerate(zip(ops, _split(y, plan.vox_off, 96))):
        assert relerr(yk, op.dsc(w[k])) <= TOL, k
    ys = [rng.standard_normal(96 * c.n_voxels).astype(np.float32) for c in inst]
    g = _np(plan.wc(D, _t(np.concatenate(ys), dev)))
    for k, (op, gk) in enumerate(zip(ops, _split(g, plan.fas_off))):
        assert relerr(gk, op.wc(ys[k])) <= TOL, k


def test_batch_sbb_step_teacher_forced(batch, dev):
    inst, ops, plan, bs = batch
    D, b = _t(inst[0].D, dev), _t(np.concatenate(bs), dev)
    w = [c.w0.astype(np.float32) for c in inst]
    for i in range(4):
        refs = [oracle.sbb_step(op, wk, i, bk) for op, wk, bk in zip(ops, w, bs)]
        wt = _t(np.concatenate(w), dev)
        st = life.new_state(dev, iteration=i, n=len(inst))
        plan.sbbnnls_step_batch(D, b, wt, st)
        got = _split(_np(wt), plan.fas_off)
        for k, ref in enumerate(refs):
            s = life.read_state(st, k)
            assert s["iter"] == i + 1
            assert relerr(got[k], ref.w) <= TOL, (i, k)
            assert abs(s["alpha"] - ref.alpha) <= TOL * ref.alpha, (i, k)
            assert abs(s["obj"] - ref.f) <= TOL * ref.f, (i, k)
        w = [ref.w.astype(np.float32) for ref in refs]


def test_batch_free_running_matches_oracle(batch, dev):
    inst, ops, plan, bs = batch
    D, b = _t(inst[0].D, dev), _t(np.concatenate(bs), dev)
    w = _t(np.concatenate([c.w0 for c in inst]), dev)
    st = life.new_state(dev, n=len(inst))
    f_gpu = []
    for _ in range(10):
        plan.sbbnnls_step_batch(D, b, w, st)
        f_gpu.append([life.read_state(st, k)["obj"] for k in range(len(inst))])
    for k, (op, c, bk) in enumerate(zip(ops, inst, bs)):
        _, hist = oracle.sbb_run(op, c.w0.astype(np.float32), bk, 10)
        f_ref = np.array([h.f for h in hist])
        assert np.max(np.abs(np.array(f_gpu)[:, k] - f_ref) / f_ref) <= 1e-4, k


def test_batch_step_graph_replay_matches_eager(batch, dev):
    """The batched iteration captured once in a hipGraph and replayed: every
    replay equals the eager iteration bitwise (eager work between replays)."""
    inst, ops, plan, bs = batch
    D, b = _t(inst[0].D, dev), _t(np.concatenate(bs), dev)
    w0 = _t(np.concatenate([c.w0 for c in inst]), dev)
    n = len(inst)
    # eager reference trajectory
    w_e, st_e = w0.clone(), life.new_state(dev, n=n)
    eager = []
    for _ in range(5):
        plan.sbbnnls_step_batch(D, b, w_e, st_e)
        torch.cuda.synchronize()
        eager.append((w_e.clone(), st_e.clone()))
    # capture
    w_g, st_g = w0.clone(), life.new_state(dev, n=n)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        w_tmp, st_tmp = w0.clone(), life.new_state(dev, n=n)
        plan.sbbnnls_step_batch(D, b, w_tmp, st_tmp)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.sbbnnls_step_batch(D, b, w_g, st_g)
    torch.cuda.synchronize()
    w_g.copy_(w0)
    st_g.copy_(life.new_state(dev, n=n))
    for i in range(5):
        graph.replay()
        torch.cuda.synchronize()
        _ = (w_g * 2.0).sum().item()           # eager work between replays
        assert torch.equal(w_g, eager[i][0]), i
        assert torch.equal(st_g, eager[i][1]), i


def test_tune_keeps_results(batch, dev):
    inst, ops, plan, _ = batch
    rng = np.random.default_rng(42)
    D = _t(inst[0].D, dev)
    w = _t(rng.random(plan.dims.n_fascicles), dev)
    y = _t(rng.standard_normal(plan.n_signal), dev)
    y0, g0 = plan.dsc(D, w).clone(), plan.wc(D, y).clone()
    pol = plan.tune(D, w, y, reps=2)
    assert pol in (0, 1, 2)
    assert torch.equal(plan.dsc(D, w), y0) and torch.equal(plan.wc(D, y), g0)
