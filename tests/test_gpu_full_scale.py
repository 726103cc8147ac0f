"""GPU parity at the full synthetic scale (N_theta = 96, N_a = 1057, ~300k voxels,
1.5M fascicles, ~90M nonzeros), with the plan the benchmark times (Morton voxel
order).

Whole outputs are compared with the multi-threaded FP64 oracle (equal, bit for
bit, to the sequential one): DSC and WC vectors, the FP32 adjoint identity, and
SBB-NNLS iterations 0 and 1 teacher-forced from the oracle's iterate (w, alpha,
f and ||g~||^2), all at normwise relative error <= 1e-5.  Samples the oracle
computes one by one (a DSC row y_v needs only the nonzeros of voxel v, a WC
entry g_f only those of fascicle f) check single entries, including the
heaviest voxel and the longest fascicle, and a property that holds at any size
checks one step: every fascicle moves along its own projected gradient with one
common step length, clipped at zero (eqs. 5-8).
"""
import numpy as np
import pytest

import oracle
from conftest import connectome, relerr

torch = pytest.importorskip("torch")
from paper_1905_06234_amd import life  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5
N_SAMPLE = 256


@pytest.fixture(scope="module")
def full():
    life.load()
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    print("[full] generating the full synthetic connectome", flush=True)
    c = connectome("full")
    print(f"[full] nnz={c.nnz}; building the plan", flush=True)
    plan = life.Plan.from_connectome(c)
    yield c, plan, dev
    plan.close()


def _sub(c, mask):
    return oracle.Operator(c.atom[mask], c.voxel[mask], c.fascicle[mask], c.phi[mask], c.D,
                           c.n_voxels, c.n_fascicles)


def _sample(rng, n, extra):
    s = np.unique(np.concatenate([rng.choice(n, size=min(n, N_SAMPLE), replace=False), np.asarray(extra, dtype=np.int64)]))
    return s[(s >= 0) & (s < n)]


def test_full_dsc_sampled(full):
    c, plan, dev = full
    rng = np.random.default_rng(11)
    occ = np.bincount(c.voxel, minlength=c.n_voxels)
    vs = _sample(rng, c.n_voxels, [0, c.n_voxels - 1, int(np.argmax(occ)), int(np.argmin(occ))])
    w = rng.random(c.n_fascicles).astype(np.float32)
    y = plan.dsc(torch.from_numpy(c.D.ravel()).to(dev), torch.from_numpy(w).to(dev))
    torch.cuda.synchronize()
    y = y.cpu().double().numpy().reshape(c.n_voxels, c.n_theta)
    ref = _sub(c, np.isin(c.voxel, vs)).dsc(w).reshape(c.n_voxels, c.n_theta)
    assert relerr(y[vs], ref[vs]) <= TOL
    for v in vs[:32]:                                     # per voxel as well
        assert relerr(y[v], ref[v]) <= TOL or np.abs(ref[v]).max() == 0.0, v


def test_full_wc_sampled(full):
    c, plan, dev = full
    rng = np.random.default_rng(12)
    cnt = np.bincount(c.fascicle, minlength=c.n_fascicles)
    fs = _sample(rng, c.n_fascicles, [0, c.n_fascicles - 1, int(np.argmax(cnt)), int(np.argmin(cnt))])
    y = rng.standard_normal(c.n_theta * c.n_voxels, dtype=np.float32)
    g = plan.wc(torch.from_numpy(c.D.ravel()).to(dev), torch.from_numpy(y).to(dev))
    torch.cuda.synchronize()
    g = g.cpu().double().numpy()
    ref = _sub(c, np.isin(c.fascicle, fs)).wc(y)
    assert relerr(g[fs], ref[fs]) <= TOL
    # a per-fascicle bound scaled by the fascicle's own magnitude sum (cancellation)
    for f in fs[:16]:
        m = c.fascicle == f
        scale = float(np.sum(np.abs(c.phi[m].astype(np.float64)) *
                             np.abs(c.D[c.atom[m]]).astype(np.float64).sum(axis=1) *
                             np.abs(y.reshape(c.n_voxels, c.n_theta)[c.voxel[m]]).max(axis=1)))
        assert abs(g[f] - ref[f]) <= TOL * max(scale, 1e-30), f


def test_full_sbb_step_moves_along_projected_gradient(full):
    c, plan, dev = full
    rng = np.random.default_rng(13)
    b = (np.abs(rng.standard_normal(c.n_theta * c.n_voxels)) * 0.1).astype(np.float32)
    w0 = c.w0.astype(np.float32)
    D = torch.from_numpy(c.D.ravel()).to(dev)
    for it in (0, 1):
        w = torch.from_numpy(w0.copy()).to(dev)
        st = life.new_state(dev, iteration=it)
        plan.sbbnnls_step(D, torch.from_numpy(b).to(dev), w, st)
        s = life.read_state(st)
        w1 = w.cpu().double().numpy()
        assert s["iter"] == it + 1 and np.isfinite(s["alpha"]) and s["alpha"] > 0
        assert np.all(np.isfinite(w1)) and w1.min() >= 0.0
        # oracle gradient on a sample of fascicles: r_v = (M w0 - b)_v on the voxels they cross
        fs = _sample(rng, c.n_fascicles, [])
        fs = fs[np.bincount(c.fascicle, minlength=c.n_fascicles)[fs] > 0][:96]
        vox = np.unique(c.voxel[np.isin(c.fascicle, fs)])
        r = _sub(c, np.isin(c.voxel, vox)).dsc(w0) - b.astype(np.float64)
        g = _sub(c, np.isin(c.fascicle, fs)).wc(r)[fs]
        gt = oracle.projected_gradient(w0[fs].astype(np.float64), g)
        moving = (np.abs(gt) > 0) & (w1[fs] > 0)
        assert moving.sum() >= 8
        a = (w0[fs][moving] - w1[fs][moving]) / gt[moving]
        alpha = float(np.median(a))
        expect = np.maximum(0.0, w0[fs] - alpha * gt)
        bound = TOL * (np.abs(w0[fs]) + np.abs(alpha * gt)) + 1e-30
        assert np.all(np.abs(w1[fs] - expect) <= bound), it
        assert abs(alpha - s["alpha"]) <= 1e-3 * s["alpha"], (alpha, s["alpha"])
        still = gt == 0
        assert np.array_equal(w1[fs][still], w0[fs][still].astype(np.float64))


# ----------------------------------------------------------------------------- whole outputs

@pytest.fixture(scope="module")
def full_ref(full):
    c, plan, dev = full
    print("[full] grouping the nonzeros for the multi-threaded oracle", flush=True)
    op = oracle.Operator.from_connectome(c)
    par = op.parallel()
    print(f"[full] oracle ready ({oracle.par_threads()} threads)", flush=True)
    yield op, par
    par.close()


def _np(t):
    return t.detach().cpu().double().numpy()


def test_full_dsc_whole(full, full_ref):
    c, plan, dev = full
    _, par = full_ref
    D = torch.from_numpy(c.D.ravel()).to(dev)
    rng = np.random.default_rng(21)
    signed = rng.standard_normal(c.n_fascicles).astype(np.float32)
    for label, w in (("w0", c.w0), ("signed", signed)):
        y = plan.dsc(D, torch.from_numpy(np.ascontiguousarray(w)).to(dev))
        err = relerr(_np(y), par.dsc(w))
        print(f"[full] DSC {label}: normwise relative error {err:.3e}", flush=True)
        assert err <= TOL, label


def test_full_wc_whole(full, full_ref):
    c, plan, dev = full
    _, par = full_ref
    D = torch.from_numpy(c.D.ravel()).to(dev)
    g = plan.wc(D, torch.from_numpy(c.noise).to(dev))
    err = relerr(_np(g), par.wc(c.noise))
    print(f"[full] WC: normwise relative error {err:.3e}", flush=True)
    assert err <= TOL


def test_full_adjoint_identity_fp32(full):
    """<M w, y> = <w, M^T y> for the device products on the whole operator, relative
    to |<M w, y>| (random-sign y: the sums cancel, so a rounding bias in either product
    shows), and <w, M^T (M w)> = ||M w||^2."""
    c, plan, dev = full
    D = torch.from_numpy(c.D.ravel()).to(dev)
    w = torch.from_numpy(c.w0).to(dev)
    y = torch.from_numpy(c.noise).to(dev)
    mw = plan.dsc(D, w)
    lhs = float(_np(mw) @ _np(y))
    rhs = float(_np(w) @ _np(plan.wc(D, y)))
    print(f"[full] adjoint residual {abs(lhs - rhs) / abs(lhs):.3e}", flush=True)
    assert abs(lhs - rhs) <= TOL * abs(lhs)
    n2, rhs2 = float(_np(mw) @ _np(mw)), float(_np(w) @ _np(plan.wc(D, mw)))
    print(f"[full] ||Mw||^2 residual {abs(n2 - rhs2) / n2:.3e}", flush=True)
    assert abs(n2 - rhs2) <= TOL * n2


def test_full_sbb_steps_teacher_forced(full, full_ref):
    """Iterations 0 (even: second WC, alpha = <v',v'>/<v'',v''>) and 1 (odd: alpha =
    <g~,g~>/<v',v'>) of Algorithm 1 on the whole problem, each from the oracle's own
    iterate, against oracle.sbb_step on b = M w_true + 5% noise."""
    c, plan, dev = full
    _, par = full_ref
    b32 = oracle.noisy_signal(par, c.w_true, c.noise).astype(np.float32)
    D = torch.from_numpy(c.D.ravel()).to(dev)
    b = torch.from_numpy(b32).to(dev)
    w = c.w0.astype(np.float32)
    for i in (0, 1):
        ref = oracle.sbb_step(par, w, i, b32)
        wt = torch.from_numpy(w.copy()).to(dev)
        st = life.new_state(dev, iteration=i)
        plan.sbbnnls_step(D, b, wt, st)
        s = life.read_state(st)
        errs = {"w": relerr(_np(wt), ref.w), "alpha": abs(s["alpha"] - ref.alpha) / ref.alpha,
                "f": abs(s["obj"] - ref.f) / ref.f, "gt2": abs(s["gt_norm2"] - ref.gt_norm2) / ref.gt_norm2,
                "num": abs(s["num"] - ref.num) / ref.num, "den": abs(s["den"] - ref.den) / ref.den}
        print(f"[full] SBB step {i}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
        assert s["iter"] == i + 1
        assert all(v <= TOL for v in errs.values()), (i, errs)
        w = ref.w.astype(np.float32)


def test_full_device_plan_equals_host_plan(full):
    """The plan the benchmark times (built on the device) equals, array for array,
    the host builder's plan of the full connectome."""
    import time
    c, plan, dev = full
    t0 = time.perf_counter()
    host = life.Plan.build(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, c.fascicle, c.phi,
                           voxel_xyz=c.voxel_xyz, host_build=True)
    t_host = time.perf_counter() - t0
    t0 = time.perf_counter()
    again = life.Plan.from_connectome(c)
    t_dev = time.perf_counter() - t0
    print(f"[full] plan: device builder {t_dev:.3f} s, host builder {t_host:.3f} s", flush=True)
    dh, dp = host.digest(), plan.digest()
    assert np.array_equal(dp, dh), np.nonzero(dp != dh)[0]
    assert np.array_equal(again.digest(), dh)
    host.close()
    again.close()
