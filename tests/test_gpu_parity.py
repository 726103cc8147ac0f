"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bar: normwise relative error <= 1e-5 for every float32 output (DSC, WC, one
SBB-NNLS iteration teacher-forced from the oracle's iterate); plans bit-exact;
repeated calls bitwise identical.
"""
import zlib

import numpy as np
import pytest

import oracle
import synth
from conftest import connectome, reference_plan, relerr

torch = pytest.importorskip("torch")
from paper_1905_06234_amd import life  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5

# (n_theta, n_atoms, n_voxels, n_fascicles, nnz, duplicates): ragged shapes around the
# 32-lane theta slices, several blocks, tails, duplicates, empty segments
RANDOM_SHAPES = {
    "r1": (1, 3, 50, 40, 600, False),
    "r5dup": (5, 7, 33, 29, 1000, True),
    "r33": (33, 9, 70, 100, 3000, False),
    "r100": (100, 40, 64, 64, 5000, True),
    "r129": (129, 17, 20, 300, 2000, False),
    "r96big": (96, 1057, 4000, 3000, 200_000, False),
    "empty": (16, 64, 512, 200, 0, False),
    "sparsevox": (64, 20, 20_000, 50, 700, False),
    # one chunk, one atom tile, hundreds of nonzeros per voxel: long runs of one
    # (atom, voxel) pair in the WC buckets and a chunk fascicle list of thousands
    "dense96": (96, 200, 64, 5000, 30_000, True),
    "dense16": (16, 512, 64, 3000, 20_000, False),
    # one chunk over 4 atom tiles, thousands of fascicles: a long WC bucket per
    # (chunk, tile) and a fascicle list near the chunk's LDS capacity
    "dense96t": (96, 1057, 64, 8000, 40_000, False),
}


@pytest.fixture(scope="module")
def dev():
    life.load()
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32).ravel())).to(dev)


def _np(t):
    return t.detach().cpu().double().numpy()


_problems = {}
_xyz = {}


def problem(name, dev):
    """(connectome, oracle operator, device plan) of a named case.  The synthetic
    connectomes are planned with their voxel coordinates (Morton order); "<name>@id"
    plans them in voxel index order; "<random shape>@xyz" gives the random COO case
    random grid coordinates (with repeats, so ties occur)."""
    if name not in _problems:
        base, _, variant = name.partition("@")
        xyz = None
        if base in ("tiny", "mid"):
            c = connectome(base)
            xyz = None if variant == "id" else c.voxel_xyz
        else:
            nt, na, nv, nf, nnz, dup = RANDOM_SHAPES[base]
            c = synth.random_coo(nt, na, nv, nf, nnz, seed=zlib.crc32(base.encode()) % 1000, duplicates=dup)
            if variant == "xyz":
                rng = np.random.default_rng(zlib.crc32(name.encode()))
                xyz = rng.integers(0, 2 * round(nv ** (1 / 3)) + 2, size=(nv, 3)).astype(np.int16)
        print(f"[parity] building plan for {name}: nnz={c.nnz}", flush=True)
        plan = life.Plan(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, c.fascicle, c.phi,
                         voxel_xyz=xyz)
        _problems[name] = (c, oracle.Operator.from_connectome(c), plan)
        _xyz[name] = xyz
    return _problems[name]


ALL = ["tiny", "mid", "tiny@id", "mid@id"] + list(RANDOM_SHAPES) + ["r33@xyz", "r96big@xyz", "sparsevox@xyz"]


@pytest.mark.parametrize("name", ALL)
def test_dsc_parity(name, dev):
    c, op, plan = problem(name, dev)
    D = _t(c.D, dev)
    for label, w in (("dense", c.w0), ("sparse", np.where(np.arange(c.n_fascicles) % 3 == 1, 0.0, c.w0))):
        y = plan.dsc(D, _t(w, dev))
        ref = op.dsc(np.asarray(w, np.float32))
        assert relerr(_np(y), ref) <= TOL, (name, label)


@pytest.mark.parametrize("name", ["tiny", "mid", "r5dup", "r100", "r96big", "dense96", "dense16", "sparsevox"])
def test_dsc_zero_weight_skip(name, dev):
    """DSC with mostly-zero weights (the zero-weight skip compacts each batch's
    nonzero products): random 90% and 99% zeros, a contiguous half of the
    fascicles zero, negative zeros, and all zeros (y must then be exactly 0)."""
    c, op, plan = problem(name, dev)
    D = _t(c.D, dev)
    rng = np.random.default_rng(17)
    nf = c.n_fascicles
    pats = {
        "90%": np.where(rng.random(nf) < 0.9, 0.0, c.w0),
        "99%": np.where(rng.random(nf) < 0.99, 0.0, c.w0),
        "half": np.where(np.arange(nf) < nf // 2, 0.0, c.w0),
        "-0": np.where(rng.random(nf) < 0.7, -0.0, c.w0),
    }
    for label, w in pats.items():
        w = np.asarray(w, np.float32)
        y = plan.dsc(D, _t(w, dev))
        ref = op.dsc(w)
        if np.abs(ref).max() == 0:
            assert np.all(_np(y) == 0), (name, label)
        else:
            assert relerr(_np(y), ref) <= TOL, (name, label)
        assert torch.equal(plan.dsc(D, _t(w, dev)), y), (name, label)   # bitwise repeatable
    y0 = plan.dsc(D, torch.zeros(nf, device=dev))
    assert torch.count_nonzero(y0).item() == 0


@pytest.mark.parametrize("name", ALL)
def test_wc_parity(name, dev):
    c, op, plan = problem(name, dev)
    D = _t(c.D, dev)
    g = plan.wc(D, _t(c.noise, dev))
    assert relerr(_np(g), op.wc(c.noise)) <= TOL, name


@pytest.mark.parametrize("name", ["tiny", "mid", "r100", "r96big"])
def test_adjoint_identity_fp32(name, dev):
    """<M w, y> = <w, M^T y> for the device DSC and WC, relative to |<M w, y>| (a
    random-sign y: the sums cancel, so a rounding bias in either product shows), and
    <w, M^T (M w)> = ||M w||^2."""
    c, op, plan = problem(name, dev)
    D = _t(c.D, dev)
    w = _t(c.w0, dev)
    y = _t(c.noise, dev)
    mw = plan.dsc(D, w)
    lhs = float(_np(mw) @ _np(y))
    rhs = float(_np(w) @ _np(plan.wc(D, y)))
    assert abs(lhs - rhs) <= TOL * abs(lhs)
    n2, rhs2 = float(_np(mw) @ _np(mw)), float(_np(w) @ _np(plan.wc(D, mw)))
    assert abs(n2 - rhs2) <= TOL * n2


@pytest.mark.parametrize("name", ["mid", "r5dup"])
def test_bitwise_deterministic(name, dev):
    c, op, plan = problem(name, dev)
    D, w, y = _t(c.D, dev), _t(c.w0, dev), _t(c.noise, dev)
    a1, a2 = plan.dsc(D, w), plan.dsc(D, w)
    b1, b2 = plan.wc(D, y), plan.wc(D, y)
    assert torch.equal(a1, a2) and torch.equal(b1, b2)


def test_interleaved_calls_on_one_plan(dev):
    """DSC and WC calls on one plan (one workspace) in any order give the results
    of calls on a fresh plan."""
    c, op, plan = problem("mid", dev)
    D, w, y = _t(c.D, dev), _t(c.w0, dev), _t(c.noise, dev)
    a1 = plan.dsc(D, w)
    b1 = plan.wc(D, y)
    a2 = plan.dsc(D, w)
    b2 = plan.wc(D, y)
    b3 = plan.wc(D, y)
    a3 = plan.dsc(D, y[:c.n_fascicles].abs())
    assert torch.equal(a1, a2) and torch.equal(b1, b2) and torch.equal(b2, b3)
    assert relerr(_np(a3), op.dsc(np.abs(c.noise[:c.n_fascicles]).astype(np.float32))) <= TOL


@pytest.mark.parametrize("name", ["mid", "r129", "empty"])
def test_profile_counts_launches(name, dev):
    c, op, plan = problem(name, dev)
    D, w, y = _t(c.D, dev), _t(c.w0, dev), _t(c.noise, dev)
    plan.profile_read()
    plan.profile_enable(True)
    plan.dsc(D, w)
    plan.wc(D, y)
    torch.cuda.synchronize()
    plan.profile_enable(False)
    ms, cnt = plan.profile_read()
    launched = 1 if c.nnz > 0 else 0
    # life_dsc first gathers w into the plan's fascicle (rank) order
    assert cnt["permute"] == 1 and cnt["dsc"] == 1, cnt
    assert cnt["wc_z"] == launched and cnt["wc_sum"] == 1, cnt
    assert all(v >= 0.0 for v in ms.values()) and sum(cnt.values()) == 3 + launched


def test_outputs_overwritten(dev):
    c, op, plan = problem("sparsevox", dev)
    D = _t(c.D, dev)
    y = torch.full((c.n_theta * c.n_voxels,), float("nan"), device=dev)
    plan.dsc(D, _t(c.w0, dev), y)
    yn = _np(y)
    assert np.isfinite(yn).all()
    empty = np.bincount(c.voxel, minlength=c.n_voxels) == 0
    assert empty.any() and np.all(yn.reshape(c.n_voxels, c.n_theta)[empty] == 0)
    g = torch.full((c.n_fascicles,), float("nan"), device=dev)
    plan.wc(D, _t(c.noise, dev), g)
    assert np.isfinite(_np(g)).all()


@pytest.mark.parametrize("name", ["tiny", "tiny@id", "r5dup", "r129", "r33@xyz"])
def test_device_plan_bit_exact(name, dev):
    c, op, plan = problem(name, dev)
    ex = plan.export()
    ref = reference_plan(c, _xyz[name])
    dsc = ref["dsc_perm"]
    assert np.array_equal(ex["vox_ptr"], ref["vox_ptr"])
    assert np.array_equal(ex["atom_v"], c.atom[dsc])
    assert np.array_equal(ex["fas_v"], ref["fas_rank"][c.fascicle[dsc]])
    assert np.array_equal(ex["phi_v"].view(np.uint32), c.phi[dsc].view(np.uint32))
    assert np.array_equal(ex["fas_rank"], ref["fas_rank"])
    assert np.array_equal(ex["fas_ptr"], ref["fas_ptr"])
    assert np.array_equal(ex["wc_perm"], ref["wc_perm"])


# ----------------------------------------------------------------------------- SBB-NNLS

_signals = {}


def _signal(name, op, c):
    if name not in _signals:
        _signals[name] = oracle.noisy_signal(op, c.w_true, c.noise).astype(np.float32)
    return _signals[name]


def _gpu_step(plan, D, b, w_np, i, dev):
    w = _t(w_np, dev)
    st = life.new_state(dev, iteration=i)
    plan.sbbnnls_step(D, b, w, st)
    return _np(w), life.read_state(st)


@pytest.mark.parametrize("name,iters", [("tiny", (0, 1, 2, 3, 8, 9)), ("mid", (0, 1)), ("r100", (0, 1, 4, 5))])
def test_sbb_step_teacher_forced(name, iters, dev):
    c, op, plan = problem(name, dev)
    b32 = _signal(name, op, c)
    D, b = _t(c.D, dev), _t(b32, dev)
    w = c.w0.astype(np.float32)
    for i in range(max(iters) + 1):
        ref = oracle.sbb_step(op, w, i, b32)
        if i in iters:
            w_gpu, st = _gpu_step(plan, D, b, w, i, dev)
            assert st["iter"] == i + 1
            assert relerr(w_gpu, ref.w) <= TOL, (name, i)
            assert abs(st["alpha"] - ref.alpha) <= TOL * ref.alpha, (name, i)
            assert abs(st["obj"] - ref.f) <= TOL * ref.f, (name, i)
            assert abs(st["gt_norm2"] - ref.gt_norm2) <= TOL * ref.gt_norm2, (name, i)
        w = ref.w.astype(np.float32)


@pytest.mark.parametrize("name,iters", [("tiny", (0, 1, 2, 3, 8, 9)), ("mid", (0, 1, 2)), ("r100", (0, 1, 4, 5)),
                                        ("r33@xyz", (0, 1, 2))])
def test_sbb_lagged_step_teacher_forced(name, iters, dev):
    c, op, plan = problem(name, dev)
    b32 = _signal(name.partition("@")[0], op, c)
    D, b = _t(c.D, dev), _t(b32, dev)
    w = c.w0.astype(np.float32)
    gprev = None
    for i in range(max(iters) + 1):
        ref = oracle.sbb_step_lagged(op, w, i, b32, gprev)
        if i in iters:
            wt = _t(w, dev)
            # at i = 0 the previous gradient must not be read: poison it
            gp = torch.full((c.n_fascicles,), float("nan"), device=dev) if gprev is None else _t(gprev, dev)
            st = life.new_state(dev, iteration=i)
            plan.sbbnnls_step_lagged(D, b, wt, gp, st)
            s = life.read_state(st)
            assert s["iter"] == i + 1
            assert relerr(_np(wt), ref.w) <= TOL, (name, i)
            assert abs(s["alpha"] - ref.alpha) <= TOL * ref.alpha, (name, i)
            assert abs(s["obj"] - ref.f) <= TOL * ref.f, (name, i)
            assert abs(s["num"] - ref.num) <= TOL * ref.num and abs(s["den"] - ref.den) <= TOL * ref.den
            assert relerr(_np(gp), ref.gt) <= TOL, (name, i)       # g~ handed to the next call
        w = ref.w.astype(np.float32)
        gprev = ref.gt.astype(np.float32)


def test_sbb_lagged_free_running_tiny(dev):
    c, op, plan = problem("tiny", dev)
    b32 = _signal("tiny", op, c)
    D, b = _t(c.D, dev), _t(b32, dev)
    w = _t(c.w0, dev)
    gp = torch.zeros(c.n_fascicles, device=dev)
    st = life.new_state(dev)
    f_gpu = []
    for _ in range(20):
        plan.sbbnnls_step_lagged(D, b, w, gp, st)
        f_gpu.append(life.read_state(st)["obj"])
    wr, gprev, f_ref = c.w0.astype(np.float64), None, []
    for i in range(20):
        r = oracle.sbb_step_lagged(op, wr, i, b32, gprev)
        f_ref.append(r.f)
        wr, gprev = r.w, r.gt
    assert np.max(np.abs(np.array(f_gpu) - np.array(f_ref)) / np.array(f_ref)) <= 1e-4
    assert f_gpu[-1] < 0.5 * f_gpu[0]


def test_sbb_free_running_tiny(dev):
    c, op, plan = problem("tiny", dev)
    b32 = _signal("tiny", op, c)
    D, b = _t(c.D, dev), _t(b32, dev)
    w = _t(c.w0, dev)
    st = life.new_state(dev)
    f_gpu = []
    for _ in range(20):
        plan.sbbnnls_step(D, b, w, st)
        f_gpu.append(life.read_state(st)["obj"])
    _, hist = oracle.sbb_run(op, c.w0.astype(np.float32), b32, 20)
    f_ref = np.array([h.f for h in hist])
    assert life.read_state(st)["iter"] == 20
    assert np.max(np.abs(np.array(f_gpu) - f_ref) / f_ref) <= 1e-4
    assert np.all(np.diff(f_gpu) <= 1e-6 * np.array(f_gpu[:-1]))    # objective does not rise


def test_sbb_zero_gradient_is_fixed_point(dev):
    # hand-worked case C of tests/golden: g~ = 0 gives alpha = 0 and w unchanged
    D = torch.tensor([1.0, -1.0, 2.0, 1.0], device=dev)
    plan = life.Plan(2, 2, 2, 2, np.array([0, 1, 1]), np.array([0, 0, 1]), np.array([0, 1, 0]),
                     np.array([1.0, 2.0, 3.0]))
    w = torch.tensor([0.0, 2.0], device=dev)
    b = torch.tensor([8.0, 4.0, -1.0, 0.0], device=dev)
    for i in (0, 1):
        st = life.new_state(dev, iteration=i)
        plan.sbbnnls_step(D, b, w, st)
        s = life.read_state(st)
        assert s["alpha"] == 0.0 and s["den"] == 0.0 and s["obj"] == 0.5
        assert _np(w).tolist() == [0.0, 2.0]
    plan.close()


def test_sbb_hand_cases_exact(dev):
    # the hand-worked cases A and B (small integers: float32 reproduces them closely)
    D = torch.tensor([1.0, -1.0, 2.0, 1.0], device=dev)
    plan = life.Plan(2, 2, 2, 2, np.array([0, 1, 1]), np.array([0, 0, 1]), np.array([0, 1, 0]),
                     np.array([1.0, 2.0, 3.0]))
    cases = [((1, 2), (8, 3, 6, 2), 0, 71 / 2885, (2601 / 2885, 5486 / 2885)),
             ((1, 2), (8, 3, 6, 2), 1, 2 / 71, (63 / 71, 134 / 71)),
             ((0, 2), (8, 3, -1, 0), 1, 1 / 20, (0, 19 / 10)),
             ((0, 2), (8, 3, -1, 0), 0, 5 / 101, (0, 192 / 101))]
    for w0, b0, i, alpha, wn in cases:
        w = torch.tensor(w0, dtype=torch.float32, device=dev)
        st = life.new_state(dev, iteration=i)
        plan.sbbnnls_step(D, torch.tensor(b0, dtype=torch.float32, device=dev), w, st)
        s = life.read_state(st)
        assert s["alpha"] == pytest.approx(alpha, rel=1e-6)
        np.testing.assert_allclose(_np(w), wn, rtol=1e-6, atol=1e-7)
    plan.close()
