"""Pins for the FP64 oracle, against things other than the oracle itself.

* hand-worked values (tests/golden/hand_example.txt, derived from eqs. 1-4 and
  Algorithm 1 by hand, exact rationals);
* brute force: a dense M assembled entry by entry from M_v = D Phi_v (eq. 3);
* closed forms / invariants: adjoint identity, linearity, order invariance,
  duplicate (COO) summation;
* a special case that reduces to a library routine: D = I turns M into a plain
  COO sparse matrix (scipy.sparse);
* SBB-NNLS properties fixed by the mathematics (exact line search on odd
  iterations, least-squares gradient-change fit on even ones, pre-projection
  descent, BB2 <= BB1) and convergence to the Lawson-Hanson NNLS solution
  (scipy.optimize.nnls) with KKT conditions.

A final group plants plausible mistakes in copies of the oracle step and checks
that these pins catch each one.
"""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse
from scipy.optimize import nnls

import oracle
import synth
from conftest import connectome, relerr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_example.txt")


def _golden():
    kv, sbb = {}, []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] in ("sbb", "lag"):
            sbb.append(tok)
        else:
            kv[tok[0]] = tok[1:]
    return kv, sbb


def _hand_operator():
    kv, _ = _golden()
    nt, na = int(kv["n_theta"][0]), int(kv["n_atoms"][0])
    D = np.array([float(x) for x in kv["D"]]).reshape(na, nt)
    return kv, oracle.Operator(np.array(kv["atom"], dtype=np.int16), np.array(kv["voxel"], dtype=np.int32),
                               np.array(kv["fascicle"], dtype=np.int32), np.array(kv["phi"], dtype=np.float64),
                               D, int(kv["n_voxels"][0]), int(kv["n_fascicles"][0]))


def dense_M(c_atom, c_voxel, c_fas, c_phi, D, n_voxels, n_fascicles):
    """Assemble M (N_theta*N_v x N_f) entry by entry: M[t + Nt*v, f] += D[t, a]*phi."""
    nt = D.shape[1]
    M = np.zeros((nt * n_voxels, n_fascicles))
    for a, v, f, p in zip(c_atom.tolist(), c_voxel.tolist(), c_fas.tolist(), np.asarray(c_phi, np.float64).tolist()):
        for t in range(nt):
            M[t + nt * v, f] += float(D[a, t]) * p
    return M


# ----------------------------------------------------------------------------- hand-worked


def test_hand_example_products():
    kv, op = _hand_operator()
    y = op.dsc(np.array(kv["dsc_w"], dtype=np.float64))
    assert np.array_equal(y, np.array(kv["dsc_y"], dtype=np.float64))
    g = op.wc(np.array(kv["wc_y"], dtype=np.float64))
    assert np.array_equal(g, np.array(kv["wc_g"], dtype=np.float64))


def test_hand_example_sbb_steps():
    _, cases = _golden()
    _, op = _hand_operator()
    cases = [c[1:] for c in cases if c[0] == "sbb"]
    assert len(cases) == 6
    for case in cases:
        name, i = case[0], int(case[1])
        w = np.array([float(Fraction(x)) for x in case[2:4]])
        b = np.array([float(Fraction(x)) for x in case[4:8]])
        f, alpha = float(Fraction(case[8])), float(Fraction(case[9]))
        w_next = np.array([float(Fraction(x)) for x in case[10:12]])
        s = oracle.sbb_step(op, w, i, b)
        assert s.f == pytest.approx(f, rel=1e-14, abs=1e-15), name
        assert s.alpha == pytest.approx(alpha, rel=1e-14, abs=1e-15), name
        np.testing.assert_allclose(s.w, w_next, rtol=1e-14, atol=1e-15, err_msg=name)
        assert np.all(np.signbit(s.w) == False)  # noqa: E712  (+0.0 after projection)


def test_hand_example_lagged_steps():
    _, cases = _golden()
    _, op = _hand_operator()
    cases = [c[1:] for c in cases if c[0] == "lag"]
    assert len(cases) == 5
    for case in cases:
        name, i = case[0], int(case[1])
        w = np.array([float(Fraction(x)) for x in case[2:4]])
        b = np.array([float(Fraction(x)) for x in case[4:8]])
        q = None if case[8] == "-" else np.array([float(Fraction(x)) for x in case[8:10]])
        f, alpha = float(Fraction(case[10])), float(Fraction(case[11]))
        w_next = np.array([float(Fraction(x)) for x in case[12:14]])
        s = oracle.sbb_step_lagged(op, w, i, b, q)
        assert s.f == pytest.approx(f, rel=1e-14), name
        assert s.alpha == pytest.approx(alpha, rel=1e-14), (name, i)
        np.testing.assert_allclose(s.w, w_next, rtol=1e-14, atol=1e-15, err_msg=f"{name} {i}")


def test_hand_example_dictionary_gradient():
    kv, op = _hand_operator()
    dD = op.dd(np.array(kv["dd_w"], dtype=np.float64), np.array(kv["dd_ybar"], dtype=np.float64))
    assert np.array_equal(dD.ravel(), np.array(kv["dd_D"], dtype=np.float64))


# ----------------------------------------------------------------------------- brute force


def test_dense_M_tiny():
    c = connectome("tiny")
    op = oracle.Operator.from_connectome(c)
    M = dense_M(c.atom, c.voxel, c.fascicle, c.phi, c.D, c.n_voxels, c.n_fascicles)
    w = c.w0.astype(np.float64)
    y = np.random.default_rng(5).standard_normal(c.n_theta * c.n_voxels)
    assert relerr(op.dsc(w), M @ w) < 1e-13
    assert relerr(op.wc(y), M.T @ y) < 1e-13


@pytest.mark.parametrize("seed,shape", [(1, (7, 5, 13, 11, 300)), (2, (33, 9, 40, 17, 777)),
                                        (3, (1, 3, 4, 5, 20))])
def test_dense_M_random_with_duplicates(seed, shape):
    nt, na, nv, nf, nnz = shape
    c = synth.random_coo(nt, na, nv, nf, nnz, seed, duplicates=True)
    op = oracle.Operator.from_connectome(c)
    M = dense_M(c.atom, c.voxel, c.fascicle, c.phi, c.D, nv, nf)
    w = c.w0.astype(np.float64)
    y = c.noise.astype(np.float64)
    assert relerr(op.dsc(w), M @ w) < 1e-13
    assert relerr(op.wc(y), M.T @ y) < 1e-13


# ----------------------------------------------------------------------------- invariants


def _mid_slice():
    # a reduced mid-shaped problem: N_theta = 96, N_a = 1057, 20k fascicles
    return connectome("mid", n_fascicles=20_000)


@pytest.mark.parametrize("which", ["tiny", "mid20k"])
def test_adjoint_identity(which):
    c = connectome("tiny") if which == "tiny" else _mid_slice()
    op = oracle.Operator.from_connectome(c)
    rng = np.random.default_rng(11)
    w = rng.standard_normal(c.n_fascicles)
    y = rng.standard_normal(c.n_theta * c.n_voxels)
    lhs = float(op.dsc(w) @ y)
    rhs = float(w @ op.wc(y))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1e-300) + 1e-12


def test_linearity():
    c = connectome("tiny")
    op = oracle.Operator.from_connectome(c)
    rng = np.random.default_rng(12)
    w1, w2 = rng.standard_normal((2, c.n_fascicles))
    y1, y2 = rng.standard_normal((2, c.n_theta * c.n_voxels))
    assert relerr(op.dsc(2.5 * w1 - 0.75 * w2), 2.5 * op.dsc(w1) - 0.75 * op.dsc(w2)) < 1e-14
    assert relerr(op.wc(-1.5 * y1 + 3.0 * y2), -1.5 * op.wc(y1) + 3.0 * op.wc(y2)) < 1e-14


def test_order_invariance_and_duplicates():
    c = connectome("tiny")
    op = oracle.Operator.from_connectome(c)
    perm = np.random.default_rng(13).permutation(c.nnz)
    op_p = oracle.Operator(c.atom[perm], c.voxel[perm], c.fascicle[perm], c.phi[perm], c.D,
                           c.n_voxels, c.n_fascicles)
    w = c.w0.astype(np.float64)
    y = np.random.default_rng(14).standard_normal(c.n_theta * c.n_voxels)
    assert relerr(op_p.dsc(w), op.dsc(w)) < 1e-14
    assert relerr(op_p.wc(y), op.wc(y)) < 1e-14
    # splitting every value in two equal duplicate nonzeros leaves M unchanged
    op_d = oracle.Operator(np.concatenate([c.atom, c.atom]), np.concatenate([c.voxel, c.voxel]),
                           np.concatenate([c.fascicle, c.fascicle]),
                           np.concatenate([c.phi, c.phi]).astype(np.float64) * 0.5, c.D,
                           c.n_voxels, c.n_fascicles)
    assert relerr(op_d.dsc(w), op.dsc(w)) < 1e-14
    assert relerr(op_d.wc(y), op.wc(y)) < 1e-14


def test_identity_dictionary_is_plain_coo_spmv():
    # N_theta = N_a and D = I: M[(a, v), f] = phi, a plain COO matrix
    rng = np.random.default_rng(21)
    na, nv, nf, nnz = 12, 50, 40, 900
    atom = rng.integers(0, na, nnz).astype(np.int16)
    voxel = rng.integers(0, nv, nnz).astype(np.int32)
    fas = rng.integers(0, nf, nnz).astype(np.int32)
    phi = rng.uniform(0.3, 1.2, nnz)
    op = oracle.Operator(atom, voxel, fas, phi, np.eye(na), nv, nf)
    S = scipy.sparse.coo_matrix((phi, (atom.astype(np.int64) + na * voxel, fas)), shape=(na * nv, nf)).tocsr()
    w = rng.standard_normal(nf)
    y = rng.standard_normal(na * nv)
    assert relerr(op.dsc(w), S @ w) < 1e-14
    assert relerr(op.wc(y), S.T @ y) < 1e-14


def test_empty_and_degenerate():
    D = np.arange(6, dtype=np.float64).reshape(2, 3)
    op = oracle.Operator(np.zeros(0, np.int16), np.zeros(0, np.int32), np.zeros(0, np.int32),
                         np.zeros(0), D, 4, 5)
    assert np.array_equal(op.dsc(np.ones(5)), np.zeros(12))
    assert np.array_equal(op.wc(np.ones(12)), np.zeros(5))
    s = oracle.sbb_step(op, np.ones(5), 0, np.ones(12))
    assert s.alpha == 0.0 and np.array_equal(s.w, np.ones(5)) and s.f == 6.0


# ----------------------------------------------------------------------------- SBB-NNLS


def _problem(sparse_truth=False):
    c = connectome("tiny")
    op = oracle.Operator.from_connectome(c)
    wt = c.w_true.astype(np.float64)
    if sparse_truth:
        wt = np.where(np.arange(c.n_fascicles) % 3 == 0, 0.0, wt)
        b = oracle.noisy_signal(op, wt, c.noise, level=0.5)
    else:
        b = oracle.noisy_signal(op, wt, c.noise)
    return c, op, b


def test_step_op_counts():
    c, op, b = _problem()
    w = c.w0.astype(np.float64)
    counts = [(s.n_dsc, s.n_wc) for s in (oracle.sbb_step(op, w, i, b) for i in range(4))]
    assert counts == [(2, 2), (2, 1), (2, 2), (2, 1)]
    # on average two M w and 1.5 M^T y per iteration
    assert np.mean([d for d, _ in counts]) == 2.0 and np.mean([t for _, t in counts]) == 1.5


def _f(op, w, b):
    return op.objective(w, b)


@pytest.mark.parametrize("sparse_truth", [False, True])
def test_step_lengths_are_the_two_bb_minimisers(sparse_truth):
    c, op, b = _problem(sparse_truth)
    w, _ = oracle.sbb_run(op, c.w0, b, 5)        # move off the start so the mask is active
    for i in (5, 6):
        s = oracle.sbb_step(op, w, i, b)
        gt = s.gt
        a = s.alpha
        assert a > 0
        if i % 2 == 1:
            # odd: alpha is the exact minimiser of f along -g~ (quadratic line search)
            phi_ = lambda t: _f(op, w - t * gt, b)  # noqa: E731
        else:
            # even: alpha minimises || g~ - t M^T M g~ ||^2
            q = op.wc(op.dsc(gt))
            phi_ = lambda t: float(np.sum((gt - t * q) ** 2))  # noqa: E731
        for d in (1e-3, 1e-2, 1e-1):
            assert phi_(a) <= phi_(a * (1 + d)) and phi_(a) <= phi_(a * (1 - d))
        w = s.w


def test_bb2_not_above_bb1_and_predescent():
    c, op, b = _problem(sparse_truth=True)
    w = c.w0.astype(np.float64)
    for i in range(12):
        s_odd = oracle.sbb_step(op, w, 1, b)
        s_even = oracle.sbb_step(op, w, 0, b)
        assert s_even.alpha <= s_odd.alpha * (1 + 1e-12)
        f0 = _f(op, w, b)
        for s in (s_odd, s_even):
            if s.gt_norm2 > 0:
                # before projection both steps decrease f (alpha < 2 ||g~||^2 / ||M g~||^2)
                assert _f(op, w - s.alpha * s.gt, b) < f0
        w = oracle.sbb_step(op, w, i, b).w


@pytest.mark.parametrize("sparse_truth", [False, True])
def test_converges_to_lawson_hanson_nnls(sparse_truth):
    c, op, b = _problem(sparse_truth)
    M = dense_M(c.atom, c.voxel, c.fascicle, c.phi, c.D, c.n_voxels, c.n_fascicles)
    assert np.linalg.svd(M, compute_uv=False)[-1] > 0.1          # full column rank: unique minimiser
    x_ls, rn = nnls(M, b, maxiter=20000)
    f_star = 0.5 * rn * rn
    w = c.w0.astype(np.float64)
    g0 = None
    for i in range(20000):
        s = oracle.sbb_step(op, w, i, b)
        g0 = g0 or np.sqrt(s.gt_norm2)
        w = s.w
        if np.sqrt(s.gt_norm2) <= 1e-11 * g0:
            break
    assert i < 19999
    assert abs(_f(op, w, b) - f_star) <= 1e-10 * f_star
    assert np.max(np.abs(w - x_ls)) < 1e-6
    if sparse_truth:
        assert (x_ls == 0).sum() > 5                              # the bound is active somewhere
        assert np.array_equal(w == 0, x_ls == 0)
    grad = op.wc(op.dsc(w) - b)                                   # KKT: w >= 0, grad >= 0 on w = 0, w.grad = 0
    assert np.all(w >= 0)
    assert np.all(grad[w == 0] >= -1e-8)
    assert abs(float(w @ grad)) < 1e-7


def test_objective_monotone_on_tiny_run():
    c, op, b = _problem()
    _, hist = oracle.sbb_run(op, c.w0, b, 20)
    f = np.array([h.f for h in hist])
    assert np.all(np.diff(f) <= 1e-12 * f[:-1])


def test_lagged_variant_converges():
    c, op, b = _problem(sparse_truth=True)
    x_ls, rn = nnls(dense_M(c.atom, c.voxel, c.fascicle, c.phi, c.D, c.n_voxels, c.n_fascicles), b,
                    maxiter=20000)
    w, gprev = c.w0.astype(np.float64), None
    for i in range(3000):
        s = oracle.sbb_step_lagged(op, w, i, b, gprev)
        w, gprev = s.w, s.gt
    assert abs(_f(op, w, b) - 0.5 * rn * rn) <= 1e-8 * 0.5 * rn * rn


# ----------------------------------------------------------------------------- planted mistakes


def _mutant_steps():
    """Copies of the oracle step, each with one plausible mistake."""
    def swapped_parity(op, w, i, b):
        return oracle.sbb_step(op, w, i + 1, b)

    def no_subspace_mask(op, w, i, b):
        r = op.dsc(w) - b
        g = op.wc(r)
        vp = op.dsc(g)
        if i % 2:
            a = float(g @ g) / float(vp @ vp)
        else:
            vpp = op.wc(vp)
            a = float(vp @ vp) / float(vpp @ vpp)
        return np.maximum(w - a * g, 0.0), a

    def plus_sign(op, w, i, b):
        s = oracle.sbb_step(op, w, i, b)
        return np.maximum(w + s.alpha * s.gt, 0.0), s.alpha

    def literal_positive_part(op, w, i, b):
        # "negative values replaced by zeros" applied to the gradient itself
        r = op.dsc(w) - b
        g = np.maximum(op.wc(r), 0.0)
        vp = op.dsc(g)
        a = float(g @ g) / float(vp @ vp) if float(vp @ vp) > 0 else 0.0
        return np.maximum(w - a * g, 0.0), a

    def wrap(fn):
        def run(op, w, i, b):
            out = fn(op, w, i, b)
            return (out.w, out.alpha) if hasattr(out, "w") else out
        return run

    return {"swapped_parity": wrap(swapped_parity), "no_subspace_mask": no_subspace_mask,
            "plus_sign": plus_sign, "literal_positive_part": literal_positive_part}


@pytest.mark.parametrize("name", ["swapped_parity", "no_subspace_mask", "plus_sign", "literal_positive_part"])
def test_pins_catch_planted_step_mistakes(name):
    step = _mutant_steps()[name]
    kv, op_h = _hand_operator()
    _, cases = _golden()
    cases = [c[1:] for c in cases if c[0] == "sbb"]
    caught = False
    for case in cases:                       # hand-worked cases
        i = int(case[1])
        w = np.array([float(Fraction(x)) for x in case[2:4]])
        b = np.array([float(Fraction(x)) for x in case[4:8]])
        alpha = float(Fraction(case[9]))
        w_next = np.array([float(Fraction(x)) for x in case[10:12]])
        wn, a = step(op_h, w, i, b)
        if not (np.allclose(wn, w_next, rtol=1e-12, atol=1e-14) and abs(a - alpha) <= 1e-12 * max(alpha, 1)):
            caught = True
    c, op, b = _problem(sparse_truth=True)   # and convergence to Lawson-Hanson
    x_ls, _ = nnls(dense_M(c.atom, c.voxel, c.fascicle, c.phi, c.D, c.n_voxels, c.n_fascicles), b,
                   maxiter=20000)
    w = c.w0.astype(np.float64)
    for i in range(300):
        w, _ = step(op, w, i, b)
        if not np.all(np.isfinite(w)):
            break
    if not (np.all(np.isfinite(w)) and np.max(np.abs(w - x_ls)) < 1e-6):
        caught = True
    assert caught, name


def test_pins_catch_transposed_dictionary():
    # a D read with the wrong stride (atom-fastest instead of theta-fastest)
    c = connectome("tiny")
    M = dense_M(c.atom, c.voxel, c.fascicle, c.phi, c.D, c.n_voxels, c.n_fascicles)
    bad = np.ascontiguousarray(c.D.T.reshape(c.D.shape))
    op_bad = oracle.Operator(c.atom, c.voxel, c.fascicle, c.phi, bad, c.n_voxels, c.n_fascicles)
    assert relerr(op_bad.dsc(c.w0), M @ c.w0.astype(np.float64)) > 1e-3


# ----------------------------------------------------------------------------- dictionary gradient


def _dd_cases():
    yield "tiny", connectome("tiny")
    yield "random_dup", synth.random_coo(7, 30, 101, 57, 5000, seed=4, duplicates=True)


@pytest.mark.parametrize("which", ["tiny", "random_dup"])
def test_dd_adjoint_of_dsc_in_the_dictionary(which):
    """y = M(D) w is linear in D, so <dd(w, ybar), E> = <ybar, M(E) w> for any E."""
    c = dict(_dd_cases())[which]
    op = oracle.Operator.from_connectome(c)
    rng = np.random.default_rng(21)
    w = rng.random(c.n_fascicles)
    ybar = rng.standard_normal(c.n_theta * c.n_voxels)
    dD = op.dd(w, ybar)
    for _ in range(3):
        E = rng.standard_normal(c.D.shape)
        lhs = float(np.sum(dD * E))
        rhs = float(ybar @ op.with_dictionary(E).dsc(w))
        assert abs(lhs - rhs) <= 1e-12 * (abs(rhs) + float(np.sum(np.abs(dD) * np.abs(E)))), which


def test_loss_gradients_match_central_differences():
    """L = ||y_obs - M(D) w||^2 is quadratic in D and in w: central differences
    are exact up to rounding (FP64, h = 1e-6, rel <= 1e-6)."""
    c = connectome("tiny")
    op = oracle.Operator.from_connectome(c)
    rng = np.random.default_rng(22)
    w = c.w0.astype(np.float64)
    y_obs = rng.standard_normal(c.n_theta * c.n_voxels)
    gD, gw = op.loss_grads(w, y_obs)
    h = 1e-6
    for _ in range(4):
        E = rng.standard_normal(c.D.shape)
        fd = (op.with_dictionary(c.D + h * E).loss(w, y_obs) - op.with_dictionary(c.D - h * E).loss(w, y_obs)) / (2 * h)
        assert abs(fd - float(np.sum(gD * E))) <= 1e-6 * abs(fd)
        e = rng.standard_normal(c.n_fascicles)
        fd = (op.loss(w + h * e, y_obs) - op.loss(w - h * e, y_obs)) / (2 * h)
        assert abs(fd - float(gw @ e)) <= 1e-6 * abs(fd)


def test_dd_pin_catches_planted_mistakes():
    """Plausible slips in the dictionary gradient (a dropped phi, w read by voxel,
    ybar read at the atom's column) all fail the adjoint identity."""
    c = connectome("tiny")
    op = oracle.Operator.from_connectome(c)
    rng = np.random.default_rng(23)
    w = rng.random(c.n_fascicles)
    ybar = rng.standard_normal(c.n_theta * c.n_voxels)
    Y = ybar.reshape(c.n_voxels, c.n_theta)
    phi = c.phi.astype(np.float64)

    def scatter(scale, cols):
        out = np.zeros_like(c.D, dtype=np.float64)
        np.add.at(out, c.atom, scale[:, None] * cols)
        return out

    mutants = {
        "no_phi": scatter(w[c.fascicle], Y[c.voxel]),
        "w_by_voxel": scatter(phi * w[c.voxel % c.n_fascicles], Y[c.voxel]),
        "ybar_at_atom": scatter(phi * w[c.fascicle], Y[c.atom % c.n_voxels]),
    }
    E = rng.standard_normal(c.D.shape)
    rhs = float(ybar @ op.with_dictionary(E).dsc(w))
    assert abs(float(np.sum(op.dd(w, ybar) * E)) - rhs) <= 1e-10 * abs(rhs)
    for name, dD in mutants.items():
        assert abs(float(np.sum(dD * E)) - rhs) > 1e-6 * abs(rhs), name


# ----------------------------------------------------------------------------- multi-threaded oracle

@pytest.mark.parametrize("case", ["tiny", "dup", "ragged", "empty", "sparsevox"])
def test_parallel_oracle_equals_sequential(case):
    """The OpenMP oracle (grouped copies, one thread per output entry) gives the
    sequential oracle's DSC and WC bit for bit: each entry receives the same
    additions in the same (input) order."""
    if case == "tiny":
        c = connectome("tiny")
    else:
        shape = {"dup": (96, 57, 300, 400, 40_000, True), "ragged": (33, 9, 70, 100, 3000, False),
                 "empty": (16, 64, 50, 20, 0, False), "sparsevox": (8, 5, 5000, 30, 200, False)}[case]
        nt, na, nv, nf, nnz, dup = shape
        c = synth.random_coo(nt, na, nv, nf, nnz, seed=17, duplicates=dup)
    op = oracle.Operator.from_connectome(c)
    par = op.parallel()
    rng = np.random.default_rng(3)
    for w in (c.w0, rng.standard_normal(c.n_fascicles)):
        a, b = op.dsc(w), par.dsc(w)
        assert np.array_equal(a, b) and relerr(b, a) <= 1e-12
    for y in (c.noise, rng.standard_normal(c.n_theta * c.n_voxels)):
        a, b = op.wc(y), par.wc(y)
        assert np.array_equal(a, b) and relerr(b, a) <= 1e-12
    # the SBB step runs on either form
    b32 = oracle.noisy_signal(op, c.w_true, c.noise)
    s1, s2 = oracle.sbb_step(op, c.w0, 0, b32), oracle.sbb_step(par, c.w0, 0, b32)
    assert np.array_equal(s1.w, s2.w) and s1.alpha == s2.alpha
    assert oracle.par_threads() >= 1
    par.close()
