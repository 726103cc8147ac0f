"""The device plan builder (the default of life_plan*) against the host builder
(LIFE_PLAN_HOST_BUILD), bit for bit: every array of the plan is hashed
(life_plan_digest) and the digests must be equal, for single problems (Morton and
index order, duplicates, ragged and empty inputs, N_theta > 128, a voxel that
crosses more fascicles than a chunk holds), for device-resident inputs, and for
batched plans; the canonical orders are also checked against numpy.lexsort."""
import numpy as np
import pytest

import oracle
import synth
from conftest import connectome, reference_plan, relerr

torch = pytest.importorskip("torch")
from paper_1905_06234_amd import life  # noqa: E402
from test_gpu_parity import RANDOM_SHAPES, _np, _t, dev  # noqa: E402,F401

pytestmark = pytest.mark.gpu


def _case(name):
    if name in ("tiny", "mid"):
        c = connectome(name)
        return c, c.voxel_xyz
    if name.endswith("@id"):
        c = connectome(name[:-3])
        return c, None
    nt, na, nv, nf, nnz, dup = RANDOM_SHAPES[name]
    c = synth.random_coo(nt, na, nv, nf, nnz, seed=len(name) * 7 + nnz % 97, duplicates=dup)
    rng = np.random.default_rng(nnz)
    return c, rng.integers(0, 2 * round(nv ** (1 / 3)) + 2, size=(nv, 3)).astype(np.int16)


CASES = ["tiny", "mid", "tiny@id", "mid@id"] + list(RANDOM_SHAPES)


def _build(c, xyz, **kw):
    return life.Plan.build(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, c.fascicle, c.phi,
                           voxel_xyz=xyz, **kw)


@pytest.mark.parametrize("name", CASES)
def test_device_builder_equals_host_builder(name, dev):
    c, xyz = _case(name)
    print(f"[plan] {name}: nnz={c.nnz}", flush=True)
    pg, ph = _build(c, xyz), _build(c, xyz, host_build=True)
    dg, dh = pg.digest(), ph.digest()
    assert np.array_equal(dg, dh), np.nonzero(dg != dh)[0]
    pd = _build(c, xyz, device_input=True)
    assert np.array_equal(pd.digest(), dh)
    ref = reference_plan(c, xyz)
    ex = pg.export()
    assert np.array_equal(ex["vox_ptr"], ref["vox_ptr"])
    assert np.array_equal(ex["fas_rank"], ref["fas_rank"])
    assert np.array_equal(ex["fas_ptr"], ref["fas_ptr"])
    assert np.array_equal(ex["atom_v"], c.atom[ref["dsc_perm"]])
    # the products of the device-built plan
    w = np.random.default_rng(3).random(c.n_fascicles).astype(np.float32)
    y = pg.dsc(_t(c.D, dev), _t(w, dev))
    assert relerr(_np(y), oracle.Operator.from_connectome(c).dsc(w)) <= 1e-5
    for p in (pg, ph, pd):
        p.close()


def test_fascicle_overflow_falls_back(dev):
    """One voxel crosses more distinct fascicles than a chunk holds: both builders
    give the same generic plan, and its products stay right."""
    rng = np.random.default_rng(9)
    nf, nv = 17000, 20
    heavy = np.arange(nf, dtype=np.int32)
    rest = rng.integers(0, nf, 3000).astype(np.int32)
    fas = np.concatenate([heavy, rest])
    vox = np.concatenate([np.zeros(nf, np.int32), rng.integers(1, nv, 3000).astype(np.int32)])
    atom = rng.integers(0, 60, fas.size).astype(np.int16)
    phi = rng.uniform(0.3, 1.2, fas.size).astype(np.float32)
    D = rng.standard_normal((60, 32)).astype(np.float32)
    c = synth.Connectome(name="overflow", n_theta=32, n_atoms=60, n_voxels=nv, n_fascicles=nf, atom=atom, voxel=vox,
                         fascicle=fas, phi=phi, D=D, w0=rng.random(nf).astype(np.float32),
                         w_true=rng.random(nf).astype(np.float32),
                         noise=rng.standard_normal(32 * nv).astype(np.float32), grid=None, voxel_xyz=None)
    ph = _build(c, None, host_build=True)
    op = oracle.Operator.from_connectome(c)
    for label, p in (("host", ph), ("device", _build(c, None))):
        print(f"[plan] overflow case, {label} builder", flush=True)
        assert np.array_equal(p.digest(), ph.digest())
        y = p.dsc(_t(c.D, dev), _t(c.w0, dev))
        assert relerr(_np(y), op.dsc(c.w0)) <= 1e-5
        g = p.wc(_t(c.D, dev), _t(c.noise, dev))
        assert relerr(_np(g), op.wc(c.noise)) <= 1e-5
    ph.close()


def test_batched_device_builder_equals_host_builder(dev):
    inst = synth.make_batch(4, seed=3, scale=0.02)
    pg, ph = life.Plan.batch(inst), life.Plan.batch(inst, host_build=True)
    assert np.array_equal(pg.digest(), ph.digest())
    pg.close()
    ph.close()


def test_bad_index_rejected_on_device(dev):
    c = connectome("tiny")
    bad = c.fascicle.copy()
    bad[17] = c.n_fascicles
    for kw in ({}, {"device_input": True}):
        with pytest.raises(life.LifeError) as e:
            life.Plan.build(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, bad, c.phi, **kw)
        assert e.value.status == 2
