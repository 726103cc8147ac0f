"""Plan geometry choices: every dictionary tiling (life_plan_flags' tile_atoms)
computes the same products, within 1e-5 of the FP64 oracle, bitwise repeatably,
with the device and host builders giving the same plan; a tiling the LDS cannot
hold is rejected; life_plan_autotune keeps one of the candidates and its plan
passes the same checks (single and batched)."""
import numpy as np
import pytest

import oracle
import synth
from conftest import connectome, relerr

torch = pytest.importorskip("torch")
from paper_1905_06234_amd import life  # noqa: E402
from test_gpu_parity import RANDOM_SHAPES, _np, _t, dev  # noqa: E402,F401

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _case(name):
    if name == "mid":
        return connectome("mid")
    nt, na, nv, nf, nnz, dup = RANDOM_SHAPES[name]
    c = synth.random_coo(nt, na, nv, nf, nnz, seed=len(name) * 7 + nnz % 97, duplicates=dup)
    rng = np.random.default_rng(nnz)
    c.voxel_xyz = rng.integers(0, 2 * round(nv ** (1 / 3)) + 2, size=(nv, 3)).astype(np.int16)
    return c


def _build(c, **kw):
    return life.Plan.build(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, c.fascicle, c.phi,
                           voxel_xyz=c.voxel_xyz, **kw)


def _check_products(plan, c, op, dev, label):
    rng = np.random.default_rng(41)
    w = rng.random(c.n_fascicles).astype(np.float32)
    y = rng.standard_normal(c.n_theta * c.n_voxels).astype(np.float32)
    D, wt, yt = _t(c.D, dev), _t(w, dev), _t(y, dev)
    y1 = plan.dsc(D, wt).clone()
    g1 = plan.wc(D, yt).clone()
    dd1 = plan.dict_grad(wt, yt).clone()
    assert relerr(_np(y1), op.dsc(w)) <= TOL, label
    assert relerr(_np(g1), op.wc(y)) <= TOL, label
    assert relerr(_np(dd1), op.dd(w, y)) <= TOL, label
    # bitwise repeatable
    assert torch.equal(plan.dsc(D, wt), y1), label
    assert torch.equal(plan.wc(D, yt), g1), label
    assert torch.equal(plan.dict_grad(wt, yt), dd1), label


@pytest.mark.parametrize("name,tiles", [("mid", [0, 32, 48, 100]),
                                        ("r96big", [0, 64, 133, 265, 354, 480]),
                                        ("r100", [0, 16, 24]),
                                        ("dense16", [0, 64, 100, 256])])
def test_every_tiling_gives_the_same_products(name, tiles, dev):
    c = _case(name)
    op = oracle.Operator.from_connectome(c)
    for ta in tiles:
        print(f"[tiling] {name}: tile_atoms={ta}", flush=True)
        p = _build(c, tile_atoms=ta)
        got = p.tile_atoms
        assert got > 0 and (ta == 0 or got <= ta)
        assert np.array_equal(p.digest(), _build(c, tile_atoms=ta, host_build=True).digest())
        _check_products(p, c, op, dev, (name, ta))
        p.close()


def test_tiling_too_large_rejected(dev):
    c = synth.random_coo(96, 500, 64, 100, 2000, seed=3)
    c.voxel_xyz = None
    _build(c, tile_atoms=499).close()      # two balanced tiles of 250 atoms fit
    for ta in (500, 1000, -1):             # one tile of all 500 atoms: its WC pass-1 block exceeds the LDS
        with pytest.raises(life.LifeError) as e:
            _build(c, tile_atoms=ta)
        assert e.value.status == 1, ta


@pytest.mark.parametrize("name", ["mid", "r96big"])
def test_autotune_single(name, dev):
    c = _case(name)
    op = oracle.Operator.from_connectome(c)
    p = life.Plan.autotune([c], _t(c.D, dev), reps=2)
    print(f"[autotune] {name}: tile_atoms={p.tile_atoms} policy={p.policy}", flush=True)
    assert p.tile_atoms > 0 and p.policy in (0, 1, 2)
    q = _build(c, tile_atoms=p.tile_atoms)
    assert q.tile_atoms == p.tile_atoms      # the chosen tiling is one life_plan_flags builds
    q.close()
    _check_products(p, c, op, dev, name)
    p.close()


def test_autotune_batched(dev):
    inst = synth.make_batch(3, seed=5, scale=0.02)
    D = inst[0].D
    p = life.Plan.autotune(inst, _t(D, dev), reps=2)
    print(f"[autotune] batch of 3: tile_atoms={p.tile_atoms} policy={p.policy}", flush=True)
    assert p.n_inst == 3 and p.tile_atoms > 0
    rng = np.random.default_rng(8)
    assert all(np.array_equal(c.D, D) for c in inst)
    w = rng.random(int(p.fas_off[-1])).astype(np.float32)
    y = p.dsc(_t(D, dev), _t(w, dev))
    for k, c in enumerate(inst):
        op = oracle.Operator.from_connectome(c)
        yk = _np(y)[p.vox_off[k] * c.n_theta:p.vox_off[k + 1] * c.n_theta]
        assert relerr(yk, op.dsc(w[p.fas_off[k]:p.fas_off[k + 1]])) <= TOL, k
    p.close()
