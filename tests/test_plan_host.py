"""Host-side checks of the C ABI (no GPU): exported symbols, restructuring plans
bit-exact against an independent numpy.lexsort, and argument/range errors."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from conftest import ROOT, connectome, reference_plan
from paper_1905_06234_amd import life

HEADER = os.path.join(ROOT, "include", "life.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(life_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = life.load()
    names = _declared_functions()
    assert "life_dsc" in names and "life_wc" in names and "life_sbbnnls_step" in names and "life_plan" in names
    for n in names:
        assert hasattr(lib, n), n
    # the binding covers every declared function
    assert set(names) <= set(life._SIGS)


def test_status_strings():
    lib = life.load()
    for s in range(5):
        assert lib.life_status_str(s).decode().startswith(life.STATUS[s])


@pytest.mark.parametrize("morton", [False, True])
@pytest.mark.parametrize("which", ["tiny", "mid20k", "random_dup", "ragged"])
def test_host_plan_bit_exact(which, morton):
    if which == "tiny":
        c = connectome("tiny")
    elif which == "mid20k":
        c = connectome("mid", n_fascicles=20_000)
    elif which == "random_dup":
        c = synth.random_coo(7, 30, 101, 57, 5000, seed=4, duplicates=True)
    else:
        c = synth.random_coo(3, 5, 9000, 3, 1234, seed=5)   # many empty voxels
    xyz = None
    if morton:
        xyz = c.voxel_xyz
        if which in ("random_dup", "ragged"):     # random coordinates with repeats (ties)
            xyz = np.random.default_rng(9).integers(0, 30, size=(c.n_voxels, 3)).astype(np.int16)
    p = life.plan_host(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, c.fascicle, xyz)
    ref = reference_plan(c, xyz)
    for k in ("dsc_perm", "vox_ptr", "fas_rank", "wc_perm", "fas_ptr"):
        assert np.array_equal(p[k], ref[k]), k


def test_morton_positions_pinned():
    """The Z-order on a 2x2x2 grid visits x fastest, then y, then z; coordinate 4 in
    x (bit 2) comes after every coordinate below 4 in all axes."""
    from conftest import morton_positions
    cube = np.array([(x, y, z) for z in range(2) for y in range(2) for x in range(2)])
    assert np.array_equal(morton_positions(cube), np.arange(8))
    pts = np.array([(4, 0, 0), (3, 3, 3), (0, 0, 1), (1, 0, 0)])
    assert np.array_equal(morton_positions(pts), [3, 2, 1, 0])


def test_fascicle_rank_key_pinned():
    """Fascicles rank by the Z-order of (first, last) voxel position, worked by hand
    on 8 voxels in index order: f2 spans (1, 1) -> Z = 0b11 = 3, f0 spans (3, 4) ->
    bits of 3 at 0, 2 and of 4 at 5 -> 37, f1 spans (0, 6) -> bits of 6 at 3, 5 -> 40;
    f3 crosses nothing and ranks last.  (The mean position would put f1, 3.0, ahead
    of f0, 3.5.)"""
    fascicle = np.array([0, 0, 1, 1, 2], np.int32)
    voxel = np.array([3, 4, 0, 6, 1], np.int32)
    p = life.plan_host(2, 1, 8, 4, np.zeros(5, np.int16), voxel, fascicle)
    assert np.array_equal(p["fas_rank"], [1, 2, 0, 3])
    from conftest import fascicle_keys
    assert np.array_equal(fascicle_keys(fascicle, voxel, 4)[:3], [37, 40, 3])


def test_negative_coordinate_rejected():
    c = connectome("tiny")
    xyz = c.voxel_xyz.copy()
    xyz[5, 1] = -1
    with pytest.raises(life.LifeError) as e:
        life.plan_host(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, c.fascicle, xyz)
    assert e.value.status == 2
    with pytest.raises(ValueError):
        life.plan_host(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, c.fascicle, xyz[:-1])


def test_host_plan_empty():
    p = life.plan_host(4, 3, 5, 6, np.zeros(0, np.int16), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert np.array_equal(p["vox_ptr"], np.zeros(6)) and np.array_equal(p["fas_ptr"], np.zeros(7))


@pytest.mark.parametrize("field,value", [("atom", 64), ("atom", -1), ("voxel", 512), ("voxel", -3),
                                         ("fascicle", 200), ("fascicle", -1)])
def test_out_of_range_index_rejected(field, value):
    c = connectome("tiny")
    arrs = {"atom": c.atom.copy(), "voxel": c.voxel.copy(), "fascicle": c.fascicle.copy()}
    arrs[field][len(arrs[field]) // 2] = value
    with pytest.raises(life.LifeError) as e:
        life.plan_host(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, arrs["atom"], arrs["voxel"], arrs["fascicle"])
    assert e.value.status == 2
    # life_plan checks indices before touching any device
    with pytest.raises(life.LifeError) as e:
        life.Plan(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, arrs["atom"], arrs["voxel"], arrs["fascicle"], c.phi)
    assert e.value.status == 2


@pytest.mark.parametrize("dims", [(0, 4, 4, 4), (1025, 4, 4, 4), (8, 0, 4, 4), (8, 40000, 4, 4),
                                  (8, 4, -1, 4), (8, 4, 4, -2)])
def test_bad_dims_rejected(dims):
    a = np.zeros(1, np.int16)
    v = np.zeros(1, np.int32)
    with pytest.raises(life.LifeError) as e:
        life.plan_host(*dims, a, v, v)
    assert e.value.status == 1


def test_null_arguments_rejected():
    lib = life.load()
    d = life.Dims(4, 4, 4, 4, 3)
    assert lib.life_plan_host(ctypes.byref(d), None, None, None, None, None, None, None, None, None) == 1
    assert lib.life_plan_host(None, None, None, None, None, None, None, None, None, None) == 1
    h = ctypes.c_void_p()
    assert lib.life_plan(ctypes.byref(d), None, None, None, None, ctypes.byref(h)) == 1
    assert lib.life_plan_ex(ctypes.byref(d), None, None, None, None, None, ctypes.byref(h)) == 1
    assert lib.life_plan_ex(ctypes.byref(d), None, None, None, None, None, None) == 1
    assert lib.life_dsc(None, None, None, None, None) == 1
    assert lib.life_wc(None, None, None, None, None) == 1
    assert lib.life_sbbnnls_step(None, None, None, None, None, None) == 1
    assert lib.life_plan_destroy(None) == 0


# ----------------------------------------------------------------------------- batched plans


def _batch_instances():
    b = synth.make_batch(3, seed=5, scale=0.02)
    # an instance with extra fascicles that cross no voxel (empty fascicles) and a random one
    r = synth.random_coo(96, 1057, 300, 80, 900, seed=11)
    r = synth.Connectome(name="r", n_theta=r.n_theta, n_atoms=r.n_atoms, n_voxels=r.n_voxels,
                         n_fascicles=r.n_fascicles + 5, atom=r.atom, voxel=r.voxel, fascicle=r.fascicle,
                         phi=r.phi, D=b[0].D, w0=np.zeros(r.n_fascicles + 5, np.float32),
                         w_true=np.zeros(r.n_fascicles + 5, np.float32), noise=r.noise, grid=r.grid,
                         voxel_xyz=np.random.default_rng(3).integers(0, 9, (r.n_voxels, 3)).astype(np.int16))
    return b[:2] + [r] + b[2:]


def _reference_batch_plan(inst, raw=None):
    """Batched restructuring computed independently: positions instance by instance
    (Morton inside, blocks padded to 64), ranks by (instance, fascicle_keys, index)
    (so empty fascicles end their instance's block), then the same lexsorts as
    reference_plan."""
    from conftest import fascicle_keys, morton_positions
    dims, vox_off, fas_off, atom, voxel, fascicle, phi, xyz = raw or life.concat_instances(inst)
    pp = np.empty(dims.n_voxels, np.int64)
    inst_of = np.empty(dims.n_fascicles, np.int64)
    base = 0
    for k in range(len(vox_off) - 1):
        v0, v1 = vox_off[k], vox_off[k + 1]
        pp[v0:v1] = base + morton_positions(xyz[v0:v1])
        base += -(-(v1 - v0) // 64) * 64
        inst_of[fas_off[k]:fas_off[k + 1]] = k
    pos = np.arange(dims.nnz)
    key = fascicle_keys(fascicle, pp[voxel], dims.n_fascicles)
    order = np.lexsort((np.arange(dims.n_fascicles), key, inst_of))
    rank = np.empty(dims.n_fascicles, np.int64)
    rank[order] = np.arange(dims.n_fascicles)
    dsc = np.lexsort((pos, fascicle, atom, voxel))
    wc_in = np.lexsort((pos, atom, pp[voxel], rank[fascicle]))
    inv = np.empty(dims.nnz, np.int64)
    inv[dsc] = pos
    return {"proc_pos": pp, "dsc_perm": dsc,
            "vox_ptr": np.searchsorted(voxel[dsc], np.arange(dims.n_voxels + 1)),
            "fas_rank": rank, "wc_perm": inv[wc_in],
            "fas_ptr": np.searchsorted(rank[fascicle[wc_in]], np.arange(dims.n_fascicles + 1))}


def test_batch_host_plan_bit_exact():
    inst = _batch_instances()
    p = life.plan_host_batch(inst)
    ref = _reference_batch_plan(inst)
    for k in ("proc_pos", "dsc_perm", "vox_ptr", "fas_rank", "wc_perm", "fas_ptr"):
        assert np.array_equal(p[k], ref[k]), k
    # every instance's fascicles take one contiguous block of ranks, in instance order
    fo = p["fas_off"]
    for k in range(len(inst)):
        assert np.array_equal(np.sort(p["fas_rank"][fo[k]:fo[k + 1]]), np.arange(fo[k], fo[k + 1]))


def test_batch_rejects_nonzero_across_instances():
    inst = _batch_instances()
    raw = list(life.concat_instances(inst))
    voxel = raw[4].copy()
    voxel[0] = raw[1][-1] - 1                   # first nonzero (instance 0) moved into the last instance
    raw[4] = voxel
    with pytest.raises(life.LifeError) as e:
        life.plan_host_batch(None, raw=tuple(raw))
    assert e.value.status == 2
    bad = list(life.concat_instances(inst))
    bad[1] = bad[1].copy()
    bad[1][1] = bad[1][2] + 1                   # offsets must not decrease
    with pytest.raises(life.LifeError) as e:
        life.plan_host_batch(None, raw=tuple(bad))
    assert e.value.status == 1


def test_batch_plan_needs_chunked_geometry():
    """Batched plans need N_theta <= 128 (checked before any device is touched)."""
    a = synth.random_coo(129, 5, 40, 10, 200, seed=1)
    b = synth.random_coo(129, 5, 30, 12, 150, seed=2)
    for c in (a, b):
        c.voxel_xyz = np.zeros((c.n_voxels, 3), np.int16)
    with pytest.raises(life.LifeError) as e:
        life.Plan.batch([a, b])
    assert e.value.status == 1


def test_explicit_tiling_checked_before_the_device():
    """life_plan_flags rejects a tiling whose LDS blocks do not fit at N_theta = 96
    (one tile of 500 atoms: the WC pass-1 block alone needs 160,000 bytes), and a
    negative tile_atoms, before any device is touched."""
    c = synth.random_coo(96, 500, 64, 100, 2000, seed=3)
    for ta in (500, -1):
        with pytest.raises(life.LifeError) as e:
            life.Plan.build(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, c.fascicle, c.phi,
                            tile_atoms=ta)
        assert e.value.status == 1, ta


def test_autotune_arguments_checked_before_the_device():
    """life_plan_autotune rejects missing offsets of a batched plan, reps < 1, a
    missing dictionary and unknown flags with LIFE_EINVAL before touching a device."""
    lib = life.load()
    c = synth.random_coo(16, 8, 40, 10, 200, seed=4)
    dims = life.Dims(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.nnz)
    arrs = [np.ascontiguousarray(a) for a in (c.atom, c.voxel, c.fascicle, c.phi)]
    ptrs = [life._np_ptr(a) for a in arrs]
    D = ctypes.c_void_p(16)   # never dereferenced: every case fails its argument checks first
    out = ctypes.c_void_p()
    ta, pol = ctypes.c_int32(), ctypes.c_int32()
    for n_inst, d, reps, flags in ((2, D, 1, 0), (1, D, 0, 0), (1, None, 1, 0), (1, D, 1, 2), (0, D, 1, 0)):
        st = lib.life_plan_autotune(ctypes.byref(dims), n_inst, None, None, *ptrs, None, flags, d, reps,
                                    ctypes.byref(ta), ctypes.byref(pol), ctypes.byref(out))
        assert st == 1, (n_inst, d, reps, flags)
        assert not out.value


def test_batch_ranks_with_empty_instances():
    """Instances without voxels (leading and in the middle) and instances whose
    fascicles are all empty: every instance's ranks are exactly its own block
    [fas_off[k], fas_off[k+1]), which the batched step kernels rely on."""
    inst = _batch_instances()[:2]
    dims, vox_off, fas_off, atom, voxel, fascicle, phi, xyz = life.concat_instances(inst)
    # insert an instance with no voxels and 3 fascicles before each real instance
    vo = np.array([0, 0, vox_off[1], vox_off[1], vox_off[2]], np.int32)
    shift = np.array([3, 6])
    fo = np.array([0, 3, 3 + fas_off[1], 6 + fas_off[1], 6 + fas_off[2]], np.int32)
    k_of = np.searchsorted(fas_off, fascicle, side="right") - 1
    fas2 = (fascicle + shift[k_of]).astype(np.int32)
    d2 = life.Dims(dims.n_theta, dims.n_atoms, dims.n_voxels, int(fo[-1]), dims.nnz)
    raw = (d2, vo, fo, atom, voxel, fas2, phi, xyz)
    p = life.plan_host_batch(None, raw=raw)
    for k in range(len(vo) - 1):
        assert np.array_equal(np.sort(p["fas_rank"][fo[k]:fo[k + 1]]), np.arange(fo[k], fo[k + 1])), k
    ref = _reference_batch_plan(None, raw=raw)
    for key in ("proc_pos", "dsc_perm", "vox_ptr", "fas_rank", "wc_perm", "fas_ptr"):
        assert np.array_equal(p[key], ref[key]), key
