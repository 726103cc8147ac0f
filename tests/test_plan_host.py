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
