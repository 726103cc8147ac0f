import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU case")


_cache = {}


def connectome(name, **kw):
    """Seeded synthetic problem, cached per test session."""
    import synth
    key = (name, tuple(sorted(kw.items())))
    if key not in _cache:
        _cache[key] = synth.make(name, **kw)
    return _cache[key]


@pytest.fixture(scope="session")
def tiny():
    return connectome("tiny")


def relerr(x, ref):
    """Normwise relative error ||x - ref||_2 / ||ref||_2 (ref = 0 -> ||x||)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm(x - ref)
    n = np.linalg.norm(ref)
    return float(d / n) if n > 0 else float(d)


def morton_positions(xyz):
    """Processing position of each voxel in Morton (Z-order) sequence of its (x, y, z)
    grid coordinates, ties by index: the key interleaves bit b of x, y, z into bits
    3b, 3b+1, 3b+2."""
    xyz = np.asarray(xyz, np.int64)
    key = np.zeros(len(xyz), np.int64)
    for b in range(16):
        for axis in range(3):
            key |= ((xyz[:, axis] >> b) & 1) << (3 * b + axis)
    order = np.argsort(key, kind="stable")
    pos = np.empty(len(xyz), np.int64)
    pos[order] = np.arange(len(xyz))
    return pos


def fascicle_keys(fascicle, vpp, n_fascicles):
    """Rank keys of the fascicles: Z(lo, hi), where lo, hi are the first and last
    processing positions of a fascicle's voxels and Z puts bit i of lo at bit 2i and
    bit i of hi at bit 2i+1; a fascicle without nonzeros gets the largest key."""
    lo = np.full(n_fascicles, np.iinfo(np.int64).max, np.int64)
    hi = np.full(n_fascicles, -1, np.int64)
    np.minimum.at(lo, fascicle, vpp)
    np.maximum.at(hi, fascicle, vpp)
    has = hi >= 0
    a = np.where(has, lo, 0).astype(np.uint64)
    b = np.where(has, hi, 0).astype(np.uint64)
    z = np.zeros(n_fascicles, np.uint64)
    for i in range(32):
        one = np.uint64(1)
        z |= ((a >> np.uint64(i)) & one) << np.uint64(2 * i)
        z |= ((b >> np.uint64(i)) & one) << np.uint64(2 * i + 1)
    return np.where(has, z, np.iinfo(np.uint64).max)


def reference_plan(c, xyz=None):
    """The restructuring plan computed independently with numpy.lexsort.

    DSC order (voxel, atom, fascicle, input position); voxel processing positions
    pp (identity, or Morton order of xyz); fascicle ranks by fascicle_keys (empty
    fascicles last, ties by index); WC order (rank, pp, atom, input position) given
    as DSC positions; segment offsets of both."""
    pos = np.arange(c.nnz)
    pp = np.arange(c.n_voxels) if xyz is None else morton_positions(xyz)
    dsc = np.lexsort((pos, c.fascicle, c.atom, c.voxel))
    key = fascicle_keys(c.fascicle, pp[c.voxel], c.n_fascicles)
    order = np.argsort(key, kind="stable")
    rank = np.empty(c.n_fascicles, np.int64)
    rank[order] = np.arange(c.n_fascicles)
    wc_in = np.lexsort((pos, c.atom, pp[c.voxel], rank[c.fascicle]))
    inv = np.empty(c.nnz, np.int64)
    inv[dsc] = pos
    return {
        "dsc_perm": dsc,
        "vox_ptr": np.searchsorted(c.voxel[dsc], np.arange(c.n_voxels + 1), side="left"),
        "fas_rank": rank,
        "wc_perm": inv[wc_in],
        "fas_ptr": np.searchsorted(rank[c.fascicle[wc_in]], np.arange(c.n_fascicles + 1), side="left"),
    }
