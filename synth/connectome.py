"""Seeded synthetic connectomes in the shape of the LiFE workloads.

This module only *draws inputs*: a dictionary D, a sparse tensor Phi given as
(atom, voxel, fascicle, value) nonzeros, weight vectors and a noise vector.  It
holds none of the method's arithmetic (no M.w, no M^T.y, no SBB step), so the
HIP path and the FP64 oracle can both be fed from it without sharing any code.

Model of the data (the paper's problem statement, Sec. 2.1, eqs. 1-4, and the
Phi representation of Sec. 2.2 as four vectors of one entry per nonzero):

* Gradient directions g_theta: uniform on the sphere.
* Atoms u_a: a Fibonacci sphere (mid/full) or uniform random unit vectors (tiny).
* Dictionary D[theta, a] = exp(-bval * (g_theta . u_a)^2) minus its mean over
  theta for each atom (the signal in eq. 1 is demeaned).  Stored theta-fastest,
  i.e. flat index theta + Ntheta*a, as the paper's offset rule Ntheta*index
  (Sec. 4.1, "Removing redundant computation") implies.
* Fascicles: random-walk polylines (step 0.7 voxel, turn angle <= 30 degrees per
  step) started inside a voxel mask and stopped at their length cap or at the
  mask boundary.  Each visited (fascicle, voxel) pair gives exactly one nonzero;
  its atom is the dictionary orientation nearest (axially) to the walk tangent
  on entry to the voxel, looked up in a precomputed cube-map table; its value
  Phi ~ U(0.3, 1.2) plays the part of the segment length in the voxel.  S0(v)
  of eq. 3 is taken as 1 (folded into Phi).
* Voxels are numbered in raster order (x fastest) over the mask.
* The nonzeros are emitted in a seeded random order, so a consumer must not rely
  on any ordering of the COO input.

The configurations are named after the workloads they stand for: ``tiny``
(8^3 grid, 200 fascicles), ``mid`` (64^3 ellipsoid, 200k fascicles, ~10M
nonzeros) and ``full`` (96^3 ellipsoid, 1.5M fascicles, ~80M nonzeros with a
lognormal start density so that voxel occupancy is heavy-tailed).
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Dict, Optional, Tuple

import numpy as np

STEP = 0.7                 # voxel lengths per walk step
MAX_TURN = math.radians(30.0)
PHI_LO, PHI_HI = 0.3, 1.2
LUT_RES = 96               # cube-map resolution per face for the atom lookup


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n_theta: int
    n_atoms: int
    atoms: str                     # "fibonacci" | "random"
    grid: Tuple[int, int, int]
    semi_axes: Optional[Tuple[float, float, float]]   # ellipsoid mask; None = full grid
    n_fascicles: int
    steps: Tuple[int, int]         # inclusive range of walk lengths (steps)
    length_dist: str               # "uniform" | "loguniform"
    density_sigma: float           # lognormal start-density log-std (0 = uniform starts)
    density_smooth: float          # Gaussian smoothing (voxels) of the density field
    bval: float
    seed: int
    dict_seed: Optional[int] = None   # seed of the gradient directions (None = seed)


CONFIGS: Dict[str, Config] = {
    "tiny": Config("tiny", 16, 64, "random", (8, 8, 8), None, 200, (7, 28),
                   "uniform", 0.0, 0.0, 1.0, 0),
    "mid": Config("mid", 96, 1057, "fibonacci", (64, 64, 64), (31.5, 30.5, 30.0),
                  200_000, (20, 120), "uniform", 0.0, 0.0, 1.0, 1),
    "full": Config("full", 96, 1057, "fibonacci", (96, 96, 96), (47.0, 41.0, 37.5),
                   1_500_000, (20, 200), "uniform", 1.2, 5.0, 1.0, 2),
}

# independent random streams of one configuration
_S_GRAD, _S_ATOM, _S_DENS, _S_WALK, _S_PHI, _S_ORDER, _S_W0, _S_WTRUE, _S_NOISE = range(9)


def _rng(cfg_seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg_seed, stream]))


@dataclasses.dataclass
class Connectome:
    """One synthetic problem.  Arrays are host numpy arrays.

    D is float32 of shape (n_atoms, n_theta) in C order, i.e. flat index
    theta + n_theta*atom.  Signals y, b, noise have length n_theta*n_voxels with
    flat index theta + n_theta*voxel.
    """
    name: str
    n_theta: int
    n_atoms: int
    n_voxels: int
    n_fascicles: int
    atom: np.ndarray       # int16  [nnz]
    voxel: np.ndarray      # int32  [nnz]
    fascicle: np.ndarray   # int32  [nnz]
    phi: np.ndarray        # float32[nnz]
    D: np.ndarray          # float32[n_atoms, n_theta]
    w0: np.ndarray         # float32[n_fascicles], U(0,1)
    w_true: np.ndarray     # float32[n_fascicles], U(0,1)
    noise: np.ndarray      # float32[n_theta*n_voxels], N(0,1); scaled by the consumer
    grid: Tuple[int, int, int]
    voxel_xyz: np.ndarray  # int16 [n_voxels, 3] grid coordinates of each voxel

    @property
    def nnz(self) -> int:
        return int(self.atom.shape[0])

    def occupancy(self) -> np.ndarray:
        return np.bincount(self.voxel, minlength=self.n_voxels)

    def summary(self) -> dict:
        occ = self.occupancy()
        flen = np.bincount(self.fascicle, minlength=self.n_fascicles)
        return {
            "name": self.name, "n_theta": self.n_theta, "n_atoms": self.n_atoms,
            "n_voxels": self.n_voxels, "n_fascicles": self.n_fascicles, "nnz": self.nnz,
            "occ_mean": float(occ.mean()), "occ_max": int(occ.max()),
            "occ_p99": float(np.percentile(occ, 99)), "occ_empty": int((occ == 0).sum()),
            "fas_len_mean": float(flen.mean()), "fas_len_max": int(flen.max()),
            "fas_empty": int((flen == 0).sum()),
        }


# ----------------------------------------------------------------------------- geometry

def _unit(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def fibonacci_sphere(n: int) -> np.ndarray:
    """n nearly uniform points on the unit sphere (golden-angle spiral)."""
    k = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * k / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def make_dictionary(g: np.ndarray, u: np.ndarray, bval: float) -> np.ndarray:
    """D[a, theta] = exp(-bval (g_theta . u_a)^2) - mean_theta(...)  (float64)."""
    e = np.exp(-bval * (u @ g.T) ** 2)           # [Na, Ntheta]
    return e - e.mean(axis=1, keepdims=True)


def _cube_lut(u: np.ndarray, res: int) -> np.ndarray:
    """Nearest atom (max |t.u_a|) for the centre of every cube-map cell."""
    s = (np.arange(res) + 0.5) / res * 2.0 - 1.0
    aa, bb = np.meshgrid(s, s, indexing="ij")
    one = np.ones_like(aa)
    faces = []
    for axis in range(3):
        for sign in (1.0, -1.0):
            comps = [None, None, None]
            comps[axis] = sign * one
            others = [i for i in range(3) if i != axis]
            comps[others[0]] = aa
            comps[others[1]] = bb
            faces.append(np.stack(comps, axis=-1).reshape(-1, 3))
    dirs = np.concatenate(faces)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    lut = np.empty(dirs.shape[0], dtype=np.int16)
    for lo in range(0, dirs.shape[0], 8192):
        lut[lo:lo + 8192] = np.argmax(np.abs(dirs[lo:lo + 8192] @ u.T), axis=1)
    return lut


def _cube_cell(t: np.ndarray, res: int) -> np.ndarray:
    """Index of the cube-map cell containing direction t (rows of t)."""
    at = np.abs(t)
    axis = np.argmax(at, axis=1)
    n = t.shape[0]
    ridx = np.arange(n)
    major = t[ridx, axis]
    face = axis * 2 + (major < 0)
    o0 = np.where(axis == 0, 1, 0)
    o1 = np.where(axis == 2, 1, 2)
    denom = np.abs(major)
    a = t[ridx, o0] / denom
    b = t[ridx, o1] / denom
    ia = np.clip(((a + 1.0) * 0.5 * res).astype(np.int64), 0, res - 1)
    ib = np.clip(((b + 1.0) * 0.5 * res).astype(np.int64), 0, res - 1)
    return face * res * res + ia * res + ib


def _mask(cfg: Config) -> np.ndarray:
    nx, ny, nz = cfg.grid
    if cfg.semi_axes is None:
        return np.ones((nz, ny, nx), dtype=bool)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cx, cy, cz = (nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0
    ax, ay, az = cfg.semi_axes
    return ((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2 + ((z - cz) / az) ** 2 <= 1.0


def _density(cfg: Config, mask: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Start-point weights over mask voxels: exp(sigma * smoothed unit Gaussian field)."""
    if cfg.density_sigma <= 0:
        return np.ones(int(mask.sum()))
    from scipy.ndimage import gaussian_filter
    f = gaussian_filter(rng.standard_normal(mask.shape), cfg.density_smooth, mode="wrap")
    f = (f - f.mean()) / f.std()
    return np.exp(cfg.density_sigma * f)[mask]


def _rotate(d: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Turn each direction by an angle U(0, 30 deg) about a random perpendicular axis."""
    r = rng.standard_normal(d.shape)
    r -= np.sum(r * d, axis=1, keepdims=True) * d
    r /= np.maximum(np.linalg.norm(r, axis=1, keepdims=True), 1e-30)
    ang = rng.uniform(0.0, MAX_TURN, size=(d.shape[0], 1))
    out = np.cos(ang) * d + np.sin(ang) * r
    return out / np.linalg.norm(out, axis=1, keepdims=True)


def _walks(cfg: Config, mask: np.ndarray, vid: np.ndarray, lut: np.ndarray,
           density: np.ndarray, rng: np.random.Generator):
    """Trace all fascicles; return (fascicle, voxel, atom) of every visited pair."""
    nz, ny, nx = mask.shape
    nf = cfg.n_fascicles
    mask_flat = np.flatnonzero(mask.ravel())
    p = density / density.sum()
    start = mask_flat[rng.choice(mask_flat.shape[0], size=nf, p=p)]
    sz, rem = np.divmod(start, ny * nx)
    sy, sx = np.divmod(rem, nx)
    pos = np.stack([sx, sy, sz], axis=1).astype(np.float64) + rng.uniform(0.0, 1.0, (nf, 3))
    d0 = _unit(rng, nf)
    lo, hi = cfg.steps
    if cfg.length_dist == "uniform":
        nsteps = rng.integers(lo, hi + 1, size=nf)
    else:
        nsteps = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi + 1), size=nf))).astype(np.int64)
    # a fascicle is traced from its seed point forwards and backwards; the two
    # halves share the step budget, and the backward half starts one step out
    fwd = (nsteps + 1) // 2
    fid = np.concatenate([np.arange(nf), np.arange(nf)]).astype(np.int64)
    nsteps = np.concatenate([fwd, nsteps - fwd])
    d = np.concatenate([d0, -d0])
    pos = np.concatenate([pos, pos - STEP * d0])
    last = np.full(2 * nf, -1, dtype=np.int64)
    out_f, out_v, out_a = [], [], []
    step = 0
    while fid.shape[0]:
        ix = np.floor(pos).astype(np.int64)
        inside = np.all((ix >= 0) & (ix < np.array([nx, ny, nz])), axis=1)
        v = np.full(fid.shape[0], -1, dtype=np.int64)
        ii = np.flatnonzero(inside)
        v[ii] = vid[ix[ii, 2], ix[ii, 1], ix[ii, 0]]
        alive = (v >= 0) & (step < nsteps)
        new = alive & (v != last)
        if new.any():
            out_f.append(fid[new].astype(np.int32))
            out_v.append(v[new].astype(np.int32))
            out_a.append(lut[_cube_cell(d[new], LUT_RES)])
        keep = np.flatnonzero(alive)
        fid, pos, d, last, nsteps = fid[keep], pos[keep], d[keep], v[keep], nsteps[keep]
        d = _rotate(d, rng)
        pos = pos + STEP * d
        step += 1
    f = np.concatenate(out_f)
    v = np.concatenate(out_v)
    a = np.concatenate(out_a)
    return f, v, a


def make(name: str, n_fascicles: Optional[int] = None) -> Connectome:
    """Build configuration ``name`` deterministically from its seed.

    ``n_fascicles`` optionally overrides the fascicle count (same seeds; used for
    reduced variants of a configuration in tests).  If the environment variable
    LIFE_SYNTH_CACHE names a directory, the arrays are cached there as .npz
    (written by this function only, read back with allow_pickle=False).
    """
    cache = os.environ.get("LIFE_SYNTH_CACHE")
    if cache:
        path = os.path.join(cache, f"{name}_{n_fascicles or 'default'}_v1.npz")
        if os.path.exists(path):
            with np.load(path, allow_pickle=False) as z:
                meta = z["meta"]
                return Connectome(name=name, n_theta=int(meta[0]), n_atoms=int(meta[1]), n_voxels=int(meta[2]),
                                  n_fascicles=int(meta[3]), grid=(int(meta[4]), int(meta[5]), int(meta[6])),
                                  **{k: z[k] for k in _ARRAYS})
        c = _make(name, n_fascicles)
        os.makedirs(cache, exist_ok=True)
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, meta=np.array([c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, *c.grid]),
                 **{k: getattr(c, k) for k in _ARRAYS})
        os.replace(tmp, path)
        return c
    return _make(name, n_fascicles)


_ARRAYS = ("atom", "voxel", "fascicle", "phi", "D", "w0", "w_true", "noise", "voxel_xyz")


def _make(name: str, n_fascicles: Optional[int]) -> Connectome:
    cfg = CONFIGS[name]
    if n_fascicles is not None:
        cfg = dataclasses.replace(cfg, n_fascicles=int(n_fascicles))
    return _make_cfg(cfg)


def _make_cfg(cfg: Config) -> Connectome:
    name, seed = cfg.name, cfg.seed
    g = _unit(_rng(cfg.dict_seed if cfg.dict_seed is not None else seed, _S_GRAD), cfg.n_theta)
    if cfg.atoms == "fibonacci":
        u = fibonacci_sphere(cfg.n_atoms)
    else:
        u = _unit(_rng(seed, _S_ATOM), cfg.n_atoms)
    D = make_dictionary(g, u, cfg.bval).astype(np.float32)

    mask = _mask(cfg)
    nv = int(mask.sum())
    vid = np.full(mask.shape, -1, dtype=np.int64)
    vid[mask] = np.arange(nv)
    zz, yy, xx = np.nonzero(mask)                 # raster order, x fastest
    voxel_xyz = np.stack([xx, yy, zz], axis=1).astype(np.int16)

    lut = _cube_lut(u, LUT_RES)
    density = _density(cfg, mask, _rng(seed, _S_DENS))
    f, v, a = _walks(cfg, mask, vid, lut, density, _rng(seed, _S_WALK))

    # one nonzero per (fascicle, voxel): keep the first visit
    key = f.astype(np.int64) * nv + v
    _, first = np.unique(key, return_index=True)
    first.sort()
    f, v, a = f[first], v[first], a[first]
    nnz = f.shape[0]
    phi = _rng(seed, _S_PHI).uniform(PHI_LO, PHI_HI, size=nnz).astype(np.float32)
    order = _rng(seed, _S_ORDER).permutation(nnz)

    nf = cfg.n_fascicles
    return Connectome(
        name=name, n_theta=cfg.n_theta, n_atoms=cfg.n_atoms, n_voxels=nv, n_fascicles=nf,
        atom=np.ascontiguousarray(a[order].astype(np.int16)),
        voxel=np.ascontiguousarray(v[order].astype(np.int32)),
        fascicle=np.ascontiguousarray(f[order].astype(np.int32)),
        phi=np.ascontiguousarray(phi[order]),
        D=np.ascontiguousarray(D),
        w0=_rng(seed, _S_W0).uniform(0.0, 1.0, nf).astype(np.float32),
        w_true=_rng(seed, _S_WTRUE).uniform(0.0, 1.0, nf).astype(np.float32),
        noise=_rng(seed, _S_NOISE).standard_normal(cfg.n_theta * nv).astype(np.float32),
        grid=cfg.grid, voxel_xyz=voxel_xyz,
    )


def make_batch(n_inst: int = 32, seed: int = 7, scale: float = 1.0,
               nv_range: Tuple[int, int] = (30_000, 150_000), nf_range: Tuple[int, int] = (20_000, 400_000),
               steps: Tuple[int, int] = (20, 120)) -> list:
    """Uneven instances that share one dictionary (the mid configuration's: 96
    directions, 1057 Fibonacci atoms).  Instance k has an ellipsoidal mask of
    about U(nv_range)*scale voxels and log-uniform(nf_range)*scale fascicles of
    uniform(steps) walk steps; each instance has its own seeds."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 99]))
    base = CONFIGS["mid"]
    out = []
    for k in range(n_inst):
        nv = max(64, int(rng.uniform(*nv_range) * scale))
        nf = max(16, int(np.exp(rng.uniform(np.log(nf_range[0]), np.log(nf_range[1]))) * scale))
        r = (nv / (4.0 / 3.0 * math.pi * 0.95 * 0.9)) ** (1.0 / 3.0)
        n = int(math.ceil(2 * r + 2))
        cfg = dataclasses.replace(base, name=f"batch{seed}_{k}", grid=(n, n, n),
                                  semi_axes=(r, 0.95 * r, 0.9 * r), n_fascicles=nf, steps=steps,
                                  seed=1000 * seed + k, dict_seed=base.seed)
        out.append(_make_cfg(cfg))
    return out


def random_coo(n_theta: int, n_atoms: int, n_voxels: int, n_fascicles: int, nnz: int,
               seed: int, duplicates: bool = False) -> Connectome:
    """Unstructured random problem of any shape (edge cases, ragged sizes).

    Indices are uniform; with ``duplicates`` some (atom, voxel, fascicle) tuples
    repeat, which COO semantics sum.
    """
    rng = _rng(seed, 100)
    atom = rng.integers(0, max(n_atoms, 1), size=nnz).astype(np.int16)
    voxel = rng.integers(0, max(n_voxels, 1), size=nnz).astype(np.int32)
    fas = rng.integers(0, max(n_fascicles, 1), size=nnz).astype(np.int32)
    if duplicates and nnz >= 4:
        k = nnz // 4
        src = rng.integers(0, nnz - k, size=k)
        atom[nnz - k:] = atom[src]
        voxel[nnz - k:] = voxel[src]
        fas[nnz - k:] = fas[src]
    D = rng.standard_normal((n_atoms, n_theta)).astype(np.float32)
    D -= D.mean(axis=1, keepdims=True)
    return Connectome(
        name=f"random{seed}", n_theta=n_theta, n_atoms=n_atoms, n_voxels=n_voxels,
        n_fascicles=n_fascicles, atom=atom, voxel=voxel, fascicle=fas,
        phi=rng.uniform(PHI_LO, PHI_HI, size=nnz).astype(np.float32),
        D=np.ascontiguousarray(D),
        w0=rng.uniform(0.0, 1.0, n_fascicles).astype(np.float32),
        w_true=rng.uniform(0.0, 1.0, n_fascicles).astype(np.float32),
        noise=rng.standard_normal(n_theta * n_voxels).astype(np.float32),
        grid=(n_voxels, 1, 1), voxel_xyz=np.zeros((n_voxels, 3), dtype=np.int16),
    )
