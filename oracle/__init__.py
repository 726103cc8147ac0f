"""FP64 CPU oracle for the LiFE hot path (DSC, WC, one SBB-NNLS iteration).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP library and never imports it; the two meet only through the seeded
inputs of the separate ``synth`` package.

What is computed and where it comes from (arxiv 1905.06234):

* ``dsc``  - y = M w, eq. 1, with M encoded by the sparse Tucker decomposition
  M_v = S0(v) D Phi_v (eq. 3) / Y = Phi x1 D x2 S0 x3 w^T (eq. 4).  S0 is folded
  into the Phi values.  Plain C loop over the nonzeros in input order
  (``life_oracle.c``), double precision.
* ``wc``   - g = M^T y, the transpose product inside the gradient of eq. 6.
* ``dd``   - d<ybar, M(D) w>/dD, the derivative of the DSC product with respect
  to the dictionary (y is linear in D through eq. 3/4); ``loss_grads`` gives
  both gradients of ||y_obs - M(D) w||^2.  The paper fits w only; this serves
  dictionary learning through the same encoding.
* ``sbb_step`` - one iteration of SBB-NNLS in the matrix form of Algorithm 1
  (Sec. 2.1), with these readings of points the text leaves open:
    - iterations are counted from i = 0; odd i uses alpha = <g~,g~>/<Mg~,Mg~>,
      even i uses alpha = <Mg~,Mg~>/<M^T M g~, M^T M g~> (Algorithm 1 (a)/(b);
      eqs. 7-8 assign the two formulas to the opposite parities and evaluate them
      at the previous iterate - the ``lagged`` variant below follows eqs. 7-8);
    - the "projected" gradient g~ keeps g_f where w_f > 0 or g_f < 0 and zeroes
      it where the weight sits on the bound and the gradient would push it out
      (the subspace of the method); the update of eq. 5 uses g~, which gives the
      same w for alpha > 0 as using the raw gradient;
    - a zero denominator gives alpha = 0 (g~ = 0: a KKT point, w unchanged);
    - the projection [x]_+ returns +0.0 for x <= 0.
  The objective reported is f(w) = 1/2 ||M w - b||^2 of eq. 2 at the incoming w.

Every array the oracle returns is float64.  Inputs may be float32 (as the HIP
path receives them); they are converted exactly to float64 first.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "life_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC_PAR = os.path.join(_HERE, "life_oracle_par.c")
_LIB_PAR = os.path.join(_HERE, "liboracle_par.so")
_lib = None
_lib_par = None


def _gcc(src: str, lib: str, force: bool, extra=()) -> str:
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        tmp = lib + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                        "-ffp-contract=off", *extra, src, "-o", tmp], check=True)
        os.replace(tmp, lib)
    return lib


def build(force: bool = False) -> str:
    """Compile life_oracle.c (plain -O2, no fast-math, sequential) and the
    multi-threaded life_oracle_par.c (the same, with OpenMP) with gcc."""
    _gcc(_SRC_PAR, _LIB_PAR, force, ("-fopenmp",))
    return _gcc(_SRC, _LIB, force)


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        for name in ("oracle_dsc", "oracle_wc", "oracle_dd"):
            fn = getattr(lib, name)
            fn.restype = None
            fn.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _load_par():
    global _lib_par
    if _lib_par is None:
        build()
        lib = ctypes.CDLL(_LIB_PAR)
        P = ctypes.c_void_p
        lib.oracle_par_new.restype = P
        lib.oracle_par_new.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P, P]
        lib.oracle_par_free.restype = None
        lib.oracle_par_free.argtypes = [P]
        for name in ("oracle_par_dsc", "oracle_par_wc"):
            fn = getattr(lib, name)
            fn.restype = None
            fn.argtypes = [P, P, P, P]
        lib.oracle_par_threads.restype = ctypes.c_int
        lib.oracle_par_threads.argtypes = []
        _lib_par = lib
    return _lib_par


def par_threads() -> int:
    """OpenMP threads the multi-threaded oracle runs with (OMP_NUM_THREADS, else all cores)."""
    return int(_load_par().oracle_par_threads())


@dataclass
class Operator:
    """The encoded matrix M: Phi nonzeros (input order) plus the dictionary D.

    D has shape (n_atoms, n_theta), i.e. flat index theta + n_theta*atom.
    """
    atom: np.ndarray
    voxel: np.ndarray
    fascicle: np.ndarray
    phi: np.ndarray
    D: np.ndarray
    n_voxels: int
    n_fascicles: int
    _phi64: np.ndarray = field(init=False, repr=False)
    _D64: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        self.atom = np.ascontiguousarray(self.atom, dtype=np.int16)
        self.voxel = np.ascontiguousarray(self.voxel, dtype=np.int32)
        self.fascicle = np.ascontiguousarray(self.fascicle, dtype=np.int32)
        self._phi64 = np.ascontiguousarray(self.phi, dtype=np.float64)
        self._D64 = np.ascontiguousarray(self.D, dtype=np.float64)
        if self._D64.ndim != 2:
            raise ValueError("D must be (n_atoms, n_theta)")

    @classmethod
    def from_connectome(cls, c) -> "Operator":
        return cls(c.atom, c.voxel, c.fascicle, c.phi, c.D, c.n_voxels, c.n_fascicles)

    @property
    def n_theta(self) -> int:
        return int(self._D64.shape[1])

    @property
    def nnz(self) -> int:
        return int(self.atom.shape[0])

    def subset(self, mask: np.ndarray) -> "Operator":
        """The operator restricted to the nonzeros selected by ``mask``."""
        return Operator(self.atom[mask], self.voxel[mask], self.fascicle[mask],
                        self._phi64[mask], self._D64, self.n_voxels, self.n_fascicles)

    def dsc(self, w: np.ndarray) -> np.ndarray:
        """y = M w (length n_theta*n_voxels, theta fastest)."""
        w64 = np.ascontiguousarray(w, dtype=np.float64)
        if w64.shape != (self.n_fascicles,):
            raise ValueError("w has the wrong length")
        y = np.empty(self.n_theta * self.n_voxels, dtype=np.float64)
        _load().oracle_dsc(self.nnz, self.n_theta, self.n_voxels, _ptr(self.atom), _ptr(self.voxel),
                           _ptr(self.fascicle), _ptr(self._phi64), _ptr(self._D64), _ptr(w64), _ptr(y))
        return y

    def wc(self, y: np.ndarray) -> np.ndarray:
        """g = M^T y (length n_fascicles)."""
        y64 = np.ascontiguousarray(y, dtype=np.float64)
        if y64.shape != (self.n_theta * self.n_voxels,):
            raise ValueError("y has the wrong length")
        g = np.empty(self.n_fascicles, dtype=np.float64)
        _load().oracle_wc(self.nnz, self.n_theta, self.n_fascicles, _ptr(self.atom), _ptr(self.voxel),
                          _ptr(self.fascicle), _ptr(self._phi64), _ptr(self._D64), _ptr(y64), _ptr(g))
        return g

    def dd(self, w: np.ndarray, ybar: np.ndarray) -> np.ndarray:
        """d<ybar, M(D) w>/dD, shape (n_atoms, n_theta) like D."""
        w64 = np.ascontiguousarray(w, dtype=np.float64)
        y64 = np.ascontiguousarray(ybar, dtype=np.float64)
        if w64.shape != (self.n_fascicles,) or y64.shape != (self.n_theta * self.n_voxels,):
            raise ValueError("w or ybar has the wrong length")
        na = int(self._D64.shape[0])
        dD = np.empty((na, self.n_theta), dtype=np.float64)
        _load().oracle_dd(self.nnz, self.n_theta, na, _ptr(self.atom), _ptr(self.voxel), _ptr(self.fascicle),
                          _ptr(self._phi64), _ptr(w64), _ptr(y64), _ptr(dD))
        return dD

    def parallel(self) -> "ParOperator":
        """The multi-threaded form of this operator (same results, bit for bit)."""
        return ParOperator(self)

    def with_dictionary(self, D: np.ndarray) -> "Operator":
        """The same nonzeros with another dictionary."""
        return Operator(self.atom, self.voxel, self.fascicle, self._phi64, D, self.n_voxels, self.n_fascicles)

    def loss(self, w: np.ndarray, y_obs: np.ndarray) -> float:
        """L = ||y_obs - M w||^2 (no 1/2), the dictionary-fitting loss."""
        r = self.dsc(w) - np.asarray(y_obs, dtype=np.float64)
        return float(r @ r)

    def loss_grads(self, w: np.ndarray, y_obs: np.ndarray):
        """(dL/dD, dL/dw) of L = ||y_obs - M(D) w||^2: with r = M w - y_obs,
        dL/dw = 2 M^T r and dL/dD = 2 dd(w, r)."""
        r = self.dsc(w) - np.asarray(y_obs, dtype=np.float64)
        return 2.0 * self.dd(w, r), 2.0 * self.wc(r)

    def objective(self, w: np.ndarray, b: np.ndarray) -> float:
        """f(w) = 1/2 ||M w - b||^2  (eq. 2)."""
        r = self.dsc(w) - np.asarray(b, dtype=np.float64)
        return 0.5 * float(r @ r)


class ParOperator:
    """The same products as ``Operator.dsc`` / ``Operator.wc`` on OpenMP threads
    (life_oracle_par.c): the nonzeros are grouped once by voxel and by fascicle
    with a stable counting sort, so each output entry gets the additions of the
    sequential loop in the same order, and the results are equal bit for bit."""

    def __init__(self, op: Operator):
        self.op = op
        lib = _load_par()
        self._h = lib.oracle_par_new(op.nnz, op.n_theta, op.n_voxels, op.n_fascicles, _ptr(op.atom),
                                     _ptr(op.voxel), _ptr(op.fascicle), _ptr(op._phi64))
        if not self._h:
            raise MemoryError("oracle_par_new failed")

    def close(self):
        if self._h:
            _load_par().oracle_par_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dsc(self, w: np.ndarray) -> np.ndarray:
        op = self.op
        w64 = np.ascontiguousarray(w, dtype=np.float64)
        if w64.shape != (op.n_fascicles,):
            raise ValueError("w has the wrong length")
        y = np.empty(op.n_theta * op.n_voxels, dtype=np.float64)
        _load_par().oracle_par_dsc(self._h, _ptr(op._D64), _ptr(w64), _ptr(y))
        return y

    def wc(self, y: np.ndarray) -> np.ndarray:
        op = self.op
        y64 = np.ascontiguousarray(y, dtype=np.float64)
        if y64.shape != (op.n_theta * op.n_voxels,):
            raise ValueError("y has the wrong length")
        g = np.empty(op.n_fascicles, dtype=np.float64)
        _load_par().oracle_par_wc(self._h, _ptr(op._D64), _ptr(y64), _ptr(g))
        return g


@dataclass
class StepResult:
    w: np.ndarray          # w^(i+1)
    alpha: float           # alpha^(i)
    f: float               # f(w^(i)) = 1/2 ||M w^(i) - b||^2
    gt_norm2: float        # ||g~||^2 at w^(i)
    num: float             # numerator of alpha
    den: float             # denominator of alpha
    n_dsc: int             # M w products evaluated in this step
    n_wc: int              # M^T y products evaluated in this step
    gt: np.ndarray         # projected gradient g~


def projected_gradient(w: np.ndarray, g: np.ndarray) -> np.ndarray:
    """g~: keep g_f unless w_f is on the bound and g_f would push it below zero."""
    return np.where((w > 0) | (g < 0), g, 0.0)


def sbb_step(op: Operator, w: np.ndarray, i: int, b: np.ndarray) -> StepResult:
    """One SBB-NNLS iteration (Algorithm 1 reading, see module docstring)."""
    w = np.asarray(w, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = op.dsc(w) - b                       # y = M w^(i) - b
    f = 0.5 * float(r @ r)
    g = op.wc(r)                            # w' = M^T y  (= grad f, eq. 6)
    gt = projected_gradient(w, g)
    vp = op.dsc(gt)                         # v' = M w'
    n_dsc, n_wc = 2, 1
    if i % 2 == 1:                          # (a) odd iteration
        num, den = float(gt @ gt), float(vp @ vp)
    else:                                   # (b) even iteration
        vpp = op.wc(vp)                     # v'' = M^T v'
        n_wc += 1
        num, den = float(vp @ vp), float(vpp @ vpp)
    alpha = num / den if den > 0.0 else 0.0
    x = w - alpha * gt                      # eq. 5
    w_next = np.where(x > 0.0, x, 0.0)
    return StepResult(w_next, alpha, f, float(gt @ gt), num, den, n_dsc, n_wc, gt)


def sbb_step_lagged(op: Operator, w: np.ndarray, i: int, b: np.ndarray,
                    gt_prev: Optional[np.ndarray]) -> StepResult:
    """Variant that follows eqs. 7-8 literally: alpha^(i) is evaluated at the
    projected gradient of the previous iterate (classic lagged Barzilai-Borwein),
    eq. 7 on even i and eq. 8 on odd i.  At i = 0 (no previous gradient) the
    current one is used."""
    w = np.asarray(w, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = op.dsc(w) - b
    f = 0.5 * float(r @ r)
    g = op.wc(r)
    gt = projected_gradient(w, g)
    q = gt if gt_prev is None else np.asarray(gt_prev, dtype=np.float64)
    mq = op.dsc(q)
    n_dsc, n_wc = 2, 1
    if i % 2 == 0:
        num, den = float(q @ q), float(mq @ mq)
    else:
        mtmq = op.wc(mq)
        n_wc += 1
        num, den = float(mq @ mq), float(mtmq @ mtmq)
    alpha = num / den if den > 0.0 else 0.0
    x = w - alpha * gt
    w_next = np.where(x > 0.0, x, 0.0)
    return StepResult(w_next, alpha, f, float(gt @ gt), num, den, n_dsc, n_wc, gt)


def sbb_run(op: Operator, w0: np.ndarray, b: np.ndarray, n_iter: int):
    """n_iter iterations from w0; returns (w, list of StepResult)."""
    w = np.asarray(w0, dtype=np.float64)
    hist = []
    for i in range(n_iter):
        s = sbb_step(op, w, i, b)
        hist.append(s)
        w = s.w
    return w, hist


def noisy_signal(op: Operator, w_true: np.ndarray, noise: np.ndarray, level: float = 0.05) -> np.ndarray:
    """b = M w_true + level * RMS(M w_true) * noise  (float64)."""
    y = op.dsc(w_true)
    rms = float(np.sqrt(np.mean(y * y))) if y.size else 0.0
    return y + level * rms * np.asarray(noise, dtype=np.float64)
