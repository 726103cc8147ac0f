"""Python binding of liblife.so: argument marshalling only.

Every computation runs in the HIP library; this module checks shapes, dtypes and
devices, passes raw device pointers and the current HIP stream, and turns status
codes into exceptions.  PyTorch serves only as the owner of device memory and
streams.  If the library is not built, every entry point raises: there is no
fallback path.

Function names follow the C ABI in include/life.h.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblife.so")

KERNELS = ("dsc", "wc_z", "wc_sum", "mask", "alpha", "update", "wc_z_2nd", "wc_sum_2nd", "permute", "dd",
           "dd_reduce")
STATUS = {0: "LIFE_OK", 1: "LIFE_EINVAL", 2: "LIFE_ERANGE", 3: "LIFE_ENOMEM", 4: "LIFE_EDEVICE"}
STATE_FIELDS = ("iter", "alpha", "obj", "gt_norm2", "num", "den")
PLAN_DEVICE_INPUT = 1   # life_plan_flags: the COO arrays are device memory
PLAN_HOST_BUILD = 2     # life_plan_flags: restructure on the host (the reference builder)
DIGEST_WORDS = 24


class LifeError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"{fn} failed: {STATUS.get(status, status)} {msg}".strip())


class Dims(ctypes.Structure):
    _fields_ = [("n_theta", ctypes.c_int32), ("n_atoms", ctypes.c_int32), ("n_voxels", ctypes.c_int32),
                ("n_fascicles", ctypes.c_int32), ("nnz", ctypes.c_int64)]


class SbbState(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int64), ("alpha", ctypes.c_double), ("obj", ctypes.c_double),
                ("gt_norm2", ctypes.c_double), ("num", ctypes.c_double), ("den", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_SIGS = {
    "life_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "life_hip_error": (ctypes.c_char_p, []),
    "life_plan_host": (ctypes.c_int, [ctypes.POINTER(Dims), _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "life_plan": (ctypes.c_int, [ctypes.POINTER(Dims), _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "life_plan_ex": (ctypes.c_int, [ctypes.POINTER(Dims), _P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "life_plan_batch": (ctypes.c_int, [ctypes.POINTER(Dims), ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P,
                                       ctypes.POINTER(_P)]),
    "life_plan_instances": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "life_plan_flags": (ctypes.c_int, [ctypes.POINTER(Dims), ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P,
                                       ctypes.c_uint32, ctypes.c_int32, ctypes.POINTER(_P)]),
    "life_plan_tile_atoms": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "life_plan_autotune": (ctypes.c_int, [ctypes.POINTER(Dims), ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P,
                                          ctypes.c_uint32, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_P)]),
    "life_plan_digest": (ctypes.c_int, [_P, _P]),
    "life_plan_host_batch": (ctypes.c_int, [ctypes.POINTER(Dims), ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P,
                                            _P, _P, _P, _P]),
    "life_plan_tune": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "life_sbbnnls_step_batch": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "life_plan_destroy": (ctypes.c_int, [_P]),
    "life_plan_dims": (ctypes.c_int, [_P, ctypes.POINTER(Dims)]),
    "life_plan_export": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "life_dsc": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "life_wc": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "life_sbbnnls_step": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "life_plan_scratch_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    "life_dsc_ws": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_uint64, _P]),
    "life_wc_ws": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_uint64, _P]),
    "life_sbbnnls_step_ws": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.c_uint64, _P]),
    "life_dsc_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "life_sbbnnls_step_lagged": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "life_dict_grad": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "life_profile_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "life_profile_read": (ctypes.c_int, [_P, _P, _P]),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblife.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(fn: str, status: int):
    if status != 0:
        detail = load().life_hip_error().decode() if status == 4 else ""
        raise LifeError(fn, status, detail)


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _coo(atom, voxel, fascicle):
    atom = np.ascontiguousarray(atom, dtype=np.int16)
    voxel = np.ascontiguousarray(voxel, dtype=np.int32)
    fascicle = np.ascontiguousarray(fascicle, dtype=np.int32)
    if not (atom.ndim == voxel.ndim == fascicle.ndim == 1 and atom.shape == voxel.shape == fascicle.shape):
        raise ValueError("atom, voxel, fascicle must be 1-D arrays of one length")
    return atom, voxel, fascicle


def _xyz(voxel_xyz, n_voxels: int):
    if voxel_xyz is None:
        return None
    xyz = np.ascontiguousarray(voxel_xyz, dtype=np.int16)
    if xyz.shape != (max(n_voxels, 0), 3):
        raise ValueError("voxel_xyz must have shape (n_voxels, 3)")
    return xyz


def plan_host(n_theta: int, n_atoms: int, n_voxels: int, n_fascicles: int, atom, voxel, fascicle,
              voxel_xyz=None) -> Dict[str, np.ndarray]:
    """Host-only restructuring (life_plan_host): permutations and segment offsets."""
    atom, voxel, fascicle = _coo(atom, voxel, fascicle)
    xyz = _xyz(voxel_xyz, n_voxels)
    nnz = atom.shape[0]
    d = Dims(n_theta, n_atoms, n_voxels, n_fascicles, nnz)
    out = {"dsc_perm": np.empty(nnz, np.int32), "vox_ptr": np.empty(max(n_voxels, 0) + 1, np.int32),
           "fas_rank": np.empty(max(n_fascicles, 0), np.int32), "wc_perm": np.empty(nnz, np.int32),
           "fas_ptr": np.empty(max(n_fascicles, 0) + 1, np.int32)}
    _check("life_plan_host", load().life_plan_host(ctypes.byref(d), _np_ptr(atom), _np_ptr(voxel),
                                                   _np_ptr(fascicle), _np_ptr(xyz), _np_ptr(out["dsc_perm"]),
                                                   _np_ptr(out["vox_ptr"]), _np_ptr(out["fas_rank"]),
                                                   _np_ptr(out["wc_perm"]), _np_ptr(out["fas_ptr"])))
    return out


def concat_instances(instances, morton: bool = True):
    """Union COO of problems sharing a dictionary: (dims, vox_off, fas_off, atom,
    voxel, fascicle, phi, voxel_xyz or None), instances concatenated in order."""
    inst = list(instances)
    if not inst:
        raise ValueError("no instances")
    nt, na = inst[0].n_theta, inst[0].n_atoms
    if any(c.n_theta != nt or c.n_atoms != na for c in inst):
        raise ValueError("instances must share the dictionary shape")
    vox_off = np.zeros(len(inst) + 1, np.int32)
    fas_off = np.zeros(len(inst) + 1, np.int32)
    vox_off[1:] = np.cumsum([c.n_voxels for c in inst])
    fas_off[1:] = np.cumsum([c.n_fascicles for c in inst])
    atom = np.concatenate([np.asarray(c.atom, np.int16) for c in inst])
    voxel = np.concatenate([np.asarray(c.voxel, np.int64) + vox_off[k] for k, c in enumerate(inst)])
    fascicle = np.concatenate([np.asarray(c.fascicle, np.int64) + fas_off[k] for k, c in enumerate(inst)])
    phi = np.ascontiguousarray(np.concatenate([np.asarray(c.phi, np.float32) for c in inst]))
    atom, voxel, fascicle = _coo(atom, voxel, fascicle)
    xyz = None
    if morton:
        xyz = _xyz(np.concatenate([np.asarray(c.voxel_xyz, np.int16) for c in inst]), int(vox_off[-1]))
    dims = Dims(nt, na, int(vox_off[-1]), int(fas_off[-1]), atom.shape[0])
    return dims, vox_off, fas_off, atom, voxel, fascicle, phi, xyz


def plan_host_batch(instances, morton: bool = True, raw=None) -> Dict[str, np.ndarray]:
    """Host-only restructuring of a batched plan (life_plan_host_batch).  raw: an
    already concatenated tuple from concat_instances (to test rejected inputs)."""
    dims, vox_off, fas_off, atom, voxel, fascicle, phi, xyz = raw or concat_instances(instances, morton)
    nnz, nv, nf = dims.nnz, dims.n_voxels, dims.n_fascicles
    out = {"proc_pos": np.empty(max(nv, 0), np.int32), "dsc_perm": np.empty(nnz, np.int32),
           "vox_ptr": np.empty(nv + 1, np.int32), "fas_rank": np.empty(nf, np.int32),
           "wc_perm": np.empty(nnz, np.int32), "fas_ptr": np.empty(nf + 1, np.int32)}
    _check("life_plan_host_batch", load().life_plan_host_batch(
        ctypes.byref(dims), len(vox_off) - 1, _np_ptr(vox_off), _np_ptr(fas_off), _np_ptr(atom), _np_ptr(voxel),
        _np_ptr(fascicle), _np_ptr(xyz), *(_np_ptr(out[k]) for k in ("proc_pos", "dsc_perm", "vox_ptr", "fas_rank",
                                                                      "wc_perm", "fas_ptr"))))
    out.update({"vox_off": vox_off, "fas_off": fas_off})
    return out


def _torch():
    import torch
    return torch


def _dev_f32(t, n: int, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous float32 tensor of {n} elements")
    return ctypes.c_void_p(t.data_ptr()) if n else None


def _stream(stream, device):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def new_state(device=None, iteration: int = 0, n: Optional[int] = None):
    """A zeroed life_sbb_state on the device (as 6 float64 slots; slot 0 is int64
    iter); n given: a contiguous array of n states (batched plans)."""
    torch = _torch()
    st = torch.zeros((n if n is not None else 1) * 6, dtype=torch.float64, device=device or "cuda")
    if iteration:
        st.view(-1, 6).view(torch.int64)[:, 0] = iteration
    return st


def read_state(state, k: Optional[int] = None) -> Dict[str, float]:
    """Fields of a state (k given: of state k of an array of states)."""
    torch = _torch()
    host = state.detach().cpu().view(-1, 6)[0 if k is None else k]
    vals = host.numpy()
    out = {kk: float(vals[i]) for i, kk in enumerate(STATE_FIELDS)}
    out["iter"] = int(host.view(torch.int64)[0])
    return out


class Plan:
    """A restructured Phi on one device (life_plan); owns its device memory."""

    def __init__(self, n_theta: int, n_atoms: int, n_voxels: int, n_fascicles: int,
                 atom, voxel, fascicle, phi, voxel_xyz=None):
        """voxel_xyz: optional (n_voxels, 3) grid coordinates; given, voxels are
        processed in Morton order (life_plan_ex)."""
        atom, voxel, fascicle = _coo(atom, voxel, fascicle)
        xyz = _xyz(voxel_xyz, n_voxels)
        phi = np.ascontiguousarray(phi, dtype=np.float32)
        if phi.shape != atom.shape:
            raise ValueError("phi must have one value per nonzero")
        self.dims = Dims(n_theta, n_atoms, n_voxels, n_fascicles, atom.shape[0])
        self._h = ctypes.c_void_p()
        lib = load()
        if xyz is None:
            _check("life_plan", lib.life_plan(ctypes.byref(self.dims), _np_ptr(atom), _np_ptr(voxel),
                                              _np_ptr(fascicle), _np_ptr(phi), ctypes.byref(self._h)))
        else:
            _check("life_plan_ex", lib.life_plan_ex(ctypes.byref(self.dims), _np_ptr(atom), _np_ptr(voxel),
                                                    _np_ptr(fascicle), _np_ptr(phi), _np_ptr(xyz),
                                                    ctypes.byref(self._h)))
        self.device = _torch().cuda.current_device()

    @classmethod
    def batch(cls, instances, morton: bool = True, host_build: bool = False) -> "Plan":
        """A batched plan (life_plan_batch) of problems sharing one dictionary.

        instances: objects with n_theta, n_atoms, n_voxels, n_fascicles, atom,
        voxel, fascicle, phi (and voxel_xyz when morton).  The union concatenates
        them in order; ``vox_off`` / ``fas_off`` give each instance's slice of the
        union's signal and weight vectors."""
        dims, vox_off, fas_off, atom, voxel, fascicle, phi, xyz = concat_instances(instances, morton)
        n_inst = len(vox_off) - 1
        self = cls.__new__(cls)
        self.dims = dims
        self._h = ctypes.c_void_p()
        if host_build:
            _check("life_plan_flags", load().life_plan_flags(
                ctypes.byref(self.dims), n_inst, _np_ptr(vox_off), _np_ptr(fas_off), _np_ptr(atom), _np_ptr(voxel),
                _np_ptr(fascicle), _np_ptr(phi), _np_ptr(xyz), PLAN_HOST_BUILD, 0, ctypes.byref(self._h)))
        else:
            _check("life_plan_batch", load().life_plan_batch(ctypes.byref(self.dims), n_inst, _np_ptr(vox_off),
                                                             _np_ptr(fas_off), _np_ptr(atom), _np_ptr(voxel),
                                                             _np_ptr(fascicle), _np_ptr(phi), _np_ptr(xyz),
                                                             ctypes.byref(self._h)))
        self.device = _torch().cuda.current_device()
        self.vox_off, self.fas_off = vox_off, fas_off
        return self

    @property
    def n_inst(self) -> int:
        n = ctypes.c_int32()
        _check("life_plan_instances", load().life_plan_instances(self._h, ctypes.byref(n)))
        return int(n.value)

    def tune(self, D, w, y, reps: int = 3) -> int:
        """Keep the fastest work schedule for this plan (life_plan_tune); returns it."""
        pol = ctypes.c_int32()
        _check("life_plan_tune", load().life_plan_tune(self._h, self._d(D), _dev_f32(w, self.dims.n_fascicles, "w"),
                                                       _dev_f32(y, self.n_signal, "y"), int(reps),
                                                       ctypes.byref(pol)))
        return int(pol.value)

    def sbbnnls_step_batch(self, D, b, w, states, stream=None):
        """One SBB-NNLS iteration of every instance; states from new_state(device, n=n_inst)."""
        torch = _torch()
        if not (isinstance(states, torch.Tensor) and states.is_cuda and states.is_contiguous()
                and states.numel() * states.element_size() == 48 * self.n_inst):
            raise ValueError("states must be a contiguous device tensor of n_inst 48-byte states (see new_state)")
        _check("life_sbbnnls_step_batch",
               load().life_sbbnnls_step_batch(self._h, self._d(D), _dev_f32(b, self.n_signal, "b"),
                                              _dev_f32(w, self.dims.n_fascicles, "w"),
                                              ctypes.c_void_p(states.data_ptr()), _stream(stream, w.device)))
        return w

    @classmethod
    def autotune(cls, instances, D, reps: int = 3, morton: bool = True) -> "Plan":
        """The fastest plan geometry for these problems (life_plan_autotune): one
        instance gives a single-problem plan, several a batched plan.  The chosen
        tiling and schedule are in ``tile_atoms`` and ``policy``."""
        dims, vox_off, fas_off, atom, voxel, fascicle, phi, xyz = concat_instances(instances, morton)
        n_inst = len(vox_off) - 1
        self = cls.__new__(cls)
        self.dims = dims
        self._h = ctypes.c_void_p()
        ta, pol = ctypes.c_int32(), ctypes.c_int32()
        _check("life_plan_autotune", load().life_plan_autotune(
            ctypes.byref(self.dims), n_inst, _np_ptr(vox_off), _np_ptr(fas_off), _np_ptr(atom), _np_ptr(voxel),
            _np_ptr(fascicle), _np_ptr(phi), _np_ptr(xyz), 0, self._d(D), int(reps), ctypes.byref(ta),
            ctypes.byref(pol), ctypes.byref(self._h)))
        self.device = _torch().cuda.current_device()
        self.vox_off, self.fas_off = vox_off, fas_off
        self.policy = int(pol.value)
        return self

    @property
    def tile_atoms(self) -> int:
        """Atoms per dictionary tile (0: generic kernels)."""
        n = ctypes.c_int32()
        _check("life_plan_tile_atoms", load().life_plan_tile_atoms(self._h, ctypes.byref(n)))
        return int(n.value)

    @classmethod
    def build(cls, n_theta: int, n_atoms: int, n_voxels: int, n_fascicles: int, atom, voxel, fascicle, phi,
              voxel_xyz=None, host_build: bool = False, device_input: bool = False, tile_atoms: int = 0) -> "Plan":
        """A single-problem plan through life_plan_flags.  host_build: restructure on
        the host (the reference builder).  atom, voxel, fascicle, phi: numpy arrays,
        or device tensors (passed as device pointers); device_input with numpy
        arrays moves them to the current device first.  tile_atoms: at most that
        many atoms per dictionary tile (0: the default tiling)."""
        torch = _torch()
        xyz = _xyz(voxel_xyz, n_voxels)
        keep = []
        if isinstance(atom, torch.Tensor):
            # device tensors (int16, int32, int32, float32, contiguous, on the current device)
            dt = (torch.int16, torch.int32, torch.int32, torch.float32)
            keep = [atom, voxel, fascicle, phi]
            n = atom.numel()
            if not all(t.is_cuda and t.is_contiguous() and t.dtype == d and t.numel() == n for t, d in zip(keep, dt)):
                raise ValueError("device COO tensors must be contiguous int16/int32/int32/float32 of one length")
            device_input = True
        else:
            atom, voxel, fascicle = _coo(atom, voxel, fascicle)
            phi = np.ascontiguousarray(phi, dtype=np.float32)
            if phi.shape != atom.shape:
                raise ValueError("phi must have one value per nonzero")
            n = atom.shape[0]
            if device_input:
                keep = [torch.from_numpy(a).cuda() for a in (atom, voxel, fascicle, phi)]
                torch.cuda.synchronize()
        self = cls.__new__(cls)
        self.dims = Dims(n_theta, n_atoms, n_voxels, n_fascicles, n)
        self._h = ctypes.c_void_p()
        flags = (PLAN_HOST_BUILD if host_build else 0) | (PLAN_DEVICE_INPUT if device_input else 0)
        if keep:
            ptrs = [ctypes.c_void_p(t.data_ptr()) if t.numel() else None for t in keep]
        else:
            ptrs = [_np_ptr(a) for a in (atom, voxel, fascicle, phi)]
        _check("life_plan_flags", load().life_plan_flags(ctypes.byref(self.dims), 1, None, None, *ptrs, _np_ptr(xyz),
                                                         flags, int(tile_atoms), ctypes.byref(self._h)))
        del keep
        self.device = torch.cuda.current_device()
        return self

    def digest(self) -> np.ndarray:
        """Per-array hashes of the plan (life_plan_digest), to compare plans bit for bit."""
        out = np.zeros(DIGEST_WORDS, np.uint64)
        _check("life_plan_digest", load().life_plan_digest(self._h, _np_ptr(out)))
        return out

    @classmethod
    def from_connectome(cls, c, morton: bool = True) -> "Plan":
        """Plan of a synthetic connectome; morton=True passes its voxel coordinates."""
        xyz = getattr(c, "voxel_xyz", None) if morton else None
        return cls(c.n_theta, c.n_atoms, c.n_voxels, c.n_fascicles, c.atom, c.voxel, c.fascicle, c.phi, xyz)

    @property
    def n_signal(self) -> int:
        return self.dims.n_theta * self.dims.n_voxels

    def close(self):
        if self._h:
            _check("life_plan_destroy", load().life_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _d(self, D):
        return _dev_f32(D, self.dims.n_theta * self.dims.n_atoms, "D")

    def scratch_bytes(self) -> int:
        """Bytes of caller scratch the *_ws calls need (life_plan_scratch_bytes)."""
        n = ctypes.c_uint64()
        _check("life_plan_scratch_bytes", load().life_plan_scratch_bytes(self._h, ctypes.byref(n)))
        return int(n.value)

    def new_scratch(self, device=None):
        """A device buffer for the scratch argument of dsc / wc / sbbnnls_step."""
        torch = _torch()
        return torch.empty(self.scratch_bytes(), dtype=torch.uint8, device=device or "cuda")

    @staticmethod
    def _scratch(scratch):
        torch = _torch()
        if not (isinstance(scratch, torch.Tensor) and scratch.is_cuda and scratch.dtype == torch.uint8
                and scratch.is_contiguous()):
            raise ValueError("scratch must be a contiguous uint8 device tensor (see new_scratch)")
        return ctypes.c_void_p(scratch.data_ptr()), ctypes.c_uint64(scratch.numel())

    def dsc(self, D, w, y=None, stream=None, scratch=None):
        """y = M w (life_dsc; life_dsc_ws with a caller scratch buffer)."""
        torch = _torch()
        if y is None:
            y = torch.empty(self.n_signal, dtype=torch.float32, device=w.device)
        args = (self._h, self._d(D), _dev_f32(w, self.dims.n_fascicles, "w"), _dev_f32(y, self.n_signal, "y"))
        if scratch is None:
            _check("life_dsc", load().life_dsc(*args, _stream(stream, w.device)))
        else:
            _check("life_dsc_ws", load().life_dsc_ws(*args, *self._scratch(scratch), _stream(stream, w.device)))
        return y

    def dsc_noalloc(self, D, w, y, stream=None):
        """y = M w into a given y with the library's static scratch (life_dsc_noalloc)."""
        _check("life_dsc_noalloc", load().life_dsc_noalloc(self._h, self._d(D), _dev_f32(w, self.dims.n_fascicles, "w"),
                                                           _dev_f32(y, self.n_signal, "y"), _stream(stream, w.device)))
        return y

    def wc(self, D, y, g=None, stream=None, scratch=None):
        """g = M^T y (life_wc; life_wc_ws with a caller scratch buffer)."""
        torch = _torch()
        if g is None:
            g = torch.empty(self.dims.n_fascicles, dtype=torch.float32, device=y.device)
        args = (self._h, self._d(D), _dev_f32(y, self.n_signal, "y"), _dev_f32(g, self.dims.n_fascicles, "g"))
        if scratch is None:
            _check("life_wc", load().life_wc(*args, _stream(stream, y.device)))
        else:
            _check("life_wc_ws", load().life_wc_ws(*args, *self._scratch(scratch), _stream(stream, y.device)))
        return g

    def dict_grad(self, w, ybar, dD=None, stream=None):
        """dD = d<ybar, M(D) w>/dD, shape (n_atoms, n_theta) like D (life_dict_grad)."""
        torch = _torch()
        d = self.dims
        if dD is None:
            dD = torch.empty((d.n_atoms, d.n_theta), dtype=torch.float32, device=ybar.device)
        _check("life_dict_grad", load().life_dict_grad(self._h, _dev_f32(w, d.n_fascicles, "w"),
                                                       _dev_f32(ybar, self.n_signal, "ybar"),
                                                       _dev_f32(dD, d.n_theta * d.n_atoms, "dD"),
                                                       _stream(stream, ybar.device)))
        return dD

    @staticmethod
    def _state(state):
        torch = _torch()
        if not (isinstance(state, torch.Tensor) and state.is_cuda and state.numel() * state.element_size() == 48
                and state.is_contiguous()):
            raise ValueError("state must be a 48-byte contiguous device tensor (see new_state)")
        return ctypes.c_void_p(state.data_ptr())

    def sbbnnls_step(self, D, b, w, state, stream=None, scratch=None):
        """One SBB-NNLS iteration (Algorithm 1) in place on w; state from new_state()
        (life_sbbnnls_step; life_sbbnnls_step_ws with a caller scratch buffer)."""
        args = (self._h, self._d(D), _dev_f32(b, self.n_signal, "b"), _dev_f32(w, self.dims.n_fascicles, "w"),
                self._state(state))
        if scratch is None:
            _check("life_sbbnnls_step", load().life_sbbnnls_step(*args, _stream(stream, w.device)))
        else:
            _check("life_sbbnnls_step_ws",
                   load().life_sbbnnls_step_ws(*args, *self._scratch(scratch), _stream(stream, w.device)))
        return w

    def sbbnnls_step_lagged(self, D, b, w, gt_prev, state, stream=None):
        """One lagged-BB SBB-NNLS iteration (eqs. 7-8) in place on w; gt_prev (N_f
        floats on the device) carries the projected gradient from call to call."""
        st = self._state(state)
        nf = self.dims.n_fascicles
        _check("life_sbbnnls_step_lagged",
               load().life_sbbnnls_step_lagged(self._h, self._d(D), _dev_f32(b, self.n_signal, "b"),
                                               _dev_f32(w, nf, "w"), _dev_f32(gt_prev, nf, "gt_prev"), st,
                                               _stream(stream, w.device)))
        return w

    def export(self) -> Dict[str, np.ndarray]:
        """The plan's device arrays, copied to host (life_plan_export)."""
        d = self.dims
        out = {"vox_ptr": np.empty(d.n_voxels + 1, np.int32), "atom_v": np.empty(d.nnz, np.int16),
               "fas_v": np.empty(d.nnz, np.int32), "phi_v": np.empty(d.nnz, np.float32),
               "fas_rank": np.empty(d.n_fascicles, np.int32),
               "fas_ptr": np.empty(d.n_fascicles + 1, np.int32), "wc_perm": np.empty(d.nnz, np.int32)}
        keys = ("vox_ptr", "atom_v", "fas_v", "phi_v", "fas_rank", "fas_ptr", "wc_perm")
        _check("life_plan_export", load().life_plan_export(self._h, *(_np_ptr(out[k]) for k in keys)))
        return out

    def profile_enable(self, on: bool = True):
        _check("life_profile_enable", load().life_profile_enable(self._h, int(bool(on))))

    def profile_read(self) -> Tuple[Dict[str, float], Dict[str, int]]:
        ms = np.zeros(len(KERNELS), np.float64)
        cnt = np.zeros(len(KERNELS), np.int64)
        _check("life_profile_read", load().life_profile_read(self._h, _np_ptr(ms), _np_ptr(cnt)))
        return dict(zip(KERNELS, ms.tolist())), dict(zip(KERNELS, cnt.tolist()))
