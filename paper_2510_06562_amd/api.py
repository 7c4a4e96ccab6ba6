"""ctypes binding of ``libdmts.so`` (argument marshalling only; every step of the path runs
in the library's HIP kernels).

PyTorch supplies device memory and streams: arrays are CUDA(HIP) tensors whose data
pointers are passed straight to the C ABI together with the current stream.  Positions and
velocities are float64 in the library's structure-of-arrays layout [3][N]; helpers convert
from the usual (N, 3) layout.

The library must be built (``python -m paper_2510_06562_amd.build``).  Loading fails
loudly when it is missing; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmts.so")

OK, E_ARG, E_BOX, E_CAPACITY, E_NONFINITE, E_HIP, E_OOM, E_STATE = range(8)
FLAG_NBR_OVERFLOW = 0x1
FLAG_NONFINITE = 0x2
KIND_ONE = 0
KIND_TWO = 1
PREC_FP32 = 0
PREC_BF16 = 1

_STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_BOX", 3: "E_CAPACITY", 4: "E_NONFINITE",
                 5: "E_HIP", 6: "E_OOM", 7: "E_STATE"}


class DmtsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_rbf", ctypes.c_int32), ("width", ctypes.c_int32),
                ("emb_dim", ctypes.c_int32), ("n_species", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("cutoff", ctypes.c_double),
                ("energy_scale", ctypes.c_double)]


class _Shape(ctypes.Structure):
    _fields_ = [("receivers_per_group", ctypes.c_int32), ("atom_tiles", ctypes.c_int32),
                ("keep_derivatives", ctypes.c_int32), ("work_groups", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double

_SIGS = {
    "dmts_last_error": ([], ctypes.c_char_p),
    "dmts_version": ([], ctypes.c_char_p),
    "nnp_model_create": ([ctypes.POINTER(_Desc), _P, _I64, ctypes.POINTER(_P)], _I32),
    "nnp_model_destroy": ([_P], None),
    "nnp_model_set_grid": ([_P, _I32], _I32),
    "nnp_model_get_grid": ([_P, ctypes.POINTER(_I32)], _I32),
    "nnp_model_set_shape": ([_P, _I32, ctypes.POINTER(_Shape)], _I32),
    "nnp_model_get_shape": ([_P, _I32, ctypes.POINTER(_Shape)], _I32),
    "nnp_autotune": ([_P, _P, _P, _P, _I32, _D, _P, _I32, _I32, _P, ctypes.POINTER(_Shape),
                      ctypes.POINTER(_D)], _I32),
    "nnp_nlist_create": ([_I32, _I64, _I32, ctypes.POINTER(_P)], _I32),
    "nnp_nlist_destroy": ([_P], None),
    "nnp_build_neighbors": ([_P, _P, _I32, _D, _P, _I32, _D, _P], _I32),
    "nnp_filter_neighbors": ([_P, _P, _P, _D, _P], _I32),
    "nnp_nlist_flags": ([_P, _P, ctypes.POINTER(ctypes.c_uint32)], _I32),
    "nnp_nlist_download": ([_P, _P, _P, _P, _P, _I64, ctypes.POINTER(_I64)], _I32),
    "nnp_energy_forces": ([_P, _P, _P, _P, _I32, _D, _P, _I32, _P, _P, _P, _P], _I32),
    "nnp_energy_forces_noalloc": ([_P, _P, _P, _P, _I32, _D, _P, _I32, _P, _P, _P, _P], _I32),
    "dmts_state_create": ([_I32, _D, _P, _P, _I32, _D, _I32, _I32, _I32, ctypes.POINTER(_P)], _I32),
    "dmts_state_destroy": ([_P], None),
    "dmts_step": ([_P, _P, _P, _P, _P, _I32, _P, _P], _I32),
    "dmts_state_reset": ([_P], _I32),
    "dmts_state_fallbacks": ([_P, ctypes.POINTER(_I64)], _I32),
    "dmts_state_set_thermostat": ([_P, _D, _D, ctypes.c_uint64], _I32),
    "dmts_state_o_steps": ([_P, ctypes.POINTER(ctypes.c_uint64)], _I32),
    "dmts_state_set_fdiff_threshold": ([_P, _D], _I32),
    "dmts_state_set_atom_masses": ([_P, _P, _I32], _I32),
    "dmts_state_fdiff": ([_P, ctypes.POINTER(_I64), ctypes.POINTER(_D)], _I32),
    "dmts_state_forces": ([_P, ctypes.POINTER(_P), ctypes.POINTER(_P)], _I32),
    "dmts_state_flags": ([_P, _P, ctypes.POINTER(ctypes.c_uint32)], _I32),
    "dmts_state_set_skin": ([_P, _D], _I32),
    "dmts_state_get_skin": ([_P, ctypes.POINTER(_D)], _I32),
    "dmts_state_list_builds": ([_P, ctypes.POINTER(_I64)], _I32),
    "dmts_prof_enable": ([ctypes.c_uint32], _I32),
    "dmts_prof_reset": ([], _I32),
    "dmts_prof_sample": ([ctypes.c_uint32], _I32),
    "dmts_prof_read": ([_I32, ctypes.POINTER(_D), ctypes.POINTER(_I64)], _I32),
}

KERNEL_CLASSES = ("small_forward", "small_backward", "pair1_forward", "pair2_forward",
                  "pair2_backward", "pair1_backward", "neighbors", "atom_gemm", "gather",
                  "integrate")

EXPORTED = tuple(_SIGS)


def lib():
    """Load the shared library (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2510_06562_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise DmtsError(status, lib().dmts_last_error().decode(errors="replace"))


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_check(t: torch.Tensor, dtype, shape=None, name="array"):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")


def to_soa(a: np.ndarray | torch.Tensor, device="cuda") -> torch.Tensor:
    """(N, 3) -> contiguous float64 device tensor [3, N]."""
    t = torch.as_tensor(np.asarray(a) if not isinstance(a, torch.Tensor) else a)
    return t.to(device=device, dtype=torch.float64).t().contiguous()


def from_soa(t: torch.Tensor) -> np.ndarray:
    """[3, N] device tensor -> (N, 3) float64 NumPy array."""
    return t.detach().to("cpu", torch.float64).t().contiguous().numpy()


# ------------------------------------------------------------------ models
@dataclass(frozen=True)
class ModelDesc:
    kind: int
    cutoff: float
    n_rbf: int
    width: int
    emb_dim: int = 16
    n_species: int = 5
    energy_scale: float = 0.01
    precision: int = PREC_FP32

    def c(self) -> _Desc:
        return _Desc(self.kind, self.n_rbf, self.width, self.emb_dim, self.n_species,
                     self.precision, self.cutoff, self.energy_scale)


class Model:
    """A potential on the device: ``Model(desc, weights)`` with a flat float32 blob."""

    def __init__(self, desc: ModelDesc, weights: np.ndarray):
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
        h = ctypes.c_void_p()
        _check(lib().nnp_model_create(ctypes.byref(desc.c()), w.ctypes.data_as(ctypes.c_void_p),
                                      w.size, ctypes.byref(h)))
        self.desc = desc
        self._h = h

    @classmethod
    def from_spec(cls, spec, weights, precision=PREC_FP32, energy_scale=None):
        """From a ``synth.ModelSpec``."""
        d = ModelDesc(kind=spec.kind, cutoff=spec.cutoff, n_rbf=spec.n_rbf, width=spec.width,
                      emb_dim=spec.emb_dim, n_species=spec.n_species,
                      energy_scale=spec.energy_scale if energy_scale is None else energy_scale,
                      precision=precision)
        return cls(d, weights)

    @property
    def handle(self):
        return self._h

    @property
    def grid(self) -> int:
        g = ctypes.c_int32()
        _check(lib().nnp_model_get_grid(self._h, ctypes.byref(g)))
        return g.value

    @grid.setter
    def grid(self, work_groups: int):
        _check(lib().nnp_model_set_grid(self._h, int(work_groups)))

    def shape(self, n_atoms: int = 0) -> dict:
        """The tile shape a system of n_atoms uses (0: the default shape)."""
        sh = _Shape()
        _check(lib().nnp_model_get_shape(self._h, int(n_atoms), ctypes.byref(sh)))
        return sh.as_dict()

    def set_shape(self, n_atoms: int = 0, receivers_per_group: int = 4, atom_tiles: int = 2,
                  keep_derivatives: int = 1, work_groups: int = 0):
        """Set the shape of n_atoms' size bucket (0: the default, forgetting every bucket)."""
        sh = _Shape(receivers_per_group, atom_tiles, keep_derivatives, work_groups)
        _check(lib().nnp_model_set_shape(self._h, int(n_atoms), ctypes.byref(sh)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.nnp_model_destroy(self._h)
            self._h = None


class NeighborList:
    def __init__(self, max_atoms: int, max_pairs: int, row_align: int = 4):
        h = ctypes.c_void_p()
        _check(lib().nnp_nlist_create(max_atoms, max_pairs, row_align, ctypes.byref(h)))
        self._h = h
        self.max_atoms = max_atoms
        self.max_pairs = max_pairs
        self.n_atoms = 0   # atoms of the last build

    @property
    def handle(self):
        return self._h

    def build(self, pos_soa: torch.Tensor, box: float, cutoff: float,
              sys_offsets: Optional[torch.Tensor] = None, stream=None):
        n = pos_soa.shape[1]
        _dev_check(pos_soa, torch.float64, (3, n), "pos")
        n_sys = 1
        if sys_offsets is not None:
            _dev_check(sys_offsets, torch.int32, None, "sys_offsets")
            n_sys = sys_offsets.numel() - 1
        _check(lib().nnp_build_neighbors(self._h, _ptr(pos_soa), n, float(box), _ptr(sys_offsets),
                                         n_sys, float(cutoff), _stream(stream)))
        self.n_atoms = n

    def filter_from(self, parent: "NeighborList", pos_soa: torch.Tensor, cutoff: float,
                    stream=None):
        """This list at `cutoff` (<= the parent's) from the parent's rows at pos_soa, which
        holds the parent's atoms."""
        _dev_check(pos_soa, torch.float64, (3, parent.n_atoms), "pos")
        _check(lib().nnp_filter_neighbors(self._h, parent.handle, _ptr(pos_soa), float(cutoff),
                                          _stream(stream)))
        self.n_atoms = parent.n_atoms

    def flags(self, stream=None) -> int:
        f = ctypes.c_uint32()
        _check(lib().nnp_nlist_flags(self._h, _stream(stream), ctypes.byref(f)))
        return f.value

    def download(self, n_atoms: int, stream=None):
        """(offs, nbr, rev) as NumPy int32 arrays (synchronizes)."""
        offs = np.zeros(n_atoms + 1, dtype=np.int32)
        cap = self.max_pairs + 4
        nbr = np.zeros(cap, dtype=np.int32)
        rev = np.zeros(cap, dtype=np.int32)
        P = ctypes.c_int64()
        _check(lib().nnp_nlist_download(self._h, _stream(stream), offs.ctypes.data_as(_P),
                                        nbr.ctypes.data_as(_P), rev.ctypes.data_as(_P), cap,
                                        ctypes.byref(P)))
        return offs, nbr[:P.value].copy(), rev[:P.value].copy()

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.nnp_nlist_destroy(self._h)
            self._h = None


def energy_forces(model: Model, nlist: NeighborList, pos_soa: torch.Tensor,
                  species: torch.Tensor, box: float, sys_offsets: Optional[torch.Tensor] = None,
                  want_forces: bool = True, atom_energy: bool = False, stream=None):
    """Energies per system (float64 [n_sys]), forces (float32 [3, N]) and optionally the
    per-atom energies, on the pairs of ``nlist`` (built from the same positions)."""
    n = pos_soa.shape[1]
    _dev_check(pos_soa, torch.float64, (3, n), "pos")
    _dev_check(species, torch.int32, (n,), "species")
    n_sys = 1 if sys_offsets is None else sys_offsets.numel() - 1
    E = torch.empty(n_sys, dtype=torch.float64, device=pos_soa.device)
    F = torch.empty((3, n), dtype=torch.float32, device=pos_soa.device) if want_forces else None
    Ea = torch.empty(n, dtype=torch.float32, device=pos_soa.device) if atom_energy else None
    _check(lib().nnp_energy_forces(model.handle, nlist.handle, _ptr(pos_soa), _ptr(species), n,
                                   float(box), _ptr(sys_offsets), n_sys, _ptr(E), _ptr(F),
                                   _ptr(Ea), _stream(stream)))
    return (E, F, Ea) if atom_energy else (E, F)


def energy_forces_noalloc(model: Model, nlist: NeighborList, pos_soa: torch.Tensor,
                          species: torch.Tensor, box: float, energy: torch.Tensor,
                          forces: Optional[torch.Tensor] = None,
                          atom_energy: Optional[torch.Tensor] = None,
                          sys_offsets: Optional[torch.Tensor] = None, stream=None):
    """nnp_energy_forces_noalloc: a one-interaction model's energies and forces into the
    caller's preallocated tensors (energy float64 [n_sys], forces float32 [3, N],
    atom_energy float32 [N]); the library allocates nothing."""
    n = pos_soa.shape[1]
    _dev_check(pos_soa, torch.float64, (3, n), "pos")
    _dev_check(species, torch.int32, (n,), "species")
    n_sys = 1 if sys_offsets is None else sys_offsets.numel() - 1
    _dev_check(energy, torch.float64, (n_sys,), "energy")
    if forces is not None:
        _dev_check(forces, torch.float32, (3, n), "forces")
    if atom_energy is not None:
        _dev_check(atom_energy, torch.float32, (n,), "atom_energy")
    _check(lib().nnp_energy_forces_noalloc(model.handle, nlist.handle, _ptr(pos_soa),
                                           _ptr(species), n, float(box), _ptr(sys_offsets),
                                           n_sys, _ptr(energy), _ptr(forces), _ptr(atom_energy),
                                           _stream(stream)))


class Potential:
    """A model with its own neighbor list: ``pot(pos_soa) -> (E, F)``.

    With ``check`` (the default) every call reads the list's device flag word afterwards
    (one synchronization) and raises DmtsError(E_CAPACITY) when a row or the list
    overflowed, so that truncated sums never pass silently; ``check=False`` leaves that to
    the caller (``nlist.flags()``)."""

    def __init__(self, model: Model, max_atoms: int, box: float, max_nbrs: int = 128,
                 sys_offsets: Optional[torch.Tensor] = None, check: bool = True):
        self.model = model
        self.box = box
        self.sys_offsets = sys_offsets
        self.check = check
        self.nlist = NeighborList(max_atoms, max_atoms * (max_nbrs + 16), 16)

    def __call__(self, pos_soa: torch.Tensor, species: torch.Tensor, want_forces=True,
                 atom_energy=False, stream=None):
        self.nlist.build(pos_soa, self.box, self.model.desc.cutoff, self.sys_offsets, stream)
        out = energy_forces(self.model, self.nlist, pos_soa, species, self.box,
                            self.sys_offsets, want_forces, atom_energy, stream)
        if self.check:
            f = self.nlist.flags(stream)
            if f & FLAG_NBR_OVERFLOW:
                raise DmtsError(E_CAPACITY, "neighbor list overflow: a row held more "
                                "neighbors than the kernels take (or the list its capacity); "
                                "the forces would be truncated")
            if f & FLAG_NONFINITE:
                raise DmtsError(E_NONFINITE, "non-finite value met in the evaluation")
        return out


def autotune(potential: "Potential", pos_soa: torch.Tensor, species: torch.Tensor,
             reps: int = 3, stream=None, cutoff: Optional[float] = None):
    """Pick the model's tile shape for this system's size bucket (see nnp_autotune); returns
    (shape dict, best_ms).  Builds the potential's list from pos_soa first, at `cutoff`
    (default: the model's; a longer one tunes for a list shared with another model)."""
    potential.nlist.build(pos_soa, potential.box,
                          potential.model.desc.cutoff if cutoff is None else cutoff,
                          potential.sys_offsets, stream)
    n = pos_soa.shape[1]
    offs = potential.sys_offsets
    n_sys = 1 if offs is None else offs.numel() - 1
    sh, t = _Shape(), ctypes.c_double()
    _check(lib().nnp_autotune(potential.model.handle, potential.nlist.handle, _ptr(pos_soa),
                              _ptr(species), n, float(potential.box), _ptr(offs), n_sys, reps,
                              _stream(stream), ctypes.byref(sh), ctypes.byref(t)))
    return sh.as_dict(), t.value


class NNPEnergy(torch.autograd.Function):
    """E = NNPEnergy.apply(pos_soa, potential, species): forward returns the energy per
    system ([n_sys], float64); backward returns dL/dx = -F_i * dL/dE_s(i) for every atom i
    of system s(i) (the library's analytic forces; atoms outside every system get zero)."""

    @staticmethod
    def forward(ctx, pos_soa, potential: Potential, species):
        E, F = potential(pos_soa.detach(), species, want_forces=True)
        ctx.save_for_backward(F)
        ctx.sys_offsets = potential.sys_offsets
        return E

    @staticmethod
    def backward(ctx, grad_E):
        (F,) = ctx.saved_tensors
        n = F.shape[1]
        g = grad_E.reshape(-1).to(torch.float64)
        offs = ctx.sys_offsets
        if offs is None:
            g_atom = g.expand(n)
        else:
            o = offs.to(device=F.device, dtype=torch.int64)
            g_atom = torch.zeros(n, dtype=torch.float64, device=F.device)
            lo, hi = int(o[0]), int(o[-1])
            g_atom[lo:hi] = torch.repeat_interleave(g, o[1:] - o[:-1], output_size=hi - lo)
        return -(F.to(torch.float64) * g_atom[None, :]), None, None


# ------------------------------------------------------------------ dynamics
class DMTS:
    """Algorithm 1 (BAOAB-RESPA) or, with small=None, single-time-step BAOAB with the
    reference model; NVE (velocity Verlet steps) until set_thermostat gives gamma > 0."""

    def __init__(self, n_atoms: int, box: float, species: torch.Tensor, masses_by_species,
                 dt_outer: float, n_inner: int, max_nbrs_small: int = 48,
                 max_nbrs_large: int = 128):
        _dev_check(species, torch.int32, (n_atoms,), "species")
        m = np.ascontiguousarray(np.asarray(masses_by_species, dtype=np.float64))
        h = ctypes.c_void_p()
        _check(lib().dmts_state_create(n_atoms, float(box), _ptr(species),
                                       m.ctypes.data_as(_P), m.size, float(dt_outer), n_inner,
                                       max_nbrs_small, max_nbrs_large, ctypes.byref(h)))
        self._h = h
        self.species = species   # keep the borrowed array alive
        self.n = n_atoms
        self.energies = torch.zeros(4, dtype=torch.float64, device=species.device)

    def step(self, x_soa: torch.Tensor, v_soa: torch.Tensor, small: Optional[Model],
             large: Model, n_outer: int = 1, stream=None):
        _dev_check(x_soa, torch.float64, (3, self.n), "x")
        _dev_check(v_soa, torch.float64, (3, self.n), "v")
        _check(lib().dmts_step(self._h, _ptr(x_soa), _ptr(v_soa),
                               small.handle if small is not None else None, large.handle,
                               n_outer, _ptr(self.energies), _stream(stream)))
        return self.energies

    def reset(self):
        _check(lib().dmts_state_reset(self._h))

    def set_thermostat(self, gamma_per_fs: float, temperature_K: float, seed: int):
        """Langevin O-step of Algorithm 1 (gamma 0 = off); resets the O-step counter."""
        _check(lib().dmts_state_set_thermostat(self._h, float(gamma_per_fs),
                                               float(temperature_K), int(seed)))

    def set_atom_masses(self, masses):
        """Per-atom masses (amu; e.g. hydrogen mass repartitioning) instead of the species
        table for the kicks, O-steps and kinetic energy; None returns to the table."""
        if masses is None:
            _check(lib().dmts_state_set_atom_masses(self._h, None, 0))
            return
        m = np.ascontiguousarray(np.asarray(masses, dtype=np.float64))
        if m.ndim != 1:
            raise DmtsError(E_ARG, "set_atom_masses: expected a 1-d array of masses")
        _check(lib().dmts_state_set_atom_masses(self._h, m.ctypes.data_as(ctypes.c_void_p),
                                                int(m.shape[0])))

    def set_fdiff_threshold(self, eV_per_A: float):
        """Redo a call as single-time-step steps when |F - F_small| of an atom exceeds
        this (0 = off; the paper's threshold is 150 kcal/mol/A = 6.505 eV/A)."""
        _check(lib().dmts_state_set_fdiff_threshold(self._h, float(eV_per_A)))

    @property
    def fdiff(self):
        """(calls redone as single-time-step steps, largest breach of the last call)."""
        n, b = ctypes.c_int64(), ctypes.c_double()
        _check(lib().dmts_state_fdiff(self._h, ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    @property
    def o_steps(self) -> int:
        """O-steps taken since set_thermostat (the noise counter of the next one)."""
        k = ctypes.c_uint64()
        _check(lib().dmts_state_o_steps(self._h, ctypes.byref(k)))
        return k.value

    def set_skin(self, skin_A: float):
        """Skin of the reference evaluations' lists (A; 0 = a fresh build every time)."""
        _check(lib().dmts_state_set_skin(self._h, float(skin_A)))

    @property
    def skin(self) -> float:
        d = ctypes.c_double()
        _check(lib().dmts_state_get_skin(self._h, ctypes.byref(d)))
        return d.value

    @property
    def list_builds(self) -> int:
        """Rebuilds of the skin list's rows so far (synchronizes the device)."""
        n = ctypes.c_int64()
        _check(lib().dmts_state_list_builds(self._h, ctypes.byref(n)))
        return n.value

    @property
    def fallbacks(self) -> int:
        """Calls redone with exact neighbor lists (an atom outran the shared list)."""
        n = ctypes.c_int64()
        _check(lib().dmts_state_fallbacks(self._h, ctypes.byref(n)))
        return n.value

    def forces(self):
        fl, fs = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().dmts_state_forces(self._h, ctypes.byref(fl), ctypes.byref(fs)))
        return fl.value, fs.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dmts_state_destroy(self._h)
            self._h = None


# ------------------------------------------------------------------ kernel timing
def prof_enable(classes=None):
    """Time the given kernel classes (names from KERNEL_CLASSES; None = all, () = off)."""
    if classes is None:
        mask = (1 << len(KERNEL_CLASSES)) - 1
    else:
        mask = 0
        for c in classes:
            mask |= 1 << KERNEL_CLASSES.index(c)
    _check(lib().dmts_prof_enable(mask))


def prof_reset():
    _check(lib().dmts_prof_reset())


def prof_sample(every: int = 1):
    """Time one launch in `every` of each enabled class (1 = all)."""
    _check(lib().dmts_prof_sample(int(every)))


def prof_read() -> dict:
    """{class: (total_ms, launches)} for every timed kernel class (synchronizes)."""
    out = {}
    for k, name in enumerate(KERNEL_CLASSES):
        t, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().dmts_prof_read(k, ctypes.byref(t), ctypes.byref(n)))
        out[name] = (t.value, n.value)
    return out
