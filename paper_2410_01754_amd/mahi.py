"""ctypes binding of libmahi.so (argument marshalling only).

Every step of an evaluation runs in the library's HIP kernels; this module
only converts Python/numpy/torch arguments into the C structs of
include/mahi.h.  Importing it without the built library raises at once: there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmahi.so")

MAHI_DEVICE_IO = 1
N_STAGES = 9
STATUS = {0: "MAHI_OK", -1: "MAHI_EINVAL", -2: "MAHI_ENOMEM", -3: "MAHI_EDEVICE", -4: "MAHI_ERANGE",
          -5: "MAHI_ESTATE", -6: "MAHI_EUNSUPPORTED"}


class MahiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _Box(ctypes.Structure):
    _fields_ = [("edge", ctypes.c_double), ("periodic", ctypes.c_int)]


class _Sites(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("forms_per_site", ctypes.POINTER(ctypes.c_int32)),
                ("atoms_per_site", ctypes.POINTER(ctypes.c_int32)), ("site_atoms", ctypes.POINTER(ctypes.c_int32)),
                ("form_charges", ctypes.POINTER(ctypes.c_double))]


class _Opts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("depth", ctypes.c_int), ("precision", ctypes.c_int),
                ("coulomb_k", ctypes.c_double), ("hip_stream", ctypes.c_void_p)]


class _EvalArgs(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("energy", ctypes.c_void_p), ("forces", ctypes.c_void_p),
                ("dvdl", ctypes.c_void_p), ("potential", ctypes.c_void_p), ("flags", ctypes.c_uint32),
                ("dedq", ctypes.c_void_p), ("energy_qi", ctypes.c_void_p), ("dvdl_qi", ctypes.c_void_p)]


class _CorrectArgs(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("potential", ctypes.c_void_p), ("energy", ctypes.c_void_p),
                ("forces", ctypes.c_void_p), ("dvdl", ctypes.c_void_p), ("dedq", ctypes.c_void_p),
                ("flags", ctypes.c_uint32)]


def _init_torch_runtime():
    """PyTorch ships its own HIP runtime.  Two runtimes share the GPU in one
    process only when torch's initialises first (initialised afterwards it
    finds no device), so start it before this library's when a GPU is visible."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libmahi.so not built at {path}; run python -m paper_2410_01754_amd.build")
    _init_torch_runtime()
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.mahi_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Box), ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_Sites), ctypes.POINTER(_Opts)]
    lib.mahi_create.restype = ctypes.c_int
    lib.mahi_set_lambda.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.mahi_set_lambda.restype = ctypes.c_int
    lib.mahi_eval.argtypes = [vp, ctypes.POINTER(_EvalArgs)]
    lib.mahi_eval.restype = ctypes.c_int
    lib.mahi_destroy.argtypes = [vp]
    lib.mahi_destroy.restype = None
    lib.mahi_strerror.argtypes = [ctypes.c_int]
    lib.mahi_strerror.restype = ctypes.c_char_p
    lib.mahi_last_error.argtypes = [vp]
    lib.mahi_last_error.restype = ctypes.c_char_p
    lib.mahi_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.mahi_info.restype = ctypes.c_int
    lib.mahi_get_stream.argtypes = [vp, ctypes.POINTER(vp)]
    lib.mahi_get_stream.restype = ctypes.c_int
    lib.mahi_host_selftest.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.mahi_host_selftest.restype = ctypes.c_int
    lib.mahi_device_selftest.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.mahi_device_selftest.restype = ctypes.c_int
    lib.mahi_profile_begin.argtypes = [vp, ctypes.c_int]
    lib.mahi_profile_begin.restype = ctypes.c_int
    lib.mahi_profile_end.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    lib.mahi_profile_end.restype = ctypes.c_int
    lib.mahi_stage_name.argtypes = [ctypes.c_int]
    lib.mahi_stage_name.restype = ctypes.c_char_p
    lib.mahi_profile_eval_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_int)]
    lib.mahi_profile_eval_times.restype = ctypes.c_int
    lib.mahi_debug_copy.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int64]
    lib.mahi_debug_copy.restype = ctypes.c_int
    lib.mahi_set_form_charges.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.mahi_set_form_charges.restype = ctypes.c_int
    lib.mahi_correct.argtypes = [vp, ctypes.POINTER(_CorrectArgs)]
    lib.mahi_correct.restype = ctypes.c_int
    lib.mahi_correct_noalloc.argtypes = [vp, ctypes.POINTER(_CorrectArgs)]
    lib.mahi_correct_noalloc.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.mahi_lambda_tilde.argtypes = [ctypes.c_int, dp, dp]
    lib.mahi_lambda_tilde.restype = ctypes.c_int
    lib.mahi_dlambda.argtypes = [ctypes.c_int, dp, dp, dp]
    lib.mahi_dlambda.restype = ctypes.c_int
    lib.mahi_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, vp]
    lib.mahi_batch_create.restype = ctypes.c_int
    lib.mahi_batch_eval.argtypes = [vp, ctypes.POINTER(_EvalArgs)]
    lib.mahi_batch_eval.restype = ctypes.c_int
    lib.mahi_batch_destroy.argtypes = [vp]
    lib.mahi_batch_destroy.restype = None
    lib.mahi_batch_last_error.argtypes = [vp]
    lib.mahi_batch_last_error.restype = ctypes.c_char_p
    ip = ctypes.POINTER(ctypes.c_int)
    lib.mahi_autotune.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ip, ip]
    lib.mahi_autotune.restype = ctypes.c_int
    lib.mahi_tune.argtypes = [vp, vp, ctypes.c_int, ip, ip]
    lib.mahi_tune.restype = ctypes.c_int
    return lib


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _check(status: int, ctx=None):
    if status != 0:
        msg = lib().mahi_last_error(ctx).decode()
        raise MahiError(status, msg)


def host_selftest(order: int) -> float:
    v = ctypes.c_double()
    _check(lib().mahi_host_selftest(order, ctypes.byref(v)))
    return v.value


def device_selftest(precision: int) -> float:
    v = ctypes.c_double()
    _check(lib().mahi_device_selftest(precision, ctypes.byref(v)))
    return v.value


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def autotune(periodic: bool, edge: float, n_atoms: int, precision: int, target_rel_err: float,
             site_extent: float = -1.0):
    """(order, depth) from the library's error and cost models (mahi_autotune);
    site_extent: largest distance between two atoms of one site in nm (< 0: unknown)."""
    o, d = ctypes.c_int(), ctypes.c_int()
    _check(lib().mahi_autotune(1 if periodic else 0, float(edge), int(n_atoms), int(precision), float(target_rel_err),
                               float(site_extent), ctypes.byref(o), ctypes.byref(d)))
    return o.value, d.value


def site_extent(system) -> float:
    """Largest distance between two atoms of one site of a synth-style system (nm),
    with periodic images taken into account; 0 without sites."""
    ext = 0.0
    for st in system.sites:
        x = np.asarray(system.x[st.atoms], dtype=np.float64)
        d = x[:, None, :] - x[None, :, :]
        if system.periodic:
            d -= system.box * np.round(d / system.box)
        ext = max(ext, float(np.sqrt((d ** 2).sum(-1)).max()))
    return ext


def lambda_tilde(lambdas) -> np.ndarray:
    """Weights of the 2^L forms of a binary site from its L original lambdas (mahi_lambda_tilde)."""
    lam = np.ascontiguousarray(lambdas, dtype=np.float64)
    out = np.zeros(1 << lam.shape[0])
    _check(lib().mahi_lambda_tilde(int(lam.shape[0]), _ptr(lam, ctypes.c_double), _ptr(out, ctypes.c_double)))
    return out


def dlambda(lambdas, dvdl) -> np.ndarray:
    """dE/dlambda_k of a binary site from its per-form dE/dlambda-tilde (mahi_dlambda)."""
    lam = np.ascontiguousarray(lambdas, dtype=np.float64)
    g = np.ascontiguousarray(dvdl, dtype=np.float64)
    if g.shape[0] != 1 << lam.shape[0]:
        raise ValueError("dvdl must have 2^len(lambdas) entries")
    out = np.zeros(lam.shape[0])
    _check(lib().mahi_dlambda(int(lam.shape[0]), _ptr(lam, ctypes.c_double), _ptr(g, ctypes.c_double),
                              _ptr(out, ctypes.c_double)))
    return out


class Mahi:
    """One MAHI evaluator: a cubic box, N charges and their titratable sites.

    sites: sequence of (atoms [n] int, form_charges [n_forms, n] float).
    """

    def __init__(self, edge: float, periodic: bool, charges, sites: Sequence = (), order: int = 8, depth: int = 3,
                 precision: int = 32, coulomb_k: float = 0.0, stream: Optional[int] = None):
        self._lib = lib()
        q = np.ascontiguousarray(charges, dtype=np.float64)
        self.n = int(q.shape[0])
        self.precision = int(precision)
        self.dtype = np.float32 if precision == 32 else np.float64
        fps = np.array([np.asarray(c).shape[0] for _, c in sites], dtype=np.int32)
        aps = np.array([len(a) for a, _ in sites], dtype=np.int32)
        atoms = np.ascontiguousarray(np.concatenate([np.asarray(a) for a, _ in sites]) if len(sites) else
                                     np.zeros(0), dtype=np.int32)
        fq = np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.float64).reshape(-1) for _, c in sites])
                                  if len(sites) else np.zeros(0), dtype=np.float64)
        self.n_forms = int(fps.sum())
        self.n_form_charges = int(fq.shape[0])
        self._keep = (q, fps, aps, atoms, fq)
        box = _Box(float(edge), 1 if periodic else 0)
        st = _Sites(len(sites), _ptr(fps, ctypes.c_int32), _ptr(aps, ctypes.c_int32), _ptr(atoms, ctypes.c_int32),
                    _ptr(fq, ctypes.c_double))
        opts = _Opts(int(order), int(depth), int(precision), float(coulomb_k), ctypes.c_void_p(stream or 0))
        h = ctypes.c_void_p()
        _check(self._lib.mahi_create(ctypes.byref(h), ctypes.byref(box), self.n, _ptr(q, ctypes.c_double),
                                     ctypes.byref(st), ctypes.byref(opts)), None)
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mahi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_lambda(self, lam_tilde):
        lt = np.ascontiguousarray(lam_tilde, dtype=np.float64)
        if lt.shape[0] != self.n_forms:
            raise ValueError("lambda_tilde has the wrong length")
        _check(self._lib.mahi_set_lambda(self._h, _ptr(lt, ctypes.c_double)), self._h)

    def set_form_charges(self, form_charges):
        """Replace every form charge (flat, the layout given at creation: per site form-major, atom-minor)."""
        fq = np.ascontiguousarray(form_charges, dtype=np.float64).reshape(-1)
        if fq.shape[0] != self.n_form_charges:
            raise ValueError("form_charges has the wrong length")
        _check(self._lib.mahi_set_form_charges(self._h, _ptr(fq, ctypes.c_double)), self._h)

    def eval(self, xyz, forces: bool = True, dvdl: bool = True, potential: bool = False, dedq: bool = False,
             qi: bool = False):
        """Host-memory evaluation; returns dict(energy, forces, dvdl, potential, dedq, energy_qi, dvdl_qi)."""
        x = np.ascontiguousarray(xyz, dtype=self.dtype)
        if x.shape != (self.n, 3):
            raise ValueError("xyz must have shape (N, 3)")
        E = np.zeros(1)
        F = np.zeros((self.n, 3), dtype=self.dtype) if forces else None
        dv = np.zeros(self.n_forms) if (dvdl and self.n_forms) else None
        pot = np.zeros(self.n, dtype=self.dtype) if potential else None
        dq = np.zeros(self.n_form_charges) if (dedq and self.n_forms) else None
        Eqi = np.zeros(1) if qi else None
        dvqi = np.zeros(self.n_forms) if (qi and self.n_forms) else None
        a = lambda v: None if v is None else v.ctypes.data  # noqa: E731
        args = _EvalArgs(x.ctypes.data, E.ctypes.data, a(F), a(dv), a(pot), 0, a(dq), a(Eqi), a(dvqi))
        _check(self._lib.mahi_eval(self._h, ctypes.byref(args)), self._h)
        return {"energy": float(E[0]), "forces": F, "dvdl": dv, "potential": pot, "dedq": dq,
                "energy_qi": None if Eqi is None else float(Eqi[0]), "dvdl_qi": dvqi}

    def eval_device(self, xyz_ptr: int, energy_ptr: int, forces_ptr: int = 0, dvdl_ptr: int = 0,
                    potential_ptr: int = 0, dedq_ptr: int = 0, energy_qi_ptr: int = 0, dvdl_qi_ptr: int = 0):
        """Asynchronous evaluation on device pointers (e.g. torch tensor data_ptr())."""
        args = _EvalArgs(xyz_ptr, energy_ptr or None, forces_ptr or None, dvdl_ptr or None, potential_ptr or None,
                         MAHI_DEVICE_IO, dedq_ptr or None, energy_qi_ptr or None, dvdl_qi_ptr or None)
        _check(self._lib.mahi_eval(self._h, ctypes.byref(args)), self._h)

    def correct(self, xyz, potential, forces=None, dvdl: bool = True, dedq: bool = False):
        """Site correction on a potential from another solver (host memory; mahi_correct).

        potential: [N] coulomb_k * charge-scaled potential.  forces: optional [N, 3]
        array of the same type as xyz; the correction is added to it in place.
        Returns dict(energy, dvdl, dedq, forces)."""
        x = np.ascontiguousarray(xyz, dtype=self.dtype)
        pot = np.ascontiguousarray(potential, dtype=self.dtype)
        if x.shape != (self.n, 3) or pot.shape != (self.n,):
            raise ValueError("xyz must have shape (N, 3) and potential (N,)")
        if forces is not None and (forces.dtype != self.dtype or forces.shape != (self.n, 3)
                                   or not forces.flags.c_contiguous):
            raise ValueError("forces must be a C-contiguous (N, 3) array of the context's type")
        E = np.zeros(1)
        dv = np.zeros(self.n_forms) if (dvdl and self.n_forms) else None
        dq = np.zeros(self.n_form_charges) if (dedq and self.n_forms) else None
        a = lambda v: None if v is None else v.ctypes.data  # noqa: E731
        args = _CorrectArgs(x.ctypes.data, pot.ctypes.data, E.ctypes.data, a(forces), a(dv), a(dq), 0)
        _check(self._lib.mahi_correct(self._h, ctypes.byref(args)), self._h)
        return {"energy": float(E[0]), "dvdl": dv, "dedq": dq, "forces": forces}

    def correct_device(self, xyz_ptr: int, potential_ptr: int, energy_ptr: int, forces_ptr: int = 0,
                       dvdl_ptr: int = 0, dedq_ptr: int = 0):
        """Asynchronous site correction on device pointers."""
        args = _CorrectArgs(xyz_ptr, potential_ptr, energy_ptr or None, forces_ptr or None, dvdl_ptr or None,
                            dedq_ptr or None, MAHI_DEVICE_IO)
        _check(self._lib.mahi_correct(self._h, ctypes.byref(args)), self._h)

    def correct_device_noalloc(self, xyz_ptr: int, potential_ptr: int, energy_ptr: int, forces_ptr: int = 0,
                               dvdl_ptr: int = 0, dedq_ptr: int = 0):
        """correct_device without any allocation (mahi_correct_noalloc: its scratch is
        a static device array shared by every call on the device)."""
        args = _CorrectArgs(xyz_ptr, potential_ptr, energy_ptr or None, forces_ptr or None, dvdl_ptr or None,
                            dedq_ptr or None, MAHI_DEVICE_IO)
        _check(self._lib.mahi_correct_noalloc(self._h, ctypes.byref(args)), self._h)

    def tune(self, xyz_ptr: int, reps: int = 3):
        """Measured choice of the M2L operator ranges and the near-field targets per
        lane for positions at device pointer xyz_ptr (mahi_tune); blocks until done.
        Returns (m2l_ranges, p2p_targets)."""
        r, t = ctypes.c_int(), ctypes.c_int()
        _check(self._lib.mahi_tune(self._h, ctypes.c_void_p(xyz_ptr), int(reps), ctypes.byref(r), ctypes.byref(t)),
               self._h)
        return r.value, t.value

    def profile_begin(self, max_evals: int):
        _check(self._lib.mahi_profile_begin(self._h, int(max_evals)), self._h)

    def profile_end(self):
        """Mean ms per stage over the evaluations since profile_begin: (dict, n_evals)."""
        ms = (ctypes.c_double * N_STAGES)()
        n = ctypes.c_int()
        _check(self._lib.mahi_profile_end(self._h, ms, ctypes.byref(n)), self._h)
        return {self._lib.mahi_stage_name(i).decode(): ms[i] for i in range(N_STAGES)}, n.value

    def profile_eval_times(self, max_evals: int = 100000) -> np.ndarray:
        """Per-evaluation durations (ms) of the last ended profile."""
        out = np.zeros(max_evals)
        n = ctypes.c_int()
        _check(self._lib.mahi_profile_eval_times(self._h, _ptr(out, ctypes.c_double), int(max_evals),
                                                 ctypes.byref(n)), self._h)
        return out[:n.value]

    def debug_copy(self, which: int, count: int):
        """Copy an internal buffer of the last evaluation (test hook; see mahi_debug_copy)."""
        dt = np.int32 if which in (2, 3) else self.dtype
        out = np.zeros(count, dtype=dt)
        _check(self._lib.mahi_debug_copy(self._h, which, out.ctypes.data, count), self._h)
        return out

    def stream_handle(self) -> int:
        """The hipStream_t (as an int) that this evaluator's evaluations run on."""
        v = ctypes.c_void_p()
        _check(self._lib.mahi_get_stream(self._h, ctypes.byref(v)), self._h)
        return int(v.value or 0)

    def info(self):
        n = ctypes.c_int64()
        ns, nf = ctypes.c_int32(), ctypes.c_int32()
        o, d, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._lib.mahi_info(self._h, ctypes.byref(n), ctypes.byref(ns), ctypes.byref(nf), ctypes.byref(o),
                                   ctypes.byref(d), ctypes.byref(p)), self._h)
        return dict(n_atoms=n.value, n_sites=ns.value, n_forms=nf.value, order=o.value, depth=d.value,
                    precision=p.value)


def from_system(system, precision: int = 32, order: Optional[int] = None, depth: Optional[int] = None,
                coulomb_k: float = 0.0, stream: Optional[int] = None) -> Mahi:
    """Build an evaluator for a synth.System-like object (x, q, sites, box, periodic)."""
    sites = [(s.atoms, s.charges) for s in system.sites]
    m = Mahi(system.box, system.periodic, system.q, sites, order=system.order if order is None else order,
             depth=system.depth if depth is None else depth, precision=precision, coulomb_k=coulomb_k, stream=stream)
    if system.sites:
        m.set_lambda(system.lam_flat())
    return m


class Batch:
    """Evaluate several evaluators together (mahi_batch_*).

    packed=False: one fork/join from `stream`, each evaluator's own evaluation.
    packed=True: every stage one launch over all systems (float32, periodic,
    one order); use_graph=True (packed only) captures those
    launches into a HIP graph and replays it."""

    GRAPH = 1
    PACKED = 2

    def __init__(self, evaluators: Sequence[Mahi], use_graph: bool = False, stream: Optional[int] = None,
                 packed: bool = False):
        self._lib = lib()
        self.evaluators = list(evaluators)
        arr = (ctypes.c_void_p * len(self.evaluators))(*[m._h.value for m in self.evaluators])
        h = ctypes.c_void_p()
        flags = (self.GRAPH if use_graph else 0) | (self.PACKED if packed else 0)
        st = self._lib.mahi_batch_create(ctypes.byref(h), arr, len(self.evaluators), flags,
                                         ctypes.c_void_p(stream or 0))
        if st != 0:
            raise MahiError(st, self._lib.mahi_batch_last_error(None).decode())
        self._h = h

    def eval_device(self, ptrs: Sequence[dict]):
        """ptrs[i]: dict of device pointers (xyz, energy, forces, dvdl, potential, dedq, energy_qi, dvdl_qi)."""
        if len(ptrs) != len(self.evaluators):
            raise ValueError("one pointer set per evaluator")
        args = (_EvalArgs * len(ptrs))()
        for a, p in zip(args, ptrs):
            a.xyz = p["xyz"]
            for k in ("energy", "forces", "dvdl", "potential", "dedq", "energy_qi", "dvdl_qi"):
                setattr(a, k, p.get(k) or None)
            a.flags = MAHI_DEVICE_IO
        st = self._lib.mahi_batch_eval(self._h, args)
        if st != 0:
            raise MahiError(st, self._lib.mahi_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mahi_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
