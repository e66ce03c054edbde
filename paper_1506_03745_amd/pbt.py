"""ctypes binding of libpbt (include/pbt.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy
arrays (and, for the device entry points, torch tensors) to pointers and
status codes to exceptions.  Importing it fails loudly when the library has
not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbt.so")

MOLECULE, CHARGED, POTENTIAL, STERN, CAVITY = 0, 1, 2, 3, 4
FP64, MIXED = 0, 1

STATUS = {0: "PBT_OK", 1: "PBT_E_INVALID", 2: "PBT_E_NOMEM", 3: "PBT_E_DEVICE",
          4: "PBT_E_NOCONVERGE", 5: "PBT_E_NUMERIC", 6: "PBT_E_STATE"}

EXPORTS = ("pbt_default_params", "pbt_create", "pbt_destroy", "pbt_last_error", "pbt_set_params",
           "pbt_set_solvent", "pbt_add_surface", "pbt_set_bc", "pbt_set_charges", "pbt_set_stern",
           "pbt_set_cavity", "pbt_enable",
           "pbt_prepare", "pbt_num_unknowns", "pbt_solve", "pbt_get_solution", "pbt_interaction_energy",
           "pbt_matvec", "pbt_matvec_dev", "pbt_rhs", "pbt_gradient", "pbt_solve_batch",
           "pbt_autotune", "pbt_last_stats", "pbt_set_schedule", "pbt_get_schedule", "pbt_set_gram_schmidt",
           "pbt_get_launch_shape",
           "pbt_quadrature_rule", "pbt_last_matvec_timing", "pbt_profile", "pbt_kernel_times",
           "pbt_set_bc_dev", "pbt_set_charges_dev", "pbt_get_solution_dev", "pbt_gradient_dev",
           "pbt_matvec_dev_static")


class PbtParams(ctypes.Structure):
    _fields_ = [("k_far", ctypes.c_int32), ("k_near", ctypes.c_int32), ("k_self_edge", ctypes.c_int32),
                ("ncrit", ctypes.c_int32), ("taylor_p", ctypes.c_int32), ("theta", ctypes.c_double),
                ("tol", ctypes.c_double), ("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("treecode", ctypes.c_int32), ("near_factor", ctypes.c_double),
                ("precond", ctypes.c_int32)]


class PbtResult(ctypes.Structure):
    _fields_ = [("F_coul", ctypes.c_double), ("F_solv", ctypes.c_double), ("F_surf", ctypes.c_double),
                ("F_total", ctypes.c_double), ("iters", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("t_setup_s", ctypes.c_double),
                ("t_solve_s", ctypes.c_double), ("p2p_pairs", ctypes.c_int64),
                ("m2p_pairs", ctypes.c_int64), ("dense_pairs", ctypes.c_int64),
                ("p2p_fused_pairs", ctypes.c_int64), ("matvecs", ctypes.c_int32),
                ("fp64_fallback", ctypes.c_int32), ("m2p_fused_pairs", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PbtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with "
                               "`python -m paper_1506_03745_amd.build` (there is no CPU fallback)")
        try:
            # PyTorch-ROCm loads its own HIP runtime (soname libamdhip64.so.7).
            # Loading it first lets the library bind to that same runtime, so
            # torch's device memory, streams and synchronisation are shared.
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, D, I32, I64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        L.pbt_default_params.argtypes = [ctypes.POINTER(PbtParams)]
        L.pbt_default_params.restype = None
        L.pbt_create.argtypes = [ctypes.POINTER(P), I32, ctypes.POINTER(PbtParams)]
        L.pbt_destroy.argtypes = [P]
        L.pbt_destroy.restype = None
        L.pbt_last_error.argtypes = [P]
        L.pbt_last_error.restype = ctypes.c_char_p
        L.pbt_set_params.argtypes = [P, ctypes.POINTER(PbtParams)]
        L.pbt_set_solvent.argtypes = [P, D, D]
        L.pbt_add_surface.argtypes = [P, I32, P, I64, P, I64, P, ctypes.POINTER(I32)]
        L.pbt_set_bc.argtypes = [P, I32, P]
        L.pbt_set_charges.argtypes = [P, I32, D, P, P, I64]
        L.pbt_set_stern.argtypes = [P, I32, I32, D]
        L.pbt_set_cavity.argtypes = [P, I32, I32, D]
        L.pbt_enable.argtypes = [P, I32, I32]
        L.pbt_num_unknowns.argtypes = [P, ctypes.POINTER(I64)]
        L.pbt_prepare.argtypes = [P]
        L.pbt_solve.argtypes = [P, P, ctypes.POINTER(PbtResult)]
        L.pbt_get_solution.argtypes = [P, I32, P, P]
        L.pbt_interaction_energy.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(PbtResult)]
        L.pbt_matvec.argtypes = [P, P, P, I32, I32]
        L.pbt_matvec_dev.argtypes = [P, P, P, I32, I32, P]
        L.pbt_rhs.argtypes = [P, P]
        L.pbt_gradient.argtypes = [P, I32, P, I32, P]
        L.pbt_solve_batch.argtypes = [P, I32, P, P, I32, P]
        L.pbt_autotune.argtypes = [P, ctypes.c_char_p]
        L.pbt_set_schedule.argtypes = [P, I32]
        L.pbt_get_schedule.argtypes = [P, ctypes.POINTER(I32)]
        L.pbt_set_gram_schmidt.argtypes = [P, I32]
        L.pbt_get_launch_shape.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
        L.pbt_last_stats.argtypes = [P, ctypes.POINTER(PbtResult)]
        L.pbt_quadrature_rule.argtypes = [I32, P, P]
        L.pbt_last_matvec_timing.argtypes = [P, P]
        L.pbt_profile.argtypes = [P, I32]
        L.pbt_set_bc_dev.argtypes = [P, I32, P, P]
        L.pbt_set_charges_dev.argtypes = [P, I32, D, P, P, I64, P]
        L.pbt_get_solution_dev.argtypes = [P, I32, P, P, P]
        L.pbt_gradient_dev.argtypes = [P, I32, P, I32, P, P]
        L.pbt_matvec_dev_static.argtypes = [P, P, P, I32, P]
        L.pbt_kernel_times.argtypes = [P, P]
        for name in EXPORTS:
            if name not in ("pbt_default_params", "pbt_destroy", "pbt_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def default_params():
    p = PbtParams()
    lib().pbt_default_params(ctypes.byref(p))
    return p


def quadrature_rule(npts: int):
    """The library's own rule: (bary (n,3), w (n,)) or GL (t, w) for npts < 0."""
    n = abs(npts)
    b = np.zeros(3 * n if npts > 0 else n)
    w = np.zeros(n)
    st = lib().pbt_quadrature_rule(npts, _ptr(b), _ptr(w))
    if st != 0:
        raise PbtError(st, f"no rule with {npts} points")
    return (b.reshape(n, 3) if npts > 0 else b), w


@dataclass
class Result:
    F_coul: float
    F_solv: float
    F_surf: float
    F_total: float
    iters: int
    outer: int
    rel_resid: float
    t_setup_s: float
    t_solve_s: float
    p2p_pairs: int
    m2p_pairs: int
    dense_pairs: int
    p2p_fused_pairs: int
    matvecs: int
    fp64_fallback: int = 0
    m2p_fused_pairs: int = 0
    status: int = 0


class Solver:
    """One library context on one HIP device."""

    def __init__(self, device: int = 0, **params):
        p = default_params()
        for k, v in params.items():
            if k == "prec" and isinstance(v, str):
                v = {"fp64": FP64, "mixed": MIXED}[v]
            setattr(p, k, v)
        self._p = p
        h = ctypes.c_void_p()
        st = lib().pbt_create(ctypes.byref(h), device, ctypes.byref(p))
        if st != 0:
            raise PbtError(st, "pbt_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().pbt_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st, ok=(0,)):
        if st not in ok:
            raise PbtError(st, lib().pbt_last_error(self._h).decode())
        return st

    @property
    def params(self):
        return self._p

    def set_params(self, **params):
        for k, v in params.items():
            if k == "prec" and isinstance(v, str):
                v = {"fp64": FP64, "mixed": MIXED}[v]
            setattr(self._p, k, v)
        self._check(lib().pbt_set_params(self._h, ctypes.byref(self._p)))

    def set_solvent(self, eps_out, kappa):
        self._check(lib().pbt_set_solvent(self._h, float(eps_out), float(kappa)))

    def add_surface(self, kind, verts, tris, bc=None) -> int:
        v = _f64(verts)
        t = np.ascontiguousarray(np.asarray(tris, dtype=np.int32))
        b = _f64(bc) if bc is not None else None
        sid = ctypes.c_int32()
        self._check(lib().pbt_add_surface(self._h, kind, _ptr(v), len(v), _ptr(t), len(t), _ptr(b),
                                          ctypes.byref(sid)))
        return sid.value

    def set_bc(self, sid, bc):
        b = _f64(bc)
        self._check(lib().pbt_set_bc(self._h, sid, _ptr(b)))

    def set_charges(self, mol_id, eps_in, xyz, q):
        x = _f64(xyz)
        qq = _f64(q)
        self._check(lib().pbt_set_charges(self._h, mol_id, float(eps_in), _ptr(x), _ptr(qq), len(qq)))

    def set_stern(self, stern_id, mol_id, eps_layer):
        self._check(lib().pbt_set_stern(self._h, stern_id, mol_id, float(eps_layer)))

    def set_cavity(self, cav_id, mol_id, eps_cavity):
        self._check(lib().pbt_set_cavity(self._h, cav_id, mol_id, float(eps_cavity)))

    def enable(self, sid, on=True):
        self._check(lib().pbt_enable(self._h, sid, 1 if on else 0))

    def prepare(self):
        self._check(lib().pbt_prepare(self._h))

    def num_unknowns(self) -> int:
        n = ctypes.c_int64()
        self._check(lib().pbt_num_unknowns(self._h, ctypes.byref(n)))
        return n.value

    def solve(self, x0=None, allow_noconverge=False) -> Result:
        r = PbtResult()
        x = _f64(x0) if x0 is not None else None
        st = self._check(lib().pbt_solve(self._h, _ptr(x), ctypes.byref(r)),
                         ok=(0, 4) if allow_noconverge else (0,))
        return Result(**r.as_dict(), status=st)

    def get_solution(self, sid, nt):
        phi = np.zeros(nt)
        d = np.zeros(nt)
        self._check(lib().pbt_get_solution(self._h, sid, _ptr(phi), _ptr(d)))
        return phi, d

    def interaction_energy(self, n_surfaces):
        f = ctypes.c_double()
        parts = (PbtResult * (n_surfaces + 1))()
        self._check(lib().pbt_interaction_energy(self._h, ctypes.byref(f), parts))
        return f.value, [Result(**p.as_dict()) for p in parts]

    def matvec(self, x, transpose=False, prec=FP64):
        x = _f64(x)
        y = np.zeros_like(x)
        self._check(lib().pbt_matvec(self._h, _ptr(x), _ptr(y), 1 if transpose else 0, prec))
        return y

    def matvec_dev(self, x, y, transpose=False, prec=FP64, stream=None):
        """x, y: contiguous float64 torch tensors on the context's device."""
        import torch
        assert x.dtype == torch.float64 and y.dtype == torch.float64 and x.is_contiguous() and y.is_contiguous()
        s = torch.cuda.current_stream(x.device) if stream is None else stream
        self._check(lib().pbt_matvec_dev(self._h, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(y.data_ptr()), 1 if transpose else 0, prec,
                                         ctypes.c_void_p(s.cuda_stream)))

    # -- device variants: float64 torch tensors on the context's device, read
    #    or written in the order of the tensor device's current stream
    @staticmethod
    def _dev(t, n=None):
        import torch
        if t is None:
            return None
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise TypeError("expected a contiguous float64 CUDA tensor")
        if n is not None and t.numel() != n:
            raise ValueError(f"expected {n} elements, got {t.numel()}")
        return ctypes.c_void_p(t.data_ptr())

    @staticmethod
    def _stream(t, stream=None):
        import torch
        s = torch.cuda.current_stream(t.device) if stream is None else stream
        return ctypes.c_void_p(s.cuda_stream)

    def set_bc_dev(self, sid, bc, stream=None):
        self._check(lib().pbt_set_bc_dev(self._h, sid, self._dev(bc), self._stream(bc, stream)))

    def set_charges_dev(self, mol_id, eps_in, q, xyz=None, stream=None):
        """q: (nq,) tensor; xyz: (nq, 3) tensor or None to keep the present positions."""
        self._check(lib().pbt_set_charges_dev(self._h, mol_id, float(eps_in), self._dev(xyz), self._dev(q),
                                              q.numel(), self._stream(q, stream)))

    def get_solution_dev(self, sid, phi, dphidn, stream=None):
        t = phi if phi is not None else dphidn
        self._check(lib().pbt_get_solution_dev(self._h, sid, self._dev(phi), self._dev(dphidn),
                                               self._stream(t, stream)))

    def gradient_dev(self, sigma_id, dsig, mol_id, dq, stream=None):
        t = dsig if dsig is not None else dq
        self._check(lib().pbt_gradient_dev(self._h, sigma_id, self._dev(dsig), mol_id, self._dev(dq),
                                           self._stream(t, stream)))

    def matvec_dev_static(self, x, y, prec=FP64, stream=None):
        """The forward product without allocations (pbt_matvec_dev_static);
        x, y: contiguous float64 torch tensors on the context's device."""
        n = self.num_unknowns()
        self._check(lib().pbt_matvec_dev_static(self._h, self._dev(x, n), self._dev(y, n), prec,
                                                self._stream(x, stream)))

    def rhs(self):
        b = np.zeros(self.num_unknowns())
        self._check(lib().pbt_rhs(self._h, _ptr(b)))
        return b

    def last_matvec_timing(self):
        out = np.zeros(5)
        self._check(lib().pbt_last_matvec_timing(self._h, _ptr(out)))
        return dict(zip(("total_ms", "p2p_ms", "m2p_ms", "moments_ms", "rest_ms"), out))

    def gradient(self, sigma_id, nt_sigma, mol_id, nq):
        ds = np.zeros(max(nt_sigma, 0))
        dq = np.zeros(max(nq, 0))
        self._check(lib().pbt_gradient(self._h, sigma_id, _ptr(ds) if sigma_id >= 0 else None, mol_id,
                                       _ptr(dq) if mol_id >= 0 else None))
        return ds, dq

    def solve_batch(self, mol_id, rot, shift):
        rot = _f64(rot).reshape(-1, 9)
        shift = _f64(shift).reshape(-1, 3)
        out = np.zeros(len(rot))
        self._check(lib().pbt_solve_batch(self._h, mol_id, _ptr(rot), _ptr(shift), len(rot), _ptr(out)))
        return out

    def autotune(self, cache_path=None):
        self._check(lib().pbt_autotune(self._h, cache_path.encode() if cache_path else None))

    def last_stats(self):
        r = PbtResult()
        self._check(lib().pbt_last_stats(self._h, ctypes.byref(r)))
        return r

    def set_schedule(self, mode):
        self._check(lib().pbt_set_schedule(self._h, int(mode)))

    def schedule(self):
        m = ctypes.c_int32()
        self._check(lib().pbt_get_schedule(self._h, ctypes.byref(m)))
        return m.value

    def launch_shape(self):
        """(P2P segment length, M2P boxes per task, stand-alone P2P and M2P work-items)."""
        out = (ctypes.c_int64 * 4)()
        self._check(lib().pbt_get_launch_shape(self._h, out))
        return tuple(int(v) for v in out)

    def profile(self, on=True):
        """Per-kernel HIP-event timing of every operator application (clears the totals)."""
        self._check(lib().pbt_profile(self._h, 1 if on else 0))

    def kernel_times(self):
        """{(prec, kind): (total ms, launches)}, prec 'fp32' / 'fp64', kind
        'p2p' / 'm2p' / 'moments' / 'combine' (see pbt_kernel_times)."""
        out = np.zeros(16)
        self._check(lib().pbt_kernel_times(self._h, _ptr(out)))
        kinds = ("p2p", "m2p", "moments", "combine")
        return {(p, k): (float(out[2 * (4 * i + j)]), int(out[2 * (4 * i + j) + 1]))
                for i, p in enumerate(("fp32", "fp64")) for j, k in enumerate(kinds)}

    def set_gram_schmidt(self, passes):
        self._check(lib().pbt_set_gram_schmidt(self._h, int(passes)))


def from_problem(problem, device=0, **params) -> tuple[Solver, list[int]]:
    """Create a Solver holding a workloads.Problem (marshalling only)."""
    prm = {k: v for k, v in getattr(problem, "params", {}).items() if k in dict(PbtParams._fields_)}
    prm.update(params)
    s = Solver(device, **prm)
    s.set_solvent(problem.eps_out, problem.kappa)
    ids = []
    for surf in problem.surfaces:
        sid = s.add_surface(surf.kind, surf.verts, surf.tris, surf.bc)
        if surf.kind == MOLECULE:
            q = surf.q if surf.q is not None else np.zeros(0)
            qp = surf.q_pos if surf.q_pos is not None else np.zeros((0, 3))
            s.set_charges(sid, surf.eps_in, qp, q)
        ids.append(sid)
    for surf, sid in zip(problem.surfaces, ids):
        if surf.kind == STERN:
            s.set_stern(sid, ids[surf.parent], surf.eps_in)
        elif surf.kind == CAVITY:
            s.set_cavity(sid, ids[surf.parent], surf.eps_in)
    return s, ids
