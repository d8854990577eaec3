"""Python binding of libpsint.so (include/psint.h): argument marshalling only.

Every step of the integral pipeline runs in the HIP library on the GPU; this module converts jobs to
the C structs, allocates device outputs as torch tensors when asked (torch is used only for device
memory and streams), and raises if the library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Iterable, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsint.so")

PS_OK, PS_E_INVALID, PS_E_UNSUPPORTED, PS_E_NOMEM, PS_E_DEVICE, PS_E_NOT_PD, PS_E_TIMEOUT, \
    PS_E_QUEUE_FULL, PS_E_NOT_FOUND = 0, -1, -2, -3, -4, -5, -6, -7, -8
PREC = {"fp64": 0, "mixed": 1}
PS_OPT_SHARE_THIRD_CENTRE = 1
PS_OPT_OVERLAP_PASSES = 2
OUTPUTS = ("S", "T", "V", "PQ", "PQ_chol", "abP")


class PsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"psint status {status}: {msg}")
        self.status = status


class Atom(C.Structure):
    _fields_ = [("xyz", C.c_double * 3), ("Z", C.c_double)]


class Sto(C.Structure):
    _fields_ = [("atom", C.c_int32), ("n", C.c_int32), ("l", C.c_int32), ("m", C.c_int32),
                ("zeta", C.c_double)]


class GridSpec(C.Structure):
    _fields_ = [("n_mu", C.c_int32), ("n_nu", C.c_int32), ("n_phi", C.c_int32), ("q", C.c_int32),
                ("n_sp", C.c_int32), ("c1_scale", C.c_double), ("c1_exp", C.c_double)]


class PairGrid(C.Structure):
    _fields_ = [("atom_a", C.c_int32), ("atom_b", C.c_int32), ("spec", GridSpec)]


_dp = C.POINTER(C.c_double)


class Job(C.Structure):
    _fields_ = [("atoms", C.POINTER(Atom)), ("n_atoms", C.c_int32),
                ("basis", C.POINTER(Sto)), ("n_bf", C.c_int32),
                ("aux", C.POINTER(Sto)), ("n_aux", C.c_int32),
                ("grid", GridSpec),
                ("pair_grids", C.POINTER(PairGrid)), ("n_pair_grids", C.c_int32),
                ("precision", C.c_int32), ("out_location", C.c_int32),
                ("S", _dp), ("T", _dp), ("V", _dp), ("PQ", _dp), ("PQ_chol", _dp), ("abP", _dp)]


class JobStats(C.Structure):
    _fields_ = [("n_grids", C.c_int64), ("n_points", C.c_int64), ("pair_points", C.c_double),
                ("queue_ms", C.c_double), ("device_ms", C.c_double), ("total_ms", C.c_double),
                ("contract_ms", C.c_double), ("contract_flops", C.c_double), ("issued_flops", C.c_double),
                ("n_passes", C.c_int64), ("graph_replay", C.c_int64),
                ("passes_overlapped", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tuning(C.Structure):
    _fields_ = [("wm", C.c_int32), ("wn", C.c_int32), ("stage_chunks", C.c_int32), ("ksplit", C.c_int32),
                ("device_ms", C.c_double), ("contract_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None


def lib():
    """Load libpsint.so; raise if it has not been built (no fallback path exists)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() or "
                              "python paper_2510_15204_amd/build.py")
        # One HIP runtime per process: torch ships its own libamdhip64 (same soname), so load torch
        # first and let libpsint bind to the runtime torch already mapped.  Otherwise a later torch
        # import would bring up a second HIP/HSA runtime that cannot see the GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.ps_create.argtypes = [C.c_int32, C.c_size_t, vp, C.POINTER(vp)]
        L.ps_destroy.argtypes = [vp]
        L.ps_compute.argtypes = [vp, C.POINTER(Job), C.POINTER(JobStats)]
        L.ps_submit.argtypes = [vp, C.POINTER(Job), C.POINTER(C.c_uint64)]
        L.ps_wait.argtypes = [vp, C.c_uint64, C.c_int64, C.POINTER(JobStats)]
        L.ps_grid_points.argtypes = [vp, C.POINTER(Atom), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     C.POINTER(GridSpec), _dp, C.POINTER(C.c_int64)]
        L.ps_eval_function.argtypes = [vp, C.c_int32, C.POINTER(Sto), _dp, C.c_int64, _dp, _dp, _dp, _dp]
        L.ps_plan_work.argtypes = [vp, C.POINTER(Job), _dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_size_t)]
        L.ps_set_tiling.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.ps_autotune.argtypes = [vp, C.POINTER(Job), C.c_int32, C.POINTER(Tuning), C.POINTER(Tuning), C.c_int32,
                                  C.POINTER(C.c_int32)]
        L.ps_ri_assemble.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp, vp, _dp]
        L.ps_mfma_rate.argtypes = [vp, C.c_int32, _dp]
        L.ps_ri_assemble_noalloc.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp, vp]
        L.ps_set_option.argtypes = [vp, C.c_int32, C.c_int64]
        L.ps_status_string.argtypes = [C.c_int32]
        L.ps_status_string.restype = C.c_char_p
        L.ps_last_error.argtypes = [vp]
        L.ps_last_error.restype = C.c_char_p
        for f in ("ps_create", "ps_destroy", "ps_compute", "ps_submit", "ps_wait", "ps_grid_points",
                  "ps_eval_function", "ps_plan_work", "ps_set_tiling", "ps_autotune", "ps_ri_assemble",
                  "ps_mfma_rate", "ps_ri_assemble_noalloc", "ps_set_option"):
            getattr(L, f).restype = C.c_int32
        _LIB = L
    return _LIB


def plan_work_host(job, precision=None):
    """Host-only planning (no GPU): pair-points, grids, points, device bytes."""
    ref = _JobRef(job, precision)
    pp = C.c_double()
    ng, npnt = C.c_int64(), C.c_int64()
    nbytes = C.c_size_t()
    rc = lib().ps_plan_work(None, C.byref(ref.j), C.byref(pp), C.byref(ng), C.byref(npnt), C.byref(nbytes))
    if rc != PS_OK:
        raise PsError(rc, lib().ps_status_string(rc).decode())
    return {"pair_points": pp.value, "n_grids": ng.value, "n_points": npnt.value, "device_bytes": nbytes.value}


def exported_symbols():
    return ["ps_create", "ps_destroy", "ps_compute", "ps_submit", "ps_wait", "ps_grid_points",
            "ps_eval_function", "ps_plan_work", "ps_set_tiling", "ps_autotune", "ps_ri_assemble",
            "ps_mfma_rate", "ps_ri_assemble_noalloc", "ps_set_option", "ps_status_string", "ps_last_error"]


def _spec(s) -> GridSpec:
    t = s.as_tuple() if hasattr(s, "as_tuple") else tuple(s)
    return GridSpec(int(t[0]), int(t[1]), int(t[2]), int(t[3]), int(t[4]), float(t[5]), float(t[6]))


def _stos(arr) -> "C.Array":
    arr = np.asarray(arr, dtype=np.float64).reshape(-1, 5)
    out = (Sto * max(len(arr), 1))()
    for i, r in enumerate(arr):
        out[i] = Sto(int(r[0]), int(r[1]), int(r[2]), int(r[3]), float(r[4]))
    return out


class _JobRef:
    """C job struct plus the buffers it points into."""

    def __init__(self, job, precision: Optional[str] = None):
        xyz = np.asarray(job.xyz, dtype=np.float64).reshape(-1, 3)
        Z = np.asarray(job.Z, dtype=np.float64)
        self.atoms = (Atom * len(xyz))()
        for i in range(len(xyz)):
            self.atoms[i] = Atom((C.c_double * 3)(*xyz[i]), float(Z[i]))
        self.basis = _stos(job.basis)
        self.aux = _stos(job.aux)
        pg = getattr(job, "pair_grids", {}) or {}
        keys = sorted(pg)
        self.pairs = (PairGrid * max(len(keys), 1))()
        for i, k in enumerate(keys):
            self.pairs[i] = PairGrid(int(k[0]), int(k[1]), _spec(pg[k]))
        j = Job()
        j.atoms = self.atoms
        j.n_atoms = len(xyz)
        j.basis = self.basis
        j.n_bf = int(np.asarray(job.basis).reshape(-1, 5).shape[0])
        j.aux = self.aux
        j.n_aux = int(np.asarray(job.aux).reshape(-1, 5).shape[0])
        j.grid = _spec(job.grid)
        j.pair_grids = self.pairs
        j.n_pair_grids = len(keys)
        prec = precision or getattr(job, "precision", "fp64")
        j.precision = PREC[prec]
        j.out_location = 0
        self.j = j
        self.n_bf = j.n_bf
        self.n_aux = j.n_aux

    def shapes(self):
        nb, na = self.n_bf, self.n_aux
        return {"S": (nb, nb), "T": (nb, nb), "V": (nb, nb), "PQ": (na, na), "PQ_chol": (na, na),
                "abP": (na, nb, nb)}


class Context:
    """A device context (ps_create).  `stream` may be a torch.cuda.Stream or a raw hipStream_t."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, stream=None):
        L = lib()
        h = C.c_void_p()
        raw = None
        if stream is not None:
            raw = C.c_void_p(getattr(stream, "cuda_stream", stream))
        rc = L.ps_create(device, budget_bytes, raw, C.byref(h))
        if rc != PS_OK:
            raise PsError(rc, L.ps_status_string(rc).decode())
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib().ps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(PS_OK,)):
        if rc not in allow:
            msg = lib().ps_last_error(self.h)
            raise PsError(rc, (msg or b"").decode() or lib().ps_status_string(rc).decode())
        return rc

    def set_option(self, option, value):
        self._check(lib().ps_set_option(self.h, int(option), int(value)))

    def set_tiling(self, wm=0, wn=0, stage_chunks=0, ksplit=0):
        self._check(lib().ps_set_tiling(self.h, wm, wn, stage_chunks, ksplit))

    def autotune(self, job, precision=None, reps=1):
        """Time every candidate contraction tiling on `job` (ps_autotune); the fastest stays set on
        the context.  Returns (best, table) as dicts."""
        ref = _JobRef(job, precision)
        best = Tuning()
        table = (Tuning * 16)()
        n = C.c_int32()
        self._check(lib().ps_autotune(self.h, C.byref(ref.j), reps, C.byref(best), table, 16, C.byref(n)))
        return best.as_dict(), [table[i].as_dict() for i in range(n.value)]

    def ri_assemble(self, abP, L, want_B=True, want_eri=True):
        """RI assembly (ps_ri_assemble) on abP [P][a][b] and the lower factor L.  numpy inputs give
        numpy outputs (host path); torch device tensors give device tensors.  Returns
        (B or None, eri or None, device_ms)."""
        na, nb = int(abP.shape[0]), int(abP.shape[1])
        npair = nb * (nb + 1) // 2
        dev = not isinstance(abP, np.ndarray)
        if dev:
            import torch
            assert abP.dtype == torch.float64 and L.dtype == torch.float64 and abP.is_cuda and L.is_cuda
            abP, L = abP.contiguous(), L.contiguous()
            mk = lambda shape: torch.empty(shape, dtype=torch.float64, device=abP.device)  # noqa: E731
            ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        else:
            abP = np.ascontiguousarray(abP, dtype=np.float64)
            L = np.ascontiguousarray(L, dtype=np.float64)
            mk = lambda shape: np.empty(shape)  # noqa: E731
            ptr = lambda a: C.c_void_p(a.ctypes.data) if a is not None else None  # noqa: E731
        B = mk((na, npair)) if want_B else None
        eri = mk((npair, npair)) if want_eri else None
        ms = C.c_double()
        self._check(lib().ps_ri_assemble(self.h, nb, na, 1 if dev else 0, ptr(abP), ptr(L), ptr(B), ptr(eri),
                                         C.byref(ms)))
        return B, eri, ms.value

    def ri_assemble_noalloc(self, abP, L, B=None, eri=None):
        """ps_ri_assemble_noalloc on device tensors: abP [P][a][b] and the lower factor L in, the
        caller's B (n_aux x n_pair) and eri (n_pair x n_pair) tensors out (None = not wanted).  The
        kernels are only enqueued on the context's stream; synchronise before reading the outputs."""
        import torch
        for t in (abP, L, B, eri):
            assert t is None or (t.dtype == torch.float64 and t.is_cuda and t.is_contiguous())
        na, nb = int(abP.shape[0]), int(abP.shape[1])
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
        self._check(lib().ps_ri_assemble_noalloc(self.h, nb, na, ptr(abP), ptr(L), ptr(B), ptr(eri)))

    def mfma_rate(self, precision="fp64"):
        """Measured matrix-pipe throughput of the device in TFLOP/s (ps_mfma_rate): FP64 MFMA for
        "fp64", FP32 MFMA for "mixed"."""
        t = C.c_double()
        self._check(lib().ps_mfma_rate(self.h, PREC[precision], C.byref(t)))
        return t.value

    def plan_work(self, job, precision=None):
        ref = _JobRef(job, precision)
        pp = C.c_double()
        ng, npnt = C.c_int64(), C.c_int64()
        nbytes = C.c_size_t()
        self._check(lib().ps_plan_work(self.h, C.byref(ref.j), C.byref(pp), C.byref(ng), C.byref(npnt),
                                       C.byref(nbytes)))
        return {"pair_points": pp.value, "n_grids": ng.value, "n_points": npnt.value,
                "device_bytes": nbytes.value}

    def _bind_outputs(self, ref, outputs, device, out_tensors):
        res = {}
        for name in OUTPUTS:
            if name not in outputs:
                setattr(ref.j, name, None)
                continue
            shape = ref.shapes()[name]
            if device:
                import torch
                if out_tensors is not None and name in out_tensors:
                    t = out_tensors[name]
                    assert t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == shape
                else:
                    t = torch.empty(shape, dtype=torch.float64, device=f"cuda:{self.device}")
                res[name] = t
                setattr(ref.j, name, C.cast(C.c_void_p(t.data_ptr()), _dp))
            else:
                a = np.zeros(shape)
                res[name] = a
                setattr(ref.j, name, a.ctypes.data_as(_dp))
        ref.j.out_location = 1 if device else 0
        return res

    def compute(self, job, outputs: Iterable[str] = OUTPUTS, precision=None, device=False,
                out_tensors: Optional[Dict] = None, allow_not_pd=True):
        """Run one job.  Returns (outputs dict, stats dict, status)."""
        ref = _JobRef(job, precision)
        res = self._bind_outputs(ref, tuple(outputs), device, out_tensors)
        st = JobStats()
        allow = (PS_OK, PS_E_NOT_PD) if allow_not_pd else (PS_OK,)
        rc = self._check(lib().ps_compute(self.h, C.byref(ref.j), C.byref(st)), allow)
        return res, st.as_dict(), rc

    def submit(self, job, outputs: Iterable[str] = OUTPUTS, precision=None, device=False):
        """Queue a job; returns a handle for wait().  Output buffers live in the handle."""
        ref = _JobRef(job, precision)
        res = self._bind_outputs(ref, tuple(outputs), device, None)
        t = C.c_uint64()
        self._check(lib().ps_submit(self.h, C.byref(ref.j), C.byref(t)))
        return {"ticket": t.value, "ref": ref, "out": res}

    def wait(self, handle, timeout_us=-1, allow_not_pd=True):
        st = JobStats()
        rc = lib().ps_wait(self.h, handle["ticket"], timeout_us, C.byref(st))
        if rc == PS_E_TIMEOUT:
            return None, None, rc
        allow = (PS_OK, PS_E_NOT_PD) if allow_not_pd else (PS_OK,)
        self._check(rc, allow)
        return handle["out"], st.as_dict(), rc

    def grid_points(self, xyz, A, B, C_=-1, spec=None, count_only=False):
        xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
        atoms = (Atom * len(xyz))()
        for i in range(len(xyz)):
            atoms[i] = Atom((C.c_double * 3)(*xyz[i]), 1.0)
        sp = _spec(spec)
        n = C.c_int64()
        self._check(lib().ps_grid_points(self.h, atoms, len(xyz), A, B, C_, C.byref(sp), None, C.byref(n)))
        if count_only:
            return n.value
        out = np.zeros((n.value, 4))
        self._check(lib().ps_grid_points(self.h, atoms, len(xyz), A, B, C_, C.byref(sp),
                                         out.ctypes.data_as(_dp), C.byref(n)))
        return out

    def eval_function(self, what, fn, center, x, y, z):
        code = {"chi": 0, "kin": 1, "pot": 2}[what]
        f = np.asarray(fn, dtype=np.float64).reshape(5)
        s = Sto(int(f[0]), int(f[1]), int(f[2]), int(f[3]), float(f[4]))
        c = np.ascontiguousarray(np.asarray(center, dtype=np.float64).reshape(3))
        x, y, z = (np.ascontiguousarray(np.asarray(v, dtype=np.float64).ravel()) for v in (x, y, z))
        out = np.zeros(x.size)
        self._check(lib().ps_eval_function(self.h, code, C.byref(s), c.ctypes.data_as(_dp), x.size,
                                           x.ctypes.data_as(_dp), y.ctypes.data_as(_dp),
                                           z.ctypes.data_as(_dp), out.ctypes.data_as(_dp)))
        return out
