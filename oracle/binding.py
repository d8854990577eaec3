"""ctypes binding of the plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Jobs are duck-typed: any object with ``xyz`` (n,3), ``Z`` (n,), ``basis`` (n_bf,5), ``aux`` (n_aux,5),
``grid`` (with ``as_tuple()``) and ``pair_grids`` ({(a,b): spec}) works.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

S, T, V, PQ, ABP = 0, 1, 2, 3, 4
KIND = {"S": S, "T": T, "V": V, "PQ": PQ, "abP": ABP}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class _Job(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32), ("xyz", _dp), ("Z", _dp),
        ("n_bf", C.c_int32), ("bf", _dp),
        ("n_aux", C.c_int32), ("aux", _dp),
        ("spec", C.c_double * 7),
        ("n_pair_specs", C.c_int32), ("pair_ab", _ip), ("pair_spec", _dp),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libpsoracle.so")
        if not os.path.exists(path):
            from .build import build
            build()
        L = C.CDLL(path)
        L.orc_gauss_legendre.argtypes = [C.c_int32, _dp, _dp]
        L.orc_grid_info.argtypes = [_dp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _dp, _lp, _dp,
                                    _dp, _dp, _dp]
        L.orc_grid_points.argtypes = [_dp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _dp, _dp, _dp,
                                      _dp, _dp]
        L.orc_eval.argtypes = [C.c_int32, _dp, _dp, C.c_int64, _dp, _dp, _dp, _dp]
        L.orc_lower_gamma.argtypes = [C.c_int32, C.c_double]
        L.orc_lower_gamma.restype = C.c_double
        L.orc_upper_gamma.argtypes = [C.c_int32, C.c_double]
        L.orc_upper_gamma.restype = C.c_double
        L.orc_compute_elements.argtypes = [C.POINTER(_Job), C.c_int64, _ip, _ip, _ip, _ip, _dp, _dp]
        L.orc_compute_full.argtypes = [C.POINTER(_Job), _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_cholesky.argtypes = [C.c_int32, _dp, _dp]
        L.orc_grid_list.argtypes = [C.POINTER(_Job), _ip, C.c_int64]
        L.orc_grid_list.restype = C.c_int64
        L.orc_route.argtypes = [C.POINTER(_Job), C.c_int32, C.c_int32, C.c_int32, C.c_int32, _ip, C.c_int32]
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_set_threads.restype = C.c_int32
        _LIB = L
    return _LIB


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _spec(s):
    return np.ascontiguousarray(np.array(s.as_tuple() if hasattr(s, "as_tuple") else s, dtype=np.float64))


def set_threads(n=0):
    return lib().orc_set_threads(int(n))


def gauss_legendre(q):
    x = np.zeros(q)
    w = np.zeros(q)
    if lib().orc_gauss_legendre(q, _d(x), _d(w)) != 0:
        raise ValueError("bad q")
    return x, w


def grid_info(xyz, A, B, C=-1, spec=None):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    sp = _spec(spec)
    info = np.zeros(8, dtype=np.int64)
    mu = np.zeros(int(sp[0]) + 1)
    nu = np.zeros(int(sp[1]) + 1)
    phi = np.zeros(int(sp[2]) + 1)
    frame = np.zeros(13)
    rc = lib().orc_grid_info(_d(xyz), xyz.shape[0], A, B, C, _d(sp), info.ctypes.data_as(_lp), _d(mu),
                             _d(nu), _d(phi), _d(frame))
    if rc:
        raise ValueError(f"grid_info rc={rc}")
    return dict(n_points=int(info[0]), moved_mu=bool(info[1]), moved_nu=bool(info[2]), split=bool(info[3]),
                istar=int(info[4]), jstar=int(info[5]), n_cells=int(info[6]), mu=mu, nu=nu, phi=phi,
                a=frame[0], M=frame[1:4], ex=frame[4:7], ey=frame[7:10], ez=frame[10:13])


def grid_points(xyz, A, B, C=-1, spec=None):
    info = grid_info(xyz, A, B, C, spec)
    n = info["n_points"]
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    sp = _spec(spec)
    x, y, z, w = (np.zeros(n) for _ in range(4))
    rc = lib().orc_grid_points(_d(xyz), xyz.shape[0], A, B, C, _d(sp), _d(x), _d(y), _d(z), _d(w))
    if rc:
        raise ValueError(f"grid_points rc={rc}")
    return x, y, z, w


def eval_fn(what, fn, center, x, y, z):
    """what: 'chi', 'kin' (-1/2 lap chi), 'pot' (Coulomb potential of chi), 'ylm'."""
    code = {"chi": 0, "kin": 1, "pot": 2, "ylm": 3}[what]
    f = np.ascontiguousarray(np.asarray(fn, dtype=np.float64).reshape(5))
    c = np.ascontiguousarray(np.asarray(center, dtype=np.float64).reshape(3))
    x, y, z = (np.ascontiguousarray(np.asarray(v, dtype=np.float64).ravel()) for v in (x, y, z))
    out = np.zeros(x.size)
    if lib().orc_eval(code, _d(f), _d(c), x.size, _d(x), _d(y), _d(z), _d(out)) != 0:
        raise ValueError("bad function")
    return out


def lower_gamma(k, x):
    return lib().orc_lower_gamma(int(k), float(x))


def upper_gamma(k, x):
    return lib().orc_upper_gamma(int(k), float(x))


class _JobRef:
    """Keeps the numpy buffers behind an orc_job alive."""

    def __init__(self, job):
        self.xyz = np.ascontiguousarray(job.xyz, dtype=np.float64)
        self.Z = np.ascontiguousarray(job.Z, dtype=np.float64)
        self.bf = np.ascontiguousarray(job.basis, dtype=np.float64).reshape(-1, 5)
        self.aux = np.ascontiguousarray(job.aux, dtype=np.float64).reshape(-1, 5)
        pg = getattr(job, "pair_grids", {}) or {}
        keys = sorted(pg)
        self.pab = np.ascontiguousarray(np.array(keys, dtype=np.int32).reshape(-1, 2))
        self.pspec = np.ascontiguousarray(
            np.array([_spec(pg[k]) for k in keys], dtype=np.float64).reshape(-1, 7))
        s = _Job()
        s.n_atoms = self.xyz.shape[0]
        s.xyz = _d(self.xyz)
        s.Z = _d(self.Z)
        s.n_bf = self.bf.shape[0]
        s.bf = _d(self.bf)
        s.n_aux = self.aux.shape[0]
        s.aux = _d(self.aux)
        for t, v in enumerate(_spec(job.grid)):
            s.spec[t] = v
        s.n_pair_specs = len(keys)
        s.pair_ab = _i(self.pab)
        s.pair_spec = _d(self.pspec)
        self.s = s


def grid_list(job):
    ref = _JobRef(job)
    n = lib().orc_grid_list(C.byref(ref.s), None, 0)
    abc = np.zeros((n, 3), dtype=np.int32)
    lib().orc_grid_list(C.byref(ref.s), _i(abc), n)
    return [tuple(int(v) for v in r) for r in abc]


def route(job, kind, i, j, k=0):
    """Contributions of one element: list of ((A, B, C), nuclei) with C = -1 for an unrefined grid."""
    ref = _JobRef(job)
    cap = 2 + ref.xyz.shape[0]
    out = np.zeros((cap, 6), dtype=np.int32)
    n = lib().orc_route(C.byref(ref.s), int(kind), int(i), int(j), int(k), _i(out), cap)
    if n < 0:
        raise ValueError(f"route rc={n}")
    return [((int(r[0]), int(r[1]), int(r[2])), tuple(int(v) for v in r[4:4 + r[3]])) for r in out[:n]]


def compute_elements(job, kinds, i, j, k=None):
    """Selected integrals.  Returns (values, pair_points)."""
    ref = _JobRef(job)
    kinds = np.ascontiguousarray(np.asarray(kinds, dtype=np.int32).ravel())
    n = kinds.size
    i = np.ascontiguousarray(np.asarray(i, dtype=np.int32).ravel())
    j = np.ascontiguousarray(np.asarray(j, dtype=np.int32).ravel())
    k = np.ascontiguousarray(np.zeros(n, dtype=np.int32) if k is None else np.asarray(k, dtype=np.int32).ravel())
    out = np.zeros(n)
    wpp = np.zeros(1)
    rc = lib().orc_compute_elements(C.byref(ref.s), n, _i(kinds), _i(i), _i(j), _i(k), _d(out), _d(wpp))
    if rc:
        raise ValueError(f"compute_elements rc={rc}")
    return out, float(wpp[0])


def compute_full(job, want=("S", "T", "V", "PQ", "PQ_chol", "abP")):
    """All requested outputs as a dict of numpy arrays, plus 'status' and 'pair_points'."""
    ref = _JobRef(job)
    nb, na = ref.bf.shape[0], ref.aux.shape[0]
    res = {}
    shapes = {"S": (nb, nb), "T": (nb, nb), "V": (nb, nb), "PQ": (na, na), "PQ_chol": (na, na),
              "abP": (na, nb, nb)}
    ptrs = []
    for key in ("S", "T", "V", "PQ", "PQ_chol", "abP"):
        if key in want:
            res[key] = np.zeros(shapes[key])
            ptrs.append(_d(res[key]))
        else:
            ptrs.append(None)
    wpp = np.zeros(1)
    rc = lib().orc_compute_full(C.byref(ref.s), *ptrs, _d(wpp))
    if rc not in (0, -5):
        raise ValueError(f"compute_full rc={rc}")
    res["status"] = rc
    res["pair_points"] = float(wpp[0])
    return res


def cholesky(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros_like(A)
    rc = lib().orc_cholesky(n, _d(A), _d(L))
    return L, rc
