"""ctypes wrapper over ``oracle.c`` (test infrastructure only; see the package docstring)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ANALYTIC, ANALYTIC_SF, TABLE, MLP = 0, 1, 2, 3
MLP_H = 32
MLP_PARAMS = MLP_H * (MLP_H + 4) + 1  # W1, b1, W2, b2, w3, b3

_lib = None


def library_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


class _Table(C.Structure):
    _fields_ = [("x0", C.c_double), ("h", C.c_double), ("n", C.c_int64),
                ("y", C.POINTER(C.c_double)), ("m", C.POINTER(C.c_double))]


class _Mlp(C.Structure):
    _fields_ = [("x_lo", C.c_double), ("x_hi", C.c_double), ("y_shift", C.c_double),
                ("y_scale", C.c_double), ("p", C.POINTER(C.c_double))]


class _Potential(C.Structure):
    _fields_ = [("mode", C.c_int32), ("pad_", C.c_int32), ("rc", C.c_double),
                ("f_beta", C.c_double), ("f_re", C.c_double), ("m_d", C.c_double),
                ("m_alpha", C.c_double), ("m_r0", C.c_double), ("emb_a", C.c_double),
                ("f", _Table), ("phi", _Table), ("emb", _Table),
                ("mf", _Mlp), ("mphi", _Mlp), ("memb", _Mlp)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int64)


def _declare(lib):
    lib.orc_spline_slopes.argtypes = [_dp, C.c_int64, _dp]
    lib.orc_spline_eval.argtypes = [C.POINTER(_Table), C.c_double, _dp, _dp]
    lib.orc_spline_eval.restype = C.c_int
    for nm in ("orc_pot_f", "orc_pot_phi"):
        getattr(lib, nm).argtypes = [C.POINTER(_Potential), C.c_double, _dp, _dp]
    lib.orc_pot_emb.argtypes = [C.POINTER(_Potential), C.c_double, _dp, _dp]
    lib.orc_mlp_eval.argtypes = [C.POINTER(_Mlp), C.c_double, _dp, _dp]
    lib.orc_mlp_eval.restype = None
    lib.orc_pot_emb.restype = C.c_int
    for nm in ("orc_eam_brute", "orc_eam_cells"):
        getattr(lib, nm).argtypes = [C.POINTER(_Potential), _dp, C.c_int64, _dp, _dp, _dp, _dp, _dp, _ip]
        getattr(lib, nm).restype = C.c_int
    lib.orc_eam_sampled.argtypes = [C.POINTER(_Potential), _dp, C.c_int64, _dp, _ip, C.c_int64, _dp, _dp, _dp,
                                    _ip]
    lib.orc_eam_sampled.restype = C.c_int
    lib.orc_neighbours.argtypes = [_dp, C.c_int64, _dp, C.c_double, C.c_int64, C.c_int, _ip, C.c_int64]
    lib.orc_neighbours.restype = C.c_int64
    lib.orc_kinetic.argtypes = [_dp, C.c_int64, C.c_double]
    lib.orc_kinetic.restype = C.c_double
    lib.orc_acc_unit.restype = C.c_double
    lib.orc_run.argtypes = [C.POINTER(_Potential), _dp, _dp, _dp, C.c_int64, _dp, C.c_double, C.c_int64,
                            C.c_double, C.c_double, C.c_int, C.c_int, _dp]
    lib.orc_run.restype = C.c_int
    lib.orc_lattice_id.argtypes = [C.c_int64] * 5
    lib.orc_lattice_id.restype = C.c_int64
    lib.orc_lattice_coords.argtypes = [C.c_int64, C.c_int64, C.c_int64, _ip, _ip, _ip]
    lib.orc_site_position.argtypes = [C.c_double, C.c_int64, C.c_int64, C.c_int64, _dp]
    lib.orc_stencil.argtypes = [C.c_double, C.c_double, C.c_int, _ip, C.c_int64]
    lib.orc_stencil.restype = C.c_int64
    lib.orc_nearest_site_brute.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_double, _dp, _dp]
    lib.orc_nearest_site_brute.restype = C.c_int64
    lib.orc_hash.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_double, _dp, _dp, _dp]
    lib.orc_hash.restype = C.c_int64
    for nm in ("orc_place", "orc_rehash"):
        getattr(lib, nm).argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_double, C.c_double, _dp, C.c_int64, _ip]
    lib.orc_num_threads.restype = C.c_int


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Potential:
    """Potential for the oracle: analytic, analytic shifted-force, splined tables,
    or surrogate networks with the tables outside their ranges.

    ``tables`` is {"f": (x0, h, y), "phi": (x0, h, y), "F": (x0, h, y)} of samples;
    node slopes are computed by the oracle's own spline routine.  ``mlp`` (mode
    MLP) is {"f": net, "phi": net, "F": net} with net = (x_lo, x_hi, y_shift,
    y_scale, params[MLP_PARAMS]).
    """

    def __init__(self, mode=ANALYTIC, rc=5.0, params=None, tables=None, mlp=None):
        p = dict(f_beta=3.0, f_re=2.47, m_d=0.4, m_alpha=1.6, m_r0=2.5, emb_a=1.0)
        if params:
            p.update(params)
        self.mode, self.rc, self.params = mode, rc, p
        self._keep = []
        s = _Potential()
        s.mode, s.rc = mode, rc
        for k, v in p.items():
            setattr(s, k, v)
        if mode in (TABLE, MLP):
            if tables is None:
                raise ValueError("table mode needs tables")
            for fld, key in (("f", "f"), ("phi", "phi"), ("emb", "F")):
                x0, h, y = tables[key]
                y = _f64(y)
                m = spline_slopes(y)
                self._keep += [y, m]
                t = _Table(float(x0), float(h), len(y), _d(y), _d(m))
                setattr(s, fld, t)
        if mode == MLP:
            if mlp is None:
                raise ValueError("MLP mode needs networks")
            for fld, key in (("mf", "f"), ("mphi", "phi"), ("memb", "F")):
                lo, hi, sh, sc, prm = mlp[key]
                prm = _f64(prm)
                if prm.shape != (MLP_PARAMS,):
                    raise ValueError("network needs %d parameters" % MLP_PARAMS)
                self._keep.append(prm)
                setattr(s, fld, _Mlp(float(lo), float(hi), float(sh), float(sc), _d(prm)))
        self._s = s

    @property
    def ref(self):
        return C.byref(self._s)

    def f(self, r):
        return self._eval("orc_pot_f", r)

    def phi(self, r):
        return self._eval("orc_pot_phi", r)

    def emb(self, rho):
        return self._eval("orc_pot_emb", rho)

    def _eval(self, name, xs):
        lib = _load()
        xs = np.atleast_1d(np.asarray(xs, dtype=np.float64))
        v = np.empty_like(xs)
        d = np.empty_like(xs)
        a, b = C.c_double(), C.c_double()
        fn = getattr(lib, name)
        for k, x in enumerate(xs):
            fn(self.ref, float(x), C.byref(a), C.byref(b))
            v[k], d[k] = a.value, b.value
        return v, d


def mlp_eval(net, xs):
    """Value and d/dx of one surrogate network (the C oracle's own evaluation)."""
    lib = _load()
    lo, hi, sh, sc, prm = net
    prm = _f64(prm)
    m = _Mlp(float(lo), float(hi), float(sh), float(sc), _d(prm))
    xs = np.atleast_1d(np.asarray(xs, dtype=np.float64))
    v = np.empty_like(xs)
    d = np.empty_like(xs)
    a, b = C.c_double(), C.c_double()
    for k, x in enumerate(xs):
        lib.orc_mlp_eval(C.byref(m), float(x), C.byref(a), C.byref(b))
        v[k], d[k] = a.value, b.value
    return v, d


def spline_slopes(y):
    lib = _load()
    y = _f64(y)
    m = np.empty_like(y)
    lib.orc_spline_slopes(_d(y), len(y), _d(m))
    return m


def spline_eval(x0, h, y, xs):
    """Value and derivative of the oracle's spline of samples y at points xs."""
    lib = _load()
    y = _f64(y)
    m = spline_slopes(y)
    t = _Table(float(x0), float(h), len(y), _d(y), _d(m))
    xs = np.atleast_1d(np.asarray(xs, dtype=np.float64))
    v, dd = np.empty_like(xs), np.empty_like(xs)
    extrap = np.zeros(len(xs), dtype=bool)
    a, b = C.c_double(), C.c_double()
    for k, x in enumerate(xs):
        extrap[k] = bool(lib.orc_spline_eval(C.byref(t), float(x), C.byref(a), C.byref(b)))
        v[k], dd[k] = a.value, b.value
    return v, dd, extrap


def eam(pot: Potential, x, box, cells=False, want_pairs=False):
    """Per-atom rho, F', forces and [E_emb, E_pair] (brute force, or exact cell-binned)."""
    lib = _load()
    x = _f64(x, (-1, 3))
    N = x.shape[0]
    L = _f64(box)
    rho, fp = np.empty(N), np.empty(N)
    F = np.empty((N, 3))
    en = np.empty(2)
    npairs = np.empty(N, dtype=np.int64)
    fn = lib.orc_eam_cells if cells else lib.orc_eam_brute
    rc = fn(pot.ref, _d(x), N, _d(L), _d(rho), _d(fp), _d(F), _d(en), _i(npairs))
    if rc < 0:
        raise MemoryError("oracle allocation failed")
    out = dict(rho=rho, fp=fp, F=F, e_emb=float(en[0]), e_pair=float(en[1]), extrapolated=bool(rc))
    if want_pairs:
        out["npairs"] = npairs
    return out


def eam_sampled(pot: Potential, x, box, sample):
    """rho, F', forces and neighbour counts of the sampled atoms only (exact, cell-binned)."""
    lib = _load()
    x = _f64(x, (-1, 3))
    L = _f64(box)
    sample = np.ascontiguousarray(sample, dtype=np.int64)
    M = len(sample)
    rho, fp, F = np.empty(M), np.empty(M), np.empty((M, 3))
    npairs = np.empty(M, dtype=np.int64)
    if lib.orc_eam_sampled(pot.ref, _d(x), x.shape[0], _d(L), _i(sample), M, _d(rho), _d(fp), _d(F),
                           _i(npairs)) < 0:
        raise MemoryError("oracle allocation failed")
    return dict(rho=rho, fp=fp, F=F, npairs=npairs)


def neighbours(x, box, rc, i, cells=False):
    lib = _load()
    x = _f64(x, (-1, 3))
    L = _f64(box)
    cap = 4096
    out = np.empty(cap, dtype=np.int64)
    n = lib.orc_neighbours(_d(x), x.shape[0], _d(L), float(rc), int(i), int(bool(cells)), _i(out), cap)
    if n < 0 or n > cap:
        raise RuntimeError("neighbour query failed")
    return np.sort(out[:n])


def kinetic(v, mass):
    lib = _load()
    v = _f64(v, (-1, 3))
    return float(lib.orc_kinetic(_d(v), v.shape[0], float(mass)))


def acc_unit():
    return float(_load().orc_acc_unit())


def run(pot: Potential, x, v, box, mass, nsteps, dt_max, dx_max=0.0, cells=False, F=None):
    """Velocity-Verlet trajectory; returns (x, v, F, log[nsteps, 5]) with
    log columns [dt, E_kin, E_emb, E_pair, max|v| at step start]."""
    lib = _load()
    x = _f64(x, (-1, 3)).copy()
    v = _f64(v, (-1, 3)).copy()
    N = x.shape[0]
    have = F is not None
    F = _f64(F, (-1, 3)).copy() if have else np.zeros((N, 3))
    L = _f64(box)
    log = np.zeros((max(int(nsteps), 1), 5))
    if lib.orc_run(pot.ref, _d(x), _d(v), _d(F), N, _d(L), float(mass), int(nsteps), float(dt_max),
                   float(dx_max), int(bool(cells)), int(have), _d(log)) < 0:
        raise MemoryError("oracle allocation failed")
    return x, v, F, log[: int(nsteps)]


def lattice_id(box_x, box_y, X, Y, Z):
    return int(_load().orc_lattice_id(int(box_x), int(box_y), int(X), int(Y), int(Z)))


def lattice_coords(box_x, box_y, idx):
    X, Y, Z = C.c_int64(), C.c_int64(), C.c_int64()
    _load().orc_lattice_coords(int(box_x), int(box_y), int(idx), C.byref(X), C.byref(Y), C.byref(Z))
    return X.value, Y.value, Z.value


def site_position(a, X, Y, Z):
    p = np.empty(3)
    _load().orc_site_position(float(a), int(X), int(Y), int(Z), _d(p))
    return p


def stencil(a, R, parity):
    """Neighbour offset index (dX, dY, dZ) of all sites strictly within R, by enumeration."""
    lib = _load()
    cap = 4096
    out = np.empty((cap, 3), dtype=np.int64)
    n = lib.orc_stencil(float(a), float(R), int(parity), _i(out), cap)
    return out[:n].copy()


def nearest_site_brute(n_cells, a, x):
    nx, ny, nz = n_cells
    d2 = C.c_double()
    x = _f64(x)
    s = _load().orc_nearest_site_brute(nx, ny, nz, float(a), _d(x), C.byref(d2))
    return int(s), d2.value


def wigner_seitz(n_cells, a, x):
    """Wigner-Seitz defect count: (vacancies, interstitials, per-site occupancy by lattice id)."""
    nx, ny, nz = n_cells
    x = _f64(x, (-1, 3))
    out = np.zeros(2, dtype=np.int64)
    occ = np.zeros(2 * nx * ny * nz, dtype=np.int32)
    lib = _load()
    lib.orc_wigner_seitz.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_double, _dp, C.c_int64,
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    lib.orc_wigner_seitz.restype = C.c_int
    if lib.orc_wigner_seitz(nx, ny, nz, float(a), _d(x), x.shape[0], out.ctypes.data_as(C.POINTER(C.c_int64)),
                            occ.ctypes.data_as(C.POINTER(C.c_int32))) < 0:
        raise MemoryError("oracle allocation failed")
    return int(out[0]), int(out[1]), occ


def hash_site(n_cells, a, x):
    """Nearest site by the hash rule: (lattice id, u = x - site, |u|^2)."""
    nx, ny, nz = n_cells
    x = _f64(x)
    u = np.empty(3)
    u2 = C.c_double()
    s = _load().orc_hash(nx, ny, nz, float(a), _d(x), _d(u), C.byref(u2))
    return int(s), u, u2.value


def place(n_cells, a, delta, x):
    """Fresh placement: per-atom lattice id of its slot, or -1 for clash/run-away atoms."""
    nx, ny, nz = n_cells
    x = _f64(x, (-1, 3))
    slot = np.empty(x.shape[0], dtype=np.int64)
    _load().orc_place(nx, ny, nz, float(a), float(delta), _d(x), x.shape[0], _i(slot))
    return slot


def rehash(n_cells, a, delta, x, slot):
    """Incremental hash update (leave, then return to empty slots by ascending id)."""
    nx, ny, nz = n_cells
    x = _f64(x, (-1, 3))
    slot = np.ascontiguousarray(slot, dtype=np.int64).copy()
    _load().orc_rehash(nx, ny, nz, float(a), float(delta), _d(x), x.shape[0], _i(slot))
    return slot


def num_threads():
    return int(_load().orc_num_threads())
