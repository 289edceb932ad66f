"""ctypes binding of libmisa.so: argument marshalling only, same names as misa.h.

PyTorch supplies device memory (the caller-owned state buffer, device-side
outputs) and the HIP stream; every step of the computation runs in the
library's HIP kernels.  Importing this module fails loudly when libmisa.so
is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmisa.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "misa.h")

MISA_OK, MISA_EINVAL, MISA_ENOMEM, MISA_EHIP, MISA_ESTATE, MISA_EOVERFLOW = 0, -1, -2, -3, -4, -5
MISA_FP64, MISA_FP32 = 0, 1
MISA_HOST, MISA_DEVICE = 0, 1
MISA_FIELD_RHO, MISA_FIELD_FPRIME, MISA_FIELD_FORCE = 0, 1, 2
MISA_EXPORT_STENCIL, MISA_EXPORT_SLOTS, MISA_EXPORT_NEIGHBOURS = 0, 1, 2
MISA_MLP = 2
MISA_PAIRS_GATHER, MISA_PAIRS_HALF = 0, 1
# batch tile shapes (x, y, z cells), in the library's order
MISA_TILE_SHAPES = ((8, 8, 8), (16, 8, 4), (8, 16, 4), (16, 4, 8), (4, 16, 8), (8, 4, 16), (4, 8, 16))
MISA_FN_F, MISA_FN_PHI, MISA_FN_EMB = 0, 1, 2
MISA_MLP_HIDDEN, MISA_MLP_PARAMS, MISA_FM_SLOTS = 32, 1153, 96

_ERRNAMES = {MISA_EINVAL: "MISA_EINVAL", MISA_ENOMEM: "MISA_ENOMEM", MISA_EHIP: "MISA_EHIP",
             MISA_ESTATE: "MISA_ESTATE", MISA_EOVERFLOW: "MISA_EOVERFLOW"}


class MisaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class misa_lattice_desc(C.Structure):
    _fields_ = [("n_cells", C.c_int32 * 3), ("pair_precision", C.c_int32), ("a", C.c_double),
                ("rc", C.c_double), ("delta", C.c_double), ("mass", C.c_double),
                ("runaway_capacity", C.c_int64), ("periodic", C.c_int32 * 3), ("ntypes", C.c_int32)]


class misa_table(C.Structure):
    _fields_ = [("x0", C.c_double), ("dx", C.c_double), ("n", C.c_int32), ("reserved", C.c_int32),
                ("y", C.POINTER(C.c_double))]


class misa_step_stats(C.Structure):
    _fields_ = [("dt", C.c_double), ("dt_next", C.c_double), ("vmax", C.c_double), ("e_kin", C.c_double),
                ("e_emb", C.c_double), ("e_pair", C.c_double), ("time", C.c_double), ("steps", C.c_int64),
                ("n_runaway", C.c_int64), ("range_violations", C.c_int64), ("overflow", C.c_int32),
                ("failed_step", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


MISA_TIMER_NAMES = ("rho", "force", "kick", "runaway", "other")


class misa_timing(C.Structure):
    _fields_ = [("ms", C.c_double * 5), ("launches", C.c_int64 * 5)]


class misa_mlp_net(C.Structure):
    _fields_ = [("x_lo", C.c_double), ("x_hi", C.c_double), ("y_shift", C.c_double), ("y_scale", C.c_double),
                ("params", C.c_float * MISA_MLP_PARAMS), ("reserved", C.c_int32)]


class misa_fit_opts(C.Structure):
    _fields_ = [("iters", C.c_int64), ("batch", C.c_int32), ("quantize", C.c_int32), ("lr", C.c_double),
                ("lr_final", C.c_double), ("lambda_", C.c_double), ("seed", C.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950). There is no CPU fallback.")
    lib = C.CDLL(LIB_PATH)
    vp, i64, dp = C.c_void_p, C.c_int64, C.POINTER(C.c_double)
    sig = {
        "misa_create_lattice": ([C.POINTER(misa_lattice_desc), vp, C.POINTER(vp)], C.c_int),
        "misa_destroy_lattice": ([vp], C.c_int),
        "misa_last_error": ([vp], C.c_char_p),
        "misa_state_bytes": ([vp, C.POINTER(i64)], C.c_int),
        "misa_bind_state": ([vp, vp, i64], C.c_int),
        "misa_set_potential_tables": ([vp, C.POINTER(misa_table), C.POINTER(misa_table), C.POINTER(misa_table)],
                                      C.c_int),
        "misa_set_state": ([vp, vp, vp, i64, C.c_int], C.c_int),
        "misa_set_state_noalloc": ([vp, vp, vp, i64], C.c_int),
        "misa_set_state_ids": ([vp, vp, vp, vp, i64], C.c_int),
        "misa_checkpoint_bytes": ([vp, C.POINTER(i64)], C.c_int),
        "misa_save_checkpoint": ([vp, vp, i64], C.c_int),
        "misa_load_checkpoint": ([vp, vp, i64], C.c_int),
        "misa_get_state": ([vp, vp, vp, C.c_int], C.c_int),
        "misa_atom_count": ([vp, C.POINTER(i64)], C.c_int),
        "misa_compute_rho": ([vp], C.c_int),
        "misa_compute_force": ([vp, vp], C.c_int),
        "misa_step": ([vp, i64, C.c_double, C.c_double, C.POINTER(misa_step_stats)], C.c_int),
        "misa_get_atom_field": ([vp, C.c_int, vp, C.c_int], C.c_int),
        "misa_set_timing": ([vp, C.c_int], C.c_int),
        "misa_set_graph": ([vp, C.c_int], C.c_int),
        "misa_get_timing": ([vp, C.POINTER(misa_timing)], C.c_int),
        "misa_debug_export": ([vp, C.c_int, C.POINTER(i64), i64], i64),
        "misa_defects": ([vp, C.POINTER(i64)], C.c_int),
        "misa_set_pair_schedule": ([vp, C.c_int], C.c_int),
        "misa_set_mlp": ([vp, C.c_int, C.POINTER(misa_mlp_net)], C.c_int),
        "misa_table_eval": ([vp, C.c_int, vp, i64, vp, vp], C.c_int),
        "misa_mlp_trainer_create": ([vp, C.POINTER(vp)], C.c_int),
        "misa_mlp_trainer_destroy": ([vp], C.c_int),
        "misa_mlp_last_error": ([vp], C.c_char_p),
        "misa_mlp_trainer_set": ([vp, C.c_int, C.POINTER(misa_mlp_net)], C.c_int),
        "misa_mlp_trainer_get": ([vp, C.c_int, C.POINTER(misa_mlp_net), vp], C.c_int),
        "misa_mlp_eval": ([vp, C.c_int, C.c_int, vp, i64, vp, vp], C.c_int),
        "misa_mlp_grad": ([vp, C.c_int, vp, vp, vp, i64, vp], C.c_int),
        "misa_mlp_adam": ([vp, C.c_int, vp, C.c_double], C.c_int),
        "misa_mlp_fit": ([vp, C.c_int, vp, vp, vp, i64, C.POINTER(misa_fit_opts), dp], C.c_int),
        "misa_mlp_fit_many": ([vp, C.c_int, vp, vp, vp, vp, vp, C.POINTER(misa_fit_opts), vp], C.c_int),
        "misa_mlp_collect": ([vp, vp, i64, vp, vp, vp, vp, vp], C.c_int),
        "misa_mlp_force_match": ([vp, vp, vp, vp, vp, vp, i64, C.POINTER(misa_fit_opts), dp], C.c_int),
        "misa_batch_create": ([C.POINTER(misa_lattice_desc), C.c_int32, vp, C.POINTER(vp)], C.c_int),
        "misa_batch_destroy": ([vp], C.c_int),
        "misa_batch_last_error": ([vp], C.c_char_p),
        "misa_batch_box": ([vp, C.c_int32, C.POINTER(vp)], C.c_int),
        "misa_batch_set_potential_tables": ([vp, C.POINTER(misa_table), C.POINTER(misa_table),
                                             C.POINTER(misa_table)], C.c_int),
        "misa_batch_step": ([vp, i64, C.c_double, C.c_double, C.POINTER(misa_step_stats)], C.c_int),
        "misa_batch_set_tile_shape": ([vp, C.c_int32, C.c_int32], C.c_int),
        "misa_batch_set_graph": ([vp, C.c_int], C.c_int),
        "misa_batch_get_tile_shape": ([vp, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
        "misa_batch_autotune": ([vp, i64, C.c_double, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                 C.POINTER(i64)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def declared_functions(header: str = HEADER):
    """Names of the entry points misa.h declares."""
    text = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char \*)\s*\*?\s*(misa_\w+)\s*\(", text, re.M)))


def _check(code, h=None):
    if code < 0:
        msg = lib.misa_last_error(h)
        raise MisaError(code, msg.decode() if msg else "")
    return code


def _ptr(a):
    """Data pointer of a torch tensor or a numpy array, and its memory kind."""
    if a is None:
        return None, MISA_HOST
    if hasattr(a, "data_ptr"):  # torch.Tensor
        return C.c_void_p(a.data_ptr()), (MISA_DEVICE if a.is_cuda else MISA_HOST)
    return C.c_void_p(a.ctypes.data), MISA_HOST


# ---------------------------------------------------------------------------
# entry points, same names as the C ABI

def misa_create_lattice(n_cells, a, rc, delta, mass, pair_precision=MISA_FP64, runaway_capacity=0,
                        hip_stream=None, periodic=(1, 1, 1), ntypes=1):
    d = misa_lattice_desc()
    d.n_cells[:] = [int(k) for k in n_cells]
    d.pair_precision, d.a, d.rc, d.delta, d.mass = int(pair_precision), float(a), float(rc), float(delta), float(mass)
    d.runaway_capacity = int(runaway_capacity)
    d.periodic[:] = [int(k) for k in periodic]
    d.ntypes = int(ntypes)
    h = C.c_void_p()
    _check(lib.misa_create_lattice(C.byref(d), C.c_void_p(hip_stream or 0), C.byref(h)))
    return h


def misa_destroy_lattice(h):
    return _check(lib.misa_destroy_lattice(h))


def misa_last_error(h):
    return lib.misa_last_error(h).decode()


def misa_state_bytes(h):
    b = C.c_int64()
    _check(lib.misa_state_bytes(h, C.byref(b)), h)
    return b.value


def misa_bind_state(h, device_ptr, nbytes):
    return _check(lib.misa_bind_state(h, C.c_void_p(device_ptr), int(nbytes)), h)


def _table(x0, dx, y):
    y = np.ascontiguousarray(y, dtype=np.float64)
    t = misa_table(float(x0), float(dx), len(y), 0, y.ctypes.data_as(C.POINTER(C.c_double)))
    return t, y


def misa_set_potential_tables(h, f, phi, emb):
    """f, phi, emb: (x0, dx, y) sample tuples."""
    tf, kf = _table(*f)
    tp, kp = _table(*phi)
    te, ke = _table(*emb)
    return _check(lib.misa_set_potential_tables(h, C.byref(tf), C.byref(tp), C.byref(te)), h)


def misa_set_state(h, x, v):
    """x, v: (N, 3) float64 numpy arrays or CUDA tensors (same kind for both)."""
    if not hasattr(x, "data_ptr"):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    n = x.shape[0]
    px, where = _ptr(x)
    pv, where_v = _ptr(v)
    if where != where_v:
        raise ValueError("x and v must live in the same memory")
    return _check(lib.misa_set_state(h, px, pv, n, where), h)


def misa_set_state_ids(h, x, v, ids):
    """x, v: (N, 3) float64 host arrays whose row i belongs to atom ids[i]; ids: a
    permutation of 0 .. N - 1 (int64)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    ids = np.ascontiguousarray(ids, dtype=np.int64).reshape(-1)
    n = x.shape[0]
    if v.shape[0] != n or ids.shape[0] != n:
        raise ValueError("x, v and ids must have the same number of rows")
    vp = C.c_void_p
    return _check(lib.misa_set_state_ids(h, x.ctypes.data_as(vp), v.ctypes.data_as(vp),
                                         ids.ctypes.data_as(vp), n), h)


def misa_checkpoint_bytes(h):
    """Size in bytes of the handle's checkpoint."""
    n = C.c_int64()
    _check(lib.misa_checkpoint_bytes(h, C.byref(n)), h)
    return n.value


def misa_save_checkpoint(h):
    """The handle's whole state as a numpy uint8 array (host memory)."""
    n = misa_checkpoint_bytes(h)
    buf = np.empty(n, dtype=np.uint8)
    _check(lib.misa_save_checkpoint(h, C.c_void_p(buf.ctypes.data), n), h)
    return buf


def misa_load_checkpoint(h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    return _check(lib.misa_load_checkpoint(h, C.c_void_p(buf.ctypes.data), buf.size), h)


MISA_NOALLOC_MAX_ATOMS = 4194304


def misa_set_state_noalloc(h, x, v):
    """x, v: (N, 3) float64 CUDA tensors on the handle's GPU; no device allocation."""
    if not (hasattr(x, "data_ptr") and x.is_cuda and hasattr(v, "data_ptr") and v.is_cuda):
        raise ValueError("misa_set_state_noalloc takes device tensors")
    return _check(lib.misa_set_state_noalloc(h, C.c_void_p(x.data_ptr()), C.c_void_p(v.data_ptr()), x.shape[0]), h)


def misa_atom_count(h):
    n = C.c_int64()
    _check(lib.misa_atom_count(h, C.byref(n)), h)
    return n.value


def misa_get_state(h, x=None, v=None):
    """Fill x / v ((N, 3) float64 numpy arrays or CUDA tensors); allocates numpy arrays if both are None."""
    if x is None and v is None:
        n = misa_atom_count(h)
        x, v = np.empty((n, 3)), np.empty((n, 3))
    px, wx = _ptr(x)
    pv, wv = _ptr(v)
    where = wx if x is not None else wv
    _check(lib.misa_get_state(h, px, pv, where), h)
    return x, v


def misa_compute_rho(h):
    return _check(lib.misa_compute_rho(h), h)


def misa_compute_force(h, energies_dev=None):
    p, _ = _ptr(energies_dev)
    return _check(lib.misa_compute_force(h, p), h)


def misa_step(h, nsteps, dt_max, dx_max=0.0, want_stats=True):
    st = misa_step_stats()
    code = lib.misa_step(h, int(nsteps), float(dt_max), float(dx_max), C.byref(st) if want_stats else None)
    if code == MISA_EOVERFLOW:  # the statistics of the state the call stopped at go with the error
        err = MisaError(code, misa_last_error(h))
        err.stats = st.as_dict() if want_stats else None
        raise err
    _check(code, h)
    return st.as_dict() if want_stats else None


def misa_set_graph(h, enable=True):
    """Replay a captured HIP graph of one step inside misa_step."""
    return _check(lib.misa_set_graph(h, int(bool(enable))), h)


def misa_set_timing(h, enable=True):
    return _check(lib.misa_set_timing(h, int(bool(enable))), h)


def misa_get_timing(h):
    """{class: (summed ms, launch groups)} since misa_set_timing."""
    t = misa_timing()
    _check(lib.misa_get_timing(h, C.byref(t)), h)
    return {n: (t.ms[k], t.launches[k]) for k, n in enumerate(MISA_TIMER_NAMES)}


def misa_get_atom_field(h, field, out=None):
    n = misa_atom_count(h) * (3 if field == MISA_FIELD_FORCE else 1)
    if out is None:
        out = np.empty(n)
    p, where = _ptr(out)
    _check(lib.misa_get_atom_field(h, int(field), p, where), h)
    return out.reshape(-1, 3) if (field == MISA_FIELD_FORCE and not hasattr(out, "data_ptr")) else out


def misa_debug_export(h, what):
    if what == MISA_EXPORT_STENCIL:
        k = _check(lib.misa_debug_export(h, what, None, 0), h)
        out = np.empty(2 * k * 3, dtype=np.int64)
        _check(lib.misa_debug_export(h, what, out.ctypes.data_as(C.POINTER(C.c_int64)), out.size), h)
        return out.reshape(2, k, 3)
    n = misa_atom_count(h)
    out = np.empty(max(n, 1), dtype=np.int64)
    _check(lib.misa_debug_export(h, what, out.ctypes.data_as(C.POINTER(C.c_int64)), out.size), h)
    return out[:n]


def misa_set_pair_schedule(h, schedule):
    """MISA_PAIRS_GATHER (each pair from both ends) or MISA_PAIRS_HALF (each pair once)."""
    return _check(lib.misa_set_pair_schedule(h, int(schedule)), h)


def misa_defects(h):
    """Wigner-Seitz count: dict(vacancies, interstitials, runaway, empty_slots)."""
    c = (C.c_int64 * 4)()
    _check(lib.misa_defects(h, c), h)
    return {"vacancies": c[0], "interstitials": c[1], "runaway": c[2], "empty_slots": c[3]}


# ---------------------------------------------------------------------------
# learned form (surrogate networks)

def _net(net):
    """dict(x_lo, x_hi, y_shift, y_scale, params[MISA_MLP_PARAMS]) -> misa_mlp_net."""
    n = misa_mlp_net()
    n.x_lo, n.x_hi = float(net["x_lo"]), float(net["x_hi"])
    n.y_shift, n.y_scale = float(net["y_shift"]), float(net["y_scale"])
    prm = np.ascontiguousarray(net["params"], dtype=np.float32)
    if prm.shape != (MISA_MLP_PARAMS,):
        raise ValueError(f"params must hold {MISA_MLP_PARAMS} values")
    C.memmove(n.params, prm.ctypes.data, prm.nbytes)
    return n


def _net_dict(n):
    return {"x_lo": n.x_lo, "x_hi": n.x_hi, "y_shift": n.y_shift, "y_scale": n.y_scale,
            "params": np.ctypeslib.as_array(n.params).copy()}


def _opts(o):
    s = misa_fit_opts()
    s.iters, s.batch, s.quantize = int(o["iters"]), int(o["batch"]), int(o.get("quantize", 1))
    s.lr, s.lr_final, s.lambda_ = float(o["lr"]), float(o.get("lr_final", 0.0)), float(o.get("lambda", 1.0))
    s.seed = int(o.get("seed", 0))
    return s


def _dev(a):
    """Device pointer of a CUDA tensor (the trainer and table calls take device arrays only)."""
    if a is None:
        return None
    if not (hasattr(a, "data_ptr") and a.is_cuda):
        raise ValueError("device (CUDA) tensor expected")
    return C.c_void_p(a.data_ptr())


def _tcheck(code, t=None):
    if code < 0:
        msg = lib.misa_mlp_last_error(t)
        raise MisaError(code, msg.decode() if msg else "")
    return code


def misa_set_mlp(h, fn, net):
    n = _net(net)
    return _check(lib.misa_set_mlp(h, int(fn), C.byref(n)), h)


def misa_table_eval(h, fn, x, y, dy):
    return _check(lib.misa_table_eval(h, int(fn), _dev(x), x.numel(), _dev(y), _dev(dy)), h)


def misa_mlp_trainer_create(hip_stream=None):
    t = C.c_void_p()
    _tcheck(lib.misa_mlp_trainer_create(C.c_void_p(hip_stream or 0), C.byref(t)))
    return t


def misa_mlp_trainer_destroy(t):
    return _tcheck(lib.misa_mlp_trainer_destroy(t))


def misa_mlp_last_error(t):
    return lib.misa_mlp_last_error(t).decode()


def misa_mlp_trainer_set(t, fn, net):
    n = _net(net)
    return _tcheck(lib.misa_mlp_trainer_set(t, int(fn), C.byref(n)), t)


def misa_mlp_trainer_get(t, fn):
    """(network dict with bfloat16-rounded params, float32 master weights)."""
    n = misa_mlp_net()
    master = np.empty(MISA_MLP_PARAMS, dtype=np.float32)
    _tcheck(lib.misa_mlp_trainer_get(t, int(fn), C.byref(n), C.c_void_p(master.ctypes.data)), t)
    return _net_dict(n), master


def misa_mlp_eval(t, fn, path, x, y, dy):
    return _tcheck(lib.misa_mlp_eval(t, int(fn), int(path), _dev(x), x.numel(), _dev(y), _dev(dy)), t)


def misa_mlp_grad(t, fn, x, c_val, c_der, grad):
    return _tcheck(lib.misa_mlp_grad(t, int(fn), _dev(x), _dev(c_val), _dev(c_der), x.numel(), _dev(grad)), t)


def misa_mlp_adam(t, fn, grad, lr):
    return _tcheck(lib.misa_mlp_adam(t, int(fn), _dev(grad), float(lr)), t)


def misa_mlp_fit(t, fn, x, y, dy, opts):
    loss = C.c_double()
    o = _opts(opts)
    _tcheck(lib.misa_mlp_fit(t, int(fn), _dev(x), _dev(y), _dev(dy), x.numel(), C.byref(o), C.byref(loss)), t)
    return loss.value


def misa_mlp_fit_many(t, fns, xs, ys, dys, opts):
    """Fit networks fns together; xs, ys, dys: lists of CUDA float64 tensors. Returns the losses."""
    k = len(fns)
    f = (C.c_int * k)(*[int(v) for v in fns])
    ptr = lambda ts: (C.c_void_p * k)(*[_dev(v) for v in ts])
    n = (C.c_int64 * k)(*[int(v.numel()) for v in xs])
    loss = (C.c_double * k)()
    o = _opts(opts)
    _tcheck(lib.misa_mlp_fit_many(t, k, f, ptr(xs), ptr(ys), ptr(dys), n, C.byref(o), loss), t)
    return list(loss)


def misa_mlp_collect(h, sites, r, dhat, fp_j, fp_i, f_ref):
    """sites: host int64 lattice ids; outputs: CUDA float64 tensors of the documented shapes."""
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    return _check(lib.misa_mlp_collect(h, C.c_void_p(sites.ctypes.data), sites.size, _dev(r), _dev(dhat),
                                       _dev(fp_j), _dev(fp_i), _dev(f_ref)), h)


def misa_mlp_force_match(t, r, dhat, fp_j, fp_i, f_ref, opts):
    loss = C.c_double()
    o = _opts(opts)
    n_env = fp_i.numel()
    _tcheck(lib.misa_mlp_force_match(t, _dev(r), _dev(dhat), _dev(fp_j), _dev(fp_i), _dev(f_ref), n_env,
                                     C.byref(o), C.byref(loss)), t)
    return loss.value


# ---------------------------------------------------------------------------
# batched replicas

def _bcheck(code, b=None):
    if code < 0:
        msg = lib.misa_batch_last_error(b)
        raise MisaError(code, msg.decode() if msg else "")
    return code


def misa_batch_create(boxes, a, rc, delta, mass, runaway_capacity=0, hip_stream=None):
    """boxes: list of n_cells triples; every box uses MISA_FP32 and the same a, rc, delta, mass;
    runaway_capacity: one value for every box or one per box."""
    n = len(boxes)
    caps = list(runaway_capacity) if hasattr(runaway_capacity, "__len__") else [runaway_capacity] * n
    descs = (misa_lattice_desc * n)()
    for k, nc in enumerate(boxes):
        d = descs[k]
        d.n_cells[:] = [int(c) for c in nc]
        d.pair_precision, d.a, d.rc, d.delta, d.mass = MISA_FP32, float(a), float(rc), float(delta), float(mass)
        d.runaway_capacity = int(caps[k])
        d.periodic[:] = [1, 1, 1]
        d.ntypes = 1
    b = C.c_void_p()
    _bcheck(lib.misa_batch_create(descs, n, C.c_void_p(hip_stream or 0), C.byref(b)))
    return b


def misa_batch_destroy(b):
    return _bcheck(lib.misa_batch_destroy(b))


def misa_batch_last_error(b):
    return lib.misa_batch_last_error(b).decode()


def misa_batch_box(b, k):
    h = C.c_void_p()
    _bcheck(lib.misa_batch_box(b, int(k), C.byref(h)), b)
    return h


def misa_batch_set_potential_tables(b, f, phi, emb):
    tf, kf = _table(*f)
    tp, kp = _table(*phi)
    te, ke = _table(*emb)
    return _bcheck(lib.misa_batch_set_potential_tables(b, C.byref(tf), C.byref(tp), C.byref(te)), b)


def misa_batch_step(b, n_boxes, nsteps, dt_max, dx_max=0.0, want_stats=True):
    st = (misa_step_stats * n_boxes)()
    code = lib.misa_batch_step(b, int(nsteps), float(dt_max), float(dx_max), st if want_stats else None)
    if code == MISA_EOVERFLOW:  # the statistics of every box go with the error
        err = MisaError(code, misa_batch_last_error(b))
        err.stats = [st[k].as_dict() for k in range(n_boxes)] if want_stats else None
        raise err
    _bcheck(code, b)
    return [st[k].as_dict() for k in range(n_boxes)] if want_stats else None


def misa_batch_set_tile_shape(b, k, shape):
    """shape: index into MISA_TILE_SHAPES."""
    return _bcheck(lib.misa_batch_set_tile_shape(b, int(k), int(shape)), b)


def misa_batch_get_tile_shape(b, k):
    s = C.c_int32()
    _bcheck(lib.misa_batch_get_tile_shape(b, int(k), C.byref(s)), b)
    return s.value


def misa_batch_autotune(b, probe_steps, dt_max, dx_max=0.0):
    """Time both tile policies and keep the faster: dict(policy, ms_per_step, steps_done)."""
    pol = C.c_int32()
    ms = (C.c_double * 2)()
    done = C.c_int64()
    _bcheck(lib.misa_batch_autotune(b, int(probe_steps), float(dt_max), float(dx_max), C.byref(pol), ms,
                                    C.byref(done)), b)
    return {"policy": pol.value, "ms_per_step": [ms[0], ms[1]], "steps_done": done.value}


def misa_batch_set_graph(b, enable=True):
    """Replay a captured HIP graph of one batched step inside misa_batch_step."""
    return _bcheck(lib.misa_batch_set_graph(b, int(bool(enable))), b)
