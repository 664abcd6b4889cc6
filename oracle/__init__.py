"""FP64 CPU oracle for the quantized MLS-MPM substep (Liu et al. 2022).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
product path (``paper_2207_04658_amd``) never imports, links or calls it, and
it imports nothing from there: the two share no code.

This module is argument marshalling over ``liboracle.so`` (plain C, built by
``oracle/build.py``).  Schemes and parameters are the plain dictionaries of
``workloads`` (input descriptions only).

Arrays are component-major structure-of-arrays: component ``c`` of particle
``p`` is ``a[c, p]``; packed words are word-major, ``words[k, p]``.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

FIELDS = {"x": 0, "v": 1, "C": 2, "F": 3, "J": 4}
MATERIALS = {"elastic": 0, "fluid": 1}


def slot3_name(scheme: dict) -> str:
    """"F" (elastic) or "J" (fluid): the field in the fourth state slot."""
    return "J" if any(f["field"] == "J" for f in scheme["fields"]) else "F"


def nc3(scheme: dict) -> int:
    return 1 if slot3_name(scheme) == "J" else scheme["dim"] ** 2
KINDS = {"fixed": 0, "shared_exp": 1, "raw_f32": 2}


class _Field(ct.Structure):
    _fields_ = [("field", ct.c_int32), ("kind", ct.c_int32), ("bits", ct.c_int32),
                ("exp_bits", ct.c_int32), ("dither", ct.c_int32), ("rel_identity", ct.c_int32),
                ("lo", ct.c_double), ("hi", ct.c_double)]


class _Scheme(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("n_fields", ct.c_int32), ("f", _Field * 4),
                ("seed", ct.c_uint64)]


class _Params(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("grid_res", ct.c_int32), ("bound_cells", ct.c_int32),
                ("sort_every", ct.c_int32), ("dt", ct.c_double), ("gravity", ct.c_double * 3),
                ("E", ct.c_double), ("nu", ct.c_double), ("rho", ct.c_double),
                ("p_vol", ct.c_double), ("material", ct.c_int32), ("pad", ct.c_int32)]


class _Stat(ct.Structure):
    _fields_ = [("sat", ct.c_int64), ("nan", ct.c_int64), ("up", ct.c_int64), ("down", ct.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ct.CDLL(LIB_PATH)
        P = ct.c_void_p
        L.orc_layout.argtypes = [ct.POINTER(_Scheme), P, P, P, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_encode.argtypes = [ct.POINTER(_Scheme), ct.c_int64, P, P, P, P, ct.c_uint32,
                                 ct.c_uint32, P, P]
        L.orc_encode_f64.argtypes = L.orc_encode.argtypes
        L.orc_decode.argtypes = [ct.POINTER(_Scheme), ct.c_int64, P, P, P, P, P]
        L.orc_validate.argtypes = [ct.POINTER(_Scheme)]
        L.orc_polar.argtypes = [ct.c_int, P, P]
        L.orc_kirchhoff.argtypes = [ct.c_int, P, ct.c_double, ct.c_double, P]
        L.orc_p2g.argtypes = [ct.POINTER(_Params), ct.c_int64, P, P, P, P, P, P]
        L.orc_grid_update.argtypes = [ct.POINTER(_Params), P, P]
        L.orc_g2p.argtypes = [ct.POINTER(_Params), ct.c_int64, P, P, P, P, P, P, P]
        L.orc_sort_order.argtypes = [ct.POINTER(_Params), ct.c_int64, P, P]
        L.orc_sim_new.argtypes = [ct.POINTER(_Scheme), ct.POINTER(_Params), ct.c_int64, P]
        L.orc_sim_new.restype = ct.c_void_p
        L.orc_sim_step.argtypes = [P, ct.c_int32]
        L.orc_sim_words.argtypes = [P, P]
        L.orc_sim_ids.argtypes = [P, P]
        L.orc_sim_stats.argtypes = [P, P]
        L.orc_sim_step_count.argtypes = [P]
        L.orc_sim_step_count.restype = ct.c_int64
        L.orc_sim_free.argtypes = [P]
        L.orc_step_exact.argtypes = [ct.POINTER(_Params), ct.c_int64, P, P]
        L.orc_step_vjp.argtypes = [ct.POINTER(_Params), ct.c_int64, P, P, P]
        L.orc_objective.argtypes = [ct.POINTER(_Params), ct.c_int64, P, ct.c_int, ct.c_int,
                                    ct.POINTER(ct.c_double), P]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def make_scheme(scheme: dict) -> _Scheme:
    s = _Scheme()
    s.dim = scheme["dim"]
    s.n_fields = len(scheme["fields"])
    for i, f in enumerate(scheme["fields"]):
        s.f[i].field = FIELDS[f["field"]]
        s.f[i].kind = KINDS[f["kind"]]
        s.f[i].bits = int(f.get("bits", 32))
        s.f[i].exp_bits = int(f.get("exp_bits", 0))
        s.f[i].dither = int(bool(f.get("dither", False)))
        s.f[i].rel_identity = int(bool(f.get("rel_identity", False)))
        s.f[i].lo = float(f.get("lo", 0.0))
        s.f[i].hi = float(f.get("hi", 1.0))
    s.seed = int(scheme.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    return s


def make_params(params: dict) -> _Params:
    p = _Params()
    p.dim = params["dim"]
    p.grid_res = params["grid_res"]
    p.bound_cells = params.get("bound_cells", 3)
    p.sort_every = params.get("sort_every", 0)
    p.dt = params["dt"]
    g = list(params.get("gravity", [0.0, -9.8, 0.0])) + [0.0, 0.0, 0.0]
    for a in range(3):
        p.gravity[a] = g[a]
    p.E = params["E"]
    p.nu = params["nu"]
    p.rho = params["rho"]
    p.p_vol = params["p_vol"]
    p.material = MATERIALS[params.get("material", "elastic")]
    return p


def validate(scheme: dict) -> bool:
    return lib().orc_validate(ct.byref(make_scheme(scheme))) == 0


def layout(scheme: dict):
    """Returns (component bit offsets [4,9], field offsets [4], total bits, W)."""
    comp = np.full(36, -1, dtype=np.int32)
    fo = np.full(4, -1, dtype=np.int32)
    tb = ct.c_int32()
    W = ct.c_int32()
    rc = lib().orc_layout(ct.byref(make_scheme(scheme)), _ptr(comp), _ptr(fo), ct.byref(tb), ct.byref(W))
    if rc:
        raise ValueError("invalid scheme")
    return comp.reshape(4, 9), fo, tb.value, W.value


def philox(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def stats_dict(st, scheme=None):
    names = ["x", "v", "C", slot3_name(scheme) if scheme else "F"]
    return {names[i]: {"sat": st[i].sat, "nan": st[i].nan, "up": st[i].up, "down": st[i].down}
            for i in range(4)}


def encode(scheme: dict, x, v, C, F, step=0, tag=2):
    """Encode float32 (or float64) SoA arrays into packed words [W, n]."""
    dim = scheme["dim"]
    f64 = np.asarray(x).dtype == np.float64
    dt = np.float64 if f64 else np.float32
    x = np.ascontiguousarray(x, dtype=dt).reshape(dim, -1)
    n = x.shape[1]
    v = np.ascontiguousarray(v, dtype=dt).reshape(dim, n)
    C = np.ascontiguousarray(C, dtype=dt).reshape(dim * dim, n)
    F = np.ascontiguousarray(F, dtype=dt).reshape(nc3(scheme), n)
    _, _, _, W = layout(scheme)
    words = np.zeros((W, n), dtype=np.uint32)
    st = (_Stat * 4)()
    fn = lib().orc_encode_f64 if f64 else lib().orc_encode
    rc = fn(ct.byref(make_scheme(scheme)), n, _ptr(x), _ptr(v), _ptr(C), _ptr(F), step, tag,
            _ptr(words), ct.cast(st, ct.c_void_p))
    if rc:
        raise ValueError("invalid scheme")
    return words, stats_dict(st, scheme)


def decode(scheme: dict, words):
    dim = scheme["dim"]
    words = np.ascontiguousarray(words, dtype=np.uint32)
    n = words.shape[1]
    x = np.zeros((dim, n)); v = np.zeros((dim, n))
    C = np.zeros((dim * dim, n)); F = np.zeros((nc3(scheme), n))
    rc = lib().orc_decode(ct.byref(make_scheme(scheme)), n, _ptr(words), _ptr(x), _ptr(v), _ptr(C), _ptr(F))
    if rc:
        raise ValueError("invalid scheme")
    return x, v, C, F


def polar(F):
    F = np.ascontiguousarray(F, dtype=np.float64)
    dim = F.shape[0]
    R = np.zeros_like(F)
    lib().orc_polar(dim, _ptr(F), _ptr(R))
    return R


def kirchhoff(F, mu, la):
    F = np.ascontiguousarray(F, dtype=np.float64)
    dim = F.shape[0]
    tau = np.zeros_like(F)
    lib().orc_kirchhoff(dim, _ptr(F), mu, la, _ptr(tau))
    return tau


def _nodes(params):
    return params["grid_res"] ** params["dim"]


def _nc3p(params):
    return 1 if params.get("material", "elastic") == "fluid" else params["dim"] ** 2


def p2g(params: dict, x, v, C, F):
    dim = params["dim"]
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(dim, -1)
    n = x.shape[1]
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(dim, n)
    C = np.ascontiguousarray(C, dtype=np.float64).reshape(dim * dim, n)
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(_nc3p(params), n)
    gm = np.zeros(_nodes(params))
    gmom = np.zeros((dim, _nodes(params)))
    lib().orc_p2g(ct.byref(make_params(params)), n, _ptr(x), _ptr(v), _ptr(C), _ptr(F), _ptr(gm), _ptr(gmom))
    return gm, gmom


def grid_update(params: dict, gm, gmom):
    gm = np.ascontiguousarray(gm, dtype=np.float64).copy()
    gv = np.ascontiguousarray(gmom, dtype=np.float64).copy()
    lib().orc_grid_update(ct.byref(make_params(params)), _ptr(gm), _ptr(gv))
    return gv


def g2p(params: dict, x, F, grid_v):
    dim = params["dim"]
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(dim, -1)
    n = x.shape[1]
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(_nc3p(params), n)
    gv = np.ascontiguousarray(grid_v, dtype=np.float64).reshape(dim, -1)
    x1 = np.zeros((dim, n)); v1 = np.zeros((dim, n))
    C1 = np.zeros((dim * dim, n)); F1 = np.zeros((_nc3p(params), n))
    lib().orc_g2p(ct.byref(make_params(params)), n, _ptr(x), _ptr(F), _ptr(gv), _ptr(x1), _ptr(v1), _ptr(C1), _ptr(F1))
    return x1, v1, C1, F1


def sort_order(params: dict, x):
    dim = params["dim"]
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(dim, -1)
    order = np.zeros(x.shape[1], dtype=np.int64)
    lib().orc_sort_order(ct.byref(make_params(params)), x.shape[1], _ptr(x), _ptr(order))
    return order


class Sim:
    """The oracle simulation: packed words in, packed words out, one substep at a time."""

    def __init__(self, scheme: dict, params: dict, words):
        self.scheme = scheme
        self._s = make_scheme(scheme)
        self._p = make_params(params)
        self.words0 = np.ascontiguousarray(words, dtype=np.uint32)
        self.W, self.n = self.words0.shape
        self._h = lib().orc_sim_new(ct.byref(self._s), ct.byref(self._p), self.n, _ptr(self.words0))
        if not self._h:
            raise ValueError("invalid scheme or params")

    def step(self, nsteps=1):
        if lib().orc_sim_step(self._h, nsteps):
            raise MemoryError("oracle step failed")

    def words(self):
        out = np.zeros((self.W, self.n), dtype=np.uint32)
        lib().orc_sim_words(self._h, _ptr(out))
        return out

    def ids(self):
        out = np.zeros(self.n, dtype=np.int64)
        lib().orc_sim_ids(self._h, _ptr(out))
        return out

    def stats(self):
        st = (_Stat * 4)()
        lib().orc_sim_stats(self._h, ct.cast(st, ct.c_void_p))
        return stats_dict(st, self.scheme)

    @property
    def step_count(self):
        return lib().orc_sim_step_count(self._h)

    def close(self):
        if self._h:
            lib().orc_sim_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ adjoint
# A "state" here is one float64 array of shape [2d + 2d^2, n]: rows x, v, C, F.

def pack_state(x, v, C, F):
    return np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64) for a in (x, v, C, F)], axis=0))


def field_rows(dim, material="elastic"):
    """Row ranges of x, v, C, F (elastic) or J (fluid) in a packed state."""
    d2 = dim * dim
    rows = {"x": (0, dim), "v": (dim, 2 * dim), "C": (2 * dim, 2 * dim + d2)}
    if material == "fluid":
        rows["J"] = (2 * dim + d2, 2 * dim + d2 + 1)
    else:
        rows["F"] = (2 * dim + d2, 2 * dim + 2 * d2)
    return rows


def step_exact(params: dict, state):
    st = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros_like(st)
    if lib().orc_step_exact(ct.byref(make_params(params)), st.shape[1], _ptr(st), _ptr(out)):
        raise MemoryError("oracle step failed")
    return out


def step_vjp(params: dict, state, lam_out):
    st = np.ascontiguousarray(state, dtype=np.float64)
    lo = np.ascontiguousarray(lam_out, dtype=np.float64)
    li = np.zeros_like(st)
    if lib().orc_step_vjp(ct.byref(make_params(params)), st.shape[1], _ptr(st), _ptr(lo), _ptr(li)):
        raise MemoryError("oracle vjp failed")
    return li


OBJECTIVES = {"com": 0, "ke": 1}


def objective(params: dict, state, kind="com", axis=1):
    st = np.ascontiguousarray(state, dtype=np.float64)
    lam = np.zeros_like(st)
    z = ct.c_double()
    lib().orc_objective(ct.byref(make_params(params)), st.shape[1], _ptr(st), OBJECTIVES[kind], axis,
                        ct.byref(z), _ptr(lam))
    return z.value, lam


def adjoint_full(params: dict, states, kind="com", axis=1):
    """Backpropagation through a recorded trajectory (Sec. 6, Eqs. 12-13).

    states[t] is the stored state the substep t -> t+1 started from
    (t = 0..T), all with the same particle order.  Returns z, and per field
    G = sum over t = 0..T, particles and components of d z / d e (the
    sensitivity to an additive error stored at step t, the adjoint of the
    stored state), g = the sum of its squares (the accumulated squared
    gradient of Eq. 8), A = the sum of its absolute values, and lambda_0."""
    dim = params["dim"]
    rows = field_rows(dim, params.get("material", "elastic"))
    T = len(states) - 1
    z, lam = objective(params, states[T], kind, axis)
    G = {f: 0.0 for f in rows}
    g = {f: 0.0 for f in rows}
    A = {f: 0.0 for f in rows}
    for t in range(T, -1, -1):
        for f, (a, b) in rows.items():
            G[f] += float(lam[a:b].sum())
            g[f] += float((lam[a:b] ** 2).sum())
            A[f] += float(np.abs(lam[a:b]).sum())
        if t > 0:
            lam = step_vjp(params, states[t - 1], lam)
    return z, G, g, A, lam


def adjoint(params: dict, states, kind="com", axis=1):
    """z, G and g of adjoint_full."""
    z, G, g, _, _ = adjoint_full(params, states, kind, axis)
    return z, G, g
