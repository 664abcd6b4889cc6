"""Quantized MLS-MPM substep on AMD MI355X -- Python binding of libmpmq.so.

Argument marshalling only: every step of the simulation runs in the HIP
kernels of ``libmpmq.so`` behind the C ABI of ``include/mpmq.h``.  PyTorch
provides device memory and the HIP stream.  There is no CPU fallback: if the
library or a GPU is missing, loading fails with an error.

Schemes and parameters are plain dictionaries (see ``workloads``):
  scheme = {"dim": 3, "seed": 0, "fields": [
      {"field": "x", "kind": "fixed", "bits": 21, "lo": 0.0, "hi": 1.0,
       "dither": True, "rel_identity": False, "exp_bits": 0}, ...]}
  params = {"dim": 3, "grid_res": 512, "bound_cells": 3, "sort_every": 0,
            "dt": 1e-4, "gravity": [0, -9.8, 0], "E": 1e3, "nu": 0.2,
            "rho": 1.0, "p_vol": ...}
"""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpmq.so")

FIELDS = {"x": 0, "v": 1, "C": 2, "F": 3, "J": 4}
MATERIALS = {"elastic": 0, "fluid": 1}


def slot3_name(scheme: dict) -> str:
    """The field in the fourth state slot: "F" (elastic solid) or "J" (fluid)."""
    return "J" if any(f["field"] == "J" for f in scheme["fields"]) else "F"
KINDS = {"fixed": 0, "shared_exp": 1, "raw_f32": 2}
REL_IDENTITY = 1

STATUS = {0: "MPMQ_OK", -1: "MPMQ_EINVAL", -2: "MPMQ_ENOMEM", -3: "MPMQ_EDEVICE",
          -4: "MPMQ_ESTATE", -5: "MPMQ_ENOTIMPL"}


class MpmqError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class mpmq_field_scheme(ct.Structure):
    _fields_ = [("field", ct.c_int32), ("kind", ct.c_int32), ("bits", ct.c_int32),
                ("exp_bits", ct.c_int32), ("dither", ct.c_int32), ("flags", ct.c_int32),
                ("lo", ct.c_double), ("hi", ct.c_double)]


class mpmq_scheme(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("n_fields", ct.c_int32),
                ("fields", ct.POINTER(mpmq_field_scheme)), ("seed", ct.c_uint64)]


class mpmq_params(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("grid_res", ct.c_int32), ("bound_cells", ct.c_int32),
                ("sort_every", ct.c_int32), ("dt", ct.c_double), ("gravity", ct.c_double * 3),
                ("E", ct.c_double), ("nu", ct.c_double), ("rho", ct.c_double), ("p_vol", ct.c_double),
                ("material", ct.c_int32), ("reserved", ct.c_int32)]


class mpmq_sizes(ct.Structure):
    _fields_ = [("words_per_particle", ct.c_int32), ("record_bits", ct.c_int32),
                ("capacity_padded", ct.c_int64), ("packed_bytes", ct.c_int64),
                ("grid_bytes", ct.c_int64), ("scratch_bytes", ct.c_int64), ("ids_bytes", ct.c_int64)]


class mpmq_buffers(ct.Structure):
    _fields_ = [("packed", ct.c_void_p), ("grid_a", ct.c_void_p), ("grid_b", ct.c_void_p),
                ("scratch", ct.c_void_p), ("ids", ct.c_void_p)]


class mpmq_stats_t(ct.Structure):
    _fields_ = [("sat", ct.c_int64 * 4), ("nan", ct.c_int64 * 4), ("up", ct.c_int64 * 4),
                ("down", ct.c_int64 * 4), ("steps", ct.c_int64), ("sorts", ct.c_int64),
                ("fallback", ct.c_int64), ("active_nodes", ct.c_int64), ("clamped", ct.c_int64),
                ("atomics", ct.c_int64), ("wide", ct.c_int64)]


class mpmq_kernel_time(ct.Structure):
    _fields_ = [("name", ct.c_char * 32), ("launches", ct.c_int64), ("total_ms", ct.c_double)]


class mpmq_adjoint_spec(ct.Structure):
    _fields_ = [("objective", ct.c_int32), ("axis", ct.c_int32), ("steps", ct.c_int32),
                ("checkpoint_every", ct.c_int32)]


class mpmq_adjoint_result(ct.Structure):
    _fields_ = [("z", ct.c_double), ("G", ct.c_double * 4), ("g", ct.c_double * 4),
                ("lo", ct.c_double * 4), ("hi", ct.c_double * 4), ("recomputed", ct.c_int64),
                ("states", ct.c_int64)]


OBJECTIVES = {"com": 0, "ke": 1}
SOLVE_MODES = {"error": 0, "memory": 1}


class mpmq_solve_input(ct.Structure):
    _fields_ = [("mode", ct.c_int32), ("n_types", ct.c_int32), ("min_bits", ct.c_int32), ("max_bits", ct.c_int32),
                ("eps", ct.c_double), ("z", ct.c_double), ("P", ct.POINTER(ct.c_double)),
                ("g", ct.POINTER(ct.c_double)), ("R", ct.POINTER(ct.c_double))]


class mpmq_solve_output(ct.Structure):
    _fields_ = [("delta", ct.POINTER(ct.c_double)), ("b_cont", ct.POINTER(ct.c_double)),
                ("bits", ct.POINTER(ct.c_int32)), ("expected_error", ct.c_double), ("total_bits", ct.c_double)]


class mpmq_auto_input(ct.Structure):
    _fields_ = [("mode", ct.c_int32), ("min_bits", ct.c_int32), ("max_bits", ct.c_int32), ("reserved", ct.c_int32),
                ("eps", ct.c_double), ("range_factor", ct.c_double), ("n_particles", ct.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libmpmq.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2207_04658_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    # torch first: the library then binds the HIP runtime torch loaded (one
    # runtime per process, so torch's device buffers and streams are valid
    # handles for the library)
    import torch  # noqa: F401
    L = ct.CDLL(path)
    P = ct.c_void_p
    S = ct.c_int
    sig = {
        "mpmq_query_sizes": [ct.POINTER(mpmq_scheme), ct.POINTER(mpmq_params), ct.c_int64, ct.POINTER(mpmq_sizes)],
        "mpmq_create": [ct.POINTER(mpmq_scheme), ct.POINTER(mpmq_params), ct.POINTER(mpmq_buffers), ct.c_int64, P,
                        ct.POINTER(P)],
        "mpmq_destroy": [P],
        "mpmq_encode": [P, P, P, P, P, ct.c_int64],
        "mpmq_decode": [P, P, P, P, P],
        "mpmq_packed": [P, ct.POINTER(P), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64)],
        "mpmq_step": [P, ct.c_int32],
        "mpmq_step_batch": [ct.POINTER(P), ct.c_int32, ct.c_int32],
        "mpmq_calib_atomics": [P, ct.c_int64, ct.c_int32, ct.c_int64, P],
        "mpmq_step_count": [P, ct.POINTER(ct.c_int64)],
        "mpmq_stats": [P, ct.POINTER(mpmq_stats_t)],
        "mpmq_reset_stats": [P],
        "mpmq_set_stats": [P, ct.c_int32],
        "mpmq_set_timing": [P, ct.c_int32],
        "mpmq_specialize": [P, ct.c_int32],
        "mpmq_kernel_times": [P, ct.POINTER(mpmq_kernel_time), ct.c_int32, ct.POINTER(ct.c_int32)],
        "mpmq_adjoint_workspace": [P, ct.POINTER(mpmq_adjoint_spec), ct.POINTER(ct.c_int64)],
        "mpmq_adjoint": [P, ct.POINTER(mpmq_adjoint_spec), P, ct.c_int64, P, ct.POINTER(mpmq_adjoint_result)],
        "mpmq_adjoint_static": [P, ct.POINTER(mpmq_adjoint_spec), P, ct.POINTER(mpmq_adjoint_result)],
        "mpmq_solve_scheme": [ct.POINTER(mpmq_solve_input), ct.POINTER(mpmq_solve_output)],
        "mpmq_auto_scheme": [ct.POINTER(mpmq_scheme), ct.POINTER(mpmq_adjoint_result), ct.POINTER(mpmq_auto_input),
                             ct.POINTER(mpmq_field_scheme), ct.POINTER(mpmq_solve_output)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = S
    L.mpmq_error_string.argtypes = [S]
    L.mpmq_error_string.restype = ct.c_char_p
    L.mpmq_last_error.argtypes = [P]
    L.mpmq_last_error.restype = ct.c_char_p
    L.mpmq_solver_error.argtypes = []
    L.mpmq_solver_error.restype = ct.c_char_p
    _lib = L
    return L


def exported_symbols():
    return ["mpmq_query_sizes", "mpmq_create", "mpmq_destroy", "mpmq_encode", "mpmq_decode",
            "mpmq_packed", "mpmq_step", "mpmq_step_batch", "mpmq_step_count", "mpmq_calib_atomics", "mpmq_stats", "mpmq_reset_stats", "mpmq_set_stats",
            "mpmq_specialize",
            "mpmq_set_timing", "mpmq_kernel_times", "mpmq_adjoint_workspace", "mpmq_adjoint", "mpmq_adjoint_static", "mpmq_solve_scheme", "mpmq_auto_scheme", "mpmq_solver_error", "mpmq_error_string",
            "mpmq_last_error"]


def _check(status, ctx=None):
    if status != 0:
        msg = load().mpmq_last_error(ctx).decode()
        raise MpmqError(status, msg)


def make_scheme(scheme: dict):
    """Returns (mpmq_scheme, keep-alive field array)."""
    fields = (mpmq_field_scheme * len(scheme["fields"]))()
    for i, f in enumerate(scheme["fields"]):
        fields[i].field = FIELDS[f["field"]]
        fields[i].kind = KINDS[f["kind"]]
        fields[i].bits = int(f.get("bits", 32))
        fields[i].exp_bits = int(f.get("exp_bits", 0))
        fields[i].dither = int(bool(f.get("dither", False)))
        fields[i].flags = REL_IDENTITY if f.get("rel_identity", False) else 0
        fields[i].lo = float(f.get("lo", 0.0))
        fields[i].hi = float(f.get("hi", 1.0))
    s = mpmq_scheme()
    s.dim = scheme["dim"]
    s.n_fields = len(scheme["fields"])
    s.fields = ct.cast(fields, ct.POINTER(mpmq_field_scheme))
    s.seed = int(scheme.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    return s, fields


def make_params(params: dict):
    p = mpmq_params()
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
    p.reserved = 0
    return p


def mpmq_query_sizes(scheme: dict, params: dict, capacity: int) -> dict:
    s, keep = make_scheme(scheme)
    p = make_params(params)
    out = mpmq_sizes()
    _check(load().mpmq_query_sizes(ct.byref(s), ct.byref(p), int(capacity), ct.byref(out)))
    return {k: getattr(out, k) for k, _ in mpmq_sizes._fields_}


# bytes of the library's static adjoint workspace (MPMQ_STATIC_WORKSPACE_BYTES)
STATIC_WORKSPACE_BYTES = 64 << 20


class Context:
    """One simulation: owns torch device buffers and an mpmq_ctx.

    Methods map one-to-one on the C ABI: encode, decode, step, packed,
    stats, kernel_times.  All device work is enqueued on `stream` (default:
    torch's current stream)."""

    def __init__(self, scheme: dict, params: dict, capacity: int, stream=None, track_ids=True,
                 device=None, specialize=False):
        import torch
        L = load()
        self.scheme, self.params = scheme, params
        self.dim = scheme["dim"]
        self.f3 = slot3_name(scheme)
        self.nc3 = 1 if self.f3 == "J" else self.dim * self.dim
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.sizes = mpmq_query_sizes(scheme, params, capacity)
        sz = self.sizes
        u8 = torch.uint8

        def buf(nbytes):
            return torch.empty(max(int(nbytes), 256), dtype=u8, device=self.device)

        self.packed = buf(sz["packed_bytes"])
        self.grid_a = buf(sz["grid_bytes"])
        self.grid_b = buf(sz["grid_bytes"])
        self.scratch = buf(sz["scratch_bytes"])
        self.ids_buf = buf(sz["ids_bytes"]) if track_ids else None
        bufs = mpmq_buffers(self.packed.data_ptr(), self.grid_a.data_ptr(), self.grid_b.data_ptr(),
                            self.scratch.data_ptr(), self.ids_buf.data_ptr() if track_ids else None)
        s, keep = make_scheme(scheme)
        p = make_params(params)
        h = ct.c_void_p()
        _check(L.mpmq_create(ct.byref(s), ct.byref(p), ct.byref(bufs), int(capacity),
                             ct.c_void_p(self.stream.cuda_stream), ct.byref(h)))
        self._h = h
        self.capacity = capacity
        self.n = 0
        if specialize:
            self.specialize(True)

    # -- C ABI calls ----------------------------------------------------------
    def encode(self, x, v, C, F):
        """x, v: [dim, n]; C: [dim*dim, n]; F: [dim*dim, n] (fluid: J [1, n])
        float32 CUDA tensors (contiguous)."""
        import torch
        ts = [t.to(device=self.device, dtype=torch.float32).contiguous() for t in (x, v, C, F)]
        n = ts[0].shape[-1]
        _check(load().mpmq_encode(self._h, *[t.data_ptr() for t in ts], int(n)), self._h)
        self._keep = ts  # inputs stay alive until the stream has consumed them
        self.n = n

    def decode(self):
        import torch
        d, n = self.dim, self.n
        out = [torch.empty((k, n), dtype=torch.float32, device=self.device) for k in (d, d, d * d, self.nc3)]
        _check(load().mpmq_decode(self._h, *[t.data_ptr() for t in out]), self._h)
        return tuple(out)

    def step(self, n_substeps=1):
        _check(load().mpmq_step(self._h, int(n_substeps)), self._h)

    def step_count(self):
        v = ct.c_int64()
        _check(load().mpmq_step_count(self._h, ct.byref(v)), self._h)
        return v.value

    def packed_view(self):
        """Packed words as a [W, n] int32 view (strided by the padded capacity)."""
        import torch
        W = self.sizes["words_per_particle"]
        cap = self.sizes["capacity_padded"]
        return self.packed[: 4 * W * cap].view(torch.int32).view(W, cap)[:, : self.n]

    def words(self):
        """Packed words copied to host as a [W, n] uint32 numpy array."""
        import numpy as np
        self.stream.synchronize()
        return self.packed_view().cpu().numpy().view(np.uint32)

    def ids(self):
        import numpy as np
        import torch
        if self.ids_buf is None:
            raise ValueError("context created without id tracking")
        self.stream.synchronize()
        return self.ids_buf[: 4 * self.n].view(torch.int32).cpu().numpy().astype(np.int64)

    def stats(self):
        st = mpmq_stats_t()
        _check(load().mpmq_stats(self._h, ct.byref(st)), self._h)
        names = ["x", "v", "C", self.f3]
        out = {names[i]: {"sat": st.sat[i], "nan": st.nan[i], "up": st.up[i], "down": st.down[i]}
               for i in range(4)}
        out.update(steps=st.steps, sorts=st.sorts, fallback=st.fallback, active_nodes=st.active_nodes,
                   clamped=st.clamped, atomics=st.atomics, wide=st.wide)
        return out

    def set_stats(self, level):
        """0: saturation and NaN counts (default); 1: also round-up/down counts."""
        _check(load().mpmq_set_stats(self._h, int(level)), self._h)

    def reset_stats(self):
        _check(load().mpmq_reset_stats(self._h), self._h)

    def specialize(self, enable=True):
        """mpmq_specialize: scheme-specialized fused kernels (same results)."""
        _check(load().mpmq_specialize(self._h, 1 if enable else 0), self._h)

    def set_timing(self, enable=True):
        _check(load().mpmq_set_timing(self._h, 1 if enable else 0), self._h)

    def kernel_times(self, clear=False):
        arr = (mpmq_kernel_time * 32)()
        cnt = ct.c_int32()
        _check(load().mpmq_kernel_times(self._h, arr, -1 if clear else 32, ct.byref(cnt)), self._h)
        if clear:
            return {}
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(cnt.value, 32))}

    def adjoint_workspace_bytes(self, steps, checkpoint_every=8, objective="com", axis=1):
        s = mpmq_adjoint_spec(OBJECTIVES[objective], int(axis), int(steps), int(checkpoint_every))
        b = ct.c_int64()
        _check(load().mpmq_adjoint_workspace(self._h, ct.byref(s), ct.byref(b)), self._h)
        return b.value

    def adjoint(self, steps, objective="com", axis=1, checkpoint_every=8, want_lambda0=False):
        """Forward `steps` substeps from the current state and back-propagate
        (mpmq_adjoint).  Returns a dict with z, G and g per field (x, v, C, F),
        the per-field value ranges lo / hi, recomputed substeps, states held
        and, with want_lambda0, lambda_0 as a [2d + 2d^2, n] float32 tensor in
        encode order."""
        import torch
        s = mpmq_adjoint_spec(OBJECTIVES[objective], int(axis), int(steps), int(checkpoint_every))
        b = ct.c_int64()
        L = load()
        _check(L.mpmq_adjoint_workspace(self._h, ct.byref(s), ct.byref(b)), self._h)
        ws = torch.empty(max(int(b.value), 256), dtype=torch.uint8, device=self.device)
        rows = 2 * self.dim + self.dim * self.dim + self.nc3
        lam0 = torch.empty((rows, self.n), dtype=torch.float32, device=self.device) if want_lambda0 else None
        res = mpmq_adjoint_result()
        _check(L.mpmq_adjoint(self._h, ct.byref(s), ct.c_void_p(ws.data_ptr()), int(b.value),
                              ct.c_void_p(lam0.data_ptr()) if lam0 is not None else None, ct.byref(res)), self._h)
        names = ["x", "v", "C", self.f3]
        out = {"z": res.z, "G": {names[i]: res.G[i] for i in range(4)}, "g": {names[i]: res.g[i] for i in range(4)},
               "lo": {names[i]: res.lo[i] for i in range(4)}, "hi": {names[i]: res.hi[i] for i in range(4)},
               "recomputed": res.recomputed, "states": res.states, "workspace_bytes": b.value}
        if lam0 is not None:
            out["lambda0"] = lam0
        return out

    def adjoint_static(self, steps, objective="com", axis=1, checkpoint_every=8, lambda0=None):
        """mpmq_adjoint_static: the adjoint with the library's static device
        workspace (STATIC_WORKSPACE_BYTES); nothing is allocated for the call.
        lambda0: optional caller-owned float32 tensor [2d + 2d^2, n] on the
        context's device that receives lambda_0.  Returns the dict of
        adjoint() (without workspace_bytes)."""
        import torch
        s = mpmq_adjoint_spec(OBJECTIVES[objective], int(axis), int(steps), int(checkpoint_every))
        if lambda0 is not None:
            rows = 2 * self.dim + self.dim * self.dim + self.nc3
            if (tuple(lambda0.shape) != (rows, self.n) or lambda0.dtype != torch.float32
                    or not lambda0.is_contiguous() or lambda0.device != self.device):
                raise ValueError(f"lambda0 must be a contiguous float32 [{rows}, {self.n}] tensor on {self.device}")
        res = mpmq_adjoint_result()
        _check(load().mpmq_adjoint_static(self._h, ct.byref(s),
                                          ct.c_void_p(lambda0.data_ptr()) if lambda0 is not None else None,
                                          ct.byref(res)), self._h)
        names = ["x", "v", "C", self.f3]
        return {"z": res.z, "G": {names[i]: res.G[i] for i in range(4)}, "g": {names[i]: res.g[i] for i in range(4)},
                "lo": {names[i]: res.lo[i] for i in range(4)}, "hi": {names[i]: res.hi[i] for i in range(4)},
                "recomputed": res.recomputed, "states": res.states}

    def close(self):
        if getattr(self, "_h", None):
            self.stream.synchronize()
            load().mpmq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def calib_atomics(buf, passes=1, stride=1, stream=None):
    """mpmq_calib_atomics on a uint64/int64 CUDA tensor (see include/mpmq.h)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(buf.device)
    s = load().mpmq_calib_atomics(ct.c_void_p(buf.data_ptr()), int(buf.numel()), int(passes), int(stride),
                                  ct.c_void_p(st.cuda_stream))
    if s != 0:
        raise MpmqError(s, load().mpmq_last_error(None).decode())


def step_batch(contexts, n_substeps=1):
    """mpmq_step_batch: advances every Context of `contexts` (same dimension,
    material and stream) by n_substeps with one launch per kernel for the
    whole batch."""
    ctxs = list(contexts)
    if not ctxs:
        return
    arr = (ct.c_void_p * len(ctxs))(*[c._h.value for c in ctxs])
    st = load().mpmq_step_batch(arr, len(ctxs), int(n_substeps))
    if st != 0:
        raise MpmqError(st, load().mpmq_last_error(ctxs[0]._h).decode())


def solve_scheme(P, g, R, mode="error", eps=1e-3, z=1.0, min_bits=1, max_bits=32):
    """mpmq_solve_scheme (host only).  Returns dict(delta, b_cont, bits,
    expected_error, total_bits) with lists per type."""
    H = len(P)
    arr = ct.c_double * H
    Pa, ga, Ra = arr(*map(float, P)), arr(*map(float, g)), arr(*map(float, R))
    d, b, bits = arr(), arr(), (ct.c_int32 * H)()
    inp = mpmq_solve_input(SOLVE_MODES[mode], H, int(min_bits), int(max_bits), float(eps), float(z),
                           Pa, ga, Ra)
    out = mpmq_solve_output(d, b, bits, 0.0, 0.0)
    st = load().mpmq_solve_scheme(ct.byref(inp), ct.byref(out))
    if st != 0:
        raise MpmqError(st, load().mpmq_solver_error().decode())
    return {"delta": list(d), "b_cont": list(b), "bits": list(bits), "expected_error": out.expected_error,
            "total_bits": out.total_bits}


def auto_scheme(base: dict, adjoint_result: dict, n: int, mode="error", eps=1e-3, range_factor=2.0,
                min_bits=1, max_bits=32):
    """Alg. 1 through mpmq_auto_scheme: a fixed-point scheme from an adjoint
    run (normally of the full-precision layout): per field, the recorded
    value range widened by `range_factor` about its centre, and the bits of
    the closed-form solver.  Placement order, dither, REL_IDENTITY and the
    seed follow `base`.  Returns (scheme dict, solver output dict)."""
    names = ["x", "v", "C", slot3_name(base)]
    res = mpmq_adjoint_result()
    res.z = float(adjoint_result["z"])
    for i, f in enumerate(names):
        res.g[i] = float(adjoint_result["g"][f])
        res.lo[i] = float(adjoint_result["lo"][f])
        res.hi[i] = float(adjoint_result["hi"][f])
    s, keep = make_scheme(base)
    inp = mpmq_auto_input(SOLVE_MODES[mode], int(min_bits), int(max_bits), 0, float(eps), float(range_factor), int(n))
    out_fields = (mpmq_field_scheme * 4)()
    arr = ct.c_double * 4
    d, b, bits = arr(), arr(), (ct.c_int32 * 4)()
    sol = mpmq_solve_output(d, b, bits, 0.0, 0.0)
    st = load().mpmq_auto_scheme(ct.byref(s), ct.byref(res), ct.byref(inp), out_fields, ct.byref(sol))
    if st != 0:
        raise MpmqError(st, load().mpmq_solver_error().decode())
    inv = {v: k for k, v in FIELDS.items()}
    fields = [{"field": inv[f.field], "kind": "fixed", "bits": f.bits, "lo": f.lo, "hi": f.hi,
               "dither": bool(f.dither), "rel_identity": bool(f.flags & REL_IDENTITY), "exp_bits": 0}
              for f in out_fields]
    return ({"dim": base["dim"], "seed": base.get("seed", 0), "fields": fields},
            {"delta": list(d), "b_cont": list(b), "bits": list(bits), "expected_error": sol.expected_error,
             "total_bits": sol.total_bits})


class QuantizedRollout:
    """torch.autograd.Function over `steps` quantized substeps.

    rollout(ctx, x, v, C, F) encodes (x, v, C, F) into the context, runs
    the forward and the hand-written adjoint (mpmq_adjoint) and returns the
    objective z as a 0-d float64 tensor; z.backward() delivers lambda_0 to the
    inputs (the quantization of the stored states enters as an additive
    error, so the encode is passed straight through).  G and g of the run are
    left in ctx.last_adjoint."""

    _fn = None

    @classmethod
    def function(cls):
        if cls._fn is None:
            import torch

            class _Rollout(torch.autograd.Function):
                @staticmethod
                def forward(fctx, handle, steps, objective, axis, checkpoint_every, x, v, C, F):
                    handle.encode(x, v, C, F)
                    res = handle.adjoint(steps, objective=objective, axis=axis, checkpoint_every=checkpoint_every,
                                         want_lambda0=True)
                    handle.last_adjoint = res
                    d = handle.dim
                    lam = res["lambda0"]
                    fctx.save_for_backward(lam[:d], lam[d:2 * d], lam[2 * d:2 * d + d * d], lam[2 * d + d * d:])
                    # (the last block has handle.nc3 rows: F, or J for a fluid)
                    return torch.tensor(res["z"], dtype=torch.float64, device=x.device)

                @staticmethod
                def backward(fctx, gz):
                    lx, lv, lC, lF = fctx.saved_tensors
                    s = gz.to(torch.float32)
                    return (None, None, None, None, None, lx * s, lv * s, lC * s, lF * s)

            cls._fn = _Rollout
        return cls._fn


def rollout(handle: Context, x, v, C, F, steps, objective="com", axis=1, checkpoint_every=8):
    """Differentiable quantized rollout (see QuantizedRollout)."""
    return QuantizedRollout.function().apply(handle, int(steps), objective, int(axis), int(checkpoint_every),
                                             x, v, C, F)
