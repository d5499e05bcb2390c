"""ctypes binding of libmrtlb.so (the C ABI in include/mrtlb.h).

Argument marshalling only: every function forwards to the C entry point of
the same name; the classes below only own handles and convert NumPy arrays
(FP64, C order) to pointers.  Importing this module does not load the
library; the first call does, and fails loudly if it has not been built.
"""

from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int64, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MRTLB_LIB points at another build of the library (tuning comparisons)
LIB_PATH = os.environ.get("MRTLB_LIB", os.path.join(_HERE, "libmrtlb.so"))

MRTLB_OK, MRTLB_EINVAL, MRTLB_ENOMEM, MRTLB_EDEVICE, MRTLB_ENUMERIC = 0, -1, -2, -3, -4
MRTLB_RD2Q25, MRTLB_RD2Q13, MRTLB_RD3Q53, MRTLB_RD3Q33, MRTLB_RD2Q21, MRTLB_D2Q21K, MRTLB_RD3Q45 = range(7)
MRTLB_RD2Q17 = {k: 6 + k for k in range(1, 6)}     # D2Q17 cases 1-5
MRTLB_D2Q9, MRTLB_D3Q27 = 12, 13                     # standard lattices, k = 1 model
MRTLB_CUSTOM = 14                                    # user-supplied velocity set
MRTLB_NSE_INC, MRTLB_NSE_COMP, MRTLB_NCDE, MRTLB_CDE = 0, 1, 2, 3
MRTLB_FP64, MRTLB_FP32, MRTLB_FP32_DEV, MRTLB_FP16_DEV, MRTLB_BF16_DEV, MRTLB_I16_DEV = 0, 1, 2, 3, 4, 5
MRTLB_FP32_DEV_F64 = 6
TRANSFORMS = {"valu": 0, "mfma": 1}

KINDS = {"rD2Q25": MRTLB_RD2Q25, "rD2Q13": MRTLB_RD2Q13, "rD3Q53": MRTLB_RD3Q53, "rD3Q33": MRTLB_RD3Q33,
         "rD2Q21": MRTLB_RD2Q21, "D2Q21K": MRTLB_D2Q21K, "rD3Q45": MRTLB_RD3Q45,
         "D2Q9": MRTLB_D2Q9, "D3Q27": MRTLB_D3Q27, "custom": MRTLB_CUSTOM, **{"rD2Q17-%d" % k: v for k, v in MRTLB_RD2Q17.items()}}
MODELS = {"NSE_INC": MRTLB_NSE_INC, "NSE_COMP": MRTLB_NSE_COMP, "NCDE": MRTLB_NCDE, "CDE": MRTLB_CDE}
STORAGES = {"fp64": MRTLB_FP64, "fp32": MRTLB_FP32, "fp32_dev": MRTLB_FP32_DEV, "fp16_dev": MRTLB_FP16_DEV,
            "bf16_dev": MRTLB_BF16_DEV, "i16_dev": MRTLB_I16_DEV, "fp32_dev_f64": MRTLB_FP32_DEV_F64}


class MrtlbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("mrtlb error %d: %s" % (status, msg))
        self.status = status


class mrtlb_lattice_desc(ctypes.Structure):
    _fields_ = [("kind", c_int), ("c", c_double * 3), ("cs2", c_double), ("free_w", c_double * 4),
                ("n_free", c_int), ("d", c_int), ("b", c_int), ("e", POINTER(c_int)), ("w", POINTER(c_double))]


class mrtlb_model_desc(ctypes.Structure):
    _fields_ = [("model", c_int), ("rho0", c_double), ("s0", c_double), ("s1", c_double), ("s_shear", c_double),
                ("s_bulk", c_double), ("s3", c_double), ("s_high", c_double), ("m30", c_int), ("D0", c_double),
                ("D2", c_double), ("adv_u", c_double * 3), ("u_bound", c_double), ("dev_bound", c_double),
                ("gn_bt", c_double * 3), ("gn_dd", c_double * 3), ("src_q", c_double), ("src_k", c_double),
                ("three_level", c_int), ("mass_src", c_double), ("g_share", c_double), ("lambda1", c_double),
                ("lambda2", c_double), ("m2g_form", c_int)]


_lib = None
_DP = POINTER(c_double)


def lib():
    """Load libmrtlb.so once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmrtlb.so is not built (expected at %s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "mrtlb_last_error": (c_char_p, []),
        "mrtlb_version": (c_int, []),
        "mrtlb_ctx_create": (c_int, [c_int, c_void_p, c_size_t, POINTER(c_void_p)]),
        "mrtlb_ctx_destroy": (None, [c_void_p]),
        "mrtlb_ctx_memory": (c_int, [c_void_p, POINTER(c_size_t), POINTER(c_size_t)]),
        "mrtlb_ctx_synchronize": (c_int, [c_void_p]),
        "mrtlb_lattice_create": (c_int, [POINTER(mrtlb_lattice_desc), POINTER(c_void_p)]),
        "mrtlb_lattice_destroy": (None, [c_void_p]),
        "mrtlb_lattice_query": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int), POINTER(c_int), _DP,
                                        POINTER(c_int), _DP, _DP]),
        "mrtlb_solve_create": (c_int, [c_void_p, c_void_p, POINTER(mrtlb_model_desc), POINTER(c_int64), c_int, c_int,
                                       POINTER(c_void_p)]),
        "mrtlb_solve_footprint": (c_int, [c_void_p, POINTER(c_int64), c_int, c_int, c_int, POINTER(c_size_t)]),
        "mrtlb_population_bytes": (c_int, [c_void_p, POINTER(c_int64), c_int, POINTER(c_size_t)]),
        "mrtlb_solve_create_external": (c_int, [c_void_p, c_void_p, POINTER(mrtlb_model_desc), POINTER(c_int64),
                                                c_int, c_int, c_void_p, c_void_p, POINTER(c_void_p)]),
        "mrtlb_solve_destroy": (None, [c_void_p]),
        "mrtlb_init_fields": (c_int, [c_void_p, _DP, _DP, _DP]),
        "mrtlb_step": (c_int, [c_void_p, c_int64]),
        "mrtlb_step_timed": (c_int, [c_void_p, c_int64, _DP]),
        "mrtlb_stream_only": (c_int, [c_void_p, c_int64, _DP]),
        "mrtlb_solve_launch_shape": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int), POINTER(c_int),
                                             POINTER(c_int64)]),
        "mrtlb_batch_step": (c_int, [POINTER(c_void_p), c_int, POINTER(c_int64)]),
        "mrtlb_read_moments": (c_int, [c_void_p, _DP, _DP]),
        "mrtlb_conserved": (c_int, [c_void_p, _DP, _DP]),
        "mrtlb_conserved_noalloc": (c_int, [c_void_p, _DP, _DP]),
        "mrtlb_solve_set_transform": (c_int, [c_void_p, c_int]),
        "mrtlb_set_velocity_field": (c_int, [c_void_p, _DP]),
        "mrtlb_set_force_field": (c_int, [c_void_p, _DP]),
        "mrtlb_set_mass_source_field": (c_int, [c_void_p, _DP]),
        "mrtlb_set_drift_correction": (c_int, [c_void_p, c_int64]),
        "mrtlb_host_alloc": (c_int, [c_size_t, POINTER(c_void_p)]),
        "mrtlb_host_free": (None, [c_void_p]),
        "mrtlb_read_populations": (c_int, [c_void_p, _DP]),
        "mrtlb_write_populations": (c_int, [c_void_p, _DP]),
        "mrtlb_solve_steps": (c_int64, [c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


EXPORTED = ["mrtlb_last_error", "mrtlb_version", "mrtlb_ctx_create", "mrtlb_ctx_destroy", "mrtlb_ctx_memory",
            "mrtlb_ctx_synchronize", "mrtlb_lattice_create", "mrtlb_lattice_destroy", "mrtlb_lattice_query",
            "mrtlb_solve_create", "mrtlb_solve_footprint", "mrtlb_solve_destroy", "mrtlb_init_fields",
            "mrtlb_step", "mrtlb_step_timed", "mrtlb_stream_only", "mrtlb_batch_step", "mrtlb_read_moments",
            "mrtlb_conserved",
            "mrtlb_read_populations", "mrtlb_write_populations", "mrtlb_solve_steps", "mrtlb_set_drift_correction",
            "mrtlb_host_alloc", "mrtlb_host_free", "mrtlb_population_bytes", "mrtlb_solve_create_external",
            "mrtlb_conserved_noalloc", "mrtlb_solve_set_transform", "mrtlb_set_velocity_field",
            "mrtlb_set_force_field", "mrtlb_set_mass_source_field", "mrtlb_solve_launch_shape"]


def _check(status):
    if status != MRTLB_OK:
        raise MrtlbError(status, lib().mrtlb_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_DP)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# thin owners of the C handles
# --------------------------------------------------------------------------

_live_contexts = weakref.WeakSet()


@atexit.register
def _close_all():
    # release device state before the HIP runtime is torn down
    for c in list(_live_contexts):
        c.close()


class Context:
    """mrtlb_ctx: device, stream (e.g. torch.cuda.current_stream().cuda_stream), HBM budget.

    Closing a context closes the solves created on it first."""

    def __init__(self, device=0, stream=None, hbm_budget=0):
        self.h = None
        self._solves = weakref.WeakSet()
        h = c_void_p()
        _check(lib().mrtlb_ctx_create(int(device), c_void_p(stream) if stream else None, c_size_t(hbm_budget),
                                      byref(h)))
        self.h = h
        _live_contexts.add(self)

    def memory(self):
        used, budget = c_size_t(), c_size_t()
        _check(lib().mrtlb_ctx_memory(self.h, byref(used), byref(budget)))
        return used.value, budget.value

    def synchronize(self):
        _check(lib().mrtlb_ctx_synchronize(self.h))

    def close(self):
        if self.h:
            for s in list(self._solves):
                s.close()
            lib().mrtlb_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lattice:
    """mrtlb_lattice built from (kind, c, cs2, free weights); kind "custom"
    takes the velocity set ``e`` (b x d integer multiples) and weights ``w``."""

    def __init__(self, kind, c, cs2, free=(), e=None, w=None):
        d = mrtlb_lattice_desc()
        d.kind = KINDS[kind] if isinstance(kind, str) else int(kind)
        for a, v in enumerate(c):
            d.c[a] = float(v)
        d.cs2 = float(cs2)
        for i, v in enumerate(free):
            d.free_w[i] = float(v)
        d.n_free = len(free)
        if e is not None:
            ea = np.ascontiguousarray(np.asarray(e, dtype=np.int32))
            wa = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
            d.b, d.d = ea.shape
            d.e = ea.ctypes.data_as(POINTER(c_int))
            d.w = _ptr(wa)
        h = c_void_p()
        _check(lib().mrtlb_lattice_create(byref(d), byref(h)))
        self.h = h
        self.kind = kind

    def query(self):
        b, d, nlow = c_int(), c_int(), c_int()
        _check(lib().mrtlb_lattice_query(self.h, byref(b), byref(d), None, None, byref(nlow), None, None))
        e = np.zeros(b.value * d.value, dtype=np.int32)
        w = np.zeros(b.value)
        H = np.zeros(nlow.value * b.value)
        n = np.zeros(nlow.value)
        _check(lib().mrtlb_lattice_query(self.h, None, None, e.ctypes.data_as(POINTER(c_int)), _ptr(w), None,
                                         _ptr(H), _ptr(n)))
        return dict(b=b.value, d=d.value, e=e.reshape(b.value, d.value), w=w, H=H.reshape(nlow.value, b.value),
                    norms=n)

    def close(self):
        if self.h:
            lib().mrtlb_lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def model_desc(eq, rho0=1.0, s0=1.2, s1=1.2, s_shear=1.25, s_bulk=1.2, s3=1.2, s_high=1.2, m30=True, D0=0.0,
               D2=0.0, adv_u=(0.0, 0.0, 0.0), u_bound=0.0, dev_bound=0.0, gn_bt=(0.0, 0.0, 0.0),
               gn_dd=(0.0, 0.0, 0.0), src_q=0.0, src_k=0.0, three_level=False, mass_src=0.0, g_share=0.0,
               lambda1=1.0, lambda2=1.0, m2g_form=0):
    """Model parameters; u_bound / dev_bound size the int16 storage's ranges
    (max |u| and max |rho - rho0| / rho0, or max |phi| for the NCDE);
    gn_bt / gn_dd are the general-NCDE coefficients A1 b_bar and diag(A2);
    src_q + src_k phi is the NCDE source, three_level selects the explicit
    three-level scheme instead of full correction (NCDE and NSE); mass_src is
    the compressible NSE's uniform mass source (the solve needs has_force);
    g_share is the share of the NSE force and mass source carried by G,
    corrected with lambda2 and lambda1; m2g_form 1 selects the gradient form
    of the NSE's auxiliary second moment."""
    m = mrtlb_model_desc()
    m.model = MODELS[eq] if isinstance(eq, str) else int(eq)
    m.rho0, m.s0, m.s1, m.s_shear, m.s_bulk, m.s3, m.s_high = rho0, s0, s1, s_shear, s_bulk, s3, s_high
    m.m30 = 1 if m30 else 0
    m.D0, m.D2 = D0, D2
    for a in range(3):
        m.adv_u[a] = float(adv_u[a]) if a < len(adv_u) else 0.0
    m.u_bound, m.dev_bound = float(u_bound), float(dev_bound)
    for a in range(3):
        m.gn_bt[a] = float(gn_bt[a]) if a < len(gn_bt) else 0.0
        m.gn_dd[a] = float(gn_dd[a]) if a < len(gn_dd) else 0.0
    m.src_q, m.src_k = float(src_q), float(src_k)
    m.three_level = 1 if three_level else 0
    m.mass_src = float(mass_src)
    m.g_share, m.lambda1, m.lambda2 = float(g_share), float(lambda1), float(lambda2)
    m.m2g_form = int(m2g_form)
    return m


class HostBuffer:
    """Page-locked float64 host array from the library (mrtlb_host_alloc);
    ``array`` is a NumPy view of it.  Freed by close() or at exit."""

    def __init__(self, n):
        p = c_void_p()
        _check(lib().mrtlb_host_alloc(int(n) * 8, byref(p)))
        self._p = p
        self.n = int(n)
        self.array = np.ctypeslib.as_array(ctypes.cast(p, POINTER(c_double)), shape=(self.n,))

    def close(self):
        if self._p is not None and self._p.value:
            self.array = None
            lib().mrtlb_host_free(self._p)
        self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MRTLB_FOOTPRINT_M2G_GRADIENT = 0x100


def footprint(lattice, shape, storage, eq, has_force=False, m2g_form=0):
    n = (c_int64 * 3)(*_nxyz(shape))
    out = c_size_t()
    st = STORAGES[storage] if isinstance(storage, str) else int(storage)
    md = MODELS[eq] if isinstance(eq, str) else int(eq)
    if m2g_form == 1:
        md |= MRTLB_FOOTPRINT_M2G_GRADIENT
    _check(lib().mrtlb_solve_footprint(lattice.h, n, st, md, 1 if has_force else 0, byref(out)))
    return out.value


def _nxyz(shape):
    """Array shape (Ny, Nx) or (Nz, Ny, Nx) -> (nx, ny, nz)."""
    if len(shape) == 2:
        return int(shape[1]), int(shape[0]), 1
    return int(shape[2]), int(shape[1]), int(shape[0])


def population_bytes(lattice, shape, storage="fp32"):
    """Bytes of one population buffer of a solve on this grid and storage."""
    n = (c_int64 * 3)(*_nxyz(shape))
    out = c_size_t()
    st = STORAGES[storage] if isinstance(storage, str) else int(storage)
    _check(lib().mrtlb_population_bytes(lattice.h, n, st, byref(out)))
    return out.value


class Solve:
    """mrtlb_solve on a periodic grid of array shape (Ny, Nx) or (Nz, Ny, Nx)."""

    def __init__(self, ctx, lattice, model, shape, storage="fp32", has_force=False, external=None):
        """``external`` = (f0, f1): two caller-owned device pointers (ints) of
        at least ``population_bytes(lattice, shape, storage)`` each."""
        self.h = None
        self.ctx, self.shape, self.d = ctx, tuple(shape), len(shape)
        self.N = int(np.prod(shape))
        info = lattice.query()
        self.b = info["b"]
        n = (c_int64 * 3)(*_nxyz(shape))
        h = c_void_p()
        st = STORAGES[storage] if isinstance(storage, str) else int(storage)
        if external is None:
            _check(lib().mrtlb_solve_create(ctx.h, lattice.h, byref(model), n, st, 1 if has_force else 0, byref(h)))
        else:
            _check(lib().mrtlb_solve_create_external(ctx.h, lattice.h, byref(model), n, st, 1 if has_force else 0,
                                                     c_void_p(external[0]), c_void_p(external[1]), byref(h)))
        self.h = h
        self.storage = storage
        ctx._solves.add(self)

    def init_fields(self, rho_or_phi, u=None, force=None):
        r, uu, ff = _f64(rho_or_phi), _f64(u), _f64(force)
        _check(lib().mrtlb_init_fields(self.h, _ptr(r), _ptr(uu), _ptr(ff)))

    def set_transform(self, transform):
        """Hermite transforms of the step kernel: "valu" (default) or "mfma"."""
        t = TRANSFORMS[transform] if isinstance(transform, str) else int(transform)
        _check(lib().mrtlb_solve_set_transform(self.h, t))

    def set_velocity_field(self, u):
        """CDE: the velocity field (d, *shape) used from the next step on."""
        _check(lib().mrtlb_set_velocity_field(self.h, _ptr(_f64(u))))

    def set_force_field(self, force):
        """NSE with a force field: the body force (d, *shape) used from the next
        step on (the three-level scheme's difference term uses the previous
        step's force)."""
        _check(lib().mrtlb_set_force_field(self.h, _ptr(_f64(force))))

    def set_mass_source_field(self, S):
        """NSE with a force field: the mass source S(x) (shape of the grid) used
        from the next step on (and by init_fields if set before it)."""
        _check(lib().mrtlb_set_mass_source_field(self.h, _ptr(_f64(S))))

    def step(self, n=1):
        _check(lib().mrtlb_step(self.h, int(n)))

    def step_timed(self, n):
        ms = c_double()
        _check(lib().mrtlb_step_timed(self.h, int(n), byref(ms)))
        return ms.value

    def stream_only(self, n=1, timed=False):
        """n passes of streaming alone (no collision), a measurement aid;
        with ``timed`` returns their device time in ms."""
        if not timed:
            _check(lib().mrtlb_stream_only(self.h, int(n), None))
            return None
        ms = c_double()
        _check(lib().mrtlb_stream_only(self.h, int(n), byref(ms)))
        return ms.value

    def launch_shape(self):
        """The step kernel's launch shape: nodes per lane, tile order
        ("xcd" ranges or "dispatch"), workgroups per CU under the occupancy
        cap (0: uncapped) and workgroups per launch."""
        v, x, w, g = c_int(), c_int(), c_int(), c_int64()
        _check(lib().mrtlb_solve_launch_shape(self.h, byref(v), byref(x), byref(w), byref(g)))
        return {"nodes_per_lane": v.value, "tile_order": "xcd" if x.value else "dispatch",
                "wg_per_cu": w.value, "workgroups": g.value}

    def read_moments(self, with_u=True, out=None):
        """(rho_or_phi, u) as arrays of the grid shape; ``out`` = (r, u) lets
        the caller supply the destination (contiguous float64, e.g. in
        page-locked memory), u may be None."""
        if out is not None:
            r, u = out
            if r.dtype != np.float64 or not r.flags.c_contiguous or r.size != self.N:
                raise ValueError("out[0] must be a contiguous float64 array of N values")
            if u is not None and (u.dtype != np.float64 or not u.flags.c_contiguous or u.size != self.d * self.N):
                raise ValueError("out[1] must be a contiguous float64 array of d*N values")
            with_u = u is not None
        else:
            r = np.empty(self.N)
            u = np.empty(self.d * self.N) if with_u else None
        _check(lib().mrtlb_read_moments(self.h, _ptr(r), _ptr(u)))
        r = r.reshape(self.shape)
        return (r, u.reshape((self.d,) + self.shape)) if with_u else r

    def set_drift_correction(self, every):
        """FP64 check of the conserved totals every ``every`` steps, the
        difference applied on the next step (0 turns it off)."""
        _check(lib().mrtlb_set_drift_correction(self.h, int(every)))

    def conserved(self):
        m = c_double()
        mom = np.zeros(3)
        _check(lib().mrtlb_conserved(self.h, byref(m), _ptr(mom)))
        return m.value, mom[: self.d].copy()

    def conserved_noalloc(self):
        """As conserved(), through the allocation-free entry point."""
        m = c_double()
        mom = np.zeros(3)
        _check(lib().mrtlb_conserved_noalloc(self.h, byref(m), _ptr(mom)))
        return m.value, mom[: self.d].copy()

    def read_populations(self):
        f = np.empty(self.b * self.N)
        _check(lib().mrtlb_read_populations(self.h, _ptr(f)))
        return f.reshape((self.b,) + self.shape)

    def write_populations(self, f):
        ff = _f64(f)
        _check(lib().mrtlb_write_populations(self.h, _ptr(ff)))

    @property
    def steps(self):
        return int(lib().mrtlb_solve_steps(self.h))

    def close(self):
        if self.h:
            if self.ctx.h:
                lib().mrtlb_solve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_step(solves, nsteps):
    """Advance solve i by nsteps[i] (or every solve by the same int)."""
    n = len(solves)
    if isinstance(nsteps, (int, np.integer)):
        nsteps = [int(nsteps)] * n
    arr = (c_void_p * n)(*[s.h for s in solves])
    cnt = (c_int64 * n)(*[int(k) for k in nsteps])
    _check(lib().mrtlb_batch_step(arr, n, cnt))
