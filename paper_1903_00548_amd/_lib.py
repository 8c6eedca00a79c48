"""ctypes binding of the qtx C ABI (include/qtx.h).

Argument marshalling only: every step of the solve runs in the HIP
library.  If the library has not been built the loader raises; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_void_p, c_char_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqtx.so")

LEFT, RIGHT = 0, 1
POT_DIAG, POT_LINEAR_FE = 0, 1
FP64, MIXED = 0, 1

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, ESTATE = range(6)
FLAG_DEC_NOTCONV, FLAG_NONFINITE, FLAG_REFINE_NOTCONV = 1, 2, 4


class qtx_c128(ctypes.Structure):
    _fields_ = [("re", c_double), ("im", c_double)]


class qtx_tune(ctypes.Structure):
    _fields_ = [("workgroups_per_cu", c_int), ("panel_width", c_int), ("refine_tiles", c_int)]


TUNE_MAX = 16


class qtx_info(ctypes.Structure):
    _fields_ = [("dec_iters", c_int), ("refine_steps", c_int), ("resid", c_double),
                ("fell_back_fp64", c_int), ("flags", c_int)]


INFO_DTYPE = np.dtype([("dec_iters", np.int32), ("refine_steps", np.int32), ("resid", np.float64),
                       ("fell_back_fp64", np.int32), ("flags", np.int32)], align=True)
assert INFO_DTYPE.itemsize == ctypes.sizeof(qtx_info)

_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "qtx_version": (c_char_p, []),
    "qtx_create": (c_int, [c_int, POINTER(c_void_p)]),
    "qtx_destroy": (None, [c_void_p]),
    "qtx_last_error": (c_char_p, [c_void_p]),
    "qtx_set_stream": (c_int, [c_void_p, c_void_p]),
    "qtx_set_lead": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_double]),
    "qtx_set_device": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "qtx_set_potential": (c_int, [c_void_p, c_void_p, c_int]),
    "qtx_solve": (c_int, [c_void_p, c_void_p, c_int, c_double, c_int, c_void_p, c_void_p, c_void_p]),
    "qtx_solve_device": (c_int, [c_void_p, c_void_p, c_int, c_double, c_int, c_void_p, c_void_p, c_void_p]),
    "qtx_solve_device_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_double, c_int, c_void_p, c_void_p,
                                         c_void_p]),
    "qtx_self_energy": (c_int, [c_void_p, c_void_p, c_int, c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "qtx_problem_create": (c_int, [c_void_p, POINTER(c_void_p)]),
    "qtx_kernel_times": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "qtx_set_option": (c_int, [c_void_p, c_char_p, c_double]),
    "qtx_sigma_cache_stats": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "qtx_bands": (c_int, [c_void_p, c_int, c_void_p, c_int, c_void_p]),
    "qtx_autotune": (c_int, [c_void_p, c_void_p, c_int, c_double, c_int, c_void_p, c_void_p, c_void_p,
                             c_void_p]),
    "qtx_solve_batch": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_double, c_int,
                                c_void_p, c_void_p]),
    "qtx_density_matrix": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_double, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p]),
    "qtx_density_matrix_device": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_double, c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_void_p]),
    "qtx_charge": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_double, c_double, c_double,
                           c_void_p]),
    "qtx_check_layouts": (c_int, [c_char_p, c_int]),
}


def load(path: str = LIB_PATH):
    """Load the HIP library once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"qtx HIP library not built: {path} is missing "
                           "(run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class QtxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qtx status {status}: {msg}")
        self.status = status


def _c128(a, shape):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape != shape:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(c_void_p)


class Context:
    """One solver context bound to a HIP device (see include/qtx.h)."""

    def __init__(self, device: int = 0, _handle=None, _parent=None):
        self.lib = load()
        self._parent = _parent
        if _handle is not None:
            self.h = _handle
        else:
            h = c_void_p()
            st = self.lib.qtx_create(device, ctypes.byref(h))
            if st != OK:
                raise QtxError(st, f"qtx_create(device={device}) failed")
            self.h = h
        self.N = None
        self.m = None

    def _check(self, st, allow_notconv=False):
        if st == OK or (allow_notconv and st == ENOTCONV):
            return st
        raise QtxError(st, self.lib.qtx_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None:
            self.lib.qtx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream_ptr: int):
        self._check(self.lib.qtx_set_stream(self.h, c_void_p(stream_ptr or None)))

    def set_lead(self, side, H00, H01, S00, S01, V=0.0):
        m = np.asarray(H00).shape[0]
        arrs = [_c128(x, (m, m)) for x in (H00, H01, S00, S01)]
        self._check(self.lib.qtx_set_lead(self.h, side, m, *[_ptr(a) for a in arrs], float(V)))
        self.m = m

    def set_device(self, N, m, Hd=None, Hu=None, Sd=None, Su=None):
        if Hd is None:
            self._check(self.lib.qtx_set_device(self.h, N, m, None, None, None, None))
        else:
            a = [_c128(Hd, (N, m, m)), _c128(Hu, (max(N - 1, 0), m, m)),
                 _c128(Sd, (N, m, m)), _c128(Su, (max(N - 1, 0), m, m))]
            self._keep = a
            self._check(self.lib.qtx_set_device(self.h, N, m, _ptr(a[0]), _ptr(a[1]) if N > 1 else None,
                                                _ptr(a[2]), _ptr(a[3]) if N > 1 else None))
        self.N, self.m = N, m

    def set_potential(self, V, mode):
        V = np.ascontiguousarray(V, dtype=np.float64)
        self._check(self.lib.qtx_set_potential(self.h, _ptr(V), int(mode)))

    def solve(self, E, eta, precision=FP64, want_ldos=True):
        """Host arrays in and out: returns T (nE,), ldos (nE, 2, N) or None,
        info (structured array), status (OK or ENOTCONV)."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        nE = E.shape[0]
        T = np.empty(nE)
        ldos = np.empty((nE, 2, self.N)) if (want_ldos and self.N) else None
        info = np.zeros(nE, dtype=INFO_DTYPE)
        st = self.lib.qtx_solve(self.h, _ptr(E), nE, float(eta), int(precision), _ptr(T), _ptr(ldos),
                                _ptr(info))
        st = self._check(st, allow_notconv=True)
        return T, ldos, info, st

    def solve_device(self, E_ptr, nE, eta, precision, T_ptr, ldos_ptr=0, info_ptr=0):
        """Device pointers (e.g. torch tensor data_ptr()); enqueued on the
        context stream."""
        st = self.lib.qtx_solve_device(self.h, c_void_p(E_ptr), int(nE), float(eta), int(precision),
                                       c_void_p(T_ptr), c_void_p(ldos_ptr or None),
                                       c_void_p(info_ptr or None))
        return self._check(st, allow_notconv=True)

    def solve_device_noalloc(self, E_ptr, nE, eta, precision, T_ptr, ldos_ptr=0, info_ptr=0):
        """qtx_solve_device_noalloc: as solve_device, with every buffer of
        the solve taken from the library's fixed device scratch."""
        st = self.lib.qtx_solve_device_noalloc(self.h, c_void_p(E_ptr), int(nE), float(eta), int(precision),
                                               c_void_p(T_ptr), c_void_p(ldos_ptr or None),
                                               c_void_p(info_ptr or None))
        return self._check(st, allow_notconv=True)

    def density_matrix(self, E, wL, wR, eta, want_ldos=False):
        """Energy-weighted density-matrix blocks (see qtx_density_matrix):
        rho_diag (N, m, m), rho_off (N-1, m, m), T (nE,), ldos (nE, 2, N)
        or None, info, status."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        nE = E.shape[0]
        wL = np.ascontiguousarray(np.broadcast_to(np.asarray(wL, dtype=np.float64), (nE,)))
        wR = np.ascontiguousarray(np.broadcast_to(np.asarray(wR, dtype=np.float64), (nE,)))
        N, m = self.N, self.m
        rd = np.empty((N, m, m), dtype=np.complex128)
        ro = np.empty((max(N - 1, 0), m, m), dtype=np.complex128)
        T = np.empty(nE)
        ldos = np.empty((nE, 2, N)) if want_ldos else None
        info = np.zeros(nE, dtype=INFO_DTYPE)
        st = self.lib.qtx_density_matrix(self.h, _ptr(E), _ptr(wL), _ptr(wR), nE, float(eta), _ptr(rd),
                                         _ptr(ro) if N > 1 else None, _ptr(T), _ptr(ldos), _ptr(info))
        st = self._check(st, allow_notconv=True)
        return rd, ro, T, ldos, info, st

    def density_matrix_device(self, E_ptr, wL_ptr, wR_ptr, nE, eta, rho_d_ptr, rho_o_ptr, T_ptr, ldos_ptr=0,
                              info_ptr=0):
        """Device pointers (e.g. torch tensor data_ptr()); enqueued on the
        context stream."""
        st = self.lib.qtx_density_matrix_device(self.h, c_void_p(E_ptr), c_void_p(wL_ptr), c_void_p(wR_ptr), int(nE),
                                                float(eta), c_void_p(rho_d_ptr), c_void_p(rho_o_ptr or None),
                                                c_void_p(T_ptr), c_void_p(ldos_ptr or None),
                                                c_void_p(info_ptr or None))
        return self._check(st, allow_notconv=True)

    def self_energy(self, E, eta):
        """Sigma (nE, 2, m, m), W (nE, 2, m, m), signs (nE, 2, m), iters (nE,)."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        nE, m = E.shape[0], self.m
        sig = np.empty((nE, 2, m, m), dtype=np.complex128)
        W = np.empty((nE, 2, m, m), dtype=np.complex128)
        s = np.empty((nE, 2, m))
        it = np.empty(nE, dtype=np.int32)
        st = self.lib.qtx_self_energy(self.h, _ptr(E), nE, float(eta), _ptr(sig), _ptr(W), _ptr(s), _ptr(it))
        self._check(st, allow_notconv=True)
        return sig, W, s, it

    def kernel_times(self, enable=True):
        """(decimate_ms, sweep_ms, sweep_launches) accumulated since the
        previous call; enable=True keeps recording for later solves."""
        d, s_, n = c_double(), c_double(), c_int()
        self._check(self.lib.qtx_kernel_times(self.h, int(enable), ctypes.byref(d), ctypes.byref(s_),
                                              ctypes.byref(n)))
        return d.value, s_.value, n.value

    def set_option(self, name: str, value: float):
        self._check(self.lib.qtx_set_option(self.h, name.encode(), float(value)))

    def autotune(self, E, eta, precision=FP64):
        """Pick the sweep's launch and tile shapes for this problem from
        timed solves of the sample energies (median of three per
        candidate).  Returns (best, candidates, times_ms): best and each
        candidate a dict with workgroups_per_cu, panel_width and
        refine_tiles."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        best = qtx_tune()
        cand = (qtx_tune * TUNE_MAX)()
        times = np.zeros(TUNE_MAX)
        n = c_int()
        self._check(self.lib.qtx_autotune(self.h, _ptr(E), len(E), float(eta), int(precision), ctypes.byref(best),
                                          cand, _ptr(times), ctypes.byref(n)))
        as_dict = lambda t: {"workgroups_per_cu": t.workgroups_per_cu, "panel_width": t.panel_width,
                             "refine_tiles": t.refine_tiles}
        return as_dict(best), [as_dict(cand[k]) for k in range(n.value)], times[:n.value].copy()

    def bands(self, side, k):
        """Band energies E_n(k) + V_lead of one lead, shape (len(k), m)."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        E = np.empty((len(k), self.m))
        self._check(self.lib.qtx_bands(self.h, int(side), _ptr(k), len(k), _ptr(E)))
        return E

    def sigma_cache_stats(self):
        """(hits, misses, entries) of the batch self-energy cache."""
        h, m_, n = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
        self._check(self.lib.qtx_sigma_cache_stats(self.h, ctypes.byref(h), ctypes.byref(m_), ctypes.byref(n)))
        return h.value, m_.value, n.value

    def problem(self):
        h = c_void_p()
        self._check(self.lib.qtx_problem_create(self.h, ctypes.byref(h)))
        return Context(_handle=h, _parent=self)


def solve_batch(ctx: Context, problems, energies, eta, precision=FP64, want_ldos=True):
    """Batched solve of several problems (each its own Context from
    ctx.problem()) on their own energy grids."""
    n = len(problems)
    Es = [np.ascontiguousarray(e, dtype=np.float64) for e in energies]
    Ts = [np.empty(len(e)) for e in Es]
    Ls = [np.empty((len(e), 2, p.N or 0)) for e, p in zip(Es, problems)] if want_ldos else None
    hp = (c_void_p * n)(*[p.h for p in problems])
    Ep = (c_void_p * n)(*[_ptr(e) for e in Es])
    nEp = (c_int * n)(*[len(e) for e in Es])
    Tp = (c_void_p * n)(*[_ptr(t) for t in Ts])
    Lp = (c_void_p * n)(*[_ptr(x) for x in Ls]) if want_ldos else None
    st = ctx.lib.qtx_solve_batch(ctx.h, n, hp, Ep, nEp, float(eta), int(precision), Tp, Lp)
    ctx._check(st, allow_notconv=True)
    return Ts, Ls, st


def charge(ldos, w, E, muL, muR, kT):
    """qtx_charge: Fermi-weighted slab charge sum_k w_k (f_L n^L + f_R n^R)
    of densities ldos (nE, 2, N) at energies E with weights w."""
    lib = load()
    ldos = np.ascontiguousarray(ldos, dtype=np.float64)
    nE, _, N = ldos.shape
    w = np.ascontiguousarray(w, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    out = np.empty(N)
    st = lib.qtx_charge(_ptr(ldos), _ptr(w), nE, N, _ptr(E), float(muL), float(muR), float(kT), _ptr(out))
    if st != OK:
        raise QtxError(st, "qtx_charge")
    return out


def context_for(dev, device: int = 0) -> Context:
    """A context loaded with one transport problem (workloads.Device)."""
    ctx = Context(device)
    fill(ctx, dev)
    return ctx


def fill(ctx: Context, dev):
    L, R = dev.lead_L, dev.lead_R
    ctx.set_lead(LEFT, L.H00, L.H01, L.S00, L.S01, L.V)
    ctx.set_lead(RIGHT, R.H00, R.H01, R.S00, R.S01, R.V)
    if dev.uniform:
        ctx.set_device(dev.N, dev.m)
    else:
        ctx.set_device(dev.N, dev.m, dev.Hd, dev.Hu, dev.Sd, dev.Su)
    ctx.set_potential(dev.V, dev.pot_mode)
    return ctx
