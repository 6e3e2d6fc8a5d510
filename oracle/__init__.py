"""FP64 CPU oracle of the linear quasistatic beam-plasma model -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package.  The product (the HIP library and its binding) never does, and this package
never imports the product.  The arithmetic lives in ``qs_oracle.c`` (plain C, FP64), which
follows the paper's per-species equations (Sec. II, Sec. III.D); this module only
marshals numpy arrays through ctypes and builds the C file with gcc when needed.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(HERE, "qs_oracle.c")
_SRC_GRID = os.path.join(HERE, "qs_grid_oracle.c")
_LIB = os.path.join(HERE, "liborc.so")

DROP_LONGITUDINAL = 1
NO_RESTORING = 2
STEADY_INFLOW = 4
STATIONARY_FRONT = 16

SEED_NOISE = 0
SEED_UNIFORM = 1
SEED_FRONT_IMPULSE = 2


def build(force: bool = False) -> str:
    """Compile qs_oracle.c and qs_grid_oracle.c into liborc.so with gcc (-O2, IEEE
    arithmetic, OpenMP)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in (_SRC, _SRC_GRID))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, _SRC_GRID, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Beam(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int),
                ("q", ctypes.POINTER(ctypes.c_double)),
                ("m", ctypes.POINTER(ctypes.c_double)),
                ("nb", ctypes.POINTER(ctypes.c_double)),
                ("gamma", ctypes.c_double),
                ("n_xi", ctypes.c_int),
                ("h", ctypes.c_double),
                ("shape", ctypes.POINTER(ctypes.c_double)),
                ("flags", ctypes.c_int)]


_lib = None

# mistakes the C source can plant (ORC_PLANT_<name>), for checking that the pins catch them
PLANTS = ("EPERP_SIGN", "BPERP_NP", "NONFLUX", "LONG_SIGN", "FACE_INDEX", "TRANS_SIGN")


def build_variant(plant: str, outdir: str | None = None) -> str:
    """Compile a copy of the oracle with one planted mistake (ORC_PLANT_<plant>) into its own
    shared library and return its path; the normal library is untouched."""
    if plant not in PLANTS:
        raise ValueError("unknown plant %r" % plant)
    outdir = outdir or tempfile.mkdtemp(prefix="orc_plant_")
    out = os.path.join(outdir, "liborc_%s.so" % plant.lower())
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-DORC_PLANT_" + plant,
                           "-o", out, _SRC, _SRC_GRID, "-lm"])
    return out


def build_sanitized(outdir: str | None = None) -> str:
    """Compile a copy of the oracle with AddressSanitizer and UndefinedBehaviorSanitizer (gcc;
    undefined behaviour aborts) for running the CPU tests under them; returns its path.  The
    process that loads it needs gcc's libasan first (LD_PRELOAD)."""
    outdir = outdir or tempfile.mkdtemp(prefix="orc_san_")
    out = os.path.join(outdir, "liborc_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                           "-o", out, _SRC, _SRC_GRID, "-lm"])
    return out


@contextlib.contextmanager
def use_library(path: str):
    """Run the oracle's functions on another build of it (e.g. build_variant) inside the block."""
    global _lib
    saved = _lib
    _lib = _declare(ctypes.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def lib():
    """The oracle library: liborc.so (built when stale), or the build named by the
    ORC_LIBRARY environment variable (e.g. build_sanitized's)."""
    global _lib
    if _lib is None:
        _lib = _declare(ctypes.CDLL(os.environ.get("ORC_LIBRARY") or build()))
    return _lib


def _declare(L):
    """Declare the C signatures on a loaded oracle library."""
    D = ctypes.POINTER(ctypes.c_double)
    B = ctypes.POINTER(_Beam)
    L.orc_splitmix64.restype = ctypes.c_uint64
    L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    L.orc_u53.restype = ctypes.c_double
    L.orc_u53.argtypes = [ctypes.c_uint64]
    L.orc_run_modes.restype = ctypes.c_int
    L.orc_run_modes.argtypes = [B, ctypes.c_int, D, ctypes.c_double, ctypes.c_int,
                                ctypes.c_int, D, D, D, D, ctypes.c_int, D, D, D,
                                ctypes.c_int, D]
    L.orc_mode_fields.restype = ctypes.c_int
    L.orc_mode_fields.argtypes = [B, ctypes.c_double, D, D, D, ctypes.c_double,
                                  D, D, D, D, D, D]
    L.orc_march_io.restype = ctypes.c_int
    L.orc_march_io.argtypes = [B, D, D, D, D]
    L.orc_collapse.restype = ctypes.c_int
    L.orc_collapse.argtypes = [B, D, D, D, D, D, D]
    L.orc_seed_mode.restype = ctypes.c_int
    L.orc_seed_mode.argtypes = [B, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                ctypes.c_uint64, D, D, D]
    return L


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Beam:
    """Beam/plasma description in the paper's normalized units.

    species: list of (q, m, nb) with nb the peak unperturbed density over n_p.
    shape: optional longitudinal profile at the cell centres (flat top if None).
    """

    def __init__(self, species, gamma, n_xi, h, shape=None, flags=0):
        self.species = [tuple(float(v) for v in s) for s in species]
        self.q = np.ascontiguousarray([s[0] for s in self.species], dtype=np.float64)
        self.m = np.ascontiguousarray([s[1] for s in self.species], dtype=np.float64)
        self.nb = np.ascontiguousarray([s[2] for s in self.species], dtype=np.float64)
        self.gamma = float(gamma)
        self.n_xi = int(n_xi)
        self.h = float(h)
        self.shape = None if shape is None else np.ascontiguousarray(shape, dtype=np.float64)
        if self.shape is not None and self.shape.shape != (self.n_xi,):
            raise ValueError("shape must have n_xi entries")
        self.flags = int(flags)
        self._c = _Beam(len(self.species), _dp(self.q), _dp(self.m), _dp(self.nb),
                        self.gamma, self.n_xi, self.h, _dp(self.shape), self.flags)

    @property
    def n_species(self):
        return len(self.species)

    def ptr(self):
        return ctypes.byref(self._c)


class ModeState:
    """Per-species state of n_modes modes: complex arrays [n_modes, n_species, n_xi]."""

    def __init__(self, n, pz, pt, log2_scale):
        self.n = np.ascontiguousarray(n, dtype=np.complex128)
        self.pz = np.ascontiguousarray(pz, dtype=np.complex128)
        self.pt = np.ascontiguousarray(pt, dtype=np.complex128)
        self.log2_scale = np.ascontiguousarray(log2_scale, dtype=np.float64)

    @classmethod
    def zeros(cls, n_modes, beam):
        shp = (n_modes, beam.n_species, beam.n_xi)
        return cls(np.zeros(shp, np.complex128), np.zeros(shp, np.complex128),
                   np.zeros(shp, np.complex128), np.zeros(n_modes))

    def copy(self):
        return ModeState(self.n.copy(), self.pz.copy(), self.pt.copy(), self.log2_scale.copy())


def seed(beam, k, kind, amp, rng_seed=0, instance=0, n_modes_total=None, mode_offset=0):
    """Initial state for the modes with wavenumbers k (see orc_seed_mode)."""
    k = np.ascontiguousarray(k, dtype=np.float64).ravel()
    nm = len(k)
    tot = nm if n_modes_total is None else int(n_modes_total)
    st = ModeState.zeros(nm, beam)
    L = lib()
    shp = (beam.n_species, beam.n_xi)
    for m in range(nm):
        n = np.zeros(shp, np.complex128)
        pz = np.zeros(shp, np.complex128)
        pt = np.zeros(shp, np.complex128)
        rc = L.orc_seed_mode(beam.ptr(), int(kind), float(amp), float(k[m]), int(rng_seed),
                             int(instance), int(mode_offset + m), int(tot),
                             _dp(n.view(np.float64)), _dp(pz.view(np.float64)),
                             _dp(pt.view(np.float64)))
        if rc != 0:
            raise ValueError("orc_seed_mode failed (kind=%d, k=%g)" % (kind, k[m]))
        st.n[m], st.pz[m], st.pt[m] = n, pz, pt
    return st


def _front(beam, front, nm):
    if not beam.flags & STATIONARY_FRONT:
        return None
    if front is None:
        raise ValueError("the stationary-front option needs the modes' front values")
    f = np.ascontiguousarray(np.broadcast_to(np.asarray(front, np.complex128), (nm,)))
    return f


def run(beam, k, dtau, n_steps, state, out_every=1, renorm=False, want_fields=True,
        want_max=True, n_threads=0, front=None):
    """Advance `state` in place by n_steps RK4 steps; returns (ln_e, ln_b, max_ln_a).

    ln_e/ln_b: [n_snap, n_xi, n_modes], max_ln_a: [n_steps, n_modes] (None if not wanted).
    front: per mode the value n_p holds ahead of the beam (complex, unscaled), required with
    the STATIONARY_FRONT flag and ignored otherwise.
    """
    k = np.ascontiguousarray(k, dtype=np.float64).ravel()
    nm = len(k)
    if state.n.shape != (nm, beam.n_species, beam.n_xi):
        raise ValueError("state shape mismatch")
    fr = _front(beam, front, nm)
    out_every = max(1, int(out_every))
    n_snap = 1 if n_steps == 0 else -(-n_steps // out_every)
    ln_e = np.empty((n_snap, beam.n_xi, nm)) if want_fields else None
    ln_b = np.empty((n_snap, beam.n_xi, nm)) if want_fields else None
    mx = np.empty((n_steps, nm)) if (want_max and n_steps > 0) else None
    rc = lib().orc_run_modes(beam.ptr(), nm, _dp(k), float(dtau), int(n_steps), out_every,
                             _dp(state.n.view(np.float64)), _dp(state.pz.view(np.float64)),
                             _dp(state.pt.view(np.float64)), _dp(state.log2_scale),
                             1 if renorm else 0, _dp(ln_e), _dp(ln_b), _dp(mx), int(n_threads),
                             None if fr is None else _dp(fr.view(np.float64)))
    if rc != 0:
        raise RuntimeError("orc_run_modes failed")
    return ln_e, ln_b, mx


def mode_fields(beam, k, state, m=0, front=None):
    """Diagnostics of mode m: dict with np (n_p at centres), e_par, ln_e, ln_b, ln_a.
    front: mode m's front value with the STATIONARY_FRONT flag."""
    fr = None
    if beam.flags & STATIONARY_FRONT:
        if front is None:
            raise ValueError("the stationary-front option needs the mode's front value")
        fr = np.array([complex(front).real, complex(front).imag])
    N = beam.n_xi
    npc = np.empty(N, np.complex128)
    epar = np.empty(N, np.complex128)
    ln_e, ln_b, ln_a = np.empty(N), np.empty(N), np.empty(N)
    n = np.ascontiguousarray(state.n[m])
    pz = np.ascontiguousarray(state.pz[m])
    pt = np.ascontiguousarray(state.pt[m])
    rc = lib().orc_mode_fields(beam.ptr(), float(k), _dp(n.view(np.float64)),
                               _dp(pz.view(np.float64)), _dp(pt.view(np.float64)),
                               float(state.log2_scale[m]), _dp(npc.view(np.float64)),
                               _dp(epar.view(np.float64)), _dp(ln_e), _dp(ln_b), _dp(ln_a), _dp(fr))
    if rc != 0:
        raise RuntimeError("orc_mode_fields failed")
    return {"np": npc, "e_par": epar, "ln_e": ln_e, "ln_b": ln_b, "ln_a": ln_a}


def march(beam, rho):
    """One plasma march for the complex cell charge density rho[n_xi]."""
    rho = np.ascontiguousarray(rho, dtype=np.complex128)
    N = beam.n_xi
    a, c, f = (np.empty(N, np.complex128) for _ in range(3))
    rc = lib().orc_march_io(beam.ptr(), _dp(rho.view(np.float64)), _dp(a.view(np.float64)),
                            _dp(c.view(np.float64)), _dp(f.view(np.float64)))
    if rc != 0:
        raise RuntimeError("orc_march_io failed")
    return a, c, f


def collapse(beam, state, m=0):
    """Charge density rho and current densities j_par (faces), j_perp of mode m."""
    N = beam.n_xi
    out = [np.empty(N, np.complex128) for _ in range(3)]
    n = np.ascontiguousarray(state.n[m])
    pz = np.ascontiguousarray(state.pz[m])
    pt = np.ascontiguousarray(state.pt[m])
    lib().orc_collapse(beam.ptr(), _dp(n.view(np.float64)), _dp(pz.view(np.float64)),
                       _dp(pt.view(np.float64)), *[_dp(o.view(np.float64)) for o in out])
    return tuple(out)


def splitmix64(seed, i):
    return int(lib().orc_splitmix64(int(seed) & (2**64 - 1), int(i) & (2**64 - 1)))


def u53(x):
    return float(lib().orc_u53(int(x)))


# ----------------------------------------------------------------------------- finite width
class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("n_xi", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("h", ctypes.c_double),
                ("gamma", ctypes.c_double), ("omega", ctypes.POINTER(ctypes.c_double)),
                ("flags", ctypes.c_int)]


class Grid:
    """A finite-width problem: nx x ny periodic transverse grid over lx x ly, n_xi cells of
    width h, Omega at cell centres [n_xi, ny, nx]."""

    def __init__(self, nx, ny, n_xi, lx, ly, h, gamma, omega, flags=0):
        self.omega = np.ascontiguousarray(omega, np.float64).reshape(n_xi, ny, nx)
        self.nx, self.ny, self.n_xi, self.lx, self.ly, self.h, self.gamma = nx, ny, n_xi, lx, ly, h, gamma
        self.flags = flags
        self.c = _Grid(nx, ny, n_xi, lx, ly, h, gamma, _dp(self.omega), flags)

    @property
    def shape(self):
        return (self.n_xi, self.ny, self.nx)

    def coords(self):
        x = (np.arange(self.nx) - self.nx // 2) * self.lx / self.nx
        y = (np.arange(self.ny) - self.ny // 2) * self.ly / self.ny
        return x, y


def _glib():
    L = lib()
    if not getattr(L, "_grid_ready", False):
        D = ctypes.POINTER(ctypes.c_double)
        G = ctypes.POINTER(_Grid)
        L.ogr_fft2.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.ogr_rates.argtypes = [G, D, D, D, D, D, D, D, D]
        L.ogr_step.argtypes = [G, ctypes.c_double, D, D, D, D]
        L.ogr_fields.argtypes = [G, D, D, D]
        L.ogr_run.argtypes = [G, ctypes.c_double, ctypes.c_int, ctypes.c_int, D, D, D, D, D, D, D]
        L.ogr_seed.argtypes = [G, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, D,
                               ctypes.c_uint64, D]
        L._grid_ready = True
    return L


def fft2(a, inverse=False):
    """The oracle's own 2D FFT of a complex array [ny, nx] (inverse includes 1/(nx ny))."""
    z = np.ascontiguousarray(a, np.complex128).copy()
    _glib().ogr_fft2(z.ctypes.data, z.shape[1], z.shape[0], 1 if inverse else 0)
    return z


class GridState:
    def __init__(self, grid):
        self.rho = np.zeros(grid.shape)
        self.jpar = np.zeros(grid.shape)
        self.jx = np.zeros(grid.shape)
        self.jy = np.zeros(grid.shape)

    def arrays(self):
        return self.rho, self.jpar, self.jx, self.jy


def grid_seed(grid, kind, amp, offset=0.0, sigma_r=0.0, f=None, rng_seed=0):
    st = GridState(grid)
    fa = None if f is None else np.ascontiguousarray(f, np.float64)
    _glib().ogr_seed(ctypes.byref(grid.c), int(kind), amp, offset, sigma_r, _dp(fa) if fa is not None else None,
                     int(rng_seed), _dp(st.rho))
    return st


def grid_rates(grid, st):
    out = GridState(grid)
    _glib().ogr_rates(ctypes.byref(grid.c), *[_dp(a) for a in st.arrays()], *[_dp(a) for a in out.arrays()])
    return out


def grid_fields(grid, rho):
    e2 = np.empty(grid.shape)
    b2 = np.empty(grid.shape)
    _glib().ogr_fields(ctypes.byref(grid.c), _dp(np.ascontiguousarray(rho, np.float64)), _dp(e2), _dp(b2))
    return e2, b2


def grid_run(grid, dtau, n_steps, st, out_every=1, want_fields=True, want_max=True):
    """Advance `st` in place; returns (ln_e, ln_b [n_snap, n_xi, ny, nx], max_ln_a [n_steps])."""
    out_every = max(1, int(out_every))
    n_snap = -(-n_steps // out_every) if n_steps > 0 else 0
    T = grid.n_xi * grid.ny * grid.nx
    ln_e = np.empty((n_snap,) + grid.shape) if want_fields else None
    ln_b = np.empty((n_snap,) + grid.shape) if want_fields else None
    mx = np.empty(n_steps) if want_max else None
    _glib().ogr_run(ctypes.byref(grid.c), dtau, int(n_steps), out_every, *[_dp(a) for a in st.arrays()],
                    _dp(ln_e) if want_fields else None, _dp(ln_b) if want_fields else None,
                    _dp(mx) if want_max else None)
    return ln_e, ln_b, mx
