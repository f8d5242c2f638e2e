"""Plain FP64 CPU oracle for the multiphase lattice Boltzmann step of
arXiv 2101.06769 (Sec. 2.2 phase field, Sec. 2.3 flow; Appendix A Hermite
terms).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library and never imports it.

Arrays are numpy float64.  Populations use this oracle's own velocity ordering
(``lattice(dim)``) and the layout [Q][nz][ny][nx] (x fastest); the state is the
pre-collision population set at time n.  Vector fields are [3][nz][ny][nx].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_WALL, BC_SYMMETRY = 0, 1, 2
COLL_CUMULANT, COLL_SRT = 0, 1
DIAG_SIZE = 320
# offsets into the diag vector written by collide_cell
D = dict(u=0, rho=3, P=4, pstar=5, omega=6, mu=7, F=8, n=11, taubar_phi=14, Xi=16, h=48,
         Pi=80, K=112, Kstar=144, Pistar=176, hstar=208, geq=240, Sbar=272)


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("bc", ctypes.c_int * 3),
        ("rho_h", ctypes.c_double),
        ("rho_l", ctypes.c_double),
        ("nu_h", ctypes.c_double),
        ("nu_l", ctypes.c_double),
        ("W", ctypes.c_double),
        ("M", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("visc_interp", ctypes.c_int),
        ("collision", ctypes.c_int),
        ("rate_bulk", ctypes.c_double),
        ("rate3", ctypes.c_double),
        ("rate4", ctypes.c_double),
        ("rate5", ctypes.c_double),
        ("rate6", ctypes.c_double),
        ("cac_edf", ctypes.c_int),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "oracle.h"))):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Params)
        lib.orc_Q.argtypes = [ctypes.c_int]
        lib.orc_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp,
                                    ctypes.POINTER(ctypes.c_int)]
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_gradients.argtypes = [pp, dp, dp, dp]
        lib.orc_init.argtypes = [pp, dp, dp, dp, dp, dp]
        lib.orc_step.argtypes = [pp, dp, dp, dp, dp]
        lib.orc_step_hist.argtypes = [pp, dp, dp, dp, dp, dp, ctypes.c_int]
        lib.orc_step_sampled.argtypes = [pp, dp, dp, ctypes.POINTER(ctypes.c_long), ctypes.c_long,
                                         dp, dp]
        lib.orc_fields.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        lib.orc_reduce.argtypes = [pp, dp, dp, dp]
        lib.orc_collide_cell.argtypes = [pp, dp, dp, ctypes.c_double, dp, ctypes.c_double, dp, dp,
                                         dp, dp, dp]
        lib.orc_central_moments.argtypes = [ctypes.c_int, dp, dp, dp]
        lib.orc_cumulants_from_central.argtypes = [ctypes.c_int, dp, dp]
        lib.orc_central_from_cumulants.argtypes = [ctypes.c_int, dp, dp]
        lib.orc_populations_from_central.argtypes = [ctypes.c_int, dp, dp, dp]
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(dim, n, bc=(0, 0, 0), rho_h=1.0, rho_l=1.0, nu_h=0.1, nu_l=None, W=4.0, M=0.1,
                sigma=0.0, g=(0.0, 0.0, 0.0), visc_interp=0, collision=COLL_CUMULANT,
                rate_bulk=1.0, rate3=1.0, rate4=1.0, rate5=1.0, rate6=1.0, cac_edf=0) -> Params:
    p = Params()
    p.dim = dim
    nn = list(n) + [1] * (3 - len(n))
    for i in range(3):
        p.n[i] = int(nn[i])
        p.bc[i] = int(bc[i]) if i < len(bc) else 0
        p.g[i] = float(g[i]) if i < len(g) else 0.0
    p.rho_h, p.rho_l = float(rho_h), float(rho_l)
    p.nu_h = float(nu_h)
    p.nu_l = float(nu_h if nu_l is None else nu_l)
    p.W, p.M, p.sigma = float(W), float(M), float(sigma)
    p.visc_interp, p.collision = int(visc_interp), int(collision)
    p.rate_bulk, p.rate3, p.rate4, p.rate5, p.rate6 = map(float, (rate_bulk, rate3, rate4, rate5,
                                                                  rate6))
    p.cac_edf = int(cac_edf)
    return p


def params_from_dict(d: dict) -> Params:
    """Build oracle parameters from a plain case dictionary (keys as in make_params)."""
    keys = ("dim", "n", "bc", "rho_h", "rho_l", "nu_h", "nu_l", "W", "M", "sigma", "g",
            "visc_interp", "collision", "rate_bulk", "rate3", "rate4", "rate5", "rate6",
            "cac_edf")
    return make_params(**{k: d[k] for k in keys if k in d})


def Q(dim):
    return _load().orc_Q(dim)


def lattice(dim):
    """(c[Q,3] int, w[Q], opp[Q]) in the oracle's ordering."""
    q = Q(dim)
    c = (ctypes.c_int * (3 * q))()
    w = np.zeros(q)
    opp = (ctypes.c_int * q)()
    _load().orc_lattice(dim, c, _ptr(w), opp)
    return np.array(list(c)).reshape(q, 3), w, np.array(list(opp))


def set_threads(n: int):
    _load().orc_set_threads(int(n))


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().orc_num_threads())


def ncells(p: Params) -> int:
    return p.n[0] * p.n[1] * p.n[2]


def _shape(p):
    return (p.n[2], p.n[1], p.n[0])


def gradients(p: Params, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    grad = np.zeros((3,) + _shape(p))
    lap = np.zeros(_shape(p))
    _check(_load().orc_gradients(ctypes.byref(p), _ptr(phi), _ptr(grad), _ptr(lap)))
    return grad, lap


def init(p: Params, phi, u, ph):
    q = Q(p.dim)
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(_shape(p))
    u = np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + _shape(p))
    ph = np.ascontiguousarray(ph, dtype=np.float64).reshape(_shape(p))
    f = np.zeros((q,) + _shape(p))
    g = np.zeros((q,) + _shape(p))
    _check(_load().orc_init(ctypes.byref(p), _ptr(phi), _ptr(u), _ptr(ph), _ptr(f), _ptr(g)))
    return f, g


def step(p: Params, f, g, nsteps: int = 1):
    """nsteps steps from (f, g).  With the first-order phase-field equilibrium
    the first step has no (phi u) history (zero time derivative) and later
    steps carry it."""
    f, g, _ = step_hist(p, f, g, nsteps, None)
    return f, g


def step_hist(p: Params, f, g, nsteps: int = 1, phiu=None):
    """As step, with the (phi u) history: phiu ([3][nz][ny][nx], or None for
    no history) is that of the step before (f, g); returns (f, g, phiu)."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    g = np.array(g, dtype=np.float64, order="C", copy=True)
    fo = np.empty_like(f)
    go = np.empty_like(g)
    have = phiu is not None
    h = (np.array(phiu, dtype=np.float64, order="C", copy=True) if have
         else np.zeros((3,) + _shape(p)))
    for _ in range(nsteps):
        _check(_load().orc_step_hist(ctypes.byref(p), _ptr(f), _ptr(g), _ptr(fo), _ptr(go),
                                     _ptr(h), 1 if have else 0))
        have = True
        f, fo = fo, f
        g, go = go, g
    return f, g, h


def step_sampled(p: Params, f, g, cells):
    q = Q(p.dim)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    m = cells.size
    fo = np.zeros((m, q))
    go = np.zeros((m, q))
    _check(_load().orc_step_sampled(ctypes.byref(p), _ptr(np.ascontiguousarray(f)),
                                    _ptr(np.ascontiguousarray(g)),
                                    cells.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), m,
                                    _ptr(fo), _ptr(go)))
    return fo, go


def fields(p: Params, f, g):
    phi = np.zeros(_shape(p))
    rho = np.zeros(_shape(p))
    u = np.zeros((3,) + _shape(p))
    ph = np.zeros(_shape(p))
    _check(_load().orc_fields(ctypes.byref(p), _ptr(np.ascontiguousarray(f)),
                              _ptr(np.ascontiguousarray(g)), _ptr(phi), _ptr(rho), _ptr(u),
                              _ptr(ph)))
    return dict(phi=phi, rho=rho, u=u, p=ph)


def reduce(p: Params, f, g):
    out = np.zeros(5)
    _check(_load().orc_reduce(ctypes.byref(p), _ptr(np.ascontiguousarray(f)),
                              _ptr(np.ascontiguousarray(g)), _ptr(out)))
    return out


def collide_cell(p: Params, f, g, phi, grad, lap, phiu_prev=None):
    """One cell's collision; phiu_prev is the cell's (phi u) of the previous
    step for the first-order phase-field equilibrium (None: no history)."""
    q = Q(p.dim)
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    gr = np.zeros(3)
    gr[:len(grad)] = grad
    fo = np.zeros(q)
    go = np.zeros(q)
    dg = np.zeros(DIAG_SIZE)
    prev = None if phiu_prev is None else np.ascontiguousarray(phiu_prev, dtype=np.float64)
    out = np.zeros(3)
    _check(_load().orc_collide_cell(ctypes.byref(p), _ptr(f), _ptr(g), float(phi), _ptr(gr),
                                    float(lap), _ptr(fo), _ptr(go), _ptr(dg), _ptr(prev),
                                    _ptr(out)))
    return fo, go, dg


def central_moments(dim, h, u):
    out = np.zeros(27)
    uu = np.zeros(3)
    uu[:len(u)] = u
    _load().orc_central_moments(dim, _ptr(np.ascontiguousarray(h, dtype=np.float64)), _ptr(uu),
                                _ptr(out))
    return out


def cumulants_from_central(dim, Pi):
    K = np.zeros(27)
    _load().orc_cumulants_from_central(dim, _ptr(np.ascontiguousarray(Pi, dtype=np.float64)),
                                       _ptr(K))
    return K


def central_from_cumulants(dim, K):
    Pi = np.zeros(27)
    _load().orc_central_from_cumulants(dim, _ptr(np.ascontiguousarray(K, dtype=np.float64)),
                                       _ptr(Pi))
    return Pi


def populations_from_central(dim, Pi, u):
    h = np.zeros(Q(dim))
    uu = np.zeros(3)
    uu[:len(u)] = u
    _check(_load().orc_populations_from_central(dim, _ptr(np.ascontiguousarray(Pi,
                                                                               dtype=np.float64)),
                                                _ptr(uu), _ptr(h)))
    return h


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle call failed with status %d" % rc)
