"""Seeded synthetic inputs: case parameters and initial fields.

This module maps the paper's dimensionless set-ups (Sec. 3) to lattice-unit
parameters and produces the initial order parameter, velocity and pressure
fields.  It contains none of the lattice Boltzmann arithmetic: the GPU library
and the CPU oracle each turn these fields into populations on their own.

Conventions
-----------
* Lattice units, heavy density 1 (Sec. 3 preamble).
* Fields are numpy float64 arrays shaped (nz, ny, nx) (x fastest); velocity is
  (3, nz, ny, nx).  In 2-D nz = 1.
* ``params`` dictionaries use the keys dim, n, bc, rho_h, rho_l, nu_h, nu_l,
  W, M, sigma, g (plus optional visc_interp, collision).
* Initial interfaces use the flat-interface profile phi = (1 + tanh(2 d / W))/2
  with d the signed distance (positive inside the heavy phase), the exact 1-D
  steady state of the conservative Allen-Cahn equation (Sec. 2.1).
* Rayleigh-Taylor scaling keeps U* = sqrt(g L) = 0.06, which reproduces both
  parameter sets the paper prints (Sec. 3.2: L = 600, g = 6e-6, nu = 0.1406 /
  0.0176 for Re = 256 / 2048; Sec. 3.3: L = 100, g = 3.6e-5, nu = 0.006).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BC_PERIODIC, BC_WALL, BC_SYMMETRY = 0, 1, 2
U_STAR = 0.06


@dataclasses.dataclass
class Case:
    name: str
    params: dict
    phi: np.ndarray
    u: np.ndarray
    p: np.ndarray
    steps: int
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def ncells(self) -> int:
        n = self.params["n"]
        return int(n[0] * n[1] * n[2])


def interface_profile(d, W):
    """Order parameter at signed distance d from the phi = 1/2 iso-surface."""
    return 0.5 * (1.0 + np.tanh(2.0 * np.asarray(d, dtype=np.float64) / W))


def atwood_to_rho_light(At, rho_h=1.0):
    """At = (rho_h - rho_l)/(rho_h + rho_l) (Sec. 3.2)."""
    return rho_h * (1.0 - At) / (1.0 + At)


def rti_parameters(L, Re, Ustar=U_STAR):
    """Gravity and viscosity for a Rayleigh-Taylor run: U* = sqrt(g L),
    Re = rho_h U* L / mu_h with rho_h = 1 (Sec. 3.2)."""
    g = Ustar * Ustar / L
    nu = Ustar * L / Re
    return g, nu


def impact_parameter(We, Re):
    """K = We^(1/2) Re^(1/4) (Sec. 3.4)."""
    return math.sqrt(We) * Re ** 0.25


def splash_parameters(D, U0, Re, We, nu_ratio=15.0, rho_ratio=1000.0, rho_h=1.0):
    """Droplet impact: Re = rho_h U0 D / mu_h; We = rho_h D U0^2 / sigma
    (liquid density); nu_l = nu_ratio nu_h; rho_l = rho_h / rho_ratio."""
    nu_h = U0 * D / Re
    return dict(nu_h=nu_h, nu_l=nu_ratio * nu_h, sigma=rho_h * D * U0 * U0 / We,
                rho_l=rho_h / rho_ratio)


def hydrostatic_pressure(phi, params):
    """Pressure in hydrostatic balance with the body force, dp/dx_i = rho g_i
    along the gravity axis, integrated column by column with the trapezoid
    rule (unit spacing) and shifted to zero mean.  rho = rho_l + (rho_h -
    rho_l) phi (Sec. 2.3).  Used as the initial pressure of gravity-driven
    cases so that runs start from rest instead of from a free fall."""
    g = params["g"]
    axis = int(np.argmax(np.abs(g)))
    if g[axis] == 0.0:
        return np.zeros_like(phi)
    rho = params["rho_l"] + (params["rho_h"] - params["rho_l"]) * phi
    ax = 2 - axis  # array axes are (z, y, x)
    r = np.moveaxis(rho, ax, 0)
    p = np.zeros_like(r)
    p[1:] = np.cumsum(0.5 * (r[1:] + r[:-1]) * g[axis], axis=0)
    p = np.moveaxis(p, 0, ax)
    return p - p.mean()


def _zeros(n):
    nx, ny, nz = n
    return np.zeros((nz, ny, nx)), np.zeros((3, nz, ny, nx))


def rti2d(nx=64, ny=256, At=0.5, Re=256.0, W=4.0, M=0.1, amp=3.0, steps=2000):
    """2-D Rayleigh-Taylor: heavy fluid on top, interface
    y = ny/2 + amp cos(2 pi x / nx), periodic in x, walls at y (Sec. 3.2)."""
    g, nu = rti_parameters(nx, Re)
    n = (nx, ny, 1)
    params = dict(dim=2, n=n, bc=(BC_PERIODIC, BC_WALL, BC_PERIODIC), rho_h=1.0,
                  rho_l=atwood_to_rho_light(At), nu_h=nu, nu_l=nu, W=W, M=M, sigma=0.0,
                  g=(0.0, -g, 0.0))
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    h = ny / 2.0 + amp * np.cos(2.0 * np.pi * x / nx)
    phi = interface_profile(y[:, None] - h[None, :], W)[None]
    _, u = _zeros(n)
    p = hydrostatic_pressure(phi, params)
    return Case("rti2d", params, phi, u, p, steps,
                dict(At=At, Re=Re, T=nx / U_STAR, L=nx, g=g))


def rti3d(nx=128, ny=128, nz=512, At=0.5, Re=1000.0, W=5.0, M=0.1, amp=0.05 * 128,
          steps=20000):
    """3-D Rayleigh-Taylor: interface z = nz/2 + amp [cos(2 pi x/L) + cos(2 pi y/L)],
    periodic in x and y, walls at z (Sec. 3.3)."""
    g, nu = rti_parameters(nx, Re)
    n = (nx, ny, nz)
    params = dict(dim=3, n=n, bc=(BC_PERIODIC, BC_PERIODIC, BC_WALL), rho_h=1.0,
                  rho_l=atwood_to_rho_light(At), nu_h=nu, nu_l=nu, W=W, M=M, sigma=0.0,
                  g=(0.0, 0.0, -g))
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    z = np.arange(nz, dtype=np.float64)
    h = nz / 2.0 + amp * (np.cos(2.0 * np.pi * x[None, :] / nx) +
                          np.cos(2.0 * np.pi * y[:, None] / ny))
    phi = interface_profile(z[:, None, None] - h[None, :, :], W)
    _, u = _zeros(n)
    p = hydrostatic_pressure(phi, params)
    return Case("rti3d", params, phi, u, p, steps,
                dict(At=At, Re=Re, T=nx / U_STAR, L=nx, g=g))


def rti3d_multimode(edge, At, Re, seed, W=5.0, M=0.1, rms=0.02, kmax=4, steps=1000):
    """3-D Rayleigh-Taylor box edge x edge x 4 edge with a seeded random-phase
    multimode interface: all modes 1 <= |k| <= kmax at equal amplitude, total
    RMS displacement rms * edge."""
    nx = ny = int(edge)
    nz = 4 * int(edge)
    g, nu = rti_parameters(nx, Re)
    rng = np.random.default_rng(seed)
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    modes = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(0, kmax + 1)
             if 1.0 <= math.hypot(kx, ky) <= kmax and (ky > 0 or kx > 0)]
    h = np.zeros((ny, nx))
    for kx, ky in modes:
        ph = rng.uniform(0.0, 2.0 * np.pi)
        h += np.cos(2.0 * np.pi * (kx * x[None, :] + ky * y[:, None]) / nx + ph)
    h *= rms * edge / max(np.sqrt(np.mean(h * h)), 1e-30)
    h += nz / 2.0
    z = np.arange(nz, dtype=np.float64)
    phi = interface_profile(z[:, None, None] - h[None, :, :], W)
    n = (nx, ny, nz)
    params = dict(dim=3, n=n, bc=(BC_PERIODIC, BC_PERIODIC, BC_WALL), rho_h=1.0,
                  rho_l=atwood_to_rho_light(At), nu_h=nu, nu_l=nu, W=W, M=M, sigma=0.0,
                  g=(0.0, 0.0, -g))
    _, u = _zeros(n)
    p = hydrostatic_pressure(phi, params)
    return Case("rti3d_multimode", params, phi, u, p, steps,
                dict(At=At, Re=Re, edge=edge, seed=seed))


def batch_rti3d(count=64, seed=0, edges=(32, 48, 64, 96, 128), At_range=(0.1, 0.9),
                Re_range=(100.0, 3000.0), steps=1000):
    """Independent 3-D Rayleigh-Taylor domains of uneven size (edge drawn from
    ``edges``, z = 4 edge), Atwood and Reynolds numbers uniform in their ranges."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        edge = int(rng.choice(edges))
        At = float(rng.uniform(*At_range))
        Re = float(rng.uniform(*Re_range))
        specs.append(dict(edge=edge, At=At, Re=Re, seed=int(seed * 100003 + i)))
    return [rti3d_multimode(s["edge"], s["At"], s["Re"], s["seed"], steps=steps) for s in specs]


def splash3d(nx=512, ny=512, nz=256, D=64.0, U0=0.05, Re=1000.0, We=8000.0, W=5.0, M=0.1,
             sheet=None, steps=10000):
    """3-D droplet impact on a thin liquid sheet (Sec. 3.4): sheet of depth
    0.1 D on the bottom wall, drop of diameter D centred W above the sheet,
    moving down at U0; walls at z, periodic in x and y, no gravity."""
    sp = splash_parameters(D, U0, Re, We)
    sheet = 0.1 * D if sheet is None else sheet
    n = (nx, ny, nz)
    params = dict(dim=3, n=n, bc=(BC_PERIODIC, BC_PERIODIC, BC_WALL), rho_h=1.0,
                  rho_l=sp["rho_l"], nu_h=sp["nu_h"], nu_l=sp["nu_l"], W=W, M=M,
                  sigma=sp["sigma"], g=(0.0, 0.0, 0.0))
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    zc = sheet + D / 2.0 + W
    r = np.sqrt((x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2 + (z - zc) ** 2)
    phi_drop = interface_profile(D / 2.0 - r, W)
    phi_sheet = interface_profile(sheet - z, W) * np.ones_like(phi_drop)
    phi = np.maximum(phi_drop, phi_sheet)
    p, u = _zeros(n)
    u[2] = -U0 * phi_drop
    return Case("splash3d", params, phi, u, p, steps,
                dict(D=D, U0=U0, Re=Re, We=We, K=impact_parameter(We, Re), T=D / U0))


def static_droplet(dim=2, n=(64, 64, 1), R=12.0, sigma=1e-3, rho_ratio=20.0, nu=0.1, W=4.0,
                   M=0.1, steps=3000):
    """Heavy droplet of radius R at the centre of a fully periodic box of light
    fluid (Sec. 3.1)."""
    n = tuple(n) + (1,) * (3 - len(n))
    params = dict(dim=dim, n=n, bc=(BC_PERIODIC,) * 3, rho_h=1.0, rho_l=1.0 / rho_ratio,
                  nu_h=nu, nu_l=nu, W=W, M=M, sigma=sigma, g=(0.0, 0.0, 0.0))
    nx, ny, nz = n
    x = np.arange(nx, dtype=np.float64)[None, None, :] - (nx - 1) / 2.0
    y = np.arange(ny, dtype=np.float64)[None, :, None] - (ny - 1) / 2.0
    z = np.arange(nz, dtype=np.float64)[:, None, None] - ((nz - 1) / 2.0 if dim == 3 else 0.0)
    r = np.sqrt(x * x + y * y + z * z)
    phi = interface_profile(R - r, W) * np.ones((nz, ny, nx))
    p, u = _zeros(n)
    return Case("static_droplet", params, phi, u, p, steps, dict(R=R, sigma=sigma))


def impacting_droplet2d(n=256, D=None, U0=0.05, Re=200.0, We=220.0, W=4.0, M=0.1, steps=2000,
                        rho_ratio=1000.0):
    """2-D droplet impact on a liquid sheet in an n x n box: walls top and
    bottom, periodic sides, sheet of depth 0.1 D."""
    D = n / 8.0 if D is None else D
    sp = splash_parameters(D, U0, Re, We, rho_ratio=rho_ratio)
    params = dict(dim=2, n=(n, n, 1), bc=(BC_PERIODIC, BC_WALL, BC_PERIODIC), rho_h=1.0,
                  rho_l=sp["rho_l"], nu_h=sp["nu_h"], nu_l=sp["nu_l"], W=W, M=M,
                  sigma=sp["sigma"], g=(0.0, 0.0, 0.0))
    x = np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(n, dtype=np.float64)[:, None]
    sheet = 0.1 * D
    yc = sheet + D / 2.0 + W
    r = np.sqrt((x - n / 2.0) ** 2 + (y - yc) ** 2)
    phi_drop = interface_profile(D / 2.0 - r, W)
    phi = np.maximum(phi_drop, interface_profile(sheet - y, W) * np.ones_like(phi_drop))[None]
    p, u = _zeros((n, n, 1))
    u[1, 0] = -U0 * phi_drop
    return Case("impacting_droplet2d", params, phi, u, p, steps,
                dict(D=D, U0=U0, Re=Re, We=We, K=impact_parameter(We, Re)))


def splash2d(D=100.0, Re=200.0, We=220.0, U0=0.05, nx=None, ny=None, W=5.0, M=0.1, sheet=None,
             rho_ratio=1000.0, nu_ratio=15.0, steps=4000):
    """2-D droplet impact on a liquid film (Sec. 3.4): walls at the top and
    bottom, symmetry planes left and right, film of depth 0.1 D on the
    bottom wall, drop of diameter D centred on the box axis W above the film
    and moving down at U0; density ratio 1000, viscosity ratio 15.  Box
    8 D x 4 D unless given, interface width W = 5 and mobility M = 0.1 (the
    paper states none of the three; at W = 4 the Re 1000, We 2200 case
    diverges at impact, where the gas squeezed out between drop and film
    reaches five times the impact velocity)."""
    nx = int(8 * D) if nx is None else int(nx)
    ny = int(4 * D) if ny is None else int(ny)
    sp = splash_parameters(D, U0, Re, We, nu_ratio=nu_ratio, rho_ratio=rho_ratio)
    params = dict(dim=2, n=(nx, ny, 1), bc=(BC_SYMMETRY, BC_WALL, BC_PERIODIC), rho_h=1.0,
                  rho_l=sp["rho_l"], nu_h=sp["nu_h"], nu_l=sp["nu_l"], W=W, M=M,
                  sigma=sp["sigma"], g=(0.0, 0.0, 0.0))
    sheet = 0.1 * D if sheet is None else sheet
    xc = nx / 2.0
    x = np.arange(nx, dtype=np.float64)[None, :] + 0.5  # cell centres, symmetric about xc
    y = np.arange(ny, dtype=np.float64)[:, None]
    yc = sheet + D / 2.0 + W
    r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    phi_drop = interface_profile(D / 2.0 - r, W)
    phi = np.maximum(phi_drop, interface_profile(sheet - y, W) * np.ones_like(phi_drop))[None]
    p, u = _zeros((nx, ny, 1))
    u[1, 0] = -U0 * phi_drop
    return Case("splash2d", params, phi, u, p, steps,
                dict(D=D, U0=U0, Re=Re, We=We, K=impact_parameter(We, Re), T=D / U0,
                     sheet=sheet, x_axis=xc - 0.5))


def random_state(params, seed, u_amp=0.04, p_amp=1e-3, modes=3):
    """Smooth seeded random fields: phi in (0, 1) built from a few random
    Fourier modes passed through the interface profile, small random velocity
    and pressure.  Returns (phi, u, p)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = params["n"]
    dim = params["dim"]
    coords = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    zz, yy, xx = [c.astype(np.float64) for c in coords]

    def smooth():
        s = np.zeros((nz, ny, nx))
        for _ in range(modes):
            k = [rng.integers(1, 3) for _ in range(3)]
            ph = rng.uniform(0, 2 * np.pi, 3)
            a = rng.uniform(0.5, 1.0)
            term = np.cos(2 * np.pi * k[0] * xx / nx + ph[0]) * np.cos(2 * np.pi * k[1] * yy / ny + ph[1])
            if dim == 3:
                term = term * np.cos(2 * np.pi * k[2] * zz / nz + ph[2])
            s += a * term
        return s / max(np.abs(s).max(), 1e-30)

    phi = interface_profile(3.0 * smooth() * params.get("W", 4.0), params.get("W", 4.0))
    u = np.zeros((3, nz, ny, nx))
    for i in range(dim):
        u[i] = u_amp * smooth()
    p = p_amp * smooth()
    return phi, u, p


def population_noise(Q, n, seed, amp):
    """Seeded zero-mean noise of shape (Q, nz, ny, nx) for perturbing
    populations away from equilibrium."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    return amp * rng.uniform(-1.0, 1.0, size=(Q, nz, ny, nx))


def serving_spec(seed=1, count=1000, rate=20.0, edge_range=(64, 1024), steps_range=(500, 20000),
                 rho_ratio_range=(3.0, 1000.0)):
    """Seeded request stream for the serving workload: Poisson arrivals at
    `rate` per second; each request is a 2-D solve of one of three types
    (Rayleigh-Taylor, static drop, impacting drop, equally likely) on an
    edge x edge lattice with the edge, the density ratio and the number of
    steps log-uniform in their ranges.  Per type: Rayleigh-Taylor Re
    log-uniform in [100, 1000]; static drop R = edge/8, sigma log-uniform in
    [1e-4, 1e-2]; impacting drop D = edge/8, U0 = 0.05, Re log-uniform in
    [100, 1000], We log-uniform in [100, 2000]; W = 4, M = 0.1.
    Returns a list of dicts (id, arrival, kind, edge, rho_ratio, steps, ...);
    `serving_case` builds the fields of one."""
    rng = np.random.default_rng(seed)

    def logu(lo, hi):
        return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))

    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        kind = ("rti", "static_drop", "impacting_drop")[int(rng.integers(0, 3))]
        spec = dict(id=i, arrival=t, kind=kind, edge=int(round(logu(*edge_range))),
                    rho_ratio=logu(*rho_ratio_range), steps=int(round(logu(*steps_range))))
        if kind == "rti":
            spec["Re"] = logu(100.0, 1000.0)
        elif kind == "static_drop":
            spec["sigma"] = logu(1e-4, 1e-2)
        else:
            spec["Re"] = logu(100.0, 1000.0)
            spec["We"] = logu(100.0, 2000.0)
        out.append(spec)
    return out


def serving_case(spec):
    """The Case of one serving request (see serving_spec)."""
    e, r = spec["edge"], spec["rho_ratio"]
    if spec["kind"] == "rti":
        At = (r - 1.0) / (r + 1.0)
        return rti2d(nx=e, ny=e, At=At, Re=spec["Re"], W=4.0, M=0.1, amp=0.05 * e,
                     steps=spec["steps"])
    if spec["kind"] == "static_drop":
        return static_droplet(dim=2, n=(e, e, 1), R=e / 8.0, sigma=spec["sigma"], rho_ratio=r,
                              nu=0.1, W=4.0, M=0.1, steps=spec["steps"])
    return impacting_droplet2d(n=e, D=e / 8.0, U0=0.05, Re=spec["Re"], We=spec["We"], W=4.0,
                               M=0.1, steps=spec["steps"], rho_ratio=r)
