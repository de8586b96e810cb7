"""Seeded synthetic inputs for the lattice Boltzmann workloads.

This module produces macroscopic initial fields (density or water height, velocity)
and per-box parameters only.  It holds none of the method's arithmetic: equilibrium
populations are computed from these fields independently by the HIP library and by
the FP64 oracle.  Every generator is deterministic given its arguments and seed
(numpy PCG64 via default_rng).

Coordinates: node x = i for i = 0 .. N-1; wave number k = 2 pi / N.
"""
import math

import numpy as np


def re_to_omega(u0, n, re):
    """Shear rate from a Reynolds number Re = u0 L / nu with L = N / (2 pi) and the
    lattice relation nu = (1/omega - 1/2) / 3."""
    nu = u0 * (n / (2.0 * math.pi)) / re
    return 1.0 / (3.0 * nu + 0.5)


def tgv2d_fields(nx, ny, nz=1, u0=0.01):
    """Taylor-Green vortex of sec. 5.1 (eq. TGA_init at t = 0), invariant along z:
    u_x = u0 cos(kx) sin(ky), u_y = -u0 sin(kx) cos(ky), u_z = 0,
    rho = 1 - 3 u0^2 / 4 (cos 2kx + cos 2ky), with k = 2 pi / nx (square in x, y).
    Returns rho (nz, ny, nx) and u (3, nz, ny, nx), float64."""
    k = 2.0 * math.pi / nx
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    shape = (nz, ny, nx)
    ux = np.broadcast_to(u0 * np.cos(k * x) * np.sin(k * y), shape)
    uy = np.broadcast_to(-u0 * np.sin(k * x) * np.cos(k * y), shape)
    rho = np.broadcast_to(1.0 - 0.75 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y)), shape)
    u = np.stack([ux, uy, np.zeros(shape)])
    return np.ascontiguousarray(rho), np.ascontiguousarray(u)


def tgv3d_fields(nx, ny=None, nz=None, u0=0.05, phase=(0.0, 0.0, 0.0), period=None):
    """Three-dimensional Taylor-Green vortex (Brachet form):
    u = (u0 sin(kx) cos(ky) cos(kz), -u0 cos(kx) sin(ky) cos(kz), 0),
    rho = 1 + 3 (u0^2 / 16) (cos 2kx + cos 2ky) (cos 2kz + 2), k = 2 pi / period,
    period defaults to nx (a cube).  phase is added to (kx, ky, kz).
    A reduced copy of a large box keeps u0 and the rates, so its kernel constants match."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    period = nx if period is None else period
    k = 2.0 * math.pi / period
    ax = k * np.arange(nx, dtype=np.float64)[None, None, :] + phase[0]
    ay = k * np.arange(ny, dtype=np.float64)[None, :, None] + phase[1]
    az = k * np.arange(nz, dtype=np.float64)[:, None, None] + phase[2]
    shape = (nz, ny, nx)
    ux = np.broadcast_to(u0 * np.sin(ax) * np.cos(ay) * np.cos(az), shape)
    uy = np.broadcast_to(-u0 * np.cos(ax) * np.sin(ay) * np.cos(az), shape)
    rho = np.broadcast_to(1.0 + 3.0 * (u0 * u0 / 16.0) * (np.cos(2 * ax) + np.cos(2 * ay))
                          * (np.cos(2 * az) + 2.0), shape)
    u = np.stack([ux, uy, np.zeros(shape)])
    return np.ascontiguousarray(rho), np.ascontiguousarray(u)


def tgv3d_points(ix, iy, iz, n, u0=0.05, phase=(0.0, 0.0, 0.0)):
    """The fields of tgv3d_fields(n, u0=u0, phase=phase) at integer nodes (ix, iy, iz) only
    (same formula, evaluated point by point): rho (m,), u (m, 3)."""
    k = 2.0 * math.pi / n
    ax = k * np.asarray(ix, dtype=np.float64) + phase[0]
    ay = k * np.asarray(iy, dtype=np.float64) + phase[1]
    az = k * np.asarray(iz, dtype=np.float64) + phase[2]
    ux = u0 * np.sin(ax) * np.cos(ay) * np.cos(az)
    uy = -u0 * np.cos(ax) * np.sin(ay) * np.cos(az)
    rho = 1.0 + 3.0 * (u0 * u0 / 16.0) * (np.cos(2 * ax) + np.cos(2 * ay)) * (np.cos(2 * az) + 2.0)
    return rho, np.stack([ux, uy, np.zeros_like(ux)], axis=1)


def sample_cells(dims, count, seed=0):
    """Distinct sample cells (x, y, z): the eight box corners, cells on each face, the rest
    uniform; returns an int array (m, 3)."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    pts = {(x, y, z) for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)}
    for _ in range(count):
        p = [int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))]
        face = int(rng.integers(0, 4))
        if face < 3:
            p[face] = 0 if rng.random() < 0.5 else (nx, ny, nz)[face] - 1
        pts.add(tuple(p))
    return np.array(sorted(pts), dtype=np.int64)


def swe_bumps(n, seed=0, nbumps=16, amp=0.1, sigma=(20.0, 100.0)):
    """Water height h = 1 + amp * sum_b exp(-d_per(x, c_b)^2 / (2 sigma_b^2)) on an n x n
    periodic grid, centres c_b uniform in [0, n)^2, sigma_b uniform in [20, 100] cells,
    zero velocity.  Returns h (1, n, n) and u (3, 1, n, n)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, n, size=(nbumps, 2))
    s = rng.uniform(sigma[0], sigma[1], size=nbumps)
    x = np.arange(n, dtype=np.float64)
    h = np.ones((n, n))
    for b in range(nbumps):
        dx = np.abs(x - c[b, 0])
        dx = np.minimum(dx, n - dx)
        dy = np.abs(x - c[b, 1])
        dy = np.minimum(dy, n - dy)
        h += amp * np.exp(-(dy[:, None] ** 2 + dx[None, :] ** 2) / (2.0 * s[b] ** 2))
    return h[None], np.zeros((3, 1, n, n))


DAM_BREAK = dict(domain_m=40.0, cells=100, dt_s=0.05, nu_m2_per_s=1.0, g_m_per_s2=9.81,
                 radius_m=2.5, column_m=2.5, depth_m=0.5)


def dam_break_lattice(p=DAM_BREAK):
    """Lattice parameters of the circular dam break of sec. 5.2: dx = domain / cells; heights
    stay in metres, so the lattice gravity is g dt^2 / dx^2 (g h then has lattice units of
    velocity squared); nu_lattice = nu dt / dx^2."""
    dx = p["domain_m"] / p["cells"]
    return {"dx": dx, "gravity": p["g_m_per_s2"] * p["dt_s"] ** 2 / dx ** 2,
            "nu": p["nu_m2_per_s"] * p["dt_s"] / dx ** 2}


def dam_break_fields(p=DAM_BREAK):
    """Water column of the given radius and height at the centre of the periodic square domain,
    the rest at the base depth, fluid at rest (sec. 5.2).  Node (i, j) sits at (i dx, j dx), the
    column centre at (domain / 2, domain / 2).  Returns h (1, n, n) and u (3, 1, n, n)."""
    n = p["cells"]
    dx = p["domain_m"] / n
    x = np.arange(n) * dx - 0.5 * p["domain_m"]
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    h = np.where(r2 < p["radius_m"] ** 2, p["column_m"], p["depth_m"])
    return h[None].astype(np.float64), np.zeros((3, 1, n, n))


def batch_ensemble(nboxes=256, seed=0, edges=(32, 48, 64, 96), nu_range=(1e-4, 1e-1),
                   u0_range=(0.01, 0.05)):
    """Parameters of an ensemble of independent periodic cubes: edge uniform in `edges`,
    viscosity log-uniform in nu_range (omega_s = 1 / (3 nu + 1/2)), Taylor-Green
    amplitude u0 uniform in u0_range and a random phase in [0, 2 pi)^3.
    Returns a list of dicts {edge, nu, omega_shear, u0, phase}."""
    rng = np.random.default_rng(seed)
    e = rng.choice(np.array(edges), size=nboxes)
    lognu = rng.uniform(math.log(nu_range[0]), math.log(nu_range[1]), size=nboxes)
    u0 = rng.uniform(u0_range[0], u0_range[1], size=nboxes)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=(nboxes, 3))
    out = []
    for b in range(nboxes):
        nu = math.exp(lognu[b])
        out.append({"edge": int(e[b]), "nu": nu, "omega_shear": 1.0 / (3.0 * nu + 0.5),
                    "u0": float(u0[b]), "phase": tuple(float(v) for v in ph[b])})
    return out


def batch_fields(box):
    """Initial Taylor-Green fields of one ensemble box."""
    n = box["edge"]
    return tgv3d_fields(n, u0=box["u0"], phase=box["phase"])


def random_near_equilibrium_fields(shape, seed=0, drho=1e-2, umax=0.05):
    """Smooth-free random fields for collision tests: rho = 1 + drho * N(0,1),
    u uniform in [-umax, umax]^3 (u_z = 0 for a 2-D shape with nz == 1 is not enforced)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + drho * rng.standard_normal(shape)
    u = rng.uniform(-umax, umax, size=(3,) + tuple(shape))
    return rho, u


def random_perturbation(q, shape, seed=0, scale=1e-4):
    """Gaussian noise (q, *shape) added to equilibrium populations to create a non-equilibrium state."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((q,) + tuple(shape))


# Parameters of the five benchmark workloads (sizes, rates, amplitudes).
WORKLOADS = {
    "d2q9_central_64": dict(stencil="D2Q9", space="central", dims=(64, 64, 1), u0=0.01,
                            omega_shear=1.6, steps=1000, storage="f64"),
    "d3q19_raw_256": dict(stencil="D3Q19", space="raw", dims=(256, 256, 256), u0=0.02,
                          omega_shear=re_to_omega(0.02, 256, 1600.0), steps=500),
    "d3q27_cumulant_512": dict(stencil="D3Q27", space="cumulant", dims=(512, 512, 512), u0=0.05,
                               omega_shear=re_to_omega(0.05, 512, 1600.0), steps=200),
    "d3q15_raw_512": dict(stencil="D3Q15", space="raw", dims=(512, 512, 512), u0=0.05,
                          omega_shear=re_to_omega(0.05, 512, 1600.0), steps=200),
    "batch_d3q27_central": dict(stencil="D3Q27", space="central", nboxes=256, steps=100,
                                storage="f32"),
    "swe_d2q9_4096": dict(stencil="D2Q9", space="central", equilibrium="swe", dims=(4096, 4096, 1),
                          gravity=0.1, omega_shear=1.0 / (3.0 * 0.3125 + 0.5), steps=1000),
}
