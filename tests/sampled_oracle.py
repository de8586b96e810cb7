"""Oracle values at sampled cells of boxes too large for the oracle to step whole.

Test infrastructure: uses only oracle/.  `fields_at(x, y, z)` returns the initial density
(m,) and velocity (m, 3) at integer nodes; the initial state is the equilibrium of those
fields.
"""
import numpy as np

import oracle as O


def one_step_samples(m, pts, dims, fields_at):
    """Expected df_i(x, 1) at the sample cells: collide the neighbours x - xi_i at t = 0."""
    st = m.st
    nx, ny, nz = dims
    src = (pts[:, None, :] - st.xi[None, :, :]) % np.array([nx, ny, nz])[None, None, :]
    flat = src.reshape(-1, 3)
    rho, u = fields_at(flat[:, 0], flat[:, 1], flat[:, 2])
    df0 = O.equilibrium_populations(m, rho, u) - m.f0
    out = O.collide_cells(m, df0, O.default_form(m)).reshape(len(pts), st.q, st.q)
    return out[:, np.arange(st.q), np.arange(st.q)]  # component i of neighbour i


def k_step_samples(m, pts, dims, fields_at, k):
    """Expected df(x, k) at the sample cells.  df(x, k) depends only on the cells within k of
    x along each axis at t = 0, so each sample gets a periodic window of (2k + 1)^3 cells
    centred on it; the windows sit side by side along x in one box, which the oracle steps k
    times.  Wrapped or neighbouring-window reads reach a cell only after more steps than its
    distance to the window's edge, so every window centre comes out exact."""
    nx, ny, nz = dims
    w = 2 * k + 1
    off = np.arange(-k, k + 1)
    zz, yy, xx = np.meshgrid(off, off, off, indexing="ij")
    rho = np.empty((w, w, w * len(pts)))
    u = np.empty((3, w, w, w * len(pts)))
    for j, (px, py, pz) in enumerate(pts):
        r, v = fields_at(((px + xx) % nx).ravel(), ((py + yy) % ny).ravel(), ((pz + zz) % nz).ravel())
        rho[:, :, j * w:(j + 1) * w] = r.reshape(w, w, w)
        u[:, :, :, j * w:(j + 1) * w] = v.T.reshape(3, w, w, w)
    df = O.step(m, O.init_equilibrium(m, rho, u), k)
    return df[:, k, k, np.arange(len(pts)) * w + k].T
