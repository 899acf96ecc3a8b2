"""Host-side measures of a state, shared by the oracle pins and the GPU
tests (no method arithmetic: they read fields and particle states)."""
import numpy as np


def rigidity_residual(u, own, P, periodic, i=0):
    """max over the nodes of particle i of |u - (U_i + omega_i x r)| in 2D,
    r = x - X_i with the minimum image on periodic axes (sec. 2.4: the
    penalization drives the velocity inside a solid toward the rigid motion
    that its momentum sums define).  u: (nz, ny, nx, 3); own: (nz, ny, nx)
    with the particle index per node.  Returns (residual, max |u| anywhere)."""
    _, ny, nx = own.shape
    zz, yy, xx = np.nonzero(own == i)
    X, U, w = P["X"][i], P["U"][i], P["omega"][i]
    rx, ry = xx - X[0], yy - X[1]
    if periodic[0]:
        rx = rx - nx * np.round(rx / nx)
    if periodic[1]:
        ry = ry - ny * np.round(ry / ny)
    du = u[zz, yy, xx, :2] - np.stack([U[0] - w[2] * ry, U[1] + w[2] * rx], axis=1)
    return float(np.sqrt((du**2).sum(axis=1)).max()), float(np.abs(u[..., :2]).max())
