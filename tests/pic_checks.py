"""Independent reference routines used to pin the oracle (brute force and closed forms).

Nothing here calls the oracle or the GPU library.  The routines restate what the paper fixes
by a different route than the oracle's code: shape functions as tent sums with minimum-image
distances, the implicit response as a matrix inverse of the defining equation, and linear
systems solved with numpy.
"""
from __future__ import annotations

import math

import numpy as np


def tent(d):
    return np.maximum(0.0, 1.0 - np.abs(d))


def min_image(d, n):
    return (d + 0.5 * n) % n - 0.5 * n


def tent_weights(nx, nz, bc_x, xi_x, xi_z):
    """Weight of every particle on every node, [n_particles, nodes_z, nodes_x], computed as a
    product of 1D tent functions of the (minimum-image) particle-node distance."""
    nxn = nx + (1 if bc_x == 1 else 0)
    nzn = nz
    xi_x = np.asarray(xi_x)[:, None]
    xi_z = np.asarray(xi_z)[:, None]
    dxs = xi_x - np.arange(nxn)[None, :]
    if bc_x == 0:
        dxs = min_image(dxs, nx)
    dzs = min_image(xi_z - np.arange(nzn)[None, :], nz)
    return tent(dzs)[:, :, None] * tent(dxs)[:, None, :]


def cross_matrix(b):
    """Matrix X with X a = a x b."""
    b = np.asarray(b, dtype=np.float64)
    return np.column_stack([np.cross(e, b) for e in np.eye(3)])


def implicit_response(q, m, dt, u, B):
    """R solving u-bar = a + u-bar x b (b = q dt B / (2 m gamma(u))) as an explicit inverse."""
    gam = math.sqrt(1.0 + float(np.dot(u, u)))
    b = q * dt / (2.0 * m * gam) * np.asarray(B, dtype=np.float64)
    return np.linalg.inv(np.eye(3) - cross_matrix(b)), gam


def rotation_about_z(theta):
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def cayley_step_matrix(A, dt):
    """(I - A dt/2)^{-1} (I + A dt/2): the implicit-midpoint map of y' = A y."""
    n = A.shape[0]
    return np.linalg.solve(np.eye(n) - 0.5 * dt * A, np.eye(n) + 0.5 * dt * A)


def curl_multipliers(kx, kz, dx, dz):
    """Fourier symbol of the 2x2-averaged central differences: d/dx -> i kappa_x, d/dz -> i kappa_z."""
    a = 0.5 * kx * dx
    b = 0.5 * kz * dz
    return 2.0 * math.sin(a) * math.cos(b) / dx, 2.0 * math.cos(a) * math.sin(b) / dz


def max_rel(a, b, scale=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.max(np.abs(b)) if scale is None else scale
    if s == 0.0:
        return float(np.max(np.abs(a - b)))
    return float(np.max(np.abs(a - b)) / s)
