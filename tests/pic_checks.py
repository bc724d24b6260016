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


def abs_deposit_scale(nx, nz, bc_x, dt, species, H):
    """Per moment plane, the largest node value of the deposit of |contribution| (the scale
    that relative errors of a plane are measured against: it does not vanish where a plane's
    signed terms cancel, as delta-j of a neutral thermal plasma does).

    ``species`` is a list of (q, m, w, xi_x, xi_z, ux, uy, uz); ``H`` is [3][nz * nx].
    Each particle's response comes from an explicit matrix inverse of the defining equation,
    its four node weights from the bilinear tent product.
    """
    nxn = nx + (1 if bc_x == 1 else 0)
    S = len(species)
    acc = np.zeros((12 + S, nz, nxn))
    H = np.asarray(H, dtype=np.float64).reshape(3, nz * nx)
    for s, (q, m, w, xi_x, xi_z, ux, uy, uz) in enumerate(species):
        if len(xi_x) == 0:
            continue
        i = np.floor(xi_x).astype(np.int64)
        k = np.floor(xi_z).astype(np.int64)
        fx = xi_x - i
        fz = xi_z - k
        u = np.stack([ux, uy, uz], axis=1)
        gam = np.sqrt(1.0 + np.sum(u * u, axis=1))
        B = H[:, k * nx + i].T
        b = (q * dt / (2.0 * m * gam))[:, None] * B
        X = np.zeros((len(gam), 3, 3))
        # X a = a x b
        X[:, 0, 1], X[:, 0, 2] = b[:, 2], -b[:, 1]
        X[:, 1, 0], X[:, 1, 2] = -b[:, 2], b[:, 0]
        X[:, 2, 0], X[:, 2, 1] = b[:, 1], -b[:, 0]
        R = np.linalg.inv(np.eye(3)[None] - X)
        Sh = (w * q * q * dt * dt / (4.0 * m * gam))[:, None, None] * R
        dj = (w * q / gam)[:, None] * np.einsum("nij,nj->ni", R, u)
        c = np.concatenate([np.abs(Sh.reshape(-1, 9)), np.abs(dj)], axis=1)
        nn = nz * nxn
        for cx in (0, 1):
            for cz in (0, 1):
                W = (fx if cx else 1.0 - fx) * (fz if cz else 1.0 - fz)
                ii = i + cx
                if bc_x == 0:
                    ii = ii % nx
                node = ((k + cz) % nz) * nxn + ii
                for p in range(12):
                    acc[p] += np.bincount(node, weights=W * c[:, p], minlength=nn).reshape(nz, nxn)
                acc[12 + s] += np.bincount(node, weights=W * abs(w), minlength=nn).reshape(nz, nxn)
    return acc.reshape(12 + S, -1).max(axis=1)
