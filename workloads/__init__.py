"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only *generates problem data* (densities, Dirichlet face values,
loss weights, batch shapes).  It contains none of the solver's arithmetic: no
Laplacian, no Runge-Kutta-Legendre stage, no transfer operator, no norm used by
the method.  Both ``oracle/`` and the GPU package may import it; it imports
neither.

Array layout everywhere: ``[k][j][i]`` (numpy shape ``(nz, ny, nx)``), x fastest,
cell-centred samples.  Face arrays for Dirichlet boundaries follow the packing
of the C ABI: x faces have shape ``(nz, ny)``, y faces ``(nz, nx)``, z faces
``(ny, nx)``; the order is x-, x+, y-, y+, z-, z+.

Workloads (paper: Mandal, Mukherjee & Mignone, "A self-gravity module for the
PLUTO code", ApJS 2023):

* ``uniform_sphere`` - a constant-density ball with Dirichlet data from its
  exterior point-mass potential -M/r (the classic isolated-sphere check).
* ``accuracy_problem`` - the paper's 3-D accuracy model (Sec. 4.1, eqs.
  source_3D / phi_3D / acceleration_3D): rho0 (1 - r^2/r0^2)^2 inside r0.
* ``gaussian_blobs`` - periodic sum of Gaussian blobs, minimum-image distance,
  lognormal amplitudes, mean removed.
* ``gaussian_random_field`` - periodic field with power spectrum P(k) ~ k^-3,
  unit variance, mean removed.
* ``batch_grid_sizes`` - uneven batch composition over {32,48,64,96,128}^3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Problem",
    "cell_centres",
    "face_centres",
    "uniform_sphere",
    "accuracy_problem",
    "gaussian_blobs",
    "gaussian_random_field",
    "batch_grid_sizes",
    "batch_blob_problems",
    "adjoint_inputs",
    "pack_faces",
]


@dataclass
class Problem:
    """One Poisson problem: density on a cell-centred box plus boundary data.

    ``bc`` is ``"dirichlet"`` or ``"periodic"``.  ``faces`` is a tuple of six
    arrays (x-, x+, y-, y+, z-, z+) of boundary values at face centres for
    Dirichlet problems, ``None`` for periodic ones.  ``phi_exact`` is the
    continuous analytic potential sampled at cell centres when one exists.
    """

    rho: np.ndarray
    h: tuple  # (hx, hy, hz)
    lo: tuple  # lower corner (x0, y0, z0)
    bc: str
    faces: tuple | None = None
    phi_exact: np.ndarray | None = None
    name: str = ""

    @property
    def shape(self):
        return self.rho.shape  # (nz, ny, nx)


def cell_centres(n, lo, h):
    """Cell-centre coordinate arrays X, Y, Z with shape (nz, ny, nx)."""
    nz, ny, nx = n
    x = lo[0] + (np.arange(nx) + 0.5) * h[0]
    y = lo[1] + (np.arange(ny) + 0.5) * h[1]
    z = lo[2] + (np.arange(nz) + 0.5) * h[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def face_centres(n, lo, h):
    """Coordinates of the six boundary-face centre sets.

    Returns a list of six (X, Y, Z) tuples in the order x-, x+, y-, y+, z-, z+.
    The x faces are indexed [k][j], the y faces [k][i], the z faces [j][i].
    """
    nz, ny, nx = n
    xs = lo[0] + (np.arange(nx) + 0.5) * h[0]
    ys = lo[1] + (np.arange(ny) + 0.5) * h[1]
    zs = lo[2] + (np.arange(nz) + 0.5) * h[2]
    x_lo, x_hi = lo[0], lo[0] + nx * h[0]
    y_lo, y_hi = lo[1], lo[1] + ny * h[1]
    z_lo, z_hi = lo[2], lo[2] + nz * h[2]
    out = []
    Zk, Yj = np.meshgrid(zs, ys, indexing="ij")
    for xv in (x_lo, x_hi):
        out.append((np.full_like(Zk, xv), Yj, Zk))
    Zk, Xi = np.meshgrid(zs, xs, indexing="ij")
    for yv in (y_lo, y_hi):
        out.append((Xi, np.full_like(Zk, yv), Zk))
    Yj, Xi = np.meshgrid(ys, xs, indexing="ij")
    for zv in (z_lo, z_hi):
        out.append((Xi, Yj, np.full_like(Yj, zv)))
    return out


def pack_faces(faces):
    """Concatenate the six face arrays into one flat float64 vector (C-ABI order)."""
    return np.concatenate([np.ascontiguousarray(f, dtype=np.float64).ravel() for f in faces])


def uniform_sphere(n=32, radius=0.3, rho0=1.0, box=(-1.0, 1.0)):
    """Constant-density ball of ``radius`` centred at the origin, Dirichlet box.

    The density is point-sampled at cell centres (rho0 where r <= radius).
    Boundary values are the exterior potential of the continuous ball,
    -M/r with M = 4 pi rho0 R^3 / 3 (G = 1).  The analytic potential is
    2 pi rho0 (r^2/3 - R^2) inside and -M/r outside.
    """
    lo = (box[0],) * 3
    h = ((box[1] - box[0]) / n,) * 3
    shape = (n, n, n)
    X, Y, Z = cell_centres(shape, lo, h)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    rho = np.where(r <= radius, rho0, 0.0).astype(np.float64)
    mass = 4.0 * math.pi * rho0 * radius**3 / 3.0

    def pot(rr):
        inside = 2.0 * math.pi * rho0 * (rr * rr / 3.0 - radius * radius)
        with np.errstate(divide="ignore"):
            outside = -mass / rr
        return np.where(rr <= radius, inside, outside)

    faces = []
    for (fx, fy, fz) in face_centres(shape, lo, h):
        faces.append(pot(np.sqrt(fx * fx + fy * fy + fz * fz)))
    return Problem(rho=rho, h=h, lo=lo, bc="dirichlet", faces=tuple(faces),
                   phi_exact=pot(r), name=f"uniform_sphere_{n}")


def uniform_disc(nx=64, ny=None, radius=0.3, rho0=1.0, box=(-1.0, 1.0)):
    """Two-dimensional analogue of ``uniform_sphere``: a constant-density disc
    of ``radius`` at the origin on a Dirichlet rectangle (nz = 1, hz = inf).

    ``box`` gives the x extent; y spans ny cells of the same width (square
    cells).  With G = 1 the continuous potential is pi rho0 r^2 inside and
    2 pi rho0 R^2 ln(r/R) + pi rho0 R^2 outside; the faces carry its values
    (z faces are zero and carry no weight in 2-D).
    """
    ny = nx if ny is None else ny
    hx = (box[1] - box[0]) / nx
    h = (hx, hx, float("inf"))
    lo = (box[0], -0.5 * ny * hx, 0.0)
    xs = lo[0] + (np.arange(nx) + 0.5) * hx
    ys = lo[1] + (np.arange(ny) + 0.5) * hx
    X = np.broadcast_to(xs[None, :], (ny, nx))
    Y = np.broadcast_to(ys[:, None], (ny, nx))
    r = np.sqrt(X * X + Y * Y)
    rho = np.where(r <= radius, rho0, 0.0)[None].astype(np.float64)

    def pot(rr):
        rr = np.asarray(rr, dtype=np.float64)
        inside = math.pi * rho0 * rr * rr
        with np.errstate(divide="ignore"):
            outside = 2.0 * math.pi * rho0 * radius * radius * np.log(rr / radius) + math.pi * rho0 * radius ** 2
        return np.where(rr <= radius, inside, outside)

    x0, x1 = lo[0], lo[0] + nx * hx
    y0, y1 = lo[1], lo[1] + ny * hx
    faces = (pot(np.hypot(x0, ys))[None, :], pot(np.hypot(x1, ys))[None, :],
             pot(np.hypot(xs, y0))[None, :], pot(np.hypot(xs, y1))[None, :],
             np.zeros((ny, nx)), np.zeros((ny, nx)))
    return Problem(rho=rho, h=h, lo=lo, bc="dirichlet", faces=faces,
                   phi_exact=pot(r)[None], name=f"uniform_disc_{nx}x{ny}")


def _smooth_disc_phi(r, rho0, r0):
    # (1/r)(r phi')' = 4 pi rho with rho = rho0 (1 - r^2/r0^2)^2 inside r0:
    # r phi' = 4 pi rho0 (r^2/2 - r^4/(2 r0^2) + r^6/(6 r0^4)); mass pi rho0 r0^2 / 3
    inside = 4.0 * math.pi * rho0 * (r * r / 4.0 - r**4 / (8.0 * r0 * r0) + r**6 / (36.0 * r0**4))
    with np.errstate(divide="ignore"):
        outside = (2.0 / 3.0) * math.pi * rho0 * r0 * r0 * np.log(r / r0) + 11.0 * math.pi * rho0 * r0 * r0 / 18.0
    return np.where(r <= r0, inside, outside)


def smooth_disc(n, rho0=1.0, r0=0.25):
    """Two-dimensional analogue of the accuracy model: rho = rho0 (1 -
    r^2/r0^2)^2 inside r0 on [-0.5, 0.5]^2 (nz = 1, hz = inf), Dirichlet data
    from the continuous potential (G = 1), which is returned as phi_exact."""
    h = 1.0 / n
    xs = -0.5 + (np.arange(n) + 0.5) * h
    r = np.sqrt(xs[None, :] ** 2 + xs[:, None] ** 2)
    rho = np.where(r <= r0, rho0 * (1.0 - r * r / (r0 * r0)) ** 2, 0.0)[None]
    edge = lambda a, b: _smooth_disc_phi(np.hypot(a, b), rho0, r0)[None, :]
    faces = (edge(-0.5, xs), edge(0.5, xs), edge(xs, -0.5), edge(xs, 0.5), np.zeros((n, n)), np.zeros((n, n)))
    return Problem(rho=rho, h=(h, h, float("inf")), lo=(-0.5, -0.5, 0.0), bc="dirichlet", faces=faces,
                   phi_exact=_smooth_disc_phi(r, rho0, r0)[None], name=f"smooth_disc_{n}")


def gaussian_blobs_2d(nx, ny=None, nblobs=8, rng=None, seed=None, sigma_range=(0.02, 0.08)):
    """Periodic Gaussian blobs on the unit square (nz = 1, hz = inf), the 2-D
    analogue of ``gaussian_blobs``; the mean is subtracted."""
    if rng is None:
        rng = np.random.default_rng(seed)
    ny = nx if ny is None else ny
    centres = rng.uniform(0.0, 1.0, size=(nblobs, 2))
    sigmas = rng.uniform(sigma_range[0], sigma_range[1], size=nblobs)
    amps = np.exp(rng.normal(0.0, 1.0, size=nblobs))
    xs = (np.arange(nx) + 0.5) / nx
    ys = (np.arange(ny) + 0.5) / ny
    rho = np.zeros((1, ny, nx), dtype=np.float64)
    for (cx, cy), sg, a in zip(centres, sigmas, amps):
        dx = xs - cx
        dx -= np.round(dx)
        dy = ys - cy
        dy -= np.round(dy)
        c = -0.5 / (sg * sg)
        rho[0] += a * (np.exp(c * dy * dy)[:, None] * np.exp(c * dx * dx)[None, :])
    rho -= rho.mean()
    return Problem(rho=rho, h=(1.0 / nx, 1.0 / ny, float("inf")), lo=(0.0, 0.0, 0.0), bc="periodic",
                   name=f"blobs2d_{nx}x{ny}_{nblobs}")


def problem_2d(nx, ny, bc, seed=0):
    """A 2-D test problem: blobs (periodic) or the uniform disc (Dirichlet)."""
    if bc == "periodic":
        return gaussian_blobs_2d(nx, ny, nblobs=8, seed=seed)
    return uniform_disc(nx, ny)


def _accuracy_phi(r, rho0, r0):
    mass = 32.0 * math.pi * rho0 * r0**3 / 105.0
    inside = (-2.0 / 3.0 * math.pi * rho0 * r0 * r0
              + 4.0 * math.pi * rho0 * (r * r / 6.0 - r**4 / (10.0 * r0 * r0)
                                         + r**6 / (42.0 * r0**4)))
    with np.errstate(divide="ignore"):
        outside = -mass / r
    return np.where(r <= r0, inside, outside)


def accuracy_problem(n, rho0=1.0, r0=0.25):
    """The paper's 3-D accuracy model (Sec. 4.1): smooth compact density.

    rho = rho0 (1 - r^2/r0^2)^2 for r <= r0, zero outside, on [-0.5, 0.5]^3;
    Dirichlet data from the exact potential (eq. phi_3D), G = 1.
    """
    lo = (-0.5,) * 3
    h = (1.0 / n,) * 3
    shape = (n, n, n)
    X, Y, Z = cell_centres(shape, lo, h)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    rho = np.where(r <= r0, rho0 * (1.0 - r * r / (r0 * r0)) ** 2, 0.0)
    faces = tuple(_accuracy_phi(np.sqrt(fx * fx + fy * fy + fz * fz), rho0, r0)
                  for (fx, fy, fz) in face_centres(shape, lo, h))
    return Problem(rho=rho, h=h, lo=lo, bc="dirichlet", faces=faces,
                   phi_exact=_accuracy_phi(r, rho0, r0), name=f"accuracy_{n}")


def accuracy_fields_device(n, device, rho0=1.0, r0=0.25):
    """The accuracy model built directly in device memory (torch), for grids
    too large to build on the host: (rho, phi_exact, g_x exact, faces) with
    faces as numpy arrays (x-, x+, y-, y+, z-, z+)."""
    import torch
    h = 1.0 / n
    c = -0.5 + (torch.arange(n, dtype=torch.float64, device=device) + 0.5) * h
    Z = c.view(n, 1, 1)
    Y = c.view(1, n, 1)
    X = c.view(1, 1, n)
    r = torch.sqrt(X * X + Y * Y + Z * Z)
    rho = torch.where(r <= r0, rho0 * (1.0 - r * r / (r0 * r0)) ** 2, torch.zeros_like(r))
    mass = 32.0 * math.pi * rho0 * r0**3 / 105.0
    inside = (-2.0 / 3.0 * math.pi * rho0 * r0 * r0
              + 4.0 * math.pi * rho0 * (r * r / 6.0 - r**4 / (10.0 * r0 * r0) + r**6 / (42.0 * r0**4)))
    phi = torch.where(r <= r0, inside, -mass / r)
    gin = -4.0 * math.pi * rho0 * (r / 3.0 - 0.4 * r**3 / r0**2 + r**5 / (7.0 * r0**4))
    gr = torch.where(r <= r0, gin, -mass / (r * r))
    gx = gr * X / r
    del inside, gin, gr
    faces = tuple(_accuracy_phi(np.sqrt(fx * fx + fy * fy + fz * fz), rho0, r0)
                  for (fx, fy, fz) in face_centres((n, n, n), (-0.5,) * 3, (h,) * 3))
    return rho, phi, gx, faces


def accuracy_acceleration_x(n, rho0=1.0, r0=0.25):
    """x-component of the analytic acceleration of the accuracy model (eq. acceleration_3D)."""
    X, Y, Z = cell_centres((n, n, n), (-0.5,) * 3, (1.0 / n,) * 3)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    mass = 32.0 * math.pi * rho0 * r0**3 / 105.0
    gin = -4.0 * math.pi * rho0 * (r / 3.0 - 0.4 * r**3 / r0**2 + r**5 / (7.0 * r0**4))
    with np.errstate(divide="ignore", invalid="ignore"):
        gout = -mass / (r * r)
        gr = np.where(r <= r0, gin, gout)
        gx = np.where(r > 0, gr * X / r, 0.0)
    return gx


def gaussian_blobs(n, nblobs=16, rng=None, seed=None, sigma_range=(0.02, 0.08),
                   subtract_mean=True):
    """Periodic sum of Gaussian blobs on the unit box [0,1]^3.

    Centres ~ U[0,1)^3, widths sigma ~ U[sigma_range], amplitudes ~ lognormal(0,1).
    rho = sum_b a_b exp(-d_b^2 / (2 sigma_b^2)) with d_b the minimum-image
    distance to centre b.  The mean is subtracted.  ``n`` is an int (cube) or a
    (nz, ny, nx) tuple.
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    nz, ny, nx = shape
    centres = rng.uniform(0.0, 1.0, size=(nblobs, 3))
    sigmas = rng.uniform(sigma_range[0], sigma_range[1], size=nblobs)
    amps = np.exp(rng.normal(0.0, 1.0, size=nblobs))
    xs = (np.arange(nx) + 0.5) / nx
    ys = (np.arange(ny) + 0.5) / ny
    zs = (np.arange(nz) + 0.5) / nz
    rho = np.zeros(shape, dtype=np.float64)
    for (cx, cy, cz), sg, a in zip(centres, sigmas, amps):
        dx = xs - cx
        dx -= np.round(dx)
        dy = ys - cy
        dy -= np.round(dy)
        dz = zs - cz
        dz -= np.round(dz)
        c = -0.5 / (sg * sg)
        # separable: exp(c(dx^2+dy^2+dz^2)) = ex * ey * ez
        ex = np.exp(c * dx * dx)
        ey = np.exp(c * dy * dy)
        ez = np.exp(c * dz * dz)
        rho += a * (ez[:, None, None] * ey[None, :, None] * ex[None, None, :])
    if subtract_mean:
        rho -= rho.mean()
    h = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    return Problem(rho=rho, h=h, lo=(0.0, 0.0, 0.0), bc="periodic",
                   name=f"blobs_{nx}x{ny}x{nz}_{nblobs}")


def gaussian_random_field(n, rng=None, seed=None, slope=-3.0):
    """Periodic Gaussian random field with P(k) ~ |k|^slope on [0,1]^3.

    Real white noise N(0,1) -> real FFT -> amplitude |k|^(slope/2) with
    k = 2 pi * integer wavenumber (k = 0 set to 0) -> inverse FFT -> subtract
    the mean -> divide by the standard deviation.  Computed in float64.
    """
    import scipy.fft as sfft

    if rng is None:
        rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n, n))
    nh = sfft.rfftn(noise, workers=-1)
    del noise
    kz = np.fft.fftfreq(n, d=1.0 / n) * 2.0 * math.pi
    kx = np.fft.rfftfreq(n, d=1.0 / n) * 2.0 * math.pi
    k2 = (kz[:, None, None] ** 2 + kz[None, :, None] ** 2 + kx[None, None, :] ** 2)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)
    nh *= amp
    del amp, k2
    field = sfft.irfftn(nh, s=(n, n, n), workers=-1)
    del nh
    field -= field.mean()
    field /= field.std()
    h = (1.0 / n,) * 3
    return Problem(rho=field, h=h, lo=(0.0, 0.0, 0.0), bc="periodic",
                   name=f"grf_{n}")


BATCH_SIZES = (32, 48, 64, 96, 128)


def batch_grid_sizes(rng=None, seed=None, total=96, sizes=BATCH_SIZES):
    """Uneven batch composition: counts ~ multinomial(total, dirichlet(1)),
    redrawn until every size occurs at least once.  Returns the list of grid
    edge lengths, ordered by size class."""
    if rng is None:
        rng = np.random.default_rng(seed)
    while True:
        counts = rng.multinomial(total, rng.dirichlet(np.ones(len(sizes))))
        if np.all(counts > 0):
            break
    out = []
    for s, c in zip(sizes, counts):
        out += [int(s)] * int(c)
    return out


def batch_blob_problems(rng=None, seed=None, total=96, sizes=BATCH_SIZES,
                        blob_range=(4, 16)):
    """The batched workload: ``total`` periodic blob fields of uneven sizes,
    each with 4..16 blobs (``rng.integers(4, 17)``)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    ns = batch_grid_sizes(rng=rng, total=total, sizes=sizes)
    probs = []
    for n in ns:
        nb = int(rng.integers(blob_range[0], blob_range[1] + 1))
        probs.append(gaussian_blobs(n, nblobs=nb, rng=rng))
    return probs


def adjoint_inputs(n, nbatch=8, ndirs=16, rng=None, seed=None):
    """Inputs of the differentiation workload: ``nbatch`` periodic blob
    densities of size n^3, loss weights w ~ N(0,1) per cell, and ``ndirs``
    unit-norm random directions per cell (N(0,1) then normalised)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    rhos = np.stack([gaussian_blobs(n, nblobs=16, rng=rng).rho for _ in range(nbatch)])
    w = rng.standard_normal(rhos.shape)
    dirs = rng.standard_normal((ndirs,) + rhos.shape)
    for d in dirs:
        d /= np.linalg.norm(d)
    return rhos, w, dirs
