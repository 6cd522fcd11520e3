"""Seeded synthetic sources for the unbounded Poisson solve.

This module only draws random numbers and samples analytic source fields; it
holds none of the solver's arithmetic and imports neither the HIP library nor
the CPU oracle, so both sides can be fed the same inputs.

Grids are cell-centred: on a box of N_i cells of spacing h the sample points
are x_i = (i + 1/2) h.  Arrays are float64, indexed [z, y, x] (x fastest);
vector fields are stacked [component][z][y][x] with components (x, y, z).

Recipes (Gaussian blobs follow the paper's exp(-|x - c|^2 / sigma^2) form):

* ``single``: centres c ~ U[0.3, 0.7] per axis (scaled by the box length),
  amplitudes A ~ N(0, 1), widths sigma fixed or ~ U[lo, hi], then optional
  white noise of amplitude ``noise`` with its mean removed.
* ``curl``: f = -curl(A) with A = sum_b a_b g_b, a_b ~ N(0, I_3),
  g_b = exp(-|x - c_b|^2 / sigma_b^2); evaluated analytically as
  curl(a g) = grad(g) x a.
* ``weight``: w = exp(0.5 sum_b s_b g_b), signs s_b = +-1.
* ``vortex_tube``: the paper's compact vortex tube along z (Sec. 5),
  omega_z(r) = (1/2pi) (2/R^2) exp(-1/(1 - (r/R)^2)) / E_2(1) for r < R about
  the axis x = y = 1/2, and the Biot-Savart source f = -curl(omega e_z) =
  (-d omega/dy, d omega/dx, 0), evaluated analytically.
"""

import numpy as np
from scipy import special


def cell_centres(n, h):
    return (np.arange(int(n), dtype=np.float64) + 0.5) * float(h)


def _blob_axis(coord, c, sigma):
    # (len(coord), nblobs)
    return np.exp(-((coord[:, None] - c[None, :]) ** 2) / (sigma[None, :] ** 2))


def blob_sum(shape, h, centers, sigmas, amps):
    """sum_b amps[b] exp(-|x - centers[b]|^2 / sigmas[b]^2) on the cell-centred
    grid of ``shape`` = (Nz, Ny, Nx); centers are (x, y, z) triples."""
    Nz, Ny, Nx = (int(s) for s in shape)
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, 3)
    sigmas = np.asarray(sigmas, dtype=np.float64).reshape(-1)
    amps = np.asarray(amps, dtype=np.float64).reshape(-1)
    gx = _blob_axis(cell_centres(Nx, h), centers[:, 0], sigmas)
    gy = _blob_axis(cell_centres(Ny, h), centers[:, 1], sigmas)
    gz = _blob_axis(cell_centres(Nz, h), centers[:, 2], sigmas)
    # separable per blob: f[z,y,x] = sum_b (A_b gz_b[z] gy_b[y]) gx_b[x]
    zy = (gz[:, None, :] * gy[None, :, :] * amps[None, None, :]).reshape(Nz * Ny, -1)
    return (zy @ gx.T).reshape(Nz, Ny, Nx)


def draw_blobs(rng, nblobs, sigma, box=(1.0, 1.0, 1.0), lo=0.3, hi=0.7):
    """Draw (centers, sigmas, amps) in a fixed order: centres, widths, amplitudes.
    ``sigma`` is a number (fixed width) or a (lo, hi) pair (uniform)."""
    box = np.asarray(box, dtype=np.float64)
    centers = rng.uniform(lo, hi, size=(nblobs, 3)) * box[None, :]
    if np.ndim(sigma) == 0:
        sigmas = np.full(nblobs, float(sigma))
    else:
        sigmas = rng.uniform(float(sigma[0]), float(sigma[1]), size=nblobs)
    amps = rng.standard_normal(nblobs)
    return centers, sigmas, amps


def blob_source(shape, h, seed, nblobs, sigma, noise=0.0):
    """Seeded Gaussian-blob source plus optional zero-mean white noise."""
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    box = (shape[2] * h, shape[1] * h, shape[0] * h)
    centers, sigmas, amps = draw_blobs(rng, nblobs, sigma, box=box)
    f = blob_sum(shape, h, centers, sigmas, amps)
    if noise:
        w = rng.standard_normal(shape)
        w -= w.mean()
        f += noise * w
    return f


def curl_source(n, h, seed, nblobs=8, sigma=(0.05, 0.1)):
    """3-component source f = -curl(sum_b a_b g_b) on an n^3 grid -> [3][z][y][x]."""
    rng = np.random.default_rng(seed)
    L = n * h
    centers = rng.uniform(0.3, 0.7, size=(nblobs, 3)) * L
    sigmas = rng.uniform(sigma[0], sigma[1], size=nblobs)
    a = rng.standard_normal((nblobs, 3))
    x = cell_centres(n, h)
    f = np.zeros((3, n, n, n))
    for b in range(nblobs):
        dx = (x - centers[b, 0])[None, None, :]
        dy = (x - centers[b, 1])[None, :, None]
        dz = (x - centers[b, 2])[:, None, None]
        g = np.exp(-(dx ** 2 + dy ** 2 + dz ** 2) / sigmas[b] ** 2)
        s = 2.0 / sigmas[b] ** 2 * g          # -grad g = s * (x - c)
        ax, ay, az = a[b]
        # -curl(a g) = -(grad g x a) = s (x - c) x a
        f[0] += s * (dy * az - dz * ay)
        f[1] += s * (dz * ax - dx * az)
        f[2] += s * (dx * ay - dy * ax)
    return f


def weight_field(n, h, seed, nblobs=4):
    """Smooth positive weight w = exp(0.5 sum_b s_b g_b) on an n^3 grid."""
    rng = np.random.default_rng(seed)
    L = n * h
    centers = rng.uniform(0.2, 0.8, size=(nblobs, 3)) * L
    sigmas = rng.uniform(0.1, 0.2, size=nblobs)
    signs = rng.choice(np.array([-1.0, 1.0]), size=nblobs)
    return np.exp(0.5 * blob_sum((n, n, n), h, centers, sigmas, signs))


# --- the five workloads -----------------------------------------------------

def config_c1():
    """32^3 on the unit cube, FP64, 3 blobs sigma = 0.08 (seed 1)."""
    n = 32
    h = 1.0 / n
    return dict(name="c1", shape=(n, n, n), h=h, prec="f64",
                f=blob_source((n, n, n), h, seed=1, nblobs=3, sigma=0.08))


def config_blobs_noise(n, seed):
    """n^3 on the unit cube: 16 blobs sigma ~ U[0.02, 0.1] plus 1e-3 noise."""
    h = 1.0 / n
    return blob_source((n, n, n), h, seed=seed, nblobs=16, sigma=(0.02, 0.1), noise=1e-3)


def config_c2():
    n = 256
    return dict(name="c2", shape=(n, n, n), h=1.0 / n, prec="f64", f=config_blobs_noise(n, 2))


def config_c3(n=512):
    return dict(name="c3", shape=(n, n, n), h=1.0 / n, prec="f32", f=config_blobs_noise(n, 2))


def batch_sizes(seed=4, count=48, lo=32, hi=192):
    """Per-solve (nz, ny, nx) drawn independently from U{lo..hi}."""
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in row) for row in rng.integers(lo, hi + 1, size=(count, 3))]


def config_c4(count=48, seed=4, vec_n=128):
    """Uneven scalar solves plus one 3-component curl source."""
    sizes = batch_sizes(seed, count)
    probs = []
    for i, (nz, ny, nx) in enumerate(sizes):
        h = 1.0 / max(nz, ny, nx)
        f = blob_source((nz, ny, nx), h, seed=seed * 1000 + i, nblobs=16,
                        sigma=(0.02, 0.1), noise=1e-3)
        probs.append(dict(shape=(nz, ny, nx), h=h, f=f))
    hv = 1.0 / vec_n
    vec = dict(shape=(vec_n, vec_n, vec_n), h=hv, f=curl_source(vec_n, hv, seed=seed * 1000 + count))
    return dict(name="c4", prec="f32", scalar=probs, vector=vec)


def config_c5(n=256):
    h = 1.0 / n
    return dict(name="c5", shape=(n, n, n), h=h, prec="f32",
                f=config_blobs_noise(n, 5), w=weight_field(n, h, seed=55))


def vortex_tube_source(n, R=0.3, nz=None):
    """-curl(omega_z e_z) for the vortex tube of radius R on the unit square
    in x and y (n cells each) and nz cells along z (default n, h = 1/n):
    array [3][nz][n][n] with components (x, y, z).  The tube does not
    depend on z."""
    n = int(n)
    nz = n if nz is None else int(nz)
    h = 1.0 / n
    x = cell_centres(n, h) - 0.5
    X, Y = np.meshgrid(x, x, indexing="xy")          # [y][x]
    q = (X * X + Y * Y) / (R * R)
    inside = q < 1.0
    c0 = 1.0 / (2.0 * np.pi) * 2.0 / (R * R) / special.expn(2, 1.0)
    om = np.zeros_like(q)
    om[inside] = c0 * np.exp(-1.0 / (1.0 - q[inside]))
    dg = np.zeros_like(q)                              # d/d(r^2) of -1/(1 - r^2/R^2), times 2
    dg[inside] = -2.0 / (R * R * (1.0 - q[inside]) ** 2)
    fx = -(om * dg * Y)                                # -d omega/dy
    fy = om * dg * X                                   # d omega/dx
    f = np.zeros((3, nz, n, n))
    f[0] = fx[None]
    f[1] = fy[None]
    return f
