"""Closed-form solutions used to pin the oracle -- ORACLE, test infrastructure
only (see ``oracle/__init__.py``).

* Gaussian charge: f = A exp(-|x - c|^2 / sigma^2) carries the total source
  Q = A pi^{3/2} sigma^3, and the decaying solution of Lap u = f
  (eq. poisson_problem, sign as printed: G < 0) is
  u = -(Q / (4 pi r)) erf(r / sigma), with u(c) = -Q / (2 pi^{3/2} sigma).
  The paper's own Gaussian (Sec. 4.1) uses the same exp(-|x|^2/sigma^2) form.
* The compact manufactured solution of Sec. 4.2 (unbounded domains):
  u_ref = u_unb(x) u_unb(y) u_unb(z), u_unb(x) = exp[10 (1 - 1/(1 - (2x-1)^2))]
  on (0, 1) and 0 outside, with f = Lap u_ref.  Because u_ref has compact
  support, it *is* the free-space solution for that f.
* The compact vortex tube of Sec. 5 (unbounded in x and y, periodic in z):
  u = (-sin(theta) u_theta, cos(theta) u_theta, 0) about the axis
  x = y = 1/2, u_theta(r) = (1/(2 pi r)) [1 - (1 - (r/R)^2) E_2(1/(1 - (r/R)^2))
  / E_2(1)] inside the tube and 1/(2 pi r) outside: the velocity whose
  Laplacian is -curl(omega e_z) for the tube's vorticity (unit circulation).
"""

from math import pi

import numpy as np
from scipy import special


def gaussian_source(X, Y, Z, center, sigma, amp):
    r2 = (X - center[0]) ** 2 + (Y - center[1]) ** 2 + (Z - center[2]) ** 2
    return amp * np.exp(-r2 / sigma ** 2)


def gaussian_potential(X, Y, Z, center, sigma, amp):
    Q = amp * pi ** 1.5 * sigma ** 3
    r = np.sqrt((X - center[0]) ** 2 + (Y - center[1]) ** 2 + (Z - center[2]) ** 2)
    out = np.empty_like(r)
    small = r < 1e-12 * sigma
    out[small] = -Q / (2.0 * pi ** 1.5 * sigma)
    rs = r[~small]
    out[~small] = -(Q / (4.0 * pi * rs)) * special.erf(rs / sigma)
    return out


def bump_1d(x):
    """u_unb(x) of Sec. 4.2; 0 outside (0, 1)."""
    x = np.asarray(x, dtype=np.float64)
    s = 2.0 * x - 1.0
    out = np.zeros_like(s)
    m = np.abs(s) < 1.0
    sm = s[m]
    out[m] = np.exp(10.0 * (1.0 - 1.0 / (1.0 - sm * sm)))
    return out


def bump_1d_dd(x):
    """d^2 u_unb / dx^2.  With s = 2x - 1 and g(s) = 10 (1 - 1/(1 - s^2)):
    g' = -20 s / (1 - s^2)^2, g'' = -20 (1 + 3 s^2) / (1 - s^2)^3 and
    u'' = 4 (g'' + g'^2) e^g."""
    x = np.asarray(x, dtype=np.float64)
    s = 2.0 * x - 1.0
    out = np.zeros_like(s)
    m = np.abs(s) < 1.0
    sm = s[m]
    q = 1.0 - sm * sm
    g = 10.0 * (1.0 - 1.0 / q)
    g1 = -20.0 * sm / q ** 2
    g2 = -20.0 * (1.0 + 3.0 * sm * sm) / q ** 3
    out[m] = 4.0 * (g2 + g1 * g1) * np.exp(g)
    return out


def bump_solution(x, y, z):
    """u_ref on the tensor grid x (len Nx), y, z -> array [z, y, x]."""
    ux, uy, uz = bump_1d(x), bump_1d(y), bump_1d(z)
    return uz[:, None, None] * uy[None, :, None] * ux[None, None, :]


def bump_source(x, y, z):
    """f = Lap u_ref = u_x'' u_y u_z + u_x u_y'' u_z + u_x u_y u_z''."""
    ux, uy, uz = bump_1d(x), bump_1d(y), bump_1d(z)
    dx, dy, dz = bump_1d_dd(x), bump_1d_dd(y), bump_1d_dd(z)
    return (uz[:, None, None] * uy[None, :, None] * dx[None, None, :]
            + uz[:, None, None] * dy[None, :, None] * ux[None, None, :]
            + dz[:, None, None] * uy[None, :, None] * ux[None, None, :])


def vortex_tube_velocity(n, R=0.3, nz=None):
    """u of the vortex tube on the cell-centred grid (n cells in x and y,
    nz along z, h = 1/n): array [3][nz][n][n], components (x, y, z)."""
    n = int(n)
    nz = n if nz is None else int(nz)
    x = (np.arange(n) + 0.5) / n - 0.5
    X, Y = np.meshgrid(x, x, indexing="xy")
    r = np.sqrt(X * X + Y * Y)
    q = (r / R) ** 2
    ut = 1.0 / (2.0 * pi * r)
    inside = q < 1.0
    a = 1.0 - q[inside]
    ut[inside] *= 1.0 - a * special.expn(2, 1.0 / a) / special.expn(2, 1.0)
    u = np.zeros((3, nz, n, n))
    u[0] = (-(Y / r) * ut)[None]
    u[1] = ((X / r) * ut)[None]
    return u
