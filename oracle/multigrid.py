r"""The multigrid V(eta1, eta2) cycle around the unbounded solve (Sec. 3.1,
Alg. amg_vcycle) -- ORACLE, test infrastructure only (see
``oracle/__init__.py``).

Grid hierarchy (the uniform-block reading of Sec. 3.1 and Fig.
grid_hierarchy): level 0 is a uniform node grid of shape n0 = (nz, ny, nx)
and spacing h0 that covers the whole domain; level k >= 1 is one box of
nodes at spacing h_k = h0 / 2^k that refines a part of level k - 1.  Patch k
is given by its origin c_k (a node of level k - 1, per axis z, y, x) and its
extent m_k in cells of level k - 1, so it holds 2 m_k + 1 nodes per axis and
its node 2 i lies on node c_k + i of its parent.  Its outer layer of nodes
is ghost data, reconstructed from the parent; the nodes inside are its
unknowns.  The patch lies strictly inside the
parent's unknowns: 1 <= c_k and c_k + m_k <= n_{k-1} - 2 (for level 0 every
node is an unknown of the direct solve, the same bound keeps the stencils
of the footprint inside the grid).  Arrays are indexed [z, y, x].

Operators (Sec. 3.1):

* Laplacian: the 7-point stencil of eq. cross_discr2 at spacing h_k;
* smooth: one Gauss-Seidel iteration on the unknowns, red-black ordered
  (red = nodes with an even index sum in the patch frame, updated first);
* residual r = f - Lap u on the unknowns;
* restriction of r: full weighting, the tensor product of (1/4)[1 2 1];
* restriction of u: injection;
* prolongation of the correction: trilinear;
* ghost reconstruction at the resolution jump: the paper keeps it apart from
  the prolongation and describes it as a (higher-order) polynomial
  interpolation; it is read here as the 4-point cubic interpolation
  (-1, 9, 9, -1)/16 at every odd fine index, one axis at a time, from the
  parent's values on the footprint extended by one node on every side.
  (Trilinear ghost values leave an O(1) truncation error on the layer next
  to the jump and make the composite solution first order; the cubic ones
  keep it second order.)

One cycle (full-approximation scheme), for k = l .. 1: fill the ghosts of u_k
from u_{k-1}, eta1 smoothing steps, r_k = f_k - Lap u_k, then on the
unknowns of the parent inside the footprint of patch k (parent nodes
c_k + 1 .. c_k + m_k - 1) u_{k-1} = injection of u_k, r_{k-1} = full
weighting of r_k, f_{k-1} = r_{k-1} + Lap u_{k-1}; store u_{k-1} on the whole
footprint (c_k .. c_k + m_k) as u_hat_{k-1}.  Level 0 is then solved directly
with the unbounded FFT convolution (any kernel callable may stand in).
For k = 1 .. l: the correction e = u_{k-1} - u_hat_{k-1} (new minus stored;
the algorithm prints the difference the other way round, which would move
u_k away from the coarse solution), u_k += trilinear prolongation of e on
the unknowns, ghosts from u_{k-1}, eta2 smoothing steps.  The sources f_k the
caller gives are not modified: each cycle works on copies, whose values in
a child's footprint are replaced by the restriction.

The converged composite solution satisfies, at every level, the 7-point
equation at each unknown outside the interior of the child's footprint,
injection consistency inside it, and ghost layers equal to the cubic
reconstruction from the parent; ``composite_dense`` solves that system
directly for pins.
"""

import numpy as np

from .lgf import lgf_table
from .solve import solve as unbounded_solve


# --- geometry --------------------------------------------------------------------------

def level_shapes(n0, patches):
    """Node shapes of levels 0 .. l; patches = [(origin(z,y,x), cells(z,y,x)), ...]."""
    shapes = [tuple(int(v) for v in n0)]
    for k, (c, m) in enumerate(patches):
        parent = shapes[-1]
        for a in range(3):
            if int(m[a]) < 2:
                raise ValueError("patch %d: at least 2 parent cells per axis" % (k + 1))
            if int(c[a]) < 1 or int(c[a]) + int(m[a]) > parent[a] - 2:
                raise ValueError("patch %d must lie strictly inside the unknowns of its parent" % (k + 1))
        shapes.append(tuple(2 * int(v) + 1 for v in m))
    return shapes


def spacings(h0, levels):
    return [float(h0) / 2 ** k for k in range(levels + 1)]


def _fp(c, m, inner):
    """Slices of the footprint of a patch in its parent: the whole footprint
    (c .. c + m) or its interior (c + 1 .. c + m - 1)."""
    if inner:
        return tuple(slice(int(ci) + 1, int(ci) + int(mi)) for ci, mi in zip(c, m))
    return tuple(slice(int(ci), int(ci) + int(mi) + 1) for ci, mi in zip(c, m))


# --- operators ----------------------------------------------------------------------------

def laplacian(u, h):
    """(1/h^2) times the 7-point stencil at the nodes whose six neighbours lie
    in the array: shape n - 2 per axis."""
    c = u[1:-1, 1:-1, 1:-1]
    s = (u[2:, 1:-1, 1:-1] + u[:-2, 1:-1, 1:-1] + u[1:-1, 2:, 1:-1] + u[1:-1, :-2, 1:-1]
         + u[1:-1, 1:-1, 2:] + u[1:-1, 1:-1, :-2] - 6.0 * c)
    return s / (h * h)


def residual(u, f, h):
    """r = f - Lap u on the unknowns, 0 on the ghost layer."""
    r = np.zeros_like(u)
    r[1:-1, 1:-1, 1:-1] = f[1:-1, 1:-1, 1:-1] - laplacian(u, h)
    return r


def _color_mask(shape, color):
    z, y, x = np.indices(shape)
    return ((z + y + x) % 2) == color


def smooth(u, f, h):
    """One red-black Gauss-Seidel iteration in place: each unknown of one
    colour is set to the value that zeroes its own residual, red first."""
    inner = tuple(slice(1, -1) for _ in range(3))
    for color in (0, 1):
        m = _color_mask(u.shape, color)[inner]
        nb = (u[2:, 1:-1, 1:-1] + u[:-2, 1:-1, 1:-1] + u[1:-1, 2:, 1:-1] + u[1:-1, :-2, 1:-1]
              + u[1:-1, 1:-1, 2:] + u[1:-1, 1:-1, :-2])
        new = (nb - h * h * f[inner]) / 6.0
        c = u[inner]
        c[m] = new[m]
    return u


def prolong(e):
    """Trilinear interpolation from (m + 1) coarse nodes to 2 m + 1 fine
    nodes per axis: even fine nodes take the coarse value, odd ones the mean
    of their two coarse neighbours, axis by axis."""
    out = np.asarray(e, dtype=np.float64)
    for a in range(3):
        n = out.shape[a]
        shp = list(out.shape)
        shp[a] = 2 * n - 1
        fine = np.zeros(shp)
        ev = [slice(None)] * 3
        ev[a] = slice(0, None, 2)
        od = [slice(None)] * 3
        od[a] = slice(1, None, 2)
        lo = [slice(None)] * 3
        lo[a] = slice(0, n - 1)
        hi = [slice(None)] * 3
        hi[a] = slice(1, n)
        fine[tuple(ev)] = out
        fine[tuple(od)] = 0.5 * (out[tuple(lo)] + out[tuple(hi)])
        out = fine
    return out


def restrict_full_weighting(r):
    """(1/4)[1 2 1] in each direction, evaluated at the fine nodes 2 i,
    i = 1 .. m - 1: shape m - 1 per axis for 2 m + 1 fine nodes."""
    out = np.asarray(r, dtype=np.float64)
    for a in range(3):
        n = out.shape[a]
        c = [slice(None)] * 3
        c[a] = slice(2, n - 2, 2)
        lo = [slice(None)] * 3
        lo[a] = slice(1, n - 3, 2)
        hi = [slice(None)] * 3
        hi[a] = slice(3, n - 1, 2)
        out = 0.25 * out[tuple(lo)] + 0.5 * out[tuple(c)] + 0.25 * out[tuple(hi)]
    return out


def inject(u):
    """Injection: the fine values at the nodes 2 i, i = 1 .. m - 1."""
    return u[2:-2:2, 2:-2:2, 2:-2:2]


def correction(u_coarse, u_hat):
    """The coarse-grid correction: new coarse values minus the stored ones."""
    return u_coarse - u_hat


def interp_cubic(E):
    """From (m + 3) parent nodes per axis (the footprint and one node beyond
    it on each side) to the 2 m + 1 fine nodes of the footprint: even fine
    nodes take the parent value, odd ones (-1, 9, 9, -1)/16 of the four
    nearest parent values; axis by axis, z, then y, then x."""
    out = np.asarray(E, dtype=np.float64)
    for a in range(3):
        n = out.shape[a]
        m = n - 3

        def sl(lo, hi):
            s = [slice(None)] * 3
            s[a] = slice(lo, hi)
            return tuple(s)
        core = out[sl(1, n - 1)]
        mid = (-out[sl(0, m)] + 9.0 * out[sl(1, m + 1)] + 9.0 * out[sl(2, m + 2)] - out[sl(3, m + 3)]) / 16.0
        shp = list(core.shape)
        shp[a] = 2 * m + 1
        fine = np.zeros(shp)
        ev = [slice(None)] * 3
        ev[a] = slice(0, None, 2)
        od = [slice(None)] * 3
        od[a] = slice(1, None, 2)
        fine[tuple(ev)] = core
        fine[tuple(od)] = mid
        out = fine
    return out


def _fp_ext(c, m):
    """The footprint extended by one parent node on every side."""
    return tuple(slice(int(ci) - 1, int(ci) + int(mi) + 2) for ci, mi in zip(c, m))


def fill_ghosts(u_fine, u_parent, c, m):
    """Ghost layer of a patch = cubic reconstruction from its parent."""
    p = interp_cubic(u_parent[_fp_ext(c, m)])
    for a in range(3):
        for side in (0, -1):
            s = [slice(None)] * 3
            s[a] = side
            u_fine[tuple(s)] = p[tuple(s)]
    return u_fine


# --- the cycle ------------------------------------------------------------------------------

def default_coarse_solve(f0, h0):
    return unbounded_solve(f0, h0)


def vcycle(us, fs, patches, h0, nu1=2, nu2=2, coarse_solve=None):
    """One V(nu1, nu2) cycle in place on us (list of level arrays); fs are the
    sources sampled on every level (not modified).  Returns us."""
    coarse_solve = default_coarse_solve if coarse_solve is None else coarse_solve
    lv = len(patches)
    hs = spacings(h0, lv)
    F = [np.array(f, dtype=np.float64) for f in fs]
    uhat = [None] * lv
    for k in range(lv, 0, -1):
        c, m = patches[k - 1]
        fill_ghosts(us[k], us[k - 1], c, m)
        for _ in range(nu1):
            smooth(us[k], F[k], hs[k])
        r = residual(us[k], F[k], hs[k])
        inner = _fp(c, m, True)
        us[k - 1][inner] = inject(us[k])
        rc = restrict_full_weighting(r)
        # Lap u_{k-1} at the footprint interior, after the injection
        lap = laplacian(us[k - 1][_fp(c, m, False)], hs[k - 1])
        F[k - 1][inner] = rc + lap
        uhat[k - 1] = us[k - 1][_fp(c, m, False)].copy()
    us[0][...] = coarse_solve(F[0], hs[0])
    for k in range(1, lv + 1):
        c, m = patches[k - 1]
        e = correction(us[k - 1][_fp(c, m, False)], uhat[k - 1])
        us[k][1:-1, 1:-1, 1:-1] += prolong(e)[1:-1, 1:-1, 1:-1]
        fill_ghosts(us[k], us[k - 1], c, m)
        for _ in range(nu2):
            smooth(us[k], F[k], hs[k])
    return us


def composite_residuals(us, fs, patches, h0):
    """Max |f_k - Lap u_k| per level over the unknowns that lie outside the
    interior of the child's footprint (level 0: its nodes whose neighbours
    are in the grid), after the ghosts are refreshed from the parents."""
    lv = len(patches)
    hs = spacings(h0, lv)
    for k in range(1, lv + 1):
        c, m = patches[k - 1]
        fill_ghosts(us[k], us[k - 1], c, m)
    out = []
    for k in range(lv + 1):
        r = np.abs(residual(us[k], np.asarray(fs[k], dtype=np.float64), hs[k]))
        if k < lv:
            r[_fp(*patches[k], True)] = 0.0
        out.append(float(r.max()))
    return out


def solve(fs, patches, h0, cycles, nu1=2, nu2=2, us=None, coarse_solve=None):
    """`cycles` V-cycles from zero (or from us); returns the level arrays."""
    shapes = level_shapes(fs[0].shape, patches)
    if us is None:
        us = [np.zeros(s) for s in shapes]
    for _ in range(cycles):
        vcycle(us, fs, patches, h0, nu1, nu2, coarse_solve)
    return us


# --- the composite system, directly (small grids; for pins) ---------------------------

def composite_dense(fs, patch, h0):
    """The fixed point of the cycle for one refined level, by a dense solve
    of the composite equations:

      u_0 = h0^2 G1 * F_0 on level 0, F_0 = f_0 off the footprint interior and
            free on it;
      u_0 = u_1 (injection) on the footprint interior;
      Lap u_1 = f_1 at the unknowns of level 1, whose ghost layer is the
            cubic reconstruction from u_0.

    Returns (u_0, u_1)."""
    f0 = np.asarray(fs[0], dtype=np.float64)
    f1 = np.asarray(fs[1], dtype=np.float64)
    c, m = patch
    n0 = f0.shape
    n1 = level_shapes(n0, [patch])[1]
    h1 = h0 / 2.0
    N0 = int(np.prod(n0))
    inner = _fp(c, m, True)
    fp_idx = np.arange(N0).reshape(n0)[inner].ravel()
    nF = fp_idx.size
    ui = tuple(s - 2 for s in n1)
    nU = int(np.prod(ui))
    ntot = N0 + nF + nU
    A = np.zeros((ntot, ntot))
    b = np.zeros(ntot)
    # rows 0 .. N0-1: u_0 - h0^2 G * F_0(free) = h0^2 G * f_0(fixed)
    G = lgf_table(*n0)
    pos = np.indices(n0).reshape(3, -1).T
    A[np.arange(N0), np.arange(N0)] = 1.0
    for j, q in enumerate(fp_idx):
        d = np.abs(pos - pos[q])
        A[:N0, N0 + j] = -h0 * h0 * G[d[:, 0], d[:, 1], d[:, 2]]
    fixed = f0.copy()
    fixed[inner] = 0.0
    b[:N0] = unbounded_solve(fixed, h0).ravel()
    # rows N0 .. N0+nF-1: u_0[footprint interior] - u_1[2 i] = 0
    fine_id = -np.ones(n1, dtype=np.int64)
    fine_id[1:-1, 1:-1, 1:-1] = np.arange(nU).reshape(ui)
    inj = fine_id[2:-2:2, 2:-2:2, 2:-2:2].ravel()
    for j, q in enumerate(fp_idx):
        A[N0 + j, q] = 1.0
        A[N0 + j, N0 + nF + inj[j]] = -1.0
    # rows N0+nF ..: Lap u_1 = f_1; ghost values are linear in u_0
    full = np.arange(N0).reshape(n0)[_fp_ext(c, m)]
    Pmat = np.zeros(tuple(n1) + (full.size,))
    for t in range(full.size):
        e = np.zeros(full.size)
        e[t] = 1.0
        Pmat[..., t] = interp_cubic(e.reshape(full.shape))
    col_of = full.ravel()
    row0 = N0 + nF
    inv_h2 = 1.0 / (h1 * h1)
    for idx in np.ndindex(*ui):
        i = tuple(v + 1 for v in idx)
        row = row0 + fine_id[i]
        b[row] = f1[i]
        for d, w in (((0, 0, 0), -6.0), ((1, 0, 0), 1.0), ((-1, 0, 0), 1.0), ((0, 1, 0), 1.0),
                     ((0, -1, 0), 1.0), ((0, 0, 1), 1.0), ((0, 0, -1), 1.0)):
            nb = (i[0] + d[0], i[1] + d[1], i[2] + d[2])
            if fine_id[nb] >= 0:
                A[row, row0 + fine_id[nb]] += w * inv_h2
            else:
                A[row, col_of] += w * inv_h2 * Pmat[nb]
    x = np.linalg.solve(A, b)
    u0 = x[:N0].reshape(n0)
    u1 = np.zeros(n1)
    u1[1:-1, 1:-1, 1:-1] = x[row0:].reshape(ui)
    fill_ghosts(u1, u0, c, m)
    return u0, u1
