"""The multigrid cycle's C ABI on the host (no GPU): hierarchy validation,
work-buffer sizes, state errors, and a host mirror of every kernel's launch
geometry and index formulas (multigrid.hip) showing that each thread's
accesses stay inside its arrays and that each kernel covers exactly the
nodes it must."""
import ctypes as C

import numpy as np
import pytest

from paper_2512_08555_amd import _capi as capi
from paper_2512_08555_amd.lengths import auto_pad
from paper_2512_08555_amd.solver import Multigrid, Plan

BX, BY = 64, 4


def _plan(shape=(20, 18, 22), prec="f64", **kw):
    return Plan(shape, 0.05, prec, setup=False, pad=auto_pad(shape, prec), **kw)


def test_shapes_and_sizes():
    p = _plan()
    mg = Multigrid(p, [((3, 2, 4), (6, 5, 7)), ((2, 3, 2), (4, 3, 5))], setup=False)
    assert mg.shapes == [(20, 18, 22), (13, 11, 15), (9, 7, 11)]
    el = 8
    r256 = lambda v: (v + 255) // 256 * 256
    want = r256(8 * 9)
    want = r256(want + 20 * 18 * 22 * el)
    want = r256(want + 13 * 11 * 15 * el)
    want = r256(want + 13 * 11 * 15 * el)              # the residual, the largest refined level
    want = r256(want + 13 * 11 * 15 * el)              # the smoother's second array of level 1
    want = r256(want + 9 * 7 * 11 * el)                # and of level 2
    want = r256(want + 7 * 6 * 8 * el)
    want = r256(want + 5 * 4 * 6 * el)
    assert mg.work_bytes == want
    assert Multigrid(_plan(prec="f32"), [], setup=False).work_bytes == 256


@pytest.mark.parametrize("patch", [((0, 2, 2), (4, 4, 4)), ((2, 2, 2), (17, 4, 4)), ((2, 2, 2), (1, 4, 4)),
                                   ((2, 2, 19), (4, 4, 2))])
def test_box_outside_its_parent_is_rejected(patch):
    with pytest.raises(capi.UpsError) as ei:
        Multigrid(_plan(), [patch], setup=False)
    assert ei.value.status == capi.UPS_ERR_INVALID_ARG


def test_unsupported_coarse_plans():
    with pytest.raises(capi.UpsError) as ei:
        Multigrid(_plan(green="mehr4"), [((2, 2, 2), (4, 4, 4))], setup=False)
    assert ei.value.status == capi.UPS_ERR_UNSUPPORTED and "7-point" in str(ei.value)
    p3 = _plan(ncomp=3)
    hier = capi.ups_mg_hierarchy()
    h = C.c_void_p()
    assert capi.lib().ups_mg_create(p3._h, C.byref(hier), C.byref(h)) == capi.UPS_ERR_UNSUPPORTED
    hier.levels = capi.UPS_MG_MAX_LEVELS + 1
    assert capi.lib().ups_mg_create(_plan()._h, C.byref(hier), C.byref(h)) == capi.UPS_ERR_UNSUPPORTED
    assert capi.lib().ups_mg_create(None, C.byref(hier), C.byref(h)) == capi.UPS_ERR_INVALID_ARG


def test_cycle_before_setup_is_a_state_error():
    mg = Multigrid(_plan(), [((2, 2, 2), (4, 4, 4))], setup=False)
    arr = (C.c_void_p * 2)(16, 16)
    st = capi.lib().ups_mg_cycle(mg._h, arr, arr, 2, 2, None)
    assert st == capi.UPS_ERR_STATE
    wb = C.c_void_p(256)
    assert capi.lib().ups_mg_setup(mg._h, wb, 0) == capi.UPS_ERR_WORKSPACE
    assert capi.lib().ups_mg_setup(mg._h, C.c_void_p(8), mg.work_bytes) == capi.UPS_ERR_INVALID_ARG


# --- host mirror of the kernels' launch geometry and index formulas ----------------------------

def _threads(grid, block):
    """All (blockIdx, threadIdx) of a launch as flat arrays per component."""
    gx, gy, gz = grid
    bx, by = block
    B = np.stack(np.meshgrid(np.arange(gz), np.arange(gy), np.arange(gx), indexing="ij"), -1).reshape(-1, 3)
    T = np.stack(np.meshgrid(np.arange(by), np.arange(bx), indexing="ij"), -1).reshape(-1, 2)
    bz_, by_, bx_ = [np.repeat(B[:, i], len(T)) for i in range(3)]
    ty, tx = [np.tile(T[:, i], len(B)) for i in range(2)]
    return bx_, by_, bz_, tx, ty


def _grid(nx, ny, nz):
    return ((nx + BX - 1) // BX, (ny + BY - 1) // BY, nz)


HIERARCHIES = [((12, 11, 13), [((3, 2, 4), (4, 5, 4))]),
               ((13, 12, 14), [((3, 3, 3), (6, 5, 7)), ((2, 2, 3), (6, 6, 5))]),
               ((9, 9, 9), [((1, 1, 1), (6, 6, 6))]),
               ((70, 5, 67), [((1, 1, 30), (66, 2, 35))])]


def _levels(n0, patches):
    shapes = [n0]
    for c, m in patches:
        shapes.append(tuple(2 * v + 1 for v in m))
    return shapes


@pytest.mark.parametrize("n0,patches", HIERARCHIES)
def test_ghost_kernel_covers_the_ghost_layer_once(n0, patches):
    for nz, ny, nx in _levels(n0, patches)[1:]:
        plane, ring = nx * ny, 2 * nx + 2 * (ny - 2)
        total = 2 * plane + (nz - 2) * ring
        t = np.arange((total + 255) // 256 * 256)
        t = t[t < total]
        z = np.where(t < plane, 0, nz - 1)
        j = np.where(t < plane, t, t - plane)
        y, x = j // nx, j % nx
        s = t - 2 * plane
        zr = 1 + s // ring
        jr = s - (zr - 1) * ring
        q = jr - 2 * nx
        yr = np.where(jr < nx, 0, np.where(jr < 2 * nx, ny - 1, 1 + (q >> 1)))
        xr = np.where(jr < nx, jr, np.where(jr < 2 * nx, jr - nx, np.where(q & 1, nx - 1, 0)))
        face = t < 2 * plane
        z, y, x = np.where(face, z, zr), np.where(face, y, yr), np.where(face, x, xr)
        hit = np.zeros((nz, ny, nx), int)
        np.add.at(hit, (z, y, x), 1)
        ghost = np.ones((nz, ny, nx), int)
        ghost[1:-1, 1:-1, 1:-1] = 0
        assert np.array_equal(hit, ghost)


def _cubic_reads(x, y, z):
    """Footprint indices (parent node origin + index) the cubic ghost
    reconstruction reads: i0 - 1 .. i0 + 2 along odd axes, i0 along even."""
    reads = []
    for a in range(4):
        for b in range(4):
            for cc in range(4):
                use = ((a == 0) | (x & 1 == 1)) & ((b == 0) | (y & 1 == 1)) & ((cc == 0) | (z & 1 == 1))
                i = (x >> 1) + np.where(x & 1, a - 1, 0)
                j = (y >> 1) + np.where(y & 1, b - 1, 0)
                k = (z >> 1) + np.where(z & 1, cc - 1, 0)
                reads.append((use, i, j, k))
    return reads


@pytest.mark.parametrize("n0,patches", HIERARCHIES)
def test_transfer_kernels_stay_in_bounds(n0, patches):
    shapes = _levels(n0, patches)
    for lev, (c, m) in enumerate(patches):
        pz, py, px = shapes[lev]
        nz, ny, nx = shapes[lev + 1]
        cz, cy, cx = c
        mz, my, mx = m
        # prolongation: one thread per footprint node (i, j, k) writes the fine
        # unknowns 2 (i, j, k) + (a, b, c) (a = 0 only where i = m), never a
        # ghost node, each unknown exactly once; it reads the cell corners.
        # With the ghost kernel it writes every node of the level, which is
        # what lets the cycle prolong into the smoother's scratch array
        bx, by, bz, tx, ty = _threads(_grid(mx + 1, my + 1, mz + 1), (BX, BY))
        k, j, i = bz, by * BY + ty, bx * BX + tx
        ok = (j <= my) & (i <= mx)
        i, j, k = i[ok], j[ok], k[ok]
        hit = np.zeros((nz, ny, nx), int)
        for c_ in (0, 1):
            for b_ in (0, 1):
                for a_ in (0, 1):
                    live = ((a_ == 0) | (i < mx)) & ((b_ == 0) | (j < my)) & ((c_ == 0) | (k < mz))
                    x, y, z = 2 * i + a_, 2 * j + b_, 2 * k + c_
                    zok = (z > 0) & (z < nz - 1) & (y > 0) & (y < ny - 1)
                    xok = np.where(a_ == 0, (i > 0) & (i < mx), True)
                    w = live & zok & xok
                    np.add.at(hit, (z[w], y[w], x[w]), 1)
                    # corners read: (i + a_, j + b_, k + c_) where live
                    assert (i + a_)[live].max() <= mx and (cx + i + a_)[live].max() <= px - 2
                    assert (j + b_)[live].max() <= my and (k + c_)[live].max() <= mz
        inner = np.zeros((nz, ny, nx), int)
        inner[1:-1, 1:-1, 1:-1] = 1
        assert np.array_equal(hit, inner)
        # ghost nodes (ghost kernel): the cubic reads stay in the parent, one
        # node beyond the footprint at most
        zz, yy, xx = np.indices((nz, ny, nx))
        ghost = inner == 0
        x, y, z = xx[ghost], yy[ghost], zz[ghost]
        for use, i2, j2, k2 in _cubic_reads(x, y, z):
            i2, j2, k2 = i2[use], j2[use], k2[use]
            if not i2.size:
                continue
            assert i2.min() >= -1 and j2.min() >= -1 and k2.min() >= -1
            assert i2.max() <= mx + 1 and j2.max() <= my + 1 and k2.max() <= mz + 1
            assert min((cx + i2).min(), (cy + j2).min(), (cz + k2).min()) >= 0
            assert (cx + i2).max() <= px - 1 and (cy + j2).max() <= py - 1 and (cz + k2).max() <= pz - 1
        # restriction: every footprint node; the interior ones read the fine
        # residual around node 2 i and the fine or parent neighbours
        bx, by, bz, tx, ty = _threads(_grid(mx + 1, my + 1, mz + 1), (BX, BY))
        k, j, i = bz, by * BY + ty, bx * BX + tx
        ok = (j <= my) & (i <= mx)
        i, j, k = i[ok], j[ok], k[ok]
        assert len(set(zip(i, j, k))) == (mx + 1) * (my + 1) * (mz + 1)
        inner = (i > 0) & (j > 0) & (k > 0) & (i < mx) & (j < my) & (k < mz)
        fi, fj, fk = 2 * i[inner], 2 * j[inner], 2 * k[inner]
        assert (fi - 1).min() >= 1 and (fi + 1).max() <= nx - 2
        assert (fj - 1).min() >= 1 and (fj + 1).max() <= ny - 2
        assert (fk - 1).min() >= 1 and (fk + 1).max() <= nz - 2
        for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            a, b, cc = i[inner] + di, j[inner] + dj, k[inner] + dk
            assert a.min() >= 0 and a.max() <= mx and b.max() <= my and cc.max() <= mz
            inn = (a > 0) & (b > 0) & (cc > 0) & (a < mx) & (b < my) & (cc < mz)
            assert (2 * a[inn]).max(initial=0) <= nx - 1
            assert (cx + a[~inn]).max(initial=0) <= px - 1 and (cz + cc[~inn]).max(initial=0) <= pz - 1
        # residual and norm: the unknowns of the level
        bx, by, bz, tx, ty = _threads(_grid(nx - 2, ny - 2, nz - 2), (BX, BY))
        z, y, x = bz + 1, by * BY + ty + 1, bx * BX + tx + 1
        ok = (y <= ny - 2) & (x <= nx - 2)
        assert len(set(zip(x[ok], y[ok], z[ok]))) == (nx - 2) * (ny - 2) * (nz - 2)
        assert (z + 1).max() <= nz - 1


@pytest.mark.parametrize("n0,patches", HIERARCHIES)
def test_residual_norm_rows_cover_the_unknowns_once(n0, patches):
    for nz, ny, nx in _levels(n0, patches):
        rows = (ny - 2) * (nz - 2)
        grid = min((rows + BY - 1) // BY, 2048)
        seen = np.zeros((nz, ny), int)
        for blk in range(grid):
            for ty in range(BY):
                r = np.arange(blk * BY + ty, rows, grid * BY)
                z = 1 + r // (ny - 2)
                y = 1 + r - (z - 1) * (ny - 2)
                np.add.at(seen, (z, y), 1)
        want = np.zeros((nz, ny), int)
        want[1:-1, 1:-1] = 1
        assert np.array_equal(seen, want)


# tile shapes of the fused red-black iteration (x width, y height, threads)
GS32 = [(256, 8, 1024), (128, 16, 1024), (64, 16, 512)]
GS64 = [(128, 16, 1024), (64, 16, 512)]


def _chunk_planes(layer, planes, slots):
    """Planes per z chunk: the chunk count n minimises rounds(n) (ceil(planes
    / n) + 8), rounds(n) = ceil(n layer / slots), over n <= planes / 8, the
    first minimum kept."""
    best = None
    for n in range(1, max(1, planes // 8) + 1):
        zc = -(-planes // n)
        cost = -(-(layer * n) // slots) * (zc + 8)
        if best is None or cost < best[0]:
            best = (cost, zc)
    return best[1]


def _chunks(layer, nz):
    # the rule's choice with one and with two resident blocks per CU on 256
    # CUs, and two fixed lengths (coverage holds for any chunk length)
    return sorted({_chunk_planes(layer, nz - 1, 256), _chunk_planes(layer, nz - 1, 512), 7, 32})


def test_chunk_rule():
    # 513^3: 128 tiles per plane, one block per CU -> 2 chunks of 256 planes;
    # 257^3: 32 tiles per plane -> 8 chunks of 32
    assert _chunk_planes(128, 512, 256) == 256
    assert _chunk_planes(32, 256, 256) == 32
    assert _chunk_planes(2048, 512, 256) == 512      # many tiles per plane: one chunk
    assert _chunk_planes(1, 4, 256) == 4              # fewer than 8 planes: one chunk
    for layer in (1, 3, 32, 96, 128, 500):
        for planes in (4, 40, 256, 512, 1000):
            zc = _chunk_planes(layer, planes, 256)
            assert 1 <= zc <= planes and (zc >= 8 or zc == planes)


def _gs_shape(prec, nx):
    # the first shape whose tiles pad the nx - 1 columns from node 1 least
    shapes = GS64 if prec == "f64" else GS32
    padded = [(nx - 2 + tx) // tx * tx for tx, _, _ in shapes]
    return shapes[padded.index(min(padded))]


def test_fused_smoothing_shape_choice():
    assert _gs_shape("f32", 513) == (256, 8, 1024)
    assert _gs_shape("f32", 257) == (256, 8, 1024)
    assert _gs_shape("f32", 385) == (128, 16, 1024)
    assert _gs_shape("f32", 301) == (64, 16, 512)
    assert _gs_shape("f32", 13) == (64, 16, 512)
    assert _gs_shape("f64", 513) == (128, 16, 1024)
    assert _gs_shape("f64", 301) == (64, 16, 512)


def _gs_frame(tx, ty):
    """Frame columns (lx, ly) of width 2 around a tx x ty tile, in the
    order the kernel numbers them (LDS coordinates, halo 2)."""
    ux, uy = tx + 4, ty + 4
    out = []
    for r in range(4 * ux + 4 * ty):
        if r < 2 * ux:
            ly, lx = r // ux, r % ux
        elif r < 4 * ux:
            ly, lx = uy - 2 + (r - 2 * ux) // ux, (r - 2 * ux) % ux
        else:
            r3 = r - 4 * ux
            c = r3 & 3
            ly, lx = 2 + (r3 >> 2), (c if c < 2 else ux - 4 + c)
        out.append((lx, ly))
    return out


@pytest.mark.parametrize("shape", GS32 + GS64[1:])
def test_fused_smoothing_frame_and_lds(shape):
    tx, ty, nt = shape
    ux, uy, hx, hy = tx + 4, ty + 4, tx + 2, ty + 2
    assert tx * ty % nt == 0
    frame = _gs_frame(tx, ty)
    assert len(set(frame)) == len(frame)
    inner = {(2 + e % tx, 2 + e // tx) for e in range(tx * ty)}
    assert inner.isdisjoint(frame) and len(inner) + len(frame) == ux * uy
    # red runs on the halo of 1 (interior plus the frame's inner ring), reads
    # U at +-1 and writes H at (lx - 1, ly - 1); black reads H at +-1
    red = inner | {(lx, ly) for lx, ly in frame if 1 <= lx <= ux - 2 and 1 <= ly <= uy - 2}
    assert len(red) == hx * hy
    for lx, ly in red:
        assert 0 <= lx - 1 and lx + 1 <= ux - 1 and 0 <= ly - 1 and ly + 1 <= uy - 1
        assert 0 <= lx - 1 < hx and 0 <= ly - 1 < hy
    for lx, ly in inner:
        # H index (lx - 1, ly - 1) and its four neighbours
        assert 0 <= lx - 2 and lx <= hx - 1 and 0 <= ly - 2 and ly <= hy - 1
    # f of an outer frame column is read at its nearest halo-1 column
    for lx, ly in frame:
        assert (min(max(lx, 1), ux - 2), min(max(ly, 1), uy - 2)) in red
    # four register slots: plane p in (p - p0) & 3; a step reads p - 2 .. p + 1
    # and loads p + 3 into the slot of p - 1 after its last use
    for k in range(4):
        assert (k + 3) % 4 == (k - 1) % 4 and (k + 2) % 4 == (k - 2) % 4
        assert len({k, (k + 1) % 4, (k + 3) % 4, (k + 2) % 4}) == 4


@pytest.mark.parametrize("n0,patches", HIERARCHIES + [((513, 70, 67), []), ((33, 65, 513), []),
                                                        ((30, 24, 140), [((4, 4, 5), (20, 16, 128))])])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_smoothing_writes_every_node_once(n0, patches, prec):
    # tiles from node 1 by chunks of zc planes from plane 1 (the XCD-aware
    # block order), the ghost faces at index 0 through the frame and the
    # first chunk: every node of the level is written exactly once, and the
    # loads (clamped) and stores stay in the level
    cases = []
    for nz, ny, nx in _levels(n0, patches):
        tx, ty, nt = _gs_shape(prec, nx)
        nty, ntx = (ny - 2 + ty) // ty, (nx - 2 + tx) // tx
        cases += [(nz, ny, nx, zc) for zc in _chunks(nty * ntx, nz)]
    for nz, ny, nx, zc in cases:
        tx, ty, nt = _gs_shape(prec, nx)
        hit = np.zeros((nz, ny, nx), int)
        nty, ntx = (ny - 2 + ty) // ty, (nx - 2 + tx) // tx
        ntiles = nty * ntx * ((nz - 2 + zc) // zc)
        per_xcd = (ntiles + 7) // 8
        frame = np.array(_gs_frame(tx, ty))
        units = []
        for b in range(8 * per_xcd):
            unit = (b % 8) * per_xcd + b // 8
            if unit < ntiles:
                units.append(unit)
        assert sorted(units) == list(range(ntiles))
        for unit in units:
            tyi, txi, tzi = unit % nty, (unit // nty) % ntx, unit // (nty * ntx)
            x0, y0, zs = 1 + txi * tx, 1 + tyi * ty, 1 + tzi * zc
            ze = min(zs + zc, nz)
            x = x0 + np.arange(tx)
            y = y0 + np.arange(ty)
            X, Y = np.meshgrid(x, y, indexing="xy")
            ok = (X < nx) & (Y < ny)
            fx, fy = x0 - 2 + frame[:, 0], y0 - 2 + frame[:, 1]
            fin = (fx >= 0) & (fy >= 0) & (fx < nx) & (fy < ny)
            gh = fin & (((fx == 0) & ((fy >= y0) | (fy == 0)) & (fy < y0 + ty)) | ((fy == 0) & (fx >= x0) & (fx < x0 + tx)))
            planes = list(range(zs, ze)) + ([0] if zs == 1 else [])
            for q in planes:
                np.add.at(hit, (q, Y[ok], X[ok]), 1)
                np.add.at(hit, (q, fy[gh], fx[gh]), 1)
        assert (hit == 1).all(), (nz, ny, nx, np.argwhere(hit != 1)[:5])


# tile shapes of the last pre-smoothing iteration fused with the residual
GR32 = [(128, 16, 1024), (64, 16, 1024)]
GR64 = [(128, 8, 1024), (64, 16, 1024)]


def _gr_shape(prec, nx):
    shapes = GR64 if prec == "f64" else GR32
    padded = [(nx - 2 + tx) // tx * tx for tx, _, _ in shapes]
    return shapes[padded.index(min(padded))]


def _gr_frame(tx, ty, w=3):
    """Frame columns (lx, ly, depth) of width 3 around a tx x ty tile in the
    kernel's order: ring d (the border of the box of (ux - 2d) x (uy - 2d)
    at (d, d)) from the outside in, each as top row, bottom row, then the two
    side columns row by row."""
    ux, uy = tx + 2 * w, ty + 2 * w
    out = []
    for r in range(ux * uy - tx * ty):
        q, wd, hh, dep = r, ux, uy, 0
        while dep < w - 1 and q >= 2 * wd + 2 * (hh - 2):
            q -= 2 * wd + 2 * (hh - 2)
            dep, wd, hh = dep + 1, wd - 2, hh - 2
        if q < wd:
            lx, ly = dep + q, dep
        elif q < 2 * wd:
            lx, ly = dep + q - wd, dep + hh - 1
        else:
            q2 = q - 2 * wd
            lx, ly = dep + (wd - 1 if q2 & 1 else 0), dep + 1 + (q2 >> 1)
        out.append((lx, ly, dep))
    return out


def test_fused_residual_shape_choice():
    assert _gr_shape("f32", 513) == (128, 16, 1024)
    assert _gr_shape("f32", 257) == (128, 16, 1024)
    assert _gr_shape("f32", 301) == (64, 16, 1024)
    assert _gr_shape("f64", 513) == (128, 8, 1024)
    assert _gr_shape("f64", 41) == (64, 16, 1024)


@pytest.mark.parametrize("shape", sorted(set(GR32 + GR64)))
def test_fused_residual_frame_and_lds(shape):
    tx, ty, nt = shape
    ux, uy = tx + 6, ty + 6
    assert tx * ty % nt == 0
    frame = _gr_frame(tx, ty)
    cols = [(lx, ly) for lx, ly, _ in frame]
    assert len(set(cols)) == len(cols)
    inner = {(3 + e % tx, 3 + e // tx) for e in range(tx * ty)}
    assert inner.isdisjoint(cols) and len(inner) + len(cols) == ux * uy
    # a frame column's depth is its distance to the frame's outer border
    for lx, ly, d in frame:
        assert d == min(lx, ly, ux - 1 - lx, uy - 1 - ly) and 0 <= d <= 2
    depth = {(lx, ly): d for lx, ly, d in frame}
    depth.update({c: 3 for c in inner})
    red = [c for c, d in depth.items() if d >= 1]
    black = [c for c, d in depth.items() if d >= 2]
    assert len(red) == (tx + 4) * (ty + 4) and len(black) == (tx + 2) * (ty + 2)
    for lx, ly in red:
        # U (halo 3) at +-1; H written at (lx - 1, ly - 1)
        assert 0 <= lx - 1 and lx + 1 < ux and 0 <= ly - 1 and ly + 1 < uy
        assert 0 <= lx - 1 < tx + 4 and 0 <= ly - 1 < ty + 4
    for lx, ly in black:
        # H read at (lx - 1 +-1, ly - 1 +-1), a red column each; V written at (lx - 2, ly - 2)
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            assert depth[(lx + dx, ly + dy)] >= 1
            assert 0 <= lx - 1 + dx < tx + 4 and 0 <= ly - 1 + dy < ty + 4
        assert 0 <= lx - 2 < tx + 2 and 0 <= ly - 2 < ty + 2
    for lx, ly in inner:
        # the residual reads V at (lx - 2 +-1, ly - 2 +-1), a black column each
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            assert depth[(lx + dx, ly + dy)] >= 2
            assert 0 <= lx - 2 + dx < tx + 2 and 0 <= ly - 2 + dy < ty + 2
    # f is read from depth 1 in; the outer ring reads its inner neighbour's
    for lx, ly, d in frame:
        assert depth[(min(max(lx, 1), ux - 2), min(max(ly, 1), uy - 2))] >= 1
    # register rings: u_in at p - 1 .. p + 2 (plane p + 3 loads into the slot
    # of p - 1 after the red step), f at p - 2 .. p (plane p + 1 loads into the
    # slot of p - 3 after the residual), H at p - 2 .. p, V at p - 3 .. p - 1
    for k in range(4):
        assert (k + 3) % 4 == (k - 1) % 4 and (k + 1) % 4 == (k - 3) % 4


@pytest.mark.parametrize("n0,patches", HIERARCHIES + [((513, 70, 67), []), ((33, 65, 513), []),
                                                        ((30, 24, 140), [((4, 4, 5), (20, 16, 128))])])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_residual_writes_every_node_once(n0, patches, prec):
    # every node of the level gets u once and every unknown gets r once; the
    # steps p0 = zs - 2 .. ze + 1 produce red at p, black at p - 1 and the
    # residual at p - 2, so the chunk's planes zs .. ze - 1 are all reached
    cases = []
    for nz, ny, nx in _levels(n0, patches):
        tx, ty, nt = _gr_shape(prec, nx)
        nty, ntx = (ny - 2 + ty) // ty, (nx - 2 + tx) // tx
        cases += [(nz, ny, nx, zc) for zc in _chunks(nty * ntx, nz)]
    for nz, ny, nx, zc in cases:
        tx, ty, nt = _gr_shape(prec, nx)
        nty, ntx = (ny - 2 + ty) // ty, (nx - 2 + tx) // tx
        hit = np.zeros((nz, ny, nx), int)
        rhit = np.zeros((nz, ny, nx), int)
        ntiles = nty * ntx * ((nz - 2 + zc) // zc)
        frame = np.array([(lx, ly) for lx, ly, _ in _gr_frame(tx, ty)])
        for unit in range(ntiles):
            tyi, txi, tzi = unit % nty, (unit // nty) % ntx, unit // (nty * ntx)
            x0, y0, zs = 1 + txi * tx, 1 + tyi * ty, 1 + tzi * zc
            ze = min(zs + zc, nz)
            X, Y = np.meshgrid(x0 + np.arange(tx), y0 + np.arange(ty), indexing="xy")
            ok = (X < nx) & (Y < ny)
            fx, fy = x0 - 3 + frame[:, 0], y0 - 3 + frame[:, 1]
            fin = (fx >= 0) & (fy >= 0) & (fx < nx) & (fy < ny)
            gh = fin & (((fx == 0) & ((fy >= y0) | (fy == 0)) & (fy < y0 + ty)) | ((fy == 0) & (fx >= x0) & (fx < x0 + tx)))
            p0, pe = zs - 2, ze + 1
            steps = range(p0, pe + 1)
            planes = [p - 1 for p in steps if zs <= p - 1 < ze] + ([0] if 0 in steps else [])
            for q in planes:
                np.add.at(hit, (q, Y[ok], X[ok]), 1)
                np.add.at(hit, (q, fy[gh], fx[gh]), 1)
            unk = ok & (X <= nx - 2) & (Y <= ny - 2)
            for q in [p - 2 for p in steps if zs <= p - 2 < ze and 1 <= p - 2 <= nz - 2]:
                np.add.at(rhit, (q, Y[unk], X[unk]), 1)
        assert (hit == 1).all(), (nz, ny, nx, np.argwhere(hit != 1)[:5])
        want = np.zeros((nz, ny, nx), int)
        want[1:-1, 1:-1, 1:-1] = 1
        assert np.array_equal(rhit, want)
