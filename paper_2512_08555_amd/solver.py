"""Python face of libups: plans bound to torch device memory and streams.

Arrays are torch tensors on the current HIP device, indexed [z, y, x] (or
[c, z, y, x] for ncomp > 1), float64 for prec="f64" and float32 for "f32".
Every numeric step runs in the library's HIP kernels; this module only
allocates buffers with torch and passes pointers and the current stream.
"""
import ctypes as C

import torch

from . import _capi as capi

PASS_NAMES = ("xfwd", "yfwd", "zconv", "yinv", "xinv")


def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


BC_CODES = {"unb": capi.UPS_BC_UNB, "per": capi.UPS_BC_PER, "even": capi.UPS_BC_EVEN, "odd": capi.UPS_BC_ODD}


GREEN_CODES = {"lgf2": capi.UPS_GREEN_LGF2, "mehr4": capi.UPS_GREEN_LGF4_MEHR, "mehr6": capi.UPS_GREEN_LGF6_MEHR}


def make_problem(shape, h, prec="f64", ncomp=1, pad=None, bc=None, green="lgf2"):
    """ups_problem for a grid of shape (nz, ny, nx) with isotropic spacing h;
    bc: None (unbounded everywhere) or one of "unb", "per", "even", "odd"
    per axis in (z, y, x) order, the same on both sides of the axis; green:
    "lgf2" (7-point operator), "mehr4" or "mehr6" (the Mehrstellen pairs)."""
    nz, ny, nx = (int(v) for v in shape)
    p = capi.ups_problem()
    capi.lib().ups_problem_init(C.byref(p))
    p.n[0], p.n[1], p.n[2] = nx, ny, nz
    for i in range(3):
        p.h[i] = float(h)
    p.prec = capi.UPS_F64 if prec == "f64" else capi.UPS_F32
    p.ncomp = int(ncomp)
    if pad is not None:
        mz, my, mx = (int(v) for v in pad)
        p.pad[0], p.pad[1], p.pad[2] = mx, my, mz
    p.green = GREEN_CODES[green] if isinstance(green, str) else int(green)
    if bc is not None:
        codes = [BC_CODES[b] if isinstance(b, str) else int(b) for b in bc]
        for axis, code in zip((2, 1, 0), codes):   # (z, y, x) -> ABI axis index
            p.bc[axis][0] = p.bc[axis][1] = code
    return p


class Plan:
    """A solve u = h^2 G1 * f on one grid (see include/ups.h).

    Plan(shape, h, prec) validates and sizes the problem; setup() (called
    by the constructor unless setup=False) allocates the green and work
    buffers with torch on the current device and builds G_hat."""

    def __init__(self, shape, h, prec="f64", ncomp=1, pad=None, setup=True, problem=None, bc=None, green="lgf2"):
        self.shape = tuple(int(v) for v in shape)
        self.h = float(h)
        self.prec = prec
        self.ncomp = int(ncomp)
        self.bc = tuple(bc) if bc is not None else ("unb",) * 3
        self.dtype = torch.float64 if prec == "f64" else torch.float32
        L = capi.lib()
        self._prob = problem if problem is not None else make_problem(self.shape, h, prec, ncomp, pad, bc, green)
        handle = C.c_void_p()
        capi.check(L.ups_plan_create(C.byref(self._prob), C.byref(handle)))
        self._h = handle
        gb, wb = C.c_size_t(), C.c_size_t()
        capi.check(L.ups_plan_sizes(self._h, C.byref(gb), C.byref(wb)))
        self.green_bytes, self.work_bytes = gb.value, wb.value
        self.green = None
        self.work = None
        if setup:
            self.setup()

    # -- lifecycle --------------------------------------------------------------
    def setup(self, device=None, stream=None):
        dev = torch.device("cuda") if device is None else torch.device(device)
        self.green = torch.empty(self.green_bytes, dtype=torch.uint8, device=dev)
        self.work = torch.empty(self.work_bytes, dtype=torch.uint8, device=dev)
        capi.check(capi.lib().ups_plan_setup(self._h, C.c_void_p(self.green.data_ptr()), self.green_bytes,
                                             C.c_void_p(self.work.data_ptr()), self.work_bytes,
                                             _stream_handle(stream)))
        return self

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().ups_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- solves -----------------------------------------------------------------
    def _shape_io(self):
        return self.shape if self.ncomp == 1 else (self.ncomp,) + self.shape

    def _check(self, t, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA/HIP tensor" % name)
        if t.dtype != self.dtype or tuple(t.shape) != self._shape_io() or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor of shape %s" % (name, self.dtype, self._shape_io()))

    def empty_like_io(self):
        return torch.empty(self._shape_io(), dtype=self.dtype, device=self.work.device)

    def solve(self, f, out=None, stream=None):
        """u = h^2 G1 * f (forward solve); out may be f (in place)."""
        self._check(f, "f")
        u = self.empty_like_io() if out is None else out
        self._check(u, "out")
        capi.check(capi.lib().ups_solve(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()),
                                        _stream_handle(stream)))
        return u

    def solve_noalloc(self, f, out=None, stream=None):
        """u = h^2 G1 * f through ups_solve_noalloc: W in the library's own
        per-device array instead of the plan's work buffer (plans whose W
        fits in UPS_NOALLOC_MAX_WORK bytes)."""
        self._check(f, "f")
        u = self.empty_like_io() if out is None else out
        self._check(u, "out")
        capi.check(capi.lib().ups_solve_noalloc(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()),
                                                _stream_handle(stream)))
        return u

    def adjoint(self, g, out=None, stream=None):
        """grad_f = K^T grad_u through ups_solve_adjoint."""
        self._check(g, "grad_u")
        r = self.empty_like_io() if out is None else out
        self._check(r, "out")
        capi.check(capi.lib().ups_solve_adjoint(self._h, C.c_void_p(g.data_ptr()), C.c_void_p(r.data_ptr()),
                                                _stream_handle(stream)))
        return r

    def run_pass(self, k, f=None, u=None, stream=None):
        """Enqueue pass k (0..4) alone on the bound work buffer (pass 0 reads f,
        pass 4 writes u)."""
        if (k == 0 and f is None) or (k == 4 and u is None):
            raise ValueError("pass 0 needs f and pass 4 needs u")
        fi = C.c_void_p(f.data_ptr()) if f is not None else C.c_void_p(None)
        uo = C.c_void_p(u.data_ptr()) if u is not None else C.c_void_p(None)
        capi.check(capi.lib().ups_run_pass(self._h, int(k), fi, uo, _stream_handle(stream)))

    def set_check_finite(self, enable=True):
        """Scan every input for NaN / Inf before solving (UpsError
        UPS_ERR_NONFINITE if one is found); off by default."""
        capi.check(capi.lib().ups_plan_set_check_finite(self._h, int(bool(enable))))

    @property
    def nyquist_packed(self):
        """Whether W's column 0 carries X[0] + i X[mx/2] (ups_plan_nyquist_packed)."""
        return capi.lib().ups_plan_nyquist_packed(self._h) == 1

    @property
    def guard_mode(self):
        """Whether the plan was created with UPS_DEBUG_GUARDS set."""
        return capi.lib().ups_plan_guard_mode(self._h) == 1

    # -- introspection ---------------------------------------------------------
    def layout(self):
        pitch, plane, comp = C.c_int(), C.c_longlong(), C.c_longlong()
        goff, gplane = C.c_size_t(), C.c_longlong()
        capi.check(capi.lib().ups_plan_layout(self._h, C.byref(pitch), C.byref(plane), C.byref(comp),
                                              C.byref(goff), C.byref(gplane)))
        return dict(pitch=pitch.value, plane=plane.value, comp_stride=comp.value,
                    ghat_offset=goff.value, ghat_plane=gplane.value)

    def kernel(self, k):
        s = capi.lib().ups_plan_kernel(self._h, int(k))
        return s.decode() if s else None

    def set_kernel(self, k, name):
        capi.check(capi.lib().ups_plan_set_kernel(self._h, int(k), name.encode()))

    @property
    def slab(self):
        """kx columns per slab of the column passes (0: one slab)."""
        return capi.lib().ups_plan_slab(self._h)

    @slab.setter
    def slab(self, columns):
        capi.check(capi.lib().ups_plan_set_slab(self._h, int(columns)))

    def set_side_stream(self, enable):
        """Run the narrow remainder launches (one slab) or the z passes of the
        slabs (several) on a second stream, or keep every launch on the
        caller's stream."""
        capi.check(capi.lib().ups_plan_set_side_stream(self._h, int(bool(enable))))

    @property
    def side_stream(self):
        """Whether the plan uses its second stream."""
        return capi.lib().ups_plan_side_stream(self._h) == 1

    def model_bytes(self, k=-1):
        return capi.lib().ups_plan_model_bytes(self._h, int(k))

    @property
    def padded(self):
        p = self._prob
        mx = p.pad[0] or 2 * p.n[0]
        my = p.pad[1] or 2 * p.n[1]
        mz = p.pad[2] or 2 * p.n[2]
        return (mz, my, mx)

    def ghat(self):
        """Copy of G_hat (octant [iz, iy, kx], plan precision) read from the green
        buffer, for inspection.  The buffer holds it as [iy][kx][iz] with the iz
        pitch ghat_plane / kx."""
        lay = self.layout()
        mz, my, mx = self.padded
        oz, oy, kx = mz // 2 + 1, my // 2 + 1, mx // 2 + 1
        esz = 8 if self.prec == "f64" else 4
        gz = lay["ghat_plane"] // kx
        n = oy * lay["ghat_plane"]
        raw = self.green[lay["ghat_offset"]: lay["ghat_offset"] + n * esz].view(self.dtype)
        g = raw.view(oy, kx, gz)[:, :, :oz]
        return g.permute(2, 0, 1).contiguous()

    def work_complex(self):
        """The work buffer viewed as complex [c][z][y][pitch] (plan precision)."""
        lay = self.layout()
        ct = torch.complex128 if self.prec == "f64" else torch.complex64
        nz = self.shape[0]
        n = self.ncomp * lay["comp_stride"]
        esz = 16 if self.prec == "f64" else 8
        off = capi.lib().ups_plan_work_offset(self._h)
        w = self.work[off: off + n * esz].view(ct)
        my = lay["plane"] // lay["pitch"]
        return w.view(self.ncomp, nz, my, lay["pitch"])


def kernel_variants(k, prec, length, fill=False):
    """Names of the compiled kernel variants of pass k for a padded length
    (fill: the mirrored-fill forward variants of an even or odd direction)."""
    L = capi.lib()
    p = capi.UPS_F64 if prec == "f64" else capi.UPS_F32
    fn = L.ups_kernel_fill_variants if fill else L.ups_kernel_variants
    n = fn(int(k), p, int(length), None, 0)
    arr = (C.c_char_p * max(n, 1))()
    fn(int(k), p, int(length), arr, n)
    return [arr[i].decode() for i in range(n)]


def solve(f, h, prec=None, pad=None):
    """One-shot solve of a [z, y, x] (or [c, z, y, x] with c = 3) tensor."""
    prec = prec or ("f64" if f.dtype == torch.float64 else "f32")
    ncomp = 1 if f.dim() == 3 else f.shape[0]
    shape = tuple(f.shape[-3:])
    return Plan(shape, h, prec, ncomp=ncomp, pad=pad).solve(f.contiguous())


def _plan_autotune(self, budget_ms=200.0, f=None, stream=None):
    """Time every compiled variant of each pass on this plan (ups_autotune),
    solving from f (a random source of the plan's shape if None) into a
    separate output array, and keep the fastest; returns the chosen kernel
    names."""
    if f is None:
        g = torch.Generator(device=self.work.device).manual_seed(0)
        f = torch.randn(self._shape_io(), dtype=self.dtype, device=self.work.device, generator=g)
    self._check(f, "f")
    u = self.empty_like_io()
    capi.check(capi.lib().ups_autotune(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()),
                                       _stream_handle(stream), float(budget_ms)))
    return [self.kernel(k) for k in range(5)]


Plan.autotune = _plan_autotune


class Batch:
    """Many independent solves (uneven shapes, vector right-hand sides) run
    as one hipGraph launch (ups_batch_*).

    specs: list of dicts {shape: (nz, ny, nx), h, prec, ncomp, pad, bc}."""

    def __init__(self, specs, setup=True):
        from .lengths import auto_pad
        L = capi.lib()
        self.specs = []
        probs = (capi.ups_problem * len(specs))()
        for i, sp in enumerate(specs):
            shape = tuple(int(v) for v in sp["shape"])
            prec = sp.get("prec", "f32")
            ncomp = int(sp.get("ncomp", 1))
            bc = sp.get("bc")
            pad = sp.get("pad") or auto_pad(shape, prec)
            probs[i] = make_problem(shape, sp["h"], prec, ncomp, pad, bc)
            self.specs.append(dict(shape=shape, h=float(sp["h"]), prec=prec, ncomp=ncomp, pad=tuple(pad),
                                   bc=tuple(bc) if bc is not None else ("unb",) * 3))
        handle = C.c_void_p()
        capi.check(L.ups_batch_create(probs, len(specs), C.byref(handle)))
        self._h = handle
        self._probs = probs
        gb, wb = C.c_size_t(), C.c_size_t()
        capi.check(L.ups_batch_sizes(self._h, C.byref(gb), C.byref(wb)))
        self.green_bytes, self.work_bytes = gb.value, wb.value
        self.green = self.work = None
        if setup:
            self.setup()

    def setup(self, device=None, stream=None):
        dev = torch.device("cuda") if device is None else torch.device(device)
        self.green = torch.empty(self.green_bytes, dtype=torch.uint8, device=dev)
        self.work = torch.empty(self.work_bytes, dtype=torch.uint8, device=dev)
        capi.check(capi.lib().ups_batch_setup(self._h, C.c_void_p(self.green.data_ptr()), self.green_bytes,
                                              C.c_void_p(self.work.data_ptr()), self.work_bytes,
                                              _stream_handle(stream)))
        return self

    def launches(self):
        return [capi.lib().ups_batch_launches(self._h, k) for k in range(5)]

    def empty_outputs(self):
        out = []
        for sp in self.specs:
            dt = torch.float64 if sp["prec"] == "f64" else torch.float32
            shape = sp["shape"] if sp["ncomp"] == 1 else (sp["ncomp"],) + sp["shape"]
            out.append(torch.empty(shape, dtype=dt, device=self.work.device))
        return out

    def solve(self, fs, us=None, stream=None):
        n = len(self.specs)
        if len(fs) != n:
            raise ValueError("expected %d source arrays" % n)
        us = self.empty_outputs() if us is None else us
        for f, u, sp in zip(fs, us, self.specs):
            dt = torch.float64 if sp["prec"] == "f64" else torch.float32
            shape = sp["shape"] if sp["ncomp"] == 1 else (sp["ncomp"],) + sp["shape"]
            for t in (f, u):
                if not t.is_cuda or t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous():
                    raise ValueError("batch array must be a contiguous %s tensor of shape %s" % (dt, shape))
        fp = (C.c_void_p * n)(*[f.data_ptr() for f in fs])
        up = (C.c_void_p * n)(*[u.data_ptr() for u in us])
        capi.check(capi.lib().ups_batch_solve(self._h, fp, up, _stream_handle(stream)))
        return us

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().ups_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Multigrid:
    """The V(nu1, nu2) cycle of ups_mg_* around a set-up Plan (level 0).

    patches: [(origin, cells), ...] for levels 1 .. l, each (z, y, x): box k
    starts at node `origin` of level k-1 and spans `cells` cells of it
    (2 cells + 1 nodes per axis).  Level arrays are torch tensors of the
    plan's dtype, shapes `self.shapes`."""

    def __init__(self, plan, patches, setup=True):
        if plan.ncomp != 1:
            raise ValueError("the coarse plan must have one component")
        self.plan = plan
        self.patches = [(tuple(int(v) for v in c), tuple(int(v) for v in m)) for c, m in patches]
        hier = capi.ups_mg_hierarchy()
        hier.levels = len(self.patches)
        for k, (c, m) in enumerate(self.patches):
            for a in range(3):                   # (z, y, x) -> ABI (x, y, z)
                hier.origin[k][a] = c[2 - a]
                hier.cells[k][a] = m[2 - a]
        L = capi.lib()
        handle = C.c_void_p()
        capi.check(L.ups_mg_create(plan._h, C.byref(hier), C.byref(handle)))
        self._h = handle
        self.shapes = []
        for k in range(len(self.patches) + 1):
            n = (C.c_int * 3)()
            capi.check(L.ups_mg_level_shape(self._h, k, n))
            self.shapes.append((n[2], n[1], n[0]))
        wb = C.c_size_t()
        capi.check(L.ups_mg_sizes(self._h, C.byref(wb)))
        self.work_bytes = wb.value
        self.work = None
        if setup:
            self.setup()

    @property
    def levels(self):
        return len(self.patches)

    def setup(self, device=None):
        dev = self.plan.work.device if device is None else torch.device(device)
        self.work = torch.empty(max(self.work_bytes, 256), dtype=torch.uint8, device=dev)
        capi.check(capi.lib().ups_mg_setup(self._h, C.c_void_p(self.work.data_ptr()), self.work_bytes))
        return self

    def zeros(self):
        return [torch.zeros(s, dtype=self.plan.dtype, device=self.work.device) for s in self.shapes]

    def _ptrs(self, arrs, name):
        if len(arrs) != len(self.shapes):
            raise ValueError("expected %d level arrays for %s" % (len(self.shapes), name))
        for t, s in zip(arrs, self.shapes):
            if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != self.plan.dtype
                    or tuple(t.shape) != s or not t.is_contiguous()):
                raise ValueError("%s: contiguous %s tensors of shapes %s" % (name, self.plan.dtype, self.shapes))
        return (C.c_void_p * len(arrs))(*[t.data_ptr() for t in arrs])

    def cycle(self, fs, us, nu1=2, nu2=2, stream=None):
        """One V(nu1, nu2) cycle; us updated in place."""
        capi.check(capi.lib().ups_mg_cycle(self._h, self._ptrs(fs, "f"), self._ptrs(us, "u"), int(nu1), int(nu2),
                                           _stream_handle(stream)))
        return us

    def residuals(self, fs, us, stream=None):
        """Composite residual norms of levels 0 .. l (waits; refreshes ghosts)."""
        out = (C.c_double * len(self.shapes))()
        capi.check(capi.lib().ups_mg_residual(self._h, self._ptrs(fs, "f"), self._ptrs(us, "u"), out,
                                              _stream_handle(stream)))
        return list(out)

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().ups_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
