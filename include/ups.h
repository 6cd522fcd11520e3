/*
 * ups.h -- C ABI of libups, an MI355X (gfx950) solver for the free-space
 * ("unbounded") Poisson equation on a uniform 3-D grid.
 *
 * What it computes.  The problem is Lap u = f with u -> 0 at infinity
 * (Poncelet et al., eq. poisson_problem and the unbounded boundary
 * conditions of Sec. 1 and Sec. 2.2).  The Laplacian is the second-order
 * 7-point cross stencil of eq. cross_discr2, and the solution is the
 * convolution of f with that stencil's lattice Green's function G1
 * (L G1 = delta, Sec. 2.2; Sec. 3.3 requires the kernel to be the LGF of the
 * operator):
 *
 *     u[i] = h^2 sum_{j in box} G1[i - j] f[j]        for every grid point i,
 *
 * i.e. the exact decaying solution of the discrete problem for a source that
 * vanishes outside the box.  It is evaluated in spectral space, u_hat =
 * G_hat f_hat (Sec. 2.2), on a grid zero-padded to M_i >= 2 N_i points per
 * axis (default 2 N_i), with the real, even spectrum G_hat of the evenly
 * periodised G1 computed once by ups_plan_setup.
 *
 * A direction may instead be periodic, even or odd (ups_bc): the kernel is
 * then the Green's function that is periodic along it, the spectral
 * expression of the LGF there (Sec. 2.2), applied to the source as it is
 * (periodic) or to its even or odd mirror image about the box faces (the
 * cosine and sine transforms of Sec. 2.2 as a length-2n DFT).  With two unbounded directions the kernel is
 * eq. 2unbkernel's: the two-dimensional LGF's spectrum on the zero
 * wavenumber of the periodic direction, the inverse symbol elsewhere; with
 * one, the LGF of the one-dimensional operator screened by the periodic
 * directions' symbol (closed-form); with none, the inverse symbol, zero at
 * wavenumber 0 (the mean-free solution of the mean-free source).
 *
 * Conventions for every call:
 *   - Every call returns a ups_status; on failure ups_last_error() holds a
 *     message (thread-local, valid until the next call on that thread).
 *   - Arguments are validated before anything is enqueued: a failing call
 *     leaves no partial work on the stream.
 *   - Device pointers are HIP device addresses on the current device; the
 *     caller owns all device memory and keeps it alive until the enqueued
 *     work completes.  The library never allocates device memory; the one
 *     device array it owns (UPS_NOALLOC_MAX_WORK bytes per device, used only
 *     by ups_solve_noalloc) is reserved when its code object loads.
 *   - Execution is stream ordered (stream = hipStream_t, NULL = the legacy
 *     default stream); no call synchronises the host except ups_plan_setup,
 *     ups_batch_setup, ups_autotune and the opt-in checks (ups_solve with
 *     ups_plan_set_check_finite on, or in guard mode).
 *   - One solve in flight per plan (and per batch): a plan owns one work
 *     buffer, one side stream and one set of fork/join events, so two solves
 *     on the same plan must not overlap.  Enqueue them on one stream, or
 *     order them with events; use one plan per concurrently running stream.
 *   - Real arrays are C-contiguous [component][z][y][x] (x fastest), in the
 *     plan's precision (double for UPS_F64, float for UPS_F32), aligned to
 *     2 * sizeof(element) bytes.
 *   - Observability.  Host calls that enqueue work open roctx ranges
 *     (rocprofv3 --marker-trace): ups_plan_setup, ups_solve and
 *     ups_solve_noalloc, with one range per pass inside ("ups:xfwd",
 *     "ups:yfwd", "ups:zconv", "ups:yinv", "ups:xinv"), ups_batch_solve,
 *     ups_mg_cycle and ups_autotune.  A range covers the host call that
 *     enqueues the work; the kernels follow on the stream.  The environment
 *     variable UPS_LOG_LEVEL (read once per process) sends lines "[ups] ..."
 *     to stderr: 0 or unset, nothing; 1, every failing call with its status
 *     and message; 2, also the decisions of plan, batch and cycle creation
 *     and of the autotuner (kernels, schedule, buffer sizes); 3, also every
 *     solve, batch launch and cycle.
 */
#ifndef UPS_H
#define UPS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UPS_ABI_VERSION 2

typedef enum {
  UPS_OK = 0,
  UPS_ERR_INVALID_ARG = 1, /* null pointer, bad size, misaligned pointer */
  UPS_ERR_UNSUPPORTED = 2, /* valid problem the library does not handle */
  UPS_ERR_WORKSPACE = 3,   /* caller buffer smaller than ups_*_sizes asked */
  UPS_ERR_DEVICE = 4,      /* no usable gfx950 device, or a HIP call failed */
  UPS_ERR_NONFINITE = 5,   /* NaN or infinite input (ups_plan_set_check_finite) */
  UPS_ERR_INTERNAL = 6,    /* library bug */
  UPS_ERR_STATE = 7        /* call out of order (e.g. solve before setup) */
} ups_status;

/* Boundary condition per axis side (Sec. 2.2: unbounded, periodic, even =
 * homogeneous Neumann, odd = homogeneous Dirichlet).  Both sides of an axis
 * carry the same condition; every combination over the three axes is
 * solved.  Even and odd directions are cell-centred (UPS_CELL): the ghost
 * cell beyond a face is the mirror image (u[-1] = u[0], u[n] = u[n-1]) or
 * its negative.  Periodic, even and odd directions take pad = 2 n; an even
 * or odd direction needs a mirrored-fill kernel for that length (powers of
 * two 32 .. 1024), and along x an even n. */
typedef enum { UPS_BC_UNB = 0, UPS_BC_PER = 1, UPS_BC_EVEN = 2, UPS_BC_ODD = 3 } ups_bc;

/* Green's kernel: the LGF of the operator the caller discretises with
 * (Sec. 3.3).  UPS_GREEN_LGF2 = LGF of the 7-point stencil (eq. cross_discr2).
 * UPS_GREEN_LGF4_MEHR / _LGF6_MEHR: the compact Mehrstellen pairs of eqs.
 * mehrstellen_discr4 / _discr6 (Sec. 3.2), (1/h^2) L u = R f with the
 * 19- or 27-point L and the right-hand-side stencil R (the printed
 * "delta_y delta_z^2" of R6 read as the symmetric d2_y d2_z): the solve
 * applies K = R G_L, G_L the LGF of L, to f -- the same as G_L applied to
 * R f for a source that vanishes outside the box -- so the correction of
 * the right-hand side costs nothing at solve time.  All six sides
 * unbounded, padded lengths up to 1024. */
typedef enum { UPS_GREEN_LGF2 = 0, UPS_GREEN_LGF4_MEHR = 1, UPS_GREEN_LGF6_MEHR = 2 } ups_green;

/* Arithmetic of the FFT stages.  UPS_F32 uses float data, float twiddles and a
 * float G_hat, all rounded from values built in double. */
typedef enum { UPS_F64 = 0, UPS_F32 = 1 } ups_prec;

/* Sample positions (cell centres or nodes).  Informational: the lattice
 * convolution does not depend on it. */
typedef enum { UPS_CELL = 0, UPS_NODE = 1 } ups_center;

typedef struct {
  int n[3];        /* grid points per axis, (x, y, z); each >= 2          */
  double h[3];     /* grid spacing per axis; must be equal (isotropic)    */
  int bc[3][2];    /* ups_bc per axis (x, y, z) and side (low, high); the
                      two sides of an axis must be equal                  */
  int green;       /* ups_green                                           */
  int prec;        /* ups_prec                                            */
  int center;      /* ups_center                                          */
  int ncomp;       /* components solved together (1..8), e.g. 3 for a
                      vector right-hand side; they share G_hat            */
  int pad[3];      /* padded FFT length per axis; 0 = 2 n. Must be even,
                      >= 2 n and a supported length (ups_supported_length);
                      exactly 2 n along a periodic, even or odd axis      */
} ups_problem;

typedef struct ups_plan_s* ups_plan_t;
typedef struct ups_batch_s* ups_batch_t;

/* Version of this ABI (UPS_ABI_VERSION). */
int ups_abi_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char* ups_last_error(void);

/* 1 if `len` is a padded length the compiled kernels handle for precision
 * `prec`, else 0. */
int ups_supported_length(int len, int prec);

/* Fill *p with defaults: UNB on every side, LGF2, F64, cell-centred,
 * ncomp = 1, default padding, n = 0, h = 0. */
void ups_problem_init(ups_problem* p);

/* Validate the problem and build a host-side plan (no device work).
 * Errors: INVALID_ARG (null, n < 2, h <= 0, ncomp out of range, pad below
 * 2 n or odd, pad other than 2 n along a periodic, even or odd axis),
 * UNSUPPORTED (the two sides of an axis differ, an even or odd direction
 * node-centred, of odd extent along x or without a mirrored-fill kernel,
 * a Mehrstellen kernel with a non-unbounded direction or a padded length
 * above 1024, anisotropic h, n > 4096, padded length without a compiled
 * kernel, per-lane offsets that would not fit 32 bits). */
ups_status ups_plan_create(const ups_problem* prob, ups_plan_t* out);

/* Bytes the caller must provide: green = G_hat octant plus twiddle tables,
 * persistent between solves; work = solve scratch (also used as scratch by
 * ups_plan_setup).  Either pointer may be NULL. */
ups_status ups_plan_sizes(ups_plan_t plan, size_t* green_bytes, size_t* work_bytes);

/* Bind the caller's buffers to the plan and build G_hat (Sec. 2.2) into
 * `green`: G1 on the octant [0, M_i/2] by a separable Bessel quadrature in
 * double, its DCT-I along the three axes, times h^2 / (Mx My Mz), rounded to
 * the plan's precision.  With periodic directions: the two-dimensional LGF
 * by the same quadrature or the screened one-dimensional LGF in closed form
 * (DCT-I along the unbounded axes), the inverse symbol elsewhere, and along
 * each periodic axis (padded to M = 2 n) twice the n-point spectrum at even
 * frequencies and zero at odd ones -- the spectrum of the n-periodic kernel
 * truncated to |d| < n, which the zero-padded convolution applies exactly;
 * along an even or odd axis the 2n-periodic spectrum itself (the forward
 * pass fills the second half of the line with the mirror image).  With a
 * Mehrstellen kernel: G_L = G1 + D on the octant extended by the radius
 * of R, D the integral of the bounded (sigma_2 - sigma_L) / (sigma_L
 * sigma_2) over the Brillouin zone by a tensor Gauss-Legendre rule graded
 * towards k = 0 (three GEMM contractions), then R G_L, its DCT-I, and the
 * same scaling (about 0.4 s at 512^3).
 * Enqueued on `stream`, then the host waits for it.
 * The buffers must stay alive and unchanged (green) for every later solve.
 * Errors: INVALID_ARG (null or misaligned pointers), WORKSPACE (sizes smaller
 * than ups_plan_sizes), DEVICE (no gfx950 device or a HIP error). */
ups_status ups_plan_setup(ups_plan_t plan, void* green, size_t green_bytes, void* work,
                          size_t work_bytes, void* stream);

/* u = h^2 G1 * f for each component (Sec. 2.2, u_hat = G_hat f_hat): five
 * kernels on `stream` -- zero-padded real FFT along x, FFT along y, FFT along
 * z fused with the multiply by G_hat and the inverse along z, inverse along
 * y, inverse real FFT along x fused with the crop.  f and u are real arrays
 * [ncomp][nz][ny][nx]; u may equal f (in place).  f is not modified unless
 * u == f.  Errors: STATE (setup not done), INVALID_ARG (null/misaligned),
 * NONFINITE (check on and f holds a NaN or infinity: nothing is solved),
 * INTERNAL (guard mode found a canary band overwritten or NaN poison in the
 * output), DEVICE (a HIP call failed).
 *
 * Guard mode: with the environment variable UPS_DEBUG_GUARDS set (and not
 * "0") when the plan is created, the work buffer holds a 64 KiB canary band
 * on each side of W (ups_plan_sizes includes them; ups_plan_work_offset
 * gives W's offset).  ups_solve then fills W with NaN words, runs the five
 * passes one at a time on the caller's stream (no side stream, no slabs),
 * poisons the rows y >= ny of W again before the last pass, checks both
 * bands after every pass and, for a finite input, checks the output for
 * NaN.  It waits for the stream after every pass: a debugging aid for
 * out-of-bounds stores and reads of unwritten data, not a fast path. */
ups_status ups_solve(ups_plan_t plan, const void* f, void* u, void* stream);

/* Maximum bytes of W (2 x element size x ncomp x nz x my x the row pitch of
 * ups_plan_layout, rounded up to 256) that ups_solve_noalloc handles. */
#define UPS_NOALLOC_MAX_WORK (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): ups_solve with W
 * in a library-owned device array of UPS_NOALLOC_MAX_WORK bytes instead of
 * the plan's work buffer.  The plan must have been set up (its green buffer
 * holds G_hat and the twiddle tables; its work buffer is not touched by this
 * call), on the device that is current.  The call allocates nothing: the
 * array is one per device, reserved when the library's code object loads
 * on that device and held until the process ends, and its address is looked
 * up once per device.  Every call on a device shares that device's array,
 * which keeps the last call's contents (no pass reads W before another pass
 * of the same solve has written it, so nothing is cleared): solves through
 * this call that overlap on one device, on any streams or plans, race, and
 * must be ordered by the caller.  Same layout, results and errors as
 * ups_solve, plus UNSUPPORTED (W larger than UPS_NOALLOC_MAX_WORK, or a
 * guard-mode plan) and INVALID_ARG (another device current than the
 * plan's). */
ups_status ups_solve_noalloc(ups_plan_t plan, const void* f, void* u, void* stream);

/* Opt-in input check (off by default): with `enable` != 0 every ups_solve
 * on this plan first scans f for NaN and infinite values on the GPU, waits
 * for the stream and returns UPS_ERR_NONFINITE without solving if it finds
 * one.  The check reads f once more and synchronises the host. */
ups_status ups_plan_set_check_finite(ups_plan_t plan, int enable);

/* 1 if the plan was created in guard mode (see ups_solve), 0 if not, -1 for
 * NULL. */
int ups_plan_guard_mode(ups_plan_t plan);

/* Byte offset of W inside the work buffer: 0, or the canary band's size in
 * guard mode. */
size_t ups_plan_work_offset(ups_plan_t plan);

/* Adjoint of ups_solve: grad_f[j] = h^2 sum_i G1[i - j] grad_u[i].  G1 is
 * even in every index (the 7-point stencil is symmetric), so this is the
 * same convolution applied to grad_u; same layout and errors as ups_solve. */
ups_status ups_solve_adjoint(ups_plan_t plan, const void* grad_u, void* grad_f, void* stream);

/* Name of the kernel variant the plan uses for pass 0..4 (x-forward,
 * y-forward, z-convolution, y-inverse, x-inverse), or NULL. */
const char* ups_plan_kernel(ups_plan_t plan, int pass);

/* Names of the compiled kernel variants of pass 0..4 for padded length
 * `len` in precision `prec` (ups_prec): writes up to `cap` of them to
 * `names` (static strings owned by the library; `names` may be NULL when cap
 * is 0) and returns how many exist (0 for bad arguments).  The first one is
 * the default a new plan uses when no tuning result is cached.  Listed are
 * the variants for unbounded and periodic directions; a forward pass along
 * an even or odd direction runs a mirrored-fill variant of its length
 * (names ending in "_e", listed by ups_kernel_fill_variants), the only
 * choices ups_plan_set_kernel accepts there. */
int ups_kernel_variants(int pass, int prec, int len, const char** names, int cap);

/* The mirrored-fill variants of forward pass 0..2 (x, y, z) for an even or
 * odd direction of padded length `len` (Sec. 2.2: the second half of each
 * line is the mirror image of the first, with the sign of the symmetry,
 * instead of the zero padding), as ups_kernel_variants lists the others;
 * the first one is the default.  0 for the inverse passes. */
int ups_kernel_fill_variants(int pass, int prec, int len, const char** names, int cap);

/* Select the compiled variant `name` for pass 0..4 (names as returned by
 * ups_plan_kernel; used by tuning).  INVALID_ARG if no such variant exists
 * for the pass, precision and padded length. */
ups_status ups_plan_set_kernel(ups_plan_t plan, int pass, const char* name);

/* Schedule of the three column passes (y-forward, z-convolution,
 * y-inverse), which treat every x frequency kx independently.  With
 * `columns` = w > 0 they run slab by slab over kx in [0, w), [w, 2w), ...
 * (the last slab also takes the remainder); 0 runs each pass once over all
 * columns.  With the side stream on (ups_plan_set_side_stream) and more than
 * one slab, the z pass of each slab runs on a plan-owned stream beside the
 * y passes of the other slabs on the caller's stream (forked and joined
 * with events; everything is complete in the caller's stream order when the
 * solve's last pass is).  The result does not depend on the schedule
 * beyond rounding: a slab's last columns may run through another compiled
 * variant of the same pass than with one slab, which can differ in the
 * last bit.  INVALID_ARG unless w is 0 or a positive multiple of 16.
 * ups_plan_create picks a default from the problem size (FP64 with at least
 * 384 columns: 128-column slabs with the side stream on; other plans: one
 * slab, side stream on);
 * ups_plan_slab returns the current width (0 = one slab), or -1 for NULL.
 * UNSUPPORTED for a w below the column count on a plan whose column 0
 * carries the Nyquist column (ups_plan_nyquist_packed). */
ups_status ups_plan_set_slab(ups_plan_t plan, int columns);
int ups_plan_slab(ups_plan_t plan);

/* 1 if W's column 0 carries X[0] + i X[mx/2] (0 if not, -1 for NULL).
 * For a real source the x transform's columns kx = 0 and kx = mx/2 are real,
 * so one complex column holds both and the column passes run over mx/2
 * columns, a multiple of the 128-byte line width, with no second narrow
 * launch.  Column 0's z transforms run in a pair launch that separates the
 * two through the Hermitian symmetry of each in (ky, kz), applies the G_hat
 * lines of kx = 0 and mx/2 and inverts: two waves per pair of lines (ky,
 * my - ky), beside the z pass's main launch on the plan's side stream.
 * ups_plan_create packs FP32 plans with mx = 1024 and mz = 512 or 1024
 * whose x and z directions are neither even nor odd (one slab); their x and
 * z passes run the wave-per-line kernels only (ups_plan_set_kernel refuses
 * the others with UNSUPPORTED).  Batches do not pack. */
int ups_plan_nyquist_packed(ups_plan_t plan);

/* Each column pass runs over the largest multiple of 8 x (columns per
 * 128-byte line) x-frequencies in one launch and over the remaining columns
 * in a second launch (a one-column kernel for one column, the pass's own
 * kernel for more); call these the narrow launches.  With one slab and
 * `enable` != 0 the narrow launches of all three column passes run on a
 * plan-owned stream, forked from the caller's stream after the x pass (FP64)
 * or after the main y-forward launch (FP32) and joined back before the
 * inverse x pass with events (ups_run_pass forks and joins around the one
 * pass); with several slabs `enable` != 0 pipelines them (see
 * ups_plan_set_slab).  0 keeps every launch on the caller's stream.
 * Results are identical either way (the same kernels run). */
ups_status ups_plan_set_side_stream(ups_plan_t plan, int enable);
/* 1 if the side stream is on for this plan, 0 if off, -1 for NULL. */
int ups_plan_side_stream(ups_plan_t plan);

/* Enqueue one pass of the solve on the bound work buffer W, for testing and
 * per-kernel timing: pass 0 reads the real array `in` and writes W; passes
 * 1-3 update W in place (in/out ignored); pass 4 reads W and writes the real
 * array `out`.  W holds complex values [c][z][y][kx] with kx fastest, row
 * pitch `pitch`, plane stride `plane` and component stride `comp_stride`
 * (complex elements); G_hat (real, plan precision) sits at byte
 * `ghat_offset` of the green buffer as [iy][kx][iz] (iz fastest), iy stride
 * `ghat_plane` and kx stride `ghat_plane` / (mx/2 + 1). */
ups_status ups_run_pass(ups_plan_t plan, int pass, const void* in, void* out, void* stream);
ups_status ups_plan_layout(ups_plan_t plan, int* pitch, long long* plane, long long* comp_stride,
                           size_t* ghat_offset, long long* ghat_plane);

/* Algorithmic HBM bytes of pass 0..4 (each element read or written once),
 * and of the whole solve for pass = -1.  Returns 0 on a bad argument. */
double ups_plan_model_bytes(ups_plan_t plan, int pass);

/* Time every compiled kernel variant of each pass, pass by pass, inside
 * whole solves from the caller's f into the caller's u (arrays laid out as
 * for ups_solve, on this plan's bound work buffer) with the current choices
 * for the other passes and the plan's schedule (HIP events on `stream`; u
 * and the work buffer are overwritten; best of two runs of 5 solves).
 * A variant replaces the current choice only if it is faster by more than
 * 1%.  Plans with at least 256 x-frequencies then also try one slab and
 * 128- or 256-column slabs pipelined over two streams (ups_plan_set_slab)
 * and keep the fastest schedule, by the same rule (the schedule is kept in
 * the plan only).  Candidates other than the current choice are skipped
 * once `budget_ms` of GPU time is spent.  The choices go to a process-wide
 * cache used by later plans and batches of the same (pass, precision,
 * padded length, size class), the size class being floor(log2) of the
 * number of lines the pass transforms (rows for the x passes, kx columns
 * times z planes for the y passes, kx times ky columns for the z pass,
 * times ncomp); keys read "zconv/f32/1024/l19" (with "/e" appended for a
 * forward pass along an even or odd direction).  With the environment
 * variable UPS_TUNE_CACHE set to a file path the cache is loaded from and
 * saved to that JSON file.  Waits for the stream.  Errors: INVALID_ARG (null
 * or misaligned f or u), STATE (setup not done), DEVICE. */
ups_status ups_autotune(ups_plan_t plan, const void* f, void* u, void* stream, double budget_ms);

/* Release the host-side plan.  Device buffers stay with the caller. */
ups_status ups_plan_destroy(ups_plan_t plan);

/* ---- batches ------------------------------------------------------------
 * A batch runs `count` independent problems (any shapes, precisions and
 * component counts; at most 200) as ONE hipGraph launch: for each of the
 * five passes the problems sharing a compiled kernel run in grouped
 * launches (a group above a quarter of the pass's algorithmic bytes is
 * split), the launches of a pass are dealt longest first to four parallel
 * chains of the graph, and the passes follow each other.  Results equal
 * those of ups_solve on each problem with the same kernel variants. */

/* Validate every problem and lay out the batch (host only).  Errors as
 * ups_plan_create for the first failing problem; UNSUPPORTED above 200. */
ups_status ups_batch_create(const ups_problem* probs, int count, ups_batch_t* out);

/* Bytes of the caller's buffers: green (every G_hat and twiddle table plus
 * the launch tables; persistent) and work (every problem's scratch). */
ups_status ups_batch_sizes(ups_batch_t batch, size_t* green_bytes, size_t* work_bytes);

/* Build every G_hat and the launch tables, capture the graph; waits for
 * `stream`.  Errors: INVALID_ARG, WORKSPACE, DEVICE, STATE (called twice). */
ups_status ups_batch_setup(ups_batch_t batch, void* green, size_t green_bytes, void* work,
                           size_t work_bytes, void* stream);

/* Solve every problem: f[i], u[i] are device arrays laid out as for
 * ups_solve on problem i (u[i] may equal f[i]).  The pointer arrays are host
 * arrays read during the call; one small kernel stores them on the device,
 * then the graph is launched on `stream`. */
ups_status ups_batch_solve(ups_batch_t batch, const void* const* f, void* const* u, void* stream);

/* Number of grouped launches (over all chains) the batch uses for pass 0..4. */
int ups_batch_launches(ups_batch_t batch, int pass);

ups_status ups_batch_destroy(ups_batch_t batch);

/* ---- multigrid cycle around the solve ---------------------------------------
 * The V(nu1, nu2) full-approximation cycle of Sec. 3.1 (Alg. amg_vcycle) on
 * a hierarchy of nested refined boxes, with an unbounded (or mixed) solve
 * of the plan as the direct solver on the coarsest level.  All levels hold
 * nodes, arrays laid out as the plan's ([z][y][x], x fastest, the plan's
 * precision):
 *   - level 0 is the plan's grid (nx, ny, nz points, spacing h);
 *   - level k >= 1 refines level k-1 by 2: a box of 2 cells[k-1][a] + 1
 *     nodes along axis a at spacing h / 2^k, whose node 2 i lies on node
 *     origin[k-1][a] + i of level k-1.  Its outer layer of nodes is ghost
 *     data, reconstructed from level k-1 by 4-point cubic interpolation
 *     ((-1, 9, 9, -1)/16 at each odd fine index, one axis at a time); the
 *     nodes inside are its unknowns.  Each box lies strictly inside its parent's unknowns:
 *     cells >= 2, origin >= 1 and origin + cells <= n_parent - 2.
 * One cycle, for k = l .. 1: ghosts of u_k from u_{k-1}, nu1 red-black
 * Gauss-Seidel iterations (red = even index sum in the box frame, first),
 * r_k = f_k - Lap u_k with the 7-point stencil of eq. cross_discr2; on the
 * parent's unknowns inside the box's footprint u_{k-1} = injection of u_k,
 * f_{k-1} = full weighting ((1/4)[1 2 1] per axis) of r_k + Lap u_{k-1};
 * u_{k-1} on the whole footprint is stored.  Level 0 is solved by the plan.
 * For k = 1 .. l: u_k += trilinear prolongation of (new minus stored
 * u_{k-1}) on the unknowns, ghosts reconstructed from u_{k-1}, nu2
 * Gauss-Seidel iterations.  The coarse kernel must be the LGF of the 7-point
 * operator (Sec. 3.3): plans with the Mehrstellen kernels are refused.  The
 * caller's sources are read only; the modified sources of levels 0 .. l-1
 * live in the work buffer. */
#define UPS_MG_MAX_LEVELS 8

typedef struct ups_mg_s* ups_mg_t;

typedef struct {
  int levels;                        /* refined levels l, 0 .. UPS_MG_MAX_LEVELS */
  int origin[UPS_MG_MAX_LEVELS][3];  /* box k+1: its node 0 in level-k nodes (x, y, z) */
  int cells[UPS_MG_MAX_LEVELS][3];   /* box k+1: its extent in level-k cells (x, y, z) */
} ups_mg_hierarchy;

/* Validate the hierarchy against the plan (host only; the plan need not be
 * set up yet, but must outlive the cycle object).  Errors: INVALID_ARG (null
 * argument, a box outside its parent's unknowns, fewer than 2 cells, more
 * than 2^31 - 1 nodes on a level), UNSUPPORTED (a plan with several
 * components or a Mehrstellen kernel, levels above UPS_MG_MAX_LEVELS). */
ups_status ups_mg_create(ups_plan_t coarse, const ups_mg_hierarchy* hier, ups_mg_t* out);

/* Node counts (x, y, z) of level 0 .. l. */
ups_status ups_mg_level_shape(ups_mg_t mg, int level, int n[3]);

/* Bytes of the work buffer: the modified sources of levels 0 .. l-1, the
 * smoother's second array of each refined level, one array of the largest
 * refined level (the residual), the stored footprints and the residual
 * norms. */
ups_status ups_mg_sizes(ups_mg_t mg, size_t* work_bytes);

/* Bind the caller's work buffer (256-byte aligned, at least ups_mg_sizes
 * bytes; the caller owns it).  Errors: INVALID_ARG, WORKSPACE. */
ups_status ups_mg_setup(ups_mg_t mg, void* work, size_t work_bytes);

/* One V(nu1, nu2) cycle on `stream`: f[k] (read only) and u[k] (updated in
 * place, ghost layers included) are device arrays of level k, k = 0 .. l.
 * Uses the plan's work buffer and side stream (one cycle or solve in flight
 * per plan).  Errors: INVALID_ARG (null or misaligned arrays, nu1 or nu2
 * outside 0 .. 64), STATE (no work buffer bound, plan not set up), DEVICE. */
ups_status ups_mg_cycle(ups_mg_t mg, const void* const* f, void* const* u, int nu1, int nu2, void* stream);

/* Composite residual norms: norms[k] = max |f_k - Lap u_k| over the
 * unknowns of level k outside the interior of box k+1's footprint (level 0:
 * its nodes with all six neighbours in the grid), after the ghosts of
 * levels 1 .. l are refreshed from their parents (u is written there).
 * Waits for `stream`.  Errors as ups_mg_cycle. */
ups_status ups_mg_residual(ups_mg_t mg, const void* const* f, void* const* u, double* norms, void* stream);

ups_status ups_mg_destroy(ups_mg_t mg);

#ifdef __cplusplus
}
#endif

#endif /* UPS_H */
