/*
 * fsp.h -- free-space Poisson solver for AMD Instinct MI355X (gfx950), C ABI.
 *
 * The library solves  -Laplace(phi) = rho  on a regular 3D grid with
 * free-space (open) boundaries by the FFT convolution of the paper
 * "A Massively Parallel Performance Portable Free-space Spectral Poisson
 * Solver" (arXiv 2405.02603):
 *
 *   Section 2.2 (Hockney-Eastwood): double the grid, zero-pad rho, transform,
 *   multiply by the transform of the mirror-extended Green's function,
 *   transform back, restrict to the physical box;
 *   Section 2.3, eq. (3) (Vico-Greengard): the same solve with the transform of
 *   the truncated kernel 2 (sin(L|k|/2)/|k|)^2 precomputed on the 4N grid;
 *   Section 2.4 (modified Vico-Greengard): that precompute done as a DCT-I on
 *   the (2N+1)^3 unique samples.
 *
 * Discrete result.  With cell-centred points x_i = lo + (i + 1/2) h,
 * h_d = (hi_d - lo_d) / n_d and V = h0 h1 h2, every solve computes
 *
 *     phi_i = V * sum_j K[|i0-j0|, |i1-j1|, |i2-j2|] * rho_j
 *
 * (the sum of eq. (2) over the grid) where K is the kernel of the chosen
 * Green's function.  Units: epsilon_0 = 1, G = +1/(4 pi r).
 *
 * Arrays.  rho and phi are C-contiguous [n0][n1][n2] arrays of float
 * (FSP_F32) or double (FSP_F64) in device memory, axis 2 fastest.
 *
 * Threads and streams.  A plan holds one workspace: at most one solve per
 * plan may be in flight at a time.  Calls on different plans may run
 * concurrently on different streams.  "stream" arguments are hipStream_t
 * values passed as void*; NULL means the null stream.
 *
 * Errors.  Every call returns an fsp_status; nothing aborts and no C++
 * exception crosses this boundary.  Argument errors are detected before
 * anything is enqueued.  Errors of earlier asynchronous device work surface as
 * FSP_ERR_DEVICE at a later call.  fsp_last_error() gives a per-thread text.
 */
#ifndef FSP_H_
#define FSP_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsp_plan_s* fsp_plan;
typedef struct fsp_batch_s* fsp_batch;

typedef enum {
  FSP_OK = 0,
  FSP_ERR_INVALID_ARG = 1,      /* NULL pointer, bad enum, lo >= hi, ...                 */
  FSP_ERR_UNSUPPORTED_SIZE = 2, /* an n_d outside {2^a, 3*2^a : 8 <= n_d <= 512}         */
  FSP_ERR_BOX_ASPECT = 3,       /* Vico-Greengard window too long for the 4N grid        */
  FSP_ERR_OUT_OF_MEMORY = 4,    /* a device allocation failed                            */
  FSP_ERR_NOT_READY = 5,        /* solve before bind/precompute                           */
  FSP_ERR_DEVICE = 6            /* a HIP runtime call or kernel launch failed             */
} fsp_status;

/* Green's function.  The names follow the paper's three solver types. */
typedef enum {
  FSP_HOCKNEY = 0,   /* Section 2.2: K = 1/(4 pi |m h|), K[0] = g0                       */
  FSP_VICO = 1,      /* Section 2.3: kernel by a (4N)^3 inverse FFT, restricted          */
  FSP_VICO_DCT = 2   /* Section 2.4: the same kernel by a DCT-I on (2N+1)^3 samples       */
} fsp_greens;

typedef enum { FSP_F32 = 0, FSP_F64 = 1 } fsp_prec;

/* Plan flags. */
#define FSP_FLAG_NONE 0u
/* Also precompute the derivative tables of the Green's function (three more
 * octants in the Green's buffer) and size the workspace for fsp_solve_grad
 * (four spectra instead of one). */
#define FSP_WANT_GRAD 1u
/* Periodic axes (Section 2.2, step 1: the grid is doubled only along the axes
 * with open boundaries).  Along a periodic axis a of n_a points the solve is a
 * cyclic convolution of period n_a whose Green's function takes, at offset d,
 * its value at the nearest image (min(d, n_a - d)): the Green's function
 * circularly shifted over the axis's own period, as step 3 shifts it over the
 * doubled period of an open axis.  The transform tables fold each periodic
 * axis that way; the passes are those of the open solve (the doubled cyclic
 * convolution with the folded table equals the n_a-periodic one).  Any Green's
 * function; not with FSP_WANT_GRAD (FSP_ERR_INVALID_ARG). */
#define FSP_PERIODIC_0 2u
#define FSP_PERIODIC_1 4u
#define FSP_PERIODIC_2 8u

typedef struct {
  int n[3];          /* grid points per axis; axis 2 is contiguous                     */
  double lo[3];      /* box lower corner                                                */
  double hi[3];      /* box upper corner (hi_d > lo_d)                                  */
  int greens;        /* fsp_greens                                                      */
  int prec;          /* fsp_prec: precision of rho, phi and the solve passes            */
  double alpha;      /* Vico-Greengard window factor, L = alpha |hi - lo|; 0 -> 1.1     */
  double g0;         /* Hockney-Eastwood K[0]; NaN -> 1/(4 pi)                           */
  unsigned flags;    /* FSP_WANT_GRAD, FSP_PERIODIC_*; other bits: FSP_ERR_INVALID_ARG  */
} fsp_plan_desc;

/* Validate a descriptor and build a plan.  Host only: no device memory is
 * touched.  Vico-Greengard plans are rejected with FSP_ERR_BOX_ASPECT when
 * alpha * |hi - lo| > 3 * min_d (hi_d - lo_d): the periodic images of the
 * truncated kernel on the 4N grid would then reach into the box (the paper
 * states the 4N grid size, Section 2.3, but not this limit).
 * On success *out owns a new plan; destroy it with fsp_plan_destroy. */
fsp_status fsp_plan_create(const fsp_plan_desc* desc, fsp_plan* out);

/* Device bytes the plan needs: *ghat_bytes for the precomputed transform of
 * the Green's function (plus the plan's twiddle tables), *work_bytes for the
 * solve workspace.  Either pointer may be NULL.  Section 3.3 accounts a
 * solver's memory as the sum of its fields (values times bytes per value);
 * these are this library's fields in that sense: the real octant of the
 * transform of G2 instead of the full doubled-grid field, and one complex
 * half spectrum (n0 x 2 n1 x (n2 + 1), padded rows) instead of the doubled
 * rho2 / phi2 fields, whose zero half is never stored (Section 2.2, steps 2
 * and 5). */
fsp_status fsp_plan_bytes(fsp_plan p, size_t* ghat_bytes, size_t* work_bytes);

/* Device bytes fsp_precompute needs transiently (freed before it returns to
 * the caller's stream order); reported for admission control.  This is the
 * pre-computation grid of Sections 2.3 and 2.4 in float64: (4N)^3 samples for
 * FSP_VICO, (2N+1)^3 for FSP_VICO_DCT (the memory reduction of Section 2.4),
 * (N+1)^3 for FSP_HOCKNEY, plus one intermediate of the per-axis transforms. */
fsp_status fsp_plan_precompute_bytes(fsp_plan p, size_t* bytes);

/* Attach device memory.  ghat_dev / work_dev are caller-owned device buffers
 * of at least the sizes from fsp_plan_bytes, aligned to 256 bytes; NULL makes
 * the plan allocate (and later free) that buffer itself.  Binding again
 * replaces the previous buffers (a plan-owned buffer is freed) and clears the
 * precompute state.  The current HIP device is the plan's device.  The paper
 * allocates its fields at solver set-up, outside the timed "Solve"
 * (Section 3.2) and counts them in Section 3.3; binding is that set-up step,
 * with the caller free to own the memory. */
fsp_status fsp_plan_bind(fsp_plan p, void* ghat_dev, void* work_dev);

/* Use src's precomputed transform in dst (same Green's function, grid, box,
 * alpha, g0 and precision, else FSP_ERR_INVALID_ARG).  dst then reads src's
 * buffer: src's Green's buffer must stay alive and unchanged while dst is used.
 * Section 2.3: the restricted G2 is computed once and reused by every later
 * solve on the same grid; a plan of another box or spacing needs its own
 * (Section 1: a bunch-fitted grid changes, so G2 is recomputed). */
fsp_status fsp_plan_share_ghat(fsp_plan dst, fsp_plan src);

/* Compute the transform of the Green's function on the device, in float64,
 * and store it (rounded once to the solve precision) in the plan's Green's
 * buffer, with the plan's twiddle tables (and, with FSP_WANT_GRAD, the three
 * derivative tables).
 *   FSP_HOCKNEY: Section 2.2 step 3 -- the kernel 1/(4 pi |x|) with the
 *     regularised value g0 at the origin, mirror-extended to the doubled grid
 *     (G2), then transformed (step 4); the transform of the mirror-even G2 is
 *     a DCT-I of length n_d + 1 along each axis.
 *   FSP_VICO: Section 2.3 -- eq. (3) sampled on the (4N)^3 frequency grid,
 *     inverse transformed and restricted to the doubled grid, then as above.
 *   FSP_VICO_DCT: Section 2.4 -- eq. (3) sampled on its (2N+1)^3 unique
 *     values, inverse transformed by a DCT-I of length 2 n_d + 1 per axis
 *     keeping the doubled grid's octant, then as above.
 * Every per-axis transform is a dense float64 cosine (or sine) contraction
 * run by this library's own kernels.  The result is reused by every later
 * solve (Section 2.3); calling this again recomputes it (a refresh, needed
 * when the grid spacing changes: Sections 1 and 2.3).  Asynchronous on
 * `stream`; allocates and frees transient float64 buffers of
 * fsp_plan_precompute_bytes bytes in stream order.
 * FSP_ERR_OUT_OF_MEMORY if the transient buffers cannot be allocated. */
fsp_status fsp_precompute(fsp_plan p, void* stream);

/* phi = the free-space solution for rho (both device arrays, [n0][n1][n2] in
 * the plan's precision): Section 2.2 steps 1, 2, 4 and 5 (zero-pad, transform,
 * multiply by the transform of G2, inverse transform, restrict), the sum of
 * eq. (2) over the grid.  phi may equal rho (in place; Section 3.3 reuses the
 * rho field for phi).  Asynchronous on `stream`; enqueues five kernels and
 * allocates nothing.  FSP_ERR_NOT_READY before bind + precompute. */
fsp_status fsp_solve(fsp_plan p, const void* rho, void* phi, void* stream);

/* The five passes of fsp_solve (Section 2.2 steps 4-5 split by axis) run one
 * range at a time: passes first..last
 * (0 = axis-2 real transform of rho, 1 = axis-1 forward, 2 = axis-0 forward,
 * multiply and inverse, 3 = axis-1 inverse, 4 = axis-2 inverse real transform
 * to phi).  Running 0..4 in order is fsp_solve; splitting the range lets a
 * caller put its own events between passes to time each kernel.  rho is read
 * only by pass 0 and phi written only by pass 4 (the other pointer may be
 * NULL when its pass is outside the range). */
fsp_status fsp_solve_passes(fsp_plan p, const void* rho, void* phi, int first, int last, void* stream);

/* The gradient of the solution: grad[a] = d phi / d x_a (E = -grad), as
 * three device arrays [3][n0][n1][n2] in the plan's precision, and phi too
 * when phi is not NULL (phi may equal rho; grad must not overlap phi).
 * The paper names the field E = -grad(phi) for its particle application
 * (Appendix B) without a method; here each component is the same discrete
 * convolution as the potential with the derivative of the kernel, which is
 * odd along its axis: for Hockney-Eastwood -x_a / (4 pi |x|^3) (0 at the
 * origin), for Vico-Greengard the inverse transform of i k_a times eq. (3) on
 * the 4N grid.  Its transform on the doubled grid is -i times a real octant
 * (sine transform along a), stored by fsp_precompute.  The forward transforms
 * along axes 2 and 1 run once; the axis-0 pass writes every output's
 * spectrum (components to the workspace's other three spectra, phi in place)
 * and one launch of each inverse pass takes them all.  The axis-0 pass has
 * variants of its own: 0 and 1 are one launch for every output (the spectrum
 * read and transformed once), 2 one launch per output (fewer registers; for
 * long pencils).  Needs a plan created with FSP_WANT_GRAD
 * (else FSP_ERR_INVALID_ARG); FSP_ERR_NOT_READY before bind + precompute.
 * Uses the plan's schedule with separate passes 1-3, the axis-0 variant as
 * chosen by fsp_autotune, else the schedule's.  Asynchronous on
 * `stream`; allocates nothing. */
fsp_status fsp_solve_grad(fsp_plan p, const void* rho, void* phi, void* grad, void* stream);

/* Schedules (no passage of the paper: how this library maps each pass onto
 * the GPU).  Every pass has NUM_VARIANTS = 3 kernel variants (radix plan,
 * threads per pencil, tile); variants[i] selects the one for pass i (0..4,
 * as in fsp_solve_passes).  The value 3 in variants[1..3] (all three) selects
 * the fused schedule for small grids with n0 == n1 (n <= 64 in float32, <= 48
 * in float64): one kernel holds a column tile's whole (axis 0, axis 1) slab in
 * LDS and runs passes 1-3 there; fsp_solve_passes then accepts only ranges
 * that contain all of 1-3 or none of them (FSP_ERR_INVALID_ARG otherwise).
 * The value 4 in variants[0] and variants[1] (both) selects the plane kernel
 * for passes 0-1, and in variants[3] and variants[4] (both) the one for passes
 * 3-4, on grids with n1 == n2 whose i0-plane of the axis-2 spectrum fits in
 * LDS (n1 in {32, 48, 64, 96, 128} in float32, {32, 48, 64} in float64): one
 * block per plane runs the axis-2 and the axis-1 transforms with the plane
 * held in LDS, so the axis-2 spectrum never goes to device memory;
 * fsp_solve_passes then accepts only ranges that contain both passes of such
 * a pair or neither (FSP_ERR_INVALID_ARG otherwise).  The plane pairs and the
 * fused schedule exclude each other.
 * Results are identical up to rounding order across schedules.  A new plan starts with the schedule last tuned for its grid and
 * precision in this process (else all zeros). */
fsp_status fsp_plan_get_schedule(fsp_plan p, int* variants /* [5] */);
fsp_status fsp_plan_set_schedule(fsp_plan p, const int* variants /* [5] */);

/* Time every variant of every pass on this plan's buffers with HIP events
 * placed around that pass inside full solves (reps timed solves per variant,
 * 1 <= reps <= 8, after a warm one), keep the
 * fastest per pass in the plan and in the process-wide table used by new
 * plans of this grid and precision (no passage of the paper; the schedule
 * changes the time only, the result up to rounding order).  rho and phi are
 * device arrays as in fsp_solve, but phi must not overlap rho
 * (FSP_ERR_INVALID_ARG): the timed solves write phi many times.  On
 * return phi holds the solve of rho with the tuned schedule.  Synchronises
 * `stream`.  times_ms (NULL or [5 * 3 + 5]) receives the median time of each
 * variant, times_ms[pass * 3 + variant], then the median time of whole solves
 * with schedules built from the best variants: times_ms[15] passes 1-3 fused,
 * [16] all passes separate, [17] both plane pairs (0-1 and 3-4), [18] the
 * plane pair 0-1 alone, [19] the pair 3-4 alone (0 where the schedule is not
 * supported); the fastest of these schedules is kept.  On a plan with
 * FSP_WANT_GRAD it also times the gradient solve's axis-0 pass (four outputs)
 * in each of its variants and keeps the fastest for fsp_solve_grad
 * (fsp_plan_set_schedule drops that choice: the gradient then follows the
 * schedule).  If a solve fails its status is returned and the plan keeps a
 * valid (untuned) schedule. */
fsp_status fsp_autotune(fsp_plan p, const void* rho, void* phi, int reps, void* stream, float* times_ms);

/* count independent solves (each with its own plan, and so its own
 * workspace) enqueued on one stream; plans may differ in size, precision and
 * Green's function.  rho[i] / phi[i] as in fsp_solve.  Solves of plans with
 * equal shape and precision are issued as shared kernel launches.  No passage
 * of the paper defines this call: it is fsp_solve for many independent right-
 * hand sides at once, each the result Section 2.2 defines. */
fsp_status fsp_solve_batched(int count, const fsp_plan* plans, const void* const* rho,
                             void* const* phi, void* stream);

/* Schedules for a set of solves launched together (no passage of the paper:
 * how the passes map onto the GPU).  Plans are grouped by grid, precision
 * and layout, whatever their schedules.  Each group's solves are timed
 * together (reps timed launches of the whole group after a warm one,
 * 1 <= reps <= 8, median) with the separate passes fsp_autotune last found
 * fastest for that grid (else the first plan's) and, on a grid that supports
 * the plane kernels, with the plane kernel for passes 0-1, for passes 3-4,
 * and for both, the axis-0 variant as last tuned.  From the fastest, each pass
 * that is not a plane kernel then tries its other variants in turn, each
 * timed the same way, and keeps one only if the group runs faster.  The
 * result is set on every plan of the group.  Groups whose tuned schedule is
 * the fused slab keep their schedules.  A single solve may prefer another
 * schedule than many solves launched together: a plane kernel has one block
 * per plane, too few to fill the GPU for one small grid, and a kernel held
 * back by its registers gains from the wider launch.  rho[i] and phi[i] as in
 * fsp_solve_batched, phi[i] must not
 * overlap rho[i] (FSP_ERR_INVALID_ARG): the timed solves write phi.  Plans not
 * ready: FSP_ERR_NOT_READY.  Synchronises `stream`; allocates nothing. */
fsp_status fsp_autotune_batch(int count, const fsp_plan* plans, const void* const* rho, void* const* phi, int reps,
                              void* stream);

/* A set of solves replayed as one HIP graph (no per-call launch cost; no
 * passage of the paper: a launch-cost device of this library).
 * fsp_batch_create records count (plan, rho, phi) triples with the rules of
 * fsp_solve_batched and writes their buffers into a device-resident table (one
 * device allocation, owned by the batch); nothing is enqueued.  Solves of equal
 * shape form one launch group, however many there are (up to 65535 per
 * group).  The group that moves the most bytes runs first; the others (up to
 * eight, the smallest, after any further ones in turn) then run together on
 * three parallel branches of the graph, each group (largest first) on the
 * branch with the fewest bytes so far.  The first
 * fsp_batch_launch captures the launches, which read every item's buffers from
 * the table when they run, and launches the graph on `stream`; later calls
 * replay it.  fsp_batch_set_io(b, rho, phi, stream) replaces the rho / phi of
 * every solve (count entries each, in the order of fsp_batch_create): one
 * small kernel per 64 solves writes them into the table on `stream`, so a
 * later launch on that stream (or one ordered after it) uses them with no new
 * capture; launches already enqueued before it use the old ones.  The plans
 * and their bound buffers must stay alive and unchanged (no re-bind) while the
 * batch exists; rho / phi must stay alive while a launch that uses them runs.
 * Concurrent launches of one batch race on its workspaces.
 * FSP_ERR_OUT_OF_MEMORY if the table cannot be allocated. */
fsp_status fsp_batch_create(int count, const fsp_plan* plans, const void* const* rho, void* const* phi,
                            fsp_batch* out);
fsp_status fsp_batch_set_io(fsp_batch b, const void* const* rho, void* const* phi, void* stream);
fsp_status fsp_batch_launch(fsp_batch b, void* stream);
fsp_status fsp_batch_destroy(fsp_batch b);

/* fsp_solve with no device allocation and no plan workspace, for callers
 * that cannot allocate device memory at solve time (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc after set-up).
 * The five passes run on a workspace inside the library: one static device
 * array of FSP_STATIC_SCRATCH_BYTES per GPU, held until the process ends.
 * Plans whose one-spectrum workspace (fsp_plan_bytes' work_bytes, a quarter
 * of it on a plan with FSP_WANT_GRAD) exceeds it are rejected with
 * FSP_ERR_UNSUPPORTED_SIZE, on the host, before the plan's state is checked
 * and before anything is enqueued: grids up to 128^3 fit in both precisions.  The plan must be bound and precomputed (its Green's
 * buffer is read; its own workspace is not used); rho and phi as in fsp_solve
 * (phi may equal rho).  Every call on one GPU shares that GPU's array: two
 * calls whose work overlaps on one GPU (any plans, any streams) race and both
 * results are undefined, so callers serialise them (one stream, or events).
 * Nothing in the array needs clearing between calls: each solve writes every
 * element it later reads.  Asynchronous on `stream`; the first call on a
 * device (or the first fsp_plan_bind there) looks up that device's copy of the
 * array. */
#define FSP_STATIC_SCRATCH_BYTES (80u * 1024u * 1024u)
fsp_status fsp_solve_static(fsp_plan p, const void* rho, void* phi, void* stream);

/* Free the plan and any buffer it allocated.  Caller-owned buffers are not
 * touched.  Work still queued on a stream must finish first.  (No passage:
 * resource management.) */
fsp_status fsp_plan_destroy(fsp_plan p);

/* Where the transform of the Green's function sits in the Green's buffer.
 * The transform of the mirror-extended G2 (Section 2.2 steps 3-4) is real and
 * even on the doubled grid, so its octant holds all of it (the symmetry
 * Section 2.4 uses).  The octant k in [0,n] (scaled by V / (8 n0 n1 n2),
 * solve precision) is
 * stored in column tiles of *tile values of k2: element (k0, k1, k2) is at
 * byte *octant_offset + sizeof(real) * (((k1 * T + k2 / tile) * (n0 + 1) + k0)
 * * tile + k2 % tile), T = ceil((n2 + 1) / tile); slots with k2 > n2 hold 0.
 * Either pointer may be NULL. */
fsp_status fsp_plan_ghat_layout(fsp_plan p, size_t* octant_offset, int* tile);

/* Byte offset in the Green's buffer of octant `component`: 0 the potential's
 * (as fsp_plan_ghat_layout), 1 + a the derivative table along axis a (plans
 * with FSP_WANT_GRAD only, else FSP_ERR_INVALID_ARG).  Same blocked layout and
 * tile; a derivative octant holds T with transform -i T, T odd along a. */
fsp_status fsp_plan_octant_offset(fsp_plan p, int component, size_t* offset);

/* Model bytes that one solve moves through HBM with this plan's schedule
 * (reads + writes of its kernels, the Green's octant included: five passes,
 * fewer where the fused slab or a plane pair keeps intermediates in LDS): the
 * memory traffic against which Section 3.4 finds the solve memory-bound. */
fsp_status fsp_plan_model_bytes(fsp_plan p, double* bytes);

/* Name of a status code, and this thread's text for the last failure (no
 * passage: diagnostics). */
const char* fsp_status_str(fsp_status s);
const char* fsp_last_error(void);

/* Library version string, e.g. "fsp 0.1.0 gfx950". */
const char* fsp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FSP_H_ */
