/*
 * dexel.h -- C ABI of libdexel: exact dilation / erosion of dexel shapes by a
 * ball on AMD Instinct MI355X (gfx950).
 *
 * Method: Chen, Panozzo, Dumas, "Half-Space Power Diagrams and Discrete
 * Surface Offsets".  A dexel shape is a 2D grid of columns, each holding a
 * sorted list of disjoint z-intervals (Sec. 3.1, "Dexel Representation").
 * Dilation by a closed ball of radius r is the set of points within r of the
 * shape (Sec. 3.1, "Dilation" equation); erosion is the complement of the
 * dilated complement (Sec. 3.1, "Erosion"); opening and closing chain the two
 * (Sec. 4, "Topological Cleaning").  The result is computed by the separable
 * two-stage scheme of Sec. 3.3: an extrusion along x whose pieces carry the
 * distance to their closest parent, then a dilation along y in which the
 * pieces are weighted seeds (weight r^2 - dx^2) of a power diagram, then a
 * per-column interval union.
 *
 * Data layout (CSR, all device memory, owned by the caller):
 *   column id c = y * nx + x (x fastest; a grid row is one contiguous span)
 *   col_ptr[c] .. col_ptr[c+1]  intervals of column c, col_ptr[0] = 0
 *   z[2k], z[2k+1]              (z_in, z_out) of interval k, float32
 * Canonical input (required): per column sorted, finite, z_in <= z_out and
 * z_out_k < z_in_{k+1} (touching intervals are merged).  Zero-length
 * intervals are allowed.  `z` must be 8-byte aligned.
 *
 * Geometry conventions: columns sit on the integer lattice with unit
 * spacing; r and z are in the same unit.  The ball is closed (a column at
 * lateral distance exactly r contributes its intervals unchanged).  Columns
 * outside the grid contribute nothing to a dilation and impose nothing on an
 * erosion (only in-grid columns are complemented).  z is unbounded.
 * Erosion output keeps only intervals of positive length.
 *
 * Numerics: every output endpoint is one float32 rounding of a - h or b + h,
 * where a, b are input endpoints (dilation) or input endpoints / +-inf
 * (erosion) and h is the float32 rounding of the double square root of
 * r^2 - d2 (d2 = integer squared lateral distance, r^2 formed exactly in
 * double).  Overlap tests use exact float32 comparisons, so the output is
 * the float32 canonical union of those chords, independent of the order or
 * pruning of the work.
 *
 * Ownership: the library never allocates device memory.  Inputs, outputs and
 * a workspace (size from dexel_workspace_size) are supplied by the caller.
 * A context owns host-side state only (autotune choices, error text); the
 * radius table of a call is computed on the host and passed to the device
 * through kernel arguments, so no host buffer outlives a call either.
 * One host thread per context at a time.
 *
 * Asynchrony and errors: host-detectable argument errors are returned before
 * anything is enqueued.  Everything else runs on `stream` (a hipStream_t, or
 * NULL for the default stream).  Device-detected conditions are written to
 * *out->status (a dexel_status) and *out->nseg_out.  Without
 * DEXEL_FLAG_SYNC the call returns DEXEL_OK meaning "enqueued"; with it, the
 * call synchronises `stream` and returns the device status.
 */
#ifndef DEXEL_H
#define DEXEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DEXEL_API_VERSION 1

typedef enum {
    DEXEL_OK = 0,
    DEXEL_ERR_INVALID = -1,       /* bad argument (null pointer, size, r < 0 or not finite, ...) */
    DEXEL_ERR_NOT_CANONICAL = -2, /* input failed validation (DEXEL_FLAG_VALIDATE)             */
    DEXEL_ERR_CAPACITY = -3,      /* output needs more than cap_seg intervals; see nseg_out     */
    DEXEL_ERR_WORKSPACE = -4,     /* workspace too small; see dexel_workspace_need               */
    DEXEL_ERR_HIP = -5,           /* a HIP runtime call failed                                   */
    DEXEL_ERR_UNSUPPORTED = -6    /* outside the supported range (e.g. r > 250)                  */
} dexel_status;

typedef enum { DEXEL_DILATE = 0, DEXEL_ERODE = 1, DEXEL_OPEN = 2, DEXEL_CLOSE = 3 } dexel_op;

#define DEXEL_FLAG_SYNC 1u     /* synchronise the stream and return the device status   */
#define DEXEL_FLAG_VALIDATE 2u /* check the input is canonical before computing          */
#define DEXEL_FLAG_RAYS_X 4u   /* dexel_dexelize only: rays along x (grid over y, z)      */
#define DEXEL_FLAG_RAYS_Y 8u   /* dexel_dexelize only: rays along y (grid over z, x)      */
/* Offsets: evaluate every column with the general (staged) kernels,
 * without the direct evaluation of fragmented passes and the tiled fast
 * paths (the thin-column erosion filter and the single-interval dilation
 * test); for comparison, the result is the same, bit for bit. */
#define DEXEL_FLAG_GENERAL 16u

typedef struct dexel_ctx dexel_ctx;

/* Input grid (device pointers). */
typedef struct {
    int32_t nx, ny;         /* grid size, both >= 1                              */
    int64_t nseg;           /* number of intervals = col_ptr[nx*ny]               */
    const int64_t* col_ptr; /* [nx*ny + 1]                                        */
    const float* z;         /* [2*nseg] (z_in, z_out) pairs                       */
} dexel_grid_view;

/* Output grid (device pointers), same nx, ny as the input. */
typedef struct {
    int32_t nx, ny;
    int64_t cap_seg;   /* capacity of z in intervals                                        */
    int64_t* col_ptr;  /* [nx*ny + 1], always written when the computation completes        */
    float* z;          /* [2*cap_seg]; untouched if the result needs more than cap_seg       */
    int64_t* nseg_out; /* device scalar: exact number of output intervals (also on overflow) */
    int32_t* status;   /* device scalar: dexel_status of the enqueued work                   */
} dexel_grid_out;

/* One request of a batch: `op` is a dexel_op. */
typedef struct {
    dexel_grid_view in;
    float r;
    int32_t op;
    dexel_grid_out out;
} dexel_batch_item;

/* Create a context on HIP device `device`.  Returns DEXEL_ERR_INVALID for a
 * null `ctx`, DEXEL_ERR_HIP if the device cannot be selected. */
dexel_status dexel_ctx_create(int device, dexel_ctx** ctx);
void dexel_ctx_destroy(dexel_ctx* ctx);

/* Bytes of workspace needed for one call of dexel_offset on `in` with radius
 * r and operation op.  `cap_hint` is the capacity, in intervals, of each
 * internal buffer; 0 picks a default from the input size (2 * nseg +
 * 2 * nx * ny).  If a call ends with DEXEL_ERR_WORKSPACE, pass the value
 * reported by dexel_workspace_need as the hint and retry.  Only nx, ny and
 * nseg of `in` are read (no device access). */
dexel_status dexel_workspace_size(dexel_ctx* ctx, const dexel_grid_view* in, float r, int32_t op,
                                  int64_t cap_hint, size_t* bytes);

/* After a call completed (stream synchronised), read the capacity hint the
 * call needed from the workspace header (a small device-to-host copy).
 * After DEXEL_ERR_WORKSPACE it is at least what the stage that ran out asked
 * for (a later stage may ask for more); after success it is the largest
 * internal buffer, in intervals, that the call used, so a workspace sized
 * with it holds the same call, with the same kernel variant, again. */
dexel_status dexel_workspace_need(dexel_ctx* ctx, const void* ws, int64_t* cap_hint);

/* Allocation-free dexel_offset, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and result as dexel_offset, without a
 * workspace argument: the workspace is a static device array of
 * DEXEL_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends (its address is looked up once per device by
 * dexel_ctx_create).  The call allocates nothing (no hipMalloc, no pinned
 * host memory, no profiling events) and records no memset, so it can be
 * captured in a graph.  Every call on one GPU uses that GPU's one array:
 * calls that overlap on a GPU (several streams, contexts or threads at
 * once) race and must be serialised by the caller.  A call whose workspace
 * (dexel_workspace_size with cap_hint 0) exceeds the array returns
 * DEXEL_ERR_UNSUPPORTED before anything is enqueued; grids up to about
 * 512 x 512 at a few intervals per column fit.  DEXEL_ERR_WORKSPACE in
 * *out->status means the input needed more internal capacity than the
 * array holds (no retry is possible: use dexel_offset). */
#define DEXEL_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
dexel_status dexel_offset_noalloc(dexel_ctx* ctx, const dexel_grid_view* in, float r, int32_t op,
                                  dexel_grid_out* out, void* stream, uint32_t flags);

/* Dilation by the closed ball of radius r (Sec. 3.1 "Dilation"; computed as
 * in Sec. 3.3).  `in` and `out` must not alias; ws/ws_bytes from
 * dexel_workspace_size with op = DEXEL_DILATE. */
dexel_status dexel_dilate(dexel_ctx* ctx, const dexel_grid_view* in, float r, dexel_grid_out* out,
                          void* ws, size_t ws_bytes, void* stream, uint32_t flags);

/* Erosion: complement, dilate, complement (Sec. 3.1 "Erosion"). */
dexel_status dexel_erode(dexel_ctx* ctx, const dexel_grid_view* in, float r, dexel_grid_out* out,
                         void* ws, size_t ws_bytes, void* stream, uint32_t flags);

/* Any dexel_op; DEXEL_OPEN = dilate(erode(S)), DEXEL_CLOSE = erode(dilate(S))
 * (Sec. 4 "Topological Cleaning").  The intermediate stays in the workspace. */
dexel_status dexel_offset(dexel_ctx* ctx, const dexel_grid_view* in, float r, int32_t op,
                          dexel_grid_out* out, void* ws, size_t ws_bytes, void* stream,
                          uint32_t flags);

/* Per-column Boolean operations (CSG) of two grids of the same nx, ny
 * (Sec. 2, item (3): CSG carried out directly in dexel space).  The shell of
 * Sec. 4, "3D Printing", is DEXEL_CSG_DIFFERENCE of a dilation and an erosion
 * of the same shape.  The operations are the regularised ones of solid
 * modelling: the result is the closure of the interior of the set
 * operation, so input intervals of zero length are ignored, touching result
 * pieces form one interval, and no piece of zero length is produced.
 * Endpoints are copied from the inputs, never computed.
 *
 * `a`, `b`: canonical grids (as for dexel_offset); `out`: same nx, ny, with
 * cap_seg intervals of room (the result has at most nseg(a) + nseg(b)); on
 * overflow out->status is DEXEL_ERR_CAPACITY and *out->nseg_out the need.
 * `ws`: device memory of dexel_csg_workspace_size bytes, 256-byte aligned,
 * used during the call only.  DEXEL_FLAG_SYNC as for dexel_offset;
 * DEXEL_FLAG_VALIDATE is not supported (DEXEL_ERR_UNSUPPORTED). */
typedef enum { DEXEL_CSG_UNION = 0, DEXEL_CSG_INTERSECT = 1, DEXEL_CSG_DIFFERENCE = 2 } dexel_csg_op;
dexel_status dexel_csg_workspace_size(dexel_ctx* ctx, const dexel_grid_view* a, size_t* bytes);
dexel_status dexel_csg(dexel_ctx* ctx, const dexel_grid_view* a, const dexel_grid_view* b, int32_t op,
                       dexel_grid_out* out, void* ws, size_t ws_bytes, void* stream, uint32_t flags);

/* Canonical form of a grid whose columns hold closed intervals in any order,
 * overlapping freely: per column, the union of its intervals listed sorted,
 * with intervals that overlap or touch joined (Sec. 3.1, "Dexel
 * Representation"; the input form every offset call expects).  Endpoints are
 * copied, never computed, so the result is exact.
 *
 * `in`: nx, ny, nseg, col_ptr (device int64[nx*ny+1], col_ptr[0] = 0,
 * non-decreasing, col_ptr[nx*ny] = nseg) and z (device float32 pairs; within
 * a column in any order).  Every interval must be finite with start <= end.
 * A violation of either rule is reported as DEXEL_ERR_INVALID in
 * out->status, and nothing is written.  `out`: same nx, ny, with cap_seg
 * intervals of room (the result has at most nseg); on overflow out->status
 * is DEXEL_ERR_CAPACITY and *out->nseg_out the need.  `ws`: device memory of
 * dexel_canonicalize_workspace_size bytes (about 4 B per column and 8 B per
 * input interval beyond dexel_csg's), 256-byte aligned, used during the call
 * only.  DEXEL_FLAG_SYNC as for dexel_offset; DEXEL_FLAG_VALIDATE is not
 * supported (the input is always checked).  A column whose running union
 * stays within 32 intervals takes a fast path; any other is sorted by one
 * GPU lane (O(m log m) for m intervals). */
dexel_status dexel_canonicalize_workspace_size(dexel_ctx* ctx, const dexel_grid_view* in, size_t* bytes);
dexel_status dexel_canonicalize(dexel_ctx* ctx, const dexel_grid_view* in, dexel_grid_out* out, void* ws,
                                size_t ws_bytes, void* stream, uint32_t flags);

/* Dexelisation of analytic primitives into an nx x ny grid (Sec. 1 and Sec.
 * 3.1, "Dexel Representation": the intersections of a solid with parallel
 * rays from a uniform 2D grid).  The rays are the z-parallel lines through
 * the cell centres (x + 0.5, y + 0.5).  `prims` (device, 8-byte aligned)
 * holds nprims records of 7 doubles (kind, a0, a1, a2, b0, b1, b2):
 *   DEXEL_PRIM_BALL: centre a, radius b0; meets the ray of a cell whose
 *     squared lateral distance rho2 to the centre is below b0^2, in the
 *     closed chord [a2 - h, a2 + h], h = sqrt(b0^2 - rho2);
 *   DEXEL_PRIM_BOX: corners a <= b; meets the rays of the cells with
 *     ceil(a0 - 0.5) <= x <= floor(b0 - 0.5) and ceil(a1 - 0.5) <= y <=
 *     floor(b1 - 0.5) (the cell centre lies in the footprint), in [a2, b2].
 * Chord ends are computed in float64 (each operation rounded once), rounded
 * once to float32, and merged per column where they overlap or touch; the
 * result is canonical.  Values must be finite and within float32 range.  A
 * column may hold at most 64 intervals (else DEXEL_ERR_UNSUPPORTED in
 * out->status); an unknown kind gives DEXEL_ERR_INVALID there.  `out` and
 * `ws` (dexel_dexelize_workspace_size bytes, 256-byte aligned) as for
 * dexel_csg; DEXEL_FLAG_VALIDATE is not supported.
 *
 * Rays along another axis (the dexel structures in three orthogonal
 * directions suggested in the "Limitations" paragraph of Sec. 4 and in
 * Sec. 5): with DEXEL_FLAG_RAYS_X the grid's two axes are y and z (nx cells
 * along y, ny along z) and the intervals lie along x; with DEXEL_FLAG_RAYS_Y they are z and x and the
 * intervals lie along y.  The rules above apply with the coordinates taken
 * in that order, (a1, a2, a0) or (a2, a0, a1), and likewise for b; a ball's
 * radius is b0 in every case.  Both flags together: DEXEL_ERR_INVALID. */
typedef enum { DEXEL_PRIM_BALL = 0, DEXEL_PRIM_BOX = 1 } dexel_prim_kind;
dexel_status dexel_dexelize_workspace_size(dexel_ctx* ctx, int32_t nx, int32_t ny, size_t* bytes);
dexel_status dexel_dexelize(dexel_ctx* ctx, int32_t nx, int32_t ny, const double* prims, int32_t nprims,
                            dexel_grid_out* out, void* ws, size_t ws_bytes, void* stream, uint32_t flags);

/* Workspace for dexel_batch_offset over `items` (the largest single-item
 * need, since items share the workspace in sequence). */
dexel_status dexel_batch_workspace_size(dexel_ctx* ctx, int32_t n, const dexel_batch_item* items,
                                        int64_t cap_hint, size_t* bytes);

/* Offset n independent shapes, each with its own radius and op, in one
 * enqueue on `stream`.  Each item's status/nseg_out are written separately. */
dexel_status dexel_batch_offset(dexel_ctx* ctx, int32_t n, const dexel_batch_item* items, void* ws,
                                size_t ws_bytes, void* stream, uint32_t flags);

/* Kernel variants.  The per-column kernels keep per-lane interval lists in
 * LDS; a variant fixes their capacities (larger lists replay fewer columns
 * from global memory, smaller ones fit more resident waves per CU).  All
 * variants compute the same result.  dexel_set_variant forces a variant
 * (0..DEXEL_NVARIANT-1) for every later call of the context, -1 restores
 * automatic choice: the variant dexel_autotune picked for a batch with the
 * same signature (item count, grid sizes, ops, radii, order of magnitude of
 * each input size), else variant 0.
 *
 * dexel_autotune runs the batch once per variant untimed and `reps` times
 * timed (HIP events on `stream`, synchronising), records the fastest for this
 * batch signature and returns it in *chosen; ms[DEXEL_NVARIANT] (optional)
 * receives the mean milliseconds per run of each variant.  Outputs and
 * workspace are used as by dexel_batch_offset; device errors are returned. */
#define DEXEL_NVARIANT 4
dexel_status dexel_set_variant(dexel_ctx* ctx, int variant);
dexel_status dexel_autotune(dexel_ctx* ctx, int32_t n, const dexel_batch_item* items, void* ws,
                            size_t ws_bytes, void* stream, int32_t reps, int32_t* chosen, float* ms);

/* Profiling.  When enabled, every pass of every later call records HIP
 * events on its stream around each of its DEXEL_NPROF launch groups: column
 * gaps, direct evaluation, thin-column erosion, chord-extreme dilation test, row offset, its
 * replays, test against the row offset and gap cut, neighbour
 * intersection, its
 * replay, extrusion seeds, their replay, y dilation with per-column union,
 * its replay, result scan, compaction copy.
 * dexel_profile_read waits for the recorded events and returns the
 * accumulated milliseconds per group and the number of passes (a dilation or
 * erosion is one pass, open/close two); reset != 0 clears the accumulators. */
#define DEXEL_NPROF 15
dexel_status dexel_profile_enable(dexel_ctx* ctx, int on);
dexel_status dexel_profile_read(dexel_ctx* ctx, double* ms, int64_t* passes, int reset);

/* Sizes recorded by the last pass of the last completed call in `ws`
 * (stream synchronised; small device-to-host copy): stats[0] row-offset
 * intervals, [1] neighbour-intersection intervals, [2] kept extrusion seeds,
 * [3] result intervals of the pass, [4] overflow-arena intervals used,
 * [5] columns replayed from global memory, [6] capacity hint needed,
 * [7] output intervals of the call (-1 if it failed). */
dexel_status dexel_workspace_stats(dexel_ctx* ctx, const void* ws, int64_t* stats);

const char* dexel_status_string(dexel_status s);
/* Text of the last host-side error of this context ("" if none). */
const char* dexel_last_error(const dexel_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DEXEL_H */
