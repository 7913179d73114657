// Internal declarations shared by the HIP kernels and the host side of libdexel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dexel {

// Device-side header at the start of every workspace.  Reset by k_init_call
// at the start of a call and (bump counters only) by k_init_pass before the
// second pass of a chain.
struct WsHeader {
    int32_t status;                 // dexel_status, first error wins (workspace-wide errors)
    int32_t abort;                  // nonzero: the remaining kernels of the call exit at once
    unsigned long long need_cap;    // largest internal-buffer size (intervals) the call used or asked for
                                    // (the current pass's counters are folded in when it is read)
    unsigned long long bumpA;       // bump allocators of the per-column lists
    unsigned long long bumpI;
    unsigned long long bumpC;
    unsigned long long arena;       // bump allocator of the overflow arena
    int64_t nseg_out;
    int32_t novf[13];               // columns on each overflow / work list (Stage)
    unsigned long long nseeds;      // kept extrusion seeds of the current pass
    int64_t reserved[2];
};
static_assert(sizeof(WsHeader) <= 256, "header must fit its slot");

// Overflow lists: columns whose per-lane list overflowed in K1, K1b, K2 (seed
// slot) and K3, replayed one lane per column; and columns deferred as heavy
// in K2, K1b and K3, or overflowing K1's lane replay, replayed one wave per
// column (z slabs); the columns the tiled dilation test leaves to the test
// against V0 (ST_SOLB), to the gap cut (ST_GAP) and to the wide gap cut
// (ST_GAPW: more gaps, one wave per column); and the columns of a direct
// evaluation whose list overflowed: the lane's (ST_DIRT, to a team of lanes)
// and the team's (ST_DIRW, to a whole wave).
enum Stage {
    ST_K1 = 0, ST_K1B = 1, ST_K2 = 2, ST_K3 = 3,
    ST_K2H = 4, ST_K1BH = 5, ST_K3H = 6, ST_K1H = 7, ST_GAP = 8, ST_SOLB = 9, ST_DIRT = 10,
    ST_DIRW = 11, ST_GAPW = 12, NSTAGE = 13
};

// Seed slots per column: the seeds of a column are written at
// B[g * slot ...] (g = global column, slot = Pass::seed_slot); a column with
// more seeds is recomputed into the workspace arena and its offset stored as
// -(pos + 1).  The slot is SEED_SLOT entries, or SEED_SLOT_WIDE for a call
// with a radius of at least SEED_WIDE_R whose wide slots take at most
// SEED_WIDE_BYTES (at such radii many columns keep more than 64 seeds, and
// each of them is evaluated twice; on large grids the wide slots would cost
// more memory than the second evaluation costs time).
constexpr int SEED_SLOT = 64;
constexpr int SEED_SLOT_WIDE = 128;
constexpr int SEED_WIDE_R = 24;
constexpr long long SEED_WIDE_BYTES = 1ll << 30;

// One shape of one pass, in device memory.  Per-column arrays are already
// offset to the shape's first global column, so kernels index them with the
// shape-local column id.
struct Shape {
    int32_t nx, ny;
    int64_t ncols;
    int64_t gbase;            // first global column of the shape in this pass (multiple of 64)
    const int64_t* col_ptr;   // input CSR
    const float2* z;
    const int64_t* zoff;      // if set, the input pairs start at z + *zoff (chained pass input)
    int64_t nseg;             // input interval count (-1: unknown on the host)
    int32_t erode;            // complement on read and on write
    int32_t R;                // floor(r)
    int32_t d2max;            // floor(r^2)
    int32_t index;            // item index (status slot)
    const float* H;           // H[d2] = float(sqrt(double(r)^2 - d2)), d2 = 0..d2max
    // per input column (k_col_gaps): largest gap, an upper bound; first and
    // last item (x, y of the first, x, y of the last; unset if empty)
    float* gap;
    float4* ends;
    int64_t* offA; int32_t* cntA;
    int64_t* offI; int32_t* cntI;
    // seed position (see SEED_SLOT), count, size of the low group, and two
    // hulls per column, [2c] low group, [2c + 1] high group (x, y: of the
    // seed chords at |dy| = 1; z, w: of the seed pieces themselves)
    int64_t* offB; int32_t* cntB; int32_t* loB; float4* hullB;
    int64_t* offC; int32_t* cntC;
    int64_t* scanC;           // global exclusive scan of the result counts
    // output
    int64_t* out_col_ptr;
    float2* out_z;
    const int64_t* out_zoff;  // if set, results are written at out_z + *out_zoff
    int64_t out_cap;
    // tiled fast paths: `fast` = FAST_THIN for an erosion pass the thin-column
    // max / min filter evaluates first, FAST_SOLID for a dilation pass whose
    // columns the chord-extreme test, the test against V0 and the gap cut
    // settle; the shape's tiles are tbase .. of the pass.  gen[c] holds GEN_*
    // bits, need[c] the general stages column c must run (NEED_* bits).
    // FAST_DIRECT: the shape is evaluated directly, without tiles.
    int32_t fast;
    int32_t pad1;
    int64_t tbase;
    uint8_t* gen;
    uint8_t* need;
    float4* lu;               // FAST_SOLID, unsettled columns: chord extremes (see k_solid_dilate)
    int32_t out_is_intermediate;
    int32_t last_pass;        // write the caller's nseg_out / status after this pass
    int64_t* out_nseg;
    int32_t* out_status;
};

// Kernel argument of every per-pass kernel.
struct Pass {
    const Shape* shapes;      // [nshapes]
    const int64_t* sbase;     // [nshapes + 1] first global column of each shape; sbase[n] = gcols
    int32_t nshapes;
    int32_t ndirect;          // the pass has shapes evaluated directly (FAST_DIRECT; 0 / 1)
    int64_t gcols;            // padded global column count of the pass
    int64_t ntiles;           // tiles of the tiled fast paths over the pass's shapes that have one
    int32_t thin_lds;         // dynamic LDS bytes of k_thin_erode (largest R of its shapes)
    int32_t solid_lds;        // dynamic LDS bytes of k_solid_dilate (largest R of its shapes)
    int16_t nthin, nsolid;    // the pass has shapes with each fast path (0 / 1)
    int32_t k1_round;         // k_row_offset's launch: 1 before the dilation tests' V0 stage, 2 after
    int32_t seed_slot;        // seed slot entries per column (SEED_SLOT or SEED_SLOT_WIDE)
    WsHeader* hdr;
    int32_t* shape_status;    // [items] per-item status (output capacity)
    int64_t cap;              // capacity (intervals) of A, I, B, C and of the arena
    float2* A;
    float2* I;
    float2* B;                // [gcols * seed_slot] seed slots, tags in tagB
    uint8_t* tagB;
    float2* C;
    int32_t* cntC_g;          // global views of the per-column result arrays (for the scan)
    int64_t* scanC_g;
    int32_t* ovf;             // [NSTAGE * gcols] overflow column lists (global ids)
    float2* arena;
    uint8_t* arena_tag;       // [cap] tags of seeds placed in the arena
    int64_t* bsum;
};

// Descriptor upload through kernel arguments (no host buffer outlives the call).
constexpr int DESC_CHUNK = 12;
struct ShapeChunk {
    Shape s[DESC_CHUNK];
    int32_t n;
    int32_t first;
};
constexpr int I64_CHUNK = 256;
struct I64Chunk {
    int64_t v[I64_CHUNK];
    int32_t n;
    int32_t first;
};

// Launchers (dexel_kernels.hip).  All enqueue on `s`, none synchronises.
hipError_t launch_put_shapes(Shape* dst, const Shape* host, int n, hipStream_t s);
hipError_t launch_put_i64(int64_t* dst, const int64_t* host, int n, hipStream_t s);
constexpr int F32_CHUNK = 256;
struct F32Chunk {
    float v[F32_CHUNK];
    int32_t n;
    int32_t first;
};
hipError_t launch_put_f32(float* dst, const float* host, int n, hipStream_t s);
hipError_t launch_init_call(WsHeader* hdr, int32_t* shape_status, int nitems, hipStream_t s);
hipError_t launch_init_pass(WsHeader* hdr, hipStream_t s);
hipError_t launch_check_input(const Pass& p, int validate, hipStream_t s);
// Profiled intervals of one pass, one per launch group: column gaps, direct
// evaluation, thin-column erosion, chord-extreme dilation test, row offset, its replays,
// test against V0 and gap cut (with the row offsets they still need),
// neighbour intersection, its replays, seeds, their replays, y dilation +
// union, its replays, result scan, compaction.
constexpr int NPROF = 15;
// FAST_DIRECT: every column of the pass is the union of its stencil's chords,
// evaluated by teams of lanes (k_direct); the staged kernels skip the shape.
enum FastPath { FAST_NONE = 0, FAST_THIN = 1, FAST_SOLID = 2, FAST_DIRECT = 3 };
// Direct evaluation is chosen for radii up to DIRECT_RMAX (its kernels stage
// one stencil row's column pointers, at most 2 * DIRECT_RMAX + 2 of them).
constexpr int DIRECT_RMAX = 16;
// Tiled fast paths: tiles of THIN_TX x THIN_TY (thin erosion) or
// THIN_TX x SOLID_TY (dilation test) output columns, radii up to THIN_RMAX.
// LDS bytes a tile stages at integer radius R: per staged column one float2
// (thin) or the first start and last end (dilation), then the stencil's half-widths
// row by row (row |dy| = k holds H[dx^2 + k^2] for dx = -w_k .. w_k, padded
// to a multiple of four floats, so that four of them are one 16-byte load;
// (R + 1) (2R + 4) floats bound the table, and the kernels place what
// follows it there), and per row its width w_k and its offset in the table.
constexpr int THIN_TX = 64;
constexpr int THIN_TY = 16;
constexpr int SOLID_TY = 8;
constexpr int THIN_RMAX = 32;
inline int thin_lds_bytes(int R, int d2max) {
    (void)d2max;
    return (THIN_TX + 2 * R) * (THIN_TY + 2 * R) * 8 + 4 * (R + 1) * (2 * R + 4) + 8 * (R + 1);
}
inline int solid_lds_bytes(int R, int d2max) {
    (void)d2max;
    return (THIN_TX + 2 * R) * (SOLID_TY + 2 * R) * 8 + 4 * (R + 1) * (2 * R + 4) + 8 * (R + 1);
}
// need[] bits: stages of the general kernels a column runs.
constexpr int NEED_UNION = 1;   // y union (the column is general itself)
constexpr int NEED_SEEDS = 2;   // neighbour intersection and seeds (a general column within R rows)
constexpr int NEED_ROW = 4;     // row offset (a general column within 2R rows)
// gen[] bits.
constexpr int GEN_V0 = 1;       // FAST_SOLID: the column's V0 is evaluated before the general stages
constexpr int GEN_GENERAL = 2;  // the column is left to the general kernels
// ev: nullptr, or NPROF + 1 events recorded on `s` at the stage boundaries.
// variant: kernel variant (per-lane LDS list capacities), 0..NVARIANT-1.
constexpr int NVARIANT = 4;
hipError_t launch_pass(const Pass& p, hipStream_t s, hipEvent_t* ev, int variant);
// Dynamic-LDS limit of the tiled kernels (once per context): sets the largest
// accepted value up to max_lds and returns it (65536 at least).
int prepare_kernels(int max_lds);
hipError_t launch_finish(const Pass& p, int64_t* zbase, hipStream_t s);

// Per-column Boolean operation of two grids (dexel_csg).  Workspace: header,
// counts [ncols], scan [ncols + 1], block sums.
enum CsgOp { CSG_UNION = 0, CSG_INTERSECT = 1, CSG_DIFFERENCE = 2 };
struct CsgArgs {
    const int64_t* a_ptr;
    const float2* a_z;
    const int64_t* b_ptr;
    const float2* b_z;
    int64_t ncols;
    int32_t op;
    int32_t pad;
    WsHeader* hdr;
    int32_t* cnt;
    int64_t* scan;
    int64_t* bsum;
    int64_t* out_ptr;
    float2* out_z;
    int64_t cap;
    int64_t* out_nseg;
    int32_t* out_status;
};
hipError_t launch_csg(const CsgArgs& a, hipStream_t s);

// Dexelisation of balls and boxes (dexel_dexelize).  Same workspace layout
// as dexel_csg.
struct DexArgs {
    const double* prims;  // [nprims * 7] records (kind, a0, a1, a2, b0, b1, b2)
    int32_t nprims;
    int32_t nx, ny;
    int32_t axis;         // the rays' axis: 0 = x, 1 = y, 2 = z
    int64_t ncols;
    WsHeader* hdr;
    int32_t* cnt;
    int64_t* scan;
    int64_t* bsum;
    int64_t* out_ptr;
    float2* out_z;
    int64_t cap;
    int64_t* out_nseg;
    int32_t* out_status;
    int32_t* spill;       // [dexelize_tiles] tiles redone with DEX_CAP slots
};
constexpr int DEX_CAP = 64;  // most intervals one column may hold

// Canonical form of per-column interval lists (dexel_canonicalize).  The
// CSG workspace layout, then the list of long columns and a scratch copy of
// the input intervals.
struct CanonArgs {
    const int64_t* in_ptr;
    const float2* in_z;
    int64_t nseg;
    int64_t ncols;
    WsHeader* hdr;
    int32_t* cnt;
    int64_t* scan;
    int64_t* bsum;
    int64_t* out_ptr;
    float2* out_z;
    int64_t cap;
    int64_t* out_nseg;
    int32_t* out_status;
    int32_t* longc;       // [ncols] columns left to the sorting tier (count in hdr->novf[0])
    float2* sorted;       // [nseg] the sorting tier's copies, at the columns' own input offsets
};
hipError_t launch_canonicalize(const CanonArgs& a, hipStream_t s);
int64_t dexelize_tiles(int32_t nx, int32_t ny);
hipError_t launch_dexelize(const DexArgs& a, hipStream_t s);

}  // namespace dexel
