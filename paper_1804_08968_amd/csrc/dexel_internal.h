// Internal declarations shared by the HIP kernels and the host side of libdexel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dexel {

// Device-side header at the start of every workspace.  Reset by k_init_call
// at the start of a call and (bump counters only) by k_init_op before each
// operation of a chain.
struct WsHeader {
    int32_t status;                 // dexel_status, first error wins
    int32_t abort;                  // nonzero: the remaining kernels of the call exit at once
    unsigned long long need_cap;    // largest internal-buffer size (intervals) the call needed
    unsigned long long bumpA;       // bump allocators of the per-column lists
    unsigned long long bumpI;
    unsigned long long bumpC;
    unsigned long long arena;       // bump allocator of the overflow arena
    int64_t nseg_out;
    int32_t novf[8];                // columns whose per-lane list overflowed LDS, per stage
    int64_t nseeds;                 // kept extrusion seeds of the last pass
    int64_t reserved[2];
};
static_assert(sizeof(WsHeader) <= 256, "header must fit its slot");

enum Stage { ST_K1 = 0, ST_K1B = 1, ST_K2C = 2, ST_K2F = 3, ST_K3 = 4, NSTAGE = 5 };

// Everything one dilation (or erosion) pass reads and writes.
struct OpParams {
    int32_t nx, ny;
    int64_t ncols;
    const int64_t* col_ptr;   // input CSR
    const float2* z;
    int64_t nseg;             // input interval count (-1: unknown on the host)
    int32_t erode;            // complement on read and on write
    int32_t R;                // floor(r)
    int32_t d2max;            // floor(r^2): integer squared distances d2 <= d2max are in the ball
    const float* H;           // H[d2] = float(sqrt(double(r)^2 - d2)), d2 = 0..d2max
    WsHeader* hdr;
    int64_t cap;              // capacity (intervals) of A, I, B, C and of the arena
    // A: per-column row offset V0 (2D dilation of the column's own row at radius r)
    int64_t* offA; int32_t* cntA; float2* A;
    // I: per-column intersection of V0 over the rows within R (excluding the own row)
    int64_t* offI; int32_t* cntI; float2* I;
    // B: per-column extrusion seeds (closest-parent pieces) kept for the y pass, CSR
    int64_t* offB; int32_t* cntB; float2* B; uint8_t* tagB;
    float2* hullB;            // per column: hull of the kept seeds' chords at |dy| = 1
    // C: per-column result (complemented for erosion)
    int64_t* offC; int32_t* cntC; float2* C;
    int32_t* ovf;             // [NSTAGE * ncols] overflow column lists
    float2* arena;            // global lists for overflow columns
    int64_t* bsum;            // scan scratch
    // output CSR
    int64_t* out_col_ptr; float2* out_z; int64_t out_cap;
    int32_t out_is_intermediate;   // 1: output overflow is a workspace error, not a capacity error
};

// Launchers (dexel_kernels.hip).  All enqueue on `s`, none synchronises.
hipError_t launch_init_call(WsHeader* hdr, hipStream_t s);
hipError_t launch_init_op(WsHeader* hdr, hipStream_t s);
hipError_t launch_check_colptr(const OpParams& p, hipStream_t s);
hipError_t launch_validate(const OpParams& p, hipStream_t s);
// Profiled intervals of one pass, one per launch group: row offset, its
// replay, neighbour intersection, its replay, seed count, its replay, seed
// scan, seed fill, its replay, y dilation + union, its replay, result scan,
// compaction copy.
constexpr int NPROF = 13;
// ev: nullptr, or NPROF + 1 events recorded on `s` at the stage boundaries.
hipError_t launch_offset_pass(const OpParams& p, hipStream_t s, hipEvent_t* ev);
hipError_t launch_finish(WsHeader* hdr, const int64_t* out_col_ptr, int64_t ncols,
                         int64_t* nseg_out, int32_t* status, hipStream_t s);

}  // namespace dexel
