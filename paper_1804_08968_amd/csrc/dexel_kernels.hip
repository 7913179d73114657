// HIP kernels of libdexel for gfx950 (CDNA4, wave64).
//
// One dilation pass of a dexel grid by a closed ball of radius r follows the
// separable scheme of Chen, Panozzo, Dumas, Sec. 3.3: every input interval is
// extruded along x to the columns within distance R = floor(r) of its own,
// keeping for each covered z the closest parent only (the extruded piece
// then carries the weight r^2 - dx^2); the weighted pieces are dilated along
// y as seeds of a power diagram (their chord at row offset dy has half-width
// sqrt(r^2 - dx^2 - dy^2)); the chords of each output column are merged.
//
// GPU organisation (one lane per output column, 64 columns per workgroup):
//   K1  row offset   V0(c) = union of the chords of the column's own row
//                    (dy = 0): the 2D offset of that row at radius r.
//   K1b neighbour    I(c)  = intersection of V0 over the rows y+-1 .. y+-R.
//                    Every output column within R rows of c contains I(c).
//   K2  seeds        closest-parent extrusion pieces of c's row at column c
//                    (tag t = |dx|), computed by painting the row's columns
//                    in order of |dx|; a piece is kept only if its chord at
//                    |dy| = 1 (its largest off-row chord) is not inside I(c):
//                    a dropped seed's power disk lies inside V0 of every row
//                    it can reach.  One traversal writes a column's seeds to
//                    its fixed slot; the rare longer lists are recomputed
//                    into the workspace arena.
//   K3  y dilation   out(c) = V0(c) U chords of the kept seeds of the rows
//                    y+-1 .. y+-R at their power weight r^2 - t^2 - dy^2.
//   K4  compaction   exclusive scan of the per-column counts, copy to CSR.
// Erosion complements each in-grid input column on read (closed gaps with
// -inf/+inf ends) and the result on write.
//
// Every candidate chord is [fl(a - H[d2]), fl(b + H[d2])] with H a float
// table and one rounding per end; the merge is an exact float union.  A
// skipped candidate is always contained in the union of kept ones, so the
// result equals the float union of all chords of the ball stencil.
//
// Per-lane interval lists live in LDS, interleaved by lane (element i of
// lane l at i*64 + l) so that lanes touching the same index hit distinct
// banks.  A list that outgrows its LDS capacity sends its column to a
// global-memory replay of the same code ("fallback"), sized from an upper
// bound and carved from the workspace arena.
#include <hip/hip_runtime.h>

#include "../../include/dexel.h"
#include "dexel_internal.h"

namespace dexel {

#define DX_INF __builtin_inff()

// Loads from workspace and input arrays go through gld(): the pointers come
// from descriptors in memory, so the compiler would otherwise emit flat
// loads, which also count against the LDS wait counter and make every LDS
// wait also wait for outstanding global loads.
#define DX_GLOBAL __attribute__((address_space(1)))
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 gld(const float2* p) {
    const f2v v = *(const DX_GLOBAL f2v*)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ float4 gld(const float4* p) {
    const f4v v = *(const DX_GLOBAL f4v*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float gld(const float* p) { return *(const DX_GLOBAL float*)p; }
__device__ __forceinline__ int64_t gld(const int64_t* p) { return *(const DX_GLOBAL int64_t*)p; }
__device__ __forceinline__ int32_t gld(const int32_t* p) { return *(const DX_GLOBAL int32_t*)p; }
__device__ __forceinline__ uint8_t gld(const uint8_t* p) { return *(const DX_GLOBAL uint8_t*)p; }
__device__ __forceinline__ void gst(float2* p, float2 v) { *(DX_GLOBAL f2v*)p = f2v{v.x, v.y}; }
__device__ __forceinline__ void gst(float4* p, float4 v) { *(DX_GLOBAL f4v*)p = f4v{v.x, v.y, v.z, v.w}; }
__device__ __forceinline__ void gst(float* p, float v) { *(DX_GLOBAL float*)p = v; }
__device__ __forceinline__ void gst(int64_t* p, int64_t v) { *(DX_GLOBAL int64_t*)p = v; }
__device__ __forceinline__ void gst(int32_t* p, int32_t v) { *(DX_GLOBAL int32_t*)p = v; }
__device__ __forceinline__ void gst(uint8_t* p, uint8_t v) { *(DX_GLOBAL uint8_t*)p = v; }

// min / max as the median of the two and an infinity (one v_med3_f32, no
// operand canonicalisation, unlike fminf / fmaxf): every value these kernels
// compare is a float endpoint, finite or infinite, so IEEE minNum / maxNum
// semantics are not needed; the thin filter's NaN markers only reach columns
// whose result is discarded, and it detects them by its own test.
__device__ __forceinline__ float mn(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, -DX_INF); }
__device__ __forceinline__ float mx(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, DX_INF); }

// Per-column view used by the algorithms: one shape's fields plus the
// shared buffers.
struct OpParams {
    int32_t nx, ny;
    int64_t ncols;
    const int64_t* col_ptr;
    const float2* z;
    int32_t erode;
    int32_t R;
    int32_t d2max;
    const float* H;
    WsHeader* hdr;
    int64_t cap;
    const float* gap;
    const float4* ends;
    int64_t* offA; int32_t* cntA; float2* A;
    int64_t* offI; int32_t* cntI; float2* I;
    int64_t* offB; int32_t* cntB; int32_t* loB; float2* B; uint8_t* tagB; float4* hullB;
    int64_t* offC; int32_t* cntC; float2* C;
    float2* arena;
    uint8_t* arena_tag;
    int32_t slot;  // seed slot entries per column
};

constexpr int WG = 64;
// Replay kernels: overflow entry i goes to block i % FALLBACK_BLOCKS, so the
// (typically heavy) replayed columns are spread over many waves instead of
// being packed 64 to a wave and run in lockstep.
constexpr int FALLBACK_BLOCKS = 1024;
// The wide gap cut's columns (one wave each, little LDS) are spread over more
// blocks: at the grid's x border a closing has thousands of them.
constexpr int GAPW_BLOCKS = 8192;
// K2 defers a column to its replay kernel when I(c) has more intervals than
// this, K3 when V0(c) has; CAP_Z is the per-lane list capacity of the z-slab
// replays.
constexpr int K2_DEFER_NI = 16;
// Entries (float2) after the seeds of a replayed column: slab range and the
// per-slab offsets of both groups (2 x 65 int32).
constexpr int SEED_META = 1 + 65;
constexpr int K3_DEFER_N = 16;
constexpr int CAP_MID = 48;  // LDS list capacity of the one-lane-per-column replays of K1b and K3
// LDS list capacity of K1's lane replay: 40 entries hold the partial unions
// of the columns it gets as a rule (20-40 intervals on lattice-like input)
// while letting eight of its waves share a CU (48 entries: six).
constexpr int K1_FB_CAP = 40;
constexpr int CAP_Z = 32;

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Per-lane interval list: element i at p[i * S].  S = WG: a lane's list in
// LDS, interleaved by lane; S = 1: a contiguous list in global memory (replay
// kernels).  The stride is a compile-time constant, so list indexing is a
// shift of a 32-bit index.
template <int S>
struct LV {
    float2* p;
    int cap;
    __device__ __forceinline__ float2 get(int i) const { return p[i * S]; }
    __device__ __forceinline__ void set(int i, float2 v) const { p[i * S] = v; }
};

__device__ __forceinline__ void set_error(WsHeader* h, int code) {
    atomicCAS(&h->status, 0, code);
    atomicExch(&h->abort, 1);
}

__device__ __forceinline__ void note_need(WsHeader* h, unsigned long long need) {
    atomicMax(&h->need_cap, need);
}

// k-th interval of a column (complemented for erosion, E: closed gaps).  The
// column walks are instantiated for both cases, so that the choice is made
// once per call rather than at every item.
template <bool E>
__device__ __forceinline__ float2 col_item(const float2* z, int64_t b, int n, int k) {
    if (!E) return gld(&z[b + k]);
    float lo = (k == 0) ? -DX_INF : gld(&z[b + k - 1]).y;
    float hi = (k == n) ? DX_INF : gld(&z[b + k]).x;
    return make_float2(lo, hi);
}

// First index i in [0, n) of a canonical list with U[i].y >= v (n if none).
template <class L>
__device__ __forceinline__ int lv_lower_hi(const L& U, int n, float v) {
    int l = 0, h = n;
    while (l < h) {
        int m = (l + h) >> 1;
        if (U.get(m).y < v) l = m + 1; else h = m;
    }
    return l;
}

// Insert the closed interval [lo, hi] into a canonical list of size n.
// Returns the new size, or -1 if the list would exceed its capacity (the list
// is unchanged then).
template <class L>
__device__ int lv_insert(const L& U, int n, float lo, float hi) {
    int i = lv_lower_hi(U, n, lo);
    if (i == n || U.get(i).x > hi) {
        if (n >= U.cap) return -1;
        for (int k = n; k > i; --k) U.set(k, U.get(k - 1));
        U.set(i, make_float2(lo, hi));
        return n + 1;
    }
    float2 ui = U.get(i);
    if (ui.x <= lo && hi <= ui.y) return n;
    // U[i] overlaps or touches; find the last j with U[j].x <= hi
    int l = i + 1, h = n;
    while (l < h) {
        int m = (l + h) >> 1;
        if (U.get(m).x <= hi) l = m + 1; else h = m;
    }
    int j = l - 1;
    float nlo = mn(lo, ui.x);
    float nhi = mx(hi, U.get(j).y);
    U.set(i, make_float2(nlo, nhi));
    int sh = j - i;
    if (sh > 0)
        for (int k = j + 1; k < n; ++k) U.set(k - sh, U.get(k));
    return n - sh;
}

// lv_insert for candidates arriving in non-decreasing order of start: the
// insertion point is found by walking forward from *hint (the position the
// previous candidate landed at) instead of a binary search.
template <class L>
__device__ int lv_insert_fwd(const L& U, int n, float lo, float hi, int* hint) {
    int i = *hint;
    while (i < n && U.get(i).y < lo) ++i;
    *hint = i;
    if (i == n || U.get(i).x > hi) {
        if (n >= U.cap) return -1;
        for (int k = n; k > i; --k) U.set(k, U.get(k - 1));
        U.set(i, make_float2(lo, hi));
        return n + 1;
    }
    float2 ui = U.get(i);
    if (ui.x <= lo && hi <= ui.y) return n;
    int j = i;
    while (j + 1 < n && U.get(j + 1).x <= hi) ++j;
    U.set(i, make_float2(mn(lo, ui.x), mx(hi, U.get(j).y)));
    int sh = j - i;
    if (sh > 0)
        for (int k = j + 1; k < n; ++k) U.set(k - sh, U.get(k));
    return n - sh;
}

// Is [lo, hi] inside one interval of the canonical list L[0..n)?
template <class Ptr>
__device__ __forceinline__ bool in_list(Ptr L, int n, float lo, float hi) {
    int l = 0, h = n;
    while (l < h) {
        int m = (l + h) >> 1;
        if (L[m].y < hi) l = m + 1; else h = m;
    }
    return l < n && L[l].x <= lo;
}

__device__ __forceinline__ int wave_excl_scan(int v, int* total) {
    int lane = threadIdx.x & 63;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    *total = __shfl(x, 63, 64);
    return x - v;
}

// Column id -> (x, y).
__device__ __forceinline__ void col_xy(const OpParams& P, int64_t c, int* x, int* y) {
    *y = (int)(c / P.nx);
    *x = (int)(c - (int64_t)(*y) * P.nx);
}

// Number of (possibly complemented) intervals of input column cc.
__device__ __forceinline__ int col_len(const OpParams& P, int64_t cc, int64_t* b) {
    *b = gld(&P.col_ptr[cc]);
    return (int)(gld(&P.col_ptr[cc + 1]) - *b);
}

// ---------------------------------------------------------------------------
// per-column computations (same code for LDS and global lists)
// ---------------------------------------------------------------------------
//
// Lanes of a wave run these loops in lockstep, so every loop body that
// inserts into a list has a single call site: a lane's candidates of one
// input column are enumerated as one index sequence, whatever the reason a
// candidate was selected.

// Merge the chords [item.x - h, item.y + h] of items [0, cnt) of one input
// column into the canonical list U of size n (chords and U both sorted by
// start).  U is first moved to the top of its buffer and the merged list is
// written from the bottom; a write may take the slot of an entry already
// read (or held in a register), never one still to be read.  Returns the new
// size, or -1 if the merged list would overtake the unread entries or exceed
// the capacity.
//
// Every step consumes exactly one chord (the U entries that start first are
// taken in an inner loop), so the column's items are kept in a ring of
// AHEAD registers: the item consumed by a step is replaced at once by the
// load of the item AHEAD steps later, so every load has AHEAD steps to
// arrive.  Loads past the end of the column are clamped to its last item and
// never used.
template <bool E, int AHEAD, class L>
__device__ int merge_column(const OpParams& P, const L& U, int n, int64_t b, int m, int cnt, float h) {
    const int top = U.cap - n, last = U.cap - 1;
    for (int i = n - 1; i >= 0; --i) U.set(top + i, U.get(i));
    // the caller guarantees m >= 1 (a complemented empty column is the one
    // chord (-inf, inf), never merged)
    const float2* zc = P.z + b;
    auto raw = [&](int j) { return gld(&zc[min(j, m - 1)]); };
    float2 ring[AHEAD];
#pragma unroll
    for (int q = 0; q < AHEAD; ++q) ring[q] = raw(q);
    float2 u0 = U.get(min(top, last));  // next unread entry of U
    float prevy = -DX_INF;              // E: end of the previous item
    float2 cur = make_float2(0.f, 0.f);  // the open output interval
    int i = 0, k = 0;
    // per-lane flags as integers, so that the divergent loops around push()
    // carry them in vector registers instead of merging lane masks at every
    // branch; push() itself runs without a branch but for the one store
    int open = 0, bad = 0;
    // push v if `doit`: every update is a select but the one store
    auto push_if = [&](bool doit, float2 v) {
        const int d = doit ? 1 : 0;
        const int ext = open & (v.x <= cur.y ? 1 : 0);
        const int emit = d & open & (ext ^ 1);
        const int room = (k <= top + i ? 1 : 0) & (k < U.cap ? 1 : 0);
        if (emit & room) U.set(k, cur);
        bad |= emit & (room ^ 1);
        k += emit;
        const float2 nc = ext ? make_float2(cur.x, mx(cur.y, v.y)) : v;
        cur = doit ? nc : cur;
        open |= d;
    };
    auto step = [&](const float2 it, int j) {
        const bool live = j < cnt;
        float2 c;
        if (E) {
            c = make_float2(prevy - h, (j < m ? it.x : DX_INF) + h);
            prevy = live ? it.y : prevy;
        } else {
            c = make_float2(it.x - h, it.y + h);
        }
        // the entries of U starting at or below c's start go first: one
        // predicated step (the usual case), then a loop for the rest
        const bool t1 = live && i < n && u0.x <= c.x;
        push_if(t1, u0);
        const float2 un = U.get(min(top + i + 1, last));
        i += t1 ? 1 : 0;
        u0 = t1 ? un : u0;
        while (live && i < n && u0.x <= c.x) {
            push_if(true, u0);
            ++i;
            u0 = U.get(min(top + i, last));
        }
        push_if(live, c);
    };
    for (int j = 0; j < cnt; j += AHEAD) {
#pragma unroll
        for (int q = 0; q < AHEAD; ++q) {
            const float2 it = ring[q];
            ring[q] = raw(j + q + AHEAD);
            step(it, j + q);
        }
    }
    while (i < n) {
        push_if(true, u0);
        ++i;
        u0 = U.get(min(top + i, last));
    }
    if (bad || k >= U.cap) return -1;
    U.set(k++, cur);
    return k;
}

// K1: V0 = union over |dx| <= R of the chords [a - H[dx^2], b + H[dx^2]] of
// the row's columns x + dx (the hull columns first, then the others in the
// spread order below).  Within a column the chord starts and the chord ends are both
// non-decreasing (disjoint sorted intervals, one half-width h), so:
// * if no gap of the column exceeds 2h, its chords chain into the single
//   interval [first start - h, last end + h] (rounding is monotone, so every
//   chord start stays at or below the previous chord's end in float too),
//   which is inserted alone (all such hulls first);
// * else, while the partial union is a single interval [L, E], only a
//   leading run of chords starting below L and a trailing run ending above E
//   can change it, and are inserted;
// * otherwise the column's chords are merged with the list (in an erosion,
//   a one-interval column against a union of two rays only moves the rays).
// Visit v of a row window, nearest columns first: x, x-1, x+1, x-2, x+2, ...
// (the order of the row offset's hull pass and slab replay, and of the direct
// evaluation's rows)
__device__ __forceinline__ int visit_col(int x, int v) {
    const int t = (v + 1) >> 1;
    return v == 0 ? x : ((v & 1) ? x - t : x + t);
}

// Visit order of the row offset's second pass, one offset of [-R, R] per
// call: first the centre (the widest chords), then the spread magnitudes
// t_j = round(j R / 8) in the order j = 4, 2, 6, 1, 3, 5, 7 (each magnitude
// once, as -t then +t), then the other magnitudes from 1 outwards.
// Neighbouring columns of a solid with through-channels tend to share the
// channel's gaps, so a partial union of near columns keeps every gap until a
// column far enough away fills it; columns spread over the window close
// most gaps early, and the later columns take the short single-interval
// path (on a thin-walled gyroid at r = 16, a CPU count of merge steps per
// column gave about a quarter of a centre-out order's).  The centre comes
// first because a far column's narrower chords, merged first with another
// far column's of another phase, can leave more intervals than the lane's
// list holds.
struct SpreadOrder {
    int R;
    int i = 0;    // 0: the centre next, 1 .. 7: the next spread index + 1, 8: the rest
    int t = 0;    // the current magnitude
    int r = 0;    // the last magnitude of the rest
    int pos = 0;  // +t is due next
    __host__ __device__ static int mag(int R, int k) {
        const int j = (0x7531624 >> (4 * k)) & 15;  // 4, 2, 6, 1, 3, 5, 7
        return (R * j + 4) >> 3;
    }
    __host__ __device__ bool spread(int tt) const {
        bool in = false;
        for (int k = 0; k < 7; ++k) in = in || mag(R, k) == tt;
        return in;
    }
    __host__ __device__ int next() {
        if (pos) {
            pos = 0;
            return t;
        }
        if (i == 0) {
            i = 1;
            return 0;
        }
        while (i < 8) {
            const int k = i - 1;
            const int tt = mag(R, k);
            bool dup = tt == 0;
            for (int q = 0; q < k; ++q) dup = dup || mag(R, q) == tt;
            ++i;
            if (!dup) {
                t = tt;
                pos = 1;
                return -t;
            }
        }
        for (++r; r <= R && spread(r); ++r) {
        }
        t = r;
        pos = 1;
        return -t;
    }
};

// K1_COVERED: the fold stopped because the partial union holds one interval
// containing the caller's range `cover` (see k_row_offset_fb).
constexpr int K1_COVERED = -2;

template <bool E, int AHEAD, class L>
__device__ int k1_column_e(const OpParams& P, int64_t c, const L& U, float2 cover) {
    int x, y;
    col_xy(P, c, &x, &y);
    const int64_t row = (int64_t)y * P.nx;
    int n = 0;
    // Pass 1: the columns whose gaps are all within 2h contribute their hull
    // alone, read from the column summary (coalesced across the wave, four
    // visits' summaries loaded together).  On most inputs this leaves the
    // union a single interval, so that pass 2 takes the short path for
    // nearly every column.  The union does not depend on the order its
    // chords are inserted in.
    for (int v0 = 0; v0 <= 2 * P.R; v0 += 4) {
        float gq[4], hq[4];
        float4 eq[4];
        bool iq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int v = v0 + q;
            const int xn = visit_col(x, v);
            const int t = min((v + 1) >> 1, P.R);
            iq[q] = v <= 2 * P.R && xn >= 0 && xn < P.nx;
            hq[q] = gld(&P.H[t * t]);
            gq[q] = iq[q] ? gld(&P.gap[row + xn]) : -1.f;
            eq[q] = iq[q] ? gld(&P.ends[row + xn]) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float gc = gq[q], h = hq[q];
            const bool empty = gc < 0.f;
            // an empty column has no chord, its complement the whole line;
            // a complemented column's hull is the whole line too
            if (!iq[q] || (empty && !E) || !(empty || gc <= 2.f * h)) continue;
            const float lo = E ? -DX_INF : eq[q].x - h;
            const float hi = E ? DX_INF : eq[q].w + h;
            n = lv_insert(U, n, lo, hi);
            if (n < 0) return -1;
        }
    }
    if (n == 1 && cover.x <= cover.y) {
        const float2 u = U.get(0);
        if (u.x <= cover.x && cover.y <= u.y) return K1_COVERED;
    }
    // Pass 2: the other columns, in the spread order.  Column pointers and
    // summaries of the next visit are loaded one visit ahead.
    int64_t b = 0, e = 0;
    float gp = 0.f;
    float4 en = make_float4(0.f, 0.f, 0.f, 0.f);
    SpreadOrder ord{P.R};
    int dn = ord.next();
    bool inr = x + dn >= 0 && x + dn < P.nx;
    if (inr) {
        b = gld(&P.col_ptr[row + x + dn]);
        e = gld(&P.col_ptr[row + x + dn + 1]);
        gp = gld(&P.gap[row + x + dn]);
        en = gld(&P.ends[row + x + dn]);
    }
    for (int v = 0; v <= 2 * P.R; ++v) {
        const int t = abs(dn);
        const float h = gld(&P.H[t * t]);
        const int64_t bc = b, ec = e;
        const float gc = gp;
        const float4 ec4 = en;
        const bool inc = inr;
        if (v < 2 * P.R) {
            dn = ord.next();
            const int xn = x + dn;
            inr = xn >= 0 && xn < P.nx;
            if (inr) {
                b = gld(&P.col_ptr[row + xn]);
                e = gld(&P.col_ptr[row + xn + 1]);
                gp = gld(&P.gap[row + xn]);
                en = gld(&P.ends[row + xn]);
            }
        }
        if (!inc) continue;
        const int m = (int)(ec - bc);
        const int cnt = E ? m + 1 : m;
        // empty columns and hulls were handled in pass 1
        if (m == 0 || gc <= 2.f * h) continue;
        // erosion of a one-interval column [a, b]: its complement is the two
        // rays (-inf, a] and [b, +inf); while the partial union is two rays
        // too, the chords (-inf, a + h] and [b - h, +inf) only move the rays'
        // ends, and the rays merge into the whole line once they meet
        if (E && m == 1 && n == 2) {
            const float2 u0 = U.get(0), u1 = U.get(1);
            if (u0.x == -DX_INF && u1.y == DX_INF) {
                const float lo = mx(u0.y, ec4.x + h), hi = mn(u1.x, ec4.w - h);
                if (hi <= lo) {
                    U.set(0, make_float2(-DX_INF, DX_INF));
                    n = 1;
                } else {
                    U.set(0, make_float2(-DX_INF, lo));
                    U.set(1, make_float2(hi, DX_INF));
                }
                continue;
            }
        }
        if (n != 1) {
            n = merge_column<E, AHEAD>(P, U, n, bc, m, cnt, h);
            if (n < 0) return -1;
            continue;
        }
        // the first and last items, from the column summary
        float2 f, l;
        if (E) {
            f = make_float2(-DX_INF, ec4.x);
            l = make_float2(ec4.w, DX_INF);
        } else {
            f = make_float2(ec4.x, ec4.y);
            l = make_float2(ec4.z, ec4.w);
        }
        // The runs are found and inserted with the items loaded four at a
        // time (independent loads, clamped to the column), so a visit waits
        // for memory about once per run instead of once per item.
        const float2 u = U.get(0);
        if (cover.x <= cover.y && u.x <= cover.x && cover.y <= u.y) return K1_COVERED;
        int k0 = 0, k1 = cnt;
        if (f.x - h < u.x) {
            k0 = 1;
            for (bool more = true; more && k0 < cnt;) {
                float2 q[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) q[i] = col_item<E>(P.z, bc, m, min(k0 + i, cnt - 1));
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (more && k0 < cnt && q[i].x - h < u.x) ++k0;
                    else more = false;
                }
            }
        }
        if (k1 > k0 && l.y + h > u.y) {
            k1 = cnt - 1;
            for (bool more = true; more && k1 > k0;) {
                float2 q[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) q[i] = col_item<E>(P.z, bc, m, max(k1 - 1 - i, 0));
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (more && k1 > k0 && q[i].y + h > u.y) --k1;
                    else more = false;
                }
            }
        }
        // candidates: items [0, k0) then [k1, cnt), inserted in that order
        const int nc = k0 + (cnt - k1);
        int hint = 0;
        for (int j = 0; j < nc; j += 4) {
            float2 q[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int jj = min(j + i, nc - 1);
                q[i] = col_item<E>(P.z, bc, m, jj < k0 ? jj : k1 + (jj - k0));
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (j + i < nc) {
                    n = lv_insert_fwd(U, n, q[i].x - h, q[i].y + h, &hint);
                    if (n < 0) return -1;
                }
            }
        }
    }
    return n;
}

constexpr int MERGE_AHEAD = 8;

// `cover` (lo <= hi) lets the fold stop with K1_COVERED once the partial
// union holds one interval containing [lo, hi]; (+inf, -inf) never stops it.
template <int AHEAD = MERGE_AHEAD, class L>
__device__ int k1_column(const OpParams& P, int64_t c, const L& U,
                         float2 cover = make_float2(DX_INF, -DX_INF)) {
    return P.erode ? k1_column_e<true, AHEAD>(P, c, U, cover) : k1_column_e<false, AHEAD>(P, c, U, cover);
}

__device__ int64_t k1_bound(const OpParams& P, int64_t c) {
    int x, y;
    col_xy(P, c, &x, &y);
    const int64_t row = (int64_t)y * P.nx;
    int x0 = max(0, x - P.R), x1 = min(P.nx - 1, x + P.R);
    return (P.col_ptr[row + x1 + 1] - P.col_ptr[row + x0]) + (int64_t)(x1 - x0 + 1) + 1;
}

// K1b: I = intersection of V0 over the in-grid rows y+-1 .. y+-R (the whole
// line if there are none).  Two lists, result in *res (0 or 1).
template <class L>
__device__ int k1b_column(const OpParams& P, int64_t c, const L& L0, const L& L1, int* res) {
    int x, y;
    col_xy(P, c, &x, &y);
    L0.set(0, make_float2(-DX_INF, DX_INF));
    int n = 1, cur = 0;
    // the list of the next row (y - dy, then y + dy, dy = 1 .. R) is located
    // one row ahead
    int64_t noff = 0;
    int ncnt = -1;
    auto fetch = [&](int q) {  // row q = 2 (dy - 1) + s
        const int yy = (q & 1) ? y + (q >> 1) + 1 : y - (q >> 1) - 1;
        const bool in = yy >= 0 && yy < P.ny;
        const int64_t cc = (int64_t)(in ? yy : y) * P.nx + x;
        noff = in ? gld(&P.offA[cc]) : 0;
        ncnt = in ? gld(&P.cntA[cc]) : -1;
    };
    if (P.R >= 1) fetch(0);
    for (int dy = 1; dy <= P.R && n > 0; ++dy) {
        for (int s = 0; s < 2 && n > 0; ++s) {
            const int q = 2 * (dy - 1) + s;
            const int64_t off = noff;
            const int m = ncnt;
            if (q + 1 < 2 * P.R) fetch(q + 1);
            if (m < 0) continue;  // row outside the grid
            const float2* J = P.A + off;
            const L& S = cur ? L1 : L0;
            const L& D = cur ? L0 : L1;
            int i = 0, j = 0, k = 0;
            while (i < n && j < m) {
                float2 a = S.get(i), bb = gld(&J[j]);
                float lo = mx(a.x, bb.x), hi = mn(a.y, bb.y);
                if (lo < hi) {
                    if (k >= D.cap) return -1;
                    D.set(k++, make_float2(lo, hi));
                }
                if (a.y < bb.y) ++i; else ++j;
            }
            n = k;
            cur ^= 1;
        }
    }
    *res = cur;
    return n;
}

__device__ int64_t k1b_bound(const OpParams& P, int64_t c) {
    int x, y;
    col_xy(P, c, &x, &y);
    int64_t b = 2;
    for (int dy = 1; dy <= P.R; ++dy)
        for (int s = 0; s < 2; ++s) {
            const int yy = s ? y + dy : y - dy;
            if (yy < 0 || yy >= P.ny) continue;
            b += gld(&P.cntA[(int64_t)yy * P.nx + x]);
        }
    return b;
}

// K2: closest-parent extrusion pieces of row y at column x (tags t = |dx|),
// painted in order of t: the pieces of tag t are the parts of the columns
// x-t and x+t not covered by the columns nearer to x.  Only pieces whose
// chord at |dy| = 1 pokes out of I(c) are kept.  A column whose whole chord
// is inside I(c) is not added to the cover list, and the cover list simply
// stops growing when its capacity is reached: either way the pieces it would
// hide are then kept whole, which adds valid seeds and changes nothing in
// the result.  The kept pieces go to a SeedSink in two groups, below and at
// or above a split height taken from the middle of I(c): a seed group lies
// near one end of the union it can change, and its hulls let the y union
// skip it whole.

// Is [lo, hi] inside I(c)?  A one-interval I is tested from registers.
template <class Ptr>
__device__ __forceinline__ bool in_I(Ptr Ip, int ni, float2 i0, float lo, float hi) {
    if (ni == 1) return i0.x <= lo && hi <= i0.y;
    return in_list(Ip, ni, lo, hi);
}

// Destination of one column's kept pieces.  Group 0: pieces whose centre is
// below zsplit; group 1: the others.  Slot mode (cap > 0): group 0 fills dlo
// upwards and group 1 fills dhi downwards, both within cap entries in total.
// Linear mode (cap == 0): each group fills its own region upwards within
// cap_lo / cap_hi entries.  Hulls per group: x, y of the chords at |dy| = 1,
// z, w of the pieces.  In slot mode the 1-byte tags are collected in wlo /
// whi and stored as whole aligned dwords (the slot's tags are 32-byte
// aligned), the last partial dword of each group by sink_flush.
struct SeedSink {
    float2* dlo;
    uint8_t* tlo;
    float2* dhi;
    uint8_t* thi;
    int cap, cap_lo, cap_hi;
    float zsplit;
    int nlo, nhi;
    float4 hlo, hhi;
    uint32_t wlo, whi;
};

__device__ __forceinline__ SeedSink sink_make(float2* dlo, uint8_t* tlo, float2* dhi, uint8_t* thi,
                                              int cap, int cap_lo, int cap_hi, float zsplit) {
    SeedSink o;
    o.dlo = dlo;
    o.tlo = tlo;
    o.dhi = dhi;
    o.thi = thi;
    o.cap = cap;
    o.cap_lo = cap_lo;
    o.cap_hi = cap_hi;
    o.zsplit = zsplit;
    o.nlo = o.nhi = 0;
    o.hlo = o.hhi = make_float4(DX_INF, -DX_INF, DX_INF, -DX_INF);
    o.wlo = o.whi = 0;
    return o;
}

__device__ __forceinline__ void hull_add(float4* h, float p, float q, float h1) {
    h->x = mn(h->x, p - h1);
    h->y = mx(h->y, q + h1);
    h->z = mn(h->z, p);
    h->w = mx(h->w, q);
}

__device__ __forceinline__ void k2_emit(float p, float q, float h1, int t, SeedSink& o) {
    const bool hi = !(0.5f * p + 0.5f * q < o.zsplit);
    const float2 v = make_float2(p, q);
    if (o.cap > 0) {
        if (o.nlo + o.nhi < o.cap) {
            if (hi) {
                // group 1 entry k is byte 3 - k % 4 of the dword ending at thi - (k & ~3)
                gst(&o.dhi[-o.nhi], v);
                o.whi |= (uint32_t)t << (8 * (3 - (o.nhi & 3)));
                if ((o.nhi & 3) == 3) {
                    gst((int32_t*)(o.thi - o.nhi), (int32_t)o.whi);
                    o.whi = 0;
                }
            } else {
                gst(&o.dlo[o.nlo], v);
                o.wlo |= (uint32_t)t << (8 * (o.nlo & 3));
                if ((o.nlo & 3) == 3) {
                    gst((int32_t*)(o.tlo + o.nlo - 3), (int32_t)o.wlo);
                    o.wlo = 0;
                }
            }
        }
    } else if (hi) {
        if (o.nhi < o.cap_hi) {
            gst(&o.dhi[o.nhi], v);
            gst(&o.thi[o.nhi], (uint8_t)t);
        }
    } else if (o.nlo < o.cap_lo) {
        gst(&o.dlo[o.nlo], v);
        gst(&o.tlo[o.nlo], (uint8_t)t);
    }
    if (hi) {
        hull_add(&o.hhi, p, q, h1);
        ++o.nhi;
    } else {
        hull_add(&o.hlo, p, q, h1);
        ++o.nlo;
    }
}

// Slot mode: store the tags of each group's last partial dword, byte by byte
// (the two groups may share that dword).  A column with more pieces than the
// slot is recomputed into the arena, so its slot tags are not needed.
__device__ __forceinline__ void sink_flush(SeedSink& o) {
    if (o.cap <= 0 || o.nlo + o.nhi > o.cap) return;
    for (int i = o.nlo & ~3; i < o.nlo; ++i) gst(&o.tlo[i], (uint8_t)(o.wlo >> (8 * (i & 3))));
    for (int i = o.nhi & ~3; i < o.nhi; ++i) gst(&o.thi[-i], (uint8_t)(o.whi >> (8 * (3 - (i & 3)))));
}

// Split height of column c: the middle of the finite extent of I(c) (0 if
// I(c) has no finite endpoint).
__device__ __forceinline__ float seed_split(const OpParams& P, int64_t c) {
    const int ni = gld(&P.cntI[c]);
    if (ni == 0) return 0.0f;
    const float2* Ip = P.I + gld(&P.offI[c]);
    const float2 a = gld(&Ip[0]), b = gld(&Ip[ni - 1]);
    const float lo = (a.x > -DX_INF) ? a.x : a.y;
    const float hi = (b.y < DX_INF) ? b.y : b.x;
    if (!(lo > -DX_INF && lo < DX_INF && hi > -DX_INF && hi < DX_INF)) return 0.0f;
    return 0.5f * lo + 0.5f * hi;
}

template <class Ptr, class L>
__device__ __forceinline__ void k2_segment(Ptr Ip, int ni, float2 i0, const L& U, int* n,
                                           float a, float e, float h1, int t, SeedSink& o) {
    if (in_I(Ip, ni, i0, a - h1, e + h1)) return;
    // parts of [a, e] not covered by U (closures): one candidate piece per
    // step, [p, q], ending at the next cover interval or at e
    int idx = lv_lower_hi(U, *n, a);
    float p = a;
    bool more = true;
    while (more) {
        float q = e, pn = p;
        bool cand;
        if (idx < *n) {
            const float2 u = U.get(idx);
            if (u.x > e) {
                cand = p < e || a == e;
                more = false;
            } else {
                q = u.x;
                cand = u.x > p;
                more = u.y < e;
                pn = mx(p, u.y);
                ++idx;
            }
        } else {
            cand = p < e || a == e;
            more = false;
        }
        if (cand && !in_I(Ip, ni, i0, p - h1, q + h1)) k2_emit(p, q, h1, t, o);
        p = pn;
    }
    const int nn = lv_insert(U, *n, a, e);
    if (nn >= 0) *n = nn;
}

template <bool E, class L>
__device__ int k2_column_e(const OpParams& P, int64_t c, const L& U, SeedSink& o) {
    int x, y;
    col_xy(P, c, &x, &y);
    const int64_t row = (int64_t)y * P.nx;
    const float2* Ip = P.I + gld(&P.offI[c]);
    const int ni = gld(&P.cntI[c]);
    float2 i0 = make_float2(0.f, 0.f);
    if (ni == 1) i0 = gld(&Ip[0]);
    const float ilo = ni > 0 ? (ni == 1 ? i0.x : gld(&Ip[0]).x) : 0.f;
    const float ihi = ni > 0 ? (ni == 1 ? i0.y : gld(&Ip[ni - 1]).y) : 0.f;
    int n = 0;
    // visits up to |dx| = tmax (the chord at |dy| = 1 must exist)
    int tmax = P.R;
    while (tmax >= 0 && tmax * tmax + 1 > P.d2max) --tmax;
    // column pointers of the next visit are loaded one visit ahead
    int64_t b = 0, e = 0;
    float4 en = make_float4(0.f, 0.f, 0.f, 0.f);
    bool inr = tmax >= 0;
    if (inr) {
        b = gld(&P.col_ptr[row + x]);
        e = gld(&P.col_ptr[row + x + 1]);
        en = gld(&P.ends[row + x]);
    }
    for (int v = 0; v <= 2 * tmax; ++v) {
        const int t = (v + 1) >> 1;
        const float h1 = gld(&P.H[t * t + 1]);
        const int64_t bc = b, ec = e;
        const float4 ec4 = en;
        const bool inc = inr;
        if (v < 2 * tmax) {
            const int xn = visit_col(x, v + 1);
            inr = xn >= 0 && xn < P.nx;
            if (inr) {
                b = gld(&P.col_ptr[row + xn]);
                e = gld(&P.col_ptr[row + xn + 1]);
                en = gld(&P.ends[row + xn]);
            }
        }
        if (!inc) continue;
        const int m = (int)(ec - bc);
        const int cnt = E ? m + 1 : m;
        if (cnt == 0) continue;
        // the first and last items, from the column summary
        float2 f, l;
        if (E) {
            f = make_float2(-DX_INF, m > 0 ? ec4.x : DX_INF);
            l = make_float2(m > 0 ? ec4.w : -DX_INF, DX_INF);
        } else {
            f = make_float2(ec4.x, ec4.y);
            l = make_float2(ec4.z, ec4.w);
        }
        auto item = [&](int k) {
            return k == 0 ? f : (k == cnt - 1 ? l : col_item<E>(P.z, bc, m, k));
        };
        // Chords that can poke out of I form one run per gap of I (the two
        // unbounded ends included), because a column's chord starts and
        // chord ends are both non-decreasing.  Short columns, and columns
        // tested against an empty I, are one run.
        const bool all = ni == 0 || cnt <= 8;
        const int nruns = all ? 1 : ni + 1;
        int next = 0;
        for (int g = 0; g < nruns; ++g) {
            int kb = 0;
            float lim = DX_INF;  // the run ends at the first chord starting at or above lim
            if (!all) {
                if (g == 0) {
                    lim = ilo;
                } else if (g == ni) {
                    kb = cnt;
                    while (kb > next && item(kb - 1).y + h1 > ihi) --kb;
                } else {  // gap (I[g-1].y, I[g].x): first chord ending above its start
                    const float glo = gld(&Ip[g - 1]).y;
                    lim = gld(&Ip[g]).x;
                    int lo = next, hh = cnt;
                    while (lo < hh) {
                        const int mid = (lo + hh) >> 1;
                        if (item(mid).y + h1 > glo) hh = mid; else lo = mid + 1;
                    }
                    kb = lo;
                }
            }
            int k = kb;
            for (; k < cnt; ++k) {
                const float2 sg = item(k);
                if (!(sg.x - h1 < lim)) break;
                k2_segment(Ip, ni, i0, U, &n, sg.x, sg.y, h1, t, o);
            }
            next = max(next, k);
        }
    }
    return o.nlo + o.nhi;
}

template <class L>
__device__ int k2_column(const OpParams& P, int64_t c, const L& U, SeedSink& o) {
    return P.erode ? k2_column_e<true>(P, c, U, o) : k2_column_e<false>(P, c, U, o);
}

// K3: V0(c) plus the chords of the kept seeds of rows y+-dy at weight
// r^2 - t^2 - dy^2, nearest rows first.  TAB: the wave's lanes (all of
// them, one shape per wave) first stage the half-widths of the current dy
// for every tag in the LDS table `tab` (negative: outside the ball); the
// per-lane work then looks up tab[t].  Without TAB the lookups read H.
// A lane stops adding chords when its list overflows (result -1) but keeps
// taking part in the staging.
// Size of the low seed group from loB: a column whose seeds the slab replay
// wrote (ordered by slab, with the slab index after them) stores ~size.
__device__ __forceinline__ int seed_lo(int v) { return v < 0 ? ~v : v; }

// The two seed groups of column cc (see SeedSink): group g has n[g] seeds at
// s[g], tags at t[g].  Slot columns hold group 0 at the slot's start and
// group 1 at its end; arena columns (offset -(pos + 1)) hold group 0 then
// group 1.
struct SeedSpans {
    const float2* s[2];
    const uint8_t* t[2];
    int n[2];
};

// Tags p[0..3] of a seed tag array, from the two aligned dwords holding them
// (bits 8q .. 8q+7 of the result are tag q).  The two dwords may cover up to
// 7 bytes around the four tags: every tag array lies inside the workspace,
// 256-byte aligned and followed by another region, so the reads stay in it;
// tags past a group's end are never used.
__device__ __forceinline__ uint64_t tags4(const uint8_t* p) {
    const uintptr_t a = (uintptr_t)p & ~(uintptr_t)3;
    const uint32_t w0 = (uint32_t)gld((const int32_t*)a), w1 = (uint32_t)gld((const int32_t*)(a + 4));
    return ((((uint64_t)w1) << 32) | w0) >> (8 * ((uintptr_t)p & 3));
}

// From the column's seed offset, count and (encoded) low-group size.
__device__ __forceinline__ SeedSpans seed_spans_of(const OpParams& P, int64_t ob, int cnt, int lov) {
    SeedSpans r;
    const int lo = seed_lo(lov);
    if (ob >= 0) {
        r.n[0] = min(lo, P.slot);
        r.n[1] = min(cnt - lo, P.slot - r.n[0]);
        r.s[0] = P.B + ob;
        r.t[0] = P.tagB + ob;
        r.s[1] = P.B + ob + P.slot - r.n[1];
        r.t[1] = P.tagB + ob + P.slot - r.n[1];
    } else {
        const int64_t a = -ob - 1;
        r.n[0] = lo;
        r.n[1] = cnt - lo;
        r.s[0] = P.arena + a;
        r.t[0] = P.arena_tag + a;
        r.s[1] = P.arena + a + lo;
        r.t[1] = P.arena_tag + a + lo;
    }
    return r;
}

__device__ __forceinline__ SeedSpans seed_spans(const OpParams& P, int64_t cc) {
    return seed_spans_of(P, gld(&P.offB[cc]), gld(&P.cntB[cc]), gld(&P.loB[cc]));
}

template <bool TAB, class L>
__device__ int k3_column(const OpParams& P, int64_t c, bool live, const L& U, float* tab) {
    int x = 0, y = 0;
    if (live) col_xy(P, c, &x, &y);
    int n = 0;
    // a per-lane flag as an integer: the divergent insert branches carry it
    // in a vector register instead of merging lane masks
    int ok = live ? 1 : 0;
    if (ok) {
        const int n0 = gld(&P.cntA[c]);
        if (n0 > U.cap) {
            ok = 0;
        } else {
            const float2* V = P.A + gld(&P.offA[c]);
            for (int i = 0; i < n0; ++i) U.set(i, gld(&V[i]));
            n = n0;
        }
    }
    // While the union has one or two intervals (a solid, or the complement
    // of one in an erosion), keep them in registers: most seed chords land
    // inside one and are dropped after a few compares.
    float2 u0 = make_float2(0.f, 0.f), u1 = make_float2(0.f, 0.f);
    if (ok && n >= 1 && n <= 2) {
        u0 = U.get(0);
        if (n == 2) u1 = U.get(1);
    }
    for (int dy = 1; dy <= P.R; ++dy) {
        const int dy2 = dy * dy;
        if (TAB) {
            __syncthreads();
            for (int t = threadIdx.x; t <= P.R; t += WG) {
                const int d2 = t * t + dy2;
                tab[t] = d2 <= P.d2max ? gld(&P.H[d2]) : -1.0f;
            }
            __syncthreads();
        }
        if (!ok) continue;
        const float hd = gld(&P.H[dy2]);
        // the hulls of both seed groups of both seed rows are loaded together
        const int64_t cl = (int64_t)(y - dy) * P.nx + x, cr = (int64_t)(y + dy) * P.nx + x;
        const float4 none = make_float4(DX_INF, -DX_INF, DX_INF, -DX_INF);
        float4 hq[4];
        hq[0] = y - dy >= 0 ? gld(&P.hullB[2 * cl]) : none;
        hq[1] = y - dy >= 0 ? gld(&P.hullB[2 * cl + 1]) : none;
        hq[2] = y + dy < P.ny ? gld(&P.hullB[2 * cr]) : none;
        hq[3] = y + dy < P.ny ? gld(&P.hullB[2 * cr + 1]) : none;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!ok) break;
            const float4 h4 = hq[k];
            // Every chord of this seed group at this dy lies inside its hull
            // at |dy| = 1 and inside its piece hull widened by H[dy^2] (the
            // widest half-width at this dy); skip the group when the tighter
            // of the two bounds is inside the union.
            if (h4.x > h4.y) continue;
            const float hlo = mx(h4.x, h4.z - hd), hhi = mn(h4.y, h4.w + hd);
            if (n <= 2) {
                if (n >= 1 && u0.x <= hlo && hhi <= u0.y) continue;
                if (n == 2 && u1.x <= hlo && hhi <= u1.y) continue;
            } else {
                const int i = lv_lower_hi(U, n, hhi);
                if (i < n && U.get(i).x <= hlo) continue;
            }
            const SeedSpans sp = seed_spans(P, (k >> 1) ? cr : cl);
            const float2* sv = sp.s[k & 1];
            const uint8_t* tv = sp.t[k & 1];
            const int nb = sp.n[k & 1];
            // seeds in groups of four: the loads of a group are in flight
            // together, its four tags in two dword loads
            for (int j = 0; j < nb && ok; j += 4) {
                int tq[4];
                float2 pq[4];
                const uint64_t tw = tags4(tv + j);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    tq[q] = (int)((tw >> (8 * q)) & 0xff);
                    pq[q] = gld(&sv[min(j + q, nb - 1)]);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // one branch per seed: most chords are inside the union
                    const int t = tq[q];
                    float h;
                    if (TAB) {
                        h = tab[t];
                    } else {
                        const int d2 = t * t + dy2;
                        h = d2 <= P.d2max ? gld(&P.H[d2]) : -1.0f;
                    }
                    const float lo = pq[q].x - h, hi = pq[q].y + h;
                    const bool inside = (n >= 1 && n <= 2 && u0.x <= lo && hi <= u0.y) ||
                                        (n == 2 && u1.x <= lo && hi <= u1.y);
                    if (ok && j + q < nb && h >= 0.0f && !inside) {
                        n = lv_insert(U, n, lo, hi);
                        if (n < 0) {
                            ok = 0;
                            n = 0;
                        } else if (n <= 2) {
                            u0 = U.get(0);
                            if (n == 2) u1 = U.get(1);
                        }
                    }
                }
            }
        }
    }
    if (!live) return 0;
    return ok ? n : -1;
}

__device__ int64_t k3_bound(const OpParams& P, int64_t c) {
    int x, y;
    col_xy(P, c, &x, &y);
    int64_t b = (int64_t)gld(&P.cntA[c]) + 1;
    for (int dy = 1; dy <= P.R; ++dy)
        for (int s = 0; s < 2; ++s) {
            const int yy = s ? y + dy : y - dy;
            if (yy < 0 || yy >= P.ny) continue;
            b += gld(&P.cntB[(int64_t)yy * P.nx + x]);
        }
    return b;
}

// ---------------------------------------------------------------------------
// z-slab evaluation of one heavy column by a whole wave
// ---------------------------------------------------------------------------
//
// A column whose lists are long (typically at the grid's x border, where the
// one-sided row window leaves many gaps) is evaluated by all 64 lanes of a
// wave: lane l restricts the computation to the closed slab [b_l, b_l+1] of
// z, with b_0 = -inf, b_64 = +inf and b_1 .. b_63 evenly spaced over the
// finite range of the data.  Restricting to a slab commutes with the union
// (clip every candidate to the slab), and two parts of one interval cut at
// a slab boundary overlap there, so the slab results concatenate to the same
// float union once intervals touching at a boundary are merged.

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = mn(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = mx(v, __shfl_xor(v, d, 64));
    return v;
}

// Slab of this lane for data spanning [zmin, zmax] (zmin > zmax: no finite data).
// Boundary b_k (k = 0 .. 64) of the slabs over [zmin, zmax] (already
// normalised: zmin <= zmax).
__device__ __forceinline__ float slab_bound(float zmin, float zmax, int k) {
    if (k <= 0) return -DX_INF;
    if (k >= 64) return DX_INF;
    return zmin + (zmax - zmin) * ((float)k * (1.0f / 64.0f));
}

__device__ __forceinline__ float2 slab_range(float zmin, float zmax) {
    if (!(zmin <= zmax)) zmin = zmax = 0.0f;
    return make_float2(zmin, zmax);
}

__device__ __forceinline__ float2 lane_slab(float zmin, float zmax) {
    const int l = threadIdx.x & 63;
    const float2 r = slab_range(zmin, zmax);
    return make_float2(slab_bound(r.x, r.y, l), slab_bound(r.x, r.y, l + 1));
}

__device__ __forceinline__ void widen(float* zmin, float* zmax, float v) {
    if (v > -DX_INF && v < DX_INF) {
        *zmin = mn(*zmin, v);
        *zmax = mx(*zmax, v);
    }
}

// K1b restricted to the slab [zs, ze]: starts from the slab itself and
// intersects it with V0 of the rows y+-1 .. y+-R, visiting only the V0
// intervals that reach the slab.  Two lists, result in *res.
template <class L>
__device__ int k1b_slab(const OpParams& P, int64_t c, float zs, float ze, const L& L0, const L& L1,
                        int* res) {
    int x, y;
    col_xy(P, c, &x, &y);
    L0.set(0, make_float2(zs, ze));
    int n = 1, cur = 0;
    for (int dy = 1; dy <= P.R && n > 0; ++dy) {
        for (int s = 0; s < 2 && n > 0; ++s) {
            const int yy = s ? y + dy : y - dy;
            if (yy < 0 || yy >= P.ny) continue;
            const int64_t cc = (int64_t)yy * P.nx + x;
            const float2* J = P.A + gld(&P.offA[cc]);
            const int m = gld(&P.cntA[cc]);
            int j = 0, hh = m;  // first V0 interval ending at or above zs
            while (j < hh) {
                const int mid = (j + hh) >> 1;
                if (gld(&J[mid]).y < zs) j = mid + 1; else hh = mid;
            }
            const L& S = cur ? L1 : L0;
            const L& D = cur ? L0 : L1;
            int i = 0, k = 0;
            while (i < n && j < m) {
                const float2 a = S.get(i), bb = gld(&J[j]);
                if (bb.x > ze) break;
                const float lo = mx(a.x, bb.x), hi = mn(a.y, bb.y);
                if (lo < hi) {
                    if (k >= D.cap) return -1;
                    D.set(k++, make_float2(lo, hi));
                }
                if (a.y < bb.y) ++i; else ++j;
            }
            n = k;
            cur ^= 1;
        }
    }
    *res = cur;
    return n;
}

// K1 restricted to the slab [zs, ze]: the chords of the row window clipped to
// the slab, nearest columns first; only the chords from the first one ending
// at or above zs to the last one starting at or below ze are visited, and the
// lane stops once its slab is covered whole.
template <bool E, class L>
__device__ int k1_slab_e(const OpParams& P, int64_t c, float zs, float ze, const L& U) {
    int x, y;
    col_xy(P, c, &x, &y);
    const int64_t row = (int64_t)y * P.nx;
    int n = 0;
    for (int v = 0; v <= 2 * P.R; ++v) {
        const int xx = visit_col(x, v);
        if (xx < 0 || xx >= P.nx) continue;
        const int t = (v + 1) >> 1;
        const float h = gld(&P.H[t * t]);
        int64_t b;
        const int m = col_len(P, row + xx, &b);
        const int cnt = E ? m + 1 : m;
        int l = 0, hh = cnt;  // first chord ending at or above zs
        while (l < hh) {
            const int mid = (l + hh) >> 1;
            if (col_item<E>(P.z, b, m, mid).y + h < zs) l = mid + 1; else hh = mid;
        }
        int hint = 0;
        for (int k = l; k < cnt; ++k) {
            const float2 it = col_item<E>(P.z, b, m, k);
            const float lo = it.x - h, hi = it.y + h;
            if (lo > ze) break;
            n = lv_insert_fwd(U, n, mx(lo, zs), mn(hi, ze), &hint);
            if (n < 0) return -1;
        }
        if (n == 1 && U.get(0).x <= zs && U.get(0).y >= ze) break;
    }
    return n;
}

// K2 restricted to the slab [zs, ze]: the input items of the row window are
// clipped to the slab before painting, so a piece cut at a slab boundary is
// kept as two pieces whose chords overlap.
template <bool E, class Ptr, class L>
__device__ int k2_slab_e(const OpParams& P, int64_t c, float zs, float ze, Ptr Ip, int ni,
                         const L& U, SeedSink& o) {
    int x, y;
    col_xy(P, c, &x, &y);
    const int64_t row = (int64_t)y * P.nx;
    float2 i0 = make_float2(0.f, 0.f);
    if (ni == 1) i0 = Ip[0];
    int n = 0;
    for (int t = 0; t <= P.R; ++t) {
        const int d2 = t * t + 1;
        if (d2 > P.d2max) break;
        const float h1 = gld(&P.H[d2]);
        for (int s = 0; s < (t ? 2 : 1); ++s) {
            const int xx = s ? x + t : x - t;
            if (xx < 0 || xx >= P.nx) continue;
            int64_t b;
            const int m = col_len(P, row + xx, &b);
            const int cnt = E ? m + 1 : m;
            int l = 0, hh = cnt;  // first item ending at or above zs
            while (l < hh) {
                const int mid = (l + hh) >> 1;
                if (col_item<E>(P.z, b, m, mid).y < zs) l = mid + 1; else hh = mid;
            }
            for (int k = l; k < cnt; ++k) {
                const float2 sg = col_item<E>(P.z, b, m, k);
                if (sg.x > ze) break;
                k2_segment(Ip, ni, i0, U, &n, mx(sg.x, zs), mn(sg.y, ze), h1, t, o);
            }
        }
    }
    return o.nlo + o.nhi;
}

template <class Ptr, class L>
__device__ int k2_slab(const OpParams& P, int64_t c, float zs, float ze, Ptr Ip, int ni, const L& U,
                       SeedSink& o) {
    return P.erode ? k2_slab_e<true>(P, c, zs, ze, Ip, ni, U, o) : k2_slab_e<false>(P, c, zs, ze, Ip, ni, U, o);
}

// K3 restricted to the slab [zs, ze]: V0(c) and every seed chord clipped to
// the slab.  Called by all lanes of a wave for one column: at each dy they
// stage the half-widths of every tag in `tab` together, and a lane stops
// adding chords once its slab holds env[dy] (the hull of every chord the rows
// dy .. R can still add) or overflows.  Returns the list size or -1 on
// overflow.
template <class L>
__device__ int k3_slab(const OpParams& P, int64_t c, float zs, float ze, const L& U, float* tab,
                       const float2* env) {
    int x, y;
    col_xy(P, c, &x, &y);
    int n = 0;
    bool ok = true;
    const float2* V = P.A + gld(&P.offA[c]);
    const int n0 = gld(&P.cntA[c]);
    for (int i = 0; i < n0 && ok; ++i) {
        const float2 v = gld(&V[i]);
        const float lo = mx(v.x, zs), hi = mn(v.y, ze);
        if (lo > hi) continue;
        if (n >= U.cap) ok = false; else U.set(n++, make_float2(lo, hi));
    }
    bool busy = ok;
    for (int dy = 1; dy <= P.R; ++dy) {
        const int dy2 = dy * dy;
        __syncthreads();
        for (int t = threadIdx.x; t <= P.R; t += WG) {
            const int d2 = t * t + dy2;
            tab[t] = d2 <= P.d2max ? gld(&P.H[d2]) : -1.0f;
        }
        __syncthreads();
        if (busy) {
            const float2 e = env[dy];
            const float lo = mx(e.x, zs), hi = mn(e.y, ze);
            if (lo > hi) {
                busy = false;
            } else {
                const int i = lv_lower_hi(U, n, hi);
                if (i < n && U.get(i).x <= lo) busy = false;
            }
        }
        if (__all(!busy)) break;
        if (!busy) continue;
        const float hd = tab[0];
        for (int k = 0; k < 4 && busy; ++k) {
            const int yy = (k >> 1) ? y + dy : y - dy;
            if (yy < 0 || yy >= P.ny) continue;
            const int64_t cc = (int64_t)yy * P.nx + x;
            const float4 h4 = gld(&P.hullB[2 * cc + (k & 1)]);
            if (h4.x > h4.y) continue;
            const float hlo = mx(mx(h4.x, h4.z - hd), zs);
            const float hhi = mn(mn(h4.y, h4.w + hd), ze);
            if (hlo > hhi) continue;
            const SeedSpans sp = seed_spans(P, cc);
            const float2* sv = (k & 1) ? sp.s[1] : sp.s[0];
            const uint8_t* tv = (k & 1) ? sp.t[1] : sp.t[0];
            int j0 = 0, nb = (k & 1) ? sp.n[1] : sp.n[0];
            const int64_t ob = gld(&P.offB[cc]);
            if (ob < 0 && gld(&P.loB[cc]) < 0) {
                // a replayed seed column is ordered by its own slabs: scan only
                // the slabs whose chords can reach [zs, ze]
                const int64_t a = -ob - 1;
                const float2* meta = P.arena + a + gld(&P.cntB[cc]);
                const float2 rg = gld(&meta[0]);
                const int* off = (const int*)(meta + 1) + 65 * (k & 1);
                int lo = 0, hi = 63;  // first slab whose top + hd reaches zs
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (slab_bound(rg.x, rg.y, mid + 1) + hd >= zs) hi = mid; else lo = mid + 1;
                }
                const int k0 = lo;
                lo = k0;
                hi = 63;  // last slab whose bottom - hd is at most ze
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (slab_bound(rg.x, rg.y, mid) - hd <= ze) lo = mid; else hi = mid - 1;
                }
                const int k1 = lo;
                j0 = gld(&off[k0]);
                nb = gld(&off[k1 + 1]);
            }
            // every lane reads the same seeds: groups of four loads in flight
            for (int j = j0; j < nb && busy; j += 4) {
                int tq[4];
                float2 pq[4];
                const uint64_t tw = tags4(tv + j);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    tq[q] = (int)((tw >> (8 * q)) & 0xff);
                    pq[q] = gld(&sv[min(j + q, nb - 1)]);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (j + q >= nb) break;
                    const float h = tab[tq[q]];
                    if (h < 0.0f) continue;
                    const float lo = mx(pq[q].x - h, zs), hi = mn(pq[q].y + h, ze);
                    if (lo > hi) continue;
                    n = lv_insert(U, n, lo, hi);
                    if (n < 0) {
                        ok = busy = false;
                        break;
                    }
                }
            }
        }
    }
    return ok ? n : -1;
}

// ---------------------------------------------------------------------------
// emission into bump-allocated per-column lists
// ---------------------------------------------------------------------------

// Write list U (or its complement's closures, dropping the unbounded ends)
// of every valid lane.  Wave-cooperative: one atomic per wave.
template <class L>
__device__ void emit_wave(const OpParams& P, int64_t c, bool valid, const L& U, int n,
                          int complement, unsigned long long* bump, int64_t* off, int32_t* cnt,
                          float2* dst) {
    const int outn = valid ? (complement ? (n > 0 ? n - 1 : 0) : n) : 0;
    int tot;
    const int pre = wave_excl_scan(outn, &tot);
    unsigned long long base = 0;
    if ((threadIdx.x & 63) == 0 && tot > 0) base = atomicAdd(bump, (unsigned long long)tot);
    base = __shfl(base, 0, 64);
    const unsigned long long end = base + (unsigned long long)tot;
    const bool ok = end <= (unsigned long long)P.cap;
    if (!ok && (threadIdx.x & 63) == 0) {
        note_need(P.hdr, end);
        set_error(P.hdr, DEXEL_ERR_WORKSPACE);
    }
    if (!valid) return;
    gst(&off[c], (int64_t)(base + pre));
    gst(&cnt[c], ok ? outn : 0);
    if (!ok) return;
    float2* d = dst + base + pre;
    if (!complement) {
        for (int i = 0; i < n; ++i) gst(&d[i], U.get(i));
    } else {
        for (int i = 0; i + 1 < n; ++i) gst(&d[i], make_float2(U.get(i).y, U.get(i + 1).x));
    }
}

// Single-lane variant for the fallback path.
template <class L>
__device__ void emit_lane(const OpParams& P, int64_t c, const L& U, int n, int complement,
                          unsigned long long* bump, int64_t* off, int32_t* cnt, float2* dst) {
    const int outn = complement ? (n > 0 ? n - 1 : 0) : n;
    const unsigned long long base = atomicAdd(bump, (unsigned long long)outn);
    const unsigned long long end = base + (unsigned long long)outn;
    off[c] = (int64_t)base;
    if (end > (unsigned long long)P.cap) {
        note_need(P.hdr, end);
        set_error(P.hdr, DEXEL_ERR_WORKSPACE);
        cnt[c] = 0;
        return;
    }
    cnt[c] = outn;
    float2* d = dst + base;
    if (!complement) {
        for (int i = 0; i < n; ++i) d[i] = U.get(i);
    } else {
        for (int i = 0; i + 1 < n; ++i) d[i] = make_float2(U.get(i).y, U.get(i + 1).x);
    }
}

// Carve `len` intervals from the arena: their position, or -1 (and a
// workspace error) if they do not fit.  The counter advances either way, so
// after a failed call it holds the arena size the replayed columns asked for
// (a column in the growing tier asks once more per overflow, so this can
// still fall short; the host grows its retries geometrically).
__device__ int64_t arena_alloc(const OpParams& P, int64_t len) {
    const unsigned long long base = atomicAdd(&P.hdr->arena, (unsigned long long)len);
    const unsigned long long end = base + (unsigned long long)len;
    if (end > (unsigned long long)P.cap) {
        note_need(P.hdr, end);
        set_error(P.hdr, DEXEL_ERR_WORKSPACE);
        return -1;
    }
    return (int64_t)base;
}

// ---------------------------------------------------------------------------
// passes over many shapes: shape lookup and per-shape views
// ---------------------------------------------------------------------------

__device__ __forceinline__ void push_overflow(const Pass& Q, int stage, int64_t g) {
    const int k = atomicAdd(&Q.hdr->novf[stage], 1);
    Q.ovf[(int64_t)stage * Q.gcols + k] = (int32_t)g;
}

// Shape holding global column g (the last s with sbase[s] <= g).
__device__ __forceinline__ int find_shape(const Pass& Q, int64_t g) {
    int l = 0, h = Q.nshapes;
    while (h - l > 1) {
        const int m = (l + h) >> 1;
        if (Q.sbase[m] <= g) l = m; else h = m;
    }
    return l;
}

__device__ __forceinline__ OpParams make_op(const Pass& Q, const Shape& S) {
    OpParams p;
    p.nx = S.nx;
    p.ny = S.ny;
    p.ncols = S.ncols;
    p.col_ptr = S.col_ptr;
    p.z = (S.zoff ? S.z + *S.zoff : S.z);
    p.erode = S.erode;
    p.R = S.R;
    p.d2max = S.d2max;
    p.H = S.H;
    p.hdr = Q.hdr;
    p.cap = Q.cap;
    p.gap = S.gap;
    p.ends = S.ends;
    p.offA = S.offA; p.cntA = S.cntA; p.A = Q.A;
    p.offI = S.offI; p.cntI = S.cntI; p.I = Q.I;
    p.offB = S.offB; p.cntB = S.cntB; p.B = Q.B;
    p.tagB = Q.tagB; p.hullB = S.hullB; p.loB = S.loB;
    p.offC = S.offC; p.cntC = S.cntC; p.C = Q.C;
    p.arena = Q.arena;
    p.arena_tag = Q.arena_tag;
    p.slot = Q.seed_slot;
    return p;
}

__device__ __forceinline__ int64_t map_block(int64_t nblocks) {
    // Blocks are dispatched round-robin over the 8 XCDs; give every XCD a
    // contiguous run of columns so that neighbouring columns (which read the
    // same input rows) share one L2.
    const int64_t b = blockIdx.x;
    const int64_t per = (nblocks + 7) / 8;
    const int64_t xcd = b & 7, k = b >> 3;
    const int64_t full = nblocks - (per - 1) * 8;  // XCDs holding `per` blocks
    int64_t start = xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1);
    return start + k;
}

// Wave-uniform placement of a fast-path block: its first global column, the
// shape, and this lane's shape-local column.
struct Place {
    int64_t g0;
    int s;
    int64_t c;
    bool valid;
};

__device__ __forceinline__ Place place_block(const Pass& Q) {
    Place pl;
    pl.g0 = map_block(Q.gcols / WG) * WG;
    pl.s = find_shape(Q, pl.g0);
    pl.c = pl.g0 - Q.sbase[pl.s] + threadIdx.x;
    pl.valid = pl.c < Q.shapes[pl.s].ncols;
    return pl;
}

// Must column c of shape S run the general stage `bit`?  Only shapes with a
// tiled fast path skip stages.  The row offset's main kernel runs twice: in
// its first round on every column of the shapes without a fast path and on
// the needed ones of FAST_THIN shapes (the columns the FAST_SOLID test did
// not settle reach the row offset through its lane replay's list); in the
// second on the FAST_SOLID columns whose V0 the general stages still need.
__device__ __forceinline__ bool needs(const Pass& Q, const Shape& S, int64_t c, int bit) {
    if (S.fast == FAST_DIRECT) return false;
    if (bit == NEED_ROW) {
        if (Q.k1_round == 2)
            return S.fast == FAST_SOLID && (gld(&S.need[c]) & NEED_ROW) && !(gld(&S.gen[c]) & GEN_V0);
        if (S.fast == FAST_NONE) return true;
        return S.fast == FAST_THIN && (gld(&S.need[c]) & NEED_ROW);
    }
    return S.fast == FAST_NONE || (gld(&S.need[c]) & bit);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

using LdsList = LV<WG>;
using MemList = LV<1>;

// Arena tier of the replays, for a column that overflowed its LDS lists:
// evaluate it into `nl` arena lists of ARENA_FIRST entries each, 4x longer
// after each overflow up to the column's upper bound `bound`.  The arena then
// holds about what the column needs, not its bound, which at large radii is
// orders of magnitude more (an abandoned attempt stays allocated: together
// at most a third of the last one).  `eval(M0, M1)` evaluates and emits the
// column and returns -1 on overflow.  If the arena runs out, the call ends
// with a workspace error and the demand counted so far.
constexpr int64_t ARENA_FIRST = 256;

template <class F>
__device__ void arena_eval(const OpParams& P, int nl, int64_t bound, F eval) {
    int64_t len = min<int64_t>(bound, ARENA_FIRST);
    for (;;) {
        const int64_t pos = arena_alloc(P, nl * len);
        if (pos < 0) return;  // the arena demand is counted
        const int cap = (int)min<int64_t>(len, 0x7fffffff);
        const MemList M0{P.arena + pos, cap};
        const MemList M1{P.arena + pos + (nl > 1 ? len : 0), cap};
        if (eval(M0, M1) >= 0) return;
        if (len >= bound) {  // the bound does not hold: never expected
            set_error(P.hdr, DEXEL_ERR_WORKSPACE);
            return;
        }
        len = min<int64_t>(bound, 4 * len);
    }
}

// Summary of every input column of the pass, GAP_LANES lanes per column: its
// first and last item, and its largest gap: between consecutive intervals
// for a dilation, the intervals' own lengths for an erosion (the gaps of the
// complement).  The gap is stored one float step above the largest float
// difference (0 if that is 0: equal floats), so that it bounds every exact
// gap from above; -1 marks an empty column.  K1 reads these per-column arrays with coalesced loads
// instead of two scattered item loads per visited column.
constexpr int GAP_LANES = 4;

__global__ void __launch_bounds__(WG) k_col_gaps(Pass Q) {
    if (Q.hdr->abort) return;
    const int64_t g = (int64_t)blockIdx.x * (WG / GAP_LANES) + threadIdx.x / GAP_LANES;
    const int l = threadIdx.x % GAP_LANES;
    const int s = find_shape(Q, g);
    const OpParams P = make_op(Q, Q.shapes[s]);
    const int64_t c = g - Q.sbase[s];
    const bool valid = c < P.ncols;
    float G = 0.f;
    int m = 0;
    if (valid) {
        const int64_t b = gld(&P.col_ptr[c]);
        m = (int)(gld(&P.col_ptr[c + 1]) - b);
        if (l == 0 && m > 0) {
            const float2 f = gld(&P.z[b]), e = gld(&P.z[b + m - 1]);
            gst(&Q.shapes[s].ends[c], make_float4(f.x, f.y, e.x, e.y));
        }
        if (P.erode) {
            for (int i = l; i < m; i += GAP_LANES) {
                const float2 v = gld(&P.z[b + i]);
                G = mx(G, v.y - v.x);
            }
        } else {
            // lane l holds items l, l + GAP_LANES, ...: the start of the item
            // after its item is the next lane's (for the group's last lane, the
            // first lane's of the next round), so each item is loaded once
            float2 v = l < m ? gld(&P.z[b + l]) : make_float2(DX_INF, DX_INF);
            for (int i0 = 0; i0 < m; i0 += GAP_LANES) {
                const int i = i0 + l;
                const float2 nv = i + GAP_LANES < m ? gld(&P.z[b + i + GAP_LANES]) : make_float2(DX_INF, DX_INF);
                const float s_in = __shfl(v.x, (l + 1) % GAP_LANES, GAP_LANES);
                const float s_nx = __shfl(nv.x, 0, GAP_LANES);
                if (i + 1 < m) G = mx(G, (l + 1 < GAP_LANES ? s_in : s_nx) - v.y);
                v = nv;
            }
        }
    }
#pragma unroll
    for (int d = GAP_LANES / 2; d > 0; d >>= 1) G = mx(G, __shfl_xor(G, d, 64));
    if (valid && l == 0) gst(&Q.shapes[s].gap[c], m == 0 ? -1.f : (G > 0.f ? nextafterf(G, DX_INF) : 0.f));
}

template <int CAP>
__global__ void __launch_bounds__(WG) k_row_offset(Pass Q) {
    __shared__ float2 lds[CAP * WG];
    if (Q.hdr->abort) return;
    const Place pl = place_block(Q);
    bool valid = pl.valid && needs(Q, Q.shapes[pl.s], pl.c, NEED_ROW);
    if (!__any(valid)) return;
    const OpParams P = make_op(Q, Q.shapes[pl.s]);
    LdsList U{&lds[threadIdx.x], CAP};
    int n = valid ? k1_column(P, pl.c, U) : 0;
    if (n < 0) {
        push_overflow(Q, ST_K1, pl.g0 + threadIdx.x);
        valid = false;
        n = 0;
    }
    emit_wave(P, pl.c, valid, U, n, 0, &Q.hdr->bumpA, P.offA, P.cntA, P.A);
}

// Replay of K1 for columns whose list overflowed: one lane per column with a
// K1_FB_CAP-entry LDS list; a column that overflows it too goes on to the
// slab replay (k_row_offset_heavy).
//
// A column the single-interval dilation test left (its gen[] is GEN_V0, its
// lu[] (L, E1, S1, U)) is settled here if the fold reaches one interval
// containing [E1, S1]: the union of [L, E1], V0 and [S1, U] is then all of
// [L, U], so the column's dilation is [L, U] (what the test against V0 would
// conclude) and the rest of its row need not be merged.  It is written like
// a column the test settled, without V0: its gen[] is cleared, so the test
// against V0 skips it and the second row-offset round evaluates its V0 if a
// general column needs it.
__global__ void __launch_bounds__(WG) k_row_offset_fb(Pass Q) {
    __shared__ float2 lds[K1_FB_CAP * WG];
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_K1];
    if ((int64_t)blockIdx.x * WG >= cnt) return;
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= cnt) return;
    const int64_t g = Q.ovf[(int64_t)ST_K1 * Q.gcols + i];
    const int s = find_shape(Q, g);
    const Shape& S = Q.shapes[s];
    const OpParams P = make_op(Q, S);
    const int64_t c = g - Q.sbase[s];
    const bool solid = S.fast == FAST_SOLID && gld(&S.gen[c]) == GEN_V0;
    float4 lu = make_float4(0.f, 0.f, 0.f, 0.f);
    if (solid) lu = gld(&S.lu[c]);
    LdsList L{&lds[threadIdx.x], K1_FB_CAP};
    const int n = k1_column(P, c, L, solid ? make_float2(lu.y, lu.z) : make_float2(DX_INF, -DX_INF));
    // the settled columns' results, one allocation per wave
    const bool done = n == K1_COVERED;
    const unsigned long long dm = __ballot(done);
    if (dm) {
        const int lane = (int)(threadIdx.x & 63);
        const int lead = __ffsll((unsigned long long)__ballot(1)) - 1;
        unsigned long long base = 0;
        if (lane == lead) base = atomicAdd(&Q.hdr->bumpC, (unsigned long long)__popcll(dm));
        base = __shfl(base, lead, 64);
        const unsigned long long end = base + (unsigned long long)__popcll(dm);
        const bool ok = end <= (unsigned long long)P.cap;
        if (!ok && lane == lead) {
            note_need(P.hdr, end);
            set_error(P.hdr, DEXEL_ERR_WORKSPACE);
        }
        if (done) {
            const unsigned long long pos = base + (unsigned long long)__popcll(dm & ((1ull << lane) - 1ull));
            gst(&S.gen[c], (uint8_t)0);
            gst(&P.offC[c], (int64_t)pos);
            gst(&P.cntC[c], ok ? 1 : 0);
            if (ok) gst(&P.C[pos], make_float2(lu.x, lu.w));
        }
    }
    if (done) return;
    if (n >= 0) emit_lane(P, c, L, n, 0, &Q.hdr->bumpA, P.offA, P.cntA, P.A);
    else push_overflow(Q, ST_K1H, g);  // long partial union: the slab replay
}

// Replay of K1 for the columns whose partial union outgrew the lane replay
// (as a rule at the grid's x borders, where the one-sided row window leaves
// the union fragmented): one wave per column, one z-slab per lane; lane 0
// stitches the slab lists into an arena list and emits it.  If a slab list
// overflows, lane 0 evaluates the column alone in the growing arena tier.
__global__ void __launch_bounds__(WG) k_row_offset_heavy(Pass Q) {
    __shared__ float2 lds[CAP_Z * WG];
    __shared__ int nsh[WG];
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_K1H];
    const int lane = threadIdx.x;
    for (int e = blockIdx.x; e < cnt; e += gridDim.x) {
        const int64_t g = Q.ovf[(int64_t)ST_K1H * Q.gcols + e];
        const int s = find_shape(Q, g);
        const OpParams P = make_op(Q, Q.shapes[s]);
        const int64_t c = g - Q.sbase[s];
        int x, y;
        col_xy(P, c, &x, &y);
        const int64_t row = (int64_t)y * P.nx;
        // finite z range of the row window's intervals (column summaries)
        float zmin = DX_INF, zmax = -DX_INF;
        for (int j = lane; j <= 2 * P.R; j += WG) {
            const int xx = x - P.R + j;
            if (xx < 0 || xx >= P.nx || gld(&P.gap[row + xx]) < 0.f) continue;
            const float4 e4 = gld(&P.ends[row + xx]);
            widen(&zmin, &zmax, e4.x);
            widen(&zmin, &zmax, e4.w);
        }
        zmin = wave_min(zmin);
        zmax = wave_max(zmax);
        const float2 sl = lane_slab(zmin, zmax);
        LdsList U{&lds[lane], CAP_Z};
        const int n = P.erode ? k1_slab_e<true>(P, c, sl.x, sl.y, U) : k1_slab_e<false>(P, c, sl.x, sl.y, U);
        __syncthreads();  // the previous column's stitch has read nsh and lds
        nsh[lane] = n;
        __syncthreads();
        const bool fail = __any(n < 0);
        if (lane != 0) continue;
        if (fail) {
            arena_eval(P, 1, k1_bound(P, c), [&](const MemList& M, const MemList&) {
                const int nn = k1_column(P, c, M);
                if (nn >= 0) emit_lane(P, c, M, nn, 0, &Q.hdr->bumpA, P.offA, P.cntA, P.A);
                return nn;
            });
            continue;
        }
        int64_t tot = 0;
        for (int l = 0; l < WG; ++l) tot += nsh[l];
        const int64_t pos = arena_alloc(P, tot > 0 ? tot : 1);
        if (pos < 0) continue;
        float2* out = P.arena + pos;
        int k = 0;
        for (int l = 0; l < WG; ++l)
            for (int i = 0; i < nsh[l]; ++i) {
                const float2 v = lds[i * WG + l];
                if (k > 0 && v.x <= out[k - 1].y) out[k - 1].y = mx(out[k - 1].y, v.y);
                else out[k++] = v;
            }
        MemList M{out, (int)min<int64_t>(tot > 0 ? tot : 1, 0x7fffffff)};
        emit_lane(P, c, M, k, 0, &Q.hdr->bumpA, P.offA, P.cntA, P.A);
    }
}

template <int CAP>
__global__ void __launch_bounds__(WG) k_neighbour(Pass Q) {
    __shared__ float2 lds[2 * CAP * WG];
    if (Q.hdr->abort) return;
    const Place pl = place_block(Q);
    const bool live = pl.valid && needs(Q, Q.shapes[pl.s], pl.c, NEED_SEEDS);
    if (!__any(live)) return;
    const OpParams P = make_op(Q, Q.shapes[pl.s]);
    // a column whose own V0 is fragmented (its neighbours' are too, as a
    // rule) goes straight to the replay
    const bool defer = live && gld(&P.cntA[pl.c]) > K3_DEFER_N;
    bool valid = live && !defer;
    LdsList L0{&lds[threadIdx.x], CAP};
    LdsList L1{&lds[CAP * WG + threadIdx.x], CAP};
    int res = 0;
    int n = valid ? k1b_column(P, pl.c, L0, L1, &res) : 0;
    // a column whose lists overflow is long enough to be worth a whole wave:
    // the slab replay splits its serial chain over 64 lanes
    if (defer || n < 0) push_overflow(Q, ST_K1BH, pl.g0 + threadIdx.x);
    if (n < 0 || defer) {
        valid = false;
        n = 0;
    }
    emit_wave(P, pl.c, valid, res ? L1 : L0, n, 0, &Q.hdr->bumpI, P.offI, P.cntI, P.I);
}

// Replay of K1b for columns whose lists overflowed: one lane per column, a
// CAP_MID-entry LDS list first, then the growing arena tier.
__global__ void __launch_bounds__(WG) k_neighbour_fb(Pass Q) {
    __shared__ float2 lds[2 * CAP_MID * WG];
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_K1B];
    if ((int64_t)blockIdx.x * WG >= cnt) return;
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= cnt) return;
    const int64_t g = Q.ovf[(int64_t)ST_K1B * Q.gcols + i];
    const int s = find_shape(Q, g);
    const OpParams P = make_op(Q, Q.shapes[s]);
    const int64_t c = g - Q.sbase[s];
    {
        LdsList L0{&lds[threadIdx.x], CAP_MID};
        LdsList L1{&lds[CAP_MID * WG + threadIdx.x], CAP_MID};
        int res = 0;
        const int n = k1b_column(P, c, L0, L1, &res);
        if (n >= 0) {
            emit_lane(P, c, res ? L1 : L0, n, 0, &Q.hdr->bumpI, P.offI, P.cntI, P.I);
            return;
        }
    }
    arena_eval(P, 2, k1b_bound(P, c), [&](const MemList& M0, const MemList& M1) {
        int res = 0;
        const int n = k1b_column(P, c, M0, M1, &res);
        if (n >= 0) emit_lane(P, c, res ? M1 : M0, n, 0, &Q.hdr->bumpI, P.offI, P.cntI, P.I);
        return n;
    });
}

// Replay of K1b for heavy columns: one wave per column, one z-slab per lane; lane 0 stitches
// the slab lists (intervals cut at a slab boundary touch there) into an arena
// list and emits it.  If a slab list overflows, lane 0 evaluates the column
// alone in the growing arena tier.
__global__ void __launch_bounds__(WG) k_neighbour_heavy(Pass Q) {
    __shared__ float2 lds[2 * CAP_Z * WG];
    __shared__ int nsh[WG];
    __shared__ int rsh[WG];
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_K1BH];
    const int lane = threadIdx.x;
    for (int e = blockIdx.x; e < cnt; e += gridDim.x) {
        const int64_t g = Q.ovf[(int64_t)ST_K1BH * Q.gcols + e];
        const int s = find_shape(Q, g);
        const OpParams P = make_op(Q, Q.shapes[s]);
        const int64_t c = g - Q.sbase[s];
        int x, y;
        col_xy(P, c, &x, &y);
        // finite z range of V0 over the rows y+-1 .. y+-R
        float zmin = DX_INF, zmax = -DX_INF;
        for (int j = lane; j < 2 * P.R; j += WG) {
            const int yy = (j & 1) ? y + (j >> 1) + 1 : y - (j >> 1) - 1;
            if (yy < 0 || yy >= P.ny) continue;
            const int64_t cc = (int64_t)yy * P.nx + x;
            const int m = gld(&P.cntA[cc]);
            if (m == 0) continue;
            const float2* J = P.A + gld(&P.offA[cc]);
            const float2 f = gld(&J[0]), l = gld(&J[m - 1]);
            widen(&zmin, &zmax, f.x);
            widen(&zmin, &zmax, f.y);
            widen(&zmin, &zmax, l.x);
            widen(&zmin, &zmax, l.y);
        }
        zmin = wave_min(zmin);
        zmax = wave_max(zmax);
        const float2 sl = lane_slab(zmin, zmax);
        LdsList L0{&lds[lane], CAP_Z};
        LdsList L1{&lds[CAP_Z * WG + lane], CAP_Z};
        int res = 0;
        const int n = k1b_slab(P, c, sl.x, sl.y, L0, L1, &res);
        __syncthreads();  // the previous column's stitch has read nsh, rsh and lds
        nsh[lane] = n;
        rsh[lane] = res;
        __syncthreads();
        const bool fail = __any(n < 0);
        if (lane != 0) continue;
        if (fail) {
            arena_eval(P, 2, k1b_bound(P, c), [&](const MemList& M0, const MemList& M1) {
                int r2 = 0;
                const int nn = k1b_column(P, c, M0, M1, &r2);
                if (nn >= 0) emit_lane(P, c, r2 ? M1 : M0, nn, 0, &Q.hdr->bumpI, P.offI, P.cntI, P.I);
                return nn;
            });
            continue;
        }
        int64_t tot = 0;
        for (int l = 0; l < WG; ++l) tot += nsh[l];
        const int64_t pos = arena_alloc(P, tot > 0 ? tot : 1);
        if (pos < 0) continue;
        float2* out = P.arena + pos;
        int k = 0;
        for (int l = 0; l < WG; ++l) {
            const int base = rsh[l] ? CAP_Z * WG : 0;
            for (int i = 0; i < nsh[l]; ++i) {
                const float2 v = lds[base + i * WG + l];
                if (k > 0 && v.x <= out[k - 1].y) out[k - 1].y = mx(out[k - 1].y, v.y);
                else out[k++] = v;
            }
        }
        MemList M{out, (int)min<int64_t>(tot > 0 ? tot : 1, 0x7fffffff)};
        emit_lane(P, c, M, k, 0, &Q.hdr->bumpI, P.offI, P.cntI, P.I);
    }
}

// One traversal per column: the seeds go to the column's slot.  A column
// tested against a fragmented I(c) is deferred, and one with more than
// P.slot seeds is redone, by k_seeds_fb.
template <int CAP>
__global__ void __launch_bounds__(WG) k_seeds(Pass Q) {
    __shared__ float2 lds[CAP * WG];
    if (Q.hdr->abort) return;
    const Place pl = place_block(Q);
    const bool live = pl.valid && needs(Q, Q.shapes[pl.s], pl.c, NEED_SEEDS);
    if (!__any(live)) return;
    const OpParams P = make_op(Q, Q.shapes[pl.s]);
    int np = 0;
    if (live) {
        const int64_t g = pl.g0 + threadIdx.x;
        if (gld(&P.cntI[pl.c]) > K2_DEFER_NI) {
            P.cntB[pl.c] = 0;
            push_overflow(Q, ST_K2H, g);
        } else {
            LdsList U{&lds[threadIdx.x], CAP};
            float2* slot = P.B + g * P.slot;
            uint8_t* tslot = P.tagB + g * P.slot;
            SeedSink o = sink_make(slot, tslot, slot + P.slot - 1, tslot + P.slot - 1, P.slot,
                                   0, 0, seed_split(P, pl.c));
            np = k2_column(P, pl.c, U, o);
            sink_flush(o);
            gst(&P.offB[pl.c], g * P.slot);
            gst(&P.cntB[pl.c], np);
            gst(&P.loB[pl.c], o.nlo);
            gst(&P.hullB[2 * pl.c], o.hlo);
            gst(&P.hullB[2 * pl.c + 1], o.hhi);
            if (np > P.slot) push_overflow(Q, ST_K2, g);
        }
    }
    int tot;
    wave_excl_scan(np, &tot);
    if ((threadIdx.x & 63) == 0 && tot > 0) atomicAdd(&Q.hdr->nseeds, (unsigned long long)tot);
}

// Replay of K2 for columns with more seeds than a slot: one lane per column,
// the same cover capacity (so the same seeds), written to the arena in one
// allocation of the count the first traversal found.
template <int CAP>
__global__ void __launch_bounds__(WG) k_seeds_fb(Pass Q) {
    __shared__ float2 lds[CAP * WG];
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_K2];
    const int i = blockIdx.x * WG + threadIdx.x;
    if ((int64_t)blockIdx.x * WG >= cnt) return;  // whole block past the list
    if (i >= cnt) return;
    const int64_t g = Q.ovf[(int64_t)ST_K2 * Q.gcols + i];
    const int s = find_shape(Q, g);
    const OpParams P = make_op(Q, Q.shapes[s]);
    const int64_t c = g - Q.sbase[s];
    const int want = gld(&P.cntB[c]);
    const int lo = gld(&P.loB[c]);
    const int64_t pos = arena_alloc(P, want);
    if (pos < 0) return;  // the arena demand is counted
    LdsList U{&lds[threadIdx.x], CAP};
    float2* d = P.arena + pos;
    uint8_t* t = P.arena_tag + pos;
    SeedSink o = sink_make(d, t, d + lo, t + lo, 0, lo, want - lo, seed_split(P, c));
    const int np = k2_column(P, c, U, o);
    if (np != want || o.nlo != lo) {
        set_error(Q.hdr, DEXEL_ERR_WORKSPACE);
        return;
    }
    P.offB[c] = -(pos + 1);
}

// Replay of K2 for the columns deferred as heavy: one wave per column,
// one z-slab per lane (count, wave scan, one arena allocation, fill).  I(c)
// is staged in LDS when it fits.
constexpr int ISH = 512;

template <int CAP>
__global__ void __launch_bounds__(WG) k_seeds_heavy(Pass Q) {
    __shared__ float2 lds[CAP * WG];
    __shared__ float2 ish[ISH];
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_K2H];
    const int lane = threadIdx.x;
    for (int e = blockIdx.x; e < cnt; e += gridDim.x) {
        const int64_t g = Q.ovf[(int64_t)ST_K2H * Q.gcols + e];
        const int s = find_shape(Q, g);
        const OpParams P = make_op(Q, Q.shapes[s]);
        const int64_t c = g - Q.sbase[s];
        const int ni = gld(&P.cntI[c]);
        const float2* Ig = P.I + gld(&P.offI[c]);
        const bool staged = ni <= ISH;
        __syncthreads();  // the previous column's readers of ish are done
        if (staged)
            for (int i = lane; i < ni; i += WG) ish[i] = gld(&Ig[i]);
        __syncthreads();
        const float2* Ip = staged ? (const float2*)ish : Ig;
        // finite z range of the row window's input
        int x, y;
        col_xy(P, c, &x, &y);
        float zmin = DX_INF, zmax = -DX_INF;
        for (int j = lane; j <= 2 * P.R; j += WG) {
            const int xx = x - P.R + j;
            if (xx < 0 || xx >= P.nx) continue;
            int64_t b;
            const int m = col_len(P, (int64_t)y * P.nx + xx, &b);
            if (m > 0) {
                widen(&zmin, &zmax, gld(&P.z[b]).x);
                widen(&zmin, &zmax, gld(&P.z[b + m - 1]).y);
            }
        }
        zmin = wave_min(zmin);
        zmax = wave_max(zmax);
        const float2 sl = lane_slab(zmin, zmax);
        LdsList U{&lds[lane], CAP};
        const float zsplit = seed_split(P, c);
        SeedSink o = sink_make(nullptr, nullptr, nullptr, nullptr, 0, 0, 0, zsplit);
        k2_slab(P, c, sl.x, sl.y, Ip, ni, U, o);
        const int nlo = o.nlo, nhi = o.nhi;
        int totlo, tothi;
        const int prelo = wave_excl_scan(nlo, &totlo);
        const int prehi = wave_excl_scan(nhi, &tothi);
        const int tot = totlo + tothi;
        int64_t pos = 0;
        if (lane == 0) pos = arena_alloc(P, tot + SEED_META);
        pos = __shfl(pos, 0, 64);
        if (pos < 0) continue;  // keep counting the arena demand
        // after the seeds: the slab range, then the first seed of every
        // slab in each group (relative to the group's start)
        {
            float2* meta = P.arena + pos + tot;
            int* off = (int*)(meta + 1);
            if (lane == 0) {
                meta[0] = slab_range(zmin, zmax);
                off[64] = totlo;
                off[65 + 64] = tothi;
            }
            off[lane] = prelo;
            off[65 + lane] = prehi;
        }
        const int64_t plo = pos + prelo, phi = pos + totlo + prehi;
        SeedSink o2 = sink_make(P.arena + plo, P.arena_tag + plo, P.arena + phi, P.arena_tag + phi, 0,
                                nlo, nhi, zsplit);
        k2_slab(P, c, sl.x, sl.y, Ip, ni, U, o2);
        if (o2.nlo != nlo || o2.nhi != nhi) set_error(Q.hdr, DEXEL_ERR_WORKSPACE);
        float4 hlo = o2.hlo, hhi = o2.hhi;
        hlo.x = wave_min(hlo.x);
        hlo.y = wave_max(hlo.y);
        hlo.z = wave_min(hlo.z);
        hlo.w = wave_max(hlo.w);
        hhi.x = wave_min(hhi.x);
        hhi.y = wave_max(hhi.y);
        hhi.z = wave_min(hhi.z);
        hhi.w = wave_max(hhi.w);
        if (lane == 0) {
            P.offB[c] = -(pos + 1);
            P.cntB[c] = tot;
            P.loB[c] = ~totlo;
            P.hullB[2 * c] = hlo;
            P.hullB[2 * c + 1] = hhi;
            atomicAdd(&Q.hdr->nseeds, (unsigned long long)tot);
        }
    }
}

template <int CAP>
__global__ void __launch_bounds__(WG) k_union(Pass Q) {
    __shared__ float2 lds[CAP * WG];
    __shared__ float tab[256];
    if (Q.hdr->abort) return;
    const Place pl = place_block(Q);
    if (!pl.valid) Q.cntC_g[pl.g0 + threadIdx.x] = 0;  // padding column
    // columns a tiled fast path finished are skipped
    const bool live = pl.valid && needs(Q, Q.shapes[pl.s], pl.c, NEED_UNION);
    if (!__any(live)) return;
    const OpParams P = make_op(Q, Q.shapes[pl.s]);
    // a column whose V0 is fragmented goes straight to the replay
    const bool defer = live && gld(&P.cntA[pl.c]) > K3_DEFER_N;
    bool valid = live && !defer;
    LdsList U{&lds[threadIdx.x], CAP};
    int n = k3_column<true>(P, pl.c, valid, U, tab);
    if (defer) push_overflow(Q, ST_K3H, pl.g0 + threadIdx.x);
    if (n < 0) push_overflow(Q, ST_K3, pl.g0 + threadIdx.x);
    if (n < 0 || defer) {
        valid = false;
        n = 0;
    }
    emit_wave(P, pl.c, valid, U, n, P.erode, &Q.hdr->bumpC, P.offC, P.cntC, P.C);
}

// Replay of K3 for columns whose list overflowed: one lane per column, a
// CAP_MID-entry LDS list first, then the growing arena tier.
__global__ void __launch_bounds__(WG) k_union_fb(Pass Q) {
    __shared__ float2 lds[CAP_MID * WG];
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_K3];
    if ((int64_t)blockIdx.x * WG >= cnt) return;
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= cnt) return;
    const int64_t g = Q.ovf[(int64_t)ST_K3 * Q.gcols + i];
    const int s = find_shape(Q, g);
    const OpParams P = make_op(Q, Q.shapes[s]);
    const int64_t c = g - Q.sbase[s];
    {
        LdsList L{&lds[threadIdx.x], CAP_MID};
        const int n = k3_column<false>(P, c, true, L, nullptr);
        if (n >= 0) {
            emit_lane(P, c, L, n, P.erode, &Q.hdr->bumpC, P.offC, P.cntC, P.C);
            return;
        }
    }
    arena_eval(P, 1, k3_bound(P, c), [&](const MemList& M, const MemList&) {
        const int n = k3_column<false>(P, c, true, M, nullptr);
        if (n >= 0) emit_lane(P, c, M, n, P.erode, &Q.hdr->bumpC, P.offC, P.cntC, P.C);
        return n;
    });
}

// Replay of K3 for heavy columns: one wave per column, one z-slab per lane; lane 0 stitches the
// slab lists into an arena list and emits it.  If a slab list overflows, lane
// 0 evaluates the column alone in the growing arena tier.
__global__ void __launch_bounds__(WG) k_union_heavy(Pass Q) {
    __shared__ float2 lds[CAP_Z * WG];
    __shared__ float tab[256];
    __shared__ float2 env[256];
    __shared__ int nsh[WG];
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_K3H];
    const int lane = threadIdx.x;
    for (int e = blockIdx.x; e < cnt; e += gridDim.x) {
        const int64_t g = Q.ovf[(int64_t)ST_K3H * Q.gcols + e];
        const int s = find_shape(Q, g);
        const OpParams P = make_op(Q, Q.shapes[s]);
        const int64_t c = g - Q.sbase[s];
        int x, y;
        col_xy(P, c, &x, &y);
        __syncthreads();  // the previous column's stitch has read nsh, lds and env
        // env[dy]: hull of the chords the seed rows y+-dy .. y+-R can add
        // (suffix over dy of the per-row bounds); z range of the data
        float zmin = DX_INF, zmax = -DX_INF;
        if (lane == 0) {
            float2 acc = make_float2(DX_INF, -DX_INF);
            for (int dy = P.R; dy >= 1; --dy) {
                const float hd = gld(&P.H[dy * dy]);
                for (int k = 0; k < 4; ++k) {
                    const int yy = (k >> 1) ? y + dy : y - dy;
                    if (yy < 0 || yy >= P.ny) continue;
                    const float4 h4 = gld(&P.hullB[2 * ((int64_t)yy * P.nx + x) + (k & 1)]);
                    if (h4.x > h4.y) continue;
                    acc.x = mn(acc.x, mx(h4.x, h4.z - hd));
                    acc.y = mx(acc.y, mn(h4.y, h4.w + hd));
                }
                env[dy] = acc;
            }
            widen(&zmin, &zmax, acc.x);
            widen(&zmin, &zmax, acc.y);
        }
        const float2* V = P.A + gld(&P.offA[c]);
        const int n0 = gld(&P.cntA[c]);
        for (int i = lane; i < n0; i += WG) {
            const float2 v = gld(&V[i]);
            widen(&zmin, &zmax, v.x);
            widen(&zmin, &zmax, v.y);
        }
        zmin = wave_min(zmin);
        zmax = wave_max(zmax);
        __syncthreads();  // env is written
        const float2 sl = lane_slab(zmin, zmax);
        LdsList U{&lds[lane], CAP_Z};
        const int n = k3_slab(P, c, sl.x, sl.y, U, tab, env);
        nsh[lane] = n;
        __syncthreads();
        const bool fail = __any(n < 0);
        if (lane != 0) continue;
        if (fail) {
            arena_eval(P, 1, k3_bound(P, c), [&](const MemList& M, const MemList&) {
                const int nn = k3_column<false>(P, c, true, M, nullptr);
                if (nn >= 0) emit_lane(P, c, M, nn, P.erode, &Q.hdr->bumpC, P.offC, P.cntC, P.C);
                return nn;
            });
            continue;
        }
        int64_t tot = 0;
        for (int l = 0; l < WG; ++l) tot += nsh[l];
        const int64_t pos = arena_alloc(P, tot > 0 ? tot : 1);
        if (pos < 0) continue;
        float2* out = P.arena + pos;
        int k = 0;
        for (int l = 0; l < WG; ++l)
            for (int i = 0; i < nsh[l]; ++i) {
                const float2 v = lds[i * WG + l];
                if (k > 0 && v.x <= out[k - 1].y) out[k - 1].y = mx(out[k - 1].y, v.y);
                else out[k++] = v;
            }
        MemList M{(float2*)out, (int)min<int64_t>(tot > 0 ? tot : 1, 0x7fffffff)};
        emit_lane(P, c, M, k, P.erode, &Q.hdr->bumpC, P.offC, P.cntC, P.C);
    }
}

// ---------------------------------------------------------------------------
// direct evaluation of fragmented passes by teams of lanes
// ---------------------------------------------------------------------------
//
// When a pass's result stays fragmented at a small radius (tens of intervals
// per column), the staged path does about the brute force's work (Sec. 4,
// "Baseline Comparison": the seed rows K3 reads hold about as many chords as
// the stencil's items) while its per-column lists overflow into the replays.
// Such a pass (FAST_DIRECT) is evaluated directly: column c's result is the
// union of the chords [a - H[d2], b + H[d2]] of the items [a, b] of every
// column of its stencil (d2 = dx^2 + dy^2 <= floor(r^2); for an erosion the
// items are the column's gaps, unbounded at the ends, and the result the
// gaps of the union), which is the definition the staged path reaches.
//
// A team of T lanes evaluates one column, lane l keeping the union
// restricted to the slab [b_l, b_l+1] of z (b_0 = -inf, b_T = +inf, the
// others evenly spaced over the column's likely range): clipping commutes
// with the union, and the pieces of an interval cut at a slab boundary touch
// there and merge again when the team leader stitches the slabs.  The team
// walks the stencil row by row, nearest rows first; a row of the stencil is
// one contiguous span of the CSR, whose column pointers the team stages in
// LDS.  Each stencil column's items are streamed in chunks of 4T: lane l
// computes the chords of items l, l + T, l + 2T and l + 3T of the chunk into
// the team's LDS buffer, and every lane then reads the whole buffer
// (broadcast reads) and merges the chords, clipped to its slab, into its
// list.  One stencil column's chords arrive in order of their starts (one
// half-width for the whole column), so the merge is a forward walk: a cursor
// in the lane's list only advances, and a chord inside the interval under the
// cursor costs two compares.
//
// The first tier (k_direct1) gives each column one lane and one list, with
// no slabs: every chord is merged once.  A column whose list overflows goes
// to a team of DT lanes (ST_DIRT), then to a whole wave (64 slabs, ST_DIRW),
// then to the arena tier (one lane).
constexpr int TEAM_BLOCKS = 4096;

// Teams of T lanes (T a power of two dividing 64), aligned in the wave.
// Boundary b_k (k = 0 .. T) of T slabs over [zmin, zmax].
template <int T>
__device__ __forceinline__ float team_bound(float zmin, float zmax, int k) {
    if (k <= 0) return -DX_INF;
    if (k >= T) return DX_INF;
    return zmin + (zmax - zmin) * ((float)k * (1.0f / (float)T));
}

template <int T>
__device__ __forceinline__ float team_min(float v) {
#pragma unroll
    for (int d = T / 2; d > 0; d >>= 1) v = mn(v, __shfl_xor(v, d, 64));
    return v;
}

template <int T>
__device__ __forceinline__ float team_max(float v) {
#pragma unroll
    for (int d = T / 2; d > 0; d >>= 1) v = mx(v, __shfl_xor(v, d, 64));
    return v;
}

// Does any lane of this lane's team hold p?  (Called by whole teams.)
template <int T>
__device__ __forceinline__ bool team_any(bool p) {
    const unsigned long long m = (unsigned long long)__ballot(p);
    if (T == 64) return m != 0;
    const int tb = (threadIdx.x & 63) & ~(T - 1);
    return ((m >> tb) & ((1ull << (T & 63)) - 1)) != 0;
}

// Orders a wave's LDS writes before its later reads of what other lanes of
// the wave wrote (a wave's LDS operations complete in order; the fences keep
// the compiler from moving accesses across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int D1_CAP = 32;   // list capacity of the lane-per-column tier
constexpr int DT = 4;        // lanes per column of the team tier
constexpr int DT_CAP = 24;   // its slab list capacity per lane
constexpr int DSPAN = 2 * DIRECT_RMAX + 2;

// Merge [lo, hi] into a canonical list of size n at position i, where every
// U[k] with k < i ends below lo and U[i] (if i < n) does not: as a new
// interval before U[i], or joined with U[i] and every later interval starting
// at or below hi.  Returns the new size (-1 if a new interval does not fit;
// the list is unchanged then); *cur is the interval now at i.
template <class L>
__device__ int lv_merge_at(const L& U, int n, int i, float lo, float hi, float2* cur) {
    if (i == n || U.get(i).x > hi) {
        if (n >= U.cap) return -1;
        for (int k = n; k > i; --k) U.set(k, U.get(k - 1));
        *cur = make_float2(lo, hi);
        U.set(i, *cur);
        return n + 1;
    }
    const float2 ui = U.get(i);
    int j = i;
    float hj = ui.y;
    while (j + 1 < n) {
        const float2 v = U.get(j + 1);
        if (v.x > hi) break;
        hj = v.y;
        ++j;
    }
    *cur = make_float2(mn(lo, ui.x), mx(hi, hj));
    U.set(i, *cur);
    const int sh = j - i;
    if (sh > 0)
        for (int k = j + 1; k < n; ++k) U.set(k - sh, U.get(k));
    return n - sh;
}

// Half-width of row dy of the stencil: the largest w with w^2 + dy^2 <=
// d2max (-1 if the row is outside).
__device__ __forceinline__ int sten_width(int d2max, int dy2) {
    const int rem = d2max - dy2;
    if (rem < 0) return -1;
    int w = (int)sqrtf((float)rem);
    while (w > 0 && w * w > rem) --w;
    while ((w + 1) * (w + 1) <= rem) ++w;
    return w;
}

// Chord of item k of the column at z[b .. b + m) widened by h: the interval
// itself, or for an erosion the column's gap k (k = 0 .. m, unbounded at the
// ends).  Past the last item: an empty chord (lo > hi).
__device__ __forceinline__ float2 item_chord(const float2* z, int64_t b, int m, int k, int erode,
                                             float h) {
    if (!erode) {
        if (k >= m) return make_float2(DX_INF, -DX_INF);
        const float2 v = gld(&z[b + k]);
        return make_float2(v.x - h, v.y + h);
    }
    if (k > m) return make_float2(DX_INF, -DX_INF);
    const float lo = k == 0 ? -DX_INF : gld(&z[b + k - 1]).y;
    const float hi = k == m ? DX_INF : gld(&z[b + k]).x;
    return make_float2(lo - h, hi + h);
}

// Direct evaluation of one column by one lane (the arena tier), and an upper
// bound of its list: every chord of the stencil.
template <class L>
__device__ int direct_column(const OpParams& P, int64_t c, const L& U) {
    int x, y;
    col_xy(P, c, &x, &y);
    int n = 0;
    for (int dy = -P.R; dy <= P.R; ++dy) {
        const int yy = y + dy;
        const int w = sten_width(P.d2max, dy * dy);
        if (yy < 0 || yy >= P.ny || w < 0) continue;
        for (int dx = -w; dx <= w; ++dx) {
            const int xx = x + dx;
            if (xx < 0 || xx >= P.nx) continue;
            const float h = gld(&P.H[dx * dx + dy * dy]);
            int64_t b;
            const int m = col_len(P, (int64_t)yy * P.nx + xx, &b);
            const int cnt = P.erode ? m + 1 : m;
            for (int k = 0; k < cnt; ++k) {
                const float2 ch = item_chord(P.z, b, m, k, P.erode, h);
                n = lv_insert(U, n, ch.x, ch.y);
                if (n < 0) return -1;
            }
        }
    }
    return n;
}

__device__ int64_t direct_bound(const OpParams& P, int64_t c) {
    int x, y;
    col_xy(P, c, &x, &y);
    int64_t b = 1;
    for (int dy = -P.R; dy <= P.R; ++dy) {
        const int yy = y + dy;
        const int w = sten_width(P.d2max, dy * dy);
        if (yy < 0 || yy >= P.ny || w < 0) continue;
        const int x0 = max(x - w, 0), x1 = min(x + w, P.nx - 1);
        const int64_t rb = (int64_t)yy * P.nx;
        b += gld(&P.col_ptr[rb + x1 + 1]) - gld(&P.col_ptr[rb + x0]) + (P.erode ? x1 - x0 + 1 : 0);
    }
    return b;
}

// Lane-per-column tier over every column of the pass's FAST_DIRECT shapes
// (64 consecutive columns per wave).  Each lane walks its stencil row by row
// and each row from the centre out (the widest chords first, which keeps the
// partial union short), and merges each stencil column's chords, loaded
// eight at a time a chunk ahead, into its list with a forward cursor.  The
// lanes of a wave run in lockstep, so a case that is rare for one lane is
// common for the wave; every case but one therefore runs without a branch: a
// chord inside the interval under the cursor (after one predicated step),
// one that extends that interval without reaching the next, and one past the
// end of the list (appended).  The remaining chords (starting a new interval
// inside the list, or joining several) are parked in a short per-lane
// pending list and inserted when the stencil column ends (or the pending
// list is full): the union does not depend on the order of its chords.
constexpr int D1_PEND = 8;

template <int CAP>
__global__ void __launch_bounds__(WG) k_direct1(Pass Q) {
    __shared__ float2 lds[CAP * WG];
    __shared__ float2 pend[D1_PEND * WG];
    if (Q.hdr->abort) return;
    const int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x;
    const int s = find_shape(Q, g < Q.gcols ? g : Q.gcols - 1);
    const Shape& S = Q.shapes[s];
    const int64_t c = g - Q.sbase[s];
    const bool live = g < Q.gcols && S.fast == FAST_DIRECT && c < S.ncols;
    if (!__any(live)) return;
    const OpParams P = make_op(Q, S);
    const LdsList U{&lds[threadIdx.x], CAP};
    const LdsList Pd{&pend[threadIdx.x], D1_PEND};
    const float2 NONE = make_float2(DX_INF, DX_INF);
    int n = 0, np = 0;
    bool ok = live;
    // insert the pending chords into the list
    auto flush = [&]() {
        for (int p = 0; p < np && ok; ++p) {
            const float2 v = Pd.get(p);
            const int nn = lv_insert(U, n, v.x, v.y);
            if (nn < 0) ok = false; else n = nn;
        }
        np = 0;
    };
    if (live) {
        int x, y;
        col_xy(P, c, &x, &y);
        for (int i = 0; i <= 2 * P.R && ok; ++i) {
            const int dy = (i & 1) ? -((i + 1) >> 1) : (i >> 1);  // 0, -1, 1, -2, 2, ...
            const int yy = y + dy;
            const int dy2 = dy * dy;
            const int w = sten_width(P.d2max, dy2);
            if (yy < 0 || yy >= P.ny || w < 0) continue;
            const int64_t rb = (int64_t)yy * P.nx;
            // the row's stencil columns in visit order (x, x - 1, x + 1, ...),
            // eight items a chunk; the next chunk's pointers and items are
            // loaded while the current one is merged
            int v = 0, k0 = 0;
            int64_t b = gld(&P.col_ptr[rb + x]), e = gld(&P.col_ptr[rb + x + 1]);
            float h = gld(&P.H[dy2]);
            float2 cq[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) cq[q] = item_chord(P.z, b, (int)(e - b), q, P.erode, h);
            int ci = 0;
            float2 cur = NONE, nxt = NONE;
            while (v <= 2 * w && ok) {
                const int m = (int)(e - b);
                int nv = v, nk = k0 + 8;
                int64_t nb = b, ne = e;
                float nhh = h;
                if (nk >= (P.erode ? m + 1 : m)) {
                    nk = 0;
                    for (nv = v + 1; nv <= 2 * w; ++nv) {
                        const int xx = visit_col(x, nv);
                        if (xx >= 0 && xx < P.nx) break;
                    }
                    if (nv <= 2 * w) {
                        const int xx = visit_col(x, nv);
                        nb = gld(&P.col_ptr[rb + xx]);
                        ne = gld(&P.col_ptr[rb + xx + 1]);
                        nhh = gld(&P.H[(xx - x) * (xx - x) + dy2]);
                    }
                }
                float2 pq[8];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    pq[q] = nv <= 2 * w ? item_chord(P.z, nb, (int)(ne - nb), nk + q, P.erode, nhh)
                                        : make_float2(DX_INF, -DX_INF);
                if (k0 == 0) {  // a new stencil column: the cursor restarts
                    ci = 0;
                    cur = n > 0 ? U.get(0) : NONE;
                    nxt = n > 1 ? U.get(1) : NONE;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float lo = cq[q].x, hi = cq[q].y;
                    // chords past the column's last item are empty (lo > hi)
                    const bool val = ok && lo <= hi;
                    // one predicated step of the cursor: U[ci] = cur is the first
                    // interval not ending below lo, nxt = U[ci + 1] (NONE past the end)
                    const bool adv = val && cur.y < lo;
                    const float2 t = U.get(min(ci + 2, CAP - 1));
                    ci += adv ? 1 : 0;
                    cur = adv ? nxt : cur;
                    nxt = adv ? (ci + 1 < n ? t : NONE) : nxt;
                    if (val && cur.y < lo) {  // more steps (rare)
                        while (cur.y < lo) {
                            ++ci;
                            cur = nxt;
                            nxt = ci + 1 < n ? U.get(ci + 1) : NONE;
                        }
                    }
                    // classify: inside cur; extends cur without reaching nxt;
                    // past the end (appended); anything else (parked)
                    const bool inside = cur.x <= lo && hi <= cur.y;
                    const bool atend = ci >= n;
                    const bool ext = val && !inside && !atend && cur.x <= hi && hi < nxt.x;
                    const bool app = val && atend && n < CAP;
                    const bool park = val && !inside && !atend && !ext;
                    if (val && atend && n >= CAP) ok = false;
                    const float2 wv = app ? make_float2(lo, hi)
                                          : make_float2(mn(cur.x, lo), mx(cur.y, hi));
                    const int wi = app ? n : ci;
                    if (ext || app) U.set(wi, wv);
                    cur = (ext || app) ? wv : cur;
                    ci = wi;
                    n += app ? 1 : 0;
                    if (park) Pd.set(np, make_float2(lo, hi));
                    np += park ? 1 : 0;
                    if (np == D1_PEND) {  // the pending list is full (rare)
                        flush();
                        ci = 0;
                        cur = n > 0 ? U.get(0) : NONE;
                        nxt = n > 1 ? U.get(1) : NONE;
                    }
                }
                if (nk == 0 && np > 0) flush();  // the stencil column ends
#pragma unroll
                for (int q = 0; q < 8; ++q) cq[q] = pq[q];
                v = nv;
                k0 = nk;
                b = nb;
                e = ne;
                h = nhh;
            }
        }
    }
    // overflowing columns go to the team tier; the others are emitted
    if (live && !ok) push_overflow(Q, ST_DIRT, g);
    emit_wave(P, c, live && ok, U, ok ? n : 0, P.erode, &Q.hdr->bumpC, P.offC, P.cntC, P.C);
}

// Team tiers: the columns on list `src` (ST_DIRT or ST_DIRW) by teams of T
// lanes; a column whose slab list overflows goes on list `dst`, or with dst
// < 0 to the arena tier.
template <int T, int CAP>
__global__ void __launch_bounds__(WG) k_direct(Pass Q, int src, int dst) {
    constexpr int TPW = WG / T;
    __shared__ float2 lds[CAP * WG];
    __shared__ float2 chs[TPW][4 * T + 2];  // padded: the teams' buffers start on different banks
    __shared__ int32_t cps[TPW][DSPAN];
    __shared__ int nsh[WG];
    if (Q.hdr->abort) return;
    const int64_t total = Q.hdr->novf[src];
    const int lane = threadIdx.x;
    const int lt = lane & (T - 1);
    const int tb = lane - lt;
    const int tm = lane / T;
    const LdsList U{&lds[lane], CAP};
    for (int64_t e0 = (int64_t)blockIdx.x * TPW; e0 < total; e0 += (int64_t)gridDim.x * TPW) {
        const int64_t e = e0 + tm;
        const int64_t ei = e < total ? e : e0;
        const int64_t g = Q.ovf[(int64_t)src * Q.gcols + ei];
        const int s = find_shape(Q, g);
        const Shape& S = Q.shapes[s];
        const int64_t c = g - Q.sbase[s];
        const bool live = e < total && S.fast == FAST_DIRECT && c < S.ncols;  // the same for a team
        const OpParams P = make_op(Q, S);
        int n = 0;
        bool ok = true;
        if (live) {
            int x, y;
            col_xy(P, c, &x, &y);
            // slab range: the items of the stencil's central row and column,
            // widened by r (the slabs only balance the lanes' work)
            float zmin = DX_INF, zmax = -DX_INF;
            const int half = 2 * P.R + 1;
            for (int p = lt; p < 2 * half; p += T) {
                const int xx = p < half ? x : x + (p - half) - P.R;
                const int yy = p < half ? y + p - P.R : y;
                if (xx < 0 || xx >= P.nx || yy < 0 || yy >= P.ny) continue;
                const int64_t cc = (int64_t)yy * P.nx + xx;
                if (gld(&P.gap[cc]) < 0.0f) continue;  // empty column
                const float4 e4 = gld(&P.ends[cc]);
                widen(&zmin, &zmax, e4.x);
                widen(&zmin, &zmax, e4.w);
            }
            zmin = team_min<T>(zmin);
            zmax = team_max<T>(zmax);
            if (zmin <= zmax) {
                const float h0 = gld(&P.H[0]);
                zmin -= h0;
                zmax += h0;
            }
            const float2 rg = slab_range(zmin, zmax);
            const float zs = team_bound<T>(rg.x, rg.y, lt), ze = team_bound<T>(rg.x, rg.y, lt + 1);
            bool fail = false;
            for (int i = 0; i <= 2 * P.R && !fail; ++i) {
                const int dy = (i & 1) ? -((i + 1) >> 1) : (i >> 1);  // 0, -1, 1, -2, 2, ...
                const int yy = y + dy;
                const int dy2 = dy * dy;
                const int w = sten_width(P.d2max, dy2);
                if (yy < 0 || yy >= P.ny || w < 0) continue;
                const int x0 = max(x - w, 0), x1 = min(x + w, P.nx - 1);
                const int64_t rb = (int64_t)yy * P.nx + x0;
                const int64_t zb = gld(&P.col_ptr[rb]);
                wave_lds_sync();  // the last row's pointers are read
                for (int j = lt; j <= x1 - x0 + 1; j += T) cps[tm][j] = (int32_t)(gld(&P.col_ptr[rb + j]) - zb);
                wave_lds_sync();
                // the row's chunks in order: stencil columns in visit order,
                // 4T items each; the next chunk's items are loaded while the
                // current one is merged
                int cv = -1, cm = 0;
                int64_t cb = 0;
                float chh = 0.0f;
                for (int v = 0; v <= 2 * w; ++v) {
                    const int xx = visit_col(x, v);
                    if (xx < x0 || xx > x1) continue;
                    const int o = cps[tm][xx - x0];
                    cm = cps[tm][xx - x0 + 1] - o;
                    if (!P.erode && cm == 0) continue;  // an empty column adds nothing
                    cb = zb + o;
                    chh = gld(&P.H[(xx - x) * (xx - x) + dy2]);
                    cv = v;
                    break;
                }
                int ck = 0;
                float2 q4[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    q4[q] = cv >= 0 ? item_chord(P.z, cb, cm, q * T + lt, P.erode, chh)
                                    : make_float2(DX_INF, -DX_INF);
                // merge cursor: U[ci] = cur is the first interval not ending below
                // the chords still to come in this stencil column (ci = n: none);
                // nxt = U[ci + 1], loaded ahead
                int ci = 0;
                float2 cur = make_float2(DX_INF, DX_INF), nxt = cur;
                while (cv >= 0 && !fail) {
                    int nv = cv, nk = ck + 4 * T, nm = cm;
                    int64_t nb = cb;
                    float nh = chh;
                    if (nk >= (P.erode ? cm + 1 : cm)) {
                        nk = 0;
                        nv = -1;
                        for (int v = cv + 1; v <= 2 * w; ++v) {
                            const int xx = visit_col(x, v);
                            if (xx < x0 || xx > x1) continue;
                            const int o = cps[tm][xx - x0];
                            nm = cps[tm][xx - x0 + 1] - o;
                            if (!P.erode && nm == 0) continue;
                            nb = zb + o;
                            nh = gld(&P.H[(xx - x) * (xx - x) + dy2]);
                            nv = v;
                            break;
                        }
                    }
                    float2 p4[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        p4[q] = nv >= 0 ? item_chord(P.z, nb, nm, nk + q * T + lt, P.erode, nh)
                                        : make_float2(DX_INF, -DX_INF);
                    if (ck == 0) {  // a new stencil column: the cursor restarts
                        ci = 0;
                        cur = n > 0 ? U.get(0) : make_float2(DX_INF, DX_INF);
                        nxt = n > 1 ? U.get(1) : make_float2(DX_INF, DX_INF);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) chs[tm][q * T + lt] = q4[q];
                    wave_lds_sync();
                    // the chunk in blocks of SB chords, each read into registers at once
                    constexpr int SB = 4 * T < 16 ? 4 * T : 16;
                    for (int u0 = 0; u0 < 4 * T; u0 += SB) {
                        float2 cq[SB];
#pragma unroll
                        for (int u = 0; u < SB; ++u) cq[u] = chs[tm][u0 + u];
#pragma unroll
                        for (int u = 0; u < SB; ++u) {
                            // chords past the column's last item are empty
                            const float lo = mx(cq[u].x, zs), hi = mn(cq[u].y, ze);
                            if (!ok || !(lo <= hi)) continue;
                            while (cur.y < lo) {
                                ++ci;
                                cur = nxt;
                                nxt = ci + 1 < n ? U.get(ci + 1) : make_float2(DX_INF, DX_INF);
                            }
                            if (cur.x <= lo && hi <= cur.y) continue;  // inside
                            const int nn = lv_merge_at(U, n, ci, lo, hi, &cur);
                            if (nn < 0) {
                                ok = false;
                            } else {
                                n = nn;
                                nxt = ci + 1 < n ? U.get(ci + 1) : make_float2(DX_INF, DX_INF);
                            }
                        }
                    }
                    wave_lds_sync();  // the buffer is read before the next chunk is written
                    fail = team_any<T>(!ok);
#pragma unroll
                    for (int q = 0; q < 4; ++q) q4[q] = p4[q];
                    cv = nv;
                    ck = nk;
                    cm = nm;
                    cb = nb;
                    chh = nh;
                }
            }
        }
        const bool fail = team_any<T>(live && !ok);
        nsh[lane] = n;
        __syncthreads();  // every slab list and its size are written
        // the team leader stitches the slab lists: count first
        int outn = 0;
        if (live && !fail && lt == 0) {
            int m = 0;
            float py = 0.0f;
            for (int l = 0; l < T; ++l)
                for (int i = 0, nl = nsh[tb + l]; i < nl; ++i) {
                    const float2 v = lds[i * WG + tb + l];
                    if (m > 0 && v.x <= py) {
                        py = mx(py, v.y);
                    } else {
                        ++m;
                        py = v.y;
                    }
                }
            outn = P.erode ? (m > 0 ? m - 1 : 0) : m;
        }
        int tot;
        const int pre = wave_excl_scan(outn, &tot);
        unsigned long long base = 0;
        if (lane == 0 && tot > 0) base = atomicAdd(&Q.hdr->bumpC, (unsigned long long)tot);
        base = __shfl(base, 0, 64);
        const unsigned long long end = base + (unsigned long long)tot;
        const bool fits = end <= (unsigned long long)Q.cap;
        if (!fits && lane == 0) {
            note_need(Q.hdr, end);
            set_error(Q.hdr, DEXEL_ERR_WORKSPACE);
        }
        if (live && lt == 0) {
            if (fail && dst >= 0) {
                push_overflow(Q, dst, g);
            } else if (fail) {
                arena_eval(P, 1, direct_bound(P, c), [&](const MemList& M, const MemList&) {
                    const int nn = direct_column(P, c, M);
                    if (nn >= 0) emit_lane(P, c, M, nn, P.erode, &Q.hdr->bumpC, P.offC, P.cntC, P.C);
                    return nn;
                });
            } else {
                gst(&P.offC[c], (int64_t)(base + pre));
                gst(&P.cntC[c], fits ? outn : 0);
                if (fits) {
                    // again, writing: the merged intervals, or the gaps
                    // between them for an erosion
                    float2* d = P.C + base + pre;
                    int m = 0;
                    float2 cur = make_float2(0.0f, 0.0f);
                    float prev_hi = 0.0f;
                    for (int l = 0; l < T; ++l)
                        for (int i = 0, nl = nsh[tb + l]; i < nl; ++i) {
                            const float2 v = lds[i * WG + tb + l];
                            if (m > 0 && v.x <= cur.y) {
                                cur.y = mx(cur.y, v.y);
                                continue;
                            }
                            if (m > 0) {
                                if (!P.erode) gst(&d[m - 1], cur);
                                else if (m >= 2) gst(&d[m - 2], make_float2(prev_hi, cur.x));
                                prev_hi = cur.y;
                            }
                            cur = v;
                            ++m;
                        }
                    if (m > 0) {
                        if (!P.erode) gst(&d[m - 1], cur);
                        else if (m >= 2) gst(&d[m - 2], make_float2(prev_hi, cur.x));
                    }
                }
            }
        }
        __syncthreads();  // the leaders have read the lists before they are reused
    }
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts into int64 offsets (with the total at [n])
// ---------------------------------------------------------------------------

constexpr int SCAN_T = 256;
constexpr int SCAN_V = 4;
constexpr int SCAN_B = SCAN_T * SCAN_V;

__device__ int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t* total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < SCAN_T; d <<= 1) {
        int64_t y = (t >= d) ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    const int64_t incl = sh[t];
    *total = sh[SCAN_T - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_reduce(const int32_t* cnt, int64_t n, int64_t* bsum,
                                                        const WsHeader* hdr) {
    __shared__ int64_t sh[SCAN_T];
    if (hdr->abort) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_B;
    int64_t s = 0;
    for (int k = 0; k < SCAN_V; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_V + k;
        if (i < n) s += cnt[i];
    }
    int64_t tot;
    block_excl_scan(s, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_bsum(int64_t* bsum, int64_t nb, const WsHeader* hdr) {
    __shared__ int64_t sh[SCAN_T];
    if (hdr->abort) return;
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_T) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nb ? bsum[i] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(v, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_apply(const int32_t* cnt, int64_t n,
                                                       const int64_t* bsum, int64_t nb, int64_t* off,
                                                       const WsHeader* hdr) {
    __shared__ int64_t sh[SCAN_T];
    if (hdr->abort) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_B;
    int32_t v[SCAN_V];
    int64_t s = 0;
    for (int k = 0; k < SCAN_V; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_V + k;
        v[k] = i < n ? cnt[i] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t run = block_excl_scan(s, sh, &tot) + bsum[blockIdx.x];
    for (int k = 0; k < SCAN_V; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_V + k;
        if (i < n) off[i] = run;
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) off[n] = bsum[nb];
}

static hipError_t scan_counts(const int32_t* cnt, int64_t n, int64_t* bsum, int64_t* off,
                              const WsHeader* hdr, hipStream_t s) {
    const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    if (nb > 0) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_T), 0, s, cnt, n, bsum, hdr);
    }
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(SCAN_T), 0, s, bsum, nb, hdr);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(SCAN_T), 0, s, cnt, n,
                       bsum, nb, off, hdr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// erosion of thin columns
// ---------------------------------------------------------------------------
//
// An erosion complements every in-grid stencil column on read.  When each of
// them holds at most one interval [a, b], its complement is the two rays
// (-inf, a] and [b, +inf) (the whole line if the column is empty), and a
// ray's chord only moves the ray's end.  The union of all chords is then
// (-inf, MA] U [MB, +inf) with MA = max fl(a + H[d2]) and MB =
// min fl(b - H[d2]) over the ball's stencil, and the eroded column is
// [MA, MB] if MA < MB, else empty: a max / min filter over the stencil, with
// the same chords and roundings as the general kernels.
//
// k_thin_erode evaluates it on tiles of THIN_TX x THIN_TY output columns of
// the pass's thin shapes: the tile's (THIN_TX + 2R) x (THIN_TY + 2R)
// neighbourhood is staged in LDS once as one (a, b) pair per column (empty:
// (+inf, -inf), so that MA = +inf; outside the grid: (-inf, +inf), which
// changes nothing; a column of two or more intervals: NaN), then each wave
// evaluates THIN_TY / 4 output rows, one lane per column.  An output column
// whose stencil holds a longer column is marked general (GEN_GENERAL) and
// left to the general kernels; k_fast_spread marks the columns those must
// evaluate for it (need[]).
constexpr int THIN_T = 256;


// One stencil row of the tiled filters: f(v, hh) for dx = -w .. w with
// v = row[dx] and hh = hq[dx + w] (the row's half-widths, contiguous and
// 16-byte aligned), the LDS loads of four points issued together and their
// four half-widths one load (the same address in every lane).
template <class T, class F>
__device__ __forceinline__ void sweep_row(const T* row, const float* hq, int w, F f) {
    const float4* h4 = (const float4*)hq;
    const int ng = (2 * w + 1) >> 2;
    int dx = -w;
    if (ng > 0) {
        T v0 = row[dx], v1 = row[dx + 1], v2 = row[dx + 2], v3 = row[dx + 3];
        float4 h = h4[0];
        for (int g = 1; g < ng; ++g) {
            const T n0 = row[dx + 4], n1 = row[dx + 5], n2 = row[dx + 6], n3 = row[dx + 7];
            const float4 nh = h4[g];
            f(v0, h.x);
            f(v1, h.y);
            f(v2, h.z);
            f(v3, h.w);
            v0 = n0; v1 = n1; v2 = n2; v3 = n3; h = nh;
            dx += 4;
        }
        f(v0, h.x);
        f(v1, h.y);
        f(v2, h.z);
        f(v3, h.w);
        dx += 4;
    }
    const float* ht = (const float*)(h4 + ng);
    for (int k = 0; dx <= w; ++dx, ++k) f(row[dx], ht[k]);
}

template <class T, class F>
__device__ __forceinline__ void sweep_row2(const T* ra, const T* rb, const float* hq, int w, F f) {
    const float4* h4 = (const float4*)hq;
    const int ng = (2 * w + 1) >> 2;
    int dx = -w;
    if (ng > 0) {
        T v0 = ra[dx], v1 = ra[dx + 1], v2 = ra[dx + 2], v3 = ra[dx + 3];
        T u0 = rb[dx], u1 = rb[dx + 1], u2 = rb[dx + 2], u3 = rb[dx + 3];
        float4 h = h4[0];
        for (int g = 1; g < ng; ++g) {
            const T n0 = ra[dx + 4], n1 = ra[dx + 5], n2 = ra[dx + 6], n3 = ra[dx + 7];
            const T m0 = rb[dx + 4], m1 = rb[dx + 5], m2 = rb[dx + 6], m3 = rb[dx + 7];
            const float4 nh = h4[g];
            f(v0, u0, h.x);
            f(v1, u1, h.y);
            f(v2, u2, h.z);
            f(v3, u3, h.w);
            v0 = n0; v1 = n1; v2 = n2; v3 = n3;
            u0 = m0; u1 = m1; u2 = m2; u3 = m3; h = nh;
            dx += 4;
        }
        f(v0, u0, h.x);
        f(v1, u1, h.y);
        f(v2, u2, h.z);
        f(v3, u3, h.w);
        dx += 4;
    }
    const float* ht = (const float*)(h4 + ng);
    for (int k = 0; dx <= w; ++dx, ++k) f(ra[dx], rb[dx], ht[k]);
}

// The stencil tables of the tiled filters, staged by the whole block (the
// caller synchronises before reading them): wd[k] = w_k, the largest |dx| of
// stencil row |dy| = k; ro[k], the offset of that row in Hr (a multiple of
// four); Hr[ro[k] + i] = H[(i - w_k)^2 + k^2] for i = 0 .. 2 w_k.  Each
// thread k works out w_j of the rows j <= k itself, so the offsets need no
// synchronisation of their own.
__device__ __forceinline__ int row_width(int d2max, int k) {
    int w = 0;
    while ((w + 1) * (w + 1) + k * k <= d2max) ++w;
    return w;
}

__device__ __forceinline__ void stage_stencil(const OpParams& P, float* Hr, int* ro, int* wd) {
    for (int k = threadIdx.x; k <= P.R; k += blockDim.x) {
        int off = 0;
        for (int j = 0; j < k; ++j) off += (2 * row_width(P.d2max, j) + 4) & ~3;
        const int w = row_width(P.d2max, k);
        wd[k] = w;
        ro[k] = off;
        for (int i = 0; i <= 2 * w; ++i) Hr[off + i] = gld(&P.H[(i - w) * (i - w) + k * k]);
    }
}

__global__ void __launch_bounds__(THIN_T) k_thin_erode(Pass Q) {
    extern __shared__ float4 thin_lds[];
    if (Q.hdr->abort) return;
    const int64_t t = map_block(Q.ntiles);
    int lo = 0, hi = Q.nshapes;  // the last shape whose tiles start at or before t
    while (hi - lo > 1) {
        const int m = (lo + hi) >> 1;
        if (Q.shapes[m].tbase <= t) lo = m; else hi = m;
    }
    const Shape& S = Q.shapes[lo];
    if (S.fast != FAST_THIN) return;
    const OpParams P = make_op(Q, S);
    const int R = P.R;
    const int ntx = (P.nx + THIN_TX - 1) / THIN_TX;
    const int64_t tl = t - S.tbase;
    const int x0 = (int)(tl % ntx) * THIN_TX, y0 = (int)(tl / ntx) * THIN_TY;
    const int SW = THIN_TX + 2 * R, SH = THIN_TY + 2 * R;
    float2* st = (float2*)thin_lds;
    float* Hr = (float*)(st + SW * SH);  // 16-byte aligned: SW * SH is even
    int* wd = (int*)(Hr + (P.R + 1) * (2 * P.R + 4));  // the table's bound
    int* ro = wd + (P.R + 1);
    stage_stencil(P, Hr, ro, wd);
    int thick = 0;
    for (int i = threadIdx.x; i < SW * SH; i += THIN_T) {
        const int sy = i / SW, sx = i - sy * SW;
        const int xx = x0 - R + sx, yy = y0 - R + sy;
        float2 v = make_float2(-DX_INF, DX_INF);
        if (xx >= 0 && xx < P.nx && yy >= 0 && yy < P.ny) {
            const int64_t c = (int64_t)yy * P.nx + xx;
            const int64_t b = gld(&P.col_ptr[c]);
            const int m = (int)(gld(&P.col_ptr[c + 1]) - b);
            if (m == 0) {
                v = make_float2(DX_INF, -DX_INF);
            } else if (m == 1) {
                v = gld(&P.z[b]);
            } else {
                v = make_float2(__builtin_nanf(""), __builtin_nanf(""));
                thick = 1;
            }
        }
        st[i] = v;
    }
    const int any_thick = __syncthreads_or(thick);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = x0 + lane;
    for (int k = 0; k < THIN_TY / 4; ++k) {
        const int ly = wv + 4 * k;
        const int y = y0 + ly;
        if (y >= P.ny) break;  // wave-uniform
        const bool live = x < P.nx;
        const float2* ctr = st + (ly + R) * SW + lane + R;
        float MA = -DX_INF, MB = DX_INF;
        bool thk = false;
        // the rows y - k and y + k together: they share their half-widths,
        // and rounding is monotone, so max(fl(a + h), fl(b + h)) =
        // fl(max(a, b) + h) (a column marked thick is left general whatever
        // its MA and MB)
        for (int k = 0; k <= R; ++k) {
            const int w = wd[k];
            const float* hr = Hr + ro[k];
            if (k == 0) {
                sweep_row(ctr, hr, w, [&](float2 v, float hh) {
                    thk |= v.x != v.x;
                    MA = mx(MA, v.x + hh);
                    MB = mn(MB, v.y - hh);
                });
            } else if (any_thick) {
                sweep_row2(ctr + k * SW, ctr - k * SW, hr, w, [&](float2 a, float2 b, float hh) {
                    thk |= (a.x != a.x) | (b.x != b.x);
                    MA = mx(MA, mx(a.x, b.x) + hh);
                    MB = mn(MB, mn(a.y, b.y) - hh);
                });
            } else {
                sweep_row2(ctr + k * SW, ctr - k * SW, hr, w, [&](float2 a, float2 b, float hh) {
                    MA = mx(MA, mx(a.x, b.x) + hh);
                    MB = mn(MB, mn(a.y, b.y) - hh);
                });
            }
        }
        const bool done = live && !thk;
        const int outn = (done && MA < MB) ? 1 : 0;
        int tot;
        const int pre = wave_excl_scan(outn, &tot);
        unsigned long long base = 0;
        if (lane == 0 && tot > 0) base = atomicAdd(&Q.hdr->bumpC, (unsigned long long)tot);
        base = __shfl(base, 0, 64);
        const unsigned long long end = base + (unsigned long long)tot;
        const bool ok = end <= (unsigned long long)P.cap;
        if (!ok && lane == 0) {
            note_need(P.hdr, end);
            set_error(P.hdr, DEXEL_ERR_WORKSPACE);
        }
        if (!live) continue;
        const int64_t c = (int64_t)y * P.nx + x;
        gst(&S.gen[c], (uint8_t)(thk ? GEN_GENERAL : 0));
        if (!done) continue;
        gst(&P.offC[c], (int64_t)(base + pre));
        gst(&P.cntC[c], ok ? outn : 0);
        if (ok && outn) gst(&P.C[base + pre], make_float2(MA, MB));
    }
}

// ---------------------------------------------------------------------------
// dilation by the chord extremes and a gap cut
// ---------------------------------------------------------------------------
//
// Every chord of an output column's stencil lies in [L, U], with
// L = min fl(af - H[d2]) and U = max fl(bl + H[d2]) over the stencil columns
// (af, bl: a column's first start and last end), and both ends belong to the
// union.  Three chords chain into [L, U] in most columns of a solid shape:
// [L, E1], where E1 is the largest end of the chords starting at L (each a
// column's first chord: it has the column's smallest start and smallest
// end); [S1, U], likewise at the top with last chords; and the hull [A, B]
// of a column whose gaps are all within 2H[d2] (its chords chain into
// [af - h, bl + h]).  If E1 >= S1, or some such hull has A <= E1 and
// B >= S1, the column's dilation is exactly [L, U] and nothing else of it is
// evaluated.  L, U, E1 and S1 are taken over the whole stencil (E1 and S1
// in a second sweep once L and U are known), the hulls only over its inner
// part (d2 <= d2max / 4), where the columns whose gaps are short enough for
// their distance are as a rule: a hull missed there only sends the column on
// to the exact evaluation.
// k_solid_dilate evaluates these filters on LDS-staged tiles of
// THIN_TX x SOLID_TY output columns ((af, bl) of each neighbourhood column;
// (bf, al) and the largest-gap bound come from the column summaries where
// needed); every other column goes to the row offset's lane replay, which
// settles most of them as soon as their partial row union spans [E1, S1],
// and the rest, with V0, to k_solid_b.
//
// k_solid_b tests a column against V0(c) = [L0 .. U0], the union of the
// chords of its own row: the union is [L, U] minus the points of the open
// gaps of [L, E1] U V0 U [S1, U] inside [L, U] that no chord of another row
// covers.  A column without such a gap is settled; one with at most GC_CAP
// goes to the gap cut (k_gap_cut), which applies the chords of the other
// rows to them, one with at most GCW_MAX to the wide gap cut (one wave per
// column, one gap per lane: at the grid's x border the one-sided row window
// leaves tens of gaps); every other column is left to the general kernels.
constexpr int GC_CAP = 4;      // open gaps the gap cut tracks per column (pieces per lane in the wide one)
constexpr int GC_BUDGET = 160; // stencil columns meeting a gap it visits before giving up
constexpr int GCW_MAX = 64;    // gaps the wide gap cut takes (one lane each)

__global__ void __launch_bounds__(THIN_T) k_solid_dilate(Pass Q) {
    extern __shared__ float4 solid_lds[];
    if (Q.hdr->abort) return;
    const int64_t t = map_block(Q.ntiles);
    int lo = 0, hi = Q.nshapes;
    while (hi - lo > 1) {
        const int m = (lo + hi) >> 1;
        if (Q.shapes[m].tbase <= t) lo = m; else hi = m;
    }
    const Shape& S = Q.shapes[lo];
    if (S.fast != FAST_SOLID) return;
    const OpParams P = make_op(Q, S);
    const int R = P.R;
    const int ntx = (P.nx + THIN_TX - 1) / THIN_TX;
    const int64_t tl = t - S.tbase;
    const int x0 = (int)(tl % ntx) * THIN_TX, y0 = (int)(tl / ntx) * SOLID_TY;
    const int SW = THIN_TX + 2 * R, SH = SOLID_TY + 2 * R;
    float2* sab = (float2*)solid_lds;        // (af, bl)
    float* Hr = (float*)(sab + SW * SH);     // 16-byte aligned: SW * SH is even
    int* wd = (int*)(Hr + (P.R + 1) * (2 * P.R + 4));  // the table's bound
    int* ro = wd + (P.R + 1);
    stage_stencil(P, Hr, ro, wd);
    // Only (af, bl) of each neighbourhood column is staged ((+inf, -inf) for
    // an empty or off-grid one: it changes no filter and is never a hull);
    // (bf, al) and the largest-gap bound are read from the column summaries
    // at the few stencil points that need them, which leaves room in LDS for
    // twice the resident tiles.
    for (int i = threadIdx.x; i < SW * SH; i += THIN_T) {
        const int sy = i / SW, sx = i - sy * SW;
        const int xx = x0 - R + sx, yy = y0 - R + sy;
        float2 ab = make_float2(DX_INF, -DX_INF);
        if (xx >= 0 && xx < P.nx && yy >= 0 && yy < P.ny) {
            const int64_t c = (int64_t)yy * P.nx + xx;
            if (gld(&P.gap[c]) >= 0.f) {
                const float4 e4 = gld(&P.ends[c]);
                ab = make_float2(e4.x, e4.w);
            }
        }
        sab[i] = ab;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = x0 + lane;
    const int d2in = P.d2max / 4;
    for (int k = 0; k < SOLID_TY / 4; ++k) {
        const int ly = wv + 4 * k;
        const int y = y0 + ly;
        if (y >= P.ny) break;  // wave-uniform
        const int ci = (ly + R) * SW + lane + R;
        // L and U over the whole stencil, row by row, with the rows whose
        // chords reach L (mL) or U (mU): bit dy + R, while 2R + 1 <= 64.
        // (Taking the rows y - k and y + k together, as the thin filter does,
        // would name both rows of a pair in the masks and double the rows
        // the E1 / S1 sweep visits.)
        float L = DX_INF, U = -DX_INF;
        uint64_t mL = 0, mU = 0;
        const bool masks = 2 * R + 1 <= 64;
        for (int dy = -R; dy <= R; ++dy) {
            // a row off the grid holds only empty cells (all lanes share y)
            if (y + dy < 0 || y + dy >= P.ny) continue;
            const int w = wd[dy < 0 ? -dy : dy];
            const float* hr = Hr + ro[dy < 0 ? -dy : dy];
            float rL = DX_INF, rU = -DX_INF;
            sweep_row(sab + ci + dy * SW, hr, w, [&](float2 v, float hh) {
                rL = mn(rL, v.x - hh);
                rU = mx(rU, v.y + hh);
            });
            const uint64_t bit = masks ? 1ull << (dy + R) : 0ull;
            mL = rL < L ? bit : (rL == L ? mL | bit : mL);
            mU = rU > U ? bit : (rU == U ? mU | bit : mU);
            L = mn(L, rL);
            U = mx(U, rU);
        }
        // E1 and S1: a row without a chord starting at L or ending at U adds
        // nothing to them, so the wave visits only the rows some lane's masks
        // name (all of them if the masks do not cover the stencil), and a
        // column's (bf, al) is read only where its chord starts at L or ends
        // at U; then a connecting hull in the stencil's inner part
        const uint64_t need = masks ? (mL | mU) : ~0ull;
        const bool empty = L > U;
        float E1 = -DX_INF, S1 = DX_INF;
        for (int dy = -R; dy <= R; ++dy) {
            if (y + dy < 0 || y + dy >= P.ny) continue;
            if (!__any(masks ? ((need >> (dy + R)) & 1ull) != 0 : true)) continue;
            const int w = wd[dy < 0 ? -dy : dy];
            const int ri = ci + dy * SW;
            const float* hr = Hr + ro[dy < 0 ? -dy : dy] + w;  // hr[dx]: H[dx^2 + dy^2]
            const int yy = y + dy;
            for (int dx = -w; dx <= w; ++dx) {
                const float2 v = sab[ri + dx];
                const float hh = hr[dx];
                const bool eL = v.x - hh == L, eU = v.y + hh == U;
                const int xx = x + dx;
                if ((eL || eU) && v.x != DX_INF && xx >= 0 && xx < P.nx && yy >= 0 && yy < P.ny) {
                    const float4 e4 = gld(&P.ends[(int64_t)yy * P.nx + xx]);
                    E1 = eL ? mx(E1, e4.y + hh) : E1;
                    S1 = eU ? mn(S1, e4.z - hh) : S1;
                }
            }
        }
        // (the inner disk's rows from the centre out, where the half-widths
        // are largest; the wave stops once no lane still looks for a hull)
        // (a column whose chords span [E1, S1] is a hull if its largest-gap
        // bound, read here, is within 2 hh)
        bool hull = false;
        for (int i = 0; i <= 2 * R; ++i) {
            const int dy = (i & 1) ? -((i + 1) >> 1) : (i >> 1);  // 0, -1, 1, -2, 2, ...
            if (dy * dy > d2in || !__any(E1 < S1 && !hull && !empty)) break;
            if (y + dy < 0 || y + dy >= P.ny) continue;
            const int wf = wd[dy < 0 ? -dy : dy];
            int w = wf;
            while (w * w + dy * dy > d2in) --w;
            const int ri = ci + dy * SW;
            const float* hr = Hr + ro[dy < 0 ? -dy : dy] + wf;  // hr[dx]: H[dx^2 + dy^2]
            const int yy = y + dy;
            for (int dx = -w; dx <= w; ++dx) {
                const float2 v = sab[ri + dx];
                const float hh = hr[dx];
                const int xx = x + dx;
                if (!hull && v.x - hh <= E1 && v.y + hh >= S1 && v.x != DX_INF && xx >= 0 && xx < P.nx &&
                    yy >= 0 && yy < P.ny)
                    hull = 0.5f * gld(&P.gap[(int64_t)yy * P.nx + xx]) <= hh;
            }
        }
        const bool live = x < P.nx;
        const int64_t c = (int64_t)y * P.nx + x;
        const bool done = live && (empty || E1 >= S1 || hull);
        const int outn = (done && !empty) ? 1 : 0;
        int tot;
        const int pre = wave_excl_scan(outn, &tot);
        unsigned long long base = 0;
        if (lane == 0 && tot > 0) base = atomicAdd(&Q.hdr->bumpC, (unsigned long long)tot);
        base = __shfl(base, 0, 64);
        const unsigned long long end = base + (unsigned long long)tot;
        const bool ok = end <= (unsigned long long)P.cap;
        if (!ok && lane == 0) {
            note_need(P.hdr, end);
            set_error(P.hdr, DEXEL_ERR_WORKSPACE);
        }
        if (!live) continue;
        gst(&S.gen[c], (uint8_t)(done ? 0 : GEN_V0));
        if (!done) {
            // (E1 = -inf, S1 = +inf if no inner chord reaches L, U: the test
            // against V0 then takes the whole of (L, L0) and (U0, U) as gaps)
            gst(&S.lu[c], make_float4(L, E1 > L ? E1 : L, S1 < U ? S1 : U, U));
            push_overflow(Q, ST_K1, S.gbase + c);
            push_overflow(Q, ST_SOLB, S.gbase + c);
            continue;
        }
        gst(&P.offC[c], (int64_t)(base + pre));
        gst(&P.cntC[c], ok ? outn : 0);
        if (ok && outn) gst(&P.C[base + pre], make_float2(L, U));
    }
}

// The columns k_solid_dilate left, now with V0, one lane each (see above).
__global__ void __launch_bounds__(WG) k_solid_b(Pass Q) {
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_SOLB];
    if ((int64_t)blockIdx.x * WG >= cnt) return;
    const int i = blockIdx.x * WG + threadIdx.x;
    const bool live0 = i < cnt;
    const int64_t g = Q.ovf[(int64_t)ST_SOLB * Q.gcols + (live0 ? i : 0)];
    const int s = find_shape(Q, g);
    const Shape& S = Q.shapes[s];
    const OpParams P = make_op(Q, S);
    const int64_t c = g - Q.sbase[s];
    // (columns the row offset's replay settled have no V0 and gen[] 0)
    const bool live = live0 && gld(&S.gen[c]) == GEN_V0;
    const float4 lu = gld(&S.lu[c]);  // (L, E1, S1, U)
    // gaps of [L, E1] U V0 U [S1, U] inside [L, U]; more than GCW_MAX: give up
    int ng = 0;
    if (live) {
        const int n0 = gld(&P.cntA[c]);
        const float2* V = P.A + gld(&P.offA[c]);
        float prev = lu.y;
        for (int j = 0; j < n0 && ng <= GCW_MAX; ++j) {
            const float2 v = gld(&V[j]);
            if (v.x > prev) ++ng;
            prev = mx(prev, v.y);
        }
        if (lu.z > prev) ++ng;
    }
    const bool done = live && ng == 0;
    const bool cut = live && ng > 0 && ng <= GC_CAP;
    const bool wide = live && ng > GC_CAP && ng <= GCW_MAX;
    const int outn = done ? 1 : 0;
    int tot;
    const int pre = wave_excl_scan(outn, &tot);
    unsigned long long base = 0;
    if (threadIdx.x == 0 && tot > 0) base = atomicAdd(&Q.hdr->bumpC, (unsigned long long)tot);
    base = __shfl(base, 0, 64);
    const unsigned long long end = base + (unsigned long long)tot;
    const bool ok = end <= (unsigned long long)P.cap;
    if (!ok && threadIdx.x == 0) {
        note_need(P.hdr, end);
        set_error(P.hdr, DEXEL_ERR_WORKSPACE);
    }
    if (!live) return;
    if (cut || wide) {
        // the gap cut reads (L, U) and the range its gaps are taken from
        gst(&S.lu[c], make_float4(lu.x, lu.w, lu.y, lu.z));
        push_overflow(Q, cut ? ST_GAP : ST_GAPW, g);
        return;
    }
    if (!done) {
        gst(&S.gen[c], (uint8_t)(GEN_V0 | GEN_GENERAL));
        return;
    }
    gst(&P.offC[c], (int64_t)(base + pre));
    gst(&P.cntC[c], ok ? 1 : 0);
    if (ok) gst(&P.C[base + pre], make_float2(lu.x, lu.w));
}

__global__ void k_reset_k1(Pass Q) {
    if (threadIdx.x == 0) {
        Q.hdr->novf[ST_K1] = 0;
        Q.hdr->novf[ST_K1H] = 0;
    }
}

// Gap cut of one column: its open gaps (at most GC_CAP, sorted, in G) are cut
// by the chords of the stencil columns outside its own row (that row is in
// V0 already), visited ring by ring from the nearest.  A chord [A, B] removes
// [A, B] from a gap (l, u) it meets (A < u, B > l), leaving (l, A) if A > l
// and (B, u) if B < u.  Returns the number of gaps left (all of them now gaps
// of the union), or -1 if they outgrow GC_CAP or the visits the budget.
template <class L>
__device__ int gap_cut(const OpParams& P, int x, int y, const L& G, const L& T, int ng) {
    int budget = GC_BUDGET;
    // the current gap list and the one the next visit writes, swapped after
    // each visit (list views held by value, so nothing is address-taken)
    L cur = G, oth = T;
    bool in_g = true;
    auto visit = [&](int dx, int dy) -> bool {  // false: give up
        const int xx = x + dx, yy = y + dy;
        if (xx < 0 || xx >= P.nx || yy < 0 || yy >= P.ny) return true;
        const int d2 = dx * dx + dy * dy;
        if (d2 > P.d2max) return true;
        const int64_t cc = (int64_t)yy * P.nx + xx;
        if (gld(&P.gap[cc]) < 0.f) return true;
        const float h = gld(&P.H[d2]);
        const float4 e4 = gld(&P.ends[cc]);
        const float A0 = e4.x - h, B1 = e4.w + h;
        bool meet = false;
        for (int j = 0; j < ng; ++j) {
            const float2 g = cur.get(j);
            meet = meet || (A0 < g.y && B1 > g.x);
        }
        if (!meet) return true;
        if (--budget < 0) return false;
        const int64_t b = gld(&P.col_ptr[cc]);
        const int m = (int)(gld(&P.col_ptr[cc + 1]) - b);
        const float2* zc = P.z + b;
        int k = 0, nn = 0;
        for (int j = 0; j < ng; ++j) {
            const float2 g = cur.get(j);
            if (!(A0 < g.y && B1 > g.x)) {
                if (nn >= GC_CAP) return false;
                oth.set(nn++, g);
                continue;
            }
            // first chord ending above the gap's start (chord ends increase)
            int l = k, hh = m;
            while (l < hh) {
                const int mid = (l + hh) >> 1;
                if (gld(&zc[mid]).y + h > g.x) hh = mid; else l = mid + 1;
            }
            k = l;
            float cl = g.x;
            for (; k < m; ++k) {
                const float2 it = gld(&zc[k]);
                const float A = it.x - h;
                if (!(A < g.y)) break;
                if (A > cl) {
                    if (nn >= GC_CAP) return false;
                    oth.set(nn++, make_float2(cl, A));
                }
                cl = mx(cl, it.y + h);
                if (!(cl < g.y)) break;
            }
            if (cl < g.y) {
                if (nn >= GC_CAP) return false;
                oth.set(nn++, make_float2(cl, g.y));
            }
            // the next gap starts above this one: resume at the last chord seen
            if (k > 0) --k;
        }
        ng = nn;
        const L tmp = cur;
        cur = oth;
        oth = tmp;
        in_g = !in_g;
        return true;
    };
    for (int r = 1; r <= P.R && ng > 0; ++r) {
        for (int s = -1; s <= 1 && ng > 0; s += 2) {          // rows y -+ r
            for (int dx = -r; dx <= r && ng > 0; ++dx)
                if (!visit(dx, s * r)) return -1;
        }
        for (int s = -1; s <= 1 && ng > 0; s += 2) {          // columns x -+ r, rows in between
            for (int dy = -(r - 1); dy <= r - 1 && ng > 0; ++dy)
                if (dy != 0 && !visit(s * r, dy)) return -1;
        }
    }
    if (!in_g)
        for (int j = 0; j < ng; ++j) G.set(j, cur.get(j));
    return ng;
}

// The columns k_solid_b left to the gap cut, one lane each: build the gaps
// of V0 inside [lu.z, lu.w], cut them, and write [L, U] = [lu.x, lu.y] minus
// what is left; a column the cut gives up on is marked general.
__global__ void __launch_bounds__(WG) k_gap_cut(Pass Q) {
    __shared__ float2 lds[2 * GC_CAP * WG];
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_GAP];
    if ((int64_t)blockIdx.x * WG >= cnt) return;
    const int i = blockIdx.x * WG + threadIdx.x;
    const bool live = i < cnt;
    const int64_t g = live ? Q.ovf[(int64_t)ST_GAP * Q.gcols + i] : Q.ovf[(int64_t)ST_GAP * Q.gcols];
    const int s = find_shape(Q, g);
    const Shape& S = Q.shapes[s];
    const OpParams P = make_op(Q, S);
    const int64_t c = g - Q.sbase[s];
    int x, y;
    col_xy(P, c, &x, &y);
    const LdsList G{&lds[threadIdx.x], GC_CAP};
    const LdsList T{&lds[GC_CAP * WG + threadIdx.x], GC_CAP};
    const float4 lu = gld(&S.lu[c]);
    int ng = 0;
    if (live) {
        // the gaps of V0 inside [lu.z, lu.w], in order
        const int n0 = gld(&P.cntA[c]);
        const float2* V = P.A + gld(&P.offA[c]);
        // (at most GC_CAP of them, as k_solid_b counted)
        float prev = lu.z;
        for (int j = 0; j < n0 && ng >= 0; ++j) {
            const float2 v = gld(&V[j]);
            if (v.x > prev) {
                if (ng < GC_CAP) G.set(ng++, make_float2(prev, v.x)); else ng = -1;
            }
            prev = mx(prev, v.y);
        }
        if (ng >= 0 && lu.w > prev) {
            if (ng < GC_CAP) G.set(ng++, make_float2(prev, lu.w)); else ng = -1;
        }
        if (ng >= 0) ng = gap_cut(P, x, y, G, T, ng);
    }
    const bool ok1 = live && ng >= 0;
    const int outn = ok1 ? ng + 1 : 0;
    int tot;
    const int pre = wave_excl_scan(outn, &tot);
    unsigned long long base = 0;
    if (threadIdx.x == 0 && tot > 0) base = atomicAdd(&Q.hdr->bumpC, (unsigned long long)tot);
    base = __shfl(base, 0, 64);
    const unsigned long long end = base + (unsigned long long)tot;
    const bool ok = end <= (unsigned long long)P.cap;
    if (!ok && threadIdx.x == 0) {
        note_need(P.hdr, end);
        set_error(P.hdr, DEXEL_ERR_WORKSPACE);
    }
    if (!live) return;
    if (!ok1) {
        gst(&S.gen[c], (uint8_t)(GEN_V0 | GEN_GENERAL));
        return;
    }
    gst(&P.offC[c], (int64_t)(base + pre));
    gst(&P.cntC[c], ok ? outn : 0);
    if (!ok) return;
    float2* d = P.C + base + pre;
    float a = lu.x;  // the union is [L, U] minus the gaps left
    for (int j = 0; j < ng; ++j) {
        const float2 gp = G.get(j);
        gst(&d[j], make_float2(a, gp.x));
        a = gp.y;
    }
    gst(&d[ng], make_float2(a, lu.y));
}

// The columns k_solid_b found with more than GC_CAP (at most GCW_MAX) gaps,
// one wave each, one gap per lane: the gaps are disjoint and what a chord
// removes from one does not depend on the others, so each lane cuts its own
// gap with the other rows' chords (gap_cut on a one-gap list, the pieces it
// splits into at most GC_CAP), and lane 0 writes [L, U] minus the pieces
// left, in order.  A lane giving up leaves the column to the general kernels.
__global__ void __launch_bounds__(WG) k_gap_cut_wide(Pass Q) {
    __shared__ float2 lds[2 * GC_CAP * WG];
    __shared__ int pcnt[WG];
    if (Q.hdr->abort) return;
    const int cnt = Q.hdr->novf[ST_GAPW];
    const int lane = threadIdx.x;
    const LdsList G{&lds[lane], GC_CAP};
    const LdsList T{&lds[GC_CAP * WG + lane], GC_CAP};
    for (int e = blockIdx.x; e < cnt; e += gridDim.x) {
        const int64_t g = Q.ovf[(int64_t)ST_GAPW * Q.gcols + e];
        const int s = find_shape(Q, g);
        const Shape& S = Q.shapes[s];
        const OpParams P = make_op(Q, S);
        const int64_t c = g - Q.sbase[s];
        int x, y;
        col_xy(P, c, &x, &y);
        const float4 lu = gld(&S.lu[c]);
        // the gaps of V0 inside [lu.z, lu.w], in order (every lane walks V0;
        // lane k keeps gap k)
        const int n0 = gld(&P.cntA[c]);
        const float2* V = P.A + gld(&P.offA[c]);
        int k = 0;
        float prev = lu.z;
        float2 mine = make_float2(0.0f, 0.0f);
        for (int j = 0; j < n0; ++j) {
            const float2 v = gld(&V[j]);
            if (v.x > prev) {
                if (k == lane) mine = make_float2(prev, v.x);
                ++k;
            }
            prev = mx(prev, v.y);
        }
        if (lu.w > prev) {
            if (k == lane) mine = make_float2(prev, lu.w);
            ++k;
        }
        const bool have = lane < k;
        int np = 0;
        if (have) {
            G.set(0, mine);
            np = gap_cut(P, x, y, G, T, 1);
        }
        const bool fail = __any(have && np < 0) || k > GCW_MAX;
        pcnt[lane] = have ? np : 0;
        __syncthreads();  // every lane's pieces and count are written
        if (lane == 0) {
            if (fail) {
                gst(&S.gen[c], (uint8_t)(GEN_V0 | GEN_GENERAL));
            } else {
                int tot = 1;
                for (int l = 0; l < k; ++l) tot += pcnt[l];
                const unsigned long long base = atomicAdd(&Q.hdr->bumpC, (unsigned long long)tot);
                const unsigned long long end = base + (unsigned long long)tot;
                const bool ok = end <= (unsigned long long)Q.cap;
                if (!ok) {
                    note_need(Q.hdr, end);
                    set_error(Q.hdr, DEXEL_ERR_WORKSPACE);
                }
                gst(&P.offC[c], (int64_t)base);
                gst(&P.cntC[c], ok ? tot : 0);
                if (ok) {
                    float2* d = P.C + base;
                    float a = lu.x;  // the union is [L, U] minus the pieces left
                    int o = 0;
                    for (int l = 0; l < k; ++l)
                        for (int i = 0; i < pcnt[l]; ++i) {
                            const float2 gp = lds[i * WG + l];  // lane l's list, element i
                            gst(&d[o++], make_float2(a, gp.x));
                            a = gp.y;
                        }
                    gst(&d[o], make_float2(a, lu.y));
                }
            }
        }
        __syncthreads();  // lane 0 has read the lists before they are reused
    }
}

// need[c] of every column of the shapes with fast path `mode`: NEED_UNION if
// the column is general itself, NEED_SEEDS if a general column lies within R
// rows of it (its seeds and intersection feed that column's y union),
// NEED_ROW if one lies within 2R rows (its row offset feeds those
// intersections).  One wave per tile of the fast path (THIN_TX columns x TY
// rows), one lane per column: the distance from each of the tile's rows to
// the nearest general row of its column comes from one scan down and one up
// over the tile's rows and 2R rows beyond them, so each gen[] entry is read
// about twice instead of once per row within 2R.
template <int TY>
__global__ void __launch_bounds__(WG) k_fast_spread(Pass Q, int mode) {
    if (Q.hdr->abort) return;
    const int64_t t = blockIdx.x;
    int lo = 0, hi = Q.nshapes;  // the last shape whose tiles start at or before t
    while (hi - lo > 1) {
        const int m = (lo + hi) >> 1;
        if (Q.shapes[m].tbase <= t) lo = m; else hi = m;
    }
    const Shape& S = Q.shapes[lo];
    if (S.fast != mode) return;
    const int ntx = (S.nx + THIN_TX - 1) / THIN_TX;
    const int64_t tl = t - S.tbase;
    const int x = (int)(tl % ntx) * THIN_TX + (int)threadIdx.x;
    const int y0 = (int)(tl / ntx) * TY;
    if (x >= S.nx) return;
    const int R2 = 2 * S.R;
    auto general = [&](int y) { return (gld(&S.gen[(int64_t)y * S.nx + x]) & GEN_GENERAL) != 0; };
    constexpr int FAR = 1 << 30;
    // downwards: the last general row at or above each tile row
    int last = -FAR;
    for (int y = max(0, y0 - R2); y < y0; ++y)
        if (general(y)) last = y;
    int gmask = 0;       // the tile's general rows
    int dup[TY];         // distance to the last general row at or above
#pragma unroll
    for (int k = 0; k < TY; ++k) {
        const int y = y0 + k;
        const bool g = y < S.ny && general(y);
        gmask |= g ? 1 << k : 0;
        last = g ? y : last;
        dup[k] = y - last;
    }
    // upwards: the next general row at or below, and the bits
    int next = FAR;
    for (int y = min(S.ny - 1, y0 + TY - 1 + R2); y >= y0 + TY; --y)
        if (general(y)) next = y;
#pragma unroll
    for (int k = TY - 1; k >= 0; --k) {
        const int y = y0 + k;
        if ((gmask >> k) & 1) next = y;
        const int d = min(dup[k], next - y);
        const int bits = d == 0 ? NEED_UNION | NEED_SEEDS | NEED_ROW
                       : d <= S.R ? NEED_SEEDS | NEED_ROW
                       : d <= R2 ? NEED_ROW : 0;
        if (y < S.ny) gst(&S.need[(int64_t)y * S.nx + x], (uint8_t)bits);
    }
}

// ---------------------------------------------------------------------------
// compaction into the output CSR, status
// ---------------------------------------------------------------------------

// One wave per 64 global columns (waves never straddle shapes).  Writes the
// shape's output column pointers always and its intervals when they fit.
__global__ void __launch_bounds__(WG) k_copy_out(Pass Q) {
    if (Q.hdr->abort) return;
    const Place pl = place_block(Q);
    const Shape& S = Q.shapes[pl.s];
    const int64_t base = S.scanC[0];
    const int64_t total = S.scanC[S.ncols] - base;
    const int64_t zb = S.out_zoff ? *S.out_zoff : 0;
    const bool fits = zb + total <= S.out_cap;
    // the intermediate grid of a chain lives in the workspace: its size
    // counts toward the call's capacity need whether or not it fits
    if (pl.c == 0 && S.out_is_intermediate) note_need(Q.hdr, (unsigned long long)(zb + total));
    if (!fits && pl.c == 0) {
        if (S.out_is_intermediate) {
            set_error(Q.hdr, DEXEL_ERR_WORKSPACE);
        } else {
            atomicCAS(&Q.shape_status[S.index], 0, DEXEL_ERR_CAPACITY);
        }
    }
    if (!pl.valid) return;
    const int64_t o = S.scanC[pl.c] - base;
    S.out_col_ptr[pl.c] = o;
    if (pl.c == S.ncols - 1) S.out_col_ptr[S.ncols] = total;
    if (!fits) return;
    const int n = S.cntC[pl.c];
    const float2* src = Q.C + S.offC[pl.c];
    float2* dst = S.out_z + zb + o;
    for (int i = 0; i < n; ++i) dst[i] = src[i];
}

__global__ void k_init_call(WsHeader* h, int32_t* shape_status, int nitems) {
    if (threadIdx.x == 0) {
        h->status = 0;
        h->abort = 0;
        h->need_cap = 0;
        h->nseg_out = -1;
        h->nseeds = 0;
        h->bumpA = h->bumpI = h->bumpC = h->arena = 0;
    }
    if (threadIdx.x < NSTAGE) h->novf[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < nitems; i += blockDim.x) shape_status[i] = 0;
}

__global__ void k_init_pass(WsHeader* h) {
    if (threadIdx.x < NSTAGE) h->novf[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        // the first pass's use of the per-column lists and the arena counts
        // toward the call's capacity need before the counters restart
        unsigned long long m = h->need_cap;
        m = m > h->bumpA ? m : h->bumpA;
        m = m > h->bumpI ? m : h->bumpI;
        m = m > h->bumpC ? m : h->bumpC;
        m = m > h->arena ? m : h->arena;
        h->need_cap = m;
        h->bumpA = h->bumpI = h->bumpC = h->arena = 0;
        h->nseeds = 0;
    }
}

__global__ void k_put_shapes(Shape* dst, ShapeChunk ch) {
    const int i = threadIdx.x;
    if (i < ch.n) dst[ch.first + i] = ch.s[i];
}

__global__ void k_put_f32(float* dst, F32Chunk ch) {
    for (int i = threadIdx.x; i < ch.n; i += blockDim.x) dst[ch.first + i] = ch.v[i];
}

__global__ void k_put_i64(int64_t* dst, I64Chunk ch) {
    for (int i = threadIdx.x; i < ch.n; i += blockDim.x) dst[ch.first + i] = ch.v[i];
}

// Input checks of the first pass.  Always: col_ptr[0] = 0, nondecreasing,
// col_ptr[ncols] = nseg (reads past the arrays are impossible afterwards).
// With `validate`: every interval finite, z_in <= z_out, strictly separated.
__global__ void __launch_bounds__(WG) k_check_input(Pass Q, int validate) {
    const Place pl = place_block(Q);
    if (!pl.valid) return;
    const Shape& S = Q.shapes[pl.s];
    const int64_t c = pl.c;
    const int64_t v = S.col_ptr[c], w = S.col_ptr[c + 1];
    bool bad = false;
    if (c == 0 && v != 0) bad = true;
    if (w < v || v < 0) bad = true;
    if (S.nseg >= 0 && w > S.nseg) bad = true;
    if (c == S.ncols - 1 && S.nseg >= 0 && w != S.nseg) bad = true;
    if (!bad && validate) {
        float prev = -DX_INF;
        for (int64_t i = v; i < w; ++i) {
            const float2 iv = S.z[i];
            if (!(iv.x == iv.x) || !(iv.y == iv.y) || isinf(iv.x) || isinf(iv.y) || iv.x > iv.y)
                bad = true;
            if (i > v && !(iv.x > prev)) bad = true;
            prev = iv.y;
        }
    }
    if (bad) set_error(Q.hdr, DEXEL_ERR_NOT_CANONICAL);
}

// Per shape: after its last pass write the caller's status and count; after
// an intermediate pass record where its result starts in the chain buffer.
__global__ void k_finish(Pass Q, int64_t* zbase) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Q.nshapes) return;
    const Shape& S = Q.shapes[s];
    const int hst = Q.hdr->status;
    const int st = hst ? hst : Q.shape_status[S.index];
    int64_t n = -1;
    if (st == 0 || st == DEXEL_ERR_CAPACITY) n = S.scanC[S.ncols] - S.scanC[0];
    if (S.out_is_intermediate) {
        if (!hst) zbase[S.index] = S.scanC[0];
        return;
    }
    if (s == 0) Q.hdr->nseg_out = n;
    if (S.last_pass) {
        if (S.out_nseg) *S.out_nseg = n;
        if (S.out_status) *S.out_status = st;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_put_shapes(Shape* dst, const Shape* host, int n, hipStream_t s) {
    for (int first = 0; first < n; first += DESC_CHUNK) {
        ShapeChunk ch;
        ch.n = n - first < DESC_CHUNK ? n - first : DESC_CHUNK;
        ch.first = first;
        for (int i = 0; i < ch.n; ++i) ch.s[i] = host[first + i];
        hipLaunchKernelGGL(k_put_shapes, dim3(1), dim3(64), 0, s, dst, ch);
    }
    return hipGetLastError();
}

hipError_t launch_put_i64(int64_t* dst, const int64_t* host, int n, hipStream_t s) {
    for (int first = 0; first < n; first += I64_CHUNK) {
        I64Chunk ch;
        ch.n = n - first < I64_CHUNK ? n - first : I64_CHUNK;
        ch.first = first;
        for (int i = 0; i < ch.n; ++i) ch.v[i] = host[first + i];
        hipLaunchKernelGGL(k_put_i64, dim3(1), dim3(256), 0, s, dst, ch);
    }
    return hipGetLastError();
}

hipError_t launch_put_f32(float* dst, const float* host, int n, hipStream_t s) {
    for (int first = 0; first < n; first += F32_CHUNK) {
        F32Chunk ch;
        ch.n = n - first < F32_CHUNK ? n - first : F32_CHUNK;
        ch.first = first;
        for (int i = 0; i < ch.n; ++i) ch.v[i] = host[first + i];
        hipLaunchKernelGGL(k_put_f32, dim3(1), dim3(256), 0, s, dst, ch);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-column Boolean operations (CSG)
// ---------------------------------------------------------------------------
//
// Regularised union, intersection and difference of two canonical grids,
// column by column (CSG in dexel space, Sec. 2 item (3); the shell of Sec. 4
// "3D Printing" is the difference of a dilation and an erosion).  One lane
// per column sweeps both sorted lists once.  Input intervals of zero length
// have no interior and are skipped; touching result pieces are one interval;
// no piece of zero length is emitted.  Endpoints are copied, never computed.
// The sweep runs once to count (then a scan) and once to write.

template <int OP, bool WRITE>
__device__ int csg_column(const CsgArgs& A, int64_t c, float2* dst) {
    const int64_t a0 = gld(&A.a_ptr[c]), a1 = gld(&A.a_ptr[c + 1]);
    const int64_t b0 = gld(&A.b_ptr[c]), b1 = gld(&A.b_ptr[c + 1]);
    const float2* az = A.a_z + a0;
    const float2* bz = A.b_z + b0;
    const int na = (int)(a1 - a0), nb = (int)(b1 - b0);
    const float2 none = make_float2(DX_INF, DX_INF);
    int k = 0;
    auto put = [&](float lo, float hi) {
        if (WRITE) gst(&dst[k], make_float2(lo, hi));
        ++k;
    };
    if (OP == CSG_UNION) {
        // merge by start; a piece starting at or before the open interval's
        // end extends it
        int i = 0, j = 0;
        float2 va = na > 0 ? gld(&az[0]) : none, vb = nb > 0 ? gld(&bz[0]) : none;
        float2 cur = make_float2(0.f, 0.f);
        bool open = false;
        while (i < na || j < nb) {
            const bool takeA = j >= nb || (i < na && va.x <= vb.x);
            const float2 v = takeA ? va : vb;
            if (takeA) {
                ++i;
                va = i < na ? gld(&az[i]) : none;
            } else {
                ++j;
                vb = j < nb ? gld(&bz[j]) : none;
            }
            if (!(v.x < v.y)) continue;
            if (open && v.x <= cur.y) {
                cur.y = mx(cur.y, v.y);
            } else {
                if (open) put(cur.x, cur.y);
                cur = v;
                open = true;
            }
        }
        if (open) put(cur.x, cur.y);
    } else if (OP == CSG_INTERSECT) {
        // overlap of the current pair; the piece ending first is done
        int i = 0, j = 0;
        float2 va = na > 0 ? gld(&az[0]) : none, vb = nb > 0 ? gld(&bz[0]) : none;
        while (i < na && j < nb) {
            const float lo = mx(va.x, vb.x), hi = mn(va.y, vb.y);
            if (lo < hi) put(lo, hi);
            if (va.y < vb.y) {
                ++i;
                va = i < na ? gld(&az[i]) : none;
            } else {
                ++j;
                vb = j < nb ? gld(&bz[j]) : none;
            }
        }
    } else {
        // A minus B: each interval of A, cut by the intervals of B over it
        int j = 0;
        for (int i = 0; i < na; ++i) {
            const float2 va = gld(&az[i]);
            if (!(va.x < va.y)) continue;
            float lo = va.x;
            while (j < nb && gld(&bz[j]).y <= lo) ++j;
            for (int q = j; q < nb; ++q) {
                const float2 vb = gld(&bz[q]);
                if (!(vb.x < va.y)) break;
                if (!(vb.x < vb.y)) continue;
                if (vb.x > lo) put(lo, vb.x);
                lo = mx(lo, vb.y);
            }
            if (lo < va.y) put(lo, va.y);
        }
    }
    return k;
}

template <int OP>
__device__ __forceinline__ int csg_count(const CsgArgs& A, int64_t c) {
    return csg_column<OP, false>(A, c, nullptr);
}

constexpr int CSG_T = 256;

__global__ void __launch_bounds__(CSG_T) k_csg_count(CsgArgs A) {
    const int64_t c = (int64_t)blockIdx.x * CSG_T + threadIdx.x;
    if (c >= A.ncols) return;
    int n;
    if (A.op == CSG_UNION) n = csg_count<CSG_UNION>(A, c);
    else if (A.op == CSG_INTERSECT) n = csg_count<CSG_INTERSECT>(A, c);
    else n = csg_count<CSG_DIFFERENCE>(A, c);
    gst(&A.cnt[c], n);
}

// Output column pointers always; intervals when the total fits the capacity;
// column 0's lane writes the end pointer, the count and the status.
__global__ void __launch_bounds__(CSG_T) k_csg_write(CsgArgs A) {
    const int64_t c = (int64_t)blockIdx.x * CSG_T + threadIdx.x;
    if (c >= A.ncols) return;
    const int64_t total = gld(&A.scan[A.ncols]);
    const int64_t off = gld(&A.scan[c]);
    gst(&A.out_ptr[c], off);
    if (c == 0) {
        gst(&A.out_ptr[A.ncols], total);
        gst(A.out_nseg, total);
        gst(A.out_status, total > A.cap ? (int32_t)DEXEL_ERR_CAPACITY : (int32_t)DEXEL_OK);
    }
    if (total > A.cap) return;
    float2* dst = A.out_z + off;
    if (A.op == CSG_UNION) csg_column<CSG_UNION, true>(A, c, dst);
    else if (A.op == CSG_INTERSECT) csg_column<CSG_INTERSECT, true>(A, c, dst);
    else csg_column<CSG_DIFFERENCE, true>(A, c, dst);
}

hipError_t launch_csg(const CsgArgs& a, hipStream_t s) {
    const unsigned nb = (unsigned)((a.ncols + CSG_T - 1) / CSG_T);
    hipLaunchKernelGGL(k_init_call, dim3(1), dim3(256), 0, s, a.hdr, (int32_t*)nullptr, 0);
    hipLaunchKernelGGL(k_csg_count, dim3(nb), dim3(CSG_T), 0, s, a);
    hipError_t e = scan_counts(a.cnt, a.ncols, a.bsum, a.scan, a.hdr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_csg_write, dim3(nb), dim3(CSG_T), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// canonical form of per-column interval lists
// ---------------------------------------------------------------------------
//
// A dexel column is a set of closed z-intervals (Sec. 3.1, "Dexel
// Representation"); its canonical form, the input form of every offset,
// lists that set sorted, with overlapping or touching intervals joined.
// The first tier gives one lane per column a canonical LDS list of
// CANON_CAP slots and inserts the column's intervals into it in input order
// (the union does not depend on the order).  A column whose list runs out
// is left to the sorting tier: one lane copies the column's intervals into
// the scratch array at the column's own input offset, sorts them in place
// by (start, end) (heapsort), and sweeps them once.  The count pass also
// checks the input: column pointers inside [0, nseg] and non-decreasing,
// and every interval finite with start <= end.

constexpr int CANON_CAP = 32;

__device__ __forceinline__ bool canon_ok(float2 v) {
    return v.x <= v.y && __builtin_isfinite(v.x) && __builtin_isfinite(v.y);
}

__device__ __forceinline__ bool canon_less(float2 a, float2 b) {
    return a.x < b.x || (a.x == b.x && a.y < b.y);
}

// Heapsort of s[0..m) by (start, end), in place.
__device__ void canon_heapsort(float2* s, int64_t m) {
    auto sift = [&](int64_t i, int64_t end) {
        const float2 v = s[i];
        while (true) {
            int64_t ch = 2 * i + 1;
            if (ch >= end) break;
            float2 cv = s[ch];
            if (ch + 1 < end) {
                const float2 c2 = s[ch + 1];
                if (canon_less(cv, c2)) {
                    ++ch;
                    cv = c2;
                }
            }
            if (!canon_less(v, cv)) break;
            s[i] = cv;
            i = ch;
        }
        s[i] = v;
    };
    for (int64_t i = m / 2 - 1; i >= 0; --i) sift(i, m);
    for (int64_t end = m - 1; end > 0; --end) {
        const float2 t = s[0];
        s[0] = s[end];
        s[end] = t;
        sift(0, end);
    }
}

template <bool WRITE>
__global__ void __launch_bounds__(WG) k_canon(CanonArgs A) {
    __shared__ float2 lds[CANON_CAP * WG];
    const int64_t c = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (c >= A.ncols) return;
    // after an error of the count pass the scan did not run: write nothing
    if (WRITE && A.hdr->abort) return;
    const int64_t b = gld(&A.in_ptr[c]), e = gld(&A.in_ptr[c + 1]);
    if (!WRITE && (b < 0 || e < b || e > A.nseg || (c == 0 && b != 0) ||
                   (c == A.ncols - 1 && e != A.nseg))) {
        set_error(A.hdr, DEXEL_ERR_INVALID);
        gst(&A.cnt[c], 0);
        return;
    }
    LdsList U{&lds[threadIdx.x], CANON_CAP};
    int n = 0;
    bool bad = false, over = false;
    for (int64_t i = b; i < e; ++i) {
        const float2 v = gld(&A.in_z[i]);
        if (!canon_ok(v)) {
            bad = true;
            break;
        }
        const int m = lv_insert(U, n, v.x, v.y);
        if (m < 0) {
            over = true;
            break;
        }
        n = m;
    }
    if (!WRITE) {
        if (bad) {
            set_error(A.hdr, DEXEL_ERR_INVALID);
            gst(&A.cnt[c], 0);
        } else if (over) {
            const int k = atomicAdd(&A.hdr->novf[0], 1);   // the sorting tier counts it
            gst(&A.longc[k], (int32_t)c);
        } else {
            gst(&A.cnt[c], n);
        }
        return;
    }
    const int64_t total = gld(&A.scan[A.ncols]);
    const int64_t off = gld(&A.scan[c]);
    gst(&A.out_ptr[c], off);
    if (c == 0) {
        gst(&A.out_ptr[A.ncols], total);
        gst(A.out_nseg, total);
    }
    if (total > A.cap || over) return;
    for (int i = 0; i < n; ++i) gst(&A.out_z[off + i], U.get(i));
}

// The sorting tier: one lane per listed column, a fixed grid walking the
// list.  The count pass copies, checks and sorts; the write pass sweeps the
// sorted copy again.
template <bool WRITE>
__global__ void __launch_bounds__(WG) k_canon_long(CanonArgs A) {
    const int nl = A.hdr->novf[0];
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < nl; i += (int64_t)gridDim.x * WG) {
        if (WRITE && A.hdr->abort) return;
        const int64_t c = gld(&A.longc[i]);
        const int64_t b = gld(&A.in_ptr[c]), e = gld(&A.in_ptr[c + 1]);
        float2* s = A.sorted + b;
        const int64_t m = e - b;
        if (m > INT32_MAX) {   // a count must fit the per-column int32 counts
            set_error(A.hdr, DEXEL_ERR_UNSUPPORTED);
            if (!WRITE) gst(&A.cnt[c], 0);
            continue;
        }
        if (!WRITE) {
            bool bad = false;
            for (int64_t k = 0; k < m; ++k) {
                const float2 v = gld(&A.in_z[b + k]);
                bad |= !canon_ok(v);
                s[k] = v;
            }
            if (bad) {
                set_error(A.hdr, DEXEL_ERR_INVALID);
                gst(&A.cnt[c], 0);
                continue;
            }
            canon_heapsort(s, m);
        }
        const int64_t off = WRITE ? gld(&A.scan[c]) : 0;
        const bool put = WRITE && gld(&A.scan[A.ncols]) <= A.cap;
        int64_t n = 0;
        float2 cur = make_float2(0.f, 0.f);
        for (int64_t k = 0; k < m; ++k) {
            const float2 v = s[k];
            if (n > 0 && v.x <= cur.y) {
                cur.y = mx(cur.y, v.y);
            } else {
                if (n > 0 && put) gst(&A.out_z[off + n - 1], cur);
                cur = v;
                ++n;
            }
        }
        if (n > 0 && put) gst(&A.out_z[off + n - 1], cur);
        if (!WRITE) gst(&A.cnt[c], (int32_t)n);
    }
}

// The device status: an error of the count pass, else capacity.
__global__ void k_canon_status(CanonArgs A) {
    const int st = A.hdr->status;
    A.out_status[0] = st != 0 ? st : (A.scan[A.ncols] > A.cap ? (int32_t)DEXEL_ERR_CAPACITY : (int32_t)DEXEL_OK);
}

hipError_t launch_canonicalize(const CanonArgs& a, hipStream_t s) {
    const unsigned nb = (unsigned)((a.ncols + WG - 1) / WG);
    const unsigned nlong = nb < 256u ? nb : 256u;
    hipLaunchKernelGGL(k_init_call, dim3(1), dim3(256), 0, s, a.hdr, (int32_t*)nullptr, 0);
    hipLaunchKernelGGL(k_canon<false>, dim3(nb), dim3(WG), 0, s, a);
    hipLaunchKernelGGL(k_canon_long<false>, dim3(nlong), dim3(WG), 0, s, a);
    hipError_t e = scan_counts(a.cnt, a.ncols, a.bsum, a.scan, a.hdr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_canon<true>, dim3(nb), dim3(WG), 0, s, a);
    hipLaunchKernelGGL(k_canon_long<true>, dim3(nlong), dim3(WG), 0, s, a);
    hipLaunchKernelGGL(k_canon_status, dim3(1), dim3(1), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dexelisation of analytic primitives
// ---------------------------------------------------------------------------
//
// The rays of a dexel structure are the z-parallel lines through the cell
// centres (x + 0.5, y + 0.5) (Sec. 1; Sec. 3.1, "Dexel Representation").  A
// ball (centre c, radius R) meets the ray of a cell when rho2 = (x + 0.5 -
// cx)^2 + (y + 0.5 - cy)^2 is below R^2, in [cz - h, cz + h] with
// h = sqrt(R^2 - rho2); a box [a, b] meets the rays of the cells with
// ceil(ax - 0.5) <= x <= floor(bx - 0.5) (and likewise in y) in [az, bz].
// Chord ends are computed in float64, each operation rounded once (no
// contraction into fused multiply-adds), then rounded once to float32 and
// merged into the column's canonical list (overlapping or touching
// intervals join).  One lane per column; each block first culls the
// primitives against its cells (below).  Run once to count, once to write.

// The chord of primitive record q on the ray of cell (x, y); false if none
// (and *bad set for an unknown kind).
__device__ bool dex_chord(const double* q, int x, int y, float* lo, float* hi, bool* bad) {
#pragma clang fp contract(off)
    const double kind = q[0];
    const double px = (double)x + 0.5, py = (double)y + 0.5;
    if (kind == 0.0) {
        const double dx = px - q[1], dy = py - q[2];
        const double rho2 = dx * dx + dy * dy;
        const double R2 = q[4] * q[4];
        if (!(rho2 < R2)) return false;
        const double h = sqrt(R2 - rho2);
        *lo = (float)(q[3] - h);
        *hi = (float)(q[3] + h);
        return true;
    }
    if (kind == 1.0) {
        if (!((double)x >= ceil(q[1] - 0.5) && (double)x <= floor(q[4] - 0.5) &&
              (double)y >= ceil(q[2] - 0.5) && (double)y <= floor(q[5] - 0.5)))
            return false;
        *lo = (float)q[3];
        *hi = (float)q[6];
        return true;
    }
    *bad = true;
    return false;
}

// May primitive record q hit a cell centre of the box [xlo, xhi] x [ylo, yhi]
// (integer cell indices)?  Conservative, with the lane test's own float
// operations: a ball is out when the squared float distance from its centre
// to the nearest centre coordinate, in x or in y, is not below R^2 (rounding
// is monotone, so every lane's rho2 is then not below R^2 either); a box is
// out when its cell range misses the block's.  Unknown kinds are kept (the
// lanes report them).
__device__ bool dex_may_hit(const double* q, int xlo, int xhi, int ylo, int yhi) {
#pragma clang fp contract(off)
    const double kind = q[0];
    if (kind == 0.0) {
        const double R2 = q[4] * q[4];
        const double pxl = (double)xlo + 0.5, pxh = (double)xhi + 0.5;
        const double pyl = (double)ylo + 0.5, pyh = (double)yhi + 0.5;
        const double cx = q[1], cy = q[2];
        const double dx = cx < pxl ? pxl - cx : (cx > pxh ? cx - pxh : 0.0);
        const double dy = cy < pyl ? pyl - cy : (cy > pyh ? cy - pyh : 0.0);
        return dx * dx < R2 && dy * dy < R2;
    }
    if (kind == 1.0)
        return floor(q[4] - 0.5) >= (double)xlo && ceil(q[1] - 0.5) <= (double)xhi &&
               floor(q[5] - 0.5) >= (double)ylo && ceil(q[2] - 0.5) <= (double)yhi;
    return true;
}

// One block of DEX_WG lanes per tile of 64 x 4 cells (256 x 1 when the grid
// has fewer than 4 rows), one lane per column.  The primitives are taken
// DEX_WG at a time (the next chunk's records are loaded while the current
// one is tested): each lane tests one against the tile's cell box, the
// survivors' records are compacted into LDS (ballot, per-wave counts,
// prefix), and every lane then runs the exact test on the survivors only,
// in primitive order.
//
// Two tiers: the first pass over all tiles keeps each lane's list in
// DEX_CAPL LDS slots (a small footprint, so several blocks share a CU); a
// tile where some lane would need more is appended to a list (its lanes
// write nothing) and redone whole by the second tier with DEX_CAP slots,
// where running out is an error.  Both tiers compute every lane the same
// way, so the redone lanes that had fit write what they would have written.
constexpr int DEX_WG = 256;
constexpr int DEX_CAPL = 12;
using DexList = LV<DEX_WG>;

__device__ __forceinline__ double dex_pick(const double* v, int i) {
    return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]);
}

// Record k in the ray frame: for rays along axis k (0 = x, 1 = y, 2 = z) the
// grid's lateral axes are (k + 1) mod 3 and (k + 2) mod 3 and the intervals
// lie along k, so the corners (and a ball's centre) are reordered to
// (lateral u, lateral v, along); a ball's radius stays in place.
__device__ __forceinline__ void dex_load(const DexArgs& A, int k, double* q) {
    if (k >= A.nprims) {
#pragma unroll
        for (int i = 0; i < 7; ++i) q[i] = 0.0;
        return;
    }
    const double* r = A.prims + 7 * (int64_t)k;
    double v[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) v[i] = r[i];
    if (A.axis == 2) {
#pragma unroll
        for (int i = 0; i < 7; ++i) q[i] = v[i];
        return;
    }
    const int u = A.axis == 0 ? 1 : 2, w = A.axis == 0 ? 2 : 0;
    q[0] = v[0];
    q[1] = dex_pick(v + 1, u);
    q[2] = dex_pick(v + 1, w);
    q[3] = dex_pick(v + 1, A.axis);
    const bool box = v[0] == 1.0;
    q[4] = box ? dex_pick(v + 4, u) : v[4];
    q[5] = box ? dex_pick(v + 4, w) : v[5];
    q[6] = box ? dex_pick(v + 4, A.axis) : v[6];
}

__host__ __device__ __forceinline__ int dex_tile_h(int ny) { return ny >= 4 ? 4 : 1; }

// Lane t of tile `tile`: its column's canonical list in U (n intervals);
// returns false when the list ran past U.cap.  Every lane of the block must
// call it (it synchronises the block).
__device__ bool dex_tile(const DexArgs& A, int64_t tile, DexList U, double (*rec)[DEX_WG], int* wsum,
                         int* x_out, int* y_out, bool* live_out, int* n_out, bool* bad) {
    const int t = threadIdx.x, w = t / WG, l = t % WG;
    const int th = dex_tile_h(A.ny), tw = DEX_WG / th;
    const int ntx = (A.nx + tw - 1) / tw;
    const int bx = (int)(tile % ntx), by = (int)(tile / ntx);
    const int xlo = bx * tw, ylo = by * th;
    const int xhi = min(xlo + tw, A.nx) - 1, yhi = min(ylo + th, A.ny) - 1;
    const int x = xlo + t % tw, y = ylo + t / tw;
    const bool live = x < A.nx && y < A.ny;
    int n = 0;
    bool over = false;
    double q[7], qn[7];
    dex_load(A, t, q);
    for (int base = 0; base < A.nprims; base += DEX_WG) {
        const bool keep = base + t < A.nprims && dex_may_hit(q, xlo, xhi, ylo, yhi);
        dex_load(A, base + DEX_WG + t, qn);
        const unsigned long long mask = __ballot(keep);
        __syncthreads();  // the previous chunk's survivors have been read
        if (l == 0) wsum[w] = __popcll(mask);
        __syncthreads();
        int pos = __popcll(mask & ((1ull << l) - 1ull)), nsurv = 0;
#pragma unroll
        for (int i = 0; i < DEX_WG / WG; ++i) {
            pos += i < w ? wsum[i] : 0;
            nsurv += wsum[i];
        }
        if (keep) {
#pragma unroll
            for (int i = 0; i < 7; ++i) rec[i][pos] = q[i];
        }
        __syncthreads();
        if (live && !over) {
            for (int j = 0; j < nsurv; ++j) {
                double p[7];
#pragma unroll
                for (int i = 0; i < 7; ++i) p[i] = rec[i][j];
                float lo, hi;
                if (!dex_chord(p, x, y, &lo, &hi, bad)) continue;
                const int m = lv_insert(U, n, lo, hi);
                if (m < 0) {
                    over = true;
                    break;
                }
                n = m;
            }
        }
#pragma unroll
        for (int i = 0; i < 7; ++i) q[i] = qn[i];
    }
    *x_out = x;
    *y_out = y;
    *live_out = live;
    *n_out = n;
    return !over;
}

// The outputs of one lane: its count (count pass), or its CSR offset and
// intervals (write pass).  `fits`: the list is whole.
template <bool WRITE>
__device__ void dex_emit(const DexArgs& A, int64_t c, DexList U, int n, bool fits, bool bad,
                         bool own_ptr) {
    if (!WRITE) {
        gst(&A.cnt[c], fits ? n : 0);
        return;
    }
    // after an error of the count pass the scan did not run: write nothing
    if (A.hdr->abort) return;
    const int64_t total = gld(&A.scan[A.ncols]);
    const int64_t off = gld(&A.scan[c]);
    if (own_ptr) {
        gst(&A.out_ptr[c], off);
        if (c == 0) {
            gst(&A.out_ptr[A.ncols], total);
            gst(A.out_nseg, total);
        }
    }
    if (total > A.cap || !fits || bad) return;
    for (int i = 0; i < n; ++i) gst(&A.out_z[off + i], U.get(i));
}

// First tier: one block per tile.  The count pass appends the tiles that
// ran out of slots to A.spill (count in hdr->novf[0]); the write pass finds
// the same tiles running out and leaves their intervals to the second tier.
template <bool WRITE>
__global__ void __launch_bounds__(DEX_WG) k_dexelize(DexArgs A) {
    __shared__ float2 lds[DEX_CAPL * DEX_WG];
    __shared__ double rec[7][DEX_WG];    // the chunk's survivors, by field
    __shared__ int wsum[DEX_WG / WG];
    DexList U{&lds[threadIdx.x], DEX_CAPL};
    int x, y, n;
    bool live, bad = false;
    const bool fits = dex_tile(A, blockIdx.x, U, rec, wsum, &x, &y, &live, &n, &bad);
    const bool spilled = __syncthreads_or(live && !fits);
    if (!WRITE && spilled && threadIdx.x == 0) {
        const int k = atomicAdd(&A.hdr->novf[0], 1);
        gst(&A.spill[k], (int32_t)blockIdx.x);
    }
    if (!live) return;
    if (bad) set_error(A.hdr, DEXEL_ERR_INVALID);
    const int64_t c = (int64_t)y * A.nx + x;
    if (!WRITE && !fits) return;    // the second tier counts it
    dex_emit<WRITE>(A, c, U, n, fits, bad, true);
}

// Second tier: the tiles listed by the first, DEX_CAP slots per lane; a
// fixed grid walks the list.
template <bool WRITE>
__global__ void __launch_bounds__(DEX_WG) k_dexelize_full(DexArgs A) {
    __shared__ float2 lds[DEX_CAP * DEX_WG];
    __shared__ double rec[7][DEX_WG];
    __shared__ int wsum[DEX_WG / WG];
    const int ntiles = A.hdr->novf[0];
    DexList U{&lds[threadIdx.x], DEX_CAP};
    for (int i = blockIdx.x; i < ntiles; i += gridDim.x) {
        const int64_t tile = gld(&A.spill[i]);
        int x, y, n;
        bool live, bad = false;
        const bool fits = dex_tile(A, tile, U, rec, wsum, &x, &y, &live, &n, &bad);
        if (live) {
            if (bad) set_error(A.hdr, DEXEL_ERR_INVALID);
            if (!fits) set_error(A.hdr, DEXEL_ERR_UNSUPPORTED);
            dex_emit<WRITE>(A, (int64_t)y * A.nx + x, U, n, fits, bad, false);
        }
        __syncthreads();   // LDS is reused by the next tile
    }
}

// The device status: an error of the count pass (unknown kind, a column past
// DEX_CAP), else capacity.
__global__ void k_dexelize_status(DexArgs A) {
    const int st = A.hdr->status;
    const int64_t total = A.scan[A.ncols];
    A.out_status[0] = st != 0 ? st : (total > A.cap ? (int32_t)DEXEL_ERR_CAPACITY : (int32_t)DEXEL_OK);
}

int64_t dexelize_tiles(int32_t nx, int32_t ny) {
    const int th = dex_tile_h(ny), tw = DEX_WG / th;
    return (int64_t)((nx + tw - 1) / tw) * ((ny + th - 1) / th);
}

hipError_t launch_dexelize(const DexArgs& a, hipStream_t s) {
    const unsigned nb = (unsigned)dexelize_tiles(a.nx, a.ny);
    const unsigned nfull = nb < 1024u ? nb : 1024u;
    hipLaunchKernelGGL(k_init_call, dim3(1), dim3(256), 0, s, a.hdr, (int32_t*)nullptr, 0);
    hipLaunchKernelGGL(k_dexelize<false>, dim3(nb), dim3(DEX_WG), 0, s, a);
    hipLaunchKernelGGL(k_dexelize_full<false>, dim3(nfull), dim3(DEX_WG), 0, s, a);
    hipError_t e = scan_counts(a.cnt, a.ncols, a.bsum, a.scan, a.hdr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dexelize<true>, dim3(nb), dim3(DEX_WG), 0, s, a);
    hipLaunchKernelGGL(k_dexelize_full<true>, dim3(nfull), dim3(DEX_WG), 0, s, a);
    hipLaunchKernelGGL(k_dexelize_status, dim3(1), dim3(1), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init_call(WsHeader* hdr, int32_t* shape_status, int nitems, hipStream_t s) {
    hipLaunchKernelGGL(k_init_call, dim3(1), dim3(256), 0, s, hdr, shape_status, nitems);
    return hipGetLastError();
}

hipError_t launch_init_pass(WsHeader* hdr, hipStream_t s) {
    hipLaunchKernelGGL(k_init_pass, dim3(1), dim3(64), 0, s, hdr);
    return hipGetLastError();
}

hipError_t launch_check_input(const Pass& p, int validate, hipStream_t s) {
    hipLaunchKernelGGL(k_check_input, dim3((unsigned)(p.gcols / WG)), dim3(WG), 0, s, p, validate);
    return hipGetLastError();
}

// Kernel variants: per-lane LDS list capacities of K1, K1b (each of two
// lists), K2 and K3.  Larger lists replay fewer columns; smaller ones leave
// room for more resident waves per CU (the default, variant 0, has small
// lists; variant 1 large ones for shapes with long lists).  The host picks
// one per call (default, forced, or autotuned).
template <int C1, int C1B, int C2, int C3>
static hipError_t pass_variant(const Pass& p, hipStream_t s, hipEvent_t* ev) {
    const unsigned nb = (unsigned)(p.gcols / WG);
    const dim3 g(nb), b(WG), gf(FALLBACK_BLOCKS);
    hipError_t e = hipSuccess;
#define DX_MARK(i) \
    if (ev && (e = hipEventRecord(ev[i], s)) != hipSuccess) return e
    DX_MARK(0);
    hipLaunchKernelGGL(k_col_gaps, dim3((unsigned)(p.gcols / (WG / GAP_LANES))), b, 0, s, p);
    DX_MARK(1);
    if (p.ndirect) {
        hipLaunchKernelGGL(k_direct1<D1_CAP>, g, b, 0, s, p);
        hipLaunchKernelGGL((k_direct<DT, DT_CAP>), dim3(TEAM_BLOCKS), b, 0, s, p, (int)ST_DIRT, (int)ST_DIRW);
        hipLaunchKernelGGL((k_direct<64, CAP_Z>), gf, b, 0, s, p, (int)ST_DIRW, -1);
    }
    DX_MARK(2);
    if (p.ntiles > 0 && p.nthin > 0) {
        hipLaunchKernelGGL(k_thin_erode, dim3((unsigned)p.ntiles), dim3(THIN_T), (unsigned)p.thin_lds, s, p);
        hipLaunchKernelGGL(k_fast_spread<THIN_TY>, dim3((unsigned)p.ntiles), b, 0, s, p, (int)FAST_THIN);
    }
    DX_MARK(3);
    if (p.ntiles > 0 && p.nsolid > 0)
        hipLaunchKernelGGL(k_solid_dilate, dim3((unsigned)p.ntiles), dim3(THIN_T), (unsigned)p.solid_lds, s, p);
    DX_MARK(4);
    Pass p1 = p;
    p1.k1_round = 1;
    hipLaunchKernelGGL(k_row_offset<C1>, g, b, 0, s, p1);
    DX_MARK(5);
    hipLaunchKernelGGL(k_row_offset_fb, g, b, 0, s, p);
    hipLaunchKernelGGL(k_row_offset_heavy, gf, b, 0, s, p);
    DX_MARK(6);
    if (p.ntiles > 0 && p.nsolid > 0) {
        hipLaunchKernelGGL(k_solid_b, g, b, 0, s, p);
        hipLaunchKernelGGL(k_gap_cut, g, b, 0, s, p);
        hipLaunchKernelGGL(k_gap_cut_wide, dim3(GAPW_BLOCKS), b, 0, s, p);
        hipLaunchKernelGGL(k_fast_spread<SOLID_TY>, dim3((unsigned)p.ntiles), b, 0, s, p, (int)FAST_SOLID);
        // the row offsets the general columns' stages still need
        hipLaunchKernelGGL(k_reset_k1, dim3(1), dim3(64), 0, s, p);
        Pass p2 = p;
        p2.k1_round = 2;
        hipLaunchKernelGGL(k_row_offset<C1>, g, b, 0, s, p2);
        hipLaunchKernelGGL(k_row_offset_fb, g, b, 0, s, p);
        hipLaunchKernelGGL(k_row_offset_heavy, gf, b, 0, s, p);
    }
    DX_MARK(7);
    hipLaunchKernelGGL(k_neighbour<C1B>, g, b, 0, s, p);
    DX_MARK(8);
    hipLaunchKernelGGL(k_neighbour_fb, g, b, 0, s, p);
    hipLaunchKernelGGL(k_neighbour_heavy, gf, b, 0, s, p);
    DX_MARK(9);
    hipLaunchKernelGGL(k_seeds<C2>, g, b, 0, s, p);
    DX_MARK(10);
    hipLaunchKernelGGL(k_seeds_fb<C2>, g, b, 0, s, p);
    hipLaunchKernelGGL(k_seeds_heavy<C2>, gf, b, 0, s, p);
    DX_MARK(11);
    hipLaunchKernelGGL(k_union<C3>, g, b, 0, s, p);
    DX_MARK(12);
    hipLaunchKernelGGL(k_union_fb, g, b, 0, s, p);
    hipLaunchKernelGGL(k_union_heavy, gf, b, 0, s, p);
    DX_MARK(13);
    e = scan_counts(p.cntC_g, p.gcols, p.bsum, p.scanC_g, p.hdr, s);
    if (e != hipSuccess) return e;
    DX_MARK(14);
    hipLaunchKernelGGL(k_copy_out, g, b, 0, s, p);
    DX_MARK(15);
#undef DX_MARK
    return hipGetLastError();
}

int prepare_kernels(int max_lds) {
    // the largest dynamic LDS both tiled kernels accept, from the device's
    // limit down; a refused setting is cleared from the runtime's error state
    for (int b = max_lds; b > 65536; b -= 16384) {
        if (hipFuncSetAttribute((const void*)k_thin_erode, hipFuncAttributeMaxDynamicSharedMemorySize, b) ==
                hipSuccess &&
            hipFuncSetAttribute((const void*)k_solid_dilate, hipFuncAttributeMaxDynamicSharedMemorySize, b) ==
                hipSuccess)
            return b;
        (void)hipGetLastError();
    }
    return 65536;
}

hipError_t launch_pass(const Pass& p, hipStream_t s, hipEvent_t* ev, int variant) {
    switch (variant) {
        case 1: return pass_variant<40, 32, 48, 32>(p, s, ev);
        case 2: return pass_variant<40, 16, 16, 16>(p, s, ev);
        case 3: return pass_variant<24, 12, 12, 8>(p, s, ev);
        default: return pass_variant<40, 12, 12, 8>(p, s, ev);
    }
}

hipError_t launch_finish(const Pass& p, int64_t* zbase, hipStream_t s) {
    const unsigned nb = (unsigned)((p.nshapes + 63) / 64);
    hipLaunchKernelGGL(k_finish, dim3(nb), dim3(64), 0, s, p, zbase);
    return hipGetLastError();
}

}  // namespace dexel
