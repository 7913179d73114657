// Host side of the libdexel C ABI (see include/dexel.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/dexel.h"
#include "dexel_internal.h"

using dexel::WsHeader;

struct dexel_ctx {
    int device = 0;
    std::string err;
    // Optional per-stage timing: HIP events recorded on the call's stream at
    // the stage boundaries of every pass, read back by dexel_profile_read.
    bool profile = false;
    std::vector<hipEvent_t> pool;
    std::vector<std::vector<hipEvent_t>> pending;
    double acc[dexel::NPROF] = {0};
    int64_t passes = 0;
    // Kernel variant: forced (>= 0) or chosen per batch signature by dexel_autotune.
    int forced_variant = -1;
    std::map<uint64_t, int> tuned;
    // LDS bytes one workgroup may take (bounds the tiled fast paths' radii)
    int max_lds = 65536;
    // device address of this device's static scratch (dexel_offset_noalloc)
    void* scratch = nullptr;
};

namespace {

constexpr float kMaxRadius = 250.0f;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

dexel_status fail(dexel_ctx* ctx, dexel_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return s;
}

uint32_t float_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

// R = floor(r), d2max = floor(r^2) with r^2 formed exactly in double.
void radius_params(float r, int* R, int* d2max) {
    const double rd = (double)r;
    *R = (int)std::floor(rd);
    *d2max = (int)std::floor(rd * rd);
}

// Workspace layout of one call (a batch of items; a single op is a batch of one).
struct Layout {
    size_t hdr, shape_status, zbase, shapes1, shapes2, sbase1, sbase2, luts;
    size_t gap, ends, offA, cntA, offI, cntI, offB, cntB, loB, hullB, offC, cntC, scanC, gen, need, lu;
    size_t A, I, B, tagB, C, ovf, arena, arena_tag, bsum, mid_ptr, mid_z, total;
    int64_t gcols1, gcols2, gmax, mid_cols;
    int seed_slot;
    std::vector<size_t> lut_off;  // per item: byte offset of its radius table (shared per radius)
};

struct ItemInfo {
    int64_t ncols;
    int R, d2max;
    bool chain;
    uint32_t rbits;  // the radius' float bits: items of one radius share its table
};

int64_t pad64(int64_t v) { return (v + 63) / 64 * 64; }

// Thresholds of the choice of evaluation (see enqueue_batch).
constexpr double kDirectKmin = 6.0;
constexpr double kDirectItems = 24000.0;
constexpr double kSolidKmin = 8.0;

bool is_chain(int op) { return op == DEXEL_OPEN || op == DEXEL_CLOSE; }

Layout make_layout(const std::vector<ItemInfo>& items, int64_t cap) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t n = items.size();
    L.gcols1 = L.gcols2 = L.mid_cols = 0;
    for (const auto& it : items) {
        L.gcols1 += pad64(it.ncols);
        if (it.chain) {
            L.gcols2 += pad64(it.ncols);
            L.mid_cols += it.ncols + 1;
        }
    }
    L.gmax = L.gcols1 > L.gcols2 ? L.gcols1 : L.gcols2;
    const size_t g = (size_t)L.gmax, cp = (size_t)cap;
    int rmax = 0;
    for (const auto& it : items) rmax = it.R > rmax ? it.R : rmax;
    L.seed_slot = rmax >= dexel::SEED_WIDE_R &&
                          (long long)g * dexel::SEED_SLOT_WIDE * 9 <= dexel::SEED_WIDE_BYTES
                      ? dexel::SEED_SLOT_WIDE
                      : dexel::SEED_SLOT;
    L.hdr = take(256);
    L.shape_status = take(4 * n);
    L.zbase = take(8 * n);
    L.shapes1 = take(sizeof(dexel::Shape) * n);
    L.shapes2 = take(sizeof(dexel::Shape) * n);
    L.sbase1 = take(8 * (n + 1));
    L.sbase2 = take(8 * (n + 1));
    L.lut_off.resize(n);
    std::map<uint32_t, size_t> lut_of_radius;
    for (size_t i = 0; i < n; ++i) {
        auto f = lut_of_radius.find(items[i].rbits);
        if (f != lut_of_radius.end()) {
            L.lut_off[i] = f->second;
        } else {
            L.lut_off[i] = take(sizeof(float) * (size_t)(items[i].d2max + 1));
            lut_of_radius[items[i].rbits] = L.lut_off[i];
        }
    }
    L.luts = n ? L.lut_off[0] : o;
    L.gap = take(4 * g);
    L.ends = take(16 * g);
    L.offA = take(8 * g);
    L.cntA = take(4 * g);
    L.offI = take(8 * g);
    L.cntI = take(4 * g);
    L.offB = take(8 * g);
    L.cntB = take(4 * g);
    L.loB = take(4 * g);
    L.hullB = take(32 * g);
    L.offC = take(8 * g);
    L.cntC = take(4 * g);
    L.scanC = take(8 * (g + 1));
    L.gen = take(g);
    L.need = take(g);
    L.lu = take(16 * g);
    L.A = take(8 * cp);
    L.I = take(8 * cp);
    L.B = take(8 * g * (size_t)L.seed_slot);
    L.tagB = take(g * (size_t)L.seed_slot);
    L.C = take(8 * cp);
    L.ovf = take(4 * g * dexel::NSTAGE);
    L.arena = take(8 * cp);
    L.arena_tag = take(cp);
    L.bsum = take(8 * ((g + 1023) / 1024 + 2));
    L.mid_ptr = take(8 * (size_t)L.mid_cols);
    L.mid_z = take(L.gcols2 ? 8 * cp : 0);
    L.total = o;
    return L;
}

int64_t default_cap(const dexel_grid_view* in) {
    const int64_t ncols = (int64_t)in->nx * in->ny;
    return in->nseg + 2 * ncols + 1024;
}

dexel_status check_view(dexel_ctx* ctx, const dexel_grid_view* in) {
    if (!in) return fail(ctx, DEXEL_ERR_INVALID, "null input view");
    if (in->nx <= 0 || in->ny <= 0) return fail(ctx, DEXEL_ERR_INVALID, "nx and ny must be >= 1");
    if ((int64_t)in->nx * in->ny >= ((int64_t)1 << 31) - 64)
        return fail(ctx, DEXEL_ERR_UNSUPPORTED, "nx * ny must be below 2^31");
    if (in->nseg < 0) return fail(ctx, DEXEL_ERR_INVALID, "nseg must be >= 0");
    if (!in->col_ptr) return fail(ctx, DEXEL_ERR_INVALID, "null input col_ptr");
    if (in->nseg > 0 && !in->z) return fail(ctx, DEXEL_ERR_INVALID, "null input z");
    if (((uintptr_t)in->z) % 8 != 0) return fail(ctx, DEXEL_ERR_INVALID, "input z must be 8-byte aligned");
    return DEXEL_OK;
}

dexel_status check_radius(dexel_ctx* ctx, float r) {
    if (!std::isfinite(r) || r < 0.0f) return fail(ctx, DEXEL_ERR_INVALID, "r must be finite and >= 0");
    if (r > kMaxRadius) return fail(ctx, DEXEL_ERR_UNSUPPORTED, "r > 250 is not supported");
    return DEXEL_OK;
}

dexel_status check_out(dexel_ctx* ctx, const dexel_grid_view* in, const dexel_grid_out* out) {
    if (!out) return fail(ctx, DEXEL_ERR_INVALID, "null output");
    if (out->nx != in->nx || out->ny != in->ny)
        return fail(ctx, DEXEL_ERR_INVALID, "output grid size differs from input");
    if (out->cap_seg < 0) return fail(ctx, DEXEL_ERR_INVALID, "cap_seg must be >= 0");
    if (!out->col_ptr || !out->nseg_out || !out->status)
        return fail(ctx, DEXEL_ERR_INVALID, "null output pointer");
    if (out->cap_seg > 0 && !out->z) return fail(ctx, DEXEL_ERR_INVALID, "null output z");
    if (((uintptr_t)out->z) % 8 != 0) return fail(ctx, DEXEL_ERR_INVALID, "output z must be 8-byte aligned");
    if ((const void*)out->z == (const void*)in->z && in->nseg > 0 && out->cap_seg > 0)
        return fail(ctx, DEXEL_ERR_INVALID, "input and output alias");
    if ((const void*)out->col_ptr == (const void*)in->col_ptr)
        return fail(ctx, DEXEL_ERR_INVALID, "input and output alias");
    return DEXEL_OK;
}

// Half-width table H[d2] = float(sqrt(double(r)^2 - d2)), d2 = 0..floor(r^2),
// computed on the host per call and uploaded through kernel arguments (no
// host buffer outlives the call, nothing is allocated).
std::vector<float> half_widths(float r, int d2max) {
    std::vector<float> h((size_t)d2max + 1);
    const double r2 = (double)r * (double)r;
    for (int d2 = 0; d2 <= d2max; ++d2) h[d2] = (float)std::sqrt(r2 - (double)d2);
    return h;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ctx, DEXEL_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

dexel_status check_items(dexel_ctx* ctx, int32_t n, const dexel_batch_item* items,
                         std::vector<ItemInfo>* info, bool outputs) {
    if (n < 0 || (n > 0 && !items)) return fail(ctx, DEXEL_ERR_INVALID, "bad item list");
    info->clear();
    for (int32_t i = 0; i < n; ++i) {
        const dexel_batch_item& it = items[i];
        dexel_status st;
        if (outputs) {
            if ((st = check_view(ctx, &it.in)) != DEXEL_OK) return st;
        } else {
            if (it.in.nx <= 0 || it.in.ny <= 0 || it.in.nseg < 0)
                return fail(ctx, DEXEL_ERR_INVALID, "bad grid size");
            if ((int64_t)it.in.nx * it.in.ny >= ((int64_t)1 << 31) - 64)
                return fail(ctx, DEXEL_ERR_UNSUPPORTED, "nx * ny must be below 2^31");
        }
        if ((st = check_radius(ctx, it.r)) != DEXEL_OK) return st;
        if (it.op < DEXEL_DILATE || it.op > DEXEL_CLOSE) return fail(ctx, DEXEL_ERR_INVALID, "unknown op");
        if (outputs && (st = check_out(ctx, &it.in, &it.out)) != DEXEL_OK) return st;
        ItemInfo ii;
        ii.ncols = (int64_t)it.in.nx * it.in.ny;
        radius_params(it.r, &ii.R, &ii.d2max);
        ii.chain = is_chain(it.op);
        ii.rbits = float_bits(it.r);
        info->push_back(ii);
    }
    return DEXEL_OK;
}

int64_t batch_default_cap(int32_t n, const dexel_batch_item* items) {
    int64_t c = 1024;
    for (int32_t i = 0; i < n; ++i) c += default_cap(&items[i].in) - 1024;
    return c;
}

// Largest internal capacity whose layout fits in ws_bytes (0 if none).
int64_t cap_for_bytes(const std::vector<ItemInfo>& info, size_t ws_bytes) {
    int64_t lo = 1, hi = 1;
    if (make_layout(info, lo).total > ws_bytes) return 0;
    while (make_layout(info, hi).total <= ws_bytes && hi < ((int64_t)1 << 40)) hi *= 2;
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (make_layout(info, mid).total <= ws_bytes) lo = mid; else hi = mid;
    }
    return lo;
}

// Signature of a batch for the autotune cache: item count, grid sizes,
// ops, radii and the order of magnitude of each input size.
uint64_t batch_signature(int32_t n, const dexel_batch_item* items) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    mix((uint64_t)n);
    for (int32_t i = 0; i < n; ++i) {
        mix((uint64_t)items[i].in.nx);
        mix((uint64_t)items[i].in.ny);
        mix((uint64_t)items[i].op);
        mix((uint64_t)float_bits(items[i].r));
        int lg = 0;
        for (int64_t v = items[i].in.nseg; v > 0; v >>= 1) ++lg;
        mix((uint64_t)lg);
    }
    return h;
}

int pick_variant(dexel_ctx* ctx, int32_t n, const dexel_batch_item* items) {
    if (ctx->forced_variant >= 0) return ctx->forced_variant;
    auto it = ctx->tuned.find(batch_signature(n, items));
    return it == ctx->tuned.end() ? 0 : it->second;
}

// Enqueue a batch (already argument-checked) into a workspace of ws_bytes.
dexel_status enqueue_batch(dexel_ctx* ctx, int32_t n, const dexel_batch_item* items,
                           const std::vector<ItemInfo>& info, void* ws, size_t ws_bytes,
                           hipStream_t s, uint32_t flags, int variant) {
    if (n == 0) return DEXEL_OK;
    if (!ws) return fail(ctx, DEXEL_ERR_INVALID, "null workspace");
    if (((uintptr_t)ws) % kAlign != 0) return fail(ctx, DEXEL_ERR_INVALID, "workspace must be 256-byte aligned");
    const int64_t cap = cap_for_bytes(info, ws_bytes);
    if (cap <= 0) return fail(ctx, DEXEL_ERR_WORKSPACE, "workspace smaller than the minimum layout");
    const Layout L = make_layout(info, cap);
    char* w = (char*)ws;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DEXEL_ERR_HIP, "hipSetDevice failed");

    std::vector<dexel::Shape> sh1, sh2;
    std::vector<int64_t> base1, base2;
    int64_t g1 = 0, g2 = 0, mid = 0;
    for (int32_t i = 0; i < n; ++i) {
        const dexel_batch_item& it = items[i];
        const ItemInfo& ii = info[i];
        const int ops[2] = {it.op == DEXEL_ERODE || it.op == DEXEL_OPEN ? 1 : 0,
                            it.op == DEXEL_CLOSE ? 1 : 0};
        auto fill = [&](dexel::Shape& S, int64_t gbase) {
            std::memset(&S, 0, sizeof(S));
            S.nx = it.in.nx;
            S.ny = it.in.ny;
            S.ncols = ii.ncols;
            S.gbase = gbase;
            S.R = ii.R;
            S.d2max = ii.d2max;
            S.index = i;
            S.H = (const float*)(w + L.lut_off[i]);
            S.gap = (float*)(w + L.gap) + gbase;
            S.ends = (float4*)(w + L.ends) + gbase;
            S.offA = (int64_t*)(w + L.offA) + gbase;
            S.cntA = (int32_t*)(w + L.cntA) + gbase;
            S.offI = (int64_t*)(w + L.offI) + gbase;
            S.cntI = (int32_t*)(w + L.cntI) + gbase;
            S.offB = (int64_t*)(w + L.offB) + gbase;
            S.cntB = (int32_t*)(w + L.cntB) + gbase;
            S.loB = (int32_t*)(w + L.loB) + gbase;
            S.hullB = (float4*)(w + L.hullB) + 2 * gbase;
            S.offC = (int64_t*)(w + L.offC) + gbase;
            S.cntC = (int32_t*)(w + L.cntC) + gbase;
            S.scanC = (int64_t*)(w + L.scanC) + gbase;
            S.gen = (uint8_t*)(w + L.gen) + gbase;
            S.need = (uint8_t*)(w + L.need) + gbase;
            S.lu = (float4*)(w + L.lu) + gbase;
        };
        // How each pass is evaluated (every choice gives the same result,
        // bit for bit; DEXEL_FLAG_GENERAL keeps the staged kernels throughout):
        // * directly (FAST_DIRECT) when the input is fragmented and the
        //   stencil small: at least DIRECT_KMIN items per column, R at most
        //   DIRECT_RMAX, and at most DIRECT_ITEMS chords per output column
        //   (stencil columns x items per column, one more for an erosion's
        //   gaps).  The second pass of a chain is judged by the call's input.
        // * else, where the tiles fit the LDS, an erosion by the thin-column
        //   filter first, and a dilation of an input with at least SOLID_KMIN
        //   items per column by the single-interval test first (on sparser
        //   input most columns fail the test, which then only adds work);
        // * else by the staged kernels alone.
        const double kbar = (double)it.in.nseg / (double)std::max<int64_t>(ii.ncols, 1);
        int64_t sten = 0;
        for (int dy = -ii.R; dy <= ii.R; ++dy) {
            int64_t w = (int64_t)std::sqrt((double)(ii.d2max - dy * dy));
            while (w > 0 && w * w + dy * dy > ii.d2max) --w;
            while ((w + 1) * (w + 1) + dy * dy <= ii.d2max) ++w;
            sten += 2 * w + 1;
        }
        auto fast_of = [&](int erode) {
            if (flags & DEXEL_FLAG_GENERAL) return (int32_t)dexel::FAST_NONE;
            if (ii.R <= dexel::DIRECT_RMAX && kbar >= kDirectKmin &&
                (double)sten * (kbar + erode) <= kDirectItems)
                return (int32_t)dexel::FAST_DIRECT;
            const int lds = erode ? dexel::thin_lds_bytes(ii.R, ii.d2max)
                                  : dexel::solid_lds_bytes(ii.R, ii.d2max);
            if (ii.R > dexel::THIN_RMAX || lds > ctx->max_lds) return (int32_t)dexel::FAST_NONE;
            if (!erode && kbar < kSolidKmin) return (int32_t)dexel::FAST_NONE;
            return (int32_t)(erode ? dexel::FAST_THIN : dexel::FAST_SOLID);
        };
        dexel::Shape a;
        fill(a, g1);
        a.col_ptr = it.in.col_ptr;
        a.z = (const float2*)it.in.z;
        a.nseg = it.in.nseg;
        a.erode = ops[0];
        a.fast = fast_of(a.erode);
        if (ii.chain) {
            int64_t* mptr = (int64_t*)(w + L.mid_ptr) + mid;
            a.out_col_ptr = mptr;
            a.out_z = (float2*)(w + L.mid_z);
            a.out_zoff = a.scanC;  // the shape's base in the pass's result scan
            a.out_cap = cap;
            a.out_is_intermediate = 1;
            dexel::Shape b;
            fill(b, g2);
            b.col_ptr = mptr;
            b.z = (const float2*)(w + L.mid_z);
            b.zoff = (const int64_t*)(w + L.zbase) + i;
            b.nseg = -1;
            b.erode = ops[1];
            b.fast = fast_of(b.erode);
            b.out_col_ptr = it.out.col_ptr;
            b.out_z = (float2*)it.out.z;
            b.out_cap = it.out.cap_seg;
            b.last_pass = 1;
            b.out_nseg = it.out.nseg_out;
            b.out_status = it.out.status;
            sh2.push_back(b);
            base2.push_back(g2);
            g2 += pad64(ii.ncols);
            mid += ii.ncols + 1;
        } else {
            a.out_col_ptr = it.out.col_ptr;
            a.out_z = (float2*)it.out.z;
            a.out_cap = it.out.cap_seg;
            a.last_pass = 1;
            a.out_nseg = it.out.nseg_out;
            a.out_status = it.out.status;
        }
        sh1.push_back(a);
        base1.push_back(g1);
        g1 += pad64(ii.ncols);
    }
    base1.push_back(g1);
    base2.push_back(g2);
    // tiles of the shapes with a tiled fast path, numbered in shape order
    auto tile_bases = [](std::vector<dexel::Shape>& sh, dexel::Pass* q) {
        int64_t t = 0;
        int32_t bt = 0, bs = 0;
        for (auto& S : sh) {
            S.tbase = t;
            if (S.fast == dexel::FAST_DIRECT) q->ndirect = 1;
            if (S.fast == dexel::FAST_NONE || S.fast == dexel::FAST_DIRECT) continue;
            const bool thin = S.fast == dexel::FAST_THIN;
            const int ty = thin ? dexel::THIN_TY : dexel::SOLID_TY;
            t += (int64_t)((S.nx + dexel::THIN_TX - 1) / dexel::THIN_TX) * ((S.ny + ty - 1) / ty);
            if (thin) {
                bt = std::max(bt, (int32_t)dexel::thin_lds_bytes(S.R, S.d2max));
                q->nthin = 1;
            } else {
                bs = std::max(bs, (int32_t)dexel::solid_lds_bytes(S.R, S.d2max));
                q->nsolid = 1;
            }
        }
        q->ntiles = t;
        q->thin_lds = bt;
        q->solid_lds = bs;
    };

    auto make_pass = [&](size_t shapes_off, size_t sbase_off, int nsh, int64_t gcols) {
        dexel::Pass q{};
        q.shapes = (const dexel::Shape*)(w + shapes_off);
        q.sbase = (const int64_t*)(w + sbase_off);
        q.nshapes = nsh;
        q.gcols = gcols;
        q.hdr = (WsHeader*)(w + L.hdr);
        q.shape_status = (int32_t*)(w + L.shape_status);
        q.cap = cap;
        q.A = (float2*)(w + L.A);
        q.I = (float2*)(w + L.I);
        q.B = (float2*)(w + L.B);
        q.tagB = (uint8_t*)(w + L.tagB);
        q.seed_slot = L.seed_slot;
        q.C = (float2*)(w + L.C);
        q.cntC_g = (int32_t*)(w + L.cntC);
        q.scanC_g = (int64_t*)(w + L.scanC);
        q.ovf = (int32_t*)(w + L.ovf);
        q.arena = (float2*)(w + L.arena);
        q.arena_tag = (uint8_t*)(w + L.arena_tag);
        q.bsum = (int64_t*)(w + L.bsum);
        return q;
    };
    dexel::Pass p1 = make_pass(L.shapes1, L.sbase1, (int)sh1.size(), g1);
    dexel::Pass p2 = make_pass(L.shapes2, L.sbase2, (int)sh2.size(), g2);
    tile_bases(sh1, &p1);
    tile_bases(sh2, &p2);
    int64_t* zbase = (int64_t*)(w + L.zbase);

    HIP_TRY(dexel::launch_init_call(p1.hdr, p1.shape_status, n, s));
    std::set<size_t> filled;  // shared radius tables already copied
    for (int32_t i = 0; i < n; ++i) {
        if (!filled.insert(L.lut_off[i]).second) continue;
        const std::vector<float> h = half_widths(items[i].r, info[i].d2max);
        HIP_TRY(dexel::launch_put_f32((float*)(w + L.lut_off[i]), h.data(), (int)h.size(), s));
    }
    HIP_TRY(dexel::launch_put_shapes((dexel::Shape*)(w + L.shapes1), sh1.data(), (int)sh1.size(), s));
    HIP_TRY(dexel::launch_put_i64((int64_t*)(w + L.sbase1), base1.data(), (int)base1.size(), s));
    if (!sh2.empty()) {
        HIP_TRY(dexel::launch_put_shapes((dexel::Shape*)(w + L.shapes2), sh2.data(), (int)sh2.size(), s));
        HIP_TRY(dexel::launch_put_i64((int64_t*)(w + L.sbase2), base2.data(), (int)base2.size(), s));
    }
    HIP_TRY(dexel::launch_check_input(p1, (flags & DEXEL_FLAG_VALIDATE) ? 1 : 0, s));

    auto run_pass = [&](const dexel::Pass& q) -> dexel_status {
        hipEvent_t* ev = nullptr;
        if (ctx->profile) {
            std::vector<hipEvent_t> group;
            for (int i = 0; i <= dexel::NPROF; ++i) {
                hipEvent_t e;
                if (!ctx->pool.empty()) {
                    e = ctx->pool.back();
                    ctx->pool.pop_back();
                } else {
                    HIP_TRY(hipEventCreate(&e));
                }
                group.push_back(e);
            }
            ctx->pending.push_back(group);
            ev = ctx->pending.back().data();
        }
        HIP_TRY(dexel::launch_pass(q, s, ev, variant));
        HIP_TRY(dexel::launch_finish(q, zbase, s));
        return DEXEL_OK;
    };
    dexel_status st = run_pass(p1);
    if (st != DEXEL_OK) return st;
    if (!sh2.empty()) {
        HIP_TRY(dexel::launch_init_pass(p2.hdr, s));
        st = run_pass(p2);
        if (st != DEXEL_OK) return st;
    }
    return DEXEL_OK;
}

dexel_status sync_status(dexel_ctx* ctx, hipStream_t s, int32_t n, const dexel_batch_item* items) {
    HIP_TRY(hipStreamSynchronize(s));
    for (int32_t i = 0; i < n; ++i) {
        int32_t st = 0;
        HIP_TRY(hipMemcpy(&st, items[i].out.status, sizeof(st), hipMemcpyDeviceToHost));
        if (st != 0) {
            char buf[96];
            std::snprintf(buf, sizeof(buf), "device status %d (item %d)", st, (int)i);
            ctx->err = buf;
            return (dexel_status)st;
        }
    }
    return DEXEL_OK;
}

}  // namespace

extern "C" {

// Workspace of dexel_offset_noalloc: one copy on every GPU the library runs
// on, held until the process ends.  On the host `noalloc_scratch` is only a
// stand-in for the symbol: host code uses the device address that
// hipGetSymbolAddress returns for the current device (one lookup per device,
// kept in noalloc_ptr), never the array's own name.
static __device__ __align__(256) unsigned char noalloc_scratch[DEXEL_NOALLOC_SCRATCH_BYTES];

static std::mutex noalloc_mu;
static std::map<int, void*> noalloc_ptr;

// Address of `device`'s scratch; `device` must be current.
static void* noalloc_scratch_of(int device) {
    std::lock_guard<std::mutex> lock(noalloc_mu);
    auto it = noalloc_ptr.find(device);
    if (it != noalloc_ptr.end()) return it->second;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || !p) return nullptr;
    noalloc_ptr[device] = p;
    return p;
}

dexel_status dexel_ctx_create(int device, dexel_ctx** ctx) {
    if (!ctx) return DEXEL_ERR_INVALID;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DEXEL_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return DEXEL_ERR_HIP;
    void* scratch = noalloc_scratch_of(device);
    if (!scratch) return DEXEL_ERR_HIP;
    dexel_ctx* c = new dexel_ctx();
    c->device = device;
    c->scratch = scratch;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->max_lds = lds;
    c->max_lds = dexel::prepare_kernels(c->max_lds);
    *ctx = c;
    return DEXEL_OK;
}

void dexel_ctx_destroy(dexel_ctx* ctx) {
    if (!ctx) return;
    for (auto& g : ctx->pending)
        for (hipEvent_t e : g) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    delete ctx;
}

dexel_status dexel_workspace_size(dexel_ctx* ctx, const dexel_grid_view* in, float r, int32_t op,
                                  int64_t cap_hint, size_t* bytes) {
    if (!ctx || !bytes) return DEXEL_ERR_INVALID;
    if (!in) return fail(ctx, DEXEL_ERR_INVALID, "null input view");
    dexel_batch_item it{};
    it.in = *in;
    it.r = r;
    it.op = op;
    return dexel_batch_workspace_size(ctx, 1, &it, cap_hint, bytes);
}

dexel_status dexel_workspace_need(dexel_ctx* ctx, const void* ws, int64_t* cap_hint) {
    if (!ctx || !ws || !cap_hint) return DEXEL_ERR_INVALID;
    WsHeader h;
    hipError_t e = hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(ctx, DEXEL_ERR_HIP, hipGetErrorString(e));
    unsigned long long m = h.need_cap;
    for (unsigned long long v : {h.bumpA, h.bumpI, h.bumpC, h.arena}) m = v > m ? v : m;
    *cap_hint = (int64_t)m;
    return DEXEL_OK;
}

dexel_status dexel_offset(dexel_ctx* ctx, const dexel_grid_view* in, float r, int32_t op,
                          dexel_grid_out* out, void* ws, size_t ws_bytes, void* stream,
                          uint32_t flags) {
    if (!ctx) return DEXEL_ERR_INVALID;
    if (!in || !out) return fail(ctx, DEXEL_ERR_INVALID, "null input or output");
    dexel_batch_item it{};
    it.in = *in;
    it.r = r;
    it.op = op;
    it.out = *out;
    return dexel_batch_offset(ctx, 1, &it, ws, ws_bytes, stream, flags);
}

dexel_status dexel_offset_noalloc(dexel_ctx* ctx, const dexel_grid_view* in, float r, int32_t op,
                                  dexel_grid_out* out, void* stream, uint32_t flags) {
    if (!ctx) return DEXEL_ERR_INVALID;
    ctx->err.clear();
    if (!in || !out) return fail(ctx, DEXEL_ERR_INVALID, "null input or output");
    if (!ctx->scratch) return fail(ctx, DEXEL_ERR_HIP, "no static scratch on this device");
    dexel_batch_item it{};
    it.in = *in;
    it.r = r;
    it.op = op;
    it.out = *out;
    std::vector<ItemInfo> info;
    dexel_status st = check_items(ctx, 1, &it, &info, true);
    if (st != DEXEL_OK) return st;
    const size_t need = make_layout(info, default_cap(in)).total;
    if (need > DEXEL_NOALLOC_SCRATCH_BYTES) {
        char buf[160];
        std::snprintf(buf, sizeof(buf),
                      "the call needs %zu bytes of workspace; the static scratch holds %zu (use dexel_offset)",
                      need, (size_t)DEXEL_NOALLOC_SCRATCH_BYTES);
        return fail(ctx, DEXEL_ERR_UNSUPPORTED, buf);
    }
    hipStream_t s = (hipStream_t)stream;
    // no profiling events: creating them would allocate
    const bool prof = ctx->profile;
    ctx->profile = false;
    st = enqueue_batch(ctx, 1, &it, info, ctx->scratch, DEXEL_NOALLOC_SCRATCH_BYTES, s, flags,
                       pick_variant(ctx, 1, &it));
    ctx->profile = prof;
    if (st != DEXEL_OK) return st;
    if (flags & DEXEL_FLAG_SYNC) return sync_status(ctx, s, 1, &it);
    return DEXEL_OK;
}

dexel_status dexel_dilate(dexel_ctx* ctx, const dexel_grid_view* in, float r, dexel_grid_out* out,
                          void* ws, size_t ws_bytes, void* stream, uint32_t flags) {
    return dexel_offset(ctx, in, r, DEXEL_DILATE, out, ws, ws_bytes, stream, flags);
}

dexel_status dexel_erode(dexel_ctx* ctx, const dexel_grid_view* in, float r, dexel_grid_out* out,
                         void* ws, size_t ws_bytes, void* stream, uint32_t flags) {
    return dexel_offset(ctx, in, r, DEXEL_ERODE, out, ws, ws_bytes, stream, flags);
}

dexel_status dexel_batch_workspace_size(dexel_ctx* ctx, int32_t n, const dexel_batch_item* items,
                                        int64_t cap_hint, size_t* bytes) {
    if (!ctx || !bytes) return DEXEL_ERR_INVALID;
    std::vector<ItemInfo> info;
    dexel_status st = check_items(ctx, n, items, &info, false);
    if (st != DEXEL_OK) return st;
    const int64_t cap = cap_hint > 0 ? cap_hint : batch_default_cap(n, items);
    *bytes = make_layout(info, cap).total;
    return DEXEL_OK;
}

dexel_status dexel_batch_offset(dexel_ctx* ctx, int32_t n, const dexel_batch_item* items, void* ws,
                                size_t ws_bytes, void* stream, uint32_t flags) {
    if (!ctx) return DEXEL_ERR_INVALID;
    ctx->err.clear();
    std::vector<ItemInfo> info;
    dexel_status st = check_items(ctx, n, items, &info, true);
    if (st != DEXEL_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = enqueue_batch(ctx, n, items, info, ws, ws_bytes, s, flags, pick_variant(ctx, n, items));
    if (st != DEXEL_OK) return st;
    if (flags & DEXEL_FLAG_SYNC) return sync_status(ctx, s, n, items);
    return DEXEL_OK;
}

dexel_status dexel_set_variant(dexel_ctx* ctx, int variant) {
    if (!ctx || variant < -1 || variant >= dexel::NVARIANT) return DEXEL_ERR_INVALID;
    ctx->forced_variant = variant;
    return DEXEL_OK;
}

dexel_status dexel_autotune(dexel_ctx* ctx, int32_t n, const dexel_batch_item* items, void* ws,
                            size_t ws_bytes, void* stream, int32_t reps, int32_t* chosen,
                            float* ms) {
    if (!ctx || reps < 1) return DEXEL_ERR_INVALID;
    ctx->err.clear();
    std::vector<ItemInfo> info;
    dexel_status st = check_items(ctx, n, items, &info, true);
    if (st != DEXEL_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const bool prof = ctx->profile;
    ctx->profile = false;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int best = 0;
    float best_ms = 0.f;
    dexel_status result = DEXEL_OK;
    bool any = false;
    for (int v = 0; v < dexel::NVARIANT && result == DEXEL_OK; ++v) {
        // one untimed run (also checks the workspace and outputs fit); a
        // variant that does not fit the caller's workspace or outputs is
        // skipped (time -1)
        result = enqueue_batch(ctx, n, items, info, ws, ws_bytes, s, 0, v);
        if (result != DEXEL_OK) break;
        result = sync_status(ctx, s, n, items);
        if (result == DEXEL_ERR_WORKSPACE || result == DEXEL_ERR_CAPACITY) {
            if (ms) ms[v] = -1.0f;
            result = DEXEL_OK;
            continue;
        }
        if (result != DEXEL_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) { result = DEXEL_ERR_HIP; break; }
        for (int k = 0; k < reps && result == DEXEL_OK; ++k)
            result = enqueue_batch(ctx, n, items, info, ws, ws_bytes, s, 0, v);
        if (result != DEXEL_OK) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            result = DEXEL_ERR_HIP;
            break;
        }
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        t /= (float)reps;
        if (ms) ms[v] = t;
        if (!any || t < best_ms) {
            best = v;
            best_ms = t;
            any = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->profile = prof;
    if (result != DEXEL_OK) return result;
    if (!any) return fail(ctx, DEXEL_ERR_WORKSPACE, "no kernel variant fits the workspace");
    // leave the outputs as the chosen variant computes them
    result = enqueue_batch(ctx, n, items, info, ws, ws_bytes, s, 0, best);
    if (result == DEXEL_OK) result = sync_status(ctx, s, n, items);
    if (result != DEXEL_OK) return result;
    ctx->tuned[batch_signature(n, items)] = best;
    if (chosen) *chosen = best;
    return DEXEL_OK;
}

dexel_status dexel_profile_enable(dexel_ctx* ctx, int on) {
    if (!ctx) return DEXEL_ERR_INVALID;
    ctx->profile = on != 0;
    return DEXEL_OK;
}

dexel_status dexel_profile_read(dexel_ctx* ctx, double* ms, int64_t* passes, int reset) {
    if (!ctx) return DEXEL_ERR_INVALID;
    for (auto& g : ctx->pending) {
        HIP_TRY(hipEventSynchronize(g.back()));
        for (int i = 0; i < dexel::NPROF; ++i) {
            float t = 0.f;
            HIP_TRY(hipEventElapsedTime(&t, g[i], g[i + 1]));
            ctx->acc[i] += t;
        }
        ctx->passes += 1;
        for (hipEvent_t e : g) ctx->pool.push_back(e);
    }
    ctx->pending.clear();
    if (ms)
        for (int i = 0; i < dexel::NPROF; ++i) ms[i] = ctx->acc[i];
    if (passes) *passes = ctx->passes;
    if (reset) {
        for (int i = 0; i < dexel::NPROF; ++i) ctx->acc[i] = 0;
        ctx->passes = 0;
    }
    return DEXEL_OK;
}

dexel_status dexel_workspace_stats(dexel_ctx* ctx, const void* ws, int64_t* stats) {
    if (!ctx || !ws || !stats) return DEXEL_ERR_INVALID;
    WsHeader h;
    hipError_t e = hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(ctx, DEXEL_ERR_HIP, hipGetErrorString(e));
    int64_t novf = 0;
    for (int i = 0; i < dexel::NSTAGE; ++i) novf += h.novf[i];
    stats[0] = (int64_t)h.bumpA;
    stats[1] = (int64_t)h.bumpI;
    stats[2] = (int64_t)h.nseeds;
    stats[3] = (int64_t)h.bumpC;
    stats[4] = (int64_t)h.arena;
    stats[5] = novf;
    stats[6] = (int64_t)h.need_cap;
    stats[7] = h.nseg_out;
    return DEXEL_OK;
}

// Workspace of dexel_csg: header, counts, scan, block sums (256-byte aligned).
static size_t csg_layout(int64_t ncols, size_t* cnt, size_t* scan, size_t* bsum) {
    size_t o = align_up(sizeof(WsHeader));
    *cnt = o;
    o = align_up(o + 4 * (size_t)ncols);
    *scan = o;
    o = align_up(o + 8 * (size_t)(ncols + 1));
    *bsum = o;
    o = align_up(o + 8 * (size_t)((ncols + 1023) / 1024 + 2));
    return o;
}

dexel_status dexel_csg_workspace_size(dexel_ctx* ctx, const dexel_grid_view* a, size_t* bytes) {
    if (!ctx || !bytes) return DEXEL_ERR_INVALID;
    dexel_status st = check_view(ctx, a);
    if (st != DEXEL_OK) return st;
    size_t c, q, b;
    *bytes = csg_layout((int64_t)a->nx * a->ny, &c, &q, &b);
    return DEXEL_OK;
}

dexel_status dexel_csg(dexel_ctx* ctx, const dexel_grid_view* a, const dexel_grid_view* b, int32_t op,
                       dexel_grid_out* out, void* ws, size_t ws_bytes, void* stream, uint32_t flags) {
    if (!ctx) return DEXEL_ERR_INVALID;
    ctx->err.clear();
    dexel_status st = check_view(ctx, a);
    if (st != DEXEL_OK) return st;
    st = check_view(ctx, b);
    if (st != DEXEL_OK) return st;
    if (!out) return fail(ctx, DEXEL_ERR_INVALID, "null output");
    if (a->nx != b->nx || a->ny != b->ny || out->nx != a->nx || out->ny != a->ny)
        return fail(ctx, DEXEL_ERR_INVALID, "the two inputs and the output must have the same nx, ny");
    if (op < DEXEL_CSG_UNION || op > DEXEL_CSG_DIFFERENCE) return fail(ctx, DEXEL_ERR_INVALID, "unknown CSG op");
    if (flags & ~(DEXEL_FLAG_SYNC | DEXEL_FLAG_VALIDATE)) return fail(ctx, DEXEL_ERR_INVALID, "unknown flags");
    if (flags & DEXEL_FLAG_VALIDATE)
        return fail(ctx, DEXEL_ERR_UNSUPPORTED, "dexel_csg does not validate its inputs");
    if (!out->col_ptr || !out->nseg_out || !out->status)
        return fail(ctx, DEXEL_ERR_INVALID, "null output col_ptr, nseg_out or status");
    if (out->cap_seg < 0 || (out->cap_seg > 0 && !out->z))
        return fail(ctx, DEXEL_ERR_INVALID, "bad output capacity or null output z");
    if (((uintptr_t)out->z) % 8 != 0) return fail(ctx, DEXEL_ERR_INVALID, "output z must be 8-byte aligned");
    if (!ws) return fail(ctx, DEXEL_ERR_INVALID, "null workspace");
    if (((uintptr_t)ws) % 256 != 0) return fail(ctx, DEXEL_ERR_INVALID, "workspace must be 256-byte aligned");
    const int64_t ncols = (int64_t)a->nx * a->ny;
    size_t o_cnt, o_scan, o_bsum;
    if (csg_layout(ncols, &o_cnt, &o_scan, &o_bsum) > ws_bytes)
        return fail(ctx, DEXEL_ERR_WORKSPACE, "workspace smaller than dexel_csg_workspace_size");
    HIP_TRY(hipSetDevice(ctx->device));
    char* w = (char*)ws;
    dexel::CsgArgs g{};
    g.a_ptr = a->col_ptr;
    g.a_z = (const float2*)a->z;
    g.b_ptr = b->col_ptr;
    g.b_z = (const float2*)b->z;
    g.ncols = ncols;
    g.op = op;
    g.hdr = (WsHeader*)w;
    g.cnt = (int32_t*)(w + o_cnt);
    g.scan = (int64_t*)(w + o_scan);
    g.bsum = (int64_t*)(w + o_bsum);
    g.out_ptr = out->col_ptr;
    g.out_z = (float2*)out->z;
    g.cap = out->cap_seg;
    g.out_nseg = out->nseg_out;
    g.out_status = out->status;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(dexel::launch_csg(g, s));
    if (!(flags & DEXEL_FLAG_SYNC)) return DEXEL_OK;
    HIP_TRY(hipStreamSynchronize(s));
    int32_t dst = 0;
    HIP_TRY(hipMemcpy(&dst, out->status, sizeof(dst), hipMemcpyDeviceToHost));
    if (dst != 0) return fail(ctx, (dexel_status)dst, "device status " + std::to_string(dst));
    return DEXEL_OK;
}

// The CSG layout (header, counts, scan), then the long-column list and the
// scratch copy of the input intervals used by dexel_canonicalize.
static size_t canon_layout(int64_t ncols, int64_t nseg, size_t* longc, size_t* sorted) {
    size_t c, q, b;
    size_t o = csg_layout(ncols, &c, &q, &b);
    *longc = o;
    o = align_up(o + 4 * (size_t)ncols);
    *sorted = o;
    return align_up(o + 8 * (size_t)nseg);
}

dexel_status dexel_canonicalize_workspace_size(dexel_ctx* ctx, const dexel_grid_view* in, size_t* bytes) {
    if (!ctx || !bytes) return DEXEL_ERR_INVALID;
    dexel_status st = check_view(ctx, in);
    if (st != DEXEL_OK) return st;
    size_t l, s;
    *bytes = canon_layout((int64_t)in->nx * in->ny, in->nseg, &l, &s);
    return DEXEL_OK;
}

dexel_status dexel_canonicalize(dexel_ctx* ctx, const dexel_grid_view* in, dexel_grid_out* out, void* ws,
                                size_t ws_bytes, void* stream, uint32_t flags) {
    if (!ctx) return DEXEL_ERR_INVALID;
    ctx->err.clear();
    dexel_status st = check_view(ctx, in);
    if (st != DEXEL_OK) return st;
    if (!out) return fail(ctx, DEXEL_ERR_INVALID, "null output");
    if (out->nx != in->nx || out->ny != in->ny) return fail(ctx, DEXEL_ERR_INVALID, "output nx, ny differ");
    if (flags & ~(DEXEL_FLAG_SYNC | DEXEL_FLAG_VALIDATE)) return fail(ctx, DEXEL_ERR_INVALID, "unknown flags");
    if (flags & DEXEL_FLAG_VALIDATE)
        return fail(ctx, DEXEL_ERR_UNSUPPORTED, "dexel_canonicalize always checks its input");
    if (!out->col_ptr || !out->nseg_out || !out->status)
        return fail(ctx, DEXEL_ERR_INVALID, "null output col_ptr, nseg_out or status");
    if (out->cap_seg < 0 || (out->cap_seg > 0 && !out->z))
        return fail(ctx, DEXEL_ERR_INVALID, "bad output capacity or null output z");
    if (((uintptr_t)out->z) % 8 != 0) return fail(ctx, DEXEL_ERR_INVALID, "output z must be 8-byte aligned");
    if (!ws) return fail(ctx, DEXEL_ERR_INVALID, "null workspace");
    if (((uintptr_t)ws) % 256 != 0) return fail(ctx, DEXEL_ERR_INVALID, "workspace must be 256-byte aligned");
    const int64_t ncols = (int64_t)in->nx * in->ny;
    size_t o_cnt, o_scan, o_bsum, o_long, o_sorted;
    csg_layout(ncols, &o_cnt, &o_scan, &o_bsum);
    if (canon_layout(ncols, in->nseg, &o_long, &o_sorted) > ws_bytes)
        return fail(ctx, DEXEL_ERR_WORKSPACE, "workspace smaller than dexel_canonicalize_workspace_size");
    HIP_TRY(hipSetDevice(ctx->device));
    char* w = (char*)ws;
    dexel::CanonArgs g{};
    g.in_ptr = in->col_ptr;
    g.in_z = (const float2*)in->z;
    g.nseg = in->nseg;
    g.ncols = ncols;
    g.hdr = (WsHeader*)w;
    g.cnt = (int32_t*)(w + o_cnt);
    g.scan = (int64_t*)(w + o_scan);
    g.bsum = (int64_t*)(w + o_bsum);
    g.out_ptr = out->col_ptr;
    g.out_z = (float2*)out->z;
    g.cap = out->cap_seg;
    g.out_nseg = out->nseg_out;
    g.out_status = out->status;
    g.longc = (int32_t*)(w + o_long);
    g.sorted = (float2*)(w + o_sorted);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(dexel::launch_canonicalize(g, s));
    if (!(flags & DEXEL_FLAG_SYNC)) return DEXEL_OK;
    HIP_TRY(hipStreamSynchronize(s));
    int32_t dst = 0;
    HIP_TRY(hipMemcpy(&dst, out->status, sizeof(dst), hipMemcpyDeviceToHost));
    if (dst != 0) return fail(ctx, (dexel_status)dst, "device status " + std::to_string(dst));
    return DEXEL_OK;
}

// The CSG layout (header, counts, scan) followed by the list of cell tiles
// that the dexelisation redoes with the full per-column capacity.
static size_t dex_layout(int32_t nx, int32_t ny, size_t* spill) {
    size_t c, q, b;
    const size_t o = csg_layout((int64_t)nx * ny, &c, &q, &b);
    *spill = o;
    return align_up(o + 4 * (size_t)dexel::dexelize_tiles(nx, ny));
}

dexel_status dexel_dexelize_workspace_size(dexel_ctx* ctx, int32_t nx, int32_t ny, size_t* bytes) {
    if (!ctx || !bytes) return DEXEL_ERR_INVALID;
    if (nx <= 0 || ny <= 0) return fail(ctx, DEXEL_ERR_INVALID, "nx and ny must be >= 1");
    if ((int64_t)nx * ny >= ((int64_t)1 << 31) - 64)
        return fail(ctx, DEXEL_ERR_UNSUPPORTED, "nx * ny must be below 2^31");
    size_t sp;
    *bytes = dex_layout(nx, ny, &sp);
    return DEXEL_OK;
}

dexel_status dexel_dexelize(dexel_ctx* ctx, int32_t nx, int32_t ny, const double* prims, int32_t nprims,
                            dexel_grid_out* out, void* ws, size_t ws_bytes, void* stream, uint32_t flags) {
    if (!ctx) return DEXEL_ERR_INVALID;
    ctx->err.clear();
    if (nx <= 0 || ny <= 0) return fail(ctx, DEXEL_ERR_INVALID, "nx and ny must be >= 1");
    if ((int64_t)nx * ny >= ((int64_t)1 << 31) - 64)
        return fail(ctx, DEXEL_ERR_UNSUPPORTED, "nx * ny must be below 2^31");
    if (nprims < 0 || (nprims > 0 && !prims)) return fail(ctx, DEXEL_ERR_INVALID, "bad primitive list");
    if (!out) return fail(ctx, DEXEL_ERR_INVALID, "null output");
    if (out->nx != nx || out->ny != ny) return fail(ctx, DEXEL_ERR_INVALID, "output nx, ny differ");
    if (flags & ~(DEXEL_FLAG_SYNC | DEXEL_FLAG_VALIDATE | DEXEL_FLAG_RAYS_X | DEXEL_FLAG_RAYS_Y))
        return fail(ctx, DEXEL_ERR_INVALID, "unknown flags");
    if (flags & DEXEL_FLAG_VALIDATE)
        return fail(ctx, DEXEL_ERR_UNSUPPORTED, "dexel_dexelize has no input to validate");
    if ((flags & DEXEL_FLAG_RAYS_X) && (flags & DEXEL_FLAG_RAYS_Y))
        return fail(ctx, DEXEL_ERR_INVALID, "DEXEL_FLAG_RAYS_X and DEXEL_FLAG_RAYS_Y together");
    if (!out->col_ptr || !out->nseg_out || !out->status)
        return fail(ctx, DEXEL_ERR_INVALID, "null output col_ptr, nseg_out or status");
    if (out->cap_seg < 0 || (out->cap_seg > 0 && !out->z))
        return fail(ctx, DEXEL_ERR_INVALID, "bad output capacity or null output z");
    if (((uintptr_t)out->z) % 8 != 0) return fail(ctx, DEXEL_ERR_INVALID, "output z must be 8-byte aligned");
    if (((uintptr_t)prims) % 8 != 0) return fail(ctx, DEXEL_ERR_INVALID, "primitives must be 8-byte aligned");
    if (!ws) return fail(ctx, DEXEL_ERR_INVALID, "null workspace");
    if (((uintptr_t)ws) % 256 != 0) return fail(ctx, DEXEL_ERR_INVALID, "workspace must be 256-byte aligned");
    const int64_t ncols = (int64_t)nx * ny;
    size_t o_cnt, o_scan, o_bsum, o_spill;
    csg_layout(ncols, &o_cnt, &o_scan, &o_bsum);
    if (dex_layout(nx, ny, &o_spill) > ws_bytes)
        return fail(ctx, DEXEL_ERR_WORKSPACE, "workspace smaller than dexel_dexelize_workspace_size");
    HIP_TRY(hipSetDevice(ctx->device));
    char* w = (char*)ws;
    dexel::DexArgs g{};
    g.prims = prims;
    g.nprims = nprims;
    g.nx = nx;
    g.ny = ny;
    g.axis = (flags & DEXEL_FLAG_RAYS_X) ? 0 : ((flags & DEXEL_FLAG_RAYS_Y) ? 1 : 2);
    g.ncols = ncols;
    g.hdr = (WsHeader*)w;
    g.cnt = (int32_t*)(w + o_cnt);
    g.scan = (int64_t*)(w + o_scan);
    g.bsum = (int64_t*)(w + o_bsum);
    g.out_ptr = out->col_ptr;
    g.out_z = (float2*)out->z;
    g.cap = out->cap_seg;
    g.out_nseg = out->nseg_out;
    g.out_status = out->status;
    g.spill = (int32_t*)(w + o_spill);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(dexel::launch_dexelize(g, s));
    if (!(flags & DEXEL_FLAG_SYNC)) return DEXEL_OK;
    HIP_TRY(hipStreamSynchronize(s));
    int32_t dst = 0;
    HIP_TRY(hipMemcpy(&dst, out->status, sizeof(dst), hipMemcpyDeviceToHost));
    if (dst != 0) return fail(ctx, (dexel_status)dst, "device status " + std::to_string(dst));
    return DEXEL_OK;
}

const char* dexel_status_string(dexel_status s) {
    switch (s) {
        case DEXEL_OK: return "ok";
        case DEXEL_ERR_INVALID: return "invalid argument";
        case DEXEL_ERR_NOT_CANONICAL: return "input is not canonical";
        case DEXEL_ERR_CAPACITY: return "output capacity exceeded";
        case DEXEL_ERR_WORKSPACE: return "workspace too small";
        case DEXEL_ERR_HIP: return "HIP runtime error";
        case DEXEL_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* dexel_last_error(const dexel_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"
