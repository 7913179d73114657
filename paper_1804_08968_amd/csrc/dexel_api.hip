// Host side of the libdexel C ABI (see include/dexel.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/dexel.h"
#include "dexel_internal.h"

using dexel::OpParams;
using dexel::WsHeader;

struct dexel_ctx {
    int device = 0;
    std::string err;
    // Radius lookup tables, one pinned host buffer per distinct radius.  A
    // table is immutable once built, so an asynchronous upload from it can
    // never observe a later call's table.
    std::map<uint32_t, float*> luts;
    // Optional per-stage timing: HIP events recorded on the call's stream at
    // the stage boundaries of every pass, read back by dexel_profile_read.
    bool profile = false;
    std::vector<hipEvent_t> pool;
    std::vector<std::vector<hipEvent_t>> pending;
    double acc[dexel::NPROF] = {0};
    int64_t passes = 0;
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

// Workspace layout for one call.
struct Layout {
    size_t hdr, lut, offA, cntA, A, offI, cntI, I, offB, cntB, B, tagB, hullB, offC, cntC, C, ovf, arena,
        bsum, mid_ptr, mid_z, total;
};

Layout make_layout(int64_t ncols, int64_t cap, int d2max, bool chain) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t nc = (size_t)ncols, cp = (size_t)cap;
    L.hdr = take(256);
    L.lut = take(sizeof(float) * (size_t)(d2max + 1));
    L.offA = take(8 * nc);
    L.cntA = take(4 * nc);
    L.A = take(8 * cp);
    L.offI = take(8 * nc);
    L.cntI = take(4 * nc);
    L.I = take(8 * cp);
    L.offB = take(8 * (nc + 1));
    L.cntB = take(4 * nc);
    L.B = take(8 * cp);
    L.tagB = take(cp);
    L.hullB = take(8 * nc);
    L.offC = take(8 * nc);
    L.cntC = take(4 * nc);
    L.C = take(8 * cp);
    L.ovf = take(4 * nc * dexel::NSTAGE);
    L.arena = take(8 * cp);
    L.bsum = take(8 * ((nc + 1023) / 1024 + 2));
    if (chain) {
        L.mid_ptr = take(8 * (nc + 1));
        L.mid_z = take(8 * cp);
    }
    L.total = o;
    return L;
}

int64_t default_cap(const dexel_grid_view* in) {
    const int64_t ncols = (int64_t)in->nx * in->ny;
    return in->nseg + 2 * ncols + 1024;
}

bool is_chain(int op) { return op == DEXEL_OPEN || op == DEXEL_CLOSE; }

dexel_status check_view(dexel_ctx* ctx, const dexel_grid_view* in) {
    if (!in) return fail(ctx, DEXEL_ERR_INVALID, "null input view");
    if (in->nx <= 0 || in->ny <= 0) return fail(ctx, DEXEL_ERR_INVALID, "nx and ny must be >= 1");
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

// Pinned host table H[d2] = float(sqrt(double(r)^2 - d2)), d2 = 0..floor(r^2).
float* lut_for(dexel_ctx* ctx, float r, int d2max) {
    const uint32_t key = float_bits(r);
    auto it = ctx->luts.find(key);
    if (it != ctx->luts.end()) return it->second;
    float* h = nullptr;
    if (hipHostMalloc((void**)&h, sizeof(float) * (size_t)(d2max + 1), hipHostMallocDefault) != hipSuccess)
        return nullptr;
    const double r2 = (double)r * (double)r;
    for (int d2 = 0; d2 <= d2max; ++d2) h[d2] = (float)std::sqrt(r2 - (double)d2);
    ctx->luts[key] = h;
    return h;
}

OpParams base_params(const Layout& L, char* ws, int64_t ncols, int64_t cap) {
    OpParams p{};
    p.ncols = ncols;
    p.hdr = (WsHeader*)(ws + L.hdr);
    p.H = (const float*)(ws + L.lut);
    p.cap = cap;
    p.offA = (int64_t*)(ws + L.offA);
    p.cntA = (int32_t*)(ws + L.cntA);
    p.A = (float2*)(ws + L.A);
    p.offI = (int64_t*)(ws + L.offI);
    p.cntI = (int32_t*)(ws + L.cntI);
    p.I = (float2*)(ws + L.I);
    p.offB = (int64_t*)(ws + L.offB);
    p.cntB = (int32_t*)(ws + L.cntB);
    p.B = (float2*)(ws + L.B);
    p.tagB = (uint8_t*)(ws + L.tagB);
    p.hullB = (float2*)(ws + L.hullB);
    p.offC = (int64_t*)(ws + L.offC);
    p.cntC = (int32_t*)(ws + L.cntC);
    p.C = (float2*)(ws + L.C);
    p.ovf = (int32_t*)(ws + L.ovf);
    p.arena = (float2*)(ws + L.arena);
    p.bsum = (int64_t*)(ws + L.bsum);
    return p;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ctx, DEXEL_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// Enqueue one operation (any dexel_op) into an already checked workspace.
dexel_status enqueue_op(dexel_ctx* ctx, const dexel_grid_view* in, float r, int op,
                        dexel_grid_out* out, void* ws, size_t ws_bytes, hipStream_t s,
                        uint32_t flags, int64_t cap_hint) {
    const int64_t ncols = (int64_t)in->nx * in->ny;
    const int64_t cap = cap_hint > 0 ? cap_hint : default_cap(in);
    int R, d2max;
    radius_params(r, &R, &d2max);
    const bool chain = is_chain(op);
    const Layout L = make_layout(ncols, cap, d2max, chain);
    if (!ws) return fail(ctx, DEXEL_ERR_INVALID, "null workspace");
    if (((uintptr_t)ws) % kAlign != 0) return fail(ctx, DEXEL_ERR_INVALID, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(ctx, DEXEL_ERR_WORKSPACE, "workspace smaller than dexel_workspace_size");
    char* w = (char*)ws;
    float* lut = lut_for(ctx, r, d2max);
    if (!lut) return fail(ctx, DEXEL_ERR_HIP, "cannot allocate pinned lookup table");

    OpParams p = base_params(L, w, ncols, cap);
    p.nx = in->nx;
    p.ny = in->ny;
    p.R = R;
    p.d2max = d2max;

    HIP_TRY(dexel::launch_init_call(p.hdr, s));
    HIP_TRY(hipMemcpyAsync(w + L.lut, lut, sizeof(float) * (size_t)(d2max + 1), hipMemcpyHostToDevice, s));

    // stage list: (erode?, source, destination)
    int ops[2] = {0, 0};
    int nops = 1;
    switch (op) {
        case DEXEL_DILATE: ops[0] = 0; break;
        case DEXEL_ERODE: ops[0] = 1; break;
        case DEXEL_OPEN: ops[0] = 1; ops[1] = 0; nops = 2; break;
        case DEXEL_CLOSE: ops[0] = 0; ops[1] = 1; nops = 2; break;
        default: return fail(ctx, DEXEL_ERR_INVALID, "unknown op");
    }
    for (int k = 0; k < nops; ++k) {
        const bool first = (k == 0), last = (k == nops - 1);
        p.erode = ops[k];
        if (first) {
            p.col_ptr = in->col_ptr;
            p.z = (const float2*)in->z;
            p.nseg = in->nseg;
        } else {
            p.col_ptr = (const int64_t*)(w + L.mid_ptr);
            p.z = (const float2*)(w + L.mid_z);
            p.nseg = -1;
        }
        if (last) {
            p.out_col_ptr = out->col_ptr;
            p.out_z = (float2*)out->z;
            p.out_cap = out->cap_seg;
            p.out_is_intermediate = 0;
        } else {
            p.out_col_ptr = (int64_t*)(w + L.mid_ptr);
            p.out_z = (float2*)(w + L.mid_z);
            p.out_cap = cap;
            p.out_is_intermediate = 1;
        }
        if (!first) HIP_TRY(dexel::launch_init_op(p.hdr, s));
        if (first) {
            HIP_TRY(dexel::launch_check_colptr(p, s));
            if (flags & DEXEL_FLAG_VALIDATE) HIP_TRY(dexel::launch_validate(p, s));
        }
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
        HIP_TRY(dexel::launch_offset_pass(p, s, ev));
    }
    HIP_TRY(dexel::launch_finish(p.hdr, out->col_ptr, ncols, out->nseg_out, out->status, s));
    return DEXEL_OK;
}

dexel_status sync_status(dexel_ctx* ctx, hipStream_t s, const int32_t* dstatus) {
    HIP_TRY(hipStreamSynchronize(s));
    int32_t st = 0;
    HIP_TRY(hipMemcpy(&st, dstatus, sizeof(st), hipMemcpyDeviceToHost));
    if (st != 0) {
        char buf[96];
        std::snprintf(buf, sizeof(buf), "device status %d", st);
        ctx->err = buf;
    }
    return (dexel_status)st;
}

}  // namespace

extern "C" {

dexel_status dexel_ctx_create(int device, dexel_ctx** ctx) {
    if (!ctx) return DEXEL_ERR_INVALID;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DEXEL_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return DEXEL_ERR_HIP;
    dexel_ctx* c = new dexel_ctx();
    c->device = device;
    *ctx = c;
    return DEXEL_OK;
}

void dexel_ctx_destroy(dexel_ctx* ctx) {
    if (!ctx) return;
    for (auto& g : ctx->pending)
        for (hipEvent_t e : g) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    for (auto& kv : ctx->luts) (void)hipHostFree(kv.second);
    delete ctx;
}

dexel_status dexel_workspace_size(dexel_ctx* ctx, const dexel_grid_view* in, float r, int32_t op,
                                  int64_t cap_hint, size_t* bytes) {
    if (!ctx || !bytes) return DEXEL_ERR_INVALID;
    if (!in) return fail(ctx, DEXEL_ERR_INVALID, "null input view");
    if (in->nx <= 0 || in->ny <= 0 || in->nseg < 0) return fail(ctx, DEXEL_ERR_INVALID, "bad grid size");
    dexel_status st = check_radius(ctx, r);
    if (st != DEXEL_OK) return st;
    if (op < DEXEL_DILATE || op > DEXEL_CLOSE) return fail(ctx, DEXEL_ERR_INVALID, "unknown op");
    int R, d2max;
    radius_params(r, &R, &d2max);
    const int64_t cap = cap_hint > 0 ? cap_hint : default_cap(in);
    *bytes = make_layout((int64_t)in->nx * in->ny, cap, d2max, is_chain(op)).total;
    return DEXEL_OK;
}

dexel_status dexel_workspace_need(dexel_ctx* ctx, const void* ws, int64_t* cap_hint) {
    if (!ctx || !ws || !cap_hint) return DEXEL_ERR_INVALID;
    WsHeader h;
    hipError_t e = hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(ctx, DEXEL_ERR_HIP, hipGetErrorString(e));
    *cap_hint = (int64_t)h.need_cap;
    return DEXEL_OK;
}

dexel_status dexel_offset(dexel_ctx* ctx, const dexel_grid_view* in, float r, int32_t op,
                          dexel_grid_out* out, void* ws, size_t ws_bytes, void* stream,
                          uint32_t flags) {
    if (!ctx) return DEXEL_ERR_INVALID;
    ctx->err.clear();
    dexel_status st = check_view(ctx, in);
    if (st != DEXEL_OK) return st;
    if ((st = check_radius(ctx, r)) != DEXEL_OK) return st;
    if ((st = check_out(ctx, in, out)) != DEXEL_OK) return st;
    if (op < DEXEL_DILATE || op > DEXEL_CLOSE) return fail(ctx, DEXEL_ERR_INVALID, "unknown op");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DEXEL_ERR_HIP, "hipSetDevice failed");
    // The internal buffers get the largest capacity whose layout fits in
    // ws_bytes (at least what dexel_workspace_size was asked for).
    const int64_t ncols = (int64_t)in->nx * in->ny;
    int R, d2max;
    radius_params(r, &R, &d2max);
    int64_t lo = 1, hi = 1;
    while (make_layout(ncols, hi, d2max, is_chain(op)).total <= ws_bytes && hi < ((int64_t)1 << 40)) hi *= 2;
    if (make_layout(ncols, lo, d2max, is_chain(op)).total > ws_bytes)
        return fail(ctx, DEXEL_ERR_WORKSPACE, "workspace smaller than the minimum layout");
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        if (make_layout(ncols, mid, d2max, is_chain(op)).total <= ws_bytes) lo = mid; else hi = mid;
    }
    hipStream_t s = (hipStream_t)stream;
    st = enqueue_op(ctx, in, r, op, out, ws, ws_bytes, s, flags, lo);
    if (st != DEXEL_OK) return st;
    if (flags & DEXEL_FLAG_SYNC) return sync_status(ctx, s, out->status);
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
    if (!ctx || !bytes || n < 0 || (n > 0 && !items)) return DEXEL_ERR_INVALID;
    size_t best = 0;
    for (int32_t i = 0; i < n; ++i) {
        size_t b = 0;
        dexel_status st = dexel_workspace_size(ctx, &items[i].in, items[i].r, items[i].op, cap_hint, &b);
        if (st != DEXEL_OK) return st;
        if (b > best) best = b;
    }
    *bytes = best;
    return DEXEL_OK;
}

dexel_status dexel_batch_offset(dexel_ctx* ctx, int32_t n, const dexel_batch_item* items, void* ws,
                                size_t ws_bytes, void* stream, uint32_t flags) {
    if (!ctx || n < 0 || (n > 0 && !items)) return DEXEL_ERR_INVALID;
    ctx->err.clear();
    for (int32_t i = 0; i < n; ++i) {
        const dexel_batch_item& it = items[i];
        dexel_grid_out o = it.out;
        dexel_status st = dexel_offset(ctx, &it.in, it.r, it.op, &o, ws, ws_bytes, stream,
                                       flags & ~DEXEL_FLAG_SYNC);
        if (st != DEXEL_OK) return st;
    }
    if (flags & DEXEL_FLAG_SYNC) {
        hipStream_t s = (hipStream_t)stream;
        HIP_TRY(hipStreamSynchronize(s));
        for (int32_t i = 0; i < n; ++i) {
            int32_t st = 0;
            HIP_TRY(hipMemcpy(&st, items[i].out.status, sizeof(st), hipMemcpyDeviceToHost));
            if (st != 0) return (dexel_status)st;
        }
    }
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
    stats[2] = h.nseeds;
    stats[3] = (int64_t)h.bumpC;
    stats[4] = (int64_t)h.arena;
    stats[5] = novf;
    stats[6] = (int64_t)h.need_cap;
    stats[7] = h.nseg_out;
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
