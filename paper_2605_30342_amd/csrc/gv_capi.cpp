// gv_capi.cpp -- C ABI of the visibility-field path: argument checks,
// workspace planning, and the launch sequence of one call.
//
// Every call runs the same pipeline over all the views it is given:
//   count (conservative culling)  -> scan -> project (+ VF query)
//   -> radix sort by depth -> per-record tile counts -> scan -> emit
//   -> radix sort by tile -> tile ranges -> raster (VF CONST or VF QUERY)
//   -> VF accumulation (build) or per-view scores (query).
// No host synchronisation happens inside the sequence: record and instance
// counts stay on the device, every kernel reads them from the workspace's
// status words and is launched with a grid that does not depend on them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gavis.h"
#include "gv_device.hpp"
#include "gv_launch.hpp"

using namespace gv;

namespace {

thread_local std::string g_err;

gv_status fail(gv_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define GV_HIP(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) return fail(GV_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_)); \
    } while (0)

#define GV_TRY(x)                   \
    do {                            \
        gv_status s_ = (x);         \
        if (s_ != GV_OK) return s_; \
    } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int old = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) == hipSuccess && old != dev) (void)hipSetDevice(dev);
        else old = -1;
    }
    ~DeviceGuard() {
        if (old >= 0) (void)hipSetDevice(old);
    }
};

// Modified spherical Bessel function i_l(x) for the vMF constants
// a_l = 4 pi e^{-kappa} i_l(kappa): ascending series for small arguments,
// upward recurrence from i_0 = sinh x / x, i_1 = (x cosh x - sinh x) / x^2
// for large ones.
double bessel_i(int l, double x) {
    if (x == 0.0) return l == 0 ? 1.0 : 0.0;
    if (x < 8.0) {
        double lead = 1.0;
        for (int k = 1; k <= l; ++k) lead *= x / (2.0 * k + 1.0);
        double term = 1.0, sum = 1.0;
        const double h = 0.5 * x * x;
        for (int k = 1; k < 200 && std::fabs(term) > 1e-17 * sum; ++k) {
            term *= h / (k * (2.0 * l + 2.0 * k + 1.0));
            sum += term;
        }
        return lead * sum;
    }
    double im1 = std::sinh(x) / x;
    if (l == 0) return im1;
    double i = (x * std::cosh(x) - std::sinh(x)) / (x * x);
    for (int k = 1; k < l; ++k) {
        const double nx = im1 - (2.0 * k + 1.0) / x * i;
        im1 = i;
        i = nx;
    }
    return i;
}

bool finite_cam(const gv_camera &c) {
    for (float v : c.R)
        if (!std::isfinite(v)) return false;
    for (float v : c.t)
        if (!std::isfinite(v)) return false;
    return std::isfinite(c.fx) && std::isfinite(c.fy) && std::isfinite(c.cx) && std::isfinite(c.cy) && c.fx > 0.f &&
           c.fy > 0.f;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t status, views, cnt, vmask, offs, blk, rec, bin, key0, val0, key1, val1, ntr, icnt, ioff, post, torder;
    size_t ikey0, ival0, ikey1, ival1, ranges, hist, dtot, accT, accC, gam32, tpart, rcc, rz;
    size_t dc_flags, dc_offs, dc_tmp, dc_misc;   // density control (kind 2)
    size_t total;
};

// Which emission a plan runs.  The scanned one has the depth sort carry each
// record's tile count into depth order (packed into the record's sort value;
// gathered by the last pass for plans of 2^PACK_SHIFT records and more) and
// scans the counts before it emits: one random 32-byte read per record,
// cheap while the records' binning lines stay in the 256 MB last-level
// cache, and its waves take
// chunks of records in turn, which balances records with many tiles.  The
// look-back one reads each binning line once and finds its offsets itself:
// it pays off where the binning lines (32 bytes per record) far exceed that
// cache and records have few tiles each.
int emit_mode_for(const gv_workspace &p) {
    return (uint64_t)p.max_records * sizeof(Bin) > ((uint64_t)256 << 20) && p.max_instances <= 4 * p.max_records
               ? 2 : 1;
}

bool emit_lookback(const gv_workspace &p) { return (p.emit_mode == 0 ? emit_mode_for(p) : p.emit_mode) == 2; }

Layout make_layout(const gv_workspace &p) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += al256(bytes > 0 ? bytes : 1);
        return at;
    };
    const uint64_t N = (uint64_t)p.n, R = (uint64_t)p.max_records, M = (uint64_t)p.max_instances;
    const uint64_t T = (uint64_t)p.total_tiles, V = (uint64_t)p.n_views;
    const int K = (p.sh_degree + 1) * (p.sh_degree + 1);
    L.status = take(sizeof(Status));
    L.views = take(V * sizeof(ViewDev));
    L.cnt = take(N * PROJ_SPLIT * 4);
    L.vmask = take(N * PROJ_SPLIT * (uint64_t)mask_words((int)V) * 4);
    L.offs = take((N * PROJ_SPLIT + 1) * 4);
    const bool lookback = emit_lookback(p);
    L.blk = take(scan_blk_count(lookback ? N * PROJ_SPLIT : std::max(N * PROJ_SPLIT, R)) * 8);
    L.rec = take(R * sizeof(Rec));
    L.bin = take(R * sizeof(Bin));
    L.key0 = take(R * 4);
    L.val0 = take(R * 4);
    L.key1 = take(R * 4);
    L.val1 = take(R * 4);
    if (lookback) {
        L.post = take(emit_post_words(R) * 8);
    } else {
        L.ntr = take((R < ((uint64_t)1 << PACK_SHIFT) ? 0 : R) * 4);   // unpacked tile counts (large plans)
        L.icnt = take(R * 4);
        L.ioff = take((R + 1) * 4);
    }
    L.ikey0 = take(M * 4);
    L.ival0 = take(M * 4);
    L.ikey1 = take(M * 4);
    L.ival1 = take(M * 4);
    L.ranges = take(T * 8);
    L.torder = take((4 * T + 64) * 4);   // cost-ordered tile schedule: sort buffers and a count
    L.hist = take((size_t)RADIX * RADIX_BLOCKS * 4);
    L.dtot = take((size_t)RADIX * 4);
    if (p.kind == 0 || p.kind == 2) {
        L.accT = take(R * 4);
        L.accC = take(R * 4);
        L.gam32 = take(N * (uint64_t)K * 4);
        if (p.kind == 2) {   // the pruning of the virtual particles (at most n of them)
            L.dc_flags = take((N + 1) * 4);
            L.dc_offs = take((N + 1) * 4);
            L.dc_tmp = take(N * 11 * 4);
            L.dc_misc = take(64);
        }
    } else {
        L.tpart = take(T * 4);
        L.rcc = take(R * 4);
        L.rz = take(R * 4);
    }
    L.total = o;
    return L;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

int bits_for(uint64_t n) {   // bits needed to hold values 0..n-1
    int b = 1;
    while (b < 32 && ((uint64_t)1 << b) < n) ++b;
    return b;
}

}  // namespace

// ---------------------------------------------------------------- static scratch

// Device memory of vf_query_views_noalloc: one array per GPU the library runs
// on, in the code object's zero-initialised data, held until the process ends.
// In host code `scratch` is only a stand-in for the symbol: its device address
// is taken once per device with hipGetSymbolAddress (scratch_address below)
// and only that address is ever handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[GV_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// The current device's scratch address (the caller has made `device`
// current); taken on the first request for each device and kept.
hipError_t scratch_address(int device, unsigned char **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

namespace {
const char *const kStageNames[GV_PROFILE_STAGES] = {"cull", "project", "sort_depth", "emit", "sort_tile",
                                                     "ranges", "raster_vis", "vf_accum", "raster_uq"};
enum Stage { ST_CULL, ST_PROJECT, ST_SORT_DEPTH, ST_EMIT, ST_SORT_TILE, ST_RANGES, ST_RASTER_VIS, ST_ACCUM,
             ST_RASTER_UQ };
struct ProfEvent {
    int stage;
    hipEvent_t a, b;
};
}  // namespace

struct gv_context {
    int device = 0;
    unsigned long long *dev_counters = nullptr;   // sizing counters
    int32_t *host_best = nullptr;       // pinned host word the device argmax writes
    int32_t *host_best_dev = nullptr;   // its device address
    ViewDev *dev_views = nullptr;                 // view table for sizing passes
    size_t dev_views_cap = 0;
    std::vector<ViewDev> host_views;
    std::vector<float> host_centres;
    // captured query sequences, most recent last
    struct Graph {
        std::vector<unsigned char> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Graph> graphs;
    // this device's static scratch (vf_query_views_noalloc); NULL if its
    // address could not be taken, with the reason in scratch_err
    unsigned char *scratch = nullptr;
    std::string scratch_err;
    bool capturing = false;
    gv_tuning tuning = {64, 256, 2, 0};   // the autotuned choice on the room workload
    hipStream_t cap_stream = nullptr;   // private stream used only to record graphs
    // stage timing
    bool prof_on = false;
    std::vector<ProfEvent> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    hipEvent_t prof_event() {
        if (!prof_pool.empty()) {
            hipEvent_t e = prof_pool.back();
            prof_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

namespace {
// Records a pair of events around one stage while profiling is enabled.
struct StageScope {
    gv_context *c;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr;
    StageScope(gv_context *c_, int st, hipStream_t s_) : c(c_), stage(st), s(s_) {
        if (c && c->prof_on && !c->capturing) {
            a = c->prof_event();
            if (a && hipEventRecord(a, s) != hipSuccess) a = nullptr;
        }
    }
    ~StageScope() {
        if (!a) return;
        hipEvent_t b = c->prof_event();
        if (b && hipEventRecord(b, s) == hipSuccess) c->prof_pending.push_back({stage, a, b});
    }
};
}  // namespace

// Fills host view descriptors; returns total tiles and pixels.
static gv_status make_views(const gv_camera *cams, int32_t n, std::vector<ViewDev> &out, int64_t &tiles,
                            int64_t &pixels) {
    out.resize((size_t)n);
    tiles = 0;
    pixels = 0;
    for (int32_t i = 0; i < n; ++i) {
        const gv_camera &c = cams[i];
        if (c.width < 1 || c.height < 1 || c.width > GV_MAX_IMAGE_SIDE || c.height > GV_MAX_IMAGE_SIDE)
            return fail(GV_ERR_INVALID_ARG, "camera %d: image size %dx%d outside 1..%d", i, c.width, c.height,
                        GV_MAX_IMAGE_SIDE);
        if (!finite_cam(c)) return fail(GV_ERR_INVALID_ARG, "camera %d: non-finite or non-positive parameters", i);
        ViewDev &V = out[(size_t)i];
        std::memset(&V, 0, sizeof(V));
        std::memcpy(V.R, c.R, sizeof(V.R));
        std::memcpy(V.t, c.t, sizeof(V.t));
        V.fx = c.fx; V.fy = c.fy; V.cx = c.cx; V.cy = c.cy;
        for (int k = 0; k < 3; ++k) {
            const double C = -((double)c.R[0 * 3 + k] * c.t[0] + (double)c.R[1 * 3 + k] * c.t[1] +
                               (double)c.R[2 * 3 + k] * c.t[2]);
            V.C[k] = (float)C;
        }
        V.w = c.width;
        V.h = c.height;
        V.tiles_x = (c.width + TILE - 1) / TILE;
        V.tiles_y = (c.height + TILE - 1) / TILE;
        V.tile_base = (int32_t)tiles;
        V.pix_base = pixels;
        tiles += (int64_t)V.tiles_x * V.tiles_y;
        pixels += (int64_t)c.width * c.height;
        if (tiles > (int64_t)1 << 30) return fail(GV_ERR_INVALID_ARG, "too many tiles in one call");
    }
    return GV_OK;
}

static gv_status check_gauss(const gv_gaussians *g) {
    if (!g) return fail(GV_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0 || g->n_virtual < 0 || g->n_virtual > g->n)
        return fail(GV_ERR_INVALID_ARG, "bad Gaussian counts n=%lld n_virtual=%lld", (long long)g->n,
                    (long long)g->n_virtual);
    if (g->n > ((int64_t)1 << 31) - 2) return fail(GV_ERR_INVALID_ARG, "n too large");
    if (g->dtype != GV_F32 && g->dtype != GV_F16 && g->dtype != GV_BF16)
        return fail(GV_ERR_INVALID_ARG, "bad Gaussian dtype %d", (int)g->dtype);
    if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacity))
        return fail(GV_ERR_INVALID_ARG, "NULL Gaussian attribute pointer");
    if (g->dtype != GV_F32 && g->n > 0 && (!g->anchors || g->anchor_block < 1))
        return fail(GV_ERR_INVALID_ARG, "half-precision means need anchors and anchor_block >= 1");
    return GV_OK;
}

static GaussArgs gargs(const gv_gaussians *g) {
    GaussArgs a;
    a.n = g->n;
    a.n_virtual = g->n_virtual;
    a.dtype = (int)g->dtype;
    a.means = g->means;
    a.scales = g->scales;
    a.quats = g->quats;
    a.opacity = g->opacity;
    a.anchors = g->anchors;
    a.anchor_block = g->anchor_block;
    return a;
}

static gv_status geom_ok(float znear, float lowpass, float cut, float eps_T) {
    if (!(std::isfinite(znear) && znear > 0.f)) return fail(GV_ERR_INVALID_ARG, "znear must be > 0");
    if (!(std::isfinite(lowpass) && lowpass >= 0.f)) return fail(GV_ERR_INVALID_ARG, "lowpass must be >= 0");
    if (!(std::isfinite(cut) && cut > 0.f)) return fail(GV_ERR_INVALID_ARG, "cut must be > 0");
    if (!(std::isfinite(eps_T) && eps_T > 0.f && eps_T < 1.f)) return fail(GV_ERR_INVALID_ARG, "eps_T must be in (0, 1)");
    return GV_OK;
}

// Measures one set of views: conservative records and exact instances.
static gv_status measure(gv_context *ctx, const gv_gaussians *g, const std::vector<ViewDev> &views,
                         const GeomArgs &geo, uint64_t &R, uint64_t &M, hipStream_t s) {
    R = M = 0;
    if (views.empty() || g->n == 0) return GV_OK;
    const size_t need = views.size() * sizeof(ViewDev);
    if (need > ctx->dev_views_cap) {
        if (ctx->dev_views) (void)hipFree(ctx->dev_views);
        ctx->dev_views = nullptr;
        ctx->dev_views_cap = 0;
        if (hipMalloc((void **)&ctx->dev_views, need) != hipSuccess)
            return fail(GV_ERR_OUT_OF_MEMORY, "cannot allocate %zu bytes for a view table", need);
        ctx->dev_views_cap = need;
    }
    GV_HIP(hipMemcpyAsync(ctx->dev_views, views.data(), need, hipMemcpyHostToDevice, s));
    GV_HIP(hipMemsetAsync(ctx->dev_counters, 0, 4 * sizeof(unsigned long long), s));
    launch_measure(gargs(g), ctx->dev_views, (int)views.size(), geo, ctx->dev_counters, s);
    GV_HIP(hipGetLastError());
    unsigned long long h[2] = {0, 0};
    GV_HIP(hipMemcpyAsync(h, ctx->dev_counters, sizeof(h), hipMemcpyDeviceToHost, s));
    GV_HIP(hipStreamSynchronize(s));
    R = h[0];
    M = h[1];
    return GV_OK;
}

static gv_status plan_check(const gv_workspace *plan, const void *ws, int kind, int64_t n, int32_t nv,
                            int64_t tiles, int64_t pixels) {
    if (!plan || !ws) return fail(GV_ERR_INVALID_ARG, "NULL workspace or plan");
    // a density-control plan (kind 2) holds the build layout and more
    if (plan->kind != kind && !(kind == 0 && plan->kind == 2))
        return fail(GV_ERR_INVALID_ARG, "workspace plan made for another call");
    if (plan->n != n) return fail(GV_ERR_INVALID_ARG, "workspace plan made for n=%lld, got %lld",
                                  (long long)plan->n, (long long)n);
    if (nv > plan->n_views || tiles > plan->total_tiles || pixels > plan->total_pixels)
        return fail(GV_ERR_CAPACITY, "workspace plan too small for these views");
    if (tiles >= (int64_t)TILE_KEY_MASK)
        return fail(GV_ERR_UNSUPPORTED, "%lld tiles in one pass; at most %u", (long long)tiles, TILE_KEY_MASK - 1u);
    if (plan->max_records < 0 || plan->max_instances < 0 || plan->max_records > 0x7fffffffLL ||
        plan->max_instances > 0x7fffffffLL)
        return fail(GV_ERR_INVALID_ARG, "workspace capacities out of range");
    if (plan->emit_mode < 0 || plan->emit_mode > 2) return fail(GV_ERR_INVALID_ARG, "emit_mode must be 0, 1 or 2");
    if (plan->bytes < make_layout(*plan).total) return fail(GV_ERR_CAPACITY, "workspace plan bytes too small");
    return GV_OK;
}

// The shared binning sequence; returns the sorted tile keys/values buffers.
struct Binned {
    const uint32_t *sval;   // record ids in depth order
    const uint32_t *ival;   // record ids in (tile, depth) order
    const uint32_t *ikey;   // their instance keys (tile id, quadrant mask)
    const uint32_t *torder; // tiles by decreasing list length (schedules 2 and 4), else NULL
};

// zero_a, zero_b (build): per-record words that the projection sets to zero
// for every record slot it writes.
static gv_status run_binning(gv_context *ctx, const gv_workspace &p, const Layout &L, void *ws, const GaussArgs &a, int nv,
                             int64_t tiles, const GeomArgs &geo, const QueryArgs *query, hipStream_t s, Binned &out,
                             int order, uint32_t *zero_a = nullptr, uint32_t *zero_b = nullptr) {
    Status *st = at<Status>(ws, L.status);
    ViewDev *views = at<ViewDev>(ws, L.views);
    uint32_t *cnt = at<uint32_t>(ws, L.cnt), *offs = at<uint32_t>(ws, L.offs), *vmask = at<uint32_t>(ws, L.vmask);
    unsigned long long *blk = at<unsigned long long>(ws, L.blk);
    Rec *rec = at<Rec>(ws, L.rec);
    Bin *bin = at<Bin>(ws, L.bin);
    uint32_t *k0 = at<uint32_t>(ws, L.key0), *v0 = at<uint32_t>(ws, L.val0);
    uint32_t *k1 = at<uint32_t>(ws, L.key1), *v1 = at<uint32_t>(ws, L.val1);
    const bool lookback = emit_lookback(p);
    unsigned long long *post = lookback ? at<unsigned long long>(ws, L.post) : nullptr;
    // scanned emission: the projection packs each record's tile count into its
    // depth-sort value (or, for plans of 2^PACK_SHIFT records and more, writes
    // the counts apart and the last depth pass gathers them)
    const bool packed = !lookback && (uint64_t)p.max_records < ((uint64_t)1 << PACK_SHIFT);
    uint32_t *ntr = lookback || packed ? nullptr : at<uint32_t>(ws, L.ntr);
    uint32_t *icnt = lookback ? nullptr : at<uint32_t>(ws, L.icnt), *ioff = lookback ? nullptr : at<uint32_t>(ws, L.ioff);
    uint32_t *ik0 = at<uint32_t>(ws, L.ikey0), *iv0 = at<uint32_t>(ws, L.ival0);
    uint32_t *ik1 = at<uint32_t>(ws, L.ikey1), *iv1 = at<uint32_t>(ws, L.ival1);
    uint2 *ranges = at<uint2>(ws, L.ranges);
    uint32_t *hist = at<uint32_t>(ws, L.hist), *dtot = at<uint32_t>(ws, L.dtot);
    const uint64_t R = (uint64_t)p.max_records, M = (uint64_t)p.max_instances;

    {
        StageScope sc(ctx, ST_CULL, s);
        // the count also clears the status and the tile ranges
        launch_count(a, views, nv, geo, cnt, vmask, reinterpret_cast<uint32_t *>(st), sizeof(Status) / 4,
                     reinterpret_cast<uint32_t *>(ranges), (uint64_t)tiles * 2, s);
        const uint64_t ne = (uint64_t)a.n * PROJ_SPLIT;
        launch_scan(cnt, offs, nullptr, ne, ne, blk, &st->R_total, &st->R_eff, R, &st->overflow, 1u, s);
    }
    {
        StageScope sc(ctx, ST_PROJECT, s);
        launch_project(a, views, nv, geo, offs, vmask, st, (uint32_t)R, query, rec, k0, bin, packed ? v0 : ntr, packed,
                       zero_a, zero_b, s);
    }
    int dres;
    {
        StageScope sc(ctx, ST_SORT_DEPTH, s);
        // scanned emission: the last pass also writes each record's tile count
        // in depth order (the count its packed value carries, or gathered);
        // only the depth order of the records is used, not their sorted keys
        dres = launch_radix_sort(k0, v0, k1, v1, &st->R_eff, 32, !packed, hist, dtot, s, DEAD_KEY, nullptr, R, ntr,
                                 icnt, false, packed ? bin : nullptr);
    }
    const uint32_t *sval = dres ? v1 : v0;
    {
        StageScope sc(ctx, ST_EMIT, s);
        const float qc = (float)(0.5 * geo.cut / std::log(2.0));
        if (lookback) {
            launch_emit(sval, bin, post, st, R, M, qc, (uint32_t)tiles, ik0, iv0, s);
        } else {
            launch_scan(icnt, ioff, &st->R_eff, 0, R, blk, &st->M_total, &st->M_eff, M, &st->overflow, 2u, s);
            launch_emit_scanned(sval, bin, ioff, st, qc, (uint32_t)tiles, ik0, iv0, packed ? PACK_RMASK : 0xFFFFFFFFu, s);
        }
    }
    int tres;
    {
        StageScope sc(ctx, ST_SORT_TILE, s);
        // tile ids 0..tiles - 1; the first pass drops the dead instances (tile
        // id `tiles`) and leaves the live count in M_live
        tres = launch_radix_sort(ik0, iv0, ik1, iv1, &st->M_eff, bits_for((uint64_t)tiles), false, hist, dtot, s,
                                 (uint32_t)tiles, &st->M_live, M);
    }
    const uint32_t *skey = tres ? ik1 : ik0;
    out.torder = nullptr;
    {
        StageScope sc(ctx, ST_RANGES, s);
        launch_ranges(skey, st, (uint32_t)tiles, ranges, s);
        if (order == 2 || order == 4)
            out.torder = launch_tile_order(ranges, (uint32_t)tiles, at<uint32_t>(ws, L.torder),
                                           at<uint32_t>(ws, L.torder) + 4 * (uint64_t)tiles, hist, dtot, s);
    }
    out.sval = sval;
    out.ival = tres ? iv1 : iv0;
    out.ikey = skey;
    return GV_OK;
}

// ============================================================================ C ABI

extern "C" {

const char *gv_last_error(void) { return g_err.c_str(); }

void gv_default_vf_params(gv_vf_params *p) {
    if (!p) return;
    p->sh_degree = 2;
    p->kappa = 1.0f;
    p->eps_T = 1e-4f;
    p->znear = 0.2f;
    p->lowpass = 0.3f;
    p->cut = 9.0f;
    p->views_per_pass = 0;
    p->accumulate = 0;
}

void gv_default_uq_params(gv_uq_params *p) {
    if (!p) return;
    p->beta = 0.5f;
    p->o0 = 0.15f;
    p->half_logdet_Q0 = 0.0f;
    p->half_logdet_Qc = (float)(3.0 * std::log(0.1));
    p->eps_T = 1e-4f;
    p->znear = 0.2f;
    p->lowpass = 0.3f;
    p->cut = 9.0f;
    p->write_maps = 0;
    p->use_graph = 0;
    p->count_pairs = 0;
    p->write_depth = 0;
}

gv_status gv_create(int device, gv_context **out) {
    if (!out) return fail(GV_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    GV_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(GV_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, ndev);
    DeviceGuard dg(device);
    gv_context *c = new gv_context();
    c->device = device;
    if (hipMalloc((void **)&c->dev_counters, 8 * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void **)&c->host_best, 64, hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->host_best_dev, c->host_best, 0) != hipSuccess) {
        if (c->dev_counters) (void)hipFree(c->dev_counters);
        if (c->host_best) (void)hipHostFree(c->host_best);
        (void)hipGetLastError();
        delete c;
        return fail(GV_ERR_OUT_OF_MEMORY, "cannot allocate context counters");
    }
    // the static scratch of vf_query_views_noalloc: its device address is
    // taken here, once per device, with that device current
    {
        const hipError_t e = scratch_address(device, &c->scratch);
        if (e != hipSuccess) {
            c->scratch = nullptr;
            c->scratch_err = hipGetErrorString(e);
            (void)hipGetLastError();
        }
    }
    // host view table of the no-allocation call, so that it never grows there
    c->host_views.reserve(GV_NOALLOC_MAX_VIEWS);
    *out = c;
    return GV_OK;
}

void gv_destroy(gv_context *ctx) {
    if (!ctx) return;
    DeviceGuard dg(ctx->device);
    if (ctx->dev_counters) (void)hipFree(ctx->dev_counters);
    if (ctx->host_best) (void)hipHostFree(ctx->host_best);
    if (ctx->dev_views) (void)hipFree(ctx->dev_views);
    for (const ProfEvent &e : ctx->prof_pending) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
    for (auto &gr : ctx->graphs) {
        (void)hipGraphExecDestroy(gr.exec);
        (void)hipGraphDestroy(gr.graph);
    }
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

size_t gv_workspace_bytes(const gv_workspace *plan) {
    if (!plan) return 0;
    return make_layout(*plan).total;
}

static gv_status build_plan(gv_context *ctx, const gv_gaussians *g, const gv_camera *train, int32_t n_train,
                            const gv_vf_params *prm, gv_workspace *plan, void *hip_stream);

gv_status vf_build_workspace_size(gv_context *ctx, const gv_gaussians *g, const gv_camera *train, int32_t n_train,
                                  const gv_vf_params *prm, gv_workspace *plan, void *hip_stream) {
    return build_plan(ctx, g, train, n_train, prm, plan, hip_stream);
}

static gv_status build_plan(gv_context *ctx, const gv_gaussians *g, const gv_camera *train, int32_t n_train,
                            const gv_vf_params *prm, gv_workspace *plan, void *hip_stream) {
    if (!ctx || !prm || !plan) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    GV_TRY(check_gauss(g));
    if (n_train < 0 || (n_train > 0 && !train)) return fail(GV_ERR_INVALID_ARG, "bad training views");
    if (prm->sh_degree < 0 || prm->sh_degree > GV_MAX_SH_DEGREE)
        return fail(GV_ERR_UNSUPPORTED, "sh_degree %d not in 0..%d", prm->sh_degree, GV_MAX_SH_DEGREE);
    GV_TRY(geom_ok(prm->znear, prm->lowpass, prm->cut, prm->eps_T));
    DeviceGuard dg(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const int32_t vp = prm->views_per_pass > 0 ? std::min(prm->views_per_pass, std::max(n_train, 1)) : std::max(n_train, 1);
    std::memset(plan, 0, sizeof(*plan));
    plan->kind = 0;
    plan->n = g->n;
    plan->sh_degree = prm->sh_degree;
    plan->n_views = vp;
    const GeomArgs geo{prm->znear, prm->lowpass, prm->cut};
    for (int32_t v0 = 0; v0 < n_train; v0 += vp) {
        const int32_t nv = std::min(vp, n_train - v0);
        std::vector<ViewDev> views;
        int64_t tiles, pixels;
        GV_TRY(make_views(train + v0, nv, views, tiles, pixels));
        uint64_t R, M;
        GV_TRY(measure(ctx, g, views, geo, R, M, s));
        plan->max_records = std::max<int64_t>(plan->max_records, (int64_t)R);
        plan->max_instances = std::max<int64_t>(plan->max_instances, (int64_t)M);
        plan->total_tiles = (int32_t)std::max<int64_t>(plan->total_tiles, tiles);
        plan->total_pixels = std::max<int64_t>(plan->total_pixels, pixels);
    }
    if (plan->max_records > 0x7fffffffLL || plan->max_instances > 0x7fffffffLL)
        return fail(GV_ERR_CAPACITY, "one pass needs more than 2^31 records or instances; lower views_per_pass");
    plan->emit_mode = emit_mode_for(*plan);
    plan->bytes = make_layout(*plan).total;
    return GV_OK;
}

gv_status vf_query_workspace_size(gv_context *ctx, const gv_gaussians *g, const gv_camera *cand, int32_t n_cand,
                                  const gv_uq_params *prm, int32_t sh_degree, gv_workspace *plan, void *hip_stream) {
    if (!ctx || !prm || !plan) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    GV_TRY(check_gauss(g));
    if (n_cand < 1 || !cand) return fail(GV_ERR_INVALID_ARG, "need at least one candidate view");
    if (sh_degree < 0 || sh_degree > GV_MAX_SH_DEGREE)
        return fail(GV_ERR_UNSUPPORTED, "sh_degree %d not in 0..%d", sh_degree, GV_MAX_SH_DEGREE);
    GV_TRY(geom_ok(prm->znear, prm->lowpass, prm->cut, prm->eps_T));
    DeviceGuard dg(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<ViewDev> views;
    int64_t tiles, pixels;
    GV_TRY(make_views(cand, n_cand, views, tiles, pixels));
    uint64_t R, M;
    GV_TRY(measure(ctx, g, views, GeomArgs{prm->znear, prm->lowpass, prm->cut}, R, M, s));
    std::memset(plan, 0, sizeof(*plan));
    plan->kind = 1;
    plan->n = g->n;
    plan->sh_degree = sh_degree;
    plan->n_views = n_cand;
    plan->max_records = (int64_t)R;
    plan->max_instances = (int64_t)M;
    plan->total_tiles = (int32_t)tiles;
    plan->total_pixels = pixels;
    if (plan->max_records > 0x7fffffffLL || plan->max_instances > 0x7fffffffLL)
        return fail(GV_ERR_CAPACITY, "more than 2^31 records or instances in one call; split the views");
    plan->emit_mode = emit_mode_for(*plan);
    plan->bytes = make_layout(*plan).total;
    return GV_OK;
}

gv_status vf_build(gv_context *ctx, const gv_gaussians *g, const gv_camera *train, int32_t n_train,
                   const gv_vf_params *prm, void *gamma, gv_dtype gamma_dtype, const gv_workspace *plan,
                   void *workspace, void *hip_stream) {
    if (!ctx || !prm) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    GV_TRY(check_gauss(g));
    if (n_train < 0 || (n_train > 0 && !train)) return fail(GV_ERR_INVALID_ARG, "bad training views");
    if (prm->sh_degree < 0 || prm->sh_degree > GV_MAX_SH_DEGREE)
        return fail(GV_ERR_UNSUPPORTED, "sh_degree %d not in 0..%d", prm->sh_degree, GV_MAX_SH_DEGREE);
    if (!(std::isfinite(prm->kappa) && prm->kappa >= 0.f)) return fail(GV_ERR_INVALID_ARG, "kappa must be >= 0");
    GV_TRY(geom_ok(prm->znear, prm->lowpass, prm->cut, prm->eps_T));
    if (gamma_dtype != GV_F32 && gamma_dtype != GV_F16 && gamma_dtype != GV_BF16)
        return fail(GV_ERR_INVALID_ARG, "bad gamma dtype");
    if (g->n > 0 && !gamma) return fail(GV_ERR_INVALID_ARG, "gamma is NULL");
    if (!plan || !workspace) return fail(GV_ERR_INVALID_ARG, "NULL workspace or plan");
    if (plan->sh_degree != prm->sh_degree) return fail(GV_ERR_INVALID_ARG, "plan made for another sh_degree");
    DeviceGuard dg(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const int L = prm->sh_degree;
    const int K = (L + 1) * (L + 1);
    float al[4] = {0, 0, 0, 0};
    for (int l = 0; l <= L; ++l) al[l] = (float)(4.0 * M_PI * std::exp(-(double)prm->kappa) * bessel_i(l, prm->kappa));
    const int32_t vp = prm->views_per_pass > 0 ? std::min(prm->views_per_pass, std::max(n_train, 1)) : std::max(n_train, 1);
    const Layout Lay = make_layout(*plan);
    const GaussArgs a = gargs(g);
    const GeomArgs geo{prm->znear, prm->lowpass, prm->cut};
    const float qcut = (float)(0.5 * prm->cut / std::log(2.0));
    const bool half_out = gamma_dtype != GV_F32;
    float *gam32 = at<float>(workspace, Lay.gam32);
    // target of the per-pass accumulation: the FP32 output directly, or an
    // FP32 copy that is rounded to the half output at the end
    void *acc_target = half_out ? (void *)gam32 : gamma;
    if (g->n == 0) return GV_OK;
    if (n_train == 0) {
        if (!prm->accumulate) {
            if (half_out) launch_fill_u32((uint32_t *)gamma, ((uint64_t)g->n * K + 1) / 2, 0u, s);
            else launch_fill_u32((uint32_t *)gamma, (uint64_t)g->n * K, 0u, s);
        }
        GV_HIP(hipGetLastError());
        return GV_OK;
    }
    bool acc = prm->accumulate != 0;
    if (half_out) {
        // FP32 staging of the half output: start from it (accumulate) or from 0
        if (acc) launch_convert(gamma, (int)gamma_dtype, gam32, 0, (uint64_t)g->n * K, s);
        else launch_fill_u32((uint32_t *)gam32, (uint64_t)g->n * K, 0u, s);
        acc = true;
    }
    for (int32_t v0 = 0; v0 < n_train; v0 += vp) {
        const int32_t nv = std::min(vp, n_train - v0);
        std::vector<ViewDev> &views = ctx->host_views;
        int64_t tiles, pixels;
        GV_TRY(make_views(train + v0, nv, views, tiles, pixels));
        GV_TRY(plan_check(plan, workspace, 0, g->n, nv, tiles, pixels));
        GV_HIP(hipMemcpyAsync(at<ViewDev>(workspace, Lay.views), views.data(), views.size() * sizeof(ViewDev),
                              hipMemcpyHostToDevice, s));
        Status *st = at<Status>(workspace, Lay.status);
        float *accT = at<float>(workspace, Lay.accT);
        uint32_t *accC = at<uint32_t>(workspace, Lay.accC);
        Binned bz;
        GV_TRY(run_binning(ctx, *plan, Lay, workspace, a, nv, tiles, geo, nullptr, s, bz, ctx->tuning.vis_order,
                           reinterpret_cast<uint32_t *>(accT), accC));
        {
            StageScope sc(ctx, ST_RASTER_VIS, s);
            launch_raster_vis(at<ViewDev>(workspace, Lay.views), nv, (int)tiles, at<uint2>(workspace, Lay.ranges),
                              bz.ival, bz.ikey, at<Rec>(workspace, Lay.rec), prm->eps_T, qcut, accT, accC,
                              ctx->tuning.vis_batch, ctx->tuning.vis_order, bz.torder, st->tile_ticket, s);
        }
        {
            StageScope sc(ctx, ST_ACCUM, s);
            launch_vf_accum(a, at<ViewDev>(workspace, Lay.views), at<uint32_t>(workspace, Lay.offs),
                            at<uint32_t>(workspace, Lay.vmask), mask_words(nv), accT, accC, st, L, al, acc_target,
                            half_out ? 0 : (int)gamma_dtype, acc, &st->measure[0], s);
        }
        GV_HIP(hipGetLastError());
        if (v0 + vp < n_train) {
            // the next pass reuses the workspace; its status must be read now
            // to report an overflow of this pass
            Status h;
            GV_HIP(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
            GV_HIP(hipStreamSynchronize(s));
            if (h.overflow) return fail(GV_ERR_CAPACITY, "workspace too small for views %d..%d", v0, v0 + nv - 1);
        }
        acc = true;
    }
    if (half_out) launch_convert(gam32, 0, gamma, (int)gamma_dtype, (uint64_t)g->n * K, s);
    GV_HIP(hipGetLastError());
    return GV_OK;
}

}  // extern "C"

// Single-view visibility of every training view, pass by pass (Alg. 2).
// multi = true: visibility[g] = 1 - prod_p (1 - v_p[g]) (Alg. 5);
// multi = false: visibility[p * n + g] = v_p[g].
static gv_status view_visibility(gv_context *ctx, const gv_gaussians *g, const gv_camera *train, int32_t n_train,
                                 const gv_vf_params *prm, float *visibility, bool multi, const gv_workspace *plan,
                                 void *workspace, void *hip_stream) {
    if (!ctx || !prm) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    GV_TRY(check_gauss(g));
    if (n_train < 0 || (n_train > 0 && !train)) return fail(GV_ERR_INVALID_ARG, "bad training views");
    GV_TRY(geom_ok(prm->znear, prm->lowpass, prm->cut, prm->eps_T));
    if (g->n > 0 && (multi || n_train > 0) && !visibility) return fail(GV_ERR_INVALID_ARG, "visibility is NULL");
    if (!plan || !workspace) return fail(GV_ERR_INVALID_ARG, "NULL workspace or plan");
    DeviceGuard dg(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    if (g->n == 0) return GV_OK;
    if (n_train == 0) {
        if (multi) launch_fill_u32(reinterpret_cast<uint32_t *>(visibility), (uint64_t)g->n, 0u, s);
        GV_HIP(hipGetLastError());
        return GV_OK;
    }
    const int32_t vp = prm->views_per_pass > 0 ? std::min(prm->views_per_pass, n_train) : n_train;
    const Layout Lay = make_layout(*plan);
    const GaussArgs a = gargs(g);
    const GeomArgs geo{prm->znear, prm->lowpass, prm->cut};
    const float qcut = (float)(0.5 * prm->cut / std::log(2.0));
    bool acc = false;
    for (int32_t v0 = 0; v0 < n_train; v0 += vp) {
        const int32_t nv = std::min(vp, n_train - v0);
        std::vector<ViewDev> &views = ctx->host_views;
        int64_t tiles, pixels;
        GV_TRY(make_views(train + v0, nv, views, tiles, pixels));
        GV_TRY(plan_check(plan, workspace, 0, g->n, nv, tiles, pixels));
        GV_HIP(hipMemcpyAsync(at<ViewDev>(workspace, Lay.views), views.data(), views.size() * sizeof(ViewDev),
                              hipMemcpyHostToDevice, s));
        Status *st = at<Status>(workspace, Lay.status);
        float *accT = at<float>(workspace, Lay.accT);
        uint32_t *accC = at<uint32_t>(workspace, Lay.accC);
        Binned bz;
        GV_TRY(run_binning(ctx, *plan, Lay, workspace, a, nv, tiles, geo, nullptr, s, bz, ctx->tuning.vis_order,
                           reinterpret_cast<uint32_t *>(accT), accC));
        {
            StageScope sc(ctx, ST_RASTER_VIS, s);
            launch_raster_vis(at<ViewDev>(workspace, Lay.views), nv, (int)tiles, at<uint2>(workspace, Lay.ranges),
                              bz.ival, bz.ikey, at<Rec>(workspace, Lay.rec), prm->eps_T, qcut, accT, accC,
                              ctx->tuning.vis_batch, ctx->tuning.vis_order, bz.torder, st->tile_ticket, s);
        }
        {
            StageScope sc(ctx, ST_ACCUM, s);
            if (multi) {
                launch_vis_logsum(g->n, at<uint32_t>(workspace, Lay.offs), accT, accC, st, visibility, acc,
                                  &st->measure[0], s);
            } else {
                float *rows = visibility + (int64_t)v0 * g->n;
                launch_fill_u32(reinterpret_cast<uint32_t *>(rows), (uint64_t)nv * (uint64_t)g->n, 0u, s);
                launch_view_vis(a, at<uint32_t>(workspace, Lay.offs), at<uint32_t>(workspace, Lay.vmask),
                                mask_words(nv), accT, accC, st, rows, &st->measure[0], s);
            }
        }
        GV_HIP(hipGetLastError());
        if (v0 + vp < n_train) {
            Status h;
            GV_HIP(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
            GV_HIP(hipStreamSynchronize(s));
            if (h.overflow) return fail(GV_ERR_CAPACITY, "workspace too small for views %d..%d", v0, v0 + nv - 1);
        }
        acc = true;
    }
    if (multi) launch_vis_finish(g->n, visibility, s);
    GV_HIP(hipGetLastError());
    return GV_OK;
}

extern "C" {

gv_status vf_multiview_visibility(gv_context *ctx, const gv_gaussians *g, const gv_camera *train, int32_t n_train,
                                  const gv_vf_params *prm, float *visibility, const gv_workspace *plan,
                                  void *workspace, void *hip_stream) {
    return view_visibility(ctx, g, train, n_train, prm, visibility, true, plan, workspace, hip_stream);
}

// Alg. 5's particle count and scale from the box and density: N_virt =
// floor(rho * volume), (4/3) pi s^3 rho = 1 + eta.
static gv_status virtual_count(const gv_density_params *dp, int64_t *nv, double *s) {
    if (!dp) return fail(GV_ERR_INVALID_ARG, "NULL density parameters");
    double vol = 1.0;
    for (int k = 0; k < 3; ++k) {
        if (!(std::isfinite(dp->lo[k]) && std::isfinite(dp->hi[k]) && dp->hi[k] > dp->lo[k]))
            return fail(GV_ERR_INVALID_ARG, "empty or non-finite box along axis %d", k);
        vol *= (double)dp->hi[k] - (double)dp->lo[k];
    }
    if (!(std::isfinite(dp->rho) && dp->rho > 0.f && std::isfinite(dp->eta) && dp->eta > -1.f &&
          std::isfinite(dp->eps_v)))
        return fail(GV_ERR_INVALID_ARG, "density parameters out of range");
    const double cnt = std::floor((double)dp->rho * vol);
    if (cnt > (double)(((int64_t)1 << 31) - 2)) return fail(GV_ERR_CAPACITY, "too many virtual particles");
    *nv = (int64_t)cnt;
    *s = std::cbrt(3.0 * (1.0 + (double)dp->eta) / (4.0 * M_PI * (double)dp->rho));
    return GV_OK;
}

// Checks of the density-control arguments shared by the sizing call and the
// call itself; writes the virtual particles into rows n_real.. of g.
static gv_status place_virtual(const gv_gaussians *g, int64_t n_real, const float *u, int64_t n_draw,
                               const gv_density_params *dp, int64_t *nv_out, hipStream_t s) {
    GV_TRY(check_gauss(g));
    if (g->dtype != GV_F32) return fail(GV_ERR_UNSUPPORTED, "density control takes FP32 attribute arrays");
    if (g->n_virtual != 0) return fail(GV_ERR_INVALID_ARG, "every Gaussian is measured: n_virtual must be 0");
    int64_t nv;
    double sc;
    GV_TRY(virtual_count(dp, &nv, &sc));
    if (n_real < 0 || g->n != n_real + nv)
        return fail(GV_ERR_INVALID_ARG, "the arrays must hold n_real + N_virt = %lld + %lld rows, n = %lld",
                    (long long)n_real, (long long)nv, (long long)g->n);
    if (n_draw < nv || (nv > 0 && !u)) return fail(GV_ERR_INVALID_ARG, "%lld uniform draws for %lld particles",
                                                   (long long)n_draw, (long long)nv);
    VirtArgs va;
    for (int k = 0; k < 3; ++k) {
        va.lo[k] = (double)dp->lo[k];
        va.span[k] = (double)dp->hi[k] - (double)dp->lo[k];
    }
    va.s = (float)sc;
    launch_place_virtual((float *)g->means, (float *)g->scales, (float *)g->quats, (float *)g->opacity, u, n_real, nv,
                         va, s);
    GV_HIP(hipGetLastError());
    *nv_out = nv;
    return GV_OK;
}

gv_status vf_virtual_particle_count(const gv_density_params *dp, int64_t *n_virt, float *scale) {
    int64_t nv;
    double sc;
    GV_TRY(virtual_count(dp, &nv, &sc));
    if (n_virt) *n_virt = nv;
    if (scale) *scale = (float)sc;
    return GV_OK;
}

gv_status vf_density_control_workspace_size(gv_context *ctx, const gv_gaussians *g, int64_t n_real, const float *u,
                                            int64_t n_draw, const gv_density_params *dp, const gv_camera *train,
                                            int32_t n_train, const gv_vf_params *prm, gv_workspace *plan,
                                            int64_t *n_virt, void *hip_stream) {
    if (!ctx || !prm || !plan) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    DeviceGuard dg(ctx->device);
    int64_t nv;
    GV_TRY(place_virtual(g, n_real, u, n_draw, dp, &nv, (hipStream_t)hip_stream));
    GV_TRY(build_plan(ctx, g, train, n_train, prm, plan, hip_stream));
    plan->kind = 2;
    plan->bytes = make_layout(*plan).total;
    if (n_virt) *n_virt = nv;
    return GV_OK;
}

gv_status vf_density_control(gv_context *ctx, const gv_gaussians *g, int64_t n_real, const float *u, int64_t n_draw,
                             const gv_density_params *dp, const gv_camera *train, int32_t n_train,
                             const gv_vf_params *prm, float *visibility, int32_t *kept, int64_t *n_kept,
                             const gv_workspace *plan, void *workspace, void *hip_stream) {
    if (!ctx || !prm || !n_kept) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    if (!plan || plan->kind != 2 || !workspace) return fail(GV_ERR_INVALID_ARG, "needs a density-control plan");
    DeviceGuard dg(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    *n_kept = 0;
    int64_t nv;
    GV_TRY(place_virtual(g, n_real, u, n_draw, dp, &nv, s));
    if (g->n > 0 && !visibility) return fail(GV_ERR_INVALID_ARG, "visibility is NULL");
    if (nv > 0 && !kept) return fail(GV_ERR_INVALID_ARG, "kept is NULL");
    if (g->n > plan->n) return fail(GV_ERR_INVALID_ARG, "plan made for fewer Gaussians");
    GV_TRY(view_visibility(ctx, g, train, n_train, prm, visibility, true, plan, workspace, hip_stream));
    if (nv == 0) return GV_OK;
    const Layout Lay = make_layout(*plan);
    uint32_t *flags = at<uint32_t>(workspace, Lay.dc_flags), *offs = at<uint32_t>(workspace, Lay.dc_offs);
    float *tmp = at<float>(workspace, Lay.dc_tmp);
    unsigned long long *tot = at<unsigned long long>(workspace, Lay.dc_misc);
    uint32_t *eff = reinterpret_cast<uint32_t *>(tot + 1), *ovf = eff + 1;
    float *means = (float *)g->means, *scales = (float *)g->scales, *quats = (float *)g->quats,
          *opac = (float *)g->opacity;
    launch_fill_u32(ovf, 1, 0u, s);
    launch_virtual_flags(visibility, n_real, nv, dp->eps_v, flags, s);
    launch_scan(flags, offs, nullptr, (uint64_t)nv, (uint64_t)nv, at<unsigned long long>(workspace, Lay.blk), tot, eff,
                (uint64_t)nv, ovf, 1u, s);
    launch_virtual_pack(flags, offs, n_real, nv, means, scales, quats, opac, kept, tmp, s);
    unsigned long long h = 0;
    Status hs;
    GV_HIP(hipMemcpyAsync(&h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
    GV_HIP(hipMemcpyAsync(&hs, at<Status>(workspace, Lay.status), sizeof(hs), hipMemcpyDeviceToHost, s));
    GV_HIP(hipStreamSynchronize(s));
    if (hs.overflow) return fail(GV_ERR_CAPACITY, "workspace too small for the density control's views");
    launch_virtual_store(tmp, n_real, (int64_t)h, means, scales, quats, opac, s);
    GV_HIP(hipGetLastError());
    *n_kept = (int64_t)h;
    return GV_OK;
}

gv_status vf_view_visibility(gv_context *ctx, const gv_gaussians *g, const gv_camera *train, int32_t n_train,
                             const gv_vf_params *prm, float *view_vis, float *train_centres,
                             const gv_workspace *plan, void *workspace, void *hip_stream) {
    GV_TRY(view_visibility(ctx, g, train, n_train, prm, view_vis, false, plan, workspace, hip_stream));
    if (train_centres && n_train > 0) {
        DeviceGuard dg(ctx->device);
        std::vector<float> &hc = ctx->host_centres;
        hc.resize((size_t)n_train * 3);
        for (int32_t p = 0; p < n_train; ++p) {
            const gv_camera &c = train[p];
            for (int k = 0; k < 3; ++k)
                hc[(size_t)p * 3 + k] = (float)(-((double)c.R[0 * 3 + k] * c.t[0] + (double)c.R[1 * 3 + k] * c.t[1] +
                                                   (double)c.R[2 * 3 + k] * c.t[2]));
        }
        GV_HIP(hipMemcpyAsync(train_centres, hc.data(), hc.size() * sizeof(float), hipMemcpyHostToDevice,
                              (hipStream_t)hip_stream));
    }
    return GV_OK;
}

}  // extern "C"

// Alg. 6 over the candidate views with the visibility source `q` (the SH
// field of Alg. 4 or the exact product of eq. vis_all).
static gv_status query_views(gv_context *ctx, const gv_gaussians *g, const QueryArgs &q, const gv_camera *cand,
                             int32_t n_cand, const gv_uq_params *prm, float *scores, float *maps,
                             const gv_workspace *plan, void *workspace, void *hip_stream) {
    if (n_cand < 1 || !cand) return fail(GV_ERR_INVALID_ARG, "need at least one candidate view");
    if (!scores) return fail(GV_ERR_INVALID_ARG, "scores is NULL");
    GV_TRY(geom_ok(prm->znear, prm->lowpass, prm->cut, prm->eps_T));
    if (!(prm->beta >= 0.f && prm->beta <= 1.f && prm->o0 >= 0.f && prm->o0 <= 1.f))
        return fail(GV_ERR_INVALID_ARG, "beta and o0 must lie in [0, 1]");
    if (!std::isfinite(prm->half_logdet_Q0) || !std::isfinite(prm->half_logdet_Qc))
        return fail(GV_ERR_INVALID_ARG, "non-finite covariance log-determinants");
    if (prm->write_maps && !maps) return fail(GV_ERR_INVALID_ARG, "write_maps set but maps is NULL");
    if (prm->write_depth && !prm->write_maps) return fail(GV_ERR_INVALID_ARG, "write_depth needs write_maps");
    DeviceGuard dg(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<ViewDev> &views = ctx->host_views;
    int64_t tiles, pixels;
    GV_TRY(make_views(cand, n_cand, views, tiles, pixels));
    GV_TRY(plan_check(plan, workspace, 1, g->n, n_cand, tiles, pixels));
    const Layout Lay = make_layout(*plan);
    GV_HIP(hipMemcpyAsync(at<ViewDev>(workspace, Lay.views), views.data(), views.size() * sizeof(ViewDev),
                          hipMemcpyHostToDevice, s));
    const GaussArgs a = gargs(g);
    const GeomArgs geo{prm->znear, prm->lowpass, prm->cut};
    const double c3 = 1.5 * std::log(2.0 * M_PI * M_E);
    UqArgs u;
    u.beta = prm->beta;
    u.o0 = prm->o0;
    u.cQc = (float)(prm->half_logdet_Qc + c3);
    u.cQ0 = (float)(prm->half_logdet_Q0 + c3);
    u.eps_T = prm->eps_T;
    u.qcut = (float)(0.5 * prm->cut / std::log(2.0));
    float *mp = prm->write_maps ? maps : nullptr;
    float *dmp = prm->write_maps && prm->write_depth ? maps + pixels : nullptr;
    QueryArgs qa = q;
    qa.c3 = (float)c3;
    qa.rcc = q.color_var ? at<float>(workspace, Lay.rcc) : nullptr;
    qa.rz = dmp ? at<float>(workspace, Lay.rz) : nullptr;
    auto enqueue = [&]() -> gv_status {
        Binned bz;
        GV_TRY(run_binning(ctx, *plan, Lay, workspace, a, n_cand, tiles, geo, &qa, s, bz, ctx->tuning.uq_order));
        float *tpart = at<float>(workspace, Lay.tpart);
        {
            StageScope sc(ctx, ST_RASTER_UQ, s);
            Status *st = at<Status>(workspace, Lay.status);
            launch_raster_uq(at<ViewDev>(workspace, Lay.views), n_cand, (int)tiles, at<uint2>(workspace, Lay.ranges),
                             bz.ival, at<Rec>(workspace, Lay.rec), qa.rcc, qa.rz, u, tpart, mp, dmp,
                             prm->count_pairs ? &st->measure[0] : nullptr, ctx->tuning.uq_batch, ctx->tuning.uq_order, bz.torder,
                             st->tile_ticket, s);
        }
        launch_scores(at<ViewDev>(workspace, Lay.views), n_cand, tpart, at<Status>(workspace, Lay.status), scores, s);
        return GV_OK;
    };
    if (!prm->use_graph) {
        GV_TRY(enqueue());
        GV_HIP(hipGetLastError());
        return GV_OK;
    }
    // Graph path: every kernel argument and grid of the sequence is fixed by
    // the key below (the cameras themselves live in the view table, uploaded
    // above on the same stream before the replay).
    // (the whole plan is part of the key: the workspace's region offsets
    // follow from its capacities, view count and tile count; the call's
    // pixel total places the depth maps behind the entropy maps)
    struct Key {
        const void *ws, *gamma, *vtrain, *tc, *cvar, *scores, *maps, *means, *scales, *quats, *opac, *anchors;
        int64_t n, n_virtual, tiles, pixels;
        gv_workspace plan;
        int32_t mode, n_cand, sh, gdt, dtype, anchor_block, count, uq_batch, uq_order, ntv, csh, depth;
        float f[10];
    } key;
    std::memset(&key, 0, sizeof(key));
    key.ws = workspace; key.gamma = q.gamma; key.vtrain = q.view_vis; key.tc = q.train_centres;
    key.cvar = q.color_var; key.csh = q.color_sh_degree; key.depth = dmp != nullptr;
    key.scores = scores; key.maps = mp;
    key.means = g->means; key.scales = g->scales; key.quats = g->quats; key.opac = g->opacity; key.anchors = g->anchors;
    key.n = g->n; key.n_virtual = g->n_virtual; key.tiles = tiles; key.pixels = pixels;
    key.plan = *plan;
    key.mode = q.mode; key.n_cand = n_cand; key.sh = q.sh_degree; key.gdt = q.gamma_dtype; key.dtype = (int)g->dtype;
    key.anchor_block = g->anchor_block; key.count = prm->count_pairs;
    key.uq_batch = ctx->tuning.uq_batch; key.uq_order = ctx->tuning.uq_order;
    key.ntv = q.n_train_views;
    const float fv[10] = {prm->beta, prm->o0, prm->half_logdet_Q0, prm->half_logdet_Qc, prm->eps_T, prm->znear,
                          prm->lowpass, prm->cut, q.n_train, q.kappa};
    std::memcpy(key.f, fv, sizeof(fv));
    const unsigned char *kb = reinterpret_cast<const unsigned char *>(&key);
    std::vector<unsigned char> kv(kb, kb + sizeof(key));
    for (size_t i = 0; i < ctx->graphs.size(); ++i) {
        if (ctx->graphs[i].key == kv) {
            GV_HIP(hipGraphLaunch(ctx->graphs[i].exec, s));
            return GV_OK;
        }
    }
    gv_context::Graph gr;
    gr.key = kv;
    if (!ctx->cap_stream) GV_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    // record on the private stream (the caller's may be the legacy default
    // stream, which cannot be captured), replay on the caller's stream
    const hipStream_t user_s = s;
    s = ctx->cap_stream;
    GV_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    const gv_status est = enqueue();
    ctx->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(s, &graph);
    s = user_s;
    if (est != GV_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return est;
    }
    if (ce != hipSuccess) return fail(GV_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ce));
    gr.graph = graph;
    GV_HIP(hipGraphInstantiate(&gr.exec, graph, nullptr, nullptr, 0));
    if (ctx->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        (void)hipGraphDestroy(ctx->graphs.front().graph);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back(gr);
    GV_HIP(hipGraphLaunch(gr.exec, s));
    return GV_OK;
}

extern "C" {

}  // extern "C"

// Argument checks shared by vf_query_views and vf_query_views_noalloc.
static gv_status check_query_args(gv_context *ctx, const gv_gaussians *g, const void *gamma, gv_dtype gamma_dtype,
                                  int32_t sh_degree, int64_t n_train, const gv_uq_params *prm) {
    if (!ctx || !prm) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    GV_TRY(check_gauss(g));
    if (sh_degree < 0 || sh_degree > GV_MAX_SH_DEGREE)
        return fail(GV_ERR_UNSUPPORTED, "sh_degree %d not in 0..%d", sh_degree, GV_MAX_SH_DEGREE);
    if (n_train < 0) return fail(GV_ERR_INVALID_ARG, "n_train < 0");
    if (n_train > 0 && g->n > 0 && !gamma) return fail(GV_ERR_INVALID_ARG, "gamma is NULL");
    if (gamma_dtype != GV_F32 && gamma_dtype != GV_F16 && gamma_dtype != GV_BF16)
        return fail(GV_ERR_INVALID_ARG, "bad gamma dtype");
    return GV_OK;
}

extern "C" {

gv_status vf_query_views(gv_context *ctx, const gv_gaussians *g, const void *gamma, gv_dtype gamma_dtype,
                         int32_t sh_degree, int64_t n_train, const gv_camera *cand, int32_t n_cand,
                         const gv_uq_params *prm, float *scores, float *maps, const gv_workspace *plan,
                         void *workspace, void *hip_stream) {
    GV_TRY(check_query_args(ctx, g, gamma, gamma_dtype, sh_degree, n_train, prm));
    if (plan && plan->sh_degree != sh_degree) return fail(GV_ERR_INVALID_ARG, "plan made for another sh_degree");
    QueryArgs q = {1, sh_degree, gamma, (int)gamma_dtype, (float)n_train, nullptr, nullptr, 0, 0.f};
    return query_views(ctx, g, q, cand, n_cand, prm, scores, maps, plan, workspace, hip_stream);
}

gv_status vf_query_views_noalloc(gv_context *ctx, const gv_gaussians *g, const void *gamma, gv_dtype gamma_dtype,
                                 int32_t sh_degree, int64_t n_train, const gv_camera *cand, int32_t n_cand,
                                 const gv_uq_params *prm, float *scores, float *maps, void *hip_stream) {
    GV_TRY(check_query_args(ctx, g, gamma, gamma_dtype, sh_degree, n_train, prm));
    if (n_cand < 1 || !cand) return fail(GV_ERR_INVALID_ARG, "need at least one candidate view");
    if (n_cand > GV_NOALLOC_MAX_VIEWS)
        return fail(GV_ERR_CAPACITY, "%d candidate views; the no-allocation call takes at most %d", n_cand,
                    GV_NOALLOC_MAX_VIEWS);
    if (prm->use_graph) return fail(GV_ERR_INVALID_ARG, "use_graph is not available without allocation");
    GV_TRY(geom_ok(prm->znear, prm->lowpass, prm->cut, prm->eps_T));
    if (!ctx->scratch)
        return fail(GV_ERR_HIP, "the static scratch has no device address: %s", ctx->scratch_err.c_str());
    DeviceGuard dg(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<ViewDev> &views = ctx->host_views;   // reserved for GV_NOALLOC_MAX_VIEWS at gv_create
    int64_t tiles, pixels;
    GV_TRY(make_views(cand, n_cand, views, tiles, pixels));
    // sizing pass: the view table goes where the query's layout keeps it
    // (its offset depends on no capacity), the counters are the context's
    gv_workspace plan;
    std::memset(&plan, 0, sizeof(plan));
    plan.kind = 1;
    plan.n = g->n;
    plan.sh_degree = sh_degree;
    plan.n_views = n_cand;
    plan.total_tiles = (int32_t)tiles;
    plan.total_pixels = pixels;
    const size_t views_at = make_layout(plan).views;
    if (views_at + views.size() * sizeof(ViewDev) > (size_t)GV_NOALLOC_SCRATCH_BYTES)
        return fail(GV_ERR_CAPACITY, "view table does not fit the static scratch");
    ViewDev *dviews = reinterpret_cast<ViewDev *>(ctx->scratch + views_at);
    uint64_t R = 0, M = 0;
    if (g->n > 0) {
        GV_HIP(hipMemcpyAsync(dviews, views.data(), views.size() * sizeof(ViewDev), hipMemcpyHostToDevice, s));
        GV_HIP(hipMemsetAsync(ctx->dev_counters, 0, 4 * sizeof(unsigned long long), s));
        launch_measure(gargs(g), dviews, n_cand, GeomArgs{prm->znear, prm->lowpass, prm->cut}, ctx->dev_counters, s);
        GV_HIP(hipGetLastError());
        unsigned long long h[2] = {0, 0};
        GV_HIP(hipMemcpyAsync(h, ctx->dev_counters, sizeof(h), hipMemcpyDeviceToHost, s));
        GV_HIP(hipStreamSynchronize(s));
        R = h[0];
        M = h[1];
    }
    if (R > 0x7fffffffULL || M > 0x7fffffffULL)
        return fail(GV_ERR_CAPACITY, "more than 2^31 records or instances in one call; split the views");
    plan.max_records = (int64_t)R;
    plan.max_instances = (int64_t)M;
    plan.bytes = make_layout(plan).total;
    if (plan.bytes > (size_t)GV_NOALLOC_SCRATCH_BYTES)
        return fail(GV_ERR_CAPACITY, "these views need %zu bytes of workspace; the static scratch holds %zu "
                                     "(use vf_query_views with a caller workspace)",
                    plan.bytes, (size_t)GV_NOALLOC_SCRATCH_BYTES);
    QueryArgs q = {1, sh_degree, gamma, (int)gamma_dtype, (float)n_train, nullptr, nullptr, 0, 0.f};
    return query_views(ctx, g, q, cand, n_cand, prm, scores, maps, &plan, ctx->scratch, hip_stream);
}

gv_status vf_query_views_color(gv_context *ctx, const gv_gaussians *g, const void *gamma, gv_dtype gamma_dtype,
                               int32_t sh_degree, int64_t n_train, const float *color_var, int32_t color_sh_degree,
                               const gv_camera *cand, int32_t n_cand, const gv_uq_params *prm, float *scores,
                               float *maps, const gv_workspace *plan, void *workspace, void *hip_stream) {
    if (!ctx || !prm) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    GV_TRY(check_gauss(g));
    if (sh_degree < 0 || sh_degree > GV_MAX_SH_DEGREE)
        return fail(GV_ERR_UNSUPPORTED, "sh_degree %d not in 0..%d", sh_degree, GV_MAX_SH_DEGREE);
    if (color_sh_degree < 0 || color_sh_degree > GV_MAX_SH_DEGREE)
        return fail(GV_ERR_UNSUPPORTED, "color_sh_degree %d not in 0..%d", color_sh_degree, GV_MAX_SH_DEGREE);
    if (n_train < 0) return fail(GV_ERR_INVALID_ARG, "n_train < 0");
    if (g->n > 0 && !color_var) return fail(GV_ERR_INVALID_ARG, "color_var is NULL");
    if (n_train > 0 && g->n > 0 && !gamma) return fail(GV_ERR_INVALID_ARG, "gamma is NULL");
    if (gamma_dtype != GV_F32 && gamma_dtype != GV_F16 && gamma_dtype != GV_BF16)
        return fail(GV_ERR_INVALID_ARG, "bad gamma dtype");
    if (plan && plan->sh_degree != sh_degree) return fail(GV_ERR_INVALID_ARG, "plan made for another sh_degree");
    QueryArgs q = {1, sh_degree, gamma, (int)gamma_dtype, (float)n_train, nullptr, nullptr, 0, 0.f};
    q.color_var = color_var;
    q.color_sh_degree = color_sh_degree;
    return query_views(ctx, g, q, cand, n_cand, prm, scores, maps, plan, workspace, hip_stream);
}

gv_status vf_query_views_exact(gv_context *ctx, const gv_gaussians *g, const float *view_vis,
                               const float *train_centres, int32_t n_train, float kappa, const gv_camera *cand,
                               int32_t n_cand, const gv_uq_params *prm, float *scores, float *maps,
                               const gv_workspace *plan, void *workspace, void *hip_stream) {
    if (!ctx || !prm) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    GV_TRY(check_gauss(g));
    if (n_train < 0) return fail(GV_ERR_INVALID_ARG, "n_train < 0");
    if (n_train > 0 && g->n > 0 && (!view_vis || !train_centres))
        return fail(GV_ERR_INVALID_ARG, "view_vis or train_centres is NULL");
    if (!(std::isfinite(kappa) && kappa >= 0.f)) return fail(GV_ERR_INVALID_ARG, "kappa must be >= 0");
    QueryArgs q = {2, 0, nullptr, 0, (float)n_train, view_vis, train_centres, n_train, kappa};
    return query_views(ctx, g, q, cand, n_cand, prm, scores, maps, plan, workspace, hip_stream);
}

gv_status gv_workspace_check(gv_context *ctx, const gv_workspace *plan, const void *workspace, int64_t out[4],
                             void *hip_stream) {
    if (!ctx || !plan || !workspace) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    DeviceGuard dg(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const Layout Lay = make_layout(*plan);
    Status h;
    GV_HIP(hipMemcpyAsync(&h, static_cast<const char *>(workspace) + Lay.status, sizeof(h), hipMemcpyDeviceToHost, s));
    GV_HIP(hipStreamSynchronize(s));
    if (out) {
        out[0] = (int64_t)h.R_total;
        out[1] = (int64_t)h.M_total;
        out[2] = (int64_t)h.overflow;
        out[3] = (int64_t)h.measure[0];
    }
    if (h.overflow) return fail(GV_ERR_CAPACITY, "workspace capacity exceeded (records %llu, instances %llu)",
                                h.R_total, h.M_total);
    return GV_OK;
}

gv_status gv_profile_enable(gv_context *ctx, int32_t on) {
    if (!ctx) return fail(GV_ERR_INVALID_ARG, "NULL context");
    ctx->prof_on = on != 0;
    return GV_OK;
}

gv_status gv_profile_read(gv_context *ctx, double *ms, int64_t *calls, void *hip_stream) {
    if (!ctx || !ms || !calls) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    DeviceGuard dg(ctx->device);
    GV_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
    for (int i = 0; i < GV_PROFILE_STAGES; ++i) {
        ms[i] = 0.0;
        calls[i] = 0;
    }
    for (const ProfEvent &e : ctx->prof_pending) {
        float t = 0.f;
        if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&t, e.a, e.b) == hipSuccess) {
            ms[e.stage] += t;
            calls[e.stage] += 1;
        }
        ctx->prof_pool.push_back(e.a);
        ctx->prof_pool.push_back(e.b);
    }
    ctx->prof_pending.clear();
    return GV_OK;
}

gv_status gv_set_tuning(gv_context *ctx, const gv_tuning *t) {
    if (!ctx || !t) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    auto ok = [](int b) { return b == 64 || b == 128 || b == 256; };
    if (!ok(t->vis_batch) || !ok(t->uq_batch)) return fail(GV_ERR_INVALID_ARG, "batch sizes must be 64, 128 or 256");
    if (t->vis_order < 0 || t->vis_order > 4 || t->uq_order < 0 || t->uq_order > 4)
        return fail(GV_ERR_INVALID_ARG, "tile orders must be 0 to 4");
    ctx->tuning = *t;
    return GV_OK;
}

gv_status gv_get_tuning(const gv_context *ctx, gv_tuning *t) {
    if (!ctx || !t) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    *t = ctx->tuning;
    return GV_OK;
}

const char *gv_profile_stage_name(int32_t stage) {
    if (stage < 0 || stage >= GV_PROFILE_STAGES) return "";
    return kStageNames[stage];
}

gv_status select_next_view(gv_context *ctx, const float *scores, int32_t n, int32_t *best, void *hip_stream) {
    if (!ctx || !scores || !best) return fail(GV_ERR_INVALID_ARG, "NULL argument");
    if (n < 1) return fail(GV_ERR_INVALID_ARG, "n must be >= 1");
    DeviceGuard dg(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    // the argmax writes the index straight into pinned host memory: no copy
    // operation after the kernel, only the wait for it
    launch_argmax(scores, n, ctx->host_best_dev, s);
    GV_HIP(hipGetLastError());
    GV_HIP(hipStreamSynchronize(s));
    *best = *reinterpret_cast<volatile int32_t *>(ctx->host_best);
    return GV_OK;
}

}  // extern "C"
