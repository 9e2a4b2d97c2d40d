// Host side of the C ABI declared in include/rtg.h: plan and workspace
// layout, argument checks, launches.  The kernels are compiled into this one
// translation unit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rtg.h"
#include "binning.hip"
#include "adding.hip"
#include "optim.hip"
#include "harness.hip"
#include "icp.hip"
#include "project.hip"
#include "raster.hip"
#include "rtg_common.h"

using namespace rtg;

enum Off { O_HDR, O_REC, O_ZKEY, O_RECT, O_GRAD, O_VIS, O_TNPX, O_TSTART, O_TEND, O_HIST, O_PIX,
           O_PXLAST, O_ITEMS, O_PAIRS, O_KEYS, O_BIGL, O_BIGL2, O_BIGR, O_SCRATCH, O_WCOUNT, O_LPART, O_PREC, O_MASKEFF, O_LWAVE,
           O_RECP, O_STAGEC, O_VCNT, O_VLIST, O_CHUNK, O_COUNT };

struct rtg_plan {
    rtg_config cfg;
    rtg_intrinsics intr;
    Dims d;
    size_t off[O_COUNT + 1];
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

WS make_ws(const rtg_plan* p, void* base) {
    char* b = static_cast<char*>(base);
    WS w;
    w.hdr = reinterpret_cast<Hdr*>(b + p->off[O_HDR]);
    w.rec = reinterpret_cast<float4*>(b + p->off[O_REC]);
    w.zkey = reinterpret_cast<float*>(b + p->off[O_ZKEY]);
    w.rect = reinterpret_cast<short4*>(b + p->off[O_RECT]);
    w.grad = reinterpret_cast<float*>(b + p->off[O_GRAD]);
    w.vis = reinterpret_cast<uint32_t*>(b + p->off[O_VIS]);
    w.tile_npx = reinterpret_cast<uint32_t*>(b + p->off[O_TNPX]);
    w.tile_start = reinterpret_cast<uint32_t*>(b + p->off[O_TSTART]);
    w.tile_end = reinterpret_cast<uint32_t*>(b + p->off[O_TEND]);
    w.hist = reinterpret_cast<uint32_t*>(b + p->off[O_HIST]);
    w.pix = reinterpret_cast<uint8_t*>(b + p->off[O_PIX]);
    w.px_aux = reinterpret_cast<uint32_t*>(b + p->off[O_PXLAST]);
    w.items = reinterpret_cast<uint32_t*>(b + p->off[O_ITEMS]);
    w.pairs = reinterpret_cast<uint32_t*>(b + p->off[O_PAIRS]);
    w.bigl = reinterpret_cast<uint32_t*>(b + p->off[O_BIGL]);
    w.bigl2 = reinterpret_cast<uint32_t*>(b + p->off[O_BIGL2]);
    w.bigr = reinterpret_cast<uint32_t*>(b + p->off[O_BIGR]);
    w.keys = reinterpret_cast<unsigned long long*>(b + p->off[O_KEYS]);
    w.scratch = reinterpret_cast<unsigned long long*>(b + p->off[O_SCRATCH]);
    w.wcount = reinterpret_cast<unsigned long long*>(b + p->off[O_WCOUNT]);
    w.lwave = reinterpret_cast<float*>(b + p->off[O_LWAVE]);
    w.prec = reinterpret_cast<float4*>(b + p->off[O_PREC]);
    w.recp = reinterpret_cast<float*>(b + p->off[O_RECP]);
    w.stagec = reinterpret_cast<uint32_t*>(b + p->off[O_STAGEC]);
    w.bfail = w.stagec + 256;
    w.vcnt = reinterpret_cast<uint32_t*>(b + p->off[O_VCNT]);
    w.vlist = reinterpret_cast<uint8_t*>(b + p->off[O_VLIST]);
    w.chunk = reinterpret_cast<unsigned long long*>(b + p->off[O_CHUNK]);
    return w;
}

bool ws_ok(const rtg_plan* p, const void* ws) {
    return p && ws && (reinterpret_cast<uintptr_t>(ws) & 255) == 0;
}

hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

rtg_status launched() { return hipGetLastError() == hipSuccess ? RTG_OK : RTG_E_HIP; }

unsigned grid_for(int64_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

// Persistent-grid size per device (CU count x resident blocks per CU).
struct DevInfo {
    int cus = 0;
    int fwd_blocks[2] = {0, 0}, bwd_blocks[2] = {0, 0};   // per depth mode
};
std::mutex g_dev_mu;
DevInfo g_dev[64];

rtg_status dev_info(DevInfo& out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return RTG_E_HIP;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DevInfo& di = g_dev[dev];
    if (di.cus == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            return RTG_E_UNSUPPORTED;
        const void* kf[2] = {reinterpret_cast<const void*>(k_raster_fwd<0>),
                             reinterpret_cast<const void*>(k_raster_fwd<1>)};
        const void* kb[2] = {reinterpret_cast<const void*>(k_raster_bwd<0>),
                             reinterpret_cast<const void*>(k_raster_bwd<1>)};
        for (int m = 0; m < 2; ++m) {
            int bf = 0, bb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bf, kf[m], 256, 0) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&bb, kb[m], 256, 0) != hipSuccess)
                return RTG_E_HIP;
            di.fwd_blocks[m] = std::min(cus * (bf > 0 ? bf : 1), kMaxWaves / 4);
            di.bwd_blocks[m] = std::min(cus * (bb > 0 ? bb : 1), kMaxWaves / 4);
        }
        di.cus = cus;
    }
    out = di;
    return RTG_OK;
}

// Fixed device scratch of rtg_forward_static: the workspace of callers that
// cannot allocate.  Host code never passes `scratch` itself (on the host it
// names a stand-in, not the device copy): the device address is looked up
// once per device with hipGetSymbolAddress and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[RTG_STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch[64];

rtg_status scratch_ptr(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return RTG_E_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RTG_E_HIP;
        if (reinterpret_cast<uintptr_t>(ptr) & 255) return RTG_E_HIP;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return RTG_OK;
}

}  // namespace

// Helpers of the adding and state-management entry points.
namespace {

AddParams add_params(const rtg_adding_params* p) {
    return AddParams{p->delta_T,        p->delta_d,        p->delta_c,      p->rate,
                     p->alpha_opaque,   p->alpha_transparent, p->r_transparent, p->thickness,
                     p->delta_eta,      p->delta_e,        p->delta_t,     p->sh_degree};
}

bool intr_ok(const rtg_intrinsics* c) {
    return c && c->width >= 1 && c->height >= 1 && c->width <= 32767 && c->height <= 32767 && c->fx > 0 &&
           c->fy > 0 && std::isfinite(c->fx) && std::isfinite(c->fy) && std::isfinite(c->cx) &&
           std::isfinite(c->cy);
}

Intr to_intr(const rtg_intrinsics* c) { return Intr{c->fx, c->fy, c->cx, c->cy, c->width, c->height}; }

// workspace of the adding passes: per-pixel codes, per-block counts and
// offsets, the candidate total
struct AddWs {
    size_t codes, counts, offsets, total, bytes;
};
AddWs add_ws(int64_t np) {
    const size_t nb = (size_t)((np + 255) / 256);
    AddWs w;
    w.codes = 0;
    w.counts = align256((size_t)np);
    w.offsets = w.counts + align256(4 * nb);
    w.total = w.offsets + align256(4 * nb);
    w.bytes = w.total + 256;
    return w;
}

__global__ void k_add_counts(const unsigned long long* total, int64_t n_cur, int64_t capacity, int64_t* out) {
    if (threadIdx.x == 0) {
        const int64_t t = (int64_t)*total;
        const int64_t room = capacity > n_cur ? capacity - n_cur : 0;
        out[0] = t < room ? t : room;
        out[1] = t;
    }
}

__global__ void k_copy_count(const unsigned long long* total, int64_t* out) {
    if (threadIdx.x == 0) out[0] = (int64_t)*total;
}

}  // namespace

extern "C" {

void rtg_config_default(rtg_config* c) {
    if (!c) return;
    c->tile_w = 16;
    c->tile_h = 16;
    c->cutoff2 = 9.0f;
    c->dilation = 0.0f;
    c->z_near = 0.2f;
    c->t_eps = 1e-8f;
    c->items_per_pop = 0;
    c->tile_filter50 = 0;
    c->sort_cap = 0;
    c->stage_cap = 0;
    c->sh_degree = 0;
    c->depth_mode = 0;
    c->straggler_lanes = 8;
    c->straggler_rest = 128;
    c->static_share = 0;
    c->fwd_items_per_pop = -1;
    c->fwd_static_share = -1;
}

rtg_status rtg_plan_create(const rtg_config* cfg, const rtg_intrinsics* intr, int64_t n, int32_t frames,
                           int64_t max_pairs, rtg_plan** out) {
    if (!cfg || !intr || !out) return RTG_E_INVALID;
    *out = nullptr;
    bool shape_ok = (cfg->tile_w == 8 && cfg->tile_h == 8) || (cfg->tile_w == 16 && cfg->tile_h == 16) ||
                    (cfg->tile_w == 32 && cfg->tile_h == 8);
    if (!shape_ok) return RTG_E_INVALID;
    if (n < 0 || frames < 1 || frames > RTG_MAX_FRAMES) return RTG_E_INVALID;
    if ((uint64_t)n * (uint64_t)frames >= (1ull << 32) || n >= (1ll << 30)) return RTG_E_INVALID;
    if (max_pairs < 1 || max_pairs >= (1ll << 31)) return RTG_E_INVALID;
    if (intr->width < 1 || intr->height < 1 || intr->width > 32767 || intr->height > 32767) return RTG_E_INVALID;
    if (!(intr->fx > 0) || !(intr->fy > 0) || !std::isfinite(intr->fx) || !std::isfinite(intr->fy) ||
        !std::isfinite(intr->cx) || !std::isfinite(intr->cy))
        return RTG_E_INVALID;
    if (!(cfg->cutoff2 > 0) || !(cfg->dilation >= 0) || !std::isfinite(cfg->z_near) || !(cfg->t_eps >= 0) ||
        cfg->items_per_pop < 0 || cfg->items_per_pop > 1024 || cfg->sort_cap < 0 || cfg->sort_cap > kSortLds ||
        cfg->stage_cap < 0 || cfg->sh_degree < 0 || cfg->sh_degree > 3 || cfg->depth_mode < 0 ||
        cfg->depth_mode > 1 || cfg->straggler_lanes < 0 || cfg->straggler_lanes > 32 || cfg->straggler_rest < 1 ||
        cfg->static_share < 0 || cfg->static_share > 100 || cfg->fwd_items_per_pop < -1 ||
        cfg->fwd_items_per_pop > 1024 || cfg->fwd_static_share < -1 || cfg->fwd_static_share > 100)
        return RTG_E_INVALID;
    rtg_plan* p = new (std::nothrow) rtg_plan;
    if (!p) return RTG_E_INVALID;
    p->cfg = *cfg;
    p->intr = *intr;
    Dims& d = p->d;
    d.N = n;
    d.F = frames;
    d.W = intr->width;
    d.H = intr->height;
    d.tw = cfg->tile_w;
    d.th = cfg->tile_h;
    d.tx = (d.W + d.tw - 1) / d.tw;
    d.ty = (d.H + d.th - 1) / d.th;
    d.ntiles = d.tx * d.ty;
    d.tarea = d.tw * d.th;
    d.ppt = (d.tarea + 63) / 64;
    d.lg_tw = ilog2(d.tw);
    d.fx = intr->fx;
    d.fy = intr->fy;
    d.cx = intr->cx;
    d.cy = intr->cy;
    d.cutoff2 = cfg->cutoff2;
    d.dilation = cfg->dilation;
    d.z_near = cfg->z_near;
    d.t_eps = cfg->t_eps;
    d.max_pairs = (uint32_t)max_pairs;
    d.items_per_pop = cfg->items_per_pop;
    d.sh_deg = cfg->sh_degree;
    d.depth_mode = cfg->depth_mode;
    d.strag_lanes = cfg->straggler_lanes;
    d.strag_rest = cfg->straggler_rest;
    d.static_share = cfg->static_share;
    d.fwd_items_per_pop = cfg->fwd_items_per_pop >= 0 ? cfg->fwd_items_per_pop : cfg->items_per_pop;
    d.fwd_static_share = cfg->fwd_static_share >= 0 ? cfg->fwd_static_share : cfg->static_share;
    d.sort_cap = cfg->sort_cap ? cfg->sort_cap : kSortLds;
    // runs of the long-list sort (sorted in LDS by one workgroup each):
    // kSortLds keys by default; with a smaller sort_cap, the power of two
    // >= 2 * sort_cap (at least 64, at most kSortLds)
    d.big_chunk = kSortLds;
    if (cfg->sort_cap) {
        int c = 64;
        while (c < 2 * cfg->sort_cap && c < kSortLds) c <<= 1;
        d.big_chunk = c;
    }
    // binning blocks: about 256 Gaussian ranges per frame (at least 256
    // Gaussians each), fewer when the per-(frame, block, tile) count matrix
    // would exceed 2^26 entries; tile chunks of at most kHistChunk tiles
    d.chunk = std::min(d.ntiles, kHistChunk);
    d.nchunks = (d.ntiles + d.chunk - 1) / d.chunk;
    {
        int64_t gpb = std::max<int64_t>(256, ((n + 255) / 256 + 255) / 256 * 256);
        int64_t nb = std::max<int64_t>(1, (n + gpb - 1) / gpb);
        while (nb > 1 && (int64_t)frames * nb * d.ntiles > (int64_t(1) << 26)) {
            gpb *= 2;
            nb = (n + gpb - 1) / gpb;
        }
        // small problems: halve the ranges (down to 256) while the count
        // matrix stays within 2^21 entries, so more workgroups share the
        // latency-bound enumeration
        while (gpb > 256 && (int64_t)frames * 2 * nb * d.ntiles <= (int64_t(1) << 21)) {
            gpb /= 2;
            nb = (n + gpb - 1) / gpb;
        }
        d.gpb = (int32_t)std::min<int64_t>(gpb, int64_t(1) << 30);
        d.nbpf = (int32_t)nb;
    }
    // staging regions over the pair records (64 bytes per pair of capacity,
    // four 16-byte entries): up to 256 regions, block k using region k mod
    // nreg, so a region serves many blocks and the claims on its counter
    // are few
    const int64_t nbb = (int64_t)frames * d.nbpf * d.nchunks;
    d.nreg = (int32_t)std::min<int64_t>(256, nbb);
    {
        const int64_t room = std::min<int64_t>(4 * max_pairs / d.nreg, 0x7fffffff);
        if (cfg->stage_cap > room) {
            delete p;
            return RTG_E_INVALID;
        }
        d.rcap = (uint32_t)(cfg->stage_cap ? cfg->stage_cap : room);
    }
    const size_t slots = (size_t)n * frames;
    const size_t ft = (size_t)frames * d.ntiles;
    size_t sz[O_COUNT];
    sz[O_HDR] = sizeof(Hdr);
    sz[O_REC] = 64 * slots;
    sz[O_ZKEY] = 4 * slots;
    sz[O_RECT] = 8 * slots;
    sz[O_GRAD] = 64 * slots;
    sz[O_VIS] = 4 * (size_t)n;
    sz[O_TNPX] = sz[O_TSTART] = sz[O_TEND] = 4 * ft;
    sz[O_HIST] = 4 * ft * (size_t)d.nbpf;
    sz[O_PIX] = ft * d.tarea;
    sz[O_PXLAST] = 8 * ft * d.tarea;
    sz[O_ITEMS] = 4 * ft * d.ppt;
    sz[O_PAIRS] = 4 * (size_t)max_pairs;
    sz[O_BIGL] = sz[O_BIGL2] = 4 * ft;
    sz[O_BIGR] = 4 * (ft + 1);
    sz[O_KEYS] = 8 * (size_t)max_pairs;
    sz[O_SCRATCH] = 8 * (size_t)max_pairs;
    sz[O_WCOUNT] = 8 * 4 * (size_t)kMaxWaves;
    sz[O_LWAVE] = 4 * 3 * (size_t)kMaxWaves;
    sz[O_LPART] = 12 * (size_t)grid_for((int64_t)ft * d.tarea, 256);
    sz[O_PREC] = 64 * (size_t)max_pairs;
    sz[O_MASKEFF] = cfg->tile_filter50 ? (size_t)frames * d.W * d.H : 0;
    sz[O_RECP] = 24 * slots;
    sz[O_STAGEC] = 4 * (256 + (size_t)nbb);
    d.ngrp = (n + 63) / 64;
    sz[O_VCNT] = 4 * (size_t)frames * d.ngrp;
    sz[O_VLIST] = 64 * (size_t)frames * d.ngrp;
    sz[O_CHUNK] = 8 * 16 * ((ft + 4095) / 4096);
    size_t o = 0;
    for (int k = 0; k < O_COUNT; ++k) {
        p->off[k] = o;
        o = align256(o + sz[k]);
    }
    p->off[O_COUNT] = o;
    *out = p;
    return RTG_OK;
}

void rtg_plan_destroy(rtg_plan* p) { delete p; }

size_t rtg_plan_workspace_bytes(const rtg_plan* p) { return p ? p->off[O_COUNT] : 0; }

int32_t rtg_plan_layout(const rtg_plan* p, int64_t* out, int32_t n) {
    if (!p || !out) return 0;
    const int idx[10] = {O_REC, O_ZKEY, O_RECT, O_VIS, O_TEND, O_TSTART, O_PAIRS, O_TNPX, O_GRAD, O_HDR};
    int k = 0;
    for (; k < n && k < 10; ++k) out[k] = (int64_t)p->off[idx[k]];
    return k;
}

rtg_status rtg_project(const rtg_plan* p, void* ws, const float* pos, const float* scale, const float* rot,
                       const float* opacity, const float* color, const uint8_t* unstable, const double* poses,
                       void* stream) {
    if (!ws_ok(p, ws) || !poses) return RTG_E_INVALID;
    if (p->d.N > 0 && (!pos || !scale || !rot || !opacity || !color || !unstable)) return RTG_E_INVALID;
    WS w = make_ws(p, ws);
    // the header is cleared by the first block of k_project; with N = 0 a
    // single block still runs for that
    unsigned g = grid_for(p->d.N, 256);
    hipLaunchKernelGGL(k_project, dim3(g ? g : 1), dim3(256), 0, S(stream), p->d, w, pos, scale, rot, opacity,
                       color, unstable, poses);
    if (p->d.sh_deg > 0 && g)
        hipLaunchKernelGGL(k_sh_color, dim3(g), dim3(256), 0, S(stream), p->d, w, pos, color, poses);
    return launched();
}

rtg_status rtg_unstable_mask(const rtg_plan* p, void* ws, uint8_t* mask_out, void* stream) {
    if (!ws_ok(p, ws) || !mask_out) return RTG_E_INVALID;
    WS w = make_ws(p, ws);
    size_t n = (size_t)p->d.F * p->d.W * p->d.H;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)std::min<size_t>((n + 255) / 256, 65535)), dim3(256), 0, S(stream),
                       mask_out, n, (uint8_t)0);
    if (launched() != RTG_OK) return RTG_E_HIP;
    if (p->d.N > 0)
        hipLaunchKernelGGL(k_unstable_mask, dim3(grid_for(p->d.N, 4)), dim3(256), 0, S(stream), p->d, w, mask_out);
    return launched();
}

namespace {

// Side stream of a device: the short-list and long-list sorts of rtg_bin
// run on it beside the mid-length sorts on the caller's stream (the run
// sorts and merges of the few long lists are launches that would otherwise
// leave much of the chip idle).  Created at the first eager
// binning call on the device and kept until the process ends; the lock
// orders the fork and join enqueues of concurrent callers.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kMaxSideDevices = 64;
constexpr int64_t kSideFrom = 16384;   // (frame, tile)s from which the sorts fork
std::mutex g_side_mu;
SideStream* g_side[kMaxSideDevices] = {};

// The current device's side stream, or nullptr (serial launches) when it
// does not exist yet and `caller` is being captured, or cannot be made.
SideStream* side_stream(hipStream_t caller) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxSideDevices) return nullptr;
    if (g_side[dev]) return g_side[dev];
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(caller, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    SideStream* ss = new (std::nothrow) SideStream;
    if (!ss) return nullptr;
    bool ok = hipStreamCreateWithFlags(&ss->s, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&ss->fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&ss->join, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        if (ss->join) (void)hipEventDestroy(ss->join);
        if (ss->fork) (void)hipEventDestroy(ss->fork);
        if (ss->s) (void)hipStreamDestroy(ss->s);
        delete ss;
        (void)hipGetLastError();
        return nullptr;
    }
    g_side[dev] = ss;
    return ss;
}

rtg_status bin_impl(const rtg_plan* p, void* ws, const uint8_t* mask, void* stream, bool allow_side);

}  // namespace

rtg_status rtg_bin(const rtg_plan* p, void* ws, const uint8_t* mask, void* stream) {
    return bin_impl(p, ws, mask, stream, true);
}

namespace {

rtg_status bin_impl(const rtg_plan* p, void* ws, const uint8_t* mask, void* stream, bool allow_side) {
    if (!ws_ok(p, ws) || !mask) return RTG_E_INVALID;
    WS w = make_ws(p, ws);
    const Dims& d = p->d;
    const uint8_t* m = mask;
    if (p->cfg.tile_filter50) {
        uint8_t* eff = static_cast<uint8_t*>(ws) + p->off[O_MASKEFF];
        int64_t blocks = (int64_t)d.F * ((d.W + 15) / 16) * ((d.H + 15) / 16);
        hipLaunchKernelGGL(k_filter50, dim3(grid_for(blocks, 4)), dim3(256), 0, S(stream), d, mask, eff);
        if (launched() != RTG_OK) return RTG_E_HIP;
        m = eff;
    }
    int64_t nft = (int64_t)d.F * d.ntiles;
    hipLaunchKernelGGL(k_tile_pixels, dim3(grid_for(nft, 4)), dim3(256), 0, S(stream), d, w, m);
    const unsigned nbb = (unsigned)((int64_t)d.F * d.nbpf * d.nchunks);
    const size_t lds = 4 * ((size_t)d.chunk + (d.chunk + 31) / 32);
    hipLaunchKernelGGL(k_pair_hist, dim3(nbb), dim3(256), lds, S(stream), d, w);
    if (nft >= kScanWideFrom)
        hipLaunchKernelGGL(k_hist_scan<64>, dim3(grid_for(nft, 64)), dim3(kScanThreads), 0, S(stream), d, w);
    else
        hipLaunchKernelGGL(k_hist_scan<16>, dim3(grid_for(nft, 16)), dim3(kScanThreads), 0, S(stream), d, w);
    if (nft <= 4096) {
        hipLaunchKernelGGL(k_tile_offsets, dim3(1), dim3(1024), 0, S(stream), d, w);
    } else {
        const unsigned nch = (unsigned)((nft + 4095) / 4096);
        hipLaunchKernelGGL(k_tile_chunk_sums, dim3(nch), dim3(1024), 0, S(stream), d, w);
        hipLaunchKernelGGL(k_tile_chunk_scan, dim3(1), dim3(1024), 0, S(stream), d, w, (int)nch);
        hipLaunchKernelGGL(k_tile_chunk_emit, dim3(nch), dim3(1024), 0, S(stream), d, w);
        hipLaunchKernelGGL(k_tile_big_order, dim3(1), dim3(1024), 0, S(stream), d, w);
    }
    // staged pairs: about 1024 of capacity per placing workgroup, at most
    // 16 workgroups per region
    const unsigned place_x =
        (unsigned)std::min<int64_t>(16, std::max<int64_t>(1, (int64_t)d.max_pairs / d.nreg / 1024));
    hipLaunchKernelGGL(k_pair_scatter, dim3(nbb + place_x * (unsigned)d.nreg), dim3(256), lds, S(stream), d, w, nbb,
                       place_x);
    if (launched() != RTG_OK) return RTG_E_HIP;
    // a listed tile holds more than sort_cap of at most max_pairs pairs
    const int64_t big_max = (int64_t)d.max_pairs / ((int64_t)d.sort_cap + 1) + 1;
    // run-sort jobs: at most max_pairs / big_chunk + one partial run per long list
    const int64_t jobs_max = (int64_t)d.max_pairs / d.big_chunk + std::min<int64_t>(big_max, nft);
    const unsigned jgrid = (unsigned)std::min<int64_t>(jobs_max, 1024);
    const int64_t big_grid = std::min<int64_t>(std::min<int64_t>(nft, 512), big_max);
    // the short lists, the run-sort jobs and the long-list merges on the
    // side stream, the mid-length lists on the caller's: they write
    // disjoint lists
    std::unique_lock<std::mutex> lock(g_side_mu, std::defer_lock);
    SideStream* side = nullptr;
    // (a small problem's sorts are short: there the cross-queue
    // synchronisation would cost more than the overlap gains)
    if (allow_side && nft >= kSideFrom) {
        lock.lock();
        side = side_stream(S(stream));
    }
    const hipStream_t sa = S(stream), sb = side ? side->s : sa;
    if (side && (hipEventRecord(side->fork, sa) != hipSuccess || hipStreamWaitEvent(sb, side->fork, 0) != hipSuccess))
        return RTG_E_HIP;
    hipLaunchKernelGGL(k_tile_sort_small, dim3((unsigned)((nft + 3) / 4)), dim3(256), 0, sb, d, w, (uint32_t)nft);
    if (side) {
        hipLaunchKernelGGL(k_tile_sort_runs, dim3(jgrid), dim3(256), 0, sb, d, w);
        hipLaunchKernelGGL(k_tile_sort_big, dim3((unsigned)big_grid), dim3(1024), 0, sb, d, w);
        hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)nft), dim3(256), 0, sa, d, w, 0u);
    } else {
        // one launch for the jobs and the mid-length lists, then the merges
        hipLaunchKernelGGL(k_tile_sort, dim3(jgrid + (unsigned)nft), dim3(256), 0, sa, d, w, jgrid);
        hipLaunchKernelGGL(k_tile_sort_big, dim3((unsigned)big_grid), dim3(1024), 0, sa, d, w);
    }
    if (side && (hipEventRecord(side->join, sb) != hipSuccess || hipStreamWaitEvent(sa, side->join, 0) != hipSuccess))
        return RTG_E_HIP;
    return launched();
}

}  // namespace

rtg_status rtg_render(const rtg_plan* p, void* ws, float* color, float* depth, float* trans, int32_t* index,
                      void* stream) {
    if (!ws_ok(p, ws) || !color || !depth || !trans || !index) return RTG_E_INVALID;
    DevInfo di;
    rtg_status st = dev_info(di);
    if (st != RTG_OK) return st;
    WS w = make_ws(p, ws);
    if (p->d.fwd_items_per_pop) hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, S(stream), &w.hdr->q_fwd);
    if (p->d.depth_mode == 0)
        hipLaunchKernelGGL(k_raster_fwd<0>, dim3(di.fwd_blocks[0]), dim3(256), 0, S(stream), p->d, w, color, depth,
                           trans, index);
    else
        hipLaunchKernelGGL(k_raster_fwd<1>, dim3(di.fwd_blocks[1]), dim3(256), 0, S(stream), p->d, w, color, depth,
                           trans, index);
    return launched();
}

rtg_status rtg_forward_static(const rtg_plan* p, const float* pos, const float* scale, const float* rot,
                              const float* opacity, const float* color, const uint8_t* unstable,
                              const double* poses, const uint8_t* mask, float* out_color, float* out_depth,
                              float* out_trans, int32_t* out_index, int32_t* status_out, void* stream) {
    if (!p) return RTG_E_INVALID;
    if (rtg_plan_workspace_bytes(p) > (size_t)RTG_STATIC_SCRATCH_BYTES) return RTG_E_TOO_LARGE;
    if (!poses || !mask || !out_color || !out_depth || !out_trans || !out_index) return RTG_E_INVALID;
    if (p->d.N > 0 && (!pos || !scale || !rot || !opacity || !color || !unstable)) return RTG_E_INVALID;
    void* ws = nullptr;
    rtg_status st = scratch_ptr(&ws);
    if (st != RTG_OK) return st;
    // projection clears the header (counters, overflow and error flags);
    // nothing else in the workspace is read before this call writes it
    if ((st = rtg_project(p, ws, pos, scale, rot, opacity, color, unstable, poses, stream)) != RTG_OK) return st;
    // (binning without the side stream: this call creates nothing)
    if ((st = bin_impl(p, ws, mask, stream, false)) != RTG_OK) return st;
    if ((st = rtg_render(p, ws, out_color, out_depth, out_trans, out_index, stream)) != RTG_OK) return st;
    if (status_out) {
        WS w = make_ws(p, ws);
        hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, S(stream), w, status_out);
        return launched();
    }
    return RTG_OK;
}

rtg_status rtg_backward(const rtg_plan* p, void* ws, const float* pos, const float* scale, const float* rot,
                        const float* opacity, const float* color, const uint8_t* unstable, const double* poses,
                        const float* out_depth, const float* out_trans, const int32_t* out_index,
                        const float* d_color, const float* d_depth, float* d_pos, float* d_scale, float* d_rot,
                        float* d_opacity, float* d_color_param, void* stream) {
    (void)opacity;
    if (!ws_ok(p, ws) || !poses || !out_depth || !out_trans || !out_index || !d_color || !d_depth)
        return RTG_E_INVALID;
    if (p->d.N > 0 && (!pos || !scale || !rot || !unstable || !d_pos || !d_scale || !d_rot || !d_opacity ||
                       !d_color_param || (p->d.sh_deg > 0 && !color)))
        return RTG_E_INVALID;
    rtg_status st = rtg_backward_raster(p, ws, out_depth, out_trans, out_index, d_color, d_depth, stream);
    if (st != RTG_OK) return st;
    return rtg_backward_project(p, ws, pos, scale, rot, color, unstable, poses, d_pos, d_scale, d_rot, d_opacity,
                                d_color_param, stream);
}

rtg_status rtg_backward_raster(const rtg_plan* p, void* ws, const float* out_depth, const float* out_trans,
                               const int32_t* out_index, const float* d_color, const float* d_depth,
                               void* stream) {
    if (!ws_ok(p, ws) || !out_depth || !out_trans || !out_index || !d_color || !d_depth) return RTG_E_INVALID;
    DevInfo di;
    rtg_status st = dev_info(di);
    if (st != RTG_OK) return st;
    WS w = make_ws(p, ws);
    const L1Up up = {nullptr, nullptr, nullptr, 0};
    if (p->d.items_per_pop) hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, S(stream), &w.hdr->q_bwd);
    if (p->d.depth_mode == 0)
        hipLaunchKernelGGL(k_raster_bwd<0>, dim3(di.bwd_blocks[0]), dim3(256), 0, S(stream), p->d, w, out_depth,
                           out_trans, out_index, d_color, d_depth, up);
    else
        hipLaunchKernelGGL(k_raster_bwd<1>, dim3(di.bwd_blocks[1]), dim3(256), 0, S(stream), p->d, w, out_depth,
                           out_trans, out_index, d_color, d_depth, up);
    return launched();
}

rtg_status rtg_backward_raster_l1(const rtg_plan* p, void* ws, const float* out_color, const float* out_depth,
                                  const float* out_trans, const int32_t* out_index, const float* color_gt,
                                  const float* depth_gt, void* stream) {
    if (!ws_ok(p, ws) || !out_color || !out_depth || !out_trans || !out_index || !color_gt || !depth_gt)
        return RTG_E_INVALID;
    // the fused form scales the colour-path and depth-path gradient slots
    // apart; the alpha-blended depth feeds the footprint and opacity slots
    // from both paths
    if (p->d.depth_mode != 0) return RTG_E_UNSUPPORTED;
    DevInfo di;
    rtg_status st = dev_info(di);
    if (st != RTG_OK) return st;
    WS w = make_ws(p, ws);
    const L1Up up = {out_color, color_gt, depth_gt, 1};
    if (p->d.items_per_pop) hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, S(stream), &w.hdr->q_bwd);
    if (p->d.depth_mode == 0)
        hipLaunchKernelGGL(k_raster_bwd<0>, dim3(di.bwd_blocks[0]), dim3(256), 0, S(stream), p->d, w, out_depth,
                           out_trans, out_index, (const float*)nullptr, (const float*)nullptr, up);
    else
        hipLaunchKernelGGL(k_raster_bwd<1>, dim3(di.bwd_blocks[1]), dim3(256), 0, S(stream), p->d, w, out_depth,
                           out_trans, out_index, (const float*)nullptr, (const float*)nullptr, up);
    return launched();
}

namespace {
rtg_status launch_project_bwd(const rtg_plan* p, void* ws, const float* pos, const float* scale, const float* rot,
                              const float* color, const uint8_t* unstable, const double* poses, float* d_pos,
                              float* d_scale, float* d_rot, float* d_opacity, float* d_color_param, L1Scale ls,
                              void* stream) {
    if (!ws_ok(p, ws) || !poses) return RTG_E_INVALID;
    if (p->d.N > 0 && (!pos || !scale || !rot || !unstable || !d_pos || !d_scale || !d_rot || !d_opacity ||
                       !d_color_param || (p->d.sh_deg > 0 && !color)))
        return RTG_E_INVALID;
    if (p->d.N == 0) return RTG_OK;
    WS w = make_ws(p, ws);
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_for(p->d.N, 256), 2048));
    if (p->d.sh_deg > 0)
        hipLaunchKernelGGL(k_sh_bwd, dim3(grid_for(p->d.N, 256)), dim3(256), 0, S(stream), p->d, w, pos, color,
                           unstable, poses, d_pos, d_color_param, ls);
    hipLaunchKernelGGL(k_project_bwd, dim3(blocks), dim3(256), 0, S(stream), p->d, w, pos, scale, rot, unstable,
                       poses, d_pos, d_scale, d_rot, d_opacity, d_color_param, ls);
    return launched();
}
}  // namespace

rtg_status rtg_backward_project(const rtg_plan* p, void* ws, const float* pos, const float* scale,
                                const float* rot, const float* color, const uint8_t* unstable, const double* poses,
                                float* d_pos, float* d_scale, float* d_rot, float* d_opacity, float* d_color_param,
                                void* stream) {
    return launch_project_bwd(p, ws, pos, scale, rot, color, unstable, poses, d_pos, d_scale, d_rot, d_opacity,
                              d_color_param, L1Scale{0.f, 0.f, nullptr, 0}, stream);
}

rtg_status rtg_backward_project_l1(const rtg_plan* p, void* ws, const float* pos, const float* scale,
                                   const float* rot, const float* color, const uint8_t* unstable,
                                   const double* poses, float w_c, float w_d, float* d_pos, float* d_scale,
                                   float* d_rot, float* d_opacity, float* d_color_param, float* loss_out,
                                   void* stream) {
    if (!loss_out) return RTG_E_INVALID;
    return launch_project_bwd(p, ws, pos, scale, rot, color, unstable, poses, d_pos, d_scale, d_rot, d_opacity,
                              d_color_param, L1Scale{w_c, w_d, loss_out, 1}, stream);
}

rtg_status rtg_loss_l1(const rtg_plan* p, void* ws, const float* color, const float* depth, const float* color_gt,
                       const float* depth_gt, float w_c, float w_d, float* d_color, float* d_depth, float* loss_out,
                       void* stream) {
    if (!ws_ok(p, ws) || !color || !depth || !color_gt || !depth_gt || !d_color || !d_depth || !loss_out)
        return RTG_E_INVALID;
    WS w = make_ws(p, ws);
    int64_t n = (int64_t)p->d.F * p->d.ntiles * p->d.tarea;
    unsigned nb = grid_for(n, 256);
    float* part = reinterpret_cast<float*>(static_cast<char*>(ws) + p->off[O_LPART]);
    hipLaunchKernelGGL(k_loss_partials, dim3(nb), dim3(256), 0, S(stream), p->d, w, color, depth, color_gt,
                       depth_gt, part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, S(stream), w, (const float*)part, (uint32_t)nb, w_c,
                       w_d, loss_out);
    hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, S(stream), p->d, w, color, depth, color_gt, depth_gt,
                       w_c, w_d, d_color, d_depth);
    return launched();
}

rtg_status rtg_adam(const rtg_plan* p, float* pos, float* scale, float* rot, float* color, const uint8_t* unstable,
                    const float* d_pos, const float* d_scale, const float* d_rot, const float* d_color, float* m,
                    float* v, int32_t* step, float lr_pos, float lr_scale, float lr_rot, float lr_color,
                    float lr_sh_rest, float beta1, float beta2, float eps, void* stream) {
    if (!p || !step || !m || !v) return RTG_E_INVALID;
    if (p->d.N > 0 && (!pos || !scale || !rot || !color || !unstable || !d_pos || !d_scale || !d_rot || !d_color))
        return RTG_E_INVALID;
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, S(stream), step);
    if (launched() != RTG_OK) return RTG_E_HIP;
    if (p->d.N == 0) return RTG_OK;
    const int32_t K = (p->d.sh_deg + 1) * (p->d.sh_deg + 1);
    AdamArgs a{lr_pos, lr_scale, lr_rot, lr_color, lr_sh_rest, beta1, beta2, eps, K};
    hipLaunchKernelGGL(k_adam, dim3(grid_for(p->d.N, 256)), dim3(256), 0, S(stream), p->d.N, pos, scale, rot, color,
                       unstable, d_pos, d_scale, d_rot, d_color, m, v, step, a);
    return launched();
}

rtg_status rtg_read_status(const rtg_plan* p, void* ws, int64_t* counts, void* stream) {
    if (!ws_ok(p, ws) || !counts) return RTG_E_INVALID;
    // the work counters are summed on the device; one 128-byte header copy
    // then carries everything (no host-side buffers)
    WS w = make_ws(p, ws);
    const uint32_t nbb = (uint32_t)((int64_t)p->d.F * p->d.nbpf * p->d.nchunks);
    hipLaunchKernelGGL(k_sum_counters, dim3(1), dim3(1024), 0, S(stream), w, nbb);
    if (launched() != RTG_OK) return RTG_E_HIP;
    Hdr h;
    if (hipMemcpyAsync(&h, static_cast<char*>(ws) + p->off[O_HDR], sizeof(Hdr), hipMemcpyDeviceToHost, S(stream)) !=
            hipSuccess ||
        hipStreamSynchronize(S(stream)) != hipSuccess)
        return RTG_E_HIP;
    counts[0] = h.n_pairs;
    counts[1] = h.n_px;
    counts[2] = h.n_items;
    counts[3] = h.overflow;
    counts[4] = h.n_big;
    counts[5] = h.err;
    for (int c = 0; c < 4; ++c) counts[6 + c] = (int64_t)h.sums[c];
    counts[10] = h.n_restaged;
    if (h.overflow) return RTG_E_CAPACITY;
    if (h.err) return RTG_E_DEVICE;
    return RTG_OK;
}

// ---- Gaussian adding and state management ---------------------------------

void rtg_adding_params_default(rtg_adding_params* a) {
    if (!a) return;
    a->delta_T = 0.5f;
    a->delta_d = 0.1f;
    a->delta_c = 0.1f;
    a->rate = 0.05f;
    a->alpha_opaque = 0.99f;
    a->alpha_transparent = 0.1f;
    a->r_transparent = 0.01f;
    a->thickness = 0.1f;
    a->delta_eta = 100;
    a->delta_e = 5;
    a->delta_t = 200;
    a->sh_degree = 0;
}

size_t rtg_adding_workspace_bytes(const rtg_intrinsics* intr) {
    if (!intr_ok(intr)) return 0;
    return add_ws((int64_t)intr->width * intr->height).bytes;
}

rtg_status rtg_add_gaussians(const rtg_intrinsics* intr, const rtg_adding_params* prm, const double* pose,
                             const float* color_in, const float* depth_in, const float* color_r,
                             const float* depth_r, const float* trans_r, const int32_t* index_r, const float* rnd,
                             int32_t frame_k, int64_t n_cur, int64_t capacity, float* pos, float* scale, float* rot,
                             float* opacity, float* color, uint8_t* unstable, int32_t* eta, int32_t* err,
                             int32_t* tstamp, uint8_t* mask_out, int64_t* counts, void* ws, size_t ws_bytes,
                             void* stream) {
    if (!intr_ok(intr) || !prm || !pose || !color_in || !depth_in || !color_r || !depth_r || !trans_r || !index_r ||
        !rnd || !pos || !scale || !rot || !opacity || !color || !unstable || !eta || !err || !tstamp || !counts)
        return RTG_E_INVALID;
    if (n_cur < 0 || capacity < n_cur || capacity >= (1ll << 30) || !(prm->rate >= 0.f && prm->rate <= 1.f) ||
        prm->sh_degree < 0 || prm->sh_degree > 3)
        return RTG_E_INVALID;
    const int64_t np = (int64_t)intr->width * intr->height;
    const AddWs L = add_ws(np);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < L.bytes) return RTG_E_INVALID;
    char* b = static_cast<char*>(ws);
    uint8_t* codes = reinterpret_cast<uint8_t*>(b + L.codes);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(b + L.counts);
    uint32_t* off = reinterpret_cast<uint32_t*>(b + L.offsets);
    unsigned long long* tot = reinterpret_cast<unsigned long long*>(b + L.total);
    const AddParams a = add_params(prm);
    const Intr c = to_intr(intr);
    const unsigned nb = grid_for(np, 256);
    hipLaunchKernelGGL(k_add_mark, dim3(nb), dim3(256), 0, S(stream), a, c, color_in, depth_in, color_r, depth_r,
                       trans_r, index_r, rnd, (const uint8_t*)unstable, n_cur, codes, mask_out, cnt);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, S(stream), (const uint32_t*)cnt, off, (uint32_t)nb, tot);
    hipLaunchKernelGGL(k_add_emit, dim3(nb), dim3(256), 0, S(stream), a, c, pose, color_in, depth_in,
                       (const uint8_t*)codes, (const uint32_t*)off, frame_k, n_cur, capacity, pos, scale, rot,
                       opacity, color, unstable, eta, err, tstamp);
    hipLaunchKernelGGL(k_add_counts, dim3(1), dim3(64), 0, S(stream), (const unsigned long long*)tot, n_cur,
                       capacity, counts);
    return launched();
}

rtg_status rtg_confidence_count(int64_t n, int32_t row_width, const uint8_t* unstable, const float* d_color,
                                int32_t* eta, void* stream) {
    if (n < 0 || row_width < 1 || row_width > 48) return RTG_E_INVALID;
    if (n == 0) return RTG_OK;
    if (!unstable || !d_color || !eta) return RTG_E_INVALID;
    hipLaunchKernelGGL(k_confidence, dim3(grid_for(n, 256)), dim3(256), 0, S(stream), n, row_width, unstable,
                       d_color, eta);
    return launched();
}

rtg_status rtg_state_update(const rtg_intrinsics* intr, const rtg_adding_params* prm, const float* color_in,
                            const float* depth_in, const float* color_r, const float* depth_r,
                            const int32_t* index_r, int32_t frame_k, int64_t n, uint8_t* unstable, int32_t* eta,
                            int32_t* err, int32_t* tstamp, uint8_t* keep, uint8_t* flag_ws, void* stream) {
    if (!intr_ok(intr) || !prm || !color_in || !depth_in || !color_r || !depth_r || !index_r || n < 0)
        return RTG_E_INVALID;
    if (n > 0 && (!unstable || !eta || !err || !tstamp || !keep || !flag_ws)) return RTG_E_INVALID;
    if (n == 0) return RTG_OK;
    const AddParams a = add_params(prm);
    const Intr c = to_intr(intr);
    const int64_t np = (int64_t)intr->width * intr->height;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65535)), dim3(256), 0,
                       S(stream), flag_ws, (size_t)n, (uint8_t)0);
    hipLaunchKernelGGL(k_state_flag, dim3(grid_for(np, 256)), dim3(256), 0, S(stream), a, c, color_in, depth_in,
                       color_r, depth_r, index_r, n, (const uint8_t*)unstable, flag_ws);
    hipLaunchKernelGGL(k_state_apply, dim3(grid_for(n, 256)), dim3(256), 0, S(stream), a, n, frame_k,
                       (const uint8_t*)flag_ws, unstable, eta, err, tstamp, keep);
    return launched();
}

size_t rtg_compact_workspace_bytes(int64_t n) {
    if (n < 0) return 0;
    const size_t nb = (size_t)((n + 255) / 256);
    return align256(4 * nb) * 2 + 256;
}

rtg_status rtg_compact_rows(int64_t n, const uint8_t* keep, int32_t n_arrays, void* const* src, void* const* dst,
                            const int32_t* row_bytes, int64_t* n_out, void* ws, size_t ws_bytes, void* stream) {
    if (n < 0 || n >= (1ll << 31) || !keep || !n_out || n_arrays < 0 || n_arrays > kCompactMax) return RTG_E_INVALID;
    if (n_arrays > 0 && (!src || !dst || !row_bytes)) return RTG_E_INVALID;
    CompactArrays A;
    A.n = n_arrays;
    for (int k = 0; k < n_arrays; ++k) {
        if (!src[k] || !dst[k] || row_bytes[k] <= 0 || row_bytes[k] > 4096 || src[k] == dst[k]) return RTG_E_INVALID;
        A.src[k] = static_cast<const uint8_t*>(src[k]);
        A.dst[k] = static_cast<uint8_t*>(dst[k]);
        A.rb[k] = row_bytes[k];
    }
    const size_t nb = (size_t)((n + 255) / 256);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < rtg_compact_workspace_bytes(n))
        return RTG_E_INVALID;
    char* b = static_cast<char*>(ws);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(b);
    uint32_t* off = reinterpret_cast<uint32_t*>(b + align256(4 * nb));
    unsigned long long* tot = reinterpret_cast<unsigned long long*>(b + 2 * align256(4 * nb));
    const unsigned g = (unsigned)std::max<size_t>(nb, 1);
    hipLaunchKernelGGL(k_compact_count, dim3(g), dim3(256), 0, S(stream), n, keep, cnt);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, S(stream), (const uint32_t*)cnt, off, (uint32_t)g, tot);
    hipLaunchKernelGGL(k_compact_move, dim3(g), dim3(256), 0, S(stream), n, keep, (const uint32_t*)off, A);
    hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(64), 0, S(stream), (const unsigned long long*)tot, n_out);
    return launched();
}

const char* rtg_status_string(rtg_status s) {
    switch (s) {
        case RTG_OK: return "ok";
        case RTG_E_INVALID: return "invalid argument";
        case RTG_E_CAPACITY: return "pair capacity exceeded";
        case RTG_E_HIP: return "HIP runtime error";
        case RTG_E_UNSUPPORTED: return "no supported device";
        case RTG_E_DEVICE: return "device error flag set";
        case RTG_E_TOO_LARGE: return "plan workspace exceeds the static scratch (RTG_STATIC_SCRATCH_BYTES)";
    }
    return "unknown status";
}

const char* rtg_version(void) { return "rtg 0.1 (gfx950)"; }

}  // extern "C"

// ---- the mapping iteration around the backward --------------------------

extern "C" {

rtg_status rtg_reg_l2(int64_t n, float w_reg, const uint8_t* transparent, const uint8_t* unstable,
                      const float* pos, const float* scale, const float* rot, const float* pos0,
                      const float* scale0, const float* rot0, float* d_pos, float* d_scale, float* d_rot,
                      double* loss_out, void* stream) {
    if (n < 0 || n >= (1ll << 31) || !loss_out || !std::isfinite(w_reg)) return RTG_E_INVALID;
    if (n == 0) return RTG_OK;
    if (!transparent || !unstable || !pos || !scale || !rot || !pos0 || !scale0 || !rot0 || !d_pos || !d_scale ||
        !d_rot)
        return RTG_E_INVALID;
    hipLaunchKernelGGL(k_reg_l2, dim3(std::min<unsigned>(grid_for(n, 256), 1024u)), dim3(256), 0, S(stream), n,
                       (double)w_reg, transparent,
                       unstable, pos, scale, rot, pos0, scale0, rot0, d_pos, d_scale, d_rot, loss_out);
    return launched();
}

rtg_status rtg_fuse(int64_t n, int32_t color_width, const int32_t* eta_prev, const int32_t* eta_cur,
                    const float* pos_prev, const float* scale_prev, const float* rot_prev, const float* color_prev,
                    float* pos, float* scale, float* rot, float* color, void* stream) {
    if (n < 0 || n >= (1ll << 31) || color_width < 1 || color_width > 48) return RTG_E_INVALID;
    if (n == 0) return RTG_OK;
    if (!eta_prev || !eta_cur || !pos_prev || !scale_prev || !rot_prev || !color_prev || !pos || !scale || !rot ||
        !color)
        return RTG_E_INVALID;
    hipLaunchKernelGGL(k_fuse, dim3(grid_for(n, 256)), dim3(256), 0, S(stream), n, color_width, eta_prev, eta_cur,
                       pos_prev, scale_prev, rot_prev, color_prev, pos, scale, rot, color);
    return launched();
}

size_t rtg_select_workspace_bytes(int32_t frames, int32_t height, int32_t width) {
    if (frames < 1 || height < 1 || width < 1 || height > 32767 || width > 32767 || frames > RTG_MAX_FRAMES)
        return 0;
    const size_t npx = (size_t)frames * height * width;
    return align256(4 * npx) + align256(4 * 256 * (size_t)frames) + align256(sizeof(SelState) * (size_t)frames);
}

rtg_status rtg_select_top_error(int32_t frames, int32_t height, int32_t width, double frac, const float* color_r,
                                const float* color_in, uint8_t* mask_out, void* ws, size_t ws_bytes,
                                void* stream) {
    const size_t need = rtg_select_workspace_bytes(frames, height, width);
    if (!need || !(frac >= 0.0 && frac <= 1.0) || !color_r || !color_in || !mask_out || !ws ||
        (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < need)
        return RTG_E_INVALID;
    const int64_t hw = (int64_t)height * width, npx = hw * frames;
    char* b = static_cast<char*>(ws);
    uint32_t* keys = reinterpret_cast<uint32_t*>(b);
    uint32_t* hist = reinterpret_cast<uint32_t*>(b + align256(4 * (size_t)npx));
    SelState* st = reinterpret_cast<SelState*>(b + align256(4 * (size_t)npx) + align256(4 * 256 * (size_t)frames));
    const uint32_t k = (uint32_t)std::floor(frac * (double)hw);
    hipLaunchKernelGGL(k_sel_keys, dim3(grid_for(npx, 256)), dim3(256), 0, S(stream), npx, color_r, color_in, keys);
    hipLaunchKernelGGL(k_sel_init, dim3(frames), dim3(256), 0, S(stream), frames, k, hist, st);
    // about 64 pixels per thread per pass, at most 1024 workgroups per frame
    const unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (hw + 16383) / 16384));
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_sel_hist, dim3(bx, frames), dim3(256), 0, S(stream), hw, shift, (const uint32_t*)keys,
                           hist, (const SelState*)st);
        hipLaunchKernelGGL(k_sel_pick, dim3(frames), dim3(256), 0, S(stream), shift, hist, st);
    }
    hipLaunchKernelGGL(k_sel_mask, dim3(grid_for(npx, 256)), dim3(256), 0, S(stream), hw, frames,
                       (const uint32_t*)keys, (const SelState*)st, mask_out);
    return launched();
}

}  // extern "C"

// ---- frame-to-model tracking ---------------------------------------------

namespace {
struct IcpLayout {
    int W[3], H[3];
    size_t off_d[3], off_dm[3], off_nm[3], off_part, total;
    int nblk0;
};

bool icp_layout(const rtg_intrinsics* intr, int levels, IcpLayout& L) {
    if (!intr_ok(intr) || levels < 1 || levels > 3) return false;
    size_t o = 0;
    for (int l = 0; l < levels; ++l) {
        L.W[l] = intr->width >> l;
        L.H[l] = intr->height >> l;
        if (L.W[l] < 2 || L.H[l] < 2) return false;
        L.off_d[l] = L.off_dm[l] = L.off_nm[l] = 0;
        if (l > 0) {
            const size_t n = (size_t)L.W[l] * L.H[l];
            L.off_d[l] = o;
            o = align256(o + 4 * n);
            L.off_dm[l] = o;
            o = align256(o + 4 * n);
            L.off_nm[l] = o;
            o = align256(o + 12 * n);
        }
    }
    L.nblk0 = (int)grid_for((int64_t)L.W[0] * L.H[0], 256);
    L.off_part = o;
    o = align256(o + 8 * (size_t)kIcpTerms * L.nblk0);
    L.total = o;
    return true;
}
}  // namespace

extern "C" {

rtg_status rtg_render_normals(const rtg_plan* p, void* ws, float* normal_out, void* stream) {
    if (!ws_ok(p, ws) || !normal_out) return RTG_E_INVALID;
    WS w = make_ws(p, ws);
    const int64_t n = (int64_t)p->d.F * p->d.ntiles * p->d.tarea;
    hipLaunchKernelGGL(k_render_normals, dim3(grid_for(n, 256)), dim3(256), 0, S(stream), p->d, w, normal_out);
    return launched();
}

void rtg_icp_params_default(rtg_icp_params* prm) {
    if (!prm) return;
    prm->levels = 3;
    prm->iters[0] = 10;
    prm->iters[1] = 5;
    prm->iters[2] = 4;
    prm->dist = 0.1;
    prm->sin_angle = 0.3420201433256687;   // sin(20 deg)
}

size_t rtg_icp_workspace_bytes(const rtg_intrinsics* intr, int32_t levels) {
    IcpLayout L;
    return icp_layout(intr, levels, L) ? L.total : 0;
}

rtg_status rtg_icp(const rtg_intrinsics* intr, const rtg_icp_params* prm, const float* depth_in,
                   const float* depth_model, const float* normal_model, const double* pose_model,
                   const double* pose_init, double* pose_out, double* trace_out, void* ws, size_t ws_bytes,
                   void* stream) {
    IcpLayout L;
    if (!prm || !icp_layout(intr, prm->levels, L) || !depth_in || !depth_model || !normal_model || !pose_model ||
        !pose_init || !pose_out || !ws || (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < L.total ||
        !(prm->dist > 0.0) || !(prm->sin_angle >= 0.0 && prm->sin_angle <= 1.0))
        return RTG_E_INVALID;
    for (int l = 0; l < prm->levels; ++l)
        if (prm->iters[l] < 0 || prm->iters[l] > 1000) return RTG_E_INVALID;
    char* b = static_cast<char*>(ws);
    const float* D[3] = {depth_in, nullptr, nullptr};
    const float* Dm[3] = {depth_model, nullptr, nullptr};
    const float* Nm[3] = {normal_model, nullptr, nullptr};
    for (int l = 1; l < prm->levels; ++l) {
        float* d = reinterpret_cast<float*>(b + L.off_d[l]);
        float* dm = reinterpret_cast<float*>(b + L.off_dm[l]);
        float* nm = reinterpret_cast<float*>(b + L.off_nm[l]);
        const unsigned g = grid_for((int64_t)L.W[l] * L.H[l], 256);
        hipLaunchKernelGGL(k_icp_down_depth, dim3(g), dim3(256), 0, S(stream), D[l - 1], L.W[l - 1], d, L.W[l],
                           L.H[l]);
        hipLaunchKernelGGL(k_icp_down_depth, dim3(g), dim3(256), 0, S(stream), Dm[l - 1], L.W[l - 1], dm, L.W[l],
                           L.H[l]);
        hipLaunchKernelGGL(k_icp_down_normal, dim3(g), dim3(256), 0, S(stream), Dm[l - 1], Nm[l - 1], L.W[l - 1],
                           nm, L.W[l], L.H[l]);
        D[l] = d;
        Dm[l] = dm;
        Nm[l] = nm;
    }
    if (pose_out != pose_init)
        hipLaunchKernelGGL(k_icp_copy_pose, dim3(1), dim3(64), 0, S(stream), pose_init, pose_out);
    double* part = reinterpret_cast<double*>(b + L.off_part);
    int row = 0;
    for (int l = prm->levels - 1; l >= 0; --l) {
        const double s = (double)(1 << l);
        IcpLevel lv{L.W[l], L.H[l], intr->fx / s, intr->fy / s, intr->cx / s, intr->cy / s, D[l], Dm[l], Nm[l]};
        // at most 512 workgroups, each striding over the level's pixels
        const int nblk = (int)std::min<unsigned>(grid_for((int64_t)L.W[l] * L.H[l], 256), 512u);
        for (int it = 0; it < prm->iters[l]; ++it, ++row) {
            hipLaunchKernelGGL(k_icp_reduce, dim3(nblk), dim3(256), 0, S(stream), lv, (const double*)pose_out,
                               pose_model, prm->dist, prm->sin_angle, part);
            hipLaunchKernelGGL(k_icp_solve, dim3(1), dim3(256), 0, S(stream), (const double*)part, nblk, pose_out,
                               trace_out ? trace_out + (int64_t)kIcpTrace * row : nullptr);
        }
    }
    return launched();
}

}  // extern "C"
