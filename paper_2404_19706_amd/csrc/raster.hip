// Steps a5 and a7: per-pixel forward compositing (Eq. 1-5) and its adjoint,
// over the masked pixels only.
//
// Work decomposition: a work item is a pack of up to 64 masked pixels of one
// (frame, tile), compacted so that sparse masks do not idle lanes.  Each
// wave64 of a persistent grid takes items either round-robin (items_per_pop
// = 0: item k goes to wave k mod waves, so the packs of one tile land on the
// waves of one workgroup, i.e. one CU and one XCD L2) or in chunks of
// items_per_pop consecutive items from an atomic queue head.
//
// Records come in list order from the 64-byte pair-order copy written by the
// per-tile sort, 64 per batch, one per lane, with one coalesced load level;
// the next batch is prefetched into registers while the current one is
// composited.  Each batch is pack-culled (records that cannot reach any pixel
// of the pack are dropped, lane-parallel) and the survivors are compacted
// into the wave's own LDS slice, from which every lane reads the same record
// (an LDS broadcast) with one lane per pixel.  A ballot ends the walk once
// every lane has finished its colour and found its depth hit.
//
// Decisions (footprint, depth hit) use the fixed binary32 sequence on the
// rounded centre; the values (f, gradients) use offsets from the centre
// including its residual.
//
// The backward pass re-walks each pixel's list back to front, recovering the
// transmission in front of each Gaussian from the stored final value
// (T_i = T_{i+1} / (1 - f_i); nothing per pair is stored).  For each unstable
// Gaussian it reduces the nine colour-path gradients of the wave's pixels,
// plus the five depth-path terms of the pixels whose depth hit it is, with
// one reduce-scatter, and adds the fourteen totals with one float atomic
// instruction into the Gaussian's per-frame camera-space accumulator.
#include <type_traits>

#include "rtg_common.h"

// Compile-time tuning knobs of the compositing kernels: records whose
// footprint and opacity are evaluated together before the sequential blend
// (instruction-level parallelism against register pressure), and the
// minimum number of resident waves per SIMD each kernel is compiled for
// (occupancy; 0 = compiler's choice).  Measured on gfx950: four records per
// group (the forward stages three record words) keep the forward at 95
// VGPRs without spills and beat groups of two by 3-4 % on long lists; the
// backward at five waves per SIMD gains ~5 % on long lists.
#ifndef RTG_FWD_GROUP
#define RTG_FWD_GROUP 4
#endif
#ifndef RTG_FWD_WAVES_PER_EU
#define RTG_FWD_WAVES_PER_EU 0
#endif
#ifndef RTG_BWD_WAVES_PER_EU
#define RTG_BWD_WAVES_PER_EU 5
#endif
#if RTG_FWD_WAVES_PER_EU > 0
#define RTG_FWD_BOUNDS __launch_bounds__(256, RTG_FWD_WAVES_PER_EU)
#else
#define RTG_FWD_BOUNDS __launch_bounds__(256)
#endif
#if RTG_BWD_WAVES_PER_EU > 0
#define RTG_BWD_BOUNDS __launch_bounds__(256, RTG_BWD_WAVES_PER_EU)
#else
#define RTG_BWD_BOUNDS __launch_bounds__(256)
#endif

namespace rtg {

struct PixelOfItem {
    uint32_t ft, r;     // (frame, tile) and rank of the pixel in the tile
    int f, px, py;
    bool act;
    float ux, uy;
    uint32_t rs, re;    // pair range of the tile
};

__device__ __forceinline__ PixelOfItem decode_item(const Dims& d, const WS& w, uint32_t it, int lane) {
    PixelOfItem p;
    uint32_t code = w.items[it];
    p.ft = code / (uint32_t)d.ppt;
    uint32_t pack = code - p.ft * (uint32_t)d.ppt;
    uint32_t npx = w.tile_npx[p.ft];
    p.r = pack * 64u + (uint32_t)lane;
    p.act = p.r < npx;
    int l = p.act ? (int)w.pix[(size_t)p.ft * d.tarea + p.r] : 0;
    p.f = (int)(p.ft / (uint32_t)d.ntiles);
    int t = (int)(p.ft - (uint32_t)p.f * (uint32_t)d.ntiles);
    p.px = (t % d.tx) * d.tw + (l & (d.tw - 1));
    p.py = (t / d.tx) * d.th + (l >> d.lg_tw);
    p.ux = (float)p.px + 0.5f;
    p.uy = (float)p.py + 0.5f;
    p.rs = w.tile_start[p.ft];
    p.re = w.tile_end[p.ft];
    return p;
}

// Bounding box of the pixels of one pack (inclusive pixel indices).
struct PackBox {
    int x0, x1, y0, y1;
};

__device__ __forceinline__ int wave_min_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ PackBox pack_box(const PixelOfItem& p) {
    PackBox b;
    b.x0 = wave_min_i(p.act ? p.px : 0x7fffffff);
    b.x1 = wave_max_i(p.act ? p.px : -1);
    b.y0 = wave_min_i(p.act ? p.py : 0x7fffffff);
    b.y1 = wave_max_i(p.act ? p.py : -1);
    return b;
}

// Conservative pack culling of one record.  For conics with condition
// number below ~1000 -- where both the binary32 decision and this binary32
// test err by well under 0.1 % -- a record is dropped when the box of the
// pack's pixel centres lies outside the cut-off ellipse's bounding box (with
// 1 % and one pixel of margin) or when the minimum of the quadratic form over
// that box (0 with the centre inside, else the clamped minimum on each edge)
// exceeds the cut-off by more than 1 %.  A dropped record has d^2 > cut-off
// at every pixel of the pack, so culling changes no output.  Records with
// worse conditioning are always kept.
__device__ __forceinline__ bool pack_keeps(float4 h0, float qc, const PackBox& b, float cut) {
    float a = h0.z, bq = 0.5f * h0.w, c = qc;
    float det = a * c - bq * bq;
    float tr = a + c;
    if (!(det > 0.f) || tr * tr >= 1000.f * det) return true;
    float idet = __builtin_amdgcn_rcpf(det);
    float ex = __builtin_sqrtf(1.01f * cut * c * idet) + 1.f;
    float ey = __builtin_sqrtf(1.01f * cut * a * idet) + 1.f;
    float lx = ((float)b.x0 + 0.5f) - h0.x, hx = ((float)b.x1 + 0.5f) - h0.x;
    float ly = ((float)b.y0 + 0.5f) - h0.y, hy = ((float)b.y1 + 0.5f) - h0.y;
    if (lx > ex || hx < -ex || ly > ey || hy < -ey) return false;
    if (lx <= 0.f && hx >= 0.f && ly <= 0.f && hy >= 0.f) return true;
    float ia = __builtin_amdgcn_rcpf(a), ic = __builtin_amdgcn_rcpf(c);
    auto q = [&](float x, float y) { return a * x * x + 2.f * bq * x * y + c * y * y; };
    float y0 = fminf(fmaxf(-bq * lx * ic, ly), hy), y1 = fminf(fmaxf(-bq * hx * ic, ly), hy);
    float x0 = fminf(fmaxf(-bq * ly * ia, lx), hx), x1 = fminf(fmaxf(-bq * hy * ia, lx), hx);
    float m = fminf(fminf(q(lx, y0), q(hx, y1)), fminf(q(x0, ly), q(x1, hy)));
    return m <= 1.01f * cut;
}

// One batch of up to 64 pair-order records, one per lane, held in registers
// (prefetched while the previous batch is composited).  Callers guarantee
// j0 < j1, so lanes past the end re-load record j0 instead of branching
// (keeps the batch in registers).
// NW = 4 loads the whole record; NW = 3 leaves out {n^c, h}, which the
// compositing passes read only for the depth-hit record of a pixel.
template <int NW>
struct Batch {
    float4 r0, r1, r2, r3;
    bool ok;
};

template <int NW>
__device__ __forceinline__ Batch<NW> load_batch(const WS& w, uint32_t j0, uint32_t j1, int lane) {
    Batch<NW> B;
    uint32_t j = j0 + (uint32_t)lane;
    B.ok = j < j1;
    const float4* src = w.prec + 4ull * (B.ok ? j : j0);
    B.r0 = src[0];
    B.r1 = src[1];
    B.r2 = src[2];
    if constexpr (NW == 4) B.r3 = src[3];
    return B;
}

// Pack-cull the batch and compact the survivors into the wave's LDS slice in
// list order; P receives their absolute pair positions.  Returns the count.
template <int NW>
__device__ __forceinline__ uint32_t compact_batch(const Batch<NW>& B, uint32_t j0, float4 (*L)[64], uint32_t* P,
                                                  int lane, const PackBox& pb, float cut, bool& anyp) {
    bool keep = B.ok && pack_keeps(B.r0, B.r1.x, pb, cut);
    uint64_t m = ballot(keep);
    anyp = ballot(keep && rec_precise(B.r2)) != 0;
    if (keep) {
        uint32_t q = (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1ull));
        L[0][q] = B.r0;
        L[1][q] = B.r1;
        L[2][q] = B.r2;
        if constexpr (NW == 4) L[3][q] = B.r3;
        P[q] = j0 + (uint32_t)lane;
    }
    return (uint32_t)__builtin_popcountll(m);
}

// Iterates the work items of one wave: round-robin over the first n_static
// items (item k to wave k mod waves), then chunks of items_per_pop
// consecutive items from an atomic queue head over the rest.  n_static is
// every item with items_per_pop = 0, none with static_share = 0, else
// static_share percent of them (a whole number of rounds).
struct ItemIter {
    uint32_t it, end, n_items, n_static, ipp, stride;
    uint32_t* queue;
    int lane;
    bool dyn;
    __device__ __forceinline__ bool next(uint32_t& out) {
        if (!dyn) {
            if (it < n_static) {
                out = it;
                it += stride;
                return true;
            }
            if (ipp == 0) return false;
            dyn = true;
            it = end = 0;
        }
        if (it >= end) {
            uint32_t it0 = 0;
            if (lane == 0) it0 = atomicAdd(queue, ipp);
            it0 = n_static + (uint32_t)readfirstlane((int)it0);
            if (it0 >= n_items) return false;
            it = it0;
            end = min(it0 + ipp, n_items);
        }
        out = it;
        it += 1u;
        return true;
    }
};

__device__ __forceinline__ ItemIter make_iter(int items_per_pop, int static_share, uint32_t n_items,
                                             uint32_t* queue, int lane) {
    ItemIter I;
    I.n_items = n_items;
    I.ipp = (uint32_t)items_per_pop;
    I.queue = queue;
    I.lane = lane;
    I.stride = gridDim.x * 4u;
    I.it = (uint32_t)readfirstlane((int)(blockIdx.x * 4u + (threadIdx.x >> 6)));
    I.end = 0;
    I.dyn = false;
    I.n_static = I.ipp == 0 ? n_items
                            : (uint32_t)((uint64_t)n_items * (uint32_t)static_share / 100u / I.stride * I.stride);
    return I;
}

// Clears a queue head before the launch that pops from it (a kernel, not
// a memset, so that the step can be captured in a graph).
__global__ void k_queue_reset(uint32_t* q) {
    if (threadIdx.x == 0) *q = 0u;
}

// Butterfly reduce-scatter of 16 per-lane values over the wave: after it,
// every lane of quad q holds the wave total of slot
// 8*b2 + 4*b3 + 2*b4 + b5 (b_k = bit k of the lane id).  Rounds on lane bits
// 5 and 4 use the gfx950 permlane32/permlane16 swaps (a swap followed by one
// add leaves each half with its own slot's partial sum); bit 3 pairs lane l
// with l ^ 15 (DPP row mirror) and bit 2 with l ^ 7 (DPP half-row mirror),
// partners that differ in that bit and agree on the bits already reduced;
// bits 1 and 0 are quad DPP adds.
__device__ __forceinline__ float swap32_sum(float a, float b) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_sum(float a, float b) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <int CTRL>
__device__ __forceinline__ float mirror_sum(float a, float b, bool hi) {
    float send = hi ? a : b;
    float keep = hi ? b : a;
    return keep + dpp_mov<CTRL>(send);
}
__device__ __forceinline__ float quad_sum(float o) {
    o += dpp_mov<0xB1>(o);   // quad_perm [1,0,3,2]
    o += dpp_mov<0x4E>(o);   // quad_perm [2,3,0,1]
    return o;
}
__device__ __forceinline__ float reduce_scatter16(const float (&v)[16], int lane) {
    float r[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = swap32_sum(v[2 * j], v[2 * j + 1]);
    float q[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) q[m] = swap16_sum(r[2 * m], r[2 * m + 1]);
    bool b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
    float p0 = mirror_sum<0x140>(q[0], q[1], b3);
    float p1 = mirror_sum<0x140>(q[2], q[3], b3);
    return quad_sum(mirror_sum<0x141>(p0, p1, b2));
}
// The same when slots 9-15 are zero (no depth-path term in the wave).
__device__ __forceinline__ float reduce_scatter9(const float (&v)[16], int lane) {
    float r[5];
#pragma unroll
    for (int j = 0; j < 4; ++j) r[j] = swap32_sum(v[2 * j], v[2 * j + 1]);
    r[4] = swap32_sum(v[8], 0.f);
    float q0 = swap16_sum(r[0], r[1]), q1 = swap16_sum(r[2], r[3]), q2 = swap16_sum(r[4], 0.f);
    bool b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
    float p0 = mirror_sum<0x140>(q0, q1, b3);
    float p1 = mirror_sum<0x140>(q2, 0.f, b3);
    return quad_sum(mirror_sum<0x141>(p0, p1, b2));
}
// The nine colour-path sums through LDS instead: every lane stores its
// nine values ([slot][lane]), then lanes 8s..8s+7 add 8 values each of slot
// s (s < 8) and combine them with three DPP steps, and the whole wave adds
// slot 8.  Lane 8s returns slot s's total, lane 0 additionally slot 8's.
__device__ __forceinline__ void lds_sum9(const float (&v)[16], float* red, int lane, float& tot, float& tot8) {
#pragma unroll
    for (int k = 0; k < 9; ++k) red[k * 64 + lane] = v[k];
    wave_lds_sync();
    const float4* r4 = reinterpret_cast<const float4*>(red + (lane >> 3) * 64 + (lane & 7) * 8);
    const float4 x = r4[0], y = r4[1];
    float t = ((x.x + x.y) + (x.z + x.w)) + ((y.x + y.y) + (y.z + y.w));
    t += dpp_mov<0xB1>(t);    // quad_perm [1,0,3,2]
    t += dpp_mov<0x4E>(t);    // quad_perm [2,3,0,1]
    t += dpp_mov<0x141>(t);   // row_half_mirror: the other quad of the eight
    tot = t;
    tot8 = wave_sum(red[8 * 64 + lane]);
    wave_lds_sync();
}

__device__ __forceinline__ int scatter_slot(int lane) {
    return 8 * ((lane >> 2) & 1) + 4 * ((lane >> 3) & 1) + 2 * ((lane >> 4) & 1) + ((lane >> 5) & 1);
}

// The Gaussian weight exp(-d^2 / 2) of both compositing kernels, as one
// multiply and the hardware base-2 exponential (the forward and the
// backward must evaluate it identically: the backward recovers the
// transmission by dividing out the forward's factors).
__device__ __forceinline__ float gauss_weight(float dd) {
    return __builtin_amdgcn_exp2f(dd * -0.72134752044448170f);   // -log2(e) / 2
}

// Lane k's value (k the same on every lane).
__device__ __forceinline__ float rdl(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ uint32_t rdl_u(uint32_t v, int k) { return (uint32_t)__builtin_amdgcn_readlane((int)v, k); }

// Decision distance dd and value opacity f = min(alpha exp(-d_v^2 / 2),
// 0.99) of one record at pixel centre (ux, uy): the fixed sequence of both
// compositing paths (pack and straggler), which therefore give the same
// bits.  PR: the record may be precise (then d_v^2 comes from the whitened
// offsets, the precise rows at rpf); `uniform`: every lane holds the same
// record (the precise test is then a uniform branch with scalar loads).
template <bool PR>
__device__ __forceinline__ float eval_rec(const float4& A, const float4& Bq, const float4& Cc, float ux, float uy,
                                          const float* rpf, bool uniform, float& fv) {
    const float dxd = ux - A.x, dyd = uy - A.y;
    const float dd = __builtin_fmaf(Bq.x * dyd, dyd, __builtin_fmaf(A.w * dxd, dyd, (A.z * dxd) * dxd));
    const float2 lo = unpack_mu_lo(Cc.w);
    const float dx = dxd - lo.x, dy = dyd - lo.y;
    float ddv = __builtin_fmaf(Bq.x * dy, dy, __builtin_fmaf(A.w * dx, dy, (A.z * dx) * dx));
    if constexpr (PR) {
        const uint32_t gw = uniform ? (uint32_t)readfirstlane((int)__float_as_uint(Cc.z)) : __float_as_uint(Cc.z);
        if (gw & kPreciseBit) {
            float e0, e1;
            precise_offsets(rpf + 6 * (int64_t)(gw & kGidMask), ux, uy, A.x, A.y, dxd, dyd, e0, e1);
            ddv = e0 * e0 + e1 * e1;
        }
    }
    fv = fminf(Bq.y * gauss_weight(ddv), 0.99f);
    return dd;
}

// DM = 0: the depth of Eq. 4-5 (first hit, disc plane or centre); DM = 1:
// the alpha-blended depth sum_i z_i f_i T_i of the depth-rendering ablation
// (z_i the record's binary32 camera depth, -1 where nothing blends), with
// the index map still by the first hit.
template <int DM>
__global__ RTG_FWD_BOUNDS void k_raster_fwd(Dims d, WS w, float* __restrict__ out_c,
                                                 float* __restrict__ out_d, float* __restrict__ out_t,
                                                 int* __restrict__ out_i) {
    __shared__ float4 lds[4][3][64];
    __shared__ uint32_t ldp[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float4(*L)[64] = lds[wv];
    uint32_t* P = ldp[wv];
    ItemIter iter = make_iter(d.fwd_items_per_pop, d.fwd_static_share, w.hdr->n_items, &w.hdr->q_fwd, lane);
    float cnt_eval = 0.f;
    uint32_t cnt_blend = 0;
    const float cut = d.cutoff2, teps = d.t_eps;
    uint32_t it;
    while (iter.next(it)) {
        PixelOfItem p = decode_item(d, w, it, lane);
        const PackBox pb = pack_box(p);
        float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, Da = 0.f;
        uint32_t last = p.rs, hitpos = 0;
        uint32_t hitg = 0;
        int hitk = -1, lastk = -1;
        uint32_t nblend = 0;
        bool cdone = !p.act, ddone = !p.act;
        Batch<3> B = {};
        if (p.rs < p.re) B = load_batch<3>(w, p.rs, p.re, lane);
        // the frame is the same for every lane of the pack: a scalar base
        const float* rpf = w.recp + 6 * ((int64_t)readfirstlane(p.f) * d.N);
        const float* zf = w.zkey + (int64_t)readfirstlane(p.f) * d.N;
        for (uint32_t b = p.rs; b < p.re; b += 64) {
            bool anyp;
            uint32_t nb = compact_batch<3>(B, b, L, P, lane, pb, cut, anyp);
            wave_lds_sync();
            if (b + 64 < p.re) B = load_batch<3>(w, b + 64, p.re, lane);
            // groups of G records, specialised on whether the batch holds a
            // precise record (the value distance of those comes from the
            // factored form; one record per group there)
            auto groups = [&](auto prec) -> bool {
                constexpr bool PR = decltype(prec)::value;
                constexpr int G = PR ? 1 : RTG_FWD_GROUP;
                for (uint32_t k0 = 0; k0 < nb; k0 += G) {
                    // independent part for G records: decision, value, opacity
                    float fvq[G], ddq[G], tauq[G], cr[G], cg[G], cb[G], zq[G];
                    uint32_t gq[G];
                    bool inq[G];
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        uint32_t k = min(k0 + u, nb - 1);
                        float4 A = L[0][k];
                        float4 Bq = L[1][k];
                        float4 Cc = L[2][k];
                        const float dd = eval_rec<PR>(A, Bq, Cc, p.ux, p.uy, rpf, true, fvq[u]);
                        inq[u] = (k0 + u < nb) && dd <= cut;
                        ddq[u] = dd;
                        tauq[u] = Bq.z;
                        cr[u] = Bq.w;
                        cg[u] = Cc.x;
                        cb[u] = Cc.y;
                        gq[u] = __float_as_uint(Cc.z);
                        // the record is the same on every lane: a scalar load
                        if constexpr (DM == 1)
                            zq[u] = zf[readfirstlane((int)(__float_as_uint(Cc.z) & kGidMask))];
                    }
                    // sequential part: compositing in list order and the depth hit
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        bool take = inq[u] && !cdone;
                        float fv = take ? fvq[u] : 0.f;
                        float wgt = fv * T;
                        C0 = __builtin_fmaf(cr[u], wgt, C0);
                        C1 = __builtin_fmaf(cg[u], wgt, C1);
                        C2 = __builtin_fmaf(cb[u], wgt, C2);
                        if constexpr (DM == 1) Da = __builtin_fmaf(zq[u], wgt, Da);
                        T = T * (1.f - fv);
                        lastk = take ? (int)(k0 + u) : lastk;
                        nblend += take ? 1u : 0u;
                        cdone = cdone || (take && T < teps);
                        bool h = inq[u] && !ddone && ddq[u] < tauq[u];
                        hitg = h ? gq[u] : hitg;
                        hitk = h ? (int)(k0 + u) : hitk;
                        ddone = ddone || h;
                    }
                    if (((k0 + G) & 7) == 0 && ballot(!(cdone && ddone)) == 0) return true;
                }
                return false;
            };
            const bool all_done = anyp ? groups(std::true_type{}) : groups(std::false_type{});
            // list positions of this batch's last blend and depth hit, and the
            // hit's normal and plane offset, before the slice is reused
            if (lastk >= 0) {
                last = P[lastk] + 1;
                lastk = -1;
            }
            if (hitk >= 0) {
                hitpos = P[hitk] + 1;
                hitk = -1;
            }
            wave_lds_sync();
            const uint64_t live = ballot(!(cdone && ddone));
            if (all_done || live == 0) break;
            // the straggler path for the rest of the list
            const uint32_t rest = b + 64 < p.re ? b + 64 : p.re;
            if (__builtin_popcountll(live) <= d.strag_lanes && p.re - rest >= (uint32_t)d.strag_rest) {
                for (uint64_t lm = live; lm != 0; lm &= lm - 1) {
                    const int l = __builtin_ctzll(lm);
                    // pixel l's state, the same on every lane
                    const float sux = rdl(p.ux, l), suy = rdl(p.uy, l);
                    float sT = rdl(T, l), sC0 = rdl(C0, l), sC1 = rdl(C1, l), sC2 = rdl(C2, l);
                    float sDa = rdl(Da, l);
                    bool scd = rdl_u(cdone ? 1u : 0u, l) != 0u, sdd = rdl_u(ddone ? 1u : 0u, l) != 0u;
                    uint32_t slast = rdl_u(last, l), shp = rdl_u(hitpos, l);
                    uint32_t shg = rdl_u(hitg, l), snb = 0;
                    for (uint32_t j0 = rest; j0 < p.re && !(scd && sdd); j0 += 64) {
                        // one record per lane, evaluated at pixel l
                        const uint32_t j = j0 + (uint32_t)lane;
                        const bool ok = j < p.re;
                        const float4* src = w.prec + 4ull * (ok ? j : j0);
                        const float4 A = src[0], Bq = src[1], Cc = src[2];
                        float fvj;
                        const float dd = eval_rec<true>(A, Bq, Cc, sux, suy, rpf, false, fvj);
                        const bool in = ok && dd <= cut;
                        const bool hj = in && dd < Bq.z;
                        float zj = 0.f;
                        if constexpr (DM == 1) zj = in ? zf[__float_as_uint(Cc.z) & kGidMask] : 0.f;
                        // the records that reach it, in list order
                        const uint64_t hm = ballot(hj);
                        for (uint64_t mi = ballot(in); mi != 0; mi &= mi - 1) {
                            const int k = __builtin_ctzll(mi);
                            if (!scd) {
                                const float fv = rdl(fvj, k);
                                const float wgt = fv * sT;
                                sC0 = __builtin_fmaf(rdl(Bq.w, k), wgt, sC0);
                                sC1 = __builtin_fmaf(rdl(Cc.x, k), wgt, sC1);
                                sC2 = __builtin_fmaf(rdl(Cc.y, k), wgt, sC2);
                                if constexpr (DM == 1) sDa = __builtin_fmaf(rdl(zj, k), wgt, sDa);
                                sT = sT * (1.f - fv);
                                slast = j0 + (uint32_t)k + 1u;
                                snb += 1u;
                                scd = sT < teps;
                            }
                            if (!sdd && ((hm >> k) & 1ull) != 0) {
                                shg = rdl_u(__float_as_uint(Cc.z), k);
                                shp = j0 + (uint32_t)k + 1u;
                                sdd = true;
                            }
                            if (scd && sdd) break;
                        }
                    }
                    if (lane == l) {
                        T = sT;
                        C0 = sC0;
                        C1 = sC1;
                        C2 = sC2;
                        Da = sDa;
                        cdone = scd;
                        ddone = sdd;
                        last = slast;
                        hitpos = shp;
                        hitg = shg;
                        nblend += snb;
                    }
                }
                break;
            }
        }
        uint32_t cterm = (T < teps) ? last : p.re;
        cnt_eval += p.act ? (float)(max(cterm, hitpos ? hitpos : p.re) - p.rs) : 0.f;
        cnt_blend += nblend;
        if (p.act) {
            size_t pix = ((size_t)p.f * d.H + p.py) * d.W + p.px;
            out_c[3 * pix + 0] = C0;
            out_c[3 * pix + 1] = C1;
            out_c[3 * pix + 2] = C2;
            out_t[pix] = T;
            const int hit = hitpos ? (int)(hitg & kGidMask) : -1;
            float D = -1.f;
            if constexpr (DM == 1) {
                D = nblend ? Da : -1.f;
            } else if (hit >= 0) {
                const float4 hn = w.prec[4ull * (hitpos - 1u) + 3];
                if (plane_branch(d, hn.x, hn.y, hn.z, p.ux, p.uy)) {
                    double d0 = ((double)p.ux - d.cx) / d.fx, d1 = ((double)p.uy - d.cy) / d.fy;
                    double dn = ((double)hn.x * d0 + (double)hn.y * d1) + (double)hn.z;
                    D = (float)((double)hn.w / dn);
                } else {
                    D = w.zkey[(int64_t)p.f * d.N + hit];
                }
            }
            out_d[pix] = D;
            out_i[pix] = hit;
            reinterpret_cast<uint2*>(w.px_aux)[(size_t)p.ft * d.tarea + p.r] = make_uint2(last, hitpos);
        }
    }
    // per-wave counters: no shared-address atomics
    {
        float se = wave_sum(cnt_eval), sb = wave_sum((float)cnt_blend);
        uint32_t gw = blockIdx.x * 4u + (uint32_t)wv;
        if (lane == 0 && gw < (uint32_t)kMaxWaves) {
            w.wcount[gw] = (unsigned long long)se;
            w.wcount[kMaxWaves + gw] = (unsigned long long)sb;
        }
        if (lane == 0 && gw == 0) w.hdr->fwd_waves = gridDim.x * 4u;
    }
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

// The upstream gradients come from gC / gD, or, with `l1` set, are the L1
// loss of Eq. 7-8 at unit scale: sign(C - C*) per channel and, on pixels
// with a hit and a valid target, sign(D - D*) (out_c, tgt_c, tgt_d the
// rendered colour and the targets).  Both gradient paths are linear in
// their upstream, so the projection backward applies w_c / (3 |M|) to the
// colour slots and w_d / |M_D| to the depth slots; each workgroup leaves its
// sums of |C - C*|, |D - D*| and its count of M_D pixels in lwave for that.
struct L1Up {
    const float* out_c;
    const float* tgt_c;
    const float* tgt_d;
    int l1;
};

template <int DM>
__global__ RTG_BWD_BOUNDS void k_raster_bwd(Dims d, WS w, const float* __restrict__ out_d,
                                                 const float* __restrict__ out_t,
                                                 const int* __restrict__ out_i,
                                                 const float* __restrict__ gC,
                                                 const float* __restrict__ gD, L1Up up) {
    __shared__ float4 lds[4][3][64];
    __shared__ uint32_t ldp[4][64];
    __shared__ __attribute__((aligned(16))) float lred[4][9 * 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float4(*L)[64] = lds[wv];
    uint32_t* P = ldp[wv];
    float* red = lred[wv];
    ItemIter iter = make_iter(d.items_per_pop, d.static_share, w.hdr->n_items, &w.hdr->q_bwd, lane);
    // this lane's L1 sums, kept in LDS (its own slots) rather than in
    // registers that would live across the whole item loop
    __shared__ float l1acc[3][4][64];
    l1acc[0][wv][lane] = 0.f;
    l1acc[1][wv][lane] = 0.f;
    l1acc[2][wv][lane] = 0.f;
    const int myslot = scatter_slot(lane);
    const bool writer = (lane & 3) == 0 && myslot < 14;
    const float cut = d.cutoff2;
    float cnt_walk = 0.f;
    unsigned long long cnt_part = 0;
    (void)out_i;   // the depth hit is identified by its list position
    uint32_t it;
    while (iter.next(it)) {
        PixelOfItem p = decode_item(d, w, it, lane);
        size_t pix = ((size_t)p.f * d.H + p.py) * d.W + p.px;
        float Tc = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, gd = 0.f, D = -1.f;
        uint32_t last = p.rs, hitpos = 0;
        if (p.act) {
            Tc = out_t[pix];
            D = out_d[pix];
            if (up.l1) {
                const float e0 = up.out_c[3 * pix] - up.tgt_c[3 * pix];
                const float e1 = up.out_c[3 * pix + 1] - up.tgt_c[3 * pix + 1];
                const float e2 = up.out_c[3 * pix + 2] - up.tgt_c[3 * pix + 2];
                g0 = sgn(e0);
                g1 = sgn(e1);
                g2 = sgn(e2);
                const float dt = up.tgt_d[pix];
                const bool vd = D != -1.f && dt > 0.f;
                gd = vd ? sgn(D - dt) : 0.f;
                l1acc[0][wv][lane] += fabsf(e0) + fabsf(e1) + fabsf(e2);
                if (vd) {
                    l1acc[1][wv][lane] += fabsf(D - dt);
                    l1acc[2][wv][lane] += 1.f;
                }
            } else {
                g0 = gC[3 * pix];
                g1 = gC[3 * pix + 1];
                g2 = gC[3 * pix + 2];
                gd = gD[pix];
            }
            uint2 aux = reinterpret_cast<const uint2*>(w.px_aux)[(size_t)p.ft * d.tarea + p.r];
            last = aux.x;
            // alpha-blended depth: the depth path follows the colour's
            hitpos = (DM == 0 && gd != 0.f) ? aux.y : 0u;
        }
        const PackBox pb = pack_box(p);
        // the frame is the same for every lane of the pack: a scalar base
        const float* rpf = w.recp + 6 * ((int64_t)readfirstlane(p.f) * d.N);
        const float* zf = w.zkey + (int64_t)readfirstlane(p.f) * d.N;
        uint32_t jend = wave_max_u32(max(last, hitpos));
        float A0 = 0.f, A1 = 0.f, A2 = 0.f, Az = 0.f;
        Batch<3> B = {};
        if (jend > p.rs) B = load_batch<3>(w, jend - p.rs > 64u ? jend - 64u : p.rs, jend, lane);
        for (uint32_t top = jend; top > p.rs;) {
            uint32_t b0 = top - p.rs > 64u ? top - 64u : p.rs;
            bool anyp;
            uint32_t nk = compact_batch<3>(B, b0, L, P, lane, pb, cut, anyp);
            wave_lds_sync();
            if (b0 > p.rs) B = load_batch<3>(w, b0 - p.rs > 64u ? b0 - 64u : p.rs, b0, lane);
            // the record loop; when the batch holds a precise record (a
            // uniform test), the value distance of those comes from the
            // whitened offsets e = U (u - mu) (Q = U^T U), and the conic
            // slots take m = g e and M = g e e^T instead of the derivatives
            // by mu and Q, which the projection backward maps back through U
            {
                for (int k = (int)nk - 1; k >= 0; --k) {
                    uint32_t j = P[k];
                    float4 A = L[0][k];
                    float4 Bq = L[1][k];
                    float4 Cc = L[2][k];
                    float dxd = p.ux - A.x, dyd = p.uy - A.y;
                    float dd = __builtin_fmaf(Bq.x * dyd, dyd, __builtin_fmaf(A.w * dxd, dyd, (A.z * dxd) * dxd));
                    bool part = (j < last) && (dd <= cut);
                    bool ish = (j + 1 == hitpos);
                    const uint64_t bp = ballot(part), bh = ballot(ish);
                    if ((bp | bh) == 0) continue;   // no pixel of the wave takes part
                    float2 lo = unpack_mu_lo(Cc.w);
                    float dx = dxd - lo.x, dy = dyd - lo.y;
                    float ddv = __builtin_fmaf(Bq.x * dy, dy, __builtin_fmaf(A.w * dx, dy, (A.z * dx) * dx));
                    if (anyp) {
                        // (dx, dy) become the whitened offsets; every lane
                        // holds the same record: a uniform branch and scalar
                        // loads
                        const uint32_t gwu = (uint32_t)readfirstlane((int)__float_as_uint(Cc.z));
                        if (gwu & kPreciseBit) {
                            const int gu = (int)(gwu & kGidMask);
                            precise_offsets(rpf + 6 * (int64_t)gu, p.ux, p.uy, A.x, A.y, dxd, dyd, dx, dy);
                            ddv = dx * dx + dy * dy;
                            // conic entries for the slots below: with
                            // Q.xx = Q.yy = -1/2 and Q.xy = 0 they take
                            // m = g e and M = g e e^T
                            A.z = -0.5f;
                            A.w = 0.f;
                            Bq.x = -0.5f;
                        }
                    }
                    float g = gauss_weight(ddv);
                    float fa = Bq.y * g;
                    bool clamped = fa > 0.99f;
                    float fv = clamped ? 0.99f : fa;
                    float om = 1.f - fv;
                    float Tb = Tc * __builtin_amdgcn_rcpf(om);
                    float zr = 0.f;
                    if constexpr (DM == 1) zr = zf[readfirstlane((int)rec_gid(Cc))];
                    // gradient terms and their reduction only for an unstable
                    // Gaussian (the record is the same on every lane: a
                    // uniform branch); a stable one only moves T and the
                    // colour behind
                    if ((readfirstlane((int)__float_as_uint(Cc.z)) & (int)kUnstableBit) != 0) {
                        float wgt = fv * Tb;
                        float gsum = (g0 * (Bq.w - A0) + g1 * (Cc.x - A1)) + g2 * (Cc.y - A2);
                        if constexpr (DM == 1) gsum = __builtin_fmaf(gd, zr - Az, gsum);
                        float gf = gsum * Tb;
                        float gdd = (part && !clamped) ? -0.5f * fv * gf : 0.f;
                        float v[16];
                        float qb = 0.5f * A.w;
                        v[0] = gdd * -2.f * (A.z * dx + qb * dy);
                        v[1] = gdd * -2.f * (qb * dx + Bq.x * dy);
                        v[2] = gdd * dx * dx;
                        v[3] = gdd * 2.f * dx * dy;
                        v[4] = gdd * dy * dy;
                        v[5] = (part && !clamped) ? gf * g : 0.f;
                        float wp = part ? wgt : 0.f;
                        v[6] = g0 * wp;
                        v[7] = g1 * wp;
                        v[8] = g2 * wp;
                        // depth path (Eq. 4-5) of the pixels whose depth hit this is
                        float da = 0.f, db0 = 0.f, db1 = 0.f, db2 = 0.f, de = 0.f;
                        if (bh != 0 && ish) {
                            const float4 nh = w.prec[4ull * j + 3];
                            if (plane_branch(d, nh.x, nh.y, nh.z, p.ux, p.uy)) {
                                float rx = (float)(((double)p.ux - d.cx) / d.fx);
                                float ry = (float)(((double)p.uy - d.cy) / d.fy);
                                float dn = (nh.x * rx + nh.y * ry) + nh.z;
                                da = gd / dn;
                                float aD = da * D;
                                db0 = aD * rx;
                                db1 = aD * ry;
                                db2 = aD;
                            } else {
                                de = gd;
                            }
                        }
                        if constexpr (DM == 1) de = gd * wp;   // dL/dz of the blended depth
                        v[9] = da;
                        v[10] = db0;
                        v[11] = db1;
                        v[12] = db2;
                        v[13] = de;
                        v[14] = 0.f;
                        v[15] = 0.f;
                        float* gr = w.grad + 16 * ((int64_t)p.f * d.N + rec_gid(Cc)) + myslot;
                        if (DM == 0 && bh == 0) {
                            float tot, tot8;
                            lds_sum9(v, red, lane, tot, tot8);
                            float* g0p = w.grad + 16 * ((int64_t)p.f * d.N + rec_gid(Cc));
                            if ((lane & 7) == 0) atomic_add_f32(g0p + (lane >> 3), tot);
                            if (lane == 1) atomic_add_f32(g0p + 8, tot8);
                        } else {
                            float tot = reduce_scatter16(v, lane);
                            if (writer) atomic_add_f32(gr, tot);
                        }
                    }
                    // (a pixel that does not take part adds 0 and keeps its
                    // colour behind: fma(0, c, 1 * A) = A exactly)
                    const float fp = part ? fv : 0.f, op = 1.f - fp;
                    A0 = __builtin_fmaf(fp, Bq.w, op * A0);
                    A1 = __builtin_fmaf(fp, Cc.x, op * A1);
                    A2 = __builtin_fmaf(fp, Cc.y, op * A2);
                    if constexpr (DM == 1) Az = __builtin_fmaf(fp, zr, op * Az);
                    Tc = part ? Tb : Tc;
                    cnt_part += (unsigned long long)__builtin_popcountll(bp);
                }
            }
            wave_lds_sync();
            top = b0;
        }
        cnt_walk += (float)(last - p.rs);
    }
    {
        float sw = wave_sum(cnt_walk);
        uint32_t gw = blockIdx.x * 4u + (uint32_t)wv;
        if (lane == 0 && gw < (uint32_t)kMaxWaves) {
            w.wcount[2 * kMaxWaves + gw] = (unsigned long long)sw;
            w.wcount[3 * kMaxWaves + gw] = cnt_part;
        }
        if (up.l1) {
            // one triple per workgroup (every wave reaches this point)
            __shared__ float l1red[3][4];
            const float sc = wave_sum(l1acc[0][wv][lane]), sd = wave_sum(l1acc[1][wv][lane]);
            const float sn = wave_sum(l1acc[2][wv][lane]);
            if (lane == 0) {
                l1red[0][wv] = sc;
                l1red[1][wv] = sd;
                l1red[2][wv] = sn;
            }
            __syncthreads();
            if (threadIdx.x == 0 && blockIdx.x < (uint32_t)kMaxWaves) {
                w.lwave[blockIdx.x] = (l1red[0][0] + l1red[0][1]) + (l1red[0][2] + l1red[0][3]);
                w.lwave[kMaxWaves + blockIdx.x] = (l1red[1][0] + l1red[1][1]) + (l1red[1][2] + l1red[1][3]);
                w.lwave[2 * kMaxWaves + blockIdx.x] = (l1red[2][0] + l1red[2][1]) + (l1red[2][2] + l1red[2][3]);
            }
        }
        if (lane == 0 && gw == 0) w.hdr->bwd_waves = gridDim.x * 4u;
    }
}

}  // namespace rtg
