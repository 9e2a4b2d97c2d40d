// Internal device-side types of the rasterizer library (gfx950).
//
// Workspace data layout (all in one caller-owned buffer; "slot" = f*N + i,
// frame-major, one per (frame, Gaussian); slots of culled pairs are never
// read):
//   hdr        counters (pairs, pixels, items, overflow, queue heads)
//   rec        4 x float4 (64 bytes) per slot: the three words the
//              compositing loops read, {mu.x, mu.y, Q.xx, 2 Q.xy}
//              {Q.yy, alpha, tau, c.r} {c.g, c.b, gid | unstable, centre
//              residual}, then {n^c.x, n^c.y, n^c.z, h = p^c . n^c}
//   zkey       float per slot: camera z rounded to float (depth key)
//   rect       short4 per slot: pixel rectangle x0, x1, y0, y1 (inclusive)
//   grad       16 floats per slot: camera-space gradient accumulator
//              [dmu.x, dmu.y, dQ.xx, dQ.xy, dQ.yy, dalpha, dc.rgb,
//               depth-plane a, b.xyz, depth-centre e, pad, pad]
//   vis        uint32 per Gaussian: bit f set iff visible in frame f
//   tile_*     uint32 per (frame, tile): masked pixels, pair start, pair end
//   hist       uint32 per (frame, binning block, tile): pair counts, then the
//              block's offset inside the tile's pair range
//   pix        uint8 per (frame, tile, rank): in-tile index of the rank-th
//              masked pixel (raster order inside the tile)
//   px_aux     2 x uint32 per (frame, tile, rank): one past the absolute
//              pair position of the last Gaussian that changed the pixel's
//              colour, and one past the position of its depth hit (0: none)
//   items      uint32 work items: (frame, tile) * packs_per_tile + pack,
//              a pack being up to 64 masked pixels of one tile
//   pairs      uint32 sorted slot ids, per tile contiguous
//   keys       uint64 sort keys of the pairs, grouped per tile
//   prec       64-byte record per pair in sorted list order: the three hot
//              float4 and {n^c, h}
//   recp       6 floats per slot, written only for precise slots (footprint
//              condition number above kPreciseKappa): the conic's upper
//              Cholesky factor U (Q = U^T U) as {r_hi, r_lo, U.xx, U.yy} with
//              r = U.xy / U.xx = Q.xy / Q.xx split into two floats, and the
//              centre residual mu - fl32(mu) as two floats
//   scratch    uint64 merge buffer for tiles above the LDS sort capacity
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtg {

constexpr int kWave = 64;

struct Hdr {
    uint32_t n_pairs;      // K
    uint32_t n_px;         // masked pixels rendered
    uint32_t n_items;      // work items
    uint32_t overflow;     // K > max_pairs
    uint32_t n_big;        // tiles sorted on the long-list path
    uint32_t err;          // device error bits
    uint32_t q_fwd, pad_fwd;   // queue heads of the compositing kernels, cleared
    uint32_t q_bwd, pad_bwd;   // by k_queue_reset before each launch that pops
    float loss_c, loss_d;  // L1 sums
    uint32_t cnt_m, cnt_md;
    uint32_t q_big;        // next entry of the long-list queue
    uint32_t pad;
    uint32_t fwd_waves, bwd_waves;   // waves of the last render / backward launch
    uint32_t n_restaged;             // binning blocks whose staging overflowed (rtg_read_status)
    uint32_t pad2[5];
    unsigned long long sums[4];      // per-wave work counters summed (rtg_read_status)
};
static_assert(sizeof(Hdr) == 128, "header layout");

// Everything a kernel needs to know about sizes; passed by value.
struct Dims {
    int64_t N;
    int32_t F, W, H;
    int32_t tw, th, tx, ty;   // tile shape, tiles per row / column
    int32_t ntiles;           // tiles per frame
    int32_t tarea;            // tw * th
    int32_t ppt;              // packs per tile = ceil(tarea / 64)
    int32_t lg_tw;            // log2(tw)
    double fx, fy, cx, cy;
    float cutoff2, dilation, z_near, t_eps;
    uint32_t max_pairs;
    int32_t items_per_pop;
    int32_t strag_lanes, strag_rest;   // straggler path of the forward compositing kernel
    int32_t static_share;              // percent of the items handed out round robin before the queue
    int32_t fwd_items_per_pop, fwd_static_share;   // the same two for the forward compositing kernel
    int32_t sort_cap;
    // binning blocks: block (f, b, c) counts / scatters the pairs of
    // Gaussians [b * gpb, (b + 1) * gpb) in frame f that fall in tiles
    // [c * chunk, (c + 1) * chunk) of the frame
    int32_t gpb, nbpf, chunk, nchunks;
    int32_t big_chunk;   // run length of the long-list sort (power of two <= 4096)
    // pair staging: binning block k stages its pairs in region k mod nreg
    // of rcap 16-byte entries (laid over the pair records, which are
    // written only after the pairs are placed)
    int32_t nreg;
    uint32_t rcap;
    int64_t ngrp;   // groups of 64 Gaussians: ceil(N / 64)
    int32_t sh_deg; // colour parameters: 0 = RGB [N][3], D = SH [N][(D+1)^2][3]
    int32_t depth_mode;  // 0 = disc depth (Eq. 4-5), 1 = alpha-blended depth
};

// Device pointers into the workspace; passed by value.
struct WS {
    Hdr* hdr;
    float4* rec;            // 4 x float4 per slot: the three hot words, then {n^c, h}
    float* zkey;
    short4* rect;
    float* grad;
    uint32_t* vis;
    uint32_t* tile_npx;
    uint32_t* tile_start;   // pair range [start, end) per (frame, tile)
    uint32_t* tile_end;
    uint32_t* hist;         // [F][nbpf][ntiles] pair counts per (frame, block, tile),
                            // then their exclusive scan over the blocks
    uint8_t* pix;
    uint32_t* px_aux;       // per masked pixel: last colour contributor, hit position + 1
    uint32_t* items;
    uint32_t* pairs;        // slot ids grouped per (frame, tile), then sorted
    uint32_t* bigl;         // (frame, tile)s whose lists exceed sort_cap, tile order
    uint32_t* bigl2;        // the same, longest lists first
    uint32_t* bigr;         // first run-sort job of each bigl2 entry, then their total
    float4* prec;           // 4 x float4 per pair, in sorted list order
    float* recp;            // 6 floats per precise slot: r_hi, r_lo, U.xx, U.yy, residual
    unsigned long long* keys;     // per pair: (depth bits << 32) | Gaussian index, grouped per tile
    unsigned long long* scratch;  // per pair: merge buffer of the long-list sort
    unsigned long long* wcount;   // [4][kMaxWaves] per-wave work counters
    float* lwave;                 // [3][kMaxWaves] per-wave L1 sums (colour, depth, depth count)
    uint32_t* stagec;             // [256] entries claimed per staging region
    uint32_t* bfail;              // per binning block: 1 if its staging overflowed
    uint32_t* vcnt;               // [F][ngrp] visible Gaussians per group of 64
    uint8_t* vlist;               // [F][ngrp][64] their indices inside the group, ascending
    unsigned long long* chunk;    // [chunks of 4096 (frame, tile)s][16]: totals and bases
};

// Hot record word 2 packs the Gaussian index with the unstable flag in bit
// 31, and word 3 the residual of the pixel centre, mu - fl32(mu), scaled by
// 2^12 as two halves: the compositing value path measures pixel offsets from
// the centre to binary32 precision of the offset itself, not of the centre.
constexpr uint32_t kUnstableBit = 0x80000000u;
constexpr float kLoScale = 4096.0f;

// Precise slots: footprints whose condition number lambda_max / lambda_min
// of Sigma_2D exceeds kPreciseKappa.  Binary32 conic entries and the
// binary32 evaluation perturb the quadratic form by a few 2^-24 kappa d^2,
// which reaches 1e-4 of a colour near kappa = 1000, so above 256 the value
// path (f, colours, gradients) evaluates d^2 from the factored form in recp
// instead (needle footprints of surfels seen edge-on; surfels of thickness
// ratio 0.1 stay below 100).
// Bit 30 of the index word marks them; Gaussian indices use bits 0-29.
constexpr uint32_t kPreciseBit = 0x40000000u;
constexpr uint32_t kGidMask = 0x3fffffffu;
constexpr double kPreciseKappa = 256.0;

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int rec_gid(float4 h2) { return (int)(__float_as_uint(h2.z) & kGidMask); }
__device__ __forceinline__ bool rec_unstable(float4 h2) { return (__float_as_uint(h2.z) & kUnstableBit) != 0u; }
__device__ __forceinline__ bool rec_precise(float4 h2) { return (__float_as_uint(h2.z) & kPreciseBit) != 0u; }

// Whitened offsets e = U (u - mu) of a pixel centre from a precise slot
// (Q = U^T U, so d^2 = e0^2 + e1^2), with e0 = U.xx (dx + r dy) and
// e1 = U.yy dy.  For a needle footprint dx + r dy cancels to a small
// fraction of its terms, so every part of it is kept exact until one
// rounding: the offsets from the binary32 centre, dxd = fl(u.x - fl32(mu.x))
// and dyd, come with their exact rounding errors (Knuth's TwoSum; the
// library is built without contraction, so the sequence is evaluated as
// written), fma(r_hi, dyd, dxd) rounds once, and the remaining small parts
// (those errors, the centre residual mu - fl32(mu), r_lo) are added after.
// The error of e0 is then a few units in the last place of e0 itself at
// any condition number.  `r` is the slot's recp entry and (mux, muy) the
// binary32 centre, the same for every lane of the wave.
__device__ __forceinline__ void precise_offsets(const float* __restrict__ r, float ux, float uy, float mux,
                                                float muy, float dxd, float dyd, float& e0, float& e1) {
    const float bx = dxd - ux, by = dyd - uy;
    const float ex = (ux - (dxd - bx)) + (-mux - bx);
    const float ey = (uy - (dyd - by)) + (-muy - by);
    const float sx = ex - r[4], sy = ey - r[5];   // small parts of dx, dy
    const float t = __builtin_fmaf(r[0], dyd, dxd);
    const float c = __builtin_fmaf(r[1], dyd, __builtin_fmaf(r[0], sy, sx));
    e0 = r[2] * (t + c);
    e1 = r[3] * (dyd + sy);
}

__device__ __forceinline__ float pack_mu_lo(float lx, float ly) {
    half2_t v = {(_Float16)(lx * kLoScale), (_Float16)(ly * kLoScale)};
    return __builtin_bit_cast(float, v);
}
__device__ __forceinline__ float2 unpack_mu_lo(float w) {
    half2_t v = __builtin_bit_cast(half2_t, w);
    return make_float2((float)v.x * (1.0f / kLoScale), (float)v.y * (1.0f / kLoScale));
}

// Value-path squared distance: offsets from the centre including its
// residual, same quadratic form as the decision.
__device__ __forceinline__ float dd_value(float4 h0, float qc, float2 lo, float ux, float uy, float& dx,
                                          float& dy) {
    dx = (ux - h0.x) - lo.x;
    dy = (uy - h0.y) - lo.y;
    float t0 = (h0.z * dx) * dx;
    float t1 = __builtin_fmaf(h0.w * dx, dy, t0);
    return __builtin_fmaf(qc * dy, dy, t1);
}

constexpr int kMaxWaves = 32768;  // per-wave counter slots of the persistent kernels

// Decision-layer squared Mahalanobis distance (binary32, fixed sequence:
// two products, then two single-rounding fused multiply-adds).
__device__ __forceinline__ float dd_decision(float mux, float muy, float qa, float qb2, float qc,
                                             float ux, float uy) {
    float dx = ux - mux;
    float dy = uy - muy;
    float t0 = (qa * dx) * dx;
    float t1 = __builtin_fmaf(qb2 * dx, dy, t0);
    return __builtin_fmaf(qc * dy, dy, t1);
}

// Eq. 5 branch: true iff the unsigned angle between the line of the normal
// and the pixel ray is below 60 degrees, (n.d)^2 > |d|^2 |n|^2 / 4 with d a
// positive multiple of K^-1 u (binary64, fixed sequence, division free).
__device__ __forceinline__ bool plane_branch(const Dims& d, float n0f, float n1f, float n2f,
                                             float ux, float uy) {
    double n0 = n0f, n1 = n1f, n2 = n2f;
    double d0 = d.fy * ((double)ux - d.cx);
    double d1 = d.fx * ((double)uy - d.cy);
    double d2 = d.fx * d.fy;
    double nd = (n0 * d0 + n1 * d1) + n2 * d2;
    double lhs = nd * nd;
    double dd = (d0 * d0 + d1 * d1) + d2 * d2;
    double nn = (n0 * n0 + n1 * n1) + n2 * n2;
    double rhs = (0.25 * dd) * nn;
    return lhs > rhs;
}

__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int readfirstlane(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the 64 lanes with DPP row operations and cross-row readlanes;
// every lane receives the total.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    v += dpp_mov<0x140>(v);  // row_mirror: every lane holds its row's sum
    float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ void atomic_add_f32(float* p, float v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ float sgn(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

}  // namespace rtg
