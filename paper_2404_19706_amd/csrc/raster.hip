// Steps a5 and a7: per-pixel forward compositing (Eq. 1-5) and its adjoint,
// over the masked pixels only.
//
// Work decomposition: a work item is a pack of up to 64 masked pixels of one
// (frame, tile), compacted so that sparse masks do not idle lanes.  Each
// wave64 of a persistent grid dequeues items_per_pop items at a time from an
// atomic queue head, stages the tile's depth-ordered Gaussian records in its
// own LDS slice 64 at a time, and walks them with one lane per pixel; every
// lane reads the same record (an LDS broadcast).  A ballot ends the walk
// once every lane has finished its colour and found its depth hit.
//
// The backward pass re-walks each pixel's list back to front, recovering the
// transmission in front of each Gaussian from the stored final value
// (T_i = T_{i+1} / (1 - f_i); nothing per pair is stored), reduces each
// unstable Gaussian's nine colour-path gradients across the wave with DPP,
// and adds them with one float atomic per value into the Gaussian's
// per-frame camera-space accumulator.
#include "rtg_common.h"

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
    p.re = p.rs + w.tile_npairs[p.ft];
    return p;
}

__device__ __forceinline__ void stage(const WS& w, float4 (*L)[64], uint32_t j, bool ok, int lane) {
    if (ok) {
        uint32_t s = w.pairs[j];
        const float4* h = w.hot + 3ull * s;
        L[0][lane] = h[0];
        L[1][lane] = h[1];
        L[2][lane] = h[2];
    }
}

__global__ __launch_bounds__(256) void k_raster_fwd(Dims d, WS w, float* __restrict__ out_c,
                                                    float* __restrict__ out_d, float* __restrict__ out_t,
                                                    int* __restrict__ out_i) {
    __shared__ float4 lds[4][3][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float4(*L)[64] = lds[wv];
    const uint32_t n_items = w.hdr->n_items;
    const uint32_t ipp = (uint32_t)d.items_per_pop;
    for (;;) {
        uint32_t it0 = 0;
        if (lane == 0) it0 = atomicAdd(&w.hdr->q_fwd, ipp);
        it0 = (uint32_t)readfirstlane((int)it0);
        if (it0 >= n_items) break;
        uint32_t it1 = min(it0 + ipp, n_items);
        for (uint32_t it = it0; it < it1; ++it) {
            PixelOfItem p = decode_item(d, w, it, lane);
            float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
            uint32_t last = p.rs;
            int hit = -1;
            bool cdone = !p.act, ddone = !p.act;
            for (uint32_t b = p.rs; b < p.re; b += 64) {
                stage(w, L, b + lane, b + lane < p.re, lane);
                wave_lds_sync();
                uint32_t nb = min(64u, p.re - b);
                bool all_done = false;
                for (uint32_t k = 0; k < nb; ++k) {
                    float4 A = L[0][k];
                    float4 B = L[1][k];
                    float dd = dd_decision(A.x, A.y, A.z, A.w, B.x, p.ux, p.uy);
                    bool in = dd <= d.cutoff2;
                    if (in && !cdone) {
                        float4 Cc = L[2][k];
                        float g = __expf(-0.5f * dd);
                        float fv = B.y * g;
                        fv = fv > 0.99f ? 0.99f : fv;
                        float wgt = fv * T;
                        C0 = __builtin_fmaf(B.w, wgt, C0);
                        C1 = __builtin_fmaf(Cc.x, wgt, C1);
                        C2 = __builtin_fmaf(Cc.y, wgt, C2);
                        T = T * (1.f - fv);
                        last = b + k + 1;
                        if (T < d.t_eps) cdone = true;
                    }
                    if (in && !ddone && dd < B.z) {
                        ddone = true;
                        hit = __float_as_int(L[2][k].z);
                    }
                    if (ballot(!(cdone && ddone)) == 0) {
                        all_done = true;
                        break;
                    }
                }
                wave_lds_sync();
                if (all_done) break;
            }
            if (p.act) {
                size_t pix = ((size_t)p.f * d.H + p.py) * d.W + p.px;
                out_c[3 * pix + 0] = C0;
                out_c[3 * pix + 1] = C1;
                out_c[3 * pix + 2] = C2;
                out_t[pix] = T;
                float D = -1.f;
                if (hit >= 0) {
                    int64_t slot = (int64_t)p.f * d.N + hit;
                    float4 cn = w.cold[slot];
                    if (plane_branch(d, cn.x, cn.y, cn.z, p.ux, p.uy)) {
                        double d0 = ((double)p.ux - d.cx) / d.fx, d1 = ((double)p.uy - d.cy) / d.fy;
                        double dn = ((double)cn.x * d0 + (double)cn.y * d1) + (double)cn.z;
                        D = (float)((double)cn.w / dn);
                    } else {
                        D = w.zkey[slot];
                    }
                }
                out_d[pix] = D;
                out_i[pix] = hit;
                w.px_last[(size_t)p.ft * d.tarea + p.r] = last;
            }
        }
    }
    if (lane == 0) {
        uint32_t prev = atomicAdd(&w.hdr->done_fwd, 1u);
        if (prev == gridDim.x * 4u - 1u) {
            w.hdr->q_fwd = 0u;
            w.hdr->done_fwd = 0u;
        }
    }
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

__global__ __launch_bounds__(256) void k_raster_bwd(Dims d, WS w, const float* __restrict__ out_d,
                                                    const float* __restrict__ out_t,
                                                    const int* __restrict__ out_i,
                                                    const float* __restrict__ gC,
                                                    const float* __restrict__ gD) {
    __shared__ float4 lds[4][3][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float4(*L)[64] = lds[wv];
    const uint32_t n_items = w.hdr->n_items;
    const uint32_t ipp = (uint32_t)d.items_per_pop;
    for (;;) {
        uint32_t it0 = 0;
        if (lane == 0) it0 = atomicAdd(&w.hdr->q_bwd, ipp);
        it0 = (uint32_t)readfirstlane((int)it0);
        if (it0 >= n_items) break;
        uint32_t it1 = min(it0 + ipp, n_items);
        for (uint32_t it = it0; it < it1; ++it) {
            PixelOfItem p = decode_item(d, w, it, lane);
            size_t pix = ((size_t)p.f * d.H + p.py) * d.W + p.px;
            float Tc = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, gd = 0.f, D = -1.f;
            int hit = -1;
            uint32_t last = p.rs;
            if (p.act) {
                Tc = out_t[pix];
                g0 = gC[3 * pix];
                g1 = gC[3 * pix + 1];
                g2 = gC[3 * pix + 2];
                gd = gD[pix];
                hit = out_i[pix];
                D = out_d[pix];
                last = w.px_last[(size_t)p.ft * d.tarea + p.r];
            }
            // depth path (Eq. 4-5): only the hit Gaussian, per-lane atomics
            if (hit >= 0 && (int64_t)hit < d.N && gd != 0.f) {
                int64_t slot = (int64_t)p.f * d.N + hit;
                if (__float_as_int(w.hot[3 * slot + 2].w) & kFlagUnstable) {
                    float* g = w.grad + 16 * slot;
                    float4 cn = w.cold[slot];
                    if (plane_branch(d, cn.x, cn.y, cn.z, p.ux, p.uy)) {
                        float dx = (float)(((double)p.ux - d.cx) / d.fx);
                        float dy = (float)(((double)p.uy - d.cy) / d.fy);
                        float dn = (cn.x * dx + cn.y * dy) + cn.z;
                        float a = gd / dn;
                        float aD = a * D;
                        atomic_add_f32(g + 9, a);
                        atomic_add_f32(g + 10, aD * dx);
                        atomic_add_f32(g + 11, aD * dy);
                        atomic_add_f32(g + 12, aD);
                    } else {
                        atomic_add_f32(g + 13, gd);
                    }
                }
            }
            // colour path, back to front from the last colour contributor
            uint32_t jend = wave_max_u32(last);
            float A0 = 0.f, A1 = 0.f, A2 = 0.f;
            for (uint32_t top = jend; top > p.rs;) {
                uint32_t b0 = top - p.rs > 64u ? top - 64u : p.rs;
                stage(w, L, b0 + lane, b0 + lane < top, lane);
                wave_lds_sync();
                for (int k = (int)(top - b0) - 1; k >= 0; --k) {
                    uint32_t j = b0 + (uint32_t)k;
                    float4 A = L[0][k];
                    float4 B = L[1][k];
                    float4 Cc = L[2][k];
                    float dd = dd_decision(A.x, A.y, A.z, A.w, B.x, p.ux, p.uy);
                    bool part = (j < last) && (dd <= d.cutoff2);
                    float g = __expf(-0.5f * dd);
                    float fa = B.y * g;
                    bool clamped = fa > 0.99f;
                    float fv = clamped ? 0.99f : fa;
                    float Tb = Tc / (1.f - fv);
                    float wgt = fv * Tb;
                    float gf = ((g0 * (B.w - A0) + g1 * (Cc.x - A1)) + g2 * (Cc.y - A2)) * Tb;
                    float gdd = clamped ? 0.f : -0.5f * fv * gf;
                    float dx = p.ux - A.x, dy = p.uy - A.y;
                    float qb = 0.5f * A.w;
                    float v0 = gdd * -2.f * (A.z * dx + qb * dy);
                    float v1 = gdd * -2.f * (qb * dx + B.x * dy);
                    float v2 = gdd * dx * dx;
                    float v3 = gdd * 2.f * dx * dy;
                    float v4 = gdd * dy * dy;
                    float v5 = clamped ? 0.f : gf * g;
                    float v6 = g0 * wgt, v7 = g1 * wgt, v8 = g2 * wgt;
                    if (part) {
                        A0 = fv * B.w + (1.f - fv) * A0;
                        A1 = fv * Cc.x + (1.f - fv) * A1;
                        A2 = fv * Cc.y + (1.f - fv) * A2;
                        Tc = Tb;
                    } else {
                        v0 = v1 = v2 = v3 = v4 = v5 = v6 = v7 = v8 = 0.f;
                    }
                    bool unst = (__float_as_int(Cc.w) & kFlagUnstable) != 0;
                    if (unst && ballot(part) != 0) {
                        float s0 = wave_sum(v0), s1 = wave_sum(v1), s2 = wave_sum(v2);
                        float s3 = wave_sum(v3), s4 = wave_sum(v4), s5 = wave_sum(v5);
                        float s6 = wave_sum(v6), s7 = wave_sum(v7), s8 = wave_sum(v8);
                        float mine = lane == 0 ? s0 : lane == 1 ? s1 : lane == 2 ? s2 : lane == 3 ? s3
                                   : lane == 4 ? s4 : lane == 5 ? s5 : lane == 6 ? s6 : lane == 7 ? s7 : s8;
                        int gid = __float_as_int(Cc.z);
                        if (lane < 9) atomic_add_f32(w.grad + 16 * ((int64_t)p.f * d.N + gid) + lane, mine);
                    }
                }
                wave_lds_sync();
                top = b0;
            }
        }
    }
    if (lane == 0) {
        uint32_t prev = atomicAdd(&w.hdr->done_bwd, 1u);
        if (prev == gridDim.x * 4u - 1u) {
            w.hdr->q_bwd = 0u;
            w.hdr->done_bwd = 0u;
        }
    }
}

}  // namespace rtg
