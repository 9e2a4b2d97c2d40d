// Steps a2-a4: masked pixels per tile, (Gaussian, tile) pairs, per-tile
// depth order (supplementary Sec. B: tiles, a key of view depth and tile id,
// sorting; the optional 50 % sparse-tile rule).
//
// Design: instead of one global radix sort of 64-bit (tile | depth) keys,
// pairs are bucketed by tile with an exclusive scan of per-tile counts and
// atomic cursors, then each tile's bucket is ordered by the 64-bit key
// (depth bits << 32 | Gaussian index) in LDS.  Keys are unique inside a
// tile, so the result is deterministic and equals the order of the full
// (frame, tile, depth, index) sort; the pair traffic is one write, one
// read-modify-write in LDS and one final write per pair.
#include "rtg_common.h"

namespace rtg {

constexpr int kSortLds = 4096;  // keys sorted in LDS per tile (32 KB)

// Sparse-tile rule on a fixed 16x16 grid: a block keeps its masked pixels
// iff 2 * masked >= in-image pixels.  One wave per (frame, block).
__global__ __launch_bounds__(256) void k_filter50(Dims d, const uint8_t* __restrict__ mask,
                                                  uint8_t* __restrict__ out) {
    int bx_n = (d.W + 15) >> 4, by_n = (d.H + 15) >> 4;
    int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (blk >= (int64_t)d.F * bx_n * by_n) return;
    int f = (int)(blk / (bx_n * by_n));
    int b = (int)(blk % (bx_n * by_n));
    int x0 = (b % bx_n) * 16, y0 = (b / bx_n) * 16;
    const uint8_t* m = mask + (size_t)f * d.W * d.H;
    uint8_t* o = out + (size_t)f * d.W * d.H;
    int cnt = 0, area = 0;
    for (int k = lane; k < 256; k += 64) {
        int px = x0 + (k & 15), py = y0 + (k >> 4);
        bool in = px < d.W && py < d.H;
        area += __builtin_popcountll(ballot(in));
        cnt += __builtin_popcountll(ballot(in && m[(size_t)py * d.W + px] != 0));
    }
    bool keep = 2 * cnt >= area;
    for (int k = lane; k < 256; k += 64) {
        int px = x0 + (k & 15), py = y0 + (k >> 4);
        if (px < d.W && py < d.H) {
            size_t o_i = (size_t)py * d.W + px;
            o[o_i] = keep ? m[o_i] : (uint8_t)0;
        }
    }
}

// Masked pixels of each (frame, tile) in raster order inside the tile; one
// wave per tile.  Also clears the tile's pair counter.
__global__ __launch_bounds__(256) void k_tile_pixels(Dims d, WS w, const uint8_t* __restrict__ mask) {
    int64_t ft = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (ft >= (int64_t)d.F * d.ntiles) return;
    int f = (int)(ft / d.ntiles), t = (int)(ft % d.ntiles);
    int ox = (t % d.tx) * d.tw, oy = (t / d.tx) * d.th;
    const uint8_t* m = mask + (size_t)f * d.W * d.H;
    uint8_t* pl = w.pix + ft * d.tarea;
    uint32_t cnt = 0;
    uint64_t lt = (1ull << lane) - 1ull;
    for (int base = 0; base < d.tarea; base += 64) {
        int l = base + lane;
        int px = ox + (l & (d.tw - 1)), py = oy + (l >> d.lg_tw);
        bool on = l < d.tarea && px < d.W && py < d.H && m[(size_t)py * d.W + px] != 0;
        uint64_t b = ballot(on);
        if (on) pl[cnt + __builtin_popcountll(b & lt)] = (uint8_t)l;
        cnt += (uint32_t)__builtin_popcountll(b);
    }
    if (lane == 0) {
        w.tile_npx[ft] = cnt;
        w.tile_npairs[ft] = 0;
    }
}

__device__ __forceinline__ void tile_range(const Dims& d, short4 r, int& a0, int& a1, int& b0, int& b1) {
    a0 = r.x >> d.lg_tw;
    a1 = r.y >> d.lg_tw;
    b0 = r.z / d.th;
    b1 = r.w / d.th;
}

// One (Gaussian, tile) pair per visible slot and active tile of its
// rectangle: count per tile.
__global__ __launch_bounds__(256) void k_pair_count(Dims d, WS w) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.N) return;
    uint32_t vis = w.vis[i];
    while (vis) {
        int f = __builtin_ctz(vis);
        vis &= vis - 1;
        int a0, a1, b0, b1;
        tile_range(d, w.rect[(int64_t)f * d.N + i], a0, a1, b0, b1);
        const uint32_t* npx = w.tile_npx + (int64_t)f * d.ntiles;
        uint32_t* np = w.tile_npairs + (int64_t)f * d.ntiles;
        for (int b = b0; b <= b1; ++b)
            for (int a = a0; a <= a1; ++a) {
                int t = b * d.tx + a;
                if (npx[t]) atomicAdd(&np[t], 1u);
            }
    }
}

// Exclusive scans over all (frame, tile) entries in one workgroup: pair
// starts (and emit cursors), work-item offsets; writes the work items and
// the totals.  On pair overflow nothing is emitted or rendered.
__global__ __launch_bounds__(1024) void k_tile_scan(Dims d, WS w) {
    __shared__ uint32_t sp[1024], si[1024], sx[1024];
    const int tid = threadIdx.x;
    const int64_t total = (int64_t)d.F * d.ntiles;
    const int64_t seg = (total + 1023) / 1024;
    const int64_t beg = tid * seg, end = min(beg + seg, total);
    uint32_t lp = 0, li = 0, lx = 0;
    for (int64_t e = beg; e < end; ++e) {
        uint32_t npx = w.tile_npx[e];
        lp += w.tile_npairs[e];
        li += (npx + 63) >> 6;
        lx += npx;
    }
    sp[tid] = lp;
    si[tid] = li;
    sx[tid] = lx;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t vp = tid >= off ? sp[tid - off] : 0u;
        uint32_t vi = tid >= off ? si[tid - off] : 0u;
        uint32_t vx = tid >= off ? sx[tid - off] : 0u;
        __syncthreads();
        sp[tid] += vp;
        si[tid] += vi;
        sx[tid] += vx;
        __syncthreads();
    }
    uint32_t K = sp[1023], I = si[1023], P = sx[1023];
    bool overflow = K > d.max_pairs;
    uint32_t op = sp[tid] - lp, oi = si[tid] - li;
    for (int64_t e = beg; e < end; ++e) {
        uint32_t npx = w.tile_npx[e];
        uint32_t n = w.tile_npairs[e];
        uint32_t packs = (npx + 63) >> 6;
        w.tile_start[e] = op;
        w.tile_cursor[e] = op;
        w.tile_itemoff[e] = oi;
        if (!overflow)
            for (uint32_t p = 0; p < packs; ++p) w.items[oi + p] = (uint32_t)e * (uint32_t)d.ppt + p;
        op += n;
        oi += packs;
    }
    if (tid == 0) {
        w.hdr->n_pairs = K;
        w.hdr->n_px = P;
        w.hdr->n_items = overflow ? 0u : I;
        w.hdr->overflow = overflow ? 1u : 0u;
    }
}

__global__ __launch_bounds__(256) void k_pair_emit(Dims d, WS w) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.N) return;
    if (w.hdr->overflow) return;
    uint32_t vis = w.vis[i];
    while (vis) {
        int f = __builtin_ctz(vis);
        vis &= vis - 1;
        int64_t slot = (int64_t)f * d.N + i;
        int a0, a1, b0, b1;
        tile_range(d, w.rect[slot], a0, a1, b0, b1);
        const uint32_t* npx = w.tile_npx + (int64_t)f * d.ntiles;
        uint32_t* cur = w.tile_cursor + (int64_t)f * d.ntiles;
        for (int b = b0; b <= b1; ++b)
            for (int a = a0; a <= a1; ++a) {
                int t = b * d.tx + a;
                if (npx[t]) {
                    uint32_t p = atomicAdd(&cur[t], 1u);
                    w.pairs[p] = (uint32_t)slot;
                }
            }
    }
}

__device__ __forceinline__ unsigned long long sort_key(const WS& w, uint32_t slot, uint32_t fbase) {
    // camera z > z_near > 0, so the float bits order like the values
    return ((unsigned long long)__float_as_uint(w.zkey[slot]) << 32) | (unsigned long long)(slot - fbase);
}

template <typename Keys>
__device__ __forceinline__ void bitonic(Keys K, uint32_t P) {
    for (uint32_t k = 2; k <= P; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t idx = threadIdx.x; idx < (P >> 1); idx += blockDim.x) {
                uint32_t i = ((idx & ~(j - 1)) << 1) | (idx & (j - 1));
                uint32_t l = i | j;
                unsigned long long a = K[i], b = K[l];
                bool asc = (i & k) == 0;
                if ((a > b) == asc) {
                    K[i] = b;
                    K[l] = a;
                }
            }
            __syncthreads();
        }
}

// Order each tile's pairs by (depth bits, Gaussian index): LDS bitonic sort
// up to sort_cap keys, a global-memory bitonic sort on scratch above it.
__global__ __launch_bounds__(256) void k_tile_sort(Dims d, WS w) {
    __shared__ unsigned long long K[kSortLds];
    int64_t ft = blockIdx.x;
    if (w.hdr->overflow) return;
    uint32_t n = w.tile_npairs[ft];
    if (n < 2) return;
    uint32_t start = w.tile_start[ft];
    uint32_t fbase = (uint32_t)((ft / d.ntiles) * d.N);
    uint32_t P = 1;
    while (P < n) P <<= 1;
    uint32_t* pr = w.pairs + start;
    if (n <= (uint32_t)d.sort_cap) {
        for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) K[j] = j < n ? sort_key(w, pr[j], fbase) : ~0ull;
        __syncthreads();
        bitonic(K, P);
        for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) pr[j] = fbase + (uint32_t)(K[j] & 0xffffffffull);
    } else {
        unsigned long long* G = w.scratch + 2ull * start;
        if (threadIdx.x == 0) atomicAdd(&w.hdr->n_big, 1u);
        for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) G[j] = j < n ? sort_key(w, pr[j], fbase) : ~0ull;
        __syncthreads();
        bitonic(G, P);
        for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) pr[j] = fbase + (uint32_t)(G[j] & 0xffffffffull);
    }
}

}  // namespace rtg
