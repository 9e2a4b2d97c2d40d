// Steps a2-a4: masked pixels per tile, (Gaussian, tile) pairs, per-tile
// depth order (supplementary Sec. B: tiles, a key of view depth and tile id,
// sorting; the optional 50 % sparse-tile rule).
//
// No shared-address device atomics anywhere (on a multi-XCD part they
// serialise far from the CU):
//   1. per (frame, tile): masked-pixel count and compacted pixel list;
//   2. one workgroup: work items, and a summed-area table of tile activity
//      per frame so a Gaussian counts the active tiles of its rectangle in
//      O(1);
//   3. per Gaussian: pair count; per block: its sum (the reduce phase);
//   4. one workgroup: exclusive scan of the block sums (the spine);
//   5. per Gaussian: block-local scan + spine offset -> deterministic slots;
//      emit (frame*tiles + tile, slot) pairs in Gaussian order;
//   6. stable LSD radix sort of the pairs by that key (8-bit digits,
//      per-block LDS histograms, digit-major scan, wave-ballot ranking);
//   7. tile ranges from the key boundaries;
//   8. each tile's pairs ordered by (depth bits, Gaussian index) in LDS
//      (bitonic; a global-memory bitonic above the LDS capacity).
// Keys are unique inside a tile, so the order equals the full (frame, tile,
// depth, index) sort and is deterministic.
#include "rtg_common.h"

namespace rtg {

constexpr int kSortLds = 4096;  // keys sorted in LDS per tile (32 KB)
constexpr int kRadixBlocks = 512;

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
// wave per tile.
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
    if (lane == 0) w.tile_npx[ft] = cnt;
}

// One workgroup: work items from the per-tile pixel counts, the per-frame
// summed-area table of active tiles (row-padded: (ty+1) x (tx+1), zero first
// row and column), and cleared pair ranges.
__global__ __launch_bounds__(1024) void k_tile_scan(Dims d, WS w) {
    __shared__ uint32_t si[1024], sx[1024];
    const int tid = threadIdx.x;
    const int64_t total = (int64_t)d.F * d.ntiles;
    const int64_t seg = (total + 1023) / 1024;
    const int64_t beg = tid * seg, end = min(beg + seg, total);
    uint32_t li = 0, lx = 0;
    for (int64_t e = beg; e < end; ++e) {
        uint32_t npx = w.tile_npx[e];
        li += (npx + 63) >> 6;
        lx += npx;
        w.tile_start[e] = 0u;
        w.tile_end[e] = 0u;
    }
    si[tid] = li;
    sx[tid] = lx;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t vi = tid >= off ? si[tid - off] : 0u;
        uint32_t vx = tid >= off ? sx[tid - off] : 0u;
        __syncthreads();
        si[tid] += vi;
        sx[tid] += vx;
        __syncthreads();
    }
    uint32_t oi = si[tid] - li;
    for (int64_t e = beg; e < end; ++e) {
        uint32_t packs = (w.tile_npx[e] + 63) >> 6;
        for (uint32_t p = 0; p < packs; ++p) w.items[oi + p] = (uint32_t)e * (uint32_t)d.ppt + p;
        oi += packs;
    }
    if (tid == 0) {
        w.hdr->n_px = sx[1023];
        w.hdr->n_items = si[1023];
    }
    // summed-area table: rows, then columns
    const int sw = d.tx + 1, sh = d.ty + 1;
    for (int r = tid; r < d.F * sh; r += 1024) {
        int f = r / sh, y = r % sh;
        uint32_t* row = w.sat + ((size_t)f * sh + y) * sw;
        uint32_t acc = 0;
        row[0] = 0u;
        for (int x = 1; x < sw; ++x) {
            if (y > 0) acc += w.tile_npx[(size_t)f * d.ntiles + (y - 1) * d.tx + (x - 1)] ? 1u : 0u;
            row[x] = acc;
        }
    }
    __syncthreads();
    for (int c = tid; c < d.F * sw; c += 1024) {
        int f = c / sw, x = c % sw;
        uint32_t* base = w.sat + (size_t)f * sh * sw + x;
        uint32_t acc = 0;
        for (int y = 0; y < sh; ++y) {
            acc += base[(size_t)y * sw];
            base[(size_t)y * sw] = acc;
        }
    }
}

__device__ __forceinline__ void tile_range(const Dims& d, short4 r, int& a0, int& a1, int& b0, int& b1) {
    a0 = r.x >> d.lg_tw;
    a1 = r.y >> d.lg_tw;
    b0 = r.z / d.th;
    b1 = r.w / d.th;
}

__device__ __forceinline__ uint32_t sat_count(const Dims& d, const uint32_t* S, int a0, int a1, int b0, int b1) {
    const int sw = d.tx + 1;
    return S[(b1 + 1) * sw + (a1 + 1)] - S[b0 * sw + (a1 + 1)] - S[(b1 + 1) * sw + a0] + S[b0 * sw + a0];
}

__device__ __forceinline__ uint32_t block_sum_256(uint32_t v, uint32_t* red) {
    // 256 threads: wave sums via ballot-free shuffles, then 4 partials
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t s = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return s;
}

// Pair count per Gaussian (active tiles of its rectangle in every frame that
// sees it) and per block (reduce phase of the scan).
__global__ __launch_bounds__(256) void k_pair_count(Dims d, WS w) {
    __shared__ uint32_t red[4];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t c = 0;
    if (i < d.N) {
        uint32_t vis = w.vis[i];
        const size_t fs = (size_t)(d.tx + 1) * (d.ty + 1);
        while (vis) {
            int f = __builtin_ctz(vis);
            vis &= vis - 1;
            int a0, a1, b0, b1;
            tile_range(d, w.rect[(int64_t)f * d.N + i], a0, a1, b0, b1);
            c += sat_count(d, w.sat + f * fs, a0, a1, b0, b1);
        }
        w.cnt[i] = c;
    }
    uint32_t s = block_sum_256(c, red);
    if (threadIdx.x == 0) w.bsum[blockIdx.x] = s;
}

// Exclusive scan of the block sums (one workgroup); total pairs, overflow.
__global__ __launch_bounds__(1024) void k_spine(Dims d, WS w, uint32_t nblocks) {
    __shared__ uint32_t s[1024];
    const int tid = threadIdx.x;
    const uint32_t seg = (nblocks + 1023) / 1024;
    const uint32_t beg = tid * seg, end = min(beg + seg, nblocks);
    uint32_t l = 0;
    for (uint32_t e = beg; e < end; ++e) l += w.bsum[e];
    s[tid] = l;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = tid >= off ? s[tid - off] : 0u;
        __syncthreads();
        s[tid] += v;
        __syncthreads();
    }
    uint32_t o = s[tid] - l;
    for (uint32_t e = beg; e < end; ++e) {
        uint32_t v = w.bsum[e];
        w.bsum[e] = o;
        o += v;
    }
    if (tid == 0) {
        uint32_t K = s[1023];
        bool overflow = K > d.max_pairs;
        w.hdr->n_pairs = K;
        w.hdr->overflow = overflow ? 1u : 0u;
        if (overflow) w.hdr->n_items = 0u;
    }
}

// Emit the pairs of each Gaussian at its scanned offset, frames then tile
// rows then tile columns; keys = frame * tiles + tile, values = slot.
// Gaussians whose rectangles span more than kSoloTiles tiles are emitted by
// the whole wave (lanes split the tiles, a ballot prefix gives the output
// positions), so one near-camera Gaussian does not serialise a thread.
constexpr int kSoloTiles = 32;

__device__ __forceinline__ int rect_tiles(const Dims& d, const WS& w, int64_t i, uint32_t vis) {
    int n = 0;
    while (vis) {
        int f = __builtin_ctz(vis);
        vis &= vis - 1;
        int a0, a1, b0, b1;
        tile_range(d, w.rect[(int64_t)f * d.N + i], a0, a1, b0, b1);
        n += (a1 - a0 + 1) * (b1 - b0 + 1);
    }
    return n;
}

__global__ __launch_bounds__(256) void k_pair_emit(Dims d, WS w) {
    __shared__ uint32_t sc[256];
    const int lane = threadIdx.x & 63;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t c = i < d.N ? w.cnt[i] : 0u;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = threadIdx.x >= (unsigned)off ? sc[threadIdx.x - off] : 0u;
        __syncthreads();
        sc[threadIdx.x] += v;
        __syncthreads();
    }
    bool ok = i < d.N && c != 0 && !w.hdr->overflow;
    uint32_t o = ok ? w.bsum[blockIdx.x] + sc[threadIdx.x] - c : 0u;
    uint32_t vis = ok ? w.vis[i] : 0u;
    bool big = ok && rect_tiles(d, w, i, vis) > kSoloTiles;
    if (ok && !big) {
        while (vis) {
            int f = __builtin_ctz(vis);
            vis &= vis - 1;
            int64_t slot = (int64_t)f * d.N + i;
            int a0, a1, b0, b1;
            tile_range(d, w.rect[slot], a0, a1, b0, b1);
            const uint32_t* npx = w.tile_npx + (int64_t)f * d.ntiles;
            uint32_t kbase = (uint32_t)f * (uint32_t)d.ntiles;
            for (int b = b0; b <= b1; ++b)
                for (int a = a0; a <= a1; ++a) {
                    int t = b * d.tx + a;
                    if (npx[t]) {
                        w.key0[o] = kbase + (uint32_t)t;
                        w.val0[o] = (uint32_t)slot;
                        ++o;
                    }
                }
        }
    }
    // wave-cooperative emission of the big rectangles, one Gaussian at a time
    uint64_t todo = ballot(big);
    const uint64_t lt = (1ull << lane) - 1ull;
    while (todo) {
        int src = __builtin_ctzll(todo);
        todo &= todo - 1;
        int64_t gi = (int64_t)__shfl((int)(i & 0x7fffffff), src);
        uint32_t go = (uint32_t)__shfl((int)o, src);
        uint32_t gvis = (uint32_t)__shfl((int)vis, src);
        while (gvis) {
            int f = __builtin_ctz(gvis);
            gvis &= gvis - 1;
            int64_t slot = (int64_t)f * d.N + gi;
            int a0, a1, b0, b1;
            tile_range(d, w.rect[slot], a0, a1, b0, b1);
            const int rw = a1 - a0 + 1, n = rw * (b1 - b0 + 1);
            const uint32_t* npx = w.tile_npx + (int64_t)f * d.ntiles;
            uint32_t kbase = (uint32_t)f * (uint32_t)d.ntiles;
            for (int base = 0; base < n; base += 64) {
                int q = base + lane;
                int t = 0;
                bool on = false;
                if (q < n) {
                    t = (b0 + q / rw) * d.tx + a0 + q % rw;
                    on = npx[t] != 0;
                }
                uint64_t bb = ballot(on);
                if (on) {
                    uint32_t pos = go + (uint32_t)__builtin_popcountll(bb & lt);
                    w.key0[pos] = kbase + (uint32_t)t;
                    w.val0[pos] = (uint32_t)slot;
                }
                go += (uint32_t)__builtin_popcountll(bb);
            }
        }
    }
}

// ---- stable LSD radix sort of (key, value) by key --------------------------

__device__ __forceinline__ void radix_chunk(uint32_t K, uint32_t& beg, uint32_t& end) {
    uint32_t chunk = (K + kRadixBlocks - 1) / kRadixBlocks;
    chunk = (chunk + 255u) & ~255u;
    beg = min(blockIdx.x * chunk, K);
    end = min(beg + chunk, K);
}

__global__ __launch_bounds__(256) void k_rs_hist(WS w, const uint32_t* __restrict__ keys, int shift, int bits) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t K = w.hdr->overflow ? 0u : w.hdr->n_pairs;
    uint32_t beg, end;
    radix_chunk(K, beg, end);
    const uint32_t mask = (1u << bits) - 1u;
    for (uint32_t e = beg + threadIdx.x; e < end; e += 256) atomicAdd(&h[(keys[e] >> shift) & mask], 1u);
    __syncthreads();
    w.rhist[threadIdx.x * kRadixBlocks + blockIdx.x] = h[threadIdx.x];
}

// Per digit row: exclusive scan of the block counts (one wave per digit,
// 64 lanes x kRadixBlocks/64 consecutive counts each) and the row total.
// The scatter kernel adds the exclusive prefix of the 256 row totals.
__global__ __launch_bounds__(256) void k_rs_scan(WS w) {
    constexpr int kPer = kRadixBlocks / 64;
    const int lane = threadIdx.x & 63;
    const int dg = blockIdx.x * 4 + (threadIdx.x >> 6);
    uint32_t* row = w.rhist + dg * kRadixBlocks + lane * kPer;
    uint32_t v[kPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        v[k] = row[k];
        s += v[k];
    }
    uint32_t incl = s;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += t;
    }
    uint32_t acc = incl - s;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        row[k] = acc;
        acc += v[k];
    }
    if (lane == 63) w.rtot[dg] = incl;
}

__global__ __launch_bounds__(256) void k_rs_scatter(WS w, const uint32_t* __restrict__ kin,
                                                    const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
                                                    uint32_t* __restrict__ vout, int shift, int bits) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // exclusive prefix of the digit totals, plus this block's offset
    {
        uint32_t t = w.rtot[tid];
        uint32_t incl = t;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t x = (uint32_t)__shfl_up((int)incl, o);
            if (lane >= o) incl += x;
        }
        if (lane == 63) wc[0][wv] = incl;
        __syncthreads();
        uint32_t wbase = 0;
        for (int q = 0; q < wv; ++q) wbase += wc[0][q];
        run[tid] = wbase + incl - t + w.rhist[tid * kRadixBlocks + blockIdx.x];
        __syncthreads();
    }
    uint32_t K = w.hdr->overflow ? 0u : w.hdr->n_pairs;
    uint32_t beg, end;
    radix_chunk(K, beg, end);
    const uint32_t mask = (1u << bits) - 1u;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (uint32_t base = beg; base < end; base += 256) {
        uint32_t e = base + tid;
        bool ok = e < end;
        uint32_t key = ok ? kin[e] : 0u;
        uint32_t val = ok ? vin[e] : 0u;
        uint32_t dg = (key >> shift) & mask;
        wc[0][tid] = 0u;
        wc[1][tid] = 0u;
        wc[2][tid] = 0u;
        wc[3][tid] = 0u;
        uint64_t m = ballot(ok);
        for (int bit = 0; bit < bits; ++bit) {
            uint64_t bb = ballot((dg >> bit) & 1u);
            m &= ((dg >> bit) & 1u) ? bb : ~bb;
        }
        __syncthreads();
        uint32_t rank = (uint32_t)__builtin_popcountll(m & lt);
        if (ok && rank == 0) wc[wv][dg] = (uint32_t)__builtin_popcountll(m);
        __syncthreads();
        if (ok) {
            uint32_t pre = 0;
            for (int q = 0; q < wv; ++q) pre += wc[q][dg];
            uint32_t pos = run[dg] + pre + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
        __syncthreads();
    }
}

// Tile ranges [start, end) from the boundaries of the sorted keys.
__global__ __launch_bounds__(256) void k_ranges(WS w, const uint32_t* __restrict__ keys) {
    uint32_t K = w.hdr->overflow ? 0u : w.hdr->n_pairs;
    uint32_t j = blockIdx.x * 256u + threadIdx.x;
    for (; j < K; j += gridDim.x * 256u) {
        uint32_t k = keys[j];
        if (j == 0 || keys[j - 1] != k) w.tile_start[k] = j;
        if (j == K - 1 || keys[j + 1] != k) w.tile_end[k] = j + 1;
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
// The sorted slot ids go to `pairs`, and each pair's 64-byte record (the
// three hot float4 and {n^c, h}) is copied into `prec` in list order, so the
// compositing kernels stage records with one coalesced load level.
__device__ __forceinline__ void put_sorted(const WS& w, uint32_t pos, uint32_t slot) {
    w.pairs[pos] = slot;
    const float4* h = w.hot + 3ull * slot;
    float4* o = w.prec + 4ull * pos;
    o[0] = h[0];
    o[1] = h[1];
    o[2] = h[2];
    o[3] = w.cold[slot];
}

__global__ __launch_bounds__(256) void k_tile_sort(Dims d, WS w) {
    __shared__ unsigned long long K[kSortLds];
    int64_t ft = blockIdx.x;
    if (w.hdr->overflow) return;
    uint32_t start = w.tile_start[ft];
    uint32_t n = w.tile_end[ft] - start;
    if (n == 0) return;
    uint32_t* pr = w.pairs + start;
    if (n == 1) {
        if (threadIdx.x == 0) put_sorted(w, start, pr[0]);
        return;
    }
    uint32_t fbase = (uint32_t)((ft / d.ntiles) * d.N);
    uint32_t P = 1;
    while (P < n) P <<= 1;
    if (n <= (uint32_t)d.sort_cap) {
        for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) K[j] = j < n ? sort_key(w, pr[j], fbase) : ~0ull;
        __syncthreads();
        bitonic(K, P);
        for (uint32_t j = threadIdx.x; j < n; j += blockDim.x)
            put_sorted(w, start + j, fbase + (uint32_t)(K[j] & 0xffffffffull));
    } else {
        unsigned long long* G = w.scratch + 2ull * start;
        if (threadIdx.x == 0) atomicAdd(&w.hdr->n_big, 1u);
        for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) G[j] = j < n ? sort_key(w, pr[j], fbase) : ~0ull;
        __syncthreads();
        bitonic(G, P);
        for (uint32_t j = threadIdx.x; j < n; j += blockDim.x)
            put_sorted(w, start + j, fbase + (uint32_t)(G[j] & 0xffffffffull));
    }
}

}  // namespace rtg
