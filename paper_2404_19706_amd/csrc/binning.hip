// Steps a2-a4: masked pixels per tile, (Gaussian, tile) pairs, per-tile
// depth order (supplementary Sec. B: tiles, a key of view depth and tile id,
// sorting; the optional 50 % sparse-tile rule).
//
// No shared-address device atomics anywhere (on a multi-XCD part they
// serialise far from the CU):
//   1. per (frame, tile): masked-pixel count and compacted pixel list;
//   2. per binning block (frame, Gaussian range, tile chunk): pair counts
//      per tile in LDS, and every pair found staged with its rank in its
//      (block, tile) group (one claim on a staging region per 64+ pairs);
//   3. per (frame, tile): exclusive scan of the block counts;
//   4. one workgroup: pair range of every tile, total, capacity check, work
//      items (packs of up to 64 masked pixels), list of long tile lists;
//   5. per staged pair: its sort key (depth bits, index) written to tile
//      start + block offset + rank; a block whose staging region overflowed
//      enumerates its pairs again instead and writes them through LDS
//      cursors;
//   6. each tile's keys ordered in LDS (wave rank sort for short lists,
//      workgroup bitonic sort up to sort_cap, sorted runs and merge-path
//      rounds above), with the sorted slot ids and the pair-order record
//      copy for the compositing kernels.
// Keys are unique inside a tile, so the order equals the full (frame, tile,
// depth, index) sort and is deterministic.
#include "rtg_common.h"

namespace rtg {

constexpr int kSortLds = 4096;     // keys sorted in LDS per tile (32 KB)
constexpr int kHistChunk = 12288;  // tiles per binning block (48 KB of LDS counters)

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

// Masked pixels of each (frame, tile), compacted in 8x8-block order (blocks
// in raster order, raster order inside a block), so a full tile's packs of
// 64 pixels are 8x8 squares; one wave per tile.
// The first workgroup also clears the staging region counters of step 2.
__global__ __launch_bounds__(256) void k_tile_pixels(Dims d, WS w, const uint8_t* __restrict__ mask) {
    if (blockIdx.x == 0) w.stagec[threadIdx.x] = 0u;
    int64_t ft = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (ft >= (int64_t)d.F * d.ntiles) return;
    int f = (int)(ft / d.ntiles), t = (int)(ft % d.ntiles);
    int ox = (t % d.tx) * d.tw, oy = (t / d.tx) * d.th;
    const uint8_t* m = mask + (size_t)f * d.W * d.H;
    uint8_t* pl = w.pix + ft * d.tarea;
    const int bxn = d.tw >> 3;
    uint32_t cnt = 0;
    uint64_t lt = (1ull << lane) - 1ull;
    for (int blk = 0; blk < d.tarea >> 6; ++blk) {
        int lx = (blk % bxn) * 8 + (lane & 7), ly = (blk / bxn) * 8 + (lane >> 3);
        int l = ly * d.tw + lx;
        int px = ox + lx, py = oy + ly;
        bool on = px < d.W && py < d.H && m[(size_t)py * d.W + px] != 0;
        uint64_t b = ballot(on);
        if (on) pl[cnt + __builtin_popcountll(b & lt)] = (uint8_t)l;
        cnt += (uint32_t)__builtin_popcountll(b);
    }
    if (lane == 0) w.tile_npx[ft] = cnt;
}

__device__ __forceinline__ void tile_range(const Dims& d, short4 r, int& a0, int& a1, int& b0, int& b1) {
    a0 = r.x >> d.lg_tw;
    a1 = r.y >> d.lg_tw;
    b0 = r.z / d.th;
    b1 = r.w / d.th;
}

// ---- pairs: per-block tile histograms, scans, direct scatter ---------------
//
// Binning block (f, b, c) owns the Gaussians [b * gpb, (b + 1) * gpb) in
// frame f and the tiles [c * chunk, (c + 1) * chunk) of that frame.  It
// enumerates every (Gaussian, active tile) pair it owns twice: once to count
// pairs per tile in LDS (k_pair_hist), once, after the scans have fixed
// where its pairs of each tile start, to write them there (k_pair_scatter).
// Ranks inside a (block, tile) come from LDS atomics, so the order inside a
// tile is arbitrary until the per-tile sorts order it by (depth, index), a total
// order: the final lists are deterministic.
//
// The candidate tiles of a wave's 64 Gaussians are numbered by a scan of
// their counts and dealt to the lanes round robin, so a wave's time follows
// its total candidate count, not its largest rectangle.

struct Chunk {
    int f, b, t0, t1;
};

__device__ __forceinline__ Chunk chunk_of_block(const Dims& d) {
    Chunk c;
    int cc = (int)(blockIdx.x % (unsigned)d.nchunks);
    int rest = (int)(blockIdx.x / (unsigned)d.nchunks);
    c.b = rest % d.nbpf;
    c.f = rest / d.nbpf;
    c.t0 = cc * d.chunk;
    c.t1 = min(c.t0 + d.chunk, d.ntiles);
    return c;
}

// Active-tile bits of the chunk into LDS (one bit per tile): each wave
// reads 64 consecutive tile counts per step (up to four steps in flight)
// and stores their ballot.
__device__ __forceinline__ void load_active(const Dims& d, const WS& w, const Chunk& c, uint32_t* act) {
    const int ct = c.t1 - c.t0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t* npx = w.tile_npx + (int64_t)c.f * d.ntiles + c.t0;
    for (int base0 = wv * 64; base0 < ct; base0 += 4 * nw * 64) {
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int t = base0 + k * nw * 64 + lane;
            v[k] = t < ct ? npx[t] : 0u;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int base = base0 + k * nw * 64;
            const uint64_t bits = ballot(v[k] != 0u);
            if (base < ct) {
                if (lane == 0) act[base >> 5] = (uint32_t)bits;
                if (lane == 1 && base + 32 < ct) act[(base >> 5) + 1] = (uint32_t)(bits >> 32);
            }
        }
    }
}

// Column of the first active tile of the chunk in columns [x, xe] of the
// tile row that starts at chunk-relative tile rt; xe + 1 when there is none.
// Tiles outside the chunk count as inactive.
__device__ __forceinline__ int next_active(const uint32_t* act, int ct, int rt, int x, int xe) {
    int t = max(rt + x, 0);
    const int te = min(rt + xe, ct - 1);
    while (t <= te) {
        const uint32_t word = act[t >> 5] >> (t & 31);
        if (word != 0u) {
            const int ta = t + __builtin_ctz(word);
            return ta <= te ? ta - rt : xe + 1;
        }
        t = (t | 31) + 1;
    }
    return xe + 1;
}

// Position of the k-th set bit (from 0) of m; k < popcount(m).
__device__ __forceinline__ int select_bit(uint64_t m, int k) {
    int pos = 0;
#pragma unroll
    for (int h = 32; h > 0; h >>= 1) {
        const int c = __builtin_popcountll(m & ((1ull << h) - 1ull));
        if (k >= c) {
            k -= c;
            m >>= h;
            pos += h;
        }
    }
    return pos;
}

// Inclusive scan over the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, int lane) {
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    return v;
}

// Pair thinning, a fixed binary64 sequence that the reference binning
// follows as well.  Tile a of tile row b is kept for a Gaussian when the
// box of the tile's pixel centres (clipped to the image) meets the ellipse
// q <= c of the decision conic, q(x, y) = Q.xx x^2 + 2 Q.xy x y + Q.yy y^2 in
// offsets from the binary32 centre.  The bound c = (cut-off * 1.001 + 1e-3)
// + 1e-6 M, where M bounds |Q.xx| x^2 + |2 Q.xy x y| + |Q.yy| y^2 over the
// rectangle's columns and the row's band, covers the binary32 rounding of
// the per-pixel evaluation of q, so a dropped pair has d^2 above the
// cut-off at every pixel of its tile.  Per row: the x-range [xl, xh] of the
// ellipse inside the band y in [ly, hy].  Its right end is the ellipse's
// rightmost point x_t = sqrt(c Q.yy / det) when that point's y_t =
// -Q.xy x_t / Q.yy lies in the band, else the larger root of q(x, y_e) = c
// on the band edge y_e nearer to y_t; the left end is the mirror image
// (leftmost point (-x_t, -y_t)).  A negative discriminant on that edge
// means the band misses the ellipse.  Tile a is kept when lx(a) <= xh and
// hx(a) >= xl, lx / hx its box's ends; both grow with a, so the kept tiles
// of a row are one run [ka, kb].  A conic whose binary32 entries do not
// form a positive definite matrix (det computed exactly in sign: both
// products are exact in binary64) keeps every tile.
struct Conic {
    float mux, muy, qa, qb2, qc;
};

__device__ __forceinline__ double box_lo(const Dims& d, int a, double mux) {
    return ((double)(a * d.tw) + 0.5) - mux;
}
__device__ __forceinline__ double box_hi(const Dims& d, int a, double mux) {
    return ((double)min(a * d.tw + d.tw, d.W) - 0.5) - mux;
}

// Kept columns [ka, kb] (empty when ka > kb) of tile row b for a Gaussian
// whose rectangle spans tile columns [a0, a1].
__device__ __forceinline__ void row_span(const Dims& d, const Conic& k, int a0, int a1, int b, int& ka, int& kb) {
    ka = a0;
    kb = a1;
    const double qa = (double)k.qa, qb = 0.5 * (double)k.qb2, qc = (double)k.qc;
    const double det = qa * qc - qb * qb;
    if (!(qa > 0.0 && det > 0.0)) return;
    const double mux = (double)k.mux, muy = (double)k.muy;
    const double ly = ((double)(b * d.th) + 0.5) - muy;
    const double hy = ((double)min(b * d.th + d.th, d.H) - 0.5) - muy;
    const double X = fmax(-box_lo(d, a0, mux), box_hi(d, a1, mux)), Y = fmax(-ly, hy);
    const double M = ((qa * X) * X + ((2.0 * fabs(qb)) * X) * Y) + (qc * Y) * Y;
    const double c = ((double)d.cutoff2 * 1.001 + 1e-3) + 1e-6 * M;
    const double xt = sqrt((c * qc) / det);
    const double yt = -(qb * xt) / qc, ym = -yt;
    const bool th = yt >= ly && yt <= hy, tl = ym >= ly && ym <= hy;
    const double eh = yt < ly ? ly : hy, el = ym < ly ? ly : hy;
    const double Dh = qa * c - det * (eh * eh), Dl = qa * c - det * (el * el);
    if ((!th && Dh < 0.0) || (!tl && Dl < 0.0)) {
        ka = 1;
        kb = 0;
        return;
    }
    const double xh = th ? xt : (-(qb * eh) + sqrt(Dh)) / qa;
    const double xl = tl ? -xt : (-(qb * el) - sqrt(Dl)) / qa;
    // first a with box_hi(a) >= xl, last a with box_lo(a) <= xh: a guess
    // from the tile grid, then exact steps (the ends are monotone in a)
    // (tile widths are powers of two: the scaling by 1 / tw is exact)
    const double gl = fmin(fmax(ceil(ldexp(xl + mux + 0.5, -d.lg_tw) - 1.0), (double)a0), (double)(a1 + 1));
    const double gh = fmin(fmax(floor(ldexp(xh + mux - 0.5, -d.lg_tw)), (double)(a0 - 1)), (double)a1);
    ka = (int)gl;
    kb = (int)gh;
    while (ka > a0 && box_hi(d, ka - 1, mux) >= xl) --ka;
    while (ka <= a1 && box_hi(d, ka, mux) < xl) ++ka;
    while (kb < a1 && box_lo(d, kb + 1, mux) <= xh) ++kb;
    while (kb >= a0 && box_lo(d, kb, mux) > xh) --kb;
}

// Calls fn(emit, t, key) with the whole wave for every pair of the block
// (emit set on the lanes that hold one; key: the pair's sort key, depth bits
// and Gaussian index): Gaussian slot, tile t of the chunk (relative index)
// active, inside the Gaussian's rectangle and kept by the thinning rule.
// The projection lists each frame's visible Gaussians per group of 64
// (count and lane indices).  The block takes its groups in windows of 256;
// wave w of the block takes groups w, w + 4, ... of a window (neighbouring
// groups, often alike in visibility, go to different waves): one count per
// lane and a wave scan number its visible Gaussians, which the wave then
// takes 64 at a time, a lane finding its group by a binary search over the
// scan.  Groups with nothing visible cost a lane's count load.  The rectangles' tile rows (inside the chunk) of up
// to 64 such Gaussians are numbered by a scan and dealt to the lanes round
// robin, a lane finding the owning Gaussian by a binary search over the
// scan (only rows whose rectangle columns hold an active tile count); the
// lane then walks the active tiles of the row's kept run.
template <typename Fn>
__device__ __forceinline__ void block_pairs(const Dims& d, const WS& w, const Chunk& c, const uint32_t* act, Fn fn) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t ngb = (int64_t)(d.gpb >> 6);
    const int64_t gr0 = (int64_t)c.b * ngb, gr1 = min(gr0 + ngb, d.ngrp);
    const uint32_t* vc = w.vcnt + (int64_t)c.f * d.ngrp;
    const uint8_t* vl = w.vlist + (int64_t)c.f * d.ngrp * 64;
    const int ry0 = c.t0 / d.tx, ry1 = (c.t1 - 1) / d.tx;
    const int ct = c.t1 - c.t0;
    for (int64_t wb = gr0 + wv; wb < gr1; wb += 256) {
        const int64_t mine = wb + 4 * lane;
        const uint32_t cnt = mine < gr1 ? vc[mine] : 0u;
        const uint32_t ginc = wave_incl_scan(cnt, lane);
        const uint32_t V = (uint32_t)__shfl((int)ginc, 63);
        for (uint32_t v0 = 0; v0 < V; v0 += 64u) {
            const uint32_t idx = v0 + (uint32_t)lane;
            bool ok = idx < V;
            // group: the number of lanes whose inclusive count is <= idx
            int gs = 0;
#pragma unroll
            for (int st = 32; st > 0; st >>= 1)
                if ((uint32_t)__shfl((int)ginc, gs + st - 1) <= idx) gs += st;
            gs = min(gs, 63);
            const uint32_t gex = (uint32_t)__shfl((int)(ginc - cnt), gs);
            int64_t i = 0;
            if (ok) {
                const int64_t gr = wb + 4 * gs;
                i = gr * 64 + vl[gr * 64 + (idx - gex)];
            }
            int a0 = 0, a1 = -1, y0 = 0, y1 = -1;
            uint32_t slot = 0, zb = 0;
            Conic k = {0.f, 0.f, 0.f, 0.f, 0.f};
            if (ok) {
                slot = (uint32_t)((int64_t)c.f * d.N + i);
                tile_range(d, w.rect[slot], a0, a1, y0, y1);
                y0 = max(y0, ry0);
                y1 = min(y1, ry1);
                ok = y0 <= y1;
                const float4 r0 = w.rec[4ull * slot], r1 = w.rec[4ull * slot + 1];
                k = Conic{r0.x, r0.y, r0.z, r0.w, r1.x};
                zb = __float_as_uint(w.zkey[slot]);
            }
            // the rows whose rectangle columns hold an active tile of the
            // chunk (bit y - y0); a rectangle of more than 64 rows keeps
            // them all
            const bool tall = ok && y1 - y0 >= 64;
            uint64_t rows = 0ull;
            if (ok && !tall)
                for (int y = y0; y <= y1; ++y)
                    if (next_active(act, ct, y * d.tx - c.t0, a0, a1) <= a1) rows |= 1ull << (y - y0);
            const int n = tall ? y1 - y0 + 1 : __builtin_popcountll(rows);
            const int incl = wave_incl_scan(n, lane);
            const int excl = incl - n;
            const int total = __shfl(incl, 63);
            for (int q0 = 0; q0 < total; q0 += 64) {
                const int q = q0 + lane;
                // owner: the number of lanes whose inclusive count is <= q
                int s = 0;
#pragma unroll
                for (int st = 32; st > 0; st >>= 1)
                    if (__shfl(incl, s + st - 1) <= q) s += st;
                s = min(s, 63);
                const int kq = q - __shfl(excl, s);
                const uint64_t srows = ((uint64_t)(uint32_t)__shfl((int)(rows >> 32), s) << 32) |
                                       (uint64_t)(uint32_t)__shfl((int)(uint32_t)rows, s);
                const int y = __shfl(y0, s) + (__shfl((int)tall, s) ? kq : select_bit(srows, kq));
                const int sa0 = __shfl(a0, s), sa1 = __shfl(a1, s);
                const uint32_t sslot = (uint32_t)__shfl((int)slot, s);
                // sort key: camera z > z_near > 0, so the float bits order
                // like the values; ties broken by the Gaussian index
                const unsigned long long key = ((unsigned long long)(uint32_t)__shfl((int)zb, s) << 32) |
                                               (unsigned long long)(sslot - (uint32_t)((int64_t)c.f * d.N));
                const Conic sk = {__shfl(k.mux, s), __shfl(k.muy, s), __shfl(k.qa, s), __shfl(k.qb2, s),
                                  __shfl(k.qc, s)};
                const int rt = y * d.tx - c.t0;
                int ka = 1, kb = 0, x = 1;
                if (q < total) {
                    row_span(d, sk, sa0, sa1, y, ka, kb);
                    x = next_active(act, ct, rt, ka, kb);
                }
                // the active tiles of the lanes' kept runs, walked in step
                // by the whole wave
                for (; ballot(x <= kb) != 0; x = next_active(act, ct, rt, x + 1, kb)) fn(x <= kb, rt + x, key);
            }
        }
    }
}

// Staged pair: {key lo, key hi, index of its (frame, block, tile) count in
// hist, rank inside that group}.  A wave collects its pairs in an LDS
// buffer and, once 64 or more are held, claims room for them in its
// block's region with one atomic and copies them there; a claim that does
// not fit marks the block failed (what fits is still written, and skipped).
constexpr int kStageBuf = 128;

// LDS: [chunk] per-tile counters, then the active bits.
__global__ __launch_bounds__(256) void k_pair_hist(Dims d, WS w) {
    extern __shared__ uint32_t lds[];
    __shared__ uint4 sbuf[4][kStageBuf];
    __shared__ uint32_t sfail;
    const Chunk c = chunk_of_block(d);
    const int ct = c.t1 - c.t0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t* h = lds;
    uint32_t* act = lds + d.chunk;
    for (int t = threadIdx.x; t < ct; t += blockDim.x) h[t] = 0u;
    if (threadIdx.x == 0) sfail = 0u;
    load_active(d, w, c, act);
    __syncthreads();
    const uint32_t hbase = (uint32_t)(((int64_t)c.f * d.nbpf + c.b) * d.ntiles + c.t0);
    const uint32_t reg = blockIdx.x % (uint32_t)d.nreg;
    uint4* region = reinterpret_cast<uint4*>(w.prec) + (int64_t)reg * d.rcap;
    uint4* buf = sbuf[wv];
    uint32_t held = 0;   // wave-uniform
    bool failed = false;
    auto flush = [&]() {
        wave_lds_sync();
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&w.stagec[reg], held);
        base = (uint32_t)readfirstlane((int)base);
        const uint32_t room = base < d.rcap ? d.rcap - base : 0u;
        for (uint32_t k = (uint32_t)lane; k < held && k < room; k += 64) region[base + k] = buf[k];
        failed = failed || held > room;
        held = 0;
        wave_lds_sync();
    };
    block_pairs(d, w, c, act, [&](bool emit, int t, unsigned long long key) {
        const uint64_t m = ballot(emit);
        if (m == 0) return;
        if (emit) {
            const uint32_t r = atomicAdd(&h[t], 1u);
            buf[held + (uint32_t)__builtin_popcountll(m & below)] =
                make_uint4((uint32_t)key, (uint32_t)(key >> 32), hbase + (uint32_t)t, r);
        }
        held += (uint32_t)__builtin_popcountll(m);
        if (held > kStageBuf - 64) flush();
    });
    if (held) flush();
    if (failed && lane == 0) sfail = 1u;
    __syncthreads();
    uint32_t* out = w.hist + hbase;
    for (int t = threadIdx.x; t < ct; t += blockDim.x) out[t] = h[t];
    if (threadIdx.x == 0) w.bfail[blockIdx.x] = sfail;
}

// Per (frame, tile): exclusive scan of the block counts (in place) and the
// tile's pair count (into tile_end, turned into the end by k_tile_offsets).
// A 1024-thread workgroup takes kScanTiles tiles x kScanSeg segments of the
// block range: segment sums, their prefix in LDS, then the in-place scan of
// each segment.  With 64 tiles the lanes of a segment (one wave) read 256 B
// of a row; 16 tiles (four segments per wave, more workgroups and shorter
// segments) serve the problems with few tiles.  A segment of at most kB
// blocks keeps its counts in registers between the two passes.
constexpr int kScanThreads = 1024;
constexpr int64_t kScanWideFrom = 16384;   // (frame, tile)s for the 64-tile layout

template <int kScanTiles>
__global__ __launch_bounds__(kScanThreads) void k_hist_scan(Dims d, WS w) {
    constexpr int kScanSeg = kScanThreads / kScanTiles;
    __shared__ uint32_t part[kScanSeg][kScanTiles + 1];
    const int tl = threadIdx.x % kScanTiles, sg = threadIdx.x / kScanTiles;
    const int64_t ft = (int64_t)blockIdx.x * kScanTiles + tl;
    const bool ok = ft < (int64_t)d.F * d.ntiles;
    const int64_t f = ok ? ft / d.ntiles : 0, t = ok ? ft - f * d.ntiles : 0;
    const int per = (d.nbpf + kScanSeg - 1) / kScanSeg;
    const int b0 = min(sg * per, d.nbpf), b1 = ok ? min(b0 + per, d.nbpf) : b0;
    uint32_t* col = w.hist + f * d.nbpf * d.ntiles + t;
    constexpr int kB = 16;
    uint32_t sum = 0;
    uint32_t v[kB];
    for (int bb = b0; bb < b1; bb += kB) {
#pragma unroll
        for (int k = 0; k < kB; ++k) v[k] = bb + k < b1 ? col[(int64_t)(bb + k) * d.ntiles] : 0u;
#pragma unroll
        for (int k = 0; k < kB; ++k) sum += v[k];
    }
    part[sg][tl] = sum;
    __syncthreads();
    uint32_t acc = 0;
    for (int k = 0; k < sg; ++k) acc += part[k][tl];
    for (int bb = b0; bb < b1; bb += kB) {
        if (b1 - b0 > kB) {   // (one chunk: its counts are still in v)
#pragma unroll
            for (int k = 0; k < kB; ++k) v[k] = bb + k < b1 ? col[(int64_t)(bb + k) * d.ntiles] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            if (bb + k < b1) col[(int64_t)(bb + k) * d.ntiles] = acc;
            acc += v[k];
        }
    }
    if (ok && sg == kScanSeg - 1) w.tile_end[ft] = acc;
}

// Exclusive scan over a 1024-thread workgroup (wave scans, then a scan of
// the 16 wave totals); returns the exclusive prefix and the total.
template <typename T>
__device__ __forceinline__ T block_excl_scan_1024(T v, T* ws, T& total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    T inc = wave_incl_scan(v, lane);
    if (lane == 63) ws[wv] = inc;
    __syncthreads();
    if (wv == 0) {
        T t = lane < 16 ? ws[lane] : T(0);
        t = wave_incl_scan(t, lane);
        if (lane < 16) ws[lane] = t;
    }
    __syncthreads();
    total = ws[15];
    T ex = inc - v + (wv > 0 ? ws[wv - 1] : T(0));
    __syncthreads();
    return ex;
}

// Pair ranges [start, end) of every (frame, tile) from the counts, the
// total K and the capacity check (on overflow nothing is scattered, sorted
// or rendered); the work items (packs of up to 64 masked pixels) with the
// pixel and item totals; and the list of tiles whose lists exceed the
// per-tile LDS sort, longest first.  Tiles are taken in chunks of 4096, four
// consecutive ones per thread of a 1024-thread workgroup, so the loads and
// stores of a wave are contiguous.  Up to one chunk in all, one workgroup
// does everything (k_tile_offsets); beyond, the chunks run in parallel:
// their totals, one workgroup scanning them into per-chunk bases, the
// chunks' ranges and items, then the long-list order.
//
// Items go out longest list first, in eight classes of list length (>= 2048,
// >= 1024, ..., >= 32, shorter), frame and tile order inside a class: the
// compositing kernels hand items to their waves round robin, so the costly
// packs start first and the waves finish close together.
constexpr int kCls = 8;
// Cost class of a tile by its list length n: 0 for n >= 2048, one more per
// halving, 7 below 32 (and for empty lists).
__device__ __forceinline__ int cost_class(uint32_t n) {
    const int lg = n ? 31 - __builtin_clz(n) : 0;
    return min(max(11 - lg, 0), kCls - 1);
}
constexpr int kPkX = 13, kPkI = 42;   // bit offsets: long lists [0, 13), pixels [13, 42), items [42, 64)
constexpr unsigned long long kPkBMask = (1ull << kPkX) - 1ull, kPkXMask = (1ull << (kPkI - kPkX)) - 1ull;

// Four consecutive tiles of a chunk of 4096 per thread: pair counts,
// masked pixels and cost classes.
struct TileQuad {
    uint32_t v[4], q[4];
    int cls[4];
};

__device__ __forceinline__ void load_quad(const WS& w, int64_t e0, int64_t total, TileQuad& t) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        t.v[k] = e0 + k < total ? w.tile_end[e0 + k] : 0u;
        t.q[k] = e0 + k < total ? w.tile_npx[e0 + k] : 0u;
        t.cls[k] = cost_class(t.v[k]);
    }
}

// The chunk's exclusive scans and totals: pairs; items, pixels and long
// lists packed (a chunk of 4096 tiles, at most 4 packs and 256 pixels each,
// fits 15, 21 and 13 bits); the items of each class, 16 bits each, four
// classes per scan.
struct QuadScan {
    unsigned long long op, tp, oib, tib, oc0, tc0, oc1, tc1;
};

__device__ __forceinline__ QuadScan quad_scans(const TileQuad& t, uint32_t cap, unsigned long long* s64) {
    unsigned long long lp = 0, lc0 = 0, lc1 = 0;
    uint32_t li = 0, lx = 0, lb = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        lp += t.v[k];
        const uint32_t packs = (t.q[k] + 63) >> 6;
        li += packs;
        lx += t.q[k];
        lb += t.v[k] > cap ? 1u : 0u;
        const unsigned long long pk = (unsigned long long)packs << (16 * (t.cls[k] & 3));
        if (t.cls[k] < 4) lc0 += pk;
        else lc1 += pk;
    }
    QuadScan r;
    r.op = block_excl_scan_1024<unsigned long long>(lp, s64, r.tp);
    r.oib = block_excl_scan_1024<unsigned long long>(
        ((unsigned long long)li << kPkI) | ((unsigned long long)lx << kPkX) | lb, s64, r.tib);
    r.oc0 = block_excl_scan_1024<unsigned long long>(lc0, s64, r.tc0);
    r.oc1 = block_excl_scan_1024<unsigned long long>(lc1, s64, r.tc1);
    return r;
}

__device__ __forceinline__ uint32_t class_field(unsigned long long lo, unsigned long long hi, int c) {
    return (uint32_t)(((c < 4 ? lo : hi) >> (16 * (c & 3))) & 0xffffu);
}

// Pair ranges, long lists and work items of this thread's four tiles, given
// the chunk's pair base co, long-list base cb and per-class item bases.
__device__ __forceinline__ void emit_quad(const Dims& d, const WS& w, int64_t e0, int64_t total, const TileQuad& t,
                                          const QuadScan& s, unsigned long long co, const uint32_t* cbase,
                                          uint32_t cb, bool overflow) {
    const uint32_t cap = (uint32_t)d.sort_cap;
    unsigned long long o = co + s.op;
    uint32_t ob = cb + (uint32_t)(s.oib & kPkBMask);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t e = e0 + k;
        if (e < total) {
            const uint32_t st = overflow ? 0u : (uint32_t)o;
            w.tile_start[e] = st;
            w.tile_end[e] = overflow ? 0u : st + t.v[k];
            if (!overflow && t.v[k] > cap) w.bigl[ob++] = (uint32_t)e;
            const uint32_t packs = (t.q[k] + 63) >> 6;
            const int c = t.cls[k];
            uint32_t oi = cbase[c] + class_field(s.oc0, s.oc1, c);
#pragma unroll
            for (int j = 0; j < k; ++j)
                if (t.cls[j] == c) oi += (t.q[j] + 63) >> 6;
            for (uint32_t pk = 0; pk < packs; ++pk) w.items[oi + pk] = (uint32_t)e * (uint32_t)d.ppt + pk;
        }
        o += t.v[k];
    }
}

// The cb long lists (bigl, tile order) longest first into bigl2 (four size
// classes: > 4, > 2, > 1 run, rest), so the workgroups that take them early
// finish together.  One workgroup of 1024.
__device__ void order_big(const Dims& d, const WS& w, uint32_t cb, unsigned long long* s64) {
    const int tid = threadIdx.x;
    const uint32_t C = (uint32_t)d.big_chunk;
    uint32_t cnt[4] = {0u, 0u, 0u, 0u};
    for (uint32_t i = tid; i < cb; i += 1024) {
        const uint32_t e = w.bigl[i];
        const uint32_t n = w.tile_end[e] - w.tile_start[e];
        const int cl = n > 4 * C ? 0 : n > 2 * C ? 1 : n > C ? 2 : 3;
        cnt[cl] += 1u;
    }
    unsigned long long t01, t23;
    const unsigned long long o01 =
        block_excl_scan_1024<unsigned long long>(((unsigned long long)cnt[0] << 32) | cnt[1], s64, t01);
    const unsigned long long o23 =
        block_excl_scan_1024<unsigned long long>(((unsigned long long)cnt[2] << 32) | cnt[3], s64, t23);
    const uint32_t tot0 = (uint32_t)(t01 >> 32), tot1 = (uint32_t)t01, tot2 = (uint32_t)(t23 >> 32);
    uint32_t pos[4] = {(uint32_t)(o01 >> 32), tot0 + (uint32_t)o01, tot0 + tot1 + (uint32_t)(o23 >> 32),
                       tot0 + tot1 + tot2 + (uint32_t)o23};
    for (uint32_t i = tid; i < cb; i += 1024) {
        const uint32_t e = w.bigl[i];
        const uint32_t n = w.tile_end[e] - w.tile_start[e];
        const int cl = n > 4 * C ? 0 : n > 2 * C ? 1 : n > C ? 2 : 3;
        w.bigl2[pos[cl]++] = e;
    }
    // runs of C keys per long list, in bigl2 order: bigr[i] is the first
    // run-sort job of list i, bigr[cb] their number
    __syncthreads();
    const uint32_t per = (cb + 1023u) / 1024u;
    const uint32_t i0 = min(cb, (uint32_t)tid * per), i1 = min(cb, i0 + per);
    uint32_t nr = 0;
    for (uint32_t i = i0; i < i1; ++i) {
        const uint32_t e = w.bigl2[i];
        nr += (w.tile_end[e] - w.tile_start[e] + C - 1u) / C;
    }
    unsigned long long tot;
    uint32_t r = (uint32_t)block_excl_scan_1024<unsigned long long>(nr, s64, tot);
    for (uint32_t i = i0; i < i1; ++i) {
        const uint32_t e = w.bigl2[i];
        w.bigr[i] = r;
        r += (w.tile_end[e] - w.tile_start[e] + C - 1u) / C;
    }
    if (tid == 0) w.bigr[cb] = (uint32_t)tot;
}

__device__ __forceinline__ void write_header(const WS& w, unsigned long long K, bool overflow, uint32_t npx,
                                             uint32_t nitems, uint32_t nbig) {
    w.hdr->n_pairs = K > 0xffffffffull ? 0xffffffffu : (uint32_t)K;
    w.hdr->overflow = overflow ? 1u : 0u;
    w.hdr->n_px = npx;
    w.hdr->n_items = overflow ? 0u : nitems;
    w.hdr->n_big = nbig;
    w.hdr->q_big = 0u;
}

// Frames of at most 4096 tiles in all: one workgroup scans the single chunk
// and writes everything.
__global__ __launch_bounds__(1024) void k_tile_offsets(Dims d, WS w) {
    __shared__ unsigned long long s64[16];
    const int tid = threadIdx.x;
    const int64_t total = (int64_t)d.F * d.ntiles;
    const int64_t e0 = 4 * tid;
    TileQuad t;
    load_quad(w, e0, total, t);
    const QuadScan s = quad_scans(t, (uint32_t)d.sort_cap, s64);
    const unsigned long long K = s.tp;
    const bool overflow = K > (unsigned long long)d.max_pairs;
    uint32_t cbase[kCls], acc = 0;
#pragma unroll
    for (int c = 0; c < kCls; ++c) {
        cbase[c] = acc;
        acc += class_field(s.tc0, s.tc1, c);
    }
    emit_quad(d, w, e0, total, t, s, 0ull, cbase, 0u, overflow);
    const uint32_t nbig = overflow ? 0u : (uint32_t)(s.tib & kPkBMask);
    __syncthreads();
    if (nbig) order_big(d, w, nbig, s64);
    if (tid == 0)
        write_header(w, K, overflow, (uint32_t)((s.tib >> kPkX) & kPkXMask), (uint32_t)(s.tib >> kPkI), nbig);
}

// More tiles: chunks of 4096 in parallel.  1: each chunk's totals
// (workgroup per chunk) into chunk[16 c + 0..3].
__global__ __launch_bounds__(1024) void k_tile_chunk_sums(Dims d, WS w) {
    __shared__ unsigned long long s64[16];
    const int64_t total = (int64_t)d.F * d.ntiles;
    TileQuad t;
    load_quad(w, (int64_t)blockIdx.x * 4096 + 4 * threadIdx.x, total, t);
    const QuadScan s = quad_scans(t, (uint32_t)d.sort_cap, s64);
    if (threadIdx.x == 0) {
        unsigned long long* c = w.chunk + 16ull * blockIdx.x;
        c[0] = s.tp;
        c[1] = s.tib;
        c[2] = s.tc0;
        c[3] = s.tc1;
    }
}

// 2: one workgroup scans the chunk totals: per chunk its pair base
// (chunk[16 c + 4]), long-list base (+5) and item base per class (+6..13,
// classes in order, each class after all items of the classes before it);
// the total K decides the overflow; the header gets the totals.
__global__ __launch_bounds__(1024) void k_tile_chunk_scan(Dims d, WS w, int nchunk) {
    __shared__ unsigned long long s64[16];
    __shared__ unsigned long long ctot[kCls];
    const int tid = threadIdx.x;
    // pass 1: class totals (32-bit fields, two classes per word)
    unsigned long long l[kCls / 2] = {0ull, 0ull, 0ull, 0ull};
    for (int c = tid; c < nchunk; c += 1024) {
        const unsigned long long* ch = w.chunk + 16ull * c;
#pragma unroll
        for (int k = 0; k < kCls; ++k)
            l[k >> 1] += (unsigned long long)class_field(ch[2], ch[3], k) << (32 * (k & 1));
    }
#pragma unroll
    for (int h = 0; h < kCls / 2; ++h) {
        unsigned long long tt;
        (void)block_excl_scan_1024<unsigned long long>(l[h], s64, tt);
        if (tid == 0) {
            ctot[2 * h] = tt & 0xffffffffull;
            ctot[2 * h + 1] = tt >> 32;
        }
    }
    __syncthreads();
    unsigned long long cls_base[kCls], acc = 0;
#pragma unroll
    for (int k = 0; k < kCls; ++k) {
        cls_base[k] = acc;
        acc += ctot[k];
    }
    // the total K first: it decides the overflow before any range is written
    unsigned long long lk = 0;
    for (int c = tid; c < nchunk; c += 1024) lk += w.chunk[16ull * c];
    unsigned long long K;
    (void)block_excl_scan_1024<unsigned long long>(lk, s64, K);
    const bool overflow = K > (unsigned long long)d.max_pairs;
    // pass 2: per-chunk bases, 1024 chunks at a time
    unsigned long long cp = 0, cib = 0, cx = 0, ccl[kCls / 2] = {0ull, 0ull, 0ull, 0ull};
    for (int c0 = 0; c0 < nchunk; c0 += 1024) {
        const int c = c0 + tid;
        unsigned long long* ch = w.chunk + 16ull * (c < nchunk ? c : 0);
        const bool ok = c < nchunk;
        const unsigned long long tp = ok ? ch[0] : 0ull, tib = ok ? ch[1] : 0ull;
        const unsigned long long items = tib >> kPkI, big = overflow ? 0ull : (tib & kPkBMask);
        unsigned long long t1, t2, t3;
        const unsigned long long op = block_excl_scan_1024<unsigned long long>(tp, s64, t1);
        const unsigned long long oib = block_excl_scan_1024<unsigned long long>((items << 32) | big, s64, t2);
        const unsigned long long ox = block_excl_scan_1024<unsigned long long>((tib >> kPkX) & kPkXMask, s64, t3);
        (void)ox;
        unsigned long long oc[kCls / 2], tc[kCls / 2];
#pragma unroll
        for (int h = 0; h < kCls / 2; ++h) {
            const unsigned long long v = ok ? (((unsigned long long)class_field(ch[2], ch[3], 2 * h)) |
                                               ((unsigned long long)class_field(ch[2], ch[3], 2 * h + 1) << 32))
                                            : 0ull;
            oc[h] = block_excl_scan_1024<unsigned long long>(v, s64, tc[h]);
        }
        if (ok) {
            ch[4] = cp + op;
            ch[5] = (cib & 0xffffffffull) + (oib & 0xffffffffull);
#pragma unroll
            for (int k = 0; k < kCls; ++k) {
                const unsigned long long within = ((ccl[k >> 1] + oc[k >> 1]) >> (32 * (k & 1))) & 0xffffffffull;
                ch[6 + k] = cls_base[k] + within;
            }
        }
        cp += t1;
        cib += t2;
        cx += t3;
#pragma unroll
        for (int h = 0; h < kCls / 2; ++h) ccl[h] += tc[h];
    }
    if (tid == 0) write_header(w, K, overflow, (uint32_t)cx, (uint32_t)(cib >> 32), (uint32_t)(cib & 0xffffffffull));
}

// 3: each chunk's ranges, long lists and items from its bases.
__global__ __launch_bounds__(1024) void k_tile_chunk_emit(Dims d, WS w) {
    __shared__ unsigned long long s64[16];
    const int64_t total = (int64_t)d.F * d.ntiles;
    const int64_t e0 = (int64_t)blockIdx.x * 4096 + 4 * threadIdx.x;
    TileQuad t;
    load_quad(w, e0, total, t);
    const QuadScan s = quad_scans(t, (uint32_t)d.sort_cap, s64);
    const unsigned long long* ch = w.chunk + 16ull * blockIdx.x;
    uint32_t cbase[kCls];
#pragma unroll
    for (int k = 0; k < kCls; ++k) cbase[k] = (uint32_t)ch[6 + k];
    emit_quad(d, w, e0, total, t, s, ch[4], cbase, (uint32_t)ch[5], w.hdr->overflow != 0u);
}

// 4: the long lists longest first.
__global__ __launch_bounds__(1024) void k_tile_big_order(Dims d, WS w) {
    __shared__ unsigned long long s64[16];
    const uint32_t nbig = w.hdr->n_big;
    if (nbig) order_big(d, w, nbig, s64);
}

// Pairs to their places.  Workgroups [0, nbb) are the binning blocks:
// those whose staging overflowed enumerate their pairs again and write them
// through LDS cursors (tile start + the block's offset in the tile); the
// others return at once.  Workgroups from nbb on move the staged pairs,
// place_x per region (region = (g - nbb) / place_x): each to tile start +
// block offset + its rank.  LDS: [chunk] write cursors, then the active
// bits.
__global__ __launch_bounds__(256) void k_pair_scatter(Dims d, WS w, uint32_t nbb, uint32_t place_x) {
    extern __shared__ uint32_t lds[];
    if (blockIdx.x >= nbb) {
        if (w.hdr->overflow) return;
        const uint32_t g = blockIdx.x - nbb;
        const uint32_t reg = g / place_x, gx = g - reg * place_x;
        const uint32_t n = min(w.stagec[reg], d.rcap);
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4* region = reinterpret_cast<const u32x4*>(w.prec) + (int64_t)reg * d.rcap;
        const uint32_t nt = (uint32_t)d.ntiles, step = place_x * 256u;
        // four staged pairs per thread in flight: the loads of the pair, of
        // its tile start and of its block offset are each one level
        for (uint32_t e0 = gx * 256u + threadIdx.x; e0 < n; e0 += 4u * step) {
            u32x4 sv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) sv[u] = region[min(e0 + (uint32_t)u * step, n - 1u)];
            uint32_t base[4], off[4], fail[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t fb = sv[u].z / nt, tt = sv[u].z - fb * nt;
                fail[u] = w.bfail[fb * (uint32_t)d.nchunks + tt / (uint32_t)d.chunk];
                base[u] = w.tile_start[(int64_t)(fb / (uint32_t)d.nbpf) * nt + tt];
                off[u] = w.hist[sv[u].z];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (e0 + (uint32_t)u * step < n && !fail[u])
                    w.keys[base[u] + off[u] + sv[u].w] = ((unsigned long long)sv[u].y << 32) | sv[u].x;
        }
        return;
    }
    if (!w.bfail[blockIdx.x]) return;
    // the overflow flag is read with the cursors and checked before any
    // pair is written
    const uint32_t overflow = w.hdr->overflow;
    const Chunk c = chunk_of_block(d);
    const int ct = c.t1 - c.t0;
    uint32_t* cur = lds;
    uint32_t* act = lds + d.chunk;
    const uint32_t* off = w.hist + ((int64_t)c.f * d.nbpf + c.b) * d.ntiles + c.t0;
    const uint32_t* st = w.tile_start + (int64_t)c.f * d.ntiles + c.t0;
    for (int t = threadIdx.x; t < ct; t += blockDim.x) cur[t] = st[t] + off[t];
    load_active(d, w, c, act);
    __syncthreads();
    if (overflow) return;
    block_pairs(d, w, c, act, [&](bool emit, int t, unsigned long long key) {
        if (emit) {
            uint32_t pos = atomicAdd(&cur[t], 1u);
            w.keys[pos] = key;
        }
    });
}

// ---- per-tile order ---------------------------------------------------------


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

// Register-resident bitonic sort of P = 256 * 2^EB keys by a workgroup of
// 256 threads, thread t holding E = 2^EB of them.  In layout s a thread's
// registers hold the keys whose index bits s .. s+EB-1 are the register
// number (the other index bits are the thread's), so the compare-exchanges
// of a stride 2^b with s <= b < s+EB stay in registers.  A merge phase takes
// its strides from the top in windows of EB bits; moving to another layout
// goes through LDS (every key stored, then loaded), a fraction of the LDS
// traffic of one store-and-load step per stride.  LDS slots are swizzled
// (index bits 0-4 XOR bits 5-9), which spreads the contiguous layout's
// accesses over the banks.
__device__ __forceinline__ uint32_t rs_slot(uint32_t g) { return g ^ ((g >> 5) & 31u); }

template <int EB>
__device__ __forceinline__ uint32_t rs_index(uint32_t t, uint32_t m, int s) {
    return (t & ((1u << s) - 1u)) | (m << s) | ((t >> s) << (s + EB));
}

// The compare-exchanges of stride 2^(s+R) in layout s, merge phase k.
template <int EB, int R>
__device__ __forceinline__ void rs_step(unsigned long long (&a)[1 << EB], uint32_t t, int s, uint32_t k) {
    if constexpr (R < EB) {
#pragma unroll
        for (int m = 0; m < (1 << EB); ++m) {
            if (m & (1 << R)) continue;
            const int m2 = m | (1 << R);
            const bool asc = (rs_index<EB>(t, (uint32_t)m, s) & k) == 0u;
            const unsigned long long x = a[m], y = a[m2];
            const bool sw = (x > y) == asc;
            a[m] = sw ? y : x;
            a[m2] = sw ? x : y;
        }
    }
}

// The n <= P keys at kin (global), padded with the largest key, sorted into
// K[0..P) in plain order (ends with a workgroup barrier).
template <int EB>
__device__ void bitonic_regs(unsigned long long* K, const unsigned long long* kin, uint32_t n) {
    static_assert(EB >= 1 && EB <= 4, "2 to 16 keys per thread");
    constexpr int E = 1 << EB, pb = 8 + EB;
    const uint32_t t = threadIdx.x;
    unsigned long long a[E];
    int cur = pb - EB;   // key t + 256 m: coalesced loads
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const uint32_t g = t + 256u * (uint32_t)m;
        a[m] = g < n ? kin[g] : ~0ull;
    }
    for (int q = 1; q <= pb; ++q) {
        const uint32_t k = 1u << q;
        for (int b = q - 1; b >= 0;) {
            const int s = min((b / EB) * EB, pb - EB);
            if (s != cur) {
#pragma unroll
                for (int m = 0; m < E; ++m) K[rs_slot(rs_index<EB>(t, (uint32_t)m, cur))] = a[m];
                __syncthreads();
#pragma unroll
                for (int m = 0; m < E; ++m) a[m] = K[rs_slot(rs_index<EB>(t, (uint32_t)m, s))];
                __syncthreads();
                cur = s;
            }
            for (; b >= s; --b) {
                switch (b - s) {
                    case 0: rs_step<EB, 0>(a, t, s, k); break;
                    case 1: rs_step<EB, 1>(a, t, s, k); break;
                    case 2: rs_step<EB, 2>(a, t, s, k); break;
                    default: rs_step<EB, 3>(a, t, s, k); break;
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < E; ++m) K[rs_index<EB>(t, (uint32_t)m, cur)] = a[m];
    __syncthreads();
}

// The n keys at kin sorted into K[0..P) (P the power of two >= n, at most
// kSortLds) by a 256-thread workgroup: registers from 1024 keys on, LDS
// steps below.
__device__ __forceinline__ void sort_keys(unsigned long long* K, const unsigned long long* kin, uint32_t n) {
    static_assert(kSortLds == (256 << 4), "the register sort covers kSortLds keys");
    uint32_t P = 1;
    while (P < n) P <<= 1;
    if (P == 4096u) {
        bitonic_regs<4>(K, kin, n);
    } else if (P == 2048u) {
        bitonic_regs<3>(K, kin, n);
    } else if (P == 1024u) {
        bitonic_regs<2>(K, kin, n);
    } else {
        for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) K[i] = i < n ? kin[i] : ~0ull;
        __syncthreads();
        bitonic(K, P);
    }
}

// Order each tile's pairs by (depth bits, Gaussian index).  Lists of at
// most sort_cap pairs: one workgroup, LDS bitonic sort.  Longer lists go to
// k_tile_sort_big.  The sorted slot ids go back to `pairs`, and each pair's
// 64-byte record (the three hot float4 and {n^c, h}) is copied into `prec`
// in list order, so the compositing kernels stage records with one
// coalesced load level.
__device__ __forceinline__ void put_sorted(const WS& w, uint32_t pos, uint32_t slot) {
    w.pairs[pos] = slot;
    const float4* h = w.rec + 4ull * slot;
    // all four loads in flight before the first store
    const float4 a = h[0], b = h[1], c = h[2], e = h[3];
    float4* o = w.prec + 4ull * pos;
    o[0] = a;
    o[1] = b;
    o[2] = c;
    o[3] = e;
}

// The same for a sorted run held in LDS, K[0..n) to list positions
// start..start+n-1, four threads per record (one float4 each): every store
// instruction of a wave writes 16 whole records contiguously and every load
// gathers 16 whole 64-byte records.  Each thread gathers kCopyBatch float4
// before it stores any, so that many loads are in flight per wave (the
// copy is bound by gather latency, not bandwidth).
constexpr int kCopyBatch = 8;

// (a plain vector type: an array of HIP's float4 struct would live in
// scratch memory)
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void put_sorted_run(const WS& w, const unsigned long long* K, uint32_t start,
                                               uint32_t n, uint32_t fbase, uint32_t tid, uint32_t nthreads) {
    const uint32_t tot = 4u * n;
    const f32x4* src = reinterpret_cast<const f32x4*>(w.rec);
    f32x4* dst = reinterpret_cast<f32x4*>(w.prec);
    for (uint32_t e0 = tid; e0 < tot; e0 += kCopyBatch * nthreads) {
        f32x4 v[kCopyBatch];
        uint32_t slot[kCopyBatch];
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u) {
            // past the end: a duplicate load of the last element (never stored)
            const uint32_t e = min(e0 + (uint32_t)u * nthreads, tot - 1u);
            slot[u] = fbase + (uint32_t)(K[e >> 2] & 0xffffffffull);
            v[u] = src[4ull * slot[u] + (e & 3u)];
        }
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u) {
            const uint32_t e = e0 + (uint32_t)u * nthreads;
            if (e < tot) {
                dst[4ull * (start + (e >> 2)) + (e & 3u)] = v[u];
                if ((e & 3u) == 0u) w.pairs[start + (e >> 2)] = slot[u];
            }
        }
    }
}

// Lists of at most kWaveSort pairs: one wave, rank sort (every key counts
// the smaller keys of its list, read as LDS broadcasts; keys are unique, so
// ranks are the positions), in k_tile_sort_small.  k_tile_sort: one
// workgroup per (frame, tile), the longer lists up to sort_cap, whole
// workgroup, LDS bitonic sort.
constexpr int kWaveSort = 256;

// rk[r] += the number of keys K[0..n8) below kv[r], for the first NR rounds
// of a lane's keys; n8 is a multiple of 8.
template <int NR>
__device__ __forceinline__ void rank_count(const unsigned long long* K, uint32_t n8, const unsigned long long* kv,
                                           uint32_t* rk) {
    for (uint32_t j0 = 0; j0 < n8; j0 += 8u) {
        unsigned long long kj[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) kj[i] = K[j0 + i];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int r = 0; r < NR; ++r) rk[r] += (kj[i] < kv[r]) ? 1u : 0u;
    }
}

// One wave: the list of n <= kWaveSort keys at kin, sorted through the
// wave's LDS slice K (kWaveSort keys).
__device__ __forceinline__ void wave_sort_list(const WS& w, unsigned long long* K, const unsigned long long* kin,
                                               uint32_t start, uint32_t n, uint32_t fbase, int lane) {
    const int nr = (int)((n + 63) >> 6);
    unsigned long long kv[4];
    uint32_t rk[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t j = (uint32_t)(lane + 64 * r);
        kv[r] = (r < nr && j < n) ? kin[j] : ~0ull;
        if (r < nr) K[j] = kv[r];
        rk[r] = 0u;
    }
    wave_lds_sync();
    // K holds nr * 64 keys (the tail padded with the largest key, which
    // counts as smaller than none), so the count runs over whole batches of
    // eight keys, read before they are compared
    const uint32_t n8 = (n + 7u) & ~7u;
    switch (nr) {
        case 1: rank_count<1>(K, n8, kv, rk); break;
        case 2: rank_count<2>(K, n8, kv, rk); break;
        case 3: rank_count<3>(K, n8, kv, rk); break;
        default: rank_count<4>(K, n8, kv, rk); break;
    }
    if (n <= 64u) {   // one record per lane: a single round of copies
        if (lane < (int)n) put_sorted(w, start + rk[0], fbase + (uint32_t)(kv[0] & 0xffffffffull));
        return;
    }
    // every lane has read every key: the sorted run can replace them
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t j = (uint32_t)(lane + 64 * r);
        if (r < nr && j < n) K[rk[r]] = kv[r];
    }
    wave_lds_sync();
    put_sorted_run(w, K, start, n, fbase, (uint32_t)lane, 64u);
}

// Lists of at most kWaveSort (and sort_cap) pairs: one wave each, four
// (frame, tile)s per workgroup, each wave with its own 2 KB of LDS keys (so
// that many such workgroups share a CU).
__global__ __launch_bounds__(256) void k_tile_sort_small(Dims d, WS w, uint32_t nft) {
    __shared__ unsigned long long K[4][kWaveSort];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t ft = 4u * blockIdx.x + (uint32_t)wv;
    if (ft >= nft) return;
    const uint32_t start = w.tile_start[ft];
    const uint32_t n = w.tile_end[ft] - start;
    if (n == 0u || n > (uint32_t)kWaveSort || n > (uint32_t)d.sort_cap) return;
    wave_sort_list(w, K[wv], w.keys + start, start, n, (ft / (uint32_t)d.ntiles) * (uint32_t)d.N, lane);
}

// Run-sort jobs of the lists longer than sort_cap: the runs of big_chunk
// keys (job j of the table of order_big), each sorted by a 256-thread
// workgroup and written back in place for the merge rounds of
// k_tile_sort_big; a list of one run is finished here.  Workgroup `first`
// of `stride` takes jobs first, first + stride, ...
__device__ __forceinline__ void run_sort_jobs(const Dims& d, const WS& w, unsigned long long* K, uint32_t first,
                                              uint32_t stride) {
    // (on a capacity overflow every range is empty and no list is long)
    const uint32_t nbig = w.hdr->n_big;
    if (nbig == 0u) return;
    const uint32_t C = (uint32_t)d.big_chunk;
    const uint32_t J = w.bigr[nbig];
    for (uint32_t j = first; j < J; j += stride) {
        // the list of job j: the last i with bigr[i] <= j
        uint32_t lo = 0, hi = nbig - 1u;
        while (lo < hi) {
            const uint32_t m = (lo + hi + 1u) >> 1;
            if (w.bigr[m] <= j) lo = m;
            else hi = m - 1u;
        }
        const uint32_t ft = w.bigl2[lo];
        const uint32_t start = w.tile_start[ft];
        const uint32_t n = w.tile_end[ft] - start;
        const uint32_t r0 = (j - w.bigr[lo]) * C, len = min(C, n - r0);
        unsigned long long* run = w.keys + start + r0;
        sort_keys(K, run, len);
        if (n <= C) {
            put_sorted_run(w, K, start, n, (ft / (uint32_t)d.ntiles) * (uint32_t)d.N, threadIdx.x, blockDim.x);
        } else {
            for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) run[i] = K[i];
        }
        __syncthreads();
    }
}

// Workgroups below jgrid: run-sort jobs (when the jobs are not launched on
// their own); the others one (frame, tile) each, the lists of kWaveSort+1
// to sort_cap keys (the short lists are sorted by k_tile_sort_small, the
// longer ones by the jobs and k_tile_sort_big).
__global__ __launch_bounds__(256) void k_tile_sort(Dims d, WS w, uint32_t jgrid) {
    __shared__ unsigned long long K[kSortLds];
    if (blockIdx.x < jgrid) {
        run_sort_jobs(d, w, K, blockIdx.x, jgrid);
        return;
    }
    const uint32_t ft = blockIdx.x - jgrid;
    const uint32_t start = w.tile_start[ft];
    const uint32_t n = w.tile_end[ft] - start;
    if (n <= (uint32_t)kWaveSort || n > (uint32_t)d.sort_cap) return;
    const uint32_t fbase = (ft / (uint32_t)d.ntiles) * (uint32_t)d.N;
    sort_keys(K, w.keys + start, n);
    put_sorted_run(w, K, start, n, fbase, threadIdx.x, blockDim.x);
}

// The run-sort jobs on their own (beside the mid-length lists).
__global__ __launch_bounds__(256) void k_tile_sort_runs(Dims d, WS w) {
    __shared__ unsigned long long K[kSortLds];
    run_sort_jobs(d, w, K, blockIdx.x, gridDim.x);
}

// ---- lists longer than sort_cap ---------------------------------------------
//
// The runs of big_chunk keys of every long list were sorted in place by the
// run-sort workgroups of k_tile_sort_runs.  Here one 1024-thread workgroup per
// listed tile merges them pairwise (merge path: the co-ranks of an output
// window's ends are found by binary search, the window's inputs are staged
// in LDS, and every thread merges its share after its own co-rank search in
// LDS) until one run remains; the last round writes the sorted pairs and
// records.  Keys are unique, so the merge needs no tie rule.
constexpr int kBigLds = 8192;

// Smallest i in [max(0, k - lb), min(k, la)] with A[i] > B[k - i - 1]: the
// number of A elements among the first k merged outputs.
template <typename KA, typename KB>
__device__ __forceinline__ uint32_t co_rank(uint32_t k, KA A, uint32_t la, KB B, uint32_t lb) {
    uint32_t lo = k > lb ? k - lb : 0u, hi = k < la ? k : la;
    while (lo < hi) {
        uint32_t i = (lo + hi) >> 1;   // i < hi <= la and k - i - 1 < lb
        if (A[i] > B[k - i - 1]) hi = i;
        else lo = i + 1;
    }
    return lo;
}

// Tiles are taken from a queue (longest lists first).  Merge rounds work in
// output windows of up to kBigLds keys, which never straddle two runs being
// merged: the co-ranks of all window starts of a round are searched in
// parallel (one thread each), then each window's inputs are staged in LDS
// and merged by the whole workgroup.
__global__ __launch_bounds__(1024) void k_tile_sort_big(Dims d, WS w) {
    __shared__ unsigned long long L[kBigLds];
    __shared__ uint32_t cr[1024];
    __shared__ uint32_t s_it;
    if (w.hdr->overflow) return;
    const uint32_t nbig = w.hdr->n_big;
    if (nbig == 0) return;
    const uint32_t C = (uint32_t)d.big_chunk;
    // the first tile by block index, the rest from the queue
    for (uint32_t it = blockIdx.x; it < nbig;) {
        const uint32_t ft = w.bigl2[it];
        const uint32_t start = w.tile_start[ft];
        const uint32_t n = w.tile_end[ft] - start;
        const uint32_t fbase = (ft / (uint32_t)d.ntiles) * (uint32_t)d.N;
        unsigned long long* S0 = w.keys + start;
        unsigned long long* S1 = w.scratch + start;
        // pairwise merges: runs of width -> 2 width (a list of one run
        // was finished by its run sort)
        unsigned long long *src = S0, *dst = S1;
        for (uint32_t width = C; width < n; width <<= 1) {
            const bool last = 2 * width >= n;
            const uint32_t win = min((uint32_t)kBigLds, 2 * width);
            const uint32_t nwin = (n + win - 1) / win;
            for (uint32_t mb = 0; mb < nwin; mb += 1023) {
                const uint32_t me = min(mb + 1023u, nwin);
                for (uint32_t m = mb + threadIdx.x; m < me; m += blockDim.x) {
                    const uint32_t r0 = (m * win) / (2 * width) * (2 * width);
                    const uint32_t la = min(width, n - r0), lb = min(width, n - r0 - la);
                    cr[m - mb] = co_rank(m * win - r0, src + r0, la, src + r0 + la, lb);
                }
                __syncthreads();
                for (uint32_t m = mb; m < me; ++m) {
                    const uint32_t r0 = (m * win) / (2 * width) * (2 * width);
                    const uint32_t la = min(width, n - r0), lb = min(width, n - r0 - la);
                    const uint32_t k0 = m * win - r0, k1 = min(k0 + win, la + lb);
                    const uint32_t a0 = cr[m - mb];
                    const uint32_t a1 = (k1 == la + lb) ? la : (m + 1 < me ? cr[m + 1 - mb] : 0u);
                    // (a window that does not end its runs is never the last of a batch
                    // unless another batch follows; that case is handled below)
                    uint32_t a1f = a1;
                    if (k1 != la + lb && m + 1 == me)
                        a1f = co_rank(k1, src + r0, la, src + r0 + la, lb);
                    const uint32_t b0 = k0 - a0, b1 = k1 - a1f;
                    const uint32_t na = a1f - a0, nb = b1 - b0;
                    const unsigned long long* A = src + r0;
                    const unsigned long long* B = src + r0 + la;
                    for (uint32_t j = threadIdx.x; j < na; j += blockDim.x) L[j] = A[a0 + j];
                    for (uint32_t j = threadIdx.x; j < nb; j += blockDim.x) L[na + j] = B[b0 + j];
                    __syncthreads();
                    const uint32_t mm = k1 - k0;
                    const uint32_t per = (mm + blockDim.x - 1) / blockDim.x;
                    const uint32_t q0 = min(threadIdx.x * per, mm), q1 = min(q0 + per, mm);
                    if (q0 < q1) {
                        uint32_t ia = co_rank(q0, L, na, L + na, nb), ib = q0 - ia;
                        for (uint32_t q = q0; q < q1; ++q) {
                            const bool takeA = ib >= nb || (ia < na && L[ia] < L[na + ib]);
                            const unsigned long long v = takeA ? L[ia] : L[na + ib];
                            ia += takeA;
                            ib += !takeA;
                            dst[r0 + k0 + q] = v;
                        }
                    }
                    __syncthreads();
                    // the final pass: the merged window's records, copied
                    // four threads per record
                    if (last) put_sorted_run(w, dst + r0 + k0, start + r0 + k0, mm, fbase, threadIdx.x, blockDim.x);
                }
            }
            unsigned long long* t = src;
            src = dst;
            dst = t;
        }
        if (threadIdx.x == 0) s_it = gridDim.x + atomicAdd(&w.hdr->q_big, 1u);
        __syncthreads();
        it = s_it;
        __syncthreads();
    }
}

}  // namespace rtg
