// Gaussian adding (Sec. 3.2 "Gaussians adding", Eq. 6) and state management
// (Sec. 3.2, end of "Gaussian optimization" and "State management"): the
// data-parallel steps either side of the optimisation, consumers of the
// render's colour, depth, transmission and index images.
//
// Adding, three passes over the frame's pixels (no shared-address
// atomics): mark (per pixel: the Eq. 6 mask, whether the pixel is sampled
// and adds a Gaussian; per 256-pixel block: how many), scan (one workgroup:
// block offsets and the total), emit (per adding pixel: its row, in raster
// order after the existing Gaussians, and the new disc).  Threshold
// decisions follow a fixed binary32 sequence, vertices and normals are
// formed in binary64 from the binary32 depth with a fixed sequence, so
// which pixels add a Gaussian, and in which order, is reproducible bit for
// bit by an independent implementation of the same rules.
#include "rtg_common.h"

namespace rtg {

struct AddParams {
    float delta_T, delta_d, delta_c, rate;
    float alpha_opaque, alpha_transparent, r_transparent, thickness;
    int32_t delta_eta, delta_e, delta_t;
    int32_t sh_degree;
};

struct Intr {
    double fx, fy, cx, cy;
    int32_t W, H;
};

// Eq. 6 on one pixel: 1 = M_s (light passes, T > delta_T, or the depth
// misses by more than delta_d), 2 = M_c (geometry right, colour L1 error
// summed over the channels above 3 delta_c), 0 = neither or invalid input
// depth (D <= 0).
__device__ __forceinline__ int add_mask(const AddParams& a, const float* cr, float dr, float tr, const float* ci,
                                        float di) {
    if (!(di > 0.f)) return 0;
    if (tr > a.delta_T || fabsf(dr - di) > a.delta_d) return 1;
    const float ec = (fabsf(cr[0] - ci[0]) + fabsf(cr[1] - ci[1])) + fabsf(cr[2] - ci[2]);
    return ec > 3.f * a.delta_c ? 2 : 0;
}

// Camera-frame vertex of pixel (x, y) at depth D (binary64).
__device__ __forceinline__ void vertex(const Intr& c, int x, int y, float D, double v[3]) {
    const double Dd = (double)D;
    v[0] = Dd * ((((double)x + 0.5) - c.cx) / c.fx);
    v[1] = Dd * ((((double)y + 0.5) - c.cy) / c.fy);
    v[2] = Dd;
}

// Unit normal at (x, y) from the forward differences to the right and lower
// neighbours (their cross product), turned towards the camera; false on the
// last row or column, with an invalid neighbour or a degenerate product.
__device__ __forceinline__ bool normal_at(const Intr& c, const float* __restrict__ depth, int x, int y, double n[3]) {
    if (x + 1 >= c.W || y + 1 >= c.H) return false;
    const float d0 = depth[(size_t)y * c.W + x], d1 = depth[(size_t)y * c.W + x + 1],
                d2 = depth[(size_t)(y + 1) * c.W + x];
    if (!(d0 > 0.f) || !(d1 > 0.f) || !(d2 > 0.f)) return false;
    double v0[3], v1[3], v2[3];
    vertex(c, x, y, d0, v0);
    vertex(c, x + 1, y, d1, v1);
    vertex(c, x, y + 1, d2, v2);
    const double a0 = v1[0] - v0[0], a1 = v1[1] - v0[1], a2 = v1[2] - v0[2];
    const double b0 = v2[0] - v0[0], b1 = v2[1] - v0[1], b2 = v2[2] - v0[2];
    n[0] = a1 * b2 - a2 * b1;
    n[1] = a2 * b0 - a0 * b2;
    n[2] = a0 * b1 - a1 * b0;
    const double l = sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
    if (!(l > 0.0)) return false;
    n[0] /= l;
    n[1] /= l;
    n[2] /= l;
    if ((n[0] * v0[0] + n[1] * v0[1]) + n[2] * v0[2] > 0.0) {
        n[0] = -n[0];
        n[1] = -n[1];
        n[2] = -n[2];
    }
    return true;
}

// Adding decision of one pixel: 0 none, 1 opaque disc (sampled M_s pixel),
// 2 transparent disc (sampled M_c pixel whose depth-hit Gaussian is stable);
// both need a normal.
__device__ __forceinline__ int add_code(const AddParams& a, const Intr& c, int x, int y,
                                        const float* __restrict__ color_in, const float* __restrict__ depth_in,
                                        const float* __restrict__ color_r, const float* __restrict__ depth_r,
                                        const float* __restrict__ trans_r, const int32_t* __restrict__ index_r,
                                        const float* __restrict__ rnd, const uint8_t* __restrict__ unstable,
                                        int64_t n_cur, int& mask) {
    const size_t p = (size_t)y * c.W + x;
    mask = add_mask(a, color_r + 3 * p, depth_r[p], trans_r[p], color_in + 3 * p, depth_in[p]);
    if (mask == 0 || !(rnd[p] < a.rate)) return 0;
    if (mask == 2) {
        const int32_t j = index_r[p];
        if (j < 0 || (int64_t)j >= n_cur || unstable[j] != 0) return 0;
    }
    double n[3];
    if (!normal_at(c, depth_in, x, y, n)) return 0;
    return mask;
}

// Pass 1: codes and per-block counts (block = 256 consecutive pixels).
__global__ __launch_bounds__(256) void k_add_mark(AddParams a, Intr c, const float* __restrict__ color_in,
                                                  const float* __restrict__ depth_in,
                                                  const float* __restrict__ color_r,
                                                  const float* __restrict__ depth_r,
                                                  const float* __restrict__ trans_r,
                                                  const int32_t* __restrict__ index_r,
                                                  const float* __restrict__ rnd,
                                                  const uint8_t* __restrict__ unstable, int64_t n_cur,
                                                  uint8_t* __restrict__ codes, uint8_t* __restrict__ mask_out,
                                                  uint32_t* __restrict__ counts) {
    __shared__ uint32_t wc[4];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t np = (int64_t)c.W * c.H;
    int code = 0, mask = 0;
    if (p < np) {
        code = add_code(a, c, (int)(p % c.W), (int)(p / c.W), color_in, depth_in, color_r, depth_r, trans_r, index_r,
                        rnd, unstable, n_cur, mask);
        codes[p] = (uint8_t)code;
        if (mask_out) mask_out[p] = (uint8_t)mask;
    }
    const uint32_t n = (uint32_t)__builtin_popcountll(ballot(code != 0));
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = (wc[0] + wc[1]) + (wc[2] + wc[3]);
}

// Exclusive scan of nb block counts by one 1024-thread workgroup (chunks of
// 1024 with a carry); the total goes to *total.
__global__ __launch_bounds__(1024) void k_scan_counts(const uint32_t* __restrict__ counts,
                                                      uint32_t* __restrict__ offsets, uint32_t nb,
                                                      unsigned long long* __restrict__ total) {
    __shared__ unsigned long long s64[16];
    unsigned long long carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
        const uint32_t b = b0 + threadIdx.x;
        const unsigned long long v = b < nb ? counts[b] : 0ull;
        unsigned long long t;
        const unsigned long long ex = block_excl_scan_1024<unsigned long long>(v, s64, t);
        if (b < nb) offsets[b] = (uint32_t)(carry + ex);
        carry += t;
    }
    if (threadIdx.x == 0) *total = carry;
}

// Unit quaternion (w, x, y, z) of the shortest rotation taking e_z to n (a
// half-turn about x when n = -e_z).
__device__ __forceinline__ void quat_z_to(const double n[3], float q[4]) {
    double w = 1.0 + n[2], x = -n[1], y = n[0], z = 0.0;
    if (w < 1e-12) {
        w = 0.0;
        x = 1.0;
        y = 0.0;
    }
    const double l = sqrt(((w * w + x * x) + y * y) + z * z);
    q[0] = (float)(w / l);
    q[1] = (float)(x / l);
    q[2] = (float)(y / l);
    q[3] = (float)(z / l);
}

// Pass 3: every adding pixel writes its disc at row n_cur + rank (rank =
// block offset + its rank in the block, raster order), while rows remain.
__global__ __launch_bounds__(256) void k_add_emit(AddParams a, Intr c, const double* __restrict__ pose,
                                                  const float* __restrict__ color_in,
                                                  const float* __restrict__ depth_in,
                                                  const uint8_t* __restrict__ codes,
                                                  const uint32_t* __restrict__ offsets, int32_t frame_k,
                                                  int64_t n_cur, int64_t capacity, float* __restrict__ pos,
                                                  float* __restrict__ scale, float* __restrict__ rot,
                                                  float* __restrict__ opacity, float* __restrict__ color,
                                                  uint8_t* __restrict__ unstable, int32_t* __restrict__ eta,
                                                  int32_t* __restrict__ err, int32_t* __restrict__ tstamp) {
    __shared__ uint32_t wc[4];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t np = (int64_t)c.W * c.H;
    const int code = p < np ? (int)codes[p] : 0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t m = ballot(code != 0);
    if (lane == 0) wc[wv] = (uint32_t)__builtin_popcountll(m);
    __syncthreads();
    if (code == 0) return;
    uint32_t r = offsets[blockIdx.x] + (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1ull));
    for (int k = 0; k < wv; ++k) r += wc[k];
    const int64_t row = n_cur + (int64_t)r;
    if (row >= capacity) return;
    const int x = (int)(p % c.W), y = (int)(p / c.W);
    const float D = depth_in[p];
    double v[3], n[3];
    vertex(c, x, y, D, v);
    normal_at(c, depth_in, x, y, n);
    const double* R = pose;
    const double* t = pose + 9;
    double nw[3];
    for (int i = 0; i < 3; ++i) {
        pos[3 * row + i] = (float)(((R[3 * i] * v[0] + R[3 * i + 1] * v[1]) + R[3 * i + 2] * v[2]) + t[i]);
        nw[i] = (R[3 * i] * n[0] + R[3 * i + 1] * n[1]) + R[3 * i + 2] * n[2];
    }
    const double f = 0.5 * (c.fx + c.fy);
    double rad = sqrt(1.0 / (3.141592653589793 * (double)a.rate)) * (double)D / f;
    if (code == 2) rad = fmin(rad, (double)a.r_transparent);
    scale[3 * row] = (float)rad;
    scale[3 * row + 1] = (float)rad;
    scale[3 * row + 2] = (float)((double)a.thickness * rad);
    float q[4];
    quat_z_to(nw, q);
    for (int i = 0; i < 4; ++i) rot[4 * row + i] = q[i];
    opacity[row] = code == 2 ? a.alpha_transparent : a.alpha_opaque;
    if (a.sh_degree == 0) {
        for (int i = 0; i < 3; ++i) color[3 * row + i] = color_in[3 * p + i];
    } else {
        // SH: the band-0 coefficient gives the pixel's colour in every
        // direction (Y_00 = 1 / (2 sqrt(pi))), the higher bands start at zero
        const int K3 = 3 * (a.sh_degree + 1) * (a.sh_degree + 1);
        float* cr = color + (int64_t)K3 * row;
        for (int i = 0; i < 3; ++i) cr[i] = (float)((double)color_in[3 * p + i] / 0.28209479177387814);
        for (int i = 3; i < K3; ++i) cr[i] = 0.f;
    }
    unstable[row] = 1;
    eta[row] = 0;
    err[row] = 0;
    tstamp[row] = frame_k;
}

// Confidence count: eta + 1 for every unstable Gaussian whose colour
// gradient row is non-zero (its colour was updated this step).
__global__ __launch_bounds__(256) void k_confidence(int64_t n, int32_t width, const uint8_t* __restrict__ unstable,
                                                    const float* __restrict__ d_color, int32_t* __restrict__ eta) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n || unstable[i] == 0) return;
    const float* g = d_color + (int64_t)width * i;
    bool any = false;
    for (int k = 0; k < width; ++k) any = any || g[k] != 0.f;
    if (any) eta[i] += 1;
}

// State management, pass 1 (per pixel): a pixel with valid input depth and
// a colour error (as in Eq. 6) or a depth error (hit pixels only) flags the
// stable Gaussian its index map names.  Every writer stores 1, so the
// order of the stores does not matter.
__global__ __launch_bounds__(256) void k_state_flag(AddParams a, Intr c, const float* __restrict__ color_in,
                                                    const float* __restrict__ depth_in,
                                                    const float* __restrict__ color_r,
                                                    const float* __restrict__ depth_r,
                                                    const int32_t* __restrict__ index_r, int64_t n,
                                                    const uint8_t* __restrict__ unstable,
                                                    uint8_t* __restrict__ flag) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)c.W * c.H) return;
    const float di = depth_in[p];
    if (!(di > 0.f)) return;
    const float dr = depth_r[p];
    const float* cr = color_r + 3 * p;
    const float* ci = color_in + 3 * p;
    const float ec = (fabsf(cr[0] - ci[0]) + fabsf(cr[1] - ci[1])) + fabsf(cr[2] - ci[2]);
    const bool bad = ec > 3.f * a.delta_c || (dr != -1.f && fabsf(dr - di) > a.delta_d);
    const int32_t j = index_r[p];
    if (bad && j >= 0 && (int64_t)j < n && unstable[j] == 0) flag[j] = 1;
}

// State management, pass 2 (per Gaussian): error count, stable -> unstable
// (e > delta_e; e, eta reset, timestamp k), unstable -> stable
// (eta > delta_eta), removal of unstable Gaussians older than delta_t.
__global__ __launch_bounds__(256) void k_state_apply(AddParams a, int64_t n, int32_t frame_k,
                                                     const uint8_t* __restrict__ flag,
                                                     uint8_t* __restrict__ unstable, int32_t* __restrict__ eta,
                                                     int32_t* __restrict__ err, int32_t* __restrict__ tstamp,
                                                     uint8_t* __restrict__ keep) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int32_t e = err[i] + (flag[i] ? 1 : 0);
    const bool was_unstable = unstable[i] != 0;
    uint8_t k = 1;
    if (!was_unstable) {
        if (e > a.delta_e) {
            unstable[i] = 1;
            e = 0;
            eta[i] = 0;
            tstamp[i] = frame_k;
        }
    } else if (eta[i] > a.delta_eta) {
        unstable[i] = 0;
    } else if (frame_k - tstamp[i] > a.delta_t) {
        k = 0;
    }
    err[i] = e;
    keep[i] = k;
}

// Stable compaction of up to kCompactMax row arrays by a keep mask: counts
// per 256-row block, a scan, then every kept row copies its bytes to its
// rank.
constexpr int kCompactMax = 16;
struct CompactArrays {
    const uint8_t* src[kCompactMax];
    uint8_t* dst[kCompactMax];
    int32_t rb[kCompactMax];
    int32_t n;
};

__global__ __launch_bounds__(256) void k_compact_count(int64_t n, const uint8_t* __restrict__ keep,
                                                       uint32_t* __restrict__ counts) {
    __shared__ uint32_t wc[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool k = i < n && keep[i] != 0;
    const uint32_t c = (uint32_t)__builtin_popcountll(ballot(k));
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = (wc[0] + wc[1]) + (wc[2] + wc[3]);
}

__global__ __launch_bounds__(256) void k_compact_move(int64_t n, const uint8_t* __restrict__ keep,
                                                      const uint32_t* __restrict__ offsets, CompactArrays A) {
    __shared__ uint32_t wc[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool k = i < n && keep[i] != 0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t m = ballot(k);
    if (lane == 0) wc[wv] = (uint32_t)__builtin_popcountll(m);
    __syncthreads();
    if (!k) return;
    int64_t r = (int64_t)offsets[blockIdx.x] + (int64_t)__builtin_popcountll(m & ((1ull << lane) - 1ull));
    for (int w = 0; w < wv; ++w) r += wc[w];
    for (int a = 0; a < A.n; ++a) {
        const int rb = A.rb[a];
        const uint8_t* s = A.src[a] + (size_t)i * rb;
        uint8_t* d = A.dst[a] + (size_t)r * rb;
        if ((rb & 3) == 0) {
            for (int b = 0; b < rb; b += 4)
                *reinterpret_cast<uint32_t*>(d + b) = *reinterpret_cast<const uint32_t*>(s + b);
        } else {
            for (int b = 0; b < rb; ++b) d[b] = s[b];
        }
    }
}

}  // namespace rtg
