// The steps of the mapping iteration either side of the backward (Sec. 3.2
// "Gaussian optimization", Eq. 8-9, and "Keyframes and global
// optimization"): the L2 regulariser of the transparent Gaussians, the
// confidence-weighted fusion of a window's result (Eq. 9), and the
// selection of a keyframe's pixels with the largest colour errors.
#include "rtg_common.h"

namespace rtg {

// L_reg = sum over transparent Gaussians of |p - p0|^2 + |q - q0|^2 +
// |s - s0|^2, weighted by w_reg: each workgroup (at most 1024, striding over
// the Gaussians) adds its binary64 partial sum of the weighted loss to
// loss_out[0] (one atomic per workgroup), and
// the gradient 2 w_reg (x - x0) goes onto the gradient rows of the unstable
// transparent Gaussians.
__global__ __launch_bounds__(256) void k_reg_l2(int64_t n, double w_reg, const uint8_t* __restrict__ transparent,
                                                const uint8_t* __restrict__ unstable,
                                                const float* __restrict__ pos, const float* __restrict__ scale,
                                                const float* __restrict__ rot, const float* __restrict__ pos0,
                                                const float* __restrict__ scale0, const float* __restrict__ rot0,
                                                float* __restrict__ d_pos, float* __restrict__ d_scale,
                                                float* __restrict__ d_rot, double* __restrict__ loss_out) {
    __shared__ double part[4];
    double l = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (!transparent[i]) continue;
        const bool un = unstable[i] != 0;
        auto term = [&](const float* x, const float* x0, float* g, int w) {
            for (int c = 0; c < w; ++c) {
                const double dx = (double)x[w * i + c] - (double)x0[w * i + c];
                l += dx * dx;
                if (un) g[w * i + c] += (float)(2.0 * w_reg * dx);
            }
        };
        term(pos, pos0, d_pos, 3);
        term(scale, scale0, d_scale, 3);
        term(rot, rot0, d_rot, 4);
    }
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = (part[0] + part[1]) + (part[2] + part[3]);
        if (t != 0.0) atomicAdd(loss_out, w_reg * t);
    }
}

// Eq. 9 per Gaussian: w = (eta' - eta_prev) / eta' (a binary32 division of
// the two counts; 1 when eta' = 0), G = fl32(fl32((1 - w) G_prev) +
// fl32(w G')) for every optimised value, written over G'.
__global__ __launch_bounds__(256) void k_fuse(int64_t n, int32_t ncol, const int32_t* __restrict__ eta_prev,
                                              const int32_t* __restrict__ eta_cur,
                                              const float* __restrict__ pos_prev,
                                              const float* __restrict__ scale_prev,
                                              const float* __restrict__ rot_prev,
                                              const float* __restrict__ col_prev, float* __restrict__ pos,
                                              float* __restrict__ scale, float* __restrict__ rot,
                                              float* __restrict__ col) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t ec = eta_cur[i];
    const float w = ec != 0 ? (float)(ec - eta_prev[i]) / (float)ec : 1.f;
    const float v = 1.f - w;
    auto mix = [&](const float* g0, float* g1, int64_t base, int cnt) {
        for (int c = 0; c < cnt; ++c) {
            const float a = v * g0[base + c];
            const float b = w * g1[base + c];
            g1[base + c] = a + b;
        }
    };
    mix(pos_prev, pos, 3 * i, 3);
    mix(scale_prev, scale, 3 * i, 3);
    mix(rot_prev, rot, 4 * i, 4);
    mix(col_prev, col, (int64_t)ncol * i, ncol);
}

// ---- top colour-error selection ---------------------------------------------
//
// Per frame: the colour error e = (|dC0| + |dC1|) + |dC2| of every pixel
// (binary32, as Eq. 6), its bits as an order-preserving key (e >= 0), and
// the k-th largest key found by four 8-bit radix passes (per-frame
// 256-bin histograms of the keys that share the prefix found so far, then
// one workgroup per frame picks the bin holding the k-th largest); the mask
// takes every pixel whose key is at least that value.

struct SelState {
    uint32_t prefix;   // high bits of the k-th largest key found so far
    uint32_t rem;      // its rank among the keys with that prefix (1-based)
    uint32_t none;     // k = 0: nothing selected
    uint32_t pad;
};

__global__ __launch_bounds__(256) void k_sel_keys(int64_t npx, const float* __restrict__ color_r,
                                                  const float* __restrict__ color_in, uint32_t* __restrict__ keys) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= npx) return;
    const float e0 = fabsf(color_r[3 * p] - color_in[3 * p]);
    const float e1 = fabsf(color_r[3 * p + 1] - color_in[3 * p + 1]);
    const float e2 = fabsf(color_r[3 * p + 2] - color_in[3 * p + 2]);
    keys[p] = __float_as_uint((e0 + e1) + e2);
}

__global__ __launch_bounds__(256) void k_sel_init(int32_t frames, uint32_t k, uint32_t* __restrict__ hist,
                                                  SelState* __restrict__ st) {
    const int f = blockIdx.x;
    if (f >= frames) return;
    hist[256 * f + threadIdx.x] = 0u;
    if (threadIdx.x == 0) st[f] = SelState{0u, k, k == 0u ? 1u : 0u, 0u};
}

// Grid (blocks per frame, frames).
__global__ __launch_bounds__(256) void k_sel_hist(int64_t hw, int shift, const uint32_t* __restrict__ keys,
                                                  uint32_t* __restrict__ hist, const SelState* __restrict__ st) {
    __shared__ uint32_t h[256];
    const int f = blockIdx.y;
    h[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t prefix = st[f].prefix;
    const uint32_t hi = shift + 8 < 32 ? (0xffffffffu << (shift + 8)) : 0u;
    const uint32_t* kf = keys + (int64_t)f * hw;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < hw; p += (int64_t)gridDim.x * 256) {
        const uint32_t key = kf[p];
        if ((key & hi) == (prefix & hi)) atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    if (c) atomicAdd(&hist[256 * f + threadIdx.x], c);
}

// One workgroup of 256 per frame: the bin b (counting from the top) whose
// keys hold the rem-th largest; prefix gains b, rem drops by the keys in
// higher bins; the histogram is cleared for the next pass.
__global__ __launch_bounds__(256) void k_sel_pick(int shift, uint32_t* __restrict__ hist, SelState* __restrict__ st) {
    __shared__ uint32_t suf[257];
    __shared__ SelState s;
    const int f = blockIdx.x;
    const int t = threadIdx.x;
    // suffix sums: suf[b] = keys in bins >= b
    const uint32_t c = hist[256 * f + t];
    suf[t] = c;
    if (t == 0) {
        suf[256] = 0u;
        s = st[f];
    }
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t add = t + o < 256 ? suf[t + o] : 0u;
        __syncthreads();
        suf[t] += add;
        __syncthreads();
    }
    // the bin with suf[b + 1] < rem <= suf[b] (exactly one when rem <= suf[0])
    if (!s.none && suf[t + 1] < s.rem && s.rem <= suf[t]) {
        st[f].prefix = s.prefix | ((uint32_t)t << shift);
        st[f].rem = s.rem - suf[t + 1];
    }
    hist[256 * f + t] = 0u;
}

__global__ __launch_bounds__(256) void k_sel_mask(int64_t hw, int32_t frames, const uint32_t* __restrict__ keys,
                                                  const SelState* __restrict__ st, uint8_t* __restrict__ mask) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= hw * frames) return;
    const SelState s = st[p / hw];
    mask[p] = (!s.none && keys[p] >= s.prefix) ? 1 : 0;
}

}  // namespace rtg
