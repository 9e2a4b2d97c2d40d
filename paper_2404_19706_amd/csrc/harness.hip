// Steps a6 and a10: the L1 loss of Eq. 7-8 with its upstream gradients,
// and Adam on the unstable rows (supp. Sec. C learning rates).  Both walk
// only what the iteration touches: the rendered pixel lists and the rows of
// unstable Gaussians.
#include "rtg_common.h"

namespace rtg {

__global__ void k_fill_u8(uint8_t* p, size_t n, uint8_t v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// Status of the calls on a workspace as an rtg_status value, written on the
// device (for callers that do not synchronise to read the header).
__global__ void k_status_out(WS w, int32_t* out) {
    if (threadIdx.x == 0) *out = w.hdr->overflow ? -2 : (w.hdr->err ? -5 : 0);
}

// Sums of the per-wave work counters of the last render and backward
// launches, and the count of the last binning's blocks that fell back to a
// second enumeration (nbb blocks), into the header (one workgroup; no
// host-side reduction).
__global__ __launch_bounds__(1024) void k_sum_counters(WS w, uint32_t nbb) {
    __shared__ unsigned long long part[4][16];
    __shared__ uint32_t nfail[16];
    const uint32_t nw[2] = {min(w.hdr->fwd_waves, (uint32_t)kMaxWaves), min(w.hdr->bwd_waves, (uint32_t)kMaxWaves)};
    for (int c = 0; c < 4; ++c) {
        unsigned long long v = 0;
        for (uint32_t k = threadIdx.x; k < nw[c / 2]; k += blockDim.x) v += w.wcount[(size_t)c * kMaxWaves + k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & 63) == 0) part[c][threadIdx.x >> 6] = v;
    }
    {
        uint32_t v = 0;
        for (uint32_t k = threadIdx.x; k < nbb; k += blockDim.x) v += w.bfail[k] ? 1u : 0u;
        for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o);
        if ((threadIdx.x & 63) == 0) nfail[threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long t = 0;
        for (int k = 0; k < 16; ++k) t += part[threadIdx.x][k];
        w.hdr->sums[threadIdx.x] = t;
    }
    if (threadIdx.x == 4) {
        uint32_t t = 0;
        for (int k = 0; k < 16; ++k) t += nfail[k];
        w.hdr->n_restaged = t;
    }
}

__device__ __forceinline__ bool pixel_of_rank(const Dims& d, const WS& w, int64_t idx, int& f, size_t& pix) {
    int64_t ft = idx / d.tarea;
    uint32_t r = (uint32_t)(idx - ft * d.tarea);
    if (ft >= (int64_t)d.F * d.ntiles) return false;
    if (r >= w.tile_npx[ft]) return false;
    int l = w.pix[idx];
    f = (int)(ft / d.ntiles);
    int t = (int)(ft % d.ntiles);
    int px = (t % d.tx) * d.tw + (l & (d.tw - 1));
    int py = (t / d.tx) * d.th + (l >> d.lg_tw);
    pix = ((size_t)f * d.H + py) * d.W + px;
    return true;
}

// Per-block partial sums of |C - C*| over the rendered pixels, |D - D*| and
// the count over pixels with a hit and a valid target (no shared-address
// atomics: one partial triple per block).
__global__ __launch_bounds__(256) void k_loss_partials(Dims d, WS w, const float* __restrict__ C,
                                                       const float* __restrict__ D,
                                                       const float* __restrict__ Cgt,
                                                       const float* __restrict__ Dgt, float* __restrict__ part) {
    __shared__ float red[3][4];
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int f;
    size_t pix;
    float sc = 0.f, sd = 0.f, nd = 0.f;
    if (pixel_of_rank(d, w, idx, f, pix)) {
        sc = fabsf(C[3 * pix] - Cgt[3 * pix]) + fabsf(C[3 * pix + 1] - Cgt[3 * pix + 1]) +
             fabsf(C[3 * pix + 2] - Cgt[3 * pix + 2]);
        if (D[pix] != -1.f && Dgt[pix] > 0.f) {
            sd = fabsf(D[pix] - Dgt[pix]);
            nd = 1.f;
        }
    }
    sc = wave_sum(sc);
    sd = wave_sum(sd);
    nd = wave_sum(nd);
    int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wv] = sc;
        red[1][wv] = sd;
        red[2][wv] = nd;
    }
    __syncthreads();
    if (threadIdx.x < 3)
        part[3 * blockIdx.x + threadIdx.x] =
            (red[threadIdx.x][0] + red[threadIdx.x][1]) + (red[threadIdx.x][2] + red[threadIdx.x][3]);
}

// One workgroup: totals of the partials, the loss value.
__global__ __launch_bounds__(1024) void k_loss_final(WS w, const float* __restrict__ part, uint32_t nparts,
                                                     float w_c, float w_d, float* __restrict__ loss_out) {
    __shared__ float red[3][16];
    float a = 0.f, b = 0.f, c = 0.f;
    for (uint32_t k = threadIdx.x; k < nparts; k += 1024) {
        a += part[3 * k];
        b += part[3 * k + 1];
        c += part[3 * k + 2];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wv] = a;
        red[1][wv] = b;
        red[2][wv] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float ta = 0.f, tb = 0.f, tc = 0.f;
        for (int q = 0; q < 16; ++q) {
            ta += red[0][q];
            tb += red[1][q];
            tc += red[2][q];
        }
        uint32_t nmd = (uint32_t)tc;
        w.hdr->loss_c = ta;
        w.hdr->loss_d = tb;
        w.hdr->cnt_md = nmd;
        float nm = (float)max(w.hdr->n_px, 1u);
        loss_out[0] = w_c * ta / (3.f * nm) + w_d * tb / (float)max(nmd, 1u);
    }
}

__global__ __launch_bounds__(256) void k_loss_grad(Dims d, WS w, const float* __restrict__ C,
                                                   const float* __restrict__ D,
                                                   const float* __restrict__ Cgt,
                                                   const float* __restrict__ Dgt, float w_c, float w_d,
                                                   float* __restrict__ gC, float* __restrict__ gD) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int f;
    size_t pix;
    if (!pixel_of_rank(d, w, idx, f, pix)) return;
    float nm = (float)max(w.hdr->n_px, 1u);
    float nmd = (float)max(w.hdr->cnt_md, 1u);
    float kc = w_c / (3.f * nm);
    for (int c = 0; c < 3; ++c) gC[3 * pix + c] = kc * sgn(C[3 * pix + c] - Cgt[3 * pix + c]);
    gD[pix] = (D[pix] != -1.f && Dgt[pix] > 0.f) ? (w_d / nmd) * sgn(D[pix] - Dgt[pix]) : 0.f;
}

__global__ void k_step_inc(int32_t* step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) step[0] += 1;
}

struct AdamArgs {
    float lr_pos, lr_scale, lr_rot, lr_col, lr_rest, b1, b2, eps;
    int32_t K;   // colour parameters per channel: 1 (RGB) or (D+1)^2 (SH)
};

__global__ __launch_bounds__(256) void k_adam(int64_t N, float* __restrict__ pos, float* __restrict__ scale,
                                              float* __restrict__ rot, float* __restrict__ col,
                                              const uint8_t* __restrict__ unstable,
                                              const float* __restrict__ gpos, const float* __restrict__ gscale,
                                              const float* __restrict__ grot, const float* __restrict__ gcol,
                                              float* __restrict__ m, float* __restrict__ v,
                                              const int32_t* __restrict__ step, AdamArgs a) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || !unstable[i]) return;
    float t = (float)step[0];
    float bc1 = 1.f - powf(a.b1, t), bc2 = 1.f - powf(a.b2, t);
    const int64_t stride = 10 + 3 * (int64_t)a.K;
    float* mi = m + stride * i;
    float* vi = v + stride * i;
    auto upd = [&](int k, float g) {
        float mk = a.b1 * mi[k] + (1.f - a.b1) * g;
        float vk = a.b2 * vi[k] + (1.f - a.b2) * g * g;
        mi[k] = mk;
        vi[k] = vk;
        return (mk / bc1) / (sqrtf(vk / bc2) + a.eps);
    };
    for (int c = 0; c < 3; ++c) pos[3 * i + c] -= a.lr_pos * upd(c, gpos[3 * i + c]);
    for (int c = 0; c < 3; ++c) {
        float s = scale[3 * i + c];
        scale[3 * i + c] = s * __expf(-a.lr_scale * upd(3 + c, s * gscale[3 * i + c]));
    }
    for (int c = 0; c < 4; ++c) rot[4 * i + c] -= a.lr_rot * upd(6 + c, grot[4 * i + c]);
    const int64_t cb = 3 * (int64_t)a.K * i;
    for (int c = 0; c < 3 * a.K; ++c) col[cb + c] -= (c < 3 ? a.lr_col : a.lr_rest) * upd(10 + c, gcol[cb + c]);
}

}  // namespace rtg
