// Step a1 (projection), step a8 (projection backward) and the M_unstable
// helper.  One thread per Gaussian walks all frames of the batch, so the
// Gaussian's parameters are read from HBM once per call whatever the number
// of keyframes.
//
// The decision quantities (cull, centre, conic, depth key, tau, normal,
// rectangle) follow one fixed binary64 operation sequence with no
// contraction (the library is built with -ffp-contract=off), each result
// rounded once to binary32; this makes every discrete decision reproducible
// bit for bit by an independent implementation of the same sequence.
#include "rtg_common.h"
#include "sh.h"

namespace rtg {

// Rotation of a raw quaternion (w, x, y, z): R = I + (2/|q|^2) M(q), which
// equals the rotation of q/|q| (Sec. 3.1 parameterises Sigma by s and q).
__device__ __forceinline__ bool quat_rot(float qw, float qx, float qy, float qz, double R[9]) {
    double w = qw, x = qx, y = qy, z = qz;
    double n2 = ((w * w + x * x) + y * y) + z * z;
    if (!(n2 > 0.0) || !isfinite(n2)) return false;
    double k = 2.0 / n2;
    R[0] = 1.0 - k * (y * y + z * z);
    R[1] = k * (x * y - w * z);
    R[2] = k * (x * z + w * y);
    R[3] = k * (x * y + w * z);
    R[4] = 1.0 - k * (x * x + z * z);
    R[5] = k * (y * z - w * x);
    R[6] = k * (x * z - w * y);
    R[7] = k * (y * z + w * x);
    R[8] = 1.0 - k * (x * x + y * y);
    return true;
}

// Inclusive pixel range [lo, hi] on one axis holding every pixel centre
// with (centre - mu)^2 <= r2, plus one pixel of slack, clipped to [0, n-1].
// E = ceil(sqrt(r2)) is settled by exact integer squares, so the result
// does not depend on the rounding of the square root.
__device__ __forceinline__ bool axis_range(double mu, double r2, int n, int& lo, int& hi) {
    if (!(r2 >= 0.0)) return false;
    if (r2 > 4096.0 * 4096.0) {
        lo = 0;
        hi = n - 1;
        return true;
    }
    double e = ceil(sqrt(r2));
    while (e > 0.0 && (e - 1.0) * (e - 1.0) >= r2) e -= 1.0;
    while (e * e < r2) e += 1.0;
    double c = floor(mu);
    double a = c - e - 2.0, b = c + e + 1.0;
    if (a > (double)(n - 1) || b < 0.0) return false;
    if (a < 0.0) a = 0.0;
    if (b > (double)(n - 1)) b = (double)(n - 1);
    lo = (int)a;
    hi = (int)b;
    return true;
}

// Frame-independent data of one Gaussian, shared through LDS by the lanes
// of its wave.
// Entry (a, b) of a symmetric 3x3 matrix stored as its upper triangle
// {xx, xy, xz, yy, yz, zz}.
__device__ constexpr int sym3(int a, int b) {
    return a <= b ? (a == 0 ? b : a == 1 ? 2 + b : 5) : (b == 0 ? a : b == 1 ? 2 + a : 5);
}

struct GaussShared {
    double S[6];       // Sigma_3D = R diag(s^2) R^T, upper triangle (sym3)
    double n0, n1, n2; // surfel normal: column of R of the smallest scale
    float p0, p1, p2;
    float alpha, tau, c0, c1, c2;
    uint32_t gidw;     // index | unstable bit
    uint32_t mask;     // frames that passed the off-image pre-cull
};

// Off-image pre-cull of one (Gaussian, frame) slot with camera-frame centre
// (x, y, z), z > z_near: true when its rectangle is certainly empty, so the
// projection chain would cull it too.  With a = x/z, b = y/z,
// ||J row 0||^2 = fx^2 (1 + a^2) / z^2 bounds Sigma_xx / lambda_max(Sigma_3D)
// (W is a rotation), likewise for y; the condition number of Sigma_2D is at
// most kappa(Sigma_3D) tr(J J^T)^2 / det(J J^T), and while that stays below
// 2.5e5 the rectangle's cut-off c_r = rho^2 / (1 - t) has t < 0.48
// (t <= 1.91e-6 kappa), so c_r < 2 rho^2 and the half-width
// E <= sqrt(2 rho^2 Sigma) + 1.  The slot is culled when its centre lies
// beyond that half-width plus three pixels of slack outside the image.
__device__ __forceinline__ bool precull(const Dims& d, double x, double y, double z, double smax2, double kap3) {
    // one hardware reciprocal (and square roots below): the slack dwarfs
    // their error
    const double iz = __builtin_amdgcn_rcp(z);
    const double ia = x * iz, ib = y * iz;
    const double fx2 = d.fx * d.fx, fy2 = d.fy * d.fy;
    const double ja = fx2 * (1.0 + ia * ia), jb = fy2 * (1.0 + ib * ib);
    const double trj = ja + jb, detj = fx2 * fy2 * (1.0 + ia * ia + ib * ib);
    if (!(kap3 * (trj * trj) < 2.5e5 * detj)) return false;
    const double z2i = iz * iz, c2 = 2.0 * (double)d.cutoff2, eps = (double)d.dilation;
    const double ex2 = c2 * ((ja * z2i) * smax2 + eps) * (1.0 + 1e-6);
    const double ey2 = c2 * ((jb * z2i) * smax2 + eps) * (1.0 + 1e-6);
    if (ex2 < 4096.0 * 4096.0) {
        const double mux = d.fx * ia + d.cx, e = __builtin_amdgcn_sqrt(ex2) + 4.0;
        if (mux - e > (double)d.W || mux + e < 0.0) return true;
    }
    if (ey2 < 4096.0 * 4096.0) {
        const double muy = d.fy * ib + d.cy, e = __builtin_amdgcn_sqrt(ey2) + 4.0;
        if (muy - e > (double)d.H || muy + e < 0.0) return true;
    }
    return false;
}

// The projection chain of one slot (fixed binary64 sequence, see the file
// head): returns whether the slot is visible and, if so, writes its record,
// depth key, rectangle (and clears its gradient accumulator when unstable).
__device__ bool project_slot(const Dims& d, const WS& w, const GaussShared& g, const double* __restrict__ poses,
                             int f, int64_t i) {
    const double* Rg = poses + 12 * f;
    const double* tg = Rg + 9;
    const double* S = g.S;
    const double n0 = g.n0, n1 = g.n1, n2 = g.n2;
    const float alpha = g.alpha, tau = g.tau, c0 = g.c0, c1 = g.c1, c2 = g.c2;
    const uint32_t gidw = g.gidw;
    const double eps = (double)d.dilation;
    const double c2cut = (double)d.cutoff2;
    double v0 = (double)g.p0 - tg[0], v1 = (double)g.p1 - tg[1], v2 = (double)g.p2 - tg[2];
    double x = (Rg[0] * v0 + Rg[3] * v1) + Rg[6] * v2;
    double y = (Rg[1] * v0 + Rg[4] * v1) + Rg[7] * v2;
    double z = (Rg[2] * v0 + Rg[5] * v1) + Rg[8] * v2;
    if (!(z > (double)d.z_near)) return false;
    double J00 = d.fx / z, J02 = -((d.fx * x) / (z * z));
    double J11 = d.fy / z, J12 = -((d.fy * y) / (z * z));
    double M[6];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        M[kk] = J00 * Rg[kk * 3 + 0] + J02 * Rg[kk * 3 + 2];
        M[3 + kk] = J11 * Rg[kk * 3 + 1] + J12 * Rg[kk * 3 + 2];
    }
    double T[6];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
            T[a * 3 + kk] = (M[a * 3 + 0] * S[sym3(0, kk)] + M[a * 3 + 1] * S[sym3(1, kk)]) +
                            M[a * 3 + 2] * S[sym3(2, kk)];
    double sxx = ((T[0] * M[0] + T[1] * M[1]) + T[2] * M[2]) + eps;
    double sxy = (T[0] * M[3] + T[1] * M[4]) + T[2] * M[5];
    double syy = ((T[3] * M[3] + T[4] * M[4]) + T[5] * M[5]) + eps;
    double det = sxx * syy - sxy * sxy;
    if (!(det > 0.0)) return false;
    double qa = syy / det, qb = -(sxy / det), qc = sxx / det;
    double mux = (d.fx * x) / z + d.cx;
    double muy = (d.fy * y) / z + d.cy;
    if (!(fabs(mux) < 16777216.0) || !(fabs(muy) < 16777216.0)) return false;
    // rectangle cut-off rho^2 / (1 - t), t = 16 * 2^-24 * K * lmax
    // (whole image when t >= 1/2): K = max(Q.xx, Q.yy) + |Q.xy|
    // bounds the form's term magnitudes per unit squared offset and
    // lmax, the largest eigenvalue of Sigma_2D, the squared offset
    // per unit of q, so every pixel the binary32 decision admits
    // (evaluation and entry rounding, at most 8 * 2^-24 times the
    // term magnitudes) lies inside
    const double Kq = fmax(qa, qc) + fabs(qb);
    const double hh = 0.5 * (sxx - syy);
    const double lmax = 0.5 * (sxx + syy) + sqrt(hh * hh + sxy * sxy);
    const double tq = 9.5367431640625e-07 * (Kq * lmax);
    const double crect = tq < 0.5 ? c2cut / (1.0 - tq) : INFINITY;
    int x0, x1, y0, y1;
    if (!axis_range(mux, crect * sxx, d.W, x0, x1)) return false;
    if (!axis_range(muy, crect * syy, d.H, y0, y1)) return false;
    double nc0 = (Rg[0] * n0 + Rg[3] * n1) + Rg[6] * n2;
    double nc1 = (Rg[1] * n0 + Rg[4] * n1) + Rg[7] * n2;
    double nc2 = (Rg[2] * n0 + Rg[5] * n1) + Rg[8] * n2;
    double h = (x * nc0 + y * nc1) + z * nc2;
    int64_t slot = (int64_t)f * d.N + i;
    // precise slot: lambda_max / lambda_min of Sigma_2D above
    // kPreciseKappa (lambda_min = det / lambda_max); its value path
    // reads the factored conic (Q = U^T U, U.xx = sqrt(Q.xx),
    // U.yy = 1 / sqrt(Sigma.yy), r = Q.xy / Q.xx as two floats) and
    // the binary32 centre residual
    const bool precise = lmax > kPreciseKappa * (det / lmax);
    float mux32 = (float)mux, muy32 = (float)muy;
    uint32_t gw = gidw;
    if (precise) {
        gw |= kPreciseBit;
        const double r = qb / qa;
        const float rhi = (float)r;
        float* rp = w.recp + 6 * slot;
        rp[0] = rhi;
        rp[1] = (float)(r - (double)rhi);
        rp[2] = (float)sqrt(qa);
        rp[3] = (float)(1.0 / sqrt(syy));
        rp[4] = (float)(mux - (double)mux32);
        rp[5] = (float)(muy - (double)muy32);
    }
    float qb32 = (float)qb;
    float lo = pack_mu_lo((float)(mux - (double)mux32), (float)(muy - (double)muy32));
    float4* rc = w.rec + 4 * slot;
    rc[0] = make_float4(mux32, muy32, (float)qa, 2.0f * qb32);
    rc[1] = make_float4((float)qc, alpha, tau, c0);
    rc[2] = make_float4(c1, c2, __uint_as_float(gw), lo);
    rc[3] = make_float4((float)nc0, (float)nc1, (float)nc2, (float)h);
    w.zkey[slot] = (float)z;
    w.rect[slot] = make_short4((short)x0, (short)x1, (short)y0, (short)y1);
    if (gidw & kUnstableBit) {
        float4* ga = reinterpret_cast<float4*>(w.grad + 16 * slot);
        float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
        ga[0] = zero;
        ga[1] = zero;
        ga[2] = zero;
        ga[3] = zero;
    }
    return true;
}

// One thread per Gaussian prepares its frame-independent data and tests
// every frame with the off-image pre-cull; the wave then spreads the
// surviving (Gaussian, frame) slots over its 64 lanes (an exclusive scan of
// the per-lane counts and a search for the owner lane), so the binary64
// chain runs on about as many slots as are visible rather than once per
// frame in every wave where any lane needs it.
__global__ __launch_bounds__(256) void k_project(Dims d, WS w, const float* __restrict__ pos,
                                                 const float* __restrict__ scale,
                                                 const float* __restrict__ rot,
                                                 const float* __restrict__ opac,
                                                 const float* __restrict__ col,
                                                 const uint8_t* __restrict__ unstable,
                                                 const double* __restrict__ poses) {
    __shared__ GaussShared gs[256];
    __shared__ uint32_t visl[256];
    __shared__ uint32_t pre[4][65];
    if (blockIdx.x == 0 && threadIdx.x < sizeof(Hdr) / 4) reinterpret_cast<uint32_t*>(w.hdr)[threadIdx.x] = 0u;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    GaussShared& g = gs[threadIdx.x];
    uint32_t mask = 0;
    if (i < d.N) {
        float s0 = scale[3 * i], s1 = scale[3 * i + 1], s2f = scale[3 * i + 2];
        float q0 = rot[4 * i], q1 = rot[4 * i + 1], q2 = rot[4 * i + 2], q3 = rot[4 * i + 3];
        double R[9];
        if (quat_rot(q0, q1, q2, q3, R)) {
            g.p0 = pos[3 * i];
            g.p1 = pos[3 * i + 1];
            g.p2 = pos[3 * i + 2];
            g.alpha = opac[i];
            // RGB colours; with SH the colour is formed per frame by
            // k_sh_color
            g.c0 = d.sh_deg ? 0.f : col[3 * i];
            g.c1 = d.sh_deg ? 0.f : col[3 * i + 1];
            g.c2 = d.sh_deg ? 0.f : col[3 * i + 2];
            g.gidw = (uint32_t)i | (unstable[i] ? kUnstableBit : 0u);
            // Sigma_3D = R diag(s^2) R^T (frame independent)
            double sq[3] = {(double)s0 * (double)s0, (double)s1 * (double)s1, (double)s2f * (double)s2f};
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = a; b < 3; ++b) {
                    double v = ((R[a * 3 + 0] * sq[0]) * R[b * 3 + 0] + (R[a * 3 + 1] * sq[1]) * R[b * 3 + 1]) +
                               (R[a * 3 + 2] * sq[2]) * R[b * 3 + 2];
                    g.S[sym3(a, b)] = v;
                }
            // surfel normal: column of R of the smallest scale, lowest index on ties
            int k = 0;
            float sk = s0;
            if (s1 < sk) { k = 1; sk = s1; }
            if (s2f < sk) k = 2;
            g.n0 = R[0 * 3 + k];
            g.n1 = R[1 * 3 + k];
            g.n2 = R[2 * 3 + k];
            double a64 = (double)g.alpha;
            g.tau = (a64 > 0.0) ? (float)(1.0 + 2.0 * log(a64)) : -INFINITY;
            // frames that may see it: in front of the near plane and not
            // certainly off-image
            const double smax2 = fmax(fmax(sq[0], sq[1]), sq[2]);
            const double smin2 = fmin(fmin(sq[0], sq[1]), sq[2]);
            const double kap3 = smin2 > 0.0 ? smax2 / smin2 : INFINITY;
            const double p0 = g.p0, p1 = g.p1, p2 = g.p2;
            for (int f = 0; f < d.F; ++f) {
                const double* Rg = poses + 12 * f;
                const double* tg = Rg + 9;
                double v0 = p0 - tg[0], v1 = p1 - tg[1], v2 = p2 - tg[2];
                double z = (Rg[2] * v0 + Rg[5] * v1) + Rg[8] * v2;
                if (!(z > (double)d.z_near)) continue;
                double x = (Rg[0] * v0 + Rg[3] * v1) + Rg[6] * v2;
                double y = (Rg[1] * v0 + Rg[4] * v1) + Rg[7] * v2;
                if (precull(d, x, y, z, smax2, kap3)) continue;
                mask |= 1u << f;
            }
        }
    }
    g.mask = mask;
    visl[threadIdx.x] = 0u;
    // exclusive scan of the per-lane slot counts over the wave
    uint32_t incl = (uint32_t)__builtin_popcount(mask);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += t;
    }
    pre[wv][lane + 1] = incl;
    if (lane == 0) pre[wv][0] = 0u;
    const uint32_t total = (uint32_t)__shfl((int)incl, 63);
    wave_lds_sync();
    for (uint32_t base = 0; base < total; base += 64) {
        const uint32_t item = base + (uint32_t)lane;
        if (item < total) {
            // owner lane: the last one whose exclusive prefix is <= item
            int lo = 0, hi = 64;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pre[wv][mid] <= item) lo = mid;
                else hi = mid;
            }
            const GaussShared& go = gs[wv * 64 + lo];
            uint32_t m = go.mask;
            for (uint32_t r = item - pre[wv][lo]; r > 0; --r) m &= m - 1u;
            const int f = __builtin_ctz(m);
            const int64_t io = (int64_t)blockIdx.x * blockDim.x + wv * 64 + lo;
            if (project_slot(d, w, go, poses, f, io)) atomicOr(&visl[wv * 64 + lo], 1u << f);
        }
    }
    wave_lds_sync();
    const uint32_t vb = visl[threadIdx.x];
    if (i < d.N) w.vis[i] = vb;
    // per frame: this wave's visible Gaussians (a group of 64) for binning
    const int64_t grp = (int64_t)blockIdx.x * 4 + wv;
    if (grp < d.ngrp) {
        const uint64_t below = (1ull << lane) - 1ull;
        for (int f = 0; f < d.F; ++f) {
            const bool v = (vb >> f) & 1u;
            const uint64_t m = ballot(v);
            const int64_t gf = (int64_t)f * d.ngrp + grp;
            if (v) w.vlist[gf * 64 + __builtin_popcountll(m & below)] = (uint8_t)lane;
            if (lane == 0) w.vcnt[gf] = (uint32_t)__builtin_popcountll(m);
        }
    }
}

// M_unstable (supp. B): one wave per Gaussian; lanes stride over the pixel
// rectangle of each frame in which the unstable Gaussian is visible and set
// the mask where the decision d^2 is within the cut-off.
__global__ __launch_bounds__(256) void k_unstable_mask(Dims d, WS w, uint8_t* __restrict__ mask) {
    int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (i >= d.N) return;
    uint32_t vis = w.vis[i];
    while (vis) {
        int f = __builtin_ctz(vis);
        vis &= vis - 1;
        int64_t slot = (int64_t)f * d.N + i;
        float4 h2 = w.rec[4 * slot + 2];
        if (!rec_unstable(h2)) return;
        float4 h0 = w.rec[4 * slot + 0];
        float4 h1 = w.rec[4 * slot + 1];
        short4 r = w.rect[slot];
        int rw = r.y - r.x + 1;
        int n = rw * (r.w - r.z + 1);
        uint8_t* m = mask + (size_t)f * d.W * d.H;
        for (int p = lane; p < n; p += 64) {
            int px = r.x + p % rw, py = r.z + p / rw;
            float dd = dd_decision(h0.x, h0.y, h0.z, h0.w, h1.x, (float)px + 0.5f, (float)py + 0.5f);
            if (dd <= d.cutoff2) m[(size_t)py * d.W + px] = 1;
        }
    }
}

// Step a8: chain rule from the per-slot camera-space gradients to the
// parameters of each unstable Gaussian, summed over the frames that see it
// (binary64).  Rows of stable Gaussians are left untouched; unstable rows
// are always written (zero when no frame sees the Gaussian).  The slot
// accumulators are cleared as they are consumed.
__device__ void project_bwd_one(const Dims& d, const WS& w, int64_t i, const float* __restrict__ pos,
                                const float* __restrict__ scale, const float* __restrict__ rot,
                                const double* __restrict__ poses, float* __restrict__ d_pos,
                                float* __restrict__ d_scale, float* __restrict__ d_rot, float* __restrict__ d_opac,
                                float* __restrict__ d_col, float kc, float kd) {
    double gp[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, ga = 0, gc[3] = {0, 0, 0};
    uint32_t vis = w.vis[i];
    if (vis) {
        double s[3] = {scale[3 * i], scale[3 * i + 1], scale[3 * i + 2]};
        float qf[4] = {rot[4 * i], rot[4 * i + 1], rot[4 * i + 2], rot[4 * i + 3]};
        double R[9];
        quat_rot(qf[0], qf[1], qf[2], qf[3], R);
        double sq[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
        double S[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                S[a * 3 + b] = R[a * 3 + 0] * sq[0] * R[b * 3 + 0] + R[a * 3 + 1] * sq[1] * R[b * 3 + 1] +
                               R[a * 3 + 2] * sq[2] * R[b * 3 + 2];
        int k = 0;
        if ((float)s[1] < (float)s[k]) k = 1;
        if ((float)s[2] < (float)s[k]) k = 2;
        double dR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        double G3s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // dL/dSigma3D summed over frames
        double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        while (vis) {
            int f = __builtin_ctz(vis);
            vis &= vis - 1;
            int64_t slot = (int64_t)f * d.N + i;
            float4* g4 = reinterpret_cast<float4*>(w.grad + 16 * slot);
            float4 ga0 = g4[0], ga1 = g4[1], ga2 = g4[2], ga3 = g4[3];
            // upstream scales of the colour slots (0-8) and depth slots (9-13)
            ga0.x *= kc; ga0.y *= kc; ga0.z *= kc; ga0.w *= kc;
            ga1.x *= kc; ga1.y *= kc; ga1.z *= kc; ga1.w *= kc;
            ga2.x *= kc; ga2.y *= kd; ga2.z *= kd; ga2.w *= kd;
            ga3.x *= kd; ga3.y *= kd;
            // consume the accumulator: a later backward on the same
            // projection starts from zero again
            const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
            g4[0] = zero;
            g4[1] = zero;
            g4[2] = zero;
            g4[3] = zero;
            // [dmu.x, dmu.y, dQxx, dQxy, | dQyy, dalpha, dc.r, dc.g, | dc.b, a, b.x, b.y, | b.z, e, -, -]
            const double* Rg = poses + 12 * f;
            const double* tg = Rg + 9;
            double v[3] = {p[0] - tg[0], p[1] - tg[1], p[2] - tg[2]};
            double x = Rg[0] * v[0] + Rg[3] * v[1] + Rg[6] * v[2];
            double y = Rg[1] * v[0] + Rg[4] * v[1] + Rg[7] * v[2];
            double z = Rg[2] * v[0] + Rg[5] * v[1] + Rg[8] * v[2];
            double fx = d.fx, fy = d.fy;
            double J00 = fx / z, J02 = -fx * x / (z * z), J11 = fy / z, J12 = -fy * y / (z * z);
            double M[6];
            for (int kk = 0; kk < 3; ++kk) {
                M[kk] = J00 * Rg[kk * 3 + 0] + J02 * Rg[kk * 3 + 2];
                M[3 + kk] = J11 * Rg[kk * 3 + 1] + J12 * Rg[kk * 3 + 2];
            }
            // Sigma_2D and its inverse Q (as in the forward, incl. dilation)
            double T[6];
            for (int a = 0; a < 2; ++a)
                for (int kk = 0; kk < 3; ++kk)
                    T[a * 3 + kk] = M[a * 3] * S[kk] + M[a * 3 + 1] * S[3 + kk] + M[a * 3 + 2] * S[6 + kk];
            double sxx = T[0] * M[0] + T[1] * M[1] + T[2] * M[2] + d.dilation;
            double sxy = T[0] * M[3] + T[1] * M[4] + T[2] * M[5];
            double syy = T[3] * M[3] + T[4] * M[4] + T[5] * M[5] + d.dilation;
            double det = sxx * syy - sxy * sxy;
            double Qa = syy / det, Qb = -sxy / det, Qc = sxx / det;
            double GS00, GS01, GS11, dmx, dmy;
            if (rec_precise(w.rec[4 * slot + 2])) {
                // precise slot: slots 0-4 hold m = sum g e and M = sum g e e^T
                // (off-diagonal twice) of the whitened offsets e = U (u - mu),
                // Q = U^T U (U upper triangular, U.xx = sqrt(Q.xx)); then
                // dL/dmu = -2 U^T m and dL/dSigma2D = -U^T M U
                const double u00 = sqrt(Qa), u01 = Qb / u00, u11 = 1.0 / sqrt(syy);
                const double m0 = ga0.x, m1 = ga0.y;
                const double M00 = ga0.z, M01 = 0.5 * (double)ga0.w, M11 = ga1.x;
                dmx = -2.0 * (u00 * m0);
                dmy = -2.0 * (u01 * m0 + u11 * m1);
                const double MU01 = M00 * u01 + M01 * u11, MU11 = M01 * u01 + M11 * u11;
                GS00 = -(u00 * (M00 * u00));
                GS01 = -(u00 * MU01);
                GS11 = -(u01 * MU01 + u11 * MU11);
            } else {
                // dL/dQ (symmetric matrix; the off-diagonal parameter enters twice)
                double Ga = ga0.z, Gb = 0.5 * (double)ga0.w, Gc = ga1.x;
                // dL/dSigma2D = -Q G Q
                double QG00 = Qa * Ga + Qb * Gb, QG01 = Qa * Gb + Qb * Gc;
                double QG10 = Qb * Ga + Qc * Gb, QG11 = Qb * Gb + Qc * Gc;
                GS00 = -(QG00 * Qa + QG01 * Qb);
                GS01 = -(QG00 * Qb + QG01 * Qc);
                GS11 = -(QG10 * Qb + QG11 * Qc);
                dmx = ga0.x;
                dmy = ga0.y;
            }
            double GS[4] = {GS00, GS01, GS01, GS11};
            // dSigma3D += M^T GS M ; dM = 2 GS M S
            double GM[6];
            for (int a = 0; a < 2; ++a)
                for (int kk = 0; kk < 3; ++kk) GM[a * 3 + kk] = GS[a * 2] * M[kk] + GS[a * 2 + 1] * M[3 + kk];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) G3s[a * 3 + b] += M[a] * GM[b] + M[3 + a] * GM[3 + b];
            double dM[6];
            for (int a = 0; a < 2; ++a)
                for (int kk = 0; kk < 3; ++kk)
                    dM[a * 3 + kk] =
                        2.0 * (GM[a * 3] * S[kk] + GM[a * 3 + 1] * S[3 + kk] + GM[a * 3 + 2] * S[6 + kk]);
            // dJ = dM Rg (only the non-zero entries of J matter)
            double dJ00 = dM[0] * Rg[0] + dM[1] * Rg[3] + dM[2] * Rg[6];
            double dJ02 = dM[0] * Rg[2] + dM[1] * Rg[5] + dM[2] * Rg[8];
            double dJ11 = dM[3] * Rg[1] + dM[4] * Rg[4] + dM[5] * Rg[7];
            double dJ12 = dM[3] * Rg[2] + dM[4] * Rg[5] + dM[5] * Rg[8];
            double z2 = z * z, z3 = z2 * z;
            // depth path: plane branch dD/dpc = a n, dD/dnc = a pc - b; centre branch e on pc.z
            double n0 = R[0 * 3 + k], n1 = R[1 * 3 + k], n2 = R[2 * 3 + k];
            double nc0 = Rg[0] * n0 + Rg[3] * n1 + Rg[6] * n2;
            double nc1 = Rg[1] * n0 + Rg[4] * n1 + Rg[7] * n2;
            double nc2 = Rg[2] * n0 + Rg[5] * n1 + Rg[8] * n2;
            double pa = ga2.y, pb0 = ga2.z, pb1 = ga2.w, pb2 = ga3.x, pe = ga3.y;
            double dpc0 = pa * nc0 + dJ02 * (-fx / z2) + dmx * fx / z;
            double dpc1 = pa * nc1 + dJ12 * (-fy / z2) + dmy * fy / z;
            double dpc2 = pa * nc2 + pe + dJ00 * (-fx / z2) + dJ02 * (2.0 * fx * x / z3) + dJ11 * (-fy / z2) +
                          dJ12 * (2.0 * fy * y / z3) - dmx * fx * x / z2 - dmy * fy * y / z2;
            double dnc0 = pa * x - pb0, dnc1 = pa * y - pb1, dnc2 = pa * z - pb2;
            for (int a = 0; a < 3; ++a) {
                gp[a] += Rg[a * 3] * dpc0 + Rg[a * 3 + 1] * dpc1 + Rg[a * 3 + 2] * dpc2;
                dR[a * 3 + k] += Rg[a * 3] * dnc0 + Rg[a * 3 + 1] * dnc1 + Rg[a * 3 + 2] * dnc2;
            }
            ga += ga1.y;
            gc[0] += ga1.z;
            gc[1] += ga1.w;
            gc[2] += ga2.x;
        }
        // Sigma3D = R S^2 R^T: dR += 2 G3 R S^2, ds_b = 2 s_b (R^T G3 R)_bb
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double t = G3s[a * 3] * R[b] + G3s[a * 3 + 1] * R[3 + b] + G3s[a * 3 + 2] * R[6 + b];
                dR[a * 3 + b] += 2.0 * t * sq[b];
            }
        for (int b = 0; b < 3; ++b) {
            double t = 0.0;
            for (int a = 0; a < 3; ++a)
                t += R[a * 3 + b] * (G3s[a * 3] * R[b] + G3s[a * 3 + 1] * R[3 + b] + G3s[a * 3 + 2] * R[6 + b]);
            gs[b] = 2.0 * s[b] * t;
        }
        // raw quaternion: R = I + kq M(q), kq = 2 / |q|^2
        double qw = qf[0], qx = qf[1], qy = qf[2], qz = qf[3];
        double n2q = qw * qw + qx * qx + qy * qy + qz * qz, kq = 2.0 / n2q;
        double Mq[9] = {-(qy * qy + qz * qz), qx * qy - qw * qz, qx * qz + qw * qy,
                        qx * qy + qw * qz, -(qx * qx + qz * qz), qy * qz - qw * qx,
                        qx * qz - qw * qy, qy * qz + qw * qx, -(qx * qx + qy * qy)};
        double gM = 0.0;
        for (int e = 0; e < 9; ++e) gM += dR[e] * Mq[e];
        // dM/dw, dM/dx, dM/dy, dM/dz contracted with dR
        double tw = dR[1] * -qz + dR[2] * qy + dR[3] * qz + dR[5] * -qx + dR[6] * -qy + dR[7] * qx;
        double tx = dR[1] * qy + dR[2] * qz + dR[3] * qy + dR[4] * (-2 * qx) + dR[5] * -qw + dR[6] * qz +
                    dR[7] * qw + dR[8] * (-2 * qx);
        double ty = dR[0] * (-2 * qy) + dR[1] * qx + dR[2] * qw + dR[3] * qx + dR[5] * qz + dR[6] * -qw +
                    dR[7] * qz + dR[8] * (-2 * qy);
        double tz = dR[0] * (-2 * qz) + dR[1] * -qw + dR[2] * qx + dR[3] * qw + dR[4] * (-2 * qz) + dR[5] * qy +
                    dR[6] * qx + dR[7] * qy;
        double c = 2.0 / n2q * gM;
        gq[0] = kq * (tw - c * qw);
        gq[1] = kq * (tx - c * qx);
        gq[2] = kq * (ty - c * qy);
        gq[3] = kq * (tz - c * qz);
    }
    // with SH colour, k_sh_bwd has written the coefficient rows and the
    // view-direction part of d_pos already
    for (int a = 0; a < 3; ++a) {
        if (d.sh_deg == 0) {
            d_pos[3 * i + a] = (float)gp[a];
            d_col[3 * i + a] = (float)gc[a];
        } else {
            d_pos[3 * i + a] += (float)gp[a];
        }
        d_scale[3 * i + a] = (float)gs[a];
    }
    for (int a = 0; a < 4; ++a) d_rot[4 * i + a] = (float)gq[a];
    d_opac[i] = (float)ga;
}

// Unstable Gaussians can be a few percent of the set, so a thread per
// Gaussian would run the double-precision chain in nearly every wave with one
// or two lanes active.  Each workgroup walks its range of Gaussians 256 at a
// time, queues the unstable ones in LDS, and runs the chain on the queue
// whenever it holds a full workgroup's worth (and at the end of the range).
// With `on` set the camera-space gradients hold the L1 loss at unit
// upstream (the backward compositing's L1 form): every workgroup adds up the
// per-workgroup counts of M_D pixels (integers, so all agree) to form the
// scales w_c / (3 |M|) and w_d / |M_D|, and the first one also writes the
// loss value w_c / (3 |M|) sum |C - C*| + w_d / |M_D| sum |D - D*| to
// loss_out[0] and the sums and count to the header.  (Per-workgroup counts
// stay exact in binary32: a workgroup's pixels number far below 2^24.)
struct L1Scale {
    float w_c, w_d;
    float* loss_out;
    int on;
};

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o);
    return v;
}

// The upstream scales of the L1 form (every workgroup of 256 threads
// computes the same values) and, with `write` set, the loss value and sums
// into loss_out[0] and the header.
__device__ void l1_scales(const WS& w, const L1Scale& ls, bool write, float& kc, float& kd) {
    __shared__ uint32_t red_n[4];
    __shared__ float red_c[4], red_d[4];
    kc = 1.f;
    kd = 1.f;
    if (!ls.on) return;
    // both header words are read up front (the masked-pixel count is
    // needed only after the barrier below)
    const uint32_t bwd_waves = w.hdr->bwd_waves, n_px = w.hdr->n_px;
    const uint32_t nw = min(bwd_waves / 4u, (uint32_t)kMaxWaves);   // workgroups
    uint32_t cn = 0;
    float cc = 0.f, cd = 0.f;
    for (uint32_t k0 = 0; k0 < nw; k0 += 4 * blockDim.x) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t k = k0 + u * blockDim.x + threadIdx.x;
            v[u] = k < nw ? w.lwave[2 * kMaxWaves + k] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) cn += (uint32_t)v[u];
    }
    if (write)
        for (uint32_t k = threadIdx.x; k < nw; k += blockDim.x) {
            cc += w.lwave[k];
            cd += w.lwave[kMaxWaves + k];
        }
    cn = wave_sum_u32(cn);
    cc = wave_sum(cc);
    cd = wave_sum(cd);
    if ((threadIdx.x & 63) == 0) {
        red_n[threadIdx.x >> 6] = cn;
        red_c[threadIdx.x >> 6] = cc;
        red_d[threadIdx.x >> 6] = cd;
    }
    __syncthreads();
    const uint32_t nmd = (red_n[0] + red_n[1]) + (red_n[2] + red_n[3]);
    const float nm = (float)max(n_px, 1u);
    kc = ls.w_c / (3.f * nm);
    kd = ls.w_d / (float)max(nmd, 1u);
    if (write && threadIdx.x == 0) {
        const float tc = (red_c[0] + red_c[1]) + (red_c[2] + red_c[3]);
        const float td = (red_d[0] + red_d[1]) + (red_d[2] + red_d[3]);
        w.hdr->loss_c = tc;
        w.hdr->loss_d = td;
        w.hdr->cnt_md = nmd;
        ls.loss_out[0] = ls.w_c * tc / (3.f * nm) + ls.w_d * td / (float)max(nmd, 1u);
    }
}

// SH colour (Sec. 3.1): the colours of a projection's visible slots from
// the coefficients [N][K][3] at the unit direction from each frame's camera
// centre to the Gaussian, into the records' colour words.  One thread per
// Gaussian, binary64.
__global__ __launch_bounds__(256) void k_sh_color(Dims d, WS w, const float* __restrict__ pos,
                                                  const float* __restrict__ col, const double* __restrict__ poses) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.N) return;
    uint32_t vis = w.vis[i];
    if (!vis) return;
    const int K = (d.sh_deg + 1) * (d.sh_deg + 1);
    const float* cf = col + 3 * (int64_t)K * i;
    const double p0 = pos[3 * i], p1 = pos[3 * i + 1], p2 = pos[3 * i + 2];
    while (vis) {
        const int f = __builtin_ctz(vis);
        vis &= vis - 1;
        const double* tg = poses + 12 * f + 9;
        const double v0 = p0 - tg[0], v1 = p1 - tg[1], v2 = p2 - tg[2];
        const double ir = 1.0 / sqrt((v0 * v0 + v1 * v1) + v2 * v2);
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        sh_basis(d.sh_deg, v0 * ir, v1 * ir, v2 * ir, [&](int k, double yk) {
            a0 += (double)cf[3 * k] * yk;
            a1 += (double)cf[3 * k + 1] * yk;
            a2 += (double)cf[3 * k + 2] * yk;
        });
        float4* rc = w.rec + 4 * ((int64_t)f * d.N + i);
        rc[1].w = (float)a0;
        rc[2].x = (float)a1;
        rc[2].y = (float)a2;
    }
}

// SH colour gradients of the unstable Gaussians, before k_project_bwd
// consumes the slot accumulators: dL/dSH_k = sum_f dL/dc_f Y_k(u_f) into
// d_col [N][K][3], and the view-direction part of dL/dp, sum_f (I - u u^T) /
// |v| sum_k (dL/dc_f . SH_k) grad Y_k(u_f), into d_pos (k_project_bwd adds
// the rest).  One thread per Gaussian, binary64 sums over the frames.
__global__ __launch_bounds__(256) void k_sh_bwd(Dims d, WS w, const float* __restrict__ pos,
                                                const float* __restrict__ col, const uint8_t* __restrict__ unstable,
                                                const double* __restrict__ poses, float* __restrict__ d_pos,
                                                float* __restrict__ d_col, L1Scale ls) {
    float kc, kd;
    l1_scales(w, ls, false, kc, kd);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.N || !unstable[i]) return;
    const int K = (d.sh_deg + 1) * (d.sh_deg + 1);
    const float* cf = col + 3 * (int64_t)K * i;
    float* dsh = d_col + 3 * (int64_t)K * i;
    for (int k = 0; k < 3 * K; ++k) dsh[k] = 0.f;
    double gp0 = 0.0, gp1 = 0.0, gp2 = 0.0;
    const double p0 = pos[3 * i], p1 = pos[3 * i + 1], p2 = pos[3 * i + 2];
    uint32_t vis = w.vis[i];
    while (vis) {
        const int f = __builtin_ctz(vis);
        vis &= vis - 1;
        const float* gr = w.grad + 16 * ((int64_t)f * d.N + i);
        const double g0 = (double)(gr[6] * kc), g1 = (double)(gr[7] * kc), g2 = (double)(gr[8] * kc);
        const double* tg = poses + 12 * f + 9;
        const double v0 = p0 - tg[0], v1 = p1 - tg[1], v2 = p2 - tg[2];
        const double ir = 1.0 / sqrt((v0 * v0 + v1 * v1) + v2 * v2);
        const double u0 = v0 * ir, u1 = v1 * ir, u2 = v2 * ir;
        sh_basis(d.sh_deg, u0, u1, u2, [&](int k, double yk) {
            dsh[3 * k] += (float)(g0 * yk);
            dsh[3 * k + 1] += (float)(g1 * yk);
            dsh[3 * k + 2] += (float)(g2 * yk);
        });
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        sh_basis_grad(d.sh_deg, u0, u1, u2, [&](int k, double e0, double e1, double e2) {
            const double sk = (g0 * cf[3 * k] + g1 * cf[3 * k + 1]) + g2 * cf[3 * k + 2];
            t0 += sk * e0;
            t1 += sk * e1;
            t2 += sk * e2;
        });
        const double tu = (u0 * t0 + u1 * t1) + u2 * t2;
        gp0 += (t0 - u0 * tu) * ir;
        gp1 += (t1 - u1 * tu) * ir;
        gp2 += (t2 - u2 * tu) * ir;
    }
    d_pos[3 * i] = (float)gp0;
    d_pos[3 * i + 1] = (float)gp1;
    d_pos[3 * i + 2] = (float)gp2;
}

__global__ __launch_bounds__(256) void k_project_bwd(Dims d, WS w, const float* __restrict__ pos,
                                                     const float* __restrict__ scale,
                                                     const float* __restrict__ rot,
                                                     const uint8_t* __restrict__ unstable,
                                                     const double* __restrict__ poses,
                                                     float* __restrict__ d_pos, float* __restrict__ d_scale,
                                                     float* __restrict__ d_rot, float* __restrict__ d_opac,
                                                     float* __restrict__ d_col, L1Scale ls) {
    __shared__ uint32_t q[512];
    __shared__ uint32_t qn;
    float kc, kd;
    l1_scales(w, ls, blockIdx.x == 0, kc, kd);
    const int64_t per = ((d.N + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(r0 + per, d.N);
    if (threadIdx.x == 0) qn = 0u;
    __syncthreads();
    for (int64_t base = r0; base < r1; base += 256) {
        const int64_t i = base + threadIdx.x;
        if (i < r1 && unstable[i]) q[atomicAdd(&qn, 1u)] = (uint32_t)(i - r0);
        __syncthreads();
        const uint32_t n = qn;
        if (n >= 256 || base + 256 >= r1) {
            if (threadIdx.x < n)
                project_bwd_one(d, w, r0 + q[threadIdx.x], pos, scale, rot, poses, d_pos, d_scale, d_rot, d_opac,
                                d_col, kc, kd);
            if (n > 256 && threadIdx.x + 256 < n)
                project_bwd_one(d, w, r0 + q[threadIdx.x + 256], pos, scale, rot, poses, d_pos, d_scale, d_rot,
                                d_opac, d_col, kc, kd);
            __syncthreads();
            if (threadIdx.x == 0) qn = 0u;
        }
        __syncthreads();
    }
}

}  // namespace rtg
