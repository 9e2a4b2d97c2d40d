// Frame-to-model tracking (Sec. 3.2 "Camera tracking", Eq. 10) on the
// rasterizer's outputs: the rendered normal map (Sec. 3.1, the hit
// Gaussian's normal per pixel) and a multi-level projective point-to-plane
// ICP of an input depth frame against the rendered depth and normals.
//
// Per level and iteration: one thread per input pixel forms the pair of
// Eq. 10 (binary64, a fixed operation sequence), its residual and Jacobian,
// and the workgroup sums the 29 terms of the normal equations (A upper
// triangle, b, r^2, count) in a fixed tree; one workgroup then adds the
// partial sums in a fixed order, solves the 6x6 system by Cholesky and
// applies the SE(3) update to the pose held in device memory, so the whole
// iteration schedule is enqueued without a host round trip.
#include "rtg_common.h"

namespace rtg {

constexpr int kIcpTerms = 29;     // 21 (A, upper triangle) + 6 (b) + r^2 + count
constexpr int kIcpTrace = 48;     // doubles per trace row

// Normal map: the hit Gaussian's camera-frame normal {n^c} per rendered
// pixel, turned to face the camera (flipped when its dot product with the
// pixel's ray direction ((x + 0.5 - cx) / fx, (y + 0.5 - cy) / fy, 1) is
// positive, binary64); 0 on rendered pixels without a hit.
__global__ __launch_bounds__(256) void k_render_normals(Dims d, WS w, float* __restrict__ out_n) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int f;
    size_t pix;
    if (!pixel_of_rank(d, w, idx, f, pix)) return;
    const uint32_t hitpos = reinterpret_cast<const uint2*>(w.px_aux)[idx].y;
    float n0 = 0.f, n1 = 0.f, n2 = 0.f;
    if (hitpos) {
        const float4 hn = w.prec[4ull * (hitpos - 1u) + 3];
        const int64_t r = (int64_t)(pix % ((size_t)d.W * d.H));
        const int x = (int)(r % d.W), y = (int)(r / d.W);
        const double rx = (((double)x + 0.5) - d.cx) / d.fx, ry = (((double)y + 0.5) - d.cy) / d.fy;
        const double s = ((double)hn.x * rx + (double)hn.y * ry) + (double)hn.z;
        const float sg = s > 0.0 ? -1.f : 1.f;
        n0 = sg * hn.x;
        n1 = sg * hn.y;
        n2 = sg * hn.z;
    }
    out_n[3 * pix] = n0;
    out_n[3 * pix + 1] = n1;
    out_n[3 * pix + 2] = n2;
}

// Depth of level l+1: the binary32 mean of the valid (> 0) depths of the
// 2 x 2 block, ((d00 + d01) + d10) + d11 over the valid ones / their count.
__global__ __launch_bounds__(256) void k_icp_down_depth(const float* __restrict__ Df, int Wf, float* __restrict__ Dc,
                                                        int Wc, int Hc) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)Wc * Hc) return;
    const int x = (int)(p % Wc), y = (int)(p / Wc);
    const float* r0 = Df + (int64_t)(2 * y) * Wf + 2 * x;
    const float* r1 = r0 + Wf;
    const float q[4] = {r0[0], r0[1], r1[0], r1[1]};
    float s = 0.f, c = 0.f;
    for (int k = 0; k < 4; ++k)
        if (q[k] > 0.f) {
            s = s + q[k];
            c = c + 1.f;
        }
    Dc[p] = c > 0.f ? s / c : 0.f;
}

// Model normal of level l+1: that of the block's first pixel (raster order)
// with a valid depth.
__global__ __launch_bounds__(256) void k_icp_down_normal(const float* __restrict__ Df, const float* __restrict__ Nf,
                                                         int Wf, float* __restrict__ Nc, int Wc, int Hc) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)Wc * Hc) return;
    const int x = (int)(p % Wc), y = (int)(p / Wc);
    float n0 = 0.f, n1 = 0.f, n2 = 0.f;
    for (int k = 3; k >= 0; --k) {
        const int64_t q = (int64_t)(2 * y + (k >> 1)) * Wf + 2 * x + (k & 1);
        if (Df[q] > 0.f) {
            n0 = Nf[3 * q];
            n1 = Nf[3 * q + 1];
            n2 = Nf[3 * q + 2];
        }
    }
    Nc[3 * p] = n0;
    Nc[3 * p + 1] = n1;
    Nc[3 * p + 2] = n2;
}

__global__ void k_icp_copy_pose(const double* __restrict__ src, double* __restrict__ dst) {
    if (threadIdx.x < 12) dst[threadIdx.x] = src[threadIdx.x];
}

struct IcpLevel {
    int W, H;
    double fx, fy, cx, cy;
    const float* D;    // input depth
    const float* Dm;   // model depth
    const float* Nm;   // model normals (camera frame of the model pose)
};

__device__ __forceinline__ void vtx(const IcpLevel& L, int x, int y, double D, double* v) {
    v[0] = D * ((((double)x + 0.5) - L.cx) / L.fx);
    v[1] = D * ((((double)y + 0.5) - L.cy) / L.fy);
    v[2] = D;
}

__device__ __forceinline__ void mat_vec(const double* R, const double* v, double* o) {
    for (int i = 0; i < 3; ++i) o[i] = (R[3 * i] * v[0] + R[3 * i + 1] * v[1]) + R[3 * i + 2] * v[2];
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot3(const double* a, const double* b) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

// The input pixels' pairs (Eq. 10, projective association) under the
// estimate T of the input frame's camera-to-world pose against the model
// rendered at Tm; each thread strides over the pixels and adds the 29 terms
// of its kept pairs, in pixel order.
__global__ __launch_bounds__(256) void k_icp_reduce(IcpLevel L, const double* __restrict__ Tdev,
                                                    const double* __restrict__ Tm, double dist, double sin_a,
                                                    double* __restrict__ partials) {
    __shared__ double red[4][kIcpTerms];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double t[kIcpTerms];
    for (int k = 0; k < kIcpTerms; ++k) t[k] = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < (int64_t)L.W * L.H;
         p += (int64_t)gridDim.x * 256) {
        const int x = (int)(p % L.W), y = (int)(p / L.W);
        bool ok = x < L.W - 1 && y < L.H - 1;
        double D = 0.0, Dr = 0.0, Dd = 0.0;
        if (ok) {
            D = L.D[p];
            Dr = L.D[p + 1];
            Dd = L.D[p + L.W];
            ok = D > 0.0 && Dr > 0.0 && Dd > 0.0;
        }
        if (ok) {
            double T[12], M[12];
            for (int k = 0; k < 12; ++k) {
                T[k] = Tdev[k];
                M[k] = Tm[k];
            }
            double V[3], Vr[3], Vd[3], a[3], b[3], Nn[3];
            vtx(L, x, y, D, V);
            vtx(L, x + 1, y, Dr, Vr);
            vtx(L, x, y + 1, Dd, Vd);
            for (int i = 0; i < 3; ++i) {
                a[i] = Vr[i] - V[i];
                b[i] = Vd[i] - V[i];
            }
            cross3(a, b, Nn);
            double P[3], dm[3], pm[3];
            mat_vec(T, V, P);
            for (int i = 0; i < 3; ++i) P[i] = P[i] + T[9 + i];
            for (int i = 0; i < 3; ++i) dm[i] = P[i] - M[9 + i];
            for (int i = 0; i < 3; ++i) pm[i] = (M[i] * dm[0] + M[3 + i] * dm[1]) + M[6 + i] * dm[2];
            ok = pm[2] > 0.0;
            int ui = 0, vi = 0;
            if (ok) {
                const double u = floor(L.fx * pm[0] / pm[2] + L.cx);
                const double v = floor(L.fy * pm[1] / pm[2] + L.cy);
                ok = u >= 0.0 && u < (double)L.W && v >= 0.0 && v < (double)L.H;
                ui = ok ? (int)u : 0;
                vi = ok ? (int)v : 0;
            }
            const int64_t q = (int64_t)vi * L.W + ui;
            double Dmq = 0.0, nm[3] = {0.0, 0.0, 0.0};
            if (ok) {
                Dmq = L.Dm[q];
                nm[0] = L.Nm[3 * q];
                nm[1] = L.Nm[3 * q + 1];
                nm[2] = L.Nm[3 * q + 2];
                ok = Dmq > 0.0 && dot3(nm, nm) > 0.0;
            }
            if (ok) {
                double Vm[3], Q[3], n[3], m[3], dd[3], cr[3];
                vtx(L, ui, vi, Dmq, Vm);
                mat_vec(M, Vm, Q);
                for (int i = 0; i < 3; ++i) Q[i] = Q[i] + M[9 + i];
                mat_vec(M, nm, n);
                mat_vec(T, Nn, m);
                for (int i = 0; i < 3; ++i) dd[i] = P[i] - Q[i];
                cross3(m, n, cr);
                ok = dot3(dd, dd) <= dist * dist && dot3(cr, cr) <= (sin_a * sin_a) * (dot3(m, m) * dot3(n, n));
                if (ok) {
                    const double r = dot3(dd, n);
                    double J[6];
                    cross3(P, n, J);
                    J[3] = n[0];
                    J[4] = n[1];
                    J[5] = n[2];
                    int k = 0;
                    for (int i = 0; i < 6; ++i)
                        for (int j = i; j < 6; ++j) t[k++] += J[i] * J[j];
                    for (int i = 0; i < 6; ++i) t[21 + i] += J[i] * r;
                    t[27] += r * r;
                    t[28] += 1.0;
                }
            }
        }
    }
    // fixed-order reduction: wave butterflies, then the four waves in order
    for (int k = 0; k < kIcpTerms; ++k) {
        double v = t[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kIcpTerms) {
        const int k = threadIdx.x;
        partials[(int64_t)blockIdx.x * kIcpTerms + k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    }
}

// SE(3) exponential of xi = (omega, v): R = I + a [w] + b [w]^2,
// t = (I + b [w] + c [w]^2) v, a = sin th / th, b = (1 - cos th) / th^2,
// c = (th - sin th) / th^3 (R = I + [w], V = I + [w] / 2 below th = 1e-12).
__device__ void se3_exp(const double* xi, double* R, double* t) {
    const double w0 = xi[0], w1 = xi[1], w2 = xi[2];
    const double th = sqrt((w0 * w0 + w1 * w1) + w2 * w2);
    const double Wx[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
    double W2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) W2[3 * i + j] = (Wx[3 * i] * Wx[j] + Wx[3 * i + 1] * Wx[3 + j]) + Wx[3 * i + 2] * Wx[6 + j];
    double a, b, bv, c;   // bv: the [w] coefficient of V
    if (th < 1e-12) {
        a = 1.0;
        b = 0.0;
        bv = 0.5;
        c = 0.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / (th * th);
        bv = b;
        c = (th - sin(th)) / (th * th * th);
    }
    double Vm[9];
    for (int k = 0; k < 9; ++k) {
        const double id = (k % 4 == 0) ? 1.0 : 0.0;
        R[k] = id + a * Wx[k] + b * W2[k];
        Vm[k] = id + bv * Wx[k] + c * W2[k];
    }
    for (int i = 0; i < 3; ++i) t[i] = (Vm[3 * i] * xi[3] + Vm[3 * i + 1] * xi[4]) + Vm[3 * i + 2] * xi[5];
}

// One workgroup: the partial sums in a fixed order, the 6x6 solve (no
// update with fewer than 6 pairs or a non-positive pivot), the pose update
// T <- exp(xi) T and the trace row (pose used, r^2, count, A, b).
__global__ __launch_bounds__(256) void k_icp_solve(const double* __restrict__ partials, int nblk,
                                                   double* __restrict__ T, double* __restrict__ trace) {
    __shared__ double red[4][kIcpTerms];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double s[kIcpTerms];
    for (int k = 0; k < kIcpTerms; ++k) s[k] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256)
        for (int k = 0; k < kIcpTerms; ++k) s[k] += partials[(int64_t)b * kIcpTerms + k];
    for (int k = 0; k < kIcpTerms; ++k) {
        double v = s[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double tot[kIcpTerms];
    for (int k = 0; k < kIcpTerms; ++k) tot[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    double A[36], bb[6];
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            A[6 * i + j] = tot[k];
            A[6 * j + i] = tot[k];
            ++k;
        }
    for (int i = 0; i < 6; ++i) bb[i] = tot[21 + i];
    if (trace) {
        for (int i = 0; i < 12; ++i) trace[i] = T[i];
        trace[12] = tot[27];
        trace[13] = tot[28];
        for (int i = 0; i < 27; ++i) trace[14 + i] = tot[i];
        for (int i = 41; i < kIcpTerms + 19; ++i) trace[i] = 0.0;
    }
    // Cholesky A = L L^T
    double Lc[36];
    bool good = tot[28] >= 6.0;
    for (int i = 0; i < 6 && good; ++i)
        for (int j = 0; j <= i; ++j) {
            double acc = A[6 * i + j];
            for (int m = 0; m < j; ++m) acc -= Lc[6 * i + m] * Lc[6 * j + m];
            if (i == j) {
                if (!(acc > 0.0)) {
                    good = false;
                    break;
                }
                Lc[6 * i + i] = sqrt(acc);
            } else {
                Lc[6 * i + j] = acc / Lc[6 * j + j];
            }
        }
    if (!good) return;
    double yv[6], xi[6];
    for (int i = 0; i < 6; ++i) {
        double acc = bb[i];
        for (int m = 0; m < i; ++m) acc -= Lc[6 * i + m] * yv[m];
        yv[i] = acc / Lc[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double acc = yv[i];
        for (int m = i + 1; m < 6; ++m) acc -= Lc[6 * m + i] * xi[m];
        xi[i] = acc / Lc[6 * i + i];
    }
    for (int i = 0; i < 6; ++i) xi[i] = -xi[i];
    double dR[9], dt[3];
    se3_exp(xi, dR, dt);
    double Rn[9], tn[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) Rn[3 * i + j] = (dR[3 * i] * T[j] + dR[3 * i + 1] * T[3 + j]) + dR[3 * i + 2] * T[6 + j];
        tn[i] = ((dR[3 * i] * T[9] + dR[3 * i + 1] * T[10]) + dR[3 * i + 2] * T[11]) + dt[i];
    }
    for (int i = 0; i < 9; ++i) T[i] = Rn[i];
    for (int i = 0; i < 3; ++i) T[9 + i] = tn[i];
}

}  // namespace rtg
