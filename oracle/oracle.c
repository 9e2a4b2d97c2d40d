/*
 * oracle.c -- plain FP64 CPU reference of the masked differentiable Gaussian
 * rasterizer of RTG-SLAM (Peng et al., SIGGRAPH 2024, arXiv 2404.19706).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP library.
 *
 * What it computes, and the passage each part follows:
 *   orc_project     Sec. 3.1 "Image rendering": camera frame of a Gaussian,
 *                   the splatted 2D Gaussian of Eq. (2) (local affine
 *                   projection of Sigma = R S S^T R^T), the surfel normal
 *                   (direction of the smallest eigenvector, Sec. 3.1), and the
 *                   per-Gaussian depth-test threshold tau derived from
 *                   delta_alpha = e^-0.5.
 *   orc_bin         Supplementary Sec. B: 16x16 (or other) tiles, one key per
 *                   (Gaussian, tile) combining view-space depth and tile id,
 *                   sorted; the optional rule that drops tiles in which fewer
 *                   than half of the pixels need rendering.  Pairs exist only
 *                   for rectangle tiles the Gaussian's cut-off ellipse
 *                   reaches (a conservative thinning: it changes which pairs
 *                   exist, never which pixels see a Gaussian).
 *   orc_render      Eq. (1) colour by front-to-back alpha blending, Eq. (2)
 *                   per-pixel opacity, Eq. (3) transmission, Eq. (4) ray/disc
 *                   intersection of the first Gaussian whose per-pixel opacity
 *                   exceeds delta_alpha, Eq. (5) depth map with the 60 degree
 *                   fallback and -1 when nothing is hit, and the index map.
 *   orc_backward    the derivative of Eqs. (1)-(5) with respect to position,
 *                   scale, rotation, opacity and colour (Sec. 3.1 states the
 *                   depth is linear in position and rotation and
 *                   differentiable; Sec. 3.2 optimises unstable Gaussians
 *                   only), summed over pixels and frames.
 *   orc_backward_bound  the same gradients with a per-entry bound on the error
 *                   of a binary32 evaluation (test tolerance, not a result).
 *   orc_pixel_lists  the list L(u) of each pixel (test helper).
 *   orc_unstable_mask  Supplementary Sec. B: M_unstable = pixels where the
 *                   transmission rendered with the unstable Gaussians alone
 *                   is below one.
 *
 * Conventions the paper leaves open (each one is listed as a reading in the
 * design notes): pixel centres at (x+0.5, y+0.5); T_g maps camera to world,
 * camera looks along +z with x right and y down; quaternion (w,x,y,z) used
 * without normalisation through R = I + (2/|q|^2) M(q) (equal to the rotation
 * of q/|q|); near-plane cull at z <= z_near; local affine (EWA) projection
 * without frustum clamp; footprint cut-off d^2 <= rho^2; per-pixel opacity
 * clamped at 0.99; front-to-back means ascending centre depth, ties by index.
 *
 * Two layers.  Every discrete decision (cull, pixel rectangle, depth key,
 * pixel inclusion, depth hit, 60 degree branch) is made by one fixed sequence
 * of IEEE-754 operations written down in the design notes, so that an
 * independent implementation following the same sequence reproduces every
 * decision bit for bit.  Every continuous value (colour, transmission, depth,
 * gradients) is computed here in binary64.
 *
 * Pins (tests/test_oracle_*.py): closed forms for one and two Gaussians, the
 * opaque disc at normal incidence, a tilted disc checked against an
 * independent world-space ray/plane intersection, Sigma_3D against scipy's
 * quaternion rotation, the projection Jacobian against finite differences of
 * the pinhole map, brute-force tile coverage (including pixels that the
 * binary32 decision admits on needle footprints), dropped pairs checked to
 * miss every pixel centre of their tile, transmission monotonicity and the
 * convex-hull property, and central finite differences of the forward pass
 * for every gradient.  The constants rho, z_near and the dilation are
 * this implementation's own choices: parity unpinned by the paper for them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Types shared with the Python binding (oracle/oracle.py mirrors them).     */

typedef struct {
    double fx, fy, cx, cy;      /* pinhole intrinsics K (Sec. 3.1)            */
    int32_t width, height;      /* image size in pixels                       */
    float cutoff2;              /* rho^2: footprint cut-off on d^2            */
    float dilation;             /* eps added to the diagonal of Sigma_2D      */
    float z_near;               /* near-plane cull distance                   */
    int32_t tile_w, tile_h;     /* tile shape for binning                     */
} orc_params;

typedef struct {
    int32_t culled;             /* 1: behind near plane / degenerate          */
    int32_t visible;            /* 0 culled, or pixel rectangle off-image     */
    int32_t rect[4];            /* x0, x1, y0, y1 inclusive, clipped          */
    int32_t axis;               /* index of the thin axis (surfel normal)     */
    float mu32[2];              /* decision-layer copies, each fl32(binary64) */
    float conic32[3];
    float z32, tau32;
    float nc32[3], h32;
    double pc[3];               /* camera-frame centre                        */
    double mu[2];               /* pixel-space centre                         */
    double cov[3];              /* Sigma_2D xx, xy, yy (incl. dilation)       */
    double conic[3];            /* Sigma_2D^-1 xx, xy, yy                     */
    double nc[3];               /* camera-frame surfel normal                 */
    double h;                   /* pc . nc (plane offset)                     */
} orc_rec;

int32_t orc_sizeof_rec(void) { return (int32_t)sizeof(orc_rec); }
int32_t orc_sizeof_params(void) { return (int32_t)sizeof(orc_params); }

int32_t orc_num_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the parallel loops below (timing harness only). */
void orc_set_num_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Rotation of a raw quaternion q = (w, x, y, z), R = I + (2/|q|^2) M(q).    */
static int quat_to_rot(const float* q, double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double n2 = ((w * w + x * x) + y * y) + z * z;
    if (!(n2 > 0.0) || !isfinite(n2)) return 0;
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
    return 1;
}

/* Inclusive pixel range on one axis that contains every pixel centre whose
 * offset from mu satisfies off^2 <= r2 (with one pixel of slack), clipped to
 * [0, n-1].  E = ceil(sqrt(r2)) is found by an exact integer fix-up so the
 * result never depends on the rounding of sqrt.  Returns 0 when empty. */
static int axis_range(double mu, double r2, int32_t n, int32_t* lo, int32_t* hi) {
    if (!(r2 >= 0.0)) return 0;
    if (r2 > 4096.0 * 4096.0) { *lo = 0; *hi = n - 1; return 1; }
    double e = ceil(sqrt(r2));
    while (e > 0.0 && (e - 1.0) * (e - 1.0) >= r2) e -= 1.0;
    while (e * e < r2) e += 1.0;
    double c = floor(mu);
    double a = c - e - 2.0, b = c + e + 1.0;
    if (a > (double)(n - 1) || b < 0.0) return 0;
    if (a < 0.0) a = 0.0;
    if (b > (double)(n - 1)) b = (double)(n - 1);
    *lo = (int32_t)a;
    *hi = (int32_t)b;
    return 1;
}

/* Cut-off for the rectangle: rho^2 / (1 - t), t = 16 * 2^-24 * K * lmax, or
 * infinite (the whole image) when t >= 1/2.  A pixel that passes the
 * binary32 decision has q <= rho^2 + 8 * 2^-24 * M under the binary64 conic
 * (binary32 evaluation of the form plus rounding of its entries), where M =
 * qa x^2 + |2 qb x y| + qc y^2 <= K (x^2 + y^2), K = max(qa, qc) + |qb|, and
 * x^2 + y^2 <= lmax q, lmax the largest eigenvalue of Sigma_2D; so q <=
 * rho^2 / (1 - t / 2) and the rectangle of rho^2 / (1 - t) holds every such
 * pixel, also for needle-like footprints. */
static double rect_cutoff(float cutoff2, double sxx, double sxy, double syy, double qa, double qb, double qc) {
    double K = (qa > qc ? qa : qc) + fabs(qb);
    double h = 0.5 * (sxx - syy);
    double lmax = 0.5 * (sxx + syy) + sqrt(h * h + sxy * sxy);
    double t = 9.5367431640625e-07 * (K * lmax);
    return t < 0.5 ? (double)cutoff2 / (1.0 - t) : INFINITY;
}

/* Projection of Gaussian (p, s, q, alpha) into the camera with pose
 * Rg (row-major camera-to-world rotation) and tg (Sec. 3.1). */
static void project_one(const orc_params* P, const double* Rg, const double* tg,
                        const float* p, const float* s, const float* q, float alpha,
                        orc_rec* r) {
    memset(r, 0, sizeof *r);
    r->culled = 1;
    r->tau32 = -INFINITY;
    /* camera frame: pc = Rg^T (p - tg) */
    double v0 = (double)p[0] - tg[0], v1 = (double)p[1] - tg[1], v2 = (double)p[2] - tg[2];
    double x = (Rg[0] * v0 + Rg[3] * v1) + Rg[6] * v2;
    double y = (Rg[1] * v0 + Rg[4] * v1) + Rg[7] * v2;
    double z = (Rg[2] * v0 + Rg[5] * v1) + Rg[8] * v2;
    r->pc[0] = x; r->pc[1] = y; r->pc[2] = z;
    if (!(z > (double)P->z_near)) return;

    double R[9];
    if (!quat_to_rot(q, R)) return;
    /* Sigma_3D = R diag(s^2) R^T */
    double s2[3] = {(double)s[0] * (double)s[0], (double)s[1] * (double)s[1],
                    (double)s[2] * (double)s[2]};
    double S[9];
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
            double v = ((R[a * 3 + 0] * s2[0]) * R[b * 3 + 0] + (R[a * 3 + 1] * s2[1]) * R[b * 3 + 1]) +
                       (R[a * 3 + 2] * s2[2]) * R[b * 3 + 2];
            S[a * 3 + b] = v;
            S[b * 3 + a] = v;
        }
    /* local affine projection J at pc, M = J Rg^T */
    double fx = P->fx, fy = P->fy;
    double J00 = fx / z, J02 = -((fx * x) / (z * z));
    double J11 = fy / z, J12 = -((fy * y) / (z * z));
    double M[6];
    for (int k = 0; k < 3; ++k) {
        M[0 * 3 + k] = J00 * Rg[k * 3 + 0] + J02 * Rg[k * 3 + 2];
        M[1 * 3 + k] = J11 * Rg[k * 3 + 1] + J12 * Rg[k * 3 + 2];
    }
    double T[6];
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k)
            T[a * 3 + k] = (M[a * 3 + 0] * S[0 * 3 + k] + M[a * 3 + 1] * S[1 * 3 + k]) +
                           M[a * 3 + 2] * S[2 * 3 + k];
    double eps = (double)P->dilation;
    double sxx = ((T[0] * M[0] + T[1] * M[1]) + T[2] * M[2]) + eps;
    double sxy = (T[0] * M[3] + T[1] * M[4]) + T[2] * M[5];
    double syy = ((T[3] * M[3] + T[4] * M[4]) + T[5] * M[5]) + eps;
    double det = sxx * syy - sxy * sxy;
    if (!(det > 0.0)) return;
    double ca = syy / det, cb = -(sxy / det), cc = sxx / det;
    double mux = (fx * x) / z + P->cx;
    double muy = (fy * y) / z + P->cy;
    if (!(fabs(mux) < 16777216.0) || !(fabs(muy) < 16777216.0)) return;

    r->culled = 0;
    r->mu[0] = mux; r->mu[1] = muy;
    r->cov[0] = sxx; r->cov[1] = sxy; r->cov[2] = syy;
    r->conic[0] = ca; r->conic[1] = cb; r->conic[2] = cc;
    r->mu32[0] = (float)mux; r->mu32[1] = (float)muy;
    r->conic32[0] = (float)ca; r->conic32[1] = (float)cb; r->conic32[2] = (float)cc;
    r->z32 = (float)z;
    double a64 = (double)alpha;
    r->tau32 = (a64 > 0.0) ? (float)(1.0 + 2.0 * log(a64)) : -INFINITY;

    /* surfel normal: column of R for the smallest scale (lowest index on ties) */
    int k = 0;
    if (s[1] < s[k]) k = 1;
    if (s[2] < s[k]) k = 2;
    r->axis = k;
    double n0 = R[0 * 3 + k], n1 = R[1 * 3 + k], n2 = R[2 * 3 + k];
    for (int j = 0; j < 3; ++j)
        r->nc[j] = (Rg[0 * 3 + j] * n0 + Rg[1 * 3 + j] * n1) + Rg[2 * 3 + j] * n2;
    r->h = (x * r->nc[0] + y * r->nc[1]) + z * r->nc[2];
    for (int j = 0; j < 3; ++j) r->nc32[j] = (float)r->nc[j];
    r->h32 = (float)r->h;

    double c2 = rect_cutoff(P->cutoff2, sxx, sxy, syy, ca, cb, cc);
    int32_t x0, x1, y0, y1;
    if (!axis_range(mux, c2 * sxx, P->width, &x0, &x1)) return;
    if (!axis_range(muy, c2 * syy, P->height, &y0, &y1)) return;
    r->visible = 1;
    r->rect[0] = x0; r->rect[1] = x1; r->rect[2] = y0; r->rect[3] = y1;
}

/* Project N Gaussians into F frames.  poses: F x 12 doubles (row-major R_g
 * then t_g).  out: F*N records, frame-major. */
void orc_project(const orc_params* P, int64_t N, int32_t F, const double* poses,
                 const float* pos, const float* scale, const float* rot, const float* opacity,
                 orc_rec* out) {
    for (int32_t f = 0; f < F; ++f) {
        const double* Rg = poses + (size_t)f * 12;
        const double* tg = Rg + 9;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i)
            project_one(P, Rg, tg, pos + 3 * i, scale + 3 * i, rot + 4 * i, opacity[i],
                        out + (size_t)f * N + i);
    }
}

/* ------------------------------------------------------------------------ */
/* Decision-layer d^2 (binary32, fixed sequence).                            */
static float dd_decision(const orc_rec* r, float ux, float uy) {
    float dx = ux - r->mu32[0];
    float dy = uy - r->mu32[1];
    float t0 = (r->conic32[0] * dx) * dx;
    float b2 = 2.0f * r->conic32[1];
    float t1 = fmaf(b2 * dx, dy, t0);
    return fmaf(r->conic32[2] * dy, dy, t1);
}

/* 60 degree rule of Eq. (5): the line of the normal and the ray make an
 * unsigned angle below 60 degrees iff (n.d)^2 > (1/4)|d|^2 |n|^2; d is a
 * positive multiple of K^-1 u so no division enters the decision. */
static int plane_branch(const orc_params* P, const float nc32[3], float ux, float uy) {
    double n0 = nc32[0], n1 = nc32[1], n2 = nc32[2];
    double d0 = P->fy * ((double)ux - P->cx);
    double d1 = P->fx * ((double)uy - P->cy);
    double d2 = P->fx * P->fy;
    double nd = (n0 * d0 + n1 * d1) + n2 * d2;
    double lhs = nd * nd;
    double dd = (d0 * d0 + d1 * d1) + d2 * d2;
    double nn = (n0 * n0 + n1 * n1) + n2 * n2;
    double rhs = (0.25 * dd) * nn;
    return lhs > rhs;
}

/* ------------------------------------------------------------------------ */
/* Binning (supplementary Sec. B).                                           */

typedef struct { int32_t frame, tile; float z; int32_t gid; } pair_t;

static int cmp_pair(const void* A, const void* B) {
    const pair_t* a = (const pair_t*)A;
    const pair_t* b = (const pair_t*)B;
    if (a->frame != b->frame) return a->frame < b->frame ? -1 : 1;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->z != b->z) return a->z < b->z ? -1 : 1;
    if (a->gid != b->gid) return a->gid < b->gid ? -1 : 1;
    return 0;
}

/* The sparse-tile rule: on a fixed 16x16 grid, a block keeps its masked
 * pixels iff at least half of its in-image pixels are masked. */
void orc_filter50(const orc_params* P, int32_t F, const uint8_t* mask, uint8_t* out) {
    int32_t W = P->width, H = P->height;
    memcpy(out, mask, (size_t)F * W * H);
    for (int32_t f = 0; f < F; ++f)
        for (int32_t by = 0; by < H; by += 16)
            for (int32_t bx = 0; bx < W; bx += 16) {
                int32_t cnt = 0, area = 0;
                for (int32_t y = by; y < by + 16 && y < H; ++y)
                    for (int32_t x = bx; x < bx + 16 && x < W; ++x) {
                        ++area;
                        cnt += mask[((size_t)f * H + y) * W + x] != 0;
                    }
                if (2 * cnt < area)
                    for (int32_t y = by; y < by + 16 && y < H; ++y)
                        for (int32_t x = bx; x < bx + 16 && x < W; ++x)
                            out[((size_t)f * H + y) * W + x] = 0;
            }
}

/* Pair thinning.  Tile (a, b) of record r's tile rectangle is kept when
 * the box of the tile's pixel centres (clipped to the image) meets the
 * ellipse q <= c of the decision-layer conic (centre mu32, conic32;
 * q(x, y) = qa x^2 + 2 qb x y + qc y^2 in offsets from the centre).  The
 * bound c = (cut * 1.001 + 1e-3) + 1e-6 M, with M = qa X^2 + |2 qb| X Y +
 * qc Y^2 for X, Y the largest offsets over the rectangle's tile columns and
 * the tile row, bounds the binary32 rounding error of the per-pixel
 * decision, so a dropped pair has d^2 > cut-off at every pixel of the tile.
 * row_interval gives the x-range [xl, xh] of the ellipse inside the row's
 * band y in [ly, hy] (returns 0 when the band misses it): the right end is
 * the ellipse's rightmost point x_t = sqrt(c qc / det) if its y_t =
 * -qb x_t / qc lies in the band, else the larger root of q(x, y_e) = c on
 * the band edge y_e nearer to y_t (a negative discriminant there: the band
 * misses the ellipse); the left end mirrors it through the centre.  A conic
 * whose binary32 entries are not positive definite (the sign of det is
 * exact: both products are exact in binary64) keeps the whole row.  A
 * fixed binary64 sequence. */
static double box_lo(const orc_params* P, int32_t a, double mux) { return ((double)(a * P->tile_w) + 0.5) - mux; }
static double box_hi(const orc_params* P, int32_t a, double mux) {
    int32_t e = a * P->tile_w + P->tile_w < P->width ? a * P->tile_w + P->tile_w : P->width;
    return ((double)e - 0.5) - mux;
}

static int row_interval(const orc_params* P, const orc_rec* r, int32_t b, double* xl, double* xh) {
    int32_t th = P->tile_h, H = P->height;
    int32_t a0 = r->rect[0] / P->tile_w, a1 = r->rect[1] / P->tile_w;
    double qa = (double)r->conic32[0], qb = (double)r->conic32[1], qc = (double)r->conic32[2];
    double det = qa * qc - qb * qb;
    if (!(qa > 0.0 && det > 0.0)) {
        *xl = -INFINITY;
        *xh = INFINITY;
        return 1;
    }
    double mux = (double)r->mu32[0], muy = (double)r->mu32[1];
    double ly = ((double)(b * th) + 0.5) - muy;
    double hy = ((double)(b * th + th < H ? b * th + th : H) - 0.5) - muy;
    double lo = -box_lo(P, a0, mux), hi = box_hi(P, a1, mux);
    double X = lo > hi ? lo : hi, Y = -ly > hy ? -ly : hy;
    double M = ((qa * X) * X + ((2.0 * fabs(qb)) * X) * Y) + (qc * Y) * Y;
    double c = ((double)P->cutoff2 * 1.001 + 1e-3) + 1e-6 * M;
    double xt = sqrt((c * qc) / det);
    double yt = -(qb * xt) / qc;
    if (yt >= ly && yt <= hy) *xh = xt;
    else {
        double ye = yt < ly ? ly : hy;
        double D = qa * c - det * (ye * ye);
        if (D < 0.0) return 0;
        *xh = (-(qb * ye) + sqrt(D)) / qa;
    }
    double ym = -yt;
    if (ym >= ly && ym <= hy) *xl = -xt;
    else {
        double ye = ym < ly ? ly : hy;
        double D = qa * c - det * (ye * ye);
        if (D < 0.0) return 0;
        *xl = (-(qb * ye) - sqrt(D)) / qa;
    }
    return 1;
}

static int tile_kept(const orc_params* P, const orc_rec* r, int32_t a, int row_ok, double xl, double xh) {
    double mux = (double)r->mu32[0];
    return row_ok && box_lo(P, a, mux) <= xh && box_hi(P, a, mux) >= xl;
}

/* Pairs (frame, tile, gid) for every visible record and every active tile
 * (one holding at least one masked pixel) inside its tile rectangle that the
 * record's cut-off ellipse can reach (tile_kept), sorted by (frame, tile,
 * depth, gid).  Returns the pair count K; arrays are filled only when
 * K <= cap.  tile_active_out: F * tiles bytes. */
int64_t orc_bin(const orc_params* P, int64_t N, int32_t F, const orc_rec* recs, const uint8_t* mask,
                int64_t cap, int32_t* out_frame, int32_t* out_tile, int32_t* out_gid,
                uint8_t* tile_active_out) {
    int32_t W = P->width, H = P->height, tw = P->tile_w, th = P->tile_h;
    int32_t tx = (W + tw - 1) / tw, ty = (H + th - 1) / th, nt = tx * ty;
    uint8_t* act = tile_active_out;
    memset(act, 0, (size_t)F * nt);
    for (int32_t f = 0; f < F; ++f)
        for (int32_t y = 0; y < H; ++y)
            for (int32_t x = 0; x < W; ++x)
                if (mask[((size_t)f * H + y) * W + x]) act[(size_t)f * nt + (y / th) * tx + x / tw] = 1;
    int64_t K = 0;
    for (int32_t f = 0; f < F; ++f)
        for (int64_t i = 0; i < N; ++i) {
            const orc_rec* r = recs + (size_t)f * N + i;
            if (!r->visible) continue;
            for (int32_t b = r->rect[2] / th; b <= r->rect[3] / th; ++b) {
                double xl, xh;
                int ok = row_interval(P, r, b, &xl, &xh);
                for (int32_t a = r->rect[0] / tw; a <= r->rect[1] / tw; ++a)
                    K += act[(size_t)f * nt + b * tx + a] && tile_kept(P, r, a, ok, xl, xh);
            }
        }
    if (K > cap) return K;
    pair_t* pr = (pair_t*)malloc(sizeof(pair_t) * (size_t)(K > 0 ? K : 1));
    int64_t k = 0;
    for (int32_t f = 0; f < F; ++f)
        for (int64_t i = 0; i < N; ++i) {
            const orc_rec* r = recs + (size_t)f * N + i;
            if (!r->visible) continue;
            for (int32_t b = r->rect[2] / th; b <= r->rect[3] / th; ++b) {
                double xl, xh;
                int ok = row_interval(P, r, b, &xl, &xh);
                for (int32_t a = r->rect[0] / tw; a <= r->rect[1] / tw; ++a)
                    if (act[(size_t)f * nt + b * tx + a] && tile_kept(P, r, a, ok, xl, xh)) {
                        pr[k].frame = f;
                        pr[k].tile = b * tx + a;
                        pr[k].z = r->z32;
                        pr[k].gid = (int32_t)i;
                        ++k;
                    }
            }
        }
    if (K > 1) qsort(pr, (size_t)K, sizeof(pair_t), cmp_pair);
    for (int64_t j = 0; j < K; ++j) {
        out_frame[j] = pr[j].frame;
        out_tile[j] = pr[j].tile;
        out_gid[j] = pr[j].gid;
    }
    free(pr);
    return K;
}

/* ------------------------------------------------------------------------ */
/* Per-pixel forward.                                                        */

typedef struct { float z; int32_t gid; } cand_t;

static int cmp_cand(const void* A, const void* B) {
    const cand_t* a = (const cand_t*)A;
    const cand_t* b = (const cand_t*)B;
    if (a->z != b->z) return a->z < b->z ? -1 : 1;
    return (a->gid > b->gid) - (a->gid < b->gid);
}

/* The list of Gaussians crossed by the ray of pixel (ux, uy) in frame f:
 * every non-culled Gaussian whose decision-layer d^2 is within the cut-off,
 * in ascending (centre depth, index) order.  Returns its length. */
static int64_t pixel_list(const orc_params* P, int64_t N, const orc_rec* fr, float ux, float uy,
                          cand_t** buf, int64_t* cap) {
    int64_t n = 0;
    for (int64_t i = 0; i < N; ++i) {
        const orc_rec* r = fr + i;
        if (r->culled) continue;
        if (!(dd_decision(r, ux, uy) <= P->cutoff2)) continue;
        if (n == *cap) {
            *cap = *cap ? 2 * *cap : 256;
            *buf = (cand_t*)realloc(*buf, sizeof(cand_t) * (size_t)*cap);
        }
        (*buf)[n].z = r->z32;
        (*buf)[n].gid = (int32_t)i;
        ++n;
    }
    if (n > 1) qsort(*buf, (size_t)n, sizeof(cand_t), cmp_cand);   /* (no call with an empty buffer) */
    return n;
}

/* Value-layer squared distance of Eq. (2), d^2 = (u - mu)^T Q (u - mu),
 * written through the Cholesky factor of Q = [[a, b], [b, c]]:
 * d^2 = a t^2 + dy^2 / Sigma_yy with t = dx + (b / a) dy (c - b^2 / a =
 * det Q / a = 1 / Sigma_yy).  Unlike the expanded form, whose terms cancel
 * on needle footprints, its binary64 rounding error stays a few units in
 * the last place of d^2 whatever the footprint's condition number. */
static double dd_value(const orc_rec* r, double ux, double uy) {
    double dx = ux - r->mu[0], dy = uy - r->mu[1];
    double t = dx + (r->conic[1] / r->conic[0]) * dy;
    return r->conic[0] * t * t + dy * dy / r->cov[2];
}

/* Q (u - mu) in the same factored form: (a t, b t + dy / Sigma_yy). */
static void q_delta(const orc_rec* r, double ux, double uy, double out[2]) {
    double dx = ux - r->mu[0], dy = uy - r->mu[1];
    double t = dx + (r->conic[1] / r->conic[0]) * dy;
    out[0] = r->conic[0] * t;
    out[1] = r->conic[1] * t + dy / r->cov[2];
}

static uint64_t fnv(uint64_t h, uint64_t v) {
    for (int b = 0; b < 8; ++b) {
        h ^= (v >> (8 * b)) & 0xff;
        h *= 1099511628211ull;
    }
    return h;
}

/* Render the pixels listed in pix (P x 3 int32: frame, x, y).  Outputs per
 * pixel: colour (3), depth, transmission, index (-1 when no hit), branch
 * (0 none, 1 ray/plane, 2 centre depth), list length, and a signature of
 * every discrete decision taken (list, clamps, hit, branch). */
void orc_render(const orc_params* P, int64_t N, int32_t F, const orc_rec* recs,
                const float* opacity, const double* color, int64_t NP, const int32_t* pix,
                double* out_color, double* out_depth, double* out_trans, int32_t* out_index,
                int32_t* out_branch, int32_t* out_nlist, uint64_t* out_sig) {
    (void)F;
#pragma omp parallel
    {
        cand_t* buf = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < NP; ++p) {
            int32_t f = pix[3 * p], px = pix[3 * p + 1], py = pix[3 * p + 2];
            const orc_rec* fr = recs + (size_t)f * N;
            float ux = (float)px + 0.5f, uy = (float)py + 0.5f;
            int64_t n = pixel_list(P, N, fr, ux, uy, &buf, &cap);
            double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
            int32_t hit = -1;
            uint64_t sig = 1469598103934665603ull;
            for (int64_t k = 0; k < n; ++k) {
                int32_t i = buf[k].gid;
                const orc_rec* r = fr + i;
                double g = exp(-0.5 * dd_value(r, ux, uy));
                double fa = (double)opacity[i] * g;
                int clamped = fa > 0.99;
                double fv = clamped ? 0.99 : fa;
                for (int c = 0; c < 3; ++c) C[c] += (double)color[3 * i + c] * fv * T;
                if (hit < 0 && dd_decision(r, ux, uy) < r->tau32) hit = i;
                T *= 1.0 - fv;
                sig = fnv(sig, ((uint64_t)(uint32_t)i << 1) | (uint64_t)clamped);
            }
            double D = -1.0;
            int32_t br = 0;
            if (hit >= 0) {
                const orc_rec* r = fr + hit;
                if (plane_branch(P, r->nc32, ux, uy)) {
                    double d0 = ((double)ux - P->cx) / P->fx, d1 = ((double)uy - P->cy) / P->fy;
                    double dn = r->nc[0] * d0 + r->nc[1] * d1 + r->nc[2];
                    D = r->h / dn;
                    br = 1;
                } else {
                    D = r->pc[2];
                    br = 2;
                }
            }
            sig = fnv(sig, (uint64_t)(int64_t)hit);
            sig = fnv(sig, (uint64_t)br);
            for (int c = 0; c < 3; ++c) out_color[3 * p + c] = C[c];
            out_depth[p] = D;
            out_trans[p] = T;
            out_index[p] = hit;
            out_branch[p] = br;
            out_nlist[p] = (int32_t)n;
            out_sig[p] = sig;
        }
        free(buf);
    }
}

/* The list L(u) of each listed pixel: the Gaussians whose decision
 * distance is within the cut-off, in (z, index) order.  out_len[p] receives
 * its length and out_gid[p * max_len ...] its first max_len entries. */
void orc_pixel_lists(const orc_params* P, int64_t N, int32_t F, const orc_rec* recs, int64_t NP,
                     const int32_t* pix, int32_t max_len, int32_t* out_gid, int32_t* out_len) {
    (void)F;
#pragma omp parallel
    {
        cand_t* buf = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < NP; ++p) {
            int32_t f = pix[3 * p], px = pix[3 * p + 1], py = pix[3 * p + 2];
            int64_t n = pixel_list(P, N, recs + (size_t)f * N, (float)px + 0.5f, (float)py + 0.5f, &buf, &cap);
            out_len[p] = (int32_t)n;
            for (int64_t k = 0; k < n && k < max_len; ++k) out_gid[p * (int64_t)max_len + k] = buf[k].gid;
        }
        free(buf);
    }
}

/* M_unstable for the listed pixels: 1 iff some non-culled unstable Gaussian
 * has the pixel inside its cut-off, which is exactly the set where the
 * transmission rendered from the unstable Gaussians alone is below one
 * (every factor 1 - f with f > 0 is below one). */
void orc_unstable_mask(const orc_params* P, int64_t N, int32_t F, const orc_rec* recs,
                       const uint8_t* unstable, int64_t NP, const int32_t* pix, uint8_t* out) {
    (void)F;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < NP; ++p) {
        int32_t f = pix[3 * p], px = pix[3 * p + 1], py = pix[3 * p + 2];
        const orc_rec* fr = recs + (size_t)f * N;
        float ux = (float)px + 0.5f, uy = (float)py + 0.5f;
        uint8_t m = 0;
        for (int64_t i = 0; i < N && !m; ++i) {
            if (!unstable[i] || fr[i].culled) continue;
            if (dd_decision(fr + i, ux, uy) <= P->cutoff2) m = 1;
        }
        out[p] = m;
    }
}

/* ------------------------------------------------------------------------ */
/* Backward.                                                                 */

/* Camera-space gradient of one record: dmu(2), dconic(3: xx, xy counted as
 * one parameter, yy), dalpha, dcolor(3), dpc(3), dnc(3). */
enum { G_MU = 0, G_CON = 2, G_AL = 5, G_COL = 6, G_PC = 9, G_NC = 12, G_N = 15 };

/* g: the contribution; with error bounds requested, e: the bound of its
 * binary32 evaluation error and t: of what a pixel's early exit may change
 * in it (see orc_backward_bound). */
typedef struct { int64_t rec; double g[G_N]; double e[G_N]; double t[G_N]; } contrib_t;

/* Chain rule from a record's camera-space gradient to the parameters of its
 * Gaussian (position 3, scale 3, rotation 4, opacity 1, colour 3), added to
 * out (14 doubles). */
static void chain_to_params(const orc_params* P, const double* Rg, const orc_rec* r,
                            const float* s, const float* q, const double* g, double* out) {
    double R[9];
    quat_to_rot(q, R);
    double x = r->pc[0], y = r->pc[1], z = r->pc[2];
    double fx = P->fx, fy = P->fy;
    double s2[3] = {(double)s[0] * s[0], (double)s[1] * s[1], (double)s[2] * s[2]};
    double S[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += R[a * 3 + k] * s2[k] * R[b * 3 + k];
            S[a * 3 + b] = v;
        }
    double J[6] = {fx / z, 0.0, -fx * x / (z * z), 0.0, fy / z, -fy * y / (z * z)};
    double M[6];
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k) {
            double v = 0.0;
            for (int b = 0; b < 3; ++b) v += J[a * 3 + b] * Rg[k * 3 + b]; /* W[b][k] = Rg[k][b] */
            M[a * 3 + k] = v;
        }
    /* dL/dQ as a symmetric matrix, then dL/dSigma2D = -Q G Q */
    double Q[4] = {r->conic[0], r->conic[1], r->conic[1], r->conic[2]};
    double G[4] = {g[G_CON + 0], 0.5 * g[G_CON + 1], 0.5 * g[G_CON + 1], g[G_CON + 2]};
    double QG[4], GS[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) QG[a * 2 + b] = Q[a * 2 + 0] * G[0 * 2 + b] + Q[a * 2 + 1] * G[1 * 2 + b];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) GS[a * 2 + b] = -(QG[a * 2 + 0] * Q[0 * 2 + b] + QG[a * 2 + 1] * Q[1 * 2 + b]);
    /* dSigma3D = M^T GS M ; dM = 2 GS M S */
    double G3[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d) v += M[c * 3 + a] * GS[c * 2 + d] * M[d * 3 + b];
            G3[a * 3 + b] = v;
        }
    double GM[6], dM[6];
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k) GM[a * 3 + k] = GS[a * 2 + 0] * M[0 * 3 + k] + GS[a * 2 + 1] * M[1 * 3 + k];
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k) {
            double v = 0.0;
            for (int c = 0; c < 3; ++c) v += GM[a * 3 + c] * S[c * 3 + k];
            dM[a * 3 + k] = 2.0 * v;
        }
    /* dJ = dM W^T = dM Rg */
    double dJ[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += dM[a * 3 + k] * Rg[k * 3 + b];
            dJ[a * 3 + b] = v;
        }
    double dpc[3] = {g[G_PC + 0], g[G_PC + 1], g[G_PC + 2]};
    double z2 = z * z, z3 = z2 * z;
    dpc[0] += dJ[2] * (-fx / z2) + g[G_MU + 0] * fx / z;
    dpc[1] += dJ[5] * (-fy / z2) + g[G_MU + 1] * fy / z;
    dpc[2] += dJ[0] * (-fx / z2) + dJ[2] * (2.0 * fx * x / z3) + dJ[4] * (-fy / z2) +
              dJ[5] * (2.0 * fy * y / z3) - g[G_MU + 0] * fx * x / z2 - g[G_MU + 1] * fy * y / z2;
    /* position: pc = Rg^T (p - tg) */
    for (int a = 0; a < 3; ++a) out[a] += Rg[a * 3 + 0] * dpc[0] + Rg[a * 3 + 1] * dpc[1] + Rg[a * 3 + 2] * dpc[2];
    /* rotation matrix gradient: from Sigma3D and from the normal column */
    double dR[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int c = 0; c < 3; ++c) v += G3[a * 3 + c] * R[c * 3 + b];
            dR[a * 3 + b] = 2.0 * v * s2[b];
        }
    int k = r->axis;
    for (int a = 0; a < 3; ++a)
        dR[a * 3 + k] += Rg[a * 3 + 0] * g[G_NC + 0] + Rg[a * 3 + 1] * g[G_NC + 1] + Rg[a * 3 + 2] * g[G_NC + 2];
    /* scale */
    for (int b = 0; b < 3; ++b) {
        double v = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) v += R[a * 3 + b] * G3[a * 3 + c] * R[c * 3 + b];
        out[3 + b] += 2.0 * (double)s[b] * v;
    }
    /* raw quaternion: R = I + kq M(q), kq = 2/|q|^2 */
    double w = q[0], qx = q[1], qy = q[2], qz = q[3];
    double n2 = w * w + qx * qx + qy * qy + qz * qz, kq = 2.0 / n2;
    double Mq[9] = {-(qy * qy + qz * qz), qx * qy - w * qz, qx * qz + w * qy,
                    qx * qy + w * qz, -(qx * qx + qz * qz), qy * qz - w * qx,
                    qx * qz - w * qy, qy * qz + w * qx, -(qx * qx + qy * qy)};
    double dMw[9] = {0, -qz, qy, qz, 0, -qx, -qy, qx, 0};
    double dMx[9] = {0, qy, qz, qy, -2 * qx, -w, qz, w, -2 * qx};
    double dMy[9] = {-2 * qy, qx, w, qx, 0, qz, -w, qz, -2 * qy};
    double dMz[9] = {-2 * qz, -w, qx, w, -2 * qz, qy, qx, qy, 0};
    const double* dMs[4] = {dMw, dMx, dMy, dMz};
    double qv[4] = {w, qx, qy, qz};
    double gM = 0.0;
    for (int e = 0; e < 9; ++e) gM += dR[e] * Mq[e];
    for (int m = 0; m < 4; ++m) {
        double v = 0.0;
        for (int e = 0; e < 9; ++e) v += dR[e] * dMs[m][e];
        out[6 + m] += kq * (v - 2.0 * qv[m] / n2 * gM);
    }
    out[10] += g[G_AL];
    for (int c = 0; c < 3; ++c) out[11 + c] += g[G_COL + c];
}

/* The same linear map as chain_to_params with every coefficient and every
 * input replaced by its absolute value: for a camera-space error vector
 * bounded componentwise by gabs, the parameter-space error is bounded by the
 * result (|A B| <= |A| |B| at every stage).  Used for the error bounds of
 * orc_backward_bound. */
static void chain_abs_to_params(const orc_params* P, const double* Rg, const orc_rec* r,
                                const float* s, const float* q, const double* gabs, double* out) {
    double R[9], aR[9], aRg[9];
    quat_to_rot(q, R);
    for (int e = 0; e < 9; ++e) { aR[e] = fabs(R[e]); aRg[e] = fabs(Rg[e]); }
    double x = r->pc[0], y = r->pc[1], z = r->pc[2];
    double fx = P->fx, fy = P->fy;
    double s2[3] = {(double)s[0] * s[0], (double)s[1] * s[1], (double)s[2] * s[2]};
    double aS[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += aR[a * 3 + k] * s2[k] * aR[b * 3 + k];
            aS[a * 3 + b] = v;
        }
    double aJ[6] = {fx / z, 0.0, fabs(fx * x) / (z * z), 0.0, fy / z, fabs(fy * y) / (z * z)};
    double aM[6];
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k) {
            double v = 0.0;
            for (int b = 0; b < 3; ++b) v += aJ[a * 3 + b] * aRg[k * 3 + b];
            aM[a * 3 + k] = v;
        }
    double aQ[4] = {fabs(r->conic[0]), fabs(r->conic[1]), fabs(r->conic[1]), fabs(r->conic[2])};
    double aG[4] = {gabs[G_CON + 0], 0.5 * gabs[G_CON + 1], 0.5 * gabs[G_CON + 1], gabs[G_CON + 2]};
    double QG[4], GS[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) QG[a * 2 + b] = aQ[a * 2 + 0] * aG[0 * 2 + b] + aQ[a * 2 + 1] * aG[1 * 2 + b];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) GS[a * 2 + b] = QG[a * 2 + 0] * aQ[0 * 2 + b] + QG[a * 2 + 1] * aQ[1 * 2 + b];
    double G3[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d) v += aM[c * 3 + a] * GS[c * 2 + d] * aM[d * 3 + b];
            G3[a * 3 + b] = v;
        }
    double GM[6], dM[6];
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k) GM[a * 3 + k] = GS[a * 2 + 0] * aM[0 * 3 + k] + GS[a * 2 + 1] * aM[1 * 3 + k];
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k) {
            double v = 0.0;
            for (int c = 0; c < 3; ++c) v += GM[a * 3 + c] * aS[c * 3 + k];
            dM[a * 3 + k] = 2.0 * v;
        }
    double dJ[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += dM[a * 3 + k] * aRg[k * 3 + b];
            dJ[a * 3 + b] = v;
        }
    double z2 = z * z, z3 = z2 * z, ax = fabs(x), ay = fabs(y);
    double dpc[3] = {gabs[G_PC + 0], gabs[G_PC + 1], gabs[G_PC + 2]};
    dpc[0] += dJ[2] * (fx / z2) + gabs[G_MU + 0] * fx / z;
    dpc[1] += dJ[5] * (fy / z2) + gabs[G_MU + 1] * fy / z;
    dpc[2] += dJ[0] * (fx / z2) + dJ[2] * (2.0 * fx * ax / z3) + dJ[4] * (fy / z2) + dJ[5] * (2.0 * fy * ay / z3) +
              gabs[G_MU + 0] * fx * ax / z2 + gabs[G_MU + 1] * fy * ay / z2;
    for (int a = 0; a < 3; ++a) out[a] += aRg[a * 3 + 0] * dpc[0] + aRg[a * 3 + 1] * dpc[1] + aRg[a * 3 + 2] * dpc[2];
    double dR[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int c = 0; c < 3; ++c) v += G3[a * 3 + c] * aR[c * 3 + b];
            dR[a * 3 + b] = 2.0 * v * s2[b];
        }
    int k = r->axis;
    for (int a = 0; a < 3; ++a)
        dR[a * 3 + k] += aRg[a * 3 + 0] * gabs[G_NC + 0] + aRg[a * 3 + 1] * gabs[G_NC + 1] + aRg[a * 3 + 2] * gabs[G_NC + 2];
    for (int b = 0; b < 3; ++b) {
        double v = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) v += aR[a * 3 + b] * G3[a * 3 + c] * aR[c * 3 + b];
        out[3 + b] += 2.0 * fabs((double)s[b]) * v;
    }
    double w = q[0], qx = q[1], qy = q[2], qz = q[3];
    double n2 = w * w + qx * qx + qy * qy + qz * qz, kq = 2.0 / n2;
    double Mq[9] = {-(qy * qy + qz * qz), qx * qy - w * qz, qx * qz + w * qy,
                    qx * qy + w * qz, -(qx * qx + qz * qz), qy * qz - w * qx,
                    qx * qz - w * qy, qy * qz + w * qx, -(qx * qx + qy * qy)};
    double dMw[9] = {0, -qz, qy, qz, 0, -qx, -qy, qx, 0};
    double dMx[9] = {0, qy, qz, qy, -2 * qx, -w, qz, w, -2 * qx};
    double dMy[9] = {-2 * qy, qx, w, qx, 0, qz, -w, qz, -2 * qy};
    double dMz[9] = {-2 * qz, -w, qx, w, -2 * qz, qy, qx, qy, 0};
    const double* dMs[4] = {dMw, dMx, dMy, dMz};
    double qv[4] = {w, qx, qy, qz};
    double gM = 0.0;
    for (int e = 0; e < 9; ++e) gM += dR[e] * fabs(Mq[e]);
    for (int m = 0; m < 4; ++m) {
        double v = 0.0;
        for (int e = 0; e < 9; ++e) v += dR[e] * fabs(dMs[m][e]);
        out[6 + m] += kq * (v + 2.0 * fabs(qv[m]) / n2 * gM);
    }
    out[10] += gabs[G_AL];
    for (int c = 0; c < 3; ++c) out[11 + c] += gabs[G_COL + c];
}

/* Gradients of L = sum_p gC[p].C(p) + gD[p].D(p) over the listed pixels with
 * respect to the parameters of every unstable Gaussian (summed over frames;
 * stable rows are left at zero).  grad_out: N x 14 doubles, overwritten.
 * With bound_out (N x 14, overwritten) also an error bound per entry (see
 * orc_backward_bound). */
static void backward_impl(const orc_params* P, int64_t N, int32_t F, const double* poses,
                          const orc_rec* recs, const float* pos, const float* scale, const float* rot,
                          const float* opacity, const double* color, const uint8_t* unstable,
                          int64_t NP, const int32_t* pix, const double* gC, const double* gD,
                          double gamma, double t_eps, double kappa_thr, double* grad_out, double* bound_out) {
    (void)pos;
    double* acc = (double*)calloc((size_t)F * N * G_N, sizeof(double));
    double* acc_abs = bound_out ? (double*)calloc((size_t)F * N * G_N, sizeof(double)) : NULL;
    double* acc_tr = bound_out ? (double*)calloc((size_t)F * N * G_N, sizeof(double)) : NULL;
    const double t_lim = 2.0 * t_eps;
    const int64_t CH = 4096;
    for (int64_t p0 = 0; p0 < NP; p0 += CH) {
        int64_t p1 = p0 + CH < NP ? p0 + CH : NP;
        contrib_t** lists = (contrib_t**)calloc((size_t)(p1 - p0), sizeof(contrib_t*));
        int64_t* lens = (int64_t*)calloc((size_t)(p1 - p0), sizeof(int64_t));
#pragma omp parallel
        {
            cand_t* buf = NULL;
            int64_t cap = 0;
#pragma omp for schedule(dynamic, 16)
            for (int64_t p = p0; p < p1; ++p) {
                int32_t f = pix[3 * p], px = pix[3 * p + 1], py = pix[3 * p + 2];
                const orc_rec* fr = recs + (size_t)f * N;
                float ux = (float)px + 0.5f, uy = (float)py + 0.5f;
                int64_t n = pixel_list(P, N, fr, ux, uy, &buf, &cap);
                contrib_t* cl = (contrib_t*)calloc((size_t)(n + 1), sizeof(contrib_t));
                double* Tk = (double*)malloc(sizeof(double) * (size_t)(n + 1));
                double* fk = (double*)malloc(sizeof(double) * (size_t)(n + 1));
                double* gk = (double*)malloc(sizeof(double) * (size_t)(n + 1));
                int* ck = (int*)malloc(sizeof(int) * (size_t)(n + 1));
                double* efk = bound_out ? (double*)malloc(sizeof(double) * (size_t)(n + 1)) : NULL;
                double T = 1.0;
                int64_t hitk = -1;
                for (int64_t k = 0; k < n; ++k) {
                    const orc_rec* r = fr + buf[k].gid;
                    if (efk) {
                        /* relative error of the binary32 f of this entry */
                        double dx = (double)ux - r->mu[0], dy = (double)uy - r->mu[1];
                        double Mf = fabs(r->conic[0]) * dx * dx + 2.0 * fabs(r->conic[1] * dx * dy) +
                                    fabs(r->conic[2]) * dy * dy;
                        double hq = 0.5 * (r->cov[0] - r->cov[2]);
                        double rq = sqrt(hq * hq + r->cov[1] * r->cov[1]);
                        double lmax = 0.5 * (r->cov[0] + r->cov[2]) + rq;
                        double lmin = (r->cov[0] * r->cov[2] - r->cov[1] * r->cov[1]) / lmax;
                        if (lmax > kappa_thr * lmin) Mf = dd_value(r, ux, uy);
                        efk[k] = gamma + 2.0 * 0x1p-24 * Mf;
                    }
                    double g = exp(-0.5 * dd_value(r, ux, uy));
                    double fa = (double)opacity[buf[k].gid] * g;
                    ck[k] = fa > 0.99;
                    fk[k] = ck[k] ? 0.99 : fa;
                    gk[k] = g;
                    Tk[k] = T;
                    if (hitk < 0 && dd_decision(r, ux, uy) < r->tau32) hitk = k;
                    T *= 1.0 - fk[k];
                }
                /* error model: amplification of each entry's f error in 1 - f;
                 * eT in front of k (prefix), eA behind k (suffix) */
                double* eTk = NULL;
                double* eAk = NULL;
                if (efk) {
                    eTk = (double*)malloc(sizeof(double) * (size_t)(n + 1));
                    eAk = (double*)malloc(sizeof(double) * (size_t)(n + 1));
                    double acc_f = 0.0;
                    for (int64_t k = 0; k < n; ++k) {
                        eTk[k] = acc_f;
                        acc_f += efk[k] * fk[k] / (1.0 - fk[k]) + 2.0 * 0x1p-24;
                    }
                    double acc_b = 0.0, mx = 0.0;
                    for (int64_t k = n - 1; k >= 0; --k) {
                        eAk[k] = acc_b + mx;
                        acc_b += efk[k] * fk[k] / (1.0 - fk[k]) + 2.0 * 0x1p-24;
                        if (efk[k] > mx) mx = efk[k];
                    }
                }
                /* colour path, back to front; A = colour accumulated behind */
                double A[3] = {0.0, 0.0, 0.0};
                const double* gc = gC + 3 * p;
                /* error bounds: the colour of the entries an early exit may
                 * drop (those reached with T below twice t_eps) and the
                 * resulting bound on the change of every kept entry's g_f */
                double drop[3] = {0.0, 0.0, 0.0};
                if (bound_out && T < t_lim)
                    for (int64_t k = 0; k < n; ++k)
                        if (Tk[k] < t_lim)
                            for (int ch = 0; ch < 3; ++ch)
                                drop[ch] += fabs((double)color[3 * buf[k].gid + ch]) * fk[k] * Tk[k];
                const double gabs = fabs(gc[0]) * drop[0] + fabs(gc[1]) * drop[1] + fabs(gc[2]) * drop[2];
                for (int64_t k = n - 1; k >= 0; --k) {
                    int32_t i = buf[k].gid;
                    const orc_rec* r = fr + i;
                    contrib_t* c = cl + k;
                    c->rec = (int64_t)((size_t)f * N + i);
                    double fv = fk[k];
                    double gf = 0.0;
                    if (efk) {
                        /* error bounds of this entry's terms (see orc_backward_bound) */
                        double rc = efk[k] + eTk[k] + gamma, ro = rc + eAk[k];
                        double Gm = 0.0;
                        for (int ch = 0; ch < 3; ++ch) {
                            double ci = fabs((double)color[3 * i + ch]);
                            Gm += fabs(gc[ch]) * Tk[k] * (ci + fabs(A[ch]));
                            c->e[G_COL + ch] = fabs(gc[ch]) * fv * Tk[k] * rc;
                        }
                        if (!ck[k]) {
                            double dx = (double)ux - r->mu[0], dy = (double)uy - r->mu[1];
                            double hd = 0.5 * fv * Gm * ro;
                            c->e[G_AL] = Gm * gk[k] * ro;
                            c->e[G_MU + 0] = hd * 2.0 * (fabs(r->conic[0] * dx) + fabs(r->conic[1] * dy));
                            c->e[G_MU + 1] = hd * 2.0 * (fabs(r->conic[1] * dx) + fabs(r->conic[2] * dy));
                            c->e[G_CON + 0] = hd * dx * dx;
                            c->e[G_CON + 1] = hd * 2.0 * fabs(dx * dy);
                            c->e[G_CON + 2] = hd * dy * dy;
                        }
                    }
                    for (int ch = 0; ch < 3; ++ch) {
                        double ci = (double)color[3 * i + ch];
                        c->g[G_COL + ch] = gc[ch] * fv * Tk[k];
                        gf += gc[ch] * Tk[k] * (ci - A[ch]);
                        A[ch] = fv * ci + (1.0 - fv) * A[ch];
                    }
                    if (!ck[k]) {
                        c->g[G_AL] = gf * gk[k];
                        double gdd = -0.5 * fv * gf;
                        double dx = (double)ux - r->mu[0], dy = (double)uy - r->mu[1];
                        /* d(dd)/dmu = -2 Q delta */
                        double qd[2];
                        q_delta(r, ux, uy, qd);
                        c->g[G_MU + 0] = gdd * -2.0 * qd[0];
                        c->g[G_MU + 1] = gdd * -2.0 * qd[1];
                        c->g[G_CON + 0] = gdd * dx * dx;
                        c->g[G_CON + 1] = gdd * 2.0 * dx * dy;
                        c->g[G_CON + 2] = gdd * dy * dy;
                    }
                    if (bound_out) {
                        if (gabs > 0.0 && !ck[k]) {
                            /* if kept, the entry's g_f changes by at most
                             * gabs / (1 - f) through the dropped colour */
                            double dg = gabs / (1.0 - fv), hd = 0.5 * fv * dg;
                            double dx = (double)ux - r->mu[0], dy = (double)uy - r->mu[1];
                            c->t[G_AL] = dg * gk[k];
                            c->t[G_MU + 0] = hd * 2.0 * fabs(r->conic[0] * dx + r->conic[1] * dy);
                            c->t[G_MU + 1] = hd * 2.0 * fabs(r->conic[1] * dx + r->conic[2] * dy);
                            c->t[G_CON + 0] = hd * dx * dx;
                            c->t[G_CON + 1] = hd * 2.0 * fabs(dx * dy);
                            c->t[G_CON + 2] = hd * dy * dy;
                        }
                        /* an entry reached below 2 t_eps may also be dropped */
                        if (Tk[k] < t_lim)
                            for (int e = 0; e < G_N; ++e) c->t[e] += fabs(c->g[e]);
                    }
                }
                /* depth path (Eq. 4-5) on the hit Gaussian only */
                int64_t nl = n;
                if (hitk >= 0 && gD[p] != 0.0) {
                    int32_t i = buf[hitk].gid;
                    const orc_rec* r = fr + i;
                    contrib_t* c = cl + n;
                    c->rec = (int64_t)((size_t)f * N + i);
                    double gd = gD[p];
                    if (plane_branch(P, r->nc32, ux, uy)) {
                        double d[3] = {((double)ux - P->cx) / P->fx, ((double)uy - P->cy) / P->fy, 1.0};
                        double dn = r->nc[0] * d[0] + r->nc[1] * d[1] + r->nc[2] * d[2];
                        double D = r->h / dn;
                        for (int a = 0; a < 3; ++a) {
                            c->g[G_PC + a] = gd * r->nc[a] / dn;
                            c->g[G_NC + a] = gd * (r->pc[a] - D * d[a]) / dn;
                        }
                    } else {
                        c->g[G_PC + 2] = gd;
                    }
                    if (bound_out) {
                        for (int e = 0; e < G_N; ++e) c->e[e] = gamma * fabs(c->g[e]);
                        if (plane_branch(P, r->nc32, ux, uy)) {
                            /* the normal term pc - D d is formed from sums of
                             * gd pc / (d.n) and gd D d / (d.n) kept apart:
                             * bound it on their magnitudes */
                            double d[3] = {((double)ux - P->cx) / P->fx, ((double)uy - P->cy) / P->fy, 1.0};
                            double dn = r->nc[0] * d[0] + r->nc[1] * d[1] + r->nc[2] * d[2];
                            double D = r->h / dn;
                            for (int a = 0; a < 3; ++a)
                                c->e[G_NC + a] = gamma * fabs(gd / dn) * (fabs(r->pc[a]) + fabs(D * d[a]));
                        }
                    }
                    nl = n + 1;
                }
                lists[p - p0] = cl;
                lens[p - p0] = nl;
                free(Tk);
                free(fk);
                free(gk);
                free(ck);
                free(efk);
                free(eTk);
                free(eAk);
            }
            free(buf);
        }
        for (int64_t p = p0; p < p1; ++p) {
            contrib_t* cl = lists[p - p0];
            for (int64_t k = 0; k < lens[p - p0]; ++k)
                for (int e = 0; e < G_N; ++e) acc[(size_t)cl[k].rec * G_N + e] += cl[k].g[e];
            if (bound_out)
                for (int64_t k = 0; k < lens[p - p0]; ++k)
                    for (int e = 0; e < G_N; ++e) {
                        acc_abs[(size_t)cl[k].rec * G_N + e] += cl[k].e[e];
                        acc_tr[(size_t)cl[k].rec * G_N + e] += cl[k].t[e];
                    }
            free(cl);
        }
        free(lists);
        free(lens);
    }
    if (N > 0) memset(grad_out, 0, sizeof(double) * 14 * (size_t)N);
    if (bound_out && N > 0) memset(bound_out, 0, sizeof(double) * 14 * (size_t)N);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        if (!unstable[i]) continue;
        for (int32_t f = 0; f < F; ++f) {
            const orc_rec* r = recs + (size_t)f * N + i;
            if (r->culled) continue;
            const double* g = acc + ((size_t)f * N + i) * G_N;
            int any = 0;
            for (int e = 0; e < G_N; ++e) any |= g[e] != 0.0;
            if (bound_out) {
                const double* ga = acc_abs + ((size_t)f * N + i) * G_N;
                const double* gt = acc_tr + ((size_t)f * N + i) * G_N;
                double gb[G_N];
                int anyb = 0;
                for (int e = 0; e < G_N; ++e) {
                    gb[e] = ga[e] + gt[e];
                    anyb |= gb[e] != 0.0;
                }
                if (anyb)
                    chain_abs_to_params(P, poses + (size_t)f * 12, r, scale + 3 * i, rot + 4 * i, gb,
                                        bound_out + 14 * (size_t)i);
            }
            if (!any) continue;
            chain_to_params(P, poses + (size_t)f * 12, r, scale + 3 * i, rot + 4 * i, g,
                            grad_out + 14 * (size_t)i);
        }
    }
    free(acc);
    free(acc_abs);
    free(acc_tr);
}

void orc_backward(const orc_params* P, int64_t N, int32_t F, const double* poses,
                  const orc_rec* recs, const float* pos, const float* scale, const float* rot,
                  const float* opacity, const double* color, const uint8_t* unstable,
                  int64_t NP, const int32_t* pix, const double* gC, const double* gD,
                  double* grad_out) {
    backward_impl(P, N, F, poses, recs, pos, scale, rot, opacity, color, unstable, NP, pix, gC, gD, 0.0, 0.0, 0.0,
                  grad_out, NULL);
}

/* orc_backward plus, per gradient entry, a bound on the error of a binary32
 * evaluation of the same sums that stops each pixel's compositing once its
 * transmission falls below t_eps: the chain rule, in absolute values, of
 * the per-slot sums of each camera-space term's magnitude times its
 * relative error, plus the same map of the terms the early exit may drop
 * (entries reached with T below 2 t_eps) and of the largest change the
 * dropped colour can make to the kept entries' terms.  The relative error
 * model of a pixel's entry k (u = 2^-24):
 *   f_k:    ef = gamma + 2 u M, M the sum of the magnitudes of the quadratic
 *           form's terms at the pixel (its binary32 evaluation errs by about
 *           4 u M, and f by half of that), or d^2 for footprints with
 *           condition number above kappa_thr (evaluated in factored form);
 *   T_k:    eT = sum over entries j in front of ef_j f_j / (1 - f_j) + 2 u
 *           (a relative error e of f_j is one of e f_j / (1 - f_j) in
 *           1 - f_j, which can be large near the opacity clamp);
 *   A_k:    eA = the same sum over the entries behind, plus their largest ef;
 *   terms:  colour terms ef + eT + gamma; the others gamma + ef + eT + eA on
 *           magnitudes that ignore cancellation (|c| + |A| for c - A,
 *           |Q| |u - mu| for Q (u - mu)).
 * bound_out: N x 14 doubles, overwritten. */
void orc_backward_bound(const orc_params* P, int64_t N, int32_t F, const double* poses,
                        const orc_rec* recs, const float* pos, const float* scale, const float* rot,
                        const float* opacity, const double* color, const uint8_t* unstable,
                        int64_t NP, const int32_t* pix, const double* gC, const double* gD, double gamma,
                        double t_eps, double kappa_thr, double* grad_out, double* bound_out) {
    backward_impl(P, N, F, poses, recs, pos, scale, rot, opacity, color, unstable, NP, pix, gC, gD, gamma, t_eps,
                  kappa_thr, grad_out, bound_out);
}
