// View-dependent colour (Sec. 3.1: the colour c_i of Eq. 1 from the
// Gaussian's SH coefficients and its view direction): the orthonormal real
// spherical harmonics up to degree 3 in their Cartesian forms on the unit
// sphere (no Condon-Shortley sign; the l = 1 forms are proportional to y, z
// and x), index k = l^2 + l + m, evaluated in binary64.
#pragma once

namespace rtg {

constexpr double kShC0 = 0.28209479177387814;   // 1 / (2 sqrt(pi))
constexpr double kShC1 = 0.4886025119029199;    // sqrt(3 / (4 pi))
constexpr double kShC2a = 1.0925484305920792;   // sqrt(15 / pi) / 2
constexpr double kShC2b = 0.31539156525252005;  // sqrt(5 / pi) / 4
constexpr double kShC2c = 0.5462742152960396;   // sqrt(15 / pi) / 4
constexpr double kShC3a = 0.5900435899266435;   // sqrt(35 / (2 pi)) / 4
constexpr double kShC3b = 2.890611442640554;    // sqrt(105 / pi) / 2
constexpr double kShC3c = 0.4570457994644658;   // sqrt(21 / (2 pi)) / 4
constexpr double kShC3d = 0.3731763325901154;   // sqrt(7 / pi) / 4
constexpr double kShC3e = 1.445305721320277;    // sqrt(105 / pi) / 4

// fn(k, Y_k(x, y, z)) for k < (degree + 1)^2 of a unit vector.
template <typename Fn>
__device__ __forceinline__ void sh_basis(int degree, double x, double y, double z, Fn fn) {
    fn(0, kShC0);
    if (degree < 1) return;
    fn(1, kShC1 * y);
    fn(2, kShC1 * z);
    fn(3, kShC1 * x);
    if (degree < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    fn(4, kShC2a * x * y);
    fn(5, kShC2a * y * z);
    fn(6, kShC2b * (3.0 * zz - 1.0));
    fn(7, kShC2a * x * z);
    fn(8, kShC2c * (xx - yy));
    if (degree < 3) return;
    fn(9, kShC3a * y * (3.0 * xx - yy));
    fn(10, kShC3b * x * y * z);
    fn(11, kShC3c * y * (5.0 * zz - 1.0));
    fn(12, kShC3d * z * (5.0 * zz - 3.0));
    fn(13, kShC3c * x * (5.0 * zz - 1.0));
    fn(14, kShC3e * z * (xx - yy));
    fn(15, kShC3a * x * (xx - 3.0 * yy));
}

// fn(k, dY_k/dx, dY_k/dy, dY_k/dz) of the same polynomial forms (only the
// part tangent to the sphere matters to a caller); k = 0 has none.
template <typename Fn>
__device__ __forceinline__ void sh_basis_grad(int degree, double x, double y, double z, Fn fn) {
    if (degree < 1) return;
    fn(1, 0.0, kShC1, 0.0);
    fn(2, 0.0, 0.0, kShC1);
    fn(3, kShC1, 0.0, 0.0);
    if (degree < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    fn(4, kShC2a * y, kShC2a * x, 0.0);
    fn(5, 0.0, kShC2a * z, kShC2a * y);
    fn(6, 0.0, 0.0, 6.0 * kShC2b * z);
    fn(7, kShC2a * z, 0.0, kShC2a * x);
    fn(8, 2.0 * kShC2c * x, -2.0 * kShC2c * y, 0.0);
    if (degree < 3) return;
    fn(9, 6.0 * kShC3a * x * y, kShC3a * (3.0 * xx - 3.0 * yy), 0.0);
    fn(10, kShC3b * y * z, kShC3b * x * z, kShC3b * x * y);
    fn(11, 0.0, kShC3c * (5.0 * zz - 1.0), 10.0 * kShC3c * y * z);
    fn(12, 0.0, 0.0, kShC3d * (15.0 * zz - 3.0));
    fn(13, kShC3c * (5.0 * zz - 1.0), 0.0, 10.0 * kShC3c * x * z);
    fn(14, 2.0 * kShC3e * x * z, -2.0 * kShC3e * y * z, kShC3e * (xx - yy));
    fn(15, kShC3a * (3.0 * xx - 3.0 * yy), -6.0 * kShC3a * x * y, 0.0);
}

}  // namespace rtg
