// Real spherical harmonics to degree 3 for the phase function of a Gaussian
// (Sec. II-B: each Gaussian carries SH coefficients, its phase function is
// the expansion evaluated at the direction towards the radar).
//
// Orthonormal on the unit sphere, without the Condon-Shortley phase; the
// coefficient of degree l and order m (-l..l) sits at index l*l + l + m.
// Each function is a polynomial in the components (x, y, z) of a unit
// vector, so the expansion's gradient is taken with respect to those
// components as independent variables; callers project it onto the sphere
// through the Jacobian of the normalisation.
#pragma once

namespace sdgr {

constexpr int SH_MAX = 16;   // coefficients up to degree 3

// normalisation of each Cartesian form: sqrt((2l + 1) / (4 pi)) with the
// order-dependent factors folded in
constexpr double SH_K0 = 0.28209479177387814;    // 1/2 sqrt(1/pi)
constexpr double SH_K1 = 0.4886025119029199;     // sqrt(3/(4 pi))
constexpr double SH_K2A = 1.0925484305920792;    // 1/2 sqrt(15/pi): xy, yz, xz
constexpr double SH_K2B = 0.31539156525252005;   // 1/4 sqrt(5/pi): 3z^2 - 1
constexpr double SH_K2C = 0.5462742152960396;    // 1/4 sqrt(15/pi): x^2 - y^2
constexpr double SH_K3A = 0.5900435899266435;    // 1/4 sqrt(35/(2 pi)): m = +-3
constexpr double SH_K3B = 2.890611442640554;     // 1/2 sqrt(105/pi): xyz
constexpr double SH_K3C = 0.4570457994644658;    // 1/4 sqrt(21/(2 pi)): m = +-1
constexpr double SH_K3D = 0.3731763325901154;    // 1/4 sqrt(7/pi): m = 0
constexpr double SH_K3E = 1.445305721320277;     // 1/4 sqrt(105/pi): z (x^2 - y^2)

// Y[0 .. n) at the unit vector (x, y, z); n is 1, 4, 9 or 16.
template <class T>
__device__ __forceinline__ void sh_basis(T x, T y, T z, int n, T* Y)
{
    Y[0] = T(SH_K0);
    if (n <= 1) return;
    Y[1] = T(SH_K1) * y;
    Y[2] = T(SH_K1) * z;
    Y[3] = T(SH_K1) * x;
    if (n <= 4) return;
    const T xx = x * x, yy = y * y, zz = z * z;
    Y[4] = T(SH_K2A) * x * y;
    Y[5] = T(SH_K2A) * y * z;
    Y[6] = T(SH_K2B) * (T(3) * zz - T(1));
    Y[7] = T(SH_K2A) * x * z;
    Y[8] = T(SH_K2C) * (xx - yy);
    if (n <= 9) return;
    Y[9] = T(SH_K3A) * y * (T(3) * xx - yy);
    Y[10] = T(SH_K3B) * x * y * z;
    Y[11] = T(SH_K3C) * y * (T(5) * zz - T(1));
    Y[12] = T(SH_K3D) * z * (T(5) * zz - T(3));
    Y[13] = T(SH_K3C) * x * (T(5) * zz - T(1));
    Y[14] = T(SH_K3E) * z * (xx - yy);
    Y[15] = T(SH_K3A) * x * (xx - T(3) * yy);
}

// Gradient of sum_k c[k] Y_k with respect to (x, y, z), into g[3].
template <class T>
__device__ __forceinline__ void sh_expansion_grad(const T* c, int n, T x, T y, T z, T* g)
{
    T gx = T(0), gy = T(0), gz = T(0);
    if (n > 1) {
        gx += T(SH_K1) * c[3];
        gy += T(SH_K1) * c[1];
        gz += T(SH_K1) * c[2];
    }
    if (n > 4) {
        const T a = T(SH_K2A);
        gx += a * (c[4] * y + c[7] * z) + T(2 * SH_K2C) * c[8] * x;
        gy += a * (c[4] * x + c[5] * z) - T(2 * SH_K2C) * c[8] * y;
        gz += a * (c[5] * y + c[7] * x) + T(6 * SH_K2B) * c[6] * z;
    }
    if (n > 9) {
        const T xx = x * x, yy = y * y, zz = z * z;
        const T p = T(5) * zz - T(1);
        // m = +-3
        gx += T(SH_K3A) * (c[9] * T(6) * x * y + c[15] * T(3) * (xx - yy));
        gy += T(SH_K3A) * (c[9] * T(3) * (xx - yy) - c[15] * T(6) * x * y);
        // xyz
        gx += T(SH_K3B) * c[10] * y * z;
        gy += T(SH_K3B) * c[10] * x * z;
        gz += T(SH_K3B) * c[10] * x * y;
        // m = +-1
        gx += T(SH_K3C) * c[13] * p;
        gy += T(SH_K3C) * c[11] * p;
        gz += T(SH_K3C) * T(10) * z * (c[11] * y + c[13] * x);
        // m = 0
        gz += T(SH_K3D) * c[12] * (T(15) * zz - T(3));
        // z (x^2 - y^2)
        gx += T(SH_K3E) * c[14] * T(2) * x * z;
        gy -= T(SH_K3E) * c[14] * T(2) * y * z;
        gz += T(SH_K3E) * c[14] * (xx - yy);
    }
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
}

}  // namespace sdgr
