// Device-side building blocks shared by the gfx950 kernels of libbhem.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bhem {

// ------------------------------------------------------------ per-shell data
// Material and grid constants of one shell, as the kernels use them.
struct ShellParams {
    double dxi1, dxi2;
    double lam, mu, h;       // plane-stress lambda = Y nu/(1 - nu^2), mu = Y/(2(1 + nu)), thickness
    double rho_h;            // areal density
    double grav[3];
    double damp;             // mass-proportional Rayleigh coefficient alpha [1/s]
    int32_t node_begin, node_end;
    int32_t patch_begin, patch_end;
};

// 4-point Gauss-Legendre rule on [0, 1] (the paper's 16-point cell rule is
// its tensor product): abscissae 1/2 -+ x/2 with x = sqrt(3/7 -+ (2/7)sqrt(6/5)),
// weights (18 -+ sqrt 30)/72.  Values to 17 significant digits.
__host__ __device__ constexpr double gauss_theta(int k) {
    return k == 0 ? 0.069431844202973713 : k == 1 ? 0.33000947820757187 : k == 2 ? 0.66999052179242813
                                                                                : 0.93056815579702629;
}
__host__ __device__ constexpr double gauss_weight(int k) {
    return (k == 0 || k == 3) ? 0.17392742256872693 : 0.32607257743127307;
}

// Cubic Hermite functions on [0,1] in factored form, index (p, r): p = end
// (0 at theta = 0, 1 at theta = 1), r = 0 value / 1 slope.  order = 0, 1, 2
// gives the function, its first or its second theta-derivative.
__host__ __device__ inline double hermite(int p, int r, int order, double t) {
    const double u = 1.0 - t;
    if (p == 0 && r == 0) return order == 0 ? (1 + 2 * t) * u * u : order == 1 ? 6 * t * (t - 1) : 12 * t - 6;
    if (p == 0 && r == 1) return order == 0 ? t * u * u : order == 1 ? u * (1 - 3 * t) : 6 * t - 4;
    if (p == 1 && r == 0) return order == 0 ? t * t * (3 - 2 * t) : order == 1 ? 6 * t * u : 6 - 12 * t;
    return order == 0 ? t * t * (t - 1) : order == 1 ? t * (3 * t - 2) : 6 * t - 2;
}

// Slots of the reduced kinematic vector at a quadrature point:
// 0 a_1, 1 a_2, 2 a_{1,1}, 3 a_{2,2}, 4 a_{1,2}, 5 x (value).
// Derivative orders (d1, d2) per slot:
__host__ __device__ constexpr int slot_d1(int a) { return a == 0 ? 1 : a == 2 ? 2 : a == 4 ? 1 : 0; }
__host__ __device__ constexpr int slot_d2(int a) { return a == 1 ? 1 : a == 3 ? 2 : a == 4 ? 1 : 0; }

// theta-space basis table: phi[g][a][I] = d^{d1} w_{p,r}(t1_g) d^{d2} w_{q,s}(t2_g),
// gp g = g1 + 4 g2, slot a, local coordinate I = 4c + k, c = p + 2q, k = r + 2s.
// Built once on the host into device memory (16*6*16 doubles).
inline void build_theta_basis(double* phi) {
    for (int g = 0; g < 16; ++g)
        for (int a = 0; a < 6; ++a)
            for (int I = 0; I < 16; ++I) {
                int c = I >> 2, k = I & 3;
                int p = c & 1, q = c >> 1, r = k & 1, s = k >> 1;
                phi[(g * 6 + a) * 16 + I] = hermite(p, r, slot_d1(a), gauss_theta(g & 3)) *
                                            hermite(q, s, slot_d2(a), gauss_theta(g >> 2));
            }
}

// --------------------------------------------------------------- 3-vectors
template <class T> struct v3 {
    T x, y, z;
};
template <class T> __device__ __forceinline__ v3<T> mk(T x, T y, T z) { return v3<T>{x, y, z}; }
template <class T> __device__ __forceinline__ v3<T> operator+(v3<T> a, v3<T> b) {
    return {a.x + b.x, a.y + b.y, a.z + b.z};
}
template <class T> __device__ __forceinline__ v3<T> operator-(v3<T> a, v3<T> b) {
    return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class T> __device__ __forceinline__ v3<T> operator*(T s, v3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> __device__ __forceinline__ T dot(v3<T> a, v3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> __device__ __forceinline__ v3<T> cross(v3<T> a, v3<T> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> __device__ __forceinline__ T cmp(const v3<T>& a, int i) { return i == 0 ? a.x : i == 1 ? a.y : a.z; }

// ------------------------------------------------------------ MFMA 16x16x4
// One 16x16x4 matrix-core product D += A B per wavefront.  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16].  The accumulator element v of lane l is
// D[row][l%16] with row = (l/16) + 4v for f64 and 4(l/16) + v for f32
// (checked on gfx950).
template <class T> struct Mfma;
template <> struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Scale of local coordinate kind k (r, s) = (k&1, k>>1) for xi-derivative DOFs:
// dxi1^r dxi2^s.
__device__ __forceinline__ double kind_scale(int k, double d1, double d2) {
    return ((k & 1) ? d1 : 1.0) * ((k & 2) ? d2 : 1.0);
}
// Scale of slot a: the theta-derivative divided by dxi1^{d1} dxi2^{d2}.
__device__ __forceinline__ double slot_scale(int a, double d1, double d2) {
    double s = 1.0;
    for (int i = 0; i < slot_d1(a); ++i) s *= d1;
    for (int i = 0; i < slot_d2(a); ++i) s *= d2;
    return 1.0 / s;
}

}  // namespace bhem
