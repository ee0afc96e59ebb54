// Kirchhoff-Love / StVK quantities at one quadrature point, in the reduced
// form used by the kernels: the areal energy psi depends on the displacement
// field only through g = (a_1, a_2, a_{1,1}, a_{2,2}, a_{1,2}) in R^15.
//
// Model (Sec. 3.2-3.3 of the paper): A = (a - abar)/2, B = (b - bbar)/2 with
// b_{ab} = a_{a,b} . a_3; psi = (h/2) alpha^T H alpha + (h^3/24) beta^T H beta,
// alpha = (A11, A22, 2A12), beta = 2(B11, B22, 2B12), H the Voigt matrix of
// (lambda/2) abar^{ab} abar^{gd} + mu abar^{bg} abar^{ad} (Appendix B.1).
//
// Strains are formed from displacements u = q - qbar (no cancellation of
// O(1) positions against small strains), which FP32 needs:
//   a_ab - abar_ab = abar_a.u_b + u_a.abar_b + u_a.u_b,
//   n = nbar + dn, dn = abar_1 x u_2 + u_1 x abar_2 + u_1 x u_2,
//   |n| - |nbar| = (2 nbar.dn + dn.dn)/(|n| + |nbar|),
//   a_3 - abar_3 = dn/|n| - nbar (|n| - |nbar|)/(|n| |nbar|),
//   b - bbar = abar_{a,b}.(a_3 - abar_3) + u_{a,b}.a_3.
//
// Derivatives (written here from the definitions; they agree with the
// paper's Appendix B expressions):
//   dpsi/da_1 = s1 a_1 + s3 a_2 + (a_2 x P)/|n|,  dpsi/da_2 = s2 a_2 + s3 a_1 + (P x a_1)/|n|,
//   dpsi/dv_k = mt_k a_3,
// with sigma = h H alpha, m = (h^3/12) H beta, mt = (m1, m2, 2 m3),
// V = sum_k mt_k v_k, P = V - (V.a_3) a_3.  The Hessian blocks are listed in
// hess_blocks() below.
#pragma once
#include "device_common.hpp"

namespace bhem {

template <class T> struct GaussPoint {
    v3<T> a1, a2, v[3], a3, t1, t2;   // deformed tangents, second derivatives, normal, a2 x a3, a3 x a1
    T s;                              // |a_1 x a_2|
    T Hm[3][3], Hb[3][3];             // h H and (h^3/12) H (Voigt)
    T alpha[3], beta[3];
    T sig[3], mom[3];                 // Hm alpha, Hb beta
    T psi;                            // areal energy
    T wq;                             // quadrature weight times sqrt(abar)
};

// kin: [0..14] reference (abar_1, abar_2, vbar_11, vbar_22, vbar_12), [15..29]
// displacement parts (u_1, u_2, u_11, u_22, u_12), all true xi-derivatives.
template <class T>
__device__ __forceinline__ void gauss_point(const T* kin, T w_theta, T lam, T mu, T h, GaussPoint<T>& G) {
    const v3<T> ab1 = mk(kin[0], kin[1], kin[2]), ab2 = mk(kin[3], kin[4], kin[5]);
    const v3<T> u1 = mk(kin[15], kin[16], kin[17]), u2 = mk(kin[18], kin[19], kin[20]);
    v3<T> vb[3], uv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        vb[k] = mk(kin[6 + 3 * k], kin[7 + 3 * k], kin[8 + 3 * k]);
        uv[k] = mk(kin[21 + 3 * k], kin[22 + 3 * k], kin[23 + 3 * k]);
    }
    G.a1 = ab1 + u1;
    G.a2 = ab2 + u2;
#pragma unroll
    for (int k = 0; k < 3; ++k) G.v[k] = vb[k] + uv[k];
    const v3<T> nb = cross(ab1, ab2);
    const v3<T> dn = cross(ab1, u2) + cross(u1, ab2) + cross(u1, u2);
    const v3<T> n = nb + dn;
    const T sb = sqrt(dot(nb, nb));
    G.s = sqrt(dot(n, n));
    G.a3 = (T(1) / G.s) * n;
    const T ds = (T(2) * dot(nb, dn) + dot(dn, dn)) / (G.s + sb);
    const v3<T> da3 = (T(1) / G.s) * dn - (ds / (G.s * sb)) * nb;
    // membrane and bending strains in Voigt form
    G.alpha[0] = dot(ab1, u1) + T(0.5) * dot(u1, u1);
    G.alpha[1] = dot(ab2, u2) + T(0.5) * dot(u2, u2);
    G.alpha[2] = dot(ab1, u2) + dot(u1, ab2) + dot(u1, u2);
    T db[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) db[k] = dot(vb[k], da3) + dot(uv[k], G.a3);
    G.beta[0] = db[0];
    G.beta[1] = db[1];
    G.beta[2] = T(2) * db[2];
    // contravariant reference metric and the Voigt matrix
    const T g11 = dot(ab1, ab1), g22 = dot(ab2, ab2), g12 = dot(ab1, ab2);
    const T det = g11 * g22 - g12 * g12;
    const T c11 = g22 / det, c22 = g11 / det, c12 = -g12 / det;
    const T l2m = lam + T(2) * mu;
    T H[3][3];
    H[0][0] = l2m * c11 * c11;
    H[1][1] = l2m * c22 * c22;
    H[2][2] = (lam + mu) * c12 * c12 + mu * c11 * c22;
    H[0][1] = H[1][0] = lam * c11 * c22 + T(2) * mu * c12 * c12;
    H[0][2] = H[2][0] = l2m * c11 * c12;
    H[1][2] = H[2][1] = l2m * c12 * c22;
    const T hb = h * h * h / T(12);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            G.Hm[i][j] = h * H[i][j];
            G.Hb[i][j] = hb * H[i][j];
        }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        G.sig[i] = G.Hm[i][0] * G.alpha[0] + G.Hm[i][1] * G.alpha[1] + G.Hm[i][2] * G.alpha[2];
        G.mom[i] = G.Hb[i][0] * G.beta[0] + G.Hb[i][1] * G.beta[1] + G.Hb[i][2] * G.beta[2];
    }
    G.psi = T(0.5) * (G.sig[0] * G.alpha[0] + G.sig[1] * G.alpha[1] + G.sig[2] * G.alpha[2] +
                      G.mom[0] * G.beta[0] + G.mom[1] * G.beta[1] + G.mom[2] * G.beta[2]);
    G.t1 = cross(G.a2, G.a3);
    G.t2 = cross(G.a3, G.a1);
    G.wq = w_theta * sb;
}

// dpsi/dg for the 5 kinematic slots (15 values, slot-major).
template <class T> __device__ __forceinline__ void dpsi_dg(const GaussPoint<T>& G, T* out) {
    const T mt[3] = {G.mom[0], G.mom[1], T(2) * G.mom[2]};
    const v3<T> V = mt[0] * G.v[0] + mt[1] * G.v[1] + mt[2] * G.v[2];
    const v3<T> P = V - dot(V, G.a3) * G.a3;
    const T is = T(1) / G.s;
    const v3<T> d1 = G.sig[0] * G.a1 + G.sig[2] * G.a2 + is * cross(G.a2, P);
    const v3<T> d2 = G.sig[1] * G.a2 + G.sig[2] * G.a1 + is * cross(P, G.a1);
    out[0] = d1.x; out[1] = d1.y; out[2] = d1.z;
    out[3] = d2.x; out[4] = d2.y; out[5] = d2.z;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        out[6 + 3 * k] = mt[k] * G.a3.x;
        out[7 + 3 * k] = mt[k] * G.a3.y;
        out[8 + 3 * k] = mt[k] * G.a3.z;
    }
}

// Packed index of entry (r, c), r <= c, of a symmetric 15x15 matrix.
__host__ __device__ constexpr int sym15(int r, int c) { return 15 * r - (r * (r - 1)) / 2 + (c - r); }

// 3x3 block accumulator, stored into the packed matrix with a scale.
template <class T> struct Blk {
    T m[3][3];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) m[i][j] = T(0);
    }
    __device__ __forceinline__ void outer(T c, v3<T> u, v3<T> w) {   // += c u w^T
        const T uu[3] = {u.x, u.y, u.z}, ww[3] = {w.x, w.y, w.z};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) m[i][j] += c * uu[i] * ww[j];
    }
    __device__ __forceinline__ void ident(T c) {
        m[0][0] += c;
        m[1][1] += c;
        m[2][2] += c;
    }
    __device__ __forceinline__ void crossmat(T c, v3<T> a) {   // += c [a], [a] x = a cross x
        m[0][1] -= c * a.z;
        m[0][2] += c * a.y;
        m[1][0] += c * a.z;
        m[1][2] -= c * a.x;
        m[2][0] -= c * a.y;
        m[2][1] += c * a.x;
    }
    __device__ __forceinline__ void store(T* W, int A, int B, T scale) const {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int r = 3 * A + i, c = 3 * B + j;
                if (r <= c) W[sym15(r, c)] = scale * m[i][j];
            }
    }
};

// Hessian d2psi/dg2 (15x15) of one quadrature point in four parts of about
// equal cost (a part is a wavefront's share for four patches, so the branch
// is uniform across the wavefront):
//   part 0: (a1,a1) and (v_0, v_l), l = 0..2;  part 1: (a2,a2) and (v_k, v_l),
//   1 <= k <= l;  part 2: (a1,a2);  part 3: (a_A, v_l), A = 0, 1, l = 0..2.
// Material part: J^T diag(Hm, Hb) J, J = d(alpha, beta)/dg, where
//   d alpha/d a_1 = (a1, 0, a2), d alpha/d a_2 = (0, a2, a1),
//   d beta_k/d a_A = c_k Z-vectors below, d beta_k/d v_k = c_k a3, c = (1,1,2).
// Geometric parts: sigma-weighted identities (membrane); for bending, with
// V = sum_k mt_k v_k, B = V.a3, P = V - B a3, U1 = a2 x P, U2 = P x a1, s = |n|:
//   D11 = -(t1 U1^T + U1 t1^T)/s^2 - (B/s^2)(a22 I - a2 a2^T - t1 t1^T)
//   D22 = -(t2 U2^T + U2 t2^T)/s^2 - (B/s^2)(a11 I - a1 a1^T - t2 t2^T)
//   D12 = -(t1 U2^T + U1 t2^T)/s^2 - (B/s^2)(a1 a2^T - a12 I - t1 t2^T) - [P]/s
// and blocks (a1, v_k) += mt_k ([a2] - t1 a3^T)/s, (a2, v_k) += mt_k (-[a1] - t2 a3^T)/s.
// The pseudo Hessian drops the bending geometric blocks.  Every value is
// multiplied by wq sc[A] sc[B] (sc = slot scales).
template <class T>
__device__ __forceinline__ void hess_blocks(const GaussPoint<T>& G, int part, int pseudo, const T* sc, T* W) {
    const T ck[3] = {T(1), T(1), T(2)};
    const T is = T(1) / G.s;
    const T mt[3] = {G.mom[0], G.mom[1], T(2) * G.mom[2]};
    Blk<T> b;
    if (part <= 1) {
        // (v_k, v_l): part 0 the row k = 0, part 1 the rows k = 1, 2
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = k; l < 3; ++l) {
                if ((k == 0) != (part == 0)) continue;
                b.zero();
                b.outer(G.Hb[k][l] * ck[k] * ck[l], G.a3, G.a3);
                b.store(W, 2 + k, 2 + l, G.wq * sc[2 + k] * sc[2 + l]);
            }
    }
    // Z_k[A] and Y_k[A] = sum_l Hb[k][l] Z_l[A], A = 0 (a1), 1 (a2)
    v3<T> Z[2][3], Y[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T bk = dot(G.v[k], G.a3);
        Z[0][k] = (ck[k] * is) * (cross(G.a2, G.v[k]) - bk * G.t1);
        Z[1][k] = (ck[k] * is) * (cross(G.v[k], G.a1) - bk * G.t2);
    }
#pragma unroll
    for (int A = 0; A < 2; ++A)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            Y[A][k] = G.Hb[k][0] * Z[A][0] + G.Hb[k][1] * Z[A][1] + G.Hb[k][2] * Z[A][2];
    const v3<T> V = mt[0] * G.v[0] + mt[1] * G.v[1] + mt[2] * G.v[2];
    const T Bv = dot(V, G.a3);
    const v3<T> P = V - Bv * G.a3;
    const T is2 = is * is;
    if (part == 0) {
        // (a1, a1)
        b.zero();
        b.outer(G.Hm[0][0], G.a1, G.a1);
        b.outer(G.Hm[0][2], G.a1, G.a2);
        b.outer(G.Hm[0][2], G.a2, G.a1);
        b.outer(G.Hm[2][2], G.a2, G.a2);
#pragma unroll
        for (int k = 0; k < 3; ++k) b.outer(T(1), Z[0][k], Y[0][k]);
        b.ident(G.sig[0]);
        if (!pseudo) {
            const v3<T> U1 = cross(G.a2, P);
            b.outer(-is2, G.t1, U1);
            b.outer(-is2, U1, G.t1);
            b.ident(-Bv * is2 * dot(G.a2, G.a2));
            b.outer(Bv * is2, G.a2, G.a2);
            b.outer(Bv * is2, G.t1, G.t1);
        }
        b.store(W, 0, 0, G.wq * sc[0] * sc[0]);
    } else if (part == 1) {
        // (a2, a2)
        b.zero();
        b.outer(G.Hm[1][1], G.a2, G.a2);
        b.outer(G.Hm[1][2], G.a1, G.a2);
        b.outer(G.Hm[1][2], G.a2, G.a1);
        b.outer(G.Hm[2][2], G.a1, G.a1);
#pragma unroll
        for (int k = 0; k < 3; ++k) b.outer(T(1), Z[1][k], Y[1][k]);
        b.ident(G.sig[1]);
        if (!pseudo) {
            const v3<T> U2 = cross(P, G.a1);
            b.outer(-is2, G.t2, U2);
            b.outer(-is2, U2, G.t2);
            b.ident(-Bv * is2 * dot(G.a1, G.a1));
            b.outer(Bv * is2, G.a1, G.a1);
            b.outer(Bv * is2, G.t2, G.t2);
        }
        b.store(W, 1, 1, G.wq * sc[1] * sc[1]);
    } else if (part == 2) {
        // (a1, a2)
        b.zero();
        b.outer(G.Hm[0][1], G.a1, G.a2);
        b.outer(G.Hm[0][2], G.a1, G.a1);
        b.outer(G.Hm[1][2], G.a2, G.a2);
        b.outer(G.Hm[2][2], G.a2, G.a1);
#pragma unroll
        for (int k = 0; k < 3; ++k) b.outer(T(1), Z[0][k], Y[1][k]);
        b.ident(G.sig[2]);
        if (!pseudo) {
            const v3<T> U1 = cross(G.a2, P), U2 = cross(P, G.a1);
            b.outer(-is2, G.t1, U2);
            b.outer(-is2, U1, G.t2);
            b.outer(-Bv * is2, G.a1, G.a2);
            b.ident(Bv * is2 * dot(G.a1, G.a2));
            b.outer(Bv * is2, G.t1, G.t2);
            b.crossmat(-is, P);
        }
        b.store(W, 0, 1, G.wq * sc[0] * sc[1]);
    } else {
        // (a_A, v_l)
#pragma unroll
        for (int A = 0; A < 2; ++A)
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                b.zero();
                b.outer(ck[l], Y[A][l], G.a3);
                if (!pseudo) {
                    const T c = mt[l] * is;
                    if (A == 0) {
                        b.crossmat(c, G.a2);
                        b.outer(-c, G.t1, G.a3);
                    } else {
                        b.crossmat(-c, G.a1);
                        b.outer(-c, G.t2, G.a3);
                    }
                }
                b.store(W, A, 2 + l, G.wq * sc[A] * sc[2 + l]);
            }
    }
}

}  // namespace bhem
