// BHEM CPU oracle -- TEST INFRASTRUCTURE ONLY (see bhem_oracle.hpp).
//
// Per-patch energy, gradient and Hessian written term by term from the paper:
//   kinematics and fundamental forms      Sec. 3.1-3.2
//   StVK Kirchhoff-Love energy density    Sec. 3.3, Eq. for the areal density
//   Voigt form, gradient                  Appendix B.1, Eq. (matrix)
//   exact Hessian, D matrices, pseudo     Appendix B.2
//   mass matrix and areal gravity         Sec. 4.3, Eq. (mass); "External Forces"
// Quadrature is the 16-point rule of Appendix A.2 applied to each patch.
#include "bhem_oracle.hpp"

#include <cstring>

namespace orc {

void hermite_1d(double t, double w[2][2], double d1[2][2], double d2[2][2]) {
    // f(t) = 2t^3 - 3t^2 + 1, g(t) = t^3 - 2t^2 + t   (Appendix A.1)
    auto f = [](double x) { return 2 * x * x * x - 3 * x * x + 1; };
    auto g = [](double x) { return x * x * x - 2 * x * x + x; };
    auto fp = [](double x) { return 6 * x * x - 6 * x; };
    auto gp = [](double x) { return 3 * x * x - 4 * x + 1; };
    auto fpp = [](double x) { return 12 * x - 6; };
    auto gpp = [](double x) { return 6 * x - 4; };
    // w_{p,r}: (0,0) f(t); (1,0) f(1-t); (0,1) g(t); (1,1) -g(1-t)
    w[0][0] = f(t);
    w[1][0] = f(1 - t);
    w[0][1] = g(t);
    w[1][1] = -g(1 - t);
    // w'_{p,r}: f'(t); -f'(1-t); g'(t); g'(1-t)
    d1[0][0] = fp(t);
    d1[1][0] = -fp(1 - t);
    d1[0][1] = gp(t);
    d1[1][1] = gp(1 - t);
    // w''_{p,r}: f''(t); f''(1-t); g''(t); -g''(1-t)
    d2[0][0] = fpp(t);
    d2[1][0] = fpp(1 - t);
    d2[0][1] = gpp(t);
    d2[1][1] = -gpp(1 - t);
}

void shape_functions(double t1, double t2, double dxi1, double dxi2, double out[6][16]) {
    double w1[2][2], a1[2][2], b1[2][2], w2[2][2], a2[2][2], b2[2][2];
    hermite_1d(t1, w1, a1, b1);
    hermite_1d(t2, w2, a2, b2);
    for (int c = 0; c < 4; ++c) {
        int p = c & 1, q = c >> 1;
        for (int k = 0; k < 4; ++k) {
            int r = k & 1, s = k >> 1;
            double scale = (r ? dxi1 : 1.0) * (s ? dxi2 : 1.0);
            int I = 4 * c + k;
            out[0][I] = scale * w1[p][r] * w2[q][s];
            out[1][I] = scale * a1[p][r] * w2[q][s] / dxi1;
            out[2][I] = scale * w1[p][r] * a2[q][s] / dxi2;
            out[3][I] = scale * b1[p][r] * w2[q][s] / (dxi1 * dxi1);
            out[4][I] = scale * w1[p][r] * b2[q][s] / (dxi2 * dxi2);
            out[5][I] = scale * a1[p][r] * a2[q][s] / (dxi1 * dxi2);
        }
    }
}

void gauss4(double theta[4], double weight[4]) {
    // Appendix A.2: offsets sqrt(3/7 -+ (2/7) sqrt(6/5)) of half a cell from
    // its centre; inner weight (18 + sqrt 30)/72, outer (18 - sqrt 30)/72.
    double xin = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    double xout = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    double win = (18.0 + std::sqrt(30.0)) / 72.0;
    double wout = (18.0 - std::sqrt(30.0)) / 72.0;
    theta[0] = 0.5 - 0.5 * xout;
    theta[1] = 0.5 - 0.5 * xin;
    theta[2] = 0.5 + 0.5 * xin;
    theta[3] = 0.5 + 0.5 * xout;
    weight[0] = wout;
    weight[1] = win;
    weight[2] = win;
    weight[3] = wout;
}

namespace {

template <class T> V3<T> combine(const double* phi, const T* q) {
    V3<T> r{T(0), T(0), T(0)};
    for (int I = 0; I < 16; ++I) {
        r.x += phi[I] * q[3 * I + 0];
        r.y += phi[I] * q[3 * I + 1];
        r.z += phi[I] * q[3 * I + 2];
    }
    return r;
}

// Geometry of the midsurface at one quadrature point (Sec. 3.1-3.2).
template <class T> struct Geo {
    V3<T> a[2];      // a_alpha = dx/dxi^alpha
    V3<T> d[2][2];   // a_{alpha,beta} = d2x / dxi^alpha dxi^beta
    V3<T> a3;        // unit normal
    T sqrta;         // |a_1 x a_2|
    T ab[2][2];      // a_{alpha beta} = a_alpha . a_beta (first fundamental form)
    T bb[2][2];      // b_{alpha beta} = a_{alpha,beta} . a_3 (second fundamental form)
};

template <class T> Geo<T> geometry(const double phi[6][16], const T* q) {
    Geo<T> g;
    g.a[0] = combine(phi[1], q);
    g.a[1] = combine(phi[2], q);
    g.d[0][0] = combine(phi[3], q);
    g.d[1][1] = combine(phi[4], q);
    g.d[0][1] = combine(phi[5], q);
    g.d[1][0] = g.d[0][1];
    V3<T> n = cross(g.a[0], g.a[1]);
    g.sqrta = asqrt(dot(n, n));
    g.a3 = (T(1) / g.sqrta) * n;
    for (int al = 0; al < 2; ++al)
        for (int be = 0; be < 2; ++be) {
            g.ab[al][be] = dot(g.a[al], g.a[be]);
            g.bb[al][be] = dot(g.d[al][be], g.a3);
        }
    return g;
}

// Contravariant metric abar^{alpha beta} = (abar_{alpha beta})^{-1}.
void inverse2(const double m[2][2], double inv[2][2]) {
    double det = m[0][0] * m[1][1] - m[0][1] * m[1][0];
    inv[0][0] = m[1][1] / det;
    inv[1][1] = m[0][0] / det;
    inv[0][1] = -m[0][1] / det;
    inv[1][0] = -m[1][0] / det;
}

// The Voigt matrix H of Appendix B.1, entry by entry as printed.
void voigt_h(double lam, double mu, const double ai[2][2], double H[3][3]) {
    H[0][0] = (lam + 2 * mu) * ai[0][0] * ai[0][0];
    H[0][1] = lam * ai[0][0] * ai[1][1] + 2 * mu * ai[0][1] * ai[0][1];
    H[0][2] = (lam + 2 * mu) * ai[0][0] * ai[0][1];
    H[1][1] = (lam + 2 * mu) * ai[1][1] * ai[1][1];
    H[1][2] = (lam + 2 * mu) * ai[0][1] * ai[1][1];
    H[2][2] = (lam + mu) * ai[0][1] * ai[0][1] + mu * ai[0][0] * ai[1][1];
    H[1][0] = H[0][1];
    H[2][0] = H[0][2];
    H[2][1] = H[1][2];
}

// Everything the three per-patch quantities need at one quadrature point.
struct QPoint {
    double phi[6][16];
    double weight;   // product Gauss weight times dxi1 dxi2
};

void quad_points(const Shell& s, QPoint qp[16]) {
    double th[4], wt[4];
    gauss4(th, wt);
    for (int g2 = 0; g2 < 4; ++g2)
        for (int g1 = 0; g1 < 4; ++g1) {
            QPoint& p = qp[g1 + 4 * g2];
            shape_functions(th[g1], th[g2], s.dxi1, s.dxi2, p.phi);
            p.weight = wt[g1] * s.dxi1 * wt[g2] * s.dxi2;
        }
}

}  // namespace

// Areal energy density of Sec. 3.3 in tensor form:
//   V = (A_ab A_gd h + (1/3) B_ab B_gd h^3) Hbar^{abgd},
//   Hbar^{abgd} = (lambda/2) abar^{ab} abar^{gd} + mu abar^{bg} abar^{ad},
// integrated against dOmega-bar = sqrt(abar) dxi1 dxi2.
template <class T> T patch_energy_tensor(const Shell& s, const T* q, const double* qb) {
    QPoint qp[16];
    quad_points(s, qp);
    const double lam = lame_lambda(s), mu = lame_mu(s), h = s.thickness;
    T energy = T(0);
    for (int g = 0; g < 16; ++g) {
        Geo<T> cur = geometry<T>(qp[g].phi, q);
        Geo<double> ref = geometry<double>(qp[g].phi, qb);
        double ai[2][2];
        inverse2(ref.ab, ai);
        T A[2][2], B[2][2];
        for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be) {
                A[al][be] = (cur.ab[al][be] - ref.ab[al][be]) * 0.5;
                B[al][be] = (cur.bb[al][be] - ref.bb[al][be]) * 0.5;
            }
        T dens = T(0);
        for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be)
                for (int ga = 0; ga < 2; ++ga)
                    for (int de = 0; de < 2; ++de) {
                        double Hb = 0.5 * lam * ai[al][be] * ai[ga][de] + mu * ai[be][ga] * ai[al][de];
                        dens += (A[al][be] * A[ga][de] * h + B[al][be] * B[ga][de] * (h * h * h / 3.0)) * Hb;
                    }
        energy += dens * (qp[g].weight * ref.sqrta);
    }
    return energy;
}

// Same energy through the Voigt quantities of Appendix B.1:
//   psi = (h/2) alpha^T H alpha + (h^3/24) beta^T H beta,
//   alpha = (A11, A22, 2A12), beta = 2 (B11, B22, 2B12).
template <class T> T patch_energy_voigt(const Shell& s, const T* q, const double* qb) {
    QPoint qp[16];
    quad_points(s, qp);
    const double lam = lame_lambda(s), mu = lame_mu(s), h = s.thickness;
    T energy = T(0);
    for (int g = 0; g < 16; ++g) {
        Geo<T> cur = geometry<T>(qp[g].phi, q);
        Geo<double> ref = geometry<double>(qp[g].phi, qb);
        double ai[2][2], H[3][3];
        inverse2(ref.ab, ai);
        voigt_h(lam, mu, ai, H);
        T al[3] = {(cur.ab[0][0] - ref.ab[0][0]) * 0.5, (cur.ab[1][1] - ref.ab[1][1]) * 0.5,
                   (cur.ab[0][1] - ref.ab[0][1])};
        T be[3] = {(cur.bb[0][0] - ref.bb[0][0]), (cur.bb[1][1] - ref.bb[1][1]),
                   2.0 * (cur.bb[0][1] - ref.bb[0][1])};
        T quad_a = T(0), quad_b = T(0);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                quad_a += al[i] * H[i][j] * al[j];
                quad_b += be[i] * H[i][j] * be[j];
            }
        T psi = quad_a * (0.5 * h) + quad_b * (h * h * h / 24.0);
        energy += psi * (qp[g].weight * ref.sqrta);
    }
    return energy;
}

namespace {

// d b_{alpha beta} / d q_I for one second-derivative vector v = a_{alpha,beta}
// and the basis values (phi_ab = Phi^I_{,alpha beta}, p1 = Phi^I_{,1},
// p2 = Phi^I_{,2}), Appendix B.1 Eq. (pbabpqi).
template <class T>
V3<T> db_dq(const Geo<T>& g, const V3<T>& v, double phi_ab, double p1, double p2) {
    V3<T> t1 = cross(g.a[1], g.a3);   // a_2 x a_3
    V3<T> t2 = cross(g.a3, g.a[0]);   // a_3 x a_1
    T vb = dot(v, g.a3);
    V3<T> inner = p1 * cross(g.a[1], v) + p2 * cross(v, g.a[0]) - vb * (p1 * t1 + p2 * t2);
    return phi_ab * g.a3 + (T(1) / g.sqrta) * inner;
}

}  // namespace

// Gradient of the elastic energy, Appendix B.1 Eq. (matrix):
//   dV/dq_I = sum_gp [ h (d alpha/d q_I)^T H alpha
//                      + (h^3/12) (d beta/d q_I)^T H beta ] sqrt(abar) w_gp
// with d a_{ab}/d q_I = Phi^I_{,a} a_b + Phi^I_{,b} a_a (Eq. paabpqi).
template <class T> void patch_gradient(const Shell& s, const T* q, const double* qb, T* grad) {
    QPoint qp[16];
    quad_points(s, qp);
    const double lam = lame_lambda(s), mu = lame_mu(s), h = s.thickness;
    for (int i = 0; i < 48; ++i) grad[i] = T(0);
    for (int g = 0; g < 16; ++g) {
        const auto& phi = qp[g].phi;
        Geo<T> cur = geometry<T>(phi, q);
        Geo<double> ref = geometry<double>(phi, qb);
        double ai[2][2], H[3][3];
        inverse2(ref.ab, ai);
        voigt_h(lam, mu, ai, H);
        T al[3] = {(cur.ab[0][0] - ref.ab[0][0]) * 0.5, (cur.ab[1][1] - ref.ab[1][1]) * 0.5,
                   (cur.ab[0][1] - ref.ab[0][1])};
        T be[3] = {(cur.bb[0][0] - ref.bb[0][0]), (cur.bb[1][1] - ref.bb[1][1]),
                   2.0 * (cur.bb[0][1] - ref.bb[0][1])};
        T Ha[3], Hbeta[3];
        for (int i = 0; i < 3; ++i) {
            Ha[i] = T(0);
            Hbeta[i] = T(0);
            for (int j = 0; j < 3; ++j) {
                Ha[i] += H[i][j] * al[j];
                Hbeta[i] += H[i][j] * be[j];
            }
        }
        double wq = qp[g].weight * ref.sqrta;
        for (int I = 0; I < 16; ++I) {
            double p1 = phi[1][I], p2 = phi[2][I];
            // d a_11, d a_22, d a_12 (Eq. paabpqi)
            V3<T> da11 = p1 * cur.a[0] + p1 * cur.a[0];
            V3<T> da22 = p2 * cur.a[1] + p2 * cur.a[1];
            V3<T> da12 = p1 * cur.a[1] + p2 * cur.a[0];
            V3<T> dalpha[3] = {0.5 * da11, 0.5 * da22, 0.5 * (2.0 * da12)};
            V3<T> db11 = db_dq(cur, cur.d[0][0], phi[3][I], p1, p2);
            V3<T> db22 = db_dq(cur, cur.d[1][1], phi[4][I], p1, p2);
            V3<T> db12 = db_dq(cur, cur.d[0][1], phi[5][I], p1, p2);
            V3<T> dbeta[3] = {db11, db22, 2.0 * db12};
            V3<T> gI{T(0), T(0), T(0)};
            for (int i = 0; i < 3; ++i) gI = gI + (h * Ha[i]) * dalpha[i] + ((h * h * h / 12.0) * Hbeta[i]) * dbeta[i];
            grad[3 * I + 0] += wq * gI.x;
            grad[3 * I + 1] += wq * gI.y;
            grad[3 * I + 2] += wq * gI.z;
        }
    }
}

namespace {

typedef double M3[3][3];

void m3_zero(M3 m) { std::memset(m, 0, sizeof(M3)); }
void outer(const V3<double>& u, const V3<double>& v, double s, M3 m) {   // m += s u v^T
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) m[r][c] += s * compc(u, r) * compc(v, c);
}
void add_identity(double s, M3 m) {
    for (int r = 0; r < 3; ++r) m[r][r] += s;
}
void add_crossmat(const V3<double>& v, double s, M3 m) {   // m += s [v]
    m[0][1] += -s * v.z;
    m[0][2] += s * v.y;
    m[1][0] += s * v.z;
    m[1][2] += -s * v.x;
    m[2][0] += -s * v.y;
    m[2][1] += s * v.x;
}

// d a_3 / d q_I (Appendix B.2):
//   (1/sqrt a) ( -Phi_{,1}[a_2] + Phi_{,2}[a_1] - a_3 (x) (Phi_{,1} t_1 + Phi_{,2} t_2) )
void da3_dq(const Geo<double>& g, double p1, double p2, M3 out) {
    V3<double> t1 = cross(g.a[1], g.a3), t2 = cross(g.a3, g.a[0]);
    m3_zero(out);
    add_crossmat(g.a[1], -p1, out);
    add_crossmat(g.a[0], p2, out);
    outer(g.a3, p1 * t1 + p2 * t2, -1.0, out);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) out[r][c] /= g.sqrta;
}

// D^{11}, D^{22}, D^{12}, D^{21} of Appendix B.2 for one second-derivative
// vector v = a_{alpha,beta}; the scalar written beta_{alpha beta} in front of
// the first bracket is read as b_{alpha beta} = v . a_3 of the deformed surface.
void d_matrices(const Geo<double>& g, const V3<double>& v, M3 D11, M3 D22, M3 D12, M3 D21) {
    const V3<double>& a1 = g.a[0];
    const V3<double>& a2 = g.a[1];
    V3<double> t1 = cross(a2, g.a3), t2 = cross(g.a3, a1);
    V3<double> s1 = cross(v, a1), s2 = cross(a2, v);
    double b = dot(v, g.a3);
    double a = g.sqrta * g.sqrta;
    double a11 = g.ab[0][0], a22 = g.ab[1][1], a12 = g.ab[0][1];
    m3_zero(D11);
    m3_zero(D22);
    m3_zero(D12);
    m3_zero(D21);
    // D11 = (1/a)( b (3 t1 t1 + a2 a2 - a22 I) - s2 t1 - t1 s2 )
    outer(t1, t1, 3 * b, D11);
    outer(a2, a2, b, D11);
    add_identity(-b * a22, D11);
    outer(s2, t1, -1, D11);
    outer(t1, s2, -1, D11);
    // D22 = (1/a)( b (3 t2 t2 + a1 a1 - a11 I) - s1 t2 - t2 s1 )
    outer(t2, t2, 3 * b, D22);
    outer(a1, a1, b, D22);
    add_identity(-b * a11, D22);
    outer(s1, t2, -1, D22);
    outer(t2, s1, -1, D22);
    // D12 = (1/a)( b (3 t1 t2 - 2 a1 a2 + a2 a1 + a12 I) - s2 t2 - t1 s1 - sqrt(a) [v] )
    outer(t1, t2, 3 * b, D12);
    outer(a1, a2, -2 * b, D12);
    outer(a2, a1, b, D12);
    add_identity(b * a12, D12);
    outer(s2, t2, -1, D12);
    outer(t1, s1, -1, D12);
    add_crossmat(v, -g.sqrta, D12);
    // D21 = (1/a)( b (3 t2 t1 - 2 a2 a1 + a1 a2 + a12 I) - s1 t1 - t2 s2 + sqrt(a) [v] )
    outer(t2, t1, 3 * b, D21);
    outer(a2, a1, -2 * b, D21);
    outer(a1, a2, b, D21);
    add_identity(b * a12, D21);
    outer(s1, t1, -1, D21);
    outer(t2, s2, -1, D21);
    add_crossmat(v, g.sqrta, D21);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            D11[r][c] /= a;
            D22[r][c] /= a;
            D12[r][c] /= a;
            D21[r][c] /= a;
        }
}

}  // namespace

// Exact Hessian (Appendix B.2):
//   d2V/dq_J dq_I = sum_gp ( h G1 + (h^3/12) G2 ) sqrt(abar) w_gp,
//   G1 = (dalpha/dq_I)^T H (dalpha/dq_J) + sum_ij d2 alpha_i/dq_J dq_I H^{ij} alpha_j,
//   G2 = (dbeta/dq_I)^T H (dbeta/dq_J) + sum_ij d2 beta_i/dq_J dq_I H^{ij} beta_j.
// Block (I,J): rows are the components of q_I, columns those of q_J.  The
// pseudo Hessian drops the sum over d2 beta_i (end of Appendix B.2).
void patch_hessian(const Shell& s, const double* q, const double* qb, int pseudo, double* hess) {
    QPoint qp[16];
    quad_points(s, qp);
    const double lam = lame_lambda(s), mu = lame_mu(s), h = s.thickness;
    for (int i = 0; i < 48 * 48; ++i) hess[i] = 0.0;
    for (int g = 0; g < 16; ++g) {
        const auto& phi = qp[g].phi;
        Geo<double> cur = geometry<double>(phi, q);
        Geo<double> ref = geometry<double>(phi, qb);
        double ai[2][2], H[3][3];
        inverse2(ref.ab, ai);
        voigt_h(lam, mu, ai, H);
        double al[3] = {(cur.ab[0][0] - ref.ab[0][0]) * 0.5, (cur.ab[1][1] - ref.ab[1][1]) * 0.5,
                        (cur.ab[0][1] - ref.ab[0][1])};
        double be[3] = {(cur.bb[0][0] - ref.bb[0][0]), (cur.bb[1][1] - ref.bb[1][1]),
                        2.0 * (cur.bb[0][1] - ref.bb[0][1])};
        double Ha[3], Hbeta[3];
        for (int i = 0; i < 3; ++i) {
            Ha[i] = Hbeta[i] = 0;
            for (int j = 0; j < 3; ++j) {
                Ha[i] += H[i][j] * al[j];
                Hbeta[i] += H[i][j] * be[j];
            }
        }
        const double wq = qp[g].weight * ref.sqrta;
        // First derivatives of alpha and beta for every I.
        V3<double> dal[16][3], dbe[16][3];
        M3 da3[16];
        for (int I = 0; I < 16; ++I) {
            double p1 = phi[1][I], p2 = phi[2][I];
            dal[I][0] = 0.5 * (2.0 * p1 * cur.a[0]);
            dal[I][1] = 0.5 * (2.0 * p2 * cur.a[1]);
            dal[I][2] = p1 * cur.a[1] + p2 * cur.a[0];
            dbe[I][0] = db_dq(cur, cur.d[0][0], phi[3][I], p1, p2);
            dbe[I][1] = db_dq(cur, cur.d[1][1], phi[4][I], p1, p2);
            dbe[I][2] = 2.0 * db_dq(cur, cur.d[0][1], phi[5][I], p1, p2);
            da3_dq(cur, p1, p2, da3[I]);
        }
        // D matrices of the three b components (11, 22, 12).
        M3 D[3][4];
        const V3<double>* vs[3] = {&cur.d[0][0], &cur.d[1][1], &cur.d[0][1]};
        for (int k = 0; k < 3; ++k) d_matrices(cur, *vs[k], D[k][0], D[k][1], D[k][2], D[k][3]);
        const int phi_ab_row[3] = {3, 4, 5};
        const double beta_fac[3] = {1.0, 1.0, 2.0};   // beta_3 = 2 (b12 - bbar12)

        for (int I = 0; I < 16; ++I)
            for (int J = 0; J < 16; ++J) {
                M3 G1, G2;
                m3_zero(G1);
                m3_zero(G2);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        outer(dal[I][i], dal[J][j], H[i][j], G1);
                        outer(dbe[I][i], dbe[J][j], H[i][j], G2);
                    }
                // sum_ij d2 alpha_i H^{ij} alpha_j with the identity blocks
                double p1I = phi[1][I], p2I = phi[2][I], p1J = phi[1][J], p2J = phi[2][J];
                double d2al[3] = {p1I * p1J, p2I * p2J, p1I * p2J + p2I * p1J};
                for (int i = 0; i < 3; ++i) add_identity(d2al[i] * Ha[i], G1);
                if (!pseudo) {
                    for (int i = 0; i < 3; ++i) {
                        // d2 b / dq_J dq_I =  Phi^I_{,ab} da3/dq_J + Phi^J_{,ab} (da3/dq_I)^T
                        //   + Phi^I_1 Phi^J_1 D11 + Phi^I_2 Phi^J_2 D22 + Phi^I_1 Phi^J_2 D12 + Phi^I_2 Phi^J_1 D21
                        M3 d2b;
                        m3_zero(d2b);
                        double pabI = phi[phi_ab_row[i]][I], pabJ = phi[phi_ab_row[i]][J];
                        for (int r = 0; r < 3; ++r)
                            for (int c = 0; c < 3; ++c) {
                                d2b[r][c] += pabI * da3[J][r][c] + pabJ * da3[I][c][r];
                                d2b[r][c] += p1I * p1J * D[i][0][r][c] + p2I * p2J * D[i][1][r][c] +
                                             p1I * p2J * D[i][2][r][c] + p2I * p1J * D[i][3][r][c];
                            }
                        double coef = beta_fac[i] * Hbeta[i];
                        for (int r = 0; r < 3; ++r)
                            for (int c = 0; c < 3; ++c) G2[r][c] += coef * d2b[r][c];
                    }
                }
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c)
                        hess[(3 * I + r) * 48 + 3 * J + c] += wq * (h * G1[r][c] + (h * h * h / 12.0) * G2[r][c]);
            }
    }
}

// Mass matrix of Eq. (mass): M^{IJ} = sum_gp rho h Phi^I Phi^J sqrt(abar) w_gp,
// times the 3x3 identity.
void patch_mass(const Shell& s, const double* qb, double* mass) {
    QPoint qp[16];
    quad_points(s, qp);
    const double rh = s.density * s.thickness;
    for (int i = 0; i < 48 * 48; ++i) mass[i] = 0.0;
    for (int g = 0; g < 16; ++g) {
        Geo<double> ref = geometry<double>(qp[g].phi, qb);
        double wq = qp[g].weight * ref.sqrta * rh;
        for (int I = 0; I < 16; ++I)
            for (int J = 0; J < 16; ++J) {
                double m = wq * qp[g].phi[0][I] * qp[g].phi[0][J];
                for (int c = 0; c < 3; ++c) mass[(3 * I + c) * 48 + 3 * J + c] += m;
            }
    }
}

// Areal gravity f = rho h g integrated against each shape function ("External Forces").
void patch_gravity(const Shell& s, const double* qb, double* f) {
    QPoint qp[16];
    quad_points(s, qp);
    const double rh = s.density * s.thickness;
    for (int i = 0; i < 48; ++i) f[i] = 0.0;
    for (int g = 0; g < 16; ++g) {
        Geo<double> ref = geometry<double>(qp[g].phi, qb);
        double wq = qp[g].weight * ref.sqrta * rh;
        for (int I = 0; I < 16; ++I)
            for (int c = 0; c < 3; ++c) f[3 * I + c] += wq * qp[g].phi[0][I] * s.gravity[c];
    }
}

// Pressure load (Sec. 4.3, "External Forces", f = p n): a pressure p acts
// on the current surface, per unit current area, along n = a_1 x a_2 /
// |a_1 x a_2|, so p n dA = p (a_1 x a_2) dxi1 dxi2 and the nodal generalized
// force is F_I = sum_gp w p Phi^I (a_1 x a_2) (no sqrt(abar): the area
// element is the current one).
void patch_pressure(const Shell& s, const double* q, double p, double* f) {
    QPoint qp[16];
    quad_points(s, qp);
    for (int i = 0; i < 48; ++i) f[i] = 0.0;
    for (int g = 0; g < 16; ++g) {
        Geo<double> cur = geometry<double>(qp[g].phi, q);
        const V3<double> n = cross(cur.a[0], cur.a[1]);
        const double wq = qp[g].weight * p;
        for (int I = 0; I < 16; ++I)
            for (int c = 0; c < 3; ++c) f[3 * I + c] += wq * qp[g].phi[0][I] * compc(n, c);
    }
}

template double patch_energy_tensor<double>(const Shell&, const double*, const double*);
template std::complex<double> patch_energy_tensor<std::complex<double>>(const Shell&, const std::complex<double>*,
                                                                        const double*);
template double patch_energy_voigt<double>(const Shell&, const double*, const double*);
template void patch_gradient<double>(const Shell&, const double*, const double*, double*);
template void patch_gradient<std::complex<double>>(const Shell&, const std::complex<double>*, const double*,
                                                   std::complex<double>*);

}  // namespace orc
