// BHEM CPU oracle -- TEST INFRASTRUCTURE ONLY (see bhem_oracle.hpp).
//
// Global quantities over a patch grid, and one implicit-Euler step (Sec. 6.1):
//   M qddot = F,  qdot^{n+1} = qdot^n + dt M^{-1} F(q^{n+1}),  q^{n+1} = q^n + dt qdot^{n+1},
// solved as the minimisation of the incremental potential
//   E(q) = (1/2dt^2)(q - qhat)^T M (q - qhat) + V(q) - f^T (q - qhat),  qhat = q^n + dt qdot^n,
// by Newton's method with a backtracking line search using quadratic then
// cubic interpolation, a direct LDL^T factorisation of the banded Hessian
// (the paper's solver class) or, for large grids, a block-Jacobi CG, and a
// diagonal regulariser when the Hessian is not positive definite.
#include <algorithm>
#include <cstring>
#include <map>
#include <utility>

#include "bhem_oracle.hpp"
#include "oracle_global.hpp"

namespace orc {

void gather(const Shell& s, int pi, int pj, const double* x, double* loc, int nodes[4]) {
    patch_nodes(s, pi, pj, nodes);
    for (int c = 0; c < 4; ++c)
        for (int d = 0; d < 12; ++d) loc[12 * c + d] = x[12 * nodes[c] + d];
}

double energy(const Shell& s, const double* q, const double* qb) {
    double e = 0.0;
#pragma omp parallel for reduction(+ : e) schedule(static)
    for (int p = 0; p < s.n1 * s.n2; ++p) {
        double lq[48], lb[48];
        int nodes[4];
        gather(s, p % s.n1, p / s.n1, q, lq, nodes);
        gather(s, p % s.n1, p / s.n1, qb, lb, nodes);
        e += patch_energy_tensor<double>(s, lq, lb);
    }
    return e;
}

void gradient(const Shell& s, const double* q, const double* qb, double* g) {
    const int ndof = 12 * num_nodes(s);
    std::memset(g, 0, sizeof(double) * ndof);
    std::vector<double> local(48 * (size_t)s.n1 * s.n2);
#pragma omp parallel for schedule(static)
    for (int p = 0; p < s.n1 * s.n2; ++p) {
        double lq[48], lb[48];
        int nodes[4];
        gather(s, p % s.n1, p / s.n1, q, lq, nodes);
        gather(s, p % s.n1, p / s.n1, qb, lb, nodes);
        patch_gradient<double>(s, lq, lb, &local[48 * (size_t)p]);
    }
    for (int p = 0; p < s.n1 * s.n2; ++p) {
        int nodes[4];
        patch_nodes(s, p % s.n1, p / s.n1, nodes);
        for (int c = 0; c < 4; ++c)
            for (int d = 0; d < 12; ++d) g[12 * nodes[c] + d] += local[48 * (size_t)p + 12 * c + d];
    }
}

// ------------------------------------------------------------ node blocks
NodeBlocks::NodeBlocks(const Shell& s) : shell(s), nn(num_nodes(s)), rows(nn) {
    for (int pj = 0; pj < s.n2; ++pj)
        for (int pi = 0; pi < s.n1; ++pi) {
            int nodes[4];
            patch_nodes(s, pi, pj, nodes);
            for (int c = 0; c < 4; ++c)
                for (int d = 0; d < 4; ++d) find_or_add(nodes[c], nodes[d]);
        }
    for (auto& r : rows) std::sort(r.begin(), r.end(), [](const Entry& a, const Entry& b) { return a.col < b.col; });
}

double* NodeBlocks::find_or_add(int r, int c) {
    for (auto& e : rows[r])
        if (e.col == c) return e.v.data();
    rows[r].push_back(Entry{c, {}});
    rows[r].back().v.fill(0.0);
    return rows[r].back().v.data();
}

double* NodeBlocks::find(int r, int c) {
    for (auto& e : rows[r])
        if (e.col == c) return e.v.data();
    return nullptr;
}

void NodeBlocks::zero() {
    for (auto& r : rows)
        for (auto& e : r) e.v.fill(0.0);
}

void NodeBlocks::add_patch(const int nodes[4], const double* m48, double scale) {
    for (int c = 0; c < 4; ++c)
        for (int d = 0; d < 4; ++d) {
            double* blk = find(nodes[c], nodes[d]);
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j) blk[12 * i + j] += scale * m48[(12 * c + i) * 48 + 12 * d + j];
        }
}

void NodeBlocks::matvec(const double* x, double* y) const {
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nn; ++r) {
        double acc[12] = {0};
        for (const auto& e : rows[r])
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j) acc[i] += e.v[12 * i + j] * x[12 * e.col + j];
        for (int i = 0; i < 12; ++i) y[12 * r + i] = acc[i];
    }
}

void assemble_hessian(const Shell& s, const double* q, const double* qb, int pseudo, NodeBlocks& K, double scale) {
    const int np = s.n1 * s.n2;
    std::vector<double> local((size_t)np * 48 * 48);
#pragma omp parallel for schedule(dynamic, 16)
    for (int p = 0; p < np; ++p) {
        double lq[48], lb[48];
        int nodes[4];
        gather(s, p % s.n1, p / s.n1, q, lq, nodes);
        gather(s, p % s.n1, p / s.n1, qb, lb, nodes);
        patch_hessian(s, lq, lb, pseudo, &local[(size_t)p * 2304]);
    }
    for (int p = 0; p < np; ++p) {
        int nodes[4];
        patch_nodes(s, p % s.n1, p / s.n1, nodes);
        K.add_patch(nodes, &local[(size_t)p * 2304], scale);
    }
}

void assemble_mass(const Shell& s, const double* qb, NodeBlocks& M, double scale) {
    for (int p = 0; p < s.n1 * s.n2; ++p) {
        double lb[48], m[2304];
        int nodes[4];
        gather(s, p % s.n1, p / s.n1, qb, lb, nodes);
        patch_mass(s, lb, m);
        M.add_patch(nodes, m, scale);
    }
}

void gravity_load(const Shell& s, const double* qb, double* f) {
    std::memset(f, 0, sizeof(double) * 12 * num_nodes(s));
    for (int p = 0; p < s.n1 * s.n2; ++p) {
        double lb[48], lf[48];
        int nodes[4];
        gather(s, p % s.n1, p / s.n1, qb, lb, nodes);
        patch_gravity(s, lb, lf);
        for (int c = 0; c < 4; ++c)
            for (int d = 0; d < 12; ++d) f[12 * nodes[c] + d] += lf[12 * c + d];
    }
}

// ------------------------------------------------------ banded LDL^T solve
// Band LDL^T without pivoting of a symmetric matrix given as node blocks.
// Returns false on a pivot that is not positive (matrix not positive definite).
bool banded_ldlt_solve(const NodeBlocks& A, const double* b, double* x) {
    const int n = 12 * A.nn;
    int bw = 0;
    for (int r = 0; r < A.nn; ++r)
        for (const auto& e : A.rows[r]) bw = std::max(bw, std::abs(12 * (r - e.col)) + 11);
    const int w = bw + 1;
    // L[i][k] stores row i, column i - bw + k (k = bw is the diagonal).
    std::vector<double> L((size_t)n * w, 0.0);
    for (int r = 0; r < A.nn; ++r)
        for (const auto& e : A.rows[r])
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j) {
                    int gi = 12 * r + i, gj = 12 * e.col + j;
                    if (gj <= gi) L[(size_t)gi * w + (gj - gi + bw)] = e.v[12 * i + j];
                }
    std::vector<double> dg(n);
    for (int j = 0; j < n; ++j) {
        double* Lj = &L[(size_t)j * w];
        int k0 = std::max(0, j - bw);
        double d = Lj[bw];
        for (int k = k0; k < j; ++k) {
            double l = Lj[k - j + bw];
            d -= l * l * dg[k];
        }
        if (!(d > 0.0)) return false;
        dg[j] = d;
        int imax = std::min(n - 1, j + bw);
#pragma omp parallel for schedule(static) if (imax - j > 64)
        for (int i = j + 1; i <= imax; ++i) {
            double* Li = &L[(size_t)i * w];
            int kk0 = std::max(0, i - bw);
            double v = Li[j - i + bw];
            for (int k = kk0; k < j; ++k) v -= Li[k - i + bw] * Lj[k - j + bw] * dg[k];
            Li[j - i + bw] = v / d;
        }
    }
    // forward: L y = b; diagonal; backward: L^T x = y
    std::vector<double> y(b, b + n);
    for (int i = 0; i < n; ++i) {
        const double* Li = &L[(size_t)i * w];
        for (int k = std::max(0, i - bw); k < i; ++k) y[i] -= Li[k - i + bw] * y[k];
    }
    for (int i = 0; i < n; ++i) y[i] /= dg[i];
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k <= std::min(n - 1, i + bw); ++k) v -= L[(size_t)k * w + (i - k + bw)] * x[k];
        x[i] = v;
    }
    return true;
}

// ----------------------------------------------------- block-Jacobi CG
// Plain preconditioned CG with the inverse of each node's 12x12 diagonal
// block as the preconditioner.  Stops when ||b - A x|| <= rtol ||b||.
// Returns 0 converged, 1 iteration cap, 2 p^T A p <= 0 or a block that is not
// positive definite.
static bool chol12_inverse(const double* a, double* inv) {
    double L[12][12] = {{0}};
    for (int j = 0; j < 12; ++j) {
        double d = a[12 * j + j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > 0.0)) return false;
        L[j][j] = std::sqrt(d);
        for (int i = j + 1; i < 12; ++i) {
            double v = a[12 * i + j];
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            L[i][j] = v / L[j][j];
        }
    }
    for (int col = 0; col < 12; ++col) {
        double e[12] = {0}, y[12];
        e[col] = 1.0;
        for (int i = 0; i < 12; ++i) {
            double v = e[i];
            for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
            y[i] = v / L[i][i];
        }
        for (int i = 11; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < 12; ++k) v -= L[k][i] * y[k];
            y[i] = v / L[i][i];
        }
        for (int i = 0; i < 12; ++i) inv[12 * i + col] = y[i];
    }
    return true;
}

int block_jacobi_cg(const NodeBlocks& A, const double* b, double* x, double rtol, int maxit, int* iters) {
    const int nn = A.nn, n = 12 * nn;
    std::vector<double> Dinv((size_t)nn * 144);
    bool ok = true;
    for (int r = 0; r < nn; ++r) {
        const double* d = nullptr;
        for (const auto& e : A.rows[r])
            if (e.col == r) d = e.v.data();
        if (!chol12_inverse(d, &Dinv[(size_t)144 * r])) ok = false;
    }
    if (!ok) return 2;
    std::vector<double> r(b, b + n), z(n), p(n), Ap(n);
    std::fill(x, x + n, 0.0);
    auto dotv = [&](const std::vector<double>& u, const std::vector<double>& v) {
        double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
        for (int i = 0; i < n; ++i) s += u[i] * v[i];
        return s;
    };
    auto precond = [&]() {
#pragma omp parallel for schedule(static)
        for (int nd = 0; nd < nn; ++nd)
            for (int i = 0; i < 12; ++i) {
                double v = 0;
                for (int j = 0; j < 12; ++j) v += Dinv[(size_t)144 * nd + 12 * i + j] * r[12 * nd + j];
                z[12 * nd + i] = v;
            }
    };
    const double bnorm = std::sqrt(dotv(r, r));
    *iters = 0;
    if (bnorm == 0.0) return 0;
    precond();
    p = z;
    double rz = dotv(r, z);
    for (int it = 0; it < maxit; ++it) {
        A.matvec(p.data(), Ap.data());
        double pAp = dotv(p, Ap);
        if (!(pAp > 0.0)) return 2;
        double al = rz / pAp;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            x[i] += al * p[i];
            r[i] -= al * Ap[i];
        }
        *iters = it + 1;
        if (std::sqrt(dotv(r, r)) <= rtol * bnorm) return 0;
        precond();
        double rz2 = dotv(r, z);
        double be = rz2 / rz;
        rz = rz2;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) p[i] = z[i] + be * p[i];
    }
    return 1;
}

// ----------------------------------------------------------- Newton step
namespace {

// Incremental potential of one implicit-Euler step with mass-proportional
// Rayleigh damping (damping force -alpha M qdot, qdot = (q - q_n)/dt):
//   E(q) = (1/2dt^2)(q - qhat)^T M (q - qhat) + (alpha/2dt)(q - q_n)^T M (q - q_n)
//          + V(q) - f^T (q - qhat),   f = areal gravity + external nodal forces,
// whose stationarity is M(q - qhat)/dt^2 + alpha M (q - q_n)/dt + grad V = f.
struct Problem {
    const Shell& s;
    const double* qb;
    const uint8_t* fixed;
    double dt;
    const double* qn = nullptr;
    std::vector<double> qhat, f;
    NodeBlocks M;
    Problem(const Shell& sh, const double* qbar, const uint8_t* fx, double dt_, const double* f_ext)
        : s(sh), qb(qbar), fixed(fx), dt(dt_), M(sh) {
        assemble_mass(s, qb, M, 1.0);
        f.resize(12 * num_nodes(s));
        gravity_load(s, qb, f.data());
        if (f_ext)
            for (size_t i = 0; i < f.size(); ++i) f[i] += f_ext[i];
    }
    int n() const { return 12 * num_nodes(s); }
    bool is_fixed(int i) const { return fixed && fixed[i]; }
    // augmented-Lagrangian point constraints: per constraint its patch's
    // nodes and the 16 shape-function values of its kind at its point
    const AlmOpts* alm = nullptr;
    std::vector<std::array<int, 4>> alm_nodes;
    std::vector<std::array<double, 16>> alm_psi;
    void set_alm(const AlmOpts* a) {
        alm = a;
        if (!a) return;
        for (int k = 0; k < a->n; ++k) {
            const PointConstraint& pc = a->pts[k];
            std::array<int, 4> nd;
            patch_nodes(s, pc.pi, pc.pj, nd.data());
            double ph[6][16];
            shape_functions(pc.t1, pc.t2, s.dxi1, s.dxi2, ph);
            std::array<double, 16> psi;
            for (int I = 0; I < 16; ++I) psi[I] = ph[pc.kind][I];
            alm_nodes.push_back(nd);
            alm_psi.push_back(psi);
        }
    }
    // c = x^(kind)(xi) - target of constraint k
    void residual(int k, const double* q, double c[3]) const {
        for (int comp = 0; comp < 3; ++comp) {
            double v = -alm->pts[k].target[comp];
            for (int I = 0; I < 16; ++I) v += alm_psi[k][I] * q[12 * alm_nodes[k][I >> 2] + 3 * (I & 3) + comp];
            c[comp] = v;
        }
    }
    // E(q), grad E(q) (zero on fixed DOFs) and |E| terms for the noise floor.
    double eval(const double* q, double* g, double* scale) {
        const int nd = n();
        std::vector<double> dq(nd), Mdq(nd), dn(nd), Mdn(nd);
        for (int i = 0; i < nd; ++i) {
            dq[i] = q[i] - qhat[i];
            dn[i] = q[i] - qn[i];
        }
        M.matvec(dq.data(), Mdq.data());
        M.matvec(dn.data(), Mdn.data());
        const double c_damp = s.damping / dt;
        double ekin = 0, edamp = 0, egrav = 0;
        for (int i = 0; i < nd; ++i) {
            ekin += 0.5 * dq[i] * Mdq[i] / (dt * dt);
            edamp += 0.5 * c_damp * dn[i] * Mdn[i];
            egrav -= f[i] * dq[i];
        }
        double eel = energy(s, q, qb);
        gradient(s, q, qb, g);
        // - lambda.c + (penalty/2)|c|^2 and its gradient C^T (penalty c - lambda)
        double ealm = 0.0;
        if (alm)
            for (int k = 0; k < alm->n; ++k) {
                double c[3];
                residual(k, q, c);
                for (int comp = 0; comp < 3; ++comp) {
                    const double lam = alm->lambda[3 * k + comp];
                    ealm += -lam * c[comp] + 0.5 * alm->penalty * c[comp] * c[comp];
                    const double w = alm->penalty * c[comp] - lam;
                    for (int I = 0; I < 16; ++I) g[12 * alm_nodes[k][I >> 2] + 3 * (I & 3) + comp] += w * alm_psi[k][I];
                }
            }
        for (int i = 0; i < nd; ++i) {
            g[i] += Mdq[i] / (dt * dt) + c_damp * Mdn[i] - f[i];
            if (is_fixed(i)) g[i] = 0.0;
        }
        if (scale)
            *scale = std::fabs(eel) + std::fabs(ekin) + std::fabs(edamp) + std::fabs(egrav) + std::fabs(ealm);
        return eel + ekin + edamp + egrav + ealm;
    }
};

double norm2(const std::vector<double>& v) {
    double s = 0;
    for (double x : v) s += x * x;
    return std::sqrt(s);
}

}  // namespace

int newton_step(const Shell& s, const double* qb, const uint8_t* fixed, double dt, const double* qn, const double* vn,
                const double* qpresc, const double* f_ext, const NewtonOpts& o, double* qn1, double* vn1,
                NewtonStats* st, NewtonTrace* tr, AlmOpts* alm) {
    Problem P(s, qb, fixed, dt, f_ext);
    P.qn = qn;
    P.set_alm(alm);
    if (alm) alm->outer_iters = 0;
    const int n = P.n();
    P.qhat.resize(n);
    for (int i = 0; i < n; ++i) P.qhat[i] = qn[i] + dt * vn[i];
    std::vector<double> q(P.qhat), g(n), d(n), qt(n), gt(n), rhs(n), absq(n), floor_v(n);
    for (int i = 0; i < n; ++i)
        if (P.is_fixed(i)) q[i] = qpresc ? qpresc[i] : qn[i];
    *st = NewtonStats{};
    double scale;
    double E = P.eval(q.data(), g.data(), &scale);
    const double g0 = norm2(g);
    st->grad_norm0 = g0;
    // Hessian of the previous iteration (no constraint rows), for the
    // rounding floor of the gradient: a state stored in FP64 is only known to
    // eps |q|, so g cannot be resolved below ~ eps |A| |q| on free rows.
    NodeBlocks Aprev(s);
    bool have_prev = false;
    int status = 1;   // Newton iteration cap
    int k_total = 0;
    for (;;) {   // augmented Lagrangian: Newton, then a multiplier update, until the constraints hold
    status = 1;
    for (int k = 0;; ++k) {
        double gn = norm2(g);
        st->grad_norm = gn;
        double floor = 0.0;
        if (have_prev) {
            for (int i = 0; i < n; ++i) absq[i] = std::fabs(q[i]);
            NodeBlocks absA(Aprev);
            for (auto& r : absA.rows)
                for (auto& e : r)
                    for (auto& v : e.v) v = std::fabs(v);
            absA.matvec(absq.data(), floor_v.data());
            double acc = 0;
            for (int i = 0; i < n; ++i)
                if (!P.is_fixed(i)) acc += floor_v[i] * floor_v[i];
            floor = 4.0 * 2.220446049250313e-16 * std::sqrt(acc);
        }
        st->grad_floor = floor;
        if (gn == 0.0 || (k > 0 && gn <= std::max(o.newton_rtol * g0, floor))) {
            status = 0;
            break;
        }
        if (k == o.newton_maxit) break;
        // A = (1/dt^2 + alpha/dt) M + K(q); the solve sees identity rows and
        // columns on fixed DOFs.
        NodeBlocks A(s);
        assemble_hessian(s, q.data(), qb, o.pseudo, A, 1.0);
        const double mcoef = 1.0 / (dt * dt) + s.damping / dt;
        for (int r = 0; r < A.nn; ++r)
            for (auto& e : A.rows[r]) {
                const double* m = P.M.find(r, e.col);
                for (int t = 0; t < 144; ++t) e.v[t] += m[t] * mcoef;
            }
        // penalty C^T C of the point constraints: penalty (psi psi^T) x I_3 on their patches
        if (alm)
            for (int kc = 0; kc < alm->n; ++kc) {
                std::vector<double> m48(48 * 48, 0.0);
                for (int I = 0; I < 16; ++I)
                    for (int J = 0; J < 16; ++J)
                        for (int comp = 0; comp < 3; ++comp)
                            m48[(3 * I + comp) * 48 + 3 * J + comp] = alm->penalty * P.alm_psi[kc][I] * P.alm_psi[kc][J];
                A.add_patch(P.alm_nodes[kc].data(), m48.data(), 1.0);
            }
        Aprev = A;
        have_prev = true;
        for (int r = 0; r < A.nn; ++r)
            for (auto& e : A.rows[r])
                for (int i = 0; i < 12; ++i)
                    for (int j = 0; j < 12; ++j) {
                        bool fi = P.is_fixed(12 * r + i), fj = P.is_fixed(12 * e.col + j);
                        if (fi || fj) e.v[12 * i + j] = (fi && fj && r == e.col && i == j) ? 1.0 : 0.0;
                    }
        for (int i = 0; i < n; ++i) rhs[i] = -g[i];
        // Diagonal regulariser: A + delta diag(A), delta = 1e-6 * 10^t up to 1e2.
        std::vector<double> diag(n);
        for (int r = 0; r < A.nn; ++r)
            for (int i = 0; i < 12; ++i) diag[12 * r + i] = A.find(r, r)[13 * i];
        double delta = 0.0;
        bool solved = false;
        for (int attempt = 0; attempt < 10 && !solved; ++attempt) {
            if (attempt > 0) {
                double nd_ = attempt == 1 ? 1e-6 : delta * 10.0;
                for (int r = 0; r < A.nn; ++r)
                    for (int i = 0; i < 12; ++i) A.find(r, r)[13 * i] += (nd_ - delta) * diag[12 * r + i];
                delta = nd_;
            }
            if (o.solver == 0) {
                solved = banded_ldlt_solve(A, rhs.data(), d.data());
            } else {
                int its = 0;
                int rc = block_jacobi_cg(A, rhs.data(), d.data(), o.pcg_rtol, o.pcg_maxit, &its);
                st->pcg_iters_total += its;
                solved = rc != 2;
            }
        }
        st->reg_delta = std::max(st->reg_delta, delta);
        if (!solved) {
            status = 3;
            break;
        }
        for (int i = 0; i < n; ++i)
            if (P.is_fixed(i)) d[i] = 0.0;
        // trace row of this iteration (recording only)
        const bool rec = tr && k < tr->cap_iters;
        if (rec) {
            tr->n_iters = k + 1;
            if (tr->delta) tr->delta[k] = delta;
            if (tr->energy) tr->energy[k] = E;
            if (tr->q_iter) std::copy(q.begin(), q.end(), tr->q_iter + (size_t)k * n);
        }
        // Backtracking line search on E along d (the paper's solver uses the
        // quadratic and cubic line searches of ArcSim): Armijo with c1 = 1e-4;
        // the first new step from a quadratic fit, later ones from a cubic
        // fit, each clamped to [0.1, 0.5] of the previous step.
        double slope = 0;
        for (int i = 0; i < n; ++i) slope += g[i] * d[i];
        const bool steepest = !(slope < 0.0);
        if (steepest) {
            for (int i = 0; i < n; ++i) d[i] = -g[i];
            slope = -gn * gn;
        }
        if (rec) {
            if (tr->slope) tr->slope[k] = slope;
            if (tr->steepest) tr->steepest[k] = steepest ? 1 : 0;
            if (tr->d_iter) std::copy(d.begin(), d.end(), tr->d_iter + (size_t)k * n);
            if (tr->n_trials) tr->n_trials[k] = 0;
        }
        double alpha = 1.0, a_prev = 0.0, E_prev = 0.0;
        bool accepted = false;
        double Et = 0, scale_t = 0;
        for (int t = 0; t < 20; ++t) {
            for (int i = 0; i < n; ++i) qt[i] = q[i] + alpha * d[i];
            Et = P.eval(qt.data(), gt.data(), &scale_t);
            if (rec) {
                if (tr->alpha) tr->alpha[20 * k + t] = alpha;
                if (tr->e_trial) tr->e_trial[20 * k + t] = Et;
                if (tr->n_trials) tr->n_trials[k] = t + 1;
            }
            if (std::isfinite(Et)) {
                if (Et <= E + 1e-4 * alpha * slope) {
                    accepted = true;
                    break;
                }
                // predicted and actual energy changes both below the energy's
                // rounding: the Armijo test is void, accept a smaller gradient
                const double noise = 1e-12 * std::max(scale, scale_t);
                if (-slope <= noise && std::fabs(Et - E) <= noise && norm2(gt) < gn) {
                    accepted = true;
                    break;
                }
            }
            double a_new;
            if (!std::isfinite(Et)) {
                a_new = 0.1 * alpha;
            } else if (t == 0) {
                a_new = -slope * alpha * alpha / (2.0 * (Et - E - slope * alpha));
            } else {
                double d1 = Et - E - slope * alpha, d2 = E_prev - E - slope * a_prev;
                double den = a_prev * a_prev * alpha * alpha * (alpha - a_prev);
                double ca = (a_prev * a_prev * d1 - alpha * alpha * d2) / den;
                double cb = (-a_prev * a_prev * a_prev * d1 + alpha * alpha * alpha * d2) / den;
                if (ca == 0.0) {
                    a_new = -slope / (2.0 * cb);
                } else {
                    double disc = cb * cb - 3.0 * ca * slope;
                    a_new = disc >= 0.0 ? (-cb + std::sqrt(disc)) / (3.0 * ca) : 0.5 * alpha;
                }
            }
            if (!std::isfinite(a_new)) a_new = 0.5 * alpha;
            a_new = std::min(std::max(a_new, 0.1 * alpha), 0.5 * alpha);
            a_prev = alpha;
            E_prev = Et;
            alpha = a_new;
            st->ls_backtracks++;
        }
        st->newton_iters = k_total + k + 1;
        if (!accepted) {
            status = 2;
            break;
        }
        q = qt;
        g = gt;
        E = Et;
        scale = scale_t;
    }
    k_total = st->newton_iters;
    if (!alm || status != 0) break;
    double cmax = 0.0;
    std::vector<double> cc(3 * alm->n);
    for (int kc = 0; kc < alm->n; ++kc) {
        P.residual(kc, q.data(), &cc[3 * kc]);
        for (int comp = 0; comp < 3; ++comp) cmax = std::max(cmax, std::fabs(cc[3 * kc + comp]));
    }
    alm->residual = cmax;
    if (cmax <= alm->tol) break;
    if (alm->outer_iters == alm->max_outer) {
        status = 1;
        break;
    }
    for (int i = 0; i < 3 * alm->n; ++i) alm->lambda[i] -= alm->penalty * cc[i];
    alm->outer_iters++;
    E = P.eval(q.data(), g.data(), &scale);
    }
    for (int i = 0; i < n; ++i) {
        qn1[i] = q[i];
        vn1[i] = (q[i] - qn[i]) / dt;
    }
    return status;
}

}  // namespace orc
