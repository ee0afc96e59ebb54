// BHEM CPU oracle -- TEST INFRASTRUCTURE ONLY (see bhem_oracle.hpp).
// C entry points for the ctypes wrapper oracle/oracle.py.
#include <complex>
#include <cstring>

#include "bhem_oracle.hpp"
#include "oracle_global.hpp"

using namespace orc;
typedef std::complex<double> cd;

extern "C" {

int orc_num_nodes(const Shell* s) { return num_nodes(*s); }

void orc_patch_nodes(const Shell* s, int pi, int pj, int* nodes) { patch_nodes(*s, pi, pj, nodes); }

void orc_hermite_1d(double t, double* w, double* d1, double* d2) {
    double a[2][2], b[2][2], c[2][2];
    hermite_1d(t, a, b, c);
    std::memcpy(w, a, sizeof a);
    std::memcpy(d1, b, sizeof b);
    std::memcpy(d2, c, sizeof c);
}

void orc_shape_functions(double t1, double t2, double dxi1, double dxi2, double* out96) {
    double o[6][16];
    shape_functions(t1, t2, dxi1, dxi2, o);
    std::memcpy(out96, o, sizeof o);
}

void orc_gauss4(double* theta, double* weight) { gauss4(theta, weight); }

double orc_patch_energy(const Shell* s, const double* q, const double* qb) {
    return patch_energy_tensor<double>(*s, q, qb);
}

double orc_patch_energy_voigt(const Shell* s, const double* q, const double* qb) {
    return patch_energy_voigt<double>(*s, q, qb);
}

void orc_patch_gradient(const Shell* s, const double* q, const double* qb, double* g) {
    patch_gradient<double>(*s, q, qb, g);
}

void orc_patch_hessian(const Shell* s, const double* q, const double* qb, int pseudo, double* h) {
    patch_hessian(*s, q, qb, pseudo, h);
}

void orc_patch_mass(const Shell* s, const double* qb, double* m) { patch_mass(*s, qb, m); }

void orc_patch_gravity(const Shell* s, const double* qb, double* f) { patch_gravity(*s, qb, f); }

// Complex-step helpers: the energy (tensor form) and the gradient evaluated
// at q + i q_im; the caller divides the imaginary part by the step.
void orc_patch_energy_cs(const Shell* s, const double* q, const double* q_im, const double* qb, double* re,
                         double* im) {
    cd z[48];
    for (int i = 0; i < 48; ++i) z[i] = cd(q[i], q_im[i]);
    cd e = patch_energy_tensor<cd>(*s, z, qb);
    *re = e.real();
    *im = e.imag();
}

void orc_patch_gradient_cs(const Shell* s, const double* q, const double* q_im, const double* qb, double* g_re,
                           double* g_im) {
    cd z[48], g[48];
    for (int i = 0; i < 48; ++i) z[i] = cd(q[i], q_im[i]);
    patch_gradient<cd>(*s, z, qb, g);
    for (int i = 0; i < 48; ++i) {
        g_re[i] = g[i].real();
        g_im[i] = g[i].imag();
    }
}

double orc_energy(const Shell* s, const double* q, const double* qb) { return energy(*s, q, qb); }

void orc_gradient(const Shell* s, const double* q, const double* qb, double* g) { gradient(*s, q, qb, g); }

void orc_gravity(const Shell* s, const double* qb, double* f) { gravity_load(*s, qb, f); }

void orc_patch_pressure(const Shell* s, const double* q, double p, double* f) { patch_pressure(*s, q, p, f); }

// Nodal pressure load of the whole shell at state q (assembled patch loads).
void orc_pressure_load(const Shell* s, const double* q, double p, double* f) {
    std::memset(f, 0, sizeof(double) * 12 * num_nodes(*s));
    for (int pj = 0; pj < s->n2; ++pj)
        for (int pi = 0; pi < s->n1; ++pi) {
            double lq[48], lf[48];
            int nodes[4];
            gather(*s, pi, pj, q, lq, nodes);
            patch_pressure(*s, lq, p, lf);
            for (int c = 0; c < 4; ++c)
                for (int d = 0; d < 12; ++d) f[12 * nodes[c] + d] += lf[12 * c + d];
        }
}

// Global matrix as node blocks.  which = 0: elastic Hessian (pseudo if
// pseudo != 0); 1: mass matrix.  Writes up to cap blocks: rows[b], cols[b],
// vals[144 b]; returns the block count.
int orc_matrix_blocks(const Shell* s, const double* q, const double* qb, int which, int pseudo, int cap, int* rows,
                      int* cols, double* vals) {
    NodeBlocks K(*s);
    if (which == 0)
        assemble_hessian(*s, q, qb, pseudo, K, 1.0);
    else
        assemble_mass(*s, qb, K, 1.0);
    int nb = 0;
    for (int r = 0; r < K.nn; ++r)
        for (const auto& e : K.rows[r]) {
            if (nb < cap) {
                rows[nb] = r;
                cols[nb] = e.col;
                std::memcpy(vals + 144 * (size_t)nb, e.v.data(), 144 * sizeof(double));
            }
            ++nb;
        }
    return nb;
}

// Dense global matrix (small grids only), same `which` as above.
void orc_matrix_dense(const Shell* s, const double* q, const double* qb, int which, int pseudo, double* out) {
    NodeBlocks K(*s);
    if (which == 0)
        assemble_hessian(*s, q, qb, pseudo, K, 1.0);
    else
        assemble_mass(*s, qb, K, 1.0);
    const int n = 12 * K.nn;
    std::memset(out, 0, sizeof(double) * (size_t)n * n);
    for (int r = 0; r < K.nn; ++r)
        for (const auto& e : K.rows[r])
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j) out[(size_t)(12 * r + i) * n + 12 * e.col + j] = e.v[12 * i + j];
}

int orc_newton_step(const Shell* s, const double* qb, const uint8_t* fixed, double dt, const double* qn,
                    const double* vn, const double* qpresc, const double* f_ext, const NewtonOpts* o, double* qn1,
                    double* vn1, NewtonStats* st) {
    return newton_step(*s, qb, fixed, dt, qn, vn, qpresc, f_ext, *o, qn1, vn1, st);
}

// The same step with a record of its iterations (see NewtonTrace).
int orc_newton_step_traced(const Shell* s, const double* qb, const uint8_t* fixed, double dt, const double* qn,
                           const double* vn, const double* qpresc, const double* f_ext, const NewtonOpts* o,
                           double* qn1, double* vn1, NewtonStats* st, NewtonTrace* tr) {
    return newton_step(*s, qb, fixed, dt, qn, vn, qpresc, f_ext, *o, qn1, vn1, st, tr);
}

// The same step with augmented-Lagrangian point constraints (AlmOpts).
int orc_newton_step_alm(const Shell* s, const double* qb, const uint8_t* fixed, double dt, const double* qn,
                        const double* vn, const double* qpresc, const double* f_ext, const NewtonOpts* o, double* qn1,
                        double* vn1, NewtonStats* st, AlmOpts* alm) {
    return newton_step(*s, qb, fixed, dt, qn, vn, qpresc, f_ext, *o, qn1, vn1, st, nullptr, alm);
}

// Solve (K + mass_scale M) x = b with fixed DOFs replaced by identity rows
// and columns; solver 0: banded LDL^T, 1: block-Jacobi CG.  For solver tests.
// Returns 0 on success.
int orc_linear_solve(const Shell* s, const double* q, const double* qb, const uint8_t* fixed, double mass_scale,
                     int solver, const double* b, double* x, double rtol, int maxit, int* iters) {
    NodeBlocks A(*s), M(*s);
    assemble_hessian(*s, q, qb, 0, A, 1.0);
    assemble_mass(*s, qb, M, 1.0);
    for (int r = 0; r < A.nn; ++r)
        for (auto& e : A.rows[r]) {
            const double* m = M.find(r, e.col);
            for (int t = 0; t < 144; ++t) e.v[t] += mass_scale * m[t];
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j) {
                    bool fi = fixed && fixed[12 * r + i], fj = fixed && fixed[12 * e.col + j];
                    if (fi || fj) e.v[12 * i + j] = (fi && fj && r == e.col && i == j) ? 1.0 : 0.0;
                }
        }
    *iters = 0;
    if (solver == 0) return banded_ldlt_solve(A, b, x) ? 0 : 2;
    return block_jacobi_cg(A, b, x, rtol, maxit, iters);
}

}  // extern "C"
