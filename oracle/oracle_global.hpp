// BHEM CPU oracle -- TEST INFRASTRUCTURE ONLY (see bhem_oracle.hpp).
#pragma once
#include <array>
#include <vector>

#include "bhem_oracle.hpp"

namespace orc {

// Global symmetric matrix kept as 12x12 blocks per (node, node) pair; the
// pattern is every pair of nodes that share a patch.
struct NodeBlocks {
    struct Entry {
        int col;
        std::array<double, 144> v;   // row-major 12x12
    };
    Shell shell;
    int nn;
    std::vector<std::vector<Entry>> rows;
    explicit NodeBlocks(const Shell& s);
    double* find_or_add(int r, int c);
    double* find(int r, int c);
    const double* find(int r, int c) const { return const_cast<NodeBlocks*>(this)->find(r, c); }
    void zero();
    void add_patch(const int nodes[4], const double* m48, double scale);
    void matvec(const double* x, double* y) const;
};

void gather(const Shell& s, int pi, int pj, const double* x, double* loc, int nodes[4]);
double energy(const Shell& s, const double* q, const double* qb);
void gradient(const Shell& s, const double* q, const double* qb, double* g);
void assemble_hessian(const Shell& s, const double* q, const double* qb, int pseudo, NodeBlocks& K, double scale);
void assemble_mass(const Shell& s, const double* qb, NodeBlocks& M, double scale);
void gravity_load(const Shell& s, const double* qb, double* f);
bool banded_ldlt_solve(const NodeBlocks& A, const double* b, double* x);
int block_jacobi_cg(const NodeBlocks& A, const double* b, double* x, double rtol, int maxit, int* iters);

struct NewtonOpts {
    int solver;         // 0: banded LDL^T, 1: block-Jacobi CG
    int pseudo;         // 1: pseudo Hessian
    int newton_maxit;
    double newton_rtol;
    int pcg_maxit;
    double pcg_rtol;
};
struct NewtonStats {
    int newton_iters, pcg_iters_total, ls_backtracks, pad;
    double grad_norm0, grad_norm, grad_floor, reg_delta;
};
// Optional record of the Newton iterations, for tests that check each step
// of the method on its own (regulariser, direction, line search).  Arrays
// hold cap_iters rows; pointers may be NULL to skip a record.
struct NewtonTrace {
    int cap_iters;     // rows available
    int n_iters;       // rows written (iterations that produced a direction)
    double* delta;     // [cap] regulariser delta of iteration k (0: none)
    double* energy;    // [cap] E at the iterate of iteration k
    double* slope;     // [cap] g . d along the direction taken
    int* steepest;     // [cap] 1: the solve's direction was not a descent direction, -g taken
    int* n_trials;     // [cap] line-search trials (the last one accepted if the search succeeded)
    double* alpha;     // [cap][20] trial step lengths
    double* e_trial;   // [cap][20] E at each trial
    double* q_iter;    // [cap][n] iterate of iteration k
    double* d_iter;    // [cap][n] direction of iteration k
};
// Positional constraints at arbitrary midsurface points (Sec. 4.2: the
// position, or a first derivative, prescribed at a point that need not be a
// node), imposed by the augmented Lagrangian method (Sec. 6.1).  Constraint
// c = x^(kind)(xi) - target (3 rows, linear in q); the Newton iteration
// minimises E(q) - lambda.c + (penalty/2)|c|^2; after it converges the
// multipliers are updated, lambda <- lambda - penalty c, until max |c| <= tol.
struct PointConstraint {
    int pi, pj;          // patch
    double t1, t2;       // local parameters in [0, 1]
    int kind;            // 0: x, 1: dx/dxi1, 2: dx/dxi2
    double target[3];
};
struct AlmOpts {
    int n;
    const PointConstraint* pts;
    double penalty;
    double tol;
    int max_outer;
    double* lambda;      // [3 n] multipliers: in, the starting values; out, the final ones
    int outer_iters;     // out: multiplier updates made
    double residual;     // out: max |c| at the end
};
// Converged when ||g_k|| <= max(newton_rtol ||g_0||, 4 eps || P_free |A_{k-1}| |q_k| ||).
// Returns 0 converged, 1 Newton iteration cap, 2 line search failed,
// 3 no positive definite system within the regulariser cap.
// f_ext (nullable): external nodal generalized forces [nodes][12], added to
// the areal gravity load.
int newton_step(const Shell& s, const double* qb, const uint8_t* fixed, double dt, const double* qn, const double* vn,
                const double* qpresc, const double* f_ext, const NewtonOpts& o, double* qn1, double* vn1,
                NewtonStats* st, NewtonTrace* trace = nullptr, AlmOpts* alm = nullptr);

}  // namespace orc
