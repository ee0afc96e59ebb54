// Control kernels of the device-driven Newton iteration (libbhem, gfx950).
//
// One implicit-Euler step is Newton's method on the incremental potential
// (Sec. 6.1) with a backtracking line search; every decision of one Newton
// iteration -- which shells still iterate, which take the block-Jacobi
// failure branch, the refinement sweeps of the mixed form, the Armijo test
// and the interpolated step lengths -- is taken here, one thread per shell,
// on per-shell state (NewtonCtl) between the iteration's matrix and vector
// kernels, so the whole iteration is one launch sequence the host captures
// once and reads back once.  The expressions and their order are those of
// the host-driven iteration in shell_api.hip, with floating-point
// contraction off in this file, so both paths take the same decisions on
// the same values.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

#pragma clang fp contract(off)

namespace bhem {

namespace {
constexpr double kEps = 2.220446049250313e-16;

__device__ __forceinline__ int shell_id() { return blockIdx.x * blockDim.x + threadIdx.x; }
}  // namespace

// After the block-Jacobi factorisation: a shell whose diagonal block failed
// leaves the device path (the host regularises it); the others are the
// shells this iteration solves for.
__global__ void k_nt_factor(int S, NewtonCtl* __restrict__ ctl, const int* __restrict__ fail_shell,
                            int* __restrict__ cg_active, double* __restrict__ cg_rtol2, int* __restrict__ cg_maxit,
                            double pcg_rtol, int pcg_maxit) {
    const int s = shell_id();
    if (s >= S) return;
    NewtonCtl& c = ctl[s];
    c.need_host = 0;
    c.searching = 0;
    c.steepest = 0;
    c.solving = 0;
    if (c.active && fail_shell[s]) c.need_host = NT_HOST_FACTOR;
    c.solving = c.active && !c.need_host;
    cg_active[s] = c.solving;
    cg_rtol2[s] = pcg_rtol * pcg_rtol;
    cg_maxit[s] = pcg_maxit;
}

// FP64 solve: one CG launch.  p^T A p <= 0 (status 2) hands the shell to the
// host (regulariser); the other statuses keep the direction as it is.
__global__ void k_nt_cg64(int S, NewtonCtl* __restrict__ ctl, const CgShellOut* __restrict__ out,
                          int* __restrict__ flag_shell) {
    const int s = shell_id();
    if (s >= S) return;
    NewtonCtl& c = ctl[s];
    flag_shell[s] = c.solving;
    if (!c.solving) return;
    c.pcg_iters += out[s].iters;
    c.sweeps += 1;
    if (out[s].status == 3) c.fault = 1;
    if (out[s].status == 2) {
        c.need_host = NT_HOST_INDEFINITE;
        c.solving = 0;
    }
}

// Mixed form, before the first sweep: bn2 = ||b||^2 (red), prev = 1.
__global__ void k_nt_ref_init(int S, NewtonCtl* __restrict__ ctl, const double* __restrict__ red,
                              int* __restrict__ cg_active, double* __restrict__ cg_rtol2, double pcg_rtol) {
    const int s = shell_id();
    if (s >= S) return;
    NewtonCtl& c = ctl[s];
    c.bn2 = red[s];
    c.prev = 1.0;
    c.solve_iters = 0;
    c.refining = c.solving && c.bn2 != 0.0;
    cg_active[s] = c.refining;
    const double inner = fmax(0.5 * pcg_rtol / c.prev, 1e-6);
    cg_rtol2[s] = inner * inner;
}

// Mixed form, after a sweep's FP32 CG: iterations, sweeps, p^T A p <= 0.
__global__ void k_nt_ref_cg(int S, NewtonCtl* __restrict__ ctl, const CgShellOut* __restrict__ out,
                            int* __restrict__ cg_active) {
    const int s = shell_id();
    if (s >= S) return;
    NewtonCtl& c = ctl[s];
    if (!c.refining) return;
    c.pcg_iters += out[s].iters;
    c.solve_iters += out[s].iters;
    c.sweeps += 1;
    if (out[s].status == 3) c.fault = 1;
    if (out[s].status == 2) {
        c.need_host = NT_HOST_INDEFINITE;
        c.refining = 0;
        c.solving = 0;
        cg_active[s] = 0;
    }
}

// Mixed form, after a sweep's FP64 residual (red = ||r||^2): converged,
// stagnating, or the next sweep's inner tolerance.
__global__ void k_nt_ref_check(int S, NewtonCtl* __restrict__ ctl, const double* __restrict__ red,
                               int* __restrict__ cg_active, double* __restrict__ cg_rtol2, double pcg_rtol,
                               int pcg_maxit) {
    const int s = shell_id();
    if (s >= S) return;
    NewtonCtl& c = ctl[s];
    if (c.refining) {
        const double rel = sqrt(red[s] / c.bn2);
        c.relres = rel;
        if (rel <= pcg_rtol) {
            c.refining = 0;
        } else if (rel > 0.5 * c.prev || c.solve_iters >= pcg_maxit) {
            c.refining = 0;   // refinement stagnates: the direction as it is
        }
        c.prev = rel;
    }
    cg_active[s] = c.refining;
    const double inner = fmax(0.5 * pcg_rtol / c.prev, 1e-6);
    cg_rtol2[s] = inner * inner;
}

// Mixed form, after the last device sweep: shells still refining go on on
// the host; flag_shell marks the shells whose direction is written now.
__global__ void k_nt_ref_end(int S, NewtonCtl* __restrict__ ctl, int* __restrict__ flag_shell) {
    const int s = shell_id();
    if (s >= S) return;
    NewtonCtl& c = ctl[s];
    if (c.refining) c.need_host = NT_HOST_REFINE;
    flag_shell[s] = c.solving;
}

// Line search start (red = g.d): the shells with a direction search from
// alpha = 1; a direction that is not one of descent is replaced by -g
// (flag_shell marks those shells).
__global__ void k_nt_ls_init(int S, NewtonCtl* __restrict__ ctl, const double* __restrict__ red,
                             double* __restrict__ alpha_shell, int* __restrict__ flag_shell,
                             int* __restrict__ write_shell) {
    const int s = shell_id();
    if (s >= S) return;
    NewtonCtl& c = ctl[s];
    c.searching = c.active && !c.need_host;
    c.steepest = 0;
    c.trial = 0;
    if (c.searching) {
        c.alpha = 1.0;
        c.slope = red[s];
        if (!(c.slope < 0.0)) {
            c.steepest = 1;
            c.slope = -c.gn * c.gn;
        }
    }
    flag_shell[s] = c.steepest;
    alpha_shell[s] = c.searching ? c.alpha : 0.0;
    write_shell[s] = c.searching;
}

// One line-search trial (energies e_shell, red = ||g(q_t)||^2): Armijo test
// (or, at the rounding level of E, a smaller gradient), else the next step
// length by a quadratic (first trial) or cubic fit, kept in [0.1, 0.5] of
// the last.  flag_shell marks the shells that accept q_t.
__global__ void k_nt_ls_step(int S, int trial, NewtonCtl* __restrict__ ctl, const double* __restrict__ e_shell,
                             const double* __restrict__ red, double* __restrict__ alpha_shell,
                             int* __restrict__ flag_shell, int* __restrict__ write_shell) {
    const int s = shell_id();
    if (s >= S) return;
    NewtonCtl& c = ctl[s];
    flag_shell[s] = 0;
    if (c.searching) {
        const double* e = e_shell + 3 * s;
        const double Et = e[0] + e[1] + e[2];
        const double sc_t = fabs(e[0]) + fabs(e[1]) + fabs(e[2]);
        const double gtn = sqrt(red[s]);
        bool ok = false;
        if (isfinite(Et) && isfinite(gtn)) {
            if (Et <= c.E + 1e-4 * c.alpha * c.slope) ok = true;
            const double noise = 1e-12 * fmax(c.Escale, sc_t);
            if (-c.slope <= noise && fabs(Et - c.E) <= noise && gtn < c.gn) ok = true;
        }
        if (ok) {
            flag_shell[s] = 1;
            c.searching = 0;
            c.E = Et;
            c.Escale = sc_t;
            c.gn = gtn;
        } else {
            double an;
            const double a = c.alpha;
            if (!isfinite(Et)) {
                an = 0.1 * a;
            } else if (trial == 0) {
                an = -c.slope * a * a / (2.0 * (Et - c.E - c.slope * a));
            } else {
                const double ap = c.a_prev;
                const double d1 = Et - c.E - c.slope * a, d2 = c.E_prev - c.E - c.slope * ap;
                const double den = ap * ap * a * a * (a - ap);
                const double ca = (ap * ap * d1 - a * a * d2) / den;
                const double cb = (-ap * ap * ap * d1 + a * a * a * d2) / den;
                if (ca == 0.0) {
                    an = -c.slope / (2.0 * cb);
                } else {
                    const double disc = cb * cb - 3.0 * ca * c.slope;
                    an = disc >= 0.0 ? (-cb + sqrt(disc)) / (3.0 * ca) : 0.5 * a;
                }
            }
            if (!isfinite(an)) an = 0.5 * a;
            an = fmin(fmax(an, 0.1 * a), 0.5 * a);
            c.a_prev = a;
            c.E_prev = Et;
            c.alpha = an;
            c.backtracks++;
        }
        c.trial = trial + 1;
    }
    alpha_shell[s] = c.searching ? c.alpha : 0.0;
    write_shell[s] = c.searching;
}

// End of the iteration's line search: the shells that finished on the
// device count the iteration; a search still going on continues on the host.
__global__ void k_nt_ls_end(int S, NewtonCtl* __restrict__ ctl) {
    const int s = shell_id();
    if (s >= S) return;
    NewtonCtl& c = ctl[s];
    if (!c.active || c.need_host) return;
    if (c.searching) {
        c.need_host = NT_HOST_LINESEARCH;
        return;
    }
    c.k += 1;
    c.newton_iters += 1;
}

// Convergence test for the next iteration of the shells that finished this
// one on the device (red = || P_free |A| |q| ||^2, the rounding floor of the
// gradient from this iteration's matrix).
__global__ void k_nt_check(int S, NewtonCtl* __restrict__ ctl, const double* __restrict__ red, double newton_rtol,
                           int newton_maxit) {
    const int s = shell_id();
    if (s >= S) return;
    NewtonCtl& c = ctl[s];
    if (!c.active || c.need_host) return;
    c.floor = 4.0 * kEps * sqrt(red[s]);
    c.grad_norm_checked = c.gn;
    if (c.gn == 0.0 || (c.k > 0 && c.gn <= fmax(newton_rtol * c.g0, c.floor))) {
        c.status = NT_STATUS_OK;
        c.active = 0;
    } else if (c.k == newton_maxit) {
        c.status = NT_STATUS_NOT_CONVERGED;
        c.active = 0;
    }
}

// ------------------------------------------------------------ launchers
static inline dim3 sgrid(int S) { return dim3((S + 255) / 256); }

void launch_nt_factor(hipStream_t st, int S, NewtonCtl* ctl, const int* fail_shell, int* cg_active, double* cg_rtol2,
                      int* cg_maxit, double pcg_rtol, int pcg_maxit) {
    hipLaunchKernelGGL(k_nt_factor, sgrid(S), dim3(256), 0, st, S, ctl, fail_shell, cg_active, cg_rtol2, cg_maxit,
                       pcg_rtol, pcg_maxit);
}
void launch_nt_cg64(hipStream_t st, int S, NewtonCtl* ctl, const CgShellOut* out, int* flag_shell) {
    hipLaunchKernelGGL(k_nt_cg64, sgrid(S), dim3(256), 0, st, S, ctl, out, flag_shell);
}
void launch_nt_ref_init(hipStream_t st, int S, NewtonCtl* ctl, const double* red, int* cg_active, double* cg_rtol2,
                        double pcg_rtol) {
    hipLaunchKernelGGL(k_nt_ref_init, sgrid(S), dim3(256), 0, st, S, ctl, red, cg_active, cg_rtol2, pcg_rtol);
}
void launch_nt_ref_cg(hipStream_t st, int S, NewtonCtl* ctl, const CgShellOut* out, int* cg_active) {
    hipLaunchKernelGGL(k_nt_ref_cg, sgrid(S), dim3(256), 0, st, S, ctl, out, cg_active);
}
void launch_nt_ref_check(hipStream_t st, int S, NewtonCtl* ctl, const double* red, int* cg_active, double* cg_rtol2,
                         double pcg_rtol, int pcg_maxit) {
    hipLaunchKernelGGL(k_nt_ref_check, sgrid(S), dim3(256), 0, st, S, ctl, red, cg_active, cg_rtol2, pcg_rtol,
                       pcg_maxit);
}
void launch_nt_ref_end(hipStream_t st, int S, NewtonCtl* ctl, int* flag_shell) {
    hipLaunchKernelGGL(k_nt_ref_end, sgrid(S), dim3(256), 0, st, S, ctl, flag_shell);
}
void launch_nt_ls_init(hipStream_t st, int S, NewtonCtl* ctl, const double* red, double* alpha_shell,
                       int* flag_shell, int* write_shell) {
    hipLaunchKernelGGL(k_nt_ls_init, sgrid(S), dim3(256), 0, st, S, ctl, red, alpha_shell, flag_shell, write_shell);
}
void launch_nt_ls_step(hipStream_t st, int S, int trial, NewtonCtl* ctl, const double* e_shell, const double* red,
                       double* alpha_shell, int* flag_shell, int* write_shell) {
    hipLaunchKernelGGL(k_nt_ls_step, sgrid(S), dim3(256), 0, st, S, trial, ctl, e_shell, red, alpha_shell,
                       flag_shell, write_shell);
}
void launch_nt_ls_end(hipStream_t st, int S, NewtonCtl* ctl) {
    hipLaunchKernelGGL(k_nt_ls_end, sgrid(S), dim3(256), 0, st, S, ctl);
}
void launch_nt_check(hipStream_t st, int S, NewtonCtl* ctl, const double* red, double newton_rtol, int newton_maxit) {
    hipLaunchKernelGGL(k_nt_check, sgrid(S), dim3(256), 0, st, S, ctl, red, newton_rtol, newton_maxit);
}

}  // namespace bhem
