// Positional constraints at arbitrary midsurface points (Sec. 4.2) imposed
// by the augmented Lagrangian method (Sec. 6.1).  Constraint j prescribes
// x^(kind)(xi_j) (the position or a first derivative of the midsurface at
// a parameter point, 3 rows), c_j = sum_I psi_I q_I - target_j with psi
// the 16 shape-function values of that kind on the point's patch.  The
// Newton iterations minimise E(q) - lambda.c + (kappa/2)|c|^2:
//   * k_alm_grad adds C^T (kappa c - lambda) to the gradient, per node DOF
//     over its incidences in a fixed order (deterministic);
//   * k_alm_energy adds -lambda.c + (kappa/2)|c|^2 to each shell's energy;
//   * k_add_sparse adds kappa C^T C, merged on the host into one value per
//     stored matrix entry, after the assembly;
//   * k_alm_residual gives c for the multiplier update on the host.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bhem {

__device__ inline double alm_c(const AlmPoint& pt, const double* __restrict__ q, int comp) {
    double v = -pt.target[comp];
#pragma unroll
    for (int I = 0; I < 16; ++I) v += pt.psi[I] * q[12 * (size_t)pt.node[I >> 2] + 3 * (I & 3) + comp];
    return v;
}

__global__ void k_alm_grad(int nnodes, const int* __restrict__ incp, const int2* __restrict__ inc,
                           const AlmPoint* __restrict__ pts, const double* __restrict__ lam, double kappa,
                           const double* __restrict__ q, const uint16_t* __restrict__ fm,
                           const int* __restrict__ node_shell, const int* __restrict__ write_shell,
                           double* __restrict__ grad) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnodes * 12) return;
    const int node = t / 12, w = t % 12, k = w / 3, comp = w % 3;
    if (incp[node] == incp[node + 1]) return;
    if (write_shell && !write_shell[node_shell[node]]) return;
    if (fm && !((fm[node] >> w) & 1u)) return;
    double acc = 0.0;
    for (int e = incp[node]; e < incp[node + 1]; ++e) {
        const int j = inc[e].x, c = inc[e].y;
        const AlmPoint& pt = pts[j];
        acc += (kappa * alm_c(pt, q, comp) - lam[3 * j + comp]) * pt.psi[4 * c + k];
    }
    grad[t] += acc;
}

// one thread per shell, its points in order: e_shell[3 s + 2] += sum -lambda.c + kappa/2 |c|^2
__global__ void k_alm_energy(int nshell, const int* __restrict__ shell_pt, const AlmPoint* __restrict__ pts,
                             const double* __restrict__ lam, double kappa, const double* __restrict__ q,
                             double* __restrict__ e_shell) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nshell || shell_pt[s] == shell_pt[s + 1]) return;
    double e = 0.0;
    for (int j = shell_pt[s]; j < shell_pt[s + 1]; ++j)
        for (int comp = 0; comp < 3; ++comp) {
            const double c = alm_c(pts[j], q, comp);
            e += -lam[3 * j + comp] * c + 0.5 * kappa * c * c;
        }
    e_shell[3 * s + 2] += e;
}

__global__ void k_alm_residual(int npts, const AlmPoint* __restrict__ pts, const double* __restrict__ q,
                               double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * npts) return;
    out[t] = alm_c(pts[t / 3], q, t % 3);
}

// vals[pos[i]] += val[i] (distinct positions)
template <class T>
__global__ void k_add_sparse(int n, const long long* __restrict__ pos, const double* __restrict__ val,
                             T* __restrict__ vals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) vals[pos[i]] += (T)val[i];
}

void launch_alm_grad(hipStream_t st, int nnodes, const int* incp, const int2* inc, const AlmPoint* pts,
                     const double* lam, double kappa, const double* q, const uint16_t* fm, const int* node_shell,
                     const int* write_shell, double* grad) {
    hipLaunchKernelGGL(k_alm_grad, dim3((unsigned)((nnodes * 12 + 255) / 256)), dim3(256), 0, st, nnodes, incp, inc,
                       pts, lam, kappa, q, fm, node_shell, write_shell, grad);
}
void launch_alm_energy(hipStream_t st, int nshell, const int* shell_pt, const AlmPoint* pts, const double* lam,
                       double kappa, const double* q, double* e_shell) {
    hipLaunchKernelGGL(k_alm_energy, dim3((unsigned)((nshell + 63) / 64)), dim3(64), 0, st, nshell, shell_pt, pts, lam,
                       kappa, q, e_shell);
}
void launch_alm_residual(hipStream_t st, int npts, const AlmPoint* pts, const double* q, double* out) {
    hipLaunchKernelGGL(k_alm_residual, dim3((unsigned)((3 * npts + 255) / 256)), dim3(256), 0, st, npts, pts, q, out);
}
void launch_add_sparse(hipStream_t st, int n, const long long* pos, const double* val, void* vals, int vals_fp32) {
    if (n == 0) return;
    if (vals_fp32)
        hipLaunchKernelGGL(k_add_sparse<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, pos, val,
                           (float*)vals);
    else
        hipLaunchKernelGGL(k_add_sparse<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, pos, val,
                           (double*)vals);
}

}  // namespace bhem
