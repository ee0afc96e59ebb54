// Collision handling of shells against static colliders (Sec. 6.2,
// "Collision Handling"), the data-parallel parts:
//   * k_coll_samples: every patch's midsurface sampled at s x s parameter
//     points; one thread per sample evaluates the point at the step's start
//     and end (the generalized coordinates move linearly over an implicit
//     Euler step, so the point moves on a straight line) and its earliest
//     contact time with the colliders (plane: a linear root; sphere: the
//     smaller root of a quadratic); per block the smallest time;
//   * k_coll_count / k_coll_compact: the samples within the simultaneity
//     window of the earliest contact, listed in sample order (a per-block
//     count, an exclusive scan of the counts, then each block writes its
//     samples in thread order: deterministic);
//   * k_coll_setup: per listed contact its 16 shape-function values, nodes,
//     point at the rolled-back state, collider normal, tangents, point on
//     the collider and normal velocity;
//   * k_coll_scatter / k_coll_gather: J^T lambda as nodal generalized
//     forces (per node DOF, its incidences in a fixed order) and J z (per
//     constraint row), the two halves of every product with J M^-1 J^T.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace bhem {

// 16 shape-function values of local coordinate I = 4c + k at (t1, t2):
// w_{p,r}(t1) w_{q,s}(t2) dxi1^r dxi2^s, c = p + 2q, k = r + 2s
__device__ inline void coll_phi(double t1, double t2, double d1, double d2, double phi[16]) {
#pragma unroll
    for (int I = 0; I < 16; ++I) {
        const int c = I >> 2, k = I & 3;
        const int p = c & 1, q = c >> 1, r = k & 1, s = k >> 1;
        phi[I] = hermite(p, r, 0, t1) * hermite(q, s, 0, t2) * (r ? d1 : 1.0) * (s ? d2 : 1.0);
    }
}

__device__ inline void coll_point(const double* __restrict__ q, const int4 nd, const double phi[16], double x[3]) {
    const int node[4] = {nd.x, nd.y, nd.z, nd.w};
    x[0] = x[1] = x[2] = 0.0;
#pragma unroll
    for (int I = 0; I < 16; ++I) {
        const double* v = q + 12 * (size_t)node[I >> 2] + 3 * (I & 3);
        x[0] += phi[I] * v[0];
        x[1] += phi[I] * v[1];
        x[2] += phi[I] * v[2];
    }
}

// earliest tau in [0, dt] at which x0 + tau v meets the collider, or inf
__device__ inline double coll_time(const CollCollider& col, const double x0[3], const double v[3], double dt) {
    if (col.kind == 0) {
        const double d0 = col.n[0] * (x0[0] - col.p[0]) + col.n[1] * (x0[1] - col.p[1]) + col.n[2] * (x0[2] - col.p[2]);
        if (d0 <= 0.0) return 0.0;
        const double dv = col.n[0] * v[0] + col.n[1] * v[1] + col.n[2] * v[2];
        if (dv >= 0.0) return INFINITY;
        const double t = -d0 / dv;
        return t <= dt ? t : INFINITY;
    }
    const double e0 = x0[0] - col.p[0], e1 = x0[1] - col.p[1], e2 = x0[2] - col.p[2];
    const double c0 = e0 * e0 + e1 * e1 + e2 * e2 - col.r * col.r;
    if (c0 <= 0.0) return 0.0;
    const double a = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double b = 2.0 * (e0 * v[0] + e1 * v[1] + e2 * v[2]);
    if (b >= 0.0 || a == 0.0) return INFINITY;
    const double disc = b * b - 4.0 * a * c0;
    if (disc < 0.0) return INFINITY;
    const double t = (-b - sqrt(disc)) / (2.0 * a);
    return t <= dt ? t : INFINITY;
}

__global__ void __launch_bounds__(256) k_coll_samples(int nsamp, int s, const int4* __restrict__ patch_nodes,
                                                      const int* __restrict__ patch_shell,
                                                      const ShellParams* __restrict__ shells,
                                                      const double* __restrict__ qn, const double* __restrict__ q1,
                                                      double dt, const CollCollider* __restrict__ cols, int ncol,
                                                      double* __restrict__ tc, int* __restrict__ cid,
                                                      double* __restrict__ blk_min) {
    __shared__ double wmin[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double best = INFINITY;
    if (i < nsamp) {
        const int ss = s * s, p = i / ss, a = (i % ss) % s, b = (i % ss) / s;
        const ShellParams& sp = shells[patch_shell[p]];
        double phi[16], x0[3], x1[3], v[3];
        coll_phi((a + 0.5) / s, (b + 0.5) / s, sp.dxi1, sp.dxi2, phi);
        const int4 nd = patch_nodes[p];
        coll_point(qn, nd, phi, x0);
        coll_point(q1, nd, phi, x1);
        for (int c = 0; c < 3; ++c) v[c] = (x1[c] - x0[c]) / dt;
        int k = -1;
        for (int j = 0; j < ncol; ++j) {
            const double t = coll_time(cols[j], x0, v, dt);
            if (t < best) {
                best = t;
                k = j;
            }
        }
        tc[i] = best;
        cid[i] = k;
    }
    for (int off = 32; off > 0; off >>= 1) best = fmin(best, __shfl_xor(best, off));
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) blk_min[blockIdx.x] = fmin(fmin(wmin[0], wmin[1]), fmin(wmin[2], wmin[3]));
}

__global__ void __launch_bounds__(256) k_coll_count(int nsamp, const double* __restrict__ tc, double thr,
                                                    int* __restrict__ blk_cnt) {
    __shared__ int wc[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < nsamp && tc[i] <= thr;
    const unsigned long long bal = __ballot(in);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

__global__ void __launch_bounds__(256) k_coll_compact(int nsamp, const double* __restrict__ tc, double thr,
                                                      const int* __restrict__ blk_off, int* __restrict__ list) {
    __shared__ int wc[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool in = i < nsamp && tc[i] <= thr;
    const unsigned long long bal = __ballot(in);
    if (lane == 0) wc[wave] = __popcll(bal);
    __syncthreads();
    int base = blk_off[blockIdx.x];
    for (int w = 0; w < wave; ++w) base += wc[w];
    if (in) list[base + __popcll(bal & ((1ull << lane) - 1))] = i;
}

// q_out = qn + f (q1 - qn), f = tau* / dt
__global__ void k_coll_rollback(int n, const double* __restrict__ qn, const double* __restrict__ q1, double f,
                                double* __restrict__ qs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) qs[i] = qn[i] + f * (q1[i] - qn[i]);
}

__global__ void __launch_bounds__(64) k_coll_setup(int ncon, int s, const int* __restrict__ list,
                                                   const int* __restrict__ cid, const int4* __restrict__ patch_nodes,
                                                   const int* __restrict__ patch_shell,
                                                   const ShellParams* __restrict__ shells,
                                                   const double* __restrict__ qs, const double* __restrict__ v,
                                                   const CollCollider* __restrict__ cols,
                                                   CollContact* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncon) return;
    CollContact ct;
    const int i = list[k], ss = s * s, p = i / ss, a = (i % ss) % s, b = (i % ss) / s;
    const ShellParams& sp = shells[patch_shell[p]];
    coll_phi((a + 0.5) / s, (b + 0.5) / s, sp.dxi1, sp.dxi2, ct.phi);
    const int4 nd = patch_nodes[p];
    ct.sample = i;
    ct.collider = cid[i];
    ct.node[0] = nd.x;
    ct.node[1] = nd.y;
    ct.node[2] = nd.z;
    ct.node[3] = nd.w;
    coll_point(qs, nd, ct.phi, ct.x);
    double vel[3];
    coll_point(v, nd, ct.phi, vel);
    const CollCollider& col = cols[ct.collider];
    double n[3];
    if (col.kind == 0) {
        for (int c = 0; c < 3; ++c) n[c] = col.n[c];
        const double d = n[0] * (ct.x[0] - col.p[0]) + n[1] * (ct.x[1] - col.p[1]) + n[2] * (ct.x[2] - col.p[2]);
        for (int c = 0; c < 3; ++c) ct.p[c] = ct.x[c] - d * n[c];
    } else {
        const double e0 = ct.x[0] - col.p[0], e1 = ct.x[1] - col.p[1], e2 = ct.x[2] - col.p[2];
        const double l = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        n[0] = e0 / l;
        n[1] = e1 / l;
        n[2] = e2 / l;
        for (int c = 0; c < 3; ++c) ct.p[c] = col.p[c] + col.r * n[c];
    }
    // tangents: the axis least aligned with n crossed with n, then n x t1
    const double an[3] = {fabs(n[0]), fabs(n[1]), fabs(n[2])};
    const int e = (an[0] <= an[1] && an[0] <= an[2]) ? 0 : (an[1] <= an[2] ? 1 : 2);
    double t1[3] = {e == 0 ? 0.0 : (e == 1 ? n[2] : -n[1]), e == 0 ? -n[2] : (e == 1 ? 0.0 : n[0]),
                    e == 0 ? n[1] : (e == 1 ? -n[0] : 0.0)};
    const double l1 = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    for (int c = 0; c < 3; ++c) t1[c] /= l1;
    const double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
    for (int c = 0; c < 3; ++c) {
        ct.dir[0][c] = n[c];
        ct.dir[1][c] = t1[c];
        ct.dir[2][c] = t2[c];
    }
    ct.vn = n[0] * vel[0] + n[1] * vel[1] + n[2] * vel[2];
    out[k] = ct;
}

// y[n][12] = sum over node n's incidences (row r of constraint slot, corner
// c): lam[r] dir(r) phi_{4c + k}; rows of contact j are row_of[j] ..
// row_of[j] + m - 1 with directions dir[0 .. m-1] (m = 0: contact not in
// this system).  Prescribed DOFs get 0.
__global__ void k_coll_scatter(int nnodes, const int* __restrict__ inc_ptr, const int2* __restrict__ inc,
                               const CollContact* __restrict__ con, const int* __restrict__ row_of, int m,
                               const double* __restrict__ lam, const uint16_t* __restrict__ fm,
                               double* __restrict__ y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnodes * 12) return;
    const int node = t / 12, w = t % 12, k = w / 3, comp = w % 3;
    double acc = 0.0;
    if ((fm[node] >> w) & 1u)
        for (int e = inc_ptr[node]; e < inc_ptr[node + 1]; ++e) {
            const int j = inc[e].x, c = inc[e].y;
            const int r0 = row_of[j];
            if (r0 < 0) continue;
            const CollContact& ct = con[j];
            double f = 0.0;
            for (int d = 0; d < m; ++d) f += lam[r0 + d] * ct.dir[d][comp];
            acc += f * ct.phi[4 * c + k];
        }
    y[t] = acc;
}

// out[row] = dir(row) . sum_I phi_I z[node(I)][3k(I) ..] for every row of
// the system (rows of contact j: row_of[j] + d, d < m)
__global__ void k_coll_gather(int ncon, const CollContact* __restrict__ con, const int* __restrict__ row_of, int m,
                              const double* __restrict__ z, double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ncon) return;
    const int r0 = row_of[j];
    if (r0 < 0) return;
    const CollContact& ct = con[j];
    double x[3] = {0.0, 0.0, 0.0};
    for (int I = 0; I < 16; ++I) {
        const double* v = z + 12 * (size_t)ct.node[I >> 2] + 3 * (I & 3);
        x[0] += ct.phi[I] * v[0];
        x[1] += ct.phi[I] * v[1];
        x[2] += ct.phi[I] * v[2];
    }
    for (int d = 0; d < m; ++d) out[r0 + d] = ct.dir[d][0] * x[0] + ct.dir[d][1] * x[1] + ct.dir[d][2] * x[2];
}

// ------------------------------------------------------------ launchers
static dim3 grid256(long long n) { return dim3((unsigned)((n + 255) / 256)); }

void launch_coll_samples(hipStream_t st, int nsamp, int s, const int4* patch_nodes, const int* patch_shell,
                         const ShellParams* shells, const double* qn, const double* q1, double dt,
                         const CollCollider* cols, int ncol, double* tc, int* cid, double* blk_min) {
    hipLaunchKernelGGL(k_coll_samples, grid256(nsamp), dim3(256), 0, st, nsamp, s, patch_nodes, patch_shell, shells,
                       qn, q1, dt, cols, ncol, tc, cid, blk_min);
}
void launch_coll_count(hipStream_t st, int nsamp, const double* tc, double thr, int* blk_cnt) {
    hipLaunchKernelGGL(k_coll_count, grid256(nsamp), dim3(256), 0, st, nsamp, tc, thr, blk_cnt);
}
void launch_coll_compact(hipStream_t st, int nsamp, const double* tc, double thr, const int* blk_off, int* list) {
    hipLaunchKernelGGL(k_coll_compact, grid256(nsamp), dim3(256), 0, st, nsamp, tc, thr, blk_off, list);
}
void launch_coll_rollback(hipStream_t st, int n, const double* qn, const double* q1, double f, double* qs) {
    hipLaunchKernelGGL(k_coll_rollback, grid256(n), dim3(256), 0, st, n, qn, q1, f, qs);
}
void launch_coll_setup(hipStream_t st, int ncon, int s, const int* list, const int* cid, const int4* patch_nodes,
                       const int* patch_shell, const ShellParams* shells, const double* qs, const double* v,
                       const CollCollider* cols, CollContact* out) {
    hipLaunchKernelGGL(k_coll_setup, dim3((unsigned)((ncon + 63) / 64)), dim3(64), 0, st, ncon, s, list, cid,
                       patch_nodes, patch_shell, shells, qs, v, cols, out);
}
void launch_coll_scatter(hipStream_t st, int nnodes, const int* inc_ptr, const int2* inc, const CollContact* con,
                         const int* row_of, int m, const double* lam, const uint16_t* fm, double* y) {
    hipLaunchKernelGGL(k_coll_scatter, grid256((long long)nnodes * 12), dim3(256), 0, st, nnodes, inc_ptr, inc, con,
                       row_of, m, lam, fm, y);
}
void launch_coll_gather(hipStream_t st, int ncon, const CollContact* con, const int* row_of, int m, const double* z,
                        double* out) {
    hipLaunchKernelGGL(k_coll_gather, grid256(ncon), dim3(256), 0, st, ncon, con, row_of, m, z, out);
}

}  // namespace bhem
