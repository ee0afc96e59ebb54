// Sparse linear algebra of libbhem (gfx950): 12x12-block matrix products,
// block-Jacobi factorisation, the persistent block-Jacobi conjugate gradient
// and per-shell reductions.
//
// Matrix storage: block rows per node (row_ptr / col_idx over nodes); each
// 12x12 block is stored column-major (entry (r, c) at c*12 + r) so that the
// lanes owning consecutive rows of a block read consecutive memory.  Rows and
// columns of prescribed DOFs stay in the matrix; the solver masks them
// (free-DOF bit masks per node), which equals replacing them by identity rows
// and columns with a zero right-hand side.
//
// SpMV lane layout: a node row is handled by L = 12/R lanes, each owning R
// consecutive rows of the 12 (R = 2 for FP64 blocks, 4 for FP32), so each
// column of a block is one 16-byte load per lane; the 12 x-values of a
// column block are exchanged within the lane group by cross-lane reads.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace bhem {

template <class TM> struct Lay {
    static constexpr int R = 16 / sizeof(TM);   // rows per lane
    static constexpr int L = 12 / R;             // lanes per node row
    static constexpr int G = 64 / L;             // node rows per wavefront
};

__device__ __forceinline__ bool is_free(const uint16_t* m, int node, int w) { return !m || ((m[node] >> w) & 1); }

template <class TM, int R> struct VecLoad;
template <> struct VecLoad<double, 2> {
    static __device__ __forceinline__ void ld(const double* p, double* o) {
        const double2 v = *reinterpret_cast<const double2*>(p);
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <> struct VecLoad<float, 4> {
    static __device__ __forceinline__ void ld(const float* p, float* o) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};

// acc[0..R) = rows R*t .. R*t+R-1 of (block row `node`) times x_eff, where
// xe(col, xv) supplies this lane's R values of column block `col`.  The next
// block's column index and x-values are fetched while the current block is
// multiplied, so the dependent index -> vector load chain overlaps the
// matrix stream.
template <class TM, class TV, class XF>
__device__ __forceinline__ void row_times(const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                                          const TM* __restrict__ vals, int node, int t, int gbase, bool absval,
                                          XF xe, TV* acc) {
    constexpr int R = Lay<TM>::R;
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = TV(0);
    const int b0 = row_ptr[node], b1 = row_ptr[node + 1];
    if (b0 >= b1) return;
    TV xv[R];
    xe(col_idx[b0], xv);
    for (int b = b0; b < b1; ++b) {
        TV xn[R];
        if (b + 1 < b1) xe(col_idx[b + 1], xn);
        const TM* blk = vals + (size_t)b * 144 + R * t;
        TM a[12][R];
#pragma unroll
        for (int c = 0; c < 12; ++c) VecLoad<TM, R>::ld(blk + c * 12, a[c]);
        if (absval)
#pragma unroll
            for (int i = 0; i < R; ++i) xv[i] = fabs(xv[i]);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const TV xc = __shfl(xv[c % R], gbase + c / R);
#pragma unroll
            for (int i = 0; i < R; ++i) acc[i] += (absval ? (TV)fabs(a[c][i]) : (TV)a[c][i]) * xc;
        }
#pragma unroll
        for (int i = 0; i < R; ++i) xv[i] = xn[i];
    }
}

// Same product for the CG, whose x-values are formed from two vectors
// (z + beta p): the column indices and x-values of a group of MB blocks are
// loaded first, all at once, so the matrix loads of the group do not wait
// on the dependent index -> vector chain block by block (that chain, with
// one wait per block, cost ~10% of a CG iteration).  Blocks past the row's
// end re-read a block of the row with x = 0.
template <class TM, class TV, class XF>
__device__ __forceinline__ void row_times_grouped(const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                                          const TM* __restrict__ vals, int node, int t, int gbase, bool absval,
                                          XF xe, TV* acc) {
    constexpr int R = Lay<TM>::R, MB = 3;
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = TV(0);
    const int b0 = row_ptr[node], b1 = row_ptr[node + 1];
    for (int bc = b0; bc < b1; bc += MB) {
        const int nb = min(MB, b1 - bc);
        int cl[MB];
#pragma unroll
        for (int u = 0; u < MB; ++u) cl[u] = col_idx[bc + (u < nb ? u : 0)];
        TV xv[MB][R];
#pragma unroll
        for (int u = 0; u < MB; ++u) {
            xe(cl[u], xv[u]);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                if (u >= nb) xv[u][i] = TV(0);
                if (absval) xv[u][i] = fabs(xv[u][i]);
            }
        }
#pragma unroll
        for (int u = 0; u < MB; ++u) {
            const TM* blk = vals + (size_t)(bc + (u < nb ? u : 0)) * 144 + R * t;
            TM a[12][R];
#pragma unroll
            for (int c = 0; c < 12; ++c) VecLoad<TM, R>::ld(blk + c * 12, a[c]);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const TV xc = __shfl(xv[u][c % R], gbase + c / R);
#pragma unroll
                for (int i = 0; i < R; ++i) acc[i] += (absval ? (TV)fabs(a[c][i]) : (TV)a[c][i]) * xc;
            }
        }
    }
}

// ------------------------------------------------------------------ SpMV
template <class TM>
__global__ __launch_bounds__(256) void k_spmv(int nnodes, const int* __restrict__ row_ptr,
                                              const int* __restrict__ col_idx, const TM* __restrict__ vals,
                                              const uint16_t* __restrict__ fm, const double* __restrict__ x,
                                              const double* __restrict__ b, double* __restrict__ y, int mode) {
    constexpr int R = Lay<TM>::R, L = Lay<TM>::L, G = Lay<TM>::G;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane / L, t = lane % L;
    const int node = (blockIdx.x * 4 + wv) * G + grp;
    if (grp >= G || node >= nnodes) return;
    const bool absval = mode & 2, resid = mode & 4;
    const uint16_t* m = (mode & 1) ? fm : nullptr;          // free columns only
    const uint16_t* mr = (mode & (1 | 8)) ? fm : nullptr;   // free rows only
    double acc[R];
    row_times<TM, double>(row_ptr, col_idx, vals, node, t, lane - t, absval,
                          [&](int col, double* xv) {
                              // unconditional loads, then a select: no branch, so no
                              // wait on the mask ahead of the matrix loads
                              const unsigned fc = m ? (unsigned)m[col] : 0xFFFFu;
#pragma unroll
                              for (int i = 0; i < R; ++i) {
                                  const int w = R * t + i;
                                  const double xx = x[(size_t)col * 12 + w];
                                  xv[i] = ((fc >> w) & 1u) ? xx : 0.0;
                              }
                          },
                          acc);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int w = R * t + i;
        double v = acc[i];
        if (resid) v = b[(size_t)node * 12 + w] - v;
        if (!is_free(mr, node, w)) v = 0.0;
        y[(size_t)node * 12 + w] = v;
    }
}

// ---------------------------------------------------- block-Jacobi factor
// Inverse of each node's 12x12 diagonal block (prescribed rows/columns
// replaced by identity) by an FP64 Cholesky factorisation; 16 lanes per node.
template <class TV>
__global__ __launch_bounds__(256) void k_bj_factor(int nnodes, const int* __restrict__ diag_blk,
                                                   const void* __restrict__ vals, int vals_fp32,
                                                   const uint16_t* __restrict__ fm, const int* __restrict__ node_shell,
                                                   TV* __restrict__ dinv, int* __restrict__ fail_shell) {
    __shared__ double A[16][12][13];
    __shared__ int bad[16];
    const int ln = threadIdx.x & 15, sub = threadIdx.x >> 4;
    const int node = blockIdx.x * 16 + sub;
    const bool act = node < nnodes;
    if (ln == 0) bad[sub] = 0;
    if (act && ln < 12) {
        const size_t base = (size_t)diag_blk[node] * 144;
        for (int c = 0; c < 12; ++c) {
            double v = vals_fp32 ? (double)((const float*)vals)[base + c * 12 + ln] : ((const double*)vals)[base + c * 12 + ln];
            const bool fr = is_free(fm, node, ln), fc = is_free(fm, node, c);
            if (!fr || !fc) v = (ln == c && !fr) ? 1.0 : 0.0;
            A[sub][ln][c] = v;
        }
    }
    __syncthreads();
    // right-looking Cholesky: A = L L^T, L stored in the lower triangle
    for (int j = 0; j < 12; ++j) {
        if (act && ln == j) {
            double d = A[sub][j][j];
            if (!(d > 0.0)) {
                bad[sub] = 1;
                d = 1.0;
            }
            A[sub][j][j] = sqrt(d);
        }
        __syncthreads();
        if (act && ln > j && ln < 12) A[sub][ln][j] /= A[sub][j][j];
        __syncthreads();
        if (act && ln > j && ln < 12)
            for (int k = j + 1; k <= ln; ++k) A[sub][ln][k] -= A[sub][ln][j] * A[sub][k][j];
        __syncthreads();
    }
    if (act && ln < 12) {
        // column ln of the inverse: L y = e_ln, L^T x = y
        double y[12];
        for (int i = 0; i < 12; ++i) {
            double v = (i == ln) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= A[sub][i][k] * y[k];
            y[i] = v / A[sub][i][i];
        }
        for (int i = 11; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < 12; ++k) v -= A[sub][k][i] * y[k];
            y[i] = v / A[sub][i][i];
        }
        for (int i = 0; i < 12; ++i) dinv[(size_t)node * 144 + i * 12 + ln] = (TV)y[i];
        if (ln == 0 && bad[sub]) atomicOr(&fail_shell[node_shell[node]], 1);
    }
}

__global__ void k_save_diag(int nnodes, const int* __restrict__ diag_blk, const void* __restrict__ vals, int fp32,
                            double* __restrict__ diag) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnodes * 12) return;
    const int node = t / 12, w = t % 12;
    const size_t at = (size_t)diag_blk[node] * 144 + w * 12 + w;
    diag[t] = fp32 ? (double)((const float*)vals)[at] : ((const double*)vals)[at];
}

// Diagonal regulariser A_ii = (1 + delta) diag_i for shells with delta > 0.
__global__ void k_regularize(int nnodes, const int* __restrict__ diag_blk, void* __restrict__ vals, int fp32,
                             const double* __restrict__ diag, const int* __restrict__ node_shell,
                             const double* __restrict__ delta_shell) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnodes * 12) return;
    const int node = t / 12, w = t % 12;
    const double dl = delta_shell[node_shell[node]];
    if (dl <= 0.0) return;
    const size_t at = (size_t)diag_blk[node] * 144 + w * 12 + w;
    const double v = (1.0 + dl) * diag[t];
    if (fp32)
        ((float*)vals)[at] = (float)v;
    else
        ((double*)vals)[at] = v;
}

// ------------------------------------------------------ block reductions

template <int N, int NW> __device__ __forceinline__ void block_sum(double (&v)[N], double* lds /* [NW][N] */) {
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) lds[wv * N + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += lds[w * N + k];
        v[k] = t;
    }
}

// Synchronisation state of one shell during a CG launch (zeroed before it).
// Arrivals go through CG_GROUPS group counters on separate 128-byte lines
// and then one top counter, so no single address takes more than about
// nblk/CG_GROUPS (or CG_GROUPS) atomic operations per barrier.
constexpr int CG_GROUPS = 16;
struct alignas(128) ShellSync {
    unsigned cnt;        // top-level arrivals (group leaders), monotone
    unsigned gen;        // barriers released so far
    unsigned pad0[30];
    double tot[2][4];    // published totals, by barrier parity
    double pad1[8];
    unsigned gcnt[CG_GROUPS][32];   // per-group arrivals, monotone, one line each
};

// Barrier over the nblk blocks of one shell that also sums one partial
// vector per block.  The last block to arrive adds the partials of the shell
// in block order (so every block gets the same, reproducible totals),
// publishes them and releases the others.  Every wait is bounded: after 2^22
// polls, or when another block has given up, the block sets abort and the
// kernel ends (legitimate waits are one matrix-product phase).
template <int N, int NW>
__device__ __forceinline__ bool reduce_barrier(ShellSync* ss, double* __restrict__ part, int blk, int sb0, int snb,
                                               unsigned k, double (&v)[N], int* abort_flag, double* lds) {
    __shared__ int s_last, s_ok;
    block_sum<N, NW>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int n = 0; n < N; ++n) part[4 * (size_t)blk + n] = v[n];
        // one release fence publishes this block's vector writes and partial
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int ng = snb < CG_GROUPS ? snb : CG_GROUPS;
        const int lb = blk - sb0, g = lb % ng;
        const unsigned gsize = (unsigned)((snb - g + ng - 1) / ng);
        int last = 0;
        const unsigned og = __hip_atomic_fetch_add(&ss->gcnt[g][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (og == gsize * (k + 1) - 1) {
            // last of its group: carry the group's arrival to the top counter
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            const unsigned ot = __hip_atomic_fetch_add(&ss->cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = ot == (unsigned)ng * (k + 1) - 1;
        }
        s_last = last;
        s_ok = 1;
    }
    __syncthreads();
    if (s_last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        double t[N];
#pragma unroll
        for (int n = 0; n < N; ++n) t[n] = 0.0;
        for (int i = threadIdx.x; i < snb; i += blockDim.x)
#pragma unroll
            for (int n = 0; n < N; ++n)
                t[n] += __hip_atomic_load(&part[4 * (size_t)(sb0 + i) + n], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        block_sum<N, NW>(t, lds);
#pragma unroll
        for (int n = 0; n < N; ++n) v[n] = t[n];
        if (threadIdx.x == 0) {
#pragma unroll
            for (int n = 0; n < N; ++n)
                __hip_atomic_store(&ss->tot[k & 1][n], t[n], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&ss->gen, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        return true;
    }
    if (threadIdx.x == 0) {
        // poll with plain coherent loads; one acquire fence once released
        unsigned spins = 0;
        while (__hip_atomic_load(&ss->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k + 1) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                ++spins > (1u << 22)) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
#pragma unroll
    for (int n = 0; n < N; ++n)
        v[n] = __hip_atomic_load(&ss->tot[k & 1][n], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return s_ok != 0;
}

// ---------------------------------------------------- persistent CG
// Block-Jacobi preconditioned CG for every shell at once.  Each shell owns a
// contiguous set of blocks and node rows; the only synchronisation is the
// per-shell reduce-barrier (two per iteration).  p is double-buffered so that
// the update p = z + beta p is fused into the matrix product:
//   phase A: p_new = z + beta p_old (own rows), q = A (z + beta p_old), sum p.q
//   phase B: x += alpha p, r -= alpha q, z = Dinv r, sums r.z and r.r
template <class TM, class TV, int NT>
__global__ __launch_bounds__(NT) void k_cg(
    const int* __restrict__ blk_shell, const int* __restrict__ blk_row0, const int* __restrict__ blk_row1,
    const int* __restrict__ shell_blk0, const int* __restrict__ shell_nblk, const int* __restrict__ row_ptr,
    const int* __restrict__ col_idx, const TM* __restrict__ vals, const TV* __restrict__ dinv,
    const uint16_t* __restrict__ fm, const double* __restrict__ b, TV* __restrict__ x, TV* __restrict__ r,
    TV* __restrict__ z, TV* __restrict__ p0, TV* __restrict__ p1, TV* __restrict__ qv, double* __restrict__ partial,
    ShellSync* __restrict__ sync, int* __restrict__ abort_flag, const double* __restrict__ rtol2_shell,
    const int* __restrict__ maxit_shell, const int* __restrict__ active_shell, CgShellOut* __restrict__ out) {
    constexpr int R = Lay<TM>::R, L = Lay<TM>::L, G = Lay<TM>::G;
    constexpr int NW = NT / 64;
    __shared__ double lds[4 * NW];
    const int blk = blockIdx.x;
    const int sh = blk_shell[blk];
    const int row0 = blk_row0[blk], row1 = blk_row1[blk];
    const int sb0 = shell_blk0[sh], snb = shell_nblk[sh];
    ShellSync* ss = sync + sh;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane / L, t = lane % L;
    const bool lane_ok = grp < G;
    const int gsrc = lane_ok ? lane - t : 0;   // first lane of this lane's group
    const int rows_per_pass = NW * G;
    unsigned nbar = 0;
    const bool leader = blk == sb0 && threadIdx.x == 0;

    if (!active_shell[sh]) {
        for (int e = threadIdx.x; e < (row1 - row0) * 12; e += blockDim.x) x[(size_t)row0 * 12 + e] = TV(0);
        if (leader) out[sh] = CgShellOut{0, 0, 0.0, 0.0};
        return;
    }

    // z = Dinv r for this lane's R rows of node (r of the node exchanged in the group)
    auto precond = [&](int node, const TV* rr, TV* zz) {
        TV rall[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) rall[c] = __shfl(rr[c % R], gsrc + c / R);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const TV* drow = dinv + (size_t)node * 144 + (R * t + i) * 12;
            TV s = TV(0);
#pragma unroll
            for (int c = 0; c < 12; ++c) s += drow[c] * rall[c];
            zz[i] = s;
        }
    };

    // ---- init: r = b (masked), x = 0, p_old = 0, z = Dinv r; sums r.z and b.b
    double sums[2] = {0.0, 0.0};
    for (int base = row0; base < row1; base += rows_per_pass) {
        const int node = base + wv * G + grp;
        const bool ok = lane_ok && node < row1;
        const int nd = ok ? node : row0;
        TV rr[R], zz[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int w = R * t + i;
            rr[i] = ok && is_free(fm, node, w) ? (TV)b[(size_t)node * 12 + w] : TV(0);
        }
        precond(nd, rr, zz);
        if (ok) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int w = R * t + i;
                const size_t at = (size_t)node * 12 + w;
                if (!is_free(fm, node, w)) zz[i] = TV(0);
                r[at] = rr[i];
                z[at] = zz[i];
                x[at] = TV(0);
                p0[at] = TV(0);
                sums[0] += (double)rr[i] * (double)zz[i];
                sums[1] += (double)rr[i] * (double)rr[i];
            }
        }
    }
    if (!reduce_barrier<2, NW>(ss, partial, blk, sb0, snb, nbar++, sums, abort_flag, lds)) {
        if (leader) out[sh] = CgShellOut{0, 3, 0.0, 0.0};
        return;
    }
    double rz = sums[0];
    const double bb = sums[1];
    const double tol2 = rtol2_shell[sh] * bb;
    const int maxit = maxit_shell[sh];
    if (bb == 0.0) {
        if (leader) out[sh] = CgShellOut{0, 0, 0.0, 0.0};
        return;
    }
    double beta = 0.0;
    TV* pin = p0;
    TV* pout = p1;
    int it = 0, status = 1;
    double rr2 = bb;
    for (; it < maxit; ++it) {
        // ---- phase A
        double pq[1] = {0.0};
        for (int base = row0; base < row1; base += rows_per_pass) {
            const int node = base + wv * G + grp;
            if (!(lane_ok && node < row1)) continue;
            const unsigned fmask = fm[node];   // loaded first: later waits on it drain nothing else
            TV acc[R];
            const TV bt = (TV)beta;
            row_times_grouped<TM, TV>(row_ptr, col_idx, vals, node, t, gsrc, false,
                              [&](int col, TV* xv) {
#pragma unroll
                                  for (int i = 0; i < R; ++i) {
                                      const size_t at = (size_t)col * 12 + R * t + i;
                                      xv[i] = z[at] + bt * pin[at];
                                  }
                              },
                              acc);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int w = R * t + i;
                const size_t at = (size_t)node * 12 + w;
                const TV pn = z[at] + bt * pin[at];
                const TV qq = ((fmask >> w) & 1u) ? acc[i] : TV(0);
                pout[at] = pn;
                qv[at] = qq;
                pq[0] += (double)pn * (double)qq;
            }
        }
        if (!reduce_barrier<1, NW>(ss, partial, blk, sb0, snb, nbar++, pq, abort_flag, lds)) {
            status = 3;
            break;
        }
        if (!(pq[0] > 0.0)) {
            status = 2;
            break;
        }
        const double alpha = rz / pq[0];
        // ---- phase B
        double s2[2] = {0.0, 0.0};
        for (int base = row0; base < row1; base += rows_per_pass) {
            const int node = base + wv * G + grp;
            const bool ok = lane_ok && node < row1;
            const int nd = ok ? node : row0;
            // every load of the row is issued before the first use
            const unsigned fmask = fm[nd];
            TV rr[R], zz[R], xo[R], pp[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const size_t at = (size_t)nd * 12 + R * t + i;
                rr[i] = r[at] - (TV)alpha * qv[at];
                xo[i] = x[at];
                pp[i] = pout[at];
            }
            precond(nd, rr, zz);
            if (ok) {
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const int w = R * t + i;
                    const size_t at = (size_t)node * 12 + w;
                    if (!((fmask >> w) & 1u)) zz[i] = TV(0);
                    x[at] = xo[i] + (TV)alpha * pp[i];
                    r[at] = rr[i];
                    z[at] = zz[i];
                    s2[0] += (double)rr[i] * (double)zz[i];
                    s2[1] += (double)rr[i] * (double)rr[i];
                }
            }
        }
        if (!reduce_barrier<2, NW>(ss, partial, blk, sb0, snb, nbar++, s2, abort_flag, lds)) {
            status = 3;
            break;
        }
        rr2 = s2[1];
        if (rr2 <= tol2) {
            status = 0;
            ++it;
            break;
        }
        beta = s2[0] / rz;
        rz = s2[0];
        TV* tmp = pin;
        pin = pout;
        pout = tmp;
    }
    if (leader) out[sh] = CgShellOut{it, status, bb, rr2};
}

// ------------------------------------------------------ per-shell dots
__global__ __launch_bounds__(256) void k_shell_dot_part(const int* __restrict__ blk_row0,
                                                        const int* __restrict__ blk_row1, const double* __restrict__ x,
                                                        const double* __restrict__ y, const uint16_t* __restrict__ fm,
                                                        double* __restrict__ part) {
    __shared__ double lds[8];
    const int blk = blockIdx.x;
    const int r0 = blk_row0[blk], r1 = blk_row1[blk];
    double s[1] = {0.0};
    for (int e = r0 * 12 + threadIdx.x; e < r1 * 12; e += blockDim.x) {
        const int node = e / 12, w = e % 12;
        if (is_free(fm, node, w)) s[0] += x[e] * y[e];
    }
    block_sum<1, 4>(s, lds);
    if (threadIdx.x == 0) part[blk] = s[0];
}

__global__ void k_shell_dot_fin(int nshell, const int* __restrict__ shell_blk0, const int* __restrict__ shell_nblk,
                                const double* __restrict__ part, double* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nshell) return;
    double v = 0.0;
    for (int i = 0; i < shell_nblk[s]; ++i) v += part[shell_blk0[s] + i];
    out[s] = v;
}

// ------------------------------------------------------------ elementwise
__global__ void k_predict(int n, const double* __restrict__ qn, const double* __restrict__ vn,
                          const double* __restrict__ qpresc, const uint16_t* __restrict__ fm,
                          const int* __restrict__ node_shell, const ShellParams* __restrict__ shells, double dt,
                          double* __restrict__ qhat, double* __restrict__ q) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double qh = qn[t] + dt * vn[t];
    const double a = shells[node_shell[t / 12]].damp * dt;
    qhat[t] = a != 0.0 ? (qh + a * qn[t]) / (1.0 + a) : qh;
    q[t] = is_free(fm, t / 12, t % 12) ? qh : (qpresc ? qpresc[t] : qn[t]);
}

// External nodal forces (see launch_nodal_load).
__global__ __launch_bounds__(256) void k_nodal_load_part(const int* __restrict__ blk_row0,
                                                         const int* __restrict__ blk_row1, const double* __restrict__ f,
                                                         const double* __restrict__ q, const double* __restrict__ qhat,
                                                         const uint16_t* __restrict__ fm,
                                                         const int* __restrict__ node_shell,
                                                         const int* __restrict__ write_shell,
                                                         double* __restrict__ grad, double* __restrict__ part) {
    __shared__ double lds[4];
    double s = 0.0;
    const int r0 = blk_row0[blockIdx.x], r1 = blk_row1[blockIdx.x];
    for (int e = r0 * 12 + threadIdx.x; e < r1 * 12; e += blockDim.x) {
        const int node = e / 12;
        if (!is_free(fm, node, e % 12)) continue;
        s += f[e] * (q[e] - qhat[e]);
        if (grad && (!write_shell || write_shell[node_shell[node]])) grad[e] -= f[e];
    }
    double v[1] = {s};
    block_sum<1, 4>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ void k_nodal_load_fin(int nshell, const int* __restrict__ shell_blk0, const int* __restrict__ shell_nblk,
                                 const double* __restrict__ part, double* __restrict__ e_shell) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nshell) return;
    double v = 0.0;
    for (int i = 0; i < shell_nblk[s]; ++i) v += part[shell_blk0[s] + i];
    e_shell[3 * s + 2] -= v;
}

__global__ void k_axpy_shell(int n, const double* __restrict__ x, const double* __restrict__ d,
                             const double* __restrict__ alpha_shell, const int* __restrict__ node_shell,
                             double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    out[t] = x[t] + alpha_shell[node_shell[t / 12]] * d[t];
}

__global__ void k_neg_masked(int n, const double* __restrict__ g, const uint16_t* __restrict__ fm,
                             const int* __restrict__ node_shell, const int* __restrict__ active_shell,
                             double* __restrict__ b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int node = t / 12;
    b[t] = (is_free(fm, node, t % 12) && active_shell[node_shell[node]]) ? -g[t] : 0.0;
}

__global__ void k_velocity(int n, const double* __restrict__ q1, const double* __restrict__ qn, double dt,
                           double* __restrict__ v) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) v[t] = (q1[t] - qn[t]) / dt;
}

__global__ void k_copy_shell(int n, const double* __restrict__ src, const int* __restrict__ node_shell,
                             const int* __restrict__ flag_shell, double* __restrict__ dst) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && flag_shell[node_shell[t / 12]]) dst[t] = src[t];
}

__global__ void k_add_shell(int n, const double* __restrict__ src, const int* __restrict__ node_shell,
                            const int* __restrict__ flag_shell, double* __restrict__ dst) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && flag_shell[node_shell[t / 12]]) dst[t] += src[t];
}

template <class TV> __global__ void k_add_to(int n, const TV* __restrict__ dx, double* __restrict__ x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] += (double)dx[t];
}

// Zero n 16-byte words, then the 4-byte tail (a kernel rather than a
// memset so that the clearing can sit inside a captured graph).
__global__ void k_zero(size_t n16, uint4* __restrict__ p, size_t n4_tail, uint32_t* __restrict__ tail) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = t; i < n16; i += stride) p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (t < n4_tail) tail[t] = 0u;
}

// ------------------------------------------------------------ launchers
static inline dim3 grid1(int n) { return dim3((n + 255) / 256); }

void launch_zero(hipStream_t st, void* p, size_t bytes) {
    const size_t n16 = bytes / 16, n4 = (bytes % 16) / 4;
    const size_t blocks = std::min<size_t>(std::max<size_t>((n16 + 255) / 256, 1), 4096);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, n16, (uint4*)p, n4,
                       (uint32_t*)((char*)p + n16 * 16));
}

template <class TM>
void launch_spmv(hipStream_t st, int nnodes, const int* row_ptr, const int* col_idx, const TM* vals,
                 const uint16_t* freemask, const double* x, const double* b, double* y, int mode) {
    if (nnodes == 0) return;
    const int rows_per_block = 4 * Lay<TM>::G;
    hipLaunchKernelGGL(k_spmv<TM>, dim3((nnodes + rows_per_block - 1) / rows_per_block), dim3(256), 0, st, nnodes,
                       row_ptr, col_idx, vals, freemask, x, b, y, mode);
}
template void launch_spmv<double>(hipStream_t, int, const int*, const int*, const double*, const uint16_t*,
                                  const double*, const double*, double*, int);
template void launch_spmv<float>(hipStream_t, int, const int*, const int*, const float*, const uint16_t*,
                                 const double*, const double*, double*, int);

template <class TV>
void launch_bj_factor(hipStream_t st, int nnodes, const int* diag_blk, const void* vals, int vals_fp32,
                      const uint16_t* freemask, const int* node_shell, TV* dinv, int* fail_shell) {
    if (nnodes == 0) return;
    hipLaunchKernelGGL(k_bj_factor<TV>, dim3((nnodes + 15) / 16), dim3(256), 0, st, nnodes, diag_blk, vals, vals_fp32,
                       freemask, node_shell, dinv, fail_shell);
}
template void launch_bj_factor<double>(hipStream_t, int, const int*, const void*, int, const uint16_t*, const int*,
                                       double*, int*);
template void launch_bj_factor<float>(hipStream_t, int, const int*, const void*, int, const uint16_t*, const int*,
                                      float*, int*);

void launch_save_diag(hipStream_t st, int nnodes, const int* diag_blk, const void* vals, int vals_fp32,
                      double* diag) {
    hipLaunchKernelGGL(k_save_diag, grid1(nnodes * 12), dim3(256), 0, st, nnodes, diag_blk, vals, vals_fp32, diag);
}

void launch_regularize(hipStream_t st, int nnodes, const int* diag_blk, void* vals, int vals_fp32,
                       const double* diag, const int* node_shell, const double* delta_shell) {
    hipLaunchKernelGGL(k_regularize, grid1(nnodes * 12), dim3(256), 0, st, nnodes, diag_blk, vals, vals_fp32, diag,
                       node_shell, delta_shell);
}

// the CG kernel instance for a block size of 256, 512 or 1024 threads
template <class TM, class TV> const void* cg_fn(int nthreads) {
    return nthreads == 1024 ? (const void*)k_cg<TM, TV, 1024>
           : nthreads == 512 ? (const void*)k_cg<TM, TV, 512>
                             : (const void*)k_cg<TM, TV, 256>;
}

template <class TM, class TV>
hipError_t launch_cg(hipStream_t st, int nblk, int nthreads, const RowBlocks& rb, const int* row_ptr,
                     const int* col_idx, const TM* vals, const TV* dinv, const uint16_t* freemask, const double* b,
                     TV* x, TV* r, TV* z, TV* p0, TV* p1, TV* qv, double* partial, void* sync, int* abort_flag,
                     const double* rtol2_shell, const int* maxit_shell, const int* active_shell, CgShellOut* out) {
    ShellSync* ss = static_cast<ShellSync*>(sync);
    void* args[] = {(void*)&rb.blk_shell, (void*)&rb.blk_row0, (void*)&rb.blk_row1, (void*)&rb.shell_blk0,
                    (void*)&rb.shell_nblk, (void*)&row_ptr, (void*)&col_idx, (void*)&vals, (void*)&dinv,
                    (void*)&freemask, (void*)&b, (void*)&x, (void*)&r, (void*)&z, (void*)&p0, (void*)&p1,
                    (void*)&qv, (void*)&partial, (void*)&ss, (void*)&abort_flag, (void*)&rtol2_shell,
                    (void*)&maxit_shell, (void*)&active_shell, (void*)&out};
    return hipLaunchCooperativeKernel(cg_fn<TM, TV>(nthreads), dim3(nblk), dim3(nthreads), args, 0, st);
}
template hipError_t launch_cg<double, double>(hipStream_t, int, int, const RowBlocks&, const int*, const int*,
                                              const double*, const double*, const uint16_t*, const double*, double*,
                                              double*, double*, double*, double*, double*, double*, void*, int*,
                                              const double*, const int*, const int*, CgShellOut*);
template hipError_t launch_cg<float, float>(hipStream_t, int, int, const RowBlocks&, const int*, const int*,
                                            const float*, const float*, const uint16_t*, const double*, float*,
                                            float*, float*, float*, float*, float*, double*, void*, int*,
                                            const double*, const int*, const int*, CgShellOut*);

size_t cg_sync_bytes() { return sizeof(ShellSync); }
int cg_rows_per_pass(int tm_fp32, int nthreads) { return (nthreads / 64) * (tm_fp32 ? Lay<float>::G : Lay<double>::G); }

int cg_max_blocks(int device, int tm_fp32, int nthreads) {
    int per_cu = 0, cus = 0;
    const void* fn = tm_fp32 ? cg_fn<float, float>(nthreads) : cg_fn<double, double>(nthreads);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nthreads, 0) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return -1;
    return per_cu * cus;
}

void launch_shell_dot(hipStream_t st, const RowBlocks& rb, int nshell, const double* x, const double* y,
                      const uint16_t* freemask, double* partial, double* out) {
    hipLaunchKernelGGL(k_shell_dot_part, dim3(rb.nblk), dim3(256), 0, st, rb.blk_row0, rb.blk_row1, x, y, freemask,
                       partial);
    hipLaunchKernelGGL(k_shell_dot_fin, grid1(nshell), dim3(256), 0, st, nshell, rb.shell_blk0, rb.shell_nblk,
                       partial, out);
}

void launch_predict(hipStream_t st, int n, const double* qn, const double* vn, const double* qpresc,
                    const uint16_t* freemask, const int* node_shell, const ShellParams* shells, double dt,
                    double* qhat, double* q) {
    hipLaunchKernelGGL(k_predict, grid1(n), dim3(256), 0, st, n, qn, vn, qpresc, freemask, node_shell, shells, dt,
                       qhat, q);
}
void launch_nodal_load(hipStream_t st, const RowBlocks& rb, int nshell, const double* f, const double* q,
                       const double* qhat, const uint16_t* freemask, const int* node_shell, const int* write_shell,
                       double* grad, double* part, double* e_shell) {
    hipLaunchKernelGGL(k_nodal_load_part, dim3(rb.nblk), dim3(256), 0, st, rb.blk_row0, rb.blk_row1, f, q, qhat,
                       freemask, node_shell, write_shell, grad, part);
    hipLaunchKernelGGL(k_nodal_load_fin, grid1(nshell), dim3(256), 0, st, nshell, rb.shell_blk0, rb.shell_nblk,
                       part, e_shell);
}
void launch_axpy_shell(hipStream_t st, int nnodes, const double* x, const double* d, const double* alpha_shell,
                       const int* node_shell, double* out) {
    const int n = nnodes * 12;
    hipLaunchKernelGGL(k_axpy_shell, grid1(n), dim3(256), 0, st, n, x, d, alpha_shell, node_shell, out);
}
void launch_neg_masked(hipStream_t st, int nnodes, const double* g, const uint16_t* freemask, const int* node_shell,
                       const int* active_shell, double* b) {
    const int n = nnodes * 12;
    hipLaunchKernelGGL(k_neg_masked, grid1(n), dim3(256), 0, st, n, g, freemask, node_shell, active_shell, b);
}
void launch_velocity(hipStream_t st, int n, const double* q1, const double* qn, double dt, double* v) {
    hipLaunchKernelGGL(k_velocity, grid1(n), dim3(256), 0, st, n, q1, qn, dt, v);
}
void launch_copy_shell(hipStream_t st, int nnodes, const double* src, const int* node_shell, const int* flag_shell,
                       double* dst) {
    const int n = nnodes * 12;
    hipLaunchKernelGGL(k_copy_shell, grid1(n), dim3(256), 0, st, n, src, node_shell, flag_shell, dst);
}
void launch_add_shell(hipStream_t st, int nnodes, const double* src, const int* node_shell, const int* flag_shell,
                      double* dst) {
    const int n = nnodes * 12;
    hipLaunchKernelGGL(k_add_shell, grid1(n), dim3(256), 0, st, n, src, node_shell, flag_shell, dst);
}
template <class TV> void launch_add_to(hipStream_t st, int n, const TV* dx, double* x) {
    hipLaunchKernelGGL(k_add_to<TV>, grid1(n), dim3(256), 0, st, n, dx, x);
}
template void launch_add_to<double>(hipStream_t, int, const double*, double*);
template void launch_add_to<float>(hipStream_t, int, const float*, double*);

}  // namespace bhem
