// Sparse linear algebra of libbhem (gfx950): 12x12-block matrix products,
// block-Jacobi factorisation, the persistent block-Jacobi conjugate gradient
// and per-shell reductions.
//
// Matrix storage (the Hessian is symmetric): block row i keeps only its
// blocks (i, j >= i), the diagonal block first.  The stored block of pair
// (i, j > i) holds A_ji column-major, which is A_ij row-major (entry (r, c)
// of A_ij at r*12 + c); the diagonal block A_ii, symmetric, keeps its 84
// distinct values in the packed layout at SYM12_VALS (the first 84 of its
// 144 places).  Rows and columns of prescribed DOFs stay in the matrix; the
// solver masks them (free-DOF bit masks per node), which equals replacing
// them by identity rows and columns with a zero right-hand side.
//
// Product lane layout: a node row is handled by L = 6 lanes.  Lane t of the
// group reads the R = 2 values at offset c*12 + 2t of every row c of a
// stored block (16 bytes for FP64 blocks, 8 for FP32; the six lanes of a
// group read one row's 12 values together, coalesced), and owns columns
// 2t, 2t+1 of A_ij.  (Four FP32 columns per lane, 16-byte loads, were
// measured slower: 21 rows per wavefront leave more blocks on a partial
// last pass and need more registers.)  Both products a stored block takes part in are then lane-local:
//   A_ij x_j   partial sums over the lane's columns for all 12 rows, summed
//              over the group once per block row;
//   A_ji x_i = A_ij^T x_i   the lane's R entries, which row j needs.
// The second product goes to a slot of its own (tslot of the block; rows
// j's slots are the contiguous range lptr[j] .. lptr[j+1], ordered by i), and
// row j adds its slots after the product phase: every entry is written by
// one lane and summed in a fixed order, so results are reproducible.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace bhem {

template <class TM> struct Lay {
    static constexpr int R = 2;        // columns per lane
    static constexpr int L = 12 / R;   // lanes per node row
    static constexpr int G = 64 / L;   // node rows per wavefront
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
template <> struct VecLoad<float, 2> {
    static __device__ __forceinline__ void ld(const float* p, float* o) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <class T> struct Vec4;
template <> struct Vec4<double> {
    static __device__ __forceinline__ void ld(const double* p, double* o) {
        const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
        o[0] = a.x;
        o[1] = a.y;
        o[2] = b.x;
        o[3] = b.y;
    }
};
template <> struct Vec4<float> {
    static __device__ __forceinline__ void ld(const float* p, float* o) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        o[0] = a.x;
        o[1] = a.y;
        o[2] = a.z;
        o[3] = a.w;
    }
};
template <class TV, int R> struct VecStore;
template <> struct VecStore<double, 2> {
    static __device__ __forceinline__ void st(double* p, const double* v) {
        *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    }
};
template <> struct VecStore<float, 2> {
    static __device__ __forceinline__ void st(float* p, const float* v) {
        *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
    }
};
template <> struct VecStore<float, 4> {
    static __device__ __forceinline__ void st(float* p, const float* v) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
};

// Orders the wavefront's LDS accesses around a cross-lane exchange (the LDS
// operations of one wavefront execute in program order; this keeps the
// compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// out[k] = sum over the L lanes of the group of part[R*t + k], through the
// wave's LDS area red[64][12]: every lane writes its 12 partials and reads
// its R entries from each lane of its group, in lane order (the same order
// on every lane, so the result is reproducible).  The partials stay in
// registers (selecting them by a lane-dependent index would move them to
// scratch memory).  The LDS operations of one wavefront execute in program
// order, so the reads see the writes and the next row's writes follow the
// reads.
template <class TV, int R, int L>
__device__ __forceinline__ void group_sum(const TV (&part)[12], int lane, int t, int gbase, TV* __restrict__ red,
                                          TV (&out)[R]) {
    constexpr int V = 16 / sizeof(TV);   // values per 16-byte LDS access
#pragma unroll
    for (int e = 0; e < 12; e += V) VecStore<TV, V>::st(red + lane * 12 + e, part + e);
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < R; ++k) out[k] = TV(0);
#pragma unroll
    for (int j = 0; j < L; ++j) {
        TV v[R];
        VecLoad<TV, R>::ld(red + (gbase + j) * 12 + R * t, v);
#pragma unroll
        for (int k = 0; k < R; ++k) out[k] += v[k];
    }
    wave_lds_sync();
}

// One stored off-diagonal block in parts of NR rows (NR loads of R values
// each): part[c] += sum_k A[c][R t + k] xv[k] and tv[k] += sum_c
// A[c][R t + k] x_i[c], with x_i[c] read from the group's LDS copy xl
// (re-read per block: kept in registers through the row, the 12 values would
// cost the registers that let 16 waves share a CU).  A scheduling barrier
// after each part keeps one part's loads in flight at a time per wave.
// NR = 12 (the whole block in flight) where the registers allow it: FP64
// CG at 2 waves per SIMD 115 -> 113 us per iteration, the SpMV 93 -> 90 us;
// the FP32 CG at 1024 threads would spill and keeps NR = 4.  pst/pv: the
// previous block's transposed product, stored after this block's first
// loads are issued (loads and stores share one in-order completion counter,
// so a store issued first would delay the wait for the loads behind it).
// The block's values already in registers (a[12][R], its 12 rows of this
// lane's columns): the same arithmetic as block_sym.
template <class TM, class TV, bool ABS>
__device__ __forceinline__ void block_sym_regs(const TM (&a)[12][Lay<TM>::R], const TV (&xv)[Lay<TM>::R],
                                               const TV* __restrict__ xl, TV (&part)[12], TV (&tv)[Lay<TM>::R]) {
    constexpr int R = Lay<TM>::R;
#pragma unroll
    for (int cc = 0; cc < 12; ++cc) {
        const TV xc = xl[cc];
        TV sacc = part[cc];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const TV av = ABS ? (TV)fabs(a[cc][k]) : (TV)a[cc][k];
            sacc += av * xv[k];
            tv[k] += av * xc;
        }
        part[cc] = sacc;
    }
}

template <class TM, class TV, bool ABS, int NR>
__device__ __forceinline__ void block_sym(const TM* __restrict__ blk, const TV (&xv)[Lay<TM>::R],
                                          const TV* __restrict__ xl, TV (&part)[12], TV (&tv)[Lay<TM>::R],
                                          TV* pst = nullptr, const TV* pv = nullptr) {
    constexpr int R = Lay<TM>::R;
    static_assert(12 % NR == 0, "parts of equal size");
    asm volatile("" ::: "memory");   // re-read xl for this block
#pragma unroll
    for (int h = 0; h < 12 / NR; ++h) {
        TM a[NR][R];
#pragma unroll
        for (int c = 0; c < NR; ++c) VecLoad<TM, R>::ld(blk + (NR * h + c) * 12, a[c]);
        if (h == 0 && pst) VecStore<TV, R>::st(pst, pv);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            const int cc = NR * h + c;
            const TV xc = xl[cc];
            TV sacc = part[cc];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const TV av = ABS ? (TV)fabs(a[c][k]) : (TV)a[c][k];
                sacc += av * xv[k];
                tv[k] += av * xc;
            }
            part[cc] = sacc;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The diagonal block of a row, kept as its 84 distinct values (packed
// layout at SYM12_VALS), against x_i: part[c] = sum_k A[c][R t + k] xv[k]
// for the 12 rows c (set, not added) and dl = sum_c x_i[c] part[c], whose
// sum over the group is x_i^T A_ii x_i (a scalar: a transposed product,
// needed only after the row's other blocks, would keep the block's registers
// live through them).
// Row pair b needs the 2x2 block (b, t): stored as such at 12 b + 4 d
// (d = t - b mod 6 <= 2) or 72 + 4 b (d = 3, b < 3), else as the transpose
// of block (t, b) at 12 t + 4 (6 - d) or 72 + 4 t.  Three parts of two row
// pairs, as block_sym.
template <class TM, class TV, bool ABS>
__device__ __forceinline__ void block_diag_sym(const TM* __restrict__ dblk, int t, const TV (&xv)[2],
                                               const TV* __restrict__ xl, TV (&part)[12], TV& dl) {
    asm volatile("" ::: "memory");   // re-read xl for this block
    // the lane-dependent positions are recomputed per row from an opaque
    // copy of t (hoisted out of the caller's loops they would hold registers)
    asm volatile("" : "+v"(t));
#pragma unroll
    for (int h = 0; h < 3; ++h) {
        TM a[2][4];
        bool tr[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int b = 2 * h + e;
            const int d = (t - b + 6) % 6;
            tr[e] = d >= 4 || (d == 3 && b >= 3);
            const int pos = d <= 2 ? 12 * b + 4 * d : d >= 4 ? 12 * t + 4 * (6 - d) : 72 + 4 * (b < 3 ? b : t);
            Vec4<TM>::ld(dblk + pos, a[e]);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int cc = 2 * (2 * h + e) + i;
                // A[cc][R t + k], k = 0, 1: entry (i, k) of block (b, t)
                const TM m0 = i == 0 ? a[e][0] : (tr[e] ? a[e][1] : a[e][2]);
                const TM m1 = i == 0 ? (tr[e] ? a[e][2] : a[e][1]) : a[e][3];
                const TV v0 = ABS ? (TV)fabs(m0) : (TV)m0, v1 = ABS ? (TV)fabs(m1) : (TV)m1;
                TV sacc = v0 * xv[0];
                sacc += v1 * xv[1];
                part[cc] = sacc;
                dl += xl[cc] * sacc;
            }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The stored blocks of block row `node` against x (see the storage note):
//   part[c] (c = 0..11): this lane's partial of row c of sum_j A_ij x_j,
//   returned: this lane's share of x_i^T A_ii x_i (for p^T A p),
//   slot[tslot[b]] <- A_ij^T x_i for every stored off-diagonal block b.
// xo: this lane's R entries of x_i (already masked and, with ABS, absolute
// values), copied for the group to xl[12] in LDS; xe(col, xv) gives this
// lane's R entries of x for column block col.  ABS multiplies by |A|
// instead of A.
// PF: the next off-diagonal block's values are loaded while the current one
// is multiplied (registers for two blocks; for blocks of few rows, whose
// product is a chain of round trips per row)
template <class TM, class TV, bool ABS, int NR, class XF, bool PF = false>
__device__ __forceinline__ TV row_sym(const SymBsr& m, const TM* __restrict__ vals, int node, int t,
                                      const TV (&xo)[Lay<TM>::R], XF xe, TV* __restrict__ xl, TV* __restrict__ slot,
                                      TV (&part)[12]) {
    constexpr int R = Lay<TM>::R;
    const int b0 = m.row_ptr[node], b1 = m.row_ptr[node + 1];
    // column of the next off-diagonal block, loaded one block ahead so that
    // x of each block's column is requested as the block starts (an index in
    // bounds is loaded also past the row's last block; the value is unused)
    int col = m.col_idx[b0 + 1 < b1 ? b0 + 1 : b0];
#pragma unroll
    for (int k = 0; k < R; ++k) xl[R * t + k] = xo[k];
    wave_lds_sync();
    static_assert(R == 2, "the packed diagonal block is read by column pairs");
    TV dl = TV(0);
    block_diag_sym<TM, TV, ABS>(vals + (size_t)b0 * 144, t, xo, xl, part, dl);
    TV pv[R];
    TV* pst = nullptr;
    if constexpr (PF) {
        TM an[12][R];
        if (b0 + 1 < b1) {
#pragma unroll
            for (int c = 0; c < 12; ++c) VecLoad<TM, R>::ld(vals + (size_t)(b0 + 1) * 144 + R * t + c * 12, an[c]);
        }
        for (int b = b0 + 1; b < b1; ++b) {
            TM a[12][R];
#pragma unroll
            for (int c = 0; c < 12; ++c)
#pragma unroll
                for (int k = 0; k < R; ++k) a[c][k] = an[c][k];
            TV xv[R], tv[R];
            xe(col, xv);
            col = m.col_idx[b + 1 < b1 ? b + 1 : b];
            const int ts = m.tslot[b];
            if (b + 1 < b1) {
#pragma unroll
                for (int c = 0; c < 12; ++c) VecLoad<TM, R>::ld(vals + (size_t)(b + 1) * 144 + R * t + c * 12, an[c]);
            }
            if (pst) VecStore<TV, R>::st(pst, pv);
#pragma unroll
            for (int k = 0; k < R; ++k) tv[k] = TV(0);
            block_sym_regs<TM, TV, ABS>(a, xv, xl, part, tv);
            pst = slot + (size_t)ts * 12 + R * t;
#pragma unroll
            for (int k = 0; k < R; ++k) pv[k] = tv[k];
        }
        if (pst) VecStore<TV, R>::st(pst, pv);
        wave_lds_sync();
        return dl;
    }
    for (int b = b0 + 1; b < b1; ++b) {
        TV xv[R], tv[R];
        xe(col, xv);
        col = m.col_idx[b + 1 < b1 ? b + 1 : b];
        const int ts = m.tslot[b];
#pragma unroll
        for (int k = 0; k < R; ++k) tv[k] = TV(0);
        block_sym<TM, TV, ABS, NR>(vals + (size_t)b * 144 + R * t, xv, xl, part, tv, pst, pv);
        pst = slot + (size_t)ts * 12 + R * t;
#pragma unroll
        for (int k = 0; k < R; ++k) pv[k] = tv[k];
    }
    if (pst) VecStore<TV, R>::st(pst, pv);
    wave_lds_sync();
    return dl;
}

// ------------------------------------------------------------------ SpMV
// y = A x in two launches: k_spmv_rows writes the stored-block part of every
// row and the transposed products to the slots; k_spmv_fin adds each row's
// slots and applies the residual form and the row mask.
//   fc: column mask (x restricted to free DOFs) or NULL
template <class TM, bool ABS>
__global__ __launch_bounds__(256) void k_spmv_rows(int nnodes, SymBsr m, const TM* __restrict__ vals,
                                                   const uint16_t* __restrict__ fc, const double* __restrict__ x,
                                                   double* __restrict__ y, double* __restrict__ slot) {
    constexpr int R = Lay<TM>::R, L = Lay<TM>::L, G = Lay<TM>::G;
    __shared__ double red[4][64 * 12];
    __shared__ double xls[4][G * 12];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane / L, t = lane % L, gbase = lane - t;
    const int node = (blockIdx.x * 4 + wv) * G + grp;
    if (grp >= G || node >= nnodes) return;
    auto xe = [&](int col, double* xv) {
        // unconditional loads, then a select: no branch, so no wait on the
        // mask ahead of the matrix loads
        const unsigned f = fc ? (unsigned)fc[col] : 0xFFFFu;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int w = R * t + i;
            const double xx = x[(size_t)col * 12 + w];
            xv[i] = ((f >> w) & 1u) ? (ABS ? fabs(xx) : xx) : 0.0;
        }
    };
    double xo[R], part[12], yo[R];
    xe(node, xo);
    (void)row_sym<TM, double, ABS, 12>(m, vals, node, t, xo, xe, xls[wv] + grp * 12, slot, part);
    group_sum<double, R, L>(part, lane, t, gbase, red[wv], yo);
#pragma unroll
    for (int i = 0; i < R; ++i) y[(size_t)node * 12 + R * t + i] = yo[i];
}

// Two entries (16 bytes) of one row per thread; the row's slots in order.
// y and b 16-byte aligned (k_spmv_fin1 otherwise: one entry per thread).
__global__ void k_spmv_fin1(int nnodes, const int* __restrict__ lptr, const double* __restrict__ slot,
                            const uint16_t* __restrict__ fr, const double* __restrict__ b, double* __restrict__ y) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nnodes * 12) return;
    const int node = e / 12, w = e % 12;
    double v = y[e];
    for (int k = lptr[node]; k < lptr[node + 1]; ++k) v += slot[(size_t)k * 12 + w];
    if (b) v = b[e] - v;
    if (!is_free(fr, node, w)) v = 0.0;
    y[e] = v;
}
__global__ void k_spmv_fin(int nnodes, const int* __restrict__ lptr, const double* __restrict__ slot,
                           const uint16_t* __restrict__ fr, const double* __restrict__ b, double* __restrict__ y) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nnodes * 6) return;
    const int node = e / 6, w = 2 * (e % 6);
    const size_t at = (size_t)node * 12 + w;
    double v[2];
    VecLoad<double, 2>::ld(y + at, v);
    const int k0 = lptr[node], k1 = lptr[node + 1];
    for (int k = k0; k < k1; ++k) {
        double sv[2];
        VecLoad<double, 2>::ld(slot + (size_t)k * 12 + w, sv);
        v[0] += sv[0];
        v[1] += sv[1];
    }
    if (b) {
        double bv[2];
        VecLoad<double, 2>::ld(b + at, bv);
        v[0] = bv[0] - v[0];
        v[1] = bv[1] - v[1];
    }
    if (!is_free(fr, node, w)) v[0] = 0.0;
    if (!is_free(fr, node, w + 1)) v[1] = 0.0;
    VecStore<double, 2>::st(y + at, v);
}

// ---------------------------------------------------- block-Jacobi factor
// Inverse of each node's 12x12 diagonal block (prescribed rows/columns
// replaced by identity) by Gauss-Jordan elimination in FP64 without
// pivoting (the block is symmetric positive definite; the pivot of step k is
// the Schur complement's diagonal entry, the square of a Cholesky factor's,
// and one <= 0 marks the block as not positive definite).  16 lanes per
// node, lane c holding column c in registers; each step takes column k from
// lane k by shuffles, so no LDS and no barrier is involved.
// The inverse is symmetric, so a node keeps its 21 distinct 2x2 blocks
// (84 values instead of 144, layout at SYM12_VALS).  A 2x2 diagonal block
// takes both off-diagonal entries from column 2a + 1, so the stored matrix
// is exactly symmetric.
template <class TV>
__global__ __launch_bounds__(256) void k_bj_factor(int nnodes, const int* __restrict__ diag_blk,
                                                   const void* __restrict__ vals, int vals_fp32,
                                                   const uint16_t* __restrict__ fm, const int* __restrict__ node_shell,
                                                   TV* __restrict__ dinv, int* __restrict__ fail_shell) {
    const int ln = threadIdx.x & 15, sub = threadIdx.x >> 4;
    const int node = blockIdx.x * 16 + sub;
    const bool act = node < nnodes;
    const int c = ln < 12 ? ln : 0;   // lanes 12..15 carry a copy of column 0, never stored
    double a[12];
    if (act) {
        const size_t base = (size_t)diag_blk[node] * 144;
        const bool fc = is_free(fm, node, c);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const size_t at = base + sym12_pos(i, c);
            double v = vals_fp32 ? (double)((const float*)vals)[at] : ((const double*)vals)[at];
            const bool fr = is_free(fm, node, i);
            if (!fr || !fc) v = (i == c && !fr) ? 1.0 : 0.0;
            a[i] = v;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 12; ++i) a[i] = i == c ? 1.0 : 0.0;
    }
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        // column k of the current matrix, from lane k of the node's lanes
        double ck[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) ck[i] = __shfl(a[i], k, 16);
        double piv = ck[k];
        if (!(piv > 0.0)) {
            bad = true;
            piv = 1.0;
        }
        // row k of this column after scaling; column k becomes that of the
        // inverse of the eliminated part
        const double rk = (c == k ? 1.0 : a[k]) / piv;
#pragma unroll
        for (int i = 0; i < 12; ++i)
            if (i != k) a[i] = (c == k ? 0.0 : a[i]) - ck[i] * rk;
        a[k] = rk;
    }
    if (act && ln < 12) {
        // column ln = 2b + j goes into the stored blocks (a, b) of column
        // pair b: a = b - k (mod 6) at 12 a + 4 k, and a = b - 3 at 72 + 4 a
        const int bc = ln >> 1, j = ln & 1;
        TV* dn = dinv + (size_t)node * SYM12_VALS;
#pragma unroll
        for (int k = 1; k < 3; ++k) {
            const int r = (bc + 6 - k) % 6;
            dn[12 * r + 4 * k + j] = (TV)a[2 * r];
            dn[12 * r + 4 * k + 2 + j] = (TV)a[2 * r + 1];
        }
        if (bc >= 3) {
            const int r = bc - 3;
            dn[72 + 4 * r + j] = (TV)a[2 * r];
            dn[72 + 4 * r + 2 + j] = (TV)a[2 * r + 1];
        }
        if (j == 0) {
            dn[12 * bc] = (TV)a[2 * bc];
        } else {
            dn[12 * bc + 1] = dn[12 * bc + 2] = (TV)a[2 * bc];
            dn[12 * bc + 3] = (TV)a[2 * bc + 1];
        }
        if (ln == 0 && bad) atomicOr(&fail_shell[node_shell[node]], 1);
    }
}

__global__ void k_save_diag(int nnodes, const int* __restrict__ diag_blk, const void* __restrict__ vals, int fp32,
                            double* __restrict__ diag) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnodes * 12) return;
    const int node = t / 12, w = t % 12;
    const size_t at = (size_t)diag_blk[node] * 144 + sym12_pos(w, w);
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
    const size_t at = (size_t)diag_blk[node] * 144 + sym12_pos(w, w);
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
// Arrivals of a shell of more than CG_GROUPS blocks go through CG_GROUPS
// group counters on separate 128-byte lines and then one top counter, so no
// single address takes more than about nblk/CG_GROUPS (or CG_GROUPS) atomic
// operations per barrier; the blocks of a smaller shell arrive at the top
// counter itself (a group of one block would only add an atomic).
constexpr int CG_GROUPS = 4;
struct alignas(128) ShellSync {
    unsigned cnt;        // top-level arrivals (group leaders, or every block of a small shell), monotone
    unsigned pad0[31];
    unsigned gcnt[CG_GROUPS][32];   // per-group arrivals, monotone, one line each
};

// Barrier over the snb blocks of one shell that also sums one partial
// vector per block.  Each block writes its partials, publishes them (and the
// phase's vector writes) with one release fence and arrives; once the top
// counter shows every group complete, each block's first wavefront sums the
// shell's partials in block order -- the same operations in every block, so
// all blocks get the same, reproducible totals, and no block has to publish
// them for the others.  Partials are double-buffered by barrier parity
// (part[2][nblk][4]): a block overwrites its record of barrier k only at
// barrier k + 2, after every block has passed barrier k + 1 and so finished
// reading it.  Every wait is bounded: after 2^22 polls, or when another
// block has given up, the block sets abort and the kernel ends (legitimate
// waits are one matrix-product phase).
template <int N, int NW>
__device__ __forceinline__ bool reduce_barrier(ShellSync* ss, double* __restrict__ part, int blk, int sb0, int snb,
                                               unsigned k, double (&v)[N], int* abort_flag, double* lds,
                                               unsigned long long* arrive = nullptr) {
    __shared__ int s_ok;
    __shared__ double s_tot[N];
    block_sum<N, NW>(v, lds);
    // a shell of one block: its sum is the block's (the block sum's barrier
    // orders the phase's writes for the block's own next phase)
    if (snb == 1) return true;
    double* buf = part + (size_t)(k & 1) * 4 * gridDim.x;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int n = 0; n < N; ++n) buf[4 * (size_t)blk + n] = v[n];
        // one release fence publishes this block's vector writes and partials
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int ng = snb <= CG_GROUPS ? snb : CG_GROUPS;
        if (snb <= CG_GROUPS) {
            __hip_atomic_fetch_add(&ss->cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const int lb = blk - sb0, g = lb % ng;
            const unsigned gsize = (unsigned)((snb - g + ng - 1) / ng);
            const unsigned og =
                __hip_atomic_fetch_add(&ss->gcnt[g][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (og == gsize * (k + 1) - 1) {
                // last of its group: carry the group's arrival to the top counter
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_fetch_add(&ss->cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (arrive) *arrive = __builtin_amdgcn_s_memrealtime();
        // poll with plain coherent loads
        int ok = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(&ss->cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)ng * (k + 1)) {
            // the abort flag is looked at every 32nd poll, so a poll is one round trip
            if ((++spins & 31u) == 0 &&
                (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || spins > (1u << 22))) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        s_ok = ok;
    }
    __syncthreads();
    if (!s_ok) return false;
    if (threadIdx.x < 64) {
        // the wavefront of the polling thread: one acquire fence, then the
        // partials in block order (lane i: blocks i, i + 64, ...) and a
        // fixed butterfly over the lanes
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        double t[N];
#pragma unroll
        for (int n = 0; n < N; ++n) t[n] = 0.0;
        // up to 8 loads per lane in flight before the first add (these
        // partials come from other XCDs' L2s: one round trip each)
        constexpr int CH = 8;
        for (int i0 = threadIdx.x; i0 < snb; i0 += 64 * CH) {
            double pv[CH][N];
#pragma unroll
            for (int c = 0; c < CH; ++c)
#pragma unroll
                for (int n = 0; n < N; ++n)
                    pv[c][n] = i0 + 64 * c < snb ? __hip_atomic_load(&buf[4 * (size_t)(sb0 + i0 + 64 * c) + n],
                                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                                 : 0.0;
#pragma unroll
            for (int c = 0; c < CH; ++c)
#pragma unroll
                for (int n = 0; n < N; ++n)
                    if (i0 + 64 * c < snb) t[n] += pv[c][n];
        }
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) t[n] += __shfl_xor(t[n], off);
        if (threadIdx.x == 0)
#pragma unroll
            for (int n = 0; n < N; ++n) s_tot[n] = t[n];
    }
    __syncthreads();
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = s_tot[n];
    return true;
}

// ---------------------------------------------------- persistent CG
// Block-Jacobi preconditioned CG for every shell at once, in the
// single-reduction form of Chronopoulos and Gear: the matrix product is
// applied to the preconditioned residual u = Dinv r instead of to the
// search direction, and A p is carried along by its own recurrence, so the
// three scalars an iteration needs -- gamma = r.u, delta = u.A u and r.r --
// are ready together and one reduce-barrier per iteration suffices:
//   phase 1 (own rows; alpha, beta from the last barrier):
//            w = (stored part of A u) + own slots (masked),
//            p = u + beta p,  s = w + beta s   (s = A p),
//            x += alpha p,  r -= alpha s,  u = Dinv r (masked);
//            partial sums r.u and r.r
//   neighbour sync: every block waits for the blocks whose rows its stored
//            blocks reach (the blocks above it) to finish phase 1, so the
//            u it reads is new and the slots it writes have been read
//   phase 2: the stored blocks give the product of u (this lane's rows) and
//            A_ji u_i into the slots; u.A u = sum_i (2 u_i.w_i - u_i^T A_ii u_i)
//   reduce-barrier (gamma, delta, r.r): beta = gamma / gamma_old,
//            alpha = gamma / (delta - beta gamma / alpha_old), the last
//            denominator being p^T A p (<= 0: the system is not positive
//            definite).
// In exact arithmetic these are the iterates of the standard method; the
// neighbour sync replaces the second grid-wide barrier of that method (a
// wait on two or three blocks instead of every block of the shell), and the
// product reads one gathered vector (u) where the fused standard form read
// two (z and the old p).
// A lane handles the same node rows (one per pass over the block's rows) in
// every phase.  With MAXP > 0 the block has at most MAXP passes and r, x,
// p, s and the stored part of w of the lane's rows stay in registers for
// the whole solve (x is written once at the end): only u and the slots,
// which other rows read, go through memory.  Writes mixed into an
// HBM-bound read stream cost several times their share of the bytes, so
// keeping these vectors resident saves more than their bytes.  MAXP = 0:
// any number of passes, the vectors in memory (r, x, p, s, w).  Odd
// iterations take a block's passes last to first, so each phase starts on
// the rows the same phase of the previous iteration touched last, the ones
// most likely still cached.

// Publish this block's writes of the phase just ended and wait until the
// blocks blk+1 .. hi of the same shell have published theirs (flag value k,
// monotone).  Bounded like reduce_barrier.
// A shell of one block (solo) has no other block to publish to or wait
// for: the block barrier alone orders its phases.
__device__ __forceinline__ bool neighbour_sync(unsigned* __restrict__ flags, int blk, int hi, unsigned k,
                                               int* abort_flag, bool solo) {
    __shared__ int s_nok;
    __syncthreads();
    if (solo) return true;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&flags[32 * (size_t)blk], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        unsigned spins = 0;
        for (int b2 = blk + 1; b2 <= hi && ok; ++b2)
            while (__hip_atomic_load(&flags[32 * (size_t)b2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
                if ((++spins & 31u) == 0 &&
                    (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || spins > (1u << 22))) {
                    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_nok = ok;
    }
    __syncthreads();
    return s_nok != 0;
}

template <class TM, class TV, int NT, int MAXP>
__global__ __launch_bounds__(NT, MAXP == 1 ? 2 : 1) void k_cg(
    const int* __restrict__ blk_shell, const int* __restrict__ blk_row0, const int* __restrict__ blk_row1,
    const int* __restrict__ shell_blk0, const int* __restrict__ shell_nblk, const int* __restrict__ blk_nbhi, SymBsr m,
    const TM* __restrict__ vals, const TV* __restrict__ dinv, const uint16_t* __restrict__ fm,
    const double* __restrict__ b, TV* __restrict__ x, TV* __restrict__ r, TV* __restrict__ u, TV* __restrict__ p,
    TV* __restrict__ s, TV* __restrict__ w, TV* __restrict__ slot, double* __restrict__ partial,
    ShellSync* __restrict__ sync, unsigned* __restrict__ nbflag, int* __restrict__ abort_flag,
    const double* __restrict__ rtol2_shell, const int* __restrict__ maxit_shell, const int* __restrict__ active_shell,
    CgShellOut* __restrict__ out, unsigned long long* __restrict__ trace) {
    constexpr int R = Lay<TM>::R, L = Lay<TM>::L, G = Lay<TM>::G;
    constexpr int NW = NT / 64;
    constexpr int NP = MAXP > 0 ? MAXP : 1;   // register-resident passes
    __shared__ double lds[4 * NW];
    __shared__ TV red[NW][64 * 12];
    __shared__ TV xls[NW][G * 12];
    const int blk = blockIdx.x;
    const int sh = blk_shell[blk];
    const int row0 = blk_row0[blk], row1 = blk_row1[blk];
    const int sb0 = shell_blk0[sh], snb = shell_nblk[sh];
    const int nbhi = blk_nbhi[blk];
    ShellSync* ss = sync + sh;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane / L, t = lane % L;
    const bool lane_ok = grp < G;
    const int gsrc = lane_ok ? lane - t : 0;   // first lane of this lane's group
    const int rows_per_pass = NW * G;
    unsigned nbar = 0, nnb = 0;
    const bool leader = blk == sb0 && threadIdx.x == 0;

    if (!active_shell[sh]) {
        for (int e = threadIdx.x; e < (row1 - row0) * 12; e += blockDim.x) x[(size_t)row0 * 12 + e] = TV(0);
        if (leader) out[sh] = CgShellOut{0, 0, 0.0, 0.0};
        return;
    }

    // Resident vectors of the lane's rows (MAXP > 0): r and w in registers,
    // x, p and s (each touched once per iteration) in LDS, which leaves the
    // registers the product needs.  Entry 0 of each register array belongs
    // to the current pass; after every pass (taken or not) the arrays rotate
    // by one, so the loop body is emitted once and indexes its registers
    // statically.  Register order: r, w.
    constexpr int NV = 2;
    TV res[NV][NP][R];
    constexpr int LROWS = MAXP > 0 ? MAXP * NW * G : 1;
    __shared__ TV xres[LROWS * 12], pres[LROWS * 12], sres[LROWS * 12];
    auto rotate = [&](bool back) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int i = 0; i < R; ++i) {
                if (back) {
                    const TV e = res[v][NP - 1][i];
#pragma unroll
                    for (int q = NP - 1; q > 0; --q) res[v][q][i] = res[v][q - 1][i];
                    res[v][0][i] = e;
                } else {
                    const TV e = res[v][0][i];
#pragma unroll
                    for (int q = 0; q + 1 < NP; ++q) res[v][q][i] = res[v][q + 1][i];
                    res[v][NP - 1][i] = e;
                }
            }
    };
    // runs f(base) over the block's passes, last pass first if rev
    auto passes = [&](auto&& f, bool rev = false) {
        if constexpr (MAXP > 0) {
#pragma unroll 1
            for (int i = 0; i < MAXP; ++i) {
                if (rev) rotate(true);
                const int base = row0 + (rev ? MAXP - 1 - i : i) * rows_per_pass;
                if (base < row1) f(base);
                if (!rev) rotate(false);
            }
        } else {
            const int np = (row1 - row0 + rows_per_pass - 1) / rows_per_pass;
            for (int i = 0; i < np; ++i) f(row0 + (rev ? np - 1 - i : i) * rows_per_pass);
        }
    };
    // vector v (0 r, 1 x, 2 p, 3 s, 4 w) of this lane's entry i of the pass
    // starting at row `base` (global entry `at`)
    TV* const vmem[5] = {r, x, p, s, w};
    auto lds_at = [&](int base, int i) {
        return (size_t)(((base - row0) / rows_per_pass) * NW * G + wv * G + grp) * 12 + R * t + i;
    };
    auto vget = [&](int v, int base, size_t at, int i) -> TV {
        if constexpr (MAXP > 0) {
            if (v == 1) return xres[lds_at(base, i)];
            if (v == 2) return pres[lds_at(base, i)];
            if (v == 3) return sres[lds_at(base, i)];
            return res[v == 0 ? 0 : 1][0][i];
        } else {
            return vmem[v][at];
        }
    };
    auto vset = [&](int v, int base, size_t at, int i, TV val) {
        if constexpr (MAXP > 0) {
            if (v == 1) xres[lds_at(base, i)] = val;
            else if (v == 2) pres[lds_at(base, i)] = val;
            else if (v == 3) sres[lds_at(base, i)] = val;
            else res[v == 0 ? 0 : 1][0][i] = val;
        } else {
            vmem[v][at] = val;
        }
    };

    // z = Dinv r for this lane's rows 2t, 2t+1 of node: the six 2x2 blocks
    // (t, b), b = t + k (mod 6), of the packed inverse times r of column
    // pair b, which lane b of the group holds
    static_assert(R == 2, "the packed inverse is read by row pairs");
    auto precond = [&](int node, const TV* rr, TV* zz) {
        // the lane-dependent offsets below are recomputed per call (an
        // opaque copy of t): hoisted out of the iteration loop they would
        // hold 9 registers through it
        int t = Lay<TM>::L;
        t = lane % t;
        asm volatile("" : "+v"(t));
        const TV* dn = dinv + (size_t)node * SYM12_VALS;
        TV mm[6][4];
        TV s0 = TV(0), s1 = TV(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            if (k == 0 || k == 3) {
                // three blocks at a time
                __builtin_amdgcn_sched_barrier(0);
                if (k == 0) {
#pragma unroll
                    for (int h = 0; h < 3; ++h) Vec4<TV>::ld(dn + 12 * t + 4 * h, mm[h]);   // (t, t+h)
                } else {
                    Vec4<TV>::ld(dn + 72 + 4 * (t % 3), mm[3]);         // (t, t+3), transposed for t >= 3
                    Vec4<TV>::ld(dn + 12 * ((t + 4) % 6) + 8, mm[4]);   // (t-2, t), transposed
                    Vec4<TV>::ld(dn + 12 * ((t + 5) % 6) + 4, mm[5]);   // (t-1, t), transposed
                }
            }
            const int src = gsrc + (t + k) % 6;
            const TV r0 = __shfl(rr[0], src), r1 = __shfl(rr[1], src);
            const bool tr = k >= 4 || (k == 3 && t >= 3);
            const TV m01 = tr ? mm[k][2] : mm[k][1], m10 = tr ? mm[k][1] : mm[k][2];
            s0 += mm[k][0] * r0;
            s0 += m01 * r1;
            s1 += m10 * r0;
            s1 += mm[k][3] * r1;
        }
        zz[0] = s0;
        zz[1] = s1;
    };

    // phase 2: the product of u over the lane's rows: w (stored part) and
    // the slots; returns the block-lane's share of u.A u
    auto product = [&](bool rev) {
        double uau = 0.0;
        passes([&](int base) {
            const int node = base + wv * G + grp;
            if (!(lane_ok && node < row1)) return;
            auto xe = [&](int col, TV* xv) {
#pragma unroll
                for (int i = 0; i < R; ++i) xv[i] = u[(size_t)col * 12 + R * t + i];
            };
            TV un[R], part[12], wr[R];
            xe(node, un);
            // FP32 blocks of one pass (small shells) load the next block's
            // values during the current one's products (in FP64 the two
            // blocks' registers spill and the plain order is faster)
            constexpr bool PF = MAXP == 1 && sizeof(TM) == 4;
            const TV dl = row_sym<TM, TV, false, sizeof(TM) == 8 || PF ? 12 : 4, decltype(xe), PF>(
                m, vals, node, t, un, xe, xls[wv] + grp * 12, slot, part);
            group_sum<TV, R, L>(part, lane, t, gsrc, red[wv], wr);
            uau -= (double)dl;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                vset(4, base, (size_t)node * 12 + R * t + i, i, wr[i]);
                uau += 2.0 * (double)un[i] * (double)wr[i];
            }
        }, rev);
        return uau;
    };

    // ---- init: r = b (masked), x = p = s = 0, u = Dinv r; sums r.u and b.b
    double sums[3] = {0.0, 0.0, 0.0};
    passes([&](int base) {
        const int node = base + wv * G + grp;
        const bool ok = lane_ok && node < row1;
        const int nd = ok ? node : row0;
        TV rr[R], zz[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int wd = R * t + i;
            rr[i] = ok && is_free(fm, node, wd) ? (TV)b[(size_t)node * 12 + wd] : TV(0);
        }
        precond(nd, rr, zz);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int wd = R * t + i;
            const size_t at = (size_t)nd * 12 + wd;
            if (!ok) continue;
            if (!is_free(fm, node, wd)) zz[i] = TV(0);
            vset(0, base, at, i, rr[i]);
            vset(1, base, at, i, TV(0));
            vset(2, base, at, i, TV(0));
            vset(3, base, at, i, TV(0));
            u[at] = zz[i];
            sums[0] += (double)rr[i] * (double)zz[i];
            sums[2] += (double)rr[i] * (double)rr[i];
        }
    });
    int it = 0, status = 1;
    if (!neighbour_sync(nbflag, blk, nbhi, ++nnb, abort_flag, snb == 1)) {
        if (leader) out[sh] = CgShellOut{0, 3, 0.0, 0.0};
        return;
    }
    sums[1] = product(false);
    if (!reduce_barrier<3, NW>(ss, partial, blk, sb0, snb, nbar++, sums, abort_flag, lds)) {
        if (leader) out[sh] = CgShellOut{0, 3, 0.0, 0.0};
        return;
    }
    double gamma = sums[0];
    const double bb = sums[2];
    const double tol2 = rtol2_shell[sh] * bb;
    const int maxit = maxit_shell[sh];
    if (bb == 0.0) {
        // x = 0 solves it (the resident instance would otherwise leave x
        // unwritten: it stores its LDS copy only after the iterations)
        for (int e = threadIdx.x; e < (row1 - row0) * 12; e += blockDim.x) x[(size_t)row0 * 12 + e] = TV(0);
        if (leader) out[sh] = CgShellOut{0, 0, 0.0, 0.0};
        return;
    }
    double rr2 = bb;
    double alpha = 0.0, beta = 0.0;
    if (!(sums[1] > 0.0)) {
        status = 2;   // p^T A p of the first direction (p = u)
    } else {
        alpha = gamma / sums[1];
        for (; it < maxit; ++it) {
            const bool rev = (it & 1) != 0;   // both phases of odd iterations run last to first
            // trace record of this block and iteration (first CG_TRACE_ITERS iterations, thread 0)
            unsigned long long* tr =
                trace && threadIdx.x == 0 && it < CG_TRACE_ITERS ? trace + ((size_t)blk * CG_TRACE_ITERS + it) * 6 : nullptr;
            if (tr) tr[0] = __builtin_amdgcn_s_memrealtime();
            // ---- phase 1
            double s1[3] = {0.0, 0.0, 0.0};
            passes([&](int base) {
                const int node = base + wv * G + grp;
                const bool ok = lane_ok && node < row1;
                const int nd = ok ? node : row0;
                // every load of the row is issued before the first use
                const unsigned fmask = fm[nd];
                const int k0 = m.lptr[nd], k1 = m.lptr[nd + 1];
                TV rr[R], ww[R], uo[R];
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const size_t at = (size_t)nd * 12 + R * t + i;
                    rr[i] = vget(0, base, at, i);
                    ww[i] = vget(4, base, at, i);
                    uo[i] = u[at];
                }
                // the transposed products of the rows above (4 per interior node)
                for (int k = k0; k < k1; k += 4) {
                    TV sv[4][R];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int kk = k + q < k1 ? k + q : k0;
                        VecLoad<TV, R>::ld(slot + (size_t)kk * 12 + R * t, sv[q]);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int i = 0; i < R; ++i)
                            if (k + q < k1) ww[i] += sv[q][i];
                }
                TV zz[R];
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const size_t at = (size_t)nd * 12 + R * t + i;
                    const bool fr = (fmask >> (R * t + i)) & 1u;
                    const TV pn = uo[i] + (TV)beta * vget(2, base, at, i);
                    const TV sn = (fr ? ww[i] : TV(0)) + (TV)beta * vget(3, base, at, i);
                    if (ok) {
                        vset(1, base, at, i, vget(1, base, at, i) + (TV)alpha * pn);
                        vset(2, base, at, i, pn);
                        vset(3, base, at, i, sn);
                    }
                    rr[i] -= (TV)alpha * sn;
                }
                precond(nd, rr, zz);
                if (ok) {
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        const int wd = R * t + i;
                        const size_t at = (size_t)node * 12 + wd;
                        if (!((fmask >> wd) & 1u)) zz[i] = TV(0);
                        vset(0, base, at, i, rr[i]);
                        u[at] = zz[i];
                        s1[0] += (double)rr[i] * (double)zz[i];
                        s1[2] += (double)rr[i] * (double)rr[i];
                    }
                }
            }, rev);
            if (tr) tr[1] = __builtin_amdgcn_s_memrealtime();
            if (!neighbour_sync(nbflag, blk, nbhi, ++nnb, abort_flag, snb == 1)) {
                status = 3;
                break;
            }
            if (tr) tr[2] = __builtin_amdgcn_s_memrealtime();
            // ---- phase 2
            s1[1] = product(rev);
            if (tr) tr[3] = __builtin_amdgcn_s_memrealtime();
            if (tr) tr[4] = 0;
            if (!reduce_barrier<3, NW>(ss, partial, blk, sb0, snb, nbar++, s1, abort_flag, lds, tr ? tr + 4 : nullptr)) {
                status = 3;
                break;
            }
            if (tr) tr[5] = __builtin_amdgcn_s_memrealtime();
            rr2 = s1[2];
            if (rr2 <= tol2) {
                status = 0;
                ++it;
                break;
            }
            beta = s1[0] / gamma;
            const double den = s1[1] - beta * s1[0] / alpha;   // p^T A p of the next direction
            if (!(den > 0.0)) {
                status = 2;
                ++it;
                break;
            }
            alpha = s1[0] / den;
            gamma = s1[0];
        }
    }
    if constexpr (MAXP > 0) {
        // the solution of the lane's rows, once
        passes([&](int base) {
            const int node = base + wv * G + grp;
            if (!(lane_ok && node < row1)) return;
#pragma unroll
            for (int i = 0; i < R; ++i) x[(size_t)node * 12 + R * t + i] = xres[lds_at(base, i)];
        });
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

// One wavefront per shell: lane l sums the shell's block partials l, l + 64,
// ... in order, then a fixed butterfly over the lanes.
__global__ __launch_bounds__(64) void k_shell_dot_fin(int nshell, const int* __restrict__ shell_blk0,
                                                      const int* __restrict__ shell_nblk,
                                                      const double* __restrict__ part, double* __restrict__ out) {
    const int s = blockIdx.x;
    if (s >= nshell) return;
    const int b0 = shell_blk0[s], nb = shell_nblk[s];
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += 64) v += part[b0 + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (threadIdx.x == 0) out[s] = v;
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

// two vectors at once: dst0 = src0 and dst1 = src1 on the flagged shells
__global__ void k_copy_shell2(int n, const double* __restrict__ src0, const double* __restrict__ src1,
                              const int* __restrict__ node_shell, const int* __restrict__ flag_shell,
                              double* __restrict__ dst0, double* __restrict__ dst1) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && flag_shell[node_shell[t / 12]]) {
        dst0[t] = src0[t];
        dst1[t] = src1[t];
    }
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

// Up to three buffers zeroed by one launch (blockIdx.y picks the buffer).
struct ZeroSpan {
    uint4* p;
    size_t n16;
    uint32_t* tail;
    size_t n4;
};
__global__ void k_zero_spans(ZeroSpan a, ZeroSpan b, ZeroSpan c) {
    const ZeroSpan z = blockIdx.y == 0 ? a : blockIdx.y == 1 ? b : c;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = t; i < z.n16; i += stride) z.p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (t < z.n4) z.tail[t] = 0u;
}

// ------------------------------------------------------------ launchers
static inline dim3 grid1(int n) { return dim3((n + 255) / 256); }

void launch_zero(hipStream_t st, void* p, size_t bytes) {
    const size_t n16 = bytes / 16, n4 = (bytes % 16) / 4;
    const size_t blocks = std::min<size_t>(std::max<size_t>((n16 + 255) / 256, 1), 4096);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, n16, (uint4*)p, n4,
                       (uint32_t*)((char*)p + n16 * 16));
}

void launch_zero3(hipStream_t st, void* p0, size_t b0, void* p1, size_t b1, void* p2, size_t b2) {
    auto span = [](void* p, size_t bytes) {
        return ZeroSpan{(uint4*)p, bytes / 16, (uint32_t*)((char*)p + bytes / 16 * 16), (bytes % 16) / 4};
    };
    const size_t n16 = std::max(b0, std::max(b1, b2)) / 16;
    const size_t blocks = std::min<size_t>(std::max<size_t>((n16 + 255) / 256, 1), 4096);
    hipLaunchKernelGGL(k_zero_spans, dim3((unsigned)blocks, 3), dim3(256), 0, st, span(p0, b0), span(p1, b1),
                       span(p2, b2));
}

template <class TM>
void launch_spmv(hipStream_t st, int nnodes, const SymBsr& m, const TM* vals, const uint16_t* freemask,
                 const double* x, const double* b, double* y, double* slot, int mode) {
    if (nnodes == 0) return;
    const int rows_per_block = 4 * Lay<TM>::G;
    const dim3 grid((nnodes + rows_per_block - 1) / rows_per_block);
    const uint16_t* fc = (mode & 1) ? freemask : nullptr;         // free columns only
    const uint16_t* fr = (mode & (1 | 8)) ? freemask : nullptr;   // free rows only
    if (mode & 2)
        hipLaunchKernelGGL((k_spmv_rows<TM, true>), grid, dim3(256), 0, st, nnodes, m, vals, fc, x, y, slot);
    else
        hipLaunchKernelGGL((k_spmv_rows<TM, false>), grid, dim3(256), 0, st, nnodes, m, vals, fc, x, y, slot);
    const double* bb = (mode & 4) ? b : nullptr;
    if ((((uintptr_t)y | (uintptr_t)bb) & 15u) == 0)
        hipLaunchKernelGGL(k_spmv_fin, grid1(nnodes * 6), dim3(256), 0, st, nnodes, m.lptr, slot, fr, bb, y);
    else
        hipLaunchKernelGGL(k_spmv_fin1, grid1(nnodes * 12), dim3(256), 0, st, nnodes, m.lptr, slot, fr, bb, y);
}
template void launch_spmv<double>(hipStream_t, int, const SymBsr&, const double*, const uint16_t*, const double*,
                                  const double*, double*, double*, int);
template void launch_spmv<float>(hipStream_t, int, const SymBsr&, const float*, const uint16_t*, const double*,
                                 const double*, double*, double*, int);

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

// Passes over a block's rows up to which the CG keeps its own rows' vectors
// in registers and LDS (beyond it the memory instance runs): 4 for FP64
// matrices at most 512 threads per block, none for FP64 at 1024 threads
// (the LDS would not hold them), 2 for FP32, within the register budget.
template <class TM> constexpr int cg_maxp(int nthreads) {
    return sizeof(TM) == 8 ? (nthreads <= 512 ? 4 : 0) : 2;
}

// the CG kernel instance for a block size of 256, 512 or 1024 threads,
// register-resident vectors or not
template <class TM, class TV> const void* cg_fn(int nthreads, bool resident) {
    if (resident)
        return nthreads == 1024 ? (const void*)k_cg<TM, TV, 1024, cg_maxp<TM>(1024)>
               : nthreads == 512 ? (const void*)k_cg<TM, TV, 512, cg_maxp<TM>(512)>
                                 : (const void*)k_cg<TM, TV, 256, cg_maxp<TM>(256)>;
    return nthreads == 1024 ? (const void*)k_cg<TM, TV, 1024, 0>
           : nthreads == 512 ? (const void*)k_cg<TM, TV, 512, 0>
                             : (const void*)k_cg<TM, TV, 256, 0>;
}

template <class TM, class TV>
hipError_t launch_cg(hipStream_t st, int nblk, int nthreads, const RowBlocks& rb, const SymBsr& m, const TM* vals,
                     const TV* dinv, const uint16_t* freemask, const double* b, TV* x, TV* r, TV* u, TV* p, TV* s,
                     TV* w, TV* slot, double* partial, void* sync, unsigned* nbflag, int* abort_flag,
                     const double* rtol2_shell, const int* maxit_shell, const int* active_shell, CgShellOut* out,
                     unsigned long long* trace) {
    ShellSync* ss = static_cast<ShellSync*>(sync);
    SymBsr mm = m;
    void* args[] = {(void*)&rb.blk_shell, (void*)&rb.blk_row0, (void*)&rb.blk_row1, (void*)&rb.shell_blk0,
                    (void*)&rb.shell_nblk, (void*)&rb.blk_nbhi, (void*)&mm, (void*)&vals, (void*)&dinv,
                    (void*)&freemask, (void*)&b, (void*)&x, (void*)&r, (void*)&u, (void*)&p, (void*)&s, (void*)&w,
                    (void*)&slot, (void*)&partial, (void*)&ss, (void*)&nbflag, (void*)&abort_flag,
                    (void*)&rtol2_shell, (void*)&maxit_shell, (void*)&active_shell, (void*)&out, (void*)&trace};
    const int pass = (nthreads / 64) * Lay<TM>::G;
    const bool resident = rb.max_rows <= cg_maxp<TM>(nthreads) * pass;
    // 256-thread blocks of one pass: the instance that loads the next
    // stored block ahead
    const void* fn = nthreads == 256 && rb.max_rows <= pass ? (const void*)k_cg<TM, TV, 256, 1>
                                                            : cg_fn<TM, TV>(nthreads, resident);
    return hipLaunchCooperativeKernel(fn, dim3(nblk), dim3(nthreads), args, 0, st);
}
template hipError_t launch_cg<double, double>(hipStream_t, int, int, const RowBlocks&, const SymBsr&, const double*,
                                              const double*, const uint16_t*, const double*, double*, double*,
                                              double*, double*, double*, double*, double*, double*, void*, unsigned*,
                                              int*, const double*, const int*, const int*, CgShellOut*,
                                              unsigned long long*);
template hipError_t launch_cg<float, float>(hipStream_t, int, int, const RowBlocks&, const SymBsr&, const float*,
                                            const float*, const uint16_t*, const double*, float*, float*, float*,
                                            float*, float*, float*, float*, double*, void*, unsigned*, int*,
                                            const double*, const int*, const int*, CgShellOut*, unsigned long long*);

size_t cg_sync_bytes() { return sizeof(ShellSync); }
int cg_rows_per_pass(int tm_fp32, int nthreads) { return (nthreads / 64) * (tm_fp32 ? Lay<float>::G : Lay<double>::G); }

int cg_max_blocks(int device, int tm_fp32, int nthreads) {
    int per_cu = 0, cus = 0;
    // the register-resident instance: it needs at least the registers of the other
    int per_cu2 = 0;
    const void* fn = tm_fp32 ? cg_fn<float, float>(nthreads, true) : cg_fn<double, double>(nthreads, true);
    const void* fn2 = tm_fp32 ? cg_fn<float, float>(nthreads, false) : cg_fn<double, double>(nthreads, false);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nthreads, 0) != hipSuccess) return -1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, fn2, nthreads, 0) != hipSuccess) return -1;
    per_cu = per_cu < per_cu2 ? per_cu : per_cu2;
    if (nthreads == 256) {   // and the one-pass instance
        const void* fn1 = tm_fp32 ? (const void*)k_cg<float, float, 256, 1> : (const void*)k_cg<double, double, 256, 1>;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, fn1, nthreads, 0) != hipSuccess) return -1;
        per_cu = per_cu < per_cu2 ? per_cu : per_cu2;
    }
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return -1;
    return per_cu * cus;
}

void launch_shell_dot(hipStream_t st, const RowBlocks& rb, int nshell, const double* x, const double* y,
                      const uint16_t* freemask, double* partial, double* out) {
    hipLaunchKernelGGL(k_shell_dot_part, dim3(rb.nblk), dim3(256), 0, st, rb.blk_row0, rb.blk_row1, x, y, freemask,
                       partial);
    hipLaunchKernelGGL(k_shell_dot_fin, dim3(nshell), dim3(64), 0, st, nshell, rb.shell_blk0, rb.shell_nblk,
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
void launch_copy_shell2(hipStream_t st, int nnodes, const double* src0, const double* src1, const int* node_shell,
                        const int* flag_shell, double* dst0, double* dst1) {
    const int n = nnodes * 12;
    hipLaunchKernelGGL(k_copy_shell2, grid1(n), dim3(256), 0, st, n, src0, src1, node_shell, flag_shell, dst0, dst1);
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
