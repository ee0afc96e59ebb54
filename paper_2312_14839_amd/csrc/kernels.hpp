// Host-side launchers of the libbhem kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace bhem {

// ------------------------------------------------------- patch kernels
// phi: the basis table Phi_g[a][I] at 96 g + 16 a + I (16 Gauss points x 6
// slots x 16 local basis functions); launch_hessian and launch_energy_grad
// also read the copies that follow it: its transpose at 1536 + 16 (16 a + I)
// + g, and by pairs at 3072 + 32 (8 a + I / 2) + 2 g + I % 2 and at
// 4608 + 32 (3 g + a / 2) + 2 I + a % 2
void launch_energy_grad(hipStream_t st, int npatch, const int4* patch_nodes, const int* patch_shell,
                        const ShellParams* shells, const double* phi, const double* q, const double* qbar,
                        const double* qhat, double mass_scale, double dt_damp, int elastic, int loads,
                        const int* eval_shell /* NULL: every shell */, double* e_patch, double* g_patch,
                        int patches_per_block /* 4, 8 or 16 */);
void launch_gather_grad(hipStream_t st, int nnodes, const int* inc_ptr, const int* inc, const double* g_patch,
                        const uint16_t* freemask, const int* node_shell, const int* write_shell, double* grad);
void launch_shell_energy(hipStream_t st, int nshell, const ShellParams* shells, const double* e_patch,
                         double* e_shell);
// per-patch pressure loads (pressure[shell], per unit current area along
// a_1 x a_2) into g_patch [P][48], to be gathered to nodes
void launch_pressure(hipStream_t st, int npatch, const int4* patch_nodes, const int* patch_shell,
                     const ShellParams* shells, const double* pressure, const double* phi, const double* q,
                     double* g_patch);
// patch_slots[16 * p + m]: stored block of the patch's m-th stored local block
// (-1 past the last), patch_kid[p]: its local block index in bits 4m..4m+3,
// patch_first[p]: bit m set where patch p is the first to reach that block
template <class T>
void launch_hessian(hipStream_t st, const int* patch_list, int nlist, const int4* patch_nodes, const int* patch_shell,
                    const int* patch_slots, const uint64_t* patch_kid, const uint16_t* patch_first,
                    const ShellParams* shells, const double* phi, const double* q, const double* qbar,
                    double mass_scale, double dt_damp, int elastic, int pseudo, T* vals,
                    int waves /* patches (wavefronts) per block: 4 or 8 */,
                    T* scr /* NULL: add into vals; else each stored local block to scr[(10 p + m) 144] */);
// patches whose Hessian blocks (4 patches each) are all resident on the device at once
int hessian_resident_patches(int device, int fp32);
// vals[sb] = sum over k in cptr[sb] .. cptr[sb + 1] of scr[cidx[k]] (144 values,
// 84 where diag[sb]): the assembly of launch_hessian's scratch output
template <class T>
void launch_gather_blocks(hipStream_t st, int nsb, const int* cptr, const int* cidx, const uint8_t* diag, const T* scr,
                          T* vals);

// --------------------------------------------------------- ray kernels
// ctrl: [P][4][4][3] Bezier control points, p_ij at ((4p + i)*4 + j)*3.
void launch_bezier(hipStream_t st, int npatch, const int4* patch_nodes, const int* patch_shell,
                   const ShellParams* shells, const double* q, double* ctrl);

constexpr int RAY_HEAP_MAX = 64;       // candidate surfaces one ray can hold
constexpr int RAY_MAX_DEPTH = 60;      // depth field of a heap entry: 6 bits
constexpr int RAY_MAX_PATCHES = (1 << 24) - 1;
constexpr int RAY_LDS_PATCHES = 128;   // scenes up to this size are staged in LDS
constexpr int RAY_MAX_POPS = 1 << 18;  // candidates one ray may examine
constexpr int RAY_CHUNK_PER_LANE = 8;  // rays per block = 256 lanes x this
constexpr int RAY_TAIL_BUDGET = 512;   // candidates before a ray goes to the cooperative search
constexpr int RAY_TAIL_SLOTS = 16384;  // rays the cooperative search takes per launch
constexpr int RAY_TAIL_STATIC_SLOTS = 4096;   // the same with the library's fixed buffer

struct RayParams {
    double eps;          // a surface whose box diagonal is <= eps |d| ends the subdivision
    double newton_tol;   // Newton converged when |x(u,v) - x0 - tau d| <= newton_tol
    double hole;         // abandoned half-width around a Newton hit, fraction of the rectangle
    int newton_iters;    // 0: midpoint subdivision only
    int max_depth;       // <= RAY_MAX_DEPTH
    int heap_cap;        // <= RAY_HEAP_MAX
};
// hit: [n][3] tau, u, v; patch: [n] (-1 miss, -2 heap full or RAY_MAX_POPS
// candidates examined, -3 invalid ray);
// pops: [n] surfaces popped, may be null.
// fixed_tail: NULL, or the device address of the library's fixed hand-over
// buffer (ray_scratch_address): no allocation, room for RAY_TAIL_STATIC_SLOTS
// handed-over rays
void launch_ray_cast(hipStream_t st, const double* ctrl, int npatch, const double* rays, long long nrays,
                     const RayParams& o, double* hit, int* patch, int* pops, void* fixed_tail = nullptr);
// Device address of the fixed hand-over buffer on `device`, which must be
// the current device (looked up once per device, then cached).
hipError_t ray_scratch_address(int device, void** out);
// Moving point x0 + t w (pts: [n][6]) against patches with control points
// ctrl + t vel over [0, dt]; hit: [n][3] t, u, v; statuses as above.
void launch_ccd(hipStream_t st, const double* ctrl, const double* vel, int npatch, const double* pts,
                long long npts, double dt, const RayParams& o, double* hit, int* patch, int* pops);

// ----------------------------------------------------- collision kernels
// A static collider: kind 0 plane through p with unit normal n (the shell
// on the side n points to), kind 1 sphere of centre p and radius r.
struct CollCollider {
    int kind;
    double p[3], n[3], r;
};
// One resolved contact: its sample, collider, patch nodes and 16 shape
// function values, the sample point x at the rolled-back state, the
// collider's normal and two tangents (dir[0..2]), the point p on the
// collider and the normal velocity of the sample before the response.
struct CollContact {
    int sample, collider, node[4];
    double phi[16];
    double dir[3][3];
    double x[3], p[3];
    double vn;
};
// per sample (s x s per patch): earliest contact time tc (inf: none) and
// collider cid; blk_min[b]: the smallest tc of block b (256 samples)
void launch_coll_samples(hipStream_t st, int nsamp, int s, const int4* patch_nodes, const int* patch_shell,
                         const ShellParams* shells, const double* qn, const double* q1, double dt,
                         const CollCollider* cols, int ncol, double* tc, int* cid, double* blk_min);
void launch_coll_count(hipStream_t st, int nsamp, const double* tc, double thr, int* blk_cnt);
void launch_coll_compact(hipStream_t st, int nsamp, const double* tc, double thr, const int* blk_off, int* list);
void launch_coll_rollback(hipStream_t st, int n, const double* qn, const double* q1, double f, double* qs);
void launch_coll_setup(hipStream_t st, int ncon, int s, const int* list, const int* cid, const int4* patch_nodes,
                       const int* patch_shell, const ShellParams* shells, const double* qs, const double* v,
                       const CollCollider* cols, CollContact* out);
// y = J^T lam as nodal vector (inc: per node its (contact, corner) pairs);
// rows of contact j: row_of[j] .. + m - 1 (row_of[j] < 0: none)
void launch_coll_scatter(hipStream_t st, int nnodes, const int* inc_ptr, const int2* inc, const CollContact* con,
                         const int* row_of, int m, const double* lam, const uint16_t* fm, double* y);
void launch_coll_gather(hipStream_t st, int ncon, const CollContact* con, const int* row_of, int m, const double* z,
                        double* out);

// ------------------------------------------------- point constraints
// Constraint x^(kind)(xi) = target at a midsurface point: its patch's four
// nodes and the 16 shape-function values psi[4c + k] of that kind (corner c,
// DOF kind k), so that c = sum_I psi_I q[node[I / 4]][3 (I % 4) + comp] - target.
struct AlmPoint {
    int node[4];
    double psi[16];
    double target[3];
};
// grad += C^T (kappa c - lam) on free DOFs (fm NULL: all) of the nodes of
// shells with write_shell set (all if NULL); inc: per node its
// (constraint, corner) pairs
void launch_alm_grad(hipStream_t st, int nnodes, const int* incp, const int2* inc, const AlmPoint* pts,
                     const double* lam, double kappa, const double* q, const uint16_t* fm, const int* node_shell,
                     const int* write_shell, double* grad);
// e_shell[3 s + 2] += sum over the shell's constraints of -lam.c + kappa/2 |c|^2
void launch_alm_energy(hipStream_t st, int nshell, const int* shell_pt, const AlmPoint* pts, const double* lam,
                       double kappa, const double* q, double* e_shell);
// out[3 j + comp] = c_j
void launch_alm_residual(hipStream_t st, int npts, const AlmPoint* pts, const double* q, double* out);
// vals[pos[i]] += val[i], distinct positions (vals FP32 or FP64)
void launch_add_sparse(hipStream_t st, int n, const long long* pos, const double* val, void* vals, int vals_fp32);

// ------------------------------------------------------ solver kernels
// Row partition of the node rows into blocks that never straddle a shell;
// used by the CG kernel and by the per-shell reductions.
struct RowBlocks {
    int nblk;
    int max_rows;            // node rows of the largest block (INT32_MAX: never register-resident)
    const int* blk_shell;    // [nblk]
    const int* blk_row0;     // [nblk]
    const int* blk_row1;     // [nblk]
    const int* shell_blk0;   // [nshell]
    const int* shell_nblk;   // [nshell]
    const int* blk_nbhi;     // [nblk] highest block of the shell owning a column of this block's stored blocks
};

struct CgShellOut {
    int iters, status;       // status: 0 converged, 1 iteration cap, 2 p^T A p <= 0, 3 barrier timeout
    double bnorm2, rnorm2;   // ||b||^2 and the final recursive ||r||^2
};

// Per-shell state of the device-driven Newton iteration (newton_kernels.hip):
// written by the host before each iteration, updated by the control kernels
// between the iteration's matrix and vector kernels, read back once.
constexpr int NT_STATUS_OK = 0, NT_STATUS_NOT_CONVERGED = -4;   // shell_status values
// stage at which a shell leaves the device iteration to the host
constexpr int NT_HOST_FACTOR = 1, NT_HOST_INDEFINITE = 2, NT_HOST_LINESEARCH = 3, NT_HOST_REFINE = 4;
struct NewtonCtl {
    double E, Escale, gn, g0;           // incremental potential, its scale, ||g||, ||g|| at the step's start
    double floor, grad_norm_checked;    // rounding floor and ||g|| at the last convergence test
    double slope, alpha, a_prev, E_prev;   // line search
    double bn2, prev, relres;           // refinement (mixed form): ||b||^2, last relative residual
    int active;                         // the shell iterates
    int k;                              // Newton iterations of this step
    int status;                         // shell status once inactive
    int need_host;                      // 0 or the NT_HOST_ stage the host takes over at
    int solving, refining, searching, steepest, trial;
    int pcg_iters, solve_iters, sweeps, backtracks, newton_iters;   // counted on the device
    int fault;                          // a CG launch gave up on its grid barrier (status 3)
};
void launch_nt_factor(hipStream_t st, int S, NewtonCtl* ctl, const int* fail_shell, int* cg_active, double* cg_rtol2,
                      int* cg_maxit, double pcg_rtol, int pcg_maxit);
void launch_nt_cg64(hipStream_t st, int S, NewtonCtl* ctl, const CgShellOut* out, int* flag_shell);
void launch_nt_ref_init(hipStream_t st, int S, NewtonCtl* ctl, const double* red, int* cg_active, double* cg_rtol2,
                        double pcg_rtol);
void launch_nt_ref_cg(hipStream_t st, int S, NewtonCtl* ctl, const CgShellOut* out, int* cg_active);
void launch_nt_ref_check(hipStream_t st, int S, NewtonCtl* ctl, const double* red, int* cg_active, double* cg_rtol2,
                         double pcg_rtol, int pcg_maxit);
void launch_nt_ref_end(hipStream_t st, int S, NewtonCtl* ctl, int* flag_shell);
void launch_nt_ls_init(hipStream_t st, int S, NewtonCtl* ctl, const double* red, double* alpha_shell,
                       int* flag_shell, int* write_shell);
void launch_nt_ls_step(hipStream_t st, int S, int trial, NewtonCtl* ctl, const double* e_shell, const double* red,
                       double* alpha_shell, int* flag_shell, int* write_shell);
void launch_nt_ls_end(hipStream_t st, int S, NewtonCtl* ctl);
void launch_nt_check(hipStream_t st, int S, NewtonCtl* ctl, const double* red, double newton_rtol, int newton_maxit);

// Symmetric block storage: block row i stores its blocks (i, j >= i), the
// diagonal first; the stored block of pair (i, j) holds A_ji column-major
// (A_ij row-major).  The product by A_ji = A_ij^T belongs to row j: it is
// written to slot tslot[b] of the 12-value slot array (-1 for diagonal
// blocks), and row j's slots are lptr[j] .. lptr[j+1].
struct SymBsr {
    const int* row_ptr;   // [nnodes + 1] stored blocks per block row
    const int* col_idx;   // [stored blocks] column node
    const int* tslot;     // [stored blocks] slot of the transposed product
    const int* lptr;      // [nnodes + 1] slots of each row
};

// y = A x; slot: scratch of 12 doubles per stored off-diagonal block
template <class TM>
void launch_spmv(hipStream_t st, int nnodes, const SymBsr& m, const TM* vals, const uint16_t* freemask,
                 const double* x, const double* b, double* y, double* slot, int mode);
// mode bits: 1 masked (free rows and columns only), 2 abs values (|A| |x|), 4 residual y = b - A x,
// 8 free rows only (all columns)

// Symmetric 12x12 blocks (the matrix's diagonal node blocks and their
// block-Jacobi inverses) keep their 21 distinct 2x2 blocks (row pair a,
// column pair b), each row-major (4 values), 84 values:
//   at 12 a + 4 k (a = 0..5, k = 0..2): block (a, (a + k) mod 6);
//   at 72 + 4 a   (a = 0..2):           block (a, a + 3).
// Row pair t then finds blocks (t, t), (t, t+1), (t, t+2) side by side and
// the other three as transposes (or, for t < 3, block (t, t+3) itself).
// Entry (2a, 2a+1) of a 2x2 diagonal block is also stored as (2a+1, 2a),
// with the same value.  A diagonal node block keeps this layout in the
// first 84 values of its 144-value place in the matrix.
constexpr int SYM12_VALS = 84;

// position of entry (r, c), either triangle
__host__ __device__ constexpr int sym12_pos(int r, int c) {
    const int a = r >> 1, i = r & 1, b = c >> 1, j = c & 1;
    const int d = (b - a + 6) % 6;
    return d <= 2 ? 12 * a + 4 * d + 2 * i + j
           : d >= 4 ? 12 * b + 4 * (6 - d) + 2 * j + i
                    : (a < 3 ? 72 + 4 * a + 2 * i + j : 72 + 4 * b + 2 * j + i);
}

// the entry (r, c) that position p holds, in the orientation the layout
// lists its 2x2 block (for p = 12a + 2 the upper one, (2a, 2a+1))
__host__ __device__ constexpr int sym12_row(int p) {
    return p < 72 ? ((p % 12) == 2 ? 2 * (p / 12) : 2 * (p / 12) + ((p >> 1) & 1)) : 2 * ((p - 72) >> 2) + ((p >> 1) & 1);
}
__host__ __device__ constexpr int sym12_col(int p) {
    return p < 72 ? ((p % 12) == 2 ? 2 * (p / 12) + 1 : 2 * ((p / 12 + (p % 12) / 4) % 6) + (p & 1))
                  : 2 * (((p - 72) >> 2) + 3) + (p & 1);
}
static_assert(sym12_pos(sym12_row(2), sym12_col(2)) == 1 && sym12_pos(11, 0) == 12 * 5 + 4 + 2 &&
                  sym12_pos(0, 11) == 12 * 5 + 4 + 2 && sym12_pos(7, 1) == 72 + 3,
              "packed symmetric layout");

template <class TV>
void launch_bj_factor(hipStream_t st, int nnodes, const int* diag_blk, const void* vals, int vals_fp32,
                      const uint16_t* freemask, const int* node_shell, TV* dinv, int* fail_shell);

void launch_save_diag(hipStream_t st, int nnodes, const int* diag_blk, const void* vals, int vals_fp32, double* diag);
void launch_regularize(hipStream_t st, int nnodes, const int* diag_blk, void* vals, int vals_fp32,
                       const double* diag, const int* node_shell, const double* delta_shell);

// Persistent block-Jacobi CG (single-reduction form); nthreads is 256, 512
// or 1024 per block.  x, r, u, p, s, w: [nnodes][12] work vectors (x the
// solution); nbflag: [nblk][32] neighbour-sync flags, zeroed before launch.
template <class TM, class TV>
hipError_t launch_cg(hipStream_t st, int nblk, int nthreads, const RowBlocks& rb, const SymBsr& m, const TM* vals,
                     const TV* dinv, const uint16_t* freemask, const double* b, TV* x, TV* r, TV* u, TV* p, TV* s,
                     TV* w, TV* slot, double* partial /* [2][nblk][4] */, void* sync, unsigned* nbflag,
                     int* abort_flag, const double* rtol2_shell, const int* maxit_shell, const int* active_shell,
                     CgShellOut* out, unsigned long long* trace /* NULL, or [nblk][CG_TRACE_ITERS][6] */);
// Phase timestamps of the CG (shell_cg_trace_*): per block and iteration,
// the constant 100 MHz clock at the iteration's start, the end of the update
// phase, the end of the neighbour wait, the end of thread 0's product
// phase, the block's arrival at the reduce-barrier (all its wavefronts done,
// partials published) and the barrier's exit.
constexpr int CG_TRACE_ITERS = 64;
int cg_max_blocks(int device, int tm_fp32, int nthreads);   // co-resident blocks of the CG kernel
size_t cg_sync_bytes();                                     // per-shell synchronisation state of the CG kernel
int cg_rows_per_pass(int tm_fp32, int nthreads);            // node rows one CG block covers per pass

// per-shell reductions over node rows (masked = free DOFs only):
// out[s] = sum x.y over shell s (y = x for norms)
void launch_shell_dot(hipStream_t st, const RowBlocks& rb, int nshell, const double* x, const double* y,
                      const uint16_t* freemask, double* partial, double* out);

// elementwise helpers
// qhat = q_n + dt v_n combined with q_n for mass-proportional damping:
// (qhat + a q_n)/(1 + a), a = alpha dt of the node's shell; q = qhat on free
// DOFs, the prescribed value (q_n if NULL) on the others
void launch_predict(hipStream_t st, int n, const double* qn, const double* vn, const double* qpresc,
                    const uint16_t* freemask, const int* node_shell, const ShellParams* shells, double dt,
                    double* qhat, double* q);
// external nodal forces: grad -= f on free DOFs (rows of shells with
// write_shell set, all if NULL) and e_shell[3s + 2] -= sum f.(q - qhat)
void launch_nodal_load(hipStream_t st, const RowBlocks& rb, int nshell, const double* f, const double* q,
                       const double* qhat, const uint16_t* freemask, const int* node_shell, const int* write_shell,
                       double* grad, double* part, double* e_shell);
void launch_axpy_shell(hipStream_t st, int nnodes, const double* x, const double* d, const double* alpha_shell,
                       const int* node_shell, double* out);
void launch_neg_masked(hipStream_t st, int nnodes, const double* g, const uint16_t* freemask,
                       const int* node_shell, const int* active_shell, double* b);
void launch_velocity(hipStream_t st, int n, const double* q1, const double* qn, double dt, double* v);
void launch_copy_shell(hipStream_t st, int nnodes, const double* src, const int* node_shell, const int* flag_shell,
                       double* dst);
// both copies of launch_copy_shell in one launch
void launch_copy_shell2(hipStream_t st, int nnodes, const double* src0, const double* src1, const int* node_shell,
                        const int* flag_shell, double* dst0, double* dst1);
template <class TV>
void launch_add_to(hipStream_t st, int n, const TV* dx, double* x);
void launch_cast_to_float(hipStream_t st, int n, const double* x, float* y);
// zero `bytes` (a multiple of 4, 16-byte aligned start) with a kernel
void launch_zero(hipStream_t st, void* p, size_t bytes);
// three buffers in one launch (each 16-byte aligned, sizes multiples of 4 bytes)
void launch_zero3(hipStream_t st, void* p0, size_t b0, void* p1, size_t b1, void* p2, size_t b2);
void launch_add_shell(hipStream_t st, int nnodes, const double* src, const int* node_shell, const int* flag_shell,
                      double* dst);

// --------------------------------------------------- warm-start network
constexpr int MLP_IN = 60, MLP_H = 128, MLP_OUT = 12;
constexpr int MLP_NPARAMS = MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H * MLP_OUT + MLP_OUT;
int mlp_bf16_elems();
size_t mlp_train_work_bytes(int batch);
void launch_mlp_pack(hipStream_t st, const float* theta, void* w_bf16);
void launch_mlp_forward(hipStream_t st, const float* theta, const void* w, const float* feat, float* out, long long n);
// loss (atomically added, mean over the batch) and gradient (atomically added) of one mini-batch
void launch_mlp_grad(hipStream_t st, const float* theta, const void* w, const float* feat, const float* tgt,
                     const long long* idx, int batch, void* work, float* grad, double* loss);
void launch_mlp_adam(hipStream_t st, float* theta, const float* g, float* m, float* v, int n, float lr, int step);
void launch_sample_idx(hipStream_t st, long long n, int batch, unsigned long long seed, long long* idx);
// per-shell, per-kind RMS scales of u = q - qbar, b, dprev: scale[s*12 + 4*quantity + kind]
void launch_feat_scale(hipStream_t st, const RowBlocks& rb, int nshell, const double* q, const double* qbar,
                       const double* b, const double* dprev, const uint16_t* fm, double* part, const int* cnt_kind,
                       float* scale);
void launch_mlp_record(hipStream_t st, int nshell, int K, unsigned long long seed, const ShellParams* shells,
                       const long long* sbase, const double* q, const double* qbar, const double* b,
                       const double* dprev, const double* d, const int* nbr8 /* [N][8] */, const float* scale,
                       float* feat_out, float* tgt_out);
void launch_mlp_guess(hipStream_t st, int nnodes, const float* theta, const void* w, const int* node_shell,
                      const int* flag, const double* q, const double* qbar, const double* b, const double* dprev,
                      const uint16_t* fm, const int* nbr8, const float* scale, double* corr);
void launch_axpy2_shell(hipStream_t st, int nnodes, const double* x, const double* d1, const double* d2,
                        const double* coef, const int* node_shell, double* y);
void launch_masked_diff(hipStream_t st, int nnodes, const double* a, const double* b, const uint16_t* fm,
                        const int* node_shell, const int* flag, double* out);

}  // namespace bhem
