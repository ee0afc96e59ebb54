// Host side of libbhem: context creation (grid layout, colouring, block
// sparsity pattern, device buffers), the C ABI of include/bhem_shell.h and
// the implicit-Euler Newton driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bhem_shell.h"
#include "device_common.hpp"
#include "kernels.hpp"

using namespace bhem;

namespace {

thread_local std::string g_create_error;

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

template <class T> T* dptr(DevBuf& b) { return static_cast<T*>(b.p); }

struct HostStats {
    double t_assemble = 0, t_pcg = 0;
};

}  // namespace

struct shell_ctx {
    shell_opts opts;
    hipStream_t stream = nullptr;
    std::string err;
    int S = 0, N = 0, P = 0;
    long long nnzb = 0;     // block non-zeros of the full matrix
    long long nnzb_u = 0;   // stored blocks (diagonal and upper triangle)
    bool fp32 = false;
    std::vector<ShellParams> shells;
    std::vector<int> h_row_ptr, h_col_idx, h_node_shell;   // full block pattern
    std::vector<int> h_urow, h_ucol;                       // stored (upper) pattern
    std::vector<uint16_t> h_freemask;
    std::vector<int> colour_off;   // [ncolour + 1] into the concatenated colour lists
    int nblk = 0;                  // CG row blocks
    int cg_max_rows = 0;           // node rows of the largest CG block
    int cg_threads = 256;          // threads per CG block
    int cg_rows_target = 0;        // node rows per CG block (before the even split of a shell)
    std::vector<int> h_shell_blk0, h_shell_nblk;
    // device data
    DevBuf patch_first;   // [P] uint16 first-touch bits of the stored local blocks
    DevBuf patch_kid;     // [P] uint64 local block index of each stored local block (4 bits each)
    // single-launch assembly (asm_gather): the patches' stored local blocks
    // in scratch [P][10][144], and per stored block the scratch entries to
    // sum, in colour order, and whether it is a diagonal block
    bool asm_gather = false, asm_eligible = false;
    DevBuf asm_scr, asm_cptr, asm_cidx, asm_diag;
    DevBuf shells_d, phi, qbar, freemask, node_shell, patch_nodes, patch_shell, patch_slots, colour_list, inc_ptr,
        inc, row_ptr, col_idx, tslot, lptr, diag_blk, vals, slot, diag0, dinv;
    DevBuf blk_shell, blk_row0, blk_row1, shell_blk0, shell_nblk, blk_nbhi, cg_nbflag;
    DevBuf e_patch, g_patch, e_shell, red_part, red_out;
    // Newton / CG work vectors (FP64 [N*12] unless noted)
    DevBuf qhat, q, qt, g, gt, dvec, rhs, cg_x, cg_r, cg_z, cg_p0, cg_p1, cg_q, r64, x64;
    DevBuf cg_partial, cg_bar, cg_abort, cg_rtol2, cg_maxit, cg_active, cg_out, fail_shell, delta_shell, alpha_shell,
        flag_shell, write_shell, nt_ctl;
    // pinned host mirrors
    double* h_e_shell = nullptr;   // [S*3]
    double* h_red = nullptr;       // [S]
    CgShellOut* h_cg_out = nullptr;
    int* h_fail = nullptr;
    NewtonCtl* h_ctl = nullptr;    // [S] per-shell state of the device-driven Newton iteration
    char* h_stage = nullptr;       // staging of control uploads
    size_t stage_cap = 0, stage_off = 0;
    // warm-start network: FP32 master weights, bf16 operand copies, Adam state
    bool mlp_ready = false;
    int adam_step = 0;
    DevBuf mlp_theta, mlp_w, mlp_m, mlp_v, mlp_grad, mlp_loss, mlp_idx, mlp_work, feat_part, feat_scale, cnt_kind,
        dstep, qstart, b0, guess, rec_base;
    DevBuf nbr8;   // [N][8] grid neighbours of each node (the node itself where there is none)
    DevBuf cg_trace;   // [nblk][CG_TRACE_ITERS][6] phase timestamps of the last CG launch, when tracing
    std::vector<char> h_hist;   // per shell: dstep holds the last step's correction
    int mlp_work_batch = 0;
    long long mlp_loss_n = 0;
    unsigned long long rec_calls = 0;
    // recording of (features, target) samples during Newton solves
    float* rec_feat = nullptr;
    float* rec_tgt = nullptr;
    long long rec_cap = 0, rec_count = 0;
    int rec_K = 0;
    unsigned long long rec_seed = 0;
    // HIP graphs of the Newton iteration's fixed launch sequences, captured
    // on a private stream and replayed on the context's stream
    struct Seg {
        hipGraphExec_t exec = nullptr;
        double key = 0.0;
    };
    bool graphs = true;
    bool cg_resident = true;   // register-resident CG vectors where the layout allows
    bool cg_tracing = false;   // the CG records its phase timestamps (shell_cg_trace_enable)
    int hs_waves = 4;          // patches (wavefronts) per block of the Hessian kernel
    int eg_patches = 16;       // patches per block of the energy and gradient kernel
    hipStream_t cap_stream = nullptr;
    Seg g_asm, g_trial, g_floor, g_cg, g_newton;
    void graphs_reset() {
        for (Seg* g : {&g_asm, &g_trial, &g_floor, &g_cg, &g_newton}) {
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
            g->exec = nullptr;
        }
    }
    // damping enters the inertia term of Newton steps only: dt there, 0 otherwise
    double dt_damp = 0.0;
    // collision handling (shell_collide): per-sample times, block minima,
    // contact lists and constraint work arrays, sized on first use
    DevBuf coll_tc, coll_cid, coll_blk, coll_cnt, coll_list, coll_cols, coll_con, coll_incp, coll_inc, coll_rowof,
        coll_lam, coll_out;
    // external nodal forces (shell_set_nodal_forces)
    DevBuf fext;
    bool has_fext = false;
    // pressure per shell (shell_set_pressure): a load evaluated at each
    // step's start, added to fext into fstep for that step
    DevBuf pressure, fstep;
    bool has_pressure = false, use_fstep = false;
    // point constraints (shell_set_point_constraints), sorted by shell:
    // alm_order[j] is the caller's index of the j-th, alm_shell_pt [S + 1]
    // their ranges; h_lam the multipliers [3 alm_n]; the penalty's matrix
    // kappa C^T C merged into alm_nsp values at positions of vals
    int alm_n = 0, alm_max_outer = 0, alm_nsp = 0;
    double alm_kappa = 0.0, alm_tol = 0.0;
    bool alm_on = false;   // set within shell_newton_step
    std::vector<int> alm_order, alm_shell_pt;
    std::vector<double> h_lam;
    DevBuf alm_pts, alm_lam, alm_incp, alm_inc, alm_spt, alm_pos, alm_val, alm_c;
    std::vector<int> grid_n1, grid_n2, grid_per;   // per shell
    const double* load_vec() { return use_fstep ? dptr<double>(fstep) : dptr<double>(fext); }
    bool has_load() const { return use_fstep || has_fext; }
    // event timing
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    shell_timing tm;
    std::vector<long long> rows_s, nnzb_s;   // per-shell node rows and stored blocks

    SymBsr sym() {
        return SymBsr{dptr<int>(row_ptr), dptr<int>(col_idx), dptr<int>(tslot), dptr<int>(lptr)};
    }

    RowBlocks rb() {
        return RowBlocks{nblk, cg_resident ? cg_max_rows : INT32_MAX, dptr<int>(blk_shell), dptr<int>(blk_row0),
                         dptr<int>(blk_row1), dptr<int>(shell_blk0), dptr<int>(shell_nblk), dptr<int>(blk_nbhi)};
    }
    ~shell_ctx() {
        graphs_reset();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (h_e_shell) (void)hipHostFree(h_e_shell);
        if (h_red) (void)hipHostFree(h_red);
        if (h_cg_out) (void)hipHostFree(h_cg_out);
        if (h_fail) (void)hipHostFree(h_fail);
        if (h_ctl) (void)hipHostFree(h_ctl);
        if (h_stage) (void)hipHostFree(h_stage);
    }
};

namespace {

struct HipErr {
    hipError_t e;
    const char* what;
};

#define HIPCHK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) throw HipErr{e_, #call};                                            \
    } while (0)

struct InvalErr {
    std::string msg;
};
struct StatusErr {
    shell_status st;
    std::string msg;
};

void alloc(DevBuf& b, size_t bytes) {
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
    }
    b.n = bytes;
    if (bytes == 0) return;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) throw StatusErr{SHELL_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
}

template <class T> void upload(DevBuf& b, const std::vector<T>& v, hipStream_t st) {
    alloc(b, v.size() * sizeof(T));
    if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

void sync(shell_ctx* c) {
    HIPCHK(hipStreamSynchronize(c->stream));
    c->stage_off = 0;
}

// Small host-to-device copy of control data, stream-ordered.  The bytes go
// through the pinned staging area first (so the caller's host array may go
// out of scope at once); the area is reused only after the stream has been
// synchronised, which is forced here when it is full.
void h2d(shell_ctx* c, void* dst, const void* src, size_t bytes) {
    const size_t need = (bytes + 15) & ~(size_t)15;
    if (need > c->stage_cap) {   // larger than the staging area: plain synchronous copy
        HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
        sync(c);
        return;
    }
    if (c->stage_off + need > c->stage_cap) sync(c);
    char* h = c->h_stage + c->stage_off;
    std::memcpy(h, src, bytes);
    c->stage_off += need;
    HIPCHK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, c->stream));
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Event timer of one kernel group (no-op unless timing is on).
struct GroupTimer {
    shell_ctx* c;
    int group;
    GroupTimer(shell_ctx* c_, int g) : c(c_), group(g) {
        if (c->timing) HIPCHK(hipEventRecord(c->ev0, c->stream));
    }
    void stop() {
        if (!c->timing) return;
        HIPCHK(hipEventRecord(c->ev1, c->stream));
        HIPCHK(hipEventSynchronize(c->ev1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        c->tm.ms[group] += ms;
        c->tm.launches[group] += 1;
    }
};

// Run `body`, which enqueues work on c->stream only (no synchronisation,
// no memset), directly or as a HIP graph captured once per key and then
// replayed.  Graphs are off while event timing is on.
template <class F> void run_graph(shell_ctx* c, shell_ctx::Seg& seg, double key, F&& body) {
    if (!c->graphs || c->timing) {
        body();
        return;
    }
    if (!seg.exec || seg.key != key) {
        if (seg.exec) {
            (void)hipGraphExecDestroy(seg.exec);
            seg.exec = nullptr;
        }
        if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t user = c->stream;
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        c->stream = c->cap_stream;
        try {
            body();
        } catch (...) {
            c->stream = user;
            (void)hipStreamEndCapture(c->cap_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        c->stream = user;
        HIPCHK(hipStreamEndCapture(c->cap_stream, &g));
        const hipError_t e = hipGraphInstantiate(&seg.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
        seg.key = key;
    }
    HIPCHK(hipGraphLaunch(seg.exec, c->stream));
}

// ----------------------------------------------------------- layout
int node_cols(const shell_desc& d) { return d.periodic1 ? d.n1 : d.n1 + 1; }
int node_count(const shell_desc& d) { return node_cols(d) * (d.n2 + 1); }

void validate(const shell_desc& d, int s) {
    auto bad = [&](const std::string& m) { throw InvalErr{"shell " + std::to_string(s) + ": " + m}; };
    if (d.n1 < 1 || d.n2 < 1) bad("n1 and n2 must be >= 1");
    if (d.periodic1 && d.n1 < 3) bad("a periodic shell needs n1 >= 3");
    if (!(d.dxi1 > 0) || !(d.dxi2 > 0)) bad("dxi1 and dxi2 must be > 0");
    if (!d.ref_host) bad("ref_host is NULL");
    if (!(d.young > 0) || !(d.poisson >= 0 && d.poisson < 0.5)) bad("need young > 0 and 0 <= poisson < 0.5");
    if (!(d.thickness > 0) || !(d.density > 0)) bad("thickness and density must be > 0");
    if ((long long)d.n1 * d.n2 > (1 << 26)) bad("grid too large");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(d.gravity[k])) bad("gravity not finite");
    if (!(d.damping >= 0) || !std::isfinite(d.damping)) bad("damping must be finite and >= 0");
    const int nn = node_count(d);
    for (long long i = 0; i < 12LL * nn; ++i)
        if (!std::isfinite(d.ref_host[i])) bad("reference coordinates not finite");
}

// CG row blocks for `nt` threads per block.  spread >= 1: rows per block a
// multiple of the rows one pass of the block covers, at least `spread` x
// the fewest that fit all blocks on the device at once; spread = 0: the
// fewest rows per block that fit (every co-resident slot used, the last
// pass of a block partly idle); spread = -1: one block per shell (the CG of
// a shell of one block needs no grid barrier).  Uploads the layout and sizes
// the per-block buffers.  False if the shells do not fit (more shells than
// co-resident blocks).
bool set_row_blocks(shell_ctx* c, int nt, int spread) {
    const int S = c->S, N = c->N;
    const int cap = cg_max_blocks(c->opts.device, c->fp32, nt);
    if (cap <= 0) throw StatusErr{SHELL_E_DEVICE, "cannot query CG kernel occupancy"};
    if (S > cap) return false;
    const int pass = spread >= 1 ? cg_rows_per_pass(c->fp32, nt) : 1;   // granularity of the rows per block
    int target = std::max(pass, (N + cap - 1) / cap);
    target = ((target + pass - 1) / pass) * pass;
    int used = 0;
    if (spread < 0) {
        target = 1;
        for (int s = 0; s < S; ++s) target = std::max(target, c->shells[s].node_end - c->shells[s].node_begin);
    } else {
        for (;; target += pass) {   // grow the rows per block until every block fits on the device at once
            used = 0;
            for (int s = 0; s < S; ++s)
                used += std::max(1, (c->shells[s].node_end - c->shells[s].node_begin + target - 1) / target);
            if (used <= cap) break;
        }
        target *= std::max(1, spread);
    }
    std::vector<int> bshell, brow0, brow1;
    c->h_shell_blk0.assign(S, 0);
    c->h_shell_nblk.assign(S, 0);
    used = 0;
    for (int s = 0; s < S; ++s) {
        const int r0 = c->shells[s].node_begin, r1 = c->shells[s].node_end;
        int nb = std::max(1, (r1 - r0 + target - 1) / target);
        c->h_shell_blk0[s] = used;
        c->h_shell_nblk[s] = nb;
        for (int k = 0; k < nb; ++k) {
            bshell.push_back(s);
            brow0.push_back(r0 + (int)((long long)(r1 - r0) * k / nb));
            brow1.push_back(r0 + (int)((long long)(r1 - r0) * (k + 1) / nb));
        }
        used += nb;
    }
    // per block, the last block whose rows its stored (upper-triangle)
    // blocks reach: the CG's neighbour sync waits for blocks k+1 .. nbhi[k]
    std::vector<int> nbhi(used);
    {
        std::vector<int> row_blk(N);
        for (int k = 0; k < used; ++k)
            for (int rr = brow0[k]; rr < brow1[k]; ++rr) row_blk[rr] = k;
        for (int k = 0; k < used; ++k) {
            int hi = k;
            for (int rr = brow0[k]; rr < brow1[k]; ++rr)
                for (int e = c->h_row_ptr[rr]; e < c->h_row_ptr[rr + 1]; ++e)
                    hi = std::max(hi, row_blk[c->h_col_idx[e]]);
            nbhi[k] = hi;
        }
    }
    hipStream_t st = c->stream;
    c->nblk = used;
    c->cg_max_rows = 0;
    for (int k = 0; k < used; ++k) c->cg_max_rows = std::max(c->cg_max_rows, brow1[k] - brow0[k]);
    c->cg_threads = nt;
    c->cg_rows_target = target;
    upload(c->blk_shell, bshell, st);
    upload(c->blk_row0, brow0, st);
    upload(c->blk_row1, brow1, st);
    upload(c->shell_blk0, c->h_shell_blk0, st);
    upload(c->shell_nblk, c->h_shell_nblk, st);
    upload(c->blk_nbhi, nbhi, st);
    alloc(c->cg_nbflag, (size_t)c->nblk * 32 * sizeof(unsigned));
    alloc(c->red_part, (size_t)c->nblk * sizeof(double));
    alloc(c->cg_partial, (size_t)c->nblk * 8 * sizeof(double));   // [2][nblk][4]: by barrier parity
    alloc(c->feat_part, (size_t)c->nblk * 12 * sizeof(double));
    if (c->cg_tracing) alloc(c->cg_trace, (size_t)c->nblk * CG_TRACE_ITERS * 6 * sizeof(unsigned long long));
    sync(c);
    c->graphs_reset();
    return true;
}

void build(shell_ctx* c, const shell_desc* ds, int S) {
    hipStream_t st = c->stream;
    c->S = S;
    c->stage_cap = std::max<size_t>(256 * 1024, (size_t)S * 64 * 16);
    HIPCHK(hipHostMalloc((void**)&c->h_stage, c->stage_cap, 0));
    // node and patch ranges
    int N = 0, P = 0;
    c->shells.resize(S);
    for (int s = 0; s < S; ++s) {
        const shell_desc& d = ds[s];
        ShellParams& sp = c->shells[s];
        sp.dxi1 = d.dxi1;
        sp.dxi2 = d.dxi2;
        sp.lam = d.young * d.poisson / (1.0 - d.poisson * d.poisson);
        sp.mu = d.young / (2.0 * (1.0 + d.poisson));
        sp.h = d.thickness;
        sp.rho_h = d.density * d.thickness;
        for (int k = 0; k < 3; ++k) sp.grav[k] = d.gravity[k];
        sp.damp = d.damping;
        sp.node_begin = N;
        N += node_count(d);
        sp.node_end = N;
        sp.patch_begin = P;
        P += d.n1 * d.n2;
        sp.patch_end = P;
        c->grid_n1.push_back(d.n1);
        c->grid_n2.push_back(d.n2);
        c->grid_per.push_back(d.periodic1 ? 1 : 0);
    }
    c->N = N;
    c->P = P;
    // per-node data
    std::vector<double> qbar((size_t)N * 12);
    c->h_freemask.assign(N, 0);
    c->h_node_shell.assign(N, 0);
    for (int s = 0; s < S; ++s) {
        const shell_desc& d = ds[s];
        const int nb = c->shells[s].node_begin, nn = node_count(d);
        std::memcpy(&qbar[(size_t)nb * 12], d.ref_host, sizeof(double) * 12 * nn);
        for (int i = 0; i < nn; ++i) {
            uint16_t m = 0;
            for (int w = 0; w < 12; ++w)
                if (!d.fixed_host || !d.fixed_host[12 * i + w]) m |= (uint16_t)(1u << w);
            c->h_freemask[nb + i] = m;
            c->h_node_shell[nb + i] = s;
        }
    }
    // the 3x3 grid neighbours of every node, row by row: (-1,-1), (0,-1),
    // (1,-1), (-1,0), (1,0), (-1,1), (0,1), (1,1); across a periodic seam
    // the column wraps, past an open edge the node stands for itself
    {
        std::vector<int> nbr((size_t)N * 8);
        for (int s = 0; s < S; ++s) {
            const shell_desc& d = ds[s];
            const int cols = node_cols(d), nb = c->shells[s].node_begin;
            for (int j = 0; j <= d.n2; ++j)
                for (int i = 0; i < cols; ++i) {
                    const int self = nb + j * cols + i;
                    int k = 0;
                    for (int dj = -1; dj <= 1; ++dj)
                        for (int di = -1; di <= 1; ++di) {
                            if (di == 0 && dj == 0) continue;
                            int ii = i + di;
                            const int jj = j + dj;
                            if (d.periodic1) ii = (ii + cols) % cols;
                            const bool in = ii >= 0 && ii < cols && jj >= 0 && jj <= d.n2;
                            nbr[(size_t)self * 8 + k++] = in ? nb + jj * cols + ii : self;
                        }
                }
        }
        upload(c->nbr8, nbr, st);
        sync(c);   // the host vector is released at the end of this scope
    }
    // patches, colours, pattern
    std::vector<int4> pnodes(P);
    std::vector<int> pshell(P);
    std::vector<std::vector<int>> colour_lists(6);
    std::vector<std::vector<int>> adj(N);
    for (int s = 0; s < S; ++s) {
        const shell_desc& d = ds[s];
        const int cols = node_cols(d), nb = c->shells[s].node_begin;
        for (int pj = 0; pj < d.n2; ++pj)
            for (int pi = 0; pi < d.n1; ++pi) {
                const int p = c->shells[s].patch_begin + pj * d.n1 + pi;
                int nd[4];
                for (int cc = 0; cc < 4; ++cc) {
                    int i = pi + (cc & 1), j = pj + (cc >> 1);
                    if (d.periodic1) i %= d.n1;
                    nd[cc] = nb + j * cols + i;
                }
                pnodes[p] = make_int4(nd[0], nd[1], nd[2], nd[3]);
                pshell[p] = s;
                // colours: patches of one colour share no node.  Along a
                // periodic direction with odd n1 the last column gets a third colour.
                int cx = pi & 1;
                if (d.periodic1 && (d.n1 & 1) && pi == d.n1 - 1) cx = 2;
                colour_lists[cx + 3 * (pj & 1)].push_back(p);
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) adj[nd[a]].push_back(nd[b]);
            }
    }
    // verify the colouring: no node touched twice within a colour
    {
        std::vector<int> seen(N, -1);
        for (int col = 0; col < 6; ++col)
            for (int p : colour_lists[col]) {
                const int nd[4] = {pnodes[p].x, pnodes[p].y, pnodes[p].z, pnodes[p].w};
                for (int a = 0; a < 4; ++a) {
                    if (seen[nd[a]] == col) throw InvalErr{"internal: patch colouring conflict"};
                    seen[nd[a]] = col;
                }
            }
    }
    c->h_row_ptr.assign(N + 1, 0);
    c->h_col_idx.clear();
    for (int n = 0; n < N; ++n) {
        auto& a = adj[n];
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
        c->h_col_idx.insert(c->h_col_idx.end(), a.begin(), a.end());
        c->h_row_ptr[n + 1] = (int)c->h_col_idx.size();
    }
    c->nnzb = (long long)c->h_col_idx.size();
    // stored pattern: the columns >= n of block row n (the diagonal first);
    // the transposed product of stored block (i, j > i) goes to the slots of
    // row j, ordered by i
    c->h_urow.assign(N + 1, 0);
    c->h_ucol.clear();
    std::vector<int> diag(N), lptr(N + 1, 0);
    for (int n = 0; n < N; ++n) {
        for (int k = c->h_row_ptr[n]; k < c->h_row_ptr[n + 1]; ++k) {
            const int col = c->h_col_idx[k];
            if (col >= n) c->h_ucol.push_back(col);
            else lptr[n + 1]++;
        }
        c->h_urow[n + 1] = (int)c->h_ucol.size();
        if (c->h_urow[n + 1] == c->h_urow[n] || c->h_ucol[c->h_urow[n]] != n)
            throw InvalErr{"internal: block row without its diagonal block"};
        diag[n] = c->h_urow[n];
    }
    for (int n = 0; n < N; ++n) lptr[n + 1] += lptr[n];
    c->nnzb_u = (long long)c->h_ucol.size();
    std::vector<int> tslot((size_t)c->nnzb_u, -1);
    {
        std::vector<int> fill(lptr.begin(), lptr.end() - 1);
        for (int n = 0; n < N; ++n)
            for (int b = c->h_urow[n] + 1; b < c->h_urow[n + 1]; ++b) tslot[b] = fill[c->h_ucol[b]]++;
        for (int n = 0; n < N; ++n)
            if (fill[n] != lptr[n + 1]) throw InvalErr{"internal: asymmetric block pattern"};
    }
    c->rows_s.assign(S, 0);
    c->nnzb_s.assign(S, 0);
    for (int s2 = 0; s2 < S; ++s2) {
        c->rows_s[s2] = c->shells[s2].node_end - c->shells[s2].node_begin;
        c->nnzb_s[s2] = c->h_urow[c->shells[s2].node_end] - c->h_urow[c->shells[s2].node_begin];
    }
    // per patch: the stored local blocks (a, b) -- the 4 diagonal ones
    // first, then those whose row node index is above the column node's
    // (that block, column-major, is the stored pair's content) -- with their
    // stored block index
    std::vector<int> slots((size_t)P * 16, -1);
    std::vector<uint64_t> kid((size_t)P, 0);
    std::vector<std::vector<int>> inc(N);
    for (int p = 0; p < P; ++p) {
        const int nd[4] = {pnodes[p].x, pnodes[p].y, pnodes[p].z, pnodes[p].w};
        for (int a = 0; a < 4; ++a) inc[nd[a]].push_back(4 * p + a);
        int mm = 0;
        for (int pass = 0; pass < 2; ++pass)   // diagonal blocks, then the others
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    if (a != b && nd[a] == nd[b]) throw InvalErr{"internal: patch with a repeated node"};
                    if (pass == 0 ? a != b : !(nd[a] > nd[b])) continue;
                    const int lo = std::min(nd[a], nd[b]), hi = std::max(nd[a], nd[b]);
                    const int* beg = &c->h_ucol[c->h_urow[lo]];
                    const int* end = &c->h_ucol[0] + c->h_urow[lo + 1];
                    const int* at = std::lower_bound(beg, end, hi);
                    if (at == end || *at != hi) throw InvalErr{"internal: patch block missing from the pattern"};
                    slots[(size_t)p * 16 + mm] = (int)(at - &c->h_ucol[0]);
                    kid[p] |= (uint64_t)(4 * a + b) << (4 * mm);
                    ++mm;
                }
    }
    std::vector<int> inc_ptr(N + 1, 0), inc_flat;
    for (int n = 0; n < N; ++n) {
        inc_flat.insert(inc_flat.end(), inc[n].begin(), inc[n].end());
        inc_ptr[n + 1] = (int)inc_flat.size();
    }
    std::vector<int> clist;
    c->colour_off.assign(1, 0);
    for (int col = 0; col < 6; ++col) {
        clist.insert(clist.end(), colour_lists[col].begin(), colour_lists[col].end());
        c->colour_off.push_back((int)clist.size());
    }
    // first touch: bit m of patch p is set when p is the first patch, in
    // colour-pass order, to add into its m-th stored local block (patches of
    // one colour never share a block), so the assembly stores instead of
    // adding there and needs no zero fill
    std::vector<uint16_t> first((size_t)P, 0);
    {
        std::vector<char> touched((size_t)c->nnzb_u, 0);
        for (int p : clist)
            for (int m = 0; m < 16; ++m) {
                const int sl = slots[(size_t)p * 16 + m];
                if (sl < 0) break;
                if (!touched[sl]) {
                    touched[sl] = 1;
                    first[p] |= (uint16_t)(1u << m);
                }
            }
        for (long long k = 0; k < c->nnzb_u; ++k)
            if (!touched[k]) throw InvalErr{"internal: matrix block without a patch"};
    }
    // CG row blocks: contiguous node rows, never straddling a shell.  Large
    // shells use big blocks (fewer blocks make the per-iteration barriers
    // cheaper): 1024 threads with FP32 matrices, 512 with FP64 ones (one
    // such block per CU leaves each wave the registers of the symmetric
    // product without spilling); small shells 256-thread blocks spread over
    // more CUs.
    int max_rows = 0;
    for (int s = 0; s < S; ++s) max_rows = std::max(max_rows, c->shells[s].node_end - c->shells[s].node_begin);
    const int big = c->fp32 ? 1024 : 512;
    const int nt0 = max_rows >= 16 * cg_rows_per_pass(c->fp32, big) ? big : 256;
    if (!set_row_blocks(c, nt0, 1) && !set_row_blocks(c, 256, 1))
        throw InvalErr{"too many shells for one context (limit " +
                       std::to_string(cg_max_blocks(c->opts.device, c->fp32, 256)) + ")"};
    // theta-space basis table Phi_g[a][I] at 96 g + 16 a + I, followed by
    // three copies ordered for the lanes that read them: its transpose at
    // 1536 + 16 (16 a + I) + g (consecutive lanes take consecutive Gauss
    // points), at 3072 + 32 (8 a + I / 2) + 2 g + I % 2 (pairs of basis
    // functions per Gauss point) and at 4608 + 32 (3 g + a / 2) + 2 I + a % 2
    // (pairs of slots per basis function)
    std::vector<double> phi(4 * 16 * 6 * 16);
    build_theta_basis(phi.data());
    for (int g = 0; g < 16; ++g)
        for (int a = 0; a < 6; ++a)
            for (int I = 0; I < 16; ++I) {
                const double v = phi[96 * g + 16 * a + I];
                phi[1536 + 16 * (16 * a + I) + g] = v;
                phi[3072 + 32 * (8 * a + I / 2) + 2 * g + I % 2] = v;
                phi[4608 + 32 * (3 * g + a / 2) + 2 * I + a % 2] = v;
            }
    // uploads
    upload(c->shells_d, c->shells, st);
    upload(c->phi, phi, st);
    upload(c->qbar, qbar, st);
    upload(c->freemask, c->h_freemask, st);
    upload(c->node_shell, c->h_node_shell, st);
    upload(c->patch_nodes, pnodes, st);
    upload(c->patch_shell, pshell, st);
    upload(c->patch_slots, slots, st);
    upload(c->patch_kid, kid, st);
    upload(c->colour_list, clist, st);
    // Where every patch's Hessian block is resident at once, one launch over
    // all patches writes the local blocks to scratch and a second sums each
    // stored block's contributions in colour order (the same additions as
    // the colour launches, so the same bits) instead of one launch per
    // colour, each a full round of block latency.
    {
        const int cap = hessian_resident_patches(c->opts.device, c->fp32);
        c->asm_eligible = c->asm_gather = P > 0 && cap > 0 && P <= cap;
        if (c->asm_gather) {
            std::vector<int> cnt((size_t)c->nnzb_u + 1, 0);
            std::vector<uint8_t> dg((size_t)c->nnzb_u, 0);
            for (int p : clist)
                for (int m = 0; m < 10; ++m) {
                    const int sl = slots[(size_t)p * 16 + m];
                    if (sl < 0) break;
                    cnt[sl + 1]++;
                    if (m < 4) dg[sl] = 1;
                }
            for (long long k = 0; k < c->nnzb_u; ++k) cnt[k + 1] += cnt[k];
            std::vector<int> cidx(cnt[c->nnzb_u]), fill(cnt.begin(), cnt.end() - 1);
            for (int p : clist)
                for (int m = 0; m < 10; ++m) {
                    const int sl = slots[(size_t)p * 16 + m];
                    if (sl < 0) break;
                    cidx[fill[sl]++] = 10 * p + m;
                }
            upload(c->asm_cptr, cnt, st);
            upload(c->asm_cidx, cidx, st);
            upload(c->asm_diag, dg, st);
            alloc(c->asm_scr, (size_t)P * 10 * 144 * (c->fp32 ? sizeof(float) : sizeof(double)));
        }
    }
    upload(c->patch_first, first, st);
    upload(c->inc_ptr, inc_ptr, st);
    upload(c->inc, inc_flat, st);
    upload(c->row_ptr, c->h_urow, st);
    upload(c->col_idx, c->h_ucol, st);
    upload(c->tslot, tslot, st);
    upload(c->lptr, lptr, st);
    upload(c->diag_blk, diag, st);
    const size_t vecb = (size_t)N * 12 * sizeof(double);
    alloc(c->vals, (size_t)c->nnzb_u * 144 * (c->fp32 ? sizeof(float) : sizeof(double)));
    alloc(c->slot, (size_t)std::max(c->nnzb_u - N, 1LL) * 12 * sizeof(double));
    alloc(c->diag0, vecb);
    alloc(c->dinv, (size_t)N * SYM12_VALS * (c->fp32 ? sizeof(float) : sizeof(double)));
    alloc(c->e_patch, (size_t)std::max(P, 1) * 3 * sizeof(double));
    alloc(c->g_patch, (size_t)std::max(P, 1) * 48 * sizeof(double));
    alloc(c->e_shell, (size_t)S * 3 * sizeof(double));
    alloc(c->red_out, (size_t)S * sizeof(double));
    for (DevBuf* b : {&c->qhat, &c->q, &c->qt, &c->g, &c->gt, &c->dvec, &c->rhs, &c->r64, &c->x64}) alloc(*b, vecb);
    const size_t tvb = (size_t)N * 12 * (c->fp32 ? sizeof(float) : sizeof(double));
    for (DevBuf* b : {&c->cg_x, &c->cg_r, &c->cg_z, &c->cg_p0, &c->cg_p1, &c->cg_q}) alloc(*b, tvb);
    alloc(c->cg_bar, (size_t)S * cg_sync_bytes());
    alloc(c->cg_abort, sizeof(int));
    alloc(c->cg_rtol2, (size_t)S * sizeof(double));
    alloc(c->cg_maxit, (size_t)S * sizeof(int));
    alloc(c->cg_active, (size_t)S * sizeof(int));
    alloc(c->cg_out, (size_t)S * sizeof(CgShellOut));
    alloc(c->fail_shell, (size_t)S * sizeof(int));
    alloc(c->delta_shell, (size_t)S * sizeof(double));
    alloc(c->alpha_shell, (size_t)2 * S * sizeof(double));
    alloc(c->flag_shell, (size_t)S * sizeof(int));
    alloc(c->write_shell, (size_t)S * sizeof(int));
    for (DevBuf* b : {&c->dstep, &c->qstart, &c->b0, &c->guess}) alloc(*b, vecb);
    c->h_hist.assign(S, 0);
    alloc(c->rec_base, (size_t)S * sizeof(long long));
    alloc(c->feat_scale, (size_t)S * 12 * sizeof(float));
    {
        std::vector<int> cnt((size_t)S * 4, 0);
        for (int n = 0; n < N; ++n)
            for (int w = 0; w < 12; ++w)
                if ((c->h_freemask[n] >> w) & 1) cnt[4 * c->h_node_shell[n] + w / 3]++;
        upload(c->cnt_kind, cnt, st);
        sync(c);
    }
    HIPCHK(hipMemsetAsync(c->dstep.p, 0, c->dstep.n, st));
    HIPCHK(hipHostMalloc((void**)&c->h_e_shell, (size_t)S * 3 * sizeof(double), 0));
    HIPCHK(hipHostMalloc((void**)&c->h_red, (size_t)S * sizeof(double), 0));
    HIPCHK(hipHostMalloc((void**)&c->h_cg_out, (size_t)S * sizeof(CgShellOut), 0));
    HIPCHK(hipHostMalloc((void**)&c->h_fail, (size_t)S * sizeof(int), 0));
    HIPCHK(hipHostMalloc((void**)&c->h_ctl, (size_t)S * sizeof(NewtonCtl), 0));
    alloc(c->nt_ctl, (size_t)S * sizeof(NewtonCtl));
    HIPCHK(hipMemsetAsync(c->vals.p, 0, c->vals.n, st));
    sync(c);
}

// -------------------------------------------------------- building blocks
// Energies (three parts per shell, host) and gradient at q_in.
// eval_shell_dev: only the patches of shells flagged there are evaluated
// (the others keep their previous patch outputs); NULL: every shell.
void eval_energy_grad(shell_ctx* c, const double* q_in, const double* qhat, double mass_scale, int loads,
                      bool masked, double* grad_out, const int* write_shell_dev, const int* eval_shell_dev = nullptr,
                      bool to_host = true) {
    hipStream_t st = c->stream;
    GroupTimer tmr(c, SHELL_T_ENERGY_GRAD);
    launch_energy_grad(st, c->P, dptr<int4>(c->patch_nodes), dptr<int>(c->patch_shell),
                       dptr<ShellParams>(c->shells_d), dptr<double>(c->phi), q_in, dptr<double>(c->qbar), qhat,
                       mass_scale, c->dt_damp, 1, loads, eval_shell_dev, dptr<double>(c->e_patch),
                       dptr<double>(c->g_patch), c->eg_patches);
    launch_shell_energy(st, c->S, dptr<ShellParams>(c->shells_d), dptr<double>(c->e_patch), dptr<double>(c->e_shell));
    if (grad_out)
        launch_gather_grad(st, c->N, dptr<int>(c->inc_ptr), dptr<int>(c->inc), dptr<double>(c->g_patch),
                           masked ? dptr<uint16_t>(c->freemask) : nullptr, dptr<int>(c->node_shell), write_shell_dev,
                           grad_out);
    if (c->alm_on) {   // -lambda.c + (kappa/2)|c|^2 of the point constraints
        if (grad_out)
            launch_alm_grad(st, c->N, dptr<int>(c->alm_incp), dptr<int2>(c->alm_inc), dptr<AlmPoint>(c->alm_pts),
                            dptr<double>(c->alm_lam), c->alm_kappa, q_in, masked ? dptr<uint16_t>(c->freemask) : nullptr,
                            dptr<int>(c->node_shell), write_shell_dev, grad_out);
        launch_alm_energy(st, c->S, dptr<int>(c->alm_spt), dptr<AlmPoint>(c->alm_pts), dptr<double>(c->alm_lam),
                          c->alm_kappa, q_in, dptr<double>(c->e_shell));
    }
    if (loads && c->has_load() && qhat)
        launch_nodal_load(st, c->rb(), c->S, c->load_vec(), q_in, qhat, dptr<uint16_t>(c->freemask),
                          dptr<int>(c->node_shell), write_shell_dev, grad_out, dptr<double>(c->red_part),
                          dptr<double>(c->e_shell));
    HIPCHK(hipGetLastError());
    tmr.stop();
    if (to_host)
        HIPCHK(hipMemcpyAsync(c->h_e_shell, c->e_shell.p, (size_t)c->S * 3 * sizeof(double), hipMemcpyDeviceToHost,
                              st));
}

// per-shell x.y over free DOFs (masked) or all DOFs; result in red_out, and
// in c->h_red after sync when to_host
void shell_dot(shell_ctx* c, const double* x, const double* y, bool masked, bool to_host = true) {
    launch_shell_dot(c->stream, c->rb(), c->S, x, y, masked ? dptr<uint16_t>(c->freemask) : nullptr,
                     dptr<double>(c->red_part), dptr<double>(c->red_out));
    if (to_host)
        HIPCHK(hipMemcpyAsync(c->h_red, c->red_out.p, (size_t)c->S * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
}

void assemble(shell_ctx* c, const double* q_in, double mass_scale, int elastic) {
    hipStream_t st = c->stream;
    GroupTimer tmr(c, SHELL_T_HESSIAN);
    const int pseudo = c->opts.hessian == SHELL_HESS_PSEUDO;
    // one launch over all patches into scratch, or one per colour into the matrix
    const int nlaunch = c->asm_gather ? 1 : (int)c->colour_off.size() - 1;
    for (int col = 0; col < nlaunch; ++col) {
        const int off = c->asm_gather ? 0 : c->colour_off[col];
        const int n = c->asm_gather ? c->P : c->colour_off[col + 1] - off;
        const int* list = dptr<int>(c->colour_list) + off;
        const int* slots = dptr<int>(c->patch_slots);
        const uint64_t* kid = dptr<uint64_t>(c->patch_kid);
        const uint16_t* first = dptr<uint16_t>(c->patch_first);
        const ShellParams* sh = dptr<ShellParams>(c->shells_d);
        const double* phi = dptr<double>(c->phi);
        const double* qbar = dptr<double>(c->qbar);
        if (c->fp32)
            launch_hessian<float>(st, list, n, dptr<int4>(c->patch_nodes), dptr<int>(c->patch_shell), slots, kid,
                                  first, sh, phi, q_in, qbar, mass_scale, c->dt_damp, elastic, pseudo,
                                  dptr<float>(c->vals), c->hs_waves,
                                  c->asm_gather ? dptr<float>(c->asm_scr) : nullptr);
        else
            launch_hessian<double>(st, list, n, dptr<int4>(c->patch_nodes), dptr<int>(c->patch_shell), slots, kid,
                                   first, sh, phi, q_in, qbar, mass_scale, c->dt_damp, elastic, pseudo,
                                   dptr<double>(c->vals), c->hs_waves,
                                   c->asm_gather ? dptr<double>(c->asm_scr) : nullptr);
    }
    if (c->asm_gather) {
        if (c->fp32)
            launch_gather_blocks<float>(st, (int)c->nnzb_u, dptr<int>(c->asm_cptr), dptr<int>(c->asm_cidx),
                                        dptr<uint8_t>(c->asm_diag), dptr<float>(c->asm_scr), dptr<float>(c->vals));
        else
            launch_gather_blocks<double>(st, (int)c->nnzb_u, dptr<int>(c->asm_cptr), dptr<int>(c->asm_cidx),
                                         dptr<uint8_t>(c->asm_diag), dptr<double>(c->asm_scr), dptr<double>(c->vals));
    }
    HIPCHK(hipGetLastError());
    tmr.stop();
    c->tm.patch_evals += c->P;
}

void spmv(shell_ctx* c, const double* x, const double* b, double* y, int mode) {
    GroupTimer tmr(c, SHELL_T_SPMV);
    if (c->fp32)
        launch_spmv<float>(c->stream, c->N, c->sym(), dptr<float>(c->vals), dptr<uint16_t>(c->freemask), x, b, y,
                           dptr<double>(c->slot), mode);
    else
        launch_spmv<double>(c->stream, c->N, c->sym(), dptr<double>(c->vals), dptr<uint16_t>(c->freemask), x, b, y,
                            dptr<double>(c->slot), mode);
    HIPCHK(hipGetLastError());
    tmr.stop();
}

// Enqueue the block-Jacobi factorisation and the copy of the per-shell
// failure flags to h_fail (valid after the next synchronisation).
void bj_factor_enqueue(shell_ctx* c) {
    hipStream_t st = c->stream;
    launch_zero(st, c->fail_shell.p, c->fail_shell.n);
    GroupTimer tmr(c, SHELL_T_BJ);
    if (c->fp32)
        launch_bj_factor<float>(st, c->N, dptr<int>(c->diag_blk), c->vals.p, 1, dptr<uint16_t>(c->freemask),
                                dptr<int>(c->node_shell), dptr<float>(c->dinv), dptr<int>(c->fail_shell));
    else
        launch_bj_factor<double>(st, c->N, dptr<int>(c->diag_blk), c->vals.p, 0, dptr<uint16_t>(c->freemask),
                                 dptr<int>(c->node_shell), dptr<double>(c->dinv), dptr<int>(c->fail_shell));
    HIPCHK(hipGetLastError());
    tmr.stop();
    HIPCHK(hipMemcpyAsync(c->h_fail, c->fail_shell.p, (size_t)c->S * sizeof(int), hipMemcpyDeviceToHost, st));
}

// Factor the block-Jacobi preconditioner; per-shell failure flags in h_fail.
void bj_factor(shell_ctx* c) {
    bj_factor_enqueue(c);
    sync(c);
}

// Enqueue one CG launch on rhs b for the shells flagged in cg_active, with
// the tolerances and caps in cg_rtol2 / cg_maxit (device); solution in cg_x,
// per-shell results in cg_out (and h_cg_out after sync when to_host).
void cg_enqueue(shell_ctx* c, const double* b, bool to_host) {
    hipStream_t st = c->stream;
    unsigned long long* trace = nullptr;
    const size_t trace_bytes = (size_t)c->nblk * CG_TRACE_ITERS * 6 * sizeof(unsigned long long);
    if (c->cg_tracing && c->cg_trace.n >= trace_bytes) {   // sized by shell_cg_trace_enable / set_row_blocks
        trace = dptr<unsigned long long>(c->cg_trace);
        launch_zero(st, c->cg_trace.p, trace_bytes);
    }
    launch_zero3(st, c->cg_bar.p, c->cg_bar.n, c->cg_nbflag.p, c->cg_nbflag.n, c->cg_abort.p, c->cg_abort.n);
    GroupTimer tmr(c, SHELL_T_CG);
    hipError_t e;
    if (c->fp32)
        e = launch_cg<float, float>(st, c->nblk, c->cg_threads, c->rb(), c->sym(), dptr<float>(c->vals),
                                    dptr<float>(c->dinv), dptr<uint16_t>(c->freemask), b,
                                    dptr<float>(c->cg_x), dptr<float>(c->cg_r), dptr<float>(c->cg_z),
                                    dptr<float>(c->cg_p0), dptr<float>(c->cg_p1), dptr<float>(c->cg_q),
                                    dptr<float>(c->slot), dptr<double>(c->cg_partial), c->cg_bar.p,
                                    dptr<unsigned>(c->cg_nbflag), dptr<int>(c->cg_abort),
                                    dptr<double>(c->cg_rtol2), dptr<int>(c->cg_maxit), dptr<int>(c->cg_active),
                                    dptr<CgShellOut>(c->cg_out), trace);
    else
        e = launch_cg<double, double>(st, c->nblk, c->cg_threads, c->rb(), c->sym(), dptr<double>(c->vals),
                                      dptr<double>(c->dinv), dptr<uint16_t>(c->freemask), b,
                                      dptr<double>(c->cg_x), dptr<double>(c->cg_r), dptr<double>(c->cg_z),
                                      dptr<double>(c->cg_p0), dptr<double>(c->cg_p1), dptr<double>(c->cg_q),
                                      dptr<double>(c->slot), dptr<double>(c->cg_partial), c->cg_bar.p,
                                      dptr<unsigned>(c->cg_nbflag), dptr<int>(c->cg_abort),
                                      dptr<double>(c->cg_rtol2), dptr<int>(c->cg_maxit), dptr<int>(c->cg_active),
                                      dptr<CgShellOut>(c->cg_out), trace);
    HIPCHK(e);
    tmr.stop();
    if (to_host)
        HIPCHK(hipMemcpyAsync(c->h_cg_out, c->cg_out.p, (size_t)c->S * sizeof(CgShellOut), hipMemcpyDeviceToHost,
                              st));
}

// One CG launch on rhs b for the shells with active[s]; solution in cg_x.
void cg_launch(shell_ctx* c, const double* b, const std::vector<int>& active, const std::vector<double>& rtol,
               int maxit) {
    std::vector<double> rt2(c->S);
    std::vector<int> mi(c->S, maxit);
    for (int s = 0; s < c->S; ++s) rt2[s] = rtol[s] * rtol[s];
    h2d(c, c->cg_rtol2.p, rt2.data(), c->S * sizeof(double));
    h2d(c, c->cg_maxit.p, mi.data(), c->S * sizeof(int));
    h2d(c, c->cg_active.p, active.data(), c->S * sizeof(int));
    run_graph(c, c->g_cg, (double)(uintptr_t)b, [&] { cg_enqueue(c, b, true); });
    sync(c);
    if (c->timing) {
        long long mx = 0;
        for (int s = 0; s < c->S; ++s)
            if (active[s]) {
                const long long it = c->h_cg_out[s].iters;
                c->tm.cg_iter_rows += it * c->rows_s[s];
                c->tm.cg_iter_blocks += it * c->nnzb_s[s];
                mx = std::max(mx, it);
            }
        c->tm.cg_iters_max += mx;
    }
    for (int s = 0; s < c->S; ++s)
        if (active[s] && c->h_cg_out[s].status == 3)
            throw StatusErr{SHELL_E_DEVICE, "CG grid barrier timed out"};
}

// ---------------------------------------------------- warm-start network
void mlp_alloc(shell_ctx* c) {
    if (c->mlp_theta.p) return;
    alloc(c->mlp_theta, MLP_NPARAMS * sizeof(float));
    alloc(c->mlp_w, (size_t)mlp_bf16_elems() * 2);
    alloc(c->mlp_m, MLP_NPARAMS * sizeof(float));
    alloc(c->mlp_v, MLP_NPARAMS * sizeof(float));
    alloc(c->mlp_grad, MLP_NPARAMS * sizeof(float));
    alloc(c->mlp_loss, sizeof(double));
}

void mlp_work(shell_ctx* c, int batch) {
    if (c->mlp_work_batch >= batch) return;
    alloc(c->mlp_work, mlp_train_work_bytes(batch));
    alloc(c->mlp_idx, (size_t)batch * sizeof(long long));
    c->mlp_work_batch = batch;
}

// Per-shell, per-kind feature scales of (q - qbar, b, dprev).
void feat_scales(shell_ctx* c, const double* q, const double* b, const double* dprev) {
    launch_feat_scale(c->stream, c->rb(), c->S, q, dptr<double>(c->qbar), b, dprev, dptr<uint16_t>(c->freemask),
                      dptr<double>(c->feat_part), dptr<int>(c->cnt_kind), dptr<float>(c->feat_scale));
    HIPCHK(hipGetLastError());
}

struct SolveResult {
    std::vector<int> iters, status, sweeps;   // status: 0 ok, 1 cap, 2 indefinite
    std::vector<double> relres;
};
// per shell: still refining, ||b||^2, last relative residual (mixed form)
struct RefineState {
    std::vector<int> active;
    std::vector<double> bn2, prev;
};
void refine_sweeps(shell_ctx* c, const double* b, const std::vector<int>& active_in, RefineState& F,
                   const std::vector<double>& rtol, int maxit, SolveResult& R, int sweep0);

// Solve A x = b (masked) for the active shells and write x into x_out for
// those shells only (other shells' entries of x_out are left as they are).
// FP64 path: one CG.  Mixed path: FP32 CG sweeps on the FP64 residual,
// x += dx, r = b - A x in FP64, until ||r|| <= rtol ||b||.
SolveResult solve(shell_ctx* c, const double* b, double* x_out, const std::vector<int>& active_in,
                  const std::vector<double>& rtol, int maxit) {
    const int S = c->S;
    hipStream_t st = c->stream;
    SolveResult R;
    R.iters.assign(S, 0);
    R.status.assign(S, 0);
    R.sweeps.assign(S, 0);
    R.relres.assign(S, 0.0);
    double* x64 = dptr<double>(c->x64);
    if (!c->fp32) {
        cg_launch(c, b, active_in, rtol, maxit);
        for (int s = 0; s < S; ++s) {
            const CgShellOut& o = c->h_cg_out[s];
            R.iters[s] = o.iters;
            R.status[s] = active_in[s] ? o.status : 0;
            R.relres[s] = o.bnorm2 > 0 ? std::sqrt(o.rnorm2 / o.bnorm2) : 0.0;
            R.sweeps[s] = 1;
        }
        h2d(c, c->flag_shell.p, active_in.data(), S * sizeof(int));
        launch_copy_shell(st, c->N, dptr<double>(c->cg_x), dptr<int>(c->node_shell), dptr<int>(c->flag_shell),
                          x_out);
        HIPCHK(hipGetLastError());
        return R;
    }
    // mixed precision refinement
    double* r64 = dptr<double>(c->r64);
    HIPCHK(hipMemsetAsync(x64, 0, (size_t)c->N * 12 * sizeof(double), st));
    HIPCHK(hipMemcpyAsync(r64, b, (size_t)c->N * 12 * sizeof(double), hipMemcpyDeviceToDevice, st));
    shell_dot(c, b, b, true);
    sync(c);
    RefineState F;
    F.bn2.assign(c->h_red, c->h_red + S);
    F.active = active_in;
    F.prev.assign(S, 1.0);
    refine_sweeps(c, b, active_in, F, rtol, maxit, R, 0);
    h2d(c, c->flag_shell.p, active_in.data(), S * sizeof(int));
    launch_copy_shell(st, c->N, x64, dptr<int>(c->node_shell), dptr<int>(c->flag_shell), x_out);
    HIPCHK(hipGetLastError());
    return R;
}

// Sweeps sweep0 .. 29 of the mixed form from the current x64 and r64 = b -
// A x64 (FP64): each asks the FP32 CG for the reduction still needed (with a
// margin) on the residual, adds its correction and recomputes the residual.
void refine_sweeps(shell_ctx* c, const double* b, const std::vector<int>& active_in, RefineState& F,
                   const std::vector<double>& rtol, int maxit, SolveResult& R, int sweep0) {
    const int S = c->S;
    hipStream_t st = c->stream;
    double* x64 = dptr<double>(c->x64);
    double* r64 = dptr<double>(c->r64);
    std::vector<int>& active = F.active;
    std::vector<double>& bn2 = F.bn2;
    std::vector<double>& prev = F.prev;
    for (int sweep = sweep0; sweep < 30; ++sweep) {
        bool any = false;
        for (int s = 0; s < S; ++s) {
            if (active[s] && bn2[s] == 0.0) active[s] = 0;
            any |= active[s] != 0;
        }
        if (!any) break;
        // each sweep asks the FP32 CG for the reduction still needed (with a
        // margin), but not below what FP32 arithmetic resolves
        std::vector<double> inner(S);
        for (int s = 0; s < S; ++s) inner[s] = std::max(0.5 * rtol[s] / prev[s], 1e-6);
        cg_launch(c, r64, active, inner, maxit);
        for (int s = 0; s < S; ++s)
            if (active[s]) {
                R.iters[s] += c->h_cg_out[s].iters;
                R.sweeps[s]++;
                if (c->h_cg_out[s].status == 2) {
                    R.status[s] = 2;
                    active[s] = 0;
                }
            }
        // CG leaves x = 0 for inactive shells, so the update touches active shells only
        launch_add_to<float>(st, c->N * 12, dptr<float>(c->cg_x), x64);
        spmv(c, x64, b, r64, 1 | 4);
        shell_dot(c, r64, r64, true);
        sync(c);
        for (int s = 0; s < S; ++s) {
            if (!active_in[s] || bn2[s] == 0.0) continue;
            const double rel = std::sqrt(c->h_red[s] / bn2[s]);
            if (!active[s]) continue;
            R.relres[s] = rel;
            if (rel <= rtol[s]) {
                active[s] = 0;
            } else if (rel > 0.5 * prev[s] || R.iters[s] >= maxit) {
                R.status[s] = 1;   // refinement stagnates
                active[s] = 0;
            }
            prev[s] = rel;
        }
    }
}

// One Newton iteration of every active shell as one launch sequence, the
// decisions taken by the control kernels of newton_kernels.hip on nt_ctl:
// A = K(q) + M/dt^2 and its block-Jacobi factors, the direction A d = -g
// (one FP64 CG, or NT_REFINE_SWEEPS sweeps of the mixed form), the slope
// g.d, NT_LS_TRIALS line-search trials, and the convergence test of the
// next iteration with the rounding floor from this iteration's matrix.  A
// shell that needs the regulariser, more sweeps or more trials is left to
// the host at that stage (NewtonCtl::need_host).  The per-shell state goes
// back to h_ctl at the end.
constexpr int NT_REFINE_SWEEPS = 2, NT_LS_TRIALS = 2;
void newton_iteration_device(shell_ctx* c, double ms, double* q, double* g, double* qt, double* gt, double* d,
                             double* rhs, const double* qhat) {
    hipStream_t st = c->stream;
    const int S = c->S, N = c->N;
    NewtonCtl* ctl = dptr<NewtonCtl>(c->nt_ctl);
    int* cg_active = dptr<int>(c->cg_active);
    int* flag = dptr<int>(c->flag_shell);
    int* wr = dptr<int>(c->write_shell);
    double* red = dptr<double>(c->red_out);
    double* alpha = dptr<double>(c->alpha_shell);
    double* x64 = dptr<double>(c->x64);
    const uint16_t* fm = dptr<uint16_t>(c->freemask);
    const int* ns = dptr<int>(c->node_shell);
    assemble(c, q, ms, 1);
    launch_save_diag(st, N, dptr<int>(c->diag_blk), c->vals.p, c->fp32, dptr<double>(c->diag0));
    bj_factor_enqueue(c);
    launch_nt_factor(st, S, ctl, dptr<int>(c->fail_shell), cg_active, dptr<double>(c->cg_rtol2),
                     dptr<int>(c->cg_maxit), c->opts.pcg_rtol, c->opts.pcg_maxit);
    launch_neg_masked(st, N, g, fm, ns, cg_active, rhs);
    if (!c->fp32) {
        // the FP64 CG's x is the direction itself
        cg_enqueue(c, rhs, false);
        launch_nt_cg64(st, S, ctl, dptr<CgShellOut>(c->cg_out), flag);
    } else {
        double* r64 = dptr<double>(c->r64);
        launch_zero(st, c->x64.p, c->x64.n);
        HIPCHK(hipMemcpyAsync(r64, rhs, (size_t)N * 12 * sizeof(double), hipMemcpyDeviceToDevice, st));
        shell_dot(c, rhs, rhs, true, false);
        launch_nt_ref_init(st, S, ctl, red, cg_active, dptr<double>(c->cg_rtol2), c->opts.pcg_rtol);
        for (int sw = 0; sw < NT_REFINE_SWEEPS; ++sw) {
            cg_enqueue(c, r64, false);
            launch_nt_ref_cg(st, S, ctl, dptr<CgShellOut>(c->cg_out), cg_active);
            launch_add_to<float>(st, N * 12, dptr<float>(c->cg_x), x64);
            spmv(c, x64, rhs, r64, 1 | 4);
            shell_dot(c, r64, r64, true, false);
            launch_nt_ref_check(st, S, ctl, red, cg_active, dptr<double>(c->cg_rtol2), c->opts.pcg_rtol,
                                c->opts.pcg_maxit);
        }
        launch_nt_ref_end(st, S, ctl, flag);
    }
    launch_copy_shell(st, N, c->fp32 ? x64 : dptr<double>(c->cg_x), ns, flag, d);
    // line search along d (-g where d is not a descent direction)
    shell_dot(c, g, d, true, false);
    launch_nt_ls_init(st, S, ctl, red, alpha, flag, wr);
    launch_neg_masked(st, N, g, fm, ns, flag, rhs);
    launch_copy_shell(st, N, rhs, ns, flag, d);
    for (int t = 0; t < NT_LS_TRIALS; ++t) {
        launch_axpy_shell(st, N, q, d, alpha, ns, qt);
        eval_energy_grad(c, qt, qhat, ms, 1, true, gt, wr, wr, false);
        shell_dot(c, gt, gt, true, false);
        launch_nt_ls_step(st, S, t, ctl, dptr<double>(c->e_shell), red, alpha, flag, wr);
        launch_copy_shell2(st, N, qt, gt, ns, flag, q, g);
    }
    launch_nt_ls_end(st, S, ctl);
    // the next iteration's convergence test
    spmv(c, q, nullptr, rhs, 8 | 2);
    shell_dot(c, rhs, rhs, true, false);
    launch_nt_check(st, S, ctl, red, c->opts.newton_rtol, c->opts.newton_maxit);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->h_ctl, c->nt_ctl.p, (size_t)S * sizeof(NewtonCtl), hipMemcpyDeviceToHost, st));
}

// Learned warm start of the Newton iteration.  Two directions from the
// step's start q_s: d1 = the previous step's correction (extrapolation) and
// d2 = the network's correction s_d y(features).  The start moves to
// q_s + c1 d1 + c2 d2 with c the Galerkin solution of the quadratic model
// of E in span{d1, d2}, whose Hessian is taken from gradient differences
// (H d_j ~ grad E(q_s + d_j) - grad E(q_s), symmetrised); a direction
// dependent on d1, or with non-positive curvature, is dropped.  The move is
// taken if E satisfies the Armijo condition and ||grad E|| is at least
// halved (Newton's convergence measure: a start that lowers E but not the
// gradient only costs iterations); if the two-direction point fails, the
// one-direction Galerkin point along d1 is tried.  A shell whose network
// output is not finite keeps q_s, as does one without a previous
// correction.  Updates q, g, E, gn of the shells that move.
void newton_warm_start(shell_ctx* c, double ms, const std::vector<int>& active, std::vector<double>& E,
                       std::vector<double>& Escale, std::vector<double>& gn, std::vector<shell_step_stats>& stats) {
    const int S = c->S;
    hipStream_t st = c->stream;
    double* q = dptr<double>(c->q);
    double* qt = dptr<double>(c->qt);
    double* g = dptr<double>(c->g);
    double* gt = dptr<double>(c->gt);
    const double* d1 = dptr<double>(c->dstep);
    double* d2 = dptr<double>(c->guess);
    std::vector<int> cand(S, 0);
    bool any = false;
    for (int s = 0; s < S; ++s) {
        cand[s] = active[s] && c->h_hist[s];
        any |= cand[s] != 0;
    }
    if (!any) return;
    h2d(c, c->flag_shell.p, cand.data(), S * sizeof(int));
    launch_mlp_guess(st, c->N, dptr<float>(c->mlp_theta), c->mlp_w.p, dptr<int>(c->node_shell),
                     dptr<int>(c->flag_shell), q, dptr<double>(c->qbar), dptr<double>(c->b0), d1,
                     dptr<uint16_t>(c->freemask), dptr<int>(c->nbr8), dptr<float>(c->feat_scale), d2);
    HIPCHK(hipGetLastError());
    auto dots = [&](const double* x, const double* y) {
        shell_dot(c, x, y, true);
        sync(c);
        return std::vector<double>(c->h_red, c->h_red + S);
    };
    std::vector<double> Et(S), Est(S), gtn(S);
    // E, ||g|| and g at q + c1 d1 + c2 d2 (coefficients per shell, 0 = unchanged)
    auto trial = [&](const std::vector<double>& coef) {
        h2d(c, c->alpha_shell.p, coef.data(), 2 * S * sizeof(double));
        launch_axpy2_shell(st, c->N, q, d1, d2, dptr<double>(c->alpha_shell), dptr<int>(c->node_shell), qt);
        eval_energy_grad(c, qt, dptr<double>(c->qhat), ms, 1, true, gt, nullptr);
        const std::vector<double> n2 = dots(gt, gt);
        for (int s = 0; s < S; ++s) {
            const double* e = c->h_e_shell + 3 * s;
            Et[s] = e[0] + e[1] + e[2];
            Est[s] = std::fabs(e[0]) + std::fabs(e[1]) + std::fabs(e[2]);
            gtn[s] = std::sqrt(n2[s]);
        }
    };
    const std::vector<double> a1 = dots(d1, g), a2 = dots(d2, g), n22 = dots(d2, d2);
    for (int s = 0; s < S; ++s)   // non-finite network output: no warm start for that shell
        if (cand[s] && !(std::isfinite(a2[s]) && std::isfinite(n22[s]))) cand[s] = 0;
    // curvature probes along d1 and along d2
    std::vector<double> coef(2 * S, 0.0);
    for (int s = 0; s < S; ++s) coef[2 * s] = cand[s] ? 1.0 : 0.0;
    trial(coef);
    const std::vector<double> h11 = dots(d1, gt), h21 = dots(d2, gt);
    for (int s = 0; s < S; ++s) coef[2 * s] = 0.0, coef[2 * s + 1] = (cand[s] && n22[s] > 0.0) ? 1.0 : 0.0;
    trial(coef);
    const std::vector<double> h12 = dots(d1, gt), h22 = dots(d2, gt);
    for (int s = 0; s < S; ++s) {
        coef[2 * s] = coef[2 * s + 1] = 0.0;
        if (!cand[s]) continue;
        const double H11 = h11[s] - a1[s];
        const double H22 = n22[s] > 0.0 ? h22[s] - a2[s] : 0.0;
        const double H12 = n22[s] > 0.0 ? 0.5 * ((h12[s] - a1[s]) + (h21[s] - a2[s])) : 0.0;
        double c1 = 0.0, c2 = 0.0;
        const double det = H11 * H22 - H12 * H12;
        if (H11 > 0.0 && H22 > 0.0 && det > 1e-8 * H11 * H22) {
            c1 = (-a1[s] * H22 + a2[s] * H12) / det;
            c2 = (-a2[s] * H11 + a1[s] * H12) / det;
        } else if (H11 > 0.0) {
            c1 = -a1[s] / H11;
        } else if (H22 > 0.0) {
            c2 = -a2[s] / H22;
        }
        if (!std::isfinite(c1) || !std::isfinite(c2) || (c1 == 0.0 && c2 == 0.0)) {
            cand[s] = 0;
            continue;
        }
        coef[2 * s] = c1;
        coef[2 * s + 1] = c2;
    }
    // try the Galerkin point; where it fails and used d2, retry along d1 alone
    auto accept = [&](const std::vector<double>& cf, const std::vector<int>& which) {
        std::vector<int> acc(S, 0);
        for (int s = 0; s < S; ++s) {
            if (!which[s]) continue;
            const double slope = cf[2 * s] * a1[s] + cf[2 * s + 1] * a2[s];
            acc[s] = std::isfinite(Et[s]) && std::isfinite(gtn[s]) && slope < 0.0 &&
                     Et[s] <= E[s] + 1e-4 * slope && gtn[s] <= 0.5 * gn[s];
        }
        h2d(c, c->flag_shell.p, acc.data(), S * sizeof(int));
        launch_copy_shell(st, c->N, qt, dptr<int>(c->node_shell), dptr<int>(c->flag_shell), q);
        launch_copy_shell(st, c->N, gt, dptr<int>(c->node_shell), dptr<int>(c->flag_shell), g);
        HIPCHK(hipGetLastError());
        for (int s = 0; s < S; ++s)
            if (acc[s]) {
                E[s] = Et[s];
                Escale[s] = Est[s];
                gn[s] = gtn[s];
                stats[s].warm_start_used = 1;
            }
        return acc;
    };
    trial(coef);
    const std::vector<int> acc = accept(coef, cand);
    std::vector<int> retry(S, 0);
    bool anyr = false;
    for (int s = 0; s < S; ++s) {
        const double H11 = h11[s] - a1[s];
        retry[s] = cand[s] && !acc[s] && coef[2 * s + 1] != 0.0 && H11 > 0.0;
        coef[2 * s] = retry[s] ? -a1[s] / H11 : 0.0;
        coef[2 * s + 1] = 0.0;
        anyr |= retry[s] != 0;
    }
    if (!anyr) return;
    trial(coef);
    accept(coef, retry);
}

// Append K sampled (features, target) rows per flagged shell to the
// recording buffers while they have room: features at the start of the
// step (qstart, b0, dstep), target from the step's correction d.
void record_samples(shell_ctx* c, const double* d, const std::vector<int>& flag) {
    if (!c->rec_feat) return;
    const int S = c->S;
    std::vector<long long> base(S, -1);
    bool any = false;
    for (int s = 0; s < S; ++s)
        if (flag[s] && c->rec_count + c->rec_K <= c->rec_cap) {
            base[s] = c->rec_count;
            c->rec_count += c->rec_K;
            any = true;
        }
    if (!any) return;
    h2d(c, c->rec_base.p, base.data(), S * sizeof(long long));
    const unsigned long long seed = c->rec_seed + 0xD1B54A32D192ED03ull * (unsigned long long)(++c->rec_calls);
    launch_mlp_record(c->stream, S, c->rec_K, seed, dptr<ShellParams>(c->shells_d), dptr<long long>(c->rec_base),
                      dptr<double>(c->qstart), dptr<double>(c->qbar), dptr<double>(c->b0), dptr<double>(c->dstep), d,
                      dptr<int>(c->nbr8), dptr<float>(c->feat_scale), c->rec_feat, c->rec_tgt);
    HIPCHK(hipGetLastError());
}

}  // namespace

// ================================================================= C ABI
extern "C" {

void shell_default_opts(shell_opts* o) {
    if (!o) return;
    o->precision = SHELL_FP64;
    o->hessian = SHELL_HESS_EXACT;
    o->warm_start = SHELL_WS_NONE;
    o->newton_maxit = 50;
    o->pcg_maxit = 100000;
    o->newton_rtol = 1e-10;
    o->pcg_rtol = 1e-10;
    o->device = 0;
    o->stream = nullptr;
    o->graphs = 1;
    o->cg_resident = 1;
    o->device_newton = 1;
}

const char* shell_last_error(const shell_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

shell_status shell_create(const shell_desc* shells, int32_t n_shells, const shell_opts* o, shell_ctx** out) {
    if (out) *out = nullptr;
    g_create_error.clear();
    if (!shells || n_shells < 1 || !out) {
        g_create_error = "shells, n_shells >= 1 and out are required";
        return SHELL_E_INVAL;
    }
    shell_opts opts;
    shell_default_opts(&opts);
    if (o) opts = *o;
    if ((opts.precision != SHELL_FP64 && opts.precision != SHELL_MIXED) ||
        (opts.hessian != SHELL_HESS_EXACT && opts.hessian != SHELL_HESS_PSEUDO) ||
        (opts.warm_start != SHELL_WS_NONE && opts.warm_start != SHELL_WS_MLP) || opts.newton_maxit < 1 ||
        opts.pcg_maxit < 1 || !(opts.newton_rtol >= 0) || !(opts.pcg_rtol > 0)) {
        g_create_error = "invalid options";
        return SHELL_E_INVAL;
    }
    shell_ctx* c = nullptr;
    try {
        for (int s = 0; s < n_shells; ++s) validate(shells[s], s);
        int ndev = 0;
        HIPCHK(hipGetDeviceCount(&ndev));
        if (opts.device < 0 || opts.device >= ndev) throw InvalErr{"invalid device ordinal"};
        HIPCHK(hipSetDevice(opts.device));
        c = new shell_ctx();
        c->opts = opts;
        c->stream = (hipStream_t)opts.stream;
        c->fp32 = opts.precision == SHELL_MIXED;
        c->graphs = opts.graphs != 0;
        c->cg_resident = opts.cg_resident != 0;
        build(c, shells, n_shells);
    } catch (const InvalErr& e) {
        g_create_error = e.msg;
        delete c;
        return SHELL_E_INVAL;
    } catch (const StatusErr& e) {
        g_create_error = e.msg;
        delete c;
        return e.st;
    } catch (const HipErr& e) {
        g_create_error = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
        delete c;
        return SHELL_E_DEVICE;
    } catch (const std::bad_alloc&) {
        g_create_error = "host out of memory";
        delete c;
        return SHELL_E_NOMEM;
    }
    *out = c;
    return SHELL_OK;
}

void shell_destroy(shell_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

shell_status shell_sizes(const shell_ctx* c, int32_t* total_nodes, int32_t* total_patches, int64_t* nnzb) {
    if (!c) return SHELL_E_INVAL;
    if (total_nodes) *total_nodes = c->N;
    if (total_patches) *total_patches = c->P;
    if (nnzb) *nnzb = c->nnzb;
    return SHELL_OK;
}

#define API_TRY try {
#define API_CATCH                                                                     \
    }                                                                                 \
    catch (const InvalErr& e) {                                                       \
        c->err = e.msg;                                                               \
        return SHELL_E_INVAL;                                                         \
    }                                                                                 \
    catch (const StatusErr& e) {                                                      \
        c->err = e.msg;                                                               \
        return e.st;                                                                  \
    }                                                                                 \
    catch (const HipErr& e) {                                                         \
        c->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e); \
        return SHELL_E_DEVICE;                                                        \
    }

shell_status shell_energy_grad_hess(shell_ctx* c, const double* q_dev, double* energy_host, double* grad_dev,
                                    int32_t assemble_hessian) {
    if (!c) return SHELL_E_INVAL;
    if (!q_dev) {
        c->err = "q_dev is NULL";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    eval_energy_grad(c, q_dev, nullptr, 0.0, 0, false, grad_dev, nullptr);
    if (assemble_hessian) assemble(c, q_dev, 0.0, 1);
    sync(c);
    for (int s = 0; s < c->S; ++s) {
        const double e = c->h_e_shell[3 * s];
        if (energy_host) energy_host[s] = e;
        if (!std::isfinite(e)) {
            c->err = "non-finite energy in shell " + std::to_string(s);
            return SHELL_E_NONFINITE;
        }
    }
    return SHELL_OK;
    API_CATCH
}

shell_status shell_assemble(shell_ctx* c, const double* q_dev, double mass_scale, int32_t elastic) {
    if (!c) return SHELL_E_INVAL;
    if (!q_dev || !std::isfinite(mass_scale)) {
        c->err = "q_dev is NULL or mass_scale not finite";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    assemble(c, q_dev, mass_scale, elastic ? 1 : 0);
    sync(c);
    return SHELL_OK;
    API_CATCH
}

shell_status shell_get_bsr(shell_ctx* c, int32_t shell, int32_t* nnzb, int32_t* row_ptr, int32_t* col_idx,
                           double* vals) {
    if (!c) return SHELL_E_INVAL;
    if (shell < 0 || shell >= c->S || !nnzb) {
        c->err = "invalid shell index or nnzb NULL";
        return SHELL_E_INVAL;
    }
    API_TRY
    const int n0 = c->shells[shell].node_begin, n1 = c->shells[shell].node_end;
    const int b0 = c->h_row_ptr[n0], b1 = c->h_row_ptr[n1];
    *nnzb = b1 - b0;
    if (row_ptr)
        for (int n = n0; n <= n1; ++n) row_ptr[n - n0] = c->h_row_ptr[n] - b0;
    if (col_idx)
        for (int b = b0; b < b1; ++b) col_idx[b - b0] = c->h_col_idx[b] - n0;
    if (vals) {
        // stored blocks of the shell's rows, then the full pattern from them
        const int u0 = c->h_urow[n0], u1 = c->h_urow[n1];
        const size_t cnt = (size_t)(u1 - u0) * 144;
        std::vector<double> tmp(cnt);
        if (c->fp32) {
            std::vector<float> f(cnt);
            HIPCHK(hipMemcpyAsync(f.data(), dptr<float>(c->vals) + (size_t)u0 * 144, cnt * sizeof(float),
                                  hipMemcpyDeviceToHost, c->stream));
            sync(c);
            for (size_t i = 0; i < cnt; ++i) tmp[i] = f[i];
        } else {
            HIPCHK(hipMemcpyAsync(tmp.data(), dptr<double>(c->vals) + (size_t)u0 * 144, cnt * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream));
            sync(c);
        }
        // The products read the stored block of pair (i, j > i) as A_ij
        // row-major and a diagonal block from its packed symmetric layout
        // (the matrix returned here is the one the products apply).  The ABI
        // returns row-major blocks: block (n, col) is the stored block
        // (n, col) as it is for col > n, the transpose of the stored block
        // (col, n) for col < n, and the expanded packed block for col = n.
        for (int n = n0; n < n1; ++n)
            for (int b = c->h_row_ptr[n]; b < c->h_row_ptr[n + 1]; ++b) {
                const int col = c->h_col_idx[b];
                const int lo = std::min(n, col), hi = std::max(n, col);
                const int ub = (int)(std::lower_bound(&c->h_ucol[0] + c->h_urow[lo], &c->h_ucol[0] + c->h_urow[lo + 1], hi) -
                                     &c->h_ucol[0]);
                const double* src = tmp.data() + (size_t)(ub - u0) * 144;
                double* dst = vals + (size_t)(b - b0) * 144;
                for (int r = 0; r < 12; ++r)
                    for (int cc = 0; cc < 12; ++cc)
                        dst[r * 12 + cc] = col == n  ? src[sym12_pos(r, cc)]
                                           : col > n ? src[r * 12 + cc]
                                                     : src[cc * 12 + r];
            }
    }
    return SHELL_OK;
    API_CATCH
}

shell_status shell_spmv(shell_ctx* c, const double* x_dev, double* y_dev, int32_t masked) {
    if (!c) return SHELL_E_INVAL;
    if (!x_dev || !y_dev) {
        c->err = "x_dev and y_dev are required";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    spmv(c, x_dev, nullptr, y_dev, masked ? 1 : 0);
    return SHELL_OK;
    API_CATCH
}

shell_status shell_pcg_solve(shell_ctx* c, const double* b_dev, double* x_dev, double rtol, int32_t maxit,
                             int32_t* iters_host, double* relres_host) {
    if (!c) return SHELL_E_INVAL;
    if (!b_dev || !x_dev || !(rtol > 0) || maxit < 1) {
        c->err = "b_dev, x_dev, rtol > 0 and maxit >= 1 are required";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    bj_factor(c);
    for (int s = 0; s < c->S; ++s)
        if (c->h_fail[s]) {
            c->err = "diagonal block not positive definite in shell " + std::to_string(s);
            return SHELL_E_INDEFINITE;
        }
    std::vector<int> active(c->S, 1);
    SolveResult R = solve(c, b_dev, x_dev, active, std::vector<double>(c->S, rtol), maxit);
    sync(c);
    shell_status st = SHELL_OK;
    for (int s = 0; s < c->S; ++s) {
        if (iters_host) iters_host[s] = R.iters[s];
        if (relres_host) relres_host[s] = R.relres[s];
        if (R.status[s] == 2) st = SHELL_E_INDEFINITE;
        else if (R.status[s] == 1 && st == SHELL_OK) st = SHELL_E_NOT_CONVERGED;
    }
    if (st != SHELL_OK) c->err = "CG did not reach the tolerance";
    return st;
    API_CATCH
}

// ---------------------------------------------------------- Newton step
shell_status shell_newton_step(shell_ctx* c, double dt, const double* q_n_dev, const double* v_n_dev,
                               const double* q_presc_dev, double* q_np1_dev, double* v_np1_dev,
                               shell_step_stats* stats_host) {
    if (!c) return SHELL_E_INVAL;
    if (!(dt > 0) || !std::isfinite(dt) || !q_n_dev || !v_n_dev || !q_np1_dev || !v_np1_dev) {
        c->err = "dt > 0 and q_n, v_n, q_np1, v_np1 are required";
        return SHELL_E_INVAL;
    }
    if (q_np1_dev == q_n_dev || v_np1_dev == v_n_dev || q_np1_dev == v_n_dev) {
        c->err = "outputs may not alias inputs";
        return SHELL_E_INVAL;
    }
    if (c->opts.warm_start == SHELL_WS_MLP && !c->mlp_ready) {
        c->err = "warm_start = SHELL_WS_MLP needs shell_mlp_set_params first";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    // damping acts on the inertia term of this step only
    struct DampScope {
        shell_ctx* c;
        ~DampScope() { c->dt_damp = 0.0; }
    } damp_scope{c};
    c->dt_damp = dt;
    // point constraints enter this step's energy, gradient and Hessian
    struct AlmScope {
        shell_ctx* c;
        ~AlmScope() { c->alm_on = false; }
    } alm_scope{c};
    c->alm_on = c->alm_n > 0;
    const double t_start = now_ms();
    const int S = c->S, N12 = c->N * 12;
    hipStream_t st = c->stream;
    const double ms = 1.0 / (dt * dt);
    double* q = dptr<double>(c->q);
    double* qt = dptr<double>(c->qt);
    double* g = dptr<double>(c->g);
    double* gt = dptr<double>(c->gt);
    double* d = dptr<double>(c->dvec);
    double* rhs = dptr<double>(c->rhs);
    double* qhat = dptr<double>(c->qhat);
    std::vector<shell_step_stats> stats(S);
    std::memset(stats.data(), 0, sizeof(shell_step_stats) * S);
    launch_predict(st, N12, q_n_dev, v_n_dev, q_presc_dev, dptr<uint16_t>(c->freemask), dptr<int>(c->node_shell),
                   dptr<ShellParams>(c->shells_d), dt, qhat, q);
    HIPCHK(hipGetLastError());
    // pressure: its load at the step's start, a dead load within the step
    struct LoadScope {
        shell_ctx* c;
        ~LoadScope() { c->use_fstep = false; }
    } load_scope{c};
    if (c->has_pressure) {
        launch_pressure(st, c->P, dptr<int4>(c->patch_nodes), dptr<int>(c->patch_shell), dptr<ShellParams>(c->shells_d),
                        dptr<double>(c->pressure), dptr<double>(c->phi), q_n_dev, dptr<double>(c->g_patch));
        launch_gather_grad(st, c->N, dptr<int>(c->inc_ptr), dptr<int>(c->inc), dptr<double>(c->g_patch), nullptr,
                           dptr<int>(c->node_shell), nullptr, dptr<double>(c->fstep));
        if (c->has_fext) launch_add_to<double>(st, N12, dptr<double>(c->fext), dptr<double>(c->fstep));
        HIPCHK(hipGetLastError());
        c->use_fstep = true;
    }
    // E, g at the initial guess
    eval_energy_grad(c, q, qhat, ms, 1, true, g, nullptr);
    shell_dot(c, g, g, true);
    sync(c);
    std::vector<double> E(S), Escale(S), gn(S), g0(S), floor_(S, 0.0);
    std::vector<int> active(S, 1), status(S, SHELL_E_NOT_CONVERGED);
    for (int s = 0; s < S; ++s) {
        const double* e = c->h_e_shell + 3 * s;
        E[s] = e[0] + e[1] + e[2];
        Escale[s] = std::fabs(e[0]) + std::fabs(e[1]) + std::fabs(e[2]);
        gn[s] = std::sqrt(c->h_red[s]);
        g0[s] = gn[s];
        stats[s].grad_norm0 = g0[s];
        if (!std::isfinite(E[s]) || !std::isfinite(gn[s])) {
            status[s] = SHELL_E_NONFINITE;
            active[s] = 0;
        }
    }
    const bool learned = c->opts.warm_start == SHELL_WS_MLP;
    if (learned || c->rec_feat) {   // features of the step's start
        HIPCHK(hipMemcpyAsync(c->qstart.p, q, (size_t)N12 * sizeof(double), hipMemcpyDeviceToDevice, st));
        h2d(c, c->cg_active.p, active.data(), S * sizeof(int));
        launch_neg_masked(st, c->N, g, dptr<uint16_t>(c->freemask), dptr<int>(c->node_shell),
                          dptr<int>(c->cg_active), dptr<double>(c->b0));
        feat_scales(c, q, dptr<double>(c->b0), dptr<double>(c->dstep));
    }
    if (learned) newton_warm_start(c, ms, active, E, Escale, gn, stats);
    const double eps = 2.220446049250313e-16;
    double t_asm = 0, t_cg = 0;
    // per shell: Newton iterations of the current augmented-Lagrangian round
    // and of the rounds before, multiplier updates, last max |c|
    std::vector<int> kk(S, 0), kbase(S, 0), outer(S, 0);
    std::vector<double> alm_res(S, 0.0), h_c;
    // Convergence test of the shells in `only` (all if NULL): the rounding
    // floor of the gradient from the current matrix, 4 eps || P_free |A| |q| ||
    // (after the first iteration), then the augmented-Lagrangian rounds.
    // Returns whether any shell still iterates.
    auto check = [&](bool have_prev, const std::vector<int>* only) -> bool {
        if (have_prev) {
            run_graph(c, c->g_floor, 0.0, [&] {
                spmv(c, q, nullptr, rhs, 8 | 2);
                shell_dot(c, rhs, rhs, true);
            });
            sync(c);
            for (int s = 0; s < S; ++s)
                if (!only || (*only)[s]) floor_[s] = 4.0 * eps * std::sqrt(c->h_red[s]);
        }
        std::vector<int> conv(S, 0);
        for (int s = 0; s < S; ++s) {
            if (!active[s] || (only && !(*only)[s])) continue;
            stats[s].grad_norm = gn[s];
            stats[s].grad_floor = floor_[s];
            if (gn[s] == 0.0 || (kk[s] > 0 && gn[s] <= std::max(c->opts.newton_rtol * g0[s], floor_[s]))) {
                status[s] = SHELL_OK;
                active[s] = 0;
                conv[s] = 1;
            } else if (kk[s] == c->opts.newton_maxit) {
                status[s] = SHELL_E_NOT_CONVERGED;
                active[s] = 0;
            }
        }
        if (c->alm_on) {
            // augmented Lagrangian (Sec. 6.1): a converged shell whose point
            // constraints are not yet met updates its multipliers and resumes
            bool chk = false;
            for (int s = 0; s < S; ++s) chk |= conv[s] && c->alm_shell_pt[s] < c->alm_shell_pt[s + 1];
            if (chk) {
                h_c.resize(3 * (size_t)c->alm_n);
                launch_alm_residual(st, c->alm_n, dptr<AlmPoint>(c->alm_pts), q, dptr<double>(c->alm_c));
                HIPCHK(hipGetLastError());
                HIPCHK(hipMemcpyAsync(h_c.data(), c->alm_c.p, h_c.size() * sizeof(double), hipMemcpyDeviceToHost, st));
                sync(c);
                std::vector<int> resume(S, 0);
                bool any_resume = false;
                for (int s = 0; s < S; ++s) {
                    const int j0 = c->alm_shell_pt[s], j1 = c->alm_shell_pt[s + 1];
                    if (!conv[s] || j0 == j1) continue;
                    double cmax = 0.0;
                    for (int i = 3 * j0; i < 3 * j1; ++i) cmax = std::max(cmax, std::fabs(h_c[i]));
                    alm_res[s] = cmax;
                    if (cmax <= c->alm_tol) continue;
                    if (outer[s] == c->alm_max_outer) {
                        status[s] = SHELL_E_NOT_CONVERGED;
                        continue;
                    }
                    for (int i = 3 * j0; i < 3 * j1; ++i) c->h_lam[i] -= c->alm_kappa * h_c[i];
                    outer[s]++;
                    kbase[s] += kk[s];
                    kk[s] = 0;
                    status[s] = SHELL_E_NOT_CONVERGED;
                    active[s] = resume[s] = 1;
                    any_resume = true;
                }
                if (any_resume) {   // E and g of the resumed shells with the new multipliers
                    h2d(c, c->alm_lam.p, c->h_lam.data(), c->h_lam.size() * sizeof(double));
                    h2d(c, c->write_shell.p, resume.data(), S * sizeof(int));
                    eval_energy_grad(c, q, qhat, ms, 1, true, g, dptr<int>(c->write_shell));
                    shell_dot(c, g, g, true);
                    sync(c);
                    for (int s = 0; s < S; ++s) {
                        if (!resume[s]) continue;
                        const double* e = c->h_e_shell + 3 * s;
                        E[s] = e[0] + e[1] + e[2];
                        Escale[s] = std::fabs(e[0]) + std::fabs(e[1]) + std::fabs(e[2]);
                        gn[s] = std::sqrt(c->h_red[s]);
                        stats[s].grad_norm = gn[s];
                    }
                }
            }
        }
        bool any = false;
        for (int s = 0; s < S; ++s) any |= active[s] != 0;
        return any;
    };
    // regulariser of the current iteration: delta diag(A) added to the
    // diagonal blocks of a shell, from 1e-6 up by factors of 10 to 1e2
    std::vector<double> delta(S, 0.0);
    auto apply_delta = [&]() {
        h2d(c, c->delta_shell.p, delta.data(), S * sizeof(double));
        launch_regularize(st, c->N, dptr<int>(c->diag_blk), c->vals.p, c->fp32, dptr<double>(c->diag0),
                          dptr<int>(c->node_shell), dptr<double>(c->delta_shell));
    };
    auto bump = [&](int s) -> bool {   // next regulariser value; false past the cap (delta stays 1e2)
        const double next = delta[s] == 0.0 ? 1e-6 : delta[s] * 10.0;
        if (next > 1e2 * (1 + 1e-12)) return false;
        delta[s] = next;
        return true;
    };
    // the shells of `sub` whose block-Jacobi factorisation failed (h_fail):
    // regularise and factor again until every diagonal block is definite
    auto factor_fixup = [&](const std::vector<int>& sub) {
        for (bool first = true;; first = false) {
            if (!first) bj_factor(c);
            bool again = false;
            for (int s = 0; s < S; ++s)
                if (sub[s] && active[s] && c->h_fail[s]) {
                    if (bump(s))
                        again = true;
                    else {
                        status[s] = SHELL_E_INDEFINITE;
                        active[s] = 0;
                    }
                }
            if (!again) break;
            apply_delta();
        }
    };
    // A d = -g for the shells of `todo`, regularising a shell whose CG finds
    // p^T A p <= 0 and solving again for it; `indefinite`: the shells whose
    // last solve found it already (regularise before the first solve)
    auto solve_fixup = [&](std::vector<int> todo, const std::vector<int>& indefinite) {
        bool pre = false;
        for (int s = 0; s < S; ++s)
            if (todo[s] && indefinite[s]) {
                if (bump(s))
                    pre = true;
                else {
                    status[s] = SHELL_E_INDEFINITE;
                    active[s] = 0;
                    todo[s] = 0;
                }
            }
        if (pre) {
            apply_delta();
            bj_factor(c);
        }
        for (;;) {
            bool anyt = false;
            for (int s = 0; s < S; ++s) anyt |= todo[s] != 0;
            if (!anyt) break;
            h2d(c, c->cg_active.p, todo.data(), S * sizeof(int));
            launch_neg_masked(st, c->N, g, dptr<uint16_t>(c->freemask), dptr<int>(c->node_shell),
                              dptr<int>(c->cg_active), rhs);
            SolveResult R = solve(c, rhs, d, todo, std::vector<double>(S, c->opts.pcg_rtol), c->opts.pcg_maxit);
            bool again = false;
            for (int s = 0; s < S; ++s) {
                if (!todo[s]) continue;
                stats[s].pcg_iters_total += R.iters[s];
                stats[s].refine_sweeps += R.sweeps[s];
                if (R.status[s] == 2) {
                    if (bump(s)) {
                        again = true;
                        continue;
                    }
                    status[s] = SHELL_E_INDEFINITE;
                    active[s] = 0;
                }
                todo[s] = 0;
            }
            if (!again) break;
            // regularise the failing shells, refactor, solve again for them
            for (int s = 0; s < S; ++s)
                if (!active[s]) todo[s] = 0;
            apply_delta();
            bj_factor(c);
        }
        // (solve() writes d only for the shells it was asked to solve, so a
        // retry after regularising one shell keeps the others' directions)
    };
    // line search along d for the shells of `sub` (their direction solved):
    // Armijo with quadratic, then cubic interpolation, up to 20 trials;
    // trial0 > 0 continues a search the device began (state in ls_*)
    std::vector<double> ls_slope(S, 0.0), ls_alpha(S, 0.0), ls_aprev(S, 0.0), ls_Eprev(S, 0.0);
    std::vector<int> ls_searching(S, 0);
    auto line_search_start = [&](const std::vector<int>& sub) {
        shell_dot(c, g, d, true);
        sync(c);
        std::vector<int> steepest(S, 0);
        bool any_steep = false;
        for (int s = 0; s < S; ++s) {
            ls_searching[s] = 0;
            if (!(sub[s] && active[s])) continue;
            ls_searching[s] = 1;
            ls_alpha[s] = 1.0;
            ls_slope[s] = c->h_red[s];
            if (!(ls_slope[s] < 0.0)) {   // not a descent direction (an indefinite system the CG did
                steepest[s] = 1;          // not detect): search along -g instead
                ls_slope[s] = -gn[s] * gn[s];
                any_steep = true;
            }
        }
        if (any_steep) {
            h2d(c, c->flag_shell.p, steepest.data(), S * sizeof(int));
            launch_neg_masked(st, c->N, g, dptr<uint16_t>(c->freemask), dptr<int>(c->node_shell),
                              dptr<int>(c->flag_shell), rhs);
            launch_copy_shell(st, c->N, rhs, dptr<int>(c->node_shell), dptr<int>(c->flag_shell), d);
            HIPCHK(hipGetLastError());
        }
    };
    auto line_search = [&](int trial0) {
        std::vector<double>& alpha = ls_alpha;
        std::vector<double>& a_prev = ls_aprev;
        std::vector<double>& E_prev = ls_Eprev;
        std::vector<double>& slope = ls_slope;
        std::vector<int>& searching = ls_searching;
        for (int trial = trial0; trial < 20; ++trial) {
            bool anys = false;
            for (int s = 0; s < S; ++s) anys |= searching[s] != 0;
            if (!anys) break;
            std::vector<double> a_dev(S);
            for (int s = 0; s < S; ++s) a_dev[s] = searching[s] ? alpha[s] : 0.0;
            h2d(c, c->alpha_shell.p, a_dev.data(), S * sizeof(double));
            run_graph(c, c->g_trial, ms, [&] {
                launch_axpy_shell(c->stream, c->N, q, d, dptr<double>(c->alpha_shell), dptr<int>(c->node_shell), qt);
                eval_energy_grad(c, qt, qhat, ms, 1, true, gt, nullptr);
                shell_dot(c, gt, gt, true);
            });
            sync(c);
            std::vector<int> accept(S, 0);
            for (int s = 0; s < S; ++s) {
                if (!searching[s]) continue;
                const double* e = c->h_e_shell + 3 * s;
                const double Et = e[0] + e[1] + e[2];
                const double sc_t = std::fabs(e[0]) + std::fabs(e[1]) + std::fabs(e[2]);
                const double gtn = std::sqrt(c->h_red[s]);
                bool ok = false;
                if (std::isfinite(Et) && std::isfinite(gtn)) {
                    if (Et <= E[s] + 1e-4 * alpha[s] * slope[s]) ok = true;
                    const double noise = 1e-12 * std::max(Escale[s], sc_t);
                    if (-slope[s] <= noise && std::fabs(Et - E[s]) <= noise && gtn < gn[s]) ok = true;
                }
                if (ok) {
                    accept[s] = 1;
                    searching[s] = 0;
                    E[s] = Et;
                    Escale[s] = sc_t;
                    gn[s] = gtn;
                    continue;
                }
                // next step: quadratic fit first, then cubic; clamped to [0.1, 0.5] alpha
                double an;
                const double a = alpha[s];
                if (!std::isfinite(Et)) {
                    an = 0.1 * a;
                } else if (trial == 0) {
                    an = -slope[s] * a * a / (2.0 * (Et - E[s] - slope[s] * a));
                } else {
                    const double ap = a_prev[s];
                    const double d1 = Et - E[s] - slope[s] * a, d2 = E_prev[s] - E[s] - slope[s] * ap;
                    const double den = ap * ap * a * a * (a - ap);
                    const double ca = (ap * ap * d1 - a * a * d2) / den;
                    const double cb = (-ap * ap * ap * d1 + a * a * a * d2) / den;
                    if (ca == 0.0)
                        an = -slope[s] / (2.0 * cb);
                    else {
                        const double disc = cb * cb - 3.0 * ca * slope[s];
                        an = disc >= 0.0 ? (-cb + std::sqrt(disc)) / (3.0 * ca) : 0.5 * a;
                    }
                }
                if (!std::isfinite(an)) an = 0.5 * a;
                an = std::min(std::max(an, 0.1 * a), 0.5 * a);
                a_prev[s] = a;
                E_prev[s] = Et;
                alpha[s] = an;
                stats[s].ls_backtracks++;
            }
            h2d(c, c->flag_shell.p, accept.data(), S * sizeof(int));
            launch_copy_shell(st, c->N, qt, dptr<int>(c->node_shell), dptr<int>(c->flag_shell), q);
            launch_copy_shell(st, c->N, gt, dptr<int>(c->node_shell), dptr<int>(c->flag_shell), g);
        }
    };
    // end of the iteration for the shells of `sub`: count it; a search that
    // found no acceptable step ends the shell's Newton iteration
    auto finish = [&](const std::vector<int>& sub) {
        for (int s = 0; s < S; ++s) {
            if (!sub[s]) continue;
            if (active[s]) stats[s].newton_iters = kbase[s] + (kk[s]++) + 1;
            if (ls_searching[s]) {
                status[s] = SHELL_E_LINESEARCH;
                active[s] = 0;
            }
        }
    };
    // The whole Newton iteration runs as one device launch sequence (one
    // graph) unless the point constraints' outer loop, event timing or the
    // option says otherwise; the host then reads the per-shell state once.
    const bool device_iter = c->opts.device_newton && !c->alm_on && !c->timing;
    bool any = check(false, nullptr);
    while (any) {
        delta.assign(S, 0.0);
        if (device_iter) {
            for (int s = 0; s < S; ++s) {
                NewtonCtl& n = c->h_ctl[s];
                std::memset(&n, 0, sizeof(n));
                n.E = E[s];
                n.Escale = Escale[s];
                n.gn = gn[s];
                n.g0 = g0[s];
                n.floor = floor_[s];
                n.active = active[s];
                n.k = kk[s];
                n.status = status[s];
            }
            h2d(c, c->nt_ctl.p, c->h_ctl, (size_t)S * sizeof(NewtonCtl));
            const double t0 = now_ms();
            run_graph(c, c->g_newton, ms, [&] {
                newton_iteration_device(c, ms, q, g, qt, gt, d, rhs, qhat);
            });
            sync(c);
            t_cg += now_ms() - t0;
            std::vector<int> handed(S, 0), indefinite(S, 0), solve_todo(S, 0), refine(S, 0), ls_more(S, 0),
                fresh_ls(S, 0);
            bool any_handed = false;
            for (int s = 0; s < S; ++s) {
                const NewtonCtl& n = c->h_ctl[s];
                if (n.fault) throw StatusErr{SHELL_E_DEVICE, "CG grid barrier timed out"};
                if (!active[s]) continue;
                stats[s].pcg_iters_total += n.pcg_iters;
                stats[s].refine_sweeps += n.sweeps;
                stats[s].ls_backtracks += n.backtracks;
                E[s] = n.E;
                Escale[s] = n.Escale;
                gn[s] = n.gn;
                if (n.need_host) {
                    handed[s] = 1;
                    any_handed = true;
                    if (n.need_host == NT_HOST_FACTOR) {
                        solve_todo[s] = fresh_ls[s] = 1;
                    } else if (n.need_host == NT_HOST_INDEFINITE) {
                        solve_todo[s] = indefinite[s] = fresh_ls[s] = 1;
                    } else if (n.need_host == NT_HOST_REFINE) {
                        refine[s] = fresh_ls[s] = 1;
                    } else {   // NT_HOST_LINESEARCH
                        ls_more[s] = 1;
                        ls_slope[s] = n.slope;
                        ls_alpha[s] = n.alpha;
                        ls_aprev[s] = n.a_prev;
                        ls_Eprev[s] = n.E_prev;
                    }
                    continue;
                }
                // finished on the device, next convergence test included
                kk[s] = n.k;
                stats[s].newton_iters = kbase[s] + kk[s];
                floor_[s] = n.floor;
                if (n.active) {
                    stats[s].grad_norm = n.grad_norm_checked;
                    stats[s].grad_floor = n.floor;
                } else {
                    stats[s].grad_norm = n.grad_norm_checked;
                    stats[s].grad_floor = n.floor;
                    status[s] = n.status;
                    active[s] = 0;
                }
            }
            if (any_handed) {
                // the rest of this iteration on the host, for the shells the
                // device handed over, then their convergence test
                factor_fixup(solve_todo);
                for (int s = 0; s < S; ++s)
                    if (!active[s]) solve_todo[s] = fresh_ls[s] = 0;
                bool anyr = false;
                for (int s = 0; s < S; ++s) anyr |= refine[s] != 0;
                if (anyr) {
                    // more sweeps of the mixed form from the device's state
                    RefineState F;
                    F.active = refine;
                    F.bn2.assign(S, 0.0);
                    F.prev.assign(S, 1.0);
                    SolveResult R;
                    R.iters.assign(S, 0);
                    R.status.assign(S, 0);
                    R.sweeps.assign(S, 0);
                    R.relres.assign(S, 0.0);
                    for (int s = 0; s < S; ++s)
                        if (refine[s]) {
                            F.bn2[s] = c->h_ctl[s].bn2;
                            F.prev[s] = c->h_ctl[s].prev;
                            R.iters[s] = c->h_ctl[s].solve_iters;
                        }
                    h2d(c, c->cg_active.p, refine.data(), S * sizeof(int));
                    launch_neg_masked(st, c->N, g, dptr<uint16_t>(c->freemask), dptr<int>(c->node_shell),
                                      dptr<int>(c->cg_active), rhs);
                    refine_sweeps(c, rhs, refine, F, std::vector<double>(S, c->opts.pcg_rtol), c->opts.pcg_maxit,
                                  R, NT_REFINE_SWEEPS);
                    h2d(c, c->flag_shell.p, refine.data(), S * sizeof(int));
                    launch_copy_shell(st, c->N, dptr<double>(c->x64), dptr<int>(c->node_shell),
                                      dptr<int>(c->flag_shell), d);
                    HIPCHK(hipGetLastError());
                    for (int s = 0; s < S; ++s) {
                        if (!refine[s]) continue;
                        stats[s].pcg_iters_total += R.iters[s] - c->h_ctl[s].solve_iters;
                        stats[s].refine_sweeps += R.sweeps[s];
                        if (R.status[s] == 2) solve_todo[s] = indefinite[s] = 1;
                    }
                }
                solve_fixup(solve_todo, indefinite);
                for (int s = 0; s < S; ++s) stats[s].reg_delta = std::max(stats[s].reg_delta, delta[s]);
                for (int s = 0; s < S; ++s)
                    if (!active[s]) fresh_ls[s] = 0;
                line_search_start(fresh_ls);
                const std::vector<int> fresh_search = ls_searching;
                // a search the device began continues at its next trial (the
                // interpolation depends on the trial), then the new searches
                std::vector<int> cont_failed(S, 0);
                bool anyc = false;
                for (int s = 0; s < S; ++s) anyc |= ls_more[s] != 0;
                if (anyc) {
                    for (int s = 0; s < S; ++s) ls_searching[s] = ls_more[s] && active[s];
                    line_search(NT_LS_TRIALS);
                    cont_failed = ls_searching;
                }
                ls_searching = fresh_search;
                line_search(0);
                for (int s = 0; s < S; ++s)
                    if (cont_failed[s]) ls_searching[s] = 1;
                finish(handed);
                any = check(true, &handed);
                for (int s = 0; s < S; ++s) any |= active[s] != 0;
            } else {
                any = false;
                for (int s = 0; s < S; ++s) any |= active[s] != 0;
            }
            continue;
        }
        // A = K(q) + M/dt^2, block-Jacobi, regulariser on failure
        double t0 = now_ms();
        run_graph(c, c->g_asm, ms, [&] {
            assemble(c, q, ms, 1);
            if (c->alm_on)   // + kappa C^T C of the point constraints
                launch_add_sparse(c->stream, c->alm_nsp, dptr<long long>(c->alm_pos), dptr<double>(c->alm_val),
                                  c->vals.p, c->fp32);
            launch_save_diag(c->stream, c->N, dptr<int>(c->diag_blk), c->vals.p, c->fp32, dptr<double>(c->diag0));
            bj_factor_enqueue(c);
        });
        sync(c);
        factor_fixup(active);
        t_asm += now_ms() - t0;
        t0 = now_ms();
        // Newton direction: A d = -g
        solve_fixup(active, std::vector<int>(S, 0));
        for (int s = 0; s < S; ++s) stats[s].reg_delta = std::max(stats[s].reg_delta, delta[s]);
        t_cg += now_ms() - t0;
        bool any2 = false;
        for (int s = 0; s < S; ++s) any2 |= active[s] != 0;
        if (!any2) break;
        // line search along d, per shell
        const std::vector<int> iter_shells = active;
        line_search_start(active);
        line_search(0);
        finish(iter_shells);
        any = check(true, nullptr);
    }
    if (learned || c->rec_feat) {
        // this step's correction q_{n+1} - q_start of the converged shells:
        // a training sample (for shells that had a previous correction) and
        // the next step's previous correction
        std::vector<int> ok(S), rec(S);
        for (int s = 0; s < S; ++s) {
            ok[s] = status[s] == SHELL_OK;
            rec[s] = ok[s] && c->h_hist[s];
        }
        h2d(c, c->flag_shell.p, ok.data(), S * sizeof(int));
        double* delta = dptr<double>(c->guess);
        launch_masked_diff(st, c->N, q, dptr<double>(c->qstart), dptr<uint16_t>(c->freemask),
                           dptr<int>(c->node_shell), dptr<int>(c->flag_shell), delta);
        HIPCHK(hipGetLastError());
        record_samples(c, delta, rec);
        h2d(c, c->flag_shell.p, ok.data(), S * sizeof(int));
        launch_copy_shell(st, c->N, delta, dptr<int>(c->node_shell), dptr<int>(c->flag_shell),
                          dptr<double>(c->dstep));
        HIPCHK(hipGetLastError());
        for (int s = 0; s < S; ++s) c->h_hist[s] = (char)ok[s];
    }
    HIPCHK(hipMemcpyAsync(q_np1_dev, q, (size_t)N12 * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_velocity(st, N12, q, q_n_dev, dt, v_np1_dev);
    HIPCHK(hipGetLastError());
    sync(c);
    const double t_step = now_ms() - t_start;
    shell_status worst = SHELL_OK;
    for (int s = 0; s < S; ++s) {
        stats[s].status = status[s];
        stats[s].t_assemble_ms = t_asm;
        stats[s].t_pcg_ms = t_cg;
        stats[s].t_step_ms = t_step;
        stats[s].alm_residual = alm_res[s];
        stats[s].alm_outer = outer[s];
        if (status[s] < worst) worst = status[s];
    }
    if (stats_host) std::memcpy(stats_host, stats.data(), sizeof(shell_step_stats) * S);
    if (worst != SHELL_OK) c->err = "Newton step did not converge for every shell (see stats)";
    return worst;
    API_CATCH
}

// ------------------------------------------------------------ loads
shell_status shell_set_pressure(shell_ctx* c, const double* pressure_host) {
    if (!c) return SHELL_E_INVAL;
    std::vector<double> p(c->S, 0.0);
    bool any = false;
    if (pressure_host)
        for (int s = 0; s < c->S; ++s) {
            if (!std::isfinite(pressure_host[s])) {
                c->err = "pressure not finite";
                return SHELL_E_INVAL;
            }
            p[s] = pressure_host[s];
            any |= p[s] != 0.0;
        }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    if (!c->pressure.p) {
        alloc(c->pressure, (size_t)c->S * sizeof(double));
        alloc(c->fstep, (size_t)c->N * 12 * sizeof(double));
    }
    HIPCHK(hipMemcpyAsync(c->pressure.p, p.data(), (size_t)c->S * sizeof(double), hipMemcpyHostToDevice, c->stream));
    sync(c);
    c->has_pressure = any;
    c->graphs_reset();
    return SHELL_OK;
    API_CATCH
}

shell_status shell_pressure_load(shell_ctx* c, const double* q_dev, double* f_dev) {
    if (!c) return SHELL_E_INVAL;
    if (!q_dev || !f_dev) {
        c->err = "q_dev and f_dev are required";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    if (!c->pressure.p) {
        alloc(c->pressure, (size_t)c->S * sizeof(double));
        alloc(c->fstep, (size_t)c->N * 12 * sizeof(double));
        launch_zero(c->stream, c->pressure.p, c->pressure.n);
    }
    launch_pressure(c->stream, c->P, dptr<int4>(c->patch_nodes), dptr<int>(c->patch_shell),
                    dptr<ShellParams>(c->shells_d), dptr<double>(c->pressure), dptr<double>(c->phi), q_dev,
                    dptr<double>(c->g_patch));
    launch_gather_grad(c->stream, c->N, dptr<int>(c->inc_ptr), dptr<int>(c->inc), dptr<double>(c->g_patch), nullptr,
                       dptr<int>(c->node_shell), nullptr, f_dev);
    HIPCHK(hipGetLastError());
    return SHELL_OK;
    API_CATCH
}

// ------------------------------------------------ point constraints
shell_status shell_set_point_constraints(shell_ctx* c, const shell_point_constraint* pts, int32_t n,
                                         const shell_alm_opts* o) {
    if (!c) return SHELL_E_INVAL;
    if (n < 0 || (n > 0 && pts && !o)) {
        c->err = "n >= 0 and options are required";
        return SHELL_E_INVAL;
    }
    if (!pts) n = 0;
    if (n > 0 && (!(o->penalty > 0) || !std::isfinite(o->penalty) || !(o->tol > 0) || !std::isfinite(o->tol) ||
                  o->max_outer < 0)) {
        c->err = "need penalty > 0, tol > 0 (finite) and max_outer >= 0";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    const int S = c->S;
    std::vector<AlmPoint> ap(n);
    std::vector<int> order(n), spt(S + 1, 0);
    for (int u = 0; u < n; ++u) {
        const shell_point_constraint& pc = pts[u];
        const std::string who = "point constraint " + std::to_string(u) + ": ";
        if (pc.shell < 0 || pc.shell >= S) throw InvalErr{who + "shell index out of range"};
        if (pc.kind < 0 || pc.kind > 2) throw InvalErr{who + "kind must be 0, 1 or 2"};
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(pc.target[k])) throw InvalErr{who + "target not finite"};
        if (!std::isfinite(pc.xi1) || !std::isfinite(pc.xi2)) throw InvalErr{who + "point not finite"};
        spt[pc.shell + 1]++;
    }
    for (int s = 0; s < S; ++s) spt[s + 1] += spt[s];
    {
        std::vector<int> fill(spt.begin(), spt.end() - 1);
        for (int u = 0; u < n; ++u) order[fill[pts[u].shell]++] = u;
    }
    for (int j = 0; j < n; ++j) {
        const shell_point_constraint& pc = pts[order[j]];
        const int s = pc.shell, n1 = c->grid_n1[s], n2 = c->grid_n2[s], per = c->grid_per[s];
        const double d1 = c->shells[s].dxi1, d2 = c->shells[s].dxi2;
        const double L1 = n1 * d1, L2 = n2 * d2;
        double xi1 = pc.xi1;
        if (per) xi1 -= L1 * std::floor(xi1 / L1);
        if (xi1 < 0 || xi1 > L1 || pc.xi2 < 0 || pc.xi2 > L2)
            throw InvalErr{"point constraint " + std::to_string(order[j]) + ": point outside the parameter domain"};
        const int pi = std::min((int)(xi1 / d1), n1 - 1), pj = std::min((int)(pc.xi2 / d2), n2 - 1);
        const double t1 = xi1 / d1 - pi, t2 = pc.xi2 / d2 - pj;
        const int cols = per ? n1 : n1 + 1;
        AlmPoint& a = ap[j];
        for (int cc = 0; cc < 4; ++cc) {
            const int p = cc & 1, qq = cc >> 1;
            int ni = pi + p;
            if (per) ni %= n1;
            a.node[cc] = c->shells[s].node_begin + (pj + qq) * cols + ni;
            for (int k = 0; k < 4; ++k) {
                const int r = k & 1, sk = k >> 1;
                // shape function of corner cc, DOF kind k, differentiated
                // along xi1 (kind 1) or xi2 (kind 2) for a tangent constraint
                const double o1 = pc.kind == 1 ? 1 : 0, o2 = pc.kind == 2 ? 1 : 0;
                a.psi[4 * cc + k] = hermite(p, r, (int)o1, t1) * hermite(qq, sk, (int)o2, t2) *
                                    (r ? d1 : 1.0) * (sk ? d2 : 1.0) / (o1 ? d1 : 1.0) / (o2 ? d2 : 1.0);
            }
        }
        for (int k = 0; k < 3; ++k) a.target[k] = pc.target[k];
    }
    // per node its (constraint, corner) incidences, in constraint order
    std::vector<int> incp(c->N + 1, 0);
    for (int j = 0; j < n; ++j)
        for (int cc = 0; cc < 4; ++cc) incp[ap[j].node[cc] + 1]++;
    for (int i = 0; i < c->N; ++i) incp[i + 1] += incp[i];
    std::vector<int2> inc(incp[c->N]);
    {
        std::vector<int> fill(incp.begin(), incp.end() - 1);
        for (int j = 0; j < n; ++j)
            for (int cc = 0; cc < 4; ++cc) inc[fill[ap[j].node[cc]]++] = make_int2(j, cc);
    }
    // kappa C^T C: kappa psi_I psi_J on each component, merged per stored value
    const double kappa = n > 0 ? o->penalty : 0.0;
    std::map<long long, double> off;
    std::map<int, std::array<double, 144>> dg;
    auto stored = [&](int lo, int hi) {
        const int* b = c->h_ucol.data() + c->h_urow[lo];
        const int* e = c->h_ucol.data() + c->h_urow[lo + 1];
        const int* f = std::lower_bound(b, e, hi);
        if (f == e || *f != hi) throw InvalErr{"point constraint outside the block pattern"};
        return (long long)(f - c->h_ucol.data());
    };
    for (int j = 0; j < n; ++j)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                const int na = ap[j].node[a], nb = ap[j].node[b];
                if (na > nb) continue;   // the stored block of the pair is A_{min, max}
                std::array<double, 144>* D = nullptr;
                long long base = 0;
                if (na == nb) {
                    auto it = dg.find(na);
                    if (it == dg.end()) {
                        std::array<double, 144> z{};
                        it = dg.emplace(na, z).first;
                    }
                    D = &it->second;
                } else {
                    base = stored(na, nb) * 144;
                }
                for (int k = 0; k < 4; ++k)
                    for (int l = 0; l < 4; ++l)
                        for (int comp = 0; comp < 3; ++comp) {
                            const double v = kappa * ap[j].psi[4 * a + k] * ap[j].psi[4 * b + l];
                            const int r = 3 * k + comp, cl = 3 * l + comp;
                            if (D)
                                (*D)[r * 12 + cl] += v;
                            else
                                off[base + r * 12 + cl] += v;
                        }
            }
    for (auto& kv : dg) {
        const long long base = stored(kv.first, kv.first) * 144;
        for (int p = 0; p < SYM12_VALS; ++p) off[base + p] += kv.second[sym12_row(p) * 12 + sym12_col(p)];
    }
    std::vector<long long> pos;
    std::vector<double> val;
    for (auto& kv : off) {
        pos.push_back(kv.first);
        val.push_back(kv.second);
    }
    hipStream_t st = c->stream;
    sync(c);
    upload(c->alm_pts, ap, st);
    upload(c->alm_incp, incp, st);
    upload(c->alm_inc, inc, st);
    upload(c->alm_spt, spt, st);
    upload(c->alm_pos, pos, st);
    upload(c->alm_val, val, st);
    c->h_lam.assign(3 * (size_t)n, 0.0);
    upload(c->alm_lam, c->h_lam, st);
    alloc(c->alm_c, 3 * (size_t)n * sizeof(double));
    sync(c);
    c->alm_n = n;
    c->alm_nsp = (int)pos.size();
    c->alm_kappa = kappa;
    c->alm_tol = n > 0 ? o->tol : 0.0;
    c->alm_max_outer = n > 0 ? o->max_outer : 0;
    c->alm_order = order;
    c->alm_shell_pt = spt;
    c->graphs_reset();
    return SHELL_OK;
    API_CATCH
}

shell_status shell_get_point_multipliers(const shell_ctx* c, double* lambda_host) {
    if (!c || (!lambda_host && c->alm_n > 0)) return SHELL_E_INVAL;
    for (int j = 0; j < c->alm_n; ++j)
        for (int k = 0; k < 3; ++k) lambda_host[3 * (size_t)c->alm_order[j] + k] = c->h_lam[3 * (size_t)j + k];
    return SHELL_OK;
}

shell_status shell_set_point_multipliers(shell_ctx* c, const double* lambda_host) {
    if (!c) return SHELL_E_INVAL;
    if (!lambda_host && c->alm_n > 0) {
        c->err = "lambda_host is required";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    for (int j = 0; j < c->alm_n; ++j)
        for (int k = 0; k < 3; ++k) {
            const double v = lambda_host[3 * (size_t)c->alm_order[j] + k];
            if (!std::isfinite(v)) throw InvalErr{"multiplier not finite"};
            c->h_lam[3 * (size_t)j + k] = v;
        }
    if (c->alm_n > 0) {
        HIPCHK(hipMemcpyAsync(c->alm_lam.p, c->h_lam.data(), c->h_lam.size() * sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
        sync(c);
    }
    return SHELL_OK;
    API_CATCH
}

shell_status shell_set_nodal_forces(shell_ctx* c, const double* f_dev) {
    if (!c) return SHELL_E_INVAL;
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    if (!f_dev) {
        if (c->has_fext) c->graphs_reset();   // the captured evaluations lose the load kernels
        c->has_fext = false;
        return SHELL_OK;
    }
    if (!c->fext.p) alloc(c->fext, (size_t)c->N * 12 * sizeof(double));
    HIPCHK(hipMemcpyAsync(c->fext.p, f_dev, c->fext.n, hipMemcpyDeviceToDevice, c->stream));
    sync(c);
    c->has_fext = true;
    c->graphs_reset();   // the captured evaluations gain the load kernels
    return SHELL_OK;
    API_CATCH
}

shell_status shell_bezier(shell_ctx* c, const double* q_dev, double* ctrl_dev) {
    if (!c) return SHELL_E_INVAL;
    if (!q_dev || !ctrl_dev) {
        c->err = "q_dev and ctrl_dev are required";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    launch_bezier(c->stream, c->P, dptr<int4>(c->patch_nodes), dptr<int>(c->patch_shell),
                  dptr<ShellParams>(c->shells_d), q_dev, ctrl_dev);
    HIPCHK(hipGetLastError());
    return SHELL_OK;
    API_CATCH
}

void shell_ray_default_opts(shell_ray_opts* o) {
    if (!o) return;
    o->eps = 1e-10;
    o->newton_tol = 1e-12;
    o->hole = 1e-3;
    o->newton_iters = 8;
    o->max_depth = RAY_MAX_DEPTH;
    o->heap_cap = RAY_HEAP_MAX;
    o->device = 0;
    o->stream = nullptr;
}

}  // extern "C"

namespace {

// shell_ray_cast and shell_ray_cast_noalloc: the same validation and
// kernels; `noalloc` hands rays over to the cooperative search through the
// library's fixed device buffer instead of a stream-ordered allocation.
shell_status ray_cast_impl(const double* ctrl_dev, int32_t n_patches, const double* rays_dev, int64_t n_rays,
                           const shell_ray_opts* o, double* hit_dev, int32_t* patch_dev, int32_t* pops_dev,
                           bool noalloc) {
    static_assert(SHELL_RAY_HEAP_MAX == RAY_HEAP_MAX, "heap size of the ABI and of the kernel");
    static_assert(SHELL_RAY_NOALLOC_TAIL_RAYS == RAY_TAIL_STATIC_SLOTS, "fixed hand-over buffer of ABI and kernel");
    g_create_error.clear();
    auto bad = [](const char* m) {
        g_create_error = m;
        return SHELL_E_INVAL;
    };
    if (!o) return bad("opts is required");
    if (n_patches < 0 || n_patches > RAY_MAX_PATCHES) return bad("n_patches must be in [0, 2^24)");
    if (n_rays < 0 || n_rays > (int64_t)256 * INT32_MAX) return bad("n_rays out of range");
    if (n_rays == 0) return SHELL_OK;
    if (!rays_dev || !hit_dev || !patch_dev || (n_patches > 0 && !ctrl_dev))
        return bad("rays_dev, hit_dev, patch_dev and (with patches) ctrl_dev are required");
    if (!(o->eps > 0) || !std::isfinite(o->eps)) return bad("eps must be > 0");
    if (!(o->newton_tol > 0) || !std::isfinite(o->newton_tol)) return bad("newton_tol must be > 0");
    if (!(o->hole > 0 && o->hole < 0.5)) return bad("hole must be in (0, 0.5)");
    if (o->newton_iters < 0 || o->newton_iters > 64) return bad("newton_iters must be in [0, 64]");
    if (o->max_depth < 1 || o->max_depth > RAY_MAX_DEPTH) return bad("max_depth must be in [1, 60]");
    if (o->heap_cap < 1 || o->heap_cap > RAY_HEAP_MAX) return bad("heap_cap must be in [1, SHELL_RAY_HEAP_MAX]");
    hipError_t e = hipSetDevice(o->device);
    void* fixed_tail = nullptr;
    if (e == hipSuccess && noalloc) e = ray_scratch_address(o->device, &fixed_tail);
    if (e == hipSuccess) {
        RayParams rp{o->eps, o->newton_tol, o->hole, o->newton_iters, o->max_depth, o->heap_cap};
        launch_ray_cast((hipStream_t)o->stream, ctrl_dev, n_patches, rays_dev, n_rays, rp, hit_dev, patch_dev,
                        pops_dev, fixed_tail);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        g_create_error = std::string("HIP error in ") + (noalloc ? "shell_ray_cast_noalloc: " : "shell_ray_cast: ") +
                         hipGetErrorString(e);
        return SHELL_E_DEVICE;
    }
    return SHELL_OK;
}

}  // namespace

extern "C" {

shell_status shell_ray_cast(const double* ctrl_dev, int32_t n_patches, const double* rays_dev, int64_t n_rays,
                            const shell_ray_opts* o, double* hit_dev, int32_t* patch_dev, int32_t* pops_dev) {
    return ray_cast_impl(ctrl_dev, n_patches, rays_dev, n_rays, o, hit_dev, patch_dev, pops_dev, false);
}

shell_status shell_ray_cast_noalloc(const double* ctrl_dev, int32_t n_patches, const double* rays_dev,
                                    int64_t n_rays, const shell_ray_opts* o, double* hit_dev, int32_t* patch_dev,
                                    int32_t* pops_dev) {
    return ray_cast_impl(ctrl_dev, n_patches, rays_dev, n_rays, o, hit_dev, patch_dev, pops_dev, true);
}

shell_status shell_ccd(const double* ctrl_dev, const double* vel_dev, int32_t n_patches, const double* points_dev,
                       int64_t n_points, double dt, const shell_ray_opts* o, double* hit_dev, int32_t* patch_dev,
                       int32_t* pops_dev) {
    g_create_error.clear();
    auto bad = [](const char* m) {
        g_create_error = m;
        return SHELL_E_INVAL;
    };
    if (!o) return bad("opts is required");
    if (n_patches < 0 || n_patches > RAY_MAX_PATCHES) return bad("n_patches must be in [0, 2^24)");
    if (n_points < 0 || n_points > (int64_t)256 * INT32_MAX) return bad("n_points out of range");
    if (!(dt > 0) || !std::isfinite(dt)) return bad("dt must be > 0");
    if (n_points == 0) return SHELL_OK;
    if (!points_dev || !hit_dev || !patch_dev || (n_patches > 0 && (!ctrl_dev || !vel_dev)))
        return bad("points_dev, hit_dev, patch_dev and (with patches) ctrl_dev and vel_dev are required");
    if (!(o->eps > 0) || !std::isfinite(o->eps)) return bad("eps must be > 0");
    if (!(o->newton_tol > 0) || !std::isfinite(o->newton_tol)) return bad("newton_tol must be > 0");
    if (!(o->hole > 0 && o->hole < 0.5)) return bad("hole must be in (0, 0.5)");
    if (o->newton_iters < 0 || o->newton_iters > 64) return bad("newton_iters must be in [0, 64]");
    if (o->max_depth < 1 || o->max_depth > RAY_MAX_DEPTH) return bad("max_depth must be in [1, 60]");
    if (o->heap_cap < 1 || o->heap_cap > RAY_HEAP_MAX) return bad("heap_cap must be in [1, SHELL_RAY_HEAP_MAX]");
    hipError_t e = hipSetDevice(o->device);
    if (e == hipSuccess) {
        RayParams rp{o->eps, o->newton_tol, o->hole, o->newton_iters, o->max_depth, o->heap_cap};
        launch_ccd((hipStream_t)o->stream, ctrl_dev, vel_dev, n_patches, points_dev, n_points, dt, rp, hit_dev,
                   patch_dev, pops_dev);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        g_create_error = std::string("HIP error in shell_ccd: ") + hipGetErrorString(e);
        return SHELL_E_DEVICE;
    }
    return SHELL_OK;
}

void shell_collide_default_opts(shell_collide_opts* o) {
    if (!o) return;
    o->samples = 3;
    o->friction = 0.0;
    o->push_out = 1e-4;
    o->simultaneous = 1e-3;
    o->rtol = 1e-12;
}

}  // extern "C"

namespace {

// Minimum-norm solution of (J M^-1 J^T) lam = b by CG on the host over the
// nrow constraint rows, each product on the device: J^T p as nodal forces
// (scatter), M^-1 by the context's block-Jacobi CG on the mass matrix
// (prescribed DOFs masked), J back (gather).  Returns the iterations; lam
// and the nodal M^-1 J^T lam (in dq) hold the result.
// dq = M^-1 J^T x (nodal; 0 on prescribed DOFs) for the nrow rows of x;
// with Sx, also Sx = J dq.  M^-1 by the context's CG on the mass matrix.
void coll_minv_jt(shell_ctx* c, int ncon, int m, int nrow, const std::vector<double>& x, double* dq,
                  std::vector<double>* Sx) {
    hipStream_t st = c->stream;
    double* lam_dev = dptr<double>(c->coll_lam);
    double* y = dptr<double>(c->rhs);
    HIPCHK(hipMemcpyAsync(lam_dev, x.data(), nrow * sizeof(double), hipMemcpyHostToDevice, st));
    launch_coll_scatter(st, c->N, dptr<int>(c->coll_incp), dptr<int2>(c->coll_inc), dptr<CollContact>(c->coll_con),
                        dptr<int>(c->coll_rowof), m, lam_dev, dptr<uint16_t>(c->freemask), y);
    HIPCHK(hipGetLastError());
    SolveResult R = solve(c, y, dq, std::vector<int>(c->S, 1), std::vector<double>(c->S, 1e-13), c->opts.pcg_maxit);
    for (int s = 0; s < c->S; ++s)
        if (R.status[s] == 2) throw StatusErr{SHELL_E_INDEFINITE, "mass matrix not positive definite"};
    if (Sx) {
        launch_coll_gather(st, ncon, dptr<CollContact>(c->coll_con), dptr<int>(c->coll_rowof), m, dq,
                           dptr<double>(c->coll_out));
        HIPCHK(hipGetLastError());
        Sx->resize(nrow);
        HIPCHK(hipMemcpyAsync(Sx->data(), c->coll_out.p, nrow * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    sync(c);
}

int coll_cg(shell_ctx* c, int ncon, int m, int nrow, const std::vector<double>& b, double rtol, double* dq,
            std::vector<double>& lam) {
    auto apply = [&](const std::vector<double>& x, std::vector<double>* Sx) {
        coll_minv_jt(c, ncon, m, nrow, x, dq, Sx);
    };
    auto dotv = [&](const std::vector<double>& a, const std::vector<double>& bb) {
        double t = 0.0;
        for (int i = 0; i < nrow; ++i) t += a[i] * bb[i];
        return t;
    };
    lam.assign(nrow, 0.0);
    std::vector<double> r = b, p = b, Sp;
    double rr = dotv(r, r);
    const double bn = std::sqrt(rr);
    int it = 0;
    if (bn > 0.0)
        for (; it < nrow + 50; ++it) {
            if (std::sqrt(rr) <= rtol * bn) break;
            apply(p, &Sp);
            const double pSp = dotv(p, Sp);
            if (!(pSp > 0.0)) break;
            const double al = rr / pSp;
            for (int i = 0; i < nrow; ++i) {
                lam[i] += al * p[i];
                r[i] -= al * Sp[i];
            }
            const double rr2 = dotv(r, r);
            const double be = rr2 / rr;
            rr = rr2;
            for (int i = 0; i < nrow; ++i) p[i] = r[i] + be * p[i];
        }
    apply(lam, nullptr);   // dq = M^-1 J^T lam
    return it;
}

}  // namespace

extern "C" {

shell_status shell_collide(shell_ctx* c, double dt, const double* q_n_dev, const double* q_np1_dev,
                           const double* v_dev, const shell_collider* colliders, int32_t n_colliders,
                           const shell_collide_opts* o, double* q_out_dev, double* v_out_dev,
                           shell_collide_stats* stats_host) {
    if (!c) return SHELL_E_INVAL;
    shell_collide_opts dflt;
    shell_collide_default_opts(&dflt);
    if (!o) o = &dflt;
    if (!(dt > 0) || !std::isfinite(dt) || !q_n_dev || !q_np1_dev || !v_dev || !q_out_dev || !v_out_dev ||
        n_colliders < 0 || (n_colliders > 0 && !colliders)) {
        c->err = "dt > 0, q_n, q_np1, v, q_out, v_out and the colliders are required";
        return SHELL_E_INVAL;
    }
    if (q_out_dev == q_n_dev || q_out_dev == q_np1_dev || q_out_dev == v_dev || v_out_dev == v_dev ||
        v_out_dev == q_n_dev || v_out_dev == q_np1_dev || v_out_dev == q_out_dev) {
        c->err = "outputs may not alias inputs or each other";
        return SHELL_E_INVAL;
    }
    if (o->samples < 1 || o->samples > 16 || !(o->friction >= 0) || !std::isfinite(o->friction) ||
        !(o->push_out >= 0) || !std::isfinite(o->push_out) || !(o->simultaneous >= 0) ||
        !std::isfinite(o->simultaneous) || !(o->rtol > 0 && o->rtol < 1)) {
        c->err = "samples in [1, 16], friction >= 0, push_out >= 0, simultaneous >= 0, rtol in (0, 1)";
        return SHELL_E_INVAL;
    }
    std::vector<CollCollider> cols(n_colliders);
    for (int k = 0; k < n_colliders; ++k) {
        const shell_collider& sc = colliders[k];
        CollCollider& cc = cols[k];
        cc.kind = sc.kind;
        for (int i = 0; i < 3; ++i) {
            cc.p[i] = sc.point[i];
            cc.n[i] = sc.normal[i];
        }
        cc.r = sc.radius;
        bool ok = (sc.kind == SHELL_COLLIDER_PLANE || sc.kind == SHELL_COLLIDER_SPHERE) && std::isfinite(sc.point[0]) &&
                  std::isfinite(sc.point[1]) && std::isfinite(sc.point[2]);
        if (ok && sc.kind == SHELL_COLLIDER_PLANE) {
            const double l = std::sqrt(cc.n[0] * cc.n[0] + cc.n[1] * cc.n[1] + cc.n[2] * cc.n[2]);
            ok = l > 0 && std::isfinite(l);
            for (int i = 0; i < 3 && ok; ++i) cc.n[i] /= l;
        }
        if (ok && sc.kind == SHELL_COLLIDER_SPHERE) ok = sc.radius > 0 && std::isfinite(sc.radius);
        if (!ok) {
            c->err = "collider " + std::to_string(k) + ": a plane needs a finite point and non-zero normal, a sphere "
                     "a finite centre and radius > 0";
            return SHELL_E_INVAL;
        }
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    hipStream_t st = c->stream;
    const int s = o->samples, N12 = c->N * 12;
    const int nsamp = c->P * s * s;
    const int nblk = (nsamp + 255) / 256;
    shell_collide_stats stt;
    std::memset(&stt, 0, sizeof(stt));
    stt.t_contact = INFINITY;
    auto pass_through = [&]() {
        HIPCHK(hipMemcpyAsync(q_out_dev, q_np1_dev, (size_t)N12 * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(v_out_dev, v_dev, (size_t)N12 * sizeof(double), hipMemcpyDeviceToDevice, st));
        sync(c);
    };
    if (nsamp == 0 || n_colliders == 0) {
        pass_through();
        if (stats_host) *stats_host = stt;
        return SHELL_OK;
    }
    if (c->coll_tc.n < (size_t)nsamp * sizeof(double)) {
        alloc(c->coll_tc, (size_t)nsamp * sizeof(double));
        alloc(c->coll_cid, (size_t)nsamp * sizeof(int));
        alloc(c->coll_list, (size_t)nsamp * sizeof(int));
        alloc(c->coll_blk, (size_t)nblk * sizeof(double));
        alloc(c->coll_cnt, (size_t)nblk * sizeof(int));
    }
    if (c->coll_cols.n < cols.size() * sizeof(CollCollider)) alloc(c->coll_cols, cols.size() * sizeof(CollCollider));
    HIPCHK(hipMemcpyAsync(c->coll_cols.p, cols.data(), cols.size() * sizeof(CollCollider), hipMemcpyHostToDevice, st));
    // 1-2: samples, earliest contact
    launch_coll_samples(st, nsamp, s, dptr<int4>(c->patch_nodes), dptr<int>(c->patch_shell),
                        dptr<ShellParams>(c->shells_d), q_n_dev, q_np1_dev, dt, dptr<CollCollider>(c->coll_cols),
                        n_colliders, dptr<double>(c->coll_tc), dptr<int>(c->coll_cid), dptr<double>(c->coll_blk));
    HIPCHK(hipGetLastError());
    std::vector<double> bmin(nblk);
    HIPCHK(hipMemcpyAsync(bmin.data(), c->coll_blk.p, nblk * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(c);
    double tstar = INFINITY;
    for (double v : bmin) tstar = std::min(tstar, v);
    if (!std::isfinite(tstar)) {
        pass_through();
        if (stats_host) *stats_host = stt;
        return SHELL_OK;
    }
    stt.t_contact = tstar;
    // 3: rollback, the earliest simultaneous contacts in sample order
    double* qs = dptr<double>(c->qt);
    launch_coll_rollback(st, N12, q_n_dev, q_np1_dev, tstar / dt, qs);
    const double thr = tstar + o->simultaneous * dt;
    launch_coll_count(st, nsamp, dptr<double>(c->coll_tc), thr, dptr<int>(c->coll_cnt));
    std::vector<int> cnt(nblk), off(nblk);
    HIPCHK(hipMemcpyAsync(cnt.data(), c->coll_cnt.p, nblk * sizeof(int), hipMemcpyDeviceToHost, st));
    sync(c);
    int K = 0;
    for (int b = 0; b < nblk; ++b) {
        off[b] = K;
        K += cnt[b];
    }
    h2d(c, c->coll_cnt.p, off.data(), nblk * sizeof(int));
    launch_coll_compact(st, nsamp, dptr<double>(c->coll_tc), thr, dptr<int>(c->coll_cnt), dptr<int>(c->coll_list));
    if (c->coll_con.n < (size_t)K * sizeof(CollContact)) {
        alloc(c->coll_con, (size_t)K * sizeof(CollContact));
        alloc(c->coll_rowof, (size_t)K * sizeof(int));
        alloc(c->coll_lam, (size_t)K * 3 * sizeof(double));
        alloc(c->coll_out, (size_t)K * 3 * sizeof(double));
    }
    launch_coll_setup(st, K, s, dptr<int>(c->coll_list), dptr<int>(c->coll_cid), dptr<int4>(c->patch_nodes),
                      dptr<int>(c->patch_shell), dptr<ShellParams>(c->shells_d), qs, v_dev,
                      dptr<CollCollider>(c->coll_cols), dptr<CollContact>(c->coll_con));
    HIPCHK(hipGetLastError());
    std::vector<CollContact> con(K);
    HIPCHK(hipMemcpyAsync(con.data(), c->coll_con.p, (size_t)K * sizeof(CollContact), hipMemcpyDeviceToHost, st));
    sync(c);
    stt.contacts = K;
    // node incidences of the contacts (contact order within every node)
    std::vector<int> incp(c->N + 1, 0);
    for (const auto& ct : con)
        for (int cc = 0; cc < 4; ++cc) incp[ct.node[cc] + 1]++;
    for (int n = 0; n < c->N; ++n) incp[n + 1] += incp[n];
    std::vector<int2> inc(std::max(incp[c->N], 1));
    {
        std::vector<int> fill(incp.begin(), incp.end() - 1);
        for (int j = 0; j < K; ++j)
            for (int cc = 0; cc < 4; ++cc) inc[fill[con[j].node[cc]]++] = make_int2(j, cc);
    }
    upload(c->coll_incp, incp, st);
    upload(c->coll_inc, inc, st);
    // the mass matrix (and its block-Jacobi factors) in the context's matrix
    assemble(c, qs, 1.0, 0);
    bj_factor(c);
    for (int sh = 0; sh < c->S; ++sh)
        if (c->h_fail[sh]) throw StatusErr{SHELL_E_INDEFINITE, "mass matrix block not positive definite"};
    // 4: impulses on the approaching contacts, zero restitution (+ friction)
    const int m = o->friction > 0.0 ? 3 : 1;
    std::vector<int> rowof(K, -1);
    int na = 0;
    for (int j = 0; j < K; ++j)
        if (con[j].vn < 0.0) rowof[j] = m * na++;
    stt.approaching = na;
    double* dq = dptr<double>(c->dvec);
    HIPCHK(hipMemcpyAsync(v_out_dev, v_dev, (size_t)N12 * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (na > 0) {
        upload(c->coll_rowof, rowof, st);
        std::vector<double> bv(m * na);
        // -J v: gathered on the device from v
        launch_coll_gather(st, K, dptr<CollContact>(c->coll_con), dptr<int>(c->coll_rowof), m, v_dev,
                           dptr<double>(c->coll_out));
        HIPCHK(hipMemcpyAsync(bv.data(), c->coll_out.p, bv.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        sync(c);
        for (double& x : bv) x = -x;
        std::vector<double> lam;
        stt.impulse_iters = coll_cg(c, K, m, m * na, bv, o->rtol, dq, lam);
        if (m == 3) {
            // Coulomb cone: |lambda_t| <= mu lambda_n, none when lambda_n <= 0
            for (int a = 0; a < na; ++a) {
                double* l = lam.data() + 3 * a;
                const double nt = std::sqrt(l[1] * l[1] + l[2] * l[2]);
                if (l[0] <= 0.0) {
                    l[1] = l[2] = 0.0;
                } else if (nt > o->friction * l[0]) {
                    l[1] *= o->friction * l[0] / nt;
                    l[2] *= o->friction * l[0] / nt;
                }
            }
            coll_minv_jt(c, K, m, m * na, lam, dq, nullptr);   // dq for the clamped impulses
        }
        launch_add_to<double>(st, N12, dq, v_out_dev);
        HIPCHK(hipGetLastError());
    }
    // 5: push-out of every resolved contact along its normal
    for (int j = 0; j < K; ++j) rowof[j] = j;
    upload(c->coll_rowof, rowof, st);
    std::vector<double> bp(K);
    for (int j = 0; j < K; ++j) {
        const CollContact& ct = con[j];
        double d = 0.0;
        for (int i = 0; i < 3; ++i) d += ct.dir[0][i] * (ct.x[i] - ct.p[i]);
        bp[j] = o->push_out - d;
    }
    std::vector<double> mu;
    stt.push_iters = coll_cg(c, K, 1, K, bp, o->rtol, dq, mu);
    HIPCHK(hipMemcpyAsync(q_out_dev, qs, (size_t)N12 * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_add_to<double>(st, N12, dq, q_out_dev);
    HIPCHK(hipGetLastError());
    sync(c);
    if (stats_host) *stats_host = stt;
    return SHELL_OK;
    API_CATCH
}

shell_status shell_point_load(const shell_desc* d, double xi1, double xi2, const double* force, double* f_nodal) {
    if (!d || !force || !f_nodal || d->n1 < 1 || d->n2 < 1 || !(d->dxi1 > 0) || !(d->dxi2 > 0) ||
        (d->periodic1 && d->n1 < 3) || !std::isfinite(xi1) || !std::isfinite(xi2))
        return SHELL_E_INVAL;
    const double L1 = d->n1 * d->dxi1, L2 = d->n2 * d->dxi2;
    if (d->periodic1) xi1 -= L1 * std::floor(xi1 / L1);
    if (xi1 < 0 || xi1 > L1 || xi2 < 0 || xi2 > L2) return SHELL_E_INVAL;
    const int i = std::min((int)(xi1 / d->dxi1), d->n1 - 1), j = std::min((int)(xi2 / d->dxi2), d->n2 - 1);
    const double t1 = xi1 / d->dxi1 - i, t2 = xi2 / d->dxi2 - j;
    const int cols = d->periodic1 ? d->n1 : d->n1 + 1;
    for (int c = 0; c < 4; ++c) {
        const int p = c & 1, q = c >> 1;
        int ni = i + p;
        if (d->periodic1) ni %= d->n1;
        const int node = (j + q) * cols + ni;
        for (int k = 0; k < 4; ++k) {
            const int r = k & 1, s = k >> 1;
            // value of the shape function of corner c, kind k (derivative DOFs
            // are xi-derivatives, hence the dxi powers)
            const double phi = hermite(p, r, 0, t1) * hermite(q, s, 0, t2) * (r ? d->dxi1 : 1.0) *
                               (s ? d->dxi2 : 1.0);
            for (int comp = 0; comp < 3; ++comp) f_nodal[(size_t)node * 12 + 3 * k + comp] += phi * force[comp];
        }
    }
    return SHELL_OK;
}

// ------------------------------------------------------------ autotuner
namespace {
struct TuneKey {
    int device, N, S, fp32;
    long long nnzb;
    bool operator<(const TuneKey& o) const {
        return std::tie(device, N, S, fp32, nnzb) < std::tie(o.device, o.N, o.S, o.fp32, o.nnzb);
    }
};
struct TuneChoice {
    int threads, spread;   // CG layout
    int hs_waves, eg_patches;   // patch kernel tiles
};
std::mutex g_tune_mutex;
std::map<TuneKey, TuneChoice> g_tune_cache;

// Wall time per CG iteration of the current layout: `iters` iterations of
// every shell on b (tolerance 0), second of two runs.
double time_cg(shell_ctx* c, const double* b, int iters) {
    const std::vector<int> act(c->S, 1);
    const std::vector<double> rt(c->S, 0.0);
    double best = 0.0;
    for (int rep = 0; rep < 2; ++rep) {
        const double t0 = now_ms();
        cg_launch(c, b, act, rt, iters);
        best = now_ms() - t0;
    }
    long long mx = 1;
    for (int s = 0; s < c->S; ++s) mx = std::max<long long>(mx, c->h_cg_out[s].iters);
    return 1e3 * best / (double)mx;
}
}  // namespace

shell_status shell_set_patch_tiles(shell_ctx* c, int32_t hess_waves, int32_t energy_patches) {
    if (!c) return SHELL_E_INVAL;
    if (!(hess_waves == 4 || hess_waves == 8) || !(energy_patches == 4 || energy_patches == 8 || energy_patches == 16)) {
        c->err = "hess_waves must be 4 or 8 and energy_patches 4, 8 or 16";
        return SHELL_E_INVAL;
    }
    c->hs_waves = hess_waves;
    c->eg_patches = energy_patches;
    c->graphs_reset();   // the captured sequences hold the launch shapes
    return SHELL_OK;
}

shell_status shell_set_assembly(shell_ctx* c, int32_t single_launch) {
    if (!c) return SHELL_E_INVAL;
    if (single_launch && !c->asm_eligible) {
        c->err = "the single-launch assembly needs every patch's Hessian block resident at once";
        return SHELL_E_INVAL;
    }
    c->asm_gather = single_launch != 0;
    c->graphs_reset();   // the captured assembly holds its launches
    return SHELL_OK;
}

shell_status shell_autotune(shell_ctx* c, int32_t cg_iters, shell_tune_result* out) {
    if (!c) return SHELL_E_INVAL;
    if (cg_iters < 1) {
        c->err = "cg_iters must be >= 1";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    shell_tune_result r;
    std::memset(&r, 0, sizeof(r));
    const TuneKey key{c->opts.device, c->N, c->S, (int)c->fp32, c->nnzb};
    bool cached = false;
    TuneChoice choice{c->cg_threads, 1, c->hs_waves, c->eg_patches};
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            choice = it->second;
            cached = true;
        }
    }
    // operator: K(qbar) + M (symmetric positive definite on the free DOFs)
    // and a smooth right-hand side; only the time per iteration matters
    const bool timing = c->timing;
    c->timing = false;
    assemble(c, dptr<double>(c->qbar), 1.0, 1);
    bj_factor(c);
    std::vector<double> ones((size_t)c->N * 12);
    for (int n = 0; n < c->N; ++n)
        for (int w = 0; w < 12; ++w) ones[(size_t)n * 12 + w] = ((c->h_freemask[n] >> w) & 1) ? 1.0 : 0.0;
    h2d(c, c->rhs.p, ones.data(), ones.size() * sizeof(double));
    sync(c);
    const int nt0 = c->cg_threads, target0 = c->cg_rows_target;
    r.us_per_iter_default = time_cg(c, dptr<double>(c->rhs), cg_iters);
    // patch kernel tiles: wall time of one assembly (Hessian kernels of all
    // colours) and of one energy and gradient evaluation, best of three
    auto time_best = [&](auto&& f) {
        double best = 1e300;
        for (int rep = 0; rep < 4; ++rep) {
            const double t0 = now_ms();
            f();
            sync(c);
            if (rep > 0) best = std::min(best, now_ms() - t0);
        }
        return 1e3 * best;
    };
    double* qb = dptr<double>(c->qbar);
    auto t_hess = [&] { return time_best([&] { assemble(c, qb, 1.0, 1); }); };
    auto t_eg = [&] { return time_best([&] { eval_energy_grad(c, qb, qb, 1.0, 1, true, dptr<double>(c->gt), nullptr); }); };
    r.hess_us_default = t_hess();
    r.energy_us_default = t_eg();
    if (!cached) {
        double best = 1e300;
        int max_rows = 0;
        for (int s = 0; s < c->S; ++s) max_rows = std::max(max_rows, c->shells[s].node_end - c->shells[s].node_begin);
        for (int nt : {256, 512, 1024})
            for (int spread : {-1, 0, 1, 2, 4}) {
                // one block per shell only where a block covers the largest
                // shell in two passes
                if (spread < 0 && max_rows > 2 * cg_rows_per_pass(c->fp32, nt)) continue;
                if (!set_row_blocks(c, nt, spread)) continue;
                const double t = time_cg(c, dptr<double>(c->rhs), cg_iters);
                r.candidates++;
                if (t < best) {
                    best = t;
                    choice.threads = nt;
                    choice.spread = spread;
                }
            }
        double bh = 1e300, be = 1e300;
        for (int w : {4, 8}) {
            c->hs_waves = w;
            const double t = t_hess();
            if (t < bh) {
                bh = t;
                choice.hs_waves = w;
            }
        }
        for (int p : {4, 8, 16}) {
            c->eg_patches = p;
            const double t = t_eg();
            if (t < be) {
                be = t;
                choice.eg_patches = p;
            }
        }
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        g_tune_cache[key] = choice;
    }
    c->hs_waves = choice.hs_waves;
    c->eg_patches = choice.eg_patches;
    r.hess_us = t_hess();
    r.energy_us = t_eg();
    r.hess_waves = c->hs_waves;
    r.energy_patches = c->eg_patches;
    if (!set_row_blocks(c, choice.threads, choice.spread)) throw StatusErr{SHELL_E_DEVICE, "autotuned layout lost"};
    r.us_per_iter = time_cg(c, dptr<double>(c->rhs), cg_iters);
    r.threads = c->cg_threads;
    r.rows_per_block = c->cg_rows_target;
    r.blocks = c->nblk;
    r.from_cache = cached ? 1 : 0;
    r.default_threads = nt0;
    r.default_rows_per_block = target0;
    c->timing = timing;
    if (out) *out = r;
    return SHELL_OK;
    API_CATCH
}

shell_status shell_timing_enable(shell_ctx* c, int32_t enable) {
    if (!c) return SHELL_E_INVAL;
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    if (!c->ev0) {
        HIPCHK(hipEventCreate(&c->ev0));
        HIPCHK(hipEventCreate(&c->ev1));
    }
    std::memset(&c->tm, 0, sizeof(c->tm));
    c->timing = enable != 0;
    return SHELL_OK;
    API_CATCH
}

shell_status shell_timing_get(const shell_ctx* c, shell_timing* out) {
    if (!c || !out) return SHELL_E_INVAL;
    *out = c->tm;
    return SHELL_OK;
}

shell_status shell_cg_trace_enable(shell_ctx* c, int32_t enable) {
    if (!c) return SHELL_E_INVAL;
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    sync(c);
    c->cg_tracing = enable != 0;
    if (c->cg_tracing) alloc(c->cg_trace, (size_t)c->nblk * CG_TRACE_ITERS * 6 * sizeof(unsigned long long));
    c->graphs_reset();   // the captured CG launches hold the trace pointer
    return SHELL_OK;
    API_CATCH
}

shell_status shell_cg_trace_get(shell_ctx* c, int32_t* nblocks, int32_t* iters, uint64_t* ts_host) {
    if (!c) return SHELL_E_INVAL;
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    sync(c);
    const size_t n = (size_t)c->nblk * CG_TRACE_ITERS * 6;
    if (nblocks) *nblocks = c->nblk;
    if (iters) *iters = CG_TRACE_ITERS;
    if (ts_host) {
        if (!c->cg_tracing || c->cg_trace.n < n * sizeof(unsigned long long)) {
            std::memset(ts_host, 0, n * sizeof(uint64_t));
        } else {
            HIPCHK(hipMemcpy(ts_host, c->cg_trace.p, n * sizeof(uint64_t), hipMemcpyDeviceToHost));
        }
    }
    return SHELL_OK;
    API_CATCH
}

// ------------------------------------------------------- warm-start network
static_assert(SHELL_MLP_PARAMS == MLP_NPARAMS && SHELL_MLP_IN == MLP_IN && SHELL_MLP_OUT == MLP_OUT &&
                  SHELL_MLP_HIDDEN == MLP_H,
              "network sizes");

shell_status shell_mlp_set_params(shell_ctx* c, const float* theta_host) {
    if (!c) return SHELL_E_INVAL;
    if (!theta_host) {
        c->err = "theta_host is NULL";
        return SHELL_E_INVAL;
    }
    for (int i = 0; i < MLP_NPARAMS; ++i)
        if (!std::isfinite(theta_host[i])) {
            c->err = "non-finite network parameter " + std::to_string(i);
            return SHELL_E_NONFINITE;
        }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    mlp_alloc(c);
    h2d(c, c->mlp_theta.p, theta_host, MLP_NPARAMS * sizeof(float));
    HIPCHK(hipMemsetAsync(c->mlp_m.p, 0, c->mlp_m.n, c->stream));
    HIPCHK(hipMemsetAsync(c->mlp_v.p, 0, c->mlp_v.n, c->stream));
    launch_mlp_pack(c->stream, dptr<float>(c->mlp_theta), c->mlp_w.p);
    HIPCHK(hipGetLastError());
    sync(c);
    c->adam_step = 0;
    c->mlp_ready = true;
    return SHELL_OK;
    API_CATCH
}

shell_status shell_mlp_get_params(shell_ctx* c, float* theta_host) {
    if (!c) return SHELL_E_INVAL;
    if (!theta_host || !c->mlp_ready) {
        c->err = "theta_host is NULL or no parameters are loaded";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    HIPCHK(hipMemcpyAsync(theta_host, c->mlp_theta.p, MLP_NPARAMS * sizeof(float), hipMemcpyDeviceToHost,
                          c->stream));
    sync(c);
    return SHELL_OK;
    API_CATCH
}

shell_status shell_mlp_forward(shell_ctx* c, const float* feat_dev, float* out_dev, int64_t n) {
    if (!c) return SHELL_E_INVAL;
    if (!c->mlp_ready || n < 0 || (n > 0 && (!feat_dev || !out_dev))) {
        c->err = "needs loaded parameters, n >= 0 and device arrays";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    if (n > 0) launch_mlp_forward(c->stream, dptr<float>(c->mlp_theta), c->mlp_w.p, feat_dev, out_dev, n);
    HIPCHK(hipGetLastError());
    sync(c);
    return SHELL_OK;
    API_CATCH
}

shell_status shell_mlp_loss_grad(shell_ctx* c, const float* feat_dev, const float* tgt_dev, int64_t n_samples,
                                 const int64_t* idx_dev, int32_t batch, double* loss_host, float* grad_host) {
    if (!c) return SHELL_E_INVAL;
    if (!c->mlp_ready || !feat_dev || !tgt_dev || !idx_dev || n_samples < 1 || batch < 32 || batch % 32) {
        c->err = "needs loaded parameters, device arrays, n_samples >= 1 and a batch that is a positive multiple "
                 "of 32";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    hipStream_t st = c->stream;
    {   // the kernels trust the indices: check them here
        std::vector<int64_t> h(batch);
        HIPCHK(hipMemcpyAsync(h.data(), idx_dev, (size_t)batch * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        sync(c);
        for (int64_t v : h)
            if (v < 0 || v >= n_samples) throw InvalErr{"sample index out of range"};
    }
    mlp_work(c, batch);
    HIPCHK(hipMemsetAsync(c->mlp_grad.p, 0, c->mlp_grad.n, st));
    HIPCHK(hipMemsetAsync(c->mlp_loss.p, 0, sizeof(double), st));
    launch_mlp_grad(st, dptr<float>(c->mlp_theta), c->mlp_w.p, feat_dev, tgt_dev, (const long long*)idx_dev, batch,
                    c->mlp_work.p, dptr<float>(c->mlp_grad), dptr<double>(c->mlp_loss));
    HIPCHK(hipGetLastError());
    if (loss_host) HIPCHK(hipMemcpyAsync(loss_host, c->mlp_loss.p, sizeof(double), hipMemcpyDeviceToHost, st));
    if (grad_host)
        HIPCHK(hipMemcpyAsync(grad_host, c->mlp_grad.p, MLP_NPARAMS * sizeof(float), hipMemcpyDeviceToHost, st));
    sync(c);
    return SHELL_OK;
    API_CATCH
}

shell_status shell_mlp_train(shell_ctx* c, const float* feat_dev, const float* tgt_dev, int64_t n_samples,
                             int32_t batch, int32_t steps, float lr, uint64_t seed, double* loss_host) {
    if (!c) return SHELL_E_INVAL;
    if (!c->mlp_ready || !feat_dev || !tgt_dev || n_samples < 1 || batch < 32 || batch % 32 || steps < 0 ||
        !(lr > 0.0f) || !std::isfinite(lr)) {
        c->err = "needs loaded parameters, device arrays, n_samples >= 1, batch a positive multiple of 32, "
                 "steps >= 0 and lr > 0";
        return SHELL_E_INVAL;
    }
    API_TRY
    HIPCHK(hipSetDevice(c->opts.device));
    hipStream_t st = c->stream;
    mlp_work(c, batch);
    if (c->mlp_loss_n < std::max(steps, 1)) {
        alloc(c->mlp_loss, (size_t)std::max(steps, 1) * sizeof(double));
        c->mlp_loss_n = std::max(steps, 1);
    }
    HIPCHK(hipMemsetAsync(c->mlp_loss.p, 0, (size_t)std::max(steps, 1) * sizeof(double), st));
    double* loss = dptr<double>(c->mlp_loss);
    for (int i = 0; i < steps; ++i) {
        launch_sample_idx(st, n_samples, batch, seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1) * 131ull,
                          dptr<long long>(c->mlp_idx));
        HIPCHK(hipMemsetAsync(c->mlp_grad.p, 0, c->mlp_grad.n, st));
        launch_mlp_grad(st, dptr<float>(c->mlp_theta), c->mlp_w.p, feat_dev, tgt_dev, dptr<long long>(c->mlp_idx),
                        batch, c->mlp_work.p, dptr<float>(c->mlp_grad), loss + i);
        launch_mlp_adam(st, dptr<float>(c->mlp_theta), dptr<float>(c->mlp_grad), dptr<float>(c->mlp_m),
                        dptr<float>(c->mlp_v), MLP_NPARAMS, lr, ++c->adam_step);
        launch_mlp_pack(st, dptr<float>(c->mlp_theta), c->mlp_w.p);
        HIPCHK(hipGetLastError());
    }
    if (loss_host && steps > 0)
        HIPCHK(hipMemcpyAsync(loss_host, loss, (size_t)steps * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(c);
    return SHELL_OK;
    API_CATCH
}

shell_status shell_mlp_record(shell_ctx* c, float* feat_dev, float* tgt_dev, int64_t capacity, int32_t per_shell,
                              uint64_t seed) {
    if (!c) return SHELL_E_INVAL;
    c->rec_count = 0;
    c->rec_calls = 0;
    if (!feat_dev) {
        c->rec_feat = nullptr;
        c->rec_tgt = nullptr;
        c->rec_cap = 0;
        return SHELL_OK;
    }
    if (!tgt_dev || capacity < 0 || per_shell < 1) {
        c->err = "recording needs tgt_dev, capacity >= 0 and per_shell >= 1";
        return SHELL_E_INVAL;
    }
    c->rec_feat = feat_dev;
    c->rec_tgt = tgt_dev;
    c->rec_cap = capacity;
    c->rec_K = per_shell;
    c->rec_seed = seed;
    return SHELL_OK;
}

shell_status shell_mlp_recorded(const shell_ctx* c, int64_t* count) {
    if (!c || !count) return SHELL_E_INVAL;
    *count = c->rec_count;
    return SHELL_OK;
}

}  // extern "C"
