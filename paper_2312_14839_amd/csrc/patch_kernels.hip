// Per-patch quadrature kernels of libbhem (gfx950).
//
//   k_energy_grad  energy and gradient of every patch (FP64), 16 lanes per
//                  patch: one lane per Gauss point, then one lane per local
//                  basis function.
//   k_hessian      48x48 patch Hessian (FP64 or FP32) scattered into the
//                  12x12-block matrix, one wavefront per patch:
//                    1. four lanes per Gauss point build the 15x15 second
//                       derivative W_g of the energy density (+ the mass term);
//                    2. per component pair (i, j) the matrix cores contract
//                       K^{ij} = sum_g Phi_g^T W_g^{ij} Phi_g  (16 x 80(96) x 16);
//                    3. the 10 node blocks the matrix stores (diagonal
//                       and upper triangle) are added into it (patches of
//                       one colour share no node, so plain
//                       read-modify-write is race free; the first patch,
//                       in colour order, to reach a block stores it, so
//                       the matrix needs no zero fill).
//
// Quadrature, basis and model follow the paper (Sec. 3-4, Appendix A-B);
// the reduced-form derivatives are documented in shell_physics.hpp.
// Local coordinates: corner c = p + 2q (node (i+p, j+q)), kind k = r + 2s,
// I = 4c + k; local DOF 12 c + 3 k + component.
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"
#include "shell_physics.hpp"

namespace bhem {

// ---------------------------------------------------------------- K1
// Energies: e_patch[p][0] elastic, [1] kinetic (mass_scale/2)(x - xhat)^T rho h (x - xhat),
// [2] load -rho h g.(x - xhat).  Gradient of their sum per patch in g_patch[p][48].
// EGP patches per block of 16 EGP threads (4, 8 or 16; chosen by the
// autotuner, 16 by default)
template <int EGP>
__global__ __launch_bounds__(16 * EGP) void k_energy_grad(int npatch, const int4* __restrict__ patch_nodes,
                                                     const int* __restrict__ patch_shell,
                                                     const ShellParams* __restrict__ shells,
                                                     const double* __restrict__ phi,
                                                     const double* __restrict__ q, const double* __restrict__ qbar,
                                                     const double* __restrict__ qhat, double mass_scale,
                                                     double dt_damp, int elastic, int loads,
                                                     const int* __restrict__ eval_shell,
                                                     double* __restrict__ e_patch,
                                                     double* __restrict__ g_patch) {
    __shared__ double s_u[EGP][48], s_b[EGP][48], s_d[EGP][48];
    __shared__ double s_dpsi[EGP][16][18];
    const int lane = threadIdx.x & 15, pl = threadIdx.x >> 4;
    const int patch = blockIdx.x * EGP + pl;
    // eval_shell (or NULL: all): the patches of other shells are skipped and
    // keep their previous outputs
    const bool active = patch < npatch && (!eval_shell || eval_shell[patch_shell[patch]]);
    ShellParams sp;
    int4 nd = make_int4(0, 0, 0, 0);
    if (active) {
        sp = shells[patch_shell[patch]];
        nd = patch_nodes[patch];
    }
    // phase 0: gather u = q - qbar, qbar and q - qhat, scaled to theta-derivatives
    if (active) {
        const int nodes[4] = {nd.x, nd.y, nd.z, nd.w};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int d = lane * 3 + t, c = d / 12, w = d % 12;
            const double ks = kind_scale(w / 3, sp.dxi1, sp.dxi2);
            const size_t gi = (size_t)nodes[c] * 12 + w;
            const double qq = q[gi], qb = qbar[gi];
            s_u[pl][d] = ks * (qq - qb);
            s_b[pl][d] = ks * qb;
            s_d[pl][d] = qhat ? ks * (qq - qhat[gi]) : 0.0;
        }
    }
    __syncthreads();
    // inertia coefficient; with damping (Newton steps only) 1/dt^2 + alpha/dt,
    // the predictor being the matching combination of qhat and q_n
    const double ms = active ? mass_scale * (1.0 + sp.damp * dt_damp) : 0.0;
    // phase 1: lane = Gauss point
    double e_el = 0.0, e_kin = 0.0, e_ld = 0.0;
    if (active) {
        const int g = lane;
        double kin[30], xd[3] = {0, 0, 0};
        // the table by Gauss point and pairs of basis functions: one 16-byte
        // load gives the lane Phi_g[a][I] and Phi_g[a][I + 1], and the 16
        // lanes of a patch read 256 consecutive bytes (each sum still runs
        // over I in ascending order)
        const double* ph = phi + 2 * 1536 + 2 * g;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const double sc = slot_scale(a, sp.dxi1, sp.dxi2);
            double sb[3] = {0.0, 0.0, 0.0}, su[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int ip = 0; ip < 8; ++ip) {
                const double2 f = *reinterpret_cast<const double2*>(ph + (a * 8 + ip) * 32);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int I = 2 * ip + h;
                    const double fv = h ? f.y : f.x;
#pragma unroll
                    for (int comp = 0; comp < 3; ++comp) {
                        sb[comp] += fv * s_b[pl][3 * I + comp];
                        su[comp] += fv * s_u[pl][3 * I + comp];
                    }
                }
            }
#pragma unroll
            for (int comp = 0; comp < 3; ++comp) {
                kin[3 * a + comp] = sc * sb[comp];
                kin[15 + 3 * a + comp] = sc * su[comp];
            }
        }
#pragma unroll
        for (int ip = 0; ip < 8; ++ip) {
            const double2 f = *reinterpret_cast<const double2*>(ph + (5 * 8 + ip) * 32);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int I = 2 * ip + h;
                const double fv = h ? f.y : f.x;
#pragma unroll
                for (int comp = 0; comp < 3; ++comp) xd[comp] += fv * s_d[pl][3 * I + comp];
            }
        }
        GaussPoint<double> G;
        const double wt = gauss_weight(g & 3) * gauss_weight(g >> 2) * sp.dxi1 * sp.dxi2;
        gauss_point<double>(kin, wt, sp.lam, sp.mu, sp.h, G);
        double dp[15];
        dpsi_dg<double>(G, dp);
        const double el = elastic ? 1.0 : 0.0;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const double sc = G.wq * el * slot_scale(a, sp.dxi1, sp.dxi2);
#pragma unroll
            for (int comp = 0; comp < 3; ++comp) s_dpsi[pl][g][3 * a + comp] = sc * dp[3 * a + comp];
        }
        const double rh = sp.rho_h * G.wq;
        const double gx = loads ? sp.grav[0] : 0.0, gy = loads ? sp.grav[1] : 0.0, gz = loads ? sp.grav[2] : 0.0;
        s_dpsi[pl][g][15] = rh * (ms * xd[0] - gx);
        s_dpsi[pl][g][16] = rh * (ms * xd[1] - gy);
        s_dpsi[pl][g][17] = rh * (ms * xd[2] - gz);
        e_el = el * G.wq * G.psi;
        e_kin = 0.5 * ms * rh * (xd[0] * xd[0] + xd[1] * xd[1] + xd[2] * xd[2]);
        e_ld = -rh * (gx * xd[0] + gy * xd[1] + gz * xd[2]);
    }
    // patch energies: reduce over the 16 lanes of the patch
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
        e_el += __shfl_xor(e_el, off, 16);
        e_kin += __shfl_xor(e_kin, off, 16);
        e_ld += __shfl_xor(e_ld, off, 16);
    }
    if (active && lane == 0) {
        e_patch[3 * (size_t)patch + 0] = e_el;
        e_patch[3 * (size_t)patch + 1] = e_kin;
        e_patch[3 * (size_t)patch + 2] = e_ld;
    }
    __syncthreads();
    // phase 2: lane = local basis function I
    if (active) {
        const int I = lane;
        const double ks = kind_scale(I & 3, sp.dxi1, sp.dxi2);
        double gr[3] = {0, 0, 0};
        // the table by Gauss point and pairs of slots: one 16-byte load gives
        // the lane Phi_g[a][I] and Phi_g[a + 1][I]
        const double* ph = phi + 3 * 1536 + 2 * I;
        for (int g = 0; g < 16; ++g) {
#pragma unroll
            for (int ap = 0; ap < 3; ++ap) {
                const double2 f = *reinterpret_cast<const double2*>(ph + (g * 3 + ap) * 32);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int a = 2 * ap + h;
                    const double fv = h ? f.y : f.x;
#pragma unroll
                    for (int comp = 0; comp < 3; ++comp) gr[comp] += fv * s_dpsi[pl][g][3 * a + comp];
                }
            }
        }
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) g_patch[48 * (size_t)patch + 3 * I + comp] = ks * gr[comp];
    }
}

// Nodal gradient: sum of the patch contributions of every node.  With
// mask != 0 prescribed DOFs get 0.  Only nodes of shells with write_shell[s]
// set are written (NULL = all).
__global__ void k_gather_grad(int nnodes, const int* __restrict__ inc_ptr, const int* __restrict__ inc,
                              const double* __restrict__ g_patch, const uint16_t* __restrict__ freemask,
                              const int* __restrict__ node_shell, const int* __restrict__ write_shell,
                              double* __restrict__ grad) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int node = t / 12, w = t % 12;
    if (node >= nnodes) return;
    if (write_shell && !write_shell[node_shell[node]]) return;
    double s = 0.0;
    for (int k = inc_ptr[node]; k < inc_ptr[node + 1]; ++k) {
        const int pc = inc[k];   // patch * 4 + corner
        s += g_patch[48 * (size_t)(pc >> 2) + 12 * (pc & 3) + w];
    }
    if (freemask && !((freemask[node] >> w) & 1)) s = 0.0;
    grad[(size_t)node * 12 + w] = s;
}

// Pressure load per patch (Sec. 4.3, "External Forces"): a pressure p of
// the patch's shell acts per unit current area along a_1 x a_2, so the
// generalized force of local coordinate I = 4c + k is
//   F_I = sum_gp w p Phi^I (a_1 x a_2),
// written as g_patch[48 p + 12 c + 3 k + comp] (gathered like the gradient).
// One thread per (patch, I); a_1, a_2 at the 16 Gauss points from the theta
// basis table (slots 0, 1 and the value slot 5).
__global__ void __launch_bounds__(256) k_pressure(int npatch, const int4* __restrict__ patch_nodes,
                                                  const int* __restrict__ patch_shell,
                                                  const ShellParams* __restrict__ shells,
                                                  const double* __restrict__ pressure, const double* __restrict__ phi,
                                                  const double* __restrict__ q, double* __restrict__ g_patch) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 16 * npatch) return;
    const int p = t >> 4, I = t & 15;
    const int sh = patch_shell[p];
    const ShellParams& sp = shells[sh];
    const double pr = pressure[sh];
    const int4 nd = patch_nodes[p];
    const int node[4] = {nd.x, nd.y, nd.z, nd.w};
    double f[3] = {0.0, 0.0, 0.0};
    if (pr != 0.0)
        for (int g = 0; g < 16; ++g) {
            const double* ph = phi + (size_t)g * 96;
            double a1[3] = {0.0, 0.0, 0.0}, a2[3] = {0.0, 0.0, 0.0};
            for (int J = 0; J < 16; ++J) {
                const double ks = kind_scale(J & 3, sp.dxi1, sp.dxi2);
                const double* v = q + 12 * (size_t)node[J >> 2] + 3 * (J & 3);
                const double p1 = ph[0 * 16 + J] * ks, p2 = ph[1 * 16 + J] * ks;
                for (int c = 0; c < 3; ++c) {
                    a1[c] += p1 * v[c];
                    a2[c] += p2 * v[c];
                }
            }
            const double s1 = slot_scale(0, sp.dxi1, sp.dxi2), s2 = slot_scale(1, sp.dxi1, sp.dxi2);
            const double n[3] = {s1 * s2 * (a1[1] * a2[2] - a1[2] * a2[1]), s1 * s2 * (a1[2] * a2[0] - a1[0] * a2[2]),
                                 s1 * s2 * (a1[0] * a2[1] - a1[1] * a2[0])};
            const double w = gauss_weight(g & 3) * gauss_weight(g >> 2) * sp.dxi1 * sp.dxi2 * pr *
                             ph[5 * 16 + I] * kind_scale(I & 3, sp.dxi1, sp.dxi2);
            for (int c = 0; c < 3; ++c) f[c] += w * n[c];
        }
    double* out = g_patch + 48 * (size_t)p + 12 * (I >> 2) + 3 * (I & 3);
    for (int c = 0; c < 3; ++c) out[c] = f[c];
}

// Per-shell sums of the three patch energies, fixed summation order: one
// block of 1024 threads per shell, each thread its strided patches in order
// (eight loads in flight), then a fixed tree.
__global__ __launch_bounds__(1024) void k_shell_energy(int nshell, const ShellParams* __restrict__ shells,
                                                       const double* __restrict__ e_patch,
                                                       double* __restrict__ e_shell) {
    const int s = blockIdx.x;
    if (s >= nshell) return;
    __shared__ double red[3][1024];
    double a0 = 0, a1 = 0, a2 = 0;
    const int p1 = shells[s].patch_end;
#pragma unroll 8
    for (int p = shells[s].patch_begin + threadIdx.x; p < p1; p += 1024) {
        a0 += e_patch[3 * (size_t)p];
        a1 += e_patch[3 * (size_t)p + 1];
        a2 += e_patch[3 * (size_t)p + 2];
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    red[2][threadIdx.x] = a2;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) e_shell[3 * s + k] = red[k][0];
}

// ---------------------------------------------------------------- K2
// NWV patches (wavefronts) per block: 4 or 8, chosen by the autotuner (4
// by default).  Each wavefront gathers, contracts and scatters its own
// patch; the second derivative of the energy density (phase 1b) is shared
// out by part instead: in each group of four wavefronts, wavefront w
// computes part w of it (hess_blocks) for the group's four patches x 16
// Gauss points, one per lane, so no wavefront diverges on the part.

__host__ __device__ constexpr int pair_index(int i, int j) {   // i <= j
    return i == j ? i : (i == 0 ? (j == 1 ? 3 : 4) : 5);
}

template <class T, int NWV>
__global__ __launch_bounds__(64 * NWV) void k_hessian(const int* __restrict__ patch_list, int nlist,
                                                 const int4* __restrict__ patch_nodes,
                                                 const int* __restrict__ patch_shell,
                                                 const int* __restrict__ patch_slots,
                                                 const uint64_t* __restrict__ patch_kid,
                                                 const uint16_t* __restrict__ patch_first,
                                                 const ShellParams* __restrict__ shells,
                                                 const double* __restrict__ phi, const double* __restrict__ q,
                                                 const double* __restrict__ qbar, double mass_scale,
                                                 double dt_damp, int elastic, int pseudo, T* __restrict__ vals,
                                                 T* __restrict__ scr) {
    typedef Mfma<T> MM;
    constexpr int WSZ = 16 * 121;   // packed W per Gauss point (+ mass term) and pair staging (6*256)
    static_assert(WSZ >= 6 * 256, "staging must fit");
    static_assert(NWV % 4 == 0, "phase 1b shares four patches among four wavefronts");
    __shared__ T s_u[NWV][48], s_b[NWV][48];
    __shared__ T s_kin[NWV][16][30];
    __shared__ T s_w[NWV][WSZ];
    // per patch of the block: lam, mu, h, dxi1, dxi2, mass coefficient
    // rho h mass_scale (1 + alpha dt_damp)
    __shared__ double s_par[NWV][6];
    // the wavefront's patch and everything derived from it are wave-uniform
    // (scalar registers and loads)
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = blockIdx.x * NWV + wv;
    const bool active = li < nlist;
    const int patch = active ? patch_list[li] : 0;
    ShellParams sp = shells[active ? patch_shell[patch] : 0];
    const int4 nd = patch_nodes[patch];
    const int nodes[4] = {nd.x, nd.y, nd.z, nd.w};
    T* W = s_w[wv];
    // phase 0: displacement and reference coordinates (theta-scaled)
    if (active && lane < 48) {
        const int c = lane / 12, w = lane % 12;
        const double ks = kind_scale(w / 3, sp.dxi1, sp.dxi2);
        const size_t gi = (size_t)nodes[c] * 12 + w;
        const double qb = qbar[gi];
        s_u[wv][lane] = (T)(ks * (q[gi] - qb));
        s_b[wv][lane] = (T)(ks * qb);
    }
    if (active && lane == 0) {
        s_par[wv][0] = sp.lam;
        s_par[wv][1] = sp.mu;
        s_par[wv][2] = sp.h;
        s_par[wv][3] = sp.dxi1;
        s_par[wv][4] = sp.dxi2;
        s_par[wv][5] = sp.rho_h * mass_scale * (1.0 + sp.damp * dt_damp);
    }
    __syncthreads();
    // phase 1a: kinematics on the matrix cores.  For slot a, the 16 Gauss
    // points' values out[g][c] = sum_I Phi_g[a][I] X[I][c] with X[I] = (the
    // reference coordinates' 3 components | the displacement's 3), a 16 x 16
    // x 16 product in four k-steps of 4 basis functions; lanes of columns
    // c < 6 keep theirs (30 values per Gauss point: s_kin[g][15 src + 3 a + comp]).
    if (active) {
        const int gc = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            typename MM::acc_t kacc{T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int I = 4 * st + kq;
                // A[row g = gc][k = I], from the transposed table
                const T av = (T)phi[16 * 96 + (a * 16 + I) * 16 + gc];
                const T bv = gc < 3 ? s_b[wv][3 * I + gc] : gc < 6 ? s_u[wv][3 * I + gc - 3] : T(0);   // B[k = I][c = gc]
                kacc = MM::mma(av, bv, kacc);
            }
            const T sc = (T)slot_scale(a, sp.dxi1, sp.dxi2);
            if (gc < 6) {
                const int vi = gc < 3 ? 3 * a + gc : 15 + 3 * a + gc - 3;
#pragma unroll
                for (int v = 0; v < 4; ++v) s_kin[wv][MM::row(lane, v)][vi] = kacc[v] * sc;
            }
        }
    }
    __syncthreads();
    // phase 1b: 15x15 second derivative of the energy density (+ mass term);
    // lane = (patch slot of the group, Gauss point), part = wavefront in group
    {
        const int part = wv & 3, slot = (wv & ~3) + (lane >> 4), gp = lane & 15;
        if (blockIdx.x * NWV + slot < nlist) {
            const double* par = s_par[slot];
            T kin[30];
#pragma unroll
            for (int k = 0; k < 30; ++k) kin[k] = s_kin[slot][gp][k];
            GaussPoint<T> G;
            const T wt = (T)(gauss_weight(gp & 3) * gauss_weight(gp >> 2) * par[3] * par[4]);
            gauss_point<T>(kin, wt, (T)par[0], (T)par[1], (T)par[2], G);
            T* Wg = s_w[slot] + gp * 121;
            if (elastic) {
                T sc[5];
#pragma unroll
                for (int a = 0; a < 5; ++a) sc[a] = (T)slot_scale(a, par[3], par[4]);
                hess_blocks<T>(G, part, pseudo, sc, Wg);
            }
            if (part == 3) Wg[120] = G.wq * (T)par[5];
        }
    }
    __syncthreads();
    // phase 2: K^{ij} = sum over (slot a, Gauss point g) of Phi^T W^{ij} Phi on the matrix cores.
    // Lane operand table: ph_l[a][m] = Phi_{g = 4m + lane/16}[a][I = lane%16].
    T ph_l[6][4];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int m = 0; m < 4; ++m) ph_l[a][m] = (T)phi[((4 * m + (lane >> 4)) * 6 + a) * 16 + (lane & 15)];
    typename MM::acc_t acc[6];
#pragma unroll
    for (int pr = 0; pr < 6; ++pr) acc[pr] = typename MM::acc_t{T(0), T(0), T(0), T(0)};
    const bool has_mass = mass_scale != 0.0;
    if (active) {
#pragma unroll
        for (int pr = 0; pr < 6; ++pr) {
            const int i = pr < 3 ? pr : (pr == 5 ? 1 : 0);
            const int j = pr < 3 ? pr : (pr == 3 ? 1 : 2);
            if (elastic) {
#pragma unroll
                for (int a = 0; a < 5; ++a)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const T* Wg = W + (4 * m + (lane >> 4)) * 121;
                        const int r = 3 * a + i;
                        T b = T(0);
#pragma unroll
                        for (int bb = 0; bb < 5; ++bb) {
                            const int c = 3 * bb + j;
                            const T wv_ = r <= c ? Wg[sym15(r, c)] : Wg[sym15(c, r)];
                            b += wv_ * ph_l[bb][m];
                        }
                        acc[pr] = MM::mma(ph_l[a][m], b, acc[pr]);
                    }
            }
            if (i == j && has_mass) {
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const T* Wg = W + (4 * m + (lane >> 4)) * 121;
                    acc[pr] = MM::mma(ph_l[5][m], Wg[120] * ph_l[5][m], acc[pr]);
                }
            }
        }
    }
    __syncthreads();
    // stage the six 16x16 pair blocks: P[pr][I][J]
    if (active) {
#pragma unroll
        for (int pr = 0; pr < 6; ++pr)
#pragma unroll
            for (int v = 0; v < 4; ++v) W[pr * 256 + MM::row(lane, v) * 16 + (lane & 15)] = acc[pr][v];
    }
    __syncthreads();
    // phase 3: add the node blocks the matrix stores (the diagonal blocks
    // and, of each pair (c, d) of distinct nodes, the one whose row node has
    // the larger index; column-major 12x12, a diagonal block in the packed
    // symmetric layout at SYM12_VALS) into the matrix.  Entry m of the
    // patch's slot list is the m-th stored local block (local index in
    // nibble m of patch_kid; the 4 diagonal blocks first, the list ends at
    // the first -1).  A block this patch touches first is stored, the others
    // are read, added to and written back.  Lane l takes elements
    // w = l + 64 u of every block (u = 0, 1, and 2 for l < 16; of a diagonal
    // block's 84 values l and, for l < 20, l + 64), so its index arithmetic
    // is done once; the block's nodes and slot are the same for the whole
    // wavefront.  Four blocks per round keep 12 reads per lane in flight.
    if (active) {
        // the scaled block value is rounded before it is added (no fused
        // multiply-add), as the single-launch form's sum in colour order does
#pragma clang fp contract(off)
        const int* slots = patch_slots + 16 * (size_t)patch;
        const uint64_t kid = patch_kid[patch];
        const unsigned first = patch_first[patch];
        // u = 0..2: off-diagonal blocks; u = 3, 4: diagonal blocks
        int lo[5];
        bool sw[5];
        T ks[5];
#pragma unroll
        for (int u = 0; u < 5; ++u) {
            int ii, jj;
            if (u < 3) {
                const int w = u < 2 ? lane + 64 * u : (lane & 15) + 128;
                jj = w / 12;   // column-major: w = jj*12 + ii
                ii = w % 12;
            } else {
                const int p = u == 3 ? lane : (lane < 20 ? lane : lane & 15) + 64;
                ii = sym12_row(p);
                jj = sym12_col(p);
            }
            const int k = ii / 3, i = ii % 3, l = jj / 3, j = jj % 3;
            // K block (I, J) = (4c + k, 4d + l) of component pair (i, j): the
            // staged pair blocks hold i <= j, so i > j reads the transpose
            sw[u] = i > j;
            lo[u] = sw[u] ? pair_index(j, i) * 256 + 16 * l + k : pair_index(i, j) * 256 + 16 * k + l;
            ks[u] = (T)(kind_scale(k, sp.dxi1, sp.dxi2) * kind_scale(l, sp.dxi1, sp.dxi2));
        }
        constexpr int MB = 4;
        // scr: each stored local block goes to its own slot of the scratch,
        // scr[(10 p + m) 144 + element], for k_gather_blocks to sum in colour
        // order, instead of into the matrix
        if (scr) {
#pragma unroll 1
            for (int m = 0; m < 10; ++m) {
                const int sl = slots[m];
                if (sl < 0) break;
                const int blk = (int)((kid >> (4 * m)) & 15u);
                const int c = blk >> 2, d = blk & 3;
                const int cd = 64 * c + 4 * d, dc = 64 * d + 4 * c;
                T* dst = scr + ((size_t)patch * 10 + m) * 144;
                const bool dg = m < 4;
                const int nu = dg ? 2 : 3;
                const bool last_ok = dg ? lane < 20 : lane < 16;
                for (int u = 0; u < nu; ++u) {
                    const int v = dg ? u + 3 : u;
                    if (u < nu - 1 || last_ok) dst[lane + 64 * u] = ks[v] * W[lo[v] + (sw[v] ? dc : cd)];
                }
            }
            return;
        }
        // one round: blocks m0 .. m0 + MB - 1 of the list, all diagonal (DG)
        // or all off the diagonal
        auto round = [&](int m0, auto dg_tag) {
#pragma clang fp contract(off)
            constexpr bool DG = decltype(dg_tag)::value;
            constexpr int NU = DG ? 2 : 3;
            const bool last_ok = DG ? lane < 20 : lane < 16;   // u = NU - 1
            T add[MB][NU], old[MB][NU];
            int sl[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int m = m0 + mb;
                sl[mb] = m < 16 ? slots[m] : -1;
                if (sl[mb] < 0) continue;
                const int blk = (int)((kid >> (4 * m)) & 15u);
                const int c = blk >> 2, d = blk & 3;
                const int cd = 64 * c + 4 * d, dc = 64 * d + 4 * c;
                const T* src = vals + (size_t)sl[mb] * 144;
                const bool fresh = (first >> m) & 1u;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const int v = DG ? u + 3 : u;
                    add[mb][u] = ks[v] * W[lo[v] + (sw[v] ? dc : cd)];
                    old[mb][u] = (fresh || (u == NU - 1 && !last_ok)) ? T(0) : src[lane + 64 * u];
                }
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                if (sl[mb] < 0) continue;
                T* dst = vals + (size_t)sl[mb] * 144;
#pragma unroll
                for (int u = 0; u < NU; ++u)
                    if (u < NU - 1 || last_ok) dst[lane + 64 * u] = old[mb][u] + add[mb][u];
            }
        };
        round(0, std::true_type{});
#pragma unroll 1
        for (int m0 = 4; m0 < 16; m0 += MB) {
            if (slots[m0] < 0) break;
            round(m0, std::false_type{});
        }
    }
}

// ------------------------------------------------------------ launchers
void launch_energy_grad(hipStream_t st, int npatch, const int4* patch_nodes, const int* patch_shell,
                        const ShellParams* shells, const double* phi, const double* q, const double* qbar,
                        const double* qhat, double mass_scale, double dt_damp, int elastic, int loads,
                        const int* eval_shell, double* e_patch, double* g_patch, int patches_per_block) {
    if (npatch == 0) return;
    const int egp = patches_per_block == 4 || patches_per_block == 8 ? patches_per_block : 16;
    const int nb = (npatch + egp - 1) / egp;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nb), dim3(16 * egp), 0, st, npatch, patch_nodes, patch_shell, shells, phi, q,
                           qbar, qhat, mass_scale, dt_damp, elastic, loads, eval_shell, e_patch, g_patch);
    };
    if (egp == 4) go(k_energy_grad<4>);
    else if (egp == 8) go(k_energy_grad<8>);
    else go(k_energy_grad<16>);
}

void launch_gather_grad(hipStream_t st, int nnodes, const int* inc_ptr, const int* inc, const double* g_patch,
                        const uint16_t* freemask, const int* node_shell, const int* write_shell, double* grad) {
    const int n = nnodes * 12;
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_grad, dim3((n + 255) / 256), dim3(256), 0, st, nnodes, inc_ptr, inc, g_patch,
                       freemask, node_shell, write_shell, grad);
}

void launch_pressure(hipStream_t st, int npatch, const int4* patch_nodes, const int* patch_shell,
                     const ShellParams* shells, const double* pressure, const double* phi, const double* q,
                     double* g_patch) {
    if (npatch == 0) return;
    hipLaunchKernelGGL(k_pressure, dim3((16 * npatch + 255) / 256), dim3(256), 0, st, npatch, patch_nodes,
                       patch_shell, shells, pressure, phi, q, g_patch);
}

void launch_shell_energy(hipStream_t st, int nshell, const ShellParams* shells, const double* e_patch,
                         double* e_shell) {
    hipLaunchKernelGGL(k_shell_energy, dim3(nshell), dim3(1024), 0, st, nshell, shells, e_patch, e_shell);
}

template <class T>
void launch_hessian(hipStream_t st, const int* patch_list, int nlist, const int4* patch_nodes, const int* patch_shell,
                    const int* patch_slots, const uint64_t* patch_kid, const uint16_t* patch_first,
                    const ShellParams* shells, const double* phi, const double* q, const double* qbar,
                    double mass_scale, double dt_damp, int elastic, int pseudo, T* vals, int waves, T* scr) {
    if (nlist == 0) return;
    const int nw = waves == 8 ? 8 : 4;
    const int nb = (nlist + nw - 1) / nw;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nb), dim3(64 * nw), 0, st, patch_list, nlist, patch_nodes, patch_shell,
                           patch_slots, patch_kid, patch_first, shells, phi, q, qbar, mass_scale, dt_damp, elastic,
                           pseudo, vals, scr);
    };
    if (nw == 8) go(k_hessian<T, 8>);
    else go(k_hessian<T, 4>);
}

// One wavefront per stored block: the sum, in colour order, of the local
// blocks in scr that the patches add to it (cptr/cidx), from 0 -- the same
// operations as the colour launches' first store and read-modify-writes.
// A diagonal block has its 84 packed values, the others 144.
template <class T>
__global__ __launch_bounds__(256) void k_gather_blocks(int nsb, const int* __restrict__ cptr,
                                                       const int* __restrict__ cidx,
                                                       const uint8_t* __restrict__ diag,
                                                       const T* __restrict__ scr, T* __restrict__ vals) {
    const int lane = threadIdx.x & 63;
    const int sb = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (sb >= nsb) return;
    const int k0 = cptr[sb], k1 = cptr[sb + 1];
    const bool dg = diag[sb] != 0;
    const int nu = dg ? 2 : 3;
    const bool last_ok = dg ? lane < 20 : lane < 16;
    for (int u = 0; u < nu; ++u) {
        if (u == nu - 1 && !last_ok) break;
        const int e = lane + 64 * u;
        T v = T(0);
        for (int k = k0; k < k1; ++k) v = v + scr[(size_t)cidx[k] * 144 + e];
        vals[(size_t)sb * 144 + e] = v;
    }
}

template <class T>
void launch_gather_blocks(hipStream_t st, int nsb, const int* cptr, const int* cidx, const uint8_t* diag, const T* scr,
                          T* vals) {
    if (nsb == 0) return;
    hipLaunchKernelGGL(k_gather_blocks<T>, dim3((nsb + 3) / 4), dim3(256), 0, st, nsb, cptr, cidx, diag, scr, vals);
}
int hessian_resident_patches(int device, int fp32) {
    int per_cu = 0, cus = 0;
    const void* fn = fp32 ? (const void*)k_hessian<float, 4> : (const void*)k_hessian<double, 4>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return 4 * per_cu * cus;
}

template void launch_gather_blocks<double>(hipStream_t, int, const int*, const int*, const uint8_t*, const double*,
                                           double*);
template void launch_gather_blocks<float>(hipStream_t, int, const int*, const int*, const uint8_t*, const float*,
                                          float*);

template void launch_hessian<double>(hipStream_t, const int*, int, const int4*, const int*, const int*,
                                     const uint64_t*, const uint16_t*, const ShellParams*, const double*, const double*,
                                     const double*, double, double, int, int, double*, int, double*);
template void launch_hessian<float>(hipStream_t, const int*, int, const int4*, const int*, const int*,
                                    const uint64_t*, const uint16_t*, const ShellParams*, const double*, const double*,
                                    const double*, double, double, int, int, float*, int, float*);

}  // namespace bhem
