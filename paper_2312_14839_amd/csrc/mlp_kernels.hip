// Per-node warm-start network of libbhem (gfx950, BF16 matrix cores).
//
// y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3, 60 -> 128 -> 128 -> 12,
// operands of every product in bfloat16, accumulation in FP32
// (v_mfma_f32_16x16x32_bf16: 16x16 output, K = 32 per instruction).
//
// A wavefront handles a tile of 16 samples.  Operand layouts (checked on
// gfx950): lane l supplies A[l%16][8*(l/16) + j] and B[8*(l/16) + j][l%16],
// j < 8; accumulator element v of lane l is D[4*(l/16) + v][l%16].
// Weights live in device memory in two bf16 layouts: "nk" = [n][k] (the
// forward B operand, k contiguous) and the math layout [k][n] (the B operand
// of the backward products).  Training keeps FP32 master weights and Adam
// moments; gradients of the weights are products over samples with the
// activations and errors stored transposed ([feature][sample]).
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace bhem {

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4_t mma_bf16(bf8_t a, bf8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf8_t load_bf8(const __bf16* p) { return *reinterpret_cast<const bf8_t*>(p); }

// Parameter offsets of the FP32 master vector (math layout, row-major):
// W1[60][128], b1[128], W2[128][128], b2[128], W3[128][12], b3[12].
constexpr int O_W1 = 0, O_B1 = O_W1 + MLP_IN * MLP_H, O_W2 = O_B1 + MLP_H, O_B2 = O_W2 + MLP_H * MLP_H,
              O_W3 = O_B2 + MLP_H, O_B3 = O_W3 + MLP_H * MLP_OUT;
static_assert(O_B3 + MLP_OUT == MLP_NPARAMS, "parameter layout");

// bf16 operand copies: forward [n][k] with K padded to a multiple of 32,
// backward math layout [k][n] with N padded to 32 for W3.
constexpr int K1P = 64;      // 60 -> 64
constexpr int N3P = 16;      // 12 -> 16 (forward output tile)
constexpr int K3BP = 32;     // 12 -> 32 (backward reduction over outputs)
constexpr int OFF_F1 = 0;                      // W1nk [128][64]
constexpr int OFF_F2 = OFF_F1 + MLP_H * K1P;   // W2nk [128][128]
constexpr int OFF_F3 = OFF_F2 + MLP_H * MLP_H; // W3nk [16][128]
constexpr int OFF_B2 = OFF_F3 + N3P * MLP_H;   // W2kn [128][128] (row k = hidden input)
constexpr int OFF_B3 = OFF_B2 + MLP_H * MLP_H; // W3kn [128][32]
constexpr int BF_TOTAL = OFF_B3 + MLP_H * K3BP;

int mlp_bf16_elems() { return BF_TOTAL; }

// Build the bf16 operand copies from the FP32 master weights.
__global__ void k_mlp_pack(const float* __restrict__ th, __bf16* __restrict__ w) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= BF_TOTAL) return;
    float v = 0.0f;
    if (t < OFF_F2) {   // W1nk[n][k] = W1[k][n]
        const int n = t / K1P, k = t % K1P;
        v = k < MLP_IN ? th[O_W1 + k * MLP_H + n] : 0.0f;
    } else if (t < OFF_F3) {
        const int e = t - OFF_F2, n = e / MLP_H, k = e % MLP_H;
        v = th[O_W2 + k * MLP_H + n];
    } else if (t < OFF_B2) {
        const int e = t - OFF_F3, n = e / MLP_H, k = e % MLP_H;
        v = n < MLP_OUT ? th[O_W3 + k * MLP_OUT + n] : 0.0f;
    } else if (t < OFF_B3) {   // W2kn[k][n] = W2[k][n]
        v = th[O_W2 + (t - OFF_B2)];
    } else {   // W3kn[k][n], n padded to 32
        const int e = t - OFF_B3, k = e / K3BP, n = e % K3BP;
        v = n < MLP_OUT ? th[O_W3 + k * MLP_OUT + n] : 0.0f;
    }
    w[t] = (__bf16)v;
}

// ------------------------------------------------------------ forward tile
// acc[t] (t < NT) += A[16][K] (LDS, row-major, lda) x B with B given as
// Bnk[n][k] (k contiguous, ldb), output columns 16t .. 16t+15.
template <int NT, int K>
__device__ __forceinline__ void tile_gemm(const __bf16* A, int lda, const __bf16* Bnk, int ldb, f4_t* acc) {
    const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int s = 0; s < K / 32; ++s) {
        const bf8_t a = load_bf8(A + r * lda + 32 * s + 8 * kq);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mma_bf16(a, load_bf8(Bnk + (16 * t + r) * ldb + 32 * s + 8 * kq), acc[t]);
    }
}

// Write acc (+bias, optional relu) of a 16 x 16*NT tile to LDS as bf16 rows.
template <int NT>
__device__ __forceinline__ void tile_store(const f4_t* acc, const float* bias, bool relu, __bf16* H, int ldh,
                                           float* Hf = nullptr) {
    const int lane = threadIdx.x & 63, c = lane & 15, rq = lane >> 4;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float x = acc[t][v] + bias[16 * t + c];
            if (relu) x = fmaxf(x, 0.0f);
            H[(4 * rq + v) * ldh + 16 * t + c] = (__bf16)x;
            if (Hf) Hf[(4 * rq + v) * ldh + 16 * t + c] = x;
        }
}

struct MlpTileLds {
    __bf16 X[16 * K1P];
    __bf16 H1[16 * MLP_H];
    __bf16 H2[16 * MLP_H];
    float Y[16 * N3P];
};

// Forward pass of one 16-sample tile whose bf16 inputs are in L.X.
__device__ __forceinline__ void mlp_forward_tile(const float* __restrict__ th, const __bf16* __restrict__ w,
                                                 MlpTileLds& L) {
    const int lane = threadIdx.x & 63, c = lane & 15, rq = lane >> 4;
    {
        f4_t acc[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = f4_t{0, 0, 0, 0};
        tile_gemm<8, K1P>(L.X, K1P, w + OFF_F1, K1P, acc);
        tile_store<8>(acc, th + O_B1, true, L.H1, MLP_H);
    }
    __syncthreads();
    {
        f4_t acc[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = f4_t{0, 0, 0, 0};
        tile_gemm<8, MLP_H>(L.H1, MLP_H, w + OFF_F2, MLP_H, acc);
        tile_store<8>(acc, th + O_B2, true, L.H2, MLP_H);
    }
    __syncthreads();
    {
        f4_t acc[1] = {f4_t{0, 0, 0, 0}};
        tile_gemm<1, MLP_H>(L.H2, MLP_H, w + OFF_F3, MLP_H, acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) L.Y[(4 * rq + v) * N3P + c] = acc[0][v] + (c < MLP_OUT ? th[O_B3 + c] : 0.0f);
    }
    __syncthreads();
}

// ---------------------------------------------------------- plain forward
constexpr int MLP_WAVES = 4;

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ th, const __bf16* __restrict__ w,
                                                     const float* __restrict__ feat, float* __restrict__ out,
                                                     long long n) {
    __shared__ MlpTileLds lds[MLP_WAVES];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    MlpTileLds& L = lds[wv];
    const long long tile0 = ((long long)blockIdx.x * MLP_WAVES + wv) * 16;
    // waves past the end run on zeros (no early exit: the block synchronises)
    for (int e = lane; e < 16 * K1P; e += 64) {
        const int r = e / K1P, k = e % K1P;
        const long long s = tile0 + r;
        L.X[e] = (__bf16)((k < MLP_IN && s < n) ? feat[s * MLP_IN + k] : 0.0f);
    }
    __syncthreads();
    mlp_forward_tile(th, w, L);
    for (int e = lane; e < 16 * MLP_OUT; e += 64) {
        const int r = e / MLP_OUT, k = e % MLP_OUT;
        if (tile0 + r < n) out[(tile0 + r) * MLP_OUT + k] = L.Y[r * N3P + k];
    }
}

// ------------------------------------------------------- forward + errors
// For a mini-batch: forward, loss partials, errors dY = 2(y - t)/B,
// dH2 = (dY W3^T) * [h2 > 0], dH1 = (dH2 W2^T) * [h1 > 0], bias gradients
// (atomic), and the transposed activations / errors for the weight products.
struct TrainWork {
    __bf16 *XT, *H1T, *H2T;      // [64][B], [128][B], [128][B]
    __bf16 *DYT, *D2T, *D1T;     // [32][B], [128][B], [128][B]
};

__global__ __launch_bounds__(256) void k_mlp_fwd_bwd(const float* __restrict__ th, const __bf16* __restrict__ w,
                                                     const float* __restrict__ feat, const float* __restrict__ tgt,
                                                     const long long* __restrict__ idx, int B, TrainWork W,
                                                     float* __restrict__ grad, double* __restrict__ loss) {
    __shared__ MlpTileLds lds[MLP_WAVES];
    __shared__ __bf16 sD[MLP_WAVES][16 * MLP_H];   // dY (ld 32) then dH2
    __shared__ __bf16 sE[MLP_WAVES][16 * MLP_H];   // dH1
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, c = lane & 15, rq = lane >> 4;
    MlpTileLds& L = lds[wv];
    const int tile0 = (blockIdx.x * MLP_WAVES + wv) * 16;
    const bool act = tile0 < B;   // B is a multiple of 16; idle waves only synchronise
    for (int e = lane; e < 16 * K1P; e += 64) {
        const int r = e / K1P, k = e % K1P;
        L.X[e] = (__bf16)((act && k < MLP_IN) ? feat[idx[tile0 + r] * MLP_IN + k] : 0.0f);
    }
    __syncthreads();
    mlp_forward_tile(th, w, L);
    // dY (bf16 rows, K padded to 32) and the loss
    float lsum = 0.0f;
    __bf16* dY = sD[wv];
    for (int e = lane; e < 16 * K3BP; e += 64) {
        const int r = e / K3BP, k = e % K3BP;
        float d = 0.0f;
        if (act && k < MLP_OUT) {
            const float diff = L.Y[r * N3P + k] - tgt[idx[tile0 + r] * MLP_OUT + k];
            lsum += diff * diff;
            d = 2.0f * diff / (float)B;
            atomicAdd(&grad[O_B3 + k], d);
        }
        dY[r * K3BP + k] = (__bf16)d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (act && lane == 0) atomicAdd(loss, (double)lsum / (double)B);
    __syncthreads();
    // transposed activations and dY for the weight products
    for (int e = lane; act && e < 16 * K1P; e += 64) {
        const int r = e % 16, k = e / 16;
        W.XT[(size_t)k * B + tile0 + r] = L.X[r * K1P + k];
    }
    for (int e = lane; act && e < 16 * MLP_H; e += 64) {
        const int r = e % 16, k = e / 16;
        W.H1T[(size_t)k * B + tile0 + r] = L.H1[r * MLP_H + k];
        W.H2T[(size_t)k * B + tile0 + r] = L.H2[r * MLP_H + k];
    }
    for (int e = lane; act && e < 16 * K3BP; e += 64) {
        const int r = e % 16, k = e / 16;
        W.DYT[(size_t)k * B + tile0 + r] = dY[r * K3BP + k];
    }
    // dH2 = (dY W3^T) * [h2 > 0]: A = dY [16][32], B[k][n] = W3[n][k] -> Bnk = W3kn rows n
    f4_t acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = f4_t{0, 0, 0, 0};
    tile_gemm<8, K3BP>(dY, K3BP, w + OFF_B3, K3BP, acc);
    __syncthreads();
    __bf16* dH2 = sD[wv];
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 4 * rq + v, col = 16 * t + c;
            const float g = (float)L.H2[r * MLP_H + col] > 0.0f ? acc[t][v] : 0.0f;
            dH2[r * MLP_H + col] = (__bf16)g;
        }
    __syncthreads();
    // dH1 = (dH2 W2^T) * [h1 > 0]: Bnk = W2kn (row n = hidden-1 index)
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = f4_t{0, 0, 0, 0};
    tile_gemm<8, MLP_H>(dH2, MLP_H, w + OFF_B2, MLP_H, acc);
    __bf16* dH1 = sE[wv];
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 4 * rq + v, col = 16 * t + c;
            const float g = (float)L.H1[r * MLP_H + col] > 0.0f ? acc[t][v] : 0.0f;
            dH1[r * MLP_H + col] = (__bf16)g;
        }
    __syncthreads();
    // bias gradients (of the bf16 errors, as used in the products) and transposes
    for (int k = lane; act && k < 2 * MLP_H; k += 64) {
        const __bf16* src = k < MLP_H ? dH2 : dH1;
        const int col = k % MLP_H;
        float s = 0.0f;
        for (int r = 0; r < 16; ++r) s += (float)src[r * MLP_H + col];
        atomicAdd(&grad[(k < MLP_H ? O_B2 : O_B1) + col], s);
    }
    for (int e = lane; act && e < 16 * MLP_H; e += 64) {
        const int r = e % 16, k = e / 16;
        W.D2T[(size_t)k * B + tile0 + r] = dH2[r * MLP_H + k];
        W.D1T[(size_t)k * B + tile0 + r] = dH1[r * MLP_H + k];
    }
}

// -------------------------------------------------------- weight products
// grad(W)[m][n] += sum over samples of AT[m][s] * DT[n][s] for one 16x16
// output tile and one slice of samples; A operand lane: AT[m = row][s..],
// B operand lane: DT[n][s..] (samples contiguous in both).
// output tiles: W1 (MLP_IN rows, padded to K1P) x 8, W2 8x8, W3 8x1
constexpr int WG_T1 = ((MLP_IN + 15) / 16) * 8, WG_T2 = WG_T1 + 64, WG_TILES = WG_T2 + 8;
static_assert(MLP_IN <= K1P, "input features fit the padded first layer");
__global__ __launch_bounds__(64) void k_mlp_wgrad(TrainWork W, int B, int slice, float* __restrict__ grad) {
    const int tile = blockIdx.x, sl = blockIdx.y;
    const int lane = threadIdx.x, r = lane & 15, kq = lane >> 4, c = lane & 15, rq = lane >> 4;
    const __bf16 *AT, *DT;
    int m0, n0, go, ldn, mlim, nlim;
    if (tile < WG_T1) {
        AT = W.XT; DT = W.D1T; m0 = 16 * (tile / 8); n0 = 16 * (tile % 8); go = O_W1; ldn = MLP_H; mlim = MLP_IN;
        nlim = MLP_H;
    } else if (tile < WG_T2) {
        const int t = tile - WG_T1;
        AT = W.H1T; DT = W.D2T; m0 = 16 * (t / 8); n0 = 16 * (t % 8); go = O_W2; ldn = MLP_H; mlim = MLP_H;
        nlim = MLP_H;
    } else {
        const int t = tile - WG_T2;
        AT = W.H2T; DT = W.DYT; m0 = 16 * t; n0 = 0; go = O_W3; ldn = MLP_OUT; mlim = MLP_H; nlim = MLP_OUT;
    }
    f4_t acc = {0, 0, 0, 0};
    const int s0 = sl * slice, s1 = min(B, s0 + slice);
    for (int s = s0; s < s1; s += 32) {
        const bf8_t a = load_bf8(AT + (size_t)(m0 + r) * B + s + 8 * kq);
        const bf8_t b = load_bf8(DT + (size_t)(n0 + r) * B + s + 8 * kq);
        acc = mma_bf16(a, b, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int m = m0 + 4 * rq + v, n = n0 + c;
        if (m < mlim && n < nlim) atomicAdd(&grad[go + m * ldn + n], acc[v]);
    }
}

// ------------------------------------------------------------------ Adam
__global__ void k_mlp_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gi = g[t];
    const float mi = b1 * m[t] + (1.0f - b1) * gi;
    const float vi = b2 * v[t] + (1.0f - b2) * gi * gi;
    m[t] = mi;
    v[t] = vi;
    th[t] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ----------------------------------------------- features of the solver
// Per shell and DOF kind (4 kinds x 3 components), sums of squares over
// free DOFs of u = q - qbar, b and dprev: part[blk][12], index 4*quantity + kind.
__global__ __launch_bounds__(256) void k_feat_scale_part(const int* __restrict__ blk_row0,
                                                         const int* __restrict__ blk_row1, const double* __restrict__ q,
                                                         const double* __restrict__ qbar, const double* __restrict__ b,
                                                         const double* __restrict__ dprev,
                                                         const uint16_t* __restrict__ fm, double* __restrict__ part) {
    __shared__ double red[12][256];
    double s[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] = 0.0;
    const int r0 = blk_row0[blockIdx.x], r1 = blk_row1[blockIdx.x];
    for (int e = r0 * 12 + threadIdx.x; e < r1 * 12; e += blockDim.x) {
        const int node = e / 12, w = e % 12, kind = w / 3;
        if (!((fm[node] >> w) & 1)) continue;
        const double u = q[e] - qbar[e];
        s[kind] += u * u;
        s[4 + kind] += b[e] * b[e];
        s[8 + kind] += dprev[e] * dprev[e];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int wd = blockDim.x / 2; wd > 0; wd >>= 1) {
        if ((int)threadIdx.x < wd)
            for (int k = 0; k < 12; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + wd];
        __syncthreads();
    }
    if (threadIdx.x < 12) part[12 * (size_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Scales per shell: RMS per kind over that kind's free DOFs; 1 where the
// quantity is zero (the feature is then 0).  scale[s*12 + 4*quantity + kind].
__global__ void k_feat_scale_fin(int nshell, const int* __restrict__ shell_blk0, const int* __restrict__ shell_nblk,
                                 const double* __restrict__ part, const int* __restrict__ cnt_kind,
                                 float* __restrict__ scale) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nshell * 12) return;
    const int s = t / 12, k = t % 12;
    double v = 0.0;
    for (int i = 0; i < shell_nblk[s]; ++i) v += part[12 * (size_t)(shell_blk0[s] + i) + k];
    const int n = cnt_kind[4 * s + k % 4];
    const double rms = n > 0 ? sqrt(v / n) : 0.0;
    scale[t] = (float)(rms > 1e-300 ? rms : 1.0);
}

// 60 features of node `node` (per kind scales sc): u / s_u, b / s_b,
// dprev / s_d, and the 3x3 grid stencil L b / s_b, L dprev / s_d with
// (L f)[n] = (4 sum over the edge neighbours + sum over the diagonal ones) / 20
// - f[n]; nbr: the node's 8 neighbours (edge ones at 1, 3, 4, 6), a missing
// neighbour given as the node itself.
__device__ __forceinline__ void node_features(int node, const double* q, const double* qbar, const double* b,
                                              const double* dprev, const int* __restrict__ nbr8, const float* sc,
                                              float* f) {
    int nb[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) nb[k] = nbr8[8 * (size_t)node + k];
#pragma unroll
    for (int w = 0; w < 12; ++w) {
        const size_t e = (size_t)node * 12 + w;
        const int kind = w / 3;
        f[w] = (float)((q[e] - qbar[e]) / sc[kind]);
        f[12 + w] = (float)(b[e] / sc[4 + kind]);
        f[24 + w] = (float)(dprev[e] / sc[8 + kind]);
        double sb = 0.0, sd = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double wk = (k == 1 || k == 3 || k == 4 || k == 6) ? 4.0 : 1.0;
            sb += wk * b[(size_t)nb[k] * 12 + w];
            sd += wk * dprev[(size_t)nb[k] * 12 + w];
        }
        f[36 + w] = (float)((sb / 20.0 - b[e]) / sc[4 + kind]);
        f[48 + w] = (float)((sd / 20.0 - dprev[e]) / sc[8 + kind]);
    }
}

// Record (features, target) of sampled nodes after a time step:
// target = (d - dprev) / s_d per kind, d the step's correction.  Sample j of
// shell s goes to row sbase[s] + j of the outputs (shells with sbase < 0
// are skipped); its node is picked by a hash of (seed, s, j).
__global__ void k_mlp_record(int nshell, int K, unsigned long long seed, const ShellParams* __restrict__ shells,
                             const long long* __restrict__ sbase, const double* __restrict__ q,
                             const double* __restrict__ qbar, const double* __restrict__ b,
                             const double* __restrict__ dprev, const double* __restrict__ d,
                             const int* __restrict__ nbr8, const float* __restrict__ scale,
                             float* __restrict__ feat_out, float* __restrict__ tgt_out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nshell * K) return;
    const int s = t / K;
    if (sbase[s] < 0) return;
    const long long row = sbase[s] + t % K;
    float* o = feat_out + row * MLP_IN;
    float* ot = tgt_out + row * MLP_OUT;
    const int n0 = shells[s].node_begin, nn = shells[s].node_end - n0;
    // splitmix64 of (seed, shell, j) picks the node
    unsigned long long x = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(t + 1);
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    const int node = n0 + (int)(x % (unsigned long long)nn);
    const float* sc = scale + 12 * s;
    float f[MLP_IN];
    node_features(node, q, qbar, b, dprev, nbr8, sc, f);
    for (int k = 0; k < MLP_IN; ++k) o[k] = f[k];
    for (int w = 0; w < 12; ++w) {
        const size_t e = (size_t)node * 12 + w;
        ot[w] = (float)((d[e] - dprev[e]) / sc[8 + w / 3]);
    }
}

// The network's correction of the extrapolated step on free DOFs of
// flagged shells (0 elsewhere): w = s_d * y(features).
__global__ __launch_bounds__(256) void k_mlp_guess(int nnodes, const float* __restrict__ th,
                                                   const __bf16* __restrict__ w, const int* __restrict__ node_shell,
                                                   const int* __restrict__ flag, const double* __restrict__ q,
                                                   const double* __restrict__ qbar, const double* __restrict__ b,
                                                   const double* __restrict__ dprev, const uint16_t* __restrict__ fm,
                                                   const int* __restrict__ nbr8, const float* __restrict__ scale,
                                                   double* __restrict__ corr) {
    __shared__ MlpTileLds lds[MLP_WAVES];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    MlpTileLds& L = lds[wv];
    const int tile0 = (blockIdx.x * MLP_WAVES + wv) * 16;
    if (lane < 16) {
        const int node = tile0 + lane;
        float f[MLP_IN];
        if (node < nnodes) node_features(node, q, qbar, b, dprev, nbr8, scale + 12 * node_shell[node], f);
        for (int k = 0; k < K1P; ++k) L.X[lane * K1P + k] = (__bf16)((k < MLP_IN && node < nnodes) ? f[k] : 0.0f);
    }
    __syncthreads();
    mlp_forward_tile(th, w, L);
    for (int e = lane; e < 16 * 12; e += 64) {
        const int r = e / 12, k = e % 12, node = tile0 + r;
        if (node >= nnodes) continue;
        const int s = node_shell[node];
        const bool on = flag[s] && ((fm[node] >> k) & 1);
        corr[(size_t)node * 12 + k] = on ? (double)scale[12 * s + 8 + k / 3] * (double)L.Y[r * N3P + k] : 0.0;
    }
}

// y = x + c[2s] d1 + c[2s+1] d2 on the nodes of shell s.
__global__ void k_axpy2_shell(int n, const double* __restrict__ x, const double* __restrict__ d1,
                              const double* __restrict__ d2, const double* __restrict__ coef,
                              const int* __restrict__ node_shell, double* __restrict__ y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int s = node_shell[t / 12];
    const double c1 = coef[2 * s], c2 = coef[2 * s + 1];
    y[t] = x[t] + (c1 != 0.0 ? c1 * d1[t] : 0.0) + (c2 != 0.0 ? c2 * d2[t] : 0.0);
}

// out = a - b on free DOFs of flagged shells, 0 on their prescribed DOFs;
// other shells' entries are left as they are.
__global__ void k_masked_diff(int n, const double* __restrict__ a, const double* __restrict__ b,
                              const uint16_t* __restrict__ fm, const int* __restrict__ node_shell,
                              const int* __restrict__ flag, double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int node = t / 12;
    if (!flag[node_shell[node]]) return;
    out[t] = ((fm[node] >> (t % 12)) & 1) ? a[t] - b[t] : 0.0;
}

// Mini-batch sample indices: splitmix64 of (seed, i) modulo n.
__global__ void k_sample_idx(long long n, int batch, unsigned long long seed, long long* __restrict__ idx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch) return;
    unsigned long long x = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    idx[i] = (long long)(x % (unsigned long long)n);
}

// ------------------------------------------------------------ launchers
void launch_mlp_pack(hipStream_t st, const float* th, void* w) {
    hipLaunchKernelGGL(k_mlp_pack, dim3((BF_TOTAL + 255) / 256), dim3(256), 0, st, th, (__bf16*)w);
}

void launch_mlp_forward(hipStream_t st, const float* th, const void* w, const float* feat, float* out, long long n) {
    const long long tiles = (n + 15) / 16;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((tiles + MLP_WAVES - 1) / MLP_WAVES)), dim3(256), 0, st, th,
                       (const __bf16*)w, feat, out, n);
}

size_t mlp_train_work_bytes(int B) { return (size_t)B * (K1P + 2 * MLP_H + K3BP + 2 * MLP_H) * sizeof(__bf16); }

void launch_mlp_grad(hipStream_t st, const float* th, const void* w, const float* feat, const float* tgt,
                     const long long* idx, int B, void* work, float* grad, double* loss) {
    __bf16* p = (__bf16*)work;
    TrainWork W;
    W.XT = p;
    W.H1T = W.XT + (size_t)K1P * B;
    W.H2T = W.H1T + (size_t)MLP_H * B;
    W.DYT = W.H2T + (size_t)MLP_H * B;
    W.D2T = W.DYT + (size_t)K3BP * B;
    W.D1T = W.D2T + (size_t)MLP_H * B;
    const int tiles = B / 16;
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((tiles + MLP_WAVES - 1) / MLP_WAVES), dim3(256), 0, st, th,
                       (const __bf16*)w, feat, tgt, idx, B, W, grad, loss);
    const int slice = 256;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(WG_TILES, (B + slice - 1) / slice), dim3(64), 0, st, W, B, slice, grad);
}

void launch_mlp_adam(hipStream_t st, float* th, const float* g, float* m, float* v, int n, float lr, int step) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((n + 255) / 256), dim3(256), 0, st, th, g, m, v, n, lr, b1, b2, 1e-8f, c1,
                       c2);
}

void launch_feat_scale(hipStream_t st, const RowBlocks& rb, int nshell, const double* q, const double* qbar,
                       const double* b, const double* dprev, const uint16_t* fm, double* part, const int* cnt_kind,
                       float* scale) {
    hipLaunchKernelGGL(k_feat_scale_part, dim3(rb.nblk), dim3(256), 0, st, rb.blk_row0, rb.blk_row1, q, qbar, b,
                       dprev, fm, part);
    hipLaunchKernelGGL(k_feat_scale_fin, dim3((nshell * 12 + 255) / 256), dim3(256), 0, st, nshell, rb.shell_blk0,
                       rb.shell_nblk, part, cnt_kind, scale);
}

void launch_mlp_record(hipStream_t st, int nshell, int K, unsigned long long seed, const ShellParams* shells,
                       const long long* sbase, const double* q, const double* qbar, const double* b,
                       const double* dprev, const double* d, const int* nbr8, const float* scale, float* feat_out,
                       float* tgt_out) {
    const int n = nshell * K;
    hipLaunchKernelGGL(k_mlp_record, dim3((n + 127) / 128), dim3(128), 0, st, nshell, K, seed, shells, sbase, q, qbar,
                       b, dprev, d, nbr8, scale, feat_out, tgt_out);
}

void launch_sample_idx(hipStream_t st, long long n, int batch, unsigned long long seed, long long* idx) {
    hipLaunchKernelGGL(k_sample_idx, dim3((batch + 255) / 256), dim3(256), 0, st, n, batch, seed, idx);
}

void launch_mlp_guess(hipStream_t st, int nnodes, const float* th, const void* w, const int* node_shell,
                      const int* flag, const double* q, const double* qbar, const double* b, const double* dprev,
                      const uint16_t* fm, const int* nbr8, const float* scale, double* corr) {
    const int tiles = (nnodes + 15) / 16;
    hipLaunchKernelGGL(k_mlp_guess, dim3((tiles + MLP_WAVES - 1) / MLP_WAVES), dim3(256), 0, st, nnodes, th,
                       (const __bf16*)w, node_shell, flag, q, qbar, b, dprev, fm, nbr8, scale, corr);
}

void launch_axpy2_shell(hipStream_t st, int nnodes, const double* x, const double* d1, const double* d2,
                        const double* coef, const int* node_shell, double* y) {
    const int n = nnodes * 12;
    hipLaunchKernelGGL(k_axpy2_shell, dim3((n + 255) / 256), dim3(256), 0, st, n, x, d1, d2, coef, node_shell, y);
}

void launch_masked_diff(hipStream_t st, int nnodes, const double* a, const double* b, const uint16_t* fm,
                        const int* node_shell, const int* flag, double* out) {
    const int n = nnodes * 12;
    hipLaunchKernelGGL(k_masked_diff, dim3((n + 255) / 256), dim3(256), 0, st, n, a, b, fm, node_shell, flag, out);
}

}  // namespace bhem
