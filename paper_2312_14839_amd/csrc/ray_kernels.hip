// Ray--patch intersection on bicubic Hermite shells (Sec. 5).
//
// k_bezier rewrites every patch in the Bernstein basis (Sec. 5, first
// equation).  k_ray_cast is the static ray--patch intersection of Sec. 5.1,
// one ray per lane:
//   * the candidates of a ray are parameter rectangles of its patches, held
//     in a private binary min-heap keyed by the smallest tau at which the ray
//     enters the rectangle's control-point bounding box (Eq. ineqray);
//   * a rectangle's control points are not stored: they are recomputed from
//     the patch's 16 points by blossoming (the Bezier coefficients of the
//     piece over [a, b] are the blossom values f(a,a,a), f(a,a,b), f(a,b,b),
//     f(b,b,b)), so a heap entry is 52 bytes instead of 436;
//   * the popped rectangle is cut into the quadrants of its midpoint, or,
//     when Newton's method from its centre converges to a hit inside it,
//     into the four rectangles around an abandoned box about the hit
//     (Figs. submid and subany);
//   * a rectangle whose box diagonal is at most eps |d| is an answer: its
//     tau interval is then narrower than eps.
// Scenes of up to RAY_LDS_PATCHES patches are staged in LDS (control points
// and root boxes) once per block.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace bhem {

// ------------------------------------------------------------ Bezier form
// Bernstein coefficient k of a cubic Hermite segment with end data
// (f0, f0', f1, f1') in xi units over a cell of width h: b0 = f0,
// b1 = f0 + h f0'/3, b2 = f1 - h f1'/3, b3 = f1.  w[2e + r] is the weight of
// the datum of end e and derivative order r.
__device__ inline void bern_weights(int k, double h, double w[4]) {
    w[0] = (k <= 1) ? 1.0 : 0.0;
    w[1] = (k == 1) ? h / 3.0 : 0.0;
    w[2] = (k >= 2) ? 1.0 : 0.0;
    w[3] = (k == 2) ? -h / 3.0 : 0.0;
}

// One thread per (patch, i): the 12 values p_i0..p_i3 (xyz).  Corner
// e1 + 2 e2 holds the node (i + e1, j + e2) of the patch; its DOF kind
// r1 + 2 r2 is the derivative of order r1 in xi1 and r2 in xi2.
__global__ void __launch_bounds__(256) k_bezier(int npatch, const int4* __restrict__ patch_nodes,
                                                const int* __restrict__ patch_shell,
                                                const ShellParams* __restrict__ shells, const double* __restrict__ q,
                                                double* __restrict__ ctrl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * npatch) return;
    const int p = t >> 2, i = t & 3;
    const int4 nd = patch_nodes[p];
    const int corner[4] = {nd.x, nd.y, nd.z, nd.w};
    const ShellParams& sp = shells[patch_shell[p]];
    double wu[4];
    bern_weights(i, sp.dxi1, wu);
    for (int j = 0; j < 4; ++j) {
        double wv[4];
        bern_weights(j, sp.dxi2, wv);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 4; ++a) {
            if (wu[a] == 0.0) continue;
            for (int b = 0; b < 4; ++b) {
                if (wv[b] == 0.0) continue;
                const double w = wu[a] * wv[b];
                const double* x = q + 12 * (long long)corner[(a >> 1) + 2 * (b >> 1)] + 3 * ((a & 1) + 2 * (b & 1));
                acc[0] += w * x[0];
                acc[1] += w * x[1];
                acc[2] += w * x[2];
            }
        }
        double* out = ctrl + 3 * ((long long)(4 * p + i) * 4 + j);
        out[0] = acc[0];
        out[1] = acc[1];
        out[2] = acc[2];
    }
}

void launch_bezier(hipStream_t st, int npatch, const int4* patch_nodes, const int* patch_shell,
                   const ShellParams* shells, const double* q, double* ctrl) {
    if (npatch <= 0) return;
    const long long thr = 4LL * npatch;
    hipLaunchKernelGGL(k_bezier, dim3((unsigned)((thr + 255) / 256)), dim3(256), 0, st, npatch, patch_nodes,
                       patch_shell, shells, q, ctrl);
}

// ------------------------------------------------------------ ray casting
__device__ inline double lerp(double p, double q, double t) { return fma(t, q - p, p); }

// Bezier coefficients of the cubic with coefficients p0..p3 restricted to
// [a, b]: the blossom values f(a,a,a), f(a,a,b), f(a,b,b), f(b,b,b).
__device__ inline void blossom4(double p0, double p1, double p2, double p3, double a, double b, double q[4]) {
    const double A0 = lerp(p0, p1, a), A1 = lerp(p1, p2, a), A2 = lerp(p2, p3, a);
    const double B0 = lerp(p0, p1, b), B1 = lerp(p1, p2, b), B2 = lerp(p2, p3, b);
    const double BB0 = lerp(B0, B1, b), BB1 = lerp(B1, B2, b);
    q[0] = lerp(lerp(A0, A1, a), lerp(A1, A2, a), a);
    q[1] = lerp(lerp(B0, B1, a), lerp(B1, B2, a), a);
    q[2] = lerp(BB0, BB1, a);
    q[3] = lerp(BB0, BB1, b);
}

// Bounding box of the control points of patch cp over [u0,u1] x [v0,v1].
__device__ inline void sub_box(const double* cp, double u0, double u1, double v0, double v1, double lo[3],
                               double hi[3]) {
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        double U[4][4];  // [i][j] after the restriction along u
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double qq[4];
            blossom4(cp[(0 * 4 + j) * 3 + c], cp[(1 * 4 + j) * 3 + c], cp[(2 * 4 + j) * 3 + c],
                     cp[(3 * 4 + j) * 3 + c], u0, u1, qq);
#pragma unroll
            for (int i = 0; i < 4; ++i) U[i][j] = qq[i];
        }
        double l = INFINITY, h = -INFINITY;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double qq[4];
            blossom4(U[i][0], U[i][1], U[i][2], U[i][3], v0, v1, qq);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                l = fmin(l, qq[k]);
                h = fmax(h, qq[k]);
            }
        }
        lo[c] = l;
        hi[c] = h;
    }
}

__device__ inline void whole_box(const double* cp, double lo[3], double hi[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double l = cp[c], h = l;
#pragma unroll
        for (int k = 1; k < 16; ++k) {
            l = fmin(l, cp[3 * k + c]);
            h = fmax(h, cp[3 * k + c]);
        }
        lo[c] = l;
        hi[c] = h;
    }
}

struct Ray {
    double o[3], d[3];
};

// Slab test of Eq. ineqray: the tau >= 0 for which o + tau d is inside
// [lo, hi]; false when empty.  diag: the box's diagonal.
__device__ inline bool slab(const Ray& r, const double lo[3], const double hi[3], double& tlo, double& thi,
                            double& diag) {
    tlo = 0.0;
    thi = INFINITY;
    double d2 = 0.0;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double e = hi[c] - lo[c];
        d2 = fma(e, e, d2);
        if (r.d[c] == 0.0) {
            ok = ok && r.o[c] >= lo[c] && r.o[c] <= hi[c];
        } else {
            const double t1 = (lo[c] - r.o[c]) / r.d[c], t2 = (hi[c] - r.o[c]) / r.d[c];
            tlo = fmax(tlo, fmin(t1, t2));
            thi = fmin(thi, fmax(t1, t2));
        }
    }
    diag = sqrt(d2);
    return ok && tlo <= thi;
}

// x, x_u, x_v of patch cp at (u, v), one coordinate per pass (the loop is
// kept rolled so that the 48 control points are not all held at once).
__device__ inline void surf_eval(const double* cp, double u, double v, double x[3], double xu[3], double xv[3]) {
    const double su = 1.0 - u, sv = 1.0 - v;
    const double Bu[4] = {su * su * su, 3.0 * u * su * su, 3.0 * u * u * su, u * u * u};
    const double Bv[4] = {sv * sv * sv, 3.0 * v * sv * sv, 3.0 * v * v * sv, v * v * v};
    // derivatives: 3 * (degree-2 Bernstein) times the forward differences
    const double Du[3] = {3.0 * su * su, 6.0 * u * su, 3.0 * u * u};
    const double Dv[3] = {3.0 * sv * sv, 6.0 * v * sv, 3.0 * v * v};
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        double s[4], t[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double p0 = cp[(4 * i + 0) * 3 + c], p1 = cp[(4 * i + 1) * 3 + c], p2 = cp[(4 * i + 2) * 3 + c],
                         p3 = cp[(4 * i + 3) * 3 + c];
            s[i] = Bv[0] * p0 + Bv[1] * p1 + Bv[2] * p2 + Bv[3] * p3;
            t[i] = Dv[0] * (p1 - p0) + Dv[1] * (p2 - p1) + Dv[2] * (p3 - p2);
        }
        const double X = Bu[0] * s[0] + Bu[1] * s[1] + Bu[2] * s[2] + Bu[3] * s[3];
        const double XU = Du[0] * (s[1] - s[0]) + Du[1] * (s[2] - s[1]) + Du[2] * (s[3] - s[2]);
        const double XV = Bu[0] * t[0] + Bu[1] * t[1] + Bu[2] * t[2] + Bu[3] * t[3];
        if (c == 0) {
            x[0] = X;
            xu[0] = XU;
            xv[0] = XV;
        } else if (c == 1) {
            x[1] = X;
            xu[1] = XU;
            xv[1] = XV;
        } else {
            x[2] = X;
            xu[2] = XU;
            xv[2] = XV;
        }
    }
}

__device__ inline void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Newton's method on x(u, v) - o - tau d = 0 from (u, v), tau starting at
// the projection of x(u, v) - o on d.  Each step solves [x_u x_v -d] delta
// = -F by triple products.
__device__ bool newton_hit(const double* cp, const Ray& r, int iters, double tol, double& u, double& v,
                           double& tau) {
    double x[3], xu[3], xv[3];
    surf_eval(cp, u, v, x, xu, xv);
    const double tol2 = tol * tol;
    {
        const double w[3] = {x[0] - r.o[0], x[1] - r.o[1], x[2] - r.o[2]};
        tau = dot3(w, r.d) / dot3(r.d, r.d);
    }
    for (int it = 0;; ++it) {
        double F[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) F[c] = x[c] - r.o[c] - tau * r.d[c];
        if (dot3(F, F) <= tol2) return isfinite(u + v + tau);
        if (it == iters) return false;
        const double nd[3] = {-r.d[0], -r.d[1], -r.d[2]};
        const double rhs[3] = {-F[0], -F[1], -F[2]};
        double bc[3], rc[3], br[3];
        cross3(xv, nd, bc);
        const double det = dot3(xu, bc);
        if (det == 0.0 || !isfinite(det)) return false;
        cross3(rhs, nd, rc);
        cross3(xv, rhs, br);
        const double inv = 1.0 / det;
        u += dot3(rhs, bc) * inv;
        v += dot3(xu, rc) * inv;
        tau += dot3(xu, br) * inv;
        if (!isfinite(u + v + tau)) return false;
        surf_eval(cp, u, v, x, xu, xv);
    }
}

// Private min-heap of candidate rectangles.  tag = patch | depth << 24 |
// answer << 30 (answer: box small enough to end the subdivision).
struct Heap {
    double key[RAY_HEAP_MAX], thi[RAY_HEAP_MAX];
    double rect[RAY_HEAP_MAX][4];
    int tag[RAY_HEAP_MAX];
    int n;

    __device__ void push(double k, double th, const double rc[4], int tg) {
        int i = n++;
        while (i > 0) {
            const int par = (i - 1) >> 1;
            if (key[par] <= k) break;
            key[i] = key[par];
            thi[i] = thi[par];
            rect[i][0] = rect[par][0];
            rect[i][1] = rect[par][1];
            rect[i][2] = rect[par][2];
            rect[i][3] = rect[par][3];
            tag[i] = tag[par];
            i = par;
        }
        key[i] = k;
        thi[i] = th;
        rect[i][0] = rc[0];
        rect[i][1] = rc[1];
        rect[i][2] = rc[2];
        rect[i][3] = rc[3];
        tag[i] = tg;
    }

    // Removes the root into (k, th, rc, tg).
    __device__ void pop(double& k, double& th, double rc[4], int& tg) {
        k = key[0];
        th = thi[0];
        rc[0] = rect[0][0];
        rc[1] = rect[0][1];
        rc[2] = rect[0][2];
        rc[3] = rect[0][3];
        tg = tag[0];
        const int m = --n;
        if (m == 0) return;
        const double lk = key[m];
        int i = 0;
        for (;;) {
            int c = 2 * i + 1;
            if (c >= m) break;
            if (c + 1 < m && key[c + 1] < key[c]) ++c;
            if (lk <= key[c]) break;
            key[i] = key[c];
            thi[i] = thi[c];
            rect[i][0] = rect[c][0];
            rect[i][1] = rect[c][1];
            rect[i][2] = rect[c][2];
            rect[i][3] = rect[c][3];
            tag[i] = tag[c];
            i = c;
        }
        key[i] = lk;
        thi[i] = thi[m];
        rect[i][0] = rect[m][0];
        rect[i][1] = rect[m][1];
        rect[i][2] = rect[m][2];
        rect[i][3] = rect[m][3];
        tag[i] = tag[m];
    }
};

// Rays are handed out per lane: a block owns `chunk` consecutive rays and
// each lane takes the next unstarted one from an LDS counter when its ray is
// done, so a lane held by a long search (a ray grazing a silhouette can
// need thousands of candidates) does not keep the other lanes of its wave
// idle.  Each loop trip either starts a ray (root boxes of every patch) or
// examines one candidate.
template <bool LDS>
__global__ void __launch_bounds__(256) k_ray_cast(const double* __restrict__ ctrl, int npatch,
                                                  const double* __restrict__ rays, long long nrays, int chunk,
                                                  RayParams o, double* __restrict__ hit, int* __restrict__ patch_out,
                                                  int* __restrict__ pops_out) {
    extern __shared__ double lds[];
    __shared__ int s_next;
    const double* cps = ctrl;
    if (threadIdx.x == 0) s_next = 0;
    if (LDS) {
        // control points, then the root boxes [P][6]
        for (int k = threadIdx.x; k < 48 * npatch; k += blockDim.x) lds[k] = ctrl[k];
        __syncthreads();
        for (int p = threadIdx.x; p < npatch; p += blockDim.x) {
            double lo[3], hi[3];
            whole_box(lds + 48 * p, lo, hi);
            double* b = lds + 48 * npatch + 6 * p;
            b[0] = lo[0];
            b[1] = lo[1];
            b[2] = lo[2];
            b[3] = hi[0];
            b[4] = hi[1];
            b[5] = hi[2];
        }
        cps = lds;
    }
    __syncthreads();
    const long long base = (long long)blockIdx.x * chunk;
    const int cnt = (int)(nrays - base < chunk ? nrays - base : chunk);

    Heap hp;
    Ray r;
    double small = 0.0, best = INFINITY, bu = 0.0, bv = 0.0;
    long long rid = 0;
    int bp = -1, pops = 0;
    bool active = false, full = false;

    for (;;) {
        if (!active) {
            const int k = atomicAdd(&s_next, 1);
            if (k >= cnt) break;
            rid = base + k;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                r.o[c] = rays[6 * rid + c];
                r.d[c] = rays[6 * rid + 3 + c];
            }
            const double dn = sqrt(dot3(r.d, r.d));
            if (!(dn > 0.0) || !isfinite(dn) || !isfinite(r.o[0] + r.o[1] + r.o[2])) {
                hit[3 * rid] = INFINITY;
                hit[3 * rid + 1] = 0.0;
                hit[3 * rid + 2] = 0.0;
                patch_out[rid] = -3;
                if (pops_out) pops_out[rid] = 0;
                continue;
            }
            small = o.eps * dn;
            hp.n = 0;
            best = INFINITY;
            bu = bv = 0.0;
            bp = -1;
            pops = 0;
            full = false;
            for (int p = 0; p < npatch && !full; ++p) {
                double lo[3], hi[3];
                if (LDS) {
                    const double* b = lds + 48 * npatch + 6 * p;
                    lo[0] = b[0];
                    lo[1] = b[1];
                    lo[2] = b[2];
                    hi[0] = b[3];
                    hi[1] = b[4];
                    hi[2] = b[5];
                } else {
                    whole_box(cps + 48 * p, lo, hi);
                }
                double tlo, thi, diag;
                if (!slab(r, lo, hi, tlo, thi, diag)) continue;
                if (hp.n == o.heap_cap) {
                    full = true;
                    break;
                }
                const double rc[4] = {0.0, 1.0, 0.0, 1.0};
                hp.push(tlo, thi, rc, p | ((diag <= small || o.max_depth == 0) ? (1 << 30) : 0));
            }
            if (full || hp.n == 0) {  // no candidate (a miss) or no room for them
                hit[3 * rid] = INFINITY;
                hit[3 * rid + 1] = 0.0;
                hit[3 * rid + 2] = 0.0;
                patch_out[rid] = full ? -2 : -1;
                if (pops_out) pops_out[rid] = 0;
                continue;
            }
            active = true;
        } else {
            // one candidate (the heap is not empty); `done` ends the search
            bool done = false;
            if (pops == RAY_MAX_POPS) {  // search budget spent: no result, like a full heap
                full = true;
            } else {
                double tlo, thi, rc[4];
                int tg;
                hp.pop(tlo, thi, rc, tg);
                ++pops;
                const int patch = tg & 0xFFFFFF, depth = (tg >> 24) & 63;
                if (!(tlo < best)) {
                    done = true;
                } else if (tg & (1 << 30)) {
                    const double t = 0.5 * (tlo + thi);
                    if (t < best) {
                        best = t;
                        bu = 0.5 * (rc[0] + rc[1]);
                        bv = 0.5 * (rc[2] + rc[3]);
                        bp = patch;
                    }
                    done = o.newton_iters == 0;
                } else {
                    const double* cp = cps + 48 * patch;
                    double cu = 0.5 * (rc[0] + rc[1]), cv = 0.5 * (rc[2] + rc[3]);
                    double ua = cu, ub = cu, va = cv, vb = cv;
                    if (o.newton_iters > 0) {
                        double u = cu, v = cv, tau;
                        if (newton_hit(cp, r, o.newton_iters, o.newton_tol, u, v, tau) && u >= rc[0] &&
                            u <= rc[1] && v >= rc[2] && v <= rc[3] && tau > 0.0) {
                            if (tau < best) {
                                best = tau;
                                bu = u;
                                bv = v;
                                bp = patch;
                            }
                            const double hu = o.hole * (rc[1] - rc[0]), hv = o.hole * (rc[3] - rc[2]);
                            ua = fmax(rc[0], u - hu);
                            ub = fmin(rc[1], u + hu);
                            va = fmax(rc[2], v - hv);
                            vb = fmin(rc[3], v + hv);
                        }
                    }
                    // quadrants of the midpoint, or the pinwheel around the
                    // abandoned box [ua, ub] x [va, vb]: left, top, bottom, right
                    const double kids[4][4] = {{rc[0], ua, va, rc[3]},
                                               {ua, rc[1], vb, rc[3]},
                                               {rc[0], ub, rc[2], va},
                                               {ub, rc[1], rc[2], vb}};
                    const int ntag = patch | ((depth + 1) << 24) | ((depth + 1 >= o.max_depth) ? (1 << 30) : 0);
#pragma unroll 1
                    for (int k = 0; k < 4; ++k) {
                        if (!(kids[k][1] > kids[k][0]) || !(kids[k][3] > kids[k][2])) continue;
                        double lo[3], hi[3];
                        sub_box(cp, kids[k][0], kids[k][1], kids[k][2], kids[k][3], lo, hi);
                        double klo, khi, diag;
                        if (!slab(r, lo, hi, klo, khi, diag) || !(klo < best)) continue;
                        if (hp.n == o.heap_cap) {
                            full = true;
                            break;
                        }
                        hp.push(klo, khi, kids[k], ntag | (diag <= small ? (1 << 30) : 0));
                    }
                }
            }
            if (done || full || hp.n == 0) {
                hit[3 * rid] = full ? INFINITY : (bp >= 0 ? best : INFINITY);
                hit[3 * rid + 1] = bu;
                hit[3 * rid + 2] = bv;
                patch_out[rid] = full ? -2 : bp;
                if (pops_out) pops_out[rid] = pops;
                active = false;
            }
        }
    }
}

void launch_ray_cast(hipStream_t st, const double* ctrl, int npatch, const double* rays, long long nrays,
                     const RayParams& o, double* hit, int* patch, int* pops) {
    if (nrays <= 0) return;
    const int chunk = 256 * RAY_CHUNK_PER_LANE;
    const unsigned nb = (unsigned)((nrays + chunk - 1) / chunk);
    if (npatch <= RAY_LDS_PATCHES) {
        const size_t lds = sizeof(double) * 54 * (size_t)npatch;
        hipLaunchKernelGGL(k_ray_cast<true>, dim3(nb), dim3(256), lds, st, ctrl, npatch, rays, nrays, chunk, o, hit,
                           patch, pops);
    } else {
        hipLaunchKernelGGL(k_ray_cast<false>, dim3(nb), dim3(256), 0, st, ctrl, npatch, rays, nrays, chunk, o, hit,
                           patch, pops);
    }
}

}  // namespace bhem
