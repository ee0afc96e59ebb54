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

#include <algorithm>
#include <cmath>
#include <mutex>

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

// Newton's method from the centre of candidate rc (accelerated form) and
// the four sub-rectangles: the quadrants of the midpoint, or the pinwheel
// around the abandoned box about a Newton hit inside rc.  Each
// sub-rectangle whose box the ray enters before `best` goes to
// emit(key, thi, rect, tag); emit returns false to stop.  A Newton hit is
// returned in (ht, hu, hv), ht = INF when there is none.
template <class Emit>
__device__ inline void expand(const double* cp, const Ray& r, const RayParams& o, double small, double best,
                              const double rc[4], int patch, int depth, double& ht, double& hu, double& hv,
                              Emit&& emit) {
    double cu = 0.5 * (rc[0] + rc[1]), cv = 0.5 * (rc[2] + rc[3]);
    double ua = cu, ub = cu, va = cv, vb = cv;
    ht = INFINITY;
    if (o.newton_iters > 0) {
        double u = cu, v = cv, tau;
        if (newton_hit(cp, r, o.newton_iters, o.newton_tol, u, v, tau) && u >= rc[0] && u <= rc[1] && v >= rc[2] &&
            v <= rc[3] && tau > 0.0) {
            ht = tau;
            hu = u;
            hv = v;
            best = fmin(best, tau);
            const double hw = o.hole * (rc[1] - rc[0]), hh = o.hole * (rc[3] - rc[2]);
            ua = fmax(rc[0], u - hw);
            ub = fmin(rc[1], u + hw);
            va = fmax(rc[2], v - hh);
            vb = fmin(rc[3], v + hh);
        }
    }
    // left, top, bottom, right of the box [ua, ub] x [va, vb]
    const double kids[4][4] = {
        {rc[0], ua, va, rc[3]}, {ua, rc[1], vb, rc[3]}, {rc[0], ub, rc[2], va}, {ub, rc[1], rc[2], vb}};
    const int ntag = patch | ((depth + 1) << 24) | ((depth + 1 >= o.max_depth) ? (1 << 30) : 0);
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
        if (!(kids[k][1] > kids[k][0]) || !(kids[k][3] > kids[k][2])) continue;
        double lo[3], hi[3];
        sub_box(cp, kids[k][0], kids[k][1], kids[k][2], kids[k][3], lo, hi);
        double klo, khi, diag;
        if (!slab(r, lo, hi, klo, khi, diag) || !(klo < best)) continue;
        if (!emit(klo, khi, kids[k], ntag | (diag <= small ? (1 << 30) : 0))) break;
    }
}

// A ray handed from the one-lane search to the cooperative one: its heap
// and its best answer so far.
struct LongRay {
    double best, bu, bv;
    int bp, pops, n;
    long long rid;
};
struct RayTail {
    int* count;          // long rays handed over
    int cap;             // slots
    LongRay* rays;       // [cap]
    double* key;         // [cap][RAY_HEAP_MAX]
    double* thi;         // [cap][RAY_HEAP_MAX]
    double* rect;        // [cap][RAY_HEAP_MAX][4]
    int* tag;            // [cap][RAY_HEAP_MAX]
    int budget;          // candidates a lane examines before handing its ray over (0: never)
};

__device__ inline void write_result(double* hit, int* patch_out, int* pops_out, long long rid, double t, double u,
                                    double v, int p, int pops) {
    hit[3 * rid] = t;
    hit[3 * rid + 1] = u;
    hit[3 * rid + 2] = v;
    patch_out[rid] = p;
    if (pops_out) pops_out[rid] = pops;
}

// Rays are handed out per lane: a block owns `chunk` consecutive rays and
// each lane takes the next unstarted one from an LDS counter when its ray is
// done, so that one lane held by a long search does not keep the rest of
// its wave idle.  Each loop trip either starts a ray (root boxes of every
// patch) or examines one candidate.  A ray still searching after
// `tail.budget` candidates (one grazing a silhouette can need tens of
// thousands) is handed to k_ray_tail, which works on it with a whole block.
template <bool LDS>
__global__ void __launch_bounds__(256) k_ray_cast(const double* __restrict__ ctrl, int npatch,
                                                  const double* __restrict__ rays, long long nrays, int chunk,
                                                  RayParams o, RayTail tail, double* __restrict__ hit,
                                                  int* __restrict__ patch_out, int* __restrict__ pops_out) {
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
    int bp = -1, pops = 0, budget = 0;
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
                write_result(hit, patch_out, pops_out, rid, INFINITY, 0.0, 0.0, -3, 0);
                continue;
            }
            small = o.eps * dn;
            hp.n = 0;
            best = INFINITY;
            bu = bv = 0.0;
            bp = -1;
            pops = 0;
            budget = tail.budget;
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
                write_result(hit, patch_out, pops_out, rid, INFINITY, 0.0, 0.0, full ? -2 : -1, 0);
                continue;
            }
            active = true;
            continue;
        }
        // one candidate (the heap is not empty); a ray that has used its
        // budget or whose heap may not take the next four children goes to
        // the cooperative search
        if (pops == budget || (budget > 0 && hp.n > o.heap_cap - 4)) {
            const int s = atomicAdd(tail.count, 1);
            if (s < tail.cap) {
                LongRay lr;
                lr.best = best;
                lr.bu = bu;
                lr.bv = bv;
                lr.bp = bp;
                lr.pops = pops;
                lr.n = hp.n;
                lr.rid = rid;
                tail.rays[s] = lr;
                for (int e = 0; e < hp.n; ++e) {
                    const long long q = (long long)s * RAY_HEAP_MAX + e;
                    tail.key[q] = hp.key[e];
                    tail.thi[q] = hp.thi[e];
                    tail.rect[4 * q] = hp.rect[e][0];
                    tail.rect[4 * q + 1] = hp.rect[e][1];
                    tail.rect[4 * q + 2] = hp.rect[e][2];
                    tail.rect[4 * q + 3] = hp.rect[e][3];
                    tail.tag[q] = hp.tag[e];
                }
                active = false;
                continue;
            }
            budget = 0;  // no slot left: finish here
        }
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
                double ht, hu, hv;
                expand(cps + 48 * patch, r, o, small, best, rc, patch, depth, ht, hu, hv,
                       [&](double k, double th, const double* kr, int tg2) {
                           if (hp.n == o.heap_cap) {
                               full = true;
                               return false;
                           }
                           hp.push(k, th, kr, tg2);
                           return true;
                       });
                if (ht < best) {
                    best = ht;
                    bu = hu;
                    bv = hv;
                    bp = patch;
                }
            }
        }
        if (done || full || hp.n == 0) {
            write_result(hit, patch_out, pops_out, rid, full ? INFINITY : (bp >= 0 ? best : INFINITY), bu, bv,
                         full ? -2 : bp, pops);
            active = false;
        }
    }
}

// ------------------------------------------------- dynamic intersection
// Sec. 5.2: control points p_ij + t v_ij and the point x0 + t w over
// [0, dt].  Per axis and per bound of Eq. ineqccd the feasible times are a
// prefix [0, L] and/or a suffix [R, dt] of the step (a union of half-lines
// a_ij + t b_ij <= 0); TimeSet intersects such sets.
struct TimeSet {
    double lo[8], hi[8];
    int n;
};

__device__ inline void meet_prefix_suffix(TimeSet& s, double L, double R, bool all, double dt) {
    if (all) return;
    TimeSet o;
    o.n = 0;
    const double pe = fmin(L, dt), ss = fmax(R, 0.0);
    const bool hp = L >= 0.0, hs = R <= dt;
    for (int k = 0; k < s.n; ++k) {
        // pieces in sorted order: the prefix part comes first
        if (hp) {
            const double a = s.lo[k], b = fmin(s.hi[k], pe);
            if (a <= b && o.n < 8) {
                o.lo[o.n] = a;
                o.hi[o.n] = b;
                ++o.n;
            }
        }
        if (hs) {
            const double a = fmax(s.lo[k], ss), b = s.hi[k];
            if (a <= b && o.n < 8) {
                if (o.n > 0 && a <= o.hi[o.n - 1]) {
                    o.hi[o.n - 1] = fmax(o.hi[o.n - 1], b);
                } else {
                    o.lo[o.n] = a;
                    o.hi[o.n] = b;
                    ++o.n;
                }
            }
        }
    }
    s = o;
}

// Earliest feasible time of the candidate [u0,u1] x [v0,v1] of a moving
// patch; false when there is none in [0, dt].
__device__ bool earliest_time(const double* cp, const double* cv, double u0, double u1, double v0, double v1,
                              const double x0[3], const double w[3], double dt, double& t0) {
    TimeSet ts;
    ts.n = 1;
    ts.lo[0] = 0.0;
    ts.hi[0] = dt;
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        double Lm = -1.0, Rm = 2.0 * dt + 1.0, Lp = -1.0, Rp = 2.0 * dt + 1.0;
        bool am = false, ap = false;
        double UP[4][4], UV[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double qp[4], qv[4];
            blossom4(cp[j * 3 + c], cp[(4 + j) * 3 + c], cp[(8 + j) * 3 + c], cp[(12 + j) * 3 + c], u0, u1, qp);
            blossom4(cv[j * 3 + c], cv[(4 + j) * 3 + c], cv[(8 + j) * 3 + c], cv[(12 + j) * 3 + c], u0, u1, qv);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                UP[i][j] = qp[i];
                UV[i][j] = qv[i];
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double qp[4], qv[4];
            blossom4(UP[i][0], UP[i][1], UP[i][2], UP[i][3], v0, v1, qp);
            blossom4(UV[i][0], UV[i][1], UV[i][2], UV[i][3], v0, v1, qv);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double a = qp[k] - x0[c], b = qv[k] - w[c];
                // some a + t b <= 0 (lower bound of the box)
                if (b > 0.0) Lm = fmax(Lm, -a / b);
                else if (b < 0.0) Rm = fmin(Rm, -a / b);
                else if (a <= 0.0) am = true;
                // some a + t b >= 0 (upper bound)
                if (b < 0.0) Lp = fmax(Lp, -a / b);
                else if (b > 0.0) Rp = fmin(Rp, -a / b);
                else if (a >= 0.0) ap = true;
            }
        }
        meet_prefix_suffix(ts, Lm, Rm, am, dt);
        meet_prefix_suffix(ts, Lp, Rp, ap, dt);
        if (ts.n == 0) return false;
    }
    t0 = ts.lo[0];
    return true;
}

// Diagonal of the control-point box of the candidate at time t.
__device__ double diag_at(const double* cp, const double* cv, double u0, double u1, double v0, double v1, double t) {
    double d2 = 0.0;
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        double U[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double qq[4];
            blossom4(fma(t, cv[j * 3 + c], cp[j * 3 + c]), fma(t, cv[(4 + j) * 3 + c], cp[(4 + j) * 3 + c]),
                     fma(t, cv[(8 + j) * 3 + c], cp[(8 + j) * 3 + c]), fma(t, cv[(12 + j) * 3 + c], cp[(12 + j) * 3 + c]),
                     u0, u1, qq);
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
        d2 = fma(h - l, h - l, d2);
    }
    return sqrt(d2);
}

// Newton's method on x(u,v) + t xdot(u,v) - x0 - t w = 0 from (u, v, t).
__device__ bool newton_ccd(const double* cp, const double* cv, const double x0[3], const double w[3], int iters,
                           double tol, double& u, double& v, double& t) {
    const double tol2 = tol * tol;
    for (int it = 0;; ++it) {
        double x[3], xu[3], xv[3], y[3], yu[3], yv[3];
        surf_eval(cp, u, v, x, xu, xv);
        surf_eval(cv, u, v, y, yu, yv);
        double F[3], a[3], b[3], c3[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            F[c] = fma(t, y[c] - w[c], x[c] - x0[c]);
            a[c] = fma(t, yu[c], xu[c]);
            b[c] = fma(t, yv[c], xv[c]);
            c3[c] = y[c] - w[c];
        }
        if (dot3(F, F) <= tol2) return isfinite(u + v + t);
        if (it == iters) return false;
        const double rhs[3] = {-F[0], -F[1], -F[2]};
        double bc[3], rc[3], br[3];
        cross3(b, c3, bc);
        const double det = dot3(a, bc);
        if (det == 0.0 || !isfinite(det)) return false;
        cross3(rhs, c3, rc);
        cross3(b, rhs, br);
        const double inv = 1.0 / det;
        u += dot3(rhs, bc) * inv;
        v += dot3(a, rc) * inv;
        t += dot3(a, br) * inv;
        if (!isfinite(u + v + t)) return false;
    }
}

// Newton's method (accelerated form) and the four sub-rectangles of a
// candidate of a moving patch, keyed by their earliest feasible times;
// emit and the Newton hit as in expand().
template <class Emit>
__device__ inline void expand_ccd(const double* cp, const double* cv, const double x0[3], const double w[3], double dt,
                                  const RayParams& o, double best, double t_key, const double rc[4], int patch,
                                  int depth, double& ht, double& hu, double& hv, Emit&& emit) {
    double cu = 0.5 * (rc[0] + rc[1]), cc = 0.5 * (rc[2] + rc[3]);
    double ua = cu, ub = cu, va = cc, vb = cc;
    ht = INFINITY;
    if (o.newton_iters > 0) {
        double u = cu, v = cc, t = t_key;
        if (newton_ccd(cp, cv, x0, w, o.newton_iters, o.newton_tol, u, v, t) && u >= rc[0] && u <= rc[1] &&
            v >= rc[2] && v <= rc[3] && t >= 0.0 && t <= dt) {
            ht = t;
            hu = u;
            hv = v;
            best = fmin(best, t);
            const double hw = o.hole * (rc[1] - rc[0]), hh = o.hole * (rc[3] - rc[2]);
            ua = fmax(rc[0], u - hw);
            ub = fmin(rc[1], u + hw);
            va = fmax(rc[2], v - hh);
            vb = fmin(rc[3], v + hh);
        }
    }
    const double kids[4][4] = {
        {rc[0], ua, va, rc[3]}, {ua, rc[1], vb, rc[3]}, {rc[0], ub, rc[2], va}, {ub, rc[1], rc[2], vb}};
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        if (!(kids[q][1] > kids[q][0]) || !(kids[q][3] > kids[q][2])) continue;
        double t0;
        if (!earliest_time(cp, cv, kids[q][0], kids[q][1], kids[q][2], kids[q][3], x0, w, dt, t0) || !(t0 < best))
            continue;
        if (!emit(t0, 0.0, kids[q], patch | ((depth + 1) << 24))) break;
    }
}

// One moving point per lane, handed out like the rays of k_ray_cast; the
// same heap search with keys = earliest feasible times and answers = boxes
// (at that time) with a diagonal <= eps; points past the budget, or whose
// heap nears capacity, go to k_ray_tail<true>.
template <bool LDS>
__global__ void __launch_bounds__(256) k_ccd(const double* __restrict__ ctrl_g, const double* __restrict__ vel_g,
                                             int npatch, const double* __restrict__ pts, long long npts, double dt,
                                             int chunk, RayParams o, RayTail tail, double* __restrict__ hit,
                                             int* __restrict__ patch_out, int* __restrict__ pops_out) {
    extern __shared__ double lds[];
    __shared__ int s_next;
    if (threadIdx.x == 0) s_next = 0;
    const double* ctrl = ctrl_g;
    const double* vel = vel_g;
    if (LDS) {  // positions, then velocities
        for (int k = threadIdx.x; k < 48 * npatch; k += blockDim.x) {
            lds[k] = ctrl_g[k];
            lds[48 * npatch + k] = vel_g[k];
        }
        ctrl = lds;
        vel = lds + 48 * npatch;
    }
    __syncthreads();
    const long long base = (long long)blockIdx.x * chunk;
    const int cnt = (int)(npts - base < chunk ? npts - base : chunk);
    Heap hp;
    for (;;) {
        const int k = atomicAdd(&s_next, 1);
        if (k >= cnt) break;
        const long long rid = base + k;
        double x0[3], w[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x0[c] = pts[6 * rid + c];
            w[c] = pts[6 * rid + 3 + c];
        }
        if (!isfinite(x0[0] + x0[1] + x0[2] + w[0] + w[1] + w[2])) {
            write_result(hit, patch_out, pops_out, rid, INFINITY, 0.0, 0.0, -3, 0);
            continue;
        }
        hp.n = 0;
        double best = INFINITY, bu = 0.0, bv = 0.0;
        int bp = -1, pops = 0, budget = tail.budget;
        bool full = false, handed = false;
        const double unit[4] = {0.0, 1.0, 0.0, 1.0};
        for (int p = 0; p < npatch && !full; ++p) {
            double t0;
            if (!earliest_time(ctrl + 48 * p, vel + 48 * p, 0.0, 1.0, 0.0, 1.0, x0, w, dt, t0)) continue;
            if (hp.n == o.heap_cap) {
                full = true;
                break;
            }
            hp.push(t0, 0.0, unit, p);
        }
        while (hp.n > 0 && !full) {
            if (pops == budget || (budget > 0 && hp.n > o.heap_cap - 4)) {
                const int s = atomicAdd(tail.count, 1);
                if (s < tail.cap) {
                    LongRay lr;
                    lr.best = best;
                    lr.bu = bu;
                    lr.bv = bv;
                    lr.bp = bp;
                    lr.pops = pops;
                    lr.n = hp.n;
                    lr.rid = rid;
                    tail.rays[s] = lr;
                    for (int e = 0; e < hp.n; ++e) {
                        const long long q = (long long)s * RAY_HEAP_MAX + e;
                        tail.key[q] = hp.key[e];
                        tail.thi[q] = 0.0;
                        tail.rect[4 * q] = hp.rect[e][0];
                        tail.rect[4 * q + 1] = hp.rect[e][1];
                        tail.rect[4 * q + 2] = hp.rect[e][2];
                        tail.rect[4 * q + 3] = hp.rect[e][3];
                        tail.tag[q] = hp.tag[e];
                    }
                    handed = true;
                    break;
                }
                budget = 0;
            }
            if (pops == RAY_MAX_POPS) {
                full = true;
                break;
            }
            double tlo, unused, rc[4];
            int tg;
            hp.pop(tlo, unused, rc, tg);
            ++pops;
            if (!(tlo < best)) break;
            const int patch = tg & 0xFFFFFF, depth = (tg >> 24) & 63;
            const double* cp = ctrl + 48 * patch;
            const double* cv = vel + 48 * patch;
            if (depth >= o.max_depth || diag_at(cp, cv, rc[0], rc[1], rc[2], rc[3], tlo) <= o.eps) {
                if (tlo < best) {
                    best = tlo;
                    bu = 0.5 * (rc[0] + rc[1]);
                    bv = 0.5 * (rc[2] + rc[3]);
                    bp = patch;
                }
                if (o.newton_iters == 0) break;
                continue;
            }
            double ht, hu, hv;
            expand_ccd(cp, cv, x0, w, dt, o, best, tlo, rc, patch, depth, ht, hu, hv,
                       [&](double k2, double th, const double* kr, int tg2) {
                           if (hp.n == o.heap_cap) {
                               full = true;
                               return false;
                           }
                           hp.push(k2, th, kr, tg2);
                           return true;
                       });
            if (ht < best) {
                best = ht;
                bu = hu;
                bv = hv;
                bp = patch;
            }
        }
        if (!handed)
            write_result(hit, patch_out, pops_out, rid, full ? INFINITY : (bp >= 0 ? best : INFINITY), bu, bv,
                         full ? -2 : bp, pops);
    }
}

void launch_ccd(hipStream_t st, const double* ctrl, const double* vel, int npatch, const double* pts,
                long long npts, double dt, const RayParams& o, double* hit, int* patch, int* pops);

// The cooperative search of one handed-over ray per block of TAIL_THREADS
// (8 waves; 4 took 1.7 times as long on the drape's grazing rays, 16 spill
// registers).  The candidates live in an LDS pool; every step sorts their
// keys (bitonic network over the pool's slots, free slots keyed +inf), takes
// the (up to) TAIL_THREADS smallest that the ray enters before the best
// answer, one per thread, and files their sub-rectangles into the slots thus
// freed.  The midpoint form ends on the step's first answer in key order;
// the accelerated form runs until no candidate is left before the best
// answer.  Block-wide values (best answer, counts) go through LDS.
constexpr int TAIL_POOL = 2048;
constexpr int TAIL_THREADS = 512;
constexpr size_t TAIL_LDS = (size_t)TAIL_POOL * (7 * sizeof(double) + sizeof(int) + sizeof(short));

template <bool MOVING>
__global__ void __launch_bounds__(TAIL_THREADS) k_ray_tail(const double* __restrict__ ctrl,
                                                           const double* __restrict__ vel,
                                                           const double* __restrict__ rays, double dt, RayParams o,
                                                           RayTail tail, double* __restrict__ hit,
                                                           int* __restrict__ patch_out, int* __restrict__ pops_out) {
    extern __shared__ double dyn[];
    double* key = dyn;
    double* thi = key + TAIL_POOL;
    double* skey = thi + TAIL_POOL;
    double(*rect)[4] = (double(*)[4])(skey + TAIL_POOL);
    int* tag = (int*)(rect + TAIL_POOL);
    short* sidx = (short*)(tag + TAIL_POOL);
    __shared__ double w_t[TAIL_THREADS / 64], s_best, s_bu, s_bv;
    __shared__ int w_i[TAIL_THREADS / 64], w_c[TAIL_THREADS / 64], s_live, s_bp;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = TAIL_THREADS / 64;
    const int count = min(*tail.count, tail.cap);
    for (int s = blockIdx.x; s < count; s += gridDim.x) {
        const LongRay lr = tail.rays[s];
        Ray r;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            r.o[c] = rays[6 * lr.rid + c];
            r.d[c] = rays[6 * lr.rid + 3 + c];
        }
        const double small = o.eps * sqrt(dot3(r.d, r.d));
        double best = lr.best, bu = lr.bu, bv = lr.bv;
        int bp = lr.bp, pops = lr.pops, hi = lr.n;
        bool over = false;
        __syncthreads();
        for (int e = tid; e < TAIL_POOL; e += TAIL_THREADS) {
            if (e < lr.n) {
                const long long q = (long long)s * RAY_HEAP_MAX + e;
                key[e] = tail.key[q];
                thi[e] = tail.thi[q];
                rect[e][0] = tail.rect[4 * q];
                rect[e][1] = tail.rect[4 * q + 1];
                rect[e][2] = tail.rect[4 * q + 2];
                rect[e][3] = tail.rect[4 * q + 3];
                tag[e] = tail.tag[q];
            } else {
                key[e] = INFINITY;
            }
        }
        __syncthreads();
        for (;;) {
            // sort (key, slot) over the used slots [0, hi)
            int n2 = 64;
            while (n2 < hi) n2 <<= 1;
            for (int e = tid; e < n2; e += TAIL_THREADS) {
                skey[e] = e < hi ? key[e] : INFINITY;
                sidx[e] = (short)e;
            }
            __syncthreads();
            for (int k = 2; k <= n2; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int e = tid; e < n2; e += TAIL_THREADS) {
                        const int f = e ^ j;
                        if (f > e) {
                            const bool up = (e & k) == 0;
                            const double a = skey[e], b = skey[f];
                            // (key, slot) order: free slots before the padding
                            const bool gt = a > b || (a == b && sidx[e] > sidx[f]);
                            if (gt == up) {
                                skey[e] = b;
                                skey[f] = a;
                                const short t = sidx[e];
                                sidx[e] = sidx[f];
                                sidx[f] = t;
                            }
                        }
                    }
                    __syncthreads();
                }
            // candidates the ray enters before the best answer (sorted: a
            // binary search)
            if (tid == 0) {
                int lo = 0, up = n2;
                while (lo < up) {
                    const int mid = (lo + up) >> 1;
                    if (skey[mid] < best) lo = mid + 1;
                    else up = mid;
                }
                s_live = lo;
            }
            __syncthreads();
            const int live = s_live;
            if (live == 0) break;
            // examined candidates free their slots and file up to 4 children
            // each: at most (TAIL_POOL - live) / 3 of them keeps the pool from
            // overflowing (the result does not depend on how many a step takes)
            int m = min(min(live, TAIL_THREADS), max(1, (TAIL_POOL - live) / 3));
            // is this thread's candidate (the tid-th smallest key) an answer box
            bool ans = false;
            if (tid < m) {
                const int e = sidx[tid];
                const int tg = tag[e];
                if constexpr (MOVING)
                    ans = ((tg >> 24) & 63) >= o.max_depth ||
                          diag_at(ctrl + 48 * (tg & 0xFFFFFF), vel + 48 * (tg & 0xFFFFFF), rect[e][0], rect[e][1],
                                  rect[e][2], rect[e][3], key[e]) <= o.eps;
                else
                    ans = (tg & (1 << 30)) != 0;
            }
            // Midpoint form: the result is the first answer in key order over
            // the whole search, so a step examines only the candidates ahead
            // of its first answer (their children may hold an answer with a
            // smaller key) and leaves that answer in the pool; only an answer
            // with the smallest key of all is taken.
            if (o.newton_iters == 0) {
                const unsigned long long bal = __ballot(ans);
                if (lane == 0) w_c[wave] = bal ? wave * 64 + (__ffsll(bal) - 1) : TAIL_THREADS;
                __syncthreads();
                int first = TAIL_THREADS;
                for (int q = 0; q < NW; ++q) first = min(first, w_c[q]);
                __syncthreads();
                m = first == 0 ? 1 : min(first, m);
            }
            if (pops + m > RAY_MAX_POPS) {
                over = true;
                break;
            }
            // this thread's candidate: an answer box, or a Newton hit
            double ct = INFINITY, cu = 0.0, cv = 0.0;
            bool is_answer = false;
            int cpatch = -1;
            double kk[4][6];
            int ktag[4];
            int nk = 0;
            if (tid < m) {
                const int e = sidx[tid];
                const double tlo = key[e], th = thi[e];
                const double rc[4] = {rect[e][0], rect[e][1], rect[e][2], rect[e][3]};
                const int tg = tag[e];
                cpatch = tg & 0xFFFFFF;
                if (ans) {
                    is_answer = true;
                    ct = MOVING ? tlo : 0.5 * (tlo + th);
                    cu = 0.5 * (rc[0] + rc[1]);
                    cv = 0.5 * (rc[2] + rc[3]);
                } else {
                    double ht, hu = 0.0, hv = 0.0;
                    auto emit = [&](double k, double th2, const double* kr, int tg2) {
                        kk[nk][0] = k;
                        kk[nk][1] = th2;
                        kk[nk][2] = kr[0];
                        kk[nk][3] = kr[1];
                        kk[nk][4] = kr[2];
                        kk[nk][5] = kr[3];
                        ktag[nk] = tg2;
                        ++nk;
                        return true;
                    };
                    if constexpr (MOVING)
                        expand_ccd(ctrl + 48 * cpatch, vel + 48 * cpatch, r.o, r.d, dt, o, best, tlo, rc, cpatch,
                                   (tg >> 24) & 63, ht, hu, hv, emit);
                    else
                        expand(ctrl + 48 * cpatch, r, o, small, best, rc, cpatch, (tg >> 24) & 63, ht, hu, hv, emit);
                    ct = ht;
                    cu = hu;
                    cv = hv;
                }
            }
            pops += m;
            // the step's result: the midpoint form takes its first answer in
            // key order, the accelerated form the smallest tau (lowest
            // thread on ties)
            double t = (o.newton_iters == 0) ? (is_answer ? (double)tid : INFINITY) : ct;
            int wl = tid;
            for (int off = 32; off > 0; off >>= 1) {
                const double t2 = __shfl_xor(t, off);
                const int w2 = __shfl_xor(wl, off);
                if (t2 < t || (t2 == t && w2 < wl)) {
                    t = t2;
                    wl = w2;
                }
            }
            if (lane == 0) {
                w_t[wave] = t;
                w_i[wave] = wl;
            }
            __syncthreads();
            double tb = w_t[0];
            int ib = w_i[0];
            for (int q = 1; q < NW; ++q)
                if (w_t[q] < tb || (w_t[q] == tb && w_i[q] < ib)) {
                    tb = w_t[q];
                    ib = w_i[q];
                }
            const bool found = o.newton_iters == 0 ? tb < INFINITY : tb < best;
            if (found && tid == ib) {
                s_best = ct;
                s_bu = cu;
                s_bv = cv;
                s_bp = cpatch;
            }
            __syncthreads();
            if (found) {
                best = s_best;
                bu = s_bu;
                bv = s_bv;
                bp = s_bp;
            }
            if (o.newton_iters == 0 && found) break;
            // free slots: the m examined, then those past the live ones
            for (int e = tid; e < n2; e += TAIL_THREADS)
                if ((e < m || e >= live) && e < hi) key[sidx[e]] = INFINITY;
            __syncthreads();
            // file the children round by round (thread order within a round)
            int filed = 0;
            const int nfree_tail = max(hi - live, 0);
            for (int k = 0; k < 4; ++k) {
                const unsigned long long bm = __ballot(nk > k);
                if (lane == 0) w_c[wave] = __popcll(bm);
                __syncthreads();
                int basew = 0, total = 0;
                for (int q = 0; q < NW; ++q) {
                    if (q < wave) basew += w_c[q];
                    total += w_c[q];
                }
                __syncthreads();
                if (total == 0) break;
                if (nk > k) {
                    const int j = filed + basew + __popcll(bm & ((1ull << lane) - 1));
                    int slot;
                    if (j < m) slot = sidx[j];
                    else if (j - m < nfree_tail) slot = sidx[live + (j - m)];
                    else slot = hi + (j - m - nfree_tail);
                    if (slot < TAIL_POOL) {
                        key[slot] = kk[k][0];
                        thi[slot] = kk[k][1];
                        rect[slot][0] = kk[k][2];
                        rect[slot][1] = kk[k][3];
                        rect[slot][2] = kk[k][4];
                        rect[slot][3] = kk[k][5];
                        tag[slot] = ktag[k];
                    }
                }
                filed += total;
            }
            const int new_hi = filed - m > nfree_tail ? hi + (filed - m - nfree_tail) : hi;
            if (new_hi > TAIL_POOL) {
                over = true;
                break;
            }
            hi = new_hi;
            __syncthreads();
        }
        __syncthreads();
        if (tid == 0)
            write_result(hit, patch_out, pops_out, lr.rid, over ? INFINITY : (bp >= 0 ? best : INFINITY), bu, bv,
                         over ? -2 : bp, pops);
    }
}

// zero the hand-over counter (a kernel, not a memset: safe in graphs)
__global__ void k_zero_int(int* p) { *p = 0; }

// bytes of the hand-over buffer per ray: its record and its heap
constexpr size_t TAIL_BYTES_PER_RAY =
    sizeof(LongRay) + RAY_HEAP_MAX * (3 * sizeof(double) + 4 * sizeof(double) + sizeof(int));

// Fixed hand-over buffer of the allocation-free ray cast: a counter line and
// RAY_TAIL_STATIC_SLOTS rays (about 15 MiB, held by every device the library
// runs on until the process ends).  Host code never passes this name to a
// kernel: it stands for a host-side shadow there; the device address comes
// from hipGetSymbolAddress (ray_scratch_address).
constexpr size_t RAY_SCRATCH_BYTES = 256 + (size_t)RAY_TAIL_STATIC_SLOTS * TAIL_BYTES_PER_RAY;
static __device__ __align__(256) unsigned char scratch[RAY_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};
}  // namespace

hipError_t ray_scratch_address(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current first
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return hipSuccess;
}

// Lay the hand-over state of `cap` rays out in `buf` (>= 256 +
// TAIL_BYTES_PER_RAY * cap bytes) and clear its counter on the stream.
static void tail_carve(hipStream_t st, void* buf, int cap, RayTail& tail) {
    char* b = (char*)buf;
    tail.cap = cap;
    tail.count = (int*)b;
    tail.rays = (LongRay*)(b + 256);
    tail.key = (double*)(tail.rays + tail.cap);
    tail.thi = tail.key + (size_t)tail.cap * RAY_HEAP_MAX;
    tail.rect = tail.thi + (size_t)tail.cap * RAY_HEAP_MAX;
    tail.tag = (int*)(tail.rect + (size_t)tail.cap * RAY_HEAP_MAX * 4);
    tail.budget = RAY_TAIL_BUDGET;
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, tail.count);
}

// The cooperative search needs more LDS than a launch gets by default.
static bool tail_lds_ok() {
    return hipFuncSetAttribute((const void*)k_ray_tail<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)TAIL_LDS) == hipSuccess &&
           hipFuncSetAttribute((const void*)k_ray_tail<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)TAIL_LDS) == hipSuccess;
}

// Hand-over buffer of one launch: the caller's fixed buffer of `fixed_slots`
// rays when `fixed` is given (nothing to free: returns NULL), else a
// stream-ordered allocation (returned, to be freed after the tail kernel).
// Without LDS or memory every ray stays on its lane.
static void* tail_setup(hipStream_t st, long long n, RayTail& tail, void* fixed, int fixed_slots) {
    tail = RayTail{};
    void* buf = nullptr;
    const bool lds_ok = tail_lds_ok();
    if (lds_ok && fixed) {
        tail_carve(st, fixed, (int)std::min<long long>(n, fixed_slots), tail);
        return nullptr;
    }
    const int cap = (int)std::min<long long>(n, RAY_TAIL_SLOTS);
    if (lds_ok && hipMallocAsync(&buf, 256 + TAIL_BYTES_PER_RAY * cap, st) == hipSuccess) {
        tail_carve(st, buf, cap, tail);
    } else {
        (void)hipGetLastError();
        buf = nullptr;
        tail.cap = 0;
        tail.budget = -1;  // never reached: every ray stays on its lane
    }
    return buf;
}

void launch_ray_cast(hipStream_t st, const double* ctrl, int npatch, const double* rays, long long nrays,
                     const RayParams& o, double* hit, int* patch, int* pops, void* fixed_tail) {
    if (nrays <= 0) return;
    const int chunk = 256 * RAY_CHUNK_PER_LANE;
    const unsigned nb = (unsigned)((nrays + chunk - 1) / chunk);
    RayTail tail;
    void* buf = tail_setup(st, nrays, tail, fixed_tail, RAY_TAIL_STATIC_SLOTS);
    if (npatch <= RAY_LDS_PATCHES) {
        const size_t lds = sizeof(double) * 54 * (size_t)npatch;
        hipLaunchKernelGGL(k_ray_cast<true>, dim3(nb), dim3(256), lds, st, ctrl, npatch, rays, nrays, chunk, o, tail,
                           hit, patch, pops);
    } else {
        hipLaunchKernelGGL(k_ray_cast<false>, dim3(nb), dim3(256), 0, st, ctrl, npatch, rays, nrays, chunk, o, tail,
                           hit, patch, pops);
    }
    if (tail.cap > 0) {
        hipLaunchKernelGGL(k_ray_tail<false>, dim3((unsigned)std::min(tail.cap, 1024)), dim3(TAIL_THREADS), TAIL_LDS,
                           st, ctrl, nullptr, rays, 0.0, o, tail, hit, patch, pops);
        if (buf) (void)hipFreeAsync(buf, st);
    }
}

void launch_ccd(hipStream_t st, const double* ctrl, const double* vel, int npatch, const double* pts,
                long long npts, double dt, const RayParams& o, double* hit, int* patch, int* pops) {
    if (npts <= 0) return;
    const int chunk = 256 * RAY_CHUNK_PER_LANE;
    RayTail tail;
    void* buf = tail_setup(st, npts, tail, nullptr, 0);
    const unsigned nb = (unsigned)((npts + chunk - 1) / chunk);
    const size_t lds = sizeof(double) * 96 * (size_t)npatch;
    if (npatch <= RAY_LDS_PATCHES &&
        hipFuncSetAttribute((const void*)k_ccd<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
            hipSuccess) {
        hipLaunchKernelGGL(k_ccd<true>, dim3(nb), dim3(256), lds, st, ctrl, vel, npatch, pts, npts, dt, chunk, o, tail,
                           hit, patch, pops);
    } else {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_ccd<false>, dim3(nb), dim3(256), 0, st, ctrl, vel, npatch, pts, npts, dt, chunk, o, tail,
                           hit, patch, pops);
    }
    if (tail.cap > 0) {
        hipLaunchKernelGGL(k_ray_tail<true>, dim3((unsigned)std::min(tail.cap, 1024)), dim3(TAIL_THREADS), TAIL_LDS,
                           st, ctrl, vel, pts, dt, o, tail, hit, patch, pops);
        if (buf) (void)hipFreeAsync(buf, st);
    }
}

}  // namespace bhem
