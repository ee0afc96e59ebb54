// BHEM CPU oracle -- TEST INFRASTRUCTURE ONLY (see bhem_oracle.hpp).
//
// Ray--patch intersection of Sec. 5 in plain FP64:
//   * the Bezier form of a bicubic Hermite patch (Sec. 5, first equation):
//     each cubic Hermite segment is rewritten in the Bernstein basis of
//     degree 3, one parameter direction at a time;
//   * the static ray--patch intersection of Sec. 5.1: a ray x0 + tau d is
//     tested against the axis-aligned bounding box of a Bezier surface's
//     control points (Eq. ineqray, the convex-hull property), candidate
//     surfaces wait in a min-heap keyed by the smallest tau of their box,
//     the popped surface is cut into four by De Casteljau's algorithm, and
//     the search ends when the popped surface's box is smaller than eps
//     (in units of tau), which bounds its tau interval by eps and also pins
//     the parameters of the hit.  The accelerated form runs Newton's method on
//     x(xi1, xi2) = x0 + tau d from the centre of each popped surface; a hit
//     inside it lowers the best tau and the surface is cut into the four
//     rectangles around a small abandoned neighbourhood of the hit
//     (Fig. subany), else at its midpoint (Fig. submid).
// Sub-surfaces carry their own 16 control points, obtained from their parent
// by De Casteljau splits, exactly as the section describes.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <queue>
#include <vector>

namespace {

struct P3 {
    double x[3];
};

// Cubic Hermite segment on the cell parameter theta in [0, 1] -> its four
// Bernstein coefficients.  With end values f0, f1 and end slopes m0, m1 taken
// with respect to theta, the Bezier control values are f0, f0 + m0/3,
// f1 - m1/3, f1 (the Bezier curve's end tangents are 3(b1 - b0) and
// 3(b3 - b2)).
void hermite_to_bernstein(const double f0, const double m0, const double f1, const double m1, double b[4]) {
    b[0] = f0;
    b[1] = f0 + m0 / 3.0;
    b[2] = f1 - m1 / 3.0;
    b[3] = f1;
}

// Bernstein polynomials of degree 3 and their first derivatives at t.
void bernstein(double t, double B[4], double dB[4]) {
    const double s = 1.0 - t;
    B[0] = s * s * s;
    B[1] = 3.0 * t * s * s;
    B[2] = 3.0 * t * t * s;
    B[3] = t * t * t;
    dB[0] = -3.0 * s * s;
    dB[1] = 3.0 * s * s - 6.0 * t * s;
    dB[2] = 6.0 * t * s - 3.0 * t * t;
    dB[3] = 3.0 * t * t;
}

struct Surf {
    P3 p[4][4];  // p[i][j], i along xi1 (u), j along xi2 (v)
};

// x(u, v) and its two parameter derivatives on a Bezier surface.
void surf_eval(const Surf& s, double u, double v, double x[3], double xu[3], double xv[3]) {
    double Bu[4], dBu[4], Bv[4], dBv[4];
    bernstein(u, Bu, dBu);
    bernstein(v, Bv, dBv);
    for (int c = 0; c < 3; ++c) {
        x[c] = xu[c] = xv[c] = 0.0;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                x[c] += Bu[i] * Bv[j] * s.p[i][j].x[c];
                xu[c] += dBu[i] * Bv[j] * s.p[i][j].x[c];
                xv[c] += Bu[i] * dBv[j] * s.p[i][j].x[c];
            }
    }
}

// De Casteljau's algorithm on one cubic: the control points of the parts
// on [0, t] and [t, 1].
void casteljau(const P3 in[4], double t, P3 left[4], P3 right[4]) {
    for (int c = 0; c < 3; ++c) {
        const double a = in[0].x[c], b = in[1].x[c], cc = in[2].x[c], d = in[3].x[c];
        const double ab = a + t * (b - a), bc = b + t * (cc - b), cd = cc + t * (d - cc);
        const double abc = ab + t * (bc - ab), bcd = bc + t * (cd - bc);
        const double abcd = abc + t * (bcd - abc);
        left[0].x[c] = a;
        left[1].x[c] = ab;
        left[2].x[c] = abc;
        left[3].x[c] = abcd;
        right[0].x[c] = abcd;
        right[1].x[c] = bcd;
        right[2].x[c] = cd;
        right[3].x[c] = d;
    }
}

// Part of a surface between local parameters [a, b] along u (dir 0) or v
// (dir 1), by two De Casteljau splits: at a (keep the right part), then at
// the position of b inside that part (keep the left part).
Surf restrict_dir(const Surf& s, int dir, double a, double b) {
    Surf out;
    for (int k = 0; k < 4; ++k) {
        P3 cur[4], l[4], r[4];
        for (int m = 0; m < 4; ++m) cur[m] = dir == 0 ? s.p[m][k] : s.p[k][m];
        double hi = b;
        if (a > 0.0) {
            casteljau(cur, a, l, r);
            std::memcpy(cur, r, sizeof cur);
            hi = (b - a) / (1.0 - a);
        }
        if (hi < 1.0) {
            casteljau(cur, hi, l, r);
            std::memcpy(cur, l, sizeof cur);
        }
        for (int m = 0; m < 4; ++m) (dir == 0 ? out.p[m][k] : out.p[k][m]) = cur[m];
    }
    return out;
}

// Eq. ineqray: the interval of tau >= 0 over which x0 + tau d lies in the
// axis-aligned box of the control points (slab by slab).  Returns false
// when it is empty.  diag = the length of the box's diagonal.
bool box_interval(const Surf& s, const double x0[3], const double d[3], double& tlo, double& thi, double& diag) {
    tlo = 0.0;
    diag = 0.0;
    thi = std::numeric_limits<double>::infinity();
    for (int c = 0; c < 3; ++c) {
        double lo = s.p[0][0].x[c], hi = lo;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                lo = std::min(lo, s.p[i][j].x[c]);
                hi = std::max(hi, s.p[i][j].x[c]);
            }
        diag += (hi - lo) * (hi - lo);
        if (d[c] == 0.0) {
            if (x0[c] < lo || x0[c] > hi) return false;
            continue;
        }
        const double t1 = (lo - x0[c]) / d[c], t2 = (hi - x0[c]) / d[c];
        tlo = std::max(tlo, std::min(t1, t2));
        thi = std::min(thi, std::max(t1, t2));
    }
    diag = std::sqrt(diag);
    return tlo <= thi;
}

struct Cand {
    double tlo, thi, diag;
    double u0, u1, v0, v1;  // parameter rectangle inside the patch
    int patch, depth;
    int64_t seq;            // insertion order: fixes the order of equal keys
    Surf s;
};

struct Later {
    bool operator()(const Cand& a, const Cand& b) const {
        return a.tlo != b.tlo ? a.tlo > b.tlo : a.seq > b.seq;
    }
};

// Newton's method on F(u, v, tau) = x(u, v) - x0 - tau d = 0 over the whole
// patch, from (u, v) and tau = the projection of x(u, v) - x0 on d.  The
// 3x3 system J [du dv dtau] = -F with J = [x_u | x_v | -d] is solved by
// Cramer's rule.  Converged when |F| <= tol.
bool newton(const Surf& patch, const double x0[3], const double d[3], int iters, double tol, double& u, double& v,
            double& tau) {
    double x[3], xu[3], xv[3];
    surf_eval(patch, u, v, x, xu, xv);
    const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    tau = ((x[0] - x0[0]) * d[0] + (x[1] - x0[1]) * d[1] + (x[2] - x0[2]) * d[2]) / dd;
    for (int it = 0;; ++it) {
        double F[3];
        for (int c = 0; c < 3; ++c) F[c] = x[c] - x0[c] - tau * d[c];
        if (std::sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]) <= tol) return std::isfinite(u + v + tau);
        if (it == iters) return false;
        const double J[3][3] = {{xu[0], xv[0], -d[0]}, {xu[1], xv[1], -d[1]}, {xu[2], xv[2], -d[2]}};
        auto det3 = [](const double M[3][3]) {
            return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                   M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                   M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
        };
        const double det = det3(J);
        if (det == 0.0 || !std::isfinite(det)) return false;
        double delta[3];
        for (int k = 0; k < 3; ++k) {
            double Mk[3][3];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) Mk[r][c] = c == k ? -F[r] : J[r][c];
            delta[k] = det3(Mk) / det;
        }
        u += delta[0];
        v += delta[1];
        tau += delta[2];
        if (!std::isfinite(u + v + tau)) return false;
        surf_eval(patch, u, v, x, xu, xv);
    }
}

// ---- Dynamic ray--patch intersection (Sec. 5.2) ----
// Control points move linearly over the step: p_ij + t v_ij, t in [0, dt];
// the point moves as x0 + t w.

struct Iv {
    double lo, hi;
};

// Intersection of two unions of closed intervals.
std::vector<Iv> meet(const std::vector<Iv>& a, const std::vector<Iv>& b) {
    std::vector<Iv> out;
    for (const Iv& x : a)
        for (const Iv& y : b) {
            const double lo = std::max(x.lo, y.lo), hi = std::min(x.hi, y.hi);
            if (lo <= hi) out.push_back({lo, hi});
        }
    std::sort(out.begin(), out.end(), [](const Iv& x, const Iv& y) { return x.lo < y.lo; });
    return out;
}

// Eq. ineqccd: the times t in [0, dt] at which the point lies in the
// axis-aligned box of the moving control points.  Per axis, with
// a_ij(t) = (p_ij - x0) + t (v_ij - w) along that axis, the lower bound holds
// where some a_ij(t) <= 0 (a union of half-lines: a prefix [0, L] and a
// suffix [R, dt]) and the upper bound where some a_ij(t) >= 0 (likewise);
// the answer is the intersection over both bounds and the three axes.
std::vector<Iv> feasible_times(const Surf& p, const Surf& v, const double x0[3], const double w[3], double dt) {
    std::vector<Iv> cur = {{0.0, dt}};
    for (int c = 0; c < 3 && !cur.empty(); ++c) {
        for (int side = 0; side < 2; ++side) {  // 0: some a <= 0, 1: some a >= 0
            double L = -1.0, R = 2.0 * dt + 1.0;  // prefix end, suffix start (empty by default)
            bool all = false;
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    double a = p.p[i][j].x[c] - x0[c], b = v.p[i][j].x[c] - w[c];
                    if (side == 1) {
                        a = -a;
                        b = -b;
                    }
                    // a + t b <= 0
                    if (b > 0.0) L = std::max(L, -a / b);
                    else if (b < 0.0) R = std::min(R, -a / b);
                    else if (a <= 0.0) all = true;
                }
            std::vector<Iv> s;
            if (all) {
                s.push_back({0.0, dt});
            } else {
                if (L >= 0.0) s.push_back({0.0, std::min(L, dt)});
                if (R <= dt) s.push_back({std::max(R, 0.0), dt});
            }
            cur = meet(cur, s);
            if (cur.empty()) break;
        }
    }
    return cur;
}

double box_diag_at(const Surf& p, const Surf& v, double t) {
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double lo = INFINITY, hi = -INFINITY;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                const double x = p.p[i][j].x[c] + t * v.p[i][j].x[c];
                lo = std::min(lo, x);
                hi = std::max(hi, x);
            }
        d2 += (hi - lo) * (hi - lo);
    }
    return std::sqrt(d2);
}

struct MCand {
    double tlo;
    double u0, u1, v0, v1;
    int patch, depth;
    int64_t seq;
    Surf p, v;
};
struct MLater {
    bool operator()(const MCand& a, const MCand& b) const {
        return a.tlo != b.tlo ? a.tlo > b.tlo : a.seq > b.seq;
    }
};

// Newton's method on F(u, v, t) = x(u, v, t) - x0 - t w over the whole
// patch from (u, v, t); J = [x_u(t) | x_v(t) | x_t(u, v) - w], Cramer's rule.
bool newton_ccd(const Surf& P, const Surf& V, const double x0[3], const double w[3], int iters, double tol,
                double& u, double& v, double& t) {
    for (int it = 0;; ++it) {
        double xp[3], xpu[3], xpv[3], xv[3], xvu[3], xvv[3];
        surf_eval(P, u, v, xp, xpu, xpv);
        surf_eval(V, u, v, xv, xvu, xvv);
        double F[3], J[3][3];
        for (int c = 0; c < 3; ++c) {
            F[c] = xp[c] + t * xv[c] - x0[c] - t * w[c];
            J[c][0] = xpu[c] + t * xvu[c];
            J[c][1] = xpv[c] + t * xvv[c];
            J[c][2] = xv[c] - w[c];
        }
        if (std::sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]) <= tol) return std::isfinite(u + v + t);
        if (it == iters) return false;
        auto det3 = [](const double M[3][3]) {
            return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                   M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
        };
        const double det = det3(J);
        if (det == 0.0 || !std::isfinite(det)) return false;
        double delta[3];
        for (int k = 0; k < 3; ++k) {
            double Mk[3][3];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) Mk[r][c] = c == k ? -F[r] : J[r][c];
            delta[k] = det3(Mk) / det;
        }
        u += delta[0];
        v += delta[1];
        t += delta[2];
        if (!std::isfinite(u + v + t)) return false;
    }
}

}  // namespace

extern "C" {

// Control points of one bicubic Hermite patch.  corner48: the 12 DOFs of its
// four corner nodes, corner c = p + 2q for node (i+p, j+q), DOF 3k + comp
// with k = 0 x, 1 x_xi1, 2 x_xi2, 3 x_xi1xi2.  xi-derivatives become
// theta-derivatives by the factors dxi1, dxi2, dxi1*dxi2.  Output
// ctrl48[(4i + j)*3 + comp] = p_ij, i along xi1.
void orc_bh_to_bezier(const double* corner48, double dxi1, double dxi2, double* ctrl48) {
    // Along xi1 first: for each end q of xi2 and each xi2-order s, the
    // Bernstein coefficients along xi1 of the value (s = 0) or of the
    // xi2-slope (s = 1).
    double row[2][2][4][3];  // [q][s][i][comp]
    for (int q = 0; q < 2; ++q)
        for (int s = 0; s < 2; ++s)
            for (int c = 0; c < 3; ++c) {
                const int k0 = s ? 2 : 0, k1 = s ? 3 : 1;  // kind of the value / of its xi1-slope
                const double sc = s ? dxi2 : 1.0;
                const double* n0 = corner48 + 12 * (0 + 2 * q);
                const double* n1 = corner48 + 12 * (1 + 2 * q);
                double b[4];
                hermite_to_bernstein(sc * n0[3 * k0 + c], sc * dxi1 * n0[3 * k1 + c], sc * n1[3 * k0 + c],
                                     sc * dxi1 * n1[3 * k1 + c], b);
                for (int i = 0; i < 4; ++i) row[q][s][i][c] = b[i];
            }
    // Then along xi2 for each i.
    for (int i = 0; i < 4; ++i)
        for (int c = 0; c < 3; ++c) {
            double b[4];
            hermite_to_bernstein(row[0][0][i][c], row[0][1][i][c], row[1][0][i][c], row[1][1][i][c], b);
            for (int j = 0; j < 4; ++j) ctrl48[(4 * i + j) * 3 + c] = b[j];
        }
}

// x(u, v), x_u, x_v of a Bezier surface given as ctrl48 (layout above).
void orc_bezier_eval(const double* ctrl48, double u, double v, double* x, double* xu, double* xv) {
    Surf s;
    std::memcpy(s.p, ctrl48, sizeof s.p);
    surf_eval(s, u, v, x, xu, xv);
}

// Static ray--patch intersection (Sec. 5.1) of one ray with P patches.
//   ctrl: [P][48] Bezier control points; ray: x0[3], d[3] (d != 0).
//   eps: a popped surface whose box diagonal is <= eps |d| (so that its tau
//        interval [tlo, thi] is narrower than eps), or whose depth reached
//        max_depth, ends the subdivision; its answer is the interval's
//        midpoint and the rectangle's centre.
//   newton_iters: 0 = midpoint subdivision only, the search stops at the
//        first such surface; > 0 = the accelerated form, the search runs
//        until the heap is empty or its smallest key is >= the best tau.
//   newton_tol: |F| at which Newton's method counts as converged.
//   hole: half-width of the abandoned neighbourhood of a Newton hit, as a
//        fraction of the popped rectangle's width in each direction.
// out[0..2] = tau, u, v of the hit; returns the patch index, -1 on a miss.
// stats (may be NULL): [0] surfaces popped, [1] largest heap size.
int orc_ray_cast(const double* ctrl, int P, const double* ray, double eps, int newton_iters, double newton_tol,
                 double hole, int max_depth, double* out, int64_t* stats) {
    const double* x0 = ray;
    const double* d = ray + 3;
    const double dnorm = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    std::priority_queue<Cand, std::vector<Cand>, Later> heap;
    int64_t seq = 0, pops = 0, peak = 0;
    double best = std::numeric_limits<double>::infinity(), bu = 0.0, bv = 0.0;
    int bp = -1;
    auto offer = [&](const Surf& s, double u0, double u1, double v0, double v1, int patch, int depth) {
        double tlo, thi, diag;
        if (!box_interval(s, x0, d, tlo, thi, diag) || !(tlo < best)) return;
        Cand c;
        c.tlo = tlo;
        c.thi = thi;
        c.diag = diag;
        c.u0 = u0;
        c.u1 = u1;
        c.v0 = v0;
        c.v1 = v1;
        c.patch = patch;
        c.depth = depth;
        c.seq = seq++;
        c.s = s;
        heap.push(c);
        peak = std::max<int64_t>(peak, (int64_t)heap.size());
    };
    std::vector<Surf> roots(P);
    for (int p = 0; p < P; ++p) {
        std::memcpy(roots[p].p, ctrl + 48 * p, sizeof roots[p].p);
        offer(roots[p], 0.0, 1.0, 0.0, 1.0, p, 0);
    }
    while (!heap.empty()) {
        const Cand c = heap.top();
        heap.pop();
        ++pops;
        if (!(c.tlo < best)) break;
        if (c.diag <= eps * dnorm || c.depth >= max_depth) {
            const double t = 0.5 * (c.tlo + c.thi);
            if (t < best) {
                best = t;
                bu = 0.5 * (c.u0 + c.u1);
                bv = 0.5 * (c.v0 + c.v1);
                bp = c.patch;
            }
            if (newton_iters == 0) break;
            continue;
        }
        double cu = 0.5 * (c.u0 + c.u1), cv = 0.5 * (c.v0 + c.v1);
        bool hit = false;
        if (newton_iters > 0) {
            double u = cu, v = cv, tau;
            if (newton(roots[c.patch], x0, d, newton_iters, newton_tol, u, v, tau) && u >= c.u0 && u <= c.u1 &&
                v >= c.v0 && v <= c.v1 && tau > 0.0) {
                hit = true;
                if (tau < best) {
                    best = tau;
                    bu = u;
                    bv = v;
                    bp = c.patch;
                }
                cu = u;
                cv = v;
            }
        }
        // The four rectangles: around the abandoned box [ua, ub] x [va, vb]
        // of a Newton hit (a pinwheel, Fig. subany), or the quadrants of the
        // midpoint (Fig. submid, where the box is the midpoint itself).
        double ua = cu, ub = cu, va = cv, vb = cv;
        if (hit) {
            const double hu = hole * (c.u1 - c.u0), hv = hole * (c.v1 - c.v0);
            ua = std::max(c.u0, cu - hu);
            ub = std::min(c.u1, cu + hu);
            va = std::max(c.v0, cv - hv);
            vb = std::min(c.v1, cv + hv);
        }
        const double rect[4][4] = {{c.u0, ua, va, c.v1},    // left, from va up
                                   {ua, c.u1, vb, c.v1},    // top, from ua right
                                   {c.u0, ub, c.v0, va},    // bottom, up to ub
                                   {ub, c.u1, c.v0, vb}};   // right, up to vb
        const double wu = c.u1 - c.u0, wv = c.v1 - c.v0;
        for (const auto& r : rect) {
            if (!(r[1] > r[0]) || !(r[3] > r[2])) continue;
            const Surf su = restrict_dir(c.s, 0, (r[0] - c.u0) / wu, (r[1] - c.u0) / wu);
            const Surf sv = restrict_dir(su, 1, (r[2] - c.v0) / wv, (r[3] - c.v0) / wv);
            offer(sv, r[0], r[1], r[2], r[3], c.patch, c.depth + 1);
        }
    }
    out[0] = bp >= 0 ? best : std::numeric_limits<double>::infinity();
    out[1] = bu;
    out[2] = bv;
    if (stats) {
        stats[0] = pops;
        stats[1] = peak;
    }
    return bp;
}

// Many rays, OpenMP over rays.  rays: [n][6]; out: [n][3]; patch: [n];
// stats (may be NULL): [n][2].
void orc_ray_cast_many(const double* ctrl, int P, const double* rays, int64_t n, double eps, int newton_iters,
                       double newton_tol, double hole, int max_depth, double* out, int* patch, int64_t* stats) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < n; ++r)
        patch[r] = orc_ray_cast(ctrl, P, rays + 6 * r, eps, newton_iters, newton_tol, hole, max_depth,
                                out + 3 * r, stats ? stats + 2 * r : nullptr);
}

// Dynamic ray--patch intersection (Sec. 5.2) of one moving point with P
// moving patches over [0, dt].  ctrl, vel: [P][48] control points and their
// velocities; pt: x0[3], w[3].  Same search as orc_ray_cast with keys = the
// earliest time of Eq. ineqccd; a candidate is an answer when its box at
// that time has a diagonal <= eps (a length), the answer being that time and
// the rectangle's centre.  Newton starts at the candidate's centre and key
// time.  out = t, u, v; returns the patch or -1.
int orc_ccd(const double* ctrl, const double* vel, int P, const double* pt, double dt, double eps, int newton_iters,
            double newton_tol, double hole, int max_depth, double* out, int64_t* stats) {
    const double* x0 = pt;
    const double* w = pt + 3;
    std::priority_queue<MCand, std::vector<MCand>, MLater> heap;
    int64_t seq = 0, pops = 0, peak = 0;
    double best = std::numeric_limits<double>::infinity(), bu = 0.0, bv = 0.0;
    int bp = -1;
    std::vector<Surf> rp(P), rv(P);
    auto offer = [&](const Surf& sp, const Surf& sv, double u0, double u1, double v0, double v1, int patch,
                     int depth) {
        const std::vector<Iv> T = feasible_times(sp, sv, x0, w, dt);
        if (T.empty() || !(T.front().lo < best)) return;
        MCand c;
        c.tlo = T.front().lo;
        c.u0 = u0;
        c.u1 = u1;
        c.v0 = v0;
        c.v1 = v1;
        c.patch = patch;
        c.depth = depth;
        c.seq = seq++;
        c.p = sp;
        c.v = sv;
        heap.push(c);
        peak = std::max<int64_t>(peak, (int64_t)heap.size());
    };
    for (int q = 0; q < P; ++q) {
        std::memcpy(rp[q].p, ctrl + 48 * q, sizeof rp[q].p);
        std::memcpy(rv[q].p, vel + 48 * q, sizeof rv[q].p);
        offer(rp[q], rv[q], 0.0, 1.0, 0.0, 1.0, q, 0);
    }
    while (!heap.empty()) {
        const MCand c = heap.top();
        heap.pop();
        ++pops;
        if (!(c.tlo < best)) break;
        if (box_diag_at(c.p, c.v, c.tlo) <= eps || c.depth >= max_depth) {
            if (c.tlo < best) {
                best = c.tlo;
                bu = 0.5 * (c.u0 + c.u1);
                bv = 0.5 * (c.v0 + c.v1);
                bp = c.patch;
            }
            if (newton_iters == 0) break;
            continue;
        }
        double cu = 0.5 * (c.u0 + c.u1), cv = 0.5 * (c.v0 + c.v1);
        bool hit = false;
        if (newton_iters > 0) {
            double u = cu, v = cv, t = c.tlo;
            if (newton_ccd(rp[c.patch], rv[c.patch], x0, w, newton_iters, newton_tol, u, v, t) && u >= c.u0 &&
                u <= c.u1 && v >= c.v0 && v <= c.v1 && t >= 0.0 && t <= dt) {
                hit = true;
                if (t < best) {
                    best = t;
                    bu = u;
                    bv = v;
                    bp = c.patch;
                }
                cu = u;
                cv = v;
            }
        }
        double ua = cu, ub = cu, va = cv, vb = cv;
        if (hit) {
            const double hu = hole * (c.u1 - c.u0), hv = hole * (c.v1 - c.v0);
            ua = std::max(c.u0, cu - hu);
            ub = std::min(c.u1, cu + hu);
            va = std::max(c.v0, cv - hv);
            vb = std::min(c.v1, cv + hv);
        }
        const double rect[4][4] = {{c.u0, ua, va, c.v1}, {ua, c.u1, vb, c.v1}, {c.u0, ub, c.v0, va}, {ub, c.u1, c.v0, vb}};
        const double wu = c.u1 - c.u0, wv = c.v1 - c.v0;
        for (const auto& r : rect) {
            if (!(r[1] > r[0]) || !(r[3] > r[2])) continue;
            const double a0 = (r[0] - c.u0) / wu, a1 = (r[1] - c.u0) / wu, b0 = (r[2] - c.v0) / wv, b1 = (r[3] - c.v0) / wv;
            const Surf sp = restrict_dir(restrict_dir(c.p, 0, a0, a1), 1, b0, b1);
            const Surf sv = restrict_dir(restrict_dir(c.v, 0, a0, a1), 1, b0, b1);
            offer(sp, sv, r[0], r[1], r[2], r[3], c.patch, c.depth + 1);
        }
    }
    out[0] = bp >= 0 ? best : std::numeric_limits<double>::infinity();
    out[1] = bu;
    out[2] = bv;
    if (stats) {
        stats[0] = pops;
        stats[1] = peak;
    }
    return bp;
}

void orc_ccd_many(const double* ctrl, const double* vel, int P, const double* pts, int64_t n, double dt, double eps,
                  int newton_iters, double newton_tol, double hole, int max_depth, double* out, int* patch,
                  int64_t* stats) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < n; ++r)
        patch[r] = orc_ccd(ctrl, vel, P, pts + 6 * r, dt, eps, newton_iters, newton_tol, hole, max_depth, out + 3 * r,
                           stats ? stats + 2 * r : nullptr);
}

}  // extern "C"
