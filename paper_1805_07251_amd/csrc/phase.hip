// Phase diagram of a two-component van der Waals mixture (Appendix A) for
// many overall compositions (A, B) in a volume of 1, each independent: the
// search runs a 16-lane group per composition (one lane per trial move), the
// classification and polish one thread per composition:
//   1. stability: the Hessian of the bulk free-energy density at (A, B)
//      (Sec. VI.A); a positive-definite point is one stable phase, no search;
//   2. direct search over three phases: phases 1 and 2 hold (A1, B1, V1) and
//      (A2, B2, V2), phase 3 follows from conservation; every iteration tries
//      each of the six variables moved by +step and by -step, takes the lowest
//      total free energy if it improves and otherwise halves the step, until
//      the step falls below the threshold;
//   3. classification: the three phases merged when their densities agree,
//      phases of negligible volume dropped, the rest sorted by rho_A - rho_B;
//   4. polish: Newton on the coexistence conditions (equal mu^c and p of
//      Sec. II, with the lever rule through (A, B) for two phases), so a
//      binodal point comes out at round-off rather than at the search's
//      resolution, and even where the search stopped at its iteration cap
//      before converging: the search supplies the phase count and the start.
//      A rejected three-phase polish merges the closest pair and polishes it
//      as two phases, and failing that drops the smallest phase and polishes
//      the other two.
// Bulk free-energy density f = sum_c rho^c kT ln(rho^c / (1 - eta))
// - sum_cc' a^{cc'} rho^c rho^c' (Eq. continuousFreeEnergy without gradients).
#include <climits>
#include <cmath>
#include <cstdint>

#include "../../include/vdwlb.h"
#include "internal.hpp"
#include "sweep.hpp"

namespace vdwlb {
namespace {

constexpr int PH_BLOCK = 64;             // one wave per workgroup: waves finish independently
constexpr int PH_GROUP = 16;             // lanes per point in the search (12 trial moves)
constexpr int PH_RESTARTS = 2;           // restarts of step 6(b) per point
// Iteration budgets of the search passes before the last (which has none): a
// pass ends when its slowest point has spent its budget, and the points still
// searching go on in the next pass, packed into fewer waves.
constexpr int PH_PASS_ITERS[] = {20000, 40000, 80000, 160000};
constexpr int PH_PASSES = sizeof(PH_PASS_ITERS) / sizeof(PH_PASS_ITERS[0]);
// Passes from this one on run workgroups of four waves, which the hardware
// spreads over the four SIMDs of one CU: with the few waves of the later
// passes, each long search then has a SIMD to itself.
constexpr int PH_WIDE = 256, PH_WIDE_FROM = 1;
constexpr int PH_MAX_ITER = 700000000;   // iterations of one search; (1 + PH_RESTARTS) of them fit an int32
static_assert((1 + PH_RESTARTS) * (long long)PH_MAX_ITER < INT_MAX, "the last pass's budget never runs out");
constexpr double MERGE_TOL = 1e-3;       // phases closer than this (max norm, relative to max(1, |rho|)) are one
constexpr double VOLUME_MIN = 1e-6;      // merged phases with less volume are dropped
constexpr double F_SLACK = 1e-12;        // a polish may not raise the free energy by more (relative to max(1, |F|))
constexpr int NEWTON2_MAXIT = 100, NEWTON3_MAXIT = 50, DAMP_MAX = 64;
constexpr double NEWTON2_TOL = 1e-14, NEWTON3_TOL = 1e-15;

struct Mix {
    double kT, a00, a01, a11, b0, b1;
};

struct Rho {
    double a, b;
};

__device__ __forceinline__ bool admissible(const Mix& m, Rho r) {
    return r.a > 0.0 && r.b > 0.0 && m.b0 * r.a + m.b1 * r.b < 1.0;
}

__device__ __forceinline__ double attraction(const Mix& m, Rho r) {
    return (r.a * m.a00 + r.b * m.a01) * r.a + (r.a * m.a01 + r.b * m.a11) * r.b;
}

__device__ __forceinline__ double free_density(const Mix& m, Rho r) {
    const double g = 1.0 - (m.b0 * r.a + m.b1 * r.b);
    return (r.a * m.kT * log(r.a / g) + r.b * m.kT * log(r.b / g)) - attraction(m, r);
}

// V f(A/V, B/V) of one phase, f extended to empty components
// (rho ln rho -> 0): negative amounts and particles without volume are
// infinitely expensive, an empty phase of zero volume costs nothing.
// The search evaluates it 24 times per iteration, so it takes the sweep's
// FP64 logarithm (an atanh series, about 1.5 ulp) and reciprocals refined
// by Newton steps (about 1 ulp) instead of the library logarithm and
// correctly rounded divisions: a third of the search's instructions.  The
// polish works from free_density and mu_p, which keep the library ones.
__device__ __forceinline__ double phase_energy(const Mix& m, double A, double B, double V) {
    if (!(V >= 0.0) || !(A >= 0.0) || !(B >= 0.0)) return INFINITY;
    if (V == 0.0) return (A == 0.0 && B == 0.0) ? 0.0 : INFINITY;
    const double iv = recip(V);
    const Rho r{A * iv, B * iv};
    const double g = 1.0 - (m.b0 * r.a + m.b1 * r.b);
    if (!(g > 0.0)) return INFINITY;
    const double ig = recip(g);
    const double ea = r.a > 0.0 ? r.a * m.kT * dlog(r.a * ig) : 0.0;
    const double eb = r.b > 0.0 ? r.b * m.kT * dlog(r.b * ig) : 0.0;
    return V * ((ea + eb) - attraction(m, r));
}

struct Sym2 {
    double xx, xy, yy;
};

// Hessian d^2 f / d rho^c d rho^c'
__device__ __forceinline__ Sym2 hessian(const Mix& m, Rho r) {
    const double g = 1.0 - (m.b0 * r.a + m.b1 * r.b), ig = 1.0 / g, t = (r.a + r.b) * ig * ig;
    Sym2 h;
    h.xx = m.kT * (1.0 / r.a + 2.0 * m.b0 * ig + m.b0 * m.b0 * t) - 2.0 * m.a00;
    h.xy = m.kT * ((m.b0 + m.b1) * ig + m.b0 * m.b1 * t) - 2.0 * m.a01;
    h.yy = m.kT * (1.0 / r.b + 2.0 * m.b1 * ig + m.b1 * m.b1 * t) - 2.0 * m.a11;
    return h;
}

__device__ __forceinline__ bool stable(const Mix& m, Rho r) {
    const Sym2 h = hessian(m, r);
    return h.xx > 0.0 && h.xx * h.yy - h.xy * h.xy > 0.0;
}

// full bulk chemical potentials (with the constant kT) and pressure
__device__ __forceinline__ void mu_p(const Mix& m, Rho r, double& mua, double& mub, double& p) {
    const double g = 1.0 - (m.b0 * r.a + m.b1 * r.b), tot = r.a + r.b;
    mua = m.kT * (log(r.a / g) + 1.0 + m.b0 * tot / g) - 2.0 * (m.a00 * r.a + m.a01 * r.b);
    mub = m.kT * (log(r.b / g) + 1.0 + m.b1 * tot / g) - 2.0 * (m.a01 * r.a + m.a11 * r.b);
    p = tot * m.kT / g - attraction(m, r);
}

// Unit eigenvector of the lowest eigenvalue, sign fixed by d.a >= 0 (d.b > 0
// when d.a = 0).
__device__ __forceinline__ Rho unstable_direction(Sym2 h) {
    Rho d;
    if (h.xy == 0.0) {
        d = h.xx <= h.yy ? Rho{1.0, 0.0} : Rho{0.0, 1.0};
    } else {
        const double hd = 0.5 * (h.xx - h.yy);
        const double lam = 0.5 * (h.xx + h.yy) - sqrt(hd * hd + h.xy * h.xy);
        const Rho v1{h.xy, lam - h.xx}, v2{lam - h.yy, h.xy};
        const double n1 = v1.a * v1.a + v1.b * v1.b, n2 = v2.a * v2.a + v2.b * v2.b;
        d = n1 >= n2 ? v1 : v2;
        const double in = 1.0 / sqrt(n1 >= n2 ? n1 : n2);
        d.a *= in;
        d.b *= in;
    }
    if (d.a < 0.0 || (d.a == 0.0 && d.b < 0.0)) {
        d.a = -d.a;
        d.b = -d.b;
    }
    return d;
}

// Solve A x = r in place (x returned in r) by Gaussian elimination with
// partial pivoting; every index is a compile-time constant so A stays in
// registers.  Returns false for a singular matrix.
template <int N>
__device__ __forceinline__ bool solve(double (&A)[N][N], double (&r)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
        for (int i = k + 1; i < N; ++i) {
            if (fabs(A[i][k]) > fabs(A[k][k])) {
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const double t = A[i][j];
                    A[i][j] = A[k][j];
                    A[k][j] = t;
                }
                const double t = r[i];
                r[i] = r[k];
                r[k] = t;
            }
        }
        if (!(A[k][k] != 0.0)) return false;
        const double ip = 1.0 / A[k][k];
#pragma unroll
        for (int i = k + 1; i < N; ++i) {
            const double f = A[i][k] * ip;
#pragma unroll
            for (int j = k; j < N; ++j) A[i][j] -= f * A[k][j];
            r[i] -= f * r[k];
        }
    }
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        double acc = r[k];
#pragma unroll
        for (int j = k + 1; j < N; ++j) acc -= A[k][j] * r[j];
        r[k] = acc / A[k][k];
    }
    return true;
}

struct Phase {
    double a, b, v;  // densities and volume
};

// Two phases of overall composition N: Newton on mu(x) = mu(y), p(x) = p(y)
// and phi x + (1 - phi) y = N (analytic Jacobian: d mu / d rho = H,
// d p / d rho = rho^T H by Gibbs-Duhem).
__device__ bool polish2(const Mix& m, Rho N, Phase& P0, Phase& P1) {
    double z[5] = {P0.a, P0.b, P1.a, P1.b, 0.0};
    const double da = P0.a - P1.a, db = P0.b - P1.b;
    z[4] = ((N.a - P1.a) * da + (N.b - P1.b) * db) / (da * da + db * db);
    for (int it = 0; it < NEWTON2_MAXIT; ++it) {
        const Rho x{z[0], z[1]}, y{z[2], z[3]};
        const double phi = z[4];
        double mxa, mxb, px, mya, myb, py;
        mu_p(m, x, mxa, mxb, px);
        mu_p(m, y, mya, myb, py);
        double r[5] = {mxa - mya, mxb - myb, px - py, phi * x.a + (1.0 - phi) * y.a - N.a,
                       phi * x.b + (1.0 - phi) * y.b - N.b};
        const Sym2 hx = hessian(m, x), hy = hessian(m, y);
        double J[5][5] = {
            {hx.xx, hx.xy, -hy.xx, -hy.xy, 0.0},
            {hx.xy, hx.yy, -hy.xy, -hy.yy, 0.0},
            {x.a * hx.xx + x.b * hx.xy, x.a * hx.xy + x.b * hx.yy, -(y.a * hy.xx + y.b * hy.xy),
             -(y.a * hy.xy + y.b * hy.yy), 0.0},
            {phi, 0.0, 1.0 - phi, 0.0, x.a - y.a},
            {0.0, phi, 0.0, 1.0 - phi, x.b - y.b},
        };
        if (!solve<5>(J, r)) return false;
        double lam = 1.0, t[5];
        int k = 0;
        for (; k < DAMP_MAX; ++k) {
#pragma unroll
            for (int i = 0; i < 5; ++i) t[i] = z[i] - lam * r[i];
            if (admissible(m, Rho{t[0], t[1]}) && admissible(m, Rho{t[2], t[3]})) break;
            lam *= 0.5;
        }
        if (k == DAMP_MAX) return false;
        double smax = 0.0, zmax = 1.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            z[i] = t[i];
            smax = fmax(smax, fabs(lam * r[i]));
            zmax = fmax(zmax, fabs(z[i]));
        }
        if (smax < NEWTON2_TOL * zmax) break;
    }
    P0 = Phase{z[0], z[1], z[4]};
    P1 = Phase{z[2], z[3], 1.0 - z[4]};
    return true;
}

// Three phases: Newton on equal mu^c and p in all three (no free variable at
// fixed temperature), then the volumes from the lever rule.
__device__ bool polish3(const Mix& m, Rho N, Phase (&P)[3]) {
    double z[6] = {P[0].a, P[0].b, P[1].a, P[1].b, P[2].a, P[2].b};
    for (int it = 0; it < NEWTON3_MAXIT; ++it) {
        const Rho r0{z[0], z[1]}, r1{z[2], z[3]}, r2{z[4], z[5]};
        double m0a, m0b, p0, m1a, m1b, p1, m2a, m2b, p2;
        mu_p(m, r0, m0a, m0b, p0);
        mu_p(m, r1, m1a, m1b, p1);
        mu_p(m, r2, m2a, m2b, p2);
        double r[6] = {m0a - m1a, m0b - m1b, m0a - m2a, m0b - m2b, p0 - p1, p0 - p2};
        const Sym2 h0 = hessian(m, r0), h1 = hessian(m, r1), h2 = hessian(m, r2);
        const double g0a = r0.a * h0.xx + r0.b * h0.xy, g0b = r0.a * h0.xy + r0.b * h0.yy;
        const double g1a = r1.a * h1.xx + r1.b * h1.xy, g1b = r1.a * h1.xy + r1.b * h1.yy;
        const double g2a = r2.a * h2.xx + r2.b * h2.xy, g2b = r2.a * h2.xy + r2.b * h2.yy;
        double J[6][6] = {
            {h0.xx, h0.xy, -h1.xx, -h1.xy, 0.0, 0.0}, {h0.xy, h0.yy, -h1.xy, -h1.yy, 0.0, 0.0},
            {h0.xx, h0.xy, 0.0, 0.0, -h2.xx, -h2.xy}, {h0.xy, h0.yy, 0.0, 0.0, -h2.xy, -h2.yy},
            {g0a, g0b, -g1a, -g1b, 0.0, 0.0},         {g0a, g0b, 0.0, 0.0, -g2a, -g2b},
        };
        if (!solve<6>(J, r)) return false;
        double lam = 1.0, t[6];
        int k = 0;
        for (; k < DAMP_MAX; ++k) {
#pragma unroll
            for (int i = 0; i < 6; ++i) t[i] = z[i] - lam * r[i];
            if (admissible(m, Rho{t[0], t[1]}) && admissible(m, Rho{t[2], t[3]}) && admissible(m, Rho{t[4], t[5]}))
                break;
            lam *= 0.5;
        }
        if (k == DAMP_MAX) return false;
        double smax = 0.0, zmax = 1.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            z[i] = t[i];
            smax = fmax(smax, fabs(lam * r[i]));
            zmax = fmax(zmax, fabs(z[i]));
        }
        if (smax < NEWTON3_TOL * zmax) break;
    }
    double M[3][3] = {{z[0], z[2], z[4]}, {z[1], z[3], z[5]}, {1.0, 1.0, 1.0}};
    double v[3] = {N.a, N.b, 1.0};
    if (!solve<3>(M, v)) return false;
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = Phase{z[2 * i], z[2 * i + 1], v[i]};
    return true;
}

__device__ __forceinline__ bool finite_phase(const Phase& p) {
    return isfinite(p.a) && isfinite(p.b) && isfinite(p.v);
}

__device__ __forceinline__ bool distinct(const Phase& p, const Phase& q) {
    const double scale = fmax(fmax(1.0, fmax(fabs(p.a), fabs(p.b))), fmax(fabs(q.a), fabs(q.b)));
    return fmax(fabs(p.a - q.a), fabs(p.b - q.b)) > MERGE_TOL * scale;
}

// Polish of n = 2 or 3 sorted distinct phases in place.  Accepted when the
// result is finite with volumes in (0, 1), its phases stay distinct (the
// equations also have the trivial root of equal phases), each phase is
// locally stable, and its free energy does not exceed the search's F_search
// by more than F_SLACK; otherwise false and P untouched.
__device__ bool polish(const Mix& m, Rho N, double F_search, Phase (&P)[3], int n) {
    Phase Q[3] = {P[0], P[1], P[2]};
    const bool ok = n == 2 ? polish2(m, N, Q[0], Q[1]) : polish3(m, N, Q);
    if (!ok) return false;
    double F = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!finite_phase(Q[i]) || !(Q[i].v > 0.0 && Q[i].v < 1.0)) return false;
        for (int j = i + 1; j < n; ++j)
            if (!distinct(Q[i], Q[j])) return false;
        if (!stable(m, Rho{Q[i].a, Q[i].b})) return false;
        F += Q[i].v * free_density(m, Rho{Q[i].a, Q[i].b});
    }
    if (!(F <= F_search + F_SLACK * fmax(1.0, fabs(F_search)))) return false;
    for (int i = 0; i < n; ++i) P[i] = Q[i];
    return true;
}

__device__ __forceinline__ void cmpswap(Phase& p, Phase& q) {
    if ((q.a - q.b) < (p.a - p.b)) {
        const Phase t = p;
        p = q;
        q = t;
    }
}

// Sort the first n <= 3 phases by rho_A - rho_B (the insertion sort's order,
// as a fixed compare-and-swap network so the phases stay in registers).
__device__ __forceinline__ void sort_phases(Phase (&P)[3], int n) {
    if (n >= 2) cmpswap(P[0], P[1]);
    if (n >= 3) {
        cmpswap(P[1], P[2]);
        cmpswap(P[0], P[1]);
    }
}

// Step 6 classification of the search's phases R: merged greedily in their
// order when their densities agree within MERGE_TOL (particles and volumes
// add), merged phases below VOLUME_MIN dropped, the rest sorted.  Returns
// their number; every array index is a compile-time constant.
__device__ __forceinline__ int distinct_phases(const Phase (&R)[3], Phase (&P)[3]) {
    double gA[3] = {0.0, 0.0, 0.0}, gB[3] = {0.0, 0.0, 0.0}, gV[3] = {0.0, 0.0, 0.0};
    int ng = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (!(R[q].v > 0.0)) continue;
        int hit = -1;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            if (g < ng && hit < 0) {
                const double ra = gA[g] / gV[g], rb = gB[g] / gV[g];
                const double scale = fmax(1.0, fmax(fabs(ra), fabs(rb)));
                if (fmax(fabs(R[q].a - ra), fabs(R[q].b - rb)) <= MERGE_TOL * scale) hit = g;
            }
        }
        if (hit < 0) hit = ng++;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            if (g == hit) {
                gA[g] += R[q].a * R[q].v;
                gB[g] += R[q].b * R[q].v;
                gV[g] += R[q].v;
            }
        }
    }
    int np = 0;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        if (g < ng && gV[g] >= VOLUME_MIN) {
            const Phase ph{gA[g] / gV[g], gB[g] / gV[g], gV[g]};
#pragma unroll
            for (int s = 0; s < 3; ++s)
                if (s == np) P[s] = ph;
            ++np;
        }
    }
    sort_phases(P, np);
    return np;
}

// The search's three phases (rho_A, rho_B, V) from the amounts z, phase 3
// holding the rest of N; a phase of zero volume has zero densities.
__device__ __forceinline__ void raw_phases(Rho N, const double (&z)[6], Phase (&R)[3]) {
    const double q[9] = {z[0], z[1], z[2], z[3], z[4], z[5], N.a - z[0] - z[3], N.b - z[1] - z[4], 1.0 - z[2] - z[5]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double V = q[3 * k + 2];
        R[k] = Phase{V > 0.0 ? q[3 * k + 0] / V : 0.0, V > 0.0 ? q[3 * k + 1] / V : 0.0, V};
    }
}

__device__ __forceinline__ int count_unstable(const Mix& m, const Phase (&P)[3], int n) {
    int u = 0;
    for (int i = 0; i < n; ++i) u += stable(m, Rho{P[i].a, P[i].b}) ? 0 : 1;
    return u;
}

// Status codes between the kernels: the public ones (-1 invalid, 0 failed,
// 1..3 phases) are final; the others mark work still to do.
constexpr int ST_INVALID = -1, ST_FAILED = 0, ST_SEARCHED = 4, ST_STABLE_PENDING = 6;

// One step of a lexicographic (value, lane) minimum across lanes: each lane
// takes the pair of the lane that the DPP control CTRL names (all lanes read
// a lane of their own row of 16) if that pair is smaller.
template <int CTRL>
__device__ __forceinline__ void row_min_step(double& best, int& bl) {
    const long long b = __double_as_longlong(best);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    const double ob = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
    const int ol = __builtin_amdgcn_update_dpp(0, bl, CTRL, 0xF, 0xF, false);
    if (ob < best || (ob == best && ol < bl)) {
        best = ob;
        bl = ol;
    }
}

// The direct search from the amounts z = (A1, B1, V1, A2, B2, V2), phase 3
// holding the rest of N, run by a group of PH_GROUP lanes: lane l < 12 owns
// the trial move of variable l / 2 by +step (l even) or -step (l odd), the
// order in which a serial scan would try them.  Each iteration every lane
// evaluates its trial (the moved phase and phase 3), the group takes the
// lexicographic minimum of (free energy, lane) -- the first strict minimum,
// as the serial scan finds it -- and every lane applies the winning move
// with the winner's phase energies, so z, F and the step stay identical in
// all lanes of the group.
//
// The search is resumable: (z, step, it) is its whole state, since the
// phase energies are a function of z (recomputing them gives the values the
// accepted moves produced, bit for bit).  Runs from that state until the
// step falls below threshold or it reaches max_iter (returns true: the search
// has ended), or until budget more iterations have run (returns false; the
// state then continues the search exactly).  F receives the total free
// energy of z; iterations are added to iters.
__device__ bool search_run(const Mix& m, Rho N, double (&z)[6], double& step, int& it, double threshold,
                           int max_iter, int& budget, int& iters, int lane, double& F) {
    double e1 = phase_energy(m, z[0], z[1], z[2]);
    double e2 = phase_energy(m, z[3], z[4], z[5]);
    double e3 = phase_energy(m, N.a - z[0] - z[3], N.b - z[1] - z[4], 1.0 - z[2] - z[5]);
    F = (e1 + e2) + e3;
    const int k = lane >> 1;
    const bool trial = lane < 12, minus = (lane & 1) != 0;
    for (; it < max_iter; ++it) {
        if (budget == 0) return false;
        --budget;
        ++iters;
        double Ft = INFINITY, em = INFINITY, t3 = e3;
        if (trial) {
            const double mv = minus ? -step : step;
            double t[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) t[j] = j == k ? z[j] + mv : z[j];
            // the moved phase (1 or 2) selected first, so that all trial lanes
            // run one phase-energy evaluation instead of both branches
            const bool first = k < 3;
            em = phase_energy(m, first ? t[0] : t[3], first ? t[1] : t[4], first ? t[2] : t[5]);
            t3 = phase_energy(m, N.a - t[0] - t[3], N.b - t[1] - t[4], 1.0 - t[2] - t[5]);
            Ft = first ? (em + e2) + t3 : (e1 + em) + t3;
        }
        // lexicographic minimum of (Ft, lane) over the group's 16 lanes (one
        // DPP row): swaps within pairs and quads, then the mirror images
        // within each half row and within the row; the order is total, so
        // every lane ends with the first strict minimum
        double best = Ft;
        int bl = lane;
        row_min_step<0xB1>(best, bl);   // quad_perm [1, 0, 3, 2]
        row_min_step<0x4E>(best, bl);   // quad_perm [2, 3, 0, 1]
        row_min_step<0x141>(best, bl);  // row_half_mirror
        row_min_step<0x140>(best, bl);  // row_mirror
        if (best < F) {
            // the winner is a trial lane: its moved phase and phase 3
            const double wm = __shfl(em, bl, PH_GROUP), w3 = __shfl(t3, bl, PH_GROUP);
            const int bk = bl >> 1;
            const double bs = (bl & 1) ? -step : step;
#pragma unroll
            for (int j = 0; j < 6; ++j)
                if (j == bk) z[j] += bs;
            F = best;
            if (bk < 3)
                e1 = wm;
            else
                e2 = wm;
            e3 = w3;
        } else {
            step *= 0.5;
            if (step < threshold) return true;
        }
    }
    return true;
}

// Step 6(b): if the distinct phases of the search's end state z include an
// unstable one, replace z by the start of a new search (the largest unstable
// phase split along its unstable direction into phases 1 and 2, phase 3 then
// holding the other phases packed together) and return true.  Kept out of
// line so that the search loop's register allocation does not carry it.
__device__ __noinline__ bool restart_start(const Mix& m, Rho N, double (&z)[6]) {
    Phase R[3], P[3];
    raw_phases(N, z, R);
    const int np = distinct_phases(R, P);
    int u = -1;
    Phase pu{0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (q < np && !stable(m, Rho{P[q].a, P[q].b}) && (u < 0 || P[q].v > pu.v)) {
            u = q;
            pu = P[q];
        }
    }
    if (u < 0) return false;
    const double Au = pu.a * pu.v, Bu = pu.b * pu.v, Vu = pu.v;
    const Rho du = unstable_direction(hessian(m, Rho{pu.a, pu.b}));
    const double eps = 0.05 * fmin(Au, Bu);
    z[0] = 0.5 * Au + 0.5 * eps * du.a;
    z[1] = 0.5 * Bu + 0.5 * eps * du.b;
    z[2] = 0.5 * Vu;
    z[3] = Au - z[0];
    z[4] = Bu - z[1];
    z[5] = 0.5 * Vu;
    return true;
}

// Steps 1 and 2 with the restarts of step 6(b): stability test, direct
// search, and, while the search ends with an unstable distinct phase (at most
// PH_RESTARTS times), a new search with the largest unstable phase split
// along its unstable direction into phases 1 and 2 and phase 3 holding the
// other phases packed together.  PH_GROUP lanes per point (every lane of a
// group takes the same decisions, lane 0 writes); a workgroup of one or four
// waves.
//
// One launch is one pass over a work list.  The first pass (list_in null)
// takes every point, tests its stability and starts its search; a later
// pass takes the points of list_in[0 .. *count_in) and resumes their
// searches from state.  A point runs until its searches end or budget
// iterations of this pass are spent; in the latter case lane 0 stores
// (z, step, it, restart) in state[i][0..8], the iterations so far in info[i][1],
// and appends i to list_out.  A point whose searches have ended writes the
// last search's three phases (rho_A, rho_B, V) to raw, its free energy to F
// and (status, iterations of all searches) to info[0..1].  Splitting the
// searches into passes keeps the results of one uninterrupted search bit for
// bit; it lets each pass start the remaining long searches in waves of their
// own, instead of leaving them to share SIMDs with waves of points that
// happened to sit next to them in the grid.
__global__ void __launch_bounds__(PH_WIDE) __attribute__((amdgpu_waves_per_eu(4)))
k_phase_search(Mix m, int n, const double* __restrict__ NA, const double* __restrict__ NB, double threshold,
               int max_iter, int budget, const int* __restrict__ list_in, const int* __restrict__ count_in,
               int* __restrict__ list_out, int* __restrict__ count_out, double* __restrict__ state,
               double* __restrict__ raw, double* __restrict__ Fout, int* __restrict__ info) {
    const int lane = threadIdx.x & (PH_GROUP - 1);
    const int slot = (int)(blockIdx.x * (blockDim.x / PH_GROUP) + threadIdx.x / PH_GROUP);  // below n + 16
    int i = slot;
    if (list_in) {
        if (slot >= *count_in) return;  // whole groups leave together
        i = list_in[slot];
    } else if (slot >= n) {
        return;
    }
    const Rho N{NA[i], NB[i]};
    double F = NAN, step = 0.01;
    int status = ST_INVALID, iters = 0, it = 0, restart = 0;
    double z[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool searching = false;
    if (list_in) {
        const double* q = state + (int64_t)i * 9;
#pragma unroll
        for (int j = 0; j < 6; ++j) z[j] = q[j];
        step = q[6];
        it = (int)q[7];
        restart = (int)q[8];
        iters = info[(int64_t)i * 4 + 1];
        searching = true;
    } else if (admissible(m, N)) {
        F = free_density(m, N);
        const Sym2 h = hessian(m, N);
        if (h.xx > 0.0 && h.xx * h.yy - h.xy * h.xy > 0.0) {
            status = ST_STABLE_PENDING;
        } else {
            // start: phase 3 empty; phases 1 and 2 split along the unstable
            // direction, phase 2 holding exactly what phase 1 does not; volumes
            // 1/3 each, the empty phase shrunk to (1 - eta_N)/2 above eta_N = 1/3
            // so that phases 1 and 2 stay below the excluded-volume limit
            const Rho d = unstable_direction(h);
            const double eps = 0.05 * fmin(N.a, N.b);
            const double V3 = fmin(1.0 / 3.0, 0.5 * (1.0 - (m.b0 * N.a + m.b1 * N.b)));
            const double V12 = 0.5 * (1.0 - V3);
            z[0] = 0.5 * N.a + 0.5 * eps * d.a;
            z[1] = 0.5 * N.b + 0.5 * eps * d.b;
            z[2] = V12;
            z[3] = N.a - z[0];
            z[4] = N.b - z[1];
            z[5] = V12;
            searching = true;
        }
    }
    if (searching) {
        for (;;) {
            if (!search_run(m, N, z, step, it, threshold, max_iter, budget, iters, lane, F)) {
                if (lane == 0) {
                    double* q = state + (int64_t)i * 9;
#pragma unroll
                    for (int j = 0; j < 6; ++j) q[j] = z[j];
                    q[6] = step;
                    q[7] = (double)it;
                    q[8] = (double)restart;
                    info[(int64_t)i * 4 + 1] = iters;
                    list_out[atomicAdd(count_out, 1)] = i;
                }
                return;
            }
            if (!isfinite(F) || restart == PH_RESTARTS || !restart_start(m, N, z)) break;
            ++restart;
            step = 0.01;
            it = 0;
        }
        status = isfinite(F) ? ST_SEARCHED : ST_FAILED;
    }
    if (lane != 0) return;
    double* w = raw + (int64_t)i * 9;
    if (status == ST_SEARCHED || status == ST_FAILED) {
        Phase R[3];
        raw_phases(N, z, R);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            w[3 * k + 0] = R[k].a;
            w[3 * k + 1] = R[k].b;
            w[3 * k + 2] = R[k].v;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) w[q] = 0.0;
    }
    Fout[i] = F;
    info[(int64_t)i * 4 + 0] = status;
    info[(int64_t)i * 4 + 1] = iters;
}

__global__ void k_phase_zero(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Steps 3 and 4: classification and polish of the searched points, one
// thread per point.  Writes phases and completes info (final status, -,
// n_unstable, polished).
__global__ void __launch_bounds__(PH_BLOCK) k_phase_classify(Mix m, int n, const double* __restrict__ NA,
                                                            const double* __restrict__ NB,
                                                            const double* __restrict__ raw,
                                                            const double* __restrict__ Fs,
                                                            double* __restrict__ phases, int* __restrict__ info) {
    const int i = blockIdx.x * PH_BLOCK + threadIdx.x;
    if (i >= n) return;
    const Rho N{NA[i], NB[i]};
    Phase P[3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    int status = info[(int64_t)i * 4 + 0], unstable_n = 0, polished = 0;
    if (status == ST_STABLE_PENDING) {
        status = 1;
        P[0] = Phase{N.a, N.b, 1.0};
    } else if (status == ST_SEARCHED) {
        const double* w = raw + (int64_t)i * 9;
        const Phase R[3] = {{w[0], w[1], w[2]}, {w[3], w[4], w[5]}, {w[6], w[7], w[8]}};
        const int np = distinct_phases(R, P);
        status = np;
        unstable_n = count_unstable(m, P, np);
        if (np == 2 || np == 3) {
            if (polish(m, N, Fs[i], P, np)) {
                polished = 1;
            } else if (np == 3) {
                // merge the closest pair and polish the two phases
                auto dist = [&](int u, int w2) { return fmax(fabs(P[u].a - P[w2].a), fabs(P[u].b - P[w2].b)); };
                int u = 0, v = 1;
                double dm = dist(0, 1);
                if (dist(0, 2) < dm) {
                    u = 0;
                    v = 2;
                    dm = dist(0, 2);
                }
                if (dist(1, 2) < dm) {
                    u = 1;
                    v = 2;
                }
                const int o = 3 - u - v;
                const double V = P[u].v + P[v].v;
                Phase two[3] = {Phase{(P[u].a * P[u].v + P[v].a * P[v].v) / V, (P[u].b * P[u].v + P[v].b * P[v].v) / V, V},
                                P[o], Phase{0.0, 0.0, 0.0}};
                sort_phases(two, 2);
                int u2 = count_unstable(m, two, 2);
                bool ok = polish(m, N, Fs[i], two, 2);
                if (!ok) {
                    // or the smallest phase is a seed the search left behind: drop it
                    int k = 0;
                    if (P[1].v < P[k].v) k = 1;
                    if (P[2].v < P[k].v) k = 2;
                    two[0] = P[k == 0 ? 1 : 0];
                    two[1] = P[k == 2 ? 1 : 2];
                    u2 = count_unstable(m, two, 2);
                    ok = polish(m, N, Fs[i], two, 2);
                }
                if (ok) {
                    polished = 1;
                    status = 2;
                    unstable_n = u2;
                    P[0] = two[0];
                    P[1] = two[1];
                    P[2] = Phase{0.0, 0.0, 0.0};
                } else {
                    polished = 2;
                }
            } else {
                polished = 2;
            }
        }
    }
    double* o = phases + (int64_t)i * 9;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const bool used = q < status;
        o[3 * q + 0] = used ? P[q].a : 0.0;
        o[3 * q + 1] = used ? P[q].b : 0.0;
        o[3 * q + 2] = used ? P[q].v : 0.0;
    }
    info[(int64_t)i * 4 + 0] = status;
    info[(int64_t)i * 4 + 2] = unstable_n;
    info[(int64_t)i * 4 + 3] = polished;
}

bool finite_host(double x) { return x == x && x - x == 0.0; }

}  // namespace
}  // namespace vdwlb

using namespace vdwlb;

extern "C" vdwlb_status vdwlb_phase_points(double kT, const double* a, const double* b, int32_t n, const double* NA,
                                           const double* NB, double threshold, int32_t max_iter, double* phases,
                                           double* raw, double* F, int32_t* info, void* stream) {
    if (!a || !b || n < 0 || n > INT_MAX - 256) return VDWLB_E_INVALID_ARG;  // thread indices stay in int
    if (!(kT > 0.0) || !finite_host(kT) || !(threshold > 0.0) || !finite_host(threshold) || max_iter < 1 ||
        max_iter > PH_MAX_ITER)
        return VDWLB_E_INVALID_ARG;
    for (int k = 0; k < 4; ++k)
        if (!finite_host(a[k])) return VDWLB_E_INVALID_ARG;
    if (a[1] != a[2]) return VDWLB_E_INVALID_ARG;
    for (int k = 0; k < 2; ++k)
        if (!(b[k] > 0.0) || !finite_host(b[k])) return VDWLB_E_INVALID_ARG;
    if (n == 0) return VDWLB_OK;
    if (!NA || !NB || !phases || !raw || !F || !info) return VDWLB_E_INVALID_ARG;
    const Mix m{kT, a[0], a[1], a[3], b[0], b[1]};
    const unsigned nb = (unsigned)(((int64_t)n + PH_BLOCK - 1) / PH_BLOCK);
    const hipStream_t s = (hipStream_t)stream;
    // stream-ordered workspace: one counter per pass, then two work lists of n
    // points (ping-pong between passes); the search state of a point that
    // goes on to the next pass is kept in its row of phases, which only the
    // classification writes afterwards
    int* ws = nullptr;
    hipError_t e = hipMallocAsync((void**)&ws, sizeof(int) * (64 + 2 * (size_t)n), s);
    if (e != hipSuccess) return set_device_error(e, "phase-point workspace");
    int* const count = ws;
    int* const list[2] = {ws + 64, ws + 64 + n};
    hipLaunchKernelGGL(k_phase_zero, dim3(1), dim3(64), 0, s, count, PH_PASSES + 1);
    e = hipGetLastError();
    for (int p = 0; p <= PH_PASSES && e == hipSuccess; ++p) {
        const bool last = p == PH_PASSES;
        const int block = p < PH_WIDE_FROM ? PH_BLOCK : PH_WIDE, points = block / PH_GROUP;
        const unsigned nbs = (unsigned)(((int64_t)n + points - 1) / points);
        hipLaunchKernelGGL(k_phase_search, dim3(nbs), dim3(block), 0, s, m, (int)n, NA, NB, threshold,
                           (int)max_iter, last ? INT_MAX : PH_PASS_ITERS[p],
                           p == 0 ? (const int*)nullptr : (const int*)list[(p - 1) & 1],
                           p == 0 ? (const int*)nullptr : (const int*)(count + p), last ? nullptr : list[p & 1],
                           last ? nullptr : count + p + 1, phases, raw, F, (int*)info);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_phase_classify, dim3(nb), dim3(PH_BLOCK), 0, s, m, (int)n, NA, NB, (const double*)raw,
                           (const double*)F, phases, (int*)info);
        e = hipGetLastError();
    }
    const hipError_t ef = hipFreeAsync(ws, s);
    if (e == hipSuccess) e = ef;
    return e == hipSuccess ? VDWLB_OK : set_device_error(e, "phase-point kernels");
}
