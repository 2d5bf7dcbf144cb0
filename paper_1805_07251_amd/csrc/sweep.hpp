// Device code of the fused D2Q9 sweep of the multicomponent van der Waals
// free-energy lattice Boltzmann method (Ridl & Wagner, arXiv:1805.07251).
//
// One kernel launch is one time step (Eq. LBequation) for every component:
//   pull-stream -> moments (Sec. III) -> chemical potential
//   (Eq. discreteChemicalPotential) -> mean-field force (Eq. forceMuLog or
//   Eq. forceMuId) -> implicit friction (Eq. forceFriction) -> forced BGK
//   collision (Eqs. BGKcollisionOperator, feq, forcing moments with
//   Eq. forceCorrectionsPsi) -> store.
//
// Work decomposition: a workgroup owns a TX x TY tile of sites.  Phase 1 pulls
// the 9C populations of each interior site into registers (they are reused by
// the collision) and the densities of a radius-2 ring from neighbouring tiles
// (re-read from L2/MALL, never stored), all into LDS.  Phase 2 evaluates the
// chemical potential on the tile plus a radius-1 ring into LDS.  Phase 3
// takes the isotropic gradients/Laplacian from LDS and collides.  HBM traffic
// per site is one read and one write of the 9C populations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vdwlb {

constexpr int Q = 9;
constexpr int MAX_C = 4;

// D2Q9 velocities, in the order fixed by the public header.
constexpr int VX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int VY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

struct Geometry {
    int nx, ny;
    int64_t plane;     // elements between (c, i) planes
    int tiles_x;       // tiles along x
    int wrap_general;  // extents too small for single-step periodic wrapping
    int band_w;        // > 0: XCD k owns the vertical band of band_w tile columns
};

// Coefficients of one lattice, precomputed on the host in double.
template <int C, typename R = double>
struct Coeffs {
    static constexpr int NTRI = C * (C + 1) / 2;           // upper triangle with the diagonal
    static constexpr int NOFF = C > 1 ? C * (C - 1) / 2 : 1;  // strictly upper triangle
    R kT;
    R omega;  // 1/tau
    R cG;     // (tau - 1/4)/tau: coefficient of G G / rho in S
    R cL;     // 1/(12 tau): coefficient of Lap(rho) in S
    R gamma;  // gamma_mu
    R a2t[NTRI];   // 2 a^{cc'} (symmetric: one triangle kept, so C = 4 fits the scalar registers)
    R kapt[NTRI];  // kappa^{cc'}
    R lamt[NOFF];  // lambda^{cc'}, c != c'
    R b[C];
    R fk;  // 1 / (1 + lambda^{01}/2): closed-form friction factor for C = 2
    int force;  // 0 log, 1 nid
    __host__ __device__ static constexpr int tri(int c, int d) {
        return c <= d ? c * C - c * (c - 1) / 2 + (d - c) : d * C - d * (d - 1) / 2 + (c - d);
    }
    __host__ __device__ static constexpr int off(int c, int d) {
        return c < d ? c * (2 * C - c - 1) / 2 + (d - c - 1) : d * (2 * C - d - 1) / 2 + (c - d - 1);
    }
    __host__ __device__ R a2(int c, int d) const { return a2t[tri(c, d)]; }
    __host__ __device__ R kap(int c, int d) const { return kapt[tri(c, d)]; }
    __host__ __device__ R lam(int c, int d) const { return c == d ? R(0) : lamt[off(c, d)]; }
};

constexpr double THETA = 1.0 / 3.0;

// The hardware hands consecutive workgroup ids to the 8 XCDs in turn.  Map
// them so that tiles that share halos run on the same XCD (and L2) at about
// the same time: either each XCD takes a contiguous range of row-major tiles
// (a horizontal band), or (band_w > 0) XCD k takes the vertical band of
// tile columns [k band_w, (k+1) band_w) and walks it row by row.
__device__ __forceinline__ void xcd_tile(int b, int n, const Geometry& g, int& tx, int& ty) {
    const int xcd = b & 7, k = b >> 3;
    if (g.band_w > 0) {
        const int r = k / g.band_w;
        tx = xcd * g.band_w + (k - r * g.band_w);
        ty = r;
        return;
    }
    const int q = n >> 3, rr = n & 7;
    const int t = xcd * q + (xcd < rr ? xcd : rr) + k;
    ty = t / g.tiles_x;
    tx = t - ty * g.tiles_x;
}

__device__ __forceinline__ int wrapc(int v, int n, int general) {
    if (general) {
        int r = v % n;
        return r < 0 ? r + n : r;
    }
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Offsets of the sources f_i(x - v_i) of site (x, y) inside one plane.
__device__ __forceinline__ void pull_offsets(const Geometry& g, int x, int y, int (&o)[Q]) {
    const int xm = wrapc(x - 1, g.nx, g.wrap_general), xp = wrapc(x + 1, g.nx, g.wrap_general);
    const int ym = wrapc(y - 1, g.ny, g.wrap_general), yp = wrapc(y + 1, g.ny, g.wrap_general);
    const int r0 = y * g.nx, rm = ym * g.nx, rp = yp * g.nx;
    o[0] = r0 + x;
    o[1] = r0 + xm;
    o[2] = rm + x;
    o[3] = r0 + xp;
    o[4] = rp + x;
    o[5] = rm + xm;
    o[6] = rm + xp;
    o[7] = rp + xp;
    o[8] = rp + xm;
}

// State layout: nine planes, one per velocity i, each `plane` sites long,
// and at each site the C components side by side:
//     f_i^c(s) = f[(i plane + s) C + c].
// The C components of one population at one site are then one vector of
// C sizeof(T) bytes (a 16-byte load for C = 2 in FP64 or C = 4 in FP32).
// Accesses use the workgroup-uniform base of plane i plus a 32-bit byte
// offset s C sizeof(T) (plans keep a plane below 2^32 bytes), so loads and
// stores take the scalar-base form with a 32-bit vector offset.
template <typename T, int C>
__device__ __forceinline__ const T* plane_base(const T* f, int i, int64_t plane) {
    return f + (int64_t)i * plane * C;
}
template <typename T, int C>
__device__ __forceinline__ T* plane_base(T* f, int i, int64_t plane) {
    return f + (int64_t)i * plane * C;
}

template <typename T>
__device__ __forceinline__ const T& at(const T* base, int idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T& at(T* base, int idx) {
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)idx * (uint32_t)sizeof(T));
}

// The C components at site s of one plane (a single vector access when C is
// 2 or 4; plans require the state to be aligned to C sizeof(T) bytes).
template <typename T, int C>
__device__ __forceinline__ void load_site(const T* base, int s, T (&v)[C]) {
    if constexpr (C == 2 || C == 4) {
        typedef T V __attribute__((ext_vector_type(C)));
        const V w = *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) +
                                                (uint32_t)s * (uint32_t)(C * sizeof(T)));
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = w[c];
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = at(base, s * C + c);
    }
}

template <typename T, int C, bool NTSTORE>
__device__ __forceinline__ void store_site(T* base, int s, const T (&v)[C]) {
    if constexpr (C == 2 || C == 4) {
        typedef T V __attribute__((ext_vector_type(C)));
        V w;
#pragma unroll
        for (int c = 0; c < C; ++c) w[c] = v[c];
        V* dst = reinterpret_cast<V*>(reinterpret_cast<char*>(base) + (uint32_t)s * (uint32_t)(C * sizeof(T)));
        if constexpr (NTSTORE) __builtin_nontemporal_store(w, dst);
        else *dst = w;
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            T& dst = at(base, s * C + c);
            if constexpr (NTSTORE) __builtin_nontemporal_store(v[c], &dst);
            else dst = v[c];
        }
    }
}

template <typename T, int C>
__device__ __forceinline__ void pull(const T* __restrict__ f, const Geometry& g, const int (&o)[Q], T (&p)[C][Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T v[C];
        load_site<T, C>(plane_base<T, C>(f, i, g.plane), o[i], v);
#pragma unroll
        for (int c = 0; c < C; ++c) p[c][i] = v[c];
    }
}

// rho = sum_i f_i, summed in velocity order.
template <typename T>
__device__ __forceinline__ T density(const T (&p)[Q]) {
    T r = p[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) r += p[i];
    return r;
}

template <typename T>
__device__ __forceinline__ void momentum(const T (&p)[Q], T& jx, T& jy) {
    jx = ((p[1] - p[3]) + (p[5] - p[6])) + (p[8] - p[7]);
    jy = ((p[2] - p[4]) + (p[5] + p[6])) - (p[7] + p[8]);
}

// Materialise v in registers at this point.  The compiler otherwise sinks
// the momentum sums past the workgroup barriers to their use in the
// collision and keeps all pulled populations live through the potential
// phase, which costs far more registers than the moments.
template <typename T>
__device__ __forceinline__ void pin(T& v) {
    asm volatile("" : "+v"(v));
}

// Isotropic 9-point stencils on an LDS array with row stride S, centred at
// (ex, ey): gradient 3 sum_i w_i v_i g(x + v_i) and Laplacian
// 6 sum_i w_i (g(x + v_i) - g(x)).
template <typename T, int S>
__device__ __forceinline__ T lap9s(const T* a, int ex, int ey) {
    const T* r0 = a + ey * S + ex;
    const T axis = (r0[1] + r0[-1]) + (r0[S] + r0[-S]);
    const T diag = (r0[S + 1] + r0[S - 1]) + (r0[-S - 1] + r0[-S + 1]);
    return (T(4) * axis + diag - T(20) * r0[0]) * T(1.0 / 6.0);
}

template <typename T, int S>
__device__ __forceinline__ void grad9s(const T* a, int ex, int ey, T& gx, T& gy) {
    const T* r0 = a + ey * S + ex;
    const T ne = r0[S + 1], nw = r0[S - 1], sw = r0[-S - 1], se = r0[-S + 1];
    gx = (T(4) * (r0[1] - r0[-1]) + ((ne - nw) + (se - sw))) * T(1.0 / 12.0);
    gy = (T(4) * (r0[S] - r0[-S]) + ((ne + nw) - (sw + se))) * T(1.0 / 12.0);
}

// Reciprocal from the hardware estimate and two Newton steps
// r <- r + r (1 - d r) (each step doubles the correct bits), about 1 ulp.
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float d) {
    const float r = __builtin_amdgcn_rcpf(d);
    return __builtin_fmaf(r, __builtin_fmaf(-d, r, 1.0f), r);
}

// Natural logarithm in FP64.  With x = 2^e m, m in [sqrt(1/2), sqrt(2)),
// ln x = e ln 2 + 2 atanh(s), s = (m - 1)/(m + 1), |s| < 0.1716, and
// atanh(s) = s (1 + z/3 + z^2/5 + ...), z = s^2, summed to z^10 (the first
// dropped term is below 2^-55 relative).  m - 1 is exact and m + 1 = d + dl
// exactly, so one correction step makes s nearly correctly rounded; ln 2 is
// split into a 32-bit head (e times it is exact) and a tail.  Worst case
// about 1.5 ulp.  x <= 0 or NaN gives NaN, so finiteness checks catch it.
__device__ __forceinline__ double dlog(double x) {
    double m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    const bool low = m < 0x1.6a09e667f3bcdp-1;  // sqrt(1/2)
    m = low ? m + m : m;
    e = low ? e - 1 : e;
    const double f = m - 1.0, d = m + 1.0, dl = m - (d - 1.0);
    const double r = recip(d);
    const double s0 = f * r;
    double t = __builtin_fma(-s0, d, f);
    t = __builtin_fma(-s0, dl, t);
    const double s = __builtin_fma(r, t, s0);
    const double z = s * s;
    double P = 1.0 / 21.0;
    P = __builtin_fma(P, z, 1.0 / 19.0);
    P = __builtin_fma(P, z, 1.0 / 17.0);
    P = __builtin_fma(P, z, 1.0 / 15.0);
    P = __builtin_fma(P, z, 1.0 / 13.0);
    P = __builtin_fma(P, z, 1.0 / 11.0);
    P = __builtin_fma(P, z, 1.0 / 9.0);
    P = __builtin_fma(P, z, 1.0 / 7.0);
    P = __builtin_fma(P, z, 1.0 / 5.0);
    P = __builtin_fma(P, z, 1.0 / 3.0);
    const double u = s + s;
    const double lm = __builtin_fma(u * z, P, u);
    const double ed = (double)e;
    const double res = __builtin_fma(ed, 0x1.62e42ff000000p-1, __builtin_fma(ed, -0x1.718432a1b0e26p-35, lm));
    return x > 0.0 ? res : __builtin_nan("");
}
__device__ __forceinline__ float dlog(float v) { return logf(v); }

// Raises the sticky unphysical-state flag.  The flag only goes from 0 to 1
// until the host clears it, so a thread that reads it already set skips the
// atomic: once a state has gone unphysical every later step would otherwise
// send one atomic per bad site to the same address.
__device__ __forceinline__ void raise_flag(int* flag) {
    if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) atomicOr(flag, 1);
}

template <typename T>
__device__ __forceinline__ bool finite_val(T v) {
    return v == v && v - v == T(0);
}

// Chemical potential (Eq. discreteChemicalPotential without the constant kT,
// with 2 sum psi rho(x + dx) = -2 a rho - kappa Lap(rho)) and the potential
// phi whose gradient drives the force: gamma mu (log) or
// gamma mu - theta ln rho (nid).  Returns false for unphysical input.
template <typename T, int C, typename R>
__device__ __forceinline__ bool potential(const T (&rho)[C], const T (&lap)[C], const Coeffs<C, R>& k, T (&phi)[C]) {
    T eta = T(0), tot = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        eta += T(k.b[c]) * rho[c];
        tot += rho[c];
    }
    const T free_vol = T(1) - eta;
    const T inv = recip(free_vol);
    bool ok = free_vol > T(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        ok = ok && rho[c] > T(0);
        T mu = T(k.kT) * (dlog(rho[c] * inv) + T(k.b[c]) * tot * inv);
#pragma unroll
        for (int d = 0; d < C; ++d) mu -= T(k.a2(c, d)) * rho[d] + T(k.kap(c, d)) * lap[d];
        phi[c] = T(k.gamma) * mu;
        if (k.force == 1) phi[c] -= T(THETA) * dlog(rho[c]);
        ok = ok && finite_val(phi[c]);
    }
    return ok;
}

// Implicit friction (Eq. forceFriction with true velocities
// uh = u + G/(2 rho), G including the friction): solve
// rho^c uh^c - 1/2 sum_c' W^{cc'} (uh^c' - uh^c) = j^c + G_mu^c / 2,
// W^{cc'} = lambda^{cc'} rho^c rho^c'/(rho^c + rho^c'), then
// G_f^c = sum_c' W^{cc'} (uh^c' - uh^c), added to g in place.  ri = 1/rho.
template <typename T, int C>
__device__ __forceinline__ void friction(const T (&rho)[C], const T (&ri)[C], const T (&j)[C], T (&g)[C],
                                         const T (&W)[C][C], T fk) {
    if constexpr (C == 2) {
        // closed form: the velocity difference shrinks by fk = 1/(1 + lambda/2)
        const T d0 = (j[1] + T(0.5) * g[1]) * ri[1] - (j[0] + T(0.5) * g[0]) * ri[0];
        const T gf = W[0][1] * fk * d0;
        g[0] += gf;
        g[1] -= gf;
    } else if constexpr (C > 2) {
        T A[C][C], r[C], uh[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            T diag = rho[c];
#pragma unroll
            for (int d = 0; d < C; ++d)
                if (d != c) {
                    diag += T(0.5) * W[c][d];
                    A[c][d] = -T(0.5) * W[c][d];
                }
            A[c][c] = diag;
            r[c] = j[c] + T(0.5) * g[c];
        }
        T ip[C];  // reciprocals of the pivots, reused by the back substitution
#pragma unroll
        for (int p = 0; p < C; ++p) {
            ip[p] = recip(A[p][p]);
#pragma unroll
            for (int q = p + 1; q < C; ++q) {
                const T f = A[q][p] * ip[p];
#pragma unroll
                for (int m = p; m < C; ++m) A[q][m] -= f * A[p][m];
                r[q] -= f * r[p];
            }
        }
#pragma unroll
        for (int p = C - 1; p >= 0; --p) {
            T acc = r[p];
#pragma unroll
            for (int m = p + 1; m < C; ++m) acc -= A[p][m] * uh[m];
            uh[p] = acc * ip[p];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            T gf = T(0);
#pragma unroll
            for (int d = 0; d < C; ++d)
                if (d != c) gf += W[c][d] * (uh[d] - uh[c]);
            g[c] += gf;
        }
    }
    (void)ri;
    (void)fk;
}

// Forced BGK collision of one component at one site: returns the 9
// post-collision populations in p (in place).
// TAU1 (tau = 1): f' = feq + F, which does not read the pulled populations,
// so kernels can drop them after the moments.  Opposite velocities share the
// even parts (in v) of feq and F and negate the odd parts, so each pair
// (1,3), (2,4), (5,7), (6,8) is evaluated once.  The rest population comes
// last, from the mass balance sum_i f'_i = rho (sum_i feq_i = rho,
// sum_i F_i = 0, and sum_i p_i = rho when tau != 1): evaluated directly, its
// w_0 rho (1 - 3/2 u^2) loses the u^2 term whenever that is below the rounding
// step, always with the same sign, and in FP32 the mass then drifts by about
// 1e-8 per step; from the balance its rounding error is that of one sum.
template <typename T, bool TAU1 = false>
__device__ __forceinline__ void collide(T (&p)[Q], T rho, T ri, T jx, T jy, T gx, T gy, T lap, T omega, T cG, T cL) {
    const T ux = jx * ri, uy = jy * ri;
    const T sxx = T(2) * gx * ux + cG * gx * gx * ri + cL * lap;
    const T syy = T(2) * gy * uy + cG * gy * gy * ri + cL * lap;
    const T sxy = gx * uy + gy * ux + cG * gx * gy * ri;
    const T uu = ux * ux + uy * uy;
    const T base = T(1) - T(1.5) * uu;
    const T ftr = -T(1.5) * (sxx + syy);
    constexpr T W1 = T(1.0 / 9.0), W2 = T(1.0 / 36.0);
    const T r1 = W1 * rho, r2 = W2 * rho;
    // new population from feq = even + odd and force = fe + fo
    auto out = [&](int i, T feq, T force) {
        if constexpr (TAU1) p[i] = feq + force;
        else p[i] = p[i] + omega * (feq - p[i]) + force;
    };
    // axis pairs: v = +-(1,0), +-(0,1)
    {
        const T ev = r1 * (base + T(4.5) * ux * ux), od = T(3) * r1 * ux;
        const T fe = W1 * (T(4.5) * sxx + ftr), fo = T(3) * W1 * gx;
        out(1, ev + od, fe + fo);
        out(3, ev - od, fe - fo);
    }
    {
        const T ev = r1 * (base + T(4.5) * uy * uy), od = T(3) * r1 * uy;
        const T fe = W1 * (T(4.5) * syy + ftr), fo = T(3) * W1 * gy;
        out(2, ev + od, fe + fo);
        out(4, ev - od, fe - fo);
    }
    // diagonal pairs: v = +-(1,1), +-(-1,1)
    const T sd = sxx + syy;
    {
        const T vu = ux + uy;
        const T ev = r2 * (base + T(4.5) * vu * vu), od = T(3) * r2 * vu;
        const T fe = W2 * (T(4.5) * (sd + T(2) * sxy) + ftr), fo = T(3) * W2 * (gx + gy);
        out(5, ev + od, fe + fo);
        out(7, ev - od, fe - fo);
    }
    {
        const T vu = uy - ux;
        const T ev = r2 * (base + T(4.5) * vu * vu), od = T(3) * r2 * vu;
        const T fe = W2 * (T(4.5) * (sd - T(2) * sxy) + ftr), fo = T(3) * W2 * (gy - gx);
        out(6, ev + od, fe + fo);
        out(8, ev - od, fe - fo);
    }
    p[0] = rho - (((p[1] + p[3]) + (p[2] + p[4])) + ((p[5] + p[7]) + (p[6] + p[8])));
}

template <int TX, int TY>
__device__ __forceinline__ void ring_coords(int r, int& ex, int& ey) {
    constexpr int EX = TX + 4, EY = TY + 4;
    if (r < 2 * EX) {
        ey = r / EX;
        ex = r - ey * EX;
    } else if (r < 4 * EX) {
        const int r2 = r - 2 * EX;
        const int q = r2 / EX;
        ey = EY - 2 + q;
        ex = r2 - q * EX;
    } else {
        const int r3 = r - 4 * EX;
        ey = 2 + (r3 >> 2);
        const int k = r3 & 3;
        ex = k < 2 ? k : EX - 4 + k;
    }
}

// Density of one site from the populations pulled into it, written to LDS
// (component c at dst[c * stride]).
template <typename T, int C>
__device__ __forceinline__ void pull_density(const T* __restrict__ f, const Geometry& g, int x, int y, T* dst,
                                             int stride) {
    int o[Q];
    pull_offsets(g, x, y, o);
    T q[C][Q];
    pull<T, C>(f, g, o, q);
#pragma unroll
    for (int c = 0; c < C; ++c) dst[c * stride] = density<T>(q[c]);
}

// Friction, collision and store of one site whose pulled populations p,
// density, momentum, mean-field force g and density Laplacian are known.
template <typename T, int C, bool NTSTORE, bool TAU1, typename R>
__device__ __forceinline__ void collide_store(T (&p)[C][Q], const T (&rho)[C], T (&jx)[C], T (&jy)[C], T (&gx)[C],
                                              T (&gy)[C], const T (&lap)[C], const Coeffs<C, R>& k,
                                              T* __restrict__ fout, int64_t plane, int s) {
    T ri[C];
#pragma unroll
    for (int c = 0; c < C; ++c) ri[c] = recip(rho[c]);
    if constexpr (C > 1) {
        // W = lambda rho rho' / (rho + rho') = lambda / (1/rho + 1/rho')
        T W[C][C];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int d = 0; d < C; ++d) W[c][d] = T(0);
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int d = c + 1; d < C; ++d) W[c][d] = W[d][c] = T(k.lam(c, d)) * recip(ri[c] + ri[d]);
        friction<T, C>(rho, ri, jx, gx, W, T(k.fk));
        friction<T, C>(rho, ri, jy, gy, W, T(k.fk));
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
        collide<T, TAU1>(p[c], rho[c], ri[c], jx[c], jy[c], gx[c], gy[c], lap[c], T(k.omega), T(k.cG), T(k.cL));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T v[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = p[c][i];
        store_site<T, C, NTSTORE>(plane_base<T, C>(fout, i, plane), s, v);
    }
}

// The plain sweep: one launch per time step, one workgroup per TX x TY tile.
// MOM: also write the moments rho^c and j^c of the pulled state to mom_out,
// as the adjoint's forward recompute keeps them.
// Phase 1 pulls the 9C populations of each interior site into registers
// (reused by the collision unless tau = 1) and the densities of the radius-2 ring around the
// tile (re-read from L2/MALL, never stored) into LDS; phase 2 evaluates the
// potential on the tile plus a radius-1 ring; phase 3 takes gradients and the
// Laplacian from LDS and collides.
// NTSTORE: non-temporal stores of the new state, so that output lines do not
// displace halo lines in L2.  OCC > 0 asks the compiler for at least OCC waves
// per SIMD (a VGPR budget of 512 / OCC).
template <typename T, int C, int TX, int TY, bool NTSTORE, int OCC, bool TAU1, bool MOM = false>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1)))
k_sweep(const T* __restrict__ fin, T* __restrict__ fout, Geometry g, Coeffs<C, T> k, int* __restrict__ flag,
        T* __restrict__ mom_out) {
    constexpr int NT = TX * TY, EX = TX + 4, EY = TY + 4, MX = TX + 2, MY = TY + 2;
    constexpr int RING = EX * EY - TX * TY;
    __shared__ T s_rho[C][EY * EX];
    __shared__ T s_phi[C][MY * MX];

    int tx_, ty_;
    xcd_tile(blockIdx.x, gridDim.x, g, tx_, ty_);
    const int x0 = tx_ * TX, y0 = ty_ * TY;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = x0 + lx, y = y0 + ly;
    const int xs = wrapc(x, g.nx, g.wrap_general), ys = wrapc(y, g.ny, g.wrap_general);

    T p[C][Q];
    int o[Q];
    pull_offsets(g, xs, ys, o);
    pull<T, C>(fin, g, o, p);
    T rho[C], jx[C], jy[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        rho[c] = density<T>(p[c]);
        momentum<T>(p[c], jx[c], jy[c]);
        if constexpr (TAU1 || C > 2) {  // fewer live registers (measured)
            pin(jx[c]);
            pin(jy[c]);
        }
        s_rho[c][(ly + 2) * EX + lx + 2] = rho[c];
    }
    if (MOM && x < g.nx && y < g.ny) {  // moments of the pulled state: rho [C][N], then j [C][2][N]
        const int64_t n = (int64_t)g.nx * g.ny, site = (int64_t)y * g.nx + x;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            mom_out[c * n + site] = rho[c];
            mom_out[(C + 2 * c) * n + site] = jx[c];
            mom_out[(C + 2 * c + 1) * n + site] = jy[c];
        }
    }
    for (int r = threadIdx.x; r < RING; r += NT) {
        int ex, ey;
        ring_coords<TX, TY>(r, ex, ey);
        pull_density<T, C>(fin, g, wrapc(x0 - 2 + ex, g.nx, g.wrap_general), wrapc(y0 - 2 + ey, g.ny, g.wrap_general),
                           &s_rho[0][ey * EX + ex], EY * EX);
    }
    __syncthreads();

    bool bad = false;
    for (int m = threadIdx.x; m < MX * MY; m += NT) {
        const int my = m / MX, mx = m - my * MX;
        T r[C], l[C], ph[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            r[c] = s_rho[c][(my + 1) * EX + mx + 1];
            l[c] = lap9s<T, EX>(s_rho[c], mx + 1, my + 1);
        }
        bad |= !potential<T, C>(r, l, k, ph);
#pragma unroll
        for (int c = 0; c < C; ++c) s_phi[c][m] = ph[c];
    }
    if (bad) raise_flag(flag);
    __syncthreads();

    if (x >= g.nx || y >= g.ny) return;
    T gx[C], gy[C], lap[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        T px, py, rx, ry;
        grad9s<T, MX>(s_phi[c], lx + 1, ly + 1, px, py);
        grad9s<T, EX>(s_rho[c], lx + 2, ly + 2, rx, ry);
        lap[c] = lap9s<T, EX>(s_rho[c], lx + 2, ly + 2);
        gx[c] = -rho[c] * px;
        gy[c] = -rho[c] * py;
        if (k.force == 0) {
            gx[c] += T(THETA) * rx;
            gy[c] += T(THETA) * ry;
        }
    }
    collide_store<T, C, NTSTORE, TAU1>(p, rho, jx, jy, gx, gy, lap, k, fout, g.plane, y * g.nx + x);
}

// The sweep with RY rows of sites per thread (RY > 1): the tile of k_sweep
// with TX x TY / RY threads, thread row lt handling tile rows lt, lt + TY/RY,
// ...  Fewer, fuller workgroups: a larger tile (a smaller density ring per
// site) keeps several workgroups per CU.  With tau = 1 the collision does not
// read the pulled populations, so a thread holds only each row's moments
// across the barriers; otherwise it pulls a row's populations again in phase 3.
template <typename T, int C, int TX, int TY, bool NTSTORE, int OCC, bool TAU1, bool MOM, int RY>
__global__ void __launch_bounds__(TX * TY / RY) __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1)))
k_sweep_rows(const T* __restrict__ fin, T* __restrict__ fout, Geometry g, Coeffs<C, T> k, int* __restrict__ flag,
        T* __restrict__ mom_out) {
    static_assert(RY > 1 && TY % RY == 0, "RY must divide TY");
    constexpr int TYT = TY / RY, NT = TX * TYT, EX = TX + 4, EY = TY + 4, MX = TX + 2, MY = TY + 2;
    constexpr int RING = EX * EY - TX * TY;
    __shared__ T s_rho[C][EY * EX];
    __shared__ T s_phi[C][MY * MX];

    int tx_, ty_;
    xcd_tile(blockIdx.x, gridDim.x, g, tx_, ty_);
    const int x0 = tx_ * TX, y0 = ty_ * TY;
    const int lx = threadIdx.x % TX, lt = threadIdx.x / TX;
    const int x = x0 + lx;
    const int xs = wrapc(x, g.nx, g.wrap_general);

    T p[C][Q];
    T rho[RY][C], jx[RY][C], jy[RY][C];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int ly = lt + r * TYT, y = y0 + ly;
        const int ys = wrapc(y, g.ny, g.wrap_general);
        int o[Q];
        pull_offsets(g, xs, ys, o);
        pull<T, C>(fin, g, o, p);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            rho[r][c] = density<T>(p[c]);
            momentum<T>(p[c], jx[r][c], jy[r][c]);
            if constexpr (TAU1 || C > 2) {  // fewer live registers (measured)
                pin(jx[r][c]);
                pin(jy[r][c]);
            }
            s_rho[c][(ly + 2) * EX + lx + 2] = rho[r][c];
        }
        if (MOM && x < g.nx && y < g.ny) {  // moments of the pulled state: rho [C][N], then j [C][2][N]
            const int64_t n = (int64_t)g.nx * g.ny, site = (int64_t)y * g.nx + x;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                mom_out[c * n + site] = rho[r][c];
                mom_out[(C + 2 * c) * n + site] = jx[r][c];
                mom_out[(C + 2 * c + 1) * n + site] = jy[r][c];
            }
        }
    }
    for (int q = threadIdx.x; q < RING; q += NT) {
        int ex, ey;
        ring_coords<TX, TY>(q, ex, ey);
        pull_density<T, C>(fin, g, wrapc(x0 - 2 + ex, g.nx, g.wrap_general), wrapc(y0 - 2 + ey, g.ny, g.wrap_general),
                           &s_rho[0][ey * EX + ex], EY * EX);
    }
    __syncthreads();

    bool bad = false;
    for (int m = threadIdx.x; m < MX * MY; m += NT) {
        const int my = m / MX, mx = m - my * MX;
        T rr[C], l[C], ph[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            rr[c] = s_rho[c][(my + 1) * EX + mx + 1];
            l[c] = lap9s<T, EX>(s_rho[c], mx + 1, my + 1);
        }
        bad |= !potential<T, C>(rr, l, k, ph);
#pragma unroll
        for (int c = 0; c < C; ++c) s_phi[c][m] = ph[c];
    }
    if (bad) raise_flag(flag);
    __syncthreads();

    if (x >= g.nx) return;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int ly = lt + r * TYT, y = y0 + ly;
        if (y >= g.ny) break;  // rows increase with r
        if constexpr (!TAU1) {
            int o[Q];
            pull_offsets(g, xs, wrapc(y, g.ny, g.wrap_general), o);
            pull<T, C>(fin, g, o, p);
        }
        T gx[C], gy[C], lap[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            T px, py, rx, ry;
            grad9s<T, MX>(s_phi[c], lx + 1, ly + 1, px, py);
            grad9s<T, EX>(s_rho[c], lx + 2, ly + 2, rx, ry);
            lap[c] = lap9s<T, EX>(s_rho[c], lx + 2, ly + 2);
            gx[c] = -rho[r][c] * px;
            gy[c] = -rho[r][c] * py;
            if (k.force == 0) {
                gx[c] += T(THETA) * rx;
                gy[c] += T(THETA) * ry;
            }
        }
        collide_store<T, C, NTSTORE, TAU1>(p, rho[r], jx[r], jy[r], gx, gy, lap, k, fout, g.plane, y * g.nx + x);
    }
}

// f_i^c = f^0_i(rho^c, u^c) (Eq. feq).
template <typename T, int C>
__global__ void k_init(T* __restrict__ f, const T* __restrict__ rho, const T* __restrict__ mom, Geometry g) {
    const int n = g.nx * g.ny;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    T p[C][Q];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const T r = rho[(int64_t)c * n + s];
#pragma unroll
        for (int i = 0; i < Q; ++i) p[c][i] = T(0);
        T jx = T(0), jy = T(0);
        if (mom) {
            jx = mom[(int64_t)(2 * c) * n + s];
            jy = mom[(int64_t)(2 * c + 1) * n + s];
        }
        // collide with omega = 1 and no force from p = 0 gives exactly f^0
        collide<T>(p[c], r, T(1) / r, jx, jy, T(0), T(0), T(0), T(1), T(0), T(0));
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T v[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = p[c][i];
        store_site<T, C, false>(plane_base<T, C>(f, i, g.plane), s, v);
    }
}

// rho^c and rho^c u^c of the streamed populations.
template <typename T, int C>
__global__ void k_moments(const T* __restrict__ f, T* __restrict__ rho, T* __restrict__ mom, Geometry g) {
    const int n = g.nx * g.ny;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int y = s / g.nx, x = s - y * g.nx;
    int o[Q];
    Geometry gg = g;
    gg.wrap_general = 1;
    pull_offsets(gg, x, y, o);
    T p[C][Q];
    pull<T, C>(f, g, o, p);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        rho[(int64_t)c * n + s] = density<T>(p[c]);
        if (mom) {
            T jx, jy;
            momentum<T>(p[c], jx, jy);
            mom[(int64_t)(2 * c) * n + s] = jx;
            mom[(int64_t)(2 * c + 1) * n + s] = jy;
        }
    }
}

// mu^c (Eq. discreteChemicalPotential without the constant kT) and the bulk
// pressure of Sec. II from a density field.
template <typename T, int C>
__global__ void k_mu_p(const T* __restrict__ rho, T* __restrict__ mu, T* __restrict__ pr, Geometry g, Coeffs<C, T> k,
                       int* __restrict__ flag) {
    const int n = g.nx * g.ny;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int y = s / g.nx, x = s - y * g.nx;
    const int xm = wrapc(x - 1, g.nx, 1), xp = wrapc(x + 1, g.nx, 1);
    const int ym = wrapc(y - 1, g.ny, 1), yp = wrapc(y + 1, g.ny, 1);
    T r[C], l[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const T* R = rho + (int64_t)c * n;
        r[c] = R[s];
        const T axis = (R[y * g.nx + xp] + R[y * g.nx + xm]) + (R[yp * g.nx + x] + R[ym * g.nx + x]);
        const T diag = (R[yp * g.nx + xp] + R[yp * g.nx + xm]) + (R[ym * g.nx + xm] + R[ym * g.nx + xp]);
        l[c] = (T(4) * axis + diag - T(20) * r[c]) * T(1.0 / 6.0);
    }
    Coeffs<C, T> kk = k;
    kk.gamma = 1.0;
    kk.force = 0;
    T m[C];
    const bool ok = potential<T, C>(r, l, kk, m);
    if (!ok) raise_flag(flag);
    if (mu)
#pragma unroll
        for (int c = 0; c < C; ++c) mu[(int64_t)c * n + s] = m[c];
    if (pr) {
        T eta = T(0), tot = T(0), att = T(0);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            eta += T(k.b[c]) * r[c];
            tot += r[c];
#pragma unroll
            for (int d = 0; d < C; ++d) att += T(0.5) * T(k.a2(c, d)) * r[c] * r[d];
        }
        pr[s] = tot * T(k.kT) / (T(1) - eta) - att;
    }
}

}  // namespace vdwlb
