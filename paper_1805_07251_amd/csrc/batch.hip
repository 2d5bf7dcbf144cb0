// Batched sweep: many independent quasi-1-D lattices (all of height NY, any
// width, own parameters) advanced by one persistent launch.
//
// Workgroups take instances from a queue ordered largest first (longest
// processing time first) and run every step of an instance before taking the
// next one: one queue pop per instance and no grid-wide synchronisation
// between steps.  (With one workgroup per CU the buffers of the instances in
// flight on an XCD exceed its L2, so each step's populations still come from
// beyond L2, as in the plain sweep.)  Each step walks the instance in
// full-height strips of TX columns whose rows wrap inside LDS (strip_step),
// with exactly the per-site arithmetic of the plain sweep.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/vdwlb.h"
#include "launch.hpp"

namespace vdwlb {

// LDS footprint of one full-height strip: the NY rows of the lattice at rows
// 1..NY, a copy of the last lattice row at row 0 and of the first at row
// NY + 1, so the periodic y neighbours sit at fixed strides; TX
// columns plus an x ring of 2 (density) / 1 (potential).
template <int TX, int NY>
struct StripLds {
    static constexpr int EX = TX + 4, MX = TX + 2, RY = NY + 2;
    static constexpr int SR = EX * RY, SP = MX * RY;
};

// Store v at padded row `row` (1..NY) of column e, and at its periodic copy.
template <typename T, int NY, int S>
__device__ __forceinline__ void put_wrapped(T* plane, int row, int e, T v) {
    plane[row * S + e] = v;
    if (row == 1) plane[(NY + 1) * S + e] = v;
    if (row == NY) plane[e] = v;
}

// One time step of the TX-column strip starting at x0 of a lattice whose
// height is exactly NY (quasi-1-D lattices): the rows wrap inside LDS, so
// only the x ring is recomputed.  Executed by TX * NY threads.  Every site
// goes through the same arithmetic as in the plain sweep (same functions and
// stencil expressions), so results are bit-identical to it.
template <typename T, int C, int TX, int NY, bool NTSTORE, bool TAU1, typename R>
__device__ __forceinline__ bool strip_step(const T* __restrict__ fin, T* __restrict__ fout, const Geometry& g,
                                           const Coeffs<C, R>& k, int x0, T* s_rho, T* s_phi) {
    using L = StripLds<TX, NY>;
    constexpr int NT = TX * NY, EX = L::EX, MX = L::MX;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = x0 + lx;
    const int xs = wrapc(x, g.nx, g.wrap_general);

    T p[C][Q];
    int o[Q];
    pull_offsets(g, xs, ly, o);
    pull<T, C>(fin, g, o, p);
    T rho[C], jx[C], jy[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        rho[c] = density<T>(p[c]);
        momentum<T>(p[c], jx[c], jy[c]);
        if constexpr (TAU1 || C > 2) {  // as in k_sweep
            pin(jx[c]);
            pin(jy[c]);
        }
        put_wrapped<T, NY, EX>(s_rho + c * L::SR, ly + 1, lx + 2, rho[c]);
    }
    for (int r = threadIdx.x; r < 4 * NY; r += NT) {
        const int row = r >> 2, kq = r & 3;
        const int ex = kq < 2 ? kq : EX - 4 + kq;
        T q[C];
        pull_density<T, C>(fin, g, wrapc(x0 - 2 + ex, g.nx, g.wrap_general), row, q, 1);
#pragma unroll
        for (int c = 0; c < C; ++c) put_wrapped<T, NY, EX>(s_rho + c * L::SR, row + 1, ex, q[c]);
    }
    __syncthreads();

    bool bad = false;
    for (int m = threadIdx.x; m < MX * NY; m += NT) {
        const int my = m / MX, mx = m - my * MX;
        T r[C], l[C], ph[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            r[c] = s_rho[c * L::SR + (my + 1) * EX + mx + 1];
            l[c] = lap9s<T, EX>(s_rho + c * L::SR, mx + 1, my + 1);
        }
        bad |= !potential<T, C>(r, l, k, ph);
#pragma unroll
        for (int c = 0; c < C; ++c) put_wrapped<T, NY, MX>(s_phi + c * L::SP, my + 1, mx, ph[c]);
    }
    __syncthreads();

    if (x < g.nx) {
        T gx[C], gy[C], lap[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            T px, py, rx, ry;
            grad9s<T, MX>(s_phi + c * L::SP, lx + 1, ly + 1, px, py);
            grad9s<T, EX>(s_rho + c * L::SR, lx + 2, ly + 1, rx, ry);
            lap[c] = lap9s<T, EX>(s_rho + c * L::SR, lx + 2, ly + 1);
            gx[c] = -rho[c] * px;
            gy[c] = -rho[c] * py;
            if (k.force == 0) {
                gx[c] += T(THETA) * rx;
                gy[c] += T(THETA) * ry;
            }
        }
        collide_store<T, C, NTSTORE, TAU1>(p, rho, jx, jy, gx, gy, lap, k, fout, g.plane, ly * g.nx + x);
    }
    return bad;
}

template <int C>
struct Instance {
    Geometry g;
    int64_t offset;      // element offset of the state in a pool
    int64_t rho_offset;  // element offset of the [C][ny][nx] block in packed density arrays
    Coeffs<C> k;
};

// Offsets of the pulled sources f_i(u - v_i) of site (u, y) in an LDS state
// buffer of NY rows of W columns (the caller keeps u - 1 and u + 1 inside the
// buffer; rows wrap).  The velocity order of pull_offsets.
template <int NY, int W>
__device__ __forceinline__ void lds_pull_offsets(int u, int y, int (&o)[Q]) {
    const int ym = y == 0 ? NY - 1 : y - 1, yp = y == NY - 1 ? 0 : y + 1;
    const int r0 = y * W, rm = ym * W, rp = yp * W;
    o[0] = r0 + u;
    o[1] = r0 + u - 1;
    o[2] = rm + u;
    o[3] = r0 + u + 1;
    o[4] = rp + u;
    o[5] = rm + u - 1;
    o[6] = rm + u + 1;
    o[7] = rp + u + 1;
    o[8] = rp + u - 1;
}

// The nine pulled C-vectors of a site from an LDS state buffer with PLANE
// sites per velocity plane.
template <typename T, int C, int PLANE>
__device__ __forceinline__ void pull_lds(const T* f, const int (&o)[Q], T (&p)[C][Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T v[C];
        load_site<T, C>(f + i * PLANE * C, o[i], v);
#pragma unroll
        for (int c = 0; c < C; ++c) p[c][i] = v[c];
    }
}

// ---------------------------------------------------------------------------
// Temporal blocking of the batched D2Q9 sweep (lattices of height NY): a
// workgroup loads a strip of TX columns and 3K columns on either side (every
// row) into LDS once, advances it K steps there, and stores the TX interior
// columns of the last step.  Each step's valid region shrinks by the 3
// columns one step reaches (the pull, radius 1, after the radius-2 density
// stencil of the potential gradient), so the halo is exactly used up.  Per K
// steps HBM sees one read of (TX + 6K)/TX of the state and one write.  Each
// thread owns one site of the W x NY block for all steps and keeps its pulled
// populations and moments in registers across the barriers; every read of a
// step's input happens before its first barrier, so the new state is written
// over the old in place (one state buffer).  Every site goes through the
// plain sweep's arithmetic (the same functions and stencil expressions), so
// results are bit-identical to it.
template <typename T, int C, int TX, int NY, int K>
struct BlockLds {
    static constexpr int W = TX + 6 * K;  // columns held
    static constexpr int RY = NY + 2;     // padded rows of the density and potential arrays
    static constexpr int PLANE = NY * W;  // sites of the block
    static constexpr int NT = (PLANE + 63) / 64 * 64;  // one thread per site, whole wavefronts
    static constexpr int STATE = Q * PLANE * C;        // elements of the state buffer
    static constexpr int FIELD = C * RY * W;           // elements of the density or the potential array
    static constexpr size_t bytes = (size_t)(STATE + 2 * FIELD) * sizeof(T);
};

// Number of steps of block b when nsteps steps run as nblocks blocks.
__device__ __forceinline__ int block_steps(int nsteps, int nblocks, int b) {
    return nsteps / nblocks + (b < nsteps % nblocks ? 1 : 0);
}

template <typename T, int C, int TX, int NY, int K, bool TAU1, typename R>
__device__ __forceinline__ void block_strip(const T* __restrict__ src, T* __restrict__ dst, const Geometry& g,
                                            const Coeffs<C, R>& k, int x0, int kk, int t0, T* s_f, T* s_rho,
                                            T* s_phi, int* s_bad) {
    using L = BlockLds<T, C, TX, NY, K>;
    constexpr int W = L::W;
    const int m = threadIdx.x;
    const bool mine = m < L::PLANE;  // this thread's site (u, y) of the block
    const int y = m / W, u = m - y * W;
    // the block as it is in HBM: this site's nine C-vectors, loads first
    {
        T v[Q][C];
        if (mine) {
            const int x = wrapc(x0 - 3 * K + u, g.nx, 1);
#pragma unroll
            for (int i = 0; i < Q; ++i) load_site<T, C>(plane_base<T, C>(src, i, g.plane), y * g.nx + x, v[i]);
#pragma unroll
            for (int i = 0; i < Q; ++i) store_site<T, C, false>(s_f + i * L::PLANE * C, m, v[i]);
        }
    }
    __syncthreads();
    for (int j = 1; j <= kk; ++j) {
        const int off = 3 * (K - kk + j);  // step j's output columns are [off, W - off)
        T p[C][Q], rho[C], jx[C], jy[C];
        // pull and densities on the output columns and a ring of 2
        const bool in_r = mine && u >= off - 2 && u < W - off + 2;
        if (in_r) {
            int o[Q];
            lds_pull_offsets<NY, W>(u, y, o);
            pull_lds<T, C, L::PLANE>(s_f, o, p);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                rho[c] = density<T>(p[c]);
                momentum<T>(p[c], jx[c], jy[c]);
                put_wrapped<T, NY, W>(s_rho + c * L::RY * W, y + 1, u, rho[c]);
            }
        }
        __syncthreads();
        // potentials on the output columns and a ring of 1
        if (mine && u >= off - 1 && u < W - off + 1) {
            T r[C], l[C], ph[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                r[c] = s_rho[c * L::RY * W + (y + 1) * W + u];
                l[c] = lap9s<T, W>(s_rho + c * L::RY * W, u, y + 1);
            }
            if (!potential<T, C>(r, l, k, ph)) atomicMin(s_bad, t0 + j);
#pragma unroll
            for (int c = 0; c < C; ++c) put_wrapped<T, NY, W>(s_phi + c * L::RY * W, y + 1, u, ph[c]);
        }
        __syncthreads();
        // forces, friction and collision on the output columns, written over
        // the old state (read in full before the first barrier); the last
        // step stores the interior columns to HBM
        if (mine && u >= off && u < W - off) {
            T gx[C], gy[C], lap[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T px, py, rx, ry;
                grad9s<T, W>(s_phi + c * L::RY * W, u, y + 1, px, py);
                grad9s<T, W>(s_rho + c * L::RY * W, u, y + 1, rx, ry);
                lap[c] = lap9s<T, W>(s_rho + c * L::RY * W, u, y + 1);
                gx[c] = -rho[c] * px;
                gy[c] = -rho[c] * py;
                if (k.force == 0) {
                    gx[c] += T(THETA) * rx;
                    gy[c] += T(THETA) * ry;
                }
            }
            if (j < kk) {
                collide_store<T, C, false, TAU1>(p, rho, jx, jy, gx, gy, lap, k, s_f, L::PLANE, m);
            } else {
                const int x = x0 + u - 3 * K;
                if (x < g.nx)
                    collide_store<T, C, false, TAU1>(p, rho, jx, jy, gx, gy, lap, k, dst, g.plane, y * g.nx + x);
            }
        }
        __syncthreads();
    }
}

// The persistent batched sweep with temporal blocking: instances from the
// largest-first queue; each instance runs its steps as nblocks blocks of at
// most K steps (the block count has the parity of nsteps, so the result lands
// in the buffer a step-by-step run would leave it in), every block strip by
// strip.  An instance that becomes unphysical stops at the end of the block
// in which it did; its status word records the first unphysical step.
template <typename T, int C, int TX, int NY, int K, int TAUS>
__global__ void __launch_bounds__((BlockLds<T, C, TX, NY, K>::NT)) k_batch_tb(
    const Instance<C>* __restrict__ inst, const int* __restrict__ order, int n, T* poolA, T* poolB, int nsteps,
    int nblocks, int* counter, int* __restrict__ status) {
    using L = BlockLds<T, C, TX, NY, K>;
    extern __shared__ __align__(16) unsigned char s_raw[];
    T* s_f = reinterpret_cast<T*>(s_raw);
    T* s_rho = s_f + L::STATE;
    T* s_phi = s_rho + L::FIELD;
    __shared__ int s_job, s_bad;
    for (;;) {
        if (threadIdx.x == 0) {
            s_job = atomicAdd(counter, 1);
            s_bad = 0x7fffffff;
        }
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(s_job);
        if (job >= n) return;  // uniform: every wave exits, the queue is drained
        const int id = __builtin_amdgcn_readfirstlane(order[job]);
        const Instance<C>& I = inst[id];
        const Geometry g = I.g;
        T* A = poolA + I.offset;
        T* B = poolB + I.offset;
        const bool tau1 = TAUS == 1 || (TAUS == 0 && I.k.omega == 1.0);
        int fail = 0, t0 = 0;
        for (int b = 0; b < nblocks; ++b) {
            const int kk = block_steps(nsteps, nblocks, b);
            const T* src = (b & 1) ? B : A;
            T* dst = (b & 1) ? A : B;
            for (int x0 = 0; x0 < g.nx; x0 += TX) {
                if constexpr (TAUS == 1)
                    block_strip<T, C, TX, NY, K, true>(src, dst, g, I.k, x0, kk, t0, s_f, s_rho, s_phi, &s_bad);
                else if constexpr (TAUS == 2)
                    block_strip<T, C, TX, NY, K, false>(src, dst, g, I.k, x0, kk, t0, s_f, s_rho, s_phi, &s_bad);
                else if (tau1)
                    block_strip<T, C, TX, NY, K, true>(src, dst, g, I.k, x0, kk, t0, s_f, s_rho, s_phi, &s_bad);
                else
                    block_strip<T, C, TX, NY, K, false>(src, dst, g, I.k, x0, kk, t0, s_f, s_rho, s_phi, &s_bad);
            }
            t0 += kk;
            if (s_bad != 0x7fffffff) {  // read after block_strip's closing barrier: uniform
                fail = s_bad;
                break;
            }
        }
        if (threadIdx.x == 0) status[id] = fail;
        __syncthreads();
    }
}

// Friction and D1Q3 collision of one site, the new populations written to
// the LDS state [i][c][x] (same arithmetic as collide_store1).
template <typename T, int C, bool TAU1, typename R>
__device__ __forceinline__ void collide_lds1(T (&p)[C][Q1], const T (&rho)[C], T (&jx)[C], T (&gx)[C],
                                             const T (&lap)[C], const Coeffs<C, R>& k, T* sf, int lmax, int x) {
    T ri[C];
#pragma unroll
    for (int c = 0; c < C; ++c) ri[c] = recip(rho[c]);
    if constexpr (C > 1) {
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
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        T q[Q1] = {p[c][0], p[c][1], p[c][2]};
        collide1<T, TAU1>(q, rho[c], ri[c], jx[c], gx[c], lap[c], T(k.omega), T(k.cG), T(k.cL));
#pragma unroll
        for (int i = 0; i < Q1; ++i) sf[(i * C + c) * lmax + x] = q[i];
    }
}

__global__ void k_reset_counter(int* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// TAUS: 1 when every instance has tau = 1, 2 when none has, 0 for a mix
// (per-instance branch; the register budget is then that of the general
// collision).
template <typename T, int C, int TX, int NY, int TAUS>
__global__ void __launch_bounds__(TX * NY) k_batch(const Instance<C>* __restrict__ inst, const int* __restrict__ order,
                                                    int n, T* poolA, T* poolB, int nsteps, int* counter,
                                                    int* __restrict__ status) {
    using L = StripLds<TX, NY>;
    __shared__ T s_rho[C * L::SR];
    __shared__ T s_phi[C * L::SP];
    __shared__ int s_job, s_bad;
    for (;;) {
        if (threadIdx.x == 0) {
            s_job = atomicAdd(counter, 1);
            s_bad = 0;
        }
        __syncthreads();
        // the job index is the same for the whole workgroup: keep it (and so
        // the instance's coefficients) in scalar registers
        const int job = __builtin_amdgcn_readfirstlane(s_job);
        if (job >= n) return;  // uniform: every wave exits, the queue is drained
        const int id = __builtin_amdgcn_readfirstlane(order[job]);
        const Instance<C>& I = inst[id];
        Geometry g = I.g;
        g.wrap_general = g.nx < TX + 8 ? 1 : 0;
        T* A = poolA + I.offset;
        T* B = poolB + I.offset;
        const bool tau1 = TAUS == 1 || (TAUS == 0 && I.k.omega == 1.0);
        int fail = 0;
        for (int t = 0; t < nsteps; ++t) {
            const T* src = (t & 1) ? B : A;
            T* dst = (t & 1) ? A : B;
            bool bad = false;
            for (int x0 = 0; x0 < g.nx; x0 += TX) {
                // same collision form as the plain sweep of this instance (tau = 1 or not)
                if constexpr (TAUS == 1)
                    bad |= strip_step<T, C, TX, NY, false, true>(src, dst, g, I.k, x0, s_rho, s_phi);
                else if constexpr (TAUS == 2)
                    bad |= strip_step<T, C, TX, NY, false, false>(src, dst, g, I.k, x0, s_rho, s_phi);
                else if (tau1)
                    bad |= strip_step<T, C, TX, NY, false, true>(src, dst, g, I.k, x0, s_rho, s_phi);
                else
                    bad |= strip_step<T, C, TX, NY, false, false>(src, dst, g, I.k, x0, s_rho, s_phi);
                __syncthreads();  // LDS reuse by the next strip; orders this step's stores before the next step
            }
            if (bad) s_bad = 1;
            __syncthreads();
            if (s_bad) {
                fail = t + 1;
                break;
            }
        }
        if (threadIdx.x == 0) status[id] = fail;
        __syncthreads();
    }
}

// Batched D1Q3 sweep with every instance resident on chip: a workgroup loads
// an instance's state into LDS, runs all its steps there (the lattice wraps
// inside LDS, so no halo is ever re-read) and writes the final state back.
// LDS holds f [3][C][lmax], rho [C][lmax] and phi [C][lmax]; each of the 256
// threads owns the sites tid + k 256, k < SPT, and keeps their pulled
// populations and moments in registers between the phases.  The per-site
// arithmetic is that of the plain D1Q3 sweep (same functions), so results
// are bit-identical to it.  The final state goes to poolA for an even step
// count and to poolB for an odd one, as with ping-pong buffers.
constexpr int B1_THREADS = 256;

template <typename T, int C, int SPT, int TAUS>
__global__ void __launch_bounds__(B1_THREADS) k_batch1(const Instance<C>* __restrict__ inst,
                                                        const int* __restrict__ order, int n, T* poolA, T* poolB,
                                                        int nsteps, int lmax, int* counter, int* __restrict__ status) {
    constexpr int NT = B1_THREADS;
    extern __shared__ __align__(16) unsigned char b1_smem[];
    T* sf = reinterpret_cast<T*>(b1_smem);  // [i][c][x]
    T* sr = sf + Q1 * C * lmax;             // [c][x]
    T* sp = sr + C * lmax;                  // [c][x]
    __shared__ int s_job, s_bad;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            s_job = atomicAdd(counter, 1);
            s_bad = 0;
        }
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(s_job);
        if (job >= n) return;  // uniform: the queue is drained
        const int id = __builtin_amdgcn_readfirstlane(order[job]);
        const Instance<C>& I = inst[id];
        const int L = I.g.nx;
        const int64_t plane = I.g.plane;
        const bool tau1 = TAUS == 1 || (TAUS == 0 && I.k.omega == 1.0);
        for (int x = tid; x < L; x += NT)
#pragma unroll
            for (int i = 0; i < Q1; ++i) {
                T v[C];
                load_site<T, C>(plane_base<T, C>(poolA + I.offset, i, plane), x, v);
#pragma unroll
                for (int c = 0; c < C; ++c) sf[(i * C + c) * lmax + x] = v[c];
            }
        __syncthreads();
        int fail = 0;
        for (int t = 0; t < nsteps; ++t) {
            T p[SPT][C][Q1], rho[SPT][C], jx[SPT][C];
            // phase 1: pull from LDS, moments
#pragma unroll
            for (int k = 0; k < SPT; ++k) {
                const int x = tid + k * NT;
                if (x < L) {
                    const int xm = x == 0 ? L - 1 : x - 1, xp = x + 1 == L ? 0 : x + 1;
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        p[k][c][0] = sf[(0 * C + c) * lmax + x];
                        p[k][c][1] = sf[(1 * C + c) * lmax + xm];
                        p[k][c][2] = sf[(2 * C + c) * lmax + xp];
                        rho[k][c] = density1<T>(p[k][c]);
                        jx[k][c] = p[k][c][1] - p[k][c][2];
                        sr[c * lmax + x] = rho[k][c];
                    }
                }
            }
            __syncthreads();
            // phase 2: potential at the own sites
            bool bad = false;
#pragma unroll
            for (int k = 0; k < SPT; ++k) {
                const int x = tid + k * NT;
                if (x < L) {
                    const int xm = x == 0 ? L - 1 : x - 1, xp = x + 1 == L ? 0 : x + 1;
                    T r[C], l[C], ph[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        r[c] = sr[c * lmax + x];
                        l[c] = lap3<T>(sr[c * lmax + xm], r[c], sr[c * lmax + xp]);
                    }
                    bad |= !potential<T, C>(r, l, I.k, ph);
#pragma unroll
                    for (int c = 0; c < C; ++c) sp[c * lmax + x] = ph[c];
                }
            }
            __syncthreads();
            // phase 3: force, friction, collision into LDS (all pulls of this
            // step were taken before the first barrier)
#pragma unroll
            for (int k = 0; k < SPT; ++k) {
                const int x = tid + k * NT;
                if (x < L) {
                    const int xm = x == 0 ? L - 1 : x - 1, xp = x + 1 == L ? 0 : x + 1;
                    T gx[C], lap[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const T rm = sr[c * lmax + xm], r0 = sr[c * lmax + x], rp = sr[c * lmax + xp];
                        lap[c] = lap3<T>(rm, r0, rp);
                        gx[c] = -rho[k][c] * grad3<T>(sp[c * lmax + xm], sp[c * lmax + xp]);
                        if (I.k.force == 0) gx[c] += T(THETA) * grad3<T>(rm, rp);
                    }
                    if (tau1)
                        collide_lds1<T, C, true>(p[k], rho[k], jx[k], gx, lap, I.k, sf, lmax, x);
                    else
                        collide_lds1<T, C, false>(p[k], rho[k], jx[k], gx, lap, I.k, sf, lmax, x);
                }
            }
            if (bad) s_bad = 1;
            __syncthreads();
            if (s_bad) {
                fail = t + 1;
                break;
            }
        }
        T* out = ((nsteps & 1) ? poolB : poolA) + I.offset;
        for (int x = tid; x < L; x += NT)
#pragma unroll
            for (int i = 0; i < Q1; ++i) {
                T v[C];
#pragma unroll
                for (int c = 0; c < C; ++c) v[c] = sf[(i * C + c) * lmax + x];
                store_site<T, C, false>(plane_base<T, C>(out, i, plane), x, v);
            }
        if (tid == 0) status[id] = fail;
        __syncthreads();
    }
}

// f = f^0(rho, u = 0) for every instance; one workgroup per instance.
template <typename T, int C>
__global__ void k_batch_init(const Instance<C>* __restrict__ inst, T* __restrict__ pool, const T* __restrict__ rho) {
    const Instance<C>& I = inst[blockIdx.x];
    const int n = I.g.nx * I.g.ny;
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        T p[C][Q];
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
            for (int i = 0; i < Q; ++i) p[c][i] = T(0);
            const T r = rho[I.rho_offset + (int64_t)c * n + s];
            collide<T>(p[c], r, T(1) / r, T(0), T(0), T(0), T(0), T(0), T(1), T(0), T(0));
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            T v[C];
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = p[c][i];
            store_site<T, C, false>(plane_base<T, C>(pool + I.offset, i, I.g.plane), s, v);
        }
    }
}

// Densities of the streamed populations of every instance.
template <typename T, int C>
__global__ void k_batch_rho(const Instance<C>* __restrict__ inst, const T* __restrict__ pool, T* __restrict__ rho) {
    const Instance<C>& I = inst[blockIdx.x];
    Geometry g = I.g;
    g.wrap_general = 1;
    const int n = g.nx * g.ny;
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        const int y = s / g.nx, x = s - y * g.nx;
        pull_density<T, C>(pool + I.offset, g, x, y, rho + I.rho_offset + s, n);
    }
}

// D1Q3 versions of the two helpers above.
template <typename T, int C>
__global__ void k_batch_init1(const Instance<C>* __restrict__ inst, T* __restrict__ pool, const T* __restrict__ rho) {
    const Instance<C>& I = inst[blockIdx.x];
    const int n = I.g.nx;
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
        T p[C][Q1];
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
            for (int i = 0; i < Q1; ++i) p[c][i] = T(0);
            const T r = rho[I.rho_offset + (int64_t)c * n + x];
            collide1<T, false>(p[c], r, T(1) / r, T(0), T(0), T(0), T(1), T(0), T(0));
        }
#pragma unroll
        for (int i = 0; i < Q1; ++i) {
            T v[C];
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = p[c][i];
            store_site<T, C, false>(plane_base<T, C>(pool + I.offset, i, I.g.plane), x, v);
        }
    }
}

template <typename T, int C>
__global__ void k_batch_rho1(const Instance<C>* __restrict__ inst, const T* __restrict__ pool, T* __restrict__ rho) {
    const Instance<C>& I = inst[blockIdx.x];
    const int n = I.g.nx;
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
        T p[C][Q1];
        pull1<T, C>(pool + I.offset, I.g.plane, x, wrapc(x - 1, n, 1), wrapc(x + 1, n, 1), p);
#pragma unroll
        for (int c = 0; c < C; ++c) rho[I.rho_offset + (int64_t)c * n + x] = density1<T>(p[c]);
    }
}

}  // namespace vdwlb

using namespace vdwlb;

struct vdwlb_batch {
    int n = 0, C = 0, dtype = 0, ny = 0;
    int taus = 0;  // 1: every instance has tau = 1, 2: none has, 0: mixed
    int dim = 2;   // 1: D1Q3 instances resident in LDS (k_batch1)
    int lmax = 0;  // D1Q3: largest instance, sites
    int spt = 1;   // D1Q3: sites per thread
    size_t lds1 = 0;  // D1Q3: dynamic LDS bytes per workgroup
    std::vector<int64_t> offset, rho_offset, sites;
    int64_t pool_elems = 0, rho_elems = 0;
    void* d_inst = nullptr;  // Instance<C>[n]
    int* d_order = nullptr;
    int* d_status = nullptr;
    int* d_counter = nullptr;
    int threads = 256;  // workgroup size of the persistent kernel
    int blocks = 0;     // resident workgroups (0: fill the device)
    int tb_k = 0;       // D2Q9: steps per temporal block (0: the step-by-step kernel)
    size_t tb_lds = 0;  // dynamic LDS bytes of the blocked kernel
    int tb_per = 1;     // resident workgroups of the blocked kernel per CU
    hipGraphExec_t graph = nullptr;
    const void *gA = nullptr, *gB = nullptr;
    int64_t gsteps = -1;
    int gblocks = 0, gthreads = 0;
    hipStream_t capture_stream = nullptr;
};

namespace {

vdwlb_status bfail(hipError_t e, const char* where) { return set_device_error(e, where); }

template <typename T, int C, int TX, int NY>
hipError_t launch_batch_shape(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s) {
    auto* inst = (const Instance<C>*)b.d_inst;
    if (b.taus == 1)
        hipLaunchKernelGGL((k_batch<T, C, TX, NY, 1>), dim3(blocks), dim3(TX * NY), 0, s, inst, b.d_order, b.n, (T*)A,
                           (T*)B, nsteps, b.d_counter, b.d_status);
    else if (b.taus == 2)
        hipLaunchKernelGGL((k_batch<T, C, TX, NY, 2>), dim3(blocks), dim3(TX * NY), 0, s, inst, b.d_order, b.n, (T*)A,
                           (T*)B, nsteps, b.d_counter, b.d_status);
    else
        hipLaunchKernelGGL((k_batch<T, C, TX, NY, 0>), dim3(blocks), dim3(TX * NY), 0, s, inst, b.d_order, b.n, (T*)A,
                           (T*)B, nsteps, b.d_counter, b.d_status);
    return hipGetLastError();
}

// Strip width of the blocked kernel for K steps per block: the block, strip
// plus halo, is W = TX + 6K = 64 columns of 4 rows, one thread per site (256
// threads; about 37-49 KB of LDS at C = 2 in FP64, so three or four
// workgroups share a CU).
template <int K>
struct TbShape {
    static constexpr int TX = 64 - 6 * K;
};

// Number of blocks of at most K steps for nsteps steps, with the parity of
// nsteps (the result then lands in the buffer a step-by-step run leaves it in).
int tb_blocks(int nsteps, int K) {
    if (nsteps <= 0) return 0;
    int nb = (nsteps + K - 1) / K;
    if ((nb ^ nsteps) & 1) ++nb;
    return nb;
}

template <typename T, int C, int K, int TAUS>
hipError_t launch_tb_k(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s, int what) {
    using S = TbShape<K>;
    using LB = BlockLds<T, C, S::TX, 4, K>;
    auto kern = k_batch_tb<T, C, S::TX, 4, K, TAUS>;
    const size_t lds = LB::bytes;
    if (what == 1) {  // LDS attribute and resident workgroups per CU, outside any stream capture
        b.tb_lds = lds;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        int per = 0;
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, LB::NT, lds);
        if (e == hipSuccess) b.tb_per = std::max(1, per);
        return e;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(LB::NT), lds, s, (const Instance<C>*)b.d_inst, b.d_order, b.n, (T*)A,
                       (T*)B, nsteps, tb_blocks(nsteps, K), b.d_counter, b.d_status);
    return hipGetLastError();
}

// what: 0 launch, 1 set the LDS attribute of every collision variant and
// record the resident workgroups per CU.
template <typename T, int C, int K>
hipError_t launch_tb_t(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s, int what) {
    if (what == 1) {
        hipError_t e = launch_tb_k<T, C, K, 0>(b, A, B, nsteps, blocks, s, 1);
        if (e == hipSuccess) e = launch_tb_k<T, C, K, 1>(b, A, B, nsteps, blocks, s, 1);
        if (e == hipSuccess) e = launch_tb_k<T, C, K, 2>(b, A, B, nsteps, blocks, s, 1);
        return e;
    }
    if (b.taus == 1) return launch_tb_k<T, C, K, 1>(b, A, B, nsteps, blocks, s, what);
    if (b.taus == 2) return launch_tb_k<T, C, K, 2>(b, A, B, nsteps, blocks, s, what);
    return launch_tb_k<T, C, K, 0>(b, A, B, nsteps, blocks, s, what);
}

template <typename T, int C>
hipError_t launch_tb_c(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s, int what) {
    switch (b.tb_k) {
        case 2: return launch_tb_t<T, C, 2>(b, A, B, nsteps, blocks, s, what);
        case 3: return launch_tb_t<T, C, 3>(b, A, B, nsteps, blocks, s, what);
        case 4: return launch_tb_t<T, C, 4>(b, A, B, nsteps, blocks, s, what);
        case 5: return launch_tb_t<T, C, 5>(b, A, B, nsteps, blocks, s, what);
        case 6: return launch_tb_t<T, C, 6>(b, A, B, nsteps, blocks, s, what);
        default: return hipErrorInvalidValue;
    }
}

// The blocked kernel exists for C = 1, 2 in either precision and height 4.
hipError_t launch_tb(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s, int what) {
    if (b.dim != 2 || b.ny != 4) return hipErrorInvalidValue;
    if (b.dtype == VDWLB_F64)
        return b.C == 1 ? launch_tb_c<double, 1>(b, A, B, nsteps, blocks, s, what)
               : b.C == 2 ? launch_tb_c<double, 2>(b, A, B, nsteps, blocks, s, what)
                          : hipErrorInvalidValue;
    return b.C == 1 ? launch_tb_c<float, 1>(b, A, B, nsteps, blocks, s, what)
           : b.C == 2 ? launch_tb_c<float, 2>(b, A, B, nsteps, blocks, s, what)
                      : hipErrorInvalidValue;
}

template <typename T, int C, int THREADS>
hipError_t launch_batch_ny(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s) {
    switch (b.ny) {
        case 1:
            if constexpr (THREADS <= 256) return launch_batch_shape<T, C, THREADS, 1>(b, A, B, nsteps, blocks, s);
            break;
        case 2:
            if constexpr (THREADS <= 256) return launch_batch_shape<T, C, THREADS / 2, 2>(b, A, B, nsteps, blocks, s);
            break;
        case 4: return launch_batch_shape<T, C, THREADS / 4, 4>(b, A, B, nsteps, blocks, s);
        case 8: return launch_batch_shape<T, C, THREADS / 8, 8>(b, A, B, nsteps, blocks, s);
        default: break;
    }
    return hipErrorInvalidValue;
}

template <typename T, int C, int SPT, int TAUS>
hipError_t launch_batch1_k(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s, bool attr_only) {
    auto kern = k_batch1<T, C, SPT, TAUS>;
    if (attr_only)  // at creation, outside any stream capture
        return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)b.lds1);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(B1_THREADS), b.lds1, s, (const Instance<C>*)b.d_inst, b.d_order, b.n,
                       (T*)A, (T*)B, nsteps, b.lmax, b.d_counter, b.d_status);
    return hipGetLastError();
}

template <typename T, int C, int SPT>
hipError_t launch_batch1_t(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s, bool attr_only) {
    if (b.taus == 1) return launch_batch1_k<T, C, SPT, 1>(b, A, B, nsteps, blocks, s, attr_only);
    if (b.taus == 2) return launch_batch1_k<T, C, SPT, 2>(b, A, B, nsteps, blocks, s, attr_only);
    return launch_batch1_k<T, C, SPT, 0>(b, A, B, nsteps, blocks, s, attr_only);
}

template <typename T, int C>
hipError_t launch_batch1(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s, bool attr_only) {
    switch (b.spt) {
        case 1: return launch_batch1_t<T, C, 1>(b, A, B, nsteps, blocks, s, attr_only);
        case 2: return launch_batch1_t<T, C, 2>(b, A, B, nsteps, blocks, s, attr_only);
        case 4: return launch_batch1_t<T, C, 4>(b, A, B, nsteps, blocks, s, attr_only);
        case 8: return launch_batch1_t<T, C, 8>(b, A, B, nsteps, blocks, s, attr_only);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int C>
hipError_t launch_batch_c(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s) {
    if (b.dim == 1) return launch_batch1<T, C>(b, A, B, nsteps, blocks, s, false);
    // 1024-thread workgroups only for heights of 4 and 8 (wide strips of
    // 1- and 2-row lattices would exceed the LDS of a workgroup)
    if (b.threads == 1024 && b.ny >= 4) return launch_batch_ny<T, C, 1024>(b, A, B, nsteps, blocks, s);
    return launch_batch_ny<T, C, 256>(b, A, B, nsteps, blocks, s);
}

template <typename T>
hipError_t launch_batch_t(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s) {
    switch (b.C) {
        case 1: return launch_batch_c<T, 1>(b, A, B, nsteps, blocks, s);
        case 2: return launch_batch_c<T, 2>(b, A, B, nsteps, blocks, s);
        case 3: return launch_batch_c<T, 3>(b, A, B, nsteps, blocks, s);
        case 4: return launch_batch_c<T, 4>(b, A, B, nsteps, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch(vdwlb_batch& b, void* A, void* B, int nsteps, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, b.d_counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b.tb_k > 0) return launch_tb(b, A, B, nsteps, blocks, s, 0);
    return b.dtype == VDWLB_F64 ? launch_batch_t<double>(b, A, B, nsteps, blocks, s)
                                : launch_batch_t<float>(b, A, B, nsteps, blocks, s);
}

template <typename T, int C>
hipError_t aux_c(vdwlb_batch& b, int what, void* pool, void* rho, hipStream_t s) {
    if (b.dim == 1) {
        if (what == 0)
            hipLaunchKernelGGL((k_batch_init1<T, C>), dim3(b.n), dim3(256), 0, s, (const Instance<C>*)b.d_inst,
                               (T*)pool, (const T*)rho);
        else
            hipLaunchKernelGGL((k_batch_rho1<T, C>), dim3(b.n), dim3(256), 0, s, (const Instance<C>*)b.d_inst,
                               (const T*)pool, (T*)rho);
        return hipGetLastError();
    }
    if (what == 0)
        hipLaunchKernelGGL((k_batch_init<T, C>), dim3(b.n), dim3(256), 0, s, (const Instance<C>*)b.d_inst, (T*)pool,
                           (const T*)rho);
    else
        hipLaunchKernelGGL((k_batch_rho<T, C>), dim3(b.n), dim3(256), 0, s, (const Instance<C>*)b.d_inst,
                           (const T*)pool, (T*)rho);
    return hipGetLastError();
}

template <typename T>
hipError_t aux_t(vdwlb_batch& b, int what, void* pool, void* rho, hipStream_t s) {
    switch (b.C) {
        case 1: return aux_c<T, 1>(b, what, pool, rho, s);
        case 2: return aux_c<T, 2>(b, what, pool, rho, s);
        case 3: return aux_c<T, 3>(b, what, pool, rho, s);
        case 4: return aux_c<T, 4>(b, what, pool, rho, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t batch_aux(vdwlb_batch& b, int what, void* pool, void* rho, hipStream_t s) {
    return b.dtype == VDWLB_F64 ? aux_t<double>(b, what, pool, rho, s) : aux_t<float>(b, what, pool, rho, s);
}

template <int C>
void fill_instances(vdwlb_batch& b, const std::vector<vdwlb_plan>& plans, std::vector<char>& bytes) {
    bytes.assign(sizeof(Instance<C>) * b.n, 0);
    Instance<C>* I = reinterpret_cast<Instance<C>*>(bytes.data());
    for (int k = 0; k < b.n; ++k) {
        const vdwlb_plan& p = plans[k];
        // the periodic-wrap mode depends on the strip width and is set in the kernel
        I[k].g = make_geometry(p, 32, b.ny);
        I[k].g.band_w = 0;
        I[k].offset = b.offset[k];
        I[k].rho_offset = b.rho_offset[k];
        I[k].k = make_coeffs<C>(p);
    }
}

bool pool_aligned(const vdwlb_batch& b, const void* pool) {
    return reinterpret_cast<uintptr_t>(pool) % state_alignment(b.C, b.dtype) == 0;
}

int device_blocks(const vdwlb_batch& b) {
    int dev = 0, cus = 256;
    size_t lds_cu = 160 * 1024;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            cus = prop.multiProcessorCount;
            if (prop.maxSharedMemoryPerMultiProcessor > 0) lds_cu = prop.maxSharedMemoryPerMultiProcessor;
        }
    }
    if (b.dim == 1) {  // as many resident workgroups as the LDS of a CU holds
        const size_t per = std::max<size_t>(1, std::min<size_t>(8, lds_cu / std::max<size_t>(b.lds1 + 64, 1)));
        return cus * (int)per;
    }
    if (b.tb_k > 0) return cus * b.tb_per;  // as many as fit a CU's LDS and waves
    const int per_cu = (b.threads == 1024 && b.ny >= 4) ? 1 : 4;
    return cus * per_cu;
}

void release_batch_graph(vdwlb_batch& b) {
    if (b.graph) (void)hipGraphExecDestroy(b.graph);
    b.graph = nullptr;
    b.gA = b.gB = nullptr;
    b.gsteps = -1;
}

}  // namespace

extern "C" {

vdwlb_status vdwlb_batch_create(int32_t n, const vdwlb_desc* descs, vdwlb_batch** out) {
    if (!out) return VDWLB_E_INVALID_ARG;
    *out = nullptr;
    if (n < 1 || !descs) return VDWLB_E_INVALID_ARG;
    std::vector<vdwlb_plan*> tmp(n, nullptr);
    std::vector<vdwlb_plan> plans;
    plans.reserve(n);
    const int C = descs[0].ncomp, dtype = descs[0].dtype, ny = descs[0].ny, dim = descs[0].dim;
    for (int k = 0; k < n; ++k) {
        if (descs[k].ncomp != C || descs[k].dtype != dtype || descs[k].ny != ny || descs[k].dim != dim)
            return VDWLB_E_INVALID_ARG;
    }
    // Validate every description with the plan rules, on host data only.
    for (int k = 0; k < n; ++k) {
        vdwlb_status st = validate_desc(&descs[k]);
        if (st != VDWLB_OK) return st;
        plans.push_back(plan_from_desc(descs[k]));
    }
    if (ny != 1 && ny != 2 && ny != 4 && ny != 8) return VDWLB_E_UNSUPPORTED;
    // D1Q3: every instance must fit the LDS of one workgroup
    int lmax = 0;
    for (const vdwlb_plan& q : plans) lmax = std::max(lmax, q.nx);
    const size_t lds1 = (size_t)5 * C * lmax * (dtype == VDWLB_F64 ? 8 : 4);
    int spt = 1;
    while (spt * 256 < lmax) spt *= 2;
    if (dim == 1) {
        int dev = 0;
        hipDeviceProp_t prop;
        size_t lds_wg = 64 * 1024;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            lds_wg = prop.sharedMemPerBlock;
        if (spt > 8 || lds1 + 64 > lds_wg) return VDWLB_E_UNSUPPORTED;
    }

    vdwlb_batch* b = new (std::nothrow) vdwlb_batch();
    if (!b) return VDWLB_E_DEVICE;
    b->n = n;
    b->C = C;
    b->dtype = dtype;
    b->ny = ny;
    b->dim = dim;
    b->lmax = lmax;
    b->spt = spt;
    b->lds1 = lds1;
    int n_tau1 = 0;
    for (const vdwlb_plan& q : plans) n_tau1 += q.tau == 1.0 ? 1 : 0;
    b->taus = n_tau1 == n ? 1 : (n_tau1 == 0 ? 2 : 0);
    b->offset.resize(n);
    b->rho_offset.resize(n);
    b->sites.resize(n);
    int64_t off = 0, roff = 0;
    for (int k = 0; k < n; ++k) {
        b->offset[k] = off;
        b->rho_offset[k] = roff;
        b->sites[k] = (int64_t)plans[k].nx * plans[k].ny;
        off += (int64_t)(dim == 1 ? Q1 : Q) * C * plans[k].plane;
        roff += (int64_t)C * b->sites[k];
    }
    b->pool_elems = off;
    b->rho_elems = roff;
    std::vector<char> bytes;
    switch (C) {
        case 1: fill_instances<1>(*b, plans, bytes); break;
        case 2: fill_instances<2>(*b, plans, bytes); break;
        case 3: fill_instances<3>(*b, plans, bytes); break;
        default: fill_instances<4>(*b, plans, bytes); break;
    }
    // Longest processing time first: largest instances at the head of the queue.
    std::vector<int> order(n);
    for (int k = 0; k < n; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return b->sites[i] > b->sites[j]; });
    hipError_t e = hipMalloc(&b->d_inst, bytes.size());
    if (e == hipSuccess) e = hipMalloc(&b->d_order, sizeof(int) * n);
    if (e == hipSuccess) e = hipMalloc(&b->d_status, sizeof(int) * n);
    if (e == hipSuccess) e = hipMalloc(&b->d_counter, 256);
    if (e == hipSuccess) e = hipMemcpy(b->d_inst, bytes.data(), bytes.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_order, order.data(), sizeof(int) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->d_status, 0, sizeof(int) * n);
    if (e == hipSuccess) e = hipMemset(b->d_counter, 0, 256);
    if (e == hipSuccess && dim == 1)
        e = b->dtype == VDWLB_F64
                ? (C == 1   ? launch_batch1<double, 1>(*b, nullptr, nullptr, 0, 0, nullptr, true)
                   : C == 2 ? launch_batch1<double, 2>(*b, nullptr, nullptr, 0, 0, nullptr, true)
                   : C == 3 ? launch_batch1<double, 3>(*b, nullptr, nullptr, 0, 0, nullptr, true)
                            : launch_batch1<double, 4>(*b, nullptr, nullptr, 0, 0, nullptr, true))
                : (C == 1   ? launch_batch1<float, 1>(*b, nullptr, nullptr, 0, 0, nullptr, true)
                   : C == 2 ? launch_batch1<float, 2>(*b, nullptr, nullptr, 0, 0, nullptr, true)
                   : C == 3 ? launch_batch1<float, 3>(*b, nullptr, nullptr, 0, 0, nullptr, true)
                            : launch_batch1<float, 4>(*b, nullptr, nullptr, 0, 0, nullptr, true));
    if (e != hipSuccess) {
        vdwlb_batch_destroy(b);
        return bfail(e, "batch device buffers");
    }
    // D2Q9 batches of height 4 run with temporal blocking by default (3 steps
    // per block: the fastest measured on the 1024-lattice workload)
    if (dim == 2 && ny == 4 && C <= 2) {
        const vdwlb_status st = vdwlb_batch_set_blocking(b, 3);
        if (st != VDWLB_OK && st != VDWLB_E_UNSUPPORTED) {
            vdwlb_batch_destroy(b);
            return st;
        }
    }
    *out = b;
    return VDWLB_OK;
}

vdwlb_status vdwlb_batch_destroy(vdwlb_batch* b) {
    if (!b) return VDWLB_OK;
    release_batch_graph(*b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->d_order) (void)hipFree(b->d_order);
    if (b->d_status) (void)hipFree(b->d_status);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
    return VDWLB_OK;
}

size_t vdwlb_batch_state_bytes(const vdwlb_batch* b) {
    return b ? (size_t)b->pool_elems * (b->dtype == VDWLB_F64 ? 8 : 4) : 0;
}

int64_t vdwlb_batch_offset(const vdwlb_batch* b, int32_t k) {
    return (b && k >= 0 && k < b->n) ? b->offset[k] : -1;
}

int64_t vdwlb_batch_density_offset(const vdwlb_batch* b, int32_t k) {
    return (b && k >= 0 && k < b->n) ? b->rho_offset[k] : -1;
}

vdwlb_status vdwlb_batch_set_launch(vdwlb_batch* b, int32_t threads, int32_t blocks) {
    if (!b || (threads != 256 && threads != 1024) || blocks < 0) return VDWLB_E_INVALID_ARG;
    if (threads != b->threads || blocks != b->blocks) release_batch_graph(*b);
    b->threads = threads;
    b->blocks = blocks;
    return VDWLB_OK;
}

vdwlb_status vdwlb_batch_set_blocking(vdwlb_batch* b, int32_t steps_per_block) {
    if (!b || steps_per_block < 0 || steps_per_block == 1 || steps_per_block > 6) return VDWLB_E_INVALID_ARG;
    if (steps_per_block == b->tb_k) return VDWLB_OK;
    if (steps_per_block > 0) {
        if (b->dim != 2 || b->ny != 4 || b->C > 2) return VDWLB_E_UNSUPPORTED;
        const int keep = b->tb_k;
        b->tb_k = steps_per_block;
        size_t lds_wg = 64 * 1024;
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            lds_wg = prop.sharedMemPerBlock;
        hipError_t e = launch_tb(*b, nullptr, nullptr, 0, 0, nullptr, 1);
        if (e == hipSuccess && b->tb_lds > lds_wg) e = hipErrorInvalidValue;
        if (e != hipSuccess) {
            b->tb_k = keep;
            (void)hipGetLastError();
            return b->tb_lds > lds_wg ? VDWLB_E_UNSUPPORTED : bfail(e, "batch blocking");
        }
    }
    release_batch_graph(*b);
    b->tb_k = steps_per_block;
    return VDWLB_OK;
}

vdwlb_status vdwlb_batch_init(vdwlb_batch* b, void* pool, const void* rho, void* stream) {
    if (!b || !pool || !rho || !pool_aligned(*b, pool)) return VDWLB_E_INVALID_ARG;
    hipError_t e = batch_aux(*b, 0, pool, const_cast<void*>(rho), (hipStream_t)stream);
    return e == hipSuccess ? VDWLB_OK : bfail(e, "batch init");
}

vdwlb_status vdwlb_batch_density(vdwlb_batch* b, const void* pool, void* rho, void* stream) {
    if (!b || !pool || !rho || !pool_aligned(*b, pool)) return VDWLB_E_INVALID_ARG;
    hipError_t e = batch_aux(*b, 1, const_cast<void*>(pool), rho, (hipStream_t)stream);
    return e == hipSuccess ? VDWLB_OK : bfail(e, "batch density");
}

vdwlb_status vdwlb_batch_run(vdwlb_batch* b, void* poolA, void* poolB, int64_t nsteps, void* stream,
                             int32_t* out_which) {
    if (!b || !poolA || !poolB || poolA == poolB || nsteps < 0 || nsteps > 0x7fffffff) return VDWLB_E_INVALID_ARG;
    if (!pool_aligned(*b, poolA) || !pool_aligned(*b, poolB)) return VDWLB_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    int blocks = b->blocks > 0 ? b->blocks : device_blocks(*b);
    if (blocks > b->n) blocks = b->n;
    if (!(b->graph && b->gA == poolA && b->gB == poolB && b->gsteps == nsteps && b->gblocks == blocks &&
          b->gthreads == b->threads)) {
        release_batch_graph(*b);
        hipError_t e = hipSuccess;
        if (!b->capture_stream) e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return bfail(e, "batch capture");
        hipError_t le = launch_batch(*b, poolA, poolB, (int)nsteps, blocks, b->capture_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->capture_stream, &g);
        if (le != hipSuccess || e != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return bfail(le != hipSuccess ? le : e, "batch capture");
        }
        e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->graph = nullptr;
            return bfail(e, "batch graph instantiate");
        }
        b->gA = poolA;
        b->gB = poolB;
        b->gsteps = nsteps;
        b->gblocks = blocks;
        b->gthreads = b->threads;
    }
    hipError_t e = hipGraphLaunch(b->graph, s);
    if (e != hipSuccess) return bfail(e, "batch graph launch");
    if (out_which) *out_which = (int32_t)(nsteps & 1);
    return VDWLB_OK;
}

vdwlb_status vdwlb_batch_status(vdwlb_batch* b, int32_t* per_instance, void* stream) {
    if (!b) return VDWLB_E_INVALID_ARG;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return bfail(e, "batch status");
    std::vector<int32_t> st(b->n);
    e = hipMemcpy(st.data(), b->d_status, sizeof(int32_t) * b->n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bfail(e, "batch status");
    if (per_instance) std::memcpy(per_instance, st.data(), sizeof(int32_t) * b->n);
    for (int k = 0; k < b->n; ++k)
        if (st[k]) return VDWLB_E_UNPHYSICAL;
    return VDWLB_OK;
}

}  // extern "C"
