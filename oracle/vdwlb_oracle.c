/*
 * Oracle for the multicomponent van der Waals free-energy lattice Boltzmann
 * sweep (Ridl & Wagner, "Lattice Boltzmann simulation of mixtures with
 * multicomponent van der Waals equation of state", arXiv:1805.07251).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, deliberately
 * unoptimised CPU implementation used to check the GPU library.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant with the GPU path.
 *
 * Everything is computed whole-lattice, one stage at a time, in the order the
 * paper states the method:
 *   stream (Eq. LBequation) -> moments (Sec. III, definitions of rho^c and
 *   rho^c u^c) -> chemical potential from the interaction function psi
 *   (Eq. discreteChemicalPotential) -> mean-field force (Eq. forceMuLog or
 *   Eq. forceMuId) -> implicit friction (Eq. forceFriction with the
 *   definition of the true velocity u-hat) -> forced BGK collision
 *   (Eqs. BGKcollisionOperator, feq and the forcing moments with the
 *   correction of Eq. forceCorrectionsPsi).
 *
 * Readings of the paper used here (each is justified by a test pin):
 *  - The force added to the momentum of component c is the physical force
 *    G^c = -gamma rho^c grad mu^c + theta grad rho^c + sum_c' lambda m (uh^c'-uh^c).
 *    The printed Eqs. forceMuLog/forceFriction carry the opposite sign (they
 *    are written as "minus the force", cf. the momentum equation of Sec. IV).
 *  - Second moment of the forcing term: S = G u + u G + (1/tau)[(tau-1/4) G G/rho
 *    + (1/12) Lap(rho) I], i.e. the sign the explicit D1Q3 update of Sec. V
 *    realises, with Psi of Eq. forceCorrectionsPsi.
 *  - u^c in f^0 and in G u is the bare j^c/rho^c; u-hat only enters friction.
 *  - kT is the thermodynamic temperature (enters mu and p); the lattice
 *    temperature theta = 1/3 enters f^0, the ideal-gas subtraction of the
 *    force and the 1/12 = theta/4 of Psi.  With kT = 1/3 this is the paper.
 *  - D2Q9 extension (the paper is 1-D): BGK with the standard D2Q9 velocity set
 *    and weights, Hermite forcing with the moments of Sec. III, the isotropic
 *    gradient 3 sum_i w_i v_i g(x+v_i), and the 2-D interaction function
 *    psi(0) = (5/3) kappa - a, psi(v_i) = -3 w_i kappa (i != 0), which obeys
 *    Eqs. a-psi and kappa-psi and reduces to the D1Q3 psi on y-uniform data.
 *  - The additive constant theta of d(rho ln rho)/d rho is dropped from mu, as
 *    in Eq. discreteChemicalPotential.
 *
 * Layout: populations f[c][i][y][x] (x fastest), sites s = y*nx + x, periodic.
 * The stored state is post-collision, pre-stream: one step pulls
 * f_i(x - v_i) and collides.
 *
 * Scalar type: built twice, once with real_t = double and once with
 * real_t = double complex (-DORC_COMPLEX, symbols suffixed _cx), so the same
 * arithmetic gives complex-step derivatives (Squire & Trapp 1998).
 *
 * Threads: the per-site loops of large lattices are split over OpenMP threads
 * (orc_set_threads).  Every site's arithmetic is the same whatever thread
 * runs it and no value is summed across sites, so results do not depend on
 * the thread count (checked bit for bit by the tests).
 */
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_COMPLEX
#include <complex.h>
typedef double complex real_t;
#define SFX(name) name##_cx
#define RE(x) creal(x)
#else
typedef double real_t;
#define SFX(name) name
#define RE(x) (x)
#endif
#include <tgmath.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Lattices with fewer sites run their loops on one thread. */
#define ORC_PAR_MIN 16384

#define ORC_OK 0
#define ORC_INVALID 1
#define ORC_UNPHYSICAL 4

/* Static description of one lattice (mirrored by a ctypes Structure). */
typedef struct {
    int dim;     /* 1: D1Q3 (ny must be 1), 2: D2Q9 */
    int nx, ny;  /* lattice extents, periodic */
    int C;       /* number of components */
    int force;   /* 0: "log" forcing (Eq. forceMuLog), 1: "nid" (Eq. forceMuId) */
    double tau;  /* BGK relaxation time */
    double gamma_mu; /* free-energy prefactor of the force (Eq. forceMuNid) */
} orc_config;

/* Lattice temperature of the BGK equilibrium, theta = 1/3 (Sec. V). */
static const double THETA_LB = 1.0 / 3.0;

/* D1Q3 (Sec. V): v in {0, +1, -1}; weights make f^0 of Eq. feq equal to the
 * explicit D1Q3 equilibria: w0 = 1 - theta, w+- = theta/2. */
static const int D1_VX[3] = {0, 1, -1};
static const double D1_W[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};

/* D2Q9: rest, four axis and four diagonal velocities. */
static const int D2_VX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int D2_VY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double D2_W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

typedef struct {
    int Q;
    const int* vx;
    int vy[9];
    const double* w;
} lattice_t;

static lattice_t lattice_of(int dim) {
    lattice_t L;
    memset(&L, 0, sizeof L);
    if (dim == 1) {
        L.Q = 3;
        L.vx = D1_VX;
        L.w = D1_W;
    } else {
        L.Q = 9;
        L.vx = D2_VX;
        for (int i = 0; i < 9; ++i) L.vy[i] = D2_VY[i];
        L.w = D2_W;
    }
    return L;
}

#ifndef ORC_COMPLEX
/* Threads for the per-site loops (n <= 0: the OpenMP default); returns the
 * count now in effect (1 without OpenMP). */
int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
#endif

static int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

static int check_config(const orc_config* k) {
    if (k->dim != 1 && k->dim != 2) return ORC_INVALID;
    if (k->nx < 1 || k->ny < 1 || k->C < 1) return ORC_INVALID;
    if (k->dim == 1 && k->ny != 1) return ORC_INVALID;
    if (!(k->tau > 0.5)) return ORC_INVALID;
    if (k->force != 0 && k->force != 1) return ORC_INVALID;
    return ORC_OK;
}

/* Parameter vector (real_t so that complex-step can perturb any entry):
 *   prm[0]                    kT
 *   prm[1 .. C*C]             a^{cc'}   (row-major, symmetric)
 *   prm[1+C*C .. C*C+C]       b^c
 *   prm[1+C*C+C .. 2C*C+C]    kappa^{cc'}
 * lambda^{cc'} (friction, Eq. forceFriction) is a separate double array. */
#define PRM_KT(prm) ((prm)[0])
#define PRM_A(prm, C, c, d) ((prm)[1 + (c) * (C) + (d)])
#define PRM_B(prm, C, c) ((prm)[1 + (C) * (C) + (c)])
#define PRM_K(prm, C, c, d) ((prm)[1 + (C) * (C) + (C) + (c) * (C) + (d)])

/* Interaction function psi^{cc'}(v_k) of Eq. discreteFreeEnergy on the lattice
 * neighbourhood.  D1Q3: psi(0) = kappa - a, psi(+-1) = -kappa/2 (Sec. V,
 * from Eqs. kappa-psi-D1Q3 and a-psi-D1Q3).  D2Q9: psi(0) = (5/3) kappa - a,
 * psi(v_k) = -3 w_k kappa, so that -sum psi = a and -sum psi v_x^2 = kappa. */
static real_t psi(const lattice_t* L, int dim, real_t a, real_t kappa, int k) {
    if (dim == 1) {
        if (k == 0) return kappa - a;
        return -0.5 * kappa;
    }
    if (k == 0) return (5.0 / 3.0) * kappa - a;
    return -3.0 * L->w[k] * kappa;
}

/* Neighbour of site s along velocity k. */
static size_t nbr(const lattice_t* L, int nx, int ny, size_t s, int k) {
    int x = (int)(s % (size_t)nx), y = (int)(s / (size_t)nx);
    return (size_t)wrap(y + L->vy[k], ny) * (size_t)nx + (size_t)wrap(x + L->vx[k], nx);
}

/* Isotropic discrete gradient, 3 sum_k w_k v_k g(x+v_k): the central
 * difference of Eqs. forceMuId/forceMuLog in 1-D. */
static void grad_at(const lattice_t* L, int nx, int ny, const real_t* g, size_t s, real_t* gx, real_t* gy) {
    real_t sx = 0, sy = 0;
    for (int k = 1; k < L->Q; ++k) {
        size_t t = nbr(L, nx, ny, s, k);
        sx += L->w[k] * L->vx[k] * g[t];
        sy += L->w[k] * L->vy[k] * g[t];
    }
    *gx = 3.0 * sx;
    *gy = 3.0 * sy;
}

/* Isotropic discrete Laplacian, 6 sum_k w_k (g(x+v_k) - g(x)): the standard
 * 3-point stencil in 1-D (Sec. V). */
static real_t lap_at(const lattice_t* L, int nx, int ny, const real_t* g, size_t s) {
    real_t acc = 0;
    for (int k = 1; k < L->Q; ++k) acc += L->w[k] * (g[nbr(L, nx, ny, s, k)] - g[s]);
    return 6.0 * acc;
}

static int is_bad(real_t v) {
    double r = RE(v);
    return !isfinite(r);
}

/* Equilibrium of Eq. feq with lattice temperature theta. */
static real_t feq(const lattice_t* L, int k, real_t rho, real_t ux, real_t uy) {
    real_t vu = L->vx[k] * ux + L->vy[k] * uy;
    real_t uu = ux * ux + uy * uy;
    return rho * L->w[k] *
           (1.0 + vu / THETA_LB + vu * vu / (2.0 * THETA_LB * THETA_LB) - uu / (2.0 * THETA_LB));
}

/* Solve A x = r for a small dense system by Gaussian elimination (A is
 * symmetric positive definite here, so no pivoting is needed). A, r are
 * overwritten. */
static void solve_small(int n, real_t* A, real_t* r, real_t* x) {
    for (int p = 0; p < n; ++p) {
        for (int q = p + 1; q < n; ++q) {
            real_t f = A[q * n + p] / A[p * n + p];
            for (int m = p; m < n; ++m) A[q * n + m] -= f * A[p * n + m];
            r[q] -= f * r[p];
        }
    }
    for (int p = n - 1; p >= 0; --p) {
        real_t acc = r[p];
        for (int m = p + 1; m < n; ++m) acc -= A[p * n + m] * x[m];
        x[p] = acc / A[p * n + p];
    }
}

/* Chemical potential of Eq. discreteChemicalPotential at every site, for
 * given density fields rho[c][s]; also flags unphysical sites. */
static int chem_pot(const orc_config* k, const lattice_t* L, const real_t* prm, const real_t* rho, real_t* mu) {
    const int C = k->C, nx = k->nx, ny = k->ny;
    const size_t N = (size_t)nx * ny;
    int bad = 0;
#pragma omp parallel for reduction(| : bad) if (N >= ORC_PAR_MIN)
    for (size_t s = 0; s < N; ++s) {
        real_t eta = 0, rt = 0;
        for (int c = 0; c < C; ++c) {
            eta += PRM_B(prm, C, c) * rho[c * N + s];
            rt += rho[c * N + s];
            if (!(RE(rho[c * N + s]) > 0.0) || is_bad(rho[c * N + s])) bad = 1;
        }
        if (!(RE(eta) < 1.0)) bad = 1;
        for (int c = 0; c < C; ++c) {
            real_t m = PRM_KT(prm) * (log(rho[c * N + s] / (1.0 - eta)) + PRM_B(prm, C, c) * rt / (1.0 - eta));
            for (int d = 0; d < C; ++d)
                for (int q = 0; q < L->Q; ++q)
                    m += 2.0 * psi(L, k->dim, PRM_A(prm, C, c, d), PRM_K(prm, C, c, d), q) *
                         rho[d * N + nbr(L, nx, ny, s, q)];
            mu[c * N + s] = m;
            if (is_bad(m)) bad = 1;
        }
    }
    return bad ? ORC_UNPHYSICAL : ORC_OK;
}

/* Moments of the streamed populations: rho^c = sum_i f_i^c,
 * rho^c u^c = sum_i f_i^c v_i (Sec. III). */
static void moments_of(const orc_config* k, const lattice_t* L, const real_t* p, real_t* rho, real_t* jx, real_t* jy) {
    const size_t N = (size_t)k->nx * k->ny;
    for (int c = 0; c < k->C; ++c)
#pragma omp parallel for if (N >= ORC_PAR_MIN)
        for (size_t s = 0; s < N; ++s) {
            real_t r = 0, x = 0, y = 0;
            for (int i = 0; i < L->Q; ++i) {
                real_t v = p[((size_t)c * L->Q + i) * N + s];
                r += v;
                x += v * L->vx[i];
                y += v * L->vy[i];
            }
            rho[c * N + s] = r;
            jx[c * N + s] = x;
            jy[c * N + s] = y;
        }
}

/* Pull-streaming: p_i(x) = f*_i(x - v_i) (Eq. LBequation, periodic). */
static void stream_pull(const orc_config* k, const lattice_t* L, const real_t* fin, real_t* p) {
    const int nx = k->nx, ny = k->ny;
    const size_t N = (size_t)nx * ny;
    for (int c = 0; c < k->C; ++c)
        for (int i = 0; i < L->Q; ++i)
#pragma omp parallel for if (N >= ORC_PAR_MIN)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t src = (size_t)wrap(y - L->vy[i], ny) * nx + (size_t)wrap(x - L->vx[i], nx);
                    p[((size_t)c * L->Q + i) * N + (size_t)y * nx + x] = fin[((size_t)c * L->Q + i) * N + src];
                }
}

/* One time step: state fin (post-collision at t) -> fout (post-collision at
 * t+1).  Returns ORC_UNPHYSICAL if any site had rho^c <= 0, eta >= 1 or a
 * non-finite value (the step is still completed). */
int SFX(orc_step)(const orc_config* k, const real_t* prm, const double* lambda, const real_t* fin, real_t* fout) {
    if (check_config(k) != ORC_OK) return ORC_INVALID;
    const lattice_t L = lattice_of(k->dim);
    const int C = k->C, nx = k->nx, ny = k->ny, Q = L.Q;
    const size_t N = (size_t)nx * ny;
    const double tau = k->tau, gam = k->gamma_mu;
    int status = ORC_OK;

    real_t* p = malloc(sizeof(real_t) * C * Q * N);
    real_t* rho = malloc(sizeof(real_t) * C * N);
    real_t* jx = malloc(sizeof(real_t) * C * N);
    real_t* jy = malloc(sizeof(real_t) * C * N);
    real_t* mu = malloc(sizeof(real_t) * C * N);
    real_t* phi = malloc(sizeof(real_t) * C * N);
    real_t* Gx = malloc(sizeof(real_t) * C * N);
    real_t* Gy = malloc(sizeof(real_t) * C * N);

    /* 1. stream */
    stream_pull(k, &L, fin, p);
    /* 2. moments */
    moments_of(k, &L, p, rho, jx, jy);
    /* 3. chemical potential (Eq. discreteChemicalPotential) */
    status = chem_pot(k, &L, prm, rho, mu);

    /* 4. mean-field force, physical sign.  log (Eq. forceMuLog):
     *    G = -rho grad(gamma mu) + theta grad(rho);
     *    nid (Eq. forceMuId): G = -rho grad(gamma mu - theta ln rho). */
    for (int c = 0; c < C; ++c)
#pragma omp parallel for if (N >= ORC_PAR_MIN)
        for (size_t s = 0; s < N; ++s)
            phi[c * N + s] = (k->force == 1) ? gam * mu[c * N + s] - THETA_LB * log(rho[c * N + s])
                                             : gam * mu[c * N + s];
    for (int c = 0; c < C; ++c)
#pragma omp parallel for if (N >= ORC_PAR_MIN)
        for (size_t s = 0; s < N; ++s) {
            real_t dpx, dpy;
            grad_at(&L, nx, ny, phi + c * N, s, &dpx, &dpy);
            Gx[c * N + s] = -rho[c * N + s] * dpx;
            Gy[c * N + s] = -rho[c * N + s] * dpy;
            if (k->force == 0) {
                real_t drx, dry;
                grad_at(&L, nx, ny, rho + c * N, s, &drx, &dry);
                Gx[c * N + s] += THETA_LB * drx;
                Gy[c * N + s] += THETA_LB * dry;
            }
        }

    /* 5. friction (Eq. forceFriction, physical sign) with the true velocities
     *    uh^c = u^c + G^c/(2 rho^c), G^c including the friction itself:
     *    rho^c uh^c - (1/2) sum_c' W^{cc'} (uh^c' - uh^c) = j^c + G^{mu,c}/2,
     *    W^{cc'} = lambda^{cc'} rho^c rho^c' / (rho^c + rho^c'). */
#pragma omp parallel if (N >= ORC_PAR_MIN)
    {
    real_t* A = malloc(sizeof(real_t) * C * C);
    real_t* r = malloc(sizeof(real_t) * C);
    real_t* uh = malloc(sizeof(real_t) * C);
    real_t* W = malloc(sizeof(real_t) * C * C);
#pragma omp for
    for (size_t s = 0; s < N; ++s) {
        for (int c = 0; c < C; ++c)
            for (int d = 0; d < C; ++d)
                W[c * C + d] = (c == d) ? 0.0
                                        : lambda[c * C + d] * rho[c * N + s] * rho[d * N + s] /
                                              (rho[c * N + s] + rho[d * N + s]);
        for (int axis = 0; axis < 2; ++axis) {
            real_t* j = axis == 0 ? jx : jy;
            real_t* G = axis == 0 ? Gx : Gy;
            for (int c = 0; c < C; ++c) {
                real_t diag = rho[c * N + s];
                for (int d = 0; d < C; ++d) {
                    if (d == c) continue;
                    diag += 0.5 * W[c * C + d];
                    A[c * C + d] = -0.5 * W[c * C + d];
                }
                A[c * C + c] = diag;
                r[c] = j[c * N + s] + 0.5 * G[c * N + s];
            }
            solve_small(C, A, r, uh);
            for (int c = 0; c < C; ++c) {
                real_t gf = 0;
                for (int d = 0; d < C; ++d) gf += W[c * C + d] * (uh[d] - uh[c]);
                G[c * N + s] += gf;
            }
        }
    }
    free(A);
    free(r);
    free(uh);
    free(W);
    }

    /* 6. forced BGK collision (Eqs. BGKcollisionOperator, feq, forcing
     *    moments with Psi of Eq. forceCorrectionsPsi). */
    int bad = 0;
    for (int c = 0; c < C; ++c)
#pragma omp parallel for reduction(| : bad) if (N >= ORC_PAR_MIN)
        for (size_t s = 0; s < N; ++s) {
            real_t rh = rho[c * N + s];
            real_t ux = jx[c * N + s] / rh, uy = jy[c * N + s] / rh;
            real_t gx = Gx[c * N + s], gy = Gy[c * N + s];
            real_t lr = lap_at(&L, nx, ny, rho + c * N, s);
            real_t iso = lr / 12.0;
            real_t Sxx = 2.0 * gx * ux + ((tau - 0.25) * gx * gx / rh + iso) / tau;
            real_t Syy = 2.0 * gy * uy + ((tau - 0.25) * gy * gy / rh + iso) / tau;
            real_t Sxy = gx * uy + ux * gy + ((tau - 0.25) * gx * gy / rh) / tau;
            for (int i = 0; i < Q; ++i) {
                size_t idx = ((size_t)c * Q + i) * N + s;
                real_t Fi;
                if (k->dim == 1) {
                    /* explicit D1Q3 forcing of Sec. V: F0 = -S, F+- = (S +- G)/2 */
                    if (i == 0) Fi = -Sxx;
                    else Fi = 0.5 * (Sxx + L.vx[i] * gx);
                } else {
                    /* Hermite form: w_i [G.v/theta + S:(v v - theta I)/(2 theta^2)] */
                    real_t vx = L.vx[i], vy = L.vy[i];
                    real_t gv = gx * vx + gy * vy;
                    real_t svv = Sxx * (vx * vx - THETA_LB) + Syy * (vy * vy - THETA_LB) + 2.0 * Sxy * vx * vy;
                    Fi = L.w[i] * (gv / THETA_LB + svv / (2.0 * THETA_LB * THETA_LB));
                }
                real_t f0 = feq(&L, i, rh, ux, uy);
                fout[idx] = p[idx] + (f0 - p[idx]) / tau + Fi;
                if (is_bad(fout[idx])) bad = 1;
            }
        }
    if (bad) status = ORC_UNPHYSICAL;

    free(p);
    free(rho);
    free(jx);
    free(jy);
    free(mu);
    free(phi);
    free(Gx);
    free(Gy);
    return status;
}

/* Run nsteps steps in place on f (work holds one extra state buffer). */
int SFX(orc_run)(const orc_config* k, const real_t* prm, const double* lambda, real_t* f, real_t* work, long nsteps) {
    if (check_config(k) != ORC_OK) return ORC_INVALID;
    const lattice_t L = lattice_of(k->dim);
    const size_t n = (size_t)k->C * L.Q * k->nx * k->ny;
    int status = ORC_OK;
    for (long t = 0; t < nsteps; ++t) {
        int st = SFX(orc_step)(k, prm, lambda, f, work);
        if (st != ORC_OK) status = st;
        memcpy(f, work, sizeof(real_t) * n);
    }
    return status;
}

/* Initial state: f_i^c = f^0_i(rho^c, u^c) with u = mom / rho (0 if mom is
 * NULL).  mom is [C][2][N] (x then y component; y ignored in 1-D). */
int SFX(orc_equilibrium_state)(const orc_config* k, const real_t* rho, const real_t* mom, real_t* f) {
    if (check_config(k) != ORC_OK) return ORC_INVALID;
    const lattice_t L = lattice_of(k->dim);
    const size_t N = (size_t)k->nx * k->ny;
    for (int c = 0; c < k->C; ++c)
        for (size_t s = 0; s < N; ++s) {
            real_t r = rho[c * N + s];
            real_t ux = mom ? mom[(2 * (size_t)c) * N + s] / r : 0.0;
            real_t uy = (mom && k->dim == 2) ? mom[(2 * (size_t)c + 1) * N + s] / r : 0.0;
            for (int i = 0; i < L.Q; ++i) f[((size_t)c * L.Q + i) * N + s] = feq(&L, i, r, ux, uy);
        }
    return ORC_OK;
}

/* Observables of a stored state: rho^c and j^c of the streamed populations,
 * mu^c (Eq. discreteChemicalPotential) and the bulk pressure
 * p = sum_c [rho^c kT/(1-eta) - sum_c' a^{cc'} rho^c rho^c'] (Sec. II).
 * Any output pointer may be NULL. mom is [C][2][N]. */
int SFX(orc_moments)(const orc_config* k, const real_t* prm, const real_t* f, real_t* rho_out, real_t* mom_out,
                     real_t* mu_out, real_t* p_out) {
    if (check_config(k) != ORC_OK) return ORC_INVALID;
    const lattice_t L = lattice_of(k->dim);
    const int C = k->C;
    const size_t N = (size_t)k->nx * k->ny;
    real_t* p = malloc(sizeof(real_t) * C * L.Q * N);
    real_t* rho = malloc(sizeof(real_t) * C * N);
    real_t* jx = malloc(sizeof(real_t) * C * N);
    real_t* jy = malloc(sizeof(real_t) * C * N);
    real_t* mu = malloc(sizeof(real_t) * C * N);
    stream_pull(k, &L, f, p);
    moments_of(k, &L, p, rho, jx, jy);
    int status = chem_pot(k, &L, prm, rho, mu);
    if (rho_out) memcpy(rho_out, rho, sizeof(real_t) * C * N);
    if (mom_out)
        for (int c = 0; c < C; ++c) {
            memcpy(mom_out + (2 * (size_t)c) * N, jx + (size_t)c * N, sizeof(real_t) * N);
            memcpy(mom_out + (2 * (size_t)c + 1) * N, jy + (size_t)c * N, sizeof(real_t) * N);
        }
    if (mu_out) memcpy(mu_out, mu, sizeof(real_t) * C * N);
    if (p_out)
        for (size_t s = 0; s < N; ++s) {
            real_t eta = 0;
            for (int c = 0; c < C; ++c) eta += PRM_B(prm, C, c) * rho[c * N + s];
            real_t pr = 0;
            for (int c = 0; c < C; ++c) {
                pr += rho[c * N + s] * PRM_KT(prm) / (1.0 - eta);
                for (int d = 0; d < C; ++d) pr -= PRM_A(prm, C, c, d) * rho[c * N + s] * rho[d * N + s];
            }
            p_out[s] = pr;
        }
    free(p);
    free(rho);
    free(jx);
    free(jy);
    free(mu);
    return status;
}
