// Diagnostics of a density field: the pressure tensor of Sec. II (the tensor
// that satisfies Eq. GibbsDuehem for the van der Waals mixture free energy)
//   P_ab = sum_c [rho^c kT/(1 - eta) - sum_c' a^{cc'} rho^c rho^c'
//                 - sum_c' kappa^{cc'} (grad rho^c . grad rho^c' + rho^c Lap rho^c')] delta_ab
//          + sum_cc' kappa^{cc'} d_a rho^c d_b rho^c'
// with the lattice's own isotropic stencils (D2Q9: 9-point gradient and
// Laplacian; D1Q3: central difference and 3-point Laplacian).  One thread per
// site reads the 3 x 3 (or 3) neighbourhood of every component.
#include "../../include/vdwlb.h"
#include "launch.hpp"

namespace vdwlb {
namespace {

template <typename T, int C, int DIM>
__global__ void __launch_bounds__(256) k_ptensor(const T* __restrict__ rho, T* __restrict__ pxx, T* __restrict__ pyy,
                                                 T* __restrict__ pxy, int nx, int ny, Coeffs<C, T> k) {
    const int n = nx * ny;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int y = s / nx, x = s - y * nx;
    const int xm = wrapc(x - 1, nx, 1), xp = wrapc(x + 1, nx, 1);
    T r[C], gx[C], gy[C], lap[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const T* R = rho + (int64_t)c * n;
        if constexpr (DIM == 1) {
            r[c] = R[x];
            gx[c] = grad3<T>(R[xm], R[xp]);
            gy[c] = T(0);
            lap[c] = lap3<T>(R[xm], r[c], R[xp]);
        } else {
            const int ym = wrapc(y - 1, ny, 1), yp = wrapc(y + 1, ny, 1);
            const int r0 = y * nx, rm = ym * nx, rp = yp * nx;
            const T c0 = R[r0 + x], e = R[r0 + xp], w = R[r0 + xm], nn = R[rp + x], ss = R[rm + x];
            const T ne = R[rp + xp], nw = R[rp + xm], sw = R[rm + xm], se = R[rm + xp];
            r[c] = c0;
            gx[c] = (T(4) * (e - w) + ((ne - nw) + (se - sw))) * T(1.0 / 12.0);
            gy[c] = (T(4) * (nn - ss) + ((ne + nw) - (sw + se))) * T(1.0 / 12.0);
            lap[c] = (T(4) * ((e + w) + (nn + ss)) + ((ne + nw) + (sw + se)) - T(20) * c0) * T(1.0 / 6.0);
        }
    }
    T eta = T(0), tot = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        eta += T(k.b[c]) * r[c];
        tot += r[c];
    }
    T scalar = tot * T(k.kT) / (T(1) - eta), txx = T(0), tyy = T(0), txy = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int d = 0; d < C; ++d) {
            const T kap = T(k.kap(c, d));
            scalar -= T(0.5) * T(k.a2(c, d)) * r[c] * r[d] + kap * ((gx[c] * gx[d] + gy[c] * gy[d]) + r[c] * lap[d]);
            txx += kap * gx[c] * gx[d];
            tyy += kap * gy[c] * gy[d];
            txy += kap * gx[c] * gy[d];
        }
    pxx[s] = scalar + txx;
    if (pyy) pyy[s] = scalar + tyy;
    if (pxy) pxy[s] = txy;
}

template <typename T, int C>
hipError_t ptensor_c(const vdwlb_plan& p, const void* rho, void* pxx, void* pyy, void* pxy, hipStream_t s) {
    const int n = p.nx * p.ny;
    const unsigned nb = (unsigned)((n + 255) / 256);
    const Coeffs<C, T> k = make_coeffs<C, T>(p);
    if (p.dim == 1)
        hipLaunchKernelGGL((k_ptensor<T, C, 1>), dim3(nb), dim3(256), 0, s, (const T*)rho, (T*)pxx, (T*)pyy, (T*)pxy,
                           p.nx, p.ny, k);
    else
        hipLaunchKernelGGL((k_ptensor<T, C, 2>), dim3(nb), dim3(256), 0, s, (const T*)rho, (T*)pxx, (T*)pyy, (T*)pxy,
                           p.nx, p.ny, k);
    return hipGetLastError();
}

template <typename T>
hipError_t ptensor_t(const vdwlb_plan& p, const void* rho, void* pxx, void* pyy, void* pxy, hipStream_t s) {
    switch (p.C) {
        case 1: return ptensor_c<T, 1>(p, rho, pxx, pyy, pxy, s);
        case 2: return ptensor_c<T, 2>(p, rho, pxx, pyy, pxy, s);
        case 3: return ptensor_c<T, 3>(p, rho, pxx, pyy, pxy, s);
        case 4: return ptensor_c<T, 4>(p, rho, pxx, pyy, pxy, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace vdwlb

using namespace vdwlb;

extern "C" vdwlb_status vdwlb_pressure_tensor(vdwlb_plan* p, const void* rho, void* pxx, void* pyy, void* pxy,
                                              void* stream) {
    if (!p || !rho || !pxx) return VDWLB_E_INVALID_ARG;
    const hipError_t e = p->dtype == VDWLB_F64 ? ptensor_t<double>(*p, rho, pxx, pyy, pxy, (hipStream_t)stream)
                                               : ptensor_t<float>(*p, rho, pxx, pyy, pxy, (hipStream_t)stream);
    return e == hipSuccess ? VDWLB_OK : set_device_error(e, "pressure tensor kernel");
}
