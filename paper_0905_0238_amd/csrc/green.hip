// Kernel (a): reference Green's-function tables g(z; |k|, w) of a layered medium.
//
// Paper, Section 2.1: the reference Green's function solves the Helmholtz
// equation (w^2/c0(z)^2) G + lap G = -delta with a laterally invariant c0, so
// its horizontal transform depends on |k| only and obeys
//     g'' + (w^2/c0(z)^2 - k^2) g = -delta(z),
// with radiation conditions at +-infinity and g, g' continuous at interfaces.
// The solution is built from the generalised reflection coefficients Rh_j of
// the stack below each interface (bottom-up recursion) and the down-going
// amplitudes b_j at the top of each layer (top-down recursion); every
// exponential has a non-negative distance times i k_z with Im k_z > 0.
//
// One wavefront per (frequency, |k| class): the lanes evaluate the vertical
// wavenumbers of all layers in parallel, lane 0 runs the two O(L) recursions
// into LDS, and then the lanes sweep depth with coalesced z-contiguous stores.

#include "dev_common.h"

namespace edt {

template <bool WRITE32>
__global__ __launch_bounds__(256) void green_kernel(const double* __restrict__ freq,
                                                    const double* __restrict__ zif,
                                                    const double* __restrict__ cls_k,
                                                    const double* __restrict__ vel, int nf, int ncls,
                                                    int nz, int L, double eps, double z0, double dz,
                                                    zd* __restrict__ g64, float2* __restrict__ g32) {
    __shared__ zd s_k[4][kMaxLayers];
    __shared__ zd s_R[4][kMaxLayers];
    __shared__ zd s_b[4][kMaxLayers];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t wid = int64_t(blockIdx.x) * 4 + wv;
    const bool active = wid < int64_t(nf) * ncls;
    const int f = active ? int(wid / ncls) : 0;
    const int c = active ? int(wid % ncls) : 0;
    const double kk = cls_k[c];
    const zd w = omega_of(freq[f], eps);
    const zd w2 = w * w;
    if (lane < L) {
        const double cl = vel[lane];
        const zd q = zd{w2.x / (cl * cl) - kk * kk, w2.y / (cl * cl)};
        s_k[wv][lane] = zsqrt(q);
    }
    __syncthreads();
    if (lane == 0 && L > 1) {
        // bottom-up: Rh_j at interface j; rho_j = Rh_j exp(2 i k_j h_j) kept in s_b
        zd rho_next = zd{0.0, 0.0};   // rho of the bottom half space
        for (int j = L - 2; j >= 0; --j) {
            const zd kj = s_k[wv][j], kn = s_k[wv][j + 1];
            const zd r = zdiv(kj - kn, kj + kn);
            zd R = r;
            if (j < L - 2) R = zdiv(r + rho_next, zd{1.0, 0.0} + r * rho_next);
            s_R[wv][j] = R;
            if (j >= 1) {
                rho_next = R * zexpi(2.0 * kj, zif[j] - zif[j - 1]);
                s_b[wv][j] = rho_next;
            }
        }
        s_b[wv][L - 1] = zd{0.0, 0.0};
        // top-down: b_1 from the source layer, then b_{j+1} from b_j
        const zd k0 = s_k[wv][0];
        const zd half = zdiv(zd{0.0, 1.0}, 2.0 * k0);   // i / (2 k0)
        zd b = half * zexpi(k0, zif[0]) * zdiv(zd{1.0, 0.0} + s_R[wv][0],
                                               zd{1.0, 0.0} + s_b[wv][1]);
        s_b[wv][1] = b;
        for (int j = 1; j < L - 1; ++j) {
            const zd rho = s_b[wv][j + 1];
            b = b * zexpi(s_k[wv][j], zif[j] - zif[j - 1]) *
                zdiv(zd{1.0, 0.0} + s_R[wv][j], zd{1.0, 0.0} + rho);
            s_b[wv][j + 1] = b;
        }
    }
    __syncthreads();
    if (!active) return;
    const double sc32 = sqrt(zabs2(w) * dz);   // |w| sqrt(dz)
    const int64_t base = (int64_t(f) * ncls + c) * nz;
    for (int i = lane; i < nz; i += 64) {
        const double z = z0 + double(i) * dz;
        // layer index = number of interfaces at or above z
        int lo = 0, hi = L - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (zif[mid] <= z) lo = mid + 1;
            else hi = mid;
        }
        const int j = lo;
        const zd kj = s_k[wv][j];
        zd g;
        if (j == 0) {
            const zd half = zdiv(zd{0.0, 1.0}, 2.0 * kj);
            zd t = zexpi(kj, fabs(z));
            if (L > 1) t = t + s_R[wv][0] * zexpi(kj, 2.0 * zif[0] - z);
            g = half * t;
        } else if (j == L - 1) {
            g = s_b[wv][j] * zexpi(kj, z - zif[j - 1]);
        } else {
            const zd t = zexpi(kj, z - zif[j - 1]) +
                         s_R[wv][j] * zexpi(kj, 2.0 * zif[j] - zif[j - 1] - z);
            g = s_b[wv][j] * t;
        }
        g64[base + i] = g;
        if (WRITE32) g32[base + i] = make_float2(float(sc32 * g.x), float(sc32 * g.y));
    }
}

hipError_t launch_green(const edt_plan* p, const double* vel, zd* g64, float2* g32, hipStream_t st) {
    const int64_t waves = int64_t(p->n_freq) * p->n_cls;
    const int blocks = int((waves + 3) / 4);
    const double* freq = dptr<const double>(p, p->lay.freq);
    const double* zif = dptr<const double>(p, p->lay.zif);
    const double* clsk = dptr<const double>(p, p->lay.cls_k);
    if (g32)
        hipLaunchKernelGGL(green_kernel<true>, dim3(blocks), dim3(256), 0, st, freq, zif, clsk, vel,
                           p->n_freq, p->n_cls, p->nz, p->n_layers, p->eps, p->z0, p->dz, g64, g32);
    else
        hipLaunchKernelGGL(green_kernel<false>, dim3(blocks), dim3(256), 0, st, freq, zif, clsk, vel,
                           p->n_freq, p->n_cls, p->nz, p->n_layers, p->eps, p->z0, p->dz, g64, g32);
    return hipGetLastError();
}

}  // namespace edt
