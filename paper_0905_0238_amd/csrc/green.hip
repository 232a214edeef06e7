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
// A block takes kGreenEntries (frequency, |k| class) entries: its threads
// evaluate the vertical wavenumbers of every (entry, layer) in parallel, one
// thread per entry runs the two O(L) recursions (sixteen recursions side by
// side in one wavefront), and then all threads sweep (entry, depth) with
// coalesced z-contiguous stores.  Interfaces and recursion state live in LDS.

#include "dev_common.h"

namespace edt {

constexpr int kGreenEntries = 16;

// Dynamic LDS (doubles) of green_kernel for L layers: interfaces (padded to an
// even count) and k_z, Rh, b of every entry.
static size_t green_lds_bytes(int L) {
    return (size_t((L + 1) & ~1) + size_t(3) * kGreenEntries * L * 2) * sizeof(double);
}

template <bool WRITE32>
__global__ __launch_bounds__(256) void green_kernel(const double* __restrict__ freq,
                                                    const double* __restrict__ zif,
                                                    const double* __restrict__ cls_k,
                                                    const double* __restrict__ vel, int nf, int ncls,
                                                    int nz, int L, double eps, double z0, double dz,
                                                    zd* __restrict__ g64, float2* __restrict__ g32) {
    extern __shared__ double gsm[];
    double* s_zif = gsm;
    zd* s_k = reinterpret_cast<zd*>(gsm + ((L + 1) & ~1));   // [entry][layer]
    zd* s_R = s_k + kGreenEntries * L;
    zd* s_b = s_R + kGreenEntries * L;
    __shared__ zd s_half[kGreenEntries];      // i / (2 k_0)
    __shared__ double s_sc[kGreenEntries];    // |w| sqrt(dz)
    const int tid = threadIdx.x;
    const int64_t n_ent = int64_t(nf) * ncls;
    const int64_t e0 = int64_t(blockIdx.x) * kGreenEntries;
    const int ne = int(min<int64_t>(kGreenEntries, n_ent - e0));
    for (int t = tid; t < L - 1; t += 256) s_zif[t] = zif[t];
    for (int t = tid; t < kGreenEntries * L; t += 256) {
        const int e = t / L, j = t - e * L;
        const int64_t id = e0 + min(e, ne - 1);
        const int f = int(id / ncls), c = int(id - int64_t(f) * ncls);
        const double kk = cls_k[c];
        const zd w = omega_of(freq[f], eps);
        const zd w2 = w * w;
        const double cl = vel[j];
        s_k[t] = zsqrt(zd{w2.x / (cl * cl) - kk * kk, w2.y / (cl * cl)});
    }
    __syncthreads();
    if (tid < kGreenEntries) {
        const int64_t id = e0 + min(tid, ne - 1);
        const zd w = omega_of(freq[int(id / ncls)], eps);
        const zd* k = s_k + tid * L;
        zd* R = s_R + tid * L;
        zd* b = s_b + tid * L;
        const zd half = zdiv(zd{0.0, 1.0}, 2.0 * k[0]);
        s_half[tid] = half;
        s_sc[tid] = sqrt(zabs2(w) * dz);
        if (L > 1) {
            // bottom-up: Rh_j at interface j; rho_j = Rh_j exp(2 i k_j h_j) kept in b
            zd rho_next = zd{0.0, 0.0};   // rho of the bottom half space
            for (int j = L - 2; j >= 0; --j) {
                const zd kj = k[j], kn = k[j + 1];
                const zd r = zdiv(kj - kn, kj + kn);
                zd Rj = r;
                if (j < L - 2) Rj = zdiv(r + rho_next, zd{1.0, 0.0} + r * rho_next);
                R[j] = Rj;
                if (j >= 1) {
                    rho_next = Rj * zexpi(2.0 * kj, s_zif[j] - s_zif[j - 1]);
                    b[j] = rho_next;
                }
            }
            b[L - 1] = zd{0.0, 0.0};
            // top-down: b_1 from the source layer, then b_{j+1} from b_j
            zd bb = half * zexpi(k[0], s_zif[0]) * zdiv(zd{1.0, 0.0} + R[0], zd{1.0, 0.0} + b[1]);
            b[1] = bb;
            for (int j = 1; j < L - 1; ++j) {
                const zd rho = b[j + 1];
                bb = bb * zexpi(k[j], s_zif[j] - s_zif[j - 1]) * zdiv(zd{1.0, 0.0} + R[j], zd{1.0, 0.0} + rho);
                b[j + 1] = bb;
            }
        }
    }
    __syncthreads();
    // Outputs: within layer j the function is u1 + u2 with u1 ~ exp(i k_j z)
    // and u2 ~ exp(-i k_j z) (u2 = 0 in the bottom half space).  Thread (e, c)
    // takes depths c, c + 16, ... of entry e: each term is evaluated directly
    // where a layer is entered and carried down by its factor exp(+-i k_j 16 dz)
    // otherwise (at most nz / 16 products, a relative error of a few units of
    // rounding), so consecutive threads still store consecutive depths.
    static_assert(kGreenEntries * 16 == 256, "16 threads per entry");
    const int e = tid >> 4, c = tid & 15;
    if (e < ne) {
        int lay = -1;
        bool have_f = false;
        zd u1{0.0, 0.0}, u2{0.0, 0.0}, f1{1.0, 0.0}, f2{1.0, 0.0};
        for (int i = c; i < nz; i += 16) {
            const double z = z0 + double(i) * dz;
            // layer index = number of interfaces at or above z
            int lo = 0, hi = L - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_zif[mid] <= z) lo = mid + 1;
                else hi = mid;
            }
            const int j = lo;
            if (j != lay || z < 0.0) {
                const zd kj = s_k[e * L + j];
                if (j == 0) {
                    u1 = s_half[e] * zexpi(kj, fabs(z));
                    u2 = L > 1 ? s_half[e] * (s_R[e * L] * zexpi(kj, 2.0 * s_zif[0] - z)) : zd{0.0, 0.0};
                } else if (j == L - 1) {
                    u1 = s_b[e * L + j] * zexpi(kj, z - s_zif[j - 1]);
                    u2 = zd{0.0, 0.0};
                } else {
                    u1 = s_b[e * L + j] * zexpi(kj, z - s_zif[j - 1]);
                    u2 = s_b[e * L + j] * (s_R[e * L + j] * zexpi(kj, 2.0 * s_zif[j] - s_zif[j - 1] - z));
                }
                lay = z < 0.0 ? -1 : j;   // above the source depth: evaluated directly
                have_f = false;
            } else {
                if (!have_f) {   // the layer's step factors, once it holds a second depth
                    const zd kj = s_k[e * L + j];
                    f1 = zexpi(kj, 16.0 * dz);
                    f2 = zexpi(kj, -16.0 * dz);
                    have_f = true;
                }
                u1 = u1 * f1;
                u2 = u2 * f2;
            }
            const zd g = u1 + u2;
            const size_t at = size_t(e0 + e) * nz + i;
            g64[at] = g;
            if (WRITE32) g32[at] = make_float2(float(s_sc[e] * g.x), float(s_sc[e] * g.y));
        }
    }
}

hipError_t launch_green(const edt_plan* p, const double* vel, zd* g64, float2* g32, hipStream_t st) {
    const int64_t n_ent = int64_t(p->n_freq) * p->n_cls;
    if (n_ent == 0) return hipSuccess;
    const unsigned blocks = unsigned((n_ent + kGreenEntries - 1) / kGreenEntries);
    const size_t lds = green_lds_bytes(p->n_layers);
    const double* freq = dptr<const double>(p, p->lay.freq);
    const double* zif = dptr<const double>(p, p->lay.zif);
    const double* clsk = dptr<const double>(p, p->lay.cls_k);
    if (g32)
        hipLaunchKernelGGL(green_kernel<true>, dim3(blocks), dim3(256), lds, st, freq, zif, clsk, vel,
                           p->n_freq, p->n_cls, p->nz, p->n_layers, p->eps, p->z0, p->dz, g64, g32);
    else
        hipLaunchKernelGGL(green_kernel<false>, dim3(blocks), dim3(256), lds, st, freq, zif, clsk, vel,
                           p->n_freq, p->n_cls, p->nz, p->n_layers, p->eps, p->z0, p->dz, g64, g32);
    return hipGetLastError();
}

}  // namespace edt
