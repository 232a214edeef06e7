// Device linear-algebra helpers shared by the solve and adjoint kernels.
#pragma once

#include "dev_common.h"

namespace edt {

constexpr int CB = 32;        // panel / solve block width
constexpr int CBP = CB + 1;   // padded LDS row

// Solve L L^T x = r for the two right-hand sides held in sx[0..nz), sx[nz..2nz)
// (LDS); the result overwrites sx.  L: lower triangle of an nz x nz row-major
// matrix in global memory.  Each 32-column block of L is first staged in LDS
// with coalesced loads (sL: nz*CBP doubles), so the serial parts never wait
// on global memory; one wave solves the diagonal block (lanes 0-31 carry the
// first right-hand side, 32-63 the second; the pivot chain uses readlane).
// sred: 16*CB doubles.  blockDim.x must be 256.
__device__ __forceinline__ void trisolve2(const double* __restrict__ L, int nz, double* sx, double* sL,
                                          double* sred) {
    const int tid = threadIdx.x;
    const int nblk = (nz + CB - 1) / CB;
    auto stage = [&](int k0, int kb) {
        const int m = nz - k0;
        for (int e = tid; e < m * CB; e += blockDim.x) {
            const int i = e / CB, j = e % CB;
            sL[i * CBP + j] = (j < kb && (i >= kb || j <= i)) ? L[size_t(k0 + i) * nz + k0 + j] : 0.0;
        }
        __syncthreads();
        if (tid < kb) sL[tid * CBP + CB] = 1.0 / sL[tid * CBP + tid];   // reciprocal pivots
        __syncthreads();
    };
    // forward: L y = r
    for (int b = 0; b < nblk; ++b) {
        const int k0 = b * CB, kb = min(CB, nz - k0), m = nz - k0;
        stage(k0, kb);
        if (tid < 64) {
            const int h = tid >> 5, i = tid & 31;
            double v = (i < kb) ? sx[h * nz + k0 + i] : 0.0;
            for (int j = 0; j < kb; ++j) {
                const double rj = sL[j * CBP + CB];
                const double y0 = readlane_d(v, j) * rj, y1 = readlane_d(v, 32 + j) * rj;
                const double yj = h ? y1 : y0;
                if (i == j) v = yj;
                else if (i > j) v -= sL[i * CBP + j] * yj;
            }
            if (i < kb) sx[h * nz + k0 + i] = v;
        }
        __syncthreads();
        for (int i = kb + tid; i < m; i += blockDim.x) {
            double s0 = 0.0, s1 = 0.0;
            for (int j = 0; j < kb; ++j) {
                const double l = sL[i * CBP + j];
                s0 += l * sx[k0 + j];
                s1 += l * sx[nz + k0 + j];
            }
            sx[k0 + i] -= s0;
            sx[nz + k0 + i] -= s1;
        }
        __syncthreads();
    }
    // backward: L^T x = y
    for (int b = nblk - 1; b >= 0; --b) {
        const int k0 = b * CB, kb = min(CB, nz - k0), m = nz - k0;
        stage(k0, kb);
        {
            const int j = tid & 31, g = tid >> 5;   // 8 groups of 32
            double s0 = 0.0, s1 = 0.0;
            if (j < kb)
                for (int i = kb + g; i < m; i += 8) {
                    const double l = sL[i * CBP + j];
                    s0 += l * sx[k0 + i];
                    s1 += l * sx[nz + k0 + i];
                }
            sred[(g * 2 + 0) * CB + j] = s0;
            sred[(g * 2 + 1) * CB + j] = s1;
        }
        __syncthreads();
        if (tid < 64) {
            const int h = tid >> 5, i = tid & 31;
            double t = 0.0;
            for (int g = 0; g < 8; ++g) t += sred[(g * 2 + h) * CB + i];
            double v = (i < kb) ? sx[h * nz + k0 + i] - t : 0.0;
            for (int jj = kb - 1; jj >= 0; --jj) {
                const double rj = sL[jj * CBP + CB];
                const double x0 = readlane_d(v, jj) * rj, x1 = readlane_d(v, 32 + jj) * rj;
                const double xj = h ? x1 : x0;
                if (i == jj) v = xj;
                else if (i < jj) v -= sL[jj * CBP + i] * xj;
            }
            if (i < kb) sx[h * nz + k0 + i] = v;
        }
        __syncthreads();
    }
}

// LDS doubles needed by trisolve2 for depth count nz (sx, sL, sred).
__host__ __device__ constexpr size_t trisolve_lds_doubles(int nz) {
    return size_t(2) * nz + size_t(nz) * CBP + 16 * CB;
}

__device__ __forceinline__ double block_sum(double v, double* sbuf) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sbuf[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) t += sbuf[w];
    return t;
}

}  // namespace edt
