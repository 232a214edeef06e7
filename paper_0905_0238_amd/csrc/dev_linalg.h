// Device linear-algebra helpers shared by the solve and adjoint kernels.
#pragma once

#include "dev_common.h"

namespace edt {

constexpr int CB = 32;        // panel / solve block width
constexpr int CBP = CB + 1;   // padded LDS row

// Solve L L^T x = r for the two right-hand sides held in sx[0..nz), sx[nz..2nz)
// (LDS); the result overwrites sx.  L: lower triangle of an nz x nz row-major
// matrix in global memory.  sD: LDS CB*CBP; sred: LDS 8*2*CB.  All threads.
__device__ __noinline__ void trisolve2(const double* __restrict__ L, int nz, double* sx, double* sD, double* sred) {
    const int tid = threadIdx.x;
    // forward: L y = r
    for (int k0 = 0; k0 < nz; k0 += CB) {
        const int kb = min(CB, nz - k0);
        for (int e = tid; e < CB * CB; e += blockDim.x) {
            const int i = e / CB, j = e % CB;
            sD[i * CBP + j] = (i < kb && j <= i) ? L[size_t(k0 + i) * nz + k0 + j] : 0.0;
        }
        __syncthreads();
        if (tid < 64) {
            const int h = tid >> 5, i = tid & 31;
            double v = (i < kb) ? sx[h * nz + k0 + i] : 0.0;
            for (int j = 0; j < kb; ++j) {
                const double yj = __shfl(v, h * 32 + j, 64) / sD[j * CBP + j];
                if (i == j) v = yj;
                else if (i > j) v -= sD[i * CBP + j] * yj;
            }
            if (i < kb) sx[h * nz + k0 + i] = v;
        }
        __syncthreads();
        for (int i = k0 + kb + tid; i < nz; i += blockDim.x) {
            const double* row = L + size_t(i) * nz + k0;
            double s0 = 0.0, s1 = 0.0;
            for (int j = 0; j < kb; ++j) {
                const double l = row[j];
                s0 += l * sx[k0 + j];
                s1 += l * sx[nz + k0 + j];
            }
            sx[i] -= s0;
            sx[nz + i] -= s1;
        }
        __syncthreads();
    }
    // backward: L^T x = y
    const int nblk = (nz + CB - 1) / CB;
    for (int b = nblk - 1; b >= 0; --b) {
        const int k0 = b * CB, kb = min(CB, nz - k0);
        {
            const int j = tid & 31, g = tid >> 5;   // 8 groups of 32 (blockDim 256)
            double s0 = 0.0, s1 = 0.0;
            if (j < kb)
                for (int i = k0 + kb + g; i < nz; i += 8) {
                    const double l = L[size_t(i) * nz + k0 + j];
                    s0 += l * sx[i];
                    s1 += l * sx[nz + i];
                }
            sred[(g * 2 + 0) * CB + j] = s0;
            sred[(g * 2 + 1) * CB + j] = s1;
        }
        for (int e = tid; e < CB * CB; e += blockDim.x) {
            const int i = e / CB, j = e % CB;
            sD[i * CBP + j] = (i < kb && j <= i) ? L[size_t(k0 + i) * nz + k0 + j] : 0.0;
        }
        __syncthreads();
        if (tid < 64) {
            const int h = tid >> 5, i = tid & 31;
            double t = 0.0;
            for (int g = 0; g < 8; ++g) t += sred[(g * 2 + h) * CB + i];
            double v = (i < kb) ? sx[h * nz + k0 + i] - t : 0.0;
            for (int jj = kb - 1; jj >= 0; --jj) {
                const double xj = __shfl(v, h * 32 + jj, 64) / sD[jj * CBP + jj];
                if (i == jj) v = xj;
                else if (i < jj) v -= sD[jj * CBP + i] * xj;
            }
            if (i < kb) sx[h * nz + k0 + i] = v;
        }
        __syncthreads();
    }
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
