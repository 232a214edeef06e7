// Kernel (c): damped normal equations per pair -- FP64 Cholesky, triangular
// solves, FP64 iterative refinement and the recombination into V~(+-k_m).
//
// Paper, Section 2.1 (eqs. VSym, Split) and Section 4 (Tikhonov damping as
// the regularisation to use on the small per-k_m systems):
//   (G + lambda I) x+- = c+-,  lambda = lambda_rel tr(G) / nz,
//   V~(k_m) = x+ + i x-,  V~(-k_m) = x+ - i x-.
// One workgroup per pair.  The factorisation is left-looking by 32-column
// panels: the panel is updated from the finished columns (staged through LDS
// in 32-column tiles) and then factored in LDS.  The factor L overwrites the
// lower triangle of the Gram in place.  The triangular solves work on
// 32-blocks: one wave solves the diagonal block with shuffles, the block
// updates the remaining right-hand sides.

#include "dev_linalg.h"

namespace edt {

// Factor gram[p] + lambda_p I in place and solve for x from rhs.
// Dynamic LDS: panel m x CBP, tile m x CBP (m <= nz), sx 2nz, sD, sred.
__global__ __launch_bounds__(256) void chol_solve_kernel(
    double* __restrict__ gram, const double* __restrict__ trace, const double* __restrict__ rhs,
    const int64_t* __restrict__ urow_off, const int32_t* __restrict__ pair_u, int nz,
    double lambda_rel, double* __restrict__ lam_out, double* __restrict__ x,
    int32_t* __restrict__ info, int32_t* __restrict__ conv, int32_t* __restrict__ steps) {
    extern __shared__ double smem[];
    double* sP = smem;
    double* sT = sP + size_t(nz) * CBP;
    double* sx = sT + size_t(nz) * CBP;
    double* sD = sx + 2 * nz;
    double* sred = sD + CB * CBP;
    __shared__ int s_bad;
    __shared__ double s_red[8];
    const int p = blockIdx.x, tid = threadIdx.x;
    double* A = gram + size_t(p) * nz * nz;
    const bool empty = urow_off[p + 1] == urow_off[p];
    const bool selfc = pair_u[2 * p] == pair_u[2 * p + 1];
    const double lam = lambda_rel * trace[p] / double(nz);
    if (tid == 0) {
        lam_out[p] = lam;
        s_bad = 0;
        if (steps) steps[p] = 0;
    }
    if (empty) {
        for (int e = tid; e < 2 * nz; e += blockDim.x) x[size_t(p) * 2 * nz + e] = 0.0;
        if (tid == 0) {
            info[p] = EDT_INFO_EMPTY;
            conv[p] = 1;
        }
        return;
    }
    for (int k0 = 0; k0 < nz; k0 += CB) {
        const int kb = min(CB, nz - k0), m = nz - k0;
        for (int e = tid; e < m * CB; e += blockDim.x) {
            const int i = e / CB, j = e % CB;
            double v = 0.0;
            if (j < kb && i >= j) {
                v = A[size_t(k0 + i) * nz + k0 + j];
                if (i == j) v += lam;
            }
            sP[i * CBP + j] = v;
        }
        __syncthreads();
        for (int t0 = 0; t0 < k0; t0 += CB) {
            for (int e = tid; e < m * CB; e += blockDim.x) {
                const int i = e / CB, t = e % CB;
                sT[i * CBP + t] = A[size_t(k0 + i) * nz + t0 + t];
            }
            __syncthreads();
            // P[i][j] -= sum_t T[i][t] T[j][t], 4 rows x 4 columns per thread
            const int nbi = (m + 3) / 4;
            for (int e = tid; e < nbi * (CB / 4); e += blockDim.x) {
                const int bi = e / (CB / 4), bj = e % (CB / 4);
                const int i0 = 4 * bi, j0 = 4 * bj;
                if (j0 >= kb || i0 + 3 < j0) continue;
                double s[4][4] = {};
                for (int t = 0; t < CB; ++t) {
                    double a[4], b[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        a[q] = (i0 + q < m) ? sT[(i0 + q) * CBP + t] : 0.0;
                        b[q] = sT[(j0 + q) * CBP + t];
                    }
#pragma unroll
                    for (int qi = 0; qi < 4; ++qi)
#pragma unroll
                        for (int qj = 0; qj < 4; ++qj) s[qi][qj] += a[qi] * b[qj];
                }
#pragma unroll
                for (int qi = 0; qi < 4; ++qi)
#pragma unroll
                    for (int qj = 0; qj < 4; ++qj) {
                        const int i = i0 + qi, j = j0 + qj;
                        if (i < m && j < kb && i >= j) sP[i * CBP + j] -= s[qi][qj];
                    }
            }
            __syncthreads();
        }
        // factor the m x kb panel (right-looking inside the panel)
        for (int j = 0; j < kb; ++j) {
            if (tid == 0) {
                double d = sP[j * CBP + j];
                if (!(d > 0.0) || !isfinite(d)) {
                    if (s_bad == 0) s_bad = k0 + j + 1;
                    d = 1.0;
                }
                sP[j * CBP + j] = sqrt(d);
            }
            __syncthreads();
            const double dj = sP[j * CBP + j];
            for (int i = j + 1 + tid; i < m; i += blockDim.x) sP[i * CBP + j] /= dj;
            __syncthreads();
            const int w = kb - j - 1;
            if (w > 0)
                for (int e = tid; e < (m - j - 1) * w; e += blockDim.x) {
                    const int i = j + 1 + e / w, jj = j + 1 + e % w;
                    if (i >= jj) sP[i * CBP + jj] -= sP[i * CBP + j] * sP[jj * CBP + j];
                }
            __syncthreads();
        }
        for (int e = tid; e < m * CB; e += blockDim.x) {
            const int i = e / CB, j = e % CB;
            if (j < kb && i >= j) A[size_t(k0 + i) * nz + k0 + j] = sP[i * CBP + j];
        }
        __syncthreads();
    }
    for (int e = tid; e < 2 * nz; e += blockDim.x) sx[e] = rhs[size_t(p) * 2 * nz + e];
    __syncthreads();
    trisolve2(A, nz, sx, sD, sred);
    for (int e = tid; e < 2 * nz; e += blockDim.x)
        x[size_t(p) * 2 * nz + e] = (selfc && e >= nz) ? 0.0 : sx[e];
    if (tid == 0) {
        info[p] = s_bad;
        conv[p] = 0;
    }
    (void)s_red;
}

// One refinement step for every unconverged pair:
//   r = (sum of the residual partials) - lambda x,  dx = (L L^T)^{-1} r,
//   x += dx, converged when ||dx|| <= tol ||x||.
__global__ __launch_bounds__(256) void refine_update_kernel(
    const double* __restrict__ gram, const double* __restrict__ rpart,
    const int32_t* __restrict__ pair_item, const int32_t* __restrict__ pair_u, int nz,
    const double* __restrict__ lam, double* __restrict__ x, int32_t* __restrict__ conv,
    int32_t* __restrict__ steps, double tol) {
    extern __shared__ double smem[];
    double* sx = smem;
    double* sD = sx + 2 * nz;
    double* sred = sD + CB * CBP;
    __shared__ double s_red[8];
    const int p = blockIdx.x, tid = threadIdx.x;
    if (conv[p]) return;
    const bool selfc = pair_u[2 * p] == pair_u[2 * p + 1];
    const int k0 = pair_item[p], k1 = pair_item[p + 1];
    const int w = 2 * nz + 1;
    double* xp = x + size_t(p) * 2 * nz;
    const double lp = lam[p];
    for (int e = tid; e < 2 * nz; e += blockDim.x) {
        double s = 0.0;
        for (int k = k0; k < k1; ++k) s += rpart[size_t(k) * w + e];
        sx[e] = (selfc && e >= nz) ? 0.0 : s - lp * xp[e];
    }
    __syncthreads();
    trisolve2(gram + size_t(p) * nz * nz, nz, sx, sD, sred);
    double dn = 0.0, xn = 0.0;
    for (int e = tid; e < 2 * nz; e += blockDim.x) {
        const double d = (selfc && e >= nz) ? 0.0 : sx[e];
        const double v = xp[e] + d;
        xp[e] = v;
        dn += d * d;
        xn += v * v;
    }
    dn = block_sum(dn, s_red);
    xn = block_sum(xn, s_red);
    if (tid == 0) {
        steps[p] += 1;
        if (dn <= tol * tol * xn) conv[p] = 1;
    }
}

// V~(u) = x+ + i x-, V~(-u) = x+ - i x-; info NOCONV / NONFINITE.
__global__ __launch_bounds__(256) void recombine_kernel(const double* __restrict__ x,
                                                        const int32_t* __restrict__ pair_u, int nz,
                                                        int refine, const int32_t* __restrict__ conv,
                                                        int32_t* __restrict__ info, zd* __restrict__ v) {
    __shared__ int s_nf;
    const int p = blockIdx.x, tid = threadIdx.x;
    const int u0 = pair_u[2 * p], u1 = pair_u[2 * p + 1];
    if (tid == 0) s_nf = 0;
    __syncthreads();
    for (int z = tid; z < nz; z += blockDim.x) {
        const double xp = x[size_t(p) * 2 * nz + z];
        const double xm = (u0 == u1) ? 0.0 : x[size_t(p) * 2 * nz + nz + z];
        if (!isfinite(xp) || !isfinite(xm)) s_nf = 1;
        v[size_t(u0) * nz + z] = zd{xp, xm};
        if (u1 != u0) v[size_t(u1) * nz + z] = zd{xp, -xm};
    }
    __syncthreads();
    if (tid == 0 && info[p] == EDT_INFO_OK) {
        if (s_nf) info[p] = EDT_INFO_NONFINITE;
        else if (refine && !conv[p]) info[p] = EDT_INFO_NOCONV;
    }
}

// ------------------------------------------------------------- launchers ---
// Allow the factorisation kernel the large dynamic LDS it needs (gfx950 has
// 160 KiB per CU).
hipError_t configure_kernels() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(chol_solve_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
}

size_t chol_lds_bytes(int nz) { return (size_t(2) * nz * CBP + 2 * nz + CB * CBP + 16 * CB) * sizeof(double); }
size_t refine_lds_bytes(int nz) { return (size_t(2) * nz + CB * CBP + 16 * CB) * sizeof(double); }

hipError_t launch_chol(const edt_plan* p, double* gram, const double* trace, const double* rhs,
                       double lambda_rel, double* lam, double* x, int32_t* info, int32_t* conv,
                       int32_t* steps, hipStream_t st) {
    if (p->n_pairs == 0) return hipSuccess;
    const size_t lds = chol_lds_bytes(p->nz);
    hipLaunchKernelGGL(chol_solve_kernel, dim3(unsigned(p->n_pairs)), dim3(256), lds, st, gram, trace,
                       rhs, dptr<const int64_t>(p, p->lay.urow_off), dptr<const int32_t>(p, p->lay.pair_u),
                       p->nz, lambda_rel, lam, x, info, conv, steps);
    return hipGetLastError();
}

hipError_t launch_refine_update(const edt_plan* p, const double* gram, const double* rpart,
                                const double* lam, double* x, int32_t* conv, int32_t* steps, double tol,
                                hipStream_t st) {
    if (p->n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(refine_update_kernel, dim3(unsigned(p->n_pairs)), dim3(256),
                       refine_lds_bytes(p->nz), st, gram, rpart, dptr<const int32_t>(p, p->lay.pair_item),
                       dptr<const int32_t>(p, p->lay.pair_u), p->nz, lam, x, conv, steps, tol);
    return hipGetLastError();
}

hipError_t launch_recombine(const edt_plan* p, const double* x, int refine, const int32_t* conv,
                            int32_t* info, zd* v, hipStream_t st) {
    if (p->n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(recombine_kernel, dim3(unsigned(p->n_pairs)), dim3(256), 0, st, x,
                       dptr<const int32_t>(p, p->lay.pair_u), p->nz, refine, conv, info, v);
    return hipGetLastError();
}

}  // namespace edt
