// Device linear-algebra helpers shared by the solve and adjoint kernels.
#pragma once

#include "dev_common.h"

namespace edt {

constexpr int CB = 32;        // panel / solve block width
// Off-diagonal part of a block row (or column) of L is read in chunks of
// kPanelGroups groups of 8 (one chunk covers nz <= 256).
constexpr int kPanelGroups = 28;
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

// Sum over the 8 lanes l ^ {1, 2, 4} of a group of 8 (every lane gets it).
__device__ __forceinline__ double sum8(double v) {
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    return v;
}

// Reduction scratch of block_solve2 (doubles).
constexpr int kSolveRed = 704;

// Solve L L^T x = r for the two right-hand sides in sx[0..nz), sx[nz..2nz)
// (LDS), in place, by block substitution with explicit inverses of the 32 x 32
// diagonal blocks of L:
//   forward   t_b = r_b - sum_{j<b} L_bj y_j,      y_b = D_b t_b,
//   backward  t_b = y_b - sum_{j>b} L_jb^T x_j,    x_b = D_b^T t_b,
// with CORR each block result followed by one correction with the block
// itself, y_b += D_b (t_b - L_bb y_b) (and the transposed form backward):
// applying an explicit inverse loses a factor up to cond(L_bb) against
// substitution, the correction restores substitution-level accuracy.  Without
// CORR (a preconditioner inside an iteration) the correction is skipped.
// L: lower triangle of a row-major nz x nz matrix (global); D: [nblk][32][32]
// row-major lower-triangular inverses (global).  No step has a serial chain
// longer than one block: 2 nblk dependent block steps.  None of the loads
// depends on the right-hand side, so the next block's D_b, L_bb and first
// panel chunk are requested while the current block is finished, and a block
// step waits on global memory only when that latency exceeds its own work.
// LDS: sred >= kSolveRed doubles, sD and sL >= 32 * CBP doubles each.
// blockDim.x must be 256.
template <bool CORR>
__device__ __forceinline__ void block_solve2(const double* __restrict__ L, const double* __restrict__ D,
                                             int nz, double* sx, double* sred, double* sD, double* sL) {
    const int tid = threadIdx.x;
    const int nblk = (nz + CB - 1) / CB;
    constexpr int PC = 8 * kPanelGroups;   // panel rows (columns) per chunk
    // the next block's D_b and L_bb (4 elements per thread) and its first
    // panel chunk, in flight
    double nd[4], nl[4], nv[kPanelGroups];
    auto fetch_diag = [&](int b) {
        const int k0 = b * CB, kb = min(CB, nz - k0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q, i = e >> 5, j = e & 31;
            nd[q] = D[size_t(b) * CB * CB + e];
            if constexpr (CORR) nl[q] = L[size_t(k0 + min(i, kb - 1)) * nz + k0 + min(j, kb - 1)];
        }
    };
    // D_b and the lower triangle of L_bb (zero elsewhere: the upper part of
    // the matrix is not part of L)
    auto put_diag = [&](int b) {
        const int k0 = b * CB, kb = min(CB, nz - k0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q, i = e >> 5, j = e & 31;
            sD[i * CBP + j] = nd[q];
            if constexpr (CORR) sL[i * CBP + j] = (i < kb && j <= i) ? nl[q] : 0.0;
        }
    };
    // forward: row i = tid / 8 of block b, columns c0 + tid % 8 + 8 u (< k0)
    auto fetch_row = [&](double (&v)[kPanelGroups], int b, int c0) {
        const int k0 = b * CB, kb = min(CB, nz - k0);
        const double* row = L + size_t(k0 + min(tid >> 3, kb - 1)) * nz;
        const int cmax = max(k0 - 1, 0);
#pragma unroll
        for (int u = 0; u < kPanelGroups; ++u) v[u] = row[min(c0 + (tid & 7) + 8 * u, cmax)];
    };
    // backward: column c = tid % 32 of block b, rows r0 + tid / 32 + 8 u (< nz)
    auto fetch_col = [&](double (&v)[kPanelGroups], int b, int r0) {
        const int k0 = b * CB, kb = min(CB, nz - k0);
        const int col = k0 + min(tid & 31, kb - 1);
#pragma unroll
        for (int u = 0; u < kPanelGroups; ++u) v[u] = L[size_t(min(r0 + (tid >> 5) + 8 * u, nz - 1)) * nz + col];
    };
    fetch_diag(0);
    fetch_row(nv, 0, 0);
    for (int b = 0; b < nblk; ++b) {
        const int k0 = b * CB, kb = min(CB, nz - k0);
        const int i = tid >> 3, part = tid & 7;   // row i of the block, 8 threads per row
        put_diag(b);
        double s0 = 0.0, s1 = 0.0;
        auto row_dot = [&](const double (&v)[kPanelGroups], int c0) {
#pragma unroll
            for (int u = 0; u < kPanelGroups; ++u) {
                const int c = c0 + part + 8 * u;
                const double l = (c < k0 && i < kb) ? v[u] : 0.0;
                const int cc = min(c, max(k0 - 1, 0));
                s0 += l * sx[cc];
                s1 += l * sx[nz + cc];
            }
        };
        row_dot(nv, 0);
        for (int c0 = PC; c0 < k0; c0 += PC) {   // nz > PC + CB only
            double lv[kPanelGroups];
            fetch_row(lv, b, c0);
            row_dot(lv, c0);
        }
        // the next block step's loads (the first backward block after the last)
        if (b + 1 < nblk) {
            fetch_diag(b + 1);
            fetch_row(nv, b + 1, 0);
        } else {
            fetch_diag(b);
            fetch_col(nv, b, k0 + CB);
        }
        s0 = sum8(s0);
        s1 = sum8(s1);
        const double t0 = i < kb ? sx[k0 + i] - s0 : 0.0;
        const double t1 = i < kb ? sx[nz + k0 + i] - s1 : 0.0;
        if (part == 0) {
            sred[i] = t0;
            sred[CB + i] = t1;
        }
        __syncthreads();
        // y = D t   (rows past kb: D and L are zero there, y = 0)
        double y0 = 0.0, y1 = 0.0;
        for (int j = part; j <= i; j += 8) {
            const double d = sD[i * CBP + j];
            y0 += d * sred[j];
            y1 += d * sred[CB + j];
        }
        y0 = sum8(y0);
        y1 = sum8(y1);
        if constexpr (!CORR) {
            if (part == 0 && i < kb) {
                sx[k0 + i] = y0;
                sx[nz + k0 + i] = y1;
            }
            __syncthreads();
            continue;
        }
        if (part == 0) {
            sred[64 + i] = y0;
            sred[96 + i] = y1;
        }
        __syncthreads();
        // e = t - L_bb y
        double r0 = 0.0, r1 = 0.0;
        for (int j = part; j <= i; j += 8) {
            const double l = sL[i * CBP + j];
            r0 += l * sred[64 + j];
            r1 += l * sred[96 + j];
        }
        r0 = sum8(r0);
        r1 = sum8(r1);
        if (part == 0) {
            sred[128 + i] = t0 - r0;
            sred[160 + i] = t1 - r1;
        }
        __syncthreads();
        // y += D e
        double c0 = 0.0, c1 = 0.0;
        for (int j = part; j <= i; j += 8) {
            const double d = sD[i * CBP + j];
            c0 += d * sred[128 + j];
            c1 += d * sred[160 + j];
        }
        c0 = sum8(c0);
        c1 = sum8(c1);
        if (part == 0 && i < kb) {
            sx[k0 + i] = y0 + c0;
            sx[nz + k0 + i] = y1 + c1;
        }
        __syncthreads();
    }
    for (int b = nblk - 1; b >= 0; --b) {
        const int k0 = b * CB, kb = min(CB, nz - k0);
        put_diag(b);
        {
            const int c = tid & 31, g = tid >> 5;   // column c of the block, 8 row groups
            double s0 = 0.0, s1 = 0.0;
            // rows k0 + CB + g + 8 u below the block, a chunk at a time
            auto col_dot = [&](const double (&v)[kPanelGroups], int r0) {
#pragma unroll
                for (int u = 0; u < kPanelGroups; ++u) {
                    const int m = r0 + g + 8 * u;
                    const double l = (m < nz && c < kb) ? v[u] : 0.0;
                    const int mm = min(m, nz - 1);
                    s0 += l * sx[mm];
                    s1 += l * sx[nz + mm];
                }
            };
            col_dot(nv, k0 + CB);
            for (int r0 = k0 + CB + PC; r0 < nz; r0 += PC) {
                double lv[kPanelGroups];
                fetch_col(lv, b, r0);
                col_dot(lv, r0);
            }
            sred[g * 64 + c] = s0;
            sred[g * 64 + CB + c] = s1;
        }
        if (b > 0) {
            fetch_diag(b - 1);
            fetch_col(nv, b - 1, k0);   // rows below block b - 1 start at its k0 + CB = k0
        }
        __syncthreads();
        if (tid < 64) {
            const int h = tid >> 5, c = tid & 31;
            double t = 0.0;
            for (int g = 0; g < 8; ++g) t += sred[g * 64 + h * CB + c];
            sred[512 + h * CB + c] = c < kb ? sx[h * nz + k0 + c] - t : 0.0;
        }
        __syncthreads();
        const int c = tid >> 3, part = tid & 7;   // column c, 8 threads per column
        // x = D^T t:  x_c = sum_{j >= c} D[j][c] t_j
        double x0 = 0.0, x1 = 0.0;
        for (int j = c + part; j < CB; j += 8) {
            const double d = sD[j * CBP + c];
            x0 += d * sred[512 + j];
            x1 += d * sred[512 + CB + j];
        }
        x0 = sum8(x0);
        x1 = sum8(x1);
        if constexpr (!CORR) {
            if (part == 0 && c < kb) {
                sx[k0 + c] = x0;
                sx[nz + k0 + c] = x1;
            }
            __syncthreads();
            continue;
        }
        if (part == 0) {
            sred[576 + c] = x0;
            sred[608 + c] = x1;
        }
        __syncthreads();
        // e = t - L_bb^T x
        double r0 = 0.0, r1 = 0.0;
        for (int j = c + part; j < CB; j += 8) {
            const double l = sL[j * CBP + c];
            r0 += l * sred[576 + j];
            r1 += l * sred[608 + j];
        }
        r0 = sum8(r0);
        r1 = sum8(r1);
        if (part == 0) {
            sred[640 + c] = sred[512 + c] - r0;
            sred[672 + c] = sred[512 + CB + c] - r1;
        }
        __syncthreads();
        // x += D^T e
        double c0 = 0.0, c1 = 0.0;
        for (int j = c + part; j < CB; j += 8) {
            const double d = sD[j * CBP + c];
            c0 += d * sred[640 + j];
            c1 += d * sred[672 + j];
        }
        c0 = sum8(c0);
        c1 = sum8(c1);
        if (part == 0 && c < kb) {
            sx[k0 + c] = x0 + c0;
            sx[nz + k0 + c] = x1 + c1;
        }
        __syncthreads();
    }
}

// LDS doubles needed by block_solve2 for depth count nz (sx, sred, sD, sL).
__host__ __device__ constexpr size_t block_solve_lds_doubles(int nz) {
    return size_t(2) * nz + kSolveRed + 2 * size_t(CB) * CBP;
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
