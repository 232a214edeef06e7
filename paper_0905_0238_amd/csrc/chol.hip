// Kernel (c): damped normal equations per pair -- FP64 Cholesky, triangular
// solves, FP64 iterative refinement and the recombination into V~(+-k_m).
//
// Paper, Section 2.1 (eqs. VSym, Split) and Section 4 (Tikhonov damping as
// the regularisation to use on the small per-k_m systems):
//   (G + lambda I) x+- = c+-,  lambda = lambda_rel tr(G) / nz,
//   V~(k_m) = x+ + i x-,  V~(-k_m) = x+ - i x-.
// One workgroup per pair.  The factorisation is left-looking by 32-column
// panels:
//  * update: P -= L[k0:, :k0] L[k0:k0+32, :k0]^T on FP64 MFMA
//    (v_mfma_f64_16x16x4) with the panel in the accumulators; the finished
//    columns are staged in LDS 32 at a time;
//  * diagonal block: one wave factors it in registers (4 x 4 blocks per
//    lane) and, in the same pivot loop, forms D = L_kk^{-1} by forward
//    substitution on the identity;
//  * the rows below: L_ik = P_ik D^T, again on FP64 MFMA (no serial
//    triangular solve).
// L overwrites the lower triangle of the Gram in place; the block inverses
// D go to a workspace, where the block solves (block_solve2) use them.
// LDS stays under 80 KiB for nz <= 256, so two pairs share a CU.

#include "dev_linalg.h"

namespace edt {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Factor gram[p] + lambda_p I in place, store the diagonal-block inverses in
// dinv[p][nblk][32][32] and solve for x from rhs (exact: with the corrected
// block solves, for a result that no refinement follows).
// Dynamic LDS: the panel (nz x CBP doubles) and D (32 x CBP doubles), reused
// by the solve afterwards.
// Q: row-block groups of the panel accumulators (wave w holds the 16-row
// blocks w + 4 q, q < Q): 4 for nz <= 256, 7 for nz <= 448.
template <int Q>
__global__ __launch_bounds__(256, Q > 4 ? 1 : 2) void chol_solve_kernel(
    double* __restrict__ gram, const double* __restrict__ trace, const double* __restrict__ rhs,
    const int64_t* __restrict__ urow_off, const int32_t* __restrict__ pair_u, int nz,
    double lambda_rel, double* __restrict__ lam_out, double* __restrict__ dinv, double* __restrict__ x,
    int32_t* __restrict__ info, int32_t* __restrict__ conv, int32_t* __restrict__ steps, int only_failed,
    int exact, int32_t* __restrict__ n_failed) {
    extern __shared__ double smem[];
    double* sP = smem;
    double* sD = smem + size_t(nz) * CBP;
    __shared__ int s_bad;
    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (only_failed && info[p] <= 0) return;   // second pass: failed factorisations only
    const int nblk = (nz + CB - 1) / CB;
    double* A = gram + size_t(p) * nz * nz;
    double* Dp = dinv + size_t(p) * nblk * CB * CB;
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
    const int li = lane & 15, lk = lane >> 4;   // MFMA operand lane: (row, k)
    for (int k0 = 0; k0 < nz; k0 += CB) {
        const int kb = min(CB, nz - k0), m = nz - k0;
        const int nrb = (m + 15) >> 4;
        // accumulators: row blocks rb = wv + 4q (q < Q), column blocks 0..1;
        // v_mfma_f64_16x16x4 lane l, register v holds (row 4v + l/16, column l%16)
        f64x4 acc[Q][2];
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rb = wv + 4 * q;
                    const int i = 16 * rb + 4 * v + lk, j = 16 * cb + li;
                    double a = 0.0;
                    if (rb < nrb && i < m && j < kb && i >= j) {
                        a = A[size_t(k0 + i) * nz + k0 + j];
                        if (i == j) a += lam;
                    }
                    acc[q][cb][v] = a;
                }
        // P -= L[k0+i][t] L[k0+j][t], t < k0: 32 finished columns at a time
        for (int t0 = 0; t0 < k0; t0 += CB) {
            // the loads of a half chunk go out together (clamped rows), then
            // the stores: two memory round trips per chunk
            for (int h = 0; 128 * h < m; ++h) {
                const int c = tid & 31, r0 = (tid >> 5) + 128 * h;
                if (r0 < m) {
                    double v[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) v[u] = A[size_t(k0 + min(r0 + 8 * u, m - 1)) * nz + t0 + c];
#pragma unroll
                    for (int u = 0; u < 16; ++u)
                        if (r0 + 8 * u < m) sP[(r0 + 8 * u) * CBP + c] = v[u];
                }
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < CB; kk += 4) {
                const double b0 = (li < kb) ? sP[li * CBP + kk + lk] : 0.0;
                const double b1 = (16 + li < kb) ? sP[(16 + li) * CBP + kk + lk] : 0.0;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int rb = wv + 4 * q;
                    if (rb < nrb) {
                        const int i = 16 * rb + li;
                        const double a = (i < m) ? -sP[i * CBP + kk + lk] : 0.0;
                        acc[q][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc[q][0], 0, 0, 0);
                        acc[q][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc[q][1], 0, 0, 0);
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rb = wv + 4 * q;
                    const int i = 16 * rb + 4 * v + lk, j = 16 * cb + li;
                    if (rb < nrb && i < m) sP[i * CBP + j] = acc[q][cb][v];
                }
        __syncthreads();
        // Factor the kb x kb diagonal block in one wave and invert it.  Lane
        // (bi, bj) = (lane / 8, lane % 8) holds the 4 x 4 blocks of rows
        // 4 bi.., columns 4 bj.. of L (a) and of D = L^{-1} (dv).  Right-
        // looking, the pivot steps unrolled by four so that register indices
        // are static, with no branches (a partial block is padded with the
        // identity): at pivot k,
        // column k of L and row k of D are scaled by their owners and passed
        // to every lane by cross-lane permutes, then rows > k of both are
        // updated.
        if (tid < 64) {
            const int bi = tid >> 3, bj = tid & 7;
            const bool act = bi >= bj;
            double a[4][4], dv[4][4];
            int bad = 0;   // first failing column of this block (wave-uniform)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int i = 4 * bi + r, jj = 4 * bj + c;
                    a[r][c] = (act && i < kb && jj < kb && jj <= i) ? sP[i * CBP + jj] : (i == jj ? 1.0 : 0.0);
                    dv[r][c] = (i == jj) ? 1.0 : 0.0;
                }
            for (int kb4 = 0; kb4 < CB / 4; ++kb4)
#pragma unroll
            for (int kr = 0; kr < 4; ++kr) {
                const int k = 4 * kb4 + kr;
                double d = readlane_d(a[kr][kr], kb4 * 9);   // lane of diagonal block (kb4, kb4)
                const bool ok = d > 0.0 && isfinite(d);
                bad = (!ok && bad == 0 && k < kb) ? k0 + k + 1 : bad;
                d = ok ? d : 1.0;
                // 1/sqrt(d) from the hardware estimate and two Newton steps
                double inv = __builtin_amdgcn_rsq(d);
                const double hd = 0.5 * d;
                inv = inv * fma(-hd * inv, inv, 1.5);
                inv = inv * fma(-hd * inv, inv, 1.5);
                const double lkk = d * inv;
                // colz: L[i][k] below the pivot, zero at and above it, so the
                // rank-1 updates below need no masks (a zero factor leaves the
                // finished rows and columns unchanged)
                double colz[4], drow[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * bi + r;
                    const double v = a[r][kr] * inv;
                    colz[r] = (i > k) ? v : 0.0;
                    if (bj == kb4) a[r][kr] = (i > k) ? v : ((i == k) ? lkk : a[r][kr]);
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double v = dv[kr][c] * inv;   // D[k][4 bj + c], final
                    drow[c] = v;
                    if (bi == kb4) dv[kr][c] = v;
                }
                double ci[4], cj[4], dr[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    ci[q] = __shfl(colz[q], 8 * bi + kb4, 64);   // L[4 bi + q][k]
                    cj[q] = __shfl(colz[q], 8 * bj + kb4, 64);   // L[4 bj + q][k]
                    dr[q] = __shfl(drow[q], 8 * kb4 + bj, 64);  // D[k][4 bj + q]
                }
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        a[r][c] -= ci[r] * cj[c];
                        dv[r][c] -= ci[r] * dr[c];
                    }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int i = 4 * bi + r, jj = 4 * bj + c;
                    if (act && i < kb && jj <= i) sP[i * CBP + jj] = a[r][c];
                    sD[i * CBP + jj] = act ? dv[r][c] : 0.0;
                }
            if (tid == 0 && bad != 0 && s_bad == 0) s_bad = bad;
        }
        __syncthreads();
        // rows below the diagonal block: L_ik = P_ik D^T on MFMA (B[k][c] = D[c][k])
        if (m > kb) {
            f64x4 t[Q][2];
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) t[q][cb][v] = 0.0;
#pragma unroll
            for (int kk = 0; kk < CB; kk += 4) {
                const double b0 = sD[li * CBP + kk + lk];
                const double b1 = sD[(16 + li) * CBP + kk + lk];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int rb = wv + 4 * q;
                    if (rb >= 2 && rb < nrb) {
                        const int i = 16 * rb + li;
                        const double a = (i < m) ? sP[i * CBP + kk + lk] : 0.0;
                        t[q][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, t[q][0], 0, 0, 0);
                        t[q][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, t[q][1], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int rb = wv + 4 * q;
                        const int i = 16 * rb + 4 * v + lk, j = 16 * cb + li;
                        if (rb >= 2 && rb < nrb && i < m) A[size_t(k0 + i) * nz + k0 + j] = t[q][cb][v];
                    }
        }
        for (int e = tid; e < kb * CB; e += blockDim.x) {
            const int i = e / CB, j = e % CB;
            if (j <= i) A[size_t(k0 + i) * nz + k0 + j] = sP[i * CBP + j];
        }
        for (int e = tid; e < CB * CB; e += blockDim.x)
            Dp[size_t(k0 / CB) * CB * CB + e] = sD[(e >> 5) * CBP + (e & 31)];
        __syncthreads();
    }
    // block solves (LDS reused)
    double* sx = smem;
    double* sred = sx + 2 * nz;
    double* sDs = sred + kSolveRed;
    double* sLs = sDs + CB * CBP;
    for (int e = tid; e < 2 * nz; e += blockDim.x) sx[e] = rhs[size_t(p) * 2 * nz + e];
    __syncthreads();
    if (exact) block_solve2<true>(A, Dp, nz, sx, sred, sDs, sLs);
    else block_solve2<false>(A, Dp, nz, sx, sred, sDs, sLs);
    for (int e = tid; e < 2 * nz; e += blockDim.x)
        x[size_t(p) * 2 * nz + e] = (selfc && e >= nz) ? 0.0 : sx[e];
    if (tid == 0) {
        info[p] = s_bad;
        conv[p] = 0;
        if (s_bad != 0 && n_failed) atomicAdd(n_failed, 1);
    }
}

// Refinement of x against the exact FP64 operator M = Re(A^H A) + lambda I
// (applied from the Born rows by resid_kernel), preconditioned by the
// factorisation L L^T of the assembled Gram (FP64 or mixed): conjugate
// gradients on M x = c, one operator sweep per iteration, ending with a plain
// correction step once it is small:
//   z = (L L^T)^{-1} r;  if ||z|| <= tol ||x + z||: x += z, converged;
//   else p = z + beta p (beta = (r.z)/(r.z)_prev, 0 first), next sweep q = M p,
//        alpha = (r.z)/(p.q), x += alpha p, r -= alpha q.
// With an accurate factorisation alpha ~ 1 and this costs the sweeps of plain
// iterative refinement (x += z per sweep); where the mixed-precision Gram is
// too far from M for that to contract (cond(M) times its relative error near
// or above 1), the Krylov steps still converge.
//   first: rpart holds c - Re(A^H A) x (swept with the data): r = it - lambda x;
//   else:  rpart holds -Re(A^H A) p: q = lambda p - it.
// conv: 0 running, 1 converged, -1 stopped (p.q <= 0 or not finite).
// next_active counts the pairs that need the next sweep.
__global__ __launch_bounds__(256) void pcg_update_kernel(
    const double* __restrict__ gram, const double* __restrict__ dinv, const double* __restrict__ rpart,
    const int32_t* __restrict__ pair_item, const int32_t* __restrict__ pair_u, int nz,
    const double* __restrict__ lam, double* __restrict__ x, double* __restrict__ r, double* __restrict__ pv,
    double* __restrict__ rho, int32_t* __restrict__ conv, int32_t* __restrict__ steps, double tol, int first,
    int32_t* __restrict__ next_active) {
    extern __shared__ double smem[];
    double* sx = smem;
    double* sq = sx + 2 * nz;
    double* sred = sq + 2 * nz;
    double* sD = sred + kSolveRed;
    double* sL = sD + CB * CBP;
    __shared__ double s_red[8];
    const int p = blockIdx.x, tid = threadIdx.x;
    if (conv[p]) return;
    const bool selfc = pair_u[2 * p] == pair_u[2 * p + 1];
    const int k0 = pair_item[p], k1 = pair_item[p + 1];
    const int w = 2 * nz + 1;
    const int nblk = (nz + CB - 1) / CB;
    double* xp = x + size_t(p) * 2 * nz;
    double* rp = r + size_t(p) * 2 * nz;
    double* pp = pv + size_t(p) * 2 * nz;
    const double lp = lam[p];
    // sum of the item partials: eight independent partial sums keep eight
    // loads in flight; the combination order is fixed (deterministic)
    double pq = 0.0;
    for (int e = tid; e < 2 * nz; e += blockDim.x) {
        double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int k = k0;
        for (; k + 8 <= k1; k += 8)
#pragma unroll
            for (int q = 0; q < 8; ++q) s8[q] += rpart[size_t(k + q) * w + e];
        for (int q = 0; k < k1; ++k, ++q) s8[q] += rpart[size_t(k) * w + e];
        const double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
        const bool zero = selfc && e >= nz;
        if (first) {
            sx[e] = zero ? 0.0 : s - lp * xp[e];
        } else {
            const double q = zero ? 0.0 : lp * pp[e] - s;
            sq[e] = q;
            pq += pp[e] * q;
        }
    }
    if (!first) {
        pq = block_sum(pq, s_red);
        const double alpha = rho[p] / pq;
        if (!(pq > 0.0) || !isfinite(alpha)) {
            if (tid == 0) {
                conv[p] = -1;
                steps[p] += 1;
            }
            return;
        }
        for (int e = tid; e < 2 * nz; e += blockDim.x) {
            xp[e] += alpha * pp[e];
            sx[e] = rp[e] - alpha * sq[e];
        }
    }
    __syncthreads();
    for (int e = tid; e < 2 * nz; e += blockDim.x) rp[e] = sx[e];
    block_solve2<false>(gram + size_t(p) * nz * nz, dinv + size_t(p) * nblk * CB * CB, nz, sx, sred, sD, sL);
    double dn = 0.0, xn = 0.0, rz = 0.0;
    for (int e = tid; e < 2 * nz; e += blockDim.x) {
        const double z = (selfc && e >= nz) ? 0.0 : sx[e];
        sx[e] = z;
        const double v = xp[e] + z;
        dn += z * z;
        xn += v * v;
        rz += rp[e] * z;
    }
    dn = block_sum(dn, s_red);
    xn = block_sum(xn, s_red);
    rz = block_sum(rz, s_red);
    const bool done = dn <= tol * tol * xn;
    const double beta = first ? 0.0 : rz / rho[p];
    for (int e = tid; e < 2 * nz; e += blockDim.x) {
        if (done) xp[e] += sx[e];
        else pp[e] = sx[e] + beta * (first ? 0.0 : pp[e]);
    }
    __syncthreads();
    if (tid == 0) {
        steps[p] += 1;
        if (done) {
            conv[p] = 1;
        } else {
            rho[p] = rz;
            atomicAdd(next_active, 1);   // this pair needs the next sweep
        }
    }
}

// Counters of one solve: active[0] = 1 (every pair takes the first sweep),
// active[1..] = 0 (pairs still iterating before each later sweep, counted by
// pcg_update_kernel), and the failed-factorisation count.
__global__ void reset_counters_kernel(int32_t* __restrict__ c, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = i == 0 ? 1 : 0;
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
        else if (refine && conv[p] != 1) info[p] = EDT_INFO_NOCONV;
    }
}

// ------------------------------------------------------------- launchers ---
size_t pcg_lds_bytes(int nz) { return (block_solve_lds_doubles(nz) + 2 * size_t(nz)) * sizeof(double); }
size_t chol_lds_bytes(int nz) {
    const size_t panel = (size_t(nz) + CB) * CBP * sizeof(double);
    const size_t solve = block_solve_lds_doubles(nz) * sizeof(double);
    return panel > solve ? panel : solve;
}
// adjoint solves still use trisolve2 (staged panels in LDS)
size_t adjoint_lds_bytes(int nz) { return trisolve_lds_doubles(nz) * sizeof(double); }

// Allow the factorisation kernel more than 64 KiB of dynamic LDS (gfx950 has
// 160 KiB per CU).
hipError_t configure_adjoint_kernels(int bytes);
hipError_t configure_gram_kernels();
hipError_t configure_lines();
hipError_t configure_aperture();
// The largest dynamic LDS any supported depth count needs.
static int max_dynamic_lds() {
    const size_t a = chol_lds_bytes(kMaxDepth), b = adjoint_lds_bytes(kMaxAdjointDepth);
    return int(a > b ? a : b);
}
hipError_t configure_kernels() {
    const int bytes = max_dynamic_lds();
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(chol_solve_kernel<4>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(chol_solve_kernel<7>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(pcg_update_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) e = configure_adjoint_kernels(bytes);
    if (e == hipSuccess) e = configure_gram_kernels();
    if (e == hipSuccess) e = configure_lines();
    if (e == hipSuccess) e = configure_aperture();
    return e;
}

hipError_t launch_chol(const edt_plan* p, double* gram, const double* trace, const double* rhs,
                       double lambda_rel, double* lam, double* dinv, double* x, int32_t* info,
                       int32_t* conv, int32_t* steps, hipStream_t st, int only_failed, int exact,
                       int32_t* n_failed) {
    if (p->n_pairs == 0) return hipSuccess;
    const size_t lds = chol_lds_bytes(p->nz);
    if (p->nz <= 256)
        hipLaunchKernelGGL(chol_solve_kernel<4>, dim3(unsigned(p->n_pairs)), dim3(256), lds, st, gram, trace,
                           rhs, dptr<const int64_t>(p, p->lay.urow_off), dptr<const int32_t>(p, p->lay.pair_u),
                           p->nz, lambda_rel, lam, dinv, x, info, conv, steps, only_failed, exact, n_failed);
    else
        hipLaunchKernelGGL(chol_solve_kernel<7>, dim3(unsigned(p->n_pairs)), dim3(256), lds, st, gram, trace,
                           rhs, dptr<const int64_t>(p, p->lay.urow_off), dptr<const int32_t>(p, p->lay.pair_u),
                           p->nz, lambda_rel, lam, dinv, x, info, conv, steps, only_failed, exact, n_failed);
    return hipGetLastError();
}

hipError_t launch_pcg_update(const edt_plan* p, const double* gram, const double* dinv, const double* rpart,
                             const double* lam, double* x, double* r, double* pv, double* rho, int32_t* conv,
                             int32_t* steps, double tol, int first, int32_t* next_active, hipStream_t st) {
    if (p->n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(pcg_update_kernel, dim3(unsigned(p->n_pairs)), dim3(256), pcg_lds_bytes(p->nz), st, gram,
                       dinv, rpart, dptr<const int32_t>(p, p->lay.pair_ritem), dptr<const int32_t>(p, p->lay.pair_u),
                       p->nz, lam, x, r, pv, rho, conv, steps, tol, first, next_active);
    return hipGetLastError();
}

hipError_t launch_reset_counters(int32_t* c, int n, hipStream_t st) {
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, c, n);
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
