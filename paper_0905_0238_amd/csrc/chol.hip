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

// Staging of finished columns for the panel update (even depth counts).  A
// 16-column block of the rows k0 .. k0 + m - 1 (padded to rows64, a multiple
// of 64) takes rows64 x 128 bytes, piece-major: the 16-byte piece p (columns
// 2p, 2p + 1) of row r sits at slot p * rows64 + r, so the 16 rows an MFMA
// operand reads at one column are 256 contiguous bytes (no bank conflict) and
// a lane's address is a fixed offset plus a wave-uniform one.  Loads go
// straight to LDS (global_load_lds_dwordx4: lane l of a wave writes the 16
// bytes at the wave's base + 16 l): one wave instruction moves one piece of
// 64 consecutive rows.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void glb_void_t;

// Pieces of 16 bytes the panel region holds (the dynamic LDS before D).
__device__ __forceinline__ int stage_pieces(int nz) { return (nz * CBP * 8) / 16; }

__device__ __forceinline__ void stage_columns(const double* __restrict__ A, int nz, int k0, int m, int c0, int nb,
                                              int rows64, double* smem, int wvu, int lane) {
    const int per_piece = rows64 >> 6;         // wave instructions per piece
    const int total = nb * 8 * per_piece;      // wave instructions of the trip
    for (int j = wvu; j < total; j += 4) {     // wave-uniform
        const int bp = j / per_piece;          // block * 8 + piece
        const int r = (j - bp * per_piece) * 64 + lane;
        const int row = min(r, m - 1);         // padding rows read a valid row
        const double* src = A + size_t(k0 + row) * nz + c0 + 16 * (bp >> 3) + 2 * (bp & 7);
        __builtin_amdgcn_global_load_lds((glb_void_t*)(src), (lds_void_t*)(smem + 128 * size_t(j)), 16, 0, 0);
    }
}

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
        // P -= L[k0+i][t] L[k0+j][t], t < k0.  Even depth counts: the finished
        // columns are staged in LDS by direct (register-free) loads, as many
        // 16-column blocks per memory round trip as the panel region holds;
        // odd depth counts (rows not 16-byte aligned): 32 columns at a time
        // through registers.
        if ((nz & 1) == 0 && k0 > 0) {
            const int rows64 = (m + 63) & ~63;
            const int blk = rows64 * 8;   // 16-byte pieces of one 16-column block
            const int nbt = max(1, min(stage_pieces(nz) / blk, k0 / 16));
            const int wvu = __builtin_amdgcn_readfirstlane(wv);
            // lane part of the operand indices: column kk + lk of staged row i
            // is at the uniform column part of kk + lo + 2 i
            const int lo = (lk >> 1) * rows64 * 2 + (lk & 1);
            for (int c0 = 0; c0 < k0; c0 += 16 * nbt) {
                const int nb = min(nbt, (k0 - c0) / 16);
                stage_columns(A, nz, k0, m, c0, nb, rows64, smem, wvu, lane);
                __builtin_amdgcn_s_waitcnt(0);   // this wave's direct loads are in LDS
                __syncthreads();
                for (int kb0 = 0; kb0 < 16 * nb; kb0 += 8) {
                    // the operands of two K steps are read before their MFMAs
                    double bv[2][2], av[2][Q];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int kk = kb0 + 4 * h;
                        const int u = (kk >> 4) * rows64 * 16 + ((kk & 15) >> 1) * rows64 * 2 + lo;
                        bv[h][0] = (li < kb) ? smem[u + 2 * li] : 0.0;
                        bv[h][1] = (16 + li < kb) ? smem[u + 2 * (16 + li)] : 0.0;
#pragma unroll
                        for (int q = 0; q < Q; ++q) {
                            const int i = 16 * (wv + 4 * q) + li;
                            av[h][q] = (wv + 4 * q < nrb && i < m) ? -smem[u + 2 * i] : 0.0;
                        }
                    }
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int q = 0; q < Q; ++q) {
                            if (wv + 4 * q < nrb) {
                                acc[q][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h][q], bv[h][0], acc[q][0], 0, 0, 0);
                                acc[q][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h][q], bv[h][1], acc[q][1], 0, 0, 0);
                            }
                        }
                }
                __syncthreads();
            }
        }
        for (int t0 = 0; (nz & 1) && t0 < k0; t0 += CB) {
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
        // Factor the kb x kb diagonal block in one wave and invert it, by
        // 4 x 4 blocks.  Lane (bi, bj) = (lane / 8, lane % 8) holds block
        // (bi, bj) of the panel's diagonal block (a, becoming L) and of the
        // identity (x, becoming D = L^{-1}); a partial block is padded with
        // the identity.  Right-looking over the diagonal blocks g:
        //  * every lane factors its own 4 x 4 block in registers (only lane
        //    (g, g)'s result is used): L_gg and D_gg = L_gg^{-1};
        //  * the column below: L_ig = A_ig D_gg^T; block row g of D:
        //    X_g = D_gg X_g;
        //  * the trailing blocks: A_ij -= L_ig L_jg^T, X_ij -= L_ig X_gj.
        // The blocks a lane needs from another pass through LDS (the panel's
        // D buffer, written with its final value afterwards); a wave-scope
        // fence pair orders each exchange (without it the compiler may run the
        // readers' branch before the writers', the branches being exclusive
        // within one lane).
        if (tid < 64) {
            auto wave_sync = [] {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            };
            const int bi = tid >> 3, bj = tid & 7;
            const bool act = bi >= bj;
            double a[4][4], x[4][4];
            int bad = 0;   // first failing column of this block (wave-uniform)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int i = 4 * bi + r, jj = 4 * bj + c;
                    a[r][c] = (act && i < kb && jj < kb && jj <= i) ? sP[i * CBP + jj] : (i == jj ? 1.0 : 0.0);
                    x[r][c] = (i == jj) ? 1.0 : 0.0;
                }
            double* sDg = sD;             // D_gg
            double* sCol = sD + 16;       // [bi][16]: L_ig
            double* sRow = sD + 16 * 9;   // [bj][16]: X_gj
            for (int g = 0; g < 8; ++g) {
                // 4 x 4 Cholesky of the lane's own block, and its inverse
                double l[4][4], d[4][4];
                int fail = 0;   // 1 + first failing pivot of the block, or 0
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int c = 0; c < 4; ++c) l[r][c] = a[r][c];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    double dk = l[k][k];
                    const bool ok = dk > 0.0 && isfinite(dk);
                    fail = (!ok && fail == 0) ? k + 1 : fail;
                    dk = ok ? dk : 1.0;
                    // 1/sqrt(dk) from the hardware estimate and two Newton steps
                    double inv = __builtin_amdgcn_rsq(dk);
                    const double hd = 0.5 * dk;
                    inv = inv * fma(-hd * inv, inv, 1.5);
                    inv = inv * fma(-hd * inv, inv, 1.5);
                    l[k][k] = dk * inv;
                    d[k][k] = inv;
#pragma unroll
                    for (int i = k + 1; i < 4; ++i) l[i][k] *= inv;
#pragma unroll
                    for (int i = k + 1; i < 4; ++i)
#pragma unroll
                        for (int j = k + 1; j <= i; ++j) l[i][j] -= l[i][k] * l[j][k];
                }
#pragma unroll
                for (int i = 1; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < i; ++j) {
                        double t = 0.0;
#pragma unroll
                        for (int k = j; k < i; ++k) t += l[i][k] * d[k][j];
                        d[i][j] = -d[i][i] * t;
                    }
                const int fg = __builtin_amdgcn_readlane(fail, 9 * g);
                bad = (bad == 0 && fg != 0 && 4 * g + fg - 1 < kb) ? k0 + 4 * g + fg : bad;
                if (bi == g && bj == g) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            a[r][c] = c <= r ? l[r][c] : 0.0;
                            sDg[4 * r + c] = c <= r ? d[r][c] : 0.0;
                        }
                }
                wave_sync();
                double dg[4][4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int c = 0; c < 4; ++c) dg[r][c] = sDg[4 * r + c];
                if (bi > g && bj == g) {   // L_ig = A_ig D_gg^T
                    double t[4][4];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            double v = 0.0;
#pragma unroll
                            for (int k = 0; k <= c; ++k) v += a[r][k] * dg[c][k];
                            t[r][c] = v;
                        }
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            a[r][c] = t[r][c];
                            sCol[16 * bi + 4 * r + c] = t[r][c];
                        }
                }
                if (bi == g && bj <= g) {   // X_gj = D_gg X_gj
                    double t[4][4];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            double v = 0.0;
#pragma unroll
                            for (int k = 0; k <= r; ++k) v += dg[r][k] * x[k][c];
                            t[r][c] = v;
                        }
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            x[r][c] = t[r][c];
                            sRow[16 * bj + 4 * r + c] = t[r][c];
                        }
                }
                wave_sync();
                if (bi > g) {
                    double li[4][4], lj[4][4];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 4; ++c) li[r][c] = sCol[16 * bi + 4 * r + c];
                    if (bj > g && act) {   // A_ij -= L_ig L_jg^T
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int c = 0; c < 4; ++c) lj[r][c] = sCol[16 * bj + 4 * r + c];
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int c = 0; c < 4; ++c) {
                                double v = a[r][c];
#pragma unroll
                                for (int k = 0; k < 4; ++k) v -= li[r][k] * lj[c][k];
                                a[r][c] = v;
                            }
                    } else if (bj <= g) {   // X_ij -= L_ig X_gj
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int c = 0; c < 4; ++c) lj[r][c] = sRow[16 * bj + 4 * r + c];
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int c = 0; c < 4; ++c) {
                                double v = x[r][c];
#pragma unroll
                                for (int k = 0; k < 4; ++k) v -= li[r][k] * lj[k][c];
                                x[r][c] = v;
                            }
                    }
                }
                wave_sync();   // every read of this step before the next step's writes
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int i = 4 * bi + r, jj = 4 * bj + c;
                    if (act && i < kb && jj <= i) sP[i * CBP + jj] = a[r][c];
                    sD[i * CBP + jj] = act ? x[r][c] : 0.0;
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
