// Kernel (e): the paper's own solver -- a truncated SVD of every pair's
// system -- computed from the pair's Gram with FP64 MFMA.
//
// Paper, Section 3.1: the reciprocal of every singular value s_j below a
// tolerance sigma is replaced by zero.  For the real form of the pair's rows
// the s_j^2 and v_j are the eigenpairs of the Gram G, and the truncated
// solution is x = sum_{s_j^2 >= sigma^2} v_j (v_j . c) / s_j^2 (c = A^T b).
// With P the spectral projector of G onto its eigenvalues >= sigma^2,
//     x = (G + sigma^2 (I - P))^{-1} P c :
// G and P commute, and the bracket is G on range(P) (eigenvalues >= sigma^2)
// and G + sigma^2 on the rest (eigenvalues in [sigma^2, 2 sigma^2)), so it is
// positive definite and the existing Cholesky solve applies.  P = (I + S)/2
// with S the matrix sign of G - sigma^2 I, by scaled Newton-Schulz steps
//     X_0 = (G - sigma^2 I) / ||G - sigma^2 I||_F,   X <- (a/2) X (3 I - a^2 X^2),
// which drive every nonzero eigenvalue of X_0 (all in [-1, 1]) to +-1.  Any
// a in [1, sqrt 3] keeps the spectrum in [-1, 1]; with a lower bound l on the
// eigenvalue magnitudes, a = sqrt(3 / (1 + l + l^2)) maps [l, 1] onto
// [f(l), 1] (the scaling of Chen and Chow for the Hermitian sign function),
// so small eigenvalues grow up to 2.6 times per step instead of 1.5; the host
// runs the bound l from a guess, caps a (see tsvd_step_scales) and sets a = 1
// (the plain step, quadratic near +-1) once l >= 0.999.  An eigenvalue below
// the guess still converges, in more steps.  Two batched FP64 products per step; a pair stops after a plain
// step once ||X^2 - I||_F <= 1e-9 (a scaled step would move it off +-1).  An
// eigenvalue of G within rounding of sigma^2 has no definite side (the
// truncation itself is discontinuous there): such a pair does not converge
// and is reported as such.
// The tolerance is relative: sigma^2 = tol_rel^2 ||G||_F.

#include "dev_common.h"

namespace edt {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr double kSignTol = 1e-9;   // ||X^2 - I||_F at which the sign iteration stops

// Scaling of each sign step from a guess l0 of the smallest eigenvalue
// magnitude of X_0 (the bound is advanced as l <- f(l)); 1 from l >= 0.999 on.
// The scaling is capped at its value for l = 0.3: a fully scaled step maps +-1
// to about +-2.6 l, by the difference of two terms of order 1, and the
// rounding of that difference then perturbs every direction's sign by about
// u / l; capped, +-1 stays above 0.57 in magnitude and small eigenvalues
// still grow about 2.23 times per step.
void tsvd_step_scales(double l0, int n, double* a) {
    constexpr double kCapBound = 0.3;
    double l = l0;
    for (int k = 0; k < n; ++k) {
        if (l >= 0.999) {
            a[k] = 1.0;
            continue;
        }
        const double lb = l > kCapBound ? l : kCapBound;
        const double s = sqrt(3.0 / (1.0 + lb + lb * lb));
        a[k] = s;
        l = 0.5 * s * l * (3.0 - s * s * l * l);
    }
}

// Per pair: the threshold, X_0 (full, row-major nz x nz) from the lower
// triangle of G, and the iteration state.  An empty pair, or one whose Gram
// is zero, gets X = -I (nothing kept) and counts as converged.
__global__ __launch_bounds__(256) void tsvd_init_kernel(const double* __restrict__ gram,
                                                        const int64_t* __restrict__ urow_off, int nz,
                                                        double tol_rel, double* __restrict__ X,
                                                        double* __restrict__ tau2, int32_t* __restrict__ conv,
                                                        int32_t* __restrict__ iters) {
    __shared__ double s_red[8];
    const int p = blockIdx.x, tid = threadIdx.x;
    const double* G = gram + size_t(p) * nz * nz;
    double* Xp = X + size_t(p) * nz * nz;
    double f2 = 0.0, tr = 0.0;
    for (int e = tid; e < nz * nz; e += 256) {
        const int i = e / nz, j = e - i * nz;
        if (j > i) continue;
        const double g = G[e];
        f2 += (i == j ? 1.0 : 2.0) * g * g;
        if (i == j) tr += g;
    }
    f2 = wave_sum(f2);
    tr = wave_sum(tr);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) {
        s_red[wv] = f2;
        s_red[4 + wv] = tr;
    }
    __syncthreads();
    f2 = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    tr = (s_red[4] + s_red[5]) + (s_red[6] + s_red[7]);
    const bool empty = urow_off[p + 1] == urow_off[p];
    const double nrm = sqrt(f2);
    const bool none = empty || !(nrm > 0.0);
    const double t2 = none ? 1.0 : tol_rel * tol_rel * nrm;
    // ||G - t2 I||_F^2 = ||G||_F^2 - 2 t2 tr G + nz t2^2
    const double a2 = f2 - 2.0 * t2 * tr + double(nz) * t2 * t2;
    const double inv = (a2 > 0.0) ? 1.0 / sqrt(a2) : 0.0;
    for (int e = tid; e < nz * nz; e += 256) {
        const int i = e / nz, j = e - i * nz;
        double v;
        if (none) v = (i == j) ? -1.0 : 0.0;
        else v = ((i >= j ? G[size_t(i) * nz + j] : G[size_t(j) * nz + i]) - (i == j ? t2 : 0.0)) * inv;
        Xp[e] = v;
    }
    if (tid == 0) {
        tau2[p] = t2;
        conv[p] = none ? 1 : 0;
        iters[p] = 0;
    }
}

// One product of the sign iteration for every pair still iterating.  Every
// iterate is a polynomial in G, so both products are symmetric: only the
// lower 64 x 64 tiles are computed (T = nt (nt + 1) / 2 per pair, dealt to
// the XCDs pair by pair) and an off-diagonal tile is also stored
// mirrored.  K runs in chunks of 32 staged in LDS, the next chunk's loads in
// flight during the current chunk's v_mfma_f64_16x16x4 (each wave a 32 x 32
// quarter: 2 x 2 MFMA tiles; lane l of register v holds row 4 v + l / 16,
// column l % 16).
//   MODE 0: C = X X,                 and per tile sum (C - I)^2 -> dpart
//   MODE 1: C = 1.5 a X - 0.5 a^3 X B      (B = X X)
template <int MODE>
__global__ __launch_bounds__(256, 4) void ns_gemm_kernel(const double* __restrict__ X, const double* __restrict__ B,
                                                      double* __restrict__ C, const int32_t* __restrict__ conv,
                                                      double* __restrict__ dpart, int nz, int nt, double a,
                                                      int n_pairs) {
    __shared__ double As[64][33];
    __shared__ double Bs[32][65];
    __shared__ double s_red[4];
    const int ntri = nt * (nt + 1) / 2;
    int p, tile;
    xcd_pair_tile(blockIdx.x, ntri, p, tile);
    if (p >= n_pairs || conv[p]) return;
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
    const int tj = tile - ti * (ti + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r0 = 64 * ti, c0 = 64 * tj;
    const size_t base = size_t(p) * nz * nz;
    const double* Xp = X + base;
    const double* Bp = B + base;
    const int li = lane & 15, lk = lane >> 4;
    const int wr = 32 * (wv >> 1), wc = 32 * (wv & 1);
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
    double ra[8], rb[8];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            const int ar = e >> 5, ak = e & 31;   // A chunk: 64 rows x 32 k
            const int gr = r0 + ar, gk = k0 + ak;
            ra[q] = (gr < nz && gk < nz) ? Xp[size_t(gr) * nz + gk] : 0.0;
            const int bk = e >> 6, bc = e & 63;   // B chunk: 32 k x 64 columns
            const int hk = k0 + bk, hc = c0 + bc;
            rb[q] = (hk < nz && hc < nz) ? Bp[size_t(hk) * nz + hc] : 0.0;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < nz; k0 += 32) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            As[e >> 5][e & 31] = ra[q];
            Bs[e >> 6][e & 63] = rb[q];
        }
        __syncthreads();
        if (k0 + 32 < nz) fetch(k0 + 32);
#pragma unroll 2
        for (int kk = 0; kk < 32; kk += 4) {
            const double a0 = As[wr + li][kk + lk], a1 = As[wr + 16 + li][kk + lk];
            const double b0 = Bs[kk + lk][wc + li], b1 = Bs[kk + lk][wc + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    const bool mirror = ti != tj;
    const double c1 = 1.5 * a, c3 = 0.5 * a * a * a;
    double d2 = 0.0;
    double* Cp = C + base;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = r0 + wr + 16 * a + 4 * v + lk, j = c0 + wc + 16 * b + li;
                if (i < nz && j < nz) {
                    const size_t at = size_t(i) * nz + j;
                    double c;
                    if constexpr (MODE == 0) {
                        c = acc[a][b][v];
                        const double e = c - (i == j ? 1.0 : 0.0);
                        d2 += (mirror ? 2.0 : 1.0) * e * e;
                    } else {
                        c = c1 * Xp[at] - c3 * acc[a][b][v];
                    }
                    Cp[at] = c;
                    if (mirror) Cp[size_t(j) * nz + i] = c;
                }
            }
    if constexpr (MODE == 0) {
        d2 = wave_sum(d2);
        if (lane == 0) s_red[wv] = d2;
        __syncthreads();
        if (tid == 0) dpart[size_t(p) * ntri + tile] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    }
}

// After one step: ||X_k^2 - I||_F from the tile partials (fixed order); the
// new iterate is accepted (iters + 1), and after a plain step (accept) the
// pair stops once X_k was within the tolerance (X_{k+1} is then closer still).
__global__ __launch_bounds__(256) void ns_check_kernel(const double* __restrict__ dpart, int nt,
                                                       int32_t* __restrict__ conv, int32_t* __restrict__ iters,
                                                       int n_pairs, int accept) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n_pairs || conv[p]) return;
    double s = 0.0;
    const int ntri = nt * (nt + 1) / 2;
    for (int t = 0; t < ntri; ++t) s += dpart[size_t(p) * ntri + t];
    iters[p] += 1;
    if (accept && sqrt(s) <= kSignTol) conv[p] = 1;
}

// P = (I + X)/2 with X the last iterate (buffer iters % 2):
// lower triangle of G <- G + tau2 (I - P) = G + tau2 (I - X)/2 (i >= j), and
// rhs' = P c for both right-hand sides (X symmetric: column reads coalesce).
__global__ __launch_bounds__(256) void tsvd_final_kernel(double* __restrict__ gram, const double* __restrict__ X0,
                                                         const double* __restrict__ X1, const double* __restrict__ rhs,
                                                         const double* __restrict__ tau2,
                                                         const int32_t* __restrict__ iters, int nz,
                                                         double* __restrict__ rhs_p) {
    const int p = blockIdx.x, tid = threadIdx.x;
    const size_t base = size_t(p) * nz * nz;
    const double* X = ((iters[p] & 1) ? X1 : X0) + base;
    double* G = gram + base;
    const double t2 = tau2[p];
    for (int e = tid; e < nz * nz; e += 256) {
        const int i = e / nz, j = e - i * nz;
        if (j <= i) G[e] += 0.5 * t2 * ((i == j ? 1.0 : 0.0) - X[e]);
    }
    const double* c = rhs + size_t(p) * 2 * nz;
    for (int i = tid; i < nz; i += 256) {
        double s0 = 0.0, s1 = 0.0;
        for (int j = 0; j < nz; ++j) {
            const double xv = X[size_t(j) * nz + i];   // = X[i][j]
            s0 += xv * c[j];
            s1 += xv * c[nz + j];
        }
        rhs_p[size_t(p) * 2 * nz + i] = 0.5 * (c[i] + s0);
        rhs_p[size_t(p) * 2 * nz + nz + i] = 0.5 * (c[nz + i] + s1);
    }
}

// ------------------------------------------------------------- launchers ---
TsvdLayout tsvd_layout(const edt_plan* p) {
    TsvdLayout l{};
    const size_t P = size_t(p->n_pairs), nz = size_t(p->nz);
    const size_t nt = (nz + 63) / 64;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~size_t(255);
        return at;
    };
    l.x0 = take(P * nz * nz * 8);
    l.x1 = take(P * nz * nz * 8);
    l.y = take(P * nz * nz * 8);
    l.rhs = take(P * 2 * nz * 8);
    l.tau2 = take(P * 8);
    l.dpart = take(P * nt * (nt + 1) / 2 * 8);
    l.conv = take(P * 4);
    l.total = off;
    return l;
}

hipError_t launch_tsvd_init(const edt_plan* p, const double* gram, double tol_rel, unsigned char* tw,
                            int32_t* iters, hipStream_t st) {
    if (p->n_pairs == 0) return hipSuccess;
    const TsvdLayout l = tsvd_layout(p);
    hipLaunchKernelGGL(tsvd_init_kernel, dim3(unsigned(p->n_pairs)), dim3(256), 0, st, gram,
                       dptr<const int64_t>(p, p->lay.urow_off), p->nz, tol_rel,
                       reinterpret_cast<double*>(tw + l.x0), reinterpret_cast<double*>(tw + l.tau2),
                       reinterpret_cast<int32_t*>(tw + l.conv), iters);
    return hipGetLastError();
}

// Step k reads X_k from buffer k % 2 and writes X_{k+1} to the other, with
// scaling a (a = 1: a plain step, after which converged pairs stop).
hipError_t launch_tsvd_step(const edt_plan* p, int k, double a, unsigned char* tw, int32_t* iters,
                            hipStream_t st) {
    if (p->n_pairs == 0) return hipSuccess;
    const TsvdLayout l = tsvd_layout(p);
    const int nz = p->nz, nt = (nz + 63) / 64;
    double* xa = reinterpret_cast<double*>(tw + ((k & 1) ? l.x1 : l.x0));
    double* xb = reinterpret_cast<double*>(tw + ((k & 1) ? l.x0 : l.x1));
    double* y = reinterpret_cast<double*>(tw + l.y);
    double* dpart = reinterpret_cast<double*>(tw + l.dpart);
    int32_t* conv = reinterpret_cast<int32_t*>(tw + l.conv);
    const int P = int(p->n_pairs);
    const dim3 grid(xcd_pair_grid(P, nt * (nt + 1) / 2));
    hipLaunchKernelGGL(ns_gemm_kernel<0>, grid, dim3(256), 0, st, xa, xa, y, conv, dpart, nz, nt, 1.0, P);
    hipLaunchKernelGGL(ns_gemm_kernel<1>, grid, dim3(256), 0, st, xa, y, xb, conv, dpart, nz, nt, a, P);
    hipLaunchKernelGGL(ns_check_kernel, dim3(unsigned((p->n_pairs + 255) / 256)), dim3(256), 0, st, dpart, nt,
                       conv, iters, int(p->n_pairs), a == 1.0 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_tsvd_final(const edt_plan* p, double* gram, const double* rhs, unsigned char* tw,
                             const int32_t* iters, hipStream_t st) {
    if (p->n_pairs == 0) return hipSuccess;
    const TsvdLayout l = tsvd_layout(p);
    hipLaunchKernelGGL(tsvd_final_kernel, dim3(unsigned(p->n_pairs)), dim3(256), 0, st, gram,
                       reinterpret_cast<const double*>(tw + l.x0), reinterpret_cast<const double*>(tw + l.x1),
                       rhs, reinterpret_cast<const double*>(tw + l.tau2), iters, p->nz,
                       reinterpret_cast<double*>(tw + l.rhs));
    return hipGetLastError();
}

}  // namespace edt
