// Restriction of each pair's unknowns to a disk in (k_m, k_z), as a
// transform of its Gram and right-hand sides (FP64 MFMA).
//
// Paper, Section 3.1: the depth integrals are rewritten over the vertical
// wavenumber k_z and V~(k_x, k_z) is kept only inside |k| <= K (K = 2.2
// w_max / c0 in the paper).  On the inversion's depth grid the transform over
// z is the discrete one, k_z,j = 2 pi j / (nz dz); at the pair of k_m the kept
// modes are those with k_z,j^2 + |k_m|^2 <= K^2, i.e. |j| <= jmax.  The
// orthogonal projector onto them is circulant,
//     Q[a][b] = q((a - b) mod nz),
//     q(d) = (1 + 2 sum_{j=1}^{jc} cos(2 pi j d / nz) + [Nyquist kept] (-1)^d) / nz,
// with jc the kept cos/sin pairs.  Solving the pair's system on range(Q) is
// solving it with the Gram Q G Q and right-hand sides Q c: Q G Q is zero on
// the complement of range(Q), so a truncated SVD drops that complement (its
// singular values are 0) and keeps the solution inside the disk.  Both
// products run on v_mfma_f64_16x16x4 with the q table in LDS:
//     T = G Q   (all 64 x 64 tiles; G read from its lower triangle)
//     G' = Q T  (lower tiles only, written over the lower triangle of G).

#include "dev_common.h"

namespace edt {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Largest kept index j in [0, nz/2] of the pair of k_m index u, or -1.  The
// comparison is evaluated exactly as written (no fused multiply-adds), so the
// kept set is a plain function of the IEEE products and sums.  On the survey
// of parallel lines u = ux n_line + c and the horizontal wavenumber is
// (k_m, k_y).
__device__ int kz_jmax(int u, int dim, int n_mid, double d_mid, int n_line, double d_line, int nz, double dz,
                       double K) {
#pragma clang fp contract(off)
    const double dk = kTwoPiD / (double(n_mid) * d_mid);
    auto sgn = [&](int v) { return v < (n_mid + 1) / 2 ? v : v - n_mid; };
    double km2;
    if (n_line > 0) {
        const int c = u % n_line;
        const double kx = double(sgn(u / n_line)) * dk;
        const double ky = double(c < (n_line + 1) / 2 ? c : c - n_line) * (kTwoPiD / (double(n_line) * d_line));
        km2 = kx * kx + ky * ky;
    } else if (dim == 3) {
        const double kx = double(sgn(u / n_mid)) * dk, ky = double(sgn(u % n_mid)) * dk;
        km2 = kx * kx + ky * ky;
    } else {
        const double k = double(sgn(u)) * dk;
        km2 = k * k;
    }
    const double dkz = kTwoPiD / (double(nz) * dz);
    const double K2 = K * K;
    int jmax = -1;
    for (int j = 0; j <= nz / 2; ++j) {
        const double kz = double(j) * dkz;
        if (kz * kz + km2 <= K2) jmax = j;
    }
    return jmax;
}

// Per pair: the circulant row q (nz values) and the number of kept modes.
__global__ __launch_bounds__(256) void kz_q_kernel(const int32_t* __restrict__ pair_u, int dim, int n_mid,
                                                   double d_mid, int n_line, double d_line, int nz, double dz,
                                                   double K, double* __restrict__ q, int32_t* __restrict__ n_keep) {
    const int p = blockIdx.x, tid = threadIdx.x;
    const int jmax = kz_jmax(pair_u[2 * p], dim, n_mid, d_mid, n_line, d_line, nz, dz, K);
    const int jc = jmax < (nz - 1) / 2 ? jmax : (nz - 1) / 2;   // cos/sin pairs j = 1..jc
    const bool nyq = (nz % 2 == 0) && jmax == nz / 2;
    for (int d = tid; d < nz; d += 256) {
        double s = jmax >= 0 ? 1.0 : 0.0;
        for (int j = 1; j <= jc; ++j) {
            const int m = int((int64_t(j) * d) % nz);   // exact reduction of the angle
            s += 2.0 * cospi(2.0 * double(m) / double(nz));
        }
        if (nyq) s += (d & 1) ? -1.0 : 1.0;
        q[size_t(p) * nz + d] = s / double(nz);
    }
    if (tid == 0 && n_keep) n_keep[p] = jmax < 0 ? 0 : 1 + 2 * jc + (nyq ? 1 : 0);
}

// One product per pair and 64 x 64 tile (tiles dealt to the XCDs pair by
// pair); K in chunks of 32 staged in LDS with
// the next chunk's operands fetched into registers during the current chunk's
// MFMAs (each wave a 32 x 32 quarter: 2 x 2 v_mfma_f64_16x16x4 tiles).
//   MODE 0: T = G Q, every tile; G from its lower triangle.
//   MODE 1: G' = Q T, lower tiles; the elements with i >= j are stored.
template <int MODE>
__global__ __launch_bounds__(256, 4) void kz_gemm_kernel(const double* __restrict__ S, const double* __restrict__ q,
                                                      double* __restrict__ C, int nz, int nt, int n_pairs) {
    __shared__ double As[64][33];
    __shared__ double Bs[32][65];
    __shared__ double s_q[kMaxDepth];
    const int ntile = MODE == 0 ? nt * nt : nt * (nt + 1) / 2;
    int p, tile;
    xcd_pair_tile(blockIdx.x, ntile, p, tile);
    if (p >= n_pairs) return;
    int ti, tj;
    if constexpr (MODE == 0) {
        ti = tile / nt;
        tj = tile - ti * nt;
    } else {
        ti = 0;
        while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
        tj = tile - ti * (ti + 1) / 2;
    }
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int d = tid; d < nz; d += 256) s_q[d] = q[size_t(p) * nz + d];
    __syncthreads();
    const int r0 = 64 * ti, c0 = 64 * tj;
    const size_t base = size_t(p) * nz * nz;
    const double* Sp = S + base;
    auto qv = [&](int a, int b) {   // Q[a][b] for 0 <= a, b < nz
        const int d = a - b;
        return s_q[d < 0 ? d + nz : d];
    };
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
    // A chunk: 64 rows x 32 k; B chunk: 32 k x 64 columns.  In MODE 0 a chunk
    // wholly above the diagonal of G is read transposed (G[k][r], coalesced
    // along r) and staged back in place.
    auto a_row_major = [&](int k0) { return MODE == 1 || !(k0 >= r0 + 64); };
    auto fetch = [&](int k0) {
        const bool rm = a_row_major(k0);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = tid + 256 * t;
            const int ar = rm ? (e >> 5) : (e & 63), ak = rm ? (e & 31) : (e >> 6);
            const int gr = r0 + ar, gk = k0 + ak;
            double av = 0.0;
            if (gr < nz && gk < nz) {
                if constexpr (MODE == 0) av = gr >= gk ? Sp[size_t(gr) * nz + gk] : Sp[size_t(gk) * nz + gr];
                else av = qv(gr, gk);
            }
            ra[t] = av;
            const int bk = e >> 6, bc = e & 63;
            const int hk = k0 + bk, hc = c0 + bc;
            double bv = 0.0;
            if (hk < nz && hc < nz) {
                if constexpr (MODE == 0) bv = qv(hk, hc);
                else bv = Sp[size_t(hk) * nz + hc];
            }
            rb[t] = bv;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < nz; k0 += 32) {
        const bool rm = a_row_major(k0);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = tid + 256 * t;
            if (rm) As[e >> 5][e & 31] = ra[t];
            else As[e & 63][e >> 6] = ra[t];
            Bs[e >> 6][e & 63] = rb[t];
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
    double* Cp = C + base;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = r0 + wr + 16 * a + 4 * v + lk, j = c0 + wc + 16 * b + li;
                if (i < nz && j < nz && (MODE == 0 || i >= j)) Cp[size_t(i) * nz + j] = acc[a][b][v];
            }
}

// c <- Q c for both right-hand sides of every pair (in place).
__global__ __launch_bounds__(256) void kz_rhs_kernel(double* __restrict__ rhs, const double* __restrict__ q,
                                                     int nz) {
    __shared__ double s_q[kMaxDepth];
    __shared__ double s_c[2 * kMaxDepth];
    const int p = blockIdx.x, tid = threadIdx.x;
    double* c = rhs + size_t(p) * 2 * nz;
    for (int d = tid; d < nz; d += 256) {
        s_q[d] = q[size_t(p) * nz + d];
        s_c[d] = c[d];
        s_c[nz + d] = c[nz + d];
    }
    __syncthreads();
    for (int i = tid; i < nz; i += 256) {
        double s0 = 0.0, s1 = 0.0;
        for (int j = 0; j < nz; ++j) {
            const int d = i - j;
            const double w = s_q[d < 0 ? d + nz : d];
            s0 += w * s_c[j];
            s1 += w * s_c[nz + j];
        }
        c[i] = s0;
        c[nz + i] = s1;
    }
}

// ------------------------------------------------------------- launcher ---
// Scratch inside the truncated-SVD workspace (free until edt_tsvd runs): the
// q table in the first sign-iterate buffer, T in the product buffer.
hipError_t launch_kz_restrict(const edt_plan* p, double K, double* gram, double* rhs, unsigned char* tw,
                              int32_t* n_keep, hipStream_t st) {
    if (p->n_pairs == 0) return hipSuccess;
    const TsvdLayout l = tsvd_layout(p);
    const int nz = p->nz, nt = (nz + 63) / 64;
    const unsigned P = unsigned(p->n_pairs);
    double* q = reinterpret_cast<double*>(tw + l.x0);
    double* T = reinterpret_cast<double*>(tw + l.y);
    hipLaunchKernelGGL(kz_q_kernel, dim3(P), dim3(256), 0, st, dptr<const int32_t>(p, p->lay.pair_u), p->dim,
                       p->n_mid, p->d_mid, p->n_line, p->d_line, nz, p->dz, K, q, n_keep);
    hipLaunchKernelGGL(kz_gemm_kernel<0>, dim3(xcd_pair_grid(P, nt * nt)), dim3(256), 0, st, gram, q, T, nz, nt,
                       int(P));
    hipLaunchKernelGGL(kz_gemm_kernel<1>, dim3(xcd_pair_grid(P, nt * (nt + 1) / 2)), dim3(256), 0, st, T, q, gram,
                       nz, nt, int(P));
    hipLaunchKernelGGL(kz_rhs_kernel, dim3(P), dim3(256), 0, st, rhs, q, nz);
    return hipGetLastError();
}

}  // namespace edt
