// Finite aperture on the 2D line survey (paper eq. M): the Gram of each pair
// under an offset window |x_R - x_S| <= 2 b.
//
// On the periodic line the window acts at each k_m as a circular convolution
// of the rows over the receiver index a with the window's DFT (the discrete
// sinc); that convolution S is an orthogonal projector, so the normal
// equations keep the right-hand sides Re(A^H d_W) of the windowed data and
// take the Gram
//     Re(A^H S A) = (1/N) sum_{o in window} Re(Ah(o)^H Ah(o)),
//     Ah(o, z) = sum_a A(a, z) e^{2 pi i a o / N},
// with the rows of one frequency transformed over a.  Per frequency: the rows
// of every pair are built over a in LDS straight from the Green's tables (zero
// where a row is cut) and transformed there, only the kept offsets go to HBM,
// and they enter a lower-tile FP64 MFMA product that accumulates over the
// frequencies.  Rows of one frequency mix, so unique rows do not merge here.

#include <cmath>

#include "dev_common.h"
#include "lines.h"

namespace edt {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kApLds = 80 * 1024;   // LDS of one row-transform block (gfx950: 160 KiB per CU)

// For the rows of pair p at frequency f0, lines z0 .. z0 + L - 1 of
//     Ah(o, z) = sum_a A(a, z) e^{2 pi i a o / N},  A(a, z) = w^2 dz g(z; k_r) g(z; k_s)
// (A = 0 where no row has receiver index a), built in LDS straight from the
// Green's tables and transformed there; only the nW kept offsets
// o = (lo + k) mod N are stored: Rh[p][k][z].  Rows of a pair are ordered by
// frequency, so those of f0 are one range, found by bisection.  A power-of-two
// N takes the radix-2 transform, any other N a direct sum for the kept
// offsets only.
template <bool POW2>
__global__ __launch_bounds__(256) void ap_rows_fft_kernel(const zd* __restrict__ g64,
                                                          const uint32_t* __restrict__ rows,
                                                          const int32_t* __restrict__ keys,
                                                          const int64_t* __restrict__ franges, int f0, int n_freq,
                                                          int n_cls, int N, int logn, int nz, int L, zd scale, int lo,
                                                          int nW, const zd* __restrict__ tw, zd* __restrict__ Rh) {
    extern __shared__ zd s_mem[];
    const int ns = lds_stride(N);
    zd* s_x = s_mem;            // L lines of N values (padded layout)
    zd* s_w = s_mem + L * ns;   // twiddles e^{2 pi i k / N}: N / 2 (radix 2) or N (direct)
    const int tid = threadIdx.x;
    const int per_pair = nz / L;
    const int p = int(blockIdx.x / unsigned(per_pair)), z0 = int(blockIdx.x % unsigned(per_pair)) * L;
    const int nw = POW2 ? N / 2 : N;
    for (int k = tid; k < nw; k += 256) s_w[k] = tw[k];
    for (int e = tid; e < L * ns; e += 256) s_x[e] = zd{0.0, 0.0};
    const int64_t r0 = franges[size_t(p) * (n_freq + 1) + f0];
    const int64_t n = franges[size_t(p) * (n_freq + 1) + f0 + 1] - r0;
    __syncthreads();
    const zd* gf = g64 + size_t(f0) * n_cls * nz;
    for (int64_t e = tid; e < n * L; e += 256) {
        const int64_t r = r0 + e / L;
        const int j = int(e % L), z = z0 + j;
        const uint32_t c = rows[2 * r + 1];
        const int a = keys[2 * r];
        const zd gr = gf[size_t(c & 0xFFFFu) * nz + z], gs = gf[size_t(c >> 16) * nz + z];
        s_x[j * ns + lds_pad(POW2 ? bit_reverse(a, logn) : a)] = scale * (gr * gs);
    }
    __syncthreads();
    zd* Rp = Rh + size_t(p) * nW * nz;
    if constexpr (POW2) {
        dit_lines(s_x, s_w, N, logn, L);
        for (int e = tid; e < L * nW; e += 256) {
            const int j = e % L, k = e / L;
            int o = (lo + k) % N;
            if (o < 0) o += N;
            Rp[size_t(k) * nz + z0 + j] = s_x[j * ns + lds_pad(o)];
        }
    } else {
        for (int e = tid; e < L * nW; e += 256) {
            const int j = e % L, k = e / L;
            int o = (lo + k) % N;
            if (o < 0) o += N;
            zd acc{0.0, 0.0};
            int m = 0;   // (a o) mod N
            for (int a = 0; a < N; ++a) {
                acc = acc + s_w[m] * s_x[j * ns + lds_pad(a)];
                m += o;
                if (m >= N) m -= N;
            }
            Rp[size_t(k) * nz + z0 + j] = acc;
        }
    }
}

// C (lower tiles, += or =) of (1/N) sum over kept offsets of Re(Ah^H Ah): a
// real product over K = 2 nW (real and imaginary parts of the nW kept
// offsets, stored compactly).  Tiles dealt to the XCDs pair by pair; K in
// chunks of 32 staged in LDS, the next chunk's loads in flight.
__global__ __launch_bounds__(256, 4) void ap_gram_kernel(const zd* __restrict__ Rh, int nz, int nt, int nW,
                                                         double invN, int first, double* __restrict__ gram,
                                                         int n_pairs) {
    __shared__ double As[64][33];
    __shared__ double Bs[32][65];
    const int ntri = nt * (nt + 1) / 2;
    int p, tile;
    xcd_pair_tile(blockIdx.x, ntri, p, tile);
    if (p >= n_pairs) return;
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
    const int tj = tile - ti * (ti + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r0 = 64 * ti, c0 = 64 * tj;
    const zd* Rp = Rh + size_t(p) * nW * nz;
    const int K = 2 * nW;
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
    // element kk of K: kept offset kk / 2, real (kk even) or imaginary part;
    // A(i, kk) = part of Ah[kk / 2][r0 + i], B(kk, j) = part of
    // Ah[kk / 2][c0 + j]; threads run along z, so loads are contiguous
    auto value = [&](int kk, int z) {
        if (kk >= K || z >= nz) return 0.0;
        const zd v = Rp[size_t(kk / 2) * nz + z];
        return (kk & 1) ? v.y : v.x;
    };
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = tid + 256 * t;
            const int zi = e & 63, kk = e >> 6;   // 64 depths x 32 k
            ra[t] = value(k0 + kk, r0 + zi);
            rb[t] = value(k0 + kk, c0 + zi);
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += 32) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = tid + 256 * t;
            As[e & 63][e >> 6] = ra[t];
            Bs[e >> 6][e & 63] = rb[t];
        }
        __syncthreads();
        if (k0 + 32 < K) fetch(k0 + 32);
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
    double* Cp = gram + size_t(p) * nz * nz;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = r0 + wr + 16 * a + 4 * v + lk, j = c0 + wc + 16 * b + li;
                if (i < nz && j < nz && i >= j) {
                    const size_t at = size_t(i) * nz + j;
                    const double c = invN * acc[a][b][v];
                    Cp[at] = first ? c : Cp[at] + c;
                }
            }
}

// Per pair: the first row of each frequency (rows of a pair are ordered by
// frequency), franges[p][f] for f = 0 .. n_freq, by bisection.
__global__ __launch_bounds__(256) void ap_ranges_kernel(const uint32_t* __restrict__ rows,
                                                        const int64_t* __restrict__ row_off, int n_freq,
                                                        int64_t* __restrict__ franges) {
    const int p = blockIdx.x;
    for (int f = threadIdx.x; f <= n_freq; f += 256) {
        int64_t a = row_off[p], b = row_off[p + 1];
        while (a < b) {
            const int64_t mid = (a + b) / 2;
            if (rows[2 * mid] < uint32_t(f)) a = mid + 1;
            else b = mid;
        }
        franges[size_t(p) * (n_freq + 1) + f] = a;
    }
}

// tw[k] = e^{2 pi i k / N}, k < n.
__global__ __launch_bounds__(256) void ap_twiddle_kernel(int N, int n, zd* __restrict__ tw) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    double sv, cv;
    sincospi(2.0 * double(k) / double(N), &sv, &cv);
    tw[k] = zd{cv, sv};
}

// trace[p] = sum of the diagonal (fixed order).
__global__ __launch_bounds__(256) void ap_trace_kernel(const double* __restrict__ gram, int nz,
                                                       double* __restrict__ trace) {
    __shared__ double s_red[4];
    const int p = blockIdx.x, tid = threadIdx.x;
    double t = 0.0;
    for (int i = tid; i < nz; i += 256) t += gram[size_t(p) * nz * nz + size_t(i) * nz + i];
    t = wave_sum(t);
    if ((tid & 63) == 0) s_red[tid >> 6] = t;
    __syncthreads();
    if (tid == 0) trace[p] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// The lower tiles of scale * Re(R_p^H R_p) for every pair's n_rows x nz complex
// rows R_p (row-major, rows of pair p at R + p n_rows nz), written (first) or
// added to gram[p]; the finite aperture's product, also used by the survey of
// parallel lines on its materialised rows.
hipError_t launch_rows_gram(const zd* R, int nz, int n_rows, double scale, int first, double* gram, int64_t P,
                            hipStream_t st) {
    if (P == 0) return hipSuccess;
    const int nt = (nz + 63) / 64;
    hipLaunchKernelGGL(ap_gram_kernel, dim3(xcd_pair_grid(P, nt * (nt + 1) / 2)), dim3(256), 0, st, R, nz, nt,
                       n_rows, scale, first, gram, int(P));
    return hipGetLastError();
}

hipError_t launch_gram_trace(const double* gram, int nz, double* trace, int64_t P, hipStream_t st) {
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(ap_trace_kernel, dim3(unsigned(P)), dim3(256), 0, st, gram, nz, trace);
    return hipGetLastError();
}

// ------------------------------------------------------------- launcher ---
// Workspace: the kept offsets of one frequency (at most P N nz complex128),
// the per-pair frequency ranges and the twiddle table.
struct ApLayout {
    size_t rh, ranges, tw, total;
};
ApLayout aperture_layout(const edt_plan* p) {
    ApLayout l{};
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    l.rh = 0;
    l.ranges = up(size_t(p->n_pairs) * p->n_mid * p->nz * sizeof(zd));
    l.tw = l.ranges + up(size_t(p->n_pairs) * (p->n_freq + 1) * sizeof(int64_t));
    l.total = l.tw + up(size_t(p->n_mid) * sizeof(zd));
    return l;
}
size_t line_aperture_work_bytes(const edt_plan* p);
size_t aperture_work_bytes(const edt_plan* p) {
    return p->n_line ? line_aperture_work_bytes(p) : aperture_layout(p).total;
}

// Kept signed offsets: |s| d_mid <= 2 b_max for s in [-N/2, (N - 1)/2]
// (the same comparison as the oracle's); a contiguous range [lo, lo + nW).
void aperture_offsets(const edt_plan* p, double b_max, int* lo, int* nW) {
    const int N = p->n_mid;
    int first = 0, count = 0;
    for (int s = -(N / 2); s <= (N - 1) / 2; ++s) {
        if (std::fabs(double(s)) * p->d_mid <= 2.0 * b_max) {
            if (!count) first = s;
            ++count;
        }
    }
    *lo = first;
    *nW = count;
}

hipError_t configure_line_aperture();
hipError_t configure_aperture() {
    for (const void* k : {reinterpret_cast<const void*>(ap_rows_fft_kernel<true>),
                          reinterpret_cast<const void*>(ap_rows_fft_kernel<false>)}) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kApLds);
        if (e != hipSuccess) return e;
    }
    return configure_line_aperture();
}

hipError_t launch_aperture_gram(const edt_plan* p, const zd* g64, double b_max, double* gram, double* trace,
                                unsigned char* work, hipStream_t st) {
    if (p->n_pairs == 0) return hipSuccess;
    const ApLayout wl = aperture_layout(p);
    zd* R = reinterpret_cast<zd*>(work + wl.rh);
    int64_t* franges = reinterpret_cast<int64_t*>(work + wl.ranges);
    zd* tw = reinterpret_cast<zd*>(work + wl.tw);
    const int N = p->n_mid, nz = p->nz, nt = (nz + 63) / 64;
    const int P = int(p->n_pairs);
    int lo = 0, nW = 0;
    aperture_offsets(p, b_max, &lo, &nW);
    const bool p2 = (N & (N - 1)) == 0;
    const int nw = p2 ? N / 2 : N;
    int logn = 0;
    while ((1 << logn) < N) ++logn;
    // lines per block: 4 adjacent depths when they fit (contiguous loads)
    int L = 1;
    for (int c : {4, 2})
        if (nz % c == 0 && size_t(c * lds_stride(N) + nw) * sizeof(zd) <= kApLds) {
            L = c;
            break;
        }
    const size_t lds = size_t(L * lds_stride(N) + nw) * sizeof(zd);
    if (lds > kApLds) return hipErrorInvalidValue;
    const unsigned blocks = unsigned(P * (nz / L));
    hipLaunchKernelGGL(ap_ranges_kernel, dim3(unsigned(P)), dim3(256), 0, st, dptr<const uint32_t>(p, p->lay.rows),
                       dptr<const int64_t>(p, p->lay.row_off), p->n_freq, franges);
    hipLaunchKernelGGL(ap_twiddle_kernel, dim3(unsigned((nw + 255) / 256)), dim3(256), 0, st, N, nw, tw);
    for (int f = 0; f < p->n_freq; ++f) {
        // w^2 dz with w = 2 pi f + i eps
        const double wr = kTwoPiD * p->freq[size_t(f)], wi = p->eps;
        const zd scale{p->dz * (wr * wr - wi * wi), p->dz * (2.0 * wr * wi)};
        if (p2)
            hipLaunchKernelGGL(ap_rows_fft_kernel<true>, dim3(blocks), dim3(256), lds, st, g64,
                               dptr<const uint32_t>(p, p->lay.rows), dptr<const int32_t>(p, p->lay.keys),
                               franges, f, p->n_freq, p->n_cls, N, logn, nz, L, scale, lo, nW, tw, R);
        else
            hipLaunchKernelGGL(ap_rows_fft_kernel<false>, dim3(blocks), dim3(256), lds, st, g64,
                               dptr<const uint32_t>(p, p->lay.rows), dptr<const int32_t>(p, p->lay.keys),
                               franges, f, p->n_freq, p->n_cls, N, logn, nz, L, scale, lo, nW, tw, R);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(ap_gram_kernel, dim3(xcd_pair_grid(P, nt * (nt + 1) / 2)), dim3(256), 0, st, R, nz, nt, nW,
                           1.0 / double(N), f == 0 ? 1 : 0, gram, P);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(ap_trace_kernel, dim3(unsigned(P)), dim3(256), 0, st, gram, nz, trace);
    return hipGetLastError();
}

}  // namespace edt
