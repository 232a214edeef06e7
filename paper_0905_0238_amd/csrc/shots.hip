// The transforms on either side of the decoupled problems (paper Section
// 2.1): shot records of the 2D line survey to the packed wavenumber-domain
// rows, and the solution spectrum V~ to the model V(x, z).
//
// Both are batches of 1D discrete Fourier transforms along one axis of a
// dense array, done one line (or a few adjacent lines) per block in LDS:
// decimation in time from bit-reversed loads for a power-of-two length (three
// radix-2 levels per pass over LDS, in registers), a direct sum over an exact
// twiddle table otherwise.  Twiddles are
// sincospi(2k/n) (exact angle reduction), so the transform is accurate to a
// few units of rounding times log2(n).  The data are streamed through HBM
// once per axis; the lines of an axis with unit stride between neighbours are
// loaded several at a time so that each load covers contiguous memory.

#include "dev_common.h"
#include "lines.h"

namespace edt {

constexpr size_t kLineLds = 80 * 1024;   // LDS of one block, values and twiddles (gfx950: 160 KiB per CU)

template <bool POW2>
__global__ __launch_bounds__(256) void dft_lines_kernel(zd* __restrict__ data, int n, int logn, Lines g, int L,
                                                        double sign, double scale) {
    extern __shared__ zd s_mem[];
    const int ns = lds_stride(n);
    zd* s_x = s_mem;            // L lines of n values (padded layout)
    zd* s_w = s_mem + L * ns;   // twiddles: n / 2 (radix 2) or n (direct)
    const int tid = threadIdx.x;
    const int64_t l0 = int64_t(blockIdx.x) * L;
    const int64_t base0 = (l0 / g.per_slab) * g.slab + (l0 % g.per_slab) * g.step;
    const bool adjacent = g.step == 1;
    const int nw = POW2 ? n / 2 : n;
    for (int k = tid; k < nw; k += 256) {
        double sv, cv;
        sincospi(2.0 * double(k) / double(n), &sv, &cv);
        s_w[k] = zd{cv, sign * sv};
    }
    auto line_of = [&](int e) { return adjacent ? e % L : e / n; };
    auto elem_of = [&](int e) { return adjacent ? e / L : e % n; };
    for (int e = tid; e < L * n; e += 256) {
        const int j = line_of(e), i = elem_of(e);
        const zd v = data[base0 + int64_t(j) * g.step + int64_t(i) * g.stride];
        int at = i;
        if constexpr (POW2) at = bit_reverse(i, logn);
        s_x[j * ns + lds_pad(at)] = v;
    }
    __syncthreads();
    if constexpr (POW2) {
        dit_lines(s_x, s_w, n, logn, L);
        for (int e = tid; e < L * n; e += 256) {
            const int j = line_of(e), i = elem_of(e);
            data[base0 + int64_t(j) * g.step + int64_t(i) * g.stride] = scale * s_x[j * ns + lds_pad(i)];
        }
    } else {
        // every line is in LDS before the first store
        for (int e = tid; e < L * n; e += 256) {
            const int j = line_of(e), k = elem_of(e);
            zd acc{0.0, 0.0};
            int m = 0;   // (k i) mod n
            for (int i = 0; i < n; ++i) {
                acc = acc + s_w[m] * s_x[j * ns + lds_pad(i)];
                m += k;
                if (m >= n) m -= n;
            }
            data[base0 + int64_t(j) * g.step + int64_t(k) * g.stride] = scale * acc;
        }
    }
}

// d_rows[r] = (F[f][a][b], F[f][-b][-a]) for the row's frequency f and key
// (a, b): the datum at +k_m and its -k_m partner (in the plan's data type).
template <class D>
__global__ __launch_bounds__(256) void rows_gather_kernel(const zd* __restrict__ F, const uint32_t* __restrict__ rows,
                                                          const int32_t* __restrict__ keys, int64_t n_rows, int N,
                                                          D* __restrict__ d_rows) {
    const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (r >= n_rows) return;
    const int64_t f = rows[2 * r];
    const int a = keys[2 * r], b = keys[2 * r + 1];
    const int a1 = b ? N - b : 0, b1 = a ? N - a : 0;
    const int64_t base = f * N * N;
    store_datum(d_rows, 2 * r, F[base + int64_t(a) * N + b]);
    store_datum(d_rows, 2 * r + 1, F[base + int64_t(a1) * N + b1]);
}

__global__ __launch_bounds__(256) void real_part_kernel(const zd* __restrict__ v, int64_t n, double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) out[i] = v[i].x;
}

// ------------------------------------------------------------- launchers ---
namespace {
bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
}  // namespace

// One batch of transforms of length n over n_slabs * g.per_slab lines.
hipError_t launch_lines(zd* data, int n, int64_t n_slabs, Lines g, double sign, double scale, hipStream_t st) {
    if (n < 1 || n > kMaxLine) return hipErrorInvalidValue;
    const bool p2 = is_pow2(n);
    const int nw = p2 ? n / 2 : n;
    // (8 adjacent lines, for 128-byte loads, measured slower: the larger
    // LDS footprint halves the blocks per CU)
    int L = 1;
    for (int c : {4, 2}) {
        if (g.per_slab % c == 0 && size_t(c * lds_stride(n) + nw) * sizeof(zd) <= kLineLds) {
            L = c;
            break;
        }
    }
    const size_t lds = size_t(L * lds_stride(n) + nw) * sizeof(zd);
    if (lds > kLineLds) return hipErrorInvalidValue;
    int logn = 0;
    while ((1 << logn) < n) ++logn;
    const int64_t blocks = n_slabs * (g.per_slab / L);
    if (blocks <= 0) return hipSuccess;
    if (p2)
        hipLaunchKernelGGL(dft_lines_kernel<true>, dim3(unsigned(blocks)), dim3(256), lds, st, data, n, logn, g, L,
                           sign, scale);
    else
        hipLaunchKernelGGL(dft_lines_kernel<false>, dim3(unsigned(blocks)), dim3(256), lds, st, data, n, logn, g,
                           L, sign, scale);
    return hipGetLastError();
}

hipError_t configure_lines() {
    for (const void* k : {reinterpret_cast<const void*>(dft_lines_kernel<true>),
                          reinterpret_cast<const void*>(dft_lines_kernel<false>)}) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(kLineLds));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// shots[f][R][S] <- dx * DFT over R and S (forward sign).
hipError_t launch_shots_fft(const edt_plan* p, zd* shots, hipStream_t st) {
    const int N = p->n_mid;
    const int64_t NN = int64_t(N) * N;
    hipError_t e = launch_lines(shots, N, p->n_freq, Lines{NN, N, 1, N}, -1.0, 1.0, st);   // along S
    if (e != hipSuccess) return e;
    return launch_lines(shots, N, p->n_freq, Lines{NN, 1, N, N}, -1.0, p->d_mid, st);        // along R
}

hipError_t launch_shots_pack(const edt_plan* p, const zd* F, void* d_rows, hipStream_t st) {
    if (p->n_rows == 0) return hipSuccess;
    const unsigned blocks = unsigned((p->n_rows + 255) / 256);
    if (p->data_c64)
        hipLaunchKernelGGL(rows_gather_kernel<float2>, dim3(blocks), dim3(256), 0, st, F,
                           dptr<const uint32_t>(p, p->lay.rows), dptr<const int32_t>(p, p->lay.keys), p->n_rows,
                           p->n_mid, static_cast<float2*>(d_rows));
    else
        hipLaunchKernelGGL(rows_gather_kernel<zd>, dim3(blocks), dim3(256), 0, st, F,
                           dptr<const uint32_t>(p, p->lay.rows), dptr<const int32_t>(p, p->lay.keys), p->n_rows,
                           p->n_mid, static_cast<zd*>(d_rows));
    return hipGetLastError();
}

// v[u][z] <- inverse DFT over u (2D) or (ux, uy) (3D), scaled by 1/N per
// axis; model = its real part.
hipError_t launch_model(const edt_plan* p, zd* v, double* model, hipStream_t st) {
    const int N = p->n_mid, nz = p->nz;
    const double inv = 1.0 / double(N);
    hipError_t e;
    if (p->dim == 3) {
        const int64_t row = int64_t(N) * nz;
        e = launch_lines(v, N, N, Lines{row, 1, nz, nz}, 1.0, inv, st);                 // along uy
        if (e != hipSuccess) return e;
        e = launch_lines(v, N, 1, Lines{row * N, 1, row, int(row)}, 1.0, inv, st);     // along ux
    } else {
        e = launch_lines(v, N, 1, Lines{int64_t(N) * nz, 1, nz, nz}, 1.0, inv, st);
    }
    if (e != hipSuccess) return e;
    const int64_t n = int64_t(p->n_km) * nz;
    hipLaunchKernelGGL(real_part_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, v, n, model);
    return hipGetLastError();
}

}  // namespace edt
