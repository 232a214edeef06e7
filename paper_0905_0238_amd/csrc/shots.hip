// The transforms on either side of the decoupled problems (paper Section
// 2.1): shot records to the packed wavenumber-domain rows, and the solution
// spectrum V~ to the model V(x, z).  The records are those of the 2D line
// survey, [f][R][S], of the 3D areal survey (Section 2.2) on the doubled
// periodic 2N x 2N grid, [f][Rx][Ry][Sx][Sy] (a row's receiver and source
// wavenumbers q +- 2n, in units of dk/2, are half-grid wavenumbers of the N
// grid and whole-grid ones of a survey of twice the period), or of the 3D
// survey of parallel lines, [f][line][R][S].
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
                                                        int64_t line0, double sign, double scale) {
    extern __shared__ zd s_mem[];
    const int ns = lds_stride(n);
    zd* s_x = s_mem;            // L lines of n values (padded layout)
    zd* s_w = s_mem + L * ns;   // twiddles: n / 2 (radix 2) or n (direct)
    const int tid = threadIdx.x;
    const int64_t l0 = line0 + int64_t(blockIdx.x) * L;
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

// 3D areal: one block per pair, k_m index q = (qx, qy) (signed); row r with
// frequency f and k_h index n = (nx, ny) reads the doubled survey's spectrum
// F[f][a][b] at a = q + 2n, b = q - 2n (mod M = 2N per axis), and the -k_m
// partner at (-b, -a); both are 4 times the row's data (the N-periodic model
// has on the 2N grid a spectrum at even indices only, 4 times its own).
template <class D>
__global__ __launch_bounds__(256) void rows_gather_areal_kernel(const zd* __restrict__ F,
                                                                const uint32_t* __restrict__ rows,
                                                                const int32_t* __restrict__ keys,
                                                                const int64_t* __restrict__ row_off,
                                                                const int32_t* __restrict__ pair_u, int N, int Nh,
                                                                D* __restrict__ d_rows) {
    const int64_t pq = blockIdx.x;
    const int u = pair_u[2 * pq];
    const int ux = u / N, uy = u % N;
    const int qx = ux < (N + 1) / 2 ? ux : ux - N, qy = uy < (N + 1) / 2 ? uy : uy - N;
    const int M = 2 * N;
    const int64_t M2 = int64_t(M) * M;
    auto wrap = [M](int v) { return ((v % M) + M) % M; };
    auto at = [&](int64_t f, int ax, int ay, int bx, int by) {
        return f * M2 * M2 + (int64_t(ax) * M + ay) * M2 + int64_t(bx) * M + by;
    };
    const int nlo = Nh / 2;
    for (int64_t r = row_off[pq] + threadIdx.x; r < row_off[pq + 1]; r += 256) {
        const int64_t f = rows[2 * r];
        const int n = keys[2 * r];
        const int nx = n / Nh - nlo, ny = n % Nh - nlo;
        const int ax = wrap(qx + 2 * nx), ay = wrap(qy + 2 * ny);
        const int bx = wrap(qx - 2 * nx), by = wrap(qy - 2 * ny);
        store_datum(d_rows, 2 * r, 0.25 * F[at(f, ax, ay, bx, by)]);
        store_datum(d_rows, 2 * r + 1, 0.25 * F[at(f, wrap(-bx), wrap(-by), wrap(-ax), wrap(-ay))]);
    }
}

// 3D survey of parallel lines: one block per pair (flattened k = ux N_y + c);
// row r with frequency f and key (a, b) reads F[f][c][a][b] and its -k
// partner F[f][-c][-b][-a].
template <class D>
__global__ __launch_bounds__(256) void rows_gather_lines_kernel(const zd* __restrict__ F,
                                                                const uint32_t* __restrict__ rows,
                                                                const int32_t* __restrict__ keys,
                                                                const int64_t* __restrict__ row_off,
                                                                const int32_t* __restrict__ pair_u, int N, int Ny,
                                                                D* __restrict__ d_rows) {
    const int64_t pq = blockIdx.x;
    const int c = pair_u[2 * pq] % Ny, c1 = c ? Ny - c : 0;
    const int64_t NN = int64_t(N) * N;
    for (int64_t r = row_off[pq] + threadIdx.x; r < row_off[pq + 1]; r += 256) {
        const int64_t f = rows[2 * r];
        const int a = keys[2 * r], b = keys[2 * r + 1];
        const int a1 = b ? N - b : 0, b1 = a ? N - a : 0;
        store_datum(d_rows, 2 * r, F[(f * Ny + c) * NN + int64_t(a) * N + b]);
        store_datum(d_rows, 2 * r + 1, F[(f * Ny + c1) * NN + int64_t(a1) * N + b1]);
    }
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
    // A grid holds fewer than 2^32 work-items: a large batch is launched in
    // runs of blocks (each block's L lines lie in one slab).
    const int64_t blocks = n_slabs * (g.per_slab / L);
    for (int64_t b0 = 0; b0 < blocks; b0 += kMaxLineBlocks) {
        const unsigned nb = unsigned(std::min(kMaxLineBlocks, blocks - b0));
        if (p2)
            hipLaunchKernelGGL(dft_lines_kernel<true>, dim3(nb), dim3(256), lds, st, data, n, logn, g, L, b0 * L,
                               sign, scale);
        else
            hipLaunchKernelGGL(dft_lines_kernel<false>, dim3(nb), dim3(256), lds, st, data, n, logn, g, L, b0 * L,
                               sign, scale);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t configure_lines() {
    for (const void* k : {reinterpret_cast<const void*>(dft_lines_kernel<true>),
                          reinterpret_cast<const void*>(dft_lines_kernel<false>)}) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(kLineLds));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// shots[f][R][S] <- dx * DFT over R and S (forward sign); 3D areal:
// shots[f][Rx][Ry][Sx][Sy] (M = 2N per axis) <- dx^2 * DFT over all four;
// parallel lines: shots[f][line][R][S] <- dx * DFT over R, S and the line.
hipError_t launch_shots_fft(const edt_plan* p, zd* shots, hipStream_t st) {
    const int N = p->n_mid;
    if (p->n_line > 0) {
        const int Ny = p->n_line;
        const int64_t NN = int64_t(N) * N, nl = int64_t(p->n_freq) * Ny;
        hipError_t e = launch_lines(shots, N, nl, Lines{NN, N, 1, N}, -1.0, 1.0, st);   // along S
        if (e == hipSuccess)   // along R (a single line takes the scale here)
            e = launch_lines(shots, N, nl, Lines{NN, 1, N, N}, -1.0, Ny == 1 ? p->d_mid : 1.0, st);
        if (e == hipSuccess && Ny > 1)   // along the line index
            e = launch_lines(shots, Ny, p->n_freq, Lines{NN * Ny, 1, NN, int(NN)}, -1.0, p->d_mid, st);
        return e;
    }
    if (p->dim == 3) {
        const int M = 2 * N;
        const int64_t M2 = int64_t(M) * M, M3 = M2 * M, nf = p->n_freq;
        hipError_t e = launch_lines(shots, M, nf * M2, Lines{M2, M, 1, M}, -1.0, 1.0, st);   // along Sy
        if (e == hipSuccess) e = launch_lines(shots, M, nf * M2, Lines{M2, 1, M, M}, -1.0, 1.0, st);   // Sx
        if (e == hipSuccess) e = launch_lines(shots, M, nf * M, Lines{M3, 1, M2, int(M2)}, -1.0, 1.0, st);   // Ry
        if (e == hipSuccess)
            e = launch_lines(shots, M, nf, Lines{M3 * M, 1, M3, int(M3)}, -1.0, p->d_mid * p->d_mid, st);   // Rx
        return e;
    }
    const int64_t NN = int64_t(N) * N;
    hipError_t e = launch_lines(shots, N, p->n_freq, Lines{NN, N, 1, N}, -1.0, 1.0, st);   // along S
    if (e != hipSuccess) return e;
    return launch_lines(shots, N, p->n_freq, Lines{NN, 1, N, N}, -1.0, p->d_mid, st);        // along R
}

hipError_t launch_shots_pack(const edt_plan* p, const zd* F, void* d_rows, hipStream_t st) {
    if (p->n_rows == 0) return hipSuccess;
    if (p->n_line > 0) {
        const unsigned np = unsigned(p->n_pairs);
        if (p->data_c64)
            hipLaunchKernelGGL(rows_gather_lines_kernel<float2>, dim3(np), dim3(256), 0, st, F,
                               dptr<const uint32_t>(p, p->lay.rows), dptr<const int32_t>(p, p->lay.keys),
                               dptr<const int64_t>(p, p->lay.row_off), dptr<const int32_t>(p, p->lay.pair_u),
                               p->n_mid, p->n_line, static_cast<float2*>(d_rows));
        else
            hipLaunchKernelGGL(rows_gather_lines_kernel<zd>, dim3(np), dim3(256), 0, st, F,
                               dptr<const uint32_t>(p, p->lay.rows), dptr<const int32_t>(p, p->lay.keys),
                               dptr<const int64_t>(p, p->lay.row_off), dptr<const int32_t>(p, p->lay.pair_u),
                               p->n_mid, p->n_line, static_cast<zd*>(d_rows));
        return hipGetLastError();
    }
    if (p->dim == 3) {
        const unsigned np = unsigned(p->n_pairs);
        if (p->data_c64)
            hipLaunchKernelGGL(rows_gather_areal_kernel<float2>, dim3(np), dim3(256), 0, st, F,
                               dptr<const uint32_t>(p, p->lay.rows), dptr<const int32_t>(p, p->lay.keys),
                               dptr<const int64_t>(p, p->lay.row_off), dptr<const int32_t>(p, p->lay.pair_u),
                               p->n_mid, p->n_off, static_cast<float2*>(d_rows));
        else
            hipLaunchKernelGGL(rows_gather_areal_kernel<zd>, dim3(np), dim3(256), 0, st, F,
                               dptr<const uint32_t>(p, p->lay.rows), dptr<const int32_t>(p, p->lay.keys),
                               dptr<const int64_t>(p, p->lay.row_off), dptr<const int32_t>(p, p->lay.pair_u),
                               p->n_mid, p->n_off, static_cast<zd*>(d_rows));
        return hipGetLastError();
    }
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

// v[u][z] <- inverse DFT over u (2D), (ux, uy) (3D areal) or (ux, c)
// (parallel lines, u = ux N_y + c), scaled by 1/length per axis; model = its
// real part.
hipError_t launch_model(const edt_plan* p, zd* v, double* model, hipStream_t st) {
    const int N = p->n_mid, nz = p->nz;
    const double inv = 1.0 / double(N);
    hipError_t e = hipSuccess;
    if (p->n_line > 0) {
        const int Ny = p->n_line;
        const int64_t row = int64_t(Ny) * nz;
        if (Ny > 1) e = launch_lines(v, Ny, N, Lines{row, 1, nz, nz}, 1.0, 1.0 / double(Ny), st);   // along c
        if (e != hipSuccess) return e;
        e = launch_lines(v, N, 1, Lines{row * N, 1, row, int(row)}, 1.0, inv, st);                // along ux
    } else if (p->dim == 3) {
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
