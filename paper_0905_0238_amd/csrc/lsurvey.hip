// The 3D survey of parallel 2D lines (paper Section 2.2, eq. Born3D and the
// decoupled 3D equation after it): per (k_m, k_y) pair, a row (f, receiver
// index a) is the sum over the line wavenumbers q of products of Green's
// functions of the 2D horizontal wavevectors (k_a, k_q) and (k_b, k_{q-c}),
// weighted w^2 dz / L_y (the k_h'' integral on the periodic grid of lines).
//
// A row is a sum of up to n_line products, not one, so the rows of one
// frequency are formed into HBM (a chunk of pairs at a time, as many slots per
// pair as the chunk's largest row count, zero past a pair's rows) and the
// finite aperture's FP64 MFMA product accumulates Re(A^H A) over the
// frequencies; the right-hand sides Re(A^H b+-) are accumulated from the same
// rows, and the trace is the Gram's diagonal.  The rows' terms (which q are
// kept) come from the planner's per-row masks, so no cut is decided here.

#include "dev_common.h"
#include "lines.h"

namespace edt {

__device__ __forceinline__ int signed_idx(int n, int N) { return n < (N + 1) / 2 ? n : n - N; }

// Value of row r (receiver index a, source index b, term mask m) at depth z.
// The terms q and -q share the receiver factor g(|(k_a, k_q)|), so the sum
// runs over |q|: one receiver load and up to two source loads per |q|.
__device__ __forceinline__ zd line_row_value(const zd* __restrict__ gf, int a, int b, uint64_t m, int qc, int Ny,
                                             int nz, int z) {
    const int ny2 = Ny / 2 + 1, ia = abs(a), ib = abs(b), h = Ny / 2;
    auto src = [&](int q) {   // g(|(k_b, k_{q-c})|)
        int pq = (q - qc) % Ny;
        pq = signed_idx(pq < 0 ? pq + Ny : pq, Ny);
        return gf[size_t(ib * ny2 + abs(pq)) * nz + z];
    };
    zd v{0.0, 0.0};
    for (int k = 0; k <= h; ++k) {
        const bool kp = k + h < Ny && ((m >> (k + h)) & 1u);   // q = +k
        const bool kn = k > 0 && ((m >> (h - k)) & 1u);        // q = -k
        if (!kp && !kn) continue;
        zd s{0.0, 0.0};
        if (kp) s = src(k);
        if (kn) s = s + src(-k);
        v = v + gf[size_t(ia * ny2 + k) * nz + z] * s;
    }
    return v;
}

// Rows of frequency f of the pairs p0 .. p0 + gridDim.x - 1, one block per
// pair, formed compactly: Rh[p - p0][i][z] holds the pair's i-th row of the
// frequency, zero for i past its rows (nr slots per pair, the chunk's largest
// row count).
__global__ __launch_bounds__(256) void line_rows_kernel(const zd* __restrict__ g64, const int32_t* __restrict__ keys,
                                                        const uint64_t* __restrict__ lmask,
                                                        const int64_t* __restrict__ lfr,
                                                        const int32_t* __restrict__ pair_u, int f, int n_freq,
                                                        int n_cls, int Nx, int Ny, int nz, int nr, zd W, int64_t p0,
                                                        zd* __restrict__ Rh) {
    const int64_t p = p0 + blockIdx.x;
    const int64_t r0 = lfr[p * (n_freq + 1) + f], n = lfr[p * (n_freq + 1) + f + 1] - r0;
    const int qc = signed_idx(pair_u[2 * p] % Ny, Ny);
    const zd* gf = g64 + size_t(f) * n_cls * nz;
    zd* out = Rh + size_t(blockIdx.x) * nr * nz;
    for (int e = threadIdx.x; e < nr * nz; e += 256) {
        const int i = e / nz, z = e % nz;
        zd v{0.0, 0.0};
        if (i < n) {
            const int64_t r = r0 + i;
            v = W * line_row_value(gf, signed_idx(keys[2 * r], Nx), signed_idx(keys[2 * r + 1], Nx), lmask[r], qc,
                                   Ny, nz, z);
        }
        out[e] = v;
    }
}

// rhs[p][0|1][z] (first: =, else +=) Re(sum over the rows of frequency f of
// conj(A(z)) b+-), b+ = (d0 + d1)/2, b- = (d0 - d1)/(2i), from the rows
// formed compactly (nr per pair).
template <class D>
__global__ __launch_bounds__(256) void line_rhs_kernel(const zd* __restrict__ Rh, const int64_t* __restrict__ lfr,
                                                       const D* __restrict__ d_rows, int f, int n_freq, int nr, int nz,
                                                       int64_t p0, int first, double* __restrict__ rhs) {
    const int64_t p = p0 + blockIdx.x;
    const int64_t r0 = lfr[p * (n_freq + 1) + f], r1 = lfr[p * (n_freq + 1) + f + 1];
    const zd* R = Rh + size_t(blockIdx.x) * nr * nz;
    for (int z = threadIdx.x; z < nz; z += 256) {
        double cp = 0.0, cm = 0.0;
        for (int64_t r = r0; r < r1; ++r) {
            const zd A = R[size_t(r - r0) * nz + z];
            const zd d0 = load_datum(d_rows, 2 * r), d1 = load_datum(d_rows, 2 * r + 1);
            const zd bp = 0.5 * (d0 + d1);
            const zd df = d0 - d1;
            const zd bm{0.5 * df.y, -0.5 * df.x};
            cp += A.x * bp.x + A.y * bp.y;
            cm += A.x * bm.x + A.y * bm.y;
        }
        double* o = rhs + size_t(p) * 2 * nz;
        o[z] = first ? cp : o[z] + cp;
        o[nz + z] = first ? cm : o[nz + z] + cm;
    }
}

// Born forward map of the line survey: d_rows[r] = (A_r . v[u], A_r . v[u_neg]);
// one wave per row, lanes over depth.
template <class D>
__global__ __launch_bounds__(256) void line_forward_kernel(const zd* __restrict__ g64, const uint32_t* __restrict__ rows,
                                                           const int32_t* __restrict__ keys,
                                                           const uint64_t* __restrict__ lmask,
                                                           const int32_t* __restrict__ lpair,
                                                           const int32_t* __restrict__ pair_u,
                                                           const double* __restrict__ freq, double eps, double scale,
                                                           int n_cls, int Nx, int Ny, int nz, int64_t R,
                                                           const zd* __restrict__ v, D* __restrict__ d_rows) {
    const int lane = threadIdx.x & 63;
    const int64_t r = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (r >= R) return;
    const int f = int(rows[2 * r]);
    const int p = lpair[r];
    const int u0 = pair_u[2 * p], u1 = pair_u[2 * p + 1];
    const int qc = signed_idx(u0 % Ny, Ny);
    const zd* gf = g64 + size_t(f) * n_cls * nz;
    const int a = signed_idx(keys[2 * r], Nx), b = signed_idx(keys[2 * r + 1], Nx);
    const uint64_t m = lmask[r];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int z = lane; z < nz; z += 64) {
        const zd A = line_row_value(gf, a, b, m, qc, Ny, nz, z);
        const zd q0 = A * v[size_t(u0) * nz + z], q1 = A * v[size_t(u1) * nz + z];
        s0 += q0.x;
        s1 += q0.y;
        s2 += q1.x;
        s3 += q1.y;
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    s3 = wave_sum(s3);
    if (lane == 0) {
        const zd w = omega_of(freq[f], eps);
        const zd W = scale * (w * w);
        store_datum(d_rows, 2 * r, W * zd{s0, s1});
        store_datum(d_rows, 2 * r + 1, W * zd{s2, s3});
    }
}

hipError_t launch_rows_gram(const zd* R, int nz, int n_rows, double scale, int first, double* gram, int64_t P,
                            hipStream_t st);
hipError_t launch_gram_trace(const double* gram, int nz, double* trace, int64_t P, hipStream_t st);

// Row slots per pair for the run of pairs p0 .. p0 + np - 1 at frequency f:
// the largest row count among them (at least one).
int line_row_slots(const edt_plan* p, int f, int64_t p0, int64_t np) {
    int64_t nr = 1;
    for (int64_t q = p0; q < p0 + np; ++q) {
        const int64_t* fr = p->lfr.data() + size_t(q) * size_t(p->n_freq + 1);
        nr = std::max<int64_t>(nr, fr[f + 1] - fr[f]);
    }
    return int(nr);
}

// The row weight w^2 dz / L_y of frequency f.
zd line_row_weight(const edt_plan* p, int f) {
    const double Ly = double(p->n_line) * p->d_line;
    const double wr = kTwoPiD * p->freq[size_t(f)], wi = p->eps;
    return zd{p->dz * (wr * wr - wi * wi) / Ly, p->dz * (2.0 * wr * wi) / Ly};
}

// The rows of frequency f of the run of pairs p0 .. p0 + np - 1, compactly
// (nr slots per pair), into Rh.
hipError_t launch_line_rows(const edt_plan* p, const zd* g64, int f, int64_t p0, int64_t np, int nr, zd* Rh,
                            hipStream_t st) {
    hipLaunchKernelGGL(line_rows_kernel, dim3(unsigned(np)), dim3(256), 0, st, g64,
                       dptr<const int32_t>(p, p->lay.keys), dptr<const uint64_t>(p, p->lay.lmask),
                       dptr<const int64_t>(p, p->lay.lfr), dptr<const int32_t>(p, p->lay.pair_u), f, p->n_freq,
                       p->n_cls, p->n_mid, p->n_line, p->nz, nr, line_row_weight(p, f), p0, Rh);
    return hipGetLastError();
}

// FP64 Gram, right-hand sides and trace of a line survey, frequency by
// frequency over chunks of pairs (the rows of one chunk and frequency live in
// work at lrows).
hipError_t launch_line_assemble(const edt_plan* p, const zd* g64, const void* d_rows, double* gram, double* rhs,
                                double* trace, unsigned char* work, hipStream_t st) {
    const int64_t P = p->n_pairs;
    if (P == 0) return hipSuccess;
    const WorkLayout wl = work_layout(p);
    zd* Rh = reinterpret_cast<zd*>(work + wl.lrows);
    const int64_t chunk = line_chunk(p);
    const int nz = p->nz;
    for (int64_t p0 = 0; p0 < P; p0 += chunk) {
        const int64_t np = std::min<int64_t>(chunk, P - p0);
        for (int f = 0; f < p->n_freq; ++f) {
            const int nr = line_row_slots(p, f, p0, np);
            hipError_t e = launch_line_rows(p, g64, f, p0, np, nr, Rh, st);
            if (e != hipSuccess) return e;
            if ((e = launch_rows_gram(Rh, nz, nr, 1.0, f == 0, gram + size_t(p0) * nz * nz, np, st)) != hipSuccess)
                return e;
            if (p->data_c64)
                hipLaunchKernelGGL(line_rhs_kernel<float2>, dim3(unsigned(np)), dim3(256), 0, st, Rh,
                                   dptr<const int64_t>(p, p->lay.lfr), static_cast<const float2*>(d_rows), f,
                                   p->n_freq, nr, nz, p0, f == 0 ? 1 : 0, rhs);
            else
                hipLaunchKernelGGL(line_rhs_kernel<zd>, dim3(unsigned(np)), dim3(256), 0, st, Rh,
                                   dptr<const int64_t>(p, p->lay.lfr), static_cast<const zd*>(d_rows), f, p->n_freq,
                                   nr, nz, p0, f == 0 ? 1 : 0, rhs);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return launch_gram_trace(gram, nz, trace, P, st);
}

// Finite aperture on the survey of parallel lines (the sinc over the offset
// wavenumber in the decoupled 3D equation).  The window |x_R - x_S| <= 2 b
// is the same on every line, so at each pair it is the circulant of the 2D
// line over the receiver index: per chunk and frequency the rows are built
// over their receiver index in LDS, transformed there
// (Ah(o) = sum_a A(a) e^{2 pi i a o / N_x}), and only the kept offsets go to
// HBM, where the FP64 product adds (1 / N_x) Re(Ah^H Ah) over them.

void aperture_offsets(const edt_plan* p, double b_max, int* lo, int* nW);

constexpr int kLineApLds = 80 * 1024;   // LDS of one build block

// Pair p0 + blockIdx.x / (nz / L), depths z0 .. z0 + L - 1: the rows of
// frequency f placed at their receiver index (fftfreq order; zero where the
// pair has no row), transformed over it, and the kept offsets
// o = (lo + k) mod N_x stored as K[p - p0][k][z].  A power-of-two N_x takes
// the radix-2 transform, any other a direct sum for the kept offsets only.
template <bool POW2>
__global__ __launch_bounds__(256) void line_ap_rows_kernel(const zd* __restrict__ g64,
                                                           const int32_t* __restrict__ keys,
                                                           const uint64_t* __restrict__ lmask,
                                                           const int64_t* __restrict__ lfr,
                                                           const int32_t* __restrict__ pair_u, int f, int n_freq,
                                                           int n_cls, int Nx, int logn, int Ny, int nz, int L, zd W,
                                                           int64_t p0, int lo, int nW, zd* __restrict__ K) {
    extern __shared__ zd s_mem[];
    const int ns = lds_stride(Nx);
    zd* s_x = s_mem;            // L lines of Nx values (padded layout)
    zd* s_w = s_mem + L * ns;   // twiddles e^{2 pi i k / Nx}: Nx / 2 (radix 2) or Nx (direct)
    const int tid = threadIdx.x;
    const int per_pair = nz / L;
    const int64_t pl = blockIdx.x / unsigned(per_pair), p = p0 + pl;
    const int z0 = int(blockIdx.x % unsigned(per_pair)) * L;
    const int nw = POW2 ? Nx / 2 : Nx;
    for (int k = tid; k < nw; k += 256) {
        double sv, cv;
        sincospi(2.0 * double(k) / double(Nx), &sv, &cv);
        s_w[k] = zd{cv, sv};
    }
    for (int e = tid; e < L * ns; e += 256) s_x[e] = zd{0.0, 0.0};
    const int64_t r0 = lfr[p * (n_freq + 1) + f], n = lfr[p * (n_freq + 1) + f + 1] - r0;
    const int qc = signed_idx(pair_u[2 * p] % Ny, Ny);
    const zd* gf = g64 + size_t(f) * n_cls * nz;
    __syncthreads();
    for (int64_t e = tid; e < n * L; e += 256) {
        const int64_t r = r0 + e / L;
        const int j = int(e % L), z = z0 + j;
        const int a = keys[2 * r];
        const zd v = W * line_row_value(gf, signed_idx(a, Nx), signed_idx(keys[2 * r + 1], Nx), lmask[r], qc, Ny,
                                        nz, z);
        s_x[j * ns + lds_pad(POW2 ? bit_reverse(a, logn) : a)] = v;
    }
    __syncthreads();
    zd* Kp = K + size_t(pl) * nW * nz;
    if constexpr (POW2) {
        dit_lines(s_x, s_w, Nx, logn, L);
        for (int e = tid; e < L * nW; e += 256) {
            const int j = e % L, k = e / L;
            int o = (lo + k) % Nx;
            if (o < 0) o += Nx;
            Kp[size_t(k) * nz + z0 + j] = s_x[j * ns + lds_pad(o)];
        }
    } else {
        for (int e = tid; e < L * nW; e += 256) {
            const int j = e % L, k = e / L;
            int o = (lo + k) % Nx;
            if (o < 0) o += Nx;
            zd acc{0.0, 0.0};
            int m = 0;   // (a o) mod Nx
            for (int a = 0; a < Nx; ++a) {
                acc = acc + s_w[m] * s_x[j * ns + lds_pad(a)];
                m += o;
                if (m >= Nx) m -= Nx;
            }
            Kp[size_t(k) * nz + z0 + j] = acc;
        }
    }
}

hipError_t configure_line_aperture() {
    for (const void* k : {reinterpret_cast<const void*>(line_ap_rows_kernel<true>),
                          reinterpret_cast<const void*>(line_ap_rows_kernel<false>)}) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kLineApLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Work: the kept offsets of one chunk and frequency.
size_t line_aperture_work_bytes(const edt_plan* p) {
    const size_t kept = (size_t(line_chunk(p)) * p->n_mid * p->nz * sizeof(zd) + 255) & ~size_t(255);
    return std::max<size_t>(256, kept);
}

hipError_t launch_line_aperture_gram(const edt_plan* p, const zd* g64, double b_max, double* gram, double* trace,
                                     unsigned char* work, hipStream_t st) {
    const int64_t P = p->n_pairs;
    if (P == 0) return hipSuccess;
    const int64_t chunk = line_chunk(p);
    const int Nx = p->n_mid, Ny = p->n_line, nz = p->nz;
    zd* K = reinterpret_cast<zd*>(work);
    int lo = 0, nW = 0;
    aperture_offsets(p, b_max, &lo, &nW);
    const bool p2 = (Nx & (Nx - 1)) == 0;
    const int nw = p2 ? Nx / 2 : Nx;
    int logn = 0;
    while ((1 << logn) < Nx) ++logn;
    // depths per block: 4 adjacent ones when they fit (contiguous stores)
    int L = 1;
    for (int c : {4, 2})
        if (nz % c == 0 && size_t(c * lds_stride(Nx) + nw) * sizeof(zd) <= kLineApLds) {
            L = c;
            break;
        }
    const size_t lds = size_t(L * lds_stride(Nx) + nw) * sizeof(zd);
    if (lds > kLineApLds) return hipErrorInvalidValue;
    const double Ly = double(Ny) * p->d_line;
    for (int64_t p0 = 0; p0 < P; p0 += chunk) {
        const int64_t np = std::min<int64_t>(chunk, P - p0);
        const unsigned blocks = unsigned(np * (nz / L));
        for (int f = 0; f < p->n_freq; ++f) {
            const double wr = kTwoPiD * p->freq[size_t(f)], wi = p->eps;
            const zd W{p->dz * (wr * wr - wi * wi) / Ly, p->dz * (2.0 * wr * wi) / Ly};
            if (p2)
                hipLaunchKernelGGL(line_ap_rows_kernel<true>, dim3(blocks), dim3(256), lds, st, g64,
                                   dptr<const int32_t>(p, p->lay.keys), dptr<const uint64_t>(p, p->lay.lmask),
                                   dptr<const int64_t>(p, p->lay.lfr), dptr<const int32_t>(p, p->lay.pair_u), f,
                                   p->n_freq, p->n_cls, Nx, logn, Ny, nz, L, W, p0, lo, nW, K);
            else
                hipLaunchKernelGGL(line_ap_rows_kernel<false>, dim3(blocks), dim3(256), lds, st, g64,
                                   dptr<const int32_t>(p, p->lay.keys), dptr<const uint64_t>(p, p->lay.lmask),
                                   dptr<const int64_t>(p, p->lay.lfr), dptr<const int32_t>(p, p->lay.pair_u), f,
                                   p->n_freq, p->n_cls, Nx, logn, Ny, nz, L, W, p0, lo, nW, K);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            if ((e = launch_rows_gram(K, nz, nW, 1.0 / double(Nx), f == 0, gram + size_t(p0) * nz * nz, np, st)) !=
                hipSuccess)
                return e;
        }
    }
    return launch_gram_trace(gram, nz, trace, P, st);
}

hipError_t launch_line_forward(const edt_plan* p, const zd* g64, const zd* v, void* d_rows, hipStream_t st) {
    const int64_t R = p->n_rows;
    if (R == 0) return hipSuccess;
    const double scale = p->dz / (double(p->n_line) * p->d_line);
    const dim3 grid(unsigned((R + 3) / 4));
    if (p->data_c64)
        hipLaunchKernelGGL(line_forward_kernel<float2>, grid, dim3(256), 0, st, g64, dptr<const uint32_t>(p, p->lay.rows),
                           dptr<const int32_t>(p, p->lay.keys), dptr<const uint64_t>(p, p->lay.lmask),
                           dptr<const int32_t>(p, p->lay.lpair), dptr<const int32_t>(p, p->lay.pair_u),
                           dptr<const double>(p, p->lay.freq), p->eps, scale, p->n_cls, p->n_mid, p->n_line, p->nz,
                           R, v, static_cast<float2*>(d_rows));
    else
        hipLaunchKernelGGL(line_forward_kernel<zd>, grid, dim3(256), 0, st, g64, dptr<const uint32_t>(p, p->lay.rows),
                           dptr<const int32_t>(p, p->lay.keys), dptr<const uint64_t>(p, p->lay.lmask),
                           dptr<const int32_t>(p, p->lay.lpair), dptr<const int32_t>(p, p->lay.pair_u),
                           dptr<const double>(p, p->lay.freq), p->eps, scale, p->n_cls, p->n_mid, p->n_line, p->nz,
                           R, v, static_cast<zd*>(d_rows));
    return hipGetLastError();
}

}  // namespace edt
