// Kernel (b): fused Born-row build + Gram matrix on MFMA.
//
// Paper, Section 2.1, eqs. M and Split: per +-k_m pair the least-squares
// normal matrix of the real unknowns is G = Re(A^H A) = Ah^T Ah with
// Ah = [Re A; Im A] and Born rows A = w^2 dz g(k_r) g(k_s).  The phase of w^2
// cancels in A^H A, so a row is built as P = s g(k_r) g(k_s) with the real
// scale s = |w^2 dz| (folded into the FP32 table, or applied here for FP64),
// times sqrt(mult) for a row that stands for `mult` identical data rows.
//
// A work item is a chunk of one pair's rows.  A 256- (512-) thread workgroup
// builds 8 complex rows (16 real rows of Ah) per stage straight from the
// Green's tables into LDS (double-buffered), and its waves feed them to MFMA
// for the whole lower triangle of the nz x nz Gram, which stays in registers
// across the chunk; A is never written to memory.  Each item stores its
// partial Gram tile by tile; a second kernel sums the items of a pair in FP64
// in a fixed order (deterministic).
//
// Precisions:
//   BF16X3: v_mfma_f32_32x32x16_bf16, each value split x = hi + lo (bf16) and
//           Ah^T Ah ~ hi^T hi + hi^T lo + lo^T hi with FP32 accumulation;
//   FP32:   v_mfma_f32_32x32x2_f32;
//   FP64:   v_mfma_f64_16x16x4_f64 on FP64 rows built from the FP64 table.

#include "dev_common.h"

namespace edt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// lower-triangular tile t -> (I, J), I >= J, row-major
__host__ __device__ constexpr int tri_I(int t) {
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    return I;
}
__host__ __device__ constexpr int tri_J(int t) { return t - tri_I(t) * (tri_I(t) + 1) / 2; }

// blocks touched by tiles [t0, t1)
__host__ __device__ constexpr uint32_t block_mask(int t0, int t1) {
    uint32_t m = 0;
    for (int t = t0; t < t1; ++t) m |= (1u << tri_I(t)) | (1u << tri_J(t));
    return m;
}

__device__ __forceinline__ uint32_t pack_bf16x2(__bf16 a, __bf16 b) {
    const uint16_t ua = __builtin_bit_cast(uint16_t, a), ub = __builtin_bit_cast(uint16_t, b);
    return uint32_t(ua) | (uint32_t(ub) << 16);
}

// ---------------------------------------------------------------- BF16x3 ---
template <int NT>
struct Bf16Cfg {
    static constexpr int NZP = 32 * NT;
    static constexpr int NTL = NT * (NT + 1) / 2;
    static constexpr int TPW = (NTL + 3) / 4;
    static constexpr int STR = 24;   // bf16 per LDS z-row: 16 real rows + 8 pad (48 B)
    static constexpr int EPT = NT;   // (8 complex rows x NZP) / 256 threads
};

template <int NT, int W>
__device__ __forceinline__ void bf16_wave_mfma(f32x16 (&acc)[Bf16Cfg<NT>::TPW], const __bf16* hi,
                                               const __bf16* lo, int lane) {
    using C = Bf16Cfg<NT>;
    constexpr int t0 = W * C::TPW;
    constexpr int t1 = (t0 + C::TPW < C::NTL) ? t0 + C::TPW : C::NTL;
    constexpr uint32_t need = t0 < t1 ? block_mask(t0, t1) : 0u;
    bf16x8 fh[NT], fl[NT];
    const int roff = (lane & 31) * C::STR + (lane >> 5) * 8;
#pragma unroll
    for (int b = 0; b < NT; ++b) {
        if (need & (1u << b)) {
            fh[b] = *reinterpret_cast<const bf16x8*>(hi + b * 32 * C::STR + roff);
            fl[b] = *reinterpret_cast<const bf16x8*>(lo + b * 32 * C::STR + roff);
        }
    }
#pragma unroll
    for (int m = 0; m < C::TPW; ++m) {
        const int t = t0 + m;
        if (t < t1) {
            const int I = tri_I(t), J = tri_J(t);
            acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh[I], fh[J], acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh[I], fl[J], acc[m], 0, 0, 0);
            acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fl[I], fh[J], acc[m], 0, 0, 0);
        }
    }
}

template <int NT, int W>
__device__ __forceinline__ void f32_store_tiles(const f32x16 (&acc)[Bf16Cfg<NT>::TPW], float* out,
                                                int lane) {
    using C = Bf16Cfg<NT>;
    constexpr int t0 = W * C::TPW;
#pragma unroll
    for (int m = 0; m < C::TPW; ++m) {
        const int t = t0 + m;
        if (t < C::NTL) {
            float* o = out + size_t(t) * 1024;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                o[i * 32 + (lane & 31)] = acc[m][v];
            }
        }
    }
}

template <int NT>
__global__ __launch_bounds__(256, 1) void gram_bf16x3_kernel(const uint32_t* __restrict__ urows,
                                                             const Item* __restrict__ items,
                                                             const int32_t* __restrict__ sched,
                                                             const float2* __restrict__ g32, int ncls,
                                                             int nz, float* __restrict__ part) {
    using C = Bf16Cfg<NT>;
    __shared__ __attribute__((aligned(16))) __bf16 sh[2][2][C::NZP * C::STR];
    const Item it = items[sched[blockIdx.x]];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = it.row_end - it.row_begin;
    const int nst = (n + 7) >> 3;
    f32x16 acc[C::TPW];
#pragma unroll
    for (int m = 0; m < C::TPW; ++m)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[m][v] = 0.0f;

    float2 ga[C::EPT], gb[C::EPT];
    float sw[C::EPT];
    auto load = [&](int s) {
#pragma unroll
        for (int e = 0; e < C::EPT; ++e) {
            const int idx = tid + 256 * e;
            const int j = idx / C::NZP, z = idx - j * C::NZP;
            const int r = s * 8 + j;
            ga[e] = make_float2(0.f, 0.f);
            gb[e] = make_float2(0.f, 0.f);
            sw[e] = 0.f;
            if (r < n && z < nz) {
                const URow u = load_urow(urows, int64_t(it.row_begin) + r);
                const int64_t fb = int64_t(u.f) * ncls;
                ga[e] = g32[(fb + u.cr) * nz + z];
                gb[e] = g32[(fb + u.cs) * nz + z];
                sw[e] = sqrtf(float(u.mult));
            }
        }
    };
    auto store = [&](int buf) {
        __bf16* hi = sh[buf][0];
        __bf16* lo = sh[buf][1];
#pragma unroll
        for (int e = 0; e < C::EPT; ++e) {
            const int idx = tid + 256 * e;
            const int j = idx / C::NZP, z = idx - j * C::NZP;
            const float pr = sw[e] * (ga[e].x * gb[e].x - ga[e].y * gb[e].y);
            const float pi = sw[e] * (ga[e].x * gb[e].y + ga[e].y * gb[e].x);
            const __bf16 hr = __bf16(pr), hm = __bf16(pi);
            const __bf16 lr = __bf16(pr - float(hr)), lm = __bf16(pi - float(hm));
            *reinterpret_cast<uint32_t*>(hi + z * C::STR + 2 * j) = pack_bf16x2(hr, hm);
            *reinterpret_cast<uint32_t*>(lo + z * C::STR + 2 * j) = pack_bf16x2(lr, lm);
        }
    };
    auto compute = [&](int buf) {
        const __bf16* hi = sh[buf][0];
        const __bf16* lo = sh[buf][1];
        if (wv == 0) bf16_wave_mfma<NT, 0>(acc, hi, lo, lane);
        else if (wv == 1) bf16_wave_mfma<NT, 1>(acc, hi, lo, lane);
        else if (wv == 2) bf16_wave_mfma<NT, 2>(acc, hi, lo, lane);
        else bf16_wave_mfma<NT, 3>(acc, hi, lo, lane);
    };

    load(0);
    store(0);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        if (s + 1 < nst) load(s + 1);
        compute(s & 1);
        if (s + 1 < nst) store((s + 1) & 1);
        __syncthreads();
    }
    float* out = part + size_t(it.slot) * C::NTL * 1024;
    if (wv == 0) f32_store_tiles<NT, 0>(acc, out, lane);
    else if (wv == 1) f32_store_tiles<NT, 1>(acc, out, lane);
    else if (wv == 2) f32_store_tiles<NT, 2>(acc, out, lane);
    else f32_store_tiles<NT, 3>(acc, out, lane);
}

// ------------------------------------------------------------------ FP32 ---
template <int NT>
struct F32Cfg {
    static constexpr int NZP = 32 * NT;
    static constexpr int NTL = NT * (NT + 1) / 2;
    static constexpr int TPW = (NTL + 3) / 4;
    static constexpr int STR = 20;   // floats per LDS z-row: [h][8] + 4 pad (80 B)
    static constexpr int EPT = NT;
};

template <int NT, int W>
__device__ __forceinline__ void f32_wave_mfma(f32x16 (&acc)[F32Cfg<NT>::TPW], const float* sh,
                                              int lane) {
    using C = F32Cfg<NT>;
    constexpr int t0 = W * C::TPW;
    constexpr int t1 = (t0 + C::TPW < C::NTL) ? t0 + C::TPW : C::NTL;
    constexpr uint32_t need = t0 < t1 ? block_mask(t0, t1) : 0u;
    float4 fa[NT][2];
    const int roff = (lane & 31) * C::STR + (lane >> 5) * 8;
#pragma unroll
    for (int b = 0; b < NT; ++b) {
        if (need & (1u << b)) {
            fa[b][0] = *reinterpret_cast<const float4*>(sh + b * 32 * C::STR + roff);
            fa[b][1] = *reinterpret_cast<const float4*>(sh + b * 32 * C::STR + roff + 4);
        }
    }
#pragma unroll
    for (int m = 0; m < C::TPW; ++m) {
        const int t = t0 + m;
        if (t < t1) {
            const int I = tri_I(t), J = tri_J(t);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const float a = (s < 4) ? fa[I][0][s] : fa[I][1][s - 4];
                const float b = (s < 4) ? fa[J][0][s] : fa[J][1][s - 4];
                acc[m] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[m], 0, 0, 0);
            }
        }
    }
}

template <int NT>
__global__ __launch_bounds__(256, 1) void gram_f32_kernel(const uint32_t* __restrict__ urows,
                                                          const Item* __restrict__ items,
                                                          const int32_t* __restrict__ sched,
                                                          const float2* __restrict__ g32, int ncls,
                                                          int nz, float* __restrict__ part) {
    using C = F32Cfg<NT>;
    __shared__ __attribute__((aligned(16))) float sh[2][C::NZP * C::STR];
    const Item it = items[sched[blockIdx.x]];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = it.row_end - it.row_begin;
    const int nst = (n + 7) >> 3;
    f32x16 acc[C::TPW];
#pragma unroll
    for (int m = 0; m < C::TPW; ++m)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[m][v] = 0.0f;
    float2 ga[C::EPT], gb[C::EPT];
    float sw[C::EPT];
    auto load = [&](int s) {
#pragma unroll
        for (int e = 0; e < C::EPT; ++e) {
            const int idx = tid + 256 * e;
            const int j = idx / C::NZP, z = idx - j * C::NZP;
            const int r = s * 8 + j;
            ga[e] = make_float2(0.f, 0.f);
            gb[e] = make_float2(0.f, 0.f);
            sw[e] = 0.f;
            if (r < n && z < nz) {
                const URow u = load_urow(urows, int64_t(it.row_begin) + r);
                const int64_t fb = int64_t(u.f) * ncls;
                ga[e] = g32[(fb + u.cr) * nz + z];
                gb[e] = g32[(fb + u.cs) * nz + z];
                sw[e] = sqrtf(float(u.mult));
            }
        }
    };
    auto store = [&](int buf) {
        float* o = sh[buf];
#pragma unroll
        for (int e = 0; e < C::EPT; ++e) {
            const int idx = tid + 256 * e;
            const int j = idx / C::NZP, z = idx - j * C::NZP;
            o[z * C::STR + j] = sw[e] * (ga[e].x * gb[e].x - ga[e].y * gb[e].y);       // k = 2j
            o[z * C::STR + 8 + j] = sw[e] * (ga[e].x * gb[e].y + ga[e].y * gb[e].x);   // k = 2j+1
        }
    };
    auto compute = [&](int buf) {
        const float* o = sh[buf];
        if (wv == 0) f32_wave_mfma<NT, 0>(acc, o, lane);
        else if (wv == 1) f32_wave_mfma<NT, 1>(acc, o, lane);
        else if (wv == 2) f32_wave_mfma<NT, 2>(acc, o, lane);
        else f32_wave_mfma<NT, 3>(acc, o, lane);
    };
    load(0);
    store(0);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        if (s + 1 < nst) load(s + 1);
        compute(s & 1);
        if (s + 1 < nst) store((s + 1) & 1);
        __syncthreads();
    }
    float* out = part + size_t(it.slot) * C::NTL * 1024;
    if (wv == 0) f32_store_tiles<NT, 0>(acc, out, lane);
    else if (wv == 1) f32_store_tiles<NT, 1>(acc, out, lane);
    else if (wv == 2) f32_store_tiles<NT, 2>(acc, out, lane);
    else f32_store_tiles<NT, 3>(acc, out, lane);
}

// ------------------------------------------------------------------ FP64 ---
template <int NT>
struct F64Cfg {
    static constexpr int NZP = 32 * NT;
    static constexpr int NB = 2 * NT;                    // 16-wide blocks
    static constexpr int NBL = NB * (NB + 1) / 2;        // lower 16x16 tiles
    static constexpr int TPW = (NBL + 7) / 8;            // 8 waves
    static constexpr int EPT = (8 * NZP + 511) / 512;    // formation elements per thread
};

template <int NT, int W>
__device__ __forceinline__ void f64_wave_mfma(f64x4 (&acc)[F64Cfg<NT>::TPW], const double* sh,
                                              int lane) {
    using C = F64Cfg<NT>;
    constexpr int t0 = W * C::TPW;
    constexpr int t1 = (t0 + C::TPW < C::NBL) ? t0 + C::TPW : C::NBL;
    constexpr uint32_t need = t0 < t1 ? block_mask(t0, t1) : 0u;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        double fa[C::NB];
        const int roff = (4 * s + (lane >> 4)) * C::NZP + (lane & 15);
#pragma unroll
        for (int b = 0; b < C::NB; ++b)
            if (need & (1u << b)) fa[b] = sh[roff + 16 * b];
#pragma unroll
        for (int m = 0; m < C::TPW; ++m) {
            const int t = t0 + m;
            if (t < t1) {
                const int I = tri_I(t), J = tri_J(t);
                acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[I], fa[J], acc[m], 0, 0, 0);
            }
        }
    }
}

template <int NT, int W>
__device__ __forceinline__ void f64_store_tiles(const f64x4 (&acc)[F64Cfg<NT>::TPW], double* out,
                                                int lane) {
    using C = F64Cfg<NT>;
    constexpr int t0 = W * C::TPW;
#pragma unroll
    for (int m = 0; m < C::TPW; ++m) {
        const int t = t0 + m;
        if (t < C::NBL) {
            const int I = tri_I(t), J = tri_J(t);
            const int T = tri_I(t) / 2 * (tri_I(t) / 2 + 1) / 2 + J / 2;   // 32-tile index
            double* o = out + size_t(T) * 1024 + (I & 1) * 16 * 32 + (J & 1) * 16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // v_mfma_f64_16x16x4: lane l, register v holds row 4 v + l/16, column l%16
                const int i = 4 * v + (lane >> 4);
                o[i * 32 + (lane & 15)] = acc[m][v];
            }
        }
    }
}

template <int NT>
__global__ __launch_bounds__(512, 1) void gram_f64_kernel(const uint32_t* __restrict__ urows,
                                                          const Item* __restrict__ items,
                                                          const int32_t* __restrict__ sched,
                                                          const zd* __restrict__ g64,
                                                          const double* __restrict__ freq, double eps,
                                                          double dz, int ncls, int nz,
                                                          double* __restrict__ part) {
    using C = F64Cfg<NT>;
    __shared__ __attribute__((aligned(16))) double sh[2][16 * C::NZP];
    const Item it = items[sched[blockIdx.x]];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = it.row_end - it.row_begin;
    const int nst = (n + 7) >> 3;
    f64x4 acc[C::TPW];
#pragma unroll
    for (int m = 0; m < C::TPW; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[m][v] = 0.0;
    zd ga[C::EPT], gb[C::EPT];
    double sw[C::EPT];
    auto load = [&](int s) {
#pragma unroll
        for (int e = 0; e < C::EPT; ++e) {
            const int idx = tid + 512 * e;
            const int j = idx / C::NZP, z = idx - j * C::NZP;
            const int r = s * 8 + j;
            ga[e] = zd{0.0, 0.0};
            gb[e] = zd{0.0, 0.0};
            sw[e] = 0.0;
            if (idx < 8 * C::NZP && r < n && z < nz) {
                const URow u = load_urow(urows, int64_t(it.row_begin) + r);
                const int64_t fb = int64_t(u.f) * ncls;
                ga[e] = g64[(fb + u.cr) * nz + z];
                gb[e] = g64[(fb + u.cs) * nz + z];
                const zd w = omega_of(freq[u.f], eps);
                sw[e] = zabs2(w) * dz * sqrt(double(u.mult));
            }
        }
    };
    auto store = [&](int buf) {
        double* o = sh[buf];
#pragma unroll
        for (int e = 0; e < C::EPT; ++e) {
            const int idx = tid + 512 * e;
            if (idx < 8 * C::NZP) {
                const int j = idx / C::NZP, z = idx - j * C::NZP;
                const zd p = ga[e] * gb[e];
                o[(2 * j) * C::NZP + z] = sw[e] * p.x;
                o[(2 * j + 1) * C::NZP + z] = sw[e] * p.y;
            }
        }
    };
    auto compute = [&](int buf) {
        const double* o = sh[buf];
        switch (wv) {
            case 0: f64_wave_mfma<NT, 0>(acc, o, lane); break;
            case 1: f64_wave_mfma<NT, 1>(acc, o, lane); break;
            case 2: f64_wave_mfma<NT, 2>(acc, o, lane); break;
            case 3: f64_wave_mfma<NT, 3>(acc, o, lane); break;
            case 4: f64_wave_mfma<NT, 4>(acc, o, lane); break;
            case 5: f64_wave_mfma<NT, 5>(acc, o, lane); break;
            case 6: f64_wave_mfma<NT, 6>(acc, o, lane); break;
            default: f64_wave_mfma<NT, 7>(acc, o, lane); break;
        }
    };
    load(0);
    store(0);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        if (s + 1 < nst) load(s + 1);
        compute(s & 1);
        if (s + 1 < nst) store((s + 1) & 1);
        __syncthreads();
    }
    double* out = part + size_t(it.slot) * (NT * (NT + 1) / 2) * 1024;
    switch (wv) {
        case 0: f64_store_tiles<NT, 0>(acc, out, lane); break;
        case 1: f64_store_tiles<NT, 1>(acc, out, lane); break;
        case 2: f64_store_tiles<NT, 2>(acc, out, lane); break;
        case 3: f64_store_tiles<NT, 3>(acc, out, lane); break;
        case 4: f64_store_tiles<NT, 4>(acc, out, lane); break;
        case 5: f64_store_tiles<NT, 5>(acc, out, lane); break;
        case 6: f64_store_tiles<NT, 6>(acc, out, lane); break;
        default: f64_store_tiles<NT, 7>(acc, out, lane); break;
    }
}

// ---------------------------------------------------------------- reduce ---
// gram[p][zi][zj] (zi >= zj) = sum over the pair's items of the partial tiles,
// accumulated in FP64 in item order.  Grid: (n_pairs, lower 32-tiles).
template <class T>
__global__ __launch_bounds__(256) void gram_reduce_kernel(const T* __restrict__ part,
                                                          const int32_t* __restrict__ pair_item,
                                                          int nz, int ntl, double* __restrict__ gram) {
    const int p = blockIdx.x, t = blockIdx.y;
    const int I = tri_I(t), J = tri_J(t);
    const int k0 = pair_item[p], k1 = pair_item[p + 1];
    double* G = gram + size_t(p) * nz * nz;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int e = threadIdx.x + 256 * m;
        const int i = e >> 5, j = e & 31;
        const int zi = 32 * I + i, zj = 32 * J + j;
        if (zi >= nz || zj > zi) continue;
        double s = 0.0;
        for (int k = k0; k < k1; ++k) s += double(part[(size_t(k) * ntl + t) * 1024 + e]);
        G[size_t(zi) * nz + zj] = s;
    }
}

// rhs[p][h][z] and trace[p] from the per-item partials, in item order.
__global__ __launch_bounds__(256) void rhs_reduce_kernel(const double* __restrict__ rpart,
                                                         const int32_t* __restrict__ pair_item,
                                                         int nz, double* __restrict__ rhs,
                                                         double* __restrict__ trace) {
    const int p = blockIdx.x;
    const int k0 = pair_item[p], k1 = pair_item[p + 1];
    const int w = 2 * nz + 1;
    for (int e = threadIdx.x; e < w; e += 256) {
        double s = 0.0;
        for (int k = k0; k < k1; ++k) s += rpart[size_t(k) * w + e];
        if (e < 2 * nz) rhs[size_t(p) * 2 * nz + e] = s;
        else trace[p] = s;
    }
}

// ------------------------------------------------------------- launchers ---
template <int NT>
static hipError_t launch_gram_nt(const edt_plan* p, edt_precision prec, const zd* g64,
                                 const float2* g32, void* part, hipStream_t st) {
    const uint32_t* urows = dptr<const uint32_t>(p, p->lay.urows);
    const Item* items = dptr<const Item>(p, p->lay.items);
    const int32_t* sched = dptr<const int32_t>(p, p->lay.sched);
    const int nit = int(p->items.size());
    if (nit == 0) return hipSuccess;
    if (prec == EDT_BF16X3)
        hipLaunchKernelGGL(gram_bf16x3_kernel<NT>, dim3(nit), dim3(256), 0, st, urows, items, sched,
                           g32, p->n_cls, p->nz, static_cast<float*>(part));
    else if (prec == EDT_FP32)
        hipLaunchKernelGGL(gram_f32_kernel<NT>, dim3(nit), dim3(256), 0, st, urows, items, sched, g32,
                           p->n_cls, p->nz, static_cast<float*>(part));
    else
        hipLaunchKernelGGL(gram_f64_kernel<NT>, dim3(nit), dim3(512), 0, st, urows, items, sched, g64,
                           dptr<const double>(p, p->lay.freq), p->eps, p->dz, p->n_cls, p->nz,
                           static_cast<double*>(part));
    return hipGetLastError();
}

hipError_t launch_gram(const edt_plan* p, edt_precision prec, const zd* g64, const float2* g32,
                       void* part, hipStream_t st) {
    const int NT = (p->nz + 31) / 32;
    hipError_t e;
    switch (NT) {
        case 1: e = launch_gram_nt<1>(p, prec, g64, g32, part, st); break;
        case 2: e = launch_gram_nt<2>(p, prec, g64, g32, part, st); break;
        case 3: e = launch_gram_nt<3>(p, prec, g64, g32, part, st); break;
        case 4: e = launch_gram_nt<4>(p, prec, g64, g32, part, st); break;
        case 5: e = launch_gram_nt<5>(p, prec, g64, g32, part, st); break;
        case 6: e = launch_gram_nt<6>(p, prec, g64, g32, part, st); break;
        case 7: e = launch_gram_nt<7>(p, prec, g64, g32, part, st); break;
        case 8: e = launch_gram_nt<8>(p, prec, g64, g32, part, st); break;
        default: return hipErrorInvalidValue;
    }
    return e;
}

hipError_t launch_gram_reduce(const edt_plan* p, edt_precision prec, const void* part, double* gram,
                              hipStream_t st) {
    const int NT = (p->nz + 31) / 32;
    const int ntl = NT * (NT + 1) / 2;
    const int32_t* pair_item = dptr<const int32_t>(p, p->lay.pair_item);
    if (p->n_pairs == 0) return hipSuccess;
    if (prec == EDT_FP64)
        hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3(unsigned(p->n_pairs), ntl), dim3(256), 0,
                           st, static_cast<const double*>(part), pair_item, p->nz, ntl, gram);
    else
        hipLaunchKernelGGL(gram_reduce_kernel<float>, dim3(unsigned(p->n_pairs), ntl), dim3(256), 0,
                           st, static_cast<const float*>(part), pair_item, p->nz, ntl, gram);
    return hipGetLastError();
}

hipError_t launch_rhs_reduce(const edt_plan* p, const double* rpart, double* rhs, double* trace,
                             hipStream_t st) {
    if (p->n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(rhs_reduce_kernel, dim3(unsigned(p->n_pairs)), dim3(256), 0, st, rpart,
                       dptr<const int32_t>(p, p->lay.pair_item), p->nz, rhs, trace);
    return hipGetLastError();
}

}  // namespace edt
