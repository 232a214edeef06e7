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
// Green's tables into LDS (a ring of stage buffers), and its waves feed them to MFMA
// for the whole lower triangle of the nz x nz Gram, which stays in registers
// across the chunk; A is never written to memory.  Each item stores its
// partial Gram tile by tile; a second kernel sums the items of a pair in FP64
// in a fixed order (deterministic).
//
// Precisions:
//   BF16X3: v_mfma_f32_32x32x16_bf16, each value split x = hi + lo (bf16) and
//           Ah^T Ah ~ hi^T hi + hi^T lo + lo^T hi with FP32 accumulation;
//   FP16X3: the same with IEEE halves (v_mfma_f32_32x32x16_f16) on rows
//           scaled by a power of two per item;
//   FP32:   v_mfma_f32_32x32x2_f32;
//   FP64:   v_mfma_f64_16x16x4_f64 on FP64 rows built from the FP64 table.

#include <cstdlib>
#include <type_traits>

#include "dev_common.h"

namespace edt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
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

// Split x = hi + lo into two 16-bit values (F16: IEEE half, else bfloat16),
// each rounded to nearest, and pack (x0, x1) halves as (hi0 | hi1 << 16),
// (lo0 | lo1 << 16).  On gfx950 the pair conversions are single packed
// instructions and x - hi folds into a mixed-precision FMA.
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <bool F16>
__device__ __forceinline__ void split_pack(float x0, float x1, uint32_t& hi, uint32_t& lo) {
    typedef typename std::conditional<F16, f16x2, bf16x2>::type v2;
    const v2 h = __builtin_convertvector(f32x2{x0, x1}, v2);
    const f32x2 r = {x0 - float(h[0]), x1 - float(h[1])};
    hi = __builtin_bit_cast(uint32_t, h);
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, v2));
}

// ------------------------------------------------------- split (16-bit) ---
// A Gram task covers the tiles between two depth super-blocks of at most 256
// depths (8 blocks of 32): a diagonal task (NTJ = 0) the lower triangle of
// one super-block of NT blocks, a rectangular task (NTJ > 0) the NT x NTJ
// tiles between NT blocks of a later super-block (the I set) and NTJ blocks
// of an earlier one (the J set).  Depth counts up to 256 need one diagonal
// task; larger ones add the super-blocks below and the rectangles between.
// Rectangle tiles are numbered column by column, so that an MFMA wave's tiles
// share their J blocks and read every I block.
template <int NT, int NTJ>
struct SplitCfg {
    static constexpr bool RECT = NTJ > 0;
    static constexpr int NZPI = 32 * NT, NZPJ = 32 * NTJ, NZP = NZPI + NZPJ;
    static constexpr int NTL = RECT ? NT * NTJ : NT * (NT + 1) / 2;
    static constexpr int TPW = (NTL + 3) / 4;
    static constexpr int STR = 24;   // 16-bit values per LDS depth row: 16 real rows + 8 pad (48 B)
    __host__ __device__ static constexpr int tI(int t) { return RECT ? t % NT : tri_I(t); }
    __host__ __device__ static constexpr int tJ(int t) { return RECT ? t / NT : tri_J(t); }
    // blocks of the I (J) set read by the tiles [t0, t1)
    __host__ __device__ static constexpr uint32_t maskI(int t0, int t1) {
        uint32_t m = 0;
        for (int t = t0; t < t1; ++t) m |= RECT ? (1u << tI(t)) : ((1u << tI(t)) | (1u << tJ(t)));
        return m;
    }
    __host__ __device__ static constexpr uint32_t maskJ(int t0, int t1) {
        uint32_t m = 0;
        if (RECT)
            for (int t = t0; t < t1; ++t) m |= 1u << tJ(t);
        return m;
    }
};

template <class C, int W, bool F16>
__device__ __forceinline__ void split3_wave_mfma(f32x16 (&acc)[C::TPW], const uint16_t* hi,
                                                 const uint16_t* lo, int lane) {
    typedef typename std::conditional<F16, f16x8, bf16x8>::type v8;
    constexpr int t0 = W * C::TPW;
    constexpr int t1 = (t0 + C::TPW < C::NTL) ? t0 + C::TPW : C::NTL;
    constexpr uint32_t needI = t0 < t1 ? C::maskI(t0, t1) : 0u;
    constexpr uint32_t needJ = t0 < t1 ? C::maskJ(t0, t1) : 0u;
    constexpr int NBI = C::NZPI / 32, NBJ = C::RECT ? C::NZPJ / 32 : 1;
    v8 fh[NBI], fl[NBI], gh[NBJ], gl[NBJ];
    const int roff = (lane & 31) * C::STR + (lane >> 5) * 8;
#pragma unroll
    for (int b = 0; b < NBI; ++b) {
        if (needI & (1u << b)) {
            fh[b] = *reinterpret_cast<const v8*>(hi + b * 32 * C::STR + roff);
            fl[b] = *reinterpret_cast<const v8*>(lo + b * 32 * C::STR + roff);
        }
    }
    if constexpr (C::RECT) {
#pragma unroll
        for (int b = 0; b < NBJ; ++b) {
            if (needJ & (1u << b)) {
                gh[b] = *reinterpret_cast<const v8*>(hi + (C::NZPI + b * 32) * C::STR + roff);
                gl[b] = *reinterpret_cast<const v8*>(lo + (C::NZPI + b * 32) * C::STR + roff);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < C::TPW; ++m) {
        const int t = t0 + m;
        if (t < t1) {
            const int I = C::tI(t), J = C::tJ(t);
            const v8 aH = fh[I], aL = fl[I];
            const v8 bH = C::RECT ? gh[J] : fh[J], bL = C::RECT ? gl[J] : fl[J];
            if constexpr (F16) {
                acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aH, bH, acc[m], 0, 0, 0);
                acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aH, bL, acc[m], 0, 0, 0);
                acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aL, bH, acc[m], 0, 0, 0);
            } else {
                acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aH, bH, acc[m], 0, 0, 0);
                acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aH, bL, acc[m], 0, 0, 0);
                acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aL, bH, acc[m], 0, 0, 0);
            }
        }
    }
}

// Store the wave's 32 x 32 accumulator tiles into the item's partial, at the
// global tile (bI0 + I, bJ0 + J) of the lower triangle of all depth blocks.
template <class C, int W>
__device__ __forceinline__ void f32_store_tiles(const f32x16 (&acc)[C::TPW], float* out, int lane,
                                                float scale, int bI0, int bJ0) {
    constexpr int t0 = W * C::TPW;
#pragma unroll
    for (int m = 0; m < C::TPW; ++m) {
        const int t = t0 + m;
        if (t < C::NTL) {
            const int Ig = bI0 + C::tI(t), Jg = bJ0 + C::tJ(t);
            float* o = out + size_t(Ig * (Ig + 1) / 2 + Jg) * 1024;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                // streaming store: the partials are read once, by the reduce,
                // and must not evict the Green's table slab from L2
                __builtin_nontemporal_store(acc[m][v] * scale, &o[i * 32 + (lane & 31)]);
            }
        }
    }
}

// Per-row records of an item in LDS for the FP32 / BF16x3 kernels:
// s_row[2 r] = {off_r, off_s, sqrt(mult), mult}, s_row[2 r + 1] = the row's
// data conj(W)/|W| (b+, b-) in FP32.  Rows are padded to a multiple of 8 with
// all-zero records (table offset 0, no weight, no data): a padding row loads
// valid table entries and contributes nothing.
__device__ __forceinline__ void stage_rows(uint4* s_row, const GRow* __restrict__ grow,
                                           const float4* __restrict__ ub32, int64_t row_begin, int n,
                                           int nst, int tid, int nthreads) {
    for (int e = tid; e < 8 * nst; e += nthreads) {
        uint4 a = make_uint4(0u, 0u, 0u, 0u), b = a;
        if (e < n) {
            const GRow g = grow[row_begin + e];
            a = make_uint4(g.off_r, g.off_s, __float_as_uint(g.sw), __float_as_uint(g.mt));
            const float4 w = ub32[row_begin + e];
            b = make_uint4(__float_as_uint(w.x), __float_as_uint(w.y), __float_as_uint(w.z),
                           __float_as_uint(w.w));
        }
        s_row[2 * e] = a;
        s_row[2 * e + 1] = b;
    }
}

// Zero stages a split kernel may append to an item (its load pipeline depth
// at most, plus one).
constexpr int kPadStages = 4;

// Producer side of the split kernels: raw table values of one stage (8
// complex rows) at one depth.
struct RawStage {
    float2 ga[8], gb[8];
};

// Split Gram (BF16x3 or FP16x3) task over one work item.  Each FP32 row value
// x is split into two 16-bit values x = hi + lo and the block
// Ah_I^T Ah_J ~ hi_I^T hi_J + hi_I^T lo_J + lo_I^T hi_J is accumulated in
// FP32: about 16 significant bits per product with bfloat16 halves, about 22
// with IEEE halves (which need the per-item scaling below).
// Warp-specialised: waves 0-3 consume 16-bit stages from LDS into MFMA, waves
// 4-7 produce them.  A producer issues the table loads of stage s+PF while it
// forms stage s+1, so each load has PF-1 MFMA stages to arrive (PF = 3 for a
// diagonal task, 2 for a rectangular one, whose two depth sets double the
// registers per stage).  A producer thread owns one depth of the I set (and
// one of the J set) and all 8 rows of a stage, so it writes its 16 hi and 16
// lo values as 16-byte stores; with the 48-byte LDS row pitch any 8
// consecutive depths hit distinct bank groups.  Row records come from LDS
// (the row of a stage is uniform over the wave: broadcast reads, and the
// table base of a load is a scalar).  Depths past nz are zeroed once per item.
// Diagonal tasks also accumulate the item's right-hand side
// c+-(z) = Re(A^H B+-) over their depths from FP32 rows (an approximation: the
// FP64 refinement residual corrects it) and the trace sum mult |A|^2, both per
// stage in FP32 and then in FP64 (so that the error does not grow with the
// item's length), into rpart[slot] (c+, c-, one trace per super-block).
template <int NT, int NTJ, bool F16>
__global__ __launch_bounds__(512, 1) void gram_split3_kernel(const Item* __restrict__ items,
                                                             const int32_t* __restrict__ sched,
                                                             const GRow* __restrict__ grow,
                                                             const float4* __restrict__ ub32,
                                                             const float2* __restrict__ g32,
                                                             const float* __restrict__ gmax, int nz,
                                                             int zI0, int zJ0, int ntot,
                                                             float* __restrict__ part,
                                                             double* __restrict__ rpart, int max_rows) {
    using C = SplitCfg<NT, NTJ>;
    // stages of table loads in flight per producer (register sets of raw values)
    constexpr int PF = 2;
    static_assert(PF + 1 <= kPadStages, "padding stages exceed the row LDS");
    __shared__ __attribute__((aligned(16))) uint16_t sh[2][2][C::NZP * C::STR];
    __shared__ double s_tr[4];
    __shared__ float s_max[8];
    extern __shared__ __attribute__((aligned(16))) uint4 s_row[];
    const int32_t k = sched[blockIdx.x];
    if (k < 0) return;   // hole in the XCD-aware schedule
    const Item it = items[k];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = min(it.row_end - it.row_begin, max_rows);
    const int nst = (n + 7) >> 3;
    // stages padded with at least one all-zero stage to a multiple of PF: the
    // producer pipeline below then runs without branches (a branch around the
    // loads would make the compiler wait for every load in flight at the join)
    const int nsp = ((nst + 1 + PF - 1) / PF) * PF;
    const int nzI = min(C::NZPI, nz - zI0);   // valid depths of the I set
    stage_rows(s_row, grow, ub32, it.row_begin, n, nsp, tid, 512);
    // FP16: the rows of the item are scaled by a power of two s so that the
    // largest |value| is near 2^14 (inside the half range, above its
    // subnormals); the partial Gram is scaled back by 1/s^2 (exact).  The
    // bound per row is max_z |g(k_r)| max_z |g(k_s)| sqrt(mult).
    float scale = 1.0f;
    if constexpr (F16) {
        float mx = 0.0f;
        for (int e = tid; e < n; e += 512) {
            const GRow g = grow[it.row_begin + e];
            mx = fmaxf(mx, gmax[g.off_r / uint32_t(nz)] * gmax[g.off_s / uint32_t(nz)] * g.sw);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) s_max[wv] = mx;
        __syncthreads();
        float m = s_max[0];
#pragma unroll
        for (int w = 1; w < 8; ++w) m = fmaxf(m, s_max[w]);
        if (m > 0.0f && isfinite(m)) scale = ldexpf(1.0f, 14 - ilogbf(m) - 1);
    }
    {
        const int z = tid - 256;
        if (z >= nzI && z < C::NZPI) {
            const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    uint4* o = reinterpret_cast<uint4*>(sh[b][h] + z * C::STR);
                    o[0] = zero;
                    o[1] = zero;
                }
        }
    }
    __syncthreads();

    const bool producer = wv >= 4;
    if (producer) {
        const int pid = tid - 256;
        const bool onI = pid < nzI;                  // this thread forms I-set depth zI0 + pid
        const bool onJ = C::RECT && pid < C::NZPJ;   // and J-set depth zJ0 + pid (always < nz)
        const int zIc = zI0 + min(pid, nzI - 1);     // clamped: loads are unconditional
        const int zJc = min(zJ0 + pid, nz - 1);
        double cp = 0.0, cm = 0.0, tr = 0.0;   // per stage in FP32, then in FP64
        auto load = [&](RawStage& R, int s, int zc) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint4 a = s_row[2 * (8 * s + j)];
                const uint32_t o_r = __builtin_amdgcn_readfirstlane(a.x);
                const uint32_t o_s = __builtin_amdgcn_readfirstlane(a.y);
                R.ga[j] = (g32 + o_r)[zc];
                R.gb[j] = (g32 + o_s)[zc];
            }
        };
        auto form = [&](const RawStage& R, int buf, int s, int row, bool diag_sums, bool on) {
            uint32_t h[8], l[8];
            float t = 0.0f, sp = 0.0f, sm = 0.0f;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint4 a = s_row[2 * (8 * s + j)];
                const float sw = __uint_as_float(a.z);
                const float px = R.ga[j].x * R.gb[j].x - R.ga[j].y * R.gb[j].y;
                const float py = R.ga[j].x * R.gb[j].y + R.ga[j].y * R.gb[j].x;
                if (diag_sums) {
                    const uint4 b = s_row[2 * (8 * s + j) + 1];
                    const float mt = __uint_as_float(a.w);
                    sp += px * __uint_as_float(b.x) + py * __uint_as_float(b.y);
                    sm += px * __uint_as_float(b.z) + py * __uint_as_float(b.w);
                    t += mt * (px * px + py * py);
                }
                const float ss = F16 ? sw * scale : sw;
                split_pack<F16>(ss * px, ss * py, h[j], l[j]);
            }
            if (diag_sums) {
                tr += double(t);
                cp += double(sp);
                cm += double(sm);
            }
            if (on) {
                uint4* hi = reinterpret_cast<uint4*>(sh[buf][0] + row * C::STR);
                uint4* lo = reinterpret_cast<uint4*>(sh[buf][1] + row * C::STR);
                hi[0] = make_uint4(h[0], h[1], h[2], h[3]);
                hi[1] = make_uint4(h[4], h[5], h[6], h[7]);
                lo[0] = make_uint4(l[0], l[1], l[2], l[3]);
                lo[1] = make_uint4(l[4], l[5], l[6], l[7]);
            }
        };
        auto load_stage = [&](RawStage (&R)[2], int s) {
            load(R[0], s, zIc);
            if constexpr (C::RECT) load(R[1], s, zJc);
        };
        auto form_stage = [&](const RawStage (&R)[2], int buf, int s) {
            form(R[0], buf, s, pid, !C::RECT, onI);
            if constexpr (C::RECT) form(R[1], buf, s, C::NZPI + pid, false, onJ);
        };
        // Stage k's raw values live in R[k % PF] ([0] I set, [1] J set): the
        // loads of stage t + PF are issued while stage t + 1 is formed, so
        // each load has PF - 1 stage periods to arrive.
        // Stage indices past the padded end are clamped to its last (zero)
        // stage: the extra loads read valid entries, and the extra form writes
        // a buffer nobody consumes and adds zeros to the sums.
        RawStage R[PF][2];
#pragma unroll
        for (int q = 0; q < PF; ++q) load_stage(R[q], q);
        form_stage(R[0], 0, 0);
        __syncthreads();
        // part t: stage t is being consumed from buffer t & 1
        for (int s = 0; s < nsp; s += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int t = s + q;
                load_stage(R[q], min(t + PF, nsp - 1));
                form_stage(R[(q + 1) % PF], (t + 1) & 1, min(t + 1, nsp - 1));
                __syncthreads();
            }
        }
        if constexpr (!C::RECT) {
            if (onI) {
                double* rp = rpart + size_t(it.slot) * rpart_width(nz);
                rp[zI0 + pid] = cp;
                rp[nz + zI0 + pid] = cm;
            }
            const double t = wave_sum(onI ? tr : 0.0);
            if (lane == 0) s_tr[wv - 4] = t;
        }
    } else {
        f32x16 acc[C::TPW];
#pragma unroll
        for (int m = 0; m < C::TPW; ++m)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[m][v] = 0.0f;
        auto compute = [&](int buf) {
            const uint16_t* hi = sh[buf][0];
            const uint16_t* lo = sh[buf][1];
            if (wv == 0) split3_wave_mfma<C, 0, F16>(acc, hi, lo, lane);
            else if (wv == 1) split3_wave_mfma<C, 1, F16>(acc, hi, lo, lane);
            else if (wv == 2) split3_wave_mfma<C, 2, F16>(acc, hi, lo, lane);
            else split3_wave_mfma<C, 3, F16>(acc, hi, lo, lane);
        };
        __syncthreads();
        for (int t = 0; t < nsp; ++t) {
            if (t < nst) compute(t & 1);   // padding stages are zero
            __syncthreads();
        }
        float* out = part + size_t(it.slot) * (ntot * (ntot + 1) / 2) * 1024;
        const float back = 1.0f / (scale * scale);
        const int bI0 = zI0 / 32, bJ0 = C::RECT ? zJ0 / 32 : zI0 / 32;
        if (wv == 0) f32_store_tiles<C, 0>(acc, out, lane, back, bI0, bJ0);
        else if (wv == 1) f32_store_tiles<C, 1>(acc, out, lane, back, bI0, bJ0);
        else if (wv == 2) f32_store_tiles<C, 2>(acc, out, lane, back, bI0, bJ0);
        else f32_store_tiles<C, 3>(acc, out, lane, back, bI0, bJ0);
    }
    if constexpr (!C::RECT) {
        __syncthreads();
        if (tid == 0)
            rpart[size_t(it.slot) * rpart_width(nz) + 2 * nz + zI0 / kSuperDepth] =
                (s_tr[0] + s_tr[1]) + (s_tr[2] + s_tr[3]);
    }
}

// ------------------------------------------------- split, diagonal ---
// Diagonal split tasks run with every wave both forming rows and issuing
// MFMA.  Default tile deal (sizes without a compact one below): the lower
// triangle in row-major order is cut into four SIMD groups of G consecutive
// tiles; waves s and s+4 (one SIMD) take the first TA and the remaining G-TA
// tiles of group s.
template <int NT>
struct UCfg {
    static constexpr int NTL = NT * (NT + 1) / 2;
    static constexpr int G = (NTL + 3) / 4;
    static constexpr int TA = (G + 1) / 2;
    static constexpr int TPW = TA;
    static constexpr int STR = 24;   // 16-bit values per LDS depth row (16 real rows + 8 pad)
    static constexpr int NZP = 32 * NT;
    __host__ __device__ static constexpr int t0(int w) {
        return w < 4 ? (w * G < NTL ? w * G : NTL) : ((w - 4) * G + TA < NTL ? (w - 4) * G + TA : NTL);
    }
    __host__ __device__ static constexpr int t1(int w) {
        return w < 4 ? (w * G + TA < NTL ? w * G + TA : NTL) : ((w - 3) * G < NTL ? (w - 3) * G : NTL);
    }
};

// raw table values of half a stage (4 complex rows) at one depth
struct RawHalf {
    float2 ga[4], gb[4];
};

// Scheduling of one stage of wave W: its fragment reads first, then each MFMA
// followed by up to V VALU instructions and one vector-memory read.
template <int NM, int NF, int V>
__device__ __forceinline__ void w_interleave() {
    __builtin_amdgcn_sched_group_barrier(0x100, NF, 0);
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, V, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    }
}


// ------------------------- split, diagonal, fragments read a stage ahead ---
// The diagonal split task with the LDS fragment reads taken off the critical
// path: rows are formed two stages ahead into a ring of three LDS stage
// buffers, and each wave reads the fragments of stage t + 1 into registers
// while it issues the MFMAs of stage t, so per stage the LDS reads, the
// matrix products and the row forming (VALU) of a wave overlap behind one
// barrier.  The tiles of the 8- and 7-block tasks are dealt in compact groups
// (2 x 2 squares of the rectangle below the half-way block, and runs of the
// two triangles), so that a wave reads at most four blocks per stage.
// Accumulation order per tile is that of the other split kernels (per stage:
// hi.hi, hi.lo, lo.hi), so the Grams are the same bit for bit.
template <int NT>
struct PCfg {
    // tile m of wave W as I * 8 + J (I >= J), or -1
    __host__ __device__ static constexpr int tile(int W, int m) {
        if constexpr (NT == 8) {
            constexpr int T[8][5] = {{32, 33, 40, 41, -1}, {34, 35, 42, 43, -1}, {48, 49, 56, 57, -1},
                                     {50, 51, 58, 59, -1}, {0, 8, 9, 16, 24},    {17, 18, 25, 26, 27},
                                     {36, 44, 45, 52, 60}, {53, 54, 61, 62, 63}};
            return m < 5 ? T[W][m] : -1;
        } else if constexpr (NT == 7) {
            constexpr int T[8][4] = {{24, 25, 26, -1}, {32, 33, 34, -1}, {40, 41, 42, -1}, {48, 49, 50, -1},
                                     {0, 8, 9, 16},    {17, 18, 27, 35}, {36, 43, 44, 45}, {51, 52, 53, 54}};
            return m < 4 ? T[W][m] : -1;
        } else {
            const int t = UCfg<NT>::t0(W) + m;
            return (m < UCfg<NT>::TPW && t < UCfg<NT>::t1(W)) ? tri_I(t) * 8 + tri_J(t) : -1;
        }
    }
    static constexpr int TPW = NT == 8 ? 5 : NT == 7 ? 4 : UCfg<NT>::TPW;
    __host__ __device__ static constexpr uint32_t mask(int W) {
        uint32_t b = 0;
        for (int m = 0; m < TPW; ++m)
            if (tile(W, m) >= 0) b |= (1u << (tile(W, m) >> 3)) | (1u << (tile(W, m) & 7));
        return b;
    }
    // position of block b among the blocks of wave W
    __host__ __device__ static constexpr int slot(int W, int b) {
        return __builtin_popcount(mask(W) & ((1u << b) - 1u));
    }
};

template <int NT, int W, bool F16>
__device__ __forceinline__ void split3p_wave(const Item& it, const GRow* __restrict__ grow,
                                             const float4* __restrict__ ub32, const float2* __restrict__ g32,
                                             const float* __restrict__ gmax, int nz, int zI0, int ntot,
                                             float* __restrict__ part, double* __restrict__ rpart, int max_rows,
                                             uint16_t (*sh)[2][UCfg<NT>::NZP * UCfg<NT>::STR], double* s_tr,
                                             float* s_max, uint4* s_row) {
    using C = UCfg<NT>;
    using P = PCfg<NT>;
    typedef typename std::conditional<F16, f16x8, bf16x8>::type v8;
    constexpr uint32_t need = P::mask(W);
    constexpr int NB = __builtin_popcount(need) > 0 ? __builtin_popcount(need) : 1;
    constexpr int NM = [] {
        int c = 0;
        for (int m = 0; m < P::TPW; ++m) c += P::tile(W, m) >= 0 ? 3 : 0;
        return c;
    }();
    static_assert(3 <= kPadStages, "padding stages exceed the row LDS");
    const int tid = threadIdx.x, lane = tid & 63;
    const int n = min(it.row_end - it.row_begin, max_rows);
    const int nst = (n + 7) >> 3;
    const int nsp = ((nst + 1 + 1) / 2) * 2;   // + zero stages, an even count
    const int nzI = min(C::NZP, nz - zI0);
    stage_rows(s_row, grow, ub32, it.row_begin, n, nsp, tid, 512);
    float scale = 1.0f;
    if constexpr (F16) {
        float mx = 0.0f;
        for (int e = tid; e < n; e += 512) {
            const GRow g = grow[it.row_begin + e];
            mx = fmaxf(mx, gmax[g.off_r / uint32_t(nz)] * gmax[g.off_s / uint32_t(nz)] * g.sw);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) s_max[W] = mx;
        __syncthreads();
        float m = s_max[0];
#pragma unroll
        for (int w = 1; w < 8; ++w) m = fmaxf(m, s_max[w]);
        if (m > 0.0f && isfinite(m)) scale = ldexpf(1.0f, 14 - ilogbf(m) - 1);
    }
    const int z = tid & 255;
    constexpr int hf = W >> 2;   // rows 4 hf .. 4 hf + 3 of a stage
    const bool on = z < nzI;
    const uint32_t zc = uint32_t(zI0 + min(z, nzI - 1));   // clamped: loads are unconditional
    const float lane_scale = on ? scale : 0.0f;             // depths past nz form zeros
    double cp = 0.0, cm = 0.0, tr = 0.0;   // per stage in FP32, then in FP64
    const uint32_t zoff = zc * uint32_t(sizeof(float2));
    // the row records of a stage (LDS broadcasts): the table offsets of the
    // loads, and the scales and data of the row forming
    auto read_off = [&](uint32_t (&o)[8], int s) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint4 a = s_row[2 * (8 * s + 4 * hf + j)];
            o[2 * j] = __builtin_amdgcn_readfirstlane(a.x);
            o[2 * j + 1] = __builtin_amdgcn_readfirstlane(a.y);
        }
    };
    auto read_rec = [&](uint4 (&ra)[4], uint4 (&rb)[4], int s) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            ra[j] = s_row[2 * (8 * s + 4 * hf + j)];
            rb[j] = s_row[2 * (8 * s + 4 * hf + j) + 1];
        }
    };
    auto load = [&](RawHalf& R, const uint32_t (&o)[8]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            R.ga[j] = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(g32 + o[2 * j]) + zoff);
            R.gb[j] = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(g32 + o[2 * j + 1]) + zoff);
        }
    };
    auto form = [&](const RawHalf& R, const uint4 (&ra)[4], const uint4 (&rb)[4], int buf) {
        uint32_t h[4], l[4];
        float t = 0.0f, sp = 0.0f, sm = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint4 a = ra[j];
            const uint4 b = rb[j];
            const float sw = __uint_as_float(a.z), mt = __uint_as_float(a.w);
            const float px = R.ga[j].x * R.gb[j].x - R.ga[j].y * R.gb[j].y;
            const float py = R.ga[j].x * R.gb[j].y + R.ga[j].y * R.gb[j].x;
            sp += px * __uint_as_float(b.x) + py * __uint_as_float(b.y);
            sm += px * __uint_as_float(b.z) + py * __uint_as_float(b.w);
            t += mt * (px * px + py * py);
            const float ss = sw * lane_scale;
            split_pack<F16>(ss * px, ss * py, h[j], l[j]);
        }
        tr += double(t);
        cp += double(sp);
        cm += double(sm);
        if (z < C::NZP) {
            reinterpret_cast<uint4*>(sh[buf][0] + z * C::STR)[hf] = make_uint4(h[0], h[1], h[2], h[3]);
            reinterpret_cast<uint4*>(sh[buf][1] + z * C::STR)[hf] = make_uint4(l[0], l[1], l[2], l[3]);
        }
    };
    // fragments of the wave's blocks, two stages' worth
    v8 fh[2][NB], fl[2][NB];
    const int roff = (lane & 31) * C::STR + (lane >> 5) * 8;
    auto frag = [&](v8 (&h)[NB], v8 (&l)[NB], int buf) {
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            if (need & (1u << b)) {
                h[P::slot(W, b)] = *reinterpret_cast<const v8*>(sh[buf][0] + b * 32 * C::STR + roff);
                l[P::slot(W, b)] = *reinterpret_cast<const v8*>(sh[buf][1] + b * 32 * C::STR + roff);
            }
        }
    };
    f32x16 acc[P::TPW];
#pragma unroll
    for (int m = 0; m < P::TPW; ++m)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[m][v] = 0.0f;
    // products of one stage, product-major (every tile's hi.hi, then hi.lo,
    // then lo.hi), so consecutive MFMAs do not wait on one accumulator
    auto mfma = [&](const v8 (&h)[NB], const v8 (&l)[NB]) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int m = 0; m < P::TPW; ++m) {
                const int tl = P::tile(W, m);
                if (tl >= 0) {
                    const int I = P::slot(W, tl >> 3), J = P::slot(W, tl & 7);
                    const v8 a = k == 2 ? l[I] : h[I];
                    const v8 b = k == 1 ? l[J] : h[J];
                    if constexpr (F16)
                        acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[m], 0, 0, 0);
                    else
                        acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[m], 0, 0, 0);
                }
            }
        }
    };
    // stage k's raw table values live in R[k % 2]; stage indices past the
    // padded end are clamped to its last (zero) stage
    RawHalf R[2];
    __syncthreads();   // rows staged
    {
        uint32_t o[8];
        uint4 ra[4], rb[4];
        read_off(o, 0);
        load(R[0], o);
        read_off(o, 1);
        load(R[1], o);
        read_rec(ra, rb, 0);
        form(R[0], ra, rb, 0);
        read_off(o, min(2, nsp - 1));
        load(R[0], o);
        read_rec(ra, rb, 1);
        form(R[1], ra, rb, 1);
        read_off(o, min(3, nsp - 1));
        load(R[1], o);
    }
    __syncthreads();
    frag(fh[0], fl[0], 0);
    // iteration t: the products of stage t (fragments read in iteration t - 1),
    // the fragments of stage t + 1, the rows of stage t + 2 (table values
    // loaded in iteration t - 2) and the table loads of stage t + 4
    for (int s = 0; s < nsp; s += 2) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int t = s + q;
            uint4 ra[4], rb[4];
            uint32_t o[8];
            read_rec(ra, rb, min(t + 2, nsp - 1));
            read_off(o, min(t + 4, nsp - 1));
            frag(fh[q ^ 1], fl[q ^ 1], (t + 1) % 3);
            mfma(fh[q], fl[q]);
            form(R[q], ra, rb, (t + 2) % 3);
            load(R[q], o);
            w_interleave<NM, 2 * NB + 12, 8>();
            __syncthreads();
        }
    }
    float* out = part + size_t(it.slot) * (ntot * (ntot + 1) / 2) * 1024;
    const float back = 1.0f / (scale * scale);
    const int bI0 = zI0 / 32;
#pragma unroll
    for (int m = 0; m < P::TPW; ++m) {
        const int tl = P::tile(W, m);
        if (tl >= 0) {
            const int Ig = bI0 + (tl >> 3), Jg = bI0 + (tl & 7);
            float* o = out + size_t(Ig * (Ig + 1) / 2 + Jg) * 1024;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                __builtin_nontemporal_store(acc[m][v] * back, &o[i * 32 + (lane & 31)]);
            }
        }
    }
    // the two row halves of depth z meet in LDS (the stage buffers are free)
    double* sc = reinterpret_cast<double*>(&sh[0][0][0]);
    if (hf == 1) {
        sc[z] = cp;
        sc[256 + z] = cm;
    }
    const double tsum = wave_sum(on ? tr : 0.0);
    if (lane == 0) s_tr[W] = tsum;
    __syncthreads();
    double* rp = rpart + size_t(it.slot) * rpart_width(nz);
    if (hf == 0 && on) {
        rp[zI0 + z] = cp + sc[z];
        rp[nz + zI0 + z] = cm + sc[256 + z];
    }
    if (tid == 0)
        rp[2 * nz + zI0 / kSuperDepth] =
            ((s_tr[0] + s_tr[1]) + (s_tr[2] + s_tr[3])) + ((s_tr[4] + s_tr[5]) + (s_tr[6] + s_tr[7]));
}

template <int NT, bool F16>
__global__ __launch_bounds__(512, 1) void gram_split3p_kernel(const Item* __restrict__ items,
                                                              const int32_t* __restrict__ sched,
                                                              const GRow* __restrict__ grow,
                                                              const float4* __restrict__ ub32,
                                                              const float2* __restrict__ g32,
                                                              const float* __restrict__ gmax, int nz, int zI0,
                                                              int ntot, float* __restrict__ part,
                                                              double* __restrict__ rpart, int max_rows) {
    using C = UCfg<NT>;
    __shared__ __attribute__((aligned(16))) uint16_t sh[3][2][C::NZP * C::STR];
    __shared__ double s_tr[8];
    __shared__ float s_max[8];
    extern __shared__ __attribute__((aligned(16))) uint4 s_row[];
    const int32_t k = sched[blockIdx.x];
    if (k < 0) return;   // hole in the XCD-aware schedule
    const Item it = items[k];
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
#define EDT_W(w)                                                                                              \
    case w:                                                                                                   \
        split3p_wave<NT, w, F16>(it, grow, ub32, g32, gmax, nz, zI0, ntot, part, rpart, max_rows, sh, s_tr, \
                                 s_max, s_row);                                                               \
        break;
        EDT_W(0) EDT_W(1) EDT_W(2) EDT_W(3) EDT_W(4) EDT_W(5) EDT_W(6) EDT_W(7)
#undef EDT_W
        default: break;
    }
}

// ------------------------------------------------------------------ FP32 ---
template <int NT>
struct F32Cfg {
    static constexpr int NZP = 32 * NT;
    static constexpr int NTL = NT * (NT + 1) / 2;
    static constexpr int TPW = (NTL + 3) / 4;
    static constexpr int STR = 20;   // floats per LDS z-row: [h][8] + 4 pad (80 B)
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

// Every thread owns one depth z of a stage (8 complex rows), forms it into
// LDS with 16-byte stores and accumulates the item's right-hand side and
// trace like the BF16x3 producers; all four waves then run MFMA on it.
template <int NT>
__global__ __launch_bounds__(256, 1) void gram_f32_kernel(const Item* __restrict__ items,
                                                          const int32_t* __restrict__ sched,
                                                          const GRow* __restrict__ grow,
                                                          const float4* __restrict__ ub32,
                                                          const float2* __restrict__ g32, int nz,
                                                          float* __restrict__ part,
                                                          double* __restrict__ rpart, int max_rows) {
    using C = F32Cfg<NT>;
    __shared__ __attribute__((aligned(16))) float sh[2][C::NZP * C::STR];
    __shared__ double s_tr[4];
    extern __shared__ __attribute__((aligned(16))) uint4 s_row[];
    const int32_t k = sched[blockIdx.x];
    if (k < 0) return;   // hole in the XCD-aware schedule
    const Item it = items[k];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = min(it.row_end - it.row_begin, max_rows);
    const int nst = (n + 7) >> 3;
    const int z = tid, zc = min(z, nz - 1);
    stage_rows(s_row, grow, ub32, it.row_begin, n, nst, tid, 256);
    if (z >= nz && z < C::NZP) {
        const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) reinterpret_cast<float4*>(sh[b] + z * C::STR)[q] = zero;
    }
    __syncthreads();
    f32x16 acc[C::TPW];
#pragma unroll
    for (int m = 0; m < C::TPW; ++m)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[m][v] = 0.0f;
    float2 ga[8], gb[8];
    double cp = 0.0, cm = 0.0, tr = 0.0;   // per stage in FP32, then in FP64
    auto load = [&](int s) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint4 a = s_row[2 * (8 * s + j)];
            const uint32_t o_r = __builtin_amdgcn_readfirstlane(a.x);
            const uint32_t o_s = __builtin_amdgcn_readfirstlane(a.y);
            ga[j] = (g32 + o_r)[zc];
            gb[j] = (g32 + o_s)[zc];
        }
    };
    auto store = [&](int buf, int s) {
        float re[8], im[8];
        float t = 0.0f, sp = 0.0f, sm = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint4 a = s_row[2 * (8 * s + j)];
            const uint4 b = s_row[2 * (8 * s + j) + 1];
            const float sw = __uint_as_float(a.z), mt = __uint_as_float(a.w);
            const float px = ga[j].x * gb[j].x - ga[j].y * gb[j].y;
            const float py = ga[j].x * gb[j].y + ga[j].y * gb[j].x;
            sp += px * __uint_as_float(b.x) + py * __uint_as_float(b.y);
            sm += px * __uint_as_float(b.z) + py * __uint_as_float(b.w);
            t += mt * (px * px + py * py);
            re[j] = sw * px;
            im[j] = sw * py;
        }
        tr += double(t);
        cp += double(sp);
        cm += double(sm);
        if (z < nz) {
            // z-row layout: real parts of the 8 rows, then imaginary parts
            float4* o = reinterpret_cast<float4*>(sh[buf] + z * C::STR);
            o[0] = make_float4(re[0], re[1], re[2], re[3]);
            o[1] = make_float4(re[4], re[5], re[6], re[7]);
            o[2] = make_float4(im[0], im[1], im[2], im[3]);
            o[3] = make_float4(im[4], im[5], im[6], im[7]);
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
    store(0, 0);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        if (s + 1 < nst) load(s + 1);
        compute(s & 1);
        if (s + 1 < nst) store((s + 1) & 1, s + 1);
        __syncthreads();
    }
    float* out = part + size_t(it.slot) * C::NTL * 1024;
    using S = SplitCfg<NT, 0>;
    if (wv == 0) f32_store_tiles<S, 0>(acc, out, lane, 1.0f, 0, 0);
    else if (wv == 1) f32_store_tiles<S, 1>(acc, out, lane, 1.0f, 0, 0);
    else if (wv == 2) f32_store_tiles<S, 2>(acc, out, lane, 1.0f, 0, 0);
    else f32_store_tiles<S, 3>(acc, out, lane, 1.0f, 0, 0);
    double* rp = rpart + size_t(it.slot) * rpart_width(nz);
    if (z < nz) {
        rp[z] = cp;
        rp[nz + z] = cm;
    }
    const double t = wave_sum(z < nz ? tr : 0.0);
    if (lane == 0) s_tr[wv] = t;
    __syncthreads();
    if (tid == 0) rp[2 * nz] = (s_tr[0] + s_tr[1]) + (s_tr[2] + s_tr[3]);
}

// ------------------------------------------------------------------ FP64 ---
// FP64 Gram task: the same super-block tasks as the split kernels, on
// 16 x 16 tiles (v_mfma_f64_16x16x4): NB (NBJ) 16-wide blocks in the I (J)
// set, lower triangle (diagonal task) or NB x NBJ rectangle, over 8 waves.
template <int NT, int NTJ>
struct F64Cfg {
    static constexpr bool RECT = NTJ > 0;
    static constexpr int NZPI = 32 * NT, NZPJ = 32 * NTJ, NZP = NZPI + NZPJ;
    static constexpr int NB = 2 * NT, NBJ = 2 * NTJ;
    static constexpr int NBL = RECT ? NB * NBJ : NB * (NB + 1) / 2;
    static constexpr int TPW = (NBL + 7) / 8;   // 8 waves
    __host__ __device__ static constexpr int tI(int t) { return RECT ? t / NBJ : tri_I(t); }
    __host__ __device__ static constexpr int tJ(int t) { return RECT ? t % NBJ : tri_J(t); }
    __host__ __device__ static constexpr uint32_t maskI(int t0, int t1) {
        uint32_t m = 0;
        for (int t = t0; t < t1; ++t) m |= RECT ? (1u << tI(t)) : ((1u << tI(t)) | (1u << tJ(t)));
        return m;
    }
    __host__ __device__ static constexpr uint32_t maskJ(int t0, int t1) {
        uint32_t m = 0;
        if (RECT)
            for (int t = t0; t < t1; ++t) m |= 1u << tJ(t);
        return m;
    }
};

template <class C, int W>
__device__ __forceinline__ void f64_wave_mfma(f64x4 (&acc)[C::TPW], const double* sh, int lane) {
    constexpr int t0 = W * C::TPW;
    constexpr int t1 = (t0 + C::TPW < C::NBL) ? t0 + C::TPW : C::NBL;
    constexpr uint32_t needI = t0 < t1 ? C::maskI(t0, t1) : 0u;
    constexpr uint32_t needJ = t0 < t1 ? C::maskJ(t0, t1) : 0u;
    constexpr int NBJX = C::RECT ? C::NBJ : 1;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        double fa[C::NB], fb[NBJX];
        const int roff = (4 * s + (lane >> 4)) * C::NZP + (lane & 15);
#pragma unroll
        for (int b = 0; b < C::NB; ++b)
            if (needI & (1u << b)) fa[b] = sh[roff + 16 * b];
        if constexpr (C::RECT) {
#pragma unroll
            for (int b = 0; b < NBJX; ++b)
                if (needJ & (1u << b)) fb[b] = sh[roff + C::NZPI + 16 * b];
        }
#pragma unroll
        for (int m = 0; m < C::TPW; ++m) {
            const int t = t0 + m;
            if (t < t1) {
                const int I = C::tI(t), J = C::tJ(t);
                const double bj = C::RECT ? fb[J] : fa[J];
                acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[I], bj, acc[m], 0, 0, 0);
            }
        }
    }
}

// Store 16 x 16 tiles into the 32 x 32 tile layout of the item's partial:
// global 16-blocks (2 bI0 + I, 2 bJ0 + J).
template <class C, int W>
__device__ __forceinline__ void f64_store_tiles(const f64x4 (&acc)[C::TPW], double* out, int lane,
                                                int bI0, int bJ0) {
    constexpr int t0 = W * C::TPW;
#pragma unroll
    for (int m = 0; m < C::TPW; ++m) {
        const int t = t0 + m;
        if (t < C::NBL) {
            const int I = 2 * bI0 + C::tI(t), J = 2 * bJ0 + C::tJ(t);
            const int T = (I / 2) * (I / 2 + 1) / 2 + J / 2;   // 32-tile index
            double* o = out + size_t(T) * 1024 + (I & 1) * 16 * 32 + (J & 1) * 16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // v_mfma_f64_16x16x4: lane l, register v holds row 4 v + l/16, column l%16
                const int i = 4 * v + (lane >> 4);
                __builtin_nontemporal_store(acc[m][v], &o[i * 32 + (lane & 15)]);
            }
        }
    }
}

// only: when set, items of pairs p with only[p] <= 0 are skipped; gate: when
// set and zero, the launch does nothing.  With fewer blocks than schedule
// entries the blocks loop over the schedule (a multiple of 8 blocks keeps
// every entry on its XCD).
// Thread t owns depth z = t % 256 of the I set (and of the J set) and the rows
// j = t / 256 + 2 i (i < 4) of each stage (the row is uniform across a wave,
// so its data come through scalar loads).  A diagonal task also yields the
// item's exact FP64 right-hand side c+-(z) = Re(A^H B+-) over its depths and
// its trace sum mult |A|^2 in rpart[slot].
template <int NT, int NTJ>
__global__ __launch_bounds__(512, 1) void gram_f64_kernel(const Item* __restrict__ items,
                                                          const int32_t* __restrict__ sched,
                                                          const GRow* __restrict__ grow,
                                                          const double* __restrict__ gsc,
                                                          const zd* __restrict__ ubw,
                                                          const zd* __restrict__ g64, int nz, int zI0,
                                                          int zJ0, int ntot, double* __restrict__ part,
                                                          double* __restrict__ rpart,
                                                          const int32_t* __restrict__ only, int nsched,
                                                          const int32_t* __restrict__ gate) {
    using C = F64Cfg<NT, NTJ>;
    __shared__ __attribute__((aligned(16))) double sh[2][16 * C::NZP];
    __shared__ double s_tr[8];
    if (gate && *gate == 0) return;   // nothing selected: one load
    // block b takes schedule entries b, b + G, ... (one each when G = nsched)
    for (int ks = blockIdx.x; ks < nsched; ks += gridDim.x) {
    const int32_t k = sched[ks];
    if (k < 0) continue;   // hole in the XCD-aware schedule
    const Item it = items[k];
    if (only && only[it.pair] <= 0) continue;   // pair not selected
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = it.row_end - it.row_begin;
    const int nst = (n + 7) >> 3;
    const int z = tid & 255, hf = __builtin_amdgcn_readfirstlane(tid >> 8);
    const int nzI = min(C::NZPI, nz - zI0);
    const bool onI = z < nzI, onJ = C::RECT && z < C::NZPJ;
    const int zIc = zI0 + min(z, nzI - 1), zJc = min(zJ0 + z, nz - 1);
    // depths past nz of the I set stay zero for the whole item
    if (z >= nzI && z < C::NZPI)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 8; ++q) sh[b][(2 * (hf + 2 * (q >> 1)) + (q & 1)) * C::NZP + z] = 0.0;
    f64x4 acc[C::TPW];
#pragma unroll
    for (int m = 0; m < C::TPW; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[m][v] = 0.0;
    zd ga[4], gb[4], ha[4], hb[4], bp[4], bm[4];
    double sw[4];
    double cp = 0.0, cm = 0.0, tr = 0.0;
    auto load = [&](int s) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = s * 8 + hf + 2 * i;
            const int64_t row = int64_t(it.row_begin) + min(r, n - 1);
            const GRow g = grow[row];
            ga[i] = g64[size_t(g.off_r) + zIc];
            gb[i] = g64[size_t(g.off_s) + zIc];
            if constexpr (C::RECT) {
                ha[i] = g64[size_t(g.off_r) + zJc];
                hb[i] = g64[size_t(g.off_s) + zJc];
            }
            const bool on = r < n;
            if constexpr (!C::RECT) {
                const zd b0 = ubw[2 * row], b1 = ubw[2 * row + 1];
                bp[i] = on ? b0 : zd{0.0, 0.0};
                bm[i] = on ? b1 : zd{0.0, 0.0};
            }
            sw[i] = on ? gsc[row] : 0.0;
        }
    };
    auto store = [&](int buf) {
        double* o = sh[buf];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = hf + 2 * i;
            const zd p = ga[i] * gb[i];
            if constexpr (!C::RECT) {
                cp += p.x * bp[i].x + p.y * bp[i].y;
                cm += p.x * bm[i].x + p.y * bm[i].y;
            }
            const double ax = sw[i] * p.x, ay = sw[i] * p.y;
            if constexpr (!C::RECT) tr += ax * ax + ay * ay;
            if (onI) {
                o[(2 * j) * C::NZP + z] = ax;
                o[(2 * j + 1) * C::NZP + z] = ay;
            }
            if constexpr (C::RECT) {
                const zd q = ha[i] * hb[i];
                if (onJ) {
                    o[(2 * j) * C::NZP + C::NZPI + z] = sw[i] * q.x;
                    o[(2 * j + 1) * C::NZP + C::NZPI + z] = sw[i] * q.y;
                }
            }
        }
    };
    auto compute = [&](int buf) {
        const double* o = sh[buf];
        switch (wv) {
            case 0: f64_wave_mfma<C, 0>(acc, o, lane); break;
            case 1: f64_wave_mfma<C, 1>(acc, o, lane); break;
            case 2: f64_wave_mfma<C, 2>(acc, o, lane); break;
            case 3: f64_wave_mfma<C, 3>(acc, o, lane); break;
            case 4: f64_wave_mfma<C, 4>(acc, o, lane); break;
            case 5: f64_wave_mfma<C, 5>(acc, o, lane); break;
            case 6: f64_wave_mfma<C, 6>(acc, o, lane); break;
            default: f64_wave_mfma<C, 7>(acc, o, lane); break;
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
    double* out = part + size_t(it.slot) * (ntot * (ntot + 1) / 2) * 1024;
    const int bI0 = zI0 / 32, bJ0 = C::RECT ? zJ0 / 32 : zI0 / 32;
    switch (wv) {
        case 0: f64_store_tiles<C, 0>(acc, out, lane, bI0, bJ0); break;
        case 1: f64_store_tiles<C, 1>(acc, out, lane, bI0, bJ0); break;
        case 2: f64_store_tiles<C, 2>(acc, out, lane, bI0, bJ0); break;
        case 3: f64_store_tiles<C, 3>(acc, out, lane, bI0, bJ0); break;
        case 4: f64_store_tiles<C, 4>(acc, out, lane, bI0, bJ0); break;
        case 5: f64_store_tiles<C, 5>(acc, out, lane, bI0, bJ0); break;
        case 6: f64_store_tiles<C, 6>(acc, out, lane, bI0, bJ0); break;
        default: f64_store_tiles<C, 7>(acc, out, lane, bI0, bJ0); break;
    }
    if constexpr (!C::RECT) {
        // the two row halves of depth z meet in LDS (stage buffers are free now)
        double* sc = sh[0];
        if (hf == 1) {
            sc[z] = cp;
            sc[256 + z] = cm;
        }
        const double t = wave_sum(onI ? tr : 0.0);
        if (lane == 0) s_tr[wv] = t;
        __syncthreads();
        double* rp = rpart + size_t(it.slot) * rpart_width(nz);
        if (hf == 0 && onI) {
            rp[zI0 + z] = cp + sc[z];
            rp[nz + zI0 + z] = cm + sc[256 + z];
        }
        if (tid == 0)
            rp[2 * nz + zI0 / kSuperDepth] =
                ((s_tr[0] + s_tr[1]) + (s_tr[2] + s_tr[3])) + ((s_tr[4] + s_tr[5]) + (s_tr[6] + s_tr[7]));
    }
    __syncthreads();   // LDS is reused by the next entry
    }
}

// ---------------------------------------------------------------- reduce ---
// gram[p][zi][zj] (zi >= zj) = sum over the pair's items of the partial tiles,
// accumulated in FP64 in item order.  Grid: (n_pairs, lower 32-tiles).
// only: when set, pairs with only[p] <= 0 are skipped (also below).
template <class T>
__global__ __launch_bounds__(256) void gram_reduce_kernel(const T* __restrict__ part,
                                                          const int32_t* __restrict__ pair_item,
                                                          int nz, int ntl, double* __restrict__ gram,
                                                          const int32_t* __restrict__ only) {
    const int p = blockIdx.x, t = blockIdx.y;
    if (only && only[p] <= 0) return;
    const int I = tri_I(t), J = tri_J(t);
    const int k0 = pair_item[p], k1 = pair_item[p + 1];
    double* G = gram + size_t(p) * nz * nz;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int e = threadIdx.x + 256 * m;
        const int i = e >> 5, j = e & 31;
        const int zi = 32 * I + i, zj = 32 * J + j;
        if (zi >= nz || zj > zi) continue;
        // eight independent partial sums keep eight loads in flight; the
        // combination order is fixed (deterministic)
        const T* src = part + size_t(t) * 1024 + e;
        const size_t stride = size_t(ntl) * 1024;
        double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int k = k0;
        for (; k + 8 <= k1; k += 8)
#pragma unroll
            for (int q = 0; q < 8; ++q) s8[q] += double(__builtin_nontemporal_load(src + size_t(k + q) * stride));
        for (int q = 0; k < k1; ++k, ++q) s8[q] += double(__builtin_nontemporal_load(src + size_t(k) * stride));
        G[size_t(zi) * nz + zj] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    }
}

// rhs[p][h][z] and trace[p] from the per-item partials, in item order (the
// trace: per super-block over the items, then over the super-blocks).
__global__ __launch_bounds__(256) void rhs_reduce_kernel(const double* __restrict__ rpart,
                                                         const int32_t* __restrict__ pair_item,
                                                         int nz, double* __restrict__ rhs,
                                                         double* __restrict__ trace,
                                                         const int32_t* __restrict__ only) {
    __shared__ double s_t[8];
    const int p = blockIdx.x;
    if (only && only[p] <= 0) return;
    const int k0 = pair_item[p], k1 = pair_item[p + 1];
    const int w = rpart_width(nz);
    for (int e = threadIdx.x; e < w; e += 256) {
        double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int k = k0;
        for (; k + 8 <= k1; k += 8)
#pragma unroll
            for (int q = 0; q < 8; ++q) s8[q] += rpart[size_t(k + q) * w + e];
        for (int q = 0; k < k1; ++k, ++q) s8[q] += rpart[size_t(k) * w + e];
        const double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
        if (e < 2 * nz) rhs[size_t(p) * 2 * nz + e] = s;
        else s_t[e - 2 * nz] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int b = 0; b < n_super(nz); ++b) t += s_t[b];
        trace[p] = t;
    }
}

// gmax[f][c] = max_z |g32[f][c][z]| (FP32), for the FP16 row scaling.
// One wave per table column.
__global__ __launch_bounds__(256) void gmax_kernel(const float2* __restrict__ g32, int64_t ncol, int nz,
                                                   float* __restrict__ gmax) {
    const int lane = threadIdx.x & 63;
    const int64_t c = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (c >= ncol) return;
    float m = 0.0f;
    for (int z = lane; z < nz; z += 64) {
        const float2 v = g32[c * nz + z];
        m = fmaxf(m, sqrtf(v.x * v.x + v.y * v.y));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    // rounded up by a few ulps: the bound must not be below the true maximum
    if (lane == 0) gmax[c] = m * 1.0001f;
}

// ------------------------------------------------------------- launchers ---
// dynamic LDS of the FP32 / split kernels: the row records of an item,
// padded to a multiple of 8 rows plus the split kernels' padding stages, 32
// bytes each
size_t row_lds_bytes(int64_t chunk_rows) { return size_t((chunk_rows + 7) / 8 + kPadStages) * 8 * 32; }

// Row data the Gram kernels read besides the tables (formed by bsum_kernel).
struct GramRowData {
    const zd* ubw;        // FP64: conj(W) (b+, b-)
    const float4* ub32;   // FP32 / split: conj(W)/|W| (b+, b-)
    const float* gmax;    // FP16x3: max_z |g32| per table column
    const int32_t* only;  // FP64: when set, only the pairs with only[p] > 0
    const int32_t* gate;  // FP64: when set and zero, nothing to do
};

// Diagonal split tasks run the unified kernel unless EDT_SPLIT_SPECIALISED is
// set in the environment (the warp-specialised kernel, kept for comparison).
static bool split_unified() {
    static const bool u = std::getenv("EDT_SPLIT_SPECIALISED") == nullptr;
    return u;
}

// One Gram task kind (diagonal NTJ = 0 or rectangular) over every item.
template <int NT, int NTJ>
static hipError_t launch_gram_task(const edt_plan* p, edt_precision prec, const zd* g64,
                                   const float2* g32, const GramRowData& rd, void* part, double* rpart,
                                   int zI0, int zJ0, int ntot, hipStream_t st) {
    // (rd.only applies to the FP64 kernel)
    const Item* items = dptr<const Item>(p, p->lay.items);
    const int32_t* sched = dptr<const int32_t>(p, p->lay.sched);
    const GRow* grow = dptr<const GRow>(p, p->lay.grow);
    const unsigned nb = unsigned(p->sched.size());
    // a gated (rarely needed) FP64 pass runs on a small persistent grid
    const unsigned grid = rd.gate ? std::min(nb, 512u) : nb;
    if ((prec == EDT_BF16X3 || prec == EDT_FP16X3) && NTJ == 0 && split_unified()) {
        if (prec == EDT_BF16X3)
            hipLaunchKernelGGL((gram_split3p_kernel<NT, false>), dim3(nb), dim3(512), row_lds_bytes(p->chunk_rows),
                               st, items, sched, grow, rd.ub32, g32, rd.gmax, p->nz, zI0, ntot,
                               static_cast<float*>(part), rpart, p->chunk_rows);
        else
            hipLaunchKernelGGL((gram_split3p_kernel<NT, true>), dim3(nb), dim3(512), row_lds_bytes(p->chunk_rows),
                               st, items, sched, grow, rd.ub32, g32, rd.gmax, p->nz, zI0, ntot,
                               static_cast<float*>(part), rpart, p->chunk_rows);
    } else if (prec == EDT_BF16X3)
        hipLaunchKernelGGL((gram_split3_kernel<NT, NTJ, false>), dim3(nb), dim3(512),
                           row_lds_bytes(p->chunk_rows), st, items, sched, grow, rd.ub32, g32, rd.gmax,
                           p->nz, zI0, zJ0, ntot, static_cast<float*>(part), rpart, p->chunk_rows);
    else if (prec == EDT_FP16X3)
        hipLaunchKernelGGL((gram_split3_kernel<NT, NTJ, true>), dim3(nb), dim3(512),
                           row_lds_bytes(p->chunk_rows), st, items, sched, grow, rd.ub32, g32, rd.gmax,
                           p->nz, zI0, zJ0, ntot, static_cast<float*>(part), rpart, p->chunk_rows);
    else if (prec == EDT_FP64) {
        if constexpr (NTJ <= 4)
            hipLaunchKernelGGL((gram_f64_kernel<NT, NTJ>), dim3(grid), dim3(512), 0, st, items, sched, grow,
                               dptr<const double>(p, p->lay.gsc), rd.ubw, g64, p->nz, zI0, zJ0, ntot,
                               static_cast<double*>(part), rpart, rd.only, int(nb), rd.gate);
        else
            return hipErrorInvalidValue;   // FP64 rectangles are half super-blocks
    } else if constexpr (NTJ == 0)
        hipLaunchKernelGGL(gram_f32_kernel<NT>, dim3(nb), dim3(256), row_lds_bytes(p->chunk_rows), st,
                           items, sched, grow, rd.ub32, g32, p->nz, static_cast<float*>(part), rpart,
                           p->chunk_rows);
    else
        return hipErrorInvalidValue;   // FP32 Gram: depth counts up to 256 only
    return hipGetLastError();
}

// Split rectangles over a whole earlier super-block (8 J blocks) for I sets
// of at most this many blocks: 8 NT tiles, 2 NT per MFMA wave, fit its
// registers; larger I sets take the two halves of the super-block in turn.
constexpr int kWideRectMaxNT = 5;

template <int NTJ>
static hipError_t launch_gram_nt(int nt, const edt_plan* p, edt_precision prec, const zd* g64,
                                 const float2* g32, const GramRowData& rd, void* part, double* rpart,
                                 int zI0, int zJ0, int ntot, hipStream_t st) {
    switch (nt) {
#define EDT_CASE(N) \
    case N: return launch_gram_task<N, NTJ>(p, prec, g64, g32, rd, part, rpart, zI0, zJ0, ntot, st);
        EDT_CASE(1) EDT_CASE(2) EDT_CASE(3) EDT_CASE(4) EDT_CASE(5) EDT_CASE(6) EDT_CASE(7) EDT_CASE(8)
#undef EDT_CASE
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_gram_wide(int nt, const edt_plan* p, edt_precision prec, const zd* g64,
                                   const float2* g32, const GramRowData& rd, void* part, double* rpart,
                                   int zI0, int zJ0, int ntot, hipStream_t st) {
    static_assert(kWideRectMaxNT == 5, "the cases below");
    switch (nt) {
#define EDT_CASE(N) \
    case N: return launch_gram_task<N, 8>(p, prec, g64, g32, rd, part, rpart, zI0, zJ0, ntot, st);
        EDT_CASE(1) EDT_CASE(2) EDT_CASE(3) EDT_CASE(4) EDT_CASE(5)
#undef EDT_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int NT, int NTJ>
static hipError_t configure_gram_task() {
    const int bytes = int(row_lds_bytes(2048));
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_split3_kernel<NT, NTJ, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_split3_kernel<NT, NTJ, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess && NTJ == 0)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_split3p_kernel<NT, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess && NTJ == 0)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_split3p_kernel<NT, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess && NTJ == 0)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_f32_kernel<NT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

template <int NT>
static hipError_t configure_gram_nt() {
    hipError_t e = configure_gram_task<NT, 0>();
    if (e == hipSuccess) e = configure_gram_task<NT, 4>();
    if constexpr (NT <= kWideRectMaxNT)
        if (e == hipSuccess) e = configure_gram_task<NT, 8>();
    return e;
}

// Allow the largest item size (2048 rows) for every task shape.
hipError_t configure_gram_kernels() {
    hipError_t e = configure_gram_nt<1>();
    if (e == hipSuccess) e = configure_gram_nt<2>();
    if (e == hipSuccess) e = configure_gram_nt<3>();
    if (e == hipSuccess) e = configure_gram_nt<4>();
    if (e == hipSuccess) e = configure_gram_nt<5>();
    if (e == hipSuccess) e = configure_gram_nt<6>();
    if (e == hipSuccess) e = configure_gram_nt<7>();
    if (e == hipSuccess) e = configure_gram_nt<8>();
    return e;
}

hipError_t launch_gmax(const edt_plan* p, const float2* g32, float* gmax, hipStream_t st) {
    const int64_t ncol = int64_t(p->n_freq) * p->n_cls;
    if (ncol == 0) return hipSuccess;
    hipLaunchKernelGGL(gmax_kernel, dim3(unsigned((ncol + 3) / 4)), dim3(256), 0, st, g32, ncol, p->nz, gmax);
    return hipGetLastError();
}

// The item partials of all tasks: a diagonal task per depth super-block and,
// for each pair of super-blocks sbi > sbj, the rectangle between them: for
// the split Grams with an I set of at most kWideRectMaxNT blocks one task
// over all of super-block sbj (which is full: only the last one can be
// partial), otherwise two tasks over its halves (128 depths).
hipError_t launch_gram(const edt_plan* p, edt_precision prec, const zd* g64, const float2* g32,
                       const zd* ubw, const float4* ub32, const float* gmax, void* part, double* rpart,
                       hipStream_t st, const int32_t* only, const int32_t* gate) {
    if (p->sched.empty()) return hipSuccess;
    const int nz = p->nz, ntot = (nz + 31) / 32, ns = n_super(nz);
    if (prec == EDT_FP32 && ns > 1) return hipErrorInvalidValue;
    if ((only || gate) && prec != EDT_FP64) return hipErrorInvalidValue;
    const GramRowData rd{ubw, ub32, gmax, only, gate};
    auto nt_of = [&](int sb) { return (std::min(kSuperDepth, nz - kSuperDepth * sb) + 31) / 32; };
    for (int sb = 0; sb < ns; ++sb) {
        const hipError_t e =
            launch_gram_nt<0>(nt_of(sb), p, prec, g64, g32, rd, part, rpart, kSuperDepth * sb, 0, ntot, st);
        if (e != hipSuccess) return e;
    }
    const bool split = prec == EDT_BF16X3 || prec == EDT_FP16X3;
    for (int sbi = 1; sbi < ns; ++sbi)
        for (int sbj = 0; sbj < sbi; ++sbj) {
            if (split && nt_of(sbi) <= kWideRectMaxNT) {
                const hipError_t e = launch_gram_wide(nt_of(sbi), p, prec, g64, g32, rd, part, rpart,
                                                      kSuperDepth * sbi, kSuperDepth * sbj, ntot, st);
                if (e != hipSuccess) return e;
                continue;
            }
            for (int h = 0; h < 2; ++h) {
                const hipError_t e = launch_gram_nt<4>(nt_of(sbi), p, prec, g64, g32, rd, part, rpart,
                                                       kSuperDepth * sbi, kSuperDepth * sbj + 128 * h, ntot, st);
                if (e != hipSuccess) return e;
            }
        }
    return hipSuccess;
}

hipError_t launch_gram_reduce(const edt_plan* p, edt_precision prec, const void* part, double* gram,
                              hipStream_t st, const int32_t* only) {
    const int NT = (p->nz + 31) / 32;
    const int ntl = NT * (NT + 1) / 2;
    const int32_t* pair_item = dptr<const int32_t>(p, p->lay.pair_item);
    if (p->n_pairs == 0) return hipSuccess;
    if (prec == EDT_FP64)
        hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3(unsigned(p->n_pairs), ntl), dim3(256), 0,
                           st, static_cast<const double*>(part), pair_item, p->nz, ntl, gram, only);
    else
        hipLaunchKernelGGL(gram_reduce_kernel<float>, dim3(unsigned(p->n_pairs), ntl), dim3(256), 0,
                           st, static_cast<const float*>(part), pair_item, p->nz, ntl, gram, only);
    return hipGetLastError();
}

hipError_t launch_rhs_reduce(const edt_plan* p, const double* rpart, double* rhs, double* trace,
                             hipStream_t st, const int32_t* only) {
    if (p->n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(rhs_reduce_kernel, dim3(unsigned(p->n_pairs)), dim3(256), 0, st, rpart,
                       dptr<const int32_t>(p, p->lay.pair_item), p->nz, rhs, trace, only);
    return hipGetLastError();
}

}  // namespace edt
