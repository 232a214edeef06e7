// FP64 row kernels: right-hand sides, trace, refinement residual, forward map.
//
// Paper, Section 2.1, eqs. DMV and Split: for a pair with rows A (complex)
// and data b+ = (d(k_m) + d(-k_m))/2, b- = (d(k_m) - d(-k_m))/(2i), the real
// unknowns x+- satisfy the normal equations with right-hand side
// c+- = Re(A^H b+-).  The refinement residual of the damped system is
// Re(A^H (b - A x)) - lambda x.  Rows are rebuilt in FP64 from the Green's
// table, A = W g(k_r) g(k_s), W = w^2 dz, and never stored.
//
// Rows that stand for several data rows (same frequency and |k_r|,|k_s|) are
// processed once: their data are summed (bsum_kernel) and their A x term is
// weighted by the multiplicity.
//
// Layout: a 256-thread block per work item; each wave takes its own rows,
// lanes span depth (ZPL depths per lane).  A x needs a sum over depth per
// row: two rows at a time are reduced with a transposing butterfly of lane
// swaps and DPP moves, so a row costs about one cross-lane exchange per lane
// instead of six.  Up to 256 depths the table columns of a wave's next two
// rows are loaded while the current two compute.

#include "dev_common.h"

namespace edt {

// Cross-lane moves of a double as two 32-bit halves.
// permlane32_swap: lanes 32..63 of x trade places with lanes 0..31 of y.
// permlane16_swap: rows 1 and 3 (16 lanes each) of x trade places with rows
// 0 and 2 of y.  mov_dpp<CTRL>: the DPP lane pattern CTRL within each row.
__device__ __forceinline__ void swap32_d(double& x, double& y) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
    x = __hiloint2double(int(hi[0]), int(lo[0]));
    y = __hiloint2double(int(hi[1]), int(lo[1]));
}
__device__ __forceinline__ void swap16_d(double& x, double& y) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
    x = __hiloint2double(int(hi[0]), int(lo[0]));
    y = __hiloint2double(int(hi[1]), int(lo[1]));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    return __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false),
                            __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false));
}
constexpr int kDppRowMirror = 0x140;       // lane i <- lane 15 - i of its row
constexpr int kDppRowHalfMirror = 0x141;   // lane i <- lane 7 - i of its half row
constexpr int kDppQuadXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppQuadXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]

// Sum each of 8 per-lane values (two rows' four partial dot products) over
// the 64 lanes; every lane receives all 8 totals.  Three halving steps leave
// lane l with the partial total of index 4*b5 + 2*b4 + b3 (b = bits of l):
// the lane swaps pair l with l ^ 32 and l ^ 16, the row mirror pairs l with a
// lane of the other bit-3 half of its row; the half-row mirror (which flips
// bits 0-2) and two quad exchanges sum the 8 lanes of each group.  No step
// goes through LDS.  The input array is overwritten.
__device__ __forceinline__ void butterfly8(double (&a)[8], double (&out)[8], int lane) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {   // bit 5
        double x = a[i], y = a[i + 4];
        swap32_d(x, y);
        a[i] = x + y;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {   // bit 4
        double x = a[i], y = a[i + 2];
        swap16_d(x, y);
        a[i] = x + y;
    }
    const bool b3 = lane & 8;
    const double lo = a[0] + dpp_d<kDppRowMirror>(a[0]);
    const double hi = a[1] + dpp_d<kDppRowMirror>(a[1]);
    double s = b3 ? hi : lo;   // bit 3
    s += dpp_d<kDppRowHalfMirror>(s);
    s += dpp_d<kDppQuadXor2>(s);
    s += dpp_d<kDppQuadXor1>(s);
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = readlane_d(s, k << 3);
}


// ub[u] = (sum of b+ over the data rows of unique row u, sum of b-) (ub
// nullable: the Gram and refinement read only the weighted forms below).
// Optionally also the data as the Gram kernels consume them (the right-hand
// side c = Re(A^H B) with A = W g g):
//   ubw[u]  = conj(W) ub             (FP64 rows are built without W)
//   ub32[u] = conj(W) / |W| ub, FP32 (FP32 rows already carry |W|)
template <class D>
__global__ __launch_bounds__(256) void bsum_kernel(const int32_t* __restrict__ umem_off,
                                                   const int32_t* __restrict__ umem,
                                                   const D* __restrict__ d_rows, int64_t U,
                                                   zd* __restrict__ ub, const uint32_t* __restrict__ urows,
                                                   const double* __restrict__ freq, double eps, double dz,
                                                   zd* __restrict__ ubw, float4* __restrict__ ub32) {
    const int64_t u = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (u >= U) return;
    zd bp{0.0, 0.0}, bm{0.0, 0.0};
    for (int k = umem_off[u]; k < umem_off[u + 1]; ++k) {
        const int64_t r = umem[k];
        const zd d0 = load_datum(d_rows, 2 * r), d1 = load_datum(d_rows, 2 * r + 1);
        bp = bp + 0.5 * (d0 + d1);
        const zd df = d0 - d1;                    // (d0 - d1) / (2i) = -i (d0 - d1) / 2
        bm = bm + zd{0.5 * df.y, -0.5 * df.x};
    }
    if (ub) {
        ub[2 * u] = bp;
        ub[2 * u + 1] = bm;
    }
    if (ubw || ub32) {
        const uint32_t a = urows[2 * u];
        const zd w = omega_of(freq[a & 0xFFFFu], eps);
        const zd cW = zconj(dz * (w * w));
        if (ubw) {
            ubw[2 * u] = cW * bp;
            ubw[2 * u + 1] = cW * bm;
        }
        if (ub32) {
            const zd ph = (1.0 / sqrt(zabs2(cW))) * cW;
            const zd a = ph * bp, b = ph * bm;
            ub32[u] = make_float4(float(a.x), float(a.y), float(b.x), float(b.y));
        }
    }
}

// Refinement residual, partial over one work item (a pair's rows within a
// group of frequencies):  r+-(z) = Re(A^H (B+- - mult A x+-)), written to
// rpart[slot][h*nz + z].  With A = W p, p = g(k_r) g(k_s) and the row data
// ubw = conj(W) B from bsum_kernel, a row contributes
//   Re(conj(p) (ubw - |W|^2 mult (p . x))),   |W|^2 mult = gsc^2.
// Without DATA the row data are taken as zero and the kernel returns the
// partial of -Re(A^H A) x (the operator applied to a search direction).
// Rows past the item (padding of the last batch) get zero data and weight and
// depths past nz get x = 0, so no per-element masking is needed; the depths
// past nz are never stored.  PIPE: two column buffers in turn (two waves per
// SIMD); without, one buffer (three waves per SIMD up to 384 depths).
template <int ZPL, int RB, bool DATA, bool PIPE = (ZPL <= 4)>
__global__ __launch_bounds__(256, PIPE || ZPL > 4 ? 2 : 3) void resid_kernel(const Item* __restrict__ items,
                                                    const int32_t* __restrict__ sched,
                                                    const GRow* __restrict__ grow,
                                                    const double* __restrict__ gsc,
                                                    const zd* __restrict__ ubw,
                                                    const zd* __restrict__ g64, int nz,
                                                    const double* __restrict__ x,
                                                    const int32_t* __restrict__ conv,
                                                    double* __restrict__ rpart, int nsched,
                                                    const int32_t* __restrict__ active) {
    static_assert(RB == 2, "two rows per wave per batch (one 8-value reduction)");
    __shared__ double s_acc[4][2][ZPL * 64];
    // no pair left iterating: the whole sweep is skipped with one load
    if (active && *active == 0) return;
    // persistent blocks: block b takes schedule entries b, b + G, ... (G a
    // multiple of the XCD count, so every entry keeps its XCD)
    for (int ks = blockIdx.x; ks < nsched; ks += gridDim.x) {
    const int32_t k = sched[ks];
    if (k < 0) continue;   // hole in the XCD-aware schedule
    const Item it = items[k];
    if (conv[it.pair]) continue;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: row data via scalar loads
    const int n = it.row_end - it.row_begin;
    double xv[2][ZPL];
#pragma unroll
    for (int q = 0; q < ZPL; ++q) {
        const int z = lane + 64 * q;
        xv[0][q] = z < nz ? x[size_t(it.pair) * 2 * nz + z] : 0.0;
        xv[1][q] = z < nz ? x[size_t(it.pair) * 2 * nz + nz + z] : 0.0;
    }
    double acc[2][ZPL];
#pragma unroll
    for (int q = 0; q < ZPL; ++q) acc[0][q] = acc[1][q] = 0.0;

    // Software pipeline: the table columns of a batch are loaded while the
    // previous batch computes, and the column offsets of the batch after
    // that are fetched at the same time (one memory latency per batch,
    // overlapped with arithmetic).
    auto row_of = [&](int b, int j) { return int64_t(it.row_begin) + min(b + RB * wv + j, n - 1); };
    // depths lane + 64 q with q < ZPL - 1 are below nz; the last one is clamped
    const int zl = min(lane + 64 * (ZPL - 1), nz - 1) - lane;
    // two column buffers in turn: batch b computes from one while batch b + 1
    // is loaded into the other
    zd ar[RB][ZPL], as[RB][ZPL], br[RB][ZPL], bs[RB][ZPL];
    (void)br;
    (void)bs;
    GRow gn[RB];
    auto load_columns = [&](zd (&gr)[RB][ZPL], zd (&gs)[RB][ZPL], const GRow (&g)[RB]) {
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const zd* cr = g64 + g[j].off_r + lane;
            const zd* cs = g64 + g[j].off_s + lane;
#pragma unroll
            for (int q = 0; q < ZPL; ++q) {
                const int dz = q < ZPL - 1 ? 64 * q : zl;
                gr[j][q] = cr[dz];
                gs[j][q] = cs[dz];
            }
        }
    };
    auto compute = [&](const zd (&gr)[RB][ZPL], const zd (&gs)[RB][ZPL], int b0) {
        zd P[RB][ZPL];
#pragma unroll
        for (int j = 0; j < RB; ++j)
#pragma unroll
            for (int q = 0; q < ZPL; ++q) P[j][q] = gr[j][q] * gs[j][q];
        double v[4 * RB], y[4 * RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
            for (int q = 0; q < ZPL; ++q) {
                a0 += P[j][q].x * xv[0][q];
                a1 += P[j][q].y * xv[0][q];
                a2 += P[j][q].x * xv[1][q];
                a3 += P[j][q].y * xv[1][q];
            }
            v[4 * j] = a0;
            v[4 * j + 1] = a1;
            v[4 * j + 2] = a2;
            v[4 * j + 3] = a3;
        }
        // the rows' data and weights (scalar loads, used after the reduction)
        zd bp[RB], bm[RB];
        double w2[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const bool on = b0 + RB * wv + j < n;
            const int64_t row = row_of(b0, j);
            const double sc = gsc[row];
            if constexpr (DATA) {
                const zd b0v = ubw[2 * row], b1v = ubw[2 * row + 1];
                bp[j] = on ? b0v : zd{0.0, 0.0};
                bm[j] = on ? b1v : zd{0.0, 0.0};
            } else {
                bp[j] = bm[j] = zd{0.0, 0.0};
            }
            w2[j] = on ? sc * sc : 0.0;
        }
        butterfly8(v, y, lane);
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const zd cp{bp[j].x - w2[j] * y[4 * j], bp[j].y - w2[j] * y[4 * j + 1]};
            const zd cm{bm[j].x - w2[j] * y[4 * j + 2], bm[j].y - w2[j] * y[4 * j + 3]};
#pragma unroll
            for (int q = 0; q < ZPL; ++q) {
                acc[0][q] = fma(P[j][q].x, cp.x, acc[0][q]);
                acc[0][q] = fma(P[j][q].y, cp.y, acc[0][q]);
                acc[1][q] = fma(P[j][q].x, cm.x, acc[1][q]);
                acc[1][q] = fma(P[j][q].y, cm.y, acc[1][q]);
            }
        }
    };
    constexpr int B = 4 * RB;   // rows of a batch (all waves)
    if constexpr (!PIPE) {
        // one buffer: each batch waits for its own columns (beyond 256
        // depths two buffers would not leave registers for two waves)
        for (int b0 = 0; b0 < n; b0 += B) {
            GRow g[RB];
#pragma unroll
            for (int j = 0; j < RB; ++j) g[j] = grow[row_of(b0, j)];
            load_columns(ar, as, g);
            compute(ar, as, b0);
        }
    } else {
    {
        GRow g0[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) g0[j] = grow[row_of(0, j)];
        load_columns(ar, as, g0);
#pragma unroll
        for (int j = 0; j < RB; ++j) gn[j] = grow[row_of(B, j)];
    }
    // (the loads are unconditional, so that the waits stay exact: past the
    // item's end they read its last row again, and those values are unused)
    for (int b0 = 0; b0 < n; b0 += 2 * B) {
        load_columns(br, bs, gn);
#pragma unroll
        for (int j = 0; j < RB; ++j) gn[j] = grow[row_of(b0 + 2 * B, j)];
        compute(ar, as, b0);
        if (b0 + B >= n) break;
        load_columns(ar, as, gn);
#pragma unroll
        for (int j = 0; j < RB; ++j) gn[j] = grow[row_of(b0 + 3 * B, j)];
        compute(br, bs, b0 + B);
    }
    }
#pragma unroll
    for (int q = 0; q < ZPL; ++q) {
        s_acc[wv][0][q * 64 + lane] = acc[0][q];
        s_acc[wv][1][q * 64 + lane] = acc[1][q];
    }
    __syncthreads();
    double* out = rpart + size_t(it.slot) * (2 * nz + 1);
    for (int e = tid; e < 2 * nz; e += 256) {
        const int h = e / nz, z = e - h * nz;
        out[e] = (s_acc[0][h][z] + s_acc[1][h][z]) + (s_acc[2][h][z] + s_acc[3][h][z]);
    }
    __syncthreads();   // s_acc is reused by the next entry
    }
}

// Born forward map: for each unique row of an item, A.v[u] and A.v[-u],
// scattered to every data row it stands for (in the plan's data type).
template <class D>
__global__ __launch_bounds__(256) void forward_kernel(const uint32_t* __restrict__ urows,
                                                     const Item* __restrict__ items,
                                                     const int32_t* __restrict__ pair_u,
                                                     const int32_t* __restrict__ umem_off,
                                                     const int32_t* __restrict__ umem,
                                                     const zd* __restrict__ g64,
                                                     const double* __restrict__ freq, double eps,
                                                     double dz, int ncls, int nz,
                                                     const zd* __restrict__ v, D* __restrict__ d_rows) {
    const Item it = items[blockIdx.x];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int u0 = pair_u[2 * it.pair], u1 = pair_u[2 * it.pair + 1];
    for (int r = it.row_begin + wv; r < it.row_end; r += 4) {
        const URow u = load_urow(urows, r);
        const int64_t fb = int64_t(u.f) * ncls;
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        for (int z = lane; z < nz; z += 64) {
            const zd P = g64[(fb + u.cr) * nz + z] * g64[(fb + u.cs) * nz + z];
            const zd q0 = P * v[size_t(u0) * nz + z];
            const zd q1 = P * v[size_t(u1) * nz + z];
            a0 += q0.x;
            a1 += q0.y;
            a2 += q1.x;
            a3 += q1.y;
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        a3 = wave_sum(a3);
        const zd w = omega_of(freq[u.f], eps);
        const zd W = dz * (w * w);
        const zd d0 = W * zd{a0, a1}, d1 = W * zd{a2, a3};
        for (int k = umem_off[r] + lane; k < umem_off[r + 1]; k += 64) {
            const int64_t dr = umem[k];
            store_datum(d_rows, 2 * dr, d0);
            store_datum(d_rows, 2 * dr + 1, d1);
        }
    }
}

// ------------------------------------------------------------- launchers ---
hipError_t launch_bsum(const edt_plan* p, const void* d_rows, zd* ub, hipStream_t st, zd* ubw,
                       float4* ub32) {
    if (p->n_urows == 0) return hipSuccess;
    const unsigned blocks = unsigned((p->n_urows + 255) / 256);
    if (p->data_c64)
        hipLaunchKernelGGL(bsum_kernel<float2>, dim3(blocks), dim3(256), 0, st,
                           dptr<const int32_t>(p, p->lay.umem_off), dptr<const int32_t>(p, p->lay.umem),
                           static_cast<const float2*>(d_rows), p->n_urows, ub, dptr<const uint32_t>(p, p->lay.urows),
                           dptr<const double>(p, p->lay.freq), p->eps, p->dz, ubw, ub32);
    else
        hipLaunchKernelGGL(bsum_kernel<zd>, dim3(blocks), dim3(256), 0, st,
                           dptr<const int32_t>(p, p->lay.umem_off), dptr<const int32_t>(p, p->lay.umem),
                           static_cast<const zd*>(d_rows), p->n_urows, ub, dptr<const uint32_t>(p, p->lay.urows),
                           dptr<const double>(p, p->lay.freq), p->eps, p->dz, ubw, ub32);
    return hipGetLastError();
}

// Blocks of the persistent residual sweep at most (a multiple of 8: each
// schedule entry stays on its XCD).
constexpr int kResidGrid = 4096;

template <int ZPL>
static hipError_t launch_resid_z(const edt_plan* p, const zd* g64, const zd* ubw, const double* x,
                                 const int32_t* conv, double* rpart, const int32_t* active, hipStream_t st) {
    // rows per wave per batch: two (one 8-value reduction)
    constexpr int kRB = 2;
    const int nit = int(p->rsched.size());
    if (nit == 0) return hipSuccess;
    const unsigned grid = unsigned(std::min(nit, kResidGrid));
    const Item* items = dptr<const Item>(p, p->lay.ritems);
    const int32_t* sched = dptr<const int32_t>(p, p->lay.rsched);
    const GRow* grow = dptr<const GRow>(p, p->lay.grow);
    const double* gsc = dptr<const double>(p, p->lay.gsc);
    if (ubw)
        hipLaunchKernelGGL((resid_kernel<ZPL, kRB, true>), dim3(grid), dim3(256), 0, st, items, sched, grow, gsc, ubw,
                           g64, p->nz, x, conv, rpart, nit, active);
    else
        hipLaunchKernelGGL((resid_kernel<ZPL, kRB, false>), dim3(grid), dim3(256), 0, st, items, sched, grow, gsc,
                           ubw, g64, p->nz, x, conv, rpart, nit, active);
    return hipGetLastError();
}

hipError_t launch_resid(const edt_plan* p, const zd* g64, const zd* ubw, const double* x,
                        const int32_t* conv, double* rpart, hipStream_t st, const int32_t* active) {
    switch ((p->nz + 63) / 64) {
        case 1: return launch_resid_z<1>(p, g64, ubw, x, conv, rpart, active, st);
        case 2: return launch_resid_z<2>(p, g64, ubw, x, conv, rpart, active, st);
        case 3: return launch_resid_z<3>(p, g64, ubw, x, conv, rpart, active, st);
        case 4: return launch_resid_z<4>(p, g64, ubw, x, conv, rpart, active, st);
        case 5: return launch_resid_z<5>(p, g64, ubw, x, conv, rpart, active, st);
        case 6: return launch_resid_z<6>(p, g64, ubw, x, conv, rpart, active, st);
        case 7: return launch_resid_z<7>(p, g64, ubw, x, conv, rpart, active, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward(const edt_plan* p, const zd* g64, const zd* v, void* d_rows, hipStream_t st) {
    const unsigned nit = unsigned(p->items.size());
    if (nit == 0) return hipSuccess;
    if (p->data_c64)
        hipLaunchKernelGGL(forward_kernel<float2>, dim3(nit), dim3(256), 0, st, dptr<const uint32_t>(p, p->lay.urows),
                           dptr<const Item>(p, p->lay.items), dptr<const int32_t>(p, p->lay.pair_u),
                           dptr<const int32_t>(p, p->lay.umem_off), dptr<const int32_t>(p, p->lay.umem), g64,
                           dptr<const double>(p, p->lay.freq), p->eps, p->dz, p->n_cls, p->nz, v,
                           static_cast<float2*>(d_rows));
    else
        hipLaunchKernelGGL(forward_kernel<zd>, dim3(nit), dim3(256), 0, st, dptr<const uint32_t>(p, p->lay.urows),
                           dptr<const Item>(p, p->lay.items), dptr<const int32_t>(p, p->lay.pair_u),
                           dptr<const int32_t>(p, p->lay.umem_off), dptr<const int32_t>(p, p->lay.umem), g64,
                           dptr<const double>(p, p->lay.freq), p->eps, p->dz, p->n_cls, p->nz, v,
                           static_cast<zd*>(d_rows));
    return hipGetLastError();
}

}  // namespace edt
