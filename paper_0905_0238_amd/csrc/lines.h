// Shared pieces of the in-LDS line transforms (record and model transforms,
// finite-aperture rows).
#pragma once

#include "dev_common.h"

namespace edt {

// LDS layout of the line transforms: element i of line j sits at
// j * lds_stride(n) + lds_pad(i).  One pad slot per 8 elements spreads the
// strided accesses of the radix-8 passes (a thread's 8 elements at stride h,
// neighbouring threads 8 h apart) over the banks.
__host__ __device__ __forceinline__ constexpr int lds_stride(int n) { return n + (n >> 3); }
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 3); }

// R consecutive radix-2 levels of decimation in time (spans h, 2h, ..., R h / 2)
// in registers: a thread takes the R elements b0 + t h of one group, so a
// length 2^m takes ceil(m / 3) passes over LDS instead of m.  At the level of
// span H = lv h (blocks of M = 2H) element i pairs with i + H under the
// twiddle W_M^(i mod H), and i mod H = pos + (t mod lv) h.
template <int R>
__device__ __forceinline__ void dit_levels(zd* s_x, const zd* s_w, int n, int h, int L) {
    const int groups = n / R, ns = lds_stride(n);
    for (int g = threadIdx.x; g < L * groups; g += 256) {
        const int j = g / groups, gg = g - j * groups;
        const int pos = gg & (h - 1), blk = gg / h;
        zd* line = s_x + j * ns;
        const int b0 = blk * R * h + pos;
        zd x[R];
#pragma unroll
        for (int t = 0; t < R; ++t) x[t] = line[lds_pad(b0 + t * h)];
#pragma unroll
        for (int lv = 1; lv < R; lv <<= 1) {
            const int tstep = n / (2 * lv * h);
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if (t & lv) continue;
                const zd u = s_w[(pos + (t & (lv - 1)) * h) * tstep] * x[t + lv];
                x[t + lv] = x[t] - u;
                x[t] = x[t] + u;
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t) line[lds_pad(b0 + t * h)] = x[t];
    }
}

// Radix-2 decimation in time over L lines of n = 2^logn values in LDS (the
// padded layout above), loaded in bit-reversed order; natural order on return.
__device__ __forceinline__ void dit_lines(zd* s_x, const zd* s_w, int n, int logn, int L) {
    int h = 1;
    for (int rem = logn; rem > 0;) {
        if (rem >= 3) {
            dit_levels<8>(s_x, s_w, n, h, L);
            h *= 8;
            rem -= 3;
        } else if (rem == 2) {
            dit_levels<4>(s_x, s_w, n, h, L);
            h *= 4;
            rem -= 2;
        } else {
            dit_levels<2>(s_x, s_w, n, h, L);
            h *= 2;
            rem -= 1;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int bit_reverse(int i, int logn) {
    return logn ? int(__brev(unsigned(i)) >> (32 - logn)) : 0;
}

}  // namespace edt
