// Device helpers: complex double arithmetic and wave-level utilities (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "edt_internal.h"

namespace edt {

struct zd {
    double x, y;
};

__device__ __forceinline__ zd zmk(double x, double y) { return zd{x, y}; }
__device__ __forceinline__ zd operator+(zd a, zd b) { return zd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ zd operator-(zd a, zd b) { return zd{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ zd operator*(zd a, zd b) {
    return zd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ zd operator*(double s, zd a) { return zd{s * a.x, s * a.y}; }
__device__ __forceinline__ zd zconj(zd a) { return zd{a.x, -a.y}; }
__device__ __forceinline__ double zabs2(zd a) { return a.x * a.x + a.y * a.y; }

// a / b by Smith's method (avoids overflow of |b|^2).
__device__ __forceinline__ zd zdiv(zd a, zd b) {
    if (fabs(b.x) >= fabs(b.y)) {
        const double r = b.y / b.x, d = b.x + r * b.y;
        return zd{(a.x + a.y * r) / d, (a.y - a.x * r) / d};
    }
    const double r = b.x / b.y, d = b.y + r * b.x;
    return zd{(a.x * r + a.y) / d, (a.y * r - a.x) / d};
}

// exp(i k d) for complex k and real distance d >= 0.
__device__ __forceinline__ zd zexpi(zd k, double d) {
    double s, c;
    sincos(k.x * d, &s, &c);
    const double m = exp(-k.y * d);
    return zd{m * c, m * s};
}

// Principal square root (branch cut on the negative real axis): for an
// argument in the upper half plane the result lies in the first quadrant.
__device__ __forceinline__ zd zsqrt(zd a) {
    const double m = hypot(a.x, a.y);
    if (m == 0.0) return zd{0.0, 0.0};
    const double t = sqrt(0.5 * (m + fabs(a.x)));
    if (a.x >= 0.0) return zd{t, a.y / (2.0 * t)};
    return zd{fabs(a.y) / (2.0 * t), copysign(t, a.y)};
}

constexpr double kTwoPiD = 2.0 * 3.141592653589793;

// Data rows are stored in complex128 or complex64 (the plan's data type);
// every kernel reads and forms them in FP64.
__device__ __forceinline__ zd load_datum(const zd* d, int64_t i) { return d[i]; }
__device__ __forceinline__ zd load_datum(const float2* d, int64_t i) {
    const float2 v = d[i];
    return zd{double(v.x), double(v.y)};
}
__device__ __forceinline__ void store_datum(zd* d, int64_t i, zd v) { d[i] = v; }
__device__ __forceinline__ void store_datum(float2* d, int64_t i, zd v) {
    d[i] = make_float2(float(v.x), float(v.y));
}

// Complex angular frequency w = 2 pi f + i eps.
__device__ __forceinline__ zd omega_of(double f, double eps) { return zd{kTwoPiD * f, eps}; }

// Unique-row descriptor: f | mult << 16, cr | cs << 16.
struct URow {
    int f, mult, cr, cs;
};
__device__ __forceinline__ URow load_urow(const uint32_t* urows, int64_t r) {
    const uint32_t a = urows[2 * r], b = urows[2 * r + 1];
    return URow{int(a & 0xFFFFu), int(a >> 16), int(b & 0xFFFFu), int(b >> 16)};
}

// Value of lane l (uniform index) of a double register, as a scalar.
__device__ __forceinline__ double readlane_d(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(u), l);
    const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(u >> 32), l);
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// Work item (pair p, tile) of block b when the P x T items of a batched
// per-pair product are dealt to the eight XCDs pair by pair (block b runs on
// XCD b % 8): every tile of a pair runs on one XCD, so the pair's matrices are
// read into one L2 instead of eight.  Grid: kXcds ceil(P / kXcds) T blocks;
// p >= P marks a block with no item.
constexpr int kXcds = 8;
__device__ __forceinline__ void xcd_pair_tile(unsigned b, int T, int& p, int& tile) {
    const unsigned j = b / unsigned(kXcds);
    p = int((j / unsigned(T)) * unsigned(kXcds) + b % unsigned(kXcds));
    tile = int(j % unsigned(T));
}
inline unsigned xcd_pair_grid(int64_t P, int T) { return unsigned((P + kXcds - 1) / kXcds * kXcds * T); }

// A batch of 1D transforms along one axis of a dense complex array: line
// l = (slab, k), k < per_slab, has element i at
// data[(l / per_slab) * slab + (l % per_slab) * step + i * stride].
struct Lines {
    int64_t slab, step, stride;
    int per_slab;
};
// sign -1: forward DFT, +1: inverse (unnormalised), then times scale.
hipError_t launch_lines(zd* data, int n, int64_t n_slabs, Lines g, double sign, double scale, hipStream_t st);

// Sum of a double over the 64 lanes of a wave (every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace edt
