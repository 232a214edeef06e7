// Internal plan layout shared by the host planner and the kernel launchers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/edt.h"

namespace edt {

// One assembly work item: a contiguous chunk of one pair's unique rows.
struct Item {
    int32_t pair;
    int32_t row_begin;   // global unique-row index
    int32_t row_end;
    int32_t slot;        // index of this item's partial-result slot
};

// Per-unique-row record of the Gram kernels, formed by the planner.
struct GRow {
    uint32_t off_r, off_s;   // table offsets (f n_cls + class) nz of g(k_r) and g(k_s)
    float sw;                // sqrt(mult), correctly rounded
    float mt;                // mult
};

// Byte offsets of the sections of the device copy of the plan.
struct DevLayout {
    size_t freq, zif, cls_k, row_off, pair_u, rows, keys, urow_off, urows, umem_off, umem,
        row_unique, urow_pair, tab_off, tab_ent, items, sched, pair_item, ritems, rsched, pair_ritem,
        grow, gsc, lmask, lfr, lpair, total;
};

// Gram tasks split the depths into super-blocks of at most 256 (8 tiles of
// 32); each item's right-hand-side/trace partial holds c+, c- and one trace
// per super-block.
constexpr int kSuperDepth = 256;
// Depth limits: the factorisation and refinement (7 accumulator row-block
// groups, LDS), and the adjoint's table kernel (4 depths per lane).
constexpr int kMaxDepth = 448;
constexpr int kMaxAdjointDepth = 256;
// Refinement sweeps of one solve at most (device counters per sweep).
constexpr int kMaxRefine = 62;
constexpr int kMaxLine = 2048;   // longest 1D transform of the shot-record and model transforms
constexpr int kMaxAreal = 128;   // largest n_mid of the 3D areal records (16 (2 n_mid)^4 bytes per frequency)
constexpr int64_t kMaxLineBlocks = int64_t(1) << 16;   // workgroups of one transform launch
constexpr int kMaxSignIter = 200;   // sign-iteration steps of the truncated-SVD solve at most
constexpr int n_super(int nz) { return (nz + kSuperDepth - 1) / kSuperDepth; }
constexpr int rpart_width(int nz) { return 2 * nz + n_super(nz); }

constexpr int kMaxLayers = 64;   // layer-recursion state is held in LDS

}  // namespace edt

struct edt_plan {
    // survey
    int dim, n_mid, n_off, n_freq, nz, n_layers;
    double d_mid, d_off, eps, z0, dz, kappa, ctop;
    int n_line = 0;                      // 3D survey of parallel lines: number of lines (0: areal)
    double d_line = 0.0;                 // line spacing
    std::vector<uint64_t> lmask;         // line survey [R]: bit (q + n_line/2) set iff term q is kept
    std::vector<int64_t> lfr;            // line survey [P][n_freq + 1]: first row of each frequency
    std::vector<int32_t> lpair;          // line survey [R]: pair of each row
    std::vector<double> freq, zif;
    // |k| classes
    int n_cls;
    std::vector<double> cls_k;
    // pairs and rows
    int64_t n_km, n_pairs, n_rows, max_rows, n_empty;
    int64_t n_pairs_all = 0, pair_begin = 0;   // the survey's pairs; first pair of this plan
    std::vector<int64_t> row_off;        // [P+1]
    std::vector<int32_t> pair_u;         // [2P]: u, -u
    std::vector<uint32_t> rows;          // [2R]: f, cr | cs << 16
    std::vector<int32_t> keys;           // [2R]
    // unique rows: data rows of one pair with equal (f, {cr, cs}) share one
    // Born row A (source-receiver reciprocity and lattice symmetry)
    int64_t n_urows;
    std::vector<int64_t> urow_off;       // [P+1]
    std::vector<uint32_t> urows;         // [2U]: f | mult << 16, cr | cs << 16
    std::vector<int32_t> umem_off;       // [U+1] members of each unique row
    std::vector<int32_t> umem;           // [R] data rows, grouped
    std::vector<int32_t> row_unique;     // [R] unique row of each data row
    std::vector<int32_t> urow_pair;      // [U] pair of each unique row
    std::vector<edt::GRow> grow;         // [U] table offsets and scales (Gram kernels)
    std::vector<double> gsc;             // [U] |w^2 dz| sqrt(mult) (FP64 Gram row scale)
    // table-entry contributors (adjoint): entry e = f*n_cls + c receives from
    // unique rows that use class c at frequency f; tab_ent = (row, other class)
    std::vector<int32_t> tab_off;        // [n_freq*n_cls + 1]
    std::vector<int32_t> tab_ent;        // [2 * 2U]
    // work items
    int chunk_rows;
    int data_c64 = 0;                    // data rows in complex64 (else complex128)
    int gram_band;                       // frequencies per Gram band
    int resid_group = 2;                 // frequencies per residual work item
    std::vector<edt::Item> items;        // Gram items (pair, frequency band), pair-major
    std::vector<int32_t> sched;          // XCD-aware launch order, -1 = hole
    std::vector<int32_t> pair_item;      // [P+1] first item of each pair
    std::vector<edt::Item> ritems;       // residual items (pair, frequency group), pair-major
    std::vector<int32_t> rsched;         // XCD-aware launch order, -1 = hole
    std::vector<int32_t> pair_ritem;     // [P+1] first residual item of each pair
    double gram_flops;
    // device copy
    edt::DevLayout lay;
    std::vector<unsigned char> host_image;
    unsigned char* dev = nullptr;
    // optional kernel timer (owned; created on first use by the HIP side)
    void* timer = nullptr;
    void (*timer_free)(void*) = nullptr;
    ~edt_plan() {
        if (timer && timer_free) timer_free(timer);
    }
};

namespace edt {

void set_error(const std::string& msg);

// Device pointers into the uploaded plan.
template <class T>
inline T* dptr(const edt_plan* p, size_t off) {
    return reinterpret_cast<T*>(p->dev + off);
}

// Workspace layout (bytes); identical for every call on a plan.
struct WorkLayout {
    size_t ub;          // [U][2] complex128 summed data b+ and b- of each unique row
    size_t ubw;         // [U][2] complex128 conj(W) ub (FP64 Gram right-hand side)
    size_t ub32;        // [U] float4 conj(W)/|W| ub (FP32 / BF16x3 Gram right-hand side)
    size_t gmax;        // [n_freq * n_cls] FP32 max_z |g32| (FP16x3 row scaling)
    size_t gram_part;   // [n_items][ntiles][tile] partial Gram tiles (FP64 or FP32)
    size_t rhs_part;    // [n_ritems][2*nz + 1] FP64 partial residuals (refinement, adjoint)
    size_t gram_rpart;  // [n_items][2*nz + n_super] FP64 partial rhs and traces from the Gram kernels
    size_t lam;         // [P] lambda per pair
    size_t dinv;        // [P][nblk][32][32] FP64 inverses of the 32 x 32 diagonal blocks of L
    size_t conv;        // [P] int32 converged flags
    size_t pcg_r;       // [P][2][nz] FP64 refinement residual
    size_t pcg_p;       // [P][2][nz] FP64 refinement search direction
    size_t pcg_rho;     // [P] FP64 r.z of the refinement
    size_t esc_rhs;     // [P][2][nz] FP64 rhs of re-assembled (escalated) pairs
    size_t esc_trace;   // [P] FP64 trace of re-assembled pairs
    size_t counters;    // [kMaxRefine + 2] int32: pairs iterating before each sweep, failed factorisations
    size_t aux;         // [P][2][nz] FP64 scratch (refinement, adjoint)
    size_t aux2;        // [P][2][nz] FP64 scratch
    size_t gbar;        // [n_freq][n_cls][nz] complex128 (adjoint table gradient)
    size_t adj_y;       // [P][2][nz] adjoint solutions
    size_t adj_dl;      // [P] dL/dlambda_p
    size_t adj_row;     // [U][4] complex128: e+, e-, A y+, A y-
    size_t adj_vel;     // [n_freq*n_cls][n_layers] per-entry velocity gradients
    size_t scal;        // [64] FP64 scalars
    size_t lrows;       // line survey: [line_chunk][n_mid][nz] complex128 rows of one frequency
    size_t total;
};
WorkLayout work_layout(const edt_plan* p);

// Layout (bytes) of the separate scratch of the truncated-SVD solve.
struct TsvdLayout {
    size_t x0, x1;   // [P][nz][nz] FP64 sign iterates (ping-pong)
    size_t y;        // [P][nz][nz] FP64 X^2
    size_t rhs;      // [P][2][nz] FP64 projected right-hand sides P c
    size_t tau2;     // [P] FP64 truncation threshold sigma^2
    size_t dpart;    // [P][nt (nt+1)/2] FP64 lower-tile partials of ||X^2 - I||_F^2
    size_t conv;     // [P] int32 sign iteration converged
    size_t total;
};
TsvdLayout tsvd_layout(const edt_plan* p);
size_t gram_part_bytes_per_item(const edt_plan* p);
// Device bytes of one pass of the plan (edt_plan_info.resident_bytes).
size_t resident_bytes(const edt_plan* p);
// Line survey: pairs whose rows of one frequency are formed at once.
int64_t line_chunk(const edt_plan* p);

}  // namespace edt
