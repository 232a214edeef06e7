// C-ABI entry points: argument checks and kernel orchestration on the
// caller's stream.  No device memory is allocated here: scratch lives in the
// caller's workspace (layout from edt::work_layout), or, for the one
// allocation-free entry point edt_solve_static, in a static device array.

#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "dev_common.h"
#include "timing.h"

namespace edt {
hipError_t launch_green(const edt_plan* p, const double* vel, zd* g64, float2* g32, hipStream_t st);
hipError_t launch_gram(const edt_plan* p, edt_precision prec, const zd* g64, const float2* g32,
                       const zd* ubw, const float4* ub32, const float* gmax, void* part, double* rpart,
                       hipStream_t st, const int32_t* only = nullptr, const int32_t* gate = nullptr);
hipError_t launch_gmax(const edt_plan* p, const float2* g32, float* gmax, hipStream_t st);
hipError_t launch_gram_reduce(const edt_plan* p, edt_precision prec, const void* part, double* gram,
                              hipStream_t st, const int32_t* only = nullptr);
hipError_t launch_rhs_reduce(const edt_plan* p, const double* rpart, double* rhs, double* trace,
                             hipStream_t st, const int32_t* only = nullptr);
hipError_t launch_bsum(const edt_plan* p, const void* d_rows, zd* ub, hipStream_t st, zd* ubw = nullptr,
                       float4* ub32 = nullptr);
hipError_t launch_resid(const edt_plan* p, const zd* g64, const zd* ubw, const double* x,
                        const int32_t* conv, double* rpart, hipStream_t st, const int32_t* active);
hipError_t launch_forward(const edt_plan* p, const zd* g64, const zd* v, void* d_rows, hipStream_t st);
hipError_t launch_chol(const edt_plan* p, double* gram, const double* trace, const double* rhs,
                       double lambda_rel, double* lam, double* dinv, double* x, int32_t* info,
                       int32_t* conv, int32_t* steps, hipStream_t st, int only_failed, int exact,
                       int32_t* n_failed);
hipError_t launch_pcg_update(const edt_plan* p, const double* gram, const double* dinv, const double* rpart,
                             const double* lam, double* x, double* r, double* pv, double* rho, int32_t* conv,
                             int32_t* steps, double tol, int first, int32_t* next_active, hipStream_t st);
hipError_t launch_reset_counters(int32_t* c, int n, hipStream_t st);
hipError_t launch_recombine(const edt_plan* p, const double* x, int refine, const int32_t* conv,
                            int32_t* info, zd* v, hipStream_t st);
hipError_t launch_line_adjoint(const edt_plan* p, const double* vel, const zd* g64, const void* d_rows,
                               const double* chol, const double* trace, const double* x, double lambda_rel,
                               const zd* grad_v, void* grad_d, double* grad_lambda, double* grad_vel,
                               unsigned char* work, hipStream_t st);
hipError_t launch_adjoint(const edt_plan* p, const double* vel, const zd* g64, const void* d_rows,
                          const double* chol, const double* trace, const double* x, double lambda_rel,
                          const zd* grad_v, void* grad_d, double* grad_lambda, double* grad_vel,
                          unsigned char* work, hipStream_t st);
hipError_t launch_tsvd_init(const edt_plan* p, const double* gram, double tol_rel, unsigned char* tw,
                            int32_t* iters, hipStream_t st);
hipError_t launch_tsvd_step(const edt_plan* p, int k, double a, unsigned char* tw, int32_t* iters,
                            hipStream_t st);
void tsvd_step_scales(double l0, int n, double* a);
hipError_t launch_tsvd_final(const edt_plan* p, double* gram, const double* rhs, unsigned char* tw,
                             const int32_t* iters, hipStream_t st);
hipError_t launch_shots_fft(const edt_plan* p, zd* shots, hipStream_t st);
hipError_t launch_shots_pack(const edt_plan* p, const zd* F, void* d_rows, hipStream_t st);
hipError_t launch_model(const edt_plan* p, zd* v, double* model, hipStream_t st);
size_t aperture_work_bytes(const edt_plan* p);
hipError_t launch_aperture_gram(const edt_plan* p, const zd* g64, double b_max, double* gram, double* trace,
                                unsigned char* work, hipStream_t st);
hipError_t launch_kz_restrict(const edt_plan* p, double K, double* gram, double* rhs, unsigned char* tw,
                              int32_t* n_keep, hipStream_t st);
size_t chol_lds_bytes(int nz);
hipError_t configure_kernels();
hipError_t launch_line_aperture_gram(const edt_plan* p, const zd* g64, double b_max, double* gram, double* trace,
                                     unsigned char* work, hipStream_t st);
hipError_t launch_line_assemble(const edt_plan* p, const zd* g64, const void* d_rows, double* gram, double* rhs,
                                double* trace, unsigned char* work, hipStream_t st);
hipError_t launch_line_forward(const edt_plan* p, const zd* g64, const zd* v, void* d_rows, hipStream_t st);

Timer& timer_of(const edt_plan* p) {
    edt_plan* q = const_cast<edt_plan*>(p);
    if (!q->timer) {
        q->timer = new Timer();
        q->timer_free = [](void* t) { delete static_cast<Timer*>(t); };
    }
    return *static_cast<Timer*>(q->timer);
}
}  // namespace edt

using namespace edt;

namespace {

edt_status hip_fail(hipError_t e, const char* where) {
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return EDT_EHIP;
}

edt_status check_plan(const edt_plan* p) {
    if (!p) {
        set_error("null plan");
        return EDT_EINVAL;
    }
    if (!p->dev) {
        set_error("plan has no device copy: call edt_plan_upload first");
        return EDT_ESTATE;
    }
    if (p->nz > kMaxDepth) {
        set_error("nz > " + std::to_string(kMaxDepth) + " is not supported by the factorisation kernels");
        return EDT_EINVAL;
    }
    return EDT_OK;
}

// launch `call` on `st`, bracketed by timer events when timing is enabled
#define EDT_TRY(call, where)                                   \
    do {                                                       \
        timer_of(p).begin(stream);                             \
        hipError_t e_ = (call);                                \
        timer_of(p).end(stream, where);                        \
        if (e_ != hipSuccess) return hip_fail(e_, where);      \
    } while (0)

}  // namespace

extern "C" {

edt_status edt_timing_enable(edt_plan* p, int enable) {
    if (!p) {
        set_error("null plan");
        return EDT_EINVAL;
    }
    timer_of(p).enabled = enable != 0;
    return EDT_OK;
}

edt_status edt_timing_read(edt_plan* p, int max_entries, char* names, double* ms, int64_t* count,
                           int* n_out) {
    if (!p || !n_out || (max_entries > 0 && (!names || !ms || !count))) {
        set_error("null argument");
        return EDT_EINVAL;
    }
    Timer& t = timer_of(p);
    std::vector<std::string> key;
    std::vector<double> tot;
    std::vector<int64_t> cnt;
    for (auto& r : t.recs) {
        if (hipEventSynchronize(r.stop) != hipSuccess) return hip_fail(hipGetLastError(), "timing read");
        float e = 0.f;
        if (hipEventElapsedTime(&e, r.start, r.stop) != hipSuccess) return hip_fail(hipGetLastError(), "timing read");
        size_t k = 0;
        while (k < key.size() && key[k] != r.name) ++k;
        if (k == key.size()) {
            key.emplace_back(r.name);
            tot.push_back(0.0);
            cnt.push_back(0);
        }
        tot[k] += double(e);
        cnt[k] += 1;
        t.pool.push_back(r.start);
        t.pool.push_back(r.stop);
    }
    t.recs.clear();
    const int n = int(key.size());
    *n_out = n;
    for (int k = 0; k < n && k < max_entries; ++k) {
        std::snprintf(names + 32 * k, 32, "%s", key[k].c_str());
        ms[k] = tot[k];
        count[k] = cnt[k];
    }
    return EDT_OK;
}

edt_status edt_plan_upload(edt_plan* p, void* dev_buf, size_t bytes, hipStream_t stream) {
    if (!p || !dev_buf) {
        set_error("null argument");
        return EDT_EINVAL;
    }
    if (bytes < p->lay.total) {
        set_error("device plan buffer too small");
        return EDT_ENOMEM;
    }
    if (reinterpret_cast<uintptr_t>(dev_buf) % 256 != 0) {
        set_error("device plan buffer must be 256-byte aligned");
        return EDT_EINVAL;
    }
    hipError_t e = configure_kernels();
    if (e == hipSuccess)
        e = hipMemcpyAsync(dev_buf, p->host_image.data(), p->lay.total, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "plan upload");
    p->dev = static_cast<unsigned char*>(dev_buf);
    return EDT_OK;
}

edt_status edt_green(const edt_plan* p, const double* vel_dev, edt_c128* g64, edt_c64* g32,
                     hipStream_t stream) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    if (!vel_dev || !g64) {
        set_error("vel_dev and g64 are required");
        return EDT_EINVAL;
    }
    EDT_TRY(launch_green(p, vel_dev, reinterpret_cast<zd*>(g64), reinterpret_cast<float2*>(g32), stream),
            "green");
    return EDT_OK;
}

edt_status edt_assemble(const edt_plan* p, const edt_c128* g64, const edt_c64* g32,
                        const void* d_rows, edt_precision prec, double* gram, double* rhs,
                        double* trace, void* work, hipStream_t stream) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    if (prec != EDT_FP64 && prec != EDT_FP32 && prec != EDT_BF16X3 && prec != EDT_FP16X3) {
        set_error("unknown precision");
        return EDT_EINVAL;
    }
    if (!g64 || !d_rows || !gram || !rhs || !trace || !work || (prec != EDT_FP64 && !g32)) {
        set_error("missing argument (g32 is required for FP32 and BF16X3)");
        return EDT_EINVAL;
    }
    if (prec == EDT_FP32 && p->nz > kSuperDepth) {
        set_error("the FP32 Gram supports nz <= 256 (use FP64, BF16X3 or FP16X3)");
        return EDT_EINVAL;
    }
    if (p->n_line) {
        // the survey of parallel lines: rows are sums over the line
        // wavenumbers, formed per frequency and multiplied in FP64
        if (prec != EDT_FP64) {
            set_error("the survey of parallel lines is assembled in FP64 only");
            return EDT_EINVAL;
        }
        EDT_TRY(launch_line_assemble(p, reinterpret_cast<const zd*>(g64), d_rows, gram, rhs, trace,
                                     static_cast<unsigned char*>(work), stream),
                "line assemble");
        return EDT_OK;
    }
    const WorkLayout wl = work_layout(p);
    unsigned char* w = static_cast<unsigned char*>(work);
    zd* ubw = reinterpret_cast<zd*>(w + wl.ubw);
    float4* ub32 = reinterpret_cast<float4*>(w + wl.ub32);
    const bool f64 = prec == EDT_FP64;
    const zd* G64 = reinterpret_cast<const zd*>(g64);
    // conj(W) B in FP64 for every precision: the FP64 Gram reads it, and the
    // data sweep of a refining edt_solve can reuse it
    EDT_TRY(launch_bsum(p, d_rows, nullptr, stream, ubw, f64 ? nullptr : ub32),
            "bsum");
    // one pass over the rows gives the Gram partials and the right-hand side
    // and trace partials of every item
    double* rpart = reinterpret_cast<double*>(w + wl.gram_rpart);
    float* gmax = reinterpret_cast<float*>(w + wl.gmax);
    if (prec == EDT_FP16X3)
        EDT_TRY(launch_gmax(p, reinterpret_cast<const float2*>(g32), gmax, stream), "gmax");
    EDT_TRY(launch_gram(p, prec, G64, reinterpret_cast<const float2*>(g32), ubw, ub32, gmax, w + wl.gram_part,
                        rpart, stream),
            f64 ? "gram_fp64"
                : (prec == EDT_FP32 ? "gram_fp32" : (prec == EDT_BF16X3 ? "gram_bf16x3" : "gram_fp16x3")));
    EDT_TRY(launch_gram_reduce(p, prec, w + wl.gram_part, gram, stream), "gram_reduce");
    EDT_TRY(launch_rhs_reduce(p, rpart, rhs, trace, stream), "rhs reduce");
    return EDT_OK;
}

}  // extern "C"

namespace {

// Device scratch of one edt_solve call: every pointer the solve path hands
// to its kernels.  Filled from the plan's workspace (edt_solve) or from the
// library's static array (edt_solve_static); a section the call does not use
// stays null.
struct SolveScratch {
    zd* ubw = nullptr;            // [U][2] conj(W) times the summed data
    double* rpart = nullptr;      // residual partials per residual item
    double* lam = nullptr;        // [P] damping
    double* dinv = nullptr;       // [P][nblk][32][32] inverses of the diagonal blocks
    int32_t* conv = nullptr;      // [P] converged flags
    int32_t* aux = nullptr;       // [P] refinement steps when the caller passes none
    int32_t* cnt = nullptr;       // [kMaxRefine + 2] sweep counters, failed factorisations
    double* pcg_r = nullptr;      // [P][2][nz]
    double* pcg_p = nullptr;      // [P][2][nz]
    double* pcg_rho = nullptr;    // [P]
    unsigned char* gram_part = nullptr;   // escalation: FP64 Gram partials per item
    double* gram_rpart = nullptr;         // escalation: rhs and trace partials per item
    double* esc_rhs = nullptr;            // escalation: [P][2][nz]
    double* esc_trace = nullptr;          // escalation: [P]
};

SolveScratch scratch_from_work(const edt_plan* p, void* work) {
    const WorkLayout wl = work_layout(p);
    unsigned char* w = static_cast<unsigned char*>(work);
    SolveScratch s;
    s.ubw = reinterpret_cast<zd*>(w + wl.ubw);
    s.rpart = reinterpret_cast<double*>(w + wl.rhs_part);
    s.lam = reinterpret_cast<double*>(w + wl.lam);
    s.dinv = reinterpret_cast<double*>(w + wl.dinv);
    s.conv = reinterpret_cast<int32_t*>(w + wl.conv);
    s.aux = reinterpret_cast<int32_t*>(w + wl.aux);
    s.cnt = reinterpret_cast<int32_t*>(w + wl.counters);
    s.pcg_r = reinterpret_cast<double*>(w + wl.pcg_r);
    s.pcg_p = reinterpret_cast<double*>(w + wl.pcg_p);
    s.pcg_rho = reinterpret_cast<double*>(w + wl.pcg_rho);
    s.gram_part = w + wl.gram_part;
    s.gram_rpart = reinterpret_cast<double*>(w + wl.gram_rpart);
    s.esc_rhs = reinterpret_cast<double*>(w + wl.esc_rhs);
    s.esc_trace = reinterpret_cast<double*>(w + wl.esc_trace);
    return s;
}

// Compact scratch of a solve that uses only what its options need, packed
// from `base` (null: sizes only).  Returns the bytes used.
size_t compact_solve_scratch(const edt_plan* p, bool refine, bool escalate, unsigned char* base,
                             SolveScratch* out) {
    const size_t P = size_t(p->n_pairs), nz = size_t(p->nz), U = size_t(p->n_urows);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) / 256 * 256;
        return base ? base + o : nullptr;
    };
    SolveScratch s;
    s.lam = reinterpret_cast<double*>(take(P * sizeof(double)));
    s.dinv = reinterpret_cast<double*>(take(P * size_t((p->nz + 31) / 32) * 32 * 32 * sizeof(double)));
    s.conv = reinterpret_cast<int32_t*>(take(P * sizeof(int32_t)));
    s.aux = reinterpret_cast<int32_t*>(take(P * sizeof(int32_t)));
    s.cnt = reinterpret_cast<int32_t*>(take((kMaxRefine + 2) * sizeof(int32_t)));
    if (refine) {
        s.ubw = reinterpret_cast<zd*>(take(U * 2 * sizeof(zd)));
        s.rpart = reinterpret_cast<double*>(take(p->ritems.size() * (2 * nz + 1) * sizeof(double)));
        s.pcg_r = reinterpret_cast<double*>(take(P * 2 * nz * sizeof(double)));
        s.pcg_p = reinterpret_cast<double*>(take(P * 2 * nz * sizeof(double)));
        s.pcg_rho = reinterpret_cast<double*>(take(P * sizeof(double)));
        if (escalate) {
            s.gram_part = take(p->items.size() * gram_part_bytes_per_item(p));
            s.gram_rpart = reinterpret_cast<double*>(take(p->items.size() * size_t(rpart_width(p->nz)) * sizeof(double)));
            s.esc_rhs = reinterpret_cast<double*>(take(P * 2 * nz * sizeof(double)));
            s.esc_trace = reinterpret_cast<double*>(take(P * sizeof(double)));
        }
    }
    if (out) *out = s;
    return off;
}

edt_status check_solve_args(const edt_plan* p, const edt_c128* g64, const void* d_rows, double* gram,
                            const double* rhs, const double* trace, double lambda_rel, const edt_solve_opts* opts,
                            double* x, edt_c128* v_out, int32_t* info) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    const int refine = opts ? opts->refine : 0;
    if (!gram || !rhs || !trace || !x || !v_out || !info || (refine && (!g64 || !d_rows))) {
        set_error("missing argument (g64 and d_rows are required with refinement)");
        return EDT_EINVAL;
    }
    if (!(lambda_rel >= 0.0)) {
        set_error("lambda_rel must be >= 0");
        return EDT_EINVAL;
    }
    if (refine && (opts->max_refine < 0 || opts->max_refine > kMaxRefine || !(opts->refine_tol > 0.0))) {
        set_error("refinement needs 0 <= max_refine <= " + std::to_string(kMaxRefine) + " and refine_tol > 0");
        return EDT_EINVAL;
    }
    if (refine && p->n_line) {
        set_error("the survey of parallel lines is solved without refinement (its Gram is FP64)");
        return EDT_EINVAL;
    }
    return EDT_OK;
}

// The solve path shared by edt_solve and edt_solve_static (arguments checked).
edt_status solve_impl(const edt_plan* p, const edt_c128* g64, const void* d_rows, double* gram,
                      const double* rhs, const double* trace, double lambda_rel, const edt_solve_opts* opts,
                      double* x, edt_c128* v_out, int32_t* info, int32_t* steps, const SolveScratch& ws,
                      hipStream_t stream) {
    const int refine = opts ? opts->refine : 0;
    int32_t* stp = steps ? steps : ws.aux;
    // counters: pairs iterating before each sweep, then the failed factorisations
    int32_t* cnt = ws.cnt;
    int32_t* n_failed = cnt + kMaxRefine + 1;
    if (refine) EDT_TRY(launch_reset_counters(cnt, kMaxRefine + 2, stream), "reset counters");
    EDT_TRY(launch_chol(p, gram, trace, rhs, lambda_rel, ws.lam, ws.dinv, x, info, ws.conv, stp, stream, 0, !refine,
                        refine ? n_failed : nullptr),
            "cholesky");
    if (refine) {
        const zd* G64 = reinterpret_cast<const zd*>(g64);
        // the summed data, conj(W) B per unique row, unless the caller states
        // that edt_assemble left them in work
        if (!opts->data_summed)
            EDT_TRY(launch_bsum(p, d_rows, nullptr, stream, ws.ubw), "bsum");
        if (opts->escalate) {
            // pairs whose factorisation failed (info > 0): FP64 Gram, rhs and
            // trace from the rows, and a second factorisation; every launch
            // returns at once for the other pairs
            EDT_TRY(launch_gram(p, EDT_FP64, G64, nullptr, ws.ubw, nullptr, nullptr, ws.gram_part, ws.gram_rpart,
                                stream, info, n_failed),
                    "escalate gram_fp64");
            EDT_TRY(launch_gram_reduce(p, EDT_FP64, ws.gram_part, gram, stream, info), "escalate gram_reduce");
            EDT_TRY(launch_rhs_reduce(p, ws.gram_rpart, ws.esc_rhs, ws.esc_trace, stream, info),
                    "escalate rhs reduce");
            EDT_TRY(launch_chol(p, gram, ws.esc_trace, ws.esc_rhs, lambda_rel, ws.lam, ws.dinv, x, info, ws.conv, stp,
                                stream, 1, 0, nullptr),
                    "escalate cholesky");
        }
        // sweep 0: the data residual at x0; then one operator sweep per step
        for (int it = 0; it < opts->max_refine; ++it) {
            EDT_TRY(launch_resid(p, G64, it == 0 ? ws.ubw : nullptr, it == 0 ? x : ws.pcg_p, ws.conv, ws.rpart,
                                 stream, cnt + it),
                    "refine residual");
            EDT_TRY(launch_pcg_update(p, gram, ws.dinv, ws.rpart, ws.lam, x, ws.pcg_r, ws.pcg_p, ws.pcg_rho, ws.conv,
                                      stp, opts->refine_tol, it == 0, cnt + it + 1, stream),
                    "refine update");
        }
    }
    EDT_TRY(launch_recombine(p, x, refine, ws.conv, info, reinterpret_cast<zd*>(v_out), stream), "recombine");
    return EDT_OK;
}

// The allocation-free solve's scratch: one array per GPU, for the life of
// the process.  Host code never passes `scratch` itself to a kernel: it is a
// host-side stand-in there; the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[EDT_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

edt_status static_scratch(unsigned char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "static scratch: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("static scratch: device index out of range");
        return EDT_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "static scratch: hipGetSymbolAddress");
        if (!ptr) {
            set_error("static scratch: no device address");
            return EDT_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return EDT_OK;
}

}  // namespace

extern "C" {

edt_status edt_solve(const edt_plan* p, const edt_c128* g64, const void* d_rows, double* gram,
                     const double* rhs, const double* trace, double lambda_rel,
                     const edt_solve_opts* opts, double* x, edt_c128* v_out, int32_t* info,
                     int32_t* steps, void* work, hipStream_t stream) {
    edt_status s = check_solve_args(p, g64, d_rows, gram, rhs, trace, lambda_rel, opts, x, v_out, info);
    if (s != EDT_OK) return s;
    if (!work) {
        set_error("missing argument: work");
        return EDT_EINVAL;
    }
    return solve_impl(p, g64, d_rows, gram, rhs, trace, lambda_rel, opts, x, v_out, info, steps,
                      scratch_from_work(p, work), stream);
}

edt_status edt_solve_static(const edt_plan* p, const edt_c128* g64, const void* d_rows, double* gram,
                            const double* rhs, const double* trace, double lambda_rel,
                            const edt_solve_opts* opts, double* x, edt_c128* v_out, int32_t* info,
                            int32_t* steps, hipStream_t stream) {
    edt_status s = check_solve_args(p, g64, d_rows, gram, rhs, trace, lambda_rel, opts, x, v_out, info);
    if (s != EDT_OK) return s;
    const bool refine = opts && opts->refine;
    const bool escalate = refine && opts->escalate;
    if (refine && opts->data_summed) {
        set_error("edt_solve_static sums the data itself: data_summed must be 0");
        return EDT_EINVAL;
    }
    const size_t need = compact_solve_scratch(p, refine, escalate, nullptr, nullptr);
    if (need > size_t(EDT_STATIC_SCRATCH_BYTES)) {
        set_error("edt_solve_static needs " + std::to_string(need) + " bytes of scratch, more than the " +
                  std::to_string(size_t(EDT_STATIC_SCRATCH_BYTES)) + " it holds (use edt_solve with a workspace)");
        return EDT_ENOMEM;
    }
    unsigned char* base = nullptr;
    s = static_scratch(&base);
    if (s != EDT_OK) return s;
    SolveScratch ws;
    compact_solve_scratch(p, refine, escalate, base, &ws);
    return solve_impl(p, g64, d_rows, gram, rhs, trace, lambda_rel, opts, x, v_out, info, steps, ws, stream);
}

edt_status edt_tsvd_work_bytes(const edt_plan* p, size_t* bytes) {
    if (!p || !bytes) {
        set_error("null argument");
        return EDT_EINVAL;
    }
    *bytes = tsvd_layout(p).total;
    return EDT_OK;
}

edt_status edt_tsvd(const edt_plan* p, double* gram, const double* rhs, double tol_rel, int max_iter, double* x,
                    edt_c128* v_out, int32_t* info, int32_t* iters, void* work, void* tsvd_work,
                    hipStream_t stream) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    if (!(tol_rel >= 0.0) || !std::isfinite(tol_rel)) {
        set_error("tol_rel must be finite and >= 0");
        return EDT_EINVAL;
    }
    if (max_iter < 1 || max_iter > kMaxSignIter) {
        set_error("max_iter must be in [1, " + std::to_string(kMaxSignIter) + "]");
        return EDT_EINVAL;
    }
    if (p->n_pairs == 0) return EDT_OK;   // an empty pair range
    if (!gram || !rhs || !x || !v_out || !info || !iters || !work || !tsvd_work) {
        set_error("missing argument");
        return EDT_EINVAL;
    }
    const WorkLayout wl = work_layout(p);
    unsigned char* w = static_cast<unsigned char*>(work);
    unsigned char* tw = static_cast<unsigned char*>(tsvd_work);
    const TsvdLayout tl = tsvd_layout(p);
    EDT_TRY(launch_tsvd_init(p, gram, tol_rel, tw, iters, stream), "tsvd init");
    // step scalings from a guess of the smallest eigenvalue magnitude of X_0:
    // a dropped direction of G (eigenvalue ~0) sits at about tol_rel^2, one
    // 1% away from the threshold at 1e-2 tol_rel^2
    std::vector<double> scale(static_cast<size_t>(max_iter));
    tsvd_step_scales(std::max(1e-2 * tol_rel * tol_rel, 1e-14), max_iter, scale.data());
    for (int k = 0; k < max_iter; ++k)
        EDT_TRY(launch_tsvd_step(p, k, scale[size_t(k)], tw, iters, stream), "tsvd sign step");
    EDT_TRY(launch_tsvd_final(p, gram, rhs, tw, iters, stream), "tsvd projector");
    // (G + sigma^2 (I - P)) x = P c by the factorisation with no damping and
    // the corrected block solves
    EDT_TRY(launch_chol(p, gram, reinterpret_cast<const double*>(tw + tl.tau2),
                        reinterpret_cast<const double*>(tw + tl.rhs), 0.0, reinterpret_cast<double*>(w + wl.lam),
                        reinterpret_cast<double*>(w + wl.dinv), x, info, reinterpret_cast<int32_t*>(w + wl.conv),
                        reinterpret_cast<int32_t*>(w + wl.aux), stream, 0, 1, nullptr),
            "tsvd cholesky");
    // pairs whose sign iteration did not converge are reported as such
    EDT_TRY(launch_recombine(p, x, 1, reinterpret_cast<const int32_t*>(tw + tl.conv), info,
                             reinterpret_cast<zd*>(v_out), stream),
            "recombine");
    return EDT_OK;
}

edt_status edt_kz_disk_radius(const edt_plan* p, double factor, double* k_disk) {
    if (!p || !k_disk || !(factor >= 0.0) || !std::isfinite(factor)) {
        set_error("plan and k_disk must be given and factor finite and >= 0");
        return EDT_EINVAL;
    }
    double fmax = 0.0;
    for (double f : p->freq) fmax = std::max(fmax, f);
    *k_disk = factor * (kTwoPiD * fmax) / p->ctop;
    return EDT_OK;
}

edt_status edt_kz_restrict(const edt_plan* p, double k_disk, double* gram, double* rhs, int32_t* n_keep,
                           void* tsvd_work, hipStream_t stream) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    if (!(k_disk >= 0.0) || !std::isfinite(k_disk)) {
        set_error("k_disk must be finite and >= 0");
        return EDT_EINVAL;
    }
    if (p->n_pairs == 0) return EDT_OK;   // an empty pair range
    if (!gram || !rhs || !tsvd_work) {
        set_error("missing argument");
        return EDT_EINVAL;
    }
    EDT_TRY(launch_kz_restrict(p, k_disk, gram, rhs, static_cast<unsigned char*>(tsvd_work), n_keep, stream),
            "kz restrict");
    return EDT_OK;
}

namespace {
// Surveys whose shot records the transform takes: the 2D line, the 3D
// survey of parallel lines, and the 3D areal survey up to n_mid = kMaxAreal
// (its doubled records).
edt_status check_records(const edt_plan* p, bool transform) {
    if (p->dim == 3 && p->n_line == 0 && p->n_mid > kMaxAreal) {
        set_error("3D areal records: n_mid > " + std::to_string(kMaxAreal) + " is not supported");
        return EDT_EINVAL;
    }
    if (transform && p->n_mid > kMaxLine) {
        set_error("n_mid > " + std::to_string(kMaxLine) + " is not supported by the transform");
        return EDT_EINVAL;
    }
    return EDT_OK;
}
}  // namespace

edt_status edt_shots_fft(const edt_plan* p, edt_c128* shots, hipStream_t stream) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    if (!shots) {
        set_error("missing argument");
        return EDT_EINVAL;
    }
    s = check_records(p, true);
    if (s != EDT_OK) return s;
    EDT_TRY(launch_shots_fft(p, reinterpret_cast<zd*>(shots), stream), "shots fft");
    return EDT_OK;
}

edt_status edt_shots_pack(const edt_plan* p, const edt_c128* spectrum, void* d_rows, hipStream_t stream) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    if (!spectrum || !d_rows) {
        set_error("missing argument");
        return EDT_EINVAL;
    }
    s = check_records(p, false);
    if (s != EDT_OK) return s;
    EDT_TRY(launch_shots_pack(p, reinterpret_cast<const zd*>(spectrum), d_rows, stream),
            "shots pack");
    return EDT_OK;
}

edt_status edt_aperture_work_bytes(const edt_plan* p, size_t* bytes) {
    if (!p || !bytes) {
        set_error("null argument");
        return EDT_EINVAL;
    }
    *bytes = aperture_work_bytes(p);
    return EDT_OK;
}

edt_status edt_aperture_gram(const edt_plan* p, const edt_c128* g64, double b_max, double* gram, double* trace,
                             void* aperture_work, hipStream_t stream) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    if (p->dim != 2 && !p->n_line) {
        set_error("finite aperture of the 2D line survey and the survey of parallel lines only");
        return EDT_EINVAL;
    }
    if (p->n_mid > kMaxLine) {
        set_error("n_mid > " + std::to_string(kMaxLine) + " is not supported by the transform");
        return EDT_EINVAL;
    }
    if (!(b_max >= 0.0) || !std::isfinite(b_max)) {
        set_error("b_max must be finite and >= 0");
        return EDT_EINVAL;
    }
    if (p->n_pairs == 0) return EDT_OK;
    if (!g64 || !gram || !trace || !aperture_work) {
        set_error("missing argument");
        return EDT_EINVAL;
    }
    if (p->n_line)
        EDT_TRY(launch_line_aperture_gram(p, reinterpret_cast<const zd*>(g64), b_max, gram, trace,
                                          static_cast<unsigned char*>(aperture_work), stream),
                "aperture gram");
    else
        EDT_TRY(launch_aperture_gram(p, reinterpret_cast<const zd*>(g64), b_max, gram, trace,
                                     static_cast<unsigned char*>(aperture_work), stream),
                "aperture gram");
    return EDT_OK;
}

edt_status edt_model(const edt_plan* p, edt_c128* v_tilde, double* model, hipStream_t stream) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    if (!v_tilde || !model) {
        set_error("missing argument");
        return EDT_EINVAL;
    }
    if (p->n_mid > kMaxLine) {
        set_error("n_mid > " + std::to_string(kMaxLine) + " is not supported by the transform");
        return EDT_EINVAL;
    }
    EDT_TRY(launch_model(p, reinterpret_cast<zd*>(v_tilde), model, stream), "model");
    return EDT_OK;
}

edt_status edt_forward(const edt_plan* p, const edt_c128* g64, const edt_c128* v_in, void* d_rows,
                       hipStream_t stream) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    if (!g64 || !v_in || !d_rows) {
        set_error("missing argument");
        return EDT_EINVAL;
    }
    if (p->n_line) {
        EDT_TRY(launch_line_forward(p, reinterpret_cast<const zd*>(g64), reinterpret_cast<const zd*>(v_in), d_rows,
                                    stream),
                "line forward");
        return EDT_OK;
    }
    EDT_TRY(launch_forward(p, reinterpret_cast<const zd*>(g64), reinterpret_cast<const zd*>(v_in), d_rows, stream),
            "forward");
    return EDT_OK;
}

edt_status edt_adjoint(const edt_plan* p, const double* vel_dev, const edt_c128* g64,
                       const void* d_rows, const double* chol, const double* trace, const double* x,
                       double lambda_rel, const edt_c128* grad_v, void* grad_d, double* grad_lambda,
                       double* grad_vel, void* work, hipStream_t stream) {
    edt_status s = check_plan(p);
    if (s != EDT_OK) return s;
    if (!vel_dev || !g64 || !d_rows || !chol || !trace || !x || !grad_v || !work) {
        set_error("missing argument");
        return EDT_EINVAL;
    }
    if (p->nz > kMaxAdjointDepth) {
        set_error("the adjoint supports nz <= 256");
        return EDT_EINVAL;
    }
    if (p->n_line)
        EDT_TRY(launch_line_adjoint(p, vel_dev, reinterpret_cast<const zd*>(g64), d_rows, chol, trace, x,
                                    lambda_rel, reinterpret_cast<const zd*>(grad_v), grad_d, grad_lambda, grad_vel,
                                    static_cast<unsigned char*>(work), stream),
                "adjoint");
    else
        EDT_TRY(launch_adjoint(p, vel_dev, reinterpret_cast<const zd*>(g64), d_rows,
                               chol, trace, x, lambda_rel, reinterpret_cast<const zd*>(grad_v),
                               grad_d, grad_lambda, grad_vel,
                               static_cast<unsigned char*>(work), stream),
                "adjoint");
    return EDT_OK;
}

}  // extern "C"
