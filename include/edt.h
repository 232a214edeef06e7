/*
 * edt.h -- C-ABI of libedt, the MI355X (gfx950) hot path of extended
 * diffraction tomography (Schlottmann, "Extended diffraction tomography").
 *
 * The paper (Section 2.1) turns the linear Born inversion of surface seismic
 * data over a depth-dependent reference medium into many independent 1D depth
 * problems, one per midpoint wavenumber k_m (eq. DMV), whose kernel M is a
 * product of two reference Green's functions (eq. M).  Because M(k_m) =
 * M(-k_m), the problems at +k_m and -k_m are solved together as one *pair*
 * for the real unknowns Re V~ and Im V~ (eqs. VSym, Split).  This library
 * computes, on one GPU:
 *
 *   edt_green     the Green's-function tables g(z; |k|, w) of the layered
 *                 reference (the 1D reference Helmholtz problem, Section 2.1)
 *   edt_assemble  per pair the Gram matrix G = Re(A^H A) of the Born rows
 *                 A = w^2 dz g(k_r) g(k_s) (eq. M, infinite-aperture limit),
 *                 the right-hand sides c = Re(A^H b+-) (eq. Split) and tr(G)
 *   edt_solve     the relatively damped normal equations
 *                 (G + lambda_rel tr(G)/nz I) x = c by Cholesky, with FP64
 *                 iterative refinement for the mixed-precision Grams, and the
 *                 recombination V~(+-k_m) = x+ +- i x-  (eq. VSym)
 *   edt_adjoint   the reverse-mode gradient of a loss on V~ with respect to
 *                 the data, lambda_rel and the layer velocities
 *   edt_forward   the Born forward map V~ -> data rows (eq. DMV), used for
 *                 data synthesis and adjoint (dot-product) checks
 *
 * Conventions shared by every call
 * --------------------------------
 * - Complex numbers are interleaved (re, im) pairs: edt_c128 == two doubles,
 *   edt_c64 == two floats (the layouts of torch.complex128 / complex64).
 * - Time dependence e^{-i w t}, complex angular frequency w = 2 pi f + i eps.
 * - Horizontal wavenumber indices are in numpy fftfreq order.  2D: the k_m
 *   index u in [0, N); 3D: u = ux*N + uy.
 * - A *row* is one datum of one pair: (frequency f, class of |k_r|, class of
 *   |k_s|).  Classes index the distinct |k| values of the plan (cls_k).
 * - Rows of a pair are contiguous, pairs are ordered by their representative
 *   k_m index; within a pair rows are ordered by frequency then (2D) by the
 *   signed receiver-wavenumber index, (3D) by the k_h index n_x*N_h + n_y.
 * - Device arrays are caller-owned (e.g. torch tensors); the library never
 *   allocates device memory.  All device work is enqueued on the caller's
 *   stream, nothing synchronises the host.
 * - Errors: a negative edt_status means nothing was enqueued (bad argument,
 *   missing upload, HIP launch failure).  Numerical outcomes are written per
 *   pair to info[] on the device and are valid after a stream sync.
 */
#ifndef EDT_H
#define EDT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } edt_c128;
typedef struct { float re, im; } edt_c64;

typedef enum {
    EDT_OK = 0,
    EDT_EINVAL = -1,   /* invalid argument; message via edt_last_error() */
    EDT_ENOMEM = -2,   /* host allocation failed, or a caller buffer is too small */
    EDT_EHIP = -3,     /* a HIP runtime call or kernel launch failed */
    EDT_ESTATE = -4    /* the plan has no device copy (edt_plan_upload not called) */
} edt_status;

/* per-pair info[] values; a positive value k means the Cholesky factorisation
 * met a non-positive pivot at column k-1 */
enum {
    EDT_INFO_OK = 0,
    EDT_INFO_EMPTY = -1,     /* no rows survive the evanescent cut: V~ = 0 */
    EDT_INFO_NOCONV = -2,    /* refinement did not reach refine_tol in max_refine steps */
    EDT_INFO_NONFINITE = -3  /* a NaN or Inf reached the solution */
};

typedef enum {
    EDT_FP64 = 0,    /* Gram on FP64 MFMA (v_mfma_f64_16x16x4) */
    EDT_FP32 = 1,    /* Gram on FP32 MFMA with FP32 accumulation */
    EDT_BF16X3 = 2,  /* Gram on BF16 MFMA: hi*hi + hi*lo + lo*hi, FP32 accumulation */
    EDT_FP16X3 = 3   /* the same split in IEEE half (about 22 bits per product), the rows of
                        each work item scaled by a power of two into the half range */
} edt_precision;

/*
 * Survey geometry (paper Sections 2.1-2.2 and 3.1).
 * dim 2: split-spread periodic line of n_mid positions at spacing d_mid, every
 *        source recorded by every receiver; rows of k_m index u are the receiver
 *        wavenumbers a with source wavenumber b = u - a (mod N).
 * dim 3: areal survey, k_m on an n_mid x n_mid grid (spacing 2 pi/(n_mid d_mid)),
 *        k_h on an n_off x n_off grid with n_off*d_off == n_mid*d_mid/2, so
 *        k_r = (k_m + k_h)/2 and k_s = (k_m - k_h)/2 (eq. COV).
 * dim 3 with n_line > 0: the survey of n_line parallel 2D lines of Section 2.2,
 *        n_line <= 64 lines at spacing d_line (periodic in y), each with n_mid
 *        positions at d_mid, every source recorded by every receiver of its
 *        own line (n_off, d_off ignored).  A subproblem is a (k_m, k_y) pair,
 *        flattened u = ux * n_line + c; its rows are (f, receiver index a),
 *        source index b = ux - a, with value
 *            (w^2 dz / L_y) sum_q g(|(k_a, k_q)|) g(|(k_b, k_{q-c})|),
 *        the sum over the line wavenumbers q (the k_h'' integral of the
 *        decoupled 3D equation, L_y = n_line d_line).  A term is kept iff both
 *        |k| are within the cut below, a row iff a term is.  This survey is
 *        assembled in FP64 and solved without refinement (edt_solve with
 *        refine = 0, or edt_tsvd), and edt_aperture_gram gives its finite-aperture
 *        Gram, edt_kz_restrict its k_z restriction and edt_adjoint its gradient.
 * Frequencies freq_hz[n_freq] are used simultaneously (Section 3.1); eps is the
 * imaginary part of w (Section 2.1; 0.15 1/s in Section 3.1).  Depths are
 * z_i = z0 + i*dz, i < nz.  A row is kept iff |k_r| and |k_s| are both
 * <= kappa * 2 pi f / c_top, with c_top the velocity of the source layer.
 */
typedef struct {
    int dim;
    int n_mid;
    double d_mid;
    int n_off;
    double d_off;
    int n_freq;
    const double* freq_hz;   /* host pointer, copied by edt_plan_create */
    double eps;
    int nz;
    double z0, dz;
    double kappa;
    int n_line;              /* dim 3: number of parallel lines (0: the areal survey) */
    double d_line;           /* dim 3 with n_line > 0: line spacing, m */
} edt_survey;

/* Layered reference c0(z) (Section 2.1): layer 0 extends up to -infinity and
 * holds sources and receivers at z = 0, so zif[0] > 0; layer n_layers-1 is a
 * half space; zif (host, length n_layers-1) is strictly increasing.  vel
 * (host) fixes c_top for the evanescent cut; the velocities used by the
 * kernels are passed to edt_green / edt_adjoint on the device. */
typedef struct {
    int n_layers;
    const double* vel;
    const double* zif;
} edt_layers;

typedef struct edt_plan edt_plan;

/* Storage type of the data rows d_rows (a plan option): complex128, or
 * complex64 (half the bytes; read and widened to FP64 by the kernels, which
 * compute in FP64 either way).  Every call that reads or writes data rows,
 * and the data gradient of edt_adjoint, uses the plan's type. */
typedef enum {
    EDT_DATA_C128 = 0,
    EDT_DATA_C64 = 1
} edt_data_type;

typedef struct {
    int64_t n_km;          /* number of k_m problems */
    int64_t n_pairs;       /* number of +-k_m pairs (factorisations) */
    int64_t n_rows;        /* rows summed over pairs (length of d_rows) */
    int64_t n_urows;       /* distinct Born rows: data rows of a pair with equal
                              (f, {|k_r|, |k_s|}) share one row of A */
    int64_t max_rows;      /* rows of the largest pair */
    int64_t n_empty;       /* pairs with no rows */
    int64_t n_items;       /* Gram work items (pair, frequency band, <= chunk_rows rows) */
    int n_freq, n_cls, nz, n_layers;
    int chunk_rows;        /* unique rows per Gram work item at most */
    int gram_band;         /* frequencies per Gram band */
    size_t table_elems;    /* n_freq * n_cls * nz: length of g64 / g32 */
    size_t dev_plan_bytes; /* size of the device copy of the plan */
    size_t work_bytes;     /* workspace needed by assemble / solve / adjoint */
    double gram_flops;     /* sum over pairs of 2 R_p nz (nz+1): algorithmic Gram work */
    int64_t n_pairs_all;   /* pairs of the whole survey */
    int64_t pair_begin;    /* survey index of this plan's first pair */
    int resid_group;       /* frequencies per residual work item */
    int data_type;         /* edt_data_type of d_rows */
    size_t resident_bytes; /* device bytes of one pass of this plan: the device plan, the
                              workspace, the data rows, the Gram, rhs, trace, x, info and steps
                              of its pairs, v_out (n_km x nz) and the survey's Green's tables
                              g64 and g32 */
} edt_plan_info;

typedef struct {
    int refine;            /* 0: one solve; 1: FP64 refinement (preconditioned CG) */
    double refine_tol;     /* stop when the correction ||z|| <= refine_tol ||x + z|| (per pair) */
    int max_refine;        /* at most this many refinement sweeps over the rows (<= 62) */
    int escalate;          /* with refine: pairs whose factorisation fails (info > 0) are
                              re-assembled with the FP64 Gram and factored again */
    int data_summed;       /* with refine: nonzero if `work` still holds the summed data
                              left by edt_assemble of this plan with these d_rows (nothing
                              written to work or d_rows since); the solve then does not
                              sum the data rows again */
} edt_solve_opts;

/* Message of the last failing call on this thread (static storage). */
const char* edt_last_error(void);

/*
 * Work-item shape and pair range of a plan (0 in a field = default).
 *   chunk_rows  unique rows per Gram work item at most (default and maximum 2048)
 *   gram_band   frequencies per Gram band (default: as many as keep one band's
 *               FP32 table slab, n_cls * nz * 8 bytes per frequency, near
 *               2.5 MB, so that it stays in one XCD's 4 MB L2, or, if more,
 *               as many as give an average item 256 unique rows)
 *   pair_begin, pair_end
 *               plan only the pairs [pair_begin, pair_end) of the survey's pair
 *               order (pair_end 0 = to the end): a batch of a survey too large
 *               for one workspace.  The |k| classes, and so the Green's table,
 *               are those of the whole survey, so that every batch uses one
 *               table; v_out of a batch's solve receives only its pairs' k_m.
 *   resid_group frequencies per residual work item (default: 2, widened
 *               where rows are sparse until an average item holds 64 rows)
 *   data_type   edt_data_type of the data rows (default complex128)
 *   hbm_budget  device bytes one pass of the plan may hold (0 = no limit):
 *               edt_plan_create returns EDT_ENOMEM, with the bytes needed in
 *               the message, when resident_bytes (edt_plan_info) exceeds it,
 *               e.g. when a pair range, down to a single pair, does not fit
 */
typedef struct {
    int chunk_rows;
    int gram_band;
    int64_t pair_begin;
    int64_t pair_end;
    int data_type;
    size_t hbm_budget;
    int resid_group;
} edt_plan_opts;

/*
 * Host planner: enumerates pairs and rows, the |k| classes, the unique rows
 * (rows of a pair with equal frequency and equal {|k_r|, |k_s|} share their
 * Born row) and the work items: for the Gram, a pair's rows within one
 * frequency band (<= chunk_rows of them); for the residual, within two
 * frequencies.  Both are laid out in an XCD-aware launch order.  opts is
 * nullable (= defaults).  Host only, no HIP calls.
 * Errors: EDT_EINVAL (dim, sizes, zif[0] <= 0, non-increasing zif, n_cls or
 * n_freq >= 65536, n_freq * n_cls * nz >= 2^32, chunk_rows, gram_band,
 * resid_group or data_type out of range), EDT_ENOMEM (host memory, or the plan's device
 * bytes above opts->hbm_budget).
 * *out is owned by the caller: edt_plan_destroy.
 */
edt_status edt_plan_create(const edt_survey* survey, const edt_layers* layers,
                           const edt_plan_opts* opts, edt_plan** out);

/*
 * Rows (data rows, before the unique-row merge) of every pair of the survey,
 * in the survey's pair order, without building a plan: for cutting a large
 * survey into pair-range batches.  *n_pairs_all receives the pair count;
 * rows_per_pair (nullable: query the count first) must hold that many.
 * Host only.  Errors: as edt_plan_create for the survey and layers.
 */
edt_status edt_survey_pair_rows(const edt_survey* survey, const edt_layers* layers, int64_t* n_pairs_all,
                                int64_t* rows_per_pair);
edt_status edt_plan_destroy(edt_plan* plan);
edt_status edt_plan_query(const edt_plan* plan, edt_plan_info* out);

/*
 * Host copies of the plan (every pointer nullable; sizes from edt_plan_query):
 *   row_off[n_pairs+1]  first row of each pair
 *   rows[n_rows*3]      (f, class of |k_r|, class of |k_s|); line survey:
 *                       (f, class of (|a|, 0), class of (|b|, 0))
 *   keys[n_rows*2]      2D and line survey: fftfreq indices (a, b) of the +k_m
 *                       datum, whose -k_m partner is (-b, -a) (line survey: at
 *                       -k_y); 3D areal: (k_h index n, 0)
 *   pair_km[n_pairs*2]  (u, index of -u); equal for a self-conjugate k_m
 *   cls_k[n_cls]        |k| of each class, rad/m
 */
edt_status edt_plan_rowmap(const edt_plan* plan, int64_t* row_off, int32_t* rows,
                           int32_t* keys, int32_t* pair_km, double* cls_k);

/*
 * Host copies of the unique rows (nullable outputs): urow_off[n_pairs+1] first
 * unique row of each pair; urows[n_urows*4] = (f, mult, class r, class s),
 * sorted by f within a pair; row_unique[n_rows] unique row of each data row.
 */
edt_status edt_plan_urows(const edt_plan* plan, int64_t* urow_off, int32_t* urows, int32_t* row_unique);

/*
 * Host copies of the work items and launch order (for checks and tools).
 * which 0: Gram items, 1: residual items.  counts[0] = number of items,
 * counts[1] = length of the launch order (items plus holes).  items (nullable,
 * counts[0]*3): pair, first and one-past-last unique row; sched (nullable,
 * counts[1]): item launched by workgroup b, -1 for a hole.  Workgroup b runs
 * on XCD b % 8.
 */
edt_status edt_plan_schedule(const edt_plan* plan, int which, int64_t* counts, int32_t* items,
                             int32_t* sched);

/*
 * Copy the plan's device tables into a caller device buffer of at least
 * dev_plan_bytes bytes (256-byte aligned) and remember it in the plan.  Must
 * precede every compute call; the buffer must outlive them.  Enqueued on
 * `stream` (an async copy from host memory owned by the plan).
 */
edt_status edt_plan_upload(edt_plan* plan, void* dev_buf, size_t bytes, hipStream_t stream);

/*
 * Kernel (a): Green's-function tables.  g64[f][c][z] = g(z_i; cls_k[c], w_f)
 * solving g'' + (w^2/c0(z)^2 - k^2) g = -delta(z) with radiation conditions
 * (Section 2.1), by a generalised reflection recursion over the layers.
 * g32 (nullable) receives the same table in FP32 scaled by |w_f| sqrt(dz), the
 * factor whose square |w_f^2 dz| multiplies Re(A^H A) (the phase of w^2 cancels).
 * vel_dev: device, n_layers doubles.  Shapes: n_freq*n_cls*nz.
 */
edt_status edt_green(const edt_plan* plan, const double* vel_dev, edt_c128* g64, edt_c64* g32,
                     hipStream_t stream);

/*
 * Kernel (b): per pair p, gram[p] (nz x nz, row-major, the lower triangle
 * i >= j is written) = Re(A_p^H A_p) in the given precision, and, from the
 * same pass over the rows, rhs[p][0|1][z] = Re(A_p^H b+-) and
 * trace[p] = tr Re(A_p^H A_p).  d_rows[r] = (datum at +k_m, datum at -k_m) of
 * row r, in the plan's data type (complex128 or complex64), so
 * b+ = (d0+d1)/2 and b- = (d0-d1)/(2i) (eq. Split), summed in FP64.
 * prec EDT_FP64 reads g64 and gives rhs and trace in FP64.  EDT_FP32,
 * EDT_BF16X3 and EDT_FP16X3 read g32 (from edt_green); their rhs and trace
 * come from FP32 rows summed per stage of 8 rows in FP32 and then in FP64
 * (the rhs is an approximation, about 1e-7 relative, that the FP64
 * refinement residual of edt_solve corrects; the trace is within about 1e-8).
 * work: device, >= work_bytes; it keeps the data summed per unique row, which
 * edt_solve can reuse (edt_solve_opts.data_summed).  Empty pairs get zero
 * Gram, rhs and trace.
 */
edt_status edt_assemble(const edt_plan* plan, const edt_c128* g64, const edt_c64* g32,
                        const void* d_rows, edt_precision prec, double* gram, double* rhs,
                        double* trace, void* work, hipStream_t stream);

/*
 * Kernel (c): lambda_p = lambda_rel * trace[p] / nz; gram[p] is overwritten by
 * the Cholesky factor L of gram + lambda_p I (lower triangle); x[p][0|1] =
 * (L L^T)^{-1} rhs[p][0|1].  With opts->refine, x is refined in FP64 against
 * the exact operator M = Re(A^H A) + lambda I, applied from g64 (the first
 * sweep forms the residual Re(A^H (b - A x)) - lambda x with d_rows): conjugate
 * gradients preconditioned by L L^T, finished by the correction z = (L L^T)^-1 r
 * once ||z|| <= refine_tol ||x + z||.  At most max_refine sweeps (per pair;
 * steps[p] counts them, info NOCONV if the tolerance was not met or the
 * iteration broke down).  With opts->escalate (and refine), a pair whose
 * factorisation hit a non-positive pivot (a mixed-precision Gram error above
 * lambda) is re-assembled from g64 and d_rows with the FP64 Gram, rhs and
 * trace and factored again before the refinement; info then reports the second
 * factorisation.  A self-conjugate k_m keeps
 * x- = 0.  v_out[u] = x+ + i x-, v_out[-u] = x+ - i x- (eq. VSym), zero for
 * empty pairs.  x: [n_pairs][2][nz]; v_out: [n_km][nz]; info, steps: [n_pairs]
 * (steps nullable).  opts nullable (= no refinement).  d_rows: the plan's data
 * type, as in edt_assemble.
 */
edt_status edt_solve(const edt_plan* plan, const edt_c128* g64, const void* d_rows,
                     double* gram, const double* rhs, const double* trace, double lambda_rel,
                     const edt_solve_opts* opts, double* x, edt_c128* v_out, int32_t* info,
                     int32_t* steps, void* work, hipStream_t stream);

/*
 * edt_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation, kernels and results as edt_solve, with its scratch in a
 * library-owned static device array of EDT_STATIC_SCRATCH_BYTES instead of a
 * caller workspace.  The caller still passes every input and output.
 *   - Scratch needed (bytes, each part rounded up to 256): the damping, the
 *     diagonal-block inverses (n_pairs * ceil(nz/32) * 8 KB), flags and
 *     counters; with refinement also the summed data (n_urows * 32), the
 *     residual partials (one 2 nz + 1 FP64 row per residual item) and three
 *     per-pair refinement vectors; with escalation also the FP64 Gram
 *     partials of every work item.  A plan needing more returns EDT_ENOMEM
 *     (message with the size) and nothing is enqueued.
 *   - opts->data_summed must be 0 (EDT_EINVAL): this call sums the data rows
 *     itself, since the static array does not hold edt_assemble's sums.
 *   - Each GPU holds one copy of the array until the process ends, shared by
 *     every call on that GPU, and it keeps the last call's contents (what must
 *     start at zero is cleared by kernels on the stream).  Calls on one stream
 *     are ordered; calls that overlap on one GPU (other streams, threads, or
 *     processes sharing a context) race on the array and must be serialised
 *     by the caller.
 *   - No hipMalloc, hipFree or allocating library routine is called; the
 *     first call on a device looks up that device's address of the array.
 */
#define EDT_STATIC_SCRATCH_BYTES (256u * 1024u * 1024u)
edt_status edt_solve_static(const edt_plan* plan, const edt_c128* g64, const void* d_rows, double* gram,
                            const double* rhs, const double* trace, double lambda_rel,
                            const edt_solve_opts* opts, double* x, edt_c128* v_out, int32_t* info,
                            int32_t* steps, hipStream_t stream);

/*
 * The paper's own solver (Section 3.1): per pair, the truncated-SVD solution
 * x+- = sum_{s_j^2 >= sigma^2} v_j (v_j . c+-) / s_j^2, where s_j^2 and v_j
 * are the eigenpairs of the pair's Gram (the squared singular values and the
 * right singular vectors of its real rows), with a relative tolerance
 * sigma^2 = tol_rel^2 ||G||_F (Frobenius norm).  Computed without an
 * eigen-decomposition: the spectral projector P onto eigenvalues >= sigma^2
 * comes from the matrix sign of G - sigma^2 I by scaled Newton-Schulz steps
 * (FP64 MFMA; the host fixes each step's scaling in advance, capped so that
 * rounding cannot flip a sign; at most max_iter <= 200 steps, a pair stopping
 * once ||X^2 - I||_F <= 1e-9 after an unscaled step), then
 * (G + sigma^2 (I - P)) x = P c is solved by the FP64 Cholesky path.
 * gram: in, the lower triangles from edt_assemble (use EDT_FP64 for an FP64
 * result); out, the factor of G + sigma^2 (I - P).  rhs: [P][2][nz] from
 * edt_assemble.  x, v_out, info as edt_solve; info is EDT_INFO_NOCONV for a
 * pair whose sign iteration did not converge (an eigenvalue within rounding
 * of sigma^2 has no definite side) and EDT_INFO_EMPTY for an empty pair (x =
 * 0).  iters[p]: sign steps taken (device, int32).  work: the plan's
 * workspace; tsvd_work: device, >= edt_tsvd_work_bytes (three nz x nz FP64
 * matrices per pair and small per-pair state).  A plan with no pairs returns
 * EDT_OK at once, its pointers unused.
 */
edt_status edt_tsvd_work_bytes(const edt_plan* plan, size_t* bytes);
edt_status edt_tsvd(const edt_plan* plan, double* gram, const double* rhs, double tol_rel, int max_iter,
                    double* x, edt_c128* v_out, int32_t* info, int32_t* iters, void* work, void* tsvd_work,
                    hipStream_t stream);

/*
 * Radius of the (k_m, k_z) disk of Section 3.1: k_disk = factor * 2 pi f_max
 * / c_top (rad/m), f_max the largest frequency of the plan and c_top the
 * velocity of the top layer (the paper's c0, undefined for a layered
 * reference); the paper's factor is 2.2.  Host only.
 */
edt_status edt_kz_disk_radius(const edt_plan* plan, double factor, double* k_disk);

/*
 * The k_z restriction of Section 3.1: every pair's unknowns are restricted to
 * the discrete Fourier modes in depth (k_z,j = 2 pi j / (nz dz)) with
 * k_z,j^2 + |k_m|^2 <= k_disk^2.  With Q the orthogonal projector onto those
 * modes (circulant in depth), the pair's Gram and right-hand sides become
 * Q G Q and Q c, in place; edt_tsvd on the result gives the truncated-SVD
 * solution restricted to the disk (Q G Q vanishes off the kept modes, whose
 * singular values are then zero and dropped; use tol_rel > 0).  Apply it
 * before edt_tsvd only: edt_solve's refinement works from the rows.  On the
 * survey of parallel lines the model's horizontal wavenumber is (k_m, k_y),
 * and |k_m|^2 above reads |k_m|^2 + |k_y|^2.
 * gram: [P][nz][nz] lower triangles from edt_assemble (EDT_FP64); rhs:
 * [P][2][nz]; both device, overwritten.  n_keep: device int32 [P] or NULL,
 * the number of kept real modes per pair (0 for a pair with |k_m| > k_disk,
 * whose Gram and rhs become zero).  tsvd_work: device, >= edt_tsvd_work_bytes,
 * used as scratch (it holds nothing between this call and edt_tsvd).
 * Errors: EDT_EINVAL for a null gram, rhs or tsvd_work, or k_disk negative
 * or not finite.  A plan with no pairs (an empty pair range) returns EDT_OK
 * at once, its pointers unused.
 */
edt_status edt_kz_restrict(const edt_plan* plan, double k_disk, double* gram, double* rhs, int32_t* n_keep,
                           void* tsvd_work, hipStream_t stream);

/*
 * The transforms on either side of the decoupled problems (Section 2.1), for
 * the 2D line survey, the 3D areal survey and the 3D survey of parallel lines
 * (Section 2.2); EDT_EINVAL for n_mid > 2048 and, on the areal survey, for
 * n_mid > 128.
 *
 * edt_shots_fft, 2D: shots[n_freq][n_mid][n_mid] (complex128, device; [f][R][S],
 * the record of the source at x_S = S d_mid by the receiver at x_R, at the
 * plan's frequency f) is overwritten by its transform
 *     d~[f][a][b] = d_mid sum_{R,S} D[f][R][S] exp(-2 pi i (a R + b S) / n_mid),
 * the data convention of every other call (a, b: receiver and source
 * wavenumber indices in fftfreq order).  One pass over the records per axis.
 *
 * edt_shots_fft, 3D areal: a row of k_m index q and k_h index n has receiver
 * and source wavenumbers q + 2n and q - 2n per axis in units of dk/2
 * (dk = 2 pi / (n_mid d_mid)): half-grid wavenumbers, which are whole-grid
 * ones of a survey of twice the period.  The records are therefore those of
 * the full-coverage periodic areal survey on the 2 n_mid x 2 n_mid grid of
 * spacing d_mid: shots[n_freq][M][M][M][M], M = 2 n_mid, [f][Rx][Ry][Sx][Sy]
 * (16 M^4 bytes per frequency: 69 GB at n_mid = 128), overwritten by
 *     F[f][a][b] = d_mid^2 sum_{R,S} D[f][R][S] exp(-2 pi i (a.R + b.S) / M)
 * (a, b: 2-vectors).  One pass over the records per axis.
 *
 * edt_shots_fft, 3D parallel lines: shots[n_freq][n_line][n_mid][n_mid]
 * ([f][j][R][S], the records of line j at y_j = j d_line) becomes
 *     d~[f][c][a][b] = d_mid sum_{j,R,S} D[f][j][R][S]
 *                      exp(-2 pi i (a R + b S) / n_mid) exp(-2 pi i c j / n_line).
 *
 * edt_shots_pack: d_rows[n_rows][2] (device, the plan's data type) from that
 * spectrum.  2D: row r with frequency f and key (a, b) (edt_plan_rowmap) gets
 * (d~[f][a][b], d~[f][-b][-a]), the datum at +k_m and its -k_m partner.  3D
 * areal: row r of the pair with k_m index q and of k_h index n gets
 * (F[f][a][b], F[f][-b][-a]) / 4 with a = q + 2n, b = q - 2n (mod M per
 * axis): the N-periodic model has on the doubled grid a spectrum at even
 * indices only, 4 times its own.  Parallel lines: row r of the pair with k_y
 * index c and key (a, b) gets (d~[f][c][a][b], d~[f][-c][-b][-a]).  The
 * spectrum is only read, so the plans of
 * several pair ranges (batches) of one survey can each pack from one
 * transform.
 */
edt_status edt_shots_fft(const edt_plan* plan, edt_c128* shots, hipStream_t stream);
edt_status edt_shots_pack(const edt_plan* plan, const edt_c128* spectrum, void* d_rows, hipStream_t stream);

/*
 * Finite aperture (eq. M) on the 2D line survey and the survey of parallel
 * lines: the Gram of every pair when
 * the records are kept only for full offsets |x_R - x_S| <= 2 b_max (b_max:
 * the largest half-offset, m).  On the periodic line the offset window acts
 * at each k_m as a circular convolution S of the rows over the receiver
 * index with the window's DFT (the discrete sinc of eq. M), an orthogonal
 * projector, so the normal equations of the windowed data keep edt_assemble's
 * right-hand sides and take the Gram Re(A^H S A), formed here per frequency
 * from the rows transformed over the receiver index, over the kept offsets.
 * gram: device [P][nz][nz], lower triangle written (FP64); trace: device [P],
 * its trace.  Solve with edt_solve without refinement (the refinement works
 * from the unwindowed rows) or edt_tsvd.  aperture_work: device, >=
 * edt_aperture_work_bytes (about P n_mid nz complex128: the transformed rows
 * of one frequency, plus per-pair frequency ranges and a twiddle table).
 * Survey of parallel lines (Section 2.2, whose decoupled equation carries the
 * same sinc over the offset wavenumber): the window acts on every line's
 * offsets alike, so each (k_m, k_y) pair takes the same circulant S over its
 * receiver index, applied to the line rows (built per chunk of pairs and
 * frequency); aperture_work then holds a chunk's kept offsets (at most
 * 256 MiB).
 * Errors: EDT_EINVAL for the 3D areal survey, n_mid > 2048, b_max negative or
 * not finite, or a null pointer (a plan with no pairs returns EDT_OK at once).
 */
edt_status edt_aperture_work_bytes(const edt_plan* plan, size_t* bytes);
edt_status edt_aperture_gram(const edt_plan* plan, const edt_c128* g64, double b_max, double* gram, double* trace,
                             void* aperture_work, hipStream_t stream);

/*
 * The model from its spectrum (Section 2.1): v_tilde[n_km][nz] (complex128,
 * device, fftfreq order; 3D areal u = ux n_mid + uy, parallel lines
 * u = ux n_line + c) is overwritten by its inverse transform over u (over ux
 * and uy, or ux and the line wavenumber c, in 3D),
 *     V(x_n, z) = (1/n) sum_u V~(u, z) exp(2 pi i u n / n)   (per axis of length n),
 * and model (double, device: [n_mid][nz], [n_mid][n_mid][nz] in 3D areal,
 * [n_mid][n_line][nz] on parallel lines) gets its real part.  EDT_EINVAL for
 * n_mid > 2048.
 */
edt_status edt_model(const edt_plan* plan, edt_c128* v_tilde, double* model, hipStream_t stream);

/*
 * Born forward map (eq. DMV): d_rows[r] = (A_r . v_in[u_p], A_r . v_in[-u_p]),
 * A_r = w_f^2 dz g(k_r) g(k_s), for every row r of pair p.
 * v_in: [n_km][nz] complex128; d_rows: [n_rows][2] in the plan's data type
 * (formed in FP64, rounded to complex64 for such a plan).
 */
edt_status edt_forward(const edt_plan* plan, const edt_c128* g64, const edt_c128* v_in,
                       void* d_rows, hipStream_t stream);

/*
 * Kernel (d): reverse-mode gradient of a real loss L(V~) given
 * grad_v = dL/dRe V~ + i dL/dIm V~ ([n_km][nz]).  Uses the factor `chol` and
 * solution `x` left by edt_solve, trace from edt_assemble, and recomputes the
 * Green's tables and their velocity sensitivities from vel_dev (g64 is the
 * table of the forward pass).  Outputs (each nullable):
 *   grad_d[r] = (dL/dd0, dL/dd1) in the same complex convention ([n_rows][2],
 *               the plan's data type, like d_rows)
 *   grad_lambda[0] = dL/dlambda_rel
 *   grad_vel[l] = dL/dc_l, l < n_layers
 * The evanescent-cut mask is held fixed.  On the survey of parallel lines a
 * row's gradient flows to both factors of every kept term of the row; those
 * table gradients are added atomically (their summation order varies from
 * call to call, at the rounding level), the other surveys' in a fixed order.
 */
edt_status edt_adjoint(const edt_plan* plan, const double* vel_dev, const edt_c128* g64,
                       const void* d_rows, const double* chol, const double* trace,
                       const double* x, double lambda_rel, const edt_c128* grad_v,
                       void* grad_d, double* grad_lambda, double* grad_vel, void* work,
                       hipStream_t stream);

/*
 * Optional kernel timing, for benchmarks: with timing enabled every kernel
 * launch made for `plan` is bracketed by two HIP events on its stream (no
 * device memory, no host sync).  edt_timing_read waits for the recorded
 * events and returns, per kernel name, the summed milliseconds and launch
 * count since the previous read: names[k*32 .. k*32+31] (NUL-terminated),
 * ms[k], count[k] for k < min(*n_out, max_entries).  Not for use while a
 * stream is being captured into a graph.
 */
edt_status edt_timing_enable(edt_plan* plan, int enable);
edt_status edt_timing_read(edt_plan* plan, int max_entries, char* names, double* ms, int64_t* count,
                           int* n_out);

#ifdef __cplusplus
}
#endif
#endif /* EDT_H */
