// Host planner: pairs, rows, |k| classes and assembly work items.
//
// Paper, Section 2.1 (eqs. DMV, M, COV, VSym, Split) and Section 3.1: each
// midpoint wavenumber k_m is an independent 1D problem whose data (rows) are
// indexed by frequency and offset wavenumber; +k_m and -k_m share their rows
// (M is even in k_m) and are solved as one pair.  Rows whose |k_r| or |k_s|
// exceed kappa * 2 pi f / c_top are cut (evanescent at the surface).
//
// The row enumeration below decides integer outcomes (which rows exist) from
// floating-point comparisons.  They are written as plain IEEE double
// expressions, evaluated left to right with no contraction (this file is
// built with -ffp-contract=off), so that any other implementation that
// evaluates the same expressions in the same order takes the same decisions.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>

#include "edt_internal.h"

namespace {

thread_local std::string g_err;

constexpr double kTwoPi = 2.0 * 3.141592653589793;   // == 2.0 * numpy.pi
constexpr int kDefaultChunk = 2048;

inline int64_t signed_of(int64_t n, int64_t N) { return n < (N + 1) / 2 ? n : n - N; }
inline int64_t wrap(int64_t n, int64_t N) { return ((n % N) + N) % N; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

edt_status fail(edt_status s, const std::string& m) {
    g_err = m;
    return s;
}

// 2D periodic split-spread survey: rows of u are receiver wavenumbers a with
// source wavenumber b = u - a (mod N); class of a wavenumber = |signed index|.
void rows_2d(edt_plan* p, const std::vector<double>& kmax, std::vector<int64_t>& cls_of_row_r,
             std::vector<int64_t>& cls_of_row_s) {
    const int64_t N = p->n_mid;
    const double dk = kTwoPi / (double(N) * p->d_mid);
    p->n_km = N;
    p->row_off.push_back(0);
    for (int64_t u = 0; u <= N / 2; ++u) {
        const int64_t un = wrap(-u, N);
        p->pair_u.push_back(int32_t(u));
        p->pair_u.push_back(int32_t(un));
        for (int f = 0; f < p->n_freq; ++f) {
            for (int64_t qa = -(N / 2); qa < N - N / 2; ++qa) {
                const int64_t qb = signed_of(wrap(u - qa, N), N);
                const bool keep = (std::fabs(double(qa)) * dk <= kmax[f]) &&
                                  (std::fabs(double(qb)) * dk <= kmax[f]);
                if (!keep) continue;
                p->rows.push_back(uint32_t(f));
                p->rows.push_back(0);   // classes filled later
                cls_of_row_r.push_back(std::llabs(qa));
                cls_of_row_s.push_back(std::llabs(qb));
                p->keys.push_back(int32_t(wrap(qa, N)));
                p->keys.push_back(int32_t(wrap(qb, N)));
            }
        }
        p->row_off.push_back(int64_t(cls_of_row_r.size()));
    }
}

// 3D areal survey: in units of dk/2, k_r = q_u + 2n and k_s = q_u - 2n for the
// signed k_m index q_u and k_h index n; class key = |k|^2 / (dk/2)^2 (integer).
void rows_3d(edt_plan* p, const std::vector<double>& kmax, std::vector<int64_t>& key_r,
             std::vector<int64_t>& key_s) {
    const int64_t N = p->n_mid, Nh = p->n_off;
    const double dk = kTwoPi / (double(N) * p->d_mid);
    const double hh = (0.5 * dk) * (0.5 * dk);
    std::vector<double> kmax2(kmax.size());
    for (size_t f = 0; f < kmax.size(); ++f) kmax2[f] = kmax[f] * kmax[f];
    p->n_km = N * N;
    p->row_off.push_back(0);
    for (int64_t u = 0; u < N * N; ++u) {
        const int64_t ux = u / N, uy = u % N;
        const int64_t un = wrap(-ux, N) * N + wrap(-uy, N);
        if (un < u) continue;
        const int64_t qx = signed_of(ux, N), qy = signed_of(uy, N);
        p->pair_u.push_back(int32_t(u));
        p->pair_u.push_back(int32_t(un));
        for (int f = 0; f < p->n_freq; ++f) {
            int64_t nflat = 0;
            for (int64_t nx = -(Nh / 2); nx < Nh - Nh / 2; ++nx) {
                for (int64_t ny = -(Nh / 2); ny < Nh - Nh / 2; ++ny, ++nflat) {
                    const int64_t sr = (qx + 2 * nx) * (qx + 2 * nx) + (qy + 2 * ny) * (qy + 2 * ny);
                    const int64_t ss = (qx - 2 * nx) * (qx - 2 * nx) + (qy - 2 * ny) * (qy - 2 * ny);
                    const bool keep = (double(sr) * hh <= kmax2[f]) && (double(ss) * hh <= kmax2[f]);
                    if (!keep) continue;
                    p->rows.push_back(uint32_t(f));
                    p->rows.push_back(0);
                    key_r.push_back(sr);
                    key_s.push_back(ss);
                    p->keys.push_back(int32_t(nflat));
                    p->keys.push_back(0);
                }
            }
        }
        p->row_off.push_back(int64_t(key_r.size()));
    }
}

}  // namespace

namespace edt {

void set_error(const std::string& msg) { g_err = msg; }

size_t gram_part_bytes_per_item(const edt_plan* p) {
    const size_t nt = size_t((p->nz + 31) / 32);
    return nt * (nt + 1) / 2 * 1024 * sizeof(double);
}

WorkLayout work_layout(const edt_plan* p) {
    WorkLayout w{};
    size_t off = 0;
    const size_t P = size_t(p->n_pairs), nz = size_t(p->nz);
    w.ub = off;
    off = align256(off + size_t(p->n_urows) * 2 * 16);
    w.gram_part = off;
    off = align256(off + size_t(p->items.size()) * gram_part_bytes_per_item(p));
    w.rhs_part = off;
    off = align256(off + size_t(p->items.size()) * (2 * nz + 1) * sizeof(double));
    w.lam = off;
    off = align256(off + P * sizeof(double));
    w.conv = off;
    off = align256(off + P * sizeof(int32_t));
    w.aux = off;
    off = align256(off + P * 2 * nz * sizeof(double));
    w.aux2 = off;
    off = align256(off + P * 2 * nz * sizeof(double));
    w.gbar = off;
    off = align256(off + size_t(p->n_freq) * size_t(p->n_cls) * nz * 2 * sizeof(double));
    w.adj_y = off;
    off = align256(off + P * 2 * nz * sizeof(double));
    w.adj_dl = off;
    off = align256(off + P * sizeof(double));
    w.adj_row = off;
    off = align256(off + size_t(p->n_urows) * 4 * 2 * sizeof(double));
    w.adj_vel = off;
    off = align256(off + size_t(p->n_freq) * size_t(p->n_cls) * size_t(p->n_layers) * sizeof(double));
    w.scal = off;
    off = align256(off + 64 * sizeof(double));
    w.total = off;
    return w;
}

}  // namespace edt

extern "C" {

const char* edt_last_error(void) { return g_err.c_str(); }

edt_status edt_plan_create(const edt_survey* s, const edt_layers* l, int chunk_rows,
                           edt_plan** out) {
    if (!s || !l || !out) return fail(EDT_EINVAL, "null argument");
    *out = nullptr;
    if (s->dim != 2 && s->dim != 3) return fail(EDT_EINVAL, "dim must be 2 or 3");
    if (s->n_mid < 2 || !(s->d_mid > 0)) return fail(EDT_EINVAL, "n_mid >= 2 and d_mid > 0 required");
    if (s->n_freq < 1 || s->n_freq >= 65536 || !s->freq_hz) return fail(EDT_EINVAL, "1 <= n_freq < 65536");
    if (s->nz < 1 || s->nz > 1024) return fail(EDT_EINVAL, "1 <= nz <= 1024");
    if (!(s->dz > 0) || !(s->eps >= 0) || !(s->kappa > 0)) return fail(EDT_EINVAL, "dz > 0, eps >= 0, kappa > 0");
    if (s->dim == 3) {
        if (s->n_off < 1 || !(s->d_off > 0)) return fail(EDT_EINVAL, "3D needs n_off >= 1, d_off > 0");
        const double a = double(s->n_off) * s->d_off, b = double(s->n_mid) * s->d_mid / 2.0;
        if (std::fabs(a - b) > 1e-9 * b) return fail(EDT_EINVAL, "3D areal survey needs n_off*d_off == n_mid*d_mid/2");
    }
    if (l->n_layers < 1 || l->n_layers > edt::kMaxLayers || !l->vel)
        return fail(EDT_EINVAL, "1 <= n_layers <= 64");
    if (l->n_layers > 1) {
        if (!l->zif) return fail(EDT_EINVAL, "zif required");
        if (!(l->zif[0] > 0)) return fail(EDT_EINVAL, "zif[0] > 0 required (sources in layer 0)");
        for (int j = 1; j < l->n_layers - 1; ++j)
            if (!(l->zif[j] > l->zif[j - 1])) return fail(EDT_EINVAL, "zif must increase");
    }
    for (int j = 0; j < l->n_layers; ++j)
        if (!(l->vel[j] > 0) || !std::isfinite(l->vel[j])) return fail(EDT_EINVAL, "velocities must be positive");
    for (int f = 0; f < s->n_freq; ++f)
        if (!(s->freq_hz[f] > 0) || !std::isfinite(s->freq_hz[f])) return fail(EDT_EINVAL, "frequencies must be positive");

    edt_plan* p = new (std::nothrow) edt_plan();
    if (!p) return fail(EDT_ENOMEM, "out of host memory");
    try {
        p->dim = s->dim;
        p->n_mid = s->n_mid;
        p->n_off = s->dim == 3 ? s->n_off : 0;
        p->n_freq = s->n_freq;
        p->nz = s->nz;
        p->n_layers = l->n_layers;
        p->d_mid = s->d_mid;
        p->d_off = s->dim == 3 ? s->d_off : 0.0;
        p->eps = s->eps;
        p->z0 = s->z0;
        p->dz = s->dz;
        p->kappa = s->kappa;
        p->ctop = l->vel[0];
        p->freq.assign(s->freq_hz, s->freq_hz + s->n_freq);
        if (l->n_layers > 1) p->zif.assign(l->zif, l->zif + l->n_layers - 1);
        std::vector<double> kmax(s->n_freq);
        for (int f = 0; f < s->n_freq; ++f) kmax[f] = p->kappa * (kTwoPi * p->freq[f]) / p->ctop;

        std::vector<int64_t> kr, ks;
        if (p->dim == 2) rows_2d(p, kmax, kr, ks);
        else rows_3d(p, kmax, kr, ks);
        p->n_pairs = int64_t(p->row_off.size()) - 1;
        p->n_rows = p->row_off.back();
        if (p->n_rows >= (int64_t(1) << 31)) { delete p; return fail(EDT_EINVAL, "more than 2^31 rows"); }

        // classes: 2D class = |q| (|k| = |q| dk); 3D class = rank of the integer key
        const double dk = kTwoPi / (double(p->n_mid) * p->d_mid);
        std::map<int64_t, int> cls;
        if (p->dim == 2) {
            int64_t mx = -1;
            for (int64_t v : kr) mx = std::max(mx, v);
            for (int64_t v : ks) mx = std::max(mx, v);
            p->n_cls = int(mx + 1);
            for (int c = 0; c < p->n_cls; ++c) p->cls_k.push_back(std::fabs(double(c)) * dk);
        } else {
            for (int64_t v : kr) cls[v] = 0;
            for (int64_t v : ks) cls[v] = 0;
            int c = 0;
            for (auto& kv : cls) {
                kv.second = c++;
                p->cls_k.push_back(std::sqrt(double(kv.first)) * (0.5 * dk));
            }
            p->n_cls = c;
        }
        if (p->n_cls == 0) { p->n_cls = 1; p->cls_k.push_back(0.0); }
        if (p->n_cls >= 65536) { delete p; return fail(EDT_EINVAL, "more than 65535 |k| classes"); }
        for (int64_t r = 0; r < p->n_rows; ++r) {
            uint32_t cr, cs;
            if (p->dim == 2) { cr = uint32_t(kr[r]); cs = uint32_t(ks[r]); }
            else { cr = uint32_t(cls[kr[r]]); cs = uint32_t(cls[ks[r]]); }
            p->rows[2 * r + 1] = cr | (cs << 16);
        }

        // unique rows: within a pair, data rows with the same frequency and the
        // same unordered class pair have the same Born row A
        p->urow_off.push_back(0);
        p->row_unique.assign(size_t(p->n_rows), -1);
        std::vector<std::vector<int32_t>> members;
        for (int64_t q = 0; q < p->n_pairs; ++q) {
            std::map<uint64_t, int64_t> seen;
            for (int64_t r = p->row_off[q]; r < p->row_off[q + 1]; ++r) {
                const uint64_t f = p->rows[2 * r];
                const uint64_t a = p->rows[2 * r + 1] & 0xFFFFu, b = p->rows[2 * r + 1] >> 16;
                const uint64_t key = (f << 32) | (std::min(a, b) << 16) | std::max(a, b);
                auto it = seen.find(key);
                int64_t uidx;
                if (it == seen.end()) {
                    uidx = int64_t(members.size());
                    seen.emplace(key, uidx);
                    members.emplace_back();
                    p->urows.push_back(uint32_t(f));
                    p->urows.push_back(uint32_t(std::min(a, b) | (std::max(a, b) << 16)));
                } else {
                    uidx = it->second;
                }
                members[size_t(uidx)].push_back(int32_t(r));
                p->row_unique[size_t(r)] = int32_t(uidx);
            }
            p->urow_off.push_back(int64_t(members.size()));
        }
        p->n_urows = int64_t(members.size());
        p->urow_pair.assign(size_t(p->n_urows), 0);
        for (int64_t q = 0; q < p->n_pairs; ++q)
            for (int64_t uidx = p->urow_off[q]; uidx < p->urow_off[q + 1]; ++uidx)
                p->urow_pair[size_t(uidx)] = int32_t(q);
        {
            // contributors of each table entry, in unique-row order (deterministic)
            const size_t ne = size_t(p->n_freq) * size_t(p->n_cls);
            std::vector<int32_t> cnt(ne + 1, 0);
            for (int64_t uidx = 0; uidx < p->n_urows; ++uidx) {
                const uint32_t f = p->urows[2 * uidx];
                const uint32_t a = p->urows[2 * uidx + 1] & 0xFFFFu, b = p->urows[2 * uidx + 1] >> 16;
                cnt[size_t(f) * p->n_cls + a + 1]++;
                cnt[size_t(f) * p->n_cls + b + 1]++;
            }
            for (size_t e = 0; e < ne; ++e) cnt[e + 1] += cnt[e];
            p->tab_off = cnt;
            p->tab_ent.assign(size_t(cnt[ne]) * 2, 0);
            std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
            for (int64_t uidx = 0; uidx < p->n_urows; ++uidx) {
                const uint32_t f = p->urows[2 * uidx];
                const uint32_t a = p->urows[2 * uidx + 1] & 0xFFFFu, b = p->urows[2 * uidx + 1] >> 16;
                int32_t k = fill[size_t(f) * p->n_cls + a]++;
                p->tab_ent[2 * size_t(k)] = int32_t(uidx);
                p->tab_ent[2 * size_t(k) + 1] = int32_t(b);
                k = fill[size_t(f) * p->n_cls + b]++;
                p->tab_ent[2 * size_t(k)] = int32_t(uidx);
                p->tab_ent[2 * size_t(k) + 1] = int32_t(a);
            }
        }
        p->umem_off.push_back(0);
        for (size_t uidx = 0; uidx < members.size(); ++uidx) {
            const size_t m = members[uidx].size();
            if (m >= 65536) { delete p; return fail(EDT_EINVAL, "row multiplicity >= 65536"); }
            p->urows[2 * uidx] |= uint32_t(m) << 16;
            for (int32_t r : members[uidx]) p->umem.push_back(r);
            p->umem_off.push_back(int32_t(p->umem.size()));
        }

        // stats (algorithmic Gram work counts every data row)
        p->max_rows = 0;
        p->n_empty = 0;
        p->gram_flops = 0;
        for (int64_t q = 0; q < p->n_pairs; ++q) {
            const int64_t R = p->row_off[q + 1] - p->row_off[q];
            p->max_rows = std::max(p->max_rows, R);
            if (R == 0) ++p->n_empty;
            p->gram_flops += 2.0 * double(R) * double(p->nz) * double(p->nz + 1);
        }

        // work items: chunks of a pair's unique rows; slots are pair-major
        p->chunk_rows = chunk_rows > 0 ? chunk_rows : kDefaultChunk;
        p->pair_item.push_back(0);
        for (int64_t q = 0; q < p->n_pairs; ++q) {
            for (int64_t b = p->urow_off[q]; b < p->urow_off[q + 1]; b += p->chunk_rows) {
                const int64_t e = std::min(p->urow_off[q + 1], b + p->chunk_rows);
                p->items.push_back(edt::Item{int32_t(q), int32_t(b), int32_t(e), int32_t(p->items.size())});
            }
            p->pair_item.push_back(int32_t(p->items.size()));
        }
        p->sched.resize(p->items.size());
        std::iota(p->sched.begin(), p->sched.end(), 0);
        std::stable_sort(p->sched.begin(), p->sched.end(), [&](int32_t a, int32_t b) {
            return (p->items[a].row_end - p->items[a].row_begin) > (p->items[b].row_end - p->items[b].row_begin);
        });

        // device image
        edt::DevLayout& L = p->lay;
        size_t off = 0;
        L.freq = off;      off = align256(off + p->freq.size() * 8);
        L.zif = off;       off = align256(off + std::max<size_t>(1, p->zif.size()) * 8);
        L.cls_k = off;     off = align256(off + p->cls_k.size() * 8);
        L.row_off = off;   off = align256(off + p->row_off.size() * 8);
        L.pair_u = off;    off = align256(off + p->pair_u.size() * 4);
        L.rows = off;      off = align256(off + std::max<size_t>(1, p->rows.size()) * 4);
        L.urow_off = off;  off = align256(off + p->urow_off.size() * 8);
        L.urows = off;     off = align256(off + std::max<size_t>(1, p->urows.size()) * 4);
        L.umem_off = off;  off = align256(off + p->umem_off.size() * 4);
        L.umem = off;      off = align256(off + std::max<size_t>(1, p->umem.size()) * 4);
        L.row_unique = off; off = align256(off + std::max<size_t>(1, p->row_unique.size()) * 4);
        L.urow_pair = off; off = align256(off + std::max<size_t>(1, p->urow_pair.size()) * 4);
        L.tab_off = off;   off = align256(off + p->tab_off.size() * 4);
        L.tab_ent = off;   off = align256(off + std::max<size_t>(1, p->tab_ent.size()) * 4);
        L.items = off;     off = align256(off + std::max<size_t>(1, p->items.size()) * sizeof(edt::Item));
        L.sched = off;     off = align256(off + std::max<size_t>(1, p->sched.size()) * 4);
        L.pair_item = off; off = align256(off + p->pair_item.size() * 4);
        L.total = off;
        p->host_image.assign(L.total, 0);
        auto put = [&](size_t o, const void* src, size_t n) { if (n) std::memcpy(p->host_image.data() + o, src, n); };
        put(L.freq, p->freq.data(), p->freq.size() * 8);
        put(L.zif, p->zif.data(), p->zif.size() * 8);
        put(L.cls_k, p->cls_k.data(), p->cls_k.size() * 8);
        put(L.row_off, p->row_off.data(), p->row_off.size() * 8);
        put(L.pair_u, p->pair_u.data(), p->pair_u.size() * 4);
        put(L.rows, p->rows.data(), p->rows.size() * 4);
        put(L.urow_off, p->urow_off.data(), p->urow_off.size() * 8);
        put(L.urows, p->urows.data(), p->urows.size() * 4);
        put(L.umem_off, p->umem_off.data(), p->umem_off.size() * 4);
        put(L.umem, p->umem.data(), p->umem.size() * 4);
        put(L.row_unique, p->row_unique.data(), p->row_unique.size() * 4);
        put(L.urow_pair, p->urow_pair.data(), p->urow_pair.size() * 4);
        put(L.tab_off, p->tab_off.data(), p->tab_off.size() * 4);
        put(L.tab_ent, p->tab_ent.data(), p->tab_ent.size() * 4);
        put(L.items, p->items.data(), p->items.size() * sizeof(edt::Item));
        put(L.sched, p->sched.data(), p->sched.size() * 4);
        put(L.pair_item, p->pair_item.data(), p->pair_item.size() * 4);
    } catch (const std::bad_alloc&) {
        delete p;
        return fail(EDT_ENOMEM, "out of host memory while planning");
    }
    *out = p;
    return EDT_OK;
}

edt_status edt_plan_destroy(edt_plan* p) {
    delete p;
    return EDT_OK;
}

edt_status edt_plan_query(const edt_plan* p, edt_plan_info* o) {
    if (!p || !o) return fail(EDT_EINVAL, "null argument");
    o->n_km = p->n_km;
    o->n_pairs = p->n_pairs;
    o->n_rows = p->n_rows;
    o->n_urows = p->n_urows;
    o->max_rows = p->max_rows;
    o->n_empty = p->n_empty;
    o->n_items = int64_t(p->items.size());
    o->n_freq = p->n_freq;
    o->n_cls = p->n_cls;
    o->nz = p->nz;
    o->n_layers = p->n_layers;
    o->chunk_rows = p->chunk_rows;
    o->table_elems = size_t(p->n_freq) * size_t(p->n_cls) * size_t(p->nz);
    o->dev_plan_bytes = p->lay.total;
    o->work_bytes = edt::work_layout(p).total;
    o->gram_flops = p->gram_flops;
    return EDT_OK;
}

edt_status edt_plan_rowmap(const edt_plan* p, int64_t* row_off, int32_t* rows, int32_t* keys,
                           int32_t* pair_km, double* cls_k) {
    if (!p) return fail(EDT_EINVAL, "null plan");
    if (row_off) std::memcpy(row_off, p->row_off.data(), p->row_off.size() * 8);
    if (rows)
        for (int64_t r = 0; r < p->n_rows; ++r) {
            rows[3 * r] = int32_t(p->rows[2 * r]);
            rows[3 * r + 1] = int32_t(p->rows[2 * r + 1] & 0xFFFFu);
            rows[3 * r + 2] = int32_t(p->rows[2 * r + 1] >> 16);
        }
    if (keys) std::memcpy(keys, p->keys.data(), p->keys.size() * 4);
    if (pair_km) std::memcpy(pair_km, p->pair_u.data(), p->pair_u.size() * 4);
    if (cls_k) std::memcpy(cls_k, p->cls_k.data(), p->cls_k.size() * 8);
    return EDT_OK;
}

}  // extern "C"
