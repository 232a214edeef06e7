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
constexpr int kMaxChunk = 2048;   // row records of an item must fit in LDS
constexpr int kFreqGroup = 2;     // frequencies per residual work item
constexpr int kResidRows = 1024;  // rows per residual work item at most
constexpr int kXcd = 8;           // accelerator dies (separate L2 caches) on MI355X
constexpr double kL2Slab = 2.5e6; // bytes of FP32 table per Gram band (an XCD's L2 is 4 MB)
constexpr int kMinItemRows = 256; // unique rows of an average Gram work item at least, where the band allows
constexpr int kMinResidRows = 64; // unique rows of an average residual work item at least

inline int64_t signed_of(int64_t n, int64_t N) { return n < (N + 1) / 2 ? n : n - N; }
inline int64_t wrap(int64_t n, int64_t N) { return ((n % N) + N) % N; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Order the unique rows of one pair and frequency along chains of shared
// table columns: a unique row joins its two |k| classes, and consecutive rows
// of a chain share one class (the 2D rows (a, u - a) form paths
// ... -|u - a|-|a|-|u + a|- ...).  Each row is oriented so that its first
// class is the one it shares with the row before it.  grp[g] = [i, j) of seg
// (sorted by the unordered class pair); walk receives (g, first | second << 16)
// in chain order.  Deterministic: classes are taken in the order the sorted
// rows first name them; paths start at odd-degree classes (path ends), then at
// any class with an unused row.  Linear in the number of rows (an adjacency
// list by counting, no sort).
void chain_order(const std::vector<std::pair<uint32_t, int32_t>>& seg,
                 const std::vector<std::pair<uint32_t, uint32_t>>& grp,
                 std::vector<std::pair<uint32_t, uint32_t>>& walk) {
    const size_t G = grp.size();
    walk.clear();
    static thread_local std::vector<int32_t> deg(65536, 0), start(65536, 0), cursor(65536, 0);
    static thread_local std::vector<uint32_t> touched, adj;
    static thread_local std::vector<char> used;
    touched.clear();
    auto ends = [&](size_t g, uint32_t& a, uint32_t& b) {
        const uint32_t key = seg[grp[g].first].first;
        a = key & 0xFFFFu;
        b = key >> 16;
    };
    for (size_t g = 0; g < G; ++g) {
        uint32_t a, b;
        ends(g, a, b);
        if (deg[a]++ == 0) touched.push_back(a);
        if (b != a && deg[b]++ == 0) touched.push_back(b);
    }
    int32_t off = 0;
    for (const uint32_t c : touched) {
        start[c] = cursor[c] = off;
        off += deg[c];
    }
    adj.resize(size_t(off));
    for (size_t g = 0; g < G; ++g) {
        uint32_t a, b;
        ends(g, a, b);
        adj[size_t(cursor[a]++)] = uint32_t(g);
        if (b != a) adj[size_t(cursor[b]++)] = uint32_t(g);
    }
    for (const uint32_t c : touched) cursor[c] = start[c];
    used.assign(G, 0);
    auto walk_from = [&](uint32_t c) {
        for (;;) {
            int32_t& cur = cursor[c];
            const int32_t end = start[c] + deg[c];
            while (cur < end && used[adj[size_t(cur)]]) ++cur;
            if (cur >= end) return;
            const uint32_t g = adj[size_t(cur)];
            used[g] = 1;
            uint32_t a, b;
            ends(g, a, b);
            const uint32_t o = a == c ? b : a;
            walk.push_back({g, c | (o << 16)});
            c = o;
        }
    };
    for (const uint32_t c : touched)
        if (deg[c] % 2 == 1) walk_from(c);
    for (const uint32_t c : touched) walk_from(c);
    for (const uint32_t c : touched) deg[c] = 0;
}

// Split every pair's unique rows (sorted by frequency) into work items that
// stay inside one band of `band` frequencies and hold at most `max_rows`
// rows.  Items are pair-major; pair_first[q] is the first item of pair q and
// band_of[i] the frequency band of item i.
void split_items(const edt_plan* p, int band, int64_t max_rows, std::vector<edt::Item>& items,
                 std::vector<int32_t>& pair_first, std::vector<int32_t>& band_of) {
    items.clear();
    pair_first.assign(1, 0);
    band_of.clear();
    for (int64_t q = 0; q < p->n_pairs; ++q) {
        int64_t b = p->urow_off[q];
        while (b < p->urow_off[q + 1]) {
            const int g = int(p->urows[2 * b] & 0xFFFFu) / band;
            int64_t e = b;
            while (e < p->urow_off[q + 1] && e - b < max_rows && int(p->urows[2 * e] & 0xFFFFu) / band == g) ++e;
            items.push_back(edt::Item{int32_t(q), int32_t(b), int32_t(e), int32_t(items.size())});
            band_of.push_back(g);
            b = e;
        }
        pair_first.push_back(int32_t(items.size()));
    }
}

// XCD-aware launch order.  Workgroup b of a launch runs on XCD b % kXcd and
// each XCD starts its workgroups in launch order.  Items sorted by (band,
// rows descending) are cut into kXcd contiguous runs of about equal row count,
// so each XCD walks a few neighbouring bands (their table slabs stay in its
// L2) and the XCDs finish together; run x fills positions x, x + kXcd, ...
// Shorter runs are padded with holes (-1), which exit at once.
std::vector<int32_t> xcd_schedule(const std::vector<edt::Item>& items, const std::vector<int32_t>& band_of) {
    std::vector<int32_t> order(items.size());
    std::iota(order.begin(), order.end(), 0);
    auto rows = [&](int32_t i) { return int64_t(items[size_t(i)].row_end) - items[size_t(i)].row_begin; };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (band_of[size_t(a)] != band_of[size_t(b)]) return band_of[size_t(a)] < band_of[size_t(b)];
        return rows(a) > rows(b);
    });
    int64_t total = 0;
    for (int32_t i : order) total += rows(i);
    std::vector<std::vector<int32_t>> run(kXcd);
    int64_t acc = 0;
    for (int32_t i : order) {
        // XCD of an item: where the midpoint of its rows falls in the total
        const int64_t mid = acc + rows(i) / 2;
        const int x = total > 0 ? int(std::min<int64_t>(kXcd - 1, mid * kXcd / total)) : 0;
        run[size_t(x)].push_back(i);
        acc += rows(i);
    }
    size_t len = 0;
    for (auto& r : run) len = std::max(len, r.size());
    std::vector<int32_t> sched(len * kXcd, -1);
    for (int x = 0; x < kXcd; ++x)
        for (size_t k = 0; k < run[size_t(x)].size(); ++k) sched[k * kXcd + size_t(x)] = run[size_t(x)][k];
    return sched;
}


edt_status fail(edt_status s, const std::string& m) {
    g_err = m;
    return s;
}

// Pairs [pb, pe) of the survey's pair order get their rows; the |k| classes
// (the columns of the Green's table) are those of the whole survey, so that
// plans of different pair ranges share one table.

// 2D periodic split-spread survey: rows of u are receiver wavenumbers a with
// source wavenumber b = u - a (mod N); class of a wavenumber = |signed index|.
// max_cls: the largest class of any row of any pair.
void rows_2d(edt_plan* p, const std::vector<double>& kmax, int64_t pb, int64_t pe, std::vector<int64_t>& cls_of_row_r,
             std::vector<int64_t>& cls_of_row_s, int64_t& max_cls, int64_t& n_all,
             std::vector<int64_t>* counts = nullptr) {
    const int64_t N = p->n_mid;
    const double dk = kTwoPi / (double(N) * p->d_mid);
    p->n_km = N;
    p->row_off.push_back(0);
    max_cls = -1;
    n_all = N / 2 + 1;
    for (int64_t u = 0; u <= N / 2; ++u) {
        const bool mine = u >= pb && u < pe;
        const int64_t un = wrap(-u, N);
        if (mine) {
            p->pair_u.push_back(int32_t(u));
            p->pair_u.push_back(int32_t(un));
        }
        int64_t kept = 0;
        for (int f = 0; f < p->n_freq; ++f) {
            for (int64_t qa = -(N / 2); qa < N - N / 2; ++qa) {
                const int64_t qb = signed_of(wrap(u - qa, N), N);
                const bool keep = (std::fabs(double(qa)) * dk <= kmax[f]) &&
                                  (std::fabs(double(qb)) * dk <= kmax[f]);
                if (!keep) continue;
                ++kept;
                max_cls = std::max<int64_t>(max_cls, std::max<int64_t>(std::llabs(qa), std::llabs(qb)));
                if (!mine) continue;
                p->rows.push_back(uint32_t(f));
                p->rows.push_back(0);   // classes filled later
                cls_of_row_r.push_back(std::llabs(qa));
                cls_of_row_s.push_back(std::llabs(qb));
                p->keys.push_back(int32_t(wrap(qa, N)));
                p->keys.push_back(int32_t(wrap(qb, N)));
            }
        }
        if (mine) p->row_off.push_back(int64_t(cls_of_row_r.size()));
        if (counts) counts->push_back(kept);
    }
}

// 3D areal survey: in units of dk/2, k_r = q_u + 2n and k_s = q_u - 2n for the
// signed k_m index q_u and k_h index n; class key = |k|^2 / (dk/2)^2 (integer).
// key_used[v] = 1 for every key v of any row of any pair.
void rows_3d(edt_plan* p, const std::vector<double>& kmax, int64_t pb, int64_t pe, std::vector<int64_t>& key_r,
             std::vector<int64_t>& key_s, std::vector<uint8_t>& key_used, int64_t& n_all,
             std::vector<int64_t>* counts = nullptr) {
    const int64_t N = p->n_mid, Nh = p->n_off;
    const double dk = kTwoPi / (double(N) * p->d_mid);
    const double hh = (0.5 * dk) * (0.5 * dk);
    std::vector<double> kmax2(kmax.size());
    for (size_t f = 0; f < kmax.size(); ++f) kmax2[f] = kmax[f] * kmax[f];
    p->n_km = N * N;
    p->row_off.push_back(0);
    // When the largest disk |a|^2 <= K (a in units of dk/2) fits inside the
    // k_m index range, every key a^2 + b^2 of the disk is used (by the row
    // k_r = k_s = a of k_m index a, k_h = 0, at the highest frequency) and no
    // other key can be: the key set is known without visiting the pairs
    // outside [pb, pe).
    double k2max = 0.0;
    for (double v : kmax2) k2max = std::max(k2max, v);
    const int64_t rmax = int64_t(std::floor(std::sqrt(k2max / hh))) + 1;
    const bool disk_inside = rmax < N / 2 - 1 && Nh >= 1;
    if (disk_inside) {
        key_used.assign(size_t(2 * rmax * rmax + 1), 0);
        for (int64_t a = -rmax; a <= rmax; ++a)
            for (int64_t b = -rmax; b <= rmax; ++b) {
                const int64_t v = a * a + b * b;
                if (double(v) * hh <= k2max) key_used[size_t(v)] = 1;
            }
    }
    int64_t gp = 0;   // pair index in the survey's pair order
    for (int64_t u = 0; u < N * N; ++u) {
        const int64_t ux = u / N, uy = u % N;
        const int64_t un = wrap(-ux, N) * N + wrap(-uy, N);
        if (un < u) continue;
        const bool mine = gp >= pb && gp < pe;
        ++gp;
        if (!mine && disk_inside && !counts) continue;
        int64_t kept = 0;
        const int64_t qx = signed_of(ux, N), qy = signed_of(uy, N);
        if (mine) {
            p->pair_u.push_back(int32_t(u));
            p->pair_u.push_back(int32_t(un));
        }
        for (int f = 0; f < p->n_freq; ++f) {
            // Only offsets inside both disks |q_u +- 2n|^2 <= K can be kept; the
            // loops are narrowed to that box (with a margin of one) and the exact
            // test below decides, so the rows are those of the full enumeration.
            const double K = kmax2[f] / hh;
            const int64_t rK = int64_t(std::floor(std::sqrt(std::max(K, 0.0)))) + 1;
            const int64_t nlo = -(Nh / 2), nhi = Nh - Nh / 2;   // [nlo, nhi)
            auto range = [&](int64_t q, int64_t& lo, int64_t& hi) {
                // 2n in [-rK - q, rK - q] and in [q - rK, q + rK]
                const int64_t a = std::max(-rK - q, q - rK), b = std::min(rK - q, q + rK);
                lo = std::max(nlo, (a >= 0 ? (a + 1) / 2 : -((-a) / 2)) - 1);
                hi = std::min(nhi, (b >= 0 ? b / 2 : -((-b + 1) / 2)) + 2);
            };
            int64_t xlo, xhi, ylo, yhi;
            range(qx, xlo, xhi);
            range(qy, ylo, yhi);
            for (int64_t nx = xlo; nx < xhi; ++nx) {
                for (int64_t ny = ylo; ny < yhi; ++ny) {
                    const int64_t sr = (qx + 2 * nx) * (qx + 2 * nx) + (qy + 2 * ny) * (qy + 2 * ny);
                    const int64_t ss = (qx - 2 * nx) * (qx - 2 * nx) + (qy - 2 * ny) * (qy - 2 * ny);
                    const bool keep = (double(sr) * hh <= kmax2[f]) && (double(ss) * hh <= kmax2[f]);
                    if (!keep) continue;
                    ++kept;
                    if (!disk_inside) {
                        const int64_t mk = std::max(sr, ss);
                        if (mk >= int64_t(key_used.size())) key_used.resize(size_t(mk + 1) * 2, 0);
                        key_used[size_t(sr)] = 1;
                        key_used[size_t(ss)] = 1;
                    }
                    if (!mine) continue;
                    const int64_t nflat = (nx - nlo) * Nh + (ny - nlo);
                    p->rows.push_back(uint32_t(f));
                    p->rows.push_back(0);
                    key_r.push_back(sr);
                    key_s.push_back(ss);
                    p->keys.push_back(int32_t(nflat));
                    p->keys.push_back(0);
                }
            }
        }
        if (mine) p->row_off.push_back(int64_t(key_r.size()));
        if (counts) counts->push_back(kept);
    }
    n_all = gp;
}

// 3D survey of parallel lines: pair (ux, c) with flattened k = ux N_y + c
// (k <= its partner's); rows (f, a) with b = ux - a, kept iff a term q of the
// line-wavenumber sum is: |(a dkx, q dky)| and |(b dkx, p dky)|, p = q - c
// (signed, wrapped), both within the cut, compared as squared lengths written
// (n dk)*(n dk) + (m dk')*(m dk').  Classes (|a|, |q|) -> |a| (N_y/2 + 1) + |q|.
void rows_lines(edt_plan* p, const std::vector<double>& kmax, int64_t pb, int64_t pe,
                std::vector<int64_t>& cls_r, std::vector<int64_t>& cls_s, int64_t& n_all,
                std::vector<int64_t>* counts = nullptr) {
    const int64_t Nx = p->n_mid, Ny = p->n_line, ny2 = Ny / 2 + 1;
    const double dkx = kTwoPi / (double(Nx) * p->d_mid);
    const double dky = kTwoPi / (double(Ny) * p->d_line);
    p->n_km = Nx * Ny;
    p->row_off.push_back(0);
    int64_t gp = 0;
    for (int64_t k = 0; k < Nx * Ny; ++k) {
        const int64_t ux = k / Ny, c = k % Ny;
        const int64_t kn = wrap(-ux, Nx) * Ny + wrap(-c, Ny);
        if (kn < k) continue;
        const bool mine = gp >= pb && gp < pe;
        ++gp;
        if (!mine && !counts) continue;
        if (mine) {
            p->pair_u.push_back(int32_t(k));
            p->pair_u.push_back(int32_t(kn));
        }
        const int64_t qc = signed_of(c, Ny);
        int64_t kept = 0;
        for (int f = 0; f < p->n_freq; ++f) {
            const double K2 = kmax[size_t(f)] * kmax[size_t(f)];
            for (int64_t a = -(Nx / 2); a < Nx - Nx / 2; ++a) {
                const int64_t b = signed_of(wrap(ux - a, Nx), Nx);
                uint64_t m = 0;
                for (int64_t q = -(Ny / 2); q < Ny - Ny / 2; ++q) {
                    const int64_t pq = signed_of(wrap(q - qc, Ny), Ny);
                    const double kr2 = (double(a) * dkx) * (double(a) * dkx) + (double(q) * dky) * (double(q) * dky);
                    const double ks2 = (double(b) * dkx) * (double(b) * dkx) + (double(pq) * dky) * (double(pq) * dky);
                    if (kr2 <= K2 && ks2 <= K2) m |= uint64_t(1) << uint64_t(q + Ny / 2);
                }
                if (!m) continue;
                ++kept;
                if (!mine) continue;
                p->rows.push_back(uint32_t(f));
                p->rows.push_back(0);
                cls_r.push_back(std::llabs(a) * ny2);
                cls_s.push_back(std::llabs(b) * ny2);
                p->keys.push_back(int32_t(wrap(a, Nx)));
                p->keys.push_back(int32_t(wrap(b, Nx)));
                p->lmask.push_back(m);
            }
        }
        if (mine) p->row_off.push_back(int64_t(cls_r.size()));
        if (counts) counts->push_back(kept);
    }
    n_all = gp;
}

}  // namespace

namespace edt {

void set_error(const std::string& msg) { g_err = msg; }

int64_t line_chunk(const edt_plan* p) {
    if (!p->n_line || p->n_pairs == 0) return 0;
    // rows of one frequency for at most 256 MiB of pairs at a time
    const int64_t per = int64_t(p->n_mid) * p->nz * 16;
    return std::max<int64_t>(1, std::min<int64_t>(p->n_pairs, (int64_t(256) << 20) / per));
}

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
    w.ubw = off;
    off = align256(off + size_t(p->n_urows) * 2 * 16);
    w.ub32 = off;
    off = align256(off + size_t(p->n_urows) * 16);
    w.gmax = off;
    off = align256(off + size_t(p->n_freq) * size_t(p->n_cls) * sizeof(float));
    w.gram_part = off;
    off = align256(off + size_t(p->items.size()) * gram_part_bytes_per_item(p));
    w.rhs_part = off;
    off = align256(off + p->ritems.size() * (2 * nz + 1) * sizeof(double));
    w.gram_rpart = off;
    off = align256(off + p->items.size() * size_t(rpart_width(p->nz)) * sizeof(double));
    w.lam = off;
    off = align256(off + P * sizeof(double));
    w.dinv = off;
    off = align256(off + P * size_t((p->nz + 31) / 32) * 32 * 32 * sizeof(double));
    w.conv = off;
    off = align256(off + P * sizeof(int32_t));
    w.pcg_r = off;
    off = align256(off + P * 2 * nz * sizeof(double));
    w.pcg_p = off;
    off = align256(off + P * 2 * nz * sizeof(double));
    w.pcg_rho = off;
    off = align256(off + P * sizeof(double));
    w.esc_rhs = off;
    off = align256(off + P * 2 * nz * sizeof(double));
    w.esc_trace = off;
    off = align256(off + P * sizeof(double));
    w.counters = off;
    off = align256(off + (edt::kMaxRefine + 2) * sizeof(int32_t));
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
    w.lrows = off;
    off = align256(off + size_t(line_chunk(p)) * size_t(p->n_mid) * nz * 16);
    w.total = off;
    return w;
}

size_t resident_bytes(const edt_plan* p) {
    const size_t P = size_t(p->n_pairs), nz = size_t(p->nz);
    const size_t datum = p->data_c64 ? 8 : 16;
    size_t b = p->lay.total + work_layout(p).total;
    b += size_t(p->n_rows) * 2 * datum;                  // d_rows
    b += P * (nz * nz + 2 * nz + 1 + 2 * nz) * 8;        // gram, rhs, trace, x
    b += P * 2 * 4;                                      // info, steps
    b += size_t(p->n_km) * nz * 16;                      // v_out
    b += size_t(p->n_freq) * size_t(p->n_cls) * nz * 24; // g64 and g32
    return b;
}

}  // namespace edt

namespace {

// Checks of a survey and its layers shared by the planner entry points.
edt_status validate(const edt_survey* s, const edt_layers* l) {
    if (s->dim != 2 && s->dim != 3) return fail(EDT_EINVAL, "dim must be 2 or 3");
    if (s->n_mid < 2 || !(s->d_mid > 0)) return fail(EDT_EINVAL, "n_mid >= 2 and d_mid > 0 required");
    if (s->n_freq < 1 || s->n_freq >= 65536 || !s->freq_hz) return fail(EDT_EINVAL, "1 <= n_freq < 65536");
    if (s->nz < 1 || s->nz > 1024) return fail(EDT_EINVAL, "1 <= nz <= 1024");
    if (!(s->dz > 0) || !(s->eps >= 0) || !(s->kappa > 0)) return fail(EDT_EINVAL, "dz > 0, eps >= 0, kappa > 0");
    if (s->n_line != 0) {
        if (s->dim != 3) return fail(EDT_EINVAL, "a survey of parallel lines has dim 3");
        if (s->n_line < 1 || s->n_line > 64 || !(s->d_line > 0))
            return fail(EDT_EINVAL, "line survey: 1 <= n_line <= 64 and d_line > 0");
        if (s->n_mid > 2048) return fail(EDT_EINVAL, "line survey: n_mid <= 2048");
    } else if (s->dim == 3) {
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

    return EDT_OK;
}

// Horizontal wavenumber limit per frequency (the evanescent cut).
std::vector<double> kmax_of(const edt_survey* s, double ctop) {
    std::vector<double> kmax(s->n_freq);
    for (int f = 0; f < s->n_freq; ++f) kmax[f] = s->kappa * (kTwoPi * s->freq_hz[f]) / ctop;
    return kmax;
}

}  // namespace

extern "C" {

const char* edt_last_error(void) { return g_err.c_str(); }

edt_status edt_survey_pair_rows(const edt_survey* s, const edt_layers* l, int64_t* n_pairs_all,
                                int64_t* rows_per_pair) {
    if (!s || !l || !n_pairs_all) return fail(EDT_EINVAL, "null argument");
    {
        const edt_status v = validate(s, l);
        if (v != EDT_OK) return v;
    }
    try {
        edt_plan q;
        q.dim = s->dim;
        q.n_mid = s->n_mid;
        q.n_off = s->dim == 3 ? s->n_off : 0;
        q.d_mid = s->d_mid;
        q.n_freq = s->n_freq;
        q.n_line = s->n_line;
        q.d_line = s->d_line;
        const std::vector<double> kmax = kmax_of(s, l->vel[0]);
        std::vector<int64_t> kr, ks, counts;
        std::vector<uint8_t> key_used;
        int64_t max_cls = -1, n_all = 0;
        if (s->dim == 2) rows_2d(&q, kmax, 0, 0, kr, ks, max_cls, n_all, &counts);
        else if (s->n_line) rows_lines(&q, kmax, 0, 0, kr, ks, n_all, &counts);
        else rows_3d(&q, kmax, 0, 0, kr, ks, key_used, n_all, &counts);
        *n_pairs_all = n_all;
        if (rows_per_pair) std::memcpy(rows_per_pair, counts.data(), counts.size() * sizeof(int64_t));
    } catch (const std::bad_alloc&) {
        return fail(EDT_ENOMEM, "out of host memory");
    }
    return EDT_OK;
}

edt_status edt_plan_create(const edt_survey* s, const edt_layers* l, const edt_plan_opts* opts,
                           edt_plan** out) {
    const int chunk_rows = opts ? opts->chunk_rows : 0;
    const int band_opt = opts ? opts->gram_band : 0;
    const int64_t pair_begin = opts ? opts->pair_begin : 0;
    const int64_t pair_end = opts && opts->pair_end > 0 ? opts->pair_end : INT64_MAX;
    const int data_type = opts ? opts->data_type : EDT_DATA_C128;
    const int rgroup_opt = opts ? opts->resid_group : 0;
    const size_t hbm_budget = opts ? opts->hbm_budget : 0;
    if (!s || !l || !out) return fail(EDT_EINVAL, "null argument");
    *out = nullptr;
    if (data_type != EDT_DATA_C128 && data_type != EDT_DATA_C64)
        return fail(EDT_EINVAL, "data_type must be EDT_DATA_C128 or EDT_DATA_C64");
    if (chunk_rows < 0 || chunk_rows > kMaxChunk) return fail(EDT_EINVAL, "0 <= chunk_rows <= 2048");
    if (band_opt < 0) return fail(EDT_EINVAL, "gram_band >= 0");
    if (rgroup_opt < 0) return fail(EDT_EINVAL, "resid_group >= 0");
    if (pair_begin < 0 || pair_begin > pair_end) return fail(EDT_EINVAL, "0 <= pair_begin <= pair_end");
    {
        const edt_status v = validate(s, l);
        if (v != EDT_OK) return v;
    }

    edt_plan* p = new (std::nothrow) edt_plan();
    if (!p) return fail(EDT_ENOMEM, "out of host memory");
    try {
        p->dim = s->dim;
        p->n_mid = s->n_mid;
        p->n_off = s->dim == 3 && !s->n_line ? s->n_off : 0;
        p->n_line = s->n_line;
        p->d_line = s->d_line;
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
        p->data_c64 = data_type == EDT_DATA_C64 ? 1 : 0;
        p->freq.assign(s->freq_hz, s->freq_hz + s->n_freq);
        if (l->n_layers > 1) p->zif.assign(l->zif, l->zif + l->n_layers - 1);
        const std::vector<double> kmax = kmax_of(s, p->ctop);

        std::vector<int64_t> kr, ks;
        std::vector<uint8_t> key_used;
        int64_t max_cls = -1, n_all = 0;
        if (p->dim == 2) rows_2d(p, kmax, pair_begin, pair_end, kr, ks, max_cls, n_all);
        else if (p->n_line) rows_lines(p, kmax, pair_begin, pair_end, kr, ks, n_all);
        else rows_3d(p, kmax, pair_begin, pair_end, kr, ks, key_used, n_all);
        if (pair_end != INT64_MAX && pair_end > n_all) {
            delete p;
            return fail(EDT_EINVAL, "pair_end beyond the survey's pairs (" + std::to_string(n_all) + ")");
        }
        p->n_pairs_all = n_all;
        p->pair_begin = std::min(pair_begin, n_all);
        p->n_pairs = int64_t(p->row_off.size()) - 1;
        p->n_rows = p->row_off.back();
        if (p->n_rows >= (int64_t(1) << 31)) { delete p; return fail(EDT_EINVAL, "more than 2^31 rows"); }

        // classes: 2D class = |q| (|k| = |q| dk); 3D class = rank of the integer key
        const double dk = kTwoPi / (double(p->n_mid) * p->d_mid);
        std::vector<int32_t> cls_of_key;
        if (p->dim == 2) {
            p->n_cls = int(max_cls + 1);
            for (int c = 0; c < p->n_cls; ++c) p->cls_k.push_back(std::fabs(double(c)) * dk);
        } else if (p->n_line) {
            // every (|a|, |q|) of the line grid: |k| = |(a dkx, q dky)|
            const double dky = kTwoPi / (double(p->n_line) * p->d_line);
            const int nx2 = p->n_mid / 2 + 1, ny2 = p->n_line / 2 + 1;
            p->n_cls = nx2 * ny2;
            for (int ia = 0; ia < nx2; ++ia)
                for (int iq = 0; iq < ny2; ++iq)
                    p->cls_k.push_back(std::sqrt((double(ia) * dk) * (double(ia) * dk) +
                                                 (double(iq) * dky) * (double(iq) * dky)));
        } else {
            // keys are small non-negative integers: rank them through a dense table
            cls_of_key.assign(key_used.size(), -1);
            int c = 0;
            for (size_t v = 0; v < key_used.size(); ++v)
                if (key_used[v]) {
                    cls_of_key[v] = c++;
                    p->cls_k.push_back(std::sqrt(double(v)) * (0.5 * dk));
                }
            p->n_cls = c;
        }
        if (p->n_cls == 0) { p->n_cls = 1; p->cls_k.push_back(0.0); }
        if (p->n_cls >= 65536) { delete p; return fail(EDT_EINVAL, "more than 65535 |k| classes"); }
        for (int64_t r = 0; r < p->n_rows; ++r) {
            uint32_t cr, cs;
            if (p->dim == 2 || p->n_line) { cr = uint32_t(kr[r]); cs = uint32_t(ks[r]); }
            else { cr = uint32_t(cls_of_key[size_t(kr[r])]); cs = uint32_t(cls_of_key[size_t(ks[r])]); }
            p->rows[2 * r + 1] = cr | (cs << 16);
        }

        // unique rows: within a pair, data rows with the same frequency and the
        // same unordered class pair have the same Born row A.  Rows of a pair
        // come frequency by frequency; each frequency's rows are grouped by
        // sorting their keys (ties keep row order), so a unique row lists its
        // data rows in increasing order and unique rows stay sorted by f.
        p->urow_off.push_back(0);
        p->umem_off.push_back(0);
        p->row_unique.assign(size_t(p->n_rows), -1);
        p->umem.reserve(size_t(p->n_rows));
        std::vector<std::pair<uint32_t, int32_t>> seg;
        std::vector<std::pair<uint32_t, uint32_t>> grp, walk;
        int64_t n_u = 0;
        for (int64_t q = 0; q < p->n_pairs; ++q) {
            int64_t r = p->row_off[q];
            while (r < p->row_off[q + 1]) {
                const uint32_t f = p->rows[2 * r];
                int64_t e = r;
                seg.clear();
                while (e < p->row_off[q + 1] && p->rows[2 * e] == f) {
                    const uint32_t a = p->rows[2 * e + 1] & 0xFFFFu, b = p->rows[2 * e + 1] >> 16;
                    seg.emplace_back(std::min(a, b) | (std::max(a, b) << 16), int32_t(e));
                    ++e;
                }
                std::sort(seg.begin(), seg.end());
                grp.clear();
                for (size_t i = 0; i < seg.size();) {
                    size_t j = i;
                    while (j < seg.size() && seg[j].first == seg[i].first) ++j;
                    if (j - i >= 65536) { delete p; return fail(EDT_EINVAL, "row multiplicity >= 65536"); }
                    grp.push_back({uint32_t(i), uint32_t(j)});
                    i = j;
                }
                chain_order(seg, grp, walk);
                for (const auto& w : walk) {
                    const auto [i, j] = grp[w.first];
                    p->urows.push_back(f | (uint32_t(j - i) << 16));
                    p->urows.push_back(w.second);
                    for (size_t k = i; k < j; ++k) {
                        p->umem.push_back(seg[k].second);
                        p->row_unique[size_t(seg[k].second)] = int32_t(n_u);
                    }
                    p->umem_off.push_back(int32_t(p->umem.size()));
                    ++n_u;
                }
                r = e;
            }
            p->urow_off.push_back(n_u);
        }
        p->n_urows = n_u;
        p->urow_pair.assign(size_t(p->n_urows), 0);
        for (int64_t q = 0; q < p->n_pairs; ++q)
            for (int64_t uidx = p->urow_off[q]; uidx < p->urow_off[q + 1]; ++uidx)
                p->urow_pair[size_t(uidx)] = int32_t(q);
        {
            // contributors of each table entry, in unique-row order (deterministic)
            const size_t ne = size_t(p->n_freq) * size_t(p->n_cls);
            std::vector<int32_t> cnt(ne + 1, 0);
            for (int64_t uidx = 0; uidx < p->n_urows; ++uidx) {
                const uint32_t f = p->urows[2 * uidx] & 0xFFFFu;
                const uint32_t a = p->urows[2 * uidx + 1] & 0xFFFFu, b = p->urows[2 * uidx + 1] >> 16;
                cnt[size_t(f) * p->n_cls + a + 1]++;
                cnt[size_t(f) * p->n_cls + b + 1]++;
            }
            for (size_t e = 0; e < ne; ++e) cnt[e + 1] += cnt[e];
            p->tab_off = cnt;
            p->tab_ent.assign(size_t(cnt[ne]) * 2, 0);
            std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
            for (int64_t uidx = 0; uidx < p->n_urows; ++uidx) {
                const uint32_t f = p->urows[2 * uidx] & 0xFFFFu;
                const uint32_t a = p->urows[2 * uidx + 1] & 0xFFFFu, b = p->urows[2 * uidx + 1] >> 16;
                int32_t k = fill[size_t(f) * p->n_cls + a]++;
                p->tab_ent[2 * size_t(k)] = int32_t(uidx);
                p->tab_ent[2 * size_t(k) + 1] = int32_t(b);
                k = fill[size_t(f) * p->n_cls + b]++;
                p->tab_ent[2 * size_t(k)] = int32_t(uidx);
                p->tab_ent[2 * size_t(k) + 1] = int32_t(a);
            }
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

        // per-unique-row records of the Gram kernels
        if (double(p->n_freq) * double(p->n_cls) * double(p->nz) >= 4294967296.0) {
            delete p;
            return fail(EDT_EINVAL, "Green's table too large for 32-bit offsets (n_freq * n_cls * nz >= 2^32)");
        }
        p->grow.resize(size_t(p->n_urows));
        p->gsc.resize(size_t(p->n_urows));
        for (int64_t u = 0; u < p->n_urows; ++u) {
            const uint32_t a = p->urows[2 * u], b = p->urows[2 * u + 1];
            const uint32_t f = a & 0xFFFFu, m = a >> 16;
            const uint64_t base = uint64_t(f) * uint64_t(p->n_cls);
            edt::GRow& g = p->grow[size_t(u)];
            g.off_r = uint32_t((base + (b & 0xFFFFu)) * uint64_t(p->nz));
            g.off_s = uint32_t((base + (b >> 16)) * uint64_t(p->nz));
            g.sw = std::sqrt(float(m));
            g.mt = float(m);
            const double wr = kTwoPi * p->freq[f];
            p->gsc[size_t(u)] = (wr * wr + p->eps * p->eps) * p->dz * std::sqrt(double(m));
        }

        // Gram work items: a pair's rows within a band of consecutive
        // frequencies (at most chunk_rows rows).  The band is sized so that
        // its FP32 Green's table slab (n_cls x nz entries per frequency) fits
        // an XCD's L2 with room for the next band; slots are pair-major.
        // Where one frequency's slab alone exceeds that (large 3D tables) the
        // band is widened until an average item holds kMinItemRows rows: an
        // item's partial Gram (nz^2 values) must stay small next to its rows.
        // (Items over all frequencies are fewer and the split Gram faster, but
        // an FP16x3 item then spans a wider range of row magnitudes under its
        // one scale, and some pairs need one more refinement sweep.)
        p->chunk_rows = chunk_rows > 0 ? chunk_rows : kDefaultChunk;
        const double per_pf = double(p->n_urows) / std::max(1.0, double(p->n_pairs - p->n_empty) * p->n_freq);
        const int64_t band_rows = int64_t(std::ceil(double(kMinItemRows) / std::max(per_pf, 1e-9)));
        const int64_t band_l2 = int64_t(kL2Slab / (double(p->n_cls) * double(p->nz) * 8.0));
        p->gram_band = band_opt > 0 ? std::min(band_opt, p->n_freq)
                                    : int(std::max<int64_t>(1, std::min<int64_t>(p->n_freq, std::max(band_l2, band_rows))));
        std::vector<int32_t> gband;
        split_items(p, p->gram_band, p->chunk_rows, p->items, p->pair_item, gband);
        p->sched = xcd_schedule(p->items, gband);

        // residual work items: a pair's rows within a group of at least
        // kFreqGroup frequencies (widened, where rows are sparse, until an
        // average item holds kMinResidRows rows; at most kResidRows rows),
        // scheduled the same way.  The residual sweep reads its table slab
        // from L2, and its partials are small (2 nz values), so its groups
        // stay narrow.
        const int64_t group_rows = int64_t(std::ceil(double(kMinResidRows) / std::max(per_pf, 1e-9)));
        p->resid_group = rgroup_opt > 0 ? std::min(rgroup_opt, p->n_freq)
                                         : int(std::max<int64_t>(kFreqGroup, std::min<int64_t>(p->n_freq, group_rows)));
        std::vector<int32_t> rgroup;
        split_items(p, p->resid_group, kResidRows, p->ritems, p->pair_ritem, rgroup);
        p->rsched = xcd_schedule(p->ritems, rgroup);

        // line survey: first row of each frequency of each pair
        if (p->n_line) {
            p->lpair.assign(size_t(p->n_rows), 0);
            for (int64_t q = 0; q < p->n_pairs; ++q)
                for (int64_t r = p->row_off[size_t(q)]; r < p->row_off[size_t(q) + 1]; ++r) p->lpair[size_t(r)] = int32_t(q);
            p->lfr.assign(size_t(p->n_pairs) * size_t(p->n_freq + 1), 0);
            for (int64_t q = 0; q < p->n_pairs; ++q) {
                int64_t r = p->row_off[size_t(q)];
                for (int f = 0; f <= p->n_freq; ++f) {
                    while (r < p->row_off[size_t(q) + 1] && int(p->rows[2 * r]) < f) ++r;
                    p->lfr[size_t(q) * size_t(p->n_freq + 1) + size_t(f)] = r;
                }
            }
        }

        // device image
        edt::DevLayout& L = p->lay;
        size_t off = 0;
        L.freq = off;      off = align256(off + p->freq.size() * 8);
        L.zif = off;       off = align256(off + std::max<size_t>(1, p->zif.size()) * 8);
        L.cls_k = off;     off = align256(off + p->cls_k.size() * 8);
        L.row_off = off;   off = align256(off + p->row_off.size() * 8);
        L.pair_u = off;    off = align256(off + p->pair_u.size() * 4);
        L.rows = off;      off = align256(off + std::max<size_t>(1, p->rows.size()) * 4);
        L.keys = off;      off = align256(off + std::max<size_t>(1, p->keys.size()) * 4);
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
        L.ritems = off;    off = align256(off + std::max<size_t>(1, p->ritems.size()) * sizeof(edt::Item));
        L.rsched = off;    off = align256(off + std::max<size_t>(1, p->rsched.size()) * 4);
        L.pair_ritem = off; off = align256(off + p->pair_ritem.size() * 4);
        L.grow = off;      off = align256(off + std::max<size_t>(1, p->grow.size()) * sizeof(edt::GRow));
        L.gsc = off;       off = align256(off + std::max<size_t>(1, p->gsc.size()) * 8);
        L.lmask = off;     off = align256(off + std::max<size_t>(1, p->lmask.size()) * 8);
        L.lfr = off;       off = align256(off + std::max<size_t>(1, p->lfr.size()) * 8);
        L.lpair = off;     off = align256(off + std::max<size_t>(1, p->lpair.size()) * 4);
        L.total = off;
        p->host_image.assign(L.total, 0);
        auto put = [&](size_t o, const void* src, size_t n) { if (n) std::memcpy(p->host_image.data() + o, src, n); };
        put(L.freq, p->freq.data(), p->freq.size() * 8);
        put(L.zif, p->zif.data(), p->zif.size() * 8);
        put(L.cls_k, p->cls_k.data(), p->cls_k.size() * 8);
        put(L.row_off, p->row_off.data(), p->row_off.size() * 8);
        put(L.pair_u, p->pair_u.data(), p->pair_u.size() * 4);
        put(L.rows, p->rows.data(), p->rows.size() * 4);
        put(L.keys, p->keys.data(), p->keys.size() * 4);
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
        put(L.ritems, p->ritems.data(), p->ritems.size() * sizeof(edt::Item));
        put(L.rsched, p->rsched.data(), p->rsched.size() * 4);
        put(L.pair_ritem, p->pair_ritem.data(), p->pair_ritem.size() * 4);
        put(L.grow, p->grow.data(), p->grow.size() * sizeof(edt::GRow));
        put(L.gsc, p->gsc.data(), p->gsc.size() * 8);
        put(L.lmask, p->lmask.data(), p->lmask.size() * 8);
        put(L.lfr, p->lfr.data(), p->lfr.size() * 8);
        put(L.lpair, p->lpair.data(), p->lpair.size() * 4);
        if (hbm_budget > 0) {
            const size_t need = edt::resident_bytes(p);
            if (need > hbm_budget) {
                const int64_t pb = p->pair_begin, pe = p->pair_begin + p->n_pairs;
                delete p;
                return fail(EDT_ENOMEM, "pairs [" + std::to_string(pb) + ", " + std::to_string(pe) + ") need " +
                                            std::to_string(need) + " device bytes, more than the budget of " +
                                            std::to_string(hbm_budget));
            }
        }
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
    o->gram_band = p->gram_band;
    o->table_elems = size_t(p->n_freq) * size_t(p->n_cls) * size_t(p->nz);
    o->dev_plan_bytes = p->lay.total;
    o->work_bytes = edt::work_layout(p).total;
    o->gram_flops = p->gram_flops;
    o->n_pairs_all = p->n_pairs_all;
    o->resid_group = p->resid_group;
    o->pair_begin = p->pair_begin;
    o->data_type = p->data_c64 ? EDT_DATA_C64 : EDT_DATA_C128;
    o->resident_bytes = edt::resident_bytes(p);
    return EDT_OK;
}

edt_status edt_plan_urows(const edt_plan* p, int64_t* urow_off, int32_t* urows, int32_t* row_unique) {
    if (!p) return fail(EDT_EINVAL, "null plan");
    if (urow_off) std::memcpy(urow_off, p->urow_off.data(), p->urow_off.size() * 8);
    if (urows)
        for (int64_t u = 0; u < p->n_urows; ++u) {
            const uint32_t a = p->urows[2 * u], b = p->urows[2 * u + 1];
            urows[4 * u] = int32_t(a & 0xFFFFu);
            urows[4 * u + 1] = int32_t(a >> 16);
            urows[4 * u + 2] = int32_t(b & 0xFFFFu);
            urows[4 * u + 3] = int32_t(b >> 16);
        }
    if (row_unique && !p->row_unique.empty()) std::memcpy(row_unique, p->row_unique.data(), p->row_unique.size() * 4);
    return EDT_OK;
}

edt_status edt_plan_schedule(const edt_plan* p, int which, int64_t* counts, int32_t* items,
                             int32_t* sched) {
    if (!p || !counts) return fail(EDT_EINVAL, "null argument");
    if (which != 0 && which != 1) return fail(EDT_EINVAL, "which must be 0 (Gram) or 1 (residual)");
    const std::vector<edt::Item>& it = which == 0 ? p->items : p->ritems;
    const std::vector<int32_t>& sc = which == 0 ? p->sched : p->rsched;
    counts[0] = int64_t(it.size());
    counts[1] = int64_t(sc.size());
    if (items)
        for (size_t i = 0; i < it.size(); ++i) {
            items[3 * i] = it[i].pair;
            items[3 * i + 1] = it[i].row_begin;
            items[3 * i + 2] = it[i].row_end;
        }
    if (sched && !sc.empty()) std::memcpy(sched, sc.data(), sc.size() * 4);
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
