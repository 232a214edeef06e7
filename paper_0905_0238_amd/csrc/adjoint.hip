// Kernel (d): reverse-mode gradient of a real loss on V~ with respect to the
// data, the relative damping and the layer velocities of the reference.
//
// Forward map (paper Section 2.1, eqs. M, VSym, Split; Tikhonov damping of
// Section 4): per pair, x+- = H^{-1} Re(A^H b+-), H = Re(A^H A) + lambda I,
// lambda = lambda_rel tr(Re A^H A)/nz, V~(+-u) = x+ +- i x-, with Born rows
// A = W g(k_r) g(k_s), W = w^2 dz, and g the layered Green's function.
//
// Complex gradients follow the convention gbar = dL/dRe + i dL/dIm; for a
// holomorphic u = h(v) the chain rule is vbar += conj(h'(v)) ubar.
//
//   1. per pair:  gx+ = Re gV(u) + Re gV(-u), gx- = Im gV(u) - Im gV(-u);
//                 y = H^{-1} gx (the stored Cholesky factor); dL/dlambda =
//                 -y.x; dL/dlambda_rel += dL/dlambda tr/nz.
//   2. per row:   A y+- (= dL/db+-, scattered to the data rows through
//                 b+ = (d0+d1)/2, b- = (d0-d1)/(2i)) and e+- = B+- - m A x+-.
//   3. per table entry (f, |k|): gbar(z) = sum over the rows using it of
//                 conj(W g_other) Abar,  Abar = sum e y^T - m (A y) x^T
//                 + m dL/dlambda (2 lambda_rel/nz) A, followed in the same
//                 wavefront by the reverse sweep of the layer recursion (the
//                 forward state is recomputed, not stored) down to
//                 dL/dc_l = Re(conj(kbar_l) dk_l/dc_l), dk_l/dc_l = -w^2/(c_l^3 k_l).
//   4. fixed-order sums over pairs / table entries (deterministic).

#include "dev_linalg.h"

namespace edt {

size_t adjoint_lds_bytes(int nz);
hipError_t launch_bsum(const edt_plan* p, const void* d_rows, zd* ub, hipStream_t st, zd* ubw = nullptr,
                       float4* ub32 = nullptr);

// ------------------------------------------------------------ 1. pairs ---
__global__ __launch_bounds__(256) void adj_pair_kernel(const double* __restrict__ chol,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ trace,
                                                       const int64_t* __restrict__ urow_off,
                                                       const int32_t* __restrict__ pair_u, int nz,
                                                       const zd* __restrict__ gv,
                                                       double* __restrict__ y,
                                                       double* __restrict__ dl,
                                                       double* __restrict__ glam_part) {
    extern __shared__ double smem[];
    double* sx = smem;
    double* sL = sx + 2 * nz;
    double* sred = sL + size_t(nz) * CBP;
    __shared__ double s_red[8];
    const int p = blockIdx.x, tid = threadIdx.x;
    const int u0 = pair_u[2 * p], u1 = pair_u[2 * p + 1];
    const bool selfc = u0 == u1;
    double* yp = y + size_t(p) * 2 * nz;
    if (urow_off[p + 1] == urow_off[p]) {
        for (int e = tid; e < 2 * nz; e += blockDim.x) yp[e] = 0.0;
        if (tid == 0) {
            dl[p] = 0.0;
            glam_part[p] = 0.0;
        }
        return;
    }
    for (int z = tid; z < nz; z += blockDim.x) {
        const zd a = gv[size_t(u0) * nz + z];
        if (selfc) {
            sx[z] = a.x;
            sx[nz + z] = 0.0;
        } else {
            const zd b = gv[size_t(u1) * nz + z];
            sx[z] = a.x + b.x;
            sx[nz + z] = a.y - b.y;
        }
    }
    __syncthreads();
    trisolve2(chol + size_t(p) * nz * nz, nz, sx, sL, sred);
    double s = 0.0;
    for (int e = tid; e < 2 * nz; e += blockDim.x) {
        const double v = (selfc && e >= nz) ? 0.0 : sx[e];
        yp[e] = v;
        s += v * x[size_t(p) * 2 * nz + e];
    }
    s = wave_sum(s);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) s_red[wv] = s;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) t += s_red[w];
        dl[p] = -t;
        glam_part[p] = -t * trace[p] / double(nz);
    }
}

// ------------------------------------------------------------- 2. rows ---
// One wave per unique row: A x+-, A y+- (sums over depth), e+- and the data
// gradient of every data row the unique row stands for (in the plan's data
// type).
template <class D>
__global__ __launch_bounds__(256) void adj_rows_kernel(
    const uint32_t* __restrict__ urows, const int32_t* __restrict__ urow_pair,
    const int32_t* __restrict__ umem_off, const int32_t* __restrict__ umem, const zd* __restrict__ g64,
    const double* __restrict__ freq, double eps, double dz, int ncls, int nz, int64_t U,
    const zd* __restrict__ ub, const double* __restrict__ x, const double* __restrict__ y,
    zd* __restrict__ rowsc, D* __restrict__ grad_d) {
    const int lane = threadIdx.x & 63;
    const int64_t r = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (r >= U) return;
    const URow u = load_urow(urows, r);
    const int p = urow_pair[r];
    const int64_t fb = int64_t(u.f) * ncls;
    const double* xp = x + size_t(p) * 2 * nz;
    const double* yp = y + size_t(p) * 2 * nz;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int z = lane; z < nz; z += 64) {
        const zd P = g64[(fb + u.cr) * nz + z] * g64[(fb + u.cs) * nz + z];
        v[0] += P.x * xp[z];
        v[1] += P.y * xp[z];
        v[2] += P.x * xp[nz + z];
        v[3] += P.y * xp[nz + z];
        v[4] += P.x * yp[z];
        v[5] += P.y * yp[z];
        v[6] += P.x * yp[nz + z];
        v[7] += P.y * yp[nz + z];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = wave_sum(v[k]);
    const zd w = omega_of(freq[u.f], eps);
    const zd W = dz * (w * w);
    const double m = double(u.mult);
    const zd axp = W * zd{v[0], v[1]}, axm = W * zd{v[2], v[3]};
    const zd ayp = W * zd{v[4], v[5]}, aym = W * zd{v[6], v[7]};
    const zd ep = ub[2 * r] - m * axp, em = ub[2 * r + 1] - m * axm;
    if (lane == 0) {
        rowsc[4 * r] = ep;
        rowsc[4 * r + 1] = em;
        rowsc[4 * r + 2] = ayp;
        rowsc[4 * r + 3] = aym;
    }
    if (grad_d) {
        // d0: b+ += d0/2, b- += d0/(2i)  ->  gd0 = gb+/2 + (i/2) gb-
        const zd ih = zd{-0.5 * aym.y, 0.5 * aym.x};   // (i/2) A y-
        const zd gd0 = 0.5 * ayp + ih, gd1 = 0.5 * ayp - ih;
        for (int k = umem_off[r] + lane; k < umem_off[r + 1]; k += 64) {
            const int64_t dr = umem[k];
            store_datum(grad_d, 2 * dr, gd0);
            store_datum(grad_d, 2 * dr + 1, gd1);
        }
    }
}

// ---------------------------------------------- 3. table + reverse scan ---
template <int ZPL>
__global__ __launch_bounds__(256) void adj_table_kernel(
    const double* __restrict__ freq, const double* __restrict__ zif, const double* __restrict__ cls_k,
    const double* __restrict__ vel, int nf, int ncls, int nz, int L, double eps, double z0, double dz,
    double lambda_rel, const uint32_t* __restrict__ urows, const int32_t* __restrict__ urow_pair,
    const int32_t* __restrict__ tab_off, const int32_t* __restrict__ tab_ent,
    const zd* __restrict__ g64, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ dl, const zd* __restrict__ rowsc, zd* __restrict__ gbar,
    const zd* __restrict__ gbar_in, double* __restrict__ vel_part) {
    __shared__ zd s_k[4][kMaxLayers], s_R[4][kMaxLayers], s_rho[4][kMaxLayers], s_b[4][kMaxLayers];
    __shared__ zd s_c[4][4][ZPL * 64];   // per-depth adjoint contributions: k, R, b, H
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t wid = int64_t(blockIdx.x) * 4 + wv;
    const bool active = wid < int64_t(nf) * ncls;
    const int f = active ? int(wid / ncls) : 0;
    const int c = active ? int(wid % ncls) : 0;
    const zd w = omega_of(freq[f], eps);
    const zd w2 = w * w;
    const zd W = dz * w2;
    const double kk = cls_k[c];

    // gbar of this entry, lanes over depth
    zd gb[ZPL];
#pragma unroll
    for (int q = 0; q < ZPL; ++q) gb[q] = zd{0.0, 0.0};
    if (active && gbar_in) {
        // gathered beforehand (the survey of parallel lines)
        const int64_t e = int64_t(f) * ncls + c;
#pragma unroll
        for (int q = 0; q < ZPL; ++q) {
            const int z = lane + 64 * q;
            if (z < nz) gb[q] = gbar_in[e * nz + z];
        }
    } else if (active) {
        const int64_t e = int64_t(f) * ncls + c;
        const zd* gself = g64 + e * nz;
        zd gs[ZPL];
#pragma unroll
        for (int q = 0; q < ZPL; ++q) {
            const int z = lane + 64 * q;
            gs[q] = z < nz ? gself[z] : zd{0.0, 0.0};
        }
        for (int k = tab_off[e]; k < tab_off[e + 1]; ++k) {
            const int64_t r = tab_ent[2 * k];
            const int oc = tab_ent[2 * k + 1];
            const int p = urow_pair[r];
            const double m = double(urows[2 * r] >> 16);
            const zd ep = rowsc[4 * r], em = rowsc[4 * r + 1];
            const zd ayp = rowsc[4 * r + 2], aym = rowsc[4 * r + 3];
            const double kap = m * dl[p] * 2.0 * lambda_rel / double(nz);
            const zd* go = g64 + (int64_t(f) * ncls + oc) * nz;
            const double* xp = x + size_t(p) * 2 * nz;
            const double* yp = y + size_t(p) * 2 * nz;
#pragma unroll
            for (int q = 0; q < ZPL; ++q) {
                const int z = lane + 64 * q;
                if (z < nz) {
                    const zd o = go[z];
                    const zd A = W * (gs[q] * o);
                    const double xpz = xp[z], xmz = xp[nz + z], ypz = yp[z], ymz = yp[nz + z];
                    zd Ab = ypz * ep + ymz * em;
                    Ab = Ab - (m * xpz) * ayp - (m * xmz) * aym;
                    Ab = Ab + kap * A;
                    gb[q] = gb[q] + zconj(W * o) * Ab;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < ZPL; ++q) {
            const int z = lane + 64 * q;
            if (z < nz && gbar) gbar[e * nz + z] = gb[q];
        }
    }

    // forward layer state (as in the table kernel)
    if (lane < L) {
        const double cl = vel[lane];
        s_k[wv][lane] = zsqrt(zd{w2.x / (cl * cl) - kk * kk, w2.y / (cl * cl)});
        s_R[wv][lane] = zd{0.0, 0.0};
        s_rho[wv][lane] = zd{0.0, 0.0};
        s_b[wv][lane] = zd{0.0, 0.0};
    }
    __syncthreads();
    if (lane == 0 && L > 1) {
        zd rho_next = zd{0.0, 0.0};
        for (int j = L - 2; j >= 0; --j) {
            const zd kj = s_k[wv][j], kn = s_k[wv][j + 1];
            const zd r = zdiv(kj - kn, kj + kn);
            zd R = r;
            if (j < L - 2) R = zdiv(r + rho_next, zd{1.0, 0.0} + r * rho_next);
            s_R[wv][j] = R;
            if (j >= 1) {
                rho_next = R * zexpi(2.0 * kj, zif[j] - zif[j - 1]);
                s_rho[wv][j] = rho_next;
            }
        }
        const zd k0 = s_k[wv][0];
        const zd H = zdiv(zd{0.0, 1.0}, 2.0 * k0);
        zd b = H * zexpi(k0, zif[0]) * zdiv(zd{1.0, 0.0} + s_R[wv][0], zd{1.0, 0.0} + s_rho[wv][1]);
        s_b[wv][1] = b;
        for (int j = 1; j < L - 1; ++j) {
            b = b * zexpi(s_k[wv][j], zif[j] - zif[j - 1]) *
                zdiv(zd{1.0, 0.0} + s_R[wv][j], zd{1.0, 0.0} + s_rho[wv][j + 1]);
            s_b[wv][j + 1] = b;
        }
    }
    __syncthreads();

    // per-depth contributions to the adjoints of k_j, R_j, b_j and H = i/(2 k0)
    const zd I1 = zd{0.0, 1.0};
#pragma unroll
    for (int q = 0; q < ZPL; ++q) {
        const int z_i = lane + 64 * q;
        zd ck{0, 0}, cR{0, 0}, cb{0, 0}, cH{0, 0};
        if (active && z_i < nz) {
            const double z = z0 + double(z_i) * dz;
            int lo = 0, hi = L - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (zif[mid] <= z) lo = mid + 1;
                else hi = mid;
            }
            const int j = lo;
            const zd kj = s_k[wv][j];
            const zd g_ = gb[q];
            if (j == 0) {
                const zd H = zdiv(I1, 2.0 * kj);
                const double d1 = fabs(z);
                const zd E1 = zexpi(kj, d1);
                zd S = E1;
                zd E2{0, 0};
                double d2 = 0.0;
                if (L > 1) {
                    d2 = 2.0 * zif[0] - z;
                    E2 = zexpi(kj, d2);
                    S = S + s_R[wv][0] * E2;
                }
                cH = zconj(S) * g_;
                const zd Sb = zconj(H) * g_;
                ck = zconj(d1 * (I1 * E1)) * Sb;
                if (L > 1) {
                    cR = zconj(E2) * Sb;
                    ck = ck + zconj(d2 * (I1 * E2)) * (zconj(s_R[wv][0]) * Sb);
                }
            } else if (j == L - 1) {
                const double d = z - zif[j - 1];
                const zd D = zexpi(kj, d);
                cb = zconj(D) * g_;
                ck = zconj(d * (I1 * D)) * (zconj(s_b[wv][j]) * g_);
            } else {
                const double d1 = z - zif[j - 1], d2 = 2.0 * zif[j] - zif[j - 1] - z;
                const zd D1 = zexpi(kj, d1), D2 = zexpi(kj, d2);
                const zd R = s_R[wv][j];
                const zd S = D1 + R * D2;
                cb = zconj(S) * g_;
                const zd Sb = zconj(s_b[wv][j]) * g_;
                cR = zconj(D2) * Sb;
                ck = zconj(d1 * (I1 * D1)) * Sb + zconj(d2 * (I1 * D2)) * (zconj(R) * Sb);
            }
        }
        s_c[wv][0][z_i] = ck;
        s_c[wv][1][z_i] = cR;
        s_c[wv][2][z_i] = cb;
        s_c[wv][3][z_i] = cH;
    }
    __syncthreads();
    if (!active || lane != 0) return;

    // serial part: per-layer sums in depth order, then the reverse recursions
    zd kb[kMaxLayers], Rb[kMaxLayers], bb[kMaxLayers], rhob[kMaxLayers];
    for (int j = 0; j < L; ++j) kb[j] = Rb[j] = bb[j] = rhob[j] = zd{0.0, 0.0};
    zd Hb{0.0, 0.0};
    {
        int j = 0;
        for (int zi = 0; zi < nz; ++zi) {
            const double z = z0 + double(zi) * dz;
            while (j < L - 1 && zif[j] <= z) ++j;
            kb[j] = kb[j] + s_c[wv][0][zi];
            Rb[j] = Rb[j] + s_c[wv][1][zi];
            bb[j] = bb[j] + s_c[wv][2][zi];
            Hb = Hb + s_c[wv][3][zi];
        }
    }
    const zd one{1.0, 0.0};
    if (L > 1) {
        // reverse of b_{j+1} = b_j E_j (1 + R_j)/(1 + rho_{j+1}), j = L-2 .. 1
        for (int j = L - 2; j >= 1; --j) {
            const double h = zif[j] - zif[j - 1];
            const zd E = zexpi(s_k[wv][j], h);
            const zd den = one + s_rho[wv][j + 1];
            const zd Q = zdiv(one + s_R[wv][j], den);
            const zd bn = bb[j + 1];
            bb[j] = bb[j] + zconj(E * Q) * bn;
            const zd Eb = zconj(s_b[wv][j] * Q) * bn;
            kb[j] = kb[j] + zconj(h * (I1 * E)) * Eb;
            const zd Qb = zconj(s_b[wv][j] * E) * bn;
            Rb[j] = Rb[j] + zconj(zdiv(one, den)) * Qb;
            if (j + 1 <= L - 2) rhob[j + 1] = rhob[j + 1] + zconj(zdiv(zd{0, 0} - (one + s_R[wv][j]), den * den)) * Qb;
        }
        // reverse of b_1 = H E_0 (1 + R_0)/(1 + rho_1)
        {
            const zd k0 = s_k[wv][0];
            const zd H = zdiv(I1, 2.0 * k0);
            const zd E0 = zexpi(k0, zif[0]);
            const zd den = one + s_rho[wv][1];
            const zd Q0 = zdiv(one + s_R[wv][0], den);
            const zd bn = bb[1];
            Hb = Hb + zconj(E0 * Q0) * bn;
            kb[0] = kb[0] + zconj(zif[0] * (I1 * E0)) * (zconj(H * Q0) * bn);
            const zd Qb = zconj(H * E0) * bn;
            Rb[0] = Rb[0] + zconj(zdiv(one, den)) * Qb;
            if (1 <= L - 2) rhob[1] = rhob[1] + zconj(zdiv(zd{0, 0} - (one + s_R[wv][0]), den * den)) * Qb;
        }
    }
    // H = i/(2 k0): dH/dk0 = -i/(2 k0^2)
    {
        const zd k0 = s_k[wv][0];
        kb[0] = kb[0] + zconj(zdiv(zd{0.0, -1.0}, 2.0 * (k0 * k0))) * Hb;
    }
    if (L > 1) {
        // reverse of the bottom-up recursion, top-down
        for (int j = 0; j <= L - 2; ++j) {
            if (j >= 1) {
                // rho_j = R_j exp(2 i k_j h_j)
                const double h = zif[j] - zif[j - 1];
                const zd E2 = zexpi(2.0 * s_k[wv][j], h);
                Rb[j] = Rb[j] + zconj(E2) * rhob[j];
                kb[j] = kb[j] + zconj((2.0 * h) * (I1 * s_rho[wv][j])) * rhob[j];
            }
            const zd kj = s_k[wv][j], kn = s_k[wv][j + 1];
            const zd sum = kj + kn;
            const zd r = zdiv(kj - kn, sum);
            zd rb = Rb[j];
            if (j < L - 2) {
                const zd rho = s_rho[wv][j + 1];
                const zd D = one + r * rho;
                const zd D2 = D * D;
                rb = zconj(zdiv(one - rho * rho, D2)) * Rb[j];
                rhob[j + 1] = rhob[j + 1] + zconj(zdiv(one - r * r, D2)) * Rb[j];
            }
            const zd s2 = sum * sum;
            kb[j] = kb[j] + zconj(zdiv(2.0 * kn, s2)) * rb;
            kb[j + 1] = kb[j + 1] + zconj(zdiv(zd{0, 0} - 2.0 * kj, s2)) * rb;
        }
    }
    double* out = vel_part + wid * L;
    for (int l = 0; l < L; ++l) {
        const double cl = vel[l];
        const zd dk = zdiv(zd{0, 0} - w2, (cl * cl * cl) * s_k[wv][l]);   // dk_l/dc_l
        const zd t = zconj(kb[l]) * dk;
        out[l] = t.x;
    }
}

hipError_t configure_adjoint_kernels(int bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(adj_pair_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// ------------------------------------------------------------ 4. sums ---
// out[k] = sum_i in[i * stride + k] for i < n, one block per k, fixed order.
__global__ __launch_bounds__(256) void ordered_sum_kernel(const double* __restrict__ in, int64_t n,
                                                          int stride, double* __restrict__ out) {
    __shared__ double s[256];
    const int k = blockIdx.x, tid = threadIdx.x;
    double a = 0.0;
    for (int64_t i = tid; i < n; i += 256) a += in[i * stride + k];
    s[tid] = a;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (tid < h) s[tid] += s[tid + h];
        __syncthreads();
    }
    if (tid == 0) out[k] = s[0];
}

// ------------------------------------------------------------- launcher ---
template <int ZPL>
static void launch_table(const edt_plan* p, const double* vel, const zd* g64, const double* x,
                         const double* y, const double* dl, const zd* rowsc, zd* gbar, const zd* gbar_in,
                         double* vpart, double lambda_rel, hipStream_t st) {
    const int64_t waves = int64_t(p->n_freq) * p->n_cls;
    hipLaunchKernelGGL(adj_table_kernel<ZPL>, dim3(unsigned((waves + 3) / 4)), dim3(256), 0, st,
                       dptr<const double>(p, p->lay.freq), dptr<const double>(p, p->lay.zif),
                       dptr<const double>(p, p->lay.cls_k), vel, p->n_freq, p->n_cls, p->nz, p->n_layers,
                       p->eps, p->z0, p->dz, lambda_rel, dptr<const uint32_t>(p, p->lay.urows),
                       dptr<const int32_t>(p, p->lay.urow_pair), dptr<const int32_t>(p, p->lay.tab_off),
                       dptr<const int32_t>(p, p->lay.tab_ent), g64, x, y, dl, rowsc, gbar, gbar_in, vpart);
}

// Table adjoint and the layer sums: grad_vel from the table gradient (gbar_in
// given) or from the rows' scalars (gathered per entry, gbar written).
static hipError_t launch_vel(const edt_plan* p, const double* vel, const zd* g64, const double* x,
                             const double* y, const double* dl, const zd* rowsc, zd* gbar, const zd* gbar_in,
                             double* vpart, double lambda_rel, double* grad_vel, hipStream_t st) {
    switch ((p->nz + 63) / 64) {
        case 1: launch_table<1>(p, vel, g64, x, y, dl, rowsc, gbar, gbar_in, vpart, lambda_rel, st); break;
        case 2: launch_table<2>(p, vel, g64, x, y, dl, rowsc, gbar, gbar_in, vpart, lambda_rel, st); break;
        case 3: launch_table<3>(p, vel, g64, x, y, dl, rowsc, gbar, gbar_in, vpart, lambda_rel, st); break;
        case 4: launch_table<4>(p, vel, g64, x, y, dl, rowsc, gbar, gbar_in, vpart, lambda_rel, st); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ordered_sum_kernel, dim3(unsigned(p->n_layers)), dim3(256), 0, st, vpart,
                       int64_t(p->n_freq) * p->n_cls, p->n_layers, grad_vel);
    return hipGetLastError();
}

hipError_t launch_adjoint(const edt_plan* p, const double* vel, const zd* g64, const void* d_rows,
                          const double* chol, const double* trace, const double* x, double lambda_rel,
                          const zd* grad_v, void* grad_d, double* grad_lambda, double* grad_vel,
                          unsigned char* work, hipStream_t st) {
    const WorkLayout wl = work_layout(p);
    zd* ub = reinterpret_cast<zd*>(work + wl.ub);
    double* y = reinterpret_cast<double*>(work + wl.adj_y);
    double* dl = reinterpret_cast<double*>(work + wl.adj_dl);
    zd* rowsc = reinterpret_cast<zd*>(work + wl.adj_row);
    double* vpart = reinterpret_cast<double*>(work + wl.adj_vel);
    double* glam_part = reinterpret_cast<double*>(work + wl.aux);
    zd* gbar = reinterpret_cast<zd*>(work + wl.gbar);
    hipError_t e;
    if (p->n_pairs == 0) return hipSuccess;
    if ((e = launch_bsum(p, d_rows, ub, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(adj_pair_kernel, dim3(unsigned(p->n_pairs)), dim3(256), adjoint_lds_bytes(p->nz), st,
                       chol, x, trace, dptr<const int64_t>(p, p->lay.urow_off),
                       dptr<const int32_t>(p, p->lay.pair_u), p->nz, grad_v, y, dl, glam_part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (p->n_urows) {
        const dim3 grid(unsigned((p->n_urows + 3) / 4));
        if (p->data_c64)
            hipLaunchKernelGGL(adj_rows_kernel<float2>, grid, dim3(256), 0, st,
                               dptr<const uint32_t>(p, p->lay.urows), dptr<const int32_t>(p, p->lay.urow_pair),
                               dptr<const int32_t>(p, p->lay.umem_off), dptr<const int32_t>(p, p->lay.umem), g64,
                               dptr<const double>(p, p->lay.freq), p->eps, p->dz, p->n_cls, p->nz, p->n_urows,
                               ub, x, y, rowsc, static_cast<float2*>(grad_d));
        else
            hipLaunchKernelGGL(adj_rows_kernel<zd>, grid, dim3(256), 0, st,
                               dptr<const uint32_t>(p, p->lay.urows), dptr<const int32_t>(p, p->lay.urow_pair),
                               dptr<const int32_t>(p, p->lay.umem_off), dptr<const int32_t>(p, p->lay.umem), g64,
                               dptr<const double>(p, p->lay.freq), p->eps, p->dz, p->n_cls, p->nz, p->n_urows,
                               ub, x, y, rowsc, static_cast<zd*>(grad_d));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (grad_vel &&
        (e = launch_vel(p, vel, g64, x, y, dl, rowsc, gbar, nullptr, vpart, lambda_rel, grad_vel, st)) !=
            hipSuccess)
        return e;
    if (grad_lambda) {
        hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(256), 0, st, glam_part, p->n_pairs, 1,
                           grad_lambda);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------- survey of parallel lines ---
// A line row is A = (w^2 dz / L_y) sum_q g(k_a, k_q) g(k_b, k_{q-c}) over its
// kept terms, formed per run of pairs and frequency into Rh (nr slots per
// pair).  One block per pair of the run, a wave per row: A x+-, A y+-, e+- =
// b+- - A x+-, the data gradient, and Abar = y+ e+ + y- e- - x+ A y+ - x- A y-
// + kappa A, which flows to both factors of every term of the row:
// gbar(k_a, k_q) += conj(W g(k_b, k_{q-c})) Abar and symmetrically (atomic
// adds: a table entry takes terms from rows of many pairs).
__device__ __forceinline__ int sidx(int n, int N) { return n < (N + 1) / 2 ? n : n - N; }

template <class D>
__global__ __launch_bounds__(256) void line_adj_kernel(
    const zd* __restrict__ Rh, const zd* __restrict__ g64, const int32_t* __restrict__ keys,
    const uint64_t* __restrict__ lmask, const int64_t* __restrict__ lfr, const int32_t* __restrict__ pair_u,
    const D* __restrict__ d_rows, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ dl, int f, int n_freq, int n_cls, int Nx, int Ny, int nz, int nr, zd W,
    double lambda_rel, int64_t p0, D* __restrict__ grad_d, zd* __restrict__ gbar) {
    const int64_t p = p0 + blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = lfr[p * (n_freq + 1) + f], n = lfr[p * (n_freq + 1) + f + 1] - r0;
    const zd* R = Rh + size_t(blockIdx.x) * nr * nz;
    const double* xp = x + size_t(p) * 2 * nz;
    const double* yp = y + size_t(p) * 2 * nz;
    const double kap = dl[p] * 2.0 * lambda_rel / double(nz);
    const int ny2 = Ny / 2 + 1, qc = sidx(pair_u[2 * p] % Ny, Ny);
    const zd* gf = g64 + size_t(f) * n_cls * nz;
    zd* gb = gbar ? gbar + size_t(f) * n_cls * nz : nullptr;
    for (int64_t i = wv; i < n; i += 4) {
        const int64_t r = r0 + i;
        const zd* A = R + size_t(i) * nz;
        double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int z = lane; z < nz; z += 64) {
            const zd a = A[z];
            v[0] += a.x * xp[z];
            v[1] += a.y * xp[z];
            v[2] += a.x * xp[nz + z];
            v[3] += a.y * xp[nz + z];
            v[4] += a.x * yp[z];
            v[5] += a.y * yp[z];
            v[6] += a.x * yp[nz + z];
            v[7] += a.y * yp[nz + z];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = wave_sum(v[k]);
        const zd axp{v[0], v[1]}, axm{v[2], v[3]}, ayp{v[4], v[5]}, aym{v[6], v[7]};
        const zd d0 = load_datum(d_rows, 2 * r), d1 = load_datum(d_rows, 2 * r + 1);
        const zd df = d0 - d1;
        const zd ep = 0.5 * (d0 + d1) - axp, em = zd{0.5 * df.y, -0.5 * df.x} - axm;
        if (grad_d && lane == 0) {
            const zd ih = zd{-0.5 * aym.y, 0.5 * aym.x};   // (i/2) A y-
            store_datum(grad_d, 2 * r, 0.5 * ayp + ih);
            store_datum(grad_d, 2 * r + 1, 0.5 * ayp - ih);
        }
        if (!gb) continue;
        const int ia = abs(sidx(keys[2 * r], Nx)), ib = abs(sidx(keys[2 * r + 1], Nx));
        const uint64_t mask = lmask[r];
        for (int z = lane; z < nz; z += 64) {
            zd Ab = yp[z] * ep + yp[nz + z] * em;
            Ab = Ab - xp[z] * ayp - xp[nz + z] * aym;
            Ab = Ab + kap * A[z];
            // the terms q and -q share the receiver-side entry (ia, |q|): their
            // contributions to it are summed before its atomic add
            const int h = Ny / 2;
            for (int k = 0; k <= h; ++k) {
                const bool kp = k + h < Ny && ((mask >> (k + h)) & 1u);   // q = +k
                const bool kn = k > 0 && ((mask >> (h - k)) & 1u);        // q = -k
                if (!kp && !kn) continue;
                const size_t ca = size_t(ia * ny2 + k) * nz + z;
                const zd tb = zconj(W * gf[ca]) * Ab;
                zd ta{0.0, 0.0};
                for (int sgn = 0; sgn < 2; ++sgn) {
                    if (!(sgn == 0 ? kp : kn)) continue;
                    const int q = sgn == 0 ? k : -k;
                    int pq = (q - qc) % Ny;
                    pq = sidx(pq < 0 ? pq + Ny : pq, Ny);
                    const size_t cb = size_t(ib * ny2 + abs(pq)) * nz + z;
                    ta = ta + zconj(W * gf[cb]) * Ab;
                    atomicAdd(&gb[cb].x, tb.x);
                    atomicAdd(&gb[cb].y, tb.y);
                }
                atomicAdd(&gb[ca].x, ta.x);
                atomicAdd(&gb[ca].y, ta.y);
            }
        }
    }
}

__global__ __launch_bounds__(256) void zero_kernel(double* __restrict__ a, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) a[i] = 0.0;
}

int line_row_slots(const edt_plan* p, int f, int64_t p0, int64_t np);
zd line_row_weight(const edt_plan* p, int f);
hipError_t launch_line_rows(const edt_plan* p, const zd* g64, int f, int64_t p0, int64_t np, int nr, zd* Rh,
                            hipStream_t st);

hipError_t launch_line_adjoint(const edt_plan* p, const double* vel, const zd* g64, const void* d_rows,
                               const double* chol, const double* trace, const double* x, double lambda_rel,
                               const zd* grad_v, void* grad_d, double* grad_lambda, double* grad_vel,
                               unsigned char* work, hipStream_t st) {
    const WorkLayout wl = work_layout(p);
    double* y = reinterpret_cast<double*>(work + wl.adj_y);
    double* dl = reinterpret_cast<double*>(work + wl.adj_dl);
    double* vpart = reinterpret_cast<double*>(work + wl.adj_vel);
    double* glam_part = reinterpret_cast<double*>(work + wl.aux);
    zd* gbar = reinterpret_cast<zd*>(work + wl.gbar);
    zd* Rh = reinterpret_cast<zd*>(work + wl.lrows);
    const int64_t P = p->n_pairs;
    if (P == 0) return hipSuccess;
    hipError_t e;
    hipLaunchKernelGGL(adj_pair_kernel, dim3(unsigned(P)), dim3(256), adjoint_lds_bytes(p->nz), st, chol, x, trace,
                       dptr<const int64_t>(p, p->lay.row_off), dptr<const int32_t>(p, p->lay.pair_u), p->nz, grad_v,
                       y, dl, glam_part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (grad_vel) {
        const int64_t nd = int64_t(p->n_freq) * p->n_cls * p->nz * 2;
        hipLaunchKernelGGL(zero_kernel, dim3(unsigned(std::min<int64_t>((nd + 255) / 256, 65536))), dim3(256), 0,
                           st, reinterpret_cast<double*>(gbar), nd);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (grad_d || grad_vel) {
        const int64_t chunk = line_chunk(p);
        for (int64_t p0 = 0; p0 < P; p0 += chunk) {
            const int64_t np = std::min<int64_t>(chunk, P - p0);
            for (int f = 0; f < p->n_freq; ++f) {
                const int nr = line_row_slots(p, f, p0, np);
                if ((e = launch_line_rows(p, g64, f, p0, np, nr, Rh, st)) != hipSuccess) return e;
                const zd W = line_row_weight(p, f);
                if (p->data_c64)
                    hipLaunchKernelGGL(line_adj_kernel<float2>, dim3(unsigned(np)), dim3(256), 0, st, Rh, g64,
                                       dptr<const int32_t>(p, p->lay.keys), dptr<const uint64_t>(p, p->lay.lmask),
                                       dptr<const int64_t>(p, p->lay.lfr), dptr<const int32_t>(p, p->lay.pair_u),
                                       static_cast<const float2*>(d_rows), x, y, dl, f, p->n_freq, p->n_cls,
                                       p->n_mid, p->n_line, p->nz, nr, W, lambda_rel, p0,
                                       static_cast<float2*>(grad_d), grad_vel ? gbar : nullptr);
                else
                    hipLaunchKernelGGL(line_adj_kernel<zd>, dim3(unsigned(np)), dim3(256), 0, st, Rh, g64,
                                       dptr<const int32_t>(p, p->lay.keys), dptr<const uint64_t>(p, p->lay.lmask),
                                       dptr<const int64_t>(p, p->lay.lfr), dptr<const int32_t>(p, p->lay.pair_u),
                                       static_cast<const zd*>(d_rows), x, y, dl, f, p->n_freq, p->n_cls,
                                       p->n_mid, p->n_line, p->nz, nr, W, lambda_rel, p0, static_cast<zd*>(grad_d),
                                       grad_vel ? gbar : nullptr);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
        }
    }
    if (grad_vel &&
        (e = launch_vel(p, vel, g64, x, y, dl, nullptr, nullptr, gbar, vpart, lambda_rel, grad_vel, st)) !=
            hipSuccess)
        return e;
    if (grad_lambda) {
        hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(256), 0, st, glam_part, P, 1, grad_lambda);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace edt
