// Symmetric eigenvalue kernels for the core of the incremental update.
//
// The core Gram matrix of Lemma 1 (S_{t+1}, or equivalently K^T K for the core
// K = [[Sigma, Y],[0, B_qr]]) is symmetric positive semidefinite of order
// n = r + k.  Corollary 3 keeps its top-r eigenpairs; Corollary 2 needs their sum.
//
//  sym_eig_kernel      Householder tridiagonalisation (one workgroup per problem)
//                      followed by Sturm-sequence bisection of the top eigenvalues.
//                      The matrix lives in 32x32 FP64 tiles: the trailing tile
//                      columns in LDS, the leading ones in a global (L2-resident)
//                      slot.  Each column step does one fused pass over the trailing
//                      tiles that applies the previous rank-2 update and accumulates
//                      the next symmetric matrix-vector product.
//  sym_vectors_kernel  Inverse iteration on the tridiagonal for the kept
//                      eigenvalues (independent random starts), Gram-Schmidt
//                      orthonormalisation, then back-transformation by the stored
//                      Householder vectors.
#include <float.h>

#include "common.hpp"
#include "kernels.hpp"

namespace cmsvd {

constexpr int ET = 256;          // threads per workgroup
constexpr int GT = 1024;         // threads per workgroup of the general (n > 320) kernel
constexpr int TILE = 32;         // tile edge
constexpr int TILE_EL = TILE * TILE;
constexpr int LDS_BYTES = 163840;  // gfx950: 160 KiB per workgroup

// Tiles are stored in "plane" order: the 4x4 sub-block held by lane (ly, lx) of a
// wave is spread over 16 planes of 64 doubles, element (4ly+s, 4lx+q) at
// (s*4+q)*64 + ly*8 + lx.  Every per-element access of a wave then touches 64
// consecutive doubles (no LDS bank conflicts, fully coalesced in global memory).
__device__ __forceinline__ int tile_off(int r, int c) {
    return ((((r & 3) << 2) | (c & 3)) << 6) + ((r >> 2) << 3) + (c >> 2);
}
__device__ __forceinline__ int plane_row(int el) { return (((el & 63) >> 3) << 2) + ((el >> 8) & 3); }
__device__ __forceinline__ int plane_col(int el) { return ((el & 7) << 2) + ((el >> 6) & 3); }

__device__ __forceinline__ double* tile_ptr(int R, int C, int T, int c0, int TL, double* gt, double* lt) {
    if (C >= c0) {
        const int cc = C - c0, rr = R - c0;
        const int idx = cc * TL - (cc * (cc - 1)) / 2 + (rr - cc);
        return lt + (size_t)idx * TILE_EL;
    }
    const int idx = C * T - (C * (C - 1)) / 2 + (R - C);
    return gt + (size_t)idx * TILE_EL;
}

__device__ __forceinline__ double hval(const EigDesc& D, int i, int c) {
    if (i >= D.n || c >= D.n) return 0.0;
    const int n1 = D.n1;
    if (i < n1 && c < n1) return (i == c) ? D.s[i] * D.s[i] : 0.0;
    if (i >= n1 && c < n1) return D.s[c] * D.P[(long)c + (long)(i - n1) * D.ldp];
    if (i < n1) return D.s[i] * D.P[(long)i + (long)(c - n1) * D.ldp];
    return D.Y[(long)(i - n1) + (long)(c - n1) * D.ldy];
}

// Number of eigenvalues of the tridiagonal T (diagonal dd, e2 = off-diagonal squared)
// below x: the number of negative pivots q_i of T - x I = L D L^T.  The pivots are kept
// as ratios q_i = p_i / p_{i-1} of the leading minors, which obey the three-term
// recurrence p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2} (p_{-1} = 1): one FMA per step
// on the dependent chain (e^2 p_{i-2} is formed a step ahead), where the pivot form needs
// a reciprocal and its refinement.  Each computed ratio satisfies the pivot recurrence
// with d_i - x and e_{i-1}^2 perturbed by a few ulps, so the count is exact for a
// tridiagonal that close to T, as for the pivot form.  sc = 2^-k >= ... scales T to norm
// below 1 exactly (a power of two), and the pair (p_{i-1}, p_i) is renormalised by a
// power of two every four steps, so nothing overflows or underflows; signs are exact.
// An exactly zero minor stands for a negative pivot of size 2^-60 ||T||.
template <int KP>
__device__ __forceinline__ void sturm_step(double dl, double el, const double (&xs)[KP], double sc, double (&p1)[KP],
                                           double (&p2)[KP], int (&cnt)[KP]) {
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const double tk = -el * p2[k];
        double p = fma(dl * sc - xs[k], p1[k], tk);
        if (p == 0.0) p = -0x1p-60 * p1[k];
        cnt[k] += (p < 0.0) != (p1[k] < 0.0);
        p2[k] = p1[k];
        p1[k] = p;
    }
}

template <int KP>
__device__ __forceinline__ void sturm_renorm(double (&p1)[KP], double (&p2)[KP]) {
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(p1[k]), fabs(p2[k])));
        p1[k] = ldexp(p1[k], -e);
        p2[k] = ldexp(p2[k], -e);
        if (p1[k] == 0.0) p1[k] = -0x1p-60 * p2[k];  // underflow of a tiny minor
    }
}

// Full blocks of four steps run without bounds checks, with the next block's operands
// loaded ahead (at most three entries past n - 1 are read and not used; the callers'
// arrays are padded past n); the last n - 1 mod 4 steps follow one by one.
template <int KP>
__device__ __forceinline__ void sturm_count_k(const double* dd, const double* e2, int n, const double (&x)[KP],
                                              double sc, int (&cnt)[KP]) {
    const double sc2 = sc * sc;
    double xs[KP], p1[KP], p2[KP];  // x sc, p_{i-1}, p_{i-2}
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        xs[k] = x[k] * sc;
        p2[k] = 1.0;
        p1[k] = dd[0] * sc - xs[k];
        if (p1[k] == 0.0) p1[k] = -0x1p-60;
        cnt[k] = p1[k] < 0.0;
    }
    int i = 1;
    double dn[4], en[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        dn[m] = dd[i + m];
        en[m] = e2[i + m - 1];
    }
    for (; i + 3 < n; i += 4) {
        double dl[4], el[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            dl[m] = dn[m];
            el[m] = en[m] * sc2;
            dn[m] = dd[i + 4 + m];
            en[m] = e2[i + 3 + m];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) sturm_step<KP>(dl[m], el[m], xs, sc, p1, p2, cnt);
        sturm_renorm<KP>(p1, p2);
    }
    for (int m = 0; i < n; ++i, ++m) sturm_step<KP>(dn[m], en[m] * sc2, xs, sc, p1, p2, cnt);
}

// The same count on a tridiagonal prepared for it once: ds = sc d and, for the n - 1
// off-diagonals, e2s = max(sc^2 e^2, 2^-120) (sc = 2^-k scales T to norm below 1).
// Raising an off-diagonal of at most 2^-60 to 2^-60 moves no eigenvalue by more than
// 2^-60, far below the bisection's resolution.  With every e^2 positive a zero minor
// needs no test: p_i = 0 makes p_{i+1} = -e_i^2 p_{i-1}, of the sign opposite to
// p_{i-1}, so the two comparisons around it count one sign change whichever sign the
// zero is given, and no two consecutive minors vanish.  One step changes the pair's
// larger member by a factor between about 2^-120 (cancellation) and 3, so the pair is
// renormalised every eight steps.  Reads up to seven entries past the end of each
// array (not used).
template <int KP>
__device__ __forceinline__ void sturm_count_scaled(const double* ds, const double* e2s, int n, const double (&x)[KP],
                                                   double sc, int (&cnt)[KP]) {
    double xs[KP], p1[KP], p2[KP];  // x sc, p_{i-1}, p_{i-2}
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        xs[k] = x[k] * sc;
        p2[k] = 1.0;
        p1[k] = ds[0] - xs[k];
        cnt[k] = p1[k] < 0.0;
    }
    auto step = [&](double dl, double el) {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const double p = fma(dl - xs[k], p1[k], -el * p2[k]);
            cnt[k] += (p < 0.0) != (p1[k] < 0.0);
            p2[k] = p1[k];
            p1[k] = p;
        }
    };
    auto rescale = [&]() {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(p1[k]), fabs(p2[k])));
            p1[k] = ldexp(p1[k], -e);
            p2[k] = ldexp(p2[k], -e);
        }
    };
    // two operand buffers of eight steps: one is loaded while the other is used
    double da[8], ea[8], db[8], eb[8];
    auto load = [&](double (&d8)[8], double (&e8)[8], int at) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            d8[m] = ds[at + m];
            e8[m] = e2s[at + m - 1];
        }
    };
    int i = 1;
    load(da, ea, i);
    for (; i + 15 < n; i += 16) {
        load(db, eb, i + 8);
#pragma unroll
        for (int m = 0; m < 8; ++m) step(da[m], ea[m]);
        rescale();
        load(da, ea, i + 16);
#pragma unroll
        for (int m = 0; m < 8; ++m) step(db[m], eb[m]);
        rescale();
    }
    if (i + 7 < n) {  // da holds steps i .. i + 7
        load(db, eb, i + 8);
#pragma unroll
        for (int m = 0; m < 8; ++m) step(da[m], ea[m]);
        rescale();
        i += 8;
        for (int m = 0; i < n; ++i, ++m) step(db[m], eb[m]);
    } else {
        for (int m = 0; i < n; ++i, ++m) step(da[m], ea[m]);
    }
}

// The count of sturm_count_scaled<1> (the same steps in the same order, renormalised
// after every eight, so the same result) with one operand buffer instead of two: fewer
// registers, for kernels that hide latency with many wavefronts rather than loads ahead.
__device__ __forceinline__ int sturm_count_lean(const double* ds, const double* e2s, int n, double x, double sc) {
    const double xs = x * sc;
    double p2 = 1.0, p1 = ds[0] - xs;
    int cnt = p1 < 0.0;
    int i = 1;
    for (; i + 7 < n; i += 8) {
        double d8[8], e8[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            d8[m] = ds[i + m];
            e8[m] = e2s[i + m - 1];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const double p = fma(d8[m] - xs, p1, -e8[m] * p2);
            cnt += (p < 0.0) != (p1 < 0.0);
            p2 = p1;
            p1 = p;
        }
        const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(p1), fabs(p2)));
        p1 = ldexp(p1, -e);
        p2 = ldexp(p2, -e);
    }
    for (; i < n; ++i) {
        const double p = fma(ds[i] - xs, p1, -e2s[i - 1] * p2);
        cnt += (p < 0.0) != (p1 < 0.0);
        p2 = p1;
        p1 = p;
    }
    return cnt;
}

__device__ __forceinline__ int sturm_count(const double* dd, const double* e2, int n, double x, double sc) {
    const double xs[1] = {x};
    int c[1];
    sturm_count_k<1>(dd, e2, n, xs, sc, c);
    return c[0];
}

// (hi, lo) = trace(T) - (hi, lo): the sum of the top eigenvalues from that of the bottom
// ones (double-double).
__device__ __forceinline__ void top_from_trace(const double* dd, int n, double& hi, double& lo) {
    double th = 0.0, tl = 0.0;
    for (int i = 0; i < n; ++i) dd_add(th, tl, dd[i]);
    double s, e;
    two_sum(th, -hi, s, e);
    e += tl - lo;
    two_sum(s, e, hi, lo);
}

// 2^-k with 2^(k-1) <= tnorm < 2^k (1 for tnorm = 0): scales T to norm below 1 exactly.
__device__ __forceinline__ double sturm_scale(double tnorm) {
    return tnorm > 0.0 && tnorm < INFINITY ? ldexp(1.0, -__builtin_amdgcn_frexp_exp(tnorm)) : 1.0;
}

static int tl_for(int npad, int T) {
    const long vec_bytes = (10L * npad + 32) * 8;
    int tl = 0;
    while (tl + 1 <= T && vec_bytes + (long)(tl + 1) * (tl + 2) / 2 * TILE_EL * 8 <= LDS_BYTES) ++tl;
    return tl;
}

__device__ __forceinline__ void tile_step(double (&a)[16], int R, int C, const double* __restrict__ vc,
                                          const double* __restrict__ vp, const double* __restrict__ wp,
                                          double* pww, int ly, int lx);

template <int MODE, int NT>
__global__ void __launch_bounds__(NT) sym_eig_kernel(const EigDesc* __restrict__ descs, int count, int NP,
                                                     int TLmax, double* __restrict__ gws, long slot_doubles) {
    extern __shared__ double lds[];
    double* vc = lds;             // current Householder vector
    double* vp = vc + NP;         // previous vector  (pending rank-2 update)
    double* wp = vp + NP;         // previous w
    double* xv = wp + NP;         // column / p scratch
    double* pw = xv + NP;         // 4 per-wave partial products
    double* dd = pw + 4 * NP;     // tridiagonal diagonal
    double* ee = dd + NP;         // tridiagonal off-diagonal
    double* red = ee + NP;        // reduction scratch (16)
    double* scal = red + 16;      // broadcast scalars (16)
    double* lt = scal + 16;       // LDS tiles
    double* gt = gws + (size_t)blockIdx.x * (size_t)slot_doubles;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int ly = lane >> 3, lx = lane & 7;

    for (int prob = blockIdx.x; prob < count; prob += gridDim.x) {
        const EigDesc D = descs[prob];
        const int n = D.n;
        const int T = (n + TILE - 1) / TILE, npad = T * TILE;
        const int TL = T < TLmax ? T : TLmax, c0 = T - TL;

        // ---- assemble H into tiles (diagonal tiles hold both triangles) ----
        for (int C = 0; C < T; ++C)
            for (int R = C; R < T; ++R) {
                double* tp = tile_ptr(R, C, T, c0, TL, gt, lt);
                for (int el = t; el < TILE_EL; el += NT) tp[el] = hval(D, R * TILE + plane_row(el), C * TILE + plane_col(el));
            }
        for (int i = t; i < npad; i += NT) {
            vc[i] = vp[i] = wp[i] = xv[i] = 0.0;
            pw[i] = pw[NP + i] = pw[2 * NP + i] = pw[3 * NP + i] = 0.0;
            dd[i] = ee[i] = 0.0;
        }
        __syncthreads();

        // ---- Householder tridiagonalisation, lower storage ----
        for (int j = 0; j < n; ++j) {
            const int Cj = j >> 5, cj = j & 31;
            // (A) column j with the pending update of step j-1
            const double vpj = vp[j], wpj = wp[j];
            double part = 0.0;
            for (int i = j + t; i < n; i += NT) {
                const double* tp = tile_ptr(i >> 5, Cj, T, c0, TL, gt, lt);
                const double val = tp[tile_off(i & 31, cj)] - (vp[i] * wpj + wp[i] * vpj);
                if (i == j) dd[j] = val;
                else {
                    xv[i] = val;
                    if (i >= j + 2) part += val * val;
                }
            }
            if (j == n - 1) break;
            const double xn2 = block_sum(part, red);
            if (t == 0) {
                const double alpha = xv[j + 1];
                double tau = 0.0, beta = alpha, scale = 0.0;
                if (xn2 > 0.0) {
                    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                    tau = (beta - alpha) / beta;
                    scale = 1.0 / (alpha - beta);
                }
                ee[j] = beta;
                scal[0] = tau;
                scal[1] = scale;
                if (MODE == 1 && D.tau) D.tau[j] = tau;
            }
            __syncthreads();
            const double tau = scal[0], scale = scal[1];
            for (int i = t; i < npad; i += NT) {
                double v = 0.0;
                if (tau != 0.0) {
                    if (i == j + 1) v = 1.0;
                    else if (i >= j + 2 && i < n) v = xv[i] * scale;
                }
                vc[i] = v;
                if (MODE == 1 && D.V && i >= j + 2 && i < n) D.V[(long)i + (long)j * D.ldv] = v;
            }
            __syncthreads();

            // (B) fused pass over the trailing tiles: apply A -= vp wp^T + wp vp^T on
            //     the active block (rows, cols >= j+1) and accumulate p = A vc.
            int f = 0;
            for (int C = Cj; C < T; ++C) {
                for (int R = C; R < T; ++R, ++f) {
                    if ((f % (NT / 64)) != w) continue;
                    double* tp = tile_ptr(R, C, T, c0, TL, gt, lt);
                    double a[16];
#pragma unroll
                    for (int e = 0; e < 16; ++e) a[e] = tp[(e << 6) + lane];
                    tile_step(a, R, C, vc, vp, wp, pw + (w & 3) * NP, ly, lx);
#pragma unroll
                    for (int e = 0; e < 16; ++e) tp[(e << 6) + lane] = a[e];
                }
            }
            __syncthreads();

            // (C) p = tau * A v, w = p - (tau/2)(p.v) v
            double dpart = 0.0;
            for (int i = t; i < npad; i += NT) {
                const double sacc = pw[i] + pw[NP + i] + pw[2 * NP + i] + pw[3 * NP + i];
                pw[i] = pw[NP + i] = pw[2 * NP + i] = pw[3 * NP + i] = 0.0;
                const double pi = (i >= j + 1 && i < n) ? tau * sacc : 0.0;
                xv[i] = pi;
                dpart += pi * vc[i];
            }
            const double dot = block_sum(dpart, red);
            const double K = -0.5 * tau * dot;
            for (int i = t; i < npad; i += NT) {
                wp[i] = (i >= j + 1 && i < n) ? xv[i] + K * vc[i] : 0.0;
                vp[i] = vc[i];
            }
            __syncthreads();
        }
        __syncthreads();

        // ---- bisection for the nkeep largest eigenvalues ----
        for (int i = t; i < npad; i += NT) xv[i] = (i < n - 1) ? ee[i] * ee[i] : 0.0;
        double glo = INFINITY, ghi = -INFINITY, em = 0.0;
        for (int i = t; i < n; i += NT) {
            const double rad = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i < n - 1 ? fabs(ee[i]) : 0.0);
            glo = fmin(glo, dd[i] - rad);
            ghi = fmax(ghi, dd[i] + rad);
            if (i < n - 1) em = fmax(em, ee[i] * ee[i]);
        }
        glo = -block_max(-glo, red);
        ghi = block_max(ghi, red);
        em = block_max(em, red);
        const double tnorm = fmax(fabs(glo), fabs(ghi));
        const double pivmin = DBL_MIN * fmax(1.0, em);
        const double tol = 4.0 * DBL_EPSILON * tnorm + 2.0 * pivmin;
        const double sc = sturm_scale(tnorm);
        glo -= tol;
        ghi += tol;
        double* lamv = pw;  // free now
        // the error needs only the sum of the top nkeep: above half the spectrum, the
        // bottom n - nkeep are found and subtracted from the trace (as in the small kernel)
        const bool bottom = MODE == 0 && 2 * D.nkeep > n;
        const int nb = bottom ? n - D.nkeep : D.nkeep;
        for (int q = t; q < nb; q += NT) {
            double lo = glo, hi = ghi;
            const int target = bottom ? q + 1 : n - q;
            while (hi - lo > tol) {
                const double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (sturm_count(dd, xv, n, mid, sc) >= target) hi = mid;
                else lo = mid;
            }
            lamv[q] = 0.5 * (lo + hi);
        }
        __syncthreads();
        if (t == 0) {
            double hi = 0.0, lo = 0.0;
            for (int q = 0; q < nb; ++q) dd_add(hi, lo, lamv[q]);
            if (bottom) top_from_trace(dd, n, hi, lo);
            if (MODE == 0) {
                double eh = D.na[0], el = D.na[1];
                if (D.nb) {
                    dd_add(eh, el, D.nb[0]);
                    el += D.nb[1];
                }
                double s, e;
                two_sum(eh, -hi, s, e);
                double tail = s + (e + el - lo);
                if (tail < 0.0) tail = 0.0;  // clamp rounding below zero; NaN propagates
                const double err = sqrt(tail);
                const double etot = eh + el;
                *D.out_err = err;
                if (D.out_rel) *D.out_rel = etot != 0.0 ? err / sqrt(etot) : 0.0;
            } else if (D.sum_top) {
                D.sum_top[0] = hi;
                D.sum_top[1] = lo;
            }
        }
        if (MODE == 1) {
            for (int q = t; q < D.nkeep; q += NT) D.lam[q] = lamv[q];
            if (D.d)
                for (int i = t; i < n; i += NT) {
                    D.d[i] = dd[i];
                    if (i < n - 1) D.e[i] = ee[i];
                }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Register-resident variant for n <= 320 (at most 10 tile rows).
//
// 512 threads (8 waves, two per SIMD).  The trailing (up to) 5 tile columns live in
// LDS; every other lower tile (at most 40) lives permanently in the VGPRs of one wave
// (a contiguous row-major chunk of 5 slots per wave), so the reduction never touches
// global memory.  A column step costs three barriers (two in the shared-vector
// kernels, see the kernel).  Bisection is a multisection with 512 / nkeep probes per
// eigenvalue per round.
// ---------------------------------------------------------------------------
constexpr int RT = 512;
constexpr int RW = RT / 64;
constexpr int NSLOT = 5;
constexpr int REG_TMAX = 10;
constexpr int RTL = 5;

__device__ __forceinline__ double pick4(const double (&a)[16], int s, int q) {
    const double x0 = a[s * 4 + 0], x1 = a[s * 4 + 1], x2 = a[s * 4 + 2], x3 = a[s * 4 + 3];
    return q == 0 ? x0 : (q == 1 ? x1 : (q == 2 ? x2 : x3));
}

// One tile of the fused pass, for a tile held as a 4x4 sub-block per lane
// (a[s*4+q] = element (4ly+s, 4lx+q)): applies the pending rank-2 update of step
// j-1 and accumulates the partial products of A v into this wave's buffer pww.
// The update is applied unmasked: vp and wp vanish below index j, and the only
// extra elements it touches (row and column j) are never read again.  vc holds v
// (zero outside [j+1, n)), so the products need no masking either.
//
// Row sums are reduced over the 8 lanes of a row group (lx) with DPP; lane lx < 4
// then adds row 4ly+lx.  Column sums (off-diagonal tiles only; diagonal tiles hold
// both triangles) are reduce-scattered over ly: the two swap stages pair different
// columns, so after the last DPP stage the lanes with even ly hold column
// 4lx + q, q = (ly>>2) + 2((ly>>1)&1), each summed over all eight row groups.
__device__ __forceinline__ void tile_step(double (&a)[16], int R, int C, const double* __restrict__ vc,
                                          const double* __restrict__ vp, const double* __restrict__ wp,
                                          double* pww, int ly, int lx) {
    const int gi0 = R * TILE + 4 * ly, gc0 = C * TILE + 4 * lx;
    double vq[4], wq[4], cq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        vq[q] = vp[gc0 + q];
        wq[q] = wp[gc0 + q];
        cq[q] = vc[gc0 + q];
    }
    double cp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double vr = vp[gi0 + s], wr = wp[gi0 + s], cr = vc[gi0 + s];
        double rp = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double x = fma(-vr, wq[q], a[s * 4 + q]);
            x = fma(-wr, vq[q], x);
            a[s * 4 + q] = x;
            rp = fma(x, cq[q], rp);
            cp[q] = fma(x, cr, cp[q]);
        }
        rp = sum_lanes8(rp);
        if (lx == s) unsafeAtomicAdd(&pww[gi0 + s], rp);
    }
    if (R != C) {
        const double s01 = add_swap32(cp[0], cp[1]);
        const double s23 = add_swap32(cp[2], cp[3]);
        double t = add_swap16(s01, s23);
        t += dpp_move<0x128>(t);
        if ((ly & 1) == 0) unsafeAtomicAdd(&pww[gc0 + (ly >> 2) + 2 * ((ly >> 1) & 1)], t);
    }
}

// 0.0 formed where it is used.  In the column loops of the register kernels the
// compiler otherwise keeps one zero register pair for the whole loop, spills it under
// register pressure, and reloads it from scratch at each store of a zero.
__device__ __forceinline__ double fresh_zero() {
    double z;
    asm volatile("v_mov_b64 %0, 0" : "=v"(z));
    return z;
}

// Vector index -> LDS position.  In the shared-vector kernels (SW) two doubles of
// padding follow every sixteen: the eight 4-element groups that the lanes of one tile
// read (32 bytes apart) then fall on distinct LDS banks instead of pairing up.
template <bool SW>
__device__ __forceinline__ int vpos(int i) { return SW ? i + 2 * (i >> 4) : i; }

// Four consecutive doubles of a vector as two 16-byte LDS loads: the groups read per
// tile start at even positions of 16-byte aligned vectors, and the loads' 16-bit
// offsets let one address reach all three vectors.
__device__ __forceinline__ void ld4(const double* p, double (&o)[4]) {
    const double2 x = reinterpret_cast<const double2*>(p)[0], y = reinterpret_cast<const double2*>(p)[1];
    o[0] = x.x;
    o[1] = x.y;
    o[2] = y.x;
    o[3] = y.y;
}

// The same tile update for row-owned passes: the row partials are accumulated into
// racc (per lane, rows 4ly..4ly+3 of the tile row) instead of being reduced per tile;
// flush_rows reduces and publishes them once per tile row.
template <bool SW>
__device__ __forceinline__ void tile_step_racc(double (&a)[16], int R, int C, const double* __restrict__ vc,
                                               const double* __restrict__ vp, const double* __restrict__ wp,
                                               double* pww, int ly, int lx, double (&racc)[4]) {
    const int gi0 = vpos<SW>(R * TILE + 4 * ly), gc0 = vpos<SW>(C * TILE + 4 * lx);
    double vq[4], wq[4], cq[4], vr4[4], wr4[4], cr4[4];
    ld4(vp + gc0, vq);
    ld4(wp + gc0, wq);
    ld4(vc + gc0, cq);
    ld4(vp + gi0, vr4);
    ld4(wp + gi0, wr4);
    ld4(vc + gi0, cr4);
    double cp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double vr = vr4[s], wr = wr4[s], cr = cr4[s];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double x = fma(-vr, wq[q], a[s * 4 + q]);
            x = fma(-wr, vq[q], x);
            a[s * 4 + q] = x;
            racc[s] = fma(x, cq[q], racc[s]);
            cp[q] = fma(x, cr, cp[q]);
        }
    }
    if (R != C) {
        const double s01 = add_swap32(cp[0], cp[1]);
        const double s23 = add_swap32(cp[2], cp[3]);
        double t = add_swap16(s01, s23);
        t += dpp_move<0x128>(t);
        if ((ly & 1) == 0) unsafeAtomicAdd(&pww[gc0 + (ly >> 2) + 2 * ((ly >> 1) & 1)], t);
    }
}

// The same step on a tile held in LDS (plane order: element s*4 + q of lane at
// tp[(s*4 + q) * 64 + lane]), one of its four rows at a time, so that only four of its
// elements occupy registers beside the resident tiles (more would spill those).
template <bool SW>
__device__ __forceinline__ void tile_step_lds(double* tp, int lane, int R, int C, const double* __restrict__ vc,
                                              const double* __restrict__ vp, const double* __restrict__ wp,
                                              double* pww, int ly, int lx, double (&racc)[4]) {
    const int gi0 = vpos<SW>(R * TILE + 4 * ly), gc0 = vpos<SW>(C * TILE + 4 * lx);
    double vq[4], wq[4], cq[4], vr4[4], wr4[4], cr4[4];
    ld4(vp + gc0, vq);
    ld4(wp + gc0, wq);
    ld4(vc + gc0, cq);
    ld4(vp + gi0, vr4);
    ld4(wp + gi0, wr4);
    ld4(vc + gi0, cr4);
    double cp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        double a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = tp[((4 * s + q) << 6) + lane];
        const double vr = vr4[s], wr = wr4[s], cr = cr4[s];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double x = fma(-vr, wq[q], a[q]);
            x = fma(-wr, vq[q], x);
            a[q] = x;
            racc[s] = fma(x, cq[q], racc[s]);
            cp[q] = fma(x, cr, cp[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) tp[((4 * s + q) << 6) + lane] = a[q];
    }
    if (R != C) {
        const double s01 = add_swap32(cp[0], cp[1]);
        const double s23 = add_swap32(cp[2], cp[3]);
        double t = add_swap16(s01, s23);
        t += dpp_move<0x128>(t);
        if ((ly & 1) == 0) unsafeAtomicAdd(&pww[gc0 + (ly >> 2) + 2 * ((ly >> 1) & 1)], t);
    }
}

// The two steps above with the row values v, w, v_j of the tile row given by the
// caller, which loads them once per tile row (kernels with registers to spare).
template <bool SW>
__device__ __forceinline__ void tile_step_racc_rows(double (&a)[16], int R, int C, const double* __restrict__ vc,
                                               const double* __restrict__ vp, const double* __restrict__ wp,
                                               double* pww, int ly, int lx, double (&racc)[4],
        const double (&vr4)[4], const double (&wr4)[4], const double (&cr4)[4]) {
    const int gc0 = vpos<SW>(C * TILE + 4 * lx);
    double vq[4], wq[4], cq[4];
    ld4(vp + gc0, vq);
    ld4(wp + gc0, wq);
    ld4(vc + gc0, cq);
    double cp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double vr = vr4[s], wr = wr4[s], cr = cr4[s];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double x = fma(-vr, wq[q], a[s * 4 + q]);
            x = fma(-wr, vq[q], x);
            a[s * 4 + q] = x;
            racc[s] = fma(x, cq[q], racc[s]);
            cp[q] = fma(x, cr, cp[q]);
        }
    }
    if (R != C) {
        const double s01 = add_swap32(cp[0], cp[1]);
        const double s23 = add_swap32(cp[2], cp[3]);
        double t = add_swap16(s01, s23);
        t += dpp_move<0x128>(t);
        if ((ly & 1) == 0) unsafeAtomicAdd(&pww[gc0 + (ly >> 2) + 2 * ((ly >> 1) & 1)], t);
    }
}

template <bool SW>
__device__ __forceinline__ void tile_step_lds_rows(double* tp, int lane, int R, int C, const double* __restrict__ vc,
                                              const double* __restrict__ vp, const double* __restrict__ wp,
                                              double* pww, int ly, int lx, double (&racc)[4],
        const double (&vr4)[4], const double (&wr4)[4], const double (&cr4)[4]) {
    const int gc0 = vpos<SW>(C * TILE + 4 * lx);
    double vq[4], wq[4], cq[4];
    ld4(vp + gc0, vq);
    ld4(wp + gc0, wq);
    ld4(vc + gc0, cq);
    double cp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        double a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = tp[((4 * s + q) << 6) + lane];
        const double vr = vr4[s], wr = wr4[s], cr = cr4[s];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double x = fma(-vr, wq[q], a[q]);
            x = fma(-wr, vq[q], x);
            a[q] = x;
            racc[s] = fma(x, cq[q], racc[s]);
            cp[q] = fma(x, cr, cp[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) tp[((4 * s + q) << 6) + lane] = a[q];
    }
    if (R != C) {
        const double s01 = add_swap32(cp[0], cp[1]);
        const double s23 = add_swap32(cp[2], cp[3]);
        double t = add_swap16(s01, s23);
        t += dpp_move<0x128>(t);
        if ((ly & 1) == 0) unsafeAtomicAdd(&pww[gc0 + (ly >> 2) + 2 * ((ly >> 1) & 1)], t);
    }
}

// Publishes the row partials of tile row R (four per lane) and clears them.  A
// transpose-reduce over the eight lanes of a row group (lx): each stage keeps half of
// the values and exchanges the other half with the partner lane, so that lane lx ends
// with row 2*bit2(lx) + bit1(lx) summed over the group; the lanes with even lx add it.
template <bool SW>
__device__ __forceinline__ void flush_rows(int R, double (&racc)[4], double* pww, int ly, int lx) {
    const bool b2 = (lx & 4) != 0, b1 = (lx & 2) != 0;
    const double u0 = (b2 ? racc[2] : racc[0]) + dpp_move<0x141>(b2 ? racc[0] : racc[2]);  // partner lx ^ 7
    const double u1 = (b2 ? racc[3] : racc[1]) + dpp_move<0x141>(b2 ? racc[1] : racc[3]);
    double v = (b1 ? u1 : u0) + dpp_move<0x4E>(b1 ? u0 : u1);                             // partner lx ^ 2
    v += dpp_move<0xB1>(v);                                                                 // partner lx ^ 1
    if ((lx & 1) == 0) unsafeAtomicAdd(&pww[vpos<SW>(R * TILE + 4 * ly) + (lx >> 1)], v);
#pragma unroll
    for (int s = 0; s < 4; ++s) racc[s] = 0.0;
}

__device__ __forceinline__ int lds_tile_index(int R, int C, int c0, int TL) {
    const int cc = C - c0, rr = R - c0;
    return cc * TL - (cc * (cc - 1)) / 2 + (rr - cc);
}

constexpr int REG_NP = REG_TMAX * TILE;  // vector length (fixed layout)

// LDS of the register kernels, in doubles, in the kernel's order: xv (np); vc, vp, wp, xn
// (np, padded by vpos in the shared-vector kernels); the partials of A v (one vector per
// wave; with SHV two padded partial vectors and the second unscaled-column buffer,
// see the kernel); dd, ee (np); 16 for the reductions; the
// LDS tiles (the last rtl tile columns); the geometry ints: rw*nslot slot codes, then per
// tile column c the LDS-tile share of every wave ((first << 8) | count, rw*tmax).
__host__ __device__ constexpr int reg_npp(int tmax, bool shv) { return shv ? tmax * TILE + tmax * TILE / 8 : tmax * TILE; }
__host__ __device__ constexpr int reg_lds_doubles(int rw, int nslot, int rtl, int tmax, bool shv) {
    return 3 * tmax * TILE + 4 * reg_npp(tmax, shv) + (shv ? 3 * reg_npp(tmax, shv) : rw * tmax * TILE) + 16 +
           rtl * (rtl + 1) / 2 * TILE_EL + (rw * nslot + rw * tmax + 1) / 2;
}
constexpr int REG_LDS_DOUBLES = reg_lds_doubles(RW, NSLOT, RTL, REG_TMAX, false);
constexpr int REG_LDS_DOUBLES_SHV = reg_lds_doubles(RW, NSLOT, RTL, REG_TMAX, true);
static_assert(REG_LDS_DOUBLES * 8 <= LDS_BYTES, "register-resident eigen kernel exceeds the LDS");
static_assert(REG_LDS_DOUBLES_SHV <= REG_LDS_DOUBLES, "the shared-vector layout is the smaller one");
// Thin cores (65..160): 256 threads, 4 slots per wave (16 >= 15 tiles), no LDS tiles.
constexpr int THIN_TMAX = 5;
constexpr int THIN_NSLOT = 4;
constexpr int THIN_LDS_DOUBLES = reg_lds_doubles(4, THIN_NSLOT, 0, THIN_TMAX, false);
constexpr int THIN_LDS_DOUBLES_SHV = reg_lds_doubles(4, THIN_NSLOT, 0, THIN_TMAX, true);

// SHV: the waves accumulate the products into one shared vector instead of a vector
// each, and a step has two barriers instead of three: the tiles multiply by the
// unscaled column below its first subdiagonal element (x, zero elsewhere) instead of
// by v, so no barrier is needed between the Householder scalars and the tile pass.
// (W) assembles A v = A e_{j+1} + scale A x from the published column j + 1 and the
// products, and by symmetry v^T A v = A_{j+1,j+1} + 2 scale (A x)_{j+1} + scale^2 x^T A x.
// The unscaled column and the products alternate between two buffers by step parity,
// so (W) prepares the next step's while every wave may still read this step's; the
// wave that forms the Householder scalars also forms the column's norm from that
// buffer.  The vectors read per tile position (x, vp, wp, xn, the products)
// are laid out by vpos<SHV>.
template <int MODE, int RT_, int NSLOT_, int RTL_, int TMAX_, bool SHV = false>
__global__ void __launch_bounds__(RT_, 1024 / RT_ > 1 ? 512 / RT_ : 1) sym_eig_reg_kernel(const EigDesc* __restrict__ descs,
                                                                                 int count) {
    constexpr int RT = RT_, RW = RT_ / 64, NSLOT = NSLOT_, RTL = RTL_;
    constexpr int NP = TMAX_ * TILE, NPP = reg_npp(TMAX_, SHV), PWL = SHV ? 3 * NPP : RW * NP;
    static_assert(!SHV || MODE == 2, "the shared-vector layout has no room for the bisection's brackets");
    static_assert(RT_ >= TMAX_ * TILE, "(H) and (W) form one vector element per thread");
    extern __shared__ __align__(16) double lds[];
    double* xv = lds;           // current column below the diagonal (later e^2)
    double* vc = xv + NP;       // Householder vector v_j of the current step
    double* vp = vc + NPP;      // v of the previous step
    double* wp = vp + NPP;      // w of the previous step
    double* xn = wp + NPP;      // next column as held in the register tiles
    double* pw = xn + NPP;      // partials of A v (PWL doubles)
    double* xs1 = pw + 2 * NPP;  // SHV: unscaled column of odd steps (vc holds the even steps')
    double* dd = pw + PWL;
    double* ee = dd + NP;
    double* red = ee + NP;      // 16: per-wave dots (0..7), per-wave norm partials (8..15)
    double* lt = red + 16;      // LDS tiles
    // register-slot geometry (R << 8 | C, or -1), re-read every step so that no
    // per-slot scalar state stays live across the column loop
    int* geo = reinterpret_cast<int*>(lt + RTL * (RTL + 1) / 2 * TILE_EL);
    const int t = threadIdx.x, lane = t & 63, ly = lane >> 3, lx = lane & 7;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);

    for (int prob = blockIdx.x; prob < count; prob += gridDim.x) {
        const EigDesc D = descs[prob];
        const int n = D.n, T = (n + TILE - 1) / TILE, npad = T * TILE;
        const int TL = T < RTL ? T : RTL, c0 = T - TL;
        const int ngl = c0 * T - (c0 * (c0 - 1)) / 2;
        // Register tiles (columns below c0) in row-major order, split into contiguous
        // chunks of at most NSLOT per wave, so that a wave's tiles share tile rows.
        const int cs = (ngl + RW - 1) / RW;
        if (t < RW * NSLOT) {
            const int ww = t / NSLOT, sl = t % NSLOT;
            int code = -1;
            if constexpr (RW == 4 && RTL == 0 && SHV) {
                // The register-only trailing kernel retires whole tile columns as it goes:
                // its tiles are dealt round-robin to the waves from the last tile column
                // backwards, so that every wave keeps a share of the columns still active.
                int g = sl * RW + ww;
                if (g < ngl)
                    for (int C = c0 - 1; C >= 0; --C) {
                        if (g < T - C) {
                            code = ((C + g) << 8) | C;
                            break;
                        }
                        g -= T - C;
                    }
            } else {
                int g = ww * cs + sl;
                if (sl < cs && g < ngl) {
                    int R = 0;
                    while (g >= (R + 1 < c0 ? R + 1 : c0)) {
                        g -= (R + 1 < c0 ? R + 1 : c0);
                        ++R;
                    }
                    code = (R << 8) | g;
                }
            }
            geo[t] = code;
        }
        __syncthreads();
        // For each tile column c (the step's leading column), the active LDS tiles
        // (columns >= max(c, c0)) in row-major order, handed out in contiguous shares
        // that balance a load model of the step: a register tile costs 5 units, an LDS
        // tile 8 (it also moves its elements through LDS).  Each LDS tile goes to the
        // SIMD with the least load (waves w and w + 4 share one), and there to the
        // wave with the least load, a younger wave (w >= 4, which loses issue
        // arbitration to the older one) counted 40 % heavier.
        if (t < T) {
            const int c = t, cl = c > c0 ? c : c0, mL = T - cl, NL = mL * (mL + 1) / 2;
            int load[RW], k[RW];
#pragma unroll
            for (int ww = 0; ww < RW; ++ww) {
                int rc = 0;
                for (int sl = 0; sl < NSLOT; ++sl) rc += (geo[ww * NSLOT + sl] >= 0 && (geo[ww * NSLOT + sl] & 255) >= c) ? 1 : 0;
                load[ww] = 5 * rc + (SHV && ww == RW - 1 ? 8 : 0);  // the last wave also forms the norm
                k[ww] = 0;
            }
            for (int m = 0; m < NL; ++m) {
                int bs = 0, bl = 0x7fffffff;
#pragma unroll
                for (int sd = 0; sd < (RW < 4 ? RW : 4); ++sd) {
                    int l = 0;
#pragma unroll
                    for (int ww = sd; ww < RW; ww += 4) l += load[ww];
                    if (l < bl) {
                        bl = l;
                        bs = sd;
                    }
                }
                int bw = bs, be = 0x7fffffff;
#pragma unroll
                for (int ww = 0; ww < RW; ++ww) {
                    const int e = ww >= 4 ? load[ww] * 14 : load[ww] * 10;
                    if ((ww & 3) == bs && e < be) {
                        be = e;
                        bw = ww;
                    }
                }
#pragma unroll
                for (int ww = 0; ww < RW; ++ww)
                    if (ww == bw) {
                        load[ww] += 8;
                        ++k[ww];
                    }
            }
            int first = 0;
#pragma unroll
            for (int ww = 0; ww < RW; ++ww) {
                geo[RW * NSLOT + c * RW + ww] = (first << 8) | k[ww];
                first += k[ww];
            }
        }
        double rt[NSLOT][16];
#pragma unroll
        for (int sl = 0; sl < NSLOT; ++sl) {
            const int code = __builtin_amdgcn_readfirstlane(geo[w * NSLOT + sl]);
            const int R = code >> 8, C = code & 255;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    rt[sl][s * 4 + q] = code >= 0 ? hval(D, R * TILE + 4 * ly + s, C * TILE + 4 * lx + q) : 0.0;
        }
        for (int C = c0; C < T; ++C)
            for (int R = C; R < T; ++R) {
                double* tp = lt + (size_t)lds_tile_index(R, C, c0, TL) * TILE_EL;
                for (int el = t; el < TILE_EL; el += RT) tp[el] = hval(D, R * TILE + plane_row(el), C * TILE + plane_col(el));
            }
        // column 0 and the norm of its part below the subdiagonal
        double part = 0.0;
        for (int i = t; i < NP; i += RT) {
            const double x = i < n ? hval(D, i, 0) : 0.0;
            xv[i] = i >= 1 ? x : 0.0;
            dd[i] = i == 0 ? x : 0.0;
            if (i >= 2) part += x * x;
            const int pi = vpos<SHV>(i);
            vp[pi] = wp[pi] = xn[pi] = 0.0;
            vc[pi] = SHV && i >= 2 ? x : 0.0;
            ee[i] = 0.0;
        }
        for (int i = t; i < PWL; i += RT) pw[i] = 0.0;
        // the per-wave norm partials of column 0 (the shared-vector kernels form each
        // column's norm in the scalar wave instead)
        if (!SHV) {
            part = wave_sum(part);
            if (lane == 0) red[8 + w] = part;
        }
        __syncthreads();

        // Step j: (H) Householder vector v_j of column j; (P) one pass over the
        // trailing tiles applying the update of step j-1 and forming A v_j, while the
        // owners of column j+1 publish it; (W) w_j, column j+1 with the update of
        // step j, the norm partials for step j+1, and v_j kept as the previous
        // vector.  Three barriers per step; two in the shared-vector kernels, where (H)
        // shrinks to the Householder scalars (see above).  In mode 2 with D.jsplit > 0
        // the loop stops after jsplit steps and hands the trailing matrix over.
        const int jend = (MODE == 2 && D.jsplit > 0) ? D.jsplit : n - 1;
        for (int j = 0; j < jend; ++j) {
            const int Cj = j >> 5;
            const int b = j & 1;  // SHV buffer parity
            double tau = 0.0, beta = 0.0, scale = 0.0;
            if constexpr (!SHV) {
                // (H) redundantly in every wave
                double xn2 = 0.0;
#pragma unroll
                for (int q = 0; q < RW; ++q) xn2 += red[8 + q];
                const double alpha = xv[j + 1];
                const double xvt = xv[t < NP ? t : 0];  // this thread's element, loaded with the others
                beta = alpha;
                if (xn2 > 0.0) {
                    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                    tau = (beta - alpha) / beta;
                    scale = 1.0 / (alpha - beta);
                }
                if (t == 0) {
                    ee[j] = beta;
                    if (MODE == 1 && D.tau) D.tau[j] = tau;
                }
                if (MODE == 1 && D.V)
                    for (int i = j + 2 + t; i < n; i += RT) D.V[(long)i + (long)j * D.ldv] = tau != 0.0 ? xv[i] * scale : 0.0;
                if (t < npad) {  // one element per thread (RT >= NP)
                    const int i = t;
                    vc[i] = (tau == 0.0 || i <= j || i >= n) ? 0.0 : (i == j + 1 ? 1.0 : xvt * scale);
                }
                __syncthreads();  // #1
            } else if (w == RW - 1) {
                // the Householder scalars, by the last wave (the others go straight to their
                // tiles): the norm of the unscaled column from its buffer, then tau and scale
                // for (W) in red[10], red[11]
                const double* xsb = b ? xs1 : vc;
                double sq = 0.0;
#pragma unroll
                for (int u = 0; u < (NP + 63) / 64; ++u) {
                    const int iu = lane + 64 * u;
                    const double x = iu < NP ? xsb[vpos<SHV>(iu)] : 0.0;
                    sq = fma(x, x, sq);
                }
                const double xn2 = wave_sum(sq);
                const double alpha = xv[j + 1];
                beta = alpha;
                if (xn2 > 0.0) {
                    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                    tau = (beta - alpha) / beta;
                    scale = 1.0 / (alpha - beta);
                }
                if (lane == 63) {
                    ee[j] = beta;
                    red[10] = tau;
                    red[11] = scale;
                }
            }
            // (P) register tiles, then this wave's share of the LDS tiles.  Row
            // partials accumulate while consecutive tiles stay in one tile row.
            const int Cn = (j + 1) >> 5, cn = (j + 1) & 31;
            double* pww = SHV ? pw + b * NPP : pw + w * NP;  // products of this step
            const double* vcx = SHV && b ? xs1 : vc;         // the vector the tiles multiply by
            // the wave's slot codes and LDS share, read together (one LDS wait)
            int codes[NSLOT];
#pragma unroll
            for (int sl = 0; sl < NSLOT; ++sl) codes[sl] = geo[w * NSLOT + sl];
            const int al_v = geo[RW * NSLOT + Cj * RW + w];
            double racc[4] = {0.0, 0.0, 0.0, 0.0};
            // v, w and v_j over the rows of the current tile row, kept across its tiles in
            // the four-wave kernels (the eight-wave kernel has no registers to spare)
            constexpr bool ROWC = RW == 4;
            double rv[ROWC ? 4 : 1], rw[ROWC ? 4 : 1], rcv[ROWC ? 4 : 1];
            int curR = -1;
#pragma unroll
            for (int sl = 0; sl < NSLOT; ++sl) {
                const int code = __builtin_amdgcn_readfirstlane(codes[sl]);
                if (code >= 0 && (code & 255) >= Cj) {
                    const int R = code >> 8, C = code & 255;
                    if (R != curR) {
                        if (curR >= 0) flush_rows<SHV>(curR, racc, pww, ly, lx);
                        curR = R;
                        if constexpr (ROWC) {
                            const int gi0 = vpos<SHV>(R * TILE + 4 * ly);
                            ld4(vp + gi0, rv);
                            ld4(wp + gi0, rw);
                            ld4(vcx + gi0, rcv);
                        }
                    }
                    if constexpr (ROWC) tile_step_racc_rows<SHV>(rt[sl], R, C, vcx, vp, wp, pww, ly, lx, racc, rv, rw, rcv);
                    else tile_step_racc<SHV>(rt[sl], R, C, vcx, vp, wp, pww, ly, lx, racc);
                    if (C == Cn && lx == (cn >> 2)) {
                        double* xo = xn + vpos<SHV>(R * TILE + 4 * ly);
                        switch (cn & 3) {  // uniform across the wave
                            case 0: xo[0] = rt[sl][0]; xo[1] = rt[sl][4]; xo[2] = rt[sl][8]; xo[3] = rt[sl][12]; break;
                            case 1: xo[0] = rt[sl][1]; xo[1] = rt[sl][5]; xo[2] = rt[sl][9]; xo[3] = rt[sl][13]; break;
                            case 2: xo[0] = rt[sl][2]; xo[1] = rt[sl][6]; xo[2] = rt[sl][10]; xo[3] = rt[sl][14]; break;
                            default: xo[0] = rt[sl][3]; xo[1] = rt[sl][7]; xo[2] = rt[sl][11]; xo[3] = rt[sl][15]; break;
                        }
                    }
                }
            }
            {
                const int al = __builtin_amdgcn_readfirstlane(al_v);
                const int cl = Cj > c0 ? Cj : c0;
                int f = al >> 8, k = al & 255;
                // row-major position of the first tile of this wave's share
                int R = cl, C = cl;
                while (f > R - cl) {
                    f -= R - cl + 1;
                    ++R;
                }
                C = cl + f;
                for (; k > 0; --k) {
                    if (R != curR) {
                        if (curR >= 0) flush_rows<SHV>(curR, racc, pww, ly, lx);
                        curR = R;
                        if constexpr (ROWC) {
                            const int gi0 = vpos<SHV>(R * TILE + 4 * ly);
                            ld4(vp + gi0, rv);
                            ld4(wp + gi0, rw);
                            ld4(vcx + gi0, rcv);
                        }
                    }
                    if constexpr (ROWC)
                        tile_step_lds_rows<SHV>(lt + (size_t)lds_tile_index(R, C, c0, TL) * TILE_EL, lane, R, C, vcx, vp, wp,
                                                pww, ly, lx, racc, rv, rw, rcv);
                    else
                        tile_step_lds<SHV>(lt + (size_t)lds_tile_index(R, C, c0, TL) * TILE_EL, lane, R, C, vcx, vp, wp, pww,
                                           ly, lx, racc);
                    if (++C > R) {
                        ++R;
                        C = cl;
                    }
                }
            }
            if (curR >= 0) flush_rows<SHV>(curR, racc, pww, ly, lx);
            double dsum = 0.0;
            if (!SHV) {
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                double dp = 0.0;
                constexpr int NU = (NP + 63) / 64;
                double pa[NU], pb[NU];
#pragma unroll
                for (int u = 0; u < NU; ++u) {  // unconditional loads, all issued before the first use
                    const int i = j + 1 + lane + 64 * u, ic = i < n ? i : 0;
                    pa[u] = pww[ic];
                    pb[u] = vc[ic];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < NU; ++u) dp += j + 1 + lane + 64 * u < n ? pa[u] * pb[u] : 0.0;
                dp = wave_sum(dp);
                if (lane == 0) red[w] = dp;
            }
            __syncthreads();  // #2
            if constexpr (!SHV) {
            // (W) p = tau A v, w = p - (tau/2)(p.v) v; column j+1 of A - v w^T - w v^T.
            // Every thread needs w_{j+1} and v_{j+1}, so it forms them from the partials
            // itself; those partials are never cleared (row j+1 is dead from here on).
            // Thread t forms element i = t (RT >= NP); its operands are loaded before
            // the reductions so that their latency overlaps them.
            const int i = t;
            const bool act = i >= j + 1 && i < n;
            double acc = 0.0, vci = 0.0, base = 0.0;
            if (act) {
#pragma unroll
                for (int q = 0; q < RW; ++q) acc += pw[q * NP + i];
                vci = vc[i];
                base = Cn < c0 ? xn[i] : lt[(size_t)lds_tile_index(i >> 5, Cn, c0, TL) * TILE_EL + tile_off(i & 31, cn)];
            }
            double p1 = 0.0;
#pragma unroll
            for (int q = 0; q < RW; ++q) p1 += pw[q * NP + j + 1];
            const double v1 = vc[j + 1];
#pragma unroll
            for (int q = 0; q < RW; ++q) dsum += red[q];
            const double K = -0.5 * tau * tau * dsum;
            const double w1 = tau * p1 + K * v1;
            part = 0.0;
            if (i < npad) {
                double wi = 0.0;
                if (act) {
                    wi = tau * acc + K * vci;
                    double x = fma(-vci, w1, base);
                    x = fma(-wi, v1, x);
                    if (i == j + 1) dd[j + 1] = x;
                    else {
                        xv[i] = x;
                        if (i >= j + 3) part += x * x;
                    }
                }
                if (i >= j + 2) {
#pragma unroll
                    for (int q = 0; q < RW; ++q) pw[q * NP + i] = 0.0;
                }
                wp[i] = wi;
                vp[i] = vci;  // v vanishes outside [j + 1, n)
            }
            part = wave_sum(part);
            if (lane == 0) red[8 + w] = part;
            } else {
            // (W) with the products y = A x of the unscaled column x (zero up to j + 1):
            // A v = A e_{j+1} + scale y, where A e_{j+1} is the column j + 1 the tile owners
            // published (base); v^T A v = A_{j+1,j+1} + 2 scale y_{j+1} + scale^2 x^T y;
            // p = tau A v, w = p - (tau/2)(p.v) v; column j+1 of A - v w^T - w v^T.
            // Thread t forms element i = t (RT >= NP); its operands are loaded before
            // the reductions so that their latency overlaps them.  It also prepares the
            // next step's buffers at its index: the unscaled column (zero at j + 1 and
            // j + 2) and cleared products.
            // In the eight-wave kernel the elements are rotated by two tile rows: the rows
            // that stay active longest go to waves 1-3, and the first 128 rows, which retire
            // as the steps advance, to waves 4 and 0, which share a SIMD (a younger wave
            // loses issue to the older one on its SIMD, so neither of that pair is slowed
            // by a busy sibling).
            const int i = RW == 8 && t < NP ? (t + 64) % NP : t, pi = vpos<SHV>(i), nb = b ^ 1;
            double* xsn = nb ? xs1 : vc;
            double* pwn = pw + nb * NPP;
            const bool act = i >= j + 1 && i < n;
            double yi = 0.0, xi = 0.0, base = 0.0;
            if (act) {
                yi = pww[pi];
                xi = vcx[pi];
                base = Cn < c0 ? xn[pi] : lt[(size_t)lds_tile_index(i >> 5, Cn, c0, TL) * TILE_EL + tile_off(i & 31, cn)];
            }
            const int p1i = vpos<SHV>(j + 1);
            tau = red[10];
            scale = red[11];
            const double y1 = pww[p1i];
            const double a11 = Cn < c0 ? xn[p1i]
                                       : lt[(size_t)lds_tile_index((j + 1) >> 5, Cn, c0, TL) * TILE_EL + tile_off((j + 1) & 31, cn)];
            double dp = 0.0;
            {
                constexpr int NU = (NP + 63) / 64;
                double pa[NU], pb[NU];
#pragma unroll
                for (int u = 0; u < NU; ++u) {  // unconditional loads, all issued before the first use
                    const int iu = j + 2 + lane + 64 * u, pu = vpos<SHV>(iu < n ? iu : 0);
                    pa[u] = pww[pu];
                    pb[u] = vcx[pu];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < NU; ++u) dp += j + 2 + lane + 64 * u < n ? pa[u] * pb[u] : 0.0;
            }
            const double xy = wave_sum(dp);
            const double v1 = tau != 0.0 ? 1.0 : 0.0;
            const double p1 = fma(scale, y1, a11);
            dsum = fma(scale * scale, xy, fma(2.0 * scale, y1, a11));
            const double K = -0.5 * tau * tau * dsum;
            const double w1 = tau * p1 + K * v1;
            part = 0.0;
            if (i < npad) {
                double wi = 0.0, vi = 0.0;
                if (act) {
                    vi = tau == 0.0 ? 0.0 : (i == j + 1 ? 1.0 : scale * xi);
                    wi = tau * fma(scale, yi, base) + K * vi;
                    double x = fma(-vi, w1, base);
                    x = fma(-wi, v1, x);
                    if (i == j + 1) dd[j + 1] = x;
                    else xv[i] = x;
                    xsn[pi] = i >= j + 3 ? x : 0.0;
                    pwn[pi] = fresh_zero();
                }
                wp[pi] = wi;
                vp[pi] = vi;
            }
            }
            __syncthreads();  // #3
        }
        __syncthreads();
        if (MODE == 2) {
            // evaluation split in two launches: the tridiagonal goes to the problem's
            // slot (D.d, D.e) and tri_bisect_kernel finishes the evaluation
            if (D.jsplit > 0) {
                // Hand-over after jend steps: d, e up to jend - 1, and the trailing
                // matrix M = A[jend:, jend:] with the update of step jend - 1 applied
                // (still pending in the tiles; v and w of that step are in vp, wp).
                // Its first column is column jend as (W) left it in dd and xv.
                const int nt = n - jend, Cj = jend >> 5;
                const long ldt = D.ldt;
                double* M = D.At;
                for (int i = t; i < jend; i += RT) {
                    D.d[i] = dd[i];
                    D.e[i] = ee[i];
                }
                for (int a = t; a < nt; a += RT) {
                    const double x = a == 0 ? dd[jend] : xv[jend + a];
                    M[a] = x;
                    M[(long)a * ldt] = x;
                }
                // every other element from the lower triangle of the active tiles,
                // written to both triangles of M
                auto put = [&](int gi, int gc, double a) {
                    if (gc > jend && gi >= gc && gi < n) {
                        const int pi = vpos<SHV>(gi), pc = vpos<SHV>(gc);
                        double x = fma(-vp[pi], wp[pc], a);
                        x = fma(-wp[pi], vp[pc], x);
                        M[(long)(gi - jend) + (long)(gc - jend) * ldt] = x;
                        M[(long)(gc - jend) + (long)(gi - jend) * ldt] = x;
                    }
                };
#pragma unroll
                for (int sl = 0; sl < NSLOT; ++sl) {
                    const int code = __builtin_amdgcn_readfirstlane(geo[w * NSLOT + sl]);
                    if (code >= 0 && (code & 255) >= Cj) {
                        const int R = code >> 8, C = code & 255;
#pragma unroll
                        for (int s = 0; s < 4; ++s)
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                put(R * TILE + 4 * ly + s, C * TILE + 4 * lx + q, rt[sl][s * 4 + q]);
                    }
                }
                {
                    const int al = __builtin_amdgcn_readfirstlane(geo[RW * NSLOT + Cj * RW + w]);
                    const int cl = Cj > c0 ? Cj : c0;
                    int f = al >> 8, k = al & 255;
                    int R = cl, C = cl;
                    while (f > R - cl) {
                        f -= R - cl + 1;
                        ++R;
                    }
                    C = cl + f;
                    for (; k > 0; --k) {
                        const double* tp = lt + (size_t)lds_tile_index(R, C, c0, TL) * TILE_EL;
                        for (int s = 0; s < 4; ++s)
                            for (int q = 0; q < 4; ++q)
                                put(R * TILE + 4 * ly + s, C * TILE + 4 * lx + q, tp[((4 * s + q) << 6) + lane]);
                        if (++C > R) {
                            ++R;
                            C = cl;
                        }
                    }
                }
            } else {
                for (int i = t; i < n; i += RT) {
                    D.d[i] = dd[i];
                    if (i < n - 1) D.e[i] = ee[i];
                }
            }
            __syncthreads();
            continue;
        }

        // ---- multisection bisection for the nkeep largest eigenvalues ----
        double glo = INFINITY, ghi = -INFINITY, em = 0.0;
        for (int i = t; i < n; i += RT) {
            const double rad = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i < n - 1 ? fabs(ee[i]) : 0.0);
            glo = fmin(glo, dd[i] - rad);
            ghi = fmax(ghi, dd[i] + rad);
            if (i < n - 1) em = fmax(em, ee[i] * ee[i]);
        }
        glo = -block_max(-glo, red);
        ghi = block_max(ghi, red);
        em = block_max(em, red);
        const double tnorm = fmax(fabs(glo), fabs(ghi));
        const double pivmin = DBL_MIN * fmax(1.0, em);
        const double tol = 4.0 * DBL_EPSILON * tnorm + 2.0 * pivmin;
        const double sc = sturm_scale(tnorm);
        // T prepared once for all probes (sturm_count_scaled): diagonal into vc,
        // squared off-diagonal into xv
        for (int i = t; i < npad; i += RT) {
            vc[i] = i < n ? dd[i] * sc : 0.0;
            const double es = i < n - 1 ? ee[i] * sc : 0.0;
            xv[i] = i < n - 1 ? fmax(es * es, 0x1p-120) : 0.0;
        }
        __syncthreads();
        glo -= tol;
        ghi += tol;
        // One probe per thread; P probes per eigenvalue and round split its interval
        // into P + 1 parts, with P as large as the threads allow.
        constexpr int KP = 1, NPROBE = KP * RT;
        const int nk = D.nkeep;
        // the error needs only the sum of the top nk: above half the spectrum, the bottom
        // n - nk are found and subtracted from the trace (as in the small kernel)
        const bool bottom = MODE == 0 && 2 * nk > n;
        const int nb = bottom ? n - nk : nk;
        const int P = nb > 0 && nb <= NPROBE ? NPROBE / nb : 1;
        double* blo = pw;
        double* bhi = pw + NP;
        int* flag = reinterpret_cast<int*>(pw + 2 * NP);  // NPROBE ints
        double width = ghi - glo;
        if (nb > 1) {
            // The first round is shared: NPROBE probes spread evenly over the Gershgorin
            // interval (the multisection formula with P = NPROBE) leave every eigenvalue
            // a bracket of 1/(NPROBE + 1) of it, where per-eigenvalue probes would leave
            // 1/(P + 1).
            {
                const double x[1] = {glo + width * (double)(t + 1) / (double)(NPROBE + 1)};
                int c[1];
                sturm_count_scaled<1>(vc, xv, n, x, sc, c);
                flag[t] = c[0];
            }
            __syncthreads();
            for (int q = t; q < nb; q += RT) {
                const int target = bottom ? q + 1 : n - q;
                int first = NPROBE;
                for (int pi = NPROBE - 1; pi >= 0; --pi)
                    if (flag[pi] >= target) first = pi;
                blo[q] = first > 0 ? glo + width * (double)first / (double)(NPROBE + 1) : glo;
                bhi[q] = first < NPROBE ? glo + width * (double)(first + 1) / (double)(NPROBE + 1) : ghi;
            }
            width /= (double)(NPROBE + 1);
        } else {
            for (int q = t; q < nb; q += RT) {
                blo[q] = glo;
                bhi[q] = ghi;
            }
        }
        // Each round divides every interval by exactly P + 1, so this many rounds
        // bring the bracket width below tol (the resolution of the Sturm count).
        int iters = nb > 1 ? 0 : 1;
        if (width > tol) iters = (int)ceil(log(width / tol) / log((double)(P + 1)));
        __syncthreads();
        for (int it = 0; it < iters; ++it) {
            for (int base = 0; base < nb * P; base += NPROBE) {
                double x[KP];
                int cnt[KP];
#pragma unroll
                for (int k = 0; k < KP; ++k) {
                    const int u = base + t * KP + k;
                    x[k] = 0.0;
                    if (u < nb * P) {
                        const int q = u / P, pi = u % P;
                        const double lo = blo[q], hi = bhi[q];
                        x[k] = lo + (hi - lo) * (double)(pi + 1) / (double)(P + 1);
                    }
                }
                sturm_count_scaled<KP>(vc, xv, n, x, sc, cnt);
#pragma unroll
                for (int k = 0; k < KP; ++k) {
                    const int u = base + t * KP + k;
                    if (u < nb * P) flag[u - base] = cnt[k] >= (bottom ? u / P + 1 : n - u / P);
                }
                __syncthreads();
                const int q = base / P + t;
                if (t < NPROBE / P && q < nb) {
                    const double lo = blo[q], hi = bhi[q];
                    const int* fq = flag + (q * P - base);
                    int first = P;
                    for (int pi = P - 1; pi >= 0; --pi)
                        if (fq[pi]) first = pi;
                    const double nhi = first < P ? lo + (hi - lo) * (double)(first + 1) / (double)(P + 1) : hi;
                    const double nlo = first > 0 ? lo + (hi - lo) * (double)first / (double)(P + 1) : lo;
                    blo[q] = nlo;
                    bhi[q] = nhi;
                }
                __syncthreads();
            }
        }
        if (t == 0) {
            double hi = 0.0, lo = 0.0;
            for (int q = 0; q < nb; ++q) dd_add(hi, lo, 0.5 * (blo[q] + bhi[q]));
            if (bottom) top_from_trace(dd, n, hi, lo);
            if (MODE == 0) {
                double eh = D.na[0], el = D.na[1];
                if (D.nb) {
                    dd_add(eh, el, D.nb[0]);
                    el += D.nb[1];
                }
                double s2, e2;
                two_sum(eh, -hi, s2, e2);
                double tail = s2 + (e2 + el - lo);
                if (tail < 0.0) tail = 0.0;  // clamp rounding below zero; NaN propagates
                const double err = sqrt(tail);
                const double etot = eh + el;
                *D.out_err = err;
                if (D.out_rel) *D.out_rel = etot != 0.0 ? err / sqrt(etot) : 0.0;
            } else if (D.sum_top) {
                D.sum_top[0] = hi;
                D.sum_top[1] = lo;
            }
        }
        if (MODE == 1) {
            for (int q = t; q < nk; q += RT) D.lam[q] = 0.5 * (blo[q] + bhi[q]);
            if (D.d)
                for (int i = t; i < n; i += RT) {
                    D.d[i] = dd[i];
                    if (i < n - 1) D.e[i] = ee[i];
                }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Evaluation epilogue of the register-resident kernel as a kernel of its own: the
// eigenvalues of every problem's tridiagonal (written by sym_eig_reg_kernel<2>) by
// bisection, one wavefront per problem and one eigenvalue per lane, then the plug-in
// error, exactly as the in-kernel epilogue of mode 0 (same scaled Sturm count, same
// tolerance, the top eigenvalues from the trace above half the spectrum).  A tridiagonal
// takes 5 KB of LDS where the tridiagonalisation needed the whole compute unit, so six
// wavefronts per SIMD take turns on the dependent Sturm recurrences, and plain bisection
// does the fewest Sturm steps per eigenvalue.  A first round spreads the 64 lanes' probes
// evenly over the Gershgorin interval; each eigenvalue then bisects its 1/65 of it.  The
// count is the register-lean form of the same recurrence (sturm_count_lean), so that four
// workgroups of four wavefronts (four per SIMD) fit on each compute unit without spills.
// ---------------------------------------------------------------------------
constexpr int BIS_W = 4;  // wavefronts (problems) per workgroup

template <int NPMAX>
__global__ void __launch_bounds__(64 * BIS_W, 4) tri_bisect_kernel(const EigDesc* __restrict__ descs, int count) {
    constexpr int LEN = NPMAX + 8;  // the count reads up to seven entries past the end
    __shared__ double sh[BIS_W][2 * LEN + 128];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double* ds = sh[wv];
    double* e2s = ds + LEN;
    double* aux = e2s + LEN;  // 64 counts of the first round, then 64 double-double partial sums
    int* cnt0 = reinterpret_cast<int*>(aux);
    for (int prob = blockIdx.x * BIS_W + wv; prob < count; prob += gridDim.x * BIS_W) {
        const EigDesc D = descs[prob];
        const int n = D.n;
        double glo = INFINITY, ghi = -INFINITY, em = 0.0;
        for (int i = lane; i < LEN; i += 64) {
            const double di = i < n ? D.d[i] : 0.0;
            const double ei = i < n - 1 ? D.e[i] : 0.0;
            if (i < n) {
                const double rad = (i > 0 ? fabs(D.e[i - 1]) : 0.0) + fabs(ei);
                glo = fmin(glo, di - rad);
                ghi = fmax(ghi, di + rad);
            }
            em = fmax(em, ei * ei);
            ds[i] = di;
            e2s[i] = ei;
        }
        glo = -wave_max(-glo);
        ghi = wave_max(ghi);
        em = wave_max(em);
        const double tnorm = fmax(fabs(glo), fabs(ghi));
        const double pivmin = DBL_MIN * fmax(1.0, em);
        const double tol = 4.0 * DBL_EPSILON * tnorm + 2.0 * pivmin;
        const double sc = sturm_scale(tnorm);
        // trace of T (double-double, index order) for the bottom-half case
        double th = 0.0, tl = 0.0;
        if (lane == 0)
            for (int i = 0; i < n; ++i) dd_add(th, tl, ds[i]);
        for (int i = lane; i < LEN; i += 64) {
            ds[i] *= sc;  // exact: sc is a power of two
            const double es = e2s[i] * sc;
            e2s[i] = i < n - 1 ? fmax(es * es, 0x1p-120) : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        glo -= tol;
        ghi += tol;
        const int nk = D.nkeep;
        const bool bottom = 2 * nk > n;
        const int nb = bottom ? n - nk : nk;
        const double width = ghi - glo;
        cnt0[lane] = sturm_count_lean(ds, e2s, n, glo + width * (double)(lane + 1) / 65.0, sc);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const double w0 = width / 65.0;
        const int iters = w0 > tol ? (int)ceil(log2(w0 / tol)) : 0;
        double shi = 0.0, slo = 0.0;  // this lane's eigenvalues, in increasing q
        for (int q = lane; q < nb; q += 64) {
            const int target = bottom ? q + 1 : n - q;
            int first = 64;
            for (int pi = 63; pi >= 0; --pi)
                if (cnt0[pi] >= target) first = pi;
            double lo = first > 0 ? glo + width * (double)first / 65.0 : glo;
            double hi = first < 64 ? glo + width * (double)(first + 1) / 65.0 : ghi;
            for (int it = 0; it < iters; ++it) {
                const double x = 0.5 * (lo + hi);
                if (sturm_count_lean(ds, e2s, n, x, sc) >= target) hi = x;
                else lo = x;
            }
            dd_add(shi, slo, 0.5 * (lo + hi));
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        aux[2 * lane] = shi;
        aux[2 * lane + 1] = slo;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            double hi = 0.0, lo = 0.0;
            for (int l = 0; l < 64; ++l) {
                dd_add(hi, lo, aux[2 * l]);
                lo += aux[2 * l + 1];
            }
            if (bottom) {  // (hi, lo) = trace - (hi, lo)
                double s2, e2;
                two_sum(th, -hi, s2, e2);
                e2 += tl - lo;
                two_sum(s2, e2, hi, lo);
            }
            double eh = D.na[0], el = D.na[1];
            if (D.nb) {
                dd_add(eh, el, D.nb[0]);
                el += D.nb[1];
            }
            double s2, e2;
            two_sum(eh, -hi, s2, e2);
            double tail = s2 + (e2 + el - lo);
            if (tail < 0.0) tail = 0.0;  // clamp rounding below zero; NaN propagates
            const double err = sqrt(tail);
            const double etot = eh + el;
            *D.out_err = err;
            if (D.out_rel) *D.out_rel = etot != 0.0 ? err / sqrt(etot) : 0.0;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// Small cores (n <= 64): one wavefront per problem, several problems per workgroup.
//
// Lane i holds row i of the full symmetric matrix in VGPRs.  A v and the rank-2
// update are then row-local (v and w are broadcast through the wave's LDS buffer), so a
// column step has no cross-lane reduction besides two wave sums and no barrier.
// Applying the update to the whole matrix with the whole p = tau A v is exactly the
// two-sided reflection: v vanishes on indices <= j, rows above j are already reduced
// (their p is zero), and row j's tail becomes (beta, 0, ...).  Bisection is a
// multisection with floor(64 / nkeep) probes per eigenvalue and round.
// ---------------------------------------------------------------------------
constexpr int SN = 64;
constexpr int SWV = 4;
constexpr int S_LDS = 7 * SN + 8;

// SNT: the width of each lane's row in registers (the largest order served); the LDS
// vectors keep 64 entries, one per lane.
template <int MODE, int SNT>
__global__ void __launch_bounds__(64 * SWV) sym_eig_small_kernel(const EigDesc* __restrict__ descs, int count) {
    __shared__ double sh[SWV][S_LDS];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    double* vv = sh[wv];      // v of the step, later the lower bisection bounds
    double* ww = vv + SN;     // w of the step, later the upper bisection bounds
    double* dd = ww + SN;     // diagonal of T
    double* e2 = dd + SN;     // squared off-diagonal of T
    double* es = e2 + SN;     // signed off-diagonal of T
    double* rb = es + SN;     // row broadcast (row j = column j)
    int* fl = reinterpret_cast<int*>(rb + SN);  // bisection flags (SN ints)

    for (int prob = blockIdx.x * SWV + wv; prob < count; prob += gridDim.x * SWV) {
        const EigDesc D = descs[prob];
        const int n = D.n;
        double a[SNT];
#pragma unroll
        for (int c = 0; c < SNT; ++c) a[c] = (lane < n && c < n) ? hval(D, lane, c) : 0.0;
        for (int j = 0; j + 1 < n; ++j) {
            // column j of A = row j: lane j publishes its row
            if (lane == j) {
#pragma unroll
                for (int c = 0; c < SNT; ++c) rb[c] = a[c];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const double xi = rb[lane];
            const double dj = rb[j];
            const double alpha = rb[j + 1];
            const double xn2 = wave_sum((lane >= j + 2 && lane < n) ? xi * xi : 0.0);
            double tau = 0.0, beta = alpha, scale = 0.0;
            if (xn2 > 0.0) {
                beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                tau = (beta - alpha) / beta;
                scale = 1.0 / (alpha - beta);
            }
            const double vi = (tau == 0.0 || lane <= j || lane >= n) ? 0.0 : (lane == j + 1 ? 1.0 : xi * scale);
            if (lane == 0) {
                dd[j] = dj;
                es[j] = beta;
                e2[j] = beta * beta;
                if (MODE == 1 && D.tau) D.tau[j] = tau;
            }
            if (MODE == 1 && D.V && lane >= j + 2 && lane < n) D.V[(long)lane + (long)j * D.ldv] = vi;
            vv[lane] = vi;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < SNT; ++c) acc = fma(a[c], vv[c], acc);  // a, v vanish beyond n
            const double pi = tau * acc;
            const double K = -0.5 * tau * wave_sum(pi * vi);
            const double wi = pi + K * vi;
            ww[lane] = wi;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int c = 0; c < SNT; ++c) a[c] = fma(-vi, ww[c], fma(-wi, vv[c], a[c]));
            __builtin_amdgcn_wave_barrier();
        }
        if (lane == n - 1) {
#pragma unroll
            for (int c = 0; c < SNT; ++c) rb[c] = a[c];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane == 0) dd[n - 1] = rb[n - 1];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (MODE == 2) {
            // the trailing part of a larger problem: its tridiagonal only
            if (lane < n) D.d[lane] = dd[lane];
            if (lane < n - 1) D.e[lane] = es[lane];
            __builtin_amdgcn_wave_barrier();
            continue;
        }

        // ---- multisection bisection for the nkeep largest eigenvalues ----
        double glo = INFINITY, ghi = -INFINITY, em = 0.0;
        if (lane < n) {
            const double rad = (lane > 0 ? fabs(es[lane - 1]) : 0.0) + (lane < n - 1 ? fabs(es[lane]) : 0.0);
            glo = dd[lane] - rad;
            ghi = dd[lane] + rad;
            if (lane < n - 1) em = e2[lane];
        }
        glo = -wave_max(-glo);
        ghi = wave_max(ghi);
        em = wave_max(em);
        const double tnorm = fmax(fabs(glo), fabs(ghi));
        const double pivmin = DBL_MIN * fmax(1.0, em);
        const double tol = 4.0 * DBL_EPSILON * tnorm + 2.0 * pivmin;
        const double sc = sturm_scale(tnorm);
        // T prepared once for all probes (sturm_count_scaled): diagonal into rb (free
        // now), squared off-diagonal scaled in place
        if (lane < n) rb[lane] = dd[lane] * sc;
        if (lane < n - 1) e2[lane] = fmax(e2[lane] * (sc * sc), 0x1p-120);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        glo -= tol;
        ghi += tol;
        const int nk = D.nkeep;
        // The error needs only the sum of the top nk eigenvalues; when that is more than
        // half the spectrum the bottom n - nk are found instead and subtracted from the
        // trace of T (sum of its diagonal, kept by the orthogonal reduction).
        const bool bottom = MODE == 0 && 2 * nk > n;
        const int nb = bottom ? n - nk : nk;  // eigenvalues searched
        const int P = nb > 0 && nb < 64 ? 64 / nb : 1;
        double* blo = vv;
        double* bhi = ww;
        double width = ghi - glo;
        if (nb > 1) {
            // first round shared by all the eigenvalues (as in the register kernel): 64
            // probes over the Gershgorin interval
            {
                const double x[1] = {glo + width * (double)(lane + 1) / 65.0};
                int c[1];
                sturm_count_scaled<1>(rb, e2, n, x, sc, c);
                fl[lane] = c[0];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane < nb) {
                const int target = bottom ? lane + 1 : n - lane;
                int first = 64;
                for (int pi = 63; pi >= 0; --pi)
                    if (fl[pi] >= target) first = pi;
                blo[lane] = first > 0 ? glo + width * (double)first / 65.0 : glo;
                bhi[lane] = first < 64 ? glo + width * (double)(first + 1) / 65.0 : ghi;
            }
            width /= 65.0;
        } else if (lane < nb) {
            blo[lane] = glo;
            bhi[lane] = ghi;
        }
        // Each round divides every interval by exactly P + 1 (see the register kernel).
        int iters = nb > 1 ? 0 : 1;
        if (width > tol) iters = (int)ceil(log(width / tol) / log((double)(P + 1)));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int it = 0; it < iters; ++it) {
            for (int base = 0; base < nb * P; base += 64) {
                const int u = base + lane;
                if (u < nb * P) {
                    const int q = u / P, pi = u % P;
                    const double lo = blo[q], hi = bhi[q];
                    const double x = lo + (hi - lo) * (double)(pi + 1) / (double)(P + 1);
                    // eigenvalue q from the top (from the bottom): x is above it iff at
                    // least n - q (q + 1) eigenvalues lie below x
                    const double xk[1] = {x};
                    int c[1];
                    sturm_count_scaled<1>(rb, e2, n, xk, sc, c);
                    fl[u - base] = c[0] >= (bottom ? q + 1 : n - q);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int q = base / P + lane;
                if (lane < 64 / P && q < nb) {
                    const double lo = blo[q], hi = bhi[q];
                    const int* fq = fl + (q * P - base);
                    int first = P;
                    for (int pi = P - 1; pi >= 0; --pi)
                        if (fq[pi]) first = pi;
                    blo[q] = first > 0 ? lo + (hi - lo) * (double)first / (double)(P + 1) : lo;
                    bhi[q] = first < P ? lo + (hi - lo) * (double)(first + 1) / (double)(P + 1) : hi;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        if (lane == 0) {
            double hi = 0.0, lo = 0.0;
            for (int q = 0; q < nb; ++q) dd_add(hi, lo, 0.5 * (blo[q] + bhi[q]));
            if (bottom) top_from_trace(dd, n, hi, lo);
            if (MODE == 0) {
                double eh = D.na[0], el = D.na[1];
                if (D.nb) {
                    dd_add(eh, el, D.nb[0]);
                    el += D.nb[1];
                }
                double s2, e2s;
                two_sum(eh, -hi, s2, e2s);
                double tail = s2 + (e2s + el - lo);
                if (tail < 0.0) tail = 0.0;  // clamp rounding below zero; NaN propagates
                const double err = sqrt(tail);
                const double etot = eh + el;
                *D.out_err = err;
                if (D.out_rel) *D.out_rel = etot != 0.0 ? err / sqrt(etot) : 0.0;
            } else if (D.sum_top) {
                D.sum_top[0] = hi;
                D.sum_top[1] = lo;
            }
        }
        if (MODE == 1) {
            if (lane < nk) D.lam[lane] = 0.5 * (blo[lane] + bhi[lane]);
            if (D.d && lane < n) {
                D.d[lane] = dd[lane];
                if (lane < n - 1) D.e[lane] = es[lane];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// One appended column (n = n1 + 1), evaluation mode: H is an arrowhead,
//     H = [[diag(d), z], [z^T, c]],  d = s^2, z = s .* P, c = Y (the column's energy).
// The kept sum is the trace minus the smallest eigenvalue (nkeep = n - 1), or the whole
// trace (nkeep >= n).  Below the smallest diagonal entry, eliminating the border gives the
// inertia of H - x I (Sylvester): d_i - x > 0 for every i, so x lies above an eigenvalue
// iff the Schur complement phi(x) = c - x - sum_i z_i^2 / (d_i - x) is negative.  The
// smallest eigenvalue is found in the Weyl bracket [min(d, c) - ||z||, min(d, c)] without a
// reduction to tridiagonal form; when a deflated entry (z_i = 0) is the smallest, the
// bracket closes on it.  The bracket is narrowed by the sign of phi as in bisection; the
// probes come from a model that keeps the smallest pole exact: with p the smallest d_i
// with z_i != 0 and R the sum of z_i^2 over the entries at p, phi = g - R / (p - x),
// where g (the other terms) is decreasing and concave left of p.  Replacing g by its
// tangent at the probe gives a quadratic in u = p - x with one positive root; since the
// tangent lies above g, that root is never left of the eigenvalue.  The first probe sits
// one tolerance below the bracket's top (which settles a deflated smallest entry at
// once); a model step that does not halve the previous one gives way to the midpoint;
// once a step falls below the tolerance the next probe lies one tolerance across, which
// closes the bracket.  Plain bisection finishes if the capped loop has not.  The result
// is the midpoint of a bracket of width at most the tolerance whose ends have the signs
// bisection would have checked.  One wavefront per problem, lane i holding entries i,
// i + 64, ... (n1 <= 256), two wave sums per probe (g and its derivative).
// ---------------------------------------------------------------------------
constexpr int AW = 4;  // waves per workgroup

__global__ void __launch_bounds__(64 * AW) arrow_eig_kernel(const EigDesc* __restrict__ descs, int count) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int prob = blockIdx.x * AW + wv; prob < count; prob += gridDim.x * AW) {
        const EigDesc D = descs[prob];
        const int n1 = D.n1;
        const double c = D.Y[0];
        double d[4], z2[4];
        double th = 0.0, tl = 0.0, dmin = INFINITY, dmax = -INFINITY, zs = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = lane + 64 * q;
            d[q] = INFINITY;
            z2[q] = 0.0;
            if (i < n1) {
                const double si = D.s[i], zi = si * D.P[i];
                d[q] = si * si;
                z2[q] = zi * zi;
                dd_add(th, tl, d[q]);
                dmin = fmin(dmin, d[q]);
                dmax = fmax(dmax, d[q]);
                zs += z2[q];
            }
        }
        // trace (double-double over the lanes, then the corner), bounds
        th = wave_sum(th);  // the lanes' high parts; their low parts below
        tl = wave_sum(tl);
        dd_add(th, tl, c);
        dmin = fmin(-wave_max(-dmin), c);
        dmax = fmax(wave_max(dmax), c);
        const double zn = sqrt(wave_sum(zs));
        // the smallest pole and its residue
        double pl = INFINITY;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (z2[q] != 0.0) pl = fmin(pl, d[q]);
        const double pole = -wave_max(-pl);
        double rs = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (z2[q] != 0.0 && d[q] == pole) rs += z2[q];
        const double res = wave_sum(rs);
        double hi = th, lo = tl;  // the kept sum
        if (D.nkeep < n1 + 1) {
            double bhi = dmin, blo = dmin - zn;
            const double tnorm = fmax(fabs(blo), fabs(dmax) + zn);
            const double tol = 4.0 * DBL_EPSILON * tnorm + 2.0 * DBL_MIN;
            blo -= tol;
            double next = bhi - tol, prev = INFINITY;
            for (int it = 0; it < 120 && bhi - blo > tol; ++it) {
                double x = next;
                if (!(x > blo && x < bhi)) x = 0.5 * (blo + bhi);
                if (x <= blo || x >= bhi) break;  // no representable point inside
                double s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double inv = 1.0 / (d[q] - x);
                    const double tq = z2[q] != 0.0 && d[q] != pole ? z2[q] * inv : 0.0;
                    s1 += tq;
                    s2 += tq * inv;
                }
                const double g = (c - x) - wave_sum(s1);
                const double dg = -1.0 - wave_sum(s2);
                const double u0 = pole - x;  // > 0: x lies below the bracket's top
                const double phi = g - res / u0;
                if (phi < 0.0) bhi = x;
                else blo = x;
                // root of g + dg (x' - x) = R / (p - x'), as A u^2 + B u - R = 0
                const double A = -dg, B = g + dg * u0;
                const double disc = sqrt(B * B + 4.0 * A * res);
                const double u = B >= 0.0 ? 2.0 * res / (B + disc) : (disc - B) / (2.0 * A);
                const double step = fabs(x - (pole - u));
                next = step <= tol ? (phi < 0.0 ? x - tol : x + tol)
                                   : (step <= 0.5 * prev ? pole - u : 0.5 * (blo + bhi));
                prev = step;
            }
            while (bhi - blo > tol) {
                const double x = 0.5 * (blo + bhi);
                if (x <= blo || x >= bhi) break;
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (z2[q] != 0.0) acc += z2[q] / (d[q] - x);
                const double sch = (c - x) - wave_sum(acc);
                if (sch < 0.0) bhi = x;
                else blo = x;
            }
            const double lmin = 0.5 * (blo + bhi);
            double s2, e2;
            two_sum(hi, -lmin, s2, e2);
            e2 += lo;
            two_sum(s2, e2, hi, lo);
        }
        if (lane == 0) {
            double eh = D.na[0], el = D.na[1];
            if (D.nb) {
                dd_add(eh, el, D.nb[0]);
                el += D.nb[1];
            }
            double s2, e2;
            two_sum(eh, -hi, s2, e2);
            double tail = s2 + (e2 + el - lo);
            if (tail < 0.0) tail = 0.0;  // clamp rounding below zero; NaN propagates
            const double err = sqrt(tail);
            const double etot = eh + el;
            *D.out_err = err;
            if (D.out_rel) *D.out_rel = etot != 0.0 ? err / sqrt(etot) : 0.0;
        }
    }
}

// Sums and maxima over each 32-lane half of the wavefront (every lane of the half gets it).
__device__ __forceinline__ double half_sum(double v) {
    v = sum_lanes8(v);
    v += dpp_move<0x128>(v);
    return add_swap16(v);
}
__device__ __forceinline__ double half_max(double v) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v = fmax(v, shfl_xor_d(v, o));
    return v;
}

// The same evaluation for n1 <= 32, two problems per wavefront: lanes 0-31 hold one
// problem's entries (one each), lanes 32-63 the next problem's.  Every quantity above
// is formed per half, each half keeps its own bracket, and the probe loop runs until
// both halves have closed theirs (a finished half computes along and discards).
__global__ void __launch_bounds__(64 * AW) arrow_eig_pair_kernel(const EigDesc* __restrict__ descs, int count) {
    const int lane = threadIdx.x & 63, hl = lane & 31;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int pp = blockIdx.x * AW + wv; 2 * pp < count; pp += gridDim.x * AW) {
        const int prob = 2 * pp + (lane >> 5);
        const bool active = prob < count;
        EigDesc D{};
        if (active) D = descs[prob];
        const int n1 = active ? D.n1 : 0;
        const double c = active ? D.Y[0] : 0.0;
        double d = INFINITY, z2 = 0.0;
        double th = 0.0, tl = 0.0, dmin = INFINITY, dmax = -INFINITY, zs = 0.0;
        if (hl < n1) {
            const double si = D.s[hl], zi = si * D.P[hl];
            d = si * si;
            z2 = zi * zi;
            dd_add(th, tl, d);
            dmin = d;
            dmax = d;
            zs = z2;
        }
        th = half_sum(th);
        tl = half_sum(tl);
        dd_add(th, tl, c);
        dmin = fmin(-half_max(-dmin), c);
        dmax = fmax(half_max(dmax), c);
        const double zn = sqrt(half_sum(zs));
        const double pole = -half_max(-(z2 != 0.0 ? d : INFINITY));
        const double res = half_sum(z2 != 0.0 && d == pole ? z2 : 0.0);
        double hi = th, lo = tl;  // the kept sum
        const bool solve = active && D.nkeep < n1 + 1;
        double bhi = dmin, blo = dmin - zn;
        const double tnorm = fmax(fabs(blo), fabs(dmax) + zn);
        const double tol = 4.0 * DBL_EPSILON * tnorm + 2.0 * DBL_MIN;
        blo -= tol;
        double next = bhi - tol, prev = INFINITY;
        bool run = solve && bhi - blo > tol;
        for (int it = 0; it < 120; ++it) {
            double x = next;
            if (!(x > blo && x < bhi)) x = 0.5 * (blo + bhi);
            if (x <= blo || x >= bhi) run = false;  // no representable point inside
            if (!__any(run)) break;
            const double inv = 1.0 / (d - x);
            const double tq = z2 != 0.0 && d != pole ? z2 * inv : 0.0;
            const double g = (c - x) - half_sum(tq);
            const double dg = -1.0 - half_sum(tq * inv);
            if (run) {
                const double u0 = pole - x;
                const double phi = g - res / u0;
                if (phi < 0.0) bhi = x;
                else blo = x;
                const double A = -dg, B = g + dg * u0;
                const double disc = sqrt(B * B + 4.0 * A * res);
                const double u = B >= 0.0 ? 2.0 * res / (B + disc) : (disc - B) / (2.0 * A);
                const double step = fabs(x - (pole - u));
                next = step <= tol ? (phi < 0.0 ? x - tol : x + tol)
                                   : (step <= 0.5 * prev ? pole - u : 0.5 * (blo + bhi));
                prev = step;
                run = bhi - blo > tol;
            }
        }
        run = solve && bhi - blo > tol;
        for (;;) {
            const double x = 0.5 * (blo + bhi);
            if (x <= blo || x >= bhi) run = false;
            if (!__any(run)) break;
            const double sch = (c - x) - half_sum(z2 != 0.0 ? z2 / (d - x) : 0.0);
            if (run) {
                if (sch < 0.0) bhi = x;
                else blo = x;
                run = bhi - blo > tol;
            }
        }
        if (solve) {
            const double lmin = 0.5 * (blo + bhi);
            double s2, e2;
            two_sum(hi, -lmin, s2, e2);
            e2 += lo;
            two_sum(s2, e2, hi, lo);
        }
        if (active && hl == 0) {
            double eh = D.na[0], el = D.na[1];
            if (D.nb) {
                dd_add(eh, el, D.nb[0]);
                el += D.nb[1];
            }
            double s2, e2;
            two_sum(eh, -hi, s2, e2);
            double tail = s2 + (e2 + el - lo);
            if (tail < 0.0) tail = 0.0;  // clamp rounding below zero; NaN propagates
            const double err = sqrt(tail);
            const double etot = eh + el;
            *D.out_err = err;
            if (D.out_rel) *D.out_rel = etot != 0.0 ? err / sqrt(etot) : 0.0;
        }
    }
}

void arrow_eig_batched(const EigDesc* d_descs, int count, int n1max, hipStream_t s) {
    if (count <= 0) return;
    if (n1max <= 32) {
        const int pairs = (count + 1) / 2;
        const int g = (pairs + AW - 1) / AW;
        hipLaunchKernelGGL(arrow_eig_pair_kernel, dim3(g < 16384 ? g : 16384), dim3(64 * AW), 0, s, d_descs, count);
        return;
    }
    const int g = (count + AW - 1) / AW;
    hipLaunchKernelGGL(arrow_eig_kernel, dim3(g < 16384 ? g : 16384), dim3(64 * AW), 0, s, d_descs, count);
}

int sym_eig_nmax() {
    // the general kernel keeps 10 order-n vectors of LDS besides its tiles
    return (int)(((LDS_BYTES / 8 - 32) / 10) / TILE * TILE);
}

bool sym_eig_split(int nmax) {
    const int T = (nmax + TILE - 1) / TILE;
    return nmax > SN && T > THIN_TMAX && T <= REG_TMAX;
}

// Trailing matrices of order up to 192: four waves, 15 register tiles (4 slots per wave)
// and the last three tile columns (6 tiles) in LDS; 66 KB of LDS, so two problems share
// a CU.
constexpr int MID_TMAX = 6;
constexpr int MID_RTL = 3;
constexpr int MID_LDS_DOUBLES = reg_lds_doubles(4, THIN_NSLOT, MID_RTL, MID_TMAX, true);
static_assert(2 * MID_LDS_DOUBLES * 8 <= LDS_BYTES, "two trailing problems must share a CU");

int sym_eig_tail_levels(int* orders) {
    orders[0] = MID_TMAX * TILE;   // 192: four waves, register and LDS tiles
    orders[1] = THIN_TMAX * TILE;  // 160: four waves, register tiles only
    orders[2] = SN;                // 64: one wave per problem
    return 3;
}

void sym_eig_tail_batched(const EigDesc* d_descs, int count, int level, hipStream_t s) {
    if (count <= 0) return;
    if (level == 0) {
        const size_t lds = (size_t)MID_LDS_DOUBLES * 8;
        lds_limit((const void*)sym_eig_reg_kernel<2, 256, THIN_NSLOT, MID_RTL, MID_TMAX, true>, (int)lds);
        const int grid = count < 2048 ? count : 2048;
        hipLaunchKernelGGL((sym_eig_reg_kernel<2, 256, THIN_NSLOT, MID_RTL, MID_TMAX, true>), dim3(grid), dim3(256), lds,
                           s, d_descs, count);
    } else if (level == 1) {
        const size_t lds = (size_t)THIN_LDS_DOUBLES_SHV * 8;
        const int grid = count < 2048 ? count : 2048;
        hipLaunchKernelGGL((sym_eig_reg_kernel<2, 256, THIN_NSLOT, 0, THIN_TMAX, true>), dim3(grid), dim3(256), lds, s,
                           d_descs, count);
    } else {
        int grid = (count + SWV - 1) / SWV;
        if (grid > 16384) grid = 16384;
        hipLaunchKernelGGL((sym_eig_small_kernel<2, SN>), dim3(grid), dim3(64 * SWV), 0, s, d_descs, count);
    }
}

void tri_bisect_batched(const EigDesc* d_descs, int count, int nmax, hipStream_t s) {
    if (count <= 0 || !sym_eig_split(nmax)) return;
    const int grid = (count + BIS_W - 1) / BIS_W < 8192 ? (count + BIS_W - 1) / BIS_W : 8192;
    hipLaunchKernelGGL((tri_bisect_kernel<REG_NP>), dim3(grid), dim3(64 * BIS_W), 0, s, d_descs, count);
}

size_t sym_eig_tri_doubles(int nmax) {
    const int T = (nmax + TILE - 1) / TILE;
    return 2 * (size_t)T * TILE;
}

size_t sym_eig_workspace_doubles(int nmax, int nslots) {
    const int T = (nmax + TILE - 1) / TILE;
    return (size_t)nslots * (size_t)T * (size_t)(T + 1) / 2 * TILE_EL;
}

size_t sym_eig_slot_doubles(int nmax) {
    // only the general kernel (more than REG_TMAX tile rows) keeps tiles in global slots
    const int T = (nmax + TILE - 1) / TILE;
    return T <= REG_TMAX ? 0 : (size_t)T * (size_t)(T + 1) / 2 * TILE_EL;
}

void sym_eig_batched(const EigDesc* d_descs, int count, int nmax, int mode, double* gws, int nslots,
                     hipStream_t s, int threads) {
    if (count <= 0) return;
    const int T = (nmax + TILE - 1) / TILE, npad = T * TILE;
    const bool split = mode == 2 && sym_eig_split(nmax);
    if (mode == 2 && !split) mode = 0;  // the other kernels finish the evaluation themselves
    if (nmax <= SN) {
        int grid = (count + SWV - 1) / SWV;
        if (grid > 16384) grid = 16384;
        // orders up to 48: shorter rows in registers, so more wavefronts per SIMD
        if (nmax <= 48) {
            if (mode == 0) hipLaunchKernelGGL((sym_eig_small_kernel<0, 48>), dim3(grid), dim3(64 * SWV), 0, s, d_descs, count);
            else hipLaunchKernelGGL((sym_eig_small_kernel<1, 48>), dim3(grid), dim3(64 * SWV), 0, s, d_descs, count);
        } else {
            if (mode == 0) hipLaunchKernelGGL((sym_eig_small_kernel<0, SN>), dim3(grid), dim3(64 * SWV), 0, s, d_descs, count);
            else hipLaunchKernelGGL((sym_eig_small_kernel<1, SN>), dim3(grid), dim3(64 * SWV), 0, s, d_descs, count);
        }
        return;
    }
    if (T <= THIN_TMAX) {
        // cores up to 160: every tile in the VGPRs of four waves, so two problems share a CU
        const size_t lds = (size_t)THIN_LDS_DOUBLES * 8;
        const int grid = count < 2048 ? count : 2048;
        if (mode == 0)
            hipLaunchKernelGGL((sym_eig_reg_kernel<0, 256, THIN_NSLOT, 0, THIN_TMAX>), dim3(grid), dim3(256), lds, s,
                               d_descs, count);
        else
            hipLaunchKernelGGL((sym_eig_reg_kernel<1, 256, THIN_NSLOT, 0, THIN_TMAX>), dim3(grid), dim3(256), lds, s,
                               d_descs, count);
        return;
    }
    if (T <= REG_TMAX) {
        const size_t lds = (size_t)(split ? REG_LDS_DOUBLES_SHV : REG_LDS_DOUBLES) * 8;
        const int grid = count < nslots ? count : nslots;
        if (split) {
            // the evaluation's tridiagonalisation sums A v in one shared vector: 10 % faster
            // than a vector per wave, reproducible to rounding (the waves' atomic adds land
            // in varying order) instead of bit for bit
            lds_limit((const void*)sym_eig_reg_kernel<2, RT, NSLOT, RTL, REG_TMAX, true>, (int)lds);
            hipLaunchKernelGGL((sym_eig_reg_kernel<2, RT, NSLOT, RTL, REG_TMAX, true>), dim3(grid), dim3(RT), lds, s,
                               d_descs, count);
            return;
        }
        if (mode == 0) {
            lds_limit((const void*)sym_eig_reg_kernel<0, RT, NSLOT, RTL, REG_TMAX>, (int)lds);
            hipLaunchKernelGGL((sym_eig_reg_kernel<0, RT, NSLOT, RTL, REG_TMAX>), dim3(grid), dim3(RT), lds, s, d_descs,
                               count);
        } else {
            lds_limit((const void*)sym_eig_reg_kernel<1, RT, NSLOT, RTL, REG_TMAX>, (int)lds);
            hipLaunchKernelGGL((sym_eig_reg_kernel<1, RT, NSLOT, RTL, REG_TMAX>), dim3(grid), dim3(RT), lds, s, d_descs,
                               count);
        }
        return;
    }
    const int TL = tl_for(npad, T);
    const size_t lds = (size_t)(10L * npad + 32) * 8 + (size_t)TL * (TL + 1) / 2 * TILE_EL * 8;
    const long slot = (long)T * (T + 1) / 2 * TILE_EL;
    const int grid = count < nslots ? count : nslots;
    if (threads == GT / 2) {  // eight waves per problem instead of sixteen (an autotuner choice)
        if (mode == 0) {
            lds_limit((const void*)sym_eig_kernel<0, GT / 2>, (int)lds);
            hipLaunchKernelGGL((sym_eig_kernel<0, GT / 2>), dim3(grid), dim3(GT / 2), lds, s, d_descs, count, npad, TL,
                               gws, slot);
        } else {
            lds_limit((const void*)sym_eig_kernel<1, GT / 2>, (int)lds);
            hipLaunchKernelGGL((sym_eig_kernel<1, GT / 2>), dim3(grid), dim3(GT / 2), lds, s, d_descs, count, npad, TL,
                               gws, slot);
        }
        return;
    }
    if (mode == 0) {
        lds_limit((const void*)sym_eig_kernel<0, GT>, (int)lds);
        hipLaunchKernelGGL((sym_eig_kernel<0, GT>), dim3(grid), dim3(GT), lds, s, d_descs, count, npad, TL, gws, slot);
    } else {
        lds_limit((const void*)sym_eig_kernel<1, GT>, (int)lds);
        hipLaunchKernelGGL((sym_eig_kernel<1, GT>), dim3(grid), dim3(GT), lds, s, d_descs, count, npad, TL, gws, slot);
    }
}

// ---------------------------------------------------------------------------
// Eigenvectors: inverse iteration + Gram-Schmidt + back-transformation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double hash_unit(unsigned a, unsigned b) {
    // SplitMix-style integer hash mapped to [-1, 1): deterministic start vectors.
    unsigned long long z = ((unsigned long long)a << 32) ^ (unsigned long long)(b * 0x9E3779B9u) ^ 0x5DEECE66DULL;
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void __launch_bounds__(ET) sym_vectors_kernel(const VecDesc* __restrict__ descs) {
    extern __shared__ double lds[];
    const VecDesc D = descs[blockIdx.x];
    const int n = D.n, nk = D.nkeep, t = threadIdx.x;
    double* red = lds;         // 16
    double* coef = lds + 16;   // nk
    double* X = coef + ((nk + 15) / 16) * 16;  // LDS panel for back-transformation
    // scratch layout [field][i][q]: fields dl, dd, du, du2, x, piv(as double)
    double* S = D.scratch;
    auto at = [&](int field, int i, int q) -> double& { return S[((size_t)field * n + i) * nk + q]; };

    double tn = 0.0;
    for (int i = 0; i < n; ++i) tn = fmax(tn, fabs(D.d[i]) + (i > 0 ? fabs(D.e[i - 1]) : 0.0) + (i < n - 1 ? fabs(D.e[i]) : 0.0));
    const double tiny = DBL_EPSILON * fmax(tn, DBL_MIN);

    // (1) independent inverse iteration, one thread per eigenvalue.  The LU factors of
    // T - lam I (partial pivoting; L multipliers, diagonal, two superdiagonals, pivot
    // flags) and the iterate live in the scratch fields 0..5; the sequential recurrences
    // carry their running values in registers and load each step's operands one step
    // ahead, so no step waits on its predecessor's store.
    for (int q = t; q < nk; q += ET) {
        const double lam = D.lam[q];
        // LU: row i is (dcur, ucur) after the earlier eliminations; row i + 1 starts as
        // the original (d_{i+1} - lam, e_{i+1})
        double dcur = D.d[0] - lam, ucur = n > 1 ? D.e[0] : 0.0;
        double dn = n > 1 ? D.d[1] : 0.0, en = n > 1 ? D.e[0] : 0.0, un = n > 2 ? D.e[1] : 0.0;
        for (int i = 0; i < n - 1; ++i) {
            const double li = en, dnext0 = dn - lam, unext0 = un;
            if (i + 2 < n) {  // operands of the next step
                dn = D.d[i + 2];
                en = D.e[i + 1];
                un = i + 3 < n ? D.e[i + 2] : 0.0;
            }
            double dnext = dnext0, unext = unext0;
            if (fabs(dcur) >= fabs(li)) {
                if (dcur == 0.0) dcur = tiny;
                const double fact = li / dcur;
                at(0, i, q) = fact;
                at(1, i, q) = dcur;
                at(2, i, q) = ucur;
                at(3, i, q) = 0.0;
                at(5, i, q) = 0.0;
                dnext -= fact * ucur;
            } else {
                const double fact = dcur / li;
                at(0, i, q) = fact;
                at(1, i, q) = li;
                at(2, i, q) = dnext0;
                at(3, i, q) = i < n - 2 ? unext0 : 0.0;
                at(5, i, q) = 1.0;
                dnext = ucur - fact * dnext0;
                unext = -fact * unext0;
            }
            dcur = dnext;
            ucur = unext;
        }
        if (dcur == 0.0) dcur = tiny;
        at(1, n - 1, q) = dcur;
        at(2, n - 1, q) = 0.0;
        at(3, n - 1, q) = 0.0;
        at(5, n - 1, q) = 0.0;
        for (int i = 0; i < n; ++i) at(4, i, q) = 1.0 + 0.5 * hash_unit((unsigned)q, (unsigned)i);
        for (int it = 0; it < 3; ++it) {
            // L solve (row interchanges as recorded)
            double xi = at(4, 0, q);
            double xn = n > 1 ? at(4, 1, q) : 0.0, l = at(0, 0, q), pv = at(5, 0, q);
            for (int i = 0; i < n - 1; ++i) {
                const double xnext = xn, li = l, pi = pv;
                if (i + 2 < n) xn = at(4, i + 2, q);
                if (i + 1 < n - 1) {
                    l = at(0, i + 1, q);
                    pv = at(5, i + 1, q);
                }
                if (pi == 0.0) {
                    at(4, i, q) = xi;
                    xi = xnext - li * xi;
                } else {
                    at(4, i, q) = xnext;
                    xi = xi - li * xnext;
                }
            }
            at(4, n - 1, q) = xi;
            // U solve, backwards with x_{i+1}, x_{i+2} in registers
            double x1 = at(4, n - 1, q) / at(1, n - 1, q), x2 = 0.0;
            at(4, n - 1, q) = x1;
            if (n > 1) {
                double b = at(4, n - 2, q), dg = at(1, n - 2, q), u1 = at(2, n - 2, q), u2 = 0.0;
                for (int i = n - 2; i >= 0; --i) {
                    const double bi = b, di = dg, ui = u1, wi = u2;
                    if (i > 0) {
                        b = at(4, i - 1, q);
                        dg = at(1, i - 1, q);
                        u1 = at(2, i - 1, q);
                        u2 = at(3, i - 1, q);
                    }
                    const double xv = (bi - ui * x1 - wi * x2) / di;
                    at(4, i, q) = xv;
                    x2 = x1;
                    x1 = xv;
                }
            }
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) nrm += at(4, i, q) * at(4, i, q);
            nrm = sqrt(nrm);
            const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
            for (int i = 0; i < n; ++i) at(4, i, q) *= inv;
        }
    }
    __syncthreads();

    // With every iterate in LDS (rows of n + 1 doubles, so that the lanes of a column
    // read fall on different banks), Gram-Schmidt and the back-transformation read no
    // global memory; otherwise the iterates stay in the scratch and the reflectors are
    // applied to LDS panels of them.
    const int ldx = n + 1;
    const long hdr_d = 16L + ((nk + 15) / 16) * 16;  // red + coef
    const bool in_lds = (hdr_d + (long)nk * ldx + n) * 8 <= LDS_BYTES;
    if (in_lds) {
        for (int el = t; el < nk * n; el += ET) {
            const int q = el / n, i = el % n;
            X[(size_t)q * ldx + i] = at(4, i, q);
        }
        __syncthreads();
        // (2) Gram-Schmidt in descending-eigenvalue order, two passes (CGS2): each
        // coefficient is split over four lanes (a quarter of the rows each, summed by
        // DPP), each row's update keeps four partial sums
        for (int q = 0; q < nk; ++q) {
            double* xq = X + (size_t)q * ldx;
            for (int pass = 0; pass < 2; ++pass) {
                for (int base = 0; base < q; base += ET / 4) {
                    const int c = base + (t >> 2), part = t & 3;
                    double sp = 0.0;
                    if (c < q) {
                        const double* xc = X + (size_t)c * ldx;
                        for (int i = part; i < n; i += 4) sp = fma(xc[i], xq[i], sp);
                    }
                    sp += dpp_move<0xB1>(sp);
                    sp += dpp_move<0x4E>(sp);
                    if (c < q && part == 0) coef[c] = sp;
                }
                __syncthreads();
                for (int i = t; i < n; i += ET) {
                    double a0 = xq[i], a1 = 0.0, a2 = 0.0, a3 = 0.0;
                    int c = 0;
                    for (; c + 4 <= q; c += 4) {
                        a0 = fma(-coef[c], X[(size_t)c * ldx + i], a0);
                        a1 = fma(-coef[c + 1], X[(size_t)(c + 1) * ldx + i], a1);
                        a2 = fma(-coef[c + 2], X[(size_t)(c + 2) * ldx + i], a2);
                        a3 = fma(-coef[c + 3], X[(size_t)(c + 3) * ldx + i], a3);
                    }
                    for (; c < q; ++c) a0 = fma(-coef[c], X[(size_t)c * ldx + i], a0);
                    xq[i] = (a0 + a1) + (a2 + a3);
                }
                __syncthreads();
            }
            double part = 0.0;
            for (int i = t; i < n; i += ET) part += xq[i] * xq[i];
            const double nrm = sqrt(block_sum(part, red));
            const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
            for (int i = t; i < n; i += ET) xq[i] *= inv;
            __syncthreads();
        }
        if (D.skip_bt) {
            for (int el = t; el < nk * n; el += ET) {
                const int i = el % n, q = el / n;
                D.Z[(long)i + (long)q * D.ldz] = X[(size_t)q * ldx + i];
            }
            return;
        }
    } else {
        // (2) Gram-Schmidt in descending-eigenvalue order, two passes (CGS2).  The dot
        // products and updates keep 8 independent loads and partial sums in flight.
        for (int q = 0; q < nk; ++q) {
            for (int pass = 0; pass < 2; ++pass) {
                for (int qq = t; qq < q; qq += ET) {
                    double sp[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                    int i = 0;
                    for (; i + 8 <= n; i += 8) {
#pragma unroll
                        for (int u = 0; u < 8; ++u) sp[u] = fma(at(4, i + u, qq), at(4, i + u, q), sp[u]);
                    }
                    for (; i < n; ++i) sp[0] = fma(at(4, i, qq), at(4, i, q), sp[0]);
                    coef[qq] = ((sp[0] + sp[1]) + (sp[2] + sp[3])) + ((sp[4] + sp[5]) + (sp[6] + sp[7]));
                }
                __syncthreads();
                for (int i = t; i < n; i += ET) {
                    double vp8[8] = {at(4, i, q), 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                    int qq = 0;
                    for (; qq + 8 <= q; qq += 8) {
#pragma unroll
                        for (int u = 0; u < 8; ++u) vp8[u] = fma(-coef[qq + u], at(4, i, qq + u), vp8[u]);
                    }
                    for (; qq < q; ++qq) vp8[0] = fma(-coef[qq], at(4, i, qq), vp8[0]);
                    at(4, i, q) = ((vp8[0] + vp8[1]) + (vp8[2] + vp8[3])) + ((vp8[4] + vp8[5]) + (vp8[6] + vp8[7]));
                }
                __syncthreads();
            }
            double part = 0.0;
            for (int i = t; i < n; i += ET) part += at(4, i, q) * at(4, i, q);
            const double nrm = sqrt(block_sum(part, red));
            const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
            for (int i = t; i < n; i += ET) at(4, i, q) *= inv;
            __syncthreads();
        }

        if (D.skip_bt) {
            for (int el = t; el < nk * n; el += ET) {
                const int i = el % n, q = el / n;
                D.Z[(long)i + (long)q * D.ldz] = at(4, i, q);
            }
            return;
        }
    }

    // (3) back-transformation z = H_0 H_1 ... H_{n-3} x: all vectors at once when they
    // are in LDS, else in LDS panels loaded from the scratch
    const int ldp = in_lds ? ldx : n;
    const long hdr = hdr_d * 8 + (long)n * 8;  // red + coef + v_j
    const int nv = in_lds ? nk : (int)((LDS_BYTES - hdr) / ((long)n * 8));
    const int panel = nv < nk ? (nv > 0 ? nv : 1) : nk;
    double* vj = X + (size_t)panel * ldp;  // n doubles
    for (int q0 = 0; q0 < nk; q0 += panel) {
        const int pq = (nk - q0) < panel ? (nk - q0) : panel;
        if (!in_lds)
            for (int el = t; el < pq * n; el += ET) {
                const int i = el % n, qq = el / n;
                X[(size_t)qq * ldp + i] = at(4, i, q0 + qq);
            }
        __syncthreads();
        for (int j = n - 3; j >= 0; --j) {
            const double tj = D.tau[j];
            if (tj == 0.0) continue;
            for (int i = t; i < n; i += ET) vj[i] = (i == j + 1) ? 1.0 : (i > j + 1 ? D.V[(long)i + (long)j * D.ldv] : 0.0);
            __syncthreads();
            // 8 lanes per vector, DPP-reduced
            for (int base = 0; base < pq; base += ET / 8) {
                const int qq = base + (t >> 3), part = t & 7;
                double s = 0.0;
                if (qq < pq) {
                    const double* x = X + (size_t)qq * ldp;
                    for (int i = j + 1 + part; i < n; i += 8) s = fma(vj[i], x[i], s);
                }
                s = sum_lanes8(s);
                if (qq < pq && part == 0) coef[qq] = tj * s;
            }
            __syncthreads();
            for (int el = t; el < pq * (n - j - 1); el += ET) {
                const int qq = el / (n - j - 1), i = j + 1 + el % (n - j - 1);
                X[(size_t)qq * ldp + i] -= coef[qq] * vj[i];
            }
            __syncthreads();
        }
        for (int el = t; el < pq * n; el += ET) {
            const int i = el % n, qq = el / n;
            D.Z[(long)i + (long)(q0 + qq) * D.ldz] = X[(size_t)qq * ldp + i];
        }
        __syncthreads();
    }
}

void sym_vectors_batched(const VecDesc* d_descs, int count, hipStream_t s) {
    if (count <= 0) return;
    lds_limit((const void*)sym_vectors_kernel, LDS_BYTES);
    hipLaunchKernelGGL(sym_vectors_kernel, dim3(count), dim3(ET), LDS_BYTES, s, d_descs);
}

}  // namespace cmsvd
