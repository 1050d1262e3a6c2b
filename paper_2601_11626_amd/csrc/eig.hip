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
constexpr int TILE = 32;         // tile edge
constexpr int TILE_EL = TILE * TILE;
constexpr int LDS_BYTES = 163840;  // gfx950: 160 KiB per workgroup

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

// Number of eigenvalues of the tridiagonal (dd, e2 = off-diagonal squared) below x.
__device__ __forceinline__ int sturm_count(const double* dd, const double* e2, int n, double x, double pivmin) {
    double q = dd[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
    for (int i = 1; i < n; ++i) {
        q = (dd[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    return cnt;
}

static int tl_for(int npad, int T) {
    const long vec_bytes = (10L * npad + 32) * 8;
    int tl = 0;
    while (tl + 1 <= T && vec_bytes + (long)(tl + 1) * (tl + 2) / 2 * TILE_EL * 8 <= LDS_BYTES) ++tl;
    return tl;
}

template <int MODE>
__global__ void __launch_bounds__(ET) sym_eig_kernel(const EigDesc* __restrict__ descs, int count, int NP,
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
                for (int el = t; el < TILE_EL; el += ET) {
                    const int li = el & 31, lc = el >> 5;
                    tp[el] = hval(D, R * TILE + li, C * TILE + lc);
                }
            }
        for (int i = t; i < npad; i += ET) {
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
            for (int i = j + t; i < n; i += ET) {
                const double* tp = tile_ptr(i >> 5, Cj, T, c0, TL, gt, lt);
                const double val = tp[cj * TILE + (i & 31)] - (vp[i] * wpj + wp[i] * vpj);
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
            for (int i = t; i < npad; i += ET) {
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
                    if ((f & 3) != w) continue;
                    double* tp = tile_ptr(R, C, T, c0, TL, gt, lt);
                    const int gi0 = R * TILE + 4 * ly, gc0 = C * TILE + 4 * lx;
                    double a[4][4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int s = 0; s < 4; ++s) a[s][q] = tp[(4 * lx + q) * TILE + 4 * ly + s];
                    double vr[4], wr[4], cr[4], vq[4], wq[4], cq[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        vr[s] = vp[gi0 + s];
                        wr[s] = wp[gi0 + s];
                        cr[s] = vc[gi0 + s];
                        vq[s] = vp[gc0 + s];
                        wq[s] = wp[gc0 + s];
                        cq[s] = vc[gc0 + s];
                    }
                    const bool any_active = (gi0 + 3 >= j + 1) && (gc0 + 3 >= j + 1);
                    if (any_active) {
#pragma unroll
                        for (int s = 0; s < 4; ++s)
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                if (gi0 + s >= j + 1 && gc0 + q >= j + 1)
                                    a[s][q] -= vr[s] * wq[q] + wr[s] * vq[q];
#pragma unroll
                        for (int q = 0; q < 4; ++q)
#pragma unroll
                            for (int s = 0; s < 4; ++s) tp[(4 * lx + q) * TILE + 4 * ly + s] = a[s][q];
                    }
                    double rp[4], cp[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) rp[s] = a[s][0] * cq[0] + a[s][1] * cq[1] + a[s][2] * cq[2] + a[s][3] * cq[3];
#pragma unroll
                    for (int q = 0; q < 4; ++q) cp[q] = a[0][q] * cr[0] + a[1][q] * cr[1] + a[2][q] * cr[2] + a[3][q] * cr[3];
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        rp[s] += shfl_xor_d(rp[s], 1);
                        rp[s] += shfl_xor_d(rp[s], 2);
                        rp[s] += shfl_xor_d(rp[s], 4);
                    }
                    if (R != C) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            cp[q] += shfl_xor_d(cp[q], 8);
                            cp[q] += shfl_xor_d(cp[q], 16);
                            cp[q] += shfl_xor_d(cp[q], 32);
                        }
                    }
                    double* pww = pw + w * NP;
                    if (lx == 0) {
#pragma unroll
                        for (int s = 0; s < 4; ++s) pww[gi0 + s] += rp[s];
                    }
                    if (R != C && ly == 0) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) pww[gc0 + q] += cp[q];
                    }
                }
            }
            __syncthreads();

            // (C) p = tau * A v, w = p - (tau/2)(p.v) v
            double dpart = 0.0;
            for (int i = t; i < npad; i += ET) {
                const double sacc = pw[i] + pw[NP + i] + pw[2 * NP + i] + pw[3 * NP + i];
                pw[i] = pw[NP + i] = pw[2 * NP + i] = pw[3 * NP + i] = 0.0;
                const double pi = (i >= j + 1 && i < n) ? tau * sacc : 0.0;
                xv[i] = pi;
                dpart += pi * vc[i];
            }
            const double dot = block_sum(dpart, red);
            const double K = -0.5 * tau * dot;
            for (int i = t; i < npad; i += ET) {
                wp[i] = (i >= j + 1 && i < n) ? xv[i] + K * vc[i] : 0.0;
                vp[i] = vc[i];
            }
            __syncthreads();
        }
        __syncthreads();

        // ---- bisection for the nkeep largest eigenvalues ----
        for (int i = t; i < npad; i += ET) xv[i] = (i < n - 1) ? ee[i] * ee[i] : 0.0;
        double glo = INFINITY, ghi = -INFINITY, em = 0.0;
        for (int i = t; i < n; i += ET) {
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
        glo -= tol;
        ghi += tol;
        double* lamv = pw;  // free now
        for (int q = t; q < D.nkeep; q += ET) {
            double lo = glo, hi = ghi;
            const int target = n - q;
            while (hi - lo > tol) {
                const double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (sturm_count(dd, xv, n, mid, pivmin) >= target) hi = mid;
                else lo = mid;
            }
            lamv[q] = 0.5 * (lo + hi);
        }
        __syncthreads();
        if (t == 0) {
            double hi = 0.0, lo = 0.0;
            for (int q = 0; q < D.nkeep; ++q) dd_add(hi, lo, lamv[q]);
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
            for (int q = t; q < D.nkeep; q += ET) D.lam[q] = lamv[q];
            if (D.d)
                for (int i = t; i < n; i += ET) {
                    D.d[i] = dd[i];
                    if (i < n - 1) D.e[i] = ee[i];
                }
        }
        __syncthreads();
    }
}

size_t sym_eig_workspace_doubles(int nmax, int nslots) {
    const int T = (nmax + TILE - 1) / TILE;
    return (size_t)nslots * (size_t)T * (size_t)(T + 1) / 2 * TILE_EL;
}

void sym_eig_batched(const EigDesc* d_descs, int count, int nmax, int mode, double* gws, int nslots,
                     hipStream_t s) {
    if (count <= 0) return;
    const int T = (nmax + TILE - 1) / TILE, npad = T * TILE;
    const int TL = tl_for(npad, T);
    const size_t lds = (size_t)(10L * npad + 32) * 8 + (size_t)TL * (TL + 1) / 2 * TILE_EL * 8;
    const long slot = (long)T * (T + 1) / 2 * TILE_EL;
    const int grid = count < nslots ? count : nslots;
    if (mode == 0) {
        (void)hipFuncSetAttribute((const void*)sym_eig_kernel<0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(sym_eig_kernel<0>, dim3(grid), dim3(ET), lds, s, d_descs, count, npad, TL, gws, slot);
    } else {
        (void)hipFuncSetAttribute((const void*)sym_eig_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(sym_eig_kernel<1>, dim3(grid), dim3(ET), lds, s, d_descs, count, npad, TL, gws, slot);
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

    // (1) independent inverse iteration, one thread per eigenvalue
    for (int q = t; q < nk; q += ET) {
        const double lam = D.lam[q];
        for (int i = 0; i < n; ++i) {
            at(0, i, q) = i < n - 1 ? D.e[i] : 0.0;  // dl
            at(1, i, q) = D.d[i] - lam;              // dd
            at(2, i, q) = i < n - 1 ? D.e[i] : 0.0;  // du
            at(3, i, q) = 0.0;                       // du2
            at(5, i, q) = 0.0;                       // pivot flag
            at(4, i, q) = 1.0 + 0.5 * hash_unit((unsigned)q, (unsigned)i);
        }
        // LU with partial pivoting of the tridiagonal T - lam I
        for (int i = 0; i < n - 1; ++i) {
            double di = at(1, i, q), li = at(0, i, q);
            if (fabs(di) >= fabs(li)) {
                if (di == 0.0) { di = tiny; at(1, i, q) = di; }
                const double fact = li / di;
                at(0, i, q) = fact;
                at(1, i + 1, q) -= fact * at(2, i, q);
            } else {
                const double fact = di / li;
                at(1, i, q) = li;
                at(0, i, q) = fact;
                const double temp = at(2, i, q);
                at(2, i, q) = at(1, i + 1, q);
                at(1, i + 1, q) = temp - fact * at(1, i + 1, q);
                if (i < n - 2) {
                    at(3, i, q) = at(2, i + 1, q);
                    at(2, i + 1, q) = -fact * at(2, i + 1, q);
                }
                at(5, i, q) = 1.0;
            }
        }
        if (at(1, n - 1, q) == 0.0) at(1, n - 1, q) = tiny;
        for (int it = 0; it < 3; ++it) {
            // L solve
            for (int i = 0; i < n - 1; ++i) {
                if (at(5, i, q) == 0.0) at(4, i + 1, q) -= at(0, i, q) * at(4, i, q);
                else {
                    const double temp = at(4, i, q);
                    at(4, i, q) = at(4, i + 1, q);
                    at(4, i + 1, q) = temp - at(0, i, q) * at(4, i, q);
                }
            }
            // U solve
            at(4, n - 1, q) /= at(1, n - 1, q);
            if (n > 1) at(4, n - 2, q) = (at(4, n - 2, q) - at(2, n - 2, q) * at(4, n - 1, q)) / at(1, n - 2, q);
            for (int i = n - 3; i >= 0; --i)
                at(4, i, q) = (at(4, i, q) - at(2, i, q) * at(4, i + 1, q) - at(3, i, q) * at(4, i + 2, q)) / at(1, i, q);
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) nrm += at(4, i, q) * at(4, i, q);
            nrm = sqrt(nrm);
            const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
            for (int i = 0; i < n; ++i) at(4, i, q) *= inv;
        }
    }
    __syncthreads();

    // (2) Gram-Schmidt in descending-eigenvalue order, two passes (CGS2)
    for (int q = 0; q < nk; ++q) {
        for (int pass = 0; pass < 2; ++pass) {
            for (int qq = t; qq < q; qq += ET) {
                double s = 0.0;
                for (int i = 0; i < n; ++i) s += at(4, i, qq) * at(4, i, q);
                coef[qq] = s;
            }
            __syncthreads();
            for (int i = t; i < n; i += ET) {
                double v = at(4, i, q);
                for (int qq = 0; qq < q; ++qq) v -= coef[qq] * at(4, i, qq);
                at(4, i, q) = v;
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

    // (3) back-transformation z = H_0 H_1 ... H_{n-3} x, vectors in LDS panels
    const long hdr = (16L + ((nk + 15) / 16) * 16) * 8 + (long)n * 8;  // red + coef + v_j
    const int nv = (int)((LDS_BYTES - hdr) / ((long)n * 8));
    const int panel = nv < nk ? (nv > 0 ? nv : 1) : nk;
    double* vj = X + (size_t)panel * n;  // n doubles
    for (int q0 = 0; q0 < nk; q0 += panel) {
        const int pq = (nk - q0) < panel ? (nk - q0) : panel;
        for (int el = t; el < pq * n; el += ET) {
            const int i = el % n, qq = el / n;
            X[(size_t)qq * n + i] = at(4, i, q0 + qq);
        }
        __syncthreads();
        for (int j = n - 3; j >= 0; --j) {
            const double tj = D.tau[j];
            if (tj == 0.0) continue;
            for (int i = t; i < n; i += ET) vj[i] = (i == j + 1) ? 1.0 : (i > j + 1 ? D.V[(long)i + (long)j * D.ldv] : 0.0);
            __syncthreads();
            for (int qq = t; qq < pq; qq += ET) {
                double s = 0.0;
                const double* x = X + (size_t)qq * n;
                for (int i = j + 1; i < n; ++i) s += vj[i] * x[i];
                coef[qq] = tj * s;
            }
            __syncthreads();
            for (int el = t; el < pq * (n - j - 1); el += ET) {
                const int qq = el / (n - j - 1), i = j + 1 + el % (n - j - 1);
                X[(size_t)qq * n + i] -= coef[qq] * vj[i];
            }
            __syncthreads();
        }
        for (int el = t; el < pq * n; el += ET) {
            const int i = el % n, qq = el / n;
            D.Z[(long)i + (long)(q0 + qq) * D.ldz] = X[(size_t)qq * n + i];
        }
        __syncthreads();
    }
}

void sym_vectors_batched(const VecDesc* d_descs, int count, hipStream_t s) {
    if (count <= 0) return;
    (void)hipFuncSetAttribute((const void*)sym_vectors_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BYTES);
    hipLaunchKernelGGL(sym_vectors_kernel, dim3(count), dim3(ET), LDS_BYTES, s, d_descs);
}

}  // namespace cmsvd
