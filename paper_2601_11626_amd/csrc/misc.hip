// Small glue kernels of the update and the clustering decision.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace cmsvd {

__global__ void assemble_kt_kernel(const KtDesc* __restrict__ descs) {
    const KtDesc D = descs[blockIdx.y];
    const int n = D.r + D.k;
    const long tot = (long)n * n;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
        const int i = (int)(e % n), c = (int)(e / n);
        double v = 0.0;
        if (c < D.r) {
            if (i < D.r) v = (i == c) ? D.s[i] : 0.0;
            else v = D.P[(long)c + (long)(i - D.r) * D.ldp];  // (P^T)[i-r][c]
        } else if (i >= D.r) {
            const int a = i - D.r, b = c - D.r;
            v = (a >= b) ? D.F[(long)a + (long)b * D.ldf] : 0.0;
        }
        D.KT[(long)i + (long)c * D.ldk] = v;
    }
}

void assemble_kt_batched(const KtDesc* d_descs, int count, int nmax, hipStream_t s) {
    if (count <= 0) return;
    const long tot = (long)nmax * nmax;
    int gx = (int)((tot + 255) / 256);
    gx = gx > 512 ? 512 : gx;
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        hipLaunchKernelGGL(assemble_kt_kernel, dim3(gx, n), dim3(256), 0, s, d_descs + base);
    }
}

// Numerically present directions: eigenvalue above the eigensolver's rounding level
// (n eps ||S||); the others are stored as sigma = 0 with a zero basis column.
__device__ __forceinline__ bool fin_keep(const FinDesc& D, int q, double cut) {
    return q < D.nkeep && D.lam[q] > cut;
}

__global__ void __launch_bounds__(256) finalize_state_kernel(const FinDesc* __restrict__ descs) {
    const FinDesc D = descs[blockIdx.x];
    __shared__ double red_h[256], red_l[256];
    const int t = threadIdx.x;
    double lm = 0.0;
    for (int q = t; q < D.nkeep; q += 256) lm = fmax(lm, D.lam[q]);
    __shared__ double redm[4];
    const double lmax = block_max(lm, redm);
    const double cut = (double)D.nc * 8.0 * 2.220446049250313e-16 * lmax;
    // kept values and their energy, over every one of the r columns
    double kh = 0.0, kl = 0.0;
    for (int q = t; q < D.r; q += 256) {
        const bool k = fin_keep(D, q, cut);
        const double sv = k ? sqrt(D.lam[q]) : 0.0;
        D.s_out[q] = sv;
        if (k) dd_add(kh, kl, sv * sv);
    }
    // zero the basis columns of dropped directions (row-major m x r)
    for (long e = t; e < (long)D.m * D.r; e += 256) {
        const int q = (int)(e % D.r);
        const long row = e / D.r;
        if (!fin_keep(D, q, cut)) D.U_out[row * D.ldu + q] = 0.0;
    }
    // double-double tree sum of the kept energy (fixed order: reproducible)
    red_h[t] = kh;
    red_l[t] = kl;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            double h = red_h[t], l = red_l[t];
            dd_add(h, l, red_h[t + o]);
            red_h[t] = h;
            red_l[t] = l + red_l[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        // energies (double-double)
        double eh = D.acc[0], el = D.acc[1];
        dd_add(eh, el, D.nb[0]);
        el += D.nb[1];
        double sin_h = 0.0, sin_l = 0.0;
        for (int q = 0; q < D.r_in; ++q) dd_add(sin_h, sin_l, D.s_in[q] * D.s_in[q]);
        // core energy = sum s_in^2 + ||B||^2; discarded = core energy - kept
        double ch = sin_h, cl = sin_l;
        dd_add(ch, cl, D.nb[0]);
        cl += D.nb[1];
        double dh = D.acc[2], dl = D.acc[3];
        dd_add(dh, dl, ch);
        dl += cl;
        dd_add(dh, dl, -D.sum_top[0]);
        dl -= D.sum_top[1];
        D.acc[0] = eh;
        D.acc[1] = el;
        D.acc[2] = dh;
        D.acc[3] = dl;
        if (D.est) {
            const double kth = red_h[0], ktl = red_l[0];
            double s, e;
            two_sum(eh, -kth, s, e);
            double tail = s + (e + el - ktl);
            D.est[0] = sqrt(tail < 0.0 ? 0.0 : tail);
            const double dtot = dh + dl;
            D.est[1] = sqrt(dtot < 0.0 ? 0.0 : dtot);
        }
    }
}

void finalize_state_batched(const FinDesc* d_descs, int count, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(finalize_state_kernel, dim3(count), dim3(256), 0, s, d_descs);
}

__global__ void add_f64_kernel(const double* __restrict__ x, double* __restrict__ y, long n) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) y[i] += x[i];
}

void add_f64(const double* x, double* y, long n, hipStream_t s) {
    if (n <= 0) return;
    long g = (n + 255) / 256;
    hipLaunchKernelGGL(add_f64_kernel, dim3((int)(g > 1024 ? 1024 : g)), dim3(256), 0, s, x, y, n);
}

__global__ void zero_upper_kernel(double* A, int k, long lda) {
    const long tot = (long)k * k;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
        const int i = (int)(e % k), c = (int)(e / k);
        if (i < c) A[(long)i + (long)c * lda] = 0.0;
    }
}

__global__ void __launch_bounds__(256) clear_kernel(const ClearDesc* __restrict__ descs) {
    const ClearDesc D = descs[blockIdx.y];
    if (D.upper) {
        // column c holds c entries above the diagonal
        for (int c = 1 + blockIdx.x; c < D.k; c += gridDim.x)
            for (int i = threadIdx.x; i < c; i += 256) D.A[(long)i + (long)c * D.ld] = 0.0;
    } else {
        for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < D.n; e += (long)gridDim.x * 256) D.A[e] = 0.0;
    }
}

void clear_batched(const ClearDesc* d_descs, int count, hipStream_t s) {
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        hipLaunchKernelGGL(clear_kernel, dim3(64, n), dim3(256), 0, s, d_descs + base);
    }
}

void zero_upper(double* A, int k, long lda, hipStream_t s) {
    if (k <= 0) return;
    long g = ((long)k * k + 255) / 256;
    hipLaunchKernelGGL(zero_upper_kernel, dim3((int)(g > 1024 ? 1024 : g)), dim3(256), 0, s, A, k, lda);
}

__global__ void __launch_bounds__(256) first_feasible_kernel(const double* __restrict__ rel, int n, double eps,
                                                             int* out) {
    __shared__ int red[256];
    int best = n;
    for (int i = threadIdx.x; i < n; i += 256)
        if (rel[i] <= eps && i < best) best = i;
    red[threadIdx.x] = best;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

void first_feasible(const double* rel, int n, double eps, int* out, hipStream_t s) {
    hipLaunchKernelGGL(first_feasible_kernel, dim3(1), dim3(256), 0, s, rel, n, eps, out);
}

__global__ void __launch_bounds__(256) colblock_sumsq_kernel(const ColNormDesc* __restrict__ descs) {
    const ColNormDesc D = descs[blockIdx.x];
    double part = 0.0;
    for (long e = threadIdx.x; e < (long)D.r * D.k; e += 256) {
        const int i = (int)(e % D.r), c = (int)(e / D.r);
        const double v = D.P[(long)i + (long)c * D.ld];
        part += v * v;
    }
    __shared__ double red[4];
    const double s = block_sum(part, red);
    if (threadIdx.x == 0) *D.out = s;
}

void colblock_sumsq_batched(const ColNormDesc* d_descs, int count, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(colblock_sumsq_kernel, dim3(count), dim3(256), 0, s, d_descs);
}

// ---------------------------------------------------------------------------
// Backward of the tail energy: small helpers.
// ---------------------------------------------------------------------------
// B (r x d, column-major, ld r) *= g[lam_i, mu_j] with lam = ev[0..nk), mu = ev[nk..nk+d):
// the divided difference lam_i / (lam_i - mu_j) of the truncation between a kept and a
// dropped eigenvalue (0 where the two coincide).
__global__ void __launch_bounds__(256) divdiff_scale_kernel(double* __restrict__ B, int r, int nk, int d,
                                                            const double* __restrict__ ev) {
    for (long e = blockIdx.x * 256L + threadIdx.x; e < (long)r * d; e += 256L * gridDim.x) {
        const int i = (int)(e % r), j = (int)(e / r);
        double g = 0.0;
        if (i < nk) {
            const double li = ev[i], den = li - ev[nk + j];
            g = den != 0.0 ? li / den : 0.0;
        }
        B[e] *= g;
    }
}

void divdiff_scale(double* B, int r, int nk, int d, const double* ev, hipStream_t s) {
    if (r <= 0 || d <= 0) return;
    const long tot = (long)r * d;
    const int grid = (int)std::min<long>((tot + 255) / 256, 1024);
    hipLaunchKernelGGL(divdiff_scale_kernel, dim3(grid), dim3(256), 0, s, B, r, nk, d, ev);
}

// A (rows x cols, column-major, ld) = v off the diagonal and dv on it.
__global__ void __launch_bounds__(256) fill_diag_kernel(double* __restrict__ A, int rows, int cols, long ld, double v,
                                                        double dv) {
    for (long e = blockIdx.x * 256L + threadIdx.x; e < (long)rows * cols; e += 256L * gridDim.x) {
        const int i = (int)(e % rows), c = (int)(e / rows);
        A[(long)i + (long)c * ld] = i == c ? dv : v;
    }
}

void fill_diag(double* A, int rows, int cols, long ld, double v, double dv, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return;
    const long tot = (long)rows * cols;
    const int grid = (int)std::min<long>((tot + 255) / 256, 2048);
    hipLaunchKernelGGL(fill_diag_kernel, dim3(grid), dim3(256), 0, s, A, rows, cols, ld, v, dv);
}

// out = (ev[nk-1] - ev[nk]) / ev[0] (relative gap at the truncation), or +inf when
// nothing is dropped.
__global__ void cut_gap_kernel(const double* __restrict__ ev, int nk, int n, double* __restrict__ out) {
    if (threadIdx.x == 0) *out = (nk < n && nk > 0 && ev[0] > 0.0) ? (ev[nk - 1] - ev[nk]) / ev[0] : INFINITY;
}

void cut_gap(const double* ev, int nk, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(cut_gap_kernel, dim3(1), dim3(64), 0, s, ev, nk, n, out);
}

// ---------------------------------------------------------------------------
// Packing of row-major blocks side by side into one row-major matrix (FP32 or FP64).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) pack_kernel(const PackDesc* __restrict__ descs) {
    const PackDesc D = descs[blockIdx.y];
    const long tot = (long)D.rows * D.cols;
    const long stride = (long)gridDim.x * 256;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < tot; e += stride) {
        long r, c;
        if (tot < 0x7fffffffL) {
            const unsigned ue = (unsigned)e, uc = (unsigned)D.cols;
            r = ue / uc;
            c = ue - (unsigned)r * uc;
        } else {
            r = e / D.cols;
            c = e - r * D.cols;
        }
        double v;
        if (D.f32_in == 1) v = (double)static_cast<const float*>(D.src)[r * D.lds + c];
        else if (D.f32_in == 2)  // BF16: the high half of an FP32 word (exact widening)
            v = (double)__uint_as_float((unsigned)static_cast<const unsigned short*>(D.src)[r * D.lds + c] << 16);
        else v = static_cast<const double*>(D.src)[r * D.lds + c];
        if (D.f32_out) static_cast<float*>(D.dst)[r * D.ldd + c] = (float)v;
        else static_cast<double*>(D.dst)[r * D.ldd + c] = v;
    }
}

void pack_batched(const PackDesc* d_descs, int count, hipStream_t s) {
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        hipLaunchKernelGGL(pack_kernel, dim3(64, n), dim3(256), 0, s, d_descs + base);
    }
}

// ---------------------------------------------------------------------------
// Dense evaluation: one eigenproblem descriptor per compact pair record.
// ---------------------------------------------------------------------------
__global__ void expand_dense_descs_kernel(const PairRec* __restrict__ pr, int count, const AnchorRec* __restrict__ A,
                                          const CandRec* __restrict__ Cr, int r, int a0, const double* C, long ldc,
                                          long cmin, double* err, double* rel, EigDesc* __restrict__ out) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) {
        const PairRec p = pr[i];
        const AnchorRec a = A[p.slot];
        const CandRec c = Cr[p.cand];
        EigDesc e{};
        e.n = r + c.k;
        e.n1 = r;
        e.nkeep = r;
        e.s = a.S;
        e.P = C + (size_t)(p.slot - a0) * r + (size_t)(c.coff - cmin) * ldc;
        e.ldp = ldc;
        e.Y = c.G;
        e.ldy = c.k;
        e.na = a.na;
        e.nb = c.nb;
        e.out_err = err + p.out;
        e.out_rel = rel ? rel + p.out : nullptr;
        out[i] = e;
    }
}

void expand_dense_descs(const PairRec* pr, int count, const AnchorRec* A, const CandRec* Cr, int r, int a0,
                        const double* C, long ldc, long cmin, double* err, double* rel, EigDesc* out, hipStream_t s) {
    if (count <= 0) return;
    const int g = (count + 255) / 256 < 4096 ? (count + 255) / 256 : 4096;
    hipLaunchKernelGGL(expand_dense_descs_kernel, dim3(g), dim3(256), 0, s, pr, count, A, Cr, r, a0, C, ldc, cmin, err,
                       rel, out);
}

// ---------------------------------------------------------------------------
// Blocked back-transformation of eigenvectors (compact WY form of the stored
// Householder reflectors).
// ---------------------------------------------------------------------------
__global__ void materialize_reflectors_kernel(double* __restrict__ V, int n, long ldv) {
    // column j (< n - 2): zeros on rows <= j, the implicit 1 on row j + 1
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < (long)(n - 2) * n; e += (long)gridDim.x * 256) {
        const int j = (int)(e / n), i = (int)(e - (long)j * n);
        if (i <= j) V[(long)i + (long)j * ldv] = 0.0;
        else if (i == j + 1) V[(long)i + (long)j * ldv] = 1.0;
    }
}

void materialize_reflectors(double* V, int n, long ldv, hipStream_t s) {
    if (n < 3) return;
    const long tot = (long)(n - 2) * n;
    const int g = (int)std::min<long>((tot + 255) / 256, 2048);
    hipLaunchKernelGGL(materialize_reflectors_kernel, dim3(g), dim3(256), 0, s, V, n, ldv);
}

// One wavefront per block (b <= 32): column i of T from the columns before it
// (forward, columnwise): T(i,i) = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) S(0:i, i).
// T is built in LDS and written out at the end.
__global__ void __launch_bounds__(64) larft_kernel(const LarftDesc* __restrict__ descs) {
    const LarftDesc D = descs[blockIdx.x];
    __shared__ double Ts[32 * 32];
    const int k = threadIdx.x, b = D.b;
    for (int e = k; e < 32 * 32; e += 64) Ts[e] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int i = 0; i < b; ++i) {
        const double ti = D.tau[i];
        double v = 0.0;
        if (k < i) {
            for (int l = k; l < i; ++l) v = fma(Ts[k + 32 * l], D.S[(long)l + (long)i * D.ld], v);
            v *= -ti;
        }
        if (k < i) Ts[k + 32 * i] = v;
        if (k == i) Ts[i + 32 * i] = ti;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (int e = k; e < b * b; e += 64) {
        const int r = e % b, c = e / b;
        D.T[(long)r + (long)c * D.ld] = Ts[r + 32 * c];
    }
}

void larft_batched(const LarftDesc* d_descs, int count, hipStream_t s) {
    if (count <= 0) return;
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        hipLaunchKernelGGL(larft_kernel, dim3(n), dim3(64), 0, s, d_descs + base);
    }
}

}  // namespace cmsvd
