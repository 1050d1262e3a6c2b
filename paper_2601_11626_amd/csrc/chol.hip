// Semidefinite Cholesky with a pivot threshold and the inverse of the kept factor.
//
// Used by CholeskyQR2 of the residual (the thin QR that Lemma 1 asks for): the
// Gram G = R^T R is factored as G = L L^T; a pivot that falls to or below the
// threshold marks a residual direction that lies (numerically) in the span of the
// previous ones, so its column of L is set to zero and the matching column of Q
// becomes zero.  Linv is the inverse of L on the kept pivots (zero rows and columns
// on dropped ones), so Q = R Linv^T is an orthonormal basis of range(R) up to the
// dropped energy, which is at most k * thresh.
#include "common.hpp"
#include "kernels.hpp"

namespace cmsvd {

constexpr int CHT = 256;              // threads per problem
constexpr int CH_LDS = 16384;         // doubles of LDS for panels (128 KiB)

// Right-looking Cholesky by panels of up to 32 columns.  The panel (all rows from
// its first column down) is factored in LDS; the trailing lower triangle is then
// updated in global memory (L2-resident), one column at a time with the rows spread
// over the threads.  Afterwards the inverse of L is formed by column blocks, each
// block held in LDS while its rows are produced in order; every entry is a dot
// product split over 8 lanes and reduced with DPP.
__global__ void __launch_bounds__(CHT) chol_semidef_kernel(const CholDesc* __restrict__ descs) {
    const CholDesc D = descs[blockIdx.x];
    const int k = D.k, t = threadIdx.x;
    double* G = D.G;
    const long ld = D.ldg;
    extern __shared__ double sm[];
    __shared__ double piv_s;
    __shared__ int ndrop_s;
    if (t == 0) ndrop_s = 0;
    const double thresh = D.thresh_scale * (D.thresh_ref ? D.thresh_ref[0] : 1.0);
    int pw = 32;
    while (pw > 1 && (long)k * pw > CH_LDS) pw >>= 1;

    for (int jb = 0; jb < k; jb += pw) {
        const int w = pw < k - jb ? pw : k - jb, h = k - jb;
        double* P = sm;  // h x w row-major: P[r * w + c] = G(jb + r, jb + c)
        __syncthreads();
        for (int r = t; r < h; r += CHT)
            for (int c = 0; c < w; ++c) P[r * w + c] = r >= c ? G[(jb + r) + (long)(jb + c) * ld] : 0.0;
        __syncthreads();
        for (int c = 0; c < w; ++c) {
            if (t == 0) {
                const double d = P[c * w + c];
                double pv = 0.0;
                if (d > thresh) pv = sqrt(d);
                else ++ndrop_s;
                P[c * w + c] = pv;
                piv_s = pv;
            }
            __syncthreads();
            const double pv = piv_s;
            const double inv = pv > 0.0 ? 1.0 / pv : 0.0;
            for (int r = c + 1 + t; r < h; r += CHT) P[r * w + c] *= inv;
            __syncthreads();
            for (int r = c + 1 + t; r < h; r += CHT) {
                const double l = P[r * w + c];
                const int cmax = r < w - 1 ? r : w - 1;
                for (int c2 = c + 1; c2 <= cmax; ++c2) P[r * w + c2] -= l * P[c2 * w + c];
            }
            __syncthreads();
        }
        for (int r = t; r < h; r += CHT)
            for (int c = 0; c < w && c <= r; ++c) G[(jb + r) + (long)(jb + c) * ld] = P[r * w + c];
        for (int l = jb + w; l < k; ++l) {
            const double* Pl = P + (l - jb) * w;
            for (int i = l + t; i < k; i += CHT) {
                const double* Pi = P + (i - jb) * w;
                double acc = 0.0;
                for (int p = 0; p < w; ++p) acc = fma(Pi[p], Pl[p], acc);
                G[i + (long)l * ld] -= acc;
            }
        }
        __syncthreads();
    }

    // Linv = L^{-1} on the kept pivots: column block [cb, cb + w) solves L X = I by
    // forward substitution, rows in order; thread t works on column c = t / 8 with
    // part t % 8 of every dot product.
    int xw = 32;
    while (xw > 1 && (long)k * xw > CH_LDS) xw >>= 1;
    const int c = t >> 3, part = t & 7;
    for (int cb = 0; cb < k; cb += xw) {
        const int w = xw < k - cb ? xw : k - cb;
        double* X = sm;  // (k - cb) x w row-major
        __syncthreads();
        for (int i = cb; i < k; ++i) {
            const double lii = G[i + (long)i * ld];
            double s = 0.0;
            const int gc = cb + c;
            if (c < w && gc < i)
                for (int b = gc + part; b < i; b += 8) s = fma(G[i + (long)b * ld], X[(b - cb) * w + c], s);
            s = sum_lanes8(s);
            if (c < w && part == 0) {
                double x = 0.0;
                if (i >= gc && lii > 0.0) x = ((i == gc ? 1.0 : 0.0) - s) / lii;
                X[(i - cb) * w + c] = x;
            }
            __syncthreads();
        }
        for (int cc = 0; cc < w; ++cc) {
            double* Xo = D.Linv + (long)(cb + cc) * D.ldi;
            for (int i = t; i < k; i += CHT) Xo[i] = i >= cb ? X[(i - cb) * w + cc] : 0.0;
        }
    }
    __syncthreads();
    // leave L with a zero strict upper triangle
    for (int cc = 1; cc < k; ++cc)
        for (int i = t; i < cc; i += CHT) G[i + (long)cc * ld] = 0.0;
    if (t == 0 && D.dropped) *D.dropped = ndrop_s;
}

void chol_semidef_batched(const CholDesc* d_descs, int count, hipStream_t s) {
    if (count <= 0) return;
    lds_limit((const void*)chol_semidef_kernel, CH_LDS * (int)sizeof(double));
    hipLaunchKernelGGL(chol_semidef_kernel, dim3(count), dim3(CHT), CH_LDS * sizeof(double), s, d_descs);
}

// Frobenius norm squared (double-double) of row-major blocks.
__global__ void __launch_bounds__(256) sumsq_kernel(const NormDesc* __restrict__ descs) {
    const NormDesc D = descs[blockIdx.x];
    __shared__ double red_hi[256], red_lo[256];
    double hi = 0.0, lo = 0.0;
    const int cols = D.cols;
    const long tot = cols > 0 ? (long)D.rows * cols : 0;
    // element e = r * cols + c, advanced by 256 without a division per element: the step
    // is q rows and rem columns, and the column wraps at most once
    const int q = cols > 0 ? 256 / cols : 0, rem = cols > 0 ? 256 % cols : 0;
    long r = cols > 0 ? (long)(threadIdx.x / cols) : 0;
    int c = cols > 0 ? (int)(threadIdx.x % cols) : 0;
    for (long e = threadIdx.x; e < tot; e += 256) {
        const double v = D.f32 ? (double)static_cast<const float*>(D.A)[r * D.ld + c]
                               : static_cast<const double*>(D.A)[r * D.ld + c];
        double p = v * v;
        double pe = fma(v, v, -p);  // exact product error
        dd_add(hi, lo, p);
        lo += pe;
        r += q;
        c += rem;
        if (c >= cols) {
            c -= cols;
            ++r;
        }
    }
    red_hi[threadIdx.x] = hi;
    red_lo[threadIdx.x] = lo;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            double h = red_hi[threadIdx.x], l = red_lo[threadIdx.x];
            dd_add(h, l, red_hi[threadIdx.x + o]);
            l += red_lo[threadIdx.x + o];
            red_hi[threadIdx.x] = h;
            red_lo[threadIdx.x] = l;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double s, e;
        two_sum(red_hi[0], red_lo[0], s, e);
        D.out[0] = s;
        D.out[1] = e;
    }
}

void sumsq_batched(const NormDesc* d_descs, int count, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(sumsq_kernel, dim3(count), dim3(256), 0, s, d_descs);
}

__global__ void __launch_bounds__(256) copy_f64_kernel(const CopyDesc* __restrict__ descs) {
    const CopyDesc D = descs[blockIdx.y];
    if (D.cols <= 0) return;
    const long tot = (long)D.rows * D.cols;
    const long e0 = (long)blockIdx.x * 256 + threadIdx.x, step = (long)gridDim.x * 256;
    // (r, c) of element e advanced by the stride without a division per element
    const long q = step / D.cols;
    const int rem = (int)(step % D.cols);
    long r = e0 / D.cols;
    int c = (int)(e0 % D.cols);
    for (long e = e0; e < tot; e += step) {
        const double v = D.f32 ? (double)static_cast<const float*>(D.A)[r * D.lda + c]
                               : static_cast<const double*>(D.A)[r * D.lda + c];
        D.B[r * D.ldb + c] = v;
        r += q;
        c += rem;
        if (c >= D.cols) {
            c -= D.cols;
            ++r;
        }
    }
}

void copy_f64_batched(const CopyDesc* d_descs, int count, int maxrows, hipStream_t s) {
    if (count <= 0) return;
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        hipLaunchKernelGGL(copy_f64_kernel, dim3(64, n), dim3(256), 0, s, d_descs + base);
    }
}

}  // namespace cmsvd
