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

__global__ void __launch_bounds__(256) chol_semidef_kernel(const CholDesc* __restrict__ descs) {
    const CholDesc D = descs[blockIdx.x];
    const int k = D.k, t = threadIdx.x;
    double* G = D.G;
    const long ld = D.ldg;
    __shared__ double colj[4096];
    __shared__ double piv;
    __shared__ int ndrop;
    if (t == 0) ndrop = 0;
    const double thresh = D.thresh_scale * (D.thresh_ref ? D.thresh_ref[0] : 1.0);
    for (int j = 0; j < k; ++j) {
        if (t == 0) {
            const double dj = G[j + j * ld];
            if (dj > thresh) piv = sqrt(dj);
            else {
                piv = 0.0;
                ++ndrop;
            }
            G[j + j * ld] = piv;
        }
        __syncthreads();
        const double pj = piv;
        for (int i = j + 1 + t; i < k; i += 256) {
            const double v = pj > 0.0 ? G[i + j * ld] / pj : 0.0;
            G[i + j * ld] = v;
            if (i < 4096) colj[i] = v;
        }
        __syncthreads();
        if (pj > 0.0) {
            // trailing update of the lower triangle: G(i,l) -= L(i,j) L(l,j), j < l <= i
            const int m = k - j - 1;
            const long tot = (long)m * m;
            for (long e = t; e < tot; e += 256) {
                const int i = (int)(e % m), l = (int)(e / m);
                if (i < l) continue;
                const int gi = j + 1 + i, gl = j + 1 + l;
                const double li = gi < 4096 ? colj[gi] : G[gi + j * ld];
                const double ll = gl < 4096 ? colj[gl] : G[gl + j * ld];
                G[gi + (long)gl * ld] -= li * ll;
            }
        }
        __syncthreads();
    }
    // Linv: forward substitution, one column of the inverse per thread
    for (int c = t; c < k; c += 256) {
        double* X = D.Linv + (long)c * D.ldi;
        for (int i = 0; i < c; ++i) X[i] = 0.0;
        const double lcc = G[c + c * ld];
        X[c] = lcc > 0.0 ? 1.0 / lcc : 0.0;
        for (int i = c + 1; i < k; ++i) {
            const double lii = G[i + i * ld];
            if (lii > 0.0) {
                double s = 0.0;
                for (int b = c; b < i; ++b) s += G[i + (long)b * ld] * X[b];
                X[i] = -s / lii;
            } else {
                X[i] = 0.0;
            }
        }
    }
    __syncthreads();
    // leave L with a zero strict upper triangle
    for (long e = t; e < (long)k * k; e += 256) {
        const int i = (int)(e % k), c = (int)(e / k);
        if (i < c) G[i + (long)c * ld] = 0.0;
    }
    if (t == 0 && D.dropped) *D.dropped = ndrop;
}

void chol_semidef_batched(const CholDesc* d_descs, int count, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(chol_semidef_kernel, dim3(count), dim3(256), 0, s, d_descs);
}

// Frobenius norm squared (double-double) of row-major blocks.
__global__ void __launch_bounds__(256) sumsq_kernel(const NormDesc* __restrict__ descs) {
    const NormDesc D = descs[blockIdx.x];
    __shared__ double red_hi[256], red_lo[256];
    double hi = 0.0, lo = 0.0;
    const long tot = (long)D.rows * D.cols;
    for (long e = threadIdx.x; e < tot; e += 256) {
        const long r = e / D.cols, c = e % D.cols;
        const double v = D.f32 ? (double)static_cast<const float*>(D.A)[r * D.ld + c]
                               : static_cast<const double*>(D.A)[r * D.ld + c];
        double p = v * v;
        double pe = fma(v, v, -p);  // exact product error
        dd_add(hi, lo, p);
        lo += pe;
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
    const long tot = (long)D.rows * D.cols;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
        const long r = e / D.cols, c = e % D.cols;
        const double v = D.f32 ? (double)static_cast<const float*>(D.A)[r * D.lda + c]
                               : static_cast<const double*>(D.A)[r * D.lda + c];
        D.B[r * D.ldb + c] = v;
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
