// Weyl-based certificate (Theorem 1) and the scan of Algorithm 1, plus the explicit
// tail of a concatenation (the reference value of the slack diagnostics).
//
// Theorem 1: for a set C of blocks, E_r^2(M_C) <= S_C - max_{j in C} h_j with S_C the
// energy and h_j = sum_{i <= r} sigma_i(A_j)^2 the block's r-head energy.  A cluster
// state is (S hi, S lo, m = max h) in device memory.
#include "common.hpp"
#include "kernels.hpp"

namespace cmsvd {

namespace {
constexpr int WT = 256;
}

// h[i] = the r-head energy of block i: its whole energy when it has at most r columns,
// else the sum of its r largest Gram eigenvalues (double-double pairs).
__global__ void weyl_heads_kernel(const double* __restrict__ a2, const double* __restrict__ top,
                                  const int* __restrict__ cols, int r, int n, double* __restrict__ h) {
    for (int i = blockIdx.x * WT + threadIdx.x; i < n; i += gridDim.x * WT)
        h[i] = cols[i] <= r ? a2[2 * i] + a2[2 * i + 1] : top[2 * i] + top[2 * i + 1];
}

void weyl_heads(const double* a2, const double* top, const int* cols, int r, int n, double* h, hipStream_t s) {
    if (n <= 0) return;
    const int g = (n + WT - 1) / WT;
    hipLaunchKernelGGL(weyl_heads_kernel, dim3(g > 1024 ? 1024 : g), dim3(WT), 0, s, a2, top, cols, r, n, h);
}

// One scan step of Algorithm 1 (one block).  Thread 0 first updates the state: init >= 0
// starts a cluster at block init; acc >= 0 adds block acc (S += a_acc, m = max(m, h_acc)).
// Then the first i in [0, count) whose block j = cand[i] keeps the ratio
// sqrt(max(0, S + a_j - max(m, h_j))) / sqrt(S + a_j) within eps is written to *first
// (count if none), and the state's own ratio to *rel.
__global__ void __launch_bounds__(WT) weyl_step_kernel(const int* __restrict__ cand, int count, int init, int acc,
                                                       const double* __restrict__ a2, const double* __restrict__ h,
                                                       double* __restrict__ state, double eps, int* __restrict__ first,
                                                       double* __restrict__ rel) {
    __shared__ double st[3];
    __shared__ int red[WT];
    const int t = threadIdx.x;
    if (t == 0) {
        double sh = state[0], sl = state[1], m = state[2];
        if (init >= 0) {
            sh = a2[2 * init];
            sl = a2[2 * init + 1];
            m = h[init];
        }
        if (acc >= 0) {
            dd_add(sh, sl, a2[2 * acc]);
            sl += a2[2 * acc + 1];
            m = fmax(m, h[acc]);
        }
        state[0] = st[0] = sh;
        state[1] = st[1] = sl;
        state[2] = st[2] = m;
        double s, e;
        two_sum(sh, -m, s, e);
        double b2 = s + (e + sl);
        if (b2 < 0.0) b2 = 0.0;
        const double tot = sh + sl;
        *rel = tot > 0.0 ? sqrt(b2) / sqrt(tot) : 0.0;
    }
    __syncthreads();
    int best = count;
    for (int i = t; i < count; i += WT) {
        const int j = cand[i];
        double sh = st[0], sl = st[1];
        dd_add(sh, sl, a2[2 * j]);
        sl += a2[2 * j + 1];
        const double m = fmax(st[2], h[j]);
        double s, e;
        two_sum(sh, -m, s, e);
        double b2 = s + (e + sl);
        if (b2 < 0.0) b2 = 0.0;
        const double tot = sh + sl;
        const double rr = tot > 0.0 ? sqrt(b2) / sqrt(tot) : 0.0;
        if (rr <= eps && i < best) best = i;
    }
    red[t] = best;
    __syncthreads();
    for (int o = WT / 2; o > 0; o >>= 1) {
        if (t < o) red[t] = min(red[t], red[t + o]);
        __syncthreads();
    }
    if (t == 0) *first = red[0];
}

void weyl_step(const int* cand, int count, int init, int acc, const double* a2, const double* h, double* state,
               double eps, int* first, double* rel, hipStream_t s) {
    hipLaunchKernelGGL(weyl_step_kernel, dim3(1), dim3(WT), 0, s, cand, count, init, acc, a2, h, state, eps, first,
                       rel);
}

// out = max(0, sum_i a_i - max_i h_i) over n blocks (Theorem 1 for the whole set).
__global__ void __launch_bounds__(WT) weyl_bound_kernel(const double* __restrict__ a2, const double* __restrict__ h,
                                                        int n, double* __restrict__ out) {
    __shared__ double rh[WT], rl[WT], rm[WT];
    const int t = threadIdx.x;
    double hi = 0.0, lo = 0.0, m = 0.0;
    for (int i = t; i < n; i += WT) {
        dd_add(hi, lo, a2[2 * i]);
        lo += a2[2 * i + 1];
        m = fmax(m, h[i]);
    }
    rh[t] = hi;
    rl[t] = lo;
    rm[t] = m;
    __syncthreads();
    if (t == 0) {
        double H = 0.0, L = 0.0, M = 0.0;
        for (int i = 0; i < WT; ++i) {
            dd_add(H, L, rh[i]);
            L += rl[i];
            M = fmax(M, rm[i]);
        }
        double s, e;
        two_sum(H, -M, s, e);
        const double b2 = s + (e + L);
        *out = b2 > 0.0 ? b2 : 0.0;
    }
}

void weyl_bound(const double* a2, const double* h, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(weyl_bound_kernel, dim3(1), dim3(WT), 0, s, a2, h, n, out);
}

// out = max(0, sum_i a_i - top) with top a double-double (the explicit tail).
__global__ void __launch_bounds__(WT) energy_minus_kernel(const double* __restrict__ a2, int n,
                                                          const double* __restrict__ top, double* __restrict__ out) {
    __shared__ double rh[WT], rl[WT];
    const int t = threadIdx.x;
    double hi = 0.0, lo = 0.0;
    for (int i = t; i < n; i += WT) {
        dd_add(hi, lo, a2[2 * i]);
        lo += a2[2 * i + 1];
    }
    rh[t] = hi;
    rl[t] = lo;
    __syncthreads();
    if (t == 0) {
        double H = 0.0, L = 0.0;
        for (int i = 0; i < WT; ++i) {
            dd_add(H, L, rh[i]);
            L += rl[i];
        }
        double s, e;
        two_sum(H, -top[0], s, e);
        const double v = s + (e + L - top[1]);
        *out = v > 0.0 ? v : 0.0;
    }
}

void energy_minus(const double* a2, int n, const double* top, double* out, hipStream_t s) {
    hipLaunchKernelGGL(energy_minus_kernel, dim3(1), dim3(WT), 0, s, a2, n, top, out);
}

// Column c of A (rows x cols, column-major, ld) times f_c, where f_c = 0 when
// lam[c] <= cut_rel * lam[0] (numerically absent direction), else 1 / sqrt(lam[c])
// (inv) or 1: the right factor of a truncated SVD from Gram eigenpairs.
__global__ void scale_cols_kernel(double* __restrict__ A, int rows, int cols, long ld, const double* __restrict__ lam,
                                  int inv, double cut_rel) {
    const double cut = cut_rel * lam[0];
    const long tot = (long)rows * cols;
    for (long e = (long)blockIdx.x * WT + threadIdx.x; e < tot; e += (long)gridDim.x * WT) {
        const int c = (int)(e / rows), i = (int)(e - (long)c * rows);
        const double l = lam[c];
        const double f = l > cut && l > 0.0 ? (inv ? 1.0 / sqrt(l) : 1.0) : 0.0;
        A[(long)i + (long)c * ld] *= f;
    }
}

void scale_cols(double* A, int rows, int cols, long ld, const double* lam, int inv, double cut_rel, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return;
    const long tot = (long)rows * cols;
    const int g = (int)((tot + WT - 1) / WT < 2048 ? (tot + WT - 1) / WT : 2048);
    hipLaunchKernelGGL(scale_cols_kernel, dim3(g), dim3(WT), 0, s, A, rows, cols, ld, lam, inv, cut_rel);
}

}  // namespace cmsvd
