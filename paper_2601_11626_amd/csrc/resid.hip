// Residual-certified clustering (Theorem 2, Corollary 1, Algorithm 2): the merge
// certificate of a candidate and the update of a cluster's residual spectrum and basis.
//
// A cluster keeps the r largest squared residual singular values L (non-increasing,
// zero-padded to r) and its energy S (double-double).  Because the residual ranges of
// the accepted blocks are mutually orthogonal, the residual spectrum of the enlarged
// cluster is the union of L and the candidate's residual spectrum, so the certificate
//     b^2 = S + ||A_j||^2 - (sum of the r largest values of L u lam_j)
// needs only a merge of two sorted lists.
#include <cfloat>

#include "common.hpp"
#include "kernels.hpp"

namespace cmsvd {

namespace {

constexpr int CT = 256;

// s[0..n) = v[0..n) clamped at 0 and made non-increasing by a running minimum: the
// eigensolver returns its values in order only up to its bisection tolerance, and the
// merge ranks below need exact order.
__device__ void stage_nonincreasing(const double* __restrict__ v, int n, double* s, double* red) {
    const int t = threadIdx.x;
    const int chunk = (n + CT - 1) / CT;
    const int b = t * chunk, e = min(n, b + chunk);
    double run = INFINITY;
    for (int i = b; i < e; ++i) {
        run = fmin(run, fmax(v[i], 0.0));
        s[i] = run;
    }
    red[t] = run;
    __syncthreads();
    for (int o = 1; o < CT; o <<= 1) {  // inclusive prefix minimum of the chunk minima
        const double x = t >= o ? red[t - o] : INFINITY;
        __syncthreads();
        red[t] = fmin(red[t], x);
        __syncthreads();
    }
    const double pre = t > 0 ? red[t - 1] : INFINITY;
    for (int i = b; i < e; ++i) s[i] = fmin(s[i], pre);
    __syncthreads();
}

// Number of leading entries of the non-increasing s[0..n) that are > x (ge: >= x).
__device__ __forceinline__ int count_lead(const double* s, int n, double x, bool ge) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ge ? s[mid] >= x : s[mid] > x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Merge ranks of L (r values, ties first) and lam (nk values): every element whose rank
// is below r is one of the r largest of the union.  COMMIT writes them to Lout in order;
// otherwise their double-double sum is returned to thread 0.
template <bool COMMIT>
__device__ void merge_top(const double* sL, int r, const double* sl, int nk, double* Lout, double* red, double* red2,
                          double& sum_hi, double& sum_lo) {
    const int t = threadIdx.x;
    double hi = 0.0, lo = 0.0;
    for (int i = t; i < r; i += CT) {
        const int rank = i + count_lead(sl, nk, sL[i], false);
        if (rank < r) {
            if (COMMIT) Lout[rank] = sL[i];
            else dd_add(hi, lo, sL[i]);
        }
    }
    for (int j = t; j < nk; j += CT) {
        const int rank = j + count_lead(sL, r, sl[j], true);
        if (rank < r) {
            if (COMMIT) Lout[rank] = sl[j];
            else dd_add(hi, lo, sl[j]);
        }
    }
    if (COMMIT) return;
    red[t] = hi;
    red2[t] = lo;
    __syncthreads();
    if (t == 0) {
        double h = 0.0, l = 0.0;
        for (int i = 0; i < CT; ++i) {
            dd_add(h, l, red[i]);
            l += red2[i];
        }
        sum_hi = h;
        sum_lo = l;
    }
}

}  // namespace

// One block per candidate.  Dynamic LDS: (r + nkmax + 2 CT) doubles.
__global__ void __launch_bounds__(CT) resid_cert_kernel(const CertDesc* __restrict__ descs, int r, int nkmax) {
    extern __shared__ double sm[];
    const CertDesc D = descs[blockIdx.x];
    double* sL = sm;
    double* sl = sL + r;
    double* red = sl + nkmax;
    double* red2 = red + CT;
    for (int i = threadIdx.x; i < r; i += CT) sL[i] = D.L[i];
    __syncthreads();
    stage_nonincreasing(D.lam, D.nk, sl, red);
    double sh = 0.0, slo = 0.0;
    merge_top<false>(sL, r, sl, D.nk, nullptr, red, red2, sh, slo);
    if (threadIdx.x == 0) {
        double eh = D.S[0], el = D.S[1];
        if (D.nb) {
            dd_add(eh, el, D.nb[0]);
            el += D.nb[1];
        }
        double s2, e2;
        two_sum(eh, -sh, s2, e2);
        double b2 = s2 + (e2 + el - slo);
        if (b2 < 0.0) b2 = 0.0;
        const double err = sqrt(b2);
        const double etot = eh + el;
        if (D.err) *D.err = err;
        if (D.rel) *D.rel = etot != 0.0 ? err / sqrt(etot) : 0.0;
    }
}

void resid_cert_batched(const CertDesc* d_descs, int count, int r, int nkmax, hipStream_t s) {
    if (count <= 0) return;
    const size_t lds = (size_t)(r + nkmax + 2 * CT) * sizeof(double);
    lds_limit(reinterpret_cast<const void*>(resid_cert_kernel), (int)lds);
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        hipLaunchKernelGGL(resid_cert_kernel, dim3(n), dim3(CT), lds, s, d_descs + base, r, nkmax);
    }
}

// Accepts a candidate: Lout = the r largest of L u lam (non-increasing), Sout = S + nb.
// One block.  Lout must not alias L.
__global__ void __launch_bounds__(CT) resid_accept_kernel(const double* __restrict__ L, int r,
                                                          const double* __restrict__ lam, int nk,
                                                          const double* __restrict__ S, const double* __restrict__ nb,
                                                          double* __restrict__ Lout, double* __restrict__ Sout) {
    extern __shared__ double sm[];
    double* sL = sm;
    double* sl = sL + r;
    double* red = sl + nk;
    for (int i = threadIdx.x; i < r; i += CT) sL[i] = L[i];
    __syncthreads();
    stage_nonincreasing(lam, nk, sl, red);
    double a = 0.0, b = 0.0;
    merge_top<true>(sL, r, sl, nk, Lout, nullptr, nullptr, a, b);
    if (threadIdx.x == 0) {
        double eh = S[0], el = S[1];
        dd_add(eh, el, nb[0]);
        el += nb[1];
        Sout[0] = eh;
        Sout[1] = el;
    }
}

void resid_accept(const double* L, int r, const double* lam, int nk, const double* S, const double* nb, double* Lout,
                  double* Sout, hipStream_t s) {
    const size_t lds = (size_t)(r + nk + CT) * sizeof(double);
    lds_limit(reinterpret_cast<const void*>(resid_accept_kernel), (int)lds);
    hipLaunchKernelGGL(resid_accept_kernel, dim3(1), dim3(CT), lds, s, L, r, lam, nk, S, nb, Lout, Sout);
}

// Kept columns of a residual basis: column c is kept when Li[c, c] != 0 (the inverse
// Cholesky factor is zero on dropped pivots).  map[c] = its position among the kept
// columns, or -1 when dropped or beyond `room`; *count = number placed.  One block.
__global__ void __launch_bounds__(CT) kept_map_kernel(const double* __restrict__ Li, long ldl, int k, int room,
                                                      int* __restrict__ map, int* __restrict__ count) {
    __shared__ int part[CT];
    const int t = threadIdx.x;
    const int chunk = (k + CT - 1) / CT;
    const int b = t * chunk, e = min(k, b + chunk);
    int c0 = 0;
    for (int c = b; c < e; ++c) c0 += Li[(long)c + (long)c * ldl] != 0.0;
    part[t] = c0;
    __syncthreads();
    for (int o = 1; o < CT; o <<= 1) {  // inclusive prefix sum
        const int x = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    int pos = t > 0 ? part[t - 1] : 0;
    for (int c = b; c < e; ++c) {
        const bool kept = Li[(long)c + (long)c * ldl] != 0.0;
        map[c] = (kept && pos < room) ? pos : -1;
        pos += kept;
    }
    if (t == CT - 1) *count = part[CT - 1] < room ? part[CT - 1] : room;
}

// Q[i, q0 + map[c]] = Qr[i, c] for the kept columns (Qr row-major m x k, ld k; Q
// row-major, ld ldq).
__global__ void __launch_bounds__(CT) scatter_cols_kernel(const double* __restrict__ Qr, int m, int k,
                                                          const int* __restrict__ map, double* __restrict__ Q, long ldq,
                                                          int q0) {
    const long tot = (long)m * k;
    for (long e = (long)blockIdx.x * CT + threadIdx.x; e < tot; e += (long)gridDim.x * CT) {
        const long i = e / k;
        const int c = (int)(e - i * k);
        const int p = map[c];
        if (p >= 0) Q[i * ldq + q0 + p] = Qr[e];
    }
}

void append_kept_columns(const double* Qr, int m, int k, const double* Li, long ldl, double* Q, long ldq, int q0,
                         int room, int* map, int* count, hipStream_t s) {
    hipLaunchKernelGGL(kept_map_kernel, dim3(1), dim3(CT), 0, s, Li, ldl, k, room, map, count);
    const long tot = (long)m * k;
    const int grid = (int)((tot + CT - 1) / CT < 2048 ? (tot + CT - 1) / CT : 2048);
    hipLaunchKernelGGL(scatter_cols_kernel, dim3(grid), dim3(CT), 0, s, Qr, m, k, map, Q, ldq, q0);
}

// Settles candidates without their residual spectrum.  With b_C^2 = S - sum L and
// tr(G_R) = ||B||^2 - ||P||^2, the r largest of L u lam sum to at least sum L and at
// most sum L + tr(G_R), so b_C^2 + ||P||^2 <= b^2 <= b_C^2 + ||B||^2.  flag = 0 when the
// lower end exceeds eps^2 (S + ||B||^2) (rejected), 2 when the upper end is below it
// (accepted), 1 otherwise; a band of 1e-8 (S + ||B||^2) around the threshold, far wider
// than the rounding of either end, is left to the certificate proper.  One block.
__global__ void __launch_bounds__(CT) resid_screen_kernel(const ScreenDesc* __restrict__ descs, int count,
                                                          const double* __restrict__ L, int r,
                                                          const double* __restrict__ S, double eps2) {
    __shared__ double red[CT], red2[CT];
    __shared__ double bc[2];
    const int t = threadIdx.x;
    double hi = 0.0, lo = 0.0;
    for (int i = t; i < r; i += CT) dd_add(hi, lo, L[i]);
    red[t] = hi;
    red2[t] = lo;
    __syncthreads();
    if (t == 0) {
        double h = S[0], l = S[1];
        for (int i = 0; i < CT; ++i) {
            dd_add(h, l, -red[i]);
            l -= red2[i];
        }
        bc[0] = h;
        bc[1] = l;
    }
    __syncthreads();
    const double b2c = bc[0] + bc[1];
    const double s_c = S[0] + S[1];
    for (int i = t; i < count; i += CT) {
        const ScreenDesc D = descs[i];
        const double a = D.nb[0] + D.nb[1];
        const double tot = s_c + a;
        const double thr = eps2 * tot, band = 1e-8 * tot;
        const double lower = b2c + *D.pn, upper = b2c + a;
        int f = 1;
        if (lower > thr + band) f = 0;
        else if (upper < thr - band) f = 2;
        *D.flag = f;
    }
}

void resid_screen(const ScreenDesc* d_descs, int count, const double* L, int r, const double* S, double eps,
                  hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(resid_screen_kernel, dim3(1), dim3(CT), 0, s, d_descs, count, L, r, S, eps * eps);
}

__global__ void fill_f64_kernel(double* __restrict__ x, long n, double v) {
    for (long i = (long)blockIdx.x * CT + threadIdx.x; i < n; i += (long)gridDim.x * CT) x[i] = v;
}

void fill_f64(double* x, long n, double v, hipStream_t s) {
    if (n <= 0) return;
    const long g = (n + CT - 1) / CT;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((int)(g > 1024 ? 1024 : g)), dim3(CT), 0, s, x, n, v);
}

// x[i] uniform in [-1, 1) from a counter-based hash of (seed, i) (SplitMix64 finaliser):
// a reproducible start basis for subspace iteration.
__global__ void fill_hash_kernel(double* __restrict__ x, long n, unsigned long long seed) {
    for (long i = (long)blockIdx.x * CT + threadIdx.x; i < n; i += (long)gridDim.x * CT) {
        unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        x[i] = (double)(z >> 11) * 0x1p-52 - 1.0;
    }
}

void fill_hash(double* x, long n, unsigned long long seed, hipStream_t s) {
    if (n <= 0) return;
    const long g = (n + CT - 1) / CT;
    hipLaunchKernelGGL(fill_hash_kernel, dim3((int)(g > 1024 ? 1024 : g)), dim3(CT), 0, s, x, n, seed);
}

}  // namespace cmsvd
