// Grouped batched FP64 GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
//   C_b = alpha * op(A_b) * op(B_b) + beta * C_b      for b = 0 .. count-1
//
// All matrices are column-major with per-problem leading dimensions; op() is the
// identity or the transpose.  A and B may be stored in FP32 or FP64 (converted to
// FP64 exactly while staging into LDS); accumulation and C are FP64.  Each problem
// carries its own M, N, K so that uneven block widths share one launch.
//
// Tiling: a 256-thread workgroup owns a 64x64 tile of C; its four waves each own a
// 32x32 quadrant made of 2x2 MFMA 16x16 blocks.  K advances in steps of 16 through a
// double-buffered LDS stage: the next K-slab is fetched into registers while the
// matrix cores work on the current one.
#include "common.hpp"
#include "kernels.hpp"

namespace cmsvd {

constexpr int GBM = 64, GBN = 64, GBK = 16;
constexpr int GPAD = 2;  // LDS row padding (doubles)

typedef double d4_t __attribute__((ext_vector_type(4)));

template <typename T, bool TRANS>
__device__ __forceinline__ void load_tile_regs(const T* __restrict__ P, long ld, int rows, int cols,
                                               int r0, int c0, double (&reg)[4], int t) {
    // Loads the 64 x 16 slab op(P)[r0:r0+64, c0:c0+16] (rows index the free dimension,
    // cols the contraction dimension).  !TRANS: P is rows x cols column-major.
    //  TRANS: P is cols x rows column-major (we read op(P) = P^T).
    if (!TRANS) {
        const int kk = t >> 4, i0 = (t & 15) * 4;
        const int c = c0 + kk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 + i0 + q;
            reg[q] = (r < rows && c < cols) ? to_d(P[(long)r + (long)c * ld]) : 0.0;
        }
    } else {
        const int i = t >> 2, k0 = (t & 3) * 4;
        const int r = r0 + i;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = c0 + k0 + q;
            reg[q] = (r < rows && c < cols) ? to_d(P[(long)c + (long)r * ld]) : 0.0;
        }
    }
}

template <bool TRANS>
__device__ __forceinline__ void store_tile_lds(double (*S)[GBM + GPAD], const double (&reg)[4], int t) {
    if (!TRANS) {
        const int kk = t >> 4, i0 = (t & 15) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) S[kk][i0 + q] = reg[q];
    } else {
        const int i = t >> 2, k0 = (t & 3) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) S[k0 + q][i] = reg[q];
    }
}

// Split K (ksplit > 1): blockIdx.x = split * maxTiles + tile; the workgroup contracts the
// K range [split * Kc, (split + 1) * Kc) (Kc a multiple of 16) and writes its unscaled
// partial tile to part (ksplit partials of maxM x maxN per problem, column-major);
// gemm_splitk_reduce then sums the partials in split order and applies alpha and beta.
template <typename TA, typename TB, bool TA_T, bool TB_T>
__global__ void __launch_bounds__(256) gemm_f64_kernel(const GemmDesc* __restrict__ descs, int base,
                                                       double alpha, double beta, int ksplit, int maxTiles,
                                                       int maxM, int maxN, double* __restrict__ part) {
    const GemmDesc d = descs[base + blockIdx.y];
    const int tilesM = (d.M + GBM - 1) / GBM;
    const int tilesN = (d.N + GBN - 1) / GBN;
    const int split = (int)blockIdx.x / maxTiles, tile = (int)blockIdx.x % maxTiles;
    if (tile >= tilesM * tilesN) return;
    const int tm = tile % tilesM, tn = tile / tilesM;
    const int m0 = tm * GBM, n0 = tn * GBN;
    int kbeg = 0, kend = d.K;
    if (ksplit > 1) {
        const int kc = ((d.K + ksplit - 1) / ksplit + GBK - 1) / GBK * GBK;
        kbeg = split * kc < d.K ? split * kc : d.K;
        kend = kbeg + kc < d.K ? kbeg + kc : d.K;
    }
    const TA* __restrict__ A = static_cast<const TA*>(d.A);
    const TB* __restrict__ B = static_cast<const TB*>(d.B);

    __shared__ double As[2][GBK][GBM + GPAD];
    __shared__ double Bs[2][GBK][GBN + GPAD];

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    d4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    // op(A) is M x K; op(B) is K x N, staged as its transpose (N x K) so that both
    // operands share the (free index, contraction index) slab loader.
    double ra[4], rb[4];
    const int nk = (kend - kbeg + GBK - 1) / GBK;
    load_tile_regs<TA, TA_T>(A, d.lda, d.M, kend, m0, kbeg, ra, t);
    load_tile_regs<TB, !TB_T>(B, d.ldb, d.N, kend, n0, kbeg, rb, t);
    store_tile_lds<TA_T>(As[0], ra, t);
    store_tile_lds<!TB_T>(Bs[0], rb, t);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) {
            load_tile_regs<TA, TA_T>(A, d.lda, d.M, kend, m0, kbeg + (kt + 1) * GBK, ra, t);
            load_tile_regs<TB, !TB_T>(B, d.ldb, d.N, kend, n0, kbeg + (kt + 1) * GBK, rb, t);
        }
#pragma unroll
        for (int k4 = 0; k4 < GBK / 4; ++k4) {
            const int krow = k4 * 4 + (lane >> 4);
            double a0 = As[cur][krow][wm * 32 + (lane & 15)];
            double a1 = As[cur][krow][wm * 32 + 16 + (lane & 15)];
            double b0 = Bs[cur][krow][wn * 32 + (lane & 15)];
            double b1 = Bs[cur][krow][wn * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (kt + 1 < nk) {
            store_tile_lds<TA_T>(As[cur ^ 1], ra, t);
            store_tile_lds<!TB_T>(Bs[cur ^ 1], rb, t);
        }
        __syncthreads();
    }
    // D[i][j] of a 16x16 FP64 block sits in lane j + 16*(i%4), element i/4.
    double* pt = part ? part + ((long)(base + blockIdx.y) * ksplit + split) * (long)maxM * maxN : nullptr;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + bi * 16 + (lane >> 4) + 4 * v;
                const int col = n0 + wn * 32 + bj * 16 + (lane & 15);
                if (row < d.M && col < d.N) {
                    if (pt) {
                        pt[(long)row + (long)col * maxM] = acc[bi][bj][v];
                    } else {
                        double* c = d.C + (long)row + (long)col * d.ldc;
                        double val = alpha * acc[bi][bj][v];
                        if (beta != 0.0) val += beta * (*c);
                        *c = val;
                    }
                }
            }
}

// C = alpha * (sum of the ksplit partials, in split order) + beta * C, per problem.
__global__ void __launch_bounds__(256) gemm_splitk_reduce(const GemmDesc* __restrict__ descs, int base, double alpha,
                                                          double beta, int ksplit, int maxM, int maxN,
                                                          const double* __restrict__ part) {
    const GemmDesc d = descs[base + blockIdx.y];
    const long tot = (long)d.M * d.N;
    const double* pb = part + (long)(base + blockIdx.y) * ksplit * (long)maxM * maxN;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
        const int col = (int)(e / d.M), row = (int)(e - (long)col * d.M);
        double sum = 0.0;
        for (int sp = 0; sp < ksplit; ++sp) sum += pb[(long)sp * maxM * maxN + row + (long)col * maxM];
        double* c = d.C + (long)row + (long)col * d.ldc;
        double val = alpha * sum;
        if (beta != 0.0) val += beta * (*c);
        *c = val;
    }
}

template <typename TA, typename TB>
static void launch_typed(const GemmDesc* descs, int count, int maxM, int maxN, bool ta, bool tb,
                         double alpha, double beta, int ksplit, double* part, hipStream_t s) {
    const int tiles = ((maxM + GBM - 1) / GBM) * ((maxN + GBN - 1) / GBN);
    const int ks = part ? ksplit : 1;
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        dim3 grid(tiles * ks, n), block(256);
        if (!ta && !tb) hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, false, false>), grid, block, 0, s, descs, base, alpha, beta, ks, tiles, maxM, maxN, part);
        if (!ta && tb) hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, false, true>), grid, block, 0, s, descs, base, alpha, beta, ks, tiles, maxM, maxN, part);
        if (ta && !tb) hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, true, false>), grid, block, 0, s, descs, base, alpha, beta, ks, tiles, maxM, maxN, part);
        if (ta && tb) hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, true, true>), grid, block, 0, s, descs, base, alpha, beta, ks, tiles, maxM, maxN, part);
        if (part) {
            const long el = (long)maxM * maxN;
            const int g = (int)((el + 255) / 256 < 64 ? (el + 255) / 256 : 64);
            hipLaunchKernelGGL(gemm_splitk_reduce, dim3(g, n), dim3(256), 0, s, descs, base, alpha, beta, ks, maxM, maxN,
                               (const double*)part);
        }
    }
}

void gemm_f64_batched(const GemmDesc* d_descs, int count, int maxM, int maxN, bool transA, bool transB,
                      bool a_f32, bool b_f32, double alpha, double beta, hipStream_t s, int ksplit, double* part) {
    if (count <= 0 || maxM <= 0 || maxN <= 0) return;
    if (ksplit <= 1) part = nullptr;
    if (a_f32 && b_f32) launch_typed<float, float>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, ksplit, part, s);
    else if (a_f32) launch_typed<float, double>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, ksplit, part, s);
    else if (b_f32) launch_typed<double, float>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, ksplit, part, s);
    else launch_typed<double, double>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, ksplit, part, s);
}

// ---------------------------------------------------------------------------
// Grouped batched GEMM with BF16 operands and FP32 accumulation on the CDNA4 matrix
// cores (v_mfma_f32_16x16x32_bf16), for the low-precision projection options.
//
//   C_b = alpha * op(A_b) * op(B_b) + beta * C_b      (C FP64, column-major)
//
// Every operand element x is rounded to FP32 (x32) and then to BF16 (hi), both
// round-to-nearest-even, while it is staged into LDS.  SPLIT = 1: op(A) op(B) is summed
// from the hi parts.  SPLIT = 3 also stages lo = BF16(x32 - hi) (the FP32 difference is
// exact) and sums lo_A hi_B + hi_A lo_B + hi_A hi_B, which carries about 16 significant
// bits per operand instead of 8.  Products of BF16 values are exact in FP32; the matrix
// cores sum them in FP32 and C receives the FP32 sums widened to FP64.
//
// Tiling: as the FP64 kernel, a 256-thread workgroup owns a 64x64 tile of C and each
// wave a 32x32 quadrant of 2x2 MFMA blocks; K advances by 32 (one MFMA depth) through
// a double-buffered LDS stage holding the operand parts as [free index][32 K values]
// rows of BF16, so that each lane's 8 consecutive K values are one 16-byte LDS read.
// ---------------------------------------------------------------------------
constexpr int BBK = 32;
constexpr int BROW = BBK + 8;  // LDS row length in BF16 (16-byte padding)

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float to_f32(double x) { return (float)x; }
__device__ __forceinline__ float to_f32(float x) { return x; }

// Loads 8 elements of the 64 x 32 slab op(X)[f0:f0+64, k0:k0+32] (free index f,
// contraction index k) and splits them into BF16 parts hi (and lo when SPLIT).
// KCONTIG: element (f, k) at X[k + f*ld] (the contraction index is contiguous; thread
// t takes row t/4, K values 8*(t%4)..+7); otherwise at X[f + k*ld] (thread t takes row
// t%64, K values 8*(t/64)..+7, so that a wave reads 64 consecutive free indices per
// load).
template <typename T, bool KCONTIG, bool SPLIT>
__device__ __forceinline__ void load_slab_bf16(const T* __restrict__ X, long ld, int nf, int nk, int f0, int k0,
                                               int t, bf8_t& hi, bf8_t& lo, int& row, int& kg) {
    if (KCONTIG) {
        row = t >> 2;
        kg = t & 3;
    } else {
        row = t & 63;
        kg = t >> 6;
    }
    const int f = f0 + row;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = k0 + kg * 8 + q;
        const bool in = f < nf && k < nk;
        const long idx = KCONTIG ? (long)k + (long)f * ld : (long)f + (long)k * ld;
        const float x = in ? to_f32(X[idx]) : 0.0f;
        const __bf16 h = (__bf16)x;
        hi[q] = h;
        if (SPLIT) lo[q] = (__bf16)(x - (float)h);
    }
}

template <typename TA, typename TB, bool TA_T, bool TB_T, bool SPLIT>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(const GemmDesc* __restrict__ descs, int base,
                                                        double alpha, double beta) {
    const GemmDesc d = descs[base + blockIdx.y];
    const int tilesM = (d.M + GBM - 1) / GBM;
    const int tilesN = (d.N + GBN - 1) / GBN;
    if ((int)blockIdx.x >= tilesM * tilesN) return;
    const int tm = blockIdx.x % tilesM, tn = blockIdx.x / tilesM;
    const int m0 = tm * GBM, n0 = tn * GBN;
    const TA* __restrict__ A = static_cast<const TA*>(d.A);
    const TB* __restrict__ B = static_cast<const TB*>(d.B);
    // op(A) = A (M x K, free index contiguous) or A^T (K contiguous);
    // op(B) = B (K x N, K contiguous) or B^T (free index contiguous).
    constexpr bool AK = TA_T, BK = !TB_T;
    constexpr int NP = SPLIT ? 2 : 1;  // staged parts per operand

    __shared__ __attribute__((aligned(16))) __bf16 As[2][NP][GBM * BROW];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][NP][GBN * BROW];

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    f4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};

    bf8_t ah, al, bh, bl;
    int ra, ka, rb, kb;
    const int nk = (d.K + BBK - 1) / BBK;
    auto stage = [&](int buf) {
        *reinterpret_cast<bf8_t*>(&As[buf][0][ra * BROW + ka * 8]) = ah;
        *reinterpret_cast<bf8_t*>(&Bs[buf][0][rb * BROW + kb * 8]) = bh;
        if (SPLIT) {
            *reinterpret_cast<bf8_t*>(&As[buf][NP - 1][ra * BROW + ka * 8]) = al;
            *reinterpret_cast<bf8_t*>(&Bs[buf][NP - 1][rb * BROW + kb * 8]) = bl;
        }
    };
    load_slab_bf16<TA, AK, SPLIT>(A, d.lda, d.M, d.K, m0, 0, t, ah, al, ra, ka);
    load_slab_bf16<TB, BK, SPLIT>(B, d.ldb, d.N, d.K, n0, 0, t, bh, bl, rb, kb);
    stage(0);
    __syncthreads();
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) {
            load_slab_bf16<TA, AK, SPLIT>(A, d.lda, d.M, d.K, m0, (kt + 1) * BBK, t, ah, al, ra, ka);
            load_slab_bf16<TB, BK, SPLIT>(B, d.ldb, d.N, d.K, n0, (kt + 1) * BBK, t, bh, bl, rb, kb);
        }
        // A operand: lane holds row (lane % 16), K values 8*(lane/16)..+7; B operand:
        // column (lane % 16), the same K values.
        bf8_t a[NP][2], b[NP][2];
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[p][i] = *reinterpret_cast<const bf8_t*>(&As[cur][p][(wm * 32 + i * 16 + lr) * BROW + lk]);
                b[p][i] = *reinterpret_cast<const bf8_t*>(&Bs[cur][p][(wn * 32 + i * 16 + lr) * BROW + lk]);
            }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (SPLIT) {  // the small cross terms first
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[NP - 1][i], b[0][j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[NP - 1][j], acc[i][j], 0, 0, 0);
                }
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
            }
        if (kt + 1 < nk) stage(cur ^ 1);
        __syncthreads();
    }
    // D[i][j] of a 16x16 FP32 block sits in lane j + 16*(i/4), element i%4.
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + bi * 16 + (lane >> 4) * 4 + v;
                const int col = n0 + wn * 32 + bj * 16 + (lane & 15);
                if (row < d.M && col < d.N) {
                    double* c = d.C + (long)row + (long)col * d.ldc;
                    double val = alpha * (double)acc[bi][bj][v];
                    if (beta != 0.0) val += beta * (*c);
                    *c = val;
                }
            }
}

template <typename TA, typename TB, bool SPLIT>
static void launch_bf16(const GemmDesc* descs, int count, int maxM, int maxN, bool ta, bool tb, double alpha,
                        double beta, hipStream_t s) {
    const int tiles = ((maxM + GBM - 1) / GBM) * ((maxN + GBN - 1) / GBN);
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        dim3 grid(tiles, n), block(256);
        if (!ta && !tb) hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, false, false, SPLIT>), grid, block, 0, s, descs, base, alpha, beta);
        if (!ta && tb) hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, false, true, SPLIT>), grid, block, 0, s, descs, base, alpha, beta);
        if (ta && !tb) hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, true, false, SPLIT>), grid, block, 0, s, descs, base, alpha, beta);
        if (ta && tb) hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, true, true, SPLIT>), grid, block, 0, s, descs, base, alpha, beta);
    }
}

template <bool SPLIT>
static void launch_bf16_types(const GemmDesc* d, int count, int maxM, int maxN, bool ta, bool tb, bool a_f32,
                              bool b_f32, double alpha, double beta, hipStream_t s) {
    if (a_f32 && b_f32) launch_bf16<float, float, SPLIT>(d, count, maxM, maxN, ta, tb, alpha, beta, s);
    else if (a_f32) launch_bf16<float, double, SPLIT>(d, count, maxM, maxN, ta, tb, alpha, beta, s);
    else if (b_f32) launch_bf16<double, float, SPLIT>(d, count, maxM, maxN, ta, tb, alpha, beta, s);
    else launch_bf16<double, double, SPLIT>(d, count, maxM, maxN, ta, tb, alpha, beta, s);
}

void gemm_bf16_batched(const GemmDesc* d_descs, int count, int maxM, int maxN, bool transA, bool transB,
                       bool a_f32, bool b_f32, int passes, double alpha, double beta, hipStream_t s) {
    if (count <= 0 || maxM <= 0 || maxN <= 0) return;
    if (passes == 3) launch_bf16_types<true>(d_descs, count, maxM, maxN, transA, transB, a_f32, b_f32, alpha, beta, s);
    else launch_bf16_types<false>(d_descs, count, maxM, maxN, transA, transB, a_f32, b_f32, alpha, beta, s);
}

// ---------------------------------------------------------------------------
// Grouped batched GEMM with FP32 operands and FP32 accumulation on the CDNA4 matrix
// cores (v_mfma_f32_16x16x4f32), for the FP32 projection option.
//
//   C_b = alpha * op(A_b) * op(B_b) + beta * C_b      (C FP64, column-major)
//
// Every operand element is rounded to FP32 (round-to-nearest-even; FP32 data stays as
// it is) while it is staged into LDS; the matrix cores sum the products in FP32 and C
// receives the sums widened to FP64.  Tiling as the FP64 kernel (a 64 x 64 C tile per
// 256-thread workgroup, a 32 x 32 quadrant of 2 x 2 MFMA blocks per wave), with K
// slabs of 32 (half the LDS bytes per element, so twice the depth per barrier),
// double-buffered.
// ---------------------------------------------------------------------------
constexpr int FBK = 32;
constexpr int FPAD = 4;  // LDS row padding (floats)

template <bool TRANS>
__device__ __forceinline__ void store_tile_lds_f32(float (*S)[GBM + FPAD], const double (&reg)[4], int t, int k0) {
    if (!TRANS) {
        const int kk = t >> 4, i0 = (t & 15) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) S[k0 + kk][i0 + q] = (float)reg[q];
    } else {
        const int i = t >> 2, kq = (t & 3) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) S[k0 + kq + q][i] = (float)reg[q];
    }
}

template <typename TA, typename TB, bool TA_T, bool TB_T>
__global__ void __launch_bounds__(256) gemm_f32_kernel(const GemmDesc* __restrict__ descs, int base,
                                                       double alpha, double beta) {
    const GemmDesc d = descs[base + blockIdx.y];
    const int tilesM = (d.M + GBM - 1) / GBM;
    const int tilesN = (d.N + GBN - 1) / GBN;
    if ((int)blockIdx.x >= tilesM * tilesN) return;
    const int tm = blockIdx.x % tilesM, tn = blockIdx.x / tilesM;
    const int m0 = tm * GBM, n0 = tn * GBN;
    const TA* __restrict__ A = static_cast<const TA*>(d.A);
    const TB* __restrict__ B = static_cast<const TB*>(d.B);

    __shared__ float As[2][FBK][GBM + FPAD];
    __shared__ float Bs[2][FBK][GBN + FPAD];

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    f4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};

    // a slab of 32 K values is two 64 x 16 half-slabs of the FP64 kernel's loader (the
    // values are exact in FP64 and rounded once, to FP32, when stored)
    double ra[2][4], rb[2][4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int hs = 0; hs < 2; ++hs) {
            load_tile_regs<TA, TA_T>(A, d.lda, d.M, d.K, m0, k0 + 16 * hs, ra[hs], t);
            load_tile_regs<TB, !TB_T>(B, d.ldb, d.N, d.K, n0, k0 + 16 * hs, rb[hs], t);
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int hs = 0; hs < 2; ++hs) {
            store_tile_lds_f32<TA_T>(As[buf], ra[hs], t, 16 * hs);
            store_tile_lds_f32<!TB_T>(Bs[buf], rb[hs], t, 16 * hs);
        }
    };
    const int nk = (d.K + FBK - 1) / FBK;
    fetch(0);
    stage(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) fetch((kt + 1) * FBK);
        // A operand: lane holds row (lane % 16), K value lane / 16 of the 4-deep step;
        // B operand: column (lane % 16), the same K value.
#pragma unroll
        for (int k4 = 0; k4 < FBK / 4; ++k4) {
            const int krow = k4 * 4 + (lane >> 4);
            const float a0 = As[cur][krow][wm * 32 + (lane & 15)];
            const float a1 = As[cur][krow][wm * 32 + 16 + (lane & 15)];
            const float b0 = Bs[cur][krow][wn * 32 + (lane & 15)];
            const float b1 = Bs[cur][krow][wn * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (kt + 1 < nk) stage(cur ^ 1);
        __syncthreads();
    }
    // D[i][j] of a 16x16 FP32 block sits in lane j + 16*(i/4), element i%4.
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + bi * 16 + (lane >> 4) * 4 + v;
                const int col = n0 + wn * 32 + bj * 16 + (lane & 15);
                if (row < d.M && col < d.N) {
                    double* c = d.C + (long)row + (long)col * d.ldc;
                    double val = alpha * (double)acc[bi][bj][v];
                    if (beta != 0.0) val += beta * (*c);
                    *c = val;
                }
            }
}

// Wide tiles for the candidate projections Y = U^T A_j (op(A) = A and op(B) = B^T, both
// with the free index contiguous in memory): a 512-thread workgroup owns a 64 x 256 tile
// of C, so a 64-column basis is read once per candidate block instead of once per 64
// columns of it; each of the eight waves owns a 32 x 64 part (2 x 4 MFMA blocks).  K
// advances by 32 through one LDS stage while the next slab waits in registers (45 KB
// of LDS: three workgroups per CU).  Operands are read four consecutive elements at a
// time (one 16-byte load where the problem's pointer and leading dimension allow it),
// rounded to FP32 as they are staged, and every lane stores its four consecutive rows
// of C as two 16-byte stores where possible.
constexpr int WBM = 64, WBN = 256, WBK = 32, WTH = 512;
constexpr int WPAD = 16;  // LDS row padding (floats): rows k and k + 1 fall 16 banks apart

template <typename T>
__device__ __forceinline__ f4_t load4_f32(const T* __restrict__ P, long off, int nvalid, bool vec) {
    f4_t r;
    if (vec && nvalid >= 4) {
        if constexpr (sizeof(T) == 4) {
            r = *reinterpret_cast<const f4_t*>(P + off);
        } else {
            typedef double d2_t __attribute__((ext_vector_type(2)));
            const d2_t x0 = *reinterpret_cast<const d2_t*>(P + off);
            const d2_t x1 = *reinterpret_cast<const d2_t*>(P + off + 2);
            r = f4_t{(float)x0[0], (float)x0[1], (float)x1[0], (float)x1[1]};
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) r[q] = q < nvalid ? (float)P[off + q] : 0.0f;
    }
    return r;
}

template <typename TA, typename TB>
__global__ void __launch_bounds__(WTH) gemm_f32_wide_kernel(const GemmDesc* __restrict__ descs, int base,
                                                            double alpha, double beta) {
    const GemmDesc d = descs[base + blockIdx.y];
    const int tilesM = (d.M + WBM - 1) / WBM;
    const int tilesN = (d.N + WBN - 1) / WBN;
    if ((int)blockIdx.x >= tilesM * tilesN) return;
    const int tm = blockIdx.x % tilesM, tn = blockIdx.x / tilesM;
    const int m0 = tm * WBM, n0 = tn * WBN;
    const TA* __restrict__ A = static_cast<const TA*>(d.A);
    const TB* __restrict__ B = static_cast<const TB*>(d.B);
    const bool vecA = (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (d.lda & 3) == 0;
    const bool vecB = (reinterpret_cast<uintptr_t>(B) & 15) == 0 && (d.ldb & 3) == 0;

    __shared__ float As[WBK][WBM + WPAD];
    __shared__ float Bs[WBK][WBN + WPAD];

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 2, wn = w & 3;
    f4_t acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};

    // slab k0 .. k0 + 31: thread t holds A rows m0 + 4 (t % 16) .. + 3 at k0 + t / 16, and
    // four runs of B: chunk c = t + 512 q covers k0 + c / 64, columns n0 + 4 (c % 64) .. + 3
    const int ak = t >> 4, ai = (t & 15) * 4;
    f4_t ra, rb[4];
    auto fetch = [&](int k0) {
        const int kk = k0 + ak;
        const int nva = kk < d.K ? min(4, d.M - (m0 + ai)) : 0;
        ra = load4_f32<TA>(A, (long)(m0 + ai) + (long)kk * d.lda, nva, vecA);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = t + WTH * q, bk = k0 + (c >> 6), bn = n0 + (c & 63) * 4;
            const int nvb = bk < d.K ? min(4, d.N - bn) : 0;
            rb[q] = load4_f32<TB>(B, (long)bn + (long)bk * d.ldb, nvb, vecB);
        }
    };
    auto stage = [&]() {
        *reinterpret_cast<f4_t*>(&As[ak][ai]) = ra;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = t + WTH * q;
            *reinterpret_cast<f4_t*>(&Bs[c >> 6][(c & 63) * 4]) = rb[q];
        }
    };
    const int nk = (d.K + WBK - 1) / WBK;
    fetch(0);
    stage();
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) fetch((kt + 1) * WBK);
        // A operand: lane holds row (lane % 16), K value lane / 16 of the 4-deep step;
        // B operand: column (lane % 16), the same K value.
#pragma unroll
        for (int k4 = 0; k4 < WBK / 4; ++k4) {
            const int krow = k4 * 4 + (lane >> 4);
            float a[2], b[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[krow][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[krow][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
        if (kt + 1 < nk) {
            stage();
            __syncthreads();
        }
    }
    // D[i][j] of a 16x16 FP32 block sits in lane j + 16*(i/4), element i%4: four
    // consecutive rows of one column of C per lane
    const bool vecC = beta == 0.0 && (reinterpret_cast<uintptr_t>(d.C) & 15) == 0 && (d.ldc & 1) == 0;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
            const int row = m0 + wm * 32 + bi * 16 + (lane >> 4) * 4;
            const int col = n0 + wn * 64 + bj * 16 + (lane & 15);
            if (col >= d.N) continue;
            double* c = d.C + (long)row + (long)col * d.ldc;
            if (vecC && row + 3 < d.M) {
                typedef double d2_t __attribute__((ext_vector_type(2)));
                *reinterpret_cast<d2_t*>(c) = d2_t{alpha * (double)acc[bi][bj][0], alpha * (double)acc[bi][bj][1]};
                *reinterpret_cast<d2_t*>(c + 2) = d2_t{alpha * (double)acc[bi][bj][2], alpha * (double)acc[bi][bj][3]};
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (row + v < d.M) {
                        double val = alpha * (double)acc[bi][bj][v];
                        if (beta != 0.0) val += beta * c[v];
                        c[v] = val;
                    }
            }
        }
}

template <typename TA, typename TB>
static void launch_f32(const GemmDesc* descs, int count, int maxM, int maxN, bool ta, bool tb, double alpha,
                       double beta, hipStream_t s) {
    if (!ta && tb && maxN > GBN) {
        // projections of candidate blocks wider than one 64-column tile: wide tiles
        const int wt = ((maxM + WBM - 1) / WBM) * ((maxN + WBN - 1) / WBN);
        for (int base = 0; base < count; base += 65535) {
            const int n = count - base < 65535 ? count - base : 65535;
            hipLaunchKernelGGL((gemm_f32_wide_kernel<TA, TB>), dim3(wt, n), dim3(WTH), 0, s, descs, base, alpha, beta);
        }
        return;
    }
    const int tiles = ((maxM + GBM - 1) / GBM) * ((maxN + GBN - 1) / GBN);
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        dim3 grid(tiles, n), block(256);
        if (!ta && !tb) hipLaunchKernelGGL((gemm_f32_kernel<TA, TB, false, false>), grid, block, 0, s, descs, base, alpha, beta);
        if (!ta && tb) hipLaunchKernelGGL((gemm_f32_kernel<TA, TB, false, true>), grid, block, 0, s, descs, base, alpha, beta);
        if (ta && !tb) hipLaunchKernelGGL((gemm_f32_kernel<TA, TB, true, false>), grid, block, 0, s, descs, base, alpha, beta);
        if (ta && tb) hipLaunchKernelGGL((gemm_f32_kernel<TA, TB, true, true>), grid, block, 0, s, descs, base, alpha, beta);
    }
}

void gemm_f32_batched(const GemmDesc* d_descs, int count, int maxM, int maxN, bool transA, bool transB,
                      bool a_f32, bool b_f32, double alpha, double beta, hipStream_t s) {
    if (count <= 0 || maxM <= 0 || maxN <= 0) return;
    if (a_f32 && b_f32) launch_f32<float, float>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, s);
    else if (a_f32) launch_f32<float, double>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, s);
    else if (b_f32) launch_f32<double, float>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, s);
    else launch_f32<double, double>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, s);
}

}  // namespace cmsvd
