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

template <typename TA, typename TB, bool TA_T, bool TB_T>
__global__ void __launch_bounds__(256) gemm_f64_kernel(const GemmDesc* __restrict__ descs, int base,
                                                       double alpha, double beta) {
    const GemmDesc d = descs[base + blockIdx.y];
    const int tilesM = (d.M + GBM - 1) / GBM;
    const int tilesN = (d.N + GBN - 1) / GBN;
    if ((int)blockIdx.x >= tilesM * tilesN) return;
    const int tm = blockIdx.x % tilesM, tn = blockIdx.x / tilesM;
    const int m0 = tm * GBM, n0 = tn * GBN;
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
    const int nk = (d.K + GBK - 1) / GBK;
    load_tile_regs<TA, TA_T>(A, d.lda, d.M, d.K, m0, 0, ra, t);
    load_tile_regs<TB, !TB_T>(B, d.ldb, d.N, d.K, n0, 0, rb, t);
    store_tile_lds<TA_T>(As[0], ra, t);
    store_tile_lds<!TB_T>(Bs[0], rb, t);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) {
            load_tile_regs<TA, TA_T>(A, d.lda, d.M, d.K, m0, (kt + 1) * GBK, ra, t);
            load_tile_regs<TB, !TB_T>(B, d.ldb, d.N, d.K, n0, (kt + 1) * GBK, rb, t);
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
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * 32 + bi * 16 + (lane >> 4) + 4 * v;
                const int col = n0 + wn * 32 + bj * 16 + (lane & 15);
                if (row < d.M && col < d.N) {
                    double* c = d.C + (long)row + (long)col * d.ldc;
                    double val = alpha * acc[bi][bj][v];
                    if (beta != 0.0) val += beta * (*c);
                    *c = val;
                }
            }
}

template <typename TA, typename TB>
static void launch_typed(const GemmDesc* descs, int count, int maxM, int maxN, bool ta, bool tb,
                         double alpha, double beta, hipStream_t s) {
    const int tiles = ((maxM + GBM - 1) / GBM) * ((maxN + GBN - 1) / GBN);
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        dim3 grid(tiles, n), block(256);
        if (!ta && !tb) hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, false, false>), grid, block, 0, s, descs, base, alpha, beta);
        if (!ta && tb) hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, false, true>), grid, block, 0, s, descs, base, alpha, beta);
        if (ta && !tb) hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, true, false>), grid, block, 0, s, descs, base, alpha, beta);
        if (ta && tb) hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, true, true>), grid, block, 0, s, descs, base, alpha, beta);
    }
}

void gemm_f64_batched(const GemmDesc* d_descs, int count, int maxM, int maxN, bool transA, bool transB,
                      bool a_f32, bool b_f32, double alpha, double beta, hipStream_t s) {
    if (count <= 0 || maxM <= 0 || maxN <= 0) return;
    if (a_f32 && b_f32) launch_typed<float, float>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, s);
    else if (a_f32) launch_typed<float, double>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, s);
    else if (b_f32) launch_typed<double, float>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, s);
    else launch_typed<double, double>(d_descs, count, maxM, maxN, transA, transB, alpha, beta, s);
}

}  // namespace cmsvd
