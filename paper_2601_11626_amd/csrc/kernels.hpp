// Internal kernel descriptors and launchers of the cmsvd HIP library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmsvd {

// One GEMM problem: C = alpha op(A) op(B) + beta C, column-major, FP64 accumulate.
struct GemmDesc {
    const void* A;
    const void* B;
    double* C;
    int M, N, K;
    long lda, ldb, ldc;
};

// ksplit > 1 with part != nullptr splits every problem's K range over ksplit workgroups
// per tile (for launches with few tiles and long K); part holds count * ksplit * maxM *
// maxN doubles of partial products, summed in a fixed order by a second kernel.
void gemm_f64_batched(const GemmDesc* d_descs, int count, int maxM, int maxN, bool transA, bool transB,
                      bool a_f32, bool b_f32, double alpha, double beta, hipStream_t s, int ksplit = 1,
                      double* part = nullptr);
// Same descriptors and semantics with the operands rounded to BF16 (through FP32, both
// round-to-nearest-even) and FP32 accumulation on the matrix cores; C stays FP64.
// passes = 1: hi parts only; 3: lo_A hi_B + hi_A lo_B + hi_A hi_B (split operands).
void gemm_bf16_batched(const GemmDesc* d_descs, int count, int maxM, int maxN, bool transA, bool transB,
                       bool a_f32, bool b_f32, int passes, double alpha, double beta, hipStream_t s);
// Same descriptors and semantics with the operands rounded to FP32 (round-to-nearest-
// even) and FP32 accumulation on the matrix cores; C stays FP64.
void gemm_f32_batched(const GemmDesc* d_descs, int count, int maxM, int maxN, bool transA, bool transB,
                      bool a_f32, bool b_f32, double alpha, double beta, hipStream_t s);

// One symmetric eigenvalue problem of order n, given in block-arrow form
//     H = [[ diag(s)^2        , diag(s) P ],
//          [ P^T diag(s)      , Y         ]]
// with s of length n1, P n1 x (n-n1) (column-major, ldp) and Y (n-n1) x (n-n1)
// symmetric (column-major, ldy, both triangles valid).  n1 = 0 gives a dense Y.
struct EigDesc {
    int n, n1, nkeep;
    const double* s;
    const double* P;
    long ldp;
    const double* Y;
    long ldy;
    // evaluation mode: plug-in error from the total energy E_tot = *na + *nb, each a
    // double-double (hi, lo) in device memory (nb may be null)
    const double* na;
    const double* nb;
    double* out_err;
    double* out_rel;
    // vector mode
    double* lam;      // nkeep eigenvalues, descending
    double* d;        // n   (tridiagonal diagonal)
    double* e;        // n-1 (tridiagonal off-diagonal)
    double* V;        // n x n column-major Householder vectors (column j holds v_j, v_j[j+1] = 1 implicit)
    long ldv;
    double* tau;      // n
    double* sum_top;  // 2 doubles: (hi, lo) of the sum of the kept eigenvalues
    // mode 2, register-resident orders above 160: jsplit > 0 stops the tridiagonalisation
    // after jsplit column steps; d and e then hold entries 0 .. jsplit - 1 and the
    // trailing matrix (order n - jsplit, with every earlier step applied) is written to
    // At (column-major, ld ldt, both triangles) for sym_eig_tail_batched
    double* At;
    long ldt;
    int jsplit;
};

// Tridiagonalisation + bisection.  mode 0: evaluation (writes out_err/out_rel);
// mode 1: vectors wanted (writes lam, d, e, V, tau, sum_top); mode 2: for orders where
// sym_eig_split(nmax) holds (the register-resident orders 161..320), only the
// tridiagonalisation, into each descriptor's d and e (sym_eig_tri_doubles(nmax) doubles
// of scratch), and tri_bisect_batched finishes the evaluation (a high-occupancy
// bisection kernel); for other orders mode 2 is mode 0.
// threads: 0 for the default workgroup of the general kernel (orders above 320: 1024
// threads), or 512 (eight waves per problem); other orders ignore it.
void sym_eig_batched(const EigDesc* d_descs, int count, int nmax, int mode, double* gws, int nslots,
                     hipStream_t s, int threads = 0);
size_t sym_eig_workspace_doubles(int nmax, int nslots);
// Scratch doubles per problem for the tridiagonal of mode 2 (d at 0, e at half of it).
size_t sym_eig_tri_doubles(int nmax);
bool sym_eig_split(int nmax);
// Hand-over levels of the evaluation's tridiagonalisation.  A mode-2 problem of order n
// above orders[0] stops after n - orders[0] steps (jsplit) and writes its trailing matrix;
// level l tridiagonalises trailing matrices of order orders[l] (descriptors with n1 = 0,
// Y = At, d and e pointing at the entries of the full problem that follow) and, except
// the last level, hands its own trailing matrix of order orders[l + 1] over the same way.
// Levels: order 192 (four waves, register and LDS tiles), 160 (four waves, register
// tiles), 64 (one wave per problem); two or more problems share a CU at every level.
int sym_eig_tail_levels(int* orders);
void sym_eig_tail_batched(const EigDesc* d_descs, int count, int level, hipStream_t s);
void tri_bisect_batched(const EigDesc* d_descs, int count, int nmax, hipStream_t s);
// Doubles of global scratch one workgroup slot of sym_eig_batched needs for order nmax
// (0 when the kernel chosen for that order keeps every tile on chip).
size_t sym_eig_slot_doubles(int nmax);
// Evaluation mode for cores of one appended column (every descriptor n = n1 + 1 with
// n1 <= 256 and nkeep >= n1): the arrowhead's smallest eigenvalue, bracketed by the sign
// of the Schur complement of the border (the inertia) with model-based probes; writes
// out_err / out_rel as mode 0 does.  n1max: the largest n1 of the batch (at most 32:
// two problems per wavefront).
void arrow_eig_batched(const EigDesc* d_descs, int count, int n1max, hipStream_t s);
// Largest order the eigenvalue (and eigenvector) kernels accept (2016 on gfx950).
int sym_eig_nmax();

// Inverse iteration on the tridiagonal (lam, d, e) for the nkeep top eigenvectors,
// orthonormalised, then back-transformed by the stored Householder vectors.  Z is
// n x nkeep column-major (ldz).  scratch: per problem 6 * n * nkeep doubles.
struct VecDesc {
    int n, nkeep;
    const double* lam;
    const double* d;
    const double* e;
    const double* V;
    long ldv;
    const double* tau;
    double* Z;
    long ldz;
    double* scratch;
    // nonzero: stop after the orthonormalisation and leave the eigenvectors of the
    // tridiagonal in Z (the caller applies the reflectors, e.g. blocked)
    int skip_bt;
};
void sym_vectors_batched(const VecDesc* d_descs, int count, hipStream_t s);

// Dense evaluation of many pairs: compact records expanded into eigenproblem
// descriptors on the device.  Pair i of a chunk: anchor slot, candidate block, output
// index; the candidate's P is read in place from the chunk's product C
// (P = C + (slot - a0) r + (coff - cmin) ldc).
struct AnchorRec {
    const double* S;   // singular values of the anchor state (r)
    const double* na;  // its energy (double-double)
};
struct CandRec {
    const double* nb;  // energy (double-double)
    const double* G;   // Gram B^T B (k x k)
    long coff;         // first column in the packed candidates
    int k;
};
struct PairRec {
    int slot, cand, out;
};
void expand_dense_descs(const PairRec* pr, int count, const AnchorRec* A, const CandRec* Cr, int r, int a0,
                        const double* C, long ldc, long cmin, double* err, double* rel, EigDesc* out, hipStream_t s);

// Blocked back-transformation helpers.  V (n x n column-major, ldv) holds reflector j
// in column j on rows >= j + 2; materialize_reflectors writes the implicit unit at row
// j + 1 and zeros above it (j < n - 2).  larft: for a block of b reflectors with Gram
// S = V_b^T V_b (b x b, ld ldst) and tau, the upper-triangular T (ld ldst) of
// H_j0 ... H_j0+b-1 = I - V_b T V_b^T.
void materialize_reflectors(double* V, int n, long ldv, hipStream_t s);
struct LarftDesc {
    const double* S;
    const double* tau;
    double* T;
    int b;
    long ld;
};
void larft_batched(const LarftDesc* d_descs, int count, hipStream_t s);

// Semidefinite Cholesky with a pivot threshold, in place on the lower triangle
// of G (column-major, ldg).  A pivot <= thresh zeroes its column of L.  Then
// writes Linv = L^{-1} restricted to the kept pivots (zero rows/cols elsewhere).
struct CholDesc {
    int k;
    double* G;
    long ldg;
    double* Linv;
    long ldi;
    double thresh_scale;        // pivot threshold = thresh_scale * (thresh_ref ? thresh_ref[0] : 1)
    const double* thresh_ref;   // device scalar (e.g. the block energy), may be null
    int* dropped;               // number of dropped pivots (output, may be null)
};
void chol_semidef_batched(const CholDesc* d_descs, int count, hipStream_t s);

// Frobenius norm squared of a row-major m x n block (FP32 or FP64), double-double.
struct NormDesc {
    const void* A;
    int rows, cols;
    long ld;
    int f32;
    double* out;  // 2 doubles (hi, lo)
};
void sumsq_batched(const NormDesc* d_descs, int count, hipStream_t s);

// Copy a row-major block (FP32/FP64) into FP64 storage with a new row stride.
struct CopyDesc {
    const void* A;
    int rows, cols;
    long lda;
    int f32;
    double* B;
    long ldb;
};
void copy_f64_batched(const CopyDesc* d_descs, int count, int maxrows, hipStream_t s);

// KT = [[diag(s), 0], [P^T, F]] ((r+k) x (r+k), column-major, ldk), F lower k x k.
struct KtDesc {
    int r, k;
    const double* s;
    const double* P;
    long ldp;
    const double* F;
    long ldf;
    double* KT;
    long ldk;
};
void assemble_kt_batched(const KtDesc* d_descs, int count, int nmax, hipStream_t s);

// Commit a state: s_out[q] = sqrt(lam[q]) (0 when lam[q] <= cut or q >= nkeep), the
// matching columns of the row-major m x r basis are zeroed; energies updated:
//   acc[0..1] += ||B||^2 (nb), acc[2..3] += (sum s_in^2 + ||B||^2) - sum_top,
//   est[0] = sqrt(max(0, E_tot - sum s_out^2)), est[1] = sqrt(D).
struct FinDesc {
    int r_in, r, nkeep, m, nc;
    const double* s_in;
    const double* lam;
    const double* sum_top;
    const double* nb;
    double* s_out;
    double* U_out;
    long ldu;
    double* acc;
    double* est;
};
void finalize_state_batched(const FinDesc* d_descs, int count, hipStream_t s);

// y[i] += x[i]
void add_f64(const double* x, double* y, long n, hipStream_t s);
// zero the strictly upper triangle of a k x k column-major matrix
void zero_upper(double* A, int k, long lda, hipStream_t s);
// Clears of many matrices in one launch: upper == 0 zeroes A[0, n); upper == 1 zeroes
// the strictly upper triangle of the k x k column-major matrix A (leading dimension ld).
struct ClearDesc {
    double* A;
    long n;
    int k;
    int upper;
    long ld;
};
void clear_batched(const ClearDesc* d_descs, int count, hipStream_t s);
// index of the first i < n with rel[i] <= eps (n if none), written to *out (device int)
void first_feasible(const double* rel, int n, double eps, int* out, hipStream_t s);
// ||P||_F^2 per column block: out[b] = sum over the r x k_b block (column-major, ld) -- plain FP64
struct ColNormDesc {
    const double* P;
    int r, k;
    long ld;
    double* out;
};
void colblock_sumsq_batched(const ColNormDesc* d_descs, int count, hipStream_t s);

// Row-major block (rows x cols, row stride lds, FP32 or FP64) copied into dst (row
// stride ldd, FP32 or FP64); an FP32 -> FP32 or FP64 -> FP64 copy is exact.
struct PackDesc {
    const void* src;
    int rows, cols;
    long lds;
    int f32_in;  // source dtype: 0 FP64, 1 FP32, 2 BF16
    void* dst;
    long ldd;
    int f32_out;
};
void pack_batched(const PackDesc* d_descs, int count, hipStream_t s);

// Residual-certified clustering (Algorithm 2).  A cluster keeps the r largest squared
// residual singular values L (non-increasing, zero-padded) and its energy S (hi, lo).
// Certificate of a candidate with residual-Gram eigenvalues lam (nk, descending):
//   b^2 = S + nb - (sum of the r largest of L u lam);  err = sqrt(max(0, b^2)),
//   rel = err / sqrt(S + nb).  nb may be null (the cluster alone).
struct CertDesc {
    const double* L;
    const double* S;
    const double* nb;
    const double* lam;
    int nk;
    double* rel;
    double* err;
};
void resid_cert_batched(const CertDesc* d_descs, int count, int r, int nkmax, hipStream_t s);
// Lout = r largest of L u lam (non-increasing), Sout = S + nb; one block, no aliasing.
void resid_accept(const double* L, int r, const double* lam, int nk, const double* S, const double* nb, double* Lout,
                  double* Sout, hipStream_t s);
// Appends the columns of Qr (row-major m x k, ld k) whose pivot survived (Li[c,c] != 0)
// to Q (row-major, ld ldq) at columns q0, q0 + 1, ... (at most `room`); *count (device)
// receives the number appended; map holds k ints of scratch.
void append_kept_columns(const double* Qr, int m, int k, const double* Li, long ldl, double* Q, long ldq, int q0,
                         int room, int* map, int* count, hipStream_t s);
void fill_f64(double* x, long n, double v, hipStream_t s);
// x[i] uniform in [-1, 1) from a counter-based hash of (seed, i).
void fill_hash(double* x, long n, unsigned long long seed, hipStream_t s);
// Eigenvalue-free settling of candidates: with b_C^2 = S - sum L,
//   b_C^2 + ||P||^2 <= b^2 <= b_C^2 + ||B||^2;
// flag = 0 (rejected), 2 (accepted) or 1 (needs the certificate).  pn = ||Q^T B||_F^2.
struct ScreenDesc {
    const double* nb;
    const double* pn;
    int* flag;
};
void resid_screen(const ScreenDesc* d_descs, int count, const double* L, int r, const double* S, double eps,
                  hipStream_t s);

// Theorem 1 / Algorithm 1 (weyl.hip).  Energies are double-double pairs a2[2i], a2[2i+1].
void weyl_heads(const double* a2, const double* top, const int* cols, int r, int n, double* h, hipStream_t s);
void weyl_step(const int* cand, int count, int init, int acc, const double* a2, const double* h, double* state,
               double eps, int* first, double* rel, hipStream_t s);
void weyl_bound(const double* a2, const double* h, int n, double* out, hipStream_t s);
void energy_minus(const double* a2, int n, const double* top, double* out, hipStream_t s);
// A[:, c] *= (lam[c] > cut_rel * lam[0]) ? (inv ? 1 / sqrt(lam[c]) : 1) : 0  (column-major)
void scale_cols(double* A, int rows, int cols, long ld, const double* lam, int inv, double cut_rel, hipStream_t s);

// Backward of the tail energy.
void divdiff_scale(double* B, int r, int nk, int d, const double* ev, hipStream_t s);
void fill_diag(double* A, int rows, int cols, long ld, double v, double dv, hipStream_t s);
void cut_gap(const double* ev, int nk, int n, double* out, hipStream_t s);

}  // namespace cmsvd
