/*
 * Plain FP64 CPU oracle for the incremental truncated-SVD merge-error
 * estimator of "Concatenated Matrix SVD: Compression Bounds, Incremental
 * Approximation, and Error-Constrained Clustering" (Shamrai, TMLR 2026).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * file; only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP
 * library.
 *
 * What it computes (all matrices column-major FP64, host memory):
 *   - a one-sided (Hestenes) Jacobi SVD, written from the textbook algorithm;
 *   - a Householder thin QR;
 *   - one incremental step of the estimator: Lemma 1 (projection Y = Q^T A,
 *     residual R = A - Q Y, thin QR of R, block Gram of the enlarged basis)
 *     followed by the rank-r truncation of Corollary 3, carried out in the
 *     square-root (SVD) form: the core K = [[diag(sigma), Y],[0, B_qr]]
 *     satisfies K K^T = S_{t+1} of Lemma 1 when the state Gram is
 *     S_t = diag(sigma^2), so its singular values are the square roots of the
 *     eigenvalues Corollary 3 keeps or discards;
 *   - the plug-in estimate of Corollary 2 and the discarded-energy tally;
 *   - the Weyl-type bound of Theorem 1 and the residual bound of Corollary 1
 *     (test invariants).
 * Readings where the paper is silent (rank bookkeeping, Jacobi stopping rule,
 * re-orthogonalisation of the residual) are listed in the project's design
 * notes and restated at each function below.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#include <pthread.h>

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ------------------------------------------------------------------ */
/* Small dense helpers                                                 */
/* ------------------------------------------------------------------ */

static double dot(int n, const double* x, const double* y) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/* Neumaier (improved Kahan) running sum: a compensated FP64 accumulator. */
typedef struct { double s, c; } csum_t;
static void csum_add(csum_t* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double csum_val(const csum_t* a) { return a->s + a->c; }

double oracle_frob2(int m, int n, const double* A, int lda) {
    csum_t acc = {0.0, 0.0};
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) csum_add(&acc, A[IDX(i, j, lda)] * A[IDX(i, j, lda)]);
    return csum_val(&acc);
}

/* ------------------------------------------------------------------ */
/* One-sided Jacobi SVD (Hestenes).                                    */
/*                                                                    */
/* Orthogonalises the columns of the m x n matrix W (overwritten) by   */
/* plane rotations applied from the right, sweeping the column pairs   */
/* in row-cyclic order.  A pair is rotated unless                      */
/*   |w_i . w_j| <= n * eps * ||w_i|| ||w_j||                          */
/* (the Demmel-Veselic relative criterion).  On exit the singular      */
/* values are the column norms, sorted descending with a stable sort;  */
/* the left singular vectors are the normalised columns (a column with */
/* zero norm gives a zero vector).  A pair whose smaller column norm   */
/* is below n * eps * ||W||_F is left alone: such a column is rounding */
/* noise (this happens for wide inputs, whose surplus columns go to 0).*/
/* Returns the number of sweeps, or -1 when max_sweeps was reached     */
/* without convergence.                                                */
/* ------------------------------------------------------------------ */
int oracle_jacobi_svd(int m, int n, double* W, int ldw, double* sigma, double* Uleft, int ldu,
                      int max_sweeps) {
    const double tol = (double)(n > 1 ? n : 1) * DBL_EPSILON;
    int sweeps = 0, converged = (n < 2);
    double* norm2 = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double fro2 = 0.0;
    for (int j = 0; j < n; ++j) {
        norm2[j] = dot(m, &W[IDX(0, j, ldw)], &W[IDX(0, j, ldw)]);
        fro2 += norm2[j];
    }
    const double negligible2 = tol * tol * fro2;
    while (!converged && sweeps < max_sweeps) {
        int rotated = 0;
        for (int i = 0; i < n - 1; ++i) {
            for (int j = i + 1; j < n; ++j) {
                double* wi = &W[IDX(0, i, ldw)];
                double* wj = &W[IDX(0, j, ldw)];
                /* recompute the norms of the pair exactly: running updates drift */
                double alpha = dot(m, wi, wi);
                double beta = dot(m, wj, wj);
                double gamma = dot(m, wi, wj);
                if (gamma == 0.0) continue;
                if (alpha <= negligible2 || beta <= negligible2) continue;
                if (fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
                rotated = 1;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int row = 0; row < m; ++row) {
                    double a = wi[row], b = wj[row];
                    wi[row] = c * a - s * b;
                    wj[row] = s * a + c * b;
                }
            }
        }
        ++sweeps;
        if (!rotated) converged = 1;
    }
    for (int j = 0; j < n; ++j) norm2[j] = dot(m, &W[IDX(0, j, ldw)], &W[IDX(0, j, ldw)]);
    /* stable selection sort by descending norm (n is small) */
    int* order = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int j = 0; j < n; ++j) order[j] = j;
    for (int a = 0; a < n; ++a) {
        int best = a;
        for (int b = a + 1; b < n; ++b)
            if (norm2[order[b]] > norm2[order[best]]) best = b;
        if (best != a) {
            int keep = order[best];
            memmove(&order[a + 1], &order[a], sizeof(int) * (size_t)(best - a));
            order[a] = keep;
        }
    }
    for (int a = 0; a < n; ++a) {
        int j = order[a];
        double s = sqrt(norm2[j]);
        sigma[a] = s;
        if (Uleft) {
            for (int row = 0; row < m; ++row)
                Uleft[IDX(row, a, ldu)] = (s > 0.0) ? W[IDX(row, j, ldw)] / s : 0.0;
        }
    }
    free(order);
    free(norm2);
    return converged ? sweeps : -1;
}

/* ------------------------------------------------------------------ */
/* Householder thin QR: R (m x k) = Q (m x kq) * Rq (kq x k),          */
/* kq = min(m, k).  Textbook reflectors H = I - tau v v^T with v(0)=1. */
/* ------------------------------------------------------------------ */
void oracle_householder_qr(int m, int k, const double* Rin, int ldr, double* Q, int ldq,
                           double* Rq, int ldrq) {
    int kq = m < k ? m : k;
    double* A = (double*)malloc(sizeof(double) * (size_t)m * (size_t)(k > 0 ? k : 1));
    double* tau = (double*)malloc(sizeof(double) * (size_t)(kq > 0 ? kq : 1));
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < m; ++i) A[IDX(i, j, m)] = Rin[IDX(i, j, ldr)];
    for (int j = 0; j < kq; ++j) {
        double alpha = A[IDX(j, j, m)];
        double xn2 = 0.0;
        for (int i = j + 1; i < m; ++i) xn2 += A[IDX(i, j, m)] * A[IDX(i, j, m)];
        if (xn2 == 0.0) {
            tau[j] = 0.0;
            continue;
        }
        double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau[j] = (beta - alpha) / beta;
        double scale = 1.0 / (alpha - beta);
        for (int i = j + 1; i < m; ++i) A[IDX(i, j, m)] *= scale;
        A[IDX(j, j, m)] = beta;
        /* apply H_j to the trailing columns */
        for (int c = j + 1; c < k; ++c) {
            double w = A[IDX(j, c, m)];
            for (int i = j + 1; i < m; ++i) w += A[IDX(i, j, m)] * A[IDX(i, c, m)];
            w *= tau[j];
            A[IDX(j, c, m)] -= w;
            for (int i = j + 1; i < m; ++i) A[IDX(i, c, m)] -= w * A[IDX(i, j, m)];
        }
    }
    /* Rq = upper trapezoid */
    for (int c = 0; c < k; ++c)
        for (int i = 0; i < kq; ++i) Rq[IDX(i, c, ldrq)] = (i <= c) ? A[IDX(i, c, m)] : 0.0;
    /* Q = H_0 H_1 ... H_{kq-1} [I; 0], accumulated backwards */
    for (int c = 0; c < kq; ++c)
        for (int i = 0; i < m; ++i) Q[IDX(i, c, ldq)] = (i == c) ? 1.0 : 0.0;
    for (int j = kq - 1; j >= 0; --j) {
        if (tau[j] == 0.0) continue;
        for (int c = j; c < kq; ++c) {
            double w = Q[IDX(j, c, ldq)];
            for (int i = j + 1; i < m; ++i) w += A[IDX(i, j, m)] * Q[IDX(i, c, ldq)];
            w *= tau[j];
            Q[IDX(j, c, ldq)] -= w;
            for (int i = j + 1; i < m; ++i) Q[IDX(i, c, ldq)] -= w * A[IDX(i, j, m)];
        }
    }
    free(tau);
    free(A);
}

/* ------------------------------------------------------------------ */
/* One incremental step (Lemma 1 + Corollary 3, square-root form).     */
/*                                                                    */
/* State in : U (m x rho, orthonormal columns), sigma (rho).           */
/* Block    : B (m x k).                                               */
/* State out: U_out (m x rho_out), sigma_out (rho_out),                */
/*            rho_out = min(r, rho + min(k, m)).                       */
/* *disc     = sum of the squared core singular values beyond rho_out  */
/*            (the energy Corollary 3 discards at this step).          */
/* sigmaK    (optional, length rho + k): all core singular values.     */
/*                                                                    */
/* Steps, in the order of Lemma 1:                                     */
/*  1. Y = U^T B, R = B - U Y, then one more projection pass          */
/*     (Y2 = U^T R, R -= U Y2, Y += Y2) so that R is orthogonal to U   */
/*     to FP64 rounding ("twice is enough");                           */
/*  2. thin QR of R by Householder: R = Q_res B_qr;                    */
/*  3. core K = [[diag(sigma), Y],[0, B_qr]] ((rho+kq) x (rho+k));     */
/*     K K^T is Lemma 1's S_{t+1} with S_t = diag(sigma^2);            */
/*  4. one-sided Jacobi SVD of K: sigma_K (descending) and the left    */
/*     singular vectors Ul = eigenvectors of S_{t+1} (Corollary 3);    */
/*  5. keep the top rho_out pairs: U_out = [U, Q_res] Ul(:, :rho_out), */
/*     sigma_out = sigma_K(:rho_out).                                  */
/* Returns Jacobi's sweep count (or -1 if it did not converge).        */
/* ------------------------------------------------------------------ */
int oracle_update(int m, int rho, const double* U, int ldu, const double* sigma, int k,
                  const double* B, int ldb, int r, double* U_out, int ldu_out,
                  double* sigma_out, int* rho_out, double* disc, double* sigmaK) {
    int kq = m < k ? m : k;
    int nr = rho + kq, nc = rho + k;
    double* Y = (double*)calloc((size_t)(rho > 0 ? rho : 1) * (size_t)(k > 0 ? k : 1), sizeof(double));
    double* R = (double*)malloc(sizeof(double) * (size_t)m * (size_t)(k > 0 ? k : 1));
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < m; ++i) R[IDX(i, j, m)] = B[IDX(i, j, ldb)];
    for (int pass = 0; pass < 2 && rho > 0; ++pass) {
        for (int j = 0; j < k; ++j) {
            for (int a = 0; a < rho; ++a) {
                double y = dot(m, &U[IDX(0, a, ldu)], &R[IDX(0, j, m)]);
                Y[IDX(a, j, rho)] += y;
                for (int i = 0; i < m; ++i) R[IDX(i, j, m)] -= U[IDX(i, a, ldu)] * y;
            }
        }
    }
    /* note: the projections are applied one basis vector at a time within a
       pass; with the second pass the result equals the block formula
       Y = U^T B, R = B - U Y to FP64 rounding. */
    double* Qres = (double*)malloc(sizeof(double) * (size_t)m * (size_t)(kq > 0 ? kq : 1));
    double* Bqr = (double*)malloc(sizeof(double) * (size_t)(kq > 0 ? kq : 1) * (size_t)(k > 0 ? k : 1));
    oracle_householder_qr(m, k, R, m, Qres, m, Bqr, kq);
    double* K = (double*)calloc((size_t)nr * (size_t)nc, sizeof(double));
    for (int a = 0; a < rho; ++a) K[IDX(a, a, nr)] = sigma[a];
    for (int j = 0; j < k; ++j) {
        for (int a = 0; a < rho; ++a) K[IDX(a, rho + j, nr)] = Y[IDX(a, j, rho)];
        for (int b = 0; b < kq; ++b) K[IDX(rho + b, rho + j, nr)] = Bqr[IDX(b, j, kq)];
    }
    double* sK = (double*)malloc(sizeof(double) * (size_t)nc);
    double* Ul = (double*)malloc(sizeof(double) * (size_t)nr * (size_t)nc);
    int sweeps = oracle_jacobi_svd(nr, nc, K, nr, sK, Ul, nr, 60);
    int ro = nr < r ? nr : r;
    /* Lemma 1 needs an orthonormal basis: directions whose singular value is at or below
       the Jacobi routine's negligibility (n_c u ||K||_F; it never rotates such columns,
       so their normalised vectors are not orthogonal to the rest) are numerically absent
       and are dropped from the state; their energy joins the discarded tally. */
    {
        csum_t f = {0.0, 0.0};
        for (int c = 0; c < nc; ++c) csum_add(&f, sK[c] * sK[c]);
        const double thr = (double)(nc > 1 ? nc : 1) * DBL_EPSILON * sqrt(csum_val(&f));
        while (ro > 0 && !(sK[ro - 1] > thr)) --ro;
    }
    /* U_out = [U, Qres] * Ul(:, :ro) */
    for (int c = 0; c < ro; ++c) {
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int a = 0; a < rho; ++a) s += U[IDX(i, a, ldu)] * Ul[IDX(a, c, nr)];
            for (int b = 0; b < kq; ++b) s += Qres[IDX(i, b, m)] * Ul[IDX(rho + b, c, nr)];
            U_out[IDX(i, c, ldu_out)] = s;
        }
        sigma_out[c] = sK[c];
    }
    csum_t d = {0.0, 0.0};
    for (int c = ro; c < nc; ++c) csum_add(&d, sK[c] * sK[c]);
    *disc = csum_val(&d);
    *rho_out = ro;
    if (sigmaK) memcpy(sigmaK, sK, sizeof(double) * (size_t)nc);
    free(Ul);
    free(sK);
    free(K);
    free(Bqr);
    free(Qres);
    free(R);
    free(Y);
    return sweeps;
}

/* ------------------------------------------------------------------ */
/* Chain: fold oracle_update over blocks in order, from the empty      */
/* state.  Per step t it reports the plug-in estimate of Corollary 2,  */
/*   est2[t] = sum_{i<=t} ||A_i||_F^2 - sum_{j<=r} sigma_j(t)^2,       */
/* (compensated, clamped at 0) and the total discarded energy disc[t]  */
/* (the two agree to rounding: Frobenius norm of each core equals the  */
/* previous state's energy plus the new block's).                      */
/* Blocks are packed column-major, block t at offset off[t], shape     */
/* m x n[t].  U_fin (m x r) and sig_fin (r) may be NULL.               */
/* ------------------------------------------------------------------ */
int oracle_chain(int m, int nblocks, const double* data, const long* off, const int* n, int r,
                 double* est2, double* disc, double* etot, double* U_fin, double* sig_fin,
                 int* rho_fin) {
    double* U = (double*)calloc((size_t)m * (size_t)(r > 0 ? r : 1), sizeof(double));
    double* Un = (double*)calloc((size_t)m * (size_t)(r > 0 ? r : 1), sizeof(double));
    double* s = (double*)calloc((size_t)(r > 0 ? r : 1), sizeof(double));
    double* sn = (double*)calloc((size_t)(r > 0 ? r : 1), sizeof(double));
    int rho = 0, worst = 0;
    csum_t E = {0.0, 0.0}, D = {0.0, 0.0};
    for (int t = 0; t < nblocks; ++t) {
        const double* B = data + off[t];
        csum_add(&E, oracle_frob2(m, n[t], B, m));
        double dstep = 0.0;
        int rn = 0;
        int sw = oracle_update(m, rho, U, m, s, n[t], B, m, r, Un, m, sn, &rn, &dstep, NULL);
        if (sw < 0) worst = -1;
        csum_add(&D, dstep);
        double* tmp = U; U = Un; Un = tmp;
        tmp = s; s = sn; sn = tmp;
        rho = rn;
        csum_t e2 = E;
        for (int j = 0; j < rho; ++j) csum_add(&e2, -s[j] * s[j]);
        double v = csum_val(&e2);
        if (est2) est2[t] = v > 0.0 ? v : 0.0;
        if (disc) disc[t] = csum_val(&D);
        if (etot) etot[t] = csum_val(&E);
    }
    if (U_fin) {
        for (int c = 0; c < r; ++c)
            for (int i = 0; i < m; ++i) U_fin[IDX(i, c, m)] = c < rho ? U[IDX(i, c, m)] : 0.0;
    }
    if (sig_fin)
        for (int c = 0; c < r; ++c) sig_fin[c] = c < rho ? s[c] : 0.0;
    if (rho_fin) *rho_fin = rho;
    free(U);
    free(Un);
    free(s);
    free(sn);
    return worst;
}

/* ------------------------------------------------------------------ */
/* Pairwise merge errors: err[p] = plug-in estimate for the ordered    */
/* pair (anchor i, appended j) = chain over [A_i, A_j];                */
/* rel[p] = err[p] / ||[A_i, A_j]||_F.  Each distinct anchor state is  */
/* computed once and reused for every pair it heads.  Pairs are split  */
/* over nthreads POSIX threads.                                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int m, r, nblocks;
    const double* data;
    const long* off;
    const int* n;
    const int* pairs;
    int npairs;
    double* err;
    double* rel;
    /* anchor states (computed lazily, guarded) */
    double** aU;
    double** aS;
    int* arho;
    double* adisc;
    double* anorm2;
    int* astate; /* 0 = not computed, 1 = in progress, 2 = ready */
    pthread_mutex_t* lock;
    pthread_cond_t* cond;
    int next;
} pairjob_t;

static void anchor_state(pairjob_t* J, int i) {
    pthread_mutex_lock(J->lock);
    while (J->astate[i] == 1) pthread_cond_wait(J->cond, J->lock);
    if (J->astate[i] == 2) {
        pthread_mutex_unlock(J->lock);
        return;
    }
    J->astate[i] = 1;
    pthread_mutex_unlock(J->lock);
    int m = J->m, r = J->r;
    double* U = (double*)calloc((size_t)m * (size_t)r, sizeof(double));
    double* S = (double*)calloc((size_t)r, sizeof(double));
    int rho = 0;
    double d = 0.0;
    oracle_update(m, 0, NULL, m, NULL, J->n[i], J->data + J->off[i], m, r, U, m, S, &rho, &d, NULL);
    double nrm = oracle_frob2(m, J->n[i], J->data + J->off[i], m);
    pthread_mutex_lock(J->lock);
    J->aU[i] = U;
    J->aS[i] = S;
    J->arho[i] = rho;
    J->adisc[i] = d;
    J->anorm2[i] = nrm;
    J->astate[i] = 2;
    pthread_cond_broadcast(J->cond);
    pthread_mutex_unlock(J->lock);
}

static void* pair_worker(void* arg) {
    pairjob_t* J = (pairjob_t*)arg;
    int m = J->m, r = J->r;
    double* Un = (double*)calloc((size_t)m * (size_t)r, sizeof(double));
    double* Sn = (double*)calloc((size_t)r, sizeof(double));
    for (;;) {
        pthread_mutex_lock(J->lock);
        int p = J->next++;
        pthread_mutex_unlock(J->lock);
        if (p >= J->npairs) break;
        int i = J->pairs[2 * p], j = J->pairs[2 * p + 1];
        anchor_state(J, i);
        const double* B = J->data + J->off[j];
        double nb = oracle_frob2(m, J->n[j], B, m);
        int rn = 0;
        double d = 0.0;
        oracle_update(m, J->arho[i], J->aU[i], m, J->aS[i], J->n[j], B, m, r, Un, m, Sn, &rn, &d,
                      NULL);
        csum_t e2 = {0.0, 0.0};
        csum_add(&e2, J->anorm2[i]);
        csum_add(&e2, nb);
        double etot = csum_val(&e2);
        for (int c = 0; c < rn; ++c) csum_add(&e2, -Sn[c] * Sn[c]);
        double v = csum_val(&e2);
        double e = sqrt(v > 0.0 ? v : 0.0);
        J->err[p] = e;
        if (J->rel) J->rel[p] = etot > 0.0 ? e / sqrt(etot) : 0.0;
    }
    free(Un);
    free(Sn);
    return NULL;
}

int oracle_merge_errors(int m, int nblocks, const double* data, const long* off, const int* n,
                        int npairs, const int* pairs, int r, int nthreads, double* err,
                        double* rel) {
    pairjob_t J;
    memset(&J, 0, sizeof(J));
    J.m = m;
    J.r = r;
    J.nblocks = nblocks;
    J.data = data;
    J.off = off;
    J.n = n;
    J.pairs = pairs;
    J.npairs = npairs;
    J.err = err;
    J.rel = rel;
    J.aU = (double**)calloc((size_t)nblocks, sizeof(double*));
    J.aS = (double**)calloc((size_t)nblocks, sizeof(double*));
    J.arho = (int*)calloc((size_t)nblocks, sizeof(int));
    J.adisc = (double*)calloc((size_t)nblocks, sizeof(double));
    J.anorm2 = (double*)calloc((size_t)nblocks, sizeof(double));
    J.astate = (int*)calloc((size_t)nblocks, sizeof(int));
    pthread_mutex_t lock = PTHREAD_MUTEX_INITIALIZER;
    pthread_cond_t cond = PTHREAD_COND_INITIALIZER;
    J.lock = &lock;
    J.cond = &cond;
    if (nthreads < 1) nthreads = 1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, pair_worker, &J);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    for (int i = 0; i < nblocks; ++i) {
        free(J.aU[i]);
        free(J.aS[i]);
    }
    free(th);
    free(J.aU);
    free(J.aS);
    free(J.arho);
    free(J.adisc);
    free(J.anorm2);
    free(J.astate);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Theorem 1 (Weyl-type upper bound):                                  */
/*   E_r^2(M) <= sum_j ||A_j||_F^2 - max_j sum_{i<=r} sigma_i^2(A_j).  */
/* ------------------------------------------------------------------ */
double oracle_weyl_bound2(int m, int nblocks, const double* data, const long* off, const int* n,
                          int r) {
    csum_t tot = {0.0, 0.0};
    double best = 0.0;
    for (int t = 0; t < nblocks; ++t) {
        const double* A = data + off[t];
        csum_add(&tot, oracle_frob2(m, n[t], A, m));
        double* W = (double*)malloc(sizeof(double) * (size_t)m * (size_t)n[t]);
        double* s = (double*)malloc(sizeof(double) * (size_t)n[t]);
        memcpy(W, A, sizeof(double) * (size_t)m * (size_t)n[t]);
        oracle_jacobi_svd(m, n[t], W, m, s, NULL, 0, 60);
        csum_t head = {0.0, 0.0};
        for (int i = 0; i < r && i < n[t]; ++i) csum_add(&head, s[i] * s[i]);
        double h = csum_val(&head);
        if (h > best) best = h;
        free(s);
        free(W);
    }
    csum_add(&tot, -best);
    return csum_val(&tot);
}

/* ------------------------------------------------------------------ */
/* Theorem 2 / Corollary 1 (residual bound).  Residuals are taken      */
/* against a full-span orthonormal basis of the blocks seen so far:    */
/*   R_i = (I - Q_{i-1} Q_{i-1}^T) A_i.                                */
/* The basis is extended by the left singular vectors of R_i whose    */
/* singular value exceeds rank_tol * ||A_i||_F (so that numerically    */
/* absent directions are not added; rank_tol < 0: sqrt(n_i u), u=2^-52)*/
/* re-orthogonalised against the basis.  mu (length                   */
/* sum n_i, descending) receives the singular values of [R_1 ... R_K]; */
/* because the residual ranges are mutually orthogonal these are the   */
/* union of the per-block residual spectra.  Returns                   */
/*   sum_i ||A_i||_F^2 - sum_{j<=r} mu_j^2.                            */
/* ------------------------------------------------------------------ */
double oracle_residual_bound2(int m, int nblocks, const double* data, const long* off,
                              const int* n, int r, double rank_tol, double* mu) {
    int ntot = 0;
    for (int t = 0; t < nblocks; ++t) ntot += n[t];
    double* Q = (double*)calloc((size_t)m * (size_t)m, sizeof(double));
    int q = 0;
    double* allmu = (double*)calloc((size_t)(ntot > 0 ? ntot : 1), sizeof(double));
    int nmu = 0;
    csum_t tot = {0.0, 0.0};
    for (int t = 0; t < nblocks; ++t) {
        int k = n[t];
        const double* A = data + off[t];
        double a2 = oracle_frob2(m, k, A, m);
        csum_add(&tot, a2);
        double* R = (double*)malloc(sizeof(double) * (size_t)m * (size_t)k);
        memcpy(R, A, sizeof(double) * (size_t)m * (size_t)k);
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < k; ++j)
                for (int a = 0; a < q; ++a) {
                    double y = dot(m, &Q[IDX(0, a, m)], &R[IDX(0, j, m)]);
                    for (int i = 0; i < m; ++i) R[IDX(i, j, m)] -= Q[IDX(i, a, m)] * y;
                }
        /* singular values of the residual */
        double* W = (double*)malloc(sizeof(double) * (size_t)m * (size_t)k);
        double* s = (double*)malloc(sizeof(double) * (size_t)k);
        double* Ul = (double*)malloc(sizeof(double) * (size_t)m * (size_t)k);
        memcpy(W, R, sizeof(double) * (size_t)m * (size_t)k);
        oracle_jacobi_svd(m, k, W, m, s, Ul, m, 60);
        /* rank_tol < 0 selects the per-block cutoff sqrt(k_i u) ||A_i||_F, u = 2^-52 */
        double thr = (rank_tol >= 0.0 ? rank_tol : sqrt((double)k * 2.220446049250313e-16)) * sqrt(a2);
        for (int j = 0; j < k; ++j) {
            allmu[nmu++] = s[j];
            if (s[j] > thr && q < m) {
                /* extend the basis by the residual's left singular vector,
                   re-orthogonalised against the current basis */
                double* col = &Q[IDX(0, q, m)];
                for (int i = 0; i < m; ++i) col[i] = Ul[IDX(i, j, m)];
                for (int pass = 0; pass < 2; ++pass)
                    for (int a = 0; a < q; ++a) {
                        double y = dot(m, &Q[IDX(0, a, m)], col);
                        for (int i = 0; i < m; ++i) col[i] -= Q[IDX(i, a, m)] * y;
                    }
                double nn = sqrt(dot(m, col, col));
                if (nn > 0.5) {
                    for (int i = 0; i < m; ++i) col[i] /= nn;
                    ++q;
                }
            }
        }
        free(Ul);
        free(s);
        free(W);
        free(R);
    }
    /* sort descending */
    for (int a = 0; a < nmu; ++a)
        for (int b = a + 1; b < nmu; ++b)
            if (allmu[b] > allmu[a]) {
                double tmp = allmu[a];
                allmu[a] = allmu[b];
                allmu[b] = tmp;
            }
    for (int j = 0; j < r && j < nmu; ++j) csum_add(&tot, -allmu[j] * allmu[j]);
    if (mu) memcpy(mu, allmu, sizeof(double) * (size_t)nmu);
    free(allmu);
    free(Q);
    return csum_val(&tot);
}
