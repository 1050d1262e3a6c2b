// Host side of libcmsvd: handle, workspace, argument validation, and the batched
// pipelines behind the three public calls.
//
//  commit pipeline (one incremental step with the state kept; Lemma 1 + Cor. 3):
//    (a) Y = U^T B and R = B - U Y, a second projection pass on R (FP64 MFMA GEMMs)
//    (b) CholeskyQR2 of R: G1 = R^T R, L1 = chol(G1) with a pivot threshold,
//        Q1 = R L1^-T, G2 = Q1^T Q1, L2 = chol(G2), Q_res = Q1 L2^-T, B_qr = L2^T L1^T
//    (c) S+ = K K^T for K = [[diag(S), Y],[0, B_qr]]; its top-r eigenpairs
//        (tridiagonalisation, bisection, inverse iteration, back-transformation)
//    (d) U+ = [U, Q_res] Z_r,  S+ = sqrt(lambda_r)
//    (e) energies and the plug-in error (compensated FP64)
//  evaluation pipeline (candidate merges; the state is not kept):
//    (a) Y = U^T B; the residual Gram is B^T B - Y^T Y (U orthonormal), so the
//        eigenvalues of S+ equal those of [[diag(S)^2, diag(S) Y],[Y^T diag(S), B^T B]]
//        (c) tridiagonalisation + bisection of that matrix, (e) plug-in error.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "cmsvd.h"
#include "kernels.hpp"

using namespace cmsvd;

namespace {

thread_local std::string g_err;

cmsvd_status fail(cmsvd_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(CMSVD_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

constexpr double EPS = 2.220446049250313e-16;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Offsets planned on the host, carved from one device arena.
struct Plan {
    size_t off = 0;
    size_t add(size_t bytes) {
        size_t o = off;
        off += align256(bytes ? bytes : 8);
        return o;
    }
};

// Host-side staging of descriptor tables (uploaded with one copy).
struct Stage {
    std::vector<char> buf;
    size_t add(const void* p, size_t bytes) {
        size_t o = buf.size();
        buf.resize(o + align256(bytes ? bytes : 8));
        if (bytes) memcpy(buf.data() + o, p, bytes);
        return o;
    }
    template <typename T>
    size_t add(const std::vector<T>& v) {
        return add(v.data(), v.size() * sizeof(T));
    }
};

}  // namespace

struct cmsvd_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    int ncu = 256;
    char* ws = nullptr;
    size_t ws_cap = 0;
    char* dsc = nullptr;
    size_t dsc_cap = 0;
    char* pin = nullptr;
    size_t pin_cap = 0;
    hipEvent_t pin_ev = nullptr;
    bool pin_ev_armed = false;
    // stage timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> marks[4];
    std::vector<hipEvent_t> pool;
};

namespace {

cmsvd_status ensure(cmsvd_ctx* h, char*& buf, size_t& cap, size_t need) {
    if (need <= cap) return CMSVD_OK;
    HIPCHK(hipStreamSynchronize(h->stream));
    if (buf) HIPCHK(hipFree(buf));
    buf = nullptr;
    cap = 0;
    size_t want = std::max(need, cap + cap / 2);
    if (hipMalloc((void**)&buf, want) != hipSuccess) {
        (void)hipGetLastError();
        buf = nullptr;
        return fail(CMSVD_ENOMEM, "hipMalloc(%zu bytes) failed", want);
    }
    cap = want;
    return CMSVD_OK;
}

// Uploads the staged descriptor tables; returns the device base pointer.
cmsvd_status upload(cmsvd_ctx* h, const Stage& st, char** dbase) {
    const size_t n = st.buf.size();
    cmsvd_status s = ensure(h, h->dsc, h->dsc_cap, n);
    if (s != CMSVD_OK) return s;
    if (n > h->pin_cap) {
        if (h->pin_ev_armed) HIPCHK(hipEventSynchronize(h->pin_ev));
        if (h->pin) HIPCHK(hipHostFree(h->pin));
        h->pin = nullptr;
        size_t want = std::max(n, h->pin_cap * 2);
        HIPCHK(hipHostMalloc((void**)&h->pin, want, hipHostMallocDefault));
        h->pin_cap = want;
    } else if (h->pin_ev_armed) {
        HIPCHK(hipEventSynchronize(h->pin_ev));
    }
    memcpy(h->pin, st.buf.data(), n);
    HIPCHK(hipMemcpyAsync(h->dsc, h->pin, n, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipEventRecord(h->pin_ev, h->stream));
    h->pin_ev_armed = true;
    *dbase = h->dsc;
    return CMSVD_OK;
}

enum { ST_PREP = 0, ST_COMMIT = 1, ST_PROJ = 2, ST_CORE = 3, NSTAGE = 4 };

hipEvent_t take_event(cmsvd_ctx* h) {
    hipEvent_t e = nullptr;
    if (!h->pool.empty()) {
        e = h->pool.back();
        h->pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        e = nullptr;
    }
    return e;
}

// Brackets the launches issued between construction and destruction.
struct StageMark {
    cmsvd_ctx* h;
    int st;
    hipEvent_t a = nullptr;
    StageMark(cmsvd_ctx* h_, int st_) : h(h_), st(st_) {
        if (h->timing && (a = take_event(h))) (void)hipEventRecord(a, h->stream);
    }
    ~StageMark() {
        if (!a) return;
        hipEvent_t b = take_event(h);
        if (!b) return;
        (void)hipEventRecord(b, h->stream);
        h->marks[st].push_back({a, b});
    }
};

cmsvd_status check_block(const cmsvd_block& b, int64_t m, const char* what, int64_t idx) {
    if (!b.ptr) return fail(CMSVD_EINVAL, "%s %lld: null data pointer", what, (long long)idx);
    if (b.dtype != CMSVD_F32 && b.dtype != CMSVD_F64)
        return fail(CMSVD_EUNSUPPORTED, "%s %lld: dtype %d not supported (F32 or F64)", what, (long long)idx, b.dtype);
    if (b.rows != m) return fail(CMSVD_ESHAPE, "%s %lld: rows %lld != m %lld", what, (long long)idx, (long long)b.rows, (long long)m);
    if (b.cols < 1) return fail(CMSVD_ESHAPE, "%s %lld: cols %lld < 1", what, (long long)idx, (long long)b.cols);
    if (b.ld < b.cols) return fail(CMSVD_ESHAPE, "%s %lld: ld %lld < cols %lld", what, (long long)idx, (long long)b.ld, (long long)b.cols);
    if (b.cols > 16384 || m > (int64_t)1 << 30) return fail(CMSVD_EUNSUPPORTED, "%s %lld: size too large", what, (long long)idx);
    return CMSVD_OK;
}

// ---------------------------------------------------------------------------
// Batched GEMM helper: groups problems that share (transA, transB, types).
// ---------------------------------------------------------------------------
struct GemmGroup {
    std::vector<GemmDesc> d;
    bool ta = false, tb = false, af32 = false, bf32 = false;
    double alpha = 1.0, beta = 0.0;
    size_t off = 0;
    int maxM = 0, maxN = 0;
    void push(const GemmDesc& g) {
        d.push_back(g);
        maxM = std::max(maxM, g.M);
        maxN = std::max(maxN, g.N);
    }
};

void run_gemm(const GemmGroup& g, char* dbase, hipStream_t s) {
    if (g.d.empty()) return;
    gemm_f64_batched(reinterpret_cast<const GemmDesc*>(dbase + g.off), (int)g.d.size(), g.maxM, g.maxN, g.ta, g.tb,
                     g.af32, g.bf32, g.alpha, g.beta, s);
}

// ---------------------------------------------------------------------------
// Commit pipeline.
// ---------------------------------------------------------------------------
struct CommitJob {
    int m;
    const double* U;  // row-major m x r_in (ld ldu) == column-major r_in x m
    long ldu;
    const double* S;
    int r_in;
    cmsvd_block B;
    int r;
    double* U_out;  // row-major m x r (ld ldu_out)
    long ldu_out;
    double* S_out;
    double* acc;
    double* est;
};

cmsvd_status commit_batched(cmsvd_ctx* h, const std::vector<CommitJob>& jobs) {
    const int J = (int)jobs.size();
    if (J == 0) return CMSVD_OK;
    Plan pl;
    struct Off {
        size_t nb, P, P2, Rt, G1, Li1, Q1, G2, Li2, Qr, F, KT, Sp, lam, d, e, V, tau, sum, Z, vs;
        int k, nc, nkeep;
    };
    std::vector<Off> o(J);
    int nmax = 0;
    for (int j = 0; j < J; ++j) {
        const CommitJob& c = jobs[j];
        const int k = (int)c.B.cols, nc = c.r_in + k, nk = std::min(c.r, nc);
        const size_t m = (size_t)c.m;
        o[j].k = k;
        o[j].nc = nc;
        o[j].nkeep = nk;
        nmax = std::max(nmax, nc);
        o[j].nb = pl.add(2 * 8);
        o[j].P = pl.add((size_t)c.r_in * k * 8);
        o[j].P2 = pl.add((size_t)c.r_in * k * 8);
        o[j].Rt = pl.add((size_t)k * m * 8);
        o[j].G1 = pl.add((size_t)k * k * 8);
        o[j].Li1 = pl.add((size_t)k * k * 8);
        o[j].Q1 = pl.add((size_t)k * m * 8);
        o[j].G2 = pl.add((size_t)k * k * 8);
        o[j].Li2 = pl.add((size_t)k * k * 8);
        o[j].Qr = pl.add((size_t)k * m * 8);
        o[j].F = pl.add((size_t)k * k * 8);
        o[j].KT = pl.add((size_t)nc * nc * 8);
        o[j].Sp = pl.add((size_t)nc * nc * 8);
        o[j].lam = pl.add((size_t)nk * 8);
        o[j].d = pl.add((size_t)nc * 8);
        o[j].e = pl.add((size_t)nc * 8);
        o[j].V = pl.add((size_t)nc * nc * 8);
        o[j].tau = pl.add((size_t)nc * 8);
        o[j].sum = pl.add(2 * 8);
        o[j].Z = pl.add((size_t)nc * nk * 8);
        o[j].vs = pl.add((size_t)6 * nc * nk * 8);
    }
    const int nslots = std::min(J, h->ncu);
    const size_t eig_off = pl.add(sym_eig_workspace_doubles(nmax, nslots) * 8);
    cmsvd_status st = ensure(h, h->ws, h->ws_cap, pl.off);
    if (st != CMSVD_OK) return st;
    char* W = h->ws;
    auto D = [&](size_t off) { return reinterpret_cast<double*>(W + off); };

    // descriptor tables
    std::vector<NormDesc> nd(J);
    std::vector<CopyDesc> cd(J);
    GemmGroup gP, gR1, gP2, gR2, gG1, gQ1, gG2, gQr, gF, gS, gU1, gU2a, gU2b;
    gP.tb = true;                        // P = Ut * Bt^T
    gR1.ta = true; gR1.alpha = -1.0; gR1.beta = 1.0;   // Rt -= P^T Ut
    gP2.tb = true;                       // P2 = Ut * Rt^T
    gR2.ta = true; gR2.alpha = -1.0; gR2.beta = 1.0;   // Rt -= P2^T Ut
    gG1.tb = true;                       // G1 = Rt Rt^T
    gG2.tb = true;                       // G2 = Q1 Q1^T
    gS.ta = true;                        // S+ = KT^T KT
    gU1.ta = true;                       // Ut+ = Ztop^T Ut
    gU2a.ta = true; gU2a.beta = 1.0;     // Ut+ += Zbot^T Qr   (jobs with a prior state)
    gU2b.ta = true;                      // Ut+  = Zbot^T Qr   (jobs from the empty state)
    std::vector<CholDesc> ch1(J), ch2(J);
    std::vector<KtDesc> kd(J);
    std::vector<EigDesc> ed(J);
    std::vector<VecDesc> vd(J);
    std::vector<FinDesc> fd(J);
    bool anyf32 = false, anyf64 = false;
    std::vector<int> f32jobs, f64jobs;
    for (int j = 0; j < J; ++j) {
        const CommitJob& c = jobs[j];
        const Off& q = o[j];
        const int k = q.k, nc = q.nc, m = c.m;
        const bool f32 = c.B.dtype == CMSVD_F32;
        (f32 ? f32jobs : f64jobs).push_back(j);
        anyf32 |= f32;
        anyf64 |= !f32;
        nd[j] = NormDesc{c.B.ptr, m, k, (long)c.B.ld, f32 ? 1 : 0, D(q.nb)};
        cd[j] = CopyDesc{c.B.ptr, m, k, (long)c.B.ld, f32 ? 1 : 0, D(q.Rt), (long)k};
        if (c.r_in > 0) {
            gR1.push(GemmDesc{D(q.P), c.U, D(q.Rt), k, m, c.r_in, (long)c.r_in, c.ldu, (long)k});
            gP2.push(GemmDesc{c.U, D(q.Rt), D(q.P2), c.r_in, k, m, c.ldu, (long)k, (long)c.r_in});
            gR2.push(GemmDesc{D(q.P2), c.U, D(q.Rt), k, m, c.r_in, (long)c.r_in, c.ldu, (long)k});
        }
        gG1.push(GemmDesc{D(q.Rt), D(q.Rt), D(q.G1), k, k, m, (long)k, (long)k, (long)k});
        ch1[j] = CholDesc{k, D(q.G1), (long)k, D(q.Li1), (long)k, (double)k * EPS, D(q.nb), nullptr};
        gQ1.push(GemmDesc{D(q.Li1), D(q.Rt), D(q.Q1), k, m, k, (long)k, (long)k, (long)k});
        gG2.push(GemmDesc{D(q.Q1), D(q.Q1), D(q.G2), k, k, m, (long)k, (long)k, (long)k});
        ch2[j] = CholDesc{k, D(q.G2), (long)k, D(q.Li2), (long)k, (double)k * k * EPS, nullptr, nullptr};
        gQr.push(GemmDesc{D(q.Li2), D(q.Q1), D(q.Qr), k, m, k, (long)k, (long)k, (long)k});
        gF.push(GemmDesc{D(q.G1), D(q.G2), D(q.F), k, k, k, (long)k, (long)k, (long)k});
        kd[j] = KtDesc{c.r_in, k, c.S, D(q.P), (long)std::max(c.r_in, 1), D(q.F), (long)k, D(q.KT), (long)nc};
        gS.push(GemmDesc{D(q.KT), D(q.KT), D(q.Sp), nc, nc, nc, (long)nc, (long)nc, (long)nc});
        EigDesc e{};
        e.n = nc;
        e.n1 = 0;
        e.nkeep = q.nkeep;
        e.s = nullptr;
        e.P = nullptr;
        e.ldp = 1;
        e.Y = D(q.Sp);
        e.ldy = nc;
        e.lam = D(q.lam);
        e.d = D(q.d);
        e.e = D(q.e);
        e.V = D(q.V);
        e.ldv = nc;
        e.tau = D(q.tau);
        e.sum_top = D(q.sum);
        ed[j] = e;
        vd[j] = VecDesc{nc, q.nkeep, D(q.lam), D(q.d), D(q.e), D(q.V), (long)nc, D(q.tau), D(q.Z), (long)nc, D(q.vs)};
        if (c.r_in > 0) {
            gU1.push(GemmDesc{D(q.Z), c.U, c.U_out, q.nkeep, m, c.r_in, (long)nc, c.ldu, c.ldu_out});
            gU2a.push(GemmDesc{D(q.Z) + c.r_in, D(q.Qr), c.U_out, q.nkeep, m, k, (long)nc, (long)k, c.ldu_out});
        } else {
            gU2b.push(GemmDesc{D(q.Z), D(q.Qr), c.U_out, q.nkeep, m, k, (long)nc, (long)k, c.ldu_out});
        }
        fd[j] = FinDesc{c.r_in, c.r, q.nkeep, m, nc, c.S, D(q.lam), D(q.sum), D(q.nb), c.S_out, c.U_out,
                        c.ldu_out, c.acc, c.est};
    }
    // P = Ut * Bt^T needs the block dtype: one group per dtype
    GemmGroup gP32 = gP, gP64 = gP;
    gP32.bf32 = true;
    for (int j = 0; j < J; ++j) {
        const CommitJob& c = jobs[j];
        if (c.r_in == 0) continue;
        const Off& q = o[j];
        GemmDesc g{c.U, c.B.ptr, D(q.P), c.r_in, q.k, c.m, c.ldu, (long)c.B.ld, (long)c.r_in};
        (c.B.dtype == CMSVD_F32 ? gP32 : gP64).push(g);
    }
    Stage stg;
    size_t o_nd = stg.add(nd), o_cd = stg.add(cd), o_ch1 = stg.add(ch1), o_ch2 = stg.add(ch2);
    size_t o_kd = stg.add(kd), o_ed = stg.add(ed), o_vd = stg.add(vd), o_fd = stg.add(fd);
    for (GemmGroup* g : {&gP32, &gP64, &gR1, &gP2, &gR2, &gG1, &gQ1, &gG2, &gQr, &gF, &gS, &gU1, &gU2a, &gU2b})
        g->off = stg.add(g->d);
    char* db = nullptr;
    st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    StageMark mark(h, ST_COMMIT);
    hipStream_t s = h->stream;
    int maxrows = 0;
    for (const auto& c : jobs) maxrows = std::max(maxrows, c.m);
    sumsq_batched(reinterpret_cast<const NormDesc*>(db + o_nd), J, s);
    run_gemm(gP32, db, s);
    run_gemm(gP64, db, s);
    copy_f64_batched(reinterpret_cast<const CopyDesc*>(db + o_cd), J, maxrows, s);
    run_gemm(gR1, db, s);
    run_gemm(gP2, db, s);
    run_gemm(gR2, db, s);
    for (int j = 0; j < J; ++j)
        if (jobs[j].r_in > 0) add_f64(D(o[j].P2), D(o[j].P), (long)jobs[j].r_in * o[j].k, s);
    run_gemm(gG1, db, s);
    chol_semidef_batched(reinterpret_cast<const CholDesc*>(db + o_ch1), J, s);
    run_gemm(gQ1, db, s);
    run_gemm(gG2, db, s);
    chol_semidef_batched(reinterpret_cast<const CholDesc*>(db + o_ch2), J, s);
    run_gemm(gQr, db, s);
    run_gemm(gF, db, s);
    assemble_kt_batched(reinterpret_cast<const KtDesc*>(db + o_kd), J, nmax, s);
    run_gemm(gS, db, s);
    sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), J, nmax, 1, D(eig_off), nslots, s);
    sym_vectors_batched(reinterpret_cast<const VecDesc*>(db + o_vd), J, s);
    run_gemm(gU1, db, s);
    run_gemm(gU2a, db, s);
    run_gemm(gU2b, db, s);
    finalize_state_batched(reinterpret_cast<const FinDesc*>(db + o_fd), J, s);
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

// ---------------------------------------------------------------------------
// Evaluation pipeline: err/rel of candidate merges against given states.
// ---------------------------------------------------------------------------
struct EvalJob {
    const double* U;  // row-major m x r (ld ldu)
    long ldu;
    const double* S;  // r
    int r;
    const double* na;  // device double-double energy of the state side
    cmsvd_block B;     // candidate block
    const double* nb;  // device double-double ||B||^2
    const double* G;   // device B^T B, k x k (ld k)
    double* err;
    double* rel;
};

cmsvd_status eval_batched(cmsvd_ctx* h, const std::vector<EvalJob>& jobs, int m) {
    const size_t total = jobs.size();
    if (total == 0) return CMSVD_OK;
    int kmax = 0, rmax = 0;
    for (const auto& j : jobs) {
        kmax = std::max(kmax, (int)j.B.cols);
        rmax = std::max(rmax, j.r);
    }
    const int nmax = rmax + kmax;
    // chunk so that the projection buffers stay within ~8 GiB
    const size_t per = (size_t)rmax * kmax * 8;
    size_t chunk = std::max<size_t>(1, ((size_t)8 << 30) / std::max<size_t>(per, 1));
    chunk = std::min(chunk, total);
    const int nslots = (int)std::min<size_t>(chunk, (size_t)h->ncu);
    for (size_t b0 = 0; b0 < total; b0 += chunk) {
        const size_t nj = std::min(chunk, total - b0);
        Plan pl;
        std::vector<size_t> poff(nj);
        for (size_t i = 0; i < nj; ++i) poff[i] = pl.add((size_t)jobs[b0 + i].r * jobs[b0 + i].B.cols * 8);
        const size_t eig_off = pl.add(sym_eig_workspace_doubles(nmax, nslots) * 8);
        cmsvd_status st = ensure(h, h->ws, h->ws_cap, pl.off);
        if (st != CMSVD_OK) return st;
        char* W = h->ws;
        GemmGroup g32, g64;
        g32.tb = g64.tb = true;
        g32.bf32 = true;
        std::vector<EigDesc> ed(nj);
        for (size_t i = 0; i < nj; ++i) {
            const EvalJob& j = jobs[b0 + i];
            const int k = (int)j.B.cols;
            double* P = reinterpret_cast<double*>(W + poff[i]);
            GemmDesc g{j.U, j.B.ptr, P, j.r, k, m, j.ldu, (long)j.B.ld, (long)j.r};
            (j.B.dtype == CMSVD_F32 ? g32 : g64).push(g);
            EigDesc e{};
            e.n = j.r + k;
            e.n1 = j.r;
            e.nkeep = j.r;
            e.s = j.S;
            e.P = P;
            e.ldp = j.r;
            e.Y = j.G;
            e.ldy = k;
            e.na = j.na;
            e.nb = j.nb;
            e.out_err = j.err;
            e.out_rel = j.rel;
            ed[i] = e;
        }
        Stage stg;
        g32.off = stg.add(g32.d);
        g64.off = stg.add(g64.d);
        const size_t o_ed = stg.add(ed);
        char* db = nullptr;
        st = upload(h, stg, &db);
        if (st != CMSVD_OK) return st;
        {
            StageMark mark(h, ST_PROJ);
            run_gemm(g32, db, h->stream);
            run_gemm(g64, db, h->stream);
        }
        {
            StageMark mark(h, ST_CORE);
            sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), (int)nj, nmax, 0,
                            reinterpret_cast<double*>(W + eig_off), nslots, h->stream);
        }
        HIPCHK(hipGetLastError());
    }
    return CMSVD_OK;
}

// Norms (double-double) and Grams B^T B of a list of blocks into caller-provided device memory.
cmsvd_status norms_and_grams(cmsvd_ctx* h, const std::vector<cmsvd_block>& bl, const std::vector<double*>& nrm,
                             const std::vector<double*>& gram) {
    Stage stg;
    std::vector<NormDesc> nd;
    GemmGroup g32, g64;
    g32.tb = g64.tb = true;
    g32.af32 = g32.bf32 = true;
    for (size_t i = 0; i < bl.size(); ++i) {
        const cmsvd_block& b = bl[i];
        const bool f32 = b.dtype == CMSVD_F32;
        nd.push_back(NormDesc{b.ptr, (int)b.rows, (int)b.cols, (long)b.ld, f32 ? 1 : 0, nrm[i]});
        if (gram[i]) {
            GemmDesc g{b.ptr, b.ptr, gram[i], (int)b.cols, (int)b.cols, (int)b.rows, (long)b.ld, (long)b.ld, (long)b.cols};
            (f32 ? g32 : g64).push(g);
        }
    }
    const size_t o_nd = stg.add(nd);
    g32.off = stg.add(g32.d);
    g64.off = stg.add(g64.d);
    char* db = nullptr;
    cmsvd_status st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    {
        StageMark mark(h, ST_PREP);
        sumsq_batched(reinterpret_cast<const NormDesc*>(db + o_nd), (int)nd.size(), h->stream);
        run_gemm(g32, db, h->stream);
        run_gemm(g64, db, h->stream);
    }
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

// Persistent device buffers owned by one call (separate from the scratch arena,
// which the pipelines above reuse).
struct DevBuf {
    char* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

// ===========================================================================
// Public C ABI
// ===========================================================================
extern "C" {

const char* cmsvd_last_error(void) { return g_err.c_str(); }

cmsvd_status cmsvd_create(cmsvd_handle* handle, void* hip_stream) {
    if (!handle) return fail(CMSVD_EINVAL, "cmsvd_create: null handle pointer");
    cmsvd_ctx* h = new cmsvd_ctx();
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(CMSVD_EHIP, "hipGetDevice failed");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) != hipSuccess) {
        delete h;
        return fail(CMSVD_EHIP, "hipGetDeviceProperties failed");
    }
    if (std::string(prop.gcnArchName).find("gfx950") != 0) {
        delete h;
        return fail(CMSVD_EUNSUPPORTED, "device %s is not gfx950", prop.gcnArchName);
    }
    h->ncu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (hipEventCreateWithFlags(&h->pin_ev, hipEventDisableTiming) != hipSuccess) {
        delete h;
        return fail(CMSVD_EHIP, "hipEventCreate failed");
    }
    *handle = h;
    return CMSVD_OK;
}

cmsvd_status cmsvd_destroy(cmsvd_handle h) {
    if (!h) return CMSVD_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->ws) (void)hipFree(h->ws);
    if (h->dsc) (void)hipFree(h->dsc);
    if (h->pin) (void)hipHostFree(h->pin);
    if (h->pin_ev) (void)hipEventDestroy(h->pin_ev);
    for (auto& v : h->marks)
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (auto e : h->pool) (void)hipEventDestroy(e);
    delete h;
    return CMSVD_OK;
}

cmsvd_status cmsvd_profile(cmsvd_handle h, int32_t enable) {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_profile: null handle");
    h->timing = enable != 0;
    return CMSVD_OK;
}

cmsvd_status cmsvd_profile_read(cmsvd_handle h, double* ms, int64_t* count) {
    if (!h || !ms || !count) return fail(CMSVD_EINVAL, "cmsvd_profile_read: null argument");
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int st = 0; st < NSTAGE; ++st) {
        double tot = 0.0;
        for (auto& pr : h->marks[st]) {
            float t = 0.0f;
            HIPCHK(hipEventElapsedTime(&t, pr.first, pr.second));
            tot += t;
            h->pool.push_back(pr.first);
            h->pool.push_back(pr.second);
        }
        ms[st] = tot;
        count[st] = (int64_t)h->marks[st].size();
        h->marks[st].clear();
    }
    return CMSVD_OK;
}

cmsvd_status cmsvd_set_stream(cmsvd_handle h, void* hip_stream) {
    if (!h) return fail(CMSVD_EINVAL, "null handle");
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return CMSVD_OK;
}

cmsvd_status cmsvd_update(cmsvd_handle h, int64_t m, const double* U, int64_t ldu, const double* S, int64_t r_in,
                          const cmsvd_block* B, int64_t r, double* U_out, int64_t ldu_out, double* S_out, double* acc,
                          double* est) {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_update: null handle");
    if (!B) return fail(CMSVD_EINVAL, "cmsvd_update: null block");
    if (m < 1) return fail(CMSVD_ESHAPE, "cmsvd_update: m < 1");
    if (r < 1 || r > m) return fail(CMSVD_ESHAPE, "cmsvd_update: need 1 <= r <= m (r=%lld, m=%lld)", (long long)r, (long long)m);
    if (r > 4096) return fail(CMSVD_EUNSUPPORTED, "cmsvd_update: r > 4096");
    if (r_in < 0 || r_in > m) return fail(CMSVD_ESHAPE, "cmsvd_update: bad r_in");
    if (r_in > 0 && (!U || !S)) return fail(CMSVD_EINVAL, "cmsvd_update: null state");
    if (r_in > 0 && ldu < r_in) return fail(CMSVD_ESHAPE, "cmsvd_update: ldu < r_in");
    if (!U_out || !S_out || !acc) return fail(CMSVD_EINVAL, "cmsvd_update: null output");
    if (ldu_out < r) return fail(CMSVD_ESHAPE, "cmsvd_update: ldu_out < r");
    if (U_out == U || S_out == S) return fail(CMSVD_EINVAL, "cmsvd_update: outputs alias inputs");
    cmsvd_status st = check_block(*B, m, "block", 0);
    if (st != CMSVD_OK) return st;
    CommitJob j{(int)m, U, (long)ldu, S, (int)r_in, *B, (int)r, U_out, (long)ldu_out, S_out, acc, est};
    return commit_batched(h, {j});
}

cmsvd_status cmsvd_merge_errors(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, const int32_t* pairs,
                                int64_t npairs, int64_t r, double* err, double* rel) {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_merge_errors: null handle");
    if (nblocks < 1 || !blocks) return fail(CMSVD_EINVAL, "cmsvd_merge_errors: no blocks");
    if (npairs < 0 || (npairs > 0 && (!pairs || !err))) return fail(CMSVD_EINVAL, "cmsvd_merge_errors: null pairs/err");
    const int64_t m = blocks[0].rows;
    if (m < 1) return fail(CMSVD_ESHAPE, "cmsvd_merge_errors: m < 1");
    if (r < 1 || r > m) return fail(CMSVD_ESHAPE, "cmsvd_merge_errors: need 1 <= r <= m");
    if (r > 4096) return fail(CMSVD_EUNSUPPORTED, "cmsvd_merge_errors: r > 4096");
    for (int64_t i = 0; i < nblocks; ++i) {
        cmsvd_status st = check_block(blocks[i], m, "block", i);
        if (st != CMSVD_OK) return st;
    }
    for (int64_t p = 0; p < npairs; ++p) {
        const int32_t a = pairs[2 * p], b = pairs[2 * p + 1];
        if (a < 0 || a >= nblocks || b < 0 || b >= nblocks)
            return fail(CMSVD_EINVAL, "cmsvd_merge_errors: pair %lld = (%d, %d) out of range", (long long)p, a, b);
    }
    if (npairs == 0) return CMSVD_OK;
    // anchors and candidates
    std::vector<int> is_anchor(nblocks, 0), is_cand(nblocks, 0), aslot(nblocks, -1), cslot(nblocks, -1);
    for (int64_t p = 0; p < npairs; ++p) {
        is_anchor[pairs[2 * p]] = 1;
        is_cand[pairs[2 * p + 1]] = 1;
    }
    std::vector<int> anchors, cands;
    for (int i = 0; i < nblocks; ++i) {
        if (is_anchor[i]) {
            aslot[i] = (int)anchors.size();
            anchors.push_back(i);
        }
        if (is_cand[i] || is_anchor[i]) {
            cslot[i] = (int)cands.size();
            cands.push_back(i);
        }
    }
    // persistent per-call buffers: norms + grams (all involved), anchor states
    Plan pl;
    std::vector<size_t> o_n(cands.size()), o_g(cands.size());
    for (size_t c = 0; c < cands.size(); ++c) {
        const int i = cands[c];
        o_n[c] = pl.add(16);
        o_g[c] = is_cand[i] ? pl.add((size_t)blocks[i].cols * blocks[i].cols * 8) : (size_t)-1;
    }
    std::vector<size_t> o_U(anchors.size()), o_S(anchors.size()), o_acc(anchors.size());
    for (size_t a = 0; a < anchors.size(); ++a) {
        o_U[a] = pl.add((size_t)m * r * 8);
        o_S[a] = pl.add((size_t)r * 8);
        o_acc[a] = pl.add(4 * 8);
    }
    DevBuf keep;
    if (hipMalloc((void**)&keep.p, pl.off) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CMSVD_ENOMEM, "cmsvd_merge_errors: hipMalloc(%zu) failed", pl.off);
    }
    auto K = [&](size_t off) { return reinterpret_cast<double*>(keep.p + off); };
    std::vector<cmsvd_block> bl;
    std::vector<double*> nrm, gram;
    for (size_t c = 0; c < cands.size(); ++c) {
        bl.push_back(blocks[cands[c]]);
        nrm.push_back(K(o_n[c]));
        gram.push_back(o_g[c] == (size_t)-1 ? nullptr : K(o_g[c]));
    }
    cmsvd_status st = norms_and_grams(h, bl, nrm, gram);
    if (st != CMSVD_OK) return st;
    // anchor states: the update from the empty state (Algorithm 3, step 1)
    for (size_t a = 0; a < anchors.size(); ++a) HIPCHK(hipMemsetAsync(K(o_acc[a]), 0, 32, h->stream));
    {
        // chunk anchors to bound the commit scratch (~ 2 k m + 8 k^2 doubles each)
        size_t per = 0;
        for (int i : anchors) {
            const size_t k = (size_t)blocks[i].cols;
            per = std::max(per, (3 * k * (size_t)m + 9 * (k + r) * (k + r)) * 8);
        }
        size_t chunk = std::max<size_t>(1, ((size_t)8 << 30) / std::max<size_t>(per, 1));
        for (size_t a0 = 0; a0 < anchors.size(); a0 += chunk) {
            std::vector<CommitJob> jobs;
            for (size_t a = a0; a < std::min(anchors.size(), a0 + chunk); ++a) {
                const int i = anchors[a];
                jobs.push_back(CommitJob{(int)m, nullptr, (long)r, nullptr, 0, blocks[i], (int)r, K(o_U[a]), (long)r,
                                         K(o_S[a]), K(o_acc[a]), nullptr});
            }
            st = commit_batched(h, jobs);
            if (st != CMSVD_OK) return st;
        }
    }
    std::vector<EvalJob> ej;
    ej.reserve((size_t)npairs);
    for (int64_t p = 0; p < npairs; ++p) {
        const int i = pairs[2 * p], jb = pairs[2 * p + 1];
        const int a = aslot[i];
        ej.push_back(EvalJob{K(o_U[a]), (long)r, K(o_S[a]), (int)r, K(o_n[cslot[i]]), blocks[jb], K(o_n[cslot[jb]]),
                             K(o_g[cslot[jb]]), err + p, rel ? rel + p : nullptr});
    }
    st = eval_batched(h, ej, (int)m);
    if (st != CMSVD_OK) return st;
    // the per-call buffers are freed on return: wait for the work that reads them
    HIPCHK(hipStreamSynchronize(h->stream));
    return CMSVD_OK;
}

cmsvd_status cmsvd_sym_eigvals(cmsvd_handle h, const double* A, int64_t n, int64_t lda, int64_t stride_a,
                               int64_t count, int64_t nkeep, double* lam) {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_sym_eigvals: null handle");
    if (!A || !lam) return fail(CMSVD_EINVAL, "cmsvd_sym_eigvals: null pointer");
    if (n < 1 || lda < n || count < 0 || nkeep < 1 || nkeep > n) return fail(CMSVD_ESHAPE, "cmsvd_sym_eigvals: bad sizes");
    if (n > 8192) return fail(CMSVD_EUNSUPPORTED, "cmsvd_sym_eigvals: n > 8192");
    if (count == 0) return CMSVD_OK;
    const int nslots = (int)std::min<int64_t>(count, h->ncu);
    Plan pl;
    const size_t eig_off = pl.add(sym_eig_workspace_doubles((int)n, nslots) * 8);
    cmsvd_status st = ensure(h, h->ws, h->ws_cap, pl.off);
    if (st != CMSVD_OK) return st;
    std::vector<EigDesc> ed((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        EigDesc e{};
        e.n = (int)n;
        e.n1 = 0;
        e.nkeep = (int)nkeep;
        e.Y = A + i * stride_a;
        e.ldy = (long)lda;
        e.lam = lam + i * nkeep;
        ed[(size_t)i] = e;
    }
    Stage stg;
    const size_t o = stg.add(ed);
    char* db = nullptr;
    st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o), (int)count, (int)n, 1,
                    reinterpret_cast<double*>(h->ws + eig_off), nslots, h->stream);
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

cmsvd_status cmsvd_gemm_f64(cmsvd_handle h, int32_t trans_a, int32_t trans_b, int64_t M, int64_t N, int64_t K,
                            double alpha, const void* A, int64_t lda, int32_t a_dtype, const void* B, int64_t ldb,
                            int32_t b_dtype, double beta, double* C, int64_t ldc) {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_gemm_f64: null handle");
    if (!A || !B || !C) return fail(CMSVD_EINVAL, "cmsvd_gemm_f64: null pointer");
    if (M < 0 || N < 0 || K < 0 || M > INT32_MAX || N > INT32_MAX || K > INT32_MAX)
        return fail(CMSVD_ESHAPE, "cmsvd_gemm_f64: bad sizes");
    if ((a_dtype != CMSVD_F32 && a_dtype != CMSVD_F64) || (b_dtype != CMSVD_F32 && b_dtype != CMSVD_F64))
        return fail(CMSVD_EUNSUPPORTED, "cmsvd_gemm_f64: dtype must be F32 or F64");
    const int64_t ar = trans_a ? K : M, br = trans_b ? N : K;
    if (lda < std::max<int64_t>(ar, 1) || ldb < std::max<int64_t>(br, 1) || ldc < std::max<int64_t>(M, 1))
        return fail(CMSVD_ESHAPE, "cmsvd_gemm_f64: leading dimension too small");
    if (M == 0 || N == 0) return CMSVD_OK;
    GemmGroup g;
    g.ta = trans_a != 0;
    g.tb = trans_b != 0;
    g.af32 = a_dtype == CMSVD_F32;
    g.bf32 = b_dtype == CMSVD_F32;
    g.alpha = alpha;
    g.beta = beta;
    g.push(GemmDesc{A, B, C, (int)M, (int)N, (int)K, (long)lda, (long)ldb, (long)ldc});
    Stage stg;
    g.off = stg.add(g.d);
    char* db = nullptr;
    cmsvd_status st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    run_gemm(g, db, h->stream);
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

cmsvd_status cmsvd_cluster(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, int64_t r, double eps,
                           int32_t sort_mode, int32_t* labels, int64_t* nclusters, double* cluster_rel) {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_cluster: null handle");
    if (nblocks < 1 || !blocks) return fail(CMSVD_EINVAL, "cmsvd_cluster: no blocks");
    if (!labels || !nclusters) return fail(CMSVD_EINVAL, "cmsvd_cluster: null output");
    if (!(eps >= 0.0)) return fail(CMSVD_EINVAL, "cmsvd_cluster: eps must be >= 0");
    if (sort_mode != 0 && sort_mode != 1) return fail(CMSVD_EINVAL, "cmsvd_cluster: sort_mode must be 0 or 1");
    const int64_t m = blocks[0].rows;
    if (m < 1) return fail(CMSVD_ESHAPE, "cmsvd_cluster: m < 1");
    if (r < 1 || r > m) return fail(CMSVD_ESHAPE, "cmsvd_cluster: need 1 <= r <= m");
    if (r > 4096) return fail(CMSVD_EUNSUPPORTED, "cmsvd_cluster: r > 4096");
    for (int64_t i = 0; i < nblocks; ++i) {
        cmsvd_status st = check_block(blocks[i], m, "block", i);
        if (st != CMSVD_OK) return st;
    }
    const int N = (int)nblocks;
    // persistent buffers: norms, grams, two state slots, eval outputs, residual-mode scratch
    Plan pl;
    std::vector<size_t> o_n(N), o_g(N);
    size_t kmax = 0;
    for (int i = 0; i < N; ++i) {
        o_n[i] = pl.add(16);
        o_g[i] = pl.add((size_t)blocks[i].cols * blocks[i].cols * 8);
        kmax = std::max(kmax, (size_t)blocks[i].cols);
    }
    size_t o_U[2], o_S[2], o_acc[2];
    for (int s = 0; s < 2; ++s) {
        o_U[s] = pl.add((size_t)m * r * 8);
        o_S[s] = pl.add((size_t)r * 8);
        o_acc[s] = pl.add(4 * 8);
    }
    const size_t o_est = pl.add(2 * 8);
    const size_t o_err = pl.add((size_t)N * 8), o_rel = pl.add((size_t)N * 8);
    const size_t o_first = pl.add(8);
    const size_t o_pn = pl.add((size_t)N * 8);  // ||Q^T A_j||^2 (residual sort)
    const size_t o_P = pl.add((size_t)r * kmax * 8);
    DevBuf keep;
    if (hipMalloc((void**)&keep.p, pl.off) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CMSVD_ENOMEM, "cmsvd_cluster: hipMalloc(%zu) failed", pl.off);
    }
    auto K = [&](size_t off) { return reinterpret_cast<double*>(keep.p + off); };
    {
        std::vector<cmsvd_block> bl(blocks, blocks + N);
        std::vector<double*> nrm, gram;
        for (int i = 0; i < N; ++i) {
            nrm.push_back(K(o_n[i]));
            gram.push_back(K(o_g[i]));
        }
        cmsvd_status st = norms_and_grams(h, bl, nrm, gram);
        if (st != CMSVD_OK) return st;
    }
    std::vector<double> n2h(2 * (size_t)N);
    for (int i = 0; i < N; ++i) HIPCHK(hipMemcpyAsync(&n2h[2 * i], K(o_n[i]), 16, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    std::vector<double> n2(N);
    for (int i = 0; i < N; ++i) n2[i] = n2h[2 * i] + n2h[2 * i + 1];
    std::vector<int> remaining(N);
    for (int i = 0; i < N; ++i) remaining[i] = i;
    std::stable_sort(remaining.begin(), remaining.end(), [&](int a, int b) { return n2[a] > n2[b]; });
    for (int i = 0; i < N; ++i) labels[i] = -1;
    int ncl = 0;
    std::vector<double> crel;
    while (!remaining.empty()) {
        const int anchor = remaining.front();
        remaining.erase(remaining.begin());
        int cur = 0;
        HIPCHK(hipMemsetAsync(K(o_acc[cur]), 0, 32, h->stream));
        cmsvd_status st = commit_batched(
            h, {CommitJob{(int)m, nullptr, (long)r, nullptr, 0, blocks[anchor], (int)r, K(o_U[cur]), (long)r, K(o_S[cur]),
                          K(o_acc[cur]), K(o_est)}});
        if (st != CMSVD_OK) return st;
        labels[anchor] = ncl;
        for (;;) {  // passes
            std::vector<int> order = remaining;
            if (sort_mode == 0) {
                std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                    return n2[a] < n2[b] || (n2[a] == n2[b] && a < b);
                });
            } else if (!order.empty()) {
                // residual norms ||A_j||^2 - ||U^T A_j||^2 against the pass-start state
                std::vector<double> res(N, 0.0);
                for (size_t c = 0; c < order.size(); ++c) {
                    const int j = order[c];
                    GemmGroup g;
                    g.tb = true;
                    g.bf32 = blocks[j].dtype == CMSVD_F32;
                    g.push(GemmDesc{K(o_U[cur]), blocks[j].ptr, K(o_P), (int)r, (int)blocks[j].cols, (int)m, (long)r,
                                    (long)blocks[j].ld, (long)r});
                    ColNormDesc cn{K(o_P), (int)r, (int)blocks[j].cols, (long)r, K(o_pn) + j};
                    Stage stg;
                    g.off = stg.add(g.d);
                    const size_t oc = stg.add(&cn, sizeof(cn));
                    char* db = nullptr;
                    st = upload(h, stg, &db);
                    if (st != CMSVD_OK) return st;
                    run_gemm(g, db, h->stream);
                    colblock_sumsq_batched(reinterpret_cast<const ColNormDesc*>(db + oc), 1, h->stream);
                }
                std::vector<double> pn(N);
                HIPCHK(hipMemcpyAsync(pn.data(), K(o_pn), (size_t)N * 8, hipMemcpyDeviceToHost, h->stream));
                HIPCHK(hipStreamSynchronize(h->stream));
                for (int j : order) res[j] = n2[j] - pn[j];
                std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                    return res[a] < res[b] || (res[a] == res[b] && a < b);
                });
            }
            bool accepted_any = false;
            size_t pos = 0;
            while (pos < order.size()) {
                std::vector<EvalJob> ej;
                for (size_t c = pos; c < order.size(); ++c) {
                    const int j = order[c];
                    ej.push_back(EvalJob{K(o_U[cur]), (long)r, K(o_S[cur]), (int)r, K(o_acc[cur]), blocks[j], K(o_n[j]),
                                         K(o_g[j]), K(o_err) + (c - pos), K(o_rel) + (c - pos)});
                }
                st = eval_batched(h, ej, (int)m);
                if (st != CMSVD_OK) return st;
                first_feasible(K(o_rel), (int)ej.size(), eps, reinterpret_cast<int*>(K(o_first)), h->stream);
                int idx = 0;
                HIPCHK(hipMemcpyAsync(&idx, K(o_first), sizeof(int), hipMemcpyDeviceToHost, h->stream));
                HIPCHK(hipStreamSynchronize(h->stream));
                if (idx >= (int)ej.size()) break;
                const int jacc = order[pos + idx];
                const int nxt = 1 - cur;
                HIPCHK(hipMemcpyAsync(K(o_acc[nxt]), K(o_acc[cur]), 32, hipMemcpyDeviceToDevice, h->stream));
                st = commit_batched(h, {CommitJob{(int)m, K(o_U[cur]), (long)r, K(o_S[cur]), (int)r, blocks[jacc], (int)r,
                                                  K(o_U[nxt]), (long)r, K(o_S[nxt]), K(o_acc[nxt]), K(o_est)}});
                if (st != CMSVD_OK) return st;
                cur = nxt;
                labels[jacc] = ncl;
                remaining.erase(std::find(remaining.begin(), remaining.end(), jacc));
                accepted_any = true;
                pos = pos + idx + 1;
            }
            if (!accepted_any) break;
        }
        // final relative error of the cluster: est[0] / sqrt(E_tot)
        double est[2] = {0, 0}, acc[4] = {0, 0, 0, 0};
        HIPCHK(hipMemcpyAsync(est, K(o_est), 16, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(acc, K(o_acc[cur]), 32, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        const double et = acc[0] + acc[1];
        crel.push_back(et > 0.0 ? est[0] / std::sqrt(et) : 0.0);
        ++ncl;
    }
    *nclusters = ncl;
    if (cluster_rel)
        for (int c = 0; c < ncl; ++c) cluster_rel[c] = crel[c];
    return CMSVD_OK;
}

}  // extern "C"
