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
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <exception>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <thread>
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

// The status of an exception caught at the C ABI (called from a handler): host
// allocation failures are CMSVD_ENOMEM, anything else an internal error.
cmsvd_status caught(const char* who) {
    try {
        throw;
    } catch (const std::bad_alloc&) {
        return fail(CMSVD_ENOMEM, "%s: host memory allocation failed", who);
    } catch (const std::length_error&) {
        return fail(CMSVD_ENOMEM, "%s: host buffer too large", who);
    } catch (const std::exception& e) {
        return fail(CMSVD_EUNSUPPORTED, "%s: internal error: %s", who, e.what());
    } catch (...) {
        return fail(CMSVD_EUNSUPPORTED, "%s: internal error", who);
    }
}

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

// timed pipeline stages (cmsvd_profile)
enum { ST_PREP = 0, ST_COMMIT = 1, ST_PROJ = 2, ST_CORE = 3, ST_BISECT = 4, ST_TAIL = 5, NSTAGE = 6 };

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
    int proj = CMSVD_PROJ_F64;  // precision of the candidate projections
    char* gsk = nullptr;        // split-K partial products of the GEMMs
    size_t gsk_cap = 0;
    char* rec_pin = nullptr;    // pinned staging of the pair records of a dense evaluation
    size_t rec_pin_cap = 0;
    char* rec = nullptr;        // their device copy
    size_t rec_cap = 0;
    hipStream_t side = nullptr;  // uploads that overlap work on the handle's stream
    hipEvent_t rec_ev = nullptr;
    char* scratch = nullptr;     // this device's copy of the fixed no-allocation scratch
    // device memory: the caller's allocator when given (cmsvd_create_ex), else hipMalloc
    void* (*alloc_fn)(size_t, void*) = nullptr;
    void (*release_fn)(void*, void*) = nullptr;
    void* alloc_ctx = nullptr;
    char* keep = nullptr;        // per-call tables of cmsvd_merge_errors (norms, Grams, anchor states)
    size_t keep_cap = 0;
    char* pan = nullptr;         // intermediate states of panelled updates
    size_t pan_cap = 0;
    char* wide = nullptr;        // FP32 copies of the BF16 blocks of the current call
    size_t wide_cap = 0;
    bool rec_ev_armed = false;   // an upload of pair records may still read rec_pin
    hipEvent_t tail_ev = nullptr;  // end of the handle stream's enqueued work (orders the side stream)
    std::vector<int32_t> cluster_trace;  // anchors and acceptances of the last cmsvd_cluster, in order
    // captured launch sequences of repeated cmsvd_merge_errors calls (cmsvd_options.graphs)
    bool graphs = false;
    uint64_t ws_gen = 0;           // bumped whenever a device workspace is reallocated
    size_t call_upload = 0;        // descriptor bytes the current call has uploaded
    struct GraphRec {              // the descriptor tables of a call being captured
        char* dev = nullptr;       // graph-owned device copy (filled once after the capture)
        size_t cap = 0;
        std::vector<char> host;
        bool overflow = false;
    };
    GraphRec* recording = nullptr;
    hipStream_t cap_stream = nullptr;  // captures run here (the handle's stream may be the legacy one)
    struct GraphEntry {
        uint64_t key = 0;
        uint64_t gen = 0;
        hipGraphExec_t exec = nullptr;
        char* dev = nullptr;       // its descriptor tables
        uint64_t last_use = 0;
    };
    std::vector<GraphEntry> graph_cache;
    std::vector<std::pair<uint64_t, size_t>> graph_seen;  // keys run once eagerly, their upload bytes
    uint64_t graph_clock = 0;
    double last_capture_ms = 0.0;
    int64_t graph_replays = 0, graph_captures = 0;
    // autotuned schedules: scan chunk of Algorithm 3 per (m, width bucket, r, projection),
    // and the general eigen kernel's workgroup per power-of-two order bucket
    std::map<std::string, int> tuned_chunk;
    std::map<int64_t, int> tuned_threads;
    int force_threads = 0;  // set by the autotuner while it measures
    // options (cmsvd_create_ex)
    double chol_c = 0.0;         // pivot threshold factor of the first Cholesky (<= 0: the block width)
    int64_t panel_cols = 0;      // cmsvd_update(_batch): widest block appended in one step (0: any)
    // stage timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> marks[NSTAGE];
    std::vector<hipEvent_t> pool;
};

// Fixed device scratch of the no-allocation entry point: an array in the code object,
// one copy per device the library runs on, held until the process ends.  Host code
// never passes the array's name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returns for the current device, looked up once per device when a
// handle is created there.
__device__ __align__(256) char scratch[CMSVD_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<char*> g_scratch_addr;  // per device ordinal; null until looked up

cmsvd_status scratch_address(int device, char** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= device) g_scratch_addr.resize((size_t)device + 1, nullptr);
    if (!g_scratch_addr[(size_t)device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(CMSVD_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                        hipGetErrorString(e));
        }
        g_scratch_addr[(size_t)device] = static_cast<char*>(p);
    }
    *out = g_scratch_addr[(size_t)device];
    return CMSVD_OK;
}

// The descriptors of cmsvd_sym_eigvals_noalloc, written on the device (no host staging).
__global__ void eigvals_descs_kernel(EigDesc* __restrict__ out, const double* A, int n, long lda, long stride_a,
                                     long count, int nkeep, double* lam) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
        EigDesc e{};
        e.n = n;
        e.n1 = 0;
        e.nkeep = nkeep;
        e.Y = A + i * stride_a;
        e.ldy = lda;
        e.lam = lam + i * nkeep;
        out[i] = e;
    }
}

// Device memory of a handle: through the caller's allocator when one was given at
// creation, otherwise hipMalloc / hipFree.  Every device buffer of the library (the
// grow-on-demand workspaces and the per-call buffers) goes through these two.
cmsvd_status dev_alloc(cmsvd_ctx* h, size_t bytes, char** out) {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    if (h->alloc_fn) {
        void* p = h->alloc_fn(bytes, h->alloc_ctx);
        if (!p) return fail(CMSVD_ENOMEM, "allocator callback returned null for %zu bytes", bytes);
        *out = static_cast<char*>(p);
        return CMSVD_OK;
    }
    if (hipMalloc((void**)out, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return fail(CMSVD_ENOMEM, "hipMalloc(%zu bytes) failed", bytes);
    }
    return CMSVD_OK;
}

void dev_free(cmsvd_ctx* h, char* p) {
    if (!p) return;
    if (h->release_fn) h->release_fn(p, h->alloc_ctx);
    else (void)hipFree(p);
}

cmsvd_status ensure(cmsvd_ctx* h, char*& buf, size_t& cap, size_t need) {
    if (need <= cap) return CMSVD_OK;
    if (h->recording)  // a captured sequence must not move the workspaces it refers to
        return fail(CMSVD_EUNSUPPORTED, "workspace growth during graph capture");
    ++h->ws_gen;
    HIPCHK(hipStreamSynchronize(h->stream));
    const size_t want = std::max(need, cap + cap / 2);
    dev_free(h, buf);
    buf = nullptr;
    cap = 0;
    cmsvd_status st = dev_alloc(h, want, &buf);
    if (st != CMSVD_OK) return st;
    cap = want;
    return CMSVD_OK;
}

// Uploads the staged descriptor tables; returns the device base pointer.
cmsvd_status upload(cmsvd_ctx* h, const Stage& st, char** dbase) {
    const size_t n = st.buf.size();
    h->call_upload += align256(n);
    if (h->recording) {
        // capture: the tables go to the graph's own device buffer (copied once, after
        // the capture), so that replays never depend on the staging buffers
        auto& g = *h->recording;
        const size_t off = g.host.size();
        if (off + align256(n) > g.cap) {
            g.overflow = true;
            return fail(CMSVD_EUNSUPPORTED, "graph capture: descriptor tables larger than recorded");
        }
        g.host.resize(off + align256(n));
        if (n) memcpy(g.host.data() + off, st.buf.data(), n);
        *dbase = g.dev + off;
        return CMSVD_OK;
    }
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

// A device allocation owned by one call (separate from the workspace arena).
struct DevBuf {
    cmsvd_ctx* h = nullptr;
    char* p = nullptr;
    cmsvd_status get(cmsvd_ctx* h_, size_t bytes) {
        h = h_;
        return dev_alloc(h, bytes, &p);
    }
    ~DevBuf() {
        if (p) dev_free(h, p);
    }
};

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

// Every symmetric eigenproblem of the library (the update's core of order r_in + k,
// a candidate's Gram, an explicit Gram) is at most sym_eig_nmax() (2016).
cmsvd_status check_order(int64_t n, const char* who) {
    if (n > sym_eig_nmax())
        return fail(CMSVD_EUNSUPPORTED, "%s: eigenproblem of order %lld exceeds %d (append wide blocks as column panels)",
                    who, (long long)n, sym_eig_nmax());
    return CMSVD_OK;
}

cmsvd_status check_block(const cmsvd_block& b, int64_t m, const char* what, int64_t idx) {
    // shape first: a zero-width block (whose storage may be null) is a shape error
    if (b.rows != m) return fail(CMSVD_ESHAPE, "%s %lld: rows %lld != m %lld", what, (long long)idx, (long long)b.rows, (long long)m);
    if (b.cols < 1) return fail(CMSVD_ESHAPE, "%s %lld: cols %lld < 1", what, (long long)idx, (long long)b.cols);
    if (b.ld < b.cols) return fail(CMSVD_ESHAPE, "%s %lld: ld %lld < cols %lld", what, (long long)idx, (long long)b.ld, (long long)b.cols);
    if (!b.ptr) return fail(CMSVD_EINVAL, "%s %lld: null data pointer", what, (long long)idx);
    if (b.dtype != CMSVD_F32 && b.dtype != CMSVD_F64)
        return fail(CMSVD_EUNSUPPORTED, "%s %lld: dtype %d not supported (F32 or F64)", what, (long long)idx, b.dtype);
    if (b.cols > 16384 || m > (int64_t)1 << 30) return fail(CMSVD_EUNSUPPORTED, "%s %lld: size too large", what, (long long)idx);
    return CMSVD_OK;
}

// ---------------------------------------------------------------------------
// Batched GEMM helper: groups problems that share (transA, transB, types).
// ---------------------------------------------------------------------------
// Operand precision of a GEMM group: the FP64 kernel, BF16 with one or three operand
// passes, or FP32 (the last three accumulate in FP32 on the matrix cores).
enum { PREC_F64 = 0, PREC_BF16 = 1, PREC_BF16X3 = 3, PREC_F32 = 32 };

// The kernel precision of the candidate projections.
int proj_prec(const cmsvd_ctx* h) {
    switch (h->proj) {
        case CMSVD_PROJ_BF16: return PREC_BF16;
        case CMSVD_PROJ_BF16X3: return PREC_BF16X3;
        case CMSVD_PROJ_F32: return PREC_F32;
        default: return PREC_F64;
    }
}

struct GemmGroup {
    std::vector<GemmDesc> d;
    bool ta = false, tb = false, af32 = false, bf32 = false;
    int prec = PREC_F64;  // operand precision (PREC_*)
    double alpha = 1.0, beta = 0.0;
    size_t off = 0;
    int maxM = 0, maxN = 0;
    void push(const GemmDesc& g) {
        d.push_back(g);
        maxM = std::max(maxM, g.M);
        maxN = std::max(maxN, g.N);
    }
};

// A launch with few output tiles and a long contraction (the single-problem Grams and
// projections of a commit at large m) would stream its whole K range through a few
// compute units; there the K range is split over up to ncu / tiles workgroups per tile
// (at least 256 K values each) and the partials are summed in a fixed order.
void run_gemm(cmsvd_ctx* h, const GemmGroup& g, char* dbase) {
    if (g.d.empty()) return;
    const GemmDesc* dd = reinterpret_cast<const GemmDesc*>(dbase + g.off);
    if (g.prec == PREC_F32) {
        gemm_f32_batched(dd, (int)g.d.size(), g.maxM, g.maxN, g.ta, g.tb, g.af32, g.bf32, g.alpha, g.beta, h->stream);
        return;
    }
    if (g.prec != PREC_F64) {
        gemm_bf16_batched(dd, (int)g.d.size(), g.maxM, g.maxN, g.ta, g.tb, g.af32, g.bf32, g.prec, g.alpha, g.beta,
                          h->stream);
        return;
    }
    int maxK = 0;
    for (const auto& x : g.d) maxK = std::max(maxK, x.K);
    const long tiles = (long)((g.maxM + 63) / 64) * ((g.maxN + 63) / 64) * (long)g.d.size();
    int ks = 1;
    if (2 * tiles <= h->ncu && maxK >= 1024) ks = (int)std::min<long>(std::min<long>(h->ncu / tiles, maxK / 256), 64);
    double* part = nullptr;
    if (ks > 1) {
        const size_t need = g.d.size() * (size_t)ks * g.maxM * g.maxN * sizeof(double);
        if (ensure(h, h->gsk, h->gsk_cap, need) == CMSVD_OK) part = reinterpret_cast<double*>(h->gsk);
        else ks = 1;  // no memory for the partials: the unsplit launch is still correct
    }
    gemm_f64_batched(dd, (int)g.d.size(), g.maxM, g.maxN, g.ta, g.tb, g.af32, g.bf32, g.alpha, g.beta, h->stream, ks,
                     part);
}

// ---------------------------------------------------------------------------
// Semidefinite Cholesky + restricted inverse for a list of Grams.
//
// Orders below 192: one workgroup per problem (chol_semidef_batched).  Larger ones
// (where one workgroup per matrix runs the factorisation and the inverse row by row,
// with a barrier per row, and a few problems leave the chip idle): right-looking by
// 64-column panels -- the panel's diagonal
// block is factored by the same kernel (pivot threshold, zeroed columns, inverse on
// the kept pivots), the panel below becomes A21 Dinv^T and the trailing matrix is
// updated by A22 -= L21 L21^T, both on the matrix cores; the inverse is then merged
// bottom-up from the diagonal blocks, inv([[A, 0], [B, C]]) = [[A', 0], [-C' B A', C']]
// (A', C' the inverses on the kept pivots).  Both orders compute the same factor and
// the same dropped pivots up to rounding.
// ---------------------------------------------------------------------------
struct CholPlan {
    static constexpr int NB = 64;
    std::vector<CholDesc> jobs;
    bool blocked = false;
    size_t o_desc = 0;
    struct Panel {
        std::vector<CholDesc> diag;
        std::vector<CopyDesc> cp;
        GemmGroup pan, trail;
        size_t o_diag = 0, o_cp = 0;
        int cprows = 0;
    };
    std::vector<Panel> panels;
    struct Level {
        GemmGroup t, x;
    };
    std::vector<Level> levels;
    // clears of the blocked path, one launch each: the inverses before the panels, the
    // factors' strict upper triangles at the end
    std::vector<ClearDesc> pre, post;
    size_t o_pre = 0, o_post = 0;

    static bool use_blocked(const std::vector<int>& ks) {
        int kmax = 0;
        for (int k : ks) kmax = std::max(kmax, k);
        return kmax >= 192;
    }
    // scratch doubles per problem of order k (blocked path): the panel copy (k x NB)
    // and the products of the inverse merge (k x k)
    static size_t scratch_doubles(int k) { return (size_t)k * NB + (size_t)k * k; }

    // `scratch[j]` points at scratch_doubles(k_j) doubles (blocked path only).
    void build(const std::vector<CholDesc>& js, const std::vector<double*>& scratch) {
        jobs = js;
        std::vector<int> ks;
        for (const auto& c : js) ks.push_back(c.k);
        blocked = use_blocked(ks);
        if (!blocked) return;
        int kmax = 0;
        for (int k : ks) kmax = std::max(kmax, k);
        for (int p = 0; p < kmax; p += NB) {
            Panel P;
            P.pan.tb = true;
            P.trail.tb = true;
            P.trail.alpha = -1.0;
            P.trail.beta = 1.0;
            for (size_t j = 0; j < js.size(); ++j) {
                const CholDesc& c = js[j];
                if (p >= c.k) continue;
                const int w = std::min(NB, c.k - p), hgt = c.k - p - w;
                double* Gpp = c.G + p + (long)p * c.ldg;
                double* Ipp = c.Linv + p + (long)p * c.ldi;
                P.diag.push_back(CholDesc{w, Gpp, c.ldg, Ipp, c.ldi, c.thresh_scale, c.thresh_ref, nullptr});
                if (hgt > 0) {
                    double* A21 = c.G + (p + w) + (long)p * c.ldg;
                    double* T = scratch[j];
                    // column-major hgt x w panel == row-major w x hgt rows of stride ldg
                    P.cp.push_back(CopyDesc{A21, w, hgt, c.ldg, 0, T, (long)hgt});
                    P.cprows = std::max(P.cprows, w);
                    P.pan.push(GemmDesc{T, Ipp, A21, hgt, w, w, (long)hgt, c.ldi, c.ldg});
                    P.trail.push(GemmDesc{A21, A21, c.G + (p + w) + (long)(p + w) * c.ldg, hgt, hgt, w, c.ldg, c.ldg,
                                          c.ldg});
                }
            }
            panels.push_back(std::move(P));
        }
        for (int s = NB; s < kmax; s *= 2) {
            Level L;
            L.x.alpha = -1.0;
            for (size_t j = 0; j < js.size(); ++j) {
                const CholDesc& c = js[j];
                double* T = scratch[j] + (size_t)c.k * NB;
                size_t toff = 0;
                for (int i = 0; i + s < c.k; i += 2 * s) {
                    const int nc = std::min(s, c.k - i - s);
                    const double* B = c.G + (i + s) + (long)i * c.ldg;         // L[C, A]
                    const double* XA = c.Linv + i + (long)i * c.ldi;            // A'
                    const double* XC = c.Linv + (i + s) + (long)(i + s) * c.ldi;  // C'
                    double* Ti = T + toff;
                    toff += (size_t)nc * s;
                    L.t.push(GemmDesc{B, XA, Ti, nc, s, s, c.ldg, c.ldi, (long)nc});
                    L.x.push(GemmDesc{XC, Ti, c.Linv + (i + s) + (long)i * c.ldi, nc, s, nc, c.ldi, (long)nc, c.ldi});
                }
            }
            levels.push_back(std::move(L));
        }
        for (const auto& c : js) {
            pre.push_back(ClearDesc{c.Linv, (long)c.ldi * c.k, c.k, 0, c.ldi});
            post.push_back(ClearDesc{c.G, 0, c.k, 1, c.ldg});  // L is lower triangular
        }
    }

    void stage(Stage& stg) {
        if (!blocked) {
            o_desc = stg.add(jobs);
            return;
        }
        for (auto& P : panels) {
            P.o_diag = stg.add(P.diag);
            P.o_cp = stg.add(P.cp);
            P.pan.off = stg.add(P.pan.d);
            P.trail.off = stg.add(P.trail.d);
        }
        for (auto& L : levels) {
            L.t.off = stg.add(L.t.d);
            L.x.off = stg.add(L.x.d);
        }
        o_pre = stg.add(pre);
        o_post = stg.add(post);
    }

    void run(cmsvd_ctx* h, char* db) {
        hipStream_t s = h->stream;
        if (!blocked) {
            chol_semidef_batched(reinterpret_cast<const CholDesc*>(db + o_desc), (int)jobs.size(), s);
            return;
        }
        clear_batched(reinterpret_cast<const ClearDesc*>(db + o_pre), (int)pre.size(), s);
        for (auto& P : panels) {
            chol_semidef_batched(reinterpret_cast<const CholDesc*>(db + P.o_diag), (int)P.diag.size(), s);
            if (!P.cp.empty()) {
                copy_f64_batched(reinterpret_cast<const CopyDesc*>(db + P.o_cp), (int)P.cp.size(), P.cprows, s);
                run_gemm(h, P.pan, db);
                run_gemm(h, P.trail, db);
            }
        }
        for (auto& L : levels) {
            run_gemm(h, L.t, db);
            run_gemm(h, L.x, db);
        }
        clear_batched(reinterpret_cast<const ClearDesc*>(db + o_post), (int)post.size(), s);
    }
};

// ---------------------------------------------------------------------------
// Eigenvectors of a few large cores: the per-workgroup kernel leaves the eigenvectors
// of the tridiagonal in Z, and the reflectors are applied in blocks of 32 in compact
// WY form, Z <- (I - V T V^T) Z from the last block to the first, as MFMA GEMMs
// batched across problems (one per block and stage).  Many small problems keep the
// one-workgroup back-transformation.
// ---------------------------------------------------------------------------
struct BackPlan {
    static constexpr int BB = 32;
    std::vector<VecDesc> jobs;
    bool blocked = false;
    size_t o_vd = 0, o_lf = 0;
    std::vector<LarftDesc> lf;
    GemmGroup gS;
    struct Step {
        GemmGroup g1, g2, g3;
    };
    std::vector<Step> steps;

    static bool use_blocked(const std::vector<int>& ns) {
        int nmax = 0;
        for (int n : ns) nmax = std::max(nmax, n);
        return nmax >= 256 && ns.size() <= 32;
    }
    static int nblocks(int n) { return n > 2 ? (n - 2 + BB - 1) / BB : 0; }
    // scratch doubles per problem: the Grams and T of its blocks, W1 and W2
    static size_t scratch_doubles(int n, int nk) { return (size_t)nblocks(n) * BB * BB * 2 + (size_t)BB * nk * 2; }

    void build(const std::vector<VecDesc>& js, const std::vector<double*>& scratch) {
        jobs = js;
        std::vector<int> ns;
        for (const auto& v : js) ns.push_back(v.n);
        blocked = use_blocked(ns);
        if (!blocked) return;
        int bmax = 0;
        for (auto& v : jobs) {
            v.skip_bt = 1;
            bmax = std::max(bmax, nblocks(v.n));
        }
        gS.ta = true;
        for (size_t p = 0; p < jobs.size(); ++p) {
            const VecDesc& v = jobs[p];
            const int nb = nblocks(v.n);
            double* S = scratch[p];
            double* T = S + (size_t)nb * BB * BB;
            for (int b = 0; b < nb; ++b) {
                const int j0 = b * BB, be = std::min(BB, v.n - 2 - j0), r0 = j0 + 1, h = v.n - r0;
                const double* Vb = v.V + r0 + (long)j0 * v.ldv;
                gS.push(GemmDesc{Vb, Vb, S + (size_t)b * BB * BB, be, be, h, v.ldv, v.ldv, (long)BB});
                lf.push_back(LarftDesc{S + (size_t)b * BB * BB, v.tau + j0, T + (size_t)b * BB * BB, be, (long)BB});
            }
        }
        for (int b = bmax - 1; b >= 0; --b) {
            Step st;
            st.g1.ta = true;
            st.g3.alpha = -1.0;
            st.g3.beta = 1.0;
            for (size_t p = 0; p < jobs.size(); ++p) {
                const VecDesc& v = jobs[p];
                const int nb = nblocks(v.n);
                if (b >= nb) continue;
                double* S = scratch[p];
                double* T = S + (size_t)nb * BB * BB;
                double* W1 = T + (size_t)nb * BB * BB;
                double* W2 = W1 + (size_t)BB * v.nkeep;
                const int j0 = b * BB, be = std::min(BB, v.n - 2 - j0), r0 = j0 + 1, h = v.n - r0;
                const double* Vb = v.V + r0 + (long)j0 * v.ldv;
                st.g1.push(GemmDesc{Vb, v.Z + r0, W1, be, v.nkeep, h, v.ldv, v.ldz, (long)BB});
                st.g2.push(GemmDesc{T + (size_t)b * BB * BB, W1, W2, be, v.nkeep, be, (long)BB, (long)BB, (long)BB});
                st.g3.push(GemmDesc{Vb, W2, v.Z + r0, h, v.nkeep, be, v.ldv, (long)BB, v.ldz});
            }
            steps.push_back(std::move(st));
        }
    }

    void stage(Stage& stg) {
        o_vd = stg.add(jobs);
        if (!blocked) return;
        o_lf = stg.add(lf);
        gS.off = stg.add(gS.d);
        for (auto& st : steps) {
            st.g1.off = stg.add(st.g1.d);
            st.g2.off = stg.add(st.g2.d);
            st.g3.off = stg.add(st.g3.d);
        }
    }

    void run(cmsvd_ctx* h, char* db) {
        hipStream_t s = h->stream;
        sym_vectors_batched(reinterpret_cast<const VecDesc*>(db + o_vd), (int)jobs.size(), s);
        if (!blocked) return;
        for (const auto& v : jobs) materialize_reflectors(const_cast<double*>(v.V), v.n, v.ldv, s);
        run_gemm(h, gS, db);
        larft_batched(reinterpret_cast<const LarftDesc*>(db + o_lf), (int)lf.size(), s);
        for (auto& st : steps) {
            run_gemm(h, st.g1, db);
            run_gemm(h, st.g2, db);
            run_gemm(h, st.g3, db);
        }
    }
};

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
    // Decomposition only (the backward of the tail energy): when Z_out is set, all
    // nc = r_in + k eigenpairs of the core are computed and returned -- Z_out (nc x nc
    // column-major, eigenvectors by descending eigenvalue), lam_out (nc) and Qr_out (the
    // residual basis transposed, k x m column-major) -- and U_out, S_out, acc and est
    // are left untouched.
    double* Z_out = nullptr;
    double* lam_out = nullptr;
    double* Qr_out = nullptr;
    // Optional: the block energy ||B||_F^2 (double-double, device) when the caller has
    // it already; otherwise the pipeline computes it.
    const double* nb_in = nullptr;
    // Optional, for r_in == 0: the block's Gram B^T B (k x k FP64, ld k, device) when the
    // caller has it already; it is copied in place of the first CholeskyQR Gram.
    const double* G_in = nullptr;
};

int eig_threads(const cmsvd_ctx* h, int64_t n);

cmsvd_status commit_batched(cmsvd_ctx* h, const std::vector<CommitJob>& jobs) {
    const int J = (int)jobs.size();
    if (J == 0) return CMSVD_OK;
    Plan pl;
    struct Off {
        size_t nb, P, P2, Rt, G1, Li1, Q1, G2, Li2, Qr, F, KT, Sp, lam, d, e, V, tau, sum, Z, vs, cs, bs;
        int k, nc, nkeep, nu;
        bool full;
    };
    std::vector<Off> o(J);
    int nmax = 0;
    std::vector<int> ks;
    for (const auto& c : jobs) ks.push_back((int)c.B.cols);
    const bool chol_blocked = CholPlan::use_blocked(ks);
    std::vector<int> ncs;
    for (const auto& c : jobs) ncs.push_back(c.r_in + (int)c.B.cols);
    const bool back_blocked = BackPlan::use_blocked(ncs);
    for (int j = 0; j < J; ++j) {
        const CommitJob& c = jobs[j];
        const bool full = c.Z_out != nullptr;
        const int k = (int)c.B.cols, nc = c.r_in + k, nk = full ? nc : std::min(c.r, nc);
        const size_t m = (size_t)c.m;
        o[j].k = k;
        o[j].nc = nc;
        o[j].nkeep = nk;
        o[j].nu = std::min(c.r, nc);
        o[j].full = full;
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
        o[j].cs = chol_blocked ? pl.add(CholPlan::scratch_doubles(k) * 8) : 0;
        o[j].bs = back_blocked ? pl.add(BackPlan::scratch_doubles(nc, nk) * 8) : 0;
    }
    const int nslots = std::min(J, h->ncu);
    const size_t eig_off = pl.add(sym_eig_workspace_doubles(nmax, nslots) * 8);
    cmsvd_status st = ensure(h, h->ws, h->ws_cap, pl.off);
    if (st != CMSVD_OK) return st;
    char* W = h->ws;
    auto D = [&](size_t off) { return reinterpret_cast<double*>(W + off); };
    // caller-owned storage for the decomposition outputs
    std::vector<double*> pQr(J), pLam(J), pZ(J);
    for (int j = 0; j < J; ++j) {
        pQr[j] = jobs[j].Qr_out ? jobs[j].Qr_out : D(o[j].Qr);
        pLam[j] = jobs[j].lam_out ? jobs[j].lam_out : D(o[j].lam);
        pZ[j] = jobs[j].Z_out ? jobs[j].Z_out : D(o[j].Z);
    }

    // descriptor tables
    std::vector<NormDesc> nd;
    std::vector<const double*> pnb(J);
    std::vector<CopyDesc> cd(J), gcd;  // block -> Rt copies; given Grams -> G1
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
        if (c.nb_in) {
            pnb[j] = c.nb_in;
        } else {
            pnb[j] = D(q.nb);
            nd.push_back(NormDesc{c.B.ptr, m, k, (long)c.B.ld, f32 ? 1 : 0, D(q.nb)});
        }
        cd[j] = CopyDesc{c.B.ptr, m, k, (long)c.B.ld, f32 ? 1 : 0, D(q.Rt), (long)k};
        if (c.r_in > 0) {
            gR1.push(GemmDesc{D(q.P), c.U, D(q.Rt), k, m, c.r_in, (long)c.r_in, c.ldu, (long)k});
            gP2.push(GemmDesc{c.U, D(q.Rt), D(q.P2), c.r_in, k, m, c.ldu, (long)k, (long)c.r_in});
            gR2.push(GemmDesc{D(q.P2), c.U, D(q.Rt), k, m, c.r_in, (long)c.r_in, c.ldu, (long)k});
        }
        if (c.r_in == 0 && c.G_in) gcd.push_back(CopyDesc{c.G_in, k, k, (long)k, 0, D(q.G1), (long)k});
        else gG1.push(GemmDesc{D(q.Rt), D(q.Rt), D(q.G1), k, k, m, (long)k, (long)k, (long)k});
        ch1[j] = CholDesc{k, D(q.G1), (long)k, D(q.Li1), (long)k, (h->chol_c > 0.0 ? h->chol_c : (double)k) * EPS,
                          pnb[j], nullptr};
        gQ1.push(GemmDesc{D(q.Li1), D(q.Rt), D(q.Q1), k, m, k, (long)k, (long)k, (long)k});
        gG2.push(GemmDesc{D(q.Q1), D(q.Q1), D(q.G2), k, k, m, (long)k, (long)k, (long)k});
        ch2[j] = CholDesc{k, D(q.G2), (long)k, D(q.Li2), (long)k, (double)k * k * EPS, nullptr, nullptr};
        gQr.push(GemmDesc{D(q.Li2), D(q.Q1), pQr[j], k, m, k, (long)k, (long)k, (long)k});
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
        e.lam = pLam[j];
        e.d = D(q.d);
        e.e = D(q.e);
        e.V = D(q.V);
        e.ldv = nc;
        e.tau = D(q.tau);
        e.sum_top = D(q.sum);
        ed[j] = e;
        vd[j] = VecDesc{nc, q.nkeep, pLam[j], D(q.d), D(q.e), D(q.V), (long)nc, D(q.tau), pZ[j], (long)nc, D(q.vs)};
        if (!q.full) {
            if (c.r_in > 0) {
                gU1.push(GemmDesc{pZ[j], c.U, c.U_out, q.nu, m, c.r_in, (long)nc, c.ldu, c.ldu_out});
                gU2a.push(GemmDesc{pZ[j] + c.r_in, pQr[j], c.U_out, q.nu, m, k, (long)nc, (long)k, c.ldu_out});
            } else {
                gU2b.push(GemmDesc{pZ[j], pQr[j], c.U_out, q.nu, m, k, (long)nc, (long)k, c.ldu_out});
            }
        }
        fd[j] = FinDesc{c.r_in, c.r, q.nkeep, m, nc, c.S, pLam[j], D(q.sum), pnb[j], c.S_out, c.U_out,
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
    CholPlan cp1, cp2;
    {
        std::vector<double*> scr(J);
        for (int j = 0; j < J; ++j) scr[j] = D(o[j].cs);
        cp1.build(ch1, scr);
        cp2.build(ch2, scr);  // runs after cp1 is done with the scratch
    }
    Stage stg;
    size_t o_nd = stg.add(nd), o_cd = stg.add(cd), o_gcd = stg.add(gcd);
    cp1.stage(stg);
    cp2.stage(stg);
    std::vector<FinDesc> fdk;
    for (int j = 0; j < J; ++j)
        if (!o[j].full) fdk.push_back(fd[j]);
    BackPlan bp;
    {
        std::vector<double*> scr(J);
        for (int j = 0; j < J; ++j) scr[j] = D(o[j].bs);
        bp.build(vd, scr);
    }
    size_t o_kd = stg.add(kd), o_ed = stg.add(ed), o_fd = stg.add(fdk);
    bp.stage(stg);
    for (GemmGroup* g : {&gP32, &gP64, &gR1, &gP2, &gR2, &gG1, &gQ1, &gG2, &gQr, &gF, &gS, &gU1, &gU2a, &gU2b})
        g->off = stg.add(g->d);
    char* db = nullptr;
    st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    StageMark mark(h, ST_COMMIT);
    hipStream_t s = h->stream;
    int maxrows = 0;
    for (const auto& c : jobs) maxrows = std::max(maxrows, c.m);
    sumsq_batched(reinterpret_cast<const NormDesc*>(db + o_nd), (int)nd.size(), s);
    run_gemm(h, gP32, db);
    run_gemm(h, gP64, db);
    copy_f64_batched(reinterpret_cast<const CopyDesc*>(db + o_cd), J, maxrows, s);
    run_gemm(h, gR1, db);
    run_gemm(h, gP2, db);
    run_gemm(h, gR2, db);
    for (int j = 0; j < J; ++j)
        if (jobs[j].r_in > 0) add_f64(D(o[j].P2), D(o[j].P), (long)jobs[j].r_in * o[j].k, s);
    if (!gcd.empty()) copy_f64_batched(reinterpret_cast<const CopyDesc*>(db + o_gcd), (int)gcd.size(), maxrows, s);
    run_gemm(h, gG1, db);
    cp1.run(h, db);
    run_gemm(h, gQ1, db);
    run_gemm(h, gG2, db);
    cp2.run(h, db);
    run_gemm(h, gQr, db);
    run_gemm(h, gF, db);
    assemble_kt_batched(reinterpret_cast<const KtDesc*>(db + o_kd), J, nmax, s);
    run_gemm(h, gS, db);
    // the workgroup size the autotuner measured for this order bucket (evaluations of
    // the same orders), else the default
    sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), J, nmax, 1, D(eig_off), nslots, s, eig_threads(h, nmax));
    bp.run(h, db);
    run_gemm(h, gU1, db);
    run_gemm(h, gU2a, db);
    run_gemm(h, gU2b, db);
    if (!fdk.empty()) finalize_state_batched(reinterpret_cast<const FinDesc*>(db + o_fd), (int)fdk.size(), s);
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

// ---------------------------------------------------------------------------
// Evaluation pipeline: err/rel of candidate merges against given states.
// ---------------------------------------------------------------------------
// Width bucket of the autotuner: the next power of two at or above k (at least 16).
int64_t width_bucket(int64_t k) {
    int64_t b = 16;
    while (b < k) b *= 2;
    return b;
}

// Workgroup size of the general eigen kernel for candidate cores of order n: what the
// autotuner measured for n's power-of-two bucket, else the default (0).
int eig_threads(const cmsvd_ctx* h, int64_t n) {
    if (h->force_threads) return h->force_threads;
    auto it = h->tuned_threads.find(width_bucket(n));
    return it == h->tuned_threads.end() ? 0 : it->second;
}

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
    // Register-resident cores above the tail order hand their trailing matrix over to the
    // four-wave kernel (two problems per CU) after n - tail column steps.
    int lvo[8];
    const int nlv = sym_eig_tail_levels(lvo);
    const int tail = lvo[0];
    const bool hand = sym_eig_split(nmax) && !(kmax == 1 && rmax <= 256);
    // chunk so that the projection buffers and trailing matrices stay within ~16 GiB (each
    // level overwrites the trailing matrix it read with the one it hands over)
    const size_t per = (size_t)rmax * kmax * 8 + (hand ? (size_t)tail * tail * 8 : 0);
    size_t chunk = std::max<size_t>(1, ((size_t)16 << 30) / std::max<size_t>(per, 1));
    chunk = std::min(chunk, total);
    const int nslots = (int)std::min<size_t>(chunk, (size_t)h->ncu);
    for (size_t b0 = 0; b0 < total; b0 += chunk) {
        const size_t nj = std::min(chunk, total - b0);
        Plan pl;
        std::vector<size_t> poff(nj);
        for (size_t i = 0; i < nj; ++i) poff[i] = pl.add((size_t)jobs[b0 + i].r * jobs[b0 + i].B.cols * 8);
        const size_t eig_off = pl.add(sym_eig_workspace_doubles(nmax, nslots) * 8);
        const size_t tri = sym_eig_tri_doubles(nmax);
        const size_t tri_off = pl.add(nj * tri * 8);  // tridiagonals of the split evaluation
        size_t nhand = 0;
        if (hand)
            for (size_t i = 0; i < nj; ++i) nhand += jobs[b0 + i].r + jobs[b0 + i].B.cols > tail ? 1 : 0;
        const size_t at_off = pl.add(nhand * (size_t)tail * tail * 8);  // trailing matrices
        cmsvd_status st = ensure(h, h->ws, h->ws_cap, pl.off);
        if (st != CMSVD_OK) return st;
        char* W = h->ws;
        GemmGroup g32, g64;
        g32.tb = g64.tb = true;
        g32.bf32 = true;
        g32.prec = g64.prec = proj_prec(h);
        std::vector<EigDesc> ed(nj);
        size_t ihand = 0;
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
            e.d = reinterpret_cast<double*>(W + tri_off) + i * tri;
            e.e = e.d + tri / 2;
            if (hand && e.n > tail) {
                e.jsplit = e.n - tail;
                e.At = reinterpret_cast<double*>(W + at_off) + (size_t)ihand++ * tail * tail;
                e.ldt = tail;
            }
            ed[i] = e;
        }
        // The eigen kernels take problems in a grid-stride order, so problems next to each
        // other in the table run at the same time on different CUs.  Grouping them by
        // candidate lets the CUs of one XCD share the candidate's Gram in its L2 instead
        // of fetching it once per problem (results do not depend on the order).
        {
            std::unordered_map<const double*, int> gid;
            std::vector<int> grp(nj), cnt;
            for (size_t i = 0; i < nj; ++i) {
                auto it = gid.emplace(ed[i].Y, (int)cnt.size()).first;
                if (it->second == (int)cnt.size()) cnt.push_back(0);
                grp[i] = it->second;
                ++cnt[(size_t)it->second];
            }
            if (cnt.size() > 1 && cnt.size() < nj) {
                std::vector<size_t> at(cnt.size(), 0);
                for (size_t g = 1; g < cnt.size(); ++g) at[g] = at[g - 1] + (size_t)cnt[g - 1];
                std::vector<EigDesc> grouped(nj);
                for (size_t i = 0; i < nj; ++i) grouped[at[(size_t)grp[i]]++] = ed[i];
                ed.swap(grouped);
            }
        }
        // the trailing problems of every hand-over level, in the (grouped) order of their
        // full problems; a level reads its matrix into tiles before it writes the next
        // level's into the same slot
        std::vector<std::vector<EigDesc>> lv((size_t)nlv);
        for (const EigDesc& e : ed) {
            if (e.jsplit <= 0) continue;
            EigDesc cur = e;
            for (int l = 0; l < nlv; ++l) {
                EigDesc t2{};
                t2.n = cur.n - cur.jsplit;
                t2.nkeep = e.nkeep;
                t2.Y = cur.At;
                t2.ldy = cur.ldt;
                t2.d = cur.d + cur.jsplit;
                t2.e = cur.e + cur.jsplit;
                if (l + 1 < nlv && t2.n > lvo[l + 1]) {
                    t2.jsplit = t2.n - lvo[l + 1];
                    t2.At = cur.At;
                    t2.ldt = lvo[l + 1];
                }
                lv[(size_t)l].push_back(t2);
                if (t2.jsplit <= 0) break;
                cur = t2;
            }
        }
        Stage stg;
        g32.off = stg.add(g32.d);
        g64.off = stg.add(g64.d);
        const size_t o_ed = stg.add(ed);
        std::vector<size_t> o_lv((size_t)nlv);
        for (int l = 0; l < nlv; ++l) o_lv[(size_t)l] = stg.add(lv[(size_t)l]);
        char* db = nullptr;
        st = upload(h, stg, &db);
        if (st != CMSVD_OK) return st;
        {
            StageMark mark(h, ST_PROJ);
            run_gemm(h, g32, db);
            run_gemm(h, g64, db);
        }
        {
            StageMark mark(h, ST_CORE);
            if (kmax == 1 && rmax <= 256)  // one-column candidates: arrowhead cores
                arrow_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), (int)nj, rmax, h->stream);
            else
                sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), (int)nj, nmax, 2,
                                reinterpret_cast<double*>(W + eig_off), nslots, h->stream, eig_threads(h, nmax));
        }
        if (!lv[0].empty()) {
            StageMark mark(h, ST_TAIL);
            for (int l = 0; l < nlv; ++l)
                sym_eig_tail_batched(reinterpret_cast<const EigDesc*>(db + o_lv[(size_t)l]), (int)lv[(size_t)l].size(), l,
                                     h->stream);
        }
        if (!(kmax == 1 && rmax <= 256) && sym_eig_split(nmax)) {
            StageMark mark(h, ST_BISECT);
            tri_bisect_batched(reinterpret_cast<const EigDesc*>(db + o_ed), (int)nj, nmax, h->stream);
        }
        HIPCHK(hipGetLastError());
    }
    return CMSVD_OK;
}

// Dense evaluation for thin blocks: when r or the candidate widths are below the
// 64-wide MFMA tile, per-pair GEMMs waste most of every tile and re-read each basis and
// block once per pair.  Then the projections of a chunk of anchors against all
// candidates are one GEMM, [U_a0 .. U_a1]^T [B_1 .. B_N], and each pair's P is read in
// place from the product.
struct DenseEval {
    const double* Uall;  // row-major m x (na * r): anchor a's basis in columns a*r .. a*r + r
    int na, r, m;
    const void* Ball;    // row-major m x ksum (row stride ldb): the candidates side by side
    bool ball_f32;
    long ksum;
    long ldb;
};

// Runs fn(t, lo, hi) over nt contiguous ranges of [0, n), range t on its own thread
// (range 0 and any range whose thread cannot be started run on the calling thread).
// fn must not throw.
template <class F>
void parallel_ranges(int64_t n, int nt, const F& fn) {
    std::vector<std::thread> th;
    int started = 1;
    try {
        th.reserve((size_t)nt);
        for (; started < nt; ++started)
            th.emplace_back(fn, started, n * started / nt, n * (started + 1) / nt);
    } catch (...) {
    }
    for (int t = started; t < nt; ++t) fn(t, n * t / nt, n * (t + 1) / nt);
    fn(0, 0, n / nt);
    for (auto& x : th) x.join();
}

// Threads for the host passes over a pair list: none below a million pairs; at most 16,
// and few enough that the per-thread tables (three ints per block) stay within 256 MB.
int pair_threads(int64_t npairs, int64_t nblocks) {
    if (npairs < ((int64_t)1 << 20)) return 1;
    const int64_t hc = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
    const int64_t by_mem = std::max<int64_t>(1, ((int64_t)256 << 20) / (12 * std::max<int64_t>(nblocks, 1)));
    return (int)std::max<int64_t>(1, std::min<int64_t>({16, hc, npairs >> 18, by_mem}));
}

// Pinned host staging for the pair records of a dense evaluation (grow-only).  The
// previous call's upload from it may still be in flight: wait for it before the
// staging is rewritten or replaced.
cmsvd_status ensure_rec_pin(cmsvd_ctx* h, size_t need) {
    if (h->rec_ev_armed) {
        HIPCHK(hipEventSynchronize(h->rec_ev));
        h->rec_ev_armed = false;
    }
    if (need <= h->rec_pin_cap) return CMSVD_OK;
    const size_t want = std::max(need, h->rec_pin_cap + h->rec_pin_cap / 2);
    if (h->rec_pin) HIPCHK(hipHostFree(h->rec_pin));
    h->rec_pin = nullptr;
    h->rec_pin_cap = 0;
    if (hipHostMalloc((void**)&h->rec_pin, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        h->rec_pin = nullptr;
        return fail(CMSVD_ENOMEM, "hipHostMalloc(%zu bytes) for the pair records failed", want);
    }
    h->rec_pin_cap = want;
    return CMSVD_OK;
}

// Layout of the staged records: anchor table, candidate table, pair records (grouped
// by anchor slot), each 256-byte aligned; the same offsets on the host and the device.
struct RecLayout {
    size_t b_a, b_c, total;
    RecLayout(size_t na, size_t nc, size_t npairs)
        : b_a(align256(na * sizeof(AnchorRec))), b_c(align256(nc * sizeof(CandRec))),
          total(b_a + b_c + npairs * sizeof(PairRec)) {}
    AnchorRec* anchors(char* base) const { return reinterpret_cast<AnchorRec*>(base); }
    CandRec* cands(char* base) const { return reinterpret_cast<CandRec*>(base + b_a); }
    PairRec* pairs(char* base) const { return reinterpret_cast<PairRec*>(base + b_a + b_c); }
};

// One chunk [a0, a1) of anchor slots of a dense evaluation: its pairs are records
// pos .. pos + nj of the grouped list, its packed candidate columns [cmin, cmax).
struct DenseChunk {
    int a0, a1;
    size_t pos, nj;
    long cmin, cmax;
    int nslots;
    double* C = nullptr;         // the chunk's products, (a1 - a0) r rows
    EigDesc* ed = nullptr;       // its eigenproblem descriptors
    double* eig_ws = nullptr;    // eigen kernel scratch
};

// Plans the chunk's workspace and launches its projection
// C = [U_a0 .. U_a1-1]^T B[:, cmin:cmax) on the handle's stream.
cmsvd_status dense_project(cmsvd_ctx* h, const DenseEval& de, int nmax, DenseChunk& ch) {
    const int r = de.r;
    const long ldc = (long)(ch.a1 - ch.a0) * r;
    Plan pl;
    const size_t c_off = pl.add((size_t)ldc * (ch.cmax - ch.cmin) * 8);
    const size_t d_off = pl.add(ch.nj * sizeof(EigDesc));
    const size_t eig_off = pl.add(sym_eig_workspace_doubles(nmax, ch.nslots) * 8);
    cmsvd_status st = ensure(h, h->ws, h->ws_cap, pl.off);
    if (st != CMSVD_OK) return st;
    ch.C = reinterpret_cast<double*>(h->ws + c_off);
    ch.ed = reinterpret_cast<EigDesc*>(h->ws + d_off);
    ch.eig_ws = reinterpret_cast<double*>(h->ws + eig_off);
    GemmGroup g;
    g.tb = true;
    g.bf32 = de.ball_f32;
    g.prec = proj_prec(h);
    const char* Bc = static_cast<const char*>(de.Ball) + (size_t)ch.cmin * (de.ball_f32 ? 4 : 8);
    g.push(GemmDesc{de.Uall + (size_t)ch.a0 * r, Bc, ch.C, (int)ldc, (int)(ch.cmax - ch.cmin), de.m, (long)de.na * r,
                    de.ldb, ldc});
    Stage stg;
    g.off = stg.add(g.d);
    char* db = nullptr;
    st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    {
        StageMark mark(h, ST_PROJ);
        run_gemm(h, g, db);
    }
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

// Expands the chunk's pair records (on the device) into eigenproblem descriptors next to
// its products and evaluates the cores; arrow: one-column candidates (arrowhead cores).
cmsvd_status dense_cores(cmsvd_ctx* h, const DenseEval& de, int nmax, bool arrow, const DenseChunk& ch,
                         const AnchorRec* dA, const CandRec* dC, const PairRec* dP, double* err, double* rel) {
    const long ldc = (long)(ch.a1 - ch.a0) * de.r;
    expand_dense_descs(dP + ch.pos, (int)ch.nj, dA, dC, de.r, ch.a0, ch.C, ldc, ch.cmin, err, rel, ch.ed, h->stream);
    {
        StageMark mark(h, ST_CORE);
        if (arrow)
            arrow_eig_batched(ch.ed, (int)ch.nj, de.r, h->stream);
        else
            sym_eig_batched(ch.ed, (int)ch.nj, nmax, 0, ch.eig_ws, ch.nslots, h->stream);
    }
    HIPCHK(hipGetLastError());
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
        run_gemm(h, g32, db);
        run_gemm(h, g64, db);
    }
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

// One GEMM (column-major, FP64 accumulate) issued on the handle's stream.
cmsvd_status gemm1(cmsvd_ctx* h, bool ta, bool tb, int M, int N, int K, double alpha, const void* A, long lda,
                   bool af32, const void* B, long ldb, bool bf32, double beta, double* C, long ldc) {
    if (M <= 0 || N <= 0) return CMSVD_OK;
    GemmGroup g;
    g.ta = ta;
    g.tb = tb;
    g.af32 = af32;
    g.bf32 = bf32;
    g.alpha = alpha;
    g.beta = beta;
    g.push(GemmDesc{A, B, C, M, N, K, lda, ldb, ldc});
    Stage stg;
    g.off = stg.add(g.d);
    char* db = nullptr;
    cmsvd_status st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    run_gemm(h, g, db);
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

// Cast-copy of a row-major block into a row-major FP64 matrix with row stride = cols.
cmsvd_status copy_block(cmsvd_ctx* h, const cmsvd_block& b, double* dst) {
    std::vector<CopyDesc> cd{CopyDesc{b.ptr, (int)b.rows, (int)b.cols, (long)b.ld, b.dtype == CMSVD_F32 ? 1 : 0, dst,
                                      (long)b.cols}};
    Stage stg;
    const size_t o = stg.add(cd);
    char* db = nullptr;
    cmsvd_status st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    copy_f64_batched(reinterpret_cast<const CopyDesc*>(db + o), 1, (int)b.rows, h->stream);
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

// ---------------------------------------------------------------------------
// Residual-certified clustering (Theorem 2, Corollary 1, Algorithm 2).
//
// Cluster state: Q, an orthonormal basis of the numerical span of the accepted blocks
// (row-major m x qcap, the first q columns valid); L, the r largest squared residual
// singular values (non-increasing, zero-padded); S, the energy (double-double).  L and
// S are ping-pong pairs so that an acceptance never reads what it writes.
// ---------------------------------------------------------------------------
struct ResidState {
    int m = 0, r = 0, qcap = 0, q = 0, cur = 0;
    double* Q = nullptr;
    double* L[2] = {nullptr, nullptr};
    double* S[2] = {nullptr, nullptr};
    int* map = nullptr;    // kmax ints
    int* count = nullptr;  // 1 int
};

struct ResidCand {
    cmsvd_block B;
    const double* nb;  // double-double ||B||^2
    const double* G;   // B^T B (k x k)
    double* lam;       // min(r, k) slots: the largest residual-Gram eigenvalues
    double* rel;
    double* err;       // may be null
};

// The residual Gram of a candidate is G - P^T P with P = Q^T B (Q orthonormal), so its
// spectrum needs one projection GEMM and a k x k eigenproblem; the certificate then
// merges the top of that spectrum with L.
cmsvd_status resid_eval(cmsvd_ctx* h, const ResidState& st, const std::vector<ResidCand>& cands) {
    const size_t total = cands.size();
    if (total == 0) return CMSVD_OK;
    const int q = st.q, r = st.r;
    size_t b0 = 0;
    while (b0 < total) {
        // chunk so that the per-candidate P and residual Gram stay within ~8 GiB
        size_t b1 = b0, bytes = 0;
        int kmax = 1;
        while (b1 < total) {
            const size_t k = (size_t)cands[b1].B.cols;
            const size_t need = q > 0 ? align256((size_t)q * k * 8) + align256(k * k * 8) : 0;
            if (b1 > b0 && bytes + need > ((size_t)8 << 30)) break;
            bytes += need;
            kmax = std::max(kmax, (int)k);
            ++b1;
        }
        const int nj = (int)(b1 - b0);
        const int nslots = std::min(nj, h->ncu);
        Plan pl;
        std::vector<size_t> oP(nj), oG(nj);
        if (q > 0)
            for (int i = 0; i < nj; ++i) {
                const size_t k = (size_t)cands[b0 + i].B.cols;
                oP[i] = pl.add((size_t)q * k * 8);
                oG[i] = pl.add(k * k * 8);
            }
        const size_t eig_off = pl.add(sym_eig_workspace_doubles(kmax, nslots) * 8);
        cmsvd_status s = ensure(h, h->ws, h->ws_cap, pl.off);
        if (s != CMSVD_OK) return s;
        auto D = [&](size_t off) { return reinterpret_cast<double*>(h->ws + off); };
        GemmGroup gP32, gP64, gS;
        gP32.tb = gP64.tb = true;  // P = Q^T B
        gP32.bf32 = true;
        gS.ta = true;              // GR -= P^T P
        gS.alpha = -1.0;
        gS.beta = 1.0;
        std::vector<CopyDesc> cd;
        std::vector<EigDesc> ed(nj);
        std::vector<CertDesc> ct(nj);
        int nkmax = 1;
        for (int i = 0; i < nj; ++i) {
            const ResidCand& c = cands[b0 + i];
            const int k = (int)c.B.cols, nk = std::min(r, k);
            nkmax = std::max(nkmax, nk);
            const double* Y = c.G;
            if (q > 0) {
                GemmDesc g{st.Q, c.B.ptr, D(oP[i]), q, k, st.m, (long)st.qcap, (long)c.B.ld, (long)q};
                (c.B.dtype == CMSVD_F32 ? gP32 : gP64).push(g);
                cd.push_back(CopyDesc{c.G, k, k, (long)k, 0, D(oG[i]), (long)k});
                gS.push(GemmDesc{D(oP[i]), D(oP[i]), D(oG[i]), k, k, q, (long)q, (long)q, (long)k});
                Y = D(oG[i]);
            }
            EigDesc e{};
            e.n = k;
            e.n1 = 0;
            e.nkeep = nk;
            e.Y = Y;
            e.ldy = k;
            e.lam = c.lam;
            ed[i] = e;
            ct[i] = CertDesc{st.L[st.cur], st.S[st.cur], c.nb, c.lam, nk, c.rel, c.err};
        }
        Stage stg;
        gP32.off = stg.add(gP32.d);
        gP64.off = stg.add(gP64.d);
        gS.off = stg.add(gS.d);
        const size_t o_cd = stg.add(cd), o_ed = stg.add(ed), o_ct = stg.add(ct);
        char* db = nullptr;
        s = upload(h, stg, &db);
        if (s != CMSVD_OK) return s;
        if (q > 0) {
            StageMark mark(h, ST_PROJ);
            run_gemm(h, gP32, db);
            run_gemm(h, gP64, db);
            copy_f64_batched(reinterpret_cast<const CopyDesc*>(db + o_cd), (int)cd.size(), kmax, h->stream);
            run_gemm(h, gS, db);
        }
        {
            StageMark mark(h, ST_CORE);
            sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), nj, kmax, 1, D(eig_off), nslots, h->stream);
        }
        resid_cert_batched(reinterpret_cast<const CertDesc*>(db + o_ct), nj, r, nkmax, h->stream);
        HIPCHK(hipGetLastError());
        b0 = b1;
    }
    return CMSVD_OK;
}

// out[j] = ||Q^T B_j||_F^2 for a list of blocks (Q m x q, row-major, row stride ldq):
// one grouped projection GEMM per 8 GiB of products, then column-block sums of squares.
cmsvd_status proj_sumsq(cmsvd_ctx* h, const double* Q, long ldq, int q, int m, const std::vector<cmsvd_block>& bl,
                        const std::vector<double*>& out) {
    const size_t total = bl.size();
    if (total == 0) return CMSVD_OK;
    if (q == 0) {
        for (double* o : out) fill_f64(o, 1, 0.0, h->stream);
        HIPCHK(hipGetLastError());
        return CMSVD_OK;
    }
    size_t b0 = 0;
    while (b0 < total) {
        size_t b1 = b0, bytes = 0;
        while (b1 < total) {
            const size_t need = align256((size_t)q * bl[b1].cols * 8);
            if (b1 > b0 && bytes + need > ((size_t)8 << 30)) break;
            bytes += need;
            ++b1;
        }
        Plan pl;
        std::vector<size_t> oP(b1 - b0);
        for (size_t i = b0; i < b1; ++i) oP[i - b0] = pl.add((size_t)q * bl[i].cols * 8);
        cmsvd_status s = ensure(h, h->ws, h->ws_cap, pl.off);
        if (s != CMSVD_OK) return s;
        GemmGroup g32, g64;
        g32.tb = g64.tb = true;
        g32.bf32 = true;
        std::vector<ColNormDesc> cn;
        for (size_t i = b0; i < b1; ++i) {
            double* P = reinterpret_cast<double*>(h->ws + oP[i - b0]);
            GemmDesc g{Q, bl[i].ptr, P, q, (int)bl[i].cols, m, ldq, (long)bl[i].ld, (long)q};
            (bl[i].dtype == CMSVD_F32 ? g32 : g64).push(g);
            cn.push_back(ColNormDesc{P, q, (int)bl[i].cols, (long)q, out[i]});
        }
        Stage stg;
        g32.off = stg.add(g32.d);
        g64.off = stg.add(g64.d);
        const size_t oc = stg.add(cn);
        char* db = nullptr;
        s = upload(h, stg, &db);
        if (s != CMSVD_OK) return s;
        {
            StageMark mark(h, ST_PROJ);
            run_gemm(h, g32, db);
            run_gemm(h, g64, db);
        }
        colblock_sumsq_batched(reinterpret_cast<const ColNormDesc*>(db + oc), (int)cn.size(), h->stream);
        HIPCHK(hipGetLastError());
        b0 = b1;
    }
    return CMSVD_OK;
}

// ||Q^T B_j||_F^2 for every candidate (the residual ordering of a pass: the residual
// energy is ||B_j||^2 minus this).
cmsvd_status resid_proj_norms(cmsvd_ctx* h, const ResidState& st, const std::vector<cmsvd_block>& bl,
                              const std::vector<double*>& out) {
    return proj_sumsq(h, st.Q, (long)st.qcap, st.q, st.m, bl, out);
}

// Accepts a block whose residual spectrum `lam` (nk values) was computed against the
// current state: merges the spectrum into L, adds the energy, and appends the
// numerically present directions of its residual to Q.  The residual is projected
// twice (classical Gram-Schmidt, twice) and orthonormalised by CholeskyQR2 with the
// semidefinite pivot threshold k u ||B||^2, so that a direction with squared singular
// value below it is not added.  Synchronises to learn the new basis width.
cmsvd_status resid_accept_block(cmsvd_ctx* h, ResidState& st, const cmsvd_block& B, const double* nb,
                                const double* lam, int nk) {
    hipStream_t s = h->stream;
    const int nxt = 1 - st.cur;
    resid_accept(st.L[st.cur], st.r, lam, nk, st.S[st.cur], nb, st.L[nxt], st.S[nxt], s);
    st.cur = nxt;
    const int k = (int)B.cols, m = st.m, q = st.q;
    if (q >= st.qcap) {
        HIPCHK(hipGetLastError());
        return CMSVD_OK;
    }
    Plan pl;
    const size_t oRt = pl.add((size_t)k * m * 8), oP = pl.add((size_t)std::max(q, 1) * k * 8),
                 oP2 = pl.add((size_t)std::max(q, 1) * k * 8), oG1 = pl.add((size_t)k * k * 8),
                 oL1 = pl.add((size_t)k * k * 8), oQ1 = pl.add((size_t)k * m * 8), oG2 = pl.add((size_t)k * k * 8),
                 oL2 = pl.add((size_t)k * k * 8), oQr = pl.add((size_t)k * m * 8),
                 oCs = pl.add(CholPlan::scratch_doubles(k) * 8);
    cmsvd_status st_ = ensure(h, h->ws, h->ws_cap, pl.off);
    if (st_ != CMSVD_OK) return st_;
    auto D = [&](size_t off) { return reinterpret_cast<double*>(h->ws + off); };
    const bool f32 = B.dtype == CMSVD_F32;
    std::vector<CopyDesc> cd{CopyDesc{B.ptr, m, k, (long)B.ld, f32 ? 1 : 0, D(oRt), (long)k}};
    GemmGroup gP, gR1, gP2, gR2, gG1, gQ1, gG2, gQr;
    gP.tb = true;
    gP.bf32 = f32;
    gR1.ta = true;
    gR1.alpha = -1.0;
    gR1.beta = 1.0;
    gP2.tb = true;
    gR2.ta = true;
    gR2.alpha = -1.0;
    gR2.beta = 1.0;
    gG1.tb = true;
    gG2.tb = true;
    if (q > 0) {
        gP.push(GemmDesc{st.Q, B.ptr, D(oP), q, k, m, (long)st.qcap, (long)B.ld, (long)q});
        gR1.push(GemmDesc{D(oP), st.Q, D(oRt), k, m, q, (long)q, (long)st.qcap, (long)k});
        gP2.push(GemmDesc{st.Q, D(oRt), D(oP2), q, k, m, (long)st.qcap, (long)k, (long)q});
        gR2.push(GemmDesc{D(oP2), st.Q, D(oRt), k, m, q, (long)q, (long)st.qcap, (long)k});
    }
    gG1.push(GemmDesc{D(oRt), D(oRt), D(oG1), k, k, m, (long)k, (long)k, (long)k});
    gQ1.push(GemmDesc{D(oL1), D(oRt), D(oQ1), k, m, k, (long)k, (long)k, (long)k});
    gG2.push(GemmDesc{D(oQ1), D(oQ1), D(oG2), k, k, m, (long)k, (long)k, (long)k});
    gQr.push(GemmDesc{D(oL2), D(oQ1), D(oQr), k, m, k, (long)k, (long)k, (long)k});
    CholPlan cp1, cp2;
    cp1.build({CholDesc{k, D(oG1), (long)k, D(oL1), (long)k, (double)k * EPS, nb, nullptr}}, {D(oCs)});
    cp2.build({CholDesc{k, D(oG2), (long)k, D(oL2), (long)k, (double)k * k * EPS, nullptr, nullptr}}, {D(oCs)});
    Stage stg;
    const size_t o_cd = stg.add(cd);
    cp1.stage(stg);
    cp2.stage(stg);
    for (GemmGroup* g : {&gP, &gR1, &gP2, &gR2, &gG1, &gQ1, &gG2, &gQr}) g->off = stg.add(g->d);
    char* db = nullptr;
    st_ = upload(h, stg, &db);
    if (st_ != CMSVD_OK) return st_;
    {
        StageMark mark(h, ST_COMMIT);
        copy_f64_batched(reinterpret_cast<const CopyDesc*>(db + o_cd), 1, m, s);
        run_gemm(h, gP, db);
        run_gemm(h, gR1, db);
        run_gemm(h, gP2, db);
        run_gemm(h, gR2, db);
        run_gemm(h, gG1, db);
        cp1.run(h, db);
        run_gemm(h, gQ1, db);
        run_gemm(h, gG2, db);
        cp2.run(h, db);
        run_gemm(h, gQr, db);
        append_kept_columns(D(oQr), m, k, D(oL2), (long)k, st.Q, (long)st.qcap, q, st.qcap - q, st.map, st.count, s);
    }
    HIPCHK(hipGetLastError());
    int added = 0;
    HIPCHK(hipMemcpyAsync(&added, st.count, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    st.q += added;
    return CMSVD_OK;
}

// Empties the state (basis width 0, L = 0, S = 0).
cmsvd_status resid_reset(cmsvd_ctx* h, ResidState& st) {
    st.q = 0;
    st.cur = 0;
    fill_f64(st.L[0], st.r, 0.0, h->stream);
    fill_f64(st.S[0], 2, 0.0, h->stream);
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}



struct ResidBuffers {
    DevBuf keep;
    std::vector<double*> nrm, gram;
    double *lam = nullptr, *rel = nullptr, *err = nullptr, *pn = nullptr;
    int* first = nullptr;
    int* flags = nullptr;  // nblocks ints
    double* own = nullptr;  // nblocks x nkcap: the largest eigenvalues of each block's own Gram
    int nkcap = 1;
    ResidState st;
};

cmsvd_status resid_setup(cmsvd_ctx* h, const cmsvd_block* blocks, int N, int64_t r, const char* who, ResidBuffers& rb) {
    if (N < 1 || !blocks) return fail(CMSVD_EINVAL, "%s: no blocks", who);
    const int64_t m = blocks[0].rows;
    if (m < 1) return fail(CMSVD_ESHAPE, "%s: m < 1", who);
    if (r < 1 || r > m) return fail(CMSVD_ESHAPE, "%s: need 1 <= r <= m", who);
    if (r > 4096) return fail(CMSVD_EUNSUPPORTED, "%s: r > 4096", who);
    int64_t kmax = 0, ksum = 0;
    for (int i = 0; i < N; ++i) {
        cmsvd_status s = check_block(blocks[i], m, "block", i);
        if (s != CMSVD_OK) return s;
        s = check_order(blocks[i].cols, who);
        if (s != CMSVD_OK) return s;
        kmax = std::max(kmax, blocks[i].cols);
        ksum += blocks[i].cols;
    }
    const int64_t qcap = std::min(m, ksum);
    rb.nkcap = (int)std::min<int64_t>(r, kmax);
    Plan pl;
    std::vector<size_t> o_n(N), o_g(N);
    const size_t o_nall = pl.add(16 * (size_t)N);  // norms side by side: one read-back
    for (int i = 0; i < N; ++i) {
        o_n[i] = o_nall + 16 * (size_t)i;
        o_g[i] = pl.add((size_t)blocks[i].cols * blocks[i].cols * 8);
    }
    const size_t o_Q = pl.add((size_t)m * qcap * 8);
    size_t o_L[2], o_S[2];
    for (int s = 0; s < 2; ++s) {
        o_L[s] = pl.add((size_t)r * 8);
        o_S[s] = pl.add(16);
    }
    const size_t o_lam = pl.add((size_t)N * rb.nkcap * 8), o_rel = pl.add((size_t)N * 8), o_err = pl.add((size_t)N * 8),
                 o_pn = pl.add((size_t)N * 8), o_first = pl.add(8), o_cnt = pl.add(8), o_map = pl.add((size_t)kmax * 4),
                 o_flags = pl.add((size_t)N * 4), o_own = pl.add((size_t)N * rb.nkcap * 8);
    {
        const cmsvd_status sa = rb.keep.get(h, pl.off);
        if (sa != CMSVD_OK) return sa;
    }
    char* base = rb.keep.p;
    auto K = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
    for (int i = 0; i < N; ++i) {
        rb.nrm.push_back(K(o_n[i]));
        rb.gram.push_back(K(o_g[i]));
    }
    rb.lam = K(o_lam);
    rb.rel = K(o_rel);
    rb.err = K(o_err);
    rb.pn = K(o_pn);
    rb.first = reinterpret_cast<int*>(base + o_first);
    rb.flags = reinterpret_cast<int*>(base + o_flags);
    rb.own = K(o_own);
    rb.st.m = (int)m;
    rb.st.r = (int)r;
    rb.st.qcap = (int)qcap;
    rb.st.Q = K(o_Q);
    for (int s = 0; s < 2; ++s) {
        rb.st.L[s] = K(o_L[s]);
        rb.st.S[s] = K(o_S[s]);
    }
    rb.st.count = reinterpret_cast<int*>(base + o_cnt);
    rb.st.map = reinterpret_cast<int*>(base + o_map);
    std::vector<cmsvd_block> bl(blocks, blocks + N);
    cmsvd_status s = norms_and_grams(h, bl, rb.nrm, rb.gram);
    if (s != CMSVD_OK) return s;
    // every block's own residual spectrum against an empty basis (the anchor's), in one
    // batched launch: the top min(r, k) eigenvalues of its Gram
    const int nslots = std::min(N, h->ncu);
    Plan pw;
    const size_t eig_off = pw.add(sym_eig_workspace_doubles((int)kmax, nslots) * 8);
    s = ensure(h, h->ws, h->ws_cap, pw.off);
    if (s != CMSVD_OK) return s;
    std::vector<EigDesc> ed(N);
    for (int i = 0; i < N; ++i) {
        EigDesc e{};
        e.n = (int)blocks[i].cols;
        e.n1 = 0;
        e.nkeep = (int)std::min<int64_t>(r, blocks[i].cols);
        e.Y = rb.gram[i];
        e.ldy = (long)blocks[i].cols;
        e.lam = rb.own + (size_t)i * rb.nkcap;
        ed[i] = e;
    }
    Stage stg;
    const size_t o = stg.add(ed);
    char* db = nullptr;
    s = upload(h, stg, &db);
    if (s != CMSVD_OK) return s;
    {
        StageMark mark(h, ST_PREP);
        sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o), N, (int)kmax, 1,
                        reinterpret_cast<double*>(h->ws + eig_off), nslots, h->stream);
    }
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

// Tests the candidates `cand` (in order) against the current state; rel[i], lam slot i.
cmsvd_status resid_test(cmsvd_ctx* h, ResidBuffers& rb, const cmsvd_block* blocks, const std::vector<int>& cand) {
    std::vector<ResidCand> rc;
    rc.reserve(cand.size());
    for (size_t i = 0; i < cand.size(); ++i) {
        const int j = cand[i];
        rc.push_back(ResidCand{blocks[j], rb.nrm[j], rb.gram[j], rb.lam + i * (size_t)rb.nkcap, rb.rel + i, rb.err + i});
    }
    return resid_eval(h, rb.st, rc);
}

// Scans the candidates `cand` (in order) for the first whose certificate is within
// eps.  Chunk by chunk: the projections P_c = Q^T B_c and ||P_c||_F^2 settle most
// candidates without eigenvalues (resid_screen); the certificate proper (residual
// Gram G - P^T P, its top eigenvalues, the merge with L) is computed only for the
// unsettled candidates ahead of the first sure acceptance, and for an accepted
// candidate whose spectrum is still missing.  *first = index of the first feasible
// candidate (cand.size() if none); its residual spectrum is then in lam slot *first.
// Synchronises once or twice per chunk.
cmsvd_status resid_scan(cmsvd_ctx* h, ResidBuffers& rb, const cmsvd_block* blocks, const std::vector<int>& cand,
                        double eps, int* first) {
    const ResidState& st = rb.st;
    const size_t total = cand.size();
    const int q = st.q, r = st.r;
    hipStream_t s = h->stream;
    *first = (int)total;
    size_t b0 = 0;
    while (b0 < total) {
        size_t b1 = b0, bytes = 0;
        int kmax = 1;
        while (b1 < total) {
            const size_t k = (size_t)blocks[cand[b1]].cols;
            const size_t need = align256((size_t)std::max(q, 1) * k * 8) + align256(k * k * 8);
            if (b1 > b0 && bytes + need > ((size_t)8 << 30)) break;
            bytes += need;
            kmax = std::max(kmax, (int)k);
            ++b1;
        }
        const int nj = (int)(b1 - b0);
        Plan pl;
        std::vector<size_t> oP(nj), oG(nj);
        for (int i = 0; i < nj; ++i) {
            const size_t k = (size_t)blocks[cand[b0 + i]].cols;
            oP[i] = pl.add((size_t)std::max(q, 1) * k * 8);
            oG[i] = pl.add(k * k * 8);
        }
        const int nslots = std::min(nj, h->ncu);
        const size_t eig_off = pl.add(sym_eig_workspace_doubles(kmax, nslots) * 8);
        cmsvd_status stt = ensure(h, h->ws, h->ws_cap, pl.off);
        if (stt != CMSVD_OK) return stt;
        auto D = [&](size_t off) { return reinterpret_cast<double*>(h->ws + off); };
        // phase 1: projections, their norms, the screen
        {
            GemmGroup g32, g64;
            g32.tb = g64.tb = true;
            g32.bf32 = true;
            std::vector<ColNormDesc> cn;
            std::vector<ScreenDesc> sd(nj);
            for (int i = 0; i < nj; ++i) {
                const int j = cand[b0 + i];
                const cmsvd_block& B = blocks[j];
                if (q > 0) {
                    GemmDesc g{st.Q, B.ptr, D(oP[i]), q, (int)B.cols, st.m, (long)st.qcap, (long)B.ld, (long)q};
                    (B.dtype == CMSVD_F32 ? g32 : g64).push(g);
                    cn.push_back(ColNormDesc{D(oP[i]), q, (int)B.cols, (long)q, rb.pn + b0 + i});
                }
                sd[i] = ScreenDesc{rb.nrm[j], rb.pn + b0 + i, rb.flags + i};
            }
            Stage stg;
            g32.off = stg.add(g32.d);
            g64.off = stg.add(g64.d);
            const size_t o_cn = stg.add(cn), o_sd = stg.add(sd);
            char* db = nullptr;
            stt = upload(h, stg, &db);
            if (stt != CMSVD_OK) return stt;
            if (q > 0) {
                StageMark mark(h, ST_PROJ);
                run_gemm(h, g32, db);
                run_gemm(h, g64, db);
                colblock_sumsq_batched(reinterpret_cast<const ColNormDesc*>(db + o_cn), (int)cn.size(), s);
            } else {
                fill_f64(rb.pn + b0, nj, 0.0, s);
            }
            resid_screen(reinterpret_cast<const ScreenDesc*>(db + o_sd), nj, st.L[st.cur], r, st.S[st.cur], eps, s);
            HIPCHK(hipGetLastError());
        }
        std::vector<int> flags(nj);
        HIPCHK(hipMemcpyAsync(flags.data(), rb.flags, (size_t)nj * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int sure = nj;
        for (int i = 0; i < nj; ++i)
            if (flags[i] == 2) {
                sure = i;
                break;
            }
        std::vector<int> need;
        for (int i = 0; i < sure; ++i)
            if (flags[i] == 1) need.push_back(i);
        if (need.empty() && sure == nj) {
            b0 = b1;
            continue;
        }
        if (sure < nj) need.push_back(sure);  // its spectrum is needed for the acceptance
        // phase 2: the certificate of the unsettled candidates (and of the sure one)
        {
            GemmGroup gS;
            gS.ta = true;
            gS.alpha = -1.0;
            gS.beta = 1.0;
            std::vector<CopyDesc> cd;
            std::vector<EigDesc> ed;
            std::vector<CertDesc> ct;
            int kneed = 1, nkmax = 1;
            for (size_t u = 0; u < need.size(); ++u) {
                const int i = need[u], j = cand[b0 + i];
                const int k = (int)blocks[j].cols, nk = std::min(r, k);
                kneed = std::max(kneed, k);
                nkmax = std::max(nkmax, nk);
                double* lam = rb.lam + (b0 + i) * (size_t)rb.nkcap;
                const double* Y = rb.gram[j];
                if (q > 0) {
                    cd.push_back(CopyDesc{rb.gram[j], k, k, (long)k, 0, D(oG[i]), (long)k});
                    gS.push(GemmDesc{D(oP[i]), D(oP[i]), D(oG[i]), k, k, q, (long)q, (long)q, (long)k});
                    Y = D(oG[i]);
                }
                EigDesc e{};
                e.n = k;
                e.n1 = 0;
                e.nkeep = nk;
                e.Y = Y;
                e.ldy = k;
                e.lam = lam;
                ed.push_back(e);
                ct.push_back(CertDesc{st.L[st.cur], st.S[st.cur], rb.nrm[j], lam, nk, rb.rel + u, rb.err + u});
            }
            Stage stg;
            gS.off = stg.add(gS.d);
            const size_t o_cd = stg.add(cd), o_ed = stg.add(ed), o_ct = stg.add(ct);
            char* db = nullptr;
            stt = upload(h, stg, &db);
            if (stt != CMSVD_OK) return stt;
            if (q > 0) {
                StageMark mark(h, ST_PROJ);
                copy_f64_batched(reinterpret_cast<const CopyDesc*>(db + o_cd), (int)cd.size(), kneed, s);
                run_gemm(h, gS, db);
            }
            {
                StageMark mark(h, ST_CORE);
                sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), (int)ed.size(), kneed, 1, D(eig_off),
                                std::min((int)ed.size(), nslots), s);
            }
            resid_cert_batched(reinterpret_cast<const CertDesc*>(db + o_ct), (int)ct.size(), r, nkmax, s);
            HIPCHK(hipGetLastError());
        }
        const int nun = (int)need.size() - (sure < nj ? 1 : 0);  // unsettled ones, in scan order
        int idx = nun;
        if (nun > 0) {
            first_feasible(rb.rel, nun, eps, rb.first, s);
            HIPCHK(hipMemcpyAsync(&idx, rb.first, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        if (idx < nun) {
            *first = (int)b0 + need[idx];
            return CMSVD_OK;
        }
        if (sure < nj) {
            *first = (int)(b0 + sure);
            return CMSVD_OK;
        }
        b0 = b1;
    }
    return CMSVD_OK;
}

// Certified ratio sqrt(max(0, S - sum L) / S) of the current state (device rel[0]).
cmsvd_status resid_state_rel(cmsvd_ctx* h, ResidBuffers& rb, double* rel_host, double* b2_host) {
    std::vector<CertDesc> ct{CertDesc{rb.st.L[rb.st.cur], rb.st.S[rb.st.cur], nullptr, rb.lam, 0, rb.rel, rb.err}};
    Stage stg;
    const size_t o = stg.add(ct);
    char* db = nullptr;
    cmsvd_status s = upload(h, stg, &db);
    if (s != CMSVD_OK) return s;
    resid_cert_batched(reinterpret_cast<const CertDesc*>(db + o), 1, rb.st.r, 1, h->stream);
    HIPCHK(hipGetLastError());
    double v[2] = {0.0, 0.0};
    HIPCHK(hipMemcpyAsync(&v[0], rb.rel, 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(&v[1], rb.err, 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (rel_host) *rel_host = v[0];
    if (b2_host) *b2_host = v[1] * v[1];
    return CMSVD_OK;
}

// ---------------------------------------------------------------------------
// Theorem 1 (Weyl-based certificate), Algorithm 1, and the explicit tail.
// ---------------------------------------------------------------------------
struct WeylBuffers {
    DevBuf keep;
    double* a2 = nullptr;     // nblocks x 2: block energies (double-double)
    double* h = nullptr;      // nblocks: r-head energies
    double* state = nullptr;  // S hi, S lo, m
    double* rel = nullptr;
    int* first = nullptr;
};

cmsvd_status weyl_setup(cmsvd_ctx* h, const cmsvd_block* blocks, int N, int64_t r, const char* who, WeylBuffers& wb) {
    if (N < 1 || !blocks) return fail(CMSVD_EINVAL, "%s: no blocks", who);
    const int64_t m = blocks[0].rows;
    if (m < 1) return fail(CMSVD_ESHAPE, "%s: m < 1", who);
    if (r < 1) return fail(CMSVD_ESHAPE, "%s: need r >= 1", who);
    int kmax = 0;
    for (int i = 0; i < N; ++i) {
        cmsvd_status s = check_block(blocks[i], m, "block", i);
        if (s != CMSVD_OK) return s;
        if (blocks[i].cols > r) {
            s = check_order(blocks[i].cols, who);
            if (s != CMSVD_OK) return s;
        }
        if (blocks[i].cols > r) kmax = std::max(kmax, (int)blocks[i].cols);
    }
    Plan pl;
    const size_t o_a2 = pl.add((size_t)N * 16), o_top = pl.add((size_t)N * 16), o_h = pl.add((size_t)N * 8),
                 o_st = pl.add(24), o_rel = pl.add(8), o_first = pl.add(8);
    {
        const cmsvd_status sa = wb.keep.get(h, pl.off);
        if (sa != CMSVD_OK) return sa;
    }
    char* base = wb.keep.p;
    wb.a2 = reinterpret_cast<double*>(base + o_a2);
    double* top = reinterpret_cast<double*>(base + o_top);
    wb.h = reinterpret_cast<double*>(base + o_h);
    wb.state = reinterpret_cast<double*>(base + o_st);
    wb.rel = reinterpret_cast<double*>(base + o_rel);
    wb.first = reinterpret_cast<int*>(base + o_first);
    // energies; Grams and head energies of the blocks wider than r
    std::vector<int> wide;
    for (int i = 0; i < N; ++i)
        if (blocks[i].cols > r) wide.push_back(i);
    Plan pw;
    std::vector<size_t> og(wide.size());
    for (size_t w = 0; w < wide.size(); ++w) og[w] = pw.add((size_t)blocks[wide[w]].cols * blocks[wide[w]].cols * 8);
    const size_t o_lam = pw.add(wide.size() * (size_t)r * 8);  // the eigenvalues themselves (unused)
    const int nslots = std::max(1, std::min((int)wide.size(), h->ncu));
    const size_t eig_off = pw.add(sym_eig_workspace_doubles(std::max(kmax, 1), nslots) * 8);
    cmsvd_status s = ensure(h, h->ws, h->ws_cap, pw.off);
    if (s != CMSVD_OK) return s;
    std::vector<cmsvd_block> bl(blocks, blocks + N);
    std::vector<double*> nrm(N), gram(N, nullptr);
    for (int i = 0; i < N; ++i) nrm[i] = wb.a2 + 2 * i;
    for (size_t w = 0; w < wide.size(); ++w) gram[wide[w]] = reinterpret_cast<double*>(h->ws + og[w]);
    s = norms_and_grams(h, bl, nrm, gram);
    if (s != CMSVD_OK) return s;
    std::vector<EigDesc> ed;
    for (size_t w = 0; w < wide.size(); ++w) {
        const int i = wide[w], k = (int)blocks[i].cols;
        EigDesc e{};
        e.n = k;
        e.n1 = 0;
        e.nkeep = (int)r;
        e.Y = gram[i];
        e.ldy = k;
        e.lam = reinterpret_cast<double*>(h->ws + o_lam) + w * (size_t)r;
        e.sum_top = top + 2 * i;
        ed.push_back(e);
    }
    std::vector<int> cols(N);
    for (int i = 0; i < N; ++i) cols[i] = (int)blocks[i].cols;
    Stage stg;
    const size_t o_ed = stg.add(ed), o_cols = stg.add(cols);
    char* db = nullptr;
    s = upload(h, stg, &db);
    if (s != CMSVD_OK) return s;
    if (!ed.empty()) {
        StageMark mark(h, ST_PREP);
        sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), (int)ed.size(), kmax, 1,
                        reinterpret_cast<double*>(h->ws + eig_off), nslots, h->stream);
    }
    weyl_heads(wb.a2, top, reinterpret_cast<const int*>(db + o_cols), (int)r, N, wb.h, h->stream);
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

cmsvd_status gemm_entry(cmsvd_handle h, const char* who, int prec, int32_t trans_a, int32_t trans_b, int64_t M,
                        int64_t N, int64_t K, double alpha, const void* A, int64_t lda, int32_t a_dtype, const void* B,
                        int64_t ldb, int32_t b_dtype, double beta, double* C, int64_t ldc) {
    if (!h) return fail(CMSVD_EINVAL, "%s: null handle", who);
    if (!A || !B || !C) return fail(CMSVD_EINVAL, "%s: null pointer", who);
    if (M < 0 || N < 0 || K < 0 || M > INT32_MAX || N > INT32_MAX || K > INT32_MAX)
        return fail(CMSVD_ESHAPE, "%s: bad sizes", who);
    if ((a_dtype != CMSVD_F32 && a_dtype != CMSVD_F64) || (b_dtype != CMSVD_F32 && b_dtype != CMSVD_F64))
        return fail(CMSVD_EUNSUPPORTED, "%s: dtype must be F32 or F64", who);
    const int64_t ar = trans_a ? K : M, br = trans_b ? N : K;
    if (lda < std::max<int64_t>(ar, 1) || ldb < std::max<int64_t>(br, 1) || ldc < std::max<int64_t>(M, 1))
        return fail(CMSVD_ESHAPE, "%s: leading dimension too small", who);
    if (M == 0 || N == 0) return CMSVD_OK;
    GemmGroup g;
    g.prec = prec;
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
    run_gemm(h, g, db);
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
}

}  // namespace

// ===========================================================================
// Public C ABI
// ===========================================================================
namespace {

// Width of the i-th column panel of a block under the handle's panel_cols option.
int64_t panel_count(const cmsvd_ctx* h, int64_t cols) {
    return h->panel_cols > 0 && cols > h->panel_cols ? (cols + h->panel_cols - 1) / h->panel_cols : 1;
}

// The largest core order of a panelled step sequence: r_in + first panel, then r + panel.
int64_t panelled_order(const cmsvd_ctx* h, int64_t r_in, int64_t r, int64_t cols) {
    if (panel_count(h, cols) == 1) return r_in + cols;
    return std::max(r_in, r) + h->panel_cols;
}

// Runs the incremental steps of `jobs` (one per independent state).  A block wider than
// the handle's panel_cols is appended as consecutive column panels of that width (the
// last one narrower): the same concatenation (Lemma 1 holds for any blocking) with a
// truncation after every panel.  Intermediate states (row-major m x r bases and their r
// singular values) alternate between two slots per state in the handle's buffer; the
// last panel writes the caller's outputs and est.
cmsvd_status commit_panelled(cmsvd_ctx* h, const std::vector<CommitJob>& jobs) {
    int64_t npmax = 1;
    for (const auto& j : jobs) npmax = std::max(npmax, panel_count(h, j.B.cols));
    if (npmax == 1) return commit_batched(h, jobs);
    const size_t J = jobs.size();
    size_t per = 0;  // doubles of one state slot
    for (const auto& j : jobs) per = std::max(per, (size_t)j.m * j.r + (size_t)j.r);
    cmsvd_status st = ensure(h, h->pan, h->pan_cap, 2 * J * align256(per * 8));
    if (st != CMSVD_OK) return st;
    auto slot = [&](size_t i, int64_t p) {
        return reinterpret_cast<double*>(h->pan + (2 * i + (size_t)(p & 1)) * align256(per * 8));
    };
    for (int64_t p = 0; p < npmax; ++p) {
        std::vector<CommitJob> step;
        for (size_t i = 0; i < J; ++i) {
            const CommitJob& c = jobs[i];
            const int64_t np = panel_count(h, c.B.cols);
            if (p >= np) continue;
            CommitJob q = c;
            const size_t esz = c.B.dtype == CMSVD_F32 ? 4 : 8;
            const int64_t c0 = p * h->panel_cols;
            q.B.ptr = static_cast<const char*>(c.B.ptr) + (size_t)c0 * esz;
            q.B.cols = np == 1 ? c.B.cols : std::min<int64_t>(h->panel_cols, c.B.cols - c0);
            if (p > 0) {  // the state the previous panel left
                double* prev = slot(i, p - 1);
                q.U = prev;
                q.ldu = c.r;
                q.S = prev + (size_t)c.m * c.r;
                q.r_in = c.r;
            }
            if (p + 1 < np) {  // not the last panel: write an intermediate state
                double* nxt = slot(i, p);
                q.U_out = nxt;
                q.ldu_out = c.r;
                q.S_out = nxt + (size_t)c.m * c.r;
                q.est = nullptr;
            }
            step.push_back(q);
        }
        st = commit_batched(h, step);
        if (st != CMSVD_OK) return st;
    }
    return CMSVD_OK;
}

std::string tune_key(const cmsvd_ctx* h, int64_t m, int64_t k, int64_t r) {
    static const char* pn[] = {"f64", "bf16", "bf16x3", "f32"};
    char buf[128];
    snprintf(buf, sizeof(buf), "gfx950 m=%lld k=%lld r=%lld proj=%s", (long long)m, (long long)width_bucket(k),
             (long long)r, pn[h->proj & 3]);
    return buf;
}

// The first scan chunk of Algorithm 3 for candidates of width about k: the autotuned
// value when the handle has one for this shape, else a quarter of the compute units.
size_t scan_chunk(const cmsvd_ctx* h, int64_t m, int64_t k, int64_t r) {
    auto it = h->tuned_chunk.find(tune_key(h, m, k, r));
    if (it != h->tuned_chunk.end()) return (size_t)it->second;
    return (size_t)std::max(16, h->ncu / 4);
}

// BF16 blocks are widened to FP32 (exactly: a BF16 value is an FP32 value with the low
// 16 bits zero) into the handle's buffer before a call uses them.
struct WidenDesc {
    const uint16_t* src;  // row-major BF16, row stride ld
    int rows, cols;
    long ld;
    float* dst;           // row-major FP32, row stride cols
};

__global__ void __launch_bounds__(256) widen_bf16_kernel(const WidenDesc* __restrict__ descs) {
    const WidenDesc D = descs[blockIdx.y];
    const long tot = (long)D.rows * D.cols;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
        const long r = e / D.cols, c = e - r * D.cols;
        D.dst[e] = __uint_as_float((uint32_t)D.src[r * D.ld + c] << 16);
    }
}

// When any of the n blocks is BF16: checks all of them as check_block does (with BF16
// allowed), widens the BF16 ones into h->wide and returns in `out` the descriptors the
// call goes on with (FP32 copies in place of BF16 blocks).  `out` stays empty when no
// block is BF16.  The copies live until the next call widens blocks on this handle;
// everything that reads them is ordered before that on the handle's stream.
cmsvd_status widen_blocks(cmsvd_ctx* h, const cmsvd_block* in, int64_t n, std::vector<cmsvd_block>& out,
                          const char* who) {
    out.clear();
    if (!in || n < 1) return CMSVD_OK;
    bool any = false;
    for (int64_t i = 0; i < n; ++i) any |= in[i].dtype == CMSVD_BF16;
    if (!any) return CMSVD_OK;
    const int64_t m = in[0].rows;
    size_t bytes = 0;
    for (int64_t i = 0; i < n; ++i) {
        cmsvd_block b = in[i];
        if (b.dtype == CMSVD_BF16) b.dtype = CMSVD_F32;  // same shape rules
        const cmsvd_status st = check_block(b, m, "block", i);
        if (st != CMSVD_OK) return st;
        if (in[i].dtype == CMSVD_BF16) bytes += align256((size_t)b.rows * b.cols * 4);
    }
    cmsvd_status st = ensure(h, h->wide, h->wide_cap, bytes);
    if (st != CMSVD_OK) return st;
    out.assign(in, in + n);
    std::vector<WidenDesc> wd;
    size_t off = 0;
    long maxel = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (in[i].dtype != CMSVD_BF16) continue;
        float* dst = reinterpret_cast<float*>(h->wide + off);
        wd.push_back(WidenDesc{static_cast<const uint16_t*>(in[i].ptr), (int)in[i].rows, (int)in[i].cols,
                               (long)in[i].ld, dst});
        maxel = std::max(maxel, (long)in[i].rows * in[i].cols);
        out[(size_t)i] = cmsvd_block{dst, in[i].rows, in[i].cols, in[i].cols, CMSVD_F32};
        off += align256((size_t)in[i].rows * in[i].cols * 4);
    }
    Stage stg;
    const size_t o = stg.add(wd);
    char* db = nullptr;
    st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    const WidenDesc* dd = reinterpret_cast<const WidenDesc*>(db + o);
    const int gx = (int)std::min<long>((maxel + 255) / 256, 1024);
    for (size_t b0 = 0; b0 < wd.size(); b0 += 65535) {
        const int nb = (int)std::min<size_t>(65535, wd.size() - b0);
        hipLaunchKernelGGL(widen_bf16_kernel, dim3(gx, nb), dim3(256), 0, h->stream, dd + b0);
    }
    HIPCHK(hipGetLastError());
    (void)who;
    return CMSVD_OK;
}

// Releases captured sequence i of the handle's cache.
void drop_graph(cmsvd_ctx* h, size_t i) {
    auto& e = h->graph_cache[i];
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    dev_free(h, e.dev);
    h->graph_cache.erase(h->graph_cache.begin() + (long)i);
}

}  // namespace

extern "C" {

const char* cmsvd_last_error(void) { return g_err.c_str(); }

cmsvd_status cmsvd_create_ex(cmsvd_handle* handle, void* hip_stream, const cmsvd_options* options,
                             void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* alloc_ctx) try {
    if (!handle) return fail(CMSVD_EINVAL, "cmsvd_create: null handle pointer");
    if ((alloc == nullptr) != (release == nullptr))
        return fail(CMSVD_EINVAL, "cmsvd_create_ex: give both allocator callbacks or neither");
    if (options) {
        const int p = options->projection;
        if (p != CMSVD_PROJ_F64 && p != CMSVD_PROJ_BF16 && p != CMSVD_PROJ_BF16X3 && p != CMSVD_PROJ_F32)
            return fail(CMSVD_EINVAL, "cmsvd_create_ex: unknown projection %d", p);
        if (options->panel_cols < 0) return fail(CMSVD_EINVAL, "cmsvd_create_ex: panel_cols < 0");
        if (!(options->chol_tau >= 0.0) || options->chol_tau > 1e12)
            return fail(CMSVD_EINVAL, "cmsvd_create_ex: chol_tau must be in [0, 1e12]");
    }
    cmsvd_ctx* h = new cmsvd_ctx();
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    h->alloc_fn = alloc;
    h->release_fn = release;
    h->alloc_ctx = alloc_ctx;
    if (options) {
        h->proj = options->projection;
        h->chol_c = options->chol_tau;
        h->panel_cols = options->panel_cols;
        h->graphs = options->graphs != 0;
    }
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
    {
        const cmsvd_status ss = scratch_address(h->device, &h->scratch);
        if (ss != CMSVD_OK) {
            delete h;
            return ss;
        }
    }
    if (hipEventCreateWithFlags(&h->pin_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->rec_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->tail_ev, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) {
        if (h->pin_ev) (void)hipEventDestroy(h->pin_ev);
        if (h->rec_ev) (void)hipEventDestroy(h->rec_ev);
        if (h->tail_ev) (void)hipEventDestroy(h->tail_ev);
        delete h;
        return fail(CMSVD_EHIP, "hipEventCreate / hipStreamCreate failed");
    }
    *handle = h;
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_create(cmsvd_handle* handle, void* hip_stream) try {
    return cmsvd_create_ex(handle, hip_stream, nullptr, nullptr, nullptr, nullptr);
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_destroy(cmsvd_handle h) try {
    if (!h) return CMSVD_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->side) (void)hipStreamSynchronize(h->side);
    while (!h->graph_cache.empty()) drop_graph(h, h->graph_cache.size() - 1);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    dev_free(h, h->ws);
    dev_free(h, h->dsc);
    dev_free(h, h->gsk);
    dev_free(h, h->rec);
    dev_free(h, h->keep);
    dev_free(h, h->pan);
    dev_free(h, h->wide);
    if (h->tail_ev) (void)hipEventDestroy(h->tail_ev);
    if (h->rec_pin) (void)hipHostFree(h->rec_pin);
    if (h->pin) (void)hipHostFree(h->pin);
    if (h->pin_ev) (void)hipEventDestroy(h->pin_ev);
    if (h->side) {
        (void)hipStreamSynchronize(h->side);
        (void)hipStreamDestroy(h->side);
    }
    if (h->rec_ev) (void)hipEventDestroy(h->rec_ev);
    for (auto& v : h->marks)
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (auto e : h->pool) (void)hipEventDestroy(e);
    delete h;
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_profile(cmsvd_handle h, int32_t enable) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_profile: null handle");
    h->timing = enable != 0;
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_profile_read(cmsvd_handle h, double* ms, int64_t* count) try {
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
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_set_projection(cmsvd_handle h, int32_t precision) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_set_projection: null handle");
    if (precision != CMSVD_PROJ_F64 && precision != CMSVD_PROJ_BF16 && precision != CMSVD_PROJ_BF16X3 &&
        precision != CMSVD_PROJ_F32)
        return fail(CMSVD_EINVAL, "cmsvd_set_projection: precision must be CMSVD_PROJ_F64, _BF16, _BF16X3 or _F32");
    h->proj = precision;
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_set_stream(cmsvd_handle h, void* hip_stream) try {
    if (!h) return fail(CMSVD_EINVAL, "null handle");
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_update(cmsvd_handle h, int64_t m, const double* U, int64_t ldu, const double* S, int64_t r_in,
                          const cmsvd_block* B, int64_t r, double* U_out, int64_t ldu_out, double* S_out, double* acc,
                          double* est) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_update: null handle");
    if (!B) return fail(CMSVD_EINVAL, "cmsvd_update: null block");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, B, 1, wide_, "cmsvd_update");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) B = wide_.data();
    }
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
    st = check_order(panelled_order(h, r_in, r, B->cols), "cmsvd_update");
    if (st != CMSVD_OK) return st;
    CommitJob j{(int)m, U, (long)ldu, S, (int)r_in, *B, (int)r, U_out, (long)ldu_out, S_out, acc, est};
    return commit_panelled(h, {j});
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_update_batch(cmsvd_handle h, int64_t count, int64_t m, const double* const* U, int64_t ldu,
                                const double* const* S, int64_t r_in, const cmsvd_block* B, int64_t r,
                                double* const* U_out, int64_t ldu_out, double* const* S_out, double* const* acc,
                                double* const* est) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_update_batch: null handle");
    if (count < 0) return fail(CMSVD_EINVAL, "cmsvd_update_batch: count < 0");
    if (count == 0) return CMSVD_OK;
    if (!B || !U_out || !S_out || !acc) return fail(CMSVD_EINVAL, "cmsvd_update_batch: null array");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, B, count, wide_, "cmsvd_update_batch");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) B = wide_.data();
    }
    if (m < 1) return fail(CMSVD_ESHAPE, "cmsvd_update_batch: m < 1");
    if (r < 1 || r > m) return fail(CMSVD_ESHAPE, "cmsvd_update_batch: need 1 <= r <= m");
    if (r > 4096) return fail(CMSVD_EUNSUPPORTED, "cmsvd_update_batch: r > 4096");
    if (r_in < 0 || r_in > m) return fail(CMSVD_ESHAPE, "cmsvd_update_batch: bad r_in");
    if (r_in > 0 && (!U || !S || ldu < r_in)) return fail(CMSVD_EINVAL, "cmsvd_update_batch: bad state arrays");
    if (ldu_out < r) return fail(CMSVD_ESHAPE, "cmsvd_update_batch: ldu_out < r");
    std::vector<CommitJob> jobs;
    for (int64_t i = 0; i < count; ++i) {
        cmsvd_status st = check_block(B[i], m, "block", i);
        if (st != CMSVD_OK) return st;
        st = check_order(panelled_order(h, r_in, r, B[i].cols), "cmsvd_update_batch");
        if (st != CMSVD_OK) return st;
        if (!U_out[i] || !S_out[i] || !acc[i]) return fail(CMSVD_EINVAL, "cmsvd_update_batch: null output %lld", (long long)i);
        if (r_in > 0 && (!U[i] || !S[i])) return fail(CMSVD_EINVAL, "cmsvd_update_batch: null state %lld", (long long)i);
        if (r_in > 0 && (U_out[i] == U[i] || S_out[i] == S[i]))
            return fail(CMSVD_EINVAL, "cmsvd_update_batch: outputs alias inputs (%lld)", (long long)i);
        jobs.push_back(CommitJob{(int)m, r_in > 0 ? U[i] : nullptr, (long)ldu, r_in > 0 ? S[i] : nullptr, (int)r_in, B[i],
                                 (int)r, U_out[i], (long)ldu_out, S_out[i], acc[i], est ? est[i] : nullptr});
    }
    return commit_panelled(h, jobs);
} catch (...) {
    return caught(__func__);
}

// The body of cmsvd_merge_errors; *dense_out tells whether the dense (thin-candidate)
// path ran, which reads the block norms back mid-call and is never captured.
static cmsvd_status merge_errors_run(cmsvd_ctx* h, const cmsvd_block* blocks, int64_t nblocks, const int32_t* pairs,
                                     int64_t npairs, int64_t r, double* err, double* rel, bool* dense_out) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_merge_errors: null handle");
    if (nblocks < 1 || !blocks) return fail(CMSVD_EINVAL, "cmsvd_merge_errors: no blocks");
    if (npairs < 0 || (npairs > 0 && (!pairs || !err))) return fail(CMSVD_EINVAL, "cmsvd_merge_errors: null pairs/err");
    if (nblocks > INT32_MAX || npairs > INT32_MAX) return fail(CMSVD_EUNSUPPORTED, "cmsvd_merge_errors: too many blocks or pairs");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, blocks, nblocks, wide_, "cmsvd_merge_errors");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) blocks = wide_.data();
    }
    const int64_t m = blocks[0].rows;
    if (m < 1) return fail(CMSVD_ESHAPE, "cmsvd_merge_errors: m < 1");
    if (r < 1 || r > m) return fail(CMSVD_ESHAPE, "cmsvd_merge_errors: need 1 <= r <= m");
    if (r > 4096) return fail(CMSVD_EUNSUPPORTED, "cmsvd_merge_errors: r > 4096");
    for (int64_t i = 0; i < nblocks; ++i) {
        cmsvd_status st = check_block(blocks[i], m, "block", i);
        if (st != CMSVD_OK) return st;
    }
    // One pass over the pairs: the range check, how often each block is an anchor and a
    // candidate, and each anchor's widest candidate (the largest eigenproblem it meets).
    // Long lists are split into contiguous ranges, one per thread, each with its own
    // tables; the record pass below uses the same ranges.
    std::vector<int> colsv(nblocks);
    for (int64_t i = 0; i < nblocks; ++i) colsv[i] = (int)blocks[i].cols;
    const int nt = pair_threads(npairs, nblocks);
    std::vector<std::vector<int>> tac(nt, std::vector<int>(nblocks, 0)), tcc(nt, std::vector<int>(nblocks, 0)),
        taw(nt, std::vector<int>(nblocks, 0));
    std::vector<int64_t> tbad(nt, -1);
    parallel_ranges(npairs, nt, [&](int t, int64_t lo, int64_t hi) {
        int* ac = tac[t].data();
        int* cc = tcc[t].data();
        int* aw = taw[t].data();
        for (int64_t p = lo; p < hi; ++p) {
            const int32_t a = pairs[2 * p], b = pairs[2 * p + 1];
            if (a < 0 || a >= nblocks || b < 0 || b >= nblocks) {
                tbad[t] = p;
                return;
            }
            ++ac[a];
            ++cc[b];
            aw[a] = std::max(aw[a], colsv[b]);
        }
    });
    for (int t = 0; t < nt; ++t)
        if (tbad[t] >= 0) {
            const int64_t p = tbad[t];
            return fail(CMSVD_EINVAL, "cmsvd_merge_errors: pair %lld = (%d, %d) out of range", (long long)p,
                        pairs[2 * p], pairs[2 * p + 1]);
        }
    std::vector<int> acount(nblocks), ccount(nblocks), awide(nblocks);
    parallel_ranges(nblocks, nt, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            int a = 0, c = 0, w = 0;
            for (int t = 0; t < nt; ++t) {
                a += tac[t][i];
                c += tcc[t][i];
                w = std::max(w, taw[t][i]);
            }
            acount[i] = a;
            ccount[i] = c;
            awide[i] = w;
        }
    });
    std::vector<std::vector<int>>().swap(tcc);
    std::vector<std::vector<int>>().swap(taw);
    for (int64_t i = 0; i < nblocks; ++i)
        if (acount[i]) {
            cmsvd_status st = check_order(std::max<int64_t>(colsv[i], std::min<int64_t>(r, colsv[i]) + awide[i]),
                                          "cmsvd_merge_errors");
            if (st != CMSVD_OK) return st;
        }
    if (npairs == 0) return CMSVD_OK;
    // anchors and candidates
    std::vector<int> is_anchor(nblocks, 0), is_cand(nblocks, 0), aslot(nblocks, -1), cslot(nblocks, -1);
    for (int64_t i = 0; i < nblocks; ++i) {
        is_anchor[i] = acount[i] > 0;
        is_cand[i] = ccount[i] > 0;
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
    // Thin blocks: one GEMM per chunk of anchors against all candidates (see eval_dense),
    // when the requested pairs cover at least a quarter of the anchor x candidate grid.
    long ksum = 0;
    int kmax_c = 0;
    bool all_f32 = true;
    std::vector<long> coff(nblocks, -1);
    for (int i = 0; i < nblocks; ++i)
        if (is_cand[i]) {
            coff[i] = ksum;
            ksum += blocks[i].cols;
            kmax_c = std::max(kmax_c, (int)blocks[i].cols);
            all_f32 &= blocks[i].dtype == CMSVD_F32;
        }
    // per-pair GEMMs fill 64 x 64 tiles: with r x k outputs well below whole tiles the
    // dense form (every anchor against a range of packed candidates) does less work
    double pair_work = 0.0, tile_work = 0.0;
    for (int i = 0; i < nblocks; ++i)
        if (ccount[i]) {
            const double k = (double)colsv[i], c = (double)ccount[i];
            pair_work += c * k;
            tile_work += c * std::ceil(k / 64.0) * 64.0 * std::ceil((double)r / 64.0) * 64.0 / (double)r;
        }
    const bool dense = pair_work < 0.5 * tile_work && (double)anchors.size() * (double)ksum <= 4.0 * pair_work;
    if (dense_out) *dense_out = dense;
    // Candidates given as consecutive column ranges of one row-major matrix (in index
    // order, one dtype and row stride) already form the packed operand: used in place.
    bool in_place = dense;
    {
        const cmsvd_block* prev = nullptr;
        for (int i = 0; i < nblocks && in_place; ++i) {
            if (!is_cand[i]) continue;
            const cmsvd_block& b = blocks[i];
            if (prev) {
                const size_t esz = prev->dtype == CMSVD_F32 ? 4 : 8;
                in_place = b.dtype == prev->dtype && b.ld == prev->ld &&
                           static_cast<const char*>(b.ptr) == static_cast<const char*>(prev->ptr) + prev->cols * esz;
            }
            prev = &b;
        }
    }
    long ldball = ksum;
    const void* ball_user = nullptr;
    for (int i = 0; i < nblocks && in_place; ++i)
        if (is_cand[i]) {
            ldball = (long)blocks[i].ld;
            ball_user = blocks[i].ptr;
            break;
        }
    // persistent per-call buffers: norms + grams (all involved), anchor states
    Plan pl;
    std::vector<size_t> o_n(cands.size()), o_g(cands.size());
    const size_t o_nall = pl.add(16 * cands.size());  // norms side by side: one read-back
    for (size_t c = 0; c < cands.size(); ++c) {
        const int i = cands[c];
        o_n[c] = o_nall + 16 * c;
        // a one-column candidate's Gram is its squared norm: the leading part of the
        // double-double norm serves as the 1 x 1 Gram (no GEMM)
        o_g[c] = !is_cand[i] ? (size_t)-1 : blocks[i].cols == 1 ? o_n[c] : pl.add((size_t)blocks[i].cols * blocks[i].cols * 8);
    }
    std::vector<size_t> o_U(anchors.size()), o_S(anchors.size()), o_acc(anchors.size());
    const long ldu_a = dense ? (long)anchors.size() * r : (long)r;  // anchors side by side when dense
    const size_t o_Uall = dense ? pl.add((size_t)m * ldu_a * 8) : 0;
    const size_t o_Ball = dense && !in_place ? pl.add((size_t)m * ksum * (all_f32 ? 4 : 8)) : 0;
    const size_t o_accall = pl.add(anchors.size() * 4 * 8);  // the accumulators side by side: one fill
    for (size_t a = 0; a < anchors.size(); ++a) {
        o_U[a] = dense ? o_Uall + (size_t)a * r * 8 : pl.add((size_t)m * r * 8);
        o_S[a] = pl.add((size_t)r * 8);
        o_acc[a] = o_accall + a * 4 * 8;
    }
    // the handle's grow-on-demand buffer: its previous contents are read only by work
    // enqueued earlier on the same stream
    {
        const cmsvd_status sa = ensure(h, h->keep, h->keep_cap, pl.off);
        if (sa != CMSVD_OK) return sa;
    }
    char* const kp = h->keep;
    auto K = [&](size_t off) { return reinterpret_cast<double*>(kp + off); };
    std::vector<cmsvd_block> bl;
    std::vector<double*> nrm, gram;
    for (size_t c = 0; c < cands.size(); ++c) {
        bl.push_back(blocks[cands[c]]);
        nrm.push_back(K(o_n[c]));
        gram.push_back(o_g[c] == (size_t)-1 || o_g[c] == o_n[c] ? nullptr : K(o_g[c]));
    }
    cmsvd_status st = norms_and_grams(h, bl, nrm, gram);
    if (st != CMSVD_OK) return st;
    if (dense) {
        // Anchors side by side and candidates packed both by decreasing norm: for the
        // usual anchor-first pair lists a chunk of anchors then pairs with a suffix of
        // the packed candidates, and its GEMM covers only that column range.
        std::vector<double> nh(2 * cands.size());
        HIPCHK(hipMemcpyAsync(nh.data(), K(o_nall), 16 * cands.size(), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        std::vector<double> n2(nblocks, 0.0);
        for (size_t c = 0; c < cands.size(); ++c) n2[cands[c]] = nh[2 * c] + nh[2 * c + 1];
        auto by_norm = [&](int a, int b) { return n2[a] > n2[b] || (n2[a] == n2[b] && a < b); };
        std::stable_sort(anchors.begin(), anchors.end(), by_norm);
        for (size_t a = 0; a < anchors.size(); ++a) aslot[anchors[a]] = (int)a;
        if (!in_place) {  // (in place the candidates keep the caller's column order)
            std::vector<int> corder;
            for (int i = 0; i < nblocks; ++i)
                if (is_cand[i]) corder.push_back(i);
            std::stable_sort(corder.begin(), corder.end(), by_norm);
            long off = 0;
            for (int i : corder) {
                coff[i] = off;
                off += blocks[i].cols;
            }
        }
    }
    // anchor states: the update from the empty state (Algorithm 3, step 1); the
    // accumulators are cleared by a kernel (a capturable node)
    fill_f64(K(o_accall), (long)anchors.size() * 4, 0.0, h->stream);
    HIPCHK(hipGetLastError());
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
                jobs.push_back(CommitJob{(int)m, nullptr, (long)r, nullptr, 0, blocks[i], (int)r, K(o_U[a]), ldu_a,
                                         K(o_S[a]), K(o_acc[a]), nullptr});
                // the norm and Gram of the block, computed above for the evaluation
                jobs.back().nb_in = K(o_n[cslot[i]]);
                if (o_g[cslot[i]] != (size_t)-1 && o_g[cslot[i]] != o_n[cslot[i]]) jobs.back().G_in = K(o_g[cslot[i]]);
            }
            st = commit_batched(h, jobs);
            if (st != CMSVD_OK) return st;
        }
    }
    if (dense && !in_place) {
        // pack the candidates side by side
        std::vector<PackDesc> pd;
        for (int i = 0; i < nblocks; ++i)
            if (is_cand[i])
                pd.push_back(PackDesc{blocks[i].ptr, (int)m, (int)blocks[i].cols, (long)blocks[i].ld,
                                      blocks[i].dtype == CMSVD_F32 ? 1 : 0,
                                      kp + o_Ball + (size_t)coff[i] * (all_f32 ? 4 : 8), ksum, all_f32 ? 1 : 0});
        Stage stg;
        const size_t o_pd = stg.add(pd);
        char* db = nullptr;
        st = upload(h, stg, &db);
        if (st != CMSVD_OK) return st;
        {
            StageMark mark(h, ST_PREP);
            pack_batched(reinterpret_cast<const PackDesc*>(db + o_pd), (int)pd.size(), h->stream);
        }
        HIPCHK(hipGetLastError());
    }
    if (dense) {
        const size_t na = anchors.size();
        const int nmax = (int)r + kmax_c;
        const bool arrow = kmax_c == 1 && r <= 256;
        DenseEval de{K(o_Uall), (int)na, (int)r, (int)m, in_place ? ball_user : kp + o_Ball, all_f32, ksum, ldball};
        // chunks of anchors bound the products to about 8 GiB; with one chunk (every
        // candidate column in use) the product needs no pair record, so it runs while the
        // records are built and uploaded
        const size_t achunk = std::max<size_t>(1, ((size_t)8 << 30) / std::max<size_t>((size_t)ksum * r * 8, 1));
        DenseChunk whole{0, (int)na, 0, (size_t)npairs, 0, ksum, (int)std::min<int64_t>(npairs, h->ncu)};
        const bool early = na <= achunk;
        if (early) {
            st = dense_project(h, de, nmax, whole);
            if (st != CMSVD_OK) return st;
        }
        // anchor and candidate tables and the pair records, grouped by anchor slot
        // (counting sort, stable), written once into pinned memory
        const RecLayout lay(na, (size_t)nblocks, (size_t)npairs);
        st = ensure_rec_pin(h, lay.total);
        if (st != CMSVD_OK) return st;
        AnchorRec* arec = lay.anchors(h->rec_pin);
        for (size_t a = 0; a < na; ++a) arec[a] = AnchorRec{K(o_S[a]), K(o_n[cslot[anchors[a]]])};
        CandRec* crec = lay.cands(h->rec_pin);
        for (int i = 0; i < nblocks; ++i)
            crec[i] = is_cand[i] ? CandRec{K(o_n[cslot[i]]), K(o_g[cslot[i]]), coff[i], colsv[i]}
                                 : CandRec{nullptr, nullptr, 0, 0};
        std::vector<size_t> start(na + 1, 0);
        for (size_t a = 0; a < na; ++a) start[a + 1] = start[a] + (size_t)acount[anchors[a]];
        // thread t writes its pairs of slot s after those of the earlier ranges
        std::vector<std::vector<size_t>> tpos(nt, std::vector<size_t>(na));
        for (size_t a = 0; a < na; ++a) {
            size_t o = start[a];
            for (int t = 0; t < nt; ++t) {
                tpos[t][a] = o;
                o += (size_t)tac[t][anchors[a]];
            }
        }
        std::vector<std::vector<long>> tmin(nt, std::vector<long>(na, ksum)), tmax(nt, std::vector<long>(na, 0));
        PairRec* prec = lay.pairs(h->rec_pin);
        parallel_ranges(npairs, nt, [&](int t, int64_t lo, int64_t hi) {
            size_t* pos = tpos[t].data();
            long* mn = tmin[t].data();
            long* mx = tmax[t].data();
            for (int64_t p = lo; p < hi; ++p) {
                const int b = pairs[2 * p + 1], sl = aslot[pairs[2 * p]];
                prec[pos[sl]++] = PairRec{sl, b, (int)p};
                mn[sl] = std::min(mn[sl], coff[b]);
                mx[sl] = std::max(mx[sl], coff[b] + (long)colsv[b]);
            }
        });
        std::vector<long> smin(na, ksum), smax(na, 0);
        for (int t = 0; t < nt; ++t)
            for (size_t a = 0; a < na; ++a) {
                smin[a] = std::min(smin[a], tmin[t][a]);
                smax[a] = std::max(smax[a], tmax[t][a]);
            }
        // one upload on the side stream; the handle's stream waits for it before expanding,
        // and the side stream waits for the work already enqueued on the handle's stream
        // (earlier calls may still read the previous records)
        st = ensure(h, h->rec, h->rec_cap, lay.total);
        if (st != CMSVD_OK) return st;
        HIPCHK(hipEventRecord(h->tail_ev, h->stream));
        HIPCHK(hipStreamWaitEvent(h->side, h->tail_ev, 0));
        HIPCHK(hipMemcpyAsync(h->rec, h->rec_pin, lay.total, hipMemcpyHostToDevice, h->side));
        HIPCHK(hipEventRecord(h->rec_ev, h->side));
        h->rec_ev_armed = true;
        HIPCHK(hipStreamWaitEvent(h->stream, h->rec_ev, 0));
        const AnchorRec* dA = lay.anchors(h->rec);
        const CandRec* dC = lay.cands(h->rec);
        const PairRec* dP = lay.pairs(h->rec);
        if (early) {
            st = dense_cores(h, de, nmax, arrow, whole, dA, dC, dP, err, rel);
        } else {
            for (size_t a0 = 0; a0 < na && st == CMSVD_OK; a0 += achunk) {
                const size_t a1 = std::min(na, a0 + achunk);
                if (start[a1] == start[a0]) continue;
                DenseChunk ch{(int)a0, (int)a1, start[a0], start[a1] - start[a0], ksum, 0, 0};
                ch.nslots = (int)std::min<size_t>(ch.nj, (size_t)h->ncu);
                for (size_t a = a0; a < a1; ++a) {
                    ch.cmin = std::min(ch.cmin, smin[a]);
                    ch.cmax = std::max(ch.cmax, smax[a]);
                }
                st = dense_project(h, de, nmax, ch);
                if (st == CMSVD_OK) st = dense_cores(h, de, nmax, arrow, ch, dA, dC, dP, err, rel);
            }
        }
    } else {
        std::vector<EvalJob> ej;
        ej.reserve((size_t)npairs);
        for (int64_t p = 0; p < npairs; ++p) {
            const int i = pairs[2 * p], jb = pairs[2 * p + 1];
            const int a = aslot[i];
            ej.push_back(EvalJob{K(o_U[a]), ldu_a, K(o_S[a]), (int)r, K(o_n[cslot[i]]), blocks[jb], K(o_n[cslot[jb]]),
                                 K(o_g[cslot[jb]]), err + p, rel ? rel + p : nullptr});
        }
        st = eval_batched(h, ej, (int)m);
    }
    return st;
} catch (...) {
    return caught(__func__);
}

// FNV-1a over the arguments that fix a merge_errors launch sequence (pointers, shapes,
// the pair list, the projection precision).
static uint64_t merge_key(const cmsvd_ctx* h, const cmsvd_block* blocks, int64_t nblocks, const int32_t* pairs,
                          int64_t npairs, int64_t r, const double* err, const double* rel) {
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t n) {
        const unsigned char* c = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < n; ++i) x = (x ^ c[i]) * 1099511628211ull;
    };
    auto mix64 = [&](uint64_t v) { mix(&v, 8); };
    mix64((uint64_t)nblocks);
    mix64((uint64_t)npairs);
    mix64((uint64_t)r);
    mix64((uint64_t)(uintptr_t)err);
    mix64((uint64_t)(uintptr_t)rel);
    mix64((uint64_t)h->proj);
    for (int64_t i = 0; i < nblocks; ++i) {
        mix64((uint64_t)(uintptr_t)blocks[i].ptr);
        mix64((uint64_t)blocks[i].rows);
        mix64((uint64_t)blocks[i].cols);
        mix64((uint64_t)blocks[i].ld);
        mix64((uint64_t)blocks[i].dtype);
    }
    if (npairs > 0) mix(pairs, (size_t)npairs * 2 * sizeof(int32_t));
    return x;
}

cmsvd_status cmsvd_merge_errors(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, const int32_t* pairs,
                                int64_t npairs, int64_t r, double* err, double* rel) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_merge_errors: null handle");
    if (!h->graphs || h->timing || npairs <= 0 || !blocks || !pairs || nblocks < 1)
        return merge_errors_run(h, blocks, nblocks, pairs, npairs, r, err, rel, nullptr);
    const uint64_t key = merge_key(h, blocks, nblocks, pairs, npairs, r, err, rel);
    // a captured sequence for the same arguments, still valid: replay it
    for (size_t i = 0; i < h->graph_cache.size(); ++i) {
        if (h->graph_cache[i].key != key) continue;
        if (h->graph_cache[i].gen == h->ws_gen) {
            HIPCHK(hipGraphLaunch(h->graph_cache[i].exec, h->stream));
            h->graph_cache[i].last_use = ++h->graph_clock;
            ++h->graph_replays;
            return CMSVD_OK;
        }
        drop_graph(h, i);  // a workspace it refers to has moved
        break;
    }
    size_t seen = (size_t)-1;
    for (const auto& sk : h->graph_seen)
        if (sk.first == key) seen = sk.second;
    if (seen == (size_t)-1) {
        // first time: run eagerly (this also sizes every workspace) and remember the
        // call if its sequence can be captured
        bool dense = false;
        h->call_upload = 0;
        const cmsvd_status st = merge_errors_run(h, blocks, nblocks, pairs, npairs, r, err, rel, &dense);
        if (st == CMSVD_OK && !dense) {
            if (h->graph_seen.size() >= 16) h->graph_seen.erase(h->graph_seen.begin());
            h->graph_seen.emplace_back(key, h->call_upload);
        }
        return st;
    }
    // second time: capture the launch sequence into a graph, then launch it
    const auto t0 = std::chrono::steady_clock::now();
    cmsvd_ctx::GraphRec rec;
    rec.cap = std::max<size_t>(seen, 256);
    {
        const cmsvd_status sa = dev_alloc(h, rec.cap, &rec.dev);
        if (sa != CMSVD_OK) return sa;
    }
    if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    // The sequence is captured on the handle's capture stream (nothing captured runs)
    // and the graph is launched on the handle's stream.
    hipGraph_t graph = nullptr;
    const hipStream_t user_stream = h->stream;
    HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    h->stream = h->cap_stream;
    h->recording = &rec;
    bool dense = false;
    const uint64_t gen0 = h->ws_gen;
    const cmsvd_status st = merge_errors_run(h, blocks, nblocks, pairs, npairs, r, err, rel, &dense);
    h->recording = nullptr;
    h->stream = user_stream;
    const hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
    hipGraphExec_t exec = nullptr;
    // why a capture was given up (kept in cmsvd_last_error; the call itself succeeds)
    std::string why;
    if (st != CMSVD_OK) why = std::string("the captured call failed: ") + g_err;
    else if (ec != hipSuccess || !graph) why = std::string("hipStreamEndCapture: ") + hipGetErrorString(ec);
    else if (dense || rec.overflow || h->ws_gen != gen0) why = "the sequence differs from the recorded call";
    if (why.empty()) {
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) why = std::string("hipGraphInstantiate: ") + hipGetErrorString(ei);
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (why.empty() && !rec.host.empty()) {
        const hipError_t em = hipMemcpy(rec.dev, rec.host.data(), rec.host.size(), hipMemcpyHostToDevice);
        if (em != hipSuccess) why = std::string("hipMemcpy of the graph's tables: ") + hipGetErrorString(em);
    }
    const bool ok = why.empty();
    for (size_t i = 0; i < h->graph_seen.size(); ++i)
        if (h->graph_seen[i].first == key) {
            h->graph_seen.erase(h->graph_seen.begin() + (long)i);
            break;
        }
    if (!ok) {
        // nothing captured ran: run the call eagerly instead
        (void)hipGetLastError();
        if (exec) (void)hipGraphExecDestroy(exec);
        dev_free(h, rec.dev);
        const cmsvd_status se = merge_errors_run(h, blocks, nblocks, pairs, npairs, r, err, rel, nullptr);
        if (se == CMSVD_OK) (void)fail(CMSVD_OK, "cmsvd_merge_errors: graph capture given up (%s)", why.c_str());
        return se;
    }
    if (h->graph_cache.size() >= 4) {  // keep the four most recently used
        size_t lru = 0;
        for (size_t i = 1; i < h->graph_cache.size(); ++i)
            if (h->graph_cache[i].last_use < h->graph_cache[lru].last_use) lru = i;
        drop_graph(h, lru);
    }
    cmsvd_ctx::GraphEntry e;
    e.key = key;
    e.gen = h->ws_gen;
    e.exec = exec;
    e.dev = rec.dev;
    e.last_use = ++h->graph_clock;
    h->graph_cache.push_back(e);
    h->last_capture_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ++h->graph_captures;
    HIPCHK(hipGraphLaunch(exec, h->stream));
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_graph_stats(cmsvd_handle h, int64_t* captures, int64_t* replays, double* last_capture_ms) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_graph_stats: null handle");
    if (captures) *captures = h->graph_captures;
    if (replays) *replays = h->graph_replays;
    if (last_capture_ms) *last_capture_ms = h->last_capture_ms;
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_sym_eigvals(cmsvd_handle h, const double* A, int64_t n, int64_t lda, int64_t stride_a,
                               int64_t count, int64_t nkeep, double* lam) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_sym_eigvals: null handle");
    if (!A || !lam) return fail(CMSVD_EINVAL, "cmsvd_sym_eigvals: null pointer");
    if (n < 1 || lda < n || count < 0 || nkeep < 1 || nkeep > n) return fail(CMSVD_ESHAPE, "cmsvd_sym_eigvals: bad sizes");
    if (n > sym_eig_nmax()) return fail(CMSVD_EUNSUPPORTED, "cmsvd_sym_eigvals: n > %d", sym_eig_nmax());
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
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_sym_eigvals_noalloc(cmsvd_handle h, const double* A, int64_t n, int64_t lda, int64_t stride_a,
                                       int64_t count, int64_t nkeep, double* lam) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_sym_eigvals_noalloc: null handle");
    if (!A || !lam) return fail(CMSVD_EINVAL, "cmsvd_sym_eigvals_noalloc: null pointer");
    if (n < 1 || lda < n || count < 0 || nkeep < 1 || nkeep > n)
        return fail(CMSVD_ESHAPE, "cmsvd_sym_eigvals_noalloc: bad sizes");
    if (n > sym_eig_nmax()) return fail(CMSVD_EUNSUPPORTED, "cmsvd_sym_eigvals_noalloc: n > %d", sym_eig_nmax());
    if (count == 0) return CMSVD_OK;
    const size_t cap = (size_t)CMSVD_NOALLOC_SCRATCH_BYTES;
    if (count > (int64_t)(cap / sizeof(EigDesc)))
        return fail(CMSVD_EUNSUPPORTED, "cmsvd_sym_eigvals_noalloc: %lld problems exceed the %zu-byte scratch",
                    (long long)count, cap);
    const size_t dbytes = align256((size_t)count * sizeof(EigDesc));
    const size_t slot = sym_eig_slot_doubles((int)n) * 8;
    int64_t nslots = std::min<int64_t>(count, h->ncu);
    if (slot > 0) nslots = std::min<int64_t>(nslots, dbytes < cap ? (int64_t)((cap - dbytes) / slot) : 0);
    if (nslots < 1)
        return fail(CMSVD_EUNSUPPORTED,
                    "cmsvd_sym_eigvals_noalloc: %lld problems of order %lld exceed the %zu-byte scratch",
                    (long long)count, (long long)n, cap);
    // scratch: [descriptors][eigen kernel slots], at this device's address of the array
    EigDesc* descs = reinterpret_cast<EigDesc*>(h->scratch);
    double* gws = reinterpret_cast<double*>(h->scratch + dbytes);
    const int grid = (int)std::min<int64_t>((count + 255) / 256, 1024);
    hipLaunchKernelGGL(eigvals_descs_kernel, dim3(grid), dim3(256), 0, h->stream, descs, A, (int)n, (long)lda,
                       (long)stride_a, (long)count, (int)nkeep, lam);
    HIPCHK(hipGetLastError());
    sym_eig_batched(descs, (int)count, (int)n, 1, gws, (int)nslots, h->stream);
    HIPCHK(hipGetLastError());
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_gemm_f64(cmsvd_handle h, int32_t trans_a, int32_t trans_b, int64_t M, int64_t N, int64_t K,
                            double alpha, const void* A, int64_t lda, int32_t a_dtype, const void* B, int64_t ldb,
                            int32_t b_dtype, double beta, double* C, int64_t ldc) try {
    return gemm_entry(h, "cmsvd_gemm_f64", 0, trans_a, trans_b, M, N, K, alpha, A, lda, a_dtype, B, ldb, b_dtype,
                      beta, C, ldc);
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_gemm_bf16(cmsvd_handle h, int32_t passes, int32_t trans_a, int32_t trans_b, int64_t M, int64_t N,
                             int64_t K, double alpha, const void* A, int64_t lda, int32_t a_dtype, const void* B,
                             int64_t ldb, int32_t b_dtype, double beta, double* C, int64_t ldc) try {
    if (passes != 1 && passes != 3) return fail(CMSVD_EINVAL, "cmsvd_gemm_bf16: passes must be 1 or 3");
    return gemm_entry(h, "cmsvd_gemm_bf16", passes, trans_a, trans_b, M, N, K, alpha, A, lda, a_dtype, B, ldb, b_dtype,
                      beta, C, ldc);
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_gemm_f32(cmsvd_handle h, int32_t trans_a, int32_t trans_b, int64_t M, int64_t N, int64_t K,
                            double alpha, const void* A, int64_t lda, int32_t a_dtype, const void* B, int64_t ldb,
                            int32_t b_dtype, double beta, double* C, int64_t ldc) try {
    return gemm_entry(h, "cmsvd_gemm_f32", PREC_F32, trans_a, trans_b, M, N, K, alpha, A, lda, a_dtype, B, ldb,
                      b_dtype, beta, C, ldc);
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_cluster(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, int64_t r, double eps,
                           int32_t sort_mode, int32_t* labels, int64_t* nclusters, double* cluster_rel) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_cluster: null handle");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, blocks, nblocks, wide_, "cmsvd_cluster");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) blocks = wide_.data();
    }
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
        st = check_order(r + blocks[i].cols, "cmsvd_cluster");
        if (st != CMSVD_OK) return st;
    }
    const int N = (int)nblocks;
    // persistent buffers: norms, grams, two state slots, eval outputs, residual-mode scratch
    Plan pl;
    std::vector<size_t> o_n(N), o_g(N);
    size_t kmax = 0;
    const size_t o_nall = pl.add(16 * (size_t)N);  // norms side by side: one read-back
    for (int i = 0; i < N; ++i) {
        o_n[i] = o_nall + 16 * (size_t)i;
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
    DevBuf keep;
    {
        const cmsvd_status sa = keep.get(h, pl.off);
        if (sa != CMSVD_OK) return sa;
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
    HIPCHK(hipMemcpyAsync(n2h.data(), K(o_nall), 16 * (size_t)N, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    std::vector<double> n2(N);
    for (int i = 0; i < N; ++i) n2[i] = n2h[2 * i] + n2h[2 * i + 1];
    std::vector<int> remaining(N);
    for (int i = 0; i < N; ++i) remaining[i] = i;
    std::stable_sort(remaining.begin(), remaining.end(), [&](int a, int b) { return n2[a] > n2[b]; });
    for (int i = 0; i < N; ++i) labels[i] = -1;
    int ncl = 0;
    std::vector<double> crel;
    h->cluster_trace.clear();
    h->cluster_trace.reserve((size_t)N);
    while (!remaining.empty()) {
        const int anchor = remaining.front();
        remaining.erase(remaining.begin());
        h->cluster_trace.push_back(anchor);
        int cur = 0;
        HIPCHK(hipMemsetAsync(K(o_acc[cur]), 0, 32, h->stream));
        CommitJob aj{(int)m, nullptr, (long)r, nullptr, 0, blocks[anchor], (int)r, K(o_U[cur]), (long)r, K(o_S[cur]),
                     K(o_acc[cur]), K(o_est)};
        aj.nb_in = K(o_n[anchor]);
        cmsvd_status st = commit_batched(h, {aj});
        if (st != CMSVD_OK) return st;
        labels[anchor] = ncl;
        for (;;) {  // passes
            std::vector<int> order = remaining;
            if (sort_mode == 0) {
                std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                    return n2[a] < n2[b] || (n2[a] == n2[b] && a < b);
                });
            } else if (!order.empty()) {
                // residual norms ||A_j||^2 - ||U^T A_j||^2 against the pass-start state,
                // all remaining candidates in one grouped projection
                std::vector<double> res(N, 0.0);
                {
                    std::vector<cmsvd_block> bl;
                    std::vector<double*> outp;
                    for (const int j : order) {
                        bl.push_back(blocks[j]);
                        outp.push_back(K(o_pn) + j);
                    }
                    st = proj_sumsq(h, K(o_U[cur]), (long)r, (int)r, (int)m, bl, outp);
                    if (st != CMSVD_OK) return st;
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
            // The scan only needs the first feasible candidate: evaluate the suffix in
            // chunks (a quarter of the compute units first, doubling while nothing in
            // the chunk is feasible) instead of all of it after every acceptance.
            size_t chunk0;
            {
                std::vector<int64_t> w;
                for (const int j : order) w.push_back(blocks[j].cols);
                std::nth_element(w.begin(), w.begin() + (long)(w.size() / 2), w.end());
                chunk0 = scan_chunk(h, m, w.empty() ? 1 : w[w.size() / 2], r);
            }
            size_t chunk = chunk0;
            while (pos < order.size()) {
                const size_t end = std::min(order.size(), pos + chunk);
                std::vector<EvalJob> ej;
                for (size_t c = pos; c < end; ++c) {
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
                if (idx >= (int)ej.size()) {
                    pos = end;
                    chunk *= 2;
                    continue;
                }
                chunk = chunk0;
                const int jacc = order[pos + idx];
                const int nxt = 1 - cur;
                HIPCHK(hipMemcpyAsync(K(o_acc[nxt]), K(o_acc[cur]), 32, hipMemcpyDeviceToDevice, h->stream));
                CommitJob cj{(int)m, K(o_U[cur]), (long)r, K(o_S[cur]), (int)r, blocks[jacc], (int)r,
                             K(o_U[nxt]), (long)r, K(o_S[nxt]), K(o_acc[nxt]), K(o_est)};
                cj.nb_in = K(o_n[jacc]);
                st = commit_batched(h, {cj});
                if (st != CMSVD_OK) return st;
                cur = nxt;
                labels[jacc] = ncl;
                h->cluster_trace.push_back(jacc);
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
} catch (...) {
    return caught(__func__);
}


cmsvd_status cmsvd_autotune(cmsvd_handle h, int64_t m, int64_t k, int64_t r, const char* cache_path,
                            int32_t force, int64_t* chunk_out) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_autotune: null handle");
    if (m < 1 || k < 1 || r < 1 || r > m || k > 16384) return fail(CMSVD_ESHAPE, "cmsvd_autotune: bad shape");
    const int64_t kb = std::min<int64_t>(width_bucket(k), sym_eig_nmax() - r);
    if (kb < 1) return fail(CMSVD_EUNSUPPORTED, "cmsvd_autotune: r leaves no room for a candidate");
    const std::string key = tune_key(h, m, k, r);
    // the cache: one JSON object, one entry per line, written by this function only
    std::vector<std::string> lines;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string ln;
        while (std::getline(in, ln))
            if (ln.find("\"gfx950 ") != std::string::npos) lines.push_back(ln);
    }
    const std::string tag = "\"" + key + "\": {\"scan_chunk\": ";
    const int64_t ob = width_bucket(r + k);  // order bucket of the cores the entry serves
    if (!force)
        for (const auto& ln : lines) {
            const size_t p = ln.find(tag);
            if (p == std::string::npos) continue;
            const int c = std::atoi(ln.c_str() + p + tag.size());
            const size_t q = ln.find("\"eig_threads\": ", p);
            const int th = q == std::string::npos ? 0 : std::atoi(ln.c_str() + q + 15);
            if (c >= 1) {
                h->tuned_chunk[key] = c;
                if (th > 0) h->tuned_threads[ob] = th;
                if (chunk_out) *chunk_out = c;
                return CMSVD_OK;
            }
        }
    // Measure: a synthetic anchor state of rank r (an m x kb block committed from the
    // empty state) and c evaluations of one synthetic m x kb candidate, for c = 16 ..
    // 1024; time per launch sequence with HIP events (best of three after a warm-up).
    Plan pl;
    const size_t o_A = pl.add((size_t)m * kb * 8), o_B = pl.add((size_t)m * kb * 8), o_U = pl.add((size_t)m * r * 8),
                 o_S = pl.add((size_t)r * 8), o_acc = pl.add(32), o_nb = pl.add(16), o_G = pl.add((size_t)kb * kb * 8),
                 o_err = pl.add(1024 * 8), o_rel = pl.add(1024 * 8);
    DevBuf mem;
    {
        const cmsvd_status sa = mem.get(h, pl.off);
        if (sa != CMSVD_OK) return sa;
    }
    auto D = [&](size_t o) { return reinterpret_cast<double*>(mem.p + o); };
    fill_hash(D(o_A), (long)m * kb, 0x5eedULL, h->stream);
    fill_hash(D(o_B), (long)m * kb, 0xca11ULL, h->stream);
    fill_f64(D(o_acc), 4, 0.0, h->stream);
    HIPCHK(hipGetLastError());
    const cmsvd_block A{D(o_A), m, kb, kb, CMSVD_F64}, B{D(o_B), m, kb, kb, CMSVD_F64};
    cmsvd_status st = commit_batched(h, {CommitJob{(int)m, nullptr, (long)r, nullptr, 0, A, (int)r, D(o_U), (long)r,
                                                   D(o_S), D(o_acc), nullptr}});
    if (st != CMSVD_OK) return st;
    st = norms_and_grams(h, {B}, {D(o_nb)}, {D(o_G)});
    if (st != CMSVD_OK) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(CMSVD_EHIP, "cmsvd_autotune: hipEventCreate failed");
    }
    // orders above 320 run the general kernel: its workgroup (1024 or 512 threads per
    // problem) is measured too, each with its own best chunk
    const bool general = r + kb > 320;
    std::vector<int> variants = general ? std::vector<int>{1024, 512} : std::vector<int>{0};
    std::vector<std::pair<int, double>> ms, best_ms;
    int best_threads = 0, chunk = 16;
    double best_rate = 1e300;
    for (const int v : variants) {
    ms.clear();
    h->force_threads = v;
    for (int c = 16; c <= 1024 && st == CMSVD_OK; c *= 2) {
        std::vector<EvalJob> ej((size_t)c, EvalJob{D(o_U), (long)r, D(o_S), (int)r, D(o_acc), B, D(o_nb), D(o_G),
                                                   D(o_err), D(o_rel)});
        for (int q = 0; q < c; ++q) {
            ej[(size_t)q].err = D(o_err) + q;
            ej[(size_t)q].rel = D(o_rel) + q;
        }
        double best = 1e300;
        for (int rep = 0; rep < 4 && st == CMSVD_OK; ++rep) {
            if (hipEventRecord(e0, h->stream) != hipSuccess) st = fail(CMSVD_EHIP, "hipEventRecord failed");
            if (st == CMSVD_OK) st = eval_batched(h, ej, (int)m);
            if (st == CMSVD_OK && (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                st = fail(CMSVD_EHIP, "hipEventRecord / hipEventSynchronize failed");
            float t = 0.0f;
            if (st == CMSVD_OK && hipEventElapsedTime(&t, e0, e1) == hipSuccess && rep > 0) best = std::min(best, (double)t);
        }
        ms.emplace_back(c, best);
    }
    if (st != CMSVD_OK) break;
    // the largest chunk that costs at most 15 % more than the smallest: candidates the
    // compute units evaluate side by side for (almost) free; between workgroup sizes,
    // the one with the lower time per candidate at its own chunk
    int cv = ms.front().first;
    double tv = ms.front().second;
    for (const auto& x : ms)
        if (x.second <= 1.15 * ms.front().second) {
            cv = x.first;
            tv = x.second;
        }
    if (tv / cv < best_rate) {
        best_rate = tv / cv;
        chunk = cv;
        best_threads = v;
        best_ms = ms;
    }
    }
    h->force_threads = 0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != CMSVD_OK) return st;
    ms = best_ms;
    h->tuned_chunk[key] = chunk;
    if (best_threads > 0) h->tuned_threads[ob] = best_threads;
    if (chunk_out) *chunk_out = chunk;
    if (cache_path) {
        std::ostringstream e;
        e << "  " << tag << chunk << ", \"eig_threads\": " << best_threads << ", \"ms\": [";
        for (size_t q = 0; q < ms.size(); ++q)
            e << (q ? ", " : "") << "[" << ms[q].first << ", " << ms[q].second << "]";
        e << "]}";
        std::vector<std::string> keep;
        for (const auto& ln : lines)
            if (ln.find(tag) == std::string::npos) keep.push_back(ln);
        keep.push_back(e.str());
        std::ofstream out(cache_path, std::ios::trunc);
        if (!out) return fail(CMSVD_EINVAL, "cmsvd_autotune: cannot write %s", cache_path);
        out << "{\n";
        for (size_t q = 0; q < keep.size(); ++q) {
            std::string ln = keep[q];
            while (!ln.empty() && (ln.back() == ',' || ln.back() == ' ')) ln.pop_back();
            out << ln << (q + 1 < keep.size() ? ",\n" : "\n");
        }
        out << "}\n";
    }
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_cluster_trace(cmsvd_handle h, int32_t* order, int64_t cap, int64_t* n) try {
    if (!h || !n) return fail(CMSVD_EINVAL, "cmsvd_cluster_trace: null handle or count");
    *n = (int64_t)h->cluster_trace.size();
    if (cap < *n) {
        if (order) return fail(CMSVD_ESHAPE, "cmsvd_cluster_trace: %lld entries do not fit in %lld", (long long)*n,
                               (long long)cap);
        return CMSVD_OK;  // size query
    }
    if (!order && *n > 0) return fail(CMSVD_EINVAL, "cmsvd_cluster_trace: null order");
    std::copy(h->cluster_trace.begin(), h->cluster_trace.end(), order);
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

/* Residual-certified clustering (Algorithm 2); see include/cmsvd.h. */

cmsvd_status cmsvd_cluster_residual(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, int64_t r, double eps,
                                    int32_t sort_mode, int32_t* labels, int64_t* nclusters, double* cluster_rel) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_cluster_residual: null handle");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, blocks, nblocks, wide_, "cmsvd_cluster_residual");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) blocks = wide_.data();
    }
    if (!labels || !nclusters) return fail(CMSVD_EINVAL, "cmsvd_cluster_residual: null output");
    if (!(eps >= 0.0)) return fail(CMSVD_EINVAL, "cmsvd_cluster_residual: eps must be >= 0");
    if (sort_mode != 0 && sort_mode != 1) return fail(CMSVD_EINVAL, "cmsvd_cluster_residual: sort_mode must be 0 or 1");
    if (nblocks > INT32_MAX) return fail(CMSVD_EUNSUPPORTED, "cmsvd_cluster_residual: too many blocks");
    const int N = (int)nblocks;
    ResidBuffers rb;
    cmsvd_status st = resid_setup(h, blocks, N, r, "cmsvd_cluster_residual", rb);
    if (st != CMSVD_OK) return st;
    std::vector<double> n2h(2 * (size_t)N);  // the norms are contiguous (resid_setup)
    HIPCHK(hipMemcpyAsync(n2h.data(), rb.nrm[0], 16 * (size_t)N, hipMemcpyDeviceToHost, h->stream));
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
        st = resid_reset(h, rb.st);
        if (st != CMSVD_OK) return st;
        st = resid_accept_block(h, rb.st, blocks[anchor], rb.nrm[anchor], rb.own + (size_t)anchor * rb.nkcap,
                                (int)std::min<int64_t>(r, blocks[anchor].cols));
        if (st != CMSVD_OK) return st;
        labels[anchor] = ncl;
        for (;;) {  // passes
            std::vector<int> order = remaining;
            if (sort_mode == 0) {
                std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                    return n2[a] < n2[b] || (n2[a] == n2[b] && a < b);
                });
            } else if (!order.empty()) {
                std::vector<cmsvd_block> bl;
                std::vector<double*> out;
                for (size_t c = 0; c < order.size(); ++c) {
                    bl.push_back(blocks[order[c]]);
                    out.push_back(rb.pn + c);
                }
                st = resid_proj_norms(h, rb.st, bl, out);
                if (st != CMSVD_OK) return st;
                std::vector<double> pn(order.size());
                HIPCHK(hipMemcpyAsync(pn.data(), rb.pn, order.size() * 8, hipMemcpyDeviceToHost, h->stream));
                HIPCHK(hipStreamSynchronize(h->stream));
                std::vector<double> res(N, 0.0);
                for (size_t c = 0; c < order.size(); ++c) res[order[c]] = n2[order[c]] - pn[c];
                std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                    return res[a] < res[b] || (res[a] == res[b] && a < b);
                });
            }
            bool accepted_any = false;
            size_t pos = 0;
            while (pos < order.size()) {
                const std::vector<int> cand(order.begin() + pos, order.end());
                int idx = 0;
                st = resid_scan(h, rb, blocks, cand, eps, &idx);
                if (st != CMSVD_OK) return st;
                if (idx >= (int)cand.size()) break;
                const int jacc = cand[idx];
                st = resid_accept_block(h, rb.st, blocks[jacc], rb.nrm[jacc], rb.lam + (size_t)idx * rb.nkcap,
                                        (int)std::min<int64_t>(r, blocks[jacc].cols));
                if (st != CMSVD_OK) return st;
                labels[jacc] = ncl;
                remaining.erase(std::find(remaining.begin(), remaining.end(), jacc));
                accepted_any = true;
                pos = pos + idx + 1;
            }
            if (!accepted_any) break;
        }
        double rel = 0.0;
        st = resid_state_rel(h, rb, &rel, nullptr);
        if (st != CMSVD_OK) return st;
        crel.push_back(rel);
        ++ncl;
    }
    *nclusters = ncl;
    if (cluster_rel)
        for (int c = 0; c < ncl; ++c) cluster_rel[c] = crel[c];
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_residual_bound(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, int64_t r,
                                  double* bound2, double* mu) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_residual_bound: null handle");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, blocks, nblocks, wide_, "cmsvd_residual_bound");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) blocks = wide_.data();
    }
    if (!bound2) return fail(CMSVD_EINVAL, "cmsvd_residual_bound: null output");
    if (nblocks > INT32_MAX) return fail(CMSVD_EUNSUPPORTED, "cmsvd_residual_bound: too many blocks");
    const int N = (int)nblocks;
    ResidBuffers rb;
    cmsvd_status st = resid_setup(h, blocks, N, r, "cmsvd_residual_bound", rb);
    if (st != CMSVD_OK) return st;
    st = resid_reset(h, rb.st);
    if (st != CMSVD_OK) return st;
    for (int j = 0; j < N; ++j) {
        st = resid_test(h, rb, blocks, {j});
        if (st != CMSVD_OK) return st;
        st = resid_accept_block(h, rb.st, blocks[j], rb.nrm[j], rb.lam, (int)std::min<int64_t>(r, blocks[j].cols));
        if (st != CMSVD_OK) return st;
    }
    st = resid_state_rel(h, rb, nullptr, bound2);
    if (st != CMSVD_OK) return st;
    if (mu) {
        std::vector<double> L((size_t)r);
        HIPCHK(hipMemcpyAsync(L.data(), rb.st.L[rb.st.cur], (size_t)r * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int64_t i = 0; i < r; ++i) mu[i] = std::sqrt(std::max(L[(size_t)i], 0.0));
    }
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}


/* Theorem 1, Algorithm 1 and the explicit tail; see include/cmsvd.h. */
cmsvd_status cmsvd_weyl_bound(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, int64_t r, double* bound2) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_weyl_bound: null handle");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, blocks, nblocks, wide_, "cmsvd_weyl_bound");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) blocks = wide_.data();
    }
    if (!bound2) return fail(CMSVD_EINVAL, "cmsvd_weyl_bound: null output");
    if (nblocks > INT32_MAX) return fail(CMSVD_EUNSUPPORTED, "cmsvd_weyl_bound: too many blocks");
    WeylBuffers wb;
    cmsvd_status st = weyl_setup(h, blocks, (int)nblocks, r, "cmsvd_weyl_bound", wb);
    if (st != CMSVD_OK) return st;
    weyl_bound(wb.a2, wb.h, (int)nblocks, wb.rel, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(bound2, wb.rel, 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_cluster_weyl(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, int64_t r, double eps,
                                int32_t* labels, int64_t* nclusters, double* cluster_rel) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_cluster_weyl: null handle");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, blocks, nblocks, wide_, "cmsvd_cluster_weyl");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) blocks = wide_.data();
    }
    if (!labels || !nclusters) return fail(CMSVD_EINVAL, "cmsvd_cluster_weyl: null output");
    if (!(eps >= 0.0)) return fail(CMSVD_EINVAL, "cmsvd_cluster_weyl: eps must be >= 0");
    if (nblocks > INT32_MAX) return fail(CMSVD_EUNSUPPORTED, "cmsvd_cluster_weyl: too many blocks");
    const int N = (int)nblocks;
    WeylBuffers wb;
    cmsvd_status st = weyl_setup(h, blocks, N, r, "cmsvd_cluster_weyl", wb);
    if (st != CMSVD_OK) return st;
    std::vector<double> a2h(2 * (size_t)N);
    HIPCHK(hipMemcpyAsync(a2h.data(), wb.a2, (size_t)N * 16, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    std::vector<double> n2(N);
    for (int i = 0; i < N; ++i) n2[i] = a2h[2 * i] + a2h[2 * i + 1];
    std::vector<int> remaining(N);
    for (int i = 0; i < N; ++i) remaining[i] = i;
    std::stable_sort(remaining.begin(), remaining.end(), [&](int a, int b) { return n2[a] > n2[b]; });
    for (int i = 0; i < N; ++i) labels[i] = -1;
    int ncl = 0;
    std::vector<double> crel;
    while (!remaining.empty()) {
        const int anchor = remaining.front();
        remaining.erase(remaining.begin());
        labels[anchor] = ncl;
        int init = anchor, acc = -1;
        for (;;) {  // passes
            std::vector<int> order = remaining;
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                return n2[a] < n2[b] || (n2[a] == n2[b] && a < b);
            });
            if (order.empty()) break;
            Stage stg;
            const size_t o_c = stg.add(order);
            char* db = nullptr;
            st = upload(h, stg, &db);
            if (st != CMSVD_OK) return st;
            const int* cand = reinterpret_cast<const int*>(db + o_c);
            bool accepted_any = false;
            size_t pos = 0;
            while (pos < order.size()) {
                const int cnt = (int)(order.size() - pos);
                weyl_step(cand + pos, cnt, init, acc, wb.a2, wb.h, wb.state, eps, wb.first, wb.rel, h->stream);
                HIPCHK(hipGetLastError());
                init = acc = -1;
                int idx = 0;
                HIPCHK(hipMemcpyAsync(&idx, wb.first, sizeof(int), hipMemcpyDeviceToHost, h->stream));
                HIPCHK(hipStreamSynchronize(h->stream));
                if (idx >= cnt) break;
                const int j = order[pos + idx];
                labels[j] = ncl;
                remaining.erase(std::find(remaining.begin(), remaining.end(), j));
                acc = j;
                accepted_any = true;
                pos += idx + 1;
            }
            if (!accepted_any) break;
        }
        // apply a pending state change and read the cluster's ratio
        weyl_step(wb.first /* unused with count 0 */, 0, init, acc, wb.a2, wb.h, wb.state, eps, wb.first, wb.rel,
                  h->stream);
        HIPCHK(hipGetLastError());
        double rel = 0.0;
        HIPCHK(hipMemcpyAsync(&rel, wb.rel, 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        crel.push_back(rel);
        ++ncl;
    }
    *nclusters = ncl;
    if (cluster_rel)
        for (int c = 0; c < ncl; ++c) cluster_rel[c] = crel[c];
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_exact_tail(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, int64_t r, double* tail2) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_exact_tail: null handle");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, blocks, nblocks, wide_, "cmsvd_exact_tail");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) blocks = wide_.data();
    }
    if (!tail2) return fail(CMSVD_EINVAL, "cmsvd_exact_tail: null output");
    if (nblocks < 1 || !blocks) return fail(CMSVD_EINVAL, "cmsvd_exact_tail: no blocks");
    if (nblocks > INT32_MAX) return fail(CMSVD_EUNSUPPORTED, "cmsvd_exact_tail: too many blocks");
    const int N = (int)nblocks;
    const int64_t m = blocks[0].rows;
    if (m < 1 || r < 1) return fail(CMSVD_ESHAPE, "cmsvd_exact_tail: need m >= 1 and r >= 1");
    int64_t ksum = 0;
    for (int i = 0; i < N; ++i) {
        cmsvd_status s = check_block(blocks[i], m, "block", i);
        if (s != CMSVD_OK) return s;
        ksum += blocks[i].cols;
    }
    const int64_t n = std::min(m, ksum);
    cmsvd_status so = check_order(n, "cmsvd_exact_tail");
    if (so != CMSVD_OK) return so;
    const int nk = (int)std::min<int64_t>(r, n);
    Plan pl;
    const size_t o_M = pl.add((size_t)m * ksum * 8), o_G = pl.add((size_t)n * n * 8), o_a2 = pl.add((size_t)N * 16),
                 o_top = pl.add(16), o_lam = pl.add((size_t)nk * 8), o_out = pl.add(8),
                 o_eig = pl.add(sym_eig_workspace_doubles((int)n, 1) * 8);
    cmsvd_status st = ensure(h, h->ws, h->ws_cap, pl.off);
    if (st != CMSVD_OK) return st;
    auto D = [&](size_t off) { return reinterpret_cast<double*>(h->ws + off); };
    std::vector<PackDesc> pk;
    std::vector<NormDesc> nd;
    long coff = 0;
    for (int i = 0; i < N; ++i) {
        const cmsvd_block& b = blocks[i];
        const bool f32 = b.dtype == CMSVD_F32;
        pk.push_back(PackDesc{b.ptr, (int)m, (int)b.cols, (long)b.ld, f32 ? 1 : 0, D(o_M) + coff, (long)ksum, 0});
        nd.push_back(NormDesc{b.ptr, (int)m, (int)b.cols, (long)b.ld, f32 ? 1 : 0, D(o_a2) + 2 * i});
        coff += b.cols;
    }
    GemmGroup g;
    if (ksum <= m) {  // M^T M
        g.tb = true;
        g.push(GemmDesc{D(o_M), D(o_M), D(o_G), (int)ksum, (int)ksum, (int)m, (long)ksum, (long)ksum, (long)ksum});
    } else {  // M M^T
        g.ta = true;
        g.push(GemmDesc{D(o_M), D(o_M), D(o_G), (int)m, (int)m, (int)ksum, (long)ksum, (long)ksum, (long)m});
    }
    EigDesc e{};
    e.n = (int)n;
    e.n1 = 0;
    e.nkeep = nk;
    e.Y = D(o_G);
    e.ldy = (long)n;
    e.lam = D(o_lam);
    e.sum_top = D(o_top);
    std::vector<EigDesc> ed{e};
    Stage stg;
    const size_t o_pk = stg.add(pk), o_nd = stg.add(nd), o_ed = stg.add(ed);
    g.off = stg.add(g.d);
    char* db = nullptr;
    st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    pack_batched(reinterpret_cast<const PackDesc*>(db + o_pk), N, h->stream);
    sumsq_batched(reinterpret_cast<const NormDesc*>(db + o_nd), N, h->stream);
    run_gemm(h, g, db);
    sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), 1, (int)n, 1, D(o_eig), 1, h->stream);
    energy_minus(D(o_a2), N, D(o_top), D(o_out), h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(tail2, D(o_out), 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}


/* Compression back-end: the truncated SVD factors of one cluster; see include/cmsvd.h. */
cmsvd_status cmsvd_compress(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, int64_t r, double* Ut,
                            int64_t ldu, double* Vt, int64_t ldv, int64_t* rank, double* tail2, double* energy) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_compress: null handle");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, blocks, nblocks, wide_, "cmsvd_compress");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) blocks = wide_.data();
    }
    if (!Ut || !Vt || !rank || !tail2) return fail(CMSVD_EINVAL, "cmsvd_compress: null output");
    if (nblocks < 1 || !blocks) return fail(CMSVD_EINVAL, "cmsvd_compress: no blocks");
    if (nblocks > INT32_MAX) return fail(CMSVD_EUNSUPPORTED, "cmsvd_compress: too many blocks");
    const int N = (int)nblocks;
    const int64_t m = blocks[0].rows;
    if (m < 1 || r < 1) return fail(CMSVD_ESHAPE, "cmsvd_compress: need m >= 1 and r >= 1");
    int64_t ncol = 0;
    for (int i = 0; i < N; ++i) {
        cmsvd_status s = check_block(blocks[i], m, "block", i);
        if (s != CMSVD_OK) return s;
        ncol += blocks[i].cols;
    }
    const int64_t n = std::min(m, ncol);
    if (ncol > INT32_MAX / 2 || m > INT32_MAX / 2 || (double)n * (double)n > 4e9)
        return fail(CMSVD_EUNSUPPORTED, "cmsvd_compress: too large");
    const int rc = (int)std::min<int64_t>(r, n);
    if (rc > sym_eig_nmax()) return fail(CMSVD_EUNSUPPORTED, "cmsvd_compress: rank %d exceeds %d", rc, sym_eig_nmax());
    if (ldu < rc || ldv < ncol) return fail(CMSVD_ESHAPE, "cmsvd_compress: ldu < rank or ldv < total columns");
    const bool cols_side = ncol <= m;  // Gram M^T M (else M M^T)
    // Above the eigen kernels' order the top eigenpairs of the Gram come from subspace
    // iteration with Rayleigh-Ritz on p columns (the Ritz problem has order p).
    const bool large = n > sym_eig_nmax();
    const int p = large ? (int)std::min<int64_t>({n, (int64_t)sym_eig_nmax(), std::max<int64_t>(2 * rc, rc + 32)})
                        : (int)n;
    const int ne = p;  // order of the eigenproblem solved
    Plan pl;
    const size_t o_M = pl.add((size_t)m * ncol * 8), o_G = pl.add((size_t)n * n * 8), o_a2 = pl.add((size_t)N * 16),
                 o_top = pl.add(16), o_lam = pl.add((size_t)rc * 8), o_d = pl.add((size_t)ne * 8),
                 o_e = pl.add((size_t)ne * 8), o_V = pl.add((size_t)ne * ne * 8), o_tau = pl.add((size_t)ne * 8),
                 o_vs = pl.add((size_t)6 * ne * rc * 8), o_Z = pl.add(cols_side ? 8 : (size_t)n * rc * 8),
                 o_out = pl.add(16), o_zero = pl.add(16), o_eig = pl.add(sym_eig_workspace_doubles(ne, 1) * 8),
                 o_bs = pl.add(BackPlan::scratch_doubles(ne, rc) * 8);
    size_t o_X = 0, o_Y = 0, o_X1 = 0, o_G1 = 0, o_G2 = 0, o_L1 = 0, o_L2 = 0, o_Zt = 0, o_yn = 0, o_cs = 0;
    if (large) {
        o_X = pl.add((size_t)n * p * 8);
        o_Y = pl.add((size_t)n * p * 8);
        o_X1 = pl.add((size_t)n * p * 8);
        o_G1 = pl.add((size_t)p * p * 8);
        o_G2 = pl.add((size_t)p * p * 8);
        o_L1 = pl.add((size_t)p * p * 8);
        o_L2 = pl.add((size_t)p * p * 8);
        o_Zt = pl.add((size_t)p * rc * 8);
        o_yn = pl.add(16);
        o_cs = pl.add(CholPlan::scratch_doubles(p) * 8);
    }
    cmsvd_status st = ensure(h, h->ws, h->ws_cap, pl.off);
    if (st != CMSVD_OK) return st;
    auto D = [&](size_t off) { return reinterpret_cast<double*>(h->ws + off); };
    std::vector<PackDesc> pk;
    std::vector<NormDesc> nd;
    long coff = 0;
    for (int i = 0; i < N; ++i) {
        const cmsvd_block& b = blocks[i];
        const bool f32 = b.dtype == CMSVD_F32;
        pk.push_back(PackDesc{b.ptr, (int)m, (int)b.cols, (long)b.ld, f32 ? 1 : 0, D(o_M) + coff, (long)ncol, 0});
        nd.push_back(NormDesc{b.ptr, (int)m, (int)b.cols, (long)b.ld, f32 ? 1 : 0, D(o_a2) + 2 * i});
        coff += b.cols;
    }
    GemmGroup gG, gV, gU;
    if (cols_side) {
        gG.tb = true;
        gG.push(GemmDesc{D(o_M), D(o_M), D(o_G), (int)ncol, (int)ncol, (int)m, (long)ncol, (long)ncol, (long)ncol});
    } else {
        gG.ta = true;
        gG.push(GemmDesc{D(o_M), D(o_M), D(o_G), (int)m, (int)m, (int)ncol, (long)ncol, (long)ncol, (long)m});
        // V (ncol x rc, column-major, ld ldv) = M^T Z
        gV.push(GemmDesc{D(o_M), D(o_Z), Vt, (int)ncol, rc, (int)m, (long)ncol, (long)m, (long)ldv});
    }
    // U S (rc x m column-major = m x rc row-major) = V^T M^T
    gU.ta = true;
    gU.push(GemmDesc{Vt, D(o_M), Ut, rc, (int)m, (int)ncol, (long)ldv, (long)ncol, (long)ldu});
    double* Z = cols_side ? Vt : D(o_Z);
    const long ldz = cols_side ? (long)ldv : (long)n;
    // the eigenproblem: the Gram itself, or the Ritz matrix T = X^T G X of the subspace
    double* Zeig = large ? D(o_Zt) : Z;
    const long ldze = large ? (long)p : ldz;
    EigDesc e{};
    e.n = ne;
    e.n1 = 0;
    e.nkeep = rc;
    e.Y = large ? D(o_G2) : D(o_G);  // T lives in the G2 buffer between orthonormalisations
    e.ldy = (long)ne;
    e.lam = D(o_lam);
    e.d = D(o_d);
    e.e = D(o_e);
    e.V = D(o_V);
    e.ldv = (long)ne;
    e.tau = D(o_tau);
    e.sum_top = D(o_top);
    std::vector<EigDesc> ed{e};
    std::vector<VecDesc> vd{VecDesc{ne, rc, D(o_lam), D(o_d), D(o_e), D(o_V), (long)ne, D(o_tau), Zeig, ldze, D(o_vs)}};
    BackPlan bp;
    bp.build(vd, {D(o_bs)});
    // subspace iteration on Xt (p x n column-major: the columns of X as rows):
    //   Yt = Xt G;  T = Xt Yt^T;  Xt = CholQR2(Yt) = L2^-1 L1^-1 Yt.
    GemmGroup gY, gT, gG1, gQ1, gG2, gQ2, gZ;
    CholPlan cp1, cp2;
    std::vector<NormDesc> yn;
    if (large) {
        gY.push(GemmDesc{D(o_X), D(o_G), D(o_Y), p, (int)n, (int)n, (long)p, (long)n, (long)p});
        gT.tb = true;
        gT.push(GemmDesc{D(o_X), D(o_Y), D(o_G2), p, p, (int)n, (long)p, (long)p, (long)p});
        gG1.tb = true;
        gG1.push(GemmDesc{D(o_Y), D(o_Y), D(o_G1), p, p, (int)n, (long)p, (long)p, (long)p});
        gQ1.push(GemmDesc{D(o_L1), D(o_Y), D(o_X1), p, (int)n, p, (long)p, (long)p, (long)p});
        gG2.tb = true;
        gG2.push(GemmDesc{D(o_X1), D(o_X1), D(o_G2), p, p, (int)n, (long)p, (long)p, (long)p});
        gQ2.push(GemmDesc{D(o_L2), D(o_X1), D(o_X), p, (int)n, p, (long)p, (long)p, (long)p});
        // Z (n x rc) = X Zt
        gZ.ta = true;
        gZ.push(GemmDesc{D(o_X), Zeig, Z, (int)n, rc, p, (long)p, (long)p, ldz});
        // pivot thresholds: u ||Y||_F^2 for the first Gram, p^2 u for the nearly orthonormal second
        cp1.build({CholDesc{p, D(o_G1), (long)p, D(o_L1), (long)p, EPS, D(o_yn), nullptr}}, {D(o_cs)});
        cp2.build({CholDesc{p, D(o_G2), (long)p, D(o_L2), (long)p, (double)p * p * EPS, nullptr, nullptr}}, {D(o_cs)});
        yn.push_back(NormDesc{D(o_Y), (int)n, p, (long)p, 0, D(o_yn)});
    }
    Stage stg;
    const size_t o_pk = stg.add(pk), o_nd = stg.add(nd), o_ed = stg.add(ed);
    const size_t o_yd = large ? stg.add(yn) : 0;
    bp.stage(stg);
    if (large) {
        cp1.stage(stg);
        cp2.stage(stg);
    }
    for (GemmGroup* g : {&gG, &gV, &gU, &gY, &gT, &gG1, &gQ1, &gG2, &gQ2, &gZ}) g->off = stg.add(g->d);
    char* db = nullptr;
    st = upload(h, stg, &db);
    if (st != CMSVD_OK) return st;
    hipStream_t s = h->stream;
    pack_batched(reinterpret_cast<const PackDesc*>(db + o_pk), N, s);
    sumsq_batched(reinterpret_cast<const NormDesc*>(db + o_nd), N, s);
    run_gemm(h, gG, db);
    if (!large) {
        sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), 1, ne, 1, D(o_eig), 1, s);
        bp.run(h, db);
    } else {
        auto orth = [&]() {  // Xt = CholQR2(Yt)
            sumsq_batched(reinterpret_cast<const NormDesc*>(db + o_yd), 1, s);
            run_gemm(h, gG1, db);
            cp1.run(h, db);
            run_gemm(h, gQ1, db);
            run_gemm(h, gG2, db);
            cp2.run(h, db);
            run_gemm(h, gQ2, db);
        };
        fill_hash(D(o_Y), (long)n * p, 0x5EEDull, s);
        orth();
        double prev = -1.0;
        for (int it = 0; it < 60; ++it) {
            run_gemm(h, gY, db);
            run_gemm(h, gT, db);
            sym_eig_batched(reinterpret_cast<const EigDesc*>(db + o_ed), 1, ne, 1, D(o_eig), 1, s);
            double top[2] = {0.0, 0.0};
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(top, D(o_top), 16, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            const double sum = top[0] + top[1];
            if (!(sum == sum)) break;  // NaN data: the outputs carry it
            if (it > 0 && std::fabs(sum - prev) <= 1e-14 * std::fabs(sum)) break;
            prev = sum;
            orth();
        }
        bp.run(h, db);  // Ritz vectors of the last T: Zt
        run_gemm(h, gZ, db);
    }
    // directions below the Gram's resolution (8 n u lam_1) are stored as zero columns
    const double cut_rel = 8.0 * (double)n * EPS;
    if (cols_side) {
        scale_cols(Vt, (int)ncol, rc, (long)ldv, D(o_lam), 0, cut_rel, s);
    } else {
        run_gemm(h, gV, db);
        scale_cols(Vt, (int)ncol, rc, (long)ldv, D(o_lam), 1, cut_rel, s);
    }
    run_gemm(h, gU, db);
    energy_minus(D(o_a2), N, D(o_top), D(o_out), s);
    fill_f64(D(o_zero), 2, 0.0, s);
    energy_minus(D(o_a2), N, D(o_zero), D(o_out) + 1, s);  // ||M_C||_F^2
    HIPCHK(hipGetLastError());
    double v[2] = {0.0, 0.0};
    HIPCHK(hipMemcpyAsync(v, D(o_out), 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *tail2 = v[0];
    if (energy) *energy = v[1];
    *rank = rc;
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}


/* Tail energy of a chain and its gradient; see include/cmsvd.h. */
cmsvd_status cmsvd_compress_partition(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks,
                                      const int32_t* labels, int64_t r, double* const* Ut, const int64_t* ldu,
                                      double* const* Vt, const int64_t* ldv, int64_t* ranks, double* tail2,
                                      double* energy, int64_t* nclusters, double* ratio, double* rel_error) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_compress_partition: null handle");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, blocks, nblocks, wide_, "cmsvd_compress_partition");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) blocks = wide_.data();
    }
    if (nblocks < 1 || !blocks || !labels) return fail(CMSVD_EINVAL, "cmsvd_compress_partition: no blocks or labels");
    if (!nclusters || !ratio || !rel_error) return fail(CMSVD_EINVAL, "cmsvd_compress_partition: null output");
    if (nblocks > INT32_MAX) return fail(CMSVD_EUNSUPPORTED, "cmsvd_compress_partition: too many blocks");
    if ((Ut == nullptr) != (Vt == nullptr) || (Ut && (!ldu || !ldv)))
        return fail(CMSVD_EINVAL, "cmsvd_compress_partition: give Ut, ldu, Vt and ldv together or none");
    if (r < 1) return fail(CMSVD_ESHAPE, "cmsvd_compress_partition: r < 1");
    const int64_t m = blocks[0].rows;
    int32_t kmax = -1;
    for (int64_t i = 0; i < nblocks; ++i) {
        cmsvd_status s = check_block(blocks[i], m, "block", i);
        if (s != CMSVD_OK) return s;
        if (labels[i] < 0 || labels[i] >= nblocks)
            return fail(CMSVD_EINVAL, "cmsvd_compress_partition: label %d of block %lld out of range", labels[i],
                        (long long)i);
        kmax = std::max(kmax, labels[i]);
    }
    const int K = kmax + 1;
    std::vector<std::vector<cmsvd_block>> members((size_t)K);
    for (int64_t i = 0; i < nblocks; ++i) members[(size_t)labels[i]].push_back(blocks[i]);
    for (int c = 0; c < K; ++c)
        if (members[(size_t)c].empty())
            return fail(CMSVD_EINVAL, "cmsvd_compress_partition: cluster %d has no block (ids must be 0..K-1)", c);
    // Without caller buffers the factors go to one scratch buffer sized for the largest
    // cluster, reused cluster after cluster (each cmsvd_compress call is synchronous).
    DevBuf tmp;
    if (!Ut) {
        size_t need = 0;
        for (const auto& mem : members) {
            int64_t N = 0;
            for (const auto& b : mem) N += b.cols;
            const int64_t rc = std::min<int64_t>({r, m, N});
            need = std::max(need, (size_t)(rc * m + rc * N) * 8);
        }
        const cmsvd_status sa = tmp.get(h, need);
        if (sa != CMSVD_OK) return sa;
    }
    double before = 0.0, after = 0.0, tails = 0.0, total = 0.0;
    for (int c = 0; c < K; ++c) {
        const auto& mem = members[(size_t)c];
        int64_t N = 0;
        for (const auto& b : mem) N += b.cols;
        const int64_t rc = std::min<int64_t>({r, m, N});
        double* u = Ut ? Ut[c] : reinterpret_cast<double*>(tmp.p);
        double* v = Ut ? Vt[c] : reinterpret_cast<double*>(tmp.p) + (size_t)rc * m;
        const int64_t lu = Ut ? ldu[c] : rc, lv = Ut ? ldv[c] : N;
        int64_t rank = 0;
        double t2 = 0.0, e2 = 0.0;
        const cmsvd_status st = cmsvd_compress(h, mem.data(), (int64_t)mem.size(), r, u, lu, v, lv, &rank, &t2, &e2);
        if (st != CMSVD_OK) return st;
        if (ranks) ranks[c] = rank;
        if (tail2) tail2[c] = t2;
        if (energy) energy[c] = e2;
        before += (double)m * (double)N;
        after += (double)rank * (double)(m + N);
        tails += t2;
        total += e2;
    }
    *nclusters = K;
    *ratio = after > 0.0 ? before / after : 0.0;
    *rel_error = total > 0.0 ? std::sqrt(tails / total) : 0.0;
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

cmsvd_status cmsvd_tail_energy_grad(cmsvd_handle h, const cmsvd_block* blocks, int64_t nblocks, int64_t r,
                                    int64_t checkpoint, double* f, double* const* grads, double* min_gap) try {
    if (!h) return fail(CMSVD_EINVAL, "cmsvd_tail_energy_grad: null handle");
    std::vector<cmsvd_block> wide_;
    {
        const cmsvd_status sw = widen_blocks(h, blocks, nblocks, wide_, "cmsvd_tail_energy_grad");
        if (sw != CMSVD_OK) return sw;
        if (!wide_.empty()) blocks = wide_.data();
    }
    if (!blocks || nblocks < 1) return fail(CMSVD_EINVAL, "cmsvd_tail_energy_grad: no blocks");
    if (!f) return fail(CMSVD_EINVAL, "cmsvd_tail_energy_grad: null f");
    if (checkpoint < 1) return fail(CMSVD_EINVAL, "cmsvd_tail_energy_grad: checkpoint must be >= 1");
    const int64_t m = blocks[0].rows;
    if (r < 1 || r > m) return fail(CMSVD_ESHAPE, "cmsvd_tail_energy_grad: need 1 <= r <= m");
    if (r > 4096) return fail(CMSVD_EUNSUPPORTED, "cmsvd_tail_energy_grad: r > 4096");
    int kmax = 0;
    for (int64_t i = 0; i < nblocks; ++i) {
        cmsvd_status st = check_block(blocks[i], m, "block", i);
        if (st != CMSVD_OK) return st;
        st = check_order(r + blocks[i].cols, "cmsvd_tail_energy_grad");
        if (st != CMSVD_OK) return st;
        if (grads && !grads[i]) return fail(CMSVD_EINVAL, "cmsvd_tail_energy_grad: null gradient %lld", (long long)i);
        kmax = std::max(kmax, (int)blocks[i].cols);
    }
    const int T = (int)nblocks, R = (int)r, M = (int)m;
    const int ck = (int)std::min<int64_t>(checkpoint, T);
    const int ncmax = R + kmax;
    // one state: U (m x r row-major) | S (r) | acc (4) | est (2) | pad (2)
    const size_t SD = (size_t)M * R + R + 8;
    const int nck = T / ck + 2;  // states at t = 0, ck, 2ck, ... and the final one
    const size_t n_doubles = SD * (size_t)(nck + ck + 1)           // checkpoints + one segment
                             + 2 * (size_t)R * R + 2 * (size_t)R * M  // C and Z of two consecutive steps
                             + 2 * (size_t)R * R + (size_t)R * M      // M, N, X^T
                             + (size_t)ncmax * R + (size_t)R * ncmax  // G, B_d
                             + 2 * (size_t)R * kmax                   // Y, V
                             + (size_t)ncmax * ncmax + ncmax          // core eigenvectors and eigenvalues
                             + (size_t)kmax * M + T + 8               // residual basis, gaps, scratch acc
                             + (size_t)R * M;                         // U_{t+1} across a segment boundary
    DevBuf mem;
    {
        const cmsvd_status sa = mem.get(h, n_doubles * 8);
        if (sa != CMSVD_OK) return sa;
    }
    double* base = reinterpret_cast<double*>(mem.p);
    double* ckp = base;
    double* seg = ckp + SD * nck;
    double* Cb[2] = {seg + SD * (ck + 1), nullptr};
    Cb[1] = Cb[0] + (size_t)R * R;
    double* Zb[2] = {Cb[1] + (size_t)R * R, nullptr};
    Zb[1] = Zb[0] + (size_t)R * M;
    double* Mm = Zb[1] + (size_t)R * M;
    double* Nm = Mm + (size_t)R * R;
    double* Xt = Nm + (size_t)R * R;
    double* G = Xt + (size_t)R * M;
    double* Bd = G + (size_t)ncmax * R;
    double* Y = Bd + (size_t)R * ncmax;
    double* V = Y + (size_t)R * kmax;
    double* Zf = V + (size_t)R * kmax;
    double* lam = Zf + (size_t)ncmax * ncmax;
    double* Qr = lam + ncmax;
    double* gaps = Qr + (size_t)kmax * M;
    double* acc_scratch = gaps + T;
    double* Ukeep = acc_scratch + 8;
    hipStream_t s = h->stream;
    auto U_of = [&](double* st) { return st; };
    auto S_of = [&](double* st) { return st + (size_t)M * R; };
    auto acc_of = [&](double* st) { return st + (size_t)M * R + R; };
    auto est_of = [&](double* st) { return st + (size_t)M * R + R + 4; };
    auto step = [&](double* from, int t_from, double* to, int b, double* acc, double* est) {
        // state after block b from the state before it (t_from = number of blocks folded in)
        HIPCHK(hipMemcpyAsync(acc, acc_of(from), 4 * sizeof(double), hipMemcpyDeviceToDevice, s));
        CommitJob j{M, U_of(from), (long)R, S_of(from), t_from == 0 ? 0 : R, blocks[b], R,
                    U_of(to), (long)R, S_of(to), acc, est};
        return commit_batched(h, {j});
    };
    cmsvd_status st;
    fill_diag(ckp, (int)SD, 1, (long)SD, 0.0, 0.0, s);  // empty state: zero accumulators
    // ---- forward: fold the chain, keeping every ck-th state and the last one ----
    {
        double* prev = ckp;
        for (int t = 1; t <= T; ++t) {
            double* next = (t % ck == 0) ? ckp + SD * (t / ck) : seg + SD * (t & 1);
            if (t == T) next = ckp + SD * (nck - 1);
            st = step(prev, t - 1, next, t - 1, acc_of(next), est_of(next));
            if (st != CMSVD_OK) return st;
            prev = next;
        }
    }
    double est_h[2];
    HIPCHK(hipMemcpyAsync(est_h, est_of(ckp + SD * (nck - 1)), 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *f = est_h[0] * est_h[0];
    if (!grads) {
        if (min_gap) *min_gap = INFINITY;
        return CMSVD_OK;
    }
    // ---- backward by segments of ck steps, newest first ----
    int cur = 0;  // (Cb[cur], Zb[cur]) hold C, Z of the step after the one being processed
    const double* Unext = nullptr;
    const int nseg = (T + ck - 1) / ck;
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int a = sg * ck, b = std::min(a + ck, T);
        // states U_a .. U_b of this segment: slot i holds U_{a+i}
        std::vector<double*> sl(b - a + 1);
        sl[0] = ckp + SD * (a / ck);
        sl[b - a] = (b == T) ? ckp + SD * (nck - 1) : ckp + SD * (b / ck);
        for (int i = 1; i < b - a; ++i) {
            sl[i] = seg + SD * i;
            st = step(sl[i - 1], a + i - 1, sl[i], a + i - 1, acc_scratch, nullptr);
            if (st != CMSVD_OK) return st;
        }
        for (int t = b; t > a; --t) {
            const cmsvd_block& B = blocks[t - 1];
            const int k = (int)B.cols, rp = (t - 1 == 0) ? 0 : R, nc = rp + k, nk = std::min(R, nc), d = nc - nk;
            const bool bf = B.dtype == CMSVD_F32;
            double* Up = U_of(sl[t - 1 - a]);
            double* Ut = U_of(sl[t - a]);
            // recompute the step's residual basis and every eigenpair of its core
            CommitJob j{M, Up, (long)R, S_of(sl[t - 1 - a]), rp, B, R, Xt, (long)R, acc_scratch, acc_scratch, nullptr};
            j.Z_out = Zf;
            j.lam_out = lam;
            j.Qr_out = Qr;
            st = commit_batched(h, {j});
            if (st != CMSVD_OK) return st;
            cut_gap(lam, nk, nc, gaps + (t - 1), s);
            double* Cn = Cb[cur ^ 1];
            double* Zn = Zb[cur ^ 1];
            if (t == T) {
                // W_T = U_T U_T^T: C = I, Z = 0
                fill_diag(Cn, R, R, R, 0.0, 1.0, s);
                fill_diag(Zn, R, M, R, 0.0, 0.0, s);
            } else {
                const double* Cp = Cb[cur];
                const double* Zp = Zb[cur];
                // X = W_{t+1} U_t with W_{t+1} = U' C' U'^T + U' Z'^T + Z' U'^T:
                // Mm = U_t^T U', Nm = Z'^T U_t, then Nm <- C' Mm^T + Nm (= E^T),
                // X^T = E U'^T + Mm Z'^T
                if ((st = gemm1(h, false, true, R, R, M, 1.0, Ut, R, false, Unext, R, false, 0.0, Mm, R))) return st;
                if ((st = gemm1(h, false, true, R, R, M, 1.0, Zp, R, false, Ut, R, false, 0.0, Nm, R))) return st;
                if ((st = gemm1(h, false, true, R, R, R, 1.0, Cp, R, false, Mm, R, false, 1.0, Nm, R))) return st;
                if ((st = gemm1(h, true, false, R, M, R, 1.0, Nm, R, false, Unext, R, false, 0.0, Xt, R))) return st;
                if ((st = gemm1(h, false, false, R, M, R, 1.0, Mm, R, false, Zp, R, false, 1.0, Xt, R))) return st;
                // G = Qhat^T X, Qhat = [U_{t-1}, Q_res]
                if ((st = gemm1(h, false, true, rp, R, M, 1.0, Up, R, false, Xt, R, false, 0.0, G, nc))) return st;
                if ((st = gemm1(h, false, true, k, R, M, 1.0, Qr, k, false, Xt, R, false, 0.0, G + rp, nc))) return st;
                // C_t = U_t^T X, in the stored basis of the state (the recomputed kept
                // eigenvectors may differ from it by signs or within clusters)
                if ((st = gemm1(h, false, true, R, R, M, 1.0, Ut, R, false, Xt, R, false, 0.0, Cn, R))) return st;
                // Ghat = Z_d (Gamma o (G^T Z_d))^T - G
                double ghat_sign = -1.0;
                if (d > 0) {
                    if ((st = gemm1(h, true, false, R, d, nc, 1.0, G, nc, false, Zf + (size_t)nk * nc, nc, false, 0.0, Bd, R)))
                        return st;
                    divdiff_scale(Bd, R, nk, d, lam, s);
                    if ((st = gemm1(h, false, true, nc, R, d, 1.0, Zf + (size_t)nk * nc, nc, false, Bd, R, false, -1.0, G, nc)))
                        return st;
                    ghat_sign = 1.0;
                }
                // Z_t^T = Ghat^T Qhat^T + X^T  (built in X^T, then moved to Zn)
                if ((st = gemm1(h, true, false, R, M, rp, ghat_sign, G, nc, false, Up, R, false, 1.0, Xt, R))) return st;
                if ((st = gemm1(h, true, false, R, M, k, ghat_sign, G + rp, nc, false, Qr, k, false, 1.0, Xt, R))) return st;
                HIPCHK(hipMemcpyAsync(Zn, Xt, (size_t)R * M * 8, hipMemcpyDeviceToDevice, s));
            }
            // grad_t = 2 A_t - 2 (U_t (C Y + V) + Z Y) with Y = U_t^T A_t, V = Z^T A_t
            double* gt = grads[t - 1];
            if ((st = gemm1(h, false, true, R, k, M, 1.0, Ut, R, false, B.ptr, B.ld, bf, 0.0, Y, R))) return st;
            if ((st = gemm1(h, false, true, R, k, M, 1.0, Zn, R, false, B.ptr, B.ld, bf, 0.0, V, R))) return st;
            if ((st = gemm1(h, false, false, R, k, R, 1.0, Cn, R, false, Y, R, false, 1.0, V, R))) return st;
            if ((st = copy_block(h, B, gt))) return st;
            if ((st = gemm1(h, true, false, k, M, R, -2.0, V, R, false, Ut, R, false, 2.0, gt, k))) return st;
            if ((st = gemm1(h, true, false, k, M, R, -2.0, Y, R, false, Zn, R, false, 1.0, gt, k))) return st;
            cur ^= 1;
            Unext = Ut;
        }
        // the next segment recomputes into the slots that may hold U_{a+1}
        if (Unext != Ukeep) {
            HIPCHK(hipMemcpyAsync(Ukeep, Unext, (size_t)R * M * 8, hipMemcpyDeviceToDevice, s));
            Unext = Ukeep;
        }
    }
    std::vector<double> gh(T);
    HIPCHK(hipMemcpyAsync(gh.data(), gaps, T * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (min_gap) {
        double g = INFINITY;
        for (double v : gh) g = std::min(g, v);
        *min_gap = g;
    }
    return CMSVD_OK;
} catch (...) {
    return caught(__func__);
}

}  // extern "C"
