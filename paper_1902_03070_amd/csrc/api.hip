// C-ABI of libtsvdmi: context, device workspace, execution plans and the
// entry points declared in include/tsvdmi.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/tsvdmi.h"
#include "internal.h"

using namespace tsvd;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct tsvd_ctx {
    int device = 0;
    int cus = 0;
    int max_sweeps = 30;
    int sync_status = 1;
    int team_size = 0;
    int team_slots = 0;  // > 0: slices in flight per XCD of the multi-workgroup kernel (forced)
    int group_lanes = 0;
    int group_cols = 0;
    int autotune = 1;
    int warm_start = -1;  // complete_tensor: -1 automatic period, 0 off, N: reset V every N iterations
    int spin_limit = 1 << 24;
    std::string err = "";
    // transform matrices: (n3, prec) -> {C, C^T} rows, element type by prec
    std::map<std::pair<int, int>, std::pair<void*, void*>> dct;
    // matrix-core fragments: (n3, engine, inverse) -> device buffer
    std::map<std::tuple<int, int, int>, void*> frag;
    // fast-transform tables of long tubes: 2 n3 + (float data) -> device buffer
    std::map<int, void*> fft;
    int dense_long = 0;  // 1: DCT tubes of 129..512 on the dense kernel where it fits
    DevBuf ws;                 // main workspace
    DevBuf ctrl;               // Ctrl + norms + history (persistent)
    Ctrl* h_ctrl = nullptr;    // pinned host mirror
    std::vector<void*> owned;  // other allocations freed at destroy
    std::mutex mu;
    // phase profiling (TSVD_OPT_PROFILE): event pairs recorded on the launch stream
    int prof = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> marks;
    // graph capture of the completion iteration
    int use_graphs = 1;
    int capturing = 0;
    hipStream_t own = nullptr;  // context stream (capture cannot use the legacy default stream)
    int noalloc = 0;            // inside tsvt_dct_noalloc: no tuning, no profiling events
    int coop = 0;               // 1: cooperative launches of the team kernel outside capture
    int gram = -1;              // block-Gram kernel: 0 a tuner candidate, 1 forced, -1 excluded
    int kept_cols = 1;          // 1: t-SVTs with cold SVDs (single calls, cold completions) run the kept-column Jacobi
    // operands of a caller-given tube transform (tsvt_transform, the DFT path), cached by content
    DevBuf xf;
    std::vector<double> xf_key;
    int xf_eng = -1;
};

// Fixed scratch of tsvt_dct_noalloc (TSVD_NOALLOC_MAX_BYTES).  Every GPU the
// library runs on holds one copy of this array for the life of the process.
// Its device address on each device is looked up once (tsvd_create, with that
// device current) and kept; host code passes that address to kernels and
// copies, never the array's name, which on the host is only a stand-in.
constexpr size_t kScratchBytes = TSVD_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

int fail(tsvd_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(tsvd_ctx* c, hipError_t e, const char* where) {
    (void)hipGetLastError();  // clear the runtime's sticky copy of a non-fatal error
    return fail(c, TSVD_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                                         \
    do {                                                          \
        hipError_t e__ = (expr);                                  \
        if (e__ != hipSuccess) return hip_fail((ctx), e__, #expr); \
    } while (0)

inline int esize(int prec) { return prec == TSVD_FP64 ? 8 : 4; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Orthonormal DCT-II matrix (Section 3, dct(.,[],3)) in FP64 on the host,
// uploaded in the element type: C row-major [k][t] and its transpose.
int get_dct(tsvd_ctx* c, int n3, int prec, const void** C, const void** Ct) {
    auto key = std::make_pair(n3, prec == TSVD_FP64 ? 0 : 1);
    auto it = c->dct.find(key);
    if (it == c->dct.end()) {
        std::vector<double> m((size_t)n3 * n3), mt((size_t)n3 * n3);
        const double pi = acos(-1.0);
        for (int k = 0; k < n3; ++k) {
            const double s = k == 0 ? sqrt(1.0 / n3) : sqrt(2.0 / n3);
            for (int t = 0; t < n3; ++t) {
                const double v = s * cos(pi * (2.0 * t + 1.0) * k / (2.0 * n3));
                m[(size_t)k * n3 + t] = v;
                mt[(size_t)t * n3 + k] = v;
            }
        }
        const size_t bytes = (size_t)n3 * n3 * esize(prec);
        void *d0 = nullptr, *d1 = nullptr;
        HIPCHK(c, hipMalloc(&d0, bytes));
        HIPCHK(c, hipMalloc(&d1, bytes));
        if (prec == TSVD_FP64) {
            HIPCHK(c, hipMemcpy(d0, m.data(), bytes, hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(d1, mt.data(), bytes, hipMemcpyHostToDevice));
        } else {
            std::vector<float> f(m.begin(), m.end()), ft(mt.begin(), mt.end());
            HIPCHK(c, hipMemcpy(d0, f.data(), bytes, hipMemcpyHostToDevice));
            HIPCHK(c, hipMemcpy(d1, ft.data(), bytes, hipMemcpyHostToDevice));
        }
        it = c->dct.emplace(key, std::make_pair(d0, d1)).first;
    }
    *C = it->second.first;
    *Ct = it->second.second;
    return TSVD_OK;
}

int tube_engine(int prec) { return prec == TSVD_FP64 ? 0 : prec == TSVD_FP32 ? 1 : 2; }

// C or C^T in fragment order for the matrix-core tube transform.
int get_frag(tsvd_ctx* c, int n3, int prec, int inverse, const void** out) {
    const int eng = tube_engine(prec);
    auto key = std::make_tuple(n3, eng, inverse);
    auto it = c->frag.find(key);
    if (it == c->frag.end()) {
        std::vector<double> m((size_t)n3 * n3);
        const double pi = acos(-1.0);
        for (int k = 0; k < n3; ++k) {
            const double sk = k == 0 ? sqrt(1.0 / n3) : sqrt(2.0 / n3);
            for (int t = 0; t < n3; ++t) {
                const double v = sk * cos(pi * (2.0 * t + 1.0) * k / (2.0 * n3));
                if (!inverse) m[(size_t)k * n3 + t] = v;   // out[k] = sum_t C[k][t] in[t]
                else m[(size_t)t * n3 + k] = v;            // out[t] = sum_k C[k][t] in[k]
            }
        }
        const size_t bytes = tube_fragment_bytes(eng, n3);
        std::vector<unsigned char> h(bytes);
        make_tube_fragments(eng, n3, m.data(), h.data());
        void* d = nullptr;
        HIPCHK(c, hipMalloc(&d, bytes));
        HIPCHK(c, hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice));
        it = c->frag.emplace(key, d).first;
    }
    *out = it->second;
    return TSVD_OK;
}

// Tube transform along n3 (forward or inverse) on the matrix cores; tubes
// longer than kMaxTube use the vector-ALU kernel with the dense matrix.
// `mat` is the transform operand: fragments for n3 <= kMaxTube, else the
// dense matrix (see launch_tube_matrix).
int run_tube_mat(tsvd_ctx* c, int prec, TubeArgs a, int inverse, const void* mat, hipStream_t s) {
    hipError_t e;
    if (a.n3 <= kMaxTube) {
        e = launch_tube_mfma(tube_engine(prec), a, mat, s);
    } else {
        if (dense_tube_lds(prec, a.n3) > kLdsBudget)
            return fail(c, TSVD_EINVAL, "tubes too long for the dense transform kernel");
        a.M = mat;
        e = launch_tube_transform(prec == TSVD_FP64 ? 0 : 1, a, s);
    }
    if (e != hipSuccess) return hip_fail(c, e, inverse ? "inverse tube transform" : "tube transform");
    return TSVD_OK;
}

// Tables of the fast transform for tubes of length n3 in the precision of the
// data (FP64 for double, FP32 for float), built once per context.
int get_fft_tables(tsvd_ctx* c, int n3, int prec, const void** out) {
    const int tp = prec == TSVD_FP64 ? 0 : 1;
    const int key = 2 * n3 + tp;
    auto it = c->fft.find(key);
    if (it == c->fft.end()) {
        const size_t bytes = fft_table_bytes(n3, tp);
        std::vector<unsigned char> h(bytes);
        make_fft_tables(n3, tp, h.data());
        void* d = nullptr;
        HIPCHK(c, hipMalloc(&d, bytes));
        const hipError_t e = hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return hip_fail(c, e, "fast-transform tables");
        }
        it = c->fft.emplace(key, d).first;
    }
    *out = it->second;
    return TSVD_OK;
}

// The fast transform of long tubes (mode: kFftDct* or kFftDft*).
int run_tube_fft(tsvd_ctx* c, int prec, const TubeArgs& a, int mode, hipStream_t s) {
    const void* tab;
    int rc = get_fft_tables(c, a.n3, prec, &tab);
    if (rc) return rc;
    const hipError_t e = launch_tube_fft(prec == TSVD_FP64 ? 0 : 1, a, tab, mode, s);
    if (e != hipSuccess) return hip_fail(c, e, (mode & 1) ? "inverse fast tube transform" : "fast tube transform");
    return TSVD_OK;
}

// Whether DCT tubes of length n3 take the fast transform.
bool use_fft(const tsvd_ctx* c, int prec, int n3) {
    if (!fft_fits(n3)) return false;
    return !(c->dense_long && dense_tube_lds(prec, n3) <= kLdsBudget);
}

// Transform operands run_tube uses (fast-transform tables, fragments or the dense
// matrices), built now: before a graph capture, which cannot allocate.
int prepare_tube(tsvd_ctx* c, int n3, int prec) {
    const void *a, *b;
    if (use_fft(c, prec, n3)) return get_fft_tables(c, n3, prec, &a);
    if (n3 <= kMaxTube) {
        int rc = get_frag(c, n3, prec, 0, &a);
        return rc ? rc : get_frag(c, n3, prec, 1, &b);
    }
    return get_dct(c, n3, prec, &a, &b);
}

int run_tube(tsvd_ctx* c, int prec, TubeArgs a, int inverse, hipStream_t s) {
    const void* mat;
    if (use_fft(c, prec, a.n3)) return run_tube_fft(c, prec, a, inverse ? kFftDctInverse : kFftDctForward, s);
    if (a.n3 <= kMaxTube) {
        int rc = get_frag(c, a.n3, prec, inverse, &mat);
        if (rc) return rc;
    } else {
        const void *C, *Ct;
        int rc = get_dct(c, a.n3, prec, &C, &Ct);
        if (rc) return rc;
        mat = inverse ? Ct : C;
    }
    return run_tube_mat(c, prec, a, inverse, mat, s);
}

// Grow-only workspace.  Growing frees the old buffer (hipFree waits for the device).
int ensure_ws(tsvd_ctx* c, size_t bytes) {
    if (c->ws.bytes >= bytes) return TSVD_OK;
    if (c->ws.p) {
        HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipFree(c->ws.p));
        c->ws.p = nullptr;
        c->ws.bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)64 << 20);
    hipError_t e = hipMalloc(&c->ws.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = hipMalloc(&c->ws.p, bytes);
        want = bytes;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->ws.p = nullptr;
        return fail(c, TSVD_ENOMEM, "workspace allocation failed");
    }
    c->ws.bytes = want;
    return TSVD_OK;
}

// Bump allocator over the workspace.
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    }
};

constexpr int kHist = 4096;  // relative-change history ring (slot = iteration mod kHist) in the control region

struct CtrlRegion {
    Ctrl* ctrl;
    double* norms;  // [2 kNormSlots]
    double* hist;   // [kHist]
};

int ensure_ctrl(tsvd_ctx* c, CtrlRegion* r) {
    const size_t bytes = 256 + 256 + sizeof(double) * kHist;
    if (!c->ctrl.p) {
        HIPCHK(c, hipMalloc(&c->ctrl.p, bytes));
        HIPCHK(c, hipMemset(c->ctrl.p, 0, bytes));
        c->ctrl.bytes = bytes;
        HIPCHK(c, hipHostMalloc((void**)&c->h_ctrl, sizeof(Ctrl), hipHostMallocDefault));
    }
    char* b = (char*)c->ctrl.p;
    r->ctrl = (Ctrl*)b;
    r->norms = (double*)(b + 256);
    r->hist = (double*)(b + 512);
    return TSVD_OK;
}

// Status code of a set of device status bits (non-finite input first, then a
// timed-out wait, then a Jacobi SVD that hit the sweep limit).
int status_code(int bits) {
    if (bits & kStNonFinite) return TSVD_ENONFINITE;
    if (bits & kStTimeout) return TSVD_ETIMEOUT;
    if (bits & kStNoConv) return TSVD_WARN_NOCONV;
    return TSVD_OK;
}

// Read and clear the accumulated device status (synchronizes `s`).
int read_status(tsvd_ctx* c, hipStream_t s, int* max_sweeps) {
    CtrlRegion cr;
    int rc = ensure_ctrl(c, &cr);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(s));
    Ctrl h;
    HIPCHK(c, hipMemcpy(&h, cr.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    Ctrl z = h;
    z.status = 0;
    z.max_sweeps = 0;
    HIPCHK(c, hipMemcpy(cr.ctrl, &z, sizeof(Ctrl), hipMemcpyHostToDevice));
    if (max_sweeps) *max_sweeps = h.max_sweeps;
    if (h.status & kStNonFinite) return fail(c, TSVD_ENONFINITE, "input holds a non-finite value");
    if (h.status & kStTimeout) return fail(c, TSVD_ETIMEOUT, "a device-side wait timed out");
    if (h.status & kStNoConv) return TSVD_WARN_NOCONV;
    return TSVD_OK;
}

// Records an event pair around the launches of one phase when profiling: every
// phase at level 1, only the Jacobi phase (1) at level 2.
struct PhaseMark {
    tsvd_ctx* c;
    int ph;
    hipStream_t s;
    hipEvent_t a = nullptr;
    bool on() const { return !c->noalloc && (c->prof == 1 || (c->prof == 2 && ph == 1)); }
    static hipEvent_t take(tsvd_ctx* c) {
        if (c->ev_used == c->ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            c->ev_pool.push_back(e);
        }
        return c->ev_pool[c->ev_used++];
    }
    PhaseMark(tsvd_ctx* c_, int ph_, hipStream_t s_) : c(c_), ph(ph_), s(s_) {
        if (on() && (a = take(c))) (void)hipEventRecord(a, s);
    }
    ~PhaseMark() {
        if (!on() || !a) return;
        hipEvent_t b = take(c);
        if (!b) return;
        (void)hipEventRecord(b, s);
        c->marks.emplace_back(ph, a, b);
    }
};

// ---------------------------------------------------------------------------
// Plan of one t-SVT / t-SVD of an n1 x n2 x n3 tensor.
// ---------------------------------------------------------------------------
struct Plan {
    int prec = 0;
    int64_t n1 = 0, n2 = 0, n3 = 0, N = 0;
    int m = 0, p = 0, trans = 0, with_v = 0;
    int team = 0;        // 0: resident kernel; 1: team kernel
    int threads = 256;
    int tile_source = 0, tile_W = 0;
    int K = 1;           // team kernel lane-group columns
    int warm = 0, warm_period = 0;  // completion warm start: A0 = Zbar V before Jacobi (V kept across iterations)
    size_t o_A0 = 0;
    int lds = 0;
    TeamSched ts{};
    JacobiJob job{};
    // workspace offsets
    size_t o_zbar, o_A, o_F, o_G, o_w, o_sig, o_ybar, o_V, o_rot, o_sw, o_bar, o_rank, o_pos, o_end;
    size_t o_ctr_begin, o_ctr_end;  // region zeroed per call (counters)
    // kept-column Jacobi and its threshold certificate (plan_kept_columns)
    int keep = 0;
    size_t o_full = 0, o_ncols = 0, o_sums = 0, o_done = 0, o_rot2 = 0, o_bar2 = 0, o_flags = 0, o_nrm2 = 0, o_As = 0, o_H = 0, o_H2 = 0;
};

// ---------------------------------------------------------------------------
// Jacobi tiles: how one tensor's slices map onto workgroups.
//   team 0: one workgroup per slice, the whole slice resident in LDS,
//           `threads` lanes (threads / G column-pair groups);
//   team 1: W workgroups per slice exchanging column blocks through the L2
//           (batched plans: a team of one workgroup of kTeamMaxThreads lanes).
// ---------------------------------------------------------------------------
struct Tile {
    int team = 0;    // 0 resident, 1 multi-workgroup (column pairs), 2 multi-workgroup block-Gram
    int G = 16;
    int W = 0;
    int threads = 0;
    int K = 1;       // team: lane-group columns (2: two I columns per group, no V)
    int slots = 0;   // team: slices in flight per XCD (0: as many as residency and n3 allow)
    int source = 0;  // 0 default heuristic, 1 autotuned, 2 forced by options
};

// Resident workgroup size: one group of G lanes per column pair of a round
// (at most 1024 lanes), or half as many groups (each takes two pairs).
int resident_threads(int p, int G, int halve) {
    const int per_wave = kWave / G;
    int ngrp = std::min((p + 1) / 2, 1024 / G);
    if (halve) ngrp = (ngrp + 1) / 2;
    ngrp = (ngrp + per_wave - 1) / per_wave * per_wave;
    return std::max(kWave, ngrp * G);
}

// Fill the Jacobi part of a plan from a tile.  Fails when the tile cannot
// hold the slice (LDS, residency, row geometry).
int apply_tile(tsvd_ctx* c, Plan& P, const Tile& t, bool batched) {
    if (t.team == 2) {
        // block-Gram: blocks of kGramB columns, 256 threads, one block pair per workgroup and step
        if (batched) return fail(c, TSVD_EINVAL, "the block-Gram kernel is a multi-workgroup kernel");
        const int lds = jacobi_gram_lds_bytes(P.prec, P.m);
        if (lds > kLdsBudget) return fail(c, TSVD_EINVAL, "slice too large for the block-Gram kernel");
        int nb = (P.p + kGramBlock - 1) / kGramBlock;
        nb += nb & 1;
        int W = std::max(1, std::min(t.W, nb / 2));
        const int cap = jacobi_gram_max_resident(P.prec, P.m, P.with_v);
        if (cap < 8) return fail(c, TSVD_EINVAL, "block-Gram kernel cannot be resident with this shape");
        W = std::min(W, cap / 8);
        const int per_xcd = std::max(1, std::min(((int)P.n3 + 7) / 8, cap / (8 * W)));
        P.team = 2;
        P.lds = lds;
        P.threads = 256;
        P.K = 1;
        P.ts.W = W;
        P.ts.nwg = 8 * W * per_xcd;
        P.job.b = kGramBlock;
        P.job.nb = nb;
        P.job.G = 16;  // lanes per pair in its rotation phase (reported by tsvd_get_tile)
        return TSVD_OK;
    }
    int R, ldv;
    if (jacobi_geometry_g(P.m, P.p, t.G, &R, &ldv)) return fail(c, TSVD_EINVAL, "lane group cannot hold the slice rows");
    P.job.G = t.G;
    P.job.R = R;
    P.job.ldv = ldv;
    if (t.G == 64 && (!t.team || batched || t.K == 2))
        return fail(c, TSVD_EINVAL, "64-lane groups exist for the multi-workgroup Jacobi kernel only");
    if (!t.team) {
        const int rl = jacobi_resident_lds_bytes(P.prec, P.m, P.p, t.G, P.with_v);
        if (rl > kLdsBudget) return fail(c, TSVD_EINVAL, "slice does not fit in LDS");
        P.team = 0;
        P.lds = rl;
        P.threads = batched ? kTeamMaxThreads : t.threads;
        if (P.threads < kWave || P.threads > 1024 || P.threads % t.G) return fail(c, TSVD_EINVAL, "bad workgroup size");
        P.job.b = 0;
        P.job.nb = 0;
        P.ts = TeamSched{1, 0, nullptr};
        return TSVD_OK;
    }
    P.team = 1;
    if (batched) {
        // a team of one workgroup with b G == kTeamMaxThreads
        const int b = kTeamMaxThreads / t.G;
        if (jacobi_team_lds_bytes(P.prec, P.m, P.p, t.G, b, P.with_v) > kLdsBudget)
            return fail(c, TSVD_EINVAL, "slice too large for the batched Jacobi kernel");
        int nb = (P.p + b - 1) / b;
        nb += nb & 1;
        P.lds = jacobi_team_lds_bytes(P.prec, P.m, P.p, t.G, b, P.with_v);
        P.threads = kTeamMaxThreads;
        P.ts = TeamSched{1, 1, nullptr};
        P.job.b = b;
        P.job.nb = nb;
        return TSVD_OK;
    }
    if (t.K == 2) {
        if (P.with_v) return fail(c, TSVD_EINVAL, "two columns per lane group need no V");
        // block width B = 2 ng columns for ng groups; ng G must fill whole wavefronts
        const int gstep = std::max(1, kWave / t.G), bstep = 2 * gstep;
        const int bmax = 2 * (kTeamMaxThreads / t.G);
        int W = std::max(1, t.W);
        int B = (P.p + 2 * W - 1) / (2 * W);
        B = (B + bstep - 1) / bstep * bstep;
        B = std::min(B, bmax);
        while (B > bstep && jacobi_team_lds_bytes(P.prec, P.m, P.p, t.G, B, 0) > kLdsBudget) B -= bstep;
        if (jacobi_team_lds_bytes(P.prec, P.m, P.p, t.G, B, 0) > kLdsBudget)
            return fail(c, TSVD_EINVAL, "slice too large for the Jacobi team kernel");
        int nb = (P.p + B - 1) / B;
        nb += nb & 1;
        if (W > nb / 2) W = nb / 2;
        P.lds = jacobi_team_lds_bytes(P.prec, P.m, P.p, t.G, B, 0);
        P.threads = (B / 2) * t.G;
        const int cap = jacobi_team_max_resident(P.prec, P.lds, P.threads, 0, R, t.G, 2);
        if (cap < 8) return fail(c, TSVD_EINVAL, "Jacobi team kernel cannot be resident with this shape");
        W = std::min(W, cap / 8);
        int per_xcd = std::max(1, std::min(((int)P.n3 + 7) / 8, cap / (8 * W)));
        if (t.slots > 0) per_xcd = std::min(per_xcd, t.slots);
        P.ts.W = W;
        P.ts.nwg = 8 * W * per_xcd;
        P.job.b = B;
        P.job.nb = nb;
        P.K = 2;
        return TSVD_OK;
    }
    P.K = 1;
    const int bstep = std::max(2, kWave / t.G);  // b G must fill whole wavefronts
    const int bmax = (t.G == 64 ? kTeamMaxThreads64 : kTeamMaxThreads) / t.G;
    int W = std::max(1, t.W);
    int b = (P.p + 2 * W - 1) / (2 * W);
    b = (b + bstep - 1) / bstep * bstep;
    b = std::min(b, bmax);
    while (b > bstep && jacobi_team_lds_bytes(P.prec, P.m, P.p, t.G, b, P.with_v) > kLdsBudget) b -= bstep;
    if (jacobi_team_lds_bytes(P.prec, P.m, P.p, t.G, b, P.with_v) > kLdsBudget)
        return fail(c, TSVD_EINVAL, "slice too large for the Jacobi team kernel");
    int nb = (P.p + b - 1) / b;
    nb += nb & 1;
    if (W > nb / 2) W = nb / 2;
    P.lds = jacobi_team_lds_bytes(P.prec, P.m, P.p, t.G, b, P.with_v);
    P.threads = b * t.G;
    const int cap = jacobi_team_max_resident(P.prec, P.lds, P.threads, P.with_v, R, t.G, 1);
    if (cap < 8) return fail(c, TSVD_EINVAL, "Jacobi team kernel cannot be resident with this shape");
    // whole teams on every XCD: the grid is a multiple of 8 W workgroups
    W = std::min(W, cap / 8);
    int per_xcd = std::max(1, std::min(((int)P.n3 + 7) / 8, cap / (8 * W)));
    if (t.slots > 0) per_xcd = std::min(per_xcd, t.slots);
    P.ts.W = W;
    P.ts.nwg = 8 * W * per_xcd;
    P.job.b = b;
    P.job.nb = nb;
    return TSVD_OK;
}

// Of an XCD's 4 MiB L2, what the slices in flight on it may hold (3.5 MiB).
constexpr size_t kL2PerXcdBudget = (size_t)7 << 19;

// Lane-group widths worth trying: those with the fewest padded rows R G.
std::vector<int> group_widths(int m, int p) {
    std::vector<int> out;
    int best = 1 << 30;
    for (int G : {16, 32}) {
        int R, ldv;
        if (!jacobi_geometry_g(m, p, G, &R, &ldv)) best = std::min(best, R * G);
    }
    // 32-lane groups first: the tuner keeps the first of two candidates within 2%
    // of each other, and for the completion at 256 x 256 x 31 (FP64) the tuner's
    // synthetic sweeps put 32-lane groups only 2.3% ahead where the real ones
    // gain 4.6%
    for (int G : {32, 16}) {
        int R, ldv;
        if (!jacobi_geometry_g(m, p, G, &R, &ldv) && R * G == best) out.push_back(G);
    }
    return out;
}

Tile default_tile(const Plan& P, int team_size, int group_lanes, int group_cols, bool batched) {
    Tile t;
    int G, R, ldv;
    jacobi_geometry(P.m, P.p, &G, &R, &ldv);
    t.G = group_lanes ? group_lanes : G;
    t.team = jacobi_resident_lds_bytes(P.prec, P.m, P.p, t.G, P.with_v) > kLdsBudget;
    t.W = t.team ? (team_size > 0 ? team_size : std::max(1, (P.p + 63) / 64)) : 0;
    t.threads = t.team ? 0 : resident_threads(P.p, t.G, 0);
    t.K = (t.team && !batched && !P.with_v && group_cols == 2) ? 2 : 1;
    return t;
}

// The forced block-Gram tile of a multi-workgroup plan (W from the team-size
// option, else one workgroup per 32 columns).
Tile gram_tile(const Plan& P, int team_size) {
    Tile t = default_tile(P, team_size, 0, 0, false);
    if (t.team) {
        t.team = 2;
        t.G = 16;
        t.K = 1;
        t.W = team_size > 0 ? team_size : std::max(1, (P.p + 31) / 32);
    }
    return t;
}

std::vector<Tile> tile_candidates(const Plan& P, bool batched, int gram) {
    std::vector<Tile> out;
    for (int G : group_widths(P.m, P.p)) {
        Tile t;
        t.G = G;
        t.team = jacobi_resident_lds_bytes(P.prec, P.m, P.p, G, P.with_v) > kLdsBudget;
        if (batched) {
            t.threads = kTeamMaxThreads;
            out.push_back(t);
        } else if (!t.team) {
            for (int h = 0; h < 2; ++h) {
                t.threads = resident_threads(P.p, G, h);
                if (out.empty() || out.back().threads != t.threads || out.back().G != G) out.push_back(t);
            }
        } else {
            for (int K : {1, 2}) {
                if (K == 2 && P.with_v) continue;
                t.K = K;
                for (int W : {1, 2, 3, 4, 6, 8, 12, 16}) {
                    t.W = W;
                    out.push_back(t);
                }
            }
        }
    }
    // multi-workgroup slices also try one column pair per wavefront (64-lane
    // groups, up to 1024 threads): twice the wavefronts per CU to hide the
    // latency of each pair's chain, at up to 8 rows per lane
    int R64, ldv64;
    if (!batched && !out.empty() && out.back().team && !jacobi_geometry_g(P.m, P.p, 64, &R64, &ldv64) && R64 <= 8) {
        Tile t;
        t.G = 64;
        t.team = 1;
        t.K = 1;
        for (int W : {2, 4, 8, 12, 16}) {
            t.W = W;
            out.push_back(t);
        }
    }
    // Slices whose A (and V) overflow an XCD's L2 when every team of the XCD
    // holds one: also try fewer slices in flight per XCD (teams then take
    // several slices in turn), with the larger team sizes to keep the CUs busy.
    if (!batched && !out.empty() && out.back().team) {
        const size_t es = P.prec == TSVD_FP64 ? 8 : 4;
        const size_t slice_bytes = ((size_t)P.m * P.p + (P.with_v ? (size_t)P.p * P.p : 0)) * es;
        const int fit = (int)(kL2PerXcdBudget / slice_bytes);
        if (fit >= 1 && fit < ((int)P.n3 + 7) / 8) {
            const size_t n0 = out.size();
            for (size_t i = 0; i < n0; ++i) {
                if (out[i].team != 1 || out[i].K != 1 || out[i].W < 8) continue;
                Tile t = out[i];
                t.slots = fit;
                out.push_back(t);
            }
        }
    }
    // and the block-Gram kernel (column blocks on the matrix cores)
    if (!batched && gram >= 0 && !out.empty() && out.back().team) {
        Tile t;
        t.team = 2;
        t.G = 16;
        t.K = 1;
        for (int W : {1, 2, 4, 8, 16}) {
            t.W = W;
            out.push_back(t);
        }
    }
    return out;
}

// ---- process-wide tile cache -----------------------------------------------
// Key: (batched, prec, m, p, n3, with_v); batched plans ignore n3.  When the
// environment variable TSVDMI_TILE_CACHE names a file, it is read at first
// use and every newly tuned tile is appended to it, one line per tile:
//   tile <batched> <prec> <m> <p> <n3> <with_v> <team> <G> <W> <threads> <K> <microseconds> [<slots>]
typedef std::tuple<int, int, int, int, int, int> TileKey;
std::mutex g_tile_mu;
std::map<TileKey, Tile> g_tiles;
bool g_tiles_loaded = false;

void tile_cache_load_locked() {
    if (g_tiles_loaded) return;
    g_tiles_loaded = true;
    const char* path = getenv("TSVDMI_TILE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        int k[6], team, G, W, th, K, slots = 0;
        double us;
        if (sscanf(line, "tile %d %d %d %d %d %d %d %d %d %d %d %lf %d", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &team,
                   &G, &W, &th, &K, &us, &slots) < 12)
            continue;
        Tile t;
        t.team = team; t.G = G; t.W = W; t.threads = th; t.K = K == 2 ? 2 : 1; t.slots = std::max(0, slots);
        t.source = 1;
        g_tiles[TileKey(k[0], k[1], k[2], k[3], k[4], k[5])] = t;
    }
    fclose(f);
}

bool tile_cache_get(const TileKey& k, Tile* t) {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    tile_cache_load_locked();
    auto it = g_tiles.find(k);
    if (it == g_tiles.end()) return false;
    *t = it->second;
    return true;
}

void tile_cache_put(const TileKey& k, const Tile& t, double us) {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    tile_cache_load_locked();
    g_tiles[k] = t;
    const char* path = getenv("TSVDMI_TILE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "tile %d %d %d %d %d %d %d %d %d %d %d %.1f %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
            std::get<3>(k), std::get<4>(k), std::get<5>(k), t.team, t.G, t.W, t.threads, t.K, us, t.slots);
    fclose(f);
}

// ---- the tuner --------------------------------------------------------------
// Times every candidate tile on synthetic slices of the plan's shape (a
// deterministic pattern, kTuneSweeps sweeps with rotation threshold 0 so that
// every candidate does the same work) on the context's own stream, and keeps
// the fastest.  Runs once per key per process.
constexpr int kTuneSweeps = 3;
constexpr int kTuneReps = 3;
constexpr int kTuneBatchTasks = 64;

int ensure_own_stream(tsvd_ctx* c) {
    if (!c->own) HIPCHK(c, hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
    return TSVD_OK;
}

// Time one candidate; returns microseconds per launch or a negative value.
double time_tile(tsvd_ctx* c, const Plan& P0, const Tile& t, bool batched, char* tb, size_t o_src, size_t o_A,
                 size_t o_V, size_t o_cnt, size_t cnt_bytes, size_t o_jobs, size_t o_tj, size_t o_tk, int ntasks,
                 hipEvent_t e0, hipEvent_t e1) {
    Plan P = P0;
    if (apply_tile(c, P, t, batched)) return -1.0;
    JacobiJob& J = P.job;
    J.src = tb + o_src;
    J.A = tb + o_A;
    J.V = P.with_v ? (void*)(tb + o_V) : nullptr;
    J.src_ss = (int64_t)P.m * P.p; J.src_rs = 1; J.src_cs = P.m;
    J.m = P.m;
    J.p = P.p;
    J.n3 = ntasks;
    J.tol = 0.0;
    J.skip2 = 0.0;
    J.refine64 = 0;
    // counters: [Ctrl 256][queue 256][sweeps 4 ntasks][rot 4 ntasks kRotStride][team ctl]
    char* cnt = tb + o_cnt;
    Ctrl* ctrl = (Ctrl*)cnt;
    int* queue = (int*)(cnt + 256);
    J.sweeps = (int*)(cnt + 512);
    J.rot = (int*)(cnt + 512 + align256((size_t)4 * ntasks));
    P.ts.ctl = (int*)(cnt + 512 + align256((size_t)4 * ntasks) + align256((size_t)4 * ntasks * kRotStride));
    if (batched && hipMemcpy(tb + o_jobs, &J, sizeof(JacobiJob), hipMemcpyHostToDevice) != hipSuccess) return -1.0;
    hipStream_t s = c->own;
    double best = -1.0;
    for (int rep = 0; rep <= kTuneReps; ++rep) {
        if (launch_fill_zero(cnt, (int64_t)cnt_bytes, s) != hipSuccess) return -1.0;
        if (hipEventRecord(e0, s) != hipSuccess) return -1.0;
        hipError_t e;
        if (batched)
            e = launch_jacobi_batched(P.prec == TSVD_FP64 ? 0 : 1, J.R, J.G, P.with_v, (const JacobiJob*)(tb + o_jobs),
                                      (const int*)(tb + o_tj), (const int*)(tb + o_tk), ntasks, queue, kTuneSweeps,
                                      ctrl, P.lds, s);
        else if (!P.team)
            e = launch_jacobi_resident(P.prec, J, nullptr, nullptr, nullptr, ntasks, kTuneSweeps, ctrl, P.lds,
                                       P.threads, P.with_v, s);
        else if (P.team == 2)
            e = launch_jacobi_gram(P.prec, J, ntasks, P.ts, kTuneSweeps, ctrl, P.with_v, c->spin_limit, c->coop, s);
        else
            e = launch_jacobi_team(P.prec, J, ntasks, P.ts, kTuneSweeps, ctrl, P.lds, P.threads, P.with_v,
                                   c->spin_limit, J.R, J.G, P.K, c->coop, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return -1.0;
        }
        if (hipEventRecord(e1, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return -1.0;
        Ctrl h;
        if (hipMemcpy(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost) != hipSuccess) return -1.0;
        // every slice must have run every sweep (threshold 0 never converges)
        if ((h.status & (kStTimeout | kStNonFinite)) || h.slice_sweeps != (unsigned long long)ntasks * kTuneSweeps)
            return -1.0;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
        if (rep > 0 && (best < 0.0 || 1e3 * ms < best)) best = 1e3 * ms;  // first run warms up
    }
    return best;
}

int tune_tile(tsvd_ctx* c, const Plan& P, bool batched, Tile* out, double* us_out) {
    std::vector<Tile> cands = tile_candidates(P, batched, c->gram);
    if (cands.size() < 2) return -1;
    int rc = ensure_own_stream(c);
    if (rc) return rc;
    const size_t es = esize(P.prec);
    const int ntasks = batched ? kTuneBatchTasks : (int)P.n3;
    const size_t slice = (size_t)P.m * P.p;
    Carve cv;
    const size_t o_src = cv.take(slice * ntasks * es), o_A = cv.take(slice * ntasks * es);
    const size_t o_V = cv.take(P.with_v ? (size_t)P.p * P.p * ntasks * es : 0);
    const size_t o_jobs = cv.take(sizeof(JacobiJob)), o_tj = cv.take((size_t)4 * ntasks),
                 o_tk = cv.take((size_t)4 * ntasks);
    const size_t cnt_bytes = 512 + align256((size_t)4 * ntasks) + align256((size_t)4 * ntasks * kRotStride) +
                             (size_t)4 * (kTeamCtlInts + 8 * 64 * 64);
    const size_t o_cnt = cv.take(cnt_bytes);
    char* tb = nullptr;
    if (hipMalloc((void**)&tb, cv.off) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best_us = -1.0;
    Tile best;
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    if (ok) {
        std::vector<int> tj(ntasks, 0), tk(ntasks);
        for (int i = 0; i < ntasks; ++i) tk[i] = i;
        ok = launch_fill_pattern(tb + o_src, (int64_t)slice * ntasks, P.prec == TSVD_FP64 ? 0 : 1, 12345u, c->own) ==
                 hipSuccess &&
             hipMemcpy(tb + o_tj, tj.data(), 4 * ntasks, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(tb + o_tk, tk.data(), 4 * ntasks, hipMemcpyHostToDevice) == hipSuccess &&
             hipStreamSynchronize(c->own) == hipSuccess;
    }
    std::vector<std::tuple<int, int, int, int, int, int>> seen;  // (team, G, threads, b, nwg, K) of applied plans
    for (size_t i = 0; ok && i < cands.size(); ++i) {
        Plan Q = P;
        if (apply_tile(c, Q, cands[i], batched)) continue;
        auto sig = std::make_tuple(Q.team, Q.job.G, Q.threads, Q.job.b, Q.ts.nwg, Q.K);
        if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
        seen.push_back(sig);
        const double us = time_tile(c, P, cands[i], batched, tb, o_src, o_A, o_V, o_cnt, cnt_bytes, o_jobs, o_tj, o_tk,
                                    ntasks, e0, e1);
        if (getenv("TSVDMI_TUNE_LOG"))
            fprintf(stderr,
                    "tsvdmi tune prec %d m %d p %d n3 %lld v %d: team %d G %d W %d threads %d K %d slots %d grid %d: "
                    "%.1f us\n",
                    P.prec, P.m, P.p, (long long)P.n3, P.with_v, cands[i].team, cands[i].G, cands[i].W, Q.threads,
                    cands[i].K, cands[i].slots, Q.ts.nwg, us);
        // a later candidate must be 2% faster to replace an earlier one, so that
        // near-ties resolve the same way from run to run
        if (us > 0.0 && (best_us < 0.0 || us < 0.98 * best_us)) {
            best_us = us;
            best = cands[i];
        }
    }
    (void)hipStreamSynchronize(c->own);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(tb);
    (void)hipGetLastError();
    c->err.clear();
    if (best_us < 0.0) return -1;
    best.source = 1;
    *out = best;
    *us_out = best_us;
    return TSVD_OK;
}

// The tile of a plan: forced by options, cached, autotuned, or the default.
int pick_tile(tsvd_ctx* c, const Plan& P, bool batched, hipStream_t s, Tile* t) {
    if (c->gram == 1 && !batched) {
        *t = gram_tile(P, c->team_size);
        t->source = 2;
        return TSVD_OK;
    }
    if (c->team_size > 0 || c->group_lanes > 0 || c->group_cols > 0 || c->team_slots > 0) {
        *t = default_tile(P, c->team_size, c->group_lanes, c->group_cols, batched);
        if (t->team == 1 && !batched) t->slots = c->team_slots;
        t->source = 2;
        return TSVD_OK;
    }
    const TileKey key(batched ? 1 : 0, P.prec, P.m, P.p, batched ? 0 : (int)P.n3, P.with_v);
    if (tile_cache_get(key, t)) return TSVD_OK;
    *t = default_tile(P, 0, 0, 0, batched);
    if (!c->autotune || c->noalloc) return TSVD_OK;  // tuning allocates its test data
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return TSVD_OK;  // no timing inside a capture: default tile, not cached
    }
    Tile tuned;
    double us = 0.0;
    if (tune_tile(c, P, batched, &tuned, &us) == TSVD_OK) {
        tile_cache_put(key, tuned, us);
        *t = tuned;
    } else {
        tile_cache_put(key, *t, 0.0);  // one candidate, or tuning failed: remember the default
    }
    return TSVD_OK;
}

int make_plan(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, int with_v, Plan& P, Carve& cv,
              hipStream_t s, bool batched = false) {
    P.prec = prec;
    P.n1 = n1; P.n2 = n2; P.n3 = n3; P.N = n1 * n2;
    P.trans = n1 < n2;
    P.m = (int)std::max(n1, n2);
    P.p = (int)std::min(n1, n2);
    P.with_v = with_v;
    if (P.m > kMaxRows) return fail(c, TSVD_EINVAL, "frontal slices larger than 512 rows/columns are not supported");
    const size_t es = esize(prec);
    const size_t slice = (size_t)n1 * n2;
    Tile t;
    int rc = pick_tile(c, P, batched, s, &t);
    if (rc) return rc;
    if ((rc = apply_tile(c, P, t, batched))) return rc;
    P.tile_source = t.source;
    P.tile_W = t.W;
    P.o_zbar = cv.take(slice * n3 * es);
    P.o_A = cv.take((size_t)P.m * P.p * n3 * es);
    P.o_F = cv.take((size_t)P.m * P.p * n3 * es);
    P.o_G = cv.take((size_t)P.p * P.p * n3 * es);
    P.o_w = cv.take((size_t)P.p * n3 * 8);
    P.o_sig = cv.take((size_t)P.p * n3 * 8);
    P.o_ybar = cv.take(slice * n3 * es);
    P.o_V = with_v ? cv.take((size_t)P.p * P.p * n3 * es) : 0;
    P.o_ctr_begin = cv.off;
    P.o_rot = cv.take((size_t)n3 * kRotStride * 4);
    P.o_sw = cv.take((size_t)n3 * 4);
    P.o_bar = cv.take((size_t)(kTeamCtlInts + (size_t)std::max(1, P.ts.nwg) * (1 + std::max(1, P.job.nb))) * 4);
    P.o_rank = cv.take((size_t)n3 * 4);
    P.o_pos = cv.take((size_t)n3 * P.p * 4);
    P.o_ctr_end = cv.off;
    P.o_end = cv.off;
    return TSVD_OK;
}

// Kept-column Jacobi for a t-SVT (cold SVDs, or the completion's warm-started
// ones carrying V): the team kernel with one column per lane group iterates
// only on the pairs that touch a column above the threshold (a slice without
// a gap below it turns into the full iteration), the threshold certificate
// checks each slice, and the full iteration runs for the slices it rejects.  Adds the mode's counters to
// the plan's zeroed region (right after the others) and its buffers after
// them.  Leaves the plan unchanged when the option is off or the tile is
// another kernel.
void plan_kept_columns(tsvd_ctx* c, Plan& P, Carve& cv) {
    P.keep = 0;
    if (!c->kept_cols || c->noalloc || P.team != 1 || P.K != 1 || P.m > kMaxRows) return;
    if (P.o_ctr_end != cv.off) return;  // the zeroed region must stay contiguous
    const size_t n3 = (size_t)P.n3, m = (size_t)P.m, p = (size_t)P.p;
    P.o_full = cv.take(n3 * 4);
    P.o_sums = cv.take(n3 * 8);
    P.o_done = cv.take(n3 * 4);
    P.o_rot2 = cv.take(n3 * kRotStride * 4);
    P.o_bar2 = cv.take((size_t)(kTeamCtlInts + (size_t)std::max(1, P.ts.nwg) * (1 + std::max(1, P.job.nb))) * 4);
    P.o_ctr_end = cv.off;
    P.o_flags = cv.take(n3 * 4);
    P.o_ncols = cv.take(n3 * 4);
    P.o_nrm2 = cv.take(n3 * p * 8);
    P.o_As = cv.take(n3 * m * p * 4);
    P.o_H = cv.take(n3 * p * p * 4);
    P.o_H2 = cv.take(n3 * p * p * 4);
    P.o_end = cv.off;
    P.keep = 1;
}

// Point the plan's Jacobi descriptor at its workspace regions.
void bind_plan(Plan& P, char* base) {
    JacobiJob& J = P.job;
    J.src = base + P.o_zbar;
    J.A = base + P.o_A;
    J.V = P.with_v ? (void*)(base + P.o_V) : nullptr;
    J.rot = (int*)(base + P.o_rot);
    J.sweeps = (int*)(base + P.o_sw);
    J.src_ss = P.N;
    if (!P.trans) { J.src_rs = 1; J.src_cs = P.n1; }
    else { J.src_rs = P.n1; J.src_cs = 1; }
    J.m = P.m;
    J.p = P.p;
    J.n3 = (int)P.n3;
    J.refine64 = (P.prec == TSVD_MIXED) ? 1 : 0;
    const double u64 = ldexp(1.0, -53), u32 = ldexp(1.0, -24);
    J.tol = P.prec == TSVD_FP64 ? P.m * u64 : P.prec == TSVD_FP32 ? 2.0 * sqrt((double)P.m) * u32 : P.m * u32;
    // A sweep whose cosines are all <= sqrt(tol) / 64 leaves the next one rotating by ~tol / 4096
    // (quadratic convergence), below the rotation threshold: the sweep that would only confirm it
    // is skipped.  MIXED hands over to its FP64 sweep once the FP32 sweeps are at cosines <= 1e-2:
    // that sweep starts from ~1e-4 and ends near 1e-8, below the FP32 rounding of the stored columns.
    J.skip2 = P.prec == TSVD_MIXED ? 1e-4 : J.tol / 4096.0;
    P.ts.ctl = (int*)(base + P.o_bar);
}

int upload_plan(tsvd_ctx* c, Plan& P, char* base) {
    (void)c;
    bind_plan(P, base);
    return TSVD_OK;
}

int clamp_sweeps(int v) { return std::max(1, std::min(v, kMaxSweeps - 1)); }

// Jacobi launch for a planned tensor.
int run_jacobi(tsvd_ctx* c, Plan& P, char* base, Ctrl* ctrl, hipStream_t s) {
    (void)base;
    hipError_t e;
    if (!P.team)
        e = launch_jacobi_resident(P.prec, P.job, nullptr, nullptr, nullptr, (int)P.n3, clamp_sweeps(c->max_sweeps),
                                   ctrl, P.lds, P.threads, P.with_v, s);
    else if (P.team == 2)
        e = launch_jacobi_gram(P.prec, P.job, (int)P.n3, P.ts, clamp_sweeps(c->max_sweeps), ctrl, P.with_v,
                               c->spin_limit, (c->capturing || !c->coop) ? 0 : 1, s);
    else
        e = launch_jacobi_team(P.prec, P.job, (int)P.n3, P.ts, clamp_sweeps(c->max_sweeps), ctrl, P.lds, P.threads,
                               P.with_v, c->spin_limit, P.job.R, P.job.G, P.K, (c->capturing || !c->coop) ? 0 : 1, s);
    if (e != hipSuccess) return hip_fail(c, e, "jacobi launch");
    return TSVD_OK;
}

// Everything after the forward transform of the t-SVT: Jacobi, thresholding,
// rebuild.  Leaves Ybar in the workspace.
int enqueue_after_jacobi(tsvd_ctx* c, Plan& P, char* base, Ctrl* ctrl, double tau_val, const double* tau_sched,
                         hipStream_t s);

int enqueue_warm_start(tsvd_ctx* c, Plan& P, char* base, Ctrl* ctrl, hipStream_t s);

// Threshold certificate after the kept-column iteration, then the full
// iteration (in place, from A') for the slices it rejects; the others are
// left alone by that launch.
int enqueue_certificate(tsvd_ctx* c, Plan& P, char* base, Ctrl* ctrl, double tau, const double* tau_sched,
                        hipStream_t s) {
    const int prec = P.prec == TSVD_FP64 ? 0 : 1;
    CertArgs a{};
    a.A = base + P.o_A;
    a.m = P.m; a.p = P.p; a.n3 = (int)P.n3;
    a.tau = tau;
    a.tau_sched = tau_sched;
    a.nrm2 = (double*)(base + P.o_nrm2);
    a.As = (float*)(base + P.o_As);
    a.H = (float*)(base + P.o_H);
    a.H2 = (float*)(base + P.o_H2);
    a.sums = (double*)(base + P.o_sums);
    a.done = (int*)(base + P.o_done);
    a.sweeps = P.job.sweeps;
    a.full = (const int*)(base + P.o_full);
    a.ncols = (int*)(base + P.o_ncols);
    a.flags = (int*)(base + P.o_flags);
    a.ctrl = ctrl;
    hipError_t e = launch_threshold_certificate(prec, a, s);
    if (e != hipSuccess) return hip_fail(c, e, "threshold certificate");
    JacobiJob J = P.job;
    J.keep = 0;
    J.keep2 = 0.0;
    J.skip = a.flags;
    J.src = base + P.o_A;
    J.src_ss = (int64_t)P.m * P.p;
    J.src_rs = 1;
    J.src_cs = P.m;
    J.rot = (int*)(base + P.o_rot2);
    if (P.with_v) J.vinit = 1;  // V continues from where the kept-column iteration left it
    TeamSched ts = P.ts;
    ts.ctl = (int*)(base + P.o_bar2);
    e = launch_jacobi_team(P.prec, J, (int)P.n3, ts, clamp_sweeps(c->max_sweeps), ctrl, P.lds, P.threads, P.with_v,
                           c->spin_limit, J.R, J.G, 1, (c->capturing || !c->coop) ? 0 : 1, s);
    if (e != hipSuccess) return hip_fail(c, e, "jacobi launch");
    return TSVD_OK;
}

int enqueue_svt_core(tsvd_ctx* c, Plan& P, char* base, Ctrl* ctrl, double tau_val, const double* tau_sched,
                     hipStream_t s) {
    if (P.warm) {
        PhaseMark pm(c, 4, s);
        int rc = enqueue_warm_start(c, P, base, ctrl, s);
        if (rc) return rc;
    }
    // the kept-column mode takes tau > 0 from the host or a schedule on the device
    // (the completion's entries are checked > 0 on the host)
    const bool keep = P.keep && (tau_sched || (tau_val > 0.0 && isfinite(tau_val)));
    P.job.keep = keep ? 1 : 0;
    P.job.keep2 = keep && !tau_sched ? tau_val * tau_val : 0.0;
    P.job.keep_sched = keep ? tau_sched : nullptr;
    P.job.skip = nullptr;
    P.job.full = keep ? (int*)(base + P.o_full) : nullptr;
    {
        PhaseMark pm(c, 1, s);
        int rc = run_jacobi(c, P, base, ctrl, s);
        if (rc) return rc;
    }
    if (keep) {
        PhaseMark pm(c, 5, s);
        int rc = enqueue_certificate(c, P, base, ctrl, tau_val, tau_sched, s);
        if (rc) return rc;
    }
    return enqueue_after_jacobi(c, P, base, ctrl, tau_val, tau_sched, s);
}

// Warm start (completion only): V of every slice is kept from the previous
// iteration (reset to the identity every warm_period iterations, 64 by
// default, which bounds the drift of V from orthogonality) and the
// Jacobi input is A0 = Zbar_k V_k, whose one-sided Jacobi ends at Zbar_k V_k J
// with V_k J the new V: the singular vectors change little between
// iterations, so A0 is nearly orthogonal already and few sweeps are needed.
int enqueue_warm_gemm(tsvd_ctx* c, Plan& P, char* base, const void* V, hipStream_t s) {
    const int prec = P.prec == TSVD_FP64 ? 0 : 1;
    GemmArgs g{};
    g.A = base + P.o_zbar;  // tall view of the slice
    if (!P.trans) { g.a_rs = 1; g.a_cs = P.n1; } else { g.a_rs = P.n1; g.a_cs = 1; }
    g.a_bs = P.N;
    g.B = V; g.b_rs = 1; g.b_cs = P.p; g.b_bs = (int64_t)P.p * P.p;
    g.C = base + P.o_A0; g.c_rs = 1; g.c_cs = P.m; g.c_bs = (int64_t)P.m * P.p;
    g.cscale = nullptr;
    g.M = P.m; g.Nn = P.p; g.K = P.p; g.Kdev = nullptr; g.Ndev = nullptr;
    g.batch = (int)P.n3;
    const hipError_t e = launch_gemm(prec, g, s);
    if (e != hipSuccess) return hip_fail(c, e, "warm start gemm");
    return TSVD_OK;
}

int enqueue_warm_start(tsvd_ctx* c, Plan& P, char* base, Ctrl* ctrl, hipStream_t s) {
    const int prec = P.prec == TSVD_FP64 ? 0 : 1;
    const hipError_t e = launch_warm_reset(prec, base + P.o_V, P.p, (int)P.n3, ctrl, P.warm_period, s);
    if (e != hipSuccess) return hip_fail(c, e, "warm reset");
    return enqueue_warm_gemm(c, P, base, base + P.o_V, s);
}

// Thresholding and rebuild (Ybar in the workspace) once A' is ready.
int enqueue_after_jacobi(tsvd_ctx* c, Plan& P, char* base, Ctrl* ctrl, double tau_val, const double* tau_sched,
                         hipStream_t s) {
    PhaseMark pm(c, 2, s);
    const int prec = P.prec == TSVD_FP64 ? 0 : 1;
    SvtPrepArgs sp{};
    sp.A = base + P.o_A; sp.m = P.m; sp.p = P.p; sp.a_ss = (int64_t)P.m * P.p;
    sp.F = base + P.o_F; sp.f_ss = (int64_t)P.m * P.p;
    sp.w = (double*)(base + P.o_w); sp.w_ss = P.p;
    sp.sig = (double*)(base + P.o_sig); sp.sig_ss = P.p;
    sp.ranks = (int*)(base + P.o_rank);
    sp.pos = (int*)(base + P.o_pos);
    sp.n3 = (int)P.n3;
    sp.tau_val = tau_val; sp.tau_sched = tau_sched; sp.ctrl = ctrl;
    hipError_t e = launch_svt_prep(prec, sp, s);
    if (e != hipSuccess) return hip_fail(c, e, "svt_prep");
    // G_k (p x r_k) = Zt_k (p x m) F_k (m x r_k) diag(w_k)
    GemmArgs g{};
    g.A = base + P.o_zbar;
    if (!P.trans) { g.a_rs = P.n1; g.a_cs = 1; } else { g.a_rs = 1; g.a_cs = P.n1; }
    g.a_bs = P.N;
    g.B = base + P.o_F; g.b_rs = 1; g.b_cs = P.m; g.b_bs = (int64_t)P.m * P.p;
    g.C = base + P.o_G; g.c_rs = 1; g.c_cs = P.p; g.c_bs = (int64_t)P.p * P.p;
    g.cscale = (const double*)(base + P.o_w); g.s_bs = P.p;
    g.M = P.p; g.Nn = P.p; g.K = P.m; g.Kdev = nullptr; g.Ndev = (const int*)(base + P.o_rank);
    g.batch = (int)P.n3;
    e = launch_gemm(prec, g, s);
    if (e != hipSuccess) return hip_fail(c, e, "svt factor gemm");
    // Ybar_k (n1 x n2) = L (n1 x r) R^T (r x n2)
    GemmArgs r{};
    if (!P.trans) {
        r.A = base + P.o_F; r.a_rs = 1; r.a_cs = P.m; r.a_bs = (int64_t)P.m * P.p;
        r.B = base + P.o_G; r.b_rs = P.p; r.b_cs = 1; r.b_bs = (int64_t)P.p * P.p;
    } else {
        r.A = base + P.o_G; r.a_rs = 1; r.a_cs = P.p; r.a_bs = (int64_t)P.p * P.p;
        r.B = base + P.o_F; r.b_rs = P.m; r.b_cs = 1; r.b_bs = (int64_t)P.m * P.p;
    }
    r.C = base + P.o_ybar; r.c_rs = 1; r.c_cs = P.n1; r.c_bs = P.N;
    r.cscale = nullptr;
    r.M = (int)P.n1; r.Nn = (int)P.n2; r.K = 0; r.Kdev = (const int*)(base + P.o_rank); r.Ndev = nullptr;
    r.batch = (int)P.n3;
    e = launch_gemm(prec, r, s);
    if (e != hipSuccess) return hip_fail(c, e, "svt rebuild gemm");
    return TSVD_OK;
}

bool bad_prec(int prec) { return prec != TSVD_FP64 && prec != TSVD_FP32 && prec != TSVD_MIXED; }

int finish_call(tsvd_ctx* c, hipStream_t s) {
    if (!c->sync_status) return TSVD_OK;
    return read_status(c, s, nullptr);
}

int tsvt_check(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, const void* Z, const void* Y,
               double tau) {
    if (bad_prec(prec)) return fail(c, TSVD_EINVAL, "unknown precision");
    if (n1 <= 0 || n2 <= 0 || n3 <= 0) return fail(c, TSVD_EINVAL, "sizes must be positive");
    if (!Z || !Y) return fail(c, TSVD_EINVAL, "null tensor pointer");
    if (!(tau >= 0.0) || !isfinite(tau)) return fail(c, TSVD_EINVAL, "tau must be finite and >= 0");
    return TSVD_OK;
}

// One t-SVT (Theorem 5) of a planned tensor on the workspace at `base`.  The
// transform operands are fwd / inv, or (nullptr) the context's cached copies.
int tsvt_enqueue(tsvd_ctx* c, Plan& P, char* base, const void* fwd, const void* inv, const void* Z, void* Y,
                 double tau, int32_t* ranks_out, hipStream_t s) {
    int rc;
    if ((rc = upload_plan(c, P, base))) return rc;
    CtrlRegion cr;
    if ((rc = ensure_ctrl(c, &cr))) return rc;
    hipError_t e = launch_fill_zero(base + P.o_ctr_begin, P.o_ctr_end - P.o_ctr_begin, s);
    if (e != hipSuccess) return hip_fail(c, e, "fill");
    TubeArgs f{};
    f.in = Z; f.out = base + P.o_zbar; f.N = P.N; f.n3 = (int)P.n3; f.ctrl = cr.ctrl; f.check_finite = 1;
    f.beta_val = 1.0;
    {
        PhaseMark pm(c, 0, s);
        rc = fwd ? run_tube_mat(c, P.prec, f, 0, fwd, s) : run_tube(c, P.prec, f, 0, s);
        if (rc) return rc;
    }
    if ((rc = enqueue_svt_core(c, P, base, cr.ctrl, tau, nullptr, s))) return rc;
    TubeArgs iv{};
    iv.in = base + P.o_ybar; iv.out = Y; iv.N = P.N; iv.n3 = (int)P.n3; iv.ctrl = cr.ctrl; iv.beta_val = 1.0;
    {
        PhaseMark pm(c, 3, s);
        rc = inv ? run_tube_mat(c, P.prec, iv, 1, inv, s) : run_tube(c, P.prec, iv, 1, s);
        if (rc) return rc;
    }
    if (ranks_out) {
        HIPCHK(c, hipMemcpyAsync(ranks_out, base + P.o_rank, P.n3 * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return read_status(c, s, nullptr);
    }
    return finish_call(c, s);
}


// ---------------------------------------------------------------------------
// Caller-given transforms along the tubes (the concluding remarks' other
// transforms) and the real Fourier transform of the DFT path.
// ---------------------------------------------------------------------------

// Inverse of a row-major n x n matrix by Gauss-Jordan elimination with
// partial pivoting, in FP64 on the host.  False when a pivot is zero or not
// finite (singular or non-finite matrix).
bool invert_host(int n, const double* L, std::vector<double>& inv) {
    std::vector<double> a(L, L + (size_t)n * n);
    inv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(a[(size_t)r * n + col]) > fabs(a[(size_t)piv * n + col])) piv = r;
        const double pv = a[(size_t)piv * n + col];
        if (!(pv != 0.0) || !isfinite(pv)) return false;
        if (piv != col)
            for (int k = 0; k < n; ++k) {
                std::swap(a[(size_t)piv * n + k], a[(size_t)col * n + k]);
                std::swap(inv[(size_t)piv * n + k], inv[(size_t)col * n + k]);
            }
        const double rp = 1.0 / pv;
        for (int k = 0; k < n; ++k) {
            a[(size_t)col * n + k] *= rp;
            inv[(size_t)col * n + k] *= rp;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = a[(size_t)r * n + col];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                a[(size_t)r * n + k] -= f * a[(size_t)col * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)col * n + k];
            }
        }
    }
    for (double v : inv)
        if (!isfinite(v)) return false;
    return true;
}

// Real form of the unnormalized DFT along a tube of length n (rows = slots):
// slot 0 the DC term sum_t x_t; for f = 1..h (h = (n-1)/2) slot 2f-1 the
// real part sum_t x_t cos(2 pi f t / n) and slot 2f the imaginary part
// -sum_t x_t sin(2 pi f t / n); for even n slot n-1 the Nyquist term
// sum_t (-1)^t x_t.  Its inverse follows from x_t = (1/n) sum_f Xt_f
// e^{2 pi i f t / n} with conjugate pairs combined.  Angles are reduced
// (f t mod n) in integers.
void real_dft_matrices(int n, std::vector<double>& R, std::vector<double>& Ri) {
    R.assign((size_t)n * n, 0.0);
    Ri.assign((size_t)n * n, 0.0);
    const double pi = acos(-1.0);
    const int h = (n - 1) / 2;
    for (int t = 0; t < n; ++t) {
        R[(size_t)0 * n + t] = 1.0;
        Ri[(size_t)t * n + 0] = 1.0 / n;
        for (int f = 1; f <= h; ++f) {
            const double a = 2.0 * pi * (double)(((int64_t)f * t) % n) / (double)n;
            R[(size_t)(2 * f - 1) * n + t] = cos(a);
            R[(size_t)(2 * f) * n + t] = -sin(a);
            Ri[(size_t)t * n + (2 * f - 1)] = 2.0 * cos(a) / n;
            Ri[(size_t)t * n + (2 * f)] = -2.0 * sin(a) / n;
        }
        if (n % 2 == 0) {
            const double sg = (t % 2) ? -1.0 : 1.0;
            R[(size_t)(n - 1) * n + t] = sg;
            Ri[(size_t)t * n + (n - 1)] = sg / n;
        }
    }
}

// Device operands (forward L, inverse Li) of a caller-given transform in the
// form run_tube_mat takes, kept in the context and rebuilt only when L or the
// engine changes.  Rebuilding waits for the stream (earlier calls may still
// read the old operands).
int get_custom_operands(tsvd_ctx* c, int prec, int n3, const double* L, const double* Li, hipStream_t s,
                        const void** fwd, const void** inv) {
    const int eng = tube_engine(prec);
    const size_t nn = (size_t)n3 * n3;
    const size_t one = align256(tube_matrix_bytes(eng, n3));
    const bool same = c->xf_eng == eng && c->xf_key.size() == nn && memcmp(c->xf_key.data(), L, nn * 8) == 0;
    if (!same) {
        std::vector<unsigned char> h(2 * one, 0);
        if (n3 <= kMaxTube) {
            make_tube_fragments(eng, n3, L, h.data());
            make_tube_fragments(eng, n3, Li, h.data() + one);
        } else {
            for (size_t e = 0; e < nn; ++e) {
                if (prec == TSVD_FP64) {
                    ((double*)h.data())[e] = L[e];
                    ((double*)(h.data() + one))[e] = Li[e];
                } else {
                    ((float*)h.data())[e] = (float)L[e];
                    ((float*)(h.data() + one))[e] = (float)Li[e];
                }
            }
        }
        HIPCHK(c, hipStreamSynchronize(s));
        if (c->xf.bytes < 2 * one) {
            if (c->xf.p) HIPCHK(c, hipFree(c->xf.p));
            c->xf.p = nullptr;
            c->xf.bytes = 0;
            HIPCHK(c, hipMalloc(&c->xf.p, 2 * one));
            c->xf.bytes = 2 * one;
        }
        HIPCHK(c, hipMemcpy(c->xf.p, h.data(), 2 * one, hipMemcpyHostToDevice));
        c->xf_key.assign(L, L + nn);
        c->xf_eng = eng;
    }
    *fwd = c->xf.p;
    *inv = (const char*)c->xf.p + one;
    return TSVD_OK;
}

// Slots of the real Fourier transform: h complex frequencies, nreal real ones.
void dft_layout(int64_t n3, int* h, int* nreal) {
    *h = (int)((n3 - 1) / 2);
    *nreal = (n3 % 2 == 0) ? 2 : 1;
}

// Singular values of every slice of a planned tensor after its Jacobi launch
// (per column, unsorted) summed on the host; synchronizes `s`.
int sum_sigma(tsvd_ctx* c, Plan& P, char* base, Ctrl* ctrl, hipStream_t s, double* out) {
    const int dp = P.prec == TSVD_FP64 ? 0 : 1;
    SvtPrepArgs sp{};
    sp.A = base + P.o_A; sp.m = P.m; sp.p = P.p; sp.a_ss = (int64_t)P.m * P.p;
    sp.F = base + P.o_F; sp.f_ss = (int64_t)P.m * P.p;
    sp.w = (double*)(base + P.o_w); sp.w_ss = P.p;
    sp.sig = (double*)(base + P.o_sig); sp.sig_ss = P.p;
    sp.ranks = (int*)(base + P.o_rank); sp.pos = (int*)(base + P.o_pos); sp.n3 = (int)P.n3; sp.tau_val = 0.0;
    sp.ctrl = ctrl;
    hipError_t e = launch_svt_prep(dp, sp, s);
    if (e != hipSuccess) return hip_fail(c, e, "singular values");
    std::vector<double> h((size_t)P.p * P.n3);
    HIPCHK(c, hipMemcpyAsync(h.data(), base + P.o_sig, h.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    double acc = 0.0;
    for (double v : h) acc += v;
    *out = acc;
    return TSVD_OK;
}

// The DFT path's plans and workspace: the real-transform slots (N elements)
// at o_zb, then the plan of the h complex slices in real form (2 n1 x 2 n2)
// and the plan of the real slices.
struct DftPlan {
    int h = 0, nreal = 0;
    size_t o_zb = 0;
    Plan E, R;
};

// kept: a t-SVT (the kept-column Jacobi where its tile allows; a TNN needs
// every singular value).
int make_dft_plan(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, DftPlan& D, Carve& cv, hipStream_t s,
                  bool kept = false) {
    if (2 * std::max(n1, n2) > kMaxRows)
        return fail(c, TSVD_EINVAL, "the DFT path takes frontal slices of at most 256 rows and columns");
    dft_layout(n3, &D.h, &D.nreal);
    D.o_zb = cv.take((size_t)n1 * n2 * n3 * esize(prec));
    int rc;
    if (D.h > 0) {
        if ((rc = make_plan(c, prec, 2 * n1, 2 * n2, D.h, 0, D.E, cv, s))) return rc;
        if (kept) plan_kept_columns(c, D.E, cv);
    }
    if ((rc = make_plan(c, prec, n1, n2, D.nreal, 0, D.R, cv, s))) return rc;
    if (kept) plan_kept_columns(c, D.R, cv);
    return TSVD_OK;
}

// Forward real DFT of X into the slots and the real forms of its slices in
// the two plans' inputs; Jacobi-ready.
int dft_forward(tsvd_ctx* c, DftPlan& D, int prec, int64_t n1, int64_t n2, int64_t n3, const void* X,
                const void* fwd, char* base, Ctrl* ctrl, hipStream_t s) {
    int rc;
    if (D.h > 0 && (rc = upload_plan(c, D.E, base))) return rc;
    if ((rc = upload_plan(c, D.R, base))) return rc;
    hipError_t e = hipSuccess;
    if (D.h > 0) e = launch_fill_zero(base + D.E.o_ctr_begin, D.E.o_ctr_end - D.E.o_ctr_begin, s);
    if (e == hipSuccess) e = launch_fill_zero(base + D.R.o_ctr_begin, D.R.o_ctr_end - D.R.o_ctr_begin, s);
    if (e != hipSuccess) return hip_fail(c, e, "fill");
    TubeArgs f{};
    f.in = X; f.out = base + D.o_zb; f.N = n1 * n2; f.n3 = (int)n3; f.ctrl = ctrl; f.check_finite = 1;
    f.beta_val = 1.0;
    {
        PhaseMark pm(c, 0, s);
        rc = fwd ? run_tube_mat(c, prec, f, 0, fwd, s) : run_tube_fft(c, prec, f, kFftDftForward, s);
        if (rc) return rc;
    }
    DftEmbedArgs ea{};
    ea.zb = base + D.o_zb;
    ea.E = D.h > 0 ? (void*)(base + D.E.o_zbar) : nullptr;
    ea.R = base + D.R.o_zbar;
    ea.n1 = n1; ea.n2 = n2; ea.n3 = (int)n3; ea.h = D.h; ea.nreal = D.nreal;
    e = launch_dft_embed(prec == TSVD_FP64 ? 0 : 1, ea, s);
    if (e != hipSuccess) return hip_fail(c, e, "dft embed");
    return TSVD_OK;
}

// Device addresses of the scratch array (see its definition above).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices];

// With `device` current: look up the device address of the scratch array.
int scratch_lookup(int device) {
    if (device < 0 || device >= kMaxDevices) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return TSVD_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return TSVD_EHIP;
    }
    g_scratch_ptr[device] = (char*)p;
    return TSVD_OK;
}

int scratch_of(tsvd_ctx* c, char** out) {
    if (scratch_lookup(c->device) != TSVD_OK)
        return fail(c, TSVD_EHIP, "address of the fixed scratch array unavailable on this device");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    *out = g_scratch_ptr[c->device];
    return TSVD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int tsvd_create(tsvd_ctx** out, int device) {
    if (!out) return TSVD_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TSVD_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return TSVD_EHIP;
    auto* c = new tsvd_ctx();
    c->device = device;
    (void)hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device);
    if (const char* v = getenv("TSVDMI_COOPERATIVE")) c->coop = strcmp(v, "1") == 0;
    CtrlRegion cr;
    if (ensure_ctrl(c, &cr) != TSVD_OK) {
        delete c;
        return TSVD_EHIP;
    }
    // device address of the no-allocation scratch on this device (a failure
    // here only disables tsvt_dct_noalloc, which reports it)
    (void)scratch_lookup(device);
    *out = c;
    return TSVD_OK;
}

void tsvd_destroy(tsvd_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : c->dct) {
        (void)hipFree(kv.second.first);
        (void)hipFree(kv.second.second);
    }
    for (auto& kv : c->frag) (void)hipFree(kv.second);
    for (auto& kv : c->fft) (void)hipFree(kv.second);
    if (c->xf.p) (void)hipFree(c->xf.p);
    if (c->ws.p) (void)hipFree(c->ws.p);
    if (c->ctrl.p) (void)hipFree(c->ctrl.p);
    if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
    if (c->own) (void)hipStreamDestroy(c->own);
    for (void* p : c->owned) (void)hipFree(p);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

const char* tsvd_last_error(const tsvd_ctx* c) { return c ? c->err.c_str() : "null context"; }

int tsvd_set_option(tsvd_ctx* c, int opt, double v) {
    if (!c) return TSVD_EINVAL;
    switch (opt) {
        case TSVD_OPT_MAX_SWEEPS:
            if (v < 1 || v > kMaxSweeps - 1) return fail(c, TSVD_EINVAL, "max_sweeps out of range 1..63");
            c->max_sweeps = (int)v;
            return TSVD_OK;
        case TSVD_OPT_SYNC_STATUS: c->sync_status = v != 0.0; return TSVD_OK;
        case TSVD_OPT_TEAM_SIZE:
            if (v < 0 || v > 64) return fail(c, TSVD_EINVAL, "team size out of range 0..64");
            c->team_size = (int)v;
            return TSVD_OK;
        case TSVD_OPT_SPIN_LIMIT:
            if (v < 1 || v > 1e9) return fail(c, TSVD_EINVAL, "spin limit out of range");
            c->spin_limit = (int)v;
            return TSVD_OK;
        case TSVD_OPT_PROFILE:
            if (v != 0.0 && v != 1.0 && v != 2.0) return fail(c, TSVD_EINVAL, "profile level is 0, 1 or 2");
            c->prof = (int)v;
            return TSVD_OK;
        case TSVD_OPT_GRAPHS: c->use_graphs = v != 0.0; return TSVD_OK;
        case TSVD_OPT_AUTOTUNE: c->autotune = v != 0.0; return TSVD_OK;
        case TSVD_OPT_GROUP_COLUMNS:
            if (v != 0 && v != 1 && v != 2) return fail(c, TSVD_EINVAL, "group columns must be 0, 1 or 2");
            c->group_cols = (int)v;
            return TSVD_OK;
        case TSVD_OPT_WARM_START:
            if (v < -1 || v > 1e6) return fail(c, TSVD_EINVAL, "warm start must be -1, 0 or a period >= 1");
            c->warm_start = (int)v;
            return TSVD_OK;
        case TSVD_OPT_GROUP_LANES:
            if (v != 0 && v != 16 && v != 32 && v != 64) return fail(c, TSVD_EINVAL, "group lanes must be 0, 16, 32 or 64");
            c->group_lanes = (int)v;
            return TSVD_OK;
        case TSVD_OPT_COOPERATIVE: c->coop = v != 0.0; return TSVD_OK;
        case TSVD_OPT_LONG_TUBES:
            if (v != 0.0 && v != 1.0) return fail(c, TSVD_EINVAL, "long-tube kernel must be 0 or 1");
            c->dense_long = (int)v;
            return TSVD_OK;
        case TSVD_OPT_GRAM:
            if (v != -1 && v != 0 && v != 1) return fail(c, TSVD_EINVAL, "gram option is -1, 0 or 1");
            c->gram = (int)v;
            return TSVD_OK;
        case TSVD_OPT_TEAM_SLOTS:
            if (v < 0 || v > 64) return fail(c, TSVD_EINVAL, "team slots out of range 0..64");
            c->team_slots = (int)v;
            return TSVD_OK;
        case TSVD_OPT_KEPT_COLUMNS:
            if (v != 0.0 && v != 1.0) return fail(c, TSVD_EINVAL, "kept-column option must be 0 or 1");
            c->kept_cols = (int)v;
            return TSVD_OK;
    }
    return fail(c, TSVD_EINVAL, "unknown option");
}

double tsvd_get_option(const tsvd_ctx* c, int opt) {
    if (!c) return -1.0;
    switch (opt) {
        case TSVD_OPT_MAX_SWEEPS: return c->max_sweeps;
        case TSVD_OPT_SYNC_STATUS: return c->sync_status;
        case TSVD_OPT_TEAM_SIZE: return c->team_size;
        case TSVD_OPT_SPIN_LIMIT: return c->spin_limit;
        case TSVD_OPT_PROFILE: return c->prof;
        case TSVD_OPT_GRAPHS: return c->use_graphs;
        case TSVD_OPT_AUTOTUNE: return c->autotune;
        case TSVD_OPT_GROUP_COLUMNS: return c->group_cols;
        case TSVD_OPT_WARM_START: return c->warm_start;
        case TSVD_OPT_GROUP_LANES: return c->group_lanes;
        case TSVD_OPT_TEAM_SLOTS: return c->team_slots;
        case TSVD_OPT_COOPERATIVE: return c->coop;
        case TSVD_OPT_GRAM: return c->gram;
        case TSVD_OPT_LONG_TUBES: return c->dense_long;
        case TSVD_OPT_KEPT_COLUMNS: return c->kept_cols;
    }
    return -1.0;
}

int tsvd_get_tile(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, int batched, int with_v,
                  int32_t* out) {
    if (!c || !out) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (bad_prec(prec)) return fail(c, TSVD_EINVAL, "unknown precision");
    if (n1 <= 0 || n2 <= 0 || n3 <= 0) return fail(c, TSVD_EINVAL, "sizes must be positive");
    HIPCHK(c, hipSetDevice(c->device));
    Plan P;
    Carve cv;
    int rc = make_plan(c, prec, n1, n2, n3, with_v ? 1 : 0, P, cv, nullptr, batched != 0);
    if (rc) return rc;
    out[0] = P.team;
    out[1] = P.job.G;
    out[2] = P.team ? P.ts.W : 0;
    out[3] = P.threads;
    out[4] = P.tile_source;
    out[5] = P.team ? P.K : 0;
    return TSVD_OK;
}

int tsvd_sync_status(tsvd_ctx* c, void* stream, int* max_sweeps_out) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    HIPCHK(c, hipSetDevice(c->device));
    return read_status(c, (hipStream_t)stream, max_sweeps_out);
}

int tsvd_get_stats(tsvd_ctx* c, void* stream, tsvd_stats* out, int reset) {
    if (!c || !out) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    HIPCHK(c, hipSetDevice(c->device));
    CtrlRegion cr;
    int rc = ensure_ctrl(c, &cr);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    HIPCHK(c, hipDeviceSynchronize());
    memset(out, 0, sizeof(*out));
    for (auto& mk : c->marks) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, std::get<1>(mk), std::get<2>(mk)));
        out->ms[std::get<0>(mk)] += ms;
        out->launches[std::get<0>(mk)] += 1;
    }
    Ctrl h;
    HIPCHK(c, hipMemcpy(&h, cr.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    out->slice_sweeps = (int64_t)h.slice_sweeps;
    out->pairs = (int64_t)h.pairs;
    out->fallback_slices = h.fallback;
    if (reset) {
        c->marks.clear();
        c->ev_used = 0;
        h.slice_sweeps = 0;
        h.pairs = 0;
        h.fallback = 0;
        HIPCHK(c, hipMemcpy(cr.ctrl, &h, sizeof(Ctrl), hipMemcpyHostToDevice));
    }
    return TSVD_OK;
}

int tsvt_dct(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, const void* Z, void* Y, double tau,
             int32_t* ranks_out, void* stream) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    int rc = tsvt_check(c, prec, n1, n2, n3, Z, Y, tau);
    if (rc) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Plan P;
    Carve cv;
    if ((rc = make_plan(c, prec, n1, n2, n3, 0, P, cv, s))) return rc;
    plan_kept_columns(c, P, cv);
    if ((rc = ensure_ws(c, P.o_end))) return rc;
    return tsvt_enqueue(c, P, (char*)c->ws.p, nullptr, nullptr, Z, Y, tau, ranks_out, s);
}

int tsvt_dct_noalloc(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, const void* Z, void* Y,
                     double tau, int32_t* ranks_out, void* stream) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    int rc = tsvt_check(c, prec, n1, n2, n3, Z, Y, tau);
    if (rc) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    char* sp = nullptr;
    if ((rc = scratch_of(c, &sp))) return rc;
    hipStream_t s = (hipStream_t)stream;
    // the call's layout in the scratch array: forward and inverse transform
    // operands, then the workspace of the plan
    const int eng = tube_engine(prec);
    Carve cv;
    const size_t o_fwd = cv.take(tube_matrix_bytes(eng, (int)n3));
    const size_t o_inv = cv.take(tube_matrix_bytes(eng, (int)n3));
    const size_t o_ws = cv.off;
    Plan P;
    Carve wv;
    c->noalloc = 1;  // make_plan: the cached or default tile, no tuning
    rc = make_plan(c, prec, n1, n2, n3, 0, P, wv, s);
    if (rc) {
        c->noalloc = 0;
        return rc;
    }
    if (o_ws + P.o_end > kScratchBytes) {
        c->noalloc = 0;
        return fail(c, TSVD_EINVAL, "tsvt_dct_noalloc: the tensor needs " + std::to_string(o_ws + P.o_end) +
                                        " bytes of scratch; the fixed scratch holds " +
                                        std::to_string(kScratchBytes));
    }
    hipError_t e = launch_tube_matrix(eng, (int)n3, 0, sp + o_fwd, s);
    if (e == hipSuccess) e = launch_tube_matrix(eng, (int)n3, 1, sp + o_inv, s);
    if (e != hipSuccess) {
        c->noalloc = 0;
        return hip_fail(c, e, "transform matrix");
    }
    rc = tsvt_enqueue(c, P, sp + o_ws, sp + o_fwd, sp + o_inv, Z, Y, tau, ranks_out, s);
    c->noalloc = 0;
    return rc;
}


int tsvt_transform(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, const double* L, const void* Z,
                   void* Y, double tau, int32_t* ranks_out, void* stream) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    int rc = tsvt_check(c, prec, n1, n2, n3, Z, Y, tau);
    if (rc) return rc;
    if (!L) return fail(c, TSVD_EINVAL, "null transform matrix");
    std::vector<double> Li;
    if (!invert_host((int)n3, L, Li)) return fail(c, TSVD_EINVAL, "transform matrix is singular or not finite");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const void *fwd, *inv;
    if ((rc = get_custom_operands(c, prec, (int)n3, L, Li.data(), s, &fwd, &inv))) return rc;
    Plan P;
    Carve cv;
    if ((rc = make_plan(c, prec, n1, n2, n3, 0, P, cv, s))) return rc;
    plan_kept_columns(c, P, cv);
    if ((rc = ensure_ws(c, P.o_end))) return rc;
    return tsvt_enqueue(c, P, (char*)c->ws.p, fwd, inv, Z, Y, tau, ranks_out, s);
}

int tsvt_dft(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, const void* Z, void* Y, double tau,
             int32_t* ranks_out, void* stream) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    int rc = tsvt_check(c, prec, n1, n2, n3, Z, Y, tau);
    if (rc) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const void *fwd = nullptr, *inv = nullptr;  // null: the fast transform (long tubes)
    if (!fft_fits((int)n3)) {
        std::vector<double> R, Ri;
        real_dft_matrices((int)n3, R, Ri);
        if ((rc = get_custom_operands(c, prec, (int)n3, R.data(), Ri.data(), s, &fwd, &inv))) return rc;
    }
    DftPlan D;
    Carve cv;
    if ((rc = make_dft_plan(c, prec, n1, n2, n3, D, cv, s, true))) return rc;
    if ((rc = ensure_ws(c, cv.off))) return rc;
    char* base = (char*)c->ws.p;
    CtrlRegion cr;
    if ((rc = ensure_ctrl(c, &cr))) return rc;
    if ((rc = dft_forward(c, D, prec, n1, n2, n3, Z, fwd, base, cr.ctrl, s))) return rc;
    if (D.h > 0 && (rc = enqueue_svt_core(c, D.E, base, cr.ctrl, tau, nullptr, s))) return rc;
    if ((rc = enqueue_svt_core(c, D.R, base, cr.ctrl, tau, nullptr, s))) return rc;
    DftEmbedArgs ea{};
    ea.zb = base + D.o_zb;
    ea.E = D.h > 0 ? (void*)(base + D.E.o_ybar) : nullptr;
    ea.R = base + D.R.o_ybar;
    ea.n1 = n1; ea.n2 = n2; ea.n3 = (int)n3; ea.h = D.h; ea.nreal = D.nreal;
    hipError_t e = launch_dft_unembed(prec == TSVD_FP64 ? 0 : 1, ea, s);
    if (e != hipSuccess) return hip_fail(c, e, "dft unembed");
    TubeArgs iv{};
    iv.in = base + D.o_zb; iv.out = Y; iv.N = n1 * n2; iv.n3 = (int)n3; iv.ctrl = cr.ctrl; iv.beta_val = 1.0;
    {
        PhaseMark pm(c, 3, s);
        rc = inv ? run_tube_mat(c, prec, iv, 1, inv, s) : run_tube_fft(c, prec, iv, kFftDftInverse, s);
        if (rc) return rc;
    }
    if (ranks_out) {
        // a complex slice's rank is half its real form's; conjugate frequencies share it
        std::vector<int32_t> re(D.h > 0 ? D.h : 1), rr(D.nreal);
        if (D.h > 0) HIPCHK(c, hipMemcpyAsync(re.data(), base + D.E.o_rank, D.h * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(rr.data(), base + D.R.o_rank, D.nreal * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        ranks_out[0] = rr[0];
        for (int f = 1; f <= D.h; ++f) ranks_out[f] = ranks_out[n3 - f] = re[f - 1] / 2;
        if (D.nreal == 2) ranks_out[n3 / 2] = rr[1];
        return read_status(c, s, nullptr);
    }
    return finish_call(c, s);
}

int tnn_c(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, const void* X, double* out, void* stream) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (bad_prec(prec)) return fail(c, TSVD_EINVAL, "unknown precision");
    if (n1 <= 0 || n2 <= 0 || n3 <= 0) return fail(c, TSVD_EINVAL, "sizes must be positive");
    if (!X || !out) return fail(c, TSVD_EINVAL, "null pointer");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Plan P;
    Carve cv;
    int rc = make_plan(c, prec, n1, n2, n3, 0, P, cv, s);
    if (rc) return rc;
    if ((rc = ensure_ws(c, P.o_end))) return rc;
    char* base = (char*)c->ws.p;
    if ((rc = upload_plan(c, P, base))) return rc;
    CtrlRegion cr;
    if ((rc = ensure_ctrl(c, &cr))) return rc;
    hipError_t e = launch_fill_zero(base + P.o_ctr_begin, P.o_ctr_end - P.o_ctr_begin, s);
    if (e != hipSuccess) return hip_fail(c, e, "fill");
    TubeArgs f{};
    f.in = X; f.out = base + P.o_zbar; f.N = P.N; f.n3 = (int)n3; f.ctrl = cr.ctrl; f.check_finite = 1;
    f.beta_val = 1.0;
    if ((rc = run_tube(c, prec, f, 0, s))) return rc;
    if ((rc = run_jacobi(c, P, base, cr.ctrl, s))) return rc;
    double acc = 0.0;
    if ((rc = sum_sigma(c, P, base, cr.ctrl, s, &acc))) return rc;
    *out = acc / (double)n3;
    return read_status(c, s, nullptr);
}

int tnn_f(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, const void* X, double* out, void* stream) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (bad_prec(prec)) return fail(c, TSVD_EINVAL, "unknown precision");
    if (n1 <= 0 || n2 <= 0 || n3 <= 0) return fail(c, TSVD_EINVAL, "sizes must be positive");
    if (!X || !out) return fail(c, TSVD_EINVAL, "null pointer");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const void *fwd = nullptr, *inv = nullptr;  // null: the fast transform (long tubes)
    int rc;
    if (!fft_fits((int)n3)) {
        std::vector<double> R, Ri;
        real_dft_matrices((int)n3, R, Ri);
        if ((rc = get_custom_operands(c, prec, (int)n3, R.data(), Ri.data(), s, &fwd, &inv))) return rc;
    }
    DftPlan D;
    Carve cv;
    if ((rc = make_dft_plan(c, prec, n1, n2, n3, D, cv, s))) return rc;
    if ((rc = ensure_ws(c, cv.off))) return rc;
    char* base = (char*)c->ws.p;
    CtrlRegion cr;
    if ((rc = ensure_ctrl(c, &cr))) return rc;
    if ((rc = dft_forward(c, D, prec, n1, n2, n3, X, fwd, base, cr.ctrl, s))) return rc;
    // a complex slice's real form has each of its singular values twice: the
    // sum over the real forms is the sum over both conjugate frequencies
    double se = 0.0, sr = 0.0;
    if (D.h > 0) {
        if ((rc = run_jacobi(c, D.E, base, cr.ctrl, s))) return rc;
        if ((rc = sum_sigma(c, D.E, base, cr.ctrl, s, &se))) return rc;
    }
    if ((rc = run_jacobi(c, D.R, base, cr.ctrl, s))) return rc;
    if ((rc = sum_sigma(c, D.R, base, cr.ctrl, s, &sr))) return rc;
    *out = (se + sr) / (double)n3;
    return read_status(c, s, nullptr);
}

int tprod_dct(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n4, int64_t n3, const void* X, const void* Yp,
              void* Z, void* stream) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (bad_prec(prec)) return fail(c, TSVD_EINVAL, "unknown precision");
    if (n1 <= 0 || n2 <= 0 || n3 <= 0 || n4 <= 0) return fail(c, TSVD_EINVAL, "sizes must be positive");
    if (!X || !Yp || !Z) return fail(c, TSVD_EINVAL, "null tensor pointer");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const size_t es = esize(prec);
    Carve cv;
    size_t oX = cv.take((size_t)n1 * n2 * n3 * es), oY = cv.take((size_t)n2 * n4 * n3 * es),
           oZ = cv.take((size_t)n1 * n4 * n3 * es);
    int rc = ensure_ws(c, cv.off);
    if (rc) return rc;
    char* base = (char*)c->ws.p;
    CtrlRegion cr;
    if ((rc = ensure_ctrl(c, &cr))) return rc;
    const void *C, *Ct;
    if ((rc = get_dct(c, (int)n3, prec, &C, &Ct))) return rc;
    const int dp = prec == TSVD_FP64 ? 0 : 1;
    TubeArgs f{};
    f.in = X; f.out = base + oX; f.M = C; f.N = n1 * n2; f.n3 = (int)n3; f.ctrl = cr.ctrl; f.check_finite = 1;
    f.beta_val = 1.0;
    if ((rc = run_tube(c, prec, f, 0, s))) return rc;
    f.in = Yp; f.out = base + oY; f.N = n2 * n4;
    if ((rc = run_tube(c, prec, f, 0, s))) return rc;
    hipError_t e;
    GemmArgs g{};
    g.A = base + oX; g.a_rs = 1; g.a_cs = n1; g.a_bs = n1 * n2;
    g.B = base + oY; g.b_rs = 1; g.b_cs = n2; g.b_bs = n2 * n4;
    g.C = base + oZ; g.c_rs = 1; g.c_cs = n1; g.c_bs = n1 * n4;
    g.M = (int)n1; g.Nn = (int)n4; g.K = (int)n2; g.batch = (int)n3;
    e = launch_gemm(dp, g, s);
    if (e != hipSuccess) return hip_fail(c, e, "slice gemm");
    TubeArgs iv{};
    iv.in = base + oZ; iv.out = Z; iv.M = Ct; iv.N = n1 * n4; iv.n3 = (int)n3; iv.ctrl = cr.ctrl; iv.beta_val = 1.0;
    if ((rc = run_tube(c, prec, iv, 1, s))) return rc;
    return finish_call(c, s);
}

int tsvd_dct(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, const void* X, void* U, void* S, void* V,
             int flags, void* stream) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (bad_prec(prec)) return fail(c, TSVD_EINVAL, "unknown precision");
    if (n1 <= 0 || n2 <= 0 || n3 <= 0) return fail(c, TSVD_EINVAL, "sizes must be positive");
    if (!X || !S) return fail(c, TSVD_EINVAL, "null tensor pointer");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Plan P;
    Carve cv;
    int rc = make_plan(c, prec, n1, n2, n3, 1, P, cv, s);
    if (rc) return rc;
    const size_t es = esize(prec);
    const bool full = (flags & TSVD_FULL) != 0;
    const int64_t ucols = full ? n1 : P.p, vcols = full ? n2 : P.p;  // columns of U and V per slice
    const size_t oU = cv.take((size_t)n1 * ucols * n3 * es), oV = cv.take((size_t)n2 * vcols * n3 * es);
    if ((rc = ensure_ws(c, cv.off))) return rc;
    char* base = (char*)c->ws.p;
    if ((rc = upload_plan(c, P, base))) return rc;
    CtrlRegion cr;
    if ((rc = ensure_ctrl(c, &cr))) return rc;
    const void *C, *Ct;
    if ((rc = get_dct(c, (int)n3, prec, &C, &Ct))) return rc;
    const int dp = prec == TSVD_FP64 ? 0 : 1;
    hipError_t e = launch_fill_zero(base + P.o_ctr_begin, P.o_ctr_end - P.o_ctr_begin, s);
    if (e != hipSuccess) return hip_fail(c, e, "fill");
    TubeArgs f{};
    f.in = X; f.out = base + P.o_zbar; f.M = C; f.N = P.N; f.n3 = (int)n3; f.ctrl = cr.ctrl; f.check_finite = 1;
    f.beta_val = 1.0;
    if ((rc = run_tube(c, prec, f, 0, s))) return rc;
    if ((rc = run_jacobi(c, P, base, cr.ctrl, s))) return rc;
    // singular values per column
    SvtPrepArgs sp{};
    sp.A = base + P.o_A; sp.m = P.m; sp.p = P.p; sp.a_ss = (int64_t)P.m * P.p;
    sp.F = base + P.o_F; sp.f_ss = (int64_t)P.m * P.p;
    sp.w = (double*)(base + P.o_w); sp.w_ss = P.p;
    sp.sig = (double*)(base + P.o_sig); sp.sig_ss = P.p;
    sp.ranks = (int*)(base + P.o_rank); sp.pos = (int*)(base + P.o_pos); sp.n3 = (int)n3; sp.tau_val = 0.0;
    sp.ctrl = cr.ctrl;
    if ((e = launch_svt_prep(dp, sp, s)) != hipSuccess) return hip_fail(c, e, "sigma");
    void* Uo = U ? U : (void*)(base + oU);
    void* Vo = V ? V : (void*)(base + oV);
    TsvdFinishArgs fa{};
    fa.A = base + P.o_A; fa.m = P.m; fa.p = P.p; fa.a_ss = (int64_t)P.m * P.p;
    fa.Vj = base + P.o_V; fa.v_ss = (int64_t)P.p * P.p;
    fa.sig = (const double*)(base + P.o_sig); fa.sig_ss = P.p;
    // tall problem: left vectors are U (n1 >= n2) or V (n1 < n2); with full factors
    // the tall side holds m columns per slice, the other side p = its full size
    const int64_t tall_cols = full ? P.m : P.p;
    fa.Ut = P.trans ? Vo : Uo; fa.ut_ss = (int64_t)P.m * tall_cols;
    fa.Vt = P.trans ? Uo : Vo; fa.vt_ss = (int64_t)P.p * P.p;
    fa.S = S; fa.s_ss = P.p; fa.n3 = (int)n3; fa.sign_from_v = P.trans;
    if ((e = launch_tsvd_finish(dp, fa, s)) != hipSuccess) return hip_fail(c, e, "tsvd finish");
    // columns of zero singular values and the full factor's extra columns
    TsvdCompleteArgs ca{};
    ca.Lt = fa.Ut; ca.lt_ss = fa.ut_ss; ca.m = P.m;
    ca.Rt = fa.Vt; ca.rt_ss = fa.vt_ss;
    ca.Vj = base + P.o_V; ca.v_ss = (int64_t)P.p * P.p;
    ca.sig = (const double*)(base + P.o_sig); ca.sig_ss = P.p;
    ca.p = P.p; ca.n3 = (int)n3; ca.full = full && P.m > P.p; ca.sign_from_v = P.trans;
    if ((e = launch_tsvd_complete(dp, ca, s)) != hipSuccess) return hip_fail(c, e, "tsvd complete");
    if (!(flags & TSVD_TRANSFORM_DOMAIN)) {
        // back to the spatial domain (in place: each workgroup owns whole tubes)
        TubeArgs iv{};
        iv.M = Ct; iv.n3 = (int)n3; iv.ctrl = cr.ctrl; iv.beta_val = 1.0;
        if (U) { iv.in = U; iv.out = U; iv.N = n1 * ucols; if ((rc = run_tube(c, prec, iv, 1, s))) return rc; }
        if (V) { iv.in = V; iv.out = V; iv.N = n2 * vcols; if ((rc = run_tube(c, prec, iv, 1, s))) return rc; }
        iv.in = S; iv.out = S; iv.N = P.p;
        if ((rc = run_tube(c, prec, iv, 1, s))) return rc;
    }
    return finish_call(c, s);
}

int complete_tensor(tsvd_ctx* c, int prec, int64_t n1, int64_t n2, int64_t n3, const void* B, const uint8_t* mask,
                    void* X, const tsvd_complete_opts* o, tsvd_complete_info* info, void* stream) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (bad_prec(prec)) return fail(c, TSVD_EINVAL, "unknown precision");
    if (n1 <= 0 || n2 <= 0 || n3 <= 0) return fail(c, TSVD_EINVAL, "sizes must be positive");
    if (!B || !mask || !X || !o) return fail(c, TSVD_EINVAL, "null pointer");
    if (o->max_iter <= 0) return fail(c, TSVD_EINVAL, "max_iter must be positive");
    if (!o->tau_schedule && !(o->beta > 0.0)) return fail(c, TSVD_EINVAL, "beta must be > 0");
    if (o->check_every < 1) return fail(c, TSVD_EINVAL, "check_every must be >= 1");
    if (o->start_iter < 0) return fail(c, TSVD_EINVAL, "start_iter must be >= 0");
    const int L = o->max_iter;
    std::vector<double> betas(L), taus(L);
    for (int l = 0; l < L; ++l) {
        const double t = o->tau_schedule ? o->tau_schedule[o->start_iter + l] : 1.0 / o->beta;
        if (!(t > 0.0) || !isfinite(t)) return fail(c, TSVD_EINVAL, "schedule entries must be finite and > 0");
        betas[l] = o->tau_schedule ? 1.0 / t : o->beta;
        taus[l] = t;
    }
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Plan P;
    Carve cv;
    const int warm_period = c->warm_start < 0 ? 64 : c->warm_start;
    int rc = make_plan(c, prec, n1, n2, n3, warm_period > 0 ? 1 : 0, P, cv, s);
    if (rc) return rc;
    // Cold SVDs take the kept-column mode as a single t-SVT does.  Warm-started
    // ones leave it few sweeps to save and, in the middle of the schedule,
    // slices the certificate rejects; they run the full iteration (measured,
    // 100 iterations: 256x256x31 MIXED 1.20 -> 0.98 ms per iteration but FP64
    // 1.57 -> 1.82, and the 144x176x100 video-shaped MIXED completion 969 ->
    // 531 t-SVT/s).
    if (warm_period == 0) plan_kept_columns(c, P, cv);
    const size_t es = esize(prec);
    const size_t oM = cv.take((size_t)P.N * n3 * es);
    if (warm_period > 0) {
        P.warm = 1;
        P.warm_period = warm_period;
        P.o_A0 = cv.take((size_t)P.m * P.p * n3 * es);
    }
    const size_t oBeta = cv.take((size_t)L * 8), oTau = cv.take((size_t)L * 8);
    if ((rc = ensure_ws(c, cv.off))) return rc;
    char* base = (char*)c->ws.p;
    if ((rc = upload_plan(c, P, base))) return rc;
    if (P.warm) {
        // Jacobi reads A0 = Zbar V (tall, column-major) and starts V from the kept V
        P.job.src = base + P.o_A0;
        P.job.src_ss = (int64_t)P.m * P.p;
        P.job.src_rs = 1;
        P.job.src_cs = P.m;
        P.job.vinit = 1;
    }
    CtrlRegion cr;
    if ((rc = ensure_ctrl(c, &cr))) return rc;
    const void *C, *Ct;
    if ((rc = get_dct(c, (int)n3, prec, &C, &Ct))) return rc;
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipMemcpy(base + oBeta, betas.data(), L * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(base + oTau, taus.data(), L * 8, hipMemcpyHostToDevice));
    if (o->init_observed) {
        const hipError_t ei = launch_observed_init(prec == TSVD_FP64 ? 0 : 1, X, B, mask, P.N * n3, s);
        if (ei != hipSuccess) return hip_fail(c, ei, "initial iterate");
    }
    if (o->M_init) HIPCHK(c, hipMemcpyAsync(base + oM, o->M_init, P.N * n3 * es, hipMemcpyDeviceToDevice, s));
    else if (launch_fill_zero(base + oM, P.N * n3 * es, s) != hipSuccess) return fail(c, TSVD_EHIP, "fill M");
    // iteration counter, norms and history start at zero (status and statistics are kept)
    HIPCHK(c, hipStreamSynchronize(s));
    {
        Ctrl h;
        HIPCHK(c, hipMemcpy(&h, cr.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        h.iter = 0;
        HIPCHK(c, hipMemcpy(cr.ctrl, &h, sizeof(Ctrl), hipMemcpyHostToDevice));
    }
    if (launch_fill_zero(cr.norms, 256 + 8 * kHist, s) != hipSuccess) return fail(c, TSVD_EHIP, "fill norms");

    auto enqueue_iter = [&](hipStream_t st) -> int {
        hipError_t e = launch_fill_zero(base + P.o_ctr_begin, P.o_ctr_end - P.o_ctr_begin, st);
        if (e != hipSuccess) return hip_fail(c, e, "fill");
        TubeArgs f{};
        f.out = base + P.o_zbar; f.M = C; f.N = P.N; f.n3 = (int)n3; f.ctrl = cr.ctrl; f.check_finite = 1;
        f.pX = X; f.pM = base + oM; f.beta_sched = (const double*)(base + oBeta);
        {
            PhaseMark pm(c, 0, st);
            int r0 = run_tube(c, prec, f, 0, st);
            if (r0) return r0;
        }
        int r2 = enqueue_svt_core(c, P, base, cr.ctrl, 0.0, (const double*)(base + oTau), st);
        if (r2) return r2;
        TubeArgs iv{};
        iv.in = base + P.o_ybar; iv.out = nullptr; iv.M = Ct; iv.N = P.N; iv.n3 = (int)n3; iv.ctrl = cr.ctrl;
        iv.eB = B; iv.emask = mask; iv.eX = X; iv.eM = base + oM; iv.norms = cr.norms;
        iv.beta_sched = (const double*)(base + oBeta);
        {
            PhaseMark pm(c, 3, st);
            int r3 = run_tube(c, prec, iv, 1, st);
            if (r3) return r3;
        }
        e = launch_iter_advance(cr.ctrl, cr.norms, cr.hist, kHist, st);
        if (e != hipSuccess) return hip_fail(c, e, "advance");
        return TSVD_OK;
    };

    int iters = 0;
    double last = 0.0;
    bool stop = false;
    const bool check = o->tol > 0.0;
    // Replay a captured iteration unless profiling (per-kernel events) is on.
    hipGraphExec_t exec = nullptr;
    hipStream_t run = s;
    if (c->use_graphs && !c->prof) {
        // everything the iteration allocates lazily must exist before capture
        if ((rc = prepare_tube(c, (int)n3, prec))) return rc;
        if (!c->own) HIPCHK(c, hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
        HIPCHK(c, hipStreamSynchronize(s));
        run = c->own;
        hipGraph_t graph = nullptr;
        HIPCHK(c, hipStreamBeginCapture(run, hipStreamCaptureModeThreadLocal));
        c->capturing = 1;
        const int rc_cap = enqueue_iter(run);
        c->capturing = 0;
        const hipError_t ec = hipStreamEndCapture(run, &graph);
        if (rc_cap) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc_cap;
        }
        if (ec != hipSuccess) return hip_fail(c, ec, "hipStreamEndCapture");
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return hip_fail(c, ei, "hipGraphInstantiate");
    }
    auto one_iter = [&]() -> int {
        if (exec) {
            hipError_t e = hipGraphLaunch(exec, run);
            return e == hipSuccess ? TSVD_OK : hip_fail(c, e, "hipGraphLaunch");
        }
        return enqueue_iter(run);
    };
    while (iters < L && !stop) {
        if ((rc = one_iter())) break;
        ++iters;
        if (check && (iters % o->check_every == 0 || iters == L)) {
            if (hipStreamSynchronize(run) != hipSuccess) { rc = fail(c, TSVD_EHIP, "sync"); break; }
            double h = 0.0;
            if (hipMemcpy(&h, cr.hist + (iters - 1) % kHist, 8, hipMemcpyDeviceToHost) != hipSuccess) {
                rc = fail(c, TSVD_EHIP, "history read");
                break;
            }
            last = h;
            if (h <= o->tol) stop = true;
        }
    }
    if (run != s) (void)hipStreamSynchronize(run);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(s));
    if (iters >= 1) HIPCHK(c, hipMemcpy(&last, cr.hist + (iters - 1) % kHist, 8, hipMemcpyDeviceToHost));
    if (o->M_out) HIPCHK(c, hipMemcpyAsync(o->M_out, base + oM, P.N * n3 * es, hipMemcpyDeviceToDevice, s));
    int msw = 0;
    rc = read_status(c, s, &msw);
    if (info) {
        info->iters = iters;
        info->rel_change = last;
        info->status = rc;
        info->max_sweeps = msw;
    }
    return rc;
}

int tsvt_dct_batched(tsvd_ctx* c, int prec, int count, const int64_t* dims, const void* const* Z, void* const* Y,
                     const double* tau, int32_t* status_out, void* stream) {
    if (!c) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (bad_prec(prec)) return fail(c, TSVD_EINVAL, "unknown precision");
    if (count <= 0 || !dims || !Z || !Y || !tau) return fail(c, TSVD_EINVAL, "bad batch arguments");
    std::vector<BatchJobSpec> jb(count);
    for (int j = 0; j < count; ++j) {
        if (dims[3 * j] <= 0 || dims[3 * j + 1] <= 0 || dims[3 * j + 2] <= 0)
            return fail(c, TSVD_EINVAL, "sizes must be positive");
        if (!Z[j] || !Y[j]) return fail(c, TSVD_EINVAL, "null tensor pointer");
        if (!(tau[j] >= 0.0) || !isfinite(tau[j])) return fail(c, TSVD_EINVAL, "tau must be finite and >= 0");
        jb[j] = BatchJobSpec{dims[3 * j], dims[3 * j + 1], dims[3 * j + 2], Z[j], Y[j], nullptr, nullptr, nullptr,
                             nullptr, 1.0, tau[j]};
    }
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    if (status_out) {
        // every tensor gets its own code; the call waits for the step
        int rc = batched_step_locked(c, prec, count, jb.data(), status_out, s);
        if (rc) return rc;
        (void)read_status(c, s, nullptr);
        return TSVD_OK;
    }
    int rc = batched_step_locked(c, prec, count, jb.data(), nullptr, s);
    if (rc) return rc;
    return finish_call(c, s);
}

}  // extern "C"

// Batched step shared by tsvt_dct_batched and the serving loop.  Called with
// the context lock held.
int batched_step_locked(tsvd_ctx* c, int prec, int count, const BatchJobSpec* jb, int* job_status, hipStream_t s) {
    std::vector<Plan> plans(count);
    Carve cv;
    int rc;
    int64_t ntasks = 0;
    for (int j = 0; j < count; ++j) {
        Plan& P = plans[j];
        const int wv = jb[j].V ? 1 : 0;
        if ((rc = make_plan(c, prec, jb[j].n1, jb[j].n2, jb[j].n3, wv, P, cv, s, true))) return rc;
        if (wv && jb[j].vinit) {
            P.warm = 1;
            P.o_A0 = cv.take((size_t)P.m * P.p * P.n3 * esize(prec));
        }
        ntasks += jb[j].n3;
    }
    const size_t o_jobs = cv.take(sizeof(JacobiJob) * count);
    const size_t o_tj = cv.take(sizeof(int) * ntasks), o_tk = cv.take(sizeof(int) * ntasks);
    const size_t o_queue = cv.take(512);  // one work counter per (V, row geometry) (16 x 32 bytes)
    const size_t o_jctrl = cv.take((size_t)kJobCtrlBytes * count);  // each job's own status and counters
    if ((rc = ensure_ws(c, cv.off))) return rc;
    char* base = (char*)c->ws.p;
    CtrlRegion cr;
    if ((rc = ensure_ctrl(c, &cr))) return rc;
    auto jctrl = [&](int j) { return (Ctrl*)(base + o_jctrl + (size_t)kJobCtrlBytes * j); };
    // job table; task lists grouped by row geometry (R, G), each sorted by
    // estimated cost (m p^2 per slice), largest first
    auto geo = [](const Plan& P) { return (P.with_v ? 8 : 0) + (P.job.G == 32 ? 4 : 0) + P.job.R / 4 - 1; };  // 0..15
    std::vector<JacobiJob> jobs(count);
    std::vector<std::pair<double, std::pair<int, int>>> order;
    order.reserve(ntasks);
    for (int j = 0; j < count; ++j) {
        Plan& P = plans[j];
        bind_plan(P, base);
        P.job.ctrl = jctrl(j);
        if (P.with_v) {
            // the job's own V, kept across steps; a warm start reads A0 = Zbar V
            P.job.V = jb[j].V;
            P.job.vinit = jb[j].vinit ? 1 : 0;
            if (P.warm) {
                P.job.src = base + P.o_A0;
                P.job.src_ss = (int64_t)P.m * P.p;
                P.job.src_rs = 1;
                P.job.src_cs = P.m;
            }
        }
        jobs[j] = P.job;
        const double cost = (double)plans[j].m * plans[j].p * plans[j].p;
        for (int k = 0; k < plans[j].n3; ++k) order.push_back({geo(plans[j]) * 1e30 - cost, {j, k}});
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<double, std::pair<int, int>>& a, const std::pair<double, std::pair<int, int>>& b) {
                         return a.first < b.first;
                     });
    std::vector<int> tj(ntasks), tk(ntasks);
    int gbeg[17] = {0}, gcnt[16] = {0};
    for (int64_t t = 0; t < ntasks; ++t) {
        tj[t] = order[t].second.first;
        tk[t] = order[t].second.second;
        gcnt[geo(plans[tj[t]])]++;
    }
    for (int g = 0; g < 16; ++g) gbeg[g + 1] = gbeg[g] + gcnt[g];
    int glds[16] = {0};
    for (int j = 0; j < count; ++j) glds[geo(plans[j])] = std::max(glds[geo(plans[j])], plans[j].lds);
    HIPCHK(c, hipStreamSynchronize(s));  // tables live in the shared workspace
    HIPCHK(c, hipMemcpy(base + o_jobs, jobs.data(), sizeof(JacobiJob) * count, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(base + o_tj, tj.data(), sizeof(int) * ntasks, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(base + o_tk, tk.data(), sizeof(int) * ntasks, hipMemcpyHostToDevice));
    hipError_t e = launch_fill_zero(base + o_queue, 512, s);
    if (e != hipSuccess) return hip_fail(c, e, "fill");
    if ((e = launch_fill_zero(base + o_jctrl, (int64_t)kJobCtrlBytes * count, s)) != hipSuccess)
        return hip_fail(c, e, "fill");
    for (int j = 0; j < count; ++j) {
        Plan& P = plans[j];
        if ((e = launch_fill_zero(base + P.o_ctr_begin, P.o_ctr_end - P.o_ctr_begin, s)) != hipSuccess)
            return hip_fail(c, e, "fill");
        TubeArgs f{};
        f.out = base + P.o_zbar; f.N = P.N; f.n3 = (int)P.n3; f.ctrl = jctrl(j); f.check_finite = 1;
        f.beta_val = jb[j].X ? jb[j].beta : 1.0;
        if (jb[j].X) { f.pX = jb[j].X; f.pM = jb[j].M; } else { f.in = jb[j].Z; }
        PhaseMark pm(c, 0, s);
        if ((rc = run_tube(c, prec, f, 0, s))) return rc;
    }
    for (int j = 0; j < count; ++j) {
        if (!plans[j].warm) continue;
        PhaseMark pm(c, 4, s);
        if ((rc = enqueue_warm_gemm(c, plans[j], base, jb[j].V, s))) return rc;
    }
    {
        PhaseMark pm(c, 1, s);
        for (int g = 0; g < 16; ++g) {
            if (!gcnt[g]) continue;
            const int G = (g % 8) >= 4 ? 32 : 16, R = 4 * (g % 4 + 1), wv = g >= 8;
            e = launch_jacobi_batched(prec == TSVD_FP64 ? 0 : 1, R, G, wv, (const JacobiJob*)(base + o_jobs),
                                      (const int*)(base + o_tj) + gbeg[g], (const int*)(base + o_tk) + gbeg[g],
                                      gcnt[g], (int*)(base + o_queue) + 8 * g, clamp_sweeps(c->max_sweeps), cr.ctrl,
                                      glds[g], s);
            if (e != hipSuccess) return hip_fail(c, e, "batched jacobi");
        }
    }
    for (int j = 0; j < count; ++j) {
        Plan& P = plans[j];
        if ((rc = enqueue_after_jacobi(c, P, base, jctrl(j), jb[j].tau, nullptr, s))) return rc;
        TubeArgs iv{};
        iv.in = base + P.o_ybar; iv.N = P.N; iv.n3 = (int)P.n3; iv.ctrl = jctrl(j); iv.beta_val = 1.0;
        if (jb[j].X) {
            iv.eB = jb[j].B; iv.emask = jb[j].mask; iv.eX = jb[j].X; iv.eM = jb[j].M; iv.beta_val = jb[j].beta;
        } else {
            iv.out = jb[j].Y;
        }
        PhaseMark pm(c, 3, s);
        if ((rc = run_tube(c, prec, iv, 1, s))) return rc;
    }
    // the jobs' statuses and counters join the context's block (tsvd_sync_status, statistics)
    if ((e = launch_fold_ctrl(cr.ctrl, jctrl(0), count, kJobCtrlBytes, s)) != hipSuccess) return hip_fail(c, e, "fold");
    if (job_status) {
        std::vector<Ctrl> h(count);
        HIPCHK(c, hipStreamSynchronize(s));
        HIPCHK(c, hipMemcpy2D(h.data(), sizeof(Ctrl), jctrl(0), kJobCtrlBytes, sizeof(Ctrl), count,
                              hipMemcpyDeviceToHost));
        for (int j = 0; j < count; ++j) job_status[j] = status_code(h[j].status);
    }
    return TSVD_OK;
}

int tsvd_batched_step_sync(tsvd_ctx* c, int prec, int count, const BatchJobSpec* jb, int* job_status,
                           hipStream_t s) {
    std::lock_guard<std::mutex> lk(c->mu);
    HIPCHK(c, hipSetDevice(c->device));
    int rc = batched_step_locked(c, prec, count, jb, job_status, s);
    if (rc) return rc;
    // per-job codes are in job_status; the context's accumulated status is cleared
    rc = read_status(c, s, nullptr);
    return rc < 0 && rc != TSVD_ENONFINITE && rc != TSVD_ETIMEOUT ? rc : TSVD_OK;
}

int tsvd_batched_shape_check(int prec, int64_t n1, int64_t n2, int with_v) {
    if (n1 <= 0 || n2 <= 0 || std::max(n1, n2) > kMaxRows) return TSVD_EINVAL;
    Plan P;
    P.prec = prec;
    P.n1 = n1; P.n2 = n2; P.n3 = 1; P.N = n1 * n2;
    P.m = (int)std::max(n1, n2);
    P.p = (int)std::min(n1, n2);
    P.with_v = with_v ? 1 : 0;
    // every candidate tile of a batched plan: one of them must hold the slice
    for (const Tile& t : tile_candidates(P, true, -1)) {
        Plan Q = P;
        if (apply_tile(nullptr, Q, t, true) == TSVD_OK) return TSVD_OK;
    }
    Plan Q = P;
    return apply_tile(nullptr, Q, default_tile(P, 0, 0, 0, true), true) == TSVD_OK ? TSVD_OK : TSVD_EINVAL;
}

size_t tsvd_batched_workspace_bytes(int prec, int64_t n1, int64_t n2, int64_t n3) {
    // mirrors make_plan's regions (upper bound: counters and alignment)
    const size_t es = prec == TSVD_FP64 ? 8 : 4;
    const size_t m = (size_t)std::max(n1, n2), p = (size_t)std::min(n1, n2), N = (size_t)n1 * n2;
    // Zbar, Ybar; A', F, A0 (warm start); G, V (workspace copy); counters
    return es * (2 * N * n3 + 3 * m * p * n3 + 2 * p * p * n3) + 20 * p * n3 + 4 * n3 * (kRotStride + 3) + 32 * 256 +
           sizeof(JacobiJob) + 8 * n3 + kJobCtrlBytes;
}

int tsvd_ctx_device(const tsvd_ctx* c) { return c->device; }

