// Internal declarations shared by the HIP translation units of libtsvdmi.
// Not part of the public interface (include/tsvdmi.h is).
#pragma once

#include <string>

#include "jacobi.h"

namespace tsvd {

// ---- launch helpers (defined in the .hip files) -----------------------------
// All return hipSuccess or the first HIP error.

// Tube transform: out[r + N*k'] = sum_k M[k'][k] in[r + N*k], r < N, k,k' < n3.
// M is row-major n3 x n3 on the device.  Optional fused prologue/epilogue for
// the completion loop (see ops.hip).
struct TubeArgs {
    const void* in;
    void* out;
    const void* M;         // transform matrix (device), row-major n3 x n3, element type = data type
    int64_t N;             // tubes = n1*n2
    int n3;
    // prologue: in = X - Mlt / beta  (when X != nullptr; `in` is then ignored)
    const void* pX;
    const void* pM;
    // epilogue (ADMM): y = transform result;
    //   Xn = mask ? B : y + Mlt/beta ; Mlt += beta (y - Xn) ; X <- Xn; out <- y (if out)
    const void* eB;
    const uint8_t* emask;
    void* eX;
    void* eM;
    double* norms;         // [2 kNormSlots]: slot pairs += (||Xn - X||^2, ||X||^2) (FP64 atomics)
    // beta: beta_val, or beta_sched[ctrl->iter] when beta_sched != nullptr
    double beta_val;
    const double* beta_sched;
    Ctrl* ctrl;
    int check_finite;      // 1: flag non-finite inputs in ctrl->status
};
hipError_t launch_tube_transform(int prec, const TubeArgs& a, hipStream_t s);
constexpr int kTubeTile = 64;  // tubes per workgroup of launch_tube_transform
// Dynamic LDS of launch_tube_transform (prec: 0 FP64, else FP32 data).
inline int dense_tube_lds(int prec, int n3) { return n3 * kTubeTile * (prec == 0 ? 8 : 4); }

// The same transform on the matrix cores for tubes of length n3 <= kMaxTube.
// eng: 0 FP64, 1 FP32, 2 BF16 hi+lo (FP32 data).  frag: M in fragment order,
// built on the host by make_tube_fragments (tube_fragment_bytes bytes).
constexpr int kMaxTube = 128;
int tube_ks(int eng, int n3);
size_t tube_fragment_bytes(int eng, int n3);
void make_tube_fragments(int eng, int n3, const double* M, void* out);
hipError_t launch_tube_mfma(int eng, const TubeArgs& a, const void* frag, hipStream_t s);
// Fast tube transforms (dct_fft.hip) for tubes of 129..512, in O(n3 log n3)
// by Bluestein's chirp with register-resident Stockham FFTs of 512 or 1024
// points, two real tubes per complex transform, in FP64 arithmetic for double
// data (prec 0) and FP32 for float data (prec 1): the orthonormal DCT-II and
// its inverse (Makhoul's reordering), and the real form of the DFT and its
// inverse (rows: Re V0, (Re Vf, Im Vf) for 1 <= f <= (n3-1)/2, Re V(n3/2) for
// even n3).  Tables built on the host by make_fft_tables (fft_table_bytes
// bytes, per precision).  hipErrorInvalidValue unless fft_fits(n3).
enum { kFftDctForward = 0, kFftDctInverse = 1, kFftDftForward = 2, kFftDftInverse = 3 };
int fft_size(int n);
size_t fft_table_bytes(int n, int prec);
void make_fft_tables(int n, int prec, void* out);
int fft_lds_bytes(int n, int prec);
bool fft_fits(int n3);  // 128 < n3 <= 512
hipError_t launch_tube_fft(int prec, const TubeArgs& a, const void* tables, int mode, hipStream_t s);

// The operand of the tube transform built on the device (no host copy): the
// fragments of engine eng for n3 <= kMaxTube, else the dense row-major matrix
// (FP64 for eng 0, FP32 otherwise).  tube_matrix_bytes gives its size.
size_t tube_matrix_bytes(int eng, int n3);
hipError_t launch_tube_matrix(int eng, int n3, int inverse, void* out, hipStream_t s);

// Batched strided GEMM with optional per-batch K (ranks) and column scale.
//   C_b(i,j) = cscale_b(j) * sum_{t < K_b} A_b(i,t) B_b(t,j)
// X_b(r,c) = X[b*bs + r*rs + c*cs].  K_b = Kdev ? Kdev[b] : K.
struct GemmArgs {
    const void* A; int64_t a_rs, a_cs, a_bs;
    const void* B; int64_t b_rs, b_cs, b_bs;
    void* C; int64_t c_rs, c_cs, c_bs;
    const double* cscale; int64_t s_bs;  // per-column scale (FP64) or nullptr
    int M, Nn, K;
    const int* Kdev;   // per-batch K, or nullptr
    const int* Ndev;   // per-batch column count (<= Nn), or nullptr
    int batch;
};
hipError_t launch_gemm(int prec, const GemmArgs& g, hipStream_t s);

// SVT factor preparation: per slice, sigma_c = ||A'(:,c)||, keep = sigma > tau,
// compacts kept columns of A' into F (ld m), w_c = (sigma_c - tau)/sigma_c^3,
// rank -> ranks[k].
struct SvtPrepArgs {
    const void* A; int m, p; int64_t a_ss;   // A' slices (ld m)
    void* F; int64_t f_ss;                    // compacted columns (ld m)
    double* w; int64_t w_ss;                  // scales
    double* sig; int64_t sig_ss;              // singular values (unsorted, per column)
    int* ranks;
    int* pos;                                 // scratch: p per slice (position of each kept column, or -1)
    int n3;
    double tau_val; const double* tau_sched; Ctrl* ctrl;
};
hipError_t launch_svt_prep(int prec, const SvtPrepArgs& a, hipStream_t s);

// DFT path: real forms of the complex Fourier slices (see ops.hip).  zb: the
// real-transform slots (n1 x n2 x n3); E: h slices of 2 n1 x 2 n2; R: nreal
// (1 or 2) real slices.  unembed writes back into zb.
struct DftEmbedArgs {
    void* zb;
    void* E;
    void* R;
    int64_t n1, n2;
    int n3, h, nreal;
};
hipError_t launch_dft_embed(int prec, const DftEmbedArgs& a, hipStream_t s);
hipError_t launch_dft_unembed(int prec, const DftEmbedArgs& a, hipStream_t s);

// Threshold certificate of the kept-column Jacobi mode (certify.hip): per
// slice, after the kept-column iteration, flags[k] = 1 when the iteration
// converged and the columns of A' with squared norm <= tau^2 have spectral
// norm <= tau (bound ||H^4||_F^2 with H their Gram matrix / tau^2, FP32 with
// a rounding margin), or when the slice converged as the full iteration;
// else 0, and ctrl->fallback += 1.  hipErrorInvalidValue when m > kMaxRows,
// or tau <= 0 without a schedule.
struct CertArgs {
    const void* A;      // A' (tall, m x p per slice, ld m, slice stride m p), FP64 for prec 0 else FP32
    int m, p, n3;
    double tau;         // the threshold (> 0), or
    const double* tau_sched;  // (device) thresholds by iteration: tau = tau_sched[ctrl->iter]
    double* nrm2;       // [n3 p] squared column norms (written)
    float* As;          // [n3 m p] A' / tau in FP32 (written)
    float* H;           // [n3 p p] Gram matrix, then H^4 (written)
    float* H2;          // [n3 p p] H^2 (written)
    double* sums;       // [n3] zero before the launch; ||H^4||_F^2
    int* done;          // [n3] zero before the launch; workgroups of the slice's sum that finished
    const int* sweeps;  // [n3] sweeps of the kept-column iteration (-1: did not converge)
    const int* full;    // [n3] 1: the slice converged as the full iteration (no certificate needed)
    int* ncols;         // [n3] (written) p for a slice to certify, 0 for one that converged as the full
                        // iteration: the column count of its GEMMs, which then skip it
    int* flags;         // [n3] result
    Ctrl* ctrl;
};
hipError_t launch_threshold_certificate(int prec, CertArgs a, hipStream_t s);

// One batched step over many tensors (used by tsvt_dct_batched and the serving
// loop).  Per tensor: either a plain t-SVT Z -> Y, or one completion iteration
// with the fused prologue Z = X - M/beta and epilogue (X, M updated in place).
struct BatchJobSpec {
    int64_t n1, n2, n3;
    const void* Z;        // plain t-SVT input (nullptr when X is given)
    void* Y;              // plain t-SVT output
    void* X;              // completion iterate (prologue input, epilogue in/out)
    void* M;              // completion multiplier (in/out)
    const void* B;        // observed data
    const uint8_t* mask;  // observed set
    double beta, tau;
    void* V;              // completion warm start: the job's V (p x p per slice) kept across steps, or nullptr
    int vinit;            // with V: 1 warm-starts from V (Jacobi input Zbar V), 0 starts V from the identity
};

// Small utility kernels.
hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s);
// n values of a deterministic pseudo-random pattern in [-1, 1) (prec 0: double, else float).
hipError_t launch_fill_pattern(void* p, int64_t n, int prec, uint32_t seed, hipStream_t s);
hipError_t launch_iter_advance(Ctrl* ctrl, double* norms, double* relchg_hist, int hist_len, hipStream_t s);
// X = mask ? B : 0 (n elements; prec 0: double, else float).
hipError_t launch_observed_init(int prec, void* X, const void* B, const uint8_t* mask, int64_t n, hipStream_t s);
// dst: status |= OR of the count per-job blocks (stride_bytes apart), max_sweeps = max, slice_sweeps += sum.
hipError_t launch_fold_ctrl(Ctrl* dst, const Ctrl* jobs, int count, int stride_bytes, hipStream_t s);
// V (p x p per slice, n3 slices) := identity when ctrl->iter % period == 0.
hipError_t launch_warm_reset(int prec, void* V, int p, int n3, const Ctrl* ctrl, int period, hipStream_t s);
// Sort singular values descending per slice and build U = A'(:,perm)/sigma, with the
// sign convention, and permute V; used by tsvd_dct.
struct TsvdFinishArgs {
    const void* A; int m, p; int64_t a_ss;   // A' (tall m x p)
    const void* Vj; int64_t v_ss;            // Jacobi V (p x p)
    const double* sig; int64_t sig_ss;
    void* Ut; int64_t ut_ss;                 // out: tall left vectors m x p
    void* Vt; int64_t vt_ss;                 // out: tall right vectors p x p
    void* S; int64_t s_ss;                   // out: singular values (data type), p per slice
    int n3;
    int sign_from_v;                         // 1: the slice's left vectors are the Jacobi V (n1 < n2)
};
hipError_t launch_tsvd_finish(int prec, const TsvdFinishArgs& a, hipStream_t s);
// Completion of the tall-side vectors after the finish: columns of zero
// singular values and, with full, the columns p..m-1 of the full factor.
struct TsvdCompleteArgs {
    void* Lt; int64_t lt_ss; int m;          // tall-side vectors, ld m, slice stride lt_ss
    void* Rt; int64_t rt_ss;                 // the other side (p x p): partner sign flips
    const void* Vj; int64_t v_ss;            // Jacobi right vectors (p x p, unsorted columns)
    const double* sig; int64_t sig_ss;       // per-column singular values (unsorted)
    int p, n3;
    int full;                                // 1: also columns p..m-1
    int sign_from_v;                         // 1: wide slice (the pair's sign comes from Vj)
};
hipError_t launch_tsvd_complete(int prec, const TsvdCompleteArgs& a, hipStream_t s);

}  // namespace tsvd

// Internal entry points of the library used by the serving loop (C++ linkage).
struct tsvd_ctx;
// One batched step of `count` jobs, each with its own device status word.
// job_status (HOST, count entries, may be NULL): when given, the call waits
// for the step and writes each job's code (TSVD_OK, TSVD_WARN_NOCONV,
// TSVD_ENONFINITE, TSVD_ETIMEOUT).  The jobs' statuses are also folded into
// the context's accumulated status.
int batched_step_locked(tsvd_ctx* c, int prec, int count, const tsvd::BatchJobSpec* jb, int* job_status,
                        hipStream_t s);
// Takes the context lock, runs one batched step on `s`, waits for it, writes
// every job's own status to job_status and clears the context's accumulated
// status.  Returns TSVD_OK, or a negative code when the step itself could not
// run (its jobs then have no result).
int tsvd_batched_step_sync(tsvd_ctx* c, int prec, int count, const tsvd::BatchJobSpec* jb, int* job_status,
                           hipStream_t s);
// 0 when a tensor of this shape can run in a batched step (frontal slices of
// at most 512 rows and columns whose Jacobi block fits one workgroup's LDS),
// else TSVD_EINVAL.  No device call.
int tsvd_batched_shape_check(int prec, int64_t n1, int64_t n2, int with_v);
// Bytes of workspace one batched step needs for a tensor of this shape.
size_t tsvd_batched_workspace_bytes(int prec, int64_t n1, int64_t n2, int64_t n3);
int tsvd_ctx_device(const tsvd_ctx* c);
